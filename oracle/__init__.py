"""CPU FP64 oracle for the DPD + CGMD multiple-time-stepping hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP path (``paper_2205_14121_amd``) and never imports it.

The numerical work lives in ``aimts_oracle.c`` (plain C, FP64), compiled with gcc
into ``liboracle.so``; the controller network's oracle is plain numpy in
``gru.py``.  This file only marshals numpy arrays into the C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aimts_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP for the timing runs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [
        ("lo", C.c_double * 3), ("L", C.c_double * 3), ("periodic", C.c_int32 * 3),
        ("wall_axis", C.c_int32), ("wall_lo", C.c_double), ("wall_hi", C.c_double),
        ("mass", C.c_double * 3),
        ("a", C.c_double), ("gamma", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("lj_eps", C.c_double), ("lj_sig", C.c_double), ("lj_rc", C.c_double),
        ("gamma_pf", C.c_double), ("sigma_pf", C.c_double), ("rc_pf", C.c_double),
        ("kb", C.c_double), ("ka", C.c_double),
        ("morse_D", C.c_double), ("morse_a", C.c_double), ("morse_r0", C.c_double),
        ("r_excl", C.c_double), ("g", C.c_double * 3), ("seed", C.c_uint64),
        ("n_fluid", C.c_int64), ("n_wall", C.c_int64), ("n_bead", C.c_int64),
        ("n_bond", C.c_int64), ("n_angle", C.c_int64), ("n_morse", C.c_int64),
        ("n_platelet", C.c_int64),
        ("body", C.c_void_p), ("rest", C.c_void_p), ("bond", C.c_void_p), ("bond_r0", C.c_void_p),
        ("angle", C.c_void_p), ("angle_th0", C.c_void_p), ("morse", C.c_void_p),
        ("platelet_area", C.c_void_p),
        ("agg_D", C.c_double), ("agg_a", C.c_double), ("agg_r0", C.c_double), ("agg_fA", C.c_double),
        ("agg_rc", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_zeta.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32]
        L.or_zeta.restype = C.c_double
        L.or_outer_forces.argtypes = [P, P, P, C.c_uint64, C.c_double, P, C.c_int64, C.c_int, C.c_int, P]
        L.or_inner_forces.argtypes = [P, P, P, C.c_uint64, C.c_double, C.c_int, P]
        L.or_energy.argtypes = [P, P, P]
        L.or_respa.argtypes = [P, P, P, P, P, P, C.c_int64, C.c_double, C.c_int, C.c_int, C.c_int]
        L.or_thermo.argtypes = [P, P, P, C.c_int, C.c_int, P]
        L.or_features.argtypes = [P, P, P, C.c_int, C.c_double, P]
        L.or_pairs_brute.argtypes = [P, P, C.c_int64, C.c_double, P, C.c_int64]
        L.or_pairs_brute.restype = C.c_int64
        L.or_pairs_cells.argtypes = [P, P, C.c_int64, C.c_double, P, C.c_int64]
        L.or_pairs_cells.restype = C.c_int64
        L.or_num_threads.restype = C.c_int
        L.or_paper_features.argtypes = [P, P, P, C.c_double, P]
        L.or_bead_stress.argtypes = [P, P, P, P]
        L.or_inner_forces3.argtypes = [P, P, P, C.c_uint64, C.c_double, P, C.c_int, C.c_int, P, P, P]
        L.or_respa3.argtypes = [P, P, P, P, P, P, P, P, C.c_int64, C.c_double, C.c_int, C.c_int, C.c_int, P,
                                C.c_int, C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function on one (counter[4], key[2]) pair."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def zeta(i, j, count, seed, group):
    """Pair-symmetric standard normal variate zeta_ij of the DPD random force."""
    return lib().or_zeta(int(i), int(j), int(count), int(seed), int(group))


class System:
    """A workload dict (from ``synth``) bound to the oracle's C struct."""

    def __init__(self, sysd: dict, params: dict | None = None):
        p = dict(sysd["params"])
        if params:
            p.update(params)
        self.d = sysd
        self.p = p
        self._keep = {k: np.ascontiguousarray(sysd[k]) for k in
                      ("body", "rest", "bonds", "bond_r0", "angles", "angle_th0", "morse", "platelet_area")}
        s = _Sys()
        s.lo[:] = list(np.asarray(sysd["box_lo"], float))
        s.L[:] = list(np.asarray(sysd["box_L"], float))
        s.periodic[:] = [int(q) for q in sysd["periodic"]]
        s.wall_axis, s.wall_lo, s.wall_hi = int(p["wall_axis"]), float(p["wall_lo"]), float(p["wall_hi"])
        s.mass[:] = [float(m) for m in p["mass"]]
        for k in ("a", "gamma", "sigma", "rc", "lj_eps", "lj_sig", "lj_rc", "gamma_pf", "sigma_pf", "rc_pf",
                  "kb", "ka", "morse_D", "morse_a", "morse_r0", "r_excl"):
            setattr(s, k, float(p[k]))
        s.g[:] = [float(q) for q in p["g"]]
        s.seed = int(p["seed"])
        s.n_fluid, s.n_wall, s.n_bead = int(sysd["n_fluid"]), int(sysd["n_wall"]), int(sysd["n_bead"])
        s.n_bond, s.n_angle = self._keep["bonds"].shape[0], self._keep["angles"].shape[0]
        s.n_morse, s.n_platelet = self._keep["morse"].shape[0], int(sysd["n_platelet"])
        s.body, s.rest = _ptr(self._keep["body"]), _ptr(self._keep["rest"])
        s.bond, s.bond_r0 = _ptr(self._keep["bonds"]), _ptr(self._keep["bond_r0"])
        s.angle, s.angle_th0 = _ptr(self._keep["angles"]), _ptr(self._keep["angle_th0"])
        s.morse, s.platelet_area = _ptr(self._keep["morse"]), _ptr(self._keep["platelet_area"])
        for k in ("agg_D", "agg_a", "agg_r0", "agg_fA", "agg_rc"):  # Eq. 4 aggregation (off at agg_rc = 0)
            setattr(s, k, float(p.get(k, 0.0)))
        self.s = s
        self.n = int(sysd["n"])

    def _sp(self):
        return C.byref(self.s)

    def outer_forces(self, x, v, count, dt, subset=None, brute=False, nthreads=1):
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        f = np.zeros((self.n, 3))
        sub = None if subset is None else np.ascontiguousarray(subset, np.int64)
        rc = lib().or_outer_forces(self._sp(), x.ctypes.data, v.ctypes.data, int(count), float(dt),
                                   _ptr(sub), 0 if sub is None else sub.size, int(brute), int(nthreads),
                                   f.ctypes.data)
        if rc:
            raise RuntimeError("oracle outer forces failed (%d)" % rc)
        return f

    def inner_forces(self, x, v, count, dt, brute=False):
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        f = np.zeros((self.n, 3))
        rc = lib().or_inner_forces(self._sp(), x.ctypes.data, v.ctypes.data, int(count), float(dt), int(brute),
                                   f.ctypes.data)
        if rc:
            raise RuntimeError("oracle inner forces failed (%d)" % rc)
        return f

    # ---- three-level MTS with per-platelet sublevels (Table 1) ----
    G_M, G_P1, G_P2 = 1, 2, 4

    def _levels(self, level):
        lv = np.ascontiguousarray(level, dtype=np.int32)
        assert lv.shape == (max(int(self.d["n_platelet"]), 1),) or lv.shape == (int(self.d["n_platelet"]),)
        return lv

    def inner_forces3(self, x, v, count, dt_m, level, due=7, brute=False):
        """(f_m, f_p1, f_p2): the interface group (random term scaled by dt_m) and the two
        platelet sublevel groups at (x, v); `level[p]` is platelet p's sublevel (1 or 2)."""
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        out = [np.zeros((self.n, 3)) for _ in range(3)]
        lv = self._levels(level)
        rc = lib().or_inner_forces3(self._sp(), x.ctypes.data, v.ctypes.data, int(count), float(dt_m),
                                    lv.ctypes.data, int(due), int(brute), *[o.ctypes.data for o in out])
        if rc:
            raise RuntimeError("oracle three-level inner forces failed (%d)" % rc)
        return tuple(out)

    def respa3(self, x, v, f_outer, f_m, f_p1, f_p2, counters, n_outer, dt, k, k_if, k_sub, level, brute=False,
               nthreads=1):
        """Advance (x, v) in place by n_outer outer steps of the three-level scheme (outer
        step k dt, interface step k_if dt, flowing sublevel k_sub dt, aggregating dt);
        the force arrays are updated in place; returns the counters."""
        cnt = np.ascontiguousarray(counters, dtype=np.uint64).copy()
        for a in (x, v, f_outer, f_m, f_p1, f_p2):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        lv = self._levels(level)
        rc = lib().or_respa3(self._sp(), x.ctypes.data, v.ctypes.data, f_outer.ctypes.data, f_m.ctypes.data,
                             f_p1.ctypes.data, f_p2.ctypes.data, cnt.ctypes.data, int(n_outer), float(dt), int(k),
                             int(k_if), int(k_sub), lv.ctypes.data, int(brute), int(nthreads))
        if rc:
            raise RuntimeError("oracle respa3 failed (%d)" % rc)
        return cnt

    def energy(self, x):
        """[U_dpd, U_lj, U_bond, U_angle, U_morse (bonds and Eq. 4 aggregation), pair virial];
        brute force, small N only."""
        out = np.zeros(6)
        lib().or_energy(self._sp(), np.ascontiguousarray(x, np.float64).ctypes.data, out.ctypes.data)
        return out

    def respa(self, x, v, f_outer, f_inner, counters, n_outer, dt_outer, k, brute=False, nthreads=1):
        """Advance (x, v) in place by ``n_outer`` RESPA outer steps; returns counters."""
        cnt = np.ascontiguousarray(counters, dtype=np.uint64).copy()
        for a in (x, v, f_outer, f_inner):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        rc = lib().or_respa(self._sp(), x.ctypes.data, v.ctypes.data, f_outer.ctypes.data, f_inner.ctypes.data,
                            cnt.ctypes.data, int(n_outer), float(dt_outer), int(k), int(brute), int(nthreads))
        if rc:
            raise RuntimeError("oracle respa failed (%d)" % rc)
        return cnt

    def thermo(self, x, v, bin_axis=1, n_bins=None):
        """[KE, T, T_peculiar, Px, Py, Pz]."""
        if n_bins is None:
            n_bins = max(1, int(np.floor(self.d["box_L"][bin_axis] / self.p["rc"])))
        out = np.zeros(6)
        lib().or_thermo(self._sp(), np.ascontiguousarray(x, np.float64).ctypes.data,
                        np.ascontiguousarray(v, np.float64).ctypes.data, int(bin_axis), int(n_bins), out.ctypes.data)
        return out

    def features(self, x, v, contact_r=1.0):
        P = int(self.d["n_platelet"])
        out = np.zeros((max(P, 1), 8))
        rc = lib().or_features(self._sp(), np.ascontiguousarray(x, np.float64).ctypes.data,
                               np.ascontiguousarray(v, np.float64).ctypes.data, 1, float(contact_r),
                               out.ctypes.data)
        if rc:
            raise RuntimeError("oracle features failed (%d)" % rc)
        return out[:P]

    def paper_features(self, x, v, flow_r=4.0):
        """[P, 6]: omega (3), translational and rotational kinetic energy, flow speed at
        the centre of mass (fluid within flow_r)."""
        P = int(self.d["n_platelet"])
        out = np.zeros((max(P, 1), 6))
        rc = lib().or_paper_features(self._sp(), np.ascontiguousarray(x, np.float64).ctypes.data,
                                     np.ascontiguousarray(v, np.float64).ctypes.data, float(flow_r), out.ctypes.data)
        if rc:
            raise RuntimeError("oracle paper features failed (%d)" % rc)
        return out[:P]

    def bead_stress(self, x, v):
        """[n_bead]: the per-bead pressure-like virial stress times volume (brute force)."""
        out = np.zeros(max(int(self.d["n_bead"]), 1))
        lib().or_bead_stress(self._sp(), np.ascontiguousarray(x, np.float64).ctypes.data,
                             np.ascontiguousarray(v, np.float64).ctypes.data, out.ctypes.data)
        return out[:int(self.d["n_bead"])]

    def pairs(self, x, n, cutoff, cells):
        x = np.ascontiguousarray(x, np.float64)
        fn = lib().or_pairs_cells if cells else lib().or_pairs_brute
        m = fn(self._sp(), x.ctypes.data, int(n), float(cutoff), None, 0)
        if m < 0:
            raise RuntimeError("cell list unavailable for this box")
        out = np.zeros((max(m, 1), 2), np.int64)
        fn(self._sp(), x.ctypes.data, int(n), float(cutoff), out.ctypes.data, m)
        return out[:m]


def num_threads() -> int:
    return int(lib().or_num_threads())
