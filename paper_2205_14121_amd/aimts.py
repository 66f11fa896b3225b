"""ctypes binding of libaimts.so (the C ABI in include/aimts.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels of the
library.  PyTorch supplies the device workspace and the HIP stream.  If the built
library is missing, importing this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaimts.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_UNSTABLE, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_HIP", -4: "E_UNSTABLE", -5: "E_STATE",
                -6: "E_UNSUPPORTED"}


class AimtsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class SystemDesc(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("L", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("force_precision", C.c_int32), ("n_fluid", C.c_int64), ("n_wall", C.c_int64),
                ("n_bead", C.c_int64), ("n_platelet", C.c_int64), ("n_bond", C.c_int64), ("n_angle", C.c_int64),
                ("n_morse", C.c_int64), ("cell_min", C.c_double), ("skin", C.c_double),
                ("inner_pair_capacity", C.c_int64), ("series_capacity", C.c_int64), ("ctrl_max_batch", C.c_int32),
                ("angle_pass", C.c_int32), ("seed", C.c_uint64), ("skin_bead", C.c_double),
                ("three_level", C.c_int32), ("reserved", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("dt_inner", C.c_double), ("k", C.c_int32), ("mode", C.c_int32), ("diag_every", C.c_int32),
                ("k_max", C.c_int32), ("rollback", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("ke", C.c_double), ("T", C.c_double),
                ("T_pec", C.c_double), ("p", C.c_double * 3), ("pe", C.c_double * 5), ("virial", C.c_double),
                ("k", C.c_int32), ("hold", C.c_int32), ("fallbacks", C.c_int32), ("inferences", C.c_int32),
                ("error_flags", C.c_uint32), ("energy_valid", C.c_int32), ("inner_members", C.c_int64),
                ("inner_pairs", C.c_int64), ("rollbacks", C.c_int32), ("rescanned", C.c_int32)]


def _load():
    # PyTorch ships its own HIP runtime under the same soname as the system one the
    # library links; load torch first so the process holds exactly one runtime (the one
    # that owns the device memory and streams handed to the library).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libaimts.so is not built (run __graft_entry__.build() or "
                           "python paper_2205_14121_amd/build.py); there is no fallback")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, F = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
    sig = {
        "aimts_workspace_size": [P, P],
        "aimts_create": [P, P, C.c_size_t, P, P],
        "aimts_destroy": [P],
        "aimts_set_state": [P, P, P],
        "aimts_set_masses": [P, P],
        "aimts_set_dpd": [P, D, D, D, D],
        "aimts_set_lj": [P, D, D, D, D],
        "aimts_set_interface": [P, D, D, D],
        "aimts_set_platelets": [P, P, P, P],
        "aimts_set_bonds": [P, I64, P, P, D],
        "aimts_set_angles": [P, I64, P, P, D],
        "aimts_set_morse": [P, I64, P, D, D, D],
        "aimts_set_aggregation": [P, D, D, D, D, D],
        "aimts_set_external": [P, P, I32, D, D],
        "aimts_set_counters": [P, C.c_uint64, C.c_uint64],
        "aimts_get_counters": [P, P, P],
        "aimts_compute_forces": [P, D, I32],
        "aimts_step": [P, I64, P],
        "aimts_get_state": [P, P, P],
        "aimts_get_forces": [P, P, P],
        "aimts_get_diag": [P, I32, P, P],
        "aimts_get_series": [P, P, I64, P],
        "aimts_get_feature_window": [P, P],
        "aimts_ctrl_num_params": [P],
        "aimts_ctrl_set_weights": [P, P, I64],
        "aimts_ctrl_get_weights": [P, P, I64],
        "aimts_ctrl_forward": [P, P, I32, P, P],
        "aimts_ctrl_backward": [P, P, P, I32, I32, P, P],
        "aimts_ctrl_train_step": [P, P, P, I32, I32, F, P],
        "aimts_ctrl_infer": [P, P, P],
        "aimts_ctrl_forward_static": [P, I64, P, I32, P, P, P],
        "aimts_get_paper_features": [P, D, P],
        "aimts_stress_sample": [P],
        "aimts_get_stress": [P, P, P, I32],
        "aimts_lstm_num_params": [P],
        "aimts_lstm_workspace_size": [I32, P],
        "aimts_lstm_filter": [P, P, I32, P, P],
        "aimts_lstm_forward": [P, P, I32, P, P, P, P, C.c_size_t, P],
        "aimts_lstm_backward": [P, P, P, I32, I32, P, P, P, C.c_size_t, P],
        "aimts_lstm_adam": [P, P, P, P, I32, I64, C.c_float, P],
        "aimts_profile": [P, I32],
        "aimts_set_levels": [P, I32, I32, P],
        "aimts_get_level_forces": [P, P, P, P],
        "aimts_get_levels": [P, P, P, P],
        "aimts_checkpoint_size": [P, P],
        "aimts_save_checkpoint": [P, P, C.c_size_t],
        "aimts_load_checkpoint": [P, P, C.c_size_t],
        "aimts_get_profile": [P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.aimts_last_error.argtypes = [P]
    L.aimts_last_error.restype = C.c_char_p
    return L


lib = _load()


def _p(a):
    """Host pointer of a C-contiguous numpy array (None for None)."""
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


def _check(ctx, status):
    if status != OK:
        raise AimtsError(status, lib.aimts_last_error(ctx).decode())


def desc_for(sysd, fp32=False, skin=0.4, series_capacity=0, ctrl_max_batch=0, inner_pair_capacity=0, skin_bead=0.0,
             angle_pass=0, three_level=False):
    """SystemDesc of a workload dict (see the ``synth`` module)."""
    d = SystemDesc()
    d.lo[:] = [float(q) for q in sysd["box_lo"]]
    d.L[:] = [float(q) for q in sysd["box_L"]]
    d.periodic[:] = [int(q) for q in sysd["periodic"]]
    d.force_precision = 1 if fp32 else 0
    d.n_fluid, d.n_wall, d.n_bead = int(sysd["n_fluid"]), int(sysd["n_wall"]), int(sysd["n_bead"])
    d.n_platelet = int(sysd["n_platelet"])
    d.n_bond, d.n_angle, d.n_morse = (int(sysd["bonds"].shape[0]), int(sysd["angles"].shape[0]),
                                      int(sysd["morse"].shape[0]))
    d.cell_min = float(sysd["params"]["rc"])
    d.skin = float(skin)
    d.skin_bead = float(skin_bead)
    d.inner_pair_capacity = int(inner_pair_capacity)
    d.series_capacity = int(series_capacity)
    d.ctrl_max_batch = int(ctrl_max_batch)
    d.angle_pass = int(angle_pass)
    d.seed = int(sysd["params"]["seed"])
    d.three_level = 1 if three_level else 0
    return d


class Context:
    """One aimts context: owns its torch workspace and uses the current torch stream."""

    def __init__(self, desc: SystemDesc, device="cuda"):
        import torch
        self.torch = torch
        self.desc = desc
        nbytes = C.c_size_t(0)
        _check(None, lib.aimts_workspace_size(C.byref(desc), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.workspace.device)
        ctx = C.c_void_p()
        _check(None, lib.aimts_create(C.byref(desc), C.c_void_p(aligned), nbytes.value,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.n = int(desc.n_fluid + desc.n_wall + desc.n_bead)

    def close(self):
        if self.ctx:
            lib.aimts_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- parameters and state ----
    def set_masses(self, m):
        _check(self.ctx, lib.aimts_set_masses(self.ctx, _p(np.ascontiguousarray(m, np.float64))))

    def set_dpd(self, a, gamma, sigma, rc):
        _check(self.ctx, lib.aimts_set_dpd(self.ctx, a, gamma, sigma, rc))

    def set_lj(self, eps, sig, rc_lj, r_excl):
        _check(self.ctx, lib.aimts_set_lj(self.ctx, eps, sig, rc_lj, r_excl))

    def set_interface(self, gamma_pf, sigma_pf, rc_pf):
        _check(self.ctx, lib.aimts_set_interface(self.ctx, gamma_pf, sigma_pf, rc_pf))

    def set_platelets(self, body, rest, area):
        _check(self.ctx, lib.aimts_set_platelets(self.ctx, _p(np.ascontiguousarray(body, np.int32)),
                                                 _p(np.ascontiguousarray(rest, np.float64)),
                                                 _p(np.ascontiguousarray(area, np.float64))))

    def set_bonds(self, ij, r0, k):
        ij = np.ascontiguousarray(ij, np.int32)
        _check(self.ctx, lib.aimts_set_bonds(self.ctx, ij.shape[0], _p(ij), _p(np.ascontiguousarray(r0, np.float64)), k))

    def set_angles(self, ijk, th0, k):
        ijk = np.ascontiguousarray(ijk, np.int32)
        _check(self.ctx, lib.aimts_set_angles(self.ctx, ijk.shape[0], _p(ijk),
                                              _p(np.ascontiguousarray(th0, np.float64)), k))

    def set_morse(self, ij, D, a, r0):
        ij = np.ascontiguousarray(ij, np.int32)
        _check(self.ctx, lib.aimts_set_morse(self.ctx, ij.shape[0], _p(ij), D, a, r0))

    def set_aggregation(self, D, a, r0, fA, rc):
        _check(self.ctx, lib.aimts_set_aggregation(self.ctx, float(D), float(a), float(r0), float(fA), float(rc)))

    def set_external(self, g, wall_axis, wall_lo, wall_hi):
        _check(self.ctx, lib.aimts_set_external(self.ctx, _p(np.ascontiguousarray(g, np.float64)), int(wall_axis),
                                                float(wall_lo), float(wall_hi)))

    def set_state(self, x, v):
        _check(self.ctx, lib.aimts_set_state(self.ctx, _p(np.ascontiguousarray(x, np.float64)),
                                             _p(np.ascontiguousarray(v, np.float64))))

    def set_counters(self, outer, inner):
        _check(self.ctx, lib.aimts_set_counters(self.ctx, int(outer), int(inner)))

    def counters(self):
        a, b = C.c_uint64(0), C.c_uint64(0)
        _check(self.ctx, lib.aimts_get_counters(self.ctx, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    # ---- hot path ----
    def compute_forces(self, dt_inner, k):
        _check(self.ctx, lib.aimts_compute_forces(self.ctx, float(dt_inner), int(k)))

    def step(self, n_outer, dt_inner, k, mode=0, diag_every=0, k_max=0, rollback=0):
        sch = Schedule(float(dt_inner), int(k), int(mode), int(diag_every), int(k_max), int(rollback))
        _check(self.ctx, lib.aimts_step(self.ctx, int(n_outer), C.byref(sch)))

    def step_status(self, n_outer, dt_inner, k, mode=0, diag_every=0, k_max=0, rollback=0):
        """Like step() but returns the status code instead of raising."""
        sch = Schedule(float(dt_inner), int(k), int(mode), int(diag_every), int(k_max), int(rollback))
        return lib.aimts_step(self.ctx, int(n_outer), C.byref(sch))

    # ---- read back ----
    def state(self):
        x = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        _check(self.ctx, lib.aimts_get_state(self.ctx, _p(x), _p(v)))
        return x, v

    def forces(self):
        fo = np.zeros((self.n, 3))
        fi = np.zeros((self.n, 3))
        _check(self.ctx, lib.aimts_get_forces(self.ctx, _p(fo), _p(fi)))
        return fo, fi

    def diag(self, energy=False, features=False):
        d = Diag()
        P = int(self.desc.n_platelet)
        feat = np.zeros((max(P, 1), 8), np.float32) if features else None
        _check(self.ctx, lib.aimts_get_diag(self.ctx, 1 if energy else 0, C.byref(d), _p(feat)))
        return (d, feat[:P]) if features else d

    def series(self, max_rows=None):
        cap = int(self.desc.series_capacity) if max_rows is None else int(max_rows)
        rows = np.zeros((max(cap, 1), 8))
        cnt = C.c_int64(0)
        _check(self.ctx, lib.aimts_get_series(self.ctx, _p(rows), cap, C.byref(cnt)))
        return rows[:min(cap, int(cnt.value))]

    def feature_window(self):
        P = int(self.desc.n_platelet)
        w = np.zeros((P, 64, 8), np.float32)
        _check(self.ctx, lib.aimts_get_feature_window(self.ctx, _p(w)))
        return w

    # ---- three-level MTS (include/aimts.h: aimts_set_levels) ----
    def set_levels(self, k_if, k_sub, level=None):
        lv = None if level is None else np.ascontiguousarray(level, np.int32)
        _check(self.ctx, lib.aimts_set_levels(self.ctx, int(k_if), int(k_sub), _p(lv)))

    def levels(self):
        a, b = C.c_int32(0), C.c_int32(0)
        lv = np.zeros(max(int(self.desc.n_platelet), 1), np.int32)
        _check(self.ctx, lib.aimts_get_levels(self.ctx, C.byref(a), C.byref(b), _p(lv)))
        return int(a.value), int(b.value), lv[:int(self.desc.n_platelet)]

    def level_forces(self):
        out = [np.zeros((self.n, 3)) for _ in range(3)]
        _check(self.ctx, lib.aimts_get_level_forces(self.ctx, *[_p(o) for o in out]))
        return tuple(out)

    # ---- checkpoint and resume ----
    def save_checkpoint(self):
        """Everything a later step depends on, as a host byte array (see include/aimts.h)."""
        n = C.c_size_t(0)
        _check(self.ctx, lib.aimts_checkpoint_size(self.ctx, C.byref(n)))
        buf = np.zeros(int(n.value), np.uint8)
        _check(self.ctx, lib.aimts_save_checkpoint(self.ctx, _p(buf), buf.size))
        return buf

    def load_checkpoint(self, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(self.ctx, lib.aimts_load_checkpoint(self.ctx, _p(buf), buf.size))

    def paper_features(self, flow_r=4.0):
        """[P, 6]: the paper's six measurements per platelet at the current state."""
        out = np.zeros((max(int(self.desc.n_platelet), 1), 6))
        _check(self.ctx, lib.aimts_get_paper_features(self.ctx, float(flow_r), _p(out)))
        return out[:int(self.desc.n_platelet)]

    def stress_sample(self):
        _check(self.ctx, lib.aimts_stress_sample(self.ctx))

    def stress(self, reset=False):
        """(mean per-bead membrane stress [n_bead], number of samples)."""
        out = np.zeros(max(int(self.desc.n_bead), 1))
        n = C.c_int64()
        _check(self.ctx, lib.aimts_get_stress(self.ctx, _p(out), C.byref(n), int(bool(reset))))
        return out[:int(self.desc.n_bead)], int(n.value)

    PROFILE_PHASES = ("outer_forces", "inner_loop", "cell_sort", "outer_kicks", "diagnostics", "platelet_lists")

    def profile(self, mask):
        """Start HIP-event timing of the phases in ``mask`` (bit q = PROFILE_PHASES[q]); 0 stops."""
        _check(self.ctx, lib.aimts_profile(self.ctx, int(mask)))

    def get_profile(self):
        ms = np.zeros(6)
        cnt = np.zeros(6, np.int64)
        _check(self.ctx, lib.aimts_get_profile(self.ctx, _p(ms), _p(cnt)))
        return ms, cnt

    def last_error(self):
        return lib.aimts_last_error(self.ctx).decode()

    # ---- controller ----
    @staticmethod
    def ctrl_num_params():
        n = C.c_int64(0)
        _check(None, lib.aimts_ctrl_num_params(C.byref(n)))
        return int(n.value)

    def ctrl_set_weights(self, params):
        p = np.ascontiguousarray(params, np.float32)
        _check(self.ctx, lib.aimts_ctrl_set_weights(self.ctx, _p(p), p.size))

    def ctrl_get_weights(self):
        p = np.zeros(self.ctrl_num_params(), np.float32)
        _check(self.ctx, lib.aimts_ctrl_get_weights(self.ctx, _p(p), p.size))
        return p

    def ctrl_forward(self, d_windows, d_latent=None, d_logits=None):
        B = int(d_windows.shape[0])
        _check(self.ctx, lib.aimts_ctrl_forward(self.ctx, d_windows.data_ptr(), B,
                                                None if d_latent is None else d_latent.data_ptr(),
                                                None if d_logits is None else d_logits.data_ptr()))

    def ctrl_backward(self, d_windows, d_labels, phase, d_grads):
        B = int(d_windows.shape[0])
        loss = C.c_float(0.0)
        _check(self.ctx, lib.aimts_ctrl_backward(self.ctx, d_windows.data_ptr(),
                                                 None if d_labels is None else d_labels.data_ptr(), B, int(phase),
                                                 d_grads.data_ptr(), C.byref(loss)))
        return float(loss.value)

    def ctrl_train_step(self, d_windows, d_labels, phase, lr):
        B = int(d_windows.shape[0])
        loss = C.c_float(0.0)
        _check(self.ctx, lib.aimts_ctrl_train_step(self.ctx, d_windows.data_ptr(),
                                                   None if d_labels is None else d_labels.data_ptr(), B, int(phase),
                                                   float(lr), C.byref(loss)))
        return float(loss.value)

    def ctrl_infer(self):
        k, h = C.c_int32(0), C.c_int32(0)
        _check(self.ctx, lib.aimts_ctrl_infer(self.ctx, C.byref(k), C.byref(h)))
        return int(k.value), int(h.value)


CTRL_STATIC_MAX_BATCH = 256


def ctrl_forward_static(d_params, d_windows, d_latent=None, d_logits=None, stream=None):
    """aimts_ctrl_forward_static: the controller's forward pass without a context, on a
    device float32 parameter vector, with the library's static device scratch (no
    allocation).  Queued on `stream` (default: torch's current stream); asynchronous."""
    import torch
    st = torch.cuda.current_stream(d_windows.device) if stream is None else stream
    _check(None, lib.aimts_ctrl_forward_static(d_params.data_ptr(), int(d_params.numel()), d_windows.data_ptr(),
                                               int(d_windows.shape[0]),
                                               None if d_latent is None else d_latent.data_ptr(),
                                               None if d_logits is None else d_logits.data_ptr(),
                                               C.c_void_p(st.cuda_stream)))


class LstmPipeline:
    """The paper's own inference pipeline (MA + Haar wavelet filter, 2-layer LSTM
    autoencoder 16/4 with 8 latents, FCN 32-16-8-1) on torch device tensors; marshalling
    only, every step runs in the library's kernels.  Calls are queued on torch's current
    stream."""

    def __init__(self, max_batch):
        import torch
        n = C.c_int64()
        _check(None, lib.aimts_lstm_num_params(C.byref(n)))
        self.n_params = int(n.value)
        b = C.c_size_t()
        _check(None, lib.aimts_lstm_workspace_size(int(max_batch), C.byref(b)))
        self.max_batch = int(max_batch)
        self.ws_bytes = int(b.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _st():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _batch(self, windows):
        B = int(windows.shape[0])
        if B > self.max_batch:
            raise ValueError("batch %d exceeds the workspace's %d" % (B, self.max_batch))
        return B

    def filter(self, params, windows):
        import torch
        out = torch.empty_like(windows)
        _check(None, lib.aimts_lstm_filter(params.data_ptr(), windows.data_ptr(), int(windows.shape[0]),
                                           out.data_ptr(), self._st()))
        return out

    def forward(self, params, windows, recon=False):
        import torch
        B = self._batch(windows)
        lat = torch.empty((B, 8), dtype=torch.float32, device="cuda")
        pred = torch.empty(B, dtype=torch.float32, device="cuda")
        rec = torch.empty((B, 50, 6), dtype=torch.float32, device="cuda") if recon else None
        _check(None, lib.aimts_lstm_forward(params.data_ptr(), windows.data_ptr(), B, lat.data_ptr(), pred.data_ptr(),
                                            None if rec is None else rec.data_ptr(), self.ws.data_ptr(),
                                            self.ws_bytes, self._st()))
        return lat, pred, rec

    def backward(self, params, windows, targets, phase):
        import torch
        B = self._batch(windows)
        grad = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(None, lib.aimts_lstm_backward(params.data_ptr(), windows.data_ptr(),
                                             None if targets is None else targets.data_ptr(), B, int(phase),
                                             grad.data_ptr(), loss.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                             self._st()))
        return grad, loss

    def adam(self, params, m, v, grad, phase, step, lr):
        _check(None, lib.aimts_lstm_adam(params.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(), int(phase),
                                         int(step), float(lr), self._st()))


def from_workload(sysd, fp32=False, skin=0.4, series_capacity=0, ctrl_max_batch=0, params=None,
                  inner_pair_capacity=0, skin_bead=0.0, angle_pass=0, three_level=False):
    """Create a context for a workload dict, set every parameter, topology and state."""
    p = dict(sysd["params"])
    if params:
        p.update(params)
    if inner_pair_capacity == 0 and p.get("agg_rc", 0.0) > 0.0 and sysd["n_bead"] > 0:
        # the automatic capacity (~96 (cutoff + skin)^3 entries per bead) at the longer
        # reach of the aggregation term
        reach = max(float(p["rc"]), float(p["agg_rc"])) + max(float(skin), float(skin_bead))
        inner_pair_capacity = int(np.ceil(96.0 * reach ** 3)) * int(sysd["n_bead"])
    ctx = Context(desc_for(sysd, fp32=fp32, skin=skin, series_capacity=series_capacity,
                           ctrl_max_batch=ctrl_max_batch, inner_pair_capacity=inner_pair_capacity,
                           skin_bead=skin_bead, angle_pass=angle_pass, three_level=three_level))
    ctx.set_masses(p["mass"])
    ctx.set_dpd(p["a"], p["gamma"], p["sigma"], p["rc"])
    if sysd["n_bead"] > 0:
        ctx.set_lj(p["lj_eps"], p["lj_sig"], p["lj_rc"], p["r_excl"])
        ctx.set_interface(p["gamma_pf"], p["sigma_pf"], p["rc_pf"])
        ctx.set_platelets(sysd["body"], sysd["rest"], sysd["platelet_area"])
        ctx.set_bonds(sysd["bonds"], sysd["bond_r0"], p["kb"])
        ctx.set_angles(sysd["angles"], sysd["angle_th0"], p["ka"])
        ctx.set_morse(sysd["morse"], p["morse_D"], p["morse_a"], p["morse_r0"])
        if p.get("agg_rc", 0.0) > 0.0:
            ctx.set_aggregation(p["agg_D"], p["agg_a"], p["agg_r0"], p["agg_fA"], p["agg_rc"])
    ctx.set_external(p["g"], p["wall_axis"], p["wall_lo"], p["wall_hi"])
    ctx.set_state(sysd["x"], sysd["v"])
    return ctx
