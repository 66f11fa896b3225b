"""Seeded synthetic inputs for the DPD + CGMD blood-clot hot path.

This module builds initial states and topologies only: particle positions and
velocities, the icosphere platelet mesh with its rest lengths and rest angles,
and the force-field parameters of each workload.  It contains none of the
method's arithmetic (no force law, no integrator, no random force) and is the
one module that both the HIP path's callers and the CPU oracle read.

Workloads (sizes from the paper's hot-path configurations):
  * ``dpd_box``      -- plain DPD fluid, 3,000 particles at density 3 in a periodic
                        10^3 box (a=25, gamma=4.5, sigma=3, kT=1, dt=0.01).
  * ``platelet_box`` -- 24,000 DPD particles in a periodic 20^3 box plus one
                        oblate icosphere platelet (level 4, 2,562 beads).
  * ``channel``      -- Poiseuille channel: frozen wall layers in y, body force
                        in x, several randomly placed platelets.

Particle order is always fluid, then wall, then beads (platelet by platelet).
The platelet mesh is an icosahedron refined by midpoint subdivision, projected
onto the unit sphere and scaled to an oblate ellipsoid whose short axis lies
along y in the body frame (the paper's platelets are discoid, Sec. 3.2).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosphere", "platelet_template", "dpd_params", "dpd_box", "platelet_box", "channel", "aggregate_box",
    "morse_bonds", "maxwell", "random_rotation",
]


# --------------------------------------------------------------------------
# Mesh
# --------------------------------------------------------------------------
def icosphere(level: int):
    """Icosahedron refined ``level`` times by edge midpoints, on the unit sphere.

    Returns (verts [V,3] float64, faces [F,3] int64) with V = 10*4^n + 2 and
    F = 20*4^n; vertex order is deterministic.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int64)


def platelet_template(level: int = 4, semi_axes=(3.0, 1.0, 3.0)):
    """Rest mesh of one platelet in its body frame.

    ``semi_axes`` are along (x, y, z); the default puts the short axis along y.
    Returns a dict with rest coordinates, edge list (bonds) with rest lengths,
    the three corner angles of every face with rest angles (radians), the faces
    and the rest surface area.
    """
    v, f = icosphere(level)
    rest = v * np.asarray(semi_axes, dtype=np.float64)[None, :]
    edges = set()
    for a, b, c in f:
        for p, q in ((a, b), (b, c), (c, a)):
            edges.add((min(p, q), max(p, q)))
    edges = np.array(sorted(edges), dtype=np.int64)
    r0 = np.linalg.norm(rest[edges[:, 0]] - rest[edges[:, 1]], axis=1)
    # corner angles: (end, vertex, end) for the corner at each vertex of each face
    ang = np.concatenate([f[:, [1, 0, 2]], f[:, [0, 1, 2]], f[:, [0, 2, 1]]], axis=0)
    ang = ang[np.lexsort((ang[:, 2], ang[:, 0], ang[:, 1]))]
    u = rest[ang[:, 0]] - rest[ang[:, 1]]
    w = rest[ang[:, 2]] - rest[ang[:, 1]]
    cosv = np.sum(u * w, axis=1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(w, axis=1))
    th0 = np.arccos(np.clip(cosv, -1.0, 1.0))
    tri = np.cross(rest[f[:, 1]] - rest[f[:, 0]], rest[f[:, 2]] - rest[f[:, 0]])
    area = 0.5 * float(np.sum(np.linalg.norm(tri, axis=1)))
    return {"rest": rest, "bonds": edges, "bond_r0": r0, "angles": ang, "angle_th0": th0,
            "faces": f, "area": area}


# --------------------------------------------------------------------------
# Random helpers
# --------------------------------------------------------------------------
def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix (from a normalised Gaussian quaternion)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def maxwell(rng: np.random.Generator, n: int, kT: float = 1.0, mass: float = 1.0) -> np.ndarray:
    """Maxwell-Boltzmann velocities with the mean removed."""
    v = rng.standard_normal((n, 3)) * math.sqrt(kT / mass)
    if n > 0:
        v -= v.mean(axis=0, keepdims=True)
    return v


def dpd_params(**over):
    """Force-field parameters shared by all workloads (overridable)."""
    p = dict(a=25.0, gamma=4.5, sigma=3.0, rc=1.0, kT=1.0,
             mass=(1.0, 1.0, 1.0),
             lj_eps=1.0, lj_sig=0.8, lj_rc=0.8 * 2.0 ** (1.0 / 6.0),
             gamma_pf=4.5, sigma_pf=3.0, rc_pf=1.0,
             kb=100.0, ka=20.0,
             morse_D=5.0, morse_a=2.0, morse_r0=1.0,
             # inter-platelet aggregation of Eq. 4 (non-bonded Morse + receptor term):
             # off unless agg_rc > 0
             agg_D=5.0, agg_a=2.0, agg_r0=1.0, agg_fA=10.0, agg_rc=0.0,
             r_excl=1.5, g=(0.0, 0.0, 0.0),
             wall_axis=-1, wall_lo=0.0, wall_hi=0.0,
             seed=20220528)
    p.update(over)
    return p


def _empty_topology():
    return {"body": np.zeros(0, np.int32), "rest": np.zeros((0, 3)),
            "bonds": np.zeros((0, 2), np.int32), "bond_r0": np.zeros(0),
            "angles": np.zeros((0, 3), np.int32), "angle_th0": np.zeros(0),
            "morse": np.zeros((0, 2), np.int32), "platelet_area": np.zeros(0)}


def _finish(sysd):
    for k in ("x", "v", "rest", "bond_r0", "angle_th0", "platelet_area"):
        sysd[k] = np.ascontiguousarray(sysd[k], dtype=np.float64)
    for k in ("body", "bonds", "angles", "morse"):
        sysd[k] = np.ascontiguousarray(sysd[k], dtype=np.int32)
    sysd["n"] = sysd["n_fluid"] + sysd["n_wall"] + sysd["n_bead"]
    assert sysd["x"].shape == (sysd["n"], 3) and sysd["v"].shape == (sysd["n"], 3)
    return sysd


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def dpd_box(n: int = 3000, L=(10.0, 10.0, 10.0), seed: int = 20220528, **over):
    """Plain periodic DPD fluid: uniform positions, Maxwell velocities."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    x = rng.random((n, 3)) * L[None, :]
    p = dpd_params(seed=seed, **over)
    v = maxwell(rng, n, p["kT"], p["mass"][0])
    sysd = dict(_empty_topology(), box_lo=np.zeros(3), box_L=L, periodic=(1, 1, 1),
                n_fluid=n, n_wall=0, n_bead=0, n_platelet=0, x=x, v=v, params=p,
                schedule=dict(dt_outer=0.01, k=1))
    return _finish(sysd)


def _place_platelets(tmpl, centres, rotations, b0):
    rest, nv = tmpl["rest"], tmpl["rest"].shape[0]
    xs, bodies, bonds, angles, r0s, th0s = [], [], [], [], [], []
    for p, (c, R) in enumerate(zip(centres, rotations)):
        xs.append(rest @ R.T + c[None, :])
        bodies.append(np.full(nv, p, np.int32))
        off = b0 + p * nv
        bonds.append(tmpl["bonds"] + off)
        angles.append(tmpl["angles"] + off)
        r0s.append(tmpl["bond_r0"])
        th0s.append(tmpl["angle_th0"])
    P = len(centres)
    return (np.concatenate(xs), np.concatenate(bodies), np.tile(rest, (P, 1)),
            np.concatenate(bonds), np.concatenate(r0s), np.concatenate(angles), np.concatenate(th0s))


def _fluid_away_from(rng, n, lo, hi, beads, min_dist, L, periodic):
    """n uniform points in [lo, hi) that keep ``min_dist`` from every bead (redraws)."""
    from scipy.spatial import cKDTree
    if beads.shape[0] == 0:
        return lo[None, :] + rng.random((n, 3)) * (hi - lo)[None, :]
    # periodic axes wrap; a non-periodic axis gets a box ten times its length so
    # that no image is ever closer than a real neighbour
    boxsize = np.array([L[k] if periodic[k] else 10.0 * L[k] for k in range(3)])
    tree = cKDTree(np.mod(beads, boxsize), boxsize=boxsize)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        need = n - out.shape[0]
        cand = lo[None, :] + rng.random((int(need * 1.05) + 16, 3)) * (hi - lo)[None, :]
        d, _ = tree.query(np.mod(cand, boxsize), k=1, distance_upper_bound=min_dist)
        out = np.concatenate([out, cand[d >= min_dist]])
    return out[:n]


def platelet_box(n_fluid: int = 24000, L=(20.0, 20.0, 20.0), level: int = 4, seed: int = 20220529,
                 semi_axes=(3.0, 1.0, 3.0), **over):
    """Periodic DPD box with one platelet at its centre (rest shape, body frame axes)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    p = dpd_params(seed=seed, **over)
    tmpl = platelet_template(level, semi_axes)
    b0 = n_fluid
    xb, body, rest, bonds, r0, angles, th0 = _place_platelets(tmpl, [L / 2.0], [np.eye(3)], b0)
    xf = _fluid_away_from(rng, n_fluid, np.zeros(3), L, xb, p["lj_sig"], L, (1, 1, 1))
    x = np.concatenate([xf, xb])
    v = maxwell(rng, x.shape[0], p["kT"], 1.0)
    sysd = dict(box_lo=np.zeros(3), box_L=L, periodic=(1, 1, 1), n_fluid=n_fluid, n_wall=0,
                n_bead=xb.shape[0], n_platelet=1, x=x, v=v, body=body, rest=rest, bonds=bonds,
                bond_r0=r0, angles=angles, angle_th0=th0, morse=np.zeros((0, 2), np.int32),
                platelet_area=np.array([tmpl["area"]]), params=p,
                schedule=dict(dt_outer=0.01, k=4))
    return _finish(sysd)


def channel(n_total: int = 2_000_000, L=(200.0, 50.0, 66.7), n_platelet: int = 4, level: int = 4,
            seed: int = 20220530, g: float = 0.02, wall_thickness: float = 1.0,
            semi_axes=(3.0, 1.0, 3.0), density: float = 3.0, **over):
    """Poiseuille channel: frozen wall layers at both ends of y, periodic x and z,
    body force ``g`` along x on the fluid, ``n_platelet`` randomly oriented
    platelets whose bounding spheres (radius max(semi_axes) + 1) are disjoint and
    clear of the wall layers by at least 1.

    ``n_total`` counts fluid + wall particles; beads come on top.
    """
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    wall_hi = L[1] - wall_thickness
    p = dpd_params(seed=seed, g=(g, 0.0, 0.0), wall_axis=1, wall_lo=wall_thickness, wall_hi=wall_hi, **over)
    n_wall = int(round(density * 2.0 * wall_thickness * L[0] * L[2]))
    n_fluid = n_total - n_wall
    tmpl = platelet_template(level, semi_axes)
    rad = max(semi_axes) + 1.0
    centres = []
    tries = 0
    while len(centres) < n_platelet:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place platelets without overlap")
        c = np.array([rng.random() * L[0],
                      wall_thickness + 1.0 + rad + rng.random() * (L[1] - 2 * (wall_thickness + 1.0 + rad)),
                      rng.random() * L[2]])
        ok = True
        for q in centres:
            d = c - q
            d[0] -= L[0] * round(d[0] / L[0])
            d[2] -= L[2] * round(d[2] / L[2])
            if np.linalg.norm(d) < 2 * rad:
                ok = False
                break
        if ok:
            centres.append(c)
    rots = [random_rotation(rng) for _ in centres]
    b0 = n_total
    if n_platelet > 0:
        xb, body, rest, bonds, r0, angles, th0 = _place_platelets(tmpl, centres, rots, b0)
        xb[:, 0] = np.mod(xb[:, 0], L[0])
        xb[:, 2] = np.mod(xb[:, 2], L[2])
    else:
        t = _empty_topology()
        xb, body, rest, bonds, r0, angles, th0 = (np.zeros((0, 3)), t["body"], t["rest"], t["bonds"],
                                                  t["bond_r0"], t["angles"], t["angle_th0"])
    lo_f = np.array([0.0, wall_thickness, 0.0])
    hi_f = np.array([L[0], wall_hi, L[2]])
    xf = _fluid_away_from(rng, n_fluid, lo_f, hi_f, xb, p["lj_sig"], L, (1, 0, 1))
    n_lo = n_wall // 2
    xw_lo = np.array([0.0, 0.0, 0.0])[None, :] + rng.random((n_lo, 3)) * np.array([L[0], wall_thickness, L[2]])
    xw_hi = np.array([0.0, wall_hi, 0.0])[None, :] + rng.random((n_wall - n_lo, 3)) * np.array(
        [L[0], wall_thickness, L[2]])
    x = np.concatenate([xf, xw_lo, xw_hi, xb])
    v = np.zeros_like(x)
    mob = np.r_[np.arange(n_fluid), np.arange(n_total, x.shape[0])]
    v[mob] = maxwell(rng, mob.size, p["kT"], 1.0)
    sysd = dict(box_lo=np.zeros(3), box_L=L, periodic=(1, 0, 1), n_fluid=n_fluid, n_wall=n_wall,
                n_bead=xb.shape[0], n_platelet=n_platelet, x=x, v=v, body=body, rest=rest, bonds=bonds,
                bond_r0=r0, angles=angles, angle_th0=th0, morse=np.zeros((0, 2), np.int32),
                platelet_area=np.full(n_platelet, tmpl["area"]), params=p,
                schedule=dict(dt_outer=0.01, k=4))
    return _finish(sysd)


def _fluid_away_from_sparse(rng, n, lo, hi, beads, min_dist, L, periodic, chunk=8_000_000):
    """Like _fluid_away_from for large n: candidates are drawn in chunks and only those in
    grid cells (side >= min_dist) next to a bead are checked against the beads."""
    from scipy.spatial import cKDTree
    side = max(min_dist, 1.0)
    nc = np.maximum((L / side).astype(np.int64), 1)
    cell = lambda p: tuple(np.minimum((np.mod(p, L) / (L / nc)).astype(np.int64), nc - 1).T)
    near = np.zeros(tuple(nc), dtype=bool)
    if beads.shape[0]:
        bc = np.stack(cell(beads), axis=1)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    q = bc + np.array([dx, dy, dz])
                    q = np.mod(q, nc)
                    near[q[:, 0], q[:, 1], q[:, 2]] = True
    boxsize = np.array([L[k] if periodic[k] else 10.0 * L[k] for k in range(3)])
    tree = cKDTree(np.mod(beads, boxsize), boxsize=boxsize) if beads.shape[0] else None
    out = np.empty((n, 3))
    got = 0
    while got < n:
        m = min(chunk, int((n - got) * 1.02) + 16)
        cand = lo[None, :] + rng.random((m, 3)) * (hi - lo)[None, :]
        if tree is not None:
            chk = near[cell(cand)]
            if chk.any():
                d, _ = tree.query(np.mod(cand[chk], boxsize), k=1, distance_upper_bound=min_dist)
                keep = np.ones(m, dtype=bool)
                keep[np.flatnonzero(chk)[d < min_dist]] = False
                cand = cand[keep]
        take = min(cand.shape[0], n - got)
        out[got:got + take] = cand[:take]
        got += take
    return out


def mutual_nearest_bonds(xb, body, r_bond, L=None, periodic=(0, 0, 0)):
    """Inter-platelet binding list for large aggregates: bead pairs of different
    platelets that are each other's nearest bead on another platelet and closer than
    `r_bond` (each bead in at most one bond).  Indices are bead indices; `body` must
    group the beads platelet by platelet."""
    from scipy.spatial import cKDTree
    nb = xb.shape[0]
    if nb == 0:
        return np.zeros((0, 2), np.int64)
    bodies = np.unique(body)
    start = {int(q): int(np.flatnonzero(body == q)[0]) for q in bodies}
    if L is not None:
        boxsize = np.array([L[k] if periodic[k] else 10.0 * L[k] for k in range(3)])
        pos = np.mod(xb, boxsize)
    else:
        boxsize, pos = None, xb
    trees = {int(q): cKDTree(pos[body == q], boxsize=boxsize) for q in bodies}
    cen = {int(q): pos[body == q].mean(axis=0) for q in bodies}
    best_d = np.full(nb, np.inf)
    best_j = np.full(nb, -1, np.int64)
    ext = max(float(np.ptp(pos[body == bodies[0]], axis=0).max()), 0.0) + r_bond
    for q in bodies:
        mine = np.flatnonzero(body == q)
        for o in bodies:
            if o == q:
                continue
            dc = cen[int(o)] - cen[int(q)]
            if boxsize is not None:
                dc -= boxsize * np.round(dc / boxsize)
            if np.linalg.norm(dc) > ext:
                continue
            d, j = trees[int(o)].query(pos[mine], k=1, distance_upper_bound=r_bond)
            better = d < best_d[mine]
            best_d[mine[better]] = d[better]
            best_j[mine[better]] = j[better] + start[int(o)]
    i = np.flatnonzero(best_j >= 0)
    mutual = best_j[best_j[i]] == i
    a = i[mutual]
    b = best_j[a]
    keep = a < b
    return np.stack([a[keep], b[keep]], axis=1).astype(np.int64)


def clot_channel(n_total: int = 100_000_000, L=(3000.0, 300.0, 37.0), n_free: int = 70, n_packed: int = 180,
                 level: int = 5, seed: int = 20220534, g: float = 0.02, wall_thickness: float = 1.0,
                 semi_axes=(3.0, 1.0, 3.0), density: float = 3.0, packed_grid=(9, 4, 5),
                 packed_spacing=(7.0, 3.0, 7.4), morse_cut=1.5, **over):
    """Largest single-GPU system: a long channel (walls in y, periodic x and z, body force
    g along x) with `n_free` randomly placed and oriented platelets and `n_packed`
    platelets pre-packed as an aggregate on the lower wall (lying flat on a lattice of
    `packed_grid` with centre spacing `packed_spacing`), bound by inter-platelet Morse
    bonds between mutually nearest beads of different platelets closer than
    morse_cut * morse_r0.  ``n_total`` counts fluid + wall particles; beads come on top.
    """
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    wall_hi = L[1] - wall_thickness
    p = dpd_params(seed=seed, g=(g, 0.0, 0.0), wall_axis=1, wall_lo=wall_thickness, wall_hi=wall_hi, **over)
    n_wall = int(round(density * 2.0 * wall_thickness * L[0] * L[2]))
    n_fluid = n_total - n_wall
    tmpl = platelet_template(level, semi_axes)
    nx, ny, nz = packed_grid
    assert nx * ny * nz == n_packed
    # the aggregate: lattice on the lower wall, centred in x
    y0 = wall_thickness + semi_axes[1] + 1.0  # beyond the WCA reach of the wall particles
    packed = []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                packed.append(np.array([0.5 * L[0] + (ix - (nx - 1) / 2) * packed_spacing[0],
                                        y0 + iy * packed_spacing[1],
                                        (iz + 0.5) * packed_spacing[2]]))
    rad = max(semi_axes) + 1.0
    agg_lo = np.array([0.5 * L[0] - (nx / 2) * packed_spacing[0] - rad, 0.0])
    agg_hi = np.array([0.5 * L[0] + (nx / 2) * packed_spacing[0] + rad, y0 + ny * packed_spacing[1] + rad])
    free = []
    tries = 0
    while len(free) < n_free:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("cannot place the free platelets")
        c = np.array([rng.random() * L[0],
                      wall_thickness + 1.0 + rad + rng.random() * (L[1] - 2 * (wall_thickness + 1.0 + rad)),
                      rng.random() * L[2]])
        if agg_lo[0] - rad < c[0] < agg_hi[0] + rad and c[1] < agg_hi[1] + rad:
            continue
        ok = True
        for q in free:
            dd = c - q
            dd[0] -= L[0] * round(dd[0] / L[0])
            dd[2] -= L[2] * round(dd[2] / L[2])
            if np.linalg.norm(dd) < 2 * rad:
                ok = False
                break
        if ok:
            free.append(c)
    centres = free + packed
    rots = [random_rotation(rng) for _ in free] + [np.eye(3)] * len(packed)
    b0 = n_total
    xb, body, rest, bonds, r0, angles, th0 = _place_platelets(tmpl, centres, rots, b0)
    xb[:, 0] = np.mod(xb[:, 0], L[0])
    xb[:, 2] = np.mod(xb[:, 2], L[2])
    nfree_beads = n_free * tmpl["rest"].shape[0]
    mb = mutual_nearest_bonds(xb[nfree_beads:], body[nfree_beads:], morse_cut * p["morse_r0"], L, (1, 0, 1))
    mb = mb + nfree_beads + b0
    lo_f = np.array([0.0, wall_thickness, 0.0])
    hi_f = np.array([L[0], wall_hi, L[2]])
    xf = _fluid_away_from_sparse(rng, n_fluid, lo_f, hi_f, xb, p["lj_sig"], L, (1, 0, 1))
    n_lo = n_wall // 2
    xw_lo = rng.random((n_lo, 3)) * np.array([L[0], wall_thickness, L[2]])
    xw_hi = np.array([0.0, wall_hi, 0.0])[None, :] + rng.random((n_wall - n_lo, 3)) * np.array(
        [L[0], wall_thickness, L[2]])
    x = np.concatenate([xf, xw_lo, xw_hi, xb])
    del xf, xw_lo, xw_hi
    v = np.zeros_like(x)
    v[:n_fluid] = maxwell(rng, n_fluid, p["kT"], 1.0)
    v[n_total:] = maxwell(rng, x.shape[0] - n_total, p["kT"], 1.0)
    P = len(centres)
    sysd = dict(box_lo=np.zeros(3), box_L=L, periodic=(1, 0, 1), n_fluid=n_fluid, n_wall=n_wall,
                n_bead=xb.shape[0], n_platelet=P, x=x, v=v, body=body, rest=rest, bonds=bonds,
                bond_r0=r0, angles=angles, angle_th0=th0, morse=mb.astype(np.int32),
                platelet_area=np.full(P, tmpl["area"]), params=p, schedule=dict(dt_outer=0.01, k=4))
    return _finish(sysd)


def morse_bonds(xb, body, r_bond):
    """Inter-platelet binding list: bead pairs of different platelets closer than
    `r_bond`, each bead in at most one bond, taken greedily by distance (ties by the
    lower index pair).  Indices are bead indices."""
    from scipy.spatial import cKDTree
    if xb.shape[0] == 0:
        return np.zeros((0, 2), np.int64)
    pairs = cKDTree(xb).query_pairs(r_bond, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros((0, 2), np.int64)
    pairs = pairs[body[pairs[:, 0]] != body[pairs[:, 1]]]
    pairs = np.sort(pairs, axis=1)
    d = np.linalg.norm(xb[pairs[:, 0]] - xb[pairs[:, 1]], axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0], d))
    used = np.zeros(xb.shape[0], bool)
    out = []
    for q in order:
        a, b = pairs[q]
        if not used[a] and not used[b]:
            used[a] = used[b] = True
            out.append((a, b))
    return np.array(out, np.int64).reshape(-1, 2)


def aggregate_box(n_fluid=20000, L=(18.0, 18.0, 18.0), grid=(1, 2, 1), spacing=(7.0, 2.8, 7.0), level=3,
                  semi_axes=(3.0, 1.0, 3.0), seed=20220532, morse_cut=1.5, **over):
    """Periodic DPD box with platelets packed on a lattice (short axis along y, centre
    spacing `spacing`), bound by inter-platelet Morse bonds between beads of different
    platelets closer than morse_cut * morse_r0 (rest distance)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    p = dpd_params(seed=seed, **over)
    tmpl = platelet_template(level, semi_axes)
    nx, ny, nz = grid
    centres = []
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                off = np.array([(ix - (nx - 1) / 2) * spacing[0], (iy - (ny - 1) / 2) * spacing[1],
                                (iz - (nz - 1) / 2) * spacing[2]])
                centres.append(L / 2.0 + off)
    b0 = n_fluid
    xb, body, rest, bonds, r0, angles, th0 = _place_platelets(tmpl, centres, [np.eye(3)] * len(centres), b0)
    mb = morse_bonds(xb, body, morse_cut * p["morse_r0"]) + b0
    xf = _fluid_away_from(rng, n_fluid, np.zeros(3), L, xb, p["lj_sig"], L, (1, 1, 1))
    x = np.concatenate([xf, xb])
    v = maxwell(rng, x.shape[0], p["kT"], 1.0)
    sysd = dict(box_lo=np.zeros(3), box_L=L, periodic=(1, 1, 1), n_fluid=n_fluid, n_wall=0,
                n_bead=xb.shape[0], n_platelet=len(centres), x=x, v=v, body=body, rest=rest, bonds=bonds,
                bond_r0=r0, angles=angles, angle_th0=th0, morse=mb, platelet_area=np.full(len(centres), tmpl["area"]),
                params=p, schedule=dict(dt_outer=0.01, k=4))
    return _finish(sysd)
