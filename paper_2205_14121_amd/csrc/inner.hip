// Platelet ("inner") force group: harmonic bonds and angles and Morse bonds (Eq. 2,
// inter-platelet binding of Eq. 4), WCA Lennard-Jones between beads (Eq. 2) and the
// platelet-fluid force of Eq. 3 (WCA + DPD dissipative + random) between beads and
// fluid or wall particles.
//
// The work is organised around a member list rebuilt with the cell list every outer
// step: the beads, then every fluid particle within reach (cutoff + skin) of a bead.
// Each member owns a CSR list of partner slots.  Forces are gathered: one thread per
// member sums the terms acting on it, so every pair is evaluated from both ends and
// no atomics are needed; both ends compute bit-identical magnitudes (the separation
// flips sign exactly and the random number is keyed symmetrically), so Newton's third
// law holds exactly and the result does not depend on scheduling.
#include "common.h"

namespace aimts {

namespace {

__device__ __forceinline__ bool bead_pair_allowed(const Dev &s, int32_t bi, int32_t bj)
{
    if (s.body[bi] != s.body[bj]) return true;
    const int64_t nb = s.nb;
    const double d0 = s.rest[bi] - s.rest[bj];
    const double d1 = s.rest[nb + bi] - s.rest[nb + bj];
    const double d2 = s.rest[2 * nb + bi] - s.rest[2 * nb + bj];
    return d0 * d0 + d1 * d1 + d2 * d2 >= s.r_excl2;
}

// Visit the cells within `reach` of the cell holding (x0,x1,x2); returns false for
// cells beyond a non-periodic face.
template <typename Fn>
__device__ __forceinline__ void for_cells(const Dev &s, double x0, double x1, double x2, Fn fn)
{
    const int cx = cell_coord(s, 0, x0), cy = cell_coord(s, 1, x1), cz = cell_coord(s, 2, x2);
    const int R = s.reach;
    for (int dy = -R; dy <= R; ++dy) {
        int iy = cy + dy;
        if (iy < 0 || iy >= s.nc[1]) {
            if (!s.per[1]) continue;
            iy = (iy + s.nc[1]) % s.nc[1];
        }
        for (int dx = -R; dx <= R; ++dx) {
            int ix = cx + dx;
            if (ix < 0 || ix >= s.nc[0]) {
                if (!s.per[0]) continue;
                ix = (ix + s.nc[0]) % s.nc[0];
            }
            for (int dz = -R; dz <= R; ++dz) {
                int iz = cz + dz;
                if (iz < 0 || iz >= s.nc[2]) {
                    if (!s.per[2]) continue;
                    iz = (iz + s.nc[2]) % s.nc[2];
                }
                fn(cell_index(s, ix, iy, iz));
            }
        }
    }
}

// Pass 0 counts partners (and flags fluid partners as members); pass 1 writes them.
__global__ void k_bead_pairs(Dev s, int pass, int32_t *flag, int32_t *cnt)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.nb) return;
    const int32_t t = s.bead_slot[b];
    const double x0 = s.x[t], x1 = s.x[s.N + t], x2 = s.x[2 * s.N + t];
    int32_t c = 0;
    const int32_t base = pass ? s.pair_off[b] : 0;
    for_cells(s, x0, x1, x2, [&](int64_t cc) {
        const int32_t beg = s.cell_start[cc], end = s.cell_start[cc + 1];
        const int32_t split = beg + s.cell_nonbead[cc];
        for (int32_t j = beg; j < end; ++j) {
            if (j == t) continue;
            const double d0 = min_image(s, 0, x0 - s.x[j]);
            const double d1 = min_image(s, 1, x1 - s.x[s.N + j]);
            const double d2 = min_image(s, 2, x2 - s.x[2 * s.N + j]);
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            bool take;
            if (j < split) {
                take = r2 < s.list_cut2;
                if (take && pass == 0 && s.id[j] < (uint64_t)s.nf) flag[j] = 1;
            } else {
                take = r2 < s.bb_cut2 && bead_pair_allowed(s, (int32_t)b, (int32_t)(s.id[j] - s.b0));
            }
            if (take) {
                if (pass == 1) {
                    const int64_t p = (int64_t)base + c;
                    if (p < s.cap_pairs) s.pair_list[p] = j;
                }
                ++c;
            }
        }
    });
    if (pass == 0) cnt[b] = c;
}

__global__ void k_compact_members(Dev s, int32_t *flag, const int32_t *flag_scan)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.N) return;
    if (flag[t]) {
        const int64_t m = s.nb + flag_scan[t];
        if (m < s.cap_members) {
            s.member_slot[m] = (int32_t)t;
            s.mos[t] = (int32_t)m;
        }
        flag[t] = 0;
    }
}

// Also closes the skin check of the outer step that just ended: a fluid particle that
// was no member stayed farther than (cutoff + skin) from every bead at the previous
// rebuild, so no pair was missed while (its path + the largest member displacement)
// and (twice the largest member displacement) stay within the skin.
__global__ void k_member_count(Dev s, const int32_t *flag_scan)
{
    const float m0 = fmaxf(__uint_as_float(s.maxdisp[0]), (float)s.disp_floor);
    const float m1 = fmaxf(__uint_as_float(s.maxdisp[1]), (float)s.disp_floor);
    if (s.nb > 0 && ((double)m0 + (double)m1 > s.skin || 2.0 * (double)m1 > s.skin)) atomicOr(s.err, kErrSkin);
    s.maxdisp[0] = 0u;
    s.maxdisp[1] = 0u;
    const int64_t tot = s.nb + flag_scan[s.N];
    if (tot > s.cap_members) atomicOr(s.err, kErrMemberCap);
    *s.n_members = (int32_t)(tot < s.cap_members ? tot : s.cap_members);
}

// Fluid members: their partners are the beads within reach.
__global__ void k_fluid_pairs(Dev s, int pass, int32_t *cnt)
{
    const int64_t m = s.nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= s.cap_members) return;
    if (m >= *s.n_members) {
        if (pass == 0) cnt[m] = 0;
        return;
    }
    const int32_t t = s.member_slot[m];
    const double x0 = s.x[t], x1 = s.x[s.N + t], x2 = s.x[2 * s.N + t];
    int32_t c = 0;
    const int32_t base = pass ? s.pair_off[m] : 0;
    for_cells(s, x0, x1, x2, [&](int64_t cc) {
        const int32_t end = s.cell_start[cc + 1];
        for (int32_t j = s.cell_start[cc] + s.cell_nonbead[cc]; j < end; ++j) {
            const double d0 = min_image(s, 0, x0 - s.x[j]);
            const double d1 = min_image(s, 1, x1 - s.x[s.N + j]);
            const double d2 = min_image(s, 2, x2 - s.x[2 * s.N + j]);
            if (d0 * d0 + d1 * d1 + d2 * d2 < s.list_cut2) {
                if (pass == 1) {
                    const int64_t p = (int64_t)base + c;
                    if (p < s.cap_pairs) s.pair_list[p] = j;
                }
                ++c;
            }
        }
    });
    if (pass == 0) cnt[m] = c;
}

__global__ void k_pair_total(Dev s)
{
    if ((int64_t)s.pair_off[s.cap_members] > s.cap_pairs) atomicOr(s.err, kErrPairCap);
}

// Reference positions for the skin check and the inner force carried over to the new
// member numbering (beads keep their index; a fluid member keeps its force if it was a
// member before the rebuild, otherwise its force was zero).
__global__ void k_member_init(Dev s, const double *fi_old, int64_t cap_old, const int32_t *mos_old,
                              const int32_t *src_of)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= *s.n_members) return;
    const int32_t t = s.member_slot[m];
#pragma unroll
    for (int k = 0; k < 3; ++k) s.xref[k * s.cap_members + m] = s.x[k * s.N + t];
    int64_t om = m;
    if (m >= s.nb) om = mos_old[src_of[t]];
#pragma unroll
    for (int k = 0; k < 3; ++k) s.fi[k * s.cap_members + m] = om >= 0 ? fi_old[k * cap_old + om] : 0.0;
}

__global__ void k_bead_members(Dev s)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.nb) return;
    s.member_slot[b] = s.bead_slot[b];
}

// ---------------------------------------------------------------------------
// Forces
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_pos(const Dev &s, int32_t t, double &a, double &b, double &c)
{
    a = s.x[t];
    b = s.x[s.N + t];
    c = s.x[2 * s.N + t];
}

// Bonded terms on bead b (slot t at (x0,x1,x2)), float64.
__device__ void bonded_on_bead(const Dev &s, int32_t b, double x0, double x1, double x2, double &f0, double &f1,
                               double &f2)
{
    for (int32_t q = s.bond_off[b]; q < s.bond_off[b + 1]; ++q) {
        double y0, y1, y2;
        load_pos(s, s.bead_slot[s.bond_other[q]], y0, y1, y2);
        const double d0 = min_image(s, 0, x0 - y0), d1 = min_image(s, 1, x1 - y1), d2 = min_image(s, 2, x2 - y2);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double fs = -2.0 * s.kb * (r - s.bond_r0[q]) / r;   // U = kb (r - r0)^2
        f0 += fs * d0;
        f1 += fs * d1;
        f2 += fs * d2;
    }
    for (int32_t q = s.mor_off[b]; q < s.mor_off[b + 1]; ++q) {
        double y0, y1, y2;
        load_pos(s, s.bead_slot[s.mor_other[q]], y0, y1, y2);
        const double d0 = min_image(s, 0, x0 - y0), d1 = min_image(s, 1, x1 - y1), d2 = min_image(s, 2, x2 - y2);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double ex = exp(-s.ma * (r - s.mr0));
        const double fs = 2.0 * s.ma * s.mD * (ex * ex - ex) / r;  // -dU/dr / r
        f0 += fs * d0;
        f1 += fs * d1;
        f2 += fs * d2;
    }
    // U = ka (theta - theta0)^2 about the vertex j of (i, j, k); a = x_i - x_j, c = x_k - x_j.
    // F_i = p (c/(|a||c|) - cos a/|a|^2), F_k = p (a/(|a||c|) - cos c/|c|^2), F_j = -(F_i + F_k),
    // p = 2 ka (theta - theta0) / sin(theta).
    for (int32_t q = s.ang_off[b]; q < s.ang_off[b + 1]; ++q) {
        const int32_t e = s.ang_ent[q];
        const int32_t ang = e >> 2, role = e & 3;
        double pi0, pi1, pi2, pj0, pj1, pj2, pk0, pk1, pk2;
        load_pos(s, s.bead_slot[s.ang_ijk[3 * ang + 0]], pi0, pi1, pi2);
        load_pos(s, s.bead_slot[s.ang_ijk[3 * ang + 1]], pj0, pj1, pj2);
        load_pos(s, s.bead_slot[s.ang_ijk[3 * ang + 2]], pk0, pk1, pk2);
        const double a0 = min_image(s, 0, pi0 - pj0), a1 = min_image(s, 1, pi1 - pj1), a2 = min_image(s, 2, pi2 - pj2);
        const double c0 = min_image(s, 0, pk0 - pj0), c1 = min_image(s, 1, pk1 - pj1), c2 = min_image(s, 2, pk2 - pj2);
        const double la = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        const double lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        double cs = (a0 * c0 + a1 * c1 + a2 * c2) / (la * lc);
        cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
        const double th = acos(cs);
        double sn = sin(th);
        sn = sn < 1e-12 ? 1e-12 : sn;
        const double p = 2.0 * s.ka * (th - s.ang_th0[ang]) / sn;
        const double iac = 1.0 / (la * lc), iaa = cs / (la * la), icc = cs / (lc * lc);
        const double fi0 = p * (c0 * iac - a0 * iaa), fi1 = p * (c1 * iac - a1 * iaa), fi2 = p * (c2 * iac - a2 * iaa);
        const double fk0 = p * (a0 * iac - c0 * icc), fk1 = p * (a1 * iac - c1 * icc), fk2 = p * (a2 * iac - c2 * icc);
        if (role == 0) { f0 += fi0; f1 += fi1; f2 += fi2; }
        else if (role == 2) { f0 += fk0; f1 += fk1; f2 += fk2; }
        else { f0 -= fi0 + fk0; f1 -= fi1 + fk1; f2 -= fi2 + fk2; }
    }
}

template <typename R>
__device__ __forceinline__ R lj_scalar(R r2, R sig2, R eps)
{
    const R sr2 = sig2 / r2;
    const R sr6 = sr2 * sr2 * sr2;
    return R(24) * eps * (R(2) * sr6 * sr6 - sr6) / r2;
}

template <typename R>
__global__ void k_inner(Dev s, uint64_t count, double inv_sqrt_dt)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= *s.n_members) return;
    const int32_t t = s.member_slot[m];
    const uint32_t idi = s.id[t];
    double x0, x1, x2;
    load_pos(s, t, x0, x1, x2);
    const double v0 = s.v[t], v1 = s.v[s.N + t], v2 = s.v[2 * s.N + t];
    const bool i_bead = m < s.nb;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    if (i_bead) bonded_on_bead(s, (int32_t)m, x0, x1, x2, f0, f1, f2);
    R p0 = R(0), p1 = R(0), p2 = R(0);
    const R lj_rc2 = (R)s.lj_rc2, sig2 = (R)s.lj_sig2, eps = (R)s.lj_eps;
    const R rcpf2 = (R)s.rc_pf2, inv_rcpf = (R)s.inv_rc_pf, gpf = (R)s.gpf, spf = (R)s.spf;
    const R isdt = (R)inv_sqrt_dt;
    const uint32_t k1 = s.key1 ^ 1u;
    // an overflowed list (flagged at rebuild) is truncated at the capacity
    const int64_t pend = s.pair_off[m + 1] < s.cap_pairs ? s.pair_off[m + 1] : s.cap_pairs;
    for (int64_t p = s.pair_off[m]; p < pend; ++p) {
        const int32_t j = s.pair_list[p];
        const R d0 = (R)min_image(s, 0, x0 - s.x[j]);
        const R d1 = (R)min_image(s, 1, x1 - s.x[s.N + j]);
        const R d2 = (R)min_image(s, 2, x2 - s.x[2 * s.N + j]);
        const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const uint32_t idj = s.id[j];
        const bool j_bead = idj >= (uint64_t)s.b0;
        R fs = R(0);
        if (r2 < lj_rc2) fs = lj_scalar<R>(r2, sig2, eps);
        if (!(i_bead && j_bead) && r2 < rcpf2) {
            const R r = sqrt(r2);
            const R w = R(1) - r * inv_rcpf;
            const R ev = (d0 * (R)(v0 - s.v[j]) + d1 * (R)(v1 - s.v[s.N + j]) + d2 * (R)(v2 - s.v[2 * s.N + j])) / r;
            uint32_t w0, w1;
            pair_words(idi, idj, count, s.key0, k1, w0, w1);
            R z;
            if constexpr (sizeof(R) == 8) z = gauss64(w0, w1);
            else z = gauss32(w0, w1);
            fs += (-gpf * w * w * ev + spf * w * z * isdt) / r;
        }
        p0 += fs * d0;
        p1 += fs * d1;
        p2 += fs * d2;
    }
    s.fi[m] = f0 + (double)p0;
    s.fi[s.cap_members + m] = f1 + (double)p1;
    s.fi[2 * s.cap_members + m] = f2 + (double)p2;
}

}  // namespace

void rebuild_inner(Dev &s, InnerBufs &b, const int32_t *src_of, hipStream_t st)
{
    const int bs = 256;
    const int64_t capS = s.cap_members - s.nb;
    // beads are always the first members
    if (s.nb > 0) hipLaunchKernelGGL(k_bead_members, dim3(nblocks(s.nb, bs)), dim3(bs), 0, st, s);
    if (s.nb > 0) hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, bs)), dim3(bs), 0, st, s, 0, b.flag_i32, b.cnt);
    scan_exclusive(b.flag_i32, b.flag_scan, s.N, b.scan_temp, st);
    hipLaunchKernelGGL(k_compact_members, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, b.flag_i32, b.flag_scan);
    hipLaunchKernelGGL(k_member_count, dim3(1), dim3(1), 0, st, s, b.flag_scan);
    if (capS > 0) hipLaunchKernelGGL(k_fluid_pairs, dim3(nblocks(capS, bs)), dim3(bs), 0, st, s, 0, b.cnt);
    scan_exclusive(b.cnt, s.pair_off, s.cap_members, b.scan_temp, st);
    hipLaunchKernelGGL(k_pair_total, dim3(1), dim3(1), 0, st, s);
    if (s.nb > 0) hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, bs)), dim3(bs), 0, st, s, 1, b.flag_i32, b.cnt);
    if (capS > 0) hipLaunchKernelGGL(k_fluid_pairs, dim3(nblocks(capS, bs)), dim3(bs), 0, st, s, 1, b.cnt);
    double *fi_old = s.fi;
    s.fi = b.fi_alt;
    b.fi_alt = fi_old;
    if (s.cap_members > 0)
        hipLaunchKernelGGL(k_member_init, dim3(nblocks(s.cap_members, bs)), dim3(bs), 0, st, s, (const double *)fi_old,
                           s.cap_members, (const int32_t *)b.mos_old, src_of);
}

void inner_forces(const Dev &s, uint64_t count, double dt_inner, hipStream_t st)
{
    if (s.cap_members == 0) return;
    const int bs = 128;
    const double isdt = 1.0 / sqrt(dt_inner);
    if (s.fp32)
        hipLaunchKernelGGL(k_inner<float>, dim3(nblocks(s.cap_members, bs)), dim3(bs), 0, st, s, count, isdt);
    else
        hipLaunchKernelGGL(k_inner<double>, dim3(nblocks(s.cap_members, bs)), dim3(bs), 0, st, s, count, isdt);
}

}  // namespace aimts
