// Diagnostics (Table 1, the step of the multiscale scheme that computes and writes out
// platelet properties; Sec. 3.3, the per-platelet time series the controller reads; Sec. 4.2,
// temperature and pressure): float64 reductions in a fixed order, so results are
// deterministic.
//
//  * thermo: kinetic energy, temperature, total momentum of the mobile particles and
//    the peculiar fluid temperature about the mean velocity of each y row of cells.
//    The cell grid is numbered y-major, so a row is a contiguous slot range and each
//    block reduces a fixed chunk of one row.
//  * features: eight numbers per platelet, one block per platelet.
//  * energy: conservative potential energies and the pair virial (on request only).
#include "kick.h"

namespace aimts {

namespace {

constexpr int kBS = 256;

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
    // fixed-order tree over the block: deterministic
    for (int q = 0; q < NV; ++q) lds[q * kBS + threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < NV; ++q) lds[q * kBS + threadIdx.x] += lds[q * kBS + threadIdx.x + w];
        __syncthreads();
    }
    for (int q = 0; q < NV; ++q) v[q] = lds[q * kBS];
    __syncthreads();
}

constexpr int kRowBS = 256;  // threads per row-chunk block of the thermo reduction

// What a row kernel does to each mobile slot of its chunk (any combination).
enum : int {
    kRowClose = 1,  // the closing outer half kick v += h F_outer / m
    kRowSum = 2,    // the thermo sums of the (kicked) velocities
    kRowOpen = 4,   // the opening of the next outer step (open_slot), from the kicked velocity
};

// Over one chunk of one y row of cells (its fluid/wall bins, then its bead bins): with
// kRowClose the closing outer half kick of each mobile slot of the chunk (every slot is
// kicked here exactly once, since the rows tile the slots), with kRowSum the sums
// partial[(row * chunks + c) * 10] = fluid {m, m v0, m v1, m v2, m v^2}, mobile
// {m v^2, m v0, m v1, m v2, count} of the kicked velocities, with kRowOpen the opening
// of the next outer step from the kicked velocity (whose closing and opening kicks then
// cost one read and one write of the state instead of two each); without kRowOpen the
// kicked velocity is stored.  Wall slots are neither kicked nor counted; with kRowOpen
// they are copied into the members' second buffer.  Fixed reduction order: per thread in
// slot order, a butterfly over each wavefront, then the wavefronts in order.
template <int F>
__global__ __launch_bounds__(kRowBS) void k_rows(Dev s, int chunks, double *partial, double h, OuterOpen op)
{
    __shared__ double lds[10][kRowBS / 64];
    const int row = blockIdx.x / chunks, c = blockIdx.x % chunks;
    const int64_t cells_per_row = (int64_t)s.nc[0] * s.nc[2];
    // the row's fluid/wall slots, then its bead slots, taken as one sequence
    const int32_t ra = s.cell_start[row * cells_per_row], la = s.cell_start[(row + 1) * cells_per_row] - ra;
    const int32_t rb = s.cell_start[s.ncell + row * cells_per_row];
    const int64_t len = la + (s.cell_start[s.ncell + (row + 1) * cells_per_row] - rb);
    const int64_t b = len * c / chunks, e = len * (c + 1) / chunks;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t N = s.N;
    bool bad = false;
    float pmax = 0.0f;  // largest lazy-drift path of a non-member (kRowOpen)
    for (int64_t f = b + threadIdx.x; f < e; f += kRowBS) {
        const int64_t t = f < la ? ra + f : rb + (f - la);
        const int ty = ptype(s, s.id[t]);
        if (ty == 1) {  // frozen walls
            if (F & kRowOpen)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    op.xa[q * N + t] = s.x[q * N + t];
                    op.va[q * N + t] = s.v[q * N + t];
                }
            continue;
        }
        double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
        if (F & kRowClose) {
            outer_half_kick(s, t, h, s.minv[ty], v0, v1, v2);
            if (!(F & kRowOpen)) {
                s.v[t] = v0;
                s.v[N + t] = v1;
                s.v[2 * N + t] = v2;
            }
            if (!isfinite(v0 + v1 + v2)) bad = true;
        }
        if (F & kRowSum) {
            const double m = s.m[ty];
            const double mv2 = m * (v0 * v0 + v1 * v1 + v2 * v2);
            if (ty == 0) {
                acc[0] += m;
                acc[1] += m * v0;
                acc[2] += m * v1;
                acc[3] += m * v2;
                acc[4] += mv2;
            }
            acc[5] += mv2;
            acc[6] += m * v0;
            acc[7] += m * v1;
            acc[8] += m * v2;
            acc[9] += 1.0;
        }
        if (F & kRowOpen) open_slot(s, t, ty, v0, v1, v2, op.h_out, op.k, op.dt, op.ls, op.xw, op.vw, pmax, bad);
    }
    if (bad) atomicOr(s.err, kErrNonFinite);
    if ((F & kRowOpen) && s.nb > 0) block_max_commit(&s.maxdisp[0], pmax, (float)s.disp_floor);
    if (F & kRowSum) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1)
#pragma unroll
            for (int q = 0; q < 10; ++q) acc[q] += __shfl_xor(acc[q], o, 64);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int q = 0; q < 10; ++q) lds[q][wv] = acc[q];
        __syncthreads();
        if (threadIdx.x < 10) {
            double t = 0.0;
            for (int w = 0; w < kRowBS / 64; ++w) t += lds[threadIdx.x][w];
            partial[(int64_t)blockIdx.x * 10 + threadIdx.x] = t;
        }
    }
}

__global__ __launch_bounds__(kBS) void k_thermo_final(Dev s, int chunks, const double *partial, double *out, double time,
                                                     int k)
{
    __shared__ double lds[8 * kBS];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // pec, nfluid-mass, occupied, mv2, p0, p1, p2, count
    for (int row = threadIdx.x; row < s.nrow; row += kBS) {
        double r[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < chunks; ++c)
            for (int q = 0; q < 10; ++q) r[q] += partial[((int64_t)row * chunks + c) * 10 + q];
        if (r[0] > 0.0) {
            acc[0] += r[4] - (r[1] * r[1] + r[2] * r[2] + r[3] * r[3]) / r[0];
            acc[1] += r[0];
            acc[2] += 1.0;
        }
        acc[3] += r[5];
        acc[4] += r[6];
        acc[5] += r[7];
        acc[6] += r[8];
        acc[7] += r[9];
    }
    block_sum<8>(acc, lds);
    if (threadIdx.x == 0) {
        const double nm = acc[7];
        const double nfl = acc[1] / s.m[0];
        out[0] = time;
        out[1] = 0.5 * acc[3];
        out[2] = nm > 1.0 ? acc[3] / (3.0 * nm - 3.0) : 0.0;
        out[3] = nfl > acc[2] ? acc[0] / (3.0 * (nfl - acc[2])) : 0.0;
        out[4] = acc[4];
        out[5] = acc[5];
        out[6] = acc[6];
        out[7] = (double)k;
    }
}

// ---------------------------------------------------------------------------
// Platelet features
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bead_pos(const Dev &s, int32_t b, double &a, double &c, double &d)
{
    const int32_t t = s.bead_slot[b];
    a = s.x[t];
    c = s.x[s.N + t];
    d = s.x[2 * s.N + t];
}

// Features in two fixed-order passes, kFeatBlocks blocks per platelet:
//   1: per block, moments about the platelet's first bead f (offsets q = x - f under the
//      minimum image): mass, m q, m v, m q x v, m q q^T, m v^2 / 2, and the shear
//      traction and contact sums and the largest bond strain;
//   2: reduce, shift the moments to the centre of mass (L = sum m q x v - c x P,
//      I from sum m q q^T - M c c^T, internal kinetic energy = K - M V^2 / 2), solve
//      I omega = L and write the eight features.
constexpr int kFeatBlocks = 160;  // ~16 beads per block of a level-4 platelet: one per 16-lane group
constexpr int kFeatNV = 20;       // partial row: 19 sums and the strain maximum

__device__ __forceinline__ void bead_range(const Dev &s, int p, int q, int32_t &b0, int32_t &b1)
{
    const int32_t lo = s.plt_off[p], n = s.plt_off[p + 1] - lo;
    b0 = lo + (int32_t)((int64_t)n * q / kFeatBlocks);
    b1 = lo + (int32_t)((int64_t)n * (q + 1) / kFeatBlocks);
}

// Totals of the kFeatBlocks partial rows of NV doubles, by one wavefront: lane r adds
// rows r, r + 64, ... in order, then a butterfly over the lanes.  Both ends of every
// butterfly step add the same two numbers, so all lanes end with identical totals.
// Columns flagged in max_mask are maxima instead of sums.
template <int NV>
__device__ __forceinline__ void wave_reduce_rows(const double *rows, double (&v)[NV], unsigned max_mask)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;  // the maxima are of non-negative quantities
    for (int r = lane; r < kFeatBlocks; r += 64)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double x = rows[r * NV + q];
            v[q] = ((max_mask >> q) & 1u) ? fmax(v[q], x) : v[q] + x;
        }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double o = __shfl_xor(v[q], m, 64);
            v[q] = ((max_mask >> q) & 1u) ? fmax(v[q], o) : v[q] + o;
        }
}

// A group of G lanes per bead (the inner kernel's lanes per bead: 16, or 8 from 131,072
// beads up, where the bead lists are long and half-empty 16-lane groups cost more than
// the longer per-lane loops): lane 0 of the group adds the bead's own moments, the group
// shares its bonds and pair list.
__global__ __launch_bounds__(kBS) void k_feat_moments(Dev s, double *part, double contact_r2, double h_pend)
{
    __shared__ double lds[kBS / 64][kFeatNV];
    const int p = blockIdx.x / kFeatBlocks, q = blockIdx.x % kFeatBlocks;
    int32_t bb0, bb1;
    bead_range(s, p, q, bb0, bb1);
    double f0, f1, f2;
    bead_pos(s, s.plt_off[p], f0, f1, f2);
    const double mb = s.m[2];
    const int64_t N = s.N;
    // M, m q (3), m v (3), m q x v (3), m q q^T (xx yy zz xy xz yz), m v^2 / 2, shear, contacts, strain
    double a[kFeatNV];
#pragma unroll
    for (int k = 0; k < kFeatNV; ++k) a[k] = 0.0;
    const double lj_rc2 = s.lj_rc2, rcpf2 = s.rc_pf2;
    const int G = inner_bead_lanes(s.nb);
    const int grp = threadIdx.x / G, u = threadIdx.x & (G - 1);
    for (int32_t b = bb0 + grp; b < bb1; b += kBS / G) {
        // the list bounds and the first entry of each list are loaded with the bead's own
        // state, and each loop fetches its next index ahead
        const int32_t t = s.bead_slot[b];
        const int32_t e0b = s.bond_off[b] + u, e1b = s.bond_off[b + 1];
        const int64_t e0p = s.pair_off[b] + u;
        const int64_t pe = s.pair_off[b + 1] < s.cap_pairs ? s.pair_off[b + 1] : s.cap_pairs;
        int32_t nbz = e0b < e1b ? s.bond_slot[e0b] : 0;
        int32_t npj = e0p < pe ? s.pair_list[e0p] : 0;
        const double y0 = s.x[t], y1 = s.x[N + t], y2 = s.x[2 * N + t];
        const double vb0 = s.v[t], vb1 = s.v[N + t], vb2 = s.v[2 * N + t];
        if (u == 0) {
            const double q0 = min_image(s, 0, y0 - f0), q1 = min_image(s, 1, y1 - f1), q2 = min_image(s, 2, y2 - f2);
            a[0] += mb;
            a[1] += mb * q0;
            a[2] += mb * q1;
            a[3] += mb * q2;
            a[4] += mb * vb0;
            a[5] += mb * vb1;
            a[6] += mb * vb2;
            a[7] += mb * (q1 * vb2 - q2 * vb1);
            a[8] += mb * (q2 * vb0 - q0 * vb2);
            a[9] += mb * (q0 * vb1 - q1 * vb0);
            a[10] += mb * q0 * q0;
            a[11] += mb * q1 * q1;
            a[12] += mb * q2 * q2;
            a[13] += mb * q0 * q1;
            a[14] += mb * q0 * q2;
            a[15] += mb * q1 * q2;
            a[16] += 0.5 * mb * (vb0 * vb0 + vb1 * vb1 + vb2 * vb2);
        }
        for (int32_t e = e0b; e < e1b; e += G) {
            const int32_t tz = nbz;
            if (e + G < e1b) nbz = s.bond_slot[e + G];
            const double z0 = s.x[tz], z1 = s.x[N + tz], z2 = s.x[2 * N + tz];
            const double d0 = min_image(s, 0, y0 - z0), d1 = min_image(s, 1, y1 - z1), d2 = min_image(s, 2, y2 - z2);
            const double st = fabs(sqrt(d0 * d0 + d1 * d1 + d2 * d2) - s.bond_r0[e]) / s.bond_r0[e];
            a[19] = st > a[19] ? st : a[19];
        }
        // shear traction from bead-fluid/wall pairs (WCA + dissipative, no random term)
        // and contacts with walls and beads of other platelets.  The list holds the fluid
        // and wall partners first; of the bead partners only those of other platelets
        // can be contacts, so a bead partner of the own platelet is passed over on its
        // platelet index alone.
        const int64_t pfl = s.pair_off[b] + s.pair_nfl[b];
        for (int64_t e = e0p; e < pe; e += G) {
            const int32_t j = npj;
            if (e + G < pe) npj = s.pair_list[e + G];
            if (e >= pfl && __float_as_int(((const float *)s.rest_slot)[4 * (int64_t)j + 3]) == p) continue;
            const uint32_t idj = s.id[j];
            const double d0 = min_image(s, 0, y0 - s.x[j]);
            const double d1 = min_image(s, 1, y1 - s.x[N + j]);
            const double d2 = min_image(s, 2, y2 - s.x[2 * N + j]);
            const double rsq = d0 * d0 + d1 * d1 + d2 * d2;
            const int tj = ptype(s, idj);
            if (rsq < contact_r2 && (tj == 1 || (tj == 2 && s.body[idj - s.b0] != p))) a[18] += 1.0;
            if (tj != 2 && rsq > 0.0) {
                double fs = 0.0;
                if (rsq < lj_rc2) {
                    const double sr2 = s.lj_sig2 / rsq;
                    const double sr6 = sr2 * sr2 * sr2;
                    fs += 24.0 * s.lj_eps * (2.0 * sr6 * sr6 - sr6) / rsq;
                }
                if (rsq < rcpf2) {
                    const double r = sqrt(rsq);
                    const double w = 1.0 - r * s.inv_rc_pf;
                    // the partner's velocity at the end of the outer step
                    double u0 = s.v[j], u1 = s.v[N + j], u2 = s.v[2 * N + j];
                    if (h_pend != 0.0 && tj == 0) outer_half_kick(s, j, h_pend, s.minv[0], u0, u1, u2);
                    const double ev = (d0 * (vb0 - u0) + d1 * (vb1 - u1) + d2 * (vb2 - u2)) / r;
                    fs += -s.gpf * w * w * ev / r;
                }
                a[17] += d1 * fs * d0;
            }
        }
    }
    // fixed-order block reduction: butterfly over each wavefront, then the wavefronts in order
#pragma unroll
    for (int o = 1; o < 64; o <<= 1)
#pragma unroll
        for (int k = 0; k < kFeatNV; ++k) {
            const double x = __shfl_xor(a[k], o, 64);
            a[k] = k == kFeatNV - 1 ? fmax(a[k], x) : a[k] + x;
        }
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < kFeatNV; ++k) lds[threadIdx.x >> 6][k] = a[k];
    __syncthreads();
    if (threadIdx.x < kFeatNV) {
        const int k = threadIdx.x;
        double t = lds[0][k];
        for (int w = 1; w < kBS / 64; ++w) t = k == kFeatNV - 1 ? fmax(t, lds[w][k]) : t + lds[w][k];
        part[(int64_t)blockIdx.x * kFeatNV + k] = t;
    }
}

// One wavefront per platelet.
__global__ __launch_bounds__(64) void k_feat_final(Dev s, const double *part, float *ring, int row, float *last)
{
    const int p = blockIdx.x;
    double a[kFeatNV];
    wave_reduce_rows<kFeatNV>(part + (int64_t)p * kFeatBlocks * kFeatNV, a, 1u << (kFeatNV - 1));
    if (threadIdx.x != 0) return;
    const double M = a[0];
    const double c0 = a[1] / M, c1 = a[2] / M, c2 = a[3] / M;
    const double P0 = a[4], P1 = a[5], P2 = a[6];
    const double V0 = P0 / M, V1 = P1 / M, V2 = P2 / M;
    // angular momentum and inertia tensor about the centre of mass
    const double L0 = a[7] - (c1 * P2 - c2 * P1), L1 = a[8] - (c2 * P0 - c0 * P2), L2 = a[9] - (c0 * P1 - c1 * P0);
    const double Sxx = a[10] - M * c0 * c0, Syy = a[11] - M * c1 * c1, Szz = a[12] - M * c2 * c2;
    const double Sxy = a[13] - M * c0 * c1, Sxz = a[14] - M * c0 * c2, Syz = a[15] - M * c1 * c2;
    const double I00 = Syy + Szz, I11 = Sxx + Szz, I22 = Sxx + Syy, I01 = -Sxy, I02 = -Sxz, I12 = -Syz;
    // omega = I^-1 L by Cramer's rule
    const double det = I00 * (I11 * I22 - I12 * I12) - I01 * (I01 * I22 - I12 * I02) + I02 * (I01 * I12 - I11 * I02);
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    if (fabs(det) > 1e-300) {
        w0 = (L0 * (I11 * I22 - I12 * I12) - I01 * (L1 * I22 - I12 * L2) + I02 * (L1 * I12 - I11 * L2)) / det;
        w1 = (I00 * (L1 * I22 - I12 * L2) - L0 * (I01 * I22 - I12 * I02) + I02 * (I01 * L2 - L1 * I02)) / det;
        w2 = (I00 * (I11 * L2 - L1 * I12) - I01 * (I01 * L2 - L1 * I02) + L0 * (I01 * I12 - I11 * I02)) / det;
    }
    float o[8];
    o[0] = (float)V0;
    o[1] = (float)V1;
    o[2] = (float)V2;
    o[3] = (float)sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    o[4] = (float)(a[16] - 0.5 * M * (V0 * V0 + V1 * V1 + V2 * V2));
    o[5] = (float)a[19];
    o[6] = (float)(a[17] / s.plt_area[p]);
    o[7] = (float)a[18];
    for (int k = 0; k < 8; ++k) {
        if (ring) ring[((int64_t)p * 64 + row) * 8 + k] = o[k];
        last[p * 8 + k] = o[k];
    }
}

// ---------------------------------------------------------------------------
// Conservative energies and pair virial: partial[block][6]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBS) void k_energy_outer(Dev s, double *partial)
{
    __shared__ double lds[2 * kBS];
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < s.N && s.id[i] < (uint64_t)s.nf) {
        const int64_t N = s.N;
        const double x0 = s.x[i], x1 = s.x[N + i], x2 = s.x[2 * N + i];
        const int cx = cell_coord(s, 0, x0), cy = cell_coord(s, 1, x1), cz = cell_coord(s, 2, x2);
        for (int dy = -1; dy <= 1; ++dy) {
            int iy = cy + dy;
            if (iy < 0 || iy >= s.nc[1]) { if (!s.per[1]) continue; iy = (iy + s.nc[1]) % s.nc[1]; }
            for (int dx = -1; dx <= 1; ++dx) {
                int ix = cx + dx;
                if (ix < 0 || ix >= s.nc[0]) { if (!s.per[0]) continue; ix = (ix + s.nc[0]) % s.nc[0]; }
                for (int dz = -1; dz <= 1; ++dz) {
                    int iz = cz + dz;
                    if (iz < 0 || iz >= s.nc[2]) { if (!s.per[2]) continue; iz = (iz + s.nc[2]) % s.nc[2]; }
                    const int64_t c = cell_index(s, ix, iy, iz);
                    const int32_t beg = s.cell_start[c], end = s.cell_start[c + 1];
                    for (int32_t j = beg; j < end; ++j) {
                        if (j == i || s.id[j] >= (uint64_t)s.b0) continue;  // beads are not DPD particles
                        const double d0 = min_image(s, 0, x0 - s.x[j]);
                        const double d1 = min_image(s, 1, x1 - s.x[N + j]);
                        const double d2 = min_image(s, 2, x2 - s.x[2 * N + j]);
                        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        if (r2 < s.rc2 && r2 > 0.0) {
                            const double r = sqrt(r2);
                            const double w = 1.0 - r * s.inv_rc;
                            // fluid-fluid pairs are seen from both ends, fluid-wall pairs from one
                            const double share = s.id[j] < (uint64_t)s.nf ? 0.5 : 1.0;
                            acc[0] += share * 0.5 * s.a * s.rc * w * w;
                            acc[1] += share * s.a * w * r;
                        }
                    }
                }
            }
        }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        double *o = partial + (int64_t)blockIdx.x * 6;
        o[0] = acc[0];
        o[1] = 0.0; o[2] = 0.0; o[3] = 0.0; o[4] = 0.0;
        o[5] = acc[1];
    }
}

__global__ __launch_bounds__(kBS) void k_energy_inner(Dev s, double *partial)
{
    __shared__ double lds[6 * kBS];
    const int64_t m = (int64_t)blockIdx.x * kBS + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};  // dpd(unused), lj, bond, angle, morse, virial
    if (m < s.nb) {
        const int32_t t = s.member_slot[m];
        const int64_t N = s.N;
        const double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
        const int64_t pe = s.pair_off[m + 1] < s.cap_pairs ? s.pair_off[m + 1] : s.cap_pairs;
        for (int64_t p = s.pair_off[m]; p < pe; ++p) {
            const int32_t j = s.pair_list[p];
            const double d0 = min_image(s, 0, x0 - s.x[j]);
            const double d1 = min_image(s, 1, x1 - s.x[N + j]);
            const double d2 = min_image(s, 2, x2 - s.x[2 * N + j]);
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (r2 < s.lj_rc2 && r2 > 0.0) {
                const double share = s.id[j] >= (uint64_t)s.b0 ? 0.5 : 1.0;  // bead-bead seen twice
                const double sr2 = s.lj_sig2 / r2;
                const double sr6 = sr2 * sr2 * sr2;
                acc[1] += share * (4.0 * s.lj_eps * (sr6 * sr6 - sr6) + s.lj_eps);
                acc[5] += share * 24.0 * s.lj_eps * (2.0 * sr6 * sr6 - sr6);
            }
            // Eq. 4 aggregation between beads of different platelets, with the Morse
            // energy, shifted to 0 at the cutoff (each pair seen from both ends)
            if (s.agg_on && r2 < s.agg_rc2 && r2 > 0.0 && s.id[j] >= (uint64_t)s.b0 &&
                s.body[s.id[j] - s.b0] != s.body[m]) {
                const double r = sqrt(r2);
                const double ex = exp(-s.agg_a * (r - s.agg_r0)), q = 1.0 - r / s.agg_r0;
                acc[4] += 0.5 * (s.agg_D * (ex * ex - 2.0 * ex) + 0.5 * s.agg_fA * s.agg_r0 * q * q - s.agg_eshift);
                acc[5] += 0.5 * (2.0 * s.agg_a * s.agg_D * (ex * ex - ex) + s.agg_fA * q) * r;
            }
        }
        for (int32_t q = s.bond_off[m]; q < s.bond_off[m + 1]; ++q) {
            const int32_t u = s.bead_slot[s.bond_other[q]];
            const double d0 = min_image(s, 0, x0 - s.x[u]), d1 = min_image(s, 1, x1 - s.x[N + u]),
                         d2 = min_image(s, 2, x2 - s.x[2 * N + u]);
            const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const double dr = r - s.bond_r0[q];
            acc[2] += 0.5 * s.kb * dr * dr;
            acc[5] += 0.5 * (-2.0 * s.kb * dr * r);
        }
        for (int32_t q = s.mor_off[m]; q < s.mor_off[m + 1]; ++q) {
            const int32_t u = s.bead_slot[s.mor_other[q]];
            const double d0 = min_image(s, 0, x0 - s.x[u]), d1 = min_image(s, 1, x1 - s.x[N + u]),
                         d2 = min_image(s, 2, x2 - s.x[2 * N + u]);
            const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const double ex = exp(-s.ma * (r - s.mr0));
            acc[4] += 0.5 * s.mD * (ex * ex - 2.0 * ex);
            acc[5] += 0.5 * 2.0 * s.ma * s.mD * (ex * ex - ex) * r;
        }
        for (int32_t q = s.ang_off[m]; q < s.ang_off[m + 1]; ++q) {
            const int32_t e = s.ang_ent[q];
            if ((e & 3) != 1) continue;  // each angle once, from its vertex
            const int32_t ang = e >> 2;
            const int32_t ti = s.bead_slot[s.ang_ijk[3 * ang]], tk = s.bead_slot[s.ang_ijk[3 * ang + 2]];
            const double a0 = min_image(s, 0, s.x[ti] - x0), a1 = min_image(s, 1, s.x[N + ti] - x1),
                         a2 = min_image(s, 2, s.x[2 * N + ti] - x2);
            const double c0 = min_image(s, 0, s.x[tk] - x0), c1 = min_image(s, 1, s.x[N + tk] - x1),
                         c2 = min_image(s, 2, s.x[2 * N + tk] - x2);
            double cs = (a0 * c0 + a1 * c1 + a2 * c2) /
                        (sqrt(a0 * a0 + a1 * a1 + a2 * a2) * sqrt(c0 * c0 + c1 * c1 + c2 * c2));
            cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
            const double dth = acos(cs) - s.ang_th0[ang];
            acc[3] += s.ka * dth * dth;
        }
    }
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) partial[(int64_t)blockIdx.x * 6 + q] = acc[q];
}

__global__ __launch_bounds__(kBS) void k_energy_final(const double *partial, int64_t nparts, double *out)
{
    __shared__ double lds[6 * kBS];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nparts; b += kBS)
        for (int q = 0; q < 6; ++q) acc[q] += partial[b * 6 + q];
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) out[q] = acc[q];
}

}  // namespace

void thermo(const Dev &s, double *partial, int chunks, double *out, double time, int k, hipStream_t st)
{
    hipLaunchKernelGGL(k_rows<kRowSum>, dim3((unsigned)(s.nrow * chunks)), dim3(kRowBS), 0, st, s, chunks, partial, 0.0,
                       OuterOpen{});
    hipLaunchKernelGGL(k_thermo_final, dim3(1), dim3(kBS), 0, st, s, chunks, (const double *)partial, out, time, k);
}

void outer_kick_thermo_rows(const Dev &s, double h_out, double *partial, int chunks, hipStream_t st)
{
    hipLaunchKernelGGL(k_rows<kRowClose | kRowSum>, dim3((unsigned)(s.nrow * chunks)), dim3(kRowBS), 0, st, s, chunks,
                       partial, h_out, OuterOpen{});
}

void outer_close_open(const Dev &s, double h_close, double *partial, int chunks, double h_out, int k, double dt_in,
                      double *xa, double *va, const LevelStep &ls, double *xw, double *vw, hipStream_t st)
{
    const OuterOpen op{h_out, k, dt_in, xa, va, xw, vw, ls};
    const dim3 grid((unsigned)(s.nrow * chunks));
    if (partial)
        hipLaunchKernelGGL(k_rows<kRowClose | kRowSum | kRowOpen>, grid, dim3(kRowBS), 0, st, s, chunks, partial,
                           h_close, op);
    else
        hipLaunchKernelGGL(k_rows<kRowClose | kRowOpen>, grid, dim3(kRowBS), 0, st, s, chunks, partial, h_close, op);
}

void thermo_final(const Dev &s, const double *partial, int chunks, double *out, double time, int k, hipStream_t st)
{
    hipLaunchKernelGGL(k_thermo_final, dim3(1), dim3(kBS), 0, st, s, chunks, partial, out, time, k);
}

void energy(const Dev &s, double *partial, double *out, hipStream_t st)
{
    const int64_t nbo = nblocks(s.N, kBS);
    const int64_t nbi = s.nb > 0 ? nblocks(s.nb, kBS) : 0;
    hipLaunchKernelGGL(k_energy_outer, dim3((unsigned)nbo), dim3(kBS), 0, st, s, partial);
    if (nbi > 0) hipLaunchKernelGGL(k_energy_inner, dim3((unsigned)nbi), dim3(kBS), 0, st, s, partial + nbo * 6);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBS), 0, st, (const double *)partial, nbo + nbi, out);
}

namespace {

__device__ __forceinline__ int32_t bead_slot_of(const Dev &s, int64_t b) { return s.bead_slot[b]; }

// The paper's six measurements of one platelet (Sec. 3.3), one block per platelet:
// angular velocity omega = I^-1 L about the centre of mass, translational and rotational
// kinetic energy, and the flow speed at the centre of mass (|mean velocity| of the fluid
// closer than flow_r).  Bead positions are unwrapped about the platelet's first bead;
// every sum is a fixed-order block reduction.
__global__ __launch_bounds__(kBS) void k_paper_feat(Dev s, double flow_r, double *out)
{
    __shared__ double lds[13 * kBS];
    __shared__ double com[3], vel[3];
    const int64_t p = blockIdx.x;
    const int64_t N = s.N;
    const int32_t b0 = s.plt_off[p], b1 = s.plt_off[p + 1];
    const double mb = s.m[2];
    if (b1 <= b0) {
        if (threadIdx.x < 6) out[6 * p + threadIdx.x] = 0.0;
        return;
    }
    const int32_t t0 = bead_slot_of(s, b0);
    const double r00 = s.x[t0], r01 = s.x[N + t0], r02 = s.x[2 * N + t0];
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t b = b0 + threadIdx.x; b < b1; b += kBS) {
        const int32_t t = bead_slot_of(s, b);
        acc[0] += mb;
        acc[1] += mb * min_image(s, 0, s.x[t] - r00);
        acc[2] += mb * min_image(s, 1, s.x[N + t] - r01);
        acc[3] += mb * min_image(s, 2, s.x[2 * N + t] - r02);
        acc[4] += mb * s.v[t];
        acc[5] += mb * s.v[N + t];
        acc[6] += mb * s.v[2 * N + t];
    }
    block_sum<12>(acc, lds);
    const double M = acc[0];
    if (threadIdx.x == 0) {
        com[0] = r00 + acc[1] / M;
        com[1] = r01 + acc[2] / M;
        com[2] = r02 + acc[3] / M;
        vel[0] = acc[4] / M;
        vel[1] = acc[5] / M;
        vel[2] = acc[6] / M;
    }
    __syncthreads();
    // angular momentum (3) and inertia tensor (6 independent entries) about the COM
    double a2[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // L, I, fluid velocity sum, fluid count
    for (int32_t b = b0 + threadIdx.x; b < b1; b += kBS) {
        const int32_t t = bead_slot_of(s, b);
        const double r0 = min_image(s, 0, s.x[t] - com[0]), r1 = min_image(s, 1, s.x[N + t] - com[1]),
                     r2 = min_image(s, 2, s.x[2 * N + t] - com[2]);
        const double u0 = s.v[t] - vel[0], u1 = s.v[N + t] - vel[1], u2 = s.v[2 * N + t] - vel[2];
        a2[0] += mb * (r1 * u2 - r2 * u1);
        a2[1] += mb * (r2 * u0 - r0 * u2);
        a2[2] += mb * (r0 * u1 - r1 * u0);
        const double rr = r0 * r0 + r1 * r1 + r2 * r2;
        a2[3] += mb * (rr - r0 * r0);
        a2[4] += mb * (-r0 * r1);
        a2[5] += mb * (-r0 * r2);
        a2[6] += mb * (rr - r1 * r1);
        a2[7] += mb * (-r1 * r2);
        a2[8] += mb * (rr - r2 * r2);
    }
    // fluid within flow_r of the COM: the cells that can hold such particles
    const int R0 = (int)ceil(flow_r / s.side[0]), R1 = (int)ceil(flow_r / s.side[1]), R2 = (int)ceil(flow_r / s.side[2]);
    const int W0 = 2 * R0 + 1, W1 = 2 * R1 + 1, W2 = 2 * R2 + 1;
    const int cx = cell_coord(s, 0, com[0]), cy = cell_coord(s, 1, com[1]), cz = cell_coord(s, 2, com[2]);
    const double fr2 = flow_r * flow_r;
    for (int q = threadIdx.x; q < W0 * W1 * W2; q += kBS) {
        int ix = cx + q % W0 - R0, iy = cy + (q / W0) % W1 - R1, iz = cz + q / (W0 * W1) - R2;
        bool ok = true;
        if (ix < 0 || ix >= s.nc[0]) { ok = ok && s.per[0] && W0 <= s.nc[0]; ix = (ix % s.nc[0] + s.nc[0]) % s.nc[0]; }
        if (iy < 0 || iy >= s.nc[1]) { ok = ok && s.per[1] && W1 <= s.nc[1]; iy = (iy % s.nc[1] + s.nc[1]) % s.nc[1]; }
        if (iz < 0 || iz >= s.nc[2]) { ok = ok && s.per[2] && W2 <= s.nc[2]; iz = (iz % s.nc[2] + s.nc[2]) % s.nc[2]; }
        if (!ok) continue;
        const int64_t c = cell_index(s, ix, iy, iz);
        for (int32_t j = s.cell_start[c]; j < s.cell_start[c + 1]; ++j) {
            if (s.id[j] >= (uint64_t)s.nf) continue;  // fluid only
            const double d0 = min_image(s, 0, s.x[j] - com[0]), d1 = min_image(s, 1, s.x[N + j] - com[1]),
                         d2 = min_image(s, 2, s.x[2 * N + j] - com[2]);
            if (d0 * d0 + d1 * d1 + d2 * d2 < fr2) {
                a2[9] += s.v[j];
                a2[10] += s.v[N + j];
                a2[11] += s.v[2 * N + j];
                a2[12] += 1.0;
            }
        }
    }
    block_sum<13>(a2, lds);
    if (threadIdx.x == 0) {
        // omega = I^-1 L by Cramer's rule
        const double I[3][3] = {{a2[3], a2[4], a2[5]}, {a2[4], a2[6], a2[7]}, {a2[5], a2[7], a2[8]}};
        const double L[3] = {a2[0], a2[1], a2[2]};
        auto det3 = [](const double (&A)[3][3]) {
            return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                   A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        };
        const double det = det3(I);
        double om[3] = {0.0, 0.0, 0.0};
        if (fabs(det) >= 1e-300)
            for (int c = 0; c < 3; ++c) {
                double Mx[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int k = 0; k < 3; ++k) Mx[r][k] = k == c ? L[r] : I[r][k];
                om[c] = det3(Mx) / det;
            }
        double *o = out + 6 * p;
        o[0] = om[0];
        o[1] = om[1];
        o[2] = om[2];
        o[3] = 0.5 * M * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]);
        o[4] = 0.5 * (om[0] * L[0] + om[1] * L[1] + om[2] * L[2]);
        o[5] = 0.0;
        if (a2[12] > 0.0) {
            const double f0 = a2[9] / a2[12], f1 = a2[10] / a2[12], f2 = a2[11] / a2[12];
            o[5] = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
        }
    }
}

// Per-bead membrane stress (Sec. 4.2, Fig. 5), added to sum[b]: the pressure-like trace
// of the per-particle virial times volume, (m |v|^2 + W) / 3, with W the bead's share
// of r.F of the conservative inner-group terms: half of every WCA pair of its list
// (fluid, wall and bead partners), of every Eq. 4 aggregation pair, bond and Morse bond.
// (Angles carry no virial: U depends on theta only, which a dilation leaves unchanged.)
__global__ __launch_bounds__(kBS) void k_bead_stress(Dev s, double *sum)
{
    const int64_t b = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (b >= s.nb) return;
    const int64_t N = s.N;
    const int32_t t = s.member_slot[b];
    const double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
    const double v0 = s.v[t], v1 = s.v[N + t], v2 = s.v[2 * N + t];
    double w = 0.0;
    const int64_t pe = s.pair_off[b + 1] < s.cap_pairs ? s.pair_off[b + 1] : s.cap_pairs;
    const int32_t body_b = s.body[b];
    for (int64_t q = s.pair_off[b]; q < pe; ++q) {
        const int32_t j = s.pair_list[q];
        const double d0 = min_image(s, 0, x0 - s.x[j]), d1 = min_image(s, 1, x1 - s.x[N + j]),
                     d2 = min_image(s, 2, x2 - s.x[2 * N + j]);
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (!(r2 > 0.0)) continue;
        if (r2 < s.lj_rc2) {
            const double sr2 = s.lj_sig2 / r2;
            const double sr6 = sr2 * sr2 * sr2;
            w += 0.5 * 24.0 * s.lj_eps * (2.0 * sr6 * sr6 - sr6);  // r.F = fs r^2
        }
        if (s.agg_on && r2 < s.agg_rc2 && s.id[j] >= (uint64_t)s.b0 && s.body[s.id[j] - s.b0] != body_b) {
            const double r = sqrt(r2);
            const double ex = exp(-s.agg_a * (r - s.agg_r0));
            w += 0.5 * (2.0 * s.agg_a * s.agg_D * (ex * ex - ex) + s.agg_fA * (1.0 - r / s.agg_r0)) * r;
        }
    }
    for (int32_t q = s.bond_off[b]; q < s.bond_off[b + 1]; ++q) {
        const int32_t u = s.bond_slot[q];
        const double d0 = min_image(s, 0, x0 - s.x[u]), d1 = min_image(s, 1, x1 - s.x[N + u]),
                     d2 = min_image(s, 2, x2 - s.x[2 * N + u]);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        w += 0.5 * (-2.0 * s.kb * (r - s.bond_r0[q]) * r);
    }
    for (int32_t q = s.mor_off[b]; q < s.mor_off[b + 1]; ++q) {
        const int32_t u = s.mor_slot[q];
        const double d0 = min_image(s, 0, x0 - s.x[u]), d1 = min_image(s, 1, x1 - s.x[N + u]),
                     d2 = min_image(s, 2, x2 - s.x[2 * N + u]);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double ex = exp(-s.ma * (r - s.mr0));
        w += 0.5 * 2.0 * s.ma * s.mD * (ex * ex - ex) * r;
    }
    sum[b] += (s.m[2] * (v0 * v0 + v1 * v1 + v2 * v2) + w) / 3.0;
}

}  // namespace

void paper_features(const Dev &s, double flow_r, double *out, hipStream_t st)
{
    if (s.P == 0) return;
    hipLaunchKernelGGL(k_paper_feat, dim3((unsigned)s.P), dim3(kBS), 0, st, s, flow_r, out);
}

void bead_stress(const Dev &s, double *sum, hipStream_t st)
{
    if (s.nb == 0) return;
    hipLaunchKernelGGL(k_bead_stress, dim3(nblocks(s.nb, kBS)), dim3(kBS), 0, st, s, sum);
}

size_t feature_scratch_doubles(int64_t P) { return (size_t)P * kFeatBlocks * kFeatNV; }

void features(const Dev &s, float *ring, int row, float *last, double *scratch, double h_pend, hipStream_t st)
{
    if (s.P == 0) return;
    const double contact_r = kContactRadius;
    const unsigned g = (unsigned)(s.P * kFeatBlocks);
    hipLaunchKernelGGL(k_feat_moments, dim3(g), dim3(kBS), 0, st, s, scratch, contact_r * contact_r, h_pend);
    hipLaunchKernelGGL(k_feat_final, dim3((unsigned)s.P), dim3(64), 0, st, s, (const double *)scratch, ring, row, last);
}

}  // namespace aimts
