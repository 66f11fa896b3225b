// Outer force group: DPD conservative + dissipative + random pair forces (Sec. 3.2,
// Eq. 1) between fluid particles and between fluid and frozen wall particles, plus the
// body force on the fluid (F^E of Eq. 1).
//
// One thread per slot gathers the forces on its particle (each pair is evaluated from
// both ends: no atomics, deterministic, exactly antisymmetric).  The work splits in two
// phases so that the expensive part does not run under a mostly inactive wavefront:
//
//  1. scan: the candidates of the 27 surrounding cells are tested against a cutoff
//     enlarged by 8 float ulps of the box extent, using the float4 copy of the positions
//     written at the rebuild (one 16-byte load per candidate).  Cells are numbered
//     z-fastest, so the three cells (ix, iy, iz-1..iz+1) are one contiguous slot range
//     (split only at a periodic z wrap): 9 long ranges instead of 27 short ones.
//     Accepted partners are appended to a per-thread list in LDS, stored lane-major so
//     that consecutive lanes touch consecutive banks.
//  2. pairs: each thread runs over its own list only -- Philox4x32-10, Box-Muller and
//     the pair law -- so ~12.6 accepted pairs cost ~12.6 iterations instead of the
//     expensive branch executing whenever any of 64 lanes accepts one of ~81 candidates.
//     The separation is formed in float64 with the minimum image and tested exactly
//     against rc (float32 mode then rounds it).  Blocks are ordered XCD-aware.
//
// R = double: all arithmetic in float64.  R = float: after the rounded separation,
// everything (including the Gaussian from the same 32-bit words) is float32 with
// float32 accumulation.
#include "common.h"

namespace aimts {

namespace {

constexpr int kBS = 256;
constexpr int kCap = 32;  // accepted partners buffered per thread before they are processed

template <typename R>
struct PairCtx {
    double x0, x1, x2, v0, v1, v2;
    uint32_t idi;
    R a, gam, sig, inv_rc, isdt;
};

// Data of one partner, fetched ahead of its use so several pairs' loads are in flight.
struct Partner {
    double x0, x1, x2, v0, v1, v2;
    uint32_t id;
};

__device__ __forceinline__ Partner fetch(const Dev &s, int32_t j)
{
    const int64_t N = s.N;
    Partner q;
    q.x0 = s.x[j];
    q.x1 = s.x[N + j];
    q.x2 = s.x[2 * N + j];
    q.v0 = s.v[j];
    q.v1 = s.v[N + j];
    q.v2 = s.v[2 * N + j];
    q.id = s.id[j];
    return q;
}

template <typename R>
__device__ __forceinline__ void pair_force(const Dev &s, const PairCtx<R> &c, const Partner &q, uint64_t count, R &f0,
                                           R &f1, R &f2)
{
    if (q.id >= (uint64_t)s.b0) return;  // beads are not in the outer group
    const double e0 = min_image(s, 0, c.x0 - q.x0);
    const double e1 = min_image(s, 1, c.x1 - q.x1);
    const double e2 = min_image(s, 2, c.x2 - q.x2);
    const double re2 = e0 * e0 + e1 * e1 + e2 * e2;
    if (!(re2 < s.rc2) || re2 == 0.0) return;  // exact test (the scan pre-filtered in float)
    const R d0 = (R)e0, d1 = (R)e1, d2 = (R)e2;
    const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const R rinv = R(1) / sqrt(r2);
    const R r = r2 * rinv;
    const R w = R(1) - r * c.inv_rc;
    const R ev = (d0 * (R)(c.v0 - q.v0) + d1 * (R)(c.v1 - q.v1) + d2 * (R)(c.v2 - q.v2)) * rinv;
    uint32_t w0, w1;
    pair_words(c.idi, q.id, count, s.key0, s.key1, w0, w1);
    R z;
    if constexpr (sizeof(R) == 8) z = gauss64(w0, w1);
    else z = gauss32(w0, w1);
    const R fs = (c.a * w - c.gam * w * w * ev + c.sig * w * z * c.isdt) * rinv;
    f0 += fs * d0;
    f1 += fs * d1;
    f2 += fs * d2;
}

// Process the n buffered partners of this thread, two at a time (both fetched first).
template <typename R>
__device__ __forceinline__ void flush(const Dev &s, const PairCtx<R> &c, const int32_t (*lst)[kBS], int n,
                                      uint64_t count, R &f0, R &f1, R &f2)
{
    int p = 0;
    for (; p + 1 < n; p += 2) {
        const Partner a = fetch(s, lst[p][threadIdx.x]);
        const Partner b = fetch(s, lst[p + 1][threadIdx.x]);
        pair_force<R>(s, c, a, count, f0, f1, f2);
        pair_force<R>(s, c, b, count, f0, f1, f2);
    }
    if (p < n) pair_force<R>(s, c, fetch(s, lst[p][threadIdx.x]), count, f0, f1, f2);
}

constexpr int kBatch = 8;  // candidates whose positions are loaded together in the scan

template <typename R>
__global__ __launch_bounds__(kBS) void k_dpd(Dev s, uint64_t count, double inv_sqrt_dt, R *f, unsigned nblk)
{
    __shared__ int32_t lst[kCap][kBS];
    const int64_t blk = xcd_block(nblk);
    if (blk < 0) return;
    const int64_t i = blk * kBS + threadIdx.x;
    if (i >= s.N) return;
    const int64_t N = s.N;
    PairCtx<R> c;
    c.idi = s.id[i];
    R f0 = R(0), f1 = R(0), f2 = R(0);
    if (c.idi < (uint64_t)s.nf) {
        c.x0 = s.x[i];
        c.x1 = s.x[N + i];
        c.x2 = s.x[2 * N + i];
        c.v0 = s.v[i];
        c.v1 = s.v[N + i];
        c.v2 = s.v[2 * N + i];
        c.a = (R)s.a;
        c.gam = (R)s.gamma;
        c.sig = (R)s.sigma;
        c.inv_rc = (R)s.inv_rc;
        c.isdt = (R)inv_sqrt_dt;
        const float pre2 = (float)s.pre_rc2;
        const float fx0 = (float)c.x0, fx1 = (float)c.x1, fx2 = (float)c.x2;
        const int cx = cell_coord(s, 0, c.x0), cy = cell_coord(s, 1, c.x1), cz = cell_coord(s, 2, c.x2);
        const int nz = s.nc[2];
        int cnt = 0;
        for (int dy = -1; dy <= 1; ++dy) {
            int iy = cy + dy;
            double sy = 0.0;
            if (iy < 0 || iy >= s.nc[1]) {
                if (!s.per[1]) continue;
                sy = iy < 0 ? s.L[1] : -s.L[1];  // the neighbour cell's image lies at -sy
                iy = iy < 0 ? iy + s.nc[1] : iy - s.nc[1];
            }
            const float hy = fx1 + (float)sy;
            for (int dx = -1; dx <= 1; ++dx) {
                int ix = cx + dx;
                double sx = 0.0;
                if (ix < 0 || ix >= s.nc[0]) {
                    if (!s.per[0]) continue;
                    sx = ix < 0 ? s.L[0] : -s.L[0];
                    ix = ix < 0 ? ix + s.nc[0] : ix - s.nc[0];
                }
                const float hx = fx0 + (float)sx;
                const int64_t row = ((int64_t)iy * s.nc[0] + ix) * nz;
                auto scan = [&](int32_t beg, int32_t end, float hz) {
                    for (int32_t j0 = beg; j0 < end; j0 += kBatch) {
                        if (cnt > kCap - kBatch) {
                            flush<R>(s, c, lst, cnt, count, f0, f1, f2);
                            cnt = 0;
                        }
                        float4 q[kBatch];
#pragma unroll
                        for (int u = 0; u < kBatch; ++u)
                            q[u] = j0 + u < end ? s.xf[j0 + u] : make_float4(3.0e38f, 3.0e38f, 3.0e38f, 0.0f);
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const float e0 = hx - q[u].x, e1 = hy - q[u].y, e2 = hz - q[u].z;
                            const float r2 = e0 * e0 + e1 * e1 + e2 * e2;
                            if (r2 < pre2 && j0 + u != i) lst[cnt++][threadIdx.x] = j0 + u;
                        }
                    }
                };
                if (cz >= 1 && cz + 1 < nz) {
                    // the three z-neighbour cells are one contiguous slot range
                    scan(s.cell_start[row + cz - 1], s.cell_start[row + cz + 2], fx2);
                } else {
                    for (int dz = -1; dz <= 1; ++dz) {
                        int iz = cz + dz;
                        double sz = 0.0;
                        if (iz < 0 || iz >= nz) {
                            if (!s.per[2]) continue;
                            sz = iz < 0 ? s.L[2] : -s.L[2];
                            iz = iz < 0 ? iz + nz : iz - nz;
                        }
                        scan(s.cell_start[row + iz], s.cell_start[row + iz + 1], fx2 + (float)sz);
                    }
                }
            }
        }
        flush<R>(s, c, lst, cnt, count, f0, f1, f2);
        f0 += (R)s.g[0];
        f1 += (R)s.g[1];
        f2 += (R)s.g[2];
    }
    f[i] = f0;
    f[N + i] = f1;
    f[2 * N + i] = f2;
}

}  // namespace

void outer_forces(const Dev &s, uint64_t count, double dt_outer, hipStream_t st)
{
    const double isdt = 1.0 / sqrt(dt_outer);
    const unsigned nblk = nblocks(s.N, kBS);
    if (s.fp32)
        hipLaunchKernelGGL(k_dpd<float>, dim3(xcd_grid(nblk)), dim3(kBS), 0, st, s, count, isdt, (float *)s.fo, nblk);
    else
        hipLaunchKernelGGL(k_dpd<double>, dim3(xcd_grid(nblk)), dim3(kBS), 0, st, s, count, isdt, (double *)s.fo, nblk);
}

}  // namespace aimts
