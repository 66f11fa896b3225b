// Outer force group: DPD conservative + dissipative + random pair forces (Sec. 3.2,
// Eq. 1) between fluid particles and between fluid and frozen wall particles, plus the
// body force on the fluid (F^E of Eq. 1).
//
// One thread per slot owns the force on its particle (each pair is evaluated from both
// ends: no atomics, deterministic, exactly antisymmetric).  The work splits in two
// phases so that neither runs under a mostly inactive wavefront:
//
//  1. scan: each lane tests the candidates of its own neighbour cells against a cutoff
//     enlarged by 8 float ulps of the box extent, using the float4 copy of the positions
//     written at the rebuild (one 16-byte load per candidate).  The cells' bins hold the
//     fluid and wall particles only (beads sort into bins of their own), so every
//     candidate is a DPD particle.  Cells are numbered z-fastest, so the z-neighbours of
//     a column are one contiguous slot range, plus one wrapped cell at a periodic z face.
//     Columns and z cells whose box lies entirely beyond that cutoff from the particle
//     are skipped.
//     Accepted partners go to a per-lane list in LDS.
//  2. pairs: lane-owned rounds (each lane its own next partner) while most lanes still
//     have one, then the rest of the 64 lists as one sequence, 64 pairs at a time (lane l
//     takes pair p0 + l whatever particle owns it), so that lanes stay busy however
//     unevenly the partners are spread.  Each balanced pair result goes to LDS and the
//     owning lane adds the results of its own pairs in list order.  A pair costs
//     Philox4x32-10, Box-Muller and the pair law; the separation is formed in float64
//     with the minimum image and tested exactly against rc (float32 mode then rounds it).
//
// Blocks are ordered XCD-aware.  R = double: all arithmetic in float64.  R = float:
// after the rounded separation everything (including the Gaussian from the same 32-bit
// words) is float32 with float32 accumulation.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>

namespace aimts {

namespace {

constexpr int kBS = 64;
constexpr int kWaves = kBS / 64;
constexpr int kCap = 24;              // partners buffered per lane before a lane-local flush
constexpr int kStride = kCap + 1;     // odd row stride: 32 consecutive lanes write 32 different banks
constexpr int kBatch = 4;             // candidates whose positions are loaded together in the scan
constexpr int kOwnMin = 40;           // fewest busy lanes for a lane-owned pair round

template <typename R>
struct Law {
    R a, gam, sig, inv_rc, isdt;
};

// Position, velocity and id of one particle.
struct Particle {
    double x0, x1, x2, v0, v1, v2;
    uint32_t id;
};

// float64 mode reads the velocities themselves; float32 mode, whose pair law rounds the
// velocity difference to float anyway, reads velocity and id in one 16-byte load from
// the float copy written at the rebuild (the pair phase is bound by its loads).
template <typename R>
__device__ __forceinline__ Particle fetch(const Dev &s, int64_t j)
{
    const int64_t N = s.N;
    Particle q;
    q.x0 = s.x[j];
    q.x1 = s.x[N + j];
    q.x2 = s.x[2 * N + j];
    if constexpr (sizeof(R) == 8) {
        q.v0 = s.v[j];
        q.v1 = s.v[N + j];
        q.v2 = s.v[2 * N + j];
        q.id = s.id[j];
    } else {
        const float4 w = s.vf[j];
        q.v0 = w.x;
        q.v1 = w.y;
        q.v2 = w.z;
        q.id = __float_as_uint(w.w);
    }
    return q;
}

// Adds the force of q on p to (g0, g1, g2) if they are closer than rc.
template <typename R>
__device__ __forceinline__ void pair_force(const Dev &s, const Law<R> &k, const Particle &p, const Particle &q,
                                           uint64_t count, R &g0, R &g1, R &g2)
{
    const double e0 = min_image(s, 0, p.x0 - q.x0);
    const double e1 = min_image(s, 1, p.x1 - q.x1);
    const double e2 = min_image(s, 2, p.x2 - q.x2);
    const double re2 = e0 * e0 + e1 * e1 + e2 * e2;
    if (!(re2 < s.rc2) || re2 == 0.0) return;  // exact test (the scan pre-filtered in float)
    const R d0 = (R)e0, d1 = (R)e1, d2 = (R)e2;
    const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
    R rinv;
    if constexpr (sizeof(R) == 8) rinv = 1.0 / sqrt(r2);
    else rinv = __builtin_amdgcn_rsqf(r2);  // hardware reciprocal square root (about 1 ulp)
    const R r = r2 * rinv;
    const R w = R(1) - r * k.inv_rc;
    const R ev = (d0 * (R)(p.v0 - q.v0) + d1 * (R)(p.v1 - q.v1) + d2 * (R)(p.v2 - q.v2)) * rinv;
    uint32_t w0, w1;
    pair_words(p.id, q.id, count, s.key0, s.key1, w0, w1);
    R z;
    if constexpr (sizeof(R) == 8) z = gauss64(w0, w1);
    else z = gauss32(w0, w1);
    const R fs = (k.a * w - k.gam * w * w * ev + k.sig * w * z * k.isdt) * rinv;
    g0 += fs * d0;
    g1 += fs * d1;
    g2 += fs * d2;
}

__device__ __forceinline__ void wave_lds_sync()
{
    // LDS traffic of one wavefront is processed in order; keep the compiler from moving
    // accesses across this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane-local processing of this lane's list (only when a list fills up mid-scan).
template <typename R>
__device__ __forceinline__ void flush_lane(const Dev &s, const Law<R> &k, const Particle &me, const int32_t *mine, int n,
                                        uint64_t count, R &f0, R &f1, R &f2)
{
    for (int p = 0; p < n; ++p) pair_force<R>(s, k, me, fetch<R>(s, mine[p]), count, f0, f1, f2);
}

// All 64 lists of the wavefront; must be called by all 64 lanes.  First come
// lane-owned rounds (round r: every lane with more than r partners takes its r-th) for
// as long as at least kOwnMin lanes take part: such a round needs no owner search, no
// reduction and no fetch of the owner, so it beats a balanced window while most lanes
// are busy.  The rest of the lists then goes as one sequence in windows of 64 pairs;
// within a window the pairs of one owner are consecutive lanes: a segmented inclusive
// scan over the lanes (fixed tree) leaves each owner's window sum in the last lane of
// its segment, which hands it to the owner through LDS.
template <typename R>
__device__ __forceinline__ void flush_wave(const Dev &s, const Law<R> &k, const int32_t *wl, R (*rs)[64], int cnt,
                                           int64_t wave0, uint64_t count, int lane, const Particle &me, R &f0,
                                           R &f1, R &f2)
{
    int r0 = 0;
    while (__popcll(__ballot(cnt > r0)) >= kOwnMin) {
        if (cnt > r0) pair_force<R>(s, k, me, fetch<R>(s, wl[lane * kStride + r0]), count, f0, f1, f2);
        ++r0;
    }
    cnt = cnt > r0 ? cnt - r0 : 0;
    int32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int32_t total = __shfl(incl, 63, 64);
    const int32_t excl = incl - cnt;
    for (int32_t p0 = 0; p0 < total; p0 += 64) {
        const int32_t p = p0 + lane;
        const bool ok = p < total;
        const int32_t pc = ok ? p : total - 1;
        int o = 0;  // owner: the number of lanes whose inclusive prefix is <= pc
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (__shfl(incl, o + step - 1, 64) <= pc) o += step;
        const int32_t oex = __shfl(excl, o, 64), oin = __shfl(incl, o, 64);
        R g0 = R(0), g1 = R(0), g2 = R(0);
        if (ok) {
            const int32_t j = wl[o * kStride + r0 + (pc - oex)];
            pair_force<R>(s, k, fetch<R>(s, wave0 + o), fetch<R>(s, j), count, g0, g1, g2);
        }
        // segmented inclusive scan: lanes [first, lane] of this owner's segment
        const int first = oex > p0 ? oex - p0 : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const R t0 = __shfl_up(g0, d, 64), t1 = __shfl_up(g1, d, 64), t2 = __shfl_up(g2, d, 64);
            if (lane - d >= first) {
                g0 += t0;
                g1 += t1;
                g2 += t2;
            }
        }
        const int last = (oin < p0 + 64 ? oin : (total < p0 + 64 ? total : p0 + 64)) - p0 - 1;
        if (ok && lane == last) {
            rs[0][o] = g0;
            rs[1][o] = g1;
            rs[2][o] = g2;
        }
        wave_lds_sync();
        if ((excl > p0 ? excl : p0) < (incl < p0 + 64 ? incl : p0 + 64)) {  // this lane owns pairs in the window
            f0 += rs[0][lane];
            f1 += rs[1][lane];
            f2 += rs[2][lane];
        }
        wave_lds_sync();
    }
}

template <typename R>
__global__ __launch_bounds__(kBS) void k_dpd(Dev s, uint64_t count, double inv_sqrt_dt, R *f, unsigned nblk)
{
    __shared__ int32_t lst[kWaves][64 * kStride];
    __shared__ R res[kWaves][3][64];
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;  // whole block
    const int64_t blk = s.dpd_order[lb];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t N = s.N;
    const int64_t wave0 = blk * kBS + wv * 64;
    const int64_t i = wave0 + lane;
    int32_t *mine = &lst[wv][lane * kStride];
    Law<R> law;
    law.a = (R)s.a;
    law.gam = (R)s.gamma;
    law.sig = (R)s.sigma;
    law.inv_rc = (R)s.inv_rc;
    law.isdt = (R)inv_sqrt_dt;
    R f0 = R(0), f1 = R(0), f2 = R(0);
    int cnt = 0;
    const bool live = i < N && s.id[i] < (uint64_t)s.nf;
    Particle me{};
    if (live) {
        me = fetch<R>(s, i);
        const float pre2 = (float)s.pre_rc2;
        const float fx0 = (float)me.x0, fx1 = (float)me.x1, fx2 = (float)me.x2;
        const int cx = cell_coord(s, 0, me.x0), cy = cell_coord(s, 1, me.x1), cz = cell_coord(s, 2, me.x2);
        // Pruning works in float with a margin far above its rounding: a cell is skipped
        // only if its box lies beyond the pre-filter cutoff + 1e-3 from the particle.  The
        // offsets inside the own cell give the gaps: side - o to the next cell above, o below.
        const float prune = sqrtf(pre2) + 1e-3f, prune2 = prune * prune;
        const float ox = (float)((me.x0 - s.lo[0]) - cx * s.side[0]);
        const float oy = (float)((me.x1 - s.lo[1]) - cy * s.side[1]);
        const float oz = (float)((me.x2 - s.lo[2]) - cz * s.side[2]);
        const float sdx = (float)s.side[0], sdy = (float)s.side[1], sdz = (float)s.side[2];
        const float gzm = oz * oz, gzp = (sdz - oz) * (sdz - oz);
        const int nz = s.nc[2];
        const int32_t i32 = (int32_t)i;
        // float4 position copies through a buffer descriptor: 32-bit offsets, and loads past
        // the end of the array return zeros (such slots are never accepted: j >= end)
        const __amdgpu_buffer_rsrc_t rx =
            __builtin_amdgcn_make_buffer_rsrc((void *)s.xf, (short)0, (int)(N * 16), 0x00020000);
        // Candidates [beg, end) seen from the image-shifted float position (hx, hy, hz).
        // Branch-free: every candidate is written to the list slot after the last accepted
        // one and kept only if accepted (the flush check leaves room for a whole batch).
        auto scan = [&](int32_t beg, int32_t end, float hx, float hy, float hz) {
            for (int32_t j0 = beg; j0 < end; j0 += kBatch) {
                if (cnt > kCap - kBatch) {
                    flush_lane<R>(s, law, me, mine, cnt, count, f0, f1, f2);
                    cnt = 0;
                }
                float qx[kBatch], qy[kBatch], qz[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rx, (j0 + u) * 16, 0, 0);
                    qx[u] = __uint_as_float(w[0]);
                    qy[u] = __uint_as_float(w[1]);
                    qz[u] = __uint_as_float(w[2]);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const float e0 = hx - qx[u], e1 = hy - qy[u], e2 = hz - qz[u];
                    const float r2 = e0 * e0 + e1 * e1 + e2 * e2;
                    const int32_t j = j0 + u;
                    const bool take = (r2 < pre2) & (j < end) & (j != i32);
                    mine[cnt] = j;
                    cnt += take ? 1 : 0;
                }
            }
        };
        for (int dy = -1; dy <= 1; ++dy) {
            const float gy = dy > 0 ? sdy - oy : oy;
            const float gy2 = dy != 0 ? gy * gy : 0.0f;
            if (gy2 >= prune2) continue;
            int iy = cy + dy;
            double sy = 0.0;
            if (iy < 0 || iy >= s.nc[1]) {
                if (!s.per[1]) continue;
                sy = iy < 0 ? s.L[1] : -s.L[1];  // the neighbour cell's image lies at -sy
                iy = iy < 0 ? iy + s.nc[1] : iy - s.nc[1];
            }
            const float hy = fx1 + (float)sy;
            for (int dx = -1; dx <= 1; ++dx) {
                const float gx = dx > 0 ? sdx - ox : ox;
                const float rem = prune2 - gy2 - (dx != 0 ? gx * gx : 0.0f);
                if (rem <= 0.0f) continue;
                int ix = cx + dx;
                double sx = 0.0;
                if (ix < 0 || ix >= s.nc[0]) {
                    if (!s.per[0]) continue;
                    sx = ix < 0 ? s.L[0] : -s.L[0];
                    ix = ix < 0 ? ix + s.nc[0] : ix - s.nc[0];
                }
                const float hx = fx0 + (float)sx;
                const int row = (iy * s.nc[0] + ix) * nz;
                const int zlo = cz - (gzm < rem ? 1 : 0), zhi = cz + (gzp < rem ? 1 : 0);
                // the column's z cells inside the box are one contiguous slot range; a
                // periodic z axis adds at most one wrapped cell (at least 5 cells per axis)
                const int mlo = zlo < 0 ? 0 : zlo, mhi = zhi >= nz ? nz - 1 : zhi;
                scan(s.cell_start[row + mlo], s.cell_start[row + mhi + 1], hx, hy, fx2);
                if (s.per[2] && (zlo < 0 || zhi >= nz)) {
                    const int wz = zlo < 0 ? nz - 1 : 0;
                    const float sz = (float)(zlo < 0 ? s.L[2] : -s.L[2]);  // the wrapped cell's image lies at -sz
                    scan(s.cell_start[row + wz], s.cell_start[row + wz + 1], hx, hy, fx2 + sz);
                }
            }
        }
    }
    flush_wave<R>(s, law, lst[wv], res[wv], cnt, wave0, count, lane, me, f0, f1, f2);
    if (i < N) {
        if (live) {
            f0 += (R)s.g[0];
            f1 += (R)s.g[1];
            f2 += (R)s.g[2];
        }
        f[i] = f0;
        f[N + i] = f1;
        f[2 * N + i] = f2;
    }
}

}  // namespace

int64_t dpd_blocks(int64_t N) { return nblocks(N, kBS); }

// The order of the DPD kernel's blocks (each 64 consecutive slots).  Slots run by cell
// column, y-major, so in slot order the three rows of columns a block reads (its own and
// the two neighbouring y rows) span two whole rows of the box: far more than one XCD's
// L2 on a long channel, and every row would be fetched from HBM three times.  Blocks are
// taken instead in tiles of columns along x, the tile's rows one after the other, so
// that the rows around the ones in flight stay in L2.  A tile row holds about 6,144
// slots (measured best between 3,000 and 14,000 on channels with 111 and 200 particles
// per column: 10-13 % faster than whole rows).  A block's column is estimated from its
// first slot and the mean number of fluid and wall particles per column (the order only
// affects locality); blocks of bead slots, which the kernel skips, come last.
void dpd_block_order(int64_t N, int64_t n_fw, const int32_t nc[3], std::vector<int32_t> &order)
{
    const int64_t nblk = dpd_blocks(N), nx = nc[0], ny = nc[1], ncol = nx * ny;
    const double per_col = n_fw > 0 ? (double)n_fw / (double)ncol : 1.0;
    const int64_t kTile = std::max<int64_t>(8, std::min<int64_t>(nx, std::llround(6144.0 / per_col)));
    std::vector<std::pair<int64_t, int32_t>> key(nblk);
    for (int64_t p = 0; p < nblk; ++p) {
        const int64_t t0 = p * kBS;
        int64_t k = INT64_MAX;
        if (t0 < n_fw) {
            const int64_t col = std::min<int64_t>((int64_t)((double)t0 / per_col), ncol - 1);
            const int64_t iy = col / nx, ix = col % nx;
            k = ((ix / kTile) * ny + iy) * nx + ix;
        }
        key[p] = {k, (int32_t)p};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<int64_t, int32_t> &a, const std::pair<int64_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    order.resize(nblk);
    for (int64_t q = 0; q < nblk; ++q) order[q] = key[q].second;
}

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
