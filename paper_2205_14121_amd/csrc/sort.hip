// Cell-list neighbour build: counting sort of all particles by cell (the paper's
// per-outer-step neighbour-list construction, MSM pseudocode Table 1), plus the
// device-wide exclusive scan it needs.  The only atomics are the integer cell
// histogram; each slot is then placed by its rank (by particle index) within its cell,
// so the resulting order is deterministic.
#include "common.h"

namespace aimts {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;                    // per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ void k_fill_i32(int32_t *p, int32_t val, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

__global__ void k_fill_f64(double *p, double val, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t val, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

// Inclusive scan of one value per thread within the block (wave64 shuffles + LDS).
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t v, int32_t *lds_warp, int32_t &block_total)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) lds_warp[wid] = v;
    __syncthreads();
    if (wid == 0) {
        int32_t w = lane < (kScanBlock / 64) ? lds_warp[lane] : 0;
#pragma unroll
        for (int o = 1; o < kScanBlock / 64; o <<= 1) {
            int32_t t = __shfl_up(w, o, 64);
            if (lane >= o) w += t;
        }
        if (lane < kScanBlock / 64) lds_warp[lane] = w;
    }
    __syncthreads();
    if (wid > 0) v += lds_warp[wid - 1];
    block_total = lds_warp[kScanBlock / 64 - 1];
    __syncthreads();
    return v;
}

// Pass 1: per-tile sums.
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int32_t *in, int64_t n, int32_t *tile_sum)
{
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + (int64_t)q * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    int32_t total;
    block_inclusive_scan(s, lds, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Pass 2: exclusive scan of the tile sums by one block (loops over chunks).
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(int32_t *tile_sum, int64_t ntiles, int32_t *total_out)
{
    __shared__ int32_t lds[kScanBlock / 64];
    int32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < ntiles ? tile_sum[i] : 0;
        int32_t tot;
        int32_t inc = block_inclusive_scan(v, lds, tot);
        if (i < ntiles) tile_sum[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

// Pass 3: scan inside each tile with the tile's offset.  Each thread owns kScanItems
// consecutive elements.
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const int32_t *in, int32_t *out, int64_t n,
                                                          const int32_t *tile_off, const int32_t *total)
{
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = *total;
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t vals[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q;
        vals[q] = i < n ? in[i] : 0;
        s += vals[q];
    }
    int32_t tot;
    int32_t inc = block_inclusive_scan(s, lds, tot);
    int32_t run = tile_off[blockIdx.x] + inc - s;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q;
        if (i < n) out[i] = run;
        run += vals[q];
    }
}

__global__ void k_scan_total(int32_t *out, int64_t n, const int32_t *total) { out[n] = *total; }

// Pass 3 without pass 2, for at most kScanFusedTiles tiles: each block adds the sums of
// the tiles before it itself (integer sums: the same result in any order).
constexpr int64_t kScanFusedTiles = 1024;
__global__ __launch_bounds__(kScanBlock) void k_scan_down_fused(const int32_t *in, int32_t *out, int64_t n,
                                                                const int32_t *tile_sum)
{
    __shared__ int32_t lds[kScanBlock / 64];
    int32_t pre = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += kScanBlock) pre += tile_sum[t];
    int32_t tile_off;
    block_inclusive_scan(pre, lds, tile_off);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t vals[kScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + q;
        vals[q] = i < n ? in[i] : 0;
        sum += vals[q];
    }
    int32_t tot;
    const int32_t inc = block_inclusive_scan(sum, lds, tot);
    int32_t run = tile_off + inc - sum;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + q;
        if (i < n) out[i] = run;
        run += vals[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_off + tot;
}

// ---------------------------------------------------------------------------
// Counting sort
// ---------------------------------------------------------------------------
// Bin of every slot (its cell, offset by ncell for a bead) and its arrival rank in the
// bin histogram.  Slots are still in the previous step's bin order, so consecutive
// lanes mostly share a bin: each run of equal bins among consecutive lanes takes one
// atomic (all runs of a wavefront in the same instruction) and its lanes rank
// themselves by lane order within it.
__global__ __launch_bounds__(256) void k_bin(Dev s, int32_t *count, int32_t *cellof, int32_t *rank)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool live = i < s.N;
    int32_t c = -1;
    if (live) {
        const double p0 = s.x[i], p1 = s.x[s.N + i], p2 = s.x[2 * s.N + i];
        const int64_t bin0 = s.id[i] >= (uint64_t)s.b0 ? s.ncell : 0;
        // A non-finite position, or one more than a cell outside the box, comes only from
        // an unstable step (whose results are discarded).  Such particles are spread over
        // the bins by slot instead of piling up in one clamped edge cell, where the
        // per-bin work of the sort, the pair kernel and the lists grows with the square
        // of the bin's size.
        const double q[3] = {floor((p0 - s.lo[0]) / s.side[0]), floor((p1 - s.lo[1]) / s.side[1]),
                             floor((p2 - s.lo[2]) / s.side[2])};
        bool inside = true;
        int ic[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            inside = inside && q[k] >= -1.0 && q[k] <= (double)s.nc[k];
            // cell_coord's mapping of the same quotient
            int ik = inside ? (int)q[k] : 0;
            if (ik < 0) ik = s.per[k] ? ik + s.nc[k] : 0;
            if (ik >= s.nc[k]) ik = s.per[k] ? ik - s.nc[k] : s.nc[k] - 1;
            ic[k] = ik < 0 ? 0 : (ik >= s.nc[k] ? s.nc[k] - 1 : ik);
        }
        if (inside) {
            c = (int32_t)(cell_index(s, ic[0], ic[1], ic[2]) + bin0);
        } else {
            c = (int32_t)(i % s.ncell + bin0);
            atomicOr(s.err, kErrNonFinite);
        }
        cellof[i] = c;
    }
    const int32_t cprev = __shfl_up(c, 1, 64);
    const bool head = live && (lane == 0 || cprev != c);
    const uint64_t heads = __ballot(head);
    const int nlive = __popcll(__ballot(live));  // live lanes are a prefix of the wavefront
    const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0..lane (all ones for lane 63)
    const int leader = 63 - __clzll(heads & upto);
    int32_t base = 0;
    if (head) {
        const uint64_t later = heads & ~upto;
        const int next = later ? __ffsll((unsigned long long)later) - 1 : nlive;
        base = atomicAdd(&count[c], next - lane);
    }
    base = __shfl(base, live ? leader : 0, 64);
    if (live) rank[i] = base + (lane - leader);
}

__global__ void k_scatter(Dev s, const int32_t *cellof, const int32_t *rank, const int32_t *start,
                          uint32_t *tmp_id, int32_t *tmp_src)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.N) return;
    const int32_t t = start[cellof[i]] + rank[i];
    tmp_id[t] = s.id[i];
    tmp_src[t] = (int32_t)i;
}

// Final slot of each scattered particle: its rank by particle index among its bin's
// slots (fully parallel; no dependent chains even in the bead bins of dense membranes
// that hold a hundred beads), where its state is gathered to.  A wavefront's 64
// scattered slots are permuted only within their bins, so its writes stay within one
// contiguous window of slots.  The first scattered slot of each bin clears the bin's
// histogram count for the next rebuild (the scan has consumed it).
__global__ void k_rank_gather(Dev s, const int32_t *cellof, const uint32_t *tmp_id, const int32_t *tmp_src,
                              int32_t *count, double *x_new, double *v_new, uint32_t *id_new, int32_t *mos_new,
                              int32_t *src_of)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= s.N) return;
    const int32_t src = tmp_src[u];
    const uint32_t id = tmp_id[u];
    // the state is fetched while the rank is found
    double xs[3], vs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xs[k] = s.x[k * s.N + src];
        vs[k] = s.v[k * s.N + src];
    }
    const int32_t c = cellof[src];
    const int32_t beg = s.cell_start[c], end = s.cell_start[c + 1];
    int32_t r = 0;
    for (int32_t w = beg; w < end; ++w) r += tmp_id[w] < id;
    if (u == beg) count[c] = 0;
    const int64_t t = beg + r;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        x_new[k * s.N + t] = xs[k];
        v_new[k * s.N + t] = vs[k];
    }
    id_new[t] = id;
    src_of[t] = src;
    s.xf[t] = make_float4((float)xs[0], (float)xs[1], (float)xs[2], __uint_as_float(id));
    s.vf[t] = make_float4((float)vs[0], (float)vs[1], (float)vs[2], __uint_as_float(id));
    if (id >= (uint64_t)s.b0) {
        const int32_t b = (int32_t)(id - s.b0);
        s.bead_slot[b] = (int32_t)t;
        mos_new[t] = b;
    } else {
        mos_new[t] = -1;
    }
}

}  // namespace

void fill_i32(int32_t *p, int32_t val, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, 256)), dim3(256), 0, st, p, val, n);
}

void fill_f64(double *p, double val, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nblocks(n, 256)), dim3(256), 0, st, p, val, n);
}

void fill_u8(uint8_t *p, uint8_t val, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u8, dim3(nblocks(n, 256)), dim3(256), 0, st, p, val, n);
}

size_t scan_temp_bytes(int64_t n) { return sizeof(int32_t) * (size_t)((n + kScanTile - 1) / kScanTile + 2); }

void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *temp, hipStream_t st)
{
    const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    int32_t *tile = temp;
    int32_t *total = temp + ntiles + 1;
    if (ntiles > 0 && ntiles <= kScanFusedTiles) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, n, tile);
        hipLaunchKernelGGL(k_scan_down_fused, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, out, n,
                           (const int32_t *)tile);
    } else if (ntiles > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, n, tile);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanBlock), 0, st, tile, ntiles, total);
        hipLaunchKernelGGL(k_scan_down, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, out, n, tile,
                           (const int32_t *)total);
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, st, total, 0, (int64_t)1);
        hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, n, total);
    }
}

void rebuild_cells(Dev &s, SortBufs &b, hipStream_t st)
{
    const int bs = 256;
    // the histogram is zero here: cleared at creation and by k_rank_gather of the last rebuild
    hipLaunchKernelGGL(k_bin, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, b.count, b.cellof, b.rank);
    scan_exclusive(b.count, s.cell_start, 2 * s.ncell, b.scan_temp, st);
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, b.cellof, b.rank, s.cell_start,
                       b.tmp_id, b.tmp_src);
    hipLaunchKernelGGL(k_rank_gather, dim3(nblocks(s.N, bs)), dim3(bs), 0, st, s, (const int32_t *)b.cellof,
                       (const uint32_t *)b.tmp_id, (const int32_t *)b.tmp_src, b.count, b.x_alt, b.v_alt, b.id_alt,
                       b.mos_alt, b.src_of);
    double *tx = s.x, *tv = s.v;
    uint32_t *tid = s.id;
    int32_t *tm = s.mos;
    s.x = b.x_alt; b.x_alt = tx;
    s.v = b.v_alt; b.v_alt = tv;
    s.id = b.id_alt; b.id_alt = tid;
    s.mos = b.mos_alt; b.mos_alt = tm;
}

}  // namespace aimts
