// Platelet ("inner") force group: harmonic bonds and angles and Morse bonds (Eq. 2,
// inter-platelet binding of Eq. 4), WCA Lennard-Jones between beads (Eq. 2) and the
// platelet-fluid force of Eq. 3 (WCA + DPD dissipative + random) between beads and
// fluid or wall particles.
//
// The work is organised around a member list rebuilt with the cell list every outer
// step: the beads, then every fluid particle within reach (cutoff + skin) of a bead.
// Each member owns a CSR list of partner slots (a fluid member's list is the transpose of
// the beads' lists, sorted by slot).  Forces are gathered: a group of 16
// lanes per member sums the terms acting on it (fixed lane assignment and reduction
// tree), so every pair is evaluated from both ends and no atomics are needed; both ends
// compute bit-identical magnitudes (the separation flips sign exactly and the random
// number is keyed symmetrically), so Newton's third law holds and the result does not
// depend on scheduling.
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

// Float pre-filter of a candidate against the list reach (enlarged by the float margin),
// from the float4 position copy written at the rebuild.  The minimum image is taken only
// along the axes flagged (wave-uniform flags, see needs_image: along the others the
// separation needs none and the arithmetic is skipped).
__device__ __forceinline__ bool prefilter(const Dev &s, float4 a, float4 b, float pre2, bool w0, bool w1, bool w2)
{
    float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z;
    if (w0) { const float h = (float)s.half[0], L = (float)s.L[0]; d0 = d0 > h ? d0 - L : (d0 < -h ? d0 + L : d0); }
    if (w1) { const float h = (float)s.half[1], L = (float)s.L[1]; d1 = d1 > h ? d1 - L : (d1 < -h ? d1 + L : d1); }
    if (w2) { const float h = (float)s.half[2], L = (float)s.L[2]; d2 = d2 > h ? d2 - L : (d2 < -h ? d2 + L : d2); }
    return d0 * d0 + d1 * d1 + d2 * d2 < pre2;
}

// Whether the candidates of a member in cell c along axis k (within s.reach cells) can
// need the minimum image: on a periodic axis, unless the reach stays inside the box and
// the axis is long enough that no separation within it exceeds half the box.
__device__ __forceinline__ bool needs_image(const Dev &s, int k, int c)
{
    const int R = s.reach;
    return s.per[k] && !(s.nc[k] >= 2 * R + 3 && c - R >= 0 && c + R <= s.nc[k] - 1);
}

// Largest two of the union of two pairs (a1 >= a2, b1 >= b2).
__device__ __forceinline__ void top2_merge(float &a1, float &a2, float b1, float b2)
{
    a2 = fmaxf(fminf(a1, b1), fmaxf(a2, b2));
    a1 = fmaxf(a1, b1);
}

// The candidates of one member in one set of bins (bin0 = 0: fluid and wall particles;
// bin0 = ncell: beads) laid end to end in (column, segment, slot) order, so that a
// wavefront tests 64 of them at a time however short the single columns are.
// Lane c < (2R+1)^2 holds column (dx, dy) = (c % W - R, c / W - R): the z-neighbour
// cells of the column that can hold a particle within `cut` of the member, merged into
// at most two contiguous slot segments (two only where the range wraps around a
// periodic z boundary), and the inclusive prefix of the column lengths.  Columns and
// cells whose box lies entirely beyond `cut` are left out, so every candidate within
// `cut` is kept.  Every call below must be made by all 64 lanes.
struct Candidates {
    int32_t b0, e0, b1, e1, incl, excl, total;
    bool wide;  // more than 32 columns

    __device__ void init(const Dev &s, int64_t bin0, double x0, double x1, double x2, double cut, int lane)
    {
        const int R = s.reach, W = 2 * R + 1;
        const int cx = cell_coord(s, 0, x0), cy = cell_coord(s, 1, x1), cz = cell_coord(s, 2, x2);
        b0 = e0 = b1 = e1 = 0;
        if (lane < W * W) {
            const int dx = lane % W - R, dy = lane / W - R;
            // offset of the member inside its cell and the gap to the column's cells
            const double fx = (x0 - s.lo[0]) - cx * s.side[0], fy = (x1 - s.lo[1]) - cy * s.side[1],
                         fz = (x2 - s.lo[2]) - cz * s.side[2];
            const double gx = dx > 0 ? dx * s.side[0] - fx : (dx < 0 ? fx + (-dx - 1) * s.side[0] : 0.0);
            const double gy = dy > 0 ? dy * s.side[1] - fy : (dy < 0 ? fy + (-dy - 1) * s.side[1] : 0.0);
            const double gx2 = gx > 0.0 ? gx * gx : 0.0, gy2 = gy > 0.0 ? gy * gy : 0.0;
            const double rem = cut * cut - gx2 - gy2;
            int ix = cx + dx, iy = cy + dy;
            bool live = rem > 0.0;
            if (iy < 0 || iy >= s.nc[1]) {
                if (!s.per[1]) live = false;
                iy = (iy + s.nc[1]) % s.nc[1];
            }
            if (ix < 0 || ix >= s.nc[0]) {
                if (!s.per[0]) live = false;
                ix = (ix + s.nc[0]) % s.nc[0];
            }
            if (live) {
                const double hz = sqrt(rem);
                int zn = 0, zp = 0;  // cells taken below and above the member's
                while (zn < R && fz + zn * s.side[2] < hz) ++zn;
                while (zp < R && (zp + 1) * s.side[2] - fz < hz) ++zp;
                const int nz = s.nc[2];
                const int64_t row = bin0 + ((int64_t)iy * s.nc[0] + ix) * nz;
                int zlo = cz - zn, zhi = cz + zp;
                if (!s.per[2]) {
                    zlo = zlo < 0 ? 0 : zlo;
                    zhi = zhi >= nz ? nz - 1 : zhi;
                    b0 = s.cell_start[row + zlo];
                    e0 = s.cell_start[row + zhi + 1];
                } else if (zlo >= 0 && zhi < nz) {
                    b0 = s.cell_start[row + zlo];
                    e0 = s.cell_start[row + zhi + 1];
                } else if (zlo < 0) {  // [nz + zlo, nz) and [0, zhi]
                    b0 = s.cell_start[row + nz + zlo];
                    e0 = s.cell_start[row + nz];
                    b1 = s.cell_start[row];
                    e1 = s.cell_start[row + zhi + 1];
                } else {  // [zlo, nz) and [0, zhi - nz]
                    b0 = s.cell_start[row + zlo];
                    e0 = s.cell_start[row + nz];
                    b1 = s.cell_start[row];
                    e1 = s.cell_start[row + zhi - nz + 1];
                }
            }
        }
        excl = (e0 - b0) + (e1 - b1);
        incl = excl;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        excl = incl - excl;
        total = __shfl(incl, 63, 64);
        wide = W * W > 32;
    }

    // Slot of flat candidate f (0 <= f < total).
    __device__ int32_t slot(int32_t f) const
    {
        // number of columns whose inclusive prefix is <= f (a binary search over the
        // lanes; with at most 32 columns, lane 31 already holds the total, so the first
        // step is never taken and is skipped)
        int col = 0;
        if (wide && __shfl(incl, 31, 64) <= f) col = 32;
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
            if (__shfl(incl, col + step - 1, 64) <= f) col += step;
        // every shuffle runs with all lanes active (a shuffle inside one arm of a select
        // could read a lane that is not active there)
        const int32_t off = f - __shfl(excl, col, 64), n0 = __shfl(e0 - b0, col, 64);
        const int32_t cb0 = __shfl(b0, col, 64), cb1 = __shfl(b1, col, 64);
        return off < n0 ? cb0 + off : cb1 + (off - n0);
    }
};

constexpr int kUnroll = 2;  // candidate batches of 64 whose loads are issued together
constexpr int kEll = 512;   // partners of a bead kept from the counting pass

// One wavefront per bead: the 64 lanes test 64 flat candidates at a time and rank the
// accepted ones with a ballot, so the list comes out in (set, column, slot) order
// whatever the scheduling (set: fluid and wall partners, then bead partners).  Pass 0
// counts partners, keeps the first kEll of them in the bead's row of `ell`, and marks
// every fluid partner as a member.  The list pass (k_bead_copy) moves the rows into the
// CSR list; pass 1 takes the beads it queued, those with more than kEll partners, which
// scan again and write their partners directly (wavefront w: bead queue[1 + w], for w
// below queue[0]).
// A candidate is listed when its float separation lies within the float reach (the
// reach plus a margin far above float rounding): the lists are supersets of the pairs
// within reach, and both ends of a pair take the same decision (the float separation
// flips sign exactly).  The same-platelet exclusion, which decides which pairs
// interact, is exact: the float rest distance settles all but borderline cases, which
// take the float64 test.
// Eight wavefronts per SIMD (64 VGPRs, a few bytes spilled): the pass waits on candidate
// loads, and the extra wavefronts hide more of that latency than the spill costs.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_bead_pairs(Dev s, int pass,
                                                                                          uint8_t *marks, int32_t *cnt,
                                                                                          int32_t *ell,
                                                                                          const int32_t *queue)
{
    const int lane = threadIdx.x & 63;
    int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pass == 1) {
        if (b >= queue[0]) return;  // whole wavefront
        b = queue[1 + b];
    }
    if (b >= s.nb) return;  // whole wavefront
    int32_t *row = ell + b * kEll;
    if (pass == 1) {
        // the queue holds only beads whose lists outgrew their rows; a row that fits
        // would only be copied (the list pass does that, with the members' counts)
        const int32_t beg = s.pair_off[b], n = s.pair_off[b + 1] - beg;
        if (n <= kEll) {
            for (int32_t q = lane; q < n; q += 64)
                if ((int64_t)beg + q < s.cap_pairs) s.pair_list[beg + q] = row[q];
            return;
        }
    }
    const int64_t N = s.N;
    const int32_t t = s.bead_slot[b];
    const double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
    const float4 fx = s.xf[t];
    const float pre2 = (float)s.pre_list2, pre_bb2 = (float)s.pre_bb2, pre_bbo2 = (float)s.pre_bbo2;
    int32_t c = 0;
    const int32_t base = pass ? s.pair_off[b] : 0;
    const uint64_t below = (1ull << lane) - 1ull;
    const float4 rb = s.rest_f[b];
    const int32_t body_b = __float_as_int(rb.w);
    const float excl_lo = (float)(s.r_excl2 * (1.0 - 1e-5)), excl_hi = (float)(s.r_excl2 * (1.0 + 1e-5));
    // the fluid and wall candidates at the list reach, then the bead candidates (the bead
    // bins) at their own, shorter reach; both sets are laid out first, so that their
    // cell-range loads overlap
    Candidates sets[2];
    sets[0].init(s, 0, x0, x1, x2, sqrt(s.pre_list2), lane);
    sets[1].init(s, s.ncell, x0, x1, x2, sqrt(s.pre_bbo2), lane);
    // away from the periodic faces no candidate needs the minimum image (the separations
    // are the same, the arithmetic is skipped)
    const bool w0 = needs_image(s, 0, cell_coord(s, 0, x0)), w1 = needs_image(s, 1, cell_coord(s, 1, x1)),
               w2 = needs_image(s, 2, cell_coord(s, 2, x2));
    for (int set = 0; set < 2; ++set) {
        const Candidates &cand = sets[set];
        if (set == 1 && pass == 0 && lane == 0) s.pair_nfl[b] = c;  // the fluid and wall partners
        for (int32_t f0 = 0; f0 < cand.total; f0 += 64 * kUnroll) {
            int32_t j[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t f = f0 + 64 * u + lane;
                ok[u] = f < cand.total;
                j[u] = cand.slot(ok[u] ? f : cand.total - 1);
            }
            float4 q[kUnroll], rj[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                q[u] = s.xf[j[u]];
                rj[u] = set ? s.rest_slot[j[u]] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                bool take = false;
                if (ok[u] && j[u] != t) {
                    const uint32_t idj = __float_as_uint(q[u].w);
                    if (set == 0) {
                        take = prefilter(s, fx, q[u], pre2, w0, w1, w2);
                        // fluid within reach becomes a member: mark its slot with a plain
                        // store (every writer stores the same 1); the members are compacted
                        // from the marks in slot order
                        if (take && pass == 0 && idj < (uint32_t)s.nf) marks[j[u]] = 1;
                    } else {
                        // beads of the same platelet to the WCA reach, beads of other
                        // platelets to the (longer) reach of the aggregation term
                        const bool same = __float_as_int(rj[u].w) == body_b;
                        take = prefilter(s, fx, q[u], same ? pre_bb2 : pre_bbo2, w0, w1, w2);
                        if (take && same) {
                            const float e0 = rb.x - rj[u].x, e1 = rb.y - rj[u].y, e2 = rb.z - rj[u].z;
                            const float rr = e0 * e0 + e1 * e1 + e2 * e2;
                            take = rr >= excl_hi ||
                                   (rr >= excl_lo && bead_pair_allowed(s, (int32_t)b, (int32_t)(idj - s.b0)));
                        }
                    }
                }
                const uint64_t mask = __ballot(take);
                if (take) {
                    const int32_t q = c + __popcll(mask & below);
                    if (pass == 0) {
                        if (q < kEll) row[q] = j[u];
                    } else {
                        const int64_t p = (int64_t)base + q;
                        if (p < s.cap_pairs) s.pair_list[p] = j[u];
                    }
                }
                c += __popcll(mask);
            }
        }
    }
    if (pass == 0 && lane == 0) cnt[b] = c;
}

// The list pass: kCopyLanes lanes per bead move its row of `ell` into the CSR list and
// count, for each fluid member among its fluid and wall partners, one partner of that
// member (the fluid members' lists are the transpose of the beads').  A bead with more
// than kEll partners goes to `queue` (queue[0] of them, from queue[1] on) for pass 1.
constexpr int kCopyLanes = 16;

__global__ __launch_bounds__(256) void k_bead_copy(Dev s, const int32_t *ell, int32_t *cnt, int32_t *queue)
{
    const int g = threadIdx.x & (kCopyLanes - 1);
    const int64_t b = (int64_t)blockIdx.x * (256 / kCopyLanes) + threadIdx.x / kCopyLanes;
    if (b >= s.nb) return;
    const int32_t beg = s.pair_off[b], n = s.pair_off[b + 1] - beg;
    if (n > kEll) {
        if (g == 0) queue[1 + atomicAdd(&queue[0], 1)] = (int32_t)b;
        return;
    }
    const int32_t nfl = s.pair_nfl[b];
    const int32_t *row = ell + b * kEll;
    for (int32_t q = g; q < n && (int64_t)beg + q < s.cap_pairs; q += kCopyLanes) {
        const int32_t j = row[q];
        s.pair_list[beg + q] = j;
        if (q < nfl) {
            const int32_t m = s.mos[j];
            if (m >= 0) atomicAdd(&cnt[m], 1);  // walls are no members
        }
    }
}

// Fluid members from the marks: one thread per 32 slots writes the member slots of its
// marked slots (offsets from an exclusive scan of the per-thread counts), in slot order,
// and clears the marks for the next rebuild.
__global__ void k_mark_counts(int64_t nwords, const uint8_t *marks, int32_t *wcount)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const uint4 *m = (const uint4 *)(marks + w * 32);
    const uint4 a = m[0], b = m[1];
    // each mark byte is 0 or 1
    const uint32_t words[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) c += __popc(words[q]);
    wcount[w] = c;
}

__global__ void k_mark_compact(Dev s, int64_t nwords, uint8_t *marks, const int32_t *wscan)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint4 *m = (uint4 *)(marks + w * 32);
    const uint4 a = m[0], b = m[1];
    const uint32_t words[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    int64_t q = s.nb + wscan[w];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint32_t v = words[k];
        any = any || v != 0u;
        while (v) {
            const int bit = __ffs(v) - 1;  // lowest marked byte of this word
            v &= ~(0xFFu << (bit & ~7));
            const int32_t t = (int32_t)(w * 32 + k * 4 + (bit >> 3));
            if (q < s.cap_members) {
                s.member_slot[q] = t;
                s.mos[t] = (int32_t)q;
            }
            ++q;
        }
    }
    if (any) {
        m[0] = make_uint4(0u, 0u, 0u, 0u);
        m[1] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// Also closes the skin check of the outer step that just ended.  The interface lists
// hold every fluid and wall particle within (cutoff + skin) of each bead at the previous
// rebuild, so no bead-fluid pair was missed while the largest bead displacement plus
// the largest fluid displacement (a fluid member's, or a non-member's lazy-drift path)
// stays within the skin (walls do not move); bead pairs farther than
// (cutoff + skin_bead) apart were not listed, which is safe while the two largest bead
// displacements add up to at most skin_bead.  One wavefront merges the per-block pairs
// left by the last inner step of the outer step (fluid members in the first pair,
// beads in the second).
__global__ __launch_bounds__(64) void k_member_count(Dev s, const int32_t *n_fluid)
{
    const int lane = threadIdx.x;
    const int64_t nw = dpart_entries(s.nb, s.cap_members);
    float a1 = 0.0f, a2 = 0.0f, b1 = 0.0f, b2 = 0.0f;  // fluid members, beads
    for (int64_t w0 = 0; w0 < nw; w0 += 4 * 64) {  // four loads in flight per lane
        float4 p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t w = w0 + u * 64 + lane;
            p[u] = w < nw ? s.dpart[w] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            top2_merge(a1, a2, p[u].x, p[u].y);
            top2_merge(b1, b2, p[u].z, p[u].w);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float c1 = __shfl_xor(a1, o, 64), c2 = __shfl_xor(a2, o, 64);
        const float e1 = __shfl_xor(b1, o, 64), e2 = __shfl_xor(b2, o, 64);
        top2_merge(a1, a2, c1, c2);
        top2_merge(b1, b2, e1, e2);
    }
    if (lane != 0) return;
    const double fl = s.disp_floor, flb = s.disp_floor_bead;
    const double m0 = fmax((double)__uint_as_float(s.maxdisp[0]), fl);
    const double m1 = fmax((double)a1, fl);
    const double m2 = fmax((double)b1, flb), m2b = fmax((double)b2, flb);
    // a failed check also keeps the largest offending sum (float bits in err[1], err[2]):
    // the interface lists pair beads with fluid and wall particles, so the largest bead
    // displacement plus the largest fluid one (member or not) bounds every listed pair
    const double ms = fmax(m2, fl) + fmax(m0, m1), mb = m2 + m2b;
    if (s.nb > 0 && ms > s.skin) {
        atomicOr(s.err, kErrSkin);
        atomicMax(s.err + 1, __float_as_uint((float)ms));
    }
    // the two largest bead displacements bound every bead pair; only when that bound
    // exceeds the bead skin does the exact stage (k_bead_skin_exact) look at which
    // pairs can interact at all
    s.maxdisp[1] = (s.nb > 0 && mb > s.skin_bead) ? 1u : 0u;
    s.maxdisp[0] = 0u;
    const int64_t tot = s.nb + *n_fluid;
    if (tot > s.cap_members) atomicOr(s.err, kErrMemberCap);
    *s.n_members = (int32_t)(tot < s.cap_members ? tot : s.cap_members);
}

// Exact stage of the bead skin check.  A bead pair missing from the lists was farther
// apart than (cutoff + skin_bead) at the rebuild, so it can have come within the cutoff
// during the outer step only if the two beads' displacements add up to more than
// skin_bead -- and only pairs that can interact at all matter: beads of different
// platelets, or of one platelet with rest distance >= r_excl.  The two largest bead
// displacements bound every pair; when that bound fails, the bound is taken over the
// pairs that can interact: for every bead c of platelet p that could be part of a
// failing pair, d_c + max(largest displacement in the other platelets, largest
// displacement of a bead of p at rest distance >= r_excl from c).  The two beads of a
// nearly collapsed surface triangle, the usual pair of fastest beads, cannot interact
// (their rest distance is far below r_excl), so this bound is far tighter and still
// guarantees that no pair within the cutoff was missed.  Displacements below the
// tracking floor count as the floor.  Rest distances are compared in float with a margin
// of 1e-5 that counts borderline pairs as interacting.  A platelet with more candidate
// beads than the stage examines keeps the bound of its two largest displacements.
constexpr int kSkinCand = 256;

__device__ __forceinline__ float block_max256(float v, float *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_plt_dmax(Dev s)
{
    __shared__ float red[4];
    const int64_t p = blockIdx.x;
    const int32_t beg = s.plt_off[p], end = s.plt_off[p + 1];
    float m = (float)s.disp_floor_bead;
    for (int32_t b = beg + (int32_t)threadIdx.x; b < end; b += 256) m = fmaxf(m, s.dmax[b]);
    m = block_max256(m, red);
    if (threadIdx.x == 0) s.plt_dmax[p] = m;
}

__global__ __launch_bounds__(256) void k_bead_skin_exact(Dev s)
{
    __shared__ float red[4];
    __shared__ int32_t cand[kSkinCand];
    __shared__ int ncand;
    if (s.maxdisp[1] == 0u) return;  // the two-largest bound already holds
    const int64_t p = blockIdx.x;
    const int32_t beg = s.plt_off[p], end = s.plt_off[p + 1];
    const float fl = (float)s.disp_floor_bead, sk = (float)s.skin_bead;
    float g = 0.0f;  // largest displacement in the other platelets
    for (int64_t q = threadIdx.x; q < s.P; q += 256)
        if (q != p) g = fmaxf(g, s.plt_dmax[q]);
    g = block_max256(g, red);
    const float d1 = s.plt_dmax[p];
    if (threadIdx.x == 0) ncand = 0;
    __syncthreads();
    // beads that could be part of a pair over the skin
    float d2 = 0.0f;  // second largest of the platelet, for the fallback bound
    float top = 0.0f;
    for (int32_t b = beg + (int32_t)threadIdx.x; b < end; b += 256) {
        const float d = fmaxf(s.dmax[b], fl);
        if (d > top) { d2 = top; top = d; } else if (d > d2) { d2 = d; }
        if (d + fmaxf(g, d1) > sk) {
            const int q = atomicAdd(&ncand, 1);
            if (q < kSkinCand) cand[q] = b;
        }
    }
    __syncthreads();
    const int nc = ncand;
    float worst = 0.0f;
    if (nc > kSkinCand) {
        // too many to examine: the bound of the platelet's two largest displacements and
        // of its largest with the other platelets'
        float t1 = top, t2 = d2;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float c1 = __shfl_xor(t1, o, 64), c2 = __shfl_xor(t2, o, 64);
            top2_merge(t1, t2, c1, c2);
        }
        __syncthreads();
        __shared__ float2 tp[4];
        if ((threadIdx.x & 63) == 0) tp[threadIdx.x >> 6] = make_float2(t1, t2);
        __syncthreads();
        for (int w = 0; w < 4; ++w)
            if (w != (int)(threadIdx.x >> 6)) top2_merge(t1, t2, tp[w].x, tp[w].y);
        worst = fmaxf(t1 + t2, t1 + g);
    } else {
        const float ex2 = (float)(s.r_excl2 * (1.0 - 1e-5));
        for (int q = 0; q < nc; ++q) {
            const int32_t c = cand[q];
            const float4 rc = s.rest_f[c];
            float far = 0.0f;
            for (int32_t b = beg + (int32_t)threadIdx.x; b < end; b += 256) {
                if (b == c) continue;
                const float4 rb = s.rest_f[b];
                const float e0 = rc.x - rb.x, e1 = rc.y - rb.y, e2 = rc.z - rb.z;
                if (e0 * e0 + e1 * e1 + e2 * e2 >= ex2) far = fmaxf(far, fmaxf(s.dmax[b], fl));
            }
            far = block_max256(far, red);
            worst = fmaxf(worst, fmaxf(s.dmax[c], fl) + fmaxf(g, far));
        }
    }
    if (threadIdx.x == 0 && worst > sk) {
        atomicOr(s.err, kErrSkinBead);
        atomicMax(s.err + 2, __float_as_uint(worst));
    }
}

// Fluid members' lists as the transpose of the beads' lists.  The fluid part of a bead's
// list holds every fluid particle within the list reach (a float test that both ends of
// a pair take alike), so the beads within reach of a fluid member are exactly the beads
// whose lists hold it.  The list pass has counted them for the beads whose rows it
// copied; this pass counts them for the beads that pass 1 scanned again (one wavefront
// per queued bead, striding over the queue).
__global__ __launch_bounds__(256) void k_queue_count(Dev s, const int32_t *queue, int32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nq = queue[0];
    for (int64_t q = w; q < nq; q += (int64_t)gridDim.x * 4) {
        const int64_t b = queue[1 + q];
        const int64_t beg = s.pair_off[b];
        int64_t end = beg + s.pair_nfl[b];
        if (end > s.cap_pairs) end = s.cap_pairs;  // an overflowed list is flagged at the rebuild
        for (int64_t e = beg + lane; e < end; e += 64) {
            const int32_t m = s.mos[s.pair_list[e]];
            if (m >= 0) atomicAdd(&cnt[m], 1);  // walls are no members
        }
    }
}

// Filling pass: each bead's slot goes to the next free entry of each fluid member's
// list (atomic cursors: the order within a list is sorted afterwards).
__global__ __launch_bounds__(256) void k_tr_fill(Dev s, int32_t *cursor)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= s.nb) return;
    const int64_t beg = s.pair_off[b];
    int64_t end = beg + s.pair_nfl[b];
    if (end > s.cap_pairs) end = s.cap_pairs;
    const int32_t tb = s.member_slot[b];
    for (int64_t e = beg + lane; e < end; e += 64) {
        const int32_t m = s.mos[s.pair_list[e]];
        if (m < 0) continue;
        const int64_t q = (int64_t)s.pair_off[m] + atomicAdd(&cursor[m], 1);
        if (q < s.cap_pairs) s.pair_list[q] = tb;
    }
}

// Sorting pass: every fluid member's list into ascending slot order, so that the inner
// force sums its pairs in an order that does not depend on scheduling.  The slots of one
// list are distinct.  Both kernels use a bitonic network over the list padded with the
// largest value to a power of two n2 (the padding stays at the end).
//
// Lists up to kSortReg entries: one wavefront per member holding the list in registers,
// lane l entries l E .. l E + E - 1 (E = n2 / 64, at least 1): stages whose partner lies
// in another lane exchange through cross-lane shuffles, the others stay in the lane.  No
// LDS and no barriers, so many wavefronts stay resident.
constexpr int kSortReg = 1024;

template <int E>
__device__ __forceinline__ void sort_list_regs(int32_t *g, int len, int n2, int lane)
{
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        v[e] = i < len ? g[i] : INT32_MAX;
    }
    // element i = lane E + e meets i ^ j at stage (k, j); it keeps the smaller value when
    // i lies in an ascending run ((i & k) == 0) and is the lower of the two ((i & j) == 0),
    // or in a descending run and is the upper one
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j >= E; j >>= 1) {  // partner in lane ^ (j / E), same e
            const int lj = j / E;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int32_t o = __shfl_xor(v[e], lj, 64);
                const int i = lane * E + e;
                const bool keep_min = ((i & k) == 0) == ((lane & lj) == 0);
                v[e] = keep_min ? min(v[e], o) : max(v[e], o);
            }
        }
#pragma unroll
        for (int j = E >> 1; j > 0; j >>= 1) {  // partner in the same lane: e ^ j
            if (j < k) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & j) continue;
                    const int i = lane * E + e;
                    const int32_t a = v[e], c = v[e + j];
                    const bool asc = (i & k) == 0;
                    v[e] = asc ? min(a, c) : max(a, c);
                    v[e + j] = asc ? max(a, c) : min(a, c);
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        if (i < len) g[i] = v[e];
    }
}

__global__ __launch_bounds__(64) void k_tr_sort_short(Dev s)
{
    const int lane = threadIdx.x;
    const int64_t nm = *s.n_members;
    for (int64_t m = s.nb + blockIdx.x; m < nm; m += gridDim.x) {
        const int64_t beg = s.pair_off[m];
        int64_t end = s.pair_off[m + 1];
        if (end > s.cap_pairs) end = s.cap_pairs;
        const int64_t len = end - beg;
        if (len < 2 || len > kSortReg) continue;  // whole wavefront
        int32_t *g = s.pair_list + beg;
        int n2 = 2;
        while (n2 < len) n2 <<= 1;
        if (n2 <= 64) sort_list_regs<1>(g, (int)len, n2, lane);
        else if (n2 <= 128) sort_list_regs<2>(g, (int)len, n2, lane);
        else if (n2 <= 256) sort_list_regs<4>(g, (int)len, n2, lane);
        else if (n2 <= 512) sort_list_regs<8>(g, (int)len, n2, lane);
        else sort_list_regs<16>(g, (int)len, n2, lane);
    }
}

// Longer lists: one block per member, every compare-exchange putting the smaller value
// at the lower index (the first step of each merge compares mirrored positions); lists
// up to kSortLds entries are sorted in LDS, longer ones in place in global memory with
// the exchanges beyond the list skipped.
constexpr int kSortBS = 256;
constexpr int kSortLds = 4096;

template <typename Get, typename Put>
__device__ __forceinline__ void bitonic_ascending(int n2, int len, int tid, Get get, Put put)
{
    auto cx = [&](int lo, int hi) {
        if (hi >= len) return;
        const int32_t a = get(lo), c = get(hi);
        if (a > c) {
            put(lo, c);
            put(hi, a);
        }
    };
    for (int k = 2; k <= n2; k <<= 1) {
        const int hk = k >> 1;
        for (int i = tid; i < (n2 >> 1); i += kSortBS) {
            const int blk = i / hk, off = i % hk;
            cx(blk * k + off, blk * k + k - 1 - off);
        }
        __syncthreads();
        for (int j = k >> 2; j > 0; j >>= 1) {
            for (int i = tid; i < (n2 >> 1); i += kSortBS) {
                const int blk = i / j, off = i % j;
                const int lo = blk * 2 * j + off;
                cx(lo, lo + j);
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSortBS) void k_tr_sort_long(Dev s)
{
    __shared__ int32_t buf[kSortLds];
    const int tid = threadIdx.x;
    const int64_t nm = *s.n_members;
    for (int64_t m = s.nb + blockIdx.x; m < nm; m += gridDim.x) {
        const int64_t beg = s.pair_off[m];
        int64_t end = s.pair_off[m + 1];
        if (end > s.cap_pairs) end = s.cap_pairs;
        if (end - beg <= kSortReg) continue;  // whole block
        const int len = (int)(end - beg);
        int32_t *g = s.pair_list + beg;
        int n2 = 1;
        while (n2 < len) n2 <<= 1;
        if (n2 <= kSortLds) {
            for (int i = tid; i < n2; i += kSortBS) buf[i] = i < len ? g[i] : INT32_MAX;
            __syncthreads();
            bitonic_ascending(n2, n2, tid, [&](int i) { return buf[i]; }, [&](int i, int32_t v) { buf[i] = v; });
            for (int i = tid; i < len; i += kSortBS) g[i] = buf[i];
        } else {
            bitonic_ascending(n2, len, tid, [&](int i) { return g[i]; }, [&](int i, int32_t v) { g[i] = v; });
        }
        __syncthreads();
    }
}

// Reference positions for the skin check and the inner force carried over to the new
// member numbering (beads keep their index; a fluid member keeps its force if it was a
// member before the rebuild, otherwise its force was zero).
__global__ void k_member_init(Dev s, const double *fi_old, int64_t cap_old, const int32_t *mos_old,
                              const int32_t *src_of)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m == 0 && (int64_t)s.pair_off[s.cap_members] > s.cap_pairs) atomicOr(s.err, kErrPairCap);
    if (m >= *s.n_members) return;
    const int32_t t = s.member_slot[m];
#pragma unroll
    for (int k = 0; k < 3; ++k) s.xref[k * s.cap_members + m] = s.x[k * s.N + t];
    s.dmax[m] = 0.0f;
    int64_t om = m;
    if (m >= s.nb) om = mos_old[src_of[t]];
    for (int k = 0; k < 3 * s.nlev; ++k) s.fi[k * s.cap_members + m] = om >= 0 ? fi_old[k * cap_old + om] : 0.0;
}

// Bead topology resolved to the current slots (bead slots change at every rebuild),
// one thread per CSR or angle entry; bead members are the beads' slots.
__global__ void k_topo_slots(Dev s)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < s.nb) {
        const int32_t t = s.bead_slot[q];
        s.member_slot[q] = t;
        s.rest_slot[t] = s.rest_f[q];
    }
    if (q < s.n_bond_ent) s.bond_slot[q] = s.bead_slot[s.bond_other[q]];
    if (s.angle_sep && q < s.n_ang_ent) s.ang_slot[q] = s.bead_slot[s.ang_ijk[q]];
    if (q < s.n_ang_ent) {
        const int32_t e = s.ang_ent[q], a = e >> 2;
        s.ang_q4[q] = make_int4(s.bead_slot[s.ang_ijk[3 * a]], s.bead_slot[s.ang_ijk[3 * a + 1]],
                                s.bead_slot[s.ang_ijk[3 * a + 2]], e);
    }
    if (q < s.n_mor_ent) s.mor_slot[q] = s.bead_slot[s.mor_other[q]];
}


// ---------------------------------------------------------------------------
// Forces
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_pos(const double *x, int64_t N, int32_t t, double &a, double &b, double &c)
{
    a = x[t];
    b = x[N + t];
    c = x[2 * N + t];
}

// U = ka (theta - theta0)^2 about the vertex j of (i, j, k); a = x_i - x_j, c = x_k - x_j.
// F_i = p (c/(|a||c|) - cos a/|a|^2), F_k = p (a/(|a||c|) - cos c/|c|^2), F_j = -(F_i + F_k),
// p = 2 ka (theta - theta0) / sin(theta).  angle_terms gives F_i and F_k of angle `a` from
// the slots of its beads; both ways of applying them below use these same operations,
// each rounded on its own, so their forces agree bit for bit.
__device__ __forceinline__ void angle_terms(const Dev &s, const double *x, int32_t si, int32_t sj, int32_t sk,
                                            int32_t a, double (&fi)[3], double (&fk)[3])
{
    // every operation rounded on its own (no fused multiply-add), so that the result does
    // not depend on the kernel this is inlined into
#pragma clang fp contract(off)
    double pi0, pi1, pi2, pj0, pj1, pj2, pk0, pk1, pk2;
    load_pos(x, s.N, si, pi0, pi1, pi2);
    load_pos(x, s.N, sj, pj0, pj1, pj2);
    load_pos(x, s.N, sk, pk0, pk1, pk2);
    const double a0 = min_image(s, 0, pi0 - pj0), a1 = min_image(s, 1, pi1 - pj1), a2 = min_image(s, 2, pi2 - pj2);
    const double c0 = min_image(s, 0, pk0 - pj0), c1 = min_image(s, 1, pk1 - pj1), c2 = min_image(s, 2, pk2 - pj2);
    const double la = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
    const double lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    double cs = (a0 * c0 + a1 * c1 + a2 * c2) / (la * lc);
    cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
    const double th = acos(cs);
    double sn = sqrt((1.0 - cs) * (1.0 + cs));  // sin(th) for th in [0, pi]
    sn = sn < 1e-12 ? 1e-12 : sn;
    const double p = 2.0 * s.ka * (th - s.ang_th0[a]) / sn;
    const double iac = 1.0 / (la * lc), iaa = cs / (la * la), icc = cs / (lc * lc);
    fi[0] = p * (c0 * iac - a0 * iaa);
    fi[1] = p * (c1 * iac - a1 * iaa);
    fi[2] = p * (c2 * iac - a2 * iaa);
    fk[0] = p * (a0 * iac - c0 * icc);
    fk[1] = p * (a1 * iac - c1 * icc);
    fk[2] = p * (a2 * iac - c2 * icc);
}

// Adds the force of the angle of CSR entry q (slots of i, j, k; angle * 4 + role) on its
// bead of that role (0: i, 1: the vertex j, 2: k).  Each bead evaluates every angle it
// belongs to, so an angle is evaluated three times, once per bead, with the same
// operands and operations: the three forces are those of a single evaluation.
__device__ __forceinline__ void angle_on(const Dev &s, const double *x, int4 q, double &f0, double &f1, double &f2)
{
    const int role = q.w & 3;
    double fi[3], fk[3];
    angle_terms(s, x, q.x, q.y, q.z, q.w >> 2, fi, fk);
    if (role == 0) {
        f0 += fi[0];
        f1 += fi[1];
        f2 += fi[2];
    } else if (role == 2) {
        f0 += fk[0];
        f1 += fk[1];
        f2 += fk[2];
    } else {
        f0 += -(fi[0] + fk[0]);
        f1 += -(fi[1] + fk[1]);
        f2 += -(fi[2] + fk[2]);
    }
}

// The separate angle pass: one thread per angle writes its forces on i, j, k to ang_f,
// which the beads then gather.
__global__ void k_angles(Dev s, const double *x)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= s.n_ang_ent / 3) return;
    double fi[3], fk[3];
    angle_terms(s, x, s.ang_slot[3 * a], s.ang_slot[3 * a + 1], s.ang_slot[3 * a + 2], (int32_t)a, fi, fk);
    double *o = s.ang_f + 9 * a;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[k] = fi[k];
        o[3 + k] = -(fi[k] + fk[k]);
        o[6 + k] = fk[k];
    }
}

template <typename R>
__device__ __forceinline__ R lj_scalar(R r2, R sig2, R eps)
{
    const R sr2 = sig2 / r2;
    const R sr6 = sr2 * sr2 * sr2;
    return R(24) * eps * (R(2) * sr6 * sr6 - sr6) / r2;
}

// Inter-platelet aggregation of Eq. 4 at squared separation r2 (inside the cutoff):
// fs with F_i = fs (x_i - x_j), from the non-bonded Morse term, -dU/dr =
// 2 a D (e^{-2a(r-r0)} - e^{-a(r-r0)}), and the receptor force fA (1 - r/r0).
template <typename R>
__device__ __forceinline__ R agg_scalar(const Dev &s, R r2)
{
    const R r = sqrt(r2);
    const R a = (R)s.agg_a, r0 = (R)s.agg_r0;
    R ex;
    if constexpr (sizeof(R) == 8) ex = exp(-a * (r - r0));
    else ex = expf(-a * (r - r0));
    const R fm = R(2) * a * (R)s.agg_D * (ex * ex - ex);
    const R fa = (R)s.agg_fA * (R(1) - r / r0);
    return (fm + fa) / r;
}

// Fixed butterfly over the G lanes of a group (G a power of two dividing 64): every lane
// ends with the same sum.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G)
{
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kFluidLanes = 64;  // lanes per fluid member: ~100-300 beads within reach

// What the inner force kernel does after the forces: nothing (forces at the current
// state), the closing half kick of this inner step and the opening half kick and drift
// of the next (an inner step inside the loop), or the closing half kick alone (the last
// inner step of an outer step).
enum InnerMode { kForceOnly = 0, kKickDrift = 1, kLastKick = 2 };

// The members' state read by an inner step (positions and velocities of the members and
// their partners) and where the integrated state of each member goes.
struct InnerIO {
    const double *xr, *vr;
    double *xw, *vw;
};

// Inner force on member m, gathered by a group of G lanes: lane g takes every G-th
// bonded term and pair of the member, the group sums in a fixed butterfly.  Lane 0 of
// the group stores the force and integrates the member as MODE says; it returns the
// member's largest displacement since the rebuild (0 on the other lanes).
//
// Three-level mode (ML): only the groups due at this inner step are evaluated, each into
// an accumulator of its own: a bead's bonds, angles and same-platelet WCA belong to its
// platelet's sublevel (P1 or P2), its Morse bonds and WCA with other platelets to P2, its
// fluid and wall partners to the interface M; a fluid member has interface terms only.
// Lane 0 stores the due groups' forces and kicks each with its own half step: closing
// kicks P2, P1, M, then (inside the loop) opening kicks M, P1, P2, as the nested levels
// close and open.
template <typename R, int MODE, bool ML>
__device__ __forceinline__ float member_force(const Dev &s, const InnerIO &io, int64_t m, int g, int G, uint64_t count,
                                              double inv_sqrt_dt, double h, double dt, const LevelStep &ls)
{
    const int64_t N = s.N, C = s.cap_members;
    const double *X = io.xr, *V = io.vr;
    const bool i_bead = m < s.nb;
    const int32_t b = (int32_t)m;
    const int lev = (ML && i_bead) ? (int)s.blev[b] : 2;
    const bool due_m = !ML || (ls.due & kDueM);
    const bool due_own = !ML || (ls.due & (lev == 1 ? kDueP1 : kDueP2));  // a bead's own terms
    const bool due_x = !ML || (ls.due & kDueP2);                          // inter-platelet terms
    const int32_t body_i = ((ML || s.agg_on) && i_bead) ? s.body[b] : -1;
    // The bounds of every term list of this lane, then the first entry of each, are
    // loaded together: the lists are short (a bead has 5-6 bonds, ~18 angle entries and
    // a few dozen pairs over 8 or 16 lanes), so a member's time is set by its chain of
    // dependent loads rather than by arithmetic.  Each loop fetches its next entry
    // before it uses the current one.
    const int32_t t = s.member_slot[m];
    int32_t bq = 0, bqe = 0, mq = 0, mqe = 0, aq = 0, aqe = 0;
    if (i_bead) {
        if (due_own) {
            bq = s.bond_off[b] + g;
            bqe = s.bond_off[b + 1];
            aq = s.ang_off[b] + g;
            aqe = s.ang_off[b + 1];
        }
        if (due_x) {
            mq = s.mor_off[b] + g;
            mqe = s.mor_off[b + 1];
        }
    }
    const int64_t pe0 = s.pair_off[m + 1];
    // an overflowed list (flagged at rebuild) is truncated at the capacity
    const int64_t pend = pe0 < s.cap_pairs ? pe0 : s.cap_pairs;
    // a bead's list holds its fluid and wall partners first, then its bead partners, which
    // need neither velocity nor id (WCA only)
    const int64_t pvel = i_bead ? s.pair_off[m] + s.pair_nfl[b] : pend;
    // three-level mode skips the interface partners at a step where M is not due (and a
    // fluid member, which has no others, its whole list)
    const int64_t pq = (due_m ? (int64_t)s.pair_off[m] : (i_bead ? pvel : pend)) + g;
    int32_t bj = bq < bqe ? s.bond_slot[bq] : 0;
    int32_t mj = mq < mqe ? s.mor_slot[mq] : 0;
    int4 aj = aq < aqe ? s.ang_q4[aq] : make_int4(0, 0, 0, 0);
    int32_t pja = pq < pend ? s.pair_list[pq] : 0;
    int32_t pjb = pq + G < pend ? s.pair_list[pq + G] : pja;
    const uint32_t idi = s.id[t];
    double x0, x1, x2;
    load_pos(X, N, t, x0, x1, x2);
    const double v0 = V[t], v1 = V[N + t], v2 = V[2 * N + t];
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (; bq < bqe; bq += G) {
        const int32_t j = bj;
        if (bq + G < bqe) bj = s.bond_slot[bq + G];
        double y0, y1, y2;
        load_pos(X, N, j, y0, y1, y2);
        const double d0 = min_image(s, 0, x0 - y0), d1 = min_image(s, 1, x1 - y1), d2 = min_image(s, 2, x2 - y2);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double fs = -2.0 * s.kb * (r - s.bond_r0[bq]) / r;  // U = kb (r - r0)^2
        f0 += fs * d0;
        f1 += fs * d1;
        f2 += fs * d2;
    }
    double fx0 = 0.0, fx1 = 0.0, fx2 = 0.0;  // three-level mode: Morse bonds (group P2)
    for (; mq < mqe; mq += G) {
        const int32_t j = mj;
        if (mq + G < mqe) mj = s.mor_slot[mq + G];
        double y0, y1, y2;
        load_pos(X, N, j, y0, y1, y2);
        const double d0 = min_image(s, 0, x0 - y0), d1 = min_image(s, 1, x1 - y1), d2 = min_image(s, 2, x2 - y2);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double ex = exp(-s.ma * (r - s.mr0));
        const double fs = 2.0 * s.ma * s.mD * (ex * ex - ex) / r;  // -dU/dr / r
        if constexpr (ML) {
            fx0 += fs * d0;
            fx1 += fs * d1;
            fx2 += fs * d2;
        } else {
            f0 += fs * d0;
            f1 += fs * d1;
            f2 += fs * d2;
        }
    }
    for (; aq < aqe; aq += G) {
        const int4 e = aj;
        if (aq + G < aqe) aj = s.ang_q4[aq + G];
        if (s.angle_sep) {
            const double *af = s.ang_f + 9 * (e.w >> 2) + 3 * (e.w & 3);
            f0 += af[0];
            f1 += af[1];
            f2 += af[2];
        } else {
            angle_on(s, X, e, f0, f1, f2);
        }
    }
    R p0 = R(0), p1 = R(0), p2 = R(0);
    R px0 = R(0), px1 = R(0), px2 = R(0);  // three-level mode: WCA with other platelets (P2)
    R pm0 = R(0), pm1 = R(0), pm2 = R(0);  // three-level mode: interface terms (M)
    const R lj_rc2 = (R)s.lj_rc2, sig2 = (R)s.lj_sig2, eps = (R)s.lj_eps;
    const R agg_rc2 = s.agg_on ? (R)s.agg_rc2 : R(-1);  // no pair passes r2 < -1
    const R rcpf2 = (R)s.rc_pf2, inv_rcpf = (R)s.inv_rc_pf, gpf = (R)s.gpf, spf = (R)s.spf;
    const R isdt = (R)inv_sqrt_dt;
    const uint32_t k1 = s.key1 ^ 1u;
    // force of the pair (this member, slot j), from j's position, velocity and id
    auto pair = [&](int32_t j, double y0, double y1, double y2, double u0, double u1, double u2, uint32_t idj) {
        const R d0 = (R)min_image(s, 0, x0 - y0);
        const R d1 = (R)min_image(s, 1, x1 - y1);
        const R d2 = (R)min_image(s, 2, x2 - y2);
        const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const bool j_bead = idj >= (uint64_t)s.b0;
        if constexpr (ML) {
            if (i_bead && j_bead) {
                // WCA between beads: the own sublevel's group within the platelet, P2 across
                // (with the aggregation term of Eq. 4)
                const bool same = __float_as_int(((const float *)s.rest_slot)[4 * (int64_t)j + 3]) == body_i;
                if (!(same ? due_own : due_x)) return;
                const bool agg = !same && r2 < agg_rc2;
                if (!(r2 < lj_rc2) && !agg) return;
                R fs = r2 < lj_rc2 ? lj_scalar<R>(r2, sig2, eps) : R(0);
                if (agg) fs += agg_scalar<R>(s, r2);
                if (same) {
                    p0 += fs * d0;
                    p1 += fs * d1;
                    p2 += fs * d2;
                } else {
                    px0 += fs * d0;
                    px1 += fs * d1;
                    px2 += fs * d2;
                }
                return;
            }
        }
        R fs = R(0);
        if (r2 < lj_rc2) fs = lj_scalar<R>(r2, sig2, eps);
        // Eq. 4 between beads of different platelets (only while aggregation is on)
        if (i_bead && j_bead && r2 < agg_rc2 &&
            __float_as_int(((const float *)s.rest_slot)[4 * (int64_t)j + 3]) != body_i)
            fs += agg_scalar<R>(s, r2);
        if (!(i_bead && j_bead) && r2 < rcpf2) {
            const R r = sqrt(r2);
            const R w = R(1) - r * inv_rcpf;
            const R ev = (d0 * (R)(v0 - u0) + d1 * (R)(v1 - u1) + d2 * (R)(v2 - u2)) / r;
            uint32_t w0, w1;
            pair_words(idi, idj, count, s.key0, k1, w0, w1);
            R z;
            if constexpr (sizeof(R) == 8) z = gauss64(w0, w1);
            else z = gauss32(w0, w1);
            fs += (-gpf * w * w * ev + spf * w * z * isdt) / r;
        }
        if constexpr (ML) {  // a fluid or wall partner: the interface group
            pm0 += fs * d0;
            pm1 += fs * d1;
            pm2 += fs * d2;
        } else {
            p0 += fs * d0;
            p1 += fs * d1;
            p2 += fs * d2;
        }
    };
    // two partners per lane and trip, their loads issued together
    for (int64_t p = pq; p < pend; p += 2 * G) {
        const bool two = p + G < pend;
        const int32_t ja = pja, jb = pjb;
        if (p + 2 * G < pend) {
            pja = s.pair_list[p + 2 * G];
            pjb = p + 3 * G < pend ? s.pair_list[p + 3 * G] : pja;
        }
        const double ya0 = X[ja], ya1 = X[N + ja], ya2 = X[2 * N + ja];
        const double yb0 = X[jb], yb1 = X[N + jb], yb2 = X[2 * N + jb];
        const bool fa = p < pvel, fb = p + G < pvel;
        const double ua0 = fa ? V[ja] : 0.0, ua1 = fa ? V[N + ja] : 0.0, ua2 = fa ? V[2 * N + ja] : 0.0;
        const double ub0 = fb ? V[jb] : 0.0, ub1 = fb ? V[N + jb] : 0.0, ub2 = fb ? V[2 * N + jb] : 0.0;
        const uint32_t ida = fa ? s.id[ja] : (uint32_t)s.b0, idb = fb ? s.id[jb] : (uint32_t)s.b0;
        pair(ja, ya0, ya1, ya2, ua0, ua1, ua2, ida);
        if (two) pair(jb, yb0, yb1, yb2, ub0, ub1, ub2, idb);
    }
    f0 = group_sum(f0, G);
    f1 = group_sum(f1, G);
    f2 = group_sum(f2, G);
    p0 = group_sum(p0, G);
    p1 = group_sum(p1, G);
    p2 = group_sum(p2, G);
    if constexpr (ML) {
        fx0 = group_sum(fx0, G);
        fx1 = group_sum(fx1, G);
        fx2 = group_sum(fx2, G);
        px0 = group_sum(px0, G);
        px1 = group_sum(px1, G);
        px2 = group_sum(px2, G);
        pm0 = group_sum(pm0, G);
        pm1 = group_sum(pm1, G);
        pm2 = group_sum(pm2, G);
        float dm = 0.0f;
        if (g == 0) {
            // the groups: M, the platelet's own terms, and the inter-platelet terms
            const double am[3] = {(double)pm0, (double)pm1, (double)pm2};
            const double ao[3] = {f0 + (double)p0, f1 + (double)p1, f2 + (double)p2};
            const double ax[3] = {fx0 + (double)px0, fx1 + (double)px1, fx2 + (double)px2};
            double a1[3], a2[3];  // P1, P2
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a1[k] = lev == 1 ? ao[k] : 0.0;
                a2[k] = lev == 1 ? ax[k] : ao[k] + ax[k];
            }
            const bool dm_ = due_m, d1_ = (ls.due & kDueP1) != 0, d2_ = (ls.due & kDueP2) != 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (dm_) s.fi[(0 + k) * C + m] = am[k];
                if (d1_ && i_bead) s.fi[(3 + k) * C + m] = a1[k];
                if (d2_ && i_bead) s.fi[(6 + k) * C + m] = a2[k];
            }
            if constexpr (MODE != kForceOnly) {
                const double mi = s.minv[ptype(s, idi)];
                const float dm_old = s.dmax[m];
                double u0 = v0, u1 = v1, u2 = v2, y0 = x0, y1 = x1, y2 = x2;
                auto kick = [&](const double (&a)[3], double hh) {
                    u0 += hh * a[0] * mi;
                    u1 += hh * a[1] * mi;
                    u2 += hh * a[2] * mi;
                };
                // closing half kicks of the levels whose step ends here, innermost first
                if (d2_ && i_bead) kick(a2, ls.h2);
                if (d1_ && i_bead && lev == 1) kick(a1, ls.h1);
                if (dm_) kick(am, ls.hm);
                if constexpr (MODE == kKickDrift) {
                    // opening half kicks of the levels whose next step starts here, outermost first
                    if (dm_) kick(am, ls.hm);
                    if (d1_ && i_bead && lev == 1) kick(a1, ls.h1);
                    if (d2_ && i_bead) kick(a2, ls.h2);
                    drift_one(s, y0, y1, y2, u0, u1, u2, dt);
                    const double e0 = min_image(s, 0, y0 - s.xref[m]);
                    const double e1 = min_image(s, 1, y1 - s.xref[C + m]);
                    const double e2 = min_image(s, 2, y2 - s.xref[2 * C + m]);
                    const double disp = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                    if (!isfinite(disp)) {
                        atomicOr(s.err, kErrNonFinite);
                    } else {
                        const float d = (float)(disp * 1.000001);  // rounded up
                        if (d > dm_old) s.dmax[m] = d;
                    }
                } else {
                    dm = dm_old;
                }
                io.xw[t] = y0;
                io.xw[N + t] = y1;
                io.xw[2 * N + t] = y2;
                io.vw[t] = u0;
                io.vw[N + t] = u1;
                io.vw[2 * N + t] = u2;
            } else {
                dm = s.dmax[m];
            }
        }
        return dm;
    }
    float dm = 0.0f;
    if (g == 0) {
        const double a0 = f0 + (double)p0, a1 = f1 + (double)p1, a2 = f2 + (double)p2;
        s.fi[m] = a0;
        s.fi[C + m] = a1;
        s.fi[2 * C + m] = a2;
        if constexpr (MODE != kForceOnly) {
            const double mi = s.minv[ptype(s, idi)];
            const float dm_old = s.dmax[m];
            double u0 = v0, u1 = v1, u2 = v2, y0 = x0, y1 = x1, y2 = x2;
            // closing half kick of this inner step, then (inside the loop) the opening
            // half kick and drift of the next
            for (int q = 0; q < (MODE == kKickDrift ? 2 : 1); ++q) {
                u0 += h * a0 * mi;
                u1 += h * a1 * mi;
                u2 += h * a2 * mi;
            }
            if constexpr (MODE == kKickDrift) {
                drift_one(s, y0, y1, y2, u0, u1, u2, dt);
                const double e0 = min_image(s, 0, y0 - s.xref[m]);
                const double e1 = min_image(s, 1, y1 - s.xref[C + m]);
                const double e2 = min_image(s, 2, y2 - s.xref[2 * C + m]);
                const double disp = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                if (!isfinite(disp)) {
                    atomicOr(s.err, kErrNonFinite);
                } else {
                    const float d = (float)(disp * 1.000001);  // rounded up
                    if (d > dm_old) s.dmax[m] = d;
                }
            } else {
                dm = dm_old;
            }
            io.xw[t] = y0;
            io.xw[N + t] = y1;
            io.xw[2 * N + t] = y2;
            io.vw[t] = u0;
            io.vw[N + t] = u1;
            io.vw[2 * N + t] = u2;
        } else {
            dm = s.dmax[m];
        }
    }
    return dm;
}

// Inner forces (and integration, per MODE).  The first nbb blocks take the beads,
// inner_bead_lanes(nb) lanes each (16 or 32 beads per block); the remaining blocks take
// the fluid members, a whole wavefront each, striding over the members the last rebuild
// found (their number stays on the device).  Except inside the loop, each block also
// leaves the two largest displacements of its fluid members and of its beads in dpart,
// one entry per block, for the skin check of the next rebuild (every thread reaches that
// reduction).  The kernel waits on the gathers of its partners' state: in float32 mode it
// runs four wavefronts per SIMD (128 VGPRs, ~150 B spilled), which beat three (no spill)
// by 16 % on 2.56 M beads and 8 % on 10^4 beads; five were slower.
template <typename R, int MODE, bool ML>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) void k_inner(
    Dev s, InnerIO io, uint64_t count, double inv_sqrt_dt, double h, double dt, unsigned nbb, LevelStep ls)
{
    float a1 = 0.0f, a2 = 0.0f, b1 = 0.0f, b2 = 0.0f;  // fluid members, beads
    if (blockIdx.x < nbb) {
        const int G = inner_bead_lanes(s.nb);
        const int g = threadIdx.x & (G - 1);
        const int64_t m = (int64_t)blockIdx.x * (256 / G) + (threadIdx.x / G);
        if (m < s.nb) {  // whole group
            b1 = member_force<R, MODE, ML>(s, io, m, g, G, count, inv_sqrt_dt, h, dt, ls);
        }
    } else {
        const int g = threadIdx.x & (kFluidLanes - 1);
        const int64_t w0 = (int64_t)(blockIdx.x - nbb) * (256 / kFluidLanes) + (threadIdx.x / kFluidLanes);
        const int64_t nw = (int64_t)(gridDim.x - nbb) * (256 / kFluidLanes);
        const int64_t nm = *s.n_members;
        for (int64_t m = s.nb + w0; m < nm; m += nw)
            top2_merge(a1, a2, member_force<R, MODE, ML>(s, io, m, g, kFluidLanes, count, inv_sqrt_dt, h, dt, ls),
                       0.0f);
    }
    if constexpr (MODE != kKickDrift) {
        __shared__ float4 part[4];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const float c1 = __shfl_xor(a1, o, 64), c2 = __shfl_xor(a2, o, 64);
            const float e1 = __shfl_xor(b1, o, 64), e2 = __shfl_xor(b2, o, 64);
            top2_merge(a1, a2, c1, c2);
            top2_merge(b1, b2, e1, e2);
        }
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = make_float4(a1, a2, b1, b2);
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w) {
                top2_merge(a1, a2, part[w].x, part[w].y);
                top2_merge(b1, b2, part[w].z, part[w].w);
            }
            s.dpart[blockIdx.x] = make_float4(a1, a2, b1, b2);
        }
    }
}

template <int MODE>
void launch_inner(const Dev &s, const InnerIO &io, uint64_t count, double dt_inner, double dt_rand, double h,
                  const LevelStep &ls, hipStream_t st)
{
    const double isdt = 1.0 / sqrt(dt_rand);
    const unsigned nbb = (unsigned)inner_bead_blocks(s.nb);
    const unsigned grid = (unsigned)inner_blocks(s.nb, s.cap_members);
    const int64_t nang = s.n_ang_ent / 3;
    if (s.angle_sep && nang > 0) hipLaunchKernelGGL(k_angles, dim3(nblocks(nang, 256)), dim3(256), 0, st, s, io.xr);
    if (s.nlev == 3) {
        if (s.fp32)
            hipLaunchKernelGGL((k_inner<float, MODE, true>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h,
                               dt_inner, nbb, ls);
        else
            hipLaunchKernelGGL((k_inner<double, MODE, true>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h,
                               dt_inner, nbb, ls);
    } else if (s.fp32) {
        hipLaunchKernelGGL((k_inner<float, MODE, false>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h, dt_inner,
                           nbb, ls);
    } else {
        hipLaunchKernelGGL((k_inner<double, MODE, false>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h,
                           dt_inner, nbb, ls);
    }
}

}  // namespace

size_t bead_list_scratch_entries(int64_t nb) { return (size_t)nb * kEll; }

void rebuild_inner(Dev &s, InnerBufs &b, const int32_t *src_of, hipStream_t st, int part)
{
    const int bs = 256;
    const int64_t capS = s.cap_members - s.nb;
    const int64_t nwords = (s.N + 31) / 32;
    if (part == 0) {
        // beads are always the first members; the member marks are zero here (cleared at
        // creation and by the compaction of the last rebuild)
        const int64_t nent = std::max(std::max(s.nb, s.n_ang_ent), std::max(s.n_bond_ent, s.n_mor_ent));
        if (nent > 0) hipLaunchKernelGGL(k_topo_slots, dim3(nblocks(nent, bs)), dim3(bs), 0, st, s);
        if (s.nb > 0)
            hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, 4)), dim3(bs), 0, st, s, 0, b.marks, b.cnt, b.ell,
                               (const int32_t *)nullptr);
        return;
    }
    if (s.nb > 0) {
        hipLaunchKernelGGL(k_mark_counts, dim3(nblocks(nwords, bs)), dim3(bs), 0, st, nwords, (const uint8_t *)b.marks,
                           b.wcount);
        scan_exclusive(b.wcount, b.wcount, nwords, b.scan_temp, st);
        hipLaunchKernelGGL(k_mark_compact, dim3(nblocks(nwords, bs)), dim3(bs), 0, st, s, nwords, b.marks,
                           (const int32_t *)b.wcount);
        hipLaunchKernelGGL(k_member_count, dim3(1), dim3(64), 0, st, s, (const int32_t *)(b.wcount + nwords));
        // the exact stage of the bead skin check, before the rebuild clears dmax
        hipLaunchKernelGGL(k_plt_dmax, dim3((unsigned)s.P), dim3(256), 0, st, s);
        hipLaunchKernelGGL(k_bead_skin_exact, dim3((unsigned)s.P), dim3(256), 0, st, s);
    } else {
        hipLaunchKernelGGL(k_member_count, dim3(1), dim3(64), 0, st, s, (const int32_t *)b.zero);
    }
    // the beads' lists first (offsets of the beads alone) with the fluid members' counts,
    // then the fluid members' lists as their transpose: offsets of all members (the beads'
    // again, unchanged), filling and sorting
    scan_exclusive(b.cnt, s.pair_off, s.nb, b.scan_temp, st);
    if (capS > 0) fill_i32(b.cnt + s.nb, 0, capS, st);
    if (s.nb > 0) {
        fill_i32(b.queue, 0, 1, st);
        hipLaunchKernelGGL(k_bead_copy, dim3(nblocks(s.nb, bs / kCopyLanes)), dim3(bs), 0, st, s,
                           (const int32_t *)b.ell, b.cnt, b.queue);
        hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, 4)), dim3(bs), 0, st, s, 1, b.marks, b.cnt, b.ell,
                           (const int32_t *)b.queue);
        if (capS > 0)
            hipLaunchKernelGGL(k_queue_count, dim3((unsigned)std::min<int64_t>(nblocks(s.nb, 4), 2048)), dim3(bs), 0,
                               st, s, (const int32_t *)b.queue, b.cnt);
    }
    if (capS > 0) {
        scan_exclusive(b.cnt, s.pair_off, s.cap_members, b.scan_temp, st);
        fill_i32(b.cnt + s.nb, 0, capS, st);
        hipLaunchKernelGGL(k_tr_fill, dim3(nblocks(s.nb, 4)), dim3(bs), 0, st, s, b.cnt);
        const int64_t sgrid = std::min<int64_t>(capS, 8 * inner_fluid_blocks(s.nb));
        hipLaunchKernelGGL(k_tr_sort_short, dim3((unsigned)sgrid), dim3(64), 0, st, s);
        hipLaunchKernelGGL(k_tr_sort_long, dim3((unsigned)std::min<int64_t>(sgrid, 1024)), dim3(kSortBS), 0, st, s);
    }
    double *fi_old = s.fi;
    s.fi = b.fi_alt;
    b.fi_alt = fi_old;
    if (s.cap_members > 0)
        hipLaunchKernelGGL(k_member_init, dim3(nblocks(s.cap_members, bs)), dim3(bs), 0, st, s, (const double *)fi_old,
                           s.cap_members, (const int32_t *)b.mos_old, src_of);
}

void inner_forces(const Dev &s, uint64_t count, double dt_rand, hipStream_t st)
{
    if (s.cap_members == 0) return;
    const LevelStep all{kDueAll, 0.0, 0.0, 0.0};
    launch_inner<kForceOnly>(s, InnerIO{s.x, s.v, nullptr, nullptr}, count, dt_rand, dt_rand, 0.0, all, st);
}

void inner_step(const Dev &s, const double *xr, const double *vr, double *xw, double *vw, uint64_t count,
                double dt_inner, double dt_rand, bool last, const LevelStep &ls, hipStream_t st)
{
    if (s.cap_members == 0) return;
    const InnerIO io{xr, vr, xw, vw};
    if (last) launch_inner<kLastKick>(s, io, count, dt_inner, dt_rand, 0.5 * dt_inner, ls, st);
    else launch_inner<kKickDrift>(s, io, count, dt_inner, dt_rand, 0.5 * dt_inner, ls, st);
}

namespace {

__global__ void k_levels_from_ratios(Dev s, const int32_t *pratio, const int32_t *decision, int32_t k_cap)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= s.P) return;
    int32_t k = decision[0];
    if (k_cap > 0 && k > k_cap) k = k_cap;
    s.plev[p] = pratio[p] > k ? 1 : 2;
}

__global__ void k_levels_to_beads(Dev s)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < s.nb) s.blev[b] = (uint8_t)(s.plev[s.body[b]] == 1 ? 1 : 2);
}

}  // namespace

void levels_from_ratios(const Dev &s, const int32_t *pratio, const int32_t *decision, int32_t k_cap, hipStream_t st)
{
    if (s.P > 0)
        hipLaunchKernelGGL(k_levels_from_ratios, dim3(nblocks(s.P, 256)), dim3(256), 0, st, s, pratio, decision, k_cap);
    levels_to_beads(s, st);
}

void levels_to_beads(const Dev &s, hipStream_t st)
{
    if (s.nb > 0) hipLaunchKernelGGL(k_levels_to_beads, dim3(nblocks(s.nb, 256)), dim3(256), 0, st, s);
}

}  // namespace aimts
