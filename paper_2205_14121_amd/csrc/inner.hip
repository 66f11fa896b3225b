// Platelet ("inner") force group: harmonic bonds and angles and Morse bonds (Eq. 2,
// inter-platelet binding of Eq. 4), WCA Lennard-Jones between beads (Eq. 2) and the
// platelet-fluid force of Eq. 3 (WCA + DPD dissipative + random) between beads and
// fluid or wall particles.
//
// The work is organised around a member list rebuilt with the cell list every outer
// step: the beads, then every fluid particle within reach (cutoff + skin) of a bead.
// Each member owns a CSR list of partner slots.  Forces are gathered: a group of 16
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
// from the float4 position copy written at the rebuild.
__device__ __forceinline__ bool prefilter(const Dev &s, float4 a, float4 b, float pre2)
{
    float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z;
    if (s.per[0]) { const float h = (float)s.half[0], L = (float)s.L[0]; d0 = d0 > h ? d0 - L : (d0 < -h ? d0 + L : d0); }
    if (s.per[1]) { const float h = (float)s.half[1], L = (float)s.L[1]; d1 = d1 > h ? d1 - L : (d1 < -h ? d1 + L : d1); }
    if (s.per[2]) { const float h = (float)s.half[2], L = (float)s.L[2]; d2 = d2 > h ? d2 - L : (d2 < -h ? d2 + L : d2); }
    return d0 * d0 + d1 * d1 + d2 * d2 < pre2;
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
    int32_t b0, e0, b1, e1, incl, total;

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
        incl = (e0 - b0) + (e1 - b1);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        total = __shfl(incl, 63, 64);
    }

    // Slot of flat candidate f (0 <= f < total).
    __device__ int32_t slot(int32_t f) const
    {
        int col = 0;  // number of columns whose inclusive prefix is <= f
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (__shfl(incl, col + step - 1, 64) <= f) col += step;
        const int32_t cb0 = __shfl(b0, col, 64), ce0 = __shfl(e0, col, 64), cb1 = __shfl(b1, col, 64);
        const int32_t excl = __shfl(incl, col, 64) - (ce0 - cb0) - (__shfl(e1, col, 64) - cb1);
        const int32_t off = f - excl;
        return off < ce0 - cb0 ? cb0 + off : cb1 + (off - (ce0 - cb0));
    }
};

constexpr int kUnroll = 2;  // candidate batches of 64 whose loads are issued together
constexpr int kEll = 512;   // partners of a bead kept from the counting pass

// One wavefront per bead: the 64 lanes test 64 flat candidates at a time and rank the
// accepted ones with a ballot, so the list comes out in (set, column, slot) order
// whatever the scheduling (set: fluid and wall partners, then bead partners).  Pass 0 counts partners, keeps the first kEll of them in the bead's
// row of `ell`, and marks every fluid partner as a member.
// Pass 1 moves each row into the CSR list; only a bead with more than kEll partners
// scans again and writes its partners directly.
// A candidate is listed when its float separation lies within the float reach (the
// reach plus a margin far above float rounding): the lists are supersets of the pairs
// within reach, and both ends of a pair take the same decision (the float separation
// flips sign exactly).  The same-platelet exclusion, which decides which pairs
// interact, is exact: the float rest distance settles all but borderline cases, which
// take the float64 test.
__global__ __launch_bounds__(256) void k_bead_pairs(Dev s, int pass, uint8_t *marks, int32_t *cnt, int32_t *ell)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= s.nb) return;  // whole wavefront
    int32_t *row = ell + b * kEll;
    if (pass == 1) {
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
    const float pre2 = (float)s.pre_list2, pre_bb2 = (float)s.pre_bb2;
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
    sets[1].init(s, s.ncell, x0, x1, x2, sqrt(s.pre_bb2), lane);
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
                        take = prefilter(s, fx, q[u], pre2);
                        // fluid within reach becomes a member: mark its slot with a plain
                        // store (every writer stores the same 1); the members are compacted
                        // from the marks in slot order
                        if (take && pass == 0 && idj < (uint32_t)s.nf) marks[j[u]] = 1;
                    } else if (prefilter(s, fx, q[u], pre_bb2)) {
                        take = true;
                        if (__float_as_int(rj[u].w) == body_b) {
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

// Also closes the skin check of the outer step that just ended.  A fluid particle that
// was no member stayed farther than (cutoff + skin) from every bead at the previous
// rebuild, so no bead-fluid pair was missed while its path plus the largest member
// displacement stays within the skin; two members that were not listed as a pair were
// farther apart than (cutoff + skin), which is safe while the two largest member
// displacements add up to at most the skin; bead pairs farther than
// (cutoff + skin_bead) apart were not listed, which is safe while the two largest bead
// displacements add up to at most skin_bead.  One wavefront merges the per-block pairs
// left by the last inner step of the outer step.
__global__ __launch_bounds__(64) void k_member_count(Dev s, const int32_t *n_fluid)
{
    const int lane = threadIdx.x;
    const int64_t nw = dpart_entries(s.nb, s.cap_members);
    float a1 = 0.0f, a2 = 0.0f, b1 = 0.0f, b2 = 0.0f;  // members, beads
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
    const double m1 = fmax((double)a1, fl), m1b = fmax((double)a2, fl);
    const double m2 = fmax((double)b1, flb), m2b = fmax((double)b2, flb);
    // a failed check also keeps the largest offending sum (float bits in err[1], err[2])
    const double ms = fmax(m0 + m1, m1 + m1b), mb = m2 + m2b;
    if (s.nb > 0 && ms > s.skin) {
        atomicOr(s.err, kErrSkin);
        atomicMax(s.err + 1, __float_as_uint((float)ms));
    }
    if (s.nb > 0 && mb > s.skin_bead) {
        atomicOr(s.err, kErrSkinBead);
        atomicMax(s.err + 2, __float_as_uint((float)mb));
    }
    s.maxdisp[0] = 0u;
    const int64_t tot = s.nb + *n_fluid;
    if (tot > s.cap_members) atomicOr(s.err, kErrMemberCap);
    *s.n_members = (int32_t)(tot < s.cap_members ? tot : s.cap_members);
}

// Fluid members: their partners are the beads within reach, enumerated from the bead
// bins.  One wavefront per member, same flat candidate order and ordered compaction as
// for beads.
__device__ __forceinline__ void fluid_pairs_one(const Dev &s, int pass, int32_t *cnt, int64_t m, int lane);

// Fluid members are strided over a fixed grid (their number is known on the device
// only); pass 0 writes a zero count for every unused member slot up to the capacity.
__global__ __launch_bounds__(256) void k_fluid_pairs(Dev s, int pass, int32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t nm = *s.n_members;
    for (int64_t m = s.nb + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); m < s.cap_members; m += nw) {
        if (m >= nm) {
            if (pass != 0) return;
            if (lane == 0) cnt[m] = 0;
            continue;
        }
        fluid_pairs_one(s, pass, cnt, m, lane);
    }
}

__device__ __forceinline__ void fluid_pairs_one(const Dev &s, int pass, int32_t *cnt, int64_t m, int lane)
{
    const int64_t N = s.N;
    const int32_t t = s.member_slot[m];
    const double x0 = s.x[t], x1 = s.x[N + t], x2 = s.x[2 * N + t];
    const float4 fx = s.xf[t];
    const float pre2 = (float)s.pre_list2;
    Candidates cand;
    cand.init(s, s.ncell, x0, x1, x2, sqrt(s.pre_list2), lane);  // the bead bins
    int32_t c = 0;
    const int32_t base = pass ? s.pair_off[m] : 0;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int32_t f0 = 0; f0 < cand.total; f0 += 64 * kUnroll) {
        int32_t j[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int32_t f = f0 + 64 * u + lane;
            ok[u] = f < cand.total;
            j[u] = cand.slot(ok[u] ? f : cand.total - 1);
        }
        float4 q[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) q[u] = s.xf[j[u]];
        bool take[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            take[u] = false;
            take[u] = ok[u] && __float_as_uint(q[u].w) >= (uint32_t)s.b0 && prefilter(s, fx, q[u], pre2);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t mask = __ballot(take[u]);
            if (pass == 1 && take[u]) {
                const int64_t p = (int64_t)base + c + __popcll(mask & below);
                if (p < s.cap_pairs) s.pair_list[p] = j[u];
            }
            c += __popcll(mask);
        }
    }
    if (pass == 0 && lane == 0) cnt[m] = c;
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
#pragma unroll
    for (int k = 0; k < 3; ++k) s.fi[k * s.cap_members + m] = om >= 0 ? fi_old[k * cap_old + om] : 0.0;
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

// Fixed butterfly over the G lanes of a group (G a power of two dividing 64): every lane
// ends with the same sum.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G)
{
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kBeadLanes = 16;   // lanes per bead: bonded terms plus ~20-50 pairs
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
template <typename R, int MODE>
__device__ __forceinline__ float member_force(const Dev &s, const InnerIO &io, int64_t m, int g, int G, uint64_t count,
                                              double inv_sqrt_dt, double h, double dt)
{
    const int64_t N = s.N, C = s.cap_members;
    const double *X = io.xr, *V = io.vr;
    const bool i_bead = m < s.nb;
    const int32_t b = (int32_t)m;
    // The bounds of every term list of this lane, then the first entry of each, are
    // loaded together: the lists are short (a bead has 5-6 bonds, ~18 angle entries and
    // a few dozen pairs over 16 lanes), so a member's time is set by its chain of
    // dependent loads rather than by arithmetic.  Each loop fetches its next entry
    // before it uses the current one.
    const int32_t t = s.member_slot[m];
    int32_t bq = 0, bqe = 0, mq = 0, mqe = 0, aq = 0, aqe = 0;
    if (i_bead) {
        bq = s.bond_off[b] + g;
        bqe = s.bond_off[b + 1];
        mq = s.mor_off[b] + g;
        mqe = s.mor_off[b + 1];
        aq = s.ang_off[b] + g;
        aqe = s.ang_off[b + 1];
    }
    const int64_t pq = s.pair_off[m] + g, pe0 = s.pair_off[m + 1];
    // an overflowed list (flagged at rebuild) is truncated at the capacity
    const int64_t pend = pe0 < s.cap_pairs ? pe0 : s.cap_pairs;
    // a bead's list holds its fluid and wall partners first, then its bead partners, which
    // need neither velocity nor id (WCA only)
    const int64_t pvel = i_bead ? s.pair_off[m] + s.pair_nfl[b] : pend;
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
    for (; mq < mqe; mq += G) {
        const int32_t j = mj;
        if (mq + G < mqe) mj = s.mor_slot[mq + G];
        double y0, y1, y2;
        load_pos(X, N, j, y0, y1, y2);
        const double d0 = min_image(s, 0, x0 - y0), d1 = min_image(s, 1, x1 - y1), d2 = min_image(s, 2, x2 - y2);
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double ex = exp(-s.ma * (r - s.mr0));
        const double fs = 2.0 * s.ma * s.mD * (ex * ex - ex) / r;  // -dU/dr / r
        f0 += fs * d0;
        f1 += fs * d1;
        f2 += fs * d2;
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
    const R lj_rc2 = (R)s.lj_rc2, sig2 = (R)s.lj_sig2, eps = (R)s.lj_eps;
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
        R fs = R(0);
        if (r2 < lj_rc2) fs = lj_scalar<R>(r2, sig2, eps);
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
        p0 += fs * d0;
        p1 += fs * d1;
        p2 += fs * d2;
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

// Inner forces (and integration, per MODE).  The first nbb blocks take the beads, 16
// lanes each (256 / 16 beads per block); the remaining blocks take the fluid members, a
// whole wavefront each, striding over the members the last rebuild found (their number
// stays on the device).  Except inside the loop, each block also leaves the two
// largest displacements of its members and of its beads in dpart, one entry per block,
// for the skin check of the next rebuild (every thread reaches that reduction).
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_inner(Dev s, InnerIO io, uint64_t count, double inv_sqrt_dt, double h,
                                               double dt, unsigned nbb)
{
    float a1 = 0.0f, a2 = 0.0f, b1 = 0.0f, b2 = 0.0f;  // members, beads
    if (blockIdx.x < nbb) {
        const int g = threadIdx.x & (kBeadLanes - 1);
        const int64_t m = (int64_t)blockIdx.x * (256 / kBeadLanes) + (threadIdx.x / kBeadLanes);
        if (m < s.nb) {  // whole group
            a1 = member_force<R, MODE>(s, io, m, g, kBeadLanes, count, inv_sqrt_dt, h, dt);
            b1 = a1;
        }
    } else {
        const int g = threadIdx.x & (kFluidLanes - 1);
        const int64_t w0 = (int64_t)(blockIdx.x - nbb) * (256 / kFluidLanes) + (threadIdx.x / kFluidLanes);
        const int64_t nw = (int64_t)(gridDim.x - nbb) * (256 / kFluidLanes);
        const int64_t nm = *s.n_members;
        for (int64_t m = s.nb + w0; m < nm; m += nw)
            top2_merge(a1, a2, member_force<R, MODE>(s, io, m, g, kFluidLanes, count, inv_sqrt_dt, h, dt), 0.0f);
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
void launch_inner(const Dev &s, const InnerIO &io, uint64_t count, double dt_inner, double h, hipStream_t st)
{
    const double isdt = 1.0 / sqrt(dt_inner);
    const unsigned nbb = (unsigned)inner_bead_blocks(s.nb);
    const unsigned grid = (unsigned)inner_blocks(s.nb, s.cap_members);
    const int64_t nang = s.n_ang_ent / 3;
    if (s.angle_sep && nang > 0) hipLaunchKernelGGL(k_angles, dim3(nblocks(nang, 256)), dim3(256), 0, st, s, io.xr);
    if (s.fp32)
        hipLaunchKernelGGL((k_inner<float, MODE>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h, dt_inner, nbb);
    else
        hipLaunchKernelGGL((k_inner<double, MODE>), dim3(grid), dim3(256), 0, st, s, io, count, isdt, h, dt_inner, nbb);
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
            hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, 4)), dim3(bs), 0, st, s, 0, b.marks, b.cnt, b.ell);
        return;
    }
    if (s.nb > 0) {
        hipLaunchKernelGGL(k_mark_counts, dim3(nblocks(nwords, bs)), dim3(bs), 0, st, nwords, (const uint8_t *)b.marks,
                           b.wcount);
        scan_exclusive(b.wcount, b.wcount, nwords, b.scan_temp, st);
        hipLaunchKernelGGL(k_mark_compact, dim3(nblocks(nwords, bs)), dim3(bs), 0, st, s, nwords, b.marks,
                           (const int32_t *)b.wcount);
        hipLaunchKernelGGL(k_member_count, dim3(1), dim3(64), 0, st, s, (const int32_t *)(b.wcount + nwords));
    } else {
        hipLaunchKernelGGL(k_member_count, dim3(1), dim3(64), 0, st, s, (const int32_t *)b.zero);
    }
    const unsigned fgrid = (unsigned)std::min<int64_t>(nblocks(capS, 4), 2 * inner_fluid_blocks(s.nb));
    if (capS > 0) hipLaunchKernelGGL(k_fluid_pairs, dim3(fgrid), dim3(bs), 0, st, s, 0, b.cnt);
    scan_exclusive(b.cnt, s.pair_off, s.cap_members, b.scan_temp, st);
    if (s.nb > 0)
        hipLaunchKernelGGL(k_bead_pairs, dim3(nblocks(s.nb, 4)), dim3(bs), 0, st, s, 1, b.marks, b.cnt, b.ell);
    if (capS > 0) hipLaunchKernelGGL(k_fluid_pairs, dim3(fgrid), dim3(bs), 0, st, s, 1, b.cnt);
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
    launch_inner<kForceOnly>(s, InnerIO{s.x, s.v, nullptr, nullptr}, count, dt_inner, 0.0, st);
}

void inner_step(const Dev &s, const double *xr, const double *vr, double *xw, double *vw, uint64_t count,
                double dt_inner, bool last, hipStream_t st)
{
    if (s.cap_members == 0) return;
    const InnerIO io{xr, vr, xw, vw};
    if (last) launch_inner<kLastKick>(s, io, count, dt_inner, 0.5 * dt_inner, st);
    else launch_inner<kKickDrift>(s, io, count, dt_inner, 0.5 * dt_inner, st);
}

}  // namespace aimts
