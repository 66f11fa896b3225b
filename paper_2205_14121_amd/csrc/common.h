// Internal device-side definitions of the aimts engine (gfx950).
//
// Data layout in the device workspace (all particle arrays are structure-of-arrays
// in "slot" order, i.e. sorted by cell after every neighbour rebuild):
//   x, v     : double [3][N]   positions / velocities (component-major)
//   fo       : double or float [3][N] outer (DPD) force
//   id       : uint32 [N]      particle index of the slot (fluid < wall < bead)
//   cell_start[2 ncell + 1]: slot ranges of 2 ncell bins: bin c < ncell holds the fluid
//              and wall particles of cell c, bin ncell + c the beads of cell c; within a
//              bin the slots are ordered by particle index.  The DPD scan sees no beads,
//              and bead partners are enumerated with their own reach.
// Cells are numbered y-major, c = (iy * nx + ix) * nz + iz, so the fluid/wall slots of
// a row of cells along y are one contiguous range, and so are its bead slots (used for
// the peculiar temperature).
// The inner ("platelet") force group works on a member list: members [0, n_bead) are
// the beads in bead order, then the fluid particles within reach of a bead, in slot
// order.  Inner forces, reference positions and the pair list are indexed by member.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aimts {

enum : uint32_t {
    kErrNonFinite = 1u,    // a non-finite velocity, or a position far outside the box, appeared
    kErrSkin = 2u,         // displacements within one outer step exceeded the neighbour skin
    kErrPairCap = 4u,      // platelet pair list capacity exceeded
    kErrMemberCap = 8u,    // inner member capacity exceeded
    kErrOutside = 16u,     // a particle left the box through a non-periodic face
    kErrSkinBead = 32u,    // bead displacements within one outer step exceeded the bead skin
};

// Contact radius of the contact-count feature: walls and beads of other platelets
// closer than this to a bead count as its contacts.
constexpr double kContactRadius = 1.0;

struct Dev {
    // geometry
    double lo[3], L[3], half[3], side[3];
    int32_t nc[3];
    int32_t per[3];
    int64_t ncell;
    int32_t reach;           // cells searched each way when building the inner pair list
    int32_t nrow;            // cell rows along y
    // counts
    int64_t N, nf, nw, nb, b0, P;
    int64_t cap_members, cap_pairs;
    // parameters
    double m[3], minv[3];
    double a, gamma, sigma, rc, rc2, inv_rc;
    double lj_eps, lj_sig2, lj_rc2, r_excl2;
    double gpf, spf, rc_pf, rc_pf2, inv_rc_pf;
    double list_cut2;        // (max(rc_pf, rc_lj) + skin)^2  bead-fluid/wall reach
    double bb_cut2;          // max(rc_lj + skin_bead, kContactRadius)^2  bead-bead reach
    double kb, ka, mD, ma, mr0;
    // inter-platelet aggregation of Eq. 4 between beads of different platelets closer
    // than sqrt(agg_rc2): non-bonded Morse (agg_D, agg_a, agg_r0) plus the receptor
    // force agg_fA (1 - r / agg_r0); agg_on = 0: off
    double agg_D, agg_a, agg_r0, agg_fA, agg_rc2, agg_eshift;
    int32_t agg_on;
    double bbo_cut2;         // (max(rc_lj, agg_rc) + skin_bead)^2: reach of beads of other platelets
    double g[3];
    int32_t wall_axis;
    int32_t fp32;
    double wall_lo, wall_hi;
    double skin, skin_bead;
    double disp_floor;       // displacements below this are not tracked (treated as equal to it)
    double disp_floor_bead;  // the same for the bead-only displacement
    uint32_t key0, key1;     // Philox key words (seed low, seed high)
    // particle arrays (slot order)
    double *x, *v;
    int32_t *dpd_order;      // [dpd_blocks(N)] the DPD kernel's blocks in the order they run (dpd.hip)
    float4 *xf;              // [N] float copy of the positions at the last rebuild (w: id bits),
                             // used only to pre-filter candidates
    float4 *vf;              // [N] float copy of the velocities at the last rebuild (w: id bits),
                             // read by the float32 DPD pair phase
    double pre_rc2;          // squared pre-filter cutoff: rc plus 8 float ulps of the box extent
    double pre_list2;        // the same for the platelet pair-list reach
    double pre_bb2;          // the same for the bead-bead reach
    double pre_bbo2;         // the same for the reach of beads of other platelets
    void *fo;
    uint32_t *id;
    int32_t *cell_start;     // [2 ncell + 1]: non-bead bins, then bead bins
    int32_t *bead_slot;      // [nb] slot of each bead
    int32_t *mos;            // [N] member index of a slot, -1 if not a member
    // inner members
    int32_t *member_slot;    // [cap_members]
    int32_t *n_members;      // device scalar
    double *fi;              // [3 nlev][cap_members] inner force: nlev = 1, the whole inner
                             // force; nlev = 3 (three-level mode), the interface group M,
                             // the flowing sublevel's P1 and the aggregating sublevel's P2,
                             // in that order
    int32_t nlev;            // 1 or 3
    uint8_t *blev;           // [nb] sublevel (1 flowing, 2 aggregating) of each bead's platelet
    int32_t *plev;           // [P] sublevel of each platelet
    double *xref;            // [3][cap_members] positions at the last rebuild
    int32_t *pair_off;       // [cap_members + 1]
    int32_t *pair_nfl;       // [nb] fluid and wall partners at the head of each bead's list
    int32_t *pair_list;      // [cap_pairs] partner slots
    // platelet topology (bead indices)
    int32_t *body;           // [nb]
    double *rest;            // [3][nb]
    float4 *rest_f;          // [nb] float copy of the rest positions (w: platelet index bits)
    float4 *rest_slot;       // [N] rest_f of the bead in each bead slot (other slots stale),
                             // written with the topology slots at every rebuild
    int32_t *bond_off, *bond_other; double *bond_r0;   // CSR per bead
    int32_t *ang_off, *ang_ent;                        // CSR per bead: angle * 4 + role
    int32_t *ang_ijk; double *ang_th0;                 // [n_angle][3] bead indices
    int4 *ang_q4;                                      // [3 n_angle] per CSR entry: the slots of the
                                                       // angle's beads i, j, k and the entry (set at every rebuild)
    int32_t angle_sep;                                 // 1: angle forces in a pass of their own:
    int32_t *ang_slot;                                 //   [n_angle][3] slots (set at every rebuild),
    double *ang_f;                                     //   [n_angle][3][3] forces on i, j, k
    int32_t *mor_off, *mor_other;                      // CSR per bead
    // the same topology resolved to slots at every rebuild
    int32_t *bond_slot;      // [2 n_bond] slot of bond_other
    int32_t *mor_slot;       // [2 n_morse] slot of mor_other
    int64_t n_bond_ent, n_mor_ent, n_ang_ent;          // 2 n_bond, 2 n_morse, 3 n_angle
    int32_t *plt_off;                                  // [P + 1] bead ranges
    double *plt_area;
    uint32_t *err;           // [4] error flags; on a failed skin check [1], [2] hold the largest
                             // member and bead displacement sums (float bits)
    uint32_t *maxdisp;       // float bits: [0] largest outer-step path of a non-member;
                             // [1] 1 while the bead skin check needs its exact stage
    float *plt_dmax;         // [P] largest bead displacement of each platelet (skin check)
    float *dmax;             // [cap_members] largest displacement of each member since the rebuild
    float4 *dpart;           // [dpart_entries(nb, cap_members)] per block of the inner force kernel:
                             // the two largest dmax of its members and of its beads, left by
                             // the last inner step of an outer step
};

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplications of the even words by odd constants, the high halves xor-ed with the
// odd words and the round key; the key advances by Weyl increments between rounds.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply (v_mad_u64_u32) gives both halves of each product
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The two 32-bit words (w0, w1) that define the pair's Gaussian.
__device__ __forceinline__ void pair_words(uint32_t ida, uint32_t idb, uint64_t count, uint32_t k0, uint32_t k1,
                                           uint32_t &w0, uint32_t &w1)
{
    uint32_t c0 = ida < idb ? ida : idb;
    uint32_t c1 = ida < idb ? idb : ida;
    uint32_t c2 = (uint32_t)count;
    uint32_t c3 = (uint32_t)(count >> 32);
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    w0 = c0;
    w1 = c1;
}

// Box-Muller in float64: sqrt(-2 ln u1) cos(2 pi u2), u = (w + 1/2) 2^-32.
__device__ __forceinline__ double gauss64(uint32_t w0, uint32_t w1)
{
    const double u1 = ((double)w0 + 0.5) * 2.3283064365386963e-10;
    const double u2 = ((double)w1 + 0.5) * 2.3283064365386963e-10;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Box-Muller in float32 with the hardware transcendentals: v_log_f32 is log2 and
// v_cos_f32 takes its argument in revolutions, so cos(2 pi u2) = v_cos_f32(u2).
__device__ __forceinline__ float gauss32(uint32_t w0, uint32_t w1)
{
    const float u1 = ((float)w0 + 0.5f) * 2.3283064365386963e-10f;
    const float u2 = ((float)w1 + 0.5f) * 2.3283064365386963e-10f;
    const float l2 = __builtin_amdgcn_logf(u1);                   // log2(u1) < 0
    return __builtin_sqrtf(-1.3862943611198906f * l2) * __builtin_amdgcn_cosf(u2);  // -2 ln2 log2(u1)
}

// ----------------------------------------------------------------------------
// Geometry
// ----------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(const Dev &s, int k, double xk)
{
    int ik = (int)floor((xk - s.lo[k]) / s.side[k]);
    if (ik < 0) ik = s.per[k] ? ik + s.nc[k] : 0;
    if (ik >= s.nc[k]) ik = s.per[k] ? ik - s.nc[k] : s.nc[k] - 1;
    ik = ik < 0 ? 0 : (ik >= s.nc[k] ? s.nc[k] - 1 : ik);
    return ik;
}

__device__ __forceinline__ int64_t cell_index(const Dev &s, int ix, int iy, int iz)
{
    return ((int64_t)iy * s.nc[0] + ix) * s.nc[2] + iz;
}

__device__ __forceinline__ double min_image(const Dev &s, int k, double d)
{
    if (s.per[k]) {
        if (d > s.half[k]) d -= s.L[k];
        else if (d < -s.half[k]) d += s.L[k];
    }
    return d;
}

__device__ __forceinline__ int ptype(const Dev &s, uint32_t id)
{
    return id < (uint64_t)s.nf ? 0 : (id < (uint64_t)s.b0 ? 1 : 2);
}

// Wrap along periodic axes and reflect at the walls (position mirrored, velocity reversed).
__device__ __forceinline__ void drift_one(const Dev &s, double &x0, double &x1, double &x2, double &v0, double &v1,
                                          double &v2, double dt)
{
    x0 += dt * v0;
    x1 += dt * v1;
    x2 += dt * v2;
    if (s.wall_axis >= 0) {
        double &y = s.wall_axis == 0 ? x0 : (s.wall_axis == 1 ? x1 : x2);
        if (y < s.wall_lo || y > s.wall_hi) {
            y = y < s.wall_lo ? 2.0 * s.wall_lo - y : 2.0 * s.wall_hi - y;
            v0 = -v0;
            v1 = -v1;
            v2 = -v2;
        }
    }
    if (s.per[0]) { const double hi = s.lo[0] + s.L[0]; if (x0 >= hi) x0 -= s.L[0]; else if (x0 < s.lo[0]) x0 += s.L[0]; }
    if (s.per[1]) { const double hi = s.lo[1] + s.L[1]; if (x1 >= hi) x1 -= s.L[1]; else if (x1 < s.lo[1]) x1 += s.L[1]; }
    if (s.per[2]) { const double hi = s.lo[2] + s.L[2]; if (x2 >= hi) x2 -= s.L[2]; else if (x2 < s.lo[2]) x2 += s.L[2]; }
}

// ----------------------------------------------------------------------------
// XCD-aware block order.  MI355X has 8 XCDs with a private L2 each, and the dispatcher
// hands workgroups to them round-robin.  A kernel launched with xcd_grid(n) blocks and
// using xcd_block() as its block index gives XCD x the contiguous logical blocks
// [x*per, (x+1)*per): neighbouring cells (and their particles) then share one L2.
// ----------------------------------------------------------------------------
constexpr int kXcds = 8;
inline unsigned xcd_grid(unsigned nblk) { return ((nblk + kXcds - 1) / kXcds) * kXcds; }
// logical block of this workgroup, or -1 for the padding blocks
__device__ __forceinline__ int64_t xcd_block(unsigned nblk)
{
    const unsigned per = (nblk + kXcds - 1) / kXcds;
    const unsigned b = blockIdx.x;
    const int64_t logical = (int64_t)(b % kXcds) * per + b / kXcds;
    return logical < nblk ? logical : -1;
}

// ----------------------------------------------------------------------------
// Launch helpers and kernel entry points (defined in the .hip files)
// ----------------------------------------------------------------------------
inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// Launch geometry of the inner force kernel (256-thread blocks): 16 or 8 lanes per bead, then
// a fixed grid of blocks striding over the fluid members (their number is known on the
// device only), scaled with the bead count (512 for ~10^4 beads).
// Lanes per bead: 16, or 8 once there are enough beads to fill the chip with wavefronts
// of eight beads (fewer idle lanes in each bead's short term lists and in its
// integration; on 2.56 M beads the inner step takes 16 % less time, on 10^4 beads half
// as many wavefronts leave the chip underused).
__host__ __device__ inline int inner_bead_lanes(int64_t nb) { return nb >= (int64_t(1) << 17) ? 8 : 16; }
__host__ __device__ inline int64_t inner_bead_blocks(int64_t nb)
{
    const int64_t per_block = 256 / inner_bead_lanes(nb);
    return (nb + per_block - 1) / per_block;
}
__host__ __device__ inline int64_t inner_fluid_blocks(int64_t nb)
{
    return nb / 20 < 512 ? 512 : (nb / 20 > 8192 ? 8192 : nb / 20);
}
__host__ __device__ inline int64_t inner_blocks(int64_t nb, int64_t cap_members)
{
    return inner_bead_blocks(nb) + (cap_members > nb ? inner_fluid_blocks(nb) : 0);
}
// one skin-check partial per block of the inner force kernel
__host__ __device__ inline int64_t dpart_entries(int64_t nb, int64_t cap_members) { return inner_blocks(nb, cap_members); }

// message of aimts_last_error(NULL), for entry points that take no context
void set_context_free_error(const char *msg);

void fill_i32(int32_t *p, int32_t val, int64_t n, hipStream_t st);
void fill_u8(uint8_t *p, uint8_t val, int64_t n, hipStream_t st);
void fill_f64(double *p, double val, int64_t n, hipStream_t st);
size_t scan_temp_bytes(int64_t n);
// exclusive prefix sum of in[0..n) into out[0..n], out[n] = total; in may alias out
void scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *temp, hipStream_t st);

struct SortBufs {
    int32_t *count, *cellof, *rank, *tmp_src, *src_of;
    uint32_t *tmp_id;
    double *x_alt, *v_alt;
    uint32_t *id_alt;
    int32_t *mos_alt;
    int32_t *scan_temp;
};
// Counting sort by cell; swaps the particle arrays of `s` with the alternates in `b`.
void rebuild_cells(Dev &s, SortBufs &b, hipStream_t st);

struct InnerBufs {
    uint8_t *marks;          // [32 ceil(N / 32)] member marks of fluid slots, 0 or 1 (cleared after use)
    int32_t *wcount;         // [ceil(N / 32) + 1] marks per word, then their exclusive scan
    int32_t *zero;           // device scalar 0
    int32_t *ell;            // [nb][bead_list_scratch_entries / nb] partners kept by the counting pass
    int32_t *cnt;            // [cap_members + 1]
    int32_t *queue;          // [nb + 1] count, then the beads whose lists are scanned again
    double *fi_alt;          // [3 nlev][cap_members]
    const int32_t *mos_old;  // [N] member of slot before the rebuild (old slot order)
    int32_t *scan_temp;
};
size_t bead_list_scratch_entries(int64_t nb);
// The platelet-list rebuild in two parts queued back to back on one stream: part 0
// resolves the topology to slots and runs the bead counting pass; part 1 does the rest.
void rebuild_inner(Dev &s, InnerBufs &b, const int32_t *src_of, hipStream_t st, int part);

void outer_forces(const Dev &s, uint64_t count, double dt_outer, hipStream_t st);
// Blocks of the DPD kernel for N slots, and the order it runs them in (host side, once
// per context): see dpd.hip.
int64_t dpd_blocks(int64_t N);
void dpd_block_order(int64_t N, int64_t n_fw, const int32_t nc[3], std::vector<int32_t> &order);

// Force groups of the inner level in three-level mode (Sec. 3.3, Table 1): the interface
// M (bead-fluid/wall), the flowing platelets' own terms P1 and the aggregating platelets'
// own terms with every inter-platelet term P2.
enum : int { kDueM = 1, kDueP1 = 2, kDueP2 = 4, kDueAll = 7 };
// What one inner step of the three-level scheme evaluates, and the half steps of the
// interface, flowing and aggregating levels (two-group mode: all due, all equal).
struct LevelStep {
    int due;
    double hm, h1, h2;
};

// Inner forces at the current positions (no integration); dt_rand scales the random
// term of the platelet-fluid interface (the step of the group it belongs to).
void inner_forces(const Dev &s, uint64_t count, double dt_rand, hipStream_t st);
// One inner step after the first drift: inner forces at the members' state in (xr, vr),
// then the closing half kicks of this inner step and, unless `last`, the opening half
// kicks and drift of the next, written to (xw, vw) (the other buffer: the partners are
// read while the members are written).  The last one also leaves the skin-check
// partials.  In three-level mode only the groups in ls.due are evaluated and kicked,
// each with its own half step.
void inner_step(const Dev &s, const double *xr, const double *vr, double *xw, double *vw, uint64_t count,
                double dt_inner, double dt_rand, bool last, const LevelStep &ls, hipStream_t st);

// Opening outer half kick of every mobile particle and all k inner drifts of the
// non-members; wall particles are copied into (xa, va), the members' second buffer.
// The members also take the opening inner half kicks (ls: of every level) and the first
// drift, written to (xw, vw).
void open_kick_lazy_drift(const Dev &s, double h_out, int k, double dt_in, double *xa, double *va,
                          const LevelStep &ls, double *xw, double *vw, hipStream_t st);
// Sublevels from the controller's per-platelet ratios (three-level mode): a platelet
// whose predicted ratio exceeds the system's ratio min(decision[0], k_cap) takes the
// flowing sublevel 1, the others the aggregating sublevel 2; then every bead's copy.
void levels_from_ratios(const Dev &s, const int32_t *pratio, const int32_t *decision, int32_t k_cap, hipStream_t st);
void levels_to_beads(const Dev &s, hipStream_t st);
void outer_kick(const Dev &s, double h_out, hipStream_t st);

// thermodynamics: out[0..7] = time, ke, T, T_pec, px, py, pz, k
void thermo(const Dev &s, double *partial, int chunks, double *out, double time, int k, hipStream_t st);
// The closing outer half kick fused with the per-row thermo sums of the kicked
// velocities (thermo_final then makes the series row).
void outer_kick_thermo_rows(const Dev &s, double h_out, double *partial, int chunks, hipStream_t st);
// The closing outer half kick h_close of the last outer step and the opening of the next
// (open_kick_lazy_drift's arguments) in one pass over the particles; with a non-null
// partial, also the thermo row sums of the closing-kicked velocities.
void outer_close_open(const Dev &s, double h_close, double *partial, int chunks, double h_out, int k, double dt_in,
                      double *xa, double *va, const LevelStep &ls, double *xw, double *vw, hipStream_t st);
void thermo_final(const Dev &s, const double *partial, int chunks, double *out, double time, int k, hipStream_t st);
// conservative energies and virial: out[0..5]
void energy(const Dev &s, double *partial, double *out, hipStream_t st);
// per-platelet features into ring row `row` of ring [P][64][8] (float); scratch holds
// feature_scratch_doubles(P) doubles
size_t feature_scratch_doubles(int64_t P);
// The paper's six measurements per platelet (omega, translational and rotational
// kinetic energy, flow speed at the centre of mass) into out[P][6], float64.
void paper_features(const Dev &s, double flow_r, double *out, hipStream_t st);
// Adds every bead's membrane stress (pressure-like virial trace times volume) to sum[nb].
void bead_stress(const Dev &s, double *sum, hipStream_t st);
// (h_pend: a closing outer half kick not yet applied to the stored velocities, which the
// traction's fluid velocities then add)
void features(const Dev &s, float *ring, int row, float *last, double *scratch, double h_pend, hipStream_t st);

}  // namespace aimts
