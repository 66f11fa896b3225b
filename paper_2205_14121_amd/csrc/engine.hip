// Host side of the aimts engine: context, workspace carve-up, argument checks,
// platelet topology (CSR per bead), the two-group RESPA scheduler (Sec. 3.3,
// MSM pseudocode Table 1) and the C ABI declared in include/aimts.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/aimts.h"
#include "common.h"
#include "ctrl.h"

using namespace aimts;

namespace {

// message of the last failed aimts_create (no context exists to hold it)
thread_local std::string g_create_error;

// hipGetLastError is sticky per thread: clear whatever an earlier, unrelated runtime call
// left behind so that only this call's launches are checked.
inline void clear_stale_hip_error() { (void)hipGetLastError(); }

constexpr int kThermoChunks = 16;
constexpr int kSeriesCols = 8;

struct Carver {
    char *base;
    size_t off = 0;
    size_t cap;
    bool dry;
    template <typename T>
    T *take(int64_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (size_t)std::max<int64_t>(n, 1);
        return p;
    }
};

constexpr int64_t kMaxParticles = (int64_t(1) << 27) - 1;

struct Geometry {
    int32_t nc[3];
    double side[3];
    int64_t ncell;
    int64_t cap_members, cap_pairs;
};

bool geometry_of(const aimts_system_desc *d, Geometry &g, std::string &why)
{
    if (!(d->cell_min > 0.0) || !std::isfinite(d->cell_min)) { why = "cell_min must be > 0"; return false; }
    for (int k = 0; k < 3; ++k) {
        if (!(d->L[k] > 0.0) || !std::isfinite(d->L[k]) || !std::isfinite(d->lo[k])) {
            why = "box lengths must be finite and > 0";
            return false;
        }
        int64_t n = (int64_t)std::floor(d->L[k] / d->cell_min);
        if (n < 1) n = 1;
        if (d->periodic[k] && n < 5) {
            why = "a periodic axis needs at least 5 cells of side >= cell_min";
            return false;
        }
        if (n > (1 << 20)) { why = "too many cells along an axis"; return false; }
        g.nc[k] = (int32_t)n;
        g.side[k] = d->L[k] / (double)n;
    }
    g.ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    const int64_t N = d->n_fluid + d->n_wall + d->n_bead;
    // slots, cells and list entries are 32-bit; the DPD kernel addresses its float4
    // position copies with 32-bit byte offsets
    if (N > kMaxParticles) { why = "at most 134,217,727 particles per context"; return false; }
    if (2 * g.ncell > (int64_t)INT32_MAX - 1) { why = "too many cells"; return false; }
    int64_t capS = d->n_bead > 0 ? std::min<int64_t>(d->n_fluid, std::max<int64_t>(4 * d->n_bead, 4096)) : 0;
    g.cap_members = d->n_bead + capS;
    // automatic pair-list capacity: pairs grow with the cube of the list reach (cutoff + skin);
    // ~96 (cutoff + skin)^3 entries per bead leaves about twice the count of a dense membrane
    const double reach = d->cell_min + d->skin;
    g.cap_pairs = d->inner_pair_capacity > 0 ? d->inner_pair_capacity
                                             : std::max<int64_t>((int64_t)std::ceil(96.0 * reach * reach * reach) * d->n_bead,
                                                                 1024);
    if (N >= ((int64_t)1 << 31) - 1 || g.cap_pairs >= ((int64_t)1 << 31) - 1) {
        why = "particle count or pair capacity exceeds 2^31";
        return false;
    }
    return true;
}

}  // namespace

namespace aimts {
// message returned by aimts_last_error(NULL): calls that have no context to hold one
void set_context_free_error(const char *msg) { g_create_error = msg ? msg : ""; }
}  // namespace aimts

constexpr int kProfPhases = 6;  // phases timed by aimts_profile

struct aimts_ctx {
    aimts_system_desc desc;
    Geometry geo;
    hipStream_t stream;
    // Most of the platelet-list rebuild runs on a second stream forked after the cell
    // sort and the bead counting pass, so that its small latency-bound kernels run
    // beside the DPD kernel (which needs only the sorted cells); `stream` waits for them
    // before anything that reads the lists.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool lists_pending = false;
    size_t prof_lists = SIZE_MAX;
    Dev s;
    SortBufs sb;
    InnerBufs ib;
    // diagnostics
    double *thermo_partial, *thermo_out, *energy_partial, *energy_out, *series;
    float *ring, *feat_last;
    double *feat_scratch;
    double *paper_feat;   // [P][6] the paper's six measurements (aimts_get_paper_features)
    double *stress_sum;   // [nb] running sum of the per-bead membrane stress
    int64_t stress_n = 0; // samples in stress_sum
    double *ck_x, *ck_v;  // rollback checkpoint: particle arrays at the start of a segment
    uint32_t *ck_id;
    CtrlState ctrl;
    // host state
    std::string err;
    bool have_state = false, have_forces = false, failed = false, have_topology = false;
    uint64_t outer_evals = 0, inner_evals = 0;
    int64_t step = 0, series_rows = 0, feat_rows = 0;
    double time = 0.0;
    int32_t k_now = 4, hold_now = 16, since_infer = 0, fallbacks = 0, inferences = 0, rollbacks = 0;
    int32_t k_if = 1, k_sub = 1;  // three-level scheme: interface and flowing-sublevel ratios
    int32_t k_outer = 0;          // ratio whose outer step scaled the random term of the current outer force
    // The closing outer half kick of the last outer step waits for the opening of the
    // next, which applies both in one pass over the particles (the velocities between
    // them are only read by the thermo row of that step, computed in the same pass, and
    // by the features, which add the pending kick themselves).  It is applied on its own
    // before anything that needs the synchronised state: a ratio change, a rollback
    // checkpoint, the end of the call.
    bool close_pending = false, row_pending = false;
    double close_h = 0.0, row_time = 0.0;
    int32_t row_k = 0;
    int64_t row_index = 0;
    double mass[3] = {1.0, 1.0, 1.0};
    double skin;
    double pre_margin = 0.0;
    std::vector<int32_t> h_body;
    // profiling: events recorded around launch groups, resolved after each step() call
    int32_t prof_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (phase, index of the start event)
    double prof_ms[kProfPhases] = {};
    int64_t prof_n[kProfPhases] = {};

    hipEvent_t next_event()
    {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    // open a timed interval of `phase`; returns the start-event index or SIZE_MAX
    size_t prof_begin(int phase, hipStream_t st)
    {
        if (!(prof_mask & (1 << phase))) return SIZE_MAX;
        hipEvent_t e = next_event();
        if (!e) return SIZE_MAX;
        (void)hipEventRecord(e, st);
        return ev_used - 1;
    }
    size_t prof_begin(int phase) { return prof_begin(phase, stream); }
    void prof_end(int phase, size_t start, hipStream_t st)
    {
        if (start == SIZE_MAX) return;
        hipEvent_t e = next_event();
        if (!e) return;
        (void)hipEventRecord(e, st);
        ev_marks.emplace_back(phase, start);
    }
    void prof_end(int phase, size_t start) { prof_end(phase, start, stream); }
    // after the stream is synchronised: accumulate the recorded intervals
    void prof_collect()
    {
        for (const auto &mk : ev_marks) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev_pool[mk.second], ev_pool[mk.second + 1]) == hipSuccess) {
                prof_ms[mk.first] += ms;
                prof_n[mk.first] += 1;
            }
        }
        ev_marks.clear();
        ev_used = 0;
    }

    aimts_status fail(aimts_status st, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return st;
    }
    aimts_status hip_check(const char *where)
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(AIMTS_E_HIP, "%s: %s", where, hipGetErrorString(e));
        return AIMTS_OK;
    }
};

namespace {

// angle forces in a pass of their own (aimts_system_desc.angle_pass)
bool angle_separate(const aimts_system_desc *d) { return d->angle_pass == 2; }

size_t carve(aimts_ctx *c, const aimts_system_desc *d, const Geometry &g, char *base, size_t cap, bool dry)
{
    Carver cv{base, 0, cap, dry};
    const int64_t N = d->n_fluid + d->n_wall + d->n_bead;
    const int64_t nb = d->n_bead, P = d->n_platelet;
    const int64_t C = g.cap_members;
    Dev s{};
    SortBufs sb{};
    InnerBufs ib{};
    s.x = cv.take<double>(3 * N);
    s.v = cv.take<double>(3 * N);
    s.dpd_order = cv.take<int32_t>(dpd_blocks(N));
    s.xf = cv.take<float4>(N);
    s.vf = cv.take<float4>(N);
    sb.x_alt = cv.take<double>(3 * N);
    sb.v_alt = cv.take<double>(3 * N);
    s.fo = cv.take<double>(3 * N);
    s.id = cv.take<uint32_t>(N);
    sb.id_alt = cv.take<uint32_t>(N);
    s.mos = cv.take<int32_t>(N);
    sb.mos_alt = cv.take<int32_t>(N);
    sb.cellof = cv.take<int32_t>(N);
    sb.rank = cv.take<int32_t>(N);
    sb.tmp_src = cv.take<int32_t>(N);
    sb.src_of = cv.take<int32_t>(N);
    sb.tmp_id = cv.take<uint32_t>(N);
    sb.count = cv.take<int32_t>(2 * g.ncell);
    s.cell_start = cv.take<int32_t>(2 * g.ncell + 1);
    const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(N, 2 * g.ncell), C) + 1;
    sb.scan_temp = cv.take<int32_t>((int64_t)(scan_temp_bytes(scan_n) / sizeof(int32_t)) + 4);
    ib.scan_temp = sb.scan_temp;
    s.bead_slot = cv.take<int32_t>(nb);
    s.member_slot = cv.take<int32_t>(C);
    s.n_members = cv.take<int32_t>(1);
    const int64_t nlev = d->three_level ? 3 : 1;  // inner force groups held per member
    s.fi = cv.take<double>(3 * nlev * C);
    ib.fi_alt = cv.take<double>(3 * nlev * C);
    s.blev = cv.take<uint8_t>(nb);
    s.plev = cv.take<int32_t>(P);
    s.xref = cv.take<double>(3 * C);
    s.pair_off = cv.take<int32_t>(C + 1);
    s.pair_nfl = cv.take<int32_t>(nb);
    ib.cnt = cv.take<int32_t>(C + 1);
    ib.ell = cv.take<int32_t>((int64_t)bead_list_scratch_entries(nb));
    ib.queue = cv.take<int32_t>(nb + 1);
    s.pair_list = cv.take<int32_t>(g.cap_pairs);
    ib.marks = cv.take<uint8_t>(32 * ((N + 31) / 32));
    ib.wcount = cv.take<int32_t>((N + 31) / 32 + 1);
    ib.zero = cv.take<int32_t>(1);
    s.body = cv.take<int32_t>(nb);
    s.rest = cv.take<double>(3 * nb);
    s.rest_f = cv.take<float4>(nb);
    s.rest_slot = cv.take<float4>(nb > 0 ? N : 0);
    s.bond_off = cv.take<int32_t>(nb + 1);
    s.bond_other = cv.take<int32_t>(2 * d->n_bond);
    s.bond_r0 = cv.take<double>(2 * d->n_bond);
    s.ang_off = cv.take<int32_t>(nb + 1);
    s.ang_ent = cv.take<int32_t>(3 * d->n_angle);
    s.ang_ijk = cv.take<int32_t>(3 * d->n_angle);
    s.ang_q4 = cv.take<int4>(3 * d->n_angle);
    s.angle_sep = angle_separate(d) ? 1 : 0;
    s.ang_slot = cv.take<int32_t>(s.angle_sep ? 3 * d->n_angle : 0);
    s.ang_f = cv.take<double>(s.angle_sep ? 9 * d->n_angle : 0);
    s.ang_th0 = cv.take<double>(d->n_angle);
    s.mor_off = cv.take<int32_t>(nb + 1);
    s.mor_other = cv.take<int32_t>(2 * d->n_morse);
    s.bond_slot = cv.take<int32_t>(2 * d->n_bond);
    s.mor_slot = cv.take<int32_t>(2 * d->n_morse);
    s.n_bond_ent = 2 * d->n_bond;
    s.n_mor_ent = 2 * d->n_morse;
    s.n_ang_ent = 3 * d->n_angle;
    s.plt_off = cv.take<int32_t>(P + 1);
    s.plt_area = cv.take<double>(P);
    s.err = cv.take<uint32_t>(4);
    s.maxdisp = cv.take<uint32_t>(4);
    s.plt_dmax = cv.take<float>(P);
    s.dmax = cv.take<float>(C);
    s.dpart = cv.take<float4>(dpart_entries(nb, C));
    double *thermo_partial = cv.take<double>((int64_t)g.nc[1] * kThermoChunks * 10);
    double *thermo_out = cv.take<double>(kSeriesCols);
    const int64_t nparts = (N + 255) / 256 + (nb + 255) / 256 + 1;
    double *energy_partial = cv.take<double>(nparts * 6);
    double *energy_out = cv.take<double>(8);
    double *series = cv.take<double>(d->series_capacity * kSeriesCols);
    float *ring = cv.take<float>(P * 64 * 8);
    float *feat_last = cv.take<float>(P * 8);
    double *feat_scratch = cv.take<double>((int64_t)feature_scratch_doubles(P));
    double *paper_feat = cv.take<double>(6 * P);
    double *stress_sum = cv.take<double>(nb);
    // rollback checkpoint of the particle arrays (slot order)
    double *ck_x = cv.take<double>(3 * N);
    double *ck_v = cv.take<double>(3 * N);
    uint32_t *ck_id = cv.take<uint32_t>(N);
    CtrlState ctrl{};
    ctrl_carve(ctrl, d->ctrl_max_batch, std::max<int64_t>(P, 1), [&](size_t bytes) -> void * {
        return cv.take<char>((int64_t)bytes);
    });
    if (!dry) {
        c->s = s;
        c->sb = sb;
        c->ib = ib;
        c->thermo_partial = thermo_partial;
        c->thermo_out = thermo_out;
        c->energy_partial = energy_partial;
        c->energy_out = energy_out;
        c->series = series;
        c->ring = ring;
        c->feat_last = feat_last;
        c->feat_scratch = feat_scratch;
        c->paper_feat = paper_feat;
        c->stress_sum = stress_sum;
        c->ck_x = ck_x;
        c->ck_v = ck_v;
        c->ck_id = ck_id;
        c->ctrl = ctrl;
    }
    return cv.off + 256;
}

bool finite_all(const double *p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

aimts_status sync_and_check(aimts_ctx *c, const char *where)
{
    aimts_status st = c->hip_check(where);
    if (st) return st;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->fail(AIMTS_E_HIP, "%s: %s", where, hipGetErrorString(e));
    return AIMTS_OK;
}

aimts_status h2d(aimts_ctx *c, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return AIMTS_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return c->fail(AIMTS_E_HIP, "copy to device: %s", hipGetErrorString(e));
    e = hipStreamSynchronize(c->stream);  // host arrays are borrowed for the call only
    if (e != hipSuccess) return c->fail(AIMTS_E_HIP, "copy to device: %s", hipGetErrorString(e));
    return AIMTS_OK;
}

aimts_status d2h(aimts_ctx *c, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return AIMTS_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->fail(AIMTS_E_HIP, "copy to host: %s", hipGetErrorString(e));
    return AIMTS_OK;
}

float bits_float(uint32_t u)
{
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

std::string err_text(uint32_t f)
{
    std::string s;
    if (f & kErrNonFinite) s += " non-finite velocity, or a position far outside the box;";
    if (f & kErrSkin) s += " displacements in one outer step exceeded the neighbour skin (raise skin or lower k);";
    if (f & kErrSkinBead) s += " bead displacements in one outer step exceeded the bead skin (raise skin_bead or lower k);";
    if (f & kErrPairCap) s += " platelet pair-list capacity exceeded (raise inner_pair_capacity);";
    if (f & kErrMemberCap) s += " too many fluid particles near platelets for the member capacity;";
    if (f & kErrOutside) s += " a particle left the box;";
    return s;
}

// Re-sort by cell and run the first part of the platelet-list rebuild (topology slots
// and the bead counting pass, whose long wavefronts would be starved beside the DPD
// kernel) on the context's stream, then fork the side stream.  rebuild_lists() queues
// the rest of the list rebuild there, after the caller has queued the DPD kernel, and
// join_lists() must come before any use of the lists.
void rebuild_cells_fork(aimts_ctx *c)
{
    size_t pe = c->prof_begin(2);
    rebuild_cells(c->s, c->sb, c->stream);
    c->prof_end(2, pe);
    c->ib.mos_old = c->sb.mos_alt;  // the member map before the sort, in the old slot order
    c->prof_lists = c->prof_begin(5);
    rebuild_inner(c->s, c->ib, c->sb.src_of, c->stream, 0);
    (void)hipEventRecord(c->ev_fork, c->stream);
}

void rebuild_lists(aimts_ctx *c)
{
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    rebuild_inner(c->s, c->ib, c->sb.src_of, c->side, 1);
    c->prof_end(5, c->prof_lists, c->side);
    (void)hipEventRecord(c->ev_join, c->side);
    c->lists_pending = true;
}

void join_lists(aimts_ctx *c)
{
    if (!c->lists_pending) return;
    (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
    c->lists_pending = false;
}

// Applies a pending closing outer half kick (with its thermo row, when one is due).
void flush_close(aimts_ctx *c)
{
    if (!c->close_pending) return;
    const size_t pe = c->prof_begin(3);
    if (c->row_pending) {
        outer_kick_thermo_rows(c->s, c->close_h, c->thermo_partial, kThermoChunks, c->stream);
        thermo_final(c->s, c->thermo_partial, kThermoChunks, c->series + c->row_index * kSeriesCols, c->row_time,
                     c->row_k, c->stream);
    } else {
        outer_kick(c->s, c->close_h, c->stream);
    }
    c->prof_end(3, pe);
    c->close_pending = c->row_pending = false;
}

void record_thermo(aimts_ctx *c, double *row)
{
    thermo(c->s, c->thermo_partial, kThermoChunks, row, c->time, c->k_now, c->stream);
}

}  // namespace

extern "C" {

aimts_status aimts_workspace_size(const aimts_system_desc *desc, size_t *bytes)
{
    if (!desc || !bytes) return AIMTS_E_INVALID;
    Geometry g;
    std::string why;
    if (desc->n_fluid < 0 || desc->n_wall < 0 || desc->n_bead < 0 || desc->n_platelet < 0 || desc->n_bond < 0 ||
        desc->n_angle < 0 || desc->n_morse < 0 || desc->series_capacity < 0 || desc->ctrl_max_batch < 0 ||
        desc->angle_pass < 0 || desc->angle_pass > 2 || desc->three_level < 0 || desc->three_level > 1)
        return AIMTS_E_INVALID;
    if (!geometry_of(desc, g, why)) return AIMTS_E_INVALID;
    *bytes = carve(nullptr, desc, g, nullptr, 0, true);
    return AIMTS_OK;
}

aimts_status aimts_create(const aimts_system_desc *desc, void *d_workspace, size_t bytes, void *hip_stream,
                          aimts_ctx **out)
{
    g_create_error.clear();
    if (!desc || !out) return AIMTS_E_INVALID;
    *out = nullptr;
    clear_stale_hip_error();
    size_t need = 0;
    if (aimts_workspace_size(desc, &need) != AIMTS_OK) return AIMTS_E_INVALID;
    if (desc->n_fluid + desc->n_wall + desc->n_bead <= 0) return AIMTS_E_INVALID;
    if (desc->n_bead > 0 && desc->n_platelet <= 0) return AIMTS_E_INVALID;
    if (desc->force_precision != 0 && desc->force_precision != 1) return AIMTS_E_INVALID;
    if (!(desc->skin >= 0.0) || !std::isfinite(desc->skin)) return AIMTS_E_INVALID;
    if (!(desc->skin_bead >= 0.0) || desc->skin_bead > desc->skin) return AIMTS_E_INVALID;
    if (!d_workspace || ((uintptr_t)d_workspace & 255u)) return AIMTS_E_INVALID;
    if (bytes < need) return AIMTS_E_NOMEM;
    aimts_ctx *c = new aimts_ctx();
    c->desc = *desc;
    std::string why;
    geometry_of(desc, c->geo, why);
    c->stream = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        g_create_error = "cannot create the side stream or its events";
        clear_stale_hip_error();
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->side) (void)hipStreamDestroy(c->side);
        delete c;
        return AIMTS_E_HIP;
    }
    carve(c, desc, c->geo, (char *)d_workspace, bytes, false);
    Dev &s = c->s;
    const Geometry &g = c->geo;
    for (int k = 0; k < 3; ++k) {
        s.lo[k] = desc->lo[k];
        s.L[k] = desc->L[k];
        s.half[k] = 0.5 * desc->L[k];
        s.side[k] = g.side[k];
        s.nc[k] = g.nc[k];
        s.per[k] = desc->periodic[k] ? 1 : 0;
        s.g[k] = 0.0;
    }
    s.ncell = g.ncell;
    {
        // 8 float ulps of the largest coordinate magnitude, added to the DPD cutoff for
        // the float pre-filter of the candidate scan
        double ext = 0.0;
        for (int k = 0; k < 3; ++k) ext = std::max(ext, std::max(std::fabs(desc->lo[k]), std::fabs(desc->lo[k] + desc->L[k])));
        const double ulp = std::ldexp(1.0, std::ilogb(std::max(ext, 1.0)) - 23);
        c->pre_margin = 8.0 * ulp;  // covers rounding of both positions and a periodic shift
    }
    s.nrow = g.nc[1];
    s.N = desc->n_fluid + desc->n_wall + desc->n_bead;
    s.nf = desc->n_fluid;
    s.nw = desc->n_wall;
    s.nb = desc->n_bead;
    s.b0 = desc->n_fluid + desc->n_wall;
    s.P = desc->n_platelet;
    s.cap_members = g.cap_members;
    s.cap_pairs = g.cap_pairs;
    s.fp32 = desc->force_precision;
    s.nlev = desc->three_level ? 3 : 1;
    s.wall_axis = -1;
    s.key0 = (uint32_t)desc->seed;
    s.key1 = (uint32_t)(desc->seed >> 32);
    for (int t = 0; t < 3; ++t) { s.m[t] = 1.0; s.minv[t] = 1.0; }
    s.rc = desc->cell_min;
    s.rc2 = s.rc * s.rc;
    s.inv_rc = 1.0 / s.rc;
    s.pre_rc2 = (s.rc + c->pre_margin) * (s.rc + c->pre_margin);
    s.rc_pf = 1.0;
    s.rc_pf2 = 1.0;
    s.inv_rc_pf = 1.0;
    c->skin = desc->skin;
    s.skin = desc->skin;
    s.skin_bead = desc->skin_bead > 0.0 ? desc->skin_bead : std::min(desc->skin, 0.5);
    s.disp_floor = 0.125 * desc->skin;
    s.disp_floor_bead = 0.125 * s.skin_bead;
    // empty topology and inner state
    fill_i32(s.bond_off, 0, s.nb + 1, c->stream);
    fill_i32(s.ang_off, 0, s.nb + 1, c->stream);
    fill_i32(s.mor_off, 0, s.nb + 1, c->stream);
    fill_i32(s.plt_off, 0, s.P + 1, c->stream);
    fill_i32((int32_t *)s.err, 0, 4, c->stream);
    fill_i32((int32_t *)s.maxdisp, 0, 4, c->stream);
    fill_i32((int32_t *)s.dmax, 0, s.cap_members, c->stream);
    fill_i32((int32_t *)s.dpart, 0, 4 * dpart_entries(s.nb, s.cap_members), c->stream);
    fill_i32(s.n_members, (int32_t)s.nb, 1, c->stream);
    // every platelet at the aggregating sublevel (the finest step) until aimts_set_levels
    fill_i32(s.plev, 2, s.P, c->stream);
    fill_u8(s.blev, 2, s.nb, c->stream);
    // counters the rebuild expects at zero (each rebuild clears them again after use)
    fill_i32(c->sb.count, 0, 2 * s.ncell, c->stream);
    fill_i32((int32_t *)c->ib.marks, 0, 8 * ((s.N + 31) / 32), c->stream);
    fill_i32(c->ib.zero, 0, 1, c->stream);
    fill_i32(c->ib.queue, 0, 1, c->stream);  // no bead scanned again before the first rebuild
    ctrl_init(c->ctrl, c->stream);
    aimts_status st = sync_and_check(c, "create");
    if (!st) {
        std::vector<int32_t> order;
        dpd_block_order(s.N, s.b0, s.nc, order);
        st = h2d(c, s.dpd_order, order.data(), sizeof(int32_t) * order.size());
    }
    if (st) {
        g_create_error = c->err;
        delete c;
        return st;
    }
    *out = c;
    return AIMTS_OK;
}

aimts_status aimts_destroy(aimts_ctx *c)
{
    if (!c) return AIMTS_E_INVALID;
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamSynchronize(c->side);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    (void)hipEventDestroy(c->ev_fork);
    (void)hipEventDestroy(c->ev_join);
    (void)hipStreamDestroy(c->side);
    delete c;
    return AIMTS_OK;
}

const char *aimts_last_error(const aimts_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

// reach of the platelet pair list in cells
static void update_reach(aimts_ctx *c)
{
    Dev &s = c->s;
    const double rin = std::max(s.rc_pf, std::sqrt(std::max(s.lj_rc2, 0.0)));
    const double cut = rin + c->skin;
    s.list_cut2 = cut * cut;
    // bead partners are listed to the WCA cutoff plus the bead skin, and at least to the
    // contact radius: the contact-count feature counts bead pairs from these lists (the
    // bead skin check still uses skin_bead)
    const double bb = std::max(std::sqrt(std::max(s.lj_rc2, 0.0)) + s.skin_bead, kContactRadius);
    s.bb_cut2 = bb * bb;
    // beads of other platelets also to the aggregation cutoff plus the bead skin
    const double bbo = s.agg_on ? std::max(bb, std::sqrt(s.agg_rc2) + s.skin_bead) : bb;
    s.bbo_cut2 = bbo * bbo;
    const double far = std::max(cut, bbo);
    const double pre = far + c->pre_margin;
    s.pre_list2 = pre * pre;
    s.pre_bb2 = (bb + c->pre_margin) * (bb + c->pre_margin);
    s.pre_bbo2 = (bbo + c->pre_margin) * (bbo + c->pre_margin);
    int R = 1;
    for (int k = 0; k < 3; ++k) R = std::max(R, (int)std::ceil(far / s.side[k]));
    s.reach = R;
}

static aimts_status check_reach(aimts_ctx *c)
{
    if ((2 * c->s.reach + 1) * (2 * c->s.reach + 1) > 64)
        return c->fail(AIMTS_E_INVALID, "platelet reach (cutoff + skin) spans %d cells; at most 3 are supported "
                                        "(lower the skin or raise cell_min)", c->s.reach);
    for (int k = 0; k < 3; ++k)
        if (c->s.per[k] && c->s.nc[k] < 2 * c->s.reach + 1)
            return c->fail(AIMTS_E_INVALID, "platelet reach (cutoff + skin) needs %d cells along axis %d, box has %d",
                           2 * c->s.reach + 1, k, c->s.nc[k]);
    return AIMTS_OK;
}

// The interface ratio of an outer step at ratio k: k_if, or k itself when smaller (both
// powers of two in three-level mode); 1 in two-group mode.
static int interface_ratio(const aimts_ctx *c, int k) { return std::min(c->k_if, std::max(k, 1)); }

aimts_status aimts_set_levels(aimts_ctx *c, int32_t k_if, int32_t k_sub, const int32_t *level)
{
    if (!c) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    auto pow2 = [](int32_t v) { return v >= 1 && v <= 64 && (v & (v - 1)) == 0; };
    if (!pow2(k_if) || !pow2(k_sub) || k_sub > k_if)
        return c->fail(AIMTS_E_INVALID, "k_if and k_sub must be powers of two in [1, 64] with k_sub <= k_if");
    if (c->s.nlev != 3 && (k_if != 1 || k_sub != 1 || level))
        return c->fail(AIMTS_E_UNSUPPORTED, "the three-level scheme needs a context created with three_level = 1");
    const int64_t P = c->s.P;
    if (level) {
        for (int64_t p = 0; p < P; ++p)
            if (level[p] != 1 && level[p] != 2) return c->fail(AIMTS_E_INVALID, "platelet sublevels must be 1 or 2");
        aimts_status st = h2d(c, c->s.plev, level, sizeof(int32_t) * P);
        if (st) return st;
        levels_to_beads(c->s, c->stream);
        if ((st = sync_and_check(c, "set_levels"))) return st;
    }
    c->k_if = k_if;
    c->k_sub = k_sub;
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_get_levels(aimts_ctx *c, int32_t *k_if, int32_t *k_sub, int32_t *level)
{
    if (!c) return AIMTS_E_INVALID;
    if (k_if) *k_if = c->k_if;
    if (k_sub) *k_sub = c->k_sub;
    if (level && c->s.P > 0) {
        if (c->s.nlev != 3) {
            for (int64_t p = 0; p < c->s.P; ++p) level[p] = 2;
            return AIMTS_OK;
        }
        return d2h(c, level, c->s.plev, sizeof(int32_t) * c->s.P);
    }
    return AIMTS_OK;
}

aimts_status aimts_get_level_forces(aimts_ctx *c, double *f_m, double *f_p1, double *f_p2)
{
    if (!c) return AIMTS_E_INVALID;
    if (!c->have_forces) return c->fail(AIMTS_E_STATE, "no forces computed");
    Dev &s = c->s;
    const int64_t N = s.N, C = s.cap_members;
    double *outs[3] = {f_m, f_p1, f_p2};
    for (double *o : outs)
        if (o) std::memset(o, 0, sizeof(double) * 3 * N);
    int32_t nm = 0;
    aimts_status st = d2h(c, &nm, s.n_members, sizeof nm);
    if (st || nm == 0) return st;
    std::vector<uint32_t> ids(N);
    std::vector<int32_t> ms(nm);
    std::vector<double> fi(3 * (size_t)s.nlev * C);
    if ((st = d2h(c, ids.data(), s.id, sizeof(uint32_t) * N))) return st;
    if ((st = d2h(c, ms.data(), s.member_slot, sizeof(int32_t) * nm))) return st;
    if ((st = d2h(c, fi.data(), s.fi, sizeof(double) * fi.size()))) return st;
    for (int l = 0; l < s.nlev; ++l) {
        if (!outs[l]) continue;
        for (int32_t m = 0; m < nm; ++m)
            for (int k = 0; k < 3; ++k) outs[l][3 * ids[ms[m]] + k] = fi[(3 * l + k) * C + m];
    }
    return AIMTS_OK;
}

aimts_status aimts_set_masses(aimts_ctx *c, const double mass[3])
{
    if (!c || !mass) return AIMTS_E_INVALID;
    for (int t = 0; t < 3; ++t)
        if (!(mass[t] > 0.0) || !std::isfinite(mass[t])) return c->fail(AIMTS_E_INVALID, "masses must be > 0");
    for (int t = 0; t < 3; ++t) {
        c->s.m[t] = mass[t];
        c->s.minv[t] = 1.0 / mass[t];
    }
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_dpd(aimts_ctx *c, double a, double gamma, double sigma, double rc)
{
    if (!c) return AIMTS_E_INVALID;
    if (!std::isfinite(a) || !(gamma >= 0.0) || !(sigma >= 0.0) || !(rc > 0.0) || !std::isfinite(gamma) ||
        !std::isfinite(sigma))
        return c->fail(AIMTS_E_INVALID, "DPD parameters must be finite, gamma, sigma >= 0, rc > 0");
    if (rc > c->desc.cell_min * (1.0 + 1e-12))
        return c->fail(AIMTS_E_INVALID, "DPD cutoff %g exceeds cell_min %g", rc, c->desc.cell_min);
    c->s.a = a;
    c->s.gamma = gamma;
    c->s.sigma = sigma;
    c->s.rc = rc;
    c->s.rc2 = rc * rc;
    c->s.inv_rc = 1.0 / rc;
    c->s.pre_rc2 = (rc + c->pre_margin) * (rc + c->pre_margin);
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_lj(aimts_ctx *c, double eps, double sig, double rc_lj, double r_excl)
{
    if (!c) return AIMTS_E_INVALID;
    if (!(eps >= 0.0) || !(sig > 0.0) || !(rc_lj >= 0.0) || !(r_excl >= 0.0) || !std::isfinite(eps) ||
        !std::isfinite(rc_lj) || !std::isfinite(r_excl))
        return c->fail(AIMTS_E_INVALID, "LJ parameters must be finite, eps >= 0, sig > 0, rc >= 0, r_excl >= 0");
    c->s.lj_eps = eps;
    c->s.lj_sig2 = sig * sig;
    c->s.lj_rc2 = rc_lj * rc_lj;
    c->s.r_excl2 = r_excl * r_excl;
    update_reach(c);
    c->have_forces = false;
    return check_reach(c);
}

aimts_status aimts_set_interface(aimts_ctx *c, double gamma_pf, double sigma_pf, double rc_pf)
{
    if (!c) return AIMTS_E_INVALID;
    if (!(gamma_pf >= 0.0) || !(sigma_pf >= 0.0) || !(rc_pf > 0.0) || !std::isfinite(gamma_pf) ||
        !std::isfinite(sigma_pf) || !std::isfinite(rc_pf))
        return c->fail(AIMTS_E_INVALID, "interface parameters must be finite, >= 0, rc_pf > 0");
    c->s.gpf = gamma_pf;
    c->s.spf = sigma_pf;
    c->s.rc_pf = rc_pf;
    c->s.rc_pf2 = rc_pf * rc_pf;
    c->s.inv_rc_pf = 1.0 / rc_pf;
    update_reach(c);
    c->have_forces = false;
    return check_reach(c);
}

aimts_status aimts_set_platelets(aimts_ctx *c, const int32_t *body, const double *rest, const double *area)
{
    if (!c) return AIMTS_E_INVALID;
    const int64_t nb = c->s.nb, P = c->s.P;
    if (nb == 0) return AIMTS_OK;
    if (!body || !rest || !area) return c->fail(AIMTS_E_INVALID, "body, rest and area are required");
    std::vector<int32_t> off(P + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        if (body[b] < 0 || body[b] >= P) return c->fail(AIMTS_E_INVALID, "bead %lld has platelet %d out of range",
                                                         (long long)b, body[b]);
        if (b > 0 && body[b] < body[b - 1]) return c->fail(AIMTS_E_INVALID, "beads must be grouped by platelet in order");
        off[body[b] + 1]++;
    }
    for (int64_t p = 0; p < P; ++p) {
        if (off[p + 1] == 0) return c->fail(AIMTS_E_INVALID, "platelet %lld has no beads", (long long)p);
        if (!(area[p] > 0.0)) return c->fail(AIMTS_E_INVALID, "platelet areas must be > 0");
        off[p + 1] += off[p];
    }
    if (!finite_all(rest, 3 * nb)) return c->fail(AIMTS_E_INVALID, "rest coordinates must be finite");
    std::vector<double> rsoa(3 * nb);
    std::vector<float4> rf(nb);
    for (int64_t b = 0; b < nb; ++b) {
        for (int k = 0; k < 3; ++k) rsoa[k * nb + b] = rest[3 * b + k];
        int32_t bw = body[b];
        float w;
        std::memcpy(&w, &bw, sizeof w);
        rf[b] = make_float4((float)rest[3 * b], (float)rest[3 * b + 1], (float)rest[3 * b + 2], w);
    }
    aimts_status st;
    if ((st = h2d(c, c->s.body, body, sizeof(int32_t) * nb))) return st;
    if ((st = h2d(c, c->s.rest, rsoa.data(), sizeof(double) * 3 * nb))) return st;
    if ((st = h2d(c, c->s.rest_f, rf.data(), sizeof(float4) * nb))) return st;
    if ((st = h2d(c, c->s.plt_off, off.data(), sizeof(int32_t) * (P + 1)))) return st;
    if ((st = h2d(c, c->s.plt_area, area, sizeof(double) * P))) return st;
    c->h_body.assign(body, body + nb);
    c->have_topology = true;
    c->have_forces = false;
    return AIMTS_OK;
}

static aimts_status pair_csr(aimts_ctx *c, int64_t n, const int32_t *ij, const double *r0, int32_t *d_off,
                             int32_t *d_other, double *d_r0, const char *what)
{
    const int64_t nb = c->s.nb, b0 = c->s.b0;
    std::vector<int32_t> off(nb + 1, 0);
    for (int64_t q = 0; q < n; ++q) {
        for (int e = 0; e < 2; ++e) {
            const int64_t i = ij[2 * q + e];
            if (i < b0 || i >= b0 + nb) return c->fail(AIMTS_E_INVALID, "%s %lld: particle %lld is not a bead", what,
                                                        (long long)q, (long long)i);
        }
        if (ij[2 * q] == ij[2 * q + 1]) return c->fail(AIMTS_E_INVALID, "%s %lld joins a bead to itself", what, (long long)q);
        off[ij[2 * q] - b0 + 1]++;
        off[ij[2 * q + 1] - b0 + 1]++;
    }
    for (int64_t b = 0; b < nb; ++b) off[b + 1] += off[b];
    std::vector<int32_t> fill(off.begin(), off.end() - 1), other(2 * n);
    std::vector<double> rr(r0 ? 2 * n : 0);
    for (int64_t q = 0; q < n; ++q) {
        const int32_t a = (int32_t)(ij[2 * q] - b0), b = (int32_t)(ij[2 * q + 1] - b0);
        other[fill[a]] = b;
        other[fill[b]] = a;
        if (r0) { rr[fill[a]] = r0[q]; rr[fill[b]] = r0[q]; }
        fill[a]++;
        fill[b]++;
    }
    aimts_status st;
    if ((st = h2d(c, d_off, off.data(), sizeof(int32_t) * (nb + 1)))) return st;
    if ((st = h2d(c, d_other, other.data(), sizeof(int32_t) * 2 * n))) return st;
    if (r0 && (st = h2d(c, d_r0, rr.data(), sizeof(double) * 2 * n))) return st;
    return AIMTS_OK;
}

aimts_status aimts_set_bonds(aimts_ctx *c, int64_t n, const int32_t *ij, const double *r0, double k)
{
    if (!c) return AIMTS_E_INVALID;
    if (n != c->desc.n_bond) return c->fail(AIMTS_E_INVALID, "bond count %lld differs from the system's %lld",
                                            (long long)n, (long long)c->desc.n_bond);
    if (n > 0 && (!ij || !r0)) return c->fail(AIMTS_E_INVALID, "bond arrays are required");
    if (!(k >= 0.0) || !std::isfinite(k)) return c->fail(AIMTS_E_INVALID, "bond constant must be finite and >= 0");
    for (int64_t q = 0; q < n; ++q)
        if (!(r0[q] > 0.0) || !std::isfinite(r0[q])) return c->fail(AIMTS_E_INVALID, "bond rest lengths must be > 0");
    aimts_status st = pair_csr(c, n, ij, r0, c->s.bond_off, c->s.bond_other, c->s.bond_r0, "bond");
    if (st) return st;
    c->s.kb = k;
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_angles(aimts_ctx *c, int64_t n, const int32_t *ijk, const double *th0, double k)
{
    if (!c) return AIMTS_E_INVALID;
    if (n != c->desc.n_angle) return c->fail(AIMTS_E_INVALID, "angle count %lld differs from the system's %lld",
                                             (long long)n, (long long)c->desc.n_angle);
    if (n > 0 && (!ijk || !th0)) return c->fail(AIMTS_E_INVALID, "angle arrays are required");
    if (!(k >= 0.0) || !std::isfinite(k)) return c->fail(AIMTS_E_INVALID, "angle constant must be finite and >= 0");
    const int64_t nb = c->s.nb, b0 = c->s.b0;
    std::vector<int32_t> off(nb + 1, 0), tri(3 * n);
    for (int64_t q = 0; q < n; ++q) {
        for (int e = 0; e < 3; ++e) {
            const int64_t i = ijk[3 * q + e];
            if (i < b0 || i >= b0 + nb) return c->fail(AIMTS_E_INVALID, "angle %lld: particle %lld is not a bead",
                                                        (long long)q, (long long)i);
            tri[3 * q + e] = (int32_t)(i - b0);
            off[i - b0 + 1]++;
        }
        if (ijk[3 * q] == ijk[3 * q + 1] || ijk[3 * q + 1] == ijk[3 * q + 2] || ijk[3 * q] == ijk[3 * q + 2])
            return c->fail(AIMTS_E_INVALID, "angle %lld repeats a bead", (long long)q);
        if (!std::isfinite(th0[q]) || th0[q] < 0.0 || th0[q] > M_PI)
            return c->fail(AIMTS_E_INVALID, "rest angles must lie in [0, pi]");
    }
    for (int64_t b = 0; b < nb; ++b) off[b + 1] += off[b];
    std::vector<int32_t> fill(off.begin(), off.end() - 1), ent(3 * n);
    for (int64_t q = 0; q < n; ++q)
        for (int e = 0; e < 3; ++e) ent[fill[tri[3 * q + e]]++] = (int32_t)(q * 4 + e);
    aimts_status st;
    if ((st = h2d(c, c->s.ang_off, off.data(), sizeof(int32_t) * (nb + 1)))) return st;
    if ((st = h2d(c, c->s.ang_ent, ent.data(), sizeof(int32_t) * 3 * n))) return st;
    if ((st = h2d(c, c->s.ang_ijk, tri.data(), sizeof(int32_t) * 3 * n))) return st;
    if ((st = h2d(c, c->s.ang_th0, th0, sizeof(double) * n))) return st;
    c->s.ka = k;
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_morse(aimts_ctx *c, int64_t n, const int32_t *ij, double D, double a, double r0)
{
    if (!c) return AIMTS_E_INVALID;
    if (n != c->desc.n_morse) return c->fail(AIMTS_E_INVALID, "Morse bond count %lld differs from the system's %lld",
                                             (long long)n, (long long)c->desc.n_morse);
    if (n > 0 && !ij) return c->fail(AIMTS_E_INVALID, "Morse bond array is required");
    if (!std::isfinite(D) || !std::isfinite(a) || !std::isfinite(r0) || !(a > 0.0) || !(r0 > 0.0))
        return c->fail(AIMTS_E_INVALID, "Morse parameters must be finite, a > 0, r0 > 0");
    aimts_status st = pair_csr(c, n, ij, nullptr, c->s.mor_off, c->s.mor_other, nullptr, "Morse bond");
    if (st) return st;
    c->s.mD = D;
    c->s.ma = a;
    c->s.mr0 = r0;
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_aggregation(aimts_ctx *c, double D, double a, double r0, double fA, double rc)
{
    if (!c) return AIMTS_E_INVALID;
    if (!std::isfinite(D) || !std::isfinite(a) || !std::isfinite(r0) || !std::isfinite(fA) || !std::isfinite(rc) ||
        !(D >= 0.0) || !(a > 0.0) || !(r0 > 0.0) || !(rc >= 0.0))
        return c->fail(AIMTS_E_INVALID, "aggregation parameters must be finite, D >= 0, a > 0, r0 > 0, rc >= 0");
    if (rc > 0.0 && c->s.nb == 0) return c->fail(AIMTS_E_INVALID, "aggregation needs platelet beads");
    Dev &s = c->s;
    s.agg_on = rc > 0.0 ? 1 : 0;
    s.agg_D = D;
    s.agg_a = a;
    s.agg_r0 = r0;
    s.agg_fA = fA;
    s.agg_rc2 = rc * rc;
    // energy of the pair at the cutoff (the reported energy is shifted to 0 there)
    const double ex = std::exp(-a * (rc - r0)), q = 1.0 - rc / r0;
    s.agg_eshift = rc > 0.0 ? D * (ex * ex - 2.0 * ex) + 0.5 * fA * r0 * q * q : 0.0;
    update_reach(c);
    c->have_forces = false;
    return check_reach(c);
}

aimts_status aimts_set_external(aimts_ctx *c, const double g[3], int32_t wall_axis, double wall_lo, double wall_hi)
{
    if (!c || !g) return AIMTS_E_INVALID;
    if (!finite_all(g, 3)) return c->fail(AIMTS_E_INVALID, "body force must be finite");
    if (wall_axis < -1 || wall_axis > 2) return c->fail(AIMTS_E_INVALID, "wall_axis must be -1, 0, 1 or 2");
    if (wall_axis >= 0) {
        if (c->s.per[wall_axis]) return c->fail(AIMTS_E_INVALID, "the wall axis must not be periodic");
        if (!(wall_lo < wall_hi) || wall_lo < c->s.lo[wall_axis] ||
            wall_hi > c->s.lo[wall_axis] + c->s.L[wall_axis])
            return c->fail(AIMTS_E_INVALID, "walls must satisfy lo <= wall_lo < wall_hi <= lo + L");
    }
    for (int k = 0; k < 3; ++k) c->s.g[k] = g[k];
    c->s.wall_axis = wall_axis;
    c->s.wall_lo = wall_lo;
    c->s.wall_hi = wall_hi;
    c->have_forces = false;
    return AIMTS_OK;
}

aimts_status aimts_set_counters(aimts_ctx *c, uint64_t outer_evals, uint64_t inner_evals)
{
    if (!c) return AIMTS_E_INVALID;
    c->outer_evals = outer_evals;
    c->inner_evals = inner_evals;
    return AIMTS_OK;
}

aimts_status aimts_get_counters(aimts_ctx *c, uint64_t *outer_evals, uint64_t *inner_evals)
{
    if (!c) return AIMTS_E_INVALID;
    if (outer_evals) *outer_evals = c->outer_evals;
    if (inner_evals) *inner_evals = c->inner_evals;
    return AIMTS_OK;
}

aimts_status aimts_set_state(aimts_ctx *c, const double *x, const double *v)
{
    if (!c || !x || !v) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    Dev &s = c->s;
    const int64_t N = s.N;
    if (!finite_all(x, 3 * N) || !finite_all(v, 3 * N)) return c->fail(AIMTS_E_INVALID, "state must be finite");
    if (s.nb > 0 && !c->have_topology) return c->fail(AIMTS_E_STATE, "aimts_set_platelets must come first");
    std::vector<double> xs(3 * N), vs(3 * N);
    std::vector<uint32_t> ids(N);
    for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) {
            double xk = x[3 * i + k];
            const double lo = s.lo[k], hi = s.lo[k] + s.L[k];
            if (s.per[k]) {
                xk = std::fmod(xk - lo, s.L[k]);
                if (xk < 0) xk += s.L[k];
                xk += lo;
                if (xk >= hi) xk = lo;
            } else if (xk < lo || xk > hi) {
                return c->fail(AIMTS_E_INVALID, "particle %lld lies outside the box along non-periodic axis %d",
                               (long long)i, k);
            }
            xs[k * N + i] = xk;
            vs[k * N + i] = (i >= s.nf && i < s.b0) ? 0.0 : v[3 * i + k];
        }
        ids[i] = (uint32_t)i;
    }
    aimts_status st;
    if ((st = h2d(c, s.x, xs.data(), sizeof(double) * 3 * N))) return st;
    if ((st = h2d(c, s.v, vs.data(), sizeof(double) * 3 * N))) return st;
    if ((st = h2d(c, s.id, ids.data(), sizeof(uint32_t) * N))) return st;
    fill_i32(s.mos, -1, N, c->stream);
    fill_i32((int32_t *)c->ib.marks, 0, 8 * ((N + 31) / 32), c->stream);
    fill_i32((int32_t *)s.err, 0, 4, c->stream);
    fill_i32((int32_t *)s.maxdisp, 0, 4, c->stream);
    fill_i32((int32_t *)s.dmax, 0, s.cap_members, c->stream);
    fill_i32((int32_t *)s.dpart, 0, 4 * dpart_entries(s.nb, s.cap_members), c->stream);
    fill_f64(s.fi, 0.0, 3 * s.nlev * s.cap_members, c->stream);
    fill_f64((double *)s.fo, 0.0, 3 * N, c->stream);
    if ((st = sync_and_check(c, "set_state"))) return st;
    c->have_state = true;
    c->have_forces = false;
    c->failed = false;
    c->close_pending = c->row_pending = false;
    c->step = 0;
    c->time = 0.0;
    c->series_rows = 0;
    c->feat_rows = 0;
    c->since_infer = 0;
    return AIMTS_OK;
}

aimts_status aimts_compute_forces(aimts_ctx *c, double dt_inner, int32_t k)
{
    if (!c) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (!c->have_state) return c->fail(AIMTS_E_STATE, "no state set");
    if (!(dt_inner > 0.0) || !std::isfinite(dt_inner) || k < 1 || k > 64)
        return c->fail(AIMTS_E_INVALID, "dt_inner must be > 0 and 1 <= k <= 64");
    if (c->s.nb > 0) {
        aimts_status st = check_reach(c);
        if (st) return st;
    }
    rebuild_cells_fork(c);
    outer_forces(c->s, c->outer_evals, k * dt_inner, c->stream);
    c->k_outer = k;
    rebuild_lists(c);
    join_lists(c);
    inner_forces(c->s, c->inner_evals, interface_ratio(c, k) * dt_inner, c->stream);
    c->inner_evals++;
    c->outer_evals++;
    aimts_status st = sync_and_check(c, "compute_forces");
    if (st) return st;
    uint32_t flags = 0;
    if ((st = d2h(c, &flags, c->s.err, sizeof flags))) return st;
    if (flags & (kErrPairCap | kErrMemberCap))
        return c->fail(AIMTS_E_NOMEM, "neighbour lists overflow:%s", err_text(flags).c_str());
    c->have_forces = true;
    return AIMTS_OK;
}

aimts_status aimts_step(aimts_ctx *c, int64_t n_outer, const aimts_schedule *sch)
{
    if (!c || !sch) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (c->failed) return c->fail(AIMTS_E_STATE, "context failed earlier; call aimts_set_state");
    if (!c->have_state || !c->have_forces) return c->fail(AIMTS_E_STATE, "call aimts_set_state and aimts_compute_forces first");
    if (n_outer < 0) return c->fail(AIMTS_E_INVALID, "n_outer must be >= 0");
    if (!(sch->dt_inner > 0.0) || !std::isfinite(sch->dt_inner)) return c->fail(AIMTS_E_INVALID, "dt_inner must be > 0");
    if (sch->k < 1 || sch->k > 64) return c->fail(AIMTS_E_INVALID, "k must lie in [1, 64]");
    if (sch->mode != 0 && sch->mode != 1) return c->fail(AIMTS_E_INVALID, "mode must be 0 or 1");
    if (sch->diag_every < 0) return c->fail(AIMTS_E_INVALID, "diag_every must be >= 0");
    if (sch->k_max < 0 || sch->k_max > 64) return c->fail(AIMTS_E_INVALID, "k_max must lie in [0, 64]");
    if (sch->rollback < 0) return c->fail(AIMTS_E_INVALID, "rollback must be >= 0");
    if (sch->mode == 1 && (c->s.P == 0 || !c->ctrl.have_weights))
        return c->fail(AIMTS_E_STATE, "controller mode needs platelets and weights");
    if (sch->mode == 0 && sch->k % interface_ratio(c, sch->k) != 0)
        return c->fail(AIMTS_E_INVALID, "k = %d is no multiple of the interface ratio %d", sch->k,
                       interface_ratio(c, sch->k));
    Dev &s = c->s;
    const double dt = sch->dt_inner;
    if (sch->mode == 0) c->k_now = sch->k;
    int32_t k_force = 0;  // > 0: the ratio of a rerun segment (no controller decisions)
    int32_t k_seen = 0;   // largest ratio of the current segment
    // One outer step of two-group RESPA at the ratio in force.
    auto outer_step = [&]() -> aimts_status {
        const int k = k_force > 0 ? k_force : c->k_now;
        k_seen = std::max(k_seen, k);
        const double Dt = k * dt;
        // A new ratio (a controller decision, a fixed-ratio call after another ratio):
        // the outer force of this instant was scaled for the previous outer step Dn, and
        // its closing half kick already used it.  The random impulse of the instant spans
        // half of each adjacent step, so its variance must be sigma^2 w^2 (Dn + Dt) / 2:
        // with the closing half kick's part fixed, the opening half kick's random term is
        // scaled by c = (sqrt(2 (Dn + Dt)) - sqrt(Dn)) / Dt (1 / sqrt(Dt) when Dn = Dt).
        // In float32 mode the pair kernel reads velocities only from the copy taken at
        // the last rebuild, which the closing kick did not touch, so evaluating it again
        // with the same counter reproduces the conservative and dissipative terms exactly
        // and only rescales the random term.
        if (s.fp32 && c->k_outer > 0 && c->k_outer != k) {
            flush_close(c);  // the closing kick uses the force as it was
            const double Dn = c->k_outer * dt;
            const double cf = (std::sqrt(2.0 * (Dn + Dt)) - std::sqrt(Dn)) / Dt;
            outer_forces(s, c->outer_evals - 1, 1.0 / (cf * cf), c->stream);
            c->k_outer = k;
        }
        // The members' state alternates between the particle arrays and the sort's spare
        // arrays (free until the next sort), so that an inner step reads its partners
        // while it writes its members.  The first drift goes to the spare arrays when k
        // is odd and stays in place when k is even; either way the last inner step
        // writes back into the particle arrays.
        double *xa = c->sb.x_alt, *va = c->sb.v_alt;
        bool spare = (k & 1) != 0;  // the members' state is in the spare arrays
        // three-level scheme: the interface steps every kif inner steps, the flowing
        // sublevel every ksub (two-group mode: every level at every inner step)
        const int kif = interface_ratio(c, k), ksub = std::min(c->k_sub, kif);
        const LevelStep open{kDueAll, 0.5 * kif * dt, 0.5 * ksub * dt, 0.5 * dt};
        size_t pe = c->prof_begin(3);
        if (c->close_pending) {
            // the last step's closing half kick (and its thermo row) with this opening
            outer_close_open(s, c->close_h, c->row_pending ? c->thermo_partial : nullptr, kThermoChunks, 0.5 * Dt, k,
                             dt, xa, va, open, spare ? xa : s.x, spare ? va : s.v, c->stream);
            if (c->row_pending)
                thermo_final(s, c->thermo_partial, kThermoChunks, c->series + c->row_index * kSeriesCols, c->row_time,
                             c->row_k, c->stream);
            c->close_pending = c->row_pending = false;
        } else {
            open_kick_lazy_drift(s, 0.5 * Dt, k, dt, xa, va, open, spare ? xa : s.x, spare ? va : s.v, c->stream);
        }
        c->prof_end(3, pe);
        pe = c->prof_begin(1);
        for (int q = 1; q <= k; ++q) {
            const double *xr = spare ? xa : s.x, *vr = spare ? va : s.v;
            double *xw = spare ? s.x : xa, *vw = spare ? s.v : va;
            LevelStep ls = open;
            ls.due = kDueP2 | (q % ksub == 0 ? kDueP1 : 0) | (q % kif == 0 ? kDueM : 0);
            // the interface group's random numbers count its own evaluations
            const uint64_t cnt = c->inner_evals;
            if (ls.due & kDueM) c->inner_evals++;
            inner_step(s, xr, vr, xw, vw, cnt, dt, kif * dt, q == k, ls, c->stream);
            spare = !spare;
        }
        c->prof_end(1, pe);
        rebuild_cells_fork(c);
        pe = c->prof_begin(0);
        outer_forces(s, c->outer_evals++, Dt, c->stream);
        c->k_outer = k;
        c->prof_end(0, pe);
        rebuild_lists(c);
        // the closing half kick waits for the next opening; a series row due after this
        // step takes its row sums in the same pass
        const bool row_due = sch->diag_every > 0 && (c->step + 1) % sch->diag_every == 0 &&
                             c->series_rows < c->desc.series_capacity;
        join_lists(c);
        c->step++;
        c->time += Dt;
        c->close_pending = true;
        c->close_h = 0.5 * Dt;
        if (row_due) {
            c->row_pending = true;
            c->row_time = c->time;
            c->row_k = k;
            c->row_index = c->series_rows++;
        }
        pe = c->prof_begin(4);
        if (s.P > 0) {
            features(s, c->ring, (int)(c->feat_rows % 64), c->feat_last, c->feat_scratch, c->close_h, c->stream);
            c->feat_rows++;
        }
        c->prof_end(4, pe);
        c->since_infer++;
        if (sch->mode == 1 && k_force == 0 && c->feat_rows >= 64 && c->since_infer >= c->hold_now) {
            int32_t kk = 4, hh = 16;
            int fb = 0;
            aimts_status st = ctrl_infer_ring(c->ctrl, s, c->ring, (int)(c->feat_rows % 64), &kk, &hh, &fb, c->stream);
            if (st) return c->fail(st, "controller inference failed");
            c->inferences++;
            c->fallbacks += fb;
            c->k_now = sch->k_max > 0 && kk > sch->k_max ? sch->k_max : kk;
            c->hold_now = hh;
            c->since_infer = 0;
            // three-level scheme: the platelets' sublevels from their own predictions
            // (Table 2, rows 5-6)
            if (s.nlev == 3) levels_from_ratios(s, c->ctrl.pratio, c->ctrl.decision, sch->k_max, c->stream);
        } else if (sch->mode == 1 && c->feat_rows < 64) {
            c->k_now = 4;  // fallback ratio until a full window exists
        }
        return AIMTS_OK;
    };
    auto read_errors = [&](uint32_t *ew) -> aimts_status {
        flush_close(c);
        aimts_status st = sync_and_check(c, "step");
        c->prof_collect();
        if (st) return st;
        return d2h(c, ew, s.err, 3 * sizeof(uint32_t));
    };
    auto unstable = [&](const uint32_t *ew) -> aimts_status {
        c->failed = true;
        std::string why = err_text(ew[0]);
        char buf[160];
        if (ew[0] & kErrSkin) {
            std::snprintf(buf, sizeof buf, " member displacement sum %.4g > skin %.4g;", (double)bits_float(ew[1]),
                          s.skin);
            why += buf;
        }
        if (ew[0] & kErrSkinBead) {
            std::snprintf(buf, sizeof buf, " bead displacement sum %.4g > skin_bead %.4g;", (double)bits_float(ew[2]),
                          s.skin_bead);
            why += buf;
        }
        return c->fail(AIMTS_E_UNSTABLE, "instability within outer steps up to %lld:%s", (long long)c->step,
                       why.c_str());
    };
    uint32_t ew[3] = {0, 0, 0};
    aimts_status st;
    if (sch->rollback == 0) {
        for (int64_t n = 0; n < n_outer; ++n)
            if ((st = outer_step())) return st;
        if ((st = read_errors(ew))) return st;
        return ew[0] ? unstable(ew) : AIMTS_OK;
    }
    // Segments of `rollback` outer steps from a device checkpoint of the particle arrays.
    // A segment that fails its stability checks is rolled back and run again at half its
    // largest ratio (4 after 8, the controller's fallback ratio), with forces recomputed
    // at the restored state, and halved again while it fails, down to one rerun at ratio
    // 1 (with fresh random numbers, as every rerun); a failure there ends the call.
    const int64_t N = s.N;
    for (int64_t done = 0; done < n_outer;) {
        const int64_t seg = std::min<int64_t>(sch->rollback, n_outer - done);
        (void)hipMemcpyAsync(c->ck_x, s.x, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->stream);
        (void)hipMemcpyAsync(c->ck_v, s.v, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->stream);
        (void)hipMemcpyAsync(c->ck_id, s.id, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, c->stream);
        const int64_t step0 = c->step, series0 = c->series_rows, feat0 = c->feat_rows;
        const double time0 = c->time;
        k_seen = 0;
        for (int64_t n = 0; n < seg; ++n)
            if ((st = outer_step())) return st;
        if ((st = read_errors(ew))) return st;
        // a failed segment is rerun at half its largest ratio, and again at half of that
        // while it keeps failing, down to one rerun at ratio 1; a failure there ends the call
        int32_t kf = k_seen, reruns_at_1 = 0;
        while (ew[0] & (kErrSkin | kErrSkinBead | kErrNonFinite)) {
            if (kf > 1) kf = std::max(1, kf / 2);
            // three-level scheme: a power of two, so that the interface ratio divides it
            if (s.nlev == 3)
                while (kf & (kf - 1)) kf &= kf - 1;
            if (kf == 1 && reruns_at_1++ == 1) break;
            (void)hipMemcpyAsync(s.x, c->ck_x, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->stream);
            (void)hipMemcpyAsync(s.v, c->ck_v, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, c->stream);
            (void)hipMemcpyAsync(s.id, c->ck_id, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, c->stream);
            // derived state as after aimts_set_state (member marks are clear after every
            // completed rebuild); the random-number counters keep advancing
            fill_i32(s.mos, -1, N, c->stream);
            fill_i32((int32_t *)s.err, 0, 4, c->stream);
            fill_i32((int32_t *)s.maxdisp, 0, 4, c->stream);
            fill_i32((int32_t *)s.dmax, 0, s.cap_members, c->stream);
            fill_i32((int32_t *)s.dpart, 0, 4 * dpart_entries(s.nb, s.cap_members), c->stream);
            fill_f64(s.fi, 0.0, 3 * s.nlev * s.cap_members, c->stream);
            rebuild_cells_fork(c);
            outer_forces(s, c->outer_evals++, kf * dt, c->stream);
            c->k_outer = kf;
            rebuild_lists(c);
            join_lists(c);
            inner_forces(s, c->inner_evals++, interface_ratio(c, kf) * dt, c->stream);
            c->step = step0;
            c->time = time0;
            c->series_rows = series0;
            c->feat_rows = feat0;
            c->rollbacks++;
            k_force = kf;
            for (int64_t n = 0; n < seg; ++n)
                if ((st = outer_step())) return st;
            k_force = 0;
            // the controller keeps the fallback ratio for its current hold, then decides again
            if (sch->mode == 1) c->k_now = kf;
            c->since_infer = 0;
            if ((st = read_errors(ew))) return st;
        }
        if (ew[0]) return unstable(ew);
        done += seg;
    }
    return AIMTS_OK;
}

aimts_status aimts_get_state(aimts_ctx *c, double *x, double *v)
{
    if (!c) return AIMTS_E_INVALID;
    if (!c->have_state) return c->fail(AIMTS_E_STATE, "no state set");
    const int64_t N = c->s.N;
    std::vector<double> xs(3 * N), vs(3 * N);
    std::vector<uint32_t> ids(N);
    aimts_status st;
    if ((st = d2h(c, ids.data(), c->s.id, sizeof(uint32_t) * N))) return st;
    if (x && (st = d2h(c, xs.data(), c->s.x, sizeof(double) * 3 * N))) return st;
    if (v && (st = d2h(c, vs.data(), c->s.v, sizeof(double) * 3 * N))) return st;
    for (int64_t t = 0; t < N; ++t) {
        const int64_t i = ids[t];
        for (int k = 0; k < 3; ++k) {
            if (x) x[3 * i + k] = xs[k * N + t];
            if (v) v[3 * i + k] = vs[k * N + t];
        }
    }
    return AIMTS_OK;
}

aimts_status aimts_get_forces(aimts_ctx *c, double *f_outer, double *f_inner)
{
    if (!c) return AIMTS_E_INVALID;
    if (!c->have_forces) return c->fail(AIMTS_E_STATE, "no forces computed");
    Dev &s = c->s;
    const int64_t N = s.N, C = s.cap_members;
    std::vector<uint32_t> ids(N);
    aimts_status st;
    if ((st = d2h(c, ids.data(), s.id, sizeof(uint32_t) * N))) return st;
    if (f_outer) {
        std::vector<double> fo(3 * N);
        if (s.fp32) {
            std::vector<float> ff(3 * N);
            if ((st = d2h(c, ff.data(), s.fo, sizeof(float) * 3 * N))) return st;
            for (int64_t q = 0; q < 3 * N; ++q) fo[q] = ff[q];
        } else if ((st = d2h(c, fo.data(), s.fo, sizeof(double) * 3 * N))) {
            return st;
        }
        for (int64_t t = 0; t < N; ++t)
            for (int k = 0; k < 3; ++k) f_outer[3 * ids[t] + k] = fo[k * N + t];
    }
    if (f_inner) {
        std::memset(f_inner, 0, sizeof(double) * 3 * N);
        int32_t nm = 0;
        if ((st = d2h(c, &nm, s.n_members, sizeof nm))) return st;
        if (nm > 0) {
            std::vector<int32_t> ms(nm);
            std::vector<double> fi(3 * (size_t)s.nlev * C);
            if ((st = d2h(c, ms.data(), s.member_slot, sizeof(int32_t) * nm))) return st;
            if ((st = d2h(c, fi.data(), s.fi, sizeof(double) * fi.size()))) return st;
            // three-level mode: the sum of the groups M, P1, P2 at their last evaluation
            for (int32_t m = 0; m < nm; ++m)
                for (int k = 0; k < 3; ++k) {
                    double a = fi[k * C + m];
                    for (int l = 1; l < s.nlev; ++l) a += fi[(3 * l + k) * C + m];
                    f_inner[3 * ids[ms[m]] + k] = a;
                }
        }
    }
    return AIMTS_OK;
}

aimts_status aimts_get_diag(aimts_ctx *c, int32_t want_energy, aimts_diag *d, float *feat)
{
    if (!c || !d) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (!c->have_state) return c->fail(AIMTS_E_STATE, "no state set");
    if (!c->have_forces && (want_energy || feat)) return c->fail(AIMTS_E_STATE, "compute forces first");
    std::memset(d, 0, sizeof *d);
    record_thermo(c, c->thermo_out);
    if (want_energy) energy(c->s, c->energy_partial, c->energy_out, c->stream);
    if (feat && c->s.P > 0) features(c->s, nullptr, 0, c->feat_last, c->feat_scratch, 0.0, c->stream);
    aimts_status st = sync_and_check(c, "get_diag");
    if (st) return st;
    double th[kSeriesCols];
    if ((st = d2h(c, th, c->thermo_out, sizeof th))) return st;
    d->step = c->step;
    d->time = c->time;
    d->ke = th[1];
    d->T = th[2];
    d->T_pec = th[3];
    d->p[0] = th[4];
    d->p[1] = th[5];
    d->p[2] = th[6];
    if (want_energy) {
        double e[6];
        if ((st = d2h(c, e, c->energy_out, sizeof e))) return st;
        for (int q = 0; q < 5; ++q) d->pe[q] = e[q];
        d->virial = e[5];
        d->energy_valid = 1;
    }
    if (feat && c->s.P > 0 && (st = d2h(c, feat, c->feat_last, sizeof(float) * 8 * c->s.P))) return st;
    d->k = c->k_now;
    d->hold = c->hold_now;
    d->fallbacks = c->fallbacks;
    d->rollbacks = c->rollbacks;
    d->inferences = c->inferences;
    uint32_t flags = 0;
    if ((st = d2h(c, &flags, c->s.err, sizeof flags))) return st;
    d->error_flags = flags;
    int32_t nm = 0, np = 0, nq = 0;
    if ((st = d2h(c, &nm, c->s.n_members, sizeof nm))) return st;
    if ((st = d2h(c, &np, c->s.pair_off + c->s.cap_members, sizeof np))) return st;
    if ((st = d2h(c, &nq, c->ib.queue, sizeof nq))) return st;
    d->inner_members = nm;
    d->inner_pairs = np;
    d->rescanned = nq;
    return AIMTS_OK;
}

aimts_status aimts_get_series(aimts_ctx *c, double *rows, int64_t max_rows, int64_t *count)
{
    if (!c || !count || max_rows < 0 || (max_rows > 0 && !rows)) return AIMTS_E_INVALID;
    *count = c->series_rows;
    const int64_t n = std::min<int64_t>(max_rows, c->series_rows);
    return d2h(c, rows, c->series, sizeof(double) * kSeriesCols * n);
}

aimts_status aimts_get_feature_window(aimts_ctx *c, float *window)
{
    if (!c || !window) return AIMTS_E_INVALID;
    const int64_t P = c->s.P;
    if (P == 0 || c->feat_rows < 64) return c->fail(AIMTS_E_STATE, "fewer than 64 feature rows recorded");
    std::vector<float> ring(P * 64 * 8);
    aimts_status st = d2h(c, ring.data(), c->ring, sizeof(float) * ring.size());
    if (st) return st;
    const int64_t head = c->feat_rows % 64;  // oldest row
    for (int64_t p = 0; p < P; ++p)
        for (int64_t r = 0; r < 64; ++r)
            std::memcpy(&window[(p * 64 + r) * 8], &ring[(p * 64 + (head + r) % 64) * 8], sizeof(float) * 8);
    return AIMTS_OK;
}

// ---- checkpoint and resume ----
// Blob layout: CkptHeader, then x, v ([N][3] float64, particle order), the outer force
// ([N][3], float32 or float64 as the context computes it, particle order), the inner
// force of every member (n_members records of particle index and [3] float64), the
// series rows, the feature ring [P][64][8] and the last features [P][8] (float32), and,
// when the context holds controller weights, the float32 master parameters and both
// Adam moments.
namespace {

constexpr char kCkptMagic[8] = {'A', 'I', 'M', 'T', 'S', 'C', 'K', '1'};

struct CkptHeader {
    char magic[8];
    uint64_t param_hash;
    int64_t N, nb, P, n_members, series_rows, feat_rows, step, np;
    uint64_t outer_evals, inner_evals;
    double time;
    int32_t fp32, k_now, hold_now, since_infer, fallbacks, inferences, rollbacks, have_weights;
    int64_t adam_t[2];
    int32_t nlev, k_if, k_sub, k_outer;
};


// FNV-1a over the system description and every force-field, external and mass
// parameter: a checkpoint only loads into a context set up the same way.
uint64_t param_hash(const aimts_ctx *c)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t q = 0; q < n; ++q) {
            h ^= b[q];
            h *= 1099511628211ull;
        }
    };
    const aimts_system_desc &d = c->desc;
    mix(d.lo, sizeof d.lo);
    mix(d.L, sizeof d.L);
    mix(d.periodic, sizeof d.periodic);
    mix(&d.force_precision, sizeof d.force_precision);
    const int64_t counts[7] = {d.n_fluid, d.n_wall, d.n_bead, d.n_platelet, d.n_bond, d.n_angle, d.n_morse};
    mix(counts, sizeof counts);
    mix(&d.seed, sizeof d.seed);
    const Dev &s = c->s;
    const double par[] = {s.m[0], s.m[1], s.m[2], s.a, s.gamma, s.sigma, s.rc, s.lj_eps, s.lj_sig2, s.lj_rc2,
                          s.r_excl2, s.gpf, s.spf, s.rc_pf, s.kb, s.ka, s.mD, s.ma, s.mr0, s.g[0], s.g[1], s.g[2],
                          s.wall_lo, s.wall_hi};
    mix(par, sizeof par);
    mix(&s.wall_axis, sizeof s.wall_axis);
    if (s.agg_on) {
        const double agg[] = {s.agg_D, s.agg_a, s.agg_r0, s.agg_fA, s.agg_rc2};
        mix(agg, sizeof agg);
    }
    return h;
}

struct CkptSizes {
    size_t header, x, fo, members, series, ring, ctrl, levels, total;
};

// one member record: particle index (8 bytes with padding), then 3 nlev float64 forces
size_t member_record_bytes(const Dev &s) { return 8 + sizeof(double) * 3 * (size_t)s.nlev; }

CkptSizes ckpt_sizes(const aimts_ctx *c, int64_t nm)
{
    const Dev &s = c->s;
    CkptSizes z{};
    z.header = sizeof(CkptHeader);
    z.x = sizeof(double) * 3 * (size_t)s.N;
    z.fo = (s.fp32 ? sizeof(float) : sizeof(double)) * 3 * (size_t)s.N;
    z.members = member_record_bytes(s) * (size_t)nm;
    z.series = sizeof(double) * kSeriesCols * (size_t)c->series_rows;
    z.ring = sizeof(float) * (size_t)s.P * (64 * 8 + 8);
    z.ctrl = c->ctrl.have_weights ? sizeof(float) * 3 * (size_t)c->ctrl.np : 0;
    z.levels = s.nlev == 3 ? sizeof(int32_t) * (size_t)s.P : 0;  // the platelets' sublevels
    z.total = z.header + 2 * z.x + z.fo + z.members + z.series + z.ring + z.ctrl + z.levels;
    return z;
}

aimts_status member_count(aimts_ctx *c, int32_t *nm)
{
    *nm = 0;
    return d2h(c, nm, c->s.n_members, sizeof *nm);
}

}  // namespace

aimts_status aimts_checkpoint_size(aimts_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return AIMTS_E_INVALID;
    if (!c->have_state || !c->have_forces) return c->fail(AIMTS_E_STATE, "no state and forces to checkpoint");
    int32_t nm = 0;
    aimts_status st = member_count(c, &nm);
    if (st) return st;
    *bytes = ckpt_sizes(c, nm).total;
    return AIMTS_OK;
}

aimts_status aimts_save_checkpoint(aimts_ctx *c, void *buf, size_t bytes)
{
    if (!c || !buf) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (c->failed) return c->fail(AIMTS_E_STATE, "context failed earlier; nothing consistent to checkpoint");
    if (!c->have_state || !c->have_forces) return c->fail(AIMTS_E_STATE, "no state and forces to checkpoint");
    Dev &s = c->s;
    const int64_t N = s.N, C = s.cap_members;
    int32_t nm = 0;
    aimts_status st = member_count(c, &nm);
    if (st) return st;
    const CkptSizes z = ckpt_sizes(c, nm);
    if (bytes < z.total) return c->fail(AIMTS_E_INVALID, "checkpoint buffer holds %zu bytes, %zu needed", bytes, z.total);
    char *out = static_cast<char *>(buf);
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, sizeof h.magic);
    h.param_hash = param_hash(c);
    h.N = N;
    h.nb = s.nb;
    h.P = s.P;
    h.n_members = nm;
    h.series_rows = c->series_rows;
    h.feat_rows = c->feat_rows;
    h.step = c->step;
    h.np = c->ctrl.np;
    h.outer_evals = c->outer_evals;
    h.inner_evals = c->inner_evals;
    h.time = c->time;
    h.fp32 = s.fp32;
    h.k_now = c->k_now;
    h.hold_now = c->hold_now;
    h.since_infer = c->since_infer;
    h.fallbacks = c->fallbacks;
    h.inferences = c->inferences;
    h.rollbacks = c->rollbacks;
    h.have_weights = c->ctrl.have_weights ? 1 : 0;
    h.adam_t[0] = c->ctrl.adam_t[0];
    h.adam_t[1] = c->ctrl.adam_t[1];
    h.nlev = s.nlev;
    h.k_if = c->k_if;
    h.k_sub = c->k_sub;
    h.k_outer = c->k_outer;
    std::memcpy(out, &h, sizeof h);
    size_t off = z.header;
    // state in particle order
    double *x = reinterpret_cast<double *>(out + off);
    double *v = reinterpret_cast<double *>(out + off + z.x);
    if ((st = aimts_get_state(c, x, v))) return st;
    off += 2 * z.x;
    std::vector<uint32_t> ids(N);
    if ((st = d2h(c, ids.data(), s.id, sizeof(uint32_t) * N))) return st;
    if (s.fp32) {
        std::vector<float> ff(3 * N);
        if ((st = d2h(c, ff.data(), s.fo, sizeof(float) * 3 * N))) return st;
        float *fo = reinterpret_cast<float *>(out + off);
        for (int64_t t = 0; t < N; ++t)
            for (int k = 0; k < 3; ++k) fo[3 * ids[t] + k] = ff[k * N + t];
    } else {
        std::vector<double> ff(3 * N);
        if ((st = d2h(c, ff.data(), s.fo, sizeof(double) * 3 * N))) return st;
        double *fo = reinterpret_cast<double *>(out + off);
        for (int64_t t = 0; t < N; ++t)
            for (int k = 0; k < 3; ++k) fo[3 * ids[t] + k] = ff[k * N + t];
    }
    off += z.fo;
    if (nm > 0) {
        std::vector<int32_t> ms(nm);
        std::vector<double> fi(3 * (size_t)s.nlev * C);
        if ((st = d2h(c, ms.data(), s.member_slot, sizeof(int32_t) * nm))) return st;
        if ((st = d2h(c, fi.data(), s.fi, sizeof(double) * fi.size()))) return st;
        const size_t rb = member_record_bytes(s);
        for (int32_t m = 0; m < nm; ++m) {
            char *r = out + off + rb * m;
            const uint64_t id = ids[ms[m]];
            std::memcpy(r, &id, 8);
            for (int k = 0; k < 3 * s.nlev; ++k) std::memcpy(r + 8 + 8 * k, &fi[k * C + m], 8);
        }
    }
    off += z.members;
    if (z.series && (st = d2h(c, out + off, c->series, z.series))) return st;
    off += z.series;
    if (s.P > 0) {
        if ((st = d2h(c, out + off, c->ring, sizeof(float) * s.P * 64 * 8))) return st;
        if ((st = d2h(c, out + off + sizeof(float) * s.P * 64 * 8, c->feat_last, sizeof(float) * s.P * 8))) return st;
    }
    off += z.ring;
    if (z.ctrl) {
        const size_t one = sizeof(float) * c->ctrl.np;
        if ((st = d2h(c, out + off, c->ctrl.master, one))) return st;
        if ((st = d2h(c, out + off + one, c->ctrl.adam_m, one))) return st;
        if ((st = d2h(c, out + off + 2 * one, c->ctrl.adam_v, one))) return st;
    }
    off += z.ctrl;
    if (z.levels && (st = d2h(c, out + off, s.plev, z.levels))) return st;
    return AIMTS_OK;
}

aimts_status aimts_load_checkpoint(aimts_ctx *c, const void *buf, size_t bytes)
{
    if (!c || !buf) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    Dev &s = c->s;
    const int64_t N = s.N, C = s.cap_members;
    CkptHeader h;
    if (bytes < sizeof h) return c->fail(AIMTS_E_INVALID, "checkpoint too short");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kCkptMagic, sizeof h.magic) != 0) return c->fail(AIMTS_E_INVALID, "not a checkpoint");
    if (h.N != N || h.nb != s.nb || h.P != s.P || h.fp32 != s.fp32 || h.nlev != s.nlev ||
        h.param_hash != param_hash(c))
        return c->fail(AIMTS_E_INVALID, "checkpoint is of another system, precision or parameter set");
    if (h.series_rows < 0 || h.series_rows > c->desc.series_capacity)
        return c->fail(AIMTS_E_INVALID, "checkpoint holds %lld series rows, capacity is %lld", (long long)h.series_rows,
                       (long long)c->desc.series_capacity);
    if (h.n_members < 0 || h.n_members > C) return c->fail(AIMTS_E_INVALID, "checkpoint member count out of range");
    if (h.have_weights && h.np != c->ctrl.np) return c->fail(AIMTS_E_INVALID, "checkpoint controller size differs");
    const int64_t saved_rows = c->series_rows;
    c->series_rows = h.series_rows;
    const bool had_weights = c->ctrl.have_weights;
    c->ctrl.have_weights = h.have_weights != 0;
    const CkptSizes z = ckpt_sizes(c, h.n_members);
    c->series_rows = saved_rows;
    c->ctrl.have_weights = had_weights;
    if (bytes < z.total) return c->fail(AIMTS_E_INVALID, "checkpoint truncated: %zu of %zu bytes", bytes, z.total);
    const char *in = static_cast<const char *>(buf);
    size_t off = z.header;
    const double *x = reinterpret_cast<const double *>(in + off);
    const double *v = reinterpret_cast<const double *>(in + off + z.x);
    aimts_status st = aimts_set_state(c, x, v);
    if (st) return st;
    off += 2 * z.x;
    // the cell sort and the platelet lists of the saved state (they depend on the
    // positions only, so they come out as the saving context had them)
    if (s.nb > 0 && (st = check_reach(c))) return st;
    rebuild_cells_fork(c);
    rebuild_lists(c);
    join_lists(c);
    if ((st = sync_and_check(c, "load_checkpoint"))) return st;
    std::vector<uint32_t> ids(N);
    if ((st = d2h(c, ids.data(), s.id, sizeof(uint32_t) * N))) return st;
    std::vector<int64_t> slot_of(N);
    for (int64_t t = 0; t < N; ++t) slot_of[ids[t]] = t;
    if (s.fp32) {
        std::vector<float> ff(3 * N);
        const float *fo = reinterpret_cast<const float *>(in + off);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) ff[k * N + slot_of[i]] = fo[3 * i + k];
        if ((st = h2d(c, s.fo, ff.data(), sizeof(float) * 3 * N))) return st;
    } else {
        std::vector<double> ff(3 * N);
        const double *fo = reinterpret_cast<const double *>(in + off);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) ff[k * N + slot_of[i]] = fo[3 * i + k];
        if ((st = h2d(c, s.fo, ff.data(), sizeof(double) * 3 * N))) return st;
    }
    off += z.fo;
    int32_t nm = 0;
    if ((st = member_count(c, &nm))) return st;
    if (nm != h.n_members) {
        c->have_forces = false;
        return c->fail(AIMTS_E_INVALID, "rebuilt platelet lists hold %d members, the checkpoint %lld", nm,
                       (long long)h.n_members);
    }
    if (nm > 0) {
        std::vector<int32_t> ms(nm);
        if ((st = d2h(c, ms.data(), s.member_slot, sizeof(int32_t) * nm))) return st;
        std::vector<double> fi(3 * (size_t)s.nlev * C, 0.0);
        const size_t rb = member_record_bytes(s);
        for (int32_t m = 0; m < nm; ++m) {
            const char *r = in + off + rb * m;
            uint64_t id = 0;
            std::memcpy(&id, r, 8);
            if (id != ids[ms[m]]) {
                c->have_forces = false;
                return c->fail(AIMTS_E_INVALID, "rebuilt platelet member %d differs from the checkpoint's", m);
            }
            for (int k = 0; k < 3 * s.nlev; ++k) std::memcpy(&fi[k * C + m], r + 8 + 8 * k, 8);
        }
        if ((st = h2d(c, s.fi, fi.data(), sizeof(double) * fi.size()))) return st;
    }
    off += z.members;
    if (z.series && (st = h2d(c, c->series, in + off, z.series))) return st;
    off += z.series;
    if (s.P > 0) {
        if ((st = h2d(c, c->ring, in + off, sizeof(float) * s.P * 64 * 8))) return st;
        if ((st = h2d(c, c->feat_last, in + off + sizeof(float) * s.P * 64 * 8, sizeof(float) * s.P * 8))) return st;
    }
    off += z.ring;
    if (z.ctrl) {
        const size_t one = sizeof(float) * c->ctrl.np;
        if ((st = h2d(c, c->ctrl.master, in + off, one))) return st;
        ctrl_after_set(c->ctrl, c->stream);  // bfloat16 copy; clears the moments and step counters
        if ((st = h2d(c, c->ctrl.adam_m, in + off + one, one))) return st;
        if ((st = h2d(c, c->ctrl.adam_v, in + off + 2 * one, one))) return st;
        c->ctrl.adam_t[0] = h.adam_t[0];
        c->ctrl.adam_t[1] = h.adam_t[1];
    }
    off += z.ctrl;
    if (z.levels) {
        if ((st = h2d(c, s.plev, in + off, z.levels))) return st;
        levels_to_beads(s, c->stream);
    }
    if ((st = sync_and_check(c, "load_checkpoint"))) return st;
    c->outer_evals = h.outer_evals;
    c->inner_evals = h.inner_evals;
    c->step = h.step;
    c->time = h.time;
    c->series_rows = h.series_rows;
    c->feat_rows = h.feat_rows;
    c->k_now = h.k_now;
    c->hold_now = h.hold_now;
    c->since_infer = h.since_infer;
    c->fallbacks = h.fallbacks;
    c->inferences = h.inferences;
    c->rollbacks = h.rollbacks;
    c->k_if = h.k_if;
    c->k_sub = h.k_sub;
    c->k_outer = h.k_outer;
    c->close_pending = c->row_pending = false;  // a checkpoint holds the synchronised state
    c->have_forces = true;
    return AIMTS_OK;
}

aimts_status aimts_profile(aimts_ctx *c, int32_t mask)
{
    if (!c) return AIMTS_E_INVALID;
    if (mask < 0 || mask >= (1 << kProfPhases))
        return c->fail(AIMTS_E_INVALID, "profile mask must lie in [0, %d]", (1 << kProfPhases) - 1);
    c->prof_mask = mask;
    for (int q = 0; q < kProfPhases; ++q) {
        c->prof_ms[q] = 0.0;
        c->prof_n[q] = 0;
    }
    return AIMTS_OK;
}

aimts_status aimts_get_profile(aimts_ctx *c, double *ms, int64_t *count)
{
    if (!c || !ms || !count) return AIMTS_E_INVALID;
    for (int q = 0; q < kProfPhases; ++q) {
        ms[q] = c->prof_ms[q];
        count[q] = c->prof_n[q];
    }
    return AIMTS_OK;
}

aimts_status aimts_get_paper_features(aimts_ctx *c, double flow_r, double *out)
{
    if (!c || !out) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (!c->have_state || !c->have_forces) return c->fail(AIMTS_E_STATE, "call aimts_compute_forces first");
    if (!(flow_r > 0.0) || !std::isfinite(flow_r)) return c->fail(AIMTS_E_INVALID, "flow_r must be > 0");
    const Dev &s = c->s;
    for (int k = 0; k < 3; ++k)
        if (s.per[k] && 2 * (int)std::ceil(flow_r / s.side[k]) + 1 > s.nc[k])
            return c->fail(AIMTS_E_INVALID, "flow_r %g spans more cells than the box has along axis %d", flow_r, k);
    if (s.P == 0) return AIMTS_OK;
    flush_close(c);
    paper_features(s, flow_r, c->paper_feat, c->stream);
    aimts_status st = sync_and_check(c, "get_paper_features");
    if (st) return st;
    return d2h(c, out, c->paper_feat, sizeof(double) * 6 * s.P);
}

aimts_status aimts_stress_sample(aimts_ctx *c)
{
    if (!c) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (!c->have_state || !c->have_forces) return c->fail(AIMTS_E_STATE, "call aimts_compute_forces first");
    if (c->s.nb == 0) return AIMTS_OK;
    flush_close(c);
    if (c->stress_n == 0) fill_f64(c->stress_sum, 0.0, c->s.nb, c->stream);
    bead_stress(c->s, c->stress_sum, c->stream);
    c->stress_n++;
    return AIMTS_OK;
}

aimts_status aimts_get_stress(aimts_ctx *c, double *mean, int64_t *samples, int32_t reset)
{
    if (!c) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    aimts_status st = sync_and_check(c, "get_stress");
    if (st) return st;
    if (samples) *samples = c->stress_n;
    if (mean && c->s.nb > 0) {
        if (c->stress_n == 0) return c->fail(AIMTS_E_STATE, "no stress samples");
        std::vector<double> h(c->s.nb);
        if ((st = d2h(c, h.data(), c->stress_sum, sizeof(double) * c->s.nb))) return st;
        for (int64_t b = 0; b < c->s.nb; ++b) mean[b] = h[b] / (double)c->stress_n;
    }
    if (reset) c->stress_n = 0;
    return AIMTS_OK;
}

// ---- controller entry points ----
aimts_status aimts_ctrl_num_params(int64_t *n)
{
    if (!n) return AIMTS_E_INVALID;
    *n = ctrl_num_params();
    return AIMTS_OK;
}

aimts_status aimts_ctrl_set_weights(aimts_ctx *c, const float *params, int64_t n)
{
    if (!c || !params) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (n != ctrl_num_params()) return c->fail(AIMTS_E_INVALID, "expected %lld parameters", (long long)ctrl_num_params());
    for (int64_t q = 0; q < n; ++q)
        if (!std::isfinite(params[q])) return c->fail(AIMTS_E_INVALID, "parameters must be finite");
    aimts_status st = h2d(c, c->ctrl.master, params, sizeof(float) * n);
    if (st) return st;
    ctrl_after_set(c->ctrl, c->stream);
    return sync_and_check(c, "ctrl_set_weights");
}

aimts_status aimts_ctrl_get_weights(aimts_ctx *c, float *params, int64_t n)
{
    if (!c || !params) return AIMTS_E_INVALID;
    if (n != ctrl_num_params()) return c->fail(AIMTS_E_INVALID, "expected %lld parameters", (long long)ctrl_num_params());
    return d2h(c, params, c->ctrl.master, sizeof(float) * n);
}

aimts_status aimts_ctrl_forward(aimts_ctx *c, const float *d_windows, int32_t batch, float *d_latent, float *d_logits)
{
    if (!c || !d_windows) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (batch < 1 || batch > c->ctrl.max_batch) return c->fail(AIMTS_E_INVALID, "batch must lie in [1, %d]", c->ctrl.max_batch);
    if (!c->ctrl.have_weights) return c->fail(AIMTS_E_STATE, "no controller weights");
    ctrl_forward(c->ctrl, d_windows, batch, c->stream, nullptr);
    ctrl_copy_outputs(c->ctrl, batch, d_latent, d_logits, c->stream);
    return sync_and_check(c, "ctrl_forward");
}

aimts_status aimts_ctrl_backward(aimts_ctx *c, const float *d_windows, const int32_t *d_labels, int32_t batch,
                                 int32_t phase, float *d_grads, float *loss)
{
    if (!c || !d_windows || !d_grads || !loss) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (batch < 1 || batch > c->ctrl.max_batch) return c->fail(AIMTS_E_INVALID, "batch must lie in [1, %d]", c->ctrl.max_batch);
    if (phase != 0 && phase != 1) return c->fail(AIMTS_E_INVALID, "phase must be 0 or 1");
    if (phase == 1 && !d_labels) return c->fail(AIMTS_E_INVALID, "labels are required for phase 1");
    if (!c->ctrl.have_weights) return c->fail(AIMTS_E_STATE, "no controller weights");
    ctrl_forward(c->ctrl, d_windows, batch, c->stream, d_labels);
    ctrl_backward(c->ctrl, d_labels, batch, phase, c->stream);
    ctrl_copy_grads(c->ctrl, d_grads, c->stream);
    aimts_status st = sync_and_check(c, "ctrl_backward");
    if (st) return st;
    return d2h(c, loss, c->ctrl.loss, sizeof(float));
}

aimts_status aimts_ctrl_train_step(aimts_ctx *c, const float *d_windows, const int32_t *d_labels, int32_t batch,
                                   int32_t phase, float lr, float *loss)
{
    if (!c || !d_windows || !loss) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (batch < 1 || batch > c->ctrl.max_batch) return c->fail(AIMTS_E_INVALID, "batch must lie in [1, %d]", c->ctrl.max_batch);
    if (phase != 0 && phase != 1) return c->fail(AIMTS_E_INVALID, "phase must be 0 or 1");
    if (phase == 1 && !d_labels) return c->fail(AIMTS_E_INVALID, "labels are required for phase 1");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return c->fail(AIMTS_E_INVALID, "lr must be > 0");
    if (!c->ctrl.have_weights) return c->fail(AIMTS_E_STATE, "no controller weights");
    ctrl_forward(c->ctrl, d_windows, batch, c->stream, d_labels);
    ctrl_backward(c->ctrl, d_labels, batch, phase, c->stream);
    ctrl_adam(c->ctrl, phase, lr, c->stream);
    aimts_status st = sync_and_check(c, "ctrl_train_step");
    if (st) return st;
    return d2h(c, loss, c->ctrl.loss, sizeof(float));
}

aimts_status aimts_ctrl_infer(aimts_ctx *c, int32_t *k, int32_t *hold)
{
    if (!c || !k || !hold) return AIMTS_E_INVALID;
    clear_stale_hip_error();
    if (c->s.P == 0 || c->feat_rows < 64) return c->fail(AIMTS_E_STATE, "fewer than 64 feature rows recorded");
    if (!c->ctrl.have_weights) return c->fail(AIMTS_E_STATE, "no controller weights");
    int fb = 0;
    aimts_status st = ctrl_infer_ring(c->ctrl, c->s, c->ring, (int)(c->feat_rows % 64), k, hold, &fb, c->stream);
    if (st) return c->fail(st, "controller inference failed");
    return AIMTS_OK;
}

}  // extern "C"
