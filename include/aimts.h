/*
 * aimts.h -- C ABI of the MI355X (gfx950) engine for the DPD + CGMD multiple-time-
 * stepping hot path of "AI-aided multiscale modeling of physiologically-significant
 * blood clots" (Zhu et al., arXiv 2205.14121).
 *
 * What the library computes (paper sections in brackets):
 *   - a cell-list neighbour build by counting sort of all particles by cell
 *     [MSM pseudocode, Table 1, neighbour-list construction];
 *   - DPD conservative + dissipative + random pair forces between fluid and
 *     fluid/wall particles, the "outer" force group [Sec. 3.2, Eq. 1];
 *   - the platelet ("inner") force group: harmonic bonds and angles and WCA
 *     Lennard-Jones between beads [Eq. 2], WCA + dissipative + random forces
 *     between beads and fluid/wall particles [Eq. 3], Morse bonds between beads of
 *     different platelets [Eqs. 2 and 4];
 *   - a body force on the fluid and frozen-particle walls [Sec. 3.1];
 *   - two-group RESPA velocity Verlet: the inner group takes k steps of dt_inner
 *     inside every outer step of k * dt_inner [Sec. 3.3, Table 1];
 *   - thermodynamic diagnostics and eight dynamics features per platelet
 *     [Table 1, the step that computes and writes out platelet properties; Sec. 3.3];
 *   - the learned timestep controller: moving-average filter, GRU autoencoder and
 *     fully connected head that choose the MTS ratio and how long to hold it,
 *     with forward, backward and Adam kernels for training on the device
 *     [Sec. 3.3, Table 2].
 *
 * Conventions for every entry point:
 *   - Every call returns an aimts_status; AIMTS_OK is 0, errors are negative.
 *     aimts_last_error() returns a message for the last failed call on a context.
 *   - Argument checks run on the host before any device work; a failing check
 *     returns AIMTS_E_INVALID and leaves the context unchanged.
 *   - Particles are ordered fluid [0, n_fluid), wall [n_fluid, n_fluid + n_wall),
 *     bead [n_fluid + n_wall, N), beads grouped platelet by platelet.  Particle
 *     index i is its identity everywhere (random numbers are keyed on it).
 *   - Host arrays (plain pointers) are read or written during the call only; the
 *     caller keeps ownership.  Positions/velocities/forces are [N][3] float64 in
 *     particle order, whatever order the device keeps them in.
 *   - Device memory: the library allocates nothing.  The caller passes one device
 *     workspace of at least aimts_workspace_size() bytes (256-byte aligned) and a
 *     HIP stream; the device work of the context is queued on that stream, except
 *     most of the platelet-list rebuild, which runs on a stream the context owns,
 *     forked from the given stream after the cell sort and joined back into it
 *     within the same call (so that it overlaps the DPD kernel).  When a call returns, all of
 *     its work is ordered before later work on the given stream.  The workspace
 *     must outlive the context.  Calls that return host data synchronise the
 *     stream; others may return before the device finishes.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - After a device-detected instability (a non-finite velocity, or a position more
 *     than one cell outside the box at a rebuild; displacements in one
 *     outer step that could have let a pair of the platelet group come within range
 *     unseen, i.e. the largest path of a fluid particle outside the platelet list plus
 *     the largest displacement of a listed particle, or the two largest displacements
 *     of listed particles together, exceeding the skin, or the two largest bead
 *     displacements together exceeding skin_bead; a neighbour-list capacity
 *     overflow) aimts_step returns
 *     AIMTS_E_UNSTABLE and the context refuses further steps with AIMTS_E_STATE
 *     until aimts_set_state.
 */
#ifndef AIMTS_H
#define AIMTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AIMTS_OK = 0,
    AIMTS_E_INVALID = -1,     /* bad argument (message says which) */
    AIMTS_E_NOMEM = -2,       /* workspace too small */
    AIMTS_E_HIP = -3,         /* HIP runtime error (message has hipGetErrorString) */
    AIMTS_E_UNSTABLE = -4,    /* device-detected instability during aimts_step */
    AIMTS_E_STATE = -5,       /* call not allowed in the current state */
    AIMTS_E_UNSUPPORTED = -6  /* valid request this library does not implement */
} aimts_status;

typedef struct aimts_ctx aimts_ctx;

/* Static description of a system; fixes every device buffer size. */
typedef struct {
    double lo[3];              /* box origin */
    double L[3];               /* box lengths (> 0) */
    int32_t periodic[3];       /* 1: periodic along this axis */
    int32_t force_precision;   /* 0: all forces in float64;
                                  1: pair forces (outer DPD, bead-fluid/wall) in float32
                                     with float32 accumulation; separations are formed in
                                     float64 and rounded; state and integrator stay float64 */
    int64_t n_fluid, n_wall, n_bead; /* n_fluid + n_wall + n_bead <= 134,217,727 */
    int64_t n_platelet;
    int64_t n_bond, n_angle, n_morse;
    double cell_min;           /* smallest allowed cell side: the DPD cutoff */
    double skin;               /* extra reach of the platelet pair list (>= 0) */
    int64_t inner_pair_capacity; /* entries of the platelet pair list; 0: automatic,
                                    ceil(96 (cell_min + skin)^3) per bead */
    int64_t series_capacity;   /* rows of the diagnostics time series (may be 0) */
    int32_t ctrl_max_batch;    /* largest training/inference batch of the controller */
    int32_t angle_pass;        /* angle forces of an inner step: 0 or 1: every bead evaluates
                                  its own angle entries inside the inner force kernel (one
                                  launch per inner step); 2: one thread per angle in a launch
                                  of its own before it, gathered by the beads (a third of the
                                  angle arithmetic, one more launch: slower on the 2 M and
                                  100 M channels alike).  Both give bitwise identical forces */
    uint64_t seed;             /* key of the pair random numbers */
    double skin_bead;          /* extra reach of the bead-bead pair lists (>= 0, at most skin);
                                  0: min(skin, 0.5).  Beads move far less in one outer step
                                  than the fastest fluid particles, which set `skin` */
    int32_t three_level;       /* 1: workspace for the three-level scheme (aimts_set_levels) */
    int32_t reserved;          /* 0 */
} aimts_system_desc;

/* Bytes of device workspace needed for `desc`. */
aimts_status aimts_workspace_size(const aimts_system_desc *desc, size_t *bytes);

/* Create a context on the current HIP device.  `d_workspace` is device memory of
 * `bytes` >= aimts_workspace_size(desc); `hip_stream` is a hipStream_t (NULL: the
 * null stream).  Default parameters: all force constants 0, masses 1. */
aimts_status aimts_create(const aimts_system_desc *desc, void *d_workspace, size_t bytes, void *hip_stream,
                          aimts_ctx **out);
aimts_status aimts_destroy(aimts_ctx *ctx);
/* Message of the last failed call on ctx; with ctx == NULL, of the calling thread's last
 * failed aimts_create or aimts_ctrl_forward_static. */
const char *aimts_last_error(const aimts_ctx *ctx);

/* Positions x and velocities v, [N][3] float64 host arrays in particle order.
 * Positions must lie in the box (periodic axes wrap, walls clamp).  Resets the
 * step counter, the simulated time and a failed state; keeps the RNG counters. */
aimts_status aimts_set_state(aimts_ctx *ctx, const double *x, const double *v);

/* Masses of fluid, wall and bead particles (> 0). */
aimts_status aimts_set_masses(aimts_ctx *ctx, const double mass[3]);

/* DPD pair force of Eq. 1 between fluid-fluid and fluid-wall pairs, r < rc:
 * F_ij = [a w - gamma w^2 (e_ij . v_ij) + sigma w zeta_ij / sqrt(dt_outer)] e_ij,
 * w = 1 - r/rc, e_ij = (x_i - x_j)/r (minimum image), v_ij = v_i - v_j.
 * zeta_ij = zeta_ji ~ N(0,1): Philox4x32-10 (Salmon et al., SC'11) of counter
 * (min(i,j), max(i,j), c_lo, c_hi) and key (seed_lo, seed_hi ^ group), group 0,
 * c = number of outer evaluations so far; u1 = (w0 + 1/2) 2^-32,
 * u2 = (w1 + 1/2) 2^-32, zeta = sqrt(-2 ln u1) cos(2 pi u2).  rc <= cell_min. */
aimts_status aimts_set_dpd(aimts_ctx *ctx, double a, double gamma, double sigma, double rc);

/* WCA Lennard-Jones of Eq. 2, U = 4 eps [(sig/r)^12 - (sig/r)^6] + eps for
 * r < rc_lj (normally 2^(1/6) sig), between beads of different platelets, beads of
 * one platelet whose rest distance is >= r_excl, and beads and fluid/wall. */
aimts_status aimts_set_lj(aimts_ctx *ctx, double eps, double sig, double rc_lj, double r_excl);

/* Dissipative + random part of the platelet-fluid force of Eq. 3 (bead with fluid
 * or wall, r < rc_pf): the DPD terms above with (gamma_pf, sigma_pf, rc_pf), group
 * 1, c = number of inner evaluations so far, dt = dt_inner; no conservative DPD term. */
aimts_status aimts_set_interface(aimts_ctx *ctx, double gamma_pf, double sigma_pf, double rc_pf);

/* Platelet topology: body[n_bead] platelet index of each bead (beads of a platelet
 * contiguous, platelets numbered 0..n_platelet-1 in order), rest[n_bead][3] rest-mesh
 * coordinates (used for the same-platelet exclusion), area[n_platelet] rest areas. */
aimts_status aimts_set_platelets(aimts_ctx *ctx, const int32_t *body, const double *rest, const double *area);

/* Harmonic bonds U = k (r - r0_b)^2 of Eq. 2; ij[n][2] bead particle indices. n == desc.n_bond. */
aimts_status aimts_set_bonds(aimts_ctx *ctx, int64_t n, const int32_t *ij, const double *r0, double k);

/* Harmonic angles U = k (theta - th0_a)^2 of Eq. 2; ijk[n][3] = (end, vertex, end). */
aimts_status aimts_set_angles(aimts_ctx *ctx, int64_t n, const int32_t *ijk, const double *th0, double k);

/* Morse bonds U = D [e^{-2a(r-r0)} - 2 e^{-a(r-r0)}] (Eq. 2 form, inter-platelet
 * binding of Eq. 4); ij[n][2] bead particle indices. */
aimts_status aimts_set_morse(aimts_ctx *ctx, int64_t n, const int32_t *ij, double D, double a, double r0);

/* Inter-platelet aggregation of Eq. 4 (Sec. 3.2): every pair of beads of different
 * platelets closer than rc interacts through the non-bonded Morse potential
 * U = D [e^{-2a(r-r0)} - 2 e^{-a(r-r0)}] (Eq. 2's form with eps = D, alpha = 2 a r0) plus
 * the receptor term, a force fA (1 - r/r0) along e_ij (a linear spring about r0).  Both
 * are cut at rc; the reported energy is shifted to 0 there.  rc = 0 turns the term off
 * (the default).  The bead-bead lists then reach rc + skin_bead for beads of other
 * platelets.  In the three-level scheme the term belongs to the aggregating group P2.
 * Errors: AIMTS_E_INVALID for non-finite values, D < 0, a <= 0, r0 <= 0, rc < 0, rc > 0
 * without beads, or a reach of more cells than the box or the list builder allows. */
aimts_status aimts_set_aggregation(aimts_ctx *ctx, double D, double a, double r0, double fA, double rc);

/* Body force g on every fluid particle (F^E of Eq. 1); walls: wall_axis (0..2 or -1
 * for none) along which mobile particles crossing wall_lo / wall_hi are reflected
 * with their whole velocity reversed.  The wall axis must not be periodic. */
aimts_status aimts_set_external(aimts_ctx *ctx, const double g[3], int32_t wall_axis, double wall_lo,
                                double wall_hi);

/* Numbers of outer and inner force evaluations done so far (RNG counters). */
aimts_status aimts_set_counters(aimts_ctx *ctx, uint64_t outer_evals, uint64_t inner_evals);
aimts_status aimts_get_counters(aimts_ctx *ctx, uint64_t *outer_evals, uint64_t *inner_evals);

/* Evaluate both force groups at the current state: the outer group with
 * dt_outer = k * dt_inner in its random term and the inner group with dt_inner,
 * at the current counters, then advance each counter by one.  Required once after
 * aimts_set_state and before the first aimts_step. */
aimts_status aimts_compute_forces(aimts_ctx *ctx, double dt_inner, int32_t k);

typedef struct {
    double dt_inner;      /* inner step; the outer step is k * dt_inner */
    int32_t k;            /* MTS ratio (1..64); mode 1: ratio before the first inference */
    int32_t mode;         /* 0: fixed ratio; 1: learned controller */
    int32_t diag_every;   /* append a diagnostics row every this many outer steps (0: never) */
    int32_t k_max;        /* mode 1: largest ratio the controller may set (0: no limit); a
                             larger prediction is lowered to it.  Bounds one outer step's
                             displacements for the neighbour skins */
    int32_t rollback;     /* 0: a failed stability check (skin, bead skin, non-finite
                             velocity or far position) ends the call with AIMTS_E_UNSTABLE.  > 0: the call
                             runs in segments of this many outer steps; the particle arrays
                             are copied on the device (workspace) at the start of each
                             segment and the host reads the error word at its end; a failed
                             segment is restored, its forces recomputed, and run again at
                             half its largest ratio (ratio 4 after 8: the fallback ratio of
                             the controller, which keeps it for its current hold), halved
                             again while it fails, down to one rerun at ratio 1; a failure
                             there ends the call with AIMTS_E_UNSTABLE (reruns draw fresh
                             random numbers) */
} aimts_schedule;

/* Three-level MTS with per-platelet sublevels [Sec. 3.3, Table 1; Table 2, rows 5-6].
 * Levels, with dt the aimts_schedule's dt_inner (the finest step) and k its ratio:
 *   fluid        k dt        the outer group (fluid DPD, body force);
 *   interface    k_if dt     group M: bead-fluid/wall WCA + dissipative + random (Eq. 3),
 *                            the random term scaled by 1/sqrt(k_if dt);
 *   flowing      k_sub dt    group P1: bonds, angles and same-platelet WCA of the
 *                            platelets at sublevel 1;
 *   aggregating  dt          group P2: the same terms of the platelets at sublevel 2 and
 *                            every inter-platelet term (WCA between platelets, Morse).
 * k_sub divides k_if and both are powers of two; an outer step at a ratio k below k_if
 * runs its interface at min(k_if, k) and its flowing sublevel at min(k_sub, that); k
 * must be a multiple of the interface ratio it gets.  All groups due at one inner step
 * are evaluated at the state after its drift; closing half kicks run innermost first,
 * opening ones outermost first.  k_if = k_sub = 1 is two-group RESPA.  level[p] in {1, 2}
 * is platelet p's sublevel ([n_platelet] host array; NULL keeps the current ones; all 2
 * at creation).  In controller mode the controller sets the sublevels at every decision:
 * a platelet whose predicted ratio exceeds the system's ratio (the minimum over platelets,
 * capped at k_max) takes sublevel 1, the others sublevel 2.  Needs a context created with
 * three_level = 1 unless k_if = k_sub = 1 (AIMTS_E_UNSUPPORTED); AIMTS_E_INVALID for other
 * ratios or levels.  The inner forces must be recomputed (aimts_compute_forces) before
 * the next aimts_step. */
aimts_status aimts_set_levels(aimts_ctx *ctx, int32_t k_if, int32_t k_sub, const int32_t *level);
/* The current ratios and the platelets' sublevels ([n_platelet]; any pointer may be NULL;
 * all 2 in two-group mode). */
aimts_status aimts_get_levels(aimts_ctx *ctx, int32_t *k_if, int32_t *k_sub, int32_t *level);
/* Inner forces by group ([N][3] float64, particle order; any may be NULL): the interface
 * group M and the platelet groups P1 and P2 at their last evaluation (three-level mode;
 * in two-group mode f_m receives the whole inner force and f_p1, f_p2 zeros). */
aimts_status aimts_get_level_forces(aimts_ctx *ctx, double *f_m, double *f_p1, double *f_p2);

/* Advance n_outer outer steps of two-group RESPA:
 *   v += (k dt/2) F_out/m;  k x [v += (dt/2) F_in/m; x += dt v; F_in; v += (dt/2) F_in/m];
 *   rebuild cell list; F_out;  v += (k dt/2) F_out/m.
 * Mode 1 runs the controller on the feature window every `hold` outer steps once 64
 * steps of features exist and takes its ratio (at most k_max when k_max > 0) and hold
 * (ratio 4 before that and on a non-finite or out-of-range output, counted as a
 * fallback). */
aimts_status aimts_step(aimts_ctx *ctx, int64_t n_outer, const aimts_schedule *schedule);

/* Current positions/velocities ([N][3] float64, particle order). Either may be NULL. */
aimts_status aimts_get_state(aimts_ctx *ctx, double *x, double *v);

/* Last outer and inner forces ([N][3] float64, particle order; float32 forces are
 * widened).  Walls carry zero force; beads carry zero outer force. Either may be NULL. */
aimts_status aimts_get_forces(aimts_ctx *ctx, double *f_outer, double *f_inner);

typedef struct {
    int64_t step;           /* outer steps since aimts_set_state */
    double time;            /* simulated time since aimts_set_state */
    double ke;              /* kinetic energy of mobile particles */
    double T;               /* sum m v^2 / (3 N_mobile - 3) */
    double T_pec;           /* fluid temperature about the mean velocity of each cell row
                               along y (rows of the cell grid; occupied rows removed from
                               the degrees of freedom) */
    double p[3];            /* total momentum of mobile particles */
    double pe[5];           /* U_dpd (a rc/2 w^2 per pair), U_lj, U_bond, U_angle, U_morse */
    double virial;          /* sum over conservative pairs of r_ij . F_ij */
    int32_t k, hold;        /* ratio and hold in force */
    int32_t fallbacks;      /* controller outputs replaced by the fallback ratio */
    int32_t inferences;     /* controller invocations */
    uint32_t error_flags;   /* device error bits (see aimts_last_error) */
    int32_t energy_valid;   /* 1 if pe[] and virial were computed by this call */
    int64_t inner_members;  /* beads + fluid particles in the platelet force group */
    int64_t inner_pairs;    /* entries of the platelet pair list (both directions) */
    int32_t rollbacks;      /* segments rolled back and rerun (aimts_schedule.rollback) */
    int32_t rescanned;      /* beads whose partners at the last list rebuild outnumbered
                               the 512 kept per bead by the first scan, so that their
                               lists were scanned again */
} aimts_diag;

/* Thermodynamics of the current state.  want_energy != 0 also evaluates the
 * conservative energies and virial (an extra force pass without advancing the RNG
 * counters).  features (may be NULL) receives [n_platelet][8] float32 features of
 * the current state: COM velocity (3), |angular velocity|, internal kinetic energy,
 * max bond strain, interfacial shear traction, contact count. */
aimts_status aimts_get_diag(aimts_ctx *ctx, int32_t want_energy, aimts_diag *diag, float *features);

/* Rows of the diagnostics time series recorded by aimts_step since aimts_set_state,
 * each [time, ke, T, T_pec, px, py, pz, k] float64 (8 columns).  Copies
 * min(count, max_rows) rows; *count receives the number recorded. */
aimts_status aimts_get_series(aimts_ctx *ctx, double *rows, int64_t max_rows, int64_t *count);

/* ---- checkpoint and resume ----
 * A checkpoint holds everything a later aimts_step depends on: positions and
 * velocities, the current outer force and the inner force of the platelet group's
 * members (the forces the next opening kick uses), the random-number counters, the
 * step count and simulated time, the diagnostics series, the 64-step feature ring, the
 * controller's ratio, hold and steps since its last decision, its counters and, when
 * set, its weights and Adam moments.  Saving it, loading it into a context created and
 * set up the same way (same system description, parameters and topology, checked) and
 * stepping on gives bit for bit the trajectory of the saving context.  The cell sort and
 * the platelet lists are rebuilt on load from the positions (they depend on nothing
 * else).  `buf` is a host buffer of at least aimts_checkpoint_size() bytes, borrowed for
 * the call; the size changes as the platelet group and the series grow.
 * aimts_save_checkpoint: AIMTS_E_STATE without state and forces or after a failure;
 * AIMTS_E_INVALID for a short buffer.  aimts_load_checkpoint: AIMTS_E_INVALID for a blob
 * of another system, precision or parameter set, a truncated blob, or one whose series
 * exceeds this context's capacity. */
aimts_status aimts_checkpoint_size(aimts_ctx *ctx, size_t *bytes);
aimts_status aimts_save_checkpoint(aimts_ctx *ctx, void *buf, size_t bytes);
aimts_status aimts_load_checkpoint(aimts_ctx *ctx, const void *buf, size_t bytes);

/* Device-time profiling with HIP events recorded on the context's stream around each
 * launch group of aimts_step, for the phases whose bit is set in `mask`:
 *   bit 0: outer (DPD) force kernel          bit 1: inner loop (platelet forces, kicks, drifts)
 *   bit 2: cell sort (counting sort, gather) bit 3: outer kicks and lazy drift
 *   bit 4: diagnostics, features, controller bit 5: platelet member and pair lists
 * mask 0 stops profiling.  Times accumulate over aimts_step calls until the next
 * aimts_profile call; aimts_get_profile returns ms[6] and the number of timed
 * intervals per phase in count[6]. */
aimts_status aimts_profile(aimts_ctx *ctx, int32_t mask);
aimts_status aimts_get_profile(aimts_ctx *ctx, double *ms, int64_t *count);

/* ---- learned controller (Table 2) ----
 * Parameters: one float32 vector in this order (row-major matrices, GRU gate
 * rows ordered r, z, n): enc0 w_ih[192][8] w_hh[192][64] b_ih[192] b_hh[192];
 * enc1 (same with w_ih[192][64]); lat_w[16][64] lat_b[16]; dec0 w_ih[192][16]
 * w_hh b_ih b_hh; dec1 (w_ih[192][64]); out_w[8][64] out_b[8]; h1_w[32][16] h1_b;
 * h2_w[16][32] h2_b; h3_w[8][16] h3_b; h4_w[9][8] h4_b[9]; norm_mean[8] norm_std[8].
 * The device keeps this float32 master copy and computes with bfloat16-rounded
 * weights (round to nearest even) and float32 activations and accumulation. */
aimts_status aimts_ctrl_num_params(int64_t *n);
aimts_status aimts_ctrl_set_weights(aimts_ctx *ctx, const float *params, int64_t n);
aimts_status aimts_ctrl_get_weights(aimts_ctx *ctx, float *params, int64_t n);

/* Forward pass on device windows d_windows[batch][64][8] (raw features): writes
 * d_latent[batch][16] and d_logits[batch][9] (5 ratio logits over {1,2,4,8,16}, 4 hold
 * logits over {16,32,64,128}); either output may be NULL. */
aimts_status aimts_ctrl_forward(aimts_ctx *ctx, const float *d_windows, int32_t batch, float *d_latent,
                                float *d_logits);

/* Loss and gradient on device data: phase 0 = reconstruction MSE of the denoised
 * window (autoencoder parameters), phase 1 = cross-entropy of both heads
 * (head parameters; d_labels[batch][2] class indices).  d_grads receives the full
 * parameter-vector gradient (zeros outside the phase) in float32; *loss the loss. */
aimts_status aimts_ctrl_backward(aimts_ctx *ctx, const float *d_windows, const int32_t *d_labels, int32_t batch,
                                 int32_t phase, float *d_grads, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step counter per
 * context) of the phase's parameters with learning rate lr. */
aimts_status aimts_ctrl_train_step(aimts_ctx *ctx, const float *d_windows, const int32_t *d_labels,
                                   int32_t batch, int32_t phase, float lr, float *loss);

/* Run the controller on the current feature window of every platelet and return the
 * system ratio and hold (minimum over platelets).  AIMTS_E_STATE before 64 steps of
 * features exist. */
aimts_status aimts_ctrl_infer(aimts_ctx *ctx, int32_t *k, int32_t *hold);

/* The last 64 feature rows of every platelet, [n_platelet][64][8] float32, oldest first. */
aimts_status aimts_get_feature_window(aimts_ctx *ctx, float *window);

/* ---- for callers that cannot allocate device memory ----
 * aimts_ctrl_forward without a context, for code under HIP graph capture, tight serving
 * loops and harnesses that forbid allocation.  It allocates nothing: the bfloat16 copy
 * of the weights and the activations of up to AIMTS_CTRL_STATIC_MAX_BATCH windows live
 * in a file-scope device array of the library (40.7 MiB, held on every GPU the library
 * runs on until the process ends).
 *   d_params  device float32 parameter vector, n_params == aimts_ctrl_num_params(),
 *             in the layout above (the caller keeps ownership; read only);
 *   d_windows device [batch][64][8] float32 raw feature windows, 1 <= batch <= 256;
 *   d_latent  device [batch][16], d_logits device [batch][9] (either may be NULL);
 *   hip_stream the hipStream_t the work is queued on (NULL: the null stream).
 * Outputs equal aimts_ctrl_forward's for the same weights and windows.  The call is
 * asynchronous: it returns once the work is queued, and the outputs are ready when the
 * stream reaches that point.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must be serialised by the
 * caller.  A batch outside [1, 256], a wrong n_params or a NULL input returns
 * AIMTS_E_INVALID before any device work; aimts_last_error(NULL) gives the message. */
#define AIMTS_CTRL_STATIC_MAX_BATCH 256
aimts_status aimts_ctrl_forward_static(const float *d_params, int64_t n_params, const float *d_windows,
                                       int32_t batch, float *d_latent, float *d_logits, void *hip_stream);

/* The paper's six platelet measurements (Sec. 3.3: "angular velocity components, kinetic
 * energies, and the surrounding flow speed at the platelet center of mass") at the
 * current state, out[n_platelet][6] float64: omega = I^-1 L about the centre of mass (3),
 * the translational kinetic energy 1/2 M |V|^2, the rotational kinetic energy
 * 1/2 omega . L, and the speed of the mean velocity of the fluid particles closer than
 * flow_r to the centre of mass (0 if none).  Synchronous.  Errors: AIMTS_E_STATE before
 * aimts_compute_forces; AIMTS_E_INVALID for flow_r <= 0 or a flow_r that spans more
 * cells than a periodic axis has. */
aimts_status aimts_get_paper_features(aimts_ctx *ctx, double flow_r, double *out);

/* Per-bead membrane stress (Sec. 4.2, Fig. 5): aimts_stress_sample adds, on the device,
 * every bead's pressure-like virial trace times volume at the current state,
 * p_b = (m |v_b|^2 + W_b) / 3, W_b = the bead's share of r.F of the conservative
 * inner-group terms (half of each WCA pair, Eq. 4 aggregation pair, bond and Morse bond;
 * angles carry no virial), to a running sum (asynchronous).  aimts_get_stress returns
 * the mean over the samples, mean[n_bead] float64 in bead order, and their number;
 * reset != 0 starts a new sum.  Errors: AIMTS_E_STATE before aimts_compute_forces or
 * when mean is requested without samples. */
aimts_status aimts_stress_sample(aimts_ctx *ctx);
aimts_status aimts_get_stress(aimts_ctx *ctx, double *mean, int64_t *samples, int32_t reset);

/* ---- the paper's own inference pipeline (Sec. 3.3, Table 2), in its sizes ----
 * Windows: float32 [batch][50][6] device arrays of the paper's six platelet measurements
 * (aimts_get_paper_features).  Pipeline: a causal 5-point moving average, a one-level
 * Haar wavelet transform with the details soft-thresholded at the universal threshold
 * (median |d| / 0.6745) sqrt(2 ln 50), the inverse transform, a z-score with the stored
 * statistics; a 2-layer LSTM encoder with 16 and 4 units (gates i, f, g, o) whose 8
 * latents are the last hidden and cell states of the 4-unit layer; an FCN 8 -> 32 -> 16
 * -> 8 -> 1 (ReLU between layers) whose output is log2 of the MTS ratio.  The decoder
 * (LSTM 8 -> 4 -> 16 fed the latent at every step, read-out 16 -> 6) serves training.
 * Parameters: one float32 vector in this order (row-major, gate rows i, f, g, o):
 * enc0 w_ih[64][6] w_hh[64][16] b_ih[64] b_hh[64]; enc1 w_ih[16][16] w_hh[16][4] b_ih[16]
 * b_hh[16]; dec0 w_ih[16][8] w_hh[16][4] b_ih[16] b_hh[16]; dec1 w_ih[64][4] w_hh[64][16]
 * b_ih[64] b_hh[64]; out_w[6][16] out_b[6]; fc1_w[32][8] fc1_b[32] fc2_w[16][32] fc2_b[16]
 * fc3_w[8][16] fc3_b[8] fc4_w[1][8] fc4_b[1]; norm_mean[6] norm_std[6].
 * These calls need no context: every buffer is a caller-owned device buffer, the
 * workspace holds the activations of up to the batch it was sized for
 * (aimts_lstm_workspace_size), and the work is queued on hip_stream (NULL: the null
 * stream).  Errors (AIMTS_E_INVALID for a null buffer, a batch < 1 or a bad phase,
 * AIMTS_E_NOMEM for a small workspace, AIMTS_E_HIP for a launch failure) leave their
 * message in aimts_last_error(NULL).  Calls that share a workspace must not overlap. */
aimts_status aimts_lstm_num_params(int64_t *n);
aimts_status aimts_lstm_workspace_size(int32_t max_batch, size_t *bytes);
/* The denoised, z-scored windows [batch][50][6] (step 2 of Table 2). */
aimts_status aimts_lstm_filter(const float *d_params, const float *d_windows, int32_t batch, float *d_out,
                               void *hip_stream);
/* Latents [batch][8] and predicted log2 ratios [batch] (either may be NULL); with a
 * non-NULL d_recon also the decoder's reconstruction [batch][50][6] of the denoised
 * windows. */
aimts_status aimts_lstm_forward(const float *d_params, const float *d_windows, int32_t batch, float *d_latent,
                                float *d_pred, float *d_recon, void *d_workspace, size_t bytes, void *hip_stream);
/* Gradient d_grad[n_params] of the batch-mean loss of phase 0 (reconstruction MSE over
 * [batch][50][6], autoencoder parameters) or phase 1 (MSE of the predicted log2 ratio
 * against d_targets[batch], FCN parameters); zeros elsewhere; the loss in d_loss[0]
 * (NULL: not written).  Deterministic: per-window sums added in window order. */
aimts_status aimts_lstm_backward(const float *d_params, const float *d_windows, const float *d_targets, int32_t batch,
                                 int32_t phase, float *d_grad, float *d_loss, void *d_workspace, size_t bytes,
                                 void *hip_stream);
/* One bias-corrected Adam step (beta 0.9, 0.999; eps 1e-8) on the parameters of the
 * phase; d_m, d_v: float32 moments [n_params] (zero before step 1); step counts from 1. */
aimts_status aimts_lstm_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, int32_t phase, int64_t step,
                             float lr, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* AIMTS_H */
