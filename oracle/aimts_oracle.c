/*
 * aimts_oracle.c -- plain FP64 CPU oracle for the DPD + CGMD multiple-time-stepping
 * hot path of "AI-aided multiscale modeling of physiologically-significant blood
 * clots" (Zhu et al., arXiv 2205.14121).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path; both read the same seeded inputs and
 * implement the same published random-number generator independently.
 *
 * Everything here is written to be checked by eye against the paper:
 *   - pair forces are the plain sum over all pairs within the cutoff, either by
 *     brute force over every pair or through a linked-cell list (Hockney-Eastwood
 *     head/next chains) whose pair set the tests compare against brute force;
 *   - the integrator is literal RESPA in the nesting of the paper's MSM pseudocode
 *     (Table 1): every particle drifts at the inner step.
 *
 * Readings of the paper that are not fixed by its text (documented with the tests):
 *   DPD (Sec. 3.2, Eq. 1): w = 1 - r/rc for r < rc, omega_R = w, omega_D = w^2;
 *     F_ij = [a w - gamma w^2 (e.v_ij) + sigma w zeta_ij / sqrt(dt)] e_ij with
 *     e_ij = (x_i - x_j)/r under the minimum image, v_ij = v_i - v_j, and dt the
 *     step of the force group the pair belongs to (Groot-Warren form of the random
 *     term; Eq. 1 writes the sqrt(dt) twice).
 *   zeta_ij = zeta_ji ~ N(0,1) from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
 *     with counter (min id, max id, c_lo, c_hi) and key (seed_lo, seed_hi ^ group);
 *     u1 = (w0 + 0.5) 2^-32, u2 = (w1 + 0.5) 2^-32, zeta = sqrt(-2 ln u1) cos(2 pi u2).
 *   Eq. 2 harmonic terms without a factor 1/2: U = kb (r - r0)^2, U = ka (th - th0)^2.
 *   LJ is the WCA form: cut at 2^(1/6) sigma and shifted by +eps.
 *   Same-platelet LJ pairs interact only if their rest-mesh distance is >= r_excl.
 *   Eq. 3 (platelet-fluid): force -grad U_LJ plus the DPD dissipative and random
 *     terms with (gamma_pf, sigma_pf, rc_pf), no DPD conservative term.
 *   Morse (Eq. 2, inter-platelet bonds of Eq. 4): U = D[e^{-2a(r-r0)} - 2 e^{-a(r-r0)}].
 *   Inter-platelet aggregation (Eq. 4), when agg_rc > 0: every pair of beads of
 *     different platelets closer than agg_rc interacts through the non-bonded Morse
 *     term (agg_D, agg_a, agg_r0) plus the receptor term, a force f^A (1 - r/r0) along
 *     e_ij with the same r0 (a linear spring about r0: U_A = (f^A r0 / 2)(1 - r/r0)^2);
 *     both are cut at agg_rc (the force jumps there; the energy is shifted to 0).
 *   External force (F^E of Eq. 1): once per fluid particle, not per pair.
 *   Walls: frozen particles (never integrated); a mobile particle that crosses a
 *     wall plane after a drift has its position reflected and its whole velocity
 *     reversed (bounce-back).
 *
 * Particle order: fluid [0, nf), wall [nf, nf+nw), beads [nf+nw, N).
 * Force groups: outer = fluid-fluid and fluid-wall DPD + body force;
 *               inner = bonds, angles, Morse bonds, bead-bead WCA, inter-platelet
 *                       aggregation, bead-fluid/wall WCA + dissipative + random.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double lo[3];
    double L[3];
    int32_t periodic[3];
    int32_t wall_axis;          /* -1: no walls */
    double wall_lo, wall_hi;    /* reflecting planes for mobile particles */
    double mass[3];             /* fluid, wall, bead */
    double a, gamma, sigma, rc; /* DPD, Eq. 1 */
    double lj_eps, lj_sig, lj_rc;
    double gamma_pf, sigma_pf, rc_pf;
    double kb, ka;
    double morse_D, morse_a, morse_r0;
    double r_excl;
    double g[3];
    uint64_t seed;
    int64_t n_fluid, n_wall, n_bead;
    int64_t n_bond, n_angle, n_morse;
    int64_t n_platelet;
    const int32_t *body;        /* [n_bead] platelet of each bead */
    const double *rest;         /* [n_bead][3] rest-mesh coordinates */
    const int32_t *bond;        /* [n_bond][2] particle indices */
    const double *bond_r0;      /* [n_bond] */
    const int32_t *angle;       /* [n_angle][3] (end, vertex, end) particle indices */
    const double *angle_th0;    /* [n_angle] radians */
    const int32_t *morse;       /* [n_morse][2] particle indices */
    const double *platelet_area;/* [n_platelet] rest surface area */
    double agg_D, agg_a, agg_r0, agg_fA, agg_rc; /* Eq. 4 aggregation; agg_rc = 0: off */
} or_system;

enum { T_FLUID = 0, T_WALL = 1, T_BEAD = 2 };

static int ptype(const or_system *s, int64_t i)
{
    if (i < s->n_fluid) return T_FLUID;
    if (i < s->n_fluid + s->n_wall) return T_WALL;
    return T_BEAD;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10: counter-based generator of Salmon et al. (SC'11).    */
/* One round multiplies the even words by two fixed odd constants and  */
/* mixes the high halves with the odd words and the round key; the key */
/* advances by two Weyl increments between rounds.                     */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Pair-symmetric Gaussian zeta_ij for the random force of Eq. 1. */
double or_zeta(uint32_t id_i, uint32_t id_j, uint64_t count, uint64_t seed, uint32_t group)
{
    uint32_t ctr[4], key[2], w[4];
    ctr[0] = id_i < id_j ? id_i : id_j;
    ctr[1] = id_i < id_j ? id_j : id_i;
    ctr[2] = (uint32_t)count;
    ctr[3] = (uint32_t)(count >> 32);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32) ^ group;
    or_philox4x32_10(ctr, key, w);
    double u1 = ((double)w[0] + 0.5) * (1.0 / 4294967296.0);
    double u2 = ((double)w[1] + 0.5) * (1.0 / 4294967296.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ------------------------------------------------------------------ */
/* Geometry                                                             */
/* ------------------------------------------------------------------ */
static void min_image(const or_system *s, const double *xi, const double *xj, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double dk = xi[k] - xj[k];
        if (s->periodic[k]) {
            if (dk > 0.5 * s->L[k]) dk -= s->L[k];
            else if (dk < -0.5 * s->L[k]) dk += s->L[k];
        }
        d[k] = dk;
    }
}

/* ------------------------------------------------------------------ */
/* Linked-cell list (head/next chains), cell side >= cutoff.           */
/* ------------------------------------------------------------------ */
typedef struct {
    int n[3];
    double side[3];
    int64_t ncell;
    int64_t *head;
    int64_t *next;
} cells_t;

static int cells_build(const or_system *s, const double *x, int64_t N, double cutoff, cells_t *c)
{
    for (int k = 0; k < 3; ++k) {
        int nk = (int)floor(s->L[k] / cutoff);
        if (nk < 1) nk = 1;
        if (s->periodic[k] && nk < 3) return -1; /* caller falls back to brute force */
        c->n[k] = nk;
        c->side[k] = s->L[k] / nk;
    }
    c->ncell = (int64_t)c->n[0] * c->n[1] * c->n[2];
    c->head = (int64_t *)malloc(sizeof(int64_t) * c->ncell);
    c->next = (int64_t *)malloc(sizeof(int64_t) * (N > 0 ? N : 1));
    if (!c->head || !c->next) { free(c->head); free(c->next); return -2; }
    for (int64_t q = 0; q < c->ncell; ++q) c->head[q] = -1;
    for (int64_t i = N - 1; i >= 0; --i) {
        int idx[3];
        for (int k = 0; k < 3; ++k) {
            int ik = (int)floor((x[3 * i + k] - s->lo[k]) / c->side[k]);
            if (ik < 0) ik = s->periodic[k] ? ik + c->n[k] : 0;
            if (ik >= c->n[k]) ik = s->periodic[k] ? ik - c->n[k] : c->n[k] - 1;
            if (ik < 0) ik = 0;
            if (ik >= c->n[k]) ik = c->n[k] - 1;
            idx[k] = ik;
        }
        int64_t q = ((int64_t)idx[0] * c->n[1] + idx[1]) * c->n[2] + idx[2];
        c->next[i] = c->head[q];
        c->head[q] = i;
    }
    return 0;
}

static void cells_free(cells_t *c) { free(c->head); free(c->next); }

/* The distinct neighbour cells of the cell holding point p (at most 27). */
static int cells_around(const or_system *s, const cells_t *c, const double *p, int64_t out[27])
{
    int idx[3];
    for (int k = 0; k < 3; ++k) {
        int ik = (int)floor((p[k] - s->lo[k]) / c->side[k]);
        if (ik < 0) ik = s->periodic[k] ? ik + c->n[k] : 0;
        if (ik >= c->n[k]) ik = s->periodic[k] ? ik - c->n[k] : c->n[k] - 1;
        if (ik < 0) ik = 0;
        if (ik >= c->n[k]) ik = c->n[k] - 1;
        idx[k] = ik;
    }
    int m = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int j[3] = {idx[0] + dx, idx[1] + dy, idx[2] + dz};
                int ok = 1;
                for (int k = 0; k < 3; ++k) {
                    if (j[k] < 0 || j[k] >= c->n[k]) {
                        if (!s->periodic[k]) { ok = 0; break; }
                        j[k] = (j[k] + c->n[k]) % c->n[k];
                    }
                }
                if (!ok) continue;
                int64_t q = ((int64_t)j[0] * c->n[1] + j[1]) * c->n[2] + j[2];
                int dup = 0;
                for (int t = 0; t < m; ++t) if (out[t] == q) { dup = 1; break; }
                if (!dup) out[m++] = q;
            }
    return m;
}

/* ------------------------------------------------------------------ */
/* Pair laws.  Each returns the scalar f such that F_on_i = f * d,      */
/* where d = x_i - x_j (minimum image) and r = |d|.                     */
/* ------------------------------------------------------------------ */

/* DPD, Eq. 1 (conservative + dissipative + random). */
static double dpd_pair(double a, double gamma, double sigma, double rc, double r, const double d[3],
                       const double vi[3], const double vj[3], double zeta, double inv_sqrt_dt)
{
    double w = 1.0 - r / rc;
    double e[3] = {d[0] / r, d[1] / r, d[2] / r};
    double ev = e[0] * (vi[0] - vj[0]) + e[1] * (vi[1] - vj[1]) + e[2] * (vi[2] - vj[2]);
    double fmag = a * w - gamma * w * w * ev + sigma * w * zeta * inv_sqrt_dt;
    return fmag / r;
}

/* WCA Lennard-Jones, Eq. 2: F = -dU/dr e. */
static double lj_pair(double eps, double sig, double r)
{
    double sr2 = (sig * sig) / (r * r);
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    return 24.0 * eps * (2.0 * sr12 - sr6) / (r * r);
}

static double lj_energy(double eps, double sig, double r)
{
    double sr6 = pow(sig / r, 6.0);
    return 4.0 * eps * (sr6 * sr6 - sr6) + eps;
}

/* Whether beads bi, bj (bead indices) interact through the non-bonded WCA term. */
static int bead_pair_allowed(const or_system *s, int64_t bi, int64_t bj)
{
    if (s->body[bi] != s->body[bj]) return 1;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = s->rest[3 * bi + k] - s->rest[3 * bj + k];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) >= s->r_excl;
}

/* Eq. 4 between beads bi, bj (bead indices) of different platelets r apart: the
 * scalar fs with F_i = fs * (x_i - x_j), or 0 beyond agg_rc or within one platelet.
 * Non-bonded Morse: -dU/dr = 2 a D (e^{-2a(r-r0)} - e^{-a(r-r0)});
 * receptor term: f^A (1 - r/r0). */
static double agg_pair(const or_system *s, int64_t bi, int64_t bj, double r)
{
    if (!(s->agg_rc > 0.0) || !(r < s->agg_rc) || s->body[bi] == s->body[bj]) return 0.0;
    double ex = exp(-s->agg_a * (r - s->agg_r0));
    double fm = 2.0 * s->agg_a * s->agg_D * (ex * ex - ex);
    double fa = s->agg_fA * (1.0 - r / s->agg_r0);
    return (fm + fa) / r;
}

/* The energy of agg_pair's force: U_M + U_A, shifted to 0 at agg_rc. */
static double agg_energy_raw(const or_system *s, double r)
{
    double ex = exp(-s->agg_a * (r - s->agg_r0));
    double q = 1.0 - r / s->agg_r0;
    return s->agg_D * (ex * ex - 2.0 * ex) + 0.5 * s->agg_fA * s->agg_r0 * q * q;
}

static double agg_energy(const or_system *s, int64_t bi, int64_t bj, double r)
{
    if (!(s->agg_rc > 0.0) || !(r < s->agg_rc) || s->body[bi] == s->body[bj]) return 0.0;
    return agg_energy_raw(s, r) - agg_energy_raw(s, s->agg_rc);
}

/* Largest pair cutoff of the inner group. */
static double inner_cut(const or_system *s)
{
    double cut = s->lj_rc > s->rc_pf ? s->lj_rc : s->rc_pf;
    if (s->agg_rc > cut) cut = s->agg_rc;
    return cut;
}

/* ------------------------------------------------------------------ */
/* Outer group: fluid-fluid and fluid-wall DPD + body force on fluid.   */
/* f is [N][3]; rows of the particles not listed in `subset` are left   */
/* untouched when a subset is given.  Returns 0 or a negative error.    */
/* ------------------------------------------------------------------ */
int or_outer_forces(const or_system *s, const double *x, const double *v, uint64_t count, double dt,
                    const int64_t *subset, int64_t nsub, int brute, int nthreads, double *f)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t NS = s->n_fluid + s->n_wall; /* beads never take part in the outer group */
    cells_t c;
    int have_cells = 0;
    if (!brute) {
        int rcode = cells_build(s, x, NS, s->rc, &c);
        if (rcode == -2) return -2;
        have_cells = (rcode == 0);
    }
    const double inv_sqrt_dt = 1.0 / sqrt(dt);
    const double rc2 = s->rc * s->rc;
    int64_t count_i = subset ? nsub : N;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) if (nthreads != 1)
#endif
    for (int64_t t = 0; t < count_i; ++t) {
        int64_t i = subset ? subset[t] : t;
        double fi[3] = {0.0, 0.0, 0.0};
        if (ptype(s, i) == T_FLUID) {
            int64_t around[27];
            int nc = 1;
            if (have_cells) nc = cells_around(s, &c, &x[3 * i], around);
            for (int q = 0; q < nc; ++q) {
                int64_t j = have_cells ? c.head[around[q]] : 0;
                while (have_cells ? (j >= 0) : (j < NS)) {
                    if (j != i) {
                        double d[3];
                        min_image(s, &x[3 * i], &x[3 * j], d);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rc2 && r2 > 0.0) {
                            double r = sqrt(r2);
                            double z = or_zeta((uint32_t)i, (uint32_t)j, count, s->seed, 0u);
                            double fs = dpd_pair(s->a, s->gamma, s->sigma, s->rc, r, d, &v[3 * i], &v[3 * j],
                                                 z, inv_sqrt_dt);
                            fi[0] += fs * d[0];
                            fi[1] += fs * d[1];
                            fi[2] += fs * d[2];
                        }
                    }
                    j = have_cells ? c.next[j] : j + 1;
                }
            }
            fi[0] += s->g[0];
            fi[1] += s->g[1];
            fi[2] += s->g[2];
        }
        f[3 * i + 0] = fi[0];
        f[3 * i + 1] = fi[1];
        f[3 * i + 2] = fi[2];
    }
    if (have_cells) cells_free(&c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Bonded terms of Eq. 2 (scatter form over the bond/angle lists).     */
/* ------------------------------------------------------------------ */
static void bonded_forces(const or_system *s, const double *x, double *f)
{
    for (int64_t b = 0; b < s->n_bond; ++b) {
        int64_t i = s->bond[2 * b], j = s->bond[2 * b + 1];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        /* U = kb (r - r0)^2  ->  F_i = -2 kb (r - r0) d / r */
        double fs = -2.0 * s->kb * (r - s->bond_r0[b]) / r;
        for (int k = 0; k < 3; ++k) { f[3 * i + k] += fs * d[k]; f[3 * j + k] -= fs * d[k]; }
    }
    for (int64_t m = 0; m < s->n_angle; ++m) {
        int64_t i = s->angle[3 * m], j = s->angle[3 * m + 1], k2 = s->angle[3 * m + 2];
        double a[3], b[3];
        min_image(s, &x[3 * i], &x[3 * j], a);
        min_image(s, &x[3 * k2], &x[3 * j], b);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double cs = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / (la * lb);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double th = acos(cs);
        double sn = sin(th);
        if (sn < 1e-12) sn = 1e-12;
        /* U = ka (th - th0)^2; F = -dU/dth * dth/dx, dth/dx = -(1/sin th) dcos/dx */
        double dudth = 2.0 * s->ka * (th - s->angle_th0[m]);
        double pref = dudth / sn; /* F_end = pref * dcos/dx_end */
        for (int q = 0; q < 3; ++q) {
            double dci = b[q] / (la * lb) - cs * a[q] / (la * la);
            double dck = a[q] / (la * lb) - cs * b[q] / (lb * lb);
            double fi = pref * dci, fk = pref * dck;
            f[3 * i + q] += fi;
            f[3 * k2 + q] += fk;
            f[3 * j + q] -= fi + fk;
        }
    }
    for (int64_t b = 0; b < s->n_morse; ++b) {
        int64_t i = s->morse[2 * b], j = s->morse[2 * b + 1];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double ex = exp(-s->morse_a * (r - s->morse_r0));
        /* U = D (ex^2 - 2 ex);  -dU/dr = 2 a D (ex^2 - ex) */
        double fs = 2.0 * s->morse_a * s->morse_D * (ex * ex - ex) / r;
        for (int k = 0; k < 3; ++k) { f[3 * i + k] += fs * d[k]; f[3 * j + k] -= fs * d[k]; }
    }
}

/* ------------------------------------------------------------------ */
/* Inner group: bonded + bead non-bonded + bead-fluid/wall (Eq. 2, 3). */
/* f is [N][3] and is overwritten for every particle.                  */
/* ------------------------------------------------------------------ */
int or_inner_forces(const or_system *s, const double *x, const double *v, uint64_t count, double dt,
                    int brute, double *f)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t b0 = s->n_fluid + s->n_wall;
    memset(f, 0, sizeof(double) * 3 * N);
    bonded_forces(s, x, f);
    double cut = inner_cut(s);
    cells_t c;
    int have_cells = 0;
    if (!brute && s->n_bead > 0) {
        int rcode = cells_build(s, x, N, cut, &c);
        if (rcode == -2) return -2;
        have_cells = (rcode == 0);
    }
    const double inv_sqrt_dt = 1.0 / sqrt(dt);
    const double lj2 = s->lj_rc * s->lj_rc, pf2 = s->rc_pf * s->rc_pf;
    for (int64_t i = b0; i < N; ++i) {
        int64_t around[27];
        int nc = 1;
        if (have_cells) nc = cells_around(s, &c, &x[3 * i], around);
        for (int q = 0; q < nc; ++q) {
            int64_t j = have_cells ? c.head[around[q]] : 0;
            while (have_cells ? (j >= 0) : (j < N)) {
                if (j != i) {
                    double d[3];
                    min_image(s, &x[3 * i], &x[3 * j], d);
                    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (ptype(s, j) == T_BEAD) {
                        /* gather form: each bead of the pair adds its own share */
                        if (r2 > 0.0) {
                            double fs = 0.0;
                            if (r2 < lj2 && bead_pair_allowed(s, i - b0, j - b0))
                                fs += lj_pair(s->lj_eps, s->lj_sig, sqrt(r2));
                            fs += agg_pair(s, i - b0, j - b0, sqrt(r2));
                            for (int k = 0; k < 3; ++k) f[3 * i + k] += fs * d[k];
                        }
                    } else if (r2 > 0.0 && (r2 < lj2 || r2 < pf2)) {
                        double r = sqrt(r2);
                        double fs = 0.0;
                        if (r2 < lj2) fs += lj_pair(s->lj_eps, s->lj_sig, r);
                        if (r2 < pf2) {
                            double z = or_zeta((uint32_t)i, (uint32_t)j, count, s->seed, 1u);
                            fs += dpd_pair(0.0, s->gamma_pf, s->sigma_pf, s->rc_pf, r, d, &v[3 * i], &v[3 * j], z,
                                           inv_sqrt_dt);
                        }
                        /* Newton's third law onto the fluid or wall particle */
                        for (int k = 0; k < 3; ++k) { f[3 * i + k] += fs * d[k]; f[3 * j + k] -= fs * d[k]; }
                    }
                }
                j = have_cells ? c.next[j] : j + 1;
            }
        }
    }
    /* frozen walls carry no force */
    for (int64_t i = s->n_fluid; i < b0; ++i) f[3 * i] = f[3 * i + 1] = f[3 * i + 2] = 0.0;
    if (have_cells) cells_free(&c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Potential energy and pair virial of the conservative terms.         */
/* out[0] = U_DPD (a rc/2 w^2 per pair), out[1] = U_LJ, out[2] = U_bond */
/* out[3] = U_angle, out[4] = U_morse (bonds and Eq. 4 aggregation),   */
/* out[5] = sum over pairs d.F                                         */
/* ------------------------------------------------------------------ */
int or_energy(const or_system *s, const double *x, double *out)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t NS = s->n_fluid + s->n_wall;
    const int64_t b0 = NS;
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    /* brute force over all pairs i < j (small systems only) */
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = i + 1; j < N; ++j) {
            int ti = ptype(s, i), tj = ptype(s, j);
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 <= 0.0) continue;
            double r = sqrt(r2);
            if (ti != T_BEAD && tj != T_BEAD) {
                if (ti == T_WALL && tj == T_WALL) continue;
                if (r < s->rc) {
                    double w = 1.0 - r / s->rc;
                    out[0] += 0.5 * s->a * s->rc * w * w;
                    out[5] += s->a * w * r;
                }
            } else {
                int lj = r < s->lj_rc;
                if (ti == T_BEAD && tj == T_BEAD) lj = lj && bead_pair_allowed(s, i - b0, j - b0);
                if (lj) {
                    out[1] += lj_energy(s->lj_eps, s->lj_sig, r);
                    out[5] += lj_pair(s->lj_eps, s->lj_sig, r) * r2;
                }
                if (ti == T_BEAD && tj == T_BEAD) {
                    /* Eq. 4 aggregation counts with the inter-platelet (Morse) energy */
                    out[4] += agg_energy(s, i - b0, j - b0, r);
                    out[5] += agg_pair(s, i - b0, j - b0, r) * r2;
                }
            }
        }
    }
    for (int64_t b = 0; b < s->n_bond; ++b) {
        double d[3];
        min_image(s, &x[3 * s->bond[2 * b]], &x[3 * s->bond[2 * b + 1]], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double dr = r - s->bond_r0[b];
        out[2] += s->kb * dr * dr;
        out[5] += -2.0 * s->kb * dr * r;
    }
    for (int64_t m = 0; m < s->n_angle; ++m) {
        double a[3], b[3];
        min_image(s, &x[3 * s->angle[3 * m]], &x[3 * s->angle[3 * m + 1]], a);
        min_image(s, &x[3 * s->angle[3 * m + 2]], &x[3 * s->angle[3 * m + 1]], b);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double cs = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / (la * lb);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double dth = acos(cs) - s->angle_th0[m];
        out[3] += s->ka * dth * dth;
    }
    for (int64_t b = 0; b < s->n_morse; ++b) {
        double d[3];
        min_image(s, &x[3 * s->morse[2 * b]], &x[3 * s->morse[2 * b + 1]], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double ex = exp(-s->morse_a * (r - s->morse_r0));
        out[4] += s->morse_D * (ex * ex - 2.0 * ex);
        out[5] += 2.0 * s->morse_a * s->morse_D * (ex * ex - ex) * r;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Integrator pieces.                                                   */
/* ------------------------------------------------------------------ */
static int mobile(const or_system *s, int64_t i) { return ptype(s, i) != T_WALL; }

static void kick(const or_system *s, double *v, const double *f, double h)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    for (int64_t i = 0; i < N; ++i) {
        if (!mobile(s, i)) continue;
        double m = s->mass[ptype(s, i)];
        for (int k = 0; k < 3; ++k) v[3 * i + k] += h * f[3 * i + k] / m;
    }
}

static void drift(const or_system *s, double *x, double *v, double h)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    for (int64_t i = 0; i < N; ++i) {
        if (!mobile(s, i)) continue;
        for (int k = 0; k < 3; ++k) x[3 * i + k] += h * v[3 * i + k];
        if (s->wall_axis >= 0) {
            int w = s->wall_axis;
            double y = x[3 * i + w];
            if (y < s->wall_lo || y > s->wall_hi) {
                x[3 * i + w] = y < s->wall_lo ? 2.0 * s->wall_lo - y : 2.0 * s->wall_hi - y;
                for (int k = 0; k < 3; ++k) v[3 * i + k] = -v[3 * i + k];
            }
        }
        for (int k = 0; k < 3; ++k) {
            if (!s->periodic[k]) continue;
            double hi = s->lo[k] + s->L[k];
            if (x[3 * i + k] >= hi) x[3 * i + k] -= s->L[k];
            else if (x[3 * i + k] < s->lo[k]) x[3 * i + k] += s->L[k];
        }
    }
}

/*
 * RESPA with an outer (fluid DPD) and an inner (platelet) force group, nested as
 * in the paper's MSM pseudocode (Table 1) with a half kick on entry and on exit of
 * each level.  On entry f_outer/f_inner hold the forces of the current state and
 * counters[0]/counters[1] the numbers of outer/inner evaluations done so far; both
 * are updated.  All mobile particles drift at the inner step dt_outer/k.
 */
int or_respa(const or_system *s, double *x, double *v, double *f_outer, double *f_inner, uint64_t *counters,
             int64_t n_outer, double dt_outer, int k, int brute, int nthreads)
{
    if (k < 1 || !(dt_outer > 0.0)) return -1;
    const double dt = dt_outer / k;
    for (int64_t n = 0; n < n_outer; ++n) {
        kick(s, v, f_outer, 0.5 * dt_outer);
        for (int sub = 0; sub < k; ++sub) {
            kick(s, v, f_inner, 0.5 * dt);
            drift(s, x, v, dt);
            int rc = or_inner_forces(s, x, v, counters[1], dt, brute, f_inner);
            if (rc) return rc;
            counters[1] += 1;
            kick(s, v, f_inner, 0.5 * dt);
        }
        int rc = or_outer_forces(s, x, v, counters[0], dt_outer, NULL, 0, brute, nthreads, f_outer);
        if (rc) return rc;
        counters[0] += 1;
        kick(s, v, f_outer, 0.5 * dt_outer);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Thermodynamic diagnostics.                                           */
/* out[0] = kinetic energy of mobile particles                          */
/* out[1] = T = sum m v^2 / (3 N_m - 3)                                 */
/* out[2] = peculiar T of the fluid: velocities relative to the mean    */
/*          velocity of their bin along axis `bin_axis` (n_bins equal    */
/*          slabs of the box), divided by 3 (N_f - occupied bins)        */
/* out[3..5] = total momentum of mobile particles                       */
/* ------------------------------------------------------------------ */
int or_thermo(const or_system *s, const double *x, const double *v, int bin_axis, int n_bins, double *out)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    double ke2 = 0.0, p[3] = {0, 0, 0};
    int64_t nm = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (!mobile(s, i)) continue;
        double m = s->mass[ptype(s, i)];
        ke2 += m * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
        for (int k = 0; k < 3; ++k) p[k] += m * v[3 * i + k];
        ++nm;
    }
    double *bm = (double *)calloc((size_t)n_bins * 4, sizeof(double));
    if (!bm) return -2;
    for (int64_t i = 0; i < s->n_fluid; ++i) {
        int b = (int)floor((x[3 * i + bin_axis] - s->lo[bin_axis]) / (s->L[bin_axis] / n_bins));
        if (b < 0) b = 0;
        if (b >= n_bins) b = n_bins - 1;
        double m = s->mass[T_FLUID];
        bm[4 * b] += m;
        for (int k = 0; k < 3; ++k) bm[4 * b + 1 + k] += m * v[3 * i + k];
    }
    double pec = 0.0;
    int64_t occupied = 0;
    for (int64_t i = 0; i < s->n_fluid; ++i) {
        int b = (int)floor((x[3 * i + bin_axis] - s->lo[bin_axis]) / (s->L[bin_axis] / n_bins));
        if (b < 0) b = 0;
        if (b >= n_bins) b = n_bins - 1;
        double m = s->mass[T_FLUID];
        for (int k = 0; k < 3; ++k) {
            double u = v[3 * i + k] - bm[4 * b + 1 + k] / bm[4 * b];
            pec += m * u * u;
        }
    }
    for (int b = 0; b < n_bins; ++b) occupied += bm[4 * b] > 0.0;
    free(bm);
    out[0] = 0.5 * ke2;
    out[1] = nm > 1 ? ke2 / (3.0 * nm - 3.0) : 0.0;
    out[2] = s->n_fluid > occupied ? pec / (3.0 * (double)(s->n_fluid - occupied)) : 0.0;
    out[3] = p[0];
    out[4] = p[1];
    out[5] = p[2];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-platelet dynamics features (eight per platelet, [P][8]):         */
/*  0..2  centre-of-mass velocity                                       */
/*  3     |omega|, omega = I^-1 L about the centre of mass              */
/*  4     internal kinetic energy 1/2 sum m |v - V|^2                   */
/*  5     max bond strain |r - r0| / r0 over the platelet's bonds       */
/*  6     interfacial shear traction: sum over bead-fluid/wall pairs of  */
/*        (y_b - y_j) * (F^LJ + F^D)_x on the bead, over the rest area  */
/*  7     contacts: pairs of a bead with a wall particle or with a bead  */
/*        of another platelet closer than contact_r                      */
/* Bead positions are unwrapped about the platelet's first bead.        */
/* ------------------------------------------------------------------ */
static int solve3(double A[3][3], const double b[3], double xo[3])
{
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                 A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                 A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (fabs(det) < 1e-300) { xo[0] = xo[1] = xo[2] = 0.0; return -1; }
    for (int c = 0; c < 3; ++c) {
        double M[3][3];
        memcpy(M, A, sizeof(M));
        for (int r = 0; r < 3; ++r) M[r][c] = b[r];
        xo[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                 M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                 M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
    }
    return 0;
}

int or_features(const or_system *s, const double *x, const double *v, int shear_axis_y, double contact_r,
                double *feat)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t b0 = s->n_fluid + s->n_wall;
    const int64_t P = s->n_platelet;
    const double mb = s->mass[T_BEAD];
    double *acc = (double *)calloc((size_t)P * 16, sizeof(double));
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (P > 0 ? P : 1));
    if (!acc || !first) { free(acc); free(first); return -2; }
    for (int64_t p = 0; p < P; ++p) first[p] = -1;
    for (int64_t b = 0; b < s->n_bead; ++b)
        if (first[s->body[b]] < 0) first[s->body[b]] = b0 + b;
    /* pass 1: mass, COM offset, momentum */
    for (int64_t b = 0; b < s->n_bead; ++b) {
        int64_t i = b0 + b, p = s->body[b];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * first[p]], d);
        double *A = &acc[16 * p];
        A[0] += mb;
        for (int k = 0; k < 3; ++k) { A[1 + k] += mb * d[k]; A[4 + k] += mb * v[3 * i + k]; }
    }
    double *Lm = (double *)calloc((size_t)P * 3, sizeof(double));
    double *In = (double *)calloc((size_t)P * 9, sizeof(double));
    double *kin = (double *)calloc((size_t)P, sizeof(double));
    if (!Lm || !In || !kin) { free(acc); free(first); free(Lm); free(In); free(kin); return -2; }
    for (int64_t b = 0; b < s->n_bead; ++b) {
        int64_t i = b0 + b, p = s->body[b];
        double *A = &acc[16 * p];
        double d[3], r[3], u[3];
        min_image(s, &x[3 * i], &x[3 * first[p]], d);
        for (int k = 0; k < 3; ++k) {
            r[k] = d[k] - A[1 + k] / A[0];
            u[k] = v[3 * i + k] - A[4 + k] / A[0];
        }
        Lm[3 * p + 0] += mb * (r[1] * u[2] - r[2] * u[1]);
        Lm[3 * p + 1] += mb * (r[2] * u[0] - r[0] * u[2]);
        Lm[3 * p + 2] += mb * (r[0] * u[1] - r[1] * u[0]);
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) In[9 * p + 3 * a + c] += mb * ((a == c ? rr : 0.0) - r[a] * r[c]);
        kin[p] += 0.5 * mb * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    double *strain = (double *)calloc((size_t)P, sizeof(double));
    double *shear = (double *)calloc((size_t)P, sizeof(double));
    double *contact = (double *)calloc((size_t)P, sizeof(double));
    if (!strain || !shear || !contact) {
        free(acc); free(first); free(Lm); free(In); free(kin); free(strain); free(shear); free(contact);
        return -2;
    }
    for (int64_t q = 0; q < s->n_bond; ++q) {
        int64_t i = s->bond[2 * q], j = s->bond[2 * q + 1];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double e = fabs(r - s->bond_r0[q]) / s->bond_r0[q];
        int64_t p = s->body[i - b0];
        if (e > strain[p]) strain[p] = e;
    }
    const double lj2 = s->lj_rc * s->lj_rc, pf2 = s->rc_pf * s->rc_pf, ct2 = contact_r * contact_r;
    double cut = s->lj_rc > s->rc_pf ? s->lj_rc : s->rc_pf;
    if (contact_r > cut) cut = contact_r;
    cells_t c;
    int have_cells = s->n_bead > 0 ? (cells_build(s, x, N, cut, &c) == 0) : 0;
    for (int64_t i = b0; i < N; ++i) {
        int64_t p = s->body[i - b0];
        int64_t around[27];
        int nc = 1;
        if (have_cells) nc = cells_around(s, &c, &x[3 * i], around);
        for (int q = 0; q < nc; ++q)
        for (int64_t j = have_cells ? c.head[around[q]] : 0; have_cells ? (j >= 0) : (j < N);
             j = have_cells ? c.next[j] : j + 1) {
            if (j == i) continue;
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            int tj = ptype(s, j);
            if (r2 < ct2 && (tj == T_WALL || (tj == T_BEAD && s->body[j - b0] != p))) contact[p] += 1.0;
            if (tj != T_BEAD && r2 > 0.0 && (r2 < lj2 || r2 < pf2)) {
                double r = sqrt(r2), fs = 0.0;
                if (r2 < lj2) fs += lj_pair(s->lj_eps, s->lj_sig, r);
                if (r2 < pf2) fs += dpd_pair(0.0, s->gamma_pf, 0.0, s->rc_pf, r, d, &v[3 * i], &v[3 * j], 0.0, 0.0);
                shear[p] += d[shear_axis_y] * fs * d[0];
            }
        }
    }
    if (have_cells) cells_free(&c);
    for (int64_t p = 0; p < P; ++p) {
        double *A = &acc[16 * p];
        double Im[3][3], om[3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) Im[a][c] = In[9 * p + 3 * a + c];
        solve3(Im, &Lm[3 * p], om);
        double *o = &feat[8 * p];
        o[0] = A[4] / A[0];
        o[1] = A[5] / A[0];
        o[2] = A[6] / A[0];
        o[3] = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
        o[4] = kin[p];
        o[5] = strain[p];
        o[6] = shear[p] / s->platelet_area[p];
        o[7] = contact[p];
    }
    free(acc); free(first); free(Lm); free(In); free(kin); free(strain); free(shear); free(contact);
    return 0;
}

/* Brute-force list of all pairs (i < j) within `cutoff` -- pin for the cell lists. */
int64_t or_pairs_brute(const or_system *s, const double *x, int64_t N, double cutoff, int64_t *out, int64_t cap)
{
    int64_t m = 0;
    double c2 = cutoff * cutoff;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = i + 1; j < N; ++j) {
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < c2) {
                if (m < cap) { out[2 * m] = i; out[2 * m + 1] = j; }
                ++m;
            }
        }
    return m;
}

/* The same pair set through the linked-cell list. */
int64_t or_pairs_cells(const or_system *s, const double *x, int64_t N, double cutoff, int64_t *out, int64_t cap)
{
    cells_t c;
    if (cells_build(s, x, N, cutoff, &c) != 0) return -1;
    int64_t m = 0;
    double c2 = cutoff * cutoff;
    for (int64_t i = 0; i < N; ++i) {
        int64_t around[27];
        int nc = cells_around(s, &c, &x[3 * i], around);
        for (int q = 0; q < nc; ++q)
            for (int64_t j = c.head[around[q]]; j >= 0; j = c.next[j]) {
                if (j <= i) continue;
                double d[3];
                min_image(s, &x[3 * i], &x[3 * j], d);
                if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < c2) {
                    if (m < cap) { out[2 * m] = i; out[2 * m + 1] = j; }
                    ++m;
                }
            }
    }
    cells_free(&c);
    return m;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Three-level MTS with per-platelet sublevels (Sec. 3.3, Table 1).     */
/*                                                                      */
/* Levels, from coarse to fine (dt the finest step):                    */
/*   fluid     Delta t_f = k dt        outer group (fluid DPD, F^E)     */
/*   interface Delta t_m = k_if dt     group M: bead-fluid/wall WCA +   */
/*                                     dissipative + random (Eq. 3),    */
/*                                     random term scaled by Delta t_m  */
/*   flowing   dt_1 = k_sub dt         group P1: bonds, angles and the  */
/*                                     same-platelet WCA of platelets   */
/*                                     at sublevel 1                    */
/*   aggregating dt_2 = dt             group P2: the same terms of the  */
/*                                     platelets at sublevel 2, and     */
/*                                     every inter-platelet term (WCA   */
/*                                     between platelets, Morse bonds)  */
/* with k_sub | k_if | k.  level[p] in {1, 2} is the sublevel of        */
/* platelet p.  A bond or angle takes the finest sublevel of its beads' */
/* platelets.  All force groups due at one instant are evaluated at the */
/* state reached after the drift, before any of that instant's kicks;   */
/* with k_if = k_sub = 1 the scheme is two-group RESPA.                 */
/* ------------------------------------------------------------------ */
enum { G3_M = 1, G3_P1 = 2, G3_P2 = 4 };

static int bead_level(const or_system *s, const int32_t *level, int64_t i)
{
    return level[s->body[i - (s->n_fluid + s->n_wall)]] == 1 ? 1 : 2;
}

/* Group of a bonded term whose beads are i, j (and k >= 0). */
static int bonded_group(const or_system *s, const int32_t *level, int64_t i, int64_t j, int64_t k)
{
    int l = bead_level(s, level, i);
    if (bead_level(s, level, j) == 2) l = 2;
    if (k >= 0 && bead_level(s, level, k) == 2) l = 2;
    return l == 1 ? G3_P1 : G3_P2;
}

static double *group_array(int g, double *f_m, double *f_p1, double *f_p2)
{
    return g == G3_M ? f_m : (g == G3_P1 ? f_p1 : f_p2);
}

/* Forces of the groups in `due` at (x, v); the arrays of the other groups are left
 * untouched.  count: the interface group's evaluation counter; dt_m: its step. */
int or_inner_forces3(const or_system *s, const double *x, const double *v, uint64_t count, double dt_m,
                     const int32_t *level, int due, int brute, double *f_m, double *f_p1, double *f_p2)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t b0 = s->n_fluid + s->n_wall;
    if (due & G3_M) memset(f_m, 0, sizeof(double) * 3 * N);
    if (due & G3_P1) memset(f_p1, 0, sizeof(double) * 3 * N);
    if (due & G3_P2) memset(f_p2, 0, sizeof(double) * 3 * N);
    /* bonds: U = kb (r - r0)^2 */
    for (int64_t b = 0; b < s->n_bond; ++b) {
        int64_t i = s->bond[2 * b], j = s->bond[2 * b + 1];
        int g = bonded_group(s, level, i, j, -1);
        if (!(due & g)) continue;
        double *f = group_array(g, f_m, f_p1, f_p2);
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double fs = -2.0 * s->kb * (r - s->bond_r0[b]) / r;
        for (int k = 0; k < 3; ++k) { f[3 * i + k] += fs * d[k]; f[3 * j + k] -= fs * d[k]; }
    }
    /* angles: U = ka (th - th0)^2 about the vertex */
    for (int64_t m = 0; m < s->n_angle; ++m) {
        int64_t i = s->angle[3 * m], j = s->angle[3 * m + 1], k2 = s->angle[3 * m + 2];
        int g = bonded_group(s, level, i, j, k2);
        if (!(due & g)) continue;
        double *f = group_array(g, f_m, f_p1, f_p2);
        double a[3], b[3];
        min_image(s, &x[3 * i], &x[3 * j], a);
        min_image(s, &x[3 * k2], &x[3 * j], b);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double cs = (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / (la * lb);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double th = acos(cs);
        double sn = sin(th);
        if (sn < 1e-12) sn = 1e-12;
        double pref = 2.0 * s->ka * (th - s->angle_th0[m]) / sn;
        for (int q = 0; q < 3; ++q) {
            double fi = pref * (b[q] / (la * lb) - cs * a[q] / (la * la));
            double fk = pref * (a[q] / (la * lb) - cs * b[q] / (lb * lb));
            f[3 * i + q] += fi;
            f[3 * k2 + q] += fk;
            f[3 * j + q] -= fi + fk;
        }
    }
    /* Morse bonds join beads of different platelets: always group P2 */
    if (due & G3_P2) {
        for (int64_t b = 0; b < s->n_morse; ++b) {
            int64_t i = s->morse[2 * b], j = s->morse[2 * b + 1];
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double ex = exp(-s->morse_a * (r - s->morse_r0));
            double fs = 2.0 * s->morse_a * s->morse_D * (ex * ex - ex) / r;
            for (int k = 0; k < 3; ++k) { f_p2[3 * i + k] += fs * d[k]; f_p2[3 * j + k] -= fs * d[k]; }
        }
    }
    /* pairs: every pair (bead i, particle j) within the cutoffs, by brute force or
     * through the linked-cell list */
    const double inv_sqrt_dt = 1.0 / sqrt(dt_m);
    const double lj2 = s->lj_rc * s->lj_rc, pf2 = s->rc_pf * s->rc_pf;
    double cut = inner_cut(s);
    cells_t c;
    int have_cells = 0;
    if (!brute && s->n_bead > 0) {
        int rcode = cells_build(s, x, N, cut, &c);
        if (rcode == -2) return -2;
        have_cells = (rcode == 0);
    }
    for (int64_t i = b0; i < N; ++i) {
        int64_t around[27];
        int nc = 1;
        if (have_cells) nc = cells_around(s, &c, &x[3 * i], around);
        for (int q = 0; q < nc; ++q)
        for (int64_t j = have_cells ? c.head[around[q]] : 0; have_cells ? (j >= 0) : (j < N);
             j = have_cells ? c.next[j] : j + 1) {
            if (j == i) continue;
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 > 0.0)) continue;
            if (ptype(s, j) == T_BEAD) {
                int same = s->body[i - b0] == s->body[j - b0];
                int g = same ? (bead_level(s, level, i) == 1 ? G3_P1 : G3_P2) : G3_P2;
                if (!(due & g)) continue;
                double *f = group_array(g, f_m, f_p1, f_p2);
                double fs = 0.0;
                if (r2 < lj2 && bead_pair_allowed(s, i - b0, j - b0)) fs += lj_pair(s->lj_eps, s->lj_sig, sqrt(r2));
                /* Eq. 4 aggregation joins different platelets: group P2 with the other
                 * inter-platelet terms */
                fs += agg_pair(s, i - b0, j - b0, sqrt(r2));
                for (int k = 0; k < 3; ++k) f[3 * i + k] += fs * d[k]; /* j adds its own share */
            } else if ((due & G3_M) && (r2 < lj2 || r2 < pf2)) {
                double r = sqrt(r2), fs = 0.0;
                if (r2 < lj2) fs += lj_pair(s->lj_eps, s->lj_sig, r);
                if (r2 < pf2) {
                    double z = or_zeta((uint32_t)i, (uint32_t)j, count, s->seed, 1u);
                    fs += dpd_pair(0.0, s->gamma_pf, s->sigma_pf, s->rc_pf, r, d, &v[3 * i], &v[3 * j], z, inv_sqrt_dt);
                }
                for (int k = 0; k < 3; ++k) { f_m[3 * i + k] += fs * d[k]; f_m[3 * j + k] -= fs * d[k]; }
            }
        }
    }
    if (have_cells) cells_free(&c);
    /* frozen walls carry no force */
    if (due & G3_M)
        for (int64_t i = s->n_fluid; i < b0; ++i) f_m[3 * i] = f_m[3 * i + 1] = f_m[3 * i + 2] = 0.0;
    return 0;
}

/* n_outer outer steps of the three-level scheme.  On entry f_outer, f_m, f_p1, f_p2 hold
 * the forces of the current state; counters[0] / counters[1] count the outer and the
 * interface evaluations so far (both are updated). */
int or_respa3(const or_system *s, double *x, double *v, double *f_outer, double *f_m, double *f_p1, double *f_p2,
              uint64_t *counters, int64_t n_outer, double dt, int k, int k_if, int k_sub, const int32_t *level,
              int brute, int nthreads)
{
    if (k_sub < 1 || k_if % k_sub || k % k_if || !(dt > 0.0)) return -1;
    const double dt_f = k * dt, dt_m = k_if * dt, dt_1 = k_sub * dt;
    for (int64_t n = 0; n < n_outer; ++n) {
        kick(s, v, f_outer, 0.5 * dt_f);
        for (int a = 0; a < k / k_if; ++a) {
            kick(s, v, f_m, 0.5 * dt_m);
            for (int b = 0; b < k_if / k_sub; ++b) {
                kick(s, v, f_p1, 0.5 * dt_1);
                for (int c = 0; c < k_sub; ++c) {
                    kick(s, v, f_p2, 0.5 * dt);
                    drift(s, x, v, dt);
                    int due = G3_P2;
                    if (c == k_sub - 1) due |= G3_P1;
                    if (c == k_sub - 1 && b == k_if / k_sub - 1) due |= G3_M;
                    int rc = or_inner_forces3(s, x, v, counters[1], dt_m, level, due, brute, f_m, f_p1, f_p2);
                    if (rc) return rc;
                    if (due & G3_M) counters[1] += 1;
                    kick(s, v, f_p2, 0.5 * dt);
                }
                kick(s, v, f_p1, 0.5 * dt_1);
            }
            kick(s, v, f_m, 0.5 * dt_m);
        }
        int rc = or_outer_forces(s, x, v, counters[0], dt_f, NULL, 0, brute, nthreads, f_outer);
        if (rc) return rc;
        counters[0] += 1;
        kick(s, v, f_outer, 0.5 * dt_f);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The paper's six platelet measurements (Sec. 3.3: angular velocity   */
/* components, kinetic energies, flow speed at the centre of mass),    */
/* [P][6]:                                                              */
/*  0..2  omega = I^-1 L about the centre of mass                       */
/*  3     translational kinetic energy 1/2 M |V|^2 of the centre of mass */
/*  4     rotational kinetic energy 1/2 omega . L                       */
/*  5     flow speed at the centre of mass: |mean velocity| of the fluid */
/*        particles closer than flow_r to it (0 if there are none)      */
/* Bead positions are unwrapped about the platelet's first bead.        */
/* ------------------------------------------------------------------ */
int or_paper_features(const or_system *s, const double *x, const double *v, double flow_r, double *feat)
{
    const int64_t b0 = s->n_fluid + s->n_wall;
    const int64_t P = s->n_platelet;
    const double mb = s->mass[T_BEAD], mf = s->mass[T_FLUID];
    for (int64_t p = 0; p < P; ++p) {
        int64_t first = -1;
        double M = 0.0, off[3] = {0, 0, 0}, mom[3] = {0, 0, 0};
        for (int64_t b = 0; b < s->n_bead; ++b) {
            if (s->body[b] != p) continue;
            if (first < 0) first = b0 + b;
            double d[3];
            min_image(s, &x[3 * (b0 + b)], &x[3 * first], d);
            M += mb;
            for (int k = 0; k < 3; ++k) { off[k] += mb * d[k]; mom[k] += mb * v[3 * (b0 + b) + k]; }
        }
        double *o = &feat[6 * p];
        for (int k = 0; k < 6; ++k) o[k] = 0.0;
        if (first < 0) continue;
        double com[3], V[3];
        for (int k = 0; k < 3; ++k) { com[k] = x[3 * first + k] + off[k] / M; V[k] = mom[k] / M; }
        double L[3] = {0, 0, 0}, I[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int64_t b = 0; b < s->n_bead; ++b) {
            if (s->body[b] != p) continue;
            double r[3], u[3];
            min_image(s, &x[3 * (b0 + b)], com, r);
            for (int k = 0; k < 3; ++k) u[k] = v[3 * (b0 + b) + k] - V[k];
            L[0] += mb * (r[1] * u[2] - r[2] * u[1]);
            L[1] += mb * (r[2] * u[0] - r[0] * u[2]);
            L[2] += mb * (r[0] * u[1] - r[1] * u[0]);
            double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) I[a][c] += mb * ((a == c ? rr : 0.0) - r[a] * r[c]);
        }
        double om[3];
        solve3(I, L, om);
        double fl[3] = {0, 0, 0};
        int64_t nfl = 0;
        for (int64_t i = 0; i < s->n_fluid; ++i) {
            double d[3];
            min_image(s, &x[3 * i], com, d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < flow_r * flow_r) {
                for (int k = 0; k < 3; ++k) fl[k] += v[3 * i + k];
                ++nfl;
            }
        }
        o[0] = om[0];
        o[1] = om[1];
        o[2] = om[2];
        o[3] = 0.5 * M * (V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
        o[4] = 0.5 * (om[0] * L[0] + om[1] * L[1] + om[2] * L[2]);
        if (nfl > 0) {
            for (int k = 0; k < 3; ++k) fl[k] /= (double)nfl;
            o[5] = sqrt(fl[0] * fl[0] + fl[1] * fl[1] + fl[2] * fl[2]);
        }
        (void)mf;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-bead membrane stress (Sec. 4.2, Fig. 5): the pressure-like trace */
/* of the per-particle virial stress times volume,                     */
/*   p_i = (m |v_i|^2 + W_i) / 3,                                       */
/* W_i = sum over the conservative inner-group terms acting on bead i   */
/* of its share of r.F: 1/2 of r_ij.F_ij for WCA pairs (with fluid,     */
/* wall and bead partners), bonds, Morse bonds and Eq. 4 aggregation    */
/* pairs, 1/3 of (a.F_i + c.F_k) for every angle (a = x_i - x_j,        */
/* c = x_k - x_j about the vertex j).  out[n_bead].                     */
/* ------------------------------------------------------------------ */
int or_bead_stress(const or_system *s, const double *x, const double *v, double *out)
{
    const int64_t N = s->n_fluid + s->n_wall + s->n_bead;
    const int64_t b0 = s->n_fluid + s->n_wall;
    const double mb = s->mass[T_BEAD];
    for (int64_t b = 0; b < s->n_bead; ++b) {
        const double *u = &v[3 * (b0 + b)];
        out[b] = mb * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    for (int64_t q = 0; q < s->n_bond; ++q) {
        int64_t i = s->bond[2 * q], j = s->bond[2 * q + 1];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double w = -2.0 * s->kb * (r - s->bond_r0[q]) * r; /* r . F for U = kb (r - r0)^2 */
        out[i - b0] += 0.5 * w;
        out[j - b0] += 0.5 * w;
    }
    for (int64_t q = 0; q < s->n_morse; ++q) {
        int64_t i = s->morse[2 * q], j = s->morse[2 * q + 1];
        double d[3];
        min_image(s, &x[3 * i], &x[3 * j], d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double ex = exp(-s->morse_a * (r - s->morse_r0));
        double w = 2.0 * s->morse_a * s->morse_D * (ex * ex - ex) * r;
        out[i - b0] += 0.5 * w;
        out[j - b0] += 0.5 * w;
    }
    for (int64_t m = 0; m < s->n_angle; ++m) {
        int64_t i = s->angle[3 * m], j = s->angle[3 * m + 1], k2 = s->angle[3 * m + 2];
        double a[3], c[3];
        min_image(s, &x[3 * i], &x[3 * j], a);
        min_image(s, &x[3 * k2], &x[3 * j], c);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        double cs = (a[0] * c[0] + a[1] * c[1] + a[2] * c[2]) / (la * lc);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double th = acos(cs);
        double sn = sin(th);
        if (sn < 1e-12) sn = 1e-12;
        double pref = 2.0 * s->ka * (th - s->angle_th0[m]) / sn;
        double w = 0.0;
        for (int q = 0; q < 3; ++q) {
            double fi = pref * (c[q] / (la * lc) - cs * a[q] / (la * la));
            double fk = pref * (a[q] / (la * lc) - cs * c[q] / (lc * lc));
            w += a[q] * fi + c[q] * fk;
        }
        out[i - b0] += w / 3.0;
        out[j - b0] += w / 3.0;
        out[k2 - b0] += w / 3.0;
    }
    /* pairs of a bead with every particle: brute force */
    const double lj2 = s->lj_rc * s->lj_rc;
    for (int64_t i = b0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(s, &x[3 * i], &x[3 * j], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 > 0.0)) continue;
            double w = 0.0;
            if (ptype(s, j) == T_BEAD) {
                if (r2 < lj2 && bead_pair_allowed(s, i - b0, j - b0)) w += lj_pair(s->lj_eps, s->lj_sig, sqrt(r2)) * r2;
                w += agg_pair(s, i - b0, j - b0, sqrt(r2)) * r2;
            } else if (r2 < lj2) {
                w += lj_pair(s->lj_eps, s->lj_sig, sqrt(r2)) * r2;
            }
            out[i - b0] += 0.5 * w;
        }
    }
    for (int64_t b = 0; b < s->n_bead; ++b) out[b] /= 3.0;
    return 0;
}
