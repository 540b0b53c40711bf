/*
 * HWFV1 CPU oracle (test infrastructure only; see hwfv1_oracle.h).
 *
 * Plain FP64, single thread, one row-major array per refinement level.  The
 * code follows the paper's description step by step:
 *   - encoding with Eq. 3a-3d and the significance test (Section 2.1.2,
 *     Algorithm 1);
 *   - neighbour regularisation of the significance flags (refine the face
 *     neighbours of every cell with a significant detail);
 *   - the recursive depth-first decoding that identifies leaf cells
 *     (Section 2.1.2, Algorithm 2);
 *   - same-level neighbour finding (Section 2.1.3, Fig. 3);
 *   - the FV1 forward-Euler update of Eq. 2 with an HLL Riemann solver on a
 *     hydrostatically reconstructed, positivity-preserving, well-balanced
 *     scheme (Section 2.1.1), then the CFL timestep (Algorithm 3).
 *
 * Where the paper is silent the oracle takes these readings:
 *   - Haar taps: orthonormal (H0 = H1 = G0 = 1/sqrt2, G1 = -1/sqrt2) with an
 *     overall factor 1/2 per level, so that every s^(n) is a cell average
 *     (Section 2.1.3 uses coarse s^(n) directly as neighbour cell values).
 *     The products of taps then reduce exactly to sums scaled by 1/4.
 *   - normalised detail: max of absolute details over s_max, where s_max of
 *     a variable is max(1, max over the finest grid of |s^(L)|), taken at the
 *     start of each step (once for the bed); a cell is significant when the
 *     normalised detail of any of h, qx, qy, z is >= 2^(n-L) eps.
 *   - regularisation: one pass, a cell is kept when it or one of its four
 *     in-domain face neighbours on the same level has a significant detail.
 *   - a neighbour position below a coarser leaf takes that coarser leaf's
 *     values (h, qx, qy and z of the leaf).
 *   - FV1 operator: Audusse hydrostatic reconstruction with Toro's HLL
 *     wave-speed estimates, then rain, inflow, clipping of negative depth,
 *     zero discharge in dry cells and point-implicit Manning friction.
 *   - after the update each leaf value is copied to all its finest
 *     descendants, which is decoding with zeroed details (Algorithm 3
 *     remarks, Algorithm 4).
 *   - timestep: CFL times the finest cell size over the largest wave speed
 *     of the updated leaves, capped at dt_max (dt_max when nothing is wet);
 *     the last step is shortened to land on t_end.
 *
 * Compile with -O2 -ffp-contract=off and without fast-math: every operation
 * is a single IEEE-754 double operation in the order written.
 *
 * Parity unpinned: the change of total mass where leaf levels jump at
 * eps > 0 has no closed form to test against (its tests bound it loosely);
 * every other step is pinned by tests/test_oracle_mra.py,
 * tests/test_oracle_fv1.py and tests/test_humps.py.
 */
#include "hwfv1_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* State                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct leaf { int n; uint32_t i, j; } leaf;

struct oracle_state {
    oracle_problem p;
    int L;
    /* s^(n) for h, qx, qy, z at every level n = 0..L (row-major). */
    double* s[4][ORACLE_MAX_L + 1];
    /* Details d_alpha, d_beta, d_gamma of the last encoding, levels 0..L-1. */
    double* d[4][3][ORACLE_MAX_L];
    uint8_t* raw[ORACLE_MAX_L];   /* significant detail (incl. bed)      */
    uint8_t* sig[ORACLE_MAX_L];   /* after regularisation                */
    uint8_t* zraw[ORACLE_MAX_L];  /* static bed flags                    */
    double smax[4];
    /* Finest-grid values after the FV1 update. */
    double* fnew[3];
    leaf* leaves;
    int64_t n_leaves;
    double t, dt;
    int64_t step;
    double mass, maxspeed;
    int64_t clips, leaf_updates;
};

static size_t side(int n) { return (size_t)1 << n; }
static size_t cells(int n) { return side(n) * side(n); }
static size_t at(int n, uint32_t i, uint32_t j) { return (size_t)j * side(n) + i; }

/* ------------------------------------------------------------------------ */
/* Z-order indexing (Section 2.2.1, Fig. 5, footnote 2)                      */
/* ------------------------------------------------------------------------ */

/* Morton code: bits of i go to the even positions, bits of j to the odd
 * positions (Fig. 5: i = 1, j = 0 -> 1; i = 0, j = 1 -> 2). */
uint32_t oracle_morton(uint32_t i, uint32_t j)
{
    uint32_t m = 0;
    for (int b = 0; b < 16; ++b) {
        m |= ((i >> b) & 1u) << (2 * b);
        m |= ((j >> b) & 1u) << (2 * b + 1);
    }
    return m;
}

/* Z-order index in the hierarchy: level curves concatenated from the
 * coarsest level, so level n starts after 1 + 4 + ... + 4^(n-1) cells. */
uint64_t oracle_zindex(int n, uint32_t i, uint32_t j)
{
    uint64_t offset = 0;
    for (int k = 0; k < n; ++k) offset += (uint64_t)cells(k);
    return offset + oracle_morton(i, j);
}

/* ------------------------------------------------------------------------ */
/* Haar encoding and decoding (Section 2.1.2, Eq. 3a-3d and Eq. 4a-4d)       */
/* ------------------------------------------------------------------------ */

/* Children s[0..3]: [0] (2i, 2j), [1] (2i+1, 2j), [2] (2i, 2j+1),
 * [3] (2i+1, 2j+1), i.e. child c sits at (c & 1, c >> 1) inside the parent,
 * matching the Morton order of Fig. 5.  Eq. 3a-3d with the orthonormal taps
 * and the averaging factor 1/2:
 *   s     = 1/2 [H0 (H0 s0 + H1 s2) + H1 (H0 s1 + H1 s3)]
 *   d_a   = 1/2 [H0 (G0 s0 + G1 s2) + H1 (G0 s1 + G1 s3)]
 *   d_b   = 1/2 [G0 (H0 s0 + H1 s2) + G1 (H0 s1 + H1 s3)]
 *   d_g   = 1/2 [G0 (G0 s0 + G1 s2) + G1 (G0 s1 + G1 s3)]
 * Each tap product is 1/2 (or -1/2), so the inner brackets are the sums and
 * differences (s0 + s2), (s1 + s3), (s0 - s2), (s1 - s3) and each result is
 * 1/4 of the outer sum or difference. */
void oracle_haar_encode(const double s[4], double out[4])
{
    double a = s[0] + s[2];
    double b = s[1] + s[3];
    double ad = s[0] - s[2];
    double bd = s[1] - s[3];
    out[0] = 0.25 * (a + b);
    out[1] = 0.25 * (ad + bd);
    out[2] = 0.25 * (a - b);
    out[3] = 0.25 * (ad - bd);
}

/* Eq. 4a-4d with the inverse factor 2:
 *   s0 = (s + d_a) + (d_b + d_g)     s2 = (s - d_a) + (d_b - d_g)
 *   s1 = (s + d_a) - (d_b + d_g)     s3 = (s - d_a) - (d_b - d_g)      */
void oracle_haar_decode(const double c[4], double out[4])
{
    double sp = c[0] + c[1];
    double sm = c[0] - c[1];
    double dp = c[2] + c[3];
    double dm = c[2] - c[3];
    out[0] = sp + dp;
    out[1] = sp - dp;
    out[2] = sm + dm;
    out[3] = sm - dm;
}

static void children_of(double* const* lev, int n, uint32_t i, uint32_t j,
                        double ch[4])
{
    const double* f = lev[n + 1];
    ch[0] = f[at(n + 1, 2 * i, 2 * j)];
    ch[1] = f[at(n + 1, 2 * i + 1, 2 * j)];
    ch[2] = f[at(n + 1, 2 * i, 2 * j + 1)];
    ch[3] = f[at(n + 1, 2 * i + 1, 2 * j + 1)];
}

static double max_abs_finest(const double* f, size_t count)
{
    double m = 0.0;
    for (size_t k = 0; k < count; ++k) {
        double a = fabs(f[k]);
        if (a > m) m = a;
    }
    return m;
}

/* s_max of Section 2.1.2, guarded below by 1 (reading). */
static double guarded_smax(const double* f, size_t count)
{
    double m = max_abs_finest(f, count);
    return m > 1.0 ? m : 1.0;
}

/* Algorithm 1 for one variable: for each level from L-1 down to 0 and each
 * cell, load the children, apply Eq. 3a-3d, form the normalised detail and
 * flag the cell when it reaches 2^(n-L) eps.  Flags are OR-ed into flag[]. */
static void encode_variable(oracle_state* st, int var, uint8_t** flag)
{
    int L = st->L;
    for (int n = L - 1; n >= 0; --n) {
        double threshold = ldexp(st->p.eps, n - L);
        for (uint32_t j = 0; j < side(n); ++j) {
            for (uint32_t i = 0; i < side(n); ++i) {
                double ch[4], c[4];
                children_of(st->s[var], n, i, j, ch);
                oracle_haar_encode(ch, c);
                size_t k = at(n, i, j);
                st->s[var][n][k] = c[0];
                st->d[var][0][n][k] = c[1];
                st->d[var][1][n][k] = c[2];
                st->d[var][2][n][k] = c[3];
                double a = fabs(c[1]);
                double b = fabs(c[2]);
                double g = fabs(c[3]);
                double dmax = a > b ? a : b;
                dmax = dmax > g ? dmax : g;
                double dnorm = dmax / st->smax[var];
                if (dnorm >= threshold) flag[n][k] = 1;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Allocation and ingest                                                     */
/* ------------------------------------------------------------------------ */

static int alloc_state(oracle_state* st)
{
    int L = st->L;
    for (int v = 0; v < 4; ++v)
        for (int n = 0; n <= L; ++n)
            if (!(st->s[v][n] = calloc(cells(n), sizeof(double)))) return 0;
    for (int v = 0; v < 4; ++v)
        for (int q = 0; q < 3; ++q)
            for (int n = 0; n < L; ++n)
                if (!(st->d[v][q][n] = calloc(cells(n), sizeof(double))))
                    return 0;
    for (int n = 0; n < L; ++n) {
        if (!(st->raw[n] = calloc(cells(n), 1))) return 0;
        if (!(st->sig[n] = calloc(cells(n), 1))) return 0;
        if (!(st->zraw[n] = calloc(cells(n), 1))) return 0;
    }
    for (int v = 0; v < 3; ++v)
        if (!(st->fnew[v] = calloc(cells(L), sizeof(double)))) return 0;
    if (!(st->leaves = calloc(cells(L), sizeof(leaf)))) return 0;
    return 1;
}

void oracle_destroy(oracle_state* st)
{
    if (!st) return;
    for (int v = 0; v < 4; ++v)
        for (int n = 0; n <= ORACLE_MAX_L; ++n) free(st->s[v][n]);
    for (int v = 0; v < 4; ++v)
        for (int q = 0; q < 3; ++q)
            for (int n = 0; n < ORACLE_MAX_L; ++n) free(st->d[v][q][n]);
    for (int n = 0; n < ORACLE_MAX_L; ++n) {
        free(st->raw[n]);
        free(st->sig[n]);
        free(st->zraw[n]);
    }
    for (int v = 0; v < 3; ++v) free(st->fnew[v]);
    free(st->leaves);
    free(st);
}

static double velocity(double h, double q, double h_tol)
{
    return h > h_tol ? q / h : 0.0;
}

/* Largest wave speed max(|u| + sqrt(g h), |v| + sqrt(g h)) of a wet cell. */
static double wave_speed(const oracle_problem* p, double h, double qx,
                         double qy)
{
    if (!(h > p->h_tol)) return 0.0;
    double c = sqrt(p->g * h);
    double u = qx / h;
    double v = qy / h;
    double su = fabs(u) + c;
    double sv = fabs(v) + c;
    return su > sv ? su : sv;
}

/* CFL timestep (Algorithm 3, timestep line): CFL times the finest cell size
 * over the largest wave speed, capped at dt_max (which is also the step when
 * nothing is wet). */
static double cfl_dt(const oracle_problem* p, double maxspeed)
{
    double dmin = p->dx < p->dy ? p->dx : p->dy;
    if (maxspeed > 0.0) {
        double dt = p->cfl * dmin / maxspeed;
        return dt < p->dt_max ? dt : p->dt_max;
    }
    return p->dt_max;
}

static double clamp_to_end(const oracle_problem* p, double t, double dt)
{
    double rest = p->t_end - t;
    return dt < rest ? dt : rest;
}

oracle_state* oracle_create(const oracle_problem* p, const double* h,
                            const double* qx, const double* qy,
                            const double* z)
{
    if (!p || p->L < 1 || p->L > ORACLE_MAX_L || !(p->eps >= 0.0)) return NULL;
    if (!(p->zsmax >= 0.0) || !isfinite(p->zsmax)) return NULL;
    oracle_state* st = calloc(1, sizeof(oracle_state));
    if (!st) return NULL;
    st->p = *p;
    st->L = p->L;
    if (!alloc_state(st)) { oracle_destroy(st); return NULL; }
    int L = st->L;
    size_t N = cells(L);
    /* Initial discretisation on the finest grid (Algorithm 3). */
    memcpy(st->s[0][L], h, N * sizeof(double));
    memcpy(st->s[1][L], qx, N * sizeof(double));
    memcpy(st->s[2][L], qy, N * sizeof(double));
    memcpy(st->s[3][L], z, N * sizeof(double));
    /* Static bed: encode once and keep its significance flags.  s_max of
     * the bed is the largest finest coefficient of the domain: over the
     * whole grid, unless the caller gives the value of a domain that was
     * padded to the square grid. */
    st->smax[3] = p->zsmax > 0.0 ? p->zsmax : guarded_smax(st->s[3][L], N);
    encode_variable(st, 3, st->zraw);
    double maxspeed = 0.0;
    for (size_t k = 0; k < N; ++k) {
        double w = wave_speed(p, h[k], qx[k], qy[k]);
        if (w > maxspeed) maxspeed = w;
    }
    st->t = 0.0;
    st->dt = clamp_to_end(p, 0.0, cfl_dt(p, maxspeed));
    st->maxspeed = maxspeed;
    st->step = 0;
    double mass = 0.0;
    for (size_t k = 0; k < N; ++k) mass += (h[k] * p->dx) * p->dy;
    st->mass = mass;
    return st;
}

void oracle_set_time(oracle_state* st, double t, double dt, int64_t step)
{
    st->t = t;
    st->dt = dt;
    st->step = step;
}

/* ------------------------------------------------------------------------ */
/* Phase 1: encoding of the flow variables with significance flags           */
/* ------------------------------------------------------------------------ */

void oracle_phase_encode(oracle_state* st)
{
    int L = st->L;
    size_t N = cells(L);
    for (int v = 0; v < 3; ++v) st->smax[v] = guarded_smax(st->s[v][L], N);
    for (int n = 0; n < L; ++n) memcpy(st->raw[n], st->zraw[n], cells(n));
    for (int v = 0; v < 3; ++v) encode_variable(st, v, st->raw);
}

/* ------------------------------------------------------------------------ */
/* Phase 2: regularisation                                                   */
/* ------------------------------------------------------------------------ */

void oracle_phase_regularise(oracle_state* st)
{
    for (int n = 0; n < st->L; ++n) {
        uint32_t S = (uint32_t)side(n);
        for (uint32_t j = 0; j < S; ++j) {
            for (uint32_t i = 0; i < S; ++i) {
                uint8_t f = st->raw[n][at(n, i, j)];
                if (i > 0) f |= st->raw[n][at(n, i - 1, j)];
                if (i + 1 < S) f |= st->raw[n][at(n, i + 1, j)];
                if (j > 0) f |= st->raw[n][at(n, i, j - 1)];
                if (j + 1 < S) f |= st->raw[n][at(n, i, j + 1)];
                st->sig[n][at(n, i, j)] = f ? 1 : 0;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Phase 3: depth-first decoding (Algorithm 2)                                */
/* ------------------------------------------------------------------------ */

/* The cell is a leaf when it is on the finest grid or its detail is not
 * significant; otherwise visit the four children in the order 0, 1, 2, 3.
 * (The children's values are already available from encoding, which is what
 * Eq. 4a-4d would reproduce.) */
static void dft(oracle_state* st, int n, uint32_t i, uint32_t j)
{
    if (n == st->L || !st->sig[n][at(n, i, j)]) {
        leaf* lf = &st->leaves[st->n_leaves++];
        lf->n = n;
        lf->i = i;
        lf->j = j;
        return;
    }
    dft(st, n + 1, 2 * i, 2 * j);
    dft(st, n + 1, 2 * i + 1, 2 * j);
    dft(st, n + 1, 2 * i, 2 * j + 1);
    dft(st, n + 1, 2 * i + 1, 2 * j + 1);
}

void oracle_phase_traverse(oracle_state* st)
{
    st->n_leaves = 0;
    dft(st, 0, 0, 0);
}

/* ------------------------------------------------------------------------ */
/* Phase 4: FV1 update on the leaves                                         */
/* ------------------------------------------------------------------------ */

typedef struct cstate { double h, qx, qy, z; } cstate;

static cstate value_at(const oracle_state* st, int n, uint32_t i, uint32_t j)
{
    cstate c;
    size_t k = at(n, i, j);
    c.h = st->s[0][n][k];
    c.qx = st->s[1][n][k];
    c.qy = st->s[2][n][k];
    c.z = st->s[3][n][k];
    return c;
}

/* Neighbour finding (Section 2.1.3, Fig. 3): the neighbour of a leaf in a
 * direction is the cell of the same level on that side.  If that cell lies
 * below a coarser leaf (an ancestor on its path is not significant), the
 * coarser leaf is used.  Outside the domain a ghost copy of the leaf is
 * used, with the normal discharge negated at a wall. */
static cstate neighbour(const oracle_state* st, int m, uint32_t i, uint32_t j,
                        int dir, cstate own)
{
    int64_t ii = i, jj = j;
    if (dir == OR_W) ii -= 1;
    if (dir == OR_E) ii += 1;
    if (dir == OR_S) jj -= 1;
    if (dir == OR_N) jj += 1;
    int64_t S = (int64_t)side(m);
    if (ii < 0 || ii >= S || jj < 0 || jj >= S) {
        cstate g = own;
        if (st->p.bc[dir] == OR_BC_WALL) {
            if (dir == OR_W || dir == OR_E) g.qx = -g.qx;
            else g.qy = -g.qy;
        }
        return g;
    }
    for (int n = 0; n < m; ++n) {
        uint32_t in = (uint32_t)(ii >> (m - n));
        uint32_t jn = (uint32_t)(jj >> (m - n));
        if (!st->sig[n][at(n, in, jn)]) return value_at(st, n, in, jn);
    }
    return value_at(st, m, (uint32_t)ii, (uint32_t)jj);
}

/* One face between a left state l and a right state r, written for the
 * x direction (normal discharge qn, tangential discharge qt).
 *  Hydrostatic reconstruction (Audusse et al. 2004): with the face bed
 *  max(z_l, z_r), the reconstructed depths are h - max(0, z_other - z_own)
 *  clipped at zero, which is max(0, eta - z_face) without forming eta.
 *  HLL flux (Harten, Lax, van Leer; wave speeds after Toro) on the
 *  reconstructed states, with the dry-side speeds u -/+ 2c. */
static void face_flux(const oracle_problem* p, double hl, double qnl,
                      double qtl, double zl, double hr, double qnr,
                      double qtr, double zr, double F[3], double* hls_out,
                      double* hrs_out)
{
    double g = p->g;
    double tol = p->h_tol;
    double unl = velocity(hl, qnl, tol);
    double utl = velocity(hl, qtl, tol);
    double unr = velocity(hr, qnr, tol);
    double utr = velocity(hr, qtr, tol);
    double dzl = zr - zl;
    double dzr = zl - zr;
    double hls = hl - (dzl > 0.0 ? dzl : 0.0);
    double hrs = hr - (dzr > 0.0 ? dzr : 0.0);
    if (!(hls > 0.0)) hls = 0.0;
    if (!(hrs > 0.0)) hrs = 0.0;
    *hls_out = hls;
    *hrs_out = hrs;
    if (hls <= tol && hrs <= tol) {
        F[0] = 0.0;
        F[1] = 0.0;
        F[2] = 0.0;
        return;
    }
    double cl = sqrt(g * hls);
    double cr = sqrt(g * hrs);
    double ustar = 0.5 * (unl + unr) + cl - cr;
    double cstar = 0.5 * (cl + cr) + 0.25 * (unl - unr);
    double sl, sr;
    if (hls <= tol) {
        sl = unr - 2.0 * cr;
    } else {
        double a = unl - cl;
        double b = ustar - cstar;
        sl = a < b ? a : b;
    }
    if (hrs <= tol) {
        sr = unl + 2.0 * cl;
    } else {
        double a = unr + cr;
        double b = ustar + cstar;
        sr = a > b ? a : b;
    }
    double ql = hls * unl;
    double qr = hrs * unr;
    double Ul[3] = { hls, ql, hls * utl };
    double Ur[3] = { hrs, qr, hrs * utr };
    double Fl[3] = { ql, ql * unl + 0.5 * g * hls * hls, ql * utl };
    double Fr[3] = { qr, qr * unr + 0.5 * g * hrs * hrs, qr * utr };
    if (sl >= 0.0) {
        F[0] = Fl[0]; F[1] = Fl[1]; F[2] = Fl[2];
    } else if (sr <= 0.0) {
        F[0] = Fr[0]; F[1] = Fr[1]; F[2] = Fr[2];
    } else {
        double slsr = sl * sr;
        double den = sr - sl;
        for (int k = 0; k < 3; ++k)
            F[k] = ((sr * Fl[k] - sl * Fr[k]) + slsr * (Ur[k] - Ul[k])) / den;
    }
}

void oracle_face_flux(const oracle_problem* p, const double left[4],
                      const double right[4], double flux[3], double hstar[2])
{
    face_flux(p, left[0], left[1], left[2], left[3], right[0], right[1],
              right[2], right[3], flux, &hstar[0], &hstar[1]);
}

/* Triangular inflow hydrograph Q(t). */
static double inflow_rate(const oracle_problem* p, double t)
{
    if (!(p->q_peak > 0.0)) return 0.0;
    if (t <= p->t_peak) return p->q_peak * t / p->t_peak;
    if (t <= p->t_base)
        return p->q_peak * (p->t_base - t) / (p->t_base - p->t_peak);
    return 0.0;
}

/* FV1 update of one cell of size dxm x dym given its state and its four
 * neighbour states (Eq. 2, forward Euler), followed by the source terms. */
static void fv1_cell(const oracle_problem* p, double dt, double t,
                     double dxm, double dym, int west_edge, double y_lo,
                     cstate c, cstate w, cstate e, cstate s, cstate nn,
                     double out[3], int64_t* clips)
{
    double FE[3], FW[3], GN[3], GS[3];
    double hcE, hcW, hcN, hcS, unused;
    /* x faces: normal discharge qx, tangential qy. */
    face_flux(p, c.h, c.qx, c.qy, c.z, e.h, e.qx, e.qy, e.z, FE, &hcE,
              &unused);
    face_flux(p, w.h, w.qx, w.qy, w.z, c.h, c.qx, c.qy, c.z, FW, &unused,
              &hcW);
    /* y faces: normal discharge qy, tangential qx. */
    face_flux(p, c.h, c.qy, c.qx, c.z, nn.h, nn.qy, nn.qx, nn.z, GN, &hcN,
              &unused);
    face_flux(p, s.h, s.qy, s.qx, s.z, c.h, c.qy, c.qx, c.z, GS, &unused,
              &hcS);
    /* Bed-slope source in Audusse form: the pressure of the own depth minus
     * that of the reconstructed depth on each face. */
    double hg = 0.5 * p->g;
    double h2 = c.h * c.h;
    double PE = hg * (h2 - hcE * hcE);
    double PW = hg * (h2 - hcW * hcW);
    double PN = hg * (h2 - hcN * hcN);
    double PS = hg * (h2 - hcS * hcS);
    double rx = dt / dxm;
    double ry = dt / dym;
    double h = c.h - rx * (FE[0] - FW[0]) - ry * (GN[0] - GS[0]);
    double qx = c.qx - rx * ((FE[1] + PE) - (FW[1] + PW))
                - ry * (GN[2] - GS[2]);
    double qy = c.qy - rx * (FE[2] - FW[2])
                - ry * ((GN[1] + PN) - (GS[1] + PS));
    /* Rain (uniform mass source). */
    if (p->rain_rate != 0.0) h = h + dt * p->rain_rate;
    /* West-edge inflow: the hydrograph spread over the inlet segment. */
    if (west_edge && p->q_peak > 0.0) {
        double lo = y_lo > p->inlet_y0 ? y_lo : p->inlet_y0;
        double yhi = y_lo + dym;
        double hi = yhi < p->inlet_y1 ? yhi : p->inlet_y1;
        double overlap = hi - lo;
        if (overlap > 0.0) {
            double width = p->inlet_y1 - p->inlet_y0;
            double q = inflow_rate(p, t);
            h = h + dt * q * overlap / (width * dxm * dym);
        }
    }
    /* Positivity: clip negative depths. */
    if (h < 0.0) {
        h = 0.0;
        *clips += 1;
    }
    /* Dry cells carry no discharge. */
    if (h <= p->h_tol) {
        qx = 0.0;
        qy = 0.0;
    } else if (p->manning_n > 0.0) {
        /* Manning friction of Eq. 1, point-implicit:
         * q_new = q / (1 + dt C_f |u| / h), C_f = g n^2 / h^(1/3). */
        double speed = sqrt(qx * qx + qy * qy) / h;
        double cf = p->g * p->manning_n * p->manning_n / cbrt(h);
        double den = 1.0 + dt * cf * speed / h;
        qx = qx / den;
        qy = qy / den;
    }
    out[0] = h;
    out[1] = qx;
    out[2] = qy;
}

/* Write the new leaf value into every finest cell it covers (decoding with
 * zero details). */
static void copy_down(oracle_state* st, int m, uint32_t i, uint32_t j,
                      const double v[3])
{
    int L = st->L;
    uint32_t w = 1u << (L - m);
    for (uint32_t jj = j * w; jj < (j + 1) * w; ++jj)
        for (uint32_t ii = i * w; ii < (i + 1) * w; ++ii)
            for (int q = 0; q < 3; ++q) st->fnew[q][at(L, ii, jj)] = v[q];
}

static void finish_step(oracle_state* st, double maxspeed, double mass)
{
    int L = st->L;
    size_t N = cells(L);
    for (int q = 0; q < 3; ++q)
        memcpy(st->s[q][L], st->fnew[q], N * sizeof(double));
    st->t = st->t + st->dt;
    st->maxspeed = maxspeed;
    st->mass = mass;
    st->dt = clamp_to_end(&st->p, st->t, cfl_dt(&st->p, maxspeed));
    st->step += 1;
}

void oracle_phase_fv1(oracle_state* st)
{
    const oracle_problem* p = &st->p;
    int L = st->L;
    double maxspeed = 0.0, mass = 0.0;
    for (int64_t k = 0; k < st->n_leaves; ++k) {
        leaf lf = st->leaves[k];
        int m = lf.n;
        double dxm = ldexp(p->dx, L - m);
        double dym = ldexp(p->dy, L - m);
        cstate c = value_at(st, m, lf.i, lf.j);
        cstate w = neighbour(st, m, lf.i, lf.j, OR_W, c);
        cstate e = neighbour(st, m, lf.i, lf.j, OR_E, c);
        cstate s = neighbour(st, m, lf.i, lf.j, OR_S, c);
        cstate nn = neighbour(st, m, lf.i, lf.j, OR_N, c);
        double out[3];
        fv1_cell(p, st->dt, st->t, dxm, dym, lf.i == 0, (double)lf.j * dym,
                 c, w, e, s, nn, out, &st->clips);
        copy_down(st, m, lf.i, lf.j, out);
        double ws = wave_speed(p, out[0], out[1], out[2]);
        if (ws > maxspeed) maxspeed = ws;
        mass += (out[0] * dxm) * dym;
    }
    st->leaf_updates += st->n_leaves;
    finish_step(st, maxspeed, mass);
}

int oracle_step(oracle_state* st)
{
    if (!(st->t < st->p.t_end)) return 0;
    oracle_phase_encode(st);
    oracle_phase_regularise(st);
    oracle_phase_traverse(st);
    oracle_phase_fv1(st);
    return 1;
}

int64_t oracle_run(oracle_state* st, int64_t max_steps)
{
    int64_t k = 0;
    while (k < max_steps && oracle_step(st)) ++k;
    return k;
}

/* Uniform-grid FV1 on the finest grid: every finest cell is updated with its
 * direct neighbours.  Used as the eps = 0 reference. */
void oracle_uniform_fv1_step(oracle_state* st)
{
    const oracle_problem* p = &st->p;
    int L = st->L;
    uint32_t S = (uint32_t)side(L);
    double maxspeed = 0.0, mass = 0.0;
    for (uint32_t j = 0; j < S; ++j) {
        for (uint32_t i = 0; i < S; ++i) {
            cstate c = value_at(st, L, i, j);
            cstate w, e, s, nn;
            if (i > 0) w = value_at(st, L, i - 1, j);
            else { w = c; if (p->bc[OR_W] == OR_BC_WALL) w.qx = -w.qx; }
            if (i + 1 < S) e = value_at(st, L, i + 1, j);
            else { e = c; if (p->bc[OR_E] == OR_BC_WALL) e.qx = -e.qx; }
            if (j > 0) s = value_at(st, L, i, j - 1);
            else { s = c; if (p->bc[OR_S] == OR_BC_WALL) s.qy = -s.qy; }
            if (j + 1 < S) nn = value_at(st, L, i, j + 1);
            else { nn = c; if (p->bc[OR_N] == OR_BC_WALL) nn.qy = -nn.qy; }
            double out[3];
            fv1_cell(p, st->dt, st->t, p->dx, p->dy, i == 0,
                     (double)j * p->dy, c, w, e, s, nn, out, &st->clips);
            for (int q = 0; q < 3; ++q) st->fnew[q][at(L, i, j)] = out[q];
            double ws = wave_speed(p, out[0], out[1], out[2]);
            if (ws > maxspeed) maxspeed = ws;
            mass += (out[0] * p->dx) * p->dy;
        }
    }
    st->leaf_updates += (int64_t)cells(L);
    st->n_leaves = (int64_t)cells(L);
    finish_step(st, maxspeed, mass);
}

/* ------------------------------------------------------------------------ */
/* Whole-field round trip (Eq. 3 then Eq. 4, Algorithm 1 then Algorithm 4)   */
/* ------------------------------------------------------------------------ */

void oracle_roundtrip(int L, const double* f, double* out)
{
    double* lev[ORACLE_MAX_L + 1] = { 0 };
    double* det[3][ORACLE_MAX_L] = { { 0 } };
    for (int n = 0; n <= L; ++n) lev[n] = calloc(cells(n), sizeof(double));
    for (int q = 0; q < 3; ++q)
        for (int n = 0; n < L; ++n) det[q][n] = calloc(cells(n), sizeof(double));
    memcpy(lev[L], f, cells(L) * sizeof(double));
    for (int n = L - 1; n >= 0; --n) {
        for (uint32_t j = 0; j < side(n); ++j) {
            for (uint32_t i = 0; i < side(n); ++i) {
                double ch[4], c[4];
                children_of(lev, n, i, j, ch);
                oracle_haar_encode(ch, c);
                size_t k = at(n, i, j);
                lev[n][k] = c[0];
                det[0][n][k] = c[1];
                det[1][n][k] = c[2];
                det[2][n][k] = c[3];
            }
        }
    }
    /* Decode from the coarsest level, overwriting the finer levels. */
    for (int n = 0; n < L; ++n) {
        for (uint32_t j = 0; j < side(n); ++j) {
            for (uint32_t i = 0; i < side(n); ++i) {
                size_t k = at(n, i, j);
                double c[4] = { lev[n][k], det[0][n][k], det[1][n][k],
                                det[2][n][k] };
                double ch[4];
                oracle_haar_decode(c, ch);
                lev[n + 1][at(n + 1, 2 * i, 2 * j)] = ch[0];
                lev[n + 1][at(n + 1, 2 * i + 1, 2 * j)] = ch[1];
                lev[n + 1][at(n + 1, 2 * i, 2 * j + 1)] = ch[2];
                lev[n + 1][at(n + 1, 2 * i + 1, 2 * j + 1)] = ch[3];
            }
        }
    }
    memcpy(out, lev[L], cells(L) * sizeof(double));
    for (int n = 0; n <= L; ++n) free(lev[n]);
    for (int q = 0; q < 3; ++q)
        for (int n = 0; n < L; ++n) free(det[q][n]);
}

/* ------------------------------------------------------------------------ */
/* Getters                                                                   */
/* ------------------------------------------------------------------------ */

void oracle_get_fine(const oracle_state* st, double* h, double* qx,
                     double* qy)
{
    size_t N = cells(st->L);
    memcpy(h, st->s[0][st->L], N * sizeof(double));
    memcpy(qx, st->s[1][st->L], N * sizeof(double));
    memcpy(qy, st->s[2][st->L], N * sizeof(double));
}

void oracle_get_hierarchy(const oracle_state* st, int var, double* out)
{
    for (int n = 0; n <= st->L; ++n)
        for (uint32_t j = 0; j < side(n); ++j)
            for (uint32_t i = 0; i < side(n); ++i)
                out[oracle_zindex(n, i, j)] = st->s[var][n][at(n, i, j)];
}

void oracle_get_details(const oracle_state* st, int var, double* out)
{
    size_t ncoarse = 0;
    for (int n = 0; n < st->L; ++n) ncoarse += cells(n);
    for (int q = 0; q < 3; ++q)
        for (int n = 0; n < st->L; ++n)
            for (uint32_t j = 0; j < side(n); ++j)
                for (uint32_t i = 0; i < side(n); ++i)
                    out[q * ncoarse + oracle_zindex(n, i, j)] =
                        st->d[var][q][n][at(n, i, j)];
}

void oracle_get_flags(const oracle_state* st, int which, uint8_t* out)
{
    for (int n = 0; n < st->L; ++n) {
        const uint8_t* src = which == 0 ? st->raw[n]
                           : which == 1 ? st->sig[n] : st->zraw[n];
        for (uint32_t j = 0; j < side(n); ++j)
            for (uint32_t i = 0; i < side(n); ++i)
                out[oracle_zindex(n, i, j)] = src[at(n, i, j)];
    }
}

int64_t oracle_get_leaves(const oracle_state* st, uint32_t* idx)
{
    if (idx)
        for (int64_t k = 0; k < st->n_leaves; ++k) {
            leaf lf = st->leaves[k];
            idx[k] = (uint32_t)oracle_zindex(lf.n, lf.i, lf.j);
        }
    return st->n_leaves;
}

void oracle_get_scalars(const oracle_state* st, double* out)
{
    out[OR_SC_T] = st->t;
    out[OR_SC_DT] = st->dt;
    out[OR_SC_STEP] = (double)st->step;
    out[OR_SC_NLEAVES] = (double)st->n_leaves;
    out[OR_SC_MASS] = st->mass;
    out[OR_SC_CLIPS] = (double)st->clips;
    out[OR_SC_MAXSPEED] = st->maxspeed;
    out[OR_SC_LEAF_UPDATES] = (double)st->leaf_updates;
    out[OR_SC_SMAX_H] = st->smax[0];
    out[OR_SC_SMAX_QX] = st->smax[1];
    out[OR_SC_SMAX_QY] = st->smax[2];
    out[OR_SC_SMAX_Z] = st->smax[3];
}

/* ------------------------------------------------------------------------ */
/* Flag-level entry points for the traversal and regularisation pins         */
/* ------------------------------------------------------------------------ */

static oracle_state* flags_only_state(int L)
{
    if (L < 1 || L > ORACLE_MAX_L) return NULL;
    oracle_state* st = calloc(1, sizeof(oracle_state));
    if (!st) return NULL;
    st->L = L;
    for (int n = 0; n < L; ++n) {
        st->raw[n] = calloc(cells(n), 1);
        st->sig[n] = calloc(cells(n), 1);
        if (!st->raw[n] || !st->sig[n]) { oracle_destroy(st); return NULL; }
    }
    st->leaves = calloc(cells(L), sizeof(leaf));
    if (!st->leaves) { oracle_destroy(st); return NULL; }
    return st;
}

int64_t oracle_dft_from_flags(int L, const uint8_t* sig, uint32_t* leaves)
{
    oracle_state* st = flags_only_state(L);
    if (!st) return -1;
    for (int n = 0; n < L; ++n)
        for (uint32_t j = 0; j < side(n); ++j)
            for (uint32_t i = 0; i < side(n); ++i)
                st->sig[n][at(n, i, j)] = sig[oracle_zindex(n, i, j)] ? 1 : 0;
    oracle_phase_traverse(st);
    int64_t count = oracle_get_leaves(st, leaves);
    oracle_destroy(st);
    return count;
}

void oracle_regularise_flags(int L, const uint8_t* raw, uint8_t* sig)
{
    oracle_state* st = flags_only_state(L);
    if (!st) return;
    for (int n = 0; n < L; ++n)
        for (uint32_t j = 0; j < side(n); ++j)
            for (uint32_t i = 0; i < side(n); ++i)
                st->raw[n][at(n, i, j)] = raw[oracle_zindex(n, i, j)] ? 1 : 0;
    oracle_phase_regularise(st);
    oracle_get_flags(st, 1, sig);
    oracle_destroy(st);
}
