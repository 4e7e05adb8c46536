/*
 * aw_oracle.c -- plain FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code, header, table or constant
 * generator with the HIP library; the two agree only through the seeded
 * counter-based generator below, which each side implements on its own from
 * the published definition of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).
 *
 * What it computes (arXiv:1107.4107):
 *   - Model, eqs. 1-2 (section "Model for Arnold Diffusion"):
 *         H(P, X) = |P|^2 / 2 + eps * Hp(X),
 *         Hp(x, y, z) = cos x * cos y * (1 + cos 2z),  M = 3.
 *   - Propagation by a symplectic map (section "Computational method"): the
 *     paper uses a 6th-order symplectic integrator whose reference is not
 *     recoverable.  The reading taken here is the closed-form triple-jump
 *     composition built on the second-order drift-kick-drift (Stormer-Verlet)
 *     step:  S2(t) = D(t/2) K(t) D(t/2),  S4(t) = S2(g1 t) S2(g0 t) S2(g1 t),
 *     S6(t) = S4(d1 t) S4(d0 t) S4(d1 t), g1 = 1/(2 - 2^(1/3)), g0 = 1 - 2 g1,
 *     d1 = 1/(2 - 2^(1/5)), d0 = 1 - 2 d1.  The first-order member kick-then-
 *     drift (STDMAP) is the coupled standard map the model section names.
 *     The composition is applied literally (no merging of adjacent drifts).
 *     A second 6th-order member (Y6) composes seven S2 steps symmetrically,
 *     S2(w3 t) S2(w2 t) S2(w1 t) S2(w0 t) S2(w1 t) S2(w2 t) S2(w3 t), with the
 *     weights solved here from the order conditions (see y6_conditions).
 *   - Per-orbit observables: the finite-time mean velocity
 *     V = [X(t + dt) - X(t)] / dt on the unwrapped coordinates (section "Main
 *     results"), the momentum drift |P(t) - P(0)|^2 (model section), and a
 *     tangent-vector growth L = ln |w_T| / |w_0| (the finite-time Lyapunov
 *     exponent the conclusions name), renormalised after every step.
 *   - Forward-mode derivatives of the step-averaged momentum drift
 *     J = (1/T) sum_k |P_k - P_0|^2 with respect to the six initial
 *     coordinates and eps (seven tangent columns).
 *   - Forward-over-forward derivatives of the tangent-growth indicator
 *     L = ln(|w_T| / |w_0|) with respect to the same seven parameters: the
 *     tangent equations differentiated once more, which brings in the third
 *     derivatives of Hp.
 *   - Histograms of per-orbit values over two key coordinates, and the
 *     equal-area histogram of the direction of V on the momentum sphere (the
 *     density F of the "Main results" section and Figs. 2-4).
 *
 * Everything is IEEE binary64, built with -ffp-contract=off; sin and cos are
 * libm's, applied to the unwrapped coordinates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_STDMAP 1
#define OR_S2 2
#define OR_S4 4
#define OR_S6 6
#define OR_Y6 7

/* Number of doubles in a resumable per-orbit record:
 * X[3] P[3] w[6] X0[3] P0[3] L Jsum steps. */
#define OR_REC 21

/* Rows of the per-orbit output. */
#define OR_L 0
#define OR_LAMBDA 1
#define OR_CHI 2
#define OR_VX 3
#define OR_VY 4
#define OR_VZ 5
#define OR_DP2 6
#define OR_J 7
#define OR_DE 8
#define OR_NOUT 9

/* pi rounded to double (the value of the POSIX M_PI). */
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Eq. 2 and its first and second derivatives, written from the formula.    */
/* ------------------------------------------------------------------------ */

static double hp_value(const double X[3])
{
    return cos(X[0]) * cos(X[1]) * (1.0 + cos(2.0 * X[2]));
}

/* g = grad Hp(X). */
static void hp_gradient(const double X[3], double g[3])
{
    double cx = cos(X[0]), sx = sin(X[0]);
    double cy = cos(X[1]), sy = sin(X[1]);
    double c2z = cos(2.0 * X[2]), s2z = sin(2.0 * X[2]);
    g[0] = -sx * cy * (1.0 + c2z);
    g[1] = -cx * sy * (1.0 + c2z);
    g[2] = -2.0 * cx * cy * s2z;
}

/* Hs = Hessian of Hp at X, as a full symmetric 3x3 matrix. */
static void hp_hessian(const double X[3], double Hs[3][3])
{
    double cx = cos(X[0]), sx = sin(X[0]);
    double cy = cos(X[1]), sy = sin(X[1]);
    double c2z = cos(2.0 * X[2]), s2z = sin(2.0 * X[2]);
    Hs[0][0] = -cx * cy * (1.0 + c2z);
    Hs[1][1] = -cx * cy * (1.0 + c2z);
    Hs[2][2] = -4.0 * cx * cy * c2z;
    Hs[0][1] = sx * sy * (1.0 + c2z);
    Hs[0][2] = 2.0 * sx * cy * s2z;
    Hs[1][2] = 2.0 * cx * sy * s2z;
    Hs[1][0] = Hs[0][1];
    Hs[2][0] = Hs[0][2];
    Hs[2][1] = Hs[1][2];
}

/* T3[i][j][k] = d^3 Hp / dx_i dx_j dx_k at X (full symmetric array), from
 * Hp = cx cy (1 + c2z):
 *   xxx = xyy = sx cy (1 + c2z)     xxy = yyy = cx sy (1 + c2z)
 *   xxz = yyz = 2 cx cy s2z         xyz = -2 sx sy s2z
 *   xzz = 4 sx cy c2z               yzz = 4 cx sy c2z
 *   zzz = 8 cx cy s2z */
static void hp_third(const double X[3], double T3[3][3][3])
{
    double cx = cos(X[0]), sx = sin(X[0]);
    double cy = cos(X[1]), sy = sin(X[1]);
    double c2z = cos(2.0 * X[2]), s2z = sin(2.0 * X[2]);
    double v[3][3][3];
    v[0][0][0] = sx * cy * (1.0 + c2z);
    v[0][0][1] = cx * sy * (1.0 + c2z);
    v[0][0][2] = 2.0 * cx * cy * s2z;
    v[0][1][1] = sx * cy * (1.0 + c2z);
    v[0][1][2] = -2.0 * sx * sy * s2z;
    v[0][2][2] = 4.0 * sx * cy * c2z;
    v[1][1][1] = cx * sy * (1.0 + c2z);
    v[1][1][2] = 2.0 * cx * cy * s2z;
    v[1][2][2] = 4.0 * cx * sy * c2z;
    v[2][2][2] = 8.0 * cx * cy * s2z;
    /* fill every permutation from the sorted-index entries */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) {
                int a = i, b = j, c = k, t;
                if (a > b) { t = a; a = b; b = t; }
                if (b > c) { t = b; b = c; c = t; }
                if (a > b) { t = a; a = b; b = t; }
                T3[i][j][k] = v[a][b][c];
            }
}

/* Eq. 1: total energy of s = (x, y, z, px, py, pz). */
static double energy(const double s[6], double eps)
{
    double p2 = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    return 0.5 * p2 + eps * hp_value(s);
}

/* ------------------------------------------------------------------------ */
/* One orbit with an optional set of tangent columns.                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double s[6];      /* x y z (unwrapped) px py pz */
    int ncol;         /* number of tangent columns */
    int eps_col;      /* index of the column that carries d/d eps, or -1 */
    double w[7][6];   /* tangent columns (dX, dP) */
    double eps;
} orbit;

/* Drift D(tau): X <- X + tau P, dX <- dX + tau dP. */
static void drift(orbit *o, double tau)
{
    for (int a = 0; a < 3; a++)
        o->s[a] = o->s[a] + tau * o->s[3 + a];
    for (int c = 0; c < o->ncol; c++)
        for (int a = 0; a < 3; a++)
            o->w[c][a] = o->w[c][a] + tau * o->w[c][3 + a];
}

/* Kick K(tau): P <- P - tau eps grad Hp(X);
 * dP <- dP - tau eps Hess(X) dX (- tau grad Hp(X) on the eps column). */
static void kick(orbit *o, double tau)
{
    double g[3];
    hp_gradient(o->s, g);
    if (o->ncol > 0) {
        double Hs[3][3];
        hp_hessian(o->s, Hs);
        for (int c = 0; c < o->ncol; c++) {
            double hv[3];
            for (int a = 0; a < 3; a++)
                hv[a] = Hs[a][0] * o->w[c][0] + Hs[a][1] * o->w[c][1] + Hs[a][2] * o->w[c][2];
            for (int a = 0; a < 3; a++) {
                double d = tau * o->eps * hv[a];
                if (c == o->eps_col)
                    d = d + tau * g[a];
                o->w[c][3 + a] = o->w[c][3 + a] - d;
            }
        }
    }
    for (int a = 0; a < 3; a++)
        o->s[3 + a] = o->s[3 + a] - tau * o->eps * g[a];
}

/* ------------------------------------------------------------------------ */
/* Weights of the 7-stage symmetric composition of order 6.                 */
/*                                                                          */
/* With log S2(t) = t A + t^3 B + t^5 C + O(t^7) (S2 is symmetric, so only  */
/* odd powers occur), the composition, built from the middle outwards by    */
/* the symmetric Baker-Campbell-Hausdorff formula                           */
/*   log(e^X e^Z e^X) = 2X + Z - [X,[X,Z]]/6 + [Z,[Z,X]]/6 + (degree 5),    */
/* has log = a t A + b t^3 B + c t^5 C + d t^5 [A,[A,B]] + O(t^7) with      */
/*   start (middle stage w0): a = w0, b = w0^3, c = w0^5, d = 0;            */
/*   each outer pair w:       k = a w^3 - b w,  d += k (a + w) / 6,         */
/*                            a += 2w, b += 2w^3, c += 2w^5                 */
/* (degree-5 brackets of A alone vanish; those holding B are O(t^7)).       */
/* Order 6 requires a = 1, b = c = d = 0.  With w0 = 1 - 2(w1 + w2 + w3)    */
/* that is three equations in (w1, w2, w3); their real roots are found by   */
/* Newton's method in long double from a grid of starts, and the root with  */
/* the smallest |w0| + 2(|w1| + |w2| + |w3|) -- the least stepping back and */
/* forth in time -- is used.                                                */
/* ------------------------------------------------------------------------ */

static void y6_conditions(const long double w[3], long double f[3])
{
    long double a = 1.0L - 2.0L * (w[0] + w[1] + w[2]);
    long double b = a * a * a, c = b * a * a, d = 0.0L;
    for (int i = 0; i < 3; i++) {
        long double v = w[i];
        long double k = a * v * v * v - b * v;
        d = d + k * (a + v) / 6.0L;
        a = a + 2.0L * v;
        b = b + 2.0L * v * v * v;
        c = c + 2.0L * v * v * v * v * v;
    }
    f[0] = b;
    f[1] = c;
    f[2] = d;
}

/* Newton's method with a central-difference Jacobian; returns 0 on
 * convergence (|f| < 1e-18), -1 otherwise. */
static int y6_newton(long double w[3])
{
    for (int it = 0; it < 200; it++) {
        long double f[3], J[3][3];
        y6_conditions(w, f);
        long double nf = fabsl(f[0]) + fabsl(f[1]) + fabsl(f[2]);
        if (!(nf < 1e6L)) return -1;
        if (nf < 1e-18L) return 0;
        for (int j = 0; j < 3; j++) {
            long double wp[3] = {w[0], w[1], w[2]}, wm[3] = {w[0], w[1], w[2]}, fp[3], fm[3];
            long double dj = 1e-7L * (1.0L + fabsl(w[j]));
            wp[j] += dj;
            wm[j] -= dj;
            y6_conditions(wp, fp);
            y6_conditions(wm, fm);
            for (int i = 0; i < 3; i++) J[i][j] = (fp[i] - fm[i]) / (2.0L * dj);
        }
        /* solve J dx = -f by Cramer's rule */
        long double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                        - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                        + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(fabsl(det) > 1e-30L)) return -1;
        long double dx[3];
        for (int c = 0; c < 3; c++) {
            long double M[3][3];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) M[i][j] = (j == c) ? -f[i] : J[i][j];
            dx[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                   - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                   + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
        }
        for (int j = 0; j < 3; j++) w[j] = w[j] + dx[j];
    }
    return -1;
}

/* Y6W = (w0, w1, w2, w3), computed once when the library is loaded. */
static double Y6W[4];

__attribute__((constructor)) static void y6_init(void)
{
    long double best[3] = {0, 0, 0}, best_cost = 1e30L;
    const long double grid[6] = {-2.5L, -1.5L, -0.5L, 0.5L, 1.5L, 2.5L};
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++)
            for (int k = 0; k < 6; k++) {
                long double w[3] = {grid[i], grid[j], grid[k]};
                if (y6_newton(w)) continue;
                long double w0 = 1.0L - 2.0L * (w[0] + w[1] + w[2]);
                long double cost = fabsl(w0) + 2.0L * (fabsl(w[0]) + fabsl(w[1]) + fabsl(w[2]));
                if (cost < best_cost) {
                    best_cost = cost;
                    for (int m = 0; m < 3; m++) best[m] = w[m];
                }
            }
    Y6W[0] = (double)(1.0L - 2.0L * (best[0] + best[1] + best[2]));
    for (int m = 0; m < 3; m++) Y6W[1 + m] = (double)best[m];
}

static double tj_g1(void) { return 1.0 / (2.0 - cbrt(2.0)); }
static double tj_d1(void) { return 1.0 / (2.0 - pow(2.0, 1.0 / 5.0)); }

static void map_s2(orbit *o, double t)
{
    drift(o, t / 2.0);
    kick(o, t);
    drift(o, t / 2.0);
}

static void map_s4(orbit *o, double t)
{
    double g1 = tj_g1(), g0 = 1.0 - 2.0 * g1;
    map_s2(o, g1 * t);
    map_s2(o, g0 * t);
    map_s2(o, g1 * t);
}

static void map_s6(orbit *o, double t)
{
    double d1 = tj_d1(), d0 = 1.0 - 2.0 * d1;
    map_s4(o, d1 * t);
    map_s4(o, d0 * t);
    map_s4(o, d1 * t);
}

static void map_y6(orbit *o, double t)
{
    const int order[7] = {3, 2, 1, 0, 1, 2, 3};
    for (int i = 0; i < 7; i++) map_s2(o, Y6W[order[i]] * t);
}

/* One application of the map of the chosen form with step h. */
static int map_step(orbit *o, int form, double h)
{
    switch (form) {
    case OR_STDMAP: kick(o, h); drift(o, h); return 0;
    case OR_S2: map_s2(o, h); return 0;
    case OR_S4: map_s4(o, h); return 0;
    case OR_S6: map_s6(o, h); return 0;
    case OR_Y6: map_y6(o, h); return 0;
    default: return -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Resumable per-orbit record with one renormalised tangent vector.         */
/* ------------------------------------------------------------------------ */

void oracle_rec_init(const double s0[6], const double w0[6], double rec[OR_REC])
{
    for (int a = 0; a < 6; a++) rec[a] = s0[a];        /* X, P */
    for (int a = 0; a < 6; a++) rec[6 + a] = w0[a];    /* w */
    for (int a = 0; a < 6; a++) rec[12 + a] = s0[a];   /* X0, P0 */
    rec[18] = 0.0;                                     /* L */
    rec[19] = 0.0;                                     /* Jsum */
    rec[20] = 0.0;                                     /* steps done */
}

/* Advance a record by nsteps map steps.  After each full step:
 * nu = |w|, L += ln nu, w /= nu, Jsum += |P_k - P_0|^2. */
int oracle_rec_advance(int form, double eps, double h, long nsteps, double rec[OR_REC])
{
    orbit o;
    o.ncol = 1;
    o.eps_col = -1;
    o.eps = eps;
    for (int a = 0; a < 6; a++) o.s[a] = rec[a];
    for (int a = 0; a < 6; a++) o.w[0][a] = rec[6 + a];
    double L = rec[18], Jsum = rec[19];
    for (long k = 0; k < nsteps; k++) {
        if (map_step(&o, form, h)) return -1;
        double n2 = 0.0;
        for (int a = 0; a < 6; a++) n2 = n2 + o.w[0][a] * o.w[0][a];
        double nu = sqrt(n2);
        L = L + log(nu);
        for (int a = 0; a < 6; a++) o.w[0][a] = o.w[0][a] / nu;
        double d2 = 0.0;
        for (int a = 0; a < 3; a++) {
            double d = o.s[3 + a] - rec[15 + a];
            d2 = d2 + d * d;
        }
        Jsum = Jsum + d2;
    }
    for (int a = 0; a < 6; a++) rec[a] = o.s[a];
    for (int a = 0; a < 6; a++) rec[6 + a] = o.w[0][a];
    rec[18] = L;
    rec[19] = Jsum;
    rec[20] = rec[20] + (double)nsteps;
    return 0;
}

/* End-of-run observables of a record (T = steps done):
 * L, lambda = L/(T h), chi = L/ln(1 + T h), V = (X_T - X_0)/(T h),
 * dP2 = |P_T - P_0|^2, J = Jsum/T, dE = H(s_T) - H(s_0). */
void oracle_rec_finish(const double rec[OR_REC], double eps, double h, double out[OR_NOUT])
{
    double T = rec[20];
    double th = T * h;
    double L = rec[18];
    out[OR_L] = L;
    out[OR_LAMBDA] = L / th;
    out[OR_CHI] = L / log(1.0 + th);
    for (int a = 0; a < 3; a++) out[OR_VX + a] = (rec[a] - rec[12 + a]) / th;
    double d2 = 0.0;
    for (int a = 0; a < 3; a++) {
        double d = rec[3 + a] - rec[15 + a];
        d2 = d2 + d * d;
    }
    out[OR_DP2] = d2;
    out[OR_J] = rec[19] / T;
    double s0[6];
    for (int a = 0; a < 6; a++) s0[a] = rec[12 + a];
    out[OR_DE] = energy(rec, eps) - energy(s0, eps);
}

/* Ensemble run over SoA initial conditions ic[6][N] and tangent starts
 * w0[6][N]; writes out[9][N] and, if state is non-NULL, the final
 * X, P and unit tangent w into state[12][N].  OpenMP over orbits. */
int oracle_ensemble(int form, double eps, double h, long T, long N,
                    const double *ic, const double *w0, double *out, double *state,
                    int nthreads)
{
    if (form != OR_STDMAP && form != OR_S2 && form != OR_S4 && form != OR_S6 && form != OR_Y6) return -1;
    if (T < 1 || N < 0) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (long n = 0; n < N; n++) {
        double s0[6], u[6], rec[OR_REC], o[OR_NOUT];
        for (int a = 0; a < 6; a++) {
            s0[a] = ic[a * N + n];
            u[a] = w0[a * N + n];
        }
        oracle_rec_init(s0, u, rec);
        oracle_rec_advance(form, eps, h, T, rec);
        oracle_rec_finish(rec, eps, h, o);
        for (int r = 0; r < OR_NOUT; r++) out[r * N + n] = o[r];
        if (state)
            for (int a = 0; a < 12; a++) state[a * N + n] = rec[a];
    }
    return 0;
}

/* Apply T map steps to a single state s[6] in place (no tangent). */
int oracle_map(int form, double eps, double h, long T, double s[6])
{
    orbit o;
    o.ncol = 0;
    o.eps_col = -1;
    o.eps = eps;
    for (int a = 0; a < 6; a++) o.s[a] = s[a];
    for (long k = 0; k < T; k++)
        if (map_step(&o, form, h)) return -1;
    for (int a = 0; a < 6; a++) s[a] = o.s[a];
    return 0;
}

/* Jacobian of T map steps at s0: M[i*6 + j] = d s_T[i] / d s0[j];
 * also returns the final state in sT. */
int oracle_jacobian(int form, double eps, double h, long T, const double s0[6],
                    double sT[6], double M[36])
{
    orbit o;
    o.ncol = 6;
    o.eps_col = -1;
    o.eps = eps;
    for (int a = 0; a < 6; a++) o.s[a] = s0[a];
    for (int c = 0; c < 6; c++)
        for (int a = 0; a < 6; a++) o.w[c][a] = (a == c) ? 1.0 : 0.0;
    for (long k = 0; k < T; k++)
        if (map_step(&o, form, h)) return -1;
    for (int a = 0; a < 6; a++) sT[a] = o.s[a];
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) M[i * 6 + j] = o.w[j][i];
    return 0;
}

/* J = (1/T) sum_{k=1..T} |P_k - P_0|^2 and its exact first derivatives by
 * forward mode: dJ[0..5] w.r.t. the initial (x, y, z, px, py, pz), dJ[6]
 * w.r.t. eps.  dJ_c = (2/T) sum_k (P_k - P_0) . (dP_k,c - dP_0,c). */
int oracle_J_grad(int form, double eps, double h, long T, const double s0[6],
                  double *J, double dJ[7])
{
    orbit o;
    o.ncol = 7;
    o.eps_col = 6;
    o.eps = eps;
    for (int a = 0; a < 6; a++) o.s[a] = s0[a];
    for (int c = 0; c < 7; c++)
        for (int a = 0; a < 6; a++) o.w[c][a] = (a == c) ? 1.0 : 0.0;
    double P0[3] = {s0[3], s0[4], s0[5]};
    double dP0[7][3];
    for (int c = 0; c < 7; c++)
        for (int a = 0; a < 3; a++) dP0[c][a] = o.w[c][3 + a];
    double Jsum = 0.0, dsum[7] = {0, 0, 0, 0, 0, 0, 0};
    for (long k = 0; k < T; k++) {
        if (map_step(&o, form, h)) return -1;
        for (int a = 0; a < 3; a++) {
            double d = o.s[3 + a] - P0[a];
            Jsum = Jsum + d * d;
            for (int c = 0; c < 7; c++)
                dsum[c] = dsum[c] + d * (o.w[c][3 + a] - dP0[c][a]);
        }
    }
    *J = Jsum / (double)T;
    for (int c = 0; c < 7; c++) dJ[c] = 2.0 * dsum[c] / (double)T;
    return 0;
}

/* oracle_J_grad over orbits ic[6][N]: J[N], dJ[7][N].  OpenMP over orbits. */
int oracle_J_grad_ensemble(int form, double eps, double h, long T, long N, const double *ic,
                           double *J, double *dJ, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(|:bad)
#endif
    for (long n = 0; n < N; n++) {
        double s0[6], d[7];
        for (int a = 0; a < 6; a++) s0[a] = ic[a * N + n];
        bad |= oracle_J_grad(form, eps, h, T, s0, &J[n], d);
        for (int c = 0; c < 7; c++) dJ[c * N + n] = d[c];
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Derivatives of the tangent-growth indicator, forward over forward.       */
/*                                                                          */
/* The orbit carries its state s = (X, P), its tangent w = (dX, dP) and,    */
/* for each of the seven parameters c (x0, y0, z0, px0, py0, pz0, eps), the */
/* first derivative of the state, a_c = ds/dc, and of the tangent,          */
/* b_c = dw/dc.  Differentiating the stages:                                */
/*   drift D(t): X += t P,  dX += t dP,  a_X += t a_P,  b_X += t b_P;       */
/*   kick  K(t): P  -= t eps g(X),                                          */
/*               dP -= t eps Hs(X) dX,                                      */
/*               a_P -= t eps Hs(X) a_X + [c = eps] t g(X),                 */
/*               b_P -= t eps (Hs(X) b_X + T3(X)[a_X, dX])                  */
/*                      + [c = eps] t Hs(X) dX,                             */
/* with g, Hs, T3 the first, second and third derivatives of Hp, all taken  */
/* at the pre-kick X (a kick changes neither X nor dX).                     */
/* The tangent is divided by nu = |w| after every step, L += ln nu, and     */
/* every b_c is divided by the same nu: the map is linear in w, so with     */
/* the scales held fixed w = W / S and b_c = dW/dc / S for the unscaled     */
/* tangent W and one common S, and                                          */
/*   dL/dc = d ln|W_T| / dc = (W_T . dW_T/dc) / |W_T|^2                     */
/*         = (w_T . b_c) / |w_T|^2.                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    double s[6], w[6];
    double a[7][6], b[7][6];
    double eps;
} orbit2;

static void drift2(orbit2 *o, double t)
{
    for (int i = 0; i < 3; i++) {
        o->s[i] = o->s[i] + t * o->s[3 + i];
        o->w[i] = o->w[i] + t * o->w[3 + i];
    }
    for (int c = 0; c < 7; c++)
        for (int i = 0; i < 3; i++) {
            o->a[c][i] = o->a[c][i] + t * o->a[c][3 + i];
            o->b[c][i] = o->b[c][i] + t * o->b[c][3 + i];
        }
}

static void kick2(orbit2 *o, double t)
{
    double g[3], Hs[3][3], T3[3][3][3];
    hp_gradient(o->s, g);
    hp_hessian(o->s, Hs);
    hp_third(o->s, T3);
    const double *dX = o->w;
    double Hw[3];
    for (int i = 0; i < 3; i++) Hw[i] = Hs[i][0] * dX[0] + Hs[i][1] * dX[1] + Hs[i][2] * dX[2];
    for (int c = 0; c < 7; c++) {
        double de = (c == 6) ? 1.0 : 0.0;
        const double *aX = o->a[c];
        const double *bX = o->b[c];
        double Ha[3], Hb[3], Tab[3];
        for (int i = 0; i < 3; i++) {
            Ha[i] = Hs[i][0] * aX[0] + Hs[i][1] * aX[1] + Hs[i][2] * aX[2];
            Hb[i] = Hs[i][0] * bX[0] + Hs[i][1] * bX[1] + Hs[i][2] * bX[2];
            Tab[i] = 0.0;
            for (int j = 0; j < 3; j++)
                for (int k = 0; k < 3; k++) Tab[i] = Tab[i] + T3[i][j][k] * aX[j] * dX[k];
        }
        for (int i = 0; i < 3; i++) {
            o->a[c][3 + i] = o->a[c][3 + i] - (t * o->eps * Ha[i] + de * t * g[i]);
            o->b[c][3 + i] = o->b[c][3 + i] - (t * o->eps * (Hb[i] + Tab[i]) + de * t * Hw[i]);
        }
    }
    for (int i = 0; i < 3; i++) {
        o->w[3 + i] = o->w[3 + i] - t * o->eps * Hw[i];
        o->s[3 + i] = o->s[3 + i] - t * o->eps * g[i];
    }
}

static void map2_s2(orbit2 *o, double t)
{
    drift2(o, t / 2.0);
    kick2(o, t);
    drift2(o, t / 2.0);
}

static void map2_s4(orbit2 *o, double t)
{
    double g1 = tj_g1(), g0 = 1.0 - 2.0 * g1;
    map2_s2(o, g1 * t);
    map2_s2(o, g0 * t);
    map2_s2(o, g1 * t);
}

static void map2_s6(orbit2 *o, double t)
{
    double d1 = tj_d1(), d0 = 1.0 - 2.0 * d1;
    map2_s4(o, d1 * t);
    map2_s4(o, d0 * t);
    map2_s4(o, d1 * t);
}

/* L = ln(|w_T| / |w_0|) after T steps from (s0, w0), and dL[7], its exact
 * derivatives with respect to the initial (x, y, z, px, py, pz) and eps at
 * fixed w0.  Also returns the final state and unit tangent in sT[12] if
 * non-NULL. */
int oracle_ftle_grad(int form, double eps, double h, long T, const double s0[6], const double w0[6],
                     double *L, double dL[7], double *sT)
{
    if (form != OR_STDMAP && form != OR_S2 && form != OR_S4 && form != OR_S6 && form != OR_Y6) return -1;
    orbit2 o;
    o.eps = eps;
    double n0 = 0.0;
    for (int i = 0; i < 6; i++) {
        o.s[i] = s0[i];
        o.w[i] = w0[i];
        n0 = n0 + w0[i] * w0[i];
    }
    for (int c = 0; c < 7; c++)
        for (int i = 0; i < 6; i++) {
            o.a[c][i] = (i == c) ? 1.0 : 0.0;
            o.b[c][i] = 0.0;
        }
    double Lsum = -0.5 * log(n0);
    for (long k = 0; k < T; k++) {
        switch (form) {
        case OR_STDMAP: kick2(&o, h); drift2(&o, h); break;
        case OR_S2: map2_s2(&o, h); break;
        case OR_S4: map2_s4(&o, h); break;
        case OR_Y6: {
            const int order[7] = {3, 2, 1, 0, 1, 2, 3};
            for (int i = 0; i < 7; i++) map2_s2(&o, Y6W[order[i]] * h);
            break;
        }
        default: map2_s6(&o, h); break;
        }
        double n2 = 0.0;
        for (int i = 0; i < 6; i++) n2 = n2 + o.w[i] * o.w[i];
        double nu = sqrt(n2);
        Lsum = Lsum + log(nu);
        for (int i = 0; i < 6; i++) o.w[i] = o.w[i] / nu;
        for (int c = 0; c < 7; c++)
            for (int i = 0; i < 6; i++) o.b[c][i] = o.b[c][i] / nu;
    }
    double ww = 0.0;
    for (int i = 0; i < 6; i++) ww = ww + o.w[i] * o.w[i];
    for (int c = 0; c < 7; c++) {
        double wb = 0.0;
        for (int i = 0; i < 6; i++) wb = wb + o.w[i] * o.b[c][i];
        dL[c] = wb / ww;
    }
    *L = Lsum;
    if (sT)
        for (int i = 0; i < 6; i++) {
            sT[i] = o.s[i];
            sT[6 + i] = o.w[i];
        }
    return 0;
}

/* oracle_ftle_grad over orbits ic[6][N] with tangent starts w0[6][N]:
 * L[N], dL[7][N].  OpenMP over orbits. */
int oracle_ftle_grad_ensemble(int form, double eps, double h, long T, long N, const double *ic,
                              const double *w0, double *L, double *dL, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(|:bad)
#endif
    for (long n = 0; n < N; n++) {
        double s0[6], u[6], d[7];
        for (int a = 0; a < 6; a++) {
            s0[a] = ic[a * N + n];
            u[a] = w0[a * N + n];
        }
        bad |= oracle_ftle_grad(form, eps, h, T, s0, u, &L[n], d, NULL);
        for (int c = 0; c < 7; c++) dL[c * N + n] = d[c];
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Counter-based SplitMix64 (Steele, Lea & Flood 2014).                     */
/* The sequential generator advances state += 0x9E3779B97F4A7C15 and        */
/* returns mix(state); output number c (from 0) is therefore                */
/* mix(seed + (c + 1) * gamma).                                             */
/* ------------------------------------------------------------------------ */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform double in [0, 1): the top 53 bits times 2^-53. */
double oracle_u01(uint64_t seed, uint64_t counter)
{
    return (double)(oracle_splitmix64(seed, counter) >> 11) * 0x1.0p-53;
}

/* Orbit index list: idx[m] if idx is non-NULL, else m. */
static long pick(const long *idx, long m) { return idx ? idx[m] : m; }

/* GRID2 slice: s = base; s[a0] = lo0 + i * ((hi0 - lo0) / nx);
 * s[a1] = lo1 + j * ((hi1 - lo1) / ny); orbit n = j * nx + i. */
int oracle_ic_grid2(int a0, int a1, double lo0, double hi0, double lo1, double hi1,
                    long nx, long ny, const double base[6], const long *idx, long M,
                    double *ic)
{
    if (a0 < 0 || a0 > 5 || a1 < 0 || a1 > 5 || a0 == a1 || nx < 1 || ny < 1) return -1;
    double d0 = (hi0 - lo0) / (double)nx;
    double d1 = (hi1 - lo1) / (double)ny;
    for (long m = 0; m < M; m++) {
        long n = pick(idx, m);
        long i = n % nx, j = n / nx;
        for (int a = 0; a < 6; a++) ic[a * M + m] = base[a];
        ic[a0 * M + m] = lo0 + (double)i * d0;
        ic[a1 * M + m] = lo1 + (double)j * d1;
    }
    return 0;
}

/* Uniform box: s_k = lo_k + (hi_k - lo_k) * U(seed, 16 n + k). */
void oracle_ic_box(const double lo[6], const double hi[6], uint64_t seed,
                   const long *idx, long M, double *ic)
{
    for (long m = 0; m < M; m++) {
        long n = pick(idx, m);
        for (int k = 0; k < 6; k++)
            ic[k * M + m] = lo[k] + (hi[k] - lo[k]) * oracle_u01(seed, 16u * (uint64_t)n + (uint64_t)k);
    }
}

/* Tangent start: u_k = 2 U(seed, 16 n + k) - 1, w0 = u / |u|. */
void oracle_w0(uint64_t seed, const long *idx, long M, double *w0)
{
    for (long m = 0; m < M; m++) {
        long n = pick(idx, m);
        double u[6], n2 = 0.0;
        for (int k = 0; k < 6; k++) {
            u[k] = 2.0 * oracle_u01(seed, 16u * (uint64_t)n + (uint64_t)k) - 1.0;
            n2 = n2 + u[k] * u[k];
        }
        double nu = sqrt(n2);
        for (int k = 0; k < 6; k++) w0[k * M + m] = u[k] / nu;
    }
}

/* Fixed-energy initial conditions (section "Main results", Figs. 2-3):
 * X uniform on the box [xlo, xhi) (the torus), the direction of P uniform on
 * the part of the sphere with phi in [phi_lo, phi_hi), mu = cos(theta) in
 * [mu_lo, mu_hi) -- uniform in (phi, mu) is uniform in area -- and |P| from
 * the energy condition H(P, X) = E:  |P| = sqrt(2 (E - eps Hp(X))).
 * Draws: X_k = U(seed, 16 n + k), k < 3; mu: U(seed, 16 n + 3); phi: U(seed, 16 n + 4). */
void oracle_ic_sphere(double E, double eps, double phi_lo, double phi_hi, double mu_lo, double mu_hi,
                      const double xlo[3], const double xhi[3], uint64_t seed, const long *idx, long M,
                      double *ic)
{
    for (long m = 0; m < M; m++) {
        long n = pick(idx, m);
        uint64_t c = 16u * (uint64_t)n;
        double X[3];
        for (int k = 0; k < 3; k++) X[k] = xlo[k] + (xhi[k] - xlo[k]) * oracle_u01(seed, c + (uint64_t)k);
        double mu = mu_lo + (mu_hi - mu_lo) * oracle_u01(seed, c + 3u);
        double phi = phi_lo + (phi_hi - phi_lo) * oracle_u01(seed, c + 4u);
        double st = sqrt(1.0 - mu * mu);
        double p = sqrt(2.0 * (E - eps * hp_value(X)));
        double P[3] = {p * st * cos(phi), p * st * sin(phi), p * mu};
        for (int k = 0; k < 3; k++) {
            ic[k * M + m] = X[k];
            ic[(3 + k) * M + m] = P[k];
        }
    }
}

/* The injected cloud of Fig. 4 (section "Main results"): the velocity
 * components (vx, vy) Gaussian around cloud[0..1] with standard deviations
 * cloud[2..3] (Box-Muller: g1 = r cos(2 pi u2), g2 = r sin(2 pi u2),
 * r = sqrt(-2 ln(1 - u1))), X uniform on the box, redrawn until the energy
 * condition H = E leaves a real vz: R = 2 (E - eps Hp(X)) - vx^2 - vy^2 >= 0
 * (at most 40 draws; after that R is taken as 0), vz = +-sqrt(R) with the
 * sign drawn with probability 1/2.  Counters: X at attempt a from
 * 128 n + 3 a + k, u1 = 128 n + 120, u2 = 128 n + 121, sign 128 n + 122. */
void oracle_ic_cloud(double E, double eps, const double cloud[4], const double xlo[3], const double xhi[3],
                     uint64_t seed, const long *idx, long M, double *ic)
{
    for (long m = 0; m < M; m++) {
        long n = pick(idx, m);
        uint64_t c = 128u * (uint64_t)n;
        double u1 = oracle_u01(seed, c + 120u), u2 = oracle_u01(seed, c + 121u);
        double r = sqrt(-2.0 * log(1.0 - u1));
        double vx = cloud[0] + cloud[2] * (r * cos(2.0 * OR_PI * u2));
        double vy = cloud[1] + cloud[3] * (r * sin(2.0 * OR_PI * u2));
        double X[3] = {0, 0, 0}, R = -1.0;
        for (int a = 0; a < 40 && R < 0.0; a++) {
            for (int k = 0; k < 3; k++)
                X[k] = xlo[k] + (xhi[k] - xlo[k]) * oracle_u01(seed, c + 3u * (uint64_t)a + (uint64_t)k);
            R = 2.0 * (E - eps * hp_value(X)) - vx * vx - vy * vy;
        }
        double vz = sqrt(R > 0.0 ? R : 0.0);
        if (oracle_u01(seed, c + 122u) < 0.5) vz = -vz;
        double s[6] = {X[0], X[1], X[2], vx, vy, vz};
        for (int k = 0; k < 6; k++) ic[k * M + m] = s[k];
    }
}

/* Mean velocities over consecutive time windows (section "Main results",
 * Fig. 4: V_w = [X(t_w + dt) - X(t_w)] / dt with t_w = w dt): V[w][3][N] for
 * w < n_windows, each window of window_steps map steps.  No tangent. */
int oracle_window_velocities(int form, double eps, double h, long N, const double *ic, long n_windows,
                             long window_steps, double *V, int nthreads)
{
    if (form != OR_STDMAP && form != OR_S2 && form != OR_S4 && form != OR_S6 && form != OR_Y6) return -1;
    if (n_windows < 1 || window_steps < 1 || N < 0) return -1;
    double dt = (double)window_steps * h;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (long n = 0; n < N; n++) {
        double s[6];
        for (int a = 0; a < 6; a++) s[a] = ic[a * N + n];
        for (long w = 0; w < n_windows; w++) {
            double x0[3] = {s[0], s[1], s[2]};
            oracle_map(form, eps, h, window_steps, s);
            for (int a = 0; a < 3; a++) V[(w * 3 + a) * N + n] = (s[a] - x0[a]) / dt;
        }
    }
    return 0;
}

/* Signed distance of the direction of P from the window in (phi, mu)
 * coordinates, phi = atan2(py, px), mu = pz / |P|: positive inside (the
 * smallest distance to an edge), negative outside. */
static double window_margin(const double P[3], const double win[4])
{
    double r = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    double phi = atan2(P[1], P[0]);
    double mu = P[2] / r;
    double d = phi - win[0];
    if (win[1] - phi < d) d = win[1] - phi;
    if (mu - win[2] < d) d = mu - win[2];
    if (win[3] - mu < d) d = win[3] - mu;
    return d;
}

/* As oracle_ensemble, and in addition the "remained within the area" test of
 * section "Main results": after every step the direction of P must lie in the
 * window win = (phi_lo, phi_hi, mu_lo, mu_hi) (edges included).  left[n] = 1
 * if it ever left; margin[n] = the smallest window margin met (negative once
 * outside), for judging decisions taken right at an edge. */
int oracle_ensemble_window(int form, double eps, double h, long T, long N, const double *ic,
                           const double *w0, const double win[4], double *out, uint8_t *left,
                           double *margin, int nthreads)
{
    if (form != OR_STDMAP && form != OR_S2 && form != OR_S4 && form != OR_S6 && form != OR_Y6) return -1;
    if (T < 1 || N < 0) return -1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (long n = 0; n < N; n++) {
        double s0[6], u[6], rec[OR_REC], o[OR_NOUT];
        for (int a = 0; a < 6; a++) {
            s0[a] = ic[a * N + n];
            u[a] = w0[a * N + n];
        }
        oracle_rec_init(s0, u, rec);
        double mmin = window_margin(s0 + 3, win);
        for (long k = 0; k < T; k++) {
            oracle_rec_advance(form, eps, h, 1, rec);
            double mk = window_margin(rec + 3, win);
            if (mk < mmin) mmin = mk;
        }
        oracle_rec_finish(rec, eps, h, o);
        for (int r = 0; r < OR_NOUT; r++) out[r * N + n] = o[r];
        left[n] = mmin < 0.0 ? 1 : 0;
        margin[n] = mmin;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Images.                                                                  */
/* ------------------------------------------------------------------------ */

/* Serial histogram in orbit order.  Bin of item n along an axis:
 * floor((a - lo) / (hi - lo) * W).  With closed_upper = 0 the range is
 * half-open and items outside [0, W) are dropped; with closed_upper = 1 an
 * item exactly at hi goes to the last bin.  Non-finite keys are dropped.
 * counts[j*W + i] += 1 and sums[j*W + i] += v[n].  Returns the number of
 * dropped items. */
long oracle_hist2d(long N, const double *a, const double *b, const double *v,
                   double lo0, double hi0, double lo1, double hi1, int W, int H,
                   int closed_upper, uint32_t *counts, double *sums)
{
    long dropped = 0;
    memset(counts, 0, sizeof(uint32_t) * (size_t)W * (size_t)H);
    memset(sums, 0, sizeof(double) * (size_t)W * (size_t)H);
    for (long n = 0; n < N; n++) {
        if (!isfinite(a[n]) || !isfinite(b[n])) { dropped++; continue; }
        double fi = floor((a[n] - lo0) / (hi0 - lo0) * (double)W);
        double fj = floor((b[n] - lo1) / (hi1 - lo1) * (double)H);
        if (closed_upper) {
            if (fi == (double)W && a[n] == hi0) fi = W - 1;
            if (fj == (double)H && b[n] == hi1) fj = H - 1;
        }
        if (fi < 0.0 || fi >= (double)W || fj < 0.0 || fj >= (double)H) { dropped++; continue; }
        long i = (long)fi, j = (long)fj;
        counts[j * W + i] += 1u;
        sums[j * W + i] = sums[j * W + i] + v[n];
    }
    return dropped;
}

/* Direction of V on the sphere as equal-area coordinates:
 * phi = atan2(Vy, Vx) in [-pi, pi], mu = Vz / |V| in [-1, 1].
 * A zero V gets NaN keys (dropped by the histogram). */
void oracle_vdir_keys(long N, const double *V, double *phi, double *mu)
{
    for (long n = 0; n < N; n++) {
        double vx = V[n], vy = V[N + n], vz = V[2 * N + n];
        double r = sqrt(vx * vx + vy * vy + vz * vz);
        if (r == 0.0) { phi[n] = NAN; mu[n] = NAN; continue; }
        phi[n] = atan2(vy, vx);
        mu[n] = vz / r;
    }
}

/* ------------------------------------------------------------------------ */
/* Small accessors used by the tests.                                        */
/* ------------------------------------------------------------------------ */

double oracle_energy(const double s[6], double eps) { return energy(s, eps); }

/* Third derivatives of Hp at X as the full array T27[i*9 + j*3 + k]. */
void oracle_hp_third(const double X[3], double T27[27])
{
    double T3[3][3][3];
    hp_third(X, T3);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) T27[i * 9 + j * 3 + k] = T3[i][j][k];
}

/* hp, gradient g[3], Hessian entries H6 = (xx, yy, zz, xy, xz, yz). */
void oracle_hp_derivs(const double X[3], double *hp, double g[3], double H6[6])
{
    double Hs[3][3];
    *hp = hp_value(X);
    hp_gradient(X, g);
    hp_hessian(X, Hs);
    H6[0] = Hs[0][0];
    H6[1] = Hs[1][1];
    H6[2] = Hs[2][2];
    H6[3] = Hs[0][1];
    H6[4] = Hs[0][2];
    H6[5] = Hs[1][2];
}

/* Weights (w0, w1, w2, w3) of the 7-stage composition, as solved here. */
void oracle_y6_weights(double w[4])
{
    for (int i = 0; i < 4; i++) w[i] = Y6W[i];
}

/* Triple-jump constants as evaluated here: g1, g0, d1, d0. */
void oracle_tj_constants(double c[4])
{
    c[0] = tj_g1();
    c[1] = 1.0 - 2.0 * c[0];
    c[2] = tj_d1();
    c[3] = 1.0 - 2.0 * c[2];
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
