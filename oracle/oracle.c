/*
 * FP64 CPU oracle for the fused lattice Boltzmann stream-and-collide step.
 *
 * TEST INFRASTRUCTURE ONLY: the plain reference the HIP path is checked
 * against.  Only tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code with the HIP library.
 *
 * Every step is written the plain way: gather a node's populations, collide
 * them (or swap them on a wall node), push each post-collision value to
 * x + e_i in a second array, swap arrays.  All arithmetic is double precision, on
 * the deviations h_i = f_i - w_i (the paper's round-off minimising formulation, from
 * its single-vs-double precision subsection): with f stored directly, double
 * rounding of rho = sum f and of the O(w) offset drifts f - w by ~1e-16 per step,
 * which over thousands of steps exceeds 1e-12 relative on slow flows.
 * Citations name the section / equation of Januszewski & Kostur, "Sailfish: a
 * flexible multi-GPU implementation of the lattice Boltzmann method" (CPC 2014).
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *  - LBGK sign: the relaxation is f + (1/tau)(feq - f), as in the GPU kernel
 *    algorithm of the software section; the sign printed in the LBGK equation is
 *    the unstable one.
 *  - The body force is an acceleration g; the force density is F = rho g.
 *  - MRT basis: the orthogonal polynomial moments of d'Humieres et al. (2002)
 *    (cited by the paper for M), m_eq = M f_eq, the Guo source relaxed as
 *    (I - S/2) M F~.
 *  - ELBM equilibrium: the product form with the factor (2 - sqrt(1+3u^2)) is
 *    exact on D2Q9; on D3Q19 the exact discrete H minimiser w_i exp(b.e_i)/Z is
 *    used, seeded with the product form's b and refined by two Newton steps.
 *  - ELBM relaxation f + alpha beta (feq - f), beta = 1/(2 tau), so alpha = 2 is LBGK.
 *  - Shan-Chen force F_A = -G psi_A sum_i w_i psi_B(x+e_i) e_i (G > 0 repulsive),
 *    EDM forcing around the common velocity.
 *  - Regularized model: the non-equilibrium part is taken about the polynomial
 *    equilibrium, and the step takes no body force (the paper pairs it with none; the
 *    projection would drop the -F/2 first moment that Guo forcing relies on).
 *  - Smagorinsky model: Q from the polynomial equilibrium at the force-shifted
 *    velocity, and the Guo prefactor 1 - 1/(2 tau) with the local tau = tau0 + tau_t.
 *  - Equilibrium velocity nodes (flag 2): a population is missing when the node it
 *    streams from is a wall node; it takes the value of the opposite population at the
 *    node; rho is summed after that; the node's post-collision state is the polynomial
 *    feq(rho, u_bc), with no relaxation and no force.  The macroscopic output of such
 *    a node is that rho and u_bc.  Single-component polynomial-equilibrium models only.
 *  - Half-way bounce-back nodes (flag 3): wet nodes; the missing populations (as above)
 *    are the reflections of those that reached the node in this step, and the node then
 *    collides like any fluid node.  Its macroscopic output is that of the completed set.
 *  - Free-energy model: the weights the paper takes from the literature are fixed here by
 *    the moment conditions they must meet: with lattice weights t_i, the non-rest weights
 *    are 3 t_i and the gradient weights t_i (4.5 e_a e_b - 3 d_ab), so that sum_i feq_i e e
 *    is P_ab + rho u u; the rest populations take what mass (rho, phi) leaves.  The bulk
 *    pressure is rho/3 + A (-phi^2/2 + 3 phi^4/4) (the sign of phi^2 that matches
 *    mu = A(-phi + phi^3)).  Gradient and Laplacian use the isotropic lattice-weight
 *    stencils; a wall neighbour contributes phi(x) (neutral wetting).  The body force
 *    enters f by the exact difference method around u = j/rho; g's equilibrium takes
 *    the velocity (j + F/2)/rho.  Initial populations are the equilibria with zero phi
 *    gradients.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19
#define MLP_H 32
#define MLP_IN 6
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

typedef struct {
    int q, d;
    int e[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} lattice_t;

/* Velocity sets in the ordering documented in oracle.h. */
static const int VEL_D2Q9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}};
static const int VEL_D3Q19[19][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Weights by link length (rest, 1, sqrt 2): the paper's weight table. */
static void make_lattice(int lattice, lattice_t *L) {
    const double wd2q9[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    const double wd3q19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    const double *wl = lattice == ORC_D2Q9 ? wd2q9 : wd3q19;
    L->q = lattice == ORC_D2Q9 ? 9 : 19;
    L->d = lattice == ORC_D2Q9 ? 2 : 3;
    for (int i = 0; i < L->q; i++) {
        const int *v = lattice == ORC_D2Q9 ? VEL_D2Q9[i] : VEL_D3Q19[i];
        int len2 = 0;
        for (int a = 0; a < 3; a++) {
            L->e[i][a] = v[a];
            len2 += v[a] * v[a];
        }
        L->w[i] = wl[len2];
    }
    /* opposite direction found by search for -e_i */
    for (int i = 0; i < L->q; i++)
        for (int j = 0; j < L->q; j++)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] && L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
}

int orc_q(int lattice) { return lattice == ORC_D2Q9 ? 9 : 19; }

void orc_tables(int lattice, int *e, double *w, int *opp) {
    lattice_t L;
    make_lattice(lattice, &L);
    for (int i = 0; i < L.q; i++) {
        for (int a = 0; a < 3; a++) e[3 * i + a] = L.e[i][a];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (n >= 1); the arithmetic does not depend on it. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---- equilibria ----------------------------------------------------------- */

/* Second-order polynomial equilibrium (equilibrium equation of section 2). */
static void feq_poly(const lattice_t *L, double rho, const double *u, double *feq) {
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; i++) {
        double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
        feq[i] = rho * L->w[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

void orc_feq(int lattice, double rho, const double *u, double *feq) {
    lattice_t L;
    make_lattice(lattice, &L);
    feq_poly(&L, rho, u, feq);
}

/* The same equilibrium minus the rest weights, written with drho = rho - 1 (the
 * round-off minimising formulation of the single-vs-double precision subsection, which
 * keeps the small deviation f - w instead of f):
 * feq_i - w_i = w_i (drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u^2)). */
static void heq_poly(const lattice_t *L, double drho, const double *u, double *heq) {
    double rho = 1.0 + drho;
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; i++) {
        double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
        heq[i] = L->w[i] * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    }
}

/* Solve the d x d system A x = r (d = 2 or 3) by Cramer's rule. */
static void solve_small(int d, double A[3][3], const double *r, double *x) {
    if (d == 2) {
        double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        x[0] = (r[0] * A[1][1] - A[0][1] * r[1]) / det;
        x[1] = (A[0][0] * r[1] - r[0] * A[1][0]) / det;
        x[2] = 0.0;
        return;
    }
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
               - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
               + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    for (int c = 0; c < 3; c++) {
        double B[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) B[a][b] = (b == c) ? r[a] : A[a][b];
        x[c] = (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1])
              - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0])
              + B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0])) / det;
    }
}

/* Discrete entropic equilibrium: the minimiser of H = sum f ln(f/w) at fixed
 * rho and rho u (entropic LBM subsection).  Its form is rho w_i exp(b.e_i)/Z.
 * The first guess b_a = ln((2u_a + sqrt(1+3u_a^2))/(1-u_a)) is the product form's
 * exponent base; two Newton steps on the momentum constraint follow (Jacobian =
 * covariance of e under the normalised weights).  Returned as dp_i = p_i - w_i with
 * p_i = w_i exp(b.e_i)/Z, evaluated through expm1 so the small deviation keeps its
 * relative accuracy: dp_i = w_i (expm1(b.e_i) - (Z - 1))/Z. */
static void entropic_dp(const lattice_t *L, const double *u, double *dp) {
    double b[3] = {0.0, 0.0, 0.0};
    double p[QMAX];
    for (int a = 0; a < L->d; a++) {
        double s = sqrt(1.0 + 3.0 * u[a] * u[a]);
        b[a] = log((2.0 * u[a] + s) / (1.0 - u[a]));
    }
    for (int it = 0; it < 2; it++) {
        double Z = 0.0, m[3] = {0, 0, 0}, C[3][3] = {{0}};
        for (int i = 0; i < L->q; i++) {
            p[i] = L->w[i] * exp(b[0] * L->e[i][0] + b[1] * L->e[i][1] + b[2] * L->e[i][2]);
            Z += p[i];
        }
        for (int i = 0; i < L->q; i++) {
            p[i] /= Z;
            for (int a = 0; a < 3; a++) {
                m[a] += p[i] * L->e[i][a];
                for (int c = 0; c < 3; c++) C[a][c] += p[i] * L->e[i][a] * L->e[i][c];
            }
        }
        double r[3], db[3];
        for (int a = 0; a < 3; a++) {
            r[a] = m[a] - u[a];
            for (int c = 0; c < 3; c++) C[a][c] -= m[a] * m[c];
        }
        solve_small(L->d, C, r, db);
        for (int a = 0; a < L->d; a++) b[a] -= db[a];
    }
    double em1[QMAX], zm1 = 0.0;
    for (int i = 0; i < L->q; i++) {
        em1[i] = expm1(b[0] * L->e[i][0] + b[1] * L->e[i][1] + b[2] * L->e[i][2]);
        zm1 += L->w[i] * em1[i];
    }
    for (int i = 0; i < L->q; i++) dp[i] = L->w[i] * (em1[i] - zm1) / (1.0 + zm1);
}

static void feq_entropic(const lattice_t *L, double rho, const double *u, double *feq) {
    double dp[QMAX];
    entropic_dp(L, u, dp);
    for (int i = 0; i < L->q; i++) feq[i] = rho * (L->w[i] + dp[i]);
}

/* entropic equilibrium minus the rest weights: rho dp_i + drho w_i */
static void heq_entropic(const lattice_t *L, double drho, const double *u, double *heq) {
    double dp[QMAX];
    entropic_dp(L, u, dp);
    for (int i = 0; i < L->q; i++) heq[i] = (1.0 + drho) * dp[i] + drho * L->w[i];
}

void orc_feq_entropic(int lattice, double rho, const double *u, double *feq) {
    lattice_t L;
    make_lattice(lattice, &L);
    feq_entropic(&L, rho, u, feq);
}

/* ---- MRT moment basis ---------------------------------------------------- */

/* Rows of the orthogonal moment matrix (d'Humieres et al. 2002, the reference
 * the MRT subsection gives for M), as polynomials of e with q = |e|^2. */
static double mrt_row(int lattice, int k, const int *e) {
    double ex = e[0], ey = e[1], ez = e[2];
    double q = ex * ex + ey * ey + ez * ez;
    if (lattice == ORC_D2Q9) {
        switch (k) {
        case 0: return 1.0;
        case 1: return 3.0 * q - 4.0;
        case 2: return (9.0 * q * q - 21.0 * q + 8.0) / 2.0;
        case 3: return ex;
        case 4: return (3.0 * q - 5.0) * ex;
        case 5: return ey;
        case 6: return (3.0 * q - 5.0) * ey;
        case 7: return ex * ex - ey * ey;
        default: return ex * ey;
        }
    }
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * q - 30.0;
    case 2: return (21.0 * q * q - 53.0 * q + 24.0) / 2.0;
    case 3: return ex;
    case 4: return (5.0 * q - 9.0) * ex;
    case 5: return ey;
    case 6: return (5.0 * q - 9.0) * ey;
    case 7: return ez;
    case 8: return (5.0 * q - 9.0) * ez;
    case 9: return 3.0 * ex * ex - q;
    case 10: return (3.0 * q - 5.0) * (3.0 * ex * ex - q);
    case 11: return ey * ey - ez * ez;
    case 12: return (3.0 * q - 5.0) * (ey * ey - ez * ez);
    case 13: return ex * ey;
    case 14: return ey * ez;
    case 15: return ex * ez;
    case 16: return (ey * ey - ez * ez) * ex;
    case 17: return (ez * ez - ex * ex) * ey;
    default: return (ex * ex - ey * ey) * ez;
    }
}

static void mrt_build(int lattice, const lattice_t *L, double M[QMAX][QMAX], double norm2[QMAX]) {
    for (int k = 0; k < L->q; k++) {
        norm2[k] = 0.0;
        for (int i = 0; i < L->q; i++) {
            M[k][i] = mrt_row(lattice, k, L->e[i]);
            norm2[k] += M[k][i] * M[k][i];
        }
    }
}

void orc_mrt_matrix(int lattice, double *Mout) {
    lattice_t L;
    double M[QMAX][QMAX], n2[QMAX];
    make_lattice(lattice, &L);
    mrt_build(lattice, &L, M, n2);
    for (int k = 0; k < L.q; k++)
        for (int i = 0; i < L.q; i++) Mout[k * L.q + i] = M[k][i];
}

/* ---- ELBM ------------------------------------------------------------------- */

static double H_of(const lattice_t *L, const double *f) {
    double h = 0.0;
    for (int i = 0; i < L->q; i++) h += f[i] * log(f[i] / L->w[i]);
    return h;
}

double orc_H(int lattice, const double *f) {
    lattice_t L;
    make_lattice(lattice, &L);
    return H_of(&L, f);
}

/* g(a) = H(f + a D) - H(f) and g'(a), D = feq - f, in a form free of the
 * cancellation between the two H values (uses sum_i D_i ln(feq_i/w_i) = 0,
 * which holds because feq is the constrained minimiser and D carries no mass
 * or momentum). */
static void g_dg(int q, const double *f, const double *D, double a, double *g, double *dg, double *gscale) {
    double s = 0.0, ds = 0.0, sc = 0.0;
    for (int i = 0; i < q; i++) {
        double la = log1p(a * D[i] / f[i]);
        double l1 = log1p(D[i] / f[i]);
        s += (f[i] + a * D[i]) * la - a * D[i] * l1;
        ds += D[i] * (la - l1);
        sc += fabs((f[i] + a * D[i]) * la) + fabs(a * D[i] * l1);
    }
    *g = s;
    *dg = ds;
    *gscale = sc;
}

/* The six MLP inputs: log10(a2/rho), a3/a2, a4/a2, max(-d), max(d), |v|^2/c_s^2 with
 * d_i = D_i/f_i and a_k = sum_i f_i d_i^k. */
static void alpha_features(int q, const double *f, const double *D, double rho, double vsq, double *feat) {
    double a2 = 0, a3 = 0, a4 = 0, mneg = -1e300, mpos = -1e300;
    for (int i = 0; i < q; i++) {
        double d = D[i] / f[i];
        a2 += f[i] * d * d;
        a3 += f[i] * d * d * d;
        a4 += f[i] * d * d * d * d;
        if (-d > mneg) mneg = -d;
        if (d > mpos) mpos = d;
    }
    feat[0] = log10(a2 / rho);
    feat[1] = a3 / a2;
    feat[2] = a4 / a2;
    feat[3] = mneg;
    feat[4] = mpos;
    feat[5] = 3.0 * vsq;
}

void orc_alpha_features(int lattice, const double *f, const double *feq, double rho, double vsq,
                        double *feat) {
    int q = orc_q(lattice);
    double D[QMAX];
    for (int i = 0; i < q; i++) D[i] = feq[i] - f[i];
    alpha_features(q, f, D, rho, vsq, feat);
}

/* MLP 6 -> 32 -> 32 -> 1, tanh hidden layers.  Parameters (1325): W1[32][6], b1[32],
 * W2[32][32], b2[32], w3[32], b3, then the input normalisation mu[6], isd[6].  The
 * network sees xn = (x - mu) * isd of the raw features x; its output is added to the
 * series estimate of the root, 2 + (x[1] - 2 x[2]) / 3 = 2 + (a3 - 2 a4)/(3 a2), so the
 * network only learns the series' residual. */
static double mlp_eval(const double *p, const double *xraw, double *xn, double *h1, double *h2) {
    const double *W1 = p, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    const double *w3 = b2 + MLP_H, *b3 = w3 + MLP_H, *mu = p + MLP_NPARAM, *isd = mu + MLP_IN;
    for (int k = 0; k < MLP_IN; k++) xn[k] = (xraw[k] - mu[k]) * isd[k];
    for (int j = 0; j < MLP_H; j++) {
        double s = b1[j];
        for (int k = 0; k < MLP_IN; k++) s += W1[j * MLP_IN + k] * xn[k];
        h1[j] = tanh(s);
    }
    for (int j = 0; j < MLP_H; j++) {
        double s = b2[j];
        for (int k = 0; k < MLP_H; k++) s += W2[j * MLP_H + k] * h1[k];
        h2[j] = tanh(s);
    }
    double y = 2.0 + (xraw[1] - 2.0 * xraw[2]) / 3.0 + b3[0];
    for (int k = 0; k < MLP_H; k++) y += w3[k] * h2[k];
    return y;
}

void orc_mlp_forward(const double *p, const double *x, int64_t n, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; r++) {
        double xn[MLP_IN], h1[MLP_H], h2[MLP_H];
        y[r] = mlp_eval(p, x + MLP_IN * r, xn, h1, h2);
    }
}

/* Mean squared error (1/n) sum (y - t)^2 and its gradient with respect to the 1313
 * network weights by back-propagation (the normalisation is held fixed). */
double orc_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t n, double *grad) {
    const double *W2 = p + MLP_H * MLP_IN + MLP_H;
    const double *w3 = W2 + MLP_H * MLP_H + MLP_H;
    double loss = 0.0;
    memset(grad, 0, sizeof(double) * MLP_NPARAM);
    for (int64_t r = 0; r < n; r++) {
        double xn[MLP_IN], h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
        const double *xr = x + MLP_IN * r;
        double y = mlp_eval(p, xr, xn, h1, h2);
        double err = y - t[r];
        loss += err * err;
        double dy = 2.0 * err / (double)n;
        double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
        double *gw3 = gb2 + MLP_H, *gb3 = gw3 + MLP_H;
        gb3[0] += dy;
        for (int j = 0; j < MLP_H; j++) {
            gw3[j] += dy * h2[j];
            d2[j] = dy * w3[j] * (1.0 - h2[j] * h2[j]);
        }
        for (int j = 0; j < MLP_H; j++) {
            gb2[j] += d2[j];
            for (int k = 0; k < MLP_H; k++) gW2[j * MLP_H + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < MLP_H; k++) {
            double s = 0.0;
            for (int j = 0; j < MLP_H; j++) s += W2[j * MLP_H + k] * d2[j];
            d1[k] = s * (1.0 - h1[k] * h1[k]);
        }
        for (int j = 0; j < MLP_H; j++) {
            gb1[j] += d1[j];
            for (int k = 0; k < MLP_IN; k++) gW1[j * MLP_IN + k] += d1[j] * xn[k];
        }
    }
    return loss / (double)n;
}

/* Nontrivial root alpha of H(f + alpha (feq - f)) = H(f) (alpha condition of the
 * entropic LBM subsection).  Close to equilibrium (max |D_i/f_i| < 1e-6) the
 * root is taken as 2, the value the paper gives for that limit.  Otherwise a
 * safeguarded Newton iteration: the bracket starts at [1, alpha_max) where
 * g(1) = H(feq) - H(f) <= 0 and alpha_max keeps every population positive;
 * stop when the Newton step |d alpha| <= tol, or when g itself is below 64 ulps of the
 * sum of the magnitudes of its terms (just above the short-cut, g' ~ sum f d^2 is so
 * small that the rounding noise of g alone moves a Newton step by more than tol);
 * otherwise a Newton iterate outside the bracket is replaced by the bracket's midpoint.
 * No convergence within maxit: alpha = min(2, 0.99 alpha_max).  f = populations,
 * D = feq - f. */
static double alpha_solve(int q, const double *f, const double *D, int init, const double *mlp, double rho,
                          double vsq, double tol, int maxit, int *iters, int *converged) {
    double dmax = 0.0, amax = INFINITY;
    for (int i = 0; i < q; i++) {
        double r = fabs(D[i] / f[i]);
        if (r > dmax) dmax = r;
        if (D[i] < 0.0 && -f[i] / D[i] < amax) amax = -f[i] / D[i];
    }
    *converged = 1;
    *iters = 0;
    if (dmax < 1e-6) return 2.0;

    double a0 = 2.0;
    if (init == 1) {
        double a2 = 0, a3 = 0, a4 = 0;
        for (int i = 0; i < q; i++) {
            double d = D[i] / f[i];
            a2 += f[i] * d * d;
            a3 += f[i] * d * d * d;
            a4 += f[i] * d * d * d * d;
        }
        a0 = 2.0 + (a3 - 2.0 * a4) / (3.0 * a2);
    } else if (init == 2 && mlp) {
        double feat[MLP_IN], xn[MLP_IN], h1[MLP_H], h2[MLP_H];
        alpha_features(q, f, D, rho, vsq, feat);
        a0 = mlp_eval(mlp, feat, xn, h1, h2);
    }
    double lo = 1.0, hi = amax, a = a0;
    if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
    for (int k = 1; k <= maxit; k++) {
        double g, dg, gs;
        g_dg(q, f, D, a, &g, &dg, &gs);
        /* g at the rounding floor of its own sum: a is the root to working precision */
        if (fabs(g) <= 64.0 * DBL_EPSILON * gs) {
            *iters = k;
            return a;
        }
        if (g < 0.0) lo = a; else hi = a;
        double an = a - g / dg;
        if (fabs(an - a) <= tol) {
            *iters = k;
            return an;
        }
        if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
        a = an;
    }
    *converged = 0;
    *iters = maxit;
    return amax * 0.99 < 2.0 ? amax * 0.99 : 2.0;
}

double orc_alpha(int lattice, const double *f, const double *feq, int init, const double *mlp,
                 double vsq, double tol, int maxit, int *iters, int *converged) {
    int q = orc_q(lattice);
    double D[QMAX], rho = 0.0;
    for (int i = 0; i < q; i++) {
        D[i] = feq[i] - f[i];
        rho += f[i];
    }
    return alpha_solve(q, f, D, init, mlp, rho, vsq, tol, maxit, iters, converged);
}

/* ---- collision ---------------------------------------------------------------- */

/* Guo source term without its (1 - 1/(2 tau)) prefactor (body forces section):
 * w_i [3 (e_i - v) + 9 (e_i . v) e_i] . F. */
static void guo_source(const lattice_t *L, const double *v, const double *F, double *Fi) {
    for (int i = 0; i < L->q; i++) {
        double ev = L->e[i][0] * v[0] + L->e[i][1] * v[1] + L->e[i][2] * v[2];
        double s = 0.0;
        for (int a = 0; a < 3; a++) s += (3.0 * (L->e[i][a] - v[a]) + 9.0 * ev * L->e[i][a]) * F[a];
        Fi[i] = L->w[i] * s;
    }
}

/* Moments of the deviations h = f - w: drho = sum h (so rho = 1 + drho) and
 * j = sum e h (= sum e f because sum w e = 0). */
static void moments(const lattice_t *L, const double *h, double *drho, double *j) {
    double r = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < L->q; i++) {
        r += h[i];
        for (int a = 0; a < 3; a++) j[a] += L->e[i][a] * h[i];
    }
    *drho = r;
}

typedef struct {
    int iters, converged;
} node_info;

/* One fluid node's collision for BGK, MRT or ELBM, on the deviations h = f - w (the
 * round-off minimising formulation of the precision subsection; every operation
 * below is linear in f or uses f = w + h explicitly, so it is the same update). */
static void collide_single(const orc_params *P, const lattice_t *L, const double *h, double *out,
                           node_info *info) {
    int q = L->q;
    double drho, rho, j[3], F[3], v[3], heq[QMAX];
    moments(L, h, &drho, j);
    rho = 1.0 + drho;
    if (P->model == ORC_ELBM) {
        double f[QMAX], D[QMAX];
        for (int a = 0; a < 3; a++) v[a] = j[a] / rho;
        heq_entropic(L, drho, v, heq);
        for (int i = 0; i < q; i++) {
            f[i] = L->w[i] + h[i];
            D[i] = heq[i] - h[i];
        }
        double vsq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        int it, conv;
        double alpha = alpha_solve(q, f, D, P->alpha_init, P->mlp, rho, vsq, P->alpha_tol, P->alpha_maxit,
                                   &it, &conv);
        if (info) {
            info->iters = it;
            info->converged = conv;
        }
        double beta = 1.0 / (2.0 * P->tau);
        for (int i = 0; i < q; i++) out[i] = h[i] + alpha * beta * D[i];
        return;
    }
    for (int a = 0; a < 3; a++) {
        F[a] = rho * P->g[a];
        v[a] = (j[a] + 0.5 * F[a]) / rho;
    }
    heq_poly(L, drho, v, heq);
    double Fi[QMAX];
    guo_source(L, v, F, Fi);
    if (P->model == ORC_BGK) {
        double omega = 1.0 / P->tau, pre = 1.0 - 1.0 / (2.0 * P->tau);
        for (int i = 0; i < q; i++) out[i] = h[i] + omega * (heq[i] - h[i]) + pre * Fi[i];
        return;
    }
    const double cs2 = 1.0 / 3.0;
    if (P->model == ORC_REG) {
        /* Regularized LBM subsection: the non-equilibrium part f_i - feq_i is replaced by
         * w_i / (2 cs^4) (e_ia e_ib - cs^2 d_ab) Pi_ab, with
         * Pi_ab = sum_i (f_i - feq_i) (e_ia e_ib - cs^2 d_ab); then the LBGK relaxation.
         * The indices run over the lattice's D dimensions. */
        double Pi[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int i = 0; i < q; i++) {
            double fneq = h[i] - heq[i];
            for (int a = 0; a < L->d; a++)
                for (int b = 0; b < L->d; b++) Pi[a][b] += fneq * (L->e[i][a] * L->e[i][b] - (a == b ? cs2 : 0.0));
        }
        double omega = 1.0 / P->tau;
        for (int i = 0; i < q; i++) {
            double s = 0.0;
            for (int a = 0; a < L->d; a++)
                for (int b = 0; b < L->d; b++) s += (L->e[i][a] * L->e[i][b] - (a == b ? cs2 : 0.0)) * Pi[a][b];
            double hreg = heq[i] + L->w[i] / (2.0 * cs2 * cs2) * s; /* regularised state, as h */
            out[i] = hreg + omega * (heq[i] - hreg);
        }
        return;
    }
    if (P->model == ORC_SMAG) {
        /* Smagorinsky subgrid model: Q_ab = sum_i e_ia e_ib (f_i - feq_i),
         * tau_t = (sqrt(tau0^2 + 4 cs^-4 C_S^2 (Q_ab Q_ab)^(1/2)) - tau0) / 2, and the LBGK
         * step (with its Guo source) at tau = tau0 + tau_t. */
        double Q[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, QQ = 0.0;
        for (int i = 0; i < q; i++)
            for (int a = 0; a < L->d; a++)
                for (int b = 0; b < L->d; b++) Q[a][b] += L->e[i][a] * L->e[i][b] * (h[i] - heq[i]);
        for (int a = 0; a < L->d; a++)
            for (int b = 0; b < L->d; b++) QQ += Q[a][b] * Q[a][b];
        double tau0 = P->tau;
        double tau_t = 0.5 * (sqrt(tau0 * tau0 + 4.0 / (cs2 * cs2) * P->cs_smag * P->cs_smag * sqrt(QQ)) - tau0);
        double tau = tau0 + tau_t, omega = 1.0 / tau, pre = 1.0 - 1.0 / (2.0 * tau);
        for (int i = 0; i < q; i++) out[i] = h[i] + omega * (heq[i] - h[i]) + pre * Fi[i];
        return;
    }
    /* MRT: m = M h, m* = m - S (m - m_eq) + (I - S/2) M F~, h* = M^-1 m*,
     * with M^-1 = M^T diag(1/|row|^2) for the orthogonal basis (linear, so the same
     * as relaxing f with m_eq = M feq). */
    double M[QMAX][QMAX], n2[QMAX], m[QMAX], meq[QMAX], mF[QMAX], ms[QMAX];
    mrt_build(P->lattice, L, M, n2);
    for (int k = 0; k < q; k++) {
        m[k] = meq[k] = mF[k] = 0.0;
        for (int i = 0; i < q; i++) {
            m[k] += M[k][i] * h[i];
            meq[k] += M[k][i] * heq[i];
            mF[k] += M[k][i] * Fi[i];
        }
        ms[k] = m[k] - P->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * P->s[k]) * mF[k];
    }
    for (int i = 0; i < q; i++) {
        double s = 0.0;
        for (int k = 0; k < q; k++) s += M[k][i] * ms[k] / n2[k];
        out[i] = s;
    }
}

void orc_collide_node(const orc_params *P, const double *f, double *out) {
    lattice_t L;
    double h[QMAX], o[QMAX];
    make_lattice(P->lattice, &L);
    for (int i = 0; i < L.q; i++) h[i] = f[i] - L.w[i];
    collide_single(P, &L, h, o, NULL);
    for (int i = 0; i < L.q; i++) out[i] = L.w[i] + o[i];
}

/* One Shan-Chen node: f2[2][q] the populations of both components at x, psi_nb[2][q]
 * psi of each component at x + e_i (psi_nb[c][0] = psi_c(x)).  Same update as in
 * orc_run: force -G psi_c(x) sum_i w_i psi_other(x + e_i) e_i + rho_c g, common
 * velocity, EDM forcing.  out2[2][q]. */
void orc_collide_node_sc(const orc_params *P, const double *f2, const double *psi_nb, double *out2) {
    lattice_t L;
    make_lattice(P->lattice, &L);
    const int q = L.q;
    double h[2][QMAX], dr[2], rc[2], jc[2][3], Fc[2][3], up[3], num[3] = {0, 0, 0}, den = 0.0;
    for (int c = 0; c < 2; c++) {
        for (int i = 0; i < q; i++) h[c][i] = f2[c * q + i] - L.w[i];
        moments(&L, h[c], &dr[c], jc[c]);
        rc[c] = 1.0 + dr[c];
    }
    for (int c = 0; c < 2; c++) {
        double s[3] = {0, 0, 0};
        for (int i = 0; i < q; i++)
            for (int a = 0; a < 3; a++) s[a] += L.w[i] * psi_nb[(1 - c) * q + i] * L.e[i][a];
        for (int a = 0; a < 3; a++) Fc[c][a] = -P->G * psi_nb[c * q] * s[a] + rc[c] * P->g[a];
        for (int a = 0; a < 3; a++) num[a] += jc[c][a] / P->tau;
        den += rc[c] / P->tau;
    }
    for (int a = 0; a < 3; a++) up[a] = num[a] / den;
    for (int c = 0; c < 2; c++) {
        double h0[QMAX], h1[QMAX], u1[3];
        for (int a = 0; a < 3; a++) u1[a] = up[a] + Fc[c][a] / rc[c];
        heq_poly(&L, dr[c], up, h0);
        heq_poly(&L, dr[c], u1, h1);
        for (int i = 0; i < q; i++)
            out2[c * q + i] = L.w[i] + (h[c][i] + (h0[i] - h[c][i]) / P->tau + (h1[i] - h0[i]));
    }
}

/* ---- full-lattice operations ------------------------------------------------------ */

static int check_params(const orc_params *P) {
    if (P->lattice != ORC_D2Q9 && P->lattice != ORC_D3Q19) return -1;
    if (P->model < ORC_BGK || P->model > ORC_FREE_ENERGY) return -1;
    if (P->model == ORC_FREE_ENERGY && !(P->tau_b > 0.5 && P->tau_phi > 0.5)) return -1;
    if (P->nx <= 0 || P->ny <= 0 || P->nz <= 0) return -1;
    if (P->lattice == ORC_D2Q9 && P->nz != 1) return -1;
    if (!(P->tau > 0.5)) return -1;
    if ((P->model == ORC_ELBM || P->model == ORC_REG) && (P->g[0] != 0.0 || P->g[1] != 0.0 || P->g[2] != 0.0))
        return -1;
    if (P->model == ORC_SMAG && !(P->cs_smag >= 0.0)) return -1;
    return 0;
}

static inline int64_t wrap(int64_t a, int64_t n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

static inline int64_t neighbour(const orc_params *P, int64_t x, int64_t y, int64_t z, const int *e) {
    int64_t X = wrap(x + e[0], P->nx), Y = wrap(y + e[1], P->ny), Z = wrap(z + e[2], P->nz);
    return X + P->nx * (Y + P->ny * Z);
}

static double psi_of(const orc_params *P, double rho) {
    return P->psi == 1 ? 1.0 - exp(-rho) : rho;
}

/* Shan-Chen interaction force on component c at node (x,y,z) (Shan-Chen
 * subsection): -G psi_c(x) sum_i w_i psi_other(x + e_i) e_i, plus rho_c g. */
static void sc_force(const orc_params *P, const lattice_t *L, const double *psi, int64_t N,
                     int64_t x, int64_t y, int64_t z, int c, double rho_c, double *F) {
    int64_t n = x + P->nx * (y + P->ny * z);
    const double *po = psi + (1 - c) * N;
    double s[3] = {0, 0, 0};
    for (int i = 0; i < L->q; i++) {
        double pn = po[neighbour(P, x, y, z, L->e[i])];
        for (int a = 0; a < 3; a++) s[a] += L->w[i] * pn * L->e[i][a];
    }
    for (int a = 0; a < 3; a++) F[a] = -P->G * psi[c * N + n] * s[a] + rho_c * P->g[a];
}

/* Boundary nodes (boundary conditions subsection): the populations that stream in
 * from wall nodes are missing and take the value of the opposite population of the same
 * node (bounce-back).  hc = the completed set (as h). */
static void complete_missing(const orc_params *P, const lattice_t *L, const uint8_t *flags, int64_t x, int64_t y,
                             int64_t z, const double *h, double *hc) {
    for (int i = 0; i < L->q; i++) {
        int back[3] = {-L->e[i][0], -L->e[i][1], -L->e[i][2]};
        int missing = flags[neighbour(P, x, y, z, back)] == 1;
        hc[i] = missing ? h[L->opp[i]] : h[i];
    }
}

/* Equilibrium velocity node: returns drho = sum of the completed set. */
static double velocity_node_drho(const orc_params *P, const lattice_t *L, const uint8_t *flags, int64_t x,
                                 int64_t y, int64_t z, const double *h) {
    double hc[QMAX], drho = 0.0;
    complete_missing(P, L, flags, x, y, z, h, hc);
    for (int i = 0; i < L->q; i++) drho += hc[i];
    return drho;
}

/* ---- free-energy binary model (free energy model subsection) ---------------------- */

static int ncomp_of(const orc_params *P) {
    return P->model == ORC_SHANCHEN || P->model == ORC_FREE_ENERGY ? 2 : 1;
}

/* d_a phi = 3 sum_i t_i e_ia phi(x + e_i), lap phi = 6 sum_i t_i (phi(x + e_i) - phi(x)) */
static void fe_stencil(const orc_params *P, const lattice_t *L, const uint8_t *flags, const double *phi,
                       int64_t x, int64_t y, int64_t z, double *grad, double *lap) {
    const int64_t n = x + P->nx * (y + P->ny * z);
    const double p0 = phi[n];
    double l = 0.0;
    grad[0] = grad[1] = grad[2] = 0.0;
    for (int i = 1; i < L->q; i++) {
        const int64_t m = neighbour(P, x, y, z, L->e[i]);
        const double pn = (flags && flags[m] == 1) ? p0 : phi[m];
        for (int a = 0; a < 3; a++) grad[a] += 3.0 * L->w[i] * L->e[i][a] * pn;
        l += 6.0 * L->w[i] * (pn - p0);
    }
    *lap = l;
}

void orc_fe_stencil(const orc_params *P, const uint8_t *flags, const double *phi, int x, int y, int z,
                    double *grad, double *lap) {
    lattice_t L;
    make_lattice(P->lattice, &L);
    fe_stencil(P, &L, flags, phi, x, y, z, grad, lap);
}

static void fe_equilibria(const orc_params *P, const lattice_t *L, double rho, double phi, const double *u,
                          const double *grad, double lap, double *feq, double *geq) {
    const double A = P->fe_a, k = P->fe_kappa;
    const double mu = A * (-phi + phi * phi * phi) - k * lap;
    const double p0 = rho / 3.0 + A * (-0.5 * phi * phi + 0.75 * phi * phi * phi * phi);
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double g2 = grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2];
    double fs = 0.0, gs = 0.0;
    for (int i = 1; i < L->q; i++) {
        const double t = L->w[i];
        const double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
        const double eg = L->e[i][0] * grad[0] + L->e[i][1] * grad[1] + L->e[i][2] * grad[2];
        const double quad = 1.5 * (eu * eu - usq / 3.0); /* 3/2 (e_a e_b - d_ab/3) u_a u_b */
        feq[i] = 3.0 * t * (p0 - k * phi * lap + eu * rho + quad * rho) + k * t * (4.5 * eg * eg - 3.0 * g2);
        geq[i] = 3.0 * t * (P->fe_gamma * mu + eu * phi + quad * phi);
        fs += feq[i];
        gs += geq[i];
    }
    feq[0] = rho - fs;
    geq[0] = phi - gs;
}

void orc_fe_equilibria(const orc_params *P, double rho, double phi, const double *u, const double *grad,
                       double lap, double *feq, double *geq) {
    lattice_t L;
    make_lattice(P->lattice, &L);
    fe_equilibria(P, &L, rho, phi, u, grad, lap, feq, geq);
}

/* One free-energy node: hf, hg the (completed) populations as deviations from w; grad,
 * lap of phi at the node.  LBGK on both lattices, tau_rho = tau_B + (phi + 1)/2
 * (tau_A - tau_B) for f and tau_phi for g; the body force by the exact difference
 * method on f. */
static void fe_collide(const orc_params *P, const lattice_t *L, const double *hf, const double *hg,
                       const double *grad, double lap, double *of, double *og) {
    const int q = L->q;
    double f[QMAX], g[QMAX], rho = 0.0, phi = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; i++) {
        f[i] = L->w[i] + hf[i];
        g[i] = L->w[i] + hg[i];
        rho += f[i];
        phi += g[i];
        for (int a = 0; a < 3; a++) j[a] += L->e[i][a] * f[i];
    }
    double u[3], u1[3], v[3];
    for (int a = 0; a < 3; a++) {
        u[a] = j[a] / rho;
        u1[a] = u[a] + P->g[a];        /* u + F/rho with F = rho g */
        v[a] = u[a] + 0.5 * P->g[a];   /* (j + F/2) / rho */
    }
    double fe0[QMAX], ge[QMAX], gdummy[QMAX], fdummy[QMAX], edm[QMAX];
    fe_equilibria(P, L, rho, phi, u, grad, lap, fe0, gdummy);
    fe_equilibria(P, L, rho, phi, v, grad, lap, fdummy, ge);
    /* feq(u1) - feq(u): only 3 t_i rho (e.u + 3/2 ((e.u)^2 - u^2/3)) depends on u, so with
     * a = u1 - u the difference is 3 t_i rho (e.a + 3/2 (e.a (2 e.u + e.a) - a.(2u + a)/3)),
     * and the rest population takes minus the sum.  Written out this way the O(F) term
     * keeps its precision; as a difference of two O(1) equilibria it would not. */
    double es = 0.0;
    for (int i = 1; i < q; i++) {
        double ea = 0.0, eu = 0.0, a2 = 0.0;
        for (int a = 0; a < 3; a++) {
            const double aa = u1[a] - u[a];
            ea += L->e[i][a] * aa;
            eu += L->e[i][a] * u[a];
            a2 += aa * (2.0 * u[a] + aa);
        }
        edm[i] = 3.0 * L->w[i] * rho * (ea + 1.5 * (ea * (2.0 * eu + ea) - a2 / 3.0));
        es += edm[i];
    }
    edm[0] = -es;
    const double tau_rho = P->tau_b + 0.5 * (phi + 1.0) * (P->tau - P->tau_b);
    for (int i = 0; i < q; i++) {
        const double fs = f[i] + (fe0[i] - f[i]) / tau_rho + edm[i];
        const double gs = g[i] + (ge[i] - g[i]) / P->tau_phi;
        of[i] = fs - L->w[i];
        og[i] = gs - L->w[i];
    }
}

int orc_init_eq(const orc_params *P, const double *rho, const double *u, const double *df, double *f) {
    if (check_params(P)) return -1;
    lattice_t L;
    make_lattice(P->lattice, &L);
    int64_t N = (int64_t)P->nx * P->ny * P->nz;
    int C = ncomp_of(P);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        double uu[3] = {0, 0, 0}, heq[QMAX];
        for (int a = 0; a < L.d; a++) uu[a] = u[a * N + n];
        if (P->model == ORC_FREE_ENERGY) {
            const double zero[3] = {0, 0, 0};
            double fe[QMAX], ge[QMAX];
            fe_equilibria(P, &L, rho[n], rho[N + n], uu, zero, 0.0, fe, ge);
            for (int i = 0; i < L.q; i++) {
                int64_t k0 = (int64_t)i * N + n, k1 = ((int64_t)L.q + i) * N + n;
                f[k0] = fe[i] + (df ? df[k0] : 0.0);
                f[k1] = ge[i] + (df ? df[k1] : 0.0);
            }
            continue;
        }
        for (int c = 0; c < C; c++) {
            double drho = rho[c * N + n] - 1.0;
            if (P->model == ORC_ELBM) heq_entropic(&L, drho, uu, heq);
            else heq_poly(&L, drho, uu, heq);
            for (int i = 0; i < L.q; i++) {
                int64_t k = ((int64_t)c * L.q + i) * N + n;
                f[k] = L.w[i] + (heq[i] + (df ? df[k] : 0.0));
            }
        }
    }
    return 0;
}

/* Runs `steps` time steps on f (canonical populations, updated in place).  The state is
 * carried as h = f - w during the run and converted back at the end. */
int orc_run(const orc_params *P, const uint8_t *flags, double *f, int steps, orc_stats *st) {
    if (check_params(P) || steps < 0) return -1;
    lattice_t L;
    make_lattice(P->lattice, &L);
    const int q = L.q;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    const int C = ncomp_of(P);
    const int FE = P->model == ORC_FREE_ENERGY;
    if (P->model == ORC_SHANCHEN && flags)
        for (int64_t n = 0; n < N; n++)
            if (flags[n]) return -2; /* walls are not defined for the two-component model */
    if (flags)
        for (int64_t n = 0; n < N; n++)
            if (flags[n] > 3 || (flags[n] >= 2 && P->model == ORC_ELBM) || (flags[n] == 2 && FE)) return -2;
    double *cur = (double *)malloc(sizeof(double) * C * q * N);
    double *nxt = (double *)malloc(sizeof(double) * C * q * N);
    double *psi = C == 2 ? (double *)malloc(sizeof(double) * 2 * N) : NULL;
    if (!cur || !nxt || (C == 2 && !psi)) {
        free(cur);
        free(nxt);
        free(psi);
        return -3;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)C * q * N; k++) cur[k] = f[k] - L.w[(k / N) % q];
    int64_t hist[32] = {0}, noconv = 0, nodes = 0;

    for (int t = 0; t < steps; t++) {
        if (FE) {
            /* macroscopic pre-pass: every node's order parameter phi = sum_i g_i at time t
             * (half-way nodes: of their completed set) */
#pragma omp parallel for schedule(static)
            for (int64_t n = 0; n < N; n++) {
                int64_t x = n % P->nx, y = (n / P->nx) % P->ny, z = n / ((int64_t)P->nx * P->ny);
                double hg[QMAX], r = 0.0;
                for (int i = 0; i < q; i++) hg[i] = cur[((int64_t)q + i) * N + n];
                if (flags && flags[n] == 3) {
                    double hc[QMAX];
                    complete_missing(P, &L, flags, x, y, z, hg, hc);
                    memcpy(hg, hc, sizeof(double) * q);
                }
                for (int i = 0; i < q; i++) r += L.w[i] + hg[i];
                psi[n] = r;
            }
        } else if (C == 2) {
            /* macroscopic pre-pass: every node's pseudopotential at time t */
#pragma omp parallel for schedule(static)
            for (int64_t n = 0; n < N; n++)
                for (int c = 0; c < 2; c++) {
                    double r = 0.0;
                    for (int i = 0; i < q; i++) r += cur[((int64_t)c * q + i) * N + n];
                    psi[c * N + n] = psi_of(P, 1.0 + r);
                }
        }
#pragma omp parallel for schedule(static) reduction(+ : noconv, nodes)
        for (int64_t n = 0; n < N; n++) {
            int64_t x = n % P->nx, y = (n / P->nx) % P->ny, z = n / ((int64_t)P->nx * P->ny);
            double hl[2][QMAX], post[2][QMAX];
            for (int c = 0; c < C; c++)
                for (int i = 0; i < q; i++) hl[c][i] = cur[((int64_t)c * q + i) * N + n];
            if (flags && flags[n] == 1) {
                /* full-way bounce-back: a wall node returns each population along the
                 * opposite direction instead of colliding (w_i = w_opp(i), so the same on h) */
                for (int c = 0; c < C; c++)
                    for (int i = 0; i < q; i++) post[c][i] = hl[c][L.opp[i]];
            } else if (FE) {
                double grad[3], lap, hf[QMAX], hg[QMAX];
                if (flags && flags[n] == 3) {
                    complete_missing(P, &L, flags, x, y, z, hl[0], hf);
                    complete_missing(P, &L, flags, x, y, z, hl[1], hg);
                } else {
                    memcpy(hf, hl[0], sizeof(double) * q);
                    memcpy(hg, hl[1], sizeof(double) * q);
                }
                fe_stencil(P, &L, flags, psi, x, y, z, grad, &lap);
                fe_collide(P, &L, hf, hg, grad, lap, post[0], post[1]);
            } else if (flags && flags[n] == 2) {
                double drho = velocity_node_drho(P, &L, flags, x, y, z, hl[0]);
                heq_poly(&L, drho, P->u_bc, post[0]);
            } else if (flags && flags[n] == 3) {
                /* half-way bounce-back node: wet; the missing populations are the reflections
                 * of the ones that reached the node in this step, then the node collides */
                double hc[QMAX];
                complete_missing(P, &L, flags, x, y, z, hl[0], hc);
                collide_single(P, &L, hc, post[0], NULL);
            } else if (C == 1) {
                node_info info = {0, 1};
                collide_single(P, &L, hl[0], post[0], &info);
                if (P->model == ORC_ELBM) {
                    int b = info.iters < 31 ? info.iters : 31;
#pragma omp atomic
                    hist[b]++;
                    noconv += !info.converged;
                    nodes++;
                }
            } else {
                /* Shan-Chen with EDM forcing around the common velocity */
                double dr[2], rc[2], jc[2][3], Fc[2][3], up[3], num[3] = {0, 0, 0}, den = 0.0;
                for (int c = 0; c < 2; c++) {
                    moments(&L, hl[c], &dr[c], jc[c]);
                    rc[c] = 1.0 + dr[c];
                    sc_force(P, &L, psi, N, x, y, z, c, rc[c], Fc[c]);
                    for (int a = 0; a < 3; a++) num[a] += jc[c][a] / P->tau;
                    den += rc[c] / P->tau;
                }
                for (int a = 0; a < 3; a++) up[a] = num[a] / den;
                for (int c = 0; c < 2; c++) {
                    double h0[QMAX], h1[QMAX], u1[3];
                    for (int a = 0; a < 3; a++) u1[a] = up[a] + Fc[c][a] / rc[c];
                    heq_poly(&L, dr[c], up, h0);
                    heq_poly(&L, dr[c], u1, h1);
                    for (int i = 0; i < q; i++)
                        post[c][i] = hl[c][i] + (h0[i] - hl[c][i]) / P->tau + (h1[i] - h0[i]);
                }
            }
            /* propagation: the value leaving node x along e_i lands on x + e_i */
            for (int i = 0; i < q; i++) {
                int64_t dst = neighbour(P, x, y, z, L.e[i]);
                for (int c = 0; c < C; c++) nxt[((int64_t)c * q + i) * N + dst] = post[c][i];
            }
        }
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)C * q * N; k++) f[k] = L.w[(k / N) % q] + cur[k];
    free(cur);
    free(nxt);
    free(psi);
    if (st) {
        for (int b = 0; b < 32; b++) st->newton_hist[b] += hist[b];
        st->nonconverged += noconv;
        st->nodes += nodes;
    }
    return 0;
}

int orc_macro(const orc_params *P, const uint8_t *flags, const double *f, double *rho, double *u) {
    if (check_params(P)) return -1;
    lattice_t L;
    make_lattice(P->lattice, &L);
    const int q = L.q;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    const int C = ncomp_of(P);
    const int FE = P->model == ORC_FREE_ENERGY;
    double *psi = NULL;
    if (C == 2 && !FE) {
        psi = (double *)malloc(sizeof(double) * 2 * N);
        if (!psi) return -3;
        for (int64_t n = 0; n < N; n++)
            for (int c = 0; c < 2; c++) {
                double r = 0.0;
                for (int i = 0; i < q; i++) r += f[((int64_t)c * q + i) * N + n] - L.w[i];
                psi[c * N + n] = psi_of(P, 1.0 + r);
            }
    }
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int64_t x = n % P->nx, y = (n / P->nx) % P->ny, z = n / ((int64_t)P->nx * P->ny);
        double rc[2], jc[2][3], hl[QMAX], dr;
        for (int c = 0; c < C; c++) {
            for (int i = 0; i < q; i++) hl[i] = f[((int64_t)c * q + i) * N + n] - L.w[i];
            if (flags && flags[n] == 3 && (C == 1 || FE)) {
                double hc[QMAX];
                complete_missing(P, &L, flags, x, y, z, hl, hc);
                memcpy(hl, hc, sizeof(double) * q);
            }
            moments(&L, hl, &dr, jc[c]);
            rc[c] = 1.0 + dr;
            rho[c * N + n] = rc[c];
        }
        if (FE) {
            /* rho[1] is phi; velocity (j + F/2)/rho of the f lattice, zero on walls */
            double v[3] = {0, 0, 0};
            if (!(flags && flags[n] == 1))
                for (int a = 0; a < 3; a++) v[a] = (jc[0][a] + 0.5 * rc[0] * P->g[a]) / rc[0];
            for (int a = 0; a < 3; a++) u[a * N + n] = v[a];
            continue;
        }
        double v[3] = {0, 0, 0};
        if (flags && flags[n] == 2 && C == 1) {
            for (int i = 0; i < q; i++) hl[i] = f[(int64_t)i * N + n] - L.w[i];
            rho[n] = 1.0 + velocity_node_drho(P, &L, flags, x, y, z, hl);
            for (int a = 0; a < 3; a++) v[a] = P->u_bc[a];
        } else if (!(flags && flags[n] == 1)) {
            if (C == 1) {
                double gfac = P->model == ORC_ELBM ? 0.0 : 0.5;
                for (int a = 0; a < 3; a++) v[a] = (jc[0][a] + gfac * rc[0] * P->g[a]) / rc[0];
            } else {
                /* mixture velocity (sum_c j_c + F_total/2) / sum_c rho_c */
                double Fc[3], num[3] = {jc[0][0] + jc[1][0], jc[0][1] + jc[1][1], jc[0][2] + jc[1][2]};
                for (int c = 0; c < 2; c++) {
                    sc_force(P, &L, psi, N, x, y, z, c, rc[c], Fc);
                    for (int a = 0; a < 3; a++) num[a] += 0.5 * Fc[a];
                }
                for (int a = 0; a < 3; a++) v[a] = num[a] / (rc[0] + rc[1]);
            }
        }
        for (int a = 0; a < 3; a++) u[a * N + n] = v[a];
    }
    free(psi);
    return 0;
}
