/*
 * FP64 CPU oracle for the fused lattice Boltzmann stream-and-collide step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the HIP path is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the HIP library: its lattice tables are typed in here
 * from the paper's weight table and the velocity ordering documented below.
 *
 * Velocity ordering (opposite pairs adjacent, opp(i) = i+1 for odd i):
 *   D2Q9 : 0 (0,0) 1 (1,0) 2 (-1,0) 3 (0,1) 4 (0,-1) 5 (1,1) 6 (-1,-1) 7 (-1,1) 8 (1,-1)
 *   D3Q19: 0 rest, 1/2 +-x, 3/4 +-y, 5/6 +-z, 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0)
 *          11 (1,0,1) 12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1)
 *          17 (0,1,-1) 18 (0,-1,1)
 *
 * Array layouts: populations f[C][Q][N], N = nx*ny*nz with x fastest
 * (node n = x + nx*(y + ny*z)); flags[N] (0 fluid, 1 full-way bounce-back wall,
 * 2 equilibrium velocity node with the velocity u_bc, 3 half-way bounce-back node);
 * densities rho[C][N]; velocities u[3][N] (the z row is zero on D2Q9).  C = 2 for the
 * Shan-Chen and free-energy models; for the latter component 1 is the order-parameter
 * lattice g and rho[1] is phi.
 *
 * Parity unpinned (no printed values in the paper): the MRT, ELBM,
 * Shan-Chen, regularized and Smagorinsky steps beyond the identities and
 * closed forms the tests check.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };
enum { ORC_BGK = 0, ORC_MRT = 1, ORC_ELBM = 2, ORC_SHANCHEN = 3, ORC_REG = 4, ORC_SMAG = 5, ORC_FREE_ENERGY = 6 };

typedef struct {
    int lattice, model;
    int nx, ny, nz;
    double tau;
    double g[3];          /* body acceleration; the force density is rho*g */
    double s[19];         /* MRT rates, moment order (see orc_mrt_matrix) */
    int alpha_init;       /* ELBM first guess: 0 -> 2, 1 -> series, 2 -> MLP */
    double alpha_tol;     /* Newton stop |d alpha| <= tol */
    int alpha_maxit;
    const double *mlp;    /* alpha_init == 2: 1325 MLP parameters (1313 weights, mu[6], isd[6]) */
    double G;             /* Shan-Chen coupling */
    int psi;              /* 0: psi = rho, 1: psi = 1 - exp(-rho) */
    double cs_smag;       /* Smagorinsky constant C_S (ORC_SMAG) */
    double u_bc[3];       /* velocity of the equilibrium velocity nodes (flag 2) */
    /* free-energy binary model: tau is tau_A (phi = +1); populations f (density) and g
     * (order parameter phi) are components 0 and 1 */
    double tau_b, tau_phi, fe_a, fe_kappa, fe_gamma;
} orc_params;

typedef struct {
    int64_t newton_hist[32];  /* ELBM nodes by Newton iteration count (0 = short-cut) */
    int64_t nonconverged;
    int64_t nodes;
} orc_stats;

int orc_q(int lattice);
void orc_tables(int lattice, int *e /* q*3 */, double *w, int *opp);
void orc_feq(int lattice, double rho, const double *u, double *feq);
void orc_feq_entropic(int lattice, double rho, const double *u, double *feq);
void orc_mrt_matrix(int lattice, double *M /* q*q row-major */);
double orc_H(int lattice, const double *f);
double orc_alpha(int lattice, const double *f, const double *feq, int init, const double *mlp,
                 double vsq, double tol, int maxit, int *iters, int *converged);
void orc_alpha_features(int lattice, const double *f, const double *feq, double rho, double vsq,
                        double *feat /* 6 */);
/* MLP on raw features x[n][6] with parameters p[1325]; gradient over the first 1313 */
void orc_mlp_forward(const double *p, const double *x, int64_t n, double *y);
double orc_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t n, double *grad);
void orc_collide_node(const orc_params *P, const double *f, double *out);
void orc_collide_node_sc(const orc_params *P, const double *f2, const double *psi_nb, double *out2);
int orc_init_eq(const orc_params *P, const double *rho, const double *u, const double *df, double *f);
int orc_run(const orc_params *P, const uint8_t *flags, double *f, int steps, orc_stats *st);
int orc_macro(const orc_params *P, const uint8_t *flags, const double *f, double *rho, double *u);
/* Free-energy equilibria of one node (full populations, not shifted), given rho, phi,
 * u[3], grad phi[3] and the Laplacian of phi. */
void orc_fe_equilibria(const orc_params *P, double rho, double phi, const double *u, const double *grad,
                       double lap, double *feq, double *geq);
/* The gradient and Laplacian stencils at node (x, y, z) of a phi[N] field. */
void orc_fe_stencil(const orc_params *P, const uint8_t *flags, const double *phi, int x, int y, int z,
                    double *grad, double *lap);
int orc_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
