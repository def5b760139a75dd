/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann stream-and-collide library.
 *
 * The operation is the fused LBM time step of Januszewski & Kostur, "Sailfish: a
 * flexible multi-GPU implementation of the lattice Boltzmann method" (CPC 2014):
 * per node, gather the populations that stream in, compute the macroscopic moments
 * (section 2, macroscopic-field equation), relax towards equilibrium (LBGK equation
 * with the sign of the GPU kernel algorithm; MRT collision equation; entropic LBM
 * equations; Shan-Chen force equation; the regularized and Smagorinsky variants of
 * LBGK from the enhanced-stability subsections), apply full-way bounce-back on wall nodes
 * (boundary-conditions subsection), and store.  Body forces use Guo's scheme (force
 * equation of the body-forces subsection), Shan-Chen uses the exact difference method.
 *
 * Conventions shared by every call:
 *  - Every call returns an int status (LBM_OK or a negative LBM_E* code); nothing
 *    throws across the ABI.  On error no state is changed and lbm_last_error() gives a
 *    message.  Calls on one handle are not thread-safe; separate handles are independent.
 *  - The library owns all device memory of a handle and frees it in lbm_destroy().
 *    Host buffers belong to the caller and are copied in or out during the call.
 *    Device pointers passed to *_device calls are borrowed for the duration of the call.
 *  - Node index n = x + nx*(y + ny*z), x fastest.  Host arrays are FP64, C order:
 *    populations f[C][Q][N] (canonical, unshifted: the value that streams along e_i into
 *    node n at the current time), densities rho[C][N], velocities u[3][N] (row z is zero
 *    on D2Q9).  C = 2 for the Shan-Chen model, else 1.
 *  - Velocity order (opposite pairs adjacent: opp(i) = i+1 for odd i, i-1 for even i>0):
 *      D2Q9 : 0 (0,0) 1 (1,0) 2 (-1,0) 3 (0,1) 4 (0,-1) 5 (1,1) 6 (-1,-1) 7 (-1,1) 8 (1,-1)
 *      D3Q19: 0 rest, 1/2 +-x, 3/4 +-y, 5/6 +-z, 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0)
 *             10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1)
 *             16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1)
 *  - Weights (paper's weight table): D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36 by link
 *    length 0, 1, sqrt 2.  Lattice units, c_s^2 = 1/3, nu = (tau - 1/2)/3.
 *  - All boundaries are periodic; walls are explicit flagged nodes.
 *  - Asynchrony: lbm_step() only enqueues kernels on the handle's stream; calls that
 *    return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sim lbm_sim; /* opaque; owned by the library */

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
/* Collision models: LBGK, MRT, entropic LBGK, two-component Shan-Chen, regularized LBGK
 * (the non-equilibrium part replaced by its second-order projection w_i/(2 cs^4)
 * (e_i e_i - cs^2 I):Pi_neq before relaxing; regularized-LBM subsection) and
 * Smagorinsky LBGK (local tau = tau0 + tau_t from the momentum flux of f - feq,
 * Smagorinsky-subgrid equations), and the free-energy binary fluid (free energy model
 * subsection: a density lattice f and an order-parameter lattice g, C = 2, with the
 * chemical potential, the pressure tensor and the gradient stencils; see
 * lbm_set_free_energy). */
enum { LBM_BGK = 0, LBM_MRT = 1, LBM_ELBM = 2, LBM_SHANCHEN = 3, LBM_REGULARIZED = 4, LBM_SMAGORINSKY = 5,
       LBM_FREE_ENERGY = 6 };
/* Storage of the populations in HBM.  S = shifted: the stored value is f_i - w_i (the
 * round-off minimising formulation of the precision subsection); compute is FP32 for
 * every storage except F64. */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F32S = 2, LBM_BF16S = 3, LBM_F16S = 4 };
/* Streaming pattern (GPU-algorithms subsection): AB = two copies, ping-pong;
 * AA = one copy updated in place, even and odd steps access different slots. */
enum { LBM_AB = 0, LBM_AA = 1 };
/* Population layouts in HBM (lbm_set_pop_layout). */
enum { LBM_POP_TILED = 0, LBM_POP_SOA = 1 };
/* uint8 node flags (boundary-conditions subsection): fluid; full-way bounce-back wall (a
 * dry node that returns what it receives); equilibrium velocity node (a fluid node on a
 * domain face whose populations streamed in from wall nodes are missing: each takes the
 * value of its opposite at the node, rho is summed over the completed set, and the node
 * leaves feq(rho, u_bc), the equilibrium approach); half-way bounce-back node (a wet
 * node next to wall nodes: its missing populations are completed the same way, which
 * reflects what reached it in the same step, and it then collides as a fluid node; the
 * wall lies beyond it). */
enum { LBM_FLUID = 0, LBM_WALL_BB = 1, LBM_VELOCITY = 2, LBM_HALFWAY_BB = 3 };
enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* invalid argument */
    LBM_ENOMEM = -2,      /* device allocation failed */
    LBM_EHIP = -3,        /* HIP runtime error */
    LBM_ESTATE = -4,      /* call out of order (e.g. step before init) */
    LBM_EUNSUPPORTED = -5,/* valid but unsupported combination */
    LBM_EDIVERGED = -6    /* non-finite or non-positive density found */
};

/* Create a simulation.  lattice LBM_D2Q9 needs nz == 1.  tau > 1/2 is the relaxation
 * time (for MRT the stress-moment rate is 1/tau unless lbm_set_mrt_rates says
 * otherwise).  force[3] is a uniform body acceleration g (force density rho g); NULL
 * means zero; force[2] is ignored on D2Q9.  ELBM and the regularized model take no
 * force (LBM_EUNSUPPORTED).  Nothing is allocated
 * on the device until lbm_init_eq() or lbm_set_f().  *out receives the handle. */
int lbm_create(int lattice, int model, int nx, int ny, int nz, double tau,
               const double *force, lbm_sim **out);

/* Storage (LBM_F64 ... LBM_F16S) and layout (LBM_AB, LBM_AA); stochastic_round != 0
 * rounds BF16/F16 stores stochastically (counter-hash seeded, unbiased) instead of to
 * nearest even (LBGK, MRT, regularized and Smagorinsky only: LBM_EUNSUPPORTED for the
 * other models).  The Shan-Chen and free-energy models keep F64, F32 or shifted F32
 * populations (LBM_EUNSUPPORTED): their component densities leave 1 by O(1), where the
 * 16-bit rounding of f - w no longer conserves mass.  Only before the first init;
 * default LBM_F32, LBM_AB, round to nearest. */
int lbm_set_storage(lbm_sim *sim, int storage, int layout, int stochastic_round);

/* Population layout in HBM.  Only before the first init; the results do not depend on
 * it (every layout gives the same fields bit for bit), only the speed does.
 *  - LBM_POP_TILED (default): f[z][y/TY][c][q][y%TY][x].  Each x row of each population
 *    is a run of nx elements rounded up to 256 bytes, plus row_pad bytes; the C*Q runs of
 *    TY = tile_rows consecutive rows lie together, followed by block_pad bytes.
 *    tile_rows 0 picks the largest power of two up to 64 whose run of TY rows holds at
 *    most 32 KB (32 rows at nx = 256 in FP32, 16 in FP64, 64 in BF16); otherwise a
 *    power of two from 1 to 64.  block_pad -1 means
 *    1024.  TY is halved while half of it still covers ny.  Grids whose tiled layout
 *    would not fit 32-bit element offsets fall back to LBM_POP_SOA.
 *  - LBM_POP_SOA: the structure of arrays f[c][q][z][y][x] of the paper's GPU data
 *    layout; consecutive population arrays are N elements apart, rounded up to 256
 *    bytes, plus soa_pad bytes (-1 means 17 * 256).
 * Pads are rounded down to whole 256 bytes and must lie in [0, 1 MiB].  Arguments that
 * do not apply to the chosen kind are checked and ignored.  Bad values: LBM_EINVAL. */
int lbm_set_pop_layout(lbm_sim *sim, int kind, int tile_rows, int64_t row_pad, int64_t block_pad,
                       int64_t soa_pad);

/* MRT relaxation rates s[q], q = 9 or 19, in the moment order of the orthogonal basis
 * of d'Humieres et al. (2002) that the MRT subsection cites: D3Q19 rows 1, e, eps,
 * jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz; D2Q9 rows
 * 1, e, eps, jx, qx, jy, qy, pxx, pxy.  The rates of conserved rows (rho, j) do not
 * affect the result.  Default: every non-conserved rate 1/tau (MRT == BGK). */
int lbm_set_mrt_rates(lbm_sim *sim, const double *s, int q);

/* ELBM alpha solve: alpha_init 0 starts Newton at 2, 1 at the series estimate, 2 at
 * the MLP proposal (weights from lbm_mlp_set_weights); tol > 0 stops Newton at
 * |d alpha| <= tol; max_iter in [1, 64].  Default 0, 1e-10, 20. */
int lbm_set_elbm(lbm_sim *sim, int alpha_init, double tol, int max_iter);

/* Shan-Chen: coupling G (G > 0 repulsive) and pseudopotential psi (0: rho,
 * 1: 1 - exp(-rho)).  Default G = 0, psi = 0. */
int lbm_set_shanchen(lbm_sim *sim, double G, int psi);

/* LBM_FREE_ENERGY parameters: f relaxes with tau_rho = tau_B + (phi + 1)/2 (tau - tau_B)
 * (tau from lbm_create is tau_A, the relaxation time where phi = +1), g with tau_phi;
 * free energy A (bulk) and kappa (interface), mobility parameter Gamma.  The equilibria
 * give the second moments the subsection requires (pressure tensor with bulk pressure
 * rho/3 + A(-phi^2/2 + 3 phi^4/4) and chemical potential A(-phi + phi^3) - kappa lap phi),
 * with isotropic lattice-weight gradient and Laplacian stencils; a wall neighbour enters
 * them with the node's own phi.  The body force acts on f by the exact difference method.
 * Populations: f is component 0, g component 1; lbm_init_eq's rho[1] and lbm_macro's
 * rho[1] are phi; the velocity is (j_f + F/2)/rho.  Storage F64, F32 or shifted F32
 * (the step works on f - w; shifted storage keeps small forces, see the tests).  Default
 * tau_B = tau, tau_phi = 1, A = 0.04, kappa = 0.04, Gamma = 1; other models:
 * LBM_EUNSUPPORTED. */
int lbm_set_free_energy(lbm_sim *sim, double tau_b, double tau_phi, double a, double kappa, double gamma);

/* Velocity u[3] of every LBM_VELOCITY node (u[2] ignored on D2Q9); default 0.  The
 * macroscopic output of such a node is the density of its completed set and this
 * velocity.  Velocity nodes are accepted by lbm_set_flags for LBM_BGK, LBM_MRT,
 * LBM_REGULARIZED and LBM_SMAGORINSKY. */
int lbm_set_velocity_bc(lbm_sim *sim, const double u[3]);

/* Smagorinsky constant C_S >= 0 of the LBM_SMAGORINSKY model (subgrid-model
 * subsection): tau_t = (sqrt(tau0^2 + 4 cs^-4 C_S^2 |Q|) - tau0)/2 with
 * Q_ab = sum_i e_ia e_ib (f_i - feq_i), |Q| = (Q_ab Q_ab)^(1/2), tau = tau0 + tau_t, and the
 * LBGK step (Guo source included) at that tau.  C_S = 0 is LBGK.  Default 0.1.  Other
 * models: LBM_EUNSUPPORTED. */
int lbm_set_smagorinsky(lbm_sim *sim, double cs);

/* HIP stream (hipStream_t cast to void*) for every launch and copy of this handle;
 * NULL = the null stream. */
int lbm_set_stream(lbm_sim *sim, void *hip_stream);

/* Node flags, host array uint8[N] (LBM_FLUID / LBM_WALL_BB / LBM_VELOCITY /
 * LBM_HALFWAY_BB), copied.  Before or after init.  Values above 3: LBM_EINVAL.  Walls
 * are not supported with LBM_SHANCHEN, velocity and half-way nodes not with LBM_SHANCHEN
 * or LBM_ELBM, velocity nodes not with LBM_FREE_ENERGY (LBM_EUNSUPPORTED).  The macroscopic output of a half-way node is that of
 * its completed population set. */
int lbm_set_flags(lbm_sim *sim, const uint8_t *flags);

/* Initialise f = f_eq(rho, u) (the entropic equilibrium for ELBM, else the polynomial
 * one) plus an optional perturbation df[C][Q][N] (NULL = none).  Host FP64 arrays
 * rho[C][N], u[D][N] (D = 2 on D2Q9, 3 on D3Q19).  Allocates device state on first use.
 * Resets the step counter to 0. */
int lbm_init_eq(lbm_sim *sim, const double *rho, const double *u, const double *df);

/* Set / get the canonical FP64 populations f[C][Q][N] (host).  lbm_set_f allocates
 * on first use and resets the step counter; values are rounded to the storage type. */
int lbm_set_f(lbm_sim *sim, const double *f);
int lbm_get_f(lbm_sim *sim, double *f);

/* Enqueue n >= 0 time steps on the handle's stream (asynchronous).  A step kernel that
 * produces a non-finite population raises a device flag; the next lbm_sync() reads it and
 * returns LBM_EDIVERGED.  From then on lbm_step() returns LBM_EDIVERGED without
 * enqueuing anything, until lbm_init_eq() or lbm_set_f() gives the handle a new state. */
int lbm_step(lbm_sim *sim, int n);

/* Macroscopic fields of the current state into host FP64 arrays rho[C][N] and
 * u[3][N].  u is the physical velocity (j + F/2)/rho (Guo); for Shan-Chen the mixture
 * velocity (sum_c j_c + sum_c F_c / 2) / sum_c rho_c; wall nodes report u = 0.
 * Synchronises; returns LBM_EDIVERGED if any density is non-finite or <= 0. */
int lbm_macro(lbm_sim *sim, double *rho, double *u);

/* Same into caller device buffers (e.g. torch tensors): rho_dev[C][N], u_dev[3][N],
 * FP64 if fp64 != 0 else FP32.  Enqueued on the handle's stream; no divergence check. */
int lbm_macro_device(lbm_sim *sim, void *rho_dev, void *u_dev, int fp64);

/* Diagnostics (section 5's kinetic energy tracked on the GPU), deterministic FP64
 * reductions: out[0..1] mass per component (out[1] = 0 if C == 1), out[2..4] total
 * momentum sum_c j_c + F/2, out[5] kinetic energy (1/2N) sum |u|^2, out[6] number of
 * nodes with non-finite or non-positive density.  Synchronises. */
int lbm_diag(lbm_sim *sim, double out[8]);

/* lbm_diag without allocating: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).  The
 * same eight sums as lbm_diag (out[7] = 0), taken straight from the populations by a
 * fused reduction (no FP64 field pass, so the sums agree with lbm_diag's to rounding
 * order, ~1e-15 relative), written into the caller's device buffer out_dev (8 doubles,
 * FP64) and enqueued on the handle's stream without synchronising.  No device memory is
 * allocated or freed: the partial sums live in a static device array of 2048 x 8 doubles
 * (131 KB per GPU, held until the process ends) that every call on that GPU shares and
 * fully overwrites, so any lattice fits and nothing needs clearing; calls that overlap on
 * one GPU (several handles on different streams) race on it.  The state must exist
 * (LBM_ESTATE otherwise). */
int lbm_diag_noalloc(lbm_sim *sim, void *out_dev);

/* ELBM Newton statistics since the last reset: hist[k] = node updates that took k
 * Newton iterations (k = 0: alpha = 2 short-cut), k < nbins <= 32; *nonconv = updates
 * without convergence.  enable != 0 turns collection on (it costs an LDS histogram per
 * block); reset != 0 clears the counters.  Synchronises when reading. */
int lbm_elbm_stats(lbm_sim *sim, int enable, int reset, int64_t *hist, int nbins, int64_t *nonconv);

/* ELBM alpha MLP (6 -> 32 -> 32 -> 1, tanh hidden units, linear output), the learned
 * first guess of the alpha Newton solve: the proposal is the series estimate
 * 2 + (x1 - 2 x2)/3 of the root plus the network's output, so the network carries only
 * the series' residual.  params[n]: n = 1313 weights W1[32][6], b1[32], W2[32][32],
 * b2[32], w3[32], b3 (inputs used as given), or n = 1325 with the input normalisation
 * mu[6], isd[6] appended (the network sees (x - mu) * isd).  FP32 in; the library keeps
 * the weights as BF16 for inference and an FP32 master copy for training.  get returns
 * the master copy (n = 1313 or 1325). */
int lbm_mlp_set_weights(lbm_sim *sim, const float *params, int n);
int lbm_mlp_get_weights(lbm_sim *sim, float *params, int n);

/* Sample n node states of the current ELBM field (node index from a counter hash of
 * seed and k) and write, into caller device buffers, the 6 alpha features
 * feat_dev[n][6] (FP32), the Newton alpha from alpha0 = 2 (alpha_dev[n], FP64), and
 * valid_dev[n] (uint8: 0 where the node is within the alpha = 2 short-cut or a wall).
 * Enqueued on the handle's stream. */
int lbm_alpha_dataset(lbm_sim *sim, int64_t n, uint64_t seed, void *feat_dev, void *alpha_dev,
                      void *valid_dev);

/* Train the MLP on device data feat_dev[n][6] (FP32) and alpha_dev[n] (FP64) with MSE
 * and Adam (beta1 0.9, beta2 0.999, eps 1e-8), FP32 master weights starting from the
 * current ones (set them first: LBM_ESTATE otherwise).  The input normalisation is
 * refitted on the data (mean, 1/std) and the current weights are carried over to it
 * exactly; the target, alpha minus the series estimate, is standardised the same way
 * (the output layer is carried into and out of those units exactly), so a new network
 * should start with a zero output layer.  Minibatches of `batch` rows of a seeded
 * permutation each epoch.  loss_out[epochs] (host, may be NULL) receives the mean
 * training loss per epoch, in alpha units. */
int lbm_mlp_train(lbm_sim *sim, const void *feat_dev, const void *alpha_dev, int64_t n,
                  int epochs, int batch, float lr, uint64_t seed, float *loss_out);

/* One forward + backward pass on device data (FP32 math) with the current FP32 master
 * weights and normalisation: mean loss and gradient grad[1313] (host).  For gradient
 * checks. */
int lbm_mlp_loss_grad(lbm_sim *sim, const void *feat_dev, const void *alpha_dev, int64_t n,
                      double *loss, float *grad);

/* MLP inference as in the entropic step: y_dev[n] (FP32 proposal) from feat_dev[n][6].
 * FP32 normalisation; the 64 rows of a wave go through the matrix cores together, with
 * the BF16 weights, the normalised inputs and the hidden activations as BF16 operands
 * and FP32 accumulation. */
int lbm_mlp_forward(lbm_sim *sim, const void *feat_dev, int64_t n, void *y_dev);

/* Steps taken since the last init / set_f. */
int lbm_steps_done(const lbm_sim *sim, int64_t *steps);

/* Wait for the handle's stream.  Returns LBM_EDIVERGED if a step since the last init
 * produced a non-finite population (see lbm_step). */
int lbm_sync(lbm_sim *sim);

/* Message for the last error on this handle (or of the calling thread when sim is NULL). */
const char *lbm_last_error(const lbm_sim *sim);

/* Release the handle and its device memory.  NULL is ignored. */
void lbm_destroy(lbm_sim *sim);

#ifdef __cplusplus
}
#endif
#endif
