// Kernel parameter block shared by the launchers and the kernels.
#pragma once
#include <stdint.h>

namespace lbm {

enum Layout { LAYOUT_AB = 0, LAYOUT_AA_EVEN = 1, LAYOUT_AA_ODD = 2 };
enum Model { M_BGK = 0, M_MRT = 1, M_ELBM = 2, M_SC = 3, M_REG = 4, M_SMAG = 5, M_FE = 6 };

constexpr int MLP_IN = 6;
constexpr int MLP_H = 32;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 1313
constexpr int MLP_NNORM = 2 * MLP_IN;                 // input normalisation mu[6], isd[6]
constexpr int MLP_NTOTAL = MLP_NPARAM + MLP_NNORM;     // 1325
constexpr int MLP_LANE_WORDS = 44;  // per-lane words of the wave-level (MFMA) network's operand table
constexpr int NEWTON_BINS = 32;

// Passed by value as the kernel argument of every step-like kernel.
struct StepParams {
    int nx, ny, nz;
    uint32_t N;                 // nodes per component
    uint32_t rp;                // population tile pitch: node (x, y, z) sits at offset
    uint32_t rpitch;            // (z ceil(ny / 2^tyl) + (y >> tyl)) rp + (y & (2^tyl - 1)) rpitch + x
    int tyl;                    // of a slot's block (SoA: rp = nx, tyl = 0)
    uint32_t S;                 // population stride in elements (>= N; padding spreads the
                                // Q streams of a row over HBM channels)
    const void *src;            // populations read (AB: current copy; AA: the single copy)
    void *dst;                  // populations written (AB: the other copy; AA: == src)
    const uint8_t *flags;       // node flags or nullptr
    // physics
    double omega;               // 1/tau
    double g[3];                // body acceleration
    float g_f[3];               // the same in FP32
    int has_force;
    // MRT relaxation with the basis row's squared norm |M_k|^2 folded in: the rescaled
    // post-collision moment is a_k = mrt[0][k] m_k + mrt[1][k] meq_k + mrt[2][k] mF_k, the
    // three being (1 - s_k), s_k and 1 - s_k/2 over |M_k|^2; for the conserved rows
    // mrt[0][k] = 1/|M_k|^2 and the others are 0.  mrt_f holds the same in FP32.
    double mrt[3][19];
    float mrt_f[3][19];
    double u_bc[3];             // velocity of the equilibrium velocity nodes (flag 2)
    double tau_a, tau_b, tau_phi;  // free energy: f relaxation at phi = +1 / -1, g relaxation
    double fe_a, fe_kappa, fe_gamma;  // free energy: A, kappa, Gamma
    double tau0;                // Smagorinsky: base relaxation time
    double smag_k;              // Smagorinsky: 4 cs^-4 C_S^2 = 36 C_S^2
    // entropic LBM
    double beta;                // 1/(2 tau)
    double alpha_tol;
    int alpha_maxit;
    int alpha_init;             // 0: 2, 1: series, 2: MLP
    const uint16_t *mlp;        // bf16 MLP weights (alpha_init == 2)
    const float *mlp_wf;        // the same weights widened to FP32, then mu[6], isd[6]
    const uint32_t *mlp_lane;   // per-lane MFMA operand table of the wave-level network
    unsigned long long *stats;  // [NEWTON_BINS] histogram + [1] non-converged, or nullptr
    // Shan-Chen
    const void *psi;            // psi[2][N] in compute precision
    double G;
    int psi_mode;               // 0: psi = rho, 1: 1 - exp(-rho)
    // stochastic rounding stream
    uint32_t seed;
    uint32_t step;
    unsigned int *diverged;     // raised by a step that produces a non-finite population
};

}  // namespace lbm
