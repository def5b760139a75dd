// Compile-time dispatch helpers and the launcher entry points implemented by the
// kernel translation units (one per collision model, plus the auxiliary kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.hpp"
#include "params.hpp"
#include "storage.hpp"

namespace lbm {

struct LaunchCfg {
    dim3 grid, block;
    hipStream_t stream;
};

template <class F>
hipError_t with_lattice(int lattice, F &&f) {
    return lattice == 0 ? f(D2Q9{}) : f(D3Q19{});
}

// Storage traits, stochastic-rounding variants included when SR_VARIANTS.
template <bool SR_VARIANTS, class F>
hipError_t with_storage(int storage, int sr, F &&f) {
    switch (storage) {
    case ST_F64: return f(StF64{});
    case ST_F32: return f(StF32{});
    case ST_F32S: return f(StF32S{});
    case ST_BF16S:
        if constexpr (SR_VARIANTS) {
            if (sr) return f(StBF16S<true>{});
        }
        return f(StBF16S<false>{});
    case ST_F16S:
        if constexpr (SR_VARIANTS) {
            if (sr) return f(StF16S<true>{});
        }
        return f(StF16S<false>{});
    default: return hipErrorInvalidValue;
    }
}

// The 4- and 8-byte storages only: the two-component models (Shan-Chen, free energy),
// whose densities leave 1 by O(1), keep no 16-bit populations.
template <class F>
hipError_t with_wide_storage(int storage, F &&f) {
    switch (storage) {
    case ST_F64: return f(StF64{});
    case ST_F32: return f(StF32{});
    case ST_F32S: return f(StF32S{});
    default: return hipErrorInvalidValue;
    }
}

template <class F>
hipError_t with_layout(int layout, F &&f) {
    switch (layout) {
    case LAYOUT_AB: return f(std::integral_constant<int, LAYOUT_AB>{});
    case LAYOUT_AA_EVEN: return f(std::integral_constant<int, LAYOUT_AA_EVEN>{});
    default: return f(std::integral_constant<int, LAYOUT_AA_ODD>{});
    }
}

// step kernels (step_bgk.hip, step_mrt.hip, step_elbm.hip, step_sc.hip); flags: 0 none,
// 1 fluid and wall nodes, 2 also equilibrium velocity nodes
hipError_t launch_step_bgk(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c);
hipError_t launch_step_mrt(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c);
// step_fe.hip: the free-energy order-parameter pre-pass (phi into p.psi) and step
hipError_t launch_fe_phi(int lattice, int storage, int layout, bool flags, const StepParams &p, const LaunchCfg &c);
hipError_t launch_step_fe(int lattice, int storage, int layout, bool flags, const StepParams &p,
                          const LaunchCfg &c);
// step_reg.hip, step_smag.hip
hipError_t launch_step_reg(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c);
hipError_t launch_step_smag(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                            const LaunchCfg &c);
hipError_t launch_step_elbm(int lattice, int storage, int layout, int flags, const StepParams &p,
                            const LaunchCfg &c);
hipError_t launch_step_sc(int lattice, int storage, int layout, const StepParams &p, const LaunchCfg &c);
hipError_t launch_psi(int lattice, int storage, int layout, const StepParams &p, const LaunchCfg &c);

// auxiliary kernels (aux.hip)
struct PlaneParams {
    int nx, ny, nz;
    uint32_t N;
    uint32_t S;        // population stride (elements)
    uint32_t rp;       // population tile pitch (elements)
    uint32_t rpitch;   // population row pitch inside a tile (elements)
    int tyl;           // log2 of the rows per tile
    int layout;        // LAYOUT_* of the state being accessed
    int comp, q;       // component and population index of the plane
    void *pop;         // population array (all components)
    double *plane;     // FP64 plane [N] on the device
    const double *rho; // init: rho of this component [N]
    const double *u;   // init: u[3][N]
    const double *df;  // init: optional perturbation plane [N]
    int entropic;      // init: entropic equilibrium instead of the polynomial one
    int fe;            // init: free-energy equilibria (zero phi gradients) of lattice comp
    const double *phi; // init, free energy: phi[N]
    double fe_a, fe_gamma;
    int plain;         // the stored values of this plane are plain f (the free-energy g
                       // lattice in every storage), not f - w
};
hipError_t launch_init_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c);
hipError_t launch_get_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c);
hipError_t launch_set_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c);

struct MacroParams {
    int nx, ny, nz;
    uint32_t N;
    uint32_t S;        // population stride (elements)
    uint32_t rp;       // population tile pitch (elements)
    uint32_t rpitch;   // population row pitch inside a tile (elements)
    int tyl;           // log2 of the rows per tile
    int layout, model, ncomp;
    const void *pop;
    const uint8_t *flags;
    const void *psi;   // Shan-Chen pseudopotential (model == SC)
    double G, g[3];
    double u_bc[3];    // velocity of the equilibrium velocity nodes (flag 2)
    void *rho_out, *u_out;
    int fp64;
    unsigned int *bad;  // count of non-finite / non-positive densities (or nullptr)
};
hipError_t launch_macro(int lattice, int storage, const MacroParams &p, const LaunchCfg &c);

// deterministic FP64 reduction of (rho[C][N], u[3][N]) into out[8]
hipError_t launch_diag_reduce(const double *rho, const double *u, uint32_t N, int ncomp, int phi2, double *partials,
                              int nblocks, double *out, hipStream_t s);
// the same sums taken straight from the populations (no field pass): nblocks partial sets
// of 8 doubles in partials[], the result in out[8]
hipError_t launch_diag_fused(int lattice, int storage, const MacroParams &p, double *partials, int nblocks,
                             double *out, hipStream_t s);

// MLP kernels (mlp.hip)
struct MlpDatasetParams {
    StepParams sp;
    int64_t n;
    uint64_t seed;
    float *feat;
    double *alpha;
    uint8_t *valid;
    int layout;
};
hipError_t launch_alpha_dataset(int lattice, int storage, const MlpDatasetParams &p, hipStream_t s);
hipError_t mlp_forward_bf16(const float *wf, const uint32_t *lane, const float *x, int64_t n, float *y,
                            hipStream_t s);
hipError_t mlp_loss_grad(const float *w, const float *x, const double *t, int64_t n, const float *mu,
                         const float *isd, float *partials, int nparts, float *grad, double *loss, hipStream_t s);
hipError_t mlp_train_batch(const float *w, const float *x, const double *t, int64_t row0, int64_t nbatch,
                           int64_t n_all, uint64_t pa, uint64_t pb, const float *mu, const float *isd, double tmean,
                           double tinv, float *partials, float *grad, double *loss_acc, hipStream_t s);
// acc[0] = sum, acc[1] = sum of squares of alpha - series base; acc[2 .. 2 + 128) scratch
hipError_t mlp_resid_moments(const float *x, const double *t, int64_t n, double *acc, hipStream_t s);
constexpr int MLP_TRAIN_BLOCK = 64;  // one wave per training block
hipError_t mlp_adam(float *w, const float *grad, float *m, float *v, int t, float lr, hipStream_t s);
hipError_t mlp_to_bf16(const float *w, const float *norm, uint16_t *wb, float *wf, uint32_t *lane, hipStream_t s);
hipError_t mlp_moments(const float *x, int64_t n, double *acc, hipStream_t s);

}  // namespace lbm
