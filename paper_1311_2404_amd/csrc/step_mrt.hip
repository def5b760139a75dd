// Step-kernel instantiations for the MRT collision (all storages, layouts, flag modes).
#include "dispatch.hpp"
#include "step.hpp"

namespace lbm {

hipError_t launch_step_mrt(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c) {
    return launch_k_step<M_MRT>(lattice, storage, sr, layout, flags, p, c);
}

}  // namespace lbm
