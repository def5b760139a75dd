// Step-kernel instantiations for the MRT collision (all storages, layouts, flag modes).
#include "dispatch.hpp"
#include "step.hpp"

namespace lbm {

hipError_t launch_step_mrt(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<true>(storage, sr, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                if (flags == 2) k_step<L, St, M_MRT, LAY, 2><<<c.grid, c.block, 0, c.stream>>>(p);
                else if (flags) k_step<L, St, M_MRT, LAY, 1><<<c.grid, c.block, 0, c.stream>>>(p);
                else k_step<L, St, M_MRT, LAY, 0><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
