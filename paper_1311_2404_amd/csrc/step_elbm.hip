// Step-kernel instantiations for the entropic collision (round-to-nearest storages).
#include "dispatch.hpp"
#include "step_elbm.hpp"

namespace lbm {

hipError_t launch_step_elbm(int lattice, int storage, int layout, int flags, const StepParams &p,
                            const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<false>(storage, 0, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                const bool mlp = p.alpha_init == 2 && p.mlp;
                if (mlp) {
                    if (flags) k_step_elbm<L, St, LAY, true, true><<<c.grid, c.block, 0, c.stream>>>(p);
                    else k_step_elbm<L, St, LAY, false, true><<<c.grid, c.block, 0, c.stream>>>(p);
                } else {
                    if (flags) k_step_elbm<L, St, LAY, true, false><<<c.grid, c.block, 0, c.stream>>>(p);
                    else k_step_elbm<L, St, LAY, false, false><<<c.grid, c.block, 0, c.stream>>>(p);
                }
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
