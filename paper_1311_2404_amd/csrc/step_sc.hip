// Two-component Shan-Chen kernels: the pseudopotential pre-pass and the step.
#include "dispatch.hpp"
#include "step_sc.hpp"

namespace lbm {

hipError_t launch_psi(int lattice, int storage, int layout, const StepParams &p, const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_wide_storage(storage, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                k_psi<L, St, LAY><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_step_sc(int lattice, int storage, int layout, const StepParams &p, const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_wide_storage(storage, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                k_step_sc<L, St, LAY><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
