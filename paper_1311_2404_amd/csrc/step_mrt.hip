// Step-kernel instantiations for the MRT collision (all storages, layouts, flag modes).
#include "dispatch.hpp"
#include "step.hpp"
#include "step_vec.hpp"

namespace lbm {

hipError_t launch_step_mrt(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                           const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<true>(storage, sr, [&](auto st) {
            using St = decltype(st);
#if defined(LBM_VEC_STEP)
            // 16-byte accesses per population when the row fits a wave
            constexpr int VW = 16 / int(sizeof(typename St::T));
            if (layout == LAYOUT_AB && flags != 2 && vec_width(p.nx, int(sizeof(typename St::T))) == VW) {
                const int R = p.nx / VW, by = 256 / R;
                const dim3 grid(1, (p.ny + by - 1) / by, p.nz), block(R, by, 1);
                if (flags) k_step_vec<L, St, M_MRT, true, VW><<<grid, block, 0, c.stream>>>(p);
                else k_step_vec<L, St, M_MRT, false, VW><<<grid, block, 0, c.stream>>>(p);
                return hipGetLastError();
            }
#endif
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
