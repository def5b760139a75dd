// Two-component Shan-Chen kernels: the pseudopotential pre-pass and the step.
#include "dispatch.hpp"
#include "step_sc.hpp"

namespace lbm {

namespace {

// The AB and AA odd kernels stage their x shifts in LDS where a workgroup is one whole
// row (no padding lanes); the LDS holds the x-moving values of both components, read and,
// in the AA odd step, written.
bool sc_xstage(int layout, const StepParams &p, const LaunchCfg &c) {
    return layout != LAYOUT_AA_EVEN && int(c.block.x) == p.nx && c.block.y == 1 && c.grid.x == 1 &&
           p.nx % 64 == 0 && p.nx <= 512;
}

template <class L, class St>
size_t sc_lds(int layout, int nx, bool step) {
    const size_t per = 2 * size_t(xmove_count<L>()) * size_t(nx) * sizeof(typename St::T);
    return (step && layout == LAYOUT_AA_ODD) ? 2 * per : per;
}

}  // namespace

hipError_t launch_psi(int lattice, int storage, int layout, const StepParams &p, const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_wide_storage(storage, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                if constexpr (LAY != LAYOUT_AA_EVEN) {
                    if (sc_xstage(LAY, p, c)) {
                        k_psi<L, St, LAY, true><<<c.grid, c.block, sc_lds<L, St>(LAY, p.nx, false), c.stream>>>(p);
                        return hipGetLastError();
                    }
                }
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
                if constexpr (LAY != LAYOUT_AA_EVEN) {
                    if (sc_xstage(LAY, p, c)) {
                        k_step_sc<L, St, LAY, true><<<c.grid, c.block, sc_lds<L, St>(LAY, p.nx, true), c.stream>>>(p);
                        return hipGetLastError();
                    }
                }
                k_step_sc<L, St, LAY><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
