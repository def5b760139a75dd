// The two-component Shan-Chen kernels (multicomponent-models subsection): the
// pseudopotential pre-pass and the step of both components.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step.hpp"

namespace lbm {

// psi_c(x) of component c from the populations that stream into node x at this step
// (the pseudopotential of the multicomponent-models subsection: psi = rho, or 1 - exp(-rho)).
template <class L, class St, int LAYOUT>
__device__ __forceinline__ typename St::C psi_node(const StepParams &p, const Geo &g, int c) {
    using T = typename St::T;
    using C = typename St::C;
    const T *fc = static_cast<const T *>(p.src) + size_t(c) * L::Q * p.S;
    C r = C(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        int slot, dx, dy, dz;
        canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
        r += St::decode(LBM_LOAD(pop_addr(fc, p.S, slot, g, dx, dy, dz), i), C(L::w(i)));
    }
    const C rho = C(1) + r;
    return p.psi_mode == 1 ? C(1) - exp(-rho) : rho;
}

// Shan-Chen pre-pass (the paper's macroscopic-field kernel): psi of both components at
// every node, for the two-kernel step.
template <class L, class St, int LAYOUT>
__global__ __launch_bounds__(512) void k_psi(StepParams p) {
    using C = typename St::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;  // one row (segment) per workgroup
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const Geo g = make_geo(x, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const uint32_t n = g.at(0, 0, 0);
    C *psi = static_cast<C *>(const_cast<void *>(p.psi));
#pragma unroll
    for (int c = 0; c < 2; c++) psi[size_t(c) * p.N + n] = psi_node<L, St, LAYOUT>(p, g, c);
}

// One node of the two-component Shan-Chen step: both components in one pass (they share
// the common velocity), equal relaxation times, EDM forcing.  psi_at(c, dx, dy, dz) gives
// psi_c at the node x + (dx, dy, dz).  Returns whether the node's result is non-finite.
template <class L, class St, int LAYOUT, class PsiAt>
__device__ __forceinline__ bool sc_node(const StepParams &p, const Geo &g, PsiAt psi_at) {
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q;
    const uint32_t S = p.S;
    const T *src = static_cast<const T *>(p.src);
    T *dst = static_cast<T *>(p.dst);

    C h[2][Q];
    Macro<C> m[2];
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int slot, dx, dy, dz;
            canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
            h[c][i] = St::decode(LBM_LOAD(pop_addr(src, S, c * Q + slot, g, dx, dy, dz), i), C(L::w(i)));
        }
        m[c] = moments<L, C>(h[c]);
    }
    // interaction forces: F_c = -G psi_c(x) sum_i w_i psi_other(x + e_i) e_i + rho_c g
    C F[2][3];
#pragma unroll
    for (int c = 0; c < 2; c++) {
        C sx = C(0), sy = C(0), sz = C(0);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const C v = C(L::w(i)) * psi_at(1 - c, L::ex(i), L::ey(i), L::ez(i));
            sx += C(L::ex(i)) * v;
            sy += C(L::ey(i)) * v;
            sz += C(L::ez(i)) * v;
        }
        const C a = -C(p.G) * psi_at(c, 0, 0, 0);
        F[c][0] = a * sx + m[c].rho * C(p.g[0]);
        F[c][1] = a * sy + m[c].rho * C(p.g[1]);
        F[c][2] = a * sz + m[c].rho * C(L::D == 3 ? p.g[2] : 0.0);
    }
    const C irs = C(1) / (m[0].rho + m[1].rho);
    const C ux = (m[0].jx + m[1].jx) * irs, uy = (m[0].jy + m[1].jy) * irs, uz = (m[0].jz + m[1].jz) * irs;
    const C usq15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
    const C omega = C(p.omega);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const C ir = C(1) / m[c].rho;
        const C dx = F[c][0] * ir, dy = F[c][1] * ir, dz = F[c][2] * ir;
        // feq(rho, u + du) - feq(rho, u) expanded so that it carries no cancellation
        const C du15 = C(1.5) * (dx * (C(2) * ux + dx) + dy * (C(2) * uy + dy) + dz * (C(2) * uz + dz));
        C o[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const C w = C(L::w(i));
            const C eu = C(L::ex(i)) * ux + C(L::ey(i)) * uy + C(L::ez(i)) * uz;
            const C ed = C(L::ex(i)) * dx + C(L::ey(i)) * dy + C(L::ez(i)) * dz;
            const C heq = w * (m[c].drho + m[c].rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
            const C edm = w * m[c].rho * (C(3) * ed + C(4.5) * ed * (C(2) * eu + ed) - du15);
            o[i] = h[c][i] + omega * (heq - h[c][i]) + edm;
        }
        // component momentum after relaxation towards rho_c u' plus the EDM kick F_c
        conserve<L, C>(o, m[c].drho, m[c].jx + omega * (m[c].rho * ux - m[c].jx) + F[c][0],
                       m[c].jy + omega * (m[c].rho * uy - m[c].jy) + F[c][1],
                       m[c].jz + omega * (m[c].rho * uz - m[c].jz) + F[c][2]);
        bad = bad || nonfinite<C>(o[0]);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int slot, dx, dy, dz;
            post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
            // buffer-descriptor stores: 146 -> 111 VGPRs in the AA odd step (3 -> 4 waves/SIMD,
            // +3.5% on the AA run at 384^3), AB unchanged
            pop_store_at<L, LAYOUT, true>(dst, S, c * Q + slot, g, dx, dy, dz, St::encode(o[i], C(L::w(i)), 0u), i);
        }
    }
    return bad;
}

// The two-kernel step, after k_psi: one thread per node, psi read from the pre-pass array.
template <class L, class St, int LAYOUT>
__global__ __launch_bounds__(512) void k_step_sc(StepParams p) {
    using C = typename St::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;  // one row (segment) per workgroup
    const int z = blockIdx.z;
    if (x >= p.nx || y >= p.ny) return;
    const Geo g = make_geo(x, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const C *__restrict__ psi = static_cast<const C *>(p.psi);
    const uint32_t N = p.N;
    const bool bad = sc_node<L, St, LAYOUT>(p, g, [&](int c, int dx, int dy, int dz) {
        return psi[size_t(c) * N + g.at(dx, dy, dz)];
    });
    raise_divergence(p, bad);
}

}  // namespace lbm
