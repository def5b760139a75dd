// The two-component Shan-Chen kernels (multicomponent-models subsection): the
// pseudopotential pre-pass and the step of both components.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "step.hpp"

namespace lbm {

// The populations of both components that stream into node x at this step, raw as
// stored.  With XSTAGE (AB and AA odd steps, one whole x row per workgroup) the x-moving
// ones are loaded on aligned segments of the lane's own x into LDS (xin: the row's values,
// 2 x xmove_count x nx) and, after a barrier, taken from x - e_x, periodic within the row:
// the shift along x of the paper's step algorithm, in LDS.
template <class L, class St, int LAYOUT, bool XSTAGE>
__device__ __forceinline__ void sc_pull(const StepParams &p, const Geo &g, int x, typename St::T (&raw)[2][L::Q],
                                        typename St::T *xin) {
    using T = typename St::T;
    constexpr int Q = L::Q, NXM = xmove_count<L>();
    const T *src = static_cast<const T *>(p.src);
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int slot, dx, dy, dz;
            canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
            if (!XSTAGE || L::ex(i) == 0)
                raw[c][i] = LBM_LOAD(pop_addr(src, p.S, c * Q + slot, g, dx, dy, dz), i);
            else
                xin[(c * NXM + xmove_index<L>(i)) * p.nx + x] =
                    __builtin_nontemporal_load(pop_addr(src, p.S, c * Q + slot, g, 0, dy, dz));
        }
    }
    if constexpr (XSTAGE) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; c++) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if (L::ex(i) == 0) continue;
                const int xs = x - L::ex(i);
                raw[c][i] = xin[(c * NXM + xmove_index<L>(i)) * p.nx + (xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs))];
            }
        }
    }
}

// psi_c(x) of one component from its pulled populations (the pseudopotential of the
// multicomponent-models subsection: psi = rho, or 1 - exp(-rho)).
template <class L, class St>
__device__ __forceinline__ typename St::C psi_of(const StepParams &p, const typename St::T *raw) {
    using C = typename St::C;
    C r = C(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) r += St::decode(raw[i], C(L::w(i)));
    const C rho = C(1) + r;
    return p.psi_mode == 1 ? C(1) - exp(-rho) : rho;
}

// Shan-Chen pre-pass (the paper's macroscopic-field kernel): psi of both components at
// every node, for the step.  XSTAGE: see sc_pull (the launch holds exactly one row per
// workgroup, so every lane reaches the barrier).
template <class L, class St, int LAYOUT, bool XSTAGE = false>
__global__ __launch_bounds__(512) void k_psi(StepParams p) {
    using T = typename St::T;
    using C = typename St::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;  // one row (segment) per workgroup
    const int z = blockIdx.z;
    if (!XSTAGE && (x >= p.nx || y >= p.ny)) return;
    const Geo g = make_geo(x, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const uint32_t n = g.at(0, 0, 0);
    [[maybe_unused]] extern __shared__ unsigned char lds_x[];
    T raw[2][L::Q];
    sc_pull<L, St, LAYOUT, XSTAGE>(p, g, x, raw, reinterpret_cast<T *>(lds_x));
    C *psi = static_cast<C *>(const_cast<void *>(p.psi));
#pragma unroll
    for (int c = 0; c < 2; c++) psi[size_t(c) * p.N + n] = psi_of<L, St>(p, raw[c]);
}

// One node of the two-component Shan-Chen step: both components in one pass (they share
// the common velocity), equal relaxation times, EDM forcing.  raw: the pulled populations
// of both components; psi_at(c, dx, dy, dz) gives psi_c at the node x + (dx, dy, dz); out:
// the post-collision values as stored.  Returns whether the node's result is non-finite.
template <class L, class St, class PsiAt>
__device__ __forceinline__ bool sc_node(const StepParams &p, const typename St::T (&raw)[2][L::Q], PsiAt psi_at,
                                        typename St::T (&out)[2][L::Q]) {
    using C = typename St::C;
    constexpr int Q = L::Q;
    C h[2][Q];
    Macro<C> m[2];
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) h[c][i] = St::decode(raw[c][i], C(L::w(i)));
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
        for (int i = 0; i < Q; i++) out[c][i] = St::encode(o[i], C(L::w(i)), 0u);
    }
    return bad;
}

// The step, after k_psi: one thread per node, psi read from the pre-pass array.  Stores go
// through buffer descriptors: 146 -> 111 VGPRs in the AA odd step (3 -> 4 waves/SIMD,
// +3.5% on the AA run at 384^3), AB unchanged.  XSTAGE (AB and AA odd, one whole row per
// workgroup): the pulls as in sc_pull, and in AA odd the x-moving stores too: lane x puts
// f*_i into LDS (xout) and, after a barrier, writes position x of slot i from lane x - e_x.
template <class L, class St, int LAYOUT, bool XSTAGE = false>
__global__ __launch_bounds__(512) void k_step_sc(StepParams p) {
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q, NXM = xmove_count<L>();
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;  // one row (segment) per workgroup
    const int z = blockIdx.z;
    if (!XSTAGE && (x >= p.nx || y >= p.ny)) return;
    const Geo g = make_geo(x, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const C *__restrict__ psi = static_cast<const C *>(p.psi);
    const uint32_t N = p.N, S = p.S;
    T *dst = static_cast<T *>(p.dst);
    [[maybe_unused]] extern __shared__ unsigned char lds_x[];
    T *xin = reinterpret_cast<T *>(lds_x);
    [[maybe_unused]] T *xout = xin + 2 * NXM * p.nx;
    T raw[2][Q], out[2][Q];
    sc_pull<L, St, LAYOUT, XSTAGE>(p, g, x, raw, xin);
    const bool bad = sc_node<L, St>(p, raw, [&](int c, int dx, int dy, int dz) {
        return psi[size_t(c) * N + g.at(dx, dy, dz)];
    }, out);
    if constexpr (XSTAGE && LAYOUT == LAYOUT_AA_ODD) {
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int i = 0; i < Q; i++)
                if (L::ex(i) != 0) xout[(c * NXM + xmove_index<L>(i)) * p.nx + x] = out[c][i];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int slot, dx, dy, dz;
            post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
            if (XSTAGE && LAYOUT == LAYOUT_AA_ODD && L::ex(i) != 0) {
                const int xs = x - L::ex(i);
                const T v = xout[(c * NXM + xmove_index<L>(i)) * p.nx + (xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs))];
                pop_store_own_x<true>(dst, S, c * Q + slot, g, dy, dz, v);
            } else {
                pop_store_at<L, LAYOUT, true>(dst, S, c * Q + slot, g, dx, dy, dz, out[c][i], i);
            }
        }
    }
    raise_divergence(p, bad);
}

}  // namespace lbm
