// The entropic step (entropic LBM subsection): one kernel for every first guess of the
// alpha solve, with the logarithmic form of the alpha condition shared through LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "elbm.hpp"
#include "step.hpp"

namespace lbm {

// Nodes whose alpha needs the logarithmic form (max |d_i| > ALPHA_SERIES_DMAX) are few
// but spread: at step 8000 of the 256^3 entropic vortex 9% of the nodes, so nearly every
// wave has some, and a divergent branch would run every wave through the logarithms for
// a few lanes.  Such nodes are queued in LDS instead (f_i, d_i, the first guess and a_max
// of each) and the workgroup's first two waves solve them with their lanes packed,
// log1p(d_i) included; each queued node then reads its alpha back.  A queue entry takes
// 472 bytes, 60 KB for 128 entries (two 4-wave workgroups of the step still fit a CU's
// LDS); at that step 13% of the 256-node rows hold 64-127 such nodes and none more.
// Nodes beyond the capacity solve in place.
constexpr int ALPHA_LOGQ = 128;

template <int Q>
struct AlphaLogQueue {
    double f[Q][ALPHA_LOGQ], d[Q][ALPHA_LOGQ], l1[Q][ALPHA_LOGQ];
    double a0[ALPHA_LOGQ], amax[ALPHA_LOGQ], alpha[ALPHA_LOGQ];
    int iters[ALPHA_LOGQ], conv[ALPHA_LOGQ];
    int count;
};

// Newton with bisection safeguard on the logarithmic form of g for queue entry e: the
// iteration of alpha_newton_log, with log1p(d_i) taken once per node instead of once per
// iteration.
template <int Q>
__device__ __forceinline__ void alpha_newton_log_queued(AlphaLogQueue<Q> &sq, int e, double tol, int maxit) {
#pragma unroll 1
    for (int i = 0; i < Q; i++) sq.l1[i][e] = log1p_series(sq.d[i][e]);
    double lo = 1.0, hi = sq.amax[e], a = sq.a0[e];
    if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
    for (int k = 1; k <= maxit; k++) {
        double g = 0.0, dg = 0.0, gs = 0.0;
#pragma unroll 1
        for (int i = 0; i < Q; i++) {
            const double f = sq.f[i][e], d = sq.d[i][e], l1 = sq.l1[i][e];
            const double ad = a * d;
            const double la = log1p_series(ad);
            const double t1 = f * (1.0 + ad) * la, t2 = f * ad * l1;
            g += t1 - t2;
            dg += f * d * (la - l1);
            gs += fabs(t1) + fabs(t2);
        }
        if (fabs(g) <= 64.0 * 2.220446049250313e-16 * gs) {
            sq.alpha[e] = a, sq.iters[e] = k, sq.conv[e] = 1;
            return;
        }
        if (g < 0.0) lo = a; else hi = a;
        double an = a - g * recip<double>(dg);
        if (fabs(an - a) <= tol) {
            sq.alpha[e] = an, sq.iters[e] = k, sq.conv[e] = 1;
            return;
        }
        if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
        a = an;
    }
    sq.alpha[e] = fmin(2.0, 0.99 * sq.amax[e]), sq.iters[e] = maxit, sq.conv[e] = 0;
}

// The entropic step.  One x row (segment) per workgroup; every lane of the workgroup runs
// the whole kernel (lanes past the row's end on a clamped node, storing nothing; wall
// nodes and nodes at the alpha = 2 short-cut keep their own result), because the MLP
// first guess runs on the matrix cores for the 64 nodes of a wave at once and the
// logarithmic fallback is shared through LDS.  MLP: alpha_init = 2 (the network's guess,
// skipped in waves where no lane needs a solve); otherwise alpha_init 0 (alpha0 = 2) or
// 1 (the series estimate).
template <class L, class St, int LAYOUT, bool FLAGS, bool MLP>
__global__ __launch_bounds__(512) void k_step_elbm(StepParams p) {
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    __shared__ uint32_t s_hist[NEWTON_BINS + 1];
    __shared__ AlphaLogQueue<Q> sq;
    if (tid == 0) sq.count = 0;
    if (p.stats)
        for (int k = tid; k < NEWTON_BINS + 1; k += nthr) s_hist[k] = 0u;
    __syncthreads();
    const bool active = x < p.nx;
    const Geo g = make_geo(active ? x : p.nx - 1, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const uint32_t n = g.at(0, 0, 0);
    const uint32_t S = p.S;
    const T *src = static_cast<const T *>(p.src);
    T *dst = static_cast<T *>(p.dst);
    T raw[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        int slot, dx, dy, dz;
        canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
        raw[i] = LBM_LOAD(pop_addr(src, S, slot, g, dx, dy, dz), i);
    }
    const bool wall = FLAGS && p.flags[n] == 1;
    C h[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) h[i] = St::decode(raw[i], C(L::w(i)));
    const Macro<C> m = moments<L, C>(h);
    const C irho = inv<C>(m.rho);
    const C vx = m.jx * irho, vy = m.jy * irho, vz = m.jz * irho;
    C heq[Q];
    entropic_heq<L, C>(m.drho, m.rho, vx, vy, vz, heq);
    AlphaNode an;
    alpha_project<L, C>(h, heq, an);
    double a0 = 2.0;
    if constexpr (MLP) {
        // the features first, so that the moments are not live across the network
        const double vsq = double(vx) * double(vx) + double(vy) * double(vy) + double(vz) * double(vz);
        float xf[MLP_IN];
        const double dmax = alpha_feature_pass<L, C>(h, heq, an, double(m.rho), vsq, xf);
        const bool want = active && !wall && dmax >= ALPHA_SHORTCUT;
#pragma unroll
        for (int k = 0; k < MLP_IN; k++) xf[k] = want ? xf[k] : 0.0f;
        // all lanes of the wave, and only in waves where some lane needs the solve (the
        // condition is wave-uniform: a scalar branch, EXEC unchanged)
        if (__builtin_amdgcn_ballot_w64(want) != 0) a0 = double(mlp_eval_wave(p.mlp_lane, p.mlp_wf, xf));
    }
    alpha_moments<L, C>(h, heq, an);
    const bool solve = active && !wall && an.dmax >= ALPHA_SHORTCUT;
    if constexpr (!MLP) {
        if (p.alpha_init == 1) a0 = 2.0 + (an.am[3] - 2.0 * an.am[4]) / (3.0 * an.am[2]);
    }
    AlphaOut ao{2.0, 0, 1};
    const bool logf = solve && an.dmax > ALPHA_SERIES_DMAX;
    if (solve && !logf) {
        if (an.khi) ao = alpha_newton_moments<ALPHA_K>(an.am, a0, 2.5, p.alpha_tol, p.alpha_maxit);
        else ao = alpha_newton_moments<ALPHA_K_LO>(an.am, a0, 2.5, p.alpha_tol, p.alpha_maxit);
    }
    int qslot = -1;
    if (logf) {
        qslot = atomicAdd(&sq.count, 1);
        if (qslot < ALPHA_LOGQ) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const double f = L::w(i) + double(h[i]);
                sq.f[i][qslot] = f;
                sq.d[i][qslot] = alpha_D<L, C>(h, heq, an, i) * recip<C>(f);
            }
            sq.a0[qslot] = a0;
            sq.amax[qslot] = an.amax;
        } else {
            ao = alpha_newton_log<L, C>(h, heq, an, a0, p.alpha_tol, p.alpha_maxit);
        }
    }
    __syncthreads();
    const int nq = min(sq.count, ALPHA_LOGQ);
    for (int e = tid; e < nq; e += nthr) alpha_newton_log_queued<Q>(sq, e, p.alpha_tol, p.alpha_maxit);
    __syncthreads();
    if (qslot >= 0 && qslot < ALPHA_LOGQ) ao = AlphaOut{sq.alpha[qslot], sq.iters[qslot], sq.conv[qslot]};
    T out[Q];
    bool bad = false;
    if (wall) {
#pragma unroll
        for (int i = 0; i < Q; i++) out[i] = raw[opp(i)];
    } else {
        const C ab = C(ao.alpha * p.beta);
        C o[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) o[i] = h[i] + ab * (heq[i] - h[i]);
        conserve<L, C>(o, m.drho, m.jx, m.jy, m.jz);
        bad = nonfinite<C>(o[0]);
#pragma unroll
        for (int i = 0; i < Q; i++) out[i] = St::encode(o[i], C(L::w(i)), 0u);
        if (p.stats && active) {
            atomicAdd(&s_hist[ao.iters < NEWTON_BINS ? ao.iters : NEWTON_BINS - 1], 1u);
            if (!ao.converged) atomicAdd(&s_hist[NEWTON_BINS], 1u);
        }
    }
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            int slot, dx, dy, dz;
            post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
            pop_store_at<L, LAYOUT, true>(dst, S, slot, g, dx, dy, dz, out[i], i);
        }
        raise_divergence(p, bad);
    }
    if (p.stats) {
        __syncthreads();
        for (int k = tid; k < NEWTON_BINS + 1; k += nthr)
            if (s_hist[k]) atomicAdd(&p.stats[k], (unsigned long long)s_hist[k]);
    }
}

}  // namespace lbm
