// Per-node collision operators of the fused step, in shifted space h_i = f_i - w_i.
//
//   BGK : h* = h + omega (heq - h) + (1 - omega/2) w_i [3(e_i - v) + 9 (e_i.v) e_i].F
//         (LBGK with the relaxation sign of the paper's GPU step algorithm, polynomial
//         equilibrium of section 2, Guo forcing of the body-forces subsection,
//         v = (j + F/2)/rho, F = rho g)
//   MRT : m* = m - S (m - m_eq) + (I - S/2) M F~ in the orthogonal moment basis of
//         d'Humieres et al. (2002), cited by the MRT subsection; transforms written with
//         pair sums/differences, equilibrium and source moments in closed form
//   ELBM: h* = h + alpha beta (heq - h), beta = 1/(2 tau), heq the discrete entropic
//         equilibrium, alpha the nontrivial root of H(f + alpha (feq - f)) = H(f)
//         (entropic LBM subsection), solved in FP64
//   SC  : two components, force -G psi_c(x) sum_i w_i psi_other(x+e_i) e_i (Shan-Chen
//         subsection), common velocity, exact-difference-method forcing
//   REG : regularized LBGK, SMAG: Smagorinsky LBGK (their subsections; below)
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "lattice.hpp"
#include "params.hpp"

namespace lbm {

template <class C>
struct Macro {
    C drho, rho, jx, jy, jz;
};

// 1/x in the compute type: FP64 divides; FP32 takes the hardware reciprocal (1 ulp)
// refined by one Newton step (within an ulp of the quotient), about a third of the
// instructions of the correctly rounded division.
template <class C>
__device__ __forceinline__ C inv(C x) {
    if constexpr (sizeof(C) == 8) {
        return C(1) / x;
    } else {
        const float r = __builtin_amdgcn_rcpf(x);
        return fmaf(fmaf(-x, r, 1.0f), r, r);
    }
}

// Step parameters in the compute type (the FP32 copies spare a conversion per wave).
template <class C>
__device__ __forceinline__ C body_g(const StepParams &p, int a) {
    if constexpr (sizeof(C) == 8) return p.g[a];
    else return p.g_f[a];
}
template <class C>
__device__ __forceinline__ C mrt_coef(const StepParams &p, int j, int k) {
    if constexpr (sizeof(C) == 8) return p.mrt[j][k];
    else return p.mrt_f[j][k];
}

template <class L, class C>
__device__ __forceinline__ Macro<C> moments(const C *h) {
    Macro<C> m;
    C r = h[0], jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        r += h[i];
        if (L::ex(i) == 1) jx += h[i];
        if (L::ex(i) == -1) jx -= h[i];
        if (L::ey(i) == 1) jy += h[i];
        if (L::ey(i) == -1) jy -= h[i];
        if (L::ez(i) == 1) jz += h[i];
        if (L::ez(i) == -1) jz -= h[i];
    }
    m.drho = r;
    m.rho = C(1) + r;
    m.jx = jx;
    m.jy = jy;
    m.jz = jz;
    return m;
}

// Restore the conserved moments of the post-collision populations.  Mass and momentum
// are conserved exactly by every collision here, but the weights are not exact binary
// numbers (in FP32, 3 sum_i w_i e_ix^2 = 1 + 3e-8), so the equilibrium's momentum
// carries a relative bias of a few 1e-8 per step that compounds into a systematic
// growth of the velocity amplitude (2.5e-5 after 1000 steps on the 256^3 vortex).
// Setting the difference of each axis pair to give the target momentum, keeping the
// pair's sum, and then the rest population to give the target mass, leaves only
// unbiased rounding.  In exact arithmetic this is the identity.
template <class L, class C>
__device__ __forceinline__ void conserve(C *o, C drho, C jx, C jy, C jz) {
    // momentum carried by every population except the axis pair of that component
    C ox = C(0), oy = C(0), oz = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        if (i != 1 && i != 2) {
            if (L::ex(i) == 1) ox += o[i];
            if (L::ex(i) == -1) ox -= o[i];
        }
        if (i != 3 && i != 4) {
            if (L::ey(i) == 1) oy += o[i];
            if (L::ey(i) == -1) oy -= o[i];
        }
        if (i != 5 && i != 6) {
            if (L::ez(i) == 1) oz += o[i];
            if (L::ez(i) == -1) oz -= o[i];
        }
    }
    C sp, dp;
    sp = o[1] + o[2];
    dp = jx - ox;
    o[1] = C(0.5) * (sp + dp);
    o[2] = C(0.5) * (sp - dp);
    sp = o[3] + o[4];
    dp = jy - oy;
    o[3] = C(0.5) * (sp + dp);
    o[4] = C(0.5) * (sp - dp);
    if constexpr (L::D == 3) {
        sp = o[5] + o[6];
        dp = jz - oz;
        o[5] = C(0.5) * (sp + dp);
        o[6] = C(0.5) * (sp - dp);
    }
    C ms = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; i++) ms += o[i];
    o[0] = drho - ms;
}

// ---------------------------------------------------------------------------- BGK
// FORCE is the wave-uniform has_force flag made a template argument, so a step without
// a body force carries no forcing arithmetic (the compiler would otherwise evaluate the
// forcing term and select it away).
template <class L, class C, bool FORCE>
__device__ __forceinline__ void collide_bgk_body(const C *h, C *o, const StepParams &p) {
    const Macro<C> m = moments<L, C>(h);
    const C omega = C(p.omega);
    const C irho = inv<C>(m.rho);
    C vx = m.jx * irho, vy = m.jy * irho, vz = m.jz * irho;
    C Fx = C(0), Fy = C(0), Fz = C(0);
    if constexpr (FORCE) {
        const C gx = body_g<C>(p, 0), gy = body_g<C>(p, 1), gz = L::D == 3 ? body_g<C>(p, 2) : C(0);
        vx += C(0.5) * gx;
        vy += C(0.5) * gy;
        vz += C(0.5) * gz;
        Fx = m.rho * gx;
        Fy = m.rho * gy;
        Fz = m.rho * gz;
    }
    const C usq15 = C(1.5) * (vx * vx + vy * vy + vz * vz);
    [[maybe_unused]] const C pre = C(1) - C(0.5) * omega;
    [[maybe_unused]] const C vF = vx * Fx + vy * Fy + vz * Fz;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const C w = C(L::w(i));
        const C eu = C(L::ex(i)) * vx + C(L::ey(i)) * vy + C(L::ez(i)) * vz;
        const C heq = w * (m.drho + m.rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
        C r = h[i] + omega * (heq - h[i]);
        if constexpr (FORCE) {
            const C eF = C(L::ex(i)) * Fx + C(L::ey(i)) * Fy + C(L::ez(i)) * Fz;
            r += pre * w * (C(3) * (eF - vF) + C(9) * eu * eF);
        }
        o[i] = r;
    }
    if constexpr (FORCE) conserve<L, C>(o, m.drho, m.jx + Fx, m.jy + Fy, m.jz + Fz);
    else conserve<L, C>(o, m.drho, m.jx, m.jy, m.jz);
}

template <class L, class C>
__device__ __forceinline__ void collide_bgk(const C *h, C *o, const StepParams &p) {
    if (p.has_force) collide_bgk_body<L, C, true>(h, o, p);
    else collide_bgk_body<L, C, false>(h, o, p);
}

// ------------------------------------------------------------ regularized and Smagorinsky
// Sums over the populations of the non-equilibrium part fn_i = h_i - heq_i: s0 = sum fn,
// and the second moments sum fn e_a e_b.  With e_a in {-1, 0, 1}, e_a^2 is 1 or 0 and
// e_a e_b is +-1 or 0, so every term is an add or a subtract.
template <class C>
struct NeqMoments {
    C s0, xx, yy, zz, xy, xz, yz;
};

template <class L, class C>
__device__ __forceinline__ void neq_moments_add(NeqMoments<C> &q, int i, C fn) {
    q.s0 += fn;
    if (L::ex(i) != 0) q.xx += fn;
    if (L::ey(i) != 0) q.yy += fn;
    if (L::ez(i) != 0) q.zz += fn;
    if (L::ex(i) * L::ey(i) == 1) q.xy += fn;
    if (L::ex(i) * L::ey(i) == -1) q.xy -= fn;
    if (L::ex(i) * L::ez(i) == 1) q.xz += fn;
    if (L::ex(i) * L::ez(i) == -1) q.xz -= fn;
    if (L::ey(i) * L::ez(i) == 1) q.yz += fn;
    if (L::ey(i) * L::ez(i) == -1) q.yz -= fn;
}

// The regularized collision fuses multiply-adds only where a source expression writes one
// (contract(on)), never across statements.  The step is compiled in several forms
// (layouts, the x staging), and across-statement fusing of this collision's products
// (the shared 1/3 t of the stress deviator) depended on the code around it: one form of
// the regularized BF16 step rounded one population to the neighbouring BF16 value, which
// broke the bit-for-bit equality of the layouts.  The default is restored after it.
#pragma clang fp contract(on)

// Regularized LBGK (regularized LBM subsection): the non-equilibrium part is replaced by
// w_i / (2 cs^4) (e_ia e_ib - cs^2 d_ab) Pi_ab, Pi_ab = sum_i fn_i (e_ia e_ib - cs^2 d_ab),
// then relaxed as in LBGK: h* = heq + (1 - omega) h_reg.  No body force (the API rejects
// one for this model).  Mass and momentum of h_reg vanish in exact arithmetic; conserve()
// removes the rounding, as for LBGK.
template <class L, class C>
__device__ __forceinline__ void collide_reg(const C *h, C *o, const StepParams &p) {
    const Macro<C> m = moments<L, C>(h);
    const C irho = inv<C>(m.rho);
    const C vx = m.jx * irho, vy = m.jy * irho, vz = m.jz * irho;
    const C usq15 = C(1.5) * (vx * vx + vy * vy + vz * vz);
    C heq[L::Q];
    NeqMoments<C> q{C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const C eu = C(L::ex(i)) * vx + C(L::ey(i)) * vy + C(L::ez(i)) * vz;
        heq[i] = C(L::w(i)) * (m.drho + m.rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
        neq_moments_add<L, C>(q, i, h[i] - heq[i]);
    }
    const C t = q.s0 * C(1.0 / 3.0);
    const C Pxx = q.xx - t, Pyy = q.yy - t, Pzz = L::D == 3 ? q.zz - t : C(0);
    const C tr3 = (Pxx + Pyy + Pzz) * C(1.0 / 3.0);
    const C k = (C(1) - C(p.omega)) * C(4.5);  // (1 - omega) / (2 cs^4)
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        C s = -tr3;
        if (L::ex(i) != 0) s += Pxx;
        if (L::ey(i) != 0) s += Pyy;
        if (L::ez(i) != 0) s += Pzz;
        if (L::ex(i) * L::ey(i) != 0) s += C(2 * L::ex(i) * L::ey(i)) * q.xy;
        if (L::ex(i) * L::ez(i) != 0) s += C(2 * L::ex(i) * L::ez(i)) * q.xz;
        if (L::ey(i) * L::ez(i) != 0) s += C(2 * L::ey(i) * L::ez(i)) * q.yz;
        o[i] = heq[i] + k * C(L::w(i)) * s;
    }
    conserve<L, C>(o, m.drho, m.jx, m.jy, m.jz);
}

#pragma clang fp contract(fast)

// Smagorinsky LBGK (Smagorinsky subgrid subsection): Q_ab = sum_i e_ia e_ib fn_i and the
// local relaxation time tau = tau0 + tau_t, tau_t = (sqrt(tau0^2 + 4 cs^-4 C_S^2 |Q|) -
// tau0) / 2, |Q| = (Q_ab Q_ab)^(1/2); evaluated as (tau0 + sqrt(tau0^2 + k |Q|)) / 2,
// which avoids the cancellation of the difference.  Then the LBGK step with its Guo
// source at that tau.
template <class L, class C, bool FORCE>
__device__ __forceinline__ void collide_smag_body(const C *h, C *o, const StepParams &p) {
    const Macro<C> m = moments<L, C>(h);
    const C irho = inv<C>(m.rho);
    C vx = m.jx * irho, vy = m.jy * irho, vz = m.jz * irho;
    C Fx = C(0), Fy = C(0), Fz = C(0);
    if constexpr (FORCE) {
        const C gx = body_g<C>(p, 0), gy = body_g<C>(p, 1), gz = L::D == 3 ? body_g<C>(p, 2) : C(0);
        vx += C(0.5) * gx;
        vy += C(0.5) * gy;
        vz += C(0.5) * gz;
        Fx = m.rho * gx;
        Fy = m.rho * gy;
        Fz = m.rho * gz;
    }
    const C usq15 = C(1.5) * (vx * vx + vy * vy + vz * vz);
    C heq[L::Q];
    NeqMoments<C> q{C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const C eu = C(L::ex(i)) * vx + C(L::ey(i)) * vy + C(L::ez(i)) * vz;
        heq[i] = C(L::w(i)) * (m.drho + m.rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
        neq_moments_add<L, C>(q, i, h[i] - heq[i]);
    }
    C QQ = q.xx * q.xx + q.yy * q.yy + C(2) * q.xy * q.xy;
    if constexpr (L::D == 3) QQ += q.zz * q.zz + C(2) * (q.xz * q.xz + q.yz * q.yz);
    const C tau0 = C(p.tau0);
    const C tau = C(0.5) * (tau0 + sqrt(tau0 * tau0 + C(p.smag_k) * sqrt(QQ)));
    const C omega = C(1) / tau;
    [[maybe_unused]] const C pre = C(1) - C(0.5) * omega;
    [[maybe_unused]] const C vF = vx * Fx + vy * Fy + vz * Fz;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        C r = h[i] + omega * (heq[i] - h[i]);
        if constexpr (FORCE) {
            const C eu = C(L::ex(i)) * vx + C(L::ey(i)) * vy + C(L::ez(i)) * vz;
            const C eF = C(L::ex(i)) * Fx + C(L::ey(i)) * Fy + C(L::ez(i)) * Fz;
            r += pre * C(L::w(i)) * (C(3) * (eF - vF) + C(9) * eu * eF);
        }
        o[i] = r;
    }
    if constexpr (FORCE) conserve<L, C>(o, m.drho, m.jx + Fx, m.jy + Fy, m.jz + Fz);
    else conserve<L, C>(o, m.drho, m.jx, m.jy, m.jz);
}

template <class L, class C>
__device__ __forceinline__ void collide_smag(const C *h, C *o, const StepParams &p) {
    if (p.has_force) collide_smag_body<L, C, true>(h, o, p);
    else collide_smag_body<L, C, false>(h, o, p);
}

// ---------------------------------------------------------------------------- MRT
// D3Q19 basis rows (q = |e|^2): 1, 19q-30, (21q^2-53q+24)/2, ex, (5q-9)ex, ey,
// (5q-9)ey, ez, (5q-9)ez, 3ex^2-q, (3q-5)(3ex^2-q), ey^2-ez^2, (3q-5)(ey^2-ez^2),
// exey, eyez, exez, (ey^2-ez^2)ex, (ez^2-ex^2)ey, (ex^2-ey^2)ez; squared norms
// 19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8.
template <class C, bool FORCE>
__device__ __forceinline__ void collide_mrt_d3q19(const C *h, C *o, const StepParams &p) {
    // pair sums and differences (opposite directions are adjacent)
    const C s1 = h[1] + h[2], d1 = h[1] - h[2];
    const C s3 = h[3] + h[4], d3 = h[3] - h[4];
    const C s5 = h[5] + h[6], d5 = h[5] - h[6];
    const C s7 = h[7] + h[8], d7 = h[7] - h[8];
    const C s9 = h[9] + h[10], d9 = h[9] - h[10];
    const C s11 = h[11] + h[12], d11 = h[11] - h[12];
    const C s13 = h[13] + h[14], d13 = h[13] - h[14];
    const C s15 = h[15] + h[16], d15 = h[15] - h[16];
    const C s17 = h[17] + h[18], d17 = h[17] - h[18];
    const C Sa = s1 + s3 + s5;
    const C Sxy = s7 + s9, Sxz = s11 + s13, Syz = s15 + s17;
    const C Sd = Sxy + Sxz + Syz;

    const C drho = h[0] + Sa + Sd;
    const C jx = d1 + d7 + d9 + d11 + d13;
    const C jy = d3 + d7 - d9 + d15 + d17;
    const C jz = d5 + d11 - d13 + d15 - d17;
    C m[19];
    m[1] = C(-30) * h[0] - C(11) * Sa + C(8) * Sd;
    m[2] = C(12) * h[0] - C(4) * Sa + Sd;
    m[4] = C(-4) * d1 + d7 + d9 + d11 + d13;
    m[6] = C(-4) * d3 + d7 - d9 + d15 + d17;
    m[8] = C(-4) * d5 + d11 - d13 + d15 - d17;
    m[9] = C(2) * s1 - s3 - s5 + Sxy + Sxz - C(2) * Syz;
    m[10] = C(-4) * s1 + C(2) * (s3 + s5) + Sxy + Sxz - C(2) * Syz;
    m[11] = s3 - s5 + Sxy - Sxz;
    m[12] = C(-2) * s3 + C(2) * s5 + Sxy - Sxz;
    m[13] = s7 - s9;
    m[14] = s15 - s17;
    m[15] = s11 - s13;
    m[16] = d7 + d9 - d11 - d13;
    m[17] = -d7 + d9 + d15 + d17;
    m[18] = d11 - d13 - d15 + d17;

    const C rho = C(1) + drho;
    const C irho = inv<C>(rho);
    C vx = jx * irho, vy = jy * irho, vz = jz * irho;
    C Fx = C(0), Fy = C(0), Fz = C(0);
    if constexpr (FORCE) {
        const C gx = body_g<C>(p, 0), gy = body_g<C>(p, 1), gz = body_g<C>(p, 2);
        vx += C(0.5) * gx;
        vy += C(0.5) * gy;
        vz += C(0.5) * gz;
        Fx = rho * gx;
        Fy = rho * gy;
        Fz = rho * gz;
    }
    const C vsq = vx * vx + vy * vy + vz * vz;
    // equilibrium moments of the polynomial equilibrium at (rho, v), shifted space
    C meq[19], mf[19];
    meq[1] = C(-11) * drho + C(19) * rho * vsq;
    meq[2] = C(3) * drho - C(5.5) * rho * vsq;
    meq[4] = C(-2.0 / 3.0) * rho * vx;
    meq[6] = C(-2.0 / 3.0) * rho * vy;
    meq[8] = C(-2.0 / 3.0) * rho * vz;
    meq[9] = rho * (C(2) * vx * vx - vy * vy - vz * vz);
    meq[10] = C(-0.5) * meq[9];
    meq[11] = rho * (vy * vy - vz * vz);
    meq[12] = C(-0.5) * meq[11];
    meq[13] = rho * vx * vy;
    meq[14] = rho * vy * vz;
    meq[15] = rho * vx * vz;
    meq[16] = meq[17] = meq[18] = C(0);
    // moments of the Guo source: the derivative of m_eq along F
    const C vF = vx * Fx + vy * Fy + vz * Fz;
    mf[1] = C(38) * vF;
    mf[2] = C(-11) * vF;
    mf[4] = C(-2.0 / 3.0) * Fx;
    mf[6] = C(-2.0 / 3.0) * Fy;
    mf[8] = C(-2.0 / 3.0) * Fz;
    mf[9] = C(2) * (C(2) * vx * Fx - vy * Fy - vz * Fz);
    mf[10] = C(-0.5) * mf[9];
    mf[11] = C(2) * (vy * Fy - vz * Fz);
    mf[12] = C(-0.5) * mf[11];
    mf[13] = vx * Fy + vy * Fx;
    mf[14] = vy * Fz + vz * Fy;
    mf[15] = vx * Fz + vz * Fx;
    mf[16] = mf[17] = mf[18] = C(0);

    // relax, each row scaled by 1/|M_k|^2 for the inverse transform (coefficients from the
    // host); conserved rows: rho unchanged, j gains F whatever their rate
    C a[19];
    a[0] = drho * mrt_coef<C>(p, 0, 0);
    // momentum after the force's full step (no add of a zero force: -0 + 0 is +0)
    const C Jx = FORCE ? jx + Fx : jx, Jy = FORCE ? jy + Fy : jy, Jz = FORCE ? jz + Fz : jz;
    a[3] = Jx * mrt_coef<C>(p, 0, 3);
    a[5] = Jy * mrt_coef<C>(p, 0, 5);
    a[7] = Jz * mrt_coef<C>(p, 0, 7);
#pragma unroll
    for (int k = 1; k < 19; k++) {
        if (k == 3 || k == 5 || k == 7) continue;
        C r = mrt_coef<C>(p, 0, k) * m[k];
        if (k < 16) {  // rows 16-18 have no equilibrium or source part
            r += mrt_coef<C>(p, 1, k) * meq[k];
            if constexpr (FORCE) r += mrt_coef<C>(p, 2, k) * mf[k];
        }
        a[k] = r;
    }
    // inverse transform M^T a, even/odd parts per opposite pair
    o[0] = a[0] - C(30) * a[1] + C(12) * a[2];
    const C Eax = a[0] - C(11) * a[1] - C(4) * a[2];
    const C Edg = a[0] + C(8) * a[1] + a[2];
    C E, O;
    E = Eax + C(2) * a[9] - C(4) * a[10];
    O = a[3] - C(4) * a[4];
    o[1] = E + O; o[2] = E - O;
    E = Eax - a[9] + C(2) * a[10] + a[11] - C(2) * a[12];
    O = a[5] - C(4) * a[6];
    o[3] = E + O; o[4] = E - O;
    E = Eax - a[9] + C(2) * a[10] - a[11] + C(2) * a[12];
    O = a[7] - C(4) * a[8];
    o[5] = E + O; o[6] = E - O;
    const C Exy = Edg + a[9] + a[10] + a[11] + a[12];
    const C Exz = Edg + a[9] + a[10] - a[11] - a[12];
    const C Eyz = Edg - C(2) * a[9] - C(2) * a[10];
    const C ox = a[3] + a[4], oy = a[5] + a[6], oz = a[7] + a[8];
    E = Exy + a[13]; O = ox + oy + a[16] - a[17];
    o[7] = E + O; o[8] = E - O;
    E = Exy - a[13]; O = ox - oy + a[16] + a[17];
    o[9] = E + O; o[10] = E - O;
    E = Exz + a[15]; O = ox + oz - a[16] + a[18];
    o[11] = E + O; o[12] = E - O;
    E = Exz - a[15]; O = ox - oz - a[16] - a[18];
    o[13] = E + O; o[14] = E - O;
    E = Eyz + a[14]; O = oy + oz + a[17] - a[18];
    o[15] = E + O; o[16] = E - O;
    E = Eyz - a[14]; O = oy - oz + a[17] + a[18];
    o[17] = E + O; o[18] = E - O;
    conserve<D3Q19, C>(o, drho, Jx, Jy, Jz);
}

// D2Q9 basis rows: 1, 3q-4, (9q^2-21q+8)/2, ex, (3q-5)ex, ey, (3q-5)ey, ex^2-ey^2, exey;
// squared norms 9, 36, 36, 6, 12, 6, 12, 4, 4.
template <class C, bool FORCE>
__device__ __forceinline__ void collide_mrt_d2q9(const C *h, C *o, const StepParams &p) {
    const C s1 = h[1] + h[2], d1 = h[1] - h[2];
    const C s3 = h[3] + h[4], d3 = h[3] - h[4];
    const C s5 = h[5] + h[6], d5 = h[5] - h[6];
    const C s7 = h[7] + h[8], d7 = h[7] - h[8];
    const C Sa = s1 + s3, Sd = s5 + s7;
    const C drho = h[0] + Sa + Sd;
    const C jx = d1 + d5 - d7;
    const C jy = d3 + d5 + d7;
    C m[9];
    m[1] = C(-4) * h[0] - Sa + C(2) * Sd;
    m[2] = C(4) * h[0] - C(2) * Sa + Sd;
    m[4] = C(-2) * d1 + d5 - d7;
    m[6] = C(-2) * d3 + d5 + d7;
    m[7] = s1 - s3;
    m[8] = s5 - s7;
    const C rho = C(1) + drho;
    const C irho = inv<C>(rho);
    C vx = jx * irho, vy = jy * irho, Fx = C(0), Fy = C(0);
    if constexpr (FORCE) {
        const C gx = body_g<C>(p, 0), gy = body_g<C>(p, 1);
        vx += C(0.5) * gx;
        vy += C(0.5) * gy;
        Fx = rho * gx;
        Fy = rho * gy;
    }
    const C vsq = vx * vx + vy * vy, vF = vx * Fx + vy * Fy;
    C meq[9], mf[9];
    meq[1] = C(-2) * drho + C(3) * rho * vsq;
    meq[2] = drho - C(3) * rho * vsq;
    meq[4] = -rho * vx;
    meq[6] = -rho * vy;
    meq[7] = rho * (vx * vx - vy * vy);
    meq[8] = rho * vx * vy;
    mf[1] = C(6) * vF;
    mf[2] = C(-6) * vF;
    mf[4] = -Fx;
    mf[6] = -Fy;
    mf[7] = C(2) * (vx * Fx - vy * Fy);
    mf[8] = vx * Fy + vy * Fx;
    C a[9];
    a[0] = drho * mrt_coef<C>(p, 0, 0);
    const C Jx = FORCE ? jx + Fx : jx, Jy = FORCE ? jy + Fy : jy;
    a[3] = Jx * mrt_coef<C>(p, 0, 3);
    a[5] = Jy * mrt_coef<C>(p, 0, 5);
#pragma unroll
    for (int k = 1; k < 9; k++) {
        if (k == 3 || k == 5) continue;
        C r = mrt_coef<C>(p, 0, k) * m[k] + mrt_coef<C>(p, 1, k) * meq[k];
        if constexpr (FORCE) r += mrt_coef<C>(p, 2, k) * mf[k];
        a[k] = r;
    }
    o[0] = a[0] - C(4) * a[1] + C(4) * a[2];
    const C Eax = a[0] - a[1] - C(2) * a[2], Edg = a[0] + C(2) * a[1] + a[2];
    C E, O;
    E = Eax + a[7]; O = a[3] - C(2) * a[4];
    o[1] = E + O; o[2] = E - O;
    E = Eax - a[7]; O = a[5] - C(2) * a[6];
    o[3] = E + O; o[4] = E - O;
    E = Edg + a[8]; O = a[3] + a[4] + a[5] + a[6];
    o[5] = E + O; o[6] = E - O;
    E = Edg - a[8]; O = -a[3] - a[4] + a[5] + a[6];
    o[7] = E + O; o[8] = E - O;
    conserve<D2Q9, C>(o, drho, Jx, Jy, C(0));
}

template <class L, class C>
__device__ __forceinline__ void collide_mrt(const C *h, C *o, const StepParams &p) {
    if constexpr (L::Q == 19) {
        if (p.has_force) collide_mrt_d3q19<C, true>(h, o, p);
        else collide_mrt_d3q19<C, false>(h, o, p);
    } else {
        if (p.has_force) collide_mrt_d2q9<C, true>(h, o, p);
        else collide_mrt_d2q9<C, false>(h, o, p);
    }
}

}  // namespace lbm
