// Entropic LBM: FP64 root of the entropy condition and the alpha MLP proposal.
//
// alpha is the nontrivial root of g(a) = H(f + a D) - H(f), D = feq - f, H = sum f ln(f/w)
// (entropic LBM subsection, alpha condition).  Because feq is the exact constrained
// minimiser and D carries no mass or momentum, sum_i D_i ln(feq_i/w_i) = 0 and
//   g(a)  = sum_i f_i [ (1 + a d_i) log1p(a d_i) - a d_i log1p(d_i) ],   d_i = D_i/f_i
//   g'(a) = sum_i f_i d_i [ log1p(a d_i) - log1p(d_i) ]
// with no cancellation between two large H values.  g is convex, g(0) = 0, g'(0) < 0
// and g(1) = H(feq) - H(f) <= 0, so the root lies in (1, a_max), a_max the largest
// step keeping every population positive.  The paper notes alpha = 2 close to
// equilibrium: nodes with max |d_i| < 1e-6 take alpha = 2 directly.  Otherwise
// Newton with bisection safeguard on the bracket [lo, hi], stopped by |d alpha| <= tol
// or by g reaching the rounding floor of its own terms (just above the short-cut,
// g' ~ sum f d^2 is tiny and rounding noise alone moves a Newton step by more than
// tol); all in FP64 with denormals kept (the paper reports flush-to-zero breaking ELBM).
//
// Power-series form.  With the moments a_k = sum_i f_i d_i^k, expanding both logarithms
// (valid for |a d_i| < 1 and |d_i| < 1) gives g as a power series in a:
//   g(a)  = a a_1 + sum_{k>=2} (-1)^k a_k [ a^k / (k (k-1)) - a / (k-1) ]
//   g'(a) =   a_1 + sum_{k>=2} (-1)^k a_k (a^(k-1) - 1) / (k-1)
// Since |a_k| <= m^(k-2) a_2 with m = max |d_i|, cutting the series after k = K leaves an
// error of about a^2 (a m)^(K-1) / (K (K+1)) relative to g' ~ a_2.  For m <= 0.1 and
// K = 16 that is below 1e-12 at the root (a ~ 2), and the root is bracketed by [1, 2.5]
// (per population, (1 + 2.5 d) log1p(2.5 d) - 2.5 d log1p(d) - 2.5 d >= 0.49 d^2 for
// |d| <= 0.1, so g(2.5) > 0).  On that bracket the Newton iteration needs only the 16
// moments, computed once, and two Horner chains per step: no logarithm per iteration.
// Nodes with m > 0.1 take the logarithmic form above.
//
// Order of the series.  The cut after k = K moves the root by about
// alpha^2 (alpha m)^(K-1) / (K (K+1)) (an upper bound, 4-5x above what random D3Q19
// states show), so (with alpha ~ 2) its effect on a population, that times m, stays below
// eps_C when 4 (2m)^(K-1) m / (K (K+1)) <= eps_C.  The common case of a resolved flow has
// m ~ 1e-3 and needs only K = 6, a third of the FP64 work of K = 16.  A wave therefore
// takes K = 6 when all its nodes have m <= m6 (m6 = 3.8e-3 for FP64 compute, with
// eps = 1e-14; 1.2e-2 for FP32 compute, with eps = 1e-11, far below FP32 rounding) and
// K = 16 otherwise.  The choice is wave-uniform (one ballot), so both orders are fully
// unrolled register code.  It is made before the FP64 pass, from the exact test
// |D_i| > m6 (w_i + h_i) in compute precision (three instructions per population).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "lattice.hpp"
#include "params.hpp"

namespace lbm {

// Discrete entropic equilibrium p_i = w_i exp(b.e_i)/Z: the minimiser of
// H = sum f ln(f/w) at fixed rho and rho u.  exp(b.e_i) is a product of per-axis
// factors, so the state is kept as E+_a = expm1(b_a), E-_a = expm1(-b_a).  Start:
// the product-form base (2u + sqrt(1+3u^2))/(1-u) per axis (entropic LBM subsection,
// with the factor 3 under the root); then Newton steps on the momentum constraint,
// Jacobian = covariance of e under p: two in FP64, one in FP32, where the seed's error
// (~1e-6 relative at |u| = 0.05) is squared by the first step to below 2e-11 of w_i
// for |u| <= 0.15, three orders under FP32 resolution, so a second step changes nothing
// FP32 can hold.  Output heq_i = rho p_i - w_i (shifted space), formed from expm1
// values so the small deviation keeps its relative accuracy.
//
// In FP32 the quotients take the hardware reciprocal (1 ulp) instead of the correctly
// rounded division sequence, and the Newton correction's expm1(+-d) its cubic Taylor
// polynomial: |d| stays below 1e-4 for |u| <= 0.15 (the seed misses the momentum by
// ~1e-5 relative), where the dropped d^4/24 is ~1e-18 of d.  The FP64 path keeps the
// divisions and expm1 of the definition.
template <class C>
__device__ __forceinline__ C eq_div(C a, C b) {
    if constexpr (sizeof(C) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}
template <class C>
__device__ __forceinline__ C eq_expm1_small(C d) {
    if constexpr (sizeof(C) == 4) return d * fmaf(d, fmaf(d, 1.0f / 6.0f, 0.5f), 1.0f);
    else return expm1(d);
}

template <class L, class C>
__device__ __forceinline__ void entropic_heq(C drho, C rho, C ux, C uy, C uz, C *heq) {
    C Ep[3], Em[3];
    const C u[3] = {ux, uy, uz};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (a >= L::D) {
            Ep[a] = Em[a] = C(0);
            continue;
        }
        const C s = sqrt(C(1) + C(3) * u[a] * u[a]);
        const C t = C(3) * u[a] + C(3) * u[a] * u[a] / (s + C(1));  // 2u + s - (1 - u)
        Ep[a] = eq_div<C>(t, C(1) - u[a]);
        Em[a] = eq_div<C>(-t, C(2) * u[a] + s);
    }
    auto em1 = [&](int i) -> C {  // expm1(b . e_i)
        C r = C(0);
        int na = 0;
        C fac[3];
        const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (e[a] == 1) fac[na++] = Ep[a];
            if (e[a] == -1) fac[na++] = Em[a];
        }
        if (na == 1) r = fac[0];
        if (na == 2) r = fac[0] + fac[1] + fac[0] * fac[1];
        return r;
    };
    constexpr int NEWTON = sizeof(C) == 8 ? 2 : 1;
    C dp[L::Q];  // p_i - w_i
    for (int it = 0; it <= NEWTON; it++) {
        C zm1 = C(0);
#pragma unroll
        for (int i = 1; i < L::Q; i++) zm1 += C(L::w(i)) * em1(i);
        const C iz = eq_div<C>(C(1), C(1) + zm1);
#pragma unroll
        for (int i = 0; i < L::Q; i++) dp[i] = C(L::w(i)) * (em1(i) - zm1) * iz;
        if (it == NEWTON) break;
        // mean and covariance of e under p
        C m[3] = {C(0), C(0), C(0)}, Cv[3][3];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) Cv[a][b] = (a == b && a < L::D) ? C(1.0 / 3.0) : C(0);
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
            const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
#pragma unroll
            for (int a = 0; a < 3; a++) {
                if (e[a]) m[a] += C(e[a]) * dp[i];
#pragma unroll
                for (int b = 0; b < 3; b++)
                    if (e[a] * e[b]) Cv[a][b] += C(e[a] * e[b]) * dp[i];
            }
        }
        C r[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            r[a] = m[a] - u[a];
#pragma unroll
            for (int b = 0; b < 3; b++) Cv[a][b] -= m[a] * m[b];
        }
        if constexpr (L::D == 2) {
            const C det = Cv[0][0] * Cv[1][1] - Cv[0][1] * Cv[1][0];
            const C idet = eq_div<C>(C(1), det);
            d[0] = (r[0] * Cv[1][1] - Cv[0][1] * r[1]) * idet;
            d[1] = (Cv[0][0] * r[1] - r[0] * Cv[1][0]) * idet;
            d[2] = C(0);
        } else {
            // inverse of the symmetric 3x3 covariance by cofactors
            const C c00 = Cv[1][1] * Cv[2][2] - Cv[1][2] * Cv[2][1];
            const C c01 = Cv[1][2] * Cv[2][0] - Cv[1][0] * Cv[2][2];
            const C c02 = Cv[1][0] * Cv[2][1] - Cv[1][1] * Cv[2][0];
            const C c11 = Cv[0][0] * Cv[2][2] - Cv[0][2] * Cv[2][0];
            const C c12 = Cv[0][1] * Cv[2][0] - Cv[0][0] * Cv[2][1];
            const C c22 = Cv[0][0] * Cv[1][1] - Cv[0][1] * Cv[1][0];
            const C idet = eq_div<C>(C(1), Cv[0][0] * c00 + Cv[0][1] * c01 + Cv[0][2] * c02);
            d[0] = (c00 * r[0] + c01 * r[1] + c02 * r[2]) * idet;
            d[1] = (c01 * r[0] + c11 * r[1] + c12 * r[2]) * idet;
            d[2] = (c02 * r[0] + c12 * r[1] + c22 * r[2]) * idet;
        }
        // b_a -= d_a  =>  E+ = E+ + (1+E+) expm1(-d), E- = E- + (1+E-) expm1(d)
#pragma unroll
        for (int a = 0; a < L::D; a++) {
            const C em = eq_expm1_small<C>(-d[a]), ep = eq_expm1_small<C>(d[a]);
            Ep[a] = Ep[a] + (C(1) + Ep[a]) * em;
            Em[a] = Em[a] + (C(1) + Em[a]) * ep;
        }
    }
#pragma unroll
    for (int i = 0; i < L::Q; i++) heq[i] = rho * dp[i] + drho * C(L::w(i));
}


struct AlphaOut {
    double alpha;
    int iters;
    int converged;
};

constexpr double ALPHA_SHORTCUT = 1e-6;
constexpr int ALPHA_K = 16;               // highest moment of the power-series form
constexpr int ALPHA_K_LO = 6;             // the order of waves whose nodes all have m <= m6
constexpr double ALPHA_SERIES_DMAX = 0.1; // largest max |d_i| handled by that form

// m6 of the compute type C (see the order of the series above)
template <class C>
__device__ __forceinline__ constexpr double alpha_m6() {
    return sizeof(C) == 8 ? 3.8e-3 : 1.2e-2;
}

// Per-node summary of the alpha problem, built from h = f - w and heq = feq - w (the
// shifted populations the collision holds in registers), so that the solve keeps no
// per-population FP64 arrays alive.  D_i = heq_i - h_i, f_i = w_i + h_i, d_i = D_i / f_i.
//
// The form of g above relies on sum_i D_i = 0 and sum_i e_i D_i = 0.  With D from an
// FP32 equilibrium those sums are ~1e-9, which near equilibrium outweighs g's own scale
// sum_i f_i d_i^2 / 2 and moves the root below 1, out of the bracket.  D is therefore
// taken with w_i (dm + 3 e_i . dj) removed, dm and dj its raw mass and momentum
// (sum w = 1, sum w e = 0, sum w e e = I/3): both sums then vanish.  For an exact D this
// is the identity, and in FP64 a change at the rounding level.
struct AlphaNode {
    double dm, jx, jy, jz;    // mass and momentum removed from D
    double dmax, amax;        // max |d_i|; largest step keeping f + a D positive
    double mneg, mpos;        // max(-d_i), max(d_i)
    double am[ALPHA_K + 1];   // am[k] = sum_i f_i d_i^k, k = 1..K (K = ALPHA_K_LO or ALPHA_K)
    bool khi;                 // the wave takes K = ALPHA_K (wave-uniform)
};

template <class L, class C>
__device__ __forceinline__ double alpha_D(const C *h, const C *heq, const AlphaNode &s, int i) {
    return (double(heq[i]) - double(h[i])) -
           L::w(i) * (s.dm + 3.0 * (L::ex(i) * s.jx + L::ey(i) * s.jy + L::ez(i) * s.jz));
}

// 1/f in FP64: the hardware reciprocal (2^-23 relative) refined by Newton steps, each of
// which doubles the correct bits: two for FP64 compute (full precision), one for FP32
// compute (2^-46, far below what FP32 populations resolve).  About half the
// instructions of a correctly rounded division.  The Newton updates of alpha take the
// two-step form: an update's last-bit rounding is corrected by the next iterate or lies
// far below the tolerance.
template <class C = double>
__device__ __forceinline__ double recip(double f) {
    double r = __builtin_amdgcn_rcp(f);
    r = fma(r, fma(-f, r, 1.0), r);
    if constexpr (sizeof(C) == 8) r = fma(r, fma(-f, r, 1.0), r);
    return r;
}

// Order of the series for this wave: K = ALPHA_K unless every node of the wave has
// |heq_i - h_i| <= m6 (w_i + h_i) for all i (wave-uniform; lanes that do not take part
// are not counted).
template <class L, class C>
__device__ __forceinline__ bool alpha_needs_khi(const C *h, const C *heq) {
    const C m6 = C(alpha_m6<C>());
    bool big = false;
#pragma unroll
    for (int i = 0; i < L::Q; i++) big |= fabs(heq[i] - h[i]) > fma(m6, h[i], C(m6 * L::w(i)));
    return __builtin_amdgcn_ballot_w64(big) != 0;
}

// log1p(x) in FP64 for x > -1, within a few ulp (host check against the C library over
// x in (-1, 20): at most 5 ulp, 0.4-0.8 ulp on average): u = 1 + x = m 2^k with m in
// [sqrt(1/2), sqrt(2)), log u = k ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.1716,
// from the odd Taylor series 2 s (1 + s^2/3 + ... + s^20/21) (the next term is below
// 2^-60 of the sum); then log1p(x) = log(u) x / (u - 1), which undoes the rounding of
// u = 1 + x to first order (the classical correction for small x).  About 40
// instructions, against 135 for the library's double-double log1p.
__device__ __forceinline__ double log1p_series(double x) {
    const double u = 1.0 + x;
    if (u == 1.0) return x;
    int k;
    double m = frexp(u, &k);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        k -= 1;
    }
    const double s = (m - 1.0) * recip(m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
#pragma unroll
    for (int j = 9; j >= 0; j--) p = fma(p, s2, 1.0 / double(2 * j + 1));
    const double lg = fma(double(k), 0.69314718055994530942, 2.0 * s * p);
    return lg * (x * recip(u - 1.0));
}

// the raw mass and momentum of heq - h (removed from D by alpha_D)
template <class L, class C>
__device__ __forceinline__ void alpha_project(const C *h, const C *heq, AlphaNode &s) {
    s.dm = s.jx = s.jy = s.jz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const double D = double(heq[i]) - double(h[i]);
        s.dm += D;
        if (L::ex(i)) s.jx += L::ex(i) * D;
        if (L::ey(i)) s.jy += L::ey(i) * D;
        if (L::ez(i)) s.jz += L::ez(i) * D;
    }
}

// The six alpha features: log10(a2/rho), a3/a2, a4/a2, max(-d), max(d), |v|^2/c_s^2,
// with a_k = sum_i f_i d_i^k.
__device__ __forceinline__ void alpha_features_m(double a2, double a3, double a4, double mneg, double mpos,
                                                 double rho, double vsq, float *x) {
    x[0] = float(log10(a2 / rho));
    x[1] = float(a3 / a2);
    x[2] = float(a4 / a2);
    x[3] = float(mneg);
    x[4] = float(mpos);
    x[5] = float(3.0 * vsq);
}

// Only what the MLP features need: a_2, a_3, a_4, max(-d), max(d) (and max |d| for the
// short-cut), after alpha_project.  Lighter than alpha_prepare, so that the network can
// run before the 16 moments exist.
template <class L, class C>
__device__ __forceinline__ double alpha_feature_pass(const C *h, const C *heq, const AlphaNode &s, double rho,
                                                     double vsq, float *x) {
    double a2 = 0.0, a3 = 0.0, a4 = 0.0, mneg = -1e300, mpos = -1e300, dmax = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const double D = alpha_D<L, C>(h, heq, s, i);
        const double d = D * recip<C>(L::w(i) + double(h[i]));
        double t = D * d;
        a2 += t;
        t *= d;
        a3 += t;
        t *= d;
        a4 += t;
        mneg = fmax(mneg, -d);
        mpos = fmax(mpos, d);
        dmax = fmax(dmax, fabs(d));
    }
    alpha_features_m(a2, a3, a4, mneg, mpos, rho, vsq, x);
    return dmax;
}

// max |d|, max(-d), max(d), a_max and the moments a_1..a_K, after alpha_project
template <class L, class C, int K>
__device__ __forceinline__ void alpha_moments_k(const C *h, const C *heq, AlphaNode &s) {
    s.dmax = 0.0;
    s.mneg = s.mpos = -1e300;
#pragma unroll
    for (int k = 0; k <= ALPHA_K; k++) s.am[k] = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const double D = alpha_D<L, C>(h, heq, s, i);
        const double d = D * recip<C>(L::w(i) + double(h[i]));
        s.dmax = fmax(s.dmax, fabs(d));
        s.mneg = fmax(s.mneg, -d);
        s.mpos = fmax(s.mpos, d);
        double t = D;  // f_i d_i
        s.am[1] += t;
#pragma unroll
        for (int k = 2; k <= K; k++) {
            t *= d;
            s.am[k] += t;
        }
    }
    // min over d_i < 0 of -1/d_i is 1 / max(-d_i)
    s.amax = s.mneg > 0.0 ? recip<double>(s.mneg) : INFINITY;
}

// the order of the wave, then its moments (after alpha_project)
template <class L, class C>
__device__ __forceinline__ void alpha_moments(const C *h, const C *heq, AlphaNode &s) {
    s.khi = alpha_needs_khi<L, C>(h, heq);
    if (s.khi) alpha_moments_k<L, C, ALPHA_K>(h, heq, s);
    else alpha_moments_k<L, C, ALPHA_K_LO>(h, heq, s);
}

template <class L, class C>
__device__ __forceinline__ void alpha_prepare(const C *h, const C *heq, AlphaNode &s) {
    alpha_project<L, C>(h, heq, s);
    alpha_moments<L, C>(h, heq, s);
}

// Newton with bisection safeguard on the logarithmic form of g, bracket [1, a_max).
// Used where max |d_i| > ALPHA_SERIES_DMAX, which is rare in resolved flows, so it is
// written for few registers: f_i and d_i go to local arrays that a rolled loop reads (the
// compiler keeps them in scratch memory, touched only when this path runs), instead of
// 19 unrolled FP64 log1p pairs that would raise the register count of the whole kernel.
template <class L, class C>
__device__ __forceinline__ AlphaOut alpha_newton_log(const C *h, const C *heq, const AlphaNode &s, double a0,
                                                     double tol, int maxit) {
    double fl[L::Q], dl[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        fl[i] = L::w(i) + double(h[i]);
        dl[i] = alpha_D<L, C>(h, heq, s, i) * recip<C>(fl[i]);
    }
    double lo = 1.0, hi = s.amax, a = a0;
    if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
    for (int k = 1; k <= maxit; k++) {
        double g = 0.0, dg = 0.0, gs = 0.0;
#pragma unroll 1
        for (int i = 0; i < L::Q; i++) {
            const double f = fl[i], d = dl[i];
            const double l1 = log1p_series(d);
            const double ad = a * d;
            const double la = log1p_series(ad);
            const double t1 = f * (1.0 + ad) * la, t2 = f * ad * l1;
            g += t1 - t2;
            dg += f * d * (la - l1);
            gs += fabs(t1) + fabs(t2);
        }
        // g at the rounding floor of its own sum: a is the root to working precision
        if (fabs(g) <= 64.0 * 2.220446049250313e-16 * gs) return {a, k, 1};
        if (g < 0.0) lo = a; else hi = a;
        double an = a - g * recip<double>(dg);
        if (fabs(an - a) <= tol) return {an, k, 1};
        if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
        a = an;
    }
    return {fmin(2.0, 0.99 * s.amax), maxit, 0};
}

// Newton with bisection safeguard on g in its power-series form of order K.  am[k] = a_k
// for k = 1..K; bracket [1, hi] with hi <= 2.5 (see above).
template <int K>
__device__ __forceinline__ AlphaOut alpha_newton_moments(const double *am, double a0, double hi, double tol,
                                                         int maxit) {
    // g(x) = x (S1(x) - B), g'(x) = S2(x) - B with S1 = sum_k c_k x^(k-1),
    // S2 = sum_k k c_k x^(k-1), c_k = (-1)^k a_k / (k (k-1)), B = sum_k (-1)^k a_k/(k-1) - a_1
    double c[K + 1], B = -am[1];
#pragma unroll
    for (int k = 2; k <= K; k++) {
        const double sk = (k & 1) ? -am[k] : am[k];
        c[k] = sk * (1.0 / double(k * (k - 1)));
        B += sk * (1.0 / double(k - 1));
    }
    double lo = 1.0, x = a0;
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 1; it <= maxit; it++) {
        double s1 = c[K], s2 = double(K) * c[K];
#pragma unroll
        for (int k = K - 1; k >= 2; k--) {
            s1 = fma(s1, x, c[k]);
            s2 = fma(s2, x, double(k) * c[k]);
        }
        s1 *= x;
        s2 *= x;
        const double g = x * (s1 - B), dg = s2 - B;
        // rounding floor of g: its two leading terms, a_2 x^2 / 2 and B x, cancel at the root
        if (fabs(g) <= 64.0 * 2.220446049250313e-16 * x * (fabs(c[2]) * x + fabs(B))) return {x, it, 1};
        if (g < 0.0) lo = x; else hi = x;
        double xn = x - g * recip<double>(dg);
        if (fabs(xn - x) <= tol) return {xn, it, 1};
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
    }
    return {2.0, maxit, 0};
}

// tanh from the identity tanh x = 1 - 2 / (e^(2x) + 1), with the hardware base-2
// exponential and reciprocal (absolute error ~2e-7; +-1 in the limits, where e^(2x)
// overflows to inf or underflows to 0).  Used for inference only; training keeps tanhf.
__device__ __forceinline__ float tanh_fast(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e)
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// The alpha proposal network, 6 -> 32 -> 32 -> 1 with tanh hidden units, evaluated for
// the 64 nodes of a wave at once on the matrix cores
// (v_mfma_f32_32x32x16_bf16: BF16 operands, FP32 accumulation).  W holds the BF16
// weights widened to FP32 (the same values) followed by the FP32 input normalisation:
// W1[32][6], b1[32], W2[32][32], b2[32], w3[32], b3, mu[6], isd[6]; the network sees
// (x - mu) * isd.  Its output is added to the series estimate of the root,
// 2 + (x1 - 2 x2)/3 = 2 + (a3 - 2 a4)/(3 a2), so it only carries the series' residual
// (which BF16 weights can represent to far better absolute accuracy than alpha - 2).
// Nodes run along N: the
// wave's lanes 0-31 and 32-63 form two blocks of 32 nodes.  With that instruction lane l
// supplies A[l%32][8(l/32) + t] and B[8(l/32) + t][l%32], t = 0..7, and gets
// D[8(r/4) + 4(l/32) + r%4][l%32] in accumulator r = 0..15.
//  - layer 1: Z1^T = [W1 | b1] [x; 1]: K = 7 used of 16, the features of the block's
//    node in lanes 0-31 (the second block's come from lane l + 32), zeros above;
//  - layer 2: Z2^T = W2 H1^T + b2: K = 32 as two chunks of 16, with the hidden index
//    permuted so that chunk c of B is accumulators 8c..8c+7 of layer 1 in the same lane
//    (no data moves between lanes); W2's columns are packed in the same order;
//  - output: each lane sums w3 tanh(z2) over its 16 rows, and the two half-sums of a node
//    (lanes l and l xor 32) are added.
// The hidden activations and the normalised inputs enter the MFMA in BF16 (2^-9 relative
// rounding); training runs in FP32 with tanhf.  MLP_LANE_WORDS words per lane, packed once when the weights change:
// [0,4) layer-1 A (8 BF16), [4,12) layer-2 A, chunks 0 and 1, [12,28) b2 and [28,44) w3
// of the lane's 16 accumulator rows.  Must be called by all 64 lanes of the wave.
typedef __bf16 mlp_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mlp_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ mlp_bf16x8 mlp_words_bf16(uint4 w) {
    return __builtin_bit_cast(mlp_bf16x8, w);
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return uint32_t(__builtin_bit_cast(uint16_t, static_cast<__bf16>(lo))) |
           (uint32_t(__builtin_bit_cast(uint16_t, static_cast<__bf16>(hi))) << 16);
}

__device__ __forceinline__ float mlp_eval_wave(const uint32_t *__restrict__ lane_w, const float *__restrict__ W,
                                               const float *xraw) {
    const int l = __lane_id();
    const uint4 *lw = reinterpret_cast<const uint4 *>(lane_w + l * MLP_LANE_WORDS);
    // this lane's normalised features with the bias input, as 8 BF16
    float xn[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) xn[k] = (xraw[k] - W[MLP_NPARAM + k]) * W[MLP_NPARAM + MLP_IN + k];
    const uint4 own = make_uint4(pack_bf16x2(xn[0], xn[1]), pack_bf16x2(xn[2], xn[3]), pack_bf16x2(xn[4], xn[5]),
                                 pack_bf16x2(1.0f, 0.0f));
    uint4 other;  // the features of lane l xor 32
    other.x = uint32_t(__shfl_xor(int(own.x), 32, 64));
    other.y = uint32_t(__shfl_xor(int(own.y), 32, 64));
    other.z = uint32_t(__shfl_xor(int(own.z), 32, 64));
    other.w = uint32_t(__shfl_xor(int(own.w), 32, 64));
    const bool lo = l < 32;
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    const mlp_bf16x8 a1 = mlp_words_bf16(lw[0]);
    const mlp_bf16x8 a2c0 = mlp_words_bf16(lw[1]), a2c1 = mlp_words_bf16(lw[2]);
    float part[2];
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        // block 0: nodes of lanes 0-31 (own features in lanes 0-31); block 1: lanes 32-63
        const uint4 bw = lo ? (blk == 0 ? own : other) : zero;
        mlp_f32x16 z1 = {};
        z1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, mlp_words_bf16(bw), z1, 0, 0, 0);
        uint4 h0, h1;  // tanh of accumulators 0-7 and 8-15 as BF16: layer 2's B chunks
        h0.x = pack_bf16x2(tanh_fast(z1[0]), tanh_fast(z1[1]));
        h0.y = pack_bf16x2(tanh_fast(z1[2]), tanh_fast(z1[3]));
        h0.z = pack_bf16x2(tanh_fast(z1[4]), tanh_fast(z1[5]));
        h0.w = pack_bf16x2(tanh_fast(z1[6]), tanh_fast(z1[7]));
        h1.x = pack_bf16x2(tanh_fast(z1[8]), tanh_fast(z1[9]));
        h1.y = pack_bf16x2(tanh_fast(z1[10]), tanh_fast(z1[11]));
        h1.z = pack_bf16x2(tanh_fast(z1[12]), tanh_fast(z1[13]));
        h1.w = pack_bf16x2(tanh_fast(z1[14]), tanh_fast(z1[15]));
        mlp_f32x16 z2;
        const float *b2 = reinterpret_cast<const float *>(lane_w + l * MLP_LANE_WORDS + 12);
#pragma unroll
        for (int r = 0; r < 16; r++) z2[r] = b2[r];
        z2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2c0, mlp_words_bf16(h0), z2, 0, 0, 0);
        z2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2c1, mlp_words_bf16(h1), z2, 0, 0, 0);
        const float *w3 = reinterpret_cast<const float *>(lane_w + l * MLP_LANE_WORDS + 28);
        float sum = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; r++) sum = fmaf(w3[r], tanh_fast(z2[r]), sum);
        part[blk] = sum + __shfl_xor(sum, 32, 64);
    }
    const float y = (lo ? part[0] : part[1]) + W[MLP_NPARAM - 1];
    return (2.0f + (xraw[1] - 2.0f * xraw[2]) * (1.0f / 3.0f)) + y;
}


// Root on the form that fits the node: the power series where max |d_i| <= 0.1, else
// the logarithms.
template <class L, class C>
__device__ __forceinline__ AlphaOut alpha_root(const C *h, const C *heq, const AlphaNode &s, double a0, double tol,
                                               int maxit) {
    if (s.dmax <= ALPHA_SERIES_DMAX) {
        if (s.khi) return alpha_newton_moments<ALPHA_K>(s.am, a0, 2.5, tol, maxit);
        return alpha_newton_moments<ALPHA_K_LO>(s.am, a0, 2.5, tol, maxit);
    }
    return alpha_newton_log<L, C>(h, heq, s, a0, tol, maxit);
}

}  // namespace lbm
