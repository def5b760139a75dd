// Auxiliary kernels: equilibrium initialisation, population plane transfer in the
// canonical (physical) layout, macroscopic output and deterministic FP64 diagnostics.
#include "dispatch.hpp"
#include "elbm.hpp"
#include "step.hpp"

namespace lbm {

namespace {

dim3 flat_grid(uint32_t N, int bs) { return dim3((N + bs - 1) / bs); }

__device__ __forceinline__ Geo geo_of(uint32_t n, int nx, int ny, int nz, uint32_t rp, uint32_t rpitch,
                                      int tyl) {
    const int x = int(n % uint32_t(nx));
    const int y = int((n / uint32_t(nx)) % uint32_t(ny));
    const int z = int(n / (uint32_t(nx) * uint32_t(ny)));
    return make_geo(x, y, z, nx, ny, nz, rp, rpitch, tyl);
}

// f_eq(rho, u)_i - w_i in FP64: the polynomial equilibrium of section 2, or the entropic one.
template <class L>
__device__ double heq_plane(int q, double rho, double ux, double uy, double uz, int entropic) {
    if (entropic) {
        double heq[L::Q];
        entropic_heq<L, double>(rho - 1.0, rho, ux, uy, uz, heq);
        double r = heq[0];
#pragma unroll
        for (int i = 1; i < L::Q; i++)
            if (i == q) r = heq[i];
        return r;
    }
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        if (i != q) continue;
        const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
        const double usq = ux * ux + uy * uy + uz * uz;
        r = L::w(i) * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
    }
    return r;
}

// Free-energy equilibrium (zero phi gradients) of population q of the f lattice (comp 0)
// or the g lattice (comp 1), as plain values: non-rest 3 t_q (p0 + rho e.u + 3/2 rho
// ((e.u)^2 - u^2/3)) resp. 3 t_q (Gamma mu + phi e.u + ...), the rest population taking
// what mass (rho resp. phi) leaves.
template <class L>
__device__ double feq_fe_plane(int comp, int q, double rho, double phi, double ux, double uy, double uz, double A,
                               double G) {
    const double mu = A * (-phi + phi * phi * phi);
    const double p0 = rho / 3.0 + A * (-0.5 * phi * phi + 0.75 * phi * phi * phi * phi);
    const double usq = ux * ux + uy * uy + uz * uz;
    double r = 0.0, sum = 0.0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const double eu = L::ex(i) * ux + L::ey(i) * uy + L::ez(i) * uz;
        const double quad = 1.5 * (eu * eu - usq / 3.0);
        const double v = comp == 0 ? 3.0 * L::w(i) * (p0 + eu * rho + quad * rho)
                                   : 3.0 * L::w(i) * (G * mu + eu * phi + quad * phi);
        sum += v;
        if (i == q) r = v;
    }
    return q == 0 ? (comp == 0 ? rho : phi) - sum : r;
}

template <class L>
__device__ __forceinline__ void canon_loc_rt(int layout, int q, const Geo &g, int &slot, uint32_t &node) {
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (i == q) canon_loc<L>(layout, i, g, slot, node);
}

template <class L, class St>
__global__ void k_init_plane(PlaneParams p) {
    using T = typename St::T;
    using C = typename St::C;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const Geo g = geo_of(n, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const double ux = p.u[n], uy = p.u[p.N + n], uz = L::D == 3 ? p.u[2 * size_t(p.N) + n] : 0.0;
    double wq = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (i == p.q) wq = L::w(i);
    double h = p.fe ? feq_fe_plane<L>(p.comp, p.q, p.rho[n], p.phi[n], ux, uy, uz, p.fe_a, p.fe_gamma) - wq
                    : heq_plane<L>(p.q, p.rho[n], ux, uy, uz, p.entropic);
    if (p.df) h += p.df[n];
    int slot;
    uint32_t nd;
    canon_loc_rt<L>(p.layout, p.q, g, slot, nd);
    double w = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (i == p.q) w = L::w(i);
    T *pop = static_cast<T *>(p.pop) + size_t(p.comp) * L::Q * p.S;
    // unshifted storages (and plain planes) round f = w + h once; shifted ones round h
    if (St::shifted && !p.plain) pop[size_t(slot) * p.S + nd] = St::encode(C(h), C(w), 0u);
    else pop[size_t(slot) * p.S + nd] = T(w + h);
}

template <class L, class St>
__global__ void k_get_plane(PlaneParams p) {
    using T = typename St::T;
    using C = typename St::C;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const Geo g = geo_of(n, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    int slot;
    uint32_t nd;
    canon_loc_rt<L>(p.layout, p.q, g, slot, nd);
    double w = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (i == p.q) w = L::w(i);
    const T *pop = static_cast<const T *>(p.pop) + size_t(p.comp) * L::Q * p.S;
    const T v = pop[size_t(slot) * p.S + nd];
    if (St::shifted && !p.plain) p.plane[n] = w + double(St::decode(v, C(w)));
    else p.plane[n] = double(v);
}

template <class L, class St>
__global__ void k_set_plane(PlaneParams p) {
    using T = typename St::T;
    using C = typename St::C;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    const Geo g = geo_of(n, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    int slot;
    uint32_t nd;
    canon_loc_rt<L>(p.layout, p.q, g, slot, nd);
    double w = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (i == p.q) w = L::w(i);
    T *pop = static_cast<T *>(p.pop) + size_t(p.comp) * L::Q * p.S;
    if (St::shifted && !p.plain) pop[size_t(slot) * p.S + nd] = St::encode(C(p.plane[n] - w), C(w), 0u);
    else pop[size_t(slot) * p.S + nd] = T(p.plane[n]);
}

// Macroscopic output.  Density per component; velocity (j + F/2)/rho for the forced
// single-component models, j/rho for ELBM, the mixture velocity for Shan-Chen; 0 on walls.
// Equilibrium velocity nodes report the density of their completed population set (the
// populations streamed from walls replaced by their opposites) and the prescribed velocity;
// half-way bounce-back nodes report the moments of their completed set.
//
// One instantiation per model kind (one component, Shan-Chen, free energy) and per presence
// of node flags, each holding only what it uses.  A single kernel for every model kept two
// components' populations, the free-energy sums and per-component arrays under runtime
// indices live at once and spilled (D3Q19: 208 B/lane with FP32 storage, 1 104 with
// shifted FP32), which made the output and the diagnostics built on it 4-5x slower.
enum { MK_ONE = 0, MK_SC = 1, MK_FE = 2 };

// The macroscopic values of node n: rho[0..NC) and v[3]; returns false where a density is
// non-finite or non-positive (phi of the free-energy model only has to be finite).
template <class L, class St, int KIND, bool FL>
__device__ __forceinline__ bool macro_node(const MacroParams &p, uint32_t n, double *rho, double *v) {
    using T = typename St::T;
    using C = typename St::C;
    constexpr int NC = KIND == MK_ONE ? 1 : 2;
    const Geo g = geo_of(n, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    double j[3] = {0.0, 0.0, 0.0}, jf[3] = {0.0, 0.0, 0.0};
    rho[0] = rho[1] = 0.0;
    const uint32_t fl = FL ? p.flags[n] : 0u;
    const bool vel = FL && KIND == MK_ONE && fl == 2u;
    const bool half = FL && KIND != MK_SC && fl == 3u;
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const T *pop = static_cast<const T *>(p.pop) + size_t(c) * L::Q * p.S;
        if (KIND == MK_FE && c == 1) {
            // the free-energy g lattice is stored plain: phi = sum_i g_i in FP64
            double gv[L::Q];
#pragma unroll
            for (int i = 0; i < L::Q; i++) {
                int slot;
                uint32_t nd;
                canon_loc<L>(p.layout, i, g, slot, nd);
                gv[i] = double(pop[size_t(slot) * p.S + nd]);
            }
            if (half) {
                double gb[L::Q];
#pragma unroll
                for (int i = 0; i < L::Q; i++) gb[i] = gv[i];
#pragma unroll
                for (int i = 0; i < L::Q; i++)
                    if (p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1) gv[i] = gb[opp(i)];
            }
            double ph = 0.0;
#pragma unroll
            for (int i = 0; i < L::Q; i++) ph += gv[i];
            rho[1] = ph;
            continue;
        }
        C h[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            int slot;
            uint32_t nd;
            canon_loc<L>(p.layout, i, g, slot, nd);
            h[i] = St::decode(pop[size_t(slot) * p.S + nd], C(L::w(i)));
        }
        if (half) {
            // half-way bounce-back node: the moments of the completed set
            C hb[L::Q];
#pragma unroll
            for (int i = 0; i < L::Q; i++) hb[i] = h[i];
#pragma unroll
            for (int i = 0; i < L::Q; i++)
                if (p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1) h[i] = hb[opp(i)];
        }
        const Macro<C> m = moments<L, C>(h);
        rho[c] = double(m.rho);
        if (vel) {
            C dr = C(0);
#pragma unroll
            for (int i = 0; i < L::Q; i++)
                dr += p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1 ? h[opp(i)] : h[i];
            rho[c] = double(C(1) + dr);
        }
        if (c == 0) {
            jf[0] = double(m.jx);
            jf[1] = double(m.jy);
            jf[2] = double(m.jz);
        }
        j[0] += double(m.jx);
        j[1] += double(m.jy);
        j[2] += double(m.jz);
    }
    v[0] = v[1] = v[2] = 0.0;
    const bool wall = fl == 1u;
    if (KIND == MK_FE) {
        // rho[1] is phi (the g lattice's zeroth moment); velocity (j + F/2)/rho of f alone
        if (!wall) {
            v[0] = (jf[0] + 0.5 * rho[0] * p.g[0]) / rho[0];
            v[1] = (jf[1] + 0.5 * rho[0] * p.g[1]) / rho[0];
            v[2] = L::D == 3 ? (jf[2] + 0.5 * rho[0] * p.g[2]) / rho[0] : 0.0;
        }
    } else if (vel) {
        for (int k = 0; k < 3; k++) v[k] = p.u_bc[k];
        if (L::D == 2) v[2] = 0.0;
    } else if (!wall) {
        if (KIND == MK_SC) {
            const double rt = rho[0] + rho[1];
            const C *psi = static_cast<const C *>(p.psi);
            double F[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const C *po = psi + size_t(1 - c) * p.N;
                double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 1; i < L::Q; i++) {
                    const double pv = L::w(i) * double(po[g.at(L::ex(i), L::ey(i), L::ez(i))]);
                    s[0] += L::ex(i) * pv;
                    s[1] += L::ey(i) * pv;
                    s[2] += L::ez(i) * pv;
                }
                const double a = -p.G * double(psi[size_t(c) * p.N + n]);
                for (int k = 0; k < 3; k++) F[k] += a * s[k] + rho[c] * p.g[k];
            }
            for (int k = 0; k < 3; k++) v[k] = (j[k] + 0.5 * F[k]) / rt;
        } else {
            const double hf = p.model == M_ELBM ? 0.0 : 0.5;
            for (int k = 0; k < 3; k++) v[k] = (j[k] + hf * rho[0] * p.g[k]) / rho[0];
        }
    }
    bool ok = (rho[0] > 0.0) && isfinite(rho[0]);
    if (KIND == MK_SC) ok = ok && (rho[1] > 0.0) && isfinite(rho[1]);
    if (KIND == MK_FE) ok = ok && isfinite(rho[1]);
    return ok;
}

template <class L, class St, int KIND, bool FL>
__global__ __launch_bounds__(256) void k_macro(MacroParams p) {
    constexpr int NC = KIND == MK_ONE ? 1 : 2;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.N) return;
    double rho[2], v[3];
    const bool ok = macro_node<L, St, KIND, FL>(p, n, rho, v);
    if (p.bad && !ok) atomicAdd(p.bad, 1u);
    if (p.fp64) {
        double *ro = static_cast<double *>(p.rho_out), *uo = static_cast<double *>(p.u_out);
#pragma unroll
        for (int c = 0; c < NC; c++) ro[size_t(c) * p.N + n] = rho[c];
        for (int k = 0; k < 3; k++) uo[size_t(k) * p.N + n] = v[k];
    } else {
        float *ro = static_cast<float *>(p.rho_out), *uo = static_cast<float *>(p.u_out);
#pragma unroll
        for (int c = 0; c < NC; c++) ro[size_t(c) * p.N + n] = float(rho[c]);
        for (int k = 0; k < 3; k++) uo[size_t(k) * p.N + n] = float(v[k]);
    }
}

constexpr int RED_BS = 256;
constexpr int RED_K = 8;  // mass0, mass1, px, py, pz, ke, bad, (unused)

// Per-block partial sums in a fixed order (grid-stride over nodes, tree in LDS).
// phi2: the second density row is the free-energy order parameter phi (no mass, may be
// negative), so momentum and the positivity check use rho alone
__global__ __launch_bounds__(RED_BS) void k_diag_partials(const double *rho, const double *u, uint32_t N, int ncomp,
                                                          int phi2, double *partials) {
    __shared__ double s[RED_K][RED_BS];
    double acc[RED_K] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t n = blockIdx.x * RED_BS + threadIdx.x; n < N; n += gridDim.x * RED_BS) {
        const double r0 = rho[n], r1 = ncomp == 2 ? rho[size_t(N) + n] : 0.0;
        const double ux = u[n], uy = u[size_t(N) + n], uz = u[2 * size_t(N) + n];
        const double rt = phi2 ? r0 : r0 + r1;
        acc[0] += r0;
        acc[1] += r1;
        acc[2] += rt * ux;
        acc[3] += rt * uy;
        acc[4] += rt * uz;
        acc[5] += ux * ux + uy * uy + uz * uz;
        bool ok = (r0 > 0.0) && isfinite(r0) && (ncomp == 1 || ((phi2 || r1 > 0.0) && isfinite(r1)));
        acc[6] += ok ? 0.0 : 1.0;
    }
    for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = RED_BS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < RED_K) partials[size_t(blockIdx.x) * RED_K + threadIdx.x] = s[threadIdx.x][0];
}

// The diagnostics without the FP64 field pass: each thread takes the macroscopic values of
// its nodes (grid-stride, nodes n = b RED_BS + t + k gridDim.x RED_BS) straight from the
// populations and adds them to its sums in the same fixed order as k_diag_partials; the
// block's tree in LDS writes one set of partial sums.  Nothing is accumulated across
// calls, so the partials need no clearing.
template <class L, class St, int KIND, bool FL>
__global__ __launch_bounds__(RED_BS) void k_diag_fused(MacroParams p, double *partials) {
    __shared__ double s[RED_K][RED_BS];
    double acc[RED_K] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t n = blockIdx.x * RED_BS + threadIdx.x; n < p.N; n += gridDim.x * RED_BS) {
        double rho[2], v[3];
        const bool ok = macro_node<L, St, KIND, FL>(p, n, rho, v);
        const double r1 = KIND == MK_ONE ? 0.0 : rho[1];
        const double rt = KIND == MK_SC ? rho[0] + r1 : rho[0];
        acc[0] += rho[0];
        acc[1] += r1;
        acc[2] += rt * v[0];
        acc[3] += rt * v[1];
        acc[4] += rt * v[2];
        acc[5] += v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        acc[6] += ok ? 0.0 : 1.0;
    }
    for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = RED_BS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < RED_K) partials[size_t(blockIdx.x) * RED_K + threadIdx.x] = s[threadIdx.x][0];
}

// The block partials summed in a fixed order: each thread takes a fixed stride of blocks,
// then a tree in LDS.  (One thread per sum walking every block was a chain of dependent
// loads: 79 us for 512 blocks.)
__global__ __launch_bounds__(RED_BS) void k_diag_final(const double *partials, int nblocks, uint32_t N,
                                                       double *out) {
    __shared__ double s[RED_K][RED_BS];
    double acc[RED_K] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += RED_BS)
        for (int k = 0; k < RED_K; k++) acc[k] += partials[size_t(b) * RED_K + k];
    for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = RED_BS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < RED_K; k++) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < RED_K) out[threadIdx.x] = threadIdx.x == 5 ? s[5][0] * (0.5 / double(N)) : s[threadIdx.x][0];
}

}  // namespace

#define LBM_AUX_LAUNCH(KERNEL, P)                                                          \
    return with_lattice(lattice, [&](auto lt) {                                            \
        using L = decltype(lt);                                                            \
        return with_storage<false>(storage, 0, [&](auto st) {                              \
            using St = decltype(st);                                                       \
            KERNEL<L, St><<<flat_grid(P.N, 256), 256, 0, c.stream>>>(P);                   \
            return hipGetLastError();                                                      \
        });                                                                                \
    })

hipError_t launch_init_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c) {
    LBM_AUX_LAUNCH(k_init_plane, p);
}
hipError_t launch_get_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c) {
    LBM_AUX_LAUNCH(k_get_plane, p);
}
hipError_t launch_set_plane(int lattice, int storage, const PlaneParams &p, const LaunchCfg &c) {
    LBM_AUX_LAUNCH(k_set_plane, p);
}
hipError_t launch_macro(int lattice, int storage, const MacroParams &p, const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<false>(storage, 0, [&](auto st) {
            using St = decltype(st);
            const dim3 grid = flat_grid(p.N, 256);
            const bool fl = p.flags != nullptr;
            if (p.model == M_SC) {
                if (fl) k_macro<L, St, MK_SC, true><<<grid, 256, 0, c.stream>>>(p);
                else k_macro<L, St, MK_SC, false><<<grid, 256, 0, c.stream>>>(p);
            } else if (p.model == M_FE) {
                if (fl) k_macro<L, St, MK_FE, true><<<grid, 256, 0, c.stream>>>(p);
                else k_macro<L, St, MK_FE, false><<<grid, 256, 0, c.stream>>>(p);
            } else {
                if (fl) k_macro<L, St, MK_ONE, true><<<grid, 256, 0, c.stream>>>(p);
                else k_macro<L, St, MK_ONE, false><<<grid, 256, 0, c.stream>>>(p);
            }
            return hipGetLastError();
        });
    });
}

hipError_t launch_diag_reduce(const double *rho, const double *u, uint32_t N, int ncomp, int phi2, double *partials,
                              int nblocks, double *out, hipStream_t s) {
    k_diag_partials<<<nblocks, RED_BS, 0, s>>>(rho, u, N, ncomp, phi2, partials);
    k_diag_final<<<1, RED_BS, 0, s>>>(partials, nblocks, N, out);
    return hipGetLastError();
}

hipError_t launch_diag_fused(int lattice, int storage, const MacroParams &p, double *partials, int nblocks,
                             double *out, hipStream_t st) {
    hipError_t e = with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<false>(storage, 0, [&](auto sto) {
            using St = decltype(sto);
            const bool fl = p.flags != nullptr;
            if (p.model == M_SC) {
                if (fl) k_diag_fused<L, St, MK_SC, true><<<nblocks, RED_BS, 0, st>>>(p, partials);
                else k_diag_fused<L, St, MK_SC, false><<<nblocks, RED_BS, 0, st>>>(p, partials);
            } else if (p.model == M_FE) {
                if (fl) k_diag_fused<L, St, MK_FE, true><<<nblocks, RED_BS, 0, st>>>(p, partials);
                else k_diag_fused<L, St, MK_FE, false><<<nblocks, RED_BS, 0, st>>>(p, partials);
            } else {
                if (fl) k_diag_fused<L, St, MK_ONE, true><<<nblocks, RED_BS, 0, st>>>(p, partials);
                else k_diag_fused<L, St, MK_ONE, false><<<nblocks, RED_BS, 0, st>>>(p, partials);
            }
            return hipGetLastError();
        });
    });
    if (e != hipSuccess) return e;
    k_diag_final<<<1, RED_BS, 0, st>>>(partials, nblocks, p.N, out);
    return hipGetLastError();
}

}  // namespace lbm
