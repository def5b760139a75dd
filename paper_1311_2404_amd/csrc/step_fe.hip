// Free-energy binary model (free energy model subsection): the order-parameter pre-pass
// and the step of both lattices (f: density, g: order parameter phi).
//
// Equilibria, for the non-rest populations (lattice weights t_i):
//   f_i = 3 t_i (p0 - kappa phi lap + rho e.u + 3/2 rho ((e.u)^2 - u^2/3))
//         + kappa t_i (4.5 (e.grad)^2 - 3 |grad|^2)
//   g_i = 3 t_i (Gamma mu + phi e.u + 3/2 phi ((e.u)^2 - u^2/3))
// with p0 = rho/3 + A(-phi^2/2 + 3 phi^4/4), mu = A(-phi + phi^3) - kappa lap; the rest
// populations take what mass leaves (f_0 = rho - sum, g_0 = phi - sum).  These weights
// meet the moment conditions the subsection states (second moment of f = the pressure
// tensor + rho u u).  grad and lap use the isotropic lattice-weight stencils on the phi
// field of the pre-pass; a wall neighbour contributes the node's own phi (neutral
// wetting).  f relaxes with tau_rho = tau_B + (phi + 1)/2 (tau_A - tau_B) and takes the
// body force by the exact difference method around u = j/rho (the difference of the
// two equilibria written out); g relaxes with tau_phi
// towards its equilibrium at the velocity (j + F/2)/rho.  Storage F64, F32 or shifted F32
// for f; g is stored plain in all of them.
#include "dispatch.hpp"
#include "step.hpp"

namespace lbm {

namespace {

// half-way bounce-back completion of a population set (missing ones from wall nodes take
// the opposite population of the node)
template <class L, class C>
__device__ __forceinline__ void fe_complete(C *v, const StepParams &p, const Geo &g) {
    C b[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) b[i] = v[i];
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1) v[i] = b[opp(i)];
}

// phi = sum_i g_i of the populations streaming into x (completed on half-way nodes); the
// g lattice is stored plain in every storage (its equilibria are O(phi, mu), not centred
// on w_i, so g - w_i would only lose digits)
// XS (AB only): 0 none; 1 rows of exactly the workgroup's width, 2 rows shorter than it.  The
// x-moving populations are loaded on aligned segments into LDS and taken from x - e_x
// there, as in the polynomial-equilibrium step; lanes past a row's end load nothing of
// their own x and leave after the barrier.
template <class L, class St, int LAYOUT, bool FLAGS, int XS = 0>
__global__ __launch_bounds__(512) void k_fe_phi(StepParams p) {
    static_assert(!XS || LAYOUT == LAYOUT_AB, "x staging: AB");
    using T = typename St::T;
    using C = typename St::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const bool active = x < p.nx && y < p.ny;
    if (!XS && !active) return;
    const Geo g = make_geo(active ? x : p.nx - 1, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    const uint32_t n = g.at(0, 0, 0);
    const T *gs = static_cast<const T *>(p.src) + size_t(L::Q) * p.S;
    [[maybe_unused]] extern __shared__ unsigned char lds_x[];
    [[maybe_unused]] T *xin = reinterpret_cast<T *>(lds_x);
    [[maybe_unused]] const int xw = XS == 2 ? int(blockDim.x) : p.nx;
    const bool hw = FLAGS && p.flags[n] == 3;
    C v[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        int slot, dx, dy, dz;
        canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
        if (!XS || L::ex(i) == 0) v[i] = C(LBM_LOAD(pop_addr(gs, p.S, slot, g, dx, dy, dz), i));
        else if (XS == 1 || active) xin[xmove_index<L>(i) * xw + x] = __builtin_nontemporal_load(pop_addr(gs, p.S, slot, g, 0, dy, dz));
    }
    if constexpr (XS != 0) {
        __syncthreads();
        const int xr = active ? x : p.nx - 1;
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            if (L::ex(i) == 0) continue;
            const int xs = xr - L::ex(i);
            v[i] = C(xin[xmove_index<L>(i) * xw + (xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs))]);
        }
        if (!active) return;
    }
    if (hw) fe_complete<L, C>(v, p, g);
    C r = C(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) r += v[i];
    static_cast<C *>(const_cast<void *>(p.psi))[n] = r;
}

// The step of both lattices.  f is computed on its deviations h = f - w (the paper's
// round-off minimising form): the f equilibria's deviations are t_i (rho - 1) + 3 t_i
// (A(...) - kappa phi lap + rho e.u + ...) + gradient terms, so no O(1) value is formed
// and a shifted storage keeps the small O(F) and O(u) parts.  g is computed and stored
// plain (k = g): its values are O(phi, mu) themselves.
// XS as for k_fe_phi.  AB steps on padded rows: lanes past the row's end run the step on the
// row's last node and store into the row's padding, which is never read, so every store
// instruction writes whole memory sectors (as the polynomial-equilibrium step does).
template <class L, class St, int LAYOUT, bool FLAGS, int XS = 0>
__global__ __launch_bounds__(512) void k_step_fe(StepParams p) {
    static_assert(!XS || LAYOUT == LAYOUT_AB, "x staging: AB");
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q, NXM = xmove_count<L>();
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const bool active = x < p.nx && y < p.ny;
    const bool pad = LAYOUT == LAYOUT_AB && x >= p.nx && x < int(p.rpitch) && y < p.ny;
    if (!XS && !active && !pad) return;
    const Geo g = make_geo(active ? x : p.nx - 1, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    Geo gs = g;  // where this lane stores in AB (its own x)
    gs.x = x;
    const uint32_t n = g.at(0, 0, 0), S = p.S;
    const T *src = static_cast<const T *>(p.src);
    T *dst = static_cast<T *>(p.dst);
    const C *__restrict__ phis = static_cast<const C *>(p.psi);
    [[maybe_unused]] extern __shared__ unsigned char lds_x[];
    [[maybe_unused]] T *xin = reinterpret_cast<T *>(lds_x);
    [[maybe_unused]] const int xw = XS == 2 ? int(blockDim.x) : p.nx;
    const uint32_t fl = FLAGS ? p.flags[n] : 0u;
    T rf[Q], rg[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        int slot, dx, dy, dz;
        canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
        if (!XS || L::ex(i) == 0) {
            rf[i] = LBM_LOAD(pop_addr(src, S, slot, g, dx, dy, dz), i);
            rg[i] = LBM_LOAD(pop_addr(src, S, Q + slot, g, dx, dy, dz), i);
        } else if (XS == 1 || active) {
            xin[xmove_index<L>(i) * xw + x] = __builtin_nontemporal_load(pop_addr(src, S, slot, g, 0, dy, dz));
            xin[(NXM + xmove_index<L>(i)) * xw + x] = __builtin_nontemporal_load(pop_addr(src, S, Q + slot, g, 0, dy, dz));
        }
    }
    if constexpr (XS != 0) {
        __syncthreads();
        const int xr = active ? x : p.nx - 1;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if (L::ex(i) == 0) continue;
            const int xs = xr - L::ex(i);
            const int xi = xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs);
            rf[i] = xin[xmove_index<L>(i) * xw + xi];
            rg[i] = xin[(NXM + xmove_index<L>(i)) * xw + xi];
        }
        if (!active && !pad) return;
    }
    T of[Q], og[Q];
    bool bad = false;
    if (fl == 1u) {
        // full-way bounce-back on both lattices
#pragma unroll
        for (int i = 0; i < Q; i++) {
            of[i] = rf[opp(i)];
            og[i] = rg[opp(i)];
        }
    } else {
        C h[Q], k[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            h[i] = St::decode(rf[i], C(L::w(i)));
            k[i] = C(rg[i]);
        }
        if (FLAGS && fl == 3u) {
            fe_complete<L, C>(h, p, g);
            fe_complete<L, C>(k, p, g);
        }
        C drho = C(0), dphi = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            drho += h[i];
            dphi += k[i];
            jx += C(L::ex(i)) * h[i];
            jy += C(L::ey(i)) * h[i];
            jz += C(L::ez(i)) * h[i];
        }
        const C rho = C(1) + drho, phi = dphi;
        // stencils on the pre-pass phi field
        const C p0x = phis[n];
        C gx = C(0), gy = C(0), gz = C(0), lap = C(0);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const uint32_t m = g.at(L::ex(i), L::ey(i), L::ez(i));
            const C pn = (FLAGS && p.flags[m] == 1) ? p0x : phis[m];
            const C tw = C(3 * L::w(i)) * pn;
            gx += C(L::ex(i)) * tw;
            gy += C(L::ey(i)) * tw;
            gz += C(L::ez(i)) * tw;
            lap += C(6 * L::w(i)) * (pn - p0x);
        }
        const C A = C(p.fe_a), kap = C(p.fe_kappa);
        const C mu = A * (-phi + phi * phi * phi) - kap * lap;
        // p0 - kappa phi lap without its rho/3 part (t_i rho - w_i = t_i (rho - 1) carries it)
        const C iso = A * (C(-0.5) * phi * phi + C(0.75) * phi * phi * phi * phi) - kap * phi * lap;
        const C g2 = gx * gx + gy * gy + gz * gz;
        const C ax = C(p.g[0]), ay = C(p.g[1]), az = C(L::D == 3 ? p.g[2] : 0.0);
        const C irho = C(1) / rho;
        const C ux = jx * irho, uy = jy * irho, uz = jz * irho;
        const C vx = ux + C(0.5) * ax, vy = uy + C(0.5) * ay, vz = uz + C(0.5) * az;
        const C usq = ux * ux + uy * uy + uz * uz;
        const C vsq = vx * vx + vy * vy + vz * vz;
        const C a2 = ax * (C(2) * ux + ax) + ay * (C(2) * uy + ay) + az * (C(2) * uz + az);
        const C itr = C(1) / (C(p.tau_b) + C(0.5) * (phi + C(1)) * (C(p.tau_a) - C(p.tau_b)));
        const C itp = C(1) / C(p.tau_phi);
        const C gmu = C(p.fe_gamma) * mu;
        C s0 = C(0), s1 = C(0), sg = C(0);
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const C t = C(L::w(i)), t3 = C(3 * L::w(i));
            const C eu = C(L::ex(i)) * ux + C(L::ey(i)) * uy + C(L::ez(i)) * uz;
            const C ea = C(L::ex(i)) * ax + C(L::ey(i)) * ay + C(L::ez(i)) * az;
            const C ev = C(L::ex(i)) * vx + C(L::ey(i)) * vy + C(L::ez(i)) * vz;
            const C eg = C(L::ex(i)) * gx + C(L::ey(i)) * gy + C(L::ez(i)) * gz;
            // deviations of the equilibria from w_i
            const C hf = t * drho + t3 * (iso + eu * rho + C(1.5) * (eu * eu - usq * C(1.0 / 3.0)) * rho) +
                         kap * t * (C(4.5) * eg * eg - C(3) * g2);
            const C hg = t3 * (gmu + ev * phi + C(1.5) * (ev * ev - vsq * C(1.0 / 3.0)) * phi);
            // feq(u + a) - feq(u), written out (an O(F) term; no cancellation of O(1) values)
            const C edm = t3 * rho * (ea + C(1.5) * (ea * (C(2) * eu + ea) - a2 * C(1.0 / 3.0)));
            s0 += hf;
            s1 += edm;
            sg += hg;
            h[i] = h[i] + (hf - h[i]) * itr + edm;
            k[i] = k[i] + (hg - k[i]) * itp;
        }
        // rest populations: what mass leaves (f_0 - w_0 = (rho - 1) - sum_i (f_i - w_i),
        // g_0 = phi - sum_i g_i)
        h[0] = h[0] + ((drho - s0) - h[0]) * itr - s1;
        k[0] = k[0] + ((phi - sg) - k[0]) * itp;
        bad = nonfinite<C>(h[0] + k[0]);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            of[i] = St::encode(h[i], C(L::w(i)), 0u);
            og[i] = T(k[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; i++) {
        int slot, dx, dy, dz;
        post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
        // buffer-descriptor stores in AB (+0.9% on the spinodal case; AA measured 0.6% slower)
        const Geo &gw = LAYOUT == LAYOUT_AB ? gs : g;
        pop_store_at<L, LAYOUT, LAYOUT == LAYOUT_AB>(dst, S, slot, gw, dx, dy, dz, of[i], i);
        pop_store_at<L, LAYOUT, LAYOUT == LAYOUT_AB>(dst, S, Q + slot, gw, dx, dy, dz, og[i], i);
    }
    raise_divergence(p, bad);
}

// The AB kernels stage their x shifts in LDS where a workgroup is one whole row (every row
// of every workgroup inside the lattice; one row per workgroup).
bool fe_xstage(const StepParams &p, const LaunchCfg &c) {
    return c.grid.x == 1 && c.block.y == 1 && int(c.block.x) >= p.nx && c.block.x <= 512;
}

}  // namespace

hipError_t launch_fe_phi(int lattice, int storage, int layout, bool flags, const StepParams &p, const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_wide_storage(storage, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                if constexpr (LAY == LAYOUT_AB) {
                    if (fe_xstage(p, c)) {
                        const size_t lds = size_t(xmove_count<L>()) * c.block.x * c.block.y * sizeof(typename St::T);
                        if (int(c.block.x) == p.nx) {
                            if (flags) k_fe_phi<L, St, LAY, true, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                            else k_fe_phi<L, St, LAY, false, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                        } else {
                            if (flags) k_fe_phi<L, St, LAY, true, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                            else k_fe_phi<L, St, LAY, false, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                        }
                        return hipGetLastError();
                    }
                }
                if (flags) k_fe_phi<L, St, LAY, true><<<c.grid, c.block, 0, c.stream>>>(p);
                else k_fe_phi<L, St, LAY, false><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_step_fe(int lattice, int storage, int layout, bool flags, const StepParams &p,
                          const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_wide_storage(storage, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                if constexpr (LAY == LAYOUT_AB) {
                    if (fe_xstage(p, c)) {
                        const size_t lds = 2 * size_t(xmove_count<L>()) * c.block.x * c.block.y * sizeof(typename St::T);
                        if (int(c.block.x) == p.nx) {
                            if (flags) k_step_fe<L, St, LAY, true, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                            else k_step_fe<L, St, LAY, false, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                        } else {
                            if (flags) k_step_fe<L, St, LAY, true, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                            else k_step_fe<L, St, LAY, false, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                        }
                        return hipGetLastError();
                    }
                }
                if (flags) k_step_fe<L, St, LAY, true><<<c.grid, c.block, 0, c.stream>>>(p);
                else k_step_fe<L, St, LAY, false><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
