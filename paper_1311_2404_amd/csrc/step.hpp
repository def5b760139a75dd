// The fused stream-and-collide kernel of the polynomial-equilibrium models (one thread
// per node) and what every step kernel shares: the streaming patterns, the population
// addresses, the boundary-node rules and the divergence flag.  The entropic step is in
// step_elbm.hpp, the two-component Shan-Chen kernels in step_sc.hpp.
//
// Streaming patterns (GPU-algorithms subsection of the paper, AB and AA):
//   AB      : read the population arriving along e_i from node x - e_i of copy A
//             (propagate on read), write the post-collision value to node x of copy B.
//             Copy A therefore holds post-collision values; the physical population
//             f_i(x, t) is A[i][x - e_i].
//   AA even : read slot i of node x, write the post-collision f*_i to slot opp(i) of x.
//   AA odd  : read slot opp(i) of node x - e_i, write f*_i to slot i of node x + e_i.
//             Each thread reads and writes exactly the same locations, so the single
//             copy is updated in place without races; after an odd step the layout is
//             the plain one again.
// Rows along x are contiguous in both population layouts (row-interleaved tiles, the
// default, and SoA f[q][z][y][x]); a workgroup covers whole x rows when nx allows, so
// the shifts along x stay inside lines the same workgroup also reads (or go through LDS,
// XSTAGE below).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "collide.hpp"
#include "lattice.hpp"
#include "params.hpp"
#include "storage.hpp"

// Population loads and stores of the step kernels carry the non-temporal hint: every
// value is read once per step and written once, and is next touched only after ~2.5 GB
// of other traffic.  Measured on the 256^3 step: +5% for FP32 stores.  Loads take it
// where it pays:
//  - AB and the AA odd step: only populations with e_x = 0.  A wave's pull of an x-moving
//    population starts one element off its 256-byte segment, so one 128-byte line is
//    shared with the neighbouring wave; marked non-temporal, that line is often gone
//    before the neighbour reads it (FETCH_SIZE 7.5% above the algorithmic bytes; exact
//    without).  AB: +0.8% over hinting every load; AA: +1.3-1.6% (FP32, FP64).
//  - AA even step: every load (all aligned; +7% over none).
//  - 2-byte elements: only in the AA even step, where every access is aligned (+13% on
//    the BF16 256^3 step); elsewhere the hint costs them 3-4%.
// Where a step stages its shifts along x in LDS (XSTAGE of k_step and of the Shan-Chen
// kernels), the x-moving values are read and written on aligned segments, with the hint.
template <class L, int LAYOUT, class T>
__device__ __forceinline__ T pop_load(const T *ptr, int i) {
    if constexpr (sizeof(T) < 4) {
        if (LAYOUT == lbm::LAYOUT_AA_EVEN) return __builtin_nontemporal_load(ptr);
        return *ptr;
    }
    if ((LAYOUT == lbm::LAYOUT_AB || LAYOUT == lbm::LAYOUT_AA_ODD) && L::ex(i) != 0) return *ptr;
    return __builtin_nontemporal_load(ptr);
}
#define LBM_LOAD(ptr, i) pop_load<L, LAYOUT>((ptr), (i))
// Stores of population i.  The AA odd step writes x-moving populations one element off
// the wave's 256-byte segment, so each wave leaves a partly written 64-byte sector at
// both ends that the neighbouring wave completes.  Those stores go without the hint: the
// line then waits in L2 for its other half instead of reaching HBM as a partial write.
template <class L, int LAYOUT, class T>
__device__ __forceinline__ void pop_store(T *ptr, T v, int i) {
    if (LAYOUT == lbm::LAYOUT_AA_ODD && L::ex(i) != 0) *ptr = v;
    else __builtin_nontemporal_store(v, ptr);
}

namespace lbm {

// Divergence flag of a step: a node whose post-collision rest population is not finite
// raises *p.diverged, which the next synchronising call of the library reads back.  The
// rest population is formed from the node's mass (the conservation restore, or the
// free-energy rest equation), so a non-finite population or moment anywhere in the node
// reaches it: one class test per node, and the rarely taken store at the kernel's end,
// after the population stores.
template <class C>
__device__ __forceinline__ bool nonfinite(C v) {
    return !__builtin_isfinite(v);
}
__device__ __forceinline__ void raise_divergence(const StepParams &p, bool bad) {
    if (bad) *p.diverged = 1u;
}

// A node and its periodic neighbours.  at() is the linear node index (flags, psi,
// macroscopic fields); pa() is the node's offset inside one population's block, which
// differs from at() in the row-interleaved population layouts (tiles of 2^tyl rows).
struct Geo {
    int x, y, z, xm, xp, ym, yp, zm, zp;
    uint32_t nx, ny, rp, rpitch;
    uint32_t nyt;  // tiles per z plane: ceil(ny / 2^tyl) (the last one padded when 2^tyl does not divide ny)
    int tyl;
    __device__ __forceinline__ uint32_t y_of(int dy) const { return uint32_t(dy == 0 ? y : (dy > 0 ? yp : ym)); }
    __device__ __forceinline__ uint32_t z_of(int dz) const { return uint32_t(dz == 0 ? z : (dz > 0 ? zp : zm)); }
    __device__ __forceinline__ uint32_t x_of(int dx) const { return uint32_t(dx == 0 ? x : (dx > 0 ? xp : xm)); }
    __device__ __forceinline__ uint32_t at(int dx, int dy, int dz) const {
        return (z_of(dz) * ny + y_of(dy)) * nx + x_of(dx);
    }
    // offset of the row of node (x, y + dy, z + dz) inside a population's block
    __device__ __forceinline__ uint32_t row_off(int dy, int dz) const {
        const uint32_t yy = y_of(dy);
        return (z_of(dz) * nyt + (yy >> tyl)) * rp + (yy & ((1u << tyl) - 1u)) * rpitch;
    }
    __device__ __forceinline__ uint32_t pa(int dx, int dy, int dz) const { return row_off(dy, dz) + x_of(dx); }
};

__device__ __forceinline__ Geo make_geo(int x, int y, int z, int nx, int ny, int nz, uint32_t rp,
                                        uint32_t rpitch, int tyl) {
    Geo g;
    g.x = x;
    g.y = y;
    g.z = z;
    g.xm = (x == 0 ? nx : x) - 1;
    g.xp = (x + 1 == nx) ? 0 : x + 1;
    g.ym = (y == 0 ? ny : y) - 1;
    g.yp = (y + 1 == ny) ? 0 : y + 1;
    g.zm = (z == 0 ? nz : z) - 1;
    g.zp = (z + 1 == nz) ? 0 : z + 1;
    g.nx = uint32_t(nx);
    g.ny = uint32_t(ny);
    g.rp = rp;
    g.rpitch = rpitch;
    g.nyt = (uint32_t(ny) + (1u << tyl) - 1u) >> tyl;
    g.tyl = tyl;
    return g;
}

// Slot and neighbour offset of the physical population f_i(x) (where it is read) and of
// the post-collision value f*_i(x) (where it is written).
template <class L>
__device__ __forceinline__ void canon_dir(int layout, int i, int &slot, int &dx, int &dy, int &dz) {
    if (layout == LAYOUT_AA_EVEN) {
        slot = i;
        dx = dy = dz = 0;
    } else {
        slot = layout == LAYOUT_AB ? i : opp(i);
        dx = -L::ex(i);
        dy = -L::ey(i);
        dz = -L::ez(i);
    }
}
template <class L>
__device__ __forceinline__ void post_dir(int layout, int i, int &slot, int &dx, int &dy, int &dz) {
    slot = layout == LAYOUT_AA_EVEN ? opp(i) : i;
    if (layout == LAYOUT_AA_ODD) {
        dx = L::ex(i);
        dy = L::ey(i);
        dz = L::ez(i);
    } else {
        dx = dy = dz = 0;
    }
}

// Store of population slot `slot` at node x + (dx, dy, dz): pop_addr and pop_store, except
// for 2-byte elements, and for every element size when BUF.  Those go through a buffer
// descriptor built on the row's base (a scalar: y and z are the same for the whole
// workgroup) with the lane's 32-bit byte offset of x.  As plain stores the compiler
// chains the 19 addresses of a node into 64-bit per-lane pointer increments, one VALU
// add per store, which costs the steps bound by VALU issue (the 16-bit steps, the
// entropic step: BUF) and registers where many addresses are live (the Shan-Chen
// step).  The memory-bound 4- and 8-byte LBGK/MRT steps keep the per-lane 64-bit
// addresses: ~1% faster, in AA odd too, where the buffer form cut 93 VGPRs to 58 and
// still ran 0.6% slower.  The descriptor's fourth word is the gfx9 family's
// untyped-buffer format; its record count only bounds the row offset (< 2^31 bytes).
template <class L, int LAYOUT, bool BUF = false, class T>
__device__ __forceinline__ void pop_store_at(T *base, uint32_t S, int slot, const Geo &g, int dx, int dy, int dz, T v,
                                             int i) {
    if constexpr (sizeof(T) == 2 || BUF) {
        T *row = base + (size_t(slot) * S + g.row_off(dy, dz));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, 0x7fffffff, 0x00020000);
        const int off = int(g.x_of(dx) * uint32_t(sizeof(T)));
        // non-temporal (aux 2) except where pop_store leaves the hint off
        const bool plain = LAYOUT == LAYOUT_AA_ODD && L::ex(i) != 0;
        if constexpr (sizeof(T) == 2) {
            const short sv = __builtin_bit_cast(short, v);
            if (plain) __builtin_amdgcn_raw_buffer_store_b16(sv, rs, off, 0, 0);
            else __builtin_amdgcn_raw_buffer_store_b16(sv, rs, off, 0, 2);
        } else if constexpr (sizeof(T) == 4) {
            const int sv = __builtin_bit_cast(int, v);
            if (plain) __builtin_amdgcn_raw_buffer_store_b32(sv, rs, off, 0, 0);
            else __builtin_amdgcn_raw_buffer_store_b32(sv, rs, off, 0, 2);
        } else {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            const u32x2 sv = __builtin_bit_cast(u32x2, v);
            if (plain) __builtin_amdgcn_raw_buffer_store_b64(sv, rs, off, 0, 0);
            else __builtin_amdgcn_raw_buffer_store_b64(sv, rs, off, 0, 2);
        }
    } else {
        pop_store<L, LAYOUT>(pop_addr(base, S, slot, g, dx, dy, dz), v, i);
    }
}

// Aligned store of the lane's own x in row (y + dy, z + dz) of slot `slot`, with the
// non-temporal hint (the staged x-moving stores of the AA odd step).
template <bool BUF, class T>
__device__ __forceinline__ void pop_store_own_x(T *base, uint32_t S, int slot, const Geo &g, int dy, int dz, T v) {
    if constexpr (BUF || sizeof(T) == 2) {
        T *row = base + (size_t(slot) * S + g.row_off(dy, dz));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, 0x7fffffff, 0x00020000);
        const int off = int(uint32_t(g.x) * uint32_t(sizeof(T)));
        if constexpr (sizeof(T) == 2) __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(short, v), rs, off, 0, 2);
        else if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), rs, off, 0, 2);
        else {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, off, 0, 2);
        }
    } else {
        __builtin_nontemporal_store(v, pop_addr(base, S, slot, g, 0, dy, dz));
    }
}

// Address of population slot `slot` at node x + (dx, dy, dz) in a copy.  In the step
// kernels y and z are the same for the whole workgroup, so the slot and row part is a
// scalar base.  For 2-byte elements the x part is added as a 32-bit byte offset, which
// lets the load take the scalar base and a 32-bit vector offset (no 64-bit address
// arithmetic per lane), part of a +6% on the VALU-bound 16-bit steps.  For 4- and 8-byte
// elements, which are bound by memory, the plain per-lane 64-bit address is ~1% faster.
template <class T>
__device__ __forceinline__ T *pop_addr(T *base, uint32_t S, int slot, const Geo &g, int dx, int dy, int dz) {
    if constexpr (sizeof(T) == 2) {
        T *row = base + (size_t(slot) * S + g.row_off(dy, dz));
        using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return reinterpret_cast<T *>(reinterpret_cast<B *>(row) + g.x_of(dx) * uint32_t(sizeof(T)));
    } else {
        return base + (size_t(slot) * S + g.pa(dx, dy, dz));
    }
}

// Where the physical population f_i(x) currently lives (slot, offset in the slot's block).
template <class L>
__device__ __forceinline__ void canon_loc(int layout, int i, const Geo &g, int &slot, uint32_t &node) {
    if (layout == LAYOUT_AA_EVEN) {
        slot = i;
        node = g.pa(0, 0, 0);
    } else {
        slot = layout == LAYOUT_AB ? i : opp(i);
        node = g.pa(-L::ex(i), -L::ey(i), -L::ez(i));
    }
}

// Half-way bounce-back node (boundary-conditions subsection): a wet node whose
// populations streamed in from wall nodes are missing; each takes the value of the
// node's opposite population, i.e. what reached the node moving towards the wall is
// reflected in the same step.  The node then collides as a fluid node.
template <class L, class C>
__device__ __forceinline__ void complete_missing(C *h, const StepParams &p, const Geo &g) {
    C hb[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; i++) hb[i] = h[i];
#pragma unroll
    for (int i = 0; i < L::Q; i++)
        if (p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1) h[i] = hb[opp(i)];
}

// Equilibrium velocity node (boundary-conditions subsection): a population that streams
// in from a wall node is missing and takes the value of the node's opposite population;
// rho sums the completed set; the node leaves feq(rho, u_bc) (no relaxation, no force).
// Only nodes on a domain face run this, so the neighbour flag loads cost nothing elsewhere.
template <class L, class C>
__device__ __forceinline__ void velocity_node(const C *h, C *o, const StepParams &p, const Geo &g) {
    C drho = C(0);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const bool missing = p.flags[g.at(-L::ex(i), -L::ey(i), -L::ez(i))] == 1;
        drho += missing ? h[opp(i)] : h[i];
    }
    const C rho = C(1) + drho;
    const C ux = C(p.u_bc[0]), uy = C(p.u_bc[1]), uz = C(L::D == 3 ? p.u_bc[2] : 0.0);
    const C usq15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const C eu = C(L::ex(i)) * ux + C(L::ey(i)) * uy + C(L::ez(i)) * uz;
        o[i] = C(L::w(i)) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - usq15));
    }
}

// Index of population i among those that move along x (e_x != 0), or -1.
template <class L>
__host__ __device__ constexpr int xmove_index(int i) {
    int k = 0;
    for (int j = 0; j < i; j++) k += L::ex(j) != 0;
    return L::ex(i) != 0 ? k : -1;
}
template <class L>
__host__ __device__ constexpr int xmove_count() {
    int k = 0;
    for (int j = 0; j < L::Q; j++) k += L::ex(j) != 0;
    return k;
}

// FLAGS: 0 no node flags, 1 fluid and wall nodes, 2 also boundary nodes (equilibrium
// velocity and half-way bounce-back; their paths are compiled only where they exist).
//
// XSTAGE (AB and AA odd steps, whole x rows per workgroup): the populations that move
// along x are read, and in AA odd also written, on aligned segments, and the one-node
// shift along x goes through LDS, as in the paper's step algorithm.  Lane x loads the
// slot it pulls from (AB: i, AA odd: opp(i)) at its own x of the source row into LDS;
// after a barrier it takes the value of x - e_x (periodic within the row).  In AA odd,
// after the collision lane x puts f*_i into LDS, and after a second barrier writes
// position x of slot i from lane x - e_x.  Every location is still read and written on
// behalf of the node that owns it in place, by the workgroup of that node's row, reads
// before the first barrier and writes after the second.  A/B of the two libraries on one
// box (GLUPS): 256^3 FP32 AB 40.1 -> 41.8, AA 41.1 -> 41.4; shifted BF16 AB 79.2 -> 83.8,
// AA 82.0 -> 85.7; the FP32 duct (two 128-node rows per workgroup) 39.7 -> 40.3.
// XSTAGE: 0 none, 1 rows of exactly the workgroup's width, 2 rows shorter than it (lanes
// past the row's end).  Only form 2 carries the per-lane tests; on whole rows they cost
// the 16-bit steps 11-18% (shifted BF16 at 256^3: AA 84.9 -> 75.4, AB 83.1 -> 70.8 GLUPS).
template <class L, class St, int MODEL, int LAYOUT, int FLAGS, int XSTAGE = 0>
__global__ __launch_bounds__(512) void k_step(StepParams p) {
    static_assert(!XSTAGE || LAYOUT == LAYOUT_AA_ODD || LAYOUT == LAYOUT_AB, "x staging: AB and AA odd steps");
    constexpr bool RAGGED = XSTAGE == 2;
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q;
    // Rows of the workgroup are whole waves, so y and z are the same for every lane of a
    // wave: all row and tile offsets are scalar; only x and x +- 1 vary.  BGK and MRT with
    // 4- and 8-byte elements take two 128-node rows per workgroup where rows are that
    // short (y made wave-uniform by readfirstlane; +2.5% on the 128-wide FP32 duct); every
    // other step takes one row per workgroup and y from the workgroup index (the
    // readfirstlane form measured 6% slower on the 16-bit steps).
    constexpr bool MULTI_ROW = sizeof(T) >= 4 && (MODEL == M_BGK || MODEL == M_MRT);
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y;
    if constexpr (MULTI_ROW) y = blockIdx.y * blockDim.y + __builtin_amdgcn_readfirstlane(threadIdx.y);
    else y = blockIdx.y;
    const int z = blockIdx.z;

    // AB steps on padded rows (row-interleaved layout): lanes past the row's end run the
    // step on the row's last node and store the result into the row's padding, which is
    // never read.  Every store instruction of the row then writes whole memory sectors;
    // a partly written 64-byte sector costs a read-modify-write (rows of 248-254 FP32
    // nodes ran at 5.3-5.4 TB/s against 6.0 for 256).
    const bool active = x < p.nx && y < p.ny;
    const bool pad = LAYOUT == LAYOUT_AB && x >= p.nx && x < int(p.rpitch) && y < p.ny;
    // with XSTAGE the launch holds whole rows per workgroup, every one inside the lattice,
    // and every lane reaches the barriers; lanes past a row's end (when nx is not a whole
    // number of waves) work on the row's last node, load nothing of their own x and store
    // only where the plain step would (AB padding lanes)
    if (XSTAGE || active || pad) {
        const Geo g = make_geo(active ? x : p.nx - 1, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
        Geo gs = g;  // where this lane stores (AB: its own x)
        gs.x = x;
        const uint32_t n = g.at(0, 0, 0);
        const uint32_t S = p.S;
        // no __restrict__: with AA the two pointers are the same copy
        const T *src = static_cast<const T *>(p.src);
        T *dst = static_cast<T *>(p.dst);
        T raw[Q];
        // LDS of the x staging: per row of the workgroup, the x-moving values read (xin) and,
        // in AA odd, written (xout)
        [[maybe_unused]] extern __shared__ unsigned char lds_x[];
        [[maybe_unused]] const int rows_lds = LAYOUT == LAYOUT_AA_ODD ? 2 : 1;
        [[maybe_unused]] const int xw = RAGGED ? int(blockDim.x) : p.nx;  // LDS row stride (>= nx)
        [[maybe_unused]] const int xr = RAGGED ? (active ? x : p.nx - 1) : x;  // the node this lane works on
        [[maybe_unused]] T *xin = reinterpret_cast<T *>(lds_x) +
                                  size_t(MULTI_ROW ? threadIdx.y : 0) * rows_lds * xmove_count<L>() * xw;
        [[maybe_unused]] T *xout = xin + xmove_count<L>() * xw;
        // the node's flag is loaded ahead of the populations: after the staging barrier its
        // latency would stand alone before the collision's branch (+2.4% on the FP32 duct,
        // +2.9% FP64, +1.2% on the cavity's AB step)
        const uint32_t fl = FLAGS ? p.flags[n] : 0u;
        if constexpr (XSTAGE) {
            if constexpr (sizeof(T) == 4 && LAYOUT == LAYOUT_AA_ODD) {
                // AA odd, 4-byte elements: the x-moving values go from HBM straight into LDS
                // (global_load_lds_dword: lane l of a wave writes dword l after the wave's LDS
                // base, taken from M0), without a VGPR and a wait per value.  The scheduling
                // barrier keeps every use of a loaded value after the last load (the LDS loads
                // share the vector memory counter, so a use between them would have to wait
                // for all); the explicit vmcnt(0) completes the LDS writes before the
                // workgroup barrier.  A/B on one box: FP32 256^3 AA 41.2 -> 41.3 GLUPS, the
                // cavity's AA 35.7 -> 36.4; in AB the same form cost the FP32 duct 1.3%.
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    int slot, dx, dy, dz;
                    canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
                    if (L::ex(i) == 0) {
                        raw[i] = LBM_LOAD(pop_addr(src, S, slot, g, dx, dy, dz), i);
                    } else if (!RAGGED || active) {
                        // rows are whole waves of the workgroup: x & ~63 is the wave's first x;
                        // aux 2 is the non-temporal hint
                        auto lp = (__attribute__((address_space(3))) T *)(xin + xmove_index<L>(i) * xw + (x & ~63));
                        const uint32_t la = __builtin_amdgcn_readfirstlane(uint32_t(uintptr_t(lp)));
                        __builtin_amdgcn_global_load_lds(pop_addr(src, S, slot, g, 0, dy, dz),
                                                         (__attribute__((address_space(3))) void *)uintptr_t(la), 4, 0, 2);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
            } else {
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    int slot, dx, dy, dz;
                    canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
                    if (L::ex(i) == 0) raw[i] = LBM_LOAD(pop_addr(src, S, slot, g, dx, dy, dz), i);
                    else if (!RAGGED || active) xin[xmove_index<L>(i) * xw + x] = __builtin_nontemporal_load(pop_addr(src, S, slot, g, 0, dy, dz));
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if (L::ex(i) == 0) continue;
                const int xs = xr - L::ex(i);
                raw[i] = xin[xmove_index<L>(i) * xw + (xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs))];
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                int slot, dx, dy, dz;
                canon_dir<L>(LAYOUT, i, slot, dx, dy, dz);
                raw[i] = LBM_LOAD(pop_addr(src, S, slot, g, dx, dy, dz), i);
            }
        }
        T out[Q];
        bool bad = false;
        // equilibrium velocity nodes exist for the polynomial-equilibrium models
        const bool vel = FLAGS == 2 && fl == 2u;
        if (fl == 1u) {
            // full-way bounce-back: the stored values are returned along -e_i untouched
#pragma unroll
            for (int i = 0; i < Q; i++) out[i] = raw[opp(i)];
        } else {
            C h[Q], o[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) h[i] = St::decode(raw[i], C(L::w(i)));
            if (FLAGS == 2 && fl == 3u) complete_missing<L, C>(h, p, g);
            if (vel) {
                velocity_node<L, C>(h, o, p, g);
            } else if constexpr (MODEL == M_BGK) {
                collide_bgk<L, C>(h, o, p);
            } else if constexpr (MODEL == M_MRT) {
                collide_mrt<L, C>(h, o, p);
            } else if constexpr (MODEL == M_REG) {
                collide_reg<L, C>(h, o, p);
            } else {
                static_assert(MODEL == M_SMAG, "k_step: LBGK, MRT, regularized or Smagorinsky collision");
                collide_smag<L, C>(h, o, p);
            }
            bad = nonfinite<C>(o[0]);
            uint32_t r0 = 0;
            if constexpr (St::stochastic) r0 = sr_word0(n, hash32(p.seed ^ hash32(p.step + 0x9e3779b9u)));
#pragma unroll
            for (int i = 0; i < Q; i++) out[i] = St::encode(o[i], C(L::w(i)), St::stochastic ? sr_word(r0, i) : 0u);
        }
        if constexpr (XSTAGE && LAYOUT == LAYOUT_AA_ODD) {
#pragma unroll
            for (int i = 0; i < Q; i++)
                if (L::ex(i) != 0) xout[xmove_index<L>(i) * xw + x] = out[i];
            __syncthreads();
            if (!RAGGED || active) {
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    int slot, dx, dy, dz;
                    post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
                    if (L::ex(i) == 0) {
                        pop_store_at<L, LAYOUT>(dst, S, slot, g, dx, dy, dz, out[i], i);
                    } else {
                        const int xs = x - L::ex(i);
                        const T v = xout[xmove_index<L>(i) * xw + (xs < 0 ? xs + p.nx : (xs >= p.nx ? xs - p.nx : xs))];
                        pop_store_own_x<false>(dst, S, slot, g, dy, dz, v);
                    }
                }
            }
        } else if (!RAGGED || active || pad) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                int slot, dx, dy, dz;
                post_dir<L>(LAYOUT, i, slot, dx, dy, dz);
                if constexpr (LAYOUT == LAYOUT_AB) pop_store_at<L, LAYOUT>(dst, S, slot, gs, 0, 0, 0, out[i], i);
                else pop_store_at<L, LAYOUT>(dst, S, slot, g, dx, dy, dz, out[i], i);
            }
        }
        raise_divergence(p, bad);
    }
}

// Launches k_step<MODEL> for every lattice, storage (with the stochastic-rounding
// variants), layout and flag mode; one translation unit per model instantiates it.
template <int MODEL>
hipError_t launch_k_step(int lattice, int storage, int sr, int layout, int flags, const StepParams &p,
                         const LaunchCfg &c) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<true>(storage, sr, [&](auto st) {
            using St = decltype(st);
            return with_layout(layout, [&](auto lay) {
                constexpr int LAY = decltype(lay)::value;
                // the AB and AA odd steps stage their x shifts in LDS where a workgroup is whole
                // rows (every row of every workgroup inside the lattice)
                const bool xstage = c.grid.x == 1 && int(c.block.x) >= p.nx && c.block.x <= 512 &&
                                    p.ny % int(c.block.y) == 0;
                if constexpr (LAY == LAYOUT_AA_ODD || LAY == LAYOUT_AB) {
                    const size_t lds = (LAY == LAYOUT_AA_ODD ? 2 : 1) * size_t(xmove_count<L>()) *
                                       size_t(c.block.x) * size_t(c.block.y) * sizeof(typename St::T);
                    if (xstage && int(c.block.x) == p.nx) {
                        if (flags == 2) k_step<L, St, MODEL, LAY, 2, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                        else if (flags) k_step<L, St, MODEL, LAY, 1, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                        else k_step<L, St, MODEL, LAY, 0, 1><<<c.grid, c.block, lds, c.stream>>>(p);
                        return hipGetLastError();
                    }
                    // Rows shorter than the workgroup are staged too, except in the Smagorinsky
                    // step: with velocity nodes it holds 103 VGPRs (4 waves per SIMD), too few
                    // waves to cover the barriers, and its staged form ran 6-7% slower on the
                    // 254-node rows of the cavity.
                    if constexpr (MODEL != M_SMAG) {
                        if (xstage) {
                            if (flags == 2) k_step<L, St, MODEL, LAY, 2, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                            else if (flags) k_step<L, St, MODEL, LAY, 1, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                            else k_step<L, St, MODEL, LAY, 0, 2><<<c.grid, c.block, lds, c.stream>>>(p);
                            return hipGetLastError();
                        }
                    }
                }
                if (flags == 2) k_step<L, St, MODEL, LAY, 2><<<c.grid, c.block, 0, c.stream>>>(p);
                else if (flags) k_step<L, St, MODEL, LAY, 1><<<c.grid, c.block, 0, c.stream>>>(p);
                else k_step<L, St, MODEL, LAY, 0><<<c.grid, c.block, 0, c.stream>>>(p);
                return hipGetLastError();
            });
        });
    });
}

}  // namespace lbm
