// Vectorised AB step: each thread owns VEC consecutive nodes along x, so every
// population moves as one aligned VEC-wide load and one aligned VEC-wide store
// (16 bytes for FP32 at VEC = 4) instead of VEC scalar accesses.  The +-1 shift of the
// x-moving populations is taken from the neighbouring lane with a lane shuffle
// (periodic inside the row), which needs each x row to lie inside one wave:
// R = nx / VEC lanes per row with R dividing 64.  Other shapes use the scalar kernel.
#pragma once
#include "step.hpp"

namespace lbm {

template <class T>
__device__ __forceinline__ T lane_pick(T v, int src_lane) {
    if constexpr (sizeof(T) == 2) return T(__shfl(int(v), src_lane, 64));
    else return __shfl(v, src_lane, 64);
}

template <class L, class St, int MODEL, bool FLAGS, int VEC>
__global__ __launch_bounds__(256) void k_step_vec(StepParams p) {
    using T = typename St::T;
    using C = typename St::C;
    using TV = T __attribute__((ext_vector_type(VEC)));
    constexpr int Q = L::Q;
    const int R = p.nx / VEC;                      // lanes per row (divides 64)
    const int r = threadIdx.x;                     // position in the row, blockDim.x == R
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (y >= p.ny) return;
    const int lane = __lane_id();
    const int base = lane - r;                     // first lane of this row in the wave
    const int left = base + (r + R - 1) % R, right = base + (r + 1) % R;
    const int x0 = r * VEC;
    const int ym = (y == 0 ? p.ny : y) - 1, yp = (y + 1 == p.ny) ? 0 : y + 1;
    const int zm = (z == 0 ? p.nz : z) - 1, zp = (z + 1 == p.nz) ? 0 : z + 1;
    auto row = [&](int dy, int dz) -> uint32_t {
        const int yy = dy == 0 ? y : (dy > 0 ? yp : ym);
        const int zz = dz == 0 ? z : (dz > 0 ? zp : zm);
        const uint32_t uy = uint32_t(yy);  // offset of the row in a population block
        const uint32_t nyt = (uint32_t(p.ny) + (1u << p.tyl) - 1u) >> p.tyl;
        return (uint32_t(zz) * nyt + (uy >> p.tyl)) * p.rp + (uy & ((1u << p.tyl) - 1u)) * p.rpitch;
    };
    const T *src = static_cast<const T *>(p.src);
    T *dst = static_cast<T *>(p.dst);
    const uint32_t S = p.S;
    const uint32_t own = row(0, 0) + uint32_t(x0);                                         // population offset
    const uint32_t own_n = (uint32_t(z) * uint32_t(p.ny) + uint32_t(y)) * uint32_t(p.nx) + uint32_t(x0);  // node index

    // gather: raw[i][v] is population i arriving at node x0 + v
    T raw[Q][VEC];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        const TV vin = *reinterpret_cast<const TV *>(src + size_t(i) * S + row(-L::ey(i), -L::ez(i)) + x0);
        T a[VEC];
#pragma unroll
        for (int v = 0; v < VEC; v++) a[v] = vin[v];
        if (L::ex(i) == 1) {  // source x - 1: last element of the left neighbour, then own 0..VEC-2
            const T carry = lane_pick(a[VEC - 1], left);
#pragma unroll
            for (int v = VEC - 1; v > 0; v--) a[v] = a[v - 1];
            a[0] = carry;
        } else if (L::ex(i) == -1) {  // source x + 1: own 1..VEC-1, then first of the right neighbour
            const T carry = lane_pick(a[0], right);
#pragma unroll
            for (int v = 0; v < VEC - 1; v++) a[v] = a[v + 1];
            a[VEC - 1] = carry;
        }
#pragma unroll
        for (int v = 0; v < VEC; v++) raw[i][v] = a[v];
    }
    uint32_t key = 0;
    if constexpr (St::stochastic) key = hash32(p.seed ^ hash32(p.step + 0x9e3779b9u));
    T out[Q][VEC];
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const bool wall = FLAGS && p.flags[own_n + v] == 1;
        if (wall) {
#pragma unroll
            for (int i = 0; i < Q; i++) out[i][v] = raw[opp(i)][v];
            continue;
        }
        C h[Q], o[Q];
#pragma unroll
        for (int i = 0; i < Q; i++) h[i] = St::decode(raw[i][v], C(L::w(i)));
        if constexpr (MODEL == M_BGK) collide_bgk<L, C>(h, o, p);
        else collide_mrt<L, C>(h, o, p);
        SrStream rs{0u};
        uint32_t draw = 0;
        if constexpr (St::stochastic) rs = sr_stream(own_n + v, key);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            uint32_t rnd = 0;
            if constexpr (St::stochastic) {
                if (i % 2 == 0) draw = rs.next();
                rnd = i % 2 == 0 ? draw : draw << 16;
            }
            out[i][v] = St::encode(o[i], C(L::w(i)), rnd);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; i++) {
        TV vo;
#pragma unroll
        for (int v = 0; v < VEC; v++) vo[v] = out[i][v];
        LBM_STORE(reinterpret_cast<TV *>(dst + size_t(i) * S + own), vo);
    }
}

// VEC usable for this lattice width, or 0 for the scalar kernel.
inline int vec_width(int nx, int elem_bytes) {
    const int want = elem_bytes == 8 ? 2 : (elem_bytes == 4 ? 4 : 8);  // 16-byte accesses
    for (int v = want; v >= 2; v /= 2)
        if (nx % v == 0 && nx / v <= 64 && 64 % (nx / v) == 0) return v;
    return 0;
}

}  // namespace lbm
