// Lattice velocity sets and weights for the HIP kernels (D2Q9, D3Q19).
//
// Weights are the paper's weight table (section 2): D2Q9 4/9, 1/9, 1/36 and D3Q19
// 1/3, 1/18, 1/36 by link length 0, 1, sqrt 2.  The velocity order puts opposite
// directions next to each other (opp(i) = i+1 for odd i, i-1 for even i > 0), which
// the bounce-back swap (boundary-conditions subsection) and the even/odd split of
// the MRT transforms use.  All accessors are constexpr so that fully unrolled loops
// fold them into immediates.
#pragma once

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    __host__ __device__ static constexpr int ex(int i) {
        constexpr int t[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i) {
        constexpr int t[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // squared norms of the MRT basis rows (the rows are listed with the MRT collision)
    __host__ __device__ static constexpr double mrt_n2(int k) {
        constexpr double t[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
        return t[k];
    }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    __host__ __device__ static constexpr int ex(int i) {
        constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i) {
        constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i) {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr double mrt_n2(int k) {
        constexpr double t[19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};
        return t[k];
    }
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

}  // namespace lbm
