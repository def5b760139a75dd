// The ELBM alpha proposal MLP: training data sampler, inference and training kernels.
//
// The network (6 -> 32 -> 32 -> 1, tanh hidden units) adds its output to the series
// estimate 2 + (a3 - 2 a4)/(3 a2) of the entropic alpha to propose the first Newton
// iterate; Newton still decides the result.  Training minimises the squared
// error of the proposal, i.e. of the network against the series residual alpha - base,
// which is formed in FP64 so that the small residual is not lost to FP32 rounding.
// Training is plain minibatch MSE with Adam in FP32; gradients are reduced across a
// wave with lane shuffles, then across the waves of a block and across blocks in a
// fixed order, so a training run is deterministic.
#include "dispatch.hpp"
#include "elbm.hpp"
#include "step.hpp"

namespace lbm {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {  // SplitMix64 finaliser
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <class L, class St>
__global__ __launch_bounds__(256) void k_alpha_dataset(MlpDatasetParams d) {
    using T = typename St::T;
    using C = typename St::C;
    constexpr int Q = L::Q;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= d.n) return;
    const StepParams &p = d.sp;
    const uint32_t n = uint32_t(mix64(d.seed ^ uint64_t(k)) % uint64_t(p.N));
    const int x = int(n % uint32_t(p.nx)), y = int((n / uint32_t(p.nx)) % uint32_t(p.ny));
    const int z = int(n / (uint32_t(p.nx) * uint32_t(p.ny)));
    const Geo g = make_geo(x, y, z, p.nx, p.ny, p.nz, p.rp, p.rpitch, p.tyl);
    float *feat = d.feat + 6 * k;
    if (p.flags && p.flags[n] == 1) {
        for (int j = 0; j < 6; j++) feat[j] = 0.0f;
        d.alpha[k] = 2.0;
        d.valid[k] = 0;
        return;
    }
    const T *src = static_cast<const T *>(p.src);
    C h[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
        int slot;
        uint32_t nd;
        canon_loc<L>(d.layout, i, g, slot, nd);
        h[i] = St::decode(src[size_t(slot) * p.S + nd], C(L::w(i)));
    }
    const Macro<C> m = moments<L, C>(h);
    const C irho = C(1) / m.rho;
    const C vx = m.jx * irho, vy = m.jy * irho, vz = m.jz * irho;
    C heq[Q];
    entropic_heq<L, C>(m.drho, m.rho, vx, vy, vz, heq);
    const double vsq = double(vx) * double(vx) + double(vy) * double(vy) + double(vz) * double(vz);
    AlphaNode an;
    alpha_prepare<L, C>(h, heq, an);
    if (an.dmax < ALPHA_SHORTCUT) {
        for (int j = 0; j < 6; j++) feat[j] = 0.0f;
        d.alpha[k] = 2.0;
        d.valid[k] = 0;
        return;
    }
    float xf[MLP_IN];
    alpha_features_m(an.am[2], an.am[3], an.am[4], an.mneg, an.mpos, double(m.rho), vsq, xf);
    const AlphaOut ao = alpha_root<L, C>(h, heq, an, 2.0, p.alpha_tol, p.alpha_maxit);
    for (int j = 0; j < 6; j++) feat[j] = xf[j];
    d.alpha[k] = ao.alpha;
    d.valid[k] = ao.converged ? 1 : 0;
}

// Every lane of a wave takes part in the wave-level evaluation; rows past n feed zeros
// and store nothing.
__global__ __launch_bounds__(256) void k_mlp_forward_bf16(const float *__restrict__ wf,
                                                         const uint32_t *__restrict__ lane, const float *x, int64_t n,
                                                         float *y) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float xr[MLP_IN];
    for (int j = 0; j < MLP_IN; j++) xr[j] = r < n ? x[MLP_IN * r + j] : 0.0f;
    const float v = mlp_eval_wave(lane, wf, xr);
    if (r < n) y[r] = v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int TB = MLP_TRAIN_BLOCK;  // samples (and threads: one wave) per training block
static_assert(TB == 64, "one wave per training block");

// Columns of the per-sample backward rows kept in LDS: A = [d1(32), d2(32), dy],
// B = [x(6), h1(32), h2(32), 1].  The gradient of weight p is sum_s A[s][ia] B[s][ib].
constexpr int GA_D1 = 0, GA_D2 = 32, GA_DY = 64, GA_W = 65;
constexpr int GB_X = 0, GB_H1 = 6, GB_H2 = 38, GB_ONE = 70, GB_W = 72;

// One block = one wave = up to 64 samples.  Sample r of the batch is row idx(r) of the
// data, idx(r) = (a r + b) mod n_all when a permutation is given (a coprime to n_all),
// the identity otherwise.  Inputs are normalised as (x - mu) * isd.  Each lane runs the
// forward and backward pass of its sample and leaves the vectors the weight gradients
// need in LDS; the lanes then sum them over the block's samples in a fixed order (W2's
// 32 x 32 gradient as 4 x 4 tiles per lane, the other 289 weights one at a time), so a
// training run is deterministic.  Writes the block's gradient (sum over its samples of
// d loss / d w, loss = mean over the batch) and squared-error sum into
// partials[block][MLP_NPARAM + 1].
__global__ __launch_bounds__(TB) void k_mlp_grad(const float *w, const float *xall, const double *tall,
                                                 int64_t row0, int64_t nbatch, int64_t n_all, uint64_t pa,
                                                 uint64_t pb, const float *mu, const float *isd, double tmean,
                                                 double tinv, float *partials) {
    __shared__ float s_w[MLP_NPARAM];
    __shared__ float sA[TB][GA_W + 1];
    __shared__ float sB[TB][GB_W + 1];
    for (int k = threadIdx.x; k < MLP_NPARAM; k += TB) s_w[k] = w[k];
    __syncthreads();
    const int lane = threadIdx.x;
    const int64_t r = int64_t(blockIdx.x) * TB + lane;
    const bool live = r < nbatch;
    float x[MLP_IN] = {0, 0, 0, 0, 0, 0};
    float base = 2.0f, t = 2.0f;
    if (live) {
        const int64_t gr = row0 + r;
        const int64_t row = pa ? int64_t((pa * uint64_t(gr) + pb) % uint64_t(n_all)) : gr;
        const float *xr = xall + MLP_IN * row;
        for (int j = 0; j < MLP_IN; j++) x[j] = (xr[j] - mu[j]) * isd[j];
        base = 2.0f + (xr[1] - 2.0f * xr[2]) * (1.0f / 3.0f);  // series estimate
        // the target: the series residual, standardised, formed in FP64 before rounding
        t = float((tall[row] - double(base) - tmean) * tinv);
    }
    const float *W1 = s_w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    const float *w3 = b2 + MLP_H, *b3 = w3 + MLP_H;
    float h1[MLP_H], h2[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; j++) {
        float s = b1[j];
#pragma unroll
        for (int k = 0; k < MLP_IN; k++) s = fmaf(W1[j * MLP_IN + k], x[k], s);
        h1[j] = tanhf(s);
    }
    float yv = b3[0];  // network output; the proposal is base + yv
#pragma unroll 4
    for (int j = 0; j < MLP_H; j++) {
        float s = b2[j];
#pragma unroll
        for (int k = 0; k < MLP_H; k++) s = fmaf(W2[j * MLP_H + k], h1[k], s);
        h2[j] = tanhf(s);
        yv = fmaf(w3[j], h2[j], yv);
    }
    const float err = live ? (yv - t) : 0.0f;
    const float dy = live ? 2.0f * err / float(nbatch) : 0.0f;
    // backward vectors of this sample into LDS (zeros for rows past the batch)
    float *A = sA[lane], *B = sB[lane];
    A[GA_DY] = dy;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) B[GB_X + k] = x[k];
    B[GB_ONE] = 1.0f;
    float d2[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; j++) {
        d2[j] = dy * w3[j] * (1.0f - h2[j] * h2[j]);
        A[GA_D2 + j] = d2[j];
        B[GB_H1 + j] = h1[j];
        B[GB_H2 + j] = h2[j];
    }
#pragma unroll 2
    for (int k = 0; k < MLP_H; k++) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < MLP_H; j++) s = fmaf(W2[j * MLP_H + k], d2[j], s);
        A[GA_D1 + k] = s * (1.0f - h1[k] * h1[k]);
    }
    const float e2 = wave_sum(err * err);
    __syncthreads();
    float *part = partials + size_t(blockIdx.x) * (MLP_NPARAM + 1);
    // W2: lane owns rows j0..j0+3 and columns k0..k0+3
    {
        const int j0 = 4 * (lane >> 3), k0 = 4 * (lane & 7);
        float acc[4][4] = {};
        for (int smp = 0; smp < TB; smp++) {
            float av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                av[q] = sA[smp][GA_D2 + j0 + q];
                bv[q] = sB[smp][GB_H1 + k0 + q];
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[q][v] = fmaf(av[q], bv[v], acc[q][v]);
        }
        float *gW2 = part + MLP_H * MLP_IN + MLP_H;
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int v = 0; v < 4; v++) gW2[(j0 + q) * MLP_H + k0 + v] = acc[q][v];
    }
    // the other weights: W1, b1 (d1 against x and 1), b2 (d2 against 1), w3, b3 (dy
    // against h2 and 1)
    constexpr int NW1 = MLP_H * MLP_IN, NREST = NW1 + MLP_H + 2 * MLP_H + 1;  // 289
    static_assert(NREST + MLP_H * MLP_H == MLP_NPARAM, "every weight but W2's once");
    for (int q = lane; q < NREST; q += TB) {
        int p, ia, ib;
        if (q < NW1) {
            p = q; ia = GA_D1 + q / MLP_IN; ib = GB_X + q % MLP_IN;                      // W1[j][k]
        } else if (q < NW1 + MLP_H) {
            p = q; ia = GA_D1 + (q - NW1); ib = GB_ONE;                                  // b1[j]
        } else {
            const int u = q - NW1 - MLP_H;                                               // b2, w3, b3
            p = NW1 + MLP_H + MLP_H * MLP_H + u;
            if (u < MLP_H) { ia = GA_D2 + u; ib = GB_ONE; }
            else if (u < 2 * MLP_H) { ia = GA_DY; ib = GB_H2 + (u - MLP_H); }
            else { ia = GA_DY; ib = GB_ONE; }
        }
        float acc = 0.0f;
        for (int smp = 0; smp < TB; smp++) acc = fmaf(sA[smp][ia], sB[smp][ib], acc);
        part[p] = acc;
    }
    if (lane == 0) part[MLP_NPARAM] = e2;
}

// The block partials summed per parameter (and the loss) in FP64, in a fixed order: four
// threads per parameter each take every fourth block, and their sums are added in LDS.
// (One thread per parameter walking every block kept only 6 workgroups busy: 16.6 us per
// 4096-row minibatch.)
constexpr int RED_SPLIT = 4;  // the LDS sum below is written out for four parts
__global__ __launch_bounds__(64 * RED_SPLIT) void k_mlp_reduce(const float *partials, int nparts, float *grad,
                                                               double *loss_acc, int64_t nbatch) {
    __shared__ double s[RED_SPLIT][64];
    const int j = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + j;
    double acc = 0.0;
    if (k <= MLP_NPARAM)
        for (int b = part; b < nparts; b += RED_SPLIT) acc += double(partials[size_t(b) * (MLP_NPARAM + 1) + k]);
    s[part][j] = acc;
    __syncthreads();
    if (part == 0 && k <= MLP_NPARAM) {
        const double tot = (s[0][j] + s[1][j]) + (s[2][j] + s[3][j]);
        if (k < MLP_NPARAM) grad[k] = float(tot);
        else if (loss_acc) *loss_acc += tot / double(nbatch);
    }
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, float b1t, float b2t, float lr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mk = b1 * m[k] + (1.0f - b1) * g[k];
    const float vk = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.0f - b1t), vh = vk / (1.0f - b2t);
    w[k] -= lr * mh / (sqrtf(vh) + eps);
}

// BF16 inference weights, and the same values widened to FP32 followed by the input
// normalisation (the layout mlp_eval reads)
__global__ void k_to_bf16(const float *w, const float *norm, uint16_t *wb, float *wf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < MLP_NPARAM) {
        const uint16_t b = __builtin_bit_cast(uint16_t, static_cast<__bf16>(w[k]));
        wb[k] = b;
        wf[k] = __uint_as_float(uint32_t(b) << 16);
    } else if (k < MLP_NTOTAL) {
        wf[k] = norm[k - MLP_NPARAM];
    }
}

// The per-lane operand table of mlp_eval_wave (64 lanes x MLP_LANE_WORDS words) from the
// BF16-valued FP32 weights.
__global__ void k_mlp_lane_pack(const float *wf, uint32_t *lane) {
    const int l = threadIdx.x;
    if (l >= 64) return;
    uint32_t *o = lane + l * MLP_LANE_WORDS;
    const float *W1 = wf, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H, *w3 = b2 + MLP_H;
    const int j = l % 32, q = l / 32;
    float a[8];
    // layer 1: [W1 row j | b1[j] | 0] in lanes 0-31 (K = 0..7), zeros for K = 8..15
    for (int t = 0; t < 8; t++) a[t] = q == 0 ? (t < MLP_IN ? W1[j * MLP_IN + t] : (t == MLP_IN ? b1[j] : 0.0f)) : 0.0f;
    for (int t = 0; t < 4; t++) o[t] = pack_bf16x2(a[2 * t], a[2 * t + 1]);
    // layer 2, chunk c: W2[j][16c + 8(t/4) + 4q + t%4]
    for (int c = 0; c < 2; c++) {
        for (int t = 0; t < 8; t++) a[t] = W2[j * MLP_H + 16 * c + 8 * (t / 4) + 4 * q + (t % 4)];
        for (int t = 0; t < 4; t++) o[4 + 4 * c + t] = pack_bf16x2(a[2 * t], a[2 * t + 1]);
    }
    // b2 and w3 of the accumulator rows 8(r/4) + 4q + r%4
    for (int r = 0; r < 16; r++) {
        const int row = 8 * (r / 4) + 4 * q + (r % 4);
        o[12 + r] = __float_as_uint(b2[row]);
        o[28 + r] = __float_as_uint(w3[row]);
    }
}

// sums and sums of squares of the series residual alpha - (2 + (x1 - 2 x2)/3)
__global__ __launch_bounds__(256) void k_resid_moments(const float *x, const double *t, int64_t n, double *partials) {
    __shared__ double s[2][256];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
        const float base = 2.0f + (x[6 * r + 1] - 2.0f * x[6 * r + 2]) * (1.0f / 3.0f);
        const double v = t[r] - double(base);
        a0 += v;
        a1 += v * v;
    }
    s[0][threadIdx.x] = a0;
    s[1][threadIdx.x] = a1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) partials[blockIdx.x * 2 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_resid_final(const double *partials, int nb, double *out) {
    const int j = threadIdx.x;
    if (j >= 2) return;
    double a = 0.0;
    for (int b = 0; b < nb; b++) a += partials[b * 2 + j];
    out[j] = a;
}

// sums and sums of squares of the 6 features (FP64, fixed-order two-level reduction)
__global__ __launch_bounds__(256) void k_moments(const float *x, int64_t n, double *partials) {
    __shared__ double s[12][256];
    double acc[12] = {0};
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256)
        for (int j = 0; j < 6; j++) {
            const double v = x[6 * r + j];
            acc[j] += v;
            acc[6 + j] += v * v;
        }
    for (int j = 0; j < 12; j++) s[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int j = 0; j < 12; j++) s[j][threadIdx.x] += s[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 12) partials[blockIdx.x * 12 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_moments_final(const double *partials, int nb, double *out) {
    const int j = threadIdx.x;
    if (j >= 12) return;
    double a = 0.0;
    for (int b = 0; b < nb; b++) a += partials[b * 12 + j];
    out[j] = a;
}

}  // namespace

hipError_t launch_alpha_dataset(int lattice, int storage, const MlpDatasetParams &p, hipStream_t s) {
    return with_lattice(lattice, [&](auto lt) {
        using L = decltype(lt);
        return with_storage<false>(storage, 0, [&](auto st) {
            using St = decltype(st);
            const int64_t nb = (p.n + 255) / 256;
            k_alpha_dataset<L, St><<<dim3(uint32_t(nb)), 256, 0, s>>>(p);
            return hipGetLastError();
        });
    });
}

hipError_t mlp_forward_bf16(const float *wf, const uint32_t *lane, const float *x, int64_t n, float *y,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_mlp_forward_bf16<<<dim3(uint32_t((n + 255) / 256)), 256, 0, s>>>(wf, lane, x, n, y);
    return hipGetLastError();
}

// grad of the mean loss over rows [0, n) of (x, t) in order (no permutation).
hipError_t mlp_loss_grad(const float *w, const float *x, const double *t, int64_t n, const float *mu,
                         const float *isd, float *partials, int nparts, float *grad, double *loss, hipStream_t s) {
    if (n <= 0 || nparts < int((n + TB - 1) / TB)) return hipErrorInvalidValue;
    const int nb = int((n + TB - 1) / TB);
    k_mlp_grad<<<nb, TB, 0, s>>>(w, x, t, 0, n, n, 0, 0, mu, isd, 0.0, 1.0, partials);
    k_mlp_reduce<<<(MLP_NPARAM + 1 + 63) / 64, 64 * RED_SPLIT, 0, s>>>(partials, nb, grad, loss, n);
    return hipGetLastError();
}

hipError_t mlp_adam(float *w, const float *grad, float *m, float *v, int t, float lr, hipStream_t s) {
    const float b1t = powf(0.9f, float(t)), b2t = powf(0.999f, float(t));
    k_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(w, grad, m, v, b1t, b2t, lr);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *w, const float *norm, uint16_t *wb, float *wf, uint32_t *lane, hipStream_t s) {
    k_to_bf16<<<(MLP_NTOTAL + 255) / 256, 256, 0, s>>>(w, norm, wb, wf);
    k_mlp_lane_pack<<<1, 64, 0, s>>>(wf, lane);
    return hipGetLastError();
}

hipError_t mlp_resid_moments(const float *x, const double *t, int64_t n, double *acc, hipStream_t s) {
    const int nb = 64;
    k_resid_moments<<<nb, 256, 0, s>>>(x, t, n, acc + 2);
    k_resid_final<<<1, 64, 0, s>>>(acc + 2, nb, acc);
    return hipGetLastError();
}

hipError_t mlp_moments(const float *x, int64_t n, double *acc, hipStream_t s) {
    const int nb = 64;
    k_moments<<<nb, 256, 0, s>>>(x, n, acc + 12);
    k_moments_final<<<1, 64, 0, s>>>(acc + 12, nb, acc);
    return hipGetLastError();
}

// One training minibatch: rows row0 .. row0 + nbatch - 1 of the permuted order.
hipError_t mlp_train_batch(const float *w, const float *x, const double *t, int64_t row0, int64_t nbatch,
                           int64_t n_all, uint64_t pa, uint64_t pb, const float *mu, const float *isd, double tmean,
                           double tinv, float *partials, float *grad, double *loss_acc, hipStream_t s) {
    const int nb = int((nbatch + TB - 1) / TB);
    k_mlp_grad<<<nb, TB, 0, s>>>(w, x, t, row0, nbatch, n_all, pa, pb, mu, isd, tmean, tinv, partials);
    k_mlp_reduce<<<(MLP_NPARAM + 1 + 63) / 64, 64 * RED_SPLIT, 0, s>>>(partials, nb, grad, loss_acc, nbatch);
    return hipGetLastError();
}

}  // namespace lbm
