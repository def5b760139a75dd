// C ABI of the LBM library (declared in include/lbm.h): argument checking, device
// memory, and the launch sequence of each call.  No computation happens here; every
// step of the method runs in the HIP kernels of this directory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dispatch.hpp"
#include "lbm.h"

using namespace lbm;

struct lbm_sim {
    int lattice = 0, model = 0, nx = 0, ny = 0, nz = 0, Q = 0, D = 0, C = 1;
    uint32_t N = 0;
    uint32_t S = 0;   // population slot stride (elements), fixed at allocation
    uint32_t rp = 0;      // population tile pitch (elements), fixed at allocation
    uint32_t rpitch = 0;  // population row pitch inside a tile (elements)
    int tyl = 0;          // log2 of the rows per tile
    size_t pop_elems = 0;  // elements of one population copy (all components)
    double tau = 1.0, g[3] = {0, 0, 0};
    int storage = LBM_F32, layout = LBM_AB, sr = 0;
    double s[19] = {0};
    int alpha_init = 0;
    double alpha_tol = 1e-10;
    int alpha_maxit = 20;
    double G = 0.0;
    int psi_mode = 0;
    double cs_smag = 0.1;  // Smagorinsky constant
    double u_bc[3] = {0.0, 0.0, 0.0};  // velocity of the equilibrium velocity nodes
    // free-energy model: tau_B, tau_phi, A, kappa, Gamma (tau is tau_A)
    double fe_tau_b = 1.0, fe_tau_phi = 1.0, fe_a = 0.04, fe_kappa = 0.04, fe_gamma = 1.0;
    hipStream_t stream = nullptr;
    int device = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t *flags_d = nullptr;
    bool has_walls = false;
    bool has_vel = false;  // some node is a boundary node (velocity or half-way bounce-back)
    void *psi_d = nullptr;
    double *stage = nullptr;
    double *macro_d = nullptr;  // FP64 rho[C][N] + u[3][N] scratch for lbm_macro / lbm_diag
    double *red_d = nullptr;    // diag partials + result
    unsigned int *bad_d = nullptr;
    unsigned int *div_d = nullptr;  // raised by a step kernel that produced a non-finite population
    bool diverged = false;          // a synchronising call has seen that flag since the last init
    // population layout (lbm_set_pop_layout): row-interleaved tiles or SoA, tile height
    // (log2, -1 = default), pads in bytes (-1 = default)
    int pop_kind = 0, pop_tyl = -1;
    int64_t row_pad = 0, block_pad = -1, soa_pad = -1;
    uint16_t *mlp_bf16 = nullptr;
    float *mlp_wf_d = nullptr;  // BF16 weights widened to FP32, then mu[6], isd[6]
    uint32_t *mlp_lane_d = nullptr;  // per-lane MFMA operand table (64 x 44 words)
    float mlp_host[MLP_NTOTAL] = {0};  // FP32 weights + input normalisation (mu, isd)
    bool mlp_set = false;
    unsigned long long *stats_d = nullptr;
    bool stats_on = false;
    // MLP training state (FP32 master weights, Adam moments, scratch)
    float *mlp_w_d = nullptr, *mlp_m_d = nullptr, *mlp_v_d = nullptr, *mlp_g_d = nullptr;
    float *mlp_norm_d = nullptr;  // mu[6], isd[6] of the inference path (FP32)
    float *mlp_tnorm_d = nullptr; // the same for a training pass
    float *mlp_part_d = nullptr;
    int64_t mlp_part_cap = 0;
    double *mlp_acc_d = nullptr;  // loss accumulator + feature moments scratch
    int64_t steps = 0;
    bool ready = false;
    uint32_t seed = 0x2013b1u;
    std::string err;
};

constexpr int DIAG_SCRATCH_BLOCKS = 2048;  // partial-sum sets of lbm_diag_noalloc's reduction
static __device__ __align__(256) double scratch[DIAG_SCRATCH_BLOCKS * 8];

namespace {

thread_local std::string t_err;

int fail(lbm_sim *s, int code, const std::string &msg) {
    t_err = msg;
    if (s) s->err = msg;
    return code;
}

int hip_fail(lbm_sim *s, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(s, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP, m);
}

#define HIPCHK(sim, expr)                                  \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(sim, e_, #expr); \
    } while (0)

constexpr uint64_t POP_RUN_BYTES_DEFAULT = 32768;  // default tile height: runs of at most this many bytes

size_t elem_size(int storage) {
    switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32:
    case LBM_F32S: return 4;
    default: return 2;
    }
}

size_t compute_size(int storage) { return storage == LBM_F64 ? 8 : 4; }

LaunchCfg node_cfg(const lbm_sim *s) {
    // x rows (or segments of at most 512 nodes) of whole waves per workgroup, so that y and
    // z are wave-uniform in the step kernels (scalar row and tile offsets).  One row per
    // workgroup, except BGK and MRT with 4- or 8-byte elements on rows of at most 128 nodes,
    // which take 256 / bx rows (their kernels read y per wave).
    const int bx = s->nx % 64 == 0 && s->nx <= 512 ? s->nx : std::min(256, ((s->nx + 63) / 64) * 64);
    int by = 1;
    if ((s->model == LBM_BGK || s->model == LBM_MRT) && elem_size(s->storage) >= 4 && bx <= 128)
        by = std::min(256 / bx, std::max(1, s->ny));
    LaunchCfg c;
    c.block = dim3(bx, by, 1);
    c.grid = dim3((s->nx + bx - 1) / bx, (s->ny + by - 1) / by, s->nz);
    c.stream = s->stream;
    return c;
}

// layout kind of the stored state after s->steps steps
int state_layout(const lbm_sim *s) {
    if (s->layout == LBM_AB) return LAYOUT_AB;
    return (s->steps & 1) ? LAYOUT_AA_ODD : LAYOUT_AA_EVEN;
}

StepParams base_params(const lbm_sim *s) {
    StepParams p;
    std::memset(&p, 0, sizeof(p));
    p.nx = s->nx;
    p.ny = s->ny;
    p.nz = s->nz;
    p.N = s->N;
    p.S = s->S;
    p.rp = s->rp;
    p.rpitch = s->rpitch;
    p.tyl = s->tyl;
    p.flags = s->has_walls ? s->flags_d : nullptr;
    p.omega = 1.0 / s->tau;
    for (int a = 0; a < 3; a++) {
        p.g[a] = s->g[a];
        p.g_f[a] = float(s->g[a]);
    }
    p.has_force = (s->g[0] != 0.0 || s->g[1] != 0.0 || s->g[2] != 0.0) ? 1 : 0;
    for (int k = 0; k < s->Q; k++) {
        const double n2 = s->lattice == LBM_D3Q19 ? D3Q19::mrt_n2(k) : D2Q9::mrt_n2(k);
        const bool conserved = k == 0 || k == 3 || k == 5 || (k == 7 && s->lattice == LBM_D3Q19);
        const double sk = s->s[k];
        p.mrt[0][k] = conserved ? 1.0 / n2 : (1.0 - sk) / n2;
        p.mrt[1][k] = conserved ? 0.0 : sk / n2;
        p.mrt[2][k] = conserved ? 0.0 : (1.0 - 0.5 * sk) / n2;
        for (int j = 0; j < 3; j++) p.mrt_f[j][k] = float(p.mrt[j][k]);
    }
    for (int a = 0; a < 3; a++) p.u_bc[a] = s->u_bc[a];
    p.tau0 = s->tau;
    p.tau_a = s->tau;
    p.tau_b = s->fe_tau_b;
    p.tau_phi = s->fe_tau_phi;
    p.fe_a = s->fe_a;
    p.fe_kappa = s->fe_kappa;
    p.fe_gamma = s->fe_gamma;
    p.smag_k = 36.0 * s->cs_smag * s->cs_smag;
    p.beta = 0.5 / s->tau;
    p.alpha_tol = s->alpha_tol;
    p.alpha_maxit = s->alpha_maxit;
    p.alpha_init = s->alpha_init;
    p.mlp = s->mlp_set ? s->mlp_bf16 : nullptr;
    p.mlp_wf = s->mlp_wf_d;
    p.mlp_lane = s->mlp_lane_d;
    p.stats = s->stats_on ? s->stats_d : nullptr;
    p.psi = s->psi_d;
    p.G = s->G;
    p.psi_mode = s->psi_mode;
    p.seed = s->seed;
    p.diverged = s->div_d;
    return p;
}

// Population layout.  Two are built:
//  - row-interleaved, f[z][y/TY][c][q][y%TY][x] (TY = 2^tyl rows per tile; by default the
//    largest power of two up to 64 whose run of TY rows holds at most 32 KB: 32 rows at
//    nx = 256 in FP32, 16 in FP64, 64 in BF16.  Against 8-row tiles, A/B on one box:
//    FP32 256^3 AA -1.2% and AB -2.6% per step, FP64 -2.6% / -1.6%, BF16 -0.9% / -0.7%,
//    the 128-wide duct FP32 -1.6% / -1.3% and FP64 -2.1% / -1.6%, the 254^3 cavity
//    -2.4% / -1.8%; 16 KB runs were slower than 8 KB ones at nx = 256 in FP32.
//    ceil(ny/TY) tiles per z plane, the last one padded with rows that are never
//    addressed when TY does not divide ny: 254 rows cost 0.8% more memory and keep the
//    tiling, which a 2-row tiling (the largest power of two dividing 254) lost:
//    33.8 against 39.5 GLUPS at 254^3):
//    each x row of every population is a run of RP
//    elements (nx rounded up to 256 bytes), and the C Q runs of one row lie together, so
//    a workgroup's pulls touch a few contiguous blocks instead of 2 C Q separate streams.
//    Slot stride RP, row pitch C Q RP plus 1 KB.  Measured on the 256^3 step against SoA:
//    FP32 +5 to +7%, FP64 +5%, the MRT duct +4%, Shan-Chen +4%; the 1 KB between row
//    blocks adds ~1% for FP32 and FP64 (0, 2, 3, 4, 5, 8 and 13 KB measured).
//    This is the default.
//  - SoA, f[c][q][z][y][x] (the paper's structure of arrays): slot stride S = N rounded
//    up to whole 256-byte units plus a pad of 17 such units, so that the Q population
//    arrays do not start at addresses that differ by a large power of two (which maps
//    the 2Q streams of a row onto the same HBM channels; measured +1 to +3% on the 256^3
//    step); row pitch nx.  Also taken when the tiled layout would not fit 32-bit offsets.
// lbm_set_pop_layout selects one and sets the tile height and the pads.  TY shrinks only
// while half of it still covers ny, so a short ny wastes less than half its tile.
void pop_geometry(lbm_sim *s) {
    const uint64_t align = 256 / elem_size(s->storage);
    const uint64_t cq = uint64_t(s->C) * s->Q;
    const uint64_t RP = (uint64_t(s->nx) + align - 1) / align * align + uint64_t(s->row_pad) / 256 * align;
    int tyl = s->pop_tyl;
    if (tyl < 0) {
        const uint64_t row_bytes = RP * elem_size(s->storage);
        tyl = 0;
        while (tyl < 6 && (row_bytes << (tyl + 1)) <= POP_RUN_BYTES_DEFAULT) tyl++;
    }
    while (tyl > 0 && (1 << (tyl - 1)) >= s->ny) tyl--;
    const uint64_t ty = uint64_t(1) << tyl, tiles = (uint64_t(s->ny) + ty - 1) / ty * s->nz;
    const uint64_t block_pad = s->block_pad >= 0 ? uint64_t(s->block_pad) : 1024;
    const uint64_t block = cq * ty * RP + block_pad / 256 * align;
    if (s->pop_kind == LBM_POP_TILED && tiles * block < (uint64_t(1) << 32)) {
        s->S = uint32_t(ty * RP);
        s->rp = uint32_t(block);
        s->rpitch = uint32_t(RP);
        s->tyl = tyl;
        s->pop_elems = size_t(tiles * block);
        return;
    }
    const uint64_t pad_bytes = s->soa_pad >= 0 ? uint64_t(s->soa_pad) : 17 * 256;
    const uint64_t S = (uint64_t(s->N) + align - 1) / align * align + pad_bytes / 256 * align;
    s->S = S >= (uint64_t(1) << 32) ? s->N : uint32_t(S);
    s->rp = uint32_t(s->nx);
    s->rpitch = 0;
    s->tyl = 0;
    s->pop_elems = size_t(cq) * s->S;
}

int ensure_alloc(lbm_sim *s) {
    if (s->ready) return LBM_OK;
    HIPCHK(s, hipSetDevice(s->device));
    pop_geometry(s);
    const size_t bytes = s->pop_elems * elem_size(s->storage);
    HIPCHK(s, hipMalloc(&s->buf[0], bytes));
    if (s->layout == LBM_AB) HIPCHK(s, hipMalloc(&s->buf[1], bytes));
    HIPCHK(s, hipMalloc(&s->stage, sizeof(double) * s->N));
    if (s->model == LBM_SHANCHEN || s->model == LBM_FREE_ENERGY)
        HIPCHK(s, hipMalloc(&s->psi_d, 2 * size_t(s->N) * compute_size(s->storage)));
    HIPCHK(s, hipMalloc(&s->bad_d, sizeof(unsigned int)));
    HIPCHK(s, hipMalloc(&s->div_d, sizeof(unsigned int)));
    HIPCHK(s, hipMemsetAsync(s->div_d, 0, sizeof(unsigned int), s->stream));
    HIPCHK(s, hipMalloc(&s->stats_d, sizeof(unsigned long long) * (NEWTON_BINS + 1)));
    HIPCHK(s, hipMemsetAsync(s->stats_d, 0, sizeof(unsigned long long) * (NEWTON_BINS + 1), s->stream));
    if (!s->flags_d) {
        HIPCHK(s, hipMalloc(&s->flags_d, s->N));
        HIPCHK(s, hipMemsetAsync(s->flags_d, 0, s->N, s->stream));
    }
    s->ready = true;
    return LBM_OK;
}

int ensure_macro_scratch(lbm_sim *s) {
    if (!s->macro_d) HIPCHK(s, hipMalloc(&s->macro_d, sizeof(double) * (size_t(s->C) + 3) * s->N));
    return LBM_OK;
}

PlaneParams plane_params(const lbm_sim *s, int layout, int c, int q) {
    PlaneParams p;
    std::memset(&p, 0, sizeof(p));
    p.nx = s->nx;
    p.ny = s->ny;
    p.nz = s->nz;
    p.N = s->N;
    p.S = s->S;
    p.rp = s->rp;
    p.rpitch = s->rpitch;
    p.tyl = s->tyl;
    p.layout = layout;
    p.comp = c;
    p.q = q;
    p.pop = s->buf[s->cur];
    p.plane = s->stage;
    p.plain = s->model == LBM_FREE_ENERGY && c == 1;  // the free-energy g lattice is stored plain
    return p;
}

int run_psi(lbm_sim *s) {
    StepParams p = base_params(s);
    p.src = s->buf[s->cur];
    HIPCHK(s, launch_psi(s->lattice, s->storage, state_layout(s), p, node_cfg(s)));
    return LBM_OK;
}

MacroParams macro_params(const lbm_sim *s, void *rho, void *u, int fp64, unsigned int *bad) {
    MacroParams m;
    std::memset(&m, 0, sizeof(m));
    m.nx = s->nx;
    m.ny = s->ny;
    m.nz = s->nz;
    m.N = s->N;
    m.S = s->S;
    m.rp = s->rp;
    m.rpitch = s->rpitch;
    m.tyl = s->tyl;
    m.layout = state_layout(s);
    m.model = s->model;
    m.ncomp = s->C;
    m.pop = s->buf[s->cur];
    m.flags = s->has_walls ? s->flags_d : nullptr;
    m.psi = s->psi_d;
    m.G = s->G;
    for (int a = 0; a < 3; a++) m.g[a] = s->g[a];
    for (int a = 0; a < 3; a++) m.u_bc[a] = s->u_bc[a];
    m.rho_out = rho;
    m.u_out = u;
    m.fp64 = fp64;
    m.bad = bad;
    return m;
}

int macro_into(lbm_sim *s, void *rho, void *u, int fp64, unsigned int *bad) {
    if (s->model == LBM_SHANCHEN) {
        int rc = run_psi(s);
        if (rc) return rc;
    }
    const MacroParams m = macro_params(s, rho, u, fp64, bad);
    HIPCHK(s, launch_macro(s->lattice, s->storage, m, node_cfg(s)));
    return LBM_OK;
}

// Scratch of lbm_diag_noalloc: the partial sums of its fused reduction (DIAG_SCRATCH_BLOCKS
// sets of 8 doubles) in a static device array, one copy per GPU, held until the process
// ends (131 KB).  Its size does not depend on the lattice: the reduction walks the nodes
// with a fixed grid.  Host code never uses the array's name as an address (it is a
// host-side stand-in): the device address is taken with hipGetSymbolAddress once per
// device, with that device current, and kept.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

int diag_scratch(lbm_sim *s, double **out) {
    if (s->device < 0 || s->device >= MAX_DEVICES) return fail(s, LBM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[s->device]) {
        HIPCHK(s, hipSetDevice(s->device));
        void *ptr = nullptr;
        HIPCHK(s, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[s->device] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[s->device];
    return LBM_OK;
}

bool valid_storage(int st) { return st >= LBM_F64 && st <= LBM_F16S; }

// flag mode of the step kernels: 0 no flags, 1 walls, 2 walls and boundary nodes
int flag_mode(const lbm_sim *s) { return s->has_walls ? (s->has_vel ? 2 : 1) : 0; }

}  // namespace

extern "C" {

int lbm_create(int lattice, int model, int nx, int ny, int nz, double tau, const double *force, lbm_sim **out) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(nullptr, LBM_EINVAL, "unknown lattice");
    if (model < LBM_BGK || model > LBM_FREE_ENERGY) return fail(nullptr, LBM_EINVAL, "unknown model");
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(nullptr, LBM_EINVAL, "grid sizes must be positive");
    if (lattice == LBM_D2Q9 && nz != 1) return fail(nullptr, LBM_EINVAL, "D2Q9 needs nz == 1");
    if (nz > 65535 || ny > 65535) return fail(nullptr, LBM_EINVAL, "ny and nz must be <= 65535");
    const double Nd = double(nx) * double(ny) * double(nz);
    if (Nd >= 4294967296.0) return fail(nullptr, LBM_EINVAL, "too many nodes (N must be < 2^32)");
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(nullptr, LBM_EINVAL, "tau must be finite and > 1/2");
    double g[3] = {0, 0, 0};
    if (force) {
        for (int a = 0; a < 3; a++) g[a] = force[a];
        if (lattice == LBM_D2Q9) g[2] = 0.0;
        for (int a = 0; a < 3; a++)
            if (!std::isfinite(g[a])) return fail(nullptr, LBM_EINVAL, "force must be finite");
    }
    if (model == LBM_ELBM && (g[0] != 0 || g[1] != 0 || g[2] != 0))
        return fail(nullptr, LBM_EUNSUPPORTED, "the entropic model takes no body force");
    if (model == LBM_REGULARIZED && (g[0] != 0 || g[1] != 0 || g[2] != 0))
        return fail(nullptr, LBM_EUNSUPPORTED, "the regularized model takes no body force");
    lbm_sim *s = new (std::nothrow) lbm_sim();
    if (!s) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    s->lattice = lattice;
    s->model = model;
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->Q = lattice == LBM_D2Q9 ? 9 : 19;
    s->D = lattice == LBM_D2Q9 ? 2 : 3;
    s->C = model == LBM_SHANCHEN || model == LBM_FREE_ENERGY ? 2 : 1;
    s->fe_tau_b = tau;
    s->N = uint32_t(Nd);
    s->tau = tau;
    for (int a = 0; a < 3; a++) s->g[a] = g[a];
    for (int k = 0; k < 19; k++) s->s[k] = 1.0 / tau;
    for (int k = 0; k < MLP_IN; k++) s->mlp_host[MLP_NPARAM + MLP_IN + k] = 1.0f;  // isd = 1
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    *out = s;
    return LBM_OK;
}

int lbm_set_storage(lbm_sim *s, int storage, int layout, int stochastic_round) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (s->ready) return fail(s, LBM_ESTATE, "storage can only be set before the first init");
    if (!valid_storage(storage)) return fail(s, LBM_EINVAL, "unknown storage");
    if (layout != LBM_AB && layout != LBM_AA) return fail(s, LBM_EINVAL, "unknown layout");
    if (stochastic_round && storage != LBM_BF16S && storage != LBM_F16S)
        return fail(s, LBM_EINVAL, "stochastic rounding applies to BF16S/F16S only");
    if (stochastic_round && (s->model == LBM_ELBM || s->model == LBM_SHANCHEN || s->model == LBM_FREE_ENERGY))
        return fail(s, LBM_EUNSUPPORTED, "stochastic rounding is built for BGK and MRT");
    if (s->model == LBM_FREE_ENERGY && storage != LBM_F64 && storage != LBM_F32 && storage != LBM_F32S)
        return fail(s, LBM_EUNSUPPORTED, "the free-energy model keeps F64, F32 or shifted F32 populations");
    // a separating mixture moves rho_c far from 1, so the shifted 16-bit values carry O(w)
    // deviations and their rounding stops conserving each component's mass (BF16: 3e-3 of
    // it in 300 steps of a 32^3 box at G = 0.9)
    if (s->model == LBM_SHANCHEN && (storage == LBM_BF16S || storage == LBM_F16S))
        return fail(s, LBM_EUNSUPPORTED, "the Shan-Chen model keeps F64, F32 or shifted F32 populations");
    s->storage = storage;
    s->layout = layout;
    s->sr = stochastic_round ? 1 : 0;
    return LBM_OK;
}

int lbm_set_pop_layout(lbm_sim *s, int kind, int tile_rows, int64_t row_pad, int64_t block_pad, int64_t soa_pad) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (s->ready) return fail(s, LBM_ESTATE, "the population layout can only be set before the first init");
    if (kind != LBM_POP_TILED && kind != LBM_POP_SOA) return fail(s, LBM_EINVAL, "unknown population layout");
    if (tile_rows != 0 && (tile_rows < 1 || tile_rows > 64 || (tile_rows & (tile_rows - 1)) != 0))
        return fail(s, LBM_EINVAL, "tile_rows must be 0 (default) or a power of two from 1 to 64");
    const int64_t lim = int64_t(1) << 20;
    if (row_pad < 0 || row_pad > lim || block_pad < -1 || block_pad > lim || soa_pad < -1 || soa_pad > lim)
        return fail(s, LBM_EINVAL, "pads must lie in [0, 1 MiB] (-1: default for block_pad and soa_pad)");
    int tyl = -1;
    if (tile_rows) {
        tyl = 0;
        while ((1 << tyl) < tile_rows) tyl++;
    }
    s->pop_kind = kind;
    s->pop_tyl = tyl;
    s->row_pad = row_pad;
    s->block_pad = block_pad;
    s->soa_pad = soa_pad;
    return LBM_OK;
}

int lbm_set_mrt_rates(lbm_sim *s, const double *rates, int q) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!rates || q != s->Q) return fail(s, LBM_EINVAL, "rates must hold Q values");
    for (int k = 0; k < q; k++)
        if (!std::isfinite(rates[k]) || rates[k] < 0.0 || rates[k] >= 2.0)
            return fail(s, LBM_EINVAL, "rates must lie in [0, 2)");
    for (int k = 0; k < q; k++) s->s[k] = rates[k];
    return LBM_OK;
}

int lbm_set_elbm(lbm_sim *s, int alpha_init, double tol, int max_iter) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (alpha_init < 0 || alpha_init > 2) return fail(s, LBM_EINVAL, "alpha_init must be 0, 1 or 2");
    if (!(tol > 0.0) || max_iter < 1 || max_iter > 64) return fail(s, LBM_EINVAL, "bad tolerance or iteration cap");
    s->alpha_init = alpha_init;
    s->alpha_tol = tol;
    s->alpha_maxit = max_iter;
    return LBM_OK;
}

int lbm_set_shanchen(lbm_sim *s, double G, int psi) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!std::isfinite(G) || (psi != 0 && psi != 1)) return fail(s, LBM_EINVAL, "bad G or psi");
    s->G = G;
    s->psi_mode = psi;
    return LBM_OK;
}

int lbm_set_free_energy(lbm_sim *s, double tau_b, double tau_phi, double a, double kappa, double gamma) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (s->model != LBM_FREE_ENERGY) return fail(s, LBM_EUNSUPPORTED, "the parameters belong to the free-energy model");
    if (!(tau_b > 0.5) || !(tau_phi > 0.5) || !std::isfinite(tau_b) || !std::isfinite(tau_phi))
        return fail(s, LBM_EINVAL, "tau_B and tau_phi must be finite and > 1/2");
    if (!std::isfinite(a) || !std::isfinite(kappa) || !std::isfinite(gamma) || kappa < 0.0 || gamma < 0.0)
        return fail(s, LBM_EINVAL, "A must be finite, kappa and Gamma finite and >= 0");
    s->fe_tau_b = tau_b;
    s->fe_tau_phi = tau_phi;
    s->fe_a = a;
    s->fe_kappa = kappa;
    s->fe_gamma = gamma;
    return LBM_OK;
}

int lbm_set_velocity_bc(lbm_sim *s, const double *u) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!u) return fail(s, LBM_EINVAL, "u is NULL");
    double v[3] = {u[0], u[1], s->D == 3 ? u[2] : 0.0};
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(v[a])) return fail(s, LBM_EINVAL, "the velocity must be finite");
    for (int a = 0; a < 3; a++) s->u_bc[a] = v[a];
    return LBM_OK;
}

int lbm_set_smagorinsky(lbm_sim *s, double cs) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (s->model != LBM_SMAGORINSKY) return fail(s, LBM_EUNSUPPORTED, "the constant belongs to the Smagorinsky model");
    if (!std::isfinite(cs) || cs < 0.0) return fail(s, LBM_EINVAL, "C_S must be finite and >= 0");
    s->cs_smag = cs;
    return LBM_OK;
}

int lbm_set_stream(lbm_sim *s, void *stream) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    s->stream = static_cast<hipStream_t>(stream);
    return LBM_OK;
}

int lbm_set_flags(lbm_sim *s, const uint8_t *flags) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!flags) return fail(s, LBM_EINVAL, "flags is NULL");
    bool walls = false, vel = false;
    for (uint32_t n = 0; n < s->N; n++) {
        if (flags[n] > LBM_HALFWAY_BB) return fail(s, LBM_EINVAL, "flag values must be 0 to 3");
        walls = walls || flags[n] != LBM_FLUID;
        vel = vel || flags[n] >= LBM_VELOCITY;
    }
    if (walls && s->model == LBM_SHANCHEN)
        return fail(s, LBM_EUNSUPPORTED, "walls are not supported with the Shan-Chen model");
    if (vel && s->model == LBM_ELBM)
        return fail(s, LBM_EUNSUPPORTED, "boundary nodes are built for the polynomial-equilibrium models");
    if (s->model == LBM_FREE_ENERGY)
        for (uint32_t n = 0; n < s->N; n++)
            if (flags[n] == LBM_VELOCITY)
                return fail(s, LBM_EUNSUPPORTED, "velocity nodes are not built for the free-energy model");
    HIPCHK(s, hipSetDevice(s->device));
    if (!s->flags_d) HIPCHK(s, hipMalloc(&s->flags_d, s->N));
    HIPCHK(s, hipMemcpyAsync(s->flags_d, flags, s->N, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->has_walls = walls;
    s->has_vel = vel;
    return LBM_OK;
}

int lbm_init_eq(lbm_sim *s, const double *rho, const double *u, const double *df) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!rho || !u) return fail(s, LBM_EINVAL, "rho and u are required");
    int rc = ensure_alloc(s);
    if (rc) return rc;
    const size_t N = s->N;
    double *rho_d = nullptr, *u_d = nullptr;
    HIPCHK(s, hipMalloc(&rho_d, sizeof(double) * s->C * N));
    HIPCHK(s, hipMalloc(&u_d, sizeof(double) * 3 * N));
    HIPCHK(s, hipMemcpyAsync(rho_d, rho, sizeof(double) * s->C * N, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(u_d, 0, sizeof(double) * 3 * N, s->stream));
    HIPCHK(s, hipMemcpyAsync(u_d, u, sizeof(double) * s->D * N, hipMemcpyHostToDevice, s->stream));
    s->steps = 0;
    s->cur = 0;
    s->diverged = false;
    HIPCHK(s, hipMemsetAsync(s->div_d, 0, sizeof(unsigned int), s->stream));
    const LaunchCfg cfg = node_cfg(s);
    for (int c = 0; c < s->C; c++)
        for (int q = 0; q < s->Q; q++) {
            PlaneParams p = plane_params(s, state_layout(s), c, q);
            p.rho = rho_d + size_t(c) * N;
            p.u = u_d;
            p.entropic = s->model == LBM_ELBM;
            if (s->model == LBM_FREE_ENERGY) {
                // rho[0] is rho, rho[1] is phi; both lattices start at their equilibria
                p.fe = 1;
                p.rho = rho_d;
                p.phi = rho_d + N;
                p.fe_a = s->fe_a;
                p.fe_gamma = s->fe_gamma;
            }
            if (df) {
                HIPCHK(s, hipMemcpyAsync(s->stage, df + (size_t(c) * s->Q + q) * N, sizeof(double) * N,
                                         hipMemcpyHostToDevice, s->stream));
                p.df = s->stage;
            }
            HIPCHK(s, launch_init_plane(s->lattice, s->storage, p, cfg));
        }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    HIPCHK(s, hipFree(rho_d));
    HIPCHK(s, hipFree(u_d));
    return LBM_OK;
}

int lbm_set_f(lbm_sim *s, const double *f) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!f) return fail(s, LBM_EINVAL, "f is NULL");
    int rc = ensure_alloc(s);
    if (rc) return rc;
    s->steps = 0;
    s->cur = 0;
    s->diverged = false;
    HIPCHK(s, hipMemsetAsync(s->div_d, 0, sizeof(unsigned int), s->stream));
    const LaunchCfg cfg = node_cfg(s);
    for (int c = 0; c < s->C; c++)
        for (int q = 0; q < s->Q; q++) {
            HIPCHK(s, hipMemcpyAsync(s->stage, f + (size_t(c) * s->Q + q) * s->N, sizeof(double) * s->N,
                                     hipMemcpyHostToDevice, s->stream));
            PlaneParams p = plane_params(s, state_layout(s), c, q);
            HIPCHK(s, launch_set_plane(s->lattice, s->storage, p, cfg));
        }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

int lbm_get_f(lbm_sim *s, double *f) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!f) return fail(s, LBM_EINVAL, "f is NULL");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    const LaunchCfg cfg = node_cfg(s);
    for (int c = 0; c < s->C; c++)
        for (int q = 0; q < s->Q; q++) {
            PlaneParams p = plane_params(s, state_layout(s), c, q);
            HIPCHK(s, launch_get_plane(s->lattice, s->storage, p, cfg));
            HIPCHK(s, hipMemcpyAsync(f + (size_t(c) * s->Q + q) * s->N, s->stage, sizeof(double) * s->N,
                                     hipMemcpyDeviceToHost, s->stream));
        }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

int lbm_step(lbm_sim *s, int n) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (n < 0) return fail(s, LBM_EINVAL, "n must be >= 0");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    if (s->model == LBM_ELBM && s->alpha_init == 2 && !s->mlp_set)
        return fail(s, LBM_ESTATE, "alpha_init = MLP needs lbm_mlp_set_weights first");
    if (s->diverged)
        return fail(s, LBM_EDIVERGED, "the state has diverged (a step produced a non-finite population); "
                                      "re-initialise it with lbm_init_eq or lbm_set_f");
    const LaunchCfg cfg = node_cfg(s);
    StepParams p = base_params(s);
    for (int k = 0; k < n; k++) {
        const int lay = state_layout(s);
        p.src = s->buf[s->cur];
        p.dst = s->layout == LBM_AB ? s->buf[1 - s->cur] : s->buf[0];
        p.step = uint32_t(s->steps);
        hipError_t e;
        switch (s->model) {
        case LBM_BGK: e = launch_step_bgk(s->lattice, s->storage, s->sr, lay, flag_mode(s), p, cfg); break;
        case LBM_MRT: e = launch_step_mrt(s->lattice, s->storage, s->sr, lay, flag_mode(s), p, cfg); break;
        case LBM_REGULARIZED: e = launch_step_reg(s->lattice, s->storage, s->sr, lay, flag_mode(s), p, cfg); break;
        case LBM_SMAGORINSKY: e = launch_step_smag(s->lattice, s->storage, s->sr, lay, flag_mode(s), p, cfg); break;
        case LBM_ELBM: e = launch_step_elbm(s->lattice, s->storage, lay, flag_mode(s), p, cfg); break;
        case LBM_FREE_ENERGY:
            e = launch_fe_phi(s->lattice, s->storage, lay, s->has_walls, p, cfg);
            if (e == hipSuccess) e = launch_step_fe(s->lattice, s->storage, lay, s->has_walls, p, cfg);
            break;
        default:
            e = launch_psi(s->lattice, s->storage, lay, p, cfg);
            if (e == hipSuccess) e = launch_step_sc(s->lattice, s->storage, lay, p, cfg);
        }
        if (e != hipSuccess) return hip_fail(s, e, "step launch");
        if (s->layout == LBM_AB) s->cur = 1 - s->cur;
        s->steps++;
    }
    return LBM_OK;
}

int lbm_macro(lbm_sim *s, double *rho, double *u) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!rho || !u) return fail(s, LBM_EINVAL, "rho and u are required");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    int rc = ensure_macro_scratch(s);
    if (rc) return rc;
    HIPCHK(s, hipMemsetAsync(s->bad_d, 0, sizeof(unsigned int), s->stream));
    double *rd = s->macro_d, *ud = s->macro_d + size_t(s->C) * s->N;
    rc = macro_into(s, rd, ud, 1, s->bad_d);
    if (rc) return rc;
    unsigned int bad = 0;
    HIPCHK(s, hipMemcpyAsync(rho, rd, sizeof(double) * s->C * s->N, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(u, ud, sizeof(double) * 3 * s->N, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(&bad, s->bad_d, sizeof(unsigned int), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (bad) return fail(s, LBM_EDIVERGED, std::to_string(bad) + " nodes with non-finite or non-positive density");
    return LBM_OK;
}

int lbm_macro_device(lbm_sim *s, void *rho_dev, void *u_dev, int fp64) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!rho_dev || !u_dev) return fail(s, LBM_EINVAL, "rho_dev and u_dev are required");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    return macro_into(s, rho_dev, u_dev, fp64 ? 1 : 0, nullptr);
}

int lbm_diag(lbm_sim *s, double out[8]) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!out) return fail(s, LBM_EINVAL, "out is NULL");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    int rc = ensure_macro_scratch(s);
    if (rc) return rc;
    const int nblocks = 2048;  // 8 workgroups per CU for the partial sums
    if (!s->red_d) HIPCHK(s, hipMalloc(&s->red_d, sizeof(double) * (size_t(nblocks) * 8 + 8)));
    double *rd = s->macro_d, *ud = s->macro_d + size_t(s->C) * s->N;
    rc = macro_into(s, rd, ud, 1, nullptr);
    if (rc) return rc;
    HIPCHK(s, launch_diag_reduce(rd, ud, s->N, s->C, s->model == LBM_FREE_ENERGY, s->red_d, nblocks,
                                 s->red_d + size_t(nblocks) * 8, s->stream));
    HIPCHK(s, hipMemcpyAsync(out, s->red_d + size_t(nblocks) * 8, sizeof(double) * 8, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    out[7] = 0.0;
    return LBM_OK;
}

int lbm_elbm_stats(lbm_sim *s, int enable, int reset, int64_t *hist, int nbins, int64_t *nonconv) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (nbins < 0 || nbins > NEWTON_BINS) return fail(s, LBM_EINVAL, "nbins must be in [0, 32]");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    if (hist || nonconv) {
        unsigned long long h[NEWTON_BINS + 1];
        HIPCHK(s, hipMemcpyAsync(h, s->stats_d, sizeof(h), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        for (int k = 0; k < nbins && hist; k++) hist[k] = int64_t(h[k]);
        if (nonconv) *nonconv = int64_t(h[NEWTON_BINS]);
    }
    if (reset) HIPCHK(s, hipMemsetAsync(s->stats_d, 0, sizeof(unsigned long long) * (NEWTON_BINS + 1), s->stream));
    s->stats_on = enable != 0;
    return LBM_OK;
}

int lbm_diag_noalloc(lbm_sim *s, void *out_dev) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!out_dev) return fail(s, LBM_EINVAL, "out_dev is NULL");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    double *partials = nullptr;
    int rc = diag_scratch(s, &partials);
    if (rc) return rc;
    if (s->model == LBM_SHANCHEN) {
        rc = run_psi(s);
        if (rc) return rc;
    }
    MacroParams m = macro_params(s, nullptr, nullptr, 1, nullptr);
    HIPCHK(s, launch_diag_fused(s->lattice, s->storage, m, partials, DIAG_SCRATCH_BLOCKS, static_cast<double *>(out_dev),
                                s->stream));
    return LBM_OK;
}

int lbm_steps_done(const lbm_sim *s, int64_t *steps) {
    if (!s || !steps) return fail(nullptr, LBM_EINVAL, "sim or steps is NULL");
    *steps = s->steps;
    return LBM_OK;
}

int lbm_sync(lbm_sim *s) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (s->ready && !s->diverged) {
        unsigned int flag = 0;
        HIPCHK(s, hipMemcpy(&flag, s->div_d, sizeof(flag), hipMemcpyDeviceToHost));
        s->diverged = flag != 0;
    }
    if (s->diverged)
        return fail(s, LBM_EDIVERGED, "a step produced a non-finite population (diverged state)");
    return LBM_OK;
}

const char *lbm_last_error(const lbm_sim *s) { return s ? s->err.c_str() : t_err.c_str(); }

void lbm_destroy(lbm_sim *s) {
    if (!s) return;
    if (s->ready || s->flags_d) (void)hipStreamSynchronize(s->stream);
    void *ptrs[] = {s->buf[0], s->buf[1], s->flags_d, s->psi_d, s->stage, s->macro_d, s->red_d, s->bad_d, s->div_d,
                    s->mlp_bf16, s->mlp_wf_d, s->mlp_lane_d, s->stats_d, s->mlp_w_d, s->mlp_m_d, s->mlp_v_d, s->mlp_g_d,
                    s->mlp_norm_d, s->mlp_tnorm_d, s->mlp_part_d, s->mlp_acc_d};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete s;
}

}  // extern "C"

namespace {

int mlp_alloc(lbm_sim *s, int64_t nbatch_max) {
    HIPCHK(s, hipSetDevice(s->device));
    if (!s->mlp_bf16) HIPCHK(s, hipMalloc(&s->mlp_bf16, sizeof(uint16_t) * MLP_NPARAM));
    if (!s->mlp_wf_d) HIPCHK(s, hipMalloc(&s->mlp_wf_d, sizeof(float) * MLP_NTOTAL));
    if (!s->mlp_lane_d) HIPCHK(s, hipMalloc(&s->mlp_lane_d, sizeof(uint32_t) * 64 * MLP_LANE_WORDS));
    if (!s->mlp_w_d) {
        HIPCHK(s, hipMalloc(&s->mlp_w_d, sizeof(float) * MLP_NPARAM));
        HIPCHK(s, hipMalloc(&s->mlp_m_d, sizeof(float) * MLP_NPARAM));
        HIPCHK(s, hipMalloc(&s->mlp_v_d, sizeof(float) * MLP_NPARAM));
        HIPCHK(s, hipMalloc(&s->mlp_g_d, sizeof(float) * MLP_NPARAM));
        HIPCHK(s, hipMalloc(&s->mlp_norm_d, sizeof(float) * MLP_NNORM));
        HIPCHK(s, hipMalloc(&s->mlp_tnorm_d, sizeof(float) * MLP_NNORM));
        HIPCHK(s, hipMalloc(&s->mlp_acc_d, sizeof(double) * (1 + 12 + 64 * 12 + 2 + 2 * 64)));
    }
    const int64_t parts = (nbatch_max + MLP_TRAIN_BLOCK - 1) / MLP_TRAIN_BLOCK;
    if (parts > s->mlp_part_cap) {
        if (s->mlp_part_d) HIPCHK(s, hipFree(s->mlp_part_d));
        s->mlp_part_d = nullptr;
        HIPCHK(s, hipMalloc(&s->mlp_part_d, sizeof(float) * size_t(parts) * (MLP_NPARAM + 1)));
        s->mlp_part_cap = parts;
    }
    return LBM_OK;
}

int mlp_upload(lbm_sim *s) {
    HIPCHK(s, hipMemcpyAsync(s->mlp_w_d, s->mlp_host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->mlp_norm_d, s->mlp_host + MLP_NPARAM, sizeof(float) * MLP_NNORM,
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, mlp_to_bf16(s->mlp_w_d, s->mlp_norm_d, s->mlp_bf16, s->mlp_wf_d, s->mlp_lane_d, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

uint64_t mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

extern "C" {

int lbm_mlp_set_weights(lbm_sim *s, const float *params, int n) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!params || (n != MLP_NPARAM && n != MLP_NTOTAL))
        return fail(s, LBM_EINVAL, "params must hold 1313 (or 1325 with normalisation) values");
    for (int k = 0; k < n; k++)
        if (!std::isfinite(params[k])) return fail(s, LBM_EINVAL, "params must be finite");
    int rc = mlp_alloc(s, 1);
    if (rc) return rc;
    std::memcpy(s->mlp_host, params, sizeof(float) * n);
    if (n == MLP_NPARAM)
        for (int k = 0; k < MLP_IN; k++) {
            s->mlp_host[MLP_NPARAM + k] = 0.0f;
            s->mlp_host[MLP_NPARAM + MLP_IN + k] = 1.0f;
        }
    rc = mlp_upload(s);
    if (rc) return rc;
    s->mlp_set = true;
    return LBM_OK;
}

int lbm_mlp_get_weights(lbm_sim *s, float *params, int n) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (!params || (n != MLP_NPARAM && n != MLP_NTOTAL))
        return fail(s, LBM_EINVAL, "params must hold 1313 (or 1325 with normalisation) values");
    std::memcpy(params, s->mlp_host, sizeof(float) * n);
    return LBM_OK;
}

int lbm_alpha_dataset(lbm_sim *s, int64_t n, uint64_t seed, void *feat_dev, void *alpha_dev, void *valid_dev) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (n < 0 || (n > 0 && (!feat_dev || !alpha_dev || !valid_dev)))
        return fail(s, LBM_EINVAL, "bad sample count or NULL buffer");
    if (n > (int64_t(1) << 31) * 256) return fail(s, LBM_EINVAL, "too many samples");
    if (s->model != LBM_ELBM) return fail(s, LBM_EUNSUPPORTED, "the alpha dataset needs the entropic model");
    if (!s->ready) return fail(s, LBM_ESTATE, "no state yet: call lbm_init_eq or lbm_set_f");
    if (n == 0) return LBM_OK;
    MlpDatasetParams d;
    std::memset(&d, 0, sizeof(d));
    d.sp = base_params(s);
    d.sp.src = s->buf[s->cur];
    d.n = n;
    d.seed = seed;
    d.feat = static_cast<float *>(feat_dev);
    d.alpha = static_cast<double *>(alpha_dev);
    d.valid = static_cast<uint8_t *>(valid_dev);
    d.layout = state_layout(s);
    HIPCHK(s, launch_alpha_dataset(s->lattice, s->storage, d, s->stream));
    return LBM_OK;
}

int lbm_mlp_forward(lbm_sim *s, const void *feat_dev, int64_t n, void *y_dev) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (n < 0 || (n > 0 && (!feat_dev || !y_dev))) return fail(s, LBM_EINVAL, "bad count or NULL buffer");
    if (!s->mlp_set) return fail(s, LBM_ESTATE, "no MLP weights set");
    HIPCHK(s, mlp_forward_bf16(s->mlp_wf_d, s->mlp_lane_d, static_cast<const float *>(feat_dev), n,
                               static_cast<float *>(y_dev), s->stream));
    return LBM_OK;
}

int lbm_mlp_loss_grad(lbm_sim *s, const void *feat_dev, const void *alpha_dev, int64_t n, double *loss, float *grad) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (n <= 0 || !feat_dev || !alpha_dev || !loss || !grad) return fail(s, LBM_EINVAL, "bad arguments");
    if (!s->mlp_set) return fail(s, LBM_ESTATE, "no MLP weights set");
    int rc = mlp_alloc(s, n);
    if (rc) return rc;
    HIPCHK(s, hipMemcpyAsync(s->mlp_w_d, s->mlp_host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->mlp_tnorm_d, s->mlp_host + MLP_NPARAM, sizeof(float) * MLP_NNORM,
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(s->mlp_acc_d, 0, sizeof(double), s->stream));
    HIPCHK(s, mlp_loss_grad(s->mlp_w_d, static_cast<const float *>(feat_dev), static_cast<const double *>(alpha_dev),
                            n, s->mlp_tnorm_d, s->mlp_tnorm_d + MLP_IN, s->mlp_part_d, int(s->mlp_part_cap),
                            s->mlp_g_d, s->mlp_acc_d, s->stream));
    HIPCHK(s, hipMemcpyAsync(grad, s->mlp_g_d, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(loss, s->mlp_acc_d, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

int lbm_mlp_train(lbm_sim *s, const void *feat_dev, const void *alpha_dev, int64_t n, int epochs, int batch, float lr,
                  uint64_t seed, float *loss_out) {
    if (!s) return fail(nullptr, LBM_EINVAL, "sim is NULL");
    if (n <= 0 || !feat_dev || !alpha_dev || epochs < 0 || batch <= 0 || !(lr > 0.0f))
        return fail(s, LBM_EINVAL, "bad training arguments");
    if (!s->mlp_set) return fail(s, LBM_ESTATE, "set initial weights with lbm_mlp_set_weights first");
    const int64_t bmax = std::min<int64_t>(batch, n);
    int rc = mlp_alloc(s, bmax);
    if (rc) return rc;
    const float *x = static_cast<const float *>(feat_dev);
    const double *t = static_cast<const double *>(alpha_dev);
    // input normalisation fitted on the data
    HIPCHK(s, mlp_moments(x, n, s->mlp_acc_d + 1, s->stream));
    double mom[12];
    HIPCHK(s, hipMemcpyAsync(mom, s->mlp_acc_d + 1, sizeof(mom), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    // input normalisation fitted on the data: mu = mean, isd = 1/std
    float norm[MLP_NNORM];
    for (int j = 0; j < MLP_IN; j++) {
        const double m = mom[j] / double(n), var = mom[6 + j] / double(n) - m * m;
        norm[j] = float(m);
        norm[MLP_IN + j] = var > 1e-30 ? float(1.0 / std::sqrt(var)) : 1.0f;
    }
    // carry the current weights over to the new normalisation exactly:
    // W1 diag(isd0) (x - mu0) + b1 = W1n diag(isd1) (x - mu1) + b1n
    float w[MLP_NTOTAL];
    std::memcpy(w, s->mlp_host, sizeof(w));
    float *W1 = w, *b1 = w + MLP_H * MLP_IN;
    const float *mu0 = s->mlp_host + MLP_NPARAM, *isd0 = mu0 + MLP_IN;
    for (int j = 0; j < MLP_H; j++)
        for (int k = 0; k < MLP_IN; k++) {
            const float a = W1[j * MLP_IN + k] * isd0[k];
            b1[j] += a * (norm[k] - mu0[k]);
            W1[j * MLP_IN + k] = a / norm[MLP_IN + k];
        }
    std::memcpy(w + MLP_NPARAM, norm, sizeof(norm));
    // the target is the series residual, standardised: r = (alpha - base - tmean) / tsd;
    // the output layer (w3, b3) is carried into those units and back exactly at the end
    double *racc = s->mlp_acc_d + 1 + 12 + 64 * 12;
    HIPCHK(s, mlp_resid_moments(x, t, n, racc, s->stream));
    double rm[2];
    HIPCHK(s, hipMemcpyAsync(rm, racc, sizeof(rm), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const double tmean = rm[0] / double(n);
    const double tvar = rm[1] / double(n) - tmean * tmean;
    const double tsd = tvar > 1e-40 ? std::sqrt(tvar) : 1.0;
    float *w3 = w + MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H, *b3 = w3 + MLP_H;
    for (int j = 0; j < MLP_H; j++) w3[j] = float(w3[j] / tsd);
    b3[0] = float((b3[0] - tmean) / tsd);
    HIPCHK(s, hipMemcpyAsync(s->mlp_tnorm_d, norm, sizeof(norm), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->mlp_w_d, w, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemsetAsync(s->mlp_m_d, 0, sizeof(float) * MLP_NPARAM, s->stream));
    HIPCHK(s, hipMemsetAsync(s->mlp_v_d, 0, sizeof(float) * MLP_NPARAM, s->stream));
    int tstep = 0;
    for (int e = 0; e < epochs; e++) {
        uint64_t pa = (mix(seed ^ (0x1000ull + e)) % uint64_t(n)) | 1ull;
        while (gcd64(pa, uint64_t(n)) != 1) pa += 2;
        pa %= uint64_t(n);
        if (pa == 0) pa = 1;
        const uint64_t pb = mix(seed ^ (0x2000ull + e)) % uint64_t(n);
        HIPCHK(s, hipMemsetAsync(s->mlp_acc_d, 0, sizeof(double), s->stream));
        int64_t nbatches = 0;
        for (int64_t r0 = 0; r0 < n; r0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - r0);
            HIPCHK(s, mlp_train_batch(s->mlp_w_d, x, t, r0, nb, n, pa, pb, s->mlp_tnorm_d, s->mlp_tnorm_d + MLP_IN,
                                      tmean, 1.0 / tsd, s->mlp_part_d, s->mlp_g_d, s->mlp_acc_d, s->stream));
            HIPCHK(s, mlp_adam(s->mlp_w_d, s->mlp_g_d, s->mlp_m_d, s->mlp_v_d, ++tstep, lr, s->stream));
            nbatches++;
        }
        if (loss_out) {
            double l = 0.0;
            HIPCHK(s, hipMemcpyAsync(&l, s->mlp_acc_d, sizeof(double), hipMemcpyDeviceToHost, s->stream));
            HIPCHK(s, hipStreamSynchronize(s->stream));
            loss_out[e] = float(l / double(nbatches) * tsd * tsd);  // in alpha units
        }
    }
    HIPCHK(s, hipMemcpyAsync(w, s->mlp_w_d, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int j = 0; j < MLP_H; j++) w3[j] = float(w3[j] * tsd);
    b3[0] = float(b3[0] * tsd + tmean);
    std::memcpy(s->mlp_host, w, sizeof(w));
    rc = mlp_upload(s);
    if (rc) return rc;
    s->mlp_set = true;
    return LBM_OK;
}

}  // extern "C"
