"""Python binding of the MI355X lattice Boltzmann library (``liblbm.so``, C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the
library.  The module-level ``lbm_*`` functions mirror the C entry points one to one;
:class:`Sim` is a small convenience wrapper around a handle.  Host arrays are numpy
float64 (C order); device buffers are torch CUDA tensors (PyTorch supplies device
memory and streams only).  The library must be built (``python -m
paper_1311_2404_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_BGK, LBM_MRT, LBM_ELBM, LBM_SHANCHEN, LBM_REGULARIZED, LBM_SMAGORINSKY, LBM_FREE_ENERGY = 0, 1, 2, 3, 4, 5, 6
LBM_F64, LBM_F32, LBM_F32S, LBM_BF16S, LBM_F16S = 0, 1, 2, 3, 4
LBM_AB, LBM_AA = 0, 1
LBM_POP_TILED, LBM_POP_SOA = 0, 1
LBM_FLUID, LBM_WALL_BB, LBM_VELOCITY, LBM_HALFWAY_BB = 0, 1, 2, 3
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_EUNSUPPORTED, LBM_EDIVERGED = 0, -1, -2, -3, -4, -5, -6
MLP_NPARAM = 1313
MLP_NTOTAL = 1325  # weights + input normalisation mu[6], isd[6]
STORAGE_NAMES = {LBM_F64: "f64", LBM_F32: "f32", LBM_F32S: "f32s", LBM_BF16S: "bf16s", LBM_F16S: "f16s"}
ELEM_BYTES = {LBM_F64: 8, LBM_F32: 4, LBM_F32S: 4, LBM_BF16S: 2, LBM_F16S: 2}

# every entry point declared in include/lbm.h: (name, restype, argtypes)
_vp, _dp, _fp, _i64 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float), C.c_int64
_SIGS = [
    ("lbm_create", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.POINTER(_vp)]),
    ("lbm_set_storage", C.c_int, [_vp, C.c_int, C.c_int, C.c_int]),
    ("lbm_set_pop_layout", C.c_int, [_vp, C.c_int, C.c_int, _i64, _i64, _i64]),
    ("lbm_set_mrt_rates", C.c_int, [_vp, _dp, C.c_int]),
    ("lbm_set_elbm", C.c_int, [_vp, C.c_int, C.c_double, C.c_int]),
    ("lbm_set_shanchen", C.c_int, [_vp, C.c_double, C.c_int]),
    ("lbm_set_velocity_bc", C.c_int, [_vp, _dp]),
    ("lbm_set_free_energy", C.c_int, [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]),
    ("lbm_set_smagorinsky", C.c_int, [_vp, C.c_double]),
    ("lbm_set_stream", C.c_int, [_vp, _vp]),
    ("lbm_set_flags", C.c_int, [_vp, C.POINTER(C.c_uint8)]),
    ("lbm_init_eq", C.c_int, [_vp, _dp, _dp, _dp]),
    ("lbm_set_f", C.c_int, [_vp, _dp]),
    ("lbm_get_f", C.c_int, [_vp, _dp]),
    ("lbm_step", C.c_int, [_vp, C.c_int]),
    ("lbm_macro", C.c_int, [_vp, _dp, _dp]),
    ("lbm_macro_device", C.c_int, [_vp, _vp, _vp, C.c_int]),
    ("lbm_diag", C.c_int, [_vp, _dp]),
    ("lbm_diag_noalloc", C.c_int, [_vp, _vp]),
    ("lbm_elbm_stats", C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(_i64), C.c_int, C.POINTER(_i64)]),
    ("lbm_mlp_set_weights", C.c_int, [_vp, _fp, C.c_int]),
    ("lbm_mlp_get_weights", C.c_int, [_vp, _fp, C.c_int]),
    ("lbm_alpha_dataset", C.c_int, [_vp, _i64, C.c_uint64, _vp, _vp, _vp]),
    ("lbm_mlp_train", C.c_int, [_vp, _vp, _vp, _i64, C.c_int, C.c_int, C.c_float, C.c_uint64, _fp]),
    ("lbm_mlp_loss_grad", C.c_int, [_vp, _vp, _vp, _i64, _dp, _fp]),
    ("lbm_mlp_forward", C.c_int, [_vp, _vp, _i64, _vp]),
    ("lbm_steps_done", C.c_int, [_vp, C.POINTER(_i64)]),
    ("lbm_sync", C.c_int, [_vp]),
    ("lbm_last_error", C.c_char_p, [_vp]),
    ("lbm_destroy", None, [_vp]),
]
ENTRY_POINTS = [s[0] for s in _SIGS]

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built; run `python -m paper_1311_2404_amd.build`")
        # torch brings its own HIP runtime: let it load first, so that the library binds
        # to the runtime torch's streams and buffers live in (loading the library before
        # torch has ended a process with a segmentation fault)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _err(sim, rc):
    if rc != LBM_OK:
        msg = lib().lbm_last_error(sim)
        raise LbmError(rc, msg.decode() if msg else "error")


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _host64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(t, numel=None, dtype=None):
    """Device pointer of a contiguous CUDA torch tensor, checked for size and dtype."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device buffers must be contiguous CUDA tensors")
    if numel is not None and t.numel() < numel:
        raise ValueError("device buffer holds %d elements, %d needed" % (t.numel(), numel))
    if dtype is not None and t.dtype != dtype:
        raise ValueError("device buffer has dtype %s, %s needed" % (t.dtype, dtype))
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- thin mirrors of the C ABI

def lbm_create(lattice, model, nx, ny, nz, tau, force=None):
    h = C.c_void_p()
    f = _host64(list(force) + [0.0] * (3 - len(force))) if force is not None else None
    _err(None, lib().lbm_create(lattice, model, nx, ny, nz, tau, _d(f), C.byref(h)))
    return h


def lbm_set_storage(sim, storage, layout=LBM_AB, stochastic_round=0):
    _err(sim, lib().lbm_set_storage(sim, storage, layout, int(stochastic_round)))


def lbm_set_pop_layout(sim, kind=LBM_POP_TILED, tile_rows=0, row_pad=0, block_pad=-1, soa_pad=-1):
    _err(sim, lib().lbm_set_pop_layout(sim, kind, tile_rows, row_pad, block_pad, soa_pad))


def lbm_set_mrt_rates(sim, s):
    s = _host64(s)
    _err(sim, lib().lbm_set_mrt_rates(sim, _d(s), s.size))


def lbm_set_elbm(sim, alpha_init=0, tol=1e-10, max_iter=20):
    _err(sim, lib().lbm_set_elbm(sim, alpha_init, tol, max_iter))


def lbm_set_shanchen(sim, G, psi=0):
    _err(sim, lib().lbm_set_shanchen(sim, G, psi))


def lbm_set_free_energy(sim, tau_b, tau_phi, a, kappa, gamma):
    _err(sim, lib().lbm_set_free_energy(sim, tau_b, tau_phi, a, kappa, gamma))


def lbm_set_velocity_bc(sim, u):
    u = _host64(list(u) + [0.0] * (3 - len(u)))
    _err(sim, lib().lbm_set_velocity_bc(sim, _d(u)))


def lbm_set_smagorinsky(sim, cs):
    _err(sim, lib().lbm_set_smagorinsky(sim, cs))


def lbm_set_stream(sim, stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None (null stream)."""
    raw = getattr(stream, "cuda_stream", stream)
    _err(sim, lib().lbm_set_stream(sim, C.c_void_p(raw) if raw else None))


def lbm_set_flags(sim, flags):
    fl = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
    _err(sim, lib().lbm_set_flags(sim, fl.ctypes.data_as(C.POINTER(C.c_uint8))))


def lbm_init_eq(sim, rho, u, df=None):
    rho, u = _host64(rho), _host64(u)
    df = _host64(df) if df is not None else None
    _err(sim, lib().lbm_init_eq(sim, _d(rho), _d(u), _d(df)))


def lbm_set_f(sim, f):
    f = _host64(f)
    _err(sim, lib().lbm_set_f(sim, _d(f)))


def lbm_get_f(sim, out):
    assert out.dtype == np.float64 and out.flags.c_contiguous
    _err(sim, lib().lbm_get_f(sim, _d(out)))
    return out


def lbm_step(sim, n):
    _err(sim, lib().lbm_step(sim, int(n)))


def lbm_macro(sim, rho_out, u_out):
    _err(sim, lib().lbm_macro(sim, _d(rho_out), _d(u_out)))
    return rho_out, u_out


def lbm_macro_device(sim, rho_t, u_t, ncomp, n):
    """rho_t[ncomp][n], u_t[3][n]: torch CUDA tensors, both float64 or both float32."""
    import torch
    dt = torch.float64 if rho_t.dtype == torch.float64 else torch.float32
    _err(sim, lib().lbm_macro_device(sim, _ptr(rho_t, ncomp * n, dt), _ptr(u_t, 3 * n, dt),
                                     int(dt == torch.float64)))


def lbm_diag(sim):
    out = np.zeros(8)
    _err(sim, lib().lbm_diag(sim, _d(out)))
    return out


def lbm_diag_noalloc(sim, out_t):
    """The diagnostics into a CUDA float64 tensor of 8 elements (enqueued, no sync)."""
    import torch
    _err(sim, lib().lbm_diag_noalloc(sim, _ptr(out_t, 8, torch.float64)))


def lbm_elbm_stats(sim, enable=True, reset=False, nbins=32):
    hist = np.zeros(nbins, dtype=np.int64)
    nc = C.c_int64()
    _err(sim, lib().lbm_elbm_stats(sim, int(enable), int(reset), hist.ctypes.data_as(C.POINTER(_i64)), nbins,
                                   C.byref(nc)))
    return hist, nc.value


def lbm_mlp_set_weights(sim, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _err(sim, lib().lbm_mlp_set_weights(sim, p.ctypes.data_as(_fp), p.size))


def lbm_mlp_get_weights(sim, with_norm=True):
    p = np.zeros(MLP_NTOTAL if with_norm else MLP_NPARAM, dtype=np.float32)
    _err(sim, lib().lbm_mlp_get_weights(sim, p.ctypes.data_as(_fp), p.size))
    return p


def mlp_initial_weights(seed):
    """Starting weights for training a new proposal network (1313 values, the layout of
    lbm_mlp_set_weights): Glorot-scaled normal hidden layers, zero biases and a zero
    output layer.  The proposal then starts as the bare series estimate, and training
    (in standardised target units) grows the output layer from zero instead of having
    to cancel a large random one, which BF16 inference weights could not represent."""
    rng = np.random.default_rng(seed)
    h, nin = 32, 6
    w1 = rng.standard_normal((h, nin)) * np.sqrt(2.0 / (h + nin))
    w2 = rng.standard_normal((h, h)) * np.sqrt(1.0 / h)
    return np.concatenate([w1.ravel(), np.zeros(h), w2.ravel(), np.zeros(h), np.zeros(h), [0.0]]).astype(np.float32)


def lbm_alpha_dataset(sim, n, seed, feat_t, alpha_t, valid_t):
    import torch
    _err(sim, lib().lbm_alpha_dataset(sim, int(n), int(seed), _ptr(feat_t, 6 * n, torch.float32),
                                      _ptr(alpha_t, n, torch.float64), _ptr(valid_t, n, torch.uint8)))


def lbm_mlp_train(sim, feat_t, alpha_t, n, epochs, batch, lr, seed):
    import torch
    loss = np.zeros(max(epochs, 1), dtype=np.float32)
    _err(sim, lib().lbm_mlp_train(sim, _ptr(feat_t, 6 * n, torch.float32), _ptr(alpha_t, n, torch.float64), int(n),
                                  epochs, batch, float(lr), int(seed), loss.ctypes.data_as(_fp)))
    return loss[:epochs]


def lbm_mlp_loss_grad(sim, feat_t, alpha_t, n):
    import torch
    loss = C.c_double()
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    _err(sim, lib().lbm_mlp_loss_grad(sim, _ptr(feat_t, 6 * n, torch.float32), _ptr(alpha_t, n, torch.float64),
                                      int(n), C.byref(loss), g.ctypes.data_as(_fp)))
    return loss.value, g


def lbm_mlp_forward(sim, feat_t, n, y_t):
    import torch
    _err(sim, lib().lbm_mlp_forward(sim, _ptr(feat_t, 6 * n, torch.float32), int(n), _ptr(y_t, n, torch.float32)))


def lbm_steps_done(sim):
    v = C.c_int64()
    _err(sim, lib().lbm_steps_done(sim, C.byref(v)))
    return v.value


def lbm_sync(sim):
    _err(sim, lib().lbm_sync(sim))


def lbm_last_error(sim=None):
    m = lib().lbm_last_error(sim)
    return m.decode() if m else ""


def lbm_destroy(sim):
    lib().lbm_destroy(sim)


# ---------------------------------------------------------------- convenience wrapper

class Sim:
    """One simulation handle.  ``stream`` defaults to torch's current stream."""

    def __init__(self, lattice, model, nx, ny, nz, tau, force=None, storage=LBM_F32, layout=LBM_AB,
                 stochastic_round=0, stream="current", pop_layout=None):
        self.lattice, self.model = lattice, model
        self.nx, self.ny, self.nz = nx, ny, nz
        self.q = 9 if lattice == LBM_D2Q9 else 19
        self.d = 2 if lattice == LBM_D2Q9 else 3
        self.ncomp = 2 if model in (LBM_SHANCHEN, LBM_FREE_ENERGY) else 1
        self.n = nx * ny * nz
        self.storage = storage
        self.h = lbm_create(lattice, model, nx, ny, nz, tau, force)
        lbm_set_storage(self.h, storage, layout, stochastic_round)
        if pop_layout is not None:
            lbm_set_pop_layout(self.h, **pop_layout)
        if stream == "current":
            import torch
            if torch.cuda.is_available():
                lbm_set_stream(self.h, torch.cuda.current_stream())
        elif stream is not None:
            lbm_set_stream(self.h, stream)

    @classmethod
    def from_case(cls, case, storage=LBM_F32, layout=LBM_AB, stochastic_round=0, init=True, **kw):
        s = cls(case.lattice, case.model, case.nx, case.ny, case.nz, case.tau, case.force, storage, layout,
                stochastic_round, **kw)
        if case.mrt_rates is not None:
            lbm_set_mrt_rates(s.h, case.mrt_rates)
        if case.model == LBM_SHANCHEN:
            lbm_set_shanchen(s.h, case.G, case.psi)
        if case.model == LBM_SMAGORINSKY:
            lbm_set_smagorinsky(s.h, case.cs_smag)
        if case.model == LBM_FREE_ENERGY:
            fe = case.fe
            lbm_set_free_energy(s.h, fe["tau_b"], fe["tau_phi"], fe["a"], fe["kappa"], fe["gamma"])
        if case.flags is not None:
            lbm_set_flags(s.h, case.flags)
        if any(case.u_bc):
            lbm_set_velocity_bc(s.h, case.u_bc)
        if init:
            s.init_eq(case.rho, case.u, case.df)
        return s

    def init_eq(self, rho, u, df=None):
        lbm_init_eq(self.h, _host64(rho, (self.ncomp, self.n)), _host64(u, (-1, self.n))[: self.d],
                    None if df is None else _host64(df, (self.ncomp, self.q, self.n)))

    def set_f(self, f):
        lbm_set_f(self.h, _host64(f, (self.ncomp, self.q, self.n)))

    def get_f(self):
        return lbm_get_f(self.h, np.zeros((self.ncomp, self.q, self.n)))

    def step(self, n=1):
        lbm_step(self.h, n)

    def macro(self):
        return lbm_macro(self.h, np.zeros((self.ncomp, self.n)), np.zeros((3, self.n)))

    def diag(self):
        return lbm_diag(self.h)

    def macro_device(self, rho_t, u_t):
        lbm_macro_device(self.h, rho_t, u_t, self.ncomp, self.n)

    def sync(self):
        lbm_sync(self.h)

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
