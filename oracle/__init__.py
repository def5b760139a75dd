"""ctypes front end of the FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are its only users.  The HIP library never
imports, links or calls it, and it shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "oracle.c")

D2Q9, D3Q19 = 0, 1
BGK, MRT, ELBM, SHANCHEN, REG, SMAG, FREE_ENERGY = 0, 1, 2, 3, 4, 5, 6
MLP_NPARAM = 1313
MLP_NTOTAL = 1325  # weights + input normalisation mu[6], isd[6]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("model", C.c_int),
                ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("tau", C.c_double), ("g", C.c_double * 3), ("s", C.c_double * 19),
                ("alpha_init", C.c_int), ("alpha_tol", C.c_double), ("alpha_maxit", C.c_int),
                ("mlp", C.POINTER(C.c_double)), ("G", C.c_double), ("psi", C.c_int),
                ("cs_smag", C.c_double), ("u_bc", C.c_double * 3),
                ("tau_b", C.c_double), ("tau_phi", C.c_double), ("fe_a", C.c_double), ("fe_kappa", C.c_double),
                ("fe_gamma", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("newton_hist", C.c_int64 * 32), ("nonconverged", C.c_int64), ("nodes", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        P = C.POINTER(Params)
        L.orc_q.argtypes = [C.c_int]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_tables.argtypes = [C.c_int, ip, dp, ip]
        L.orc_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_feq_entropic.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_mrt_matrix.argtypes = [C.c_int, dp]
        L.orc_H.argtypes = [C.c_int, dp]
        L.orc_H.restype = C.c_double
        L.orc_alpha.argtypes = [C.c_int, dp, dp, C.c_int, dp, C.c_double, C.c_double, C.c_int, ip, ip]
        L.orc_alpha.restype = C.c_double
        L.orc_alpha_features.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, dp]
        L.orc_mlp_forward.argtypes = [dp, dp, C.c_int64, dp]
        L.orc_mlp_loss_grad.argtypes = [dp, dp, dp, C.c_int64, dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_collide_node.argtypes = [P, dp, dp]
        L.orc_collide_node_sc.argtypes = [P, dp, dp, dp]
        L.orc_init_eq.argtypes = [P, dp, dp, dp, dp]
        L.orc_run.argtypes = [P, C.c_void_p, dp, C.c_int, C.POINTER(Stats)]
        L.orc_macro.argtypes = [P, C.c_void_p, dp, dp, dp]
        L.orc_fe_equilibria.argtypes = [P, C.c_double, C.c_double, dp, dp, C.c_double, dp, dp]
        L.orc_fe_equilibria.restype = None
        L.orc_fe_stencil.argtypes = [P, C.c_void_p, dp, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_fe_stencil.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def q_of(lattice):
    return 9 if lattice == D2Q9 else 19


def tables(lattice):
    q = q_of(lattice)
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    lib().orc_tables(lattice, e.ctypes.data_as(C.POINTER(C.c_int)), _dp(w),
                     opp.ctypes.data_as(C.POINTER(C.c_int)))
    return e, w, opp


def feq(lattice, rho, u):
    out = np.zeros(q_of(lattice))
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    lib().orc_feq(lattice, rho, _dp(uu), _dp(out))
    return out


def feq_entropic(lattice, rho, u):
    out = np.zeros(q_of(lattice))
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    lib().orc_feq_entropic(lattice, rho, _dp(uu), _dp(out))
    return out


def mrt_matrix(lattice):
    q = q_of(lattice)
    M = np.zeros((q, q))
    lib().orc_mrt_matrix(lattice, _dp(M))
    return M


def H(lattice, f):
    return lib().orc_H(lattice, _dp(_f64(f)))


def alpha(lattice, f, fe, init=0, mlp=None, vsq=0.0, tol=1e-10, maxit=20):
    it, conv = C.c_int(), C.c_int()
    mp = _dp(_f64(mlp)) if mlp is not None else None
    fa, fea = _f64(f), _f64(fe)
    a = lib().orc_alpha(lattice, _dp(fa), _dp(fea), init, mp, vsq, tol, maxit,
                        C.byref(it), C.byref(conv))
    return a, it.value, bool(conv.value)


def alpha_features(lattice, f, fe, rho, vsq):
    out = np.zeros(6)
    lib().orc_alpha_features(lattice, _dp(_f64(f)), _dp(_f64(fe)), rho, vsq, _dp(out))
    return out


def with_identity_norm(weights):
    """1313 network weights -> 1325 parameters with mu = 0, isd = 1."""
    return np.concatenate([_f64(weights)[:MLP_NPARAM], np.zeros(6), np.ones(6)])


def mlp_forward(params, x):
    """params: 1325 values (or 1313 weights, identity normalisation); x raw features."""
    params = _f64(params)
    if params.size == MLP_NPARAM:
        params = with_identity_norm(params)
    x = _f64(x).reshape(-1, 6)
    y = np.zeros(x.shape[0])
    lib().orc_mlp_forward(_dp(_f64(params)), _dp(x), x.shape[0], _dp(y))
    return y


def mlp_loss_grad(params, x, t):
    params = _f64(params)
    if params.size == MLP_NPARAM:
        params = with_identity_norm(params)
    x = _f64(x).reshape(-1, 6)
    t = _f64(t)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_dp(_f64(params)), _dp(x), _dp(t), x.shape[0], _dp(g))
    return loss, g


class Oracle:
    """One simulation held by the oracle: parameters plus the population array."""

    def __init__(self, lattice, model, nx, ny, nz, tau, force=(0.0, 0.0, 0.0), mrt_rates=None,
                 alpha_init=0, alpha_tol=1e-10, alpha_maxit=20, mlp=None, G=0.0, psi=0, cs_smag=0.1,
                 u_bc=(0.0, 0.0, 0.0), fe=None):
        self.p = Params()
        self.p.lattice, self.p.model = lattice, model
        self.p.nx, self.p.ny, self.p.nz = nx, ny, nz
        self.p.tau = tau
        for a in range(3):
            self.p.g[a] = float(force[a]) if a < len(force) else 0.0
        if mrt_rates is not None:
            for k, s in enumerate(mrt_rates):
                self.p.s[k] = float(s)
        self.p.alpha_init, self.p.alpha_tol, self.p.alpha_maxit = alpha_init, alpha_tol, alpha_maxit
        self._mlp = _f64(mlp) if mlp is not None else None
        self.p.mlp = _dp(self._mlp) if mlp is not None else None
        self.p.G, self.p.psi = G, psi
        self.p.cs_smag = cs_smag
        for a in range(3):
            self.p.u_bc[a] = float(u_bc[a]) if a < len(u_bc) else 0.0
        if fe is not None:
            self.p.tau_b, self.p.tau_phi = fe["tau_b"], fe["tau_phi"]
            self.p.fe_a, self.p.fe_kappa, self.p.fe_gamma = fe["a"], fe["kappa"], fe["gamma"]
        self.q = q_of(lattice)
        self.n = nx * ny * nz
        self.ncomp = 2 if model in (SHANCHEN, FREE_ENERGY) else 1
        self.f = np.zeros((self.ncomp, self.q, self.n))
        self.flags = None
        self.stats = Stats()

    @classmethod
    def from_case(cls, case, **kw):
        kw.setdefault("cs_smag", case.cs_smag)
        kw.setdefault("u_bc", case.u_bc)
        kw.setdefault("fe", case.fe)
        o = cls(case.lattice, case.model, case.nx, case.ny, case.nz, case.tau, case.force,
                case.mrt_rates, G=case.G, psi=case.psi, **kw)
        if case.flags is not None:
            o.set_flags(case.flags)
        o.init_eq(case.rho, case.u, case.df)
        return o

    def set_flags(self, flags):
        self.flags = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)

    def init_eq(self, rho, u, df=None):
        rho = _f64(rho).reshape(self.ncomp, self.n)
        uu = np.zeros((3, self.n))
        u = _f64(u).reshape(-1, self.n)
        uu[:u.shape[0]] = u
        dfa = _f64(df).reshape(self.ncomp, self.q, self.n) if df is not None else None
        rc = lib().orc_init_eq(C.byref(self.p), _dp(rho), _dp(uu), _dp(dfa) if dfa is not None else None,
                               _dp(self.f))
        if rc:
            raise ValueError("oracle init rejected the parameters (%d)" % rc)

    def set_f(self, f):
        self.f = _f64(f).reshape(self.ncomp, self.q, self.n).copy()

    def collide_node(self, fnode):
        out = np.zeros(self.q)
        lib().orc_collide_node(C.byref(self.p), _dp(_f64(fnode)), _dp(out))
        return out

    def collide_node_sc(self, f2, psi_nb):
        """f2[2][q] populations at x, psi_nb[2][q] pseudopotential at x + e_i."""
        out = np.zeros((2, self.q))
        lib().orc_collide_node_sc(C.byref(self.p), _dp(_f64(f2)), _dp(_f64(psi_nb)), _dp(out))
        return out

    def run(self, steps):
        fl = self.flags.ctypes.data if self.flags is not None else None
        rc = lib().orc_run(C.byref(self.p), fl, _dp(self.f), steps, C.byref(self.stats))
        if rc:
            raise ValueError("oracle run rejected the parameters (%d)" % rc)
        return self

    def macro(self):
        rho = np.zeros((self.ncomp, self.n))
        u = np.zeros((3, self.n))
        fl = self.flags.ctypes.data if self.flags is not None else None
        rc = lib().orc_macro(C.byref(self.p), fl, _dp(self.f), _dp(rho), _dp(u))
        if rc:
            raise ValueError("oracle macro rejected the parameters (%d)" % rc)
        return rho, u

    def fe_equilibria(self, rho, phi, u, grad, lap):
        fe, ge = np.zeros(self.q), np.zeros(self.q)
        lib().orc_fe_equilibria(C.byref(self.p), rho, phi, _dp(_f64(list(u) + [0.0] * (3 - len(u)))),
                                _dp(_f64(list(grad) + [0.0] * (3 - len(grad)))), lap, _dp(fe), _dp(ge))
        return fe, ge

    def fe_stencil(self, phi, x, y, z, flags=None):
        grad, lap = np.zeros(3), C.c_double()
        fl = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1) if flags is not None else None
        ph = _f64(phi).reshape(-1)
        lib().orc_fe_stencil(C.byref(self.p), fl.ctypes.data if fl is not None else None, _dp(ph), x, y, z,
                             _dp(grad), C.byref(lap))
        return grad, lap.value

    def newton_hist(self):
        return np.array(self.stats.newton_hist[:]), self.stats.nonconverged, self.stats.nodes


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))
