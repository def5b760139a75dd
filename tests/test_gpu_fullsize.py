"""The measured configurations at their full sizes, in the benchmark's launch setup.

The oracle cannot run these lattices for thousands of steps, so parity is checked on
sampled nodes after one step (the oracle's single-node collision applied to the
GPU's own pre-step state, compared with where the GPU's post-collision values landed),
and whole runs are checked through properties that hold at any size: the
Navier-Stokes kinetic-energy law, conservation of mass and momentum, and the error of
each storage format against the FP64 run of the same kernel (itself matched to the
oracle to 1e-12 in the parity tests).
"""
import os

import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")

_CACHE = {}
NSAMPLE = 3000


def c2_case():
    if "c2" not in _CACHE:
        _CACHE["c2"] = S.c2_taylor_green(n=256, steps=1000)
    return _CACHE["c2"]


def sample_nodes(n_nodes, seed, k=NSAMPLE):
    return np.random.default_rng(seed).choice(n_nodes, size=k, replace=False)


def neighbours(case, nodes, e):
    x = nodes % case.nx
    y = (nodes // case.nx) % case.ny
    z = nodes // (case.nx * case.ny)
    out = []
    for i in range(len(e)):
        out.append(((x + e[i, 0]) % case.nx) + case.nx * (((y + e[i, 1]) % case.ny)
                                                           + case.ny * ((z + e[i, 2]) % case.nz)))
    return np.stack(out)  # [q][k]


def one_step_sampled(case, storage, seed=0, elbm=None, layout=P.LBM_AB):
    """GPU state before and after one step, plus the oracle's post-collision values at
    sampled nodes computed from the GPU's pre-step state."""
    s = P.Sim.from_case(case, storage, layout)
    if elbm is not None:
        P.lbm_set_elbm(s.h, *elbm)
    f0 = s.get_f()
    s.step(1)
    f1 = s.get_f()
    s.close()
    e, w, _ = oracle.tables(case.lattice)
    nodes = sample_nodes(case.n, seed)
    nb = neighbours(case, nodes, e)
    o = oracle.Oracle(case.lattice, case.model, case.nx, case.ny, case.nz, case.tau, case.force, case.mrt_rates,
                      G=case.G, psi=case.psi)
    flags = case.flags.reshape(-1) if case.flags is not None else np.zeros(case.n, np.uint8)
    if case.model == S.SHANCHEN:
        rho = f0.sum(axis=1)  # psi = rho at every node
        want = np.empty((2, 19, len(nodes)))
        got = np.empty_like(want)
        for k, node in enumerate(nodes):
            want[:, :, k] = o.collide_node_sc(f0[:, :, node], rho[:, nb[:, k]])
            got[:, :, k] = f1[:, np.arange(19), nb[:, k]]
        return got - w[None, :, None], want - w[None, :, None]
    want = np.empty((len(w), len(nodes)))
    got = np.empty_like(want)
    for k, node in enumerate(nodes):
        if flags[node] == 1:
            want[:, k] = f0[0, [int(i) for i in oracle.tables(case.lattice)[2]], node]
        else:
            want[:, k] = o.collide_node(f0[0, :, node])
        got[:, k] = f1[0, np.arange(len(w)), nb[:, k]]
    return got - w[:, None], want - w[:, None]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------- C2: D3Q19 BGK 256^3 vortex

@pytest.mark.parametrize("storage,tol,layout", [(P.LBM_F64, 1e-12, P.LBM_AB), (P.LBM_F32, 3e-6, P.LBM_AB),
                                                (P.LBM_F32, 3e-6, P.LBM_AA), (P.LBM_F32S, 3e-6, P.LBM_AB),
                                                (P.LBM_BF16S, 8e-3, P.LBM_AB), (P.LBM_F16S, 1e-3, P.LBM_AB)])
def test_c2_fullsize_one_step_sampled(storage, tol, layout):
    got, want = one_step_sampled(c2_case(), storage, layout=layout)
    assert rel(got, want) <= tol, (P.STORAGE_NAMES[storage], rel(got, want))


def test_c2_fullsize_1000_steps_decay_and_conservation():
    """FP32, 1000 steps: KE ratio within 5e-3 of exp(-6 nu k^2 t) (the 3-D vortex is not an
    exact Navier-Stokes solution; nonlinear and lattice terms are a few 1e-3), mass and
    momentum conserved, and the velocity within 1e-5 (relative L2) of the FP64 run."""
    c = c2_case()
    runs = {}
    for st in (P.LBM_F64, P.LBM_F32):
        s = P.Sim.from_case(c, st, P.LBM_AB)
        d0 = s.diag()
        s.step(1000)
        d1 = s.diag()
        runs[st] = s.macro()[1]
        s.close()
        assert abs(d1[0] - d0[0]) <= (1e-13 if st == P.LBM_F64 else 1e-7) * d0[0]
        assert np.abs(d1[2:5] - d0[2:5]).max() <= 1e-8 * d0[0] * 0.04
        k = 2 * np.pi / 256
        law = np.exp(-6 * c.extra["nu"] * k * k * 1000)
        assert abs(d1[5] / d0[5] - law) <= 5e-3 * law
    assert rel(runs[P.LBM_F32], runs[P.LBM_F64]) <= 1e-5
    # the timed configuration streams in place (AA): the same 1000 steps, bit for bit
    s = P.Sim.from_case(c, P.LBM_F32, P.LBM_AA)
    s.step(1000)
    u_aa = s.macro()[1]
    s.close()
    assert np.array_equal(u_aa, runs[P.LBM_F32])


C2_REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_taylor_green_256.npz")


@pytest.mark.parametrize("storage,layout,tol", [(P.LBM_F64, P.LBM_AA, 1e-12), (P.LBM_F64, P.LBM_AB, 1e-12),
                                                (P.LBM_F32, P.LBM_AB, 1e-5), (P.LBM_F32, P.LBM_AA, 1e-5),
                                                (P.LBM_F32S, P.LBM_AA, 1e-5)])
def test_c2_fullsize_1000_steps_vs_oracle(storage, layout, tol):
    """The metric's configuration itself, 256^3 for its 1000 steps, against the FP64
    oracle's own run of it (stored by tests/golden/make_c2_reference.py, which calls
    only the oracle): the velocity at 8192 sampled nodes, and over the whole lattice the
    per-plane sums of |u|^2 and of (rho - 1)^2 and the kinetic energy.  FP64 storage:
    1e-12 relative on velocity (and density); FP32 compute: 1e-5 on velocity."""
    ref = np.load(C2_REF)
    c = c2_case()
    s = P.Sim.from_case(c, storage, layout)
    s.step(int(ref["steps"]))
    rho, u = s.macro()
    s.close()
    n = int(ref["n"])
    nodes = ref["nodes"]
    err_u = rel(u[:, nodes], ref["u"])
    pu2 = (u.reshape(3, n, n * n) ** 2).sum(axis=2).sum(axis=0)
    err_plane = float(np.abs(pu2 / ref["plane_u2"].sum(axis=0) - 1.0).max())
    ke = 0.5 * float((u * u).sum()) / n ** 3
    print("%s layout %d: sampled velocity %.2e, per-plane |u|^2 %.2e, KE %.2e" % (
        P.STORAGE_NAMES[storage], layout, err_u, err_plane, abs(ke / ref["ke"][1] - 1)))
    assert err_u <= tol
    # |u|^2 is quadratic in u: a relative velocity error e moves it by at most ~2e
    assert err_plane <= 2 * tol
    assert abs(ke / ref["ke"][1] - 1.0) <= 2 * tol
    if storage == P.LBM_F64:
        # rho - 1 ~ 1e-3 (the vortex's pressure); floor of 1e-15 of rho per node
        dr = rho[0, nodes] - ref["rho"]
        assert np.linalg.norm(dr) <= tol * np.linalg.norm(ref["rho"] - 1) + 1e-15 * np.linalg.norm(ref["rho"])
        pr2 = ((rho[0].reshape(n, n * n) - 1.0) ** 2).sum(axis=1)
        assert np.abs(pr2 / ref["plane_drho2"] - 1.0).max() <= 2 * tol + 1e-12


# ----------------------------------------------------------- C3: D3Q19 MRT duct 128x128x512

def c3_case():
    if "c3" not in _CACHE:
        _CACHE["c3"] = S.c3_duct(128, 128, 512, steps=5000)
    return _CACHE["c3"]


def test_c3_fullsize_one_step_sampled_fp64():
    """From a developed random flow so that the comparison is not at the rounding floor."""
    c = c3_case()
    c2 = S.Case(c.name, c.lattice, c.model, c.nx, c.ny, c.nz, c.tau, c.force, 1, c.flags,
                *S.random_state_fields(c.nx, c.ny, c.nz, 3, 5, 0.04, 0.02), mrt_rates=c.mrt_rates)
    got, want = one_step_sampled(c2, P.LBM_F64, seed=3)
    assert rel(got, want) <= 1e-12


def test_c3_fullsize_5000_steps_storage_errors():
    """Velocity after the configuration's 5000 steps for each storage, against the FP64
    run (FP64 matches the oracle to 1e-12).  The bounds are the stated errors with a
    margin; plain FP32 and round-to-nearest BF16 lose the small per-step force
    increment (it falls below half an ulp of the stored f or f - w)."""
    c = c3_case()
    u = {}
    for st, sr in [(P.LBM_F64, 0), (P.LBM_F32, 0), (P.LBM_F32S, 0), (P.LBM_BF16S, 1), (P.LBM_F16S, 0),
                   (P.LBM_F16S, 1)]:
        s = P.Sim.from_case(c, st, P.LBM_AA, sr)
        s.step(c.steps)
        d = s.diag()
        assert abs(d[0] - c.n) <= 1e-4 * c.n
        u[(st, sr)] = s.macro()[1]
        s.close()
    ref = u[(P.LBM_F64, 0)]
    assert 4.5e-3 < ref[2].max() < 5.5e-3  # plug-flow core velocity ~ g t at 5000 steps
    err = {k: rel(v, ref) for k, v in u.items()}
    print({"%s_sr%d" % (P.STORAGE_NAMES[k[0]], k[1]): "%.3e" % v for k, v in err.items()})
    # FP32 compute misses the 1e-5 target here (measured 4.6e-5 plain, 3.3e-5 shifted).  The
    # bounds are about twice the measured errors, so a regression shows: BF16 with stochastic
    # rounding 1.35e-3, F16 3.1e-3 to 4.0e-3 (round to nearest moves with the arithmetic's
    # rounding order), F16 with stochastic rounding 1.77e-4
    assert err[(P.LBM_F32S, 0)] <= 7e-5, err
    assert err[(P.LBM_F32, 0)] <= 1e-4, err
    assert err[(P.LBM_BF16S, 1)] <= 3e-3, err
    assert err[(P.LBM_F16S, 0)] <= 8e-3, err
    assert err[(P.LBM_F16S, 1)] <= 4e-4, err


# ----------------------------------------------------------- C4: D3Q19 ELBM 256^3

def test_c4_fullsize_one_step_sampled():
    """ELBM at 256^3 with seeded noise so that the alpha Newton solve runs at every node."""
    c = S.c4_elbm_taylor_green(n=256)
    c.df = S.uniform_pm(7, 0, (1, 19, c.n), 2e-4)
    for st, tol in [(P.LBM_F64, 1e-12), (P.LBM_F32, 1e-5)]:
        got, want = one_step_sampled(c, st, seed=5, elbm=(0, 1e-10, 20))
        assert rel(got, want) <= tol, (st, rel(got, want))


def test_c4_fullsize_1000_steps_fp32_vs_fp64():
    """1000 steps of the 256^3 entropic vortex with FP32 storage and arithmetic (FP64 alpha
    solve) against the same run in FP64, which the parity tests tie to the oracle: velocity
    within 1e-5 relative L2, every alpha solve converged, mass conserved.  Where alpha
    departs from 2 the entropic step dissipates more than nu = 1e-5 alone (whose energy
    law gives a 4e-5 decrease), so the energy is compared between the two runs."""
    c = S.c4_elbm_taylor_green(n=256)
    res = {}
    for st in (P.LBM_F32, P.LBM_F64):
        s = P.Sim.from_case(c, st, P.LBM_AB)
        P.lbm_elbm_stats(s.h, enable=True, reset=True)
        d0 = s.diag()
        s.step(1000)
        d1 = s.diag()
        hist, nonconv = P.lbm_elbm_stats(s.h, enable=False)
        u = s.macro()[1]
        s.close()
        print("storage %d: KE ratio %.6e, mean Newton iterations %.3f" % (
            st, d1[5] / d0[5], (np.arange(len(hist)) * hist).sum() / hist.sum()))
        assert hist.sum() == 1000 * c.n and nonconv == 0, (st, nonconv)
        assert d1[6] == 0 and abs(d1[0] - d0[0]) <= 1e-7 * d0[0]
        res[st] = (u, d1[5] / d0[5])
    u32, u64 = res[P.LBM_F32][0], res[P.LBM_F64][0]
    err = np.linalg.norm(u32 - u64) / np.linalg.norm(u64)
    print("FP32 vs FP64 velocity rel L2 after 1000 steps: %.3e" % err)
    assert err <= 1e-5
    # the energy is quadratic in u: a relative velocity error e moves it by at most ~2e
    assert abs(res[P.LBM_F32][1] - res[P.LBM_F64][1]) <= 2e-5 * res[P.LBM_F64][1]


# ----------------------------------------------------------- C5: Shan-Chen 384^3

def c5_case():
    if "c5" not in _CACHE:
        _CACHE["c5"] = S.c5_shan_chen(n=384, steps=2000)
    return _CACHE["c5"]


def test_c5_fullsize_one_step_sampled_fp32():
    """Plain FP32 storage rounds f ~ w to 2^-24 relative, 4e-9 absolute, against deviations
    f - w ~ 5e-4 here: the bound is that storage rounding, not the arithmetic."""
    got, want = one_step_sampled(c5_case(), P.LBM_F32, seed=9)
    assert rel(got, want) <= 2e-5


def test_c5_fullsize_2000_steps_conservation():
    """Per-component mass conserved over 2000 steps with shifted FP32 storage, and total
    momentum to the FP32 rounding bound below.  G = 0.9 lies above this scheme's separation threshold for psi = rho at
    rho_A = rho_B = 1 (the oracle puts it between G = 0.5 and 0.6), so the +-1%
    perturbations grow into separated domains: rho_A ends with a spread of order one
    while both densities stay positive.  (Plain FP32 storage, which rounds f ~ w to
    2^-24 relative, drifts the mass by ~1e-5 over the same run once the interfaces form.)"""
    c = c5_case()
    s = P.Sim.from_case(c, P.LBM_F32S, P.LBM_AA)
    rho0, _ = s.macro()
    s.step(c.steps)
    rho1, u1 = s.macro()
    s.close()
    m0, m1 = rho0.sum(axis=1), rho1.sum(axis=1)
    np.testing.assert_allclose(m1, m0, rtol=1e-7)
    # Total momentum is zero in exact arithmetic (the pair forces cancel between nodes).
    # In FP32 their rounding does not, and along flat interfaces, where many nodes share
    # one state, it adds up coherently instead of as a random walk: the mean velocity
    # reaches ~4e-8 after 2000 steps.
    p = (rho1.sum(0) * u1).sum(axis=1)
    print("mean velocity %s, rms velocity %.3e" % (p / m0.sum(), np.sqrt((u1 ** 2).sum(0).mean())))
    assert np.abs(p).max() <= 2e-7 * m0.sum()
    assert rho1.min() > 0.0 and np.isfinite(u1).all()
    assert rho1[0].std() > 0.3 > 10 * rho0[0].std()
