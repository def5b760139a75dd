"""The free-energy binary model: HIP path vs the FP64 oracle through the C ABI.

FP64 storage within 1e-12 relative L2 of the oracle on f - w and g - w, u, rho and phi,
on 2-D and 3-D periodic boxes with random order parameter and a body force, and on the
binary Poiseuille channel with half-way bounce-back walls; FP32 on the channel's steady
profile; AA and AB and every population layout bit for bit.
"""
import numpy as np
import pytest

import synthetic as S
from test_gpu_parity import _POP_LAYOUTS, check_f64, gpu_run, oracle_run, rel

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")

FE = {"tau_b": 0.8, "tau_phi": 0.9, "a": 0.04, "kappa": 0.03, "gamma": 1.5}


def fe_random(lattice, nx, ny, nz, seed=5, force=(1e-5, -2e-5, 0.0)):
    d = 2 if lattice == S.D2Q9 else 3
    rho, u = S.random_state_fields(nx, ny, nz, d, seed, 0.02, 0.01)
    phi = S.uniform_pm(seed, 5, (nx * ny * nz,), 0.6)
    return S.Case("fe_random", lattice, S.FREE_ENERGY, nx, ny, nz, 0.7, force, 0, None, np.vstack([rho, phi]), u,
                  fe=FE)


@pytest.mark.parametrize("lattice,shape", [(S.D2Q9, (130, 37, 1)), (S.D3Q19, (70, 13, 6))])
def test_free_energy_random_fp64(lattice, shape):
    check_f64(fe_random(lattice, *shape), 40)


def test_binary_poiseuille_fp64():
    # force 1e-5: a flow started from rest by a smaller force is, after 300 steps, small
    # against the rounding unit of f ~ 0.2 that both sides carry
    c = S.binary_poiseuille(nx=70, ny=42, g=1e-5)
    check_f64(c, 300)


def test_binary_poiseuille_fp32_steady_profile():
    """FP32 compute to the steady state (60 000 steps) against the oracle's FP64 run.  The
    force adds ~1e-7 per step to f populations of ~0.1, a few units in the last place of a
    plain FP32 f: plain storage ends 5.5e-4 to 7.7e-4 off (the figure follows the rounding
    pattern of the compiled step), the shifted form (f - w stored) 5.6e-5.  The rest is the
    order parameter: phi = +-1 in the bulk is held to the FP32 unit of 1 (6e-8), and the
    steady profile depends on where the viscosity jump sits.  (Storing g - w instead of g
    gives 4.5e-6 here but 1e-4 on the small-phi spinodal state, where plain g gives 1e-6;
    the plain form is kept.)  Bar: 1e-4, and 5x better than plain."""
    c = S.binary_poiseuille(nx=4, ny=42, g=1e-6)
    _, _, uo = oracle_run(c, 60000)
    errs = {}
    for st in (P.LBM_F32S, P.LBM_F32):
        for lay in (P.LBM_AB, P.LBM_AA):
            _, _, ug = gpu_run(c, 60000, st, lay)
            errs[(st, lay)] = rel(ug, uo)
            print("binary Poiseuille %s layout %d: velocity rel L2 %.3g" % (P.STORAGE_NAMES[st], lay, errs[(st, lay)]))
    for lay in (P.LBM_AB, P.LBM_AA):
        assert errs[(P.LBM_F32S, lay)] <= 1e-4
        assert errs[(P.LBM_F32, lay)] > 5 * errs[(P.LBM_F32S, lay)]


@pytest.mark.parametrize("storage", [P.LBM_F64, P.LBM_F32, P.LBM_F32S])
def test_free_energy_aa_equals_ab_bitwise(storage):
    c = S.binary_poiseuille(nx=40, ny=22, g=1e-6)
    for steps in (1, 6, 7):
        fa, ra, ua = gpu_run(c, steps, storage, P.LBM_AB)
        fb, rb, ub = gpu_run(c, steps, storage, P.LBM_AA)
        assert np.array_equal(fa, fb) and np.array_equal(ua, ub) and np.array_equal(ra, rb), (storage, steps)


def test_free_energy_population_layouts_agree_bitwise():
    c = fe_random(S.D3Q19, 37, 12, 6)
    for st in (P.LBM_F64, P.LBM_F32):
        for lay in (P.LBM_AB, P.LBM_AA):
            ref = gpu_run(c, 5, st, lay)
            for pl in _POP_LAYOUTS:
                got = gpu_run(c, 5, st, lay, pop_layout=pl)
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), (st, lay, pl)
