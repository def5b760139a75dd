"""Equilibrium velocity nodes (the lid of the cavity): HIP path vs the FP64 oracle.

FP64 storage within 1e-12 relative L2 of the oracle on f - w, u and rho (the lid nodes'
macroscopic output included), for every model that takes velocity nodes, on 2-D and 3-D
cavities whose sides are not multiples of the workgroup width; FP32 within the stated
velocity bound; AA and AB and every population layout bit for bit.
"""
import numpy as np
import pytest

import synthetic as S
from test_gpu_parity import _POP_LAYOUTS, check_f64, gpu_run, oracle_run, rel

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")


def cavity(lattice, model, nx, ny, nz, tau=0.58, u_lid=0.06):
    d = 2 if lattice == S.D2Q9 else 3
    rho, u = S.rest_fields(nx, ny, nz, d)
    if lattice == S.D2Q9:
        fl = np.zeros((1, ny, nx), np.uint8)
        fl[:, :, 0] = S.VELOCITY
        fl[:, :, nx - 1] = S.WALL
        fl[:, 0, :] = S.WALL
        fl[:, ny - 1, :] = S.WALL
    else:
        fl = S.cavity_flags(nx, ny, nz)
    rates = None
    if model == S.MRT:
        rates = (S.mrt_rates_d2q9 if lattice == S.D2Q9 else S.mrt_rates_d3q19)(1 / tau, 1.2)
    return S.Case("cavity", lattice, model, nx, ny, nz, tau, (0.0, 0.0, 0.0), 0, fl, rho, u,
                  mrt_rates=rates, cs_smag=0.2, u_bc=(0.0, u_lid, 0.0))


@pytest.mark.parametrize("model", [S.BGK, S.MRT, S.REG, S.SMAG])
@pytest.mark.parametrize("lattice,shape", [(S.D2Q9, (130, 37, 1)), (S.D3Q19, (34, 21, 18)),
                                           (S.D2Q9, (256, 21, 1)), (S.D3Q19, (256, 9, 7)), (S.D3Q19, (62, 12, 7))])
def test_cavity_fp64(model, lattice, shape):
    """Rows of 256 and 62 nodes take the AB and AA odd steps that shift along x through LDS."""
    check_f64(cavity(lattice, model, *shape), 60)


def test_cavity_fp32_velocity():
    """FP32 compute, plain and shifted FP32 storage, 600 steps of a 40^3 cavity at
    Re ~ 100 (developed corner vortices), AB and AA."""
    c = S.lid_driven_cavity(40, S.BGK, re=100.0, u_lid=0.05)
    _, _, uo = oracle_run(c, 600)
    for st in (P.LBM_F32, P.LBM_F32S):
        for lay in (P.LBM_AB, P.LBM_AA):
            _, _, ug = gpu_run(c, 600, st, lay)
            err = rel(ug, uo)
            print("storage %s layout %d: velocity rel L2 %.3g" % (P.STORAGE_NAMES[st], lay, err))
            assert err <= 1e-5, (st, lay, err)


@pytest.mark.parametrize("storage", [P.LBM_F64, P.LBM_F32, P.LBM_BF16S])
def test_cavity_aa_equals_ab_bitwise(storage):
    c = cavity(S.D3Q19, S.BGK, 40, 11, 9)
    for steps in (1, 6, 7):
        fa, ra, ua = gpu_run(c, steps, storage, P.LBM_AB)
        fb, rb, ub = gpu_run(c, steps, storage, P.LBM_AA)
        assert np.array_equal(fa, fb) and np.array_equal(ua, ub) and np.array_equal(ra, rb), (storage, steps)


def test_cavity_population_layouts_agree_bitwise():
    c = cavity(S.D3Q19, S.SMAG, 37, 12, 6)
    for st in (P.LBM_F64, P.LBM_F32):
        for lay in (P.LBM_AB, P.LBM_AA):
            ref = gpu_run(c, 5, st, lay)
            for pl in _POP_LAYOUTS:
                got = gpu_run(c, 5, st, lay, pop_layout=pl)
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), (st, lay, pl)


def halfway_channel(lattice, model, nx, ny, nz, tau=0.6, force=(2e-5, 0.0, 0.0), seed=3):
    """Channel along x with dry walls on y = 0, ny - 1 and half-way bounce-back nodes on
    y = 1, ny - 2, from a seeded random state."""
    d = 2 if lattice == S.D2Q9 else 3
    rho, u = S.random_state_fields(nx, ny, nz, d, seed, 0.03, 0.01)
    fl = np.zeros((nz, ny, nx), np.uint8)
    fl[:, 0, :] = S.WALL
    fl[:, ny - 1, :] = S.WALL
    fl[:, 1, :] = S.HALFWAY
    fl[:, ny - 2, :] = S.HALFWAY
    rates = None
    if model == S.MRT:
        rates = (S.mrt_rates_d2q9 if lattice == S.D2Q9 else S.mrt_rates_d3q19)(1 / tau, 1.2)
    if model == S.REG:
        force = (0.0, 0.0, 0.0)
    return S.Case("halfway", lattice, model, nx, ny, nz, tau, force, 0, fl, rho, u, mrt_rates=rates, cs_smag=0.2)


@pytest.mark.parametrize("model", [S.BGK, S.MRT, S.REG, S.SMAG])
@pytest.mark.parametrize("lattice,shape", [(S.D2Q9, (130, 19, 1)), (S.D3Q19, (70, 13, 6))])
def test_halfway_channel_fp64(model, lattice, shape):
    check_f64(halfway_channel(lattice, model, *shape), 60)


@pytest.mark.parametrize("storage", [P.LBM_F64, P.LBM_F32, P.LBM_BF16S])
def test_halfway_aa_equals_ab_bitwise(storage):
    c = halfway_channel(S.D3Q19, S.BGK, 40, 11, 9)
    for steps in (1, 6, 7):
        fa, ra, ua = gpu_run(c, steps, storage, P.LBM_AB)
        fb, rb, ub = gpu_run(c, steps, storage, P.LBM_AA)
        assert np.array_equal(fa, fb) and np.array_equal(ua, ub) and np.array_equal(ra, rb), (storage, steps)
