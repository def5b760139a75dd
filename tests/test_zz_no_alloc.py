"""lbm_diag_noalloc, the allocation-free diagnostics, against lbm_diag on the same states:
two calls in a row on one GPU, the second on a smaller lattice (the shared scratch array
keeps the first call's partial sums), then a third model kind."""
import numpy as np
import pytest

import synthetic as S
from test_gpu_parity import random_case

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")
torch = pytest.importorskip("torch")


def _scales(d):
    """Per-sum scales of the tolerance: mass and kinetic energy by their own size, the
    momentum sums (zero in exact arithmetic for some states) by mass times a speed."""
    m = abs(d[0]) + abs(d[1])
    return np.array([abs(d[0]), abs(d[1]), m * 0.1, m * 0.1, m * 0.1, abs(d[5]), 1.0, 1.0]) + 1e-300


def _check(case, storage, layout=P.LBM_AB, steps=7):
    s = P.Sim.from_case(case, storage, layout)
    s.step(steps)
    want = s.diag()
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    P.lbm_diag_noalloc(s.h, out)
    s.sync()
    got = out.cpu().numpy()
    s.close()
    # FP64 sums of the same per-node values in another order: rounding only
    assert np.all(np.abs(got - want) <= 1e-12 * _scales(want)), (case.name, storage, got, want)
    assert got[6] == want[6] and got[7] == 0.0
    return got


def test_noalloc_diag_matches_diag_two_calls_second_smaller():
    big = random_case(S.D3Q19, S.BGK, 96, 40, 24, force=(1e-5, 0, -2e-5), walls=True)
    small = random_case(S.D3Q19, S.BGK, 37, 11, 7, force=(2e-5, 1e-5, 0), walls=True, seed=4)
    g1 = _check(big, P.LBM_F64)
    g2 = _check(small, P.LBM_F32S, P.LBM_AA)
    assert g2[0] < 0.2 * g1[0]  # the second call saw only its own nodes


@pytest.mark.parametrize("kind", ["shan_chen", "free_energy", "bf16", "elbm_d2q9"])
def test_noalloc_diag_other_models(kind):
    from test_gpu_free_energy import fe_random
    if kind == "shan_chen":
        _check(random_case(S.D3Q19, S.SHANCHEN, 40, 12, 9, tau=0.9, G=0.9, du=0.02, drho=0.05), P.LBM_F32)
    elif kind == "free_energy":
        _check(fe_random(S.D3Q19, 37, 12, 6), P.LBM_F64)
    elif kind == "bf16":
        _check(random_case(S.D3Q19, S.MRT, 64, 20, 10, tau=0.6, force=(0, 0, 1e-5), walls=True,
                           mrt_rates=S.mrt_rates_d3q19(1 / 0.6, 1.2)), P.LBM_BF16S)
    else:
        _check(random_case(S.D2Q9, S.ELBM, 130, 14, 1, tau=0.51, noise=2e-2), P.LBM_F64)


def test_noalloc_diag_needs_a_state():
    s = P.Sim(S.D3Q19, S.BGK, 8, 8, 8, 0.7)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(P.LbmError) as ei:
        P.lbm_diag_noalloc(s.h, out)
    assert ei.value.code == P.LBM_ESTATE
    s.close()
