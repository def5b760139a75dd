"""The widened workloads at the sizes the benchmark runs them, in its launch setup
(FP32 or shifted FP32 storage, AB), against the FP64 oracle run on the whole lattice for
a few steps: the lid-driven cavity 254^3 (walls, equilibrium lid, 254-wide rows with
their padding stores), the Kida vortex 256^3 with the Smagorinsky model, and the
free-energy spinodal decomposition 254x100x100.  Bars: the FP32 velocity target; for
the order parameter, FP32 resolution of phi."""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def run_both(case, steps, storage):
    s = P.Sim.from_case(case, storage, P.LBM_AB)
    s.step(steps)
    rg, ug = s.macro()
    s.close()
    o = oracle.Oracle.from_case(case)
    o.run(steps)
    ro, uo = o.macro()
    return rg, ug, ro, uo


def test_cavity_254_fullsize():
    c = S.lid_driven_cavity(254, S.BGK, re=1000.0)
    rg, ug, ro, uo = run_both(c, 4, P.LBM_F32)
    print("cavity 254^3, 4 steps: velocity rel L2 %.3g" % rel(ug, uo))
    assert rel(ug, uo) <= 1e-5
    assert np.abs(rg - ro).max() <= 1e-6


def test_kida_256_smagorinsky_fullsize():
    c = S.kida_vortex(256, S.SMAG, re=1.28e5)
    rg, ug, ro, uo = run_both(c, 4, P.LBM_F32)
    print("Kida 256^3 Smagorinsky, 4 steps: velocity rel L2 %.3g" % rel(ug, uo))
    assert rel(ug, uo) <= 1e-5


def test_spinodal_fullsize():
    c = S.spinodal()
    rg, ug, ro, uo = run_both(c, 4, P.LBM_F32S)
    print("spinodal 254x100x100, 4 steps: velocity rel L2 %.3g, phi max dev %.3g"
          % (rel(ug, uo), np.abs(rg[1] - ro[1]).max()))
    assert rel(ug, uo) <= 1e-5
    assert np.abs(rg[1] - ro[1]).max() <= 1e-6
    assert np.abs(rg[0] - ro[0]).max() <= 1e-6
