"""The C ABI: every entry point declared in include/lbm.h is exported by the built
library, and argument errors are reported without touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lbm():
    import paper_1311_2404_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("liblbm.so not built")
    return P


def test_header_and_binding_agree(lbm):
    assert _declared() == sorted(lbm.ENTRY_POINTS)


def test_library_exports_every_declared_symbol(lbm):
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lbm_[a-z_0-9]+)$", out, flags=re.M))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    L = ctypes.CDLL(lbm.LIB_PATH)
    for s in _declared():
        assert getattr(L, s) is not None


@pytest.mark.parametrize("args,code", [
    ((5, 0, 8, 8, 1, 0.8), -1),      # unknown lattice
    ((0, 9, 8, 8, 1, 0.8), -1),      # unknown model
    ((0, 0, 0, 8, 1, 0.8), -1),      # empty grid
    ((0, 0, 8, 8, 2, 0.8), -1),      # D2Q9 with nz > 1
    ((1, 0, 8, 8, 8, 0.5), -1),      # tau must exceed 1/2
    ((1, 0, 8, 8, 8, float("nan")), -1),
    ((1, 0, 70000, 70000, 1000, 0.8), -1),  # ny > 65535 and N >= 2^32
    ((1, 0, 8, 65536, 8, 0.8), -1),         # ny > 65535 (grid y limit)
    ((1, 0, 8, 8, 65536, 0.8), -1),         # nz > 65535 (grid z limit)
    ((1, 0, 65536, 65535, 2, 0.8), -1),     # N = 2^33 - 2^17 >= 2^32 with ny, nz in range
    ((1, 0, 65536, 256, 256, 0.8), -1),     # N = 2^32 exactly
])
def test_create_rejects_bad_arguments(lbm, args, code):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(*args)
    assert ei.value.code == code
    assert lbm.lbm_last_error(None)


def test_create_accepts_the_largest_grid(lbm):
    # N = 2^32 - 2^24 nodes, every axis within its limit; create allocates nothing
    h = lbm.lbm_create(1, 0, 65536, 256, 255, 0.8)
    lbm.lbm_destroy(h)


def test_elbm_rejects_force_and_state_errors(lbm):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_ELBM, 4, 4, 4, 0.6, (1e-5, 0, 0))
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_BGK, 4, 4, 4, 0.6)
    try:
        for call, code in [(lambda: lbm.lbm_step(h, 1), lbm.LBM_ESTATE),
                           (lambda: lbm.lbm_step(h, -1), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_get_f(h, np.zeros((1, 19, 64))), lbm.LBM_ESTATE),
                           (lambda: lbm.lbm_set_storage(h, 9), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_storage(h, lbm.LBM_F32, 0, 1), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_mrt_rates(h, np.ones(9)), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_mrt_rates(h, np.full(19, 2.5)), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_elbm(h, 3), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_elbm(h, 0, -1.0), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_set_shanchen(h, float("inf")), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_mlp_set_weights(h, np.zeros(10)), lbm.LBM_EINVAL),
                           (lambda: lbm.lbm_mlp_get_weights(h), None)]:
            if code is None:
                call()
                continue
            with pytest.raises(lbm.LbmError) as ei:
                call()
            assert ei.value.code == code
    finally:
        lbm.lbm_destroy(h)
    lbm.lbm_destroy(None)


def test_shan_chen_rejects_walls_and_sr(lbm):
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_SHANCHEN, 4, 4, 4, 1.0)
    try:
        fl = np.zeros(64, np.uint8)
        fl[0] = 1
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_flags(h, fl)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_storage(h, lbm.LBM_BF16S, lbm.LBM_AB, 1)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
        bad = np.full(64, 4, np.uint8)
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_flags(h, bad)
        assert ei.value.code == lbm.LBM_EINVAL
    finally:
        lbm.lbm_destroy(h)


def test_regularized_and_smagorinsky_arguments(lbm):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_REGULARIZED, 4, 4, 4, 0.6, (0, 1e-5, 0))
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_BGK, 4, 4, 4, 0.6)
    try:
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_smagorinsky(h, 0.1)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
    finally:
        lbm.lbm_destroy(h)
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_SMAGORINSKY, 4, 4, 4, 0.6, (0, 1e-5, 0))
    try:
        lbm.lbm_set_smagorinsky(h, 0.0)
        lbm.lbm_set_smagorinsky(h, 0.17)
        for bad in (-0.1, float("nan"), float("inf")):
            with pytest.raises(lbm.LbmError) as ei:
                lbm.lbm_set_smagorinsky(h, bad)
            assert ei.value.code == lbm.LBM_EINVAL
    finally:
        lbm.lbm_destroy(h)


def test_velocity_nodes_arguments(lbm):
    for kind in (lbm.LBM_VELOCITY, lbm.LBM_HALFWAY_BB):
        fl = np.zeros(64, np.uint8)
        fl[:16] = kind
        for model in (lbm.LBM_ELBM, lbm.LBM_SHANCHEN):
            h = lbm.lbm_create(lbm.LBM_D3Q19, model, 4, 4, 4, 0.6)
            try:
                with pytest.raises(lbm.LbmError) as ei:
                    lbm.lbm_set_flags(h, fl)
                assert ei.value.code == lbm.LBM_EUNSUPPORTED
            finally:
                lbm.lbm_destroy(h)
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_BGK, 4, 4, 4, 0.6)
    try:
        lbm.lbm_set_velocity_bc(h, (0.0, 0.05, 0.0))
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_velocity_bc(h, (0.0, float("nan"), 0.0))
        assert ei.value.code == lbm.LBM_EINVAL
    finally:
        lbm.lbm_destroy(h)


def test_free_energy_arguments(lbm):
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_BGK, 4, 4, 4, 0.6)
    try:
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_free_energy(h, 0.8, 1.0, 0.04, 0.04, 1.0)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
    finally:
        lbm.lbm_destroy(h)
    h = lbm.lbm_create(lbm.LBM_D3Q19, lbm.LBM_FREE_ENERGY, 4, 4, 4, 0.6, (1e-6, 0, 0))
    try:
        lbm.lbm_set_free_energy(h, 0.8, 1.0, 0.04, 0.04, 1.0)
        for bad in [(0.5, 1.0, 0.04, 0.04, 1.0), (0.8, 0.4, 0.04, 0.04, 1.0), (0.8, 1.0, float("nan"), 0.04, 1.0),
                    (0.8, 1.0, 0.04, -1.0, 1.0), (0.8, 1.0, 0.04, 0.04, -1.0)]:
            with pytest.raises(lbm.LbmError) as ei:
                lbm.lbm_set_free_energy(h, *bad)
            assert ei.value.code == lbm.LBM_EINVAL
        for st, sr in [(lbm.LBM_BF16S, 0), (lbm.LBM_F16S, 0), (lbm.LBM_F16S, 1)]:
            with pytest.raises(lbm.LbmError) as ei:
                lbm.lbm_set_storage(h, st, lbm.LBM_AB, sr)
            assert ei.value.code == lbm.LBM_EUNSUPPORTED
        fl = np.zeros(64, np.uint8)
        fl[:4] = lbm.LBM_VELOCITY
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_flags(h, fl)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
    finally:
        lbm.lbm_destroy(h)


def test_pop_layout_setter_rejects_bad_arguments(lbm):
    h = lbm.lbm_create(1, 0, 8, 8, 8, 0.7)
    try:
        for bad in (dict(kind=2), dict(tile_rows=3), dict(tile_rows=128), dict(tile_rows=-1), dict(row_pad=-1),
                    dict(block_pad=-2), dict(soa_pad=1 << 21), dict(row_pad=(1 << 20) + 1)):
            with pytest.raises(lbm.LbmError) as ei:
                lbm.lbm_set_pop_layout(h, **bad)
            assert ei.value.code == lbm.LBM_EINVAL, bad
        for good in (dict(kind=lbm.LBM_POP_SOA, soa_pad=0), dict(tile_rows=1), dict(tile_rows=64, block_pad=-1),
                     dict(row_pad=1 << 20)):
            lbm.lbm_set_pop_layout(h, **good)
    finally:
        lbm.lbm_destroy(h)


@pytest.mark.parametrize("model", [3, 6])  # Shan-Chen, free energy
@pytest.mark.parametrize("storage", [3, 4])  # BF16S, F16S
def test_two_component_models_refuse_16_bit_storage(lbm, model, storage):
    h = lbm.lbm_create(1, model, 8, 8, 8, 0.9)
    try:
        with pytest.raises(lbm.LbmError) as ei:
            lbm.lbm_set_storage(h, storage, lbm.LBM_AB, 0)
        assert ei.value.code == lbm.LBM_EUNSUPPORTED
        lbm.lbm_set_storage(h, lbm.LBM_F32S, lbm.LBM_AA, 0)
    finally:
        lbm.lbm_destroy(h)
