"""The learned ELBM alpha proposal: GPU inference, gradients and the data sampler
against the FP64 oracle, and what the trained network gains over Newton from alpha = 2."""
import numpy as np
import pytest

import oracle
import synthetic as S

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_2404_amd")
torch = pytest.importorskip("torch")


def bf16_round(a):
    """Round FP32 values to bfloat16 (nearest even), returned as float64."""
    b = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = (scale * rng.standard_normal(P.MLP_NPARAM)).astype(np.float32)
    p[-1] = 0.0
    return p


def elbm_case(n, u0=0.08, nu=1e-4, noise=3e-4, seed=3):
    c = S.c4_elbm_taylor_green(n=n, u0=u0, nu=nu)
    c.df = S.uniform_pm(seed, 0, (1, 19, n ** 3), noise)
    return c


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def mfma_rounding_model(p, mu, isd, x):
    """Per sample, how far the wave-level network may sit from the exact one with the
    same BF16 weights.  The normalised inputs and the layer-1 outputs enter the matrix
    cores rounded to BF16 (unit roundoff u = 2^-8), tanh is evaluated from exp2 and a
    reciprocal (absolute 3e-7 here), and the sums accumulate in FP32.  Returns a
    first-order worst-case bound (absolute error terms summed) and the standard deviation
    of the same errors taken as independent and uniform (variances summed)."""
    H, I = 32, 6
    W1 = p[:H * I].reshape(H, I); b1 = p[H * I:H * I + H]
    o = H * I + H
    W2 = p[o:o + H * H].reshape(H, H); b2 = p[o + H * H:o + H * H + H]
    w3 = p[o + H * H + H:o + H * H + 2 * H]
    u, e32, et = 2.0 ** -8, 2.0 ** -24, 3e-7
    xn = (x - mu) * isd
    z1 = xn @ W1.T + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = np.tanh(z2)
    # worst case
    dz1 = u * np.abs(xn) @ np.abs(W1).T + 8 * e32 * (np.abs(xn) @ np.abs(W1).T + np.abs(b1))
    dh1 = dz1 + u * np.abs(h1) + et
    dz2 = dh1 @ np.abs(W2).T + 34 * e32 * (np.abs(h1) @ np.abs(W2).T + np.abs(b2))
    bound = (dz2 + et) @ np.abs(w3) + 34 * e32 * (np.abs(h2) @ np.abs(w3))
    # independent uniform rounding errors: variance u^2 v^2 / 3 for a value v
    v1 = (u * u / 3) * (xn * xn) @ (W1 * W1).T
    vh1 = v1 * (1 - h1 * h1) ** 2 + (u * u / 3) * h1 * h1
    vz2 = vh1 @ (W2 * W2).T
    sigma = np.sqrt((vz2 * (1 - h2 * h2) ** 2) @ (w3 * w3))
    return bound, sigma


def test_forward_bf16_matches_oracle():
    """The wave-level network (BF16 weights on the matrix cores, FP32 accumulation) vs the
    FP64 oracle on the same BF16-rounded weights.  Every sample lies within the worst-case
    bound of the BF16 operands the matrix cores take, and the errors have the size that
    rounding predicts (a misplaced weight or bias would not).  The proposal is the series
    estimate plus the network.  5000 rows: 78 waves and a partial one."""
    s = P.Sim.from_case(elbm_case(8), P.LBM_F32)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5000, 6)).astype(np.float32)
    for with_norm in (False, True):
        p = init_params(2)
        mu, isd = np.zeros(6, np.float32), np.ones(6, np.float32)
        if with_norm:
            mu = rng.standard_normal(6).astype(np.float32)
            isd = (0.5 + rng.random(6)).astype(np.float32)
        P.lbm_mlp_set_weights(s.h, np.concatenate([p, mu, isd]).astype(np.float32))
        y = torch.empty(len(x), dtype=torch.float32, device="cuda")
        P.lbm_mlp_forward(s.h, dev(x, torch.float32), len(x), y)
        torch.cuda.synchronize()
        pb = bf16_round(p)
        want = oracle.mlp_forward(np.concatenate([pb, mu, isd]), x.astype(np.float64))
        bound, sigma = mfma_rounding_model(pb, mu.astype(np.float64), isd.astype(np.float64), x.astype(np.float64))
        err = y.cpu().numpy() - want
        assert np.all(np.abs(err) <= bound + 2e-6), np.abs(err / bound).max()
        z = np.sqrt(np.mean((err / sigma) ** 2))
        print("normalised RMS error %.3f, max |err| / bound %.3f" % (z, np.abs(err / bound).max()))
        assert 0.2 < z < 5.0, z
    s.close()


def test_loss_and_gradient_match_oracle():
    s = P.Sim.from_case(elbm_case(8), P.LBM_F32)
    rng = np.random.default_rng(4)
    n = 3000
    x = rng.standard_normal((n, 6)).astype(np.float32)
    t = 2.0 + 0.05 * rng.standard_normal(n)
    p = init_params(5)
    P.lbm_mlp_set_weights(s.h, p)
    loss, g = P.lbm_mlp_loss_grad(s.h, dev(x, torch.float32), dev(t, torch.float64), n)
    lo, go = oracle.mlp_loss_grad(p.astype(np.float64), x.astype(np.float64), t)
    # FP32 forward and backward per sample, FP32 sums over a block's 64 samples in a fixed
    # order, FP64 over blocks: a few 1e-7 relative; 3 000 rows span 47 blocks and a ragged tail
    assert abs(loss - lo) <= 1e-6 * lo
    assert np.linalg.norm(g - go) <= 5e-6 * np.linalg.norm(go)
    s.close()


def test_alpha_dataset_matches_oracle():
    c = elbm_case(24)
    s = P.Sim.from_case(c, P.LBM_F64, P.LBM_AA)
    s.step(3)
    f = s.get_f()
    n, seed = 4000, 77
    feat = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    alpha = torch.empty(n, dtype=torch.float64, device="cuda")
    valid = torch.empty(n, dtype=torch.uint8, device="cuda")
    P.lbm_alpha_dataset(s.h, n, seed, feat, alpha, valid)
    torch.cuda.synchronize()
    feat, alpha, valid = feat.cpu().numpy(), alpha.cpu().numpy(), valid.cpu().numpy()
    s.close()
    nodes = (S.splitmix64(np.uint64(seed) ^ np.arange(n, dtype=np.uint64)) % np.uint64(c.n)).astype(np.int64)
    e, _, _ = oracle.tables(S.D3Q19)
    checked = 0
    for k in range(0, n, 7):
        fk = f[0, :, nodes[k]]
        rho = fk.sum()
        u = e.T @ fk / rho
        fe = oracle.feq_entropic(S.D3Q19, rho, u)
        a, it, conv = oracle.alpha(S.D3Q19, fk, fe)
        if it == 0:
            assert valid[k] == 0
            continue
        assert valid[k] == 1 and conv
        assert abs(alpha[k] - a) <= 1e-9
        want = oracle.alpha_features(S.D3Q19, fk, fe, rho, float(u @ u))
        np.testing.assert_allclose(feat[k], want, rtol=2e-5, atol=1e-12)
        checked += 1
    assert checked > 200


def _mean_iters(hist):
    k = np.arange(len(hist))
    return float((k * hist).sum() / hist.sum())


def test_trained_mlp_cuts_newton_iterations():
    """Train on (state, alpha) pairs the plain solver produces, then run the same steps
    from the same state with alpha0 = 2 and with alpha0 = MLP: Newton still decides alpha, so
    the fields agree to the Newton tolerance while the MLP start needs fewer iterations."""
    c = elbm_case(32, u0=0.1, nu=2e-4, noise=5e-4)
    s = P.Sim.from_case(c, P.LBM_F64, P.LBM_AB)
    s.step(40)
    nsamp = 200000
    feats, alphas = [], []
    for snap in range(2):
        feat = torch.empty((nsamp, 6), dtype=torch.float32, device="cuda")
        alpha = torch.empty(nsamp, dtype=torch.float64, device="cuda")
        valid = torch.empty(nsamp, dtype=torch.uint8, device="cuda")
        P.lbm_alpha_dataset(s.h, nsamp, 1000 + snap, feat, alpha, valid)
        keep = valid.bool()
        feats.append(feat[keep])
        alphas.append(alpha[keep])
        s.step(20)
    feat = torch.cat(feats).contiguous()
    alpha = torch.cat(alphas).contiguous()
    ntr = int(0.9 * len(alpha))
    P.lbm_mlp_set_weights(s.h, P.mlp_initial_weights(11))
    loss = P.lbm_mlp_train(s.h, feat[:ntr].contiguous(), alpha[:ntr].contiguous(), ntr, 20, 4096, 1e-3, 5)
    assert loss[-1] < 0.05 * loss[0], loss
    # held-out: the proposal is closer to the root than 2 and than the bare series
    y = torch.empty(len(alpha) - ntr, dtype=torch.float32, device="cuda")
    P.lbm_mlp_forward(s.h, feat[ntr:].contiguous(), len(y), y)
    torch.cuda.synchronize()
    av = alpha[ntr:].cpu().numpy()
    xv = feat[ntr:].cpu().numpy().astype(np.float64)
    err_mlp = np.median(np.abs(y.cpu().numpy() - av))
    err_two = np.median(np.abs(2.0 - av))
    err_ser = np.median(np.abs(2 + (xv[:, 1] - 2 * xv[:, 2]) / 3 - av))
    print("held-out median |alpha0 - alpha|: 2 -> %.3e, series -> %.3e, MLP -> %.3e" % (err_two, err_ser, err_mlp))
    assert err_mlp < 0.05 * err_two and err_mlp <= 0.5 * err_ser, (err_mlp, err_ser, err_two)

    f0 = s.get_f()
    res = {}
    for init in (0, 2, 1):
        s.set_f(f0)
        P.lbm_set_elbm(s.h, init, 1e-10, 20)
        P.lbm_elbm_stats(s.h, enable=True, reset=True)
        s.step(10)
        hist, nonconv = P.lbm_elbm_stats(s.h, enable=False)
        res[init] = (hist, nonconv, s.macro()[1])
    s.close()
    it0, it2, it1 = (_mean_iters(res[k][0]) for k in (0, 2, 1))
    print("mean Newton iterations: alpha0=2 %.3f, MLP %.3f, series %.3f" % (it0, it2, it1))
    assert res[0][1] == 0 and res[2][1] == 0
    assert it2 < it0 - 0.3
    assert it2 <= it1 + 0.05  # at least as good a start as the bare series
    u0 = res[0][2]
    for k in (1, 2):
        assert np.linalg.norm(res[k][2] - u0) <= 1e-9 * np.linalg.norm(u0)
