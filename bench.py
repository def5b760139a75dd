#!/usr/bin/env python3
"""Throughput of the fused LBM stream-and-collide step on one MI355X.

Workload (synthetic, shaped like the paper's periodic vortex benchmarks): D3Q19 LBGK,
3-D Taylor-Green vortex on a 256^3 periodic lattice, u0 = 0.04, nu = 0.01, rho = 1, plus
seeded U(+-1e-6) noise on every population.  A step is one fused stream-and-collide
kernel over all 16.8 M nodes (inputs resident in HBM).

Prints ONE JSON line: MLUPS of the FP32 run (``value``), the roofline of the step
kernel (algorithmic bytes / measured kernel time vs 8 TB/s), the shifted BF16/F16/FP32
storage variants with their MLUPS and velocity error after 1000 steps, and the FP64
oracle timed on the host cores (``cpu_baseline``).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_SIDE = 256
ERR_STEPS = 1000
VARIANT_STEPS, VARIANT_WARMUP = 400, 200  # steady-state window of the storage variants


def kernel_source_hash(tu="step_bgk.hip"):
    """Hash of the translation unit that builds the timed step kernel and of every header
    it includes, so stored counter readings go stale when that kernel's source changes."""
    import re
    d = os.path.join(ROOT, "paper_1311_2404_amd", "csrc")
    seen, todo = [], [tu]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.append(f)
        todo += re.findall(r'#include "([^"]+)"', open(os.path.join(d, f)).read())
    h = hashlib.sha256()
    for f in sorted(seen):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_tag, per_launch_nodes):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only if they were
    taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel_tag)
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


# VALU issue slots of the chip: 256 CUs x 4 SIMDs at 2.4 GHz, in SIMD-cycles per second.
# A full-rate wave64 instruction holds a 16-lane SIMD for 4 cycles, a transcendental for 16.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9


def stored_valu(kernel_tag, tu):
    """SIMD-cycles per node of an ALU-bound step from committed rocprofv3 VALU counter
    summaries, only if they were taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "valu_%s.json" % kernel_tag)
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("source_hash") != kernel_source_hash(tu):
        return None
    return rec


def bytes_per_node(storage):
    from paper_1311_2404_amd import ELEM_BYTES
    return 2 * 19 * ELEM_BYTES[storage]


def _time_steps(sim, stream, torch, steps):
    sim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    sim.sync()
    return e0.elapsed_time(e1) / steps


def entropic_profile(P, S, stream, torch, steps, warmup, alpha_init=1):
    """The entropic step alone, for kernel traces and counter passes: the 256^3 vortex in
    FP32 storage, AB, Newton from the series first guess (alpha_init 1), from 2 (0) or from
    the network's (2; the untrained network of mlp_initial_weights, whose zero output layer
    proposes the series estimate, so the instruction mix is the network's and the
    iterations are the series').  `warmup` steps run with the Newton statistics on; then
    `steps` steps are timed without them."""
    c4 = S.c4_elbm_taylor_green(n=256)
    s = P.Sim.from_case(c4, P.LBM_F32, P.LBM_AB, stream=stream)
    if alpha_init == 2:
        P.lbm_mlp_set_weights(s.h, P.mlp_initial_weights(20131124))
    P.lbm_set_elbm(s.h, alpha_init, 1e-10, 20)
    P.lbm_elbm_stats(s.h, enable=True, reset=True)
    s.step(warmup)
    hist, nonconv = P.lbm_elbm_stats(s.h, enable=False)
    ms = _time_steps(s, stream, torch, steps)
    s.close()
    k = np.arange(len(hist))
    guess = ("2", "the series guess", "the network's guess")[alpha_init]
    return {"workload": "D3Q19 entropic LBM 256^3 vortex, u0=0.05, nu=1e-5, FP32 storage, AB, "
                        "Newton from " + guess, "nodes": c4.n, "warmup": warmup, "steps": steps,
            "alpha_init": alpha_init,
            "mlups": round(c4.n / ms / 1e3, 1), "ms_per_step": round(ms, 4),
            "warmup_mean_newton_iters": round(float((k * hist).sum() / max(hist.sum(), 1)), 4),
            "warmup_nonconverged": int(nonconv)}


def duct_profile(P, S, stream, torch, steps, warmup, storage, sr):
    """The MRT duct 128x128x512 step alone (AB, with its four walls and body force), for
    kernel traces and counter passes: `warmup` steps, then `steps` timed steps."""
    c3 = S.c3_duct(128, 128, 512, steps=5000)
    st = {"f32": P.LBM_F32, "bf16s": P.LBM_BF16S, "f16s": P.LBM_F16S}[storage]
    s = P.Sim.from_case(c3, st, P.LBM_AB, sr, stream=stream)
    s.step(warmup)
    ms = _time_steps(s, stream, torch, steps)
    s.close()
    b = bytes_per_node(st) + 1
    return {"workload": "D3Q19 MRT duct 128x128x512, AB, %s storage%s" % (storage, ", stochastic rounding" if sr else ""),
            "nodes": c3.n, "warmup": warmup, "steps": steps, "mlups": round(c3.n / ms / 1e3, 1),
            "ms_per_step": round(ms, 4), "hbm_gbs_algorithmic": round(b * c3.n / (ms * 1e-3) / 1e9, 1)}


def sc_profile(P, S, stream, torch, steps, warmup):
    """The two-component Shan-Chen 384^3 step alone (FP32 storage), AA and then AB, for
    kernel traces and counter passes: `warmup` steps, then `steps` timed steps each."""
    c5 = S.c5_shan_chen(n=384)
    out = {"workload": "D3Q19 two-component Shan-Chen 384^3, G=0.9, psi=rho, FP32 storage", "nodes": c5.n,
           "warmup": warmup, "steps": steps}
    for lay, name in ((P.LBM_AA, "aa"), (P.LBM_AB, "ab")):
        s = P.Sim.from_case(c5, P.LBM_F32, lay, stream=stream)
        s.step(warmup)
        ms = _time_steps(s, stream, torch, steps)
        s.close()
        out[name] = {"mlups": round(c5.n / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                     "hbm_gbs_algorithmic": round(472 * c5.n / (ms * 1e-3) / 1e9, 1)}
    return out


def elbm_regimes(P, S, stream, torch):
    """D3Q19 entropic LBM 256^3 (u0 0.05, nu 1e-5), run to 8000 steps with Newton from the
    series estimate: (state, alpha) pairs every 500 steps, the network trained on 90% of
    them, and each first guess (2, series, MLP) timed over 100 steps from the states at
    steps 1000 and 8000, with its Newton histogram."""
    c4 = S.c4_elbm_taylor_green(n=256)
    s = P.Sim.from_case(c4, P.LBM_F32, P.LBM_AB, stream=stream)
    P.lbm_set_elbm(s.h, 1, 1e-10, 20)
    feats, alphas, snaps, states = [], [], [], {}
    nsamp = 62500
    for k in range(16):
        s.step(500)
        step_no = 500 * (k + 1)
        feat = torch.empty((nsamp, 6), dtype=torch.float32, device="cuda")
        alpha = torch.empty(nsamp, dtype=torch.float64, device="cuda")
        valid = torch.empty(nsamp, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        P.lbm_alpha_dataset(s.h, nsamp, 4242 + k, feat, alpha, valid)
        s.sync()
        keep = valid.bool()
        feats.append(feat[keep])
        alphas.append(alpha[keep])
        a = alpha[keep].cpu().numpy()
        x = feat[keep].cpu().numpy()
        dmax = np.maximum(x[:, 3], x[:, 4]) if len(x) else np.zeros(1)
        snaps.append({"step": step_no, "median_abs_alpha_minus_2": float(np.median(np.abs(a - 2))) if len(a) else 0.0,
                      "frac_abs_alpha_minus_2_gt_1e-3": float(np.mean(np.abs(a - 2) > 1e-3)) if len(a) else 0.0,
                      "median_max_abs_d": float(np.median(dmax)), "frac_max_abs_d_gt_0.1": float(np.mean(dmax > 0.1))})
        if step_no in (1000, 8000):
            states[step_no] = s.get_f()
    feat = torch.cat(feats).contiguous()
    alpha = torch.cat(alphas).contiguous()
    n_pairs = len(alpha)
    ntr = int(0.9 * n_pairs)
    torch.cuda.synchronize()  # produced on torch's stream, consumed on the library's
    P.lbm_mlp_set_weights(s.h, P.mlp_initial_weights(20131124))
    t0 = time.perf_counter()
    loss = P.lbm_mlp_train(s.h, feat[:ntr].contiguous(), alpha[:ntr].contiguous(), ntr, 20, 4096, 1e-3, 7)
    t_train = time.perf_counter() - t0
    y = torch.empty(n_pairs - ntr, dtype=torch.float32, device="cuda")
    P.lbm_mlp_forward(s.h, feat[ntr:].contiguous(), n_pairs - ntr, y)
    torch.cuda.synchronize()
    av = alpha[ntr:].cpu().numpy()
    xv = feat[ntr:].cpu().numpy().astype(np.float64)
    elbm = {"snapshots": snaps, "dataset_pairs": int(n_pairs), "train_pairs": ntr, "train_s": round(t_train, 2),
            "loss_first_last": [float(loss[0]), float(loss[-1])],
            "heldout_median_abs_err": {"alpha0_2": float(np.median(np.abs(2.0 - av))),
                                       "series": float(np.median(np.abs(2 + (xv[:, 1] - 2 * xv[:, 2]) / 3 - av))),
                                       "mlp": float(np.median(np.abs(y.cpu().numpy() - av)))}}
    del feat, alpha, feats, alphas
    for step_no, f0 in states.items():
        rows, u_ref = {}, None
        for init, name in [(0, "newton_from_2"), (1, "newton_from_series"), (2, "newton_from_mlp")]:
            s.set_f(f0)
            P.lbm_set_elbm(s.h, init, 1e-10, 20)
            P.lbm_elbm_stats(s.h, enable=True, reset=True)
            ms = _time_steps(s, stream, torch, 100)
            hist, nonconv = P.lbm_elbm_stats(s.h, enable=False)
            u = s.macro()[1]
            if u_ref is None:
                u_ref = u
            k = np.arange(len(hist))
            rows[name] = {"mlups": round(c4.n / ms / 1e3, 1),
                          "mean_newton_iters": round(float((k * hist).sum() / max(hist.sum(), 1)), 4),
                          "newton_hist": [int(v) for v in hist[:8]], "nonconverged": int(nonconv),
                          "vel_rel_l2_vs_newton_from_2": float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))}
            tag = {1: "d3q19_elbm_f32_ab_256", 2: "d3q19_elbm_mlp_f32_ab_256"}.get(init)
            rec = stored_valu(tag, "step_elbm.hip") if tag and step_no == 1000 else None
            if rec:
                # VALU-issue roofline from the SIMD-cycles per node counted at step 1000 of the
                # same vortex (series guess; the network's instruction mix for its row)
                ach = rec["simd_cycles_per_node"] * c4.n / (ms * 1e-3)
                rows[name]["roofline"] = {"bound": "alu", "achieved": round(ach / 1e12, 4),
                                          "peak": round(VALU_ISSUE_PEAK / 1e12, 4),
                                          "unit": "T SIMD-cycles/s (VALU issue)",
                                          "frac": round(ach / VALU_ISSUE_PEAK, 4),
                                          "simd_cycles_per_node": rec["simd_cycles_per_node"]}
        elbm["from_step_%d" % step_no] = rows
    s.close()
    return elbm


def run_extras(P, S, stream, torch):
    """The other measured configurations (throughput and stated errors), one GPU."""
    out = {}
    # D3Q19 MRT duct 128x128x512, 5000 steps: each storage's velocity error vs FP64
    c3 = S.c3_duct(128, 128, 512, steps=5000)
    us, rows = {}, {}
    for st, sr in [(P.LBM_F64, 0), (P.LBM_F32, 0), (P.LBM_F32S, 0), (P.LBM_BF16S, 0), (P.LBM_BF16S, 1),
                   (P.LBM_F16S, 0), (P.LBM_F16S, 1)]:
        s = P.Sim.from_case(c3, st, P.LBM_AB, sr, stream=stream)
        s.step(VARIANT_WARMUP)  # past the clock's ramp after the host-side set-up
        ms = _time_steps(s, stream, torch, VARIANT_STEPS)
        s.close()
        s = P.Sim.from_case(c3, st, P.LBM_AB, sr, stream=stream)
        s.step(c3.steps)
        us[(st, sr)] = s.macro()[1]
        s.close()
        b = bytes_per_node(st) + 1  # populations read and written, plus the flag byte
        rows[P.STORAGE_NAMES[st] + ("_sr" if sr else "")] = {
            "mlups": round(c3.n / ms / 1e3, 1), "bytes_per_node": b,
            "hbm_gbs_algorithmic": round(b * c3.n / (ms * 1e-3) / 1e9, 1)}
    ref, ref32 = us[(P.LBM_F64, 0)], us[(P.LBM_F32, 0)]
    for (st, sr), u in us.items():
        row = rows[P.STORAGE_NAMES[st] + ("_sr" if sr else "")]
        row["vel_rel_l2_vs_fp64"] = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
        row["vel_rel_l2_vs_f32"] = float(np.linalg.norm(u - ref32) / np.linalg.norm(ref32))
    out["d3q19_mrt_duct_128x128x512_5000_steps"] = rows
    print("[bench] MRT duct done", file=sys.stderr, flush=True)

    # Diagnostics (kinetic energy, mass, momentum) on the 256^3 Taylor-Green state: one call
    # is the macroscopic pass (populations in, FP64 rho and u out), the two-stage FP64
    # reduction over those fields and the copy of the 8 sums to the host
    c2 = S.c2_taylor_green(n=256)
    diag = {}
    for st in (P.LBM_F32, P.LBM_F32S, P.LBM_BF16S):
        s = P.Sim.from_case(c2, st, P.LBM_AB, stream=stream)
        s.diag()
        t0 = time.perf_counter()
        for _ in range(20):
            s.diag()
        ms = (time.perf_counter() - t0) / 20 * 1e3
        s.close()
        b = bytes_per_node(st) // 2 + 4 * 8 + 4 * 8  # populations read, FP64 rho and u written, read back
        diag[P.STORAGE_NAMES[st]] = {"ms_per_call": round(ms, 4), "bytes_per_node": b,
                                     "hbm_gbs_algorithmic": round(b * c2.n / (ms * 1e-3) / 1e9, 1)}
    out["d3q19_diagnostics_256"] = diag
    del c2
    print("[bench] diagnostics done", file=sys.stderr, flush=True)

    out["d3q19_elbm_taylor_green_256_fp32"] = elbm_regimes(P, S, stream, torch)
    print("[bench] ELBM done", file=sys.stderr, flush=True)

    # D3Q19 two-component Shan-Chen 384^3, FP32 compute: throughput and per-component
    # conservation with plain and shifted FP32 storage (same bytes per node), AB and AA
    c5 = S.c5_shan_chen(n=384)
    for st, lay, tag in [(P.LBM_F32, P.LBM_AB, "fp32"), (P.LBM_F32, P.LBM_AA, "fp32_aa"), (P.LBM_F32S, P.LBM_AB, "f32s")]:
        s = P.Sim.from_case(c5, st, lay, stream=stream)
        d0 = s.diag()
        ms = _time_steps(s, stream, torch, 100)
        d1 = s.diag()
        s.close()
        out["d3q19_shan_chen_384_" + tag] = {"mlups": round(c5.n / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                             "layout": "aa" if lay == P.LBM_AA else "ab", "bytes_per_node": 472,
                                             "hbm_gbs_algorithmic": round(472 * c5.n / (ms * 1e-3) / 1e9, 1),
                                             "steps": 100,
                                             "mass_rel_change": [float(abs(d1[c] - d0[c]) / d0[c]) for c in (0, 1)]}
    print("[bench] Shan-Chen done", file=sys.stderr, flush=True)

    # D3Q19 Kida vortex 256^3, FP32 storage, AB and AA: LBGK and regularized LBGK at
    # Re 4000, Smagorinsky LBGK (C_S = 0.1) at Re 1.28e5
    kida = {}
    for model, re, name in [(S.BGK, 4000.0, "bgk_re4000"), (S.REG, 4000.0, "regularized_re4000"),
                            (S.SMAG, 1.28e5, "smagorinsky_re128000")]:
        ck = S.kida_vortex(256, model, re=re)
        for lay, tag in [(P.LBM_AB, ""), (P.LBM_AA, "_aa")]:
            s = P.Sim.from_case(ck, P.LBM_F32, lay, stream=stream)
            ke0 = s.diag()[5]
            s.step(20)
            ms = _time_steps(s, stream, torch, 200)
            d = s.diag()
            s.close()
            kida[name + tag] = {"mlups": round(ck.n / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                "bytes_per_node": 152, "hbm_gbs_algorithmic": round(152 * ck.n / (ms * 1e-3) / 1e9, 1),
                                "tau": round(ck.tau, 6), "ke_ratio_after_220_steps": float(d[5] / ke0),
                                "nonfinite_nodes": int(d[6])}
    out["d3q19_kida_256_fp32"] = kida
    print("[bench] Kida done", file=sys.stderr, flush=True)

    # D3Q19 lid-driven cavity 254^3 at Re 1000, FP32 storage, AB: full-way bounce-back
    # walls and an equilibrium-velocity lid (u = 0.05), for each model that takes it
    ldc = {}
    for model, name in [(S.BGK, "bgk"), (S.MRT, "mrt"), (S.REG, "regularized"), (S.SMAG, "smagorinsky")]:
        cl = S.lid_driven_cavity(254, model, re=1000.0)
        s = P.Sim.from_case(cl, P.LBM_F32, P.LBM_AB, stream=stream)
        s.step(20)
        ms = _time_steps(s, stream, torch, 200)
        d = s.diag()
        s.close()
        ldc[name] = {"mlups": round(cl.n / ms / 1e3, 1), "ms_per_step": round(ms, 4), "bytes_per_node": 153,
                     "hbm_gbs_algorithmic": round(153 * cl.n / (ms * 1e-3) / 1e9, 1), "tau": round(cl.tau, 6),
                     "ke_after_220_steps": float(d[5]), "nonfinite_nodes": int(d[6])}
    out["d3q19_ldc_254_re1000_fp32"] = ldc
    print("[bench] cavity done", file=sys.stderr, flush=True)

    # free-energy binary fluid: spinodal decomposition 254x100x100, the paper's binary
    # benchmark (phi pre-pass + step of both lattices; algorithmic bytes per node: f and g
    # read and written 2 x 2 x 19 x 4, the pre-pass's g read 19 x 4 and phi write 4, the
    # step's phi read 4), and the binary Poiseuille flow of the validation section on its
    # 64x256 grid run to the steady state, against the sharp-interface solution
    fe = {}
    cs = S.spinodal()
    for st, tag, lay in [(P.LBM_F32S, "f32s", P.LBM_AB), (P.LBM_F32, "f32", P.LBM_AB), (P.LBM_F32S, "f32s_aa", P.LBM_AA)]:
        s = P.Sim.from_case(cs, st, lay, stream=stream)
        s.step(20)
        ms = _time_steps(s, stream, torch, 200)
        d = s.diag()
        s.close()
        fe["spinodal_254x100x100_" + tag] = {"mlups": round(cs.n / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                             "bytes_per_node": 388,
                                             "hbm_gbs_algorithmic": round(388 * cs.n / (ms * 1e-3) / 1e9, 1),
                                             "nonfinite_nodes": int(d[6])}
    cp = S.binary_poiseuille()
    s = P.Sim.from_case(cp, P.LBM_F32S, P.LBM_AB, stream=stream)
    prev, steps = None, 0
    while steps < 1000000:
        s.step(50000)
        steps += 50000
        ux = s.macro()[1][0].reshape(cp.ny, cp.nx)[:, 0].copy()
        if prev is not None and np.abs(ux - prev).max() < 1e-5 * np.abs(ux).max():
            break
        prev = ux
    s.close()
    yc, L, nu0, nu1, g = (cp.extra[k] for k in ("yc", "L", "nu0", "nu1", "g"))
    yy = np.arange(cp.ny) - yc
    ana = np.where(np.abs(yy) > L / 2, g / (2 * nu0) * (L ** 2 - yy ** 2),
                   g * L ** 2 / 8 * (3 / nu0 + 1 / nu1 * (1 - 4 * yy ** 2 / L ** 2)))
    fe["binary_poiseuille_64x256_f32s"] = {"steps": steps, "umax": float(ux.max()), "umax_analytic": float(ana.max()),
                                           "vel_rel_l2_vs_analytic": float(np.linalg.norm(ux[1:-1] - ana[1:-1]) /
                                                                           np.linalg.norm(ana[1:-1]))}
    out["free_energy"] = fe
    print("[bench] free energy done", file=sys.stderr, flush=True)
    return out


PRECISION_U0 = (0.0005, 0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1)


def precision_sweep(P, S, stream, n=256, re=1000.0, u0s=PRECISION_U0, runs=None):
    """The paper's single-precision study (Impact of single precision): D2Q9 LBGK decaying
    Taylor-Green vortex on a periodic n^2 lattice at Re = u0 n / nu = 1000, every u0 run to
    the same physical time (1e6 steps at u0 = 0.0005 on 256^2), here for every storage,
    stochastic rounding included.  Velocity and density are compared with the analytic
    solution, u = u0 (-cos kx sin ky, sin kx cos ky) exp(-2 nu k^2 t) and
    rho - 1 = -(3/4) u0^2 (cos 2kx + cos 2ky) exp(-4 nu k^2 t), as relative L2 norms."""
    import numpy as np
    k = 2 * np.pi / n
    x, y, _ = S._grid(n, n, 1)
    runs = runs or [("f64", P.LBM_F64, 0), ("f32", P.LBM_F32, 0), ("f32s", P.LBM_F32S, 0),
                    ("bf16s", P.LBM_BF16S, 0), ("bf16s_sr", P.LBM_BF16S, 1), ("f16s", P.LBM_F16S, 0),
                    ("f16s_sr", P.LBM_F16S, 1)]
    out = {}
    for name, st, sr in runs:
        rows = []
        for u0 in u0s:
            nu = u0 * n / re
            steps = int(round(1e6 * 0.0005 / u0 * n / 256))
            _, u = S.taylor_green_2d(n, n, u0)
            drho = -0.75 * u0 ** 2 * (np.cos(2 * k * x) + np.cos(2 * k * y))
            c = S.Case("tg2d", S.D2Q9, S.BGK, n, n, 1, S.tau_from_nu(nu), (0.0, 0.0, 0.0), steps, None,
                       (1.0 + drho)[None], u)
            s = P.Sim.from_case(c, st, P.LBM_AB, sr, stream=stream)
            s.step(steps)
            rho, ug = s.macro()
            s.close()
            ue = u * np.exp(-2 * nu * k * k * steps)
            de = drho * np.exp(-4 * nu * k * k * steps)
            rows.append({"u0": u0, "steps": steps,
                         "vel_rel_l2": float(np.sqrt(((ug[:2] - ue) ** 2).sum() / (ue ** 2).sum())),
                         "rho_rel_l2": float(np.sqrt(((rho[0] - 1.0 - de) ** 2).sum() / (de ** 2).sum()))})
        out[name] = rows
        print("[bench] precision sweep %s done" % name, file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--layout", choices=["ab", "aa"], default="ab",
                    help="streaming layout of the timed step (AB, the default: two copies; AA: in place, even "
                         "and odd kernels)")
    ap.add_argument("--n", type=int, default=N_SIDE, help="lattice side (default 256)")
    ap.add_argument("--no-variants", action="store_true", help="time the FP32 run only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the MRT duct, entropic/MLP and Shan-Chen rows")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the 1000-step velocity-error runs (for short profiled runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run 3 plain device copies of MIB MiB (calibrates HBM byte counters in profiles)")
    ap.add_argument("--precision-sweep", action="store_true",
                    help="run only the D2Q9 Taylor-Green precision study over u0 and storages (JSON line)")
    ap.add_argument("--entropic-profile", action="store_true",
                    help="run only the entropic 256^3 step (first guess from --alpha-init), for traces and counters (JSON line)")
    ap.add_argument("--alpha-init", type=int, default=1, choices=[0, 1, 2],
                    help="first guess of the alpha solve for --entropic-profile (0: 2, 1: series, 2: network)")
    ap.add_argument("--duct-profile", choices=["f32", "bf16s", "f16s"],
                    help="run only the MRT duct 128x128x512 step in this storage, for traces and counters (JSON line)")
    ap.add_argument("--sr", type=int, default=0, choices=[0, 1], help="stochastic rounding for --duct-profile")
    ap.add_argument("--sc-profile", action="store_true",
                    help="run only the Shan-Chen 384^3 step, AA then AB, for traces and counters (JSON line)")
    ap.add_argument("--elbm-regimes", action="store_true",
                    help="run only the entropic 256^3 vortex to 8000 steps: MLP training and the first guesses "
                         "timed at steps 1000 and 8000 (JSON line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one process drives one device).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1311_2404_amd as P
    import synthetic as S

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    if args.precision_sweep:
        t0 = time.perf_counter()
        res = precision_sweep(P, S, stream)
        print(json.dumps({"precision_sweep": res, "lattice": "D2Q9 256^2", "re": 1000,
                          "wall_s": round(time.perf_counter() - t0, 1)}))
        return
    if args.entropic_profile:
        print(json.dumps(entropic_profile(P, S, stream, torch, args.steps, args.warmup, args.alpha_init)))
        return
    if args.duct_profile:
        print(json.dumps(duct_profile(P, S, stream, torch, args.steps, args.warmup, args.duct_profile, args.sr)))
        return
    if args.sc_profile:
        print(json.dumps(sc_profile(P, S, stream, torch, args.steps, args.warmup)))
        return
    if args.elbm_regimes:
        print(json.dumps(elbm_regimes(P, S, stream, torch)))
        return
    layout = P.LBM_AA if args.layout == "aa" else P.LBM_AB
    n = args.n
    N = n ** 3
    case = S.c2_taylor_green(n=n, steps=ERR_STEPS)
    print("[bench] inputs ready: D3Q19 BGK TGV %d^3" % n, file=sys.stderr, flush=True)

    def make(storage, lay=None):
        s = P.Sim.from_case(case, storage, layout if lay is None else lay, stream=stream)
        return s

    def timed(storage, steps, warmup, lay=None):
        s = make(storage, lay)
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = e0.elapsed_time(e1) / steps
        s.close()
        return wall, kern_ms

    if args.copy_probe:
        a = torch.empty(args.copy_probe * 2 ** 20 // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # headline: FP32 storage
    wall, kern_ms = timed(P.LBM_F32, args.steps, args.warmup)
    mlups = N * args.steps / wall / 1e6
    bpn = bytes_per_node(P.LBM_F32)
    achieved = bpn * N / (kern_ms * 1e-3) / 1e9
    print("[bench] fp32: %.1f MLUPS, %.4f ms/step" % (mlups, wall / args.steps * 1e3), file=sys.stderr, flush=True)

    # velocity error after the configuration's 1000 steps, vs the FP64 run of the same kernel
    # (which matches the FP64 oracle to 1e-12 in the parity tests) and vs the Navier-Stokes KE law
    def run_fields(storage):
        s = make(storage)
        s.step(ERR_STEPS)
        rho, u = s.macro()
        s.close()
        return u

    u64 = None if args.no_errors else run_fields(P.LBM_F64)
    k = 2 * np.pi / n
    ke_law = float(np.exp(-6 * case.extra["nu"] * k * k * ERR_STEPS))
    ke0 = float((case.u ** 2).sum())

    def errs(storage):
        if u64 is None:
            return {}
        u = run_fields(storage)
        return {"vel_rel_l2_vs_fp64": float(np.linalg.norm(u - u64) / np.linalg.norm(u64)),
                "ke_ratio": float((u ** 2).sum() / ke0), "ke_ratio_ns_law": ke_law}

    variants = {"f32": dict(mlups=round(mlups, 1), bytes_per_node=bpn, **errs(P.LBM_F32))}
    # The variants are timed over a steady-state window whatever --steps and --warmup say:
    # after host-side set-up leaves the GPU idle, its clock dips for a few ms once a
    # sustained load starts (a 20-step run of the 16-bit steps, which issue close to the
    # VALU limit, ran 10% slower than 1000 steps; the memory-bound FP32 step did not move).
    vsteps, vwarm = max(args.steps, VARIANT_STEPS), max(args.warmup, VARIANT_WARMUP)
    if not args.no_variants:
        for st in (P.LBM_F32S, P.LBM_BF16S, P.LBM_F16S, P.LBM_F64):
            w2, k2 = timed(st, vsteps, vwarm)
            m2 = N * vsteps / w2 / 1e6
            b2 = bytes_per_node(st)
            v = dict(mlups=round(m2, 1), bytes_per_node=b2, steps=vsteps, warmup=vwarm,
                     hbm_gbs_algorithmic=round(b2 * N / (k2 * 1e-3) / 1e9, 1))
            # the same storage with the other streaming layout (the 16-bit steps are faster in AA)
            other = P.LBM_AB if layout == P.LBM_AA else P.LBM_AA
            w3, _ = timed(st, vsteps, vwarm, other)
            v["mlups_" + ("ab" if other == P.LBM_AB else "aa")] = round(N * vsteps / w3 / 1e6, 1)
            if st != P.LBM_F64:
                v.update(errs(st))
            variants[P.STORAGE_NAMES[st]] = v
            print("[bench] %s: %.1f MLUPS" % (P.STORAGE_NAMES[st], m2), file=sys.stderr, flush=True)
        # the same FP32 step with the other streaming layout (same algorithmic bytes)
        other = P.LBM_AB if layout == P.LBM_AA else P.LBM_AA
        w2, k2 = timed(P.LBM_F32, vsteps, vwarm, other)
        tag = "f32_" + ("ab" if other == P.LBM_AB else "aa")
        variants[tag] = dict(mlups=round(N * vsteps / w2 / 1e6, 1), bytes_per_node=bpn, steps=vsteps, warmup=vwarm,
                             hbm_gbs_algorithmic=round(bpn * N / (k2 * 1e-3) / 1e9, 1))
        print("[bench] %s: %.1f MLUPS" % (tag, variants[tag]["mlups"]), file=sys.stderr, flush=True)

    extras = {} if args.no_extras else run_extras(P, S, stream, torch)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Oracle.from_case(case)
        o.run(1)  # first touch of the second copy
        t0 = time.perf_counter()
        o.run(args.cpu_steps)
        dt = time.perf_counter() - t0
        cores = oracle.threads()
        # the same oracle on one thread, over a shorter sample
        oracle.set_threads(1)
        t1 = time.perf_counter()
        o.run(1)
        dt1 = time.perf_counter() - t1
        oracle.set_threads(cores)
        cpu = {"value": round(N * args.cpu_steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
               "kind": "oracle",
               "sample": "FP64 oracle, the same 256^3 D3Q19 BGK Taylor-Green state, %d steps (%.1f s)"
                         % (args.cpu_steps, dt),
               "single_thread_mlups": round(N / dt1 / 1e6, 3)}

    tag = "d3q19_bgk_f32_%s_%d" % (args.layout, n)
    traffic = stored_traffic(tag, N)
    out = {
        "metric": "MLUPS and % of HBM roofline, D3Q19 256^3 FP32 vs shifted-BF16 at stated error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D3Q19 LBGK 3-D Taylor-Green vortex %d^3 periodic, u0=0.04, nu=0.01, "
                               "+-1e-6 seeded noise, FP32 storage, %s streaming" % (n, args.layout.upper()),
                   "nodes": N, "layout": args.layout},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_step<D3Q19, F32, BGK>" + (" (AA even and odd, averaged)" if args.layout == "aa" else ""),
                     "bytes_per_node": bpn,
                     "kernel_ms_per_launch": round(kern_ms, 5)},
        "variants": variants,
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
