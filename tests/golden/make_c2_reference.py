"""Writes ``c2_taylor_green_256.npz``: the FP64 oracle's state after the 1000 steps of the
D3Q19 LBGK Taylor-Green configuration on the 256^3 periodic lattice (u0 = 0.04,
nu = 0.01, rho = 1, seeded U(+-1e-6) noise on every population), reduced to what a test
can compare against a GPU run in seconds:

- ``nodes``: 8192 node indices drawn by a SplitMix64 counter hash (seed 31337), with
  ``rho`` and ``u`` of the oracle at those nodes (full FP64);
- ``plane_u2`` [3][256]: per z plane, the sums over every node of u_x^2, u_y^2, u_z^2;
- ``plane_drho2`` [256]: per z plane, the sum of (rho - 1)^2;
- ``ke``: (1/2N) sum |u|^2 over the whole lattice at steps 0 and 1000.

It calls only the oracle and the input generators, so every stored value comes from the
oracle.  Run it from the repository root: ``python tests/golden/make_c2_reference.py``
(about 25 minutes on 8 cores, 10 GB of host memory).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_taylor_green_256.npz")
N_SIDE, STEPS, N_SAMPLES, SAMPLE_SEED = 256, 1000, 8192, 31337


def sample_nodes(n_nodes, count=N_SAMPLES, seed=SAMPLE_SEED):
    """Distinct node indices from a SplitMix64 counter hash, in draw order."""
    out, seen, k = [], set(), 0
    while len(out) < count:
        idx = np.arange(k, k + 2 * count, dtype=np.uint64)
        for v in (S.splitmix64(np.uint64(seed) ^ idx) % np.uint64(n_nodes)).astype(np.int64):
            if v not in seen:
                seen.add(v)
                out.append(v)
                if len(out) == count:
                    break
        k += 2 * count
    return np.array(out, dtype=np.int64)


def summarise(rho, u, n):
    r = rho[0].reshape(n, n * n)
    uu = u.reshape(3, n, n * n)
    return (uu * uu).sum(axis=2), ((r - 1.0) ** 2).sum(axis=1), 0.5 * float((u * u).sum()) / (n ** 3)


def main():
    c = S.c2_taylor_green(n=N_SIDE, steps=STEPS)
    t0 = time.time()
    o = oracle.Oracle.from_case(c)
    c.df = None  # the oracle holds its own copy of the initial populations
    ke0 = summarise(*o.macro(), N_SIDE)[2]
    done = 0
    while done < STEPS:
        o.run(100)
        done += 100
        print("oracle step %d (%.0f s)" % (done, time.time() - t0), flush=True)
    rho, u = o.macro()
    plane_u2, plane_drho2, ke1 = summarise(rho, u, N_SIDE)
    nodes = sample_nodes(N_SIDE ** 3)
    np.savez_compressed(OUT, nodes=nodes, rho=rho[0, nodes], u=u[:, nodes], plane_u2=plane_u2,
                        plane_drho2=plane_drho2, ke=np.array([ke0, ke1]), steps=np.array(STEPS),
                        n=np.array(N_SIDE))
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
