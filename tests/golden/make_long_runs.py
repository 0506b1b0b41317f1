"""Writes the stored oracle results of the long full-size parity runs.

TEST INFRASTRUCTURE.  This script calls only the FP64 oracle (`oracle/`) and the seeded
input generators (`workloads/`); nothing here comes from the GPU library.  The GPU tests
(tests/test_gpu_sparse.py, tests/test_gpu_bf16.py, tests/test_gpu_fullsize_next.py)
regenerate the same inputs from the same seeds and compare against these files.

  c1_prefix.npz  the headline workload (CSR 1,000,000 x 500,000, 10 distinct uniform
                 columns per row, values N(0,1) e^(r_i + c_j), r, c ~ N(0, 2^2), generator
                 seed 1001), Algorithm 1 (Section 3.2) with k = 16 probes per step,
                 gamma = 0.1, M = 10, alpha = (n/m)^(1/4), beta = (m/n)^(1/4), probe seed
                 2001: u_bar and v_bar after 500, 1000 and 2000 steps (the benchmarked
                 run), at every STRIDE-th row and column (original order).  The running
                 average after T steps does not depend on how many steps follow.
  c3_bf16.npz    dense 16384 x 8192, sigma = 3, generator seed 1003, rounded to bf16
                 (round-to-nearest-even, once, from FP64); the oracle runs on the rounded
                 values in FP64.  Algorithm 1 with k = 64, gamma = 0.1, M = 10, probe
                 seed 2003, 500 steps: u_bar, v_bar in full.
  var_targets.npz, var_blocks.npz  the Section 6 variants on the headline matrix, 500
                 steps (k = 16, gamma = VAR_GAMMA = 4, M = 10, probe seed 2001; at
                 gamma = 0.1 these runs are chaotic: rounding-level changes of the
                 estimates move u_bar by O(1e-2 - 1) within 100 steps, while at gamma = 4
                 they die out): per-index squared
                 targets alpha^2 U[0.5, 2] and beta^2 U[0.5, 2] (numpy default_rng(5),
                 rows then columns), and row blocks of 16 / column blocks of 8 with the
                 default alpha, beta; u_bar, v_bar at every STRIDE-th index.
  var_symmetric.npz  Algorithm 2 on the symmetric 1,000,000 x 1,000,000 matrix
                 (symmetric_sparse, 5 random columns per row of G, sigma = 2, seed 1005),
                 alpha = 1, 500 steps, gamma = VAR_GAMMA, same other parameters: u_bar at
                 every STRIDE-th index.

Usage: python tests/golden/make_long_runs.py [c1] [c3] [var_targets] [var_blocks] [var_symmetric]
       (c1: ~40 min, c3: ~3 min, each variant ~10-15 min)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import algorithm1 as A1  # noqa: E402
from oracle import variants as V  # noqa: E402
from workloads import round_to_bf16, scaled_dense, scaled_sparse, symmetric_sparse  # noqa: E402

STRIDE = 13
C1 = dict(m=1_000_000, n=500_000, nnz_row=10, sigma=2.0, gen_seed=1001, k=16, gamma=0.1, M=10.0,
          seed=2001, checkpoints=(500, 1000, 2000))
C3 = dict(m=16384, n=8192, sigma=3.0, gen_seed=1003, k=64, gamma=0.1, M=10.0, seed=2003, steps=500)


def make_c1(path):
    c = C1
    csr = scaled_sparse(c["m"], c["n"], c["nnz_row"], c["sigma"], c["gen_seed"])
    al, be = A1.default_alpha_beta(c["m"], c["n"])
    ri = np.arange(0, c["m"], STRIDE)
    ci = np.arange(0, c["n"], STRIDE)
    saved = {}
    t_start = time.time()

    def on_step(t, u, v, u_bar, v_bar):
        if t % 20 == 0:
            print(f"c1 oracle step {t} ({time.time() - t_start:.0f} s)", flush=True)
        if t in c["checkpoints"]:
            saved[f"u_bar_{t}"] = u_bar[ri].copy()
            saved[f"v_bar_{t}"] = v_bar[ci].copy()

    A1.equilibrate(csr.to_scipy(), al, be, c["gamma"], c["M"], max(c["checkpoints"]), k=c["k"],
                   seed=c["seed"], on_step=on_step)
    np.savez(path, stride=np.int32(STRIDE), checkpoints=np.array(c["checkpoints"], dtype=np.int32), **saved)


def make_c3(path):
    c = C3
    A = scaled_dense(c["m"], c["n"], c["sigma"], c["gen_seed"])
    _, Ar = round_to_bf16(A)
    del A
    al, be = A1.default_alpha_beta(c["m"], c["n"])
    t_start = time.time()

    def on_step(t, u, v, u_bar, v_bar):
        if t % 25 == 0:
            print(f"c3 oracle step {t} ({time.time() - t_start:.0f} s)", flush=True)

    o = A1.equilibrate(Ar, al, be, c["gamma"], c["M"], c["steps"], k=c["k"], seed=c["seed"], on_step=on_step)
    np.savez(path, u_bar=o["u_bar"], v_bar=o["v_bar"], steps=np.int32(c["steps"]))


VAR_STEPS = 500
VAR_GAMMA = 4.0


def variant_inputs():
    """The headline matrix with the variants' targets and block boundaries."""
    c = C1
    csr = scaled_sparse(c["m"], c["n"], c["nnz_row"], c["sigma"], c["gen_seed"])
    al, be = A1.default_alpha_beta(c["m"], c["n"])
    g = np.random.default_rng(5)
    rt = al**2 * g.uniform(0.5, 2.0, c["m"])
    ct = be**2 * g.uniform(0.5, 2.0, c["n"])
    rp = list(range(0, c["m"], 16)) + [c["m"]]
    cp = list(range(0, c["n"], 8)) + [c["n"]]
    return csr, al, be, rt, ct, rp, cp


def make_var(kind, path):
    c = C1
    if kind == "var_symmetric":
        S = symmetric_sparse(1_000_000, 5, 2.0, 1005)
        o = V.equilibrate_symmetric(S.to_scipy(), 1.0, VAR_GAMMA, c["M"], VAR_STEPS, k=c["k"], seed=c["seed"])
        np.savez(path, stride=np.int32(STRIDE), steps=np.int32(VAR_STEPS), gamma=np.float64(VAR_GAMMA),
                 u_bar=o["u_bar"][::STRIDE].copy())
        return
    csr, al, be, rt, ct, rp, cp = variant_inputs()
    As = csr.to_scipy()
    if kind == "var_targets":
        o = V.equilibrate_general(As, VAR_GAMMA, c["M"], VAR_STEPS, k=c["k"], seed=c["seed"], row_target=rt,
                                  col_target=ct)
    else:
        o = V.equilibrate_general(As, VAR_GAMMA, c["M"], VAR_STEPS, k=c["k"], seed=c["seed"], row_ptr=rp,
                                  col_ptr=cp, alpha=al, beta=be)
    np.savez(path, stride=np.int32(STRIDE), steps=np.int32(VAR_STEPS), gamma=np.float64(VAR_GAMMA),
             u_bar=o["u_bar"][::STRIDE].copy(), v_bar=o["v_bar"][::STRIDE].copy())


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c3"]
    if "c1" in which:
        make_c1(os.path.join(HERE, "c1_prefix.npz"))
    if "c3" in which:
        make_c3(os.path.join(HERE, "c3_bf16.npz"))
    for kind in ("var_targets", "var_blocks", "var_symmetric"):
        if kind in which:
            t = time.time()
            make_var(kind, os.path.join(HERE, kind + ".npz"))
            print(f"{kind}: {time.time() - t:.0f} s", flush=True)
