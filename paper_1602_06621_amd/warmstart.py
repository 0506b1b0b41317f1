"""Learned warm start: training-set construction, training and use (orchestration over the
C ABI; every arithmetic step runs in libmfe's kernels).

Pipeline (see include/mfe.h, "learned warm start"):
  labels   plain Algorithm 1 (t0 = 0) run to convergence on generated matrices, all in
           one batched plan (one launch per direction and step for all matrices);
  features probe sketches of every row and column (mfe_plan_sketch_features);
  targets  label minus the sketch initialisation (the network learns the correction);
  training Adam on the mean squared error (mfe_mlp_train);
  use      u0 = clip(sketch init + MLP(features), -M, M), then Algorithm 1 with t0 > 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _ffi as F


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, in the flat order
    W1 (8 x 64), b1, W2 (64 x 64), b2, w3, b3."""
    s = F.mlp_sizes()
    nf, h = s["features"], s["width"]
    g = np.random.Generator(np.random.PCG64(seed))
    parts = [g.uniform(-1, 1, nf * h) / np.sqrt(nf), np.zeros(h), g.uniform(-1, 1, h * h) / np.sqrt(h), np.zeros(h),
             g.uniform(-1, 1, h) / np.sqrt(h), np.zeros(1)]
    theta = np.concatenate(parts)
    assert theta.size == s["params"]
    return torch.tensor(theta, dtype=torch.float32, device=device)


def training_set(plan, sketch_seed, label_out, per_matrix=4096, probes=4, gamma=0.1, M=10.0, seed=0):
    """(X, t) from a plan whose matrices were equilibrated into `label_out` (u_bar, v_bar):
    up to `per_matrix` rows and as many columns of every matrix, one per stratum
    (mfe_plan_training_set: features, label - sketch targets and the sampling all run in
    the library)."""
    X, t, _ = plan.training_set(sketch_seed, label_out["u_bar"], label_out["v_bar"], per_matrix=per_matrix,
                                sample_seed=seed, probes=probes, gamma=gamma, M=M)
    return X, t


def train(X, t, iters=1500, batch=4096, lr=2e-3, seed=0, init_seed=1):
    """Adam from a seeded initialisation.  Returns (params, loss trace)."""
    params = init_params(init_seed, device=X.device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = F.mlp_train(params, m, v, 0, X, t, batch, iters, lr, seed)
    return params, loss


def warm_start(plan, params, sketch_seed, probes=4, gamma=0.1, M=10.0, learned=True):
    """(u0, v0) for every matrix of the plan: the sketch initialisation, corrected by the
    network when learned is True (one library call, mfe_plan_warmstart)."""
    return plan.warm_start(params, sketch_seed, probes, gamma, M, learned)


def steps_to_residual(trace, target, every):
    """First step count at which a residual trace (one value every `every` steps) is at or
    below `target`; None if never."""
    hit = np.nonzero(np.asarray(trace) <= target)[0]
    return int((hit[0] + 1) * every) if hit.size else None


def tune_t0(plan, params, sketch_seed, alpha, beta, candidates=(5, 10, 20, 30, 50), learned=True, gamma=0.1,
            M=10.0, probes=16, seed=0, steps=1500, every=5, rel=1.2):
    """Step offset that reaches rel x (plain run's final residual) in the fewest steps on the
    single matrix of `plan` (a training-distribution matrix, not an evaluation one).
    Returns (best t0, {t0: steps})."""
    _, plain = plan.equilibrate_trace(alpha, beta, gamma, M, steps, probes, seed, trace_every=every)
    target = rel * plain[-1]
    u0, v0 = warm_start(plan, params, sketch_seed, gamma=gamma, M=M, learned=learned)
    got = {}
    for t0 in candidates:
        _, tr = plan.equilibrate_trace(alpha, beta, gamma, M, steps, probes, seed, t0=t0, u0=u0, v0=v0,
                                       trace_every=every)
        s = steps_to_residual(tr, target, every)
        got[t0] = s if s is not None else steps + 1
    best = min(got, key=lambda c: (got[c], c))
    return best, got
