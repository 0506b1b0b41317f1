"""Algorithm 1 of the paper (projected stochastic gradient for problem
(prob:reg-constr-equil), Section 3.2), in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper taken here:
  * Jacobi order: both the u and the v update at step t use (u^(t-1), v^(t-1)),
    exactly as Algorithm 1 writes D and E from the previous iterate.
  * k probes per step: the squared products are averaged over k independent
    probe columns.  k = 1 is Algorithm 1 verbatim.
  * Step offset t0 (0 = Algorithm 1): step size 2/(gamma (tau + 1)) and the
    running average weights use tau = t + t0.  Used by warm starts, where with
    t0 = 0 the first step (eta gamma = 1) would discard u^0.
  * The running average starts at the initial point (u_bar = u^0); with
    u^0 = 0 this is the paper's u_bar = 0.  The recursion
    u_bar <- 2 u^t/(tau+2) + tau u_bar/(tau+2) then equals the closed-form weights
    2(t+1)/((T+1)(T+2)) of Section 3.2 for t0 = 0.
  * A non-finite estimate or iterate is an error (the clip would hide a NaN).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import signs as _signs
from .theory import gradient_estimate


class NonFiniteError(ValueError):
    pass


def as_operator(A):
    """FP64 view of A: dense ndarray or scipy CSR (values cast exactly)."""
    if sp.issparse(A):
        return sp.csr_matrix(A, dtype=np.float64)
    return np.asarray(A, dtype=np.float64)


def step_size(gamma: float, tau: int) -> float:
    """eta_tau = 2 / (mu (tau + 1)) with mu = gamma (Section 3.2)."""
    return 2.0 / (gamma * (tau + 1.0))


def probes(seed, batch, t, m, n, k):
    """(S, W): S [n, k] for the A-side (side 0), W [m, k] for the A^T-side (side 1)."""
    S = _signs.signs(seed, batch, t, 0, n, k)
    W = _signs.signs(seed, batch, t, 1, m, k)
    return S, W


def equilibrate(A, alpha, beta, gamma, M, steps, k=1, seed=0, t0=0, u0=None, v0=None,
                batch=0, on_step=None, z_hook=None):
    """Run T = `steps` iterations of Algorithm 1.

    Returns a dict with u_bar, v_bar (the outputs, log D and log E), d = e^u_bar,
    e = e^v_bar, and the last iterates u, v.
    on_step(t, u, v, u_bar, v_bar) is called after every step (for tests).
    z_hook(z_u, z_v) -> (z_u, z_v) may perturb the estimates (sensitivity studies).
    """
    if not (alpha > 0 and beta > 0 and gamma > 0 and M > 0):
        raise ValueError("alpha, beta, gamma and M must be positive")
    if steps < 0 or k < 1:
        raise ValueError("steps must be >= 0 and k >= 1")
    A = as_operator(A)
    m, n = A.shape
    u = np.zeros(m) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(n) if v0 is None else np.array(v0, dtype=np.float64)
    u_bar = u.copy()
    v_bar = v.copy()
    for t in range(1, steps + 1):
        tau = t + t0
        S, W = probes(seed, batch, t, m, n, k)
        g_u, g_v, z_u, z_v = gradient_estimate(A, u, v, S, W, alpha, beta, gamma)
        if z_hook is not None:
            z_u, z_v = z_hook(z_u, z_v)
            g_u = z_u - alpha**2 + gamma * u
            g_v = z_v - beta**2 + gamma * v
        if not (np.all(np.isfinite(z_u)) and np.all(np.isfinite(z_v))):
            raise NonFiniteError(f"non-finite gradient estimate at step {t}")
        eta = step_size(gamma, tau)
        u_new = np.clip(u - eta * g_u, -M, M)
        v_new = np.clip(v - eta * g_v, -M, M)
        u_bar = 2.0 * u_new / (tau + 2.0) + tau * u_bar / (tau + 2.0)
        v_bar = 2.0 * v_new / (tau + 2.0) + tau * v_bar / (tau + 2.0)
        u, v = u_new, v_new
        if on_step is not None:
            on_step(t, u, v, u_bar, v_bar)
    return dict(u_bar=u_bar, v_bar=v_bar, d=np.exp(u_bar), e=np.exp(v_bar), u=u, v=v)


def default_alpha_beta(m: int, n: int):
    """alpha = (n/m)^(1/4), beta = (m/n)^(1/4) (Section 4): m alpha^2 = n beta^2, alpha beta = 1."""
    return (n / m) ** 0.25, (m / n) ** 0.25
