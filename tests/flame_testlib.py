"""Helpers shared by the GPU tests: oracle runs and spectral norms (host only)."""

import numpy as np

import oracle
import synth


def weighted_sq(half):
    """sum over the full box of |c_k|^2 from a canonical half array (k2 > 0 counted twice)."""
    h = np.asarray(half, dtype=np.complex128)
    w = np.full(h.shape, 2.0)
    w[:, 0] = 1.0
    return float((w * np.abs(h) ** 2).sum())


def rel_l2(got, ref):
    """Relative L2 error of the physical field, from canonical half spectra (Parseval)."""
    return np.sqrt(weighted_sq(np.asarray(got) - np.asarray(ref)) / weighted_sq(ref))


def oracle_params(w):
    return oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)


def oracle_trajectory(half0, p, checkpoints):
    """Run the oracle from a canonical half array, returning half arrays at the given steps."""
    full = oracle.half_to_full(np.asarray(half0, dtype=np.complex128), p.n1, p.n2)
    out = {}
    cps = sorted(set(checkpoints))
    cur = oracle.run(full, p, 0)
    n = 0
    for c in cps:
        cur = oracle.run(cur, p, c - n, n_start=n)
        n = c
        out[c] = oracle.full_to_half(cur, p.n1, p.n2)
    return out


def workload_ic(name):
    w = synth.WORKLOADS[name]
    return w, synth.workload_spectrum(w)
