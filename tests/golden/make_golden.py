#!/usr/bin/env python3
"""Write sampled FP64 oracle states of the full-size workloads (test fixtures).

Calls only the oracle (and the seeded input generator for the initial
conditions). For each workload and checkpoint step it stores: a fixed sample
of spectral coefficients (all modes with |k1| <= 8, 0 <= k2 <= 16, plus 1024
modes drawn with numpy.random.default_rng(7) from the canonical half array),
the full weighted norm sum_k |Phi~_k|^2 over the box, and the oracle's
diagnostics (mean radius, averaged velocity, area excess).

    python tests/golden/make_golden.py flame512x1024 flame2048x4096
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CHECKPOINTS = {"flame512x1024": [200, 1000], "flame2048x4096": [50, 500], "adjoint1024x2048": [500]}


def sample_indices(shape):
    k1max = (shape[0] - 1) // 2
    rows, cols = [], []
    for a in range(-8, 9):
        for b in range(0, 17):
            rows.append(a + k1max)
            cols.append(b)
    rng = np.random.default_rng(7)
    flat = rng.choice(shape[0] * shape[1], size=1024, replace=False)
    rows += list((flat // shape[1]).tolist())
    cols += list((flat % shape[1]).tolist())
    return np.array(rows), np.array(cols)


def main(names):
    for name in names:
        w = synth.WORKLOADS[name]
        half = synth.workload_spectrum(w)
        p = oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
        cur = oracle.run(oracle.half_to_full(half.astype(np.complex128), w.n1, w.n2), p, 0)
        rows, cols = sample_indices(half.shape)
        out = {"workload": name, "grid": [w.n1, w.n2], "dt": w.dt, "t0": w.t0, "gamma": w.gamma,
               "theta_pi": w.theta_pi, "seed": w.seed, "rows": rows.tolist(), "cols": cols.tolist(),
               "checkpoints": {}}
        n = 0
        t0 = time.time()
        for c in CHECKPOINTS[name]:
            cur = oracle.run(cur, p, c - n, n_start=n)
            n = c
            h = oracle.full_to_half(cur, w.n1, w.n2)
            wgt = np.full(h.shape, 2.0)
            wgt[:, 0] = 1.0
            r, v, a = oracle.diagnostics(cur, p, n)
            out["checkpoints"][str(c)] = {
                "re": [float(f"{x:.12e}") for x in h[rows, cols].real],
                "im": [float(f"{x:.12e}") for x in h[rows, cols].imag],
                "norm_sq": float((wgt * np.abs(h) ** 2).sum()),
                "mean_radius": r, "velocity": v, "area_excess": a,
            }
            print(f"{name}: step {c} done at {time.time() - t0:.0f} s", flush=True)
        path = os.path.join(HERE, f"oracle_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CHECKPOINTS))
