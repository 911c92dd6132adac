#!/usr/bin/env python3
"""Write the FP64 oracle's gradient of the area excess for the adjoint workload.

Calls only the oracle (and the seeded input generators). Workload: one flame
of 1024 x 2048, 500 steps of dt = 0.1 from t0 = 200, modal initial condition
(|k| <= 64, amplitudes 1e-3 N(0,1)/|k|, seed 5); J = area excess at the end.
Stored: J; the gradient with respect to the grid values of the initial field
at 4096 grid points drawn with numpy.random.default_rng(9); and for 16
directions v_i (N(0,1) per node with seed 500 + i, projected onto the box and
scaled to the norm of the initial field) the directional derivative <grad J, v_i>
from the adjoint and from FP64 central differences of J with step 1e-4.

    python tests/golden/make_golden_adjoint.py [n_directions]
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main(ndir):
    w = synth.WORKLOADS["adjoint1024x2048"]
    half = synth.workload_spectrum(w)
    p = oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    full0 = oracle.half_to_full(half.astype(np.complex128), w.n1, w.n2)
    t0 = time.time()
    value, lam = oracle.trajectory_gradient(full0, p, w.steps, checkpoint_every=50)
    grad = oracle.synthesize(lam).real
    print(f"adjoint done at {time.time() - t0:.0f} s, J = {value:.6e}", flush=True)
    rng = np.random.default_rng(9)
    j1 = rng.integers(0, w.n1, 4096)
    j2 = rng.integers(0, w.n2, 4096)
    phi0 = oracle.synthesize(full0).real
    norm0 = np.linalg.norm(phi0)
    dirs = []
    for i in range(ndir):
        v = synth.physical_noise(w.n1, w.n2, seed=500 + i, kind="normal").astype(np.float64)
        vp = oracle.synthesize(oracle.project(v)).real
        vp *= norm0 / np.linalg.norm(vp)
        adj = float((grad * vp).sum())
        eps = 1e-4
        vhat = oracle.analyse(vp) * oracle.box_mask(w.n1, w.n2)

        def J(x):
            return oracle.area_excess(oracle.run(x, p, w.steps), p, w.steps)

        fd = (J(full0 + eps * vhat) - J(full0 - eps * vhat)) / (2 * eps)
        dirs.append({"seed": 500 + i, "adjoint": adj, "fd": fd})
        print(f"direction {i}: adjoint {adj:.9e} fd {fd:.9e} rel {abs(adj - fd) / abs(fd):.2e} "
              f"at {time.time() - t0:.0f} s", flush=True)
    out = {"workload": w.name, "grid": [w.n1, w.n2], "steps": w.steps, "dt": w.dt, "t0": w.t0, "seed": w.seed,
           "checkpoint_every": 50, "J": value, "norm_phi0": float(norm0),
           "points": {"j1": j1.tolist(), "j2": j2.tolist(), "grad": [float(f"{x:.12e}") for x in grad[j1, j2]]},
           "grad_norm": float(np.linalg.norm(grad)), "directions": dirs}
    path = os.path.join(HERE, f"oracle_{w.name}_gradient.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 16)
