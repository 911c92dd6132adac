"""Gradient of the final area excess for the 1024 x 2048 adjoint workload
(500 steps of dt = 0.1, checkpoints every 50 steps) against the FP64 oracle.

tests/golden/make_golden_adjoint.py wrote the fixture with the oracle alone:
J, the grid-value gradient at 4096 sampled nodes, and for 16 random
directions the directional derivative from the oracle's adjoint and from FP64
central differences of J. The GPU gradient comes from flame_area's backward
pass (the library's adjoint step, autograd Function, checkpointed recompute).
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "oracle_adjoint1024x2048_gradient.json")


def test_adjoint_workload_gradient_matches_oracle_and_differences():
    from paper_0911_2889_amd import FlameSim, flame_area

    if not os.path.exists(FIXTURE):
        pytest.skip("fixture has not been generated")
    with open(FIXTURE) as f:
        fx = json.load(f)
    w = synth.WORKLOADS["adjoint1024x2048"]
    assert fx["grid"] == [w.n1, w.n2] and fx["steps"] == w.steps and fx["seed"] == w.seed
    half = synth.workload_spectrum(w)
    sim = FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    sim.set_spectrum(half)
    phi0 = sim.phi().detach().clone().requires_grad_(True)  # the modal initial field on the grid
    J = flame_area(phi0, sim, w.steps, checkpoint_every=fx["checkpoint_every"])
    J.backward()
    grad = phi0.grad.double().cpu().numpy()
    assert abs(J.item() - fx["J"]) < 1e-5 * abs(fx["J"]), (J.item(), fx["J"])

    pts = fx["points"]
    got = grad[np.array(pts["j1"]), np.array(pts["j2"])]
    want = np.array(pts["grad"])
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 1e-5, err
    assert abs(np.linalg.norm(grad) - fx["grad_norm"]) < 1e-5 * fx["grad_norm"]

    # directions v_i: N(0,1) per node, projected onto the box and scaled to |phi0|;
    # the projection is orthogonal, so <grad, P v> is read off the GPU gradient
    for d in fx["directions"]:
        v = synth.physical_noise(w.n1, w.n2, seed=d["seed"], kind="normal").astype(np.float64)
        vp = oracle.synthesize(oracle.project(v)).real
        vp *= fx["norm_phi0"] / np.linalg.norm(vp)
        dd = float((grad * vp).sum())
        assert abs(dd - d["adjoint"]) < 1e-5 * abs(d["adjoint"]) + 1e-6 * fx["grad_norm"] * fx["norm_phi0"], d
        assert abs(dd - d["fd"]) < 1e-5 * abs(d["fd"]) + 1e-6 * fx["grad_norm"] * fx["norm_phi0"], d
