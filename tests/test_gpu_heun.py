"""Integrating-factor Heun (integrator 1) on the GPU against the FP64 oracle's
"rk2" step: grids, both product-grid settings and points-per-thread variants,
forcing, a tabulated reference radius, graph replays, mixed ensembles and the
full-size workload in the benchmark's launch configuration."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import oracle_trajectory, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def flame():
    import paper_0911_2889_amd
    return paper_0911_2889_amd


def workload(n1, n2, seed, amp=0.1, t0=5.0, dt=0.2):
    return synth.Workload(f"h{n1}x{n2}", n1, n2, 1, dt, "disc", amp, -1.0, seed, max_norm=24, t0=t0)


def params(w, integrator="rk2", **kw):
    return oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, integrator=integrator,
                         **kw)


def heun_sim(flame, w, **kw):
    return flame.FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, integrator=1, **kw)


@pytest.mark.parametrize("n1,n2,product,pts", [
    (16, 32, None, (16, 16)), (64, 128, None, (16, 16)), (64, 128, None, (8, 8)),
    (256, 512, True, (16, 16)), (256, 512, True, (8, 8)), (256, 512, False, (16, 16)),
    (256, 512, False, (8, 16)), (2048, 64, True, (16, 16)), (128, 4096, True, (8, 16)),
    (32, 4096, None, (16, 16)), (4096, 32, True, (16, 16)), (4096, 32, False, (16, 16))])
def test_heun_matches_oracle(flame, n1, n2, product, pts):
    w = workload(n1, n2, seed=n1 + 7 * n2)
    half = synth.workload_spectrum(w)
    refs = oracle_trajectory(half, params(w), [1, 20])
    euler = oracle_trajectory(half, params(w, "euler"), [1])[1]
    # the corrector must differ visibly from the Euler step it starts from
    assert rel_l2(refs[1], euler) > 1e-4
    sim = heun_sim(flame, w)
    if product is not None:
        sim.set_product_grid(n1, n2, product)
    sim.set_points_per_thread(n1, n2, *pts)
    sim.set_spectrum(half)
    sim.step(1)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[1]) < 1e-6
    sim.step(19)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[20]) < 1e-5


def test_heun_with_forcing_and_tabulated_radius(flame):
    n1, n2, steps = 256, 512, 20
    law = lambda t: 2.0 + 0.5 * t  # noqa: E731
    w = workload(n1, n2, seed=31)
    half = synth.workload_spectrum(w)
    fh = synth.forcing_spectrum(w, amp=0.02)
    p = params(w, r0_law=law, forcing=oracle.half_to_full(fh.astype(np.complex128), n1, n2))
    ref = oracle_trajectory(half, p, [steps])[steps]
    rows = []
    for n in range(steps + 1):
        _, i1, i2 = oracle.step_scalars(p, n)
        rows.append((p.r0(p.time(n)), i1, i2))
    table = torch.tensor(rows, dtype=torch.float64, device="cuda")
    sim = heun_sim(flame, w, r0_law=1)
    sim.set_spectrum(half)
    sim.set_forcing(fh)
    sim.set_r0_table(table[:steps])  # the corrector of step n reads entry n + 1
    with pytest.raises(flame.native.FlameError):
        sim.step(steps)
    sim.set_r0_table(table)
    sim.step(steps)
    assert rel_l2(sim.spectrum().cpu().numpy(), ref) < 1e-5


def test_heun_graph_replays_equal_direct_launches(flame):
    n1, n2 = 256, 512
    w = workload(n1, n2, seed=5)
    half = synth.workload_spectrum(w)
    out = []
    for gs in (0, 10):
        sim = heun_sim(flame, w)
        sim.set_graph_steps(gs)
        sim.set_spectrum(half)
        sim.step(25)  # two replays and five direct steps
        torch.cuda.synchronize()
        out.append(sim.spectrum().cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_mixed_integrators_in_one_plan(flame):
    """Euler and Heun flames of the same grid run in separate launch groups;
    each is bitwise its solo run."""
    base = dict(n1=256, n2=512, t0=5.0, dt=0.2)
    descs = [dict(base, integrator=0), dict(base, integrator=1), dict(base, integrator=1),
             dict(base, integrator=0), dict(n1=64, n2=128, t0=5.0, dt=0.2, integrator=1)]
    ens = flame.FlameEnsemble(descs)
    halves = []
    for i, d in enumerate(descs):
        h = synth.workload_spectrum(workload(d["n1"], d["n2"], seed=60 + i))
        halves.append(h)
        ens.set_spectrum(h, flame=i)
    ens.set_graph_steps(5)
    ens.step(12)
    for i, d in enumerate(descs):
        solo = flame.FlameSim(**d)
        solo.set_spectrum(halves[i])
        solo.step(12)
        assert np.array_equal(solo.spectrum().cpu().numpy(), ens.spectrum(flame=i).cpu().numpy()), i
    w = workload(256, 512, seed=61)
    ref = oracle_trajectory(halves[1], params(w), [12])[12]
    assert rel_l2(ens.spectrum(flame=1).cpu().numpy(), ref) < 1e-5


def test_heun_autotune_keeps_state_and_adjoint_is_refused(flame):
    n1, n2 = 256, 512
    w = workload(n1, n2, seed=8)
    half = synth.workload_spectrum(w)
    sim = heun_sim(flame, w)
    sim.set_spectrum(half)
    sim.step(3)
    before = sim.spectrum().cpu().numpy()
    assert sim.autotune(steps=2) in (30, 32)  # (grid, points per thread, store kind), + W only / Q only
    assert sim.step_index == 3
    assert np.array_equal(sim.spectrum().cpu().numpy(), before)
    sim.step(5)
    ref = oracle_trajectory(half, params(w), [8])[8]
    assert rel_l2(sim.spectrum().cpu().numpy(), ref) < 1e-5
    lam = sim.new_cotangent()
    with pytest.raises(flame.native.FlameError):
        sim.adjoint_step(3, sim.states[0], lam, lam)


def test_full_size_heun_steps_match_oracle(flame):
    """2048 x 4096 in the benchmark's launch configuration (autotuned, graph
    replays of 2 steps): two Heun steps against the FP64 oracle."""
    w = synth.WORKLOADS["flame2048x4096"]
    half = synth.workload_spectrum(w)
    ref = oracle_trajectory(half, params(w), [2])[2]
    sim = heun_sim(flame, w)
    sim.set_spectrum(half)
    sim.autotune(steps=3)
    sim.set_graph_steps(2)
    sim.set_spectrum(half)
    sim.step(2)
    got = sim.spectrum().cpu().numpy()
    assert rel_l2(got, half) > 1e-3
    assert rel_l2(got, ref) < 1e-5


@pytest.mark.parametrize("n1,n2", [(64, 128), (128, 256)])
def test_dt_convergence_orders_on_the_gpu(flame, n1, n2):
    """dt-convergence study of the GPU stepper over t in [5, 7] (amplitude 0.1,
    so the quadratic term matters) against DOP853 on the oracle's right-hand
    side of Eq. (1): the error falls by about 2 per halving of dt for Euler
    and by about 4 for Heun (observed orders 1 and 2)."""
    from scipy.integrate import solve_ivp

    w = synth.Workload("conv", n1, n2, 1, 0.2, "disc", 0.1, -1.0, 11, max_norm=24, t0=5.0)
    half = synth.workload_spectrum(w)
    t0, T = 5.0, 2.0
    full0 = oracle.run(oracle.half_to_full(half.astype(np.complex128), n1, n2), oracle.Params(n1, n2, t0=t0), 0)
    mask = oracle.box_mask(n1, n2)
    pp = oracle.Params(n1, n2, t0=t0, dt=1.0)
    sol = solve_ivp(lambda t, y: (oracle.rhs(y.reshape(n1, n2), pp, t) * mask).ravel(), (t0, t0 + T),
                    (full0 * mask).ravel(), method="DOP853", rtol=1e-12, atol=1e-16)
    ref = oracle.full_to_half(sol.y[:, -1].reshape(n1, n2), n1, n2)
    errs = {}
    for integ in (0, 1):
        errs[integ] = []
        for ns in (10, 20, 40, 80):
            sim = flame.FlameSim(n1, n2, t0=t0, dt=T / ns, integrator=integ)
            sim.set_spectrum(half)
            sim.step(ns)
            errs[integ].append(rel_l2(sim.spectrum().cpu().numpy(), ref))
    r_euler = [a / b for a, b in zip(errs[0], errs[0][1:])]
    r_heun = [a / b for a, b in zip(errs[1], errs[1][1:])]
    assert all(1.8 < r < 2.6 for r in r_euler), (errs, r_euler)
    assert all(3.0 < r < 4.6 for r in r_heun) and r_heun[-1] > 3.6, (errs, r_heun)
    assert errs[1][-1] < 0.1 * errs[0][-1]
