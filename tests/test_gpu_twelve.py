"""Parity of the 12-points-per-thread step kernels (through the C ABI) with
the FP64 oracle: the column transforms of length 3 N1/4 (product grid along
theta) and the row kernel that forms the quadratic term on 3 N2/4 phi points
(product grid along phi), alone and together, Euler, Heun and forced."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import oracle_params, oracle_trajectory, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def flame():
    import paper_0911_2889_amd
    return paper_0911_2889_amd


def make_sim(mod, w, **kw):
    return mod.FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, **kw)


def small_workload(n1, n2, seed, amp=0.1, dt=0.2, t0=5.0):
    return synth.Workload(f"t{n1}x{n2}", n1, n2, 1, dt, "all", amp, -1.0, seed, t0=t0)


@pytest.mark.parametrize("n1,n2", [(128, 256), (256, 64), (512, 1024), (1024, 128), (2048, 64), (4096, 64),
                                   (128, 4096), (8192, 64), (128, 8192)])
def test_twelve_point_kernels_match_oracle(flame, n1, n2):
    """One step and 20 steps on (col, row) points per thread (12, 12),
    (12, 16), (16, 12) and (8, 12), against the oracle (the quadratic term on
    the N1 x N2 augmented grid) and against the same run with (16, 16)."""
    w = small_workload(n1, n2, seed=n1 + 7 * n2)
    half = synth.workload_spectrum(w)
    refs = oracle_trajectory(half, oracle_params(w), [1, 20])
    assert rel_l2(refs[1], half) > 1e-3
    runs = {}
    for cp, rp in ((12, 12), (12, 16), (16, 12), (8, 12), (16, 16)):
        sim = make_sim(flame, w)
        sim.set_points_per_thread(n1, n2, cp, rp)
        assert sim.points_per_thread(n1, n2) == (cp, rp)
        sim.set_spectrum(half)
        sim.step(1)
        one = sim.spectrum().cpu().numpy()
        sim.step(19)
        twenty = sim.spectrum().cpu().numpy()
        assert rel_l2(one, refs[1]) < 1e-6, (cp, rp, rel_l2(one, refs[1]))
        assert rel_l2(twenty, refs[20]) < 1e-5, (cp, rp, rel_l2(twenty, refs[20]))
        runs[(cp, rp)] = twenty
    for key in runs:
        assert rel_l2(runs[key], runs[(16, 16)]) < 2e-6, key


@pytest.mark.parametrize("n1,n2", [(64, 128), (64, 4096)])
def test_twelve_point_rows_on_n1_grid(flame, n1, n2):
    """The phi product grid under the N1-row column kernel (n1 < 128 has no theta product grid)."""
    w = small_workload(n1, n2, seed=3 * n1 + n2)
    half = synth.workload_spectrum(w)
    ref = oracle_trajectory(half, oracle_params(w), [10])[10]
    sim = make_sim(flame, w)
    sim.set_points_per_thread(n1, n2, 16, 12)
    sim.set_spectrum(half)
    sim.step(10)
    assert rel_l2(sim.spectrum().cpu().numpy(), ref) < 1e-5


def test_twelve_point_configuration_errors(flame):
    w = small_workload(256, 512, seed=1)
    sim = make_sim(flame, w)
    sim.set_product_grid(256, 512, False)
    with pytest.raises(flame.native.FlameError):
        sim.set_points_per_thread(256, 512, 12, 16)  # the 12-point column kernel needs the product grid
    sim.set_product_grid(256, 512, True)
    sim.set_points_per_thread(256, 512, 12, 12)
    with pytest.raises(flame.native.FlameError):
        sim.set_product_grid(256, 512, False)
    small = small_workload(64, 32, seed=2)
    sim2 = make_sim(flame, small)
    with pytest.raises(flame.native.FlameError):
        sim2.set_points_per_thread(64, 32, 16, 12)  # n2 < 64


@pytest.mark.parametrize("n1,n2", [(256, 512), (1024, 128)])
def test_twelve_point_heun_and_forcing(flame, n1, n2):
    """Heun's two stages and a bound forcing on the 12-point kernels."""
    w = small_workload(n1, n2, seed=n1 + n2 + 11, amp=0.05)
    half = synth.workload_spectrum(w)
    fh = synth.forcing_spectrum(w, amp=1e-2)
    forcing_full = oracle.half_to_full(fh.astype(np.complex128), n1, n2)
    for integrator in ("euler", "rk2"):
        p = oracle.Params(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, forcing=forcing_full,
                          integrator=integrator)
        ref = oracle_trajectory(half, p, [10])[10]
        sim = make_sim(flame, w, integrator=integrator)
        sim.set_points_per_thread(n1, n2, 12, 12)
        sim.set_forcing(fh)
        sim.set_spectrum(half)
        sim.step(10)
        assert rel_l2(sim.spectrum().cpu().numpy(), ref) < 1e-5, integrator


def test_twelve_point_graph_replays_are_bitwise_direct(flame):
    w = small_workload(512, 1024, seed=5)
    half = synth.workload_spectrum(w)
    outs = []
    for gs in (0, 10):
        sim = make_sim(flame, w)
        sim.set_points_per_thread(512, 1024, 12, 12)
        sim.set_graph_steps(gs)
        sim.set_spectrum(half)
        sim.step(25)
        outs.append(sim.spectrum().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_twelve_point_full_size_steps_match_oracle(flame):
    """2048 x 4096 (the benchmark workload) with both 12-point kernels and
    non-temporal stores: 2 steps against the oracle on the whole box."""
    w = synth.WORKLOADS["flame2048x4096"]
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_points_per_thread(w.n1, w.n2, 12, 12)
    sim.set_streaming_stores(w.n1, w.n2, True)
    sim.set_spectrum(half)
    sim.step(2)
    got = sim.spectrum().cpu().numpy()
    ref = oracle_trajectory(half, oracle_params(w), [2])[2]
    assert rel_l2(got, ref) < 1e-6
