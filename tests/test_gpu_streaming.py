"""Non-temporal stores of the step's intermediates (flame_set_streaming_stores):
the same kernels with another store kind for Q, W or both, so every result must be
bitwise the plain-store result, for each kernel variant (both grids, both
points-per-thread choices, the split product kernel, forcing, Heun, graph
replays, ensembles), and the oracle's within the step's tolerance."""

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


def workload(n1, n2, seed, amp=0.05, t0=5.0, dt=0.2):
    return synth.Workload(f"s{n1}x{n2}", n1, n2, 1, dt, "disc", amp, -1.0, seed, max_norm=24, t0=t0)


def run(flame, w, half, steps, streaming, product=None, pts=None, graph_steps=0, integrator=0, forcing=None):
    print(f"case {w.n1}x{w.n2} streaming={streaming} product={product} pts={pts} graph={graph_steps} "
          f"integrator={integrator} forced={forcing is not None}", flush=True)
    sim = flame.FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, integrator=integrator)
    if product is not None:
        sim.set_product_grid(w.n1, w.n2, product)
    if pts is not None:
        sim.set_points_per_thread(w.n1, w.n2, *pts)
    sim.set_streaming_stores(w.n1, w.n2, streaming)
    assert sim.streaming_stores(w.n1, w.n2) == streaming
    if forcing is not None:
        sim.set_forcing(forcing)
    sim.set_graph_steps(graph_steps)
    sim.set_spectrum(half)
    sim.step(steps)
    torch.cuda.synchronize()
    return sim.spectrum().cpu().numpy()


@pytest.mark.parametrize("n1,n2,product,pts", [
    (16, 32, None, (16, 16)), (64, 128, None, (8, 8)), (256, 512, True, (16, 16)), (256, 512, True, (8, 16)),
    (256, 512, False, (16, 8)), (2048, 64, True, (16, 8)), (128, 4096, True, (16, 16)), (4096, 32, False, (8, 8))])
def test_streaming_stores_give_the_plain_bits(flame, n1, n2, product, pts):
    w = workload(n1, n2, seed=n1 + 11 * n2 + pts[0])
    half = synth.workload_spectrum(w)
    plain = run(flame, w, half, 6, False, product, pts)
    streamed = run(flame, w, half, 6, True, product, pts)
    assert np.array_equal(plain, streamed)
    for kind in (2, 3):  # W only, Q only
        assert np.array_equal(plain, run(flame, w, half, 6, kind, product, pts)), kind
    p = oracle.Params(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    ref = oracle_trajectory(half, p, [6])[6]
    assert rel_l2(ref, half) > 1e-3
    assert rel_l2(streamed, ref) < 1e-5


@pytest.mark.parametrize("integrator,forced", [(0, True), (1, False), (1, True)])
def test_streaming_stores_with_forcing_heun_and_graph_replays(flame, integrator, forced):
    n1, n2 = 256, 512
    w = workload(n1, n2, seed=70 + integrator + 2 * forced)
    half = synth.workload_spectrum(w)
    f = synth.forcing_spectrum(w, amp=1e-3) if forced else None
    plain = run(flame, w, half, 13, False, graph_steps=0, integrator=integrator, forcing=f)
    # a graph of 5 steps replayed twice, then 3 direct steps
    streamed = run(flame, w, half, 13, True, graph_steps=5, integrator=integrator, forcing=f)
    assert np.array_equal(plain, streamed)
    fo = oracle.half_to_full(np.asarray(f, dtype=np.complex128), n1, n2) if forced else None
    p = oracle.Params(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt,
                      integrator="rk2" if integrator else "euler", forcing=fo)
    assert rel_l2(streamed, oracle_trajectory(half, p, [13])[13]) < 1e-5


def test_streaming_is_set_per_grid_in_an_ensemble(flame):
    descs = [dict(n1=256, n2=512, t0=5.0, dt=0.2), dict(n1=64, n2=128, t0=5.0, dt=0.2),
             dict(n1=256, n2=512, t0=5.0, dt=0.2)]
    halves = [synth.workload_spectrum(workload(d["n1"], d["n2"], seed=90 + i)) for i, d in enumerate(descs)]
    outs = []
    for streaming in (False, True):
        ens = flame.FlameEnsemble(descs)
        if streaming:
            ens.set_streaming_stores(256, 512, True)
        assert ens.streaming_stores(256, 512) == streaming
        assert not ens.streaming_stores(64, 128)
        for i, h in enumerate(halves):
            ens.set_spectrum(h, flame=i)
        ens.set_graph_steps(4)
        ens.step(10)
        torch.cuda.synchronize()
        outs.append([ens.spectrum(i).cpu().numpy() for i in range(len(descs))])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    with pytest.raises(flame.native.FlameError):
        ens.set_streaming_stores(128, 128, True)
    with pytest.raises(flame.native.FlameError):
        ens.streaming_stores(512, 512)
    with pytest.raises(flame.native.FlameError):
        ens.set_streaming_stores(256, 512, 4)


def test_switching_the_store_kind_between_graph_replays(flame):
    """The setting discards the step graph; the next replay is rebuilt with the
    other kernels and continues the same trajectory bit for bit."""
    n1, n2 = 256, 512
    w = workload(n1, n2, seed=123)
    half = synth.workload_spectrum(w)
    ref = run(flame, w, half, 20, False, graph_steps=5)
    sim = flame.FlameSim(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    sim.set_graph_steps(5)
    sim.set_spectrum(half)
    for k, streaming in enumerate((False, True, 2, 3)):
        sim.set_streaming_stores(n1, n2, streaming)
        sim.step(5)
        assert sim.step_index == 5 * (k + 1)
    torch.cuda.synchronize()
    assert np.array_equal(sim.spectrum().cpu().numpy(), ref)
