"""Graph-launched stepping and mixed-grid ensembles against eager runs and the oracle."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import oracle_params, oracle_trajectory, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def member_descs(members):
    return [dict(n1=w.n1, n2=w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt) for w in members]


def test_graph_replays_match_eager_steps():
    from paper_0911_2889_amd import FlameSim
    w = synth.Workload("g", 128, 256, 1, 0.25, "disc", 1e-2, -1.0, 31, max_norm=20)
    half = synth.workload_spectrum(w)
    eager = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
    eager.set_spectrum(half)
    graph = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
    graph.set_spectrum(half)
    graph.set_graph_steps(10)
    for rep in range(4):
        eager.step(10)
        graph.step(10)  # one replay of the same instantiated graph
        # eager work and a synchronisation between replays
        d = graph.diagnostics()
        torch.cuda.synchronize()
        assert d["finite"]
        assert graph.step_index == eager.step_index == 10 * (rep + 1)
        assert np.array_equal(graph.spectrum().cpu().numpy(), eager.spectrum().cpu().numpy()), rep


def test_graph_with_remainder_and_restart():
    from paper_0911_2889_amd import FlameSim
    w = synth.Workload("g", 64, 128, 1, 0.25, "disc", 1e-2, -1.0, 32, max_norm=12)
    half = synth.workload_spectrum(w)
    a = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
    a.set_spectrum(half)
    a.step(37)
    b = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
    b.set_graph_steps(8)
    b.set_spectrum(half)
    b.step(25)          # 3 graphs + 1 direct step
    saved = b.states[0].clone()
    b.step(3)
    b.states[0].copy_(saved)
    b.state_modified(25)  # stale intermediates are rebuilt before the next graph
    b.step(12)          # 1 graph + 4 direct steps
    assert b.step_index == 37
    assert np.array_equal(a.spectrum().cpu().numpy(), b.spectrum().cpu().numpy())


def test_small_mixed_ensemble_graph():
    from paper_0911_2889_amd import FlameEnsemble, FlameSim
    members = []
    for i, (n1, n2) in enumerate([(64, 128)] * 5 + [(128, 256)] * 3 + [(256, 512)] * 2 + [(128, 64)]):
        members.append(synth.Workload(f"m{i}", n1, n2, 40, 0.25, "disc", 1e-3, -1.0, 2000 + i, max_norm=16))
    ens = FlameEnsemble(member_descs(members))
    ens.set_graph_steps(20)
    halves = [synth.workload_spectrum(w) for w in members]
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    ens.step(40)
    for f, w in enumerate(members):
        solo = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
        solo.set_spectrum(halves[f])
        solo.step(40)
        assert np.array_equal(ens.spectrum(f).cpu().numpy(), solo.spectrum().cpu().numpy()), f
    for f in (0, 5, 8, 10):
        ref = oracle_trajectory(halves[f], oracle_params(members[f]), [40])[40]
        assert rel_l2(ens.spectrum(f).cpu().numpy(), ref) < 1e-5


def test_full_ensemble_256_flames():
    """The batched workload: 128 x 128x256, 96 x 256x512, 32 x 512x1024, 200 steps,
    one graph of 50 steps per launch; every member equals its solo run bit for
    bit, and two members per grid match the FP64 oracle."""
    from paper_0911_2889_amd import FlameEnsemble, FlameSim
    members = synth.ensemble_members()
    assert len(members) == 256
    ens = FlameEnsemble(member_descs(members))
    ens.set_graph_steps(50)
    halves = [synth.workload_spectrum(w) for w in members]
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    ens.step(200)
    for f, w in enumerate(members):
        solo = FlameSim(w.n1, w.n2, t0=w.t0, dt=w.dt)
        solo.set_spectrum(halves[f])
        solo.step(200)
        assert np.array_equal(ens.spectrum(f).cpu().numpy(), solo.spectrum().cpu().numpy()), f
        solo.close()
    for f in (0, 127, 128, 223, 224, 255):
        ref = oracle_trajectory(halves[f], oracle_params(members[f]), [200])[200]
        err = rel_l2(ens.spectrum(f).cpu().numpy(), ref)
        assert err < 1e-5, (f, err)
    assert all(ens.diagnostics(f)["finite"] for f in range(0, 256, 17))


@pytest.mark.parametrize("graph_steps", [0, 6])
def test_autotune_keeps_the_state_and_agrees_with_the_oracle(graph_steps):
    """With and without graph replays set on the plan."""
    from paper_0911_2889_amd import FlameEnsemble
    members = [synth.Workload(f"a{i}", n1, n2, 20, 0.25, "disc", 1e-3, -1.0, 3000 + i, max_norm=12)
               for i, (n1, n2) in enumerate([(64, 128), (64, 128), (256, 512), (128, 64)])]
    ens = FlameEnsemble(member_descs(members))
    ens.set_graph_steps(graph_steps)
    halves = [synth.workload_spectrum(w) for w in members]
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f, n=0)
    ens.step(5)
    before = [ens.spectrum(f).cpu().numpy() for f in range(len(members))]
    # per group: (col, row) points per thread in {16, 8} x {16, 8, 12} on N1
    # rows (12 rows: the phi product grid, n2 >= 64), and {16, 8, 12}^2 on the
    # theta product grid where n1 >= 128 (256x512 and 128x64), each with
    # plain and with non-temporal stores
    # (a group whose choice has Q and W non-temporal also times W only and Q only)
    tried = ens.autotune(steps=4)
    assert tried - (12 + 30 + 30) in (0, 2, 4, 6), tried
    assert ens.step_index == 5
    for f in range(len(members)):
        assert np.array_equal(ens.spectrum(f).cpu().numpy(), before[f])
        assert ens.points_per_thread(members[f].n1, members[f].n2)[0] in (8, 12, 16)
    ens.step(15)
    for f in range(len(members)):
        ref = oracle_trajectory(halves[f], oracle_params(members[f]), [20])[20]
        assert rel_l2(ens.spectrum(f).cpu().numpy(), ref) < 1e-5
