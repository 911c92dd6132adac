"""The persistent ensemble launch against per-group launches, graphs and the oracle."""

import numpy as np
import pytest

import synth
from flame_testlib import oracle_params, oracle_trajectory, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def member_descs(members):
    return [dict(n1=w.n1, n2=w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt) for w in members]


def make_ensemble(members, halves):
    """An ensemble on the persistent kernel's configuration (product grid,
    12 column and 16 row points per thread, plain stores), states set."""
    from paper_0911_2889_amd import FlameEnsemble
    ens = FlameEnsemble(member_descs(members))
    for n1, n2 in sorted({(w.n1, w.n2) for w in members}):
        ens.set_points_per_thread(n1, n2, 12, 16)
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    return ens


MIXED = [(128, 256)] * 5 + [(256, 512)] * 3 + [(512, 1024)] * 2 + [(1024, 2048), (128, 128), (256, 2048)]


@pytest.mark.parametrize("workgroups", [0, 6, 37])
def test_persistent_matches_direct_launches_bit_for_bit(workgroups):
    """Every grid the persistent kernel has bodies for, split over all the
    workgroups that fit (large flames over many parts), over one workgroup per
    grid group (several flames per workgroup), and over an uneven count; two
    calls in a row, so the second launch starts from the first one's counters."""
    members = [synth.Workload(f"p{i}", n1, n2, 30, 0.25, "disc", 1e-3, -1.0, 4100 + i, max_norm=16)
               for i, (n1, n2) in enumerate(MIXED)]
    halves = [synth.workload_spectrum(w) for w in members]
    print(f"persistent case: {len(members)} flames, workgroups {workgroups}", flush=True)
    direct = make_ensemble(members, halves)
    direct.step(30)
    pers = make_ensemble(members, halves)
    pers.set_persistent(True, workgroups=workgroups)
    pers.step(17)
    pers.step(13)
    on, wgs = pers.persistent()
    assert on and 6 <= wgs <= (workgroups or 4096)
    assert pers.step_index == direct.step_index == 30
    for f in range(len(members)):
        assert np.array_equal(pers.spectrum(f).cpu().numpy(), direct.spectrum(f).cpu().numpy()), f
    for f in (0, 5, 11):
        ref = oracle_trajectory(halves[f], oracle_params(members[f]), [30])[30]
        err = rel_l2(pers.spectrum(f).cpu().numpy(), ref)
        assert err < 1e-5, (f, err)


def test_persistent_full_ensemble_matches_graph_replays():
    """The 256-flame workload (128 x 128x256, 96 x 256x512, 32 x 512x1024),
    200 steps: one persistent launch against graphs of 50 steps, bit for bit,
    and members of each grid against the FP64 oracle."""
    members = synth.ensemble_members()
    halves = [synth.workload_spectrum(w) for w in members]
    print("persistent case: 256-flame ensemble, 200 steps", flush=True)
    graph = make_ensemble(members, halves)
    graph.set_graph_steps(50)
    graph.step(200)
    pers = make_ensemble(members, halves)
    pers.set_persistent(True)
    pers.step(200)
    assert pers.persistent()[1] > 0
    for f in range(len(members)):
        assert np.array_equal(pers.spectrum(f).cpu().numpy(), graph.spectrum(f).cpu().numpy()), f
    for f in (0, 128, 255):
        ref = oracle_trajectory(halves[f], oracle_params(members[f]), [200])[200]
        err = rel_l2(pers.spectrum(f).cpu().numpy(), ref)
        assert err < 1e-5, (f, err)
    assert all(pers.diagnostics(f)["finite"] for f in range(0, 256, 51))


def test_persistent_wait_limit_reports_a_timeout_and_the_plan_recovers():
    """A 1-microsecond bound on the waits of a flame shared by many
    workgroups runs out (the first workgroup at a counter waits for the
    others' atomics): flame_step reports FLAME_ERR_TIMEOUT after every
    workgroup has stopped. With the default bound the same plan then steps
    normally."""
    from paper_0911_2889_amd import native
    members = [synth.Workload("t0", 512, 1024, 10, 0.25, "disc", 1e-3, -1.0, 4200, max_norm=16)]
    halves = [synth.workload_spectrum(w) for w in members]
    print("persistent case: wait limit 1 us", flush=True)
    ens = make_ensemble(members, halves)
    ens.set_persistent(True, wait_limit_us=1)
    with pytest.raises(native.FlameError) as exc:
        ens.step(20)
    assert exc.value.code == native.FLAME_ERR_TIMEOUT
    ens.set_persistent(True)
    ens.set_spectrum(halves[0], flame=0, n=0)
    ens.step(10)
    direct = make_ensemble(members, halves)
    direct.step(10)
    assert np.array_equal(ens.spectrum(0).cpu().numpy(), direct.spectrum(0).cpu().numpy())


def test_persistent_refuses_configurations_it_has_no_kernel_for():
    from paper_0911_2889_amd import FlameEnsemble, native
    ens = FlameEnsemble([dict(n1=128, n2=256)])  # default: 16 column points per thread
    with pytest.raises(native.FlameError) as exc:
        ens.set_persistent(True)
    assert exc.value.code == native.FLAME_ERR_INVALID_ARG
    small = FlameEnsemble([dict(n1=64, n2=128)])  # no product grid below n1 = 128
    with pytest.raises(native.FlameError):
        small.set_persistent(True)
    ok = FlameEnsemble([dict(n1=128, n2=256)])
    ok.set_points_per_thread(128, 256, 12, 16)
    ok.set_persistent(True)
    with pytest.raises(native.FlameError) as exc:
        ok.autotune(steps=1)  # the persistent kernel's configuration is fixed
    assert exc.value.code == native.FLAME_ERR_INVALID_ARG
    ok.set_streaming_stores(128, 256, True)
    with pytest.raises(native.FlameError) as exc:
        ok.step(1)  # a later change the persistent kernel lacks is refused at the step
    assert exc.value.code == native.FLAME_ERR_INVALID_ARG


@pytest.mark.parametrize("graph_steps", [1, 8, 50])
def test_persistent_graph_replays_match_direct_launches_bit_for_bit(graph_steps):
    """The persistent launch captured in a graph of graph_steps steps (reset
    node, then the cooperative kernel node reading the step index from the
    workspace), replayed with a direct launch for the remainder: 30 and then
    23 steps, so replays start at several step indices, against per-group
    launches bit for bit."""
    members = [synth.Workload(f"g{i}", n1, n2, 30, 0.25, "disc", 1e-3, -1.0, 4300 + i, max_norm=16)
               for i, (n1, n2) in enumerate(MIXED)]
    halves = [synth.workload_spectrum(w) for w in members]
    print(f"persistent case: graph replays of {graph_steps} steps", flush=True)
    direct = make_ensemble(members, halves)
    direct.step(53)
    pers = make_ensemble(members, halves)
    pers.set_persistent(True)
    pers.set_graph_steps(graph_steps)
    pers.step(30)
    pers.step(23)
    assert pers.step_index == 53
    for f in range(len(members)):
        assert np.array_equal(pers.spectrum(f).cpu().numpy(), direct.spectrum(f).cpu().numpy()), f
    # a change of the wait bound rebuilds the graph; the plan keeps stepping
    pers.set_persistent(True, wait_limit_us=500000)
    pers.step(8)
    direct.step(8)
    for f in (0, 8, 12):
        assert np.array_equal(pers.spectrum(f).cpu().numpy(), direct.spectrum(f).cpu().numpy()), f


def test_persistent_configuration_from_any_autotuned_choice():
    """The benchmark's switch to the persistent kernel's configuration works from
    every choice the autotuner can leave a group in (N1 rows with 8 or 16 column
    points per thread, non-temporal stores), and the persistent launch then
    matches per-group launches on the same configuration bit for bit."""
    import bench
    members = [synth.Workload(f"c{i}", n1, n2, 30, 0.25, "disc", 1e-3, -1.0, 4400 + i, max_norm=16)
               for i, (n1, n2) in enumerate([(128, 256), (128, 256), (256, 512), (512, 1024)])]
    halves = [synth.workload_spectrum(w) for w in members]
    grids = sorted({(w.n1, w.n2) for w in members})
    from paper_0911_2889_amd import FlameEnsemble
    outs = []
    for persistent in (False, True):
        ens = FlameEnsemble(member_descs(members))
        for (n1, n2), (cp, stores) in zip(grids, ((8, 1), (16, 3), (16, 0))):
            ens.set_product_grid(n1, n2, False)
            ens.set_points_per_thread(n1, n2, cp, 16)
            ens.set_streaming_stores(n1, n2, stores)
        print(f"persistent case: configuration switch, persistent {persistent}", flush=True)
        bench.use_persistent_config(ens, grids)
        for n1, n2 in grids:
            assert ens.points_per_thread(n1, n2) == (12, 16) and ens.product_grid(n1, n2)
        for f, h in enumerate(halves):
            ens.set_spectrum(h, flame=f)
        if persistent:
            ens.set_persistent(True)
        ens.step(12)
        outs.append([ens.spectrum(f).cpu().numpy() for f in range(len(members))])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
