"""Parity of the HIP step (through the C ABI) with the FP64 oracle."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import oracle_params, oracle_trajectory, rel_l2, weighted_sq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def flame():
    from paper_0911_2889_amd import FlameEnsemble, FlameSim  # noqa: F401
    import paper_0911_2889_amd
    return paper_0911_2889_amd


def make_sim(mod, w, **kw):
    return mod.FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, **kw)


def small_workload(n1, n2, seed, amp=1e-2, max_norm=None, dt=0.25, t0=200.0):
    return synth.Workload(f"t{n1}x{n2}", n1, n2, 1, dt, "disc" if max_norm else "all", amp, -1.0, seed,
                          max_norm=max_norm, t0=t0)


def test_spectrum_roundtrip_is_exact(flame):
    w = small_workload(64, 128, 1)
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    back = sim.spectrum().cpu().numpy()
    assert np.array_equal(back, half)


@pytest.mark.parametrize("n1,n2", [(16, 16), (32, 64), (128, 64), (256, 512), (2048, 128), (64, 4096)])
def test_projection_and_synthesis(flame, n1, n2):
    phi = synth.physical_noise(n1, n2, seed=n1 + n2, kind="uniform", scale=1e-3)
    w = small_workload(n1, n2, 0)
    sim = make_sim(flame, w)
    sim.set_phi(phi)
    got = sim.spectrum().cpu().numpy()
    ref = oracle.full_to_half(oracle.symmetrise(oracle.project(phi.astype(np.float64))), n1, n2)
    assert rel_l2(got, ref) < 1e-6
    # synthesis of the projected state against the oracle's synthesis of the same coefficients
    field = sim.phi().cpu().numpy()
    ref_field = oracle.synthesize(oracle.half_to_full(got.astype(np.complex128), n1, n2)).real
    assert np.linalg.norm(field - ref_field) / np.linalg.norm(ref_field) < 1e-6


@pytest.mark.parametrize("n1,n2,amp", [(16, 32, 1.0), (64, 128, 0.3), (128, 64, 0.3), (256, 512, 0.05),
                                       (512, 128, 0.1), (32, 4096, 0.02), (4096, 32, 0.02)])
def test_single_step_matches_oracle(flame, n1, n2, amp):
    # large amplitude and small t0 so the quadratic term is a sizeable part of the step
    w = small_workload(n1, n2, seed=n1 * 7 + n2, amp=amp, t0=5.0, dt=0.2)
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    sim.step(1)
    got = sim.spectrum().cpu().numpy()
    p = oracle_params(w)
    ref = oracle_trajectory(half, p, [1])[1]
    # the update must differ visibly from the initial state, and match the oracle
    assert rel_l2(ref, half) > 1e-3
    assert rel_l2(got, ref) < 1e-6


def test_axis_scales_and_theta(flame):
    n1, n2 = 64, 64
    w = small_workload(n1, n2, seed=5, amp=0.2, t0=5.0, dt=0.1)
    half = synth.workload_spectrum(w)
    sim = flame.FlameSim(n1, n2, gamma=0.6, theta_pi=2.0, t0=5.0, dt=0.1, axis_scale=(1.5, 0.5))
    sim.set_spectrum(half)
    sim.step(5)
    got = sim.spectrum().cpu().numpy()
    p = oracle.Params(n1, n2, gamma=0.6, theta_pi=2.0, t0=5.0, dt=0.1, axis_scale=(1.5, 0.5))
    ref = oracle_trajectory(half, p, [5])[5]
    assert rel_l2(got, ref) < 2e-6


def test_flame64x128_full_horizon(flame):
    w = synth.WORKLOADS["flame64x128"]
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    p = oracle_params(w)
    ref = oracle_trajectory(half, p, [50, 100, 150, 200])
    for n in (50, 100, 150, 200):
        sim.step(50)
        got = sim.spectrum().cpu().numpy()
        err = rel_l2(got, ref[n])
        assert err < 1e-5, (n, err)


def test_stress256x512_nonlinear(flame):
    w = synth.WORKLOADS["stress256x512"]
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    p = oracle_params(w)
    ref = oracle_trajectory(half, p, [100, 500])
    sim.step(100)
    assert rel_l2(sim.spectrum().cpu().numpy(), ref[100]) < 1e-5
    sim.step(400)
    got = sim.spectrum().cpu().numpy()
    assert rel_l2(got, ref[500]) < 1e-5


def test_repeat_runs_are_bitwise_identical(flame):
    w = small_workload(256, 512, seed=9, amp=0.05)
    half = synth.workload_spectrum(w)
    outs = []
    for _ in range(2):
        sim = make_sim(flame, w)
        sim.set_spectrum(half)
        sim.step(20)
        outs.append(sim.spectrum().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_workspace_poison_does_not_change_result(flame):
    # a workspace filled with NaN bytes before the plan is built must give the same
    # bits: no kernel may read an intermediate it has not written
    w = small_workload(128, 256, seed=10, amp=0.05)
    half = synth.workload_spectrum(w)
    res = []
    for fill in (None, 0xFF):
        sim = make_sim(flame, w, ws_fill=fill)
        sim.set_spectrum(half)
        sim.step(10)
        res.append(sim.spectrum().cpu().numpy())
    assert np.array_equal(res[0], res[1])


def test_diagnostics_match_oracle(flame):
    w = synth.WORKLOADS["stress256x512"]
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    p = oracle_params(w)
    full0 = oracle.half_to_full(half.astype(np.complex128), w.n1, w.n2)
    for n in (0, 40):
        if n:
            sim.step(n)
            full0 = oracle.run(full0, p, n)
        d = sim.diagnostics()
        r, v, a = oracle.diagnostics(oracle.symmetrise(full0), p, n)
        assert d["finite"]
        assert abs(d["mean_radius"] - r) < 1e-9 * r
        assert abs(d["velocity"] - v) < 2e-5 * abs(v)
        assert abs(d["area_excess"] - a) < 2e-5 * abs(a)


def test_nonfinite_state_is_flagged(flame):
    w = small_workload(64, 64, seed=3)
    half = synth.workload_spectrum(w)
    half[3, 4] = np.nan
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    assert not sim.diagnostics()["finite"]
    # the host-synchronising call reports it as FLAME_ERR_NONFINITE
    with pytest.raises(flame.native.FlameError) as err:
        sim.check_finite()
    assert err.value.code == flame.native.FLAME_ERR_NONFINITE
    ok = make_sim(flame, w)
    ok.set_spectrum(synth.workload_spectrum(w))
    d = ok.check_finite()
    assert d["finite"] and d == ok.diagnostics()


def test_ensemble_members_match_solo_runs(flame):
    specs = [(64, 128, 1), (64, 128, 2), (128, 64, 3), (256, 512, 4), (64, 128, 5)]
    descs, halves = [], []
    for n1, n2, seed in specs:
        w = small_workload(n1, n2, seed, amp=0.05)
        descs.append(dict(n1=n1, n2=n2, gamma=0.8, theta_pi=1.0, t0=200.0, dt=0.25))
        halves.append(synth.workload_spectrum(w))
    ens = flame.FlameEnsemble(descs)
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    ens.step(10)
    for f, (n1, n2, seed) in enumerate(specs):
        solo = flame.FlameSim(n1, n2, t0=200.0, dt=0.25)
        solo.set_spectrum(halves[f])
        solo.step(10)
        assert np.array_equal(ens.spectrum(f).cpu().numpy(), solo.spectrum().cpu().numpy())


def test_checkpoint_restart_equivalence(flame):
    w = small_workload(128, 256, seed=12, amp=0.05)
    half = synth.workload_spectrum(w)
    a = make_sim(flame, w)
    a.set_spectrum(half)
    a.step(30)
    b = make_sim(flame, w)
    b.set_spectrum(half)
    b.step(12)
    saved = b.states[0].clone()
    b.step(5)  # wander off, then restore
    b.states[0].copy_(saved)
    b.state_modified(12)
    b.step(18)
    assert np.array_equal(a.spectrum().cpu().numpy(), b.spectrum().cpu().numpy())


def test_zero_state_stays_zero(flame):
    w = small_workload(64, 128, seed=1)
    sim = make_sim(flame, w)
    sim.set_spectrum(np.zeros(sim.half_shape(), dtype=np.complex64))
    sim.step(5)
    assert weighted_sq(sim.spectrum().cpu().numpy()) == 0.0


@pytest.mark.parametrize("n1,n2", [(64, 128), (256, 512), (2048, 64), (32, 4096), (4096, 32)])
@pytest.mark.parametrize("cp,rp", [(8, 8), (8, 16), (16, 8)])
def test_points_per_thread_variants_match_oracle(flame, n1, n2, cp, rp):
    w = small_workload(n1, n2, seed=n1 + 3 * n2 + cp + rp, amp=0.05, t0=5.0, dt=0.2)
    half = synth.workload_spectrum(w)
    sim = make_sim(flame, w)
    if n1 >= 128:
        sim.set_product_grid(n1, n2, False)  # col_pts applies to the N1-row grid
    sim.set_points_per_thread(n1, n2, cp, rp)
    assert sim.points_per_thread(n1, n2) == (cp, rp)
    sim.set_spectrum(half)
    sim.step(3)
    got = sim.spectrum().cpu().numpy()
    ref = oracle_trajectory(half, oracle_params(w), [3])[3]
    assert rel_l2(got, ref) < 2e-6


@pytest.mark.parametrize("n1,n2", [(128, 256), (256, 64), (512, 1024), (1024, 128), (2048, 64), (4096, 32),
                                   (128, 4096)])
def test_product_grid_matches_oracle_and_physical_grid(flame, n1, n2):
    """The quadratic term formed on 3*N1/4 theta rows: one step and 20 steps
    against the oracle (which forms it on the N1 x N2 augmented grid of
    Section 3), and against the same run on N1 rows, for several points per
    thread of the column and row kernels."""
    w = small_workload(n1, n2, seed=n1 + 5 * n2, amp=0.1, t0=5.0, dt=0.2)
    half = synth.workload_spectrum(w)
    p = oracle_params(w)
    refs = oracle_trajectory(half, p, [1, 20])
    assert rel_l2(refs[1], half) > 1e-3
    runs = {}
    for product in (True, False):
        for cp, rp in ((16, 16), (8, 8), (8, 16)):
            sim = make_sim(flame, w)
            assert sim.product_grid(n1, n2)  # the default for n1 >= 128
            sim.set_product_grid(n1, n2, product)
            sim.set_points_per_thread(n1, n2, cp, rp)
            assert sim.product_grid(n1, n2) == product
            sim.set_spectrum(half)
            sim.step(1)
            one = sim.spectrum().cpu().numpy()
            sim.step(19)
            twenty = sim.spectrum().cpu().numpy()
            assert rel_l2(one, refs[1]) < 1e-6, (product, cp, rp)
            assert rel_l2(twenty, refs[20]) < 1e-5, (product, cp, rp)
            runs[(product, cp, rp)] = twenty
    assert rel_l2(runs[(True, 16, 16)], runs[(False, 16, 16)]) < 2e-6
    assert rel_l2(runs[(True, 8, 8)], runs[(True, 16, 16)]) < 2e-6


def test_product_grid_switches_mid_run_and_keeps_diagnostics(flame):
    """Switching grids between steps rebuilds the intermediates; diagnostics
    (a grid mean on the N1 x N2 grid) do not disturb the product grid's step."""
    n1, n2 = 256, 512
    w = small_workload(n1, n2, seed=77, amp=0.1, t0=5.0, dt=0.2)
    half = synth.workload_spectrum(w)
    p = oracle_params(w)
    refs = oracle_trajectory(half, p, [10, 20, 30])
    sim = make_sim(flame, w)
    sim.set_spectrum(half)
    sim.step(10)
    d = sim.diagnostics()
    ref_area = oracle.diagnostics(oracle.half_to_full(refs[10], n1, n2), p, 10)[2]
    assert abs(d["area_excess"] - ref_area) < 2e-5 * abs(ref_area)
    sim.step(10)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[20]) < 1e-5
    sim.set_product_grid(n1, n2, False)
    sim.step(5)
    sim.set_product_grid(n1, n2, True)
    sim.step(5)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[30]) < 1e-5
    with pytest.raises(RuntimeError):
        small = make_sim(flame, small_workload(64, 128, 1))
        small.set_product_grid(64, 128, True)


def r0_table(p, n_entries):
    """The oracle's reference-radius scalars as the library's table rows
    (r0(t_n), I1_n, I2_n); I1, I2 by the oracle's FP64 quadrature."""
    rows = []
    for n in range(n_entries):
        _, i1, i2 = oracle.step_scalars(p, n)
        rows.append((p.r0(p.time(n)), i1, i2))
    return torch.tensor(rows, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n1,n2,product", [(64, 128, False), (256, 512, True), (256, 512, False)])
def test_tabulated_reference_radius_matches_oracle(flame, n1, n2, product):
    """A reference radius other than the paper's r0 = t (here r0 = 2 + 0.5 t),
    given to the library as a table: steps, diagnostics and the adjoint step
    against the oracle integrating the same law by quadrature."""
    law = lambda t: 2.0 + 0.5 * t  # noqa: E731
    t0, dt, steps = 4.0, 0.2, 30
    w = small_workload(n1, n2, seed=n1 + 11, amp=0.05, t0=t0, dt=dt)
    half = synth.workload_spectrum(w)
    p = oracle.Params(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=t0, dt=dt, r0_law=law)
    refs = oracle_trajectory(half, p, [steps])
    p_t = oracle.Params(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=t0, dt=dt)
    assert rel_l2(refs[steps], oracle_trajectory(half, p_t, [steps])[steps]) > 1e-3  # the law matters
    sim = flame.FlameSim(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=t0, dt=dt, r0_law=1)
    if n1 >= 128:
        sim.set_product_grid(n1, n2, product)
    sim.set_spectrum(half)
    with pytest.raises(flame.native.FlameError):
        sim.step(1)  # no table yet
    sim.set_r0_table(r0_table(p, steps + 1))
    sim.step(steps)
    got = sim.spectrum().cpu().numpy()
    assert rel_l2(got, refs[steps]) < 1e-5
    d = sim.diagnostics()
    mr, vel, area = oracle.diagnostics(oracle.half_to_full(refs[steps], n1, n2), p, steps)
    # r_bar = r0(t) + Re Phi~_0: the FP32 mean mode within the parity budget
    phi0 = mr - law(p.time(steps))
    assert abs(d["mean_radius"] - mr) < 1e-5 * abs(phi0) + 1e-12 * mr
    assert abs(d["velocity"] - vel) < 2e-5 * abs(vel)
    assert abs(d["area_excess"] - area) < 2e-5 * abs(area)
    with pytest.raises(flame.native.FlameError):
        sim.step(2)  # the second step needs entry 31, beyond the table
    assert sim.step_index == steps
    # one adjoint step at n = 5 with the law's scalars
    lam = synth.workload_spectrum(small_workload(n1, n2, seed=n2 + 1, amp=1.0, t0=t0, dt=dt))
    st = sim.new_cotangent()
    st.copy_(sim.states[0])
    li = sim.new_cotangent()
    sim.set_spectrum(lam, n=steps)
    li.copy_(sim.states[0])
    lo = sim.new_cotangent()
    sim.adjoint_step(5, st, li, lo)
    sf = oracle.half_to_full(got.astype(np.complex128), n1, n2)
    lf = oracle.half_to_full(lam.astype(np.complex128), n1, n2)
    ref = oracle.full_to_half(oracle.step_adjoint(sf, lf, p, 5), n1, n2)
    sim.states[0].copy_(lo)
    assert rel_l2(sim.spectrum().cpu().numpy(), ref) < 1e-5


def test_degenerate_cases(flame):
    """gamma = 0 (no instability: every small mode decays), a step of 0
    steps, a very long time step, and a state holding only the mean mode
    (E_0 = 1 and the quadratic term vanishes, so it must not change)."""
    n1, n2 = 64, 128
    # gamma = 0 against the oracle, and every mode's magnitude decays
    w = small_workload(n1, n2, seed=21, amp=1e-4, t0=5.0, dt=0.2)
    half = synth.workload_spectrum(w)
    sim = flame.FlameSim(n1, n2, gamma=0.0, t0=w.t0, dt=w.dt)
    sim.set_spectrum(half)
    sim.step(10)
    got = sim.spectrum().cpu().numpy()
    p = oracle.Params(n1, n2, gamma=0.0, t0=w.t0, dt=w.dt)
    assert rel_l2(got, oracle_trajectory(half, p, [10])[10]) < 1e-5
    nz = np.abs(half) > 0
    assert np.all(np.abs(got[nz]) < np.abs(half[nz]))
    # zero steps change nothing, not even the step index
    before = sim.spectrum().cpu().numpy()
    sim.step(0)
    assert sim.step_index == 10 and np.array_equal(sim.spectrum().cpu().numpy(), before)
    # a long step (dt = 50 at t0 = 200): high modes are damped to zero, no overflow
    w2 = small_workload(n1, n2, seed=22, amp=1e-2, t0=200.0, dt=50.0)
    half2 = synth.workload_spectrum(w2)
    sim2 = make_sim(flame, w2)
    sim2.set_spectrum(half2)
    sim2.step(3)
    got2 = sim2.spectrum().cpu().numpy()
    assert np.all(np.isfinite(got2))
    assert rel_l2(got2, oracle_trajectory(half2, oracle_params(w2), [3])[3]) < 1e-5
    # only the mean mode: unchanged bit for bit, everything else stays zero
    k1max = (half.shape[0] - 1) // 2
    mean_only = np.zeros_like(half)
    mean_only[k1max, 0] = np.complex64(0.37)
    sim3 = make_sim(flame, w)
    sim3.set_spectrum(mean_only)
    sim3.step(7)
    assert np.array_equal(sim3.spectrum().cpu().numpy(), mean_only)
