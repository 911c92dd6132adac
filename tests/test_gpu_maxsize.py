"""The largest supported transform lengths, 8192 and 16384, against the FP64
oracle: the step on both grids and points-per-thread variants, the adjoint
step, the area gradient, projection and synthesis, circles of 16384 points,
and a property check of one step of an 8192 x 8192 flame."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import oracle_trajectory, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def sim_or_skip(n1, n2, **kw):
    """A FlameSim, or a skip if this device's LDS per workgroup is below what
    the 8192-point kernels need (flame_init reports it)."""
    from paper_0911_2889_amd import FlameSim, native
    try:
        return FlameSim(n1, n2, **kw)
    except native.FlameError as e:
        if "bytes of LDS" in str(e):
            pytest.skip(str(e))
        raise


def workload(n1, n2, seed, amp=0.05, t0=5.0, dt=0.2, max_norm=24):
    return synth.Workload(f"m{n1}x{n2}", n1, n2, 1, dt, "disc", amp, -1.0, seed, max_norm=max_norm, t0=t0)


@pytest.mark.parametrize("n1,n2,product,pts", [
    (8192, 64, None, (16, 16)), (8192, 64, None, (8, 8)), (64, 8192, None, (16, 16)), (64, 8192, None, (8, 8)),
    (8192, 128, True, (16, 16)), (8192, 128, True, (8, 16)), (8192, 128, False, (16, 8)),
    (128, 8192, True, (16, 16)),
    (16384, 64, True, (16, 16)), (16384, 64, False, (16, 16)), (16384, 64, True, (12, 16)),
    (64, 16384, None, (16, 16)), (64, 16384, None, (16, 12)), (128, 16384, True, (12, 12))])
def test_step_at_the_largest_lengths_matches_oracle(n1, n2, product, pts):
    # modes up to |k| = 1000 reach deep into the long axis's box (K = 2047)
    w = workload(n1, n2, seed=n1 + n2 + pts[0], amp=0.02, max_norm=1000)
    half = synth.workload_spectrum(w)
    p = oracle.Params(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    refs = oracle_trajectory(half, p, [1, 10])
    assert rel_l2(refs[1], half) > 1e-3
    sim = sim_or_skip(n1, n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt)
    if product is not None:
        sim.set_product_grid(n1, n2, product)
    sim.set_points_per_thread(n1, n2, *pts)
    sim.set_spectrum(half)
    sim.step(1)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[1]) < 1e-6
    sim.step(9)
    assert rel_l2(sim.spectrum().cpu().numpy(), refs[10]) < 1e-5


def to_internal(half, n1, n2):
    s = np.zeros((n2 // 4, n1 // 2), dtype=np.complex64)
    s[:, 1:] = np.asarray(half).T
    return torch.from_numpy(s.reshape(-1)).to("cuda")


def from_internal(t, n1, n2):
    return t.cpu().numpy().reshape(n2 // 4, n1 // 2)[:, 1:].T.copy()


@pytest.mark.parametrize("n1,n2", [(8192, 64), (64, 8192), (8192, 128), (16384, 64), (64, 16384), (16384, 128)])
def test_adjoint_and_area_gradient_at_the_largest_lengths(n1, n2):
    t0, dt, n = 5.0, 0.2, 2
    state = synth.workload_spectrum(synth.Workload("s", n1, n2, 1, dt, "all", 0.3, -1.0, 5))
    lam = synth.workload_spectrum(synth.Workload("l", n1, n2, 1, dt, "all", 1.0, -1.0, 6))
    sim = sim_or_skip(n1, n2, t0=t0, dt=dt)
    st, li = to_internal(state, n1, n2), to_internal(lam, n1, n2)
    lo = torch.zeros_like(li)
    sim.adjoint_step(n, st, li, lo)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    sf = oracle.half_to_full(state.astype(np.complex128), n1, n2)
    lf = oracle.half_to_full(lam.astype(np.complex128), n1, n2)
    ref = oracle.full_to_half(oracle.step_adjoint(sf, lf, p, n), n1, n2)
    assert rel_l2(from_internal(lo, n1, n2), ref) < 1e-5
    g = torch.zeros_like(li)
    sim.area_gradient(n, st, g)
    ref_g = oracle.full_to_half(oracle.area_gradient(sf, p, n), n1, n2)
    assert rel_l2(from_internal(g, n1, n2), ref_g) < 1e-5


@pytest.mark.parametrize("n1,n2", [(8192, 32), (32, 8192), (16384, 32), (32, 16384)])
def test_projection_and_synthesis_at_the_largest_lengths(n1, n2):
    phi = synth.physical_noise(n1, n2, seed=3, kind="uniform", scale=1e-3)
    sim = sim_or_skip(n1, n2)
    sim.set_phi(phi)
    got = sim.spectrum().cpu().numpy()
    ref = oracle.full_to_half(oracle.symmetrise(oracle.project(phi.astype(np.float64))), n1, n2)
    assert rel_l2(got, ref) < 1e-6
    field = sim.phi().cpu().numpy()
    ref_field = oracle.synthesize(oracle.half_to_full(got.astype(np.complex128), n1, n2)).real
    assert np.linalg.norm(field - ref_field) / np.linalg.norm(ref_field) < 1e-6


@pytest.mark.parametrize("product", [True, False])
def test_full_8192_square_step_moves_the_mean_mode_by_the_velocity(product):
    """8192 x 8192 (16.8 M modes; too large for the oracle in a test): for the
    Euler step E_0 = 1 and the quadratic term's k = 0 entry is
    c_n sum_k |kappa|^2 |Phi~_k|^2, so Phi~_0 must grow by dt times the
    velocity diagnostic <Phi_t> (an FP64 sum over the spectrum, checked
    against the oracle at smaller sizes). The step forms that entry through
    the whole transform chain from every mode of the box."""
    n = 8192
    w = synth.Workload("sq", n, n, 1, 0.05, "all", 0.05, -1.0, 9, t0=20.0)
    half = synth.workload_spectrum(w)
    sim = sim_or_skip(n, n, t0=w.t0, dt=w.dt)
    sim.set_product_grid(n, n, product)
    sim.set_spectrum(half)
    d0 = sim.diagnostics()
    k1max = (half.shape[0] - 1) // 2
    phi0 = float(sim.spectrum()[k1max, 0].real)
    sim.step(1)
    spec = sim.spectrum()
    phi1 = float(spec[k1max, 0].real)
    assert abs((phi1 - phi0) - w.dt * d0["velocity"]) < 1e-4 * w.dt * d0["velocity"]
    assert sim.diagnostics()["finite"]
    # every other mode moved by its propagator and the quadratic term: the
    # state must stay Hermitian in its k2 = 0 column after the symmetrisation
    col0 = spec[:, 0].cpu().numpy()
    assert np.array_equal(col0[:k1max], np.conj(col0[k1max + 1:][::-1]))


def test_eight_points_per_thread_stops_at_8192():
    from paper_0911_2889_amd import native
    sim = sim_or_skip(16384, 64)
    with pytest.raises(native.FlameError) as err:
        sim.set_points_per_thread(16384, 64, 8, 16)
    assert err.value.code == native.FLAME_ERR_UNSUPPORTED_SIZE
    tried = sim.autotune(steps=1)
    assert sim.points_per_thread(16384, 64)[0] in (12, 16)
    # (16 | 16, 12) x rows (16, 8, 12), plain and non-temporal; + W only / Q only after a both choice
    assert tried in (2 * (1 * 3 + 2 * 3), 2 * (1 * 3 + 2 * 3) + 2)


def test_circles_of_16384_points_match_oracle():
    from paper_0911_2889_amd import CircleBatch
    n, count = 16384, 3
    spec = synth.circle_spectra(n, count, seed=4, amp=0.2)
    b = CircleBatch(n, count, gamma=0.8, seg=1.0, t0=6.0, dt=0.1)
    b.set_spectra(spec)
    b.step(1)
    one = b.states.cpu().numpy()
    b.step(9)
    ten = b.states.cpu().numpy()
    p = oracle.CircleParams(n, gamma=0.8, seg=1.0, t0=6.0, dt=0.1)
    w = np.full(n // 4, 2.0)
    w[0] = 1.0
    for c in range(count):
        f0 = oracle.half_to_circle(spec[c].astype(np.complex128), n)
        for got, steps, tol in ((one[c], 1, 1e-6), (ten[c], 10, 1e-5)):
            ref = oracle.circle_to_half(oracle.circle_run(f0, p, steps))
            err = np.sqrt((w * np.abs(got - ref) ** 2).sum() / (w * np.abs(ref) ** 2).sum())
            assert err < tol, (c, steps, err)
    d = b.diagnostics().cpu().numpy()
    assert (d[:, 3] == 1.0).all()
