"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""

import numpy as np
import pytest

import oracle
import pins
import synth


def test_transform_convention_matches_bruteforce_dft():
    # Phi = sum_k Phi~_k exp(i k.x): synthesis without 1/P, analysis with 1/P
    for n1, n2, seed in ((8, 16, 0), (12, 20, 1), (16, 32, 2)):
        assert pins.pin_transform_bruteforce(n1, n2, seed) < 1e-13


def test_single_mode_synthesis_is_a_cosine():
    n1, n2, k, a, psi = 24, 40, (3, -5), 0.7, 1.3
    coef = {k: 0.5 * a * np.exp(1j * psi), (-k[0], -k[1]): 0.5 * a * np.exp(-1j * psi)}
    phys = oracle.synthesize(pins.dict_to_full(coef, n1, n2))
    j1 = np.arange(n1)[:, None]
    j2 = np.arange(n2)[None, :]
    ref = a * np.cos(2 * np.pi * (k[0] * j1 / n1 + k[1] * j2 / n2) + psi)
    assert np.abs(phys - ref).max() < 1e-14


@pytest.mark.parametrize("n1,n2,s,herm", [
    (13, 17, (1.0, 1.0), True),    # k0 = 0: the smallest augmented array
    (16, 16, (1.0, 1.0), True),    # k0 = 3: power of two
    (16, 24, (2.0, 0.5), True),    # anisotropic axis scales
    (13, 13, (1.0, 1.0), False),   # the identity holds for any coefficients
])
def test_quadratic_term_equals_literal_eq1_sum(n1, n2, s, herm):
    # Section 3: the augmented-array FFT product equals the convolution sum of Eq. (1)
    assert pins.pin_convolution_direct(n1, n2, seed=n1 + n2, s=s, hermitian=herm) < 1e-13


def test_quadratic_term_single_and_two_cosines():
    assert pins.pin_single_cosine() < 1e-14
    assert pins.pin_single_cosine(s=(1.5, 0.75)) < 1e-14
    assert pins.pin_two_cosines() < 1e-13


def test_linear_growth_matches_closed_form():
    # small-amplitude modes follow exp(int sigma_k dt) with r0 = t for any dt
    assert pins.pin_linear_growth(dt=1.0, nsteps=50) < 1e-12
    assert pins.pin_linear_growth(dt=10.0, nsteps=5) < 1e-12


def test_linear_growth_matches_ode_solver():
    assert pins.pin_linear_growth_ode() < 1e-10


def test_dispersion_relation_facts():
    # neutral wavenumber |k| = gamma r0 / (2 theta_pi): zero growth rate at t
    p = oracle.Params(400, 400, t0=200.0, dt=1e-6)
    ex = oracle.growth_exponent(p, 0)
    k1 = oracle.wavenumbers(400)
    i80 = int(np.nonzero(k1 == 80)[0][0])
    i40 = int(np.nonzero(k1 == 40)[0][0])
    assert abs(ex[i80, 0]) / 1e-6 < 1e-6
    # fastest growth at kappa = gamma r0 / 4 with rate gamma^2 / 16
    rate = ex[:, 0] / 1e-6
    assert int(k1[np.argmax(rate)]) == 40
    assert abs(rate[i40] - 0.8 ** 2 / 16) < 1e-6


def test_first_step_worked_example():
    assert pins.pin_first_step_worked_example() < 1e-13


def test_mean_mode_follows_parseval_identity():
    # k = 0 row of Eq. (1): d Phi~_0 / dt = c(t) sum_k |k|^2 |Phi~_k|^2
    assert pins.pin_k0_parseval() < 1e-13


def test_step_converges_first_order_to_eq1_solution():
    errs = pins.pin_convergence()
    assert errs[-1] < 5e-3
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2


def test_state_stays_hermitian_and_real():
    rng = np.random.default_rng(11)
    n1, n2 = 24, 32
    p = oracle.Params(n1, n2, t0=5.0, dt=0.2)
    full = pins.dict_to_full(pins.random_hermitian(n1, n2, rng, 0.3), n1, n2)
    out = oracle.run(full, p, 10)
    k1 = oracle.wavenumbers(n1)
    k2 = oracle.wavenumbers(n2)
    neg = out[np.ix_((-k1) % n1, (-k2) % n2)]
    assert np.array_equal(neg, np.conj(out))
    assert out[0, 0].imag == 0.0
    assert np.abs(oracle.synthesize(out).imag).max() < 1e-12 * np.abs(out).sum()
    assert np.all(out[~oracle.box_mask(n1, n2)] == 0)


def test_symmetrise_copies_upper_half():
    n = 12
    full = np.zeros((n, n), dtype=np.complex128)
    full[2, 1] = 1 + 2j          # k = (2, 1) in H
    full[n - 2, n - 1] = 5 + 5j  # k = (-2, -1): overwritten
    full[3, 0] = 1 - 1j          # k = (3, 0) in H
    full[0, 0] = 2 + 3j
    out = oracle.symmetrise(full)
    assert out[n - 2, n - 1] == 1 - 2j
    assert out[n - 3, 0] == 1 + 1j
    assert out[0, 0] == 2


def test_diagnostics_single_cosine():
    assert pins.pin_diagnostics_single_cosine() < 1e-13
    assert pins.pin_diagnostics_single_cosine(a=0.01, n=3) < 1e-12


def test_projection_recovers_band_limited_field():
    n1, n2 = 20, 28
    rng = np.random.default_rng(2)
    coef = pins.random_hermitian(n1, n2, rng)
    phys = pins.dft_synthesis(coef, n1, n2).real
    full = oracle.project(phys)
    ref = pins.dict_to_full(coef, n1, n2)
    assert np.abs(full - ref).max() < 1e-13


def test_half_layout_roundtrip():
    n1, n2 = 16, 24
    w = synth.Workload("t", n1, n2, 1, 0.1, "disc", 1e-3, -1.0, 9, max_norm=4)
    half = synth.workload_spectrum(w).astype(np.complex128)
    full = oracle.half_to_full(half, n1, n2)
    assert np.array_equal(oracle.full_to_half(full, n1, n2), half)
    assert np.array_equal(oracle.symmetrise(full), full)


def test_adjoint_dot_product():
    assert pins.pin_adjoint_dot_product() < 1e-12
    assert pins.pin_adjoint_dot_product(n1=13, n2=21, seed=8) < 1e-12


def test_area_gradient_matches_finite_differences():
    assert pins.pin_area_gradient_fd() < 1e-6


def test_trajectory_gradient_matches_finite_differences():
    assert pins.pin_trajectory_gradient_fd() < 1e-6


@pytest.mark.parametrize("every", [1, 3, 10])
def test_checkpointed_trajectory_gradient_matches_finite_differences(every):
    # the checkpoint branch (recomputed segments) from a nonzero step index
    assert pins.pin_trajectory_gradient_fd(n_start=5, checkpoint_every=every) < 1e-6


def test_checkpointed_gradient_is_bitwise_the_full_storage_one():
    assert pins.pin_checkpointed_gradient_identical() == 0
    assert pins.pin_checkpointed_gradient_identical(n1=13, n2=20, seed=11, nsteps=5, n_start=0) == 0


def test_area_excess_matches_series_and_diagnostics():
    assert pins.pin_area_excess_series() < 1e-12
    assert pins.pin_area_excess_series(k=(0, 5), a=0.3, n=0) < 1e-12


def test_gradient_is_band_limited():
    rng = np.random.default_rng(3)
    n1, n2 = 16, 24
    p = oracle.Params(n1, n2, t0=3.0, dt=0.2)
    phi0 = oracle.symmetrise(pins.dict_to_full(pins.random_hermitian(n1, n2, rng, 0.5), n1, n2))
    _, lam = oracle.trajectory_gradient(phi0, p, 4)
    assert np.all(lam[~oracle.box_mask(n1, n2)] == 0)
    grid = oracle.synthesize(lam)
    assert np.abs(grid.imag).max() < 1e-12 * np.abs(grid.real).max()


def test_general_r0_law_scalars_match_closed_forms():
    """A user reference-radius law goes through FP64 adaptive quadrature; for
    r0 = t and for a linear law r0 = a + b t the integrals have closed forms."""
    for n in (0, 7, 123):
        p0 = oracle.Params(16, 16, t0=200.0, dt=0.3)
        pq = oracle.Params(16, 16, t0=200.0, dt=0.3, r0_law=lambda t: t)
        c0, a0, b0 = oracle.step_scalars(p0, n)
        cq, aq, bq = oracle.step_scalars(pq, n)
        assert abs(cq - c0) <= 1e-15 * c0 and abs(aq - a0) <= 1e-13 * a0 and abs(bq - b0) <= 1e-13 * b0
    a, b, dt, t0 = 150.0, 0.5, 0.4, 3.0
    p = oracle.Params(16, 16, t0=t0, dt=dt, r0_law=lambda t: a + b * t)
    for n in (0, 11):
        t, t1 = t0 + n * dt, t0 + (n + 1) * dt
        c, i1, i2 = oracle.step_scalars(p, n)
        assert abs(c - 1.0 / (2.0 * (a + b * t) ** 2)) <= 1e-15 * c
        assert abs(i1 - np.log1p(b * dt / (a + b * t)) / b) <= 1e-13 * i1
        assert abs(i2 - dt / ((a + b * t) * (a + b * t1))) <= 1e-13 * i2


def test_constant_radius_linear_growth_is_exponential():
    """With r0 = R fixed, a small single mode grows by exactly
    exp(n dt (-|k|^2/R^2 + gamma |k| / (2R))) (the linear part is integrated
    exactly by the scheme; the quadratic term is negligible at amplitude 1e-30)."""
    R, n1, n2, dt, steps = 30.0, 32, 64, 0.5, 40
    p = oracle.Params(n1, n2, t0=1.0, dt=dt, gamma=0.8, r0_law=lambda t: R)
    full = np.zeros((n1, n2), dtype=np.complex128)
    full[3, 5] = 1e-30 * (0.6 + 0.8j)
    full[-3, -5] = np.conj(full[3, 5])
    out = oracle.run(full, p, steps)
    kap = np.hypot(3.0, 5.0)
    sigma = -kap ** 2 / R ** 2 + 0.8 * kap / (2.0 * R)
    want = full[3, 5] * np.exp(steps * dt * sigma)
    assert abs(out[3, 5] - want) <= 1e-12 * abs(want)


def test_constant_forcing_response_is_a_geometric_series():
    """With a constant radius, a constant forcing on one small mode and a zero
    initial state the scheme sums a geometric series (the mirror mode holds
    the conjugate)."""
    assert pins.pin_forcing_geometric_series() < 1e-12
    assert pins.pin_forcing_geometric_series(R=12.0, dt=0.2, steps=40, mode=(5, 1)) < 1e-12


def test_forcing_enters_the_exact_solution_of_eq1():
    """The forced step converges at first order to the ODE solution of Eq. (1)
    with the same forcing (DOP853 on the literal right-hand side)."""
    from scipy.integrate import solve_ivp

    n1 = n2 = 16
    rng = np.random.default_rng(3)
    half = (rng.standard_normal((2 * 3 + 1, 4)) + 1j * rng.standard_normal((2 * 3 + 1, 4))) * 1e-2
    full0 = oracle.symmetrise(oracle.half_to_full(half, n1, n2))  # real fields: Hermitian arrays
    force = oracle.symmetrise(oracle.half_to_full(
        (rng.standard_normal((7, 4)) + 1j * rng.standard_normal((7, 4))) * 1e-3, n1, n2))
    forcing = lambda t: force * np.cos(0.3 * t)  # noqa: E731
    t0, T = 5.0, 2.0
    mask = oracle.box_mask(n1, n2)

    def f(t, y):
        full = y.reshape(n1, n2)
        pp = oracle.Params(n1, n2, t0=t0, dt=1.0, forcing=forcing)
        return (oracle.rhs(full, pp, t) * mask).ravel()

    ref = solve_ivp(f, (t0, t0 + T), (full0 * mask).ravel().astype(np.complex128), method="DOP853",
                    rtol=1e-11, atol=1e-16).y[:, -1].reshape(n1, n2)
    errs = []
    for nsteps in (20, 40, 80):
        p = oracle.Params(n1, n2, t0=t0, dt=T / nsteps, forcing=forcing)
        errs.append(np.linalg.norm(oracle.run(full0, p, nsteps) - ref) / np.linalg.norm(ref))
    assert errs[-1] < 1e-3
    for a, b in zip(errs, errs[1:]):
        assert 1.6 < a / b < 2.4


def test_heun_is_exact_for_the_linear_part():
    assert pins.pin_linear_growth(dt=1.0, nsteps=50, integrator="rk2") < 1e-12
    assert pins.pin_linear_growth(dt=10.0, nsteps=5, integrator="rk2") < 1e-12


def test_heun_converges_at_second_order_to_eq1_solution():
    errs = pins.pin_convergence(integrator="rk2")
    euler = pins.pin_convergence()
    assert errs[-1] < 1e-4 and errs[-1] < 0.05 * euler[-1]
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5


def test_heun_constant_forcing_sums_its_series():
    assert pins.pin_forcing_geometric_series(integrator="rk2") < 1e-12
    assert pins.pin_forcing_geometric_series(R=12.0, dt=0.2, steps=40, mode=(5, 1), integrator="rk2") < 1e-12


def test_heun_with_time_dependent_forcing_converges_at_second_order():
    """Heun with f~(t) = cos(0.3 t) F against DOP853 on the forced Eq. (1):
    the forcing enters the corrector at t_{n+1}."""
    from scipy.integrate import solve_ivp

    n1 = n2 = 16
    rng = np.random.default_rng(3)
    half = (rng.standard_normal((7, 4)) + 1j * rng.standard_normal((7, 4))) * 1e-2
    full0 = oracle.symmetrise(oracle.half_to_full(half, n1, n2))
    force = oracle.symmetrise(oracle.half_to_full(
        (rng.standard_normal((7, 4)) + 1j * rng.standard_normal((7, 4))) * 1e-3, n1, n2))
    forcing = lambda t: force * np.cos(0.3 * t)  # noqa: E731
    t0, T = 5.0, 2.0
    mask = oracle.box_mask(n1, n2)

    def f(t, y):
        pp = oracle.Params(n1, n2, t0=t0, dt=1.0, forcing=forcing)
        return (oracle.rhs(y.reshape(n1, n2), pp, t) * mask).ravel()

    ref = solve_ivp(f, (t0, t0 + T), (full0 * mask).ravel().astype(np.complex128), method="DOP853",
                    rtol=1e-12, atol=1e-17).y[:, -1].reshape(n1, n2)
    errs = []
    for nsteps in (10, 20, 40):
        p = oracle.Params(n1, n2, t0=t0, dt=T / nsteps, forcing=forcing, integrator="rk2")
        errs.append(np.linalg.norm(oracle.run(full0, p, nsteps) - ref) / np.linalg.norm(ref))
    for a, b in zip(errs, errs[1:]):
        assert 3.4 < a / b < 4.6, errs


def test_threaded_transforms_match_the_default_to_round_off():
    """set_fft_workers (timing the oracle on all host cores) computes the same
    step as the default single-threaded transforms, up to rounding."""
    import os
    rng = np.random.default_rng(12)
    n1, n2 = 64, 96
    p = oracle.Params(n1, n2, t0=5.0, dt=0.2)
    full = oracle.symmetrise(pins.dict_to_full(pins.random_hermitian(n1, n2, rng, 0.3), n1, n2))
    ref = oracle.run(full, p, 3)
    try:
        oracle.set_fft_workers(os.cpu_count() or 2)
        got = oracle.run(full, p, 3)
    finally:
        oracle.set_fft_workers(None)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert pins.pin_convolution_direct(16, 24, seed=40) < 1e-12
