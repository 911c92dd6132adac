"""The circular-flame oracle (one-dimensional form of Eq. (1)) against what
the mathematics fixes, and against the two-dimensional oracle on the modes
k1 = 0 (CPU only)."""

import numpy as np
import pytest

import oracle
import pins


@pytest.mark.parametrize("n,s", [(21, 1.0), (32, 1.0), (40, 2.5), (13, 0.5)])
def test_circle_quadratic_term_equals_literal_sum(n, s):
    assert pins.pin_circle_literal_sum(n=n, seed=n, s=s) < 1e-13


def test_circle_single_cosine_closed_form():
    assert pins.pin_circle_single_cosine() < 1e-14
    assert pins.pin_circle_single_cosine(n=50, k=7, s=1.0) < 1e-14


def test_circle_linear_growth_closed_form():
    assert pins.pin_circle_linear_growth() < 1e-12
    assert pins.pin_circle_linear_growth(dt=5.0, nsteps=8, k=12, s=1.5) < 1e-12


def test_circle_is_the_k1_zero_restriction_of_eq1():
    assert pins.pin_circle_is_sphere_restriction() < 1e-13
    assert pins.pin_circle_is_sphere_restriction(n1=20, n=64, s=(1.0, 1.0), seed=60) < 1e-13


def test_circle_k0_mode_follows_parseval():
    assert pins.pin_circle_k0_parseval() < 1e-13


def test_circle_integrator_first_order():
    errs = pins.pin_circle_convergence()
    assert errs[-1] < 1e-2
    assert all(1.8 < a / b < 2.2 for a, b in zip(errs, errs[1:]))


def test_circle_diagnostics_single_cosine():
    assert pins.pin_circle_diagnostics() < 1e-12


def test_circle_half_layout_roundtrip():
    rng = np.random.default_rng(4)
    n = 64
    K = oracle.truncation(n)
    half = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
    half[0] = half[0].real
    full = oracle.half_to_circle(half, n)
    assert np.array_equal(oracle.circle_to_half(full), half)
    assert np.array_equal(oracle.circle_symmetrise(full), full)
    grid = np.fft.ifft(full) * n
    assert np.abs(grid.imag).max() < 1e-13


# Planted mistakes in the circular oracle, each of which some pin must catch.
ocirc = __import__("importlib").import_module("oracle.circle")


def _circle_pins_failing():
    bad = []
    checks = [
        ("literal", lambda: pins.pin_circle_literal_sum(n=21, seed=21, s=1.0) < 1e-13),
        ("literal_s", lambda: pins.pin_circle_literal_sum(n=40, seed=40, s=2.5) < 1e-13),
        ("cosine", lambda: pins.pin_circle_single_cosine() < 1e-14),
        ("growth", lambda: pins.pin_circle_linear_growth() < 1e-12),
        ("restriction", lambda: pins.pin_circle_is_sphere_restriction() < 1e-13),
        ("parseval", lambda: pins.pin_circle_k0_parseval() < 1e-13),
        ("diagnostics", lambda: pins.pin_circle_diagnostics() < 1e-12),
    ]
    for name, fn in checks:
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            bad.append(name)
    return bad


def _conv_sign(mp):
    orig = ocirc.circle_convolution_sum
    mp.setattr(ocirc, "circle_convolution_sum", lambda f, p: -orig(f, p))


def _c_without_half(mp):
    orig = ocirc.circle_scalars

    def sc(p, n):
        c, i1, i2 = orig(p, n)
        return 2 * c, i1, i2
    mp.setattr(ocirc, "circle_scalars", sc)


def _no_padding(mp):
    # the product on the 2K+1 points of the box: a circular convolution that aliases
    def conv(full, p):
        n = p.n
        K = (n - 1) // 4
        m = 2 * K + 1
        small = np.zeros(m, dtype=complex)
        kk = np.zeros(m)
        for k in range(-K, K + 1):
            small[k % m] = full[k % n]
            kk[k % m] = p.seg * k
        h = np.fft.ifft(kk * small) * m
        back = np.fft.fft(h * h) / m
        out = np.zeros(n, dtype=complex)
        for k in range(-K, K + 1):
            out[k % n] = back[k % m]
        return out
    mp.setattr(ocirc, "circle_convolution_sum", conv)


def _seg_once(mp):
    # the segment integer applied once to the quadratic term instead of per factor
    def conv(full, p):
        k = oracle.wavenumbers(p.n).astype(np.float64)
        h = np.fft.ifft(k * full) * p.n
        return p.seg * np.fft.fft(h * h) / p.n * p.mask()
    mp.setattr(ocirc, "circle_convolution_sum", conv)


def _growth_with_k_squared_only(mp):
    def step(full, p, n):
        c, i1, i2 = ocirc.circle_scalars(p, n)
        kap = p.kappa()
        e = np.exp(-kap * kap * i2)
        new = e * (full - p.dt * c * ocirc.circle_convolution_sum(full, p)) * p.mask()
        return ocirc.circle_symmetrise(new)
    mp.setattr(ocirc, "circle_step", step)


def _velocity_without_half(mp):
    orig = ocirc.circle_diagnostics

    def diag(full, p, n):
        r, v, a = orig(full, p, n)
        return r, 2 * v, a
    mp.setattr(ocirc, "circle_diagnostics", diag)
    mp.setattr(oracle, "circle_diagnostics", diag)


CIRCLE_MUTATIONS = [_conv_sign, _c_without_half, _no_padding, _seg_once, _growth_with_k_squared_only,
                    _velocity_without_half]


def test_unmutated_circle_oracle_passes_its_pins():
    assert _circle_pins_failing() == []


@pytest.mark.parametrize("mutation", CIRCLE_MUTATIONS, ids=[m.__name__.strip("_") for m in CIRCLE_MUTATIONS])
def test_circle_mutation_is_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    assert _circle_pins_failing(), f"no pin caught {mutation.__name__}"
