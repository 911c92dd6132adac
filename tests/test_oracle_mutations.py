"""Plant plausible mistakes in the oracle (on the CPU) and check a pin catches each.

Each mutation is applied with monkeypatch to the oracle's own module, the
pins are re-evaluated, and at least one must exceed its threshold.
"""

import importlib

import numpy as np
import pytest

import oracle
import pins

# the package re-exports functions named like some submodules, so fetch modules directly
oadj = importlib.import_module("oracle.adjoint")
odiag = importlib.import_module("oracle.diagnostics")
om = importlib.import_module("oracle.model")

THRESHOLDS = {
    "pin_convolution_direct": 1e-12,
    "pin_convolution_direct_anisotropic": 1e-12,
    "pin_single_cosine": 1e-12,
    "pin_linear_growth": 1e-10,
    "pin_first_step_worked_example": 1e-12,
    "pin_k0_parseval": 1e-12,
    "pin_diagnostics_single_cosine": 1e-12,
    "pin_adjoint_dot_product": 1e-10,
    "pin_trajectory_gradient_fd": 1e-5,
    "pin_forcing_geometric_series": 1e-12,
    "pin_area_excess_series": 1e-12,
}

# pins that take arguments: (label, callable, threshold)
CALL_PINS = [
    ("pin_trajectory_gradient_fd_checkpointed",
     lambda: pins.pin_trajectory_gradient_fd(n_start=5, checkpoint_every=3), 1e-6),
    ("pin_checkpointed_gradient_identical", pins.pin_checkpointed_gradient_identical, 0),
]


def failing_pins():
    bad = []
    for name, tol in THRESHOLDS.items():
        try:
            v = getattr(pins, name)()
        except Exception:  # a crash also counts as caught
            bad.append(name)
            continue
        if not np.isfinite(v) or v > tol:
            bad.append(name)
    for name, fn, tol in CALL_PINS:
        try:
            v = fn()
        except Exception:
            bad.append(name)
            continue
        if not np.isfinite(v) or v > tol:
            bad.append(name)
    conv = pins.pin_convergence()
    if not (conv[-1] < 5e-3 and all(1.8 < a / b < 2.2 for a, b in zip(conv, conv[1:]))):
        bad.append("pin_convergence")
    conv2 = pins.pin_convergence(integrator="rk2")
    if not (conv2[-1] < 1e-4 and all(3.5 < a / b < 4.5 for a, b in zip(conv2, conv2[1:]))):
        bad.append("pin_convergence_rk2")
    try:
        if not pins.pin_forcing_geometric_series(integrator="rk2") < 1e-12:
            bad.append("pin_forcing_geometric_series_rk2")
    except Exception:
        bad.append("pin_forcing_geometric_series_rk2")
    return bad


def test_unmutated_oracle_passes_all_pins():
    assert failing_pins() == []


def _flip_nonlinear_sign(monkeypatch):
    orig = om.convolution_sum
    monkeypatch.setattr(om, "convolution_sum", lambda f, p: -orig(f, p))


def _drop_instability_term(monkeypatch):
    def growth(p, n):
        _, i1, i2 = om.step_scalars(p, n)
        k1, k2 = p.kappa()
        return -(k1 * k1 + k2 * k2) * i2
    monkeypatch.setattr(om, "growth_exponent", growth)


def _euler_radius_integral(monkeypatch):
    def scalars(p, n):
        t = p.time(n)
        return 1.0 / (2 * t * t), p.dt / t, p.dt / (t * t)
    monkeypatch.setattr(om, "step_scalars", scalars)


def _missing_half_in_c(monkeypatch):
    orig = om.step_scalars

    def scalars(p, n):
        c, i1, i2 = orig(p, n)
        return 2 * c, i1, i2
    monkeypatch.setattr(om, "step_scalars", scalars)


def _transposed_kappa(monkeypatch):
    orig = om.Params.kappa

    def kappa(self):
        k1, k2 = orig(self)
        s1, s2 = self.scales()
        return k1 / s1 * s2, k2 / s2 * s1
    monkeypatch.setattr(om.Params, "kappa", kappa)


def _cross_term_dropped(monkeypatch):
    def conv(full, p):
        n1, n2 = p.n1, p.n2
        k1, k2 = p.kappa()
        h1 = np.fft.ifft2(k1 * full) * full.size
        return np.fft.fft2(h1 * h1) / full.size * oracle.box_mask(n1, n2)
    monkeypatch.setattr(om, "convolution_sum", conv)


def _aliased_grid(monkeypatch):
    # evaluate the product without padding: a circular convolution on the box only
    def conv(full, p):
        n1, n2 = p.n1, p.n2
        K1, K2 = (n1 - 1) // 4, (n2 - 1) // 4
        m1, m2 = 2 * K1 + 1, 2 * K2 + 1
        k1, k2 = p.kappa()
        small = np.zeros((m1, m2), dtype=complex)
        kk1 = np.zeros((m1, m2))
        kk2 = np.zeros((m1, m2))
        for a in range(-K1, K1 + 1):
            for b in range(-K2, K2 + 1):
                small[a % m1, b % m2] = full[a % n1, b % n2]
                kk1[a % m1, b % m2] = k1[a % n1, 0]
                kk2[a % m1, b % m2] = k2[0, b % n2]
        h1 = np.fft.ifft2(kk1 * small) * small.size
        h2 = np.fft.ifft2(kk2 * small) * small.size
        back = np.fft.fft2(h1 * h1 + h2 * h2) / small.size
        out = np.zeros_like(full)
        for a in range(-K1, K1 + 1):
            for b in range(-K2, K2 + 1):
                out[a % n1, b % n2] = back[a % m1, b % m2]
        return out
    monkeypatch.setattr(om, "convolution_sum", conv)


def _nonlinear_at_new_time(monkeypatch):
    orig = om.step_scalars

    def scalars(p, n):
        _, i1, i2 = orig(p, n)
        t1 = p.time(n) + p.dt
        return 1.0 / (2 * t1 * t1), i1, i2
    monkeypatch.setattr(om, "step_scalars", scalars)


def _velocity_without_half(monkeypatch):
    orig = odiag.diagnostics

    def diag(full, p, n):
        r, v, a = orig(full, p, n)
        return r, 2 * v, a
    monkeypatch.setattr(oracle, "diagnostics", diag)


def _area_without_sqrt(monkeypatch):
    orig = odiag.diagnostics

    def diag(full, p, n):
        r, v, _ = orig(full, p, n)
        t = p.time(n)
        g1, g2 = odiag.gradient_fields(full, p)
        return r, v, float(((g1 * g1 + g2 * g2) / (t * t)).mean() / 2)
    monkeypatch.setattr(oracle, "diagnostics", diag)


def _adjoint_missing_factor_two(monkeypatch):
    def adj(state_n, lam_next, p, n):
        c, _, _ = om.step_scalars(p, n)
        mu = np.exp(om.growth_exponent(p, n)) * lam_next * oracle.box_mask(p.n1, p.n2)
        m = oracle.synthesize(mu).real
        g1, g2 = odiag.gradient_fields(state_n, p)
        return (mu - p.dt * c * oadj._div(m * g1, m * g2, p)) * oracle.box_mask(p.n1, p.n2)
    monkeypatch.setattr(oracle, "step_adjoint", adj)
    monkeypatch.setattr(oadj, "step_adjoint", adj)


def _adjoint_without_decay(monkeypatch):
    def adj(state_n, lam_next, p, n):
        c, _, _ = om.step_scalars(p, n)
        mu = lam_next * oracle.box_mask(p.n1, p.n2)
        m = oracle.synthesize(mu).real
        g1, g2 = odiag.gradient_fields(state_n, p)
        return (mu - 2 * p.dt * c * oadj._div(m * g1, m * g2, p)) * oracle.box_mask(p.n1, p.n2)
    monkeypatch.setattr(oracle, "step_adjoint", adj)
    monkeypatch.setattr(oadj, "step_adjoint", adj)


def _forcing_outside_integrating_factor(monkeypatch):
    # the forcing added after the decay/growth factor instead of inside it
    def step(full, p, n):
        c, _, _ = om.step_scalars(p, n)
        e = np.exp(om.growth_exponent(p, n))
        new = e * (full - p.dt * c * om.convolution_sum(full, p))
        f = p.forcing_at(p.time(n))
        if f is not None:
            new = new + p.dt * f
        return om.symmetrise(new * oracle.box_mask(p.n1, p.n2))
    monkeypatch.setattr(om, "step", step)


def _heun_corrector_at_old_time(monkeypatch):
    # the corrector's quadratic term and forcing taken at t_n instead of t_{n+1}
    def step(full, p, n):
        e = np.exp(om.growth_exponent(p, n))
        mask = oracle.box_mask(p.n1, p.n2)
        pred = om.symmetrise(e * (full + p.dt * om.explicit_terms(full, p, n)) * mask)
        if p.integrator == "euler":
            return pred
        return om.symmetrise(0.5 * (pred + e * full + p.dt * om.explicit_terms(pred, p, n)) * mask)
    monkeypatch.setattr(om, "step", step)


def _heun_propagator_on_corrector(monkeypatch):
    # E applied to the corrector's explicit terms as well
    def step(full, p, n):
        e = np.exp(om.growth_exponent(p, n))
        mask = oracle.box_mask(p.n1, p.n2)
        pred = om.symmetrise(e * (full + p.dt * om.explicit_terms(full, p, n)) * mask)
        if p.integrator == "euler":
            return pred
        return om.symmetrise(0.5 * (pred + e * (full + p.dt * om.explicit_terms(pred, p, n + 1))) * mask)
    monkeypatch.setattr(om, "step", step)


def _checkpoint_recompute_off_by_one(monkeypatch):
    # each recomputed segment state advanced with the step index one too far
    def traj(full0, p, nsteps, n_start=0, checkpoint_every=None):
        every = nsteps if not checkpoint_every else int(checkpoint_every)
        checkpoints, cur, n = [], om.run(full0, p, 0, n_start), 0
        while n < nsteps:
            checkpoints.append((n, cur))
            k = min(every, nsteps - n)
            for i in range(k):
                cur = om.step(cur, p, n_start + n + i)
            n += k
        value = oadj.area_excess(cur, p, n_start + nsteps)
        lam = oadj.area_gradient(cur, p, n_start + nsteps)
        for n0, saved in reversed(checkpoints):
            k = min(every, nsteps - n0)
            states = [saved]
            for i in range(1, k):
                states.append(om.step(states[-1], p, n_start + n0 + i))
            for i in reversed(range(k)):
                lam = oadj.step_adjoint(states[i], lam, p, n_start + n0 + i)
        return value, lam
    monkeypatch.setattr(oracle, "trajectory_gradient", traj)
    monkeypatch.setattr(oadj, "trajectory_gradient", traj)


def _adjoint_steps_from_zero_index(monkeypatch):
    # the adjoint steps of a trajectory that starts at n_start taken at 0 .. nsteps-1
    orig = oadj.trajectory_gradient

    def traj(full0, p, nsteps, n_start=0, checkpoint_every=None):
        saved = oadj.step_adjoint

        def adj(state_n, lam_next, pp, n):
            return saved(state_n, lam_next, pp, n - n_start)
        monkeypatch.setattr(oadj, "step_adjoint", adj)
        try:
            return orig(full0, p, nsteps, n_start, checkpoint_every)
        finally:
            monkeypatch.setattr(oadj, "step_adjoint", saved)
    monkeypatch.setattr(oracle, "trajectory_gradient", traj)


def _area_excess_plain_mean_of_x(monkeypatch):
    # J taken as half the mean of x (the small-slope limit) in the adjoint module
    def area(full, p, n):
        rr = p.r0(p.time(n))
        g1, g2 = odiag.gradient_fields(full, p)
        return float(((g1 * g1 + g2 * g2) / (rr * rr)).mean() / 2)
    monkeypatch.setattr(oracle, "area_excess", area)
    monkeypatch.setattr(oadj, "area_excess", area)


MUTATIONS = [
    _flip_nonlinear_sign, _drop_instability_term, _euler_radius_integral, _missing_half_in_c,
    _transposed_kappa, _cross_term_dropped, _aliased_grid, _nonlinear_at_new_time,
    _velocity_without_half, _area_without_sqrt, _adjoint_missing_factor_two,
    _adjoint_without_decay, _forcing_outside_integrating_factor, _heun_corrector_at_old_time,
    _heun_propagator_on_corrector, _checkpoint_recompute_off_by_one, _adjoint_steps_from_zero_index,
    _area_excess_plain_mean_of_x,
]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m.__name__.strip("_") for m in MUTATIONS])
def test_mutation_is_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    assert failing_pins(), f"no pin caught {mutation.__name__}"
