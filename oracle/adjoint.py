"""Discrete adjoint of the oracle's step and of the area functional (FP64).

Test infrastructure only (see the package docstring). The paper has no
adjoint; this is the transpose of the step in ``model.py`` derived by hand.

Inner product: the real grid product <a, b> = sum_j a(x_j) b(x_j). For
fields band-limited to the box with Fourier coefficients a~, b~ it equals
P * Re sum_k conj(a~_k) b~_k (Parseval, P = N1*N2). A cotangent is held as
the Fourier coefficients of a real band-limited grid field (a Hermitian full
array), so the gradient of a functional with respect to the grid values of
Phi is the synthesis of that array.

Forward step (Lawson Euler, ``model.step``):
    Phi^{n+1} = E^n (Phi^n + dt c_n Pi |grad Phi^n|^2)
Its tangent:
    dPhi^{n+1} = E^n (dPhi + 2 dt c_n Pi (grad Phi^n . grad dPhi))
E^n is a real multiplier even in k, hence self-adjoint; Pi (projection onto
the box) is self-adjoint; the adjoint of the spectral gradient restricted to
the box is -Pi div, with div taken by the grid transform. So
    lambda^n = mu - 2 dt c_n Pi div(m grad Phi^n),   mu = E^n lambda^{n+1},
with m the grid field of mu. Symmetrisation is the identity on real fields.

Area functional (``diagnostics``): J = (1/P) sum_j f(x_j), f = sqrt(1+x) - 1,
x = |grad Phi|^2 / r0^2, whose gradient is
    dJ/dPhi = -Pi div( grad Phi / (P r0^2 sqrt(1 + x)) ).
"""

import numpy as np

from .diagnostics import gradient_fields
from .model import growth_exponent, run, step, step_scalars
from .spectral import analyse, box_mask, synthesize


def _div(w1, w2, p):
    """Coefficients of Pi div(w) for grid fields w1, w2 (grid transform)."""
    k1, k2 = p.kappa()
    return (1j * k1 * analyse(w1) + 1j * k2 * analyse(w2)) * box_mask(p.n1, p.n2)


def area_excess(full, p, n):
    """J at step n, the cancellation-free grid mean of sqrt(1 + x) - 1."""
    rr = p.r0(p.time(n))
    g1, g2 = gradient_fields(full, p)
    x = (g1 * g1 + g2 * g2) / (rr * rr)
    return float((x / (1.0 + np.sqrt(1.0 + x))).mean())


def area_gradient(full, p, n):
    """Coefficients of dJ/dPhi (grid-value gradient) at step n."""
    rr = p.r0(p.time(n))
    g1, g2 = gradient_fields(full, p)
    x = (g1 * g1 + g2 * g2) / (rr * rr)
    scale = 1.0 / (p.n1 * p.n2 * rr * rr * np.sqrt(1.0 + x))
    return -_div(g1 * scale, g2 * scale, p)


def step_adjoint(state_n, lam_next, p, n):
    """lambda^n from lambda^{n+1} for the step n -> n+1 taken from state_n."""
    c, _, _ = step_scalars(p, n)
    mu = np.exp(growth_exponent(p, n)) * lam_next * box_mask(p.n1, p.n2)
    m = synthesize(mu).real
    g1, g2 = gradient_fields(state_n, p)
    return (mu - 2.0 * p.dt * c * _div(m * g1, m * g2, p)) * box_mask(p.n1, p.n2)


def trajectory_gradient(full0, p, nsteps, n_start=0, checkpoint_every=None):
    """(J(Phi^T), coefficients of dJ/dPhi^0) for nsteps steps from full0.

    Without checkpoint_every the whole trajectory is stored; with it only every
    checkpoint_every-th state is kept and each segment is recomputed from its
    checkpoint before its adjoint steps (the same states, so the same result).
    The grid-value gradient with respect to a physical initial field that is
    first projected onto the box is the synthesis of the returned coefficients.
    """
    every = nsteps if not checkpoint_every else int(checkpoint_every)
    checkpoints = []
    cur = run(full0, p, 0, n_start)
    n = 0
    while n < nsteps:
        checkpoints.append((n, cur))
        k = min(every, nsteps - n)
        for i in range(k):
            cur = step(cur, p, n_start + n + i)
        n += k
    n_end = n_start + nsteps
    value = area_excess(cur, p, n_end)
    lam = area_gradient(cur, p, n_end)
    for n0, saved in reversed(checkpoints):
        k = min(every, nsteps - n0)
        states = [saved]
        for i in range(1, k):
            states.append(step(states[-1], p, n_start + n0 + i - 1))
        for i in reversed(range(k)):
            lam = step_adjoint(states[i], lam, p, n_start + n0 + i)
    return value, lam
