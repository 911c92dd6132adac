"""Circular (two-dimensional) flames in FP64 (oracle; test infrastructure only).

Section 2 compares the spherical flames of Eq. (1) with two-dimensional
circular ones (the averaged-velocity figure, left panel; its text states
that their expansion rate settles to a (t - t*)^(1/4) law) but leaves the
circular model to its references. Reading taken here: the one-dimensional
form of Eq. (1) for the perturbation Phi(phi, t) of a circle of radius
r0(t) = t,

    dPhi~_k/dt = (-kappa_k^2 / r0^2 + gamma |kappa_k| / (2 r0)) Phi~_k
                 - 1/(2 r0^2) sum_l kappa_l kappa_{k-l} Phi~_l Phi~_{k-l},

with integer k, l and kappa_k = s k for the segment integer s (s = 1: the
whole circle). It is Eq. (1) restricted to the modes with k1 = 0, a set the
equation maps into itself (sums of k1 = 0 wavenumbers keep k1 = 0), which
the tests check against the two-dimensional oracle. Agreement with the
references' own circular model is not pinned.

The rest follows the two-dimensional oracle: Fourier-series normalisation,
truncation |k| <= K with K = floor((N - 1)/4) on the N-point augmented grid
of Section 3, integrating-factor Euler with the exact linear propagator,
Phi~(-k) = conj(Phi~(k)) and Im Phi~_0 = 0 after each step. Arrays are
"full": N complex coefficients in numpy FFT order.
"""

from dataclasses import dataclass

import numpy as np

from .spectral import truncation, wavenumbers


@dataclass
class CircleParams:
    n: int
    gamma: float = 0.8       # Section 2: gamma = 0.8 in the figures
    seg: float = 1.0         # segment integer (the whole circle)
    t0: float = 200.0        # Section 2: t0 = 200
    dt: float = 0.25

    def time(self, n):
        return self.t0 + n * self.dt

    def kappa(self):
        return self.seg * wavenumbers(self.n).astype(np.float64)

    def mask(self):
        return np.abs(wavenumbers(self.n)) <= truncation(self.n)


def circle_symmetrise(full):
    """Phi~(-k) := conj(Phi~(k)) for k > 0 and Im Phi~_0 := 0."""
    n = full.shape[0]
    out = np.array(full, dtype=np.complex128, copy=True)
    k = wavenumbers(n)
    pos = np.nonzero(k > 0)[0]
    out[(-k[pos]) % n] = np.conj(out[pos])
    out[0] = out[0].real
    return out


def circle_convolution_sum(full, p):
    """sum_l kappa_l kappa_{k-l} Phi~_l Phi~_{k-l} on the box, by the
    circular convolution on the N-point augmented grid (Section 3)."""
    h = np.fft.ifft(p.kappa() * full) * p.n
    return np.fft.fft(h * h) / p.n * p.mask()


def circle_scalars(p, n):
    """(c_n, I1, I2) of step n -> n+1 for r0 = t: c_n = 1/(2 t_n^2),
    I1 = ln(t_{n+1}/t_n), I2 = 1/t_n - 1/t_{n+1}."""
    t = p.time(n)
    return 1.0 / (2.0 * t * t), np.log1p(p.dt / t), p.dt / (t * (t + p.dt))


def circle_step(full, p, n):
    """One integrating-factor Euler step n -> n+1:
    Phi~ <- E_k (Phi~ - dt c_n sum_l kappa_l kappa_{k-l} Phi~_l Phi~_{k-l}),
    E_k = exp(-kappa_k^2 I2 + gamma |kappa_k| I1 / 2)."""
    c, i1, i2 = circle_scalars(p, n)
    kap = p.kappa()
    e = np.exp(-kap * kap * i2 + 0.5 * p.gamma * np.abs(kap) * i1)
    new = e * (full - p.dt * c * circle_convolution_sum(full, p)) * p.mask()
    return circle_symmetrise(new)


def circle_run(full, p, nsteps, n_start=0):
    cur = circle_symmetrise(np.asarray(full, dtype=np.complex128) * p.mask())
    for i in range(nsteps):
        cur = circle_step(cur, p, n_start + i)
    return cur


def circle_diagnostics(full, p, n):
    """(mean radius r0 + Re Phi~_0, averaged velocity <Phi_t> = dPhi~_0/dt,
    length excess <sqrt(1 + x) - 1> with x = Phi_phi^2 / r0^2 in kappa
    scaling) at step n, the one-dimensional counterparts of the sphere's
    averages."""
    t = p.time(n)
    g = (np.fft.ifft(1j * p.kappa() * full) * p.n).real
    q = g * g
    x = q / (t * t)
    return float(t + full[0].real), float(q.mean() / (2.0 * t * t)), float((x / (1.0 + np.sqrt(1.0 + x))).mean())


def half_to_circle(half, n):
    """Coefficients k = 0..K (complex, Im of k = 0 ignored) to a full array."""
    K = truncation(n)
    half = np.asarray(half)
    if half.shape != (K + 1,):
        raise ValueError(f"circle spectrum has shape {half.shape}, expected {(K + 1,)}")
    full = np.zeros(n, dtype=np.complex128)
    full[: K + 1] = half
    full[n - K:] = np.conj(half[1:][::-1])
    full[0] = full[0].real
    return full


def circle_to_half(full):
    n = full.shape[0]
    return np.asarray(full)[: truncation(n) + 1].copy()
