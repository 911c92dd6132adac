"""Eq. (1) and its time stepping in FP64 (oracle; test infrastructure only).

Eq. (1) (Section 2) for the Fourier components of the flame perturbation:

    dPhi~_k/dt = sigma_k(t) Phi~_k
                 - theta^2/(2 r0^2) * sum_l l.(k-l) Phi~_l Phi~_{k-l} + f~_k(t),
    sigma_k(t) = -theta^2 |k|^2 / r0^2 + gamma*theta*|k| / (2 r0),

with r0(t) = t (Section 2, choice of the reference radius; another law can
be given) and f~ = 0 as in the paper's runs (a forcing can be given). Writing kappa = (s1 k1, s2 k2) with the axis
scales s1 = s2 = theta_pi gives the literal equation; other scales are an
option of this implementation (anisotropic reading of the segment), in which
sigma_k = -|kappa|^2/r0^2 + gamma |kappa| / (2 r0) and the sum carries
kappa_l . kappa_{k-l}.

Readings of points the paper leaves open (each is also listed in the design
notes):

* Time integrator (the paper defers it to its references): integrating-factor
  (Lawson) Euler. The linear part is integrated exactly over the step,
  E_k = exp(int_{t_n}^{t_{n+1}} sigma_k dt); the quadratic term is taken
  explicitly at t_n:  Phi~^{n+1} = E_k (Phi~^n + dt * N_k(Phi~^n, t_n)).
  A second-order option is the integrating-factor form of Heun's method
  (Lawson's RK2): with v = Phi~ / E_k(t_n, t), the trapezoid rule on
  dv/dt = E^-1 N(E v, t) gives the Euler predictor Phi* above and
  Phi~^{n+1} = (Phi* + E_k Phi~^n + dt N_k(Phi*, t_{n+1})) / 2,
  both stages symmetrised.
* With r0 = t:  int r0^-2 dt = 1/t_n - 1/t_{n+1},  int r0^-1 dt = ln(t_{n+1}/t_n).
* Truncation is the box |k_i| <= K_i (Section 2 and Section 3).
* Symmetrisation copies the upper half H = {k2 > 0} or {k2 = 0, k1 > 0} onto
  -H and zeroes Im Phi~_0 (Section 3, symmetrisation paragraph and figure).
"""

from dataclasses import dataclass, field

import numpy as np

from .spectral import box_mask, wavenumbers


@dataclass
class Params:
    n1: int
    n2: int
    gamma: float = 0.8          # Section 2, figure captions: gamma = 0.8
    theta_pi: float = 1.0       # Section 2, segment definition (value unstated)
    t0: float = 200.0           # Section 2, initial time of the runs
    dt: float = 0.25
    axis_scale: tuple = field(default=None)
    # reference radius law t -> r0(t); None is the paper's r0(t) = t (Section 2)
    r0_law: object = field(default=None)
    # forcing f~_k(t) of Eq. (1): None (the paper's runs), a full Hermitian
    # coefficient array, or a function t -> such an array
    forcing: object = field(default=None)
    # time integrator: "euler" (integrating-factor Euler) or "rk2"
    # (integrating-factor Heun, second order)
    integrator: str = "euler"

    def forcing_at(self, t):
        if self.forcing is None:
            return None
        return self.forcing(t) if callable(self.forcing) else self.forcing

    def scales(self):
        if self.axis_scale is None:
            return (float(self.theta_pi), float(self.theta_pi))
        return (float(self.axis_scale[0]), float(self.axis_scale[1]))

    def kappa(self):
        """Scaled wavenumber components on the full FFT-ordered grid."""
        s1, s2 = self.scales()
        k1 = s1 * wavenumbers(self.n1).astype(np.float64)[:, None]
        k2 = s2 * wavenumbers(self.n2).astype(np.float64)[None, :]
        return np.broadcast_to(k1, (self.n1, self.n2)), np.broadcast_to(k2, (self.n1, self.n2))

    def time(self, n):
        return self.t0 + n * self.dt

    def r0(self, t):
        return r0(t) if self.r0_law is None else float(self.r0_law(t))


def r0(t):
    """Reference radius law of Section 2: r0(t) = t."""
    return t


def step_scalars(p, n):
    """Scalars of step n -> n+1: (c_n, I1, I2).

    c_n = 1/(2 r0(t_n)^2) is the coefficient of the quadratic term once the
    theta_pi factors are carried by kappa; I1 = int r0^-1 dt and
    I2 = int r0^-2 dt over [t_n, t_{n+1}]: in closed form for r0 = t, by
    adaptive Gauss-Kronrod quadrature in FP64 for any other law.
    """
    t = p.time(n)
    t1 = t + p.dt
    c = 1.0 / (2.0 * p.r0(t) ** 2)
    if p.r0_law is None:
        i1 = np.log1p(p.dt / t)
        i2 = p.dt / (t * t1)
    else:
        from scipy.integrate import quad

        i1 = quad(lambda s: 1.0 / p.r0(s), t, t1, epsabs=0.0, epsrel=1e-13)[0]
        i2 = quad(lambda s: 1.0 / p.r0(s) ** 2, t, t1, epsabs=0.0, epsrel=1e-13)[0]
    return c, i1, i2


def growth_exponent(p, n):
    """int_{t_n}^{t_{n+1}} sigma_k(t) dt on the full grid."""
    _, i1, i2 = step_scalars(p, n)
    k1, k2 = p.kappa()
    kap2 = k1 * k1 + k2 * k2
    return -kap2 * i2 + 0.5 * p.gamma * np.sqrt(kap2) * i1


# Threads of the one-dimensional transforms of convolution_sum: None uses
# numpy's (single-threaded) FFT; an integer uses scipy.fft with that many
# workers (the same transforms, for timing the oracle on all host cores).
_FFT_WORKERS = None


def set_fft_workers(workers):
    """None: numpy.fft (the default); k: scipy.fft with k worker threads."""
    global _FFT_WORKERS
    _FFT_WORKERS = None if workers is None else int(workers)


def _fft(x, axis, inverse):
    if _FFT_WORKERS is None:
        return np.fft.ifft(x, axis=axis) if inverse else np.fft.fft(x, axis=axis)
    import scipy.fft
    return (scipy.fft.ifft if inverse else scipy.fft.fft)(x, axis=axis, workers=_FFT_WORKERS)


def convolution_sum(full, p):
    """sum_l kappa_l . kappa_{k-l} Phi~_l Phi~_{k-l} for every k in the box.

    Evaluated the way Section 3 describes: on the augmented (padded) array,
    one-dimensional transforms along the first index of kappa1*Psi and
    kappa2*Psi, then along the second index; the element-by-element product
    (sum of squares) of the two transformed arrays; then the inverse
    transforms along the second and first index. On a grid with
    N_i >= 4 K_i + 1 this circular convolution equals the linear one on the box.
    """
    n1, n2 = p.n1, p.n2
    k1, k2 = p.kappa()
    h1 = _fft(k1 * full, 0, True) * n1
    h2 = _fft(k2 * full, 0, True) * n1
    h1 = _fft(h1, 1, True) * n2
    h2 = _fft(h2, 1, True) * n2
    prod = h1 * h1 + h2 * h2
    back = _fft(prod, 1, False) / n2
    back = _fft(back, 0, False) / n1
    return back * box_mask(n1, n2)


def rhs(full, p, t):
    """Right-hand side of Eq. (1) at time t (full array), with the forcing if given."""
    k1, k2 = p.kappa()
    kap = np.sqrt(k1 * k1 + k2 * k2)
    rr = p.r0(t)
    sigma = -kap * kap / rr ** 2 + p.gamma * kap / (2.0 * rr)
    out = sigma * full - convolution_sum(full, p) / (2.0 * rr ** 2)
    f = p.forcing_at(t)
    if f is not None:
        out = out + f
    return out * box_mask(p.n1, p.n2)


def symmetrise(full):
    """Copy the upper half H onto -H by Psi(-k) = conj(Psi(k)); Im Psi(0) = 0."""
    n1, n2 = full.shape
    out = np.array(full, dtype=np.complex128, copy=True)
    k1 = wavenumbers(n1)[:, None] + np.zeros((1, n2), dtype=np.int64)
    k2 = wavenumbers(n2)[None, :] + np.zeros((n1, 1), dtype=np.int64)
    upper = (k2 > 0) | ((k2 == 0) & (k1 > 0))
    src = np.nonzero(upper)
    dst = ((-k1[upper]) % n1, (-k2[upper]) % n2)
    out[dst] = np.conj(out[src])
    out[0, 0] = out[0, 0].real
    return out


def explicit_terms(full, p, n):
    """N_k(Phi~, t_n) + f~_k(t_n): the quadratic term of Eq. (1) with c_n =
    1/(2 r0(t_n)^2), plus the forcing if given (full array)."""
    c, _, _ = step_scalars(p, n)
    out = -c * convolution_sum(full, p)
    f = p.forcing_at(p.time(n))
    if f is not None:
        out = out + f
    return out


def step(full, p, n):
    """One step n -> n+1 of Eq. (1) (full array).

    Integrating-factor Euler: the forcing, like the quadratic term, is taken
    explicitly at t_n: Phi~^{n+1} = E_k (Phi~^n + dt (N_k(Phi~^n, t_n) + f~_k(t_n))).
    Integrating-factor Heun ("rk2"): that Euler step is the predictor Phi*
    (symmetrised), and Phi~^{n+1} = (Phi* + E_k Phi~^n + dt (N_k(Phi*, t_{n+1})
    + f~_k(t_{n+1}))) / 2.
    """
    e = np.exp(growth_exponent(p, n))
    mask = box_mask(p.n1, p.n2)
    pred = symmetrise(e * (full + p.dt * explicit_terms(full, p, n)) * mask)
    if p.integrator == "euler":
        return pred
    if p.integrator != "rk2":
        raise ValueError(f"unknown integrator {p.integrator!r}")
    new = 0.5 * (pred + e * full + p.dt * explicit_terms(pred, p, n + 1)) * mask
    return symmetrise(new)


def run(full, p, nsteps, n_start=0, callback=None):
    """Advance nsteps steps starting at step index n_start."""
    cur = symmetrise(np.asarray(full, dtype=np.complex128) * box_mask(p.n1, p.n2))
    for i in range(nsteps):
        cur = step(cur, p, n_start + i)
        if callback is not None:
            callback(n_start + i + 1, cur)
    return cur
