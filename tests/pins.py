"""Independent checks that pin the FP64 oracle to the paper and to mathematics.

Each function returns a discrepancy (max relative or absolute error) so the
tests can assert thresholds and the mutation tests can show that a planted
mistake in the oracle makes at least one of them fail. Nothing here reuses
the oracle's arithmetic: transforms are explicit DFT matrices, the quadratic
term is the literal double sum of Eq. (1), growth factors are integrated by
hand or by scipy's ODE solver.
"""

import numpy as np
from scipy.integrate import solve_ivp

import oracle

GAMMA = 0.8


# ----------------------------------------------------------------- helpers

def box_modes(n1, n2):
    K1, K2 = (n1 - 1) // 4, (n2 - 1) // 4
    return [(a, b) for a in range(-K1, K1 + 1) for b in range(-K2, K2 + 1)]


def random_hermitian(n1, n2, rng, scale=1.0):
    """Random Hermitian coefficients on the box as a dict {k: value}."""
    K1, K2 = (n1 - 1) // 4, (n2 - 1) // 4
    coef = {}
    for a in range(-K1, K1 + 1):
        for b in range(-K2, K2 + 1):
            if (b > 0) or (b == 0 and a > 0):
                v = scale * (rng.standard_normal() + 1j * rng.standard_normal())
                coef[(a, b)] = v
                coef[(-a, -b)] = np.conj(v)
    coef[(0, 0)] = scale * rng.standard_normal() + 0j
    return coef


def dict_to_full(coef, n1, n2):
    full = np.zeros((n1, n2), dtype=np.complex128)
    for (a, b), v in coef.items():
        full[a % n1, b % n2] = v
    return full


def dft_synthesis(coef, n1, n2):
    """Phi(x_j) = sum_k c_k exp(i k.x_j) by an explicit double loop over modes."""
    j1 = np.arange(n1)[:, None]
    j2 = np.arange(n2)[None, :]
    out = np.zeros((n1, n2), dtype=np.complex128)
    for (a, b), v in coef.items():
        out += v * np.exp(2j * np.pi * (a * j1 / n1 + b * j2 / n2))
    return out


def direct_convolution(coef, n1, n2, s=(1.0, 1.0)):
    """Literal Eq. (1) sum: sum_l kappa_l . kappa_{k-l} c_l c_{k-l} for k in the box."""
    K1, K2 = (n1 - 1) // 4, (n2 - 1) // 4
    out = {}
    for k in box_modes(n1, n2):
        acc = 0j
        for l, cl in coef.items():
            m = (k[0] - l[0], k[1] - l[1])
            if abs(m[0]) > K1 or abs(m[1]) > K2 or m not in coef:
                continue
            dot = s[0] * l[0] * s[0] * m[0] + s[1] * l[1] * s[1] * m[1]
            acc += dot * cl * coef[m]
        out[k] = acc
    return out


def eq1_rhs_direct(coef_vec, keys, t, s=(1.0, 1.0), gamma=GAMMA):
    """Eq. (1) right-hand side with the literal sum, r0 = t, f = 0."""
    coef = dict(zip(keys, coef_vec))
    n1 = 4 * max(abs(k[0]) for k in keys) + 1
    n2 = 4 * max(abs(k[1]) for k in keys) + 1
    conv = direct_convolution(coef, n1, n2, s)
    out = np.empty(len(keys), dtype=np.complex128)
    for i, k in enumerate(keys):
        kap = np.hypot(s[0] * k[0], s[1] * k[1])
        sigma = -kap * kap / t ** 2 + gamma * kap / (2 * t)
        out[i] = sigma * coef[k] - conv[k] / (2 * t ** 2)
    return out


# -------------------------------------------------------------------- pins

def pin_transform_bruteforce(n1=12, n2=20, seed=0):
    rng = np.random.default_rng(seed)
    coef = random_hermitian(n1, n2, rng)
    full = dict_to_full(coef, n1, n2)
    ref = dft_synthesis(coef, n1, n2)
    e1 = np.abs(oracle.synthesize(full) - ref).max() / np.abs(ref).max()
    back = oracle.analyse(ref)
    e2 = np.abs(back - full).max() / np.abs(full).max()
    return max(e1, e2)


def pin_convolution_direct(n1=13, n2=17, seed=1, s=(1.0, 1.0), hermitian=True):
    rng = np.random.default_rng(seed)
    if hermitian:
        coef = random_hermitian(n1, n2, rng)
    else:
        coef = {k: rng.standard_normal() + 1j * rng.standard_normal() for k in box_modes(n1, n2)}
    full = dict_to_full(coef, n1, n2)
    p = oracle.Params(n1, n2, axis_scale=s)
    got = oracle.convolution_sum(full, p)
    ref = direct_convolution(coef, n1, n2, s)
    scale = max(abs(v) for v in ref.values())
    err = max(abs(got[k[0] % n1, k[1] % n2] - v) for k, v in ref.items())
    outside = np.abs(got * ~oracle.box_mask(n1, n2)).max()
    return max(err, outside) / scale


def pin_single_cosine(n1=32, n2=48, k=(3, 4), a=0.7, psi=0.3, s=(1.0, 1.0)):
    coef = {k: 0.5 * a * np.exp(1j * psi), (-k[0], -k[1]): 0.5 * a * np.exp(-1j * psi)}
    full = dict_to_full(coef, n1, n2)
    p = oracle.Params(n1, n2, axis_scale=s)
    got = oracle.convolution_sum(full, p)
    kap2 = (s[0] * k[0]) ** 2 + (s[1] * k[1]) ** 2
    ref = np.zeros_like(got)
    ref[0, 0] = -a * a * kap2 / 2
    ref[(2 * k[0]) % n1, (2 * k[1]) % n2] = a * a * kap2 / 4 * np.exp(2j * psi)
    ref[(-2 * k[0]) % n1, (-2 * k[1]) % n2] = a * a * kap2 / 4 * np.exp(-2j * psi)
    return np.abs(got - ref).max() / (a * a * kap2)


def pin_two_cosines(n1=48, n2=48, k=(2, 5), l=(3, -1), a=0.4, b=0.9, p1=0.2, p2=1.1):
    coef = {}
    for kk, amp, ph in ((k, a, p1), (l, b, p2)):
        coef[kk] = 0.5 * amp * np.exp(1j * ph)
        coef[(-kk[0], -kk[1])] = 0.5 * amp * np.exp(-1j * ph)
    full = dict_to_full(coef, n1, n2)
    p = oracle.Params(n1, n2)
    got = oracle.convolution_sum(full, p)
    dot = k[0] * l[0] + k[1] * l[1]
    kk2, ll2 = k[0] ** 2 + k[1] ** 2, l[0] ** 2 + l[1] ** 2
    ref = {}

    def put(m, v):
        ref[m] = ref.get(m, 0) + v

    put((0, 0), -(a * a * kk2 + b * b * ll2) / 2)
    for sgn in (1, -1):
        put((sgn * 2 * k[0], sgn * 2 * k[1]), a * a * kk2 / 4 * np.exp(sgn * 2j * p1))
        put((sgn * 2 * l[0], sgn * 2 * l[1]), b * b * ll2 / 4 * np.exp(sgn * 2j * p2))
        put((sgn * (k[0] + l[0]), sgn * (k[1] + l[1])), a * b * dot / 2 * np.exp(sgn * 1j * (p1 + p2)))
        put((sgn * (k[0] - l[0]), sgn * (k[1] - l[1])), -a * b * dot / 2 * np.exp(sgn * 1j * (p1 - p2)))
    refarr = np.zeros_like(got)
    for m, v in ref.items():
        refarr[m[0] % n1, m[1] % n2] += v
    return np.abs(got - refarr).max() / (a * b * abs(dot))


def hand_growth(kap, t, t0, gamma=GAMMA):
    """exp of int_{t0}^{t} (-kap^2/s^2 + gamma kap/(2 s)) ds, integrated by hand."""
    return np.exp(kap * kap * (1.0 / t - 1.0 / t0) + 0.5 * gamma * kap * np.log(t / t0))


def pin_linear_growth(dt=1.0, nsteps=50, t0=200.0, amp=1e-30, integrator="euler"):
    """Small modes grow by the hand-integrated exp(int sigma_k dt): both
    integrating-factor schemes are exact for the linear part of Eq. (1)."""
    modes = [(1, 0), (3, 4), (6, 8), (0, 13), (24, 32), (48, 64), (72, 96)]
    n1, n2 = 300, 400
    coef = {}
    for m in modes:
        coef[m] = amp
        coef[(-m[0], -m[1])] = amp
    p = oracle.Params(n1, n2, t0=t0, dt=dt, integrator=integrator)
    out = oracle.run(dict_to_full(coef, n1, n2), p, nsteps)
    t = t0 + nsteps * dt
    err = 0.0
    for m in modes:
        g = hand_growth(np.hypot(*m), t, t0)
        err = max(err, abs(out[m[0] % n1, m[1] % n2] / amp - g) / g)
    return err


def pin_linear_growth_ode(kap=37.0, t0=200.0, t1=260.0):
    """scipy DOP853 on dy/dt = sigma(t) y against the oracle's step factors."""
    sol = solve_ivp(lambda t, y: (-kap * kap / t ** 2 + GAMMA * kap / (2 * t)) * y,
                    (t0, t1), [1.0], method="DOP853", rtol=1e-12, atol=1e-14)
    ref = sol.y[0, -1]
    n1 = n2 = 4 * 40 + 4
    p = oracle.Params(n1, n2, t0=t0, dt=(t1 - t0) / 12)
    acc = 1.0
    k1 = oracle.wavenumbers(n1)
    i = int(np.nonzero(k1 == 37)[0][0])
    for n in range(12):
        acc *= np.exp(oracle.growth_exponent(p, n))[i, 0]
    return abs(acc - ref) / abs(ref)


def pin_first_step_worked_example():
    """One step from a single mode k = (3, 4), a = 1e-3, psi = 0, dt = 0.25, t0 = 200."""
    n1 = n2 = 64
    a = 1e-3
    coef = {(3, 4): a / 2, (-3, -4): a / 2}
    p = oracle.Params(n1, n2, t0=200.0, dt=0.25)
    out = oracle.step(dict_to_full(coef, n1, n2), p, 0)
    # mode 0: E_0 = 1, N_0 = c * a^2 |k|^2 / 2 with c = 1/(2*200^2)
    e0 = abs(out[0, 0] - 3.90625e-11) / 3.90625e-11
    e10 = hand_growth(10.0, 200.25, 200.0)
    ref = e10 * (-1.953125e-11)
    e1 = abs(out[6, 8] - ref) / abs(ref)
    return max(e0, e1)


def pin_k0_parseval(n1=24, n2=40, seed=3):
    rng = np.random.default_rng(seed)
    coef = random_hermitian(n1, n2, rng, scale=0.3)
    full = oracle.symmetrise(dict_to_full(coef, n1, n2))
    p = oracle.Params(n1, n2, t0=50.0, dt=0.5)
    out = oracle.step(full, p, 3)
    t = 50.0 + 3 * 0.5
    kap2 = 0.0
    for (a, b), v in coef.items():
        kap2 += (a * a + b * b) * abs(v) ** 2
    ref = 0.5 * kap2 / (2 * t * t)
    return abs((out[0, 0] - full[0, 0]) - ref) / abs(ref)


def reference_trajectory(n=13, t0=5.0, t1=7.0, seed=4, amp=0.5):
    rng = np.random.default_rng(seed)
    coef = random_hermitian(n, n, rng, scale=amp)
    keys = list(coef.keys())
    y0 = np.array([coef[k] for k in keys])

    def f(t, y):
        c = y[: len(keys)] + 1j * y[len(keys):]
        r = eq1_rhs_direct(c, keys, t)
        return np.concatenate([r.real, r.imag])

    sol = solve_ivp(f, (t0, t1), np.concatenate([y0.real, y0.imag]), method="DOP853",
                    rtol=1e-11, atol=1e-13)
    yT = sol.y[: len(keys), -1] + 1j * sol.y[len(keys):, -1]
    return coef, keys, yT


def pin_convergence(n=13, t0=5.0, t1=7.0, steps=(20, 40, 80), integrator="euler"):
    """Relative errors against DOP853 on the literal Eq. (1) sum at each step
    count: they fall by 2 per halving of dt for Euler, by 4 for Heun."""
    coef, keys, yT = reference_trajectory(n, t0, t1)
    full = dict_to_full(coef, n, n)
    errs = []
    for ns in steps:
        p = oracle.Params(n, n, t0=t0, dt=(t1 - t0) / ns, integrator=integrator)
        out = oracle.run(full, p, ns)
        got = np.array([out[k[0] % n, k[1] % n] for k in keys])
        errs.append(np.linalg.norm(got - yT) / np.linalg.norm(yT))
    return errs


def area_series(b, terms=60):
    """(1/2pi) int_0^{2pi} sqrt(1 + b sin^2 u) du - 1 as a power series in b (b < 1)."""
    total = 0.0
    binom = 1.0
    central = 1.0
    for j in range(1, terms):
        binom *= (0.5 - (j - 1)) / j        # C(1/2, j)
        central *= (2 * j) * (2 * j - 1) / (j * j) / 4.0   # C(2j, j) / 4^j
        total += binom * central * b ** j
    return total


def pin_diagnostics_single_cosine(n1=32, n2=64, k=(2, 3), a=0.5, psi=0.4, mean=0.05, n=0):
    p = oracle.Params(n1, n2, t0=3.0, dt=0.1)
    coef = {k: 0.5 * a * np.exp(1j * psi), (-k[0], -k[1]): 0.5 * a * np.exp(-1j * psi),
            (0, 0): mean + 0j}
    full = dict_to_full(coef, n1, n2)
    rbar, vel, area = oracle.diagnostics(full, p, n)
    r = 3.0 + n * 0.1
    kap2 = k[0] ** 2 + k[1] ** 2
    e_r = abs(rbar - (r + mean)) / (r + mean)
    e_v = abs(vel - a * a * kap2 / 2 / (2 * r * r)) / (a * a * kap2 / 2 / (2 * r * r))
    b = a * a * kap2 / (r * r)
    ref_area = area_series(b)
    e_a = abs(area - ref_area) / ref_area
    return max(e_r, e_v, e_a)


def real_inner(a, b):
    """Grid inner product of two band-limited real fields from their coefficients."""
    return float(a.size * np.real(np.vdot(a, b)))


def pin_adjoint_dot_product(n1=16, n2=24, seed=5, t0=5.0, dt=0.3):
    """<lambda, J d> = <J^T lambda, d> for one step; J d by central differences,
    which are exact up to rounding because the step is quadratic in Phi."""
    rng = np.random.default_rng(seed)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    phi = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, 0.4), n1, n2))
    d = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, 1.0), n1, n2))
    lam = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, 1.0), n1, n2))
    eps = 1e-3
    jd = (oracle.step(phi + eps * d, p, 2) - oracle.step(phi - eps * d, p, 2)) / (2 * eps)
    lhs = real_inner(lam, jd)
    rhs = real_inner(oracle.step_adjoint(phi, lam, p, 2), d)
    return abs(lhs - rhs) / abs(lhs)


def pin_area_gradient_fd(n1=16, n2=24, seed=6, t0=2.0, amp=0.6):
    """dJ/dPhi against central differences of J at one state."""
    rng = np.random.default_rng(seed)
    p = oracle.Params(n1, n2, t0=t0, dt=0.1)
    phi = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, amp), n1, n2))
    g = oracle.area_gradient(phi, p, 0)
    worst = 0.0
    for _ in range(4):
        v = oracle.project(rng.standard_normal((n1, n2)))
        eps = 1e-5
        fd = (oracle.area_excess(phi + eps * v, p, 0) - oracle.area_excess(phi - eps * v, p, 0)) / (2 * eps)
        worst = max(worst, abs(fd - real_inner(g, v)) / abs(fd))
    return worst


def pin_trajectory_gradient_fd(n1=16, n2=24, seed=7, t0=3.0, dt=0.2, nsteps=10, amp=0.5, n_start=0,
                               checkpoint_every=None):
    """Gradient of J(Phi^T) with respect to a projected physical initial field
    against central differences along random grid directions.

    The trajectory starts at step index n_start (time t0 + n_start dt) and
    ends at n_start + nsteps; with checkpoint_every the gradient goes through
    the branch that keeps only every checkpoint_every-th state and recomputes
    each segment. The differences of J are formed from the forward run alone
    (``run`` and the grid mean of sqrt(1 + x) - 1), so a wrong step index in
    the recomputation or in the adjoint steps shows up as a mismatch."""
    rng = np.random.default_rng(seed)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    phi0 = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, amp), n1, n2))
    _, lam = oracle.trajectory_gradient(phi0, p, nsteps, n_start=n_start, checkpoint_every=checkpoint_every)
    grad_grid = oracle.synthesize(lam).real
    worst = 0.0
    for _ in range(4):
        v = rng.standard_normal((n1, n2))
        vp = oracle.project(v)
        eps = 1e-5

        def J(x):
            return area_mean(oracle.run(x, p, nsteps, n_start), p, n_start + nsteps)

        fd = (J(phi0 + eps * vp) - J(phi0 - eps * vp)) / (2 * eps)
        worst = max(worst, abs(fd - float((grad_grid * v).sum())) / abs(fd))
    return worst


def area_mean(full, p, n):
    """Grid mean of sqrt(1 + x) - 1, x = |grad Phi|^2 / r0(t_n)^2, written out
    here from the gradient's definition (spectral derivative, then synthesis)
    and evaluated the plain way; used as the functional of the finite
    differences, so that they do not rely on the oracle's own J."""
    k1, k2 = p.kappa()
    g1 = np.fft.ifft2(1j * k1 * full).real * full.size
    g2 = np.fft.ifft2(1j * k2 * full).real * full.size
    rr = p.r0(p.time(n))
    x = (g1 * g1 + g2 * g2) / (rr * rr)
    return float((np.sqrt(1.0 + x) - 1.0).mean())


def pin_checkpointed_gradient_identical(n1=16, n2=24, seed=9, t0=3.0, dt=0.2, nsteps=7, n_start=4, amp=0.5):
    """The checkpointed gradient recomputes the same states in the same order
    as the full-storage one, so every checkpoint spacing must give the same
    value and coefficients bit for bit (returns the number of spacings that
    differ, 0 when all agree)."""
    rng = np.random.default_rng(seed)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    phi0 = oracle.symmetrise(dict_to_full(random_hermitian(n1, n2, rng, amp), n1, n2))
    ref_v, ref_l = oracle.trajectory_gradient(phi0, p, nsteps, n_start=n_start)
    bad = 0
    for every in (1, 2, 3, nsteps - 1, nsteps, nsteps + 5):
        v, lam = oracle.trajectory_gradient(phi0, p, nsteps, n_start=n_start, checkpoint_every=every)
        if not (v == ref_v and np.array_equal(lam, ref_l)):
            bad += 1
    return bad


def pin_area_excess_series(n1=32, n2=64, k=(2, 3), a=0.5, psi=0.4, n=3):
    """oracle.area_excess (the J of the adjoint module) against the exact
    series for a single cosine, and against diagnostics()[2]."""
    p = oracle.Params(n1, n2, t0=3.0, dt=0.1)
    coef = {k: 0.5 * a * np.exp(1j * psi), (-k[0], -k[1]): 0.5 * a * np.exp(-1j * psi)}
    full = dict_to_full(coef, n1, n2)
    r = 3.0 + n * 0.1
    b = a * a * (k[0] ** 2 + k[1] ** 2) / (r * r)
    j = oracle.area_excess(full, p, n)
    e_series = abs(j - area_series(b)) / area_series(b)
    e_diag = abs(j - oracle.diagnostics(full, p, n)[2]) / abs(j)
    return max(e_series, e_diag)


def pin_convolution_direct_anisotropic():
    return pin_convolution_direct(16, 24, seed=40, s=(2.0, 0.5))


def pin_forcing_geometric_series(R=30.0, n1=32, n2=64, dt=0.5, steps=25, mode=(2, 3), integrator="euler"):
    """Constant radius R, constant forcing F on one small mode, zero start.

    Eq. (1) is then linear in that mode with a constant rate sigma_k. The
    integrating-factor Euler step Phi^{n+1} = E (Phi^n + dt F) sums to the
    geometric series dt F E (1 - E^n) / (1 - E), E = exp(dt sigma_k); Heun's
    Phi^{n+1} = E Phi^n + dt F (1 + E)/2 to dt F (1 + E)/2 (1 - E^n) / (1 - E)
    (both written by hand); the mirror mode must hold the conjugate.
    """
    f = np.zeros((n1, n2), dtype=np.complex128)
    a, b = mode
    f[a, b] = 1e-28 * (0.3 - 0.4j)
    f[-a, -b] = np.conj(f[a, b])
    p = oracle.Params(n1, n2, t0=1.0, dt=dt, gamma=GAMMA, r0_law=lambda t: R, forcing=f, integrator=integrator)
    out = oracle.run(np.zeros((n1, n2), dtype=np.complex128), p, steps)
    kap = np.hypot(float(a), float(b))
    e = np.exp(dt * (-kap ** 2 / R ** 2 + GAMMA * kap / (2.0 * R)))
    gain = e if integrator == "euler" else 0.5 * (1.0 + e)
    want = dt * f[a, b] * gain * (1.0 - e ** steps) / (1.0 - e)
    return max(abs(out[a, b] - want), abs(out[-a, -b] - np.conj(want))) / abs(want)


# ---------------------------------------------------------------- circles
# Pins of the circular-flame oracle (oracle/circle.py): the one-dimensional
# form of Eq. (1). Each is written from the definitions, not from the
# oracle's code.

def random_circle(n, rng, amp):
    """Hermitian coefficients on |k| <= K (full FFT-ordered array, Im of k = 0 zero)."""
    K = oracle.truncation(n)
    full = np.zeros(n, dtype=np.complex128)
    for k in range(1, K + 1):
        v = amp * (rng.standard_normal() + 1j * rng.standard_normal()) / k
        full[k] = v
        full[-k] = np.conj(v)
    full[0] = amp * rng.standard_normal()
    return full


def pin_circle_literal_sum(n=21, seed=50, s=1.0):
    """The oracle's FFT convolution against the literal double sum
    sum_l kappa_l kappa_{k-l} Phi_l Phi_{k-l} over |l|, |k - l| <= K."""
    rng = np.random.default_rng(seed)
    p = oracle.CircleParams(n, seg=s)
    full = random_circle(n, rng, 1.0)
    K = oracle.truncation(n)
    worst, scale = 0.0, 0.0
    got = oracle.circle_convolution_sum(full, p)
    for k in range(-K, K + 1):
        acc = 0j
        for l in range(-K, K + 1):
            if abs(k - l) <= K:
                acc += (s * l) * (s * (k - l)) * full[l % n] * full[(k - l) % n]
        worst = max(worst, abs(got[k % n] - acc))
        scale = max(scale, abs(acc))
    return worst / scale


def pin_circle_single_cosine(n=64, k=5, a=0.3, psi=0.7, s=2.0):
    """Phi = a cos(k phi + psi): Phi_phi = -a kappa sin(.), so the sum is
    -F[Phi_phi^2] with F[.]_0 = a^2 kappa^2/2 and F[.]_{+-2k} = -a^2 kappa^2/4 e^{+-2i psi}."""
    p = oracle.CircleParams(n, seg=s)
    full = np.zeros(n, dtype=np.complex128)
    full[k] = 0.5 * a * np.exp(1j * psi)
    full[-k] = np.conj(full[k])
    got = oracle.circle_convolution_sum(full, p)
    kap = s * k
    want = np.zeros(n, dtype=np.complex128)
    want[0] = -a * a * kap * kap / 2
    if 2 * k <= oracle.truncation(n):  # outside the box the sum is not kept
        want[2 * k] = a * a * kap * kap / 4 * np.exp(2j * psi)
        want[-2 * k] = np.conj(want[2 * k])
    return np.abs(got - want).max() / (a * a * kap * kap / 2)


def pin_circle_linear_growth(n=256, k=30, dt=0.5, nsteps=40, t0=200.0, s=1.0):
    """A tiny single mode grows as (t/t0)^(gamma kappa/2) exp(kappa^2 (1/t - 1/t0)),
    the exact solution of the linear part with r0 = t."""
    p = oracle.CircleParams(n, seg=s, t0=t0, dt=dt)
    full = np.zeros(n, dtype=np.complex128)
    full[k] = 1e-20 * (0.6 + 0.8j)
    full[-k] = np.conj(full[k])
    out = oracle.circle_run(full, p, nsteps)
    t = t0 + nsteps * dt
    kap = s * k
    g = (t / t0) ** (0.8 * kap / 2) * np.exp(kap * kap * (1.0 / t - 1.0 / t0))
    return abs(out[k] - g * full[k]) / abs(g * full[k])


def pin_circle_is_sphere_restriction(n1=16, n=40, s=(0.7, 1.5), steps=6, seed=51):
    """Eq. (1) maps states confined to k1 = 0 into themselves: the
    two-dimensional oracle run on such a state (axis scales s) must equal the
    circular oracle with segment integer s2, and keep every k1 != 0 mode zero."""
    rng = np.random.default_rng(seed)
    p2 = oracle.Params(n1, n, t0=3.0, dt=0.1, axis_scale=s)
    pc = oracle.CircleParams(n, seg=s[1], t0=3.0, dt=0.1)
    c = random_circle(n, rng, 0.3)
    full2 = np.zeros((n1, n), dtype=np.complex128)
    full2[0, :] = c
    out2 = oracle.run(full2, p2, steps)
    outc = oracle.circle_run(c, pc, steps)
    off = np.abs(out2[1:, :]).max()
    return max(np.abs(out2[0, :] - outc).max() / np.abs(outc).max(), off)


def pin_circle_k0_parseval(n=48, seed=52, dt=0.3):
    """k = 0 has sigma = 0, so one step adds dt c sum_l kappa_l^2 |Phi_l|^2 to Phi~_0."""
    rng = np.random.default_rng(seed)
    p = oracle.CircleParams(n, seg=1.3, t0=4.0, dt=dt)
    full = random_circle(n, rng, 0.2)
    out = oracle.circle_step(full, p, 0)
    t = p.t0
    kap = p.seg * oracle.wavenumbers(n)
    want = full[0].real + dt / (2 * t * t) * float((kap * kap * np.abs(full) ** 2).sum())
    return abs(out[0] - want) / abs(want)


def pin_circle_convergence(n=24, seed=53, T=1.0, t0=2.0, amp=0.4):
    """Integrating-factor Euler converges at first order to a DOP853 solution
    of the ODE written with the literal sum (errors at 20, 40, 80 steps)."""
    from scipy.integrate import solve_ivp
    rng = np.random.default_rng(seed)
    K = oracle.truncation(n)
    c0 = random_circle(n, rng, amp)
    ks = np.arange(-K, K + 1)

    def rhs(t, y):
        ph = y[: 2 * K + 1] + 1j * y[2 * K + 1:]
        out = np.zeros(2 * K + 1, dtype=np.complex128)
        for a, k in enumerate(ks):
            acc = 0j
            for b, l in enumerate(ks):
                if abs(k - l) <= K:
                    acc += l * (k - l) * ph[b] * ph[(k - l) + K]
            sig = -k * k / t ** 2 + 0.8 * abs(k) / (2 * t)
            out[a] = sig * ph[a] - acc / (2 * t * t)
        return np.concatenate([out.real, out.imag])

    y0 = np.array([c0[k % n] for k in ks])
    sol = solve_ivp(rhs, (t0, t0 + T), np.concatenate([y0.real, y0.imag]), method="DOP853", rtol=1e-12, atol=1e-14)
    ref = sol.y[: 2 * K + 1, -1] + 1j * sol.y[2 * K + 1:, -1]
    errs = []
    for steps in (20, 40, 80):
        p = oracle.CircleParams(n, t0=t0, dt=T / steps)
        out = oracle.circle_run(c0, p, steps)
        errs.append(np.abs(np.array([out[k % n] for k in ks]) - ref).max() / np.abs(ref).max())
    return errs


def pin_circle_diagnostics(n=128, k=3, a=0.4, psi=0.2, mean=0.01, nstep=2):
    """Single cosine: mean radius r0 + mean, <Phi_t> = a^2 kappa^2 / (4 r0^2),
    length excess the series of <sqrt(1 + b sin^2) - 1>, b = a^2 kappa^2 / r0^2."""
    p = oracle.CircleParams(n, seg=1.0, t0=3.0, dt=0.5)
    full = np.zeros(n, dtype=np.complex128)
    full[k] = 0.5 * a * np.exp(1j * psi)
    full[-k] = np.conj(full[k])
    full[0] = mean
    r = 3.0 + nstep * 0.5
    rbar, vel, exc = oracle.circle_diagnostics(full, p, nstep)
    kap = float(k)
    b = a * a * kap * kap / (r * r)
    return max(abs(rbar - (r + mean)) / (r + mean), abs(vel - a * a * kap * kap / (4 * r * r)) / (a * a * kap * kap / (4 * r * r)),
               abs(exc - area_series(b)) / area_series(b))
