"""Seeded initial perturbations for the flame workloads.

The paper's own runs start from Phi(theta, phi, t0) = eps * eta with eta
drawn uniformly in [-1, 1] at every grid node, eps = 1e-3 and t0 = 200
(Section 2). The benchmark workloads below instead start from sums of
random cosine modes a_k cos(k.x + psi_k) over k in the upper half-plane
H = {k2 > 0} or {k2 = 0, k1 > 0}; their Fourier coefficients are
Phi~_{+k} = (a_k/2) exp(+i psi_k) and Phi~_{-k} = (a_k/2) exp(-i psi_k).

Draw order for a modal IC with generator numpy.random.default_rng(seed):
the mode set (if it is a random subset), then amplitudes xi ~ N(0, 1) for
every mode, then phases psi ~ U(0, 2 pi); a_k = amp * xi_k * |k|^power.
Coefficients are returned rounded to complex64, the precision both the
GPU path and (after widening) the oracle start from.

Layout returned: the canonical half array of shape (2K1+1, K2+1) with entry
[k1 + K1, k2], K_i = floor((N_i - 1)/4). Both signs of k1 are filled in the
k2 = 0 column.
"""

from dataclasses import dataclass

import numpy as np


def half_dims(n1, n2):
    k1max, k2max = (n1 - 1) // 4, (n2 - 1) // 4
    return k1max, k2max


def _upper_half_modes(k1max, k2max):
    """All k in H within the box, lexicographic in (k1, k2)."""
    k1 = np.arange(-k1max, k1max + 1)
    k2 = np.arange(0, k2max + 1)
    a, b = np.meshgrid(k1, k2, indexing="ij")
    a, b = a.ravel(), b.ravel()
    keep = (b > 0) | ((b == 0) & (a > 0))
    return a[keep], b[keep]


def mode_table(n1, n2, rule, amp, power, seed, count=None, max_box=None, max_norm=None):
    """Draw (k1, k2, a, psi) arrays for a modal initial condition.

    rule: "box"   -> k in H with 1 <= max(|k1|, |k2|) <= max_box,
                     a random subset of `count` modes without replacement;
          "disc"  -> every k in H with 1 <= |k| <= max_norm;
          "all"   -> every k in H within the retained box.
    """
    k1max, k2max = half_dims(n1, n2)
    rng = np.random.default_rng(seed)
    k1, k2 = _upper_half_modes(k1max, k2max)
    if rule == "box":
        m = np.maximum(np.abs(k1), np.abs(k2))
        sel = (m >= 1) & (m <= max_box)
        k1, k2 = k1[sel], k2[sel]
        pick = rng.choice(k1.size, size=count, replace=False)
        k1, k2 = k1[pick], k2[pick]
    elif rule == "disc":
        r = np.hypot(k1, k2)
        sel = (r >= 1) & (r <= max_norm)
        k1, k2 = k1[sel], k2[sel]
    elif rule == "all":
        pass
    else:
        raise ValueError(rule)
    xi = rng.standard_normal(k1.size)
    psi = rng.uniform(0.0, 2.0 * np.pi, k1.size)
    a = amp * xi * np.hypot(k1, k2) ** power
    return k1, k2, a, psi


def modal_spectrum(n1, n2, k1, k2, a, psi):
    """Canonical half array (complex64) of sum_k a_k cos(k.x + psi_k)."""
    k1max, k2max = half_dims(n1, n2)
    half = np.zeros((2 * k1max + 1, k2max + 1), dtype=np.complex128)
    coef = 0.5 * a * np.exp(1j * psi)
    half[k1 + k1max, k2] += coef
    zero_col = k2 == 0
    half[-k1[zero_col] + k1max, 0] += np.conj(coef[zero_col])
    return half.astype(np.complex64)


def physical_noise(n1, n2, seed, kind="uniform", scale=1.0):
    """Grid field of independent draws per node, float32.

    kind "uniform": scale * U(-1, 1) (the paper's eps * eta with scale = eps);
    kind "normal":  scale * N(0, 1) (random directions for gradient checks).
    """
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        v = rng.uniform(-1.0, 1.0, size=(n1, n2))
    elif kind == "normal":
        v = rng.standard_normal((n1, n2))
    else:
        raise ValueError(kind)
    return (scale * v).astype(np.float32)


@dataclass(frozen=True)
class Workload:
    name: str
    n1: int
    n2: int
    steps: int
    dt: float
    rule: str
    amp: float
    power: float
    seed: int
    count: int = None
    max_box: int = None
    max_norm: float = None
    gamma: float = 0.8
    theta_pi: float = 1.0
    t0: float = 200.0

    @property
    def points(self):
        return self.n1 * self.n2

    def modes(self, seed=None):
        return mode_table(self.n1, self.n2, self.rule, self.amp, self.power,
                          self.seed if seed is None else seed, count=self.count,
                          max_box=self.max_box, max_norm=self.max_norm)


WORKLOADS = {
    # one flame, 64 x 128, 200 steps: 32 random low-wavenumber modes, N(0, 1e-3)
    "flame64x128": Workload("flame64x128", 64, 128, 200, 0.25, "box", 1e-3, 0.0, 0,
                            count=32, max_box=8),
    # one flame, 512 x 1024, 1000 steps: modes up to |k| = 64, amplitudes N(0,1e-3)/|k|
    "flame512x1024": Workload("flame512x1024", 512, 1024, 1000, 0.05, "disc", 1e-3, -1.0, 2,
                              max_norm=64),
    # one flame, 2048 x 4096, 500 steps: spectrum-shaped perturbation of every mode
    "flame2048x4096": Workload("flame2048x4096", 2048, 4096, 500, 0.1, "all", 1e-3, -1.0, 1),
    # adjoint workload, 1024 x 2048, 500 steps, modes up to |k| = 64
    "adjoint1024x2048": Workload("adjoint1024x2048", 1024, 2048, 500, 0.1, "disc", 1e-3, -1.0, 5,
                                 max_norm=64),
    # nonlinear stress case, 256 x 512, amplitudes 100x larger
    "stress256x512": Workload("stress256x512", 256, 512, 500, 0.1, "disc", 1e-1, -1.0, 3,
                              max_norm=64),
}

# Batched ensemble: 128 flames of 128 x 256, 96 of 256 x 512, 32 of 512 x 1024,
# 200 steps each, modes |k| <= 16, seed 1000 + flame index.
ENSEMBLE_GROUPS = ((128, 128, 256), (96, 256, 512), (32, 512, 1024))


def ensemble_members():
    out = []
    idx = 0
    for count, n1, n2 in ENSEMBLE_GROUPS:
        for _ in range(count):
            out.append(Workload(f"member{idx}", n1, n2, 200, 0.25, "disc", 1e-3, -1.0,
                                1000 + idx, max_norm=16))
            idx += 1
    return out


def workload_spectrum(w, seed=None):
    k1, k2, a, psi = w.modes(seed)
    return modal_spectrum(w.n1, w.n2, k1, k2, a, psi)


def forcing_spectrum(w, amp=1e-5, seed=None):
    """Seeded forcing f~_k of Eq. (1) for workload w (the paper's runs use f~ = 0):
    every mode of the retained box, a_k = amp * xi_k / |k| with random phases
    (the "all" rule above), drawn with seed w.seed + 7919 unless given;
    canonical half array, complex64."""
    k1, k2, a, psi = mode_table(w.n1, w.n2, "all", amp, -1.0, w.seed + 7919 if seed is None else seed)
    return modal_spectrum(w.n1, w.n2, k1, k2, a, psi)


def circle_spectra(n, count, seed, amp, power=-1.0):
    """Seeded initial spectra of `count` circular flames of n points: for each
    circle in turn, amplitudes xi_k ~ N(0, 1) for k = 1 .. K, then phases
    psi_k ~ U(0, 2 pi), with generator numpy.random.default_rng(seed);
    Phi~_k = (a_k / 2) exp(i psi_k), a_k = amp xi_k k^power (the cosine
    modes a_k cos(k phi + psi_k)), Phi~_0 = 0. Returns a complex64 array of
    shape (count, K + 1), K = floor((n - 1)/4), entry k = 0 .. K."""
    rng = np.random.default_rng(seed)
    K = (n - 1) // 4
    k = np.arange(1, K + 1, dtype=np.float64)
    out = np.zeros((count, K + 1), dtype=np.complex64)
    for c in range(count):
        a = amp * rng.standard_normal(K) * k ** power
        psi = rng.uniform(0.0, 2.0 * np.pi, K)
        out[c, 1:] = (0.5 * a * np.exp(1j * psi)).astype(np.complex64)
    return out
