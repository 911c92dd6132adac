"""Spectral bookkeeping of the oracle (FP64, numpy).

Test infrastructure only (see the package docstring).

Conventions (Section 2, Eq. (1) and the truncation paragraph; Section 3,
augmented-array paragraph):

* The physical grid is N1 x N2 with nodes x_j = (2*pi*j1/N1, 2*pi*j2/N2).
* The field is a Fourier series, Phi(x) = sum_k Phi~_k exp(i k.x); Eq. (1)'s
  convolution form implies this normalisation (no 1/P on synthesis, 1/P on
  analysis, P = N1*N2).
* The retained box is |k1| <= K1, |k2| <= K2 with K_i = floor((N_i - 1)/4),
  so that N_i = 4 K_i + k0 + 1 with k0 >= 0 (Section 3: the augmented array
  has size 4K + k0 + 1).
* A "full" array is N1 x N2 complex in numpy FFT index order.
* A "half" array is the canonical exchange layout of the spectral state:
  shape (2K1+1, K2+1), entry [k1 + K1, k2] for k2 in [0, K2]. The k2 = 0
  column keeps both signs of k1.
"""

import numpy as np


def truncation(n):
    """K for an augmented-array size n: the largest K with 4K + 1 <= n."""
    if n < 5:
        raise ValueError("grid size must be at least 5")
    return (n - 1) // 4


def wavenumbers(n):
    """Integer wavenumber held at each FFT index 0..n-1."""
    idx = np.arange(n)
    return np.where(idx < (n + 1) // 2, idx, idx - n).astype(np.int64)


def box_mask(n1, n2):
    k1 = wavenumbers(n1)[:, None]
    k2 = wavenumbers(n2)[None, :]
    return (np.abs(k1) <= truncation(n1)) & (np.abs(k2) <= truncation(n2))


def half_shape(n1, n2):
    return (2 * truncation(n1) + 1, truncation(n2) + 1)


def half_to_full(half, n1, n2):
    """Spread the canonical half array over the full FFT-ordered array.

    Entries with k2 > 0 are mirrored to -k by Phi~(-k) = conj(Phi~(k)); the
    k2 = 0 column is copied as given (both signs of k1 are stored there).
    """
    K1, K2 = truncation(n1), truncation(n2)
    half = np.asarray(half)
    if half.shape != (2 * K1 + 1, K2 + 1):
        raise ValueError(f"half array has shape {half.shape}, expected {(2*K1+1, K2+1)}")
    full = np.zeros((n1, n2), dtype=np.complex128)
    k1 = np.arange(-K1, K1 + 1)
    rows = k1 % n1
    for k2 in range(K2 + 1):
        full[rows, k2] = half[:, k2]
    for k2 in range(1, K2 + 1):
        full[(-k1) % n1, (-k2) % n2] = np.conj(half[:, k2])
    return full


def full_to_half(full, n1, n2):
    K1, K2 = truncation(n1), truncation(n2)
    k1 = np.arange(-K1, K1 + 1)
    return np.asarray(full)[np.ix_(k1 % n1, np.arange(K2 + 1))].copy()


def synthesize(full):
    """Phi(x_j) = sum_k Phi~_k exp(i k.x_j) on the grid (complex result)."""
    full = np.asarray(full)
    return np.fft.ifft2(full) * full.size


def analyse(phys):
    """Phi~_k = (1/P) sum_j Phi(x_j) exp(-i k.x_j) for every k of the grid."""
    phys = np.asarray(phys)
    return np.fft.fft2(phys) / phys.size


def project(phys):
    """Galerkin projection of a grid field onto the retained box (full array)."""
    n1, n2 = np.asarray(phys).shape
    return analyse(phys) * box_mask(n1, n2)
