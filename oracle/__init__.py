"""FP64 CPU oracle for the pseudo-spectral flame-front step of Eq. (1).

This package is test infrastructure. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product library
never calls it and shares no code with it.

What it follows (V. Karlin, "Global communications in multiprocessor
simulations of flames"):

* Section 2, Eq. (1): the Fourier-space evolution equation for the flame
  perturbation, with the reference radius r0(t) = t (or a given law) and no
  forcing.
* Section 2, truncation paragraph: harmonics beyond K are dropped and the
  quadratic term is a circular convolution evaluated with FFTs.
* Section 3, augmented-array paragraph: the K_Psi = 4K + k0 + 1 padded array,
  column transforms of k1*Psi and k2*Psi, transpose, row transforms,
  element-by-element product, and the same in reverse.
* Section 3, symmetrisation paragraph and its figure: the upper half of the
  spectrum is copied onto the lower half by Psi(-k) = conj(Psi(k)).
* Section 3, averages paragraph and Section 2 (averaged flame velocity).
* Section 2, the circular flames of the averaged-velocity figure: a reading
  (the one-dimensional form of Eq. (1)) in ``circle.py``.

Readings where the paper is silent are listed in ``model.py`` and in the
design notes; the integrator (integrating-factor Euler) is one of them, so
agreement with the paper's own unstated integrator is "parity unpinned".
Everything else here is pinned by the CPU tests in ``tests/test_oracle_*.py``.
"""

from .spectral import (  # noqa: F401
    truncation, wavenumbers, box_mask, half_shape, half_to_full, full_to_half,
    synthesize, analyse, project,
)
from .model import (  # noqa: F401
    Params, step_scalars, growth_exponent, convolution_sum, rhs, symmetrise,
    step, run, set_fft_workers,
)
from .diagnostics import diagnostics  # noqa: F401
from .adjoint import (  # noqa: F401
    area_gradient, step_adjoint, trajectory_gradient, area_excess,
)
from .circle import (  # noqa: F401
    CircleParams, circle_symmetrise, circle_convolution_sum, circle_scalars, circle_step, circle_run,
    circle_diagnostics, half_to_circle, circle_to_half,
)
