"""Integral diagnostics of the flame state in FP64 (oracle; test infrastructure only).

Section 3 (averages paragraph) mentions averages of the solution without
listing them; Section 2 plots the averaged flame velocity <Phi_t>.
The readings used here:

* mean radius  r_bar = r0(t) + Re Phi~_0  (r = r0 + Phi, Section 2);
* averaged velocity <Phi_t> = d Phi~_0/dt, the k = 0 component of Eq. (1)'s
  right-hand side (sigma_0 = 0, f = 0), i.e. the grid mean of
  |grad Phi|^2 / (2 r0^2) with the gradient in scaled (kappa) coordinates;
* area excess J = < sqrt(1 + x) - 1 > over the grid with
  x = |grad Phi|^2 / r0^2 (graph area of the segment in the model's local
  metric, relative to the reference segment), evaluated as x/(1 + sqrt(1 + x))
  to avoid the cancellation at small slopes.
"""

import numpy as np

from .spectral import synthesize


def gradient_fields(full, p):
    """Real grid fields g1 = d Phi/d x1, g2 = d Phi/d x2 in kappa scaling."""
    k1, k2 = p.kappa()
    g1 = synthesize(1j * k1 * full).real
    g2 = synthesize(1j * k2 * full).real
    return g1, g2


def diagnostics(full, p, n):
    """(mean radius, averaged velocity <Phi_t>, area excess J) at step n."""
    t = p.time(n)
    rr = p.r0(t)
    g1, g2 = gradient_fields(full, p)
    q = g1 * g1 + g2 * g2
    mean_radius = rr + full[0, 0].real
    velocity = q.mean() / (2.0 * rr * rr)
    x = q / (rr * rr)
    area = (x / (1.0 + np.sqrt(1.0 + x))).mean()
    return float(mean_radius), float(velocity), float(area)
