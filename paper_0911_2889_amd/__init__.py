"""MI355X-native spectral stepper for the Sivashinsky-type flame model of
Eq. (1) (V. Karlin, "Global communications in multiprocessor simulations of
flames"): HIP kernels for gfx950 behind the C ABI in include/flame.h.

The compute path is the in-tree library libflamefront.so; importing the
classes below requires it to be built (``python -m paper_0911_2889_amd.build``).
"""

from .sim import CircleBatch, FlameEnsemble, FlameSim, flame_area  # noqa: F401
