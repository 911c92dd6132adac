"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package draws random numbers and lays them out; it holds none of the
method's arithmetic (no transforms, no time stepping), so both the product
path and the oracle can consume what it makes.
"""

from .ics import (  # noqa: F401
    ENSEMBLE_GROUPS, WORKLOADS, Workload, circle_spectra, ensemble_members, forcing_spectrum, half_dims,
    mode_table,
    modal_spectrum, physical_noise, workload_spectrum,
)
