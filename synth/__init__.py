"""Seeded synthetic workloads for the synchrotron-emission path.

This package holds only workload definitions: physical constants converted to
normalised units, the five configurations, the initial particle states and the
prescribed standing-wave field sampled on a Yee grid.  It contains none of the
emission method's arithmetic, and both the HIP path's tests and the CPU oracle
take their inputs from it.

Normalised units: c = m = e = 1; time in 1/omega_r, length c/omega_r, momentum
mc, fields eE/(mc omega_r) and eB/(m omega_r).
"""
from .workloads import (  # noqa: F401
    ALPHA, CONFIGS, Config, config, field_at, gen_particles, standing_wave_grid,
    yee_offsets,
)
