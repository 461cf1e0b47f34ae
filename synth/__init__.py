"""Seeded synthetic workloads for the synchrotron-emission path.

This package holds only workload definitions: physical constants converted to
normalised units, the configurations, the initial particle states, the
prescribed standing-wave field sampled on a Yee grid, and the plasma weight and
laser pulse of the PIC-loop workload.  It contains none of the
emission method's arithmetic, and both the HIP path's tests and the CPU oracle
take their inputs from it.

Normalised units: c = m = e = 1; time in 1/omega_r, length c/omega_r, momentum
mc, fields eE/(mc omega_r) and eB/(m omega_r).
"""
from .workloads import (  # noqa: F401
    ALPHA, CONFIGS, Config, config, field_at, gen_particles, standing_wave_grid,
    yee_offsets, plasma_weight, laser_pulse_grid, C6_DENSITY,
)
