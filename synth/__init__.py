"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws point clouds and evaluates the point-source holograms the
reconstruction is tested and benchmarked on.  It holds none of the NU-FDS
arithmetic (no spectra, stretch maps, Fresnel transforms or interpolation):
a hologram here is only the field radiated by a set of points, written out
from its definition.

Point clouds follow the recipe used for every configuration: for each point,
in this order over the whole cloud, ``z_p ~ U[z_lo, z_hi]``, then ``x_p`` and
``y_p ~ U[-L, L]`` with ``L = 0.9 (z_p tan(theta) - N pitch / 2)`` (inside the
field-of-view cone, with a margin that keeps the local frequency of every
point below the Nyquist limit over the whole aperture), then amplitude
``a ~ U[0.5, 1]`` and phase ``phi ~ U[0, 2 pi)``.  ``sin(theta) =
wavelength / (2 pitch)``.
"""
from .points import PointCloud, draw_points, CONFIG_SEEDS, fov_pitch
from .hologram import point_hologram, point_hologram_at, converging_point_hologram

__all__ = ["PointCloud", "draw_points", "CONFIG_SEEDS", "fov_pitch",
           "point_hologram", "point_hologram_at", "converging_point_hologram"]
