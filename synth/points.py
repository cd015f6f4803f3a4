"""Seeded point clouds inside the field-of-view cone of a hologram."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Seeds of the named workloads: 1024^2 60 deg, 4096^2 90 deg, 16384^2 120 deg,
# the 8192^2 serving hologram, and the base of the 64-hologram mixed batch
# (hologram i uses 1005 + i).
CONFIG_SEEDS = {"c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "c5": 1005}


def fov_pitch(wavelength: float, fov_deg: float) -> float:
    """Pixel pitch whose diffraction-limited field of view is ``fov_deg``."""
    return wavelength / (2.0 * math.sin(math.radians(fov_deg) / 2.0))


@dataclass
class PointCloud:
    x: np.ndarray      # metres
    y: np.ndarray      # metres
    z: np.ndarray      # metres, distance from the hologram plane
    amp: np.ndarray    # real amplitude
    phase: np.ndarray  # radians

    def __len__(self) -> int:
        return int(self.x.shape[0])

    def as_array(self) -> np.ndarray:
        """(P, 5) float64 array with columns x, y, z, amplitude, phase."""
        return np.stack([self.x, self.y, self.z, self.amp, self.phase], axis=1).copy()


def draw_points(seed: int, n_points: int, nx: int, ny: int, pitch: float,
                wavelength: float, z_lo: float, z_hi: float) -> PointCloud:
    """Draw ``n_points`` points with ``numpy.random.Generator(PCG64(seed))``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = wavelength / (2.0 * pitch)
    if not (0.0 < s < 1.0):
        raise ValueError("wavelength / (2 pitch) must lie in (0, 1)")
    tan_t = s / math.sqrt(1.0 - s * s)
    z = rng.uniform(z_lo, z_hi, n_points)
    half_ap = 0.5 * max(nx, ny) * pitch
    lim = 0.9 * (z * tan_t - half_ap)
    if np.any(lim <= 0.0):
        raise ValueError("points too close: the aperture is wider than the cone")
    x = rng.uniform(-1.0, 1.0, n_points) * lim
    y = rng.uniform(-1.0, 1.0, n_points) * lim
    amp = rng.uniform(0.5, 1.0, n_points)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_points)
    return PointCloud(x=x, y=y, z=z, amp=amp, phase=phase)
