"""Holograms of point sources, written out from their definition in float64.

Pixel (i, j) of an ``ny x nx`` hologram with pitch ``pitch`` sits at
``x = (j - nx/2) pitch``, ``y = (i - ny/2) pitch`` in the hologram plane.
"""
from __future__ import annotations

import math

import numpy as np

from .points import PointCloud


def point_hologram(points: PointCloud, nx: int, ny: int, pitch: float,
                   wavelength: float, rows_per_block: int = 64) -> np.ndarray:
    """Diverging-wave hologram ``H = sum_p a_p e^{i phi_p} e^{i k r} / r``.

    ``r`` is the distance from the pixel to point p.  Returns complex128
    ``[ny, nx]``.  The sum runs point by point in float64.
    """
    k = 2.0 * math.pi / wavelength
    xs = (np.arange(nx) - nx // 2) * pitch
    out = np.zeros((ny, nx), dtype=np.complex128)
    coef = points.amp * np.exp(1j * points.phase)
    for r0 in range(0, ny, rows_per_block):
        r1 = min(ny, r0 + rows_per_block)
        ys = (np.arange(r0, r1) - ny // 2) * pitch
        acc = np.zeros((r1 - r0, nx), dtype=np.complex128)
        for p in range(len(points)):
            dx2 = (xs - points.x[p]) ** 2
            dy2 = (ys - points.y[p]) ** 2
            r = np.sqrt(dy2[:, None] + dx2[None, :] + points.z[p] ** 2)
            acc += coef[p] * np.exp(1j * k * r) / r
        out[r0:r1] = acc
    return out


def point_hologram_at(points: PointCloud, rows: np.ndarray, cols: np.ndarray,
                      nx: int, ny: int, pitch: float, wavelength: float) -> np.ndarray:
    """The same field as :func:`point_hologram`, at selected pixels only."""
    k = 2.0 * math.pi / wavelength
    x = (np.asarray(cols) - nx // 2) * pitch
    y = (np.asarray(rows) - ny // 2) * pitch
    acc = np.zeros(x.shape, dtype=np.complex128)
    coef = points.amp * np.exp(1j * points.phase)
    for p in range(len(points)):
        r = np.sqrt((x - points.x[p]) ** 2 + (y - points.y[p]) ** 2 + points.z[p] ** 2)
        acc += coef[p] * np.exp(1j * k * r) / r
    return acc


def converging_point_hologram(xo: float, yo: float, zo: float, nx: int, ny: int,
                              pitch: float, wavelength: float) -> np.ndarray:
    """Unit-amplitude wave converging to (xo, yo, zo): ``exp(-i k R_o)``."""
    k = 2.0 * math.pi / wavelength
    xs = (np.arange(nx) - nx // 2) * pitch
    ys = (np.arange(ny) - ny // 2) * pitch
    R = np.sqrt((xs[None, :] - xo) ** 2 + (ys[:, None] - yo) ** 2 + zo * zo)
    return np.exp(-1j * k * R)
