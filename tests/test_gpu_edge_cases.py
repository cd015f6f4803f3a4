"""Edge cases of the reconstruction on the GPU, each against the float64 oracle.

An all-zero hologram (exactly zero output), the smallest holograms, a rectangular one with few rows,
one-pixel and odd-sized views at the corner of the image area, and a 170 deg field of view, where
the band reaches close to the rim of the propagating disk (the stretch's pre-images and their
Jacobian are singular at the rim, reading 5).
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_13474_amd import nufds as N  # noqa: E402

LAM = 0.5e-6
TOL = {"c128": 1e-10, "c64": 1e-4}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    N.load()
    yield
    torch.cuda.synchronize()


def _run(H, dp, z, prec, view=None, flags=0):
    ny, nx = H.shape
    dt = np.complex64 if prec == "c64" else np.complex128
    Ht = torch.from_numpy(H.astype(dt)).cuda()
    plan = N.Plan(LAM, dp, nx, ny, z, view=view, precision=prec, flags=flags)
    out = plan(Ht).cpu().numpy().astype(np.complex128)
    plan.close()
    return out


def _check(H, dp, z, prec, view=None, flags=0):
    got = _run(H, dp, z, prec, view=view, flags=flags)
    src = H.astype(np.complex64).astype(np.complex128) if prec == "c64" else H
    ref = O.reconstruct(src, LAM, dp, z, view=view, flags=flags)
    assert got.shape == ref.shape
    err = O.rel_l2(got, ref)
    say(f"   {H.shape} view {None if view is None else (view['nx'], view['ny'])}: rel L2 {err:.2e}")
    assert err <= TOL[prec]


def _points(seed, n_points, nx, ny, fov):
    dp = synth.fov_pitch(LAM, fov)
    pc = synth.draw_points(seed, n_points, nx, ny, dp, LAM, 4 * max(nx, ny) * dp, 6 * max(nx, ny) * dp)
    return dp, float(np.median(pc.z)), synth.point_hologram(pc, nx, ny, dp, LAM)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_zero_hologram_gives_zero(prec):
    say(f"zero hologram {prec}")
    dp = synth.fov_pitch(LAM, 120.0)
    H = np.zeros((128, 192), dtype=np.complex128)
    out = _run(H, dp, 1e-4, prec)
    assert np.count_nonzero(out) == 0
    B = O.image_size(LAM, dp, 1e-4)
    out = _run(H, dp, 1e-4, prec, view=dict(center_x=0.3 * B, center_y=0.1 * B, pitch_x=0.0, pitch_y=0.0,
                                              nx=40, ny=24))
    assert out.shape == (24, 40) and np.count_nonzero(out) == 0


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(16, 16), (8, 12), (10, 256)])
def test_small_holograms(prec, shape):
    say(f"small hologram {shape} {prec}")
    ny, nx = shape
    dp, z, H = _points(40 + nx + ny, 2, nx, ny, 90.0)
    _check(H, dp, z, prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_one_pixel_and_odd_views_at_the_corner(prec):
    say(f"corner views {prec}")
    n = 96
    dp, z, H = _points(51, 3, n, n, 120.0)
    B = O.image_size(LAM, dp, z)
    df = LAM * z / (n * dp)
    for nxv, nyv in ((1, 1), (3, 5), (7, 2)):
        # the window's far corner one FrT sample inside the image corner (B/2, -B/2)
        cx = 0.5 * B - (nxv / 2 + 1) * df
        cy = -0.5 * B + (nyv / 2 + 1) * df
        _check(H, dp, z, prec, view=dict(center_x=cx, center_y=cy, pitch_x=0.0, pitch_y=0.0, nx=nxv, ny=nyv))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_near_rim_field_of_view(prec):
    """FoV 170 deg: s = sin 85 deg, the band's corners are deep in the evanescent region and its edge
    samples pre-images within a few 1e-3 of the rim."""
    say(f"170 deg {prec}")
    n = 64
    dp, z, H = _points(52, 3, n, n, 170.0)
    _check(H, dp, z, prec)
    _check(H, dp, z, prec, flags=N.FLAG_NO_REMAP)
