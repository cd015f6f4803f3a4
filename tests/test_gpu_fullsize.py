"""GPU checks at the full sizes the benchmark times (16384^2 at 120 deg, 4096^2 at 90 deg).

The float64 oracle cannot run these sizes in a test, so they are checked through properties that
hold at any size: the complex64 path against the all-float64 path (rel-L2 <= 1e-4, the bar of the
float32 path), finiteness, run-to-run determinism, and the focus of a single wide-angle point source
at its true position (the property the method exists for, Sec. 4).  The launch configuration is
the one bench.py times (same plan geometry, full view).
"""
import math
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_13474_amd import nufds as N  # noqa: E402

LAM = 0.5e-6


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
    torch.cuda.empty_cache()


def _gpu_hologram(n, fov, seed, n_points, z_lo, z_hi):
    dp = synth.fov_pitch(LAM, fov)
    pc = synth.draw_points(seed, n_points, n, n, dp, LAM, z_lo, z_hi)
    H = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    N.synth_hologram(pc.as_array(), n, n, dp, LAM, H)
    return dp, H


def _rel(a, b):
    return float(torch.linalg.vector_norm(a.to(torch.complex128) - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("n,fov,z,seed,pts,zlo,zhi", [
    (16384, 120.0, 15e-3, 1003, 1024, 10e-3, 20e-3),
    (4096, 90.0, 7.5e-3, 1002, 4096, 5e-3, 10e-3),
])
def test_fullsize_fp32_path_matches_fp64_path(n, fov, z, seed, pts, zlo, zhi):
    say(f"full size {n} {fov}: complex64 vs complex128")
    dp, H128 = _gpu_hologram(n, fov, seed, pts, zlo, zhi)
    p128 = N.Plan(LAM, dp, n, n, z, precision="c128")
    o128 = p128(H128)
    torch.cuda.synchronize()
    p128.close()
    H64 = H128.to(torch.complex64)
    del H128
    p64 = N.Plan(LAM, dp, n, n, z, precision="c64")
    o64 = p64(H64)
    o64b = p64(H64)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(o64)).all()
    assert torch.isfinite(torch.view_as_real(o128)).all()
    assert torch.equal(o64, o64b)                    # run to run
    err = _rel(o64, o128)
    say(f"  rel L2 complex64 vs complex128: {err:.3e}")
    assert err <= 1e-4
    p64.close()


@pytest.mark.parametrize("where", ["axis", "off_axis_diagonal"])
def test_fullsize_point_focus(where):
    """One point at 16384^2 / 120 deg, z = 15 mm (about 3.2 apertures), view of 256^2 at Delta_F
    centred on it.  On the axis the focus sits exactly at the view centre by symmetry, which exercises
    the full-size index arithmetic.  Off the axis the method itself displaces the focus: the stretch
    and the output map of Eqs. 17-18 follow the wave's frequency at the hologram centre, and the
    residual aberration over a wide aperture grows with the number of samples at a fixed geometry
    (the float64 oracle and this path agree on it at 1024^2-8192^2: 1, 1, 7 and 15 samples at 46 deg),
    and even on the axis the focus spreads as the band widens (oracle, 9 x 9-sample energy 0.99, 0.96,
    0.88 at 1024^2, 2048^2, 4096^2 of the same geometry).
    Here the point sits on the diagonal at 20 deg, where the oracle's runs of the same geometry
    scaled to 2048^2, 4096^2 and 8192^2 put it 1, 1 and 2 samples off; the bar is 5."""
    say(f"full size point focus ({where})")
    n = 16384
    dp = synth.fov_pitch(LAM, 120.0)
    z = 15e-3
    if where == "axis":
        x0 = y0 = 0.0
        tol = 1
    else:
        r = z * math.tan(math.radians(20.0)) / math.sqrt(2.0)
        x0, y0 = r, -r
        tol = 5
    pts = np.array([[x0, y0, z, 1.0, 0.3]], dtype=np.float64)
    H = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    N.synth_hologram(pts, n, n, dp, LAM, H)
    view = dict(center_x=x0, center_y=y0, pitch_x=0.0, pitch_y=0.0, nx=256, ny=256)
    plan = N.Plan(LAM, dp, n, n, z, view=view, precision="c64")
    out = plan(H)
    torch.cuda.synchronize()
    a = out.abs()
    i, j = divmod(int(torch.argmax(a)), 256)
    say(f"  peak at ({i}, {j}), centre (128, 128)")
    assert abs(i - 128) <= tol and abs(j - 128) <= tol
    # a focus, not noise: the peak stands far above the mean of the view (the method's own
    # aberration at this geometry spreads it over a few samples; see the docstring)
    assert float(a.max()) > 20.0 * float(a.mean())
    plan.close()


def test_fullsize_focal_stack_matches_plans():
    """16384^2 / 120 deg (the benchmark's hologram), depths 15 and 20 mm sharing the FrT size of the
    nearer one (M = 25600): each depth against a complex64 plan at that depth with the same size
    (the same method through the chained passes; float32 rounding apart, rel-L2 <= 1e-5)."""
    say("full size focal stack")
    n = 16384
    dp, H128 = _gpu_hologram(n, 120.0, 1003, 1024, 10e-3, 20e-3)
    H = H128.to(torch.complex64)
    del H128
    zs = [15e-3, 20e-3]
    st = N.Stack(LAM, dp, n, n, zs, precision="c64")
    assert {(i["mx"], i["my"]) for i in st.infos} == {(25600, 25600)}
    outs = st(H)
    torch.cuda.synchronize()
    for z, o, info in zip(zs, outs, st.infos):
        assert torch.isfinite(torch.view_as_real(o)).all()
        plan = N.Plan(LAM, dp, n, n, z, precision="c64", frt_size=(info["mx"], info["my"]))
        ref = plan(H)
        torch.cuda.synchronize()
        err = _rel(o, ref)
        say(f"  z {z * 1e3:.1f} mm: rel L2 stack vs plan {err:.3e}")
        assert err <= 1e-5
        plan.close()
        del ref
    st.close()
