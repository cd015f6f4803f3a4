"""GPU parity: libnufds through its C ABI against the float64 oracle, element by element.

Bars: relative L2 error <= 1e-10 for the all-float64 path (NUFDS_C128) and
<= 1e-4 for complex64 data with float64 maps and phases (NUFDS_C64).  The
float32 path is compared on the same input rounded to complex64.  Sizes
span several LDS tiles and ragged tails; the four-step passes are driven at
small sizes by lowering the tile capacity (NUFDS_MAX_TILE_ELEMS).
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_13474_amd import nufds as N  # noqa: E402

TOL = {"c128": 1e-10, "c64": 1e-4}
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


def _tile_cap(cap):
    if cap:
        os.environ["NUFDS_MAX_TILE_ELEMS"] = str(cap)
    else:
        os.environ.pop("NUFDS_MAX_TILE_ELEMS", None)


def _hologram(seed, n_points, nx, ny, fov, z_lo, z_hi):
    dp = synth.fov_pitch(LAM, fov)
    pc = synth.draw_points(seed, n_points, nx, ny, dp, LAM, z_lo, z_hi)
    return dp, pc, synth.point_hologram(pc, nx, ny, dp, LAM)


def _gpu_run(H, dp, z, prec, view=None, flags=0, pad=None, frt_size=None, tile_cap=None, oversample=None,
             map_model=None):
    _tile_cap(tile_cap)
    try:
        ny, nx = H.shape
        plan = N.Plan(LAM, dp, nx, ny, z, view=view, precision=prec, flags=flags, pad=pad, frt_size=frt_size,
                      oversample=oversample, map_model=map_model)
    finally:
        _tile_cap(None)
    dt = torch.complex64 if prec == "c64" else torch.complex128
    Ht = torch.from_numpy(H.astype(np.complex64 if prec == "c64" else np.complex128)).to("cuda")
    out = plan(Ht)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128), plan


def _oracle_input(H, prec):
    return H.astype(np.complex64).astype(np.complex128) if prec == "c64" else H


# ------------------------------------------------------------- test input generator

@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_synth_matches_cpu_generator(prec):
    say(f"synth {prec}")
    nx, ny = 200, 136
    dp = synth.fov_pitch(LAM, 90.0)
    pc = synth.draw_points(77, 9, nx, ny, dp, LAM, 1e-3, 2e-3)
    ref = synth.point_hologram(pc, nx, ny, dp, LAM)
    dt = torch.complex64 if prec == "c64" else torch.complex128
    out = torch.empty((ny, nx), dtype=dt, device="cuda")
    N.synth_hologram(pc.as_array(), nx, ny, dp, LAM, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    # float64 phases k r ~ 3e4 rad: the two evaluation orders differ by a few ulp of k r
    assert err <= (1e-10 if prec == "c128" else 2e-7)


# ------------------------------------------------------------- stage parity

@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(256, 256), (320, 192)])
def test_spectrum_parity(prec, shape):
    nx, ny = shape
    say(f"spectrum {prec} {shape}")
    dp, pc, H = _hologram(5, 6, nx, ny, 90.0, 4 * nx * dp_(90.0), 6 * nx * dp_(90.0))
    z = float(np.mean(pc.z))
    _, plan = _gpu_run(H, dp, z, prec)
    got = plan.debug_copy(1).cpu().numpy().astype(np.complex128)
    ref = O.centred_dft2(np.conj(_oracle_input(H, prec)))
    assert O.rel_l2(got, ref) <= (1e-13 if prec == "c128" else 1e-6)


def dp_(fov):
    return synth.fov_pitch(LAM, fov)


@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
def test_map_table_parity(fov):
    say(f"map table {fov}")
    n = 512
    dp = dp_(fov)
    z = 6 * n * dp
    H = np.zeros((n, n), dtype=np.complex128)
    _, plan = _gpu_run(H, dp, z, "c128")
    tab = plan.debug_copy(3).cpu().numpy().reshape(-1, 2)
    b = O.plan_band(n, n, LAM, dp, z)
    kx_ext = max(abs(b.kcx - b.mx // 2), abs(b.kcx + b.mx // 2 - 1))
    nxt = int(round(math.sqrt(tab.shape[0])))  # square band here
    assert nxt * nxt == tab.shape[0]
    k = np.arange(nxt, dtype=np.float64)
    KX, KY = np.meshgrid(k, k)
    up = KX * LAM / (n * dp)
    vp = KY * LAM / (n * dp)
    u, v, valid = O.inverse_stretch(up, vp)
    s = LAM / (2 * dp)
    valid = valid & (np.abs(u) <= s) & (np.abs(v) <= s)
    gx = tab[:, 0].reshape(nxt, nxt)
    gy = tab[:, 1].reshape(nxt, nxt)
    assert np.array_equal(~np.isnan(gx), valid)
    px, py = u * (n * dp / LAM), v * (n * dp / LAM)
    assert np.max(np.abs(gx[valid] - px[valid])) <= 1e-9
    assert np.max(np.abs(gy[valid] - py[valid])) <= 1e-9
    assert nxt - 1 <= kx_ext


# ------------------------------------------------------------- end to end

def _check(H, dp, z, prec, view=None, flags=0, pad=None, frt_size=None, tile_cap=None, tol=None, oversample=None,
           map_model=None):
    got, plan = _gpu_run(H, dp, z, prec, view=view, flags=flags, pad=pad, frt_size=frt_size, tile_cap=tile_cap,
                         oversample=oversample, map_model=map_model)
    ref = O.reconstruct(_oracle_input(H, prec), LAM, dp, z, view=view, flags=flags, pad=pad, frt_size=frt_size,
                        oversample=oversample or 1, map_model=map_model or "exact")
    err = O.rel_l2(got, ref)
    say(f"   rel_l2 = {err:.3e}  (M = {plan.info['mx']} x {plan.info['my']})")
    assert err <= (tol or TOL[prec])
    return plan


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
def test_full_view_parity(prec, fov):
    say(f"full view {prec} {fov}")
    n = 256
    dp = dp_(fov)
    dp, pc, H = _hologram(int(fov) + 11, 5, n, n, fov, 4 * n * dp, 7 * n * dp)
    _check(H, dp, float(np.median(pc.z)), prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_rectangular_hologram_parity(prec):
    say(f"rectangular {prec}")
    nx, ny = 384, 256
    dp = dp_(100.0)
    dp, pc, H = _hologram(31, 4, nx, ny, 100.0, 4 * nx * dp, 6 * nx * dp)
    _check(H, dp, float(pc.z[0]), prec)


PARTIAL = [
    # view centre as a fraction of B/2, output size, output pitch in units of Delta_F
    ((0.3, -0.2), (200, 136), 1.0),
    ((-0.55, 0.4), (97, 61), 0.5),
    ((0.0, 0.6), (128, 40), 2.0),
    ((0.7, 0.7), (1, 1), 1.0),
]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(PARTIAL)))
def test_partial_view_parity(prec, case):
    (fx, fy), (sx, sy), pf = PARTIAL[case]
    say(f"partial {prec} case {case}")
    n = 320
    dp = dp_(120.0)
    dp, pc, H = _hologram(100 + case, 6, n, n, 120.0, 3 * n * dp, 5 * n * dp)
    z = float(pc.z[1])
    B = O.image_size(LAM, dp, z)
    df = LAM * z / (n * dp)
    do = pf * df
    cx = fx * (0.5 * B - 0.5 * sx * do)
    cy = fy * (0.5 * B - 0.5 * sy * do)
    view = dict(center_x=cx, center_y=cy, pitch_x=do, pitch_y=do, nx=sx, ny=sy)
    _check(H, dp, z, prec, view=view, tol=None if sx * sy > 1 else TOL[prec] * 10)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("flags", [O.CONVERGING, O.NO_REMAP, O.NO_STRETCH, O.NO_STRETCH | O.NO_REMAP])
def test_flag_parity(prec, flags):
    say(f"flags {prec} {flags}")
    n = 256
    dp = dp_(90.0)
    dp, pc, H = _hologram(7 + flags, 4, n, n, 90.0, 4 * n * dp, 6 * n * dp)
    if flags & O.CONVERGING:
        H = np.conj(H)
    z = float(pc.z[0])
    B = O.image_size(LAM, dp, z)
    view = dict(center_x=0.1 * B, center_y=-0.05 * B, pitch_x=0.0, pitch_y=0.0, nx=160, ny=120)
    _check(H, dp, z, prec, view=view, flags=flags)


def test_small_fov_identity_on_gpu():
    """NO_STRETCH | NO_REMAP with M = S = N, K_c = 0, Delta_o = Delta_F, pad = 0 is the plain FrT of Eq. 2."""
    say("identity")
    n = 192
    dp, z = 0.5e-6, 1.5e-3
    rng = np.random.default_rng(8)
    H = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    df = LAM * z / (n * dp)
    view = dict(center_x=0.0, center_y=0.0, pitch_x=df, pitch_y=df, nx=n, ny=n)
    flags = O.CONVERGING | O.NO_STRETCH | O.NO_REMAP
    plan = _check(H, dp, z, "c128", view=view, flags=flags, pad=0.0)
    assert (plan.info["mx"], plan.info["kcx"]) == (n, 0)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_pad_and_forced_size_parity(prec):
    say(f"pad/forced {prec}")
    n = 256
    dp = dp_(120.0)
    dp, pc, H = _hologram(61, 5, n, n, 120.0, 4 * n * dp, 6 * n * dp)
    z = float(pc.z[0])
    _check(H, dp, z, prec, pad=0.5 * 0.5 * n * dp)
    _check(H, dp, z, prec, frt_size=(450, 384))


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("fov", [60.0, 120.0])
def test_oversampled_parity(prec, fov):
    """Spectrum of the hologram zero-padded to 2N (oversample = 2): full view, a partial view, a
    rectangular hologram, and the four-step passes of the 2N-point hologram transform."""
    say(f"oversampled {prec} {fov}")
    n = 256
    dp = dp_(fov)
    dp, pc, H = _hologram(int(fov) + 71, 5, n, n, fov, 4 * n * dp, 7 * n * dp)
    z = float(np.median(pc.z))
    plan = _check(H, dp, z, prec, oversample=2)
    assert plan.info["oversample"] == 2
    assert plan.debug_copy(1).shape == (2 * n, 2 * n)
    B = plan.info["image_size"]
    view = dict(center_x=0.2 * B, center_y=-0.15 * B, pitch_x=0.0, pitch_y=0.0, nx=72, ny=48)
    _check(H, dp, z, prec, view=view, oversample=2)
    _check(H, dp, z, prec, oversample=2, tile_cap=1024)
    dp2, pc2, H2 = _hologram(int(fov) + 72, 4, 320, 192, fov, 4 * 320 * dp, 6 * 320 * dp)
    _check(H2, dp2, float(np.median(pc2.z)), prec, oversample=2)


@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
def test_paper_map_model_table_parity(fov):
    """The map table under the paper's polynomial model (Newton from the exact pre-image) against the
    oracle's: the same mask, pre-images to 1e-9 samples."""
    say(f"paper map table {fov}")
    n = 256
    dp = dp_(fov)
    z = 6 * n * dp
    plan = N.Plan(LAM, dp, n, n, z, precision="c128", map_model="paper")
    assert plan.info["map_model"] == 1
    tab = plan.debug_copy(3).cpu().numpy().reshape(-1, 2)
    nxt = int(round(math.sqrt(tab.shape[0])))
    assert nxt * nxt == tab.shape[0]
    k = np.arange(nxt, dtype=np.float64)
    KX, KY = np.meshgrid(k, k)
    c = O.paper_polynomial(LAM / (2 * dp))
    u, v, valid = O.inverse_stretch_paper(KX * LAM / (n * dp), KY * LAM / (n * dp), c)
    s = LAM / (2 * dp)
    valid = valid & (np.abs(u) <= s) & (np.abs(v) <= s)
    gx = tab[:, 0].reshape(nxt, nxt)
    gy = tab[:, 1].reshape(nxt, nxt)
    assert np.array_equal(~np.isnan(gx), valid)
    assert np.max(np.abs(gx[valid] - u[valid] * (n * dp / LAM))) <= 1e-9
    assert np.max(np.abs(gy[valid] - v[valid] * (n * dp / LAM))) <= 1e-9
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("fov", [60.0, 120.0])
def test_paper_map_model_parity(prec, fov):
    """Reconstruction with the paper's polynomial model of Eq. 16 (steps 1 and 4), full and partial."""
    say(f"paper map model {prec} {fov}")
    n = 256
    dp = dp_(fov)
    dp, pc, H = _hologram(int(fov) + 91, 5, n, n, fov, 4 * n * dp, 7 * n * dp)
    z = float(np.median(pc.z))
    _check(H, dp, z, prec, map_model="paper")
    B = O.image_size(LAM, dp, z)
    view = dict(center_x=-0.25 * B, center_y=0.2 * B, pitch_x=0.0, pitch_y=0.0, nx=64, ny=80)
    _check(H, dp, z, prec, view=view, map_model="paper")


@pytest.mark.parametrize("flags", [N.FLAG_NO_STRETCH, N.FLAG_NO_REMAP, N.FLAG_CONVERGING,
                                   N.FLAG_NO_STRETCH | N.FLAG_NO_REMAP])
def test_oversampled_flag_parity(flags):
    say(f"oversampled flags {flags}")
    n = 192
    dp = dp_(90.0)
    dp, pc, H = _hologram(81, 4, n, n, 90.0, 4 * n * dp, 6 * n * dp)
    _check(H, dp, float(np.median(pc.z)), "c128", flags=flags, oversample=2)


def test_oversampled_plan_refuses_a_cached_spectrum():
    say("oversampled vs spectrum")
    n = 128
    dp = dp_(60.0)
    dp, pc, H = _hologram(82, 2, n, n, 60.0, 4 * n * dp, 6 * n * dp)
    Ht = torch.from_numpy(H.astype(np.complex64)).cuda()
    plan = N.Plan(LAM, dp, n, n, float(pc.z[0]), precision="c64", oversample=2)
    spec = N.Spectrum(Ht, LAM, dp)
    out = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    with pytest.raises(N.NufdsError) as e:
        plan.execute_spectrum(spec, out)
    assert e.value.status == N.ERR_INVALID_ARG
    spec.close()
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_four_step_passes_parity(prec):
    """Tile capacity 1024 elements: hologram columns, FrT rows and columns all take the four-step path."""
    say(f"four-step {prec}")
    n = 512
    dp = dp_(90.0)
    dp, pc, H = _hologram(91, 5, n, n, 90.0, 3 * n * dp, 5 * n * dp)
    z = float(pc.z[0])
    plan = _check(H, dp, z, prec, tile_cap=1024)
    assert plan.info["mx"] > 1024 // 16
    # rows longer than the tile as well (M > 1024)
    _check(H, dp, z, prec, frt_size=(1152, 720), tile_cap=1024)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_row_chain_pass_parity(prec):
    """FrT rows of 6400 under a 4096-element tile: complex64 runs the x chain (IDFT, chirp, DFT) in one
    pass with the row in registers and its real and imaginary parts exchanged through LDS in turn
    (the kernel of the 25600-long rows of the 16384^2 workload, with the same radices 32 and 25 and
    both forms of exchange); complex128 takes the four-step passes.  Full view and an off-centre
    partial view."""
    say(f"row chain {prec}")
    n = 512
    dp = dp_(120.0)
    dp, pc, H = _hologram(93, 5, n, n, 120.0, 3 * n * dp, 5 * n * dp)
    z = float(pc.z[0])
    plan = _check(H, dp, z, prec, frt_size=(6400, 720), tile_cap=4096)
    Ht = torch.from_numpy(H.astype(np.complex64 if prec == "c64" else np.complex128)).to("cuda")
    plan.set_timing(1)
    plan(Ht)
    torch.cuda.synchronize()
    names = [t[0] for t in plan.timings()]
    if prec == "c64":
        assert "xop" in names and "xop_a" not in names
    else:
        assert "xop_a" in names and "xop" not in names
    B = O.image_size(LAM, dp, z)
    view = dict(center_x=0.21 * B, center_y=-0.13 * B, pitch_x=0.0, pitch_y=0.0, nx=200, ny=120)
    _check(H, dp, z, prec, view=view, frt_size=(6400, 720), tile_cap=4096)
    # FrT rows of 32768 (the radix 32 32 32 plan, past the default tile) on a 512 x 16 hologram
    dp2, pc2, H2 = _hologram(97, 3, 512, 16, 120.0, 3 * 512 * dp, 5 * 512 * dp)
    z2 = float(pc2.z[0])
    my2 = N.plan_geometry(LAM, dp2, 512, 16, z2)["my"]
    _check(H2, dp2, z2, prec, frt_size=(32768, my2))


@pytest.mark.parametrize("flags", [N.FLAG_NO_STRETCH, N.FLAG_NO_REMAP, N.FLAG_CONVERGING,
                                   N.FLAG_NO_STRETCH | N.FLAG_NO_REMAP])
def test_row_chain_pass_flag_parity(flags):
    """The one-pass x chain (complex64, FrT rows of 6400 under a 4096-element tile) under each flag."""
    say(f"row chain flags {flags}")
    n = 384
    dp = dp_(120.0)
    dp, pc, H = _hologram(94, 4, n, n, 120.0, 3 * n * dp, 5 * n * dp)
    _check(H, dp, float(pc.z[0]), "c64", flags=flags, frt_size=(6400, 864), tile_cap=4096)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_row_transform_pass_spectrum_parity(prec):
    """Hologram rows of 6400 under a 4096-element tile, and the 32768-point rows of a 16384-wide
    hologram's oversampled spectrum: complex64 runs each row's DFT in one pass (the single-transform
    form of the one-pass row kernel, whose loads conjugate, centre by (-1)^n and, for the oversampled
    spectrum, read a window of the zero-padded row); complex128 takes the four-step passes.  The
    spectrum against the oracle's centred DFT of the (padded) hologram."""
    say(f"row transform {prec}")
    tol = 1e-13 if prec == "c128" else 1e-6
    # the 32768-point rows exceed the default tile (its FrT rows of 25000 need it for their split);
    # a converging hologram is transformed without conjugation
    cases = ((6400, 40, None, 4096, 0), (6400, 40, None, 4096, N.FLAG_CONVERGING), (3200, 40, 2, 4096, 0),
             (16384, 8, 2, None, 0))
    for nx, ny, over, cap, flags in cases:
        dp, pc, H = _hologram(95 + nx // 1000, 3, nx, ny, 90.0, 2 * nx * dp_(90.0), 3 * nx * dp_(90.0))
        _, plan = _gpu_run(H, dp, float(pc.z[0]), prec, tile_cap=cap, oversample=over, flags=flags)
        got = plan.debug_copy(1).cpu().numpy().astype(np.complex128)
        src = _oracle_input(H, prec) if flags & N.FLAG_CONVERGING else np.conj(_oracle_input(H, prec))
        if over:
            padded = np.zeros((over * ny, over * nx), dtype=np.complex128)
            oy, ox = (over * ny - ny) // 2, (over * nx - nx) // 2
            padded[oy:oy + ny, ox:ox + nx] = src
            src = padded
        ref = O.centred_dft2(src)
        err = O.rel_l2(got, ref)
        say(f"   {nx} x {ny} oversample {over} flags {flags}: rel_l2 = {err:.3e}")
        assert got.shape == ref.shape and err <= tol
        plan.close()


def test_execute_is_deterministic_and_repeatable():
    say("determinism")
    n = 256
    dp = dp_(120.0)
    dp, pc, H = _hologram(3, 4, n, n, 120.0, 4 * n * dp, 6 * n * dp)
    z = float(pc.z[0])
    plan = N.Plan(LAM, dp, n, n, z, precision="c64")
    Ht = torch.from_numpy(H.astype(np.complex64)).cuda()
    a = plan(Ht)
    b = plan(Ht)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c = plan(Ht, stream=s)
    s.synchronize()
    assert torch.equal(a, c)


def test_invalid_execute_arguments():
    say("invalid execute")
    n = 64
    plan = N.Plan(LAM, 0.5e-6, n, n, 1e-3, precision="c64")
    Ht = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        plan.execute(Ht, torch.zeros((n, n + 2), dtype=torch.complex64, device="cuda"))
    with pytest.raises(N.NufdsError):
        N.Plan(LAM, 0.5e-6, 2 * 7 * 11, 64, 1e-3)   # 154 is not 5-smooth


# ------------------------------------------------------------- the 1024^2 60 deg workload

@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_c1_full_view_parity(prec):
    """1024^2 hologram, 64 points, lambda = pitch = 0.5 um (60 deg), z = 3 mm, full 1024^2 view."""
    say(f"C1 {prec}")
    n = 1024
    dp = 0.5e-6
    pc = synth.draw_points(synth.CONFIG_SEEDS["c1"], 64, n, n, dp, LAM, 2e-3, 4e-3)
    H = synth.point_hologram(pc, n, n, dp, LAM)
    plan = _check(H, dp, 3e-3, prec)
    assert plan.info["mx"] == 1280
