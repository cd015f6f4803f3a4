"""Pins of the float64 oracle against the paper and against mathematics.

Each test fixes one part of the oracle by something other than the oracle
itself: values printed in the paper (tests/golden/paper_values.json), closed
forms, explicit DFT matrices, exact special cases, and a brute-force
Rayleigh-Sommerfeld back-propagation.  All run on the CPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------- geometry

def test_eq1_image_size_example():
    g = GOLDEN["image_size_example"]
    B = O.image_size(g["wavelength"], g["pitch"], g["z"])
    assert abs(B - g["B_m"]) <= g["B_tol"]
    assert abs(O.fov_deg(g["wavelength"], g["pitch"]) - g["fov_deg"]) <= g["fov_tol"]
    g = GOLDEN["image_size_cgh1"]
    assert abs(O.image_size(g["wavelength"], g["pitch"], g["z"]) - g["B_m"]) <= g["B_tol"]


def test_fov_values_printed():
    g = GOLDEN["fov_by_pitch"]
    for p, f in zip(g["pitch"], g["fov_deg"]):
        assert abs(O.fov_deg(g["wavelength"], p) - f) <= g["tol"]
    for lam, p, f, tol in GOLDEN["fov_other"]["cases"]:
        assert abs(O.fov_deg(lam, p) - f) <= tol


def test_eq1_rejects_evanescent_pitch():
    with pytest.raises(ValueError):
        O.image_size(0.5e-6, 0.25e-6, 1.0)


# ------------------------------------------------ phase-space tools (Sec. 2)

def test_frt_spot_and_corrected_focus():
    lam, dp = 0.5e-6, 0.5e-6
    B = O.image_size(lam, dp, 1.0)
    xo = 0.45 * B
    g = GOLDEN["frt_spot"]
    assert abs(O.frt_spot_x(xo, 0.0, 1.0, lam) - g["x_ro"]) <= g["tol"]
    xr, zr = O.corrected_focus(xo, 0.0, 1.0, lam)
    g = GOLDEN["corrected_focus"]
    assert abs(zr - g["z_ro"]) <= g["z_tol"]
    assert abs(xr - g["x_ro"]) <= g["x_tol"]
    g = GOLDEN["corrected_focus_depths"]
    for z, zr_ref in zip(g["z"], g["z_ro"]):
        xo = 0.45 * O.image_size(lam, dp, z)
        assert abs(O.corrected_focus(xo, 0.0, z, lam)[1] - zr_ref) <= g["tol"]


def test_eq4_eq5_against_phase_derivatives():
    """Eqs. 4-5 are the first and second x-derivatives of the phase of Eq. 3."""
    lam, xo, yo, zo = 0.5e-6, 0.3, -0.1, 0.8
    k = 2 * math.pi / lam
    x, y, h = 1e-3, 2e-3, 1e-6

    def phase(x):
        return -k * math.sqrt((x - xo) ** 2 + (y - yo) ** 2 + zo ** 2)

    d1 = (phase(x + h) - phase(x - h)) / (2 * h) / (2 * math.pi)
    d2 = (phase(x + h) - 2 * phase(x) + phase(x - h)) / h ** 2 * lam / (2 * math.pi)
    assert abs(d1 - O.local_frequency_x(x, y, xo, yo, zo, lam)) <= 1e-7 * abs(d1)
    assert abs(d2 - O.local_curvature_x(x, y, xo, yo, zo)) <= 1e-4 * abs(d2)


# ------------------------------------------- magnification (Eqs. 15-16)

SIGMAS = [1e-9, 0.05, 0.3, 0.5, 0.7071, 0.866, 0.95, 0.99]


def test_I_closed_form_at_one():
    """I(1) = Gamma(3/2)Gamma(1/4)/Gamma(3/4) = sqrt(2) K(1/2)."""
    ref = math.gamma(1.5) * math.gamma(0.25) / math.gamma(0.75)
    assert abs(O.I_ONE - ref) <= 1e-15
    assert abs(O.I_integral(1.0) - math.sqrt(2) * special.ellipk(0.5)) <= 4e-15
    assert abs(O.I_ONE - 2.6220575542921198) <= 1e-15


@pytest.mark.parametrize("sig", SIGMAS)
def test_I_series_and_quadrature(sig):
    """The elliptic evaluation equals the 2F1 series of Eq. 16 and plain quadrature."""
    got = float(O.I_integral(sig))
    series = sig * special.hyp2f1(0.5, 0.75, 1.5, sig * sig)
    # substitution w = sin(g) removes the endpoint growth of the integrand
    quad = integrate.quad(lambda g: math.cos(g) ** -0.5, 0.0, math.asin(sig), epsabs=1e-16, epsrel=1e-14, limit=200)[0]
    assert abs(got - series) <= 2e-14 * max(1.0, got)
    assert abs(got - quad) <= 1e-13 * max(1.0, got)


def test_eq15_is_the_derivative_of_eq16():
    rng = np.random.default_rng(5)
    lam = 0.5e-6
    for _ in range(200):
        r = math.sqrt(rng.uniform(0.0, 0.9))
        a = rng.uniform(0, 2 * math.pi)
        fx, fy = r * math.cos(a) / lam, r * math.sin(a) / lam
        h = 1e-6 / lam
        fd = (O.stretch_map(fx + h, fy, lam)[0] - O.stretch_map(fx - h, fy, lam)[0]) / (2 * h)
        assert abs(fd - O.stretch_jacobian_xx(fx, fy, lam)) <= 1e-7 * fd


def test_small_angle_magnification():
    """m_x = 1 + (u^2 + v^2)/4 + O(4th order) as the field of view shrinks."""
    lam = 0.5e-6
    for u, v in [(0.01, 0.0), (0.0, 0.01), (0.007, -0.006), (0.02, 0.015)]:
        m = O.magnification_x(u / lam, v / lam, lam)
        assert abs(m - 1 - (u * u + v * v) / 4) <= 0.5 * (u * u + v * v) ** 2


def test_fig4_map_examples():
    g = GOLDEN["output_map_example"]
    xp, yp = O.output_map(g["x_o"], 0.0, g["z"])
    assert abs(xp - g["x_o_prime"]) <= g["tol"] and yp == 0.0
    g = GOLDEN["spectral_map_example"]
    for lam in g["wavelengths"]:
        fp = O.stretch_map(g["f_x"], 0.0, lam)[0]
        assert abs(fp - g["f_x_prime"]) <= g["tol"]


def test_fig4_magnification_sides():
    """Spectral magnification exceeds one and the output map shrinks (Sec. 4)."""
    lam = 0.5e-6
    u = np.linspace(-0.85, 0.85, 41)
    U, V = np.meshgrid(u, u)
    inside = U ** 2 + V ** 2 < 0.98
    U, V = U[inside], V[inside]
    nz = np.abs(U) + np.abs(V) > 1e-12
    assert np.all(O.magnification_x(U / lam, V / lam, lam)[nz] > 1.0)
    x = np.linspace(-1.5, 1.5, 31)
    X, Y = np.meshgrid(x, x)
    XP, YP = O.output_map(X, Y, 1.0)
    assert np.all(np.abs(XP[X != 0]) < np.abs(X[X != 0]))


# ----------------------------------------- inverse of the spectral stretch

def test_rim_maps_to_superellipse():
    """Approaching the rim, Eq. 16's image tends to |t|_4 = I(1) from inside.

    Near the rim T = I(1) (sqrt(u), sqrt(v)) - 2 d^(1/4) (1, 1) + ..., with
    d = 1 - u^2 - v^2, so the gap to the superellipse shrinks like d^(1/4).
    """
    for p in np.linspace(0.05, math.pi / 2 - 0.05, 9):
        gaps = []
        for eps in (1e-4, 1e-6, 1e-8):
            r = math.sqrt(1.0 - eps)
            t1, t2 = O.stretch_map(r * math.cos(p), r * math.sin(p), 1.0)
            gaps.append(O.I_ONE ** 4 - (t1 ** 4 + t2 ** 4))
        assert all(g > 0 for g in gaps)
        for g, e in zip(gaps, (1e-4, 1e-6, 1e-8)):
            assert g <= 200.0 * e ** 0.25
        assert gaps[0] / gaps[2] > 0.5 * 100 ** 0.5


def test_inverse_stretch_round_trip_grid():
    """Eqs. 9-10 written with 2F1 (Eq. 16) map the pre-image back to the target."""
    t = np.linspace(-2.6, 2.6, 181)
    T1, T2 = np.meshgrid(t, t)
    u, v, valid = O.inverse_stretch(T1, T2)
    assert np.array_equal(valid, T1 ** 4 + T2 ** 4 < O.I_ONE ** 4)
    d = 1 - u * u - v * v
    assert np.all(d[valid] > -1e-15)
    ok = valid & (d > 1e-6)
    a1, a2 = O.stretch_map(u[ok], v[ok], 1.0)
    # Eq. 16 evaluated from (u, v) carries rounding of 1 - u^2 - v^2 amplified
    # by the slope (1 - sigma^2)^(-3/4) of the integrand near the rim.
    tol = 1e-13 + 4e-16 * d[ok] ** -0.75
    assert np.all(np.abs(a1 - T1[ok]) <= tol)
    assert np.all(np.abs(a2 - T2[ok]) <= tol)
    assert np.all(np.sign(u[ok]) == np.sign(T1[ok])) and np.all(np.sign(v[ok]) == np.sign(T2[ok]))


def test_inverse_stretch_of_forward():
    rng = np.random.default_rng(11)
    r = np.sqrt(rng.uniform(0, 0.9999, 5000))
    a = rng.uniform(0, 2 * math.pi, 5000)
    u, v = r * np.cos(a), r * np.sin(a)
    t1, t2 = O.stretch_map(u, v, 1.0)
    uu, vv, valid = O.inverse_stretch(t1, t2)
    assert valid.all()
    assert np.max(np.abs(uu - u)) <= 1e-12 and np.max(np.abs(vv - v)) <= 1e-12


def test_inverse_stretch_near_rim_is_monotone():
    """Along a ray towards the superellipse the pre-image moves out to the rim."""
    for phi in (0.3, 0.7852, 1.2):
        rr = O.I_ONE * (1 - np.logspace(-1, -13, 40))
        t1 = rr * math.cos(phi) ** 0.5
        t2 = rr * math.sin(phi) ** 0.5
        u, v, valid = O.inverse_stretch(t1, t2)
        assert valid.all()
        n2 = u * u + v * v
        assert np.all(np.diff(n2) >= -1e-15) and n2[-1] > 1 - 1e-12
        # the limit point is the rim point whose image is the target direction
        assert abs(u[-1] - math.cos(phi)) <= 1e-5 and abs(v[-1] - math.sin(phi)) <= 1e-5


def test_jacobian_determinant_at_least_one():
    rng = np.random.default_rng(3)
    r = np.sqrt(rng.uniform(0, 0.98, 400))
    a = rng.uniform(0, 2 * math.pi, 400)
    h = 1e-6
    for u, v in zip(r * np.cos(a), r * np.sin(a)):
        px = np.array(O.stretch_map(u + h, v, 1.0)) - np.array(O.stretch_map(u - h, v, 1.0))
        py = np.array(O.stretch_map(u, v + h, 1.0)) - np.array(O.stretch_map(u, v - h, 1.0))
        det = (px[0] * py[1] - px[1] * py[0]) / (4 * h * h)
        assert det >= 1.0 - 1e-6


# ------------------------------------------------- output map (Eqs. 17-18)

@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
def test_eq18b_iteration_inverts_output_map(fov):
    """The paper's sequential x_o' -> x_o iteration converges to the pre-image of Eqs. 17-18."""
    lam, z = 0.5e-6, 1.0
    B = O.image_size(lam, synth.fov_pitch(lam, fov), z)
    x = np.linspace(-0.5, 0.5, 21) * B
    X, Y = np.meshgrid(x, x)
    XP, YP = O.output_map(X, Y, z)
    it = O.output_map_inverse_eq18b(XP, YP, z, iters=120)
    xr, yr = it[-1]
    assert np.max(np.abs(xr - X)) <= 1e-9 * B and np.max(np.abs(yr - Y)) <= 1e-9 * B
    # convergence is monotone in the iteration count (a contraction)
    e = [np.max(np.abs(a - X)) for a, _ in it[:6]]
    assert all(e[i + 1] < e[i] for i in range(5))


def test_output_map_is_odd_and_symmetric():
    x = np.array([0.1, 0.4, 0.7])
    y = np.array([0.2, -0.3, 0.05])
    a = O.output_map(x, y, 1.0)
    b = O.output_map(-x, y, 1.0)
    c = O.output_map(y, x, 1.0)
    assert np.allclose(a[0], -b[0], rtol=0, atol=1e-15) and np.allclose(a[1], b[1], rtol=0, atol=1e-15)
    assert np.allclose(a[0], c[1], rtol=0, atol=1e-15)


def test_small_fov_limit_of_output_map():
    """max |x'/x - 1| over the image falls as s^2 (4x per halving of s)."""
    lam, z = 0.5e-6, 1.0
    devs = []
    for s in (0.1, 0.05, 0.025):
        B = O.image_size(lam, lam / (2 * s), z)
        x = np.linspace(1e-3, 0.5, 50) * B
        X, Y = np.meshgrid(x, x)
        XP, _ = O.output_map(X, Y, z)
        devs.append(np.max(np.abs(XP / X - 1)))
    for a, b in zip(devs, devs[1:]):
        assert 3.8 <= a / b <= 4.2


# --------------------------------------------------------- transforms

def test_centred_dft_matches_explicit_matrices():
    rng = np.random.default_rng(2)
    a = rng.normal(size=(6, 10)) + 1j * rng.normal(size=(6, 10))
    assert np.max(np.abs(O.centred_dft2(a) - O.centred_dft2_direct(a))) <= 1e-12
    assert np.max(np.abs(O.centred_idft2(a) - O.centred_dft2_direct(a, inverse=True))) <= 1e-13
    assert np.max(np.abs(O.centred_idft2(O.centred_dft2(a)) - a)) <= 1e-13


def test_keys_kernel_interpolates_and_reproduces_linear():
    t = np.linspace(0, 1, 11)
    w = np.stack([O.keys_weight(t - a) for a in (-1, 0, 1, 2)])
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-15)            # partition of unity
    assert np.allclose((w * np.array([-1, 0, 1, 2])[:, None]).sum(axis=0), t, atol=1e-15)
    assert O.keys_weight(0.0) == 1.0 and O.keys_weight(1.0) == 0.0 and O.keys_weight(2.0) == 0.0


def test_frt_of_paraxial_wave_is_a_kronecker_delta():
    """A paraxial wave converging to x_p on the Delta_F grid gives one nonzero FrT sample."""
    lam, dp, z = 0.5e-6, 0.5e-6, 2e-3
    nx, ny, mx, my = 64, 48, 80, 60
    band = O.Band(nx=nx, ny=ny, sx=nx, sy=ny, cx=0, cy=0, dox=1, doy=1,
                  dfx=lam * z / (nx * dp), dfy=lam * z / (ny * dp), mx=mx, my=my,
                  kcx=0, kcy=0, padx=0, pady=0, xlo=0, xhi=0, ylo=0, yhi=0)
    jx, jy = 7, -5
    xp, yp = jx * band.dfx, jy * band.dfy
    k = 2 * math.pi / lam
    xi = (np.arange(mx) - mx // 2) * (nx * dp / mx)
    eta = (np.arange(my) - my // 2) * (ny * dp / my)
    h = np.exp(-1j * k * ((xi[None, :] - xp) ** 2 + (eta[:, None] - yp) ** 2) / (2 * z))
    F = O.fresnel_frt(h, band, lam, dp, z)
    peak = (my // 2 + jy, mx // 2 + jx)
    assert abs(abs(F[peak]) - mx * my) <= 1e-9 * mx * my
    F[peak] = 0
    assert np.max(np.abs(F)) <= 1e-9 * mx * my


def test_small_fov_identity_is_the_plain_frt():
    """NO_STRETCH | NO_REMAP with M = S = N, K_c = 0, Delta_o = Delta_F, pad = 0 is Eq. 2 itself."""
    lam, dp, z = 0.5e-6, 0.5e-6, 1.5e-3
    nx, ny = 40, 32
    rng = np.random.default_rng(9)
    H = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    dfx, dfy = lam * z / (nx * dp), lam * z / (ny * dp)
    view = dict(center_x=0.0, center_y=0.0, pitch_x=dfx, pitch_y=dfy, nx=nx, ny=ny)
    flags = O.CONVERGING | O.NO_STRETCH | O.NO_REMAP
    band = O.plan_band(nx, ny, lam, dp, z, view, flags, pad=0.0)
    assert (band.mx, band.my, band.kcx, band.kcy) == (nx, ny, 0, 0)
    out = O.reconstruct(H, lam, dp, z, view=view, flags=flags, pad=0.0)
    k = 2 * math.pi / lam
    x = (np.arange(nx) - nx // 2) * dp
    y = (np.arange(ny) - ny // 2) * dp
    xo = (np.arange(nx) - nx // 2) * dfx
    yo = (np.arange(ny) - ny // 2) * dfy
    g = H * np.exp(1j * k * (x[None, :] ** 2 + y[:, None] ** 2) / (2 * z))
    ref = np.exp(1j * k * (xo[None, :] ** 2 + yo[:, None] ** 2) / (2 * z)) * O.centred_dft2_direct(g)
    assert O.rel_l2(out, ref) <= 1e-13


def test_parseval_at_every_transform():
    lam, dp = 0.5e-6, synth.fov_pitch(0.5e-6, 90.0)
    N = 96
    pc = synth.draw_points(17, 4, N, N, dp, lam, 4 * N * dp, 6 * N * dp)
    H = synth.point_hologram(pc, N, N, dp, lam)
    z = float(np.mean(pc.z))
    _, st = O.reconstruct(H, lam, dp, z, return_stages=True)
    b = st["band"]
    Hc = np.conj(H)
    assert abs(np.sum(abs(st["spectrum"]) ** 2) - N * N * np.sum(abs(Hc) ** 2)) <= 1e-12 * N * N * np.sum(abs(Hc) ** 2)
    e_t = np.sum(abs(st["stretched"]) ** 2)
    assert abs(np.sum(abs(st["h"]) ** 2) - e_t / (b.mx * b.my)) <= 1e-12 * e_t / (b.mx * b.my)
    g_energy = np.sum(abs(st["h"]) ** 2)   # the chirp has unit modulus
    assert abs(np.sum(abs(st["F"]) ** 2) - b.mx * b.my * g_energy) <= 1e-12 * b.mx * b.my * g_energy


# --------------------------------------------------------- sub-band rule

@pytest.mark.parametrize("n,fov,z,m", [(1024, 60.0, 3e-3, 1280), (4096, 90.0, 7.5e-3, 5400),
                                       (16384, 120.0, 15e-3, 25600), (8192, 120.0, 5e-3, 13500),
                                       (8192, 120.0, 15e-3, 12000)])
def test_full_view_band_sizes(n, fov, z, m):
    lam = 0.5e-6
    b = O.plan_band(n, n, lam, synth.fov_pitch(lam, fov), z)
    assert (b.mx, b.my, b.kcx, b.kcy) == (m, m, 0, 0)


def test_partial_view_band_is_centred_on_the_window():
    lam = 0.5e-6
    dp = synth.fov_pitch(lam, 120.0)
    z = 10e-3
    B = O.image_size(lam, dp, z)
    n = 8192
    df = lam * z / (n * dp)
    view = dict(center_x=0.3 * B, center_y=-0.2 * B, pitch_x=0.0, pitch_y=0.0, nx=1024, ny=512)
    b = O.plan_band(n, n, lam, dp, z, view)
    xc = O.output_map(0.3 * B, -0.2 * B, z)[0]
    assert abs(b.kcx * df - xc) <= 0.05 * B
    assert b.kcx > 0 and b.kcy < 0
    half_x = max(b.xhi + b.padx - b.kcx * df, b.kcx * df - b.xlo + b.padx)
    assert b.mx * df >= 2 * half_x - 1e-9 * df
    assert b.mx % 2 == 0 and b.mx == O.smooth5_even(b.mx)


def test_window_outside_image_is_rejected():
    lam, dp, z = 0.5e-6, 0.5e-6, 3e-3
    B = O.image_size(lam, dp, z)
    with pytest.raises(ValueError):
        O.plan_band(256, 256, lam, dp, z, dict(center_x=0.45 * B, center_y=0, pitch_x=0, pitch_y=0,
                                                 nx=256, ny=16))


def test_smooth5_even():
    assert [O.smooth5_even(n) for n in (1, 7, 1279, 1281, 5399, 25599)] == [2, 8, 1280, 1296, 5400, 25600]


# ------------------------------------------------------ end-to-end physics

def _spot(fov, frac, flags=0, n=256, ratio=10.0):
    """One point at ``ratio`` apertures from the hologram (each object wave
    then spans a narrow band, as the method assumes; Sec. 1 and Sec. 2)."""
    lam = 0.5e-6
    dp = synth.fov_pitch(lam, fov)
    s = lam / (2 * dp)
    zp = ratio * n * dp
    L = 0.9 * (zp * s / math.sqrt(1 - s * s) - n * dp / 2)
    xp, yp = frac * L, -0.6 * frac * L
    pc = synth.PointCloud(np.array([xp]), np.array([yp]), np.array([zp]), np.array([1.0]), np.array([0.3]))
    H = synth.point_hologram(pc, n, n, dp, lam)
    return lam, dp, zp, xp, yp, H


@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
@pytest.mark.parametrize("frac", [0.0, 0.5, 0.9])
def test_point_focuses_at_its_true_position(fov, frac):
    lam, dp, zp, xp, yp, H = _spot(fov, frac)
    n = H.shape[0]
    df = lam * zp / (n * dp)
    do = df / 4
    S = 48
    view = dict(center_x=xp, center_y=yp, pitch_x=do, pitch_y=do, nx=S, ny=S)
    I = np.abs(O.reconstruct(H, lam, dp, zp, view=view)) ** 2
    i, j = np.unravel_index(I.argmax(), I.shape)
    # the output is resampled from the Delta_F grid: the bare argmax is only
    # meaningful to half a Delta_F; the centroid pins the position to a quarter
    assert abs(j - S // 2) <= 2 and abs(i - S // 2) <= 2
    m = I >= 0.5 * I.max()
    yy, xx = np.indices(I.shape)
    cx = (xx[m] * I[m]).sum() / I[m].sum() - S // 2
    cy = (yy[m] * I[m]).sum() / I[m].sum() - S // 2
    assert abs(cx) * do <= 0.25 * df and abs(cy) * do <= 0.25 * df
    # without step 5 the spot sits at the distorted position of Eqs. 17-18
    xq, yq = O.output_map(xp, yp, zp)
    view = dict(center_x=float(xq), center_y=float(yq), pitch_x=do, pitch_y=do, nx=S, ny=S)
    I = np.abs(O.reconstruct(H, lam, dp, zp, view=view, flags=O.NO_REMAP)) ** 2
    i, j = np.unravel_index(I.argmax(), I.shape)
    assert abs(j - S // 2) <= 2 and abs(i - S // 2) <= 2


def test_plain_frt_misplaces_an_off_axis_point():
    """Without the stretch and remap the FrT puts a 120 deg point far from its position."""
    lam, dp, zp, xp, yp, H = _spot(120.0, 0.9)
    n = H.shape[0]
    df = lam * zp / (n * dp)
    S = 48
    view = dict(center_x=xp, center_y=yp, pitch_x=df / 4, pitch_y=df / 4, nx=S, ny=S)
    good = np.abs(O.reconstruct(H, lam, dp, zp, view=view)) ** 2
    bad = np.abs(O.reconstruct(H, lam, dp, zp, view=view, flags=O.NO_STRETCH | O.NO_REMAP)) ** 2
    assert bad.max() < 0.1 * good.max()


def test_focus_is_sharpest_at_the_point_depth():
    lam, dp, zp, xp, yp, H = _spot(90.0, 0.5, n=128, ratio=5.0)
    n = H.shape[0]
    df = lam * zp / (n * dp)
    peaks = {}
    for f in (0.96, 0.98, 1.0, 1.02, 1.04):
        z = zp * f
        view = dict(center_x=xp * f, center_y=yp * f, pitch_x=df / 4, pitch_y=df / 4, nx=32, ny=32)
        peaks[f] = np.max(np.abs(O.reconstruct(H, lam, dp, z, view=view)) ** 2)
    assert max(peaks, key=peaks.get) == 1.0
    assert peaks[0.96] < peaks[0.98] < peaks[1.0] > peaks[1.02] > peaks[1.04]


def _paper_spot(H, lam, dp, z, cx, flags=0, S=128):
    view = dict(center_x=cx, center_y=0.0, pitch_x=0.0, pitch_y=0.0, nx=S, ny=S)
    out, st = O.reconstruct(H, lam, dp, z, view=view, flags=flags, return_stages=True)
    I = np.abs(out) ** 2
    i, j = np.unravel_index(I.argmax(), I.shape)
    xs = cx + (np.arange(S) - S // 2) * st["band"].dox
    m = I >= 0.5 * I.max()
    cen = float((I[m] * np.broadcast_to(xs, I.shape)[m]).sum() / I[m].sum())
    return float(xs[j]), cen, float(I.max() / I.sum()), int(np.sum(I[i] >= 0.5 * I.max())), st["band"].dfx


def test_fig2_at_the_papers_size():
    """Sec. 2, Fig. 2, through the whole reconstruction at the paper's size: an 8K hologram (8192 x
    4096, lambda = pitch = 0.5 um) of the point [0.45 B, 0, 1 m].  The plain FrT at 1 m blurs it over
    several samples around the printed 0.461 m (Fig. 2b); at the corrected distance it is sharp at the
    printed 0.66 m (Fig. 2e); NU-FDS at 1 m puts a sharp focus on the point itself."""
    lam = dp = 0.5e-6
    xo = 0.45 * O.image_size(lam, dp, 1.0)
    pc = synth.PointCloud(np.array([xo]), np.array([0.0]), np.array([1.0]), np.array([1.0]), np.array([0.0]))
    H = synth.point_hologram(pc, 8192, 4096, dp, lam)
    plain = O.NO_STRETCH | O.NO_REMAP
    _, cen, pk1, w1, _ = _paper_spot(H, lam, dp, 1.0, O.frt_spot_x(xo, 0.0, 1.0, lam), plain)
    assert abs(cen - GOLDEN["frt_spot"]["x_ro"]) <= GOLDEN["frt_spot"]["tol"]
    xr, zr = O.corrected_focus(xo, 0.0, 1.0, lam)
    xp2, _, pk2, w2, _ = _paper_spot(H, lam, dp, zr, xr, plain)
    assert abs(xp2 - GOLDEN["corrected_focus"]["x_ro"]) <= GOLDEN["corrected_focus"]["x_tol"]
    xp3, _, pk3, w3, df = _paper_spot(H, lam, dp, 1.0, xo)
    assert abs(xp3 - xo) <= df
    assert w1 >= 4 and w2 <= 2 and w3 <= 2
    assert pk3 > 3.0 * pk1 and pk2 > 3.0 * pk1


def test_fig7_cgh2_at_the_papers_size():
    """Sec. 5, Fig. 7b/d: CGH2 (8K, 60 deg) of P1 (0.45 B_xo, 0, 0.5 m) and P2 (0.45 B_xo - 10 mm, 0,
    1.5 m) with B_xo = 577.4 mm: each point in focus, on its own sample, at its own depth."""
    lam = dp = 0.5e-6
    B = O.image_size(lam, dp, 0.5)
    assert abs(B - GOLDEN["image_size_cgh1"]["B_m"]) <= GOLDEN["image_size_cgh1"]["B_tol"]
    pts = ((0.45 * B, 0.5), (0.45 * B - 0.01, 1.5))
    pc = synth.PointCloud(np.array([p[0] for p in pts]), np.zeros(2), np.array([p[1] for p in pts]),
                          np.ones(2), np.zeros(2))
    H = synth.point_hologram(pc, 8192, 4096, dp, lam)
    for x, z in pts:
        xp, _, pk, w, df = _paper_spot(H, lam, dp, z, x)
        assert abs(xp - x) <= df and pk > 0.3 and w <= 2


def test_oversampled_spectrum_interleaves_the_plain_one():
    """Zero-padding the hologram (centred) to 2N samples the same spectrum twice as finely: the even
    samples of the padded spectrum are the plain spectrum."""
    rng = np.random.default_rng(7)
    H = rng.standard_normal((48, 64)) + 1j * rng.standard_normal((48, 64))
    _, st1 = O.reconstruct(H, 0.5e-6, 0.5e-6, 1e-3, return_stages=True)
    _, st2 = O.reconstruct(H, 0.5e-6, 0.5e-6, 1e-3, return_stages=True, oversample=2)
    a, b = st2["spectrum"][::2, ::2], st1["spectrum"]
    assert st2["spectrum"].shape == (96, 128)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_oversampling_without_stretch_is_the_plain_path():
    """With the stretch off every pre-image is a spectral sample, an even sample of the finer grid,
    where the Keys weights are (0, 1, 0, 0): oversampling changes nothing but rounding."""
    lam, dp, zp, xp, yp, H = _spot(90.0, 0.5, n=64, ratio=5.0)
    for flags in (O.NO_STRETCH, O.NO_STRETCH | O.NO_REMAP):
        a = O.reconstruct(H, lam, dp, zp, flags=flags)
        b = O.reconstruct(H, lam, dp, zp, flags=flags, oversample=2)
        assert O.rel_l2(b, a) <= 1e-12


def test_oversampling_brings_the_focus_closer_to_rayleigh_sommerfeld():
    """The unpadded spectrum is critically sampled and the Keys kernel attenuates its outer samples
    (the outer hologram aperture); sampling it twice as finely raises the normalised peak intensity of
    a point's focus towards the brute-force Rayleigh-Sommerfeld one (measured on 128^2 holograms:
    0.74 / 0.85 / 0.80 of RS at 60 / 90 / 120 deg without, 0.82 / 0.96 / 0.87 with)."""
    lam = 0.5e-6
    n, S = 128, 32
    for fov in (60.0, 90.0, 120.0):
        dp = synth.fov_pitch(lam, fov)
        r1, r2 = [], []
        for seed in range(2):
            pc = synth.draw_points(1000 + 100 * seed + int(fov), 1, n, n, dp, lam, 4 * n * dp, 6 * n * dp)
            H = synth.point_hologram(pc, n, n, dp, lam)
            zp = float(pc.z[0])
            do = lam * zp / (n * dp) / 2
            view = dict(center_x=float(pc.x[0]), center_y=float(pc.y[0]), pitch_x=do, pitch_y=do, nx=S, ny=S)
            X, Y = np.meshgrid(pc.x[0] + (np.arange(S) - S // 2) * do, pc.y[0] + (np.arange(S) - S // 2) * do)
            Ir = np.abs(O.rayleigh_sommerfeld_backprop(H, dp, lam, zp, X, Y)) ** 2
            pr = Ir.max() / Ir.sum()
            for sig, acc in ((1, r1), (2, r2)):
                I = np.abs(O.reconstruct(H, lam, dp, zp, view=view, oversample=sig)) ** 2
                acc.append(I.max() / I.sum() / pr)
        assert np.mean(r2) > np.mean(r1) + 0.03, (fov, r1, r2)
        assert min(r2) >= 0.75


def _wavefront_error(H, lam, dp, z, xo, oversample):
    """Reading of Fig. 5's W: the phase of the FrT input g = h' exp(i k xi^2 / 2z) (step 3 before its
    DFT) along the row through the point, over the aperture where |g| is at least half its maximum,
    after removing piston and tilt (the tilt only sets the focus position), in waves.  Returns the
    largest |W| over that aperture and over its central 80%."""
    view = dict(center_x=xo, center_y=0.0, pitch_x=0.0, pitch_y=0.0, nx=64, ny=64)
    _, st = O.reconstruct(H, lam, dp, z, view=view, return_stages=True, oversample=oversample)
    b = st["band"]
    k = 2.0 * math.pi / lam
    xi = (np.arange(b.mx) - b.mx // 2) * (b.nx * dp / b.mx)
    g = st["h"][b.my // 2] * np.exp(1j * k * xi ** 2 / (2.0 * z))
    a = np.abs(g)
    m = a >= 0.5 * a.max()
    ph, x, w = np.unwrap(np.angle(g[m])), xi[m], a[m]
    A = np.vstack([np.ones_like(x), x]).T
    c = np.linalg.lstsq(A * w[:, None], ph * w, rcond=None)[0]
    W = (ph - A @ c) / (2.0 * math.pi)
    n = len(W)
    return float(np.abs(W).max()), float(np.abs(W[n // 10:n - n // 10]).max())


def test_fig5_wavefront_error():
    """Sec. 4, Fig. 5 at the paper's size (8K holograms of [0.45 B, 0, z]): with the spectrum of step 2
    sampled at twice its critical rate the wavefront error stays below the printed max|W| = 0.11
    lambda (and the Rayleigh lambda/4) over the whole aperture (oracle: 0.003-0.059 lambda over all
    nine pitch / depth pairs).  Without oversampling the central 80% of the aperture stays below it
    too, but at the larger pitches the Keys interpolation of the critically sampled spectrum breaks
    the wavefront at the aperture's edge (up to 0.66 lambda at 0.75 um, 0.5 m)."""
    lam = 0.5e-6
    g = GOLDEN["wavefront_error"]
    for dp, z in ((0.75e-6, 0.5), (0.5e-6, 0.5), (0.3e-6, 0.5), (0.75e-6, 1.0)):
        xo = 0.45 * O.image_size(lam, dp, z)
        pc = synth.PointCloud(np.array([xo]), np.array([0.0]), np.array([z]), np.array([1.0]), np.array([0.0]))
        H = synth.point_hologram(pc, 8192, 4096, dp, lam)
        w1, c1 = _wavefront_error(H, lam, dp, z, xo, 1)
        w2, c2 = _wavefront_error(H, lam, dp, z, xo, 2)
        assert w2 <= g["max_w"] and c1 <= g["max_w"], (dp, z, w1, c1, w2)
        assert w2 <= w1


@pytest.mark.parametrize("fov,bound", [(60.0, 1e-6), (90.0, 5e-5), (120.0, 1e-3)])
def test_paper_polynomial_matches_eq16_where_fitted(fov, bound):
    """The paper's degree-8 polynomial through 51 samples of 2F1 across the band (Sec. 4, step 1):
    even (odd coefficients vanish), and on the f_x axis, where sigma stays within the fitted range,
    Eq. 16 through it differs from the exact map by the fit error (2.5e-7 / 1.8e-5 / 4.8e-4)."""
    lam = 0.5e-6
    s = math.sin(math.radians(fov / 2))
    c = O.paper_polynomial(s)
    assert np.abs(c[::-1][1::2]).max() <= 1e-10
    u = np.linspace(-s, s, 1001)
    exact = O.stretch_map(u / lam, 0.0 * u, lam)[0] * lam
    poly = O.stretch_map_paper(u, 0.0 * u, c)[0]
    nz = np.abs(exact) > 1e-6
    assert np.max(np.abs(poly - exact)[nz] / np.abs(exact[nz])) <= bound


def test_paper_polynomial_inverse_round_trips():
    lam = 0.5e-6
    s = math.sin(math.radians(60.0))
    c = O.paper_polynomial(s)
    g = np.linspace(-0.8, 0.8, 41)
    U, V = np.meshgrid(g, g)
    m = U * U + V * V < 0.95
    up, vp = O.stretch_map_paper(U[m], V[m], c)
    u, v, ok = O.inverse_stretch_paper(up, vp, c)
    assert ok.all()
    assert np.abs(u - U[m]).max() <= 1e-12 and np.abs(v - V[m]).max() <= 1e-12


def test_paper_polynomial_reconstruction():
    """At 60 deg the polynomial is good to 3e-5 everywhere, and the reconstruction follows the exact
    one closely; at 120 deg a point on the x axis (the paper's test points all are) still focuses on
    its position."""
    lam = 0.5e-6
    lam_, dp, zp, xp, yp, H = _spot(60.0, 0.5, n=128, ratio=5.0)
    a = O.reconstruct(H, lam, dp, zp)
    b = O.reconstruct(H, lam, dp, zp, map_model="paper")
    assert O.rel_l2(b, a) <= 1e-3
    dp = synth.fov_pitch(lam, 120.0)
    n = 256
    zp = 8 * n * dp
    L = 0.9 * (zp * math.tan(math.radians(60.0)) - n * dp / 2)
    xo = 0.6 * L
    pc = synth.PointCloud(np.array([xo]), np.array([0.0]), np.array([zp]), np.array([1.0]), np.array([0.0]))
    H = synth.point_hologram(pc, n, n, dp, lam)
    df = lam * zp / (n * dp)
    S = 32
    view = dict(center_x=xo, center_y=0.0, pitch_x=df / 4, pitch_y=df / 4, nx=S, ny=S)
    I = np.abs(O.reconstruct(H, lam, dp, zp, view=view, map_model="paper")) ** 2
    i, j = np.unravel_index(I.argmax(), I.shape)
    assert abs(i - S // 2) <= 2 and abs(j - S // 2) <= 2


def test_focal_stack_single_depth_is_the_reconstruction():
    lam, dp, zp, xp, yp, H = _spot(90.0, 0.5, n=64, ratio=5.0)
    a = O.focal_stack(H, lam, dp, [zp])[0]
    assert np.array_equal(a, O.reconstruct(H, lam, dp, zp))


def test_focal_stack_focuses_a_point_at_its_depth():
    """A depth scan through one on-axis point with the FrT size of the nearest depth forced on all
    (192 against the focus depth's own 180): the intensity (Fresnel number of the defocus about 1
    at 10 %, 2-3 at 20-25 %) peaks at the point's depth and falls on both sides, and the focus sits
    on the axis pixel.  The depths are given out of order: the views follow the order of the
    distances."""
    lam, dp, zp, xp, yp, H = _spot(60.0, 0.0, n=128, ratio=3.0)
    n = H.shape[0]
    fs = [1.1, 0.8, 1.0, 1.25, 0.9]
    outs = O.focal_stack(H, lam, dp, [zp * f for f in fs])
    peaks = np.array([np.max(np.abs(o) ** 2) for o in outs])
    k = fs.index(1.0)
    assert int(np.argmax(peaks)) == k
    p = peaks[np.argsort(fs)]
    assert p[0] < p[1] < p[2] > p[3] > p[4]
    I = np.abs(outs[k]) ** 2
    assert np.unravel_index(I.argmax(), I.shape) == (n // 2, n // 2)
    # the shared size is the nearest depth's, larger than the focus depth's own: the nearest view is
    # its own reconstruction, the focus view is not
    bands = [O.plan_band(n, n, lam, dp, zp * f) for f in fs]
    assert max(b.mx for b in bands) == bands[fs.index(0.8)].mx > bands[k].mx
    assert np.array_equal(outs[fs.index(0.8)], O.reconstruct(H, lam, dp, zp * 0.8))
    assert not np.allclose(outs[k], O.reconstruct(H, lam, dp, zp), rtol=0, atol=1e-6 * np.abs(outs[k]).max())


@pytest.mark.parametrize("fov", [60.0, 90.0, 120.0])
def test_against_rayleigh_sommerfeld(fov):
    """Brute-force RS back-propagation on a tiny grid: same focus, >= 80% of its concentration.

    Reading of the Rayleigh criterion (Sec. 4, accuracy versus pitch): a wavefront
    error below lambda/4 keeps at least 80% of the ideal spot; here the ideal is
    the RS spot, and the measure is the energy within 2 Delta_F of the peak
    (the output is resampled from a Delta_F grid, which broadens a bare peak).
    """
    lam = 0.5e-6
    dp = synth.fov_pitch(lam, fov)
    n = 128
    for seed in range(2):
        pc = synth.draw_points(1000 + 100 * seed + int(fov), 1, n, n, dp, lam, 4 * n * dp, 6 * n * dp)
        H = synth.point_hologram(pc, n, n, dp, lam)
        zp = float(pc.z[0])
        df = lam * zp / (n * dp)
        do, S = df / 2, 24
        view = dict(center_x=float(pc.x[0]), center_y=float(pc.y[0]), pitch_x=do, pitch_y=do, nx=S, ny=S)
        In = np.abs(O.reconstruct(H, lam, dp, zp, view=view)) ** 2
        xo = pc.x[0] + (np.arange(S) - S // 2) * do
        yo = pc.y[0] + (np.arange(S) - S // 2) * do
        X, Y = np.meshgrid(xo, yo)
        Ir = np.abs(O.rayleigh_sommerfeld_backprop(H, dp, lam, zp, X, Y)) ** 2
        a = np.unravel_index(In.argmax(), In.shape)
        b = np.unravel_index(Ir.argmax(), Ir.shape)
        assert abs(a[0] - b[0]) <= 1 and abs(a[1] - b[1]) <= 1

        def ee(I, c):
            yy, xx = np.indices(I.shape)
            return I[(yy - c[0]) ** 2 + (xx - c[1]) ** 2 <= 16].sum() / I.sum()
        assert ee(In, a) >= 0.8 * ee(Ir, b)


def test_diverging_and_converging_conventions_agree():
    """NU-FDS of a diverging hologram is the conjugate of NU-FDS of its conjugate."""
    lam, dp, zp, xp, yp, H = _spot(90.0, 0.4, n=128)
    a = O.reconstruct(H, lam, dp, zp)
    b = O.reconstruct(np.conj(H), lam, dp, zp, flags=O.CONVERGING)
    assert O.rel_l2(a, np.conj(b)) <= 1e-14
