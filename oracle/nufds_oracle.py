"""Float64 CPU oracle of the NU-FDS reconstruction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute this module.  It is a plain, slow
statement of what the reconstruction computes, written from Kozacki et al.,
"Non-uniform Fourier Domain Stretching method for ultra-wide-angle wave
propagation" (arXiv 2410.13474), and it shares no code with the GPU library.

NU-FDS is an approximation (every object wave is replaced by a parabolic wave
whose focus is moved by a non-uniform stretch of the spectrum), so the oracle
takes the paper's five steps in order (Sec. 4, Fig. 3):

  step 1  magnification m_x, m_y of the spectrum (Eq. 16), used through the
          stretch of Eqs. 9-10;
  step 2  FFT of the hologram, non-uniform mapping onto a uniform f' grid
          (as a pull: the stretched spectrum at f' is the spectrum at the
          pre-image of f'), inverse FFT;
  step 3  FFT-based Fresnel transform FrT (Eq. 2);
  step 4  output spatial map x_o -> x_o' (Eqs. 17-18);
  step 5  distortion correction: O(x_o) = O'(x_o'), resampled on the
          uniform output grid, then cropped to the requested view.

Where the paper is silent or garbled the oracle takes one reading; every
reading is named in the docstring that uses it (wave sign, pull vs push,
interpolation kernel, FrT pitch, sub-band rule, evanescent samples).

Notation follows the paper: ``wavelength`` (lambda), ``pitch`` (Delta),
``z`` (z_o), ``k = 2 pi / lambda``, spatial frequencies f_x, f_y, direction
sines u = lambda f_x, v = lambda f_y, stretched quantities primed.

Parity note: the interpolation kernel (Keys cubic), the aperture pad of the
sub-band rule and the phase convention of the output are design readings the
paper does not fix; they are checked only by GPU-vs-oracle parity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import special

__all__ = [
    "CONVERGING", "NO_STRETCH", "NO_REMAP",
    "sine_max", "fov_deg", "image_size", "frt_pitch",
    "local_frequency_x", "local_curvature_x", "frt_spot_x", "corrected_focus",
    "I_integral", "I_ONE", "magnification_x", "magnification_y",
    "stretch_map", "stretch_jacobian_xx", "inverse_stretch",
    "output_map", "output_map_inverse_eq18b",
    "keys_weight", "smooth5_even", "Band", "plan_band",
    "centred_dft2", "centred_idft2", "centred_dft2_direct",
    "stretch_gather", "fresnel_frt", "reconstruct", "focal_stack",
    "paper_polynomial", "I_paper", "stretch_map_paper", "inverse_stretch_paper", "output_map_paper",
    "rayleigh_sommerfeld_backprop", "rel_l2",
]

# Flags (same meaning as the library's public flags).
CONVERGING = 1   # input follows Eq. 3, exp(-i k R); default: diverging exp(+i k r)/r
NO_STRETCH = 2   # m_x = m_y = 1 (the stretch of step 2 is the identity)
NO_REMAP = 4     # skip step 5: output sampled at the distorted coordinates x'

_SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------------------
# Geometry (Sec. 2, Eq. 1 and the FrT sampling stated after Eq. 2)
# --------------------------------------------------------------------------

def sine_max(wavelength: float, pitch: float) -> float:
    """s = lambda / (2 Delta): sine of the half field of view (Sec. 2, Eq. 1)."""
    s = wavelength / (2.0 * pitch)
    if not (0.0 < s < 1.0):
        raise ValueError("wavelength / (2 pitch) must lie in (0, 1)")
    return s


def fov_deg(wavelength: float, pitch: float) -> float:
    """Full field of view 2 asin(lambda / 2 Delta), in degrees (Sec. 2)."""
    return 2.0 * math.degrees(math.asin(sine_max(wavelength, pitch)))


def image_size(wavelength: float, pitch: float, z: float) -> float:
    """Image size B_xo = 2 z_o tan(asin(lambda / 2 Delta)) (Sec. 2, Eq. 1)."""
    return 2.0 * z * math.tan(math.asin(sine_max(wavelength, pitch)))


def frt_pitch(wavelength: float, z: float, n: int, pitch: float) -> float:
    """Sampling of the FrT output, lambda z_o / (N Delta) (Sec. 2, after Eq. 2)."""
    return wavelength * z / (n * pitch)


# --------------------------------------------------------------------------
# Phase-space tools of the point hologram of Eq. 3 (Sec. 2, Eqs. 4-5)
# --------------------------------------------------------------------------

def local_frequency_x(x, y, xo, yo, zo, wavelength):
    """Local spatial frequency of exp(-i k R_o): -(x - x_o)/(lambda R_o) (Eq. 4)."""
    R = np.sqrt((x - xo) ** 2 + (y - yo) ** 2 + zo * zo)
    return -(x - xo) / (wavelength * R)


def local_curvature_x(x, y, xo, yo, zo):
    """Local spatial curvature -((y - y_o)^2 + z_o^2) / R_o^3 (Eq. 5)."""
    R = np.sqrt((x - xo) ** 2 + (y - yo) ** 2 + zo * zo)
    return -((y - yo) ** 2 + zo * zo) / R ** 3


def frt_spot_x(xo, yo, zo, wavelength):
    """Where a plain FrT at z_o puts the point: z_o lambda f_xl(0,0) (Sec. 2)."""
    return zo * wavelength * local_frequency_x(0.0, 0.0, xo, yo, zo, wavelength)


def corrected_focus(xo, yo, zo, wavelength):
    """Focus of the paraxial wave equivalent at the hologram centre (Sec. 2).

    Returns (x_ro, z_ro) = (lambda f_xl(0,0) / |c_xl(0,0)|, 1 / |c_xl(0,0)|).
    Reading: Eq. 5 carries a minus sign for a converging wave, and the paper
    quotes the distance as a positive number, so the magnitude is taken.
    """
    f = local_frequency_x(0.0, 0.0, xo, yo, zo, wavelength)
    c = abs(local_curvature_x(0.0, 0.0, xo, yo, zo))
    return wavelength * f / c, 1.0 / c


# --------------------------------------------------------------------------
# Step 1: the non-uniform magnification (Sec. 3-4, Eqs. 9-10, 15-16)
# --------------------------------------------------------------------------

def _I_from_sc(sigma, c):
    """I(sigma) = int_0^sigma (1 - w^2)^(-3/4) dw, given c = sqrt(1 - sigma^2).

    Uses I(sigma) = sqrt(2) F(beta | 1/2) with cos^2(beta) = c, the
    substitution w = sin(gamma), cos(gamma) = cos^2(beta) taking the
    integrand to an incomplete elliptic integral of the first kind.  Passing
    c separately keeps the value accurate when sigma is within rounding of 1.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    beta = np.arctan2(np.abs(sigma) / np.sqrt(1.0 + c), np.sqrt(c))
    return np.sign(sigma) * _SQRT2 * special.ellipkinc(beta, 0.5)


def I_integral(sigma):
    """I(sigma) = int_0^sigma (1 - w^2)^(-3/4) dw = sigma 2F1(1/2, 3/4; 3/2; sigma^2).

    This is the integral of Eq. 15 along f_x; Eq. 16 is u m_x = sqrt(a) I(u/a)
    with a = sqrt(1 - v^2).  Evaluated through the elliptic form above.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    return _I_from_sc(sigma, np.sqrt(np.maximum(0.0, 1.0 - sigma * sigma)))


# I(1) = Gamma(3/2) Gamma(1/4) / Gamma(3/4), Gauss's value of 2F1 at 1.
I_ONE = float(special.gamma(1.5) * special.gamma(0.25) / special.gamma(0.75))


def magnification_x(fx, fy, wavelength):
    """m_x(f_x, f_y) of Eq. 16, written out with the hypergeometric function.

    m_x = (1 - lambda^2 f_y^2)^(-1/4) 2F1(1/2, 3/4; 3/2; lambda^2 f_x^2 / (1 - lambda^2 f_y^2)).
    """
    fx = np.asarray(fx, dtype=np.float64)
    fy = np.asarray(fy, dtype=np.float64)
    a2 = 1.0 - (wavelength * fy) ** 2
    return a2 ** -0.25 * special.hyp2f1(0.5, 0.75, 1.5, (wavelength * fx) ** 2 / a2)


def magnification_y(fx, fy, wavelength):
    """m_y(f_x, f_y): Eq. 16 with the axes exchanged (Sec. 4)."""
    return magnification_x(fy, fx, wavelength)


def stretch_map(fx, fy, wavelength):
    """f' = (f_x m_x(f_x, f_y), f_y m_y(f_x, f_y)) -- Eqs. 9-10 with Eq. 16."""
    return (fx * magnification_x(fx, fy, wavelength),
            fy * magnification_y(fx, fy, wavelength))


def stretch_jacobian_xx(fx, fy, wavelength):
    """d f_x' / d f_x from the magnification condition (Eq. 15)."""
    u = wavelength * np.asarray(fx, dtype=np.float64)
    v = wavelength * np.asarray(fy, dtype=np.float64)
    return np.sqrt(1.0 - v * v) * (1.0 - v * v - u * u) ** -0.75


def _level_point(v, t1):
    """Point (u, v) on the curve T_1(u, v) = t1, with the accurate rim distance.

    With a_v = sqrt(1 - v^2), T_1 = sqrt(a_v) I(u / a_v) = t1 fixes
    sigma_1 = u / a_v = I^{-1}(t1 / sqrt(a_v)).  Inverting I through Jacobi's
    elliptic functions, I(sigma) = sqrt(2) F(beta | 1/2) gives cn(y) = cos(beta)
    with y = t1 / sqrt(2 a_v), so sigma_1 = sqrt(1 - cn^4), and the distance
    to the rim of the unit disk is d = 1 - u^2 - v^2 = a_v^2 cn^4.
    """
    av = np.sqrt((1.0 - v) * (1.0 + v))
    y = t1 / (_SQRT2 * np.sqrt(av))
    sn, cn, _, _ = special.ellipj(y, 0.5)
    sigma1 = np.abs(sn) * np.sqrt(1.0 + cn * cn)
    u = av * sigma1
    d = av * av * cn ** 4
    au = np.sqrt(v * v + d)                      # sqrt(1 - u^2), accurate near the rim
    safe = au > 0.0
    au_s = np.where(safe, au, 1.0)
    sigma2 = np.where(safe, v / au_s, 0.0)
    c2 = np.where(safe, av * cn * cn / au_s, 1.0)  # sqrt(1 - sigma2^2)
    I2 = _I_from_sc(sigma2, c2)
    Iv1 = t1 / np.sqrt(av)
    return u, d, au, av, sigma1, Iv1, sigma2, I2, np.abs(cn)


def _level_residual(v, t1, t2):
    """h(v) = T_2 - t2 along T_1 = t1, and dh/dv (det J / J_11, Eq. 15 terms)."""
    u, d, au, av, s1, Iv1, s2, I2, acn = _level_point(v, t1)
    h = np.sqrt(au) * I2 - t2
    d14 = np.sqrt(av) * acn                      # d^(1/4)
    dh = (d14 / (au * av * av)
          + (u * v / (2.0 * av)) * (s1 * I2 * au ** -1.5 + s2 * Iv1 * av ** -1.5)
          - u * v * Iv1 * I2 * d14 ** 3 / (4.0 * au ** 1.5 * av ** 2.5))
    return h, dh, u


def inverse_stretch(up, vp, max_iter=60):
    """Pre-image (u, v) of stretched direction sines (u', v') under Eqs. 9-10.

    Reading (pull form of step 2): the paper pushes each spectral sample to
    f' = f m(f) and interpolates the scattered result; the same continuous
    operator is the stretched spectrum H'(f') = H(f) at the pre-image f of f',
    which is what is computed here.

    The map (u, v) -> (sqrt(a_v) I(u/a_v), sqrt(a_u) I(v/a_u)) is odd in each
    axis and symmetric under exchange of the axes, so the pre-image is found
    for (|u'|, |v'|) ordered so that |u'| >= |v'|, and signs and order are
    restored.  The rim u^2 + v^2 = 1 maps onto |u'|^4 + |v'|^4 = I(1)^4, so a
    pre-image inside the open unit disk exists exactly when
    |u'|^4 + |v'|^4 < I(1)^4; otherwise ``valid`` is False.  Inside, v solves
    h(v) = 0 along the curve T_1 = |u'| on [0, sqrt(1 - (|u'|/I(1))^4)],
    by Newton's method kept inside a bisection bracket (h increases with v).

    Returns (u, v, valid) as float64 arrays.
    """
    up = np.asarray(up, dtype=np.float64)
    vp = np.asarray(vp, dtype=np.float64)
    shape = np.broadcast(up, vp).shape
    up = np.broadcast_to(up, shape).ravel()
    vp = np.broadcast_to(vp, shape).ravel()
    au_, av_ = np.abs(up), np.abs(vp)
    swap = av_ > au_
    t1 = np.where(swap, av_, au_)
    t2 = np.where(swap, au_, av_)
    valid = t1 ** 4 + t2 ** 4 < I_ONE ** 4
    t1 = np.where(valid, t1, 0.0)
    t2 = np.where(valid, t2, 0.0)
    vmax = np.sqrt(np.maximum(0.0, 1.0 - (t1 / I_ONE) ** 4))
    lo = np.zeros_like(t1)
    hi = vmax.copy()
    v = np.clip(t2 / (1.0 + 0.25 * (t1 * t1 + t2 * t2)), 0.0, vmax)
    active = valid & (t2 > 0.0)
    v = np.where(t2 > 0.0, v, 0.0)
    for _ in range(max_iter):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        va = v[idx]
        h, dh, _ = _level_residual(va, t1[idx], t2[idx])
        l_ = np.where(h <= 0.0, va, lo[idx])
        h_ = np.where(h > 0.0, va, hi[idx])
        vn = va - h / dh
        out = ~((vn >= l_) & (vn <= h_)) | ~np.isfinite(vn)
        vn = np.where(out, 0.5 * (l_ + h_), vn)
        lo[idx], hi[idx], v[idx] = l_, h_, vn
        done = (np.abs(vn - va) <= 4e-16) | (h == 0.0) | (h_ - l_ <= 4e-16)
        active[idx] = ~done
    u, _, _, _, _, _, _, _, _ = _level_point(v, t1)
    u = np.where(valid, u, 0.0)
    v = np.where(valid, v, 0.0)
    uu = np.where(swap, v, u) * np.sign(up)
    vv = np.where(swap, u, v) * np.sign(vp)
    return uu.reshape(shape), vv.reshape(shape), valid.reshape(shape)


# --------------------------------------------------------------------------
# The paper's own approximation of Eq. 16 (step 1), for comparison
# --------------------------------------------------------------------------

def paper_polynomial(s, degree=8, samples=51):
    """Coefficients (highest power first) of the paper's stand-in for the hypergeometric function.

    Sec. 4, step 1: a degree-8 polynomial fitted to 51 frequencies spread uniformly across the
    hologram's band, whose coefficients replace 2F1 in Eq. 16.  Reading: the samples are Eq. 16 on
    the f_x axis, m_x(f_x, 0) = 2F1(1/2, 3/4; 3/2; u^2) at u = lambda f_x in [-s, s], fitted by least
    squares as a polynomial p(u); wherever Eq. 16 needs 2F1 at sigma^2 (sigma = u / a_v) it takes
    p(sigma), so I(sigma) = sigma 2F1(...; sigma^2) becomes I_P(sigma) = sigma p(sigma).  Beyond the
    fitted range (|sigma| > s, reached off the axes) the polynomial is extrapolated, as in the paper.
    """
    u = np.linspace(-s, s, samples)
    return np.polyfit(u, special.hyp2f1(0.5, 0.75, 1.5, u * u), degree)


def I_paper(sigma, coef):
    """I_P(sigma) = sigma p(sigma) and its derivative p(sigma) + sigma p'(sigma)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    p = np.polyval(coef, sigma)
    dp = np.polyval(np.polyder(coef), sigma)
    return sigma * p, p + sigma * dp


def stretch_map_paper(u, v, coef):
    """(u', v') = (sqrt(a_v) I_P(u / a_v), sqrt(a_u) I_P(v / a_u)): Eqs. 9-10 with the polynomial."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    av, au = np.sqrt(1.0 - v * v), np.sqrt(1.0 - u * u)
    return np.sqrt(av) * I_paper(u / av, coef)[0], np.sqrt(au) * I_paper(v / au, coef)[0]


def inverse_stretch_paper(up, vp, coef, iters=12):
    """Pre-image (u, v) of (u', v') under the polynomial map, by 2-D Newton from the exact pre-image.

    The two maps differ by the fit error, so the exact pre-image starts Newton within its quadratic
    range.  Masked where the exact inverse is (no pre-image on the open disk), and where Newton
    leaves the disk or its residual after the fixed iteration count stays above 1e-10 (a converged
    residual is ~1e-16, an unconverged one far larger: the decision does not hang on rounding).
    Returns (u, v, valid).
    """
    up = np.asarray(up, dtype=np.float64)
    vp = np.asarray(vp, dtype=np.float64)
    u, v, valid = inverse_stretch(up, vp)
    for _ in range(iters):
        av, au = np.sqrt(np.maximum(1.0 - v * v, 1e-300)), np.sqrt(np.maximum(1.0 - u * u, 1e-300))
        s1, s2 = u / av, v / au
        I1, dI1 = I_paper(s1, coef)
        I2, dI2 = I_paper(s2, coef)
        r1 = np.sqrt(av) * I1 - up
        r2 = np.sqrt(au) * I2 - vp
        # Jacobian: d sqrt(a) I(x / a) / dx = dI / sqrt(a); d / dy through a = sqrt(1 - y^2)
        j11 = dI1 / np.sqrt(av)
        j12 = (0.5 * I1 / np.sqrt(av) - dI1 * s1 / np.sqrt(av)) * (-v / av)
        j22 = dI2 / np.sqrt(au)
        j21 = (0.5 * I2 / np.sqrt(au) - dI2 * s2 / np.sqrt(au)) * (-u / au)
        det = j11 * j22 - j12 * j21
        du = (r1 * j22 - r2 * j12) / det
        dv = (r2 * j11 - r1 * j21) / det
        u = np.where(valid, u - du, u)
        v = np.where(valid, v - dv, v)
    r1, r2 = stretch_map_paper(u, v, coef)
    ok = valid & (u * u + v * v < 1.0) & (np.abs(r1 - up) <= 1e-10) & (np.abs(r2 - vp) <= 1e-10)
    return np.where(ok, u, 0.0), np.where(ok, v, 0.0), ok


def output_map_paper(xo, yo, z, coef):
    """Eqs. 17-18 with the polynomial: x_o' = z sqrt(a_v) I_P(u / a_v) at u = x_o / R, v = y_o / R."""
    xo = np.asarray(xo, dtype=np.float64)
    yo = np.asarray(yo, dtype=np.float64)
    R = np.sqrt(xo * xo + yo * yo + z * z)
    xp, yp = stretch_map_paper(xo / R, yo / R, coef)
    return z * xp, z * yp


# --------------------------------------------------------------------------
# Step 4: output spatial map x_o -> x_o' (Sec. 4, Eqs. 17-18)
# --------------------------------------------------------------------------

def output_map(xo, yo, z, wavelength=1.0):
    """(x_o', y_o') = z_o lambda (f_x m_x, f_y m_y) at the centre frequency.

    Eqs. 17-18, with the frequency the point generates at the hologram
    centre, f_x0 = x_o / (lambda R), f_y0 = y_o / (lambda R),
    R = sqrt(x_o^2 + y_o^2 + z_o^2) (Sec. 3, before Eq. 13).  The result does
    not depend on lambda.
    """
    xo = np.asarray(xo, dtype=np.float64)
    yo = np.asarray(yo, dtype=np.float64)
    R = np.sqrt(xo * xo + yo * yo + z * z)
    fx0 = xo / (wavelength * R)
    fy0 = yo / (wavelength * R)
    return (z * wavelength * fx0 * magnification_x(fx0, fy0, wavelength),
            z * wavelength * fy0 * magnification_y(fx0, fy0, wavelength))


def output_map_inverse_eq18b(xp, yp, z, iters=4, wavelength=1.0):
    """The paper's sequential inversion x_o' -> x_o of step 4 (second Eq. 18).

    x_o(k) = x_o' sqrt(x_o(k-1)^2 + y_o(k-1)^2 + z^2) / (z m_x(f_x0(k-1), f_y0(k-1))),
    likewise for y, starting from x_o(1) = x_o'.  Returns the list of iterates
    [x_o(1), ..., x_o(iters)] as (x, y) pairs.
    """
    xp = np.asarray(xp, dtype=np.float64)
    yp = np.asarray(yp, dtype=np.float64)
    x, y = xp.copy(), yp.copy()
    out = [(x, y)]
    for _ in range(iters - 1):
        R = np.sqrt(x * x + y * y + z * z)
        fx0 = x / (wavelength * R)
        fy0 = y / (wavelength * R)
        x, y = (xp * R / (z * magnification_x(fx0, fy0, wavelength)),
                yp * R / (z * magnification_y(fx0, fy0, wavelength)))
        out.append((x, y))
    return out


# --------------------------------------------------------------------------
# Interpolation kernel and sizes (readings: the paper does not name them)
# --------------------------------------------------------------------------

def keys_weight(t):
    """Keys cubic convolution weight with a = -1/2 (Keys, 1981).

    Reading: the paper interpolates in steps 2 and 5 without naming the
    kernel; a separable 4 x 4 Keys kernel is used in both.
    """
    t = np.abs(np.asarray(t, dtype=np.float64))
    w_in = (1.5 * t - 2.5) * t * t + 1.0
    w_out = ((-0.5 * t + 2.5) * t - 4.0) * t + 2.0
    return np.where(t <= 1.0, w_in, np.where(t < 2.0, w_out, 0.0))


def smooth5_even(n: int) -> int:
    """Smallest even integer >= n whose only prime factors are 2, 3 and 5."""
    n = max(2, int(n))
    while True:
        if n % 2 == 0:
            m = n
            for p in (2, 3, 5):
                while m % p == 0:
                    m //= p
            if m == 1:
                return n
        n += 1


@dataclass
class Band:
    """Sizes and offsets of one reconstruction (per axis x, y)."""
    nx: int
    ny: int
    sx: int          # output samples
    sy: int
    cx: float        # output window centre, metres
    cy: float
    dox: float       # output pitch, metres
    doy: float
    dfx: float       # FrT output pitch Delta_F = lambda z / (N Delta)
    dfy: float
    mx: int          # FrT size (sub-band width in spectral samples)
    my: int
    kcx: int         # sub-band centre, in spectral samples / FrT pixels
    kcy: int
    padx: float
    pady: float
    xlo: float       # x' extent of the window (before padding)
    xhi: float
    ylo: float
    yhi: float


def _xprime_extremes(x_lo, x_hi, y_lo, y_hi, z, remap):
    """Smallest and largest x' over the window rectangle.

    x' = z I(x / sqrt(x^2 + z^2)) ((x^2 + z^2) / (x^2 + y^2 + z^2))^(1/4) grows
    with x and its magnitude falls with |y| (Eqs. 17-18), so both extremes sit
    on the vertical edges, at the y closest to 0 when the edge lies on the
    same side as the extreme, and at the farthest y otherwise.
    """
    if not remap:
        return x_lo, x_hi
    y_near = min(max(0.0, y_lo), y_hi)
    y_far = y_lo if abs(y_lo) > abs(y_hi) else y_hi
    hi = output_map(x_hi, y_near if x_hi >= 0.0 else y_far, z)[0]
    lo = output_map(x_lo, y_near if x_lo <= 0.0 else y_far, z)[0]
    return float(lo), float(hi)


def plan_band(nx, ny, wavelength, pitch, z, view=None, flags=0, pad=None,
              frt_size=None) -> Band:
    """Output grid, sub-band centre K_c and FrT size M of one reconstruction.

    Readings (Sec. 4, output parameter selection and partial view):
      * the FrT runs at Delta_F = lambda z / (N Delta), the spectral pitch of
        the hologram, whatever the output pitch; step 5 resamples to the
        output pitch (coupling the FrT pitch to the output pitch would alias
        whenever Delta_o > Delta_F);
      * the processed band is the rectangle of stretched frequencies whose
        FrT image covers the window's x' extent plus an aperture pad of
        N Delta / 2 on each side (room for the chirp bandwidth of a point
        seen through the whole aperture);
      * K_c = round(centre / Delta_F), M = smallest even 5-smooth integer
        >= 2 ceil(half width / Delta_F), with a 1e-9 sample tolerance in the
        ceiling.
    ``view`` is None (full view: the whole image B x B of Eq. 1 on nx x ny
    samples) or a dict with keys center_x, center_y, pitch_x, pitch_y
    (<= 0 means Delta_F), nx, ny.
    """
    s = sine_max(wavelength, pitch)
    B = image_size(wavelength, pitch, z)
    dfx = frt_pitch(wavelength, z, nx, pitch)
    dfy = frt_pitch(wavelength, z, ny, pitch)
    if view is None:
        cx = cy = 0.0
        sx, sy = nx, ny
        dox, doy = B / nx, B / ny
    else:
        cx, cy = float(view["center_x"]), float(view["center_y"])
        sx, sy = int(view["nx"]), int(view["ny"])
        dox = float(view.get("pitch_x", 0.0))
        doy = float(view.get("pitch_y", 0.0))
        dox = dfx if dox <= 0.0 else dox
        doy = dfy if doy <= 0.0 else doy
    if sx <= 0 or sy <= 0:
        raise ValueError("output size must be positive")
    x_lo, x_hi = cx - 0.5 * sx * dox, cx + 0.5 * sx * dox
    y_lo, y_hi = cy - 0.5 * sy * doy, cy + 0.5 * sy * doy
    tol = 1e-9 * B
    if x_lo < -0.5 * B - tol or x_hi > 0.5 * B + tol or y_lo < -0.5 * B - tol or y_hi > 0.5 * B + tol:
        raise ValueError("view window leaves the image area of Eq. 1")
    remap = not (flags & NO_REMAP)
    xl, xh = _xprime_extremes(x_lo, x_hi, y_lo, y_hi, z, remap)
    yl, yh = _xprime_extremes(y_lo, y_hi, x_lo, x_hi, z, remap)
    if pad is None:
        padx, pady = 0.5 * nx * pitch, 0.5 * ny * pitch
    else:
        padx = pady = float(pad)

    def axis(lo, hi, df, pad_, forced):
        lo, hi = lo - pad_, hi + pad_
        kc = math.floor(0.5 * (lo + hi) / df + 0.5)
        half = max(hi - kc * df, kc * df - lo) / df
        m = int(forced) if forced else smooth5_even(2 * math.ceil(half - 1e-9))
        return kc, m

    fx_, fy_ = frt_size if frt_size else (None, None)
    kcx, mx = axis(xl, xh, dfx, padx, fx_)
    kcy, my = axis(yl, yh, dfy, pady, fy_)
    return Band(nx=nx, ny=ny, sx=sx, sy=sy, cx=cx, cy=cy, dox=dox, doy=doy,
                dfx=dfx, dfy=dfy, mx=mx, my=my, kcx=kcx, kcy=kcy,
                padx=padx, pady=pady, xlo=xl, xhi=xh, ylo=yl, yhi=yh)


# --------------------------------------------------------------------------
# Centred discrete Fourier transforms (steps 2 and 3)
# --------------------------------------------------------------------------

def centred_dft2(a):
    """A[k] = sum_n a[n] exp(-2 pi i (k - N/2)(n - N/2) / N) on both axes.

    Unnormalised; index N/2 is the zero coordinate / frequency (even sizes).
    """
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(a)))


def centred_idft2(a):
    """a[n] = (1 / (M_x M_y)) sum_k A[k] exp(+2 pi i (k - M/2)(n - M/2) / M)."""
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(a)))


def centred_dft2_direct(a, inverse=False):
    """The same transforms as explicit DFT matrices (small sizes only)."""
    ny, nx = a.shape
    sgn = 1.0 if inverse else -1.0
    cx = np.arange(nx) - nx // 2
    cy = np.arange(ny) - ny // 2
    Wx = np.exp(sgn * 2j * np.pi * np.outer(cx, cx) / nx)
    Wy = np.exp(sgn * 2j * np.pi * np.outer(cy, cy) / ny)
    out = Wy @ a @ Wx.T
    return out / (nx * ny) if inverse else out


# --------------------------------------------------------------------------
# Step 2: stretch of the spectrum onto the uniform f' grid of the sub-band
# --------------------------------------------------------------------------

def _keys_gather(A, py, px, periodic):
    """sum_{a,b=-1..2} w(p_x - floor(p_x) - a) w(p_y - floor(p_y) - b) A[.., ..].

    ``periodic``: indices wrap (the DFT spectrum is periodic); otherwise taps
    outside the array contribute zero.
    """
    ny, nx = A.shape
    fx, fy = np.floor(px), np.floor(py)
    ix, iy = fx.astype(np.int64), fy.astype(np.int64)
    tx, ty = px - fx, py - fy
    out = np.zeros(px.shape, dtype=np.complex128)
    for b in range(-1, 3):
        wy = keys_weight(ty - b)
        jy = iy + b
        if periodic:
            jy_c, oky = np.mod(jy, ny), True
        else:
            oky = (jy >= 0) & (jy < ny)
            jy_c = np.clip(jy, 0, ny - 1)
        for a in range(-1, 3):
            wx = keys_weight(tx - a)
            jx = ix + a
            if periodic:
                jx_c, okx = np.mod(jx, nx), True
            else:
                okx = (jx >= 0) & (jx < nx)
                jx_c = np.clip(jx, 0, nx - 1)
            val = A[jy_c, jx_c]
            if not periodic:
                val = np.where(oky & okx, val, 0.0)
            out += wx * wy * val
    return out


def stretch_gather(Hs, band: Band, wavelength, pitch, flags=0, coef=None):
    """Stretched spectrum H'(f'_u) on the M_y x M_x sub-band (step 2).

    Sample (k'_y, k'_x) is the stretched frequency f' = (K_c + k' - M/2) / (N Delta)
    per axis.  Its pre-image f under Eqs. 9-10 is found by
    :func:`inverse_stretch`; the hologram spectrum is interpolated there with
    the Keys kernel, periodically (source index p = u N Delta / lambda + N/2).
    Reading: a sample is zero when f' has no pre-image on the propagating
    disk, or when the pre-image lies outside the hologram band
    |u|, |v| <= lambda / (2 Delta).
    ``Hs`` may be the spectrum of the hologram zero-padded to sigma N (frequency
    pitch 1 / (sigma N Delta)): the source index is then p = u sigma N Delta / lambda
    + sigma N / 2 on that grid.  ``coef``: the paper's polynomial stand-in for 2F1
    (:func:`paper_polynomial`) instead of the exact map.
    Returns (H', u, v, valid).
    """
    nys, nxs = Hs.shape
    nx, ny = band.nx, band.ny                 # the hologram's own grid sets f'
    sig_x, sig_y = nxs // nx, nys // ny
    s = sine_max(wavelength, pitch)
    kgx = band.kcx + np.arange(band.mx) - band.mx // 2
    kgy = band.kcy + np.arange(band.my) - band.my // 2
    KX, KY = np.meshgrid(kgx.astype(np.float64), kgy.astype(np.float64))
    if flags & NO_STRETCH:
        # m = 1: the pre-image of spectral sample k_g is sample k_g itself.
        px, py = sig_x * KX + nxs // 2, sig_y * KY + nys // 2
        u = KX * wavelength / (nx * pitch)
        v = KY * wavelength / (ny * pitch)
        # |u| <= s is |k_g| <= N/2 in index units; tested exactly there
        valid = (np.abs(KX) <= nx // 2) & (np.abs(KY) <= ny // 2)
    else:
        up = KX * wavelength / (nx * pitch)
        vp = KY * wavelength / (ny * pitch)
        if coef is None:
            u, v, valid = inverse_stretch(up, vp)
        else:
            u, v, valid = inverse_stretch_paper(up, vp, coef)
        valid = valid & (np.abs(u) <= s) & (np.abs(v) <= s)
        px = u * (nxs * pitch / wavelength) + nxs // 2
        py = v * (nys * pitch / wavelength) + nys // 2
    px = np.where(valid, px, 0.0)
    py = np.where(valid, py, 0.0)
    Ht = _keys_gather(Hs, py, px, periodic=True)
    return np.where(valid, Ht, 0.0), u, v, valid


# --------------------------------------------------------------------------
# Step 3: FFT-based Fresnel transform (Eq. 2)
# --------------------------------------------------------------------------

def fresnel_frt(h, band: Band, wavelength, pitch, z):
    """F = DFT(h exp(+i k (xi_x^2 + xi_y^2) / 2 z_o)) of Eq. 2 (step 3).

    h is sampled at xi = (n - M/2) N Delta / M (the inverse transform of M
    spectral samples at pitch 1 / (N Delta)); F[m] sits at
    x' = K_c Delta_F + (m - M/2) Delta_F.  The carrier of an off-centre
    sub-band cancels against the FrT kernel because Delta_F / (lambda z) is
    the spectral pitch, so the transform is centred and only the output is
    offset.  The outer chirp of Eq. 2 is applied after resampling (step 5).
    """
    k = 2.0 * math.pi / wavelength
    xi_x = (np.arange(band.mx) - band.mx // 2) * (band.nx * pitch / band.mx)
    xi_y = (np.arange(band.my) - band.my // 2) * (band.ny * pitch / band.my)
    chirp = np.exp(1j * k * (xi_y[:, None] ** 2 + xi_x[None, :] ** 2) / (2.0 * z))
    return centred_dft2(h * chirp)


# --------------------------------------------------------------------------
# The whole reconstruction (steps 1-5)
# --------------------------------------------------------------------------

def reconstruct(H, wavelength, pitch, z, view=None, flags=0, pad=None,
                frt_size=None, return_stages=False, oversample=1, map_model="exact"):
    """NU-FDS reconstruction of hologram ``H`` at distance ``z`` (float64).

    ``H`` is ``[ny, nx]`` complex, pixel (i, j) at ((j - nx/2) Delta, (i - ny/2) Delta).
    Returns the ``[S_y, S_x]`` complex128 output whose pixel (i, j) sits at
    (c_x + (j - S_x/2) Delta_ox, c_y + (i - S_y/2) Delta_oy) at distance z.

    Reading (wave sign): the paper's Eq. 2 focuses waves converging as in
    Eq. 3, exp(-i k R).  A hologram of diverging waves exp(+i k r)/r (the
    default) is its complex conjugate, so it is conjugated on input and the
    output is conjugated back; ``CONVERGING`` skips both.

    ``oversample`` = 2 computes the spectrum of step 2 from the hologram
    zero-padded (centred) to 2N x 2N, i.e. the same spectrum sampled twice as
    finely, before the stretch interpolates it; everything else is unchanged.
    ``map_model`` = "paper" uses the paper's polynomial stand-in for the
    hypergeometric function (:func:`paper_polynomial`) in steps 1 and 4.
    """
    H = np.asarray(H, dtype=np.complex128)
    ny, nx = H.shape
    if nx % 2 or ny % 2:
        raise ValueError("hologram sizes must be even")
    band = plan_band(nx, ny, wavelength, pitch, z, view, flags, pad, frt_size)
    if map_model not in ("exact", "paper"):
        raise ValueError("map_model must be 'exact' or 'paper'")
    # the paper variant changes steps 1 and 4 only; the band stays the exact map's (the pad covers
    # the fit error's few-sample shift of the window's distorted image)
    coef = paper_polynomial(sine_max(wavelength, pitch)) if map_model == "paper" else None
    k = 2.0 * math.pi / wavelength
    if not (flags & CONVERGING):
        H = np.conj(H)
    # step 2: spectrum, stretch onto the uniform f' grid, inverse transform
    if oversample not in (1, 2):
        raise ValueError("oversample must be 1 or 2")
    if oversample > 1:
        Hp = np.zeros((oversample * ny, oversample * nx), dtype=np.complex128)
        oy, ox = (oversample - 1) * ny // 2, (oversample - 1) * nx // 2
        Hp[oy:oy + ny, ox:ox + nx] = H
        H = Hp
    Hs = centred_dft2(H)
    Ht, _, _, _ = stretch_gather(Hs, band, wavelength, pitch, flags, coef)
    h = centred_idft2(Ht)
    # step 3: FrT
    F = fresnel_frt(h, band, wavelength, pitch, z)
    # steps 4-5: output grid in true coordinates, its distorted position,
    # resampling of the pre-chirp FrT and the outer chirp of Eq. 2
    xo = band.cx + (np.arange(band.sx) - band.sx // 2) * band.dox
    yo = band.cy + (np.arange(band.sy) - band.sy // 2) * band.doy
    XO, YO = np.meshgrid(xo, yo)
    if flags & NO_REMAP:
        XP, YP = XO, YO
    else:
        XP, YP = output_map(XO, YO, z) if coef is None else output_map_paper(XO, YO, z, coef)
    qx = (XP - band.kcx * band.dfx) / band.dfx + band.mx // 2
    qy = (YP - band.kcy * band.dfy) / band.dfy + band.my // 2
    O = _keys_gather(F, qy, qx, periodic=False)
    O = O * np.exp(1j * k * (XP * XP + YP * YP) / (2.0 * z))
    if not (flags & CONVERGING):
        O = np.conj(O)
    if return_stages:
        return O, dict(band=band, spectrum=Hs, stretched=Ht, h=h, F=F, xp=XP, yp=YP)
    return O


def focal_stack(H, wavelength, pitch, zs, flags=0):
    """Full views of hologram ``H`` at each distance in ``zs``, with one FrT size for all of them.

    The paper reconstructs one hologram at several depths (Sec. 5, Figs. 8 and 10).  At the FrT
    pitch Delta_F = lambda z / (N Delta) the spectral pitch of the stretched band is 1 / (N Delta)
    whatever z, so steps 1-2 (the stretch of Eqs. 9-10 with Eq. 16 and the inverse transform) give
    the same array for every depth that shares the band.  Reading: the shared FrT size is the
    largest the band rule gives over the depths (the aperture pad N Delta / 2 spans the most FrT
    samples at the smallest z); each depth is then ``reconstruct`` at its z with that size forced.
    Returns the list of [ny, nx] complex128 views in the order of ``zs``.
    """
    H = np.asarray(H, dtype=np.complex128)
    ny, nx = H.shape
    bands = [plan_band(nx, ny, wavelength, pitch, z, None, flags) for z in zs]
    size = (max(b.mx for b in bands), max(b.my for b in bands))
    return [reconstruct(H, wavelength, pitch, z, flags=flags, frt_size=size) for z in zs]


# --------------------------------------------------------------------------
# Independent physics reference and error measure
# --------------------------------------------------------------------------

def rayleigh_sommerfeld_backprop(H, pitch, wavelength, z, xo, yo):
    """Direct back-propagation U(x_o) = sum_n H_n conj(h(r_n)) of a diverging hologram.

    h(r) = (z / (i lambda r^2)) (1 - 1 / (i k r)) e^{i k r} is the first
    Rayleigh-Sommerfeld kernel; the conjugate kernel undoes a diverging wave.
    ``xo``, ``yo`` are arrays of output positions.  Plain double loop over
    the output, O(N^2) per output sample: tiny grids only.
    """
    ny, nx = H.shape
    k = 2.0 * math.pi / wavelength
    xs = (np.arange(nx) - nx // 2) * pitch
    ys = (np.arange(ny) - ny // 2) * pitch
    X, Y = np.meshgrid(xs, ys)
    xo = np.asarray(xo, dtype=np.float64)
    yo = np.asarray(yo, dtype=np.float64)
    out = np.zeros(xo.shape, dtype=np.complex128)
    flat_x, flat_y, flat_o = xo.ravel(), yo.ravel(), out.reshape(-1)
    for i in range(flat_x.size):
        r = np.sqrt((flat_x[i] - X) ** 2 + (flat_y[i] - Y) ** 2 + z * z)
        kern = (z / (1j * wavelength * r * r)) * (1.0 - 1.0 / (1j * k * r)) * np.exp(1j * k * r)
        flat_o[i] = np.sum(H * np.conj(kern))
    return out


def rel_l2(a, ref):
    """||a - ref||_2 / ||ref||_2."""
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))
