// Float64 special functions of the NU-FDS stretch and output maps (host and device).
//
// The magnification of Eq. 16 integrates Eq. 15; along one axis it reduces to
//   I(sigma) = int_0^sigma (1 - w^2)^(-3/4) dw = sigma 2F1(1/2, 3/4; 3/2; sigma^2),
// and u m_x(u, v) = sqrt(a) I(u / a) with a = sqrt(1 - v^2).  With the
// substitution w = sin(g), cos(g) = cos^2(beta), I(sigma) = sqrt(2) F(beta | 1/2),
// an incomplete elliptic integral of the first kind, evaluated here through
// Carlson's symmetric integral R_F (duplication algorithm, Carlson 1995).
// Its inverse goes through Jacobi's elliptic functions at parameter 1/2,
// computed with the arithmetic-geometric mean and descending Landen steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace nufds {

#define NUFDS_HD __host__ __device__ __forceinline__

// I(1) = Gamma(3/2) Gamma(1/4) / Gamma(3/4) = sqrt(2) K(1/2).
constexpr double kIOne = 2.6220575542921198;
constexpr double kSqrt2 = 1.4142135623730951;

// Carlson's R_F(x, y, z) for x, y, z >= 0 with at most one zero.
NUFDS_HD double carlson_rf(double x, double y, double z) {
    double a0 = (x + y + z) * (1.0 / 3.0);
    double dx0 = a0 - x, dy0 = a0 - y, dz0 = a0 - z;
    double q = fmax(fabs(dx0), fmax(fabs(dy0), fabs(dz0)));
    // stop once 4^-m (3 r)^(-1/6) q < |A_m| with r = 2^-53: (3 r)^(-1/6) = 380, rounded up
    q *= 400.0;
    double a = a0, pow4 = 1.0;
    for (int m = 0; m < 30; ++m) {
        if (q * pow4 < fabs(a)) break;
        double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        double lam = sx * sy + sx * sz + sy * sz;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        a = 0.25 * (a + lam);
        pow4 *= 0.25;
    }
    double inv = pow4 / a;
    double X = dx0 * inv, Y = dy0 * inv;
    double Z = -(X + Y);
    double e2 = X * Y - Z * Z;
    double e3 = X * Y * Z;
    double poly = 1.0 - 0.1 * e2 + e3 * (1.0 / 14.0) + e2 * e2 * (1.0 / 24.0) - e2 * e3 * (3.0 / 44.0);
    return poly / sqrt(a);
}

// I(sigma) for sigma in [0, 1], given c = sqrt(1 - sigma^2) computed accurately by the caller:
// F(beta | 1/2) = sin(beta) R_F(cos^2 beta, 1 - sin^2(beta)/2, 1) with cos^2 beta = c, and
// sin(beta) = sqrt(1 - c) = sigma / sqrt(1 + c).
NUFDS_HD double integral_i(double sigma, double c) {
    return kSqrt2 * sigma / sqrt(1.0 + c) * carlson_rf(c, 0.5 * (1.0 + c), 1.0);
}

// Jacobi sn(y | 1/2) and cn(y | 1/2) by the AGM: a0 = 1, b0 = sqrt(1/2), c0 = sqrt(1/2);
// phi_N = 2^N a_N y, then phi_{n-1} = (phi_n + asin((c_n / a_n) sin phi_n)) / 2.
NUFDS_HD void jacobi_sn_cn_half(double y, double* sn, double* cn) {
    constexpr int kSteps = 6;
    double a[kSteps + 1], c[kSteps + 1];
    a[0] = 1.0;
    double b = 0.70710678118654752;
    c[0] = 0.70710678118654752;
    int n = 0;
    while (n < kSteps && fabs(c[n]) > 1e-17) {
        double an = a[n];
        a[n + 1] = 0.5 * (an + b);
        c[n + 1] = 0.5 * (an - b);
        b = sqrt(an * b);
        ++n;
    }
    double phi = ldexp(a[n] * y, n);
    for (int i = n; i > 0; --i) phi = 0.5 * (phi + asin(c[i] / a[i] * sin(phi)));
    *sn = sin(phi);
    *cn = cos(phi);
}

// A point of the level curve T_1(u, v) = t1 of the stretch (Eqs. 9-10, 16), at ordinate v:
// sigma_1 = u / a_v solves sqrt(a_v) I(sigma_1) = t1, i.e. cos(beta_1) = cn(t1 / sqrt(2 a_v) | 1/2).
struct LevelPoint {
    double u, v, av, au, acn, s1, s2, i2, iv1;
};

NUFDS_HD LevelPoint level_point(double v, double t1) {
    LevelPoint p;
    p.v = v;
    p.av = sqrt((1.0 - v) * (1.0 + v));
    double sn, cn;
    jacobi_sn_cn_half(t1 / (kSqrt2 * sqrt(p.av)), &sn, &cn);
    p.acn = fabs(cn);
    p.s1 = fabs(sn) * sqrt(1.0 + cn * cn);        // sqrt(1 - cn^4)
    p.u = p.av * p.s1;
    double d = p.av * p.av * (cn * cn) * (cn * cn);  // 1 - u^2 - v^2 without cancellation
    p.au = sqrt(v * v + d);                        // sqrt(1 - u^2)
    if (p.au > 0.0) {
        p.s2 = v / p.au;
        double c2 = p.av * cn * cn / p.au;          // sqrt(1 - s2^2)
        p.i2 = integral_i(p.s2, c2);
    } else {
        p.s2 = 0.0;
        p.i2 = 0.0;
    }
    p.iv1 = t1 / sqrt(p.av);
    return p;
}

// Pre-image (u, v) >= 0 of stretched direction sines (t1, t2) >= 0 under
//   (u, v) -> (sqrt(a_v) I(u / a_v), sqrt(a_u) I(v / a_u)),  a_v = sqrt(1 - v^2), a_u = sqrt(1 - u^2).
// The rim u^2 + v^2 = 1 maps onto t1^4 + t2^4 = I(1)^4, so a pre-image in the open disk
// exists exactly inside that curve.  The map is symmetric under exchange of the axes; the
// larger target is put first, so the pre-image has v <= u.  Along T_1 = t1, h(v) = T_2 - t2
// increases with v on [0, sqrt(1 - (t1 / I(1))^4)]; Newton steps are kept inside the bracket.
// dh/dv = det J / J_11 with J from Eq. 15 and its cross derivative, written so that the
// terms that grow at the rim cancel analytically.  Returns false when there is no pre-image.
NUFDS_HD bool stretch_preimage(double t1_in, double t2_in, double* u_out, double* v_out) {
    bool swap = t2_in > t1_in;
    double t1 = swap ? t2_in : t1_in;
    double t2 = swap ? t1_in : t2_in;
    double r1 = t1 / kIOne, r2 = t2 / kIOne;
    double q1 = r1 * r1, q2 = r2 * r2;
    if (q1 * q1 + q2 * q2 >= 1.0) return false;
    double vmax = sqrt(fmax(0.0, (1.0 - q1) * (1.0 + q1)));
    double v = 0.0;
    if (t2 > 0.0) {
        double lo = 0.0, hi = vmax;
        v = fmin(t2 / (1.0 + 0.25 * (t1 * t1 + t2 * t2)), vmax);
        for (int it = 0; it < 60; ++it) {
            LevelPoint p = level_point(v, t1);
            double h = sqrt(p.au) * p.i2 - t2;
            if (h == 0.0) break;
            if (h < 0.0) lo = v; else hi = v;
            double d14 = sqrt(p.av) * p.acn;
            double au32 = p.au * sqrt(p.au), av32 = p.av * sqrt(p.av);
            double dh = d14 / (p.au * p.av * p.av)
                        + (p.u * v / (2.0 * p.av)) * (p.s1 * p.i2 / au32 + p.s2 * p.iv1 / av32)
                        - p.u * v * p.iv1 * p.i2 * d14 * d14 * d14 / (4.0 * au32 * av32 * p.av);
            double vn = v - h / dh;
            if (!(vn >= lo && vn <= hi)) vn = 0.5 * (lo + hi);
            double step = fabs(vn - v);
            v = vn;
            if (step <= 4e-16 || hi - lo <= 4e-16) break;
        }
    }
    LevelPoint p = level_point(v, t1);
    double u = p.u;
    *u_out = swap ? v : u;
    *v_out = swap ? u : v;
    return true;
}

// Distorted output coordinate of Eqs. 17-18 for a true object-plane point (x, y) at distance z:
//   x' = z sqrt(a_v) I(u / a_v) with u = x / R, a_v = sqrt(1 - (y/R)^2) = sqrt(x^2 + z^2) / R,
// so u / a_v = x / sqrt(x^2 + z^2) depends on x alone and
//   x' = A(x) R^(-1/2),  A(x) = z I(x / sqrt(x^2 + z^2)) (x^2 + z^2)^(1/4),  R = sqrt(x^2 + y^2 + z^2).
NUFDS_HD double output_map_factor(double x, double z) {
    double r2 = x * x + z * z;
    double r = sqrt(r2);
    double sigma = fabs(x) / r;
    double c = z / r;  // sqrt(1 - sigma^2)
    double a = z * integral_i(sigma, c) * sqrt(r);
    return x < 0.0 ? -a : a;
}

// ---------------------------------------------------------------- the paper's polynomial model
// Sec. 4, step 1: the hypergeometric function of Eq. 16 replaced by a degree-8 polynomial fitted to
// 51 frequencies spread uniformly across the band.  Read as p(u) ~ 2F1(1/2, 3/4; 3/2; u^2) on
// u in [-s, s], used wherever Eq. 16 takes 2F1 at sigma^2, so I(sigma) becomes I_P(sigma) =
// sigma p(sigma) (extrapolated beyond the fitted range).
struct PaperPoly {
    double c[9];  // p(u) = sum_k c[k] u^k
};

// Least-squares fit of the polynomial (host): 51 samples 2F1(u^2) = I(u) / u, columns (u / s)^k
// triangularised by Householder reflections, back substitution, then rescaled to powers of u.
inline PaperPoly paper_polynomial(double s) {
    constexpr int NS = 51, ND = 9;
    double A[NS][ND], b[NS];
    for (int i = 0; i < NS; ++i) {
        const double u = -s + 2.0 * s * i / (NS - 1);
        const double au = std::fabs(u);
        b[i] = au > 0.0 ? integral_i(au, std::sqrt((1.0 - au) * (1.0 + au))) / au : 1.0;
        double x = 1.0;
        for (int k = 0; k < ND; ++k) {
            A[i][k] = x;
            x *= u / s;
        }
    }
    for (int k = 0; k < ND; ++k) {
        double norm = 0.0;
        for (int i = k; i < NS; ++i) norm += A[i][k] * A[i][k];
        norm = std::sqrt(norm);
        const double alpha = A[k][k] > 0.0 ? -norm : norm;
        double v[NS];
        for (int i = 0; i < NS; ++i) v[i] = i < k ? 0.0 : A[i][k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < NS; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        for (int j = k; j < ND; ++j) {
            double d = 0.0;
            for (int i = k; i < NS; ++i) d += v[i] * A[i][j];
            d *= 2.0 / vv;
            for (int i = k; i < NS; ++i) A[i][j] -= d * v[i];
        }
        double d = 0.0;
        for (int i = k; i < NS; ++i) d += v[i] * b[i];
        d *= 2.0 / vv;
        for (int i = k; i < NS; ++i) b[i] -= d * v[i];
    }
    double x[ND];
    for (int k = ND - 1; k >= 0; --k) {
        double r = b[k];
        for (int j = k + 1; j < ND; ++j) r -= A[k][j] * x[j];
        x[k] = r / A[k][k];
    }
    PaperPoly P;
    double scale = 1.0;
    for (int k = 0; k < ND; ++k) {
        P.c[k] = x[k] / scale;
        scale *= s;
    }
    return P;
}

// I_P(sigma) = sigma p(sigma) and its derivative p(sigma) + sigma p'(sigma) (Horner).
NUFDS_HD double paper_i(const PaperPoly& P, double sigma, double* d_out) {
    double p = P.c[8], dp = 0.0;
    for (int k = 7; k >= 0; --k) {
        dp = dp * sigma + p;
        p = p * sigma + P.c[k];
    }
    *d_out = p + sigma * dp;
    return sigma * p;
}

// Pre-image under (u, v) -> (sqrt(a_v) I_P(u / a_v), sqrt(a_u) I_P(v / a_u)) by 2-D Newton from the
// exact pre-image (the two maps differ by the fit error).  False where the exact map has no
// pre-image, or where after the fixed 12 steps the point is off the open disk or its residual is
// above 1e-10 (converged residuals are ~1e-16).
NUFDS_HD bool stretch_preimage_paper(const PaperPoly& P, double t1, double t2, double* u_out, double* v_out) {
    double u, v;
    if (!stretch_preimage(t1, t2, &u, &v)) return false;
    for (int it = 0; it < 12; ++it) {
        const double av = sqrt(fmax(1.0 - v * v, 1e-300)), au = sqrt(fmax(1.0 - u * u, 1e-300));
        const double sav = sqrt(av), sau = sqrt(au);
        const double s1 = u / av, s2 = v / au;
        double d1, d2;
        const double i1 = paper_i(P, s1, &d1), i2 = paper_i(P, s2, &d2);
        const double r1 = sav * i1 - t1, r2 = sau * i2 - t2;
        const double j11 = d1 / sav, j22 = d2 / sau;
        const double j12 = (0.5 * i1 / sav - d1 * s1 / sav) * (-v / av);
        const double j21 = (0.5 * i2 / sau - d2 * s2 / sau) * (-u / au);
        const double det = j11 * j22 - j12 * j21;
        u -= (r1 * j22 - r2 * j12) / det;
        v -= (r2 * j11 - r1 * j21) / det;
    }
    const double av = sqrt(fmax(1.0 - v * v, 1e-300)), au = sqrt(fmax(1.0 - u * u, 1e-300));
    double d;
    const double r1 = sqrt(av) * paper_i(P, u / av, &d) - t1;
    const double r2 = sqrt(au) * paper_i(P, v / au, &d) - t2;
    if (!(u * u + v * v < 1.0) || !(fabs(r1) <= 1e-10) || !(fabs(r2) <= 1e-10)) return false;
    *u_out = u;
    *v_out = v;
    return true;
}

// Eqs. 17-18 with the polynomial: A_P(x) = z I_P(x / sqrt(x^2 + z^2)) (x^2 + z^2)^(1/4).
NUFDS_HD double output_map_factor_paper(const PaperPoly& P, double x, double z) {
    const double r = sqrt(x * x + z * z);
    double d;
    return z * paper_i(P, x / r, &d) * sqrt(r);
}

}  // namespace nufds
