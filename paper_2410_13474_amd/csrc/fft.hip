// Stockham FFT pass kernel (gfx950) and its launch helpers.
#include "fft.h"

#include <cmath>
#include <utility>
#include <vector>
#include <algorithm>

namespace nufds {

// ------------------------------------------------------------ small DFTs
// X_t = sum_s x_s exp(sign 2 pi i s t / R), in registers.

template <typename R>
__device__ __forceinline__ cpx<R> rot_i(cpx<R> a, int sign) {  // a * (sign * i)
    return sign < 0 ? mul_mi(a) : mul_pi(a);
}

template <typename R>
__device__ __forceinline__ void dft2(cpx<R>& a, cpx<R>& b) {
    cpx<R> t = a - b;
    a = a + b;
    b = t;
}

template <typename R>
__device__ __forceinline__ void dft4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3, int sign) {
    cpx<R> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot_i(a1 - a3, sign);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

// SmallDft<R, RAD>::run transforms v in place; output X_t is left in v[perm(t)] (a static
// register renaming, so the larger radices need no temporaries).
template <typename R, int RAD>
struct SmallDft;

template <typename R>
struct SmallDft<R, 2> {
    __device__ static constexpr int perm(int t) { return t; }
    __device__ __forceinline__ static void run(cpx<R>* v, int) { dft2(v[0], v[1]); }
};

template <typename R>
struct SmallDft<R, 4> {
    __device__ static constexpr int perm(int t) { return t; }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) { dft4(v[0], v[1], v[2], v[3], sign); }
};

template <typename R>
struct SmallDft<R, 3> {
    __device__ static constexpr int perm(int t) { return t; }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) {
        const R c = R(-0.5);
        const R s = R(0.86602540378443864676) * R(sign);
        cpx<R> t = v[1] + v[2];
        cpx<R> d = v[1] - v[2];
        cpx<R> m = v[0] + t * c;
        cpx<R> j = mk(-d.y * s, d.x * s);  // i * s * d
        v[0] = v[0] + t;
        v[1] = m + j;
        v[2] = m - j;
    }
};

template <typename R>
struct SmallDft<R, 5> {
    __device__ static constexpr int perm(int t) { return t; }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) {
        const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
        const R s1 = R(0.95105651629515357212) * R(sign), s2 = R(0.58778525229247312917) * R(sign);
        cpx<R> t1 = v[1] + v[4], t2 = v[2] + v[3];
        cpx<R> d1 = v[1] - v[4], d2 = v[2] - v[3];
        cpx<R> a = v[0] + t1 * c1 + t2 * c2;
        cpx<R> b = v[0] + t1 * c2 + t2 * c1;
        cpx<R> p = d1 * s1 + d2 * s2;   // times i below
        cpx<R> q = d1 * s2 - d2 * s1;
        cpx<R> ip = mk(-p.y, p.x), iq = mk(-q.y, q.x);
        v[0] = v[0] + t1 + t2;
        v[1] = a + ip;
        v[4] = a - ip;
        v[2] = b + iq;
        v[3] = b - iq;
    }
};

template <typename R>
struct SmallDft<R, 8> {
    // evens and odds transformed in place at v[0,2,4,6] and v[1,3,5,7]; X_k at v[2k], X_(k+4) at v[2k+1]
    __device__ static constexpr int perm(int t) { return t < 4 ? 2 * t : 2 * (t - 4) + 1; }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) {
        dft4(v[0], v[2], v[4], v[6], sign);
        dft4(v[1], v[3], v[5], v[7], sign);
        const R h = R(0.70710678118654752440);
        // w8^1 = h (1 + sign i), w8^2 = sign i, w8^3 = h (-1 + sign i)
        v[3] = (v[3] + rot_i(v[3], sign)) * h;
        v[5] = rot_i(v[5], sign);
        v[7] = (rot_i(v[7], sign) - v[7]) * h;
        dft2(v[0], v[1]);
        dft2(v[2], v[3]);
        dft2(v[4], v[5]);
        dft2(v[6], v[7]);
    }
};

template <typename R>
struct SmallDft<R, 16> {
    // n = n2 + 4 n1, k = k1 + 4 k2: 4-point DFTs over n1 in place (y[n2][k1] at v[n2 + 4 k1]),
    // twiddle w16^(n2 k1), 4-point DFTs over n2 in place; X_(k1 + 4 k2) ends in v[4 k1 + k2].
    __device__ static constexpr int perm(int t) { return 4 * (t & 3) + (t >> 2); }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) {
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12], sign);
        const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173) * R(sign);
        const R h = R(0.70710678118654752440), hs = h * R(sign);
        const cpx<R> w1 = mk(c1, s1), w2 = mk(h, hs), w3 = mk(s1 * R(sign), c1 * R(sign));
        v[1 + 4] = v[1 + 4] * w1;
        v[1 + 8] = v[1 + 8] * w2;
        v[1 + 12] = v[1 + 12] * w3;
        v[2 + 4] = v[2 + 4] * w2;
        v[2 + 8] = rot_i(v[2 + 8], sign);
        v[2 + 12] = v[2 + 12] * mk(-h, hs);
        v[3 + 4] = v[3 + 4] * w3;
        v[3 + 8] = v[3 + 8] * mk(-h, hs);
        v[3 + 12] = v[3 + 12] * mk(-c1, -s1);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3], sign);
    }
};

// ---- composite radices R = A B built in registers from the small DFTs above.
// Compile-time twiddles: cos / sin of 2 pi m / R by an octant reduction and a Taylor series
// (|x| <= pi / 4, 12 terms: below double rounding).
constexpr double kTwoPi = 6.28318530717958647692;

constexpr double taylor_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 12; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double taylor_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 12; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

// cos and sin of 2 pi m / R
constexpr double turn_cos(int m, int R) {
    const int mm = ((m % R) + R) % R;
    const double f = (double)mm / (double)R;
    const int q = (int)(4.0 * f + 0.5);
    const double x = kTwoPi * (f - 0.25 * q);
    return (q % 4 == 0) ? taylor_cos(x) : (q % 4 == 1) ? -taylor_sin(x) : (q % 4 == 2) ? -taylor_cos(x) : taylor_sin(x);
}
constexpr double turn_sin(int m, int R) {
    const int mm = ((m % R) + R) % R;
    const double f = (double)mm / (double)R;
    const int q = (int)(4.0 * f + 0.5);
    const double x = kTwoPi * (f - 0.25 * q);
    return (q % 4 == 0) ? taylor_sin(x) : (q % 4 == 1) ? taylor_cos(x) : (q % 4 == 2) ? -taylor_sin(x) : -taylor_cos(x);
}

template <int M, int R>
struct TwC {
    static constexpr double c = turn_cos(M, R);
    static constexpr double s = turn_sin(M, R);
};

// R = A B with n = n2 + B n1, k = k1 + A k2: A-point DFTs over n1 in place (y[n2][k1] at v[n2 + B k1]),
// twiddle w_R^(n2 k1), B-point DFTs over n2 in place; X_(k1 + A k2) ends in v[B k1 + k2].  The
// sub-DFTs' outputs are taken back in natural order through their own perm.
template <typename R, int A, int B>
struct Composite {
    static constexpr int RAD = A * B;
    __device__ static constexpr int perm(int t) { return B * (t % A) + t / A; }

    template <int N2, int K1>
    __device__ __forceinline__ static void twiddle(cpx<R>* v, int sign) {
        constexpr int M = (N2 * K1) % RAD;
        cpx<R>& x = v[N2 + B * K1];
        if constexpr (M == 0) {
        } else if constexpr (4 * M == RAD) {          // exp(sign i pi / 2) = sign i
            x = sign < 0 ? mul_mi(x) : mul_pi(x);
        } else if constexpr (2 * M == RAD) {          // -1
            x = mk(-x.x, -x.y);
        } else if constexpr (4 * M == 3 * RAD) {      // -sign i
            x = sign < 0 ? mul_pi(x) : mul_mi(x);
        } else {
            const R c = R(TwC<N2 * K1, RAD>::c);
            const R s = R(TwC<N2 * K1, RAD>::s) * R(sign);
            x = x * mk(c, s);
        }
    }
    template <int N2>
    __device__ __forceinline__ static void inner(cpx<R>* v, int sign) {
        cpx<R> t[A];
#pragma unroll
        for (int i = 0; i < A; ++i) t[i] = v[N2 + B * i];
        SmallDft<R, A>::run(t, sign);
#pragma unroll
        for (int i = 0; i < A; ++i) v[N2 + B * i] = t[SmallDft<R, A>::perm(i)];
        twiddle_row<N2>(v, sign, std::make_integer_sequence<int, A>{});
    }
    template <int N2, int... K1>
    __device__ __forceinline__ static void twiddle_row(cpx<R>* v, int sign, std::integer_sequence<int, K1...>) {
        (twiddle<N2, K1>(v, sign), ...);
    }
    template <int... N2>
    __device__ __forceinline__ static void inners(cpx<R>* v, int sign, std::integer_sequence<int, N2...>) {
        (inner<N2>(v, sign), ...);
    }
    __device__ __forceinline__ static void run(cpx<R>* v, int sign) {
        inners(v, sign, std::make_integer_sequence<int, B>{});
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            cpx<R> t[B];
#pragma unroll
            for (int i = 0; i < B; ++i) t[i] = v[B * k1 + i];
            SmallDft<R, B>::run(t, sign);
#pragma unroll
            for (int i = 0; i < B; ++i) v[B * k1 + i] = t[SmallDft<R, B>::perm(i)];
        }
    }
};

template <typename R> struct SmallDft<R, 6> : Composite<R, 3, 2> {};
template <typename R> struct SmallDft<R, 9> : Composite<R, 3, 3> {};
template <typename R> struct SmallDft<R, 10> : Composite<R, 5, 2> {};
template <typename R> struct SmallDft<R, 12> : Composite<R, 4, 3> {};
template <typename R> struct SmallDft<R, 15> : Composite<R, 5, 3> {};
template <typename R> struct SmallDft<R, 25> : Composite<R, 5, 5> {};  // one-pass row chains only
template <typename R> struct SmallDft<R, 32> : Composite<R, 16, 2> {};

// q = j / n for 0 <= j < 2^24 through a float reciprocal, corrected to exact.
__device__ __forceinline__ int fdiv(int j, int n, float inv) {
    int q = (int)((float)j * inv);
    int r = j - q * n;
    if (r >= n) { ++q; r -= n; }
    if (r < 0) { --q; }
    return q;
}

// Powers w^1 .. w^(RAD-1) by a balanced product tree (w^t = w^(t/2) w^(t - t/2)): one table load
// per butterfly, and every power is at most ~log2(RAD) rounded products away from the table value.
template <typename R, int RAD>
__device__ __forceinline__ void twiddle_powers(cpx<R> w, cpx<R>* wp) {
    wp[1] = w;
#pragma unroll
    for (int t = 2; t < RAD; ++t) wp[t] = wp[t / 2] * wp[t - t / 2];
}

// v[t] *= w^t for t = 1 .. RAD-1.  Up to radix 8 the powers come from a product tree; above,
// w^t = (w^4)^(t/4) w^(t%4), which keeps 4 + ceil(RAD/4) values live instead of RAD (a few
// more roundings, ~1e-6 in float32, ~1e-15 in float64).
template <typename R, int RAD>
__device__ __forceinline__ void apply_twiddles(cpx<R>* v, cpx<R> w) {
    if constexpr (RAD <= 8) {
        cpx<R> wp[RAD];
        twiddle_powers<R, RAD>(w, wp);
#pragma unroll
        for (int t = 1; t < RAD; ++t) v[t] = v[t] * wp[t];
    } else {
        cpx<R> lo[4];
        lo[0] = mk(R(1), R(0));
        lo[1] = w;
        lo[2] = w * w;
        lo[3] = lo[2] * w;
        const cpx<R> w4 = lo[2] * lo[2];
        cpx<R> hi = mk(R(1), R(0));
#pragma unroll
        for (int t = 1; t < RAD; ++t) {
            if (t % 4 == 0) hi = (t == 4) ? w4 : hi * w4;
            // below t = 4 hi is 1: no product with it (x * 0 does not fold in IEEE arithmetic)
            v[t] = v[t] * (t < 4 ? lo[t] : ((t % 4) ? hi * lo[t % 4] : hi));
        }
    }
}

// Affine description of one tile: element (n, w) lives at base + n sn + w sw; its index along the
// transformed axis is n an + w aw + a0 (input) or k bn + w bw + b0 (output); the chain multiply of a
// fused pass reads the vector at n cn + w cw + c0; the transverse index is t0 + w t1; the four-step
// twiddle exponent of the store is (m0 + w m1) k.
__host__ __device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

struct TileMap {
    int ib, isn, isw, ob, osn, osw;  // element offsets: every array holds fewer than 2^31 elements
    int an, aw, a0, bn, bw, b0, cn, cw, c0, t0, t1, m0, m1;
    int wvalid;
    bool in_nfast, out_nfast, twiddle;
};

__host__ __device__ __forceinline__ TileMap tile_map(const PassDesc& d, int a, int b) {
    TileMap m;
    const int W = d.W;
    m.twiddle = false;
    m.m0 = m.m1 = 0;
    m.cn = 1; m.cw = 0; m.c0 = 0;
    switch (d.kind) {
        case K_ROW1: {
            int r0 = a * W;
            m.wvalid = imin(W, d.rows - r0);
            m.ib = r0 * (int)d.in_pitch; m.isn = 1; m.isw = (int)d.in_pitch;
            m.ob = r0 * (int)d.out_pitch; m.osn = 1; m.osw = (int)d.out_pitch;
            m.an = 1; m.aw = 0; m.a0 = 0; m.bn = 1; m.bw = 0; m.b0 = 0; m.t0 = r0; m.t1 = 1;
            m.in_nfast = m.out_nfast = true;
            break;
        }
        case K_COL1: {
            int c0 = b * W;
            m.wvalid = imin(W, d.cols - c0);
            m.ib = c0; m.isn = (int)d.in_pitch; m.isw = 1;
            m.ob = c0; m.osn = (int)d.out_pitch; m.osw = 1;
            m.an = 1; m.aw = 0; m.a0 = 0; m.bn = 1; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_ROWA: {
            int row = a, n20 = b * W;
            m.wvalid = imin(W, d.L2 - n20);
            m.ib = row * (int)d.in_pitch + n20; m.isn = d.L2; m.isw = 1;
            m.ob = row * (int)d.out_pitch + n20; m.osn = d.L2; m.osw = 1;
            m.an = d.L2; m.aw = 1; m.a0 = n20; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = row; m.t1 = 0;
            m.twiddle = true; m.m0 = n20; m.m1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_ROWB: {
            int row = a, k10 = b * W;
            m.wvalid = imin(W, d.L1 - k10);
            m.ib = row * (int)d.in_pitch + k10 * d.L2; m.isn = 1; m.isw = d.L2;
            m.ob = row * (int)d.out_pitch + k10; m.osn = d.L1; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = d.L1; m.bw = 1; m.b0 = k10; m.t0 = row; m.t1 = 0;
            m.in_nfast = true; m.out_nfast = false;
            break;
        }
        case K_ROWBA: {
            // input as ROWB (k1 = k10 + w, n over k2); output position q1 L1 + k1 with twiddle w^(k1 q1)
            int row = a, k10 = b * W;
            m.wvalid = imin(W, d.L1 - k10);
            m.ib = row * (int)d.in_pitch + k10 * d.L2; m.isn = 1; m.isw = d.L2;
            m.ob = row * (int)d.out_pitch + k10; m.osn = d.L1; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = row; m.t1 = 0;
            m.cn = d.L1; m.cw = 1; m.c0 = k10;
            m.twiddle = true; m.m0 = k10; m.m1 = 1;
            m.in_nfast = true; m.out_nfast = false;
            break;
        }
        case K_COLA: {
            int n2 = a, c0 = b * W;
            m.wvalid = imin(W, d.cols - c0);
            m.ib = n2 * (int)d.in_pitch + c0; m.isn = d.L2 * (int)d.in_pitch; m.isw = 1;
            m.ob = n2 * (int)d.out_pitch + c0; m.osn = d.L2 * (int)d.out_pitch; m.osw = 1;
            m.an = d.L2; m.aw = 0; m.a0 = n2; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.twiddle = true; m.m0 = n2; m.m1 = 0;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_COLB: {
            int k1 = a, c0 = b * W;
            m.wvalid = imin(W, d.cols - c0);
            m.ib = k1 * d.L2 * (int)d.in_pitch + c0; m.isn = (int)d.in_pitch; m.isw = 1;
            m.ob = k1 * (int)d.out_pitch + c0; m.osn = d.L1 * (int)d.out_pitch; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = d.L1; m.bw = 0; m.b0 = k1; m.t0 = c0; m.t1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        default: {  // K_COLBA: input as COLB, output row q1 L1 + k1 with twiddle w^(k1 q1)
            int k1 = a, c0 = b * W;
            m.wvalid = imin(W, d.cols - c0);
            m.ib = k1 * d.L2 * (int)d.in_pitch + c0; m.isn = (int)d.in_pitch; m.isw = 1;
            m.ob = k1 * (int)d.out_pitch + c0; m.osn = d.L1 * (int)d.out_pitch; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.cn = d.L1; m.cw = 0; m.c0 = k1;
            m.twiddle = true; m.m0 = k1; m.m1 = 0;
            m.in_nfast = m.out_nfast = false;
            break;
        }
    }
    return m;
}

// Global accesses as a wave-uniform base plus a 32-bit per-lane byte offset.  The base is pinned to
// scalar registers (it is uniform; the read-first-lane only tells the compiler so), which gives the
// scalar-base form of the load and store: one address register per lane, shared by every element
// of a butterfly, instead of a 64-bit address per element.
typedef __attribute__((address_space(1))) char gbyte;

template <typename T>
__device__ __forceinline__ gbyte* uniform_base(const T* p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (gbyte*)(((uint64_t)hi << 32) | lo);
}
template <typename R>
using vec2 = R __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ cpx<R> load_at(gbyte* base, uint32_t off) {
    const vec2<R> v = *reinterpret_cast<const vec2<R> __attribute__((address_space(1)))*>(base + off);
    return mk(R(v.x), R(v.y));
}
template <typename R>
__device__ __forceinline__ void store_at(gbyte* base, uint32_t off, cpx<R> v) {
    vec2<R> w;
    w.x = v.x;
    w.y = v.y;
    *reinterpret_cast<vec2<R> __attribute__((address_space(1)))*>(base + off) = w;
}

// Butterflies a thread holds in one stage of radix RAD (the host sizes its thread count by the same rule).
template <int RAD, int MAXE, int NBMAX>
struct StageNb {
    static constexpr int a = MAXE / RAD < NBMAX ? MAXE / RAD : NBMAX;
    static constexpr int value = a < kMaxBfly ? a : kMaxBfly;
};

// One Stockham stage of radix RAD (Govindaraju et al., SC 2008 formulation): butterfly j reads
// x[j + t L/RAD], twiddles by w_(Ns RAD)^(t k), k = j mod Ns, and writes (j / Ns) Ns RAD + k + t Ns.
// The first stage of a pass reads its inputs from global memory and the last stage writes its
// outputs to global memory (with the four-step twiddle of A passes), so the tile crosses LDS only
// between stages.  Element n = j + t L/RAD of lane (j, w) sits at a wave-uniform base (tile origin plus
// t L/RAD rows) plus a per-lane offset that is the same for every t.  Threads take butterflies in the
// order that makes their global accesses contiguous (j fastest for transforms that run along memory,
// w fastest for tiles of adjacent columns).  Reads of a stage all happen before the barrier that
// precedes its LDS writes; every branch-free read uses a clamped in-bounds offset.
template <typename R, int RAD, int MAXE, int NBMAX, bool PAD, bool FIRST, bool LAST, bool CHAIN, int SGN, int LC = 0,
          int NSC = 0, int WLOG = -1, bool WIN = false>
__device__ __forceinline__ void fft_stage(cpx<R>* lds, const PassDesc& d, const TileMap& m, const LoadPlain<R>& ld,
                                          const StorePlain<R>& st, const ChainMul<R>& ch,
                                          const cpx<R>* __restrict__ tw, const cpx<R>* __restrict__ twf, int Ns,
                                          int tid, int T) {
    constexpr int sign = SGN;  // transform direction, a compile-time constant of the stage
    constexpr int NB = StageNb<RAD, MAXE, NBMAX>::value;
    constexpr uint32_t ES = sizeof(cpx<R>);
    // per-stage opaque copy of the thread index: keeps the compiler from hoisting every
    // butterfly's addresses out of the stage loop (they would stay live across all stages)
    int tid_s = tid;
    asm volatile("" : "+v"(tid_s));
    // the same for the tile origins and the length, which would otherwise pin every stage's
    // global bases and loop bounds in scalar registers for the whole kernel
    int ib_s = __builtin_amdgcn_readfirstlane(m.ib), ob_s = __builtin_amdgcn_readfirstlane(m.ob);
    int L = __builtin_amdgcn_readfirstlane(d.L);
    asm volatile("" : "+s"(ib_s), "+s"(ob_s), "+s"(L));
    // kernels specialised for one radix plan know the length, the stride and the tile width
    if constexpr (LC > 0) L = LC;
    if constexpr (NSC > 0) Ns = NSC;
    const int lw = WLOG >= 0 ? WLOG : d.logW, W = 1 << lw;
    const int LR = L / RAD;
    const int B = LR << lw;
    // the first stage has Ns = 1 (q = j, k = 0), the last Ns = L / RAD (q = 0, k = j)
    const int tstride = (FIRST || LAST) ? 1 : L / (Ns * RAD);
    const float invNs = (FIRST || LAST) ? 1.0f : __builtin_amdgcn_rcpf((float)Ns);  // fdiv corrects the last bit
    const float invLR = __builtin_amdgcn_rcpf((float)LR);
    const bool jfast = FIRST ? m.in_nfast : (LAST ? m.out_nfast : (W == 1));
    cpx<R> v[NB][RAD];
    cpx<R> cw[NB];
    cpx<R> c4a[NB], c4b[NB];
    cpx<R> cv[CHAIN ? NB : 1][CHAIN ? RAD : 1];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b0 = tid_s + i * T;
        const int b = b0 < B ? b0 : 0;
        int j, w;
        if (jfast) { w = fdiv(b, LR, invLR); j = b - w * LR; }
        else { w = b & (W - 1); j = b >> lw; }
        const int q = FIRST ? j : (LAST ? 0 : fdiv(j, Ns, invNs));
        const int k = FIRST ? 0 : (LAST ? j : j - q * Ns);
        if (!FIRST) cw[i] = load_at<R>(uniform_base(tw), (uint32_t)(k * tstride) * ES);
        if (FIRST) {
            const bool valid = b0 < B && w < m.wvalid;
            const uint32_t lo = valid ? (uint32_t)(j * m.isn + w * m.isw) * ES : 0u;
            if constexpr (WIN) {
                // index along the axis of the element each lane reads (padding lanes read their
                // tile's first element, whose index this is too)
                const int ax0 = valid ? j * m.an + w * m.aw + m.a0 : m.a0;
#pragma unroll
                for (int t = 0; t < RAD; ++t) {
                    const int ix = ax0 + t * LR * m.an;
                    v[i][t] = mk(R(0), R(0));
                    if (ix >= ld.win_lo && ix < ld.win_hi)
                        v[i][t] = load_at<R>(uniform_base(ld.in + ((int64_t)ib_s + (int64_t)(t * LR) * m.isn)), lo);
                }
            } else {
#pragma unroll
                for (int t = 0; t < RAD; ++t)
                    v[i][t] = load_at<R>(uniform_base(ld.in + ((int64_t)ib_s + (int64_t)(t * LR) * m.isn)), lo);
            }
        } else {
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[i][t] = lds[lds_index<PAD>(((j + t * LR) << lw) + w)];
        }
        if (CHAIN) {
            // last stage of the first transform of a chain pass: outputs sit at natural positions
            // pos = j + t LR; fetch the chain vector at pos cn + w cw + c0 now, so the loads overlap
            // the barrier and the butterfly
            // (the vector is short: one scalar base, 32-bit offsets)
            const int c = j * m.cn + (w < m.wvalid ? w : 0) * m.cw + m.c0;
#pragma unroll
            for (int t = 0; t < RAD; ++t)
                cv[i][t] = load_at<R>(uniform_base(ch.vec), (uint32_t)(c + t * LR * m.cn) * ES);
        }
        if (LAST && m.twiddle) {
            // outputs sit at pos = j + t LR (Ns = LR in the last stage); the four-step twiddle
            // w_Lf^(e pos) = w^(e j) (w^(e LR))^t with e = m0 + w m1; e pos < Lf never wraps
            const int e = (w < m.wvalid) ? m.m0 + w * m.m1 : 0;
            c4a[i] = load_at<R>(uniform_base(twf), (uint32_t)(e * j) * ES);
            c4b[i] = load_at<R>(uniform_base(twf), (uint32_t)(e * LR) * ES);
        }
    }
    if (!FIRST && !LAST) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid_s + i * T;
        if (b < B) {
            int j, w;
            if (jfast) { w = fdiv(b, LR, invLR); j = b - w * LR; }
            else { w = b & (W - 1); j = b >> lw; }
            const int q = FIRST ? j : (LAST ? 0 : fdiv(j, Ns, invNs));
            const int k = FIRST ? 0 : (LAST ? j : j - q * Ns);
            if (FIRST) {
                // fused load work: conjugation, (-1)^(axis index) centring, scale (padding lanes
                // hold finite values of valid rows; their transforms are never stored)
                if (!ld.plain) {
                    // index along the axis (padding lanes of a partial tile take their tile's first)
                    const int ax0 = j * m.an + (w < m.wvalid ? w : 0) * m.aw + m.a0;
                    const int par = ax0 & 1;
#pragma unroll
                    for (int t = 0; t < RAD; ++t) {
                        const bool flip = ld.sign_axis && ((par + t * LR * m.an) & 1);
                        const R f = flip ? -ld.scale : ld.scale;
                        v[i][t] = mk(v[i][t].x * f, (ld.conj ? -v[i][t].y : v[i][t].y) * f);
                    }
                    if (ld.mul) {
#pragma unroll
                        for (int t = 0; t < RAD; ++t)
                            v[i][t] = v[i][t] * load_at<R>(uniform_base(ld.mul), (uint32_t)(ax0 + t * LR * m.an) * ES);
                    }
                }
            } else {
                cpx<R> c = cw[i];
                if (sign > 0) c.y = -c.y;
                if (sizeof(R) == 4) {
                    apply_twiddles<R, RAD>(v[i], c);
                } else {
                    // float64: a running product (<= RAD - 2 roundings, ~1e-15) keeps registers free
                    cpx<R> p = c;
#pragma unroll
                    for (int t = 1; t < RAD; ++t) {
                        v[i][t] = v[i][t] * p;
                        if (t + 1 < RAD) p = p * c;
                    }
                }
            }
            SmallDft<R, RAD>::run(v[i], sign);
            if (LAST) {
                // pos = j + t LR
                if (w < m.wvalid) {
                    cpx<R> tf = mk(R(1), R(0)), step = mk(R(1), R(0));
                    if (m.twiddle) {
                        tf = c4a[i];
                        step = c4b[i];
                        if (sign > 0) {
                            tf.y = -tf.y;
                            step.y = -step.y;
                        }
                    }
                    const uint32_t lo = (uint32_t)(j * m.osn + w * m.osw) * ES;
                    if (!st.plain) {
                        const int par = (j * m.bn + w * m.bw + m.b0) & 1;
#pragma unroll
                        for (int t = 0; t < RAD; ++t) {
                            const bool flip = st.sign_axis && ((par + t * LR * m.bn) & 1);
                            const R f = flip ? -st.scale : st.scale;
                            v[i][SmallDft<R, RAD>::perm(t)] = v[i][SmallDft<R, RAD>::perm(t)] * f;
                        }
                    }
#pragma unroll
                    for (int t = 0; t < RAD; ++t) {
                        store_at<R>(uniform_base(st.out + ((int64_t)ob_s + (int64_t)(t * LR) * m.osn)), lo,
                                 m.twiddle ? v[i][SmallDft<R, RAD>::perm(t)] * tf : v[i][SmallDft<R, RAD>::perm(t)]);
                        if (m.twiddle) tf = tf * step;
                    }
                }
            } else if (CHAIN) {
#pragma unroll
                for (int t = 0; t < RAD; ++t)
                    lds[lds_index<PAD>(((j + t * LR) << lw) + w)] = v[i][SmallDft<R, RAD>::perm(t)] * cv[i][t];
            } else {
                const int base = q * Ns * RAD + k;
#pragma unroll
                for (int t = 0; t < RAD; ++t)
                    lds[lds_index<PAD>(((base + t * Ns) << lw) + w)] = v[i][SmallDft<R, RAD>::perm(t)];
            }
        }
    }
    if (!LAST) __syncthreads();
}

template <typename R, int MAXE, int NBMAX, bool PAD, bool FIRST, bool LAST, bool CHAIN, int SGN, bool WIN = false>
__device__ __forceinline__ void fft_stage_r(int r, cpx<R>* lds, const PassDesc& d, const TileMap& m,
                                            const LoadPlain<R>& ld, const StorePlain<R>& st, const ChainMul<R>& ch,
                                            const cpx<R>* __restrict__ tw, const cpx<R>* __restrict__ twf, int Ns,
                                            int tid, int T) {
#define NUFDS_STAGE(RR)                                                                             \
    if constexpr ((RR) <= MAXE)                                                                     \
        fft_stage<R, RR, MAXE, NBMAX, PAD, FIRST, LAST, CHAIN, SGN, 0, 0, -1, WIN>(lds, d, m, ld, st, ch, tw, twf, Ns, \
                                                                                 tid, T)
    switch (r) {
        case 16: NUFDS_STAGE(16); break;
        case 8: NUFDS_STAGE(8); break;
        case 4: NUFDS_STAGE(4); break;
        case 2: NUFDS_STAGE(2); break;
        case 5: NUFDS_STAGE(5); break;
        case 3: NUFDS_STAGE(3); break;
        case 6: NUFDS_STAGE(6); break;
        case 9: NUFDS_STAGE(9); break;
        case 10: NUFDS_STAGE(10); break;
        case 12: NUFDS_STAGE(12); break;
        default: NUFDS_STAGE(15); break;
    }
#undef NUFDS_STAGE
}

// NBMAX: butterflies a thread holds per stage.  NBMAX = 1 is the small-tile variant (one butterfly
// per thread, more threads, fewer live registers); the other variant serves long single-pass rows.
// WIN: the first stage reads through the load window of LoadPlain (non-chain passes only).
template <typename R, int MAXE, int NBMAX, int MAXT, bool CHAINP, bool PAD, int SGN, bool WIN = false>
__global__ void __launch_bounds__(MAXT) fft_pass_kernel(PassDesc d, LoadPlain<R> ld, StorePlain<R> st,
                                                        const cpx<R>* __restrict__ tw,
                                                        const cpx<R>* __restrict__ twf,
                                                        const cpx<R>* __restrict__ chainvec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x, T = blockDim.x;
    int ta = blockIdx.y, tb = blockIdx.x;
    if (d.xcd_rows) {
        // workgroups are dispatched round-robin over the XCDs: give each XCD a contiguous range of
        // tile rows so that neighbouring rows (which gather from neighbouring spectrum rows) share
        // one L2
        // (the grid has kXcds * per rows, per = ceil(tiles_a / kXcds), so every XCD owns exactly
        // per * nb workgroup slots; rows past tiles_a return at once)
        const int nb = gridDim.x, na = d.tiles_a;
        const int lin = blockIdx.y * nb + blockIdx.x;
        const int xcd = lin % kXcds, slot = lin / kXcds;
        const int per = (na + kXcds - 1) / kXcds;   // rows per XCD
        const int row = xcd * per + slot / nb;
        if (row >= na) return;
        ta = row;
        tb = slot % nb;
    }
    const TileMap m = tile_map(d, ta, tb);
    const int nst = d.nst;

    const ChainMul<R> ch{chainvec};

    // transform 1: stage 0 reads global memory; the last stage writes global memory, or, in a chain
    // pass, multiplies by the chain vector (the chirp of Eq. 2) on its way to LDS
    int Ns = 1;
#define NUFDS_RUN(F, L, C) \
    fft_stage_r<R, MAXE, NBMAX, PAD, F, L, C, SGN, WIN && !CHAINP>(r, lds, d, m, ld, st, ch, tw, twf, Ns, tid, T)
    if constexpr (!CHAINP) {
        for (int s = 0; s < nst; ++s) {
            const int r = d.rad[s];
            const bool first = s == 0, last = s == nst - 1;
            if (first && last) NUFDS_RUN(true, true, false);
            else if (first) NUFDS_RUN(true, false, false);
            else if (last) NUFDS_RUN(false, true, false);
            else NUFDS_RUN(false, false, false);
            Ns *= r;
        }
        return;
    } else {
    for (int s = 0; s < nst; ++s) {
        const int r = d.rad[s];
        const bool first = s == 0, last = s == nst - 1;
        if (first && last) NUFDS_RUN(true, false, true);
        else if (first) NUFDS_RUN(true, false, false);
        else if (last) NUFDS_RUN(false, false, true);
        else NUFDS_RUN(false, false, false);
        Ns *= r;
    }
#undef NUFDS_RUN
    // transform 2 (opposite sign): from LDS, the last stage to global memory
    Ns = 1;
    for (int s = 0; s < nst; ++s) {
        const int r = d.rad[s];
        if (s == nst - 1)
            fft_stage_r<R, MAXE, NBMAX, PAD, false, true, false, -SGN>(r, lds, d, m, ld, st, ch, tw, twf, Ns, tid, T);
        else
            fft_stage_r<R, MAXE, NBMAX, PAD, false, false, false, -SGN>(r, lds, d, m, ld, st, ch, tw, twf, Ns, tid, T);
        Ns *= r;
    }
    }
}

// The stages of one transform with its radix plan known at compile time (Ns, the length and the
// tile width become constants).  G_IN: the first stage reads global memory; G_OUT: the last stage
// writes global memory; CH: the last stage applies the chain vector on its way to LDS.
template <typename R, int MAXE, int NBMAX, bool PAD, bool G_IN, bool G_OUT, bool CH, int SGN, int LC, int WLOG,
          int NS, int R0, int... RS>
__device__ __forceinline__ void fixed_stages(cpx<R>* lds, const PassDesc& d, const TileMap& m, const LoadPlain<R>& ld,
                                             const StorePlain<R>& st, const ChainMul<R>& ch,
                                             const cpx<R>* __restrict__ tw, const cpx<R>* __restrict__ twf, int tid,
                                             int T) {
    constexpr bool last = sizeof...(RS) == 0;
    fft_stage<R, R0, MAXE, NBMAX, PAD, G_IN && NS == 1, last && G_OUT, last && CH, SGN, LC, NS, WLOG>(
        lds, d, m, ld, st, ch, tw, twf, NS, tid, T);
    if constexpr (!last)
        fixed_stages<R, MAXE, NBMAX, PAD, G_IN, G_OUT, CH, SGN, LC, WLOG, NS * R0, RS...>(lds, d, m, ld, st, ch, tw,
                                                                                         twf, tid, T);
}

// fft_pass_kernel for one radix plan (RADS, product LC) and tile width 2^WLOG.
template <typename R, int MAXE, int NBMAX, int MAXT, bool CHAINP, bool PAD, int SGN, int WLOG, int... RADS>
__global__ void __launch_bounds__(MAXT) fft_fixed_kernel(PassDesc d, LoadPlain<R> ld, StorePlain<R> st,
                                                         const cpx<R>* __restrict__ tw,
                                                         const cpx<R>* __restrict__ twf,
                                                         const cpx<R>* __restrict__ chainvec) {
    constexpr int LC = (RADS * ...);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tid = threadIdx.x, T = blockDim.x;
    int ta = blockIdx.y, tb = blockIdx.x;
    if (d.xcd_rows) {
        const int nb = gridDim.x, na = d.tiles_a;
        const int lin = blockIdx.y * nb + blockIdx.x;
        const int xcd = lin % kXcds, slot = lin / kXcds;
        const int per = (na + kXcds - 1) / kXcds;
        const int row = xcd * per + slot / nb;
        if (row >= na) return;
        ta = row;
        tb = slot % nb;
    }
    const TileMap m = tile_map(d, ta, tb);
    const ChainMul<R> ch{chainvec};
    if constexpr (!CHAINP) {
        fixed_stages<R, MAXE, NBMAX, PAD, true, true, false, SGN, LC, WLOG, 1, RADS...>(lds, d, m, ld, st, ch, tw, twf,
                                                                                      tid, T);
    } else {
        fixed_stages<R, MAXE, NBMAX, PAD, true, false, true, SGN, LC, WLOG, 1, RADS...>(lds, d, m, ld, st, ch, tw, twf,
                                                                                      tid, T);
        fixed_stages<R, MAXE, NBMAX, PAD, false, true, false, -SGN, LC, WLOG, 1, RADS...>(lds, d, m, ld, st, ch, tw,
                                                                                        twf, tid, T);
    }
}

template <typename R, int MAXE, int NBMAX, int MAXT, bool CHAINP, bool PAD, int SGN, int WLOG, int... RADS>
static hipError_t launch_fixed(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                               const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s) {
    static bool attr_set = false;
    auto kern = &fft_fixed_kernel<R, MAXE, NBMAX, MAXT, CHAINP, PAD, SGN, WLOG, RADS...>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t shm = (size_t)lds_elems(d.L * d.W) * sizeof(cpx<R>);
    const int ga = d.xcd_rows ? kXcds * ((d.tiles_a + kXcds - 1) / kXcds) : d.tiles_a;
    dim3 grid(d.tiles_b, ga), block(d.nthreads);
    hipLaunchKernelGGL(kern, grid, block, shm, s, d, ld, st, tw, twf, chainvec);
    return hipGetLastError();
}

// Radix plans with a specialised kernel: the transforms of the common sizes (lengths 128 and 160,
// the halves of 16384 and 25600, over tiles of 8-32 columns; 16384 in one pass).
template <typename R, int SG>
static bool launch_specialised(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                               const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s, hipError_t* err) {
    constexpr int OE = OneBflyElems<R>::value, OT = OneBflyThreads<R>::value, ME = MaxElems<R>::value;
    auto is = [&](int L, int W, int n, int r0, int r1, int r2, int r3) {
        return d.L == L && d.W == W && d.nst == n && d.rad[0] == r0 && d.rad[1] == r1 && (n < 3 || d.rad[2] == r2) &&
               (n < 4 || d.rad[3] == r3);
    };
#define NUFDS_FIX2(LL, WW, WL, A, B)                                                                            \
    if (d.one_bfly && is(LL, WW, 2, A, B, 0, 0)) {                                                              \
        *err = d.chain ? launch_fixed<R, OE, 1, OT, true, (WW < 8), SG, WL, A, B>(d, ld, st, tw, twf, chainvec, s)  \
                       : launch_fixed<R, OE, 1, OT, false, (WW < 8), SG, WL, A, B>(d, ld, st, tw, twf, chainvec, s); \
        return true;                                                                                            \
    }
    NUFDS_FIX2(160, 32, 5, 16, 10)
    NUFDS_FIX2(160, 16, 4, 16, 10)
    NUFDS_FIX2(160, 8, 3, 16, 10)
    NUFDS_FIX2(128, 32, 5, 16, 8)
    NUFDS_FIX2(128, 16, 4, 16, 8)
    NUFDS_FIX2(128, 8, 3, 16, 8)
#undef NUFDS_FIX2
    if constexpr (sizeof(R) == 4) {  // complex64 only: 16384 elements fit one tile
        if (!d.one_bfly && !d.chain && is(16384, 1, 4, 16, 16, 16, 4)) {
            *err = launch_fixed<R, ME, 64, 1024, false, true, SG, 0, 16, 16, 16, 4>(d, ld, st, tw, twf, chainvec, s);
            return true;
        }
    }
    return false;
}

template <typename R, int MAXE, int NBMAX, int MAXT, bool CHAINP, bool PAD, int SGN, bool WIN = false>
static hipError_t launch_variant(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                                 const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s) {
    static bool attr_set = false;
    auto kern = &fft_pass_kernel<R, MAXE, NBMAX, MAXT, CHAINP, PAD, SGN, WIN>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t shm = (size_t)lds_elems(d.L * d.W) * sizeof(cpx<R>);  // padded size covers both layouts
    const int ga = d.xcd_rows ? kXcds * ((d.tiles_a + kXcds - 1) / kXcds) : d.tiles_a;
    dim3 grid(d.tiles_b, ga), block(d.nthreads);
    hipLaunchKernelGGL(kern, grid, block, shm, s, d, ld, st, tw, twf, chainvec);
    return hipGetLastError();
}

template <typename R, int SG>
static hipError_t launch_signed(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                                const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s) {
    constexpr int OE = OneBflyElems<R>::value, OT = OneBflyThreads<R>::value, ME = MaxElems<R>::value;
    // tiles of 8 or more columns keep their lanes on consecutive LDS words without padding; the
    // several-butterflies variant serves long rows (narrow tiles) only
    const bool pad = d.W < 8;
    if (ld.win_lo < ld.win_hi) {
        // windowed loads: forward, non-chain passes only (the transform of a zero-padded hologram)
        if constexpr (SG < 0) {
            if (!d.chain) {
                if (d.one_bfly) {
                    if (pad) return launch_variant<R, OE, 1, OT, false, true, SG, true>(d, ld, st, tw, twf, chainvec, s);
                    return launch_variant<R, OE, 1, OT, false, false, SG, true>(d, ld, st, tw, twf, chainvec, s);
                }
                return launch_variant<R, ME, 64, 1024, false, true, SG, true>(d, ld, st, tw, twf, chainvec, s);
            }
        }
        return hipErrorInvalidValue;
    }
    if (d.chain) {
        if (d.one_bfly) {
            if (pad) return launch_variant<R, OE, 1, OT, true, true, SG>(d, ld, st, tw, twf, chainvec, s);
            return launch_variant<R, OE, 1, OT, true, false, SG>(d, ld, st, tw, twf, chainvec, s);
        }
        return launch_variant<R, ME, 64, 1024, true, true, SG>(d, ld, st, tw, twf, chainvec, s);
    }
    if (d.one_bfly) {
        if (pad) return launch_variant<R, OE, 1, OT, false, true, SG>(d, ld, st, tw, twf, chainvec, s);
        return launch_variant<R, OE, 1, OT, false, false, SG>(d, ld, st, tw, twf, chainvec, s);
    }
    return launch_variant<R, ME, 64, 1024, false, true, SG>(d, ld, st, tw, twf, chainvec, s);
}


// ------------------------------------------------------------ row chain in one pass
// A transform, or the chain IDFT . vec . DFT, along rows whose complex64 tile exceeds LDS (25600
// elements: 200 KB; 32768: 256 KB) while a plane of their real parts fits (100 KB; 128 KB).  One
// workgroup holds one row in registers,
// L / T elements per thread; every exchange between two stages passes through a float plane in
// LDS twice, real parts and then imaginary parts.  The first transform's last stage and the
// second's first stage have the same radix, so each lane already holds the elements
// j + t L/RAD that it needs and the chain multiply takes no exchange.  Stages are the
// Stockham stages of fft_stage: butterfly j reads x[j + t L/RAD], twiddles by
// w_(Ns RAD)^(t k) with k = j mod Ns, and writes (j / Ns) Ns RAD + k + t Ns.
// Butterfly j = tid + i T of a stage exists for j < L/RAD; with T a multiple of 64 a wave's
// butterflies i either all exist or none does past the first partial wave, and waves without
// one skip the round (wave_has); lanes past the end in a partial wave work on butterfly 0's
// elements and store nothing.

template <int A, int... REST>
struct FirstOf {
    static constexpr int value = A;
};

// butterflies per thread of a radix-RAD stage
template <int L, int T, int RAD>
struct RcNb {
    static constexpr int value = (L / RAD + T - 1) / T;
};

// registers of a radix-RAD stage: RcNb butterflies of RAD elements
template <int L, int T, int RAD>
using RcRegs = cpx<float>[RcNb<L, T, RAD>::value][RAD];

constexpr int rc_gcd(int a, int b) { return b == 0 ? a : rc_gcd(b, a % b); }

// Plane layout of the exchange from a radix-RA stage after NSA to a radix-RB stage: one pad word
// after every P words, P chosen so that both sides' addresses are affine in the element t of a
// butterfly (the writer's pos = (j / NSA) NSA RA + j mod NSA + t NSA, the reader's j + t L/RB):
// P = RA when NSA = 1 (pos / RA = j), else P divides NSA; and P divides L/RB.  The pads also
// break the writer's strides across the LDS banks (RA + 1 words between lanes when NSA = 1).
template <int L, int RA, int NSA, int RB>
struct RcLayout {
    static constexpr int LRB = L / RB;
    static constexpr int P = NSA == 1 ? RA : rc_gcd(NSA, LRB);
    static_assert(P >= 8 && LRB % P == 0 && (NSA == 1 || NSA % P == 0), "no affine plane layout");
    static constexpr int wstride = NSA + NSA / P;  // writer: words between t and t + 1
    static constexpr int rstride = LRB + LRB / P;  // reader
};

// words of the plane for every layout above (P >= 8)
__host__ __device__ constexpr int rc_plane_words(int L) { return L + L / 8 + 1; }

// whether the wave holding this thread has butterfly round i of a stage with LR butterflies
template <int T>
__device__ __forceinline__ bool wave_has(int wbase, int i, int LR) { return wbase + i * T < LR; }

template <int L, int T, int RAD, int NS, int SGN>
__device__ __forceinline__ void rc_butterflies(RcRegs<L, T, RAD>& v, const cpx<float>* __restrict__ tw, int tid,
                                               int wbase) {
    constexpr int NB = RcNb<L, T, RAD>::value;
    constexpr int LR = L / RAD;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if (!wave_has<T>(wbase, i, LR)) continue;
        if constexpr (NS > 1) {
            const int j0 = tid + i * T;
            const int j = j0 < LR ? j0 : 0;
            const int k = j % NS;
            cpx<float> c = load_at<float>(uniform_base(tw), (uint32_t)(k * (L / (NS * RAD))) * 8u);
            if (SGN > 0) c.y = -c.y;
            apply_twiddles<float, RAD>(v[i], c);
        }
        SmallDft<float, RAD>::run(v[i], SGN);
    }
}

// Outputs of a stage (radix RA after NSA, X_t in o[i][perm(t)]) to the inputs of a radix-RB stage.
template <int L, int T, int RA, int NSA, int RB>
__device__ __forceinline__ void rc_exchange(float* plane, RcRegs<L, T, RA>& o, RcRegs<L, T, RB>& u, int tid,
                                            int wbase) {
    using Lay = RcLayout<L, RA, NSA, RB>;
    constexpr int NBA = RcNb<L, T, RA>::value, NBB = RcNb<L, T, RB>::value;
    constexpr int LRA = L / RA, LRB = L / RB, P = Lay::P;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        __syncthreads();  // the previous readers of the plane are done
        // opaque copies of the thread index: the plane addresses are recomputed in each sweep
        // instead of being held in registers across the barriers
        int tw_ = tid, tr_ = tid;
        asm volatile("" : "+v"(tw_));
#pragma unroll
        for (int i = 0; i < NBA; ++i) {
            const int j = tw_ + i * T;
            if (wave_has<T>(wbase, i, LRA) && j < LRA) {
                int a0;
                if constexpr (NSA == 1) {
                    a0 = j * (RA + 1);
                } else {
                    const int q = j / NSA, k = j - q * NSA;
                    const int p0 = q * NSA * RA + k;
                    a0 = p0 + p0 / P;
                }
#pragma unroll
                for (int t = 0; t < RA; ++t) {
                    const cpx<float> x = o[i][SmallDft<float, RA>::perm(t)];
                    plane[a0 + t * Lay::wstride] = part ? x.y : x.x;
                }
            }
        }
        __syncthreads();
        asm volatile("" : "+v"(tr_));
#pragma unroll
        for (int i = 0; i < NBB; ++i) {
            if (!wave_has<T>(wbase, i, LRB)) continue;
            const int j0 = tr_ + i * T;
            const int j = j0 < LRB ? j0 : 0;
            const int a0 = j + j / P;
#pragma unroll
            for (int t = 0; t < RB; ++t) {
                const float x = plane[a0 + t * Lay::rstride];
                if (part) u[i][t].y = x;
                else u[i][t].x = x;
            }
        }
    }
}

// The stages of one transform, from a stage's inputs in v; fin receives the last stage's outputs
// (X_t of butterfly j in v[i][perm(t)], at j + t L/RAD).
template <int L, int T, int SGN, int NS, int RAD, int... RS, typename F>
__device__ __forceinline__ void rc_stages(float* plane, RcRegs<L, T, RAD>& v, const cpx<float>* __restrict__ tw,
                                          int tid, int wbase, F&& fin) {
    rc_butterflies<L, T, RAD, NS, SGN>(v, tw, tid, wbase);
    if constexpr (sizeof...(RS) == 0) {
        static_assert(NS * RAD == L, "radices must multiply to the length");
        fin(v);
    } else {
        constexpr int RB = FirstOf<RS...>::value;
        RcRegs<L, T, RB> u;
        rc_exchange<L, T, RAD, NS, RB>(plane, v, u, tid, wbase);
        rc_stages<L, T, SGN, NS * RAD, RS...>(plane, u, tw, tid, wbase, fin);
    }
}

template <int... RS>
struct Radices {};

// Row 'blockIdx.x': out = st(DFT_-SGN(vec . DFT_SGN(ld(in)))) for a chain, st(DFT_SGN(ld(in)))
// otherwise; T1 and T2 are the two transforms' radices (T2 opens with T1's last radix).  A chain
// loads plain copies; a single transform applies everything LoadPlain describes.  The store applies
// the axis sign and scale.
template <int L, int T, int SGN, bool CHAIN, int... A, int... B>
__device__ __forceinline__ void row_chain_body(Radices<A...>, Radices<B...>, const PassDesc& d,
                                               const LoadPlain<float>& ld, const StorePlain<float>& st,
                                               const cpx<float>* __restrict__ tw, const cpx<float>* __restrict__ vec,
                                               float* plane) {
    static_assert(T % 64 == 0, "whole waves");
    constexpr int R0 = FirstOf<A...>::value;
    constexpr int LR0 = L / R0;
    const int tid = threadIdx.x;
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    const int64_t row = blockIdx.x;
    const cpx<float>* rin = ld.in + row * d.in_pitch;
    cpx<float>* rout = st.out + row * d.out_pitch;
    RcRegs<L, T, R0> v;
    const bool win = !CHAIN && ld.win_lo < ld.win_hi;
#pragma unroll
    for (int i = 0; i < RcNb<L, T, R0>::value; ++i) {
        if (!wave_has<T>(wbase, i, LR0)) continue;
        const int j0 = tid + i * T;
        const int j = j0 < LR0 ? j0 : 0;
#pragma unroll
        for (int t = 0; t < R0; ++t) {
            const int pos = j + t * LR0;
            if (win) {  // outside the window the input is zero and is not read
                v[i][t] = mk(0.0f, 0.0f);
                if (pos >= ld.win_lo && pos < ld.win_hi)
                    v[i][t] = load_at<float>(uniform_base(rin + t * LR0), (uint32_t)j * 8u);
            } else {
                v[i][t] = load_at<float>(uniform_base(rin + t * LR0), (uint32_t)j * 8u);
            }
        }
        if (!CHAIN && !ld.plain) {
#pragma unroll
            for (int t = 0; t < R0; ++t) {
                const int pos = j + t * LR0;
                const bool flip = ld.sign_axis && (pos & 1);
                const float f = flip ? -ld.scale : ld.scale;
                v[i][t] = mk(v[i][t].x * f, (ld.conj ? -v[i][t].y : v[i][t].y) * f);
            }
            if (ld.mul) {
                // the vector in factored form: element j + t LR0 is c_j a_j^t b_t, two loads per
                // thread instead of R0 (rows would otherwise read the whole vector each)
                const cpx<float> cj = load_at<float>(uniform_base(ld.mul), (uint32_t)(2 * j) * 8u);
                const cpx<float> aj = load_at<float>(uniform_base(ld.mul), (uint32_t)(2 * j + 1) * 8u);
                cpx<float> pw = cj;
#pragma unroll
                for (int t = 0; t < R0; ++t) {
                    const cpx<float> bt = load_at<float>(uniform_base(ld.mul + 2 * LR0), (uint32_t)t * 8u);
                    v[i][t] = v[i][t] * (pw * bt);
                    if (t + 1 < R0) pw = pw * aj;
                }
            }
        }
    }
    auto store = [&](auto& o) {
        constexpr int RL = sizeof(o[0]) / sizeof(o[0][0]);
        constexpr int NB = sizeof(o) / sizeof(o[0]);
        constexpr int LR = L / RL;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = tid + i * T;
            if (wave_has<T>(wbase, i, LR) && j < LR) {
#pragma unroll
                for (int t = 0; t < RL; ++t) {
                    cpx<float> x = o[i][SmallDft<float, RL>::perm(t)];
                    if (!st.plain) {
                        const bool flip = st.sign_axis && ((j + t * LR) & 1);
                        const float f = flip ? -st.scale : st.scale;
                        x = mk(x.x * f, x.y * f);
                    }
                    store_at<float>(uniform_base(rout + t * LR), (uint32_t)j * 8u, x);
                }
            }
        }
    };
    auto middle = [&](auto& o) {
        constexpr int RL = sizeof(o[0]) / sizeof(o[0][0]);
        constexpr int NB = sizeof(o) / sizeof(o[0]);
        constexpr int LR = L / RL;
        static_assert(RL == FirstOf<B...>::value, "the second transform opens with the first's last radix");
        RcRegs<L, T, RL> u;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (!wave_has<T>(wbase, i, LR)) continue;
            const int j0 = tid + i * T;
            const int j = j0 < LR ? j0 : 0;
#pragma unroll
            for (int t = 0; t < RL; ++t)
                u[i][t] = o[i][SmallDft<float, RL>::perm(t)] *
                          load_at<float>(uniform_base(vec), (uint32_t)(j + t * LR) * 8u);
        }
        rc_stages<L, T, -SGN, 1, B...>(plane, u, tw, tid, wbase, store);
    };
    if constexpr (CHAIN) rc_stages<L, T, SGN, 1, A...>(plane, v, tw, tid, wbase, middle);
    else rc_stages<L, T, SGN, 1, A...>(plane, v, tw, tid, wbase, store);
}

// Radix plans: 25600 = 32 32 25 (then 25 32 32) over 1024 threads, one butterfly per thread and
// stage; 32768 = 32 32 32 over 1024 threads (the rows of a 16384-wide hologram's oversampled
// spectrum; its plane with pads is 144 KB); 6400 = 32 8 25 over 256 threads, the same radices and
// both forms of exchange at a length the tests reach with a lowered tile capacity.
template <int L>
struct RowChainPlan;
template <>
struct RowChainPlan<25600> {
    static constexpr int T = 1024;
    using A = Radices<32, 32, 25>;
    using B = Radices<25, 32, 32>;
};
template <>
struct RowChainPlan<32768> {
    static constexpr int T = 1024;
    using A = Radices<32, 32, 32>;
    using B = Radices<32, 32, 32>;
};
template <>
struct RowChainPlan<6400> {
    static constexpr int T = 256;
    using A = Radices<32, 8, 25>;
    using B = Radices<25, 8, 32>;
};

template <int L, int SGN, bool CHAIN>
__global__ void __launch_bounds__(RowChainPlan<L>::T)
    row_chain_kernel(PassDesc d, LoadPlain<float> ld, StorePlain<float> st, const cpx<float>* __restrict__ tw,
                     const cpx<float>* __restrict__ vec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* plane = reinterpret_cast<float*>(smem_raw);
    using P = RowChainPlan<L>;
    row_chain_body<L, P::T, SGN, CHAIN>(typename P::A{}, typename P::B{}, d, ld, st, tw, vec, plane);
}

template <int L, int SGN, bool CHAIN>
static hipError_t launch_row_chain_l(const PassDesc& d, const LoadPlain<float>& ld, const StorePlain<float>& st,
                                     const cpx<float>* tw, const cpx<float>* vec, hipStream_t s) {
    static_assert(rc_plane_words(L) * sizeof(float) <= 160 * 1024, "the plane must fit LDS");
    if (d.rows <= 0) return hipSuccess;  // nothing to transform (a zero-sized grid is not a launch)
    static bool attr_set = false;
    auto kern = &row_chain_kernel<L, SGN, CHAIN>;
    const size_t shm = (size_t)rc_plane_words(L) * sizeof(float);
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(d.rows), dim3(RowChainPlan<L>::T), shm, s, d, ld, st, tw, vec);
    return hipGetLastError();
}

template <int A, int... REST>
constexpr int first_of(Radices<A, REST...>) { return A; }

int row_chain_first_radix(int L) {
    if (L == 25600) return first_of(RowChainPlan<25600>::A{});
    if (L == 32768) return first_of(RowChainPlan<32768>::A{});
    if (L == 6400) return first_of(RowChainPlan<6400>::A{});
    return 0;
}

int row_chain_threads(int L) {
    if (L == 25600) return RowChainPlan<25600>::T;
    if (L == 32768) return RowChainPlan<32768>::T;
    if (L == 6400) return RowChainPlan<6400>::T;
    return 0;
}

template <typename R>
static hipError_t launch_row_chain(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st,
                                   const cpx<R>* tw, const cpx<R>* vec, hipStream_t s) {
    if constexpr (sizeof(R) != 4) {
        return hipErrorInvalidValue;
    } else {
        // a chain loads plain copies and multiplies by its vector between the transforms
        if ((d.chain && (!vec || !ld.plain || ld.win_lo < ld.win_hi)) || d.W != 1 || d.L != d.cols ||
            d.nthreads != row_chain_threads(d.L))
            return hipErrorInvalidValue;
#define NUFDS_ROWC(LL)                                                                                      \
    if (d.L == LL) {                                                                                        \
        if (d.chain)                                                                                        \
            return d.sign < 0 ? launch_row_chain_l<LL, -1, true>(d, ld, st, tw, vec, s)                     \
                              : launch_row_chain_l<LL, 1, true>(d, ld, st, tw, vec, s);                     \
        return d.sign < 0 ? launch_row_chain_l<LL, -1, false>(d, ld, st, tw, vec, s)                        \
                          : launch_row_chain_l<LL, 1, false>(d, ld, st, tw, vec, s);                        \
    }
        NUFDS_ROWC(25600)
        NUFDS_ROWC(32768)
        NUFDS_ROWC(6400)
#undef NUFDS_ROWC
        return hipErrorInvalidValue;
    }
}

// The transform direction is a template parameter of the kernel (the sign folds into the butterflies).
template <typename R>
hipError_t launch_pass(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                       const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s) {
    if (d.kind == K_ROWC) return launch_row_chain<R>(d, ld, st, tw, chainvec, s);
    hipError_t e = hipSuccess;
    const bool win = ld.win_lo < ld.win_hi;  // the specialised kernels read without a window
    if (d.sign < 0) {
        if (!win && launch_specialised<R, -1>(d, ld, st, tw, twf, chainvec, s, &e)) return e;
        return launch_signed<R, -1>(d, ld, st, tw, twf, chainvec, s);
    }
    if (!win && launch_specialised<R, 1>(d, ld, st, tw, twf, chainvec, s, &e)) return e;
    return launch_signed<R, 1>(d, ld, st, tw, twf, chainvec, s);
}

template hipError_t launch_pass<float>(const PassDesc&, const LoadPlain<float>&,
                                                         const StorePlain<float>&, const cpx<float>*,
                                                         const cpx<float>*, const cpx<float>*, hipStream_t);
template hipError_t launch_pass<double>(const PassDesc&, const LoadPlain<double>&,
                                                           const StorePlain<double>&, const cpx<double>*,
                                                           const cpx<double>*, const cpx<double>*, hipStream_t);
// Radix sequence of a 5-smooth length with the fewest stages (then the largest leading radices)
// from the radices the kernel implements; radices above max_radix are not used.
bool factor_radices(int L, int* nst, int* rad, int max_radix) {
    static const int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
    // best[n] = fewest stages for length n (n <= L), by dynamic programming over divisors
    std::vector<int> best(L + 1, 1 << 20), pick(L + 1, 0);
    best[1] = 0;
    for (int n = 2; n <= L; ++n) {
        if (L % n) continue;
        for (int r : kRadices) {
            if (r > max_radix || n % r) continue;
            if (best[n / r] + 1 < best[n]) {
                best[n] = best[n / r] + 1;
                pick[n] = r;
            }
        }
    }
    if (best[L] >= (1 << 20) || best[L] > kMaxStages) return false;
    int n = L, k = 0;
    while (n > 1) {
        rad[k++] = pick[n];
        n /= pick[n];
    }
    *nst = k;
    return true;
}

// The per-lane byte offsets of a pass's first-stage loads and last-stage stores (element j + t L/r of
// lane (j, w) sits at the uniform base of row t plus the lane offset) must fit in 32 bits.
bool pass_offsets_fit(const PassDesc& d, int esize) {
    const TileMap m = tile_map(d, 0, 0);
    const int64_t W = d.W;
    const int64_t lin = (int64_t)(d.L / d.rad[0] - 1) * m.isn + (W - 1) * m.isw;
    const int64_t lout = (int64_t)(d.L / d.rad[d.nst - 1] - 1) * m.osn + (W - 1) * m.osw;
    const int64_t lim = (int64_t)1 << 32;
    return lin >= 0 && lout >= 0 && lin * esize < lim && lout * esize < lim;
}

// Threads for one butterfly per thread per stage: the largest stage's butterfly count, rounded up to
// whole waves; -1 if that exceeds max_threads.
int pick_threads_one(int L, int W, int nst, const int* rad, int max_threads) {
    int need = 0;
    for (int s = 0; s < nst; ++s) need = std::max(need, (L / rad[s]) * W);
    const int T = (need + 63) / 64 * 64;
    return T <= max_threads ? T : -1;
}

int pick_threads(int L, int W, int nst, const int* rad, int max_elems) {
    for (int T = 64; T <= 1024; T += 64) {
        bool ok = true;
        for (int s = 0; s < nst && ok; ++s) {
            int r = rad[s];
            int B = (L / r) * W;
            int per = (B + T - 1) / T;
            if (per > std::min(max_elems / r, kMaxBfly)) ok = false;
        }
        if (ok) return T;
    }
    return -1;
}

}  // namespace nufds
