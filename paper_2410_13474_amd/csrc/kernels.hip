// Map-table, output-gather and test-input kernels of libnufds (gfx950).
#include "kernels.h"

#include <climits>

#include "special.h"

namespace nufds {

// ------------------------------------------------------------ step 1: stretch map
// Entry (ky, kx) of the quadrant table holds the pre-image, in spectral samples from the
// centre, of the stretched frequency (kx / (N_x D), ky / (N_y D)) under Eqs. 9-10 with Eq. 16:
// (u N_x D / lambda, v N_y D / lambda), or NaN when there is no pre-image on the propagating
// disk or it falls outside the hologram band |u|, |v| <= lambda / (2 D).  With use_poly the map is
// the paper's polynomial model (I replaced by I_P), inverted by Newton from the exact pre-image.
__global__ void map_table_kernel(double* __restrict__ table, int kxt, int kyt, double wavelength,
                                 double npx, double npy, double s, PaperPoly poly, int use_poly) {
    const int kx = blockIdx.x * blockDim.x + threadIdx.x;
    const int ky = blockIdx.y * blockDim.y + threadIdx.y;
    if (kx > kxt || ky > kyt) return;
    const double t1 = (double)kx * wavelength / npx;
    const double t2 = (double)ky * wavelength / npy;
    double u, v;
    double px = __builtin_nan(""), py = __builtin_nan("");
    const bool ok = use_poly ? stretch_preimage_paper(poly, t1, t2, &u, &v) : stretch_preimage(t1, t2, &u, &v);
    if (ok && fabs(u) <= s && fabs(v) <= s) {
        px = u * (npx / wavelength);
        py = v * (npy / wavelength);
    }
    const int64_t e = (int64_t)ky * (kxt + 1) + kx;
    table[2 * e] = px;
    table[2 * e + 1] = py;
}

__global__ void tile_bounds_kernel(const double* __restrict__ table, int kxt, int kyt, double sigma,
                                   int4* __restrict__ bounds);

hipError_t launch_map_table(double* table, int kxt, int kyt, double wavelength, double npx, double npy,
                            double s, int sigma, const PaperPoly* poly, hipStream_t st) {
    dim3 block(64, 4);
    dim3 grid((kxt + 1 + 63) / 64, (kyt + 1 + 3) / 4);
    PaperPoly p{};
    if (poly) p = *poly;
    hipLaunchKernelGGL(map_table_kernel, grid, block, 0, st, table, kxt, kyt, wavelength, npx, npy, s, p,
                       poly ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int4* bounds = reinterpret_cast<int4*>(reinterpret_cast<char*>(table) + map_entries_bytes(kxt, kyt));
    hipLaunchKernelGGL(tile_bounds_kernel, dim3(map_tiles_x(kxt), map_tiles_y(kyt)), dim3(kGatherTile * kGatherTile), 0,
                       st, table, kxt, kyt, (double)sigma, bounds);
    return hipGetLastError();
}

// Keys cubic convolution weights (a = -1/2) of the taps at floor-1 .. floor+2 for fraction t.
template <typename R>
__device__ __forceinline__ void keys4(R t, R* w) {
    R t2 = t * t, t3 = t2 * t;
    w[0] = R(-0.5) * t3 + t2 - R(0.5) * t;
    w[1] = R(1.5) * t3 - R(2.5) * t2 + R(1);
    w[2] = R(-1.5) * t3 + R(2) * t2 + R(0.5) * t;
    w[3] = R(0.5) * t3 - R(0.5) * t2;
}

// Keys 4 x 4 interpolation of the [ny][nx] spectrum at fractional sample (px, py), periodic.  In
// complex64 the four taps of a row are two 16-byte loads when they do not wrap (8-byte alignment is
// enough for global loads), which halves the cache accesses of the gather.
template <typename R>
__device__ __forceinline__ cpx<R> keys_spectrum(const cpx<R>* __restrict__ spec, int nx, int ny, double px,
                                                double py) {
    const double fx = floor(px), fy = floor(py);
    const int ix = (int)fx - 1, iy = (int)fy - 1;
    R wx[4], wy[4];
    keys4<R>(R(px - fx), wx);
    keys4<R>(R(py - fy), wy);
    int rows[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int r = iy + b;
        rows[b] = r < 0 ? r + ny : (r >= ny ? r - ny : r);
    }
    cpx<R> acc = mk(R(0), R(0));
    if (sizeof(R) == 4 && ix >= 0 && ix + 3 < nx) {
        typedef R pair_t __attribute__((ext_vector_type(4), aligned(8)));
        pair_t q[4][2];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const cpx<R>* row = spec + (int64_t)rows[b] * nx + ix;
            q[b][0] = *reinterpret_cast<const pair_t*>(row);
            q[b][1] = *reinterpret_cast<const pair_t*>(row + 2);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const cpx<R> racc = mk(q[b][0].x, q[b][0].y) * wx[0] + mk(q[b][0].z, q[b][0].w) * wx[1] +
                                mk(q[b][1].x, q[b][1].y) * wx[2] + mk(q[b][1].z, q[b][1].w) * wx[3];
            acc = acc + racc * wy[b];
        }
        return acc;
    }
    int cols[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int c = ix + a;
        cols[a] = c < 0 ? c + nx : (c >= nx ? c - nx : c);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const cpx<R>* row = spec + (int64_t)rows[b] * nx;
        cpx<R> racc = mk(R(0), R(0));
#pragma unroll
        for (int a = 0; a < 4; ++a) racc = racc + row[cols[a]] * wx[a];
        acc = acc + racc * wy[b];
    }
    return acc;
}

// ------------------------------------------------------------ step 2: stretch-gather
// Pull form of step 2: the stretched spectrum at band sample k' (stretched frequency index
// k_g = K_c + k' - M/2) is the hologram spectrum Keys-interpolated at the pre-image of k_g.  The map
// is odd in each axis, so the pre-image of (+-|k_gx|, +-|k_gy|) is (+-P_x, +-P_y) from one table entry.
// Output carries the (-1)^(k'_x) centring sign of the inverse transform that follows.

// Window bounds of one 16 x 16 tile of table entries (layout in kernels.h); one workgroup per tile.
__global__ void __launch_bounds__(256) tile_bounds_kernel(const double* __restrict__ table, int kxt, int kyt,
                                                          double sigma, int4* __restrict__ bounds) {
    constexpr int T = kGatherTile;
    __shared__ int red[4][4];
    const int tid = threadIdx.x;
    const int kx = blockIdx.x * T + tid % T, ky = blockIdx.y * T + tid / T;
    bool valid = kx <= kxt && ky <= kyt;
    const int64_t e = valid ? (int64_t)ky * (kxt + 1) + kx : 0;
    const double px = table[2 * e], py = table[2 * e + 1];
    valid = valid && px == px;
    const int fx = valid ? (int)floor(sigma * px) - 1 : 0, fy = valid ? (int)floor(sigma * py) - 1 : 0;
    int r[4] = {valid ? fx : INT_MAX, valid ? -fx : INT_MAX, valid ? fy : INT_MAX, valid ? -fy : INT_MAX};
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = min(r[i], __shfl_xor(r[i], o));
    if ((tid & 63) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[tid >> 6][i] = r[i];
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = min(min(red[0][i], red[1][i]), min(red[2][i], red[3][i]));
        int4 b;
        b.x = r[0];
        b.y = r[0] == INT_MAX ? INT_MAX : -r[1];
        b.z = r[0] == INT_MAX ? INT_MAX : r[2];
        b.w = r[0] == INT_MAX ? INT_MAX : -r[3];
        bounds[blockIdx.y * gridDim.x + blockIdx.x] = b;
    }
}

// Global accesses as a wave-uniform base (scalar registers) plus a 32-bit per-lane byte offset.
typedef __attribute__((address_space(1))) char gbyte;
template <typename T>
__device__ __forceinline__ gbyte* uniform_ptr(const T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gbyte*)(((uint64_t)hi << 32) | lo);
}
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(8)));  // two complex64 samples
typedef double d2_t __attribute__((ext_vector_type(2)));              // one complex128 sample
template <typename R> struct Load16 { typedef f4u_t type; };
template <> struct Load16<double> { typedef d2_t type; };
template <typename V>
__device__ __forceinline__ V load16(gbyte* base, uint32_t off) {
    return *reinterpret_cast<const V __attribute__((address_space(1)))*>(base + off);
}
template <typename R>
__device__ __forceinline__ void store_cpx(gbyte* base, uint32_t off, cpx<R> v) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = v.x;
    w.y = v.y;
    *reinterpret_cast<v2 __attribute__((address_space(1)))*>(base + off) = w;
}

// Window of one mirror in LDS: rows of a fixed pitch P (odd, so that rows start on different banks),
// at most kGatherRows rows.  A 16 x 16 tile's windows measure at most 21 x 21 samples (the inverse
// stretch contracts, so neighbouring entries' pre-images are at most a sample apart along the tile,
// plus the drift across it and the 4-tap stencil).
template <typename R> struct GatherPitch { static constexpr int value = 25; };
template <> struct GatherPitch<double> { static constexpr int value = 21; };
constexpr int kGatherRows = 24;

// One workgroup covers a 16 x 16 tile of quadrant entries.  The window bounds of the tile come from
// the table (computed once per table), so the workgroup starts copying the four mirrored spectrum
// windows under its stencils into LDS at once, alongside its entries' own table loads, and then
// interpolates from LDS: each spectrum sample is fetched once per tile instead of once per tap.  The
// Keys kernel is even, so the mirror -p uses the weights of p in reverse order on the taps
// floor(-p) - 1 .. floor(-p) + 2 reflected, i.e. from N - (first tap of p) - 3 on; one set of 16
// weight products serves all four mirrors, with the centring sign (equal for both x mirrors, whose
// k'_x differ by 2 |k_gx|) and the mask folded in.  A window that crosses the spectrum's edge is
// copied with periodic indices; one that would not fit LDS (none at the sizes measured) is
// interpolated straight from global memory.
template <typename R>
__global__ void __launch_bounds__(256) stretch_gather_kernel(GatherArgs<R> a) {
    constexpr int T = kGatherTile, P = GatherPitch<R>::value, WY = kGatherRows, CAP = P * WY;
    constexpr int ES = sizeof(cpx<R>);
    __shared__ cpx<R> win[4 * CAP];
    // consecutive tile rows to one XCD (round-robin dispatch): their windows share L2 lines
    const int nb = gridDim.x;
    const int lin = blockIdx.y * nb + blockIdx.x;
    const int xcd = lin % kXcds, slot = lin / kXcds;
    const int per = (a.nty + kXcds - 1) / kXcds;
    const int brow = xcd * per + slot / nb;
    if (brow >= a.nty) return;
    const int tx = a.tx0 + slot % nb, ty = a.ty0 + brow;
    const int tid = threadIdx.x, lx = tid % T, ly = tid / T;
    const int ax = tx * T + lx, ay = ty * T + ly;
    const bool inr = ax >= a.ax0 && ax < a.ax0 + a.nax && ay >= a.ay0 && ay < a.ay0 + a.nay;
    const int hx = a.nx >> 1, hy = a.ny >> 1;
    // this entry's pre-image (independent of the window: its load overlaps the fill)
    double px, py;
    bool valid;
    int bx0, bx1, by0, by1;
    if (a.nostretch) {
        // the pre-image of entry k is k itself, sigma k on the spectrum's grid
        const int chx = hx / a.sigma, chy = hy / a.sigma;
        valid = inr && ax <= chx && ay <= chy;
        px = valid ? (double)(a.sigma * ax) : 0.0;
        py = valid ? (double)(a.sigma * ay) : 0.0;
        const int lox = max(tx * T, a.ax0), hix = min(min(tx * T + T - 1, a.ax0 + a.nax - 1), chx);
        const int loy = max(ty * T, a.ay0), hiy = min(min(ty * T + T - 1, a.ay0 + a.nay - 1), chy);
        bx0 = (lox <= hix && loy <= hiy) ? a.sigma * lox - 1 : INT_MAX;
        bx1 = a.sigma * hix - 1;
        by0 = a.sigma * loy - 1;
        by1 = a.sigma * hiy - 1;
    } else {
        valid = inr && ax <= a.kxt && ay <= a.kyt;
        const int64_t e = valid ? (int64_t)ay * (a.kxt + 1) + ax : 0;
        const double tx_ = a.table[2 * e], ty_ = a.table[2 * e + 1];
        valid = valid && tx_ == tx_;
        // masked entries (NaN in the table, or beyond it) never reach the index arithmetic; the
        // table holds positions on the hologram's spectral grid, the spectrum may be sigma times finer
        px = valid ? a.sigma * tx_ : 0.0;
        py = valid ? a.sigma * ty_ : 0.0;
        bx0 = bx1 = by0 = by1 = INT_MAX;  // a tile beyond the table has no valid entry
        if (tx < a.tbx && ty < a.tby) {
            const int4 b = a.bounds[ty * a.tbx + tx];
            bx0 = b.x;
            bx1 = b.y;
            by0 = b.z;
            by1 = b.w;
        }
    }
    bx0 = __builtin_amdgcn_readfirstlane(bx0);
    const bool empty = bx0 == INT_MAX;  // no valid entry in the tile
    if (empty) bx1 = by0 = by1 = bx0 = 0;
    const int mnx = __builtin_amdgcn_readfirstlane(bx0) + hx, mxx = __builtin_amdgcn_readfirstlane(bx1) + hx;
    const int mny = __builtin_amdgcn_readfirstlane(by0) + hy, mxy = __builtin_amdgcn_readfirstlane(by1) + hy;
    const int wx = mxx - mnx + 4, wy = mxy - mny + 4;
    const bool fits = !empty && wx <= P && wy <= WY;
    // window origins of the mirrors: x from mnx (+) or nx - mxx - 3 (-); likewise y
    const int xo0 = mnx, xo1 = a.nx - mxx - 3, yo0 = mny, yo1 = a.ny - mxy - 3;
    constexpr int SPL = sizeof(R) == 4 ? 2 : 1;  // samples per 16-byte load
    const int wxl = (wx + SPL - 1) / SPL * SPL;
    const bool inside = min(xo0, xo1) >= 0 && max(xo0, xo1) + wxl <= a.nx && min(yo0, yo1) >= 0 &&
                        max(yo0, yo1) + wy <= a.ny;
    if (fits && inside) {
        // 16-byte row loads from a scalar base per mirror; one lane offset serves the four mirrors
        constexpr int LPR = 32 / SPL, RG = 256 / LPR, KP = (WY + RG - 1) / RG;
        typedef typename Load16<R>::type V;
        const int c = SPL * (tid % LPR), rg = tid / LPR;
        const bool cin = c < wx;
        uint32_t off[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int r = rg + k * RG;
            off[k] = (uint32_t)(((r < wy ? r : 0) * a.nx + (cin ? c : 0)) * ES);  // every lane in bounds
        }
        V tmp[4][KP];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            gbyte* base = uniform_ptr(a.spec + ((int64_t)((m >> 1) ? yo1 : yo0) * a.nx + ((m & 1) ? xo1 : xo0)));
#pragma unroll
            for (int k = 0; k < KP; ++k) tmp[m][k] = load16<V>(base, off[k]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int r = rg + k * RG;
                if (cin && r < wy) {
                    cpx<R>* d = win + m * CAP + r * P + c;
                    d[0] = mk(R(tmp[m][k][0]), R(tmp[m][k][1]));
                    if constexpr (SPL == 2) {
                        if (c + 1 < wx) d[1] = mk(R(tmp[m][k][2]), R(tmp[m][k][3]));
                    }
                }
            }
        __syncthreads();
    } else if (fits) {
        // the window crosses the spectrum's edge: one sample per lane, periodic indices
        constexpr int K = (WY + 7) / 8;
        const int c = tid % 32, rg = tid / 32;
        const bool cin = c < wx;
        cpx<R> tmp[4][K];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int x0 = (m & 1) ? xo1 : xo0, y0 = (m >> 1) ? yo1 : yo0;
            int gc = x0 + (cin ? c : 0);
            gc = gc < 0 ? gc + a.nx : (gc >= a.nx ? gc - a.nx : gc);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = rg + k * 8;
                int gr = y0 + (r < wy ? r : 0);
                gr = gr < 0 ? gr + a.ny : (gr >= a.ny ? gr - a.ny : gr);
                tmp[m][k] = a.spec[(int64_t)gr * a.nx + gc];
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = rg + k * 8;
                if (cin && r < wy) win[m * CAP + r * P + c] = tmp[m][k];
            }
        __syncthreads();
    }
    // Keys weights of the (+, +) mirror; products with the centring sign and the mask folded in
    const double fx = floor(px), fy = floor(py);
    R wgx[4], wgy[4];
    keys4<R>(R(px - fx), wgx);
    keys4<R>(R(py - fy), wgy);
    const R sg = valid ? (((ax - a.gx0) & 1) ? R(-1) : R(1)) : R(0);
    R w[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const R yb = wgy[b] * sg;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[b][q] = yb * wgx[q];
    }
    // first taps in spectrum indices (masked entries: the window's corner, in range)
    const int ixp = valid ? (int)fx - 1 + hx : mnx, iyp = valid ? (int)fy - 1 + hy : mny;
    const int cw0 = ixp - mnx, cw1 = mxx - ixp, rw0 = iyp - mny, rw1 = mxy - iyp;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
        const int ky = (sy ? -ay : ay) - a.gy0;
        const bool yin = inr && ky >= 0 && ky < a.my && !(sy && ay == 0);
        // output rows of this mirror from a scalar base at the tile's first row in memory order
        const int row0 = sy ? -(ty * T + T - 1) - a.gy0 : ty * T - a.gy0;
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
            const int kx = (sx ? -ax : ax) - a.gx0;
            const bool in = yin && kx >= 0 && kx < a.mx && !(sx && ax == 0);
            R re = R(0), im = R(0);
            if (fits) {
                const cpx<R>* s0 = win + (2 * sy + sx) * CAP + (sy ? rw1 : rw0) * P + (sx ? cw1 : cw0);
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const R wt = w[sy ? 3 - b : b][sx ? 3 - q : q];
                        const cpx<R> t = s0[b * P + q];
                        re = fma(wt, t.x, re);
                        im = fma(wt, t.y, im);
                    }
            } else if (!empty) {
                // taps from global memory: first tap (+) ixp, (-) nx - ixp - 3, weights as above
                const int cb = sx ? a.nx - ixp - 3 : ixp, rb = sy ? a.ny - iyp - 3 : iyp;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    int r = rb + b;
                    r = r < 0 ? r + a.ny : (r >= a.ny ? r - a.ny : r);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int cc = cb + q;
                        cc = cc < 0 ? cc + a.nx : (cc >= a.nx ? cc - a.nx : cc);
                        const R wt = w[sy ? 3 - b : b][sx ? 3 - q : q];
                        const cpx<R> t = a.spec[(int64_t)r * a.nx + cc];
                        re = fma(wt, t.x, re);
                        im = fma(wt, t.y, im);
                    }
                }
            }
            if (in) {
                const int col0 = sx ? -(tx * T + T - 1) - a.gx0 : tx * T - a.gx0;
                gbyte* base = uniform_ptr(a.out + ((int64_t)row0 * a.mx + col0));
                const uint32_t o = (uint32_t)(((sy ? T - 1 - ly : ly) * a.mx + (sx ? T - 1 - lx : lx)) * ES);
                store_cpx<R>(base, o, mk(re, im));
            }
        }
    }
}

template <typename R>
hipError_t launch_stretch_gather(const GatherArgs<R>& a, hipStream_t st) {
    if (a.ntx <= 0 || a.nty <= 0) return hipSuccess;
    dim3 block(kGatherTile * kGatherTile);
    const int per = (a.nty + kXcds - 1) / kXcds;
    dim3 grid(a.ntx, kXcds * per);
    hipLaunchKernelGGL(stretch_gather_kernel<R>, grid, block, 0, st, a);
    return hipGetLastError();
}
template hipError_t launch_stretch_gather<float>(const GatherArgs<float>&, hipStream_t);
template hipError_t launch_stretch_gather<double>(const GatherArgs<double>&, hipStream_t);

// ------------------------------------------------------------ step 5: output gather
// For output pixel (i, j) at true coordinates (x, y): distorted position (x', y') of Eqs. 17-18
// (x' = A(x) R^-1/2, y' = B(y) R^-1/2 with per-column / per-row factors A, B), its fractional
// FrT index q = (x' - K_c D_F) / D_F + M/2, a 4 x 4 Keys interpolation of F (zero outside the
// FrT grid; F already carries the centring signs), times the outer chirp exp(+i k (x'^2 + y'^2) / 2z)
// of Eq. 2 with the phase reduced mod 2 pi in float64, conjugated for diverging holograms.
// sin and cos of a float64 phase of any magnitude, rounded to R.  complex64: Cody-Waite reduction by
// pi/2 in float64 (two-part constant), then on [-pi/4, pi/4] the Taylor series of sin to x^9 and of
// cos to x^10 in float32 (truncation below 2e-9, under half an ulp of 1), and the quadrant's swap and
// signs.  complex128: reduction by 2 pi in float64 and the library sincos.
template <typename R>
__device__ __forceinline__ void sincos_phase(double ph, R* s, R* c);
template <>
__device__ __forceinline__ void sincos_phase<float>(double ph, float* s, float* c) {
    const double n = rint(ph * 0.63661977236758134308);  // 2 / pi
    double r = fma(-n, 1.5707963267948966192, ph);
    r = fma(-n, 6.1232339957367658e-17, r);
    const float x = (float)r, x2 = x * x;
    const float sn = fmaf(x * x2, fmaf(x2, fmaf(x2, fmaf(x2, 2.7557319e-6f, -1.9841270e-4f), 8.3333333e-3f),
                                       -0.16666667f), x);
    const float cs = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, -2.7557319e-7f, 2.4801587e-5f), -1.3888889e-3f),
                                             4.1666667e-2f), -0.5f), 1.0f);
    const int q = (int)(int64_t)n & 3;  // sin(x + q pi/2), cos(x + q pi/2)
    float so = (q & 1) ? cs : sn, co = (q & 1) ? sn : cs;
    *s = (q & 2) ? -so : so;
    *c = ((q + 1) & 2) ? -co : co;
}
template <>
__device__ __forceinline__ void sincos_phase<double>(double ph, double* s, double* c) {
    const double n = rint(ph * 0.15915494309189533577);
    ph = fma(-n, 6.283185307179586232, ph);
    ph = fma(-n, 2.4492935982947064e-16, ph);
    sincos(ph, s, c);
}

template <typename R>
__global__ void output_gather_kernel(OutputArgs<R> a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (j >= a.sx || i >= a.sy) return;
    const double x = a.cx + (double)(j - (a.sx >> 1)) * a.dox;
    const double y = a.cy + (double)(i - (a.sy >> 1)) * a.doy;
    double xp, yp;
    if (a.remap) {
        // R^(-1/2) = r2^(-1/4): a float seed from the square-root and reciprocal-square-root
        // instructions (a few ulp; r2 within float's normal range), then Newton steps
        // y <- y (5 - r2 y^4) / 4 in float64, each squaring the relative error (times 5/2): one
        // step leaves ~2e-13 (complex64), two reach float64 rounding (complex128)
        const double r2 = x * x + y * y + a.z * a.z;
        double t = (double)__builtin_amdgcn_rsqf(__builtin_amdgcn_sqrtf((float)r2));
        double t2 = t * t;
        t = t * (5.0 - r2 * (t2 * t2)) * 0.25;
        if constexpr (sizeof(R) == 8) {
            t2 = t * t;
            t = t * (5.0 - r2 * (t2 * t2)) * 0.25;
        }
        xp = a.ax[j] * t;
        yp = a.by[i] * t;
    } else {
        xp = x;
        yp = y;
    }
    const double qx = xp * a.inv_dfx + a.qx0;   // (x' - K_c D_F) / D_F + M/2
    const double qy = yp * a.inv_dfy + a.qy0;
    const double fx = floor(qx), fy = floor(qy);
    const int ix = (int)fx - 1, iy = (int)fy - 1;
    R wx[4], wy[4];
    keys4<R>(R(qx - fx), wx);
    keys4<R>(R(qy - fy), wy);
    cpx<R> acc = mk(R(0), R(0));
    if (sizeof(R) == 4 && ix >= 0 && ix + 3 < a.mx && iy >= 0 && iy + 3 < a.my) {
        // interior: each row's four taps are two 16-byte loads
        typedef R pair_t __attribute__((ext_vector_type(4), aligned(8)));
        pair_t q[4][2];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const cpx<R>* row = a.F + (int64_t)(iy + b) * a.mx + ix;
            q[b][0] = *reinterpret_cast<const pair_t*>(row);
            q[b][1] = *reinterpret_cast<const pair_t*>(row + 2);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const cpx<R> racc = mk(q[b][0].x, q[b][0].y) * wx[0] + mk(q[b][0].z, q[b][0].w) * wx[1] +
                                mk(q[b][1].x, q[b][1].y) * wx[2] + mk(q[b][1].z, q[b][1].w) * wx[3];
            acc = acc + racc * wy[b];
        }
    } else {
        // taps outside the FrT grid get weight 0 and read a clamped (in-bounds) sample: no branches,
        // so the 16 loads are in flight together
        int cols[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = ix + c;
            wx[c] = (col >= 0 && col < a.mx) ? wx[c] : R(0);
            cols[c] = min(max(col, 0), a.mx - 1);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = iy + b;
            const R wb = (r >= 0 && r < a.my) ? wy[b] : R(0);
            const cpx<R>* row = a.F + (int64_t)min(max(r, 0), a.my - 1) * a.mx;
            cpx<R> racc = mk(R(0), R(0));
#pragma unroll
            for (int c = 0; c < 4; ++c) racc = racc + row[cols[c]] * wx[c];
            acc = acc + racc * wb;
        }
    }
    // outer chirp, phase in float64
    R sn, cs;
    sincos_phase<R>((xp * xp + yp * yp) * a.kz2, &sn, &cs);
    cpx<R> o = acc * mk(cs, sn);
    if (a.conj_out) o.y = -o.y;
    a.out[(int64_t)i * a.sx + j] = o;
}

template <typename R>
hipError_t launch_output_gather(const OutputArgs<R>& a, hipStream_t st) {
    dim3 block(64, 4);
    dim3 grid((a.sx + 63) / 64, (a.sy + 3) / 4);
    hipLaunchKernelGGL(output_gather_kernel<R>, grid, block, 0, st, a);
    return hipGetLastError();
}
template hipError_t launch_output_gather<float>(const OutputArgs<float>&, hipStream_t);
template hipError_t launch_output_gather<double>(const OutputArgs<double>&, hipStream_t);

// ------------------------------------------------------------ test input
// H[i][j] = sum_p a_p exp(i (k r + phi_p)) / r in float64, rounded to R on store.
template <typename R>
__global__ void synth_kernel(const double* __restrict__ pts, int np, int nx, int ny, double pitch, double k,
                             cpx<R>* __restrict__ out) {
    __shared__ double sp[5 * 256];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const double x = (double)(j - (nx >> 1)) * pitch;
    const double y = (double)(i - (ny >> 1)) * pitch;
    double re = 0.0, im = 0.0;
    for (int p0 = 0; p0 < np; p0 += 256) {
        const int cnt = min(256, np - p0);
        __syncthreads();
        for (int t = threadIdx.x; t < 5 * cnt; t += blockDim.x) sp[t] = pts[5 * p0 + t];
        __syncthreads();
        if (j < nx) {
            for (int p = 0; p < cnt; ++p) {
                const double dx = x - sp[5 * p], dy = y - sp[5 * p + 1], zp = sp[5 * p + 2];
                const double r = sqrt(dx * dx + dy * dy + zp * zp);
                double sn, cs;
                sincos(k * r + sp[5 * p + 4], &sn, &cs);
                const double amp = sp[5 * p + 3] / r;
                re = fma(amp, cs, re);
                im = fma(amp, sn, im);
            }
        }
    }
    if (j < nx) out[(int64_t)i * nx + j] = mk(R(re), R(im));
}

template <typename R>
hipError_t launch_synth(const double* d_pts, int np, int nx, int ny, double pitch, double k, cpx<R>* out,
                        hipStream_t st) {
    dim3 block(256);
    dim3 grid((nx + 255) / 256, ny);
    hipLaunchKernelGGL(synth_kernel<R>, grid, block, 0, st, d_pts, np, nx, ny, pitch, k, out);
    return hipGetLastError();
}
template hipError_t launch_synth<float>(const double*, int, int, int, double, double, cpx<float>*, hipStream_t);
template hipError_t launch_synth<double>(const double*, int, int, int, double, double, cpx<double>*, hipStream_t);

}  // namespace nufds
