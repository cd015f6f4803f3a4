// Map-table, output-gather and test-input kernels of libnufds (gfx950).
#include "kernels.h"

#include <climits>

#include "special.h"

namespace nufds {

// ------------------------------------------------------------ step 1: stretch map
// Entry (ky, kx) of the quadrant table holds the pre-image, in spectral samples from the
// centre, of the stretched frequency (kx / (N_x D), ky / (N_y D)) under Eqs. 9-10 with Eq. 16:
// (u N_x D / lambda, v N_y D / lambda), or NaN when there is no pre-image on the propagating
// disk or it falls outside the hologram band |u|, |v| <= lambda / (2 D).
__global__ void map_table_kernel(double* __restrict__ table, int kxt, int kyt, double wavelength,
                                 double npx, double npy, double s) {
    const int kx = blockIdx.x * blockDim.x + threadIdx.x;
    const int ky = blockIdx.y * blockDim.y + threadIdx.y;
    if (kx > kxt || ky > kyt) return;
    const double t1 = (double)kx * wavelength / npx;
    const double t2 = (double)ky * wavelength / npy;
    double u, v;
    double px = __builtin_nan(""), py = __builtin_nan("");
    if (stretch_preimage(t1, t2, &u, &v) && u <= s && v <= s) {
        px = u * (npx / wavelength);
        py = v * (npy / wavelength);
    }
    const int64_t e = (int64_t)ky * (kxt + 1) + kx;
    table[2 * e] = px;
    table[2 * e + 1] = py;
}

hipError_t launch_map_table(double* table, int kxt, int kyt, double wavelength, double npx, double npy,
                            double s, hipStream_t st) {
    dim3 block(64, 4);
    dim3 grid((kxt + 1 + 63) / 64, (kyt + 1 + 3) / 4);
    hipLaunchKernelGGL(map_table_kernel, grid, block, 0, st, table, kxt, kyt, wavelength, npx, npy, s);
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
// Keys 4 x 4 from a window of the spectrum held in LDS ([rows][wx]; taps at r0..r0+3, c0..c0+3).
template <typename R>
__device__ __forceinline__ cpx<R> keys_window(const cpx<R>* w, int wx, int c0, int r0, const R* kx, const R* ky) {
    cpx<R> acc = mk(R(0), R(0));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const cpx<R>* row = w + (r0 + b) * wx + c0;
        const cpx<R> racc = row[0] * kx[0] + row[1] * kx[1] + row[2] * kx[2] + row[3] * kx[3];
        acc = acc + racc * ky[b];
    }
    return acc;
}

// One workgroup covers a 16 x 16 tile of quadrant entries.  The pre-images of a tile lie within about
// 20 x 20 spectral samples (the inverse stretch contracts), so the workgroup first copies the four
// mirrored spectrum windows under its stencils into LDS with plain row loads and then interpolates
// from LDS: each spectrum sample is fetched once per tile instead of once per tap, which relieves the
// texture-address unit that bounds a per-tap gather.  The Keys kernel is even, so the mirror -p uses
// the weights of p in reverse order on the taps floor(-p) - 1 .. floor(-p) + 2 reflected, i.e. from
// N - (first tap of p) - 3 on; one set of weights per axis serves all four mirrors.  A tile whose
// window would not fit (none at the sizes measured) interpolates straight from global memory.
constexpr int kGatherTile = 16;
constexpr int kGatherWinX = 32;  // window columns at most (one per lane of half a wave)
constexpr int kGatherWinY = 24;  // window rows at most

template <typename R>
__global__ void __launch_bounds__(256) stretch_gather_kernel(GatherArgs<R> a) {
    constexpr int T = kGatherTile, WXM = kGatherWinX, WYM = kGatherWinY;
    // complex128 windows are held compactly in at most 512 samples (tiles measure <= 21 x 21)
    constexpr int CAP = sizeof(R) == 4 ? WXM * WYM : 512;
    constexpr int RG = 256 / WXM;             // row groups of the fill
    constexpr int K = (WYM + RG - 1) / RG;    // fill loads per thread and mirror
    __shared__ cpx<R> win[4][CAP];
    __shared__ int red[4][4];
    // consecutive tile rows to one XCD (round-robin dispatch): their windows share L2 lines
    const int nb = gridDim.x;
    const int nrows = (a.nay + T - 1) / T;
    const int lin = blockIdx.y * nb + blockIdx.x;
    const int xcd = lin % kXcds, slot = lin / kXcds;
    const int per = (nrows + kXcds - 1) / kXcds;
    const int brow = xcd * per + slot / nb;
    if (brow >= nrows) return;
    const int tid = threadIdx.x;
    const int ax = a.ax0 + (slot % nb) * T + (tid % T);
    const int ay = a.ay0 + brow * T + tid / T;
    const bool inr = ax < a.ax0 + a.nax && ay < a.ay0 + a.nay;
    double px, py;
    bool valid;
    if (a.nostretch) {
        valid = inr && ax <= (a.nx >> 1) && ay <= (a.ny >> 1);
        px = valid ? ax : 0.0;
        py = valid ? ay : 0.0;
    } else {
        valid = inr && ax <= a.kxt && ay <= a.kyt;
        const int64_t e = valid ? (int64_t)ay * (a.kxt + 1) + ax : 0;
        const double tx = a.table[2 * e], ty = a.table[2 * e + 1];
        valid = valid && tx == tx;
        // masked entries (NaN in the table, or beyond it) never reach the index arithmetic
        px = valid ? tx : 0.0;
        py = valid ? ty : 0.0;
    }
    const int hx = a.nx >> 1, hy = a.ny >> 1;
    const double fx = floor(px), fy = floor(py);
    R wgx[4], wgy[4];
    keys4<R>(R(px - fx), wgx);
    keys4<R>(R(py - fy), wgy);
    // first tap of the (+, +) mirror in spectrum indices, and its extent over the tile's valid entries
    const int ixp = (int)fx - 1 + hx, iyp = (int)fy - 1 + hy;
    int r0 = valid ? ixp : INT_MAX, r1 = valid ? -ixp : INT_MAX;
    int r2 = valid ? iyp : INT_MAX, r3 = valid ? -iyp : INT_MAX;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r0 = min(r0, __shfl_xor(r0, o));
        r1 = min(r1, __shfl_xor(r1, o));
        r2 = min(r2, __shfl_xor(r2, o));
        r3 = min(r3, __shfl_xor(r3, o));
    }
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = r0;
        red[tid >> 6][1] = r1;
        red[tid >> 6][2] = r2;
        red[tid >> 6][3] = r3;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        r0 = min(r0, red[w][0]);
        r1 = min(r1, red[w][1]);
        r2 = min(r2, red[w][2]);
        r3 = min(r3, red[w][3]);
    }
    const bool any = r0 != INT_MAX;  // uniform over the workgroup
    const int mnx = r0, mxx = -r1, mny = r2, mxy = -r3;
    // windows: x from mnx (mirror +) or nx - mxx - 3 (mirror -), wx columns; likewise y
    const int wx = mxx - mnx + 4, wy = mxy - mny + 4;
    const bool fits = any && wx <= WXM && wy <= WYM && wx * wy <= CAP;
    if (fits && sizeof(R) == 4) {
        // complex64: each lane copies two adjacent samples of a window row with one 16-byte load
        // (16 lanes per row, 16 rows per pass); a pair that would run off the spectrum's last
        // column takes its second sample from column 0 (periodic wrap)
        constexpr int PX = WXM / 2, PR = 256 / PX, KP = (WYM + PR - 1) / PR;
        typedef R pair_t __attribute__((ext_vector_type(4), aligned(8)));
        const int c = 2 * (tid % PX), rg = tid / PX;
        const bool cin = c < wx;
        pair_t tmp[4][KP];
        int gcs[4], grs[4][KP];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int sx = m & 1, sy = m >> 1;
            const int x0 = sx ? a.nx - mxx - 3 : mnx, y0 = sy ? a.ny - mxy - 3 : mny;
            int gc = x0 + (cin ? c : 0);
            gc = gc < 0 ? gc + a.nx : (gc >= a.nx ? gc - a.nx : gc);
            gcs[m] = gc;
            const int gcl = gc == a.nx - 1 ? a.nx - 2 : gc;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int r = rg + k * PR;
                int gr = y0 + (r < wy ? r : 0);  // branch-free: every thread loads in bounds
                gr = gr < 0 ? gr + a.ny : (gr >= a.ny ? gr - a.ny : gr);
                grs[m][k] = gr;
                tmp[m][k] = *reinterpret_cast<const pair_t*>(a.spec + (int64_t)gr * a.nx + gcl);
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int r = rg + k * PR;
                if (cin && r < wy) {
                    cpx<R> s0 = mk(R(tmp[m][k].x), R(tmp[m][k].y)), s1 = mk(R(tmp[m][k].z), R(tmp[m][k].w));
                    if (gcs[m] == a.nx - 1) {  // rare: the window crosses the last column
                        s0 = s1;
                        s1 = a.spec[(int64_t)grs[m][k] * a.nx];
                    }
                    win[m][r * wx + c] = s0;
                    if (c + 1 < wx) win[m][r * wx + c + 1] = s1;
                }
            }
        __syncthreads();
    } else if (fits) {
        const int c = tid % WXM, rg = tid / WXM;
        const bool cin = c < wx;
        cpx<R> tmp[4][K];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int sx = m & 1, sy = m >> 1;
            const int x0 = sx ? a.nx - mxx - 3 : mnx, y0 = sy ? a.ny - mxy - 3 : mny;
            int gc = x0 + (cin ? c : 0);
            gc = gc < 0 ? gc + a.nx : (gc >= a.nx ? gc - a.nx : gc);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = rg + k * RG;
                int gr = y0 + (r < wy ? r : 0);  // branch-free: every thread loads in bounds
                gr = gr < 0 ? gr + a.ny : (gr >= a.ny ? gr - a.ny : gr);
                tmp[m][k] = a.spec[(int64_t)gr * a.nx + gc];
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int r = rg + k * RG;
                if (cin && r < wy) win[m][r * wx + c] = tmp[m][k];
            }
        __syncthreads();
    }
    const R scale = valid ? R(1) : R(0);
    const int c0 = valid ? ixp - mnx : 0, rr0 = valid ? iyp - mny : 0;  // (+) mirror window offsets
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
        const int ky = (sy ? -ay : ay) - a.gy0;
        const bool yin = inr && ky >= 0 && ky < a.my && !(sy && ay == 0);
        R ky4[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) ky4[b] = sy ? wgy[3 - b] : wgy[b];
        // mirror row offset: (ny - iyp - 3) - (ny - mxy - 3) = mxy - iyp
        const int r0w = sy ? (valid ? mxy - iyp : 0) : rr0;
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
            const int kx = (sx ? -ax : ax) - a.gx0;
            const bool in = yin && kx >= 0 && kx < a.mx && !(sx && ax == 0);
            R kx4[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) kx4[b] = sx ? wgx[3 - b] : wgx[b];
            cpx<R> v;
            if (fits) {
                const int c0w = sx ? (valid ? mxx - ixp : 0) : c0;
                v = keys_window<R>(win[2 * sy + sx], wx, c0w, r0w, kx4, ky4);
            } else {
                // taps from global memory: first tap (+) ixp, (-) nx - ixp - 3, weights as above
                cpx<R> acc = mk(R(0), R(0));
                const int cb = sx ? a.nx - ixp - 3 : ixp, rb = sy ? a.ny - iyp - 3 : iyp;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    int r = rb + b;
                    r = r < 0 ? r + a.ny : (r >= a.ny ? r - a.ny : r);
                    cpx<R> racc = mk(R(0), R(0));
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int cc = cb + q;
                        cc = cc < 0 ? cc + a.nx : (cc >= a.nx ? cc - a.nx : cc);
                        racc = racc + a.spec[(int64_t)r * a.nx + cc] * kx4[q];
                    }
                    acc = acc + racc * ky4[b];
                }
                v = acc;
            }
            v = v * ((kx & 1) ? -scale : scale);
            if (in) a.out[(int64_t)ky * a.mx + kx] = v;
        }
    }
}

template <typename R>
hipError_t launch_stretch_gather(const GatherArgs<R>& a, hipStream_t st) {
    constexpr int T = kGatherTile;
    dim3 block(T * T);
    const int nb = (a.nax + T - 1) / T;
    const int nrows = (a.nay + T - 1) / T;
    const int per = (nrows + kXcds - 1) / kXcds;
    dim3 grid(nb, kXcds * per);
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
template <typename R>
__device__ __forceinline__ void sincos_t(R ph, R* s, R* c);
template <>
__device__ __forceinline__ void sincos_t<float>(float ph, float* s, float* c) { sincosf(ph, s, c); }
template <>
__device__ __forceinline__ void sincos_t<double>(double ph, double* s, double* c) { sincos(ph, s, c); }

template <typename R>
__global__ void output_gather_kernel(OutputArgs<R> a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (j >= a.sx || i >= a.sy) return;
    const double x = a.cx + (double)(j - (a.sx >> 1)) * a.dox;
    const double y = a.cy + (double)(i - (a.sy >> 1)) * a.doy;
    double xp, yp;
    if (a.remap) {
        // R^(-1/2) = r2^(-1/4): float seed, then two Newton steps y <- y (5 - r2 y^4) / 4 in float64
        const double r2 = x * x + y * y + a.z * a.z;
        double t = (double)rsqrtf(sqrtf((float)r2));
        double t2 = t * t;
        t = t * (5.0 - r2 * (t2 * t2)) * 0.25;
        t2 = t * t;
        t = t * (5.0 - r2 * (t2 * t2)) * 0.25;
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
    // outer chirp, phase in float64 reduced by a two-part 2 pi
    double ph = (xp * xp + yp * yp) * a.kz2;
    const double n = rint(ph * 0.15915494309189533577);
    ph = fma(-n, 6.283185307179586232, ph);
    ph = fma(-n, 2.4492935982947064e-16, ph);
    R sn, cs;
    sincos_t<R>(R(ph), &sn, &cs);
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
