// Map-table, output-gather and test-input kernels of libnufds (gfx950).
#include "kernels.h"

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
        const double rr = sqrt(x * x + y * y + a.z * a.z);
        const double rs = 1.0 / sqrt(rr);
        xp = a.ax[j] * rs;
        yp = a.by[i] * rs;
    } else {
        xp = x;
        yp = y;
    }
    const double qx = (xp - a.kcx * a.dfx) / a.dfx + (double)(a.mx >> 1);
    const double qy = (yp - a.kcy * a.dfy) / a.dfy + (double)(a.my >> 1);
    const double fx = floor(qx), fy = floor(qy);
    const int ix = (int)fx - 1, iy = (int)fy - 1;
    R wx[4], wy[4];
    keys4<R>(R(qx - fx), wx);
    keys4<R>(R(qy - fy), wy);
    cpx<R> acc = mk(R(0), R(0));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = iy + b;
        if (r < 0 || r >= a.my) continue;
        const cpx<R>* row = a.F + (int64_t)r * a.mx;
        cpx<R> racc = mk(R(0), R(0));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = ix + c;
            if (col >= 0 && col < a.mx) racc = racc + row[col] * wx[c];
        }
        acc = acc + racc * wy[b];
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
