// Launch helpers of the non-FFT kernels of libnufds.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"

namespace nufds {

template <typename R>
struct OutputArgs {
    const cpx<R>* F;     // [my][mx], centring signs applied
    cpx<R>* out;         // [sy][sx]
    const double* ax;    // per-column factor A(x_j) of the output map (remap only)
    const double* by;    // per-row factor B(y_i)
    int sx, sy, mx, my, kcx, kcy;
    double cx, cy, dox, doy, z, kz2;  // kz2 = k / (2 z)
    double inv_dfx, inv_dfy;          // 1 / D_F
    double qx0, qy0;                  // M/2 - K_c: FrT index of x' = 0
    int remap, conj_out;
};

// Stand-alone stretch-gather (step 2) into the [my][mx] sub-band: one thread per quadrant-table
// entry (|k_gx|, |k_gy|) of the band's bounding box, writing each of the up to four mirrored samples
// (+-k_gx, +-k_gy) that fall inside the band, so every table entry is read once.
template <typename R>
struct GatherArgs {
    const cpx<R>* spec;   // [ny][nx], centred
    cpx<R>* out;          // [my][mx]
    const double* table;  // [kyt + 1][kxt + 1] pairs, NaN = masked
    int kxt, kyt;
    int nx, ny, mx, my;
    int gx0, gy0;         // k_g of band sample (0, 0): K_c - M/2
    int ax0, ay0, nax, nay;
    int nostretch;
};

template <typename R>
hipError_t launch_stretch_gather(const GatherArgs<R>& a, hipStream_t st);

hipError_t launch_map_table(double* table, int kxt, int kyt, double wavelength, double npx, double npy,
                            double s, hipStream_t st);

template <typename R>
hipError_t launch_output_gather(const OutputArgs<R>& a, hipStream_t st);

template <typename R>
hipError_t launch_synth(const double* d_pts, int np, int nx, int ny, double pitch, double k, cpx<R>* out,
                        hipStream_t st);

}  // namespace nufds
