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
    double cx, cy, dox, doy, dfx, dfy, z, kz2;  // kz2 = k / (2 z)
    int remap, conj_out;
};

hipError_t launch_map_table(double* table, int kxt, int kyt, double wavelength, double npx, double npy,
                            double s, hipStream_t st);

template <typename R>
hipError_t launch_output_gather(const OutputArgs<R>& a, hipStream_t st);

template <typename R>
hipError_t launch_synth(const double* d_pts, int np, int nx, int ny, double pitch, double k, cpx<R>* out,
                        hipStream_t st);

}  // namespace nufds
