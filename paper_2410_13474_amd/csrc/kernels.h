// Launch helpers of the non-FFT kernels of libnufds.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"
#include "special.h"

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
// The entries are processed in 16 x 16 tiles aligned to the table (tile (tx, ty) covers |k_gx| in
// [16 tx, 16 tx + 16), |k_gy| in [16 ty, 16 ty + 16)); tx0 .. tx0 + ntx - 1 and ty0 .. ty0 + nty - 1
// cover the rectangle ax0 .. ax0 + nax - 1, ay0 .. ay0 + nay - 1 of the entries the band needs.
template <typename R>
struct GatherArgs {
    const cpx<R>* spec;   // [ny][nx], centred
    cpx<R>* out;          // [my][mx]
    const double* table;  // [kyt + 1][kxt + 1] pairs, NaN = masked
    const int4* bounds;   // per tile of the table (see map_table_bytes)
    int kxt, kyt;
    int tbx, tby;         // tiles of the table per row and per column
    int nx, ny, mx, my;
    int gx0, gy0;         // k_g of band sample (0, 0): K_c - M/2
    int ax0, ay0, nax, nay;
    int tx0, ty0, ntx, nty;
    int nostretch;
    int sigma;            // spectral grid of the spectrum relative to the table's (1 or 2)
};

constexpr int kGatherTile = 16;

// Layout of a stretch-map table: [kyt + 1][kxt + 1] float64 pairs (the pre-image P of every quadrant
// entry, in samples of the hologram's spectral grid), then one int4 per 16 x 16 tile of entries,
// row-major over ceil((kxt + 1) / 16) tiles per row: the least and greatest first Keys tap
// floor(sigma P) - 1 over the tile's valid entries on a spectral grid sigma times as fine (sigma = 1,
// or 2 for an oversampled spectrum), in samples from the spectrum centre, {min x, max x, min y,
// max y}; min x = INT_MAX for a tile with no valid entry.
inline int map_tiles_x(int kxt) { return (kxt + kGatherTile) / kGatherTile; }
inline int map_tiles_y(int kyt) { return (kyt + kGatherTile) / kGatherTile; }
inline size_t map_entries_bytes(int kxt, int kyt) { return (size_t)(kxt + 1) * (kyt + 1) * 2 * sizeof(double); }
inline size_t map_table_bytes(int kxt, int kyt) {
    return map_entries_bytes(kxt, kyt) + (size_t)map_tiles_x(kxt) * map_tiles_y(kyt) * sizeof(int4);
}

template <typename R>
hipError_t launch_stretch_gather(const GatherArgs<R>& a, hipStream_t st);

// Fills a table of map_table_bytes(kxt, kyt) bytes: the entries, then the tile bounds for a spectrum
// on a grid sigma times as fine as the hologram's.  poly: the paper's polynomial model of Eq. 16
// instead of the exact map (NULL: exact).
hipError_t launch_map_table(double* table, int kxt, int kyt, double wavelength, double npx, double npy,
                            double s, int sigma, const PaperPoly* poly, hipStream_t st);

template <typename R>
hipError_t launch_output_gather(const OutputArgs<R>& a, hipStream_t st);

template <typename R>
hipError_t launch_synth(const double* d_pts, int np, int nx, int ny, double pitch, double k, cpx<R>* out,
                        hipStream_t st);

}  // namespace nufds
