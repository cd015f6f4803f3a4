// Batched Stockham FFT passes for gfx950, with fused loads and stores.
//
// One pass transforms a tile of W independent sequences of length L held in LDS
// (layout [n][w]); threads hold whole radix-r butterflies in registers between
// two barriers, so a single LDS buffer serves every stage.  Eight pass kinds cover
// the transforms of a row-major [rows][cols] array along either axis:
//   ROW1 / COL1   the whole transform in one pass (rows: W consecutive rows per
//                 tile; columns: W consecutive columns, 128-byte runs per row);
//   ROWA / ROWB,  the two passes of a four-step split L = L1 L2 (n = n1 L2 + n2):
//   COLA / COLB   A transforms over n1 and multiplies by w_L^(n2 k1); B
//                 transforms over n2 and writes k1 + L1 k2, so output is in
//                 natural order.
//   ROWBA / COLBA the B pass of one transform, an element-wise multiply at the natural
//                 index k1 + L1 k2, and the A pass of the next transform, whose split
//                 takes the factors in the other order (slow digit k2): one pass
//                 instead of two for the IDFT . chirp . DFT chain.
// Loads and stores carry the fused element-wise work of the reconstruction:
// conjugation of diverging holograms, the (-1)^n centring of the transforms, the
// stretch-gather of step 2, and the chirp of the Fresnel transform.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace nufds {

enum PassKind : int {
    K_ROW1 = 0, K_COL1 = 1,  // whole transform in one pass
    K_ROWA = 2, K_ROWB = 3,  // four-step A and B passes along rows
    K_COLA = 4, K_COLB = 5,  // ... along columns
    K_ROWBA = 6, K_COLBA = 7 // B pass of one transform, chain multiply, A pass of the next
};

// LDS index with one pad element every 32: breaks the power-of-two strides of the first
// Stockham stage and of the column tiles across the LDS banks.
__host__ __device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }
__host__ __device__ __forceinline__ int lds_elems(int n) { return n + (n >> 5) + 1; }

constexpr int kXcds = 8;  // MI355X: 8 XCDs, each with its own L2

constexpr int kMaxStages = 16;

struct PassDesc {
    int kind;
    int L;          // length transformed by this pass
    int W;          // transforms per tile (power of two)
    int logW;
    int nthreads;
    int nst;
    int rad[kMaxStages];
    int L1, L2, Lf; // four-step factors and full length
    int64_t in_pitch, out_pitch;  // elements between consecutive rows
    int rows, cols; // logical array being transformed
    int sign;       // -1 forward, +1 inverse (first transform of the pass)
    int chain;      // 1: multiply by chain vector, then transform again with the opposite sign
    int tiles_a, tiles_b;
    int xcd_rows;   // 1: hand consecutive tile rows (a) to the same XCD (L2 reuse of gathers)
};

// Elements a thread may hold in registers during one stage.
template <typename R> struct MaxElems { static constexpr int value = 32; };
template <> struct MaxElems<double> { static constexpr int value = 16; };

// ---------------------------------------------------------------- loads

// in[offset], optionally conjugated, times (-1)^axis, times scale.
template <typename R>
struct LoadPlain {
    static constexpr int batch = sizeof(R) == 4 ? 16 : 8;  // loads a thread issues before storing to LDS
    const cpx<R>* in;
    int conj;
    int sign_axis;
    R scale;
    // Branch-free: the caller passes an in-bounds offset even for padding elements (valid = false),
    // so that a thread's loads can all be in flight together.
    __device__ __forceinline__ cpx<R> operator()(int64_t off, int axis, int, bool valid) const {
        cpx<R> v = in[off];
        R s = (sign_axis && (axis & 1)) ? -scale : scale;
        s = valid ? s : R(0);
        return mk(v.x * s, (conj ? -v.y : v.y) * s);
    }
};

// Keys cubic convolution weights (a = -1/2) of the taps at floor-1 .. floor+2 for fraction t.
template <typename R>
__device__ __forceinline__ void keys4(R t, R* w) {
    R t2 = t * t, t3 = t2 * t;
    w[0] = R(-0.5) * t3 + t2 - R(0.5) * t;
    w[1] = R(1.5) * t3 - R(2.5) * t2 + R(1);
    w[2] = R(-1.5) * t3 + R(2) * t2 + R(0.5) * t;
    w[3] = R(0.5) * t3 - R(0.5) * t2;
}

// Keys 4 x 4 interpolation of the [ny][nx] spectrum at fractional sample (px, py), periodic.
template <typename R>
__device__ __forceinline__ cpx<R> keys_spectrum(const cpx<R>* __restrict__ spec, int nx, int ny, double px,
                                                double py) {
    const double fx = floor(px), fy = floor(py);
    const int ix = (int)fx - 1, iy = (int)fy - 1;
    R wx[4], wy[4];
    keys4<R>(R(px - fx), wx);
    keys4<R>(R(py - fy), wy);
    int cols[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int c = ix + a;
        c = c < 0 ? c + nx : (c >= nx ? c - nx : c);
        cols[a] = c;
    }
    cpx<R> acc = mk(R(0), R(0));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int r = iy + b;
        r = r < 0 ? r + ny : (r >= ny ? r - ny : r);
        const cpx<R>* row = spec + (int64_t)r * nx;
        cpx<R> racc = mk(R(0), R(0));
#pragma unroll
        for (int a = 0; a < 4; ++a) racc = racc + row[cols[a]] * wx[a];
        acc = acc + racc * wy[b];
    }
    return acc;
}

// Step 2 of Sec. 4, pull form: sample (trans, axis) = (k'_y, k'_x) of the sub-band sits at the
// stretched frequency index k_g = K_c + k' - M/2; its pre-image P (spectral samples from the centre)
// comes from the quadrant table (odd in each axis), and the spectrum is Keys-interpolated there,
// periodically.  NaN in the table marks "no pre-image in the propagating disk or outside the band".
// The result carries the (-1)^(k'_x) of the centred inverse transform that follows.
template <typename R>
struct LoadGather {
    static constexpr int batch = sizeof(R) == 4 ? 2 : 1;  // each element already issues 17 loads
    const cpx<R>* spec;
    const double* table;  // (P_x, P_y) pairs, [kyt + 1][kxt + 1]
    int nx, ny, kxt, kyt;
    int mx, my, kcx, kcy;
    int nostretch;
    __device__ __forceinline__ cpx<R> operator()(int64_t, int axis, int trans, bool valid) const {
        const int kgx = kcx + axis - (mx >> 1);
        const int kgy = kcy + trans - (my >> 1);
        double px, py;
        if (nostretch) {
            valid = valid && abs(kgx) <= (nx >> 1) && abs(kgy) <= (ny >> 1);
            px = valid ? kgx : 0;   // masked samples read the centre (in bounds) and are zeroed
            py = valid ? kgy : 0;
        } else {
            const int ax = abs(kgx), ay = abs(kgy);
            valid = valid && ax <= kxt && ay <= kyt;
            const int64_t e = valid ? (int64_t)ay * (kxt + 1) + ax : 0;
            const double tx = table[2 * e], ty = table[2 * e + 1];
            valid = valid && tx == tx;
            px = valid ? (kgx < 0 ? -tx : tx) : 0.0;
            py = valid ? (kgy < 0 ? -ty : ty) : 0.0;
        }
        const cpx<R> acc = keys_spectrum<R>(spec, nx, ny, px + (double)(nx >> 1), py + (double)(ny >> 1));
        const R s = valid ? ((axis & 1) ? R(-1) : R(1)) : R(0);
        return acc * s;
    }
};

// ---------------------------------------------------------------- stores

// out[offset] = v * (vec ? vec[axis] : 1) * scale * ((-1)^axis if sign_axis).
template <typename R>
struct StorePlain {
    cpx<R>* out;
    const cpx<R>* vec;
    int sign_axis;
    R scale;
    __device__ __forceinline__ void operator()(int64_t off, int axis, int, cpx<R> v) const {
        if (vec) v = v * vec[axis];
        R s = (sign_axis && (axis & 1)) ? -scale : scale;
        out[off] = v * s;
    }
};

// ---------------------------------------------------------------- host side

struct FftTables;  // per-length twiddle tables, owned by a plan

template <typename R, typename LD>
hipError_t launch_pass(const PassDesc& d, const LD& ld, const StorePlain<R>& st, const cpx<R>* tw,
                       const cpx<R>* twf, const cpx<R>* chainvec, R chainscale, hipStream_t s);

// Radix sequence of a 5-smooth length (16, 8, 4, 2 first, then 5, 3); false if not 5-smooth.
bool factor_radices(int L, int* nst, int* rad);

// Threads per block such that no thread holds more than the register budget in any stage.
int pick_threads(int L, int W, int nst, const int* rad, int max_elems);

}  // namespace nufds
