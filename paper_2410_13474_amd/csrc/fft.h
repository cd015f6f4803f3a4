// Batched Stockham FFT passes for gfx950, with fused loads and stores.
//
// One pass transforms a tile of W independent sequences of length L held in LDS
// (layout [n][w]); threads hold whole radix-r butterflies in registers between
// two barriers, so a single LDS buffer serves every stage.  Nine pass kinds cover
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
//   ROWC          a whole complex64 row (transform or chain) too long for a complex tile:
//                 the row in registers, exchanged between stages through LDS as a plane of
//                 real parts and then one of imaginary parts.
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
    K_ROWBA = 6, K_COLBA = 7, // B pass of one transform, chain multiply, A pass of the next
    K_ROWC = 8                // whole transform or chain along rows too long for a complex tile (complex64)
};

// LDS index of tile element i = n W + w.  Narrow tiles (PAD) insert one pad element every 32 to
// break the power-of-two strides of the Stockham writes across the LDS banks; tiles of 8 or more
// columns keep adjacent lanes on adjacent words and need none.
template <bool PAD>
__host__ __device__ __forceinline__ int lds_index(int i) { return PAD ? i + (i >> 5) : i; }
__host__ __device__ __forceinline__ int lds_elems(int n) { return n + (n >> 5) + 1; }

constexpr int kXcds = 8;  // MI355X: 8 XCDs, each with its own L2

constexpr int kMaxStages = 16;
constexpr int kMaxBfly = 4;  // butterflies a thread holds in one stage, at most

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
    int one_bfly;   // 1: one butterfly per thread per stage (small tiles)
};

// Elements a thread may hold in registers during one stage of the several-butterflies variant
// (with 1024 threads: single-pass tiles of up to 16384 complex64 or 8192 complex128 elements).
template <typename R> struct MaxElems { static constexpr int value = 16; };
template <> struct MaxElems<double> { static constexpr int value = 8; };
// Largest radix of the one-butterfly-per-thread variant.
template <typename R> struct OneBflyElems { static constexpr int value = 16; };
template <> struct OneBflyElems<double> { static constexpr int value = 16; };
// Largest workgroup of the one-butterfly variant (complex128: 512, leaving 256 registers per lane).
template <typename R> struct OneBflyThreads { static constexpr int value = 1024; };
template <> struct OneBflyThreads<double> { static constexpr int value = 512; };

// ---------------------------------------------------------------- loads

// Source of a pass: in[offset], optionally conjugated, times (-1)^(index along the transformed axis)
// if sign_axis, times scale, times mul[index along the transformed axis] if mul is set (first pass of
// a transform only: the per-axis chirp of a cached band).  With win_lo < win_hi (first pass only),
// elements whose index along the axis lies outside [win_lo, win_hi) are zero and are not read: a
// zero-padded input held without its padding.  In a one-pass row transform (K_ROWC, not a chain)
// mul holds the vector in factored form: for the first-stage radix R and LR = L/R, the pairs
// (c_j, a_j), j < LR, then b_t, t < R, with mul[j + t LR] = c_j a_j^t b_t (a chirp factors so).
template <typename R>
struct LoadPlain {
    const cpx<R>* in;
    int conj;
    int sign_axis;
    R scale;
    int plain;  // no conjugation, sign, scale or multiply: the load is a copy
    const cpx<R>* mul;
    int win_lo, win_hi;
};

// ---------------------------------------------------------------- stores

// Destination of a pass: out[offset] = v * scale * ((-1)^(index along the axis) if sign_axis).
template <typename R>
struct StorePlain {
    cpx<R>* out;
    int sign_axis;
    R scale;
    int plain;  // no sign or scale: the store is a copy
};

// Element-wise factor between the two transforms of a chain pass: vec[n cn + w cw + c0] (the
// caller folds any scale into the vector).
template <typename R>
struct ChainMul {
    const cpx<R>* vec;
};

// ---------------------------------------------------------------- host side

struct FftTables;  // per-length twiddle tables, owned by a plan

template <typename R>
hipError_t launch_pass(const PassDesc& d, const LoadPlain<R>& ld, const StorePlain<R>& st, const cpx<R>* tw,
                       const cpx<R>* twf, const cpx<R>* chainvec, hipStream_t s);

// Radix sequence of a 5-smooth length with the fewest stages (radices 2-6, 8-10, 12, 15, 16 up to
// max_radix); false if there is none.
bool factor_radices(int L, int* nst, int* rad, int max_radix);

// Threads of the one-pass row kernel (a transform or a chain) for rows of L complex64 elements
// (rows whose complex tile exceeds LDS but whose real-part plane fits), or 0 if there is none for L.
int row_chain_threads(int L);
// Radix of that kernel's first stage: a thread loads elements j + t L/R of its row, t < R.
int row_chain_first_radix(int L);

// Whether the 32-bit per-lane offsets of the pass's global accesses can address its tiles.
bool pass_offsets_fit(const PassDesc& d, int esize);

// Threads per block such that no thread holds more than the register budget in any stage.
int pick_threads(int L, int W, int nst, const int* rad, int max_elems);
// Threads for one butterfly per thread per stage, or -1 if a stage has more than max_threads butterflies.
int pick_threads_one(int L, int W, int nst, const int* rad, int max_threads);

}  // namespace nufds
