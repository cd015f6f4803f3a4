// Stockham FFT pass kernel (gfx950) and its launch helpers.
#include "fft.h"

#include <cmath>

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

// One Stockham stage of radix RAD over the LDS tile (Govindaraju et al., SC 2008 formulation):
// butterfly j reads x[j + t L/RAD], twiddles by w_(Ns RAD)^(t k), k = j mod Ns, and writes
// (j / Ns) Ns RAD + k + t Ns.  All reads happen before the barrier, all writes after.
template <typename R, int RAD, int MAXE>
__device__ __forceinline__ void fft_stage(cpx<R>* lds, int L, int lw, int Ns, const cpx<R>* __restrict__ tw,
                                          int sign, int tid, int T) {
    constexpr int NB = MAXE / RAD;
    // per-stage opaque copy of the thread index: keeps the compiler from hoisting every
    // butterfly's LDS addresses out of the stage loop (they would stay live across all stages)
    int tid_s = tid;
    asm volatile("" : "+v"(tid_s));
    const int W = 1 << lw;
    const int LR = L / RAD;
    const int B = LR << lw;
    const int tstride = L / (Ns * RAD);
    const float inv = 1.0f / (float)Ns;
    cpx<R> v[NB][RAD];
    cpx<R> cw[NB];
    // reads: LDS inputs and the butterfly's twiddle, all issued before the barrier and without
    // branches (butterflies past B read butterfly 0 and are not written back)
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b0 = tid_s + i * T;
        const int b = b0 < B ? b0 : 0;
        const int w = b & (W - 1), j = b >> lw;
        const int q = fdiv(j, Ns, inv);
        const int k = j - q * Ns;
        cw[i] = tw[k * tstride];
#pragma unroll
        for (int t = 0; t < RAD; ++t) v[i][t] = lds[lds_pad(((j + t * LR) << lw) + w)];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid_s + i * T;
        if (b < B) {
            const int w = b & (W - 1), j = b >> lw;
            const int q = fdiv(j, Ns, inv);
            const int k = j - q * Ns;
            cpx<R> c = cw[i];
            if (sign > 0) c.y = -c.y;
            if (sizeof(R) == 4) {
                cpx<R> wp[RAD];
                twiddle_powers<R, RAD>(c, wp);
#pragma unroll
                for (int t = 1; t < RAD; ++t) v[i][t] = v[i][t] * wp[t];
            } else {
                // float64: a running product (<= RAD - 2 roundings, ~1e-15) keeps registers free
                cpx<R> p = c;
#pragma unroll
                for (int t = 1; t < RAD; ++t) {
                    v[i][t] = v[i][t] * p;
                    if (t + 1 < RAD) p = p * c;
                }
            }
            SmallDft<R, RAD>::run(v[i], sign);
            const int base = q * Ns * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t)
                lds[lds_pad(((base + t * Ns) << lw) + w)] = v[i][SmallDft<R, RAD>::perm(t)];
        }
    }
    __syncthreads();
}

template <typename R, int MAXE>
__device__ __forceinline__ void fft_tile(cpx<R>* lds, const PassDesc& d, const cpx<R>* __restrict__ tw, int sign,
                                         int tid, int T) {
    int Ns = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int r = d.rad[s];
        switch (r) {
            case 16: fft_stage<R, 16, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
            case 8: fft_stage<R, 8, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
            case 4: fft_stage<R, 4, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
            case 2: fft_stage<R, 2, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
            case 5: fft_stage<R, 5, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
            default: fft_stage<R, 3, MAXE>(lds, d.L, d.logW, Ns, tw, sign, tid, T); break;
        }
        Ns *= r;
    }
}

// Affine description of one tile: element (n, w) lives at base + n sn + w sw; its index along the
// transformed axis is n an + w aw + a0 (input) or k bn + w bw + b0 (output); the chain multiply of a
// fused pass reads the vector at n cn + w cw + c0; the transverse index is t0 + w t1; the four-step
// twiddle exponent of the store is (m0 + w m1) k.
struct TileMap {
    int64_t ib, isn, isw, ob, osn, osw;
    int an, aw, a0, bn, bw, b0, cn, cw, c0, t0, t1, m0, m1;
    int wvalid;
    bool in_nfast, out_nfast, twiddle;
};

__device__ __forceinline__ TileMap tile_map(const PassDesc& d, int a, int b) {
    TileMap m;
    const int W = d.W;
    m.twiddle = false;
    m.m0 = m.m1 = 0;
    m.cn = 1; m.cw = 0; m.c0 = 0;
    switch (d.kind) {
        case K_ROW1: {
            int r0 = a * W;
            m.wvalid = min(W, d.rows - r0);
            m.ib = r0 * d.in_pitch; m.isn = 1; m.isw = d.in_pitch;
            m.ob = r0 * d.out_pitch; m.osn = 1; m.osw = d.out_pitch;
            m.an = 1; m.aw = 0; m.a0 = 0; m.bn = 1; m.bw = 0; m.b0 = 0; m.t0 = r0; m.t1 = 1;
            m.in_nfast = m.out_nfast = true;
            break;
        }
        case K_COL1: {
            int c0 = b * W;
            m.wvalid = min(W, d.cols - c0);
            m.ib = c0; m.isn = d.in_pitch; m.isw = 1;
            m.ob = c0; m.osn = d.out_pitch; m.osw = 1;
            m.an = 1; m.aw = 0; m.a0 = 0; m.bn = 1; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_ROWA: {
            int row = a, n20 = b * W;
            m.wvalid = min(W, d.L2 - n20);
            m.ib = row * d.in_pitch + n20; m.isn = d.L2; m.isw = 1;
            m.ob = row * d.out_pitch + n20; m.osn = d.L2; m.osw = 1;
            m.an = d.L2; m.aw = 1; m.a0 = n20; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = row; m.t1 = 0;
            m.twiddle = true; m.m0 = n20; m.m1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_ROWB: {
            int row = a, k10 = b * W;
            m.wvalid = min(W, d.L1 - k10);
            m.ib = row * d.in_pitch + (int64_t)k10 * d.L2; m.isn = 1; m.isw = d.L2;
            m.ob = row * d.out_pitch + k10; m.osn = d.L1; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = d.L1; m.bw = 1; m.b0 = k10; m.t0 = row; m.t1 = 0;
            m.in_nfast = true; m.out_nfast = false;
            break;
        }
        case K_ROWBA: {
            // input as ROWB (k1 = k10 + w, n over k2); output position q1 L1 + k1 with twiddle w^(k1 q1)
            int row = a, k10 = b * W;
            m.wvalid = min(W, d.L1 - k10);
            m.ib = row * d.in_pitch + (int64_t)k10 * d.L2; m.isn = 1; m.isw = d.L2;
            m.ob = row * d.out_pitch + k10; m.osn = d.L1; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = row; m.t1 = 0;
            m.cn = d.L1; m.cw = 1; m.c0 = k10;
            m.twiddle = true; m.m0 = k10; m.m1 = 1;
            m.in_nfast = true; m.out_nfast = false;
            break;
        }
        case K_COLA: {
            int n2 = a, c0 = b * W;
            m.wvalid = min(W, d.cols - c0);
            m.ib = n2 * d.in_pitch + c0; m.isn = (int64_t)d.L2 * d.in_pitch; m.isw = 1;
            m.ob = n2 * d.out_pitch + c0; m.osn = (int64_t)d.L2 * d.out_pitch; m.osw = 1;
            m.an = d.L2; m.aw = 0; m.a0 = n2; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.twiddle = true; m.m0 = n2; m.m1 = 0;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        case K_COLB: {
            int k1 = a, c0 = b * W;
            m.wvalid = min(W, d.cols - c0);
            m.ib = (int64_t)k1 * d.L2 * d.in_pitch + c0; m.isn = d.in_pitch; m.isw = 1;
            m.ob = k1 * d.out_pitch + c0; m.osn = (int64_t)d.L1 * d.out_pitch; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = d.L1; m.bw = 0; m.b0 = k1; m.t0 = c0; m.t1 = 1;
            m.in_nfast = m.out_nfast = false;
            break;
        }
        default: {  // K_COLBA: input as COLB, output row q1 L1 + k1 with twiddle w^(k1 q1)
            int k1 = a, c0 = b * W;
            m.wvalid = min(W, d.cols - c0);
            m.ib = (int64_t)k1 * d.L2 * d.in_pitch + c0; m.isn = d.in_pitch; m.isw = 1;
            m.ob = k1 * d.out_pitch + c0; m.osn = (int64_t)d.L1 * d.out_pitch; m.osw = 1;
            m.an = 0; m.aw = 0; m.a0 = 0; m.bn = 0; m.bw = 0; m.b0 = 0; m.t0 = c0; m.t1 = 1;
            m.cn = d.L1; m.cw = 0; m.c0 = k1;
            m.twiddle = true; m.m0 = k1; m.m1 = 0;
            m.in_nfast = m.out_nfast = false;
            break;
        }
    }
    return m;
}

template <typename R, typename LD>
__global__ void __launch_bounds__(1024) fft_pass_kernel(PassDesc d, LD ld, StorePlain<R> st,
                                                        const cpx<R>* __restrict__ tw,
                                                        const cpx<R>* __restrict__ twf,
                                                        const cpx<R>* __restrict__ chainvec, R chainscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    constexpr int MAXE = MaxElems<R>::value;
    const int tid = threadIdx.x, T = blockDim.x;
    const int L = d.L, lw = d.logW, W = 1 << lw;
    const int E = L << lw;
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
    const float invL = 1.0f / (float)L;

    // global -> LDS in rounds of LD::batch elements per thread.  The loads carry no branches
    // (padding elements load the tile's first element and are zeroed), so all loads of a round are
    // in flight together before its LDS stores.
    constexpr int G = LD::batch;
    for (int r0 = 0; r0 < E; r0 += G * T) {
        cpx<R> buf[G];
        int dst[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int e0 = r0 + tid + i * T;
            const int e = e0 < E ? e0 : 0;
            int n, w;
            if (m.in_nfast) { w = fdiv(e, L, invL); n = e - w * L; }
            else { w = e & (W - 1); n = e >> lw; }
            const bool valid = e0 < E && w < m.wvalid;
            const int nn = valid ? n : 0, ww = valid ? w : 0;
            buf[i] = ld(m.ib + nn * m.isn + ww * m.isw, n * m.an + w * m.aw + m.a0, m.t0 + w * m.t1, valid);
            dst[i] = e0 < E ? lds_pad((n << lw) + w) : -1;
        }
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (dst[i] >= 0) lds[dst[i]] = buf[i];
    }
    __syncthreads();

    fft_tile<R, MAXE>(lds, d, tw, d.sign, tid, T);
    int osign = d.sign;
    if (d.chain) {
        // element-wise multiply by the chain vector (the chirp of Eq. 2), vector loads batched
        constexpr int GC = MaxElems<R>::value / 2;
        for (int r0 = 0; r0 < E; r0 += GC * T) {
            cpx<R> cv[GC];
#pragma unroll
            for (int i = 0; i < GC; ++i) {
                const int e0 = r0 + tid + i * T;
                const int e = e0 < E ? e0 : 0;
                const int w = e & (W - 1), n = e >> lw;
                cv[i] = chainvec[n * m.cn + w * m.cw + m.c0];
            }
#pragma unroll
            for (int i = 0; i < GC; ++i) {
                const int e = r0 + tid + i * T;
                if (e < E) {
                    const int p = lds_pad(e);
                    lds[p] = lds[p] * cv[i] * chainscale;
                }
            }
        }
        __syncthreads();
        osign = -d.sign;
        fft_tile<R, MAXE>(lds, d, tw, osign, tid, T);
    }

    // LDS -> global in rounds: the LDS reads and twiddle loads of a round are issued first (no
    // branches), then its stores
    constexpr int GS = MaxElems<R>::value / 2;
    for (int r0 = 0; r0 < E; r0 += GS * T) {
        cpx<R> buf[GS];
        cpx<R> cw[GS];
#pragma unroll
        for (int i = 0; i < GS; ++i) {
            const int e0 = r0 + tid + i * T;
            const int e = e0 < E ? e0 : 0;
            int k, w;
            if (m.out_nfast) { w = fdiv(e, L, invL); k = e - w * L; }
            else { w = e & (W - 1); k = e >> lw; }
            buf[i] = lds[lds_pad((k << lw) + w)];
            // exponent < L1 L2 = Lf: the digit products of a four-step split never wrap
            const int ex = (m.twiddle && w < m.wvalid) ? (m.m0 + w * m.m1) * k : 0;
            cw[i] = m.twiddle ? twf[ex] : mk(R(1), R(0));
        }
#pragma unroll
        for (int i = 0; i < GS; ++i) {
            const int e = r0 + tid + i * T;
            if (e < E) {
                int k, w;
                if (m.out_nfast) { w = fdiv(e, L, invL); k = e - w * L; }
                else { w = e & (W - 1); k = e >> lw; }
                cpx<R> c = cw[i];
                if (osign > 0) c.y = -c.y;
                if (w < m.wvalid)
                    st(m.ob + k * m.osn + w * m.osw, k * m.bn + w * m.bw + m.b0, m.t0 + w * m.t1, buf[i] * c);
            }
        }
    }
}

template <typename R, typename LD>
hipError_t launch_pass(const PassDesc& d, const LD& ld, const StorePlain<R>& st, const cpx<R>* tw,
                       const cpx<R>* twf, const cpx<R>* chainvec, R chainscale, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_pass_kernel<R, LD>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    size_t shm = (size_t)lds_elems(d.L * d.W) * sizeof(cpx<R>);
    const int ga = d.xcd_rows ? kXcds * ((d.tiles_a + kXcds - 1) / kXcds) : d.tiles_a;
    dim3 grid(d.tiles_b, ga), block(d.nthreads);
    hipLaunchKernelGGL((fft_pass_kernel<R, LD>), grid, block, shm, s, d, ld, st, tw, twf, chainvec, chainscale);
    return hipGetLastError();
}

template hipError_t launch_pass<float, LoadPlain<float>>(const PassDesc&, const LoadPlain<float>&,
                                                         const StorePlain<float>&, const cpx<float>*,
                                                         const cpx<float>*, const cpx<float>*, float, hipStream_t);
template hipError_t launch_pass<double, LoadPlain<double>>(const PassDesc&, const LoadPlain<double>&,
                                                           const StorePlain<double>&, const cpx<double>*,
                                                           const cpx<double>*, const cpx<double>*, double,
                                                           hipStream_t);
template hipError_t launch_pass<float, LoadGather<float>>(const PassDesc&, const LoadGather<float>&,
                                                          const StorePlain<float>&, const cpx<float>*,
                                                          const cpx<float>*, const cpx<float>*, float,
                                                          hipStream_t);
template hipError_t launch_pass<double, LoadGather<double>>(const PassDesc&, const LoadGather<double>&,
                                                            const StorePlain<double>&, const cpx<double>*,
                                                            const cpx<double>*, const cpx<double>*, double,
                                                            hipStream_t);

bool factor_radices(int L, int* nst, int* rad) {
    int n = 0, m = L;
    const int order[6] = {16, 8, 4, 2, 5, 3};
    for (int r : order) {
        while (m % r == 0) {
            if (n >= kMaxStages) return false;
            rad[n++] = r;
            m /= r;
        }
    }
    *nst = n;
    return m == 1;
}

int pick_threads(int L, int W, int nst, const int* rad, int max_elems) {
    for (int T = 64; T <= 1024; T += 64) {
        bool ok = true;
        for (int s = 0; s < nst && ok; ++s) {
            int r = rad[s];
            int B = (L / r) * W;
            int per = (B + T - 1) / T;
            if (per > max_elems / r) ok = false;
        }
        if (ok) return T;
    }
    return -1;
}

}  // namespace nufds
