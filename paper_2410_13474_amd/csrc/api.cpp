// C ABI of libnufds: plan geometry, plan lifecycle and the execute sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "fft.h"
#include "kernels.h"
#include "nufds.h"
#include "plan.h"
#include "special.h"

namespace nufds {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

nufds_status_t fail(nufds_status_t st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

nufds_status_t hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NUFDS_ERR_OUT_OF_MEMORY : NUFDS_ERR_HIP;
}

// ------------------------------------------------------------------ geometry

bool smooth5(int n) {
    if (n <= 0) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static int smooth5_even_at_least(long n) {
    if (n < 2) n = 2;
    for (long m = n;; ++m)
        if (m % 2 == 0 && smooth5((int)m)) return (int)m;
}

// x' of Eqs. 17-18 for the true point (x, y) at distance z: A(x) R^-1/2.
static double xprime(double x, double y, double z) {
    const double r = std::sqrt(x * x + y * y + z * z);
    return output_map_factor(x, z) / std::sqrt(r);
}

// Extremes of x' over the window [xlo, xhi] x [ylo, yhi]: x' grows with x and its magnitude
// falls with |y|, so both sit on the vertical edges, at the y nearest 0 when the edge lies on the
// same side as the extreme and at the farthest y otherwise.
static void xprime_extremes(double xlo, double xhi, double ylo, double yhi, double z, bool remap, double* lo,
                            double* hi) {
    if (!remap) {
        *lo = xlo;
        *hi = xhi;
        return;
    }
    const double ynear = std::min(std::max(0.0, ylo), yhi);
    const double yfar = std::fabs(ylo) > std::fabs(yhi) ? ylo : yhi;
    *hi = xprime(xhi, xhi >= 0.0 ? ynear : yfar, z);
    *lo = xprime(xlo, xlo <= 0.0 ? ynear : yfar, z);
}

nufds_status_t compute_geometry(double wavelength, double pitch, int nx, int ny, double z, const nufds_view_t* view,
                                uint32_t flags, const nufds_options_t* opt, nufds_plan_info_t* out) {
    if (!out) return fail(NUFDS_ERR_INVALID_ARG, "out is NULL");
    if (!(wavelength > 0.0) || !(pitch > 0.0) || !(z > 0.0) || !std::isfinite(wavelength) || !std::isfinite(pitch) ||
        !std::isfinite(z))
        return fail(NUFDS_ERR_INVALID_ARG, "wavelength, pitch and z must be positive and finite");
    const double s = wavelength / (2.0 * pitch);
    if (!(s < 1.0)) return fail(NUFDS_ERR_INVALID_ARG, "wavelength / (2 pitch) must be < 1");
    if (nx <= 0 || ny <= 0 || (nx & 1) || (ny & 1)) return fail(NUFDS_ERR_INVALID_ARG, "hologram sizes must be even and positive");
    if (flags & ~7u) return fail(NUFDS_ERR_INVALID_ARG, "unknown flag bits");
    std::memset(out, 0, sizeof(*out));
    const double B = 2.0 * z * std::tan(std::asin(s));
    const double dfx = wavelength * z / (nx * pitch);
    const double dfy = wavelength * z / (ny * pitch);
    double cx = 0, cy = 0, dox, doy;
    int sx, sy;
    if (!view) {
        sx = nx;
        sy = ny;
        dox = B / nx;
        doy = B / ny;
    } else {
        cx = view->center_x;
        cy = view->center_y;
        sx = view->nx;
        sy = view->ny;
        dox = view->pitch_x > 0.0 ? view->pitch_x : dfx;
        doy = view->pitch_y > 0.0 ? view->pitch_y : dfy;
        if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(dox) || !std::isfinite(doy))
            return fail(NUFDS_ERR_INVALID_ARG, "view values must be finite");
    }
    if (sx <= 0 || sy <= 0) return fail(NUFDS_ERR_INVALID_ARG, "view size must be positive");
    const double xlo = cx - 0.5 * sx * dox, xhi = cx + 0.5 * sx * dox;
    const double ylo = cy - 0.5 * sy * doy, yhi = cy + 0.5 * sy * doy;
    const double tol = 1e-9 * B;
    if (xlo < -0.5 * B - tol || xhi > 0.5 * B + tol || ylo < -0.5 * B - tol || yhi > 0.5 * B + tol)
        return fail(NUFDS_ERR_INVALID_ARG, "view window leaves the image area [-B/2, B/2]^2 of Eq. 1");
    const bool remap = !(flags & NUFDS_FLAG_NO_REMAP);
    double xl, xh, yl, yh;
    xprime_extremes(xlo, xhi, ylo, yhi, z, remap, &xl, &xh);
    xprime_extremes(ylo, yhi, xlo, xhi, z, remap, &yl, &yh);
    double padx = 0.5 * nx * pitch, pady = 0.5 * ny * pitch;
    int forced_x = 0, forced_y = 0, oversample = 1, map_model = 0;
    if (opt) {
        if (opt->oversample < 0 || opt->oversample > 2)
            return fail(NUFDS_ERR_INVALID_ARG, "oversample must be 0, 1 or 2");
        if (opt->map_model < 0 || opt->map_model > 1) return fail(NUFDS_ERR_INVALID_ARG, "map_model must be 0 or 1");
        map_model = opt->map_model;
        oversample = opt->oversample == 2 ? 2 : 1;
        if (opt->pad >= 0.0) padx = pady = opt->pad;
        forced_x = opt->frt_size_x;
        forced_y = opt->frt_size_y;
        if (forced_x < 0 || forced_y < 0 || (forced_x & 1) || (forced_y & 1))
            return fail(NUFDS_ERR_INVALID_ARG, "forced FrT sizes must be even and non-negative");
    }
    auto axis = [](double lo, double hi, double df, double pad, int forced, int* kc, int* m) {
        lo -= pad;
        hi += pad;
        const double k = std::floor(0.5 * (lo + hi) / df + 0.5);
        const double half = std::max(hi - k * df, k * df - lo) / df;
        *kc = (int)k;
        if (forced) {
            *m = forced;
        } else {
            const double need = 2.0 * std::ceil(half - 1e-9);
            *m = need > 1e9 ? -1 : smooth5_even_at_least((long)need);
        }
    };
    int kcx, kcy, mx, my;
    axis(xl, xh, dfx, padx, forced_x, &kcx, &mx);
    axis(yl, yh, dfy, pady, forced_y, &kcy, &my);
    out->nx = nx;
    out->ny = ny;
    out->sx = sx;
    out->sy = sy;
    out->mx = mx;
    out->my = my;
    out->kcx = kcx;
    out->kcy = kcy;
    out->dfx = dfx;
    out->dfy = dfy;
    out->dox = dox;
    out->doy = doy;
    out->cx = cx;
    out->cy = cy;
    out->image_size = B;
    out->xlo = xl;
    out->xhi = xh;
    out->ylo = yl;
    out->yhi = yh;
    out->padx = padx;
    out->pady = pady;
    out->flags = flags;
    out->oversample = oversample;
    out->map_model = map_model;
    // FrT columns the view reads: the taps of x' over the window (plus two samples of margin for the
    // GPU's own evaluation of the map), from a 16-column boundary; the y transform runs on these only
    if (mx > 0) {
        const double q0 = xl / dfx - kcx + mx / 2, q1 = xh / dfx - kcx + mx / 2;
        long c0 = (long)std::floor(q0) - 3, c1 = (long)std::floor(q1) + 4;
        c0 = std::max(0L, c0) / 16 * 16;
        c1 = std::min((long)mx - 1, c1);
        if (c1 < c0) c1 = c0;
        out->fcx0 = (int32_t)c0;
        out->fcxn = (int32_t)(c1 - c0 + 1);
    }
    if (mx <= 0 || my <= 0) return fail(NUFDS_ERR_UNSUPPORTED, "FrT size out of range");
    return NUFDS_OK;
}

// ------------------------------------------------------------------ plan

// Largest T(1) of the map over the band square |u|, |v| <= s of the unit disk: at u = s and the
// largest admissible |v| (T_1 grows with both |u| and |v|).
double stretch_extent(double s) {
    const double v = std::min(s, std::sqrt((1.0 - s) * (1.0 + s)));
    const double av = std::sqrt((1.0 - v) * (1.0 + v));
    const double sig = std::min(1.0, s / av);
    const double c = std::sqrt(std::max(0.0, (1.0 - sig) * (1.0 + sig)));
    return std::sqrt(av) * integral_i(sig, c);
}

// Quadrant table extent |k_g| <= floor(T_max N D / lambda) + 2 per axis: every stretched frequency
// with a pre-image in the hologram band.
void table_extent(double wavelength, double pitch, int nx, int ny, int* kxt, int* kyt) {
    const double ext = stretch_extent(wavelength / (2.0 * pitch));
    *kxt = (int)std::floor(ext * nx * pitch / wavelength) + 2;
    *kyt = (int)std::floor(ext * ny * pitch / wavelength) + 2;
}

nufds_status_t check_sizes(const nufds_plan_info_t& g) {
    const int64_t snx = (int64_t)spectrum_factor(g) * g.nx, sny = (int64_t)spectrum_factor(g) * g.ny;
    if (g.mx > kMaxLen || g.my > kMaxLen || snx > kMaxLen || sny > kMaxLen || !smooth5(g.nx) || !smooth5(g.ny))
        return fail(NUFDS_ERR_UNSUPPORTED, "sizes (the oversampled spectrum's included) must be 5-smooth and at most 65536");
    const int64_t kMaxArray = (int64_t)1 << 31;  // the FFT passes index elements with 32-bit integers
    if (snx * sny >= kMaxArray || (int64_t)g.mx * g.my >= kMaxArray || (int64_t)g.sx * g.sy >= kMaxArray)
        return fail(NUFDS_ERR_UNSUPPORTED, "hologram, FrT and output arrays must hold fewer than 2^31 elements");
    return NUFDS_OK;
}

TwiddleCache::~TwiddleCache() {
    for (auto& kv : tables) (void)hipFree(kv.second);
}

nufds_status_t dev_alloc(DevBuf& b, size_t bytes) {
    b.bytes = bytes;
    if (bytes == 0) return NUFDS_OK;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(NUFDS_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return NUFDS_OK;
}

void dev_free(DevBuf& b) {
    if (b.p && b.owned) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

static void plan_free(nufds_plan* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    dev_free(p->spec);
    dev_free(p->work1);
    dev_free(p->work2);
    dev_free(p->table);
    dev_free(p->chirp_x);
    dev_free(p->chirp_y);
    dev_free(p->chirp_xf);
    dev_free(p->ax);
    dev_free(p->by);
    p->twiddles.reset();
    if (p->done) (void)hipEventDestroy(p->done);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    delete p;
}

template <typename R>
static nufds_status_t upload_complex(DevBuf& b, const std::vector<double>& re, const std::vector<double>& im) {
    std::vector<cpx<R>> h(re.size());
    for (size_t i = 0; i < re.size(); ++i) h[i] = mk(R(re[i]), R(im[i]));
    nufds_status_t st = dev_alloc(b, h.size() * sizeof(cpx<R>));
    if (st != NUFDS_OK) return st;
    NUFDS_HIP_TRY(hipMemcpy(b.p, h.data(), b.bytes, hipMemcpyHostToDevice));
    return NUFDS_OK;
}

// exp(-2 pi i m / L), m = 0 .. L-1, in float64 then rounded; created once per length and cache.
template <typename R>
static nufds_status_t twiddle_table(nufds_plan* p, int L, const cpx<R>** out) {
    auto& tabs = p->twiddles->tables;
    auto it = tabs.find(L);
    if (it != tabs.end()) {
        *out = static_cast<const cpx<R>*>(it->second);
        return NUFDS_OK;
    }
    std::vector<cpx<R>> h(L);
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m] = mk(R(std::cos(a)), R(std::sin(a)));
    }
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, L * sizeof(cpx<R>));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(twiddles)");
    e = hipMemcpy(d, h.data(), L * sizeof(cpx<R>), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "hipMemcpy(twiddles)");
    }
    tabs[L] = d;
    *out = static_cast<const cpx<R>*>(d);
    return NUFDS_OK;
}

// The chirp exp(+i k xi^2 / 2z) of Eq. 2 at xi = (n - M/2) N D / M, phase in float64 reduced mod 2 pi,
// times 1/M: the normalisation of the centred inverse DFT that precedes it in the chain.
void chirp_vector(int M, int N, double pitch, double wavelength, double z, std::vector<double>& re,
                  std::vector<double>& im) {
    re.resize(M);
    im.resize(M);
    const double cycles_per_m2 = 1.0 / (2.0 * wavelength * z);  // k xi^2 / 2z = 2 pi xi^2 / (2 lambda z)
    for (int n = 0; n < M; ++n) {
        const double xi = (double)(n - M / 2) * (N * pitch / M);
        double cyc = xi * xi * cycles_per_m2;
        cyc -= std::floor(cyc);
        const double ph = 2.0 * M_PI * cyc;
        re[n] = std::cos(ph) / M;
        im[n] = std::sin(ph) / M;
    }
}

// chirp_vector at n = j + t LR (LR = M / R, t < R) in factored form for a one-pass row transform:
// with m = j - M/2 and D = (N pitch / M)^2 / (2 lambda z) cycles, the phase D (m + t LR)^2 is
// D m^2 + t (2 D m LR) + t^2 (D LR^2), so c[j + t LR] = c_j a_j^t b_t with c_j = c[j],
// a_j = exp(2 pi i 2 D m LR), b_t = exp(2 pi i D LR^2 t^2).  Output: (c_j, a_j) for j < LR, then b_t
// for t < R; every phase in float64 reduced mod 1 cycle.
void chirp_row_factors(int M, int N, double pitch, double wavelength, double z, int R, std::vector<double>& re,
                       std::vector<double>& im) {
    const int LR = M / R;
    const double delta = N * pitch / M;
    const double D = delta * delta / (2.0 * wavelength * z);
    re.assign(2 * (size_t)LR + R, 0.0);
    im.assign(2 * (size_t)LR + R, 0.0);
    auto put = [&](size_t i, double cyc, double scale) {
        cyc -= std::floor(cyc);
        re[i] = std::cos(2.0 * M_PI * cyc) * scale;
        im[i] = std::sin(2.0 * M_PI * cyc) * scale;
    };
    for (int j = 0; j < LR; ++j) {
        const double m = (double)(j - M / 2);
        put(2 * (size_t)j, D * m * m, 1.0 / M);
        put(2 * (size_t)j + 1, 2.0 * D * m * (double)LR, 1.0);
    }
    for (int t = 0; t < R; ++t) put(2 * (size_t)LR + t, D * (double)LR * (double)LR * (double)t * (double)t, 1.0);
}

// ---------------------------------------------------------- pass construction

struct Limits {
    size_t esize;    // bytes per complex element
    int tile_elems;  // LDS tile capacity, elements
    int row_w;       // transforms per tile of the four-step row passes
    int col_w;       // columns per tile of the plain column passes (256-byte runs)
    int chain_w;     // columns per tile of the fused column chain pass
    int max_elems;   // register budget per thread and stage
};

// NUFDS_MAX_TILE_ELEMS lowers the LDS tile capacity (tests use it to drive the four-step passes
// at small sizes); a plan reads it once, when it is created.
int tile_override() {
    const char* e = std::getenv("NUFDS_MAX_TILE_ELEMS");
    return e ? std::atoi(e) : 0;
}

// NUFDS_COL_W sets the columns per tile of the column passes (a power of two, 1-64), for tuning.
int col_w_override() {
    const char* e = std::getenv("NUFDS_COL_W");
    const int w = e ? std::atoi(e) : 0;
    return (w >= 1 && w <= 64 && (w & (w - 1)) == 0) ? w : 0;
}

static Limits limits_for(size_t esize, int cap, int colw) {
    Limits l;
    l.esize = esize;
    // logical elements whose padded LDS footprint (one pad per 32) fits in 160 KB
    l.tile_elems = (int)(((160 * 1024) / esize - 1) * 32 / 33);
    if (cap > 0) l.tile_elems = std::min(l.tile_elems, cap);
    l.row_w = 16;  // complex64 and complex128 (8 complex128 rows per tile ran the x passes 3-9% slower)
    l.col_w = colw > 0 ? colw : (esize == 8 ? 32 : 16);
    l.chain_w = esize == 8 ? 32 : 16;
    l.max_elems = esize == 8 ? 16 : 8;
    return l;
}

static int ilog2(int w) {
    int l = 0;
    while ((1 << l) < w) ++l;
    return l;
}

static bool finish_desc(PassDesc& d, const Limits& lim) {
    d.logW = ilog2(d.W);
    if ((1 << d.logW) != d.W) return false;
    if ((int64_t)d.L * d.W > lim.tile_elems) return false;  // padded LDS footprint within 160 KB
    // radices up to 16; if no thread count fits them (a radix-2 stage with too many butterflies for
    // one per thread, and radices beyond the register budget of several), radices up to 8
    for (int max_radix : {16, 8}) {
        if (!factor_radices(d.L, &d.nst, d.rad, max_radix)) return false;
        // prefer one butterfly per thread and stage; else several (long single-pass rows)
        d.nthreads = pick_threads_one(d.L, d.W, d.nst, d.rad, lim.esize == 8 ? 1024 : 512);
        d.one_bfly = d.nthreads > 0 ? 1 : 0;
        if (!d.one_bfly) d.nthreads = pick_threads(d.L, d.W, d.nst, d.rad, lim.max_elems);
        if (d.nthreads > 0) break;
    }
    if (d.nthreads <= 0) return false;
    return pass_offsets_fit(d, (int)lim.esize);
}

// Split L = L1 L2 so that both passes' tiles (L1 x W and L2 x W) fit, as balanced as possible.
static bool four_step_split(int L, int W, const Limits& lim, int* L1, int* L2) {
    int best = -1, best_span = 0;
    for (int a = 2; a < L; ++a) {
        if (L % a) continue;
        const int b = L / a;
        if ((int64_t)a * W > lim.tile_elems || (int64_t)b * W > lim.tile_elems) continue;
        const int span = std::max(a, b);
        if (best < 0 || span < best_span) {
            best = a;
            best_span = span;
        }
    }
    if (best < 0) return false;
    *L1 = best;
    *L2 = L / best;
    return true;
}

// The passes of one axis transform of a [rows][cols] array (axis 0: along rows = x; axis 1: along
// columns = y), for a single forward/inverse transform (chain = 0) or the IDFT . vec . DFT chain
// (chain = 1).  Fills 'passes'; the caller binds buffers.
struct AxisPlan {
    bool single = true;
    std::vector<PassDesc> passes;  // single: 1 pass; four-step: 2 (plain) or 4 (chain)
};

static bool build_axis(int axis, int L, int other, int64_t pitch, int sign, int chain, const Limits& lim,
                       AxisPlan* ap) {
    ap->passes.clear();
    PassDesc d{};
    d.sign = sign;
    d.in_pitch = d.out_pitch = pitch;
    d.xcd_rows = 0;
    if (axis == 0) {
        d.rows = other;
        d.cols = L;
        if (L <= lim.tile_elems) {
            d.kind = K_ROW1;
            d.L = L;
            int w = 1;
            while (w < 16 && (int64_t)L * w * 2 <= 4096 && (int64_t)L * w * 2 <= lim.tile_elems) w *= 2;
            d.W = w;
            d.chain = chain;
            d.tiles_a = (other + w - 1) / w;
            d.tiles_b = 1;
            if (finish_desc(d, lim)) {
                ap->single = true;
                ap->passes.push_back(d);
                return true;
            }  // else more elements per thread than the registers hold: four-step
        }
        if (lim.esize == 8 && L > lim.tile_elems && row_chain_threads(L) > 0) {
            // complex64 rows past the complex tile: the whole transform (or chain) in one pass, the
            // row in registers and its real and imaginary parts in turn through LDS
            d.kind = K_ROWC;
            d.L = L;
            d.W = 1;
            d.logW = 0;
            d.chain = chain;
            d.tiles_a = other;
            d.tiles_b = 1;
            d.nthreads = row_chain_threads(L);
            ap->single = true;
            ap->passes.push_back(d);
            return true;
        }
    } else {
        d.rows = L;
        d.cols = other;
        // widest column tile that holds the whole column (down to 64-byte runs)
        int w = chain ? lim.chain_w : lim.col_w;
        const int wmin = lim.esize == 8 ? 8 : 4;
        while (w > wmin && (int64_t)L * w > lim.tile_elems) w /= 2;
        if ((int64_t)L * w <= lim.tile_elems) {
            d.kind = K_COL1;
            d.L = L;
            d.W = w;
            d.chain = chain;
            d.tiles_a = 1;
            d.tiles_b = (other + d.W - 1) / d.W;
            if (finish_desc(d, lim)) {
                ap->single = true;
                ap->passes.push_back(d);
                return true;
            }
        }
    }
    // four-step: A (over n1) then B (over n2); a chain fuses the first B and the second A
    int L1, L2;
    int Wp = axis == 0 ? lim.row_w : lim.col_w;       // plain passes
    int Wc = axis == 0 ? lim.row_w : lim.chain_w;     // fused chain pass
    // narrower tiles when no split fits the wide ones (small LDS capacities)
    const int wmin = lim.esize == 8 ? 8 : 4;
    while (!four_step_split(L, std::max(Wp, Wc), lim, &L1, &L2)) {
        if (std::max(Wp, Wc) <= wmin) return false;
        Wp = std::max(wmin, Wp / 2);
        Wc = std::max(wmin, Wc / 2);
    }
    ap->single = false;
    PassDesc a = d, b = d;
    a.L1 = b.L1 = L1;
    a.L2 = b.L2 = L2;
    a.Lf = b.Lf = L;
    a.chain = b.chain = 0;
    a.W = Wp;
    b.W = chain ? Wc : Wp;
    a.L = L1;
    b.L = L2;
    if (axis == 0) {
        a.kind = K_ROWA;
        a.tiles_a = other;
        a.tiles_b = (L2 + a.W - 1) / a.W;
        b.kind = chain ? K_ROWBA : K_ROWB;
        b.tiles_a = other;
        b.tiles_b = (L1 + b.W - 1) / b.W;
    } else {
        a.kind = K_COLA;
        a.tiles_a = L2;
        a.tiles_b = (other + a.W - 1) / a.W;
        b.kind = chain ? K_COLBA : K_COLB;
        b.tiles_a = L1;
        b.tiles_b = (other + b.W - 1) / b.W;
    }
    b.chain = chain;
    if (!finish_desc(a, lim) || !finish_desc(b, lim)) return false;
    ap->passes.push_back(a);
    ap->passes.push_back(b);
    if (chain) {
        // the second transform's B pass, with the split taken as L = L2 L1
        PassDesc c = d;
        c.L1 = L2;
        c.L2 = L1;
        c.Lf = L;
        c.L = L1;
        c.W = Wp;
        c.chain = 0;
        c.sign = -sign;
        if (axis == 0) {
            c.kind = K_ROWB;
            c.tiles_a = other;
            c.tiles_b = (L2 + Wp - 1) / Wp;
        } else {
            c.kind = K_COLB;
            c.tiles_a = L2;
            c.tiles_b = (other + Wp - 1) / Wp;
        }
        if (!finish_desc(c, lim)) return false;
        ap->passes.push_back(c);
    }
    return true;
}

// ---------------------------------------------------------- execute

// Timing bracket: when the plan times its executes, record an event pair around the launch.
static nufds_status_t timing_begin(nufds_plan* p, const char* name, uint64_t bytes, hipStream_t s) {
    if (!p->recording) return NUFDS_OK;
    const size_t i = (size_t)p->nlaunch;
    while (p->ev.size() < 2 * (i + 1)) {
        hipEvent_t e;
        NUFDS_HIP_TRY(hipEventCreate(&e));
        p->ev.push_back(e);
    }
    if (p->launches.size() < i + 1) p->launches.resize(i + 1);
    nufds_kernel_time_t& k = p->launches[i];
    std::memset(&k, 0, sizeof(k));
    std::strncpy(k.name, name, sizeof(k.name) - 1);
    k.bytes = bytes;
    NUFDS_HIP_TRY(hipEventRecord(p->ev[2 * i], s));
    return NUFDS_OK;
}

static nufds_status_t timing_end(nufds_plan* p, hipStream_t s) {
    if (!p->recording) return NUFDS_OK;
    NUFDS_HIP_TRY(hipEventRecord(p->ev[2 * (size_t)p->nlaunch + 1], s));
    ++p->nlaunch;
    return NUFDS_OK;
}

// Algorithmic bytes of an FFT pass over a [rows][cols] array: every element read once and written once.
static uint64_t pass_bytes(const PassDesc& d, size_t esize) { return 2ull * d.rows * d.cols * esize; }

template <typename R>
static nufds_status_t run_pass(nufds_plan* p, const char* name, const PassDesc& d, const void* in, void* out,
                               int load_conj, int load_sign, int store_sign, R store_scale,
                               const cpx<R>* chainvec, hipStream_t s, const cpx<R>* load_mul = nullptr,
                               int win_lo = 0, int win_hi = 0) {
    const cpx<R>* tw;
    nufds_status_t st = twiddle_table<R>(p, d.L, &tw);
    if (st != NUFDS_OK) return st;
    const cpx<R>* twf = nullptr;
    if (d.kind == K_ROWA || d.kind == K_COLA || d.kind == K_ROWBA || d.kind == K_COLBA) {
        st = twiddle_table<R>(p, d.Lf, &twf);
        if (st != NUFDS_OK) return st;
    }
    LoadPlain<R> ld{static_cast<const cpx<R>*>(in), load_conj, load_sign, R(1),
                    (!load_conj && !load_sign && !load_mul) ? 1 : 0, load_mul, win_lo, win_hi};
    StorePlain<R> sto{static_cast<cpx<R>*>(out), store_sign, store_scale, (!store_sign && store_scale == R(1)) ? 1 : 0};
    NUFDS_TRY(timing_begin(p, name, pass_bytes(d, sizeof(cpx<R>)), s));
    NUFDS_HIP_TRY((launch_pass<R>(d, ld, sto, tw, twf, chainvec, s)));
    return timing_end(p, s);
}

// |k| range of band samples g0 .. g1 (inclusive) along one axis.
static void abs_range(int g0, int g1, int* lo, int* hi) {
    if (g0 <= 0 && g1 >= 0) {
        *lo = 0;
        *hi = std::max(-g0, g1);
    } else {
        *lo = std::min(std::abs(g0), std::abs(g1));
        *hi = std::max(std::abs(g0), std::abs(g1));
    }
}

template <typename R>
static nufds_status_t run_stretch_gather(nufds_plan* p, const void* spec, void* out, hipStream_t s) {
    const nufds_plan_info_t& g = p->info;
    GatherArgs<R> a;
    a.spec = static_cast<const cpx<R>*>(spec);
    a.out = static_cast<cpx<R>*>(out);
    a.table = static_cast<const double*>(p->table.p);
    a.kxt = p->kxt;
    a.kyt = p->kyt;
    a.bounds = nullptr;
    a.tbx = a.tby = 0;
    if (p->table.p) {
        a.bounds = reinterpret_cast<const int4*>(static_cast<const char*>(p->table.p) + map_entries_bytes(p->kxt, p->kyt));
        a.tbx = map_tiles_x(p->kxt);
        a.tby = map_tiles_y(p->kyt);
    }
    a.sigma = spectrum_factor(g);
    a.nx = a.sigma * g.nx;  // the spectrum's grid
    a.ny = a.sigma * g.ny;
    a.mx = g.mx;
    a.my = g.my;
    a.gx0 = g.kcx - g.mx / 2;
    a.gy0 = g.kcy - g.my / 2;
    int lo, hi;
    abs_range(a.gx0, a.gx0 + g.mx - 1, &lo, &hi);
    a.ax0 = lo;
    a.nax = hi - lo + 1;
    abs_range(a.gy0, a.gy0 + g.my - 1, &lo, &hi);
    a.ay0 = lo;
    a.nay = hi - lo + 1;
    a.tx0 = a.ax0 / kGatherTile;
    a.ty0 = a.ay0 / kGatherTile;
    a.ntx = (a.ax0 + a.nax - 1) / kGatherTile - a.tx0 + 1;
    a.nty = (a.ay0 + a.nay - 1) / kGatherTile - a.ty0 + 1;
    a.nostretch = (p->flags & NUFDS_FLAG_NO_STRETCH) ? 1 : 0;
    const uint64_t es = sizeof(cpx<R>);
    const uint64_t mm = (uint64_t)g.mx * g.my, nn = (uint64_t)a.nx * a.ny;
    const uint64_t sig2 = (uint64_t)a.sigma * a.sigma;
    NUFDS_TRY(timing_begin(p, "stretch_gather", p->table.bytes + std::min(sig2 * mm, nn) * es + mm * es, s));
    NUFDS_HIP_TRY(launch_stretch_gather<R>(a, s));
    return timing_end(p, s);
}

template <typename R>
nufds_status_t run_fft1(nufds_plan* p, const void* d_in, void* spec, void* w1, hipStream_t s) {
    const Limits lim = limits_for(sizeof(cpx<R>), p->tile_cap, p->col_w);
    const int sf = spectrum_factor(p->info);
    const int hx = p->info.nx, hy = p->info.ny;     // hologram
    const int nx = sf * hx, ny = sf * hy;            // spectrum
    // oversampled: the centred DFT of the hologram zero-padded (centred) to nx x ny.  The padding is
    // never stored: the row transforms run on the hy hologram rows only, each read as a length-nx
    // sequence that is zero outside columns ox .. ox + hx - 1, into rows oy .. oy + hy - 1 of the
    // spectrum; the column transforms read those rows and take the others as zero.
    const int ox = (nx - hx) / 2, oy = (ny - hy) / 2;
    const int xw_lo = sf > 1 ? ox : 0, xw_hi = sf > 1 ? ox + hx : 0;
    const int yw_lo = sf > 1 ? oy : 0, yw_hi = sf > 1 ? oy + hy : 0;
    // column n of a row is hologram column n - ox; the base is formed as an address (the columns
    // before the hologram lie outside the load window and are never read)
    const cpx<R>* in =
        reinterpret_cast<const cpx<R>*>(reinterpret_cast<uintptr_t>(d_in) - (uintptr_t)ox * sizeof(cpx<R>));
    cpx<R>* rows_out = static_cast<cpx<R>*>(spec) + (size_t)oy * nx;
    const int conj_in = (p->flags & NUFDS_FLAG_CONVERGING) ? 0 : 1;
    AxisPlan ap;

    // step 2a: centred forward DFT of the hologram, Ĥ[k] = (-1)^(k + N/2) DFT[(-1)^n H] per axis
    if (!build_axis(0, nx, hy, nx, -1, 0, lim, &ap)) return fail(NUFDS_ERR_UNSUPPORTED, "hologram row length");
    ap.passes[0].in_pitch = hx;  // the first row pass reads the hologram itself
    const R sgx = ((nx / 2) & 1) ? R(-1) : R(1);
    if (ap.single) {
        NUFDS_TRY(run_pass<R>(p, "fft1_row", ap.passes[0], in, rows_out, conj_in, 1, 1, sgx, nullptr, s, nullptr,
                              xw_lo, xw_hi));
    } else {
        NUFDS_TRY(run_pass<R>(p, "fft1_row_a", ap.passes[0], in, w1, conj_in, 1, 0, R(1), nullptr, s, nullptr,
                              xw_lo, xw_hi));
        NUFDS_TRY(run_pass<R>(p, "fft1_row_b", ap.passes[1], w1, rows_out, 0, 0, 1, sgx, nullptr, s));
    }
    if (!build_axis(1, ny, nx, nx, -1, 0, lim, &ap)) return fail(NUFDS_ERR_UNSUPPORTED, "hologram column length");
    const R sgy = ((ny / 2) & 1) ? R(-1) : R(1);
    if (ap.single) {
        NUFDS_TRY(run_pass<R>(p, "fft1_col", ap.passes[0], spec, spec, 0, 1, 1, sgy, nullptr, s, nullptr, yw_lo,
                              yw_hi));
    } else {
        NUFDS_TRY(run_pass<R>(p, "fft1_col_a", ap.passes[0], spec, w1, 0, 1, 0, R(1), nullptr, s, nullptr, yw_lo,
                              yw_hi));
        NUFDS_TRY(run_pass<R>(p, "fft1_col_b", ap.passes[1], w1, spec, 0, 0, 1, sgy, nullptr, s));
    }
    return NUFDS_OK;
}

// Step 5: output gather from the FrT F ([my][mx], centring signs applied) into d_out.
template <typename R>
static nufds_status_t run_output_gather(nufds_plan* p, const void* F, void* d_out, hipStream_t s) {
    const nufds_plan_info_t& g = p->info;
    const int mx = g.mx, my = g.my;
    const int conj_in = (p->flags & NUFDS_FLAG_CONVERGING) ? 0 : 1;
    OutputArgs<R> oa;
    oa.F = static_cast<const cpx<R>*>(F);
    oa.out = static_cast<cpx<R>*>(d_out);
    oa.ax = static_cast<const double*>(p->ax.p);
    oa.by = static_cast<const double*>(p->by.p);
    oa.sx = g.sx;
    oa.sy = g.sy;
    oa.mx = mx;
    oa.my = my;
    oa.kcx = g.kcx;
    oa.kcy = g.kcy;
    oa.cx = g.cx;
    oa.cy = g.cy;
    oa.dox = g.dox;
    oa.doy = g.doy;
    oa.inv_dfx = 1.0 / g.dfx;
    oa.inv_dfy = 1.0 / g.dfy;
    oa.qx0 = (double)(mx / 2) - (double)g.kcx;
    oa.qy0 = (double)(my / 2) - (double)g.kcy;
    oa.z = p->z;
    oa.kz2 = (2.0 * M_PI / p->wavelength) / (2.0 * p->z);
    oa.remap = (p->flags & NUFDS_FLAG_NO_REMAP) ? 0 : 1;
    oa.conj_out = conj_in;
    // algorithmic bytes: the FrT samples under the window's distorted image (plus the 4-tap
    // support), read once, and the output written once
    const double fxs = std::min((double)mx, (g.xhi - g.xlo) / g.dfx + 4.0);
    const double fys = std::min((double)my, (g.yhi - g.ylo) / g.dfy + 4.0);
    const uint64_t obytes = (uint64_t)(fxs * fys) * sizeof(cpx<R>) + (uint64_t)g.sx * g.sy * sizeof(cpx<R>);
    NUFDS_TRY(timing_begin(p, "output_gather", obytes, s));
    NUFDS_HIP_TRY(launch_output_gather<R>(oa, s));
    return timing_end(p, s);
}

// One DFT of length L along an axis of a [rows][pitch] array without chain: a single pass from in to
// out, or the four-step A pass into work and the B pass into out.  load_sign / store_sign apply the
// centring factor (-1)^index on the input / output axis; load_mul (length L, or NULL) multiplies the
// input by a vector along the axis; load_mul_rows is the same vector in the factored form of
// chirp_row_factors, which a one-pass row transform (K_ROWC) reads instead.
template <typename R>
static nufds_status_t run_transform(nufds_plan* p, const char* name_a, const char* name_b, int axis, int L, int other,
                                    int64_t pitch, int sign, const void* in, void* work, void* out, int load_sign,
                                    int store_sign, const cpx<R>* load_mul, hipStream_t s,
                                    const cpx<R>* load_mul_rows = nullptr) {
    const Limits lim = limits_for(sizeof(cpx<R>), p->tile_cap, p->col_w);
    AxisPlan ap;
    if (!build_axis(axis, L, other, pitch, sign, 0, lim, &ap)) return fail(NUFDS_ERR_UNSUPPORTED, "transform length");
    if (ap.single && ap.passes[0].kind == K_ROWC && load_mul) {
        if (!load_mul_rows) return fail(NUFDS_ERR_UNSUPPORTED, "one-pass row transform without a factored vector");
        load_mul = load_mul_rows;
    }
    if (ap.single)
        return run_pass<R>(p, name_a, ap.passes[0], in, out, 0, load_sign, store_sign, R(1), nullptr, s, load_mul);
    NUFDS_TRY(run_pass<R>(p, name_a, ap.passes[0], in, work, 0, load_sign, 0, R(1), nullptr, s, load_mul));
    return run_pass<R>(p, name_b, ap.passes[1], work, out, 0, 0, store_sign, R(1), nullptr, s);
}

template <typename R>
nufds_status_t run_band(nufds_plan* p, const void* spec, void* d_out, hipStream_t s) {
    const Limits lim = limits_for(sizeof(cpx<R>), p->tile_cap, p->col_w);
    const nufds_plan_info_t& g = p->info;
    const int mx = g.mx, my = g.my;
    void* w1 = p->work1.p;
    void* w2 = p->work2.p;
    AxisPlan ap;

    // steps 2b-3 along x: stretch-gather, centred IDFT, chirp / M_x, centred DFT (signs cancel to
    // (-1)^k' on input and (-1)^m on output)
    const cpx<R>* cxv = static_cast<const cpx<R>*>(p->chirp_x.p);
    const cpx<R>* cyv = static_cast<const cpx<R>*>(p->chirp_y.p);
    if (!build_axis(0, mx, my, mx, +1, 1, lim, &ap)) return fail(NUFDS_ERR_UNSUPPORTED, "FrT row length");
    void* res;
    // the stretch-gather runs as a kernel of its own (2-D tiles, each quadrant table entry read once)
    NUFDS_TRY(run_stretch_gather<R>(p, spec, w2, s));
    if (ap.single) {
        NUFDS_TRY(run_pass<R>(p, "xop", ap.passes[0], w2, w1, 0, 0, 1, R(1), cxv, s));
        res = w1;
    } else {
        NUFDS_TRY(run_pass<R>(p, "xop_a", ap.passes[0], w2, w1, 0, 0, 0, R(1), nullptr, s));
        NUFDS_TRY(run_pass<R>(p, "xop_ba", ap.passes[1], w1, w2, 0, 0, 0, R(1), cxv, s));
        NUFDS_TRY(run_pass<R>(p, "xop_b", ap.passes[2], w2, w1, 0, 0, 1, R(1), nullptr, s));
        res = w1;
    }
    // and along y
    // only the columns the output gather reads (fcx0 .. fcx0 + fcxn - 1) need the y transform
    if (!build_axis(1, my, g.fcxn, mx, +1, 1, lim, &ap)) return fail(NUFDS_ERR_UNSUPPORTED, "FrT column length");
    const size_t coff = (size_t)g.fcx0 * sizeof(cpx<R>);
    auto col = [coff](void* b) { return static_cast<void*>(static_cast<char*>(b) + coff); };
    if (ap.single) {
        NUFDS_TRY(run_pass<R>(p, "yop", ap.passes[0], col(res), col(res), 0, 1, 1, R(1), cyv, s));
    } else {
        void* oth = (res == w1) ? w2 : w1;
        NUFDS_TRY(run_pass<R>(p, "yop_a", ap.passes[0], col(res), col(oth), 0, 1, 0, R(1), nullptr, s));
        NUFDS_TRY(run_pass<R>(p, "yop_ba", ap.passes[1], col(oth), col(res), 0, 0, 0, R(1), cyv, s));
        NUFDS_TRY(run_pass<R>(p, "yop_b", ap.passes[2], col(res), col(oth), 0, 0, 1, R(1), nullptr, s));
        res = oth;
    }
    p->result = res;
    return run_output_gather<R>(p, res, d_out, s);
}

template <typename R>
nufds_status_t prepare_twiddles(nufds_plan* p, bool fft1, bool band) {
    const Limits lim = limits_for(sizeof(cpx<R>), p->tile_cap, p->col_w);
    const nufds_plan_info_t& g = p->info;
    // every transform must have a pass plan; create the twiddle tables its passes read, so that
    // execute only enqueues kernels
    const int snx = spectrum_factor(g) * g.nx, sny = spectrum_factor(g) * g.ny;
    const int axes[4][5] = {{0, snx, sny, snx, 0}, {1, sny, snx, snx, 0}, {0, g.mx, g.my, g.mx, 1},
                            {1, g.my, g.fcxn, g.mx, 1}};
    for (int i = fft1 ? 0 : 2; i < (band ? 4 : 2); ++i) {
        const auto& a = axes[i];
        AxisPlan ap;
        if (!build_axis(a[0], a[1], a[2], a[3], a[4] ? 1 : -1, a[4], lim, &ap))
            return fail(NUFDS_ERR_UNSUPPORTED, "no FFT pass plan for a transform of length " + std::to_string(a[1]));
        for (const PassDesc& d : ap.passes) {
            const cpx<R>* t;
            NUFDS_TRY(twiddle_table<R>(p, d.L, &t));
            if (d.kind == K_ROWA || d.kind == K_COLA || d.kind == K_ROWBA || d.kind == K_COLBA)
                NUFDS_TRY(twiddle_table<R>(p, d.Lf, &t));
        }
    }
    return NUFDS_OK;
}

template nufds_status_t run_fft1<float>(nufds_plan*, const void*, void*, void*, hipStream_t);
template nufds_status_t run_fft1<double>(nufds_plan*, const void*, void*, void*, hipStream_t);
template nufds_status_t run_band<float>(nufds_plan*, const void*, void*, hipStream_t);
template nufds_status_t run_band<double>(nufds_plan*, const void*, void*, hipStream_t);
template nufds_status_t prepare_twiddles<float>(nufds_plan*, bool, bool);
template nufds_status_t prepare_twiddles<double>(nufds_plan*, bool, bool);

// Output-map factors A(x_j), B(y_i) of Eqs. 17-18 for the plan's output grid, float64 on the host.
static nufds_status_t upload_output_map(nufds_plan* p) {
    if (p->flags & NUFDS_FLAG_NO_REMAP) return NUFDS_OK;
    const nufds_plan_info_t& g = p->info;
    std::vector<double> ax(g.sx), by(g.sy);
    const PaperPoly poly = paper_polynomial(p->wavelength / (2.0 * p->pitch));
    auto factor = [&](double x) {
        return g.map_model == 1 ? output_map_factor_paper(poly, x, p->z) : output_map_factor(x, p->z);
    };
    for (int j = 0; j < g.sx; ++j) ax[j] = factor(g.cx + (double)(j - g.sx / 2) * g.dox);
    for (int i = 0; i < g.sy; ++i) by[i] = factor(g.cy + (double)(i - g.sy / 2) * g.doy);
    NUFDS_TRY(dev_alloc(p->ax, g.sx * sizeof(double)));
    NUFDS_TRY(dev_alloc(p->by, g.sy * sizeof(double)));
    NUFDS_HIP_TRY(hipMemcpy(p->ax.p, ax.data(), p->ax.bytes, hipMemcpyHostToDevice));
    NUFDS_HIP_TRY(hipMemcpy(p->by.p, by.data(), p->by.bytes, hipMemcpyHostToDevice));
    return NUFDS_OK;
}

// Chirp vectors of the plan's depth, one per axis (each carrying the 1/M of its inverse DFT).
template <typename R>
static nufds_status_t upload_chirps(nufds_plan* p) {
    const nufds_plan_info_t& g = p->info;
    std::vector<double> re, im;
    chirp_vector(g.mx, g.nx, p->pitch, p->wavelength, p->z, re, im);
    NUFDS_TRY(upload_complex<R>(p->chirp_x, re, im));
    chirp_vector(g.my, g.ny, p->pitch, p->wavelength, p->z, re, im);
    NUFDS_TRY(upload_complex<R>(p->chirp_y, re, im));
    if (sizeof(R) == 4 && row_chain_threads(g.mx) > 0) {
        // for x transforms that multiply the chirp on load in one pass (the focal stack's)
        chirp_row_factors(g.mx, g.nx, p->pitch, p->wavelength, p->z, row_chain_first_radix(g.mx), re, im);
        NUFDS_TRY(upload_complex<R>(p->chirp_xf, re, im));
    }
    return NUFDS_OK;
}

template <typename R>
static nufds_status_t prepare_impl(nufds_plan* p) {
    NUFDS_TRY(prepare_twiddles<R>(p, true, true));
    return upload_chirps<R>(p);
}

static nufds_status_t plan_create_impl(nufds_plan_t* out, double wavelength, double pitch, int32_t nx, int32_t ny,
                                       double z, const nufds_view_t* view, nufds_precision_t precision,
                                       uint32_t flags, const nufds_options_t* opt) {
    if (!out) return fail(NUFDS_ERR_INVALID_ARG, "plan is NULL");
    *out = nullptr;
    if (precision != NUFDS_C64 && precision != NUFDS_C128) return fail(NUFDS_ERR_INVALID_ARG, "unknown precision");
    nufds_plan_info_t g;
    NUFDS_TRY(compute_geometry(wavelength, pitch, nx, ny, z, view, flags, opt, &g));
    NUFDS_TRY(check_sizes(g));
    nufds_plan* p = new (std::nothrow) nufds_plan();
    if (!p) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->info = g;
    p->info.precision = precision;
    p->wavelength = wavelength;
    p->pitch = pitch;
    p->z = z;
    p->flags = flags;
    p->prec = precision;
    p->esize = precision == NUFDS_C64 ? 8 : 16;
    p->tile_cap = tile_override();
    p->col_w = col_w_override();
    p->twiddles = std::make_shared<TwiddleCache>();
    p->twiddles->esize = p->esize;
    auto bail = [&](nufds_status_t st) {
        std::string msg = nufds_last_error();
        plan_free(p);
        set_error(msg);
        return st;
    };
    hipError_t he = hipGetDevice(&p->device);
    if (he != hipSuccess) return bail(hip_fail(he, "hipGetDevice"));
    const int sf = spectrum_factor(g);
    const size_t nn = (size_t)sf * sf * nx * ny, mm = (size_t)g.mx * g.my;
    const size_t big = std::max(nn, mm);
    nufds_status_t st;
    if ((st = dev_alloc(p->spec, nn * p->esize)) != NUFDS_OK) return bail(st);
    if ((st = dev_alloc(p->work1, big * p->esize)) != NUFDS_OK) return bail(st);
    if ((st = dev_alloc(p->work2, big * p->esize)) != NUFDS_OK) return bail(st);
    // stretch-map table: quadrant |k_g| <= min(band extent, stretch extent) per axis
    const double s = wavelength / (2.0 * pitch);
    if (!(flags & NUFDS_FLAG_NO_STRETCH)) {
        int kmx, kmy;
        table_extent(wavelength, pitch, nx, ny, &kmx, &kmy);
        const int bx = std::max(std::abs(g.kcx - g.mx / 2), std::abs(g.kcx + g.mx / 2 - 1));
        const int by = std::max(std::abs(g.kcy - g.my / 2), std::abs(g.kcy + g.my / 2 - 1));
        p->kxt = std::min(bx, kmx);
        p->kyt = std::min(by, kmy);
        if ((st = dev_alloc(p->table, map_table_bytes(p->kxt, p->kyt))) != NUFDS_OK) return bail(st);
        const PaperPoly poly = paper_polynomial(s);
        he = launch_map_table(static_cast<double*>(p->table.p), p->kxt, p->kyt, wavelength, nx * pitch, ny * pitch, s,
                              sf, g.map_model == 1 ? &poly : nullptr, nullptr);
        if (he != hipSuccess) return bail(hip_fail(he, "map table launch"));
    }
    if ((st = upload_output_map(p)) != NUFDS_OK) return bail(st);
    st = precision == NUFDS_C64 ? prepare_impl<float>(p) : prepare_impl<double>(p);
    if (st != NUFDS_OK) return bail(st);
    he = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (he != hipSuccess) return bail(hip_fail(he, "hipEventCreate"));
    he = hipDeviceSynchronize();
    if (he != hipSuccess) return bail(hip_fail(he, "plan build"));
    size_t total = p->spec.bytes + p->work1.bytes + p->work2.bytes + p->table.bytes + p->chirp_x.bytes +
                   p->chirp_y.bytes + p->chirp_xf.bytes + p->ax.bytes + p->by.bytes;
    p->info.map_bytes = p->table.bytes;
    p->info.workspace_bytes = total;
    *out = p;
    return NUFDS_OK;
}

}  // namespace nufds

// ------------------------------------------------------------------ C ABI

using namespace nufds;

extern "C" {

nufds_status_t nufds_plan_geometry(double wavelength, double pitch, int32_t nx, int32_t ny, double z,
                                   const nufds_view_t* view, uint32_t flags, const nufds_options_t* opt,
                                   nufds_plan_info_t* out) {
    nufds_status_t st = compute_geometry(wavelength, pitch, nx, ny, z, view, flags, opt, out);
    if (st == NUFDS_OK) set_error("");
    return st;
}

nufds_status_t nufds_plan_create(nufds_plan_t* plan, double wavelength, double pitch, int32_t nx, int32_t ny,
                                 double z, const nufds_view_t* view, nufds_precision_t precision, uint32_t flags) {
    return plan_create_impl(plan, wavelength, pitch, nx, ny, z, view, precision, flags, nullptr);
}

nufds_status_t nufds_plan_create_ex(nufds_plan_t* plan, double wavelength, double pitch, int32_t nx, int32_t ny,
                                    double z, const nufds_view_t* view, nufds_precision_t precision, uint32_t flags,
                                    const nufds_options_t* opt) {
    return plan_create_impl(plan, wavelength, pitch, nx, ny, z, view, precision, flags, opt);
}

nufds_status_t nufds_plan_info(nufds_plan_t plan, nufds_plan_info_t* out) {
    if (!plan || !out) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    *out = plan->info;
    return NUFDS_OK;
}

}  // extern "C"

// Shared by nufds_execute and nufds_execute_spectrum: the one-execute-in-flight rule, timing
// bookkeeping and the completion event; d_hologram NULL means spec already holds the spectrum.
static nufds_status_t execute_common(nufds_plan_t plan, const void* d_hologram, const void* spec, void* d_out,
                                     hipStream_t s) {
    if (plan->has_run && s != plan->last_stream) {
        hipError_t q = hipEventQuery(plan->done);
        if (q == hipErrorNotReady) return fail(NUFDS_ERR_BUSY, "previous execute still running on another stream");
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    plan->recording = plan->timed_execs < plan->timing_cap;
    nufds_status_t st = NUFDS_OK;
    if (plan->prec == NUFDS_C64) {
        if (d_hologram) st = run_fft1<float>(plan, d_hologram, plan->spec.p, plan->work1.p, s);
        if (st == NUFDS_OK) st = run_band<float>(plan, spec, d_out, s);
    } else {
        if (d_hologram) st = run_fft1<double>(plan, d_hologram, plan->spec.p, plan->work1.p, s);
        if (st == NUFDS_OK) st = run_band<double>(plan, spec, d_out, s);
    }
    if (plan->recording) ++plan->timed_execs;
    plan->recording = false;
    if (st != NUFDS_OK) return st;
    NUFDS_HIP_TRY(hipEventRecord(plan->done, s));
    plan->last_stream = s;
    plan->has_run = true;
    return NUFDS_OK;
}

// ------------------------------------------------------------ focal stack
struct nufds_stack {
    nufds_plan* base = nullptr;      // full plan of depth 0 at the shared FrT size: spectrum, work, table
    std::vector<nufds_plan*> depth;  // per depth: geometry, chirps, output map (depth[0] is base)
    nufds::DevBuf cache;             // inverse DFT of the stretched band, [my][mx]
    size_t bytes = 0;
};

// A depth of a stack: its own geometry, chirp vectors and output-map factors; the spectrum, work
// buffers, map table and twiddles are the base plan's.
static nufds_status_t depth_plan(nufds_plan* base, double z, const nufds_options_t* opt, nufds_plan** out) {
    *out = nullptr;
    nufds_plan_info_t g;
    NUFDS_TRY(compute_geometry(base->wavelength, base->pitch, base->info.nx, base->info.ny, z, nullptr, base->flags,
                               opt, &g));
    if (g.mx != base->info.mx || g.my != base->info.my || g.kcx != base->info.kcx || g.kcy != base->info.kcy)
        return fail(NUFDS_ERR_UNSUPPORTED, "the depths do not share one band");
    nufds_plan* p = new (std::nothrow) nufds_plan();
    if (!p) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->info = g;
    p->info.precision = base->info.precision;
    p->wavelength = base->wavelength;
    p->pitch = base->pitch;
    p->z = z;
    p->flags = base->flags;
    p->prec = base->prec;
    p->esize = base->esize;
    p->device = base->device;
    p->tile_cap = base->tile_cap;
    p->col_w = base->col_w;
    p->twiddles = base->twiddles;
    p->spec = borrow(base->spec.p, base->spec.bytes);
    p->work1 = borrow(base->work1.p, base->work1.bytes);
    p->work2 = borrow(base->work2.p, base->work2.bytes);
    p->table = borrow(base->table.p, base->table.bytes);
    p->kxt = base->kxt;
    p->kyt = base->kyt;
    nufds_status_t st = upload_output_map(p);
    if (st == NUFDS_OK) st = p->prec == NUFDS_C64 ? upload_chirps<float>(p) : upload_chirps<double>(p);
    if (st != NUFDS_OK) {
        std::string msg = nufds_last_error();
        plan_free(p);
        set_error(msg);
        return st;
    }
    *out = p;
    return NUFDS_OK;
}

// Steps 2-2c once (FFT of the hologram, stretch-gather, inverse DFT of the band along x then y, kept
// in the cache), then per depth the chirp-in and the centred forward DFT of Eq. 2 and the output
// gather.  The chirp is separable and each axis' factor depends on that axis alone, so the x factor
// multiplies the x transform's loads and the y factor the y transform's.  Centring: the gather
// carries (-1)^k'_x and the y inverse DFT applies (-1)^k'_y on load; the (-1)^(n + M/2) of each
// inverse DFT's output cancels against the (-1)^n of the forward DFT's input (M even), which leaves
// (-1)^m on the forward DFT's output.
template <typename R>
static nufds_status_t run_stack(nufds_stack* S, const void* d_hologram, void* const* d_outs, hipStream_t s) {
    nufds_plan* b = S->base;
    const int mx = b->info.mx, my = b->info.my;
    char* w1 = static_cast<char*>(b->work1.p);
    char* w2 = static_cast<char*>(b->work2.p);
    void* q = S->cache.p;
    NUFDS_TRY(run_fft1<R>(b, d_hologram, b->spec.p, w1, s));
    NUFDS_TRY(run_stretch_gather<R>(b, b->spec.p, w2, s));
    NUFDS_TRY(run_transform<R>(b, "idft_x_a", "idft_x_b", 0, mx, my, mx, +1, w2, w1, w2, 0, 0, nullptr, s));
    NUFDS_TRY(run_transform<R>(b, "idft_y_a", "idft_y_b", 1, my, mx, mx, +1, w2, w1, q, 1, 0, nullptr, s));
    for (size_t i = 0; i < S->depth.size(); ++i) {
        nufds_plan* d = S->depth[i];
        const cpx<R>* cxv = static_cast<const cpx<R>*>(d->chirp_x.p);
        const cpx<R>* cyv = static_cast<const cpx<R>*>(d->chirp_y.p);
        NUFDS_TRY(run_transform<R>(d, "dft_x_a", "dft_x_b", 0, mx, my, mx, -1, q, w2, w1, 0, 1, cxv, s,
                                   static_cast<const cpx<R>*>(d->chirp_xf.p)));
        // only the columns this depth's output gather reads need the y transform
        const size_t coff = (size_t)d->info.fcx0 * sizeof(cpx<R>);
        NUFDS_TRY(run_transform<R>(d, "dft_y_a", "dft_y_b", 1, my, d->info.fcxn, mx, -1, w1 + coff, w2 + coff,
                                   w1 + coff, 0, 1, cyv, s));
        NUFDS_TRY(run_output_gather<R>(d, w1, d_outs[i], s));
    }
    b->result = w1;
    return NUFDS_OK;
}

static void stack_free(nufds_stack* S) {
    if (!S) return;
    (void)hipDeviceSynchronize();
    for (nufds_plan* d : S->depth)
        if (d != S->base) plan_free(d);
    plan_free(S->base);
    dev_free(S->cache);
    delete S;
}

static nufds_status_t stack_create_impl(nufds_stack_t* out, double wavelength, double pitch, int32_t nx, int32_t ny,
                                        const double* z, int32_t n_z, nufds_precision_t precision, uint32_t flags) {
    if (!out) return fail(NUFDS_ERR_INVALID_ARG, "stack is NULL");
    *out = nullptr;
    if (!z || n_z < 1 || n_z > 64) return fail(NUFDS_ERR_INVALID_ARG, "a stack has 1 to 64 depths");
    // the shared FrT size: the largest the size rule gives over the depths
    nufds_options_t opt;
    opt.pad = -1.0;
    opt.frt_size_x = opt.frt_size_y = 0;
    opt.oversample = 0;
    opt.map_model = 0;
    for (int i = 0; i < n_z; ++i) {
        nufds_plan_info_t g;
        NUFDS_TRY(compute_geometry(wavelength, pitch, nx, ny, z[i], nullptr, flags, nullptr, &g));
        opt.frt_size_x = std::max(opt.frt_size_x, g.mx);
        opt.frt_size_y = std::max(opt.frt_size_y, g.my);
    }
    nufds_stack* S = new (std::nothrow) nufds_stack();
    if (!S) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    auto bail = [&](nufds_status_t st) {
        std::string msg = nufds_last_error();
        stack_free(S);
        set_error(msg);
        return st;
    };
    nufds_plan_t base = nullptr;
    nufds_status_t st = plan_create_impl(&base, wavelength, pitch, nx, ny, z[0], nullptr, precision, flags, &opt);
    if (st != NUFDS_OK) return bail(st);
    S->base = base;
    S->depth.push_back(base);
    if ((st = dev_alloc(S->cache, (size_t)base->info.mx * base->info.my * base->esize)) != NUFDS_OK) return bail(st);
    S->bytes = base->info.workspace_bytes + S->cache.bytes;
    for (int i = 1; i < n_z; ++i) {
        nufds_plan* d = nullptr;
        if ((st = depth_plan(base, z[i], &opt, &d)) != NUFDS_OK) return bail(st);
        S->depth.push_back(d);
        S->bytes += d->chirp_x.bytes + d->chirp_y.bytes + d->chirp_xf.bytes + d->ax.bytes + d->by.bytes;
    }
    *out = S;
    return NUFDS_OK;
}

extern "C" {

nufds_status_t nufds_stack_create(nufds_stack_t* stack, double wavelength, double pitch, int32_t nx, int32_t ny,
                                  const double* z, int32_t n_z, nufds_precision_t precision, uint32_t flags) {
    return stack_create_impl(stack, wavelength, pitch, nx, ny, z, n_z, precision, flags);
}

nufds_status_t nufds_stack_info(nufds_stack_t stack, int32_t i, nufds_plan_info_t* out) {
    if (!stack || !out) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    if (i < 0 || i >= (int32_t)stack->depth.size()) return fail(NUFDS_ERR_INVALID_ARG, "depth index out of range");
    *out = stack->depth[i]->info;
    out->workspace_bytes = stack->bytes;
    out->map_bytes = stack->base->table.bytes;
    return NUFDS_OK;
}

nufds_status_t nufds_stack_execute(nufds_stack_t stack, const void* d_hologram, void* const* d_outs, void* stream) {
    if (!stack || !d_hologram || !d_outs) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    const size_t n = stack->depth.size();
    for (size_t i = 0; i < n; ++i) {
        if (!d_outs[i]) return fail(NUFDS_ERR_INVALID_ARG, "NULL output");
        if (d_outs[i] == d_hologram) return fail(NUFDS_ERR_INVALID_ARG, "an output aliases the hologram");
        for (size_t j = 0; j < i; ++j)
            if (d_outs[j] == d_outs[i]) return fail(NUFDS_ERR_INVALID_ARG, "two outputs alias");
    }
    nufds_plan* b = stack->base;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->has_run && s != b->last_stream) {
        hipError_t q = hipEventQuery(b->done);
        if (q == hipErrorNotReady) return fail(NUFDS_ERR_BUSY, "previous execute still running on another stream");
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    nufds_status_t st = b->prec == NUFDS_C64 ? run_stack<float>(stack, d_hologram, d_outs, s)
                                              : run_stack<double>(stack, d_hologram, d_outs, s);
    if (st != NUFDS_OK) return st;
    NUFDS_HIP_TRY(hipEventRecord(b->done, s));
    b->last_stream = s;
    b->has_run = true;
    return NUFDS_OK;
}

nufds_status_t nufds_stack_destroy(nufds_stack_t stack) {
    stack_free(stack);
    return NUFDS_OK;
}

nufds_status_t nufds_execute(nufds_plan_t plan, const void* d_hologram, void* d_out, void* stream) {
    if (!plan || !d_hologram || !d_out) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    if (d_hologram == d_out) return fail(NUFDS_ERR_INVALID_ARG, "output aliases the hologram");
    return execute_common(plan, d_hologram, plan->spec.p, d_out, static_cast<hipStream_t>(stream));
}

nufds_status_t nufds_execute_spectrum(nufds_plan_t plan, nufds_spectrum_t spectrum, void* d_out, void* stream) {
    if (!plan || !spectrum || !d_out) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    if (spectrum->nx != plan->info.nx || spectrum->ny != plan->info.ny || spectrum->prec != plan->prec ||
        spectrum->wavelength != plan->wavelength || spectrum->pitch != plan->pitch ||
        (spectrum->flags & NUFDS_FLAG_CONVERGING) != (plan->flags & NUFDS_FLAG_CONVERGING))
        return fail(NUFDS_ERR_INVALID_ARG, "spectrum and plan differ in size, wavelength, pitch, precision or sign");
    if (spectrum_factor(plan->info) != 1)
        return fail(NUFDS_ERR_INVALID_ARG, "a cached spectrum is not oversampled; the plan is");
    return execute_common(plan, nullptr, spectrum->spec.p, d_out, static_cast<hipStream_t>(stream));
}

nufds_status_t nufds_debug_copy(nufds_plan_t plan, int32_t which, void* d_dst, uint64_t* bytes, void* stream) {
    if (!plan || !bytes) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    const void* src = nullptr;
    uint64_t n = 0;
    switch (which) {
        case 1: {
            const uint64_t f = spectrum_factor(plan->info);
            src = plan->spec.p;
            n = f * f * plan->info.nx * plan->info.ny * plan->esize;
            break;
        }
        case 2: src = plan->result; n = (uint64_t)plan->info.mx * plan->info.my * plan->esize; break;
        case 3: src = plan->table.p; n = plan->table.p ? map_entries_bytes(plan->kxt, plan->kyt) : 0; break;
        default: return fail(NUFDS_ERR_INVALID_ARG, "unknown buffer");
    }
    *bytes = n;
    if (!d_dst) return NUFDS_OK;
    if (!src) return fail(NUFDS_ERR_INVALID_ARG, "buffer not available (no execute yet, or no table)");
    NUFDS_HIP_TRY(hipMemcpyAsync(d_dst, src, n, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return NUFDS_OK;
}

nufds_status_t nufds_set_timing(nufds_plan_t plan, int32_t n_executes) {
    if (!plan || n_executes < 0) return fail(NUFDS_ERR_INVALID_ARG, "NULL plan or negative count");
    NUFDS_HIP_TRY(hipDeviceSynchronize());
    plan->timing_cap = n_executes;
    plan->timed_execs = 0;
    plan->nlaunch = 0;
    return NUFDS_OK;
}

nufds_status_t nufds_get_timings(nufds_plan_t plan, nufds_kernel_time_t* out, int32_t max_entries,
                                 int32_t* n_entries) {
    if (!plan || !n_entries) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    if (plan->timing_cap == 0) return fail(NUFDS_ERR_INVALID_ARG, "timing is not enabled");
    const int n = plan->nlaunch;
    *n_entries = n;
    if (!out) return NUFDS_OK;
    if (n > 0) NUFDS_HIP_TRY(hipEventSynchronize(plan->ev[2 * (size_t)n - 1]));
    for (int i = 0; i < n && i < max_entries; ++i) {
        float ms = 0.0f;
        NUFDS_HIP_TRY(hipEventElapsedTime(&ms, plan->ev[2 * (size_t)i], plan->ev[2 * (size_t)i + 1]));
        out[i] = plan->launches[i];
        out[i].ms = ms;
    }
    return NUFDS_OK;
}

nufds_status_t nufds_destroy(nufds_plan_t plan) {
    plan_free(plan);
    return NUFDS_OK;
}

nufds_status_t nufds_synth_hologram(const double* h_points, int32_t n_points, int32_t nx, int32_t ny, double pitch,
                                    double wavelength, nufds_precision_t precision, void* d_out, void* stream) {
    if (!h_points || n_points <= 0 || nx <= 0 || ny <= 0 || !d_out || !(pitch > 0) || !(wavelength > 0))
        return fail(NUFDS_ERR_INVALID_ARG, "invalid synth arguments");
    if (precision != NUFDS_C64 && precision != NUFDS_C128) return fail(NUFDS_ERR_INVALID_ARG, "unknown precision");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* d_pts = nullptr;
    const size_t bytes = (size_t)n_points * 5 * sizeof(double);
    hipError_t e = hipMallocAsync(&d_pts, bytes, s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(points)");
    e = hipMemcpyAsync(d_pts, h_points, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host array may go away after return
    if (e == hipSuccess) {
        const double k = 2.0 * M_PI / wavelength;
        e = precision == NUFDS_C64
                ? launch_synth<float>(static_cast<double*>(d_pts), n_points, nx, ny, pitch, k, static_cast<cpx<float>*>(d_out), s)
                : launch_synth<double>(static_cast<double*>(d_pts), n_points, nx, ny, pitch, k, static_cast<cpx<double>*>(d_out), s);
    }
    hipError_t e2 = hipFreeAsync(d_pts, s);
    if (e != hipSuccess) return hip_fail(e, "synth");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync(points)");
    return NUFDS_OK;
}

const char* nufds_status_string(nufds_status_t status) {
    switch (status) {
        case NUFDS_OK: return "ok";
        case NUFDS_ERR_INVALID_ARG: return "invalid argument";
        case NUFDS_ERR_UNSUPPORTED: return "unsupported";
        case NUFDS_ERR_OUT_OF_MEMORY: return "out of memory";
        case NUFDS_ERR_HIP: return "HIP error";
        case NUFDS_ERR_BUSY: return "busy";
    }
    return "unknown status";
}

const char* nufds_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
