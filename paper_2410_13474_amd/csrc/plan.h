// Internal plan layout and execute steps of libnufds, shared by the plan API and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "nufds.h"

namespace nufds {

#define NUFDS_TRY(x)                        \
    do {                                    \
        nufds_status_t st_ = (x);           \
        if (st_ != NUFDS_OK) return st_;    \
    } while (0)

// Device buffer; a borrowed one (owned = false) belongs to someone else and is never freed here.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool owned = true;
};

nufds_status_t dev_alloc(DevBuf& b, size_t bytes);
void dev_free(DevBuf& b);
inline DevBuf borrow(void* p, size_t bytes) {
    DevBuf b;
    b.p = p;
    b.bytes = bytes;
    b.owned = false;
    return b;
}

// Twiddle tables exp(-2 pi i m / L) by length, for one element type; shared by the plans that use it.
struct TwiddleCache {
    size_t esize = 8;
    std::map<int, void*> tables;
    ~TwiddleCache();
};

constexpr int kMaxLen = 65536;

bool smooth5(int n);
nufds_status_t compute_geometry(double wavelength, double pitch, int nx, int ny, double z, const nufds_view_t* view,
                                uint32_t flags, const nufds_options_t* opt, nufds_plan_info_t* out);
// Spectral grid of step 2 relative to the hologram's (2 when oversampled).
inline int spectrum_factor(const nufds_plan_info_t& g) { return g.oversample == 2 ? 2 : 1; }
// Size limits of the kernels (5-smooth, at most kMaxLen, arrays below 2^31 elements).
nufds_status_t check_sizes(const nufds_plan_info_t& g);
// Largest T_1 of the stretch over the hologram band, and the quadrant table extent it implies.
double stretch_extent(double s);
void table_extent(double wavelength, double pitch, int nx, int ny, int* kxt, int* kyt);
void chirp_vector(int M, int N, double pitch, double wavelength, double z, std::vector<double>& re,
                  std::vector<double>& im);
void chirp_row_factors(int M, int N, double pitch, double wavelength, double z, int R, std::vector<double>& re,
                       std::vector<double>& im);
int tile_override();
int col_w_override();

}  // namespace nufds

struct nufds_plan {
    nufds_plan_info_t info{};
    double wavelength = 0, pitch = 0, z = 0;
    uint32_t flags = 0;
    int prec = 0;
    int device = 0;
    size_t esize = 8;
    nufds::DevBuf spec, work1, work2, table, chirp_x, chirp_y, ax, by;
    nufds::DevBuf chirp_xf;  // chirp_x factored for one-pass row transforms (complex64, K_ROWC rows)
    int kxt = -1, kyt = -1;
    std::shared_ptr<nufds::TwiddleCache> twiddles;
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_run = false;
    void* result = nullptr;  // buffer holding F after the last execute
    int tile_cap = 0;        // LDS tile capacity override captured at creation (0: none)
    int col_w = 0;           // column-tile width override captured at creation (0: default)
    // per-launch timing
    int timing_cap = 0;                        // executes to record (0: timing off)
    int timed_execs = 0;                       // executes recorded so far
    bool recording = false;                    // the current execute is being recorded
    std::vector<hipEvent_t> ev;                // pairs (start, end) per recorded launch
    std::vector<nufds_kernel_time_t> launches; // names and bytes of the recorded launches
    int nlaunch = 0;
};

// A cached hologram spectrum (the forward FFT of step 2).
struct nufds_spectrum {
    int nx = 0, ny = 0;
    double wavelength = 0, pitch = 0;
    int prec = 0;
    uint32_t flags = 0;  // NUFDS_FLAG_CONVERGING or 0
    size_t esize = 8;
    int device = 0;
    nufds::DevBuf spec;
};

namespace nufds {

// Step 2a: centred forward DFT of the [ny][nx] hologram into spec (work: scratch of nx ny elements
// for four-step passes).  Uses p->info.nx/ny, flags, esize, tile overrides, twiddles, timing.
template <typename R>
nufds_status_t run_fft1(nufds_plan* p, const void* d_in, void* spec, void* work, hipStream_t s);
// Steps 2b-5 from a centred spectrum: stretch-gather, the x and y Fresnel operators, output gather.
template <typename R>
nufds_status_t run_band(nufds_plan* p, const void* spec, void* d_out, hipStream_t s);
// Twiddle tables every pass of the hologram transform (fft1) and of the band transforms needs.
template <typename R>
nufds_status_t prepare_twiddles(nufds_plan* p, bool fft1, bool band);

}  // namespace nufds
