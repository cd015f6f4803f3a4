/*
 * libnufds -- NU-FDS reconstruction of wide-angle holograms on one MI355X (gfx950).
 *
 * Method: Kozacki et al., "Non-uniform Fourier Domain Stretching method for
 * ultra-wide-angle wave propagation", arXiv 2410.13474, Sec. 4 (Fig. 3):
 *   step 2  FFT of the hologram, non-uniform stretch of its spectrum onto a
 *           uniform f' grid (Eqs. 9-10 with the magnification of Eq. 16),
 *           inverse FFT;
 *   step 3  FFT-based Fresnel transform (chirp . FFT . chirp, Eq. 2);
 *   step 5  remap of the distorted output x' (Eqs. 17-18) onto the true
 *           object-plane grid, cropped to a full or partial view (Sec. 4,
 *           partial view).
 * Steps 1 and 4 (the maps) are evaluated when a plan is created.
 *
 * Conventions shared by every entry point:
 *   - Complex data are interleaved (re, im): float pairs for NUFDS_C64,
 *     double pairs for NUFDS_C128.  Arrays are row-major [rows][cols].
 *   - Hologram pixel (i, j) of an ny x nx hologram with pitch D sits at
 *     x = (j - nx/2) D, y = (i - ny/2) D.  nx and ny are even.
 *   - Output pixel (i, j) of a view sits at
 *     (center_x + (j - view.nx/2) pitch_x, center_y + (i - view.ny/2) pitch_y)
 *     in the object plane at distance z (true coordinates, metres).
 *   - Default input: diverging point waves exp(+i k r)/r.  The paper's
 *     Eq. 2 focuses converging waves exp(-i k R) (Eq. 3); a diverging
 *     hologram is conjugated on input and the output conjugated back.
 *     NUFDS_FLAG_CONVERGING skips both.
 *   - Device pointers are HIP device memory of the current device; a stream
 *     argument is a hipStream_t passed as void* (NULL = default stream).
 *   - Every call returns a status; no C++ exception crosses this boundary.
 *     On failure nufds_last_error() returns a thread-local message.
 */
#ifndef NUFDS_H
#define NUFDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nufds_plan* nufds_plan_t;

typedef enum {
    NUFDS_OK = 0,
    NUFDS_ERR_INVALID_ARG = 1,   /* a value outside its documented range */
    NUFDS_ERR_UNSUPPORTED = 2,   /* valid, but beyond what the kernels handle */
    NUFDS_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
    NUFDS_ERR_HIP = 4,           /* a HIP runtime call failed (see nufds_last_error) */
    NUFDS_ERR_BUSY = 5           /* the plan is already executing */
} nufds_status_t;

typedef enum {
    NUFDS_C64 = 0,   /* complex64 data; the stretch map, chirp phases and output map in float64 */
    NUFDS_C128 = 1   /* complex128 throughout */
} nufds_precision_t;

enum {
    NUFDS_FLAG_CONVERGING = 1u, /* input follows Eq. 3, exp(-i k R) */
    NUFDS_FLAG_NO_STRETCH = 2u, /* m_x = m_y = 1: step 2 leaves the spectrum on its own grid */
    NUFDS_FLAG_NO_REMAP = 4u    /* skip step 5: output sampled at the distorted x' of Eqs. 17-18 */
};

/* A view: the rectangle of the object plane to reconstruct (Sec. 4, partial view). */
typedef struct {
    double center_x, center_y; /* metres, true coordinates at distance z */
    double pitch_x, pitch_y;   /* metres; <= 0 selects Delta_F = lambda z / (N D) on that axis */
    int32_t nx, ny;            /* output samples, > 0 */
} nufds_view_t;

/* Options of nufds_plan_create_ex. */
typedef struct {
    double pad;                      /* aperture pad added to the window's x' extent, metres;
                                        < 0 selects N D / 2 per axis, 0 is the paper-literal band */
    int32_t frt_size_x, frt_size_y;  /* 0: size rule below; else a forced even 5-smooth FrT size */
    int32_t oversample;              /* 0 or 1: the spectrum of step 2 on the hologram's own
                                        frequency grid; 2: on a grid twice as fine (the hologram
                                        zero-padded to 2N x 2N before its DFT), so that the Keys
                                        interpolation of the stretch sees a spectrum sampled at twice
                                        its critical rate */
    int32_t map_model;               /* 0: Eq. 16 exactly; 1: the paper's stand-in (Sec. 4, step 1),
                                        the hypergeometric function replaced by a degree-8 polynomial
                                        fitted by least squares to 51 samples across the band, in the
                                        stretch (step 1) and the output map (step 4), for comparison */
} nufds_options_t;

/* Geometry of one reconstruction, as computed by the plan (host, float64). */
typedef struct {
    int32_t nx, ny;          /* hologram samples */
    int32_t sx, sy;          /* output samples */
    int32_t mx, my;          /* FrT size M (the width of the processed sub-band, in spectral samples) */
    int32_t kcx, kcy;        /* sub-band centre K_c in spectral samples (= FrT output offset in Delta_F) */
    double dfx, dfy;         /* Delta_F = lambda z / (N D): FrT output pitch */
    double dox, doy;         /* output pitch */
    double cx, cy;           /* output window centre */
    double image_size;       /* B = 2 z tan(asin(lambda / 2 D)), Eq. 1 */
    double xlo, xhi, ylo, yhi; /* extent of the window's distorted image x', y' (before the pad) */
    double padx, pady;       /* pad used */
    uint64_t workspace_bytes; /* device bytes owned by the plan */
    uint64_t map_bytes;       /* of which the stretch-map table */
    int32_t precision;       /* nufds_precision_t */
    uint32_t flags;
    int32_t fcx0, fcxn;      /* FrT columns the view reads (first, count): the y transform runs on
                                these only */
    int32_t oversample;      /* 1 or 2: spectral grid of step 2 relative to the hologram's */
    int32_t map_model;       /* 0 exact, 1 the paper's polynomial model */
} nufds_plan_info_t;

/*
 * nufds_plan_geometry -- the plan's geometry without touching the GPU.
 *
 * Computes what nufds_plan_create would use (Sec. 2, Eq. 1 and the FrT
 * sampling after Eq. 2; Sec. 4, output parameter selection and partial
 * view): the output grid, the distorted extent of the window under
 * Eqs. 17-18, and the processed sub-band:
 *   K_c = round(centre of [x'_lo - pad, x'_hi + pad] / Delta_F),
 *   M   = smallest even 5-smooth integer >= 2 ceil(half width / Delta_F)
 *         (ceiling taken with a 1e-9 sample tolerance), per axis.
 * The FrT always runs at Delta_F; step 5 resamples to the output pitch.
 *
 * wavelength, pitch, z > 0 (metres) with wavelength / (2 pitch) < 1;
 * nx, ny even and > 0; view NULL selects the full view (nx x ny samples
 * over the B x B image of Eq. 1), otherwise its window must lie inside
 * [-B/2, B/2]^2; opt may be NULL.  Writes *out.
 * Errors: NUFDS_ERR_INVALID_ARG for any violated range or a NULL out.
 */
nufds_status_t nufds_plan_geometry(double wavelength, double pitch, int32_t nx, int32_t ny,
                                   double z, const nufds_view_t* view, uint32_t flags,
                                   const nufds_options_t* opt, nufds_plan_info_t* out);

/*
 * nufds_plan_create / nufds_plan_create_ex -- build a reconstruction plan.
 *
 * Arguments as in nufds_plan_geometry, plus the precision.  The plan owns
 * device workspace (the spectrum, two FrT-size buffers) and the stretch-map
 * table: for every stretched frequency of the sub-band, the pre-image under
 * the stretch of Eqs. 9-10 with m_x, m_y of Eq. 16 (step 1, evaluated
 * exactly in float64 on the GPU, one quadrant by the map's odd symmetry).
 * Allocates on the current device and synchronises it before returning.
 * *plan receives the handle, which the caller releases with nufds_destroy.
 * Errors: INVALID_ARG (ranges, NULL plan), UNSUPPORTED (a size beyond the
 * kernels: FrT or hologram sizes must be 5-smooth and at most 65536),
 * OUT_OF_MEMORY, HIP.  On error *plan is set to NULL and nothing leaks.
 */
nufds_status_t nufds_plan_create(nufds_plan_t* plan, double wavelength, double pitch,
                                 int32_t nx, int32_t ny, double z, const nufds_view_t* view,
                                 nufds_precision_t precision, uint32_t flags);
nufds_status_t nufds_plan_create_ex(nufds_plan_t* plan, double wavelength, double pitch,
                                    int32_t nx, int32_t ny, double z, const nufds_view_t* view,
                                    nufds_precision_t precision, uint32_t flags,
                                    const nufds_options_t* opt);

/* nufds_plan_info -- copy the plan's geometry into *out.  Errors: INVALID_ARG on NULL. */
nufds_status_t nufds_plan_info(nufds_plan_t plan, nufds_plan_info_t* out);

/*
 * nufds_execute -- reconstruct one hologram (steps 2, 3 and 5 of Sec. 4).
 *
 * d_hologram: device, [ny][nx] complex of the plan's precision, read only.
 * d_out: device, [view.ny][view.nx] complex of the plan's precision,
 *        written completely.  Must not alias d_hologram.
 * stream: hipStream_t as void*, or NULL.  The call only enqueues work on
 * the stream and returns; buffers must stay valid until the stream reaches
 * that point.  Output pixel = exp(+i k (x'^2 + y'^2) / 2z) times the Keys
 * interpolation of the FrT at the pixel's distorted position (x', y').
 * One execute may be in flight per plan: a second call while the first is
 * still enqueued-but-unfinished on another stream is allowed only after
 * the caller orders the streams; the library tracks this with an event and
 * returns NUFDS_ERR_BUSY if the previous execute has not completed and the
 * new call uses a different stream.
 * Errors: INVALID_ARG (NULL plan or pointers), BUSY, HIP.
 */
nufds_status_t nufds_execute(nufds_plan_t plan, const void* d_hologram, void* d_out, void* stream);

/*
 * nufds_debug_copy -- copy an internal buffer of the last execute (tests).
 *
 * which: 1 = hologram spectrum (step 2 FFT, [ny][nx]),
 *        2 = pre-chirp FrT F ([my][mx], F[m] at x' = K_c D_F + (m - M/2) D_F; only columns
 *            fcx0 .. fcx0 + fcxn - 1 of nufds_plan_info hold F, the others the x transform alone),
 *        3 = stretch-map table (float64 pairs, see nufds_plan_info map_bytes).
 * d_dst: device buffer of at least *bytes; if d_dst is NULL only *bytes is
 * set.  Enqueued on stream.  Errors: INVALID_ARG.
 */
nufds_status_t nufds_debug_copy(nufds_plan_t plan, int32_t which, void* d_dst, uint64_t* bytes,
                                void* stream);

/* Per-launch timing of the last execute (measurement). */
typedef struct {
    char name[32];     /* kernel role, e.g. "fft1_row", "xop_gather", "yop", "output_gather" */
    double ms;         /* launch duration from HIP events recorded on the execute stream */
    uint64_t bytes;    /* algorithmic bytes of the launch (unique data it must read and write) */
} nufds_kernel_time_t;

/*
 * nufds_set_timing -- record per-launch timing of the next n_executes executes (0 turns it off).
 * While recording, execute records a HIP event before and after each kernel it
 * enqueues, on the caller's stream; nothing synchronises.  Calling this clears
 * earlier records (it synchronises the device once).  Errors: INVALID_ARG
 * (NULL plan, negative count), HIP.
 */
nufds_status_t nufds_set_timing(nufds_plan_t plan, int32_t n_executes);

/*
 * nufds_get_timings -- per-launch records of the executes recorded since nufds_set_timing,
 * in launch order.  Waits for the last recorded event.  Writes up to max_entries
 * records to out (may be NULL to query the count) and the number available to
 * *n_entries.  Errors: INVALID_ARG (NULL plan or n_entries, timing never
 * enabled), HIP.
 */
nufds_status_t nufds_get_timings(nufds_plan_t plan, nufds_kernel_time_t* out, int32_t max_entries,
                                 int32_t* n_entries);

/* nufds_destroy -- wait for the plan's work and free everything it owns.  NULL is a no-op. */
nufds_status_t nufds_destroy(nufds_plan_t plan);

/*
 * nufds_synth_hologram -- test input: a point-source hologram on the GPU.
 *
 * Evaluates H[i][j] = sum_p a_p exp(i phi_p) exp(i k r) / r, r the distance
 * from pixel (i, j) to point p, accumulated in float64 and rounded to the
 * precision.  h_points: host array of n_points rows (x, y, z, amplitude,
 * phase), metres and radians; copied before return.  d_out: device
 * [ny][nx].  Enqueued on stream.  This is the field radiated by a point
 * cloud (Sec. 2, Eq. 3 with the diverging sign), not part of the method.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
nufds_status_t nufds_synth_hologram(const double* h_points, int32_t n_points, int32_t nx,
                                    int32_t ny, double pitch, double wavelength,
                                    nufds_precision_t precision, void* d_out, void* stream);

/* ------------------------------------------------------------------ serving
 * A hologram is often reconstructed many times: partial views of chosen
 * position and size (Sec. 4, partial view) at several depths.  The forward
 * FFT of step 2 depends only on the hologram, and the stretch map of step 1
 * (Eqs. 9-10 with Eq. 16) only on the hologram's size, pitch and wavelength,
 * so both are computed once and every request runs steps 2b-5 on the
 * sub-band its view needs.
 */

typedef struct nufds_spectrum* nufds_spectrum_t;

/*
 * nufds_spectrum_create -- the centred forward FFT of one hologram (Sec. 4,
 * step 2, before the stretch), kept in device memory for any number of
 * reconstructions.
 *
 * wavelength, pitch, nx, ny, precision: as for nufds_plan_create.
 * flags: only NUFDS_FLAG_CONVERGING may be set (diverging input is
 * conjugated here).  d_hologram: device [ny][nx] of the precision, read
 * during the call.  The transform is enqueued on stream and the call waits
 * for it, so the hologram may be freed on return.  The spectrum owns
 * nx * ny complex elements of device memory until nufds_spectrum_destroy.
 * Errors: INVALID_ARG (ranges, NULLs, other flag bits), UNSUPPORTED (sizes
 * beyond the kernels), OUT_OF_MEMORY, HIP.  On error *spectrum is NULL.
 */
nufds_status_t nufds_spectrum_create(nufds_spectrum_t* spectrum, double wavelength, double pitch,
                                     int32_t nx, int32_t ny, nufds_precision_t precision,
                                     uint32_t flags, const void* d_hologram, void* stream);

/* nufds_spectrum_destroy -- wait for the device and free the spectrum.  NULL is a no-op.  No
 * queued or running execute or server request may still read it. */
nufds_status_t nufds_spectrum_destroy(nufds_spectrum_t spectrum);

/*
 * nufds_execute_spectrum -- nufds_execute from a cached spectrum: the stretch,
 * inverse FFT, Fresnel transform and output remap (steps 2-5 after the
 * forward FFT).  The plan and the spectrum must agree on nx, ny, wavelength,
 * pitch, precision and NUFDS_FLAG_CONVERGING, else INVALID_ARG.  Otherwise
 * as nufds_execute (asynchronous on stream, one execute in flight per plan);
 * the output is bit-identical to nufds_execute of the same hologram.
 */
nufds_status_t nufds_execute_spectrum(nufds_plan_t plan, nufds_spectrum_t spectrum, void* d_out,
                                      void* stream);

typedef struct nufds_server* nufds_server_t;

typedef struct {
    int32_t precision;            /* nufds_precision_t of every spectrum served */
    int32_t max_frt_size;         /* largest FrT size M (either axis) of a request, even, > 0 */
    int32_t max_view_size;        /* largest output side of a request, samples, > 0 */
    int32_t max_inflight;         /* requests executing at once (one stream each), >= 1 */
    uint64_t max_workspace_bytes; /* device bytes of all workspaces together; 0 = no limit */
} nufds_server_options_t;

/*
 * nufds_server_create -- a server of views of cached spectra.
 *
 * The server owns `slots` workspaces, each two max_frt_size^2 complex
 * buffers plus the request's chirp and output-map vectors and one HIP
 * stream (default priority): slots = max_inflight, lowered until
 * slots * workspace <= max_workspace_bytes (admission by memory).  A
 * dispatcher thread starts queued requests in arrival order as soon as a
 * slot is free (continuous batching: a request starts when any earlier one
 * ends, not when a batch fills) and a completion thread records each
 * request's latency.  The stretch-map table of each hologram geometry is
 * built on first use and shared by all requests of that geometry.  Uses the
 * current device.  Errors: INVALID_ARG (NULLs, ranges), OUT_OF_MEMORY (not
 * one workspace fits), HIP.  On error *server is NULL.
 */
nufds_status_t nufds_server_create(nufds_server_t* server, const nufds_server_options_t* opt);

/*
 * nufds_server_submit -- queue one view of a spectrum at distance z (metres).
 *
 * view as for nufds_plan_create (NULL: full view).  flags: NUFDS_FLAG_NO_STRETCH
 * and NUFDS_FLAG_NO_REMAP apply per request; NUFDS_FLAG_CONVERGING is the
 * spectrum's.  d_out: device [view.ny][view.nx] complex of the server's
 * precision, written by the request; it must stay valid until the request
 * ends.  The request's geometry is checked before it is queued.  *ticket
 * receives its id.  Thread-safe.  Errors: INVALID_ARG (NULLs, ranges,
 * precision mismatch), UNSUPPORTED (FrT size or view beyond the server's
 * limits or the kernels'), or the error a stopped server reports.
 */
nufds_status_t nufds_server_submit(nufds_server_t server, nufds_spectrum_t spectrum, double z,
                                   const nufds_view_t* view, uint32_t flags, void* d_out,
                                   uint64_t* ticket);

/*
 * nufds_server_poll -- state of a request without consuming it: *state is
 * 0 (queued or running), 1 (done) or 2 (failed); once done, *latency_ms is
 * the host time from submit to the completion of its last kernel.
 * Errors: INVALID_ARG (NULLs, unknown ticket).
 */
nufds_status_t nufds_server_poll(nufds_server_t server, uint64_t ticket, int32_t* state,
                                 double* latency_ms);

/*
 * nufds_server_wait -- block until the request ends, write its latency
 * (latency_ms may be NULL), release the ticket and return the request's
 * status (its message through nufds_last_error on the calling thread).
 * Errors: INVALID_ARG (NULL server, unknown ticket), or the request's own.
 */
nufds_status_t nufds_server_wait(nufds_server_t server, uint64_t ticket, double* latency_ms);

/* nufds_server_destroy -- run every queued request to its end, stop the threads and free the
 * workspaces and tables.  NULL is a no-op. */
nufds_status_t nufds_server_destroy(nufds_server_t server);

/* ------------------------------------------------------------------ focal stack
 *
 * Full views of one hologram at several depths, as in the multi-depth
 * reconstructions of Sec. 5 (Figs. 8 and 10: the same hologram brought to
 * focus at two distances).  At the FrT pitch D_F = lambda z / (N D) the
 * stretched band (steps 1-2, Eqs. 9-10 with Eq. 16) and its inverse DFT do
 * not depend on z, so a stack computes them once per execute into a cached
 * array and runs only the z-dependent part per depth: the chirp-in and the
 * forward DFT of Eq. 2, and the output gather of Eqs. 17-18.  All depths
 * share one FrT size: the largest the size rule gives over the depths (the
 * aperture pad N D / 2 is the most samples at the smallest z), so depth i
 * equals nufds_plan_create_ex at z[i] with that FrT size forced.
 */
typedef struct nufds_stack* nufds_stack_t;

/*
 * nufds_stack_create -- build a focal stack of n_z full views (nx x ny
 * outputs over B(z) of Eq. 1 each) of an nx x ny hologram.
 *
 * z: host array of n_z distances in metres (any order; 1 <= n_z <= 64),
 * copied.  precision and flags as for nufds_plan_create.  The stack owns
 * the buffers of one plan at the shared FrT size M_x x M_y plus one cached
 * M_x M_y array and, per depth, its chirp and output-map vectors.  Uses the
 * current device.  Errors: INVALID_ARG (NULLs, ranges, as for
 * nufds_plan_create at each depth), UNSUPPORTED (sizes beyond the kernels),
 * OUT_OF_MEMORY, HIP.  On error *stack is NULL.
 */
nufds_status_t nufds_stack_create(nufds_stack_t* stack, double wavelength, double pitch, int32_t nx,
                                  int32_t ny, const double* z, int32_t n_z, nufds_precision_t precision,
                                  uint32_t flags);

/* nufds_stack_info -- geometry of depth i (0 <= i < n_z); workspace_bytes
 * is the whole stack's.  Errors: INVALID_ARG (NULLs, i out of range). */
nufds_status_t nufds_stack_info(nufds_stack_t stack, int32_t i, nufds_plan_info_t* out);

/*
 * nufds_stack_execute -- reconstruct every depth of the stack from one
 * hologram.
 *
 * d_hologram: device [ny][nx] complex of the stack's precision (read only).
 * d_outs: host array of n_z device pointers, d_outs[i] receiving the
 * [ny][nx] view of depth i (none may alias the hologram or another).
 * Enqueued on stream, asynchronous; one execute at a time per stack.
 * Errors: INVALID_ARG (NULLs, aliasing), HIP.
 */
nufds_status_t nufds_stack_execute(nufds_stack_t stack, const void* d_hologram, void* const* d_outs,
                                   void* stream);

/* nufds_stack_destroy -- wait for the device and free everything the stack
 * owns.  NULL is a no-op. */
nufds_status_t nufds_stack_destroy(nufds_stack_t stack);

/* nufds_status_string -- static text of a status code. */
const char* nufds_status_string(nufds_status_t status);

/* nufds_last_error -- thread-local detail of the last failure on this thread ("" if none). */
const char* nufds_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NUFDS_H */
