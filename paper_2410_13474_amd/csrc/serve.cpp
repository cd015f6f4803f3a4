// Spectrum cache and the view server of libnufds.
//
// A request is steps 2b-5 (stretch-gather, inverse FFT, chirp, FFT, output remap) of one view of a
// cached spectrum.  Requests queue in arrival order; a dispatcher thread starts each one on a free
// workspace slot (its own stream and buffers) and a completion thread polls the slots' events and
// timestamps the ends.  Nothing here computes: every step is a kernel of the plan path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "nufds.h"
#include "plan.h"
#include "special.h"

namespace nufds {

using Clock = std::chrono::steady_clock;

struct Slot {
    DevBuf w1, w2, cx, cy, ax, by;
    void* staging = nullptr;  // pinned host copy of the chirps and output-map factors
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    nufds_plan plan;          // the running request's plan (borrowed buffers)
};

struct Request {
    nufds_spectrum* spec = nullptr;
    double z = 0;
    nufds_view_t view{};
    bool has_view = false;
    uint32_t flags = 0;
    void* out = nullptr;
    Clock::time_point t0;
    int state = 0;  // 0 queued or running, 1 done, 2 failed
    nufds_status_t status = NUFDS_OK;
    std::string err;
    double latency_ms = 0;
    int slot = -1;
};

// Stretch-map table of one hologram geometry, full quadrant extent.
struct MapTable {
    int nx, ny;
    double wavelength, pitch;
    DevBuf buf;
    int kxt, kyt;
};

}  // namespace nufds

using namespace nufds;

struct nufds_server {
    nufds_server_options_t opt{};
    size_t esize = 8;
    int device = 0;
    int tile_cap = 0, col_w = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::shared_ptr<TwiddleCache> twiddles;
    std::vector<std::unique_ptr<MapTable>> tables;  // touched by the dispatcher thread only
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    std::vector<int> free_slots;
    std::vector<uint64_t> inflight;
    int dispatching = 0;  // requests taken off the queue and not yet running or failed
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread dispatcher, completer;
};

namespace nufds {

// ------------------------------------------------------------------ spectrum

static nufds_status_t spectrum_create_impl(nufds_spectrum_t* out, double wavelength, double pitch, int32_t nx,
                                           int32_t ny, nufds_precision_t precision, uint32_t flags,
                                           const void* d_hologram, hipStream_t s) {
    if (!out) return fail(NUFDS_ERR_INVALID_ARG, "spectrum is NULL");
    *out = nullptr;
    if (!d_hologram) return fail(NUFDS_ERR_INVALID_ARG, "hologram is NULL");
    if (precision != NUFDS_C64 && precision != NUFDS_C128) return fail(NUFDS_ERR_INVALID_ARG, "unknown precision");
    if (flags & ~(uint32_t)NUFDS_FLAG_CONVERGING)
        return fail(NUFDS_ERR_INVALID_ARG, "a spectrum takes NUFDS_FLAG_CONVERGING only");
    nufds_plan_info_t g;  // validates wavelength, pitch and the sizes (z and view do not matter)
    NUFDS_TRY(compute_geometry(wavelength, pitch, nx, ny, 1.0, nullptr, flags, nullptr, &g));
    g.mx = g.my = 2;
    g.sx = g.sy = 2;
    NUFDS_TRY(check_sizes(g));
    std::unique_ptr<nufds_spectrum> sp(new (std::nothrow) nufds_spectrum());
    if (!sp) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    sp->nx = nx;
    sp->ny = ny;
    sp->wavelength = wavelength;
    sp->pitch = pitch;
    sp->prec = precision;
    sp->flags = flags;
    sp->esize = precision == NUFDS_C64 ? 8 : 16;
    NUFDS_HIP_TRY(hipGetDevice(&sp->device));
    const size_t nn = (size_t)nx * ny;
    NUFDS_TRY(dev_alloc(sp->spec, nn * sp->esize));
    // a transient plan for the forward transform: its scratch and twiddles go away with it
    nufds_plan t;
    t.info = g;
    t.wavelength = wavelength;
    t.pitch = pitch;
    t.flags = flags;
    t.prec = precision;
    t.esize = sp->esize;
    t.device = sp->device;
    t.tile_cap = tile_override();
    t.col_w = col_w_override();
    t.twiddles = std::make_shared<TwiddleCache>();
    t.twiddles->esize = sp->esize;
    nufds_status_t st = dev_alloc(t.work1, nn * sp->esize);
    if (st == NUFDS_OK)
        st = precision == NUFDS_C64 ? prepare_twiddles<float>(&t, true, false) : prepare_twiddles<double>(&t, true, false);
    if (st == NUFDS_OK)
        st = precision == NUFDS_C64 ? run_fft1<float>(&t, d_hologram, sp->spec.p, t.work1.p, s)
                                    : run_fft1<double>(&t, d_hologram, sp->spec.p, t.work1.p, s);
    hipError_t e = hipStreamSynchronize(s);
    dev_free(t.work1);
    if (st != NUFDS_OK) {
        dev_free(sp->spec);
        return st;
    }
    if (e != hipSuccess) {
        dev_free(sp->spec);
        return hip_fail(e, "spectrum transform");
    }
    *out = sp.release();
    return NUFDS_OK;
}

// ------------------------------------------------------------------ server

static size_t slot_bytes(const nufds_server_options_t& o, size_t esize) {
    const size_t m = (size_t)o.max_frt_size;
    return 2 * m * m * esize + 2 * m * esize + 2 * (size_t)o.max_view_size * sizeof(double);
}

static void slot_free(Slot& sl) {
    dev_free(sl.w1);
    dev_free(sl.w2);
    dev_free(sl.cx);
    dev_free(sl.cy);
    dev_free(sl.ax);
    dev_free(sl.by);
    if (sl.staging) (void)hipHostFree(sl.staging);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    sl.staging = nullptr;
    sl.done = nullptr;
    sl.stream = nullptr;
}

static nufds_status_t slot_alloc(Slot& sl, const nufds_server_options_t& o, size_t esize) {
    const size_t m = (size_t)o.max_frt_size, v = (size_t)o.max_view_size;
    NUFDS_TRY(dev_alloc(sl.w1, m * m * esize));
    NUFDS_TRY(dev_alloc(sl.w2, m * m * esize));
    NUFDS_TRY(dev_alloc(sl.cx, m * esize));
    NUFDS_TRY(dev_alloc(sl.cy, m * esize));
    NUFDS_TRY(dev_alloc(sl.ax, v * sizeof(double)));
    NUFDS_TRY(dev_alloc(sl.by, v * sizeof(double)));
    NUFDS_HIP_TRY(hipHostMalloc(&sl.staging, 2 * m * esize + 2 * v * sizeof(double), hipHostMallocDefault));
    NUFDS_HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    NUFDS_HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    return NUFDS_OK;
}

// The map table of the spectrum's geometry, built on first use (dispatcher thread only).
static nufds_status_t get_table(nufds_server* S, const nufds_spectrum* sp, hipStream_t s, MapTable** out) {
    for (auto& t : S->tables)
        if (t->nx == sp->nx && t->ny == sp->ny && t->wavelength == sp->wavelength && t->pitch == sp->pitch) {
            *out = t.get();
            return NUFDS_OK;
        }
    std::unique_ptr<MapTable> t(new (std::nothrow) MapTable());
    if (!t) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    t->nx = sp->nx;
    t->ny = sp->ny;
    t->wavelength = sp->wavelength;
    t->pitch = sp->pitch;
    table_extent(sp->wavelength, sp->pitch, sp->nx, sp->ny, &t->kxt, &t->kyt);
    NUFDS_TRY(dev_alloc(t->buf, map_table_bytes(t->kxt, t->kyt)));
    hipError_t e = launch_map_table(static_cast<double*>(t->buf.p), t->kxt, t->kyt, sp->wavelength,
                                    sp->nx * sp->pitch, sp->ny * sp->pitch, sp->wavelength / (2.0 * sp->pitch), 1, nullptr, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // other slots' streams read it next
    if (e != hipSuccess) {
        dev_free(t->buf);
        return hip_fail(e, "map table");
    }
    *out = t.get();
    S->tables.push_back(std::move(t));
    return NUFDS_OK;
}

template <typename R>
static nufds_status_t launch_request_t(nufds_server* S, Slot& sl, const Request& rq) {
    const nufds_spectrum* sp = rq.spec;
    const uint32_t flags = (rq.flags & ~(uint32_t)NUFDS_FLAG_CONVERGING) | (sp->flags & NUFDS_FLAG_CONVERGING);
    nufds_plan_info_t g;
    NUFDS_TRY(compute_geometry(sp->wavelength, sp->pitch, sp->nx, sp->ny, rq.z, rq.has_view ? &rq.view : nullptr,
                               flags, nullptr, &g));
    nufds_plan& p = sl.plan;
    p.info = g;
    p.info.precision = sp->prec;
    p.wavelength = sp->wavelength;
    p.pitch = sp->pitch;
    p.z = rq.z;
    p.flags = flags;
    p.prec = sp->prec;
    p.esize = sizeof(cpx<R>);
    p.device = S->device;
    p.tile_cap = S->tile_cap;
    p.col_w = S->col_w;
    p.twiddles = S->twiddles;
    p.work1 = borrow(sl.w1.p, sl.w1.bytes);
    p.work2 = borrow(sl.w2.p, sl.w2.bytes);
    p.chirp_x = borrow(sl.cx.p, (size_t)g.mx * sizeof(cpx<R>));
    p.chirp_y = borrow(sl.cy.p, (size_t)g.my * sizeof(cpx<R>));
    p.ax = borrow(sl.ax.p, (size_t)g.sx * sizeof(double));
    p.by = borrow(sl.by.p, (size_t)g.sy * sizeof(double));
    p.table = DevBuf();
    p.kxt = p.kyt = -1;
    if (!(flags & NUFDS_FLAG_NO_STRETCH)) {
        MapTable* mt = nullptr;
        NUFDS_TRY(get_table(S, sp, sl.stream, &mt));
        p.table = borrow(mt->buf.p, mt->buf.bytes);
        p.kxt = mt->kxt;
        p.kyt = mt->kyt;
    }
    NUFDS_TRY(prepare_twiddles<R>(&p, false, true));
    // chirps (Eq. 2) and output-map factors (Eqs. 17-18) on the host, float64, then one copy each
    const size_t m = (size_t)S->opt.max_frt_size;
    cpx<R>* hcx = static_cast<cpx<R>*>(sl.staging);
    cpx<R>* hcy = hcx + m;
    double* hax = reinterpret_cast<double*>(hcy + m);
    double* hby = hax + S->opt.max_view_size;
    std::vector<double> re, im;
    chirp_vector(g.mx, g.nx, p.pitch, p.wavelength, p.z, re, im);
    for (int i = 0; i < g.mx; ++i) hcx[i] = mk(R(re[i]), R(im[i]));
    chirp_vector(g.my, g.ny, p.pitch, p.wavelength, p.z, re, im);
    for (int i = 0; i < g.my; ++i) hcy[i] = mk(R(re[i]), R(im[i]));
    const hipStream_t s = sl.stream;
    NUFDS_HIP_TRY(hipMemcpyAsync(p.chirp_x.p, hcx, p.chirp_x.bytes, hipMemcpyHostToDevice, s));
    NUFDS_HIP_TRY(hipMemcpyAsync(p.chirp_y.p, hcy, p.chirp_y.bytes, hipMemcpyHostToDevice, s));
    if (!(flags & NUFDS_FLAG_NO_REMAP)) {
        for (int j = 0; j < g.sx; ++j) hax[j] = output_map_factor(g.cx + (double)(j - g.sx / 2) * g.dox, rq.z);
        for (int i = 0; i < g.sy; ++i) hby[i] = output_map_factor(g.cy + (double)(i - g.sy / 2) * g.doy, rq.z);
        NUFDS_HIP_TRY(hipMemcpyAsync(p.ax.p, hax, p.ax.bytes, hipMemcpyHostToDevice, s));
        NUFDS_HIP_TRY(hipMemcpyAsync(p.by.p, hby, p.by.bytes, hipMemcpyHostToDevice, s));
    }
    NUFDS_TRY(run_band<R>(&p, sp->spec.p, rq.out, s));
    NUFDS_HIP_TRY(hipEventRecord(sl.done, s));
    return NUFDS_OK;
}

static void dispatch_loop(nufds_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return S->stop || (!S->queue.empty() && !S->free_slots.empty()); });
        if (S->stop) break;
        const uint64_t t = S->queue.front();
        S->queue.pop_front();
        const int si = S->free_slots.back();
        S->free_slots.pop_back();
        ++S->dispatching;
        Request rq = S->reqs[t];
        lk.unlock();
        set_error("");
        nufds_status_t st;
        try {
            st = S->esize == 8 ? launch_request_t<float>(S, *S->slots[si], rq)
                               : launch_request_t<double>(S, *S->slots[si], rq);
        } catch (const std::exception& ex) {
            st = fail(NUFDS_ERR_OUT_OF_MEMORY, std::string("request setup: ") + ex.what());
        }
        // a request that failed part-way may have work queued on the slot: let it drain before the
        // slot (and its staging memory) is reused
        if (st != NUFDS_OK) (void)hipStreamSynchronize(S->slots[si]->stream);
        const std::string err = nufds_last_error();
        lk.lock();
        --S->dispatching;
        Request& r = S->reqs[t];
        r.slot = si;
        if (st != NUFDS_OK) {
            r.state = 2;
            r.status = st;
            r.err = err;
            r.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r.t0).count();
            S->free_slots.push_back(si);
        } else {
            S->inflight.push_back(t);
        }
        S->cv.notify_all();
    }
}

static void complete_loop(nufds_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return S->stop || !S->inflight.empty(); });
        if (S->inflight.empty()) break;  // stopped with nothing running
        std::vector<std::pair<uint64_t, int>> cur;
        for (uint64_t t : S->inflight) cur.emplace_back(t, S->reqs[t].slot);
        lk.unlock();
        std::vector<std::pair<uint64_t, hipError_t>> ended;
        for (auto& c : cur) {
            const hipError_t q = hipEventQuery(S->slots[c.second]->done);
            if (q != hipErrorNotReady) ended.emplace_back(c.first, q);
        }
        const Clock::time_point now = Clock::now();
        if (ended.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
        for (auto& e : ended) {
            Request& r = S->reqs[e.first];
            r.latency_ms = std::chrono::duration<double, std::milli>(now - r.t0).count();
            if (e.second == hipSuccess) {
                r.state = 1;
            } else {
                r.state = 2;
                r.status = NUFDS_ERR_HIP;
                r.err = std::string("request: ") + hipGetErrorString(e.second);
            }
            S->free_slots.push_back(r.slot);
            S->inflight.erase(std::find(S->inflight.begin(), S->inflight.end(), e.first));
        }
        if (!ended.empty()) S->cv.notify_all();
    }
}

static void server_free(nufds_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // finish what was submitted, then stop both threads
        S->cv.wait(lk, [&] { return S->queue.empty() && S->dispatching == 0 && S->inflight.empty(); });
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->dispatcher.joinable()) S->dispatcher.join();
    if (S->completer.joinable()) S->completer.join();
    (void)hipDeviceSynchronize();
    for (auto& sl : S->slots) slot_free(*sl);
    for (auto& t : S->tables) dev_free(t->buf);
    S->twiddles.reset();
    delete S;
}

static nufds_status_t server_create_impl(nufds_server_t* out, const nufds_server_options_t* o) {
    if (!out || !o) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (o->precision != NUFDS_C64 && o->precision != NUFDS_C128) return fail(NUFDS_ERR_INVALID_ARG, "unknown precision");
    if (o->max_frt_size <= 0 || (o->max_frt_size & 1) || o->max_frt_size > kMaxLen || o->max_view_size <= 0 ||
        o->max_inflight < 1)
        return fail(NUFDS_ERR_INVALID_ARG, "server limits out of range");
    const size_t esize = o->precision == NUFDS_C64 ? 8 : 16;
    const size_t per = slot_bytes(*o, esize);
    int nslots = o->max_inflight;
    if (o->max_workspace_bytes > 0) nslots = (int)std::min<uint64_t>(nslots, o->max_workspace_bytes / per);
    if (nslots < 1) return fail(NUFDS_ERR_OUT_OF_MEMORY, "max_workspace_bytes holds no workspace");
    std::unique_ptr<nufds_server> S(new (std::nothrow) nufds_server());
    if (!S) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
    S->opt = *o;
    S->esize = esize;
    S->tile_cap = tile_override();
    S->col_w = col_w_override();
    S->twiddles = std::make_shared<TwiddleCache>();
    S->twiddles->esize = esize;
    NUFDS_HIP_TRY(hipGetDevice(&S->device));
    for (int i = 0; i < nslots; ++i) {
        S->slots.emplace_back(new (std::nothrow) Slot());
        if (!S->slots.back()) return fail(NUFDS_ERR_OUT_OF_MEMORY, "host allocation failed");
        nufds_status_t st = slot_alloc(*S->slots.back(), *o, esize);
        if (st != NUFDS_OK) {
            const std::string msg = nufds_last_error();
            for (auto& sl : S->slots) slot_free(*sl);
            set_error(msg);
            return st;
        }
        S->free_slots.push_back(i);
    }
    nufds_server* raw = S.release();
    raw->dispatcher = std::thread(dispatch_loop, raw);
    raw->completer = std::thread(complete_loop, raw);
    *out = raw;
    return NUFDS_OK;
}

static nufds_status_t server_submit_impl(nufds_server* S, nufds_spectrum* sp, double z, const nufds_view_t* view,
                                         uint32_t flags, void* d_out, uint64_t* ticket) {
    if (!S || !sp || !d_out || !ticket) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    if (sp->prec != S->opt.precision) return fail(NUFDS_ERR_INVALID_ARG, "spectrum precision differs from the server's");
    if (flags & ~7u) return fail(NUFDS_ERR_INVALID_ARG, "unknown flag bits");
    const uint32_t f = (flags & ~(uint32_t)NUFDS_FLAG_CONVERGING) | (sp->flags & NUFDS_FLAG_CONVERGING);
    nufds_plan_info_t g;
    NUFDS_TRY(compute_geometry(sp->wavelength, sp->pitch, sp->nx, sp->ny, z, view, f, nullptr, &g));
    NUFDS_TRY(check_sizes(g));
    if (g.mx > S->opt.max_frt_size || g.my > S->opt.max_frt_size)
        return fail(NUFDS_ERR_UNSUPPORTED, "the view needs FrT size " + std::to_string(std::max(g.mx, g.my)) +
                                               " > the server's max_frt_size");
    if (g.sx > S->opt.max_view_size || g.sy > S->opt.max_view_size)
        return fail(NUFDS_ERR_UNSUPPORTED, "view larger than the server's max_view_size");
    Request r;
    r.spec = sp;
    r.z = z;
    r.has_view = view != nullptr;
    if (view) r.view = *view;
    r.flags = flags;
    r.out = d_out;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(NUFDS_ERR_INVALID_ARG, "server is stopping");
    const uint64_t t = S->next_ticket++;
    r.t0 = Clock::now();
    S->reqs.emplace(t, r);
    S->queue.push_back(t);
    *ticket = t;
    S->cv.notify_all();
    return NUFDS_OK;
}

}  // namespace nufds

extern "C" {

nufds_status_t nufds_spectrum_create(nufds_spectrum_t* spectrum, double wavelength, double pitch, int32_t nx,
                                     int32_t ny, nufds_precision_t precision, uint32_t flags, const void* d_hologram,
                                     void* stream) {
    return spectrum_create_impl(spectrum, wavelength, pitch, nx, ny, precision, flags, d_hologram,
                                static_cast<hipStream_t>(stream));
}

nufds_status_t nufds_spectrum_destroy(nufds_spectrum_t spectrum) {
    if (!spectrum) return NUFDS_OK;
    (void)hipDeviceSynchronize();
    dev_free(spectrum->spec);
    delete spectrum;
    return NUFDS_OK;
}

nufds_status_t nufds_server_create(nufds_server_t* server, const nufds_server_options_t* opt) {
    return server_create_impl(server, opt);
}

nufds_status_t nufds_server_submit(nufds_server_t server, nufds_spectrum_t spectrum, double z,
                                   const nufds_view_t* view, uint32_t flags, void* d_out, uint64_t* ticket) {
    return server_submit_impl(server, spectrum, z, view, flags, d_out, ticket);
}

nufds_status_t nufds_server_poll(nufds_server_t server, uint64_t ticket, int32_t* state, double* latency_ms) {
    if (!server || !state || !latency_ms) return fail(NUFDS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->reqs.find(ticket);
    if (it == server->reqs.end()) return fail(NUFDS_ERR_INVALID_ARG, "unknown ticket");
    *state = it->second.state;
    *latency_ms = it->second.state ? it->second.latency_ms : 0.0;
    return NUFDS_OK;
}

nufds_status_t nufds_server_wait(nufds_server_t server, uint64_t ticket, double* latency_ms) {
    if (!server) return fail(NUFDS_ERR_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(server->mu);
    auto it = server->reqs.find(ticket);
    if (it == server->reqs.end()) return fail(NUFDS_ERR_INVALID_ARG, "unknown ticket");
    server->cv.wait(lk, [&] { return it->second.state != 0; });
    const Request r = it->second;
    server->reqs.erase(it);
    if (latency_ms) *latency_ms = r.latency_ms;
    if (r.status != NUFDS_OK) return fail(r.status, r.err);
    return NUFDS_OK;
}

nufds_status_t nufds_server_destroy(nufds_server_t server) {
    server_free(server);
    return NUFDS_OK;
}

}  // extern "C"
