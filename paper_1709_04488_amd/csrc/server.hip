// Request executor for serving: slots of one HIP stream and one context
// each, driven by a few native worker threads.  Every HIP call a slot makes
// (its context, its device arrays, its pinned staging, its stream) happens on
// the worker thread that owns the slot; the caller's threads only hand
// requests over and collect them.
//
// A worker owns slots k, k + T, k + 2T, ... (T threads).  For each request
// handed to one of them it stages the nine input arrays into the slot's
// pinned memory, copies them to the device in one transfer and enqueues the
// request (sph_evaluate, or sph_upload_state + captured steps +
// sph_download_state) and the copies of its outputs back, then goes on to its
// other slots.  When a slot's stream reports the work done, the worker reads
// the status and counters, writes the outputs into the caller's arrays and
// marks the slot idle before publishing the request as done.  So a thread
// keeps several requests in flight on the GPU while it stages the next.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sph.h"

namespace {

constexpr int kI32 = 2;         // nngb, nforce
constexpr int kMaxSlots = 64;
// device bytes per particle of a slot's arrays: every FP64 field and both counts
constexpr size_t kArrayBytesPerParticle = SPH_NF64 * sizeof(double) + kI32 * sizeof(int32_t);

struct Worker;

struct Slot {
    int idx = 0;
    Worker *w = nullptr;
    // guarded by w->mu
    sph_request *job = nullptr;  // handed over, not yet started
    bool busy = false;           // from submit until the request is published
    bool release = false;        // the caller asks the worker to free its buffers
    // owned by the worker thread
    sph_request *run = nullptr;  // enqueued on the stream, not yet finished
    bool eval = false;           // the running request's kind
    bool block = false;          // block time-steps: a sub-step is in flight
    int64_t block_pairs = 0;     // pairs of the sub-steps so far
    int lo = 0, hi = -1;         // rows of the outputs copied back
    std::chrono::steady_clock::time_point t_enqueued;
    hipStream_t stream = nullptr;
    hipError_t stream_err = hipSuccess;
    sph_ctx *ctx = nullptr;
    sph_params cur{};
    double *dev = nullptr;       // SPH_NF64 rows of n, then the int32 rows
    int64_t cap = 0;             // particles dev holds
    double *pin = nullptr;       // pinned staging: SPH_NF64 rows, then the int32 rows
    int64_t pcap = 0;
    std::atomic<size_t> bytes{0};
};

struct Worker {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Slot *> slots;
    bool quit = false;
};

// a worker with a request in flight looks at its streams this often
constexpr auto kPoll = std::chrono::microseconds(20);

}  // namespace

struct sph_server {
    int device = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<std::unique_ptr<Worker>> workers;
    std::mutex mu;               // guards done and running
    std::condition_variable cv;
    std::deque<sph_request *> done;
    int running = 0;
};

namespace {

void set_error(sph_request *r, int32_t status, const std::string &msg)
{
    r->status = status;
    std::snprintf(r->error, sizeof(r->error), "%s", msg.c_str());
}

sph_status hip_fail(sph_request *r, hipError_t e, const char *what)
{
    set_error(r, SPH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return SPH_EDEVICE;
}

void free_buffers(Slot &s)
{
    if (s.ctx) { (void)sph_destroy(s.ctx); s.ctx = nullptr; }
    if (s.dev) { (void)hipFree(s.dev); s.dev = nullptr; }
    if (s.pin) { (void)hipHostFree(s.pin); s.pin = nullptr; }
    s.cap = s.pcap = 0;
    s.bytes.store(0);
}

// The slot's context with the request's parameters, its device arrays and
// pinned staging for n particles (grown, never shrunk, until released).
sph_status prepare(Slot &s, sph_request *r)
{
    if (s.stream_err != hipSuccess) return hip_fail(r, s.stream_err, "hipStreamCreate");
    if (!s.ctx) {
        sph_status st = sph_create(&s.ctx, &r->params, s.stream, 0);
        if (st != SPH_OK) {
            set_error(r, st, "sph_create rejected the request's parameters or device");
            s.ctx = nullptr;
            return st;
        }
        s.cur = r->params;
    } else if (std::memcmp(&s.cur, &r->params, sizeof(sph_params)) != 0) {
        sph_status st = sph_set_params(s.ctx, &r->params);
        if (st != SPH_OK) {
            set_error(r, st, std::string("sph_set_params: ") + sph_last_error(s.ctx));
            return st;
        }
        s.cur = r->params;
    }
    const int64_t n = r->n;
    const size_t bytes = (size_t)n * kArrayBytesPerParticle;
    if (n > s.cap) {
        if (s.dev) {
            hipError_t e = hipStreamSynchronize(s.stream);
            if (e != hipSuccess) return hip_fail(r, e, "hipStreamSynchronize");
            (void)hipFree(s.dev);
            s.dev = nullptr;
            s.cap = 0;
        }
        hipError_t e = hipMalloc(&s.dev, bytes);
        if (e != hipSuccess) {
            s.dev = nullptr;
            set_error(r, SPH_ENOMEM, "slot arrays: " + std::string(hipGetErrorString(e)));
            return SPH_ENOMEM;
        }
        s.cap = n;
    }
    if (n > s.pcap) {
        if (s.pin) { (void)hipHostFree(s.pin); s.pin = nullptr; s.pcap = 0; }
        hipError_t e = hipHostMalloc((void **)&s.pin, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            s.pin = nullptr;
            set_error(r, SPH_ENOMEM, "pinned staging: " + std::string(hipGetErrorString(e)));
            return SPH_ENOMEM;
        }
        s.pcap = n;
    }
    s.bytes.store(sph_device_bytes(s.ctx) + (size_t)s.cap * kArrayBytesPerParticle);
    return SPH_OK;
}

// Rows of n values at the start of a buffer: the SPH_NF64 FP64 fields, then
// the two int32 counts.
sph_particles device_view(double *base, int64_t n)
{
    sph_particles d{};
    double *f[SPH_NF64];
    for (int k = 0; k < SPH_NF64; k++) f[k] = base + (size_t)k * n;
    int32_t *iv = reinterpret_cast<int32_t *>(base + (size_t)SPH_NF64 * n);
    d.n = n;
    d.x = f[SPH_F_X]; d.y = f[SPH_F_Y]; d.z = f[SPH_F_Z];
    d.vx = f[SPH_F_VX]; d.vy = f[SPH_F_VY]; d.vz = f[SPH_F_VZ];
    d.m = f[SPH_F_M]; d.u = f[SPH_F_U]; d.h = f[SPH_F_H];
    d.rho = f[SPH_F_RHO]; d.omega = f[SPH_F_OMEGA];
    d.pressure = f[SPH_F_PRESSURE]; d.cs = f[SPH_F_CS];
    d.ax = f[SPH_F_AX]; d.ay = f[SPH_F_AY]; d.az = f[SPH_F_AZ];
    d.dudt = f[SPH_F_DUDT]; d.vsig = f[SPH_F_VSIG]; d.dt = f[SPH_F_DT];
    d.nngb = iv; d.nforce = iv + n;
    return d;
}

double seconds_since(std::chrono::steady_clock::time_point &t)
{
    const auto now = std::chrono::steady_clock::now();
    const double d = std::chrono::duration<double>(now - t).count();
    t = now;
    return d;
}

// Stage and enqueue request r on slot s.  Returns true when the request is
// in flight; false when it is already complete (n = 0 or an error, with
// r->status set).
bool enqueue_outputs(Slot &s, sph_request *r, const sph_particles &d);

bool start(Slot &s, sph_request *r)
{
    const int64_t n = r->n;
    if (n == 0) {               // nothing to compute, nothing allocated
        set_error(r, SPH_OK, "");
        return false;
    }
    auto t = std::chrono::steady_clock::now();
    if (prepare(s, r) != SPH_OK) return false;
    const size_t row = (size_t)n * sizeof(double);
    for (int k = 0; k < SPH_NIN; k++) std::memcpy(s.pin + (size_t)k * n, r->in[k], row);
    r->host_seconds[0] = seconds_since(t);
    hipError_t e = hipMemcpyAsync(s.dev, s.pin, SPH_NIN * row, hipMemcpyHostToDevice, s.stream);
    if (e != hipSuccess) { hip_fail(r, e, "input copy"); return false; }
    sph_particles d = device_view(s.dev, n);

    s.eval = r->kind == SPH_REQUEST_EVALUATE;
    s.block = false;
    s.block_pairs = 0;
    sph_status st;
    if (s.eval) {
        st = sph_evaluate(s.ctx, &d);
    } else if (r->params.block_lmax > 0) {
        // block time-steps: one sub-step at a time; the worker reads the
        // device clock whenever the stream drains (advance) and enqueues the
        // next sub-step, or the download once nsteps level-0 steps are done
        st = sph_upload_state(s.ctx, &d);
        if (st == SPH_OK && r->nsteps > 0) {
            st = sph_substep(s.ctx);
            s.block = st == SPH_OK;
        }
        if (st == SPH_OK && !s.block) st = sph_download_state(s.ctx, &d);
    } else {
        st = sph_upload_state(s.ctx, &d);
        // two steps per replay of a captured graph, then one eager step for an
        // odd count
        int32_t left = r->nsteps;
        if (st == SPH_OK && left >= 2) {
            st = sph_capture_steps(s.ctx, 0.0);
            for (; st == SPH_OK && left >= 2; left -= 2) st = sph_replay_steps(s.ctx);
        }
        for (; st == SPH_OK && left > 0; left--) st = sph_step(s.ctx, 0.0, nullptr);
        if (st == SPH_OK) st = sph_download_state(s.ctx, &d);
    }
    if (st != SPH_OK) {
        set_error(r, st, sph_last_error(s.ctx));
        (void)sph_sync(s.ctx);   // clear the sticky status for the slot's next request
        return false;
    }
    if (!s.block && !enqueue_outputs(s, r, d)) return false;
    r->host_seconds[1] = seconds_since(t);
    s.t_enqueued = t;
    return true;
}

// The copies of the wanted outputs to the pinned staging (after the
// evaluation or the download on the slot's stream).
bool enqueue_outputs(Slot &s, sph_request *r, const sph_particles &d)
{
    const int64_t n = r->n;
    const size_t row = (size_t)n * sizeof(double);
    hipError_t e;
    // the wanted outputs: one copy of the rows from the first to the last wanted
    s.lo = SPH_NF64;
    s.hi = -1;
    for (int k = 0; k < SPH_NF64; k++) {
        const bool written = s.eval ? k >= SPH_F_H : k != SPH_F_M;
        if (written && r->out[k]) { s.lo = std::min(s.lo, k); s.hi = std::max(s.hi, k); }
    }
    if (s.hi >= 0) {
        e = hipMemcpyAsync(s.pin + (size_t)s.lo * n, d.x + (size_t)s.lo * n,
                           (size_t)(s.hi - s.lo + 1) * row, hipMemcpyDeviceToHost, s.stream);
        if (e != hipSuccess) { hip_fail(r, e, "output copy"); return false; }
    }
    if (r->iout[0] || r->iout[1]) {
        e = hipMemcpyAsync(s.pin + (size_t)SPH_NF64 * n, d.nngb, (size_t)kI32 * n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s.stream);
        if (e != hipSuccess) { hip_fail(r, e, "count copy"); return false; }
    }
    return true;
}

// A block request whose sub-step has drained: count its pairs, then enqueue
// the next sub-step, or the download and output copies once the clock has
// completed nsteps level-0 steps.  false: the request failed (error set).
bool advance(Slot &s, sph_request *r)
{
    sph_state_stats info;
    // the stream is idle, so neither call waits; a status the device raised
    // in the sub-step (e.g. a level beyond block_lmax) ends the request now
    sph_status st = sph_sync(s.ctx);
    if (st == SPH_OK) st = sph_state_info(s.ctx, &info);
    if (st == SPH_OK) {
        s.block_pairs += info.n_dens_pairs + info.n_force_pairs;
        if (info.block_full_steps < r->nsteps) {
            st = sph_substep(s.ctx);
            if (st == SPH_OK) return true;
        } else {
            s.block = false;
            sph_particles d = device_view(s.dev, r->n);
            st = sph_download_state(s.ctx, &d);
            if (st == SPH_OK) return enqueue_outputs(s, r, d);
        }
    }
    set_error(r, st, sph_last_error(s.ctx));
    (void)sph_sync(s.ctx);
    return false;
}

// The request in flight on slot s, whose stream has drained: its status,
// counters and outputs.
void finish(Slot &s, sph_request *r)
{
    auto t = std::chrono::steady_clock::now();
    r->host_seconds[2] = std::chrono::duration<double>(t - s.t_enqueued).count();
    const int64_t n = r->n;
    sph_status st = sph_sync(s.ctx);
    if (st != SPH_OK) {
        set_error(r, st, sph_last_error(s.ctx));
        (void)sph_sync(s.ctx);
        return;
    }
    st = sph_state_info(s.ctx, &r->info);
    if (st != SPH_OK) {
        set_error(r, st, sph_last_error(s.ctx));
        return;
    }
    const size_t row = (size_t)n * sizeof(double);
    for (int k = s.lo; k <= s.hi; k++)
        if (r->out[k] && (s.eval ? k >= SPH_F_H : k != SPH_F_M))
            std::memcpy(r->out[k], s.pin + (size_t)k * n, row);
    const int32_t *ipin = reinterpret_cast<const int32_t *>(s.pin + (size_t)SPH_NF64 * n);
    for (int k = 0; k < kI32; k++)
        if (r->iout[k]) std::memcpy(r->iout[k], ipin + (size_t)k * n, n * sizeof(int32_t));
    r->host_seconds[3] = seconds_since(t);
    const int64_t pairs = r->info.n_dens_pairs + r->info.n_force_pairs;
    // block time-steps: the pairs of all sub-steps (active particles only)
    r->interactions = s.eval ? pairs
                      : (r->params.block_lmax > 0 && r->nsteps > 0)
                          ? s.block_pairs
                          : pairs * std::max<int64_t>(r->nsteps, 1);
    set_error(r, SPH_OK, "");
}

// Mark the slot idle, then hand the request to the waiters (the worker's lock
// is held on entry and on return, not while the server's is taken).
void publish(sph_server *S, Slot &s, sph_request *r, std::unique_lock<std::mutex> &lk)
{
    s.busy = false;
    lk.unlock();
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->done.push_back(r);
        S->running--;
    }
    S->cv.notify_all();
    lk.lock();
}

void worker(sph_server *S, Worker *W)
{
    (void)hipSetDevice(S->device);
    for (Slot *s : W->slots) {
        s->stream_err = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (s->stream_err != hipSuccess) s->stream = nullptr;
    }
    std::unique_lock<std::mutex> lk(W->mu);
    for (;;) {
        bool did = false, running = false, waiting = false;
        for (Slot *s : W->slots) {
            if (s->release) {
                lk.unlock();
                free_buffers(*s);
                lk.lock();
                s->release = false;
                s->busy = false;
                W->cv.notify_all();
                did = true;
            }
            if (s->job) {
                sph_request *r = s->job;
                s->job = nullptr;
                lk.unlock();
                std::memset(&r->info, 0, sizeof(r->info));
                std::memset(r->host_seconds, 0, sizeof(r->host_seconds));
                r->interactions = 0;
                r->slot = s->idx;
                const bool flying = start(*s, r);
                lk.lock();
                if (flying) s->run = r;
                else publish(S, *s, r, lk);
                did = true;
            }
        }
        for (Slot *s : W->slots) {
            if (!s->run) continue;
            lk.unlock();
            const bool drained = hipStreamQuery(s->stream) != hipErrorNotReady;
            bool ready = false;
            if (drained && s->block) {
                // a block sub-step has finished: the next one (or the
                // download) is in flight again, or the request failed (its
                // error set; nothing to finish)
                ready = !advance(*s, s->run);
            } else if (drained) {
                finish(*s, s->run);
                ready = true;
            }
            lk.lock();
            if (ready) {
                sph_request *r = s->run;
                s->run = nullptr;
                publish(S, *s, r, lk);
                did = true;
            } else {
                running = true;
            }
        }
        for (Slot *s : W->slots) waiting = waiting || s->job || s->release;
        if (did || waiting) continue;
        if (running) {
            W->cv.wait_for(lk, kPoll);
        } else {
            if (W->quit) break;
            W->cv.wait(lk, [&] {
                bool any = W->quit;
                for (Slot *s : W->slots) any = any || s->job || s->release;
                return any;
            });
        }
    }
    lk.unlock();
    for (Slot *s : W->slots) {
        free_buffers(*s);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        s->stream = nullptr;
    }
}

}  // namespace

extern "C" {

sph_status sph_server_create(sph_server **out, int32_t slots, int32_t threads)
{
    if (!out) return SPH_EINVAL;
    *out = nullptr;
    if (slots < 1 || slots > kMaxSlots || threads < 0 || threads > slots) return SPH_EINVAL;
    if (threads == 0) threads = slots;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return SPH_EDEVICE;
    auto *S = new sph_server;
    S->device = device;
    for (int k = 0; k < threads; k++) S->workers.emplace_back(new Worker);
    for (int k = 0; k < slots; k++) {
        S->slots.emplace_back(new Slot);
        Slot *s = S->slots.back().get();
        s->idx = k;
        s->w = S->workers[k % threads].get();
        s->w->slots.push_back(s);
    }
    for (auto &w : S->workers) w->th = std::thread(worker, S, w.get());
    *out = S;
    return SPH_OK;
}

sph_status sph_server_submit(sph_server *S, int32_t slot, sph_request *r)
{
    if (!S || !r || slot < 0 || slot >= (int32_t)S->slots.size()) return SPH_EINVAL;
    if (r->kind != SPH_REQUEST_EVALUATE && r->kind != SPH_REQUEST_INTEGRATE) return SPH_EINVAL;
    if (r->n < 0 || r->nsteps < 0) return SPH_EINVAL;
    if (r->n > 0)
        for (int k = 0; k < SPH_NIN; k++)
            if (!r->in[k]) return SPH_EINVAL;
    Slot &s = *S->slots[slot];
    Worker &W = *s.w;
    {
        std::lock_guard<std::mutex> lk(W.mu);
        if (s.busy || W.quit) return SPH_EINVAL;
        s.busy = true;
        s.job = r;
        r->status = SPH_OK;
        r->error[0] = '\0';
        std::lock_guard<std::mutex> lk2(S->mu);
        S->running++;
    }
    W.cv.notify_all();
    return SPH_OK;
}

int32_t sph_server_wait(sph_server *S, sph_request **done, int32_t max, double timeout_s)
{
    if (!S || !done || max < 1) return -1;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return !S->done.empty(); };
    if (timeout_s < 0)
        S->cv.wait(lk, [&] { return ready() || S->running == 0; });
    else if (timeout_s > 0 && !ready())
        S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    int32_t k = 0;
    while (k < max && !S->done.empty()) {
        done[k++] = S->done.front();
        S->done.pop_front();
    }
    return k;
}

sph_status sph_server_release(sph_server *S, int32_t slot)
{
    if (!S || slot < 0 || slot >= (int32_t)S->slots.size()) return SPH_EINVAL;
    Slot &s = *S->slots[slot];
    Worker &W = *s.w;
    std::unique_lock<std::mutex> lk(W.mu);
    if (s.busy || W.quit) return SPH_EINVAL;
    s.busy = true;
    s.release = true;
    W.cv.notify_all();
    W.cv.wait(lk, [&] { return !s.busy; });
    return SPH_OK;
}

size_t sph_server_slot_bytes(sph_server *S, int32_t slot)
{
    if (!S || slot < 0 || slot >= (int32_t)S->slots.size()) return 0;
    return S->slots[slot]->bytes.load();
}

size_t sph_server_plan_bytes(const sph_params *p, int64_t n)
{
    if (!p || n < 0) return 0;
    return sph_plan_bytes(p, n) + (size_t)std::max<int64_t>(n, 1) * kArrayBytesPerParticle;
}

sph_status sph_server_destroy(sph_server *S)
{
    if (!S) return SPH_OK;
    for (auto &w : S->workers) {
        {
            std::lock_guard<std::mutex> lk(w->mu);
            w->quit = true;
        }
        w->cv.notify_all();
    }
    for (auto &w : S->workers)
        if (w->th.joinable()) w->th.join();
    delete S;
    return SPH_OK;
}

}  // extern "C"
