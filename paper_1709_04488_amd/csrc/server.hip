// Request executor for serving: one worker thread, one HIP stream and one
// context per slot.  Every HIP call a slot makes (its context, its device
// arrays, its pinned staging, its stream) happens on that slot's own thread;
// the caller's threads only hand requests over and collect them.
//
// A slot's worker takes a request, stages its nine input arrays into pinned
// memory, copies them to the device in one transfer, runs the request through
// the public entry points (sph_evaluate, or sph_upload_state + captured steps +
// sph_download_state), brings the wanted outputs back in one transfer, writes
// them into the caller's arrays and marks the slot idle before the request is
// published as done.
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

struct Slot {
    int idx = 0;
    std::thread th;
    // guarded by mu
    std::mutex mu;
    std::condition_variable cv;
    sph_request *job = nullptr;  // handed over, not yet taken by the worker
    bool busy = false;           // from submit until the request is published
    bool release = false;        // the caller asks the worker to free its buffers
    bool quit = false;
    // owned by the worker thread
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

}  // namespace

struct sph_server {
    int device = 0;
    std::vector<std::unique_ptr<Slot>> slots;
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

// One request on the slot's stream; returns the request's status.
sph_status run(Slot &s, sph_request *r)
{
    const int64_t n = r->n;
    if (n == 0) {               // nothing to compute, nothing allocated
        set_error(r, SPH_OK, "");
        return SPH_OK;
    }
    sph_status st = prepare(s, r);
    if (st != SPH_OK) return st;
    const size_t row = (size_t)n * sizeof(double);
    for (int k = 0; k < SPH_NIN; k++) std::memcpy(s.pin + (size_t)k * n, r->in[k], row);
    hipError_t e = hipMemcpyAsync(s.dev, s.pin, SPH_NIN * row, hipMemcpyHostToDevice, s.stream);
    if (e != hipSuccess) return hip_fail(r, e, "input copy");
    sph_particles d = device_view(s.dev, n);

    const bool eval = r->kind == SPH_REQUEST_EVALUATE;
    if (eval) {
        st = sph_evaluate(s.ctx, &d);
    } else {
        st = sph_upload_state(s.ctx, &d);
        // two steps per replay of a captured graph, then one eager step for an
        // odd count; block time-steps are not captured and step eagerly
        const bool graph = r->params.block_lmax == 0 && r->nsteps >= 2;
        int32_t left = r->nsteps;
        if (st == SPH_OK && graph) {
            st = sph_capture_steps(s.ctx, 0.0);
            for (; st == SPH_OK && left >= 2; left -= 2) st = sph_replay_steps(s.ctx);
        }
        for (; st == SPH_OK && left > 0; left--) st = sph_step(s.ctx, 0.0, nullptr);
        if (st == SPH_OK) st = sph_download_state(s.ctx, &d);
    }
    if (st == SPH_OK) st = sph_sync(s.ctx);
    if (st != SPH_OK) {
        set_error(r, st, sph_last_error(s.ctx));
        (void)sph_sync(s.ctx);   // clear the sticky status for the slot's next request
        return st;
    }

    // the wanted outputs: one copy of the rows from the first to the last wanted
    int lo = SPH_NF64, hi = -1;
    for (int k = 0; k < SPH_NF64; k++) {
        const bool written = eval ? k >= SPH_F_H : k != SPH_F_M;
        if (written && r->out[k]) { lo = std::min(lo, k); hi = std::max(hi, k); }
    }
    const bool counts = r->iout[0] || r->iout[1];
    if (hi >= 0) {
        e = hipMemcpyAsync(s.pin + (size_t)lo * n, d.x + (size_t)lo * n, (size_t)(hi - lo + 1) * row,
                           hipMemcpyDeviceToHost, s.stream);
        if (e != hipSuccess) return hip_fail(r, e, "output copy");
    }
    int32_t *ipin = reinterpret_cast<int32_t *>(s.pin + (size_t)SPH_NF64 * n);
    if (counts) {
        e = hipMemcpyAsync(ipin, d.nngb, (size_t)kI32 * n * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s.stream);
        if (e != hipSuccess) return hip_fail(r, e, "count copy");
    }
    // sph_state_info waits for the stream, so the copies above are complete
    st = sph_state_info(s.ctx, &r->info);
    if (st != SPH_OK) {
        set_error(r, st, sph_last_error(s.ctx));
        return st;
    }
    for (int k = lo; k <= hi; k++)
        if (r->out[k] && (eval ? k >= SPH_F_H : k != SPH_F_M))
            std::memcpy(r->out[k], s.pin + (size_t)k * n, row);
    for (int k = 0; k < kI32; k++)
        if (r->iout[k]) std::memcpy(r->iout[k], ipin + (size_t)k * n, n * sizeof(int32_t));
    const int64_t pairs = r->info.n_dens_pairs + r->info.n_force_pairs;
    r->interactions = eval ? pairs : pairs * std::max<int64_t>(r->nsteps, 1);
    set_error(r, SPH_OK, "");
    return SPH_OK;
}

void worker(sph_server *S, Slot *s)
{
    (void)hipSetDevice(S->device);
    s->stream_err = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (s->stream_err != hipSuccess) s->stream = nullptr;
    for (;;) {
        sph_request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->job || s->release || s->quit; });
            if (s->release) {
                free_buffers(*s);
                s->release = false;
                s->busy = false;
                lk.unlock();
                s->cv.notify_all();
                continue;
            }
            if (!s->job) break;   // quit with nothing handed over
            r = s->job;
            s->job = nullptr;
        }
        std::memset(&r->info, 0, sizeof(r->info));
        r->interactions = 0;
        r->slot = s->idx;
        (void)run(*s, r);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->busy = false;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->done.push_back(r);
            S->running--;
        }
        S->cv.notify_all();
    }
    free_buffers(*s);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
}

}  // namespace

extern "C" {

sph_status sph_server_create(sph_server **out, int32_t slots)
{
    if (!out) return SPH_EINVAL;
    *out = nullptr;
    if (slots < 1 || slots > kMaxSlots) return SPH_EINVAL;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return SPH_EDEVICE;
    auto *S = new sph_server;
    S->device = device;
    for (int k = 0; k < slots; k++) {
        S->slots.emplace_back(new Slot);
        S->slots.back()->idx = k;
    }
    for (auto &sl : S->slots) sl->th = std::thread(worker, S, sl.get());
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
    {
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.busy || s.quit) return SPH_EINVAL;
        s.busy = true;
        s.job = r;
        r->status = SPH_OK;
        r->error[0] = '\0';
        std::lock_guard<std::mutex> lk2(S->mu);
        S->running++;
    }
    s.cv.notify_all();
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
    std::unique_lock<std::mutex> lk(s.mu);
    if (s.busy || s.quit) return SPH_EINVAL;
    s.busy = true;
    s.release = true;
    s.cv.notify_all();
    s.cv.wait(lk, [&] { return !s.busy; });
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
    for (auto &sl : S->slots) {
        {
            std::lock_guard<std::mutex> lk(sl->mu);
            sl->quit = true;
        }
        sl->cv.notify_all();
    }
    for (auto &sl : S->slots)
        if (sl->th.joinable()) sl->th.join();
    delete S;
    return SPH_OK;
}

}  // extern "C"
