// Request server: continuous batching of replanning requests from many
// vehicles on one GPU.
//
//  * Vehicle table: each vehicle keeps only its nominal controls U (float64)
//    and its iteration state (Philox counter) on the device.  Its first
//    request starts from U = 0; every later request first shifts U by one
//    step (warm start of Alg. 1) and then runs one iteration.
//  * Admission by HBM budget: the per-request scratch (applied noise, costs,
//    tile partials) comes from one device allocation of the configured
//    budget, carved first-fit.  Requests are admitted in arrival order; the
//    first one that does not fit waits until memory frees up.
//  * Per-vehicle order: at most one request of a vehicle is in flight; later
//    ones wait behind it.
//  * Continuous batching: whenever one of the server's streams is idle, the
//    scheduler thread launches every admissible request as one batch (one
//    direct launch per kernel variant present: batch compositions rarely
//    repeat, so they are not captured as graphs).  Batches on different
//    streams overlap on the device; a completion thread per stream copies the
//    results back and stamps completion times.
//  * Latency = completion - arrival stamp given at submit (the replay driver
//    stamps the scheduled arrival, so queueing before submission counts).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mppi_host.hpp"

using namespace mppi_impl;

namespace {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int kSlotDoubles = 2 * kMaxT + 2;  // U, status, iteration counter

struct Req {
    uint64_t ticket = 0;
    int vid = 0;
    double x0[4];
    std::vector<double> wp, ci;
    uint64_t t_arr = 0, t_done = 0;
    int status = 0;
    bool done = false;
    bool keep = true;  // keep the result until polled
    std::vector<double> U;
    uint64_t n_iter = 0;
    size_t off = 0, bytes = 0;
    int lanes = 1;
};

struct Vehicle {
    mppi_t* h = nullptr;
    bool busy = false;
    uint64_t admitted = 0;
    std::deque<Req*> fifo;
};

struct StreamCtx {
    hipStream_t s = nullptr;
    BatchWs* ws = nullptr;
    // per-request results (U, status, iteration), written by the gather
    // kernel straight into this pinned coherent host buffer (gather_hdev:
    // its device address), so no copy back follows the batch
    double* gather_host = nullptr;
    double* gather_hdev = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Req*> batch;
    bool busy = false;
    bool launched = false;
    std::condition_variable cv;
    std::thread completer;
};

// First-fit allocator over the scratch arena (offsets only).
struct Pool {
    size_t cap = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t c)
    {
        cap = c;
        free_.clear();
        free_[0] = c;
    }
    bool alloc(size_t n, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

struct mppi_server {
    mppi_server_config cfg;
    std::mutex mu;
    std::condition_variable cv;       // scheduler wake-ups
    std::condition_variable done_cv;  // completions
    bool stop = false;
    mppi_status sticky = MPPI_OK;
    std::vector<Vehicle> veh;
    std::list<Req*> pending;  // arrival (submit) order
    std::unordered_map<uint64_t, Req*> live;
    uint64_t next_ticket = 1;
    size_t queued = 0;  // pending + in flight
    unsigned char* arena = nullptr;
    Pool pool;
    std::vector<std::unique_ptr<StreamCtx>> streams;
    std::thread scheduler;
    // statistics
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, launches = 0, batched = 0;
    size_t max_queue = 0;
    std::vector<double> lat_ms;
};

namespace {

size_t request_bytes(const mppi_config& c, int lanes)
{
    const size_t tiles = (size_t)(c.K + (kBlock / lanes) - 1) / (kBlock / lanes);
    size_t b = a256(sizeof(float) * c.K) + a256(sizeof(float2) * (size_t)c.T * c.K) +
               a256(sizeof(double) * partial_doubles(c.T, c.per_step_weights, tiles));
    if (c.per_step_weights)
        b += a256(sizeof(float) * (size_t)c.T * c.K) + a256(sizeof(double) * (size_t)c.T * c.K);
    return b;
}

void finish_request(mppi_server* srv, Req* r)
{
    r->done = true;
    if (!r->keep) {
        srv->live.erase(r->ticket);
        delete r;
    }
}

void completer_loop(mppi_server* srv, StreamCtx* sc)
{
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        sc->cv.wait(lk, [&] { return sc->launched || srv->stop; });
        if (!sc->launched) return;
        lk.unlock();
        const hipError_t e = hipEventSynchronize(sc->done);
        const uint64_t t = now_ns();
        lk.lock();
        for (size_t i = 0; i < sc->batch.size(); ++i) {
            Req* r = sc->batch[i];
            Vehicle& v = srv->veh[r->vid];
            const int T = v.h->cfg.T;
            const double* o = sc->gather_host + i * (size_t)kSlotDoubles;
            if (e == hipSuccess) {
                r->U.assign(o, o + 2 * T);
                r->status = (int)o[2 * T];
                r->n_iter = (uint64_t)o[2 * T + 1];
            } else {
                r->status = MPPI_E_DEVICE;
                srv->sticky = MPPI_E_DEVICE;
            }
            r->t_done = t;
            if (r->status != 0) ++srv->failed;
            ++srv->completed;
            srv->lat_ms.push_back((double)(r->t_done - r->t_arr) * 1e-6);
            srv->pool.release(r->off, r->bytes);
            v.busy = false;
            v.fifo.pop_front();
            --srv->queued;
            finish_request(srv, r);
        }
        sc->batch.clear();
        sc->launched = false;
        sc->busy = false;
        srv->cv.notify_all();
        srv->done_cv.notify_all();
    }
}

// Admissible requests in arrival order: vehicle idle, head of its FIFO, and
// scratch available (strict arrival order on memory).
std::vector<Req*> collect(mppi_server* srv)
{
    std::vector<Req*> b;
    const int cap = srv->cfg.plain ? 1 : srv->cfg.max_batch;
    for (auto it = srv->pending.begin(); it != srv->pending.end() && (int)b.size() < cap;) {
        Req* r = *it;
        Vehicle& v = srv->veh[r->vid];
        if (v.busy || v.fifo.front() != r) {
            ++it;
            continue;
        }
        if (!srv->pool.alloc(r->bytes, &r->off)) break;
        v.busy = true;
        b.push_back(r);
        it = srv->pending.erase(it);
    }
    return b;
}

void scheduler_loop(mppi_server* srv)
{
    std::unique_lock<std::mutex> lk(srv->mu);
    while (!srv->stop) {
        StreamCtx* sc = nullptr;
        for (auto& s : srv->streams)
            if (!s->busy) {
                sc = s.get();
                break;
            }
        std::vector<Req*> b;
        if (sc && srv->sticky == MPPI_OK) b = collect(srv);
        if (b.empty()) {
            srv->cv.wait_for(lk, std::chrono::microseconds(500));
            continue;
        }
        sc->busy = true;
        // per-request launch inputs (vehicle state is not touched by others
        // while busy)
        const int n = (int)b.size();
        std::vector<mppi_t*> hs(n);
        std::vector<double> x0s(4 * n);
        std::vector<mppi_scene> scs(n);
        std::vector<InstExtra> ex(n);
        for (int i = 0; i < n; ++i) {
            Req* r = b[i];
            Vehicle& v = srv->veh[r->vid];
            hs[i] = v.h;
            memcpy(&x0s[4 * i], r->x0, sizeof r->x0);
            scs[i].waypoints = r->wp.data();
            scs[i].n_waypoints = (int)(r->wp.size() / 4);
            scs[i].circles = r->ci.empty() ? nullptr : r->ci.data();
            scs[i].n_circles = (int)(r->ci.size() / 5);
            const mppi_config& c = v.h->cfg;
            unsigned char* base = srv->arena + r->off;
            const size_t tiles = (size_t)(c.K + (kBlock / r->lanes) - 1) / (kBlock / r->lanes);
            ex[i].S = reinterpret_cast<float*>(base);
            base += a256(sizeof(float) * c.K);
            ex[i].eps = reinterpret_cast<float2*>(base);
            base += a256(sizeof(float2) * (size_t)c.T * c.K);
            ex[i].partials = reinterpret_cast<double*>(base);
            base += a256(sizeof(double) * partial_doubles(c.T, c.per_step_weights, tiles));
            ex[i].q = nullptr;
            ex[i].Stk = nullptr;
            if (c.per_step_weights) {
                ex[i].q = reinterpret_cast<float*>(base);
                base += a256(sizeof(float) * (size_t)c.T * c.K);
                ex[i].Stk = reinterpret_cast<double*>(base);
            }
            ex[i].shift = v.admitted > 0 ? 1 : 0;
            ex[i].out_slot = i;
            ++v.admitted;
        }
        ++srv->launches;
        srv->batched += n;
        lk.unlock();
        // every batch has its own composition: direct launches, no graph
        mppi_status st = batch_enqueue(sc->ws, sc->s, hs.data(), x0s.data(), scs.data(), ex.data(),
                                       n, nullptr, sc->gather_hdev, kSlotDoubles, false);
        hipError_t e = hipSuccess;
        if (st == MPPI_OK) e = hipEventRecord(sc->done, sc->s);
        lk.lock();
        if (st != MPPI_OK || e != hipSuccess) {
            srv->sticky = MPPI_E_DEVICE;
            for (Req* r : b) {
                Vehicle& v = srv->veh[r->vid];
                r->status = MPPI_E_DEVICE;
                r->t_done = now_ns();
                srv->pool.release(r->off, r->bytes);
                v.busy = false;
                v.fifo.pop_front();
                --srv->queued;
                ++srv->failed;
                ++srv->completed;
                finish_request(srv, r);
            }
            sc->busy = false;
            srv->done_cv.notify_all();
            continue;
        }
        // the scenes were staged by the launch; the requests keep only what
        // poll returns
        for (Req* r : b) {
            std::vector<double>().swap(r->wp);
            std::vector<double>().swap(r->ci);
        }
        sc->batch = std::move(b);
        sc->launched = true;
        sc->cv.notify_one();
    }
}

void server_release(mppi_server* srv)
{
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    for (auto& s : srv->streams) s->cv.notify_all();
    if (srv->scheduler.joinable()) srv->scheduler.join();
    for (auto& s : srv->streams) {
        // a launched batch is still completed by its thread
        if (s->completer.joinable()) {
            s->cv.notify_all();
            s->completer.join();
        }
        if (s->s) (void)hipStreamSynchronize(s->s);
        ws_destroy(s->ws);
        if (s->gather_host) (void)hipHostFree(s->gather_host);
        if (s->done) (void)hipEventDestroy(s->done);
        if (s->s) (void)hipStreamDestroy(s->s);
    }
    for (Vehicle& v : srv->veh) {
        handle_release(v.h);
        delete v.h;
    }
    for (auto& kv : srv->live) delete kv.second;
    (void)hipFree(srv->arena);
}

mppi_status server_usable(mppi_server* srv)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    if (srv->sticky != MPPI_OK) return fail(srv->sticky, "server stopped after a device failure");
    return MPPI_OK;
}

}  // namespace

extern "C" {

uint64_t mppi_server_now_ns(void) { return now_ns(); }

mppi_status mppi_server_create(const mppi_server_config* cfg, mppi_server_t** out)
{
    if (!cfg || !out) return fail(MPPI_E_INVALID, "config and out must not be NULL");
    *out = nullptr;
    if (cfg->hbm_budget_bytes < 4096 || cfg->n_streams < 1 || cfg->n_streams > 8 ||
        cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->queue_cap < 1 ||
        !(cfg->deadline_ms >= 0.0) || !isfinite(cfg->deadline_ms))
        return fail(MPPI_E_INVALID,
                    "budget >= 4096, 1 <= n_streams <= 8, 1 <= max_batch <= 4096, queue_cap >= 1, "
                    "finite deadline_ms >= 0");
    mppi_server* srv = new (std::nothrow) mppi_server();
    if (!srv) return fail(MPPI_E_NOMEM, "host allocation failed");
    srv->cfg = *cfg;
    if (srv->cfg.plain) {
        srv->cfg.n_streams = 1;
        srv->cfg.max_batch = 1;
    }
    hipError_t e = hipMalloc((void**)&srv->arena, cfg->hbm_budget_bytes);
    if (e == hipSuccess) srv->pool.init(cfg->hbm_budget_bytes);
    for (int i = 0; i < srv->cfg.n_streams && e == hipSuccess; ++i) {
        auto sc = std::make_unique<StreamCtx>();
        e = hipStreamCreateWithFlags(&sc->s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sc->done, hipEventDisableTiming);
        const size_t gb = sizeof(double) * kSlotDoubles * (size_t)srv->cfg.max_batch;
        if (e == hipSuccess) e = hipHostMalloc((void**)&sc->gather_host, gb, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&sc->gather_hdev, sc->gather_host, 0);
        if (e == hipSuccess && ws_create(&sc->ws) != MPPI_OK) e = hipErrorOutOfMemory;
        srv->streams.push_back(std::move(sc));
    }
    if (e != hipSuccess) {
        server_release(srv);
        delete srv;
        return fail(MPPI_E_NOMEM, "server resources: %s", hipGetErrorString(e));
    }
    srv->lat_ms.reserve(1 << 20);
    for (auto& s : srv->streams) s->completer = std::thread(completer_loop, srv, s.get());
    srv->scheduler = std::thread(scheduler_loop, srv);
    *out = srv;
    return MPPI_OK;
}

mppi_status mppi_server_destroy(mppi_server_t* srv)
{
    if (!srv) return MPPI_OK;
    server_release(srv);
    delete srv;
    return MPPI_OK;
}

mppi_status mppi_server_add_vehicle(mppi_server_t* srv, const mppi_config* cfg, int32_t* vid)
{
    mppi_status s = server_usable(srv);
    if (s != MPPI_OK) return s;
    if (!vid) return fail(MPPI_E_INVALID, "vid is NULL");
    if (cfg && cfg->model != 0)
        return fail(MPPI_E_INVALID, "served vehicles use the 4-state model (model = 0)");
    mppi_t* h = nullptr;
    if ((s = handle_create(cfg, srv->streams[0]->s, false, &h)) != MPPI_OK) return s;
    // the worst-case request of this vehicle must fit the budget
    size_t worst = 0;
    for (int g : {1, 2, 4, 8, 16}) worst = std::max(worst, request_bytes(*cfg, g));
    if (worst > srv->cfg.hbm_budget_bytes) {
        handle_release(h);
        delete h;
        return fail(MPPI_E_NOMEM, "one request needs %zu bytes, budget is %llu", worst,
                    (unsigned long long)srv->cfg.hbm_budget_bytes);
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    Vehicle v;
    v.h = h;
    srv->veh.push_back(std::move(v));
    *vid = (int32_t)srv->veh.size() - 1;
    return MPPI_OK;
}

mppi_status mppi_server_submit(mppi_server_t* srv, int32_t vid, const double x0[4],
                               const mppi_scene* scene, uint64_t t_arrival_ns, uint64_t* ticket)
{
    mppi_status s = server_usable(srv);
    if (s != MPPI_OK) return s;
    Req* r = new (std::nothrow) Req();
    if (!r) return fail(MPPI_E_NOMEM, "host allocation failed");
    mppi_config c;
    int lanes_req = 0;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (vid < 0 || vid >= (int)srv->veh.size()) {
            delete r;
            return fail(MPPI_E_INVALID, "unknown vehicle %d", vid);
        }
        c = srv->veh[vid].h->cfg;
        lanes_req = srv->veh[vid].h->lanes_req;
    }
    // the scene is checked outside the server lock
    if ((s = validate_scene(c, x0, scene)) != MPPI_OK) {
        delete r;
        return s;
    }
    r->lanes = lanes_req ? lanes_req : auto_lanes(c, scene->n_circles);
    r->bytes = request_bytes(c, r->lanes);
    r->vid = vid;
    memcpy(r->x0, x0, sizeof r->x0);
    r->wp.assign(scene->waypoints, scene->waypoints + 4 * scene->n_waypoints);
    if (scene->n_circles > 0) r->ci.assign(scene->circles, scene->circles + 5 * scene->n_circles);
    r->t_arr = t_arrival_ns ? t_arrival_ns : now_ns();
    r->keep = ticket != nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->queued >= (size_t)srv->cfg.queue_cap) {
            ++srv->rejected;
            delete r;
            return fail(MPPI_E_BUSY, "queue full (%d requests)", srv->cfg.queue_cap);
        }
        r->ticket = srv->next_ticket++;
        if (ticket) *ticket = r->ticket;
        srv->live[r->ticket] = r;
        srv->veh[vid].fifo.push_back(r);
        srv->pending.push_back(r);
        ++srv->queued;
        ++srv->submitted;
        srv->max_queue = std::max(srv->max_queue, srv->queued);
    }
    srv->cv.notify_one();
    return MPPI_OK;
}

mppi_status mppi_server_poll(mppi_server_t* srv, uint64_t ticket, double* controls, size_t n,
                             uint64_t* t_done_ns)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->live.find(ticket);
    if (it == srv->live.end()) return fail(MPPI_E_INVALID, "unknown ticket");
    Req* r = it->second;
    if (!r->done) return MPPI_E_NOT_READY;
    if (controls) {
        if (n < r->U.size()) return fail(MPPI_E_INVALID, "controls buffer needs %zu doubles",
                                         r->U.size());
        memcpy(controls, r->U.data(), sizeof(double) * r->U.size());
    }
    if (t_done_ns) *t_done_ns = r->t_done;
    const int status = r->status;
    srv->live.erase(it);
    delete r;
    if (status == -4) return fail(MPPI_E_NONFINITE, "every sample cost was non-finite");
    if (status != 0) return fail(MPPI_E_DEVICE, "request failed on the device");
    return MPPI_OK;
}

mppi_status mppi_server_wait_idle(mppi_server_t* srv)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->done_cv.wait(lk, [&] { return srv->queued == 0 || srv->sticky != MPPI_OK; });
    return srv->sticky;
}

mppi_status mppi_server_get_stats(mppi_server_t* srv, mppi_server_stats* out)
{
    if (!srv || !out) return fail(MPPI_E_INVALID, "server and out must not be NULL");
    std::vector<double> lat;
    std::lock_guard<std::mutex> lk(srv->mu);
    memset(out, 0, sizeof *out);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->failed = srv->failed;
    out->launches = srv->launches;
    out->mean_batch = srv->launches ? (double)srv->batched / srv->launches : 0.0;
    out->hbm_peak_bytes = srv->pool.peak;
    out->max_queue = (int32_t)srv->max_queue;
    lat = srv->lat_ms;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(lat.size() - 1, floor(p * (lat.size() - 1) + 0.5));
            return lat[i];
        };
        double sum = 0.0;
        for (double v : lat) sum += v;
        out->mean_ms = sum / lat.size();
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->p999_ms = pct(0.999);
        out->max_ms = lat.back();
        if (srv->cfg.deadline_ms > 0.0)
            out->deadline_misses = (uint64_t)(lat.end() - std::upper_bound(lat.begin(), lat.end(),
                                                                            srv->cfg.deadline_ms));
    }
    return MPPI_OK;
}

mppi_status mppi_server_reset_stats(mppi_server_t* srv)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted = srv->completed = srv->rejected = srv->failed = 0;
    srv->launches = srv->batched = 0;
    srv->max_queue = srv->queued;
    srv->pool.peak = srv->pool.used;
    srv->lat_ms.clear();
    return MPPI_OK;
}

mppi_status mppi_server_get_vehicle_state(mppi_server_t* srv, int32_t vid, double* U, size_t n,
                                          uint64_t* n_iter, uint64_t* requests)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (vid < 0 || vid >= (int)srv->veh.size()) return fail(MPPI_E_INVALID, "unknown vehicle");
    Vehicle& v = srv->veh[vid];
    if (v.busy || !v.fifo.empty()) return fail(MPPI_E_BUSY, "vehicle has requests in flight");
    mppi_t* h = v.h;
    if (!U || n < (size_t)2 * h->cfg.T) return fail(MPPI_E_INVALID, "U needs 2T doubles");
    DevState st;
    HIP_TRY(hipMemcpy(U, h->U, sizeof(double) * 2 * h->cfg.T, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&st, h->st, sizeof st, hipMemcpyDeviceToHost));
    if (n_iter) *n_iter = st.n_iter;
    if (requests) *requests = v.admitted;
    return MPPI_OK;
}

mppi_status mppi_server_set_vehicle_state(mppi_server_t* srv, int32_t vid, const double* U,
                                          size_t n, uint64_t n_iter, uint64_t requests)
{
    if (!srv) return fail(MPPI_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (vid < 0 || vid >= (int)srv->veh.size()) return fail(MPPI_E_INVALID, "unknown vehicle");
    Vehicle& v = srv->veh[vid];
    if (v.busy || !v.fifo.empty()) return fail(MPPI_E_BUSY, "vehicle has requests in flight");
    mppi_t* h = v.h;
    if (!U || n < (size_t)2 * h->cfg.T) return fail(MPPI_E_INVALID, "U needs 2T doubles");
    for (int i = 0; i < 2 * h->cfg.T; ++i)
        if (!isfinite(U[i])) return fail(MPPI_E_INVALID, "controls must be finite");
    DevState st;
    memset(&st, 0, sizeof st);
    st.n_iter = n_iter;
    HIP_TRY(hipMemcpy(h->U, U, sizeof(double) * 2 * h->cfg.T, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->st, &st, sizeof st, hipMemcpyHostToDevice));
    v.admitted = requests;
    return MPPI_OK;
}

mppi_status mppi_server_replay(mppi_server_t* srv, const mppi_replay_plan* plan, double* latency_ms)
{
    mppi_status s = server_usable(srv);
    if (s != MPPI_OK) return s;
    if (!plan || plan->n_requests < 0 || !plan->vid || !plan->x0 || !plan->scene ||
        !plan->scenes || !plan->arrival_ns)
        return fail(MPPI_E_INVALID, "incomplete replay plan");
    const int n = plan->n_requests;
    for (int i = 0; i < n; ++i)
        if (plan->scene[i] < 0 || plan->scene[i] >= plan->n_scenes)
            return fail(MPPI_E_INVALID, "scene index out of range at request %d", i);
    std::vector<uint64_t> tickets(n, 0), t_arr(n, 0);
    {
        // every request stays in the ticket table until it is polled below:
        // size the table now, so that no rehash runs under the server lock
        // while requests are in flight
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->live.reserve(srv->live.size() + (size_t)n);
        srv->lat_ms.reserve(srv->lat_ms.size() + (size_t)n);
    }
    const uint64_t t0 = now_ns() + 2000000;  // start 2 ms from now
    for (int i = 0; i < n; ++i) {
        const uint64_t target = t0 + plan->arrival_ns[i];
        for (;;) {
            const uint64_t t = now_ns();
            if (t >= target) break;
            if (target - t > 200000)
                std::this_thread::sleep_for(std::chrono::nanoseconds(target - t - 100000));
            else
                std::this_thread::yield();
        }
        t_arr[i] = target;
        s = mppi_server_submit(srv, plan->vid[i], plan->x0 + 4 * i, &plan->scenes[plan->scene[i]],
                               target, &tickets[i]);
        if (s == MPPI_E_BUSY) {
            tickets[i] = 0;
            continue;
        }
        if (s != MPPI_OK) return s;
    }
    for (int i = 0; i < n; ++i) {
        if (!tickets[i]) {
            if (latency_ms) latency_ms[i] = NAN;
            continue;
        }
        uint64_t t_done = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(srv->mu);
                auto it = srv->live.find(tickets[i]);
                if (it == srv->live.end()) return fail(MPPI_E_DEVICE, "lost request");
                if (!it->second->done)
                    srv->done_cv.wait_for(lk, std::chrono::milliseconds(50));
                if (srv->sticky != MPPI_OK) return srv->sticky;
            }
            s = mppi_server_poll(srv, tickets[i], nullptr, 0, &t_done);
            if (s != MPPI_E_NOT_READY) break;
        }
        if (latency_ms) latency_ms[i] = (s == MPPI_OK) ? (double)(t_done - t_arr[i]) * 1e-6 : NAN;
    }
    return MPPI_OK;
}

}  // extern "C"
