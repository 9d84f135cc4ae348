// Host runtime behind the C ABI of include/mppi.h: handle life cycle,
// validation, ego-frame staging of the scene, single and batched launches
// (batches replayed as HIP graphs), result export, checkpointing, the
// launch-shape tuning table and profiling.
#include <hip/hip_runtime.h>
#include <dlfcn.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mppi_host.hpp"

using namespace mppi_impl;

namespace mppi_impl {

thread_local std::string g_last_error;

mppi_status fail(mppi_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

size_t pow2_at_least(size_t v, size_t lo)
{
    size_t p = lo;
    while (p < v) p <<= 1;
    return p;
}

static size_t scene_bytes(int n_wp, int n_c) { return scene_layout(n_wp, n_c).bytes; }

// ---- validation ---------------------------------------------------------------

mppi_status validate_scene(const mppi_config& c, const double x0[4], const mppi_scene* sc)
{
    if (!x0 || !sc) return fail(MPPI_E_INVALID, "x0 and scene must not be NULL");
    for (int i = 0; i < 4; ++i)
        if (!isfinite(x0[i])) return fail(MPPI_E_INVALID, "x0[%d] is not finite", i);
    const int n_wp = sc->n_waypoints, n_c = sc->n_circles;
    if (n_wp < 1 || n_wp > c.max_waypoints || !sc->waypoints)
        return fail(MPPI_E_INVALID, "n_waypoints=%d outside [1, %d] or waypoints NULL", n_wp,
                    c.max_waypoints);
    if (n_c < 0 || n_c > c.max_circles || (n_c > 0 && !sc->circles))
        return fail(MPPI_E_INVALID, "n_circles=%d outside [0, %d] or circles NULL", n_c,
                    c.max_circles);
    for (int i = 0; i < 4 * n_wp; ++i)
        if (!isfinite(sc->waypoints[i])) return fail(MPPI_E_INVALID, "waypoint value not finite");
    for (int i = 0; i < 5 * n_c; ++i)
        if (!isfinite(sc->circles[i])) return fail(MPPI_E_INVALID, "circle value not finite");
    return MPPI_OK;
}

mppi_status validate_config(const mppi_config* c)
{
    if (!c) return fail(MPPI_E_INVALID, "config is NULL");
    if (c->K < 1 || c->K > kMaxK) return fail(MPPI_E_INVALID, "K=%d outside [1, %d]", c->K, kMaxK);
    if (c->T < 1 || c->T > kMaxT) return fail(MPPI_E_INVALID, "T=%d outside [1, %d]", c->T, kMaxT);
    if (!(c->dt > 0) || !isfinite(c->dt)) return fail(MPPI_E_INVALID, "dt must be finite and > 0");
    if (!(c->wheelbase > 0) || !isfinite(c->wheelbase))
        return fail(MPPI_E_INVALID, "wheelbase must be finite and > 0");
    if (!(c->lambda > 0) || !isfinite(c->lambda))
        return fail(MPPI_E_INVALID, "lambda must be finite and > 0");
    if (!(c->gamma > 0) || !isfinite(c->gamma)) return fail(MPPI_E_INVALID, "gamma must be > 0");
    for (int i = 0; i < 2; ++i) {
        if (!(c->sigma[i] >= 0) || !isfinite(c->sigma[i]))
            return fail(MPPI_E_INVALID, "sigma[%d] must be finite and >= 0", i);
        if (isnan(c->u_min[i]) || isnan(c->u_max[i]) || !(c->u_min[i] <= c->u_max[i]))
            return fail(MPPI_E_INVALID, "u_min[%d] <= u_max[%d] required", i, i);
        if (c->u_min[i] == INFINITY || c->u_max[i] == -INFINITY)
            return fail(MPPI_E_INVALID, "bounds %d exclude every control", i);
    }
    if (isnan(c->v_max)) return fail(MPPI_E_INVALID, "v_max is NaN");
    const double ws[6] = {c->w_track, c->w_speed, c->w_effort, c->w_coll, c->d_safe_c, c->d_safe_0};
    for (double w : ws)
        if (!isfinite(w)) return fail(MPPI_E_INVALID, "cost weights must be finite");
    if (c->n_ego < 0 || c->n_ego > kMaxEgo)
        return fail(MPPI_E_INVALID, "n_ego=%d outside [0, %d]", c->n_ego, kMaxEgo);
    if (!isfinite(c->ego_r)) return fail(MPPI_E_INVALID, "ego_r must be finite");
    for (int e = 0; e < c->n_ego; ++e)
        if (!isfinite(c->ego_off[e])) return fail(MPPI_E_INVALID, "ego_off must be finite");
    if (c->max_waypoints < 1 || c->max_waypoints > kMaxWaypoints)
        return fail(MPPI_E_INVALID, "max_waypoints=%d outside [1, %d]", c->max_waypoints,
                    kMaxWaypoints);
    if (c->max_circles < 0 || c->max_circles > kMaxCircles)
        return fail(MPPI_E_INVALID, "max_circles=%d outside [0, %d]", c->max_circles,
                    kMaxCircles);
    if (c->smoothing != 0 && c->smoothing != 1)
        return fail(MPPI_E_INVALID, "smoothing must be 0 or 1");
    if (!isfinite(c->w_target) || !isfinite(c->w_yaw))
        return fail(MPPI_E_INVALID, "w_target and w_yaw must be finite");
    if (c->collision_only != 0 && c->collision_only != 1)
        return fail(MPPI_E_INVALID, "collision_only must be 0 or 1");
    if (c->model != 0 && c->model != 1) return fail(MPPI_E_INVALID, "model must be 0 or 1");
    if (c->per_step_weights != 0 && c->per_step_weights != 1)
        return fail(MPPI_E_INVALID, "per_step_weights must be 0 or 1");
    return MPPI_OK;
}

mppi_status usable(mppi_t* h)
{
    if (!h) return fail(MPPI_E_INVALID, "handle is NULL");
    if (h->sticky != MPPI_OK)
        return fail(h->sticky, "handle is unusable after an earlier device failure");
    return MPPI_OK;
}

// ---- scene staging ------------------------------------------------------------

SceneLayout scene_layout(int n_wp, int n_c)
{
    SceneLayout L;
    L.o_pv = 0;
    L.o_xy = L.o_pv + align_up((size_t)n_c * 16, 16);
    // waypoints padded to whole chunks (points at infinity)
    L.o_vr = L.o_xy + align_up((size_t)(n_wp + kChunk - 1) / kChunk * kChunk * 8, 16);
    L.o_yw = L.o_vr + align_up((size_t)n_wp * 4, 16);
    L.o_rr = L.o_yw + align_up((size_t)n_wp * 4, 16);
    // bounding box of every chunk, then the scene's flags
    L.o_box = L.o_rr + align_up((size_t)n_c * 4, 16);
    L.o_flags = L.o_box + (size_t)(n_wp + kChunk - 1) / kChunk * 16;
    L.bytes = L.o_flags + 16;
    return L;
}

// Ego-frame float32 copy of the scene (float64 subtraction of the origin).
void write_scene(unsigned char* dst, const SceneLayout& L, const mppi_config& c,
                 const double origin[2], const mppi_scene* sc)
{
    float4* pv = reinterpret_cast<float4*>(dst + L.o_pv);
    float2* xy = reinterpret_cast<float2*>(dst + L.o_xy);
    float* vr = reinterpret_cast<float*>(dst + L.o_vr);
    float* yw = reinterpret_cast<float*>(dst + L.o_yw);
    float* rr = reinterpret_cast<float*>(dst + L.o_rr);
    for (int i = 0; i < sc->n_waypoints; ++i) {
        const double* w = sc->waypoints + 4 * i;
        xy[i] = make_float2((float)(w[0] - origin[0]), (float)(w[1] - origin[1]));
        vr[i] = (float)w[3];
        yw[i] = (float)w[2];
    }
    for (int i = sc->n_waypoints; i % kChunk; ++i) xy[i] = make_float2(INFINITY, INFINITY);
    // (x_lo, x_hi, y_lo, y_hi) of each chunk's float32 positions, for the
    // culling; flag 0: one reference speed for every waypoint
    float4* box = reinterpret_cast<float4*>(dst + L.o_box);
    for (int c = 0; c * kChunk < sc->n_waypoints; ++c) {
        float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        for (int j = c * kChunk; j < std::min((c + 1) * kChunk, (int)sc->n_waypoints); ++j) {
            b.x = fminf(b.x, xy[j].x);
            b.y = fmaxf(b.y, xy[j].x);
            b.z = fminf(b.z, xy[j].y);
            b.w = fmaxf(b.w, xy[j].y);
        }
        box[c] = b;
    }
    int* flags = reinterpret_cast<int*>(dst + L.o_flags);
    flags[0] = 1;
    for (int i = 1; i < sc->n_waypoints; ++i)
        if (vr[i] != vr[0]) flags[0] = 0;
    flags[1] = flags[2] = flags[3] = 0;
    for (int i = 0; i < sc->n_circles; ++i) {
        const double* o = sc->circles + 5 * i;
        pv[i] = make_float4((float)(o[0] - origin[0]), (float)(o[1] - origin[1]), (float)o[3],
                            (float)o[4]);
        rr[i] = (float)(o[2] + c.ego_r);
    }
}

// ---- launch-shape tuning table ------------------------------------------------
// Lines "k_log2 t_bucket c_bucket lanes" written by the autotuner
// (paper_2308_01654_amd/autotune.py) into tuning.txt next to the library, or
// the file named by MPPI_TUNING_FILE.  A shape's lanes per sample depends only
// on its own (K, T, circle count).

struct TuneEntry {
    int k, t, c, lanes;
    int stage;  // 1: the tiles may keep their perturbations in LDS; 0: read back from L2
    int occ;    // 1: the high-occupancy compilation of the iteration kernel
};
static std::vector<TuneEntry> g_tune;
static std::once_flag g_tune_once;

static int k_bucket(int K)
{
    int b = 0;
    while ((1 << b) < K && b < 30) ++b;
    return b;
}
static int t_bucket(int T)
{
    return T <= 16 ? 0 : T <= 32 ? 1 : T <= 64 ? 2 : T <= 128 ? 3 : T <= 256 ? 4 : 5;
}
static int c_bucket(int n) { return n == 0 ? 0 : n <= 16 ? 1 : n <= 64 ? 2 : n <= 256 ? 3 : 4; }

static void load_tuning()
{
    std::string path;
    if (const char* e = getenv("MPPI_TUNING_FILE")) {
        path = e;
    } else {
        Dl_info info;
        if (dladdr((void*)&load_tuning, &info) && info.dli_fname) {
            path = info.dli_fname;
            const size_t slash = path.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) +
                   "/tuning.txt";
        }
    }
    FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        TuneEntry t;
        t.stage = 1;  // the optional fifth and sixth columns
        t.occ = 0;
        const int n = sscanf(line, "%d %d %d %d %d %d", &t.k, &t.t, &t.c, &t.lanes, &t.stage,
                             &t.occ);
        if (n >= 4 && (t.stage == 0 || t.stage == 1) && t.occ >= 0 && t.occ < kOccModes &&
            (t.lanes == 1 || t.lanes == 2 || t.lanes == 4 || t.lanes == 8 || t.lanes == 16))
            g_tune.push_back(t);
    }
    fclose(f);
}

static int heuristic_lanes(const mppi_config& c)
{
    // Enough lanes to give every SIMD of the 256 CUs two waves.
    const long target = 2L * 256 * 4 * 64;
    int g = 1;
    while (g < 16 && (long)g * c.K < target) g <<= 1;
    return g;
}

int auto_lanes(const mppi_config& c, int n_c)
{
    std::call_once(g_tune_once, load_tuning);
    const int kb = k_bucket(c.K), tb = t_bucket(c.T), cb = c_bucket(n_c);
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : g_tune)
        if (e.t == tb && e.c == cb && (!best || abs(e.k - kb) < abs(best->k - kb))) best = &e;
    int g = best ? best->lanes : heuristic_lanes(c);
    while (g > 1 && g > c.T) g >>= 1;
    return g;
}

static const TuneEntry* tune_entry(const mppi_config& c, int n_c)
{
    std::call_once(g_tune_once, load_tuning);
    const int kb = k_bucket(c.K), tb = t_bucket(c.T), cb = c_bucket(n_c);
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : g_tune)
        if (e.t == tb && e.c == cb && (!best || abs(e.k - kb) < abs(best->k - kb))) best = &e;
    return best;
}

// The tuning table's staging choice for the bucket auto_lanes uses (1 when
// the table has no such column or no bucket).
int auto_stage(const mppi_config& c, int n_c)
{
    const TuneEntry* e = tune_entry(c, n_c);
    return e ? e->stage : 1;
}

int auto_occ(const mppi_config& c, int n_c)
{
    const TuneEntry* e = tune_entry(c, n_c);
    return e ? e->occ : 0;
}

int occ_choice(const mppi_t* h, int n_c, int lanes)
{
    // the other compilations exist for 8 and 16 lanes per sample
    if (lanes < 8) return kOccDefault;
    return h->occ_req >= 0 ? h->occ_req : auto_occ(h->cfg, n_c);
}

// ---- profiling --------------------------------------------------------------------

// Events come from the handle's pool (created on first use) so that
// profiling adds little host time between launches.
static hipError_t pool_event(mppi_t* h, hipEvent_t* e)
{
    if (!h->event_pool.empty()) {
        *e = h->event_pool.back();
        h->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

mppi_status record_launch(mppi_t* h, int kind, hipEvent_t* a)
{
    (void)kind;
    if (!h || !h->prof) return MPPI_OK;
    HIP_TRY(pool_event(h, a));
    HIP_TRY(hipEventRecord(*a, h->stream));
    return MPPI_OK;
}

mppi_status record_end(mppi_t* h, int kind, hipEvent_t a)
{
    if (!h || !h->prof) return MPPI_OK;
    hipEvent_t b;
    HIP_TRY(pool_event(h, &b));
    HIP_TRY(hipEventRecord(b, h->stream));
    h->events.push_back(ProfEvent{a, b, kind});
    return MPPI_OK;
}

static mppi_status drain_profile(mppi_t* h)
{
    if (h->events.empty()) return MPPI_OK;
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (const ProfEvent& e : h->events) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
        h->prof_ms[e.kind] += ms;
        h->prof_n[e.kind] += 1;
        h->event_pool.push_back(e.a);
        h->event_pool.push_back(e.b);
    }
    h->events.clear();
    return MPPI_OK;
}

template <typename F>
static mppi_status launch_aux(mppi_t* h, F&& f)
{
    hipEvent_t a = nullptr;
    mppi_status s = record_launch(h, 1, &a);
    if (s != MPPI_OK) return s;
    HIP_TRY(f());
    return record_end(h, 1, a);
}

// The pinned, coherent host buffers the device writes results into (U and
// the state; the optimal trajectory), made on first use so that handles
// that never read them back -- a server's vehicles -- hold no pinned pages.
static mppi_status host_buffers(mppi_t* h)
{
    if (h->ctl_host) return MPPI_OK;
    const size_t T = (size_t)h->cfg.T;
    hipError_t e;
    if ((e = hipHostMalloc((void**)&h->traj, sizeof(double) * (5 * (T + 1) + 2 * T),
                           hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&h->traj_dev, h->traj, 0)) != hipSuccess ||
        (e = hipHostMalloc((void**)&h->ctl_host, sizeof(double) * 2 * T + sizeof(DevState),
                           hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&h->ctl_dev, h->ctl_host, 0)) != hipSuccess) {
        if (h->traj) (void)hipHostFree(h->traj);
        if (h->ctl_host) (void)hipHostFree(h->ctl_host);
        h->traj = h->traj_dev = h->ctl_host = h->ctl_dev = nullptr;
        return fail(MPPI_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    return MPPI_OK;
}

// The device state after the handle's stream has drained: written by one
// small kernel into the pinned host buffer, then one synchronisation.
static mppi_status read_state(mppi_t* h, DevState* out)
{
    const mppi_status s = host_buffers(h);
    if (s != MPPI_OK) return s;
    const int nu = 2 * h->cfg.T;
    DevState* dst = reinterpret_cast<DevState*>(h->ctl_dev + nu);
    HIP_TRY(launch_export_controls(h->U, 0, h->st, h->ctl_dev, dst, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    *out = *reinterpret_cast<const DevState*>(h->ctl_host + nu);
    return MPPI_OK;
}

static mppi_status sync_status(mppi_t* h)
{
    if (!h->stepped) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        return MPPI_OK;
    }
    DevState st;
    const mppi_status s = read_state(h, &st);
    if (s != MPPI_OK) return s;
    if (st.status != 0)
        return fail(MPPI_E_NONFINITE, "every sample cost of the last step was non-finite");
    return MPPI_OK;
}

// ---- handles ----------------------------------------------------------------------

void handle_release(mppi_t* h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (const ProfEvent& e : h->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    (void)hipFree(h->U);
    (void)hipFree(h->S);
    (void)hipFree(h->eps);
    (void)hipFree(h->partials);
    (void)hipFree(h->q);
    (void)hipFree(h->Stk);
    (void)hipFree(h->wbuf);
    if (h->traj) (void)hipHostFree(h->traj);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    (void)hipFree(h->st);
    (void)hipFree(h->scene);
    if (h->batch) {
        ws_destroy(h->batch);
        h->batch = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        if (h->staging[i]) (void)hipHostFree(h->staging[i]);
        if (h->staged[i]) (void)hipEventDestroy(h->staged[i]);
    }
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

mppi_status handle_create(const mppi_config* cfg, void* hip_stream, bool with_scratch,
                          mppi_t** out)
{
    if (!out) return fail(MPPI_E_INVALID, "out is NULL");
    *out = nullptr;
    mppi_status s = validate_config(cfg);
    if (s != MPPI_OK) return s;
    mppi_t* h = new (std::nothrow) mppi();
    if (!h) return fail(MPPI_E_NOMEM, "host allocation failed");
    h->cfg = *cfg;
    const int K = cfg->K, T = cfg->T;
    h->max_tiles = (K + (kBlock / 16) - 1) / (kBlock / 16);
    h->scene_cap = scene_bytes(cfg->max_waypoints, cfg->max_circles);
    auto bail = [&](mppi_status st, const char* what, hipError_t e) {
        handle_release(h);
        delete h;
        return fail(st, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e;
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(MPPI_E_DEVICE, "hipStreamCreate", e);
        h->own_stream = true;
    }
    if ((e = hipMalloc((void**)&h->U, sizeof(double) * 2 * T)) != hipSuccess ||
        (e = hipMalloc((void**)&h->st, state_bytes(h->max_tiles))) != hipSuccess)
        return bail(MPPI_E_NOMEM, "hipMalloc", e);
    if (with_scratch) {
        struct { void** p; size_t n; } allocs[] = {
            {(void**)&h->S, sizeof(float) * K},
            {(void**)&h->eps, sizeof(float2) * (size_t)T * K},
            {(void**)&h->partials,
             sizeof(double) * partial_doubles(T, cfg->per_step_weights, (size_t)h->max_tiles)},
            {(void**)&h->wbuf, sizeof(double) * (size_t)K},
            {(void**)&h->scene, h->scene_cap},
        };
        for (auto& a : allocs)
            if ((e = hipMalloc(a.p, a.n)) != hipSuccess) return bail(MPPI_E_NOMEM, "hipMalloc", e);
        if (cfg->per_step_weights &&
            ((e = hipMalloc((void**)&h->q, sizeof(float) * (size_t)T * K)) != hipSuccess ||
             (e = hipMalloc((void**)&h->Stk, sizeof(double) * (size_t)T * K)) != hipSuccess))
            return bail(MPPI_E_NOMEM, "hipMalloc", e);
        for (int i = 0; i < 2; ++i) {
            if ((e = hipHostMalloc((void**)&h->staging[i], h->scene_cap, hipHostMallocDefault)) !=
                hipSuccess)
                return bail(MPPI_E_NOMEM, "hipHostMalloc", e);
            if ((e = hipEventCreateWithFlags(&h->staged[i], hipEventDisableTiming)) != hipSuccess)
                return bail(MPPI_E_DEVICE, "hipEventCreate", e);
        }
        if ((e = hipMemsetAsync(h->S, 0, sizeof(float) * K, h->stream)) != hipSuccess)
            return bail(MPPI_E_DEVICE, "initialise device state", e);
    }
    if ((e = hipMemsetAsync(h->U, 0, sizeof(double) * 2 * T, h->stream)) != hipSuccess ||
        (e = hipMemsetAsync(h->st, 0, state_bytes(h->max_tiles), h->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return bail(MPPI_E_DEVICE, "initialise device state", e);
    if (const char* env = getenv("MPPI_LANES_PER_SAMPLE")) {
        const int g = atoi(env);
        if (g == 1 || g == 2 || g == 4 || g == 8 || g == 16) h->lanes_req = g;
    }
    *out = h;
    return MPPI_OK;
}

// Descriptor of one iteration of handle h from state x0 on the scene at
// `scene` (device), staged relative to `origin`.
// Whether the tiles of d keep their perturbations in LDS (see kLdsShared).
int stage_allowed(const mppi_t* h, int n_c)
{
    return h->stage_req >= 0 ? h->stage_req : auto_stage(h->cfg, n_c);
}

void choose_eps_stage(InstDesc& d, bool alone, int allowed)
{
    const LdsLayout L = lds_layout(d.n_wp, d.n_c, d.T, kBlock / d.lanes, 1, d.per_step, !d.cull);
    d.eps_stage = allowed && L.eps_staged &&
                  (L.total <= kLdsShared || (alone && d.n_tiles <= 512 && L.total <= kLdsAlone));
}

void fill_desc(InstDesc& d, const mppi_t* h, const double x0[4], const double origin[2],
               const unsigned char* scene, const SceneLayout& L, int n_wp, int n_c, int shift)
{
    const mppi_config& c = h->cfg;
    memset(&d, 0, sizeof d);
    d.K = c.K;
    d.T = c.T;
    d.n_wp = n_wp;
    d.n_c = n_c;
    d.lanes = h->lanes_req ? h->lanes_req : auto_lanes(c, n_c);
    d.n_tiles = (c.K + (kBlock / d.lanes) - 1) / (kBlock / d.lanes);
    // two or more waves per SIMD (256 compute units x 4): the block-ordered
    // wave priority pays; with fewer it only costs its instructions
    d.wave_prio = (long)c.K * d.lanes >= 2L * 1024 * 64 ? 1 : 0;
    d.occ = occ_choice(h, n_c, d.lanes);
    d.dt = (float)c.dt;
    d.inv_dt = (float)(1.0 / c.dt);
    d.inv_L = (float)(1.0 / c.wheelbase);
    d.sig_a = (float)c.sigma[0];
    d.sig_d = (float)c.sigma[1];
    d.a_min = (float)c.u_min[0];
    d.a_max = (float)c.u_max[0];
    d.d_min = (float)c.u_min[1];
    d.d_max = (float)c.u_max[1];
    d.v_max = (float)c.v_max;
    d.w_track = (float)c.w_track;
    d.w_speed = (float)c.w_speed;
    d.w_effort = (float)c.w_effort;
    d.alpha = (float)((c.gamma - 1.0) / (2.0 * c.gamma));
    d.w_coll = (float)c.w_coll;
    d.d_safe_c = (float)c.d_safe_c;
    d.d_safe_0 = (float)c.d_safe_0;
    d.n_ego = c.n_ego;
    for (int e = 0; e < kMaxEgo; ++e) d.ego_off[e] = e < c.n_ego ? (float)c.ego_off[e] : 0.f;
    d.px0 = (float)(x0[0] - origin[0]);
    d.py0 = (float)(x0[1] - origin[1]);
    d.th0 = (float)x0[2];
    d.v0 = (float)x0[3];
    d.lambda = c.lambda;
    d.key0 = (uint32_t)c.seed;
    d.key1 = (uint32_t)(c.seed >> 32);
    d.shift = shift;
    d.cull = h->no_cull ? 0 : 1;
    d.smooth = c.smoothing;
    d.w_target = (float)c.w_target;
    d.w_yaw = (float)c.w_yaw;
    d.coll_only = c.collision_only;
    d.model = c.model;
    d.per_step = c.per_step_weights;
    d.steer0 = (float)h->steer0;
    d.ego_ext = 0.f;
    for (int e = 0; e < c.n_ego; ++e) d.ego_ext = fmaxf(d.ego_ext, (float)fabs(c.ego_off[e]));
    d.out_slot = -1;
    d.c_pv = reinterpret_cast<const float4*>(scene + L.o_pv);
    d.wp_xy = reinterpret_cast<const float2*>(scene + L.o_xy);
    d.wp_vref = reinterpret_cast<const float*>(scene + L.o_vr);
    d.wp_yaw = reinterpret_cast<const float*>(scene + L.o_yw);
    d.wp_box = reinterpret_cast<const float4*>(scene + L.o_box);
    d.scene_flags = reinterpret_cast<const int*>(scene + L.o_flags);
    d.c_rr = reinterpret_cast<const float*>(scene + L.o_rr);
    d.U = h->U;
    d.S = h->S;
    d.eps = h->eps;
    d.partials = h->partials;
    d.q = h->q;
    d.Stk = h->Stk;
    d.st = h->st;
    choose_eps_stage(d, false, stage_allowed(h, n_c));
}

// ---- batched launches ---------------------------------------------------------------

static bool graphs_enabled()
{
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("MPPI_BATCH_GRAPH");
        on = (e && e[0] == '0') ? 0 : 1;
    }
    return on == 1;
}

mppi_status ws_create(BatchWs** out)
{
    BatchWs* b = new (std::nothrow) BatchWs();
    if (!b) return fail(MPPI_E_NOMEM, "host allocation failed");
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        delete b;
        return fail(MPPI_E_DEVICE, "batch workspace: %s", hipGetErrorString(e));
    }
    *out = b;
    return MPPI_OK;
}

static void ws_drop_graphs(BatchWs* b)
{
    for (GraphEntry& g : b->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    b->graphs.clear();
}

void ws_destroy(BatchWs* b)
{
    if (!b) return;
    for (int i = 0; i < 2; ++i)
        if (b->pending[i]) (void)hipEventSynchronize(b->done[i]);
    ws_drop_graphs(b);
    (void)hipFree(b->arena);
    for (int i = 0; i < 2; ++i) {
        if (b->stage[i]) (void)hipHostFree(b->stage[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    }
    delete b;
}

static hipError_t ws_reserve(BatchWs* b, size_t cap, hipStream_t stream)
{
    if (b->cap >= cap) return hipSuccess;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    ws_drop_graphs(b);
    (void)hipFree(b->arena);
    b->arena = nullptr;
    for (int i = 0; i < 2; ++i) {
        if (b->stage[i]) (void)hipHostFree(b->stage[i]);
        b->stage[i] = nullptr;
        b->pending[i] = false;
    }
    b->cap = 0;
    if ((e = hipMalloc((void**)&b->arena, cap)) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
        if ((e = hipHostMalloc((void**)&b->stage[i], cap, hipHostMallocDefault)) != hipSuccess)
            return e;
    b->cap = cap;
    return hipSuccess;
}

mppi_status batch_enqueue(BatchWs* ws, hipStream_t stream, mppi_t* const* hs, const double* x0s,
                          const mppi_scene* scenes, const InstExtra* extra, int n, mppi_t* prof,
                          double* gather_dev, int slot_doubles, bool use_graph)
{
    mppi_t* h = prof;  // HIP_TRY marks it unusable on a device failure
    const size_t off_prefix = align_up(sizeof(BatchHdr), 16);
    const size_t off_descs = align_up(off_prefix + sizeof(int) * (size_t)(n + 1), 16);
    size_t bytes = align_up(off_descs + sizeof(InstDesc) * (size_t)n, 16);
    std::vector<SceneLayout> lay(n);
    std::vector<size_t> soff(n, 0);
    if (scenes) {
        for (int i = 0; i < n; ++i) {
            lay[i] = scene_layout(scenes[i].n_waypoints, scenes[i].n_circles);
            soff[i] = bytes;
            bytes += align_up(lay[i].bytes, 16);
        }
    }
    const size_t bucket = pow2_at_least(bytes, 64 << 10);
    HIP_TRY(ws_reserve(ws, bucket, stream));
    const BatchHdr* hdr_dev = reinterpret_cast<const BatchHdr*>(ws->arena);
    const int b = ws->cur;
    if (ws->pending[b]) {
        HIP_TRY(hipEventSynchronize(ws->done[b]));
        ws->pending[b] = false;
    }
    unsigned char* host = ws->stage[b];

    // group by kernel variant, longest tiles first inside a group
    std::vector<int> order(n), cls(n);
    std::vector<double> work(n);
    for (int i = 0; i < n; ++i) {
        const mppi_config& c = hs[i]->cfg;
        const int nw = scenes ? scenes[i].n_waypoints : hs[i]->n_wp;
        const int nc = scenes ? scenes[i].n_circles : hs[i]->n_c;
        const int g = hs[i]->lanes_req ? hs[i]->lanes_req : auto_lanes(c, nc);
        const int gi = g == 1 ? 0 : g == 2 ? 1 : g == 4 ? 2 : g == 8 ? 3 : 4;
        order[i] = i;
        cls[i] = 50 * occ_choice(hs[i], nc, g) + 25 * (c.model ? 1 : 0) + 5 * gi +
                 active_ego(c.n_ego, nc);
        work[i] = (double)c.T * (73.0 + 6.0 * nw + 7.0 * c.n_ego * nc);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return cls[a] != cls[c] ? cls[a] < cls[c] : work[a] > work[c];
    });
    BatchHdr* hdr = reinterpret_cast<BatchHdr*>(host);
    int* prefix = reinterpret_cast<int*>(host + off_prefix);
    InstDesc* descs = reinterpret_cast<InstDesc*>(host + off_descs);
    long total = 0;
    size_t smem = 0;
    int any_shift = 0, any_out = 0, combine_g = 0, max_nodes = 0;
    for (int j = 0; j < n; ++j) {
        const int i = order[j];
        mppi_t* hi = hs[i];
        const double* x0 = x0s + 4 * i;
        const InstExtra* ex = extra ? &extra[i] : nullptr;
        const int sh = ex && ex->shift ? 1 : 0;
        if (scenes) {
            const double origin[2] = {x0[0], x0[1]};
            write_scene(host + soff[i], lay[i], hi->cfg, origin, &scenes[i]);
            fill_desc(descs[j], hi, x0, origin, ws->arena + soff[i], lay[i], scenes[i].n_waypoints,
                      scenes[i].n_circles, sh);
        } else {
            fill_desc(descs[j], hi, x0, hi->origin, hi->scene, hi->lay, hi->n_wp, hi->n_c, sh);
        }
        if (ex) {
            descs[j].S = ex->S;
            descs[j].eps = ex->eps;
            descs[j].partials = ex->partials;
            descs[j].q = ex->q;
            descs[j].Stk = ex->Stk;
            descs[j].out_slot = ex->out_slot;
            any_out |= ex->out_slot >= 0;
        }
        prefix[j] = (int)total;
        total += descs[j].n_tiles;
        smem = std::max(smem, lds_layout(descs[j].n_wp, descs[j].n_c, descs[j].T,
                                         kBlock / descs[j].lanes, descs[j].eps_stage,
                                         descs[j].per_step, !descs[j].cull).total);
        any_shift |= sh;
        combine_g = std::max(combine_g, combine_groups(descs[j].T));
        max_nodes = std::max(max_nodes, combine_nodes(descs[j].n_tiles, nullptr));
    }
    if (total > (1L << 30)) return fail(MPPI_E_INVALID, "batch too large");
    prefix[n] = (int)total;
    hdr->n_inst = n;
    hdr->total_tiles = (int)total;
    hdr->off_prefix = (int)off_prefix;
    hdr->off_descs = (int)off_descs;
    int grids[kLaneClasses];
    {
        int j = 0;
        for (int c = 0; c < kLaneClasses; ++c) {
            hdr->cls_begin[c] = j;
            while (j < n && cls[order[j]] == c) ++j;
            const int tiles = prefix[j] - prefix[hdr->cls_begin[c]];
            grids[c] = tiles > 0 ? (int)pow2_at_least((size_t)tiles, 1) : 0;
        }
        hdr->cls_begin[kLaneClasses] = n;
    }
    const size_t smem_b = align_up(smem, 4096);
    const int node_limit = max_nodes <= kDirectSmall ? kDirectSmall : kDirect;
    const int n_blocks = (int)pow2_at_least((size_t)n, 1);
    const int shift_blocks = any_shift ? n_blocks : 0;
    const int gather_blocks = (gather_dev && any_out) ? n_blocks : 0;
    static const int kClassLanes[5] = {1, 2, 4, 8, 16};
    auto enqueue_device_work = [&](size_t copy_bytes) -> hipError_t {
        hipError_t e = hipMemcpyAsync(ws->arena, host, copy_bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && shift_blocks) e = launch_shift_batch(hdr_dev, shift_blocks, stream);
        for (int c = 0; c < kLaneClasses && e == hipSuccess; ++c)
            if (grids[c] > 0)
                e = launch_batch(kClassLanes[(c % 25) / 5], c % 5, (c % 50) / 25, c / 50, nullptr,
                                 hdr_dev, c,
                                 grids[c], smem_b, stream);
        if (e == hipSuccess && combine_g)
            e = launch_combine(nullptr, hdr_dev, combine_g, n_blocks, max_nodes, stream);
        if (e == hipSuccess && gather_blocks)
            e = launch_gather(hdr_dev, gather_blocks, gather_dev, slot_doubles, stream);
        return e;
    };

    hipEvent_t a = nullptr;
    mppi_status s = record_launch(prof, 0, &a);
    if (s != MPPI_OK) return s;
    if (use_graph && graphs_enabled()) {
        GraphEntry* ge = nullptr;
        for (GraphEntry& g : ws->graphs)
            if (g.bytes == bucket && g.smem == smem_b && g.buf == b &&
                g.shift_blocks == shift_blocks && g.gather_blocks == gather_blocks &&
                g.combine_g == combine_g && g.combine_y == (combine_g ? n_blocks : 0) &&
                g.combine_nodes == node_limit && memcmp(g.grids, grids, sizeof grids) == 0)
                ge = &g;
        if (!ge) {
            if (ws->graphs.size() >= 64) {
                // a cached graph may still be running on the stream
                HIP_TRY(hipStreamSynchronize(stream));
                ws_drop_graphs(ws);
            }
            GraphEntry g;
            g.bytes = bucket;
            g.smem = smem_b;
            memcpy(g.grids, grids, sizeof grids);
            g.buf = b;
            g.shift_blocks = shift_blocks;
            g.gather_blocks = gather_blocks;
            g.combine_g = combine_g;
            g.combine_y = combine_g ? n_blocks : 0;
            g.combine_nodes = node_limit;
            g.graph = nullptr;
            g.exec = nullptr;
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_device_work(bucket);
            const hipError_t e2 = hipStreamEndCapture(stream, &g.graph);
            HIP_TRY(e);
            HIP_TRY(e2);
            HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
            ws->graphs.push_back(g);
            ge = &ws->graphs.back();
        }
        HIP_TRY(hipGraphLaunch(ge->exec, stream));
    } else {
        HIP_TRY(enqueue_device_work(bytes));
    }
    if ((s = record_end(prof, 0, a)) != MPPI_OK) return s;
    HIP_TRY(hipEventRecord(ws->done[b], stream));
    ws->pending[b] = true;
    ws->cur ^= 1;
    for (int j = 0; j < n; ++j) {
        hs[order[j]]->stepped = true;
        hs[order[j]]->last_lanes = descs[j].lanes;
        memcpy(hs[order[j]]->last_x0, x0s + 4 * order[j], sizeof(double) * 4);
        hs[order[j]]->last_steer0 = hs[order[j]]->steer0;
    }
    return MPPI_OK;
}

}  // namespace mppi_impl

// =====================================================================================
// C ABI
// =====================================================================================

extern "C" {

const char* mppi_version(void) { return "mppi-mi355x 0.2 (gfx950)"; }

const char* mppi_status_str(mppi_status s)
{
    switch (s) {
    case MPPI_OK: return "ok";
    case MPPI_E_INVALID: return "invalid argument";
    case MPPI_E_NOMEM: return "out of memory";
    case MPPI_E_DEVICE: return "device failure";
    case MPPI_E_NONFINITE: return "all sample costs non-finite";
    case MPPI_E_BUSY: return "busy";
    case MPPI_E_NOT_READY: return "not ready";
    default: return "unknown status";
    }
}

const char* mppi_last_error(void) { return g_last_error.c_str(); }

mppi_status mppi_create(const mppi_config* cfg, void* hip_stream, mppi_t** out)
{
    return handle_create(cfg, hip_stream, true, out);
}

mppi_status mppi_destroy(mppi_t* h)
{
    if (!h) return MPPI_OK;
    handle_release(h);
    delete h;
    return MPPI_OK;
}

mppi_status mppi_set_scene(mppi_t* h, const double x0[4], const mppi_scene* sc)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if ((s = validate_scene(h->cfg, x0, sc)) != MPPI_OK) return s;
    const int b = h->cur;
    if (h->staged_pending[b]) {
        HIP_TRY(hipEventSynchronize(h->staged[b]));
        h->staged_pending[b] = false;
    }
    const SceneLayout L = scene_layout(sc->n_waypoints, sc->n_circles);
    const double origin[2] = {x0[0], x0[1]};
    write_scene(h->staging[b], L, h->cfg, origin, sc);
    HIP_TRY(hipMemcpyAsync(h->scene, h->staging[b], L.bytes, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipEventRecord(h->staged[b], h->stream));
    h->staged_pending[b] = true;
    h->cur ^= 1;
    h->has_scene = true;
    h->origin[0] = origin[0];
    h->origin[1] = origin[1];
    h->n_wp = sc->n_waypoints;
    h->n_c = sc->n_circles;
    h->lay = L;
    return MPPI_OK;
}

mppi_status mppi_step_resident(mppi_t* h, const double x0[4])
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!h->has_scene) return fail(MPPI_E_INVALID, "no scene has been set");
    if (!x0) return fail(MPPI_E_INVALID, "x0 must not be NULL");
    for (int i = 0; i < 4; ++i)
        if (!isfinite(x0[i])) return fail(MPPI_E_INVALID, "x0[%d] is not finite", i);
    InstDesc d;
    fill_desc(d, h, x0, h->origin, h->scene, h->lay, h->n_wp, h->n_c, 0);
    choose_eps_stage(d, true, stage_allowed(h, h->n_c));
    const size_t smem =
        lds_layout(d.n_wp, d.n_c, d.T, kBlock / d.lanes, d.eps_stage, d.per_step, !d.cull).total;
    hipEvent_t a = nullptr;
    if ((s = record_launch(h, 0, &a)) != MPPI_OK) return s;
    hipEvent_t a2 = nullptr;
    if ((s = record_launch(h, 2, &a2)) != MPPI_OK) return s;
    HIP_TRY(launch_batch(d.lanes, active_ego(d.n_ego, d.n_c), d.model, d.occ, &d, nullptr, 0,
                         d.n_tiles,
                         smem, h->stream));
    if ((s = record_end(h, 2, a2)) != MPPI_OK) return s;
    HIP_TRY(launch_combine(&d, nullptr, combine_groups(d.T), 1, combine_nodes(d.n_tiles, nullptr),
                           h->stream));
    if ((s = record_end(h, 0, a)) != MPPI_OK) return s;
    h->last_lanes = d.lanes;
    h->stepped = true;
    memcpy(h->last_x0, x0, sizeof(double) * 4);
    h->last_steer0 = h->steer0;
    return MPPI_OK;
}

mppi_status mppi_step(mppi_t* h, const double x0[4], const mppi_scene* sc)
{
    mppi_status s = mppi_set_scene(h, x0, sc);
    if (s != MPPI_OK) return s;
    return mppi_step_resident(h, x0);
}

mppi_status mppi_step_batch(mppi_t* const* hs, const double* x0s, const mppi_scene* scenes,
                            int32_t n)
{
    if (!hs || !x0s || n < 1) return fail(MPPI_E_INVALID, "handles, states and n >= 1 required");
    mppi_t* lead = hs[0];
    mppi_status s;
    for (int i = 0; i < n; ++i) {
        if ((s = usable(hs[i])) != MPPI_OK) return s;
        if (!hs[i]->S) return fail(MPPI_E_INVALID, "handle %d has no iteration buffers", i);
        if (hs[i]->stream != lead->stream)
            return fail(MPPI_E_INVALID, "every handle of a batch must use the same stream");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return fail(MPPI_E_INVALID, "handle %d appears twice", i);
        if (scenes) {
            if ((s = validate_scene(hs[i]->cfg, x0s + 4 * i, &scenes[i])) != MPPI_OK) return s;
        } else {
            if (!hs[i]->has_scene) return fail(MPPI_E_INVALID, "handle %d has no scene", i);
            for (int k = 0; k < 4; ++k)
                if (!isfinite(x0s[4 * i + k])) return fail(MPPI_E_INVALID, "x0 not finite");
        }
    }
    if (!lead->batch && (s = ws_create(&lead->batch)) != MPPI_OK) return s;
    return batch_enqueue(lead->batch, lead->stream, hs, x0s, scenes, nullptr, n, lead, nullptr, 0,
                         true);
}

mppi_status mppi_sync(mppi_t* h)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    return sync_status(h);
}

mppi_status mppi_get_controls(mppi_t* h, double* out, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out || n < (size_t)2 * h->cfg.T)
        return fail(MPPI_E_INVALID, "output buffer needs %d doubles", 2 * h->cfg.T);
    // U and the state written by one small kernel straight into pinned host
    // memory, then one synchronisation (no copies back to wait for)
    if ((s = host_buffers(h)) != MPPI_OK) return s;
    const int nu = 2 * h->cfg.T;
    HIP_TRY(launch_export_controls(h->U, nu, h->st, h->ctl_dev,
                                   reinterpret_cast<DevState*>(h->ctl_dev + nu), h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    memcpy(out, h->ctl_host, sizeof(double) * nu);
    if (h->stepped && reinterpret_cast<const DevState*>(h->ctl_host + nu)->status != 0)
        return fail(MPPI_E_NONFINITE, "every sample cost of the last step was non-finite");
    return MPPI_OK;
}

mppi_status mppi_set_controls(mppi_t* h, const double* U, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!U || n < (size_t)2 * h->cfg.T)
        return fail(MPPI_E_INVALID, "controls need %d doubles", 2 * h->cfg.T);
    for (int i = 0; i < 2 * h->cfg.T; ++i)
        if (!isfinite(U[i])) return fail(MPPI_E_INVALID, "controls must be finite");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(h->U, U, sizeof(double) * 2 * h->cfg.T, hipMemcpyHostToDevice));
    return MPPI_OK;
}

mppi_status mppi_shift(mppi_t* h, int32_t steps)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (steps < 0) return fail(MPPI_E_INVALID, "steps must be >= 0");
    if (steps == 0) return MPPI_OK;
    return launch_aux(h, [&] { return launch_shift(h->U, h->cfg.T, steps, h->stream); });
}

mppi_status mppi_get_state(mppi_t* h, double* U, size_t n, uint64_t* n_iter, uint64_t* seed)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!U || n < (size_t)2 * h->cfg.T)
        return fail(MPPI_E_INVALID, "state buffer needs %d doubles", 2 * h->cfg.T);
    // U and the state through the pinned export buffer (one small kernel,
    // one synchronisation)
    if ((s = host_buffers(h)) != MPPI_OK) return s;
    const int nu = 2 * h->cfg.T;
    HIP_TRY(launch_export_controls(h->U, nu, h->st, h->ctl_dev,
                                   reinterpret_cast<DevState*>(h->ctl_dev + nu), h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    memcpy(U, h->ctl_host, sizeof(double) * nu);
    if (n_iter) *n_iter = reinterpret_cast<const DevState*>(h->ctl_host + nu)->n_iter;
    if (seed) *seed = h->cfg.seed;
    return MPPI_OK;
}

mppi_status mppi_set_state(mppi_t* h, const double* U, size_t n, uint64_t n_iter)
{
    mppi_status s = mppi_set_controls(h, U, n);
    if (s != MPPI_OK) return s;
    DevState st;
    HIP_TRY(hipMemcpy(&st, h->st, sizeof st, hipMemcpyDeviceToHost));
    st.n_iter = n_iter;
    st.reserved = 0;
    st.status = 0;
    HIP_TRY(hipMemcpy(h->st, &st, sizeof st, hipMemcpyHostToDevice));
    h->stepped = false;
    return MPPI_OK;
}

mppi_status mppi_get_costs(mppi_t* h, float* out, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out || n < (size_t)h->cfg.K) return fail(MPPI_E_INVALID, "buffer needs K floats");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->S, sizeof(float) * h->cfg.K, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

mppi_status mppi_get_weights(mppi_t* h, double* out, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out || n < (size_t)h->cfg.K) return fail(MPPI_E_INVALID, "buffer needs K doubles");
    if ((s = sync_status(h)) != MPPI_OK) return s;
    if (!h->stepped) return fail(MPPI_E_NOT_READY, "no step has completed");
    InstDesc d;
    memset(&d, 0, sizeof d);
    d.K = h->cfg.K;
    d.S = h->S;
    d.per_step = h->cfg.per_step_weights;
    d.Stk = h->Stk;
    d.lambda = h->cfg.lambda;
    d.st = h->st;
    s = launch_aux(h, [&] { return launch_weights(d, h->wbuf, h->stream); });
    if (s != MPPI_OK) return s;
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->wbuf, sizeof(double) * h->cfg.K, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

mppi_status mppi_get_noise(mppi_t* h, float* out, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    const size_t need = (size_t)2 * h->cfg.T * h->cfg.K;
    if (!out || n < need) return fail(MPPI_E_INVALID, "buffer needs 2*T*K floats");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->eps, sizeof(float) * need, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

mppi_status mppi_get_trajectory(mppi_t* h, double* states, size_t n_states, double* controls,
                                size_t n_controls)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    const int T = h->cfg.T;
    const size_t cols = h->cfg.model ? 5 : 4;
    if (!h->stepped) return fail(MPPI_E_INVALID, "no step has been taken");
    if (states && n_states < cols * (T + 1))
        return fail(MPPI_E_INVALID, "states needs %zu*(T+1) doubles", cols);
    if (controls && n_controls < (size_t)2 * T)
        return fail(MPPI_E_INVALID, "controls needs 2*T doubles");
    TrajArgs a;
    const mppi_config& c = h->cfg;
    for (int i = 0; i < 4; ++i) a.x0[i] = h->last_x0[i];
    a.steer0 = h->last_steer0;
    a.T = T;
    a.model = c.model;
    a.dt = c.dt;
    a.wheelbase = c.wheelbase;
    a.a_min = c.u_min[0];
    a.a_max = c.u_max[0];
    a.d_min = c.u_min[1];
    a.d_max = c.u_max[1];
    a.v_max = c.v_max;
    // states then controls, written by the kernel straight into the pinned
    // host buffer: no copy back to wait for
    const size_t ns = cols * (T + 1), nu = (size_t)2 * T;
    if ((s = host_buffers(h)) != MPPI_OK) return s;
    HIP_TRY(launch_trajectory(a, h->U, h->traj_dev, h->traj_dev + ns, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (states) memcpy(states, h->traj, sizeof(double) * ns);
    if (controls) memcpy(controls, h->traj + ns, sizeof(double) * nu);
    return MPPI_OK;
}

mppi_status mppi_get_stage_costs(mppi_t* h, float* out, size_t n)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!h->cfg.per_step_weights || !h->q)
        return fail(MPPI_E_INVALID, "stage costs are kept only with per-step weights");
    const size_t need = (size_t)h->cfg.T * h->cfg.K;
    if (!out || n < need) return fail(MPPI_E_INVALID, "buffer needs T*K floats");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->q, sizeof(float) * need, hipMemcpyDeviceToHost));
    return MPPI_OK;
}

mppi_status mppi_set_steering(mppi_t* h, double delta0)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!isfinite(delta0)) return fail(MPPI_E_INVALID, "steering angle must be finite");
    h->steer0 = delta0;
    return MPPI_OK;
}

mppi_status mppi_get_iter_stats(mppi_t* h, mppi_iter_stats* out)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out) return fail(MPPI_E_INVALID, "out is NULL");
    DevState st;
    s = read_state(h, &st);
    if (s != MPPI_OK) return s;
    out->s_min = st.s_min;
    out->log_z = st.log_z;
    out->ess = st.ess;
    out->n_iter = st.n_iter;
    out->status = st.status;
    out->lanes_per_sample = h->last_lanes;
    return MPPI_OK;
}

mppi_status mppi_set_lanes_per_sample(mppi_t* h, int32_t lanes)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!(lanes == 0 || lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16))
        return fail(MPPI_E_INVALID, "lanes per sample must be 0, 1, 2, 4, 8 or 16");
    h->lanes_req = lanes;
    return MPPI_OK;
}

mppi_status mppi_set_occupancy(mppi_t* h, int32_t mode)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (mode < -1 || mode >= kOccModes)
        return fail(MPPI_E_INVALID, "occupancy mode must be -1, 0 or 1");
    h->occ_req = mode;
    return MPPI_OK;
}

mppi_status mppi_set_staging(mppi_t* h, int32_t mode)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (mode < -1 || mode > 1) return fail(MPPI_E_INVALID, "staging mode must be -1, 0 or 1");
    h->stage_req = mode;
    return MPPI_OK;
}

mppi_status mppi_set_culling(mppi_t* h, int32_t on)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    h->no_cull = on ? 0 : 1;
    return MPPI_OK;
}

mppi_status mppi_get_stream(mppi_t* h, void** stream)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!stream) return fail(MPPI_E_INVALID, "stream is NULL");
    *stream = (void*)h->stream;
    return MPPI_OK;
}

mppi_status mppi_set_profiling(mppi_t* h, int32_t on)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if ((s = drain_profile(h)) != MPPI_OK) return s;
    h->prof = on != 0;
    if (on) {
        h->prof_ms[0] = h->prof_ms[1] = h->prof_ms[2] = 0.0;
        h->prof_n[0] = h->prof_n[1] = h->prof_n[2] = 0;
        // events for a few hundred profiled steps, created now rather than
        // between launches
        while (h->event_pool.size() < 1024) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            h->event_pool.push_back(e);
        }
    }
    return MPPI_OK;
}

mppi_status mppi_get_profile(mppi_t* h, mppi_profile* out)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out) return fail(MPPI_E_INVALID, "out is NULL");
    if ((s = drain_profile(h)) != MPPI_OK) return s;
    out->iter_ms = h->prof_ms[0];
    out->iter_launches = h->prof_n[0];
    out->aux_ms = h->prof_ms[1];
    out->aux_launches = h->prof_n[1];
    out->rollout_ms = h->prof_ms[2];
    out->rollout_launches = h->prof_n[2];
    return MPPI_OK;
}

mppi_status mppi_debug_philox(uint64_t seed, uint64_t n_iter, uint32_t k0, uint32_t nk,
                              uint32_t j0, uint32_t nj, uint32_t* out, size_t n)
{
    const uint64_t cnt = (uint64_t)nk * nj;
    if (!out || n < 4 * cnt) return fail(MPPI_E_INVALID, "buffer needs 4*nk*nj words");
    if (cnt == 0) return MPPI_OK;
    if (cnt > (1ull << 28)) return fail(MPPI_E_INVALID, "nk*nj too large");
    uint32_t* dev = nullptr;
    hipError_t e = hipMalloc((void**)&dev, sizeof(uint32_t) * 4 * cnt);
    if (e != hipSuccess) return fail(MPPI_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    e = launch_debug_philox((uint32_t)seed, (uint32_t)(seed >> 32), n_iter, k0, nk, j0, nj, dev,
                            nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(out, dev, sizeof(uint32_t) * 4 * cnt, hipMemcpyDeviceToHost);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(MPPI_E_DEVICE, "debug philox: %s", hipGetErrorString(e));
    return MPPI_OK;
}

mppi_status mppi_bench_copy(size_t bytes, int32_t reps)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0 || reps < 1) return fail(MPPI_E_INVALID, "bytes >= 16 and reps >= 1 required");
    float4 *a = nullptr, *b = nullptr;
    hipError_t e = hipMalloc((void**)&a, n16 * 16);
    if (e == hipSuccess) e = hipMalloc((void**)&b, n16 * 16);
    if (e == hipSuccess) e = hipMemset(a, 0, n16 * 16);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(a, b, n16, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(MPPI_E_DEVICE, "copy: %s", hipGetErrorString(e));
    return MPPI_OK;
}

}  // extern "C"
