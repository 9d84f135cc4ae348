// Host runtime behind the C ABI of include/mppi.h: handle life cycle,
// validation, ego-frame staging of the scene, kernel launches, result
// export, checkpointing and profiling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_internal.hpp"

using namespace mppi_impl;

namespace {

thread_local std::string g_last_error;

mppi_status fail(mppi_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
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

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            h->sticky = MPPI_E_DEVICE;                                                       \
            return fail(MPPI_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                                 \
        }                                                                                    \
    } while (0)

struct ProfEvent {
    hipEvent_t a, b;
    int kind;  // 0 = iteration kernel, 1 = auxiliary
};

int next_pow2(long v)
{
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

}  // namespace

struct mppi {
    mppi_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int lanes_req = 0;   // 0 = automatic
    int last_lanes = 0;
    mppi_status sticky = MPPI_OK;
    // device memory
    double* U = nullptr;
    float* S = nullptr;
    float2* eps = nullptr;
    double* partials = nullptr;
    double* scales = nullptr;
    double* wbuf = nullptr;    // [K] weights export
    DevState* st = nullptr;
    unsigned char* scene = nullptr;
    size_t scene_cap = 0;
    // pinned staging, double-buffered
    unsigned char* staging[2] = {nullptr, nullptr};
    hipEvent_t staged[2] = {nullptr, nullptr};
    bool staged_pending[2] = {false, false};
    int cur = 0;
    int max_tiles = 0;
    // resident scene
    bool has_scene = false;
    double origin[2] = {0.0, 0.0};
    int n_wp = 0, n_c = 0;
    size_t o_pv = 0, o_xy = 0, o_vr = 0, o_rr = 0;
    // last step
    bool stepped = false;
    // profiling
    bool prof = false;
    std::vector<ProfEvent> events;
    double prof_ms[2] = {0.0, 0.0};
    int64_t prof_n[2] = {0, 0};
};

namespace {

size_t scene_bytes(int n_wp, int n_c)
{
    return align_up((size_t)n_c * 16, 16) + align_up((size_t)n_wp * 8, 16) +
           align_up((size_t)n_wp * 4, 16) + align_up((size_t)n_c * 4, 16);
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
    return MPPI_OK;
}

mppi_status usable(mppi_t* h)
{
    if (!h) return fail(MPPI_E_INVALID, "handle is NULL");
    if (h->sticky != MPPI_OK)
        return fail(h->sticky, "handle is unusable after an earlier device failure");
    return MPPI_OK;
}

int auto_lanes(const mppi_config& c)
{
    // Enough lanes to give every SIMD of the 256 CUs two waves.
    const long target = 2L * 256 * 4 * 64;
    int g = next_pow2((target + c.K - 1) / c.K);
    g = std::min(g, 16);
    while (g > 1 && g > c.T) g >>= 1;
    return std::max(g, 1);
}

mppi_status record_launch(mppi_t* h, int kind, hipEvent_t* a)
{
    if (!h->prof) return MPPI_OK;
    HIP_TRY(hipEventCreate(a));
    HIP_TRY(hipEventRecord(*a, h->stream));
    (void)kind;
    return MPPI_OK;
}

mppi_status record_end(mppi_t* h, int kind, hipEvent_t a)
{
    if (!h->prof) return MPPI_OK;
    hipEvent_t b;
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(b, h->stream));
    h->events.push_back(ProfEvent{a, b, kind});
    return MPPI_OK;
}

mppi_status drain_profile(mppi_t* h)
{
    if (h->events.empty()) return MPPI_OK;
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (const ProfEvent& e : h->events) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
        h->prof_ms[e.kind] += ms;
        h->prof_n[e.kind] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    h->events.clear();
    return MPPI_OK;
}

template <typename F>
mppi_status launch_aux(mppi_t* h, F&& f)
{
    hipEvent_t a = nullptr;
    mppi_status s = record_launch(h, 1, &a);
    if (s != MPPI_OK) return s;
    HIP_TRY(f());
    return record_end(h, 1, a);
}

mppi_status sync_status(mppi_t* h)
{
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (!h->stepped) return MPPI_OK;
    DevState st;
    HIP_TRY(hipMemcpy(&st, h->st, sizeof st, hipMemcpyDeviceToHost));
    if (st.status != 0) return fail(MPPI_E_NONFINITE, "every sample cost of the last step was non-finite");
    return MPPI_OK;
}

void release(mppi_t* h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (const ProfEvent& e : h->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    (void)hipFree(h->U);
    (void)hipFree(h->S);
    (void)hipFree(h->eps);
    (void)hipFree(h->partials);
    (void)hipFree(h->scales);
    (void)hipFree(h->wbuf);
    (void)hipFree(h->st);
    (void)hipFree(h->scene);
    for (int i = 0; i < 2; ++i) {
        if (h->staging[i]) (void)hipHostFree(h->staging[i]);
        if (h->staged[i]) (void)hipEventDestroy(h->staged[i]);
    }
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

}  // namespace

extern "C" {

const char* mppi_version(void) { return "mppi-mi355x 0.1 (gfx950)"; }

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
        release(h);
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
    struct { void** p; size_t n; } allocs[] = {
        {(void**)&h->U, sizeof(double) * 2 * T},
        {(void**)&h->S, sizeof(float) * K},
        {(void**)&h->eps, sizeof(float2) * (size_t)T * K},
        {(void**)&h->partials, sizeof(double) * (size_t)h->max_tiles * (kPartialHead + 2 * T)},
        {(void**)&h->scales, sizeof(double) * (size_t)h->max_tiles},
        {(void**)&h->wbuf, sizeof(double) * (size_t)K},
        {(void**)&h->st, sizeof(DevState)},
        {(void**)&h->scene, h->scene_cap},
    };
    for (auto& a : allocs)
        if ((e = hipMalloc(a.p, a.n)) != hipSuccess) return bail(MPPI_E_NOMEM, "hipMalloc", e);
    for (int i = 0; i < 2; ++i) {
        if ((e = hipHostMalloc((void**)&h->staging[i], h->scene_cap, hipHostMallocDefault)) != hipSuccess)
            return bail(MPPI_E_NOMEM, "hipHostMalloc", e);
        if ((e = hipEventCreateWithFlags(&h->staged[i], hipEventDisableTiming)) != hipSuccess)
            return bail(MPPI_E_DEVICE, "hipEventCreate", e);
    }
    if ((e = hipMemsetAsync(h->U, 0, sizeof(double) * 2 * T, h->stream)) != hipSuccess ||
        (e = hipMemsetAsync(h->st, 0, sizeof(DevState), h->stream)) != hipSuccess ||
        (e = hipMemsetAsync(h->S, 0, sizeof(float) * K, h->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess)
        return bail(MPPI_E_DEVICE, "initialise device state", e);
    if (const char* env = getenv("MPPI_LANES_PER_SAMPLE")) {
        int g = atoi(env);
        if (g == 1 || g == 2 || g == 4 || g == 8 || g == 16) h->lanes_req = g;
    }
    *out = h;
    return MPPI_OK;
}

mppi_status mppi_destroy(mppi_t* h)
{
    if (!h) return MPPI_OK;
    release(h);
    delete h;
    return MPPI_OK;
}

mppi_status mppi_set_scene(mppi_t* h, const double x0[4], const mppi_scene* sc)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    const mppi_config& c = h->cfg;
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

    // ego-frame staging (float64 subtraction, then float32), double-buffered
    const int b = h->cur;
    if (h->staged_pending[b]) {
        HIP_TRY(hipEventSynchronize(h->staged[b]));
        h->staged_pending[b] = false;
    }
    unsigned char* stg = h->staging[b];
    const size_t o_pv = 0;
    const size_t o_xy = o_pv + align_up((size_t)n_c * 16, 16);
    const size_t o_vr = o_xy + align_up((size_t)n_wp * 8, 16);
    const size_t o_rr = o_vr + align_up((size_t)n_wp * 4, 16);
    const size_t bytes = o_rr + align_up((size_t)n_c * 4, 16);
    float4* pv = reinterpret_cast<float4*>(stg + o_pv);
    float2* xy = reinterpret_cast<float2*>(stg + o_xy);
    float* vr = reinterpret_cast<float*>(stg + o_vr);
    float* rr = reinterpret_cast<float*>(stg + o_rr);
    for (int i = 0; i < n_wp; ++i) {
        const double* w = sc->waypoints + 4 * i;
        xy[i] = make_float2((float)(w[0] - x0[0]), (float)(w[1] - x0[1]));
        vr[i] = (float)w[3];
    }
    for (int i = 0; i < n_c; ++i) {
        const double* o = sc->circles + 5 * i;
        pv[i] = make_float4((float)(o[0] - x0[0]), (float)(o[1] - x0[1]), (float)o[3], (float)o[4]);
        rr[i] = (float)(o[2] + c.ego_r);
    }
    HIP_TRY(hipMemcpyAsync(h->scene, stg, bytes, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipEventRecord(h->staged[b], h->stream));
    h->staged_pending[b] = true;
    h->cur ^= 1;
    h->has_scene = true;
    h->origin[0] = x0[0];
    h->origin[1] = x0[1];
    h->n_wp = n_wp;
    h->n_c = n_c;
    h->o_pv = o_pv;
    h->o_xy = o_xy;
    h->o_vr = o_vr;
    h->o_rr = o_rr;
    return MPPI_OK;
}

mppi_status mppi_step_resident(mppi_t* h, const double x0[4])
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    const mppi_config& c = h->cfg;
    if (!h->has_scene) return fail(MPPI_E_INVALID, "no scene has been set");
    if (!x0) return fail(MPPI_E_INVALID, "x0 must not be NULL");
    for (int i = 0; i < 4; ++i)
        if (!isfinite(x0[i])) return fail(MPPI_E_INVALID, "x0[%d] is not finite", i);

    InstDesc d;
    memset(&d, 0, sizeof d);
    d.K = c.K;
    d.T = c.T;
    d.n_wp = h->n_wp;
    d.n_c = h->n_c;
    d.lanes = h->lanes_req ? h->lanes_req : auto_lanes(c);
    d.n_tiles = (c.K + (kBlock / d.lanes) - 1) / (kBlock / d.lanes);
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
    d.px0 = (float)(x0[0] - h->origin[0]);
    d.py0 = (float)(x0[1] - h->origin[1]);
    d.th0 = (float)x0[2];
    d.v0 = (float)x0[3];
    d.lambda = c.lambda;
    d.key0 = (uint32_t)c.seed;
    d.key1 = (uint32_t)(c.seed >> 32);
    d.c_pv = reinterpret_cast<const float4*>(h->scene + h->o_pv);
    d.wp_xy = reinterpret_cast<const float2*>(h->scene + h->o_xy);
    d.wp_vref = reinterpret_cast<const float*>(h->scene + h->o_vr);
    d.c_rr = reinterpret_cast<const float*>(h->scene + h->o_rr);
    d.U = h->U;
    d.S = h->S;
    d.eps = h->eps;
    d.partials = h->partials;
    d.scales = h->scales;
    d.st = h->st;

    hipEvent_t a = nullptr;
    if ((s = record_launch(h, 0, &a)) != MPPI_OK) return s;
    HIP_TRY(launch_iteration(d, h->stream));
    if ((s = record_end(h, 0, a)) != MPPI_OK) return s;
    h->last_lanes = d.lanes;
    h->stepped = true;
    return MPPI_OK;
}

mppi_status mppi_step(mppi_t* h, const double x0[4], const mppi_scene* sc)
{
    mppi_status s = mppi_set_scene(h, x0, sc);
    if (s != MPPI_OK) return s;
    return mppi_step_resident(h, x0);
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
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->U, sizeof(double) * 2 * h->cfg.T, hipMemcpyDeviceToHost));
    return sync_status(h);
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
    HIP_TRY(hipStreamSynchronize(h->stream));
    DevState st;
    HIP_TRY(hipMemcpy(&st, h->st, sizeof st, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(U, h->U, sizeof(double) * 2 * h->cfg.T, hipMemcpyDeviceToHost));
    if (n_iter) *n_iter = st.n_iter;
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
    st.ticket = 0;
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
    double* w = h->wbuf;
    InstDesc d;
    memset(&d, 0, sizeof d);
    d.K = h->cfg.K;
    d.S = h->S;
    d.lambda = h->cfg.lambda;
    d.st = h->st;
    s = launch_aux(h, [&] { return launch_weights(d, w, h->stream); });
    if (s != MPPI_OK) return s;
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, w, sizeof(double) * h->cfg.K, hipMemcpyDeviceToHost));
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

mppi_status mppi_get_iter_stats(mppi_t* h, mppi_iter_stats* out)
{
    mppi_status s = usable(h);
    if (s != MPPI_OK) return s;
    if (!out) return fail(MPPI_E_INVALID, "out is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    DevState st;
    HIP_TRY(hipMemcpy(&st, h->st, sizeof st, hipMemcpyDeviceToHost));
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
        h->prof_ms[0] = h->prof_ms[1] = 0.0;
        h->prof_n[0] = h->prof_n[1] = 0;
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
