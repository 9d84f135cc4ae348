/*
 * mppi.h -- C ABI of an MI355X (gfx950) library that runs the sampling-based
 * motion planner of Testouri, Elghazaly and Frank, "Towards a Safe Real-Time
 * Motion Planning Framework for Autonomous Driving Systems: A Model
 * Predictive Path Integral Approach" (arXiv 2308.01654).
 *
 * One call of mppi_step is one MPPI iteration (Algorithm 1, from the noise
 * generation through the input update):
 *   - draw K perturbation sequences eps_k in R^{T x 2} (Philox4x32-10 +
 *     Box-Muller, counter = (k, t/2, n_lo, n_hi), key = seed);
 *   - apply the noise check of Sec. III-A (clamp into [u_min, u_max], cap the
 *     acceleration so that v never exceeds v_max, braking bound last);
 *   - roll out the kinematic bicycle of eq. (5) (state x, y, yaw, v; controls
 *     acceleration and steering angle; explicit Euler) for T steps;
 *   - accumulate the Sec. III input cost and the Sec. IV-C state costs on
 *     every new state: tracking (squared distance to the closest waypoint),
 *     speed (against that waypoint's reference speed) and the obstacle cost
 *     over circle-approximated obstacles with the safety distance
 *     d_safe = d_safe_c v + d_safe_0;
 *   - weights w_k = exp(-(S_k - S_min)/lambda) / sum_j exp(-(S_j - S_min)/lambda)
 *     and the update U_t += sum_k w_k eps_eff[k][t] (eq. (update-input)).
 * The problem tuple P = <V, S, B, J> of Sec. II-A maps onto the two structs:
 * mppi_config holds the vehicle model V, the objective J and the sampling
 * parameters; mppi_scene holds the scene S (obstacle circles) and the road
 * boundary B (reference waypoints).
 *
 * Conventions for every function:
 *   - Return value: MPPI_OK (0) or a negative mppi_status.  On error the
 *     handle's controls U, iteration counter n and stored results are left
 *     unchanged, and mppi_last_error() describes the failure.
 *   - Pointers are host pointers unless stated otherwise.  Every input array
 *     is copied before the call returns; the caller keeps ownership and may
 *     free or reuse it at once.  Outputs go into caller buffers whose length
 *     (in elements) is passed explicitly; a buffer that is too small gives
 *     MPPI_E_INVALID and nothing is written.
 *   - The library owns all device memory and releases it in mppi_destroy.
 *   - Work is enqueued on the handle's HIP stream; calls that return data to
 *     the host synchronize that stream.  A device failure is sticky
 *     (MPPI_E_DEVICE) and makes the handle unusable.
 *   - A handle is not thread-safe; distinct handles may be used from distinct
 *     threads.  No C++ exception crosses this interface.
 *   - Arrays are row-major, float64 unless stated otherwise.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mppi_status;
#define MPPI_OK            0
#define MPPI_E_INVALID   (-1) /* bad argument, size or value                     */
#define MPPI_E_NOMEM     (-2) /* device or host allocation failed                */
#define MPPI_E_DEVICE    (-3) /* HIP runtime / kernel failure (sticky)           */
#define MPPI_E_NONFINITE (-4) /* every sample cost was non-finite; U unchanged   */
#define MPPI_E_BUSY      (-5) /* reserved for queue-capacity refusals            */
#define MPPI_E_NOT_READY (-6) /* result not available yet                        */

/* Vehicle model, objective and sampling parameters (Sec. II-A, Sec. III,
 * Sec. IV-C, Table I).  Bounds may be +-INFINITY to disable them. */
typedef struct mppi_config {
    int32_t K;             /* samples per iteration (Alg. 1: M), 1..2^24              */
    int32_t T;             /* horizon steps, 1..2048                                   */
    double dt;             /* step length [s], > 0                                     */
    double wheelbase;      /* l of eq. (5) [m], > 0                                    */
    double lambda;         /* temperature of the weights, > 0                          */
    double gamma;          /* alpha = (gamma-1)/(2 gamma) of the input cost, > 0        */
    double sigma[2];       /* noise std dev of (acceleration, steering), >= 0           */
    double u_min[2];       /* lower bounds (a_min, delta_min)                           */
    double u_max[2];       /* upper bounds (a_max, delta_max)                           */
    double v_max;          /* speed cap of the noise check (target speed v_G)          */
    double w_track;        /* weight of c_dist                                          */
    double w_speed;        /* weight of c_speed                                         */
    double w_effort;       /* R = w_effort * I of the input cost                        */
    double w_coll;         /* weight of the obstacle cost c_safe_dist                   */
    double d_safe_c;       /* safe-distance coefficient [s]                             */
    double d_safe_0;       /* minimal safe distance [m]                                 */
    int32_t n_ego;         /* ego circles, 0..4                                         */
    double ego_r;          /* radius of every ego circle [m]                            */
    double ego_off[4];     /* ego circle centres along the heading from (x, y) [m]      */
    uint64_t seed;         /* Philox key                                                */
    int32_t max_waypoints; /* capacity for mppi_scene.n_waypoints, 1..2048              */
    int32_t max_circles;   /* capacity for mppi_scene.n_circles, 0..1024                */
    int32_t smoothing;     /* 1: end every iteration with the Savitzky-Golay filter of
                              eq. (sg) (window (-3,12,17,12,-3)/35, end values repeated
                              beyond the horizon), which replaces U -- the last steps of
                              Alg. 1, so a warm-start shift then shifts u*; 0: off      */
    double w_target;       /* weight of c_target (Sec. IV-C): 1 when a step ends farther
                              from the target point (the last waypoint) than it began   */
    double w_yaw;          /* weight of c_yaw (Sec. IV-C): heading minus the closest
                              waypoint's yaw, wrapped into [-pi, pi), squared            */
    int32_t collision_only;/* 1: c_safe_dist only when an object is hit, d_obj <= 0
                              (the paper's object-avoidance mode); 0: always            */
    int32_t model;         /* 0: 4-state bicycle, controls (a, steering angle delta);
                              1: the 5-state model of eq. (5), the steering angle is
                              state and the second control is the steering rate omega
                              (sigma[1], u_min[1], u_max[1] then bound omega, e.g.
                              +-omega_max); the initial angle comes from
                              mppi_set_steering.  Served vehicles must use 0.          */
    int32_t per_step_weights; /* 1: the update of U_t weights the samples by their
                              cost-to-go from t, S_t,k = sum_{s>=t} q_s,k, with a
                              minimum per t (eq. (update-input) indexed by t); 0: one
                              total cost per sample for every t                        */
} mppi_config;

/* Scene and road model of one request, world coordinates. */
typedef struct mppi_scene {
    const double* waypoints; /* [n_waypoints][4]: x, y, yaw, v_ref                    */
    int32_t n_waypoints;     /* 1..max_waypoints                                        */
    const double* circles;   /* [n_circles][5]: x, y, r, vx, vy at request time;
                                the centre moves at (vx, vy); may be NULL if n == 0   */
    int32_t n_circles;       /* 0..max_circles                                          */
} mppi_scene;

typedef struct mppi mppi_t;

/* Per-iteration summary of the last completed step. */
typedef struct mppi_iter_stats {
    double s_min;      /* S_min of Alg. 1                                           */
    double log_z;      /* log sum_k exp(-(S_k - S_min)/lambda)                      */
    double ess;        /* effective sample size 1 / sum_k w_k^2                     */
    uint64_t n_iter;   /* iteration counter after the step                          */
    int32_t status;    /* MPPI_OK or MPPI_E_NONFINITE of the last step              */
    int32_t lanes_per_sample; /* launch shape used by the last step                */
} mppi_iter_stats;

/* Accumulated device time while profiling is on (HIP events). */
typedef struct mppi_profile {
    double iter_ms;        /* iterations: iteration kernel and combine kernel         */
    int64_t iter_launches;
    double aux_ms;         /* every other kernel of the handle                        */
    int64_t aux_launches;
    double rollout_ms;     /* the iteration kernel alone (sampling, rollouts, costs,
                              tile partials) of single-instance steps                */
    int64_t rollout_launches;
} mppi_profile;

/* ---- single planning instance -------------------------------------------- */

/* Create a planning instance.  hip_stream: a hipStream_t of the caller (work
 * is enqueued on it) or NULL to let the library create its own.  U starts at
 * zero and the iteration counter n at 0.  Allocates device memory for
 * K x T perturbations (8 bytes each) plus the scene capacity. */
mppi_status mppi_create(const mppi_config* cfg, void* hip_stream, mppi_t** out);

/* Release every resource of the handle (synchronizes its stream).  NULL is a
 * no-op. */
mppi_status mppi_destroy(mppi_t* h);

/* One MPPI iteration (Alg. 1, noise generation through input update) from
 * state x0 = (x, y, yaw, v) in the given scene.  Asynchronous: returns after
 * the work is enqueued.  Uses and then increments the handle's iteration
 * counter n (the Philox counter); a step whose every sample cost is
 * non-finite leaves U and n unchanged and is reported by the next
 * synchronizing call as MPPI_E_NONFINITE. */
mppi_status mppi_step(mppi_t* h, const double x0[4], const mppi_scene* scene);

/* Stage a scene on the device (the first half of mppi_step): validates it,
 * converts it to float32 coordinates relative to origin = (x, y) of the given
 * state (the ego frame) and enqueues the host-to-device copy.  The scene then
 * stays resident until the next mppi_set_scene / mppi_step. */
mppi_status mppi_set_scene(mppi_t* h, const double x0[4], const mppi_scene* scene);

/* One MPPI iteration from state x0 (world coordinates) on the resident scene
 * (the second half of mppi_step); no host-to-device traffic besides the
 * kernel arguments.  MPPI_E_INVALID if no scene has been set. */
mppi_status mppi_step_resident(mppi_t* h, const double x0[4]);

/* One MPPI iteration of each of n planning instances in ONE persistent launch
 * (replayed as a captured HIP graph).  Instances may differ in K, T, scene
 * size and launch shape; each computes exactly the bits it computes alone,
 * because its lanes-per-sample shape and tile split depend only on its own
 * configuration.
 *   hs      [n] distinct handles that all enqueue on the same HIP stream
 *   x0s     [n][4] initial states (world coordinates)
 *   scenes  [n] scenes copied for this call, or NULL to use every handle's
 *           resident scene (mppi_set_scene); a batch does not change the
 *           handles' resident scenes
 * Asynchronous on that stream; results are read per handle as after
 * mppi_step.  Validation failures leave every handle unchanged. */
mppi_status mppi_step_batch(mppi_t* const* hs, const double* x0s, const mppi_scene* scenes,
                            int32_t n);

/* Wait for the handle's stream; returns the status of the last step.
 * mppi_sync, mppi_get_controls, mppi_get_state, mppi_get_iter_stats and
 * mppi_get_trajectory have the device write their results into a small
 * pinned host buffer of the handle, made by the first of them that reads
 * a result (mppi_sync reads one only once the handle has stepped);
 * MPPI_E_NOMEM if it cannot be made. */
mppi_status mppi_sync(mppi_t* h);

/* Copy U (the nominal controls, [T][2] = (a, delta)) into out; n >= 2T.
 * Synchronizes; returns the status of the last step. */
mppi_status mppi_get_controls(mppi_t* h, double* out, size_t n);

/* Replace U ([T][2], n >= 2T, finite). */
mppi_status mppi_set_controls(mppi_t* h, const double* U, size_t n);

/* Receding-horizon warm start (Alg. 1, shift of the input sequence):
 * U_t <- U_{t+steps} for t < T - steps, the remaining entries repeat the last
 * control.  0 <= steps. */
mppi_status mppi_shift(mppi_t* h, int32_t steps);

/* Checkpoint: U ([T][2], n >= 2T), iteration counter and seed. */
mppi_status mppi_get_state(mppi_t* h, double* U, size_t n, uint64_t* n_iter, uint64_t* seed);
/* Restore a checkpoint; the Philox stream continues bit-identically. */
mppi_status mppi_set_state(mppi_t* h, const double* U, size_t n, uint64_t n_iter);

/* Results of the last step (synchronize).  Costs S_k as float32 [K];
 * normalised weights as float64 [K] (with per-step weights: those of step 0,
 * formed from the float64 cost-to-go S_0,k); applied perturbations eps_eff
 * as float32 [T][K][2]; summary statistics. */
mppi_status mppi_get_costs(mppi_t* h, float* out, size_t n);
mppi_status mppi_get_weights(mppi_t* h, double* out, size_t n);
mppi_status mppi_get_noise(mppi_t* h, float* out, size_t n);

/* Per-step stage costs of the last step (cfg.per_step_weights = 1 only):
 * [T][K] float32, q_t,k on the state x_{t+1} of sample k; synchronises.
 * MPPI_E_INVALID for a short buffer or when per-step weights are off. */
mppi_status mppi_get_stage_costs(mppi_t* h, float* out, size_t n);

/* Steering angle delta0 [rad] of the next steps' initial state for the
 * 5-state model (cfg.model = 1; ignored otherwise).  Default 0; kept until
 * changed.  MPPI_E_INVALID if not finite. */
mppi_status mppi_set_steering(mppi_t* h, double delta0);

/* The optimal trajectory of Alg. 1 (the rollout after the update): from the
 * x0 of the last completed step, x*_{t+1} = F(x*_t, u*_t) (eq. (5), explicit
 * Euler) under the handle's current nominal controls u* (the smoothed
 * sequence when cfg.smoothing = 1), each control put through the noise check
 * with zero noise so that the trajectory respects the bounds and the speed
 * cap.  Computed in float64 on the device; synchronises the handle's stream.
 * states: [T+1][4] world-frame (x, y, yaw, v) -- [T+1][5] with the steering
 * angle for the 5-state model --, n_states >= columns (T+1);
 * controls: [T][2] applied (a, delta), n_controls >= 2T (either may be NULL).
 * MPPI_E_INVALID before the first step or for short buffers (nothing
 * written). */
mppi_status mppi_get_trajectory(mppi_t* h, double* states, size_t n_states, double* controls,
                                size_t n_controls);
mppi_status mppi_get_iter_stats(mppi_t* h, mppi_iter_stats* out);

/* Launch shape: lanes cooperating on one sample (1, 2, 4, 8 or 16), or 0 to
 * let the library pick from its tuning table. */
mppi_status mppi_set_lanes_per_sample(mppi_t* h, int32_t lanes);

/* LDS copy of each tile's applied perturbations for its weighted sums:
 * -1 (default) the tuning table's choice for the instance's shape, 0 never
 * (the sums read them back from L2), 1 whenever the copy fits the LDS.
 * Results are identical bit for bit. */
mppi_status mppi_set_staging(mppi_t* h, int32_t mode);

/* Compilation of the iteration kernel (the parallel rollout of Alg. 1,
 * Sec. III-A): -1 (default) the tuning table's choice for the instance's
 * shape, 0 the default register budget, 1 the variant compiled for five
 * waves per SIMD (instances with far more waves than the GPU holds at
 * once; at 8 and 16 lanes per sample, other shapes use 0).  Results are
 * identical bit for bit.  MPPI_E_INVALID for other values. */
mppi_status mppi_set_occupancy(mppi_t* h, int32_t mode);

/* Wave-level culling of the two scans of the stage cost (on by default):
 * waypoint chunks and obstacle circles that provably cannot change any
 * lane's tracking minimum or obstacle cost are skipped.  Results are
 * identical bit for bit; off (0) runs the full scans. */
mppi_status mppi_set_culling(mppi_t* h, int32_t on);

/* The HIP stream the handle enqueues on (as void*). */
mppi_status mppi_get_stream(mppi_t* h, void** stream);

/* Profiling: when on, every kernel of the handle is bracketed by HIP events
 * and its device time is accumulated; mppi_get_profile synchronizes and
 * returns the totals since the last reset (on = 1 resets them). */
mppi_status mppi_set_profiling(mppi_t* h, int32_t on);
mppi_status mppi_get_profile(mppi_t* h, mppi_profile* out);

/* ---- served replanning (continuous batching) -------------------------------
 * A server owns a table of vehicles and plans for them on one GPU.  Each
 * vehicle keeps its nominal controls U and its Philox iteration counter on
 * the device between requests; its first request starts from U = 0 and
 * every later request first shifts U by one step (the warm start of Alg. 1).
 * Requests are admitted in arrival order while their scratch memory (applied
 * noise, costs, partials: about 8 K T bytes) fits the HBM budget, at most one
 * request per vehicle is in flight, and whenever one of the server's streams
 * is idle every admissible request is launched as one batch; batches on
 * different streams overlap on the device.  All server calls are thread-safe. */

typedef struct mppi_server mppi_server_t;

typedef struct mppi_server_config {
    uint64_t hbm_budget_bytes; /* device scratch for requests in flight, >= 4096     */
    int32_t n_streams;         /* concurrent batches, 1..8                            */
    int32_t max_batch;         /* requests per launch, 1..4096                        */
    int32_t queue_cap;         /* queued + in-flight requests before MPPI_E_BUSY      */
    int32_t plain;             /* 1: one request at a time, no batching, no overlap   */
    double deadline_ms;        /* replanning period for the miss count (50 ms at the
                                  20 Hz of Sec. IV-D); 0: no count                    */
} mppi_server_config;

typedef struct mppi_server_stats {
    uint64_t submitted, completed, rejected, failed;
    uint64_t launches;         /* batches launched                                    */
    double mean_batch;         /* requests per batch                                  */
    double mean_ms, p50_ms, p99_ms, p999_ms, max_ms; /* completion - arrival          */
    uint64_t hbm_peak_bytes;   /* peak scratch in use                                 */
    int32_t max_queue;         /* peak queued + in-flight requests                    */
    uint64_t deadline_misses;  /* completed requests whose latency exceeded
                                  deadline_ms                                         */
} mppi_server_stats;

/* Open-loop load: request i of vehicle vid[i] from state x0[i] in scene
 * scenes[scene[i]], submitted at arrival_ns[i] after the start (arrivals
 * nondecreasing).  Latency is measured from the scheduled arrival. */
typedef struct mppi_replay_plan {
    int32_t n_requests;
    const int32_t* vid;           /* [n]                                             */
    const double* x0;             /* [n][4]                                          */
    const int32_t* scene;         /* [n] index into scenes                           */
    const mppi_scene* scenes;     /* [n_scenes]                                      */
    int32_t n_scenes;
    const uint64_t* arrival_ns;   /* [n] offsets from the start                      */
} mppi_replay_plan;

/* Clock of the arrival and completion stamps (steady, nanoseconds). */
uint64_t mppi_server_now_ns(void);
mppi_status mppi_server_create(const mppi_server_config* cfg, mppi_server_t** out);
/* Stops the scheduler after the launched batches finish; frees everything. */
mppi_status mppi_server_destroy(mppi_server_t* srv);
/* Add a vehicle with its planner configuration; MPPI_E_NOMEM if one of its
 * requests could never fit the budget.  Returns its id in *vid. */
mppi_status mppi_server_add_vehicle(mppi_server_t* srv, const mppi_config* cfg, int32_t* vid);
/* Queue a replanning request (inputs copied).  t_arrival_ns: arrival stamp
 * on the mppi_server_now_ns clock (0 = now).  ticket may be NULL (the result
 * is then discarded).  MPPI_E_BUSY when queue_cap requests are pending. */
mppi_status mppi_server_submit(mppi_server_t* srv, int32_t vid, const double x0[4],
                               const mppi_scene* scene, uint64_t t_arrival_ns, uint64_t* ticket);
/* MPPI_E_NOT_READY until the request completed; then copies its controls
 * ([T][2], n >= 2T; may be NULL), the completion stamp, forgets the ticket
 * and returns the request's status. */
mppi_status mppi_server_poll(mppi_server_t* srv, uint64_t ticket, double* controls, size_t n,
                             uint64_t* t_done_ns);
/* Block until no request is queued or in flight. */
mppi_status mppi_server_wait_idle(mppi_server_t* srv);
mppi_status mppi_server_get_stats(mppi_server_t* srv, mppi_server_stats* out);
mppi_status mppi_server_reset_stats(mppi_server_t* srv);
/* Checkpoint / restore of an idle vehicle: U [T][2], iteration counter and
 * the number of requests it has run (0 means the next one starts cold). */
mppi_status mppi_server_get_vehicle_state(mppi_server_t* srv, int32_t vid, double* U, size_t n,
                                          uint64_t* n_iter, uint64_t* requests);
mppi_status mppi_server_set_vehicle_state(mppi_server_t* srv, int32_t vid, const double* U,
                                          size_t n, uint64_t n_iter, uint64_t requests);
/* Run an open-loop load (blocks until every request completed); latency_ms
 * [n] receives completion - scheduled arrival (NaN for refused requests). */
mppi_status mppi_server_replay(mppi_server_t* srv, const mppi_replay_plan* plan,
                               double* latency_ms);

/* ---- allocation-free iteration ------------------------------------------- */

/* Largest scratch of one mppi_step_static call, in bytes (the library's
 * file-scope device array; every GPU it runs on holds one until the process
 * ends). */
#define MPPI_STATIC_SCRATCH_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory while they plan (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * one iteration with the work and the bits of mppi_step (scene staging, the
 * iteration kernel and the combine kernel at the launch shape mppi_step
 * picks), with no handle and no allocation.  Costs, applied perturbations,
 * tile partials, the staged scene and the device state live in one
 * file-scope device array of MPPI_STATIC_SCRATCH_BYTES per GPU, looked up
 * once per device; the call calls no hipMalloc, hipFree or other allocating
 * routine.
 *   cfg        configuration, validated as by mppi_create; the 4-state model
 *              only (model = 0)
 *   x0, scene  host arrays as for mppi_step (copied before the call returns)
 *   U          DEVICE pointer to the caller's [T][2] float64 controls, read
 *              and updated in place on hip_stream (U_t += sum_k w_k eps_eff)
 *   n_iter     iteration counter of the Philox stream; the caller keeps it
 *              and passes n, n + 1, ... (mppi_step keeps it in the handle)
 *   stats      optional DEVICE pointer, receives the iteration's statistics
 *              on hip_stream (status MPPI_E_NONFINITE, U unchanged, when no
 *              sample cost is finite)
 *   hip_stream hipStream_t to enqueue on (NULL: the null stream)
 * Asynchronous.  MPPI_E_INVALID (nothing enqueued) for a bad configuration,
 * scene or pointer, or when K x T x 8 bytes of perturbations plus the rest
 * exceed MPPI_STATIC_SCRATCH_BYTES (e.g. K = 8192, T = 100 needs 7.4 MB).
 * All calls on one GPU share its array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialized by the caller; calls in order on one stream
 * are safe. */
mppi_status mppi_step_static(const mppi_config* cfg, const double x0[4], const mppi_scene* scene,
                             double* U, uint64_t n_iter, mppi_iter_stats* stats,
                             void* hip_stream);

/* ---- Philox words as the rollout consumes them ---------------------------- */

/* Philox4x32-10 (Salmon et al., SC'11) of counters (k, j, n_lo, n_hi) for
 * k in [k0, k0+nk), j in [j0, j0+nj) under key = seed, computed on the
 * device by the same function the rollout uses.  out: [nk][nj][4] uint32,
 * n >= 4 nk nj.  Synchronous. */
mppi_status mppi_debug_philox(uint64_t seed, uint64_t n_iter, uint32_t k0, uint32_t nk,
                              uint32_t j0, uint32_t nj, uint32_t* out, size_t n);

/* ---- measurement helper ---------------------------------------------------- */

/* Plain device-to-device copy of `bytes` bytes (rounded down to 16), run
 * `reps` times by a simple streaming kernel on freshly allocated buffers:
 * the reference dispatch against which hardware traffic counters (bytes
 * fetched / written per dispatch) are calibrated.  Synchronous. */
mppi_status mppi_bench_copy(size_t bytes, int32_t reps);

/* ---- diagnostics ---------------------------------------------------------- */

const char* mppi_status_str(mppi_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char* mppi_last_error(void);
/* Library version string. */
const char* mppi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPPI_H */
