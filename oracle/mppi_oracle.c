/*
 * FP64 CPU oracle for one MPPI iteration (Testouri, Elghazaly, Frank,
 * "Towards a Safe Real-Time Motion Planning Framework for Autonomous Driving
 * Systems: A Model Predictive Path Integral Approach", arXiv 2308.01654).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load it; the product library never links,
 * calls or includes it, and it shares no code, header or table with that
 * library.
 *
 * What it computes (one iteration of Algorithm 1, the sampling, parallel
 * rollout, minimum-cost shift and weighted update, with the Section IV-C
 * costs restricted to tracking, speed, control effort and obstacles):
 *
 *   for every sample k (Alg. 1, "for m in parallel"):
 *     x <- x0, S_k <- 0
 *     for t = 0 .. T-1:
 *       eps        ~ N(0, diag(sigma^2))           Philox4x32-10 + Box-Muller
 *       u~         = clamp(U_t + eps)              the noise check of Sec. III-A
 *       eps_eff    = u~ - U_t
 *       x'         = F(x, u~)                      eq. (5), explicit Euler
 *       S_k       += w_track c_dist + w_speed c_speed + q_u + w_coll c_safe
 *       x <- x'
 *   S_min = min_k S_k                               Alg. 1, minimum step
 *   w_k   = exp(-(S_k - S_min)/lambda) / sum_j exp(-(S_j - S_min)/lambda)
 *   U_t  += sum_k w_k eps_eff[t][k]                 eq. (update-input)
 *
 * Readings of passages that are silent or garbled (each one is listed with
 * its justification in the design notes of the repository):
 *   - vehicle model: the 4-state kinematic bicycle (x, y, yaw, v) with
 *     controls (acceleration, steering angle); eq. (5) with the steering
 *     angle promoted to a control.  Explicit Euler, every right-hand side
 *     from the old state.
 *   - the running cost is evaluated on x_{t+1} for t = 0..T-1 and there is no
 *     separate terminal term (equal to the Sec. III cost sum up to a
 *     sample-independent constant, so weights and update are unchanged).
 *   - input cost q_u = w_effort (alpha eps^T eps + U^T eps + 1/2 U^T U),
 *     alpha = (gamma-1)/(2 gamma), evaluated with eps_eff (R = w_effort I).
 *   - one total cost S_k per sample is used in the weights (the minimum is
 *     taken over totals in Alg. 1).
 *   - the "noise check" clamps the perturbed control into
 *     [u_min, u_max], caps the acceleration so that v_{t+1} <= v_max, then
 *     re-applies a >= a_min.
 *   - c_dist = min_j ||P - W_j||^2 over all waypoints; v_ref is read at the
 *     closest waypoint (lowest index on exact ties).
 *   - obstacle distance d_obj is the minimum over ego circles e and obstacle
 *     circles c of ||P_e - O_c|| - r_c - r_e; O_c moves at constant velocity
 *     and is evaluated at time (t+1) dt; d_safe = d_safe_c v + d_safe_0;
 *     c_safe = max(d_safe - d_obj, 0)^2; no circles means c_safe = 0.
 *   - noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *     key = (seed_lo, seed_hi) and counter = (k, t/2, n_lo, n_hi); words
 *     (r0, r1) feed even t and (r2, r3) odd t; u = ((r >> 9) + 0.5) 2^-23
 *     (2^23 midpoints of (0, 1), every one exact in binary32 and binary64);
 *     Box-Muller (1958): rho = sqrt(-2 ln u1), z_a = rho cos(2 pi u2),
 *     z_d = rho sin(2 pi u2).
 *   - a non-finite S_k counts as +inf; if every S_k is non-finite the
 *     iteration fails and U is left unchanged.
 *   - the 5-state model of eq. (5) (cfg.model = 1): the state carries the
 *     steering angle delta (initial value cfg.steer0) and the second
 *     control is the steering rate omega, clamped to [u_min, u_max] of that
 *     control (+-omega_max) by the noise check; explicit Euler from the old
 *     state: theta' = theta + dt v tan(delta) / l, delta' = delta + dt omega.
 *   - per-step weights (cfg.per_step = 1): the update of U_t weights the
 *     samples by their cost-to-go S_{t,k} = sum_{s >= t} q_{s,k} (the
 *     eq. (update-input) form with S indexed by t), with its own minimum
 *     per t; the default uses one total per sample (S_{0,k}) for every t.
 *   - the other Sec. IV-C terms (zero weight unless configured):
 *     c_target = 1 when the step ends farther from the target point T_P
 *     than it started (squared distances compared), T_P being the last
 *     waypoint of the path; c_yaw = wrap(theta - theta_r)^2 with the
 *     difference wrapped into [-pi, pi) and theta_r the yaw of the closest
 *     waypoint; in the collision-only mode (object avoidance) c_safe_dist
 *     counts only when d_obj <= 0.
 *
 * The last steps of Algorithm 1 (optional, cfg.smoothing = 1):
 *   u*    = SavitzkyGolay(U)                        eq. (sg): the 5-point
 *           window (-3, 12, 17, 12, -3)/35; beyond either end of the
 *           sequence the end value is repeated (the paper leaves the ends
 *           open).  The smoothed sequence replaces U, so the warm start of
 *           the next iteration shifts u* as Alg. 1 does.
 *   x*_0 = x0, x*_{t+1} = F(x*_t, u*_t)             the optimal rollout; each
 *           u*_t goes through the same noise check as the samples (with zero
 *           noise), so the output trajectory {x*, u*} respects the bounds.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so mppi_oracle.c -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_cfg {
    int32_t K, T;
    double dt, wheelbase, lambda, gamma;
    double sigma_a, sigma_d;
    double a_min, a_max, d_min, d_max;
    double v_max;
    double w_track, w_speed, w_effort, w_coll;
    double d_safe_c, d_safe_0;
    int32_t n_ego;
    double ego_r;
    double ego_off[4];
    uint64_t seed;
    int32_t smoothing;  /* 1: Savitzky-Golay smoothing ends the iteration */
    double w_target;    /* weight of c_target (Sec. IV-C) */
    double w_yaw;       /* weight of c_yaw (Sec. IV-C) */
    int32_t collision_only; /* 1: c_safe_dist only when an object is hit */
    int32_t model;      /* 0: 4-state, steering-angle control; 1: eq. (5) 5-state */
    double steer0;      /* initial steering angle of the 5-state model */
    int32_t per_step;   /* 1: weights per step from the cost-to-go S_t,k */
} orc_cfg;

enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_NONFINITE = -4 };

/* Threads the parallel loops of this oracle use. */
int orc_max_threads(void) { return omp_get_max_threads(); }
/* Thread count of the parallel loops over samples (the host baseline times
 * the oracle on all cores and on one); n < 1 leaves it unchanged. */
void orc_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
}

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, Section 4.2 / Table 2 constants).
 * One round: (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
 *                               hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
 * the key is bumped by the Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
static const uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PH_M0 * c0;
        uint64_t p1 = (uint64_t)PH_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PH_W0; k1 += PH_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox of n counters ctr[n][4] under one key; out[n][4]. */
void orc_philox_batch(const uint32_t* ctr, int64_t n, const uint32_t key[2], uint32_t* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* The two 32-bit words that drive step t of sample k at iteration n. */
static void noise_words(uint64_t seed, uint64_t n, int k, int t, uint32_t w[2])
{
    uint32_t ctr[4] = { (uint32_t)k, (uint32_t)(t >> 1), (uint32_t)n, (uint32_t)(n >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    if ((t & 1) == 0) { w[0] = r[0]; w[1] = r[1]; }
    else              { w[0] = r[2]; w[1] = r[3]; }
}

/* uniform in (0,1): ((r >> 9) + 1/2) / 2^23 -- the 2^23 midpoints of a
 * uniform grid; each needs 24 significant bits, so it is exact in binary32 */
double orc_uniform(uint32_t r)
{
    return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Box-Muller: two uniforms -> two independent standard normals */
void orc_box_muller(double u1, double u2, double z[2])
{
    const double two_pi = 6.283185307179586476925286766559;
    double rho = sqrt(-2.0 * log(u1));
    z[0] = rho * cos(two_pi * u2);
    z[1] = rho * sin(two_pi * u2);
}

/* Raw Gaussian perturbation (before the noise check) of step t of sample k. */
void orc_noise(const orc_cfg* c, uint64_t n, int k, int t, double eps[2])
{
    uint32_t w[2];
    double z[2];
    noise_words(c->seed, n, k, t, w);
    orc_box_muller(orc_uniform(w[0]), orc_uniform(w[1]), z);
    eps[0] = c->sigma_a * z[0];
    eps[1] = c->sigma_d * z[1];
}

static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* Noise check: the applied control for nominal U_t, raw noise eps, speed v. */
void orc_apply_limits(const orc_cfg* c, const double U[2], const double eps[2], double v,
                      double applied[2])
{
    double a = clampd(U[0] + eps[0], c->a_min, c->a_max);
    double cap = (c->v_max - v) / c->dt;   /* keeps v + dt a <= v_max */
    if (a > cap) a = cap;
    if (a < c->a_min) a = c->a_min;        /* the braking bound wins */
    applied[0] = a;
    applied[1] = clampd(U[1] + eps[1], c->d_min, c->d_max);
}

/* Eq. (5), explicit Euler with every right-hand side from the old state.
 * States have 5 entries (x, y, theta, v, delta); with the 4-state model the
 * steering angle is the control u[1] and x[4] is carried unchanged. */
void orc_dynamics(const orc_cfg* c, const double x[5], const double u[2], double xn[5])
{
    double dt = c->dt;
    double delta = c->model ? x[4] : u[1];
    xn[0] = x[0] + dt * x[3] * cos(x[2]);
    xn[1] = x[1] + dt * x[3] * sin(x[2]);
    xn[2] = x[2] + dt * x[3] * tan(delta) / c->wheelbase;
    xn[3] = x[3] + dt * u[0];
    xn[4] = c->model ? x[4] + dt * u[1] : x[4];
}

/* c_dist and the reference yaw and speed of the closest waypoint (Sec. IV-C). */
static void tracking(const double* wp, int n_wp, const double P[2], double* c_dist,
                     double* yaw_ref, double* v_ref)
{
    double best = INFINITY;
    int bj = 0;
    for (int j = 0; j < n_wp; ++j) {
        double dx = P[0] - wp[4 * j + 0];
        double dy = P[1] - wp[4 * j + 1];
        double d = dx * dx + dy * dy;
        if (d < best) { best = d; bj = j; }
    }
    *c_dist = best;
    *yaw_ref = wp[4 * bj + 2];
    *v_ref = wp[4 * bj + 3];
}

/* An angle difference brought into [-pi, pi). */
static double wrap_angle(double d)
{
    const double pi = 3.14159265358979323846;
    return d - 2.0 * pi * floor((d + pi) / (2.0 * pi));
}

/* d_obj of Sec. IV-C over ego circles and (moving) obstacle circles. */
static double object_distance(const orc_cfg* c, const double* circ, int n_c,
                              const double x[4], double tau)
{
    double d_obj = INFINITY;
    double ct = cos(x[2]), st = sin(x[2]);
    for (int e = 0; e < c->n_ego; ++e) {
        double ex = x[0] + c->ego_off[e] * ct;
        double ey = x[1] + c->ego_off[e] * st;
        for (int i = 0; i < n_c; ++i) {
            const double* o = circ + 5 * i;
            double ox = o[0] + tau * o[3];
            double oy = o[1] + tau * o[4];
            double d = sqrt((ex - ox) * (ex - ox) + (ey - oy) * (ey - oy)) - o[2] - c->ego_r;
            if (d < d_obj) d_obj = d;
        }
    }
    return d_obj;
}

/* Stage cost of Sec. III (input part) and Sec. IV-C (state part) evaluated on
 * the new state x' reached from x (previous state) with nominal U_t and
 * applied perturbation e.  parts: c_dist, c_speed, q_u, c_safe, c_target,
 * c_yaw. */
double orc_stage_cost(const orc_cfg* c, const double* wp, int n_wp, const double* circ, int n_c,
                      const double xn[4], const double U[2], const double e[2], int t,
                      const double xp[4], double parts[6])
{
    double P[2] = { xn[0], xn[1] };
    double c_dist, yaw_ref, v_ref;
    tracking(wp, n_wp, P, &c_dist, &yaw_ref, &v_ref);
    double c_speed = (xn[3] - v_ref) * (xn[3] - v_ref);
    const double tpx = wp[4 * (n_wp - 1) + 0], tpy = wp[4 * (n_wp - 1) + 1];
    double dn = (xn[0] - tpx) * (xn[0] - tpx) + (xn[1] - tpy) * (xn[1] - tpy);
    double dp = (xp[0] - tpx) * (xp[0] - tpx) + (xp[1] - tpy) * (xp[1] - tpy);
    double c_target = dn > dp ? 1.0 : 0.0;
    double dyaw = wrap_angle(xn[2] - yaw_ref);
    double c_yaw = dyaw * dyaw;
    double alpha = (c->gamma - 1.0) / (2.0 * c->gamma);
    double q_u = c->w_effort * (alpha * (e[0] * e[0] + e[1] * e[1])
                                + (U[0] * e[0] + U[1] * e[1])
                                + 0.5 * (U[0] * U[0] + U[1] * U[1]));
    double tau = (double)(t + 1) * c->dt;
    double d_obj = object_distance(c, circ, n_c, xn, tau);
    double d_safe = c->d_safe_c * xn[3] + c->d_safe_0;
    double g = d_safe - d_obj;
    double c_safe = g > 0.0 ? g * g : 0.0;
    if (c->collision_only && !(d_obj <= 0.0)) c_safe = 0.0;
    if (parts) {
        parts[0] = c_dist; parts[1] = c_speed; parts[2] = q_u; parts[3] = c_safe;
        parts[4] = c_target; parts[5] = c_yaw;
    }
    return c->w_track * c_dist + c->w_target * c_target + c->w_yaw * c_yaw +
           c->w_speed * c_speed + q_u + c->w_coll * c_safe;
}

static int cfg_ok(const orc_cfg* c, int n_wp, int n_c)
{
    if (c->K < 1 || c->T < 1 || !(c->dt > 0) || !(c->lambda > 0) || !(c->wheelbase > 0)) return 0;
    if (!(c->gamma > 0) || c->n_ego < 0 || c->n_ego > 4 || n_wp < 1 || n_c < 0) return 0;
    if (!(c->sigma_a >= 0) || !(c->sigma_d >= 0)) return 0;
    return 1;
}

/*
 * Rollouts of all K samples (Alg. 1, the parallel loop).
 *   U       [T][2] nominal controls
 *   eps_in  optional [T][K][2]: applied perturbations to use instead of
 *           sampling (the applied control is then U_t + eps_in, no clamp)
 *   S_out   [K] total costs
 *   eps_out optional [T][K][2] applied perturbations eps_eff
 */
int orc_rollout(const orc_cfg* c, const double x0[4], const double* wp, int n_wp,
                const double* circ, int n_c, const double* U, uint64_t n_iter,
                const double* eps_in, double* S_out, double* eps_out, double* q_out)
{
    if (!cfg_ok(c, n_wp, n_c)) return ORC_E_INVALID;
    const int K = c->K, T = c->T;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        double x[5] = { x0[0], x0[1], x0[2], x0[3], c->steer0 };
        double S = 0.0;
        for (int t = 0; t < T; ++t) {
            const double* Ut = U + 2 * t;
            double e[2], u[2];
            if (eps_in) {
                e[0] = eps_in[((size_t)t * K + k) * 2 + 0];
                e[1] = eps_in[((size_t)t * K + k) * 2 + 1];
                u[0] = Ut[0] + e[0];
                u[1] = Ut[1] + e[1];
            } else {
                double raw[2];
                orc_noise(c, n_iter, k, t, raw);
                orc_apply_limits(c, Ut, raw, x[3], u);
                e[0] = u[0] - Ut[0];
                e[1] = u[1] - Ut[1];
            }
            if (eps_out) {
                eps_out[((size_t)t * K + k) * 2 + 0] = e[0];
                eps_out[((size_t)t * K + k) * 2 + 1] = e[1];
            }
            double xn[5];
            orc_dynamics(c, x, u, xn);
            const double q = orc_stage_cost(c, wp, n_wp, circ, n_c, xn, Ut, e, t, x, NULL);
            if (q_out) q_out[(size_t)t * K + k] = q;
            S += q;
            memcpy(x, xn, sizeof x);
        }
        S_out[k] = S;
    }
    return ORC_OK;
}

/*
 * Rollouts of the selected samples ks[0..nk) only (their noise is the noise
 * of those sample indices in the full iteration).  eps_in / eps_out are
 * [T][nk][2]; S_out is [nk].  Used for sampled checks of large iterations.
 */
int orc_rollout_samples(const orc_cfg* c, const double x0[4], const double* wp, int n_wp,
                        const double* circ, int n_c, const double* U, uint64_t n_iter,
                        const int32_t* ks, int nk, const double* eps_in, double* S_out,
                        double* eps_out)
{
    if (!cfg_ok(c, n_wp, n_c) || nk < 0) return ORC_E_INVALID;
    const int T = c->T;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nk; ++i) {
        const int k = ks[i];
        double x[5] = { x0[0], x0[1], x0[2], x0[3], c->steer0 };
        double S = 0.0;
        for (int t = 0; t < T; ++t) {
            const double* Ut = U + 2 * t;
            double e[2], u[2];
            if (eps_in) {
                e[0] = eps_in[((size_t)t * nk + i) * 2 + 0];
                e[1] = eps_in[((size_t)t * nk + i) * 2 + 1];
                u[0] = Ut[0] + e[0];
                u[1] = Ut[1] + e[1];
            } else {
                double raw[2];
                orc_noise(c, n_iter, k, t, raw);
                orc_apply_limits(c, Ut, raw, x[3], u);
                e[0] = u[0] - Ut[0];
                e[1] = u[1] - Ut[1];
            }
            if (eps_out) {
                eps_out[((size_t)t * nk + i) * 2 + 0] = e[0];
                eps_out[((size_t)t * nk + i) * 2 + 1] = e[1];
            }
            double xn[5];
            orc_dynamics(c, x, u, xn);
            S += orc_stage_cost(c, wp, n_wp, circ, n_c, xn, Ut, e, t, x, NULL);
            memcpy(x, xn, sizeof x);
        }
        S_out[i] = S;
    }
    return ORC_OK;
}

/* Deterministic rollout of one control sequence (no noise); states [T+1][4],
 * stage costs [T] and their parts [T][6] (c_dist, c_speed, q_u, c_safe,
 * c_target, c_yaw). */
int orc_simulate(const orc_cfg* c, const double x0[4], const double* wp, int n_wp,
                 const double* circ, int n_c, const double* U, const double* eps,
                 double* states, double* costs, double* parts)
{
    if (!cfg_ok(c, n_wp, n_c)) return ORC_E_INVALID;
    const int ns = 4 + (c->model ? 1 : 0);  /* state columns written */
    double x[5] = { x0[0], x0[1], x0[2], x0[3], c->steer0 };
    memcpy(states, x, ns * sizeof(double));
    for (int t = 0; t < c->T; ++t) {
        double e[2] = { eps ? eps[2 * t] : 0.0, eps ? eps[2 * t + 1] : 0.0 };
        double u[2] = { U[2 * t] + e[0], U[2 * t + 1] + e[1] };
        double xn[5];
        orc_dynamics(c, x, u, xn);
        costs[t] = orc_stage_cost(c, wp, n_wp, circ, n_c, xn, U + 2 * t, e, t, x,
                                  parts ? parts + 6 * t : NULL);
        memcpy(states + ns * (t + 1), xn, ns * sizeof(double));
        memcpy(x, xn, sizeof x);
    }
    return ORC_OK;
}

/* Minimum-cost shift and normalised weights (Alg. 1 and eq. (update-input)).
 * Non-finite costs count as +inf.  Writes w[K], S_min, log Z (Z of the
 * shifted exponentials). */
int orc_weights(const double* S, int K, double lambda, double* w, double* s_min, double* log_z)
{
    if (K < 1 || !(lambda > 0)) return ORC_E_INVALID;
    double m = INFINITY;
    for (int k = 0; k < K; ++k)
        if (isfinite(S[k]) && S[k] < m) m = S[k];
    if (!isfinite(m)) return ORC_E_NONFINITE;
    double Z = 0.0;
    for (int k = 0; k < K; ++k) {
        double om = isfinite(S[k]) ? exp(-(S[k] - m) / lambda) : 0.0;
        w[k] = om;
        Z += om;
    }
    for (int k = 0; k < K; ++k) w[k] /= Z;
    if (s_min) *s_min = m;
    if (log_z) *log_z = log(Z);
    return ORC_OK;
}

/* U_t += sum_k w_k eps[t][k]  (eq. (update-input)); eps is [T][K][2]. */
void orc_update(double* U, int T, int K, const double* w, const double* eps)
{
    for (int t = 0; t < T; ++t) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < K; ++k) {
            s0 += w[k] * eps[((size_t)t * K + k) * 2 + 0];
            s1 += w[k] * eps[((size_t)t * K + k) * 2 + 1];
        }
        U[2 * t + 0] += s0;
        U[2 * t + 1] += s1;
    }
}

/* Eq. (sg): out[t] = (-3 u[t-2] + 12 u[t-1] + 17 u[t] + 12 u[t+1] - 3 u[t+2]) / 35
 * for each control, with u[i] = u[0] for i < 0 and u[i] = u[T-1] for i >= T. */
void orc_sg_smooth(const double* U, int T, double* out)
{
    static const double z[5] = {-3.0, 12.0, 17.0, 12.0, -3.0};
    for (int t = 0; t < T; ++t) {
        for (int d = 0; d < 2; ++d) {
            double acc = 0.0;
            for (int j = -2; j <= 2; ++j) {
                int i = t + j;
                if (i < 0) i = 0;
                if (i > T - 1) i = T - 1;
                acc += z[j + 2] * U[2 * i + d];
            }
            out[2 * t + d] = acc / 35.0;
        }
    }
}

/* The optimal rollout of Alg. 1 from x0 under the controls Us [T][2]: each
 * control passes the noise check with zero noise; states [T+1][4] ([T+1][5]
 * with the steering angle for the 5-state model) and the applied controls
 * [T][2] are returned. */
void orc_optimal_trajectory(const orc_cfg* c, const double x0[4], const double* Us,
                            double* states, double* applied)
{
    static const double zero[2] = {0.0, 0.0};
    const int ns = 4 + (c->model ? 1 : 0);
    double x[5] = { x0[0], x0[1], x0[2], x0[3], c->steer0 }, xn[5];
    memcpy(states, x, ns * sizeof(double));
    for (int t = 0; t < c->T; ++t) {
        orc_apply_limits(c, Us + 2 * t, zero, x[3], applied + 2 * t);
        orc_dynamics(c, x, applied + 2 * t, xn);
        memcpy(states + ns * (t + 1), xn, ns * sizeof(double));
        memcpy(x, xn, sizeof x);
    }
}

/* Per-step update: from stage costs q [T][K], the cost-to-go
 * S_{t,k} = q_{t,k} + S_{t+1,k} (summed from the last step back), then for
 * every t the weights of S_{t,.} with their own minimum and
 * U_t += sum_k w_{t,k} eps[t][k].  Optional outputs: S_tk [T][K], w0 [K]
 * (the weights of t = 0), the minimum and log Z of t = 0.  Fails without
 * touching U if some t has no finite cost-to-go. */
int orc_update_per_step(double* U, int T, int K, const double* q, const double* eps,
                        double lambda, double* S_tk, double* w0, double* s_min, double* log_z)
{
    double* S = S_tk ? S_tk : (double*)malloc((size_t)T * K * sizeof(double));
    double* w = (double*)malloc((size_t)T * K * sizeof(double));
    double* mins = (double*)malloc((size_t)T * 2 * sizeof(double));
    int rc = (S && w && mins) ? ORC_OK : ORC_E_INVALID;
    for (int k = 0; rc == ORC_OK && k < K; ++k) {
        double acc = 0.0;
        for (int t = T - 1; t >= 0; --t) {
            acc += q[(size_t)t * K + k];
            S[(size_t)t * K + k] = acc;
        }
    }
    for (int t = 0; rc == ORC_OK && t < T; ++t)
        rc = orc_weights(S + (size_t)t * K, K, lambda, w + (size_t)t * K, mins + 2 * t,
                         mins + 2 * t + 1);
    if (rc == ORC_OK) {
        for (int t = 0; t < T; ++t) {
            double s0 = 0.0, s1 = 0.0;
            for (int k = 0; k < K; ++k) {
                s0 += w[(size_t)t * K + k] * eps[((size_t)t * K + k) * 2 + 0];
                s1 += w[(size_t)t * K + k] * eps[((size_t)t * K + k) * 2 + 1];
            }
            U[2 * t + 0] += s0;
            U[2 * t + 1] += s1;
        }
        if (w0) memcpy(w0, w, (size_t)K * sizeof(double));
        if (s_min) *s_min = mins[0];
        if (log_z) *log_z = mins[1];
    }
    if (!S_tk) free(S);
    free(w);
    free(mins);
    return rc;
}

/* One full iteration; U is updated in place only on success.
 * Optional outputs: S[K], w[K], eps[T][K][2]. */
int orc_iteration(const orc_cfg* c, const double x0[4], const double* wp, int n_wp,
                  const double* circ, int n_c, double* U, uint64_t n_iter,
                  double* S_out, double* w_out, double* eps_out, double* s_min, double* log_z)
{
    if (!cfg_ok(c, n_wp, n_c)) return ORC_E_INVALID;
    size_t K = (size_t)c->K, T = (size_t)c->T;
    double* S = S_out ? S_out : (double*)malloc(K * sizeof(double));
    double* w = w_out ? w_out : (double*)malloc(K * sizeof(double));
    double* e = eps_out ? eps_out : (double*)malloc(T * K * 2 * sizeof(double));
    double* q = c->per_step ? (double*)malloc(T * K * sizeof(double)) : NULL;
    int rc = (S && w && e && (q || !c->per_step)) ? ORC_OK : ORC_E_INVALID;
    if (rc == ORC_OK) rc = orc_rollout(c, x0, wp, n_wp, circ, n_c, U, n_iter, NULL, S, e, q);
    if (rc == ORC_OK && c->per_step) {
        rc = orc_update_per_step(U, c->T, c->K, q, e, c->lambda, NULL, w, s_min, log_z);
    } else {
        if (rc == ORC_OK) rc = orc_weights(S, c->K, c->lambda, w, s_min, log_z);
        if (rc == ORC_OK) orc_update(U, c->T, c->K, w, e);
    }
    free(q);
    if (rc == ORC_OK && c->smoothing) {
        double* sm = (double*)malloc(T * 2 * sizeof(double));
        if (!sm) {
            rc = ORC_E_INVALID;
        } else {
            orc_sg_smooth(U, c->T, sm);
            memcpy(U, sm, T * 2 * sizeof(double));
            free(sm);
        }
    }
    if (!S_out) free(S);
    if (!w_out) free(w);
    if (!eps_out) free(e);
    return rc;
}
