// HIP kernels (gfx950 / CDNA4) for one MPPI iteration of the planner of
// arXiv 2308.01654 (Algorithm 1, noise generation through the input update,
// with the costs of Sec. III and Sec. IV-C).
//
// An iteration is two launches.  The iteration kernel (k_batch) gives each
// workgroup a tile of samples; G lanes ("lanes per sample", 1..16)
// cooperate on one sample:
//
//   phase 1  rollout.  The horizon is walked in blocks of G steps.  Lane r of
//            a group draws the Philox/Box-Muller perturbation of step t0+r
//            and applies the control bounds; the speed before each step
//            (the noise check's speed cap) and the heading and position of
//            eq. (5) come from prefix sums over the G lanes, so each lane
//            holds the state reached at its own step.  Each lane then
//            evaluates the (expensive) stage cost of its own step: the
//            waypoint scan and the ego-circle x obstacle-circle distances,
//            culled per wave.  Costs are Kahan-summed per lane and combined
//            per sample in float64.  Applied perturbations are stored
//            time-major [T][K] as float2 (and kept in LDS for phase 2).
//   phase 2  tile partials.  Tile minimum m_b, then (float64)
//            omega_i = exp(-(S_i - m_b)/lambda), Z_b = sum omega_i and, for
//            every (t, control) column, the float64 sum of the products
//            omega_i * eps_eff[t][i] over the tile.
//   phase 3  (tiles above kDirect only) a fixed-shape tree merges tiles
//            until kDirect nodes remain.
//
// The combine kernel (k_combine) merges the node rows in node order with the
// rescale exp(-(m_b - m)/lambda) and updates U in float64: U_t += N_t / Z
// (eq. (update-input)); it bumps the iteration counter and records S_min,
// log Z and the effective sample size.  Every order of summation is fixed,
// so results do not depend on which workgroup finishes first.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "mppi_internal.hpp"

namespace mppi_impl {

// Accesses to the instance's global arrays through pointers typed as global
// memory: the descriptor's pointers are generic, and generic (flat)
// accesses also count against the counter that scalar and LDS loads wait
// on, so every wait for a scalar candidate load would also wait for the
// rollout's in-flight global loads and stores.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p)
{
    return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ T ld_g(const T* p, size_t i)
{
    return as_global(p)[i];
}
__device__ __forceinline__ float2 ld_g(const float2* p, size_t i)
{
    const f2v v = as_global(reinterpret_cast<const f2v*>(p))[i];
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_g(const float4* p, size_t i)
{
    const f4v v = as_global(reinterpret_cast<const f4v*>(p))[i];
    return make_float4(v.x, v.y, v.z, v.w);
}
// Element i (below 2^32 bytes from p) of a small array: a 32-bit offset from
// a uniform base, without 64-bit address arithmetic per lane.
__device__ __forceinline__ float2 ld_g32(const float2* p, unsigned i)
{
    const f2v v = *(gptr<const f2v>)((gptr<const char>)(const char*)p + i * 8u);
    return make_float2(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void st_g(T* p, size_t i, T v)
{
    as_global(p)[i] = v;
}
__device__ __forceinline__ void st_g(float2* p, size_t i, float2 v)
{
    f2v w;
    w.x = v.x;
    w.y = v.y;
    as_global(reinterpret_cast<f2v*>(p))[i] = w;
}
// A store written through the XCD's L2 to the device's coherence point (a
// relaxed agent-scope atomic store; its bits are those of the plain store).
// Each XCD has its own write-back L2, so the release at the end of a kernel
// writes back every line still dirty there before a dependent kernel can
// start; data written through is already out, and that release has less to
// do.  Used for the applied perturbations, written once and read by the
// host (and the next launch only through another kernel).
__device__ __forceinline__ void st_wt(float2* p, size_t i, float2 v)
{
    const unsigned long long bits = (unsigned long long)__float_as_uint(v.x) |
                                    ((unsigned long long)__float_as_uint(v.y) << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p) + i, bits, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 S-box (two 32x32->64 multiplies, xor with the other half and the key)
// with a Weyl-sequence key schedule.
// ----------------------------------------------------------------------------
// (v_bitop3 with truth table 0x96 is the three-input exclusive or of gfx950)
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96),
                       (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96),
                       (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Gaussian perturbation (before the noise check) of step t of sample k at
// iteration n: counter (k, t/2, n_lo, n_hi); words (r0, r1) for even t and
// (r2, r3) for odd t; u = ((r >> 9) + 1/2) 2^-23 is exact in float32;
// Box-Muller with the angle taken in revolutions by the hardware sin/cos.
__device__ __forceinline__ uint4 noise_words(const InstDesc& d, int k, int pair,
                                             unsigned long long n)
{
    return philox4x32_10(make_uint4((uint32_t)k, (uint32_t)pair, (uint32_t)n, (uint32_t)(n >> 32)),
                         d.key0, d.key1);
}

__device__ __forceinline__ float2 noise_from_words(const InstDesc& d, uint32_t ra, uint32_t rb)
{
    const float u1 = ((float)(ra >> 9) + 0.5f) * 0x1p-23f;
    const float u2 = ((float)(rb >> 9) + 0.5f) * 0x1p-23f;
    // -2 ln u1 = -2 ln(2) log2(u1)
    const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    return make_float2(d.sig_a * rho * __builtin_amdgcn_cosf(u2),
                       d.sig_d * rho * __builtin_amdgcn_sinf(u2));
}

__device__ __forceinline__ float2 draw_noise(const InstDesc& d, int k, int t,
                                             unsigned long long n)
{
    const uint4 r = noise_words(d, k, t >> 1, n);
    return noise_from_words(d, (t & 1) ? r.z : r.x, (t & 1) ? r.w : r.y);
}

struct Lds {
    float4* c_pv;
    float4* wp_box;
    float2* wp_xy;
    double* red;
    float* wp_vref;
    float* wp_yaw;
    float* c_rr;
    double* omega; // [spb] the tile's float64 exponential weights
    float* eps;  // [2T][spb + 1]: column 2t + c, sample j at (2t + c)(spb + 1) + j
    float* qs;   // [T][spb + 1] stage costs (per-step weights)
    double* ss;  // [T][spb + 1] cost-to-go (per-step weights), rows padded by one
};

__device__ __forceinline__ Lds lds_bind(unsigned char* base, const LdsLayout& L)
{
    Lds s;
    s.c_pv = reinterpret_cast<float4*>(base + L.c_pv);
    s.wp_box = reinterpret_cast<float4*>(base + L.wp_box);
    s.wp_xy = reinterpret_cast<float2*>(base + L.wp_xy);
    s.red = reinterpret_cast<double*>(base + L.red);
    s.wp_vref = reinterpret_cast<float*>(base + L.wp_vref);
    s.wp_yaw = reinterpret_cast<float*>(base + L.wp_yaw);
    s.c_rr = reinterpret_cast<float*>(base + L.c_rr);
    s.omega = reinterpret_cast<double*>(base + L.omega);
    s.eps = reinterpret_cast<float*>(base + L.eps);
    s.qs = reinterpret_cast<float*>(base + L.qs);
    s.ss = reinterpret_cast<double*>(base + L.ss);
    return s;
}

// Closest-waypoint update over chunk ch (kChunk consecutive waypoints, padded
// with points at infinity): the chunk is read with 16-byte LDS reads (two
// points each) and its distances are compared in index order, so ties keep
// the lowest index.
__device__ __forceinline__ void scan_chunk(const Lds& s, int ch, float x, float y, float& best,
                                           int& bj)
{
    const float4* p = reinterpret_cast<const float4*>(s.wp_xy) + ch * kChunkQ;
#pragma unroll
    for (int u = 0; u < kChunkQ; ++u) {
        const float4 q = p[u];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float dx = x - (h ? q.z : q.x);
            const float dy = y - (h ? q.w : q.y);
            const float dd = fmaf(dy, dy, dx * dx);
            if (dd < best) {
                best = dd;
                bj = ch * kChunk + 2 * u + h;
            }
        }
    }
}

// Clearance between the ego circles (centres ex, ey) and obstacle circle p
// at time tau: min_e ||P_e - O|| - (r_c + r_ego), with the square root taken
// once, of the smallest squared distance (the root is monotone).
template <int NE>
__device__ __forceinline__ float circle_gap(const float (&ex)[NE > 0 ? NE : 1],
                                            const float (&ey)[NE > 0 ? NE : 1], const float4& p,
                                            float rr, float tau)
{
    const float ox = fmaf(tau, p.z, p.x);
    const float oy = fmaf(tau, p.w, p.y);
    float m2 = 0.0f;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const float dx = ex[e] - ox;
        const float dy = ey[e] - oy;
        const float d2 = fmaf(dy, dy, dx * dx);
        m2 = e == 0 ? d2 : fminf(m2, d2);
    }
    return __builtin_amdgcn_sqrtf(m2) - rr;
}

// The Sec. IV-C terms beyond tracking, speed and obstacles, each skipped at
// zero weight: c_target = 1 when the step from (xp, yp) to (x, y) ends
// farther from the target point (the last waypoint) -- the sign of
// |P - T|^2 - |P_prev - T|^2 = (P - P_prev).(P + P_prev - 2 T) -- and c_yaw,
// the heading th minus the yaw of closest waypoint bj, wrapped into
// [-pi, pi), squared.
// The waypoint arrays are read from wxy / wyaw: the tile's LDS copy, or
// (GLOBAL) the scene in global memory -- the same values either way.
template <bool GLOBAL>
__device__ __forceinline__ float extra_terms(const InstDesc& d, const float2* wxy,
                                             const float* wyaw, int bj, float x, float y,
                                             float th, float xp, float yp)
{
    float e = 0.0f;
    if (d.w_target != 0.0f) {
        const float2 tp = GLOBAL ? ld_g(wxy, d.n_wp - 1) : wxy[d.n_wp - 1];
        const float dx = x - xp, dy = y - yp;
        const float sx = (x - tp.x) + (xp - tp.x), sy = (y - tp.y) + (yp - tp.y);
        e = fmaf(d.w_target, fmaf(dx, sx, dy * sy) > 0.0f ? 1.0f : 0.0f, e);
    }
    if (d.w_yaw != 0.0f) {
        float dyaw = th - (GLOBAL ? ld_g(wyaw, bj) : wyaw[bj]);
        dyaw -= 6.28318530717958647692f *
                floorf((dyaw + 3.14159265358979323846f) * 0.15915494309189533577f);
        e = fmaf(d.w_yaw, dyaw * dyaw, e);
    }
    return e;
}

// Obstacle cost from the clearance d_obj and the safety distance ds; in the
// collision-only mode it counts only when an object is hit (d_obj <= 0).
__device__ __forceinline__ float safe_cost(const InstDesc& d, float ds, float d_obj)
{
    const float g = ds - d_obj;
    return (g > 0.0f && (!d.coll_only || d_obj <= 0.0f)) ? g * g : 0.0f;
}

// Stage cost on the state reached at step t (Sec. III input cost, Sec. IV-C
// tracking, speed and obstacle costs).  Every lane of the wave runs the same
// waypoint and circle loops, so the LDS reads are broadcasts.
template <int NE>
__device__ __forceinline__ float stage_cost(const InstDesc& d, const Lds& s, float x, float y,
                                            float c, float sn, float v, float Ua, float Ud,
                                            float ea, float ed, int t, float th, float xp,
                                            float yp)
{
    // c_dist = min_j ||P - W_j||^2; reference speed of the closest waypoint
    float best = INFINITY;
    int bj = 0;
    for (int ch = 0; ch * kChunk < d.n_wp; ++ch) scan_chunk(s, ch, x, y, best, bj);
    const float ext = extra_terms<false>(d, s.wp_xy, s.wp_yaw, bj, x, y, th, xp, yp);
    const float dv = v - s.wp_vref[bj];
    // q_u = w_effort (alpha eps.eps + U.eps + U.U / 2)
    const float q = d.w_effort * (d.alpha * fmaf(ea, ea, ed * ed) + fmaf(Ua, ea, Ud * ed) +
                                  0.5f * fmaf(Ua, Ua, Ud * Ud));
    float cost = fmaf(d.w_track, best, fmaf(d.w_speed, dv * dv, q));
    if (NE > 0) {
        float ex[NE > 0 ? NE : 1], ey[NE > 0 ? NE : 1];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            ex[e] = fmaf(d.ego_off[e], c, x);
            ey[e] = fmaf(d.ego_off[e], sn, y);
        }
        const float tau = (float)(t + 1) * d.dt;
        float d_obj = INFINITY;
        for (int i = 0; i < d.n_c; ++i) {
            const float4 p = s.c_pv[i];
            const float rr = s.c_rr[i];
            d_obj = fminf(d_obj, circle_gap<NE>(ex, ey, p, rr, tau));
        }
        cost = fmaf(d.w_coll, safe_cost(d, fmaf(d.d_safe_c, v, d.d_safe_0), d_obj), cost);
    }
    return cost + ext;
}

// ----------------------------------------------------------------------------
// Wave-level culling helpers.
// ----------------------------------------------------------------------------

// Order-preserving map of float32 onto int32 (its own inverse): for non-NaN
// values the integer order of the keys is the float order, so wave minima and
// maxima run on integer DPP operations without NaN canonicalisation.
__device__ __forceinline__ int fkey(float f)
{
    const int b = __builtin_bit_cast(int, f);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float fkey_inv(int k)
{
    return __builtin_bit_cast(float, k ^ ((k >> 31) & 0x7fffffff));
}
constexpr int kKeyPosInf = 0x7f800000;          // fkey(+inf)
constexpr int kKeyNegInf = (int)0x807fffffu;    // fkey(-inf)

// Cross-lane move by a DPP control; lanes outside row_mask receive `idv`,
// the identity of the reduction that consumes the value.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int idv, int x)
{
    return __builtin_amdgcn_update_dpp(idv, x, CTRL, ROW_MASK, 0xf, false);
}
constexpr int kIntMax = 0x7fffffff;
constexpr int kIntMin = (int)0x80000000u;

// Prefix sums inside aligned groups of G lanes (G <= 16, so a group lies in
// one DPP row): the inclusive sum (or maximum) up to lane r of the group,
// the value of lane r - 1 (0 for the first lane), and the group's last
// lane's value.  With G = 16 a group is a whole row, and a row shift by N
// already gives lanes r < N nothing from another group (bound_ctrl reads 0;
// without it the lane keeps the identity passed as the old value), so no
// lane mask is needed.
template <int N>
__device__ __forceinline__ float dpp_shr(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + N, 0xf, 0xf, true));
}
template <int G>
__device__ __forceinline__ float seg_scan(float v, int r)
{
    if (G == 16) {
        v += dpp_shr<1>(v);
        v += dpp_shr<2>(v);
        v += dpp_shr<4>(v);
        v += dpp_shr<8>(v);
        return v;
    }
    if (G >= 2) { const float u = dpp_shr<1>(v); v += r >= 1 ? u : 0.0f; }
    if (G >= 4) { const float u = dpp_shr<2>(v); v += r >= 2 ? u : 0.0f; }
    if (G >= 8) { const float u = dpp_shr<4>(v); v += r >= 4 ? u : 0.0f; }
    return v;
}
template <int G>
__device__ __forceinline__ float seg_scan_max(float v, int r)
{
    if (G == 16) {
        // on order-preserving integer keys (non-NaN floats): one DPP max per
        // stage; lanes r < N keep the identity
        int k = fkey(v);
        k = max(k, dpp_i<0x111>(kIntMin, k));
        k = max(k, dpp_i<0x112>(kIntMin, k));
        k = max(k, dpp_i<0x114>(kIntMin, k));
        k = max(k, dpp_i<0x118>(kIntMin, k));
        return fkey_inv(k);
    }
    if (G >= 2) { const float u = dpp_shr<1>(v); v = r >= 1 ? fmaxf(v, u) : v; }
    if (G >= 4) { const float u = dpp_shr<2>(v); v = r >= 2 ? fmaxf(v, u) : v; }
    if (G >= 8) { const float u = dpp_shr<4>(v); v = r >= 4 ? fmaxf(v, u) : v; }
    return v;
}
template <int G>
__device__ __forceinline__ float seg_prev(float incl, int r)
{
    if (G == 1) return 0.0f;
    const float u = dpp_shr<1>(incl);
    if (G == 16) return u;
    return r >= 1 ? u : 0.0f;
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
// The group's last lane's value in every lane of the group, by DPP: quad
// permutes for groups of 2 and 4, row broadcasts (row_newbcast) of lanes 7
// and 15 for groups of 8 and 16.
template <int G>
__device__ __forceinline__ float group_last(float v, int gbase)
{
    (void)gbase;
    if (G == 1) return v;
    if (G == 2) return dpp_f<0xF5>(v);   // quad_perm [1, 1, 3, 3]
    if (G == 4) return dpp_f<0xFF>(v);   // quad_perm [3, 3, 3, 3]
    const float hi = dpp_f<0x15F>(v);    // row_newbcast:15
    if (G == 16) return hi;
    const float lo = dpp_f<0x157>(v);    // row_newbcast:7
    return (threadIdx.x & 8) ? hi : lo;
}

// Wave-wide reduction stages: swap neighbours and quad halves, mirror inside
// half rows and rows (every lane then holds its row's result), broadcast lane
// 15 into rows 1 and 3 and lane 31 into rows 2 and 3; lane 63 ends with the
// result over all 64 lanes.  Five independent reductions (two minima, three
// maxima) advance stage by stage so that their DPP latencies overlap.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ void red5_stage(int& a, int& b, int& c, int& e, int& f)
{
    a = min(a, dpp_i<CTRL, ROW_MASK>(kIntMax, a));
    b = min(b, dpp_i<CTRL, ROW_MASK>(kIntMax, b));
    c = max(c, dpp_i<CTRL, ROW_MASK>(kIntMin, c));
    e = max(e, dpp_i<CTRL, ROW_MASK>(kIntMin, e));
    f = max(f, dpp_i<CTRL, ROW_MASK>(kIntMin, f));
}

__device__ __forceinline__ int lane63(int x) { return __builtin_amdgcn_readlane(x, 63); }

// Bounding box of the positions of the lanes with inc set, and the largest
// safety distance among them (keys of +-inf for an empty set).
struct WaveBox {
    float xlo, xhi, ylo, yhi, dsmax;
};

__device__ __forceinline__ WaveBox wave_box(bool inc, float x, float y, float ds)
{
    int a = inc ? fkey(x) : kKeyPosInf;
    int b = inc ? fkey(y) : kKeyPosInf;
    int c = inc ? fkey(x) : kKeyNegInf;
    int e = inc ? fkey(y) : kKeyNegInf;
    int f = inc ? fkey(ds) : kKeyNegInf;
    red5_stage<0xB1>(a, b, c, e, f);       // quad_perm [1,0,3,2]
    red5_stage<0x4E>(a, b, c, e, f);       // quad_perm [2,3,0,1]
    red5_stage<0x141>(a, b, c, e, f);      // row_half_mirror
    red5_stage<0x140>(a, b, c, e, f);      // row_mirror
    red5_stage<0x142, 0xa>(a, b, c, e, f); // row_bcast:15
    red5_stage<0x143, 0xc>(a, b, c, e, f); // row_bcast:31
    WaveBox w;
    w.xlo = fkey_inv(lane63(a));
    w.ylo = fkey_inv(lane63(b));
    w.xhi = fkey_inv(lane63(c));
    w.yhi = fkey_inv(lane63(e));
    w.dsmax = fkey_inv(lane63(f));
    return w;
}

// Wave minimum and maximum of non-negative floats (their bit patterns are
// ordered), advanced stage by stage together.
__device__ __forceinline__ void wave_minmax_nonneg(float vmin, float vmax, float& omin,
                                                   float& omax)
{
    int a = __builtin_bit_cast(int, vmin);
    int b = __builtin_bit_cast(int, vmax);
    a = min(a, dpp_i<0xB1>(kIntMax, a));
    b = max(b, dpp_i<0xB1>(kIntMin, b));
    a = min(a, dpp_i<0x4E>(kIntMax, a));
    b = max(b, dpp_i<0x4E>(kIntMin, b));
    a = min(a, dpp_i<0x141>(kIntMax, a));
    b = max(b, dpp_i<0x141>(kIntMin, b));
    a = min(a, dpp_i<0x140>(kIntMax, a));
    b = max(b, dpp_i<0x140>(kIntMin, b));
    a = min(a, dpp_i<0x142, 0xa>(kIntMax, a));
    b = max(b, dpp_i<0x142, 0xa>(kIntMin, b));
    a = min(a, dpp_i<0x143, 0xc>(kIntMax, a));
    b = max(b, dpp_i<0x143, 0xc>(kIntMin, b));
    omin = __builtin_bit_cast(float, lane63(a));
    omax = __builtin_bit_cast(float, lane63(b));
}

// Wave minimum of non-negative floats.
__device__ __forceinline__ float wave_min_nonneg(float v)
{
    int a = __builtin_bit_cast(int, v);
    a = min(a, dpp_i<0xB1>(kIntMax, a));
    a = min(a, dpp_i<0x4E>(kIntMax, a));
    a = min(a, dpp_i<0x141>(kIntMax, a));
    a = min(a, dpp_i<0x140>(kIntMax, a));
    a = min(a, dpp_i<0x142, 0xa>(kIntMax, a));
    a = min(a, dpp_i<0x143, 0xc>(kIntMax, a));
    return __builtin_bit_cast(float, lane63(a));
}

// Read-only scene data fetched with wave-uniform addresses: the constant
// address space makes these scalar loads.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ const_ptr<float> as_const(const T* p)
{
    return (const_ptr<float>)(reinterpret_cast<const float*>(p));
}

// Element i of a float4 array seen as floats.
__device__ __forceinline__ float4 ld4(const_ptr<float> p, int i)
{
    return make_float4(p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]);
}

// Smallest squared distance from (x, y) to the 8 points of a waypoint chunk
// (padded at the end with points at infinity).
__device__ __forceinline__ float chunk_min(const float4 (&q)[kChunkQ], float x, float y)
{
    float m = INFINITY;
#pragma unroll
    for (int u = 0; u < kChunkQ; ++u) {
        const float dx0 = x - q[u].x, dy0 = y - q[u].y;
        const float dx1 = x - q[u].z, dy1 = y - q[u].w;
        m = fminf(m, fmaf(dy0, dy0, dx0 * dx0));
        m = fminf(m, fmaf(dy1, dy1, dx1 * dx1));
    }
    return m;
}

// Scans the chunks whose bits are set in m (ascending, kChunkTrip per memory
// round trip, read from global memory with scalar loads): best = smallest
// squared distance, bch = first chunk that attains it.  A short last group
// repeats its first chunk: the repeat cannot be strictly smaller, so nothing
// changes, and the group's loads are issued together without a branch
// between them.
__device__ __forceinline__ void scan_chunks(const_ptr<float> wp4, int base, unsigned long long m,
                                            float x, float y, float& best, int& bch)
{
    while (m) {
        int c[kChunkTrip];
        c[0] = base + __builtin_ctzll(m);
        m &= m - 1;
#pragma unroll
        for (int i = 1; i < kChunkTrip; ++i) {
            c[i] = m ? base + __builtin_ctzll(m) : c[0];
            m &= m - 1;
        }
        float4 q[kChunkTrip][kChunkQ];
#pragma unroll
        for (int i = 0; i < kChunkTrip; ++i)
#pragma unroll
            for (int u = 0; u < kChunkQ; ++u) q[i][u] = ld4(wp4, c[i] * kChunkQ + u);
#pragma unroll
        for (int i = 0; i < kChunkTrip; ++i) {
            const float mi = chunk_min(q[i], x, y);
            if (mi < best) {
                best = mi;
                bch = c[i];
            }
        }
    }
}

// Index of the first point of chunk bch at squared distance best from
// (x, y): together with scan_chunks this is the lowest index attaining the
// minimum, as in the sequential scan (index 0 when no distance is finite).
__device__ __forceinline__ int chunk_argmin(const float2* wxy, int bch, float best, float x,
                                            float y)
{
    if (!(best < INFINITY)) return 0;
    const float4* p = reinterpret_cast<const float4*>(wxy) + bch * kChunkQ;
    int bj = bch * kChunk;
#pragma unroll
    for (int u = kChunkQ - 1; u >= 0; --u) {
        const float4 q = ld_g(p, u);
#pragma unroll
        for (int h = 1; h >= 0; --h) {
            const float dx = x - (h ? q.z : q.x);
            const float dy = y - (h ? q.w : q.y);
            if (fmaf(dy, dy, dx * dx) == best) bj = bch * kChunk + 2 * u + h;
        }
    }
    return bj;
}

// Per-lane culling data that stays in registers through the rollout: the
// bounding box of chunk `lane` and obstacle circle `lane` (the first 64 of
// each; larger scenes read the rest from global memory).
struct LaneCull {
    float4 box;   // (x_lo, x_hi, y_lo, y_hi) of chunk lane; empty past the end
    float4 cpv;   // circle lane (x, y, vx, vy); at infinity past the end
    float crr;    // its radius plus the ego radius
};

// The stage cost of stage_cost, with the two scans restricted to what can
// matter for this wave (all 64 lanes call it; `act` lanes are evaluated).
// The result is bit-identical to the full scans:
//  * waypoints: two bounds on every lane's nearest distance^2 -- the
//    smallest over chunks of the largest distance^2 between the wave's
//    position box and the chunk box, and the largest over lanes of the
//    lane's own distance^2 (same arithmetic as the scan) to three waypoints
//    ahead of its previous closest chunk; UB is the smaller.  A chunk whose
//    smallest distance^2 to the wave box exceeds UB (with a relative margin
//    far above float32 rounding) holds no candidate, and the remaining
//    chunks are scanned in index order, so ties resolve exactly as in the
//    full scan;
//  * circles: a circle whose centre, swept over the wave's time range, stays
//    farther than max(d_safe) + r_c + r_ego from the box of the wave's ego
//    circles cannot make c_safe positive for any lane, so it is skipped.
// Lanes whose position or safety distance is not finite are left out of the
// wave box: their own cost is not finite under either scan.  The scene is
// read from global memory (wave-uniform candidates through the scalar
// cache); own_d2 is the lane's squared distance to the nearest of three
// waypoints ahead of its previous closest chunk (+inf without one), formed
// by the caller, and vref0 the reference speed of waypoint 0.
template <int NE>
__device__ __forceinline__ float stage_cost_culled(const InstDesc& d, float own_d2,
                                                   float vref0, const LaneCull& lc,
                                                   bool vref_uniform, bool act,
                                                   int& seed, float x, float y,
                                                   float c, float sn, float v, float Ua, float Ud,
                                                   float ea, float ed, int t, int t_lo, int t_hi,
                                                   float th, float xp, float yp)
{
    const int lane = threadIdx.x & 63;
    const float ds = fmaf(d.d_safe_c, v, d.d_safe_0);
    const bool inc = act && isfinite(x) && isfinite(y) && isfinite(ds);
    const WaveBox wb = wave_box(inc, x, y, ds);

    // ---- waypoints
    const int n_ch = (d.n_wp + kChunk - 1) / kChunk;
    const const_ptr<float> wp4 = as_const(d.wp_xy);
    float best = INFINITY;
    int bch = 0;
    auto far2 = [&](const float4& b) {  // largest distance^2, wave box to chunk box
        const float dx = fmaxf(wb.xhi - b.x, b.y - wb.xlo);
        const float dy = fmaxf(wb.yhi - b.z, b.w - wb.ylo);
        return fmaf(dy, dy, dx * dx);
    };
    auto near2 = [&](const float4& b) {  // smallest distance^2, wave box to chunk box
        const float gx = fmaxf(fmaxf(b.x - wb.xhi, wb.xlo - b.y), 0.0f);
        const float gy = fmaxf(fmaxf(b.z - wb.yhi, wb.ylo - b.w), 0.0f);
        return fmaf(gy, gy, gx * gx);
    };
    // A second bound from the lane itself: its distance^2 to three waypoints
    // ahead of the chunk it was closest to at its previous step (seed), the
    // largest over the lanes of the wave; lanes without a seed give +inf.
    const float own = inc ? own_d2 : 0.0f;
    if (n_ch <= 64) {
        float ub_box, ub_own;
        wave_minmax_nonneg(far2(lc.box), own, ub_box, ub_own);
        const float thr = fmaf(fminf(ub_box, ub_own), 1.0f + 1e-5f, 1e-6f);
        scan_chunks(wp4, 0, __ballot(near2(lc.box) <= thr), x, y, best, bch);
    } else {
        const float4 empty = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        float ub, ub_own;
        wave_minmax_nonneg(far2(lc.box), own, ub, ub_own);
        ub = fminf(ub, ub_own);
        for (int base = 64; base < n_ch; base += 64)
            ub = fminf(ub, wave_min_nonneg(far2(base + lane < n_ch ? ld_g(d.wp_box, base + lane) : empty)));
        const float thr = fmaf(ub, 1.0f + 1e-5f, 1e-6f);
        scan_chunks(wp4, 0, __ballot(near2(lc.box) <= thr), x, y, best, bch);
        for (int base = 64; base < n_ch; base += 64) {
            const float4 b = base + lane < n_ch ? ld_g(d.wp_box, base + lane) : empty;
            scan_chunks(wp4, base, __ballot(near2(b) <= thr), x, y, best, bch);
        }
    }
    if (best < INFINITY) seed = bch;
    // the closest index, needed for its reference speed (unless every
    // waypoint has the same one) and for its yaw
    const bool need_idx = !vref_uniform || d.w_yaw != 0.0f;
    const int bj = need_idx ? chunk_argmin(d.wp_xy, bch, best, x, y) : 0;
    const float vref = vref_uniform ? vref0 : ld_g(d.wp_vref, bj);
    const float ext = extra_terms<true>(d, d.wp_xy, d.wp_yaw, bj, x, y, th, xp, yp);
    const float dv = v - vref;
    const float q = d.w_effort * (d.alpha * fmaf(ea, ea, ed * ed) + fmaf(Ua, ea, Ud * ed) +
                                  0.5f * fmaf(Ua, Ua, Ud * Ud));
    float cost = fmaf(d.w_track, best, fmaf(d.w_speed, dv * dv, q));

    // ---- obstacle circles
    if (NE > 0) {
        float ex[NE > 0 ? NE : 1], ey[NE > 0 ? NE : 1];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            ex[e] = fmaf(d.ego_off[e], c, x);
            ey[e] = fmaf(d.ego_off[e], sn, y);
        }
        const float exlo = wb.xlo - d.ego_ext, exhi = wb.xhi + d.ego_ext;
        const float eylo = wb.ylo - d.ego_ext, eyhi = wb.yhi + d.ego_ext;
        const float tau_lo = (float)(t_lo + 1) * d.dt;
        const float tau_hi = (float)(t_hi + 1) * d.dt;
        const float tau = (float)(t + 1) * d.dt;
        auto close = [&](const float4& p, float rr) {
            const float xa = fmaf(tau_lo, p.z, p.x), xb = fmaf(tau_hi, p.z, p.x);
            const float ya = fmaf(tau_lo, p.w, p.y), yb = fmaf(tau_hi, p.w, p.y);
            const float gx = fmaxf(fmaxf(fminf(xa, xb) - exhi, exlo - fmaxf(xa, xb)), 0.0f);
            const float gy = fmaxf(fmaxf(fminf(ya, yb) - eyhi, eylo - fmaxf(ya, yb)), 0.0f);
            // collision-only: only circles that can reach an ego circle matter
            const float lim = (d.coll_only ? 0.0f : wb.dsmax) + rr + 0.01f;
            return lim > 0.0f && fmaf(gy, gy, gx * gx) < lim * lim;
        };
        const const_ptr<float> cpv = as_const(d.c_pv);
        const const_ptr<float> crr = as_const(d.c_rr);
        float d_obj = INFINITY;
        for (int base = 0; base < d.n_c; base += 64) {
            bool need;
            if (base == 0) {
                need = close(lc.cpv, lc.crr);
            } else {
                need = base + lane < d.n_c && close(ld_g(d.c_pv, base + lane), ld_g(d.c_rr, base + lane));
            }
            unsigned long long m = __ballot(need);
            while (m) {
                // four candidates per round trip, loads issued together; a
                // short last group repeats its first candidate (the minimum
                // is unchanged)
                int idx[4];
                idx[0] = base + __builtin_ctzll(m);
                m &= m - 1;
#pragma unroll
                for (int u = 1; u < 4; ++u) {
                    idx[u] = m ? base + __builtin_ctzll(m) : idx[0];
                    m &= m - 1;
                }
                float4 p[4];
                float rr[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    p[u] = ld4(cpv, idx[u]);
                    rr[u] = crr[idx[u]];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) d_obj = fminf(d_obj, circle_gap<NE>(ex, ey, p[u], rr[u], tau));
            }
        }
        cost = fmaf(d.w_coll, safe_cost(d, ds, d_obj), cost);
    }
    return cost + ext;
}

// A float64 value of another lane by DPP (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// A float64 value of one lane, wave-uniform (two lane reads into scalar
// registers).
__device__ __forceinline__ double lane_d(double v, int lane)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Butterfly reductions over the 64 lanes of a wave (every lane active; every
// lane ends with the same value): lane pairs and quad halves by quad
// permutes; then, each quad holding one value, the half-row mirror pairs
// each quad with the other quad of its half-row, and the row mirror each
// half-row with the other half; the four row values, read into scalar
// registers, are combined as (row 0 with row 1) with (row 2 with row 3) --
// the value the cross-row butterfly gives in every lane.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

__device__ __forceinline__ double wave_min(double v)
{
    v = fmin(v, dpp_d<0xB1>(v));
    v = fmin(v, dpp_d<0x4E>(v));
    v = fmin(v, dpp_d<0x141>(v));
    v = fmin(v, dpp_d<0x140>(v));
    return fmin(fmin(lane_d(v, 0), lane_d(v, 16)), fmin(lane_d(v, 32), lane_d(v, 48)));
}

// v plus the value of the lane 16 (32) apart, the same in both lanes of the
// pair.  With both operands equal, the gfx950 permlane swap leaves each lane
// its own value in one result and its partner's in the other (which is
// which depends on the lane), so their sum is the pair's sum either way.
__device__ __forceinline__ double add_lanes_16_apart(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __builtin_bit_cast(double, ((long long)hi[0] << 32) | (long long)lo[0]);
    const double y = __builtin_bit_cast(double, ((long long)hi[1] << 32) | (long long)lo[1]);
    return x + y;
}
__device__ __forceinline__ double add_lanes_32_apart(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __builtin_bit_cast(double, ((long long)hi[0] << 32) | (long long)lo[0]);
    const double y = __builtin_bit_cast(double, ((long long)hi[1] << 32) | (long long)lo[1]);
    return x + y;
}

// M5: the 5-state model of eq. (5) -- the steering angle is part of the state
// and the second control is the steering rate.
template <int G, int NE, bool M5>
__device__ __forceinline__ void iteration_tile(const InstDesc& d, int tile, unsigned char* smem)
{
    const int tid = threadIdx.x;
    constexpr int SPB = kBlock / G;  // samples per tile
    const int T = d.T;
    const int K = d.K;
    const LdsLayout L = lds_layout(d.n_wp, d.n_c, T, SPB, d.eps_stage, d.per_step, !d.cull);
    const Lds s = lds_bind(smem, L);

    // The culled scans read the scene from global memory, so the rollout
    // starts at once; the full scans (no culling) read a copy in LDS.
    if (!d.cull) {
        for (int i = tid; i < d.n_c; i += kBlock) {
            s.c_pv[i] = ld_g(d.c_pv, i);
            s.c_rr[i] = ld_g(d.c_rr, i);
        }
        const int n_wp_pad = (d.n_wp + kChunk - 1) / kChunk * kChunk;
        for (int i = tid; i < n_wp_pad; i += kBlock) {
            // padding points at infinity are never the closest
            s.wp_xy[i] = ld_g(d.wp_xy, i);
            if (i < d.n_wp) {
                s.wp_vref[i] = ld_g(d.wp_vref, i);
                s.wp_yaw[i] = ld_g(d.wp_yaw, i);
            }
        }
        // (x_lo, x_hi, y_lo, y_hi) of every chunk, formed with the scene
        for (int c = tid; c * kChunk < d.n_wp; c += kBlock) s.wp_box[c] = ld_g(d.wp_box, c);
    }
    // the controls sampled around, kept for the smoothing combine
    if (d.smooth && tile == 0) {
        double* keep = d.partials + (size_t)d.n_tiles * partial_stride(T, d.per_step);
        for (int i = tid; i < 2 * T; i += kBlock) st_g(keep, i, ld_g(d.U, i));
    }
    const unsigned long long n_iter = ld_g(&d.st->n_iter, 0);
    // one reference speed for every waypoint: the closest index is not needed
    const bool vref_uniform = ld_g(d.scene_flags, 0) != 0;
    const float vref0 = as_const(d.wp_vref)[0];
    if (!d.cull) __syncthreads();

    // ---------------------------------------------------------------- phase 1
    const int grp = tid / G;
    const int r = tid % G;
    const int k_base = tile * SPB;
    const int k = k_base + grp;
    const bool valid = k < K;
    const int kk = valid ? k : K - 1;  // idle groups replay the last sample

    LaneCull lc;
    {
        const int lane = tid & 63;
        const int n_ch = (d.n_wp + kChunk - 1) / kChunk;
        lc.box = lane < n_ch ? ld_g(d.wp_box, lane) : make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        lc.cpv = lane < d.n_c ? ld_g(d.c_pv, lane) : make_float4(INFINITY, INFINITY, 0.0f, 0.0f);
        lc.crr = lane < d.n_c ? ld_g(d.c_rr, lane) : 0.0f;
    }
    float x = d.px0, y = d.py0, th = d.th0, v = d.v0;
    float delta = d.steer0;  // steering angle (5-state model only)
    float S = 0.0f, comp = 0.0f;  // Kahan pair of this lane's steps
    int seed = -1;                // closest chunk at this lane's previous step
    const int gbase = tid & ~(G - 1);  // first lane of this sample's group
    uint4 held = make_uint4(0u, 0u, 0u, 0u);  // Philox words kept for the next block
    // A horizon that is not a whole number of blocks starts with the partial
    // block (its leading lanes own no step), where the samples are still
    // close together and the culled scans are short, rather than ending with
    // it, where they have spread the most.  Kept even so that Philox step
    // pairs stay within a lane pair.
    const int rem = T % G;
    const int t_first = (rem != 0 && (rem & 1) == 0) ? rem - G : 0;
    // the nominal control of the lane's step (float64 in global memory),
    // fetched one block ahead
    double ua_next = ld_g(d.U, 2 * min(max(t_first + r, 0), T - 1));
    double ud_next = ld_g(d.U, 2 * min(max(t_first + r, 0), T - 1) + 1);
    int blk = 0;
    for (int t0 = t_first; t0 < T; t0 += G, ++blk) {
        // Where two waves share a SIMD, the one in the earlier block issues
        // first (wave priority 3 in blocks 0-1, 2 in 2-3, 1 in 4-5, then 0),
        // so that the pair tends to finish together instead of leaving the
        // later one to run alone at the end.
        if (d.wave_prio) {
            switch (min(blk >> 1, 3)) {
            case 0: __builtin_amdgcn_s_setprio(3); break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            case 2: __builtin_amdgcn_s_setprio(1); break;
            default: __builtin_amdgcn_s_setprio(0); break;
            }
        }
        const int tm = t0 + r;
        const float2 Um = make_float2((float)ua_next, (float)ud_next);
        if (t0 + G < T) {
            const int tn = min(max(t0 + G + r, 0), T - 1);
            ua_next = ld_g(d.U, 2 * tn);
            ud_next = ld_g(d.U, 2 * tn + 1);
        }
        // the lane's waypoints ahead of its previous closest chunk (the
        // culling's own bound), fetched before they are needed
        float2 sw[3];
        if (d.cull) {
            const int sb = max(seed, 0) * kChunk;
#pragma unroll
            for (int u = 0; u < 3; ++u) sw[u] = ld_g32(d.wp_xy, (unsigned)min(sb + (u + 1) * kSeedAhead, d.n_wp - 1));
        }
        const bool lead = tm < 0;  // before the horizon: no step, no increment
        // The lane's step within the block, opaque to the compiler so that the
        // per-step "own step" tests stay in the loop as vector compares
        // instead of G hoisted scalar masks (which exhaust the SGPRs).
        int rb = r;
        asm volatile("" : "+v"(rb));
        const int tc = min(max(tm, 0), T - 1);
        // This lane's step: perturbation, the state-independent part of the
        // noise check (control bounds) and -- for the steering-angle control --
        // its tangent.  With the 5-state model the second control is the
        // steering rate.
        // One Philox call gives the words of two consecutive steps.  With
        // G >= 2 lanes per sample the calls of two blocks are made together
        // in the first of them: lane 2i holds step pair i of that block and
        // lane 2i + 1 pair i of the next, and each lane takes its step's two
        // words from itself or its neighbour (quad-permute DPP).  Lanes
        // outside the horizon draw the words of their own (unused) steps.
        float2 em;
        if (G == 1) {
            em = draw_noise(d, kk, tc, n_iter);
        } else {
            const bool second = (blk & 1) != 0;
            if (!second) held = noise_words(d, kk, t0 / 2 + ((r & 1) ? G / 2 : 0) + (r >> 1), n_iter);
            uint32_t ra, rb;
            if (!second) {  // odd lanes take the odd-step words of the even lane below
                const uint32_t nz = (uint32_t)dpp_i<0xA0>(0, (int)held.z);
                const uint32_t nw = (uint32_t)dpp_i<0xA0>(0, (int)held.w);
                ra = (r & 1) ? nz : held.x;
                rb = (r & 1) ? nw : held.y;
            } else {        // even lanes take the even-step words of the odd lane above
                const uint32_t nx = (uint32_t)dpp_i<0xF5>(0, (int)held.x);
                const uint32_t ny = (uint32_t)dpp_i<0xF5>(0, (int)held.y);
                ra = (r & 1) ? held.z : nx;
                rb = (r & 1) ? held.w : ny;
            }
            em = noise_from_words(d, ra, rb);
        }
        const float a0m = fminf(fmaxf(Um.x + em.x, d.a_min), d.a_max);
        const float dlm = fminf(fmaxf(Um.y + em.y, d.d_min), d.d_max);
        const float tnm = M5 ? dlm : __tanf(dlm);
        // Speed before the own step.  The noise check caps the acceleration
        // so that v <= v_max and applies the braking bound last.  With
        // a_min <= 0 and the speed at the block start within v_max the
        // braking bound cannot bind (the cap (v_max - v)/dt is >= 0 >= a_min),
        // and the capped recursion v_{i+1} = min(v_i + dt a_i, v_max) has the
        // closed form
        //   v_r = min(v_0 + S_r, v_max + S_r - max_{1<=k<=r} S_k),
        // S_k = sum_{j<k} dt a_j: a prefix sum and a prefix maximum over the G
        // lanes.  Otherwise (a_min > 0, where the braking bound lifts the speed
        // above v_max whenever the cap falls below a_min, or a wave with a
        // sample above v_max) the G lanes run the recursion step by step
        // (accelerations exchanged PF at a time), each keeping the speed
        // before its own step.  Steps past the horizon (last block) are run
        // too; the lanes that own them are inactive.  Lanes before it (first
        // block) add zero increments, which leave the closed form unchanged
        // (their prefix sums equal v_0 <= v_max's).
        float vr = v;
        if (!(d.a_min > 0.0f) && __ballot(v > d.v_max) == 0ull) {
            const float sincl = seg_scan<G>(lead ? 0.0f : d.dt * a0m, r);
            const float sr = seg_prev<G>(sincl, r);
            const float qr = seg_scan_max<G>(r >= 1 ? sr : -INFINITY, r);
            vr = fminf(v + sr, d.v_max + (sr - qr));
        } else {
            constexpr int PF = G < 4 ? G : 4;
            float apf[PF];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i % PF == 0) {
#pragma unroll
                    for (int u = 0; u < PF; ++u)
                        apf[u] = G > 1 ? __shfl(a0m, gbase + i + u, 64) : a0m;
                }
                vr = i == rb ? v : vr;
                if (t0 + i >= 0) {
                    float a = fminf(apf[i % PF], (d.v_max - v) * d.inv_dt);
                    a = fmaxf(a, d.a_min);
                    v = fmaf(d.dt, a, v);
                }
            }
        }
        // the own step's applied acceleration (noise check: speed cap,
        // braking bound last) and the speed after it; the block ends at the
        // last lane's
        float ma = fminf(a0m, (d.v_max - vr) * d.inv_dt);
        ma = fmaxf(ma, d.a_min);
        const float mv = fmaf(d.dt, ma, vr);
        v = group_last<G>(mv, gbase);
        // Eq. (5), explicit Euler: given the speeds, heading and position are
        // sums of per-step increments, formed by prefix sums over the G lanes
        // of the group (each lane adds its own step's increment).  With the
        // 5-state model the heading turns with the steering angle before the
        // step, itself the sum of the applied rates.
        const float vdt = lead ? 0.0f : vr * d.dt;
        float tn = tnm;
        float ddel_blk = 0.0f;
        if (M5) {
            const float dincl = seg_scan<G>(lead ? 0.0f : d.dt * tnm, r);
            tn = __tanf(delta + seg_prev<G>(dincl, r));
            ddel_blk = group_last<G>(dincl, gbase);
        }
        const float thincl = seg_scan<G>(vdt * d.inv_L * tn, r);
        const float thb = th + seg_prev<G>(thincl, r);  // heading before the own step
        const float mth = th + thincl;                  // and after it
        const float xincl = seg_scan<G>(vdt * __cosf(thb), r);
        const float yincl = seg_scan<G>(vdt * __sinf(thb), r);
        const float mx = x + xincl, my = y + yincl;
        // position before this lane's step (for c_target): the previous
        // lane's position after its step, the block start for the first
        float pxp = 0.0f, pyp = 0.0f;
        if (d.w_target != 0.0f) {
            pxp = x + seg_prev<G>(xincl, r);
            pyp = y + seg_prev<G>(yincl, r);
        }
        // the state at the end of the block (the last lane's), for the next
        x += group_last<G>(xincl, gbase);
        y += group_last<G>(yincl, gbase);
        th += group_last<G>(thincl, gbase);
        if (M5) delta += ddel_blk;
        const float mc = __cosf(mth), ms = __sinf(mth);
        const float mUa = Um.x, mUd = Um.y;
        const float mea = ma - Um.x, med = dlm - Um.y;
        const bool act = !lead && tm < T;
        // the culling's own bound (consumes the waypoint loads of the block
        // start before the store below enters the vector-memory counter)
        float own_d2 = INFINITY;
        if (d.cull && seed >= 0) {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const float dx = mx - sw[u].x;
                const float dy = my - sw[u].y;
                own_d2 = fminf(own_d2, fmaf(dy, dy, dx * dx));
            }
        }
        // The applied perturbation is stored now, before the stage cost: the
        // store then retires during the scans instead of holding up the next
        // block's first wait on the vector-memory counter (loads and stores
        // share it and complete in order).
        if (act) {
            if (valid) st_wt(d.eps, (size_t)tm * K + k, make_float2(mea, med));
            if (L.eps_staged) {
                s.eps[(2 * tm) * (SPB + 1) + grp] = mea;
                s.eps[(2 * tm + 1) * (SPB + 1) + grp] = med;
            }
        }
        float q = 0.0f;
        if (d.cull)
            q = stage_cost_culled<NE>(d, own_d2, vref0, lc, vref_uniform, act, seed, mx, my, mc, ms, mv, mUa, mUd, mea, med, tm,
                                      max(t0, 0), min(t0 + G, T) - 1, mth, pxp, pyp);
        else if (act)
            q = stage_cost<NE>(d, s, mx, my, mc, ms, mv, mUa, mUd, mea, med, tm, mth, pxp, pyp);
        if (act && d.per_step) {
            if (valid) st_g(d.q, (size_t)tm * K + k, q);
            if (L.eps_staged) s.qs[tm * (SPB + 1) + grp] = q;
        }
        if (act) {
            const float yk = q - comp;
            const float tk = S + yk;
            comp = (tk - S) - yk;
            S = tk;
        }
    }

    // per-sample total over the G lanes (float64)
    double Sd = (double)S - (double)comp;
    if (G >= 2) Sd += dpp_d<0xB1>(Sd);
    if (G >= 4) Sd += dpp_d<0x4E>(Sd);
    if (G >= 8) Sd += dpp_d<0x141>(Sd);
    if (G >= 16) Sd += dpp_d<0x140>(Sd);
    float Sk = (float)Sd;
    if (!valid || !isfinite(Sk)) Sk = INFINITY;
    if (valid && r == 0) st_g(d.S, k, (float)Sd);

    // ---------------------------------------------------------------- phase 2
    // the tile's last steps go first
    if (d.wave_prio) __builtin_amdgcn_s_setprio(3);
    const int stride = partial_stride(T, d.per_step);
    double* part = d.partials + (size_t)tile * stride;
    const int n_valid = min(SPB, K - k_base);
    if (d.per_step) {
        // Per-step weights: the cost-to-go of every sample of the tile in
        // float64, then per step the tile minimum, the shifted exponential
        // sums and the weighted perturbations (one thread per step, samples
        // in index order).  The cost-to-go is summed by segments of steps, G
        // threads per sample: each sums its segment from its end back, then
        // adds the totals of the later segments, last first.  The cost-to-go
        // of step 0 (the total the weights of step 0 are formed from) is also
        // written out.  From the tile's LDS copies when they fit, else
        // through global memory.
        __syncthreads();  // the tile's stage costs are stored
        const bool lds = L.eps_staged;
        {
            const int j = tid % SPB, p = tid / SPB;
            const int len = (T + G - 1) / G;
            const int ta = min(p * len, T), tb = min(ta + len, T);
            const bool on = j < n_valid;
            auto st_ld = [&](int t) {
                return lds ? s.ss[t * (SPB + 1) + j] : ld_g(d.Stk, (size_t)t * K + k_base + j);
            };
            auto st_st = [&](int t, double v) {
                if (lds) s.ss[t * (SPB + 1) + j] = v;
                else st_g(d.Stk, (size_t)t * K + k_base + j, v);
            };
            if (on) {
                double acc = 0.0;
                for (int t = tb - 1; t >= ta; --t) {
                    acc += lds ? (double)s.qs[t * (SPB + 1) + j] : (double)ld_g(d.q, (size_t)t * K + k_base + j);
                    st_st(t, acc);
                }
            }
            __syncthreads();
            double off = 0.0;
            if (on)
                for (int pp = G - 1; pp > p; --pp)
                    if (pp * len < T) off += st_ld(pp * len);
            __syncthreads();  // segment totals are read before they change
            if (on && p < G - 1 && ta < T) {
                for (int t = ta; t < tb; ++t) st_st(t, st_ld(t) + off);
                if (lds && p == 0) st_g(d.Stk, k_base + j, st_ld(0));
            } else if (on && lds && p == 0) {
                st_g(d.Stk, k_base + j, st_ld(0));
            }
        }
        __syncthreads();
        if (lds) {
            // In LDS the three passes spread over the whole workgroup: the
            // per-step minima (one thread per step, kept where the stage
            // costs were), every sample's shifted exponential of every step
            // (written over its cost-to-go), then the sums per step in
            // sample order.
            double* mt = reinterpret_cast<double*>(s.qs);
            for (int t = tid; t < T; t += kBlock) {
                double m = INFINITY;
#pragma unroll 4
                for (int j = 0; j < n_valid; ++j) {
                    const double v = s.ss[t * (SPB + 1) + j];
                    if (isfinite(v) && v < m) m = v;
                }
                mt[t] = m;
            }
            __syncthreads();
            for (int i = tid; i < T * SPB; i += kBlock) {
                const int t = i / SPB, j = i % SPB;
                if (j >= n_valid) continue;
                double& sv = s.ss[t * (SPB + 1) + j];
                const double m = mt[t], v = sv;
                sv = isfinite(m) && isfinite(v) ? exp(-(v - m) / d.lambda) : 0.0;
            }
            __syncthreads();
            for (int t = tid; t < T; t += kBlock) {
                double z = 0.0, qq = 0.0, na = 0.0, nd = 0.0;
#pragma unroll 4
                for (int j = 0; j < n_valid; ++j) {
                    const double om = s.ss[t * (SPB + 1) + j];
                    z += om;
                    qq += om * om;
                    na += om * (double)s.eps[(2 * t) * (SPB + 1) + j];
                    nd += om * (double)s.eps[(2 * t + 1) * (SPB + 1) + j];
                }
                double* o = part + 5 * t;
                st_g(o, 0, mt[t]);
                st_g(o, 1, z);
                st_g(o, 2, qq);
                st_g(o, 3, na);
                st_g(o, 4, nd);
            }
        }
        for (int t = tid; t < T && !lds; t += kBlock) {
            auto st_at = [&](int j) { return ld_g(d.Stk, (size_t)t * K + k_base + j); };
            double m = INFINITY;
            for (int j = 0; j < n_valid; ++j) {
                const double v = st_at(j);
                if (isfinite(v) && v < m) m = v;
            }
            double z = 0.0, qq = 0.0, na = 0.0, nd = 0.0;
            if (isfinite(m)) {
#pragma unroll 4
                for (int j = 0; j < n_valid; ++j) {
                    const double v = st_at(j);
                    const double om = isfinite(v) ? exp(-(v - m) / d.lambda) : 0.0;
                    const float2 ev = ld_g(d.eps, (size_t)t * K + k_base + j);
                    z += om;
                    qq += om * om;
                    na += om * (double)ev.x;
                    nd += om * (double)ev.y;
                }
            }
            double* o = part + 5 * t;
            st_g(o, 0, m);
            st_g(o, 1, z);
            st_g(o, 2, qq);
            st_g(o, 3, na);
            st_g(o, 4, nd);
        }
    } else {
        // Tile minimum, then the tile's exponential sums: wave results through
        // LDS, combined in wave order (two barriers).
        const int wv = tid >> 6;
        const bool lane0 = (tid & 63) == 0;
        const double wmin = wave_min((double)Sk);
        if (lane0) s.red[wv] = wmin;
        __syncthreads();
        double m_b = s.red[0];
#pragma unroll
        for (int i = 1; i < kBlock / 64; ++i) m_b = fmin(m_b, s.red[i]);
        double om = 0.0;
        if (r == 0 && isfinite(m_b) && Sk < INFINITY) om = exp(-((double)Sk - m_b) / d.lambda);
        if (r == 0) s.omega[grp] = om;
        const double wz = wave_sum(om);
        const double wq = wave_sum(om * om);
        if (lane0) {
            s.red[4 + wv] = wz;
            s.red[8 + wv] = wq;
        }
        __syncthreads();  // also orders the omega stores
        double z_b = s.red[4], q_b = s.red[8];
#pragma unroll
        for (int i = 1; i < kBlock / 64; ++i) {
            z_b += s.red[4 + i];
            q_b += s.red[8 + i];
        }
        // Weighted perturbation sums, one column (step, control) per thread,
        // the float64 weights (the ones Z_b sums) times the float32
        // perturbations, summed in float64 in sample order: from
        // the tile's LDS copy of its perturbations (rows padded by one so
        // that the lanes of a wave read distinct banks) or, when that copy
        // does not fit, from global memory, sixteen loads in flight.
        constexpr int NB = SPB < 16 ? SPB : 16;
        for (int col = tid; col < 2 * T; col += kBlock) {
            if (L.eps_staged) {
                const float* e = s.eps + col * (SPB + 1);
                double acc = 0.0;
                // whole tiles: every LDS read issued before the chain of FMAs
                constexpr int NU = SPB < 16 ? SPB : 16;
                if (n_valid == SPB) {
                    for (int j0 = 0; j0 < SPB; j0 += NU) {
                        double om[NU];
                        float ev[NU];
#pragma unroll
                        for (int u = 0; u < NU; ++u) {
                            om[u] = s.omega[j0 + u];
                            ev[u] = e[j0 + u];
                        }
#pragma unroll
                        for (int u = 0; u < NU; ++u) acc = fma(om[u], (double)ev[u], acc);
                    }
                } else {
                    for (int j = 0; j < n_valid; ++j)
                        acc = fma(s.omega[j], (double)e[j], acc);
                }
                st_g(part, col, acc);
                continue;
            }
            const int t = col >> 1;
            const float* e =
                reinterpret_cast<const float*>(d.eps + (size_t)t * K + k_base) + (col & 1);
            double acc = 0.0;
            for (int i0 = 0; i0 < n_valid; i0 += NB) {
                float ev[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) ev[u] = (i0 + u < n_valid) ? ld_g(e, 2 * (i0 + u)) : 0.0f;
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if (i0 + u < n_valid) acc = fma(s.omega[i0 + u], (double)ev[u], acc);
            }
            st_g(part, col, acc);
        }
        if (tid == 0) {
            double* hd = d.partials + partial_heads_offset(T, 0, d.n_tiles) + kHeadDoubles * tile;
            st_g(hd, 0, m_b);
            st_g(hd, 1, z_b);
            st_g(hd, 2, q_b);
            st_g(hd, 3, 0.0);
        }
    }

    // ---------------------------------------------------------------- phase 3
    // The tile rows are merged by the combine kernel, which runs after this
    // one.  More than kDirect tiles
    // are first merged here, kFanIn at a time in tile order with the
    // log-sum-exp shift to their common minimum, until at most kDirect nodes
    // remain; a node's row and head are those of its first tile.
    if (d.per_step || d.n_tiles <= kDirect) return;
    double* heads = d.partials + partial_heads_offset(T, 0, d.n_tiles);
    // first ticket on the 128-byte line after the state
    unsigned int* tickets = reinterpret_cast<unsigned int*>(
        (reinterpret_cast<uintptr_t>(d.st + 1) + 4 * kTicketStride - 1) & ~(uintptr_t)(4 * kTicketStride - 1));
    unsigned int* flag = reinterpret_cast<unsigned int*>(s.red + 63);
    double* sc_lds = s.red + 8;  // kFanIn child scales
    int n_l = d.n_tiles;         // nodes at this level
    int idx = tile;              // index of this node at this level
    size_t span = 1;             // tiles per node at this level
    int toff = 0;                // first ticket of this level
    for (;;) {
        const int g = idx / kFanIn;
        const int first = g * kFanIn;
        const int nc = min(kFanIn, n_l - first);
        // The barrier orders the workgroup's row stores before the ticket;
        // the release increment publishes them device-wide.  Only the member
        // that completes the group pays for the acquire (below).
        __syncthreads();
        if (tid == 0) {
            unsigned int* tk = &tickets[(size_t)(toff + g) * kTicketStride];
            const unsigned int prev =
                __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const bool last = prev == (unsigned int)(nc - 1);
            // every member has arrived: the ticket is free for the next iteration
            if (last) __hip_atomic_store(tk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            flag[0] = last ? 1u : 0u;
        }
        __syncthreads();
        if (flag[0] == 0u) return;
        __threadfence();  // acquire the rows of every member

        double* rows = d.partials + (size_t)first * span * stride;
        const size_t cstride = span * stride;  // between consecutive children
        double* head = heads + kHeadDoubles * (size_t)first * span;
        if (tid < 64) {
            const double* h = head + kHeadDoubles * (size_t)min(tid, nc - 1) * span;
            const double mi = tid < nc ? ld_g(h, 0) : INFINITY;
            const double zi = tid < nc ? ld_g(h, 1) : 0.0;
            const double qi = tid < nc ? ld_g(h, 2) : 0.0;
            const double mm = wave_min(mi);
            // a child whose samples are all non-finite has m = +inf and weight 0
            const double sc = (tid < nc && isfinite(mi)) ? exp(-(mi - mm) / d.lambda) : 0.0;
            const double zz = wave_sum(zi * sc);
            const double qq = wave_sum(qi * sc * sc);
            if (tid < kFanIn) sc_lds[tid] = sc;
            if (tid == 0) {
                s.red[0] = mm;
                s.red[1] = zz;
                s.red[2] = qq;
            }
        }
        __syncthreads();
        for (int col = tid; col < 2 * T; col += kBlock) {
            const double* src = rows + col;
            // every child in flight at once, merged in child order
            double pv[kFanIn];
#pragma unroll
            for (int u = 0; u < kFanIn; ++u) pv[u] = u < nc ? ld_g(src, (size_t)u * cstride) : 0.0;
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < kFanIn; ++u)
                if (u < nc) acc += pv[u] * sc_lds[u];
            st_g(rows, col, acc);
        }
        if (tid == 0) {
            st_g(head, 0, s.red[0]);
            st_g(head, 1, s.red[1]);
            st_g(head, 2, s.red[2]);
        }
        toff += (n_l + kFanIn - 1) / kFanIn;
        n_l = (n_l + kFanIn - 1) / kFanIn;
        if (n_l <= kDirect) return;
        idx = g;
        span *= kFanIn;
    }
}

// Combine (Alg. 1, the normaliser and the input update of eq.
// (update-input)): merges the KH * kBlock (<= kDirect) or fewer remaining node rows of one
// instance.  Every workgroup forms the global minimum m and the node scales
// exp(-(m_b - m)/lambda), Z and Q itself (node order, fixed trees), then
// updates kCombineSteps steps of U: U_t += N_t / Z with N_t summed over the
// nodes in a fixed order (each thread a chunk of consecutive nodes in order,
// the chunks of a wave by a fixed butterfly, then the four waves in order).
// With smoothing it also updates the two steps on either side
// (from the controls the iteration kernel kept) and writes its own steps
// after eq. (sg).  Workgroup 0 records the statistics and bumps the
// iteration counter.  Nothing is written if no sample cost is finite.
template <int KH>
__device__ void combine(const InstDesc& d, int cg)
{
    extern __shared__ __align__(16) unsigned char csm[];
    double* sc = reinterpret_cast<double*>(csm);   // [KH * kBlock + 16] node scales
    double* red = sc + KH * kBlock + 16;           // [64] reductions
    double* part = red + 64;                       // [4 waves][16 slots] column partials
    double* un = part + kBlock;                    // [16] updated worked columns
    const int tid = threadIdx.x;
    const int T = d.T;
    const int s0 = cg * kCombineSteps;
    if (s0 >= T) return;
    const int s1 = min(s0 + kCombineSteps, T);
    const int w0 = d.smooth ? max(s0 - 2, 0) : s0;
    const int w1 = d.smooth ? min(s1 + 2, T) : s1;
    const int ncol = 2 * (w1 - w0);          // worked columns, 2 * w0 first
    const int slots = ncol <= 8 ? 8 : 16;    // threads per chunk
    const int chunks = kBlock / slots;
    const int stride = partial_stride(T, 0);
    size_t span = 1;
    const int n = combine_nodes(d.n_tiles, &span);
    const size_t nstride = span * stride;    // between nodes
    const double* rows = d.partials;
    const double* heads = d.partials + partial_heads_offset(T, 0, d.n_tiles);

    // One round trip: the node heads (KH per thread, from the
    // compact head array), the controls sampled around and the first sixteen
    // nodes of this thread's chunk of its worked column.  Every load is
    // issued unconditionally at an index clamped into its array and the
    // value is replaced by the neutral element afterwards, so the heads can
    // be used while the row loads are still in flight and the sums below run
    // without branches (an added +0.0 leaves a sum that started at +0.0
    // unchanged, so the results are those of skipping the term).
    constexpr int kH = KH;
    double mh[kH], zh[kH], qh[kH];
#pragma unroll
    for (int r = 0; r < kH; ++r) {
        const int i = tid + r * kBlock;
        const double* h = heads + kHeadDoubles * (size_t)min(i, n - 1) * span;
        mh[r] = ld_g(h, 0);
        zh[r] = ld_g(h, 1);
        qh[r] = ld_g(h, 2);
    }
    const int slot = tid % slots, chunk = tid / slots;
    const int per = (n + chunks - 1) / chunks;
    const int i0 = min(chunk * per, n), i1 = min(i0 + per, n);
    const bool worked = slot < ncol;
    const double* src = rows + min(2 * w0 + slot, 2 * T - 1);
    // the controls the iteration sampled around (kept after the tile rows when
    // smoothing, since other workgroups rewrite U), loaded with the rest
    const double* u_old = d.smooth ? d.partials + (size_t)d.n_tiles * stride : d.U;
    const double u_ld = ld_g(u_old, min(2 * w0 + tid, 2 * T - 1));
    double pv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) pv[u] = ld_g(src, (size_t)min(i0 + u, n - 1) * nstride);
    // (z and q masked by a product, which keeps their loads ahead of the
    // rows': a select lets the compiler sink them into the branch below)
#pragma unroll
    for (int r = 0; r < kH; ++r) {
        const bool in = tid + r * kBlock < n;
        const double keep = in ? 1.0 : 0.0;
        mh[r] = in ? mh[r] : INFINITY;
        zh[r] *= keep;
        qh[r] *= keep;
    }

    // global minimum
    double mloc = mh[0];
#pragma unroll
    for (int r = 1; r < kH; ++r) mloc = fmin(mloc, mh[r]);
    const double wm = wave_min(mloc);
    const int wv = tid >> 6;
    if ((tid & 63) == 0) red[wv] = wm;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) m = fmin(m, red[i]);
    if (!isfinite(m)) {
        if (cg == 0 && tid == 0) d.st->status = -4;  // MPPI_E_NONFINITE: U and n unchanged
        return;
    }
    // node scales (every slot of the scale array written, 0 beyond the
    // nodes and in the 16 slots of padding), Z and Q (thread, wave, then
    // waves in order)
    if (tid < 16) sc[kH * kBlock + tid] = 0.0;
    double zl = 0.0, ql = 0.0;
#pragma unroll
    for (int r = 0; r < kH; ++r) {
        const double si = isfinite(mh[r]) ? exp(-(mh[r] - m) / d.lambda) : 0.0;
        sc[tid + r * kBlock] = si;
        zl += zh[r] * si;
        ql += qh[r] * si * si;
    }
    const double wz = wave_sum(zl), wq = wave_sum(ql);
    if ((tid & 63) == 0) {
        red[4 + wv] = wz;
        red[8 + wv] = wq;
    }
    __syncthreads();  // also publishes the scales
    double z = red[4], q = red[8];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) {
        z += red[4 + i];
        q += red[8 + i];
    }

    // weighted perturbation sums of the worked columns, nodes in order
    // (i0 + u and b + u stay below n + 16: the padding covers them)
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const double pu = (worked && i0 + u < i1) ? pv[u] : 0.0;
        acc += pu * sc[i0 + u];
    }
    for (int b = i0 + 16; b < i1; b += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u) pv[u] = ld_g(src, (size_t)min(b + u, n - 1) * nstride);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const double pu = (worked && b + u < i1) ? pv[u] : 0.0;
            acc += pu * sc[b + u];
        }
    }
    // the column's sum over the chunks: the chunks of a wave (lanes slots
    // apart) by a fixed butterfly, then the four waves in order
    if (slots == 8) acc += dpp_d<0x128>(acc);  // row_ror:8, lanes 8 apart in a row
    acc = add_lanes_16_apart(acc);
    acc = add_lanes_32_apart(acc);
    if ((tid & 63) < slots) part[wv * 16 + (tid & 63)] = acc;
    __syncthreads();
    if (tid < ncol) {
        const double nsum = ((part[tid] + part[16 + tid]) + part[32 + tid]) + part[48 + tid];
        const int col = 2 * w0 + tid;
        const double u = u_ld + nsum / z;
        if (d.smooth) un[tid] = u;
        else d.U[col] = u;
    }
    if (d.smooth) {
        __syncthreads();
        // eq. (sg) on the own steps: u*_t = (-3 u_{t-2} + 12 u_{t-1} + 17 u_t +
        // 12 u_{t+1} - 3 u_{t+2}) / 35, the end values repeated beyond the horizon
        const int own = 2 * (s1 - s0);
        if (tid < own) {
            const int t = s0 + (tid >> 1), c2 = tid & 1;
            auto at = [&](int i) { return un[2 * (min(max(i, 0), T - 1) - w0) + c2]; };
            const double sm = -3.0 * at(t - 2) + 12.0 * at(t - 1) + 17.0 * at(t) +
                              12.0 * at(t + 1) - 3.0 * at(t + 2);
            d.U[2 * s0 + tid] = sm / 35.0;
        }
    }
    if (cg == 0 && tid == 0) {
        d.st->s_min = m;
        d.st->z = z;
        d.st->log_z = log(z);
        d.st->ess = z * z / q;
        d.st->status = 0;
        d.st->n_iter = d.st->n_iter + 1ull;
    }
}

// Combine with per-step weights: the tile rows hold, per step t, the tile
// minimum m_b,t of the cost-to-go and the shifted sums Z, Q, N_a, N_d.  A
// workgroup updates kCombineSteps steps (and, with smoothing, the two on
// either side): per step the minimum over the tiles, each tile's sums
// shifted to it by exp(-(m_b,t - m_t)/lambda), U_t += N_t / Z_t.  Thread
// (chunk, slot) takes step slot over a chunk of consecutive tiles, in tile
// order; the chunks of a wave are merged by a fixed butterfly, then the four
// waves in order.  The step-0 heads and the first kPsBatch rows of the
// thread's chunk are loaded in one round trip and kept in registers for both
// passes.  A sample whose total cost is finite has a finite cost-to-go at
// every step, so every step is finite exactly when step 0 is; without a
// finite step 0 nothing is written.  Workgroup 0 records the statistics of
// step 0.
constexpr int kPsBatch = 16;

__device__ void combine_per_step(const InstDesc& d, int cg)
{
    extern __shared__ __align__(16) unsigned char csm[];
    double* red = reinterpret_cast<double*>(csm);  // [64]
    double* part = red + 64;                       // [4 waves][8 slots][4] wave partials
    double* mt = part + 4 * kBlock;                // [8] step minima
    double* un = mt + 8;                           // [16] updated worked columns
    const int tid = threadIdx.x;
    const int T = d.T;
    const int s0 = cg * kCombineSteps;
    if (s0 >= T) return;
    const int s1 = min(s0 + kCombineSteps, T);
    const int w0 = d.smooth ? max(s0 - 2, 0) : s0;
    const int w1 = d.smooth ? min(s1 + 2, T) : s1;
    const int nst = w1 - w0;                 // worked steps (at most 8)
    constexpr int kSlots = 8;                // threads per chunk
    constexpr int kChunks = kBlock / kSlots;
    const size_t stride = partial_stride(T, 1);
    const int n = d.n_tiles;
    const double* rows = d.partials;
    const int wv = tid >> 6;

    const int slot = tid % kSlots, chunk = tid / kSlots;
    const bool worked = slot < nst;
    const int t = w0 + min(slot, nst - 1);
    const int per = (n + kChunks - 1) / kChunks;
    const int b0 = min(chunk * per, n), b1 = min(b0 + per, n);
    const double* col = rows + 5 * (size_t)t;
    const double* u_old = d.smooth ? d.partials + (size_t)n * stride : d.U;
    // One round trip: the step-0 heads, the controls sampled around and the
    // chunk's first rows.  Loads are issued unconditionally at indices
    // clamped into the arrays and the neutral values selected afterwards
    // (+inf for a minimum; the sums below then add exact zeros), so that no
    // load waits behind a branch.
    const int uc = 2 * (w0 + min(tid, nst - 1));
    const double ua_ld = ld_g(u_old, uc), ud_ld = ld_g(u_old, uc + 1);
    double m0v[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) m0v[r] = ld_g(rows, (size_t)min(tid + r * kBlock, n - 1) * stride);
    double hv[kPsBatch][5];
#pragma unroll
    for (int u = 0; u < kPsBatch; ++u) {
        const double* h = col + (size_t)min(b0 + u, n - 1) * stride;
#pragma unroll
        for (int c = 0; c < 5; ++c) hv[u][c] = ld_g(h, c);
    }
    double m0 = INFINITY;
#pragma unroll
    for (int r = 0; r < 2; ++r) m0 = fmin(m0, tid + r * kBlock < n ? m0v[r] : INFINITY);
    for (int b = tid + 2 * kBlock; b < n; b += kBlock) m0 = fmin(m0, rows[(size_t)b * stride]);
#pragma unroll
    for (int u = 0; u < kPsBatch; ++u) {
        const bool on = worked && b0 + u < b1;
        const double keep = on ? 1.0 : 0.0;
        hv[u][0] = on ? hv[u][0] : INFINITY;
#pragma unroll
        for (int c = 1; c < 5; ++c) hv[u][c] *= keep;
    }

    // step 0: minimum over the tiles (every workgroup)
    const double w0m = wave_min(m0);
    if ((tid & 63) == 0) red[wv] = w0m;
    __syncthreads();
    m0 = red[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) m0 = fmin(m0, red[i]);
    if (!isfinite(m0)) {
        if (cg == 0 && tid == 0) d.st->status = -4;  // MPPI_E_NONFINITE: U and n unchanged
        return;
    }

    // per-step minimum: the chunk (rows past the first batch loaded again),
    // the chunks of the wave, then the waves
    double ml = INFINITY;
#pragma unroll
    for (int u = 0; u < kPsBatch; ++u) ml = fmin(ml, hv[u][0]);
    if (worked)
        for (int b = b0 + kPsBatch; b < b1; ++b) ml = fmin(ml, col[(size_t)b * stride]);
#pragma unroll
    for (int o = kSlots; o < 64; o <<= 1) ml = fmin(ml, __shfl_xor(ml, o, 64));
    if ((tid & 63) < kSlots) part[4 * (wv * kSlots + slot)] = ml;
    __syncthreads();
    if (tid < kSlots) {
        double m = part[4 * tid];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) m = fmin(m, part[4 * (w * kSlots + tid)]);
        mt[tid] = m;
    }
    __syncthreads();

    // shifted sums of the chunk's tiles in tile order
    // (m is finite for a worked step, so a tile with m_b,t = +inf -- or a
    // slot of the batch past the chunk -- gets exp(-inf) = +0 exactly and
    // adds zeros: no branch per tile)
    double z = 0.0, qq = 0.0, na = 0.0, nd = 0.0;
    if (worked) {
        const double m = mt[slot];
        const double lam = d.lambda;
        auto add = [&](const double (&h)[5]) {
            const double sc = exp(-(h[0] - m) / lam);
            z += h[1] * sc;
            qq += h[2] * sc * sc;
            na += h[3] * sc;
            nd += h[4] * sc;
        };
#pragma unroll
        for (int u = 0; u < kPsBatch; ++u) add(hv[u]);
        for (int b = b0 + kPsBatch; b < b1; ++b) {
            const double* hp = col + (size_t)b * stride;
            const double h[5] = {hp[0], hp[1], hp[2], hp[3], hp[4]};
            add(h);
        }
    }
#pragma unroll
    for (int o = kSlots; o < 64; o <<= 1) {
        z += __shfl_xor(z, o, 64);
        qq += __shfl_xor(qq, o, 64);
        na += __shfl_xor(na, o, 64);
        nd += __shfl_xor(nd, o, 64);
    }
    __syncthreads();  // the minima in part are read
    if ((tid & 63) < kSlots) {
        double* pw = part + 4 * (wv * kSlots + slot);
        pw[0] = z;
        pw[1] = qq;
        pw[2] = na;
        pw[3] = nd;
    }
    __syncthreads();
    if (tid < nst) {
        double zt = 0.0, qt = 0.0, sa = 0.0, sd = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            const double* pc = part + 4 * (w * kSlots + tid);
            zt += pc[0];
            qt += pc[1];
            sa += pc[2];
            sd += pc[3];
        }
        const int tt = w0 + tid;
        const double ua = ua_ld + sa / zt;
        const double ud = ud_ld + sd / zt;
        if (d.smooth) {
            un[2 * tid] = ua;
            un[2 * tid + 1] = ud;
        } else {
            d.U[2 * tt] = ua;
            d.U[2 * tt + 1] = ud;
        }
        if (cg == 0 && tt == 0) {
            d.st->s_min = mt[0];
            d.st->z = zt;
            d.st->log_z = log(zt);
            d.st->ess = zt * zt / qt;
            d.st->status = 0;
            d.st->n_iter = d.st->n_iter + 1ull;
        }
    }
    if (d.smooth) {
        __syncthreads();
        const int own = 2 * (s1 - s0);
        if (tid < own) {
            const int ts = s0 + (tid >> 1), c2 = tid & 1;
            auto at = [&](int i) { return un[2 * (min(max(i, 0), T - 1) - w0) + c2]; };
            const double sm = -3.0 * at(ts - 2) + 12.0 * at(ts - 1) + 17.0 * at(ts) +
                              12.0 * at(ts + 1) - 3.0 * at(ts + 2);
            d.U[2 * s0 + tid] = sm / 35.0;
        }
    }
}

// One instance (d0, hdr == nullptr) or instance blockIdx.y of a batch; KH
// node heads per thread.
template <int KH>
__global__ __launch_bounds__(kBlock) void k_combine(InstDesc d0, const BatchHdr* __restrict__ hdr)
{
    const int cg = combine_group_of_block(blockIdx.x, gridDim.x);
    if (!hdr) {
        if (d0.per_step) combine_per_step(d0, cg);
        else combine<KH>(d0, cg);
        return;
    }
    if ((int)blockIdx.y >= hdr->n_inst) return;
    const InstDesc& d = reinterpret_cast<const InstDesc*>(
        reinterpret_cast<const unsigned char*>(hdr) + hdr->off_descs)[blockIdx.y];
    if (d.per_step) combine_per_step(d, cg);
    else combine<KH>(d, cg);
}

hipError_t launch_combine(const InstDesc* d0, const BatchHdr* hdr_dev, int groups, int n_inst,
                          int max_nodes, hipStream_t stream)
{
    InstDesc zero;
    memset(&zero, 0, sizeof zero);
    if (max_nodes <= kDirectSmall) {
        constexpr int KH = kDirectSmall / kBlock;
        const size_t smem = sizeof(double) * (KH * kBlock + 64 + 4 * kBlock + 8 + 16);
        hipLaunchKernelGGL(k_combine<KH>, dim3(combine_grid(groups, n_inst), n_inst), dim3(kBlock), smem, stream,
                           d0 ? *d0 : zero, hdr_dev);
    } else {
        constexpr int KH = kDirect / kBlock;
        const size_t smem = sizeof(double) * (KH * kBlock + 64 + 4 * kBlock + 8 + 16);
        hipLaunchKernelGGL(k_combine<KH>, dim3(combine_grid(groups, n_inst), n_inst), dim3(kBlock), smem, stream,
                           d0 ? *d0 : zero, hdr_dev);
    }
    return hipGetLastError();
}

// Exclusive prefix sum (MAX = false) or maximum (MAX = true) over the
// threads of a workgroup in thread order (float64): shuffles inside a wave,
// the totals of the earlier waves through LDS (red: kBlock / 64 doubles).
// Thread 0 gets 0 (sum) or -inf (maximum).
template <bool MAX>
__device__ __forceinline__ double block_excl(double v, double* red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double id = MAX ? -INFINITY : 0.0;
    double incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_up(incl, o, 64);
        if (lane >= o) incl = MAX ? fmax(incl, u) : incl + u;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = id;
    __syncthreads();  // red is free
    if (lane == 63) red[wv] = incl;
    __syncthreads();
    double before = id;
    for (int i = 0; i < wv; ++i) before = MAX ? fmax(before, red[i]) : before + red[i];
    return MAX ? fmax(before, excl) : before + excl;
}

// Optimal rollout of Alg. 1 in float64 and world coordinates: from x0,
// x*_{t+1} = F(x*_t, u*_t) (eq. (5), explicit Euler from the old state), each
// nominal control put through the noise check with zero noise (bounds, speed
// cap, braking bound last).  One workgroup, each thread a run of consecutive
// steps.  While the start is within v_max and a_min <= 0 the braking bound
// cannot bind and the capped speeds have the closed form of the iteration
// kernel's walk (v_t = min(v_0 + S_t, v_max + S_t - max_{1<=k<=t} S_k), S_t
// the sum of the first t commanded changes); heading, steering angle
// (5-state model) and position are prefix sums of their increments.  A start
// above v_max, or a positive a_min (the braking bound then lifts the speed
// above v_max whenever the cap falls below it), is walked step by step by one
// thread.
__global__ __launch_bounds__(kBlock) void k_trajectory(TrajArgs a, const double* __restrict__ U,
                                                       double* __restrict__ xs,
                                                       double* __restrict__ us)
{
    __shared__ double red[kBlock / 64];
    const int cols = a.model ? 5 : 4;  // the 5-state model also writes delta
    const int T = a.T;
    auto put = [&](int t, double x, double y, double th, double v, double delta) {
        double* o = xs + (size_t)cols * t;
        o[0] = x;
        o[1] = y;
        o[2] = th;
        o[3] = v;
        if (a.model) o[4] = delta;
    };
    if (!(a.x0[3] <= a.v_max) || a.a_min > 0.0) {
        if (threadIdx.x != 0) return;
        double x = a.x0[0], y = a.x0[1], th = a.x0[2], v = a.x0[3], delta = a.steer0;
        put(0, x, y, th, v, delta);
        for (int t = 0; t < T; ++t) {
            double acc = fmin(fmax(U[2 * t], a.a_min), a.a_max);
            acc = fmax(fmin(acc, (a.v_max - v) / a.dt), a.a_min);
            const double u2 = fmin(fmax(U[2 * t + 1], a.d_min), a.d_max);
            const double vdt = a.dt * v;
            const double xn = x + vdt * cos(th);
            const double yn = y + vdt * sin(th);
            // the steering angle is the control, or (5-state model) the state
            const double thn = th + vdt * tan(a.model ? delta : u2) / a.wheelbase;
            if (a.model) delta += a.dt * u2;
            v += a.dt * acc;
            x = xn;
            y = yn;
            th = thn;
            us[2 * t] = acc;
            us[2 * t + 1] = u2;
            put(t + 1, x, y, th, v, delta);
        }
        return;
    }
    constexpr int kP = kMaxT / kBlock;  // steps per thread at most
    const int P = (T + kBlock - 1) / kBlock;
    const int t0 = threadIdx.x * P;
    double acmd[kP], u2[kP], ds[kP];
    // commanded speed changes and their sums before each own step
    double run = 0.0;
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const int t = t0 + j;
        acmd[j] = u2[j] = 0.0;
        if (j < P && t < T) {
            acmd[j] = fmin(fmax(U[2 * t], a.a_min), a.a_max);
            u2[j] = fmin(fmax(U[2 * t + 1], a.d_min), a.d_max);
        }
        ds[j] = run;
        run += a.dt * acmd[j];
    }
    const double s_before = block_excl<false>(run, red);  // S at this thread's first step
    // S_t of every own step, and the maximum of S_k over 1 <= k <= t: the
    // earlier threads' maximum, then this thread's running one
    double sv[kP], qv[kP];
    double qrun = -INFINITY;
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        sv[j] = s_before + ds[j];
        if (j < P && t0 + j >= 1 && t0 + j < T) qrun = fmax(qrun, sv[j]);
        qv[j] = qrun;
    }
    const double qp = block_excl<true>(qrun, red);
    double v[kP], acc[kP], dth[kP], dd[kP];
    double drun = 0.0;
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const double q = fmax(qp, qv[j]);
        v[j] = t0 + j == 0 ? a.x0[3] : fmin(a.x0[3] + sv[j], a.v_max + sv[j] - q);
        acc[j] = fmax(fmin(acmd[j], (a.v_max - v[j]) / a.dt), a.a_min);
        dd[j] = drun;  // steering change before the own step, within the thread
        drun += a.model ? a.dt * u2[j] : 0.0;
    }
    const double d_before = a.model ? block_excl<false>(drun, red) : 0.0;
    double run_th = 0.0;
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const double delta = a.steer0 + d_before + dd[j];
        const double tn = tan(a.model ? delta : u2[j]);
        dth[j] = run_th;
        run_th += (j < P && t0 + j < T) ? a.dt * v[j] * tn / a.wheelbase : 0.0;
    }
    const double th_before = block_excl<false>(run_th, red);
    double run_x = 0.0, run_y = 0.0, dx[kP], dy[kP];
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const double th = a.x0[2] + th_before + dth[j];
        dx[j] = run_x;
        dy[j] = run_y;
        if (j < P && t0 + j < T) {
            run_x += a.dt * v[j] * cos(th);
            run_y += a.dt * v[j] * sin(th);
        }
    }
    const double x_before = block_excl<false>(run_x, red);
    const double y_before = block_excl<false>(run_y, red);
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const int t = t0 + j;
        if (j >= P || t >= T) break;
        us[2 * t] = acc[j];
        us[2 * t + 1] = u2[j];
        put(t, a.x0[0] + x_before + dx[j], a.x0[1] + y_before + dy[j], a.x0[2] + th_before + dth[j],
            v[j], a.steer0 + d_before + dd[j]);
        if (t == T - 1) {
            // the state after the last step
            const double vdt = a.dt * v[j];
            const double th = a.x0[2] + th_before + dth[j];
            const double delta = a.steer0 + d_before + dd[j];
            put(T, a.x0[0] + x_before + dx[j] + vdt * cos(th), a.x0[1] + y_before + dy[j] + vdt * sin(th),
                th + vdt * tan(a.model ? delta : u2[j]) / a.wheelbase, v[j] + a.dt * acc[j],
                delta + (a.model ? a.dt * u2[j] : 0.0));
        }
    }
}

// Iteration kernel for one or many instances of one launch shape (G lanes
// per sample): one workgroup per tile.  Tile w of a batch belongs to the
// instance whose tile range [prefix[i], prefix[i+1]) contains it; instances
// are ordered longest tile first, and the hardware dispatcher hands tiles to
// compute units as they free up.  The lanes-per-sample shape is a property of
// the instance, so an instance computes the same bits alone or in any batch.
// Workgroups past the last tile of the class (the grid is rounded up so that
// captured graphs can be replayed for other batches) return at once.
template <int G, int NE, bool M5>
__device__ __forceinline__ void batch_tile(const InstDesc& d0, const BatchHdr* __restrict__ hdr,
                                           int cls, unsigned char* smem)
{
    const int w = blockIdx.x;
    if (!hdr) {
        if (w < d0.n_tiles) iteration_tile<G, NE, M5>(d0, w, smem);
        return;
    }
    const unsigned char* base = reinterpret_cast<const unsigned char*>(hdr);
    const int i0 = hdr->cls_begin[cls];
    const int i1 = hdr->cls_begin[cls + 1];
    const int* prefix = reinterpret_cast<const int*>(base + hdr->off_prefix);
    const InstDesc* descs = reinterpret_cast<const InstDesc*>(base + hdr->off_descs);
    const int gw = w + prefix[i0];
    if (gw >= prefix[i1]) return;
    int lo = i0, hi = i1 - 1;  // largest i with prefix[i] <= gw
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= gw) lo = mid; else hi = mid - 1;
    }
    iteration_tile<G, NE, M5>(descs[lo], gw - prefix[lo], smem);
}

template <int G, int NE, bool M5>
__global__ __launch_bounds__(kBlock) void k_batch(InstDesc d0, const BatchHdr* __restrict__ hdr,
                                                  int cls)
{
    extern __shared__ __align__(16) unsigned char smem[];
    batch_tile<G, NE, M5>(d0, hdr, cls, smem);
}

// The same kernel compiled for five waves per SIMD (at most 96 VGPRs, a few
// spilled in some variants): the shape for instances with many more waves
// than the GPU holds at once, where the extra wave hides more latency than
// the spills cost.
template <int G, int NE, bool M5>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kHiOccWaves)))
void k_batch_hi(InstDesc d0, const BatchHdr* __restrict__ hdr, int cls)
{
    extern __shared__ __align__(16) unsigned char smem[];
    batch_tile<G, NE, M5>(d0, hdr, cls, smem);
}

// occ: kOccDefault or kOccHigh (the latter for 8 and 16 lanes per sample
// only; other shapes take the default compilation).
template <int G, bool M5, int OCC>
static hipError_t launch_gm(int ne, const InstDesc& a, const BatchHdr* hdr_dev, int cls, int grid,
                            size_t smem, hipStream_t stream)
{
    const dim3 g(grid), b(kBlock);
#define MPPI_LAUNCH_NE(N)                                                                        \
    case N:                                                                                       \
        if constexpr (OCC == kOccHigh)                                                            \
            hipLaunchKernelGGL((k_batch_hi<G, N, M5>), g, b, smem, stream, a, hdr_dev, cls);     \
        else                                                                                      \
            hipLaunchKernelGGL((k_batch<G, N, M5>), g, b, smem, stream, a, hdr_dev, cls);        \
        break;
    switch (ne) {
    MPPI_LAUNCH_NE(0)
    MPPI_LAUNCH_NE(1)
    MPPI_LAUNCH_NE(2)
    MPPI_LAUNCH_NE(3)
    MPPI_LAUNCH_NE(4)
    default: return hipErrorInvalidValue;
    }
#undef MPPI_LAUNCH_NE
    return hipGetLastError();
}

template <int G, int OCC>
static hipError_t launch_go(int ne, int model, const InstDesc& a, const BatchHdr* hdr_dev,
                            int cls, int grid, size_t smem, hipStream_t stream)
{
    return model ? launch_gm<G, true, OCC>(ne, a, hdr_dev, cls, grid, smem, stream)
                 : launch_gm<G, false, OCC>(ne, a, hdr_dev, cls, grid, smem, stream);
}

template <int G>
static hipError_t launch_g(int ne, int model, int occ, const InstDesc& a, const BatchHdr* hdr_dev,
                           int cls, int grid, size_t smem, hipStream_t stream)
{
    if constexpr (G >= 8) {
        if (occ == kOccHigh) return launch_go<G, kOccHigh>(ne, model, a, hdr_dev, cls, grid, smem, stream);
    }
    return launch_go<G, kOccDefault>(ne, model, a, hdr_dev, cls, grid, smem, stream);
}

hipError_t launch_batch(int lanes, int ne, int model, int occ, const InstDesc* d0,
                        const BatchHdr* hdr_dev, int cls, int grid, size_t smem,
                        hipStream_t stream)
{
    InstDesc zero;
    memset(&zero, 0, sizeof zero);
    const InstDesc& a = d0 ? *d0 : zero;
    switch (lanes) {
    case 1: return launch_g<1>(ne, model, occ, a, hdr_dev, cls, grid, smem, stream);
    case 2: return launch_g<2>(ne, model, occ, a, hdr_dev, cls, grid, smem, stream);
    case 4: return launch_g<4>(ne, model, occ, a, hdr_dev, cls, grid, smem, stream);
    case 8: return launch_g<8>(ne, model, occ, a, hdr_dev, cls, grid, smem, stream);
    case 16: return launch_g<16>(ne, model, occ, a, hdr_dev, cls, grid, smem, stream);
    default: return hipErrorInvalidValue;
    }
}

// Receding-horizon shift of every instance that asks for it (one workgroup
// per instance): U_t <- U_{min(t + 1, T-1)}.
__global__ void k_shift_batch(const BatchHdr* __restrict__ hdr)
{
    __shared__ double buf[2 * kMaxT];
    const InstDesc* descs = reinterpret_cast<const InstDesc*>(
        reinterpret_cast<const unsigned char*>(hdr) + hdr->off_descs);
    const int inst = blockIdx.x;
    if (inst >= hdr->n_inst) return;
    const InstDesc& d = descs[inst];
    if (!d.shift) return;
    const int T = d.T;
    for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) buf[i] = d.U[i];
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) {
        const int t = min((i >> 1) + 1, T - 1);
        d.U[i] = buf[2 * t + (i & 1)];
    }
}

hipError_t launch_shift_batch(const BatchHdr* hdr_dev, int n_inst, hipStream_t stream)
{
    hipLaunchKernelGGL(k_shift_batch, dim3(n_inst), dim3(256), 0, stream, hdr_dev);
    return hipGetLastError();
}

__global__ void k_gather(const BatchHdr* __restrict__ hdr, double* __restrict__ out,
                         int slot_doubles)
{
    const InstDesc* descs = reinterpret_cast<const InstDesc*>(
        reinterpret_cast<const unsigned char*>(hdr) + hdr->off_descs);
    const int inst = blockIdx.x;
    if (inst >= hdr->n_inst) return;
    const InstDesc& d = descs[inst];
    if (d.out_slot < 0) return;
    double* o = out + (size_t)d.out_slot * slot_doubles;
    for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) o[i] = d.U[i];
    if (threadIdx.x == 0) {
        o[2 * d.T] = (double)d.st->status;
        o[2 * d.T + 1] = (double)d.st->n_iter;
    }
}

hipError_t launch_gather(const BatchHdr* hdr_dev, int n_inst, double* out, int slot_doubles,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(k_gather, dim3(n_inst), dim3(256), 0, stream, hdr_dev, out, slot_doubles);
    return hipGetLastError();
}

// Normalised weights of the last iteration: w_k = exp(-(S_k - S_min)/lambda)/Z,
// from the float32 totals S or, with per-step weights, from the float64
// cost-to-go of step 0 (S0, the totals those weights were formed from).
__global__ void k_weights(const float* __restrict__ S, const double* __restrict__ S0, int K,
                          double lambda, const DevState* __restrict__ st, double* __restrict__ w)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double sk = S0 ? S0[k] : (double)S[k];
    w[k] = isfinite(sk) ? exp(-(sk - st->s_min) / lambda) / st->z : 0.0;
}

// The nominal controls and the device state copied into the caller's pinned
// host memory: one launch instead of two copies back.
__global__ __launch_bounds__(kBlock) void k_export_controls(const double* __restrict__ U, int n,
                                                            const DevState* __restrict__ st,
                                                            double* __restrict__ out_u,
                                                            DevState* __restrict__ out_st)
{
    for (int i = threadIdx.x; i < n; i += kBlock) out_u[i] = U[i];
    if (threadIdx.x == 0) *out_st = *st;
}

hipError_t launch_export_controls(const double* U, int n, const DevState* st, double* out_u,
                                  DevState* out_st, hipStream_t stream)
{
    hipLaunchKernelGGL(k_export_controls, dim3(1), dim3(kBlock), 0, stream, U, n, st, out_u,
                       out_st);
    return hipGetLastError();
}

hipError_t launch_trajectory(const TrajArgs& a, const double* U, double* states, double* applied,
                             hipStream_t stream)
{
    hipLaunchKernelGGL(k_trajectory, dim3(1), dim3(kBlock), 0, stream, a, U, states, applied);
    return hipGetLastError();
}

hipError_t launch_weights(const InstDesc& d, double* w_out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_weights, dim3((d.K + 255) / 256), dim3(256), 0, stream, d.S,
                       d.per_step ? d.Stk : nullptr, d.K, d.lambda, d.st, w_out);
    return hipGetLastError();
}

// Receding-horizon shift: U_t <- U_{min(t + steps, T-1)}.
__global__ void k_shift(double* U, int T, int steps)
{
    extern __shared__ double buf[];
    for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) buf[i] = U[i];
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) {
        const int t = min((i >> 1) + steps, T - 1);
        U[i] = buf[2 * t + (i & 1)];
    }
}

hipError_t launch_shift(double* U, int T, int steps, hipStream_t stream)
{
    hipLaunchKernelGGL(k_shift, dim3(1), dim3(256), (size_t)T * 2 * sizeof(double), stream, U,
                       T, steps);
    return hipGetLastError();
}

// Streaming copy used to calibrate traffic counters.
__global__ void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(const float4* src, float4* dst, size_t n16, hipStream_t stream)
{
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, stream, src, dst, n16);
    return hipGetLastError();
}

__global__ void k_debug_philox(uint32_t key0, uint32_t key1, unsigned long long n_iter,
                               uint32_t k0, uint32_t nk, uint32_t j0, uint32_t nj, uint32_t* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)nk * nj) return;
    const uint32_t k = k0 + (uint32_t)(i / nj);
    const uint32_t j = j0 + (uint32_t)(i % nj);
    const uint4 r = philox4x32_10(make_uint4(k, j, (uint32_t)n_iter, (uint32_t)(n_iter >> 32)),
                                  key0, key1);
    reinterpret_cast<uint4*>(out)[i] = r;
}

hipError_t launch_debug_philox(uint32_t key0, uint32_t key1, unsigned long long n_iter,
                               uint32_t k0, uint32_t nk, uint32_t j0, uint32_t nj,
                               uint32_t* out, hipStream_t stream)
{
    const uint64_t n = (uint64_t)nk * nj;
    hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       key0, key1, n_iter, k0, nk, j0, nj, out);
    return hipGetLastError();
}

}  // namespace mppi_impl
