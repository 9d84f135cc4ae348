// Internal definitions shared by the HIP kernels and the host runtime of the
// MPPI library.  Nothing here is part of the public C ABI (include/mppi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi_impl {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxEgo = 4;
constexpr int kMaxT = 2048;
constexpr int kMaxWaypoints = 2048;
constexpr int kMaxCircles = 1024;
constexpr int kMaxK = 1 << 24;

// Per-instance state that stays resident on the device between iterations.
// The allocation continues with the group tickets of the in-kernel partial
// tree (combine_tickets(max tiles) tickets of kTicketStride unsigned ints
// each, zero between iterations).
struct DevState {
    unsigned long long n_iter;  // Philox counter words 2-3: iteration number
    unsigned int reserved;
    int status;                 // 0 or MPPI_E_NONFINITE of the last iteration
    double s_min;               // min_k S_k
    double z;                   // sum_k exp(-(S_k - s_min)/lambda)
    double log_z;
    double ess;                 // z^2 / sum_k exp(-2 (S_k - s_min)/lambda)
};

// Partial results of one tile of samples: a row of the shifted weighted
// perturbation sums N_b of every (t, control) at [2t + d], and a head
//   [0] m_b (tile minimum)  [1] Z_b  [2] Q_b (sum of squares)  [3] unused
// kept in a compact array of its own (heads of consecutive tiles are
// consecutive), so that the combine reads all heads in a few lines.
constexpr int kHeadDoubles = 4;

// With per-step weights a partial row holds, for every step t, the tile
// minimum of the cost-to-go, the shifted exponential sums and the two
// weighted perturbation sums ([5t .. 5t+4]); there is no head array.
inline __host__ __device__ int partial_stride(int T, int per_step)
{
    return per_step ? 5 * T : 2 * T;
}

// Layout of the partials buffer of an instance: the tile rows, then 2T
// doubles where the iteration kernel keeps the controls it sampled around
// (read by the combine kernel when it smooths), then (total-cost weights)
// the tile heads.
inline __host__ __device__ size_t partial_heads_offset(int T, int per_step, size_t tiles)
{
    return tiles * (size_t)partial_stride(T, per_step) + 2 * (size_t)T;
}
inline __host__ __device__ size_t partial_doubles(int T, int per_step, size_t tiles)
{
    return partial_heads_offset(T, per_step, tiles) + (per_step ? 0 : kHeadDoubles * tiles);
}

// Tile partials are merged by the combine kernel, which takes up to kDirect
// rows in one pass.  Larger instances first merge their tiles inside the
// iteration kernel by a tree of fixed shape: a node of level l + 1 merges up
// to kFanIn consecutive nodes of level l, until at most kDirect nodes
// remain.  Each group has a ticket; the member that completes it merges the
// group into the row of its first tile.  The shape depends on the tile count
// only.
constexpr int kDirect = 2048;
// The combine kernel comes in two widths: up to kDirectSmall nodes (two heads
// per thread) and up to kDirect (eight per thread); a launch takes the
// narrowest that holds its largest instance.
constexpr int kDirectSmall = 512;
constexpr int kFanIn = 16;
// Tickets sit on separate 128-byte lines so that groups finishing at the same
// time do not contend for one line.
constexpr int kTicketStride = 32;

inline __host__ __device__ int combine_tickets(int n_tiles)
{
    int total = 0;
    for (int n = n_tiles; n > kDirect; n = (n + kFanIn - 1) / kFanIn) total += (n + kFanIn - 1) / kFanIn;
    return total;
}

// Nodes left for the combine kernel and the tiles each one spans.
inline __host__ __device__ int combine_nodes(int n_tiles, size_t* span)
{
    int n = n_tiles;
    size_t sp = 1;
    while (n > kDirect) {
        n = (n + kFanIn - 1) / kFanIn;
        sp *= kFanIn;
    }
    if (span) *span = sp;
    return n;
}

// Steps of U each combine workgroup updates.
constexpr int kCombineSteps = 4;
inline __host__ __device__ int combine_groups(int T) { return (T + kCombineSteps - 1) / kCombineSteps; }
// Step group of combine workgroup b of a grid `groups` wide.  A group's
// columns are 64 bytes of each tile row, the other half of their 128-byte
// line belongs to the neighbouring group; workgroups reach the 8 XCDs round
// robin (b and b + 8 share one), so within every whole run of 16 groups,
// groups 2p and 2p + 1 are given to two such blocks and the second finds
// the lines in their XCD's L2 instead of fetching them again.  A last run
// shorter than 16 keeps block b on group b.  A single instance's grid is
// padded to whole runs (blocks past the horizon return at once); a batch's,
// one row per instance, is not, to spare it the empty blocks.
inline __host__ __device__ int combine_group_of_block(int b, int grid)
{
    if ((b | 15) >= grid) return b;
    return (b & ~15) + 2 * (b & 7) + ((b >> 3) & 1);
}
inline __host__ __device__ int combine_grid(int groups, int n_inst)
{
    return n_inst == 1 ? (groups + 15) / 16 * 16 : groups;
}

// Everything one launch needs to run one MPPI iteration of one instance.
// Scene arrays are in the ego frame (x0's position subtracted) and float32.
struct InstDesc {
    int K, T, n_wp, n_c;
    int lanes;            // lanes per sample (G)
    int n_tiles;          // ceil(K / (kBlock / lanes))
    float dt, inv_dt, inv_L;
    float sig_a, sig_d;
    float a_min, a_max, d_min, d_max, v_max;
    float w_track, w_speed, w_effort, alpha, w_coll;
    float d_safe_c, d_safe_0;
    float ego_off[kMaxEgo];
    int n_ego;
    float px0, py0;       // initial position relative to the scene origin
    float th0, v0;        // initial yaw and speed
    double lambda;
    uint32_t key0, key1;  // Philox key = seed
    int shift;            // shift U by one step before the iteration (warm start)
    int cull;             // wave-level culling of waypoint chunks and circles
    int smooth;           // end with the Savitzky-Golay filter of eq. (sg)
    float w_target, w_yaw;// weights of c_target and c_yaw (0: term skipped)
    int coll_only;        // c_safe_dist only when d_obj <= 0
    int per_step;         // 1: weights from the cost-to-go per step
    int eps_stage;        // 1: tiles keep their perturbations in LDS (lds_layout)
    int wave_prio;        // 1: wave priority falls with the block index (see iteration_tile)
    int occ;              // compilation it is launched with, kOccDefault or kOccHigh (host-side)
    int model;            // 1: 5-state model of eq. (5), steering-rate control
    float steer0;         // its initial steering angle
    float ego_ext;        // max |ego_off|
    int out_slot;         // slot in the gathered results of a batch (-1: none)
    // device pointers
    const float2* wp_xy;  // [n_wp]
    const float* wp_vref; // [n_wp]
    const float* wp_yaw;  // [n_wp]
    const float4* wp_box; // [chunks] (x_lo, x_hi, y_lo, y_hi) of each chunk
    const int* scene_flags; // [0]: every waypoint has the same reference speed
    const float4* c_pv;   // [n_c] (x, y, vx, vy)
    const float* c_rr;    // [n_c] r_c + r_ego
    double* U;            // [T][2]
    float* S;             // [K]
    float2* eps;          // [T][K]
    double* partials;     // partial_doubles(T, per_step, n_tiles)
    float* q;             // [T][K] stage costs (per-step weights)
    double* Stk;          // [T][K] cost-to-go (per-step weights; row 0 always, the
                          // other rows only when a tile works in global memory)
    DevState* st;         // followed by the partial-tree tickets
};

// Compilations of the iteration kernel (the "occupancy" launch choice): the
// default one, and one for kHiOccWaves waves per SIMD (8 and 16 lanes per
// sample only).
constexpr int kOccDefault = 0;
constexpr int kOccHigh = 1;
constexpr int kOccModes = 2;
constexpr int kHiOccWaves = 5;

// Header of a batch arena in device memory: followed by the tile prefix
// (n_inst + 1 ints) at off_prefix and the descriptors at off_descs.
// Instances are grouped by kernel variant: class c = 50 * occ + 25 * model +
// 5 * lane_index + ne (occ the compilation, kOccDefault or kOccHigh; model 0
// or 1 (5-state); lane_index 0..4 for 1, 2, 4, 8, 16 lanes per sample; ne =
// ego circles that meet obstacle circles, 0..4) owns instances
// [cls_begin[c], cls_begin[c+1]).
constexpr int kLaneClasses = 50 * kOccModes;
struct BatchHdr {
    int n_inst;
    int total_tiles;
    int off_prefix;
    int off_descs;
    int cls_begin[kLaneClasses + 1];
    int pad[2];
};

// Dynamic LDS layout of the iteration kernel for a given scene size.
struct LdsLayout {
    size_t c_pv, wp_box, wp_xy, red, wp_vref, wp_yaw, c_rr, omega, eps, qs, ss, total;
    int eps_staged;  // the tile's applied perturbations are kept at eps, and
                     // with per-step weights its stage costs at qs and its
                     // cost-to-go at ss
};

// Largest LDS copy of a tile's applied perturbations ([2T][spb + 1] floats)
// and, with per-step weights, stage costs ([T][spb + 1] floats) and
// cost-to-go ([T][spb + 1] doubles, rows padded by one).
constexpr size_t kEpsStageMax = 48 << 10;
// The copy is made when the workgroup's LDS stays within kLdsShared (five
// workgroups per compute unit), or within kLdsAlone for an instance launched
// alone with at most two tiles per compute unit (256 units).
constexpr size_t kLdsShared = 32 << 10;
constexpr size_t kLdsAlone = 64 << 10;

// Waypoints are grouped in chunks of this many consecutive points; each chunk
// has an axis-aligned bounding box in LDS for the wave-level culling.  A
// chunk is kChunkQ 16-byte (two-point) reads; the culled scan fetches
// kChunkTrip chunks per memory round trip.  (At the sine-lane workload
// chunks of 16 are 2% faster and chunks of 4 are 4% slower; at the paper's
// small scenes chunks of 16 are 5-8% slower.)
constexpr int kChunk = 8;
static_assert(kChunk == 4 || kChunk == 8 || kChunk == 16, "chunks of 4, 8 or 16 waypoints");
constexpr int kChunkQ = kChunk / 2;
constexpr int kChunkTrip = kChunk < 16 ? 16 / kChunk : 1;
// The per-lane culling bound takes the waypoints kSeedAhead, 2 kSeedAhead and
// 3 kSeedAhead after the start of the lane's previous closest chunk.
constexpr int kSeedAhead = 4;

inline __host__ __device__ size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// scene_lds: the tile keeps a copy of the scene in LDS (the full scans of an
// instance without culling read it there; the culled scans read the scene
// from global memory, through the scalar cache for wave-uniform candidates).
inline __host__ __device__ LdsLayout lds_layout(int n_wp, int n_c, int T, int spb, int eps_stage,
                                                int per_step, int scene_lds)
{
    LdsLayout L;
    size_t o = 0;
    const size_t sc = scene_lds ? 1 : 0;
    L.c_pv = o;    o += sc * (size_t)n_c * 16;
    L.wp_box = o;  o += sc * (size_t)((n_wp + kChunk - 1) / kChunk) * 16;
    L.wp_xy = o;   o += sc * (size_t)((n_wp + kChunk - 1) / kChunk) * kChunk * 8;  // padded
    L.red = o;     o += 64 * 8;           // block reduction scratch (doubles)
    L.wp_vref = o; o += sc * (size_t)n_wp * 4;
    L.wp_yaw = o;  o += sc * (size_t)n_wp * 4;
    L.c_rr = o;    o += sc * (size_t)n_c * 4;
    o = align_up(o, 8);
    L.omega = o;   o += (size_t)spb * 8;   // float64 weights
    const size_t eb = (size_t)2 * T * (spb + 1) * 4;
    const size_t qb = per_step ? align_up((size_t)T * (spb + 1) * 4, 8) : 0;
    const size_t sb = per_step ? (size_t)T * (spb + 1) * 8 : 0;
    L.eps_staged = eps_stage && eb + qb + sb <= kEpsStageMax;
    L.eps = o;     o += L.eps_staged ? eb : 0;
    o = align_up(o, 8);
    L.qs = o;      o += L.eps_staged ? qb : 0;
    L.ss = o;      o += L.eps_staged ? sb : 0;
    L.total = align_up(o, 16);
    return L;
}

// Launchers (mppi_kernels.hip).  All enqueue on `stream` and return the
// launch error, if any.
// Iteration kernel, one workgroup per tile: one instance (d0, hdr_dev ==
// nullptr) or lanes class `cls` of the batch described by the arena at
// hdr_dev (lanes is the launch shape of every instance it processes).
hipError_t launch_batch(int lanes, int ne, int model, int occ, const InstDesc* d0,
                        const BatchHdr* hdr_dev, int cls, int grid, size_t smem,
                        hipStream_t stream);

// Combine of the tile rows of one instance (d0, hdr_dev == nullptr) or of
// every instance of a batch (n_inst rows of the grid, groups = largest
// combine_groups(T) among them).
// max_nodes: the largest combine_nodes() among the instances.
hipError_t launch_combine(const InstDesc* d0, const BatchHdr* hdr_dev, int groups, int n_inst,
                          int max_nodes, hipStream_t stream);

// Ego circles that take part in the obstacle term of an instance.
inline int active_ego(int n_ego, int n_c) { return n_c > 0 ? n_ego : 0; }
hipError_t launch_shift_batch(const BatchHdr* hdr_dev, int n_inst, hipStream_t stream);
// Copies, for every instance with out_slot >= 0, U [2T], the status and the
// iteration counter to out + out_slot * slot_doubles.
hipError_t launch_gather(const BatchHdr* hdr_dev, int n_inst, double* out, int slot_doubles,
                         hipStream_t stream);
hipError_t launch_weights(const InstDesc& d, double* w_out, hipStream_t stream);

// Optimal rollout of Alg. 1 (float64, world frame) from x0 under the nominal
// controls U [T][2]: states [T+1][4] and applied controls [T][2].
struct TrajArgs {
    double x0[4];
    double steer0;  // initial steering angle (model 1)
    int T;
    int model;      // 1: 5-state model, states written with 5 columns
    double dt, wheelbase, a_min, a_max, d_min, d_max, v_max;
};
// U [n] and the device state into host memory the device can write (pinned).
hipError_t launch_export_controls(const double* U, int n, const DevState* st, double* out_u,
                                  DevState* out_st, hipStream_t stream);
hipError_t launch_trajectory(const TrajArgs& a, const double* U, double* states, double* applied,
                             hipStream_t stream);
hipError_t launch_shift(double* U, int T, int steps, hipStream_t stream);
hipError_t launch_copy(const float4* src, float4* dst, size_t n16, hipStream_t stream);
hipError_t launch_debug_philox(uint32_t key0, uint32_t key1, unsigned long long n_iter,
                               uint32_t k0, uint32_t nk, uint32_t j0, uint32_t nj,
                               uint32_t* out, hipStream_t stream);

}  // namespace mppi_impl
