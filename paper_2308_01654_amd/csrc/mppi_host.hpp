// Host-side internals of the MPPI library shared by the C-ABI runtime
// (mppi_api.hip) and the request server (mppi_server.hip).  Not part of the
// public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_internal.hpp"

namespace mppi_impl {

mppi_status fail(mppi_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// A captured batch launch: arena copy + kernels, for one size class.
struct GraphEntry {
    size_t bytes, smem;
    int grids[kLaneClasses];
    int buf, shift_blocks, gather_blocks, combine_g, combine_y;
    int combine_nodes;  // the combine width's node limit (kDirectSmall or kDirect)
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// Staging and device arena of batched launches (descriptors + scenes), and
// the instantiated graphs that replay them.
struct BatchWs {
    unsigned char* arena = nullptr;
    unsigned char* stage[2] = {nullptr, nullptr};
    size_t cap = 0;
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    int cur = 0;
    std::vector<GraphEntry> graphs;
};

struct ProfEvent {
    hipEvent_t a, b;
    int kind;  // 0 = iteration (iteration and combine kernels), 1 = auxiliary,
               // 2 = iteration kernel alone
};

// Offsets of the four scene arrays inside a staged scene block.
struct SceneLayout {
    size_t o_pv, o_xy, o_vr, o_yw, o_rr, o_box, o_flags, bytes;
};

// Per-instance extras of a batched launch: scratch buffers that replace the
// handle's own (server vehicles own no scratch), the warm-start shift flag,
// and the slot of the instance in the gathered result buffer (-1: none).
struct InstExtra {
    float* S;
    float2* eps;
    double* partials;
    float* q;
    double* Stk;
    int shift;
    int out_slot;
};

}  // namespace mppi_impl

// One planning instance (opaque mppi_t of the C ABI).
struct mppi {
    mppi_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int lanes_req = 0;  // 0 = tuning table
    int stage_req = -1; // -1 = tuning table, 0 = no LDS copy of the perturbations, 1 = when it fits
    int occ_req = -1;   // -1 = tuning table, else kOccDefault or kOccHigh
    int no_cull = 0;    // 1: full waypoint and circle scans
    int last_lanes = 0;
    mppi_status sticky = MPPI_OK;
    // device memory
    double* U = nullptr;
    float* S = nullptr;
    float2* eps = nullptr;
    double* partials = nullptr;
    float* q = nullptr;      // [T][K] stage costs (per-step weights)
    double* Stk = nullptr;   // [T][K] cost-to-go (per-step weights)
    double* wbuf = nullptr;  // [K] weights export
    // optimal trajectory: states [T+1][4 or 5], controls [T][2], in pinned
    // coherent host memory that k_trajectory writes directly (traj_dev is
    // its device address)
    double* traj = nullptr;
    double* traj_dev = nullptr;
    // pinned coherent host buffer that k_export_controls writes: U [T][2],
    // then the device state (ctl_dev: its device address)
    double* ctl_host = nullptr;
    double* ctl_dev = nullptr;
    mppi_impl::DevState* st = nullptr;
    unsigned char* scene = nullptr;
    size_t scene_cap = 0;
    // pinned scene staging, double-buffered
    unsigned char* staging[2] = {nullptr, nullptr};
    hipEvent_t staged[2] = {nullptr, nullptr};
    bool staged_pending[2] = {false, false};
    int cur = 0;
    int max_tiles = 0;
    mppi_impl::BatchWs* batch = nullptr;  // created when this handle leads a batch
    // resident scene
    bool has_scene = false;
    double origin[2] = {0.0, 0.0};
    int n_wp = 0, n_c = 0;
    mppi_impl::SceneLayout lay = {0, 0, 0, 0, 0, 0};
    // last step
    bool stepped = false;
    double last_x0[4] = {0.0, 0.0, 0.0, 0.0};
    double steer0 = 0.0;      // initial steering angle (5-state model)
    double last_steer0 = 0.0; // the one the last step used
    // profiling
    bool prof = false;
    std::vector<mppi_impl::ProfEvent> events;
    std::vector<hipEvent_t> event_pool;  // recorded and read events, for reuse
    double prof_ms[3] = {0.0, 0.0, 0.0};
    int64_t prof_n[3] = {0, 0, 0};
};

namespace mppi_impl {

// Reports a HIP failure as MPPI_E_DEVICE (sticky on handle `h`, if any).
#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            if (h) h->sticky = MPPI_E_DEVICE;                                                \
            return ::mppi_impl::fail(MPPI_E_DEVICE, "%s: %s (%s:%d)", #expr,                 \
                                     hipGetErrorString(e_), __FILE__, __LINE__);            \
        }                                                                                    \
    } while (0)

SceneLayout scene_layout(int n_wp, int n_c);
// Bytes of a handle's device state: DevState and the partial-tree tickets
// for up to max_tiles tiles.
inline size_t state_bytes(int max_tiles)
{
    return sizeof(DevState) +
           sizeof(unsigned int) * kTicketStride * ((size_t)combine_tickets(max_tiles) + 1);
}
void write_scene(unsigned char* dst, const SceneLayout& L, const mppi_config& c,
                 const double origin[2], const mppi_scene* sc);
mppi_status validate_scene(const mppi_config& c, const double x0[4], const mppi_scene* sc);
mppi_status validate_config(const mppi_config* c);
mppi_status usable(mppi_t* h);
int auto_lanes(const mppi_config& c, int n_c);
size_t pow2_at_least(size_t v, size_t lo);
mppi_status record_launch(mppi_t* h, int kind, hipEvent_t* a);
mppi_status record_end(mppi_t* h, int kind, hipEvent_t a);
void fill_desc(InstDesc& d, const mppi_t* h, const double x0[4], const double origin[2],
               const unsigned char* scene, const SceneLayout& L, int n_wp, int n_c, int shift);
// Whether the tiles of d keep their perturbations in LDS: within kLdsShared,
// or within kLdsAlone for an instance launched alone (alone = true) with at
// most 512 tiles.
void choose_eps_stage(InstDesc& d, bool alone, int allowed);
// Whether h's tiles may keep their perturbations in LDS (its own setting or
// the tuning table's choice for its shape).
int stage_allowed(const mppi_t* h, int n_c);
int auto_stage(const mppi_config& c, int n_c);
// The compilation of the iteration kernel an instance is launched with: the
// tuning table's choice (kOccDefault when it has no such column) unless the
// handle requests one; kOccDefault below 8 lanes per sample.
int auto_occ(const mppi_config& c, int n_c);
int occ_choice(const mppi_t* h, int n_c, int lanes);
mppi_status ws_create(BatchWs** out);
void ws_destroy(BatchWs* b);
// Create a handle; with_scratch = false leaves S/eps/partials/scales/scene
// unallocated (server vehicles take them from the request pool).
mppi_status handle_create(const mppi_config* cfg, void* hip_stream, bool with_scratch,
                          mppi_t** out);
void handle_release(mppi_t* h);
// Enqueue one iteration of hs[0..n) as one launch per kernel variant on
// `stream`.  scenes == nullptr: resident scenes.  extra: optional per-instance
// scratch/shift/result slot.  gather_dev: optional buffer the device can
// write (device memory, or the device address of pinned host memory)
// receiving, per instance with out_slot >= 0, U [2T] doubles followed by the
// status and the iteration counter at slot * slot_doubles.  use_graph: capture the
// launch sequence per size class and replay it (repeated batches of one
// shape); otherwise launch directly (batches whose composition changes).
mppi_status batch_enqueue(BatchWs* ws, hipStream_t stream, mppi_t* const* hs, const double* x0s,
                          const mppi_scene* scenes, const InstExtra* extra, int n, mppi_t* prof,
                          double* gather_dev, int slot_doubles, bool use_graph);

}  // namespace mppi_impl
