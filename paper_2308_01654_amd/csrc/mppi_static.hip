// Allocation-free single iteration (mppi_step_static of include/mppi.h): the
// work of mppi_step -- scene staging, the iteration kernel and the combine
// kernel, the same launch shape and therefore the same bits -- with every
// intermediate buffer carved out of one file-scope device array instead of
// memory the library allocates.
//
// Layout of the array for one call (each region 256-byte aligned):
//   device state (DevState), then the partial-tree tickets from the next
//   128-byte line (where the iteration kernel looks for them)
//   S      float  [K]
//   eps    float2 [T][K]
//   partials      partial_doubles(T, per_step, tiles)
//   q      float  [T][K]   (per-step weights only)
//   Stk    double [T][K]   (per-step weights only)
//   scene  the staged ego-frame scene
// The caller owns the controls U (device memory, updated in place) and the
// optional statistics (device memory).  Host-side staging of the scene uses a
// file-scope host buffer under a mutex, copied with hipMemcpyAsync from
// pageable memory, which the HIP runtime performs synchronously with respect
// to the host, so the buffer may be refilled as soon as the copy call
// returns.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>

#include "mppi_host.hpp"

using namespace mppi_impl;

namespace {

constexpr size_t kStaticScratchBytes = (size_t)MPPI_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// The scratch array: one copy per GPU, resident from the module load until
// the process ends.  Host code never passes its name to a kernel or a copy:
// it uses the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_mu;                               // staging buffer and the table below
unsigned char* g_dev_ptr[kMaxDevices] = {};    // address of `scratch` per device
alignas(256) unsigned char g_stage[64 << 10];  // host staging of one scene

static_assert(sizeof(g_stage) >= 1024 * 16 + 2048 * 8 + 2 * 2048 * 4 + 1024 * 4 + 256 * 16 + 256,
              "the host staging buffer holds the largest scene");

// Start of an iteration: the iteration counter the Philox counters use, a
// clean status and zero partial-tree tickets (the tree leaves them at zero
// after every iteration; a fresh array is cleared here as well).
__global__ void k_static_begin(DevState* st, unsigned int* tickets, int n_ticket_words,
                               unsigned long long n_iter)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_iter = n_iter;
        st->reserved = 0;
        st->status = 0;
        st->s_min = 0.0;
        st->z = 0.0;
        st->log_z = 0.0;
        st->ess = 0.0;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_ticket_words; i += gridDim.x * blockDim.x)
        tickets[i] = 0u;
}

// End of an iteration: the statistics of the combine kernel into the
// caller's device struct.
__global__ void k_static_end(const DevState* st, mppi_iter_stats* out, int lanes)
{
    if (threadIdx.x != 0) return;
    out->s_min = st->s_min;
    out->log_z = st->log_z;
    out->ess = st->ess;
    out->n_iter = st->n_iter;
    out->status = st->status;
    out->lanes_per_sample = lanes;
}

// Address of `scratch` on the current device, looked up once per device
// (with that device current).
mppi_status device_scratch(unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MPPI_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(MPPI_E_INVALID, "device %d out of range", dev);
    if (!g_dev_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MPPI_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_dev_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_dev_ptr[dev];
    return MPPI_OK;
}

// Whether p points into device (or managed) memory, the only memory the
// kernels may write.
bool device_memory(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // an unknown host pointer is reported, not sticky
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

}  // namespace

extern "C" mppi_status mppi_step_static(const mppi_config* cfg, const double x0[4],
                                        const mppi_scene* scene, double* U, uint64_t n_iter,
                                        mppi_iter_stats* stats, void* hip_stream)
{
    mppi_t* h = nullptr;  // no handle: HIP_TRY marks nothing sticky
    mppi_status s = validate_config(cfg);
    if (s != MPPI_OK) return s;
    if ((s = validate_scene(*cfg, x0, scene)) != MPPI_OK) return s;
    if (!device_memory(U)) return fail(MPPI_E_INVALID, "U must be a device pointer to [T][2] doubles");
    if (stats && !device_memory(stats))
        return fail(MPPI_E_INVALID, "stats must be a device pointer or NULL");
    if (cfg->model != 0)
        return fail(MPPI_E_INVALID, "the allocation-free iteration runs the 4-state model only");
    const hipStream_t stream = (hipStream_t)hip_stream;

    // An instance description with the caller's controls and the array's
    // regions: fill_desc then gives exactly mppi_step's descriptor.
    mppi_t inst;
    inst.cfg = *cfg;
    inst.stream = stream;
    const int K = cfg->K, T = cfg->T;
    const int n_wp = scene->n_waypoints, n_c = scene->n_circles;
    const SceneLayout lay = scene_layout(n_wp, n_c);
    const int lanes = auto_lanes(*cfg, n_c);
    const int tiles = (K + kBlock / lanes - 1) / (kBlock / lanes);
    const int n_tickets = combine_tickets(tiles) * kTicketStride;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t o_st = carve(state_bytes(tiles));
    const size_t o_S = carve(sizeof(float) * (size_t)K);
    const size_t o_eps = carve(sizeof(float2) * (size_t)T * K);
    const size_t o_part =
        carve(sizeof(double) * partial_doubles(T, cfg->per_step_weights, (size_t)tiles));
    const size_t o_q = cfg->per_step_weights ? carve(sizeof(float) * (size_t)T * K) : 0;
    const size_t o_stk = cfg->per_step_weights ? carve(sizeof(double) * (size_t)T * K) : 0;
    const size_t o_scene = carve(lay.bytes);
    if (off > kStaticScratchBytes)
        return fail(MPPI_E_INVALID,
                    "the iteration needs %zu bytes of scratch; the allocation-free path holds "
                    "at most %zu (K x T x 8 bytes of perturbations dominate)",
                    off, kStaticScratchBytes);

    std::lock_guard<std::mutex> lock(g_mu);
    unsigned char* base = nullptr;
    if ((s = device_scratch(&base)) != MPPI_OK) return s;
    inst.U = U;
    inst.st = reinterpret_cast<DevState*>(base + o_st);
    inst.S = reinterpret_cast<float*>(base + o_S);
    inst.eps = reinterpret_cast<float2*>(base + o_eps);
    inst.partials = reinterpret_cast<double*>(base + o_part);
    inst.q = cfg->per_step_weights ? reinterpret_cast<float*>(base + o_q) : nullptr;
    inst.Stk = cfg->per_step_weights ? reinterpret_cast<double*>(base + o_stk) : nullptr;
    inst.scene = base + o_scene;

    // the scene in the ego frame, as mppi_set_scene stages it
    const double origin[2] = {x0[0], x0[1]};
    write_scene(g_stage, lay, *cfg, origin, scene);
    HIP_TRY(hipMemcpyAsync(inst.scene, g_stage, lay.bytes, hipMemcpyHostToDevice, stream));

    InstDesc d;
    fill_desc(d, &inst, x0, origin, inst.scene, lay, n_wp, n_c, 0);
    choose_eps_stage(d, true, stage_allowed(&inst, n_c));  // launched alone, as mppi_step_resident
    const size_t smem =
        lds_layout(d.n_wp, d.n_c, d.T, kBlock / d.lanes, d.eps_stage, d.per_step, !d.cull).total;
    unsigned int* tickets = reinterpret_cast<unsigned int*>(
        align_up(reinterpret_cast<uintptr_t>(inst.st + 1), 4 * kTicketStride));
    hipLaunchKernelGGL(k_static_begin, dim3(1), dim3(256), 0, stream, inst.st, tickets, n_tickets,
                       (unsigned long long)n_iter);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_batch(d.lanes, active_ego(d.n_ego, d.n_c), d.model, d.occ, &d, nullptr, 0,
                         d.n_tiles,
                         smem, stream));
    HIP_TRY(launch_combine(&d, nullptr, combine_groups(d.T), 1, combine_nodes(d.n_tiles, nullptr),
                           stream));
    if (stats) {
        hipLaunchKernelGGL(k_static_end, dim3(1), dim3(64), 0, stream, inst.st, stats, d.lanes);
        HIP_TRY(hipGetLastError());
    }
    return MPPI_OK;
}
