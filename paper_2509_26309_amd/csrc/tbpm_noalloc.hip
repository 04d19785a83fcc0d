// Allocation-free variant of tbpm_propagate_dos.
//
// The propagation buffers (random-phase state, the rotating Chebyshev
// vectors, per-workgroup partial sums, the device rows of C(t) and the norms)
// are carved from one file-scope device array instead of being allocated, so
// the call performs no hipMalloc / hipFree and no allocation through the
// context's allocator, no pinned host allocation and no graph instantiation.
// Each device the library runs on holds its own copy of the array (the
// loader places it with the code object) until the process ends.
//
// Host code never uses the array's name as an address: its device address is
// looked up once per device with hipGetSymbolAddress when a context is
// created on that device, and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tbpm_engine.h"
#include "tbpm_trace.h"

namespace tbpm {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)TBPM_NOALLOC_MAX_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// With `device` current: records the device address of `scratch` on it (once).
hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device])
        return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    if (!ptr)
        return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

static void *noalloc_ptr(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace tbpm

using namespace tbpm;

extern "C" tbpm_status tbpm_propagate_dos_noalloc(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                                  double *corr, double *norms, double *corr_mean)
{
    if (!ctx || !ham)
        return TBPM_ERR_ARG;
    if (ham->ctx != ctx) {
        ctx->last_error = "Hamiltonian belongs to another context";
        return TBPM_ERR_ARG;
    }
    if (!corr) {
        ctx->last_error = "corr must not be NULL";
        return TBPM_ERR_ARG;
    }
    if (params && params->num_ldos_sites > 0) {
        ctx->last_error = "the allocation-free propagation takes no LDOS sites";
        return TBPM_ERR_ARG;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->last_error = "hipSetDevice failed";
        return TBPM_ERR_HIP;
    }
    TraceRange range("tbpm_propagate_dos_noalloc");
    char *base = static_cast<char *>(noalloc_ptr(ctx->device));
    if (!base) {
        ctx->last_error = std::string("the scratch area of this device is not available: ") +
                          hipGetErrorString(ctx->noalloc_status);
        return TBPM_ERR_HIP;
    }
    Job job;
    job.arena = base;
    job.arena_bytes = NOALLOC_SCRATCH_BYTES;
    job.direct_corr = corr;
    job.direct_norms = norms;
    tbpm_status s = job.setup(ctx, ham, params, ctx->stream);
    if (s == TBPM_OK && job.arena_need() > NOALLOC_SCRATCH_BYTES)
        s = job.fail_with(TBPM_ERR_TOO_LARGE,
                          "the propagation needs " + std::to_string(job.arena_need()) +
                              " bytes of device buffers; the allocation-free scratch area holds " +
                              std::to_string(NOALLOC_SCRATCH_BYTES));
    if (s == TBPM_OK)
        s = job.allocate();
    if (s == TBPM_OK)
        s = job.advance(INT32_MAX);
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (s == TBPM_OK && e != hipSuccess) {
        ctx->last_error = std::string("propagation: ") + hipGetErrorString(e);
        return TBPM_ERR_HIP;
    }
    if (s == TBPM_OK)
        s = job.finish(corr, norms, nullptr, corr_mean);
    if (s != TBPM_OK)
        ctx->last_error = job.error;
    return s;
}
