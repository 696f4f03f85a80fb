// Solve entry point for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the same plain pipeline as
// pe_solve, with every transient buffer carved from one fixed per-device array instead of the
// context's growable workspace.
//
// The array below lives in this library's code object; each GPU the library runs on holds its
// own copy, at its own address, until the process ends.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): pe_ctx_create looks the
// device address up once per device with that device current, and every kernel argument and
// clear goes through that looked-up pointer.  Every buffer the pipeline reads before writing
// (tile counters, list counters, march queues) is cleared by a fill kernel inside the call, so
// the contents left by an earlier call never matter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pe_device.h"
#include "pe_runtime.h"
#include "pointemray.h"

namespace pe {

constexpr size_t kScratchBytes = (size_t)PE_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
struct DeviceScratch {
    void* ptr = nullptr;       // device address of `scratch` on this device
    hipError_t status = hipSuccess;
    std::mutex mu;             // calls on one device share the array: one at a time
};
std::mutex g_table_mu;
std::map<int, DeviceScratch*> g_table;  // entries live until the process ends

DeviceScratch* entry(int device) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    DeviceScratch*& e = g_table[device];
    if (!e) e = new DeviceScratch();
    return e;
}
}  // namespace

// Called by pe_ctx_create with `device` current: the first call per device looks up the array's
// address on that device; the result (or the HIP error) is kept for the entry point.
void scratch_init(int device) {
    DeviceScratch* e = entry(device);
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->ptr || e->status != hipSuccess) return;
    void* p = nullptr;
    const hipError_t st = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (st != hipSuccess || !p) {
        e->status = st != hipSuccess ? st : hipErrorInvalidSymbol;
        (void)hipGetLastError();
        return;
    }
    e->ptr = p;
}

}  // namespace pe

using namespace pe;

extern "C" pe_status pe_solve_noalloc(pe_ctx ctx, pe_scene scene, const pe_solve_desc* desc,
                                      pe_result* res, void* hip_stream) {
    API_BEGIN
    if (!ctx || !res || !res->E) return set_error(PE_EINVAL, "null context or result buffer");
    validate_solve(scene, desc);
    if (scene->ctx != ctx) return set_error(PE_EINVAL, "scene belongs to another context");
    if (desc->geometry != PE_GEOM_PLAIN)
        return set_error(PE_EUNSUPPORTED, "the no-allocation solve supports plain geometry only");
    // One incidence's batch must fit the array (the rest of the pipeline checks every buffer
    // it carves against the array's end before launching anything that uses it).
    const uint64_t px = (uint64_t)desc->screen_w * desc->screen_h;
    const uint64_t one = px * batch_bytes_per_pixel(desc) + (4ull << 20);
    if (one > kScratchBytes)
        return set_error(PE_ENOMEM, "screen of " + std::to_string(px) + " pixels needs about " +
                                        std::to_string(one) + " bytes of scratch; the fixed "
                                        "array holds " + std::to_string(kScratchBytes));
    DeviceScratch* e = entry(ctx->device);
    std::lock_guard<std::mutex> dev_lk(e->mu);
    if (e->status != hipSuccess || !e->ptr)
        return set_error(PE_EDEVICE, std::string("scratch array unavailable on this device: ") +
                                         hipGetErrorString(e->status));
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const auto t0 = std::chrono::steady_clock::now();
    Workspace ws(ctx, e->ptr, kScratchBytes);
    pe_stats acc{};
    const int n_obs = desc->obs_dir ? desc->n_obs : 1;
    const uint64_t per_inc = (uint64_t)n_obs * desc->n_freq * 4;
    // Incidences per batch: as many as the array holds by the per-pixel estimate; a batch that
    // still runs past the end is retried with half as many (a single incidence that does not
    // fit is an error).
    int per = (int)std::max<uint64_t>(1, kScratchBytes / (one + one / 4));
    per = std::min(per, std::min(desc->n_inc, kMaxSlots));
    for (int i0 = 0; i0 < desc->n_inc;) {
        const int cnt = std::min(per, desc->n_inc - i0);
        try {
            run_field_batch(ws, st, make_slots(scene, desc, i0, cnt), desc->contrib,
                            desc->precision, res->E + i0 * per_inc * 2,
                            res->rcs_dbsm ? res->rcs_dbsm + i0 * per_inc : nullptr, &acc,
                            desc->secondary);
        } catch (const Error& err) {
            if (err.status != PE_ENOMEM || cnt == 1) throw;
            HIPCHK(hipStreamSynchronize(st));
            per = cnt / 2;
            continue;
        }
        i0 += cnt;
    }
    HIPCHK(hipStreamSynchronize(st));
    acc.time_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (res->stats) *res->stats = acc;
    return PE_OK;
    API_END
}
