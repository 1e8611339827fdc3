// Allocation-free single solve (est_rotation_noalloc_dev): the same pipeline
// as est_rotation_dev, with every device buffer of the plan carved from one
// file-scope device array and every host staging buffer from one file-scope
// host array.  It calls no hipMalloc, hipFree or hipHostMalloc: the angle and
// disk tables are built on the host into the staging array and copied into the
// device array with the plan.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace aoresp {
namespace {

// Device scratch: tables, per-correspondence records (64 B each), grid and
// arenas, result slots.  96 MiB holds a solve of 10^6 correspondences on a
// 1024 x 1024 grid with 64 x 64 refinement and 3600 angle bins (about 69 MB).
constexpr size_t kScratchBytes = (size_t)96 << 20;
// Host staging: the tables' image, the plan blob and the results copy.
constexpr size_t kStageBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];
alignas(256) static unsigned char g_stage[kStageBytes];

std::mutex g_mu;                         // one call at a time in the process
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Device address of this device's copy of the scratch array (looked up once
// per device; the caller holds g_mu and has the device current).
void* scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace aoresp

using namespace aoresp;

extern "C" aoresp_status est_rotation_noalloc_dev(const float* P, const float* Q, size_t n,
                                                  const aoresp_params* prm, aoresp_result* out,
                                                  uint8_t* inlier_mask, void* hip_stream) {
    if (!out || (n > 0 && (!P || !Q))) return AORESP_EINVAL;
    if (n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    if ((size_t)rp.B * 12 > 160 * 1024) return AORESP_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (n < 2) {
        identity_result(out, rp.G);
        if (inlier_mask && n) {
            if (hipMemsetAsync(inlier_mask, 0, n, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
                return AORESP_EDEVICE;
        }
        return AORESP_ENODATA;
    }
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    char* base = static_cast<char*>(scratch_of(ctx->device));
    if (!base) return AORESP_EDEVICE;

    // tables first: their image at the head of the staging array, their
    // device copy at the head of the scratch array
    TableSink sink;
    sink.host = reinterpret_cast<char*>(g_stage);
    sink.dev = base;
    sink.cap = kStageBytes;
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = 1;
    if ((st = build_plan_with(ctx, off, 1, &rp, &npk, nullptr, plan, &sink)) != AORESP_OK)
        return st == AORESP_ENOMEM || st == AORESP_EINVAL ? st : AORESP_EDEVICE;
    const size_t table_bytes = up256(sink.used);

    // every device buffer of the plan, in order, after the tables
    Workspace w;
    BufNeed need[kPlanBuffers];
    plan_buffers(w, plan, need);
    size_t used = table_bytes;
    for (int i = 0; i < kPlanBuffers; ++i) {
        const size_t b = up256(need[i].bytes);
        if (used + b > kScratchBytes) return AORESP_ENOMEM;
        need[i].buf->ptr = base + used;
        need[i].buf->bytes = b;
        need[i].buf->fixed = true;
        used += b;
    }
    // host staging after the tables' image: the plan blob, then the results
    const OutLayout ol(plan.nres);
    size_t hused = table_bytes;
    const size_t blob = up256(plan_blob_bytes(plan));
    if (hused + blob + up256(ol.bytes) > kStageBytes) return AORESP_ENOMEM;
    w.h_plan.ptr = g_stage + hused;
    w.h_plan.bytes = blob;
    w.h_plan.fixed = true;
    hused += blob;
    w.h_out.ptr = g_stage + hused;
    w.h_out.bytes = up256(ol.bytes);
    w.h_out.fixed = true;

    if (sink.used && hipMemcpyAsync(base, g_stage, sink.used, hipMemcpyHostToDevice, s) != hipSuccess)
        return AORESP_EDEVICE;
    if ((st = enqueue_plan(ctx, w, plan, P, Q, inlier_mask, s)) != AORESP_OK) return st;
    std::vector<int> valid;
    if ((st = finish_plan(w, plan, out, valid, s)) != AORESP_OK) return st;
    if (!valid[0]) {
        identity_result(out, rp.G);
        return AORESP_ENODATA;
    }
    return AORESP_OK;
}
