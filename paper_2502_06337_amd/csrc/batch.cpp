// Batched solves (est_rotation_batch): many independent instances of uneven
// size in one launch per stage.  Every stage runs over the instance table;
// the coarse vote uses persistent work-groups pulling (instance, pass, band,
// chunk) items ordered largest first.  The stage sequence of a batch is
// captured into one hipGraph and launched as a whole (the executable graph is
// updated in place for the next batch).  Instance b's result is bit-identical
// to est_rotation on its own columns with the same parameters: the kernels
// are the same and each instance only touches its own grid, windows and
// histograms.  A layout (offsets, parameters, work splits, device pointers)
// that comes twice in a row on the device, with no other solve in between,
// is recorded as one graph and launched again while it keeps coming, without
// planning or capturing.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace aoresp;

static aoresp_status batch_common(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                  const aoresp_params* prm, uint32_t prm_count, aoresp_result* out, uint8_t* masks,
                                  bool host, hipStream_t s) {
    if (!off || !out || batch == 0 || (prm_count != 0 && prm_count != 1 && prm_count != batch)) return AORESP_EINVAL;
    if (prm_count > 0 && !prm) return AORESP_EINVAL;
    const uint64_t N = off[batch];
    if (off[0] != 0 || N > (uint64_t)INT32_MAX) return AORESP_EINVAL;
    if (N > 0 && (!P || !Q)) return AORESP_EINVAL;
    std::vector<ResolvedParams> rps(batch);
    std::vector<int64_t> offs(batch + 1);
    std::vector<int> npk(batch, 1);
    for (uint32_t b = 0; b < batch; ++b) {
        if (off[b + 1] < off[b]) return AORESP_EINVAL;
        const aoresp_params* p = prm_count == 0 ? nullptr : (prm_count == 1 ? prm : prm + b);
        aoresp_status st = resolve_params(p, off[b + 1] - off[b], rps[b]);
        if (st != AORESP_OK) return st;
        offs[b] = (int64_t)off[b];
    }
    offs[batch] = (int64_t)N;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Workspace& w = ctx->ws;
    aoresp_status st;
    const float* dP = P;
    const float* dQ = Q;
    uint8_t* dM = masks;
    if (host) {
        s = internal_stream(ctx);
        if (!s) return AORESP_EDEVICE;
        if ((st = w.P.ensure(3 * N * sizeof(float) + 4)) != AORESP_OK) return st;
        if ((st = w.Q.ensure(3 * N * sizeof(float) + 4)) != AORESP_OK) return st;
        if (masks && (st = w.masks.ensure(N + 4)) != AORESP_OK) return st;
        if (N && hipMemcpyAsync(w.P.ptr, P, 3 * N * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
            return AORESP_EDEVICE;
        if (N && hipMemcpyAsync(w.Q.ptr, Q, 3 * N * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
            return AORESP_EDEVICE;
        dP = w.P.as<float>();
        dQ = w.Q.as<float>();
        dM = masks ? w.masks.as<uint8_t>() : nullptr;
    }
    // the whole batched pipeline, recorded as one graph once the same layout
    // comes twice in a row and launched again while it keeps coming
    Plan scratch;
    const Plan* plan_used = nullptr;
    if ((st = run_plan(ctx, w, plan_key(ctx, offs.data(), (int)batch, rps.data(), npk.data(), dP, dQ, dM),
                       offs.data(), (int)batch, rps.data(), npk.data(), dP, dQ, dM, s, scratch, &plan_used)) !=
        AORESP_OK)
        return st;
    const Plan& plan = *plan_used;
    if (host && masks && N && hipMemcpyAsync(masks, w.masks.ptr, N, hipMemcpyDeviceToHost, s) != hipSuccess)
        return AORESP_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return AORESP_EDEVICE;
    std::vector<int> valid;
    if ((st = collect_plan(w, plan, out, valid)) != AORESP_OK) return st;
    // instances with fewer than two correspondences or no vote: R = I
    for (uint32_t b = 0; b < batch; ++b) {
        if (off[b + 1] - off[b] < 2 || !valid[b]) {
            identity_result(&out[b], rps[b].G);
        }
    }
    return AORESP_OK;
}

extern "C" aoresp_status est_rotation_batch_dev(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                                const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                                uint8_t* masks, void* hip_stream) {
    return batch_common(P, Q, off, batch, prm, prm_count, out, masks, false, (hipStream_t)hip_stream);
}

extern "C" aoresp_status est_rotation_batch(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                            const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                            uint8_t* masks) {
    return batch_common(P, Q, off, batch, prm, prm_count, out, masks, true, nullptr);
}
