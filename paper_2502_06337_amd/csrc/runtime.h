// Host runtime of libaoresp: per-device context, cached workspace and tables,
// and the enqueue functions shared by the single, top-k, batched and served
// solves.  Internal; the public surface is include/aoresp.h.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace aoresp {

struct ResolvedParams {
    int G, M, w, B, rad;
    float tau;
};

aoresp_status resolve_params(const aoresp_params* prm, size_t n, ResolvedParams& rp);

// Device buffers of one angle-table size B.
struct AngleTables {
    float* tc = nullptr;   // boundary directions cos(phi_k), phi_k = -pi + k*2pi/B
    float* ts = nullptr;
    float* th = nullptr;   // bin centres -pi + (k + 1/2) 2pi/B
    float* ct = nullptr;
    float* st = nullptr;
};

// Growable device buffer.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    aoresp_status ensure(size_t need);
    void release();
    template <class T>
    T* as() const { return static_cast<T*>(ptr); }
};

// Everything one solve enqueues into, for up to kMaxPeaks peaks.
struct SolveBuffers {
    DevBuf abc, colp, rowp, clip;   // per correspondence
    DevBuf grid;                    // G*G
    DevBuf fine;                    // kMaxPeaks*M*M
    DevBuf hist;                    // kMaxPeaks*B
    DevBuf keys, st, res, err;      // small
    DevBuf P, Q, masks;             // staging for host-pointer entry points
    aoresp_result* h_res = nullptr; // pinned host mirror of res (kMaxPeaks)
    PeakState* h_st = nullptr;      // pinned host mirror of st
    uint32_t* h_err = nullptr;
    hipStream_t stream = nullptr;   // internal stream for host-pointer calls
};

struct DeviceCtx {
    int device = 0;
    int cu_count = 256;
    std::mutex mu;                  // serialises use of `buf`
    SolveBuffers buf;
    std::map<int, AngleTables> angle;   // by B
    std::map<int, int16_t*> disk;       // by G
    std::mutex table_mu;
};

DeviceCtx* device_ctx();            // context of the current HIP device
const AngleTables* angle_tables(DeviceCtx* ctx, int B);
const int16_t* disk_table(DeviceCtx* ctx, int G);
int coarse_chunks(DeviceCtx* ctx, int64_t n, int G);

// Enqueue a full solve of `npk` peaks on stream s into ctx->buf (caller holds
// ctx->mu).  P, Q, masks are device pointers.  grid/fine/hist debug copies may
// be null.  Does not synchronise.
// Stage boundaries recorded when `marks` is non-null (kNumStages + 1 events).
enum Stage { kStageSetup = 0, kStageCoarse, kStagePeak, kStageFine, kStageAngle, kStageInliers, kNumStages };
aoresp_status enqueue_solve(DeviceCtx* ctx, const float* P, const float* Q, int64_t n, const ResolvedParams& rp,
                            int npk, uint8_t* masks, uint32_t* grid_out, uint32_t* fine_out, uint32_t* hist_out,
                            hipStream_t s, hipEvent_t* marks = nullptr);
// Copy results back, synchronise, translate into statuses.
aoresp_status finish_solve(DeviceCtx* ctx, int npk, aoresp_result* out, uint32_t* k_found, hipStream_t s);

}  // namespace aoresp
