// Host runtime of libaoresp: per-device context, cached workspace and tables,
// and the batch planner shared by the single, top-k, batched and served
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

// Growable pinned host buffer.
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    aoresp_status ensure(size_t need);
    template <class T>
    T* as() const { return static_cast<T*>(ptr); }
};

// Everything a batch enqueues into.
struct Workspace {
    DevBuf abc, colp, rowp, geo;    // per global column
    DevBuf grid, fine, hist;        // arenas
    DevBuf keys, st, res, err;      // per result slot (+ err flag, vote counter)
    DevBuf plan;                    // instance table + work items
    DevBuf P, Q, masks;             // staging for host-pointer entry points
    HostBuf h_plan, h_res, h_st;    // pinned mirrors
    hipStream_t stream = nullptr;   // internal stream for host-pointer calls
};

// A batch laid out for the kernels.
struct Plan {
    std::vector<Inst> insts;
    std::vector<int4> vote_items, cell_items, corr_items, list_items;
    int64_t N = 0;
    size_t grid_cells = 0, fine_cells = 0, hist_cells = 0;
    int nres = 0;              // result slots (sum of npk)
    int max_npk = 0, maxM = 0;
    size_t hist_lds = 0;
};

struct DeviceCtx {
    int device = 0;
    int cu_count = 256;
    std::mutex mu;                      // serialises use of `ws`
    Workspace ws;
    std::map<int, AngleTables> angle;   // by B
    std::map<int, int16_t*> disk;       // by G
    std::mutex table_mu;
};

DeviceCtx* device_ctx();            // context of the current HIP device
const AngleTables* angle_tables(DeviceCtx* ctx, int B);
const int16_t* disk_table(DeviceCtx* ctx, int G);

// Instance b owns global columns [off[b], off[b+1]).
aoresp_status build_plan(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rp, const int* npk,
                         Plan& plan);

// Stage boundaries recorded when `marks` is non-null (kNumStages + 1 events).
enum Stage { kStageSetup = 0, kStageCoarse, kStagePeak, kStageFine, kStageAngle, kStageInliers, kNumStages };

// Enqueue the whole pipeline of a plan on stream s into ctx->ws (caller holds
// ctx->mu).  P, Q ((3, N) SoA), masks (max_npk * N or null) are device
// pointers.  Debug copies (single-instance plans) may be null.  No sync.
aoresp_status enqueue_plan(DeviceCtx* ctx, Workspace& w, const Plan& plan, const float* P, const float* Q,
                           uint8_t* masks, hipStream_t s, hipEvent_t* marks = nullptr, uint32_t* grid_out = nullptr,
                           uint32_t* fine_out = nullptr, uint32_t* hist_out = nullptr);
// Enqueue the copy of the nres results (and the check flag) into w's pinned
// mirrors; collect_plan reads them after the stream has been synchronised.
aoresp_status fetch_plan(Workspace& w, const Plan& plan, hipStream_t s);
aoresp_status collect_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid);
// fetch + synchronise + collect.
aoresp_status finish_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid,
                          hipStream_t s);
void release_workspace(Workspace& w);

}  // namespace aoresp
