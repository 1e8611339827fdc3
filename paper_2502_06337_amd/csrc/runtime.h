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
    int gate, F;   // angle gate on/off; fine angle factor (1 = none)
    int rule, J;   // coarse accumulator rule (0 per-cell, 1 sampling); samples per circle
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

// Growable device buffer, or (fixed) a view of caller-provided memory whose
// ensure() never allocates and fails with ENOMEM beyond its size.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
    bool tight = false;   // grow to the need exactly (else with a quarter of headroom)
    aoresp_status ensure(size_t need);
    void release();
    template <class T>
    T* as() const { return static_cast<T*>(ptr); }
};

// Growable pinned host buffer, or (fixed) a view of caller-provided host memory.
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
    aoresp_status ensure(size_t need);
    template <class T>
    T* as() const { return static_cast<T*>(ptr); }
};

// Angle tables of B bins (angle_table_floats(B) floats: boundary cos and sin,
// each followed by kDirPad NaNs; centre angle, cos, sin) and the in-disk cross
// ranges of a G x G grid (2 G int16), written into host memory.
size_t angle_table_floats(int B);
void fill_angle_tables(float* h, int B);
void fill_disk_table(int16_t* h, int G);

// Where build_plan takes its device tables from when not from the per-device
// caches: an image in host memory at `host`, to be copied by the caller to the
// device address `dev` before the plan runs (a single-instance plan uses at
// most 3 angle-table sizes and one disk table).
struct TableSink {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0, used = 0;
    int nangle = 0;
    int angle_B[4] = {0, 0, 0, 0};
    AngleTables angle[4];
    int disk_G = 0;
    const int16_t* disk = nullptr;
    const AngleTables* angle_tables(int B);
    const int16_t* disk_table(int G);
};

// A plan's outputs in one device buffer (and its pinned mirror), so that one
// copy brings them back: results, peak states, then the internal-check flag
// and the coarse vote's work counter.
struct OutLayout {
    size_t o_res, o_st, o_err, bytes;
    explicit OutLayout(int nres) {
        auto up = [](size_t b) { return (b + 15) / 16 * 16; };
        o_res = 0;
        o_st = up((size_t)nres * sizeof(aoresp_result));
        o_err = o_st + up((size_t)nres * sizeof(PeakState));
        bytes = o_err + 64;   // flag, then the coarse vote's kVoteQueues work counters
    }
};

// A batch laid out for the kernels.
struct Plan {
    std::vector<Inst> insts;
    std::vector<int4> vote_items, cell_items, corr_items, list_items;
    VoteQueues vote_q;         // vote_items in kVoteQueues consecutive queues
    std::vector<int4> sample_setup_items, sample_items;   // sampling rule: circle records, band items
    int64_t N = 0;
    size_t grid_cells = 0, fine_cells = 0, hist_cells = 0;
    size_t fhist_cells = 0;    // fine-angle windows, after the histograms in the same arena
    int nres = 0;              // result slots (sum of npk)
    int max_npk = 0, maxM = 0, maxG = 0;
    size_t hist_lds = 0;
    size_t fhist_lds = 0;      // 0: no instance refines its angle
    size_t sample_lds = 0;     // LDS of the sampling band pass (0: no instance uses the sampling rule)
    size_t sample_recs = 0;    // circle records of the sampling rule
    size_t sample_part = 0;    // u32 cells of its partial tiles
    size_t lmax_words = 0;     // local-maximum bitmaps (G*G/32 words per instance with npk > 1)
};

// Everything a batch enqueues into.
struct Workspace {
    DevBuf abc, colp, rowp, geo;    // per global column
    DevBuf grid, fine, hist;        // arenas
    DevBuf keys;                    // per result slot: peak search keys
    DevBuf lmax;                    // local-maximum bitmaps of instances with several peaks
    DevBuf out;                     // results, peak states, flag and counter (OutLayout)
    DevBuf icount;                  // partial inlier counters (kCountSlots per result slot)
    DevBuf lsum;                    // least-squares sums per correspondence item (kLsWords doubles)
    DevBuf srec, spart;             // sampling rule: circle records, partial band tiles
    DevBuf plan;                    // instance table + work items
    DevBuf P, Q, masks;             // staging for host-pointer entry points
    HostBuf h_plan, h_out;          // pinned mirrors
    hipStream_t stream = nullptr;   // internal stream for host-pointer calls
    hipStream_t cap_stream = nullptr;   // stream that batched plans are captured on
    hipGraphExec_t gexec = nullptr;     // last captured plan, updated in place when the topology repeats
    uint64_t gen = 0;                   // bumped by every enqueue_plan into this workspace
    // A batched call kept for replay: the key it was recorded for (offsets,
    // resolved parameters, work splits, device pointers), the workspace
    // generation right after recording, and its plan.  A later call with the
    // same key and no other use of the workspace in between launches gexec
    // again without planning or capturing.
    std::vector<uint64_t> replay_key;
    uint64_t replay_gen = 0;
    Plan replay_plan;
    std::vector<uint64_t> last_key;     // key of the last call run eagerly (recorded if it comes again)
    uint64_t last_gen = 0;
};


// Work split of the coarse vote for one (G, n bucket): LDS tile cells and
// votes per work item.  Any choice gives the same grid; only speed differs.
struct Tuning {
    int tile_cells = kTileCells;
    double vote_target = 3.0e6;
    float vote_ms = -1.0f;   // measured coarse-vote time of this choice (-1: default, not measured)
};
int n_bucket(int64_t n);     // floor(log2(n)), 0 for n < 2

struct DeviceCtx {
    int device = 0;
    int cu_count = 256;
    std::mutex mu;                      // serialises use of `ws`
    Workspace ws;
    std::map<int, AngleTables> angle;   // by B
    std::map<int, int16_t*> disk;       // by G
    std::mutex table_mu;
    std::map<std::pair<int, int>, Tuning> tune;   // by (G, n bucket)
    std::mutex tune_mu;
};

Tuning tuning_for(DeviceCtx* ctx, int G, int64_t n);

DeviceCtx* device_ctx();            // context of the current HIP device (creates no stream)
hipStream_t internal_stream(DeviceCtx* ctx);   // its stream for host-pointer calls, created on first use
const AngleTables* angle_tables(DeviceCtx* ctx, int B);
const int16_t* disk_table(DeviceCtx* ctx, int G);

// Instance b owns global columns [off[b], off[b+1]).
aoresp_status build_plan(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rp, const int* npk,
                         Plan& plan);
// The same with the coarse-vote work split forced (autotuner candidates).
aoresp_status build_plan_with(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rp, const int* npk,
                              const Tuning* force, Plan& plan, TableSink* tables = nullptr);
// Single solve on device pointers with optional stage events (kNumStages + 1).
aoresp_status solve_dev_common(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                               aoresp_result* out, uint8_t* masks, uint32_t* k_found, uint32_t* grid_out,
                               uint32_t* fine_out, uint32_t* hist_out, hipStream_t s, hipEvent_t* marks);

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
// R = R_ls = I, zero counts, grid G: the result of a solve without data.
void identity_result(aoresp_result* r, int G);
aoresp_status collect_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid);
// fetch + synchronise + collect.
aoresp_status finish_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid,
                          hipStream_t s);
void release_workspace(Workspace& w);
void release_workspace_buffers(Workspace& w);   // device and pinned buffers only
// Allocation half of enqueue_plan + fetch_plan; size of the uploaded blob.
aoresp_status reserve_plan(Workspace& w, const Plan& plan);
// The device buffers of reserve_plan with the bytes each needs for `plan`
// (kPlanBuffers entries, in a fixed order).
constexpr int kPlanBuffers = 15;
struct BufNeed {
    DevBuf* buf;
    size_t bytes;
};
void plan_buffers(Workspace& w, const Plan& plan, BufNeed* out);
size_t plan_blob_bytes(const Plan& plan);
// What a recorded plan depends on: offsets, peaks per instance, resolved
// parameters, the coarse vote's work split per instance and the device
// pointers of the inputs and masks.
std::vector<uint64_t> plan_key(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rps,
                               const int* npk, const float* P, const float* Q, const uint8_t* masks);
// Run a plan's pipeline and result copy on s (caller holds ctx->mu):
// a call whose key equals the one recorded last in w, with no other use of w
// in between, launches the recorded graph again without planning; one whose
// key equals the previous eager call's is planned, recorded and launched;
// any other is planned and enqueued directly.  *used points to the plan the
// results are read with (valid until the next call on w).
aoresp_status run_plan(DeviceCtx* ctx, Workspace& w, std::vector<uint64_t>&& key, const int64_t* off, int ninst,
                       const ResolvedParams* rps, const int* npk, const float* P, const float* Q, uint8_t* masks,
                       hipStream_t s, Plan& scratch, const Plan** used);
// enqueue_plan + fetch_plan captured into one hipGraph and launched on s
// (caller holds ctx->mu; no stage marks or debug copies).
aoresp_status launch_plan_graph(DeviceCtx* ctx, Workspace& w, const Plan& plan, const float* P, const float* Q,
                                uint8_t* masks, hipStream_t s);

}  // namespace aoresp
