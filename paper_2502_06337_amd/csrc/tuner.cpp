// Autotuner of the coarse vote's work split.  For a (G, n bucket) it times
// the coarse-vote stage of one solve on the caller's data under each
// candidate (LDS tile size x votes per work item), keeps the fastest in the
// per-device table that build_plan consults, and can save and load that
// table as JSON lines.  The grid resolution is not tuned here, at run time:
// G is the caller's choice or aoresp_grid_for_n(n), a table fixed when the
// library is built (from the offline sweep of tune_grid.py), so results never
// depend on tuning, batch composition or machine.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace aoresp;

namespace {

const int kTiles[] = {16384, 32768, 65536};
const double kTargets[] = {0.75e6, 1.5e6, 3.0e6, 6.0e6};

// Coarse-vote time (ms) of one solve of (P, Q) with the work split forced.
aoresp_status time_candidate(DeviceCtx* ctx, const float* P, const float* Q, size_t n, const ResolvedParams& rp,
                             const Tuning& tu, hipStream_t s, hipEvent_t* ev, float* ms) {
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = 1;
    aoresp_status st = build_plan_with(ctx, off, 1, &rp, &npk, &tu, plan);
    if (st != AORESP_OK) return st;
    if ((st = enqueue_plan(ctx, ctx->ws, plan, P, Q, nullptr, s, ev)) != AORESP_OK) return st;
    std::vector<int> valid;
    std::vector<aoresp_result> out(plan.nres);
    if ((st = finish_plan(ctx->ws, plan, out.data(), valid, s)) != AORESP_OK) return st;
    if (hipEventElapsedTime(ms, ev[kStageCoarse], ev[kStageCoarse + 1]) != hipSuccess) return AORESP_EDEVICE;
    return AORESP_OK;
}

}  // namespace

extern "C" {

aoresp_status aoresp_autotune_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                  aoresp_tuning* chosen, void* hip_stream) {
    if (!P || !Q || n < 2 || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[kNumStages + 1];
    for (int k = 0; k <= kNumStages; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) return AORESP_EDEVICE;
    Tuning best;
    best.vote_ms = -1.0f;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        // one untimed run so that buffers and tables exist before timing
        Tuning dflt;
        float ms = 0.0f;
        st = time_candidate(ctx, P, Q, n, rp, dflt, s, ev, &ms);
        for (int ti = 0; st == AORESP_OK && ti < (int)(sizeof(kTiles) / sizeof(kTiles[0])); ++ti) {
            for (int vi = 0; st == AORESP_OK && vi < (int)(sizeof(kTargets) / sizeof(kTargets[0])); ++vi) {
                Tuning tu;
                tu.tile_cells = kTiles[ti];
                tu.vote_target = kTargets[vi];
                float m = 0.0f;
                st = time_candidate(ctx, P, Q, n, rp, tu, s, ev, &m);
                if (st == AORESP_OK && (best.vote_ms < 0.0f || m < best.vote_ms)) {
                    best = tu;
                    best.vote_ms = m;
                }
            }
        }
    }
    for (int k = 0; k <= kNumStages; ++k) (void)hipEventDestroy(ev[k]);
    if (st != AORESP_OK && st != AORESP_ENODATA) return st;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        ctx->tune[{rp.G, n_bucket((int64_t)n)}] = best;
    }
    if (chosen) {
        chosen->grid = (uint32_t)rp.G;
        chosen->n_bucket = (uint32_t)n_bucket((int64_t)n);
        chosen->tile_cells = (uint32_t)best.tile_cells;
        chosen->vote_target = (float)best.vote_target;
        chosen->vote_ms = best.vote_ms;
    }
    return AORESP_OK;
}

aoresp_status aoresp_tuner_get(uint32_t grid, uint64_t n, aoresp_tuning* out) {
    if (!out) return AORESP_EINVAL;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    Tuning tu = tuning_for(ctx, (int)grid, (int64_t)n);
    out->grid = grid;
    out->n_bucket = (uint32_t)n_bucket((int64_t)n);
    out->tile_cells = (uint32_t)tu.tile_cells;
    out->vote_target = (float)tu.vote_target;
    out->vote_ms = tu.vote_ms;
    return AORESP_OK;
}

aoresp_status aoresp_tuner_save(const char* path) {
    if (!path) return AORESP_EINVAL;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    FILE* f = std::fopen(path, "w");
    if (!f) return AORESP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    for (const auto& kv : ctx->tune)
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"grid\": %d, \"n_bucket\": %d, \"tile_cells\": %d, \"vote_target\": %.6g, "
                     "\"vote_ms\": %.6g}\n",
                     arch.c_str(), kv.first.first, kv.first.second, kv.second.tile_cells, kv.second.vote_target,
                     (double)kv.second.vote_ms);
    std::fclose(f);
    return AORESP_OK;
}

// Reads what aoresp_tuner_save writes (one object per line, keys in that
// order); entries for another architecture and malformed lines are skipped.
aoresp_status aoresp_tuner_load(const char* path) {
    if (!path) return AORESP_EINVAL;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    FILE* f = std::fopen(path, "r");
    if (!f) return AORESP_EINVAL;
    char line[512], a[128];
    int G, b, tile;
    double target, ms;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line,
                        " {\"arch\": \"%127[^\"]\", \"grid\": %d, \"n_bucket\": %d, \"tile_cells\": %d, "
                        "\"vote_target\": %lf, \"vote_ms\": %lf}",
                        a, &G, &b, &tile, &target, &ms) != 6)
            continue;
        if (arch != a) continue;
        if (tile < 1024 || tile > kTileCells || (tile & (tile - 1)) || target < 1e4 || target > 1e9) continue;
        Tuning tu;
        tu.tile_cells = tile;
        tu.vote_target = target;
        tu.vote_ms = (float)ms;
        ctx->tune[{G, b}] = tu;
    }
    std::fclose(f);
    return AORESP_OK;
}

aoresp_status aoresp_tuner_clear(void) {
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tune.clear();
    return AORESP_OK;
}

}  // extern "C"
