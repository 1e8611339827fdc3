// C ABI of libaoresp (include/aoresp.h): parameter checks, per-device
// workspace and tables, and the single / top-k solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "runtime.h"

namespace aoresp {

// Set AORESP_DEBUG=1 to print the HIP error behind an AORESP_EDEVICE.
static bool debug_on() {
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("AORESP_DEBUG");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

static aoresp_status hip_fail(hipError_t e, const char* what, int line) {
    if (debug_on()) fprintf(stderr, "aoresp: %s failed at api.cpp:%d: %s\n", what, line, hipGetErrorString(e));
    return AORESP_EDEVICE;
}

#define AOR_HIP(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__); \
    } while (0)

static bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

aoresp_status resolve_params(const aoresp_params* prm, size_t n, ResolvedParams& rp) {
    aoresp_params p{};
    if (prm) p = *prm;
    rp.G = p.grid ? (int)p.grid : (int)aoresp_grid_for_n(n);
    rp.M = (int)p.refine_grid;
    rp.w = p.refine_halfwin ? (int)p.refine_halfwin : 1;
    rp.B = p.angle_bins ? (int)p.angle_bins : 360;
    rp.rad = p.nms_radius ? (int)p.nms_radius : 5;
    rp.tau = p.inlier_thresh > 0.0f ? p.inlier_thresh : 0.05f;
    if (!is_pow2((uint32_t)rp.G) || rp.G < 64 || rp.G > 4096) return AORESP_EINVAL;
    if (rp.M != 0 && (!is_pow2((uint32_t)rp.M) || rp.M < 8 || rp.M > 128 || (int64_t)rp.G * rp.M > 262144))
        return AORESP_EINVAL;
    if (rp.w > 8) return AORESP_EINVAL;
    if (rp.B < 2 || rp.B > 8192) return AORESP_EINVAL;
    if (rp.rad > 1024) return AORESP_EINVAL;
    if (!std::isfinite(rp.tau)) return AORESP_EINVAL;
    return AORESP_OK;
}

aoresp_status DevBuf::ensure(size_t need) {
    if (need <= bytes) return AORESP_OK;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    size_t want = need + need / 4 + 256;
    if (hipMalloc(&ptr, want) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return AORESP_ENOMEM;
    }
    bytes = want;
    return AORESP_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

static std::mutex g_ctx_mu;
static std::map<int, std::unique_ptr<DeviceCtx>> g_ctx;

DeviceCtx* device_ctx() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto it = g_ctx.find(dev);
    if (it != g_ctx.end()) return it->second.get();
    auto ctx = std::make_unique<DeviceCtx>();
    ctx->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ctx->cu_count = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&ctx->buf.stream, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipHostMalloc((void**)&ctx->buf.h_res, sizeof(aoresp_result) * kMaxPeaks, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&ctx->buf.h_st, sizeof(PeakState) * kMaxPeaks, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ctx->buf.h_err, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
        return nullptr;
    DeviceCtx* raw = ctx.get();
    g_ctx[dev] = std::move(ctx);
    return raw;
}

// Angle tables: boundary k at phi_k = -pi + k * (2 pi / B) and bin centres
// -pi + (k + 1/2) (2 pi / B), evaluated in double and rounded once to float.
const AngleTables* angle_tables(DeviceCtx* ctx, int B) {
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto it = ctx->angle.find(B);
    if (it != ctx->angle.end()) return &it->second;
    std::vector<float> h(5 * (size_t)B);
    const double step = (2.0 * M_PI) / (double)B;
    for (int k = 0; k < B; ++k) {
        double phi = -M_PI + (double)k * step;
        h[k] = (float)std::cos(phi);
        h[B + k] = (float)std::sin(phi);
        double ph = -M_PI + ((double)k + 0.5) * step;
        h[2 * B + k] = (float)ph;
        h[3 * B + k] = (float)std::cos(ph);
        h[4 * B + k] = (float)std::sin(ph);
    }
    float* d = nullptr;
    if (hipMalloc((void**)&d, h.size() * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    AngleTables t;
    t.tc = d;
    t.ts = d + B;
    t.th = d + 2 * B;
    t.ct = d + 3 * B;
    t.st = d + 4 * B;
    return &(ctx->angle[B] = t);
}

// In-disk cross range of every cell line of a G x G grid over [-1, 1]^2: cell
// (j, k) meets the closed unit disk iff min over its corners of
// u^2 + v^2 - 1 <= 0; with u = (2j - G)/G this is an integer test.
const int16_t* disk_table(DeviceCtx* ctx, int G) {
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto it = ctx->disk.find(G);
    if (it != ctx->disk.end()) return it->second;
    std::vector<int16_t> h(2 * (size_t)G);
    auto mind = [G](int j) {
        long a = std::labs(2L * j - G), b = std::labs(2L * j + 2 - G);
        return a < b ? a : b;
    };
    const long GG = (long)G * G;
    for (int j = 0; j < G; ++j) {
        long mu = mind(j);
        int lo = G, hi = -1;
        for (int k = 0; k < G; ++k) {
            long mv = mind(k);
            if (mu * mu + mv * mv <= GG) {
                if (k < lo) lo = k;
                hi = k;
            }
        }
        h[2 * j] = (int16_t)lo;
        h[2 * j + 1] = (int16_t)hi;
    }
    int16_t* d = nullptr;
    if (hipMalloc((void**)&d, h.size() * sizeof(int16_t)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(int16_t), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    ctx->disk[G] = d;
    return d;
}

// Work split of the coarse vote: enough (band, chunk) work-groups to cover the
// chip twice, without chunks smaller than a few thousand correspondences.
int coarse_chunks(DeviceCtx* ctx, int64_t n, int G) {
    int bw = coarse_band_width(G);
    int nbands = (G + bw - 1) / bw;
    int target = 2 * ctx->cu_count;
    int ch = (target + 2 * nbands - 1) / (2 * nbands);
    int64_t maxch = (n + 4095) / 4096;
    if (ch > maxch) ch = (int)maxch;
    if (ch < 1) ch = 1;
    return ch;
}

aoresp_status enqueue_solve(DeviceCtx* ctx, const float* P, const float* Q, int64_t n, const ResolvedParams& rp,
                            int npk, uint8_t* masks, uint32_t* grid_out, uint32_t* fine_out, uint32_t* hist_out,
                            hipStream_t s, hipEvent_t* marks) {
    SolveBuffers& b = ctx->buf;
    auto mark = [&](int k) {
        if (marks) (void)hipEventRecord(marks[k], s);
    };
    const int G = rp.G, M = rp.M, B = rp.B;
    aoresp_status st;
    if ((st = b.abc.ensure((size_t)n * sizeof(float4))) != AORESP_OK) return st;
    if ((st = b.colp.ensure((size_t)n * sizeof(int4))) != AORESP_OK) return st;
    if ((st = b.rowp.ensure((size_t)n * sizeof(int4))) != AORESP_OK) return st;
    if ((st = b.clip.ensure((size_t)n * sizeof(int32_t))) != AORESP_OK) return st;
    if ((st = b.grid.ensure((size_t)G * G * 4)) != AORESP_OK) return st;
    if ((st = b.fine.ensure((size_t)kMaxPeaks * (M > 0 ? M * M : 1) * 4)) != AORESP_OK) return st;
    if ((st = b.hist.ensure((size_t)kMaxPeaks * B * 4)) != AORESP_OK) return st;
    if ((st = b.keys.ensure(kMaxPeaks * sizeof(unsigned long long))) != AORESP_OK) return st;
    if ((st = b.st.ensure(kMaxPeaks * sizeof(PeakState))) != AORESP_OK) return st;
    if ((st = b.res.ensure(kMaxPeaks * sizeof(aoresp_result))) != AORESP_OK) return st;
    if ((st = b.err.ensure(sizeof(uint32_t))) != AORESP_OK) return st;
    const AngleTables* at = angle_tables(ctx, B);
    const int16_t* disk = disk_table(ctx, G);
    if (!at || !disk) return AORESP_ENOMEM;
    ArcRecs R{b.abc.as<float4>(), b.colp.as<int4>(), b.rowp.as<int4>(), b.clip.as<int32_t>()};
    PeakState* stt = b.st.as<PeakState>();
    aoresp_result* res = b.res.as<aoresp_result>();
    uint32_t* fine = b.fine.as<uint32_t>();
    uint32_t* hist = b.hist.as<uint32_t>();
    unsigned long long* keys = b.keys.as<unsigned long long>();

    mark(0);
    launch_zero_u32(b.err.as<uint32_t>(), 1, s);
    launch_zero_u32(reinterpret_cast<uint32_t*>(keys), 2 * kMaxPeaks, s);
    launch_zero_u32(reinterpret_cast<uint32_t*>(stt), kMaxPeaks * sizeof(PeakState) / 4, s);
    launch_zero_u32(reinterpret_cast<uint32_t*>(res), kMaxPeaks * sizeof(aoresp_result) / 4, s);
    launch_arc_setup(P, Q, n, G, R, s);
    launch_zero_u32(b.grid.as<uint32_t>(), (size_t)G * G, s);
    mark(1);
    launch_coarse_vote(R, n, G, disk, b.grid.as<uint32_t>(), b.err.as<uint32_t>(), coarse_chunks(ctx, n, G), s);
    mark(2);
    for (int t = 0; t < npk; ++t) {
        launch_peak(b.grid.as<uint32_t>(), G, (int64_t)G * G, stt, t, rp.rad, keys + t, s);
        launch_peak_finish(keys + t, G, M, rp.w, stt, t, s);
    }
    mark(3);
    if (M > 0) launch_zero_u32(fine, (size_t)npk * M * M, s);
    for (int t = 0; t < npk; ++t) {
        if (M > 0) launch_fine_vote(R, n, M, stt, t, fine + (size_t)t * M * M, b.err.as<uint32_t>(), s);
        launch_fine_peak(fine + (size_t)t * (M > 0 ? M * M : 0), G, M, stt, t, s);
    }
    mark(4);
    launch_zero_u32(hist, (size_t)npk * B, s);
    // histograms of several peaks share one pass while the LDS allows it
    int per = (int)((160 * 1024 - (size_t)B * 8) / ((size_t)B * 4));
    if (per < 1) return AORESP_EINVAL;
    for (int t0 = 0; t0 < npk; t0 += per) {
        int cnt = npk - t0 < per ? npk - t0 : per;
        launch_angle_hist(P, Q, n, stt + t0, cnt, B, at->tc, at->ts, hist + (size_t)t0 * B, s);
    }
    for (int t = 0; t < npk; ++t) launch_angle_peak(hist, B, at->th, at->ct, at->st, stt, t, G, res, s);
    mark(5);
    launch_inliers(P, Q, n, stt, npk, rp.tau, res, masks, s);
    mark(6);
    if (grid_out)
        AOR_HIP(hipMemcpyAsync(grid_out, b.grid.ptr, (size_t)G * G * 4, hipMemcpyDeviceToDevice, s));
    if (fine_out && M > 0)
        AOR_HIP(hipMemcpyAsync(fine_out, fine, (size_t)npk * M * M * 4, hipMemcpyDeviceToDevice, s));
    if (hist_out) AOR_HIP(hipMemcpyAsync(hist_out, hist, (size_t)npk * B * 4, hipMemcpyDeviceToDevice, s));
    AOR_HIP(hipGetLastError());
    return AORESP_OK;
}

aoresp_status finish_solve(DeviceCtx* ctx, int npk, aoresp_result* out, uint32_t* k_found, hipStream_t s) {
    SolveBuffers& b = ctx->buf;
    AOR_HIP(hipMemcpyAsync(b.h_res, b.res.ptr, sizeof(aoresp_result) * npk, hipMemcpyDeviceToHost, s));
    AOR_HIP(hipMemcpyAsync(b.h_st, b.st.ptr, sizeof(PeakState) * npk, hipMemcpyDeviceToHost, s));
    AOR_HIP(hipMemcpyAsync(b.h_err, b.err.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    AOR_HIP(hipStreamSynchronize(s));
    if (*b.h_err) {
        if (debug_on()) fprintf(stderr, "aoresp: internal check flag 0x%x\n", *b.h_err);
        return AORESP_EDEVICE;
    }
    uint32_t found = 0;
    for (int t = 0; t < npk; ++t) {
        out[t] = b.h_res[t];
        if (b.h_st[t].valid) ++found;
    }
    if (k_found) *k_found = found;
    return found ? AORESP_OK : AORESP_ENODATA;
}

static void identity_result(aoresp_result* r, int G) {
    std::memset(r, 0, sizeof(*r));
    r->R[0] = r->R[4] = r->R[8] = 1.0f;
    r->grid = (uint32_t)G;
}

static aoresp_status solve_dev_common(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                      aoresp_result* out, uint8_t* masks, uint32_t* k_found, uint32_t* grid_out,
                                      uint32_t* fine_out, uint32_t* hist_out, hipStream_t s) {
    if (!out || (n > 0 && (!P || !Q)) || k < 1 || k > (uint32_t)kMaxPeaks) return AORESP_EINVAL;
    if (n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    if (n < 2) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        if (k_found) *k_found = 0;
        if (masks && n) {
            if (hipMemsetAsync(masks, 0, n * k, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
                return AORESP_EDEVICE;
        }
        return AORESP_ENODATA;
    }
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    st = enqueue_solve(ctx, P, Q, (int64_t)n, rp, (int)k, masks, grid_out, fine_out, hist_out, s);
    if (st != AORESP_OK) return st;
    st = finish_solve(ctx, (int)k, out, k_found, s);
    if (st == AORESP_ENODATA)
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
    return st;
}

static aoresp_status solve_host_common(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                       aoresp_result* out, uint8_t* masks, uint32_t* k_found) {
    if (!out || (n > 0 && (!P || !Q)) || k < 1 || k > (uint32_t)kMaxPeaks) return AORESP_EINVAL;
    if (n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    if (n < 2) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        if (k_found) *k_found = 0;
        if (masks && n) std::memset(masks, 0, n * k);
        return AORESP_ENODATA;
    }
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    SolveBuffers& b = ctx->buf;
    hipStream_t s = b.stream;
    if ((st = b.P.ensure(3 * n * sizeof(float))) != AORESP_OK) return st;
    if ((st = b.Q.ensure(3 * n * sizeof(float))) != AORESP_OK) return st;
    if (masks && (st = b.masks.ensure(n * k)) != AORESP_OK) return st;
    AOR_HIP(hipMemcpyAsync(b.P.ptr, P, 3 * n * sizeof(float), hipMemcpyHostToDevice, s));
    AOR_HIP(hipMemcpyAsync(b.Q.ptr, Q, 3 * n * sizeof(float), hipMemcpyHostToDevice, s));
    st = enqueue_solve(ctx, b.P.as<float>(), b.Q.as<float>(), (int64_t)n, rp, (int)k,
                       masks ? b.masks.as<uint8_t>() : nullptr, nullptr, nullptr, nullptr, s);
    if (st != AORESP_OK) return st;
    if (masks) AOR_HIP(hipMemcpyAsync(masks, b.masks.ptr, n * k, hipMemcpyDeviceToHost, s));
    st = finish_solve(ctx, (int)k, out, k_found, s);
    if (st == AORESP_ENODATA) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        if (masks) std::memset(masks, 0, n * k);
    }
    return st;
}

}  // namespace aoresp

using namespace aoresp;

extern "C" {

uint32_t aoresp_grid_for_n(uint64_t n) {
    if (n < 2000) return 128;
    if (n < 20000) return 256;
    if (n < 200000) return 512;
    return 1024;
}

aoresp_status est_rotation(const float* P, const float* Q, size_t n, const aoresp_params* prm, aoresp_result* out,
                           uint8_t* inlier_mask) {
    return solve_host_common(P, Q, n, 1, prm, out, inlier_mask, nullptr);
}

aoresp_status est_rotation_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm, aoresp_result* out,
                               uint8_t* inlier_mask, void* hip_stream) {
    return solve_dev_common(P, Q, n, 1, prm, out, inlier_mask, nullptr, nullptr, nullptr, nullptr,
                            (hipStream_t)hip_stream);
}

aoresp_status est_rotations_topk(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                 aoresp_result* out, uint8_t* masks, uint32_t* k_found) {
    return solve_host_common(P, Q, n, k, prm, out, masks, k_found);
}

aoresp_status est_rotations_topk_dev(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                     aoresp_result* out, uint8_t* masks, uint32_t* k_found, void* hip_stream) {
    return solve_dev_common(P, Q, n, k, prm, out, masks, k_found, nullptr, nullptr, nullptr,
                            (hipStream_t)hip_stream);
}

aoresp_status aoresp_solve_debug_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     aoresp_result* out, uint8_t* inlier_mask, uint32_t* grid_out, uint32_t* fine_out,
                                     uint32_t* hist_out, void* hip_stream) {
    return solve_dev_common(P, Q, n, 1, prm, out, inlier_mask, nullptr, grid_out, fine_out, hist_out,
                            (hipStream_t)hip_stream);
}

aoresp_status aoresp_coarse_grid_dev(const float* P, const float* Q, size_t n, uint32_t G, uint32_t* grid,
                                     void* hip_stream) {
    if (!grid || (n > 0 && (!P || !Q)) || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    if (!is_pow2(G) || G < 64 || G > 4096) return AORESP_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    SolveBuffers& b = ctx->buf;
    aoresp_status st;
    size_t nn = n ? n : 1;
    if ((st = b.abc.ensure(nn * sizeof(float4))) != AORESP_OK) return st;
    if ((st = b.colp.ensure(nn * sizeof(int4))) != AORESP_OK) return st;
    if ((st = b.rowp.ensure(nn * sizeof(int4))) != AORESP_OK) return st;
    if ((st = b.clip.ensure(nn * sizeof(int32_t))) != AORESP_OK) return st;
    if ((st = b.err.ensure(sizeof(uint32_t))) != AORESP_OK) return st;
    const int16_t* disk = disk_table(ctx, (int)G);
    if (!disk) return AORESP_ENOMEM;
    ArcRecs R{b.abc.as<float4>(), b.colp.as<int4>(), b.rowp.as<int4>(), b.clip.as<int32_t>()};
    launch_zero_u32(b.err.as<uint32_t>(), 1, s);
    launch_zero_u32(grid, (size_t)G * G, s);
    if (n) {
        launch_arc_setup(P, Q, (int64_t)n, (int)G, R, s);
        launch_coarse_vote(R, (int64_t)n, (int)G, disk, grid, b.err.as<uint32_t>(), coarse_chunks(ctx, n, G), s);
    }
    AOR_HIP(hipGetLastError());
    AOR_HIP(hipMemcpyAsync(b.h_err, b.err.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    AOR_HIP(hipStreamSynchronize(s));
    if (*b.h_err && debug_on()) fprintf(stderr, "aoresp: internal check flag 0x%x\n", *b.h_err);
    return *b.h_err ? AORESP_EDEVICE : AORESP_OK;
}

aoresp_status aoresp_stage_times_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     float* ms_out, uint32_t* n_stages, void* hip_stream) {
    if (!ms_out || !n_stages || n < 2 || !P || !Q || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipEvent_t ev[kNumStages + 1];
    for (int k = 0; k <= kNumStages; ++k) AOR_HIP(hipEventCreate(&ev[k]));
    st = enqueue_solve(ctx, P, Q, (int64_t)n, rp, 1, nullptr, nullptr, nullptr, nullptr, s, ev);
    aoresp_result tmp;
    if (st == AORESP_OK) st = finish_solve(ctx, 1, &tmp, nullptr, s);
    if (st == AORESP_OK || st == AORESP_ENODATA) {
        for (int k = 0; k < kNumStages; ++k) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) ms = -1.0f;
            ms_out[k] = ms;
        }
        *n_stages = kNumStages;
    }
    for (int k = 0; k <= kNumStages; ++k) (void)hipEventDestroy(ev[k]);
    return st;
}

const char* aoresp_strerror(aoresp_status st) {
    switch (st) {
        case AORESP_OK: return "ok";
        case AORESP_EINVAL: return "invalid argument";
        case AORESP_ENOMEM: return "out of device memory or budget";
        case AORESP_EDEVICE: return "device error or internal check failed";
        case AORESP_ENODATA: return "no data: fewer than two correspondences or no vote";
        case AORESP_EBUSY: return "request not finished";
        case AORESP_ETIMEDOUT: return "request timed out";
    }
    return "unknown status";
}

const char* aoresp_version(void) { return "aoresp 0.1 gfx950"; }

}  // extern "C"
