// C ABI of libaoresp (include/aoresp.h): parameter checks, per-device
// workspace and tables, and the single / top-k solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <limits>
#include <memory>
#include <vector>

#include "runtime.h"

namespace aoresp {
#include "grid_table.inc"
}

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
    rp.gate = (int)p.angle_gate;
    rp.F = p.angle_refine > 1 ? (int)p.angle_refine : 1;
    rp.rule = (int)p.vote_rule;
    rp.J = p.circle_samples ? (int)p.circle_samples : 8 * rp.G;
    if (!is_pow2((uint32_t)rp.G) || rp.G < 64 || rp.G > 4096) return AORESP_EINVAL;
    if (rp.M != 0 && (!is_pow2((uint32_t)rp.M) || rp.M < 8 || rp.M > 128 || (int64_t)rp.G * rp.M > 262144))
        return AORESP_EINVAL;
    if (rp.w > 8) return AORESP_EINVAL;
    if (rp.B < 2 || rp.B > 8192) return AORESP_EINVAL;
    if (rp.rad > 1024) return AORESP_EINVAL;
    if (!std::isfinite(rp.tau)) return AORESP_EINVAL;
    if (p.angle_gate > 1) return AORESP_EINVAL;
    if (p.angle_refine > 256 || (int64_t)rp.B * rp.F > 65536) return AORESP_EINVAL;
    if (p.vote_rule > 1) return AORESP_EINVAL;
    if (p.circle_samples > 65536 || (p.circle_samples != 0 && p.circle_samples < 4)) return AORESP_EINVAL;
    return AORESP_OK;
}

aoresp_status DevBuf::ensure(size_t need) {
    if (need <= bytes) return AORESP_OK;
    if (fixed) return AORESP_ENOMEM;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    size_t want = tight ? (need + 255) / 256 * 256 : need + need / 4 + 256;
    if (hipMalloc(&ptr, want) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return AORESP_ENOMEM;
    }
    bytes = want;
    return AORESP_OK;
}

void DevBuf::release() {
    if (fixed) return;
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
    init_kernel_attributes();
    DeviceCtx* raw = ctx.get();
    g_ctx[dev] = std::move(ctx);
    return raw;
}

hipStream_t internal_stream(DeviceCtx* ctx) {
    // callers hold ctx->mu
    if (!ctx->ws.stream && hipStreamCreateWithFlags(&ctx->ws.stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->ws.stream = nullptr;
        (void)hipGetLastError();
    }
    return ctx->ws.stream;
}

// Angle tables: boundary k at phi_k = -pi + k * (2 pi / B) and bin centres
// -pi + (k + 1/2) (2 pi / B), evaluated in double and rounded once to float.
// Layout: cos, kDirPad NaNs, sin, kDirPad NaNs, centre angle, cos, sin.
size_t angle_table_floats(int B) { return 5 * (size_t)B + 2 * kDirPad; }

void fill_angle_tables(float* h, int B) {
    const double step = (2.0 * M_PI) / (double)B;
    float* hc = h;
    float* hs = h + B + kDirPad;
    float* hr = hs + B + kDirPad;
    for (int k = 0; k < B; ++k) {
        double phi = -M_PI + (double)k * step;
        hc[k] = (float)std::cos(phi);
        hs[k] = (float)std::sin(phi);
        double ph = -M_PI + ((double)k + 0.5) * step;
        hr[k] = (float)ph;
        hr[B + k] = (float)std::cos(ph);
        hr[2 * B + k] = (float)std::sin(ph);
    }
    for (int k = 0; k < kDirPad; ++k) hc[B + k] = hs[B + k] = std::numeric_limits<float>::quiet_NaN();
}

static AngleTables split_angle_tables(float* d, int B) {
    AngleTables t;
    t.tc = d;
    t.ts = d + B + kDirPad;
    t.th = t.ts + B + kDirPad;
    t.ct = t.th + B;
    t.st = t.th + 2 * B;
    return t;
}

const AngleTables* angle_tables(DeviceCtx* ctx, int B) {
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto it = ctx->angle.find(B);
    if (it != ctx->angle.end()) return &it->second;
    std::vector<float> h(angle_table_floats(B));
    fill_angle_tables(h.data(), B);
    float* d = nullptr;
    if (hipMalloc((void**)&d, h.size() * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return &(ctx->angle[B] = split_angle_tables(d, B));
}

// In-disk cross range of every cell line of a G x G grid over [-1, 1]^2: cell
// (j, k) meets the closed unit disk iff min over its corners of
// u^2 + v^2 - 1 <= 0; with u = (2j - G)/G this is an integer test.
void fill_disk_table(int16_t* h, int G) {
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
}

const int16_t* disk_table(DeviceCtx* ctx, int G) {
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto it = ctx->disk.find(G);
    if (it != ctx->disk.end()) return it->second;
    std::vector<int16_t> h(2 * (size_t)G);
    fill_disk_table(h.data(), G);
    int16_t* d = nullptr;
    if (hipMalloc((void**)&d, h.size() * sizeof(int16_t)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(int16_t), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    ctx->disk[G] = d;
    return d;
}

const AngleTables* TableSink::angle_tables(int B) {
    for (int i = 0; i < nangle; ++i)
        if (angle_B[i] == B) return &angle[i];
    const size_t bytes = (angle_table_floats(B) * sizeof(float) + 255) / 256 * 256;
    if (nangle == 4 || used + bytes > cap) return nullptr;
    fill_angle_tables(reinterpret_cast<float*>(host + used), B);
    angle_B[nangle] = B;
    angle[nangle] = split_angle_tables(reinterpret_cast<float*>(dev + used), B);
    used += bytes;
    return &angle[nangle++];
}

const int16_t* TableSink::disk_table(int G) {
    if (disk) return disk_G == G ? disk : nullptr;
    const size_t bytes = (2 * (size_t)G * sizeof(int16_t) + 255) / 256 * 256;
    if (used + bytes > cap) return nullptr;
    fill_disk_table(reinterpret_cast<int16_t*>(host + used), G);
    disk_G = G;
    disk = reinterpret_cast<const int16_t*>(dev + used);
    used += bytes;
    return disk;
}

aoresp_status HostBuf::ensure(size_t need) {
    if (need <= bytes) return AORESP_OK;
    if (fixed) return AORESP_ENOMEM;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
    size_t want = need + need / 4 + 4096;
    if (hipHostMalloc(&ptr, want, hipHostMallocDefault) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return AORESP_ENOMEM;
    }
    bytes = want;
    return AORESP_OK;
}

// Batch layout.  Coarse vote items: (instance, pass, band, chunk of arcs),
// sized so that one item carries about Tuning::vote_target votes, ordered
// largest first for the persistent work-groups.  Peak items: 8192 cells.  Correspondence
// items (angle histogram): 2048 correspondences; refinement list items: 2048.
static constexpr int kCellChunk = 8192;
static constexpr int kCorrChunk = 2048;
static constexpr int kListChunk = 2048;

int n_bucket(int64_t n) {
    int b = 0;
    while (n >= 2) {
        n >>= 1;
        ++b;
    }
    return b;
}

Tuning tuning_for(DeviceCtx* ctx, int G, int64_t n) {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    auto it = ctx->tune.find({G, n_bucket(n)});
    return it == ctx->tune.end() ? Tuning() : it->second;
}

aoresp_status build_plan(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rps, const int* npk,
                         Plan& plan) {
    return build_plan_with(ctx, off, ninst, rps, npk, nullptr, plan);
}

aoresp_status build_plan_with(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rps, const int* npk,
                              const Tuning* force, Plan& plan, TableSink* tables) {
    auto angle_of = [ctx, tables](int B) { return tables ? tables->angle_tables(B) : angle_tables(ctx, B); };
    plan = Plan();
    plan.insts.resize(ninst);
    std::vector<std::pair<double, int4>> samples;
    // coarse-vote items grouped by chunk of correspondences: (weight, item)
    std::vector<std::vector<std::pair<double, int4>>> chunks;
    size_t hist_lds = 0;
    for (int b = 0; b < ninst; ++b) {
        const ResolvedParams& rp = rps[b];
        Inst& I = plan.insts[b];
        std::memset(&I, 0, sizeof(I));
        I.off = off[b];
        int64_t n = off[b + 1] - off[b];
        if (n < 0 || n > INT32_MAX) return AORESP_EINVAL;
        I.n = (int32_t)n;
        I.G = rp.G;
        I.M = rp.M;
        I.w = rp.w;
        I.B = rp.B;
        I.rad = rp.rad;
        I.tau = rp.tau;
        I.npk = npk[b];
        I.res_off = plan.nres;
        plan.nres += I.npk;
        I.grid_off = (int64_t)plan.grid_cells;
        plan.grid_cells += (size_t)rp.G * rp.G;
        I.lmax_off = (int64_t)plan.lmax_words;
        if (npk[b] > 1) plan.lmax_words += (size_t)rp.G * rp.G / 32;
        I.fine_off = (int64_t)plan.fine_cells;
        plan.fine_cells += (size_t)I.npk * rp.M * rp.M;
        I.hist_off = (int64_t)plan.hist_cells;
        plan.hist_cells += (size_t)I.npk * rp.B;
        I.item0 = (int32_t)plan.corr_items.size();
        I.nitems = 0;
        const AngleTables* at = angle_of(rp.B);
        const int16_t* disk = tables ? tables->disk_table(rp.G) : disk_table(ctx, rp.G);
        if (!at || !disk) return AORESP_ENOMEM;
        I.disk = disk;
        I.tc = at->tc;
        I.ts = at->ts;
        I.th = at->th;
        I.ct = at->ct;
        I.st = at->st;
        if (I.npk > plan.max_npk) plan.max_npk = I.npk;
        if (rp.M > plan.maxM) plan.maxM = rp.M;
        if (rp.G > plan.maxG) plan.maxG = rp.G;
        size_t lds = (size_t)rp.B * 8 + (size_t)I.npk * rp.B * 4;
        if (lds > 160 * 1024) return AORESP_EINVAL;
        if (lds > hist_lds) hist_lds = lds;
        I.gate = rp.gate;
        I.F = rp.F;
        if (rp.F > 1) {
            const AngleTables* ft = angle_of(rp.B * rp.F);
            if (!ft) return AORESP_ENOMEM;
            I.ftc = ft->tc;
            I.fts = ft->ts;
            I.fth = ft->th;
            I.fct = ft->ct;
            I.fst = ft->st;
            I.fhist_off = (int64_t)plan.fhist_cells;   // made absolute below
            plan.fhist_cells += (size_t)I.npk * 3 * rp.F;
            const size_t flds = angle_fine_lds_bytes(I.npk, rp.F);
            if (flds > 160 * 1024) return AORESP_EINVAL;
            if (flds > plan.fhist_lds) plan.fhist_lds = flds;
        }
        I.rule = rp.rule;
        I.J = rp.J;
        if (rp.rule == 1) {
            const AngleTables* sd = angle_of(rp.J);   // cos, sin of -pi + j 2pi/J
            if (!sd) return AORESP_ENOMEM;
            I.scs = sd->tc;
            I.ssn = sd->ts;
            const SampleLayout sl = sample_plan(rp.G, rp.J, n);
            I.sbw = sl.bw;
            I.shalf = sl.half;
            I.sdir_lds = sl.dirs_lds;
            I.snb = rp.G / I.sbw;
            I.schunk = (int32_t)sl.chunk;
            I.ssetup_off = (int64_t)plan.sample_recs;
            plan.sample_recs += (size_t)n;
            I.spart_off = (int64_t)plan.sample_part;
            plan.sample_part += (size_t)sl.part_words;
            if (sl.lds_bytes > plan.sample_lds) plan.sample_lds = sl.lds_bytes;
        }
        // coarse-vote work split: forced (tuner candidate), tuned for (G, n), or default
        const Tuning tu = force ? *force : tuning_for(ctx, rp.G, n);
        const int bw = coarse_band_width(rp.G, tu.tile_cells);
        I.bw = bw;
        if (n == 0) continue;
        int nbands = (rp.G + bw - 1) / bw;
        double per_arc = 1.42 * rp.G / (2.0 * nbands);
        int64_t chunk = (int64_t)(tu.vote_target / per_arc);
        chunk = (chunk + kVoteThreads - 1) / kVoteThreads * kVoteThreads;
        if (chunk < kVoteThreads) chunk = kVoteThreads;
        if (chunk > kMaxItemArcs) chunk = kMaxItemArcs;   // 16-bit tile counters
        if (rp.rule == 1) {
            for (int64_t i0 = 0; i0 < n; i0 += kSampleSetupChunk) {
                int64_t i1 = i0 + kSampleSetupChunk < n ? i0 + kSampleSetupChunk : n;
                plan.sample_setup_items.push_back(make_int4(b, (int)i0, (int)i1, 0));
            }
            // band items, central bands (more samples) first
            for (int band = 0; band < I.snb; ++band)
                for (int64_t i0 = 0; i0 < n; i0 += I.schunk) {
                    int64_t i1 = i0 + I.schunk < n ? i0 + I.schunk : n;
                    double c = (band + 0.5) * I.sbw / (double)rp.G * 2.0 - 1.0;
                    double share = std::sqrt(std::max(0.05, 1.0 - c * c));
                    samples.push_back({share * (double)(i1 - i0), make_int4(b, band, (int)i0, (int)i1)});
                }
        }
        if (rp.rule == 0)
            for (int64_t i0 = 0; i0 < n; i0 += chunk) {
                int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
                chunks.emplace_back();
                for (int mode = 0; mode < 2; ++mode)
                    for (int band = 0; band < nbands; ++band) {
                        // central bands carry more votes: weight by the band's in-disk share
                        double c = (band + 0.5) * bw / (double)rp.G * 2.0 - 1.0;
                        double share = std::sqrt(std::max(0.05, 1.0 - c * c));
                        chunks.back().push_back({per_arc * (double)(i1 - i0) * share,
                                                 make_int4(b, mode | (band << 1), (int)i0, (int)i1)});
                    }
            }
        for (int64_t c0 = 0; c0 < (int64_t)rp.G * rp.G; c0 += kCellChunk) {
            int64_t c1 = c0 + kCellChunk < (int64_t)rp.G * rp.G ? c0 + kCellChunk : (int64_t)rp.G * rp.G;
            plan.cell_items.push_back(make_int4(b, (int)c0, (int)c1, 0));
        }
        for (int64_t i0 = 0; i0 < n; i0 += kCorrChunk) {
            int64_t i1 = i0 + kCorrChunk < n ? i0 + kCorrChunk : n;
            plan.corr_items.push_back(make_int4(b, (int)i0, (int)i1, 0));
        }
        I.nitems = (int)plan.corr_items.size() - I.item0;
        if (rp.M > 0)
            for (int64_t i0 = 0; i0 < n; i0 += kListChunk) {
                int64_t i1 = i0 + kListChunk < n ? i0 + kListChunk : n;
                plan.list_items.push_back(make_int4(b, (int)i0, (int)i1, 0));
            }
    }
    for (Inst& I : plan.insts) I.fhist_off += (int64_t)plan.hist_cells;
    // Coarse-vote queues, one per XCD: chunks (largest first) go to the
    // least-loaded queue; a queue lists its chunks one after the other, each
    // chunk's band items largest first, so that the work-groups of an XCD
    // take the bands of the same correspondences at the same time.
    auto heavier = [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) { return x.first > y.first; };
    std::vector<std::pair<double, int>> order;
    for (size_t c = 0; c < chunks.size(); ++c) {
        std::stable_sort(chunks[c].begin(), chunks[c].end(), heavier);
        double wsum = 0.0;
        for (auto& v : chunks[c]) wsum += v.first;
        order.push_back({wsum, (int)c});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first > y.first; });
    std::vector<int> queue_of(chunks.size(), 0);
    double load[kVoteQueues] = {};
    for (auto& o : order) {
        int q = 0;
        for (int k = 1; k < kVoteQueues; ++k)
            if (load[k] < load[q]) q = k;
        queue_of[o.second] = q;
        load[q] += o.first;
    }
    for (int q = 0; q < kVoteQueues; ++q) {
        plan.vote_q.first[q] = (int32_t)plan.vote_items.size();
        for (auto& o : order)
            if (queue_of[o.second] == q)
                for (auto& v : chunks[o.second]) plan.vote_items.push_back(v.second);
    }
    plan.vote_q.first[kVoteQueues] = (int32_t)plan.vote_items.size();
    std::stable_sort(samples.begin(), samples.end(),
                     [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) { return x.first > y.first; });
    for (auto& v : samples) plan.sample_items.push_back(v.second);
    plan.N = off[ninst];
    plan.hist_lds = hist_lds;
    return AORESP_OK;
}

// Bytes of the uploaded blob: instance table (padded to 256 B), then the
// vote, cell, correspondence and list items.
size_t plan_blob_bytes(const Plan& plan) {
    const size_t b_inst = plan.insts.size() * sizeof(Inst);
    const size_t o_vote = (b_inst + 255) / 256 * 256;
    return o_vote + (plan.vote_items.size() + plan.cell_items.size() + plan.corr_items.size() +
                     plan.list_items.size() + plan.sample_setup_items.size() + plan.sample_items.size()) *
                        sizeof(int4) + 16;
}

aoresp_status enqueue_plan(DeviceCtx* ctx, Workspace& w, const Plan& plan, const float* P, const float* Q,
                           uint8_t* masks, hipStream_t s, hipEvent_t* marks, uint32_t* grid_out, uint32_t* fine_out,
                           uint32_t* hist_out) {
    const int64_t N = plan.N;
    const int ninst = (int)plan.insts.size();
    aoresp_status st;
    auto mark = [&](int k) {
        if (marks) (void)hipEventRecord(marks[k], s);
    };
    if ((st = reserve_plan(w, plan)) != AORESP_OK) return st;
    ++w.gen;
    const OutLayout ol(plan.nres);
    // instance table and work items, uploaded as one blob
    const size_t b_inst = (size_t)ninst * sizeof(Inst);
    const size_t o_vote = (b_inst + 255) / 256 * 256;
    const size_t o_cell = o_vote + plan.vote_items.size() * sizeof(int4);
    const size_t o_corr = o_cell + plan.cell_items.size() * sizeof(int4);
    const size_t o_list = o_corr + plan.corr_items.size() * sizeof(int4);
    const size_t o_sset = o_list + plan.list_items.size() * sizeof(int4);
    const size_t o_samp = o_sset + plan.sample_setup_items.size() * sizeof(int4);
    const size_t total = plan_blob_bytes(plan);
    char* hb = w.h_plan.as<char>();
    std::memcpy(hb, plan.insts.data(), b_inst);
    if (!plan.vote_items.empty())
        std::memcpy(hb + o_vote, plan.vote_items.data(), plan.vote_items.size() * sizeof(int4));
    if (!plan.cell_items.empty())
        std::memcpy(hb + o_cell, plan.cell_items.data(), plan.cell_items.size() * sizeof(int4));
    if (!plan.corr_items.empty())
        std::memcpy(hb + o_corr, plan.corr_items.data(), plan.corr_items.size() * sizeof(int4));
    if (!plan.list_items.empty())
        std::memcpy(hb + o_list, plan.list_items.data(), plan.list_items.size() * sizeof(int4));
    if (!plan.sample_setup_items.empty())
        std::memcpy(hb + o_sset, plan.sample_setup_items.data(), plan.sample_setup_items.size() * sizeof(int4));
    if (!plan.sample_items.empty())
        std::memcpy(hb + o_samp, plan.sample_items.data(), plan.sample_items.size() * sizeof(int4));
    AOR_HIP(hipMemcpyAsync(w.plan.ptr, hb, total, hipMemcpyHostToDevice, s));
    char* db = w.plan.as<char>();
    const Inst* insts = reinterpret_cast<const Inst*>(db);
    const int4* vote_items = reinterpret_cast<const int4*>(db + o_vote);
    const int4* cell_items = reinterpret_cast<const int4*>(db + o_cell);
    const int4* corr_items = reinterpret_cast<const int4*>(db + o_corr);
    const int4* list_items = reinterpret_cast<const int4*>(db + o_list);
    const int4* sample_setup_items = reinterpret_cast<const int4*>(db + o_sset);
    const int4* sample_items = reinterpret_cast<const int4*>(db + o_samp);

    ArcRecs R{w.abc.as<float4>(), w.colp.as<int4>(), w.rowp.as<int4>(), w.geo.as<int4>()};
    char* ob = w.out.as<char>();
    PeakState* stt = reinterpret_cast<PeakState*>(ob + ol.o_st);
    aoresp_result* res = reinterpret_cast<aoresp_result*>(ob + ol.o_res);
    unsigned long long* keys = w.keys.as<unsigned long long>();
    uint32_t* err = reinterpret_cast<uint32_t*>(ob + ol.o_err);
    uint32_t* counters = err + 1;   // kVoteQueues of them, zeroed with the out region

    mark(0);
    // every accumulator and flag of the plan starts at zero: one launch
    ZeroList zl{};
    auto zero = [&zl](void* p, size_t words) {
        zl.ptr[zl.count] = static_cast<uint32_t*>(p);
        zl.words[zl.count] = words;
        ++zl.count;
    };
    zero(w.out.ptr, ol.bytes / 4);
    zero(keys, (size_t)plan.nres * 2);
    zero(w.grid.ptr, plan.grid_cells);
    zero(w.fine.ptr, plan.maxM > 0 ? plan.fine_cells : 0);
    zero(w.hist.ptr, plan.hist_cells + plan.fhist_cells);
    zero(w.icount.ptr, (size_t)plan.nres * kCountSlots);
    launch_zero_list(zl, s);
    launch_arc_setup(P, Q, N, insts, ninst, R, s);
    mark(1);
    launch_vote(R, insts, vote_items, plan.vote_q, counters, w.grid.as<uint32_t>(), err,
                ctx->cu_count, s);
    launch_sample_vote(P, Q, N, insts, sample_setup_items, (int)plan.sample_setup_items.size(), sample_items,
                       (int)plan.sample_items.size(), cell_items, (int)plan.cell_items.size(), w.srec.as<uint32_t>(),
                       w.spart.as<uint32_t>(), w.grid.as<uint32_t>(), plan.sample_lds, s);
    mark(2);
    if (plan.max_npk > 1)
        launch_local_max(w.grid.as<uint32_t>(), insts, cell_items, (int)plan.cell_items.size(), w.lmax.as<uint32_t>(),
                         plan.maxG, s);
    for (int t = 0; t < plan.max_npk; ++t) {
        launch_peak(w.grid.as<uint32_t>(), insts, cell_items, (int)plan.cell_items.size(), stt, t,
                    w.lmax.as<uint32_t>(), keys, s);
        launch_peak_finish(insts, ninst, keys, stt, t, s);
    }
    mark(3);
    for (int t = 0; t < plan.max_npk; ++t) {
        if (plan.maxM > 0) {
            launch_fine_vote(R, insts, list_items, (int)plan.list_items.size(), stt, t, w.fine.as<uint32_t>(), err,
                             plan.maxM, s);
        }
        launch_fine_peak(w.fine.as<uint32_t>(), insts, ninst, stt, t, s);
    }
    mark(4);
    launch_angle_hist(P, Q, N, insts, corr_items, (int)plan.corr_items.size(), stt, w.hist.as<uint32_t>(),
                      plan.hist_lds, s);
    for (int t = 0; t < plan.max_npk; ++t) launch_angle_peak(w.hist.as<uint32_t>(), insts, ninst, stt, t, res, s);
    if (plan.fhist_lds > 0) {
        launch_angle_fine_hist(P, Q, N, insts, corr_items, (int)plan.corr_items.size(), stt, res,
                               w.hist.as<uint32_t>(), plan.fhist_lds, s);
        for (int t = 0; t < plan.max_npk; ++t)
            launch_angle_fine_peak(w.hist.as<uint32_t>(), insts, ninst, stt, t, res, s);
    }
    mark(5);
    launch_inliers(P, Q, N, insts, ninst, stt, res, plan.nres, masks, w.icount.as<uint32_t>(), s);
    for (int t = 0; t < plan.max_npk; ++t) {
        launch_ls_accum(P, Q, N, insts, corr_items, (int)plan.corr_items.size(), stt, res, t, w.lsum.as<double>(), s);
        launch_ls_finish(insts, ninst, w.lsum.as<double>(), stt, res, t, s);
    }
    mark(6);
    if (ninst == 1) {
        const Inst& I = plan.insts[0];
        if (grid_out)
            AOR_HIP(hipMemcpyAsync(grid_out, w.grid.ptr, (size_t)I.G * I.G * 4, hipMemcpyDeviceToDevice, s));
        if (fine_out && I.M > 0)
            AOR_HIP(hipMemcpyAsync(fine_out, w.fine.ptr, plan.fine_cells * 4, hipMemcpyDeviceToDevice, s));
        if (hist_out) AOR_HIP(hipMemcpyAsync(hist_out, w.hist.ptr, plan.hist_cells * 4, hipMemcpyDeviceToDevice, s));
    }
    AOR_HIP(hipGetLastError());
    return AORESP_OK;
}

aoresp_status fetch_plan(Workspace& w, const Plan& plan, hipStream_t s) {
    const OutLayout ol(plan.nres);
    aoresp_status st;
    if ((st = w.h_out.ensure(ol.bytes)) != AORESP_OK) return st;
    // results, peak states and the flag in one copy
    AOR_HIP(hipMemcpyAsync(w.h_out.ptr, w.out.ptr, ol.o_err + sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    return AORESP_OK;
}

aoresp_status collect_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid) {
    const OutLayout ol(plan.nres);
    const char* hb = w.h_out.as<char>();
    const uint32_t* herr = reinterpret_cast<const uint32_t*>(hb + ol.o_err);
    if (*herr) {
        if (debug_on()) fprintf(stderr, "aoresp: internal check flag 0x%x\n", *herr);
        return AORESP_EDEVICE;
    }
    const aoresp_result* hr = reinterpret_cast<const aoresp_result*>(hb + ol.o_res);
    const PeakState* hs = reinterpret_cast<const PeakState*>(hb + ol.o_st);
    valid.assign(plan.nres, 0);
    for (int t = 0; t < plan.nres; ++t) {
        out[t] = hr[t];
        valid[t] = hs[t].valid ? 1 : 0;
    }
    return AORESP_OK;
}

aoresp_status finish_plan(Workspace& w, const Plan& plan, aoresp_result* out, std::vector<int>& valid,
                          hipStream_t s) {
    aoresp_status st = fetch_plan(w, plan, s);
    if (st != AORESP_OK) return st;
    AOR_HIP(hipStreamSynchronize(s));
    return collect_plan(w, plan, out, valid);
}

// Record the whole plan (pipeline + result copies) into one graph by stream
// capture and launch it on s.  Every buffer is sized by a first, eager pass
// over the allocation steps (enqueue_plan's ensure calls are then no-ops), so
// nothing allocates while the stream is captured.  The executable graph is
// kept in the workspace and updated in place when the next plan has the same
// topology; otherwise it is instantiated again.
aoresp_status launch_plan_graph(DeviceCtx* ctx, Workspace& w, const Plan& plan, const float* P, const float* Q,
                                uint8_t* masks, hipStream_t s) {
    aoresp_status st;
    if ((st = reserve_plan(w, plan)) != AORESP_OK) return st;
    if (!w.cap_stream && hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking) != hipSuccess)
        return AORESP_EDEVICE;
    if (hipStreamBeginCapture(w.cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return AORESP_EDEVICE;
    aoresp_status rec = enqueue_plan(ctx, w, plan, P, Q, masks, w.cap_stream);
    if (rec == AORESP_OK) rec = fetch_plan(w, plan, w.cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(w.cap_stream, &graph);
    if (rec != AORESP_OK || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rec != AORESP_OK ? rec : AORESP_EDEVICE;
    }
    bool updated = false;
    if (w.gexec) {
        hipGraphExecUpdateResult how;
        hipGraphNode_t bad_node = nullptr;
        updated = hipGraphExecUpdate(w.gexec, graph, &bad_node, &how) == hipSuccess && how == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(w.gexec);
            w.gexec = nullptr;
        }
    }
    if (!updated && hipGraphInstantiate(&w.gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        w.gexec = nullptr;
        return AORESP_EDEVICE;
    }
    (void)hipGraphDestroy(graph);
    AOR_HIP(hipGraphLaunch(w.gexec, s));
    return AORESP_OK;
}

std::vector<uint64_t> plan_key(DeviceCtx* ctx, const int64_t* off, int ninst, const ResolvedParams* rps,
                               const int* npk, const float* P, const float* Q, const uint8_t* masks) {
    std::vector<uint64_t> key;
    key.reserve(4 + 7 * (size_t)ninst);
    key.push_back((uint64_t)ninst);
    key.push_back((uint64_t)(uintptr_t)P);
    key.push_back((uint64_t)(uintptr_t)Q);
    key.push_back((uint64_t)(uintptr_t)masks);
    for (int b = 0; b < ninst; ++b) {
        const ResolvedParams& r = rps[b];
        uint32_t tau_bits;
        std::memcpy(&tau_bits, &r.tau, 4);
        const Tuning tu = tuning_for(ctx, r.G, off[b + 1] - off[b]);
        uint64_t vt;
        std::memcpy(&vt, &tu.vote_target, 8);
        key.push_back((uint64_t)off[b + 1] | (uint64_t)npk[b] << 40);
        key.push_back((uint64_t)r.G | (uint64_t)r.M << 16 | (uint64_t)r.w << 32 | (uint64_t)r.rad << 40);
        key.push_back((uint64_t)r.B | (uint64_t)r.F << 16 | (uint64_t)r.gate << 40 | (uint64_t)r.rule << 48);
        key.push_back((uint64_t)r.J | (uint64_t)tau_bits << 32);
        key.push_back((uint64_t)tu.tile_cells);
        key.push_back(vt);
    }
    return key;
}

aoresp_status run_plan(DeviceCtx* ctx, Workspace& w, std::vector<uint64_t>&& key, const int64_t* off, int ninst,
                       const ResolvedParams* rps, const int* npk, const float* P, const float* Q, uint8_t* masks,
                       hipStream_t s, Plan& scratch, const Plan** used) {
    aoresp_status st;
    if (w.gexec && w.gen == w.replay_gen && key == w.replay_key) {
        AOR_HIP(hipGraphLaunch(w.gexec, s));
        *used = &w.replay_plan;
        return AORESP_OK;
    }
    const bool again = w.gen == w.last_gen && key == w.last_key;
    if ((st = build_plan(ctx, off, ninst, rps, npk, scratch)) != AORESP_OK) return st;
    if (again) {
        // the same layout twice in a row: record it for the calls to come
        w.replay_key.clear();
        if ((st = launch_plan_graph(ctx, w, scratch, P, Q, masks, s)) != AORESP_OK) return st;
        w.replay_key = std::move(key);
        w.replay_gen = w.gen;
        w.replay_plan = std::move(scratch);
        w.last_key.clear();
        *used = &w.replay_plan;
        return AORESP_OK;
    }
    if ((st = enqueue_plan(ctx, w, scratch, P, Q, masks, s)) != AORESP_OK) return st;
    if ((st = fetch_plan(w, scratch, s)) != AORESP_OK) return st;
    w.last_key = std::move(key);
    w.last_gen = w.gen;
    *used = &scratch;
    return AORESP_OK;
}

void plan_buffers(Workspace& w, const Plan& plan, BufNeed* out) {
    const size_t nn = plan.N > 0 ? (size_t)plan.N : 1;
    const OutLayout ol(plan.nres);
    const BufNeed list[kPlanBuffers] = {
        {&w.abc, nn * sizeof(float4)},
        {&w.colp, nn * sizeof(int4)},
        {&w.rowp, nn * sizeof(int4)},
        {&w.geo, nn * sizeof(int4)},
        {&w.grid, plan.grid_cells * 4 + 4},
        {&w.fine, plan.fine_cells * 4 + 4},
        {&w.hist, (plan.hist_cells + plan.fhist_cells) * 4 + 4},
        {&w.keys, (size_t)plan.nres * 8},
        {&w.lmax, plan.lmax_words * 4 + 4},
        {&w.out, ol.bytes},
        {&w.icount, (size_t)plan.nres * kCountSlots * 4},
        {&w.lsum, (plan.corr_items.size() + 1) * kLsWords * sizeof(double)},
        {&w.srec, plan.sample_recs * kSampleRec * 4 + 4},
        {&w.spart, plan.sample_part * 4 + 4},
        {&w.plan, plan_blob_bytes(plan)},
    };
    for (int i = 0; i < kPlanBuffers; ++i) out[i] = list[i];
}

// All device and pinned buffers a plan needs (the allocation half of
// enqueue_plan and fetch_plan).
aoresp_status reserve_plan(Workspace& w, const Plan& plan) {
    BufNeed need[kPlanBuffers];
    plan_buffers(w, plan, need);
    aoresp_status st;
    for (int i = 0; i < kPlanBuffers; ++i)
        if ((st = need[i].buf->ensure(need[i].bytes)) != AORESP_OK) return st;
    const OutLayout ol(plan.nres);
    if ((st = w.h_out.ensure(ol.bytes)) != AORESP_OK) return st;
    if ((st = w.h_plan.ensure(plan_blob_bytes(plan))) != AORESP_OK) return st;
    return AORESP_OK;
}

void release_workspace(Workspace& w) {
    if (w.gexec) (void)hipGraphExecDestroy(w.gexec);
    w.gexec = nullptr;
    if (w.cap_stream) (void)hipStreamDestroy(w.cap_stream);
    w.cap_stream = nullptr;
    release_workspace_buffers(w);
}

void release_workspace_buffers(Workspace& w) {
    DevBuf* bufs[] = {&w.abc, &w.colp, &w.rowp, &w.geo, &w.grid, &w.fine, &w.hist, &w.keys, &w.lmax, &w.out,
                      &w.icount, &w.lsum, &w.srec, &w.spart, &w.plan, &w.P, &w.Q, &w.masks};
    for (DevBuf* b : bufs) b->release();
    HostBuf* hb[] = {&w.h_plan, &w.h_out};
    for (HostBuf* b : hb) {
        if (b->fixed) continue;
        if (b->ptr) (void)hipHostFree(b->ptr);
        b->ptr = nullptr;
        b->bytes = 0;
    }
}

void identity_result(aoresp_result* r, int G) {
    std::memset(r, 0, sizeof(*r));
    r->R[0] = r->R[4] = r->R[8] = 1.0f;
    r->R_ls[0] = r->R_ls[4] = r->R_ls[8] = 1.0f;
    r->grid = (uint32_t)G;
}

// Single instance with k peaks on device pointers.
aoresp_status solve_dev_common(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                               aoresp_result* out, uint8_t* masks, uint32_t* k_found, uint32_t* grid_out,
                               uint32_t* fine_out, uint32_t* hist_out, hipStream_t s, hipEvent_t* marks) {
    if (!out || (n > 0 && (!P || !Q)) || k < 1 || k > (uint32_t)kMaxPeaks) return AORESP_EINVAL;
    if (n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    if ((size_t)rp.B * 8 + (size_t)k * rp.B * 4 > 160 * 1024) return AORESP_EINVAL;
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
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = (int)k;
    std::vector<int> valid;
    if (marks || grid_out || fine_out || hist_out) {
        // stage marks or debug copies: an eager run
        if ((st = build_plan(ctx, off, 1, &rp, &npk, plan)) != AORESP_OK) return st;
        if ((st = enqueue_plan(ctx, ctx->ws, plan, P, Q, masks, s, marks, grid_out, fine_out, hist_out)) != AORESP_OK)
            return st;
        if ((st = finish_plan(ctx->ws, plan, out, valid, s)) != AORESP_OK) return st;
    } else {
        const Plan* used = nullptr;
        if ((st = run_plan(ctx, ctx->ws, plan_key(ctx, off, 1, &rp, &npk, P, Q, masks), off, 1, &rp, &npk, P, Q, masks,
                           s, plan, &used)) != AORESP_OK)
            return st;
        AOR_HIP(hipStreamSynchronize(s));
        if ((st = collect_plan(ctx->ws, *used, out, valid)) != AORESP_OK) return st;
    }
    uint32_t found = 0;
    while (found < k && valid[found]) ++found;
    if (k_found) *k_found = found;
    if (found == 0) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        return AORESP_ENODATA;
    }
    return AORESP_OK;
}

static aoresp_status solve_host_common(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                       aoresp_result* out, uint8_t* masks, uint32_t* k_found) {
    if (!out || (n > 0 && (!P || !Q)) || k < 1 || k > (uint32_t)kMaxPeaks) return AORESP_EINVAL;
    if (n > (size_t)INT32_MAX) return AORESP_EINVAL;
    ResolvedParams rp;
    aoresp_status st = resolve_params(prm, n, rp);
    if (st != AORESP_OK) return st;
    if ((size_t)rp.B * 8 + (size_t)k * rp.B * 4 > 160 * 1024) return AORESP_EINVAL;
    if (n < 2) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        if (k_found) *k_found = 0;
        if (masks && n) std::memset(masks, 0, n * k);
        return AORESP_ENODATA;
    }
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Workspace& w = ctx->ws;
    hipStream_t s = internal_stream(ctx);
    if (!s) return AORESP_EDEVICE;
    if ((st = w.P.ensure(3 * n * sizeof(float))) != AORESP_OK) return st;
    if ((st = w.Q.ensure(3 * n * sizeof(float))) != AORESP_OK) return st;
    if (masks && (st = w.masks.ensure(n * k)) != AORESP_OK) return st;
    AOR_HIP(hipMemcpyAsync(w.P.ptr, P, 3 * n * sizeof(float), hipMemcpyHostToDevice, s));
    AOR_HIP(hipMemcpyAsync(w.Q.ptr, Q, 3 * n * sizeof(float), hipMemcpyHostToDevice, s));
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = (int)k;
    if ((st = build_plan(ctx, off, 1, &rp, &npk, plan)) != AORESP_OK) return st;
    if ((st = enqueue_plan(ctx, ctx->ws, plan, w.P.as<float>(), w.Q.as<float>(), masks ? w.masks.as<uint8_t>() : nullptr, s)) !=
        AORESP_OK)
        return st;
    if (masks) AOR_HIP(hipMemcpyAsync(masks, w.masks.ptr, n * k, hipMemcpyDeviceToHost, s));
    std::vector<int> valid;
    if ((st = finish_plan(ctx->ws, plan, out, valid, s)) != AORESP_OK) return st;
    uint32_t found = 0;
    while (found < k && valid[found]) ++found;
    if (k_found) *k_found = found;
    if (found == 0) {
        for (uint32_t t = 0; t < k; ++t) identity_result(&out[t], rp.G);
        if (masks) std::memset(masks, 0, n * k);
        return AORESP_ENODATA;
    }
    return AORESP_OK;
}

}  // namespace aoresp

using namespace aoresp;

extern "C" {

uint32_t aoresp_grid_for_n(uint64_t n) {
    // the autotuned table, by size bucket floor(log2 n)
    int b = 0;
    while (n >= 2) {
        n >>= 1;
        ++b;
    }
    int i = b - kGridTableFirst;
    const int last = (int)(sizeof(kGridTable) / sizeof(kGridTable[0])) - 1;
    i = i < 0 ? 0 : (i > last ? last : i);
    return (uint32_t)kGridTable[i];
}

aoresp_status est_rotation(const float* P, const float* Q, size_t n, const aoresp_params* prm, aoresp_result* out,
                           uint8_t* inlier_mask) {
    return solve_host_common(P, Q, n, 1, prm, out, inlier_mask, nullptr);
}

aoresp_status est_rotation_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm, aoresp_result* out,
                               uint8_t* inlier_mask, void* hip_stream) {
    return solve_dev_common(P, Q, n, 1, prm, out, inlier_mask, nullptr, nullptr, nullptr, nullptr,
                            (hipStream_t)hip_stream, nullptr);
}

aoresp_status est_rotations_topk(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                 aoresp_result* out, uint8_t* masks, uint32_t* k_found) {
    return solve_host_common(P, Q, n, k, prm, out, masks, k_found);
}

aoresp_status est_rotations_topk_dev(const float* P, const float* Q, size_t n, uint32_t k, const aoresp_params* prm,
                                     aoresp_result* out, uint8_t* masks, uint32_t* k_found, void* hip_stream) {
    return solve_dev_common(P, Q, n, k, prm, out, masks, k_found, nullptr, nullptr, nullptr,
                            (hipStream_t)hip_stream, nullptr);
}

aoresp_status aoresp_solve_debug_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     aoresp_result* out, uint8_t* inlier_mask, uint32_t* grid_out, uint32_t* fine_out,
                                     uint32_t* hist_out, void* hip_stream) {
    return solve_dev_common(P, Q, n, 1, prm, out, inlier_mask, nullptr, grid_out, fine_out, hist_out,
                            (hipStream_t)hip_stream, nullptr);
}

aoresp_status aoresp_coarse_grid_dev(const float* P, const float* Q, size_t n, uint32_t G, uint32_t* grid,
                                     void* hip_stream) {
    if (!grid || (n > 0 && (!P || !Q)) || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    if (!is_pow2(G) || G < 64 || G > 4096) return AORESP_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    // a single correspondence still votes: n = 1 runs the vote path like any n
    aoresp_params prm{};
    prm.grid = G;
    aoresp_result out;
    if (n == 0) {
        launch_zero_u32(grid, (size_t)G * G, s);
        AOR_HIP(hipGetLastError());
        AOR_HIP(hipStreamSynchronize(s));
        return AORESP_OK;
    }
    // the full single solve writes its coarse grid into `grid`
    ResolvedParams rp;
    aoresp_status st = resolve_params(&prm, n, rp);
    if (st != AORESP_OK) return st;
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return AORESP_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = 1;
    if ((st = build_plan(ctx, off, 1, &rp, &npk, plan)) != AORESP_OK) return st;
    if ((st = enqueue_plan(ctx, ctx->ws, plan, P, Q, nullptr, s, nullptr, grid, nullptr, nullptr)) != AORESP_OK) return st;
    std::vector<int> valid;
    st = finish_plan(ctx->ws, plan, &out, valid, s);
    return st;
}

aoresp_status aoresp_stage_times_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     float* ms_out, uint32_t* n_stages, void* hip_stream) {
    if (!ms_out || !n_stages || n < 2 || !P || !Q || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[kNumStages + 1];
    for (int k = 0; k <= kNumStages; ++k) AOR_HIP(hipEventCreate(&ev[k]));
    aoresp_result tmp;
    aoresp_status st = solve_dev_common(P, Q, n, 1, prm, &tmp, nullptr, nullptr, nullptr, nullptr, nullptr, s, ev);
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
