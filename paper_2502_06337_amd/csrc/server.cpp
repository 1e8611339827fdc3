// Request loop (aoresp_server_*): continuous batching of rotation solves.
//
// Clients submit problems of any size at any time.  A scheduler thread
// (scheduler.h) keeps up to two batches in flight on two streams, each with
// its own workspace: while one batch runs on the device, requests that
// arrived meanwhile are admitted, uploaded and launched on the other stream,
// so their work overlaps on the GPU.  Admission keeps the device bytes both
// pipelines hold (their cached workspaces and batch arrays included) within
// the budget.  Every request is solved by the batched kernels, so its result
// equals est_rotation on the same inputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"
#include "scheduler.h"

using namespace aoresp;
using Clock = std::chrono::steady_clock;

namespace {

// Pinned host blocks in power-of-two size classes, kept for reuse until the
// server is destroyed: a request's inputs are copied once, at submit, into a
// pinned block, and uploaded from there without a staging copy.
class PinnedPool {
  public:
    ~PinnedPool() {
        for (auto& fl : free_)
            for (void* b : fl) (void)hipHostFree(b);
    }
    // A block of at least `bytes`; *cls receives its class (for put).
    void* get(size_t bytes, int* cls) {
        int c = 16;   // 64 KiB minimum
        while (((size_t)1 << c) < bytes) ++c;
        *cls = c;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (c < (int)free_.size() && !free_[c].empty()) {
                void* b = free_[c].back();
                free_[c].pop_back();
                return b;
            }
        }
        void* b = nullptr;
        if (hipHostMalloc(&b, (size_t)1 << c, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return b;
    }
    void put(void* b, int cls) {
        if (!b) return;
        std::lock_guard<std::mutex> lk(mu_);
        if ((int)free_.size() <= cls) free_.resize(cls + 1);
        free_[cls].push_back(b);
    }

  private:
    std::mutex mu_;
    std::vector<std::vector<void*>> free_;
};

// Executor data of one request: its pinned copy of the inputs, its
// parameters and what it adds to each device buffer of a batch.
struct HostReq {
    float* host = nullptr;       // pinned copy: P rows x, y, z then Q rows x, y, z (n floats each)
    int host_cls = 0;
    ResolvedParams rp{};
    // device bytes it adds to each plan buffer (kPlanBuffers, in plan_buffers
    // order), then to the batch's P, Q and mask arrays: an upper bound, since
    // every buffer's size is a sum over instances plus a constant
    size_t need[kPlanBuffers + 3] = {};
};
constexpr int kPipeBufs = kPlanBuffers + 3;

struct Pipeline {
    Workspace ws;
    hipStream_t stream = nullptr;
    DevBuf P, Q, masks;          // batch inputs / outputs on the device
    HostBuf hmask;               // pinned mask staging
    Plan plan;
    hipEvent_t done_ev = nullptr;
    int64_t N = 0;

    // the device buffers of this pipeline, in HostReq::need order
    void buffers(DevBuf** out) {
        BufNeed bn[kPlanBuffers];
        plan_buffers(ws, Plan(), bn);
        for (int i = 0; i < kPlanBuffers; ++i) out[i] = bn[i].buf;
        out[kPlanBuffers] = &P;
        out[kPlanBuffers + 1] = &Q;
        out[kPlanBuffers + 2] = &masks;
    }
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }
// capacity DevBuf::ensure leaves for a need beyond the current one
size_t grown(size_t need) { return need + need / 4 + 256; }

class HipExecutor final : public Executor {
  public:
    DeviceCtx* ctx = nullptr;
    Pipeline pipes[Scheduler::kPipes];
    PinnedPool pool;

    int64_t now_us() override {
        return std::chrono::duration_cast<std::chrono::microseconds>(Clock::now().time_since_epoch()).count();
    }
    size_t held(int p) override {
        DevBuf* b[kPipeBufs];
        pipes[p].buffers(b);
        size_t s = 0;
        for (int i = 0; i < kPipeBufs; ++i) s += b[i]->bytes;
        return s;
    }
    size_t held_after(int p, const std::vector<ReqPtr>& batch, bool exact) override {
        DevBuf* b[kPipeBufs];
        pipes[p].buffers(b);
        size_t s = 0;
        for (int i = 0; i < kPipeBufs; ++i) {
            size_t need = 0;
            for (auto& r : batch) need += static_cast<HostReq*>(r->payload)->need[i];
            if (exact) s += up256(need);
            else s += need <= b[i]->bytes ? b[i]->bytes : grown(need);
        }
        return s;
    }
    void release(int p) override {
        Pipeline& pl = pipes[p];
        release_workspace_buffers(pl.ws);
        pl.P.release();
        pl.Q.release();
        pl.masks.release();
    }
    aoresp_status launch(int p, const std::vector<ReqPtr>& batch, bool exact) override {
        Pipeline& pl = pipes[p];
        DevBuf* b[kPipeBufs];
        pl.buffers(b);
        for (int i = 0; i < kPipeBufs; ++i) b[i]->tight = exact;
        const int nb = (int)batch.size();
        std::vector<int64_t> off(nb + 1, 0);
        std::vector<ResolvedParams> rps(nb);
        std::vector<int> npk(nb, 1);
        for (int k = 0; k < nb; ++k) {
            off[k + 1] = off[k] + (int64_t)batch[k]->n;
            rps[k] = static_cast<HostReq*>(batch[k]->payload)->rp;
        }
        const size_t N = (size_t)off[nb];
        pl.N = (int64_t)N;
        aoresp_status st;
        if ((st = pl.hmask.ensure(N + 16)) != AORESP_OK) return st;
        if ((st = pl.P.ensure(3 * N * 4 + 16)) != AORESP_OK) return st;
        if ((st = pl.Q.ensure(3 * N * 4 + 16)) != AORESP_OK) return st;
        if ((st = pl.masks.ensure(N + 16)) != AORESP_OK) return st;
        // each request's rows go straight from its pinned block into the
        // batch's (3, N) device arrays at its column offset
        for (int k = 0; k < nb; ++k) {
            const HostReq& h = *static_cast<HostReq*>(batch[k]->payload);
            const size_t n = batch[k]->n;
            if (n == 0) continue;
            for (int c = 0; c < 3; ++c) {
                if (hipMemcpyAsync(pl.P.as<float>() + c * N + off[k], h.host + c * n, n * 4, hipMemcpyHostToDevice,
                                   pl.stream) != hipSuccess ||
                    hipMemcpyAsync(pl.Q.as<float>() + c * N + off[k], h.host + (3 + c) * n, n * 4,
                                   hipMemcpyHostToDevice, pl.stream) != hipSuccess)
                    return AORESP_EDEVICE;
            }
        }
        if ((st = build_plan(ctx, off.data(), nb, rps.data(), npk.data(), pl.plan)) != AORESP_OK) return st;
        // the step's pipeline and result copies as one captured graph
        if ((st = launch_plan_graph(ctx, pl.ws, pl.plan, pl.P.as<float>(), pl.Q.as<float>(), pl.masks.as<uint8_t>(),
                                    pl.stream)) != AORESP_OK)
            return st;
        if (hipMemcpyAsync(pl.hmask.ptr, pl.masks.ptr, N, hipMemcpyDeviceToHost, pl.stream) != hipSuccess)
            return AORESP_EDEVICE;
        if (hipEventRecord(pl.done_ev, pl.stream) != hipSuccess) return AORESP_EDEVICE;
        return AORESP_OK;
    }
    int query(int p) override {
        const hipError_t q = hipEventQuery(pipes[p].done_ev);
        if (q == hipSuccess) return 1;
        if (q == hipErrorNotReady) return 0;
        (void)hipGetLastError();
        return -1;
    }
    aoresp_status collect(int p, const std::vector<ReqPtr>& batch) override {
        Pipeline& pl = pipes[p];
        std::vector<aoresp_result> out(pl.plan.nres);
        std::vector<int> valid;
        aoresp_status st = collect_plan(pl.ws, pl.plan, out.data(), valid);
        if (st != AORESP_OK) return st;
        const uint8_t* hm = pl.hmask.as<uint8_t>();
        for (size_t k = 0; k < batch.size(); ++k) {
            SchedRequest& r = *batch[k];
            const int64_t o = pl.plan.insts[k].off;
            r.result = out[k];
            r.mask.assign(hm + o, hm + o + r.n);
            r.status = AORESP_OK;
            if (r.n < 2 || !valid[k]) {
                identity_result(&r.result, static_cast<HostReq*>(r.payload)->rp.G);
                std::fill(r.mask.begin(), r.mask.end(), 0);
                r.status = AORESP_ENODATA;
            }
        }
        return AORESP_OK;
    }
    void drop(SchedRequest& r) override {
        HostReq* h = static_cast<HostReq*>(r.payload);
        if (!h) return;
        pool.put(h->host, h->host_cls);
        delete h;
        r.payload = nullptr;
    }
};

// Per-buffer device bytes of a request alone (an upper bound of what it adds
// to a batch), from its single-instance plan.
aoresp_status request_need(DeviceCtx* ctx, size_t n, const ResolvedParams& rp, size_t* need) {
    Plan plan;
    int64_t off[2] = {0, (int64_t)n};
    int npk = 1;
    aoresp_status st = build_plan(ctx, off, 1, &rp, &npk, plan);
    if (st != AORESP_OK) return st;
    Workspace w;
    BufNeed bn[kPlanBuffers];
    plan_buffers(w, plan, bn);
    for (int i = 0; i < kPlanBuffers; ++i) need[i] = bn[i].bytes;
    need[kPlanBuffers] = 3 * n * 4 + 16;
    need[kPlanBuffers + 1] = 3 * n * 4 + 16;
    need[kPlanBuffers + 2] = n + 16;
    return AORESP_OK;
}

}  // namespace

struct aoresp_server {
    int device = 0;
    size_t budget = 0;
    HipExecutor ex;
    std::unique_ptr<Scheduler> sched;
    std::thread thr;

    void loop() {
        (void)hipSetDevice(device);
        for (;;) {
            const bool progress = sched->step();
            if (sched->drained()) break;
            if (progress) continue;
            if (sched->any_busy()) std::this_thread::sleep_for(std::chrono::microseconds(20));
            else sched->wait_work(50000);
        }
    }
};

extern "C" {

aoresp_status aoresp_server_create(const aoresp_server_cfg* cfg, aoresp_server** out) {
    if (!out) return AORESP_EINVAL;
    auto s = std::make_unique<aoresp_server>();
    aoresp_server_cfg c{};
    if (cfg) c = *cfg;
    if (!c.hbm_budget_bytes) c.hbm_budget_bytes = (size_t)8 << 30;
    if (!c.max_slots) c.max_slots = 256;
    if (hipGetDevice(&s->device) != hipSuccess) return AORESP_EDEVICE;
    s->ex.ctx = device_ctx();
    if (!s->ex.ctx) return AORESP_EDEVICE;
    for (auto& p : s->ex.pipes) {
        if (hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking) != hipSuccess) return AORESP_EDEVICE;
        if (hipEventCreateWithFlags(&p.done_ev, hipEventDisableTiming) != hipSuccess) return AORESP_EDEVICE;
    }
    s->budget = c.hbm_budget_bytes;
    s->sched = std::make_unique<Scheduler>(&s->ex, c.hbm_budget_bytes, c.max_slots, c.timeout_us);
    aoresp_server* raw = s.release();
    raw->thr = std::thread([raw] { raw->loop(); });
    *out = raw;
    return AORESP_OK;
}

aoresp_status aoresp_submit(aoresp_server* s, const float* P, const float* Q, size_t n, const aoresp_params* prm,
                            uint64_t* req_id) {
    if (!s || !req_id || (n > 0 && (!P || !Q)) || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    if (s->sched->stopping()) return AORESP_EINVAL;
    auto h = std::make_unique<HostReq>();
    aoresp_status st = resolve_params(prm, n, h->rp);
    if (st != AORESP_OK) return st;
    if ((st = request_need(s->ex.ctx, n, h->rp, h->need)) != AORESP_OK) return st;
    // the request alone, in a pipeline sized exactly for it
    size_t alone = 0;
    for (int i = 0; i < kPipeBufs; ++i) alone += up256(h->need[i]);
    if (alone > s->budget) return AORESP_ENOMEM;
    if (n) {
        h->host = static_cast<float*>(s->ex.pool.get(6 * n * sizeof(float), &h->host_cls));
        if (!h->host) return AORESP_ENOMEM;
        std::memcpy(h->host, P, 3 * n * sizeof(float));
        std::memcpy(h->host + 3 * n, Q, 3 * n * sizeof(float));
    }
    auto r = std::make_shared<SchedRequest>();
    r->n = n;
    r->payload = h.release();
    *req_id = s->sched->submit(r);
    return AORESP_OK;
}

aoresp_status aoresp_poll(aoresp_server* s, uint64_t req_id, aoresp_result* out, uint8_t* mask, int64_t timeout_us) {
    if (!s) return AORESP_EINVAL;
    return s->sched->poll(req_id, out, mask, timeout_us);
}

aoresp_status aoresp_server_stats(aoresp_server* s, double* p50_us, double* p99_us, double* req_per_s,
                                  uint64_t* completed) {
    if (!s) return AORESP_EINVAL;
    s->sched->stats(p50_us, p99_us, req_per_s, completed);
    return AORESP_OK;
}

void aoresp_server_destroy(aoresp_server* s) {
    if (!s) return;
    s->sched->stop();
    if (s->thr.joinable()) s->thr.join();
    for (int k = 0; k < Scheduler::kPipes; ++k) {
        Pipeline& p = s->ex.pipes[k];
        s->ex.release(k);
        release_workspace(p.ws);
        if (p.hmask.ptr) (void)hipHostFree(p.hmask.ptr);
        p.hmask.ptr = nullptr;
        if (p.done_ev) (void)hipEventDestroy(p.done_ev);
        if (p.stream) (void)hipStreamDestroy(p.stream);
    }
    s->sched.reset();   // requests still in the table drop their pinned blocks into the pool first
    delete s;
}

}  // extern "C"
