// Request loop (aoresp_server_*): continuous batching of rotation solves.
//
// Clients submit problems of any size at any time.  A scheduler thread keeps
// up to two batches in flight on two streams, each with its own workspace:
// while one batch runs on the device, requests that arrived meanwhile are
// admitted (as long as the device bytes of everything admitted stay within
// the budget and a batch has a free slot), uploaded and launched on the other
// stream, so their work overlaps on the GPU.  Every request is solved by the
// batched kernels, so its result equals est_rotation on the same inputs.
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

struct Request {
    uint64_t id = 0;
    float* host = nullptr;       // pinned copy: P rows x, y, z then Q rows x, y, z (n floats each)
    int host_cls = 0;
    size_t n = 0;
    ResolvedParams rp{};
    size_t bytes = 0;            // device bytes while admitted
    Clock::time_point t_submit;
    Clock::time_point deadline;
    bool has_deadline = false;
    // completion
    bool done = false;
    aoresp_status status = AORESP_EBUSY;
    aoresp_result result{};
    std::vector<uint8_t> mask;
    double latency_us = 0.0;
};

struct Pipeline {
    Workspace ws;
    hipStream_t stream = nullptr;
    DevBuf P, Q, masks;          // batch inputs / outputs on the device
    HostBuf hmask;               // pinned mask staging
    std::vector<std::shared_ptr<Request>> reqs;
    Plan plan;
    hipEvent_t done_ev = nullptr;
    bool busy = false;
    size_t bytes = 0;
};

// Device bytes a request holds while in a batch: inputs, per-correspondence
// records, mask, its coarse grid, fine grid, histograms and, under the
// sampling rule, its circle records and partial band tiles.
size_t request_bytes(size_t n, const ResolvedParams& rp) {
    size_t b = n * (24 + 64 + 1) + (size_t)rp.G * rp.G * 4 + (size_t)rp.M * rp.M * 4 + (size_t)rp.B * 4 + 4096;
    if (rp.F > 1) b += (size_t)rp.F * 3 * 4;
    if (rp.rule == 1 && n > 0) b += n * kSampleRec * 4 + (size_t)sample_plan(rp.G, rp.J, (int64_t)n).part_words * 4;
    return b;
}

}  // namespace

struct aoresp_server {
    aoresp_server_cfg cfg{};
    int device = 0;
    DeviceCtx* ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv_work;   // scheduler wake-up
    std::condition_variable cv_done;   // poll wake-up
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
    uint64_t next_id = 1;
    bool stopping = false;
    size_t bytes_in_flight = 0;
    Pipeline pipes[2];
    PinnedPool pool;
    std::thread thr;
    // stats
    std::vector<double> lat_us;
    uint64_t completed = 0;
    Clock::time_point t_first, t_last;
    bool any = false;
    aoresp_status fatal = AORESP_OK;

    void complete(const std::shared_ptr<Request>& r, aoresp_status st) {
        r->status = st;
        r->done = true;
        auto now = Clock::now();
        r->latency_us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
        lat_us.push_back(r->latency_us);
        ++completed;
        if (!any) {
            t_first = r->t_submit;
            any = true;
        }
        if (r->t_submit < t_first) t_first = r->t_submit;
        t_last = now;
        pool.put(r->host, r->host_cls);
        r->host = nullptr;
    }

    // Launch one batch on pipeline p from the head of the queue (mu held).
    // Returns false if nothing could be admitted.
    bool launch(Pipeline& p, std::unique_lock<std::mutex>& lk) {
        std::vector<std::shared_ptr<Request>> batch;
        size_t bytes = 0;
        auto now = Clock::now();
        while (!queue.empty() && batch.size() < cfg.max_slots) {
            auto& r = queue.front();
            if (r->has_deadline && now > r->deadline) {
                complete(r, AORESP_ETIMEDOUT);
                queue.pop_front();
                continue;
            }
            if (bytes_in_flight + bytes + r->bytes > cfg.hbm_budget_bytes) break;
            bytes += r->bytes;
            batch.push_back(r);
            queue.pop_front();
        }
        if (!batch.empty()) cv_done.notify_all();
        if (batch.empty()) return false;
        bytes_in_flight += bytes;
        p.bytes = bytes;
        p.reqs = std::move(batch);
        lk.unlock();
        aoresp_status st = upload_and_enqueue(p);
        lk.lock();
        if (st != AORESP_OK) {
            for (auto& r : p.reqs) complete(r, st);
            bytes_in_flight -= p.bytes;
            p.reqs.clear();
            cv_done.notify_all();
            return true;
        }
        p.busy = true;
        return true;
    }

    aoresp_status upload_and_enqueue(Pipeline& p) {
        const int nb = (int)p.reqs.size();
        std::vector<int64_t> off(nb + 1, 0);
        std::vector<ResolvedParams> rps(nb);
        std::vector<int> npk(nb, 1);
        for (int b = 0; b < nb; ++b) {
            off[b + 1] = off[b] + (int64_t)p.reqs[b]->n;
            rps[b] = p.reqs[b]->rp;
        }
        const size_t N = (size_t)off[nb];
        aoresp_status st;
        if ((st = p.hmask.ensure(N + 16)) != AORESP_OK) return st;
        if ((st = p.P.ensure(3 * N * 4 + 16)) != AORESP_OK) return st;
        if ((st = p.Q.ensure(3 * N * 4 + 16)) != AORESP_OK) return st;
        if ((st = p.masks.ensure(N + 16)) != AORESP_OK) return st;
        // each request's rows go straight from its pinned block into the
        // batch's (3, N) device arrays at its column offset
        for (int b = 0; b < nb; ++b) {
            const Request& r = *p.reqs[b];
            if (r.n == 0) continue;
            for (int c = 0; c < 3; ++c) {
                if (hipMemcpyAsync(p.P.as<float>() + c * N + off[b], r.host + c * r.n, r.n * 4,
                                   hipMemcpyHostToDevice, p.stream) != hipSuccess ||
                    hipMemcpyAsync(p.Q.as<float>() + c * N + off[b], r.host + (3 + c) * r.n, r.n * 4,
                                   hipMemcpyHostToDevice, p.stream) != hipSuccess)
                    return AORESP_EDEVICE;
            }
        }
        if ((st = build_plan(ctx, off.data(), nb, rps.data(), npk.data(), p.plan)) != AORESP_OK) return st;
        // the step's pipeline and result copies as one captured graph
        if ((st = launch_plan_graph(ctx, p.ws, p.plan, p.P.as<float>(), p.Q.as<float>(), p.masks.as<uint8_t>(),
                                    p.stream)) != AORESP_OK)
            return st;
        if (hipMemcpyAsync(p.hmask.ptr, p.masks.ptr, N, hipMemcpyDeviceToHost, p.stream) != hipSuccess)
            return AORESP_EDEVICE;
        if (hipEventRecord(p.done_ev, p.stream) != hipSuccess) return AORESP_EDEVICE;
        return AORESP_OK;
    }

    // Retire a finished pipeline (mu held).
    void retire(Pipeline& p) {
        std::vector<aoresp_result> out(p.plan.nres);
        std::vector<int> valid;
        aoresp_status st = collect_plan(p.ws, p.plan, out.data(), valid);
        const uint8_t* hm = p.hmask.as<uint8_t>();
        for (size_t b = 0; b < p.reqs.size(); ++b) {
            auto& r = p.reqs[b];
            if (st != AORESP_OK) {
                complete(r, st);
                continue;
            }
            r->result = out[b];
            const int64_t o = p.plan.insts[b].off;
            r->mask.assign(hm + o, hm + o + r->n);
            aoresp_status rs = AORESP_OK;
            if (r->n < 2 || !valid[b]) {
                identity_result(&r->result, r->rp.G);
                std::fill(r->mask.begin(), r->mask.end(), 0);
                rs = AORESP_ENODATA;
            }
            complete(r, rs);
        }
        bytes_in_flight -= p.bytes;
        p.bytes = 0;
        p.reqs.clear();
        p.busy = false;
        cv_done.notify_all();
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        int next = 0;
        for (;;) {
            // admit and launch on every free pipeline
            bool launched = false;
            for (int k = 0; k < 2; ++k) {
                Pipeline& p = pipes[(next + k) % 2];
                if (!p.busy && !queue.empty()) {
                    if (launch(p, lk)) {
                        launched = true;
                        next = (next + k + 1) % 2;
                    }
                }
            }
            bool any_busy = pipes[0].busy || pipes[1].busy;
            if (!any_busy) {
                if (stopping && queue.empty()) break;
                if (!launched) cv_work.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
            // retire finished batches; poll so that arrivals keep being admitted
            bool retired = false;
            for (int k = 0; k < 2; ++k) {
                Pipeline& p = pipes[k];
                if (!p.busy) continue;
                hipError_t q = hipEventQuery(p.done_ev);
                if (q == hipSuccess) {
                    retire(p);
                    retired = true;
                } else if (q != hipErrorNotReady) {
                    (void)hipGetLastError();
                    for (auto& r : p.reqs) complete(r, AORESP_EDEVICE);
                    bytes_in_flight -= p.bytes;
                    p.reqs.clear();
                    p.busy = false;
                    cv_done.notify_all();
                    retired = true;
                }
            }
            if (!retired && !launched) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
};

extern "C" {

aoresp_status aoresp_server_create(const aoresp_server_cfg* cfg, aoresp_server** out) {
    if (!out) return AORESP_EINVAL;
    auto s = std::make_unique<aoresp_server>();
    if (cfg) s->cfg = *cfg;
    if (!s->cfg.hbm_budget_bytes) s->cfg.hbm_budget_bytes = (size_t)8 << 30;
    if (!s->cfg.max_slots) s->cfg.max_slots = 256;
    if (hipGetDevice(&s->device) != hipSuccess) return AORESP_EDEVICE;
    s->ctx = device_ctx();
    if (!s->ctx) return AORESP_EDEVICE;
    for (auto& p : s->pipes) {
        if (hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking) != hipSuccess) return AORESP_EDEVICE;
        if (hipEventCreateWithFlags(&p.done_ev, hipEventDisableTiming) != hipSuccess) return AORESP_EDEVICE;
    }
    aoresp_server* raw = s.release();
    raw->thr = std::thread([raw] { raw->loop(); });
    *out = raw;
    return AORESP_OK;
}

aoresp_status aoresp_submit(aoresp_server* s, const float* P, const float* Q, size_t n, const aoresp_params* prm,
                            uint64_t* req_id) {
    if (!s || !req_id || (n > 0 && (!P || !Q)) || n > (size_t)INT32_MAX) return AORESP_EINVAL;
    auto r = std::make_shared<Request>();
    aoresp_status st = resolve_params(prm, n, r->rp);
    if (st != AORESP_OK) return st;
    r->n = n;
    r->bytes = request_bytes(n, r->rp);
    if (r->bytes > s->cfg.hbm_budget_bytes) return AORESP_ENOMEM;
    if (n) {
        r->host = static_cast<float*>(s->pool.get(6 * n * sizeof(float), &r->host_cls));
        if (!r->host) return AORESP_ENOMEM;
        std::memcpy(r->host, P, 3 * n * sizeof(float));
        std::memcpy(r->host + 3 * n, Q, 3 * n * sizeof(float));
    }
    r->t_submit = Clock::now();
    if (s->cfg.timeout_us) {
        r->has_deadline = true;
        r->deadline = r->t_submit + std::chrono::microseconds(s->cfg.timeout_us);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            s->pool.put(r->host, r->host_cls);
            return AORESP_EINVAL;
        }
        r->id = s->next_id++;
        s->table[r->id] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *req_id = r->id;
    return AORESP_OK;
}

aoresp_status aoresp_poll(aoresp_server* s, uint64_t req_id, aoresp_result* out, uint8_t* mask, int64_t timeout_us) {
    if (!s) return AORESP_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->table.find(req_id);
    if (it == s->table.end()) return AORESP_EINVAL;
    std::shared_ptr<Request> r = it->second;
    if (!r->done) {
        if (timeout_us == 0) return AORESP_EBUSY;
        if (timeout_us < 0) {
            s->cv_done.wait(lk, [&] { return r->done; });
        } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; })) {
            return AORESP_EBUSY;
        }
    }
    if (r->status == AORESP_OK || r->status == AORESP_ENODATA) {
        if (out) *out = r->result;
        if (mask && !r->mask.empty()) std::memcpy(mask, r->mask.data(), r->mask.size());
        if (mask && r->mask.empty() && r->n) std::memset(mask, 0, r->n);
    }
    aoresp_status st = r->status;
    s->table.erase(it);
    return st;
}

aoresp_status aoresp_server_stats(aoresp_server* s, double* p50_us, double* p99_us, double* req_per_s,
                                  uint64_t* completed) {
    if (!s) return AORESP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
        if (v.empty()) return 0.0;
        size_t i = (size_t)std::min<double>((double)v.size() - 1, std::floor(q * (double)(v.size() - 1) + 0.5));
        return v[i];
    };
    if (p50_us) *p50_us = pct(0.50);
    if (p99_us) *p99_us = pct(0.99);
    if (req_per_s) {
        double secs = s->any ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
        *req_per_s = secs > 0 ? (double)s->completed / secs : 0.0;
    }
    if (completed) *completed = s->completed;
    return AORESP_OK;
}

void aoresp_server_destroy(aoresp_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable()) s->thr.join();
    for (auto& p : s->pipes) {
        release_workspace(p.ws);
        p.P.release();
        p.Q.release();
        p.masks.release();
        HostBuf* hb[] = {&p.hmask};
        for (HostBuf* b : hb) {
            if (b->ptr) (void)hipHostFree(b->ptr);
            b->ptr = nullptr;
        }
        if (p.done_ev) (void)hipEventDestroy(p.done_ev);
        if (p.stream) (void)hipStreamDestroy(p.stream);
    }
    delete s;
}

}  // extern "C"
