// CPU harness of the request loop's scheduler (paper_2502_06337_amd/csrc/
// scheduler.h) with a fake executor: a manual clock, a device-memory model
// with the same growth rule as the library's buffers (a need beyond the
// current size grows it to need + need/4 + 256), batches that finish a fixed
// time after launch, and injected failures (allocation, launch, device).
// Built with g++ by tests/test_sched.py; no GPU is involved.
#include <cstdint>
#include <cstring>
#include <vector>

#include "../paper_2502_06337_amd/csrc/scheduler.h"

using namespace aoresp;

namespace {

struct FakeExec final : Executor {
    int64_t clock = 0;
    size_t cap[Scheduler::kPipes] = {0, 0};
    int64_t done_at[Scheduler::kPipes] = {0, 0};
    int64_t step_us = 1000;          // batch duration
    size_t bytes_per_corr = 100;
    int fail_alloc = 0;              // next `fail_alloc` allocations that grow a buffer fail
    int fail_alloc_always = 0;       // every allocation fails
    int fail_device_next = 0;        // the next launched batch reports a device error
    bool device_fail[Scheduler::kPipes] = {false, false};
    size_t max_total = 0;            // largest cap[0] + cap[1] seen
    int launches = 0, releases = 0;
    std::vector<uint64_t> order;     // request ids in launch order

    size_t need_of(const std::vector<ReqPtr>& b) const {
        size_t s = 0;
        for (auto& r : b) s += r->n * bytes_per_corr + 64;
        return s;
    }
    int64_t now_us() override { return clock; }
    size_t held(int p) override { return cap[p]; }
    size_t held_after(int p, const std::vector<ReqPtr>& b, bool exact) override {
        const size_t need = need_of(b);
        if (exact) return (need + 255) / 256 * 256;
        return need <= cap[p] ? cap[p] : need + need / 4 + 256;
    }
    void release(int p) override {
        if (cap[p]) ++releases;
        cap[p] = 0;
    }
    aoresp_status launch(int p, const std::vector<ReqPtr>& b, bool exact) override {
        const size_t need = need_of(b);
        if (need > cap[p] || exact) {
            if (fail_alloc_always || fail_alloc > 0) {
                if (fail_alloc > 0) --fail_alloc;
                return AORESP_ENOMEM;
            }
            cap[p] = exact ? (need + 255) / 256 * 256 : need + need / 4 + 256;
        }
        if (cap[0] + cap[1] > max_total) max_total = cap[0] + cap[1];
        ++launches;
        for (auto& r : b) order.push_back(r->id);
        done_at[p] = clock + step_us;
        device_fail[p] = fail_device_next > 0;
        if (fail_device_next > 0) --fail_device_next;
        return AORESP_OK;
    }
    int query(int p) override {
        if (clock < done_at[p]) return 0;
        return device_fail[p] ? -1 : 1;
    }
    aoresp_status collect(int p, const std::vector<ReqPtr>& b) override {
        (void)p;
        for (auto& r : b) {
            std::memset(&r->result, 0, sizeof(r->result));
            r->result.n_inliers = (uint32_t)r->n;   // a recognisable result
            r->mask.assign(r->n, 1);
            r->status = r->n < 2 ? AORESP_ENODATA : AORESP_OK;
        }
        return AORESP_OK;
    }
    void drop(SchedRequest& r) override { r.payload = nullptr; }
};

struct Harness {
    FakeExec ex;
    Scheduler sched;
    size_t budget;
    Harness(size_t b, uint32_t slots, uint32_t timeout) : sched(&ex, b, slots, timeout), budget(b) {}
};

}  // namespace

extern "C" {

void* fs_create(uint64_t budget, uint32_t max_slots, uint32_t timeout_us) {
    return new Harness((size_t)budget, max_slots, timeout_us);
}
void fs_destroy(void* h) { delete static_cast<Harness*>(h); }

// Queue a request of n correspondences; 0 if it alone exceeds the budget
// (what aoresp_submit answers with ENOMEM).
uint64_t fs_submit(void* hv, uint64_t n) {
    Harness* h = static_cast<Harness*>(hv);
    auto r = std::make_shared<SchedRequest>();
    r->n = (size_t)n;
    std::vector<ReqPtr> one{r};
    if (h->ex.held_after(0, one, true) > h->budget) return 0;
    return h->sched.submit(r);
}
int fs_step(void* h) { return static_cast<Harness*>(h)->sched.step() ? 1 : 0; }
void fs_advance(void* h, int64_t us) { static_cast<Harness*>(h)->ex.clock += us; }
// Status of a request (EBUSY while pending); n_inliers of its result.
int fs_poll(void* h, uint64_t id, uint32_t* n_inliers) {
    aoresp_result r{};
    const aoresp_status st = static_cast<Harness*>(h)->sched.poll(id, &r, nullptr, 0);
    if (n_inliers) *n_inliers = r.n_inliers;
    return (int)st;
}
uint64_t fs_max_total(void* h) { return static_cast<Harness*>(h)->ex.max_total; }
uint64_t fs_held(void* h, int p) { return static_cast<Harness*>(h)->ex.cap[p]; }
uint64_t fs_peak_held(void* h) { return static_cast<Harness*>(h)->sched.peak_held(); }
int fs_launches(void* h) { return static_cast<Harness*>(h)->ex.launches; }
int fs_releases(void* h) { return static_cast<Harness*>(h)->ex.releases; }
int fs_order(void* h, uint64_t* out, int cap) {
    auto& o = static_cast<Harness*>(h)->ex.order;
    int k = 0;
    for (; k < (int)o.size() && k < cap; ++k) out[k] = o[k];
    return (int)o.size();
}
void fs_set(void* hv, int fail_alloc, int fail_alloc_always, int fail_device_next, int64_t step_us) {
    FakeExec& e = static_cast<Harness*>(hv)->ex;
    e.fail_alloc = fail_alloc;
    e.fail_alloc_always = fail_alloc_always;
    e.fail_device_next = fail_device_next;
    if (step_us > 0) e.step_us = step_us;
}
void fs_stats(void* h, double* p50, double* p99, uint64_t* completed) {
    static_cast<Harness*>(h)->sched.stats(p50, p99, nullptr, completed);
}

}  // extern "C"
