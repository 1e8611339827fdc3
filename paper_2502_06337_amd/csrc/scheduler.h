// Continuous-batching scheduler of the request loop, independent of the
// device.  It owns the queue, the two pipelines' states, admission under a
// byte budget, deadlines, retirement and failure handling; an Executor does
// the device work (sizing, allocation, upload, launch, completion query,
// results) and supplies the clock.  The server drives it with a HIP executor;
// the CPU tests drive it with a fake executor and a fake clock.
//
// Budget rule: what both pipelines hold on the device (their cached buffers,
// which outlive a batch) plus what the next batch needs beyond its pipeline's
// cache stays within the budget at every launch.  A batch is taken from the
// head of the queue in arrival order while it fits; if not even the head
// request fits, idle caches are released (the pipeline then sizes its buffers
// exactly) before the request waits for the other pipeline to finish.
// Deadlines (from submit) apply while a request waits and when its batch
// retires: a result that arrives late is reported as ETIMEDOUT.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/aoresp.h"

namespace aoresp {

struct SchedRequest {
    uint64_t id = 0;
    size_t n = 0;
    int64_t t_submit_us = 0;
    int64_t deadline_us = -1;          // < 0: none
    bool done = false;
    aoresp_status status = AORESP_EBUSY;
    aoresp_result result{};
    std::vector<uint8_t> mask;         // n bytes once done (OK / ENODATA)
    double latency_us = 0.0;
    void* payload = nullptr;           // executor data (host copy of the inputs, parameters)
};
using ReqPtr = std::shared_ptr<SchedRequest>;

class Executor {
  public:
    virtual ~Executor() = default;
    virtual int64_t now_us() = 0;
    // Device bytes pipeline `pipe` holds now (its cached buffers).
    virtual size_t held(int pipe) = 0;
    // Device bytes it would hold after running `batch`: with exact = false
    // its buffers grow with headroom and are kept, with exact = true they are
    // reallocated to the batch's exact size.
    virtual size_t held_after(int pipe, const std::vector<ReqPtr>& batch, bool exact) = 0;
    // Free an idle pipeline's cached buffers.
    virtual void release(int pipe) = 0;
    // Size the buffers (as held_after with `exact`), upload and enqueue.
    virtual aoresp_status launch(int pipe, const std::vector<ReqPtr>& batch, bool exact) = 0;
    // 1: finished, 0: running, < 0: the device reported an error.
    virtual int query(int pipe) = 0;
    // Results and masks of a finished batch into the requests (status OK or
    // ENODATA per request), or a status for the whole batch.
    virtual aoresp_status collect(int pipe, const std::vector<ReqPtr>& batch) = 0;
    // The request's executor data is no longer needed.
    virtual void drop(SchedRequest& r) = 0;
};

class Scheduler {
  public:
    static constexpr int kPipes = 2;

    Scheduler(Executor* ex, size_t budget, uint32_t max_slots, uint32_t timeout_us)
        : ex_(ex), budget_(budget), max_slots_(max_slots ? max_slots : 1), timeout_us_(timeout_us) {}

    // Queue a request (its payload set by the caller); returns its id.
    uint64_t submit(const ReqPtr& r) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            r->id = next_id_++;
            r->t_submit_us = ex_->now_us();
            r->deadline_us = timeout_us_ ? r->t_submit_us + (int64_t)timeout_us_ : -1;
            table_[r->id] = r;
            queue_.push_back(r);
        }
        cv_work_.notify_one();
        return r->id;
    }

    bool stopping() {
        std::lock_guard<std::mutex> lk(mu_);
        return stopping_;
    }
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
        }
        cv_work_.notify_all();
    }
    // True once stop() was called and nothing is queued or running.
    bool drained() {
        std::lock_guard<std::mutex> lk(mu_);
        return stopping_ && queue_.empty() && !busy_[0] && !busy_[1];
    }

    // One scheduling pass: retire finished batches, expire waiting requests,
    // admit and launch on free pipelines.  Returns true if anything changed.
    bool step() {
        std::unique_lock<std::mutex> lk(mu_);
        bool progress = false;
        for (int p = 0; p < kPipes; ++p) {
            if (!busy_[p]) continue;
            const int q = ex_->query(p);
            if (q == 0) continue;
            std::vector<ReqPtr> batch = std::move(batch_[p]);
            batch_[p].clear();
            aoresp_status st = q > 0 ? ex_->collect(p, batch) : AORESP_EDEVICE;
            busy_[p] = false;
            const int64_t now = ex_->now_us();
            for (auto& r : batch) {
                aoresp_status rs = st != AORESP_OK ? st : r->status;
                if (rs == AORESP_OK || rs == AORESP_ENODATA) {
                    if (r->deadline_us >= 0 && now > r->deadline_us) rs = AORESP_ETIMEDOUT;
                }
                complete(*r, rs, now);
            }
            progress = true;
        }
        const int64_t now = ex_->now_us();
        for (auto it = queue_.begin(); it != queue_.end();) {
            if ((*it)->deadline_us >= 0 && now > (*it)->deadline_us) {
                complete(**it, AORESP_ETIMEDOUT, now);
                it = queue_.erase(it);
                progress = true;
            } else {
                ++it;
            }
        }
        for (int k = 0; k < kPipes; ++k) {
            const int p = (next_ + k) % kPipes;
            if (busy_[p] || queue_.empty()) continue;
            if (admit_and_launch(p, lk)) {
                progress = true;
                next_ = (p + 1) % kPipes;
            }
        }
        if (progress) cv_done_.notify_all();
        return progress;
    }

    bool idle() {
        std::lock_guard<std::mutex> lk(mu_);
        return queue_.empty() && !busy_[0] && !busy_[1];
    }
    bool any_busy() {
        std::lock_guard<std::mutex> lk(mu_);
        return busy_[0] || busy_[1];
    }
    // Wait up to `us` for a submit or a stop (scheduler thread, nothing busy).
    void wait_work(int64_t us) {
        std::unique_lock<std::mutex> lk(mu_);
        if (!queue_.empty() || stopping_) return;
        cv_work_.wait_for(lk, std::chrono::microseconds(us));
    }

    // aoresp_poll semantics.  wait_us: 0 = do not wait, < 0 = until done.
    aoresp_status poll(uint64_t id, aoresp_result* out, uint8_t* mask, int64_t wait_us) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = table_.find(id);
        if (it == table_.end()) return AORESP_EINVAL;
        ReqPtr r = it->second;
        if (!r->done) {
            if (wait_us == 0) return AORESP_EBUSY;
            if (wait_us < 0) {
                cv_done_.wait(lk, [&] { return r->done; });
            } else if (!cv_done_.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return r->done; })) {
                return AORESP_EBUSY;
            }
        }
        if (r->status == AORESP_OK || r->status == AORESP_ENODATA) {
            if (out) *out = r->result;
            if (mask && r->n) {
                if (r->mask.size() == r->n) std::memcpy(mask, r->mask.data(), r->n);
                else std::memset(mask, 0, r->n);
            }
        }
        const aoresp_status st = r->status;
        table_.erase(it);
        return st;
    }

    void stats(double* p50, double* p99, double* rate, uint64_t* completed) {
        std::lock_guard<std::mutex> lk(mu_);
        std::vector<double> v = lat_us_;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            if (v.empty()) return 0.0;
            size_t i = (size_t)std::min<double>((double)v.size() - 1, std::floor(q * (double)(v.size() - 1) + 0.5));
            return v[i];
        };
        if (p50) *p50 = pct(0.50);
        if (p99) *p99 = pct(0.99);
        if (rate) {
            const double secs = completed_ ? (double)(t_last_ - t_first_) * 1e-6 : 0.0;
            *rate = secs > 0 ? (double)completed_ / secs : 0.0;
        }
        if (completed) *completed = completed_;
    }

    // Largest device bytes held by both pipelines together at a launch.
    size_t peak_held() {
        std::lock_guard<std::mutex> lk(mu_);
        return peak_held_;
    }

  private:
    void complete(SchedRequest& r, aoresp_status st, int64_t now) {
        r.status = st;
        r.done = true;
        if (st != AORESP_OK && st != AORESP_ENODATA) r.mask.clear();
        r.latency_us = (double)(now - r.t_submit_us);
        lat_us_.push_back(r.latency_us);
        if (!completed_ || r.t_submit_us < t_first_) t_first_ = r.t_submit_us;
        t_last_ = std::max(t_last_, now);
        ++completed_;
        ex_->drop(r);
    }

    // Batch for pipeline p from the head of the queue (mu_ held); launches it
    // with mu_ released.  Returns true if a batch was launched or failed.
    bool admit_and_launch(int p, std::unique_lock<std::mutex>& lk) {
        const int o = (p + 1) % kPipes;
        for (int attempt = 0; attempt < 3; ++attempt) {
            const bool exact = attempt > 0;
            if (exact) {
                // make room: drop this pipeline's cache, then the other's if idle
                ex_->release(p);
                if (attempt == 2) {
                    if (busy_[o]) return false;
                    ex_->release(o);
                }
            }
            std::vector<ReqPtr> batch;
            size_t after = 0;
            for (auto it = queue_.begin(); it != queue_.end() && batch.size() < max_slots_; ++it) {
                batch.push_back(*it);
                const size_t need = ex_->held_after(p, batch, exact);
                if (ex_->held(o) + need > budget_) {
                    batch.pop_back();
                    break;
                }
                after = need;
            }
            if (batch.empty()) continue;
            queue_.erase(queue_.begin(), queue_.begin() + (std::ptrdiff_t)batch.size());
            busy_[p] = true;
            peak_held_ = std::max(peak_held_, ex_->held(o) + after);
            lk.unlock();
            aoresp_status st = ex_->launch(p, batch, exact);
            if (st == AORESP_ENOMEM && !exact) {
                // allocation failed with headroom: once more at the exact size
                ex_->release(p);
                st = ex_->launch(p, batch, true);
            }
            lk.lock();
            if (st != AORESP_OK) {
                busy_[p] = false;
                const int64_t now = ex_->now_us();
                for (auto& r : batch) complete(*r, st, now);
                return true;
            }
            batch_[p] = std::move(batch);
            return true;
        }
        return false;
    }

    Executor* ex_;
    size_t budget_;
    uint32_t max_slots_;
    uint32_t timeout_us_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<ReqPtr> queue_;
    std::unordered_map<uint64_t, ReqPtr> table_;
    uint64_t next_id_ = 1;
    bool stopping_ = false;
    bool busy_[kPipes] = {false, false};
    std::vector<ReqPtr> batch_[kPipes];
    int next_ = 0;
    std::vector<double> lat_us_;
    uint64_t completed_ = 0;
    int64_t t_first_ = 0, t_last_ = 0;
    size_t peak_held_ = 0;
};

}  // namespace aoresp
