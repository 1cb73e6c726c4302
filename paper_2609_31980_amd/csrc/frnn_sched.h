// Device-memory budget ledger of the serving loop (host logic only, no HIP).
//
// Two kinds of reservation share one limit:
//   * pre-count: taken when events are admitted into a batch (their input,
//     index and per-query work), returned when the batch completes;
//   * output: taken after the batch's count pass, when its exact output
//     size is known, and returned when the client releases the result.
// A batch waiting for its output reservation holds its pre-count one, so
// two batches could wait on each other forever.  The rule that prevents
// it: the oldest running batch may always take its output reservation.
// Nothing new is admitted while the ledger is over the limit, so the excess
// is at most one output per batch that was running when the limit was
// first exceeded (at most max_inflight outputs).
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <set>

namespace frnn {

class BudgetLedger {
public:
    explicit BudgetLedger(int64_t limit) : limit_(limit) {}

    // Admit the longest prefix of `pre` (pre-count bytes per queued event,
    // in arrival order) that fits, at most max_n; reserves it and returns
    // its length.  Nothing is admitted when the first event does not fit.
    int admit(const int64_t *pre, int n, int max_n) {
        std::lock_guard<std::mutex> g(mu_);
        int k = 0;
        while (k < n && k < max_n && used_ + pre[k] <= limit_) {
            used_ += pre[k];
            ++k;
        }
        peak_ = std::max(peak_, used_);
        return k;
    }

    // Admit the longest prefix k (1..n) of the queue whose charge(k) fits,
    // reserving charge(k); charge must not decrease with k.  0 when even
    // charge(1) does not fit.
    template <class F>
    int admit_prefix(F &&charge, int n, int64_t *charged) {
        std::lock_guard<std::mutex> g(mu_);
        int k = 0;
        int64_t c = 0;
        for (int i = 1; i <= n; ++i) {
            const int64_t ci = charge(i);
            if (used_ + ci > limit_) break;
            k = i;
            c = ci;
        }
        used_ += c;
        peak_ = std::max(peak_, used_);
        *charged = c;
        return k;
    }

    // Take bytes without a wait or a check (a held context growing: the
    // caller's admission already reserved the difference).
    void take(int64_t bytes) {
        std::lock_guard<std::mutex> g(mu_);
        used_ += bytes;
        peak_ = std::max(peak_, used_);
    }

    // Wait (up to timeout_s) until anything is returned.
    void wait_release(double timeout_s) {
        std::unique_lock<std::mutex> l(mu_);
        cv_.wait_until(l, deadline(timeout_s));
    }

    void begin(int batch) {
        std::lock_guard<std::mutex> g(mu_);
        running_.insert(batch);
    }

    // Output reservation after the count pass: waits until it fits or the
    // batch is the oldest running one.  False on timeout.
    bool reserve_output(int batch, int64_t bytes, double timeout_s) {
        std::unique_lock<std::mutex> l(mu_);
        const bool ok = cv_.wait_until(l, deadline(timeout_s), [&] {
            return used_ + bytes <= limit_ || (!running_.empty() && *running_.begin() == batch);
        });
        if (!ok) return false;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
    }

    void release(int64_t bytes) {
        {
            std::lock_guard<std::mutex> g(mu_);
            used_ -= bytes;
        }
        cv_.notify_all();
    }

    // Batch done: its pre-count reservation is returned.
    void end(int batch, int64_t precount_total) {
        {
            std::lock_guard<std::mutex> g(mu_);
            running_.erase(batch);
            used_ -= precount_total;
        }
        cv_.notify_all();
    }

    int64_t limit() const { return limit_; }
    int64_t used() {
        std::lock_guard<std::mutex> g(mu_);
        return used_;
    }
    int64_t peak() {
        std::lock_guard<std::mutex> g(mu_);
        return peak_;
    }

private:
    // system_clock deadlines: waits then use pthread_cond_timedwait
    static std::chrono::system_clock::time_point deadline(double s) {
        return std::chrono::system_clock::now() +
               std::chrono::duration_cast<std::chrono::system_clock::duration>(std::chrono::duration<double>(s));
    }
    std::mutex mu_;
    std::condition_variable cv_;
    const int64_t limit_;
    int64_t used_ = 0, peak_ = 0;
    std::set<int> running_;
};

}  // namespace frnn
