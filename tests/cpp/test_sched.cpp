// Simulation of the serving loop's budget rule with a fake executor: several
// workers admit events from a shared queue, "count" them (a random delay),
// reserve a random output size, and hand the output to a client thread that
// releases it later.  Checks: every event is served exactly once, no output
// reservation times out (no deadlock), and the limit is never exceeded by
// more than one output per worker (batches in flight).
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "frnn_sched.h"

int main(int argc, char **argv) {
    const int n_events = argc > 1 ? std::atoi(argv[1]) : 3000;
    const int workers = 4;
    const int64_t limit = 1000, max_out = 300, max_pre = 400;
    frnn::BudgetLedger L(limit);
    std::mutex qmu;
    std::deque<std::pair<int, int64_t>> queue;
    std::mt19937 rng(7);
    for (int i = 0; i < n_events; ++i) queue.push_back({i, 1 + (int64_t)(rng() % max_pre)});
    std::vector<std::atomic<int>> served(n_events);
    for (auto &s : served) s = 0;
    std::mutex rmu;
    std::deque<int64_t> pending;  // outputs the client still holds
    std::atomic<bool> done{false}, bad{false};
    std::atomic<int> next_batch{0};

    std::thread client([&] {
        std::mt19937 r(11);
        while (!done || true) {
            int64_t b = -1;
            {
                std::lock_guard<std::mutex> g(rmu);
                if (!pending.empty()) {
                    b = pending.front();
                    pending.pop_front();
                } else if (done) {
                    break;
                }
            }
            if (b >= 0) {
                std::this_thread::sleep_for(std::chrono::microseconds(r() % 50));
                L.release(b);
            } else {
                std::this_thread::yield();
            }
        }
    });
    std::vector<std::thread> ws;
    for (int w = 0; w < workers; ++w) {
        ws.emplace_back([&, w] {
            std::mt19937 r(100 + w);
            for (;;) {
                std::vector<std::pair<int, int64_t>> batch;
                int bid;
                {
                    std::unique_lock<std::mutex> lk(qmu);
                    if (queue.empty()) return;
                    std::vector<int64_t> pre;
                    for (size_t i = 0; i < queue.size() && i < 8; ++i) pre.push_back(queue[i].second);
                    const int k = L.admit(pre.data(), (int)pre.size(), 8);
                    if (k == 0) {
                        lk.unlock();
                        L.wait_release(0.001);
                        continue;
                    }
                    for (int i = 0; i < k; ++i) {
                        batch.push_back(queue.front());
                        queue.pop_front();
                    }
                    bid = next_batch++;
                    L.begin(bid);
                }
                std::this_thread::sleep_for(std::chrono::microseconds(r() % 100));  // count pass
                const int64_t out = 1 + (int64_t)(r() % max_out);
                if (!L.reserve_output(bid, out, 10.0)) {
                    std::fprintf(stderr, "output reservation timed out (deadlock)\n");
                    bad = true;
                    L.end(bid, 0);
                    return;
                }
                if (L.used() > limit + workers * max_out) {
                    std::fprintf(stderr, "limit exceeded by more than one output per worker: %lld\n",
                                 (long long)L.used());
                    bad = true;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(r() % 50));  // fill pass
                int64_t pre_total = 0;
                for (auto &e : batch) {
                    served[e.first]++;
                    pre_total += e.second;
                }
                {
                    std::lock_guard<std::mutex> g(rmu);
                    pending.push_back(out);
                }
                L.end(bid, pre_total);
            }
        });
    }
    for (auto &t : ws) t.join();
    done = true;
    client.join();
    for (int i = 0; i < n_events; ++i)
        if (served[i] != 1) {
            std::fprintf(stderr, "event %d served %d times\n", i, (int)served[i]);
            bad = true;
        }
    if (L.used() != 0) {
        std::fprintf(stderr, "ledger not balanced: %lld\n", (long long)L.used());
        bad = true;
    }
    std::printf("batches %d peak %lld limit %lld\n", (int)next_batch, (long long)L.peak(), (long long)limit);
    return bad ? 1 : 0;
}
