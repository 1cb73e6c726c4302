// Simulation of the serving loop's budget rule with a fake executor: several
// workers admit events from a shared queue, "count" them (a random delay),
// reserve a random output size, and hand the output to a client thread that
// releases it later.  As in the server, each worker keeps a context whose
// charge grows with the batches it has run (a held context that fits costs
// nothing more; one that must grow reserves the growth at admission) and
// gives it back when nothing can be admitted.  Checks: every event is served
// exactly once, no output reservation times out (no deadlock), the limit is
// never exceeded by more than one output per worker (batches in flight), and
// the ledger balances at the end.
#include <algorithm>
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
            int64_t held = 0;  // this worker's context charge
            // context bytes for a batch of k events (grows in classes)
            auto ctx_of = [](int k) {
                int c = 1;
                while (c < k) c *= 2;
                return (int64_t)40 * c;
            };
            for (;;) {
                std::vector<std::pair<int, int64_t>> batch;
                int bid;
                int64_t in_charge = 0;
                {
                    std::unique_lock<std::mutex> lk(qmu);
                    if (queue.empty()) {
                        lk.unlock();
                        L.release(held);
                        return;
                    }
                    const int n = (int)std::min<size_t>(queue.size(), 8);
                    std::vector<int64_t> inb(n + 1, 0);
                    for (int i = 0; i < n; ++i) inb[i + 1] = inb[i] + queue[i].second;
                    auto charge = [&](int k) { return inb[k] + std::max<int64_t>(0, ctx_of(k) - held); };
                    int64_t charged = 0;
                    const int k = L.admit_prefix(charge, n, &charged);
                    if (k == 0) {
                        lk.unlock();
                        if (held) {
                            L.release(held);
                            held = 0;
                            continue;
                        }
                        L.wait_release(0.001);
                        continue;
                    }
                    for (int i = 0; i < k; ++i) {
                        batch.push_back(queue.front());
                        queue.pop_front();
                    }
                    in_charge = inb[k];
                    held += charged - in_charge;
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
                for (auto &e : batch) served[e.first]++;
                {
                    std::lock_guard<std::mutex> g(rmu);
                    pending.push_back(out);
                }
                L.end(bid, in_charge);
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
