// Serving loop: continuous batching of arriving events under an HBM budget.
//
// Submissions are copied to host memory and queued.  A dispatcher inside
// each of max_inflight worker threads (each with its own HIP stream) takes
// whatever is queued, admits the longest prefix of the queue whose device
// bytes fit the budget, and runs it as one batch through the batched
// pipeline.  Because several workers run at once, a new batch is binned and
// counted on one stream while earlier batches are still being filled on
// others.  After the count pass the batch's exact output size is known; it
// is reserved against the budget (waiting for releases if needed) before the
// fill.  Output bytes stay charged until the client releases the result.
// The ledger's rules (frnn_sched.h) keep this free of deadlock.
//
// What is charged is what the pool hands out, in its size classes: each
// event's input copy (from admission to the end of its batch), each
// worker's batch context (its binning and work buffers, kept and reused
// while the next batch fits it, charged for as long as the worker holds it)
// and each output (from the count pass until the client releases it).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "frnn_batch.h"
#include "frnn_runtime.h"
#include "frnn_sched.h"

using namespace frnn;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int64_t N = 0;
    std::vector<float> host;   // submitted points
    int64_t precount = 0;      // bytes reserved at admission
    frnn_timing tm{};
    frnn_csr out{};
    frnn_status st = FRNN_OK;
    std::string err;
    bool done = false;
};

}  // namespace

struct frnn_server_s {
    frnn_server_opts o{};
    Opts opts;
    std::shared_ptr<BudgetLedger> budget;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> live;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
    int next_batch = 0;

    // device bytes of an event's input copy
    int64_t input_bytes(int64_t N) const {
        return Pool::class_bytes(sizeof(float) * (size_t)std::max<int64_t>(1, N) * o.D);
    }
    // the context shape of a batch of events of these sizes
    BatchContext::Shape shape_of(const int64_t *n, int k) const {
        std::vector<frnn_event> ev(k);
        for (int i = 0; i < k; ++i) ev[i] = frnn_event{nullptr, n[i], nullptr, 0};
        return BatchContext::shape_for(ev.data(), k, o.D, o.r, o.K, o.flags, opts);
    }
    void worker(int id);
};

void frnn_server_s::worker(int id) {
    (void)id;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    const bool want_d2 = o.flags & FRNN_WANT_DIST2;
    std::unique_ptr<BatchContext> ctx;  // this worker's context
    int64_t ctx_charge = 0;             // its bytes, charged while it is held
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        int bid = 0;
        int64_t in_charge = 0;  // this batch's input copies
        BatchContext::Shape need{};
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop && queue.empty()) break;
            // admit in arrival order the longest prefix whose inputs, and the
            // growth of this worker's context if it must grow, fit
            const int n = (int)std::min<size_t>(queue.size(), (size_t)o.max_batch_events);
            std::vector<int64_t> sizes(n), inb(n + 1, 0);
            for (int i = 0; i < n; ++i) {
                sizes[i] = queue[i]->N;
                inb[i + 1] = inb[i] + input_bytes(sizes[i]);
            }
            auto charge = [&](int k) {
                const BatchContext::Shape sh = shape_of(sizes.data(), k);
                const int64_t grow =
                    ctx && ctx->fits(sh) ? 0 : std::max<int64_t>(0, BatchContext::bytes_for(sh) - ctx_charge);
                return inb[k] + grow;
            };
            int64_t charged = 0;
            const int k = budget->admit_prefix(charge, n, &charged);
            if (k == 0) {
                lk.unlock();
                if (ctx) {
                    // this idle worker's context may be what blocks the
                    // budget: give its bytes back and try again
                    (void)hipStreamSynchronize(s);
                    ctx->retire();
                    ctx.reset();
                    budget->release(ctx_charge);
                    ctx_charge = 0;
                    continue;
                }
                // over budget: wait for a release, then try again
                budget->wait_release(0.002);
                continue;
            }
            const double ta = now_s();
            for (int i = 0; i < k; ++i) {
                queue.front()->tm.admit_s = ta;
                batch.push_back(queue.front());
                queue.pop_front();
            }
            in_charge = inb[k];
            need = shape_of(sizes.data(), k);
            // the reserved growth now belongs to the context
            ctx_charge += charged - in_charge;
            bid = next_batch++;
            budget->begin(bid);
            if (!queue.empty()) cv_work.notify_one();
        }
        const int E = (int)batch.size();
        const double t0 = now_s();
        for (auto &r : batch) {
            r->tm.start_s = t0;
            r->tm.batch_id = bid;
            r->tm.batch_events = E;
        }
        frnn_status st = FRNN_OK;
        std::string err;
        std::vector<frnn_csr> outs(E);
        try {
            std::vector<DevBuf> inputs(E);
            std::vector<frnn_event> ev(E);
            for (int e = 0; e < E; ++e) {
                const size_t bytes = sizeof(float) * std::max<int64_t>(1, batch[e]->N) * o.D;
                inputs[e].reset(bytes, s);
                if (batch[e]->N)
                    FRNN_HIP(hipMemcpyAsync(inputs[e].get(), batch[e]->host.data(),
                                            sizeof(float) * batch[e]->N * o.D, hipMemcpyHostToDevice, s));
                ev[e] = frnn_event{inputs[e].as<float>(), batch[e]->N, nullptr, 0};
            }
            if (!ctx || !ctx->fits(need)) {
                // the old context's buffers go back to the pool first, then
                // the new one takes its charge (the growth reserved above;
                // a smaller replacement returns the difference)
                ctx.reset();
                try {
                    ctx.reset(new BatchContext(need, s));
                } catch (...) {
                    budget->release(ctx_charge);
                    ctx_charge = 0;
                    throw;
                }
                const int64_t now = ctx->device_bytes();
                if (now < ctx_charge) budget->release(ctx_charge - now);
                else budget->take(now - ctx_charge);
                ctx_charge = now;
            }
            {
                ctx->set_inputs(ev.data(), E, s);
                ctx->phase_a(s);
                BatchCounts c = ctx->read_counts(s);
                if (c.build_status & kStatusNonfinitePts)
                    throw Fail{FRNN_ERR_NONFINITE, "non-finite coordinate in the points"};
                // post-count reservation of the exact output
                const int64_t outb = output_bytes(*ctx, (int64_t)c.ctr.nnz, (int64_t)c.ctr.long_total, want_d2);
                if (outb > budget->limit()) throw Fail{FRNN_ERR_BUDGET, "batch output exceeds the budget"};
                if (!budget->reserve_output(bid, outb, 30.0))
                    throw Fail{FRNN_ERR_BUDGET, "timed out waiting for budget"};
                BatchOutput bo;
                try {
                    bo = alloc_output(*ctx, c, want_d2, s);
                } catch (...) {
                    budget->release(outb);
                    throw;
                }
                std::shared_ptr<BudgetLedger> bud = budget;
                bo.own->on_release = [bud, outb]() { bud->release(outb); };
                try {
                    ctx->phase_b(bo.od, c.ctr.long_total > 0, s);
                    bo.own->long_ran = c.ctr.long_total > 0;
                } catch (...) {
                    delete bo.own;  // returns the reservation
                    throw;
                }
                hand_out(*ctx, c, bo, outs.data());
            }
            FRNN_HIP(hipStreamSynchronize(s));  // results complete on the device
            // the client may release the results after this stream is gone
            if (E > 0 && outs[0].owner_) static_cast<OutputOwner *>(outs[0].owner_)->buf.mark_complete();
            for (auto &in : inputs) in.mark_complete();
        } catch (const Fail &f) {
            st = f.st;
            err = f.msg;
        } catch (const std::exception &x) {
            st = FRNN_ERR_INTERNAL;
            err = x.what();
        }
        const double t1 = now_s();
        budget->end(bid, in_charge);
        {
            std::lock_guard<std::mutex> g(mu);
            for (int e = 0; e < E; ++e) {
                auto &r = batch[e];
                r->tm.done_s = t1;
                r->st = st;
                r->err = err;
                if (st == FRNN_OK) r->out = outs[e];
                r->host.clear();
                r->host.shrink_to_fit();
                r->done = true;
            }
        }
        if (st != FRNN_OK)
            for (auto &oc : outs) frnn_csr_release(&oc);
        cv_done.notify_all();
    }
    if (ctx) {
        (void)hipStreamSynchronize(s);
        ctx->retire();
        ctx.reset();
        budget->release(ctx_charge);
    }
    (void)hipStreamDestroy(s);
}

extern "C" {

void frnn_server_opts_default(frnn_server_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->D = 8;
    o->r = 0.1f;
    o->K = 0;
    o->flags = FRNN_WANT_DIST2 | FRNN_SELF_QUERY;
    o->hbm_budget_bytes = (int64_t)64 << 30;
    o->max_batch_events = 64;
    o->max_inflight = 2;
    frnn_opts_default(&o->opts);
}

frnn_status frnn_server_create(const frnn_server_opts *o, frnn_server *out) {
    if (out) *out = nullptr;
    try {
        if (!o || !out) return fail(FRNN_ERR_INVALID_ARG, "null argument");
        if (o->D < 1 || o->D > kDMax) return fail(FRNN_ERR_INVALID_ARG, "D must be in 1..32");
        if (!(o->r >= 0.f) || !std::isfinite(o->r)) return fail(FRNN_ERR_INVALID_ARG, "bad radius");
        if (o->hbm_budget_bytes <= 0) return fail(FRNN_ERR_INVALID_ARG, "budget must be positive");
        if (o->max_batch_events < 1 || o->max_batch_events > 1024)
            return fail(FRNN_ERR_INVALID_ARG, "max_batch_events out of 1..1024");
        if (o->max_inflight < 1 || o->max_inflight > 8) return fail(FRNN_ERR_INVALID_ARG, "max_inflight out of 1..8");
        if (o->flags & ~(uint32_t)(FRNN_WANT_DIST2 | FRNN_SELF_QUERY | FRNN_EXCLUDE_SELF))
            return fail(FRNN_ERR_INVALID_ARG, "unknown flag");
        auto *s = new frnn_server_s();
        s->o = *o;
        s->o.flags |= FRNN_SELF_QUERY;
        s->opts = Opts::from(&o->opts);
        std::string why;
        frnn_status st = s->opts.validate(&why);
        if (st) {
            delete s;
            return fail(st, why);
        }
        s->budget = std::make_shared<BudgetLedger>(o->hbm_budget_bytes);
        for (int i = 0; i < o->max_inflight; ++i) s->workers.emplace_back([s, i] { s->worker(i); });
        *out = s;
        return FRNN_OK;
    } catch (const std::exception &x) {
        return fail(FRNN_ERR_INTERNAL, x.what());
    }
}

frnn_status frnn_server_submit(frnn_server s, const float *points, int64_t N, uint64_t *ticket) {
    if (ticket) *ticket = 0;
    try {
        if (!s || !ticket || N < 0 || N >= ((int64_t)1 << 31) || (N > 0 && !points))
            return fail(FRNN_ERR_INVALID_ARG, "bad submission");
        auto r = std::make_shared<Request>();
        r->N = N;
        r->precount = s->input_bytes(N) + BatchContext::bytes_for(s->shape_of(&N, 1));
        if (r->precount > s->budget->limit()) return fail(FRNN_ERR_BUDGET, "event larger than the whole budget");
        r->host.assign(points, points + N * (int64_t)s->o.D);
        r->tm.submit_s = now_s();
        {
            std::lock_guard<std::mutex> g(s->mu);
            if (s->stop) return fail(FRNN_ERR_INVALID_ARG, "server is stopping");
            r->ticket = s->next_ticket++;
            s->live[r->ticket] = r;
            s->queue.push_back(r);
        }
        s->cv_work.notify_one();
        *ticket = r->ticket;
        return FRNN_OK;
    } catch (const std::bad_alloc &) {
        return fail(FRNN_ERR_OOM, "host allocation failed");
    } catch (const std::exception &x) {
        return fail(FRNN_ERR_INTERNAL, x.what());
    }
}

frnn_status frnn_server_wait(frnn_server s, uint64_t ticket, double timeout_s, frnn_csr *out,
                             frnn_timing *timing) {
    if (out) std::memset(out, 0, sizeof(*out));
    try {
        if (!s || !out) return fail(FRNN_ERR_INVALID_ARG, "null argument");
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end()) return fail(FRNN_ERR_INVALID_ARG, "unknown ticket");
        std::shared_ptr<Request> r = it->second;
        auto ready = [&] { return r->done; };
        if (timeout_s < 0) {
            s->cv_done.wait(lk, ready);
        } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
            return fail(FRNN_ERR_NOT_READY, "ticket still in flight");
        }
        s->live.erase(ticket);
        if (timing) *timing = r->tm;
        if (r->st != FRNN_OK) return fail(r->st, r->err);
        *out = r->out;
        r->out = frnn_csr{};
        return FRNN_OK;
    } catch (const std::exception &x) {
        return fail(FRNN_ERR_INTERNAL, x.what());
    }
}

frnn_status frnn_server_memory(frnn_server s, int64_t *held_bytes, int64_t *peak_bytes) {
    if (!s) return fail(FRNN_ERR_INVALID_ARG, "null server");
    if (held_bytes) *held_bytes = s->budget->used();
    if (peak_bytes) *peak_bytes = s->budget->peak();
    return FRNN_OK;
}

void frnn_server_destroy(frnn_server s) {
    if (!s) return;
    try {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        for (auto &kv : s->live) frnn_csr_release(&kv.second->out);
        delete s;
    } catch (...) {
    }
}

}  // extern "C"
