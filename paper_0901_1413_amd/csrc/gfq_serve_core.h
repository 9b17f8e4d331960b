// gfq_serve_core.h -- the product server's worker, with the device behind an executor.
//
// Plain C++ with no HIP calls, so that the library (gfq_server.cpp, with the HIP executor)
// and host-only checks (a fake executor, built with thread and address sanitizers) run the
// same code.  The worker owns an arrival-ordered queue and a budgeted arena (gfq_sched.h):
// while a slot is free it admits a batch (arrival order, request and tile limits, arena
// room), hands it to the executor and polls the slots in flight; completed batches release
// their arena ranges and queue one completion per request.  A slot whose batch has not
// completed within the watchdog time is abandoned: its requests complete with
// GFQ_EHIP, its arena ranges are never reused (the device may still write them), the slot
// is retired and the server is marked failed (later submissions return GFQ_EHIP).
//
// Executor interface (E):
//   int  slots() const;                              slots, fixed for the executor's life
//   int  launch(int slot, const Batch &b);           0, or a status that fails the batch
//   int  poll(int slot);                             0 done, 1 pending, < 0 failed (status)
//   void drain(int slot);                            wait for the slot's device work
//   void retire(int slot);                           the watchdog gave up on the slot: never
//                                                    wait for it or free its buffers
// Request type (R): the fields arrival (us), bytes (arena), items (tiles), tag.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "gfq_sched.h"

namespace gfq {

// Status values shared with the C ABI (gfq.h).
constexpr int kServeOk = 0;
constexpr int kServeNoMem = -7;
constexpr int kServeHip = -8;

struct ServeCompletion {
    uint64_t tag;
    int status;
    int batch_size;
    double arrival_us, launch_us, done_us;
};

struct ServeLimits {
    int max_batch = 256;
    size_t max_items = 65536;
    double watchdog_us = 0;        // 0: no watchdog
};

template <class R, class E>
class ServeCore {
  public:
    typedef std::vector<std::pair<R, uintptr_t>> Batch;   // request, arena address

    ServeCore(E &exec, Arena &arena, ServeLimits lim)
        : exec_(exec), arena_(arena), lim_(lim), t0_(Clock::now()), slots_(exec.slots()) {}
    ~ServeCore() { stop(); }

    void start() { worker_ = std::thread([this] { run(); }); }
    // the same, with `init` run first on the worker thread (e.g. selecting its device)
    template <class F> void start_on(F init) {
        worker_ = std::thread([this, init] {
            init();
            run();
        });
    }

    // Stop admitting, wait for the batches in flight (retired slots excepted), join.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (worker_.joinable()) worker_.join();
    }

    double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0_).count(); }

    // Queue requests (already validated); false if the server has failed.
    bool submit(std::vector<R> &v) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (failed_) return false;
            for (R &r : v) incoming_.push_back(r);
        }
        submitted += (int64_t)v.size();
        cv_work_.notify_one();
        return true;
    }

    // Up to max completions, waiting up to timeout_us for the first (negative: forever).
    int poll(ServeCompletion *out, int max, double timeout_us) {
        std::unique_lock<std::mutex> lk(mu_);
        if (completions_.empty() && timeout_us != 0) {
            auto ready = [this] { return !completions_.empty(); };
            if (timeout_us < 0) cv_done_.wait(lk, ready);
            else cv_done_.wait_for(lk, std::chrono::microseconds((int64_t)timeout_us), ready);
        }
        int n = 0;
        while (n < max && !completions_.empty()) {
            out[n++] = completions_.front();
            completions_.pop_front();
        }
        return n;
    }

    bool failed() {
        std::lock_guard<std::mutex> lk(mu_);
        return failed_;
    }

    std::atomic<int64_t> submitted{0}, completed{0}, batches{0}, admitted{0}, max_batch_seen{0};
    std::atomic<size_t> a_in_use{0}, a_held{0}, a_peak{0};

  private:
    typedef std::chrono::steady_clock Clock;
    struct Slot {
        bool busy = false, retired = false;
        double launch_us = 0;
        Batch reqs;
    };

    void complete(Slot &sl, int status, bool release) {
        const double t = now();
        std::vector<ServeCompletion> out;
        out.reserve(sl.reqs.size());
        for (auto &rp : sl.reqs) {
            if (release) arena_.release(rp.second, rp.first.bytes);
            out.push_back(ServeCompletion{rp.first.tag, status, (int)sl.reqs.size(), rp.first.arrival, sl.launch_us, t});
        }
        a_in_use = arena_.in_use();
        sl.reqs.clear();
        sl.busy = false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto &c : out) completions_.push_back(c);
            if (status != kServeOk) failed_ = true;
        }
        completed += (int64_t)out.size();
        cv_done_.notify_all();
    }

    // Poll the busy slots; the watchdog retires a slot whose batch is overdue.
    void reap() {
        for (int i = 0; i < (int)slots_.size(); i++) {
            Slot &sl = slots_[i];
            if (!sl.busy) continue;
            const int st = exec_.poll(i);
            if (st == 1) {
                if (lim_.watchdog_us > 0 && now() - sl.launch_us > lim_.watchdog_us) {
                    sl.retired = true;
                    exec_.retire(i);
                    complete(sl, kServeHip, false);
                }
                continue;
            }
            complete(sl, st == 0 ? kServeOk : st, true);
        }
    }

    bool all_idle() const {
        for (const Slot &x : slots_)
            if (x.busy) return false;
        return true;
    }

    void admit() {
        int retries = 0;
        for (int i = 0; i < (int)slots_.size(); i++) {
            Slot &sl = slots_[i];
            if (sl.busy || sl.retired) continue;
            while (true) {
                const double t = now();
                sl.reqs.clear();
                const bool ok = admit_batch(queue_, arena_, t, lim_.max_batch, lim_.max_items,
                                            [](const R &r) { return r.items; }, [](const R &r) { return r.bytes; },
                                            &sl.reqs, all_idle());
                if (!ok) {
                    // nothing in flight and the head request fits no free extent: start the
                    // arena afresh once; if even that fails, the device has no memory for it
                    if (retries++ == 0 && !any_retired()) {
                        arena_.reset();
                        a_held = 0;
                        continue;
                    }
                    R head = queue_.front();
                    queue_.pop();
                    admitted++;
                    {
                        std::lock_guard<std::mutex> lk(mu_);
                        completions_.push_back(ServeCompletion{head.tag, kServeNoMem, 0, head.arrival, t, t});
                    }
                    completed++;
                    cv_done_.notify_all();
                    retries = 0;
                    continue;
                }
                break;
            }
            if (sl.reqs.empty()) break;
            admitted += (int64_t)sl.reqs.size();
            a_in_use = arena_.in_use();
            a_held = arena_.held();
            if (a_in_use > a_peak) a_peak = a_in_use.load();
            if ((int64_t)sl.reqs.size() > max_batch_seen) max_batch_seen = (int64_t)sl.reqs.size();
            sl.launch_us = now();
            batches++;
            sl.busy = true;
            const int st = exec_.launch(i, sl.reqs);
            if (st != 0) {
                exec_.drain(i);
                complete(sl, st, true);
            }
        }
    }

    bool any_retired() const {
        for (const Slot &x : slots_)
            if (x.retired) return true;
        return false;
    }

    void run() {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            for (R &r : incoming_) queue_.push(r.arrival, r);
            incoming_.clear();
            const bool stopping = stop_;
            lk.unlock();
            reap();
            if (!stopping) admit();
            const bool busy = !all_idle();
            const double next = queue_.next_arrival();
            lk.lock();
            if (stopping && !busy) break;
            if (!incoming_.empty()) continue;
            if (busy) {
                // batches in flight: poll their completion closely (it is the latency)
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else if (!queue_.empty() && !stopping) {
                const double wait = next - now();
                if (wait > 300.0) {
                    cv_work_.wait_for(lk, std::chrono::microseconds((int64_t)(wait - 150.0)));
                } else if (wait > 0) {
                    lk.unlock();
                    std::this_thread::yield();
                    lk.lock();
                }
            } else if (!stopping) {
                cv_work_.wait(lk, [this] { return stop_ || !incoming_.empty(); });
            }
        }
    }

    E &exec_;
    Arena &arena_;
    ServeLimits lim_;
    Clock::time_point t0_;
    std::vector<Slot> slots_;               // worker only
    ArrivalQueue<R> queue_;                 // worker only
    std::mutex mu_;                         // guards incoming_, completions_, stop_, failed_
    std::condition_variable cv_work_, cv_done_;
    std::vector<R> incoming_;
    std::deque<ServeCompletion> completions_;
    bool stop_ = false, failed_ = false;
    std::thread worker_;
};

}  // namespace gfq
