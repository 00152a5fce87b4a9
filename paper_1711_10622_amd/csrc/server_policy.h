// Host-side scheduling of the solve server: requests, per-matrix lanes, the
// slot and admission policy and the device-memory budget.  Nothing here
// touches the GPU: a lane drives its matrix's block engine through the small
// Device interface below (server.hip implements it with HIP; the CPU test
// suite implements it with a fake engine to force thread interleavings).
//
// Policy (the m realizations of Section 2.2 arriving as separate requests):
//   * every registered matrix has a lane: a host thread, a queue of requests
//     with columns still to admit, and kSlots column slots of one engine;
//   * a request's columns join free slots between rounds, oldest request
//     first, and leave as soon as their column ends;
//   * device memory is admitted against a budget: registered matrices plus
//     the engine of every lane that holds one.  A lane with work and no engine
//     joins the budget queue (first come, first served); while that queue is
//     not empty, lanes holding an engine admit no new columns (except the
//     first batch after they acquired it, so every turn makes progress),
//     finish their columns in flight and give the engine back;
//   * registration keeps every resident matrix plus the largest engine within
//     the budget, so each lane's engine fits once the others are released.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mrhs.h"

namespace mrhs {
namespace sched {

constexpr int kSlots = 16;

// The device side of one lane.  acquire/release hold and free the engine's
// memory; column(c) is a host buffer of n values that carries slot c's
// right-hand side in and its solution out; round() starts the slots in
// `admit` (their right-hand sides are in their column buffers), runs one
// round of iterations for the occupied slots, and for every occupied slot
// whose column ended sets its bit in *fin, writes its solution to column(c)
// and its outcome to info[c].  false = device failure.
class Device {
  public:
    virtual ~Device() = default;
    virtual bool acquire() = 0;
    virtual void release() = 0;
    virtual double *column(int slot) = 0;
    virtual bool round(uint32_t admit, uint32_t occupied, const double *tol, const int32_t *maxit,
                       uint32_t *fin, mrhs_col_info *info) = 0;
};

// Test instrumentation: before_wait runs with the server lock held just
// before a lane sleeps; after_wake runs with the lock released right after
// it wakes (the lane re-checks everything afterwards, so a hook that blocks
// there only delays it).  `why` is one of WaitWhy.
enum WaitWhy : int { WAIT_IDLE = 0, WAIT_BUDGET = 1 };
struct Hooks {
    void (*before_wait)(void *ctx, int lane, int why) = nullptr;
    void (*after_wake)(void *ctx, int lane, int why) = nullptr;
    void *ctx = nullptr;
};

inline double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int32_t matrix = 0;
    int32_t k = 0;
    double tol = 0.0;
    int32_t maxit = 0;
    std::vector<double> B;  // column-major n x k
    std::vector<double> X;  // column-major n x k
    std::vector<mrhs_col_info> info;
    int32_t next_col = 0;   // columns not yet admitted start here
    int32_t cols_done = 0;
    double t_submit = 0.0, t_done = 0.0;
    bool done = false;
};

class Server;

struct Slot {
    std::shared_ptr<Request> req;
    int32_t col = -1;
};

// One matrix: its queue of pending columns and the engine that solves them.
struct Lane {
    Server *srv = nullptr;
    int32_t id = 0;
    int32_t n = 0;
    size_t engine_bytes = 0;
    std::unique_ptr<Device> dev;
    std::deque<std::shared_ptr<Request>> queue;  // requests with columns still to admit
    std::thread th;
    bool has_engine = false;  // device memory currently held
    bool fresh = false;       // engine just acquired: may admit one batch even while others wait
};

struct Stats {
    double p50_ms = 0, p99_ms = 0, rhs_per_s = 0;
    int64_t submitted = 0, completed = 0, queued = 0, rhs_completed = 0;
    size_t admitted_bytes = 0;
};

class Server {
  public:
    explicit Server(size_t budget) : budget_(budget) {}
    ~Server() { shutdown(); }
    Server(const Server &) = delete;
    Server &operator=(const Server &) = delete;

    void set_hooks(const Hooks &h)
    {
        std::lock_guard<std::mutex> lk(mu_);
        hooks_ = h;
    }

    // Adds a lane for a matrix of n rows holding matrix_bytes of device
    // memory whose engine needs engine_bytes.  EBUDGET unless every resident
    // matrix, this one and the largest engine fit the budget together.
    mrhs_status add_lane(std::unique_ptr<Device> dev, int32_t n, size_t matrix_bytes, size_t engine_bytes,
                         int32_t *id, std::string *err)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (shutdown_) {
            *err = "server is shutting down";
            return MRHS_ESHUTDOWN;
        }
        size_t max_eb = engine_bytes;
        for (auto &L : lanes_)
            max_eb = std::max(max_eb, L->engine_bytes);
        if (matrix_bytes_ + matrix_bytes + max_eb > budget_) {
            *err = "resident matrices (" + std::to_string(matrix_bytes_) + " B) plus this one (" +
                   std::to_string(matrix_bytes) + " B) and the largest engine (" + std::to_string(max_eb) +
                   " B) exceed the budget (" + std::to_string(budget_) + " B)";
            return MRHS_EBUDGET;
        }
        auto L = std::make_unique<Lane>();
        L->srv = this;
        L->id = static_cast<int32_t>(lanes_.size());
        L->n = n;
        L->engine_bytes = engine_bytes;
        L->dev = std::move(dev);
        used_ += matrix_bytes;
        matrix_bytes_ += matrix_bytes;
        Lane *raw = L.get();
        lanes_.push_back(std::move(L));
        raw->th = std::thread([this, raw] { run_lane(raw); });
        *id = raw->id;
        return MRHS_OK;
    }

    // Queues k right-hand sides (host, n x k row-major) for lane `id`.
    mrhs_status submit(int32_t id, const double *B, int32_t k, double tol, int32_t maxit, uint64_t *ticket,
                       std::string *err)
    {
        int32_t n = 0;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (id < 0 || id >= static_cast<int32_t>(lanes_.size())) {
                *err = "unknown matrix id " + std::to_string(id);
                return MRHS_ENOTFOUND;
            }
            n = lanes_[id]->n;
        }
        auto r = std::make_shared<Request>();
        r->matrix = id;
        r->k = k;
        r->tol = tol;
        r->maxit = maxit;
        r->B.resize(static_cast<size_t>(n) * k);
        r->X.assign(static_cast<size_t>(n) * k, 0.0);
        r->info.assign(k, mrhs_col_info{0, 0, 0, MRHS_EAGAIN, 0.0});
        for (int32_t i = 0; i < n; ++i)  // (n, k) row-major in, column-major kept
            for (int32_t j = 0; j < k; ++j)
                r->B[static_cast<size_t>(j) * n + i] = B[static_cast<size_t>(i) * k + j];
        std::lock_guard<std::mutex> lk(mu_);
        if (shutdown_) {
            *err = "server is shutting down";
            return MRHS_ESHUTDOWN;
        }
        r->ticket = next_ticket_++;
        r->t_submit = now_s();
        if (submitted_ == 0)
            t_first_ = r->t_submit;
        submitted_ += 1;
        requests_[r->ticket] = r;
        lanes_[id]->queue.push_back(r);
        *ticket = r->ticket;
        cv_.notify_all();
        return MRHS_OK;
    }

    // EAGAIN while running; else copies X (host n x k row-major, may be
    // null) and info (k entries, may be null), forgets the ticket and returns
    // the worst column status.
    mrhs_status poll(uint64_t ticket, double *X, mrhs_col_info *info, std::string *err)
    {
        std::shared_ptr<Request> r;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = requests_.find(ticket);
            if (it == requests_.end()) {
                *err = "unknown ticket " + std::to_string(ticket);
                return MRHS_ENOTFOUND;
            }
            if (!it->second->done)
                return MRHS_EAGAIN;
            r = it->second;
            requests_.erase(it);
        }
        const int32_t n = static_cast<int32_t>(r->X.size() / r->k);
        if (X)
            for (int32_t i = 0; i < n; ++i)
                for (int32_t j = 0; j < r->k; ++j)
                    X[static_cast<size_t>(i) * r->k + j] = r->X[static_cast<size_t>(j) * n + i];
        mrhs_status worst = MRHS_OK;
        for (int32_t j = 0; j < r->k; ++j) {
            if (info)
                info[j] = r->info[j];
            if (r->info[j].status < worst)
                worst = static_cast<mrhs_status>(r->info[j].status);
        }
        return worst;
    }

    Stats stats()
    {
        std::lock_guard<std::mutex> lk(mu_);
        Stats st;
        std::vector<double> lat = latencies_ms_;
        if (!lat.empty()) {
            std::sort(lat.begin(), lat.end());
            auto pct = [&](double p) {
                const size_t i = static_cast<size_t>(p * (lat.size() - 1) + 0.5);
                return lat[std::min(i, lat.size() - 1)];
            };
            st.p50_ms = pct(0.50);
            st.p99_ms = pct(0.99);
        }
        const double span = t_last_ - t_first_;
        st.rhs_per_s = (span > 0.0) ? static_cast<double>(rhs_completed_) / span : 0.0;
        st.submitted = submitted_;
        st.completed = completed_;
        for (auto &L : lanes_)
            st.queued += static_cast<int64_t>(L->queue.size());
        st.rhs_completed = rhs_completed_;
        st.admitted_bytes = used_;
        return st;
    }

    // Stops every lane (work in progress is abandoned) and joins the threads.
    void shutdown()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            shutdown_ = true;
            cv_.notify_all();
        }
        for (auto &L : lanes_)
            if (L->th.joinable())
                L->th.join();
    }

    std::string thread_error()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return thread_error_;
    }

  private:
    void wait(std::unique_lock<std::mutex> &lk, const Lane *L, int why)
    {
        if (hooks_.before_wait)
            hooks_.before_wait(hooks_.ctx, L->id, why);
        cv_.wait(lk);
        if (hooks_.after_wake) {
            const Hooks h = hooks_;
            lk.unlock();
            h.after_wake(h.ctx, L->id, why);
            lk.lock();
        }
    }

    // caller holds mu_
    void complete_col(const std::shared_ptr<Request> &r, int col, const mrhs_col_info &info)
    {
        r->info[col] = info;
        if (++r->cols_done == r->k && !r->done) {
            r->done = true;
            r->t_done = now_s();
            completed_ += 1;
            rhs_completed_ += r->k;
            latencies_ms_.push_back((r->t_done - r->t_submit) * 1e3);
            t_last_ = r->t_done;
        }
    }

    void run_lane(Lane *L)
    {
        const int32_t n = L->n;
        const size_t vbytes = sizeof(double) * static_cast<size_t>(n);
        Slot slots[kSlots];
        auto active_count = [&]() {
            int a = 0;
            for (auto &sl : slots)
                a += sl.req != nullptr;
            return a;
        };
        for (;;) {
            uint32_t admit = 0, occupied = 0;
            double tol[kSlots] = {};
            int32_t maxit[kSlots] = {};
            {
                std::unique_lock<std::mutex> lk(mu_);
                for (;;) {
                    if (shutdown_)
                        break;
                    const int active = active_count();
                    // another lane waits for device memory: hand this engine
                    // back as soon as none of its columns is in flight
                    if (L->has_engine && active == 0 && !budget_queue_.empty()) {
                        lk.unlock();
                        L->dev->release();
                        lk.lock();
                        L->has_engine = false;
                        used_ -= L->engine_bytes;
                        cv_.notify_all();
                        continue;
                    }
                    if (active == 0 && L->queue.empty()) {
                        wait(lk, L, WAIT_IDLE);
                        continue;
                    }
                    if (!L->has_engine) {
                        auto &q = budget_queue_;
                        if (std::find(q.begin(), q.end(), L->id) == q.end()) {
                            q.push_back(L->id);
                            // an idle lane holding an engine gives it back only
                            // when it sees someone waiting: wake it up
                            cv_.notify_all();
                        }
                        if (q.front() != L->id || used_ + L->engine_bytes > budget_) {
                            wait(lk, L, WAIT_BUDGET);
                            continue;
                        }
                        q.pop_front();
                        used_ += L->engine_bytes;
                        L->has_engine = true;
                        L->fresh = true;
                        lk.unlock();
                        const bool ok = L->dev->acquire();
                        lk.lock();
                        cv_.notify_all();  // the next in line may fit as well
                        if (!ok) {
                            L->has_engine = false;
                            used_ -= L->engine_bytes;
                            thread_error_ = "engine allocation failed";
                            for (auto &r : L->queue)
                                for (int c = r->next_col; c < r->k; ++c)
                                    complete_col(r, c, mrhs_col_info{0, 0, 0, MRHS_ENOMEM, 0.0});
                            L->queue.clear();
                            continue;
                        }
                    }
                    break;
                }
                if (shutdown_)
                    break;
                // admit queued columns into free slots, oldest request first;
                // while another lane waits for device memory, only the first
                // batch after this engine was acquired
                const bool may_admit = budget_queue_.empty() || L->fresh;
                L->fresh = false;
                for (int c = 0; c < kSlots && !L->queue.empty() && may_admit; ++c) {
                    if (slots[c].req)
                        continue;
                    std::shared_ptr<Request> r = L->queue.front();
                    slots[c].req = r;
                    slots[c].col = r->next_col++;
                    tol[c] = r->tol;
                    maxit[c] = r->maxit;
                    admit |= 1u << c;
                    std::memcpy(L->dev->column(c), r->B.data() + static_cast<size_t>(slots[c].col) * n, vbytes);
                    if (r->next_col >= r->k)
                        L->queue.pop_front();
                }
                for (int c = 0; c < kSlots; ++c)
                    if (slots[c].req)
                        occupied |= 1u << c;
            }
            uint32_t fin = 0;
            mrhs_col_info info[kSlots] = {};
            const bool ok = L->dev->round(admit, occupied, tol, maxit, &fin, info);
            std::lock_guard<std::mutex> lk(mu_);
            if (!ok) {
                thread_error_ = "device error in the serving engine";
                for (auto &sl : slots)
                    if (sl.req) {
                        complete_col(sl.req, sl.col, mrhs_col_info{0, 0, 0, MRHS_EDEVICE, 0.0});
                        sl.req.reset();
                    }
                cv_.notify_all();
                continue;
            }
            fin &= occupied;
            if (fin) {
                for (int c = 0; c < kSlots; ++c) {
                    if (!((fin >> c) & 1u))
                        continue;
                    Request &r = *slots[c].req;
                    const int col = slots[c].col;
                    std::memcpy(r.X.data() + static_cast<size_t>(col) * n, L->dev->column(c), vbytes);
                    complete_col(slots[c].req, col, info[c]);
                    slots[c].req.reset();
                    slots[c].col = -1;
                }
                cv_.notify_all();
            }
        }
        L->dev->release();
    }

    std::mutex mu_;
    std::condition_variable cv_;
    Hooks hooks_;
    size_t budget_ = 0;
    size_t used_ = 0;          // resident matrices + live engines
    size_t matrix_bytes_ = 0;  // resident matrices alone
    bool shutdown_ = false;
    std::deque<int32_t> budget_queue_;  // lanes waiting for device memory, in order
    uint64_t next_ticket_ = 1;
    std::vector<std::unique_ptr<Lane>> lanes_;
    std::map<uint64_t, std::shared_ptr<Request>> requests_;
    std::vector<double> latencies_ms_;
    int64_t submitted_ = 0, completed_ = 0, rhs_completed_ = 0;
    double t_first_ = 0.0, t_last_ = 0.0;
    std::string thread_error_;
};

} // namespace sched
} // namespace mrhs
