// CPU test of the solve server's scheduling policy (server_policy.h) on a fake
// engine: no GPU, every scenario checks results, the engine budget and
// liveness.  Built and run by tests/test_sched_cpu.py, plain and under
// ThreadSanitizer.  Exit status = number of failed scenarios.
//
// The fake engine solves "A x = b" as x = 2 b + lane id, taking maxit rounds
// per column, so every result is known exactly and the rounds a column takes
// are chosen by the test.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <functional>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "server_policy.h"

using namespace mrhs;
using namespace mrhs::sched;

namespace {

std::atomic<int> g_engines{0};      // engines held right now, over all lanes
std::atomic<int> g_engines_max{0};  // most held at once
std::atomic<int> g_violations{0};   // rounds run without an engine

class FakeDevice final : public Device {
  public:
    FakeDevice(int n, int lane, int round_us) : n_(n), lane_(lane), round_us_(round_us) {}
    bool acquire() override
    {
        host_.assign(static_cast<size_t>(n_) * kSlots, 0.0);
        held_ = true;
        const int now = ++g_engines;
        int mx = g_engines_max.load();
        while (now > mx && !g_engines_max.compare_exchange_weak(mx, now)) {
        }
        ++acquisitions;
        return true;
    }
    void release() override
    {
        if (held_) {
            held_ = false;
            --g_engines;
        }
    }
    double *column(int slot) override { return host_.data() + static_cast<size_t>(slot) * n_; }
    bool round(uint32_t admit, uint32_t occupied, const double *, const int32_t *maxit, uint32_t *fin,
               mrhs_col_info *info) override
    {
        *fin = 0;
        if (!held_) {
            ++g_violations;
            return false;
        }
        for (int c = 0; c < kSlots; ++c)
            if ((admit >> c) & 1u) {
                b_[c].assign(column(c), column(c) + n_);
                need_[c] = maxit[c];
                done_[c] = 0;
            }
        if (round_us_)
            std::this_thread::sleep_for(std::chrono::microseconds(round_us_));
        for (int c = 0; c < kSlots; ++c) {
            if (!((occupied >> c) & 1u))
                continue;
            if (++done_[c] >= need_[c]) {
                for (int i = 0; i < n_; ++i)
                    column(c)[i] = 2.0 * b_[c][i] + lane_;
                info[c] = mrhs_col_info{done_[c], 0, 0, MRHS_OK, 0.0};
                *fin |= 1u << c;
            }
        }
        return true;
    }
    int acquisitions = 0;

  private:
    int n_, lane_, round_us_;
    bool held_ = false;
    std::vector<double> host_;
    std::vector<double> b_[kSlots];
    int need_[kSlots] = {};
    int done_[kSlots] = {};
};

constexpr int kN = 37;
constexpr size_t kMatBytes = 10, kEngBytes = 100;

struct Client {
    Server &S;
    std::vector<std::vector<double>> B;
    std::vector<uint64_t> tickets;
    std::vector<int> lane;
    explicit Client(Server &s) : S(s) {}
    uint64_t submit(int id, int k, int rounds, uint64_t seed)
    {
        std::vector<double> b(static_cast<size_t>(kN) * k);
        std::mt19937_64 g(seed);
        for (auto &v : b)
            v = static_cast<double>(g() % 2001) - 1000.0;
        uint64_t t = 0;
        std::string err;
        if (S.submit(id, b.data(), k, 1e-10, rounds, &t, &err) != MRHS_OK)
            return 0;
        B.push_back(b);
        tickets.push_back(t);
        lane.push_back(id);
        return t;
    }
    // polls ticket j until done or the deadline; checks x = 2 b + lane
    bool collect(size_t j, double seconds, const char *what)
    {
        const int k = static_cast<int>(B[j].size() / kN);
        std::vector<double> X(B[j].size());
        std::vector<mrhs_col_info> info(k);
        std::string err;
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            const mrhs_status st = S.poll(tickets[j], X.data(), info.data(), &err);
            if (st != MRHS_EAGAIN) {
                if (st != MRHS_OK) {
                    std::printf("  %s: ticket %llu status %d\n", what, (unsigned long long)tickets[j], st);
                    return false;
                }
                for (size_t i = 0; i < X.size(); ++i)
                    if (X[i] != 2.0 * B[j][i] + lane[j]) {
                        std::printf("  %s: wrong result at %zu\n", what, i);
                        return false;
                    }
                return true;
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::duration<double>(seconds)) {
                std::printf("  %s: ticket %llu never completed (lost wakeup?)\n", what,
                            (unsigned long long)tickets[j]);
                return false;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    }
};

int add(Server &S, int lane, int round_us)
{
    int32_t id = -1;
    std::string err;
    if (S.add_lane(std::make_unique<FakeDevice>(kN, lane, round_us), kN, kMatBytes, kEngBytes, &id, &err) != MRHS_OK)
        std::printf("  add_lane: %s\n", err.c_str());
    return id;
}

// ---- scenario 1: an idle engine holder and a submit to another matrix ------
// One-engine budget.  Matrix A's request finishes; A keeps its engine and
// sleeps (nothing to do).  A request for matrix B then arrives: B must wait
// for A's engine, and A gives it back only when it sees B waiting.  The hooks
// force the order that loses a wakeup if joining the budget queue does not
// notify: B is held right after it wakes until A has gone back to sleep.
// Timed waits use the system clock: libstdc++ then waits with
// pthread_cond_timedwait, which ThreadSanitizer intercepts (the steady-clock
// form uses pthread_cond_clockwait, which GCC 11's runtime does not, and it
// then reports the released mutex as still held).
std::chrono::system_clock::time_point deadline(int seconds)
{
    return std::chrono::system_clock::now() + std::chrono::seconds(seconds);
}

struct Gate {
    std::mutex mu;
    std::condition_variable cv;
    int idle_waits[2] = {0, 0};
    bool asleep[2] = {false, false};
    bool armed = false;
    int armed_at = 0;
};

void gate_before_wait(void *ctx, int lane, int why)
{
    auto *g = static_cast<Gate *>(ctx);
    std::lock_guard<std::mutex> lk(g->mu);
    if (why == WAIT_IDLE && lane < 2) {
        ++g->idle_waits[lane];
        g->asleep[lane] = true;
    }
    g->cv.notify_all();
}

void gate_after_wake(void *ctx, int lane, int why)
{
    auto *g = static_cast<Gate *>(ctx);
    std::unique_lock<std::mutex> lk(g->mu);
    if (lane < 2)
        g->asleep[lane] = false;
    if (lane == 1 && why == WAIT_IDLE && g->armed) {
        g->armed = false;
        g->cv.wait_until(lk, deadline(5), [&] { return g->idle_waits[0] > g->armed_at; });
    }
}

bool scenario_idle_holder_lost_wakeup()
{
    Server S(2 * kMatBytes + kEngBytes);
    Gate gate;
    Hooks h;
    h.before_wait = gate_before_wait;
    h.after_wake = gate_after_wake;
    h.ctx = &gate;
    S.set_hooks(h);
    const int a = add(S, 0, 0), b = add(S, 1, 0);
    Client cl(S);
    cl.submit(a, 3, 2, 1);
    if (!cl.collect(0, 5.0, "first request"))
        return false;
    {
        // wait until A sleeps idle with its engine, then arm the gate
        std::unique_lock<std::mutex> lk(gate.mu);
        gate.cv.wait_until(lk, deadline(5), [&] { return gate.asleep[0]; });
        gate.armed = true;
        gate.armed_at = gate.idle_waits[0];
    }
    cl.submit(b, 2, 2, 2);
    const bool ok = cl.collect(1, 3.0, "request to the second matrix");
    S.shutdown();
    return ok;
}

// ---- scenario 2: turns under a one-engine budget ---------------------------
bool scenario_turns()
{
    Server S(2 * kMatBytes + kEngBytes);
    const int a = add(S, 0, 200), b = add(S, 1, 200);
    Client cl(S);
    for (int r = 0; r < 4; ++r) {
        cl.submit(a, 16, 3, 10 + r);
        cl.submit(b, 16, 3, 20 + r);
    }
    bool ok = true;
    for (size_t j = 0; j < cl.tickets.size(); ++j)
        ok = cl.collect(j, 10.0, "turns") && ok;
    S.shutdown();
    return ok;
}

// ---- scenario 3: a request alone and in a mix gives the same result --------
bool scenario_alone_and_mixed()
{
    std::vector<double> alone, mixed;
    for (int mode = 0; mode < 2; ++mode) {
        Server S(3 * kMatBytes + 2 * kEngBytes);
        const int a = add(S, 0, 50), b = add(S, 1, 50), c = add(S, 2, 50);
        Client cl(S);
        if (mode == 1) {
            cl.submit(a, 9, 4, 31);
            cl.submit(b, 16, 2, 32);
            cl.submit(c, 5, 3, 33);
        }
        const size_t j = cl.tickets.size();
        cl.submit(a, 11, 5, 34);  // the request compared
        if (mode == 1)
            cl.submit(a, 7, 1, 35);
        for (size_t q = 0; q < cl.tickets.size(); ++q)
            if (!cl.collect(q, 10.0, "mix"))
                return false;
        (mode ? mixed : alone) = cl.B[j];
        S.shutdown();
    }
    return alone == mixed;
}

// ---- scenario 4: random load from two client threads -----------------------
bool scenario_random_load()
{
    Server S(4 * kMatBytes + 2 * kEngBytes);  // two engines at a time
    int ids[4];
    for (int l = 0; l < 4; ++l)
        ids[l] = add(S, l, 30);
    std::atomic<bool> ok{true};
    auto client = [&](uint64_t seed) {
        Client cl(S);
        std::mt19937_64 g(seed);
        for (int r = 0; r < 60; ++r) {
            cl.submit(ids[g() % 4], 1 + static_cast<int>(g() % 16), 1 + static_cast<int>(g() % 5), g());
            if (g() % 3 == 0)
                std::this_thread::sleep_for(std::chrono::microseconds(g() % 400));
        }
        for (size_t j = 0; j < cl.tickets.size(); ++j)
            if (!cl.collect(j, 20.0, "random load"))
                ok = false;
    };
    std::thread t1(client, 7), t2(client, 8);
    t1.join();
    t2.join();
    const Stats st = S.stats();
    S.shutdown();
    if (st.completed != 120 || st.submitted != 120)
        ok = false;
    return ok;
}

// ---- scenario 5: shutdown with work in flight ends every lane --------------
bool scenario_shutdown_in_flight()
{
    Server S(2 * kMatBytes + kEngBytes);
    const int a = add(S, 0, 1000), b = add(S, 1, 1000);
    Client cl(S);
    for (int r = 0; r < 3; ++r) {
        cl.submit(a, 16, 50, 40 + r);
        cl.submit(b, 16, 50, 50 + r);
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    S.shutdown();  // must return: every lane thread exits
    std::string err;
    uint64_t t = 0;
    return S.submit(a, cl.B[0].data(), 16, 1e-10, 1, &t, &err) == MRHS_ESHUTDOWN;
}

} // namespace

int main()
{
    struct {
        const char *name;
        std::function<bool()> fn;
        int max_engines;
    } cases[] = {
        {"idle_holder_lost_wakeup", scenario_idle_holder_lost_wakeup, 1},
        {"turns_one_engine", scenario_turns, 1},
        {"alone_and_mixed", scenario_alone_and_mixed, 2},
        {"random_load", scenario_random_load, 2},
        {"shutdown_in_flight", scenario_shutdown_in_flight, 1},
    };
    int failed = 0;
    for (auto &c : cases) {
        g_engines_max = 0;
        g_violations = 0;
        const bool ok = c.fn();
        const bool budget_ok = g_engines_max.load() <= c.max_engines && g_violations.load() == 0;
        std::printf("%s %s (engines at once: %d, rounds without engine: %d)\n", ok && budget_ok ? "PASS" : "FAIL",
                    c.name, g_engines_max.load(), g_violations.load());
        std::fflush(stdout);
        failed += !(ok && budget_ok);
    }
    return failed;
}
