// Solve server: continuous batching of pressure solves from independent
// ensemble members (the m realizations of Section 2 arriving as separate
// requests).  Every registered matrix stays resident; its right-hand sides
// are solved in a block of kMaxM column slots by one engine (solver.hip)
// driven by its own host thread on its own HIP stream, so different matrices
// overlap on the device.  A request's columns join the block as slots free
// up, between rounds of iterations, and leave it as soon as they finish.
// Device memory is admitted against a byte budget: a matrix's engine is
// allocated when it has work and the budget allows.  Matrices waiting for
// budget are served first come, first served; while one waits, every engine
// stops admitting new columns, finishes the ones in flight and is released,
// so a busy matrix cannot starve another.  Registration keeps every resident
// matrix plus the largest engine within the budget, so each matrix's engine
// fits once the others are released.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {
namespace {

constexpr int kSlots = kMaxM;

__global__ void k_scatter_col(double *__restrict__ blk, const double *__restrict__ v, int32_t n, int c)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        blk[i * kSlots + c] = v[i];
}

__global__ void k_gather_col(double *__restrict__ v, const double *__restrict__ blk, int32_t n, int c)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        v[i] = blk[i * kSlots + c];
}

double now_s()
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

struct Slot {
    std::shared_ptr<Request> req;
    int32_t col = -1;
};

struct Server;

// One matrix: its queue of pending columns and the engine that solves them.
struct Lane {
    Server *srv = nullptr;
    int32_t id = 0;
    mrhs_csr A = nullptr;
    size_t engine_bytes = 0;
    std::deque<std::shared_ptr<Request>> queue;  // requests with columns still to admit
    std::thread th;
    bool has_engine = false;  // device memory currently held
    bool fresh = false;       // engine just acquired: may admit one batch even while others wait
};

struct Server {
    std::mutex mu;
    std::condition_variable cv;
    size_t budget = 0;
    size_t used = 0;  // resident matrices + live engines
    uint32_t flags = 0;
    bool shutdown = false;
    size_t matrix_bytes = 0;                // resident matrices alone
    std::deque<int32_t> budget_queue;       // lanes waiting for device memory, in order
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::map<uint64_t, std::shared_ptr<Request>> requests;
    std::vector<double> latencies_ms;
    int64_t submitted = 0, completed = 0, rhs_completed = 0;
    double t_first = 0.0, t_last = 0.0;
    std::string thread_error;
};

// Device resources of one engine.
struct EngineMem {
    hipStream_t s = nullptr;
    void *ws = nullptr;
    double *B = nullptr, *X = nullptr, *stage = nullptr;  // stage: kSlots contiguous n-vectors
    double *host = nullptr;                               // pinned, kSlots n-vectors
    std::unique_ptr<Engine> eng;

    void release()
    {
        eng.reset();
        if (s)
            (void)hipStreamSynchronize(s);
        void *dev[] = {ws, B, X, stage};
        for (void *p : dev)
            if (p)
                (void)hipFree(p);
        if (host)
            (void)hipHostFree(host);
        if (s)
            (void)hipStreamDestroy(s);
        s = nullptr;
        ws = nullptr;
        B = X = stage = host = nullptr;
    }
};

size_t engine_bytes(const mrhs_csr_s &A, uint32_t flags)
{
    const size_t blk = sizeof(double) * static_cast<size_t>(A.n) * kSlots;
    return Engine::workspace_bytes(A, kSlots, flags) + 3 * blk;
}

bool alloc_engine(EngineMem &em, const mrhs_csr_s &A, uint32_t flags)
{
    const size_t blk = sizeof(double) * static_cast<size_t>(A.n) * kSlots;
    if (hipStreamCreateWithFlags(&em.s, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&em.ws, Engine::workspace_bytes(A, kSlots, flags)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&em.B), blk) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&em.X), blk) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&em.stage), blk) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&em.host), blk, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        em.release();
        return false;
    }
    em.eng.reset(new Engine(A, kSlots, flags, em.ws, em.B, em.X, em.s));
    if (em.eng->reset() != MRHS_OK) {
        em.release();
        return false;
    }
    return true;
}

void fail_request_col(Server &S, const std::shared_ptr<Request> &r, int col, mrhs_status st)
{
    r->info[col] = mrhs_col_info{0, 0, 0, st, 0.0};
    if (++r->cols_done == r->k && !r->done) {
        r->done = true;
        r->t_done = now_s();
        S.completed += 1;
        S.rhs_completed += r->k;
        S.latencies_ms.push_back((r->t_done - r->t_submit) * 1e3);
        S.t_last = r->t_done;
    }
}

void lane_main(Lane *L)
{
    Server &S = *L->srv;
    const mrhs_csr_s &A = *L->A;
    (void)hipSetDevice(A.device);
    const uint32_t eflags = (S.flags & MRHS_SERVER_MIXED) ? MRHS_MIXED : 0u;
    const int32_t n = A.n;
    const size_t vbytes = sizeof(double) * static_cast<size_t>(n);
    EngineMem em;
    Slot slots[kSlots];
    auto active_count = [&]() {
        int a = 0;
        for (auto &sl : slots)
            a += sl.req != nullptr;
        return a;
    };
    const unsigned grid = static_cast<unsigned>((n + 255) / 256);
    for (;;) {
        uint32_t admit = 0;
        double tol[kSlots] = {};
        int32_t maxit[kSlots] = {};
        {
            std::unique_lock<std::mutex> lk(S.mu);
            for (;;) {
                if (S.shutdown)
                    break;
                const int active = active_count();
                // another matrix waits for device memory: hand this engine back
                // as soon as none of its columns is in flight
                if (L->has_engine && active == 0 && !S.budget_queue.empty()) {
                    lk.unlock();
                    em.release();
                    lk.lock();
                    L->has_engine = false;
                    S.used -= L->engine_bytes;
                    S.cv.notify_all();
                    continue;
                }
                if (active == 0 && L->queue.empty()) {
                    S.cv.wait(lk);
                    continue;
                }
                if (!L->has_engine) {
                    auto &q = S.budget_queue;
                    if (std::find(q.begin(), q.end(), L->id) == q.end())
                        q.push_back(L->id);
                    if (q.front() != L->id || S.used + L->engine_bytes > S.budget) {
                        S.cv.wait(lk);
                        continue;
                    }
                    q.pop_front();
                    S.used += L->engine_bytes;
                    L->has_engine = true;
                    L->fresh = true;
                    lk.unlock();
                    const bool ok = alloc_engine(em, A, eflags);
                    lk.lock();
                    S.cv.notify_all();  // the next in line may fit as well
                    if (!ok) {
                        L->has_engine = false;
                        S.used -= L->engine_bytes;
                        S.thread_error = "engine allocation failed";
                        for (auto &r : L->queue)
                            for (int c = r->next_col; c < r->k; ++c)
                                fail_request_col(S, r, c, MRHS_ENOMEM);
                        L->queue.clear();
                        continue;
                    }
                }
                break;
            }
            if (S.shutdown)
                break;
            // admit queued columns into free slots, oldest request first; while
            // another matrix waits for device memory, only the first batch
            // after this engine was acquired (so every turn makes progress)
            const bool may_admit = S.budget_queue.empty() || L->fresh;
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
                std::memcpy(em.host + static_cast<size_t>(c) * n,
                            r->B.data() + static_cast<size_t>(slots[c].col) * n, vbytes);
                if (r->next_col >= r->k)
                    L->queue.pop_front();
            }
        }
        bool ok = true;
        if (admit) {
            for (int c = 0; c < kSlots && ok; ++c) {
                if (!((admit >> c) & 1u))
                    continue;
                ok = hipMemcpyAsync(em.stage + static_cast<size_t>(c) * n, em.host + static_cast<size_t>(c) * n,
                                    vbytes, hipMemcpyHostToDevice, em.s) == hipSuccess;
                hipLaunchKernelGGL(k_scatter_col, dim3(grid), dim3(256), 0, em.s, em.B,
                                   em.stage + static_cast<size_t>(c) * n, n, c);
                ok = ok && hipGetLastError() == hipSuccess;
            }
            ok = ok && em.eng->start(admit, tol, maxit, false) == MRHS_OK;
        }
        bool busy = false;
        ok = ok && em.eng->advance(&busy) == MRHS_OK;
        uint32_t fin = 0;
        if (ok) {
            const uint32_t term = em.eng->terminal_mask();
            for (int c = 0; c < kSlots; ++c)
                if (slots[c].req && ((term >> c) & 1u))
                    fin |= 1u << c;
        }
        if (ok && fin) {
            ok = em.eng->finish(fin) == MRHS_OK;
            for (int c = 0; c < kSlots && ok; ++c) {
                if (!((fin >> c) & 1u))
                    continue;
                hipLaunchKernelGGL(k_gather_col, dim3(grid), dim3(256), 0, em.s,
                                   em.stage + static_cast<size_t>(c) * n, em.X, n, c);
                ok = hipGetLastError() == hipSuccess &&
                     hipMemcpyAsync(em.host + static_cast<size_t>(c) * n, em.stage + static_cast<size_t>(c) * n,
                                    vbytes, hipMemcpyDeviceToHost, em.s) == hipSuccess;
            }
            ok = ok && em.eng->read_ctl() == MRHS_OK;
        }
        std::lock_guard<std::mutex> lk(S.mu);
        if (!ok) {
            S.thread_error = "device error in the serving engine";
            for (auto &sl : slots)
                if (sl.req) {
                    fail_request_col(S, sl.req, sl.col, MRHS_EDEVICE);
                    sl.req.reset();
                }
            S.cv.notify_all();
            continue;
        }
        if (fin) {
            const Ctl &h = em.eng->host();
            const bool mixed = (eflags & MRHS_MIXED) != 0;
            for (int c = 0; c < kSlots; ++c) {
                if (!((fin >> c) & 1u))
                    continue;
                Request &r = *slots[c].req;
                const int col = slots[c].col;
                std::memcpy(r.X.data() + static_cast<size_t>(col) * n, em.host + static_cast<size_t>(c) * n,
                            vbytes);
                r.info[col] = mrhs_col_info{mixed ? h.total_iters[c] : h.iters[c], h.restarts[c],
                                            mixed ? h.outer[c] : 0, column_status(h.status[c]), h.relres[c]};
                if (++r.cols_done == r.k) {
                    r.done = true;
                    r.t_done = now_s();
                    S.completed += 1;
                    S.rhs_completed += r.k;
                    S.latencies_ms.push_back((r.t_done - r.t_submit) * 1e3);
                    S.t_last = r.t_done;
                }
                slots[c].req.reset();
                slots[c].col = -1;
            }
            S.cv.notify_all();
        }
        (void)busy;
    }
    em.release();
}

} // namespace
} // namespace mrhs

struct mrhs_server_s {
    mrhs::Server impl;
};

using namespace mrhs;

MRHS_API mrhs_status solve_server_create(size_t hbm_budget_bytes, uint32_t flags, mrhs_server *out)
{
    clear_error();
    if (!out)
        return set_error(MRHS_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~MRHS_SERVER_MIXED)
        return set_error(MRHS_EINVAL, "unknown flags 0x%x", flags);
    auto *s = new (std::nothrow) mrhs_server_s();
    if (!s)
        return set_error(MRHS_ENOMEM, "host allocation failed");
    s->impl.budget = hbm_budget_bytes;
    s->impl.flags = flags;
    *out = s;
    return MRHS_OK;
}

MRHS_API mrhs_status solve_server_register(mrhs_server srv, mrhs_csr A, int32_t *matrix_id)
{
    clear_error();
    if (!srv || !A || !matrix_id)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (A->n == 0)
        return set_error(MRHS_EINVAL, "empty matrix");
    if (A->zero_diag)
        return set_error(MRHS_EINVAL, "the matrix has a zero diagonal entry");
    Server &S = srv->impl;
    const uint32_t eflags = (S.flags & MRHS_SERVER_MIXED) ? MRHS_MIXED : 0u;
    const size_t eb = engine_bytes(*A, eflags);
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.shutdown)
        return set_error(MRHS_ESHUTDOWN, "server is shutting down");
    // every resident matrix plus the largest engine must fit, so that each
    // matrix can run once the other engines are released
    size_t max_eb = eb;
    for (auto &L : S.lanes)
        max_eb = std::max(max_eb, L->engine_bytes);
    if (S.matrix_bytes + A->bytes + max_eb > S.budget)
        return set_error(MRHS_EBUDGET,
                         "resident matrices (%zu B) plus this one (%zu B) and the largest engine (%zu B) "
                         "exceed the budget (%zu B)",
                         S.matrix_bytes, A->bytes, max_eb, S.budget);
    auto L = std::make_unique<Lane>();
    L->srv = &S;
    L->id = static_cast<int32_t>(S.lanes.size());
    L->A = A;
    L->engine_bytes = eb;
    S.used += A->bytes;
    S.matrix_bytes += A->bytes;
    Lane *raw = L.get();
    S.lanes.push_back(std::move(L));
    raw->th = std::thread(lane_main, raw);
    *matrix_id = raw->id;
    return MRHS_OK;
}

MRHS_API mrhs_status solve_server_submit(mrhs_server srv, int32_t matrix_id, const double *B, int32_t k, double tol,
                                         int32_t maxit, uint64_t *ticket)
{
    clear_error();
    if (!srv || !B || !ticket)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (k < 1)
        return set_error(MRHS_EINVAL, "k = %d < 1", k);
    if (!(tol > 0.0) || maxit < 1)
        return set_error(MRHS_EINVAL, "tol must be positive and maxit at least 1");
    Server &S = srv->impl;
    int32_t n = 0;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (matrix_id < 0 || matrix_id >= static_cast<int32_t>(S.lanes.size()))
            return set_error(MRHS_ENOTFOUND, "unknown matrix id %d", matrix_id);
        n = S.lanes[matrix_id]->A->n;
    }
    auto r = std::make_shared<Request>();
    r->matrix = matrix_id;
    r->k = k;
    r->tol = tol;
    r->maxit = maxit;
    r->B.resize(static_cast<size_t>(n) * k);
    r->X.assign(static_cast<size_t>(n) * k, 0.0);
    r->info.assign(k, mrhs_col_info{0, 0, 0, MRHS_EAGAIN, 0.0});
    for (int32_t i = 0; i < n; ++i)  // (n, k) row-major in, column-major kept
        for (int32_t j = 0; j < k; ++j)
            r->B[static_cast<size_t>(j) * n + i] = B[static_cast<size_t>(i) * k + j];
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.shutdown)
        return set_error(MRHS_ESHUTDOWN, "server is shutting down");
    r->ticket = S.next_ticket++;
    r->t_submit = now_s();
    if (S.submitted == 0)
        S.t_first = r->t_submit;
    S.submitted += 1;
    S.requests[r->ticket] = r;
    S.lanes[matrix_id]->queue.push_back(r);
    *ticket = r->ticket;
    S.cv.notify_all();
    return MRHS_OK;
}

MRHS_API mrhs_status solve_server_poll(mrhs_server srv, uint64_t ticket, double *X, mrhs_col_info *info)
{
    clear_error();
    if (!srv)
        return set_error(MRHS_EINVAL, "server handle is NULL");
    Server &S = srv->impl;
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.requests.find(ticket);
        if (it == S.requests.end())
            return set_error(MRHS_ENOTFOUND, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
        if (!it->second->done)
            return MRHS_EAGAIN;
        r = it->second;
        S.requests.erase(it);
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

MRHS_API mrhs_status solve_server_stats(mrhs_server srv, mrhs_server_stats *out)
{
    clear_error();
    if (!srv || !out)
        return set_error(MRHS_EINVAL, "NULL argument");
    Server &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    mrhs_server_stats st{};
    std::vector<double> lat = S.latencies_ms;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const size_t i = static_cast<size_t>(p * (lat.size() - 1) + 0.5);
            return lat[std::min(i, lat.size() - 1)];
        };
        st.p50_ms = pct(0.50);
        st.p99_ms = pct(0.99);
    }
    const double span = S.t_last - S.t_first;
    st.rhs_per_s = (span > 0.0) ? static_cast<double>(S.rhs_completed) / span : 0.0;
    st.submitted = S.submitted;
    st.completed = S.completed;
    int64_t queued = 0;
    for (auto &L : S.lanes)
        queued += static_cast<int64_t>(L->queue.size());
    st.queued = queued;
    st.rhs_completed = S.rhs_completed;
    st.admitted_bytes = S.used;
    *out = st;
    return MRHS_OK;
}

MRHS_API mrhs_status solve_server_destroy(mrhs_server srv)
{
    clear_error();
    if (!srv)
        return MRHS_OK;
    Server &S = srv->impl;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.shutdown = true;
        S.cv.notify_all();
    }
    for (auto &L : S.lanes)
        if (L->th.joinable())
            L->th.join();
    delete srv;
    return MRHS_OK;
}
