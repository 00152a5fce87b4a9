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
#include <memory>
#include <string>

#include "internal.h"
#include "server_policy.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {
namespace {

constexpr int kSlots = sched::kSlots;
static_assert(kSlots == kMaxM, "a lane's slots are the columns of one engine block");

// column c of the engine's block (solver numbering: row i is the caller's
// row perm[i], or row i) from / to an n-vector in the caller's numbering
__global__ void k_scatter_col(double *__restrict__ blk, const double *__restrict__ v, const int32_t *__restrict__ perm,
                              int32_t n, int c)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        blk[i * kSlots + c] = v[perm ? perm[i] : i];
}

__global__ void k_gather_col(double *__restrict__ v, const double *__restrict__ blk, const int32_t *__restrict__ perm,
                             int32_t n, int c)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        v[perm ? perm[i] : i] = blk[i * kSlots + c];
}

size_t engine_bytes(const mrhs_csr_s &A, uint32_t flags, const AmgDev *amg)
{
    const size_t blk = sizeof(double) * static_cast<size_t>(A.n) * kSlots;
    return Engine::workspace_bytes(A, kSlots, flags, amg) + 3 * blk;
}

// The engine of one lane on the GPU: a stream, the block workspace, device
// blocks B and X of n x kSlots, a staging block (kSlots contiguous
// n-vectors) and pinned host columns; with an AMG hierarchy (owned by the
// lane) the engine runs AMG-preconditioned BiCGStab.
class HipDevice final : public sched::Device {
  public:
    HipDevice(const mrhs_csr_s &A, uint32_t eflags, mrhs_amg H)
        : A_(A), eflags_(eflags), H_(H), amg_(H ? amg_dev_of(H) : nullptr)
    {
    }
    ~HipDevice() override
    {
        release();
        if (H_)
            (void)amg_destroy(H_);
    }

    bool acquire() override
    {
        (void)hipSetDevice(A_.device);
        const size_t blk = sizeof(double) * static_cast<size_t>(A_.n) * kSlots;
        if (hipStreamCreateWithFlags(&s_, hipStreamNonBlocking) != hipSuccess ||
            hipMalloc(&ws_, Engine::workspace_bytes(A_, kSlots, eflags_, amg_)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&B_), blk) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&X_), blk) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&stage_), blk) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&host_), blk, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            release();
            return false;
        }
        eng_.reset(new Engine(A_, kSlots, eflags_, ws_, B_, X_, s_, nullptr, amg_));
        if (eng_->reset() != MRHS_OK) {
            release();
            return false;
        }
        return true;
    }

    void release() override
    {
        eng_.reset();
        if (s_)
            (void)hipStreamSynchronize(s_);
        void *dev[] = {ws_, B_, X_, stage_};
        for (void *p : dev)
            if (p)
                (void)hipFree(p);
        if (host_)
            (void)hipHostFree(host_);
        if (s_)
            (void)hipStreamDestroy(s_);
        s_ = nullptr;
        ws_ = nullptr;
        B_ = X_ = stage_ = host_ = nullptr;
    }

    // only called while the engine is held (columns are admitted and
    // collected only then)
    double *column(int slot) override { return host_ + static_cast<size_t>(slot) * A_.n; }

    bool round(uint32_t admit, uint32_t occupied, const double *tol, const int32_t *maxit, uint32_t *fin,
               mrhs_col_info *info) override
    {
        *fin = 0;
        if (!eng_ || !host_)
            return false;
        const int32_t n = A_.n;
        const size_t vbytes = sizeof(double) * static_cast<size_t>(n);
        const unsigned grid = static_cast<unsigned>((n + 255) / 256);
        bool ok = true;
        if (admit) {
            for (int c = 0; c < kSlots && ok; ++c) {
                if (!((admit >> c) & 1u))
                    continue;
                ok = hipMemcpyAsync(stage_ + static_cast<size_t>(c) * n, host_ + static_cast<size_t>(c) * n, vbytes,
                                    hipMemcpyHostToDevice, s_) == hipSuccess;
                hipLaunchKernelGGL(k_scatter_col, dim3(grid), dim3(256), 0, s_, B_,
                                   stage_ + static_cast<size_t>(c) * n, A_.perm, n, c);
                ok = ok && hipGetLastError() == hipSuccess;
            }
            ok = ok && eng_->start(admit, tol, maxit, false) == MRHS_OK;
        }
        bool busy = false;
        ok = ok && eng_->advance(&busy) == MRHS_OK;
        if (!ok)
            return false;
        const uint32_t done = eng_->terminal_mask() & occupied;
        if (!done)
            return true;
        ok = eng_->finish(done) == MRHS_OK;
        for (int c = 0; c < kSlots && ok; ++c) {
            if (!((done >> c) & 1u))
                continue;
            hipLaunchKernelGGL(k_gather_col, dim3(grid), dim3(256), 0, s_, stage_ + static_cast<size_t>(c) * n, X_,
                               A_.perm, n, c);
            ok = hipGetLastError() == hipSuccess &&
                 hipMemcpyAsync(host_ + static_cast<size_t>(c) * n, stage_ + static_cast<size_t>(c) * n, vbytes,
                                hipMemcpyDeviceToHost, s_) == hipSuccess;
        }
        ok = ok && eng_->read_ctl() == MRHS_OK;
        if (!ok)
            return false;
        const Ctl &h = eng_->host();
        const bool mixed = (eflags_ & MRHS_MIXED) != 0;
        for (int c = 0; c < kSlots; ++c)
            if ((done >> c) & 1u)
                info[c] = mrhs_col_info{mixed ? h.total_iters[c] : h.iters[c], h.restarts[c], mixed ? h.outer[c] : 0,
                                        column_status(h.status[c]), h.relres[c]};
        *fin = done;
        return true;
    }

  private:
    const mrhs_csr_s &A_;
    uint32_t eflags_;
    mrhs_amg H_ = nullptr;
    const AmgDev *amg_ = nullptr;
    hipStream_t s_ = nullptr;
    void *ws_ = nullptr;
    double *B_ = nullptr, *X_ = nullptr, *stage_ = nullptr;
    double *host_ = nullptr;  // pinned, kSlots n-vectors
    std::unique_ptr<Engine> eng_;
};

} // namespace
} // namespace mrhs

struct mrhs_server_s {
    explicit mrhs_server_s(size_t budget) : impl(budget) {}
    mrhs::sched::Server impl;
    uint32_t flags = 0;
};

using namespace mrhs;

MRHS_API mrhs_status solve_server_create(size_t hbm_budget_bytes, uint32_t flags, mrhs_server *out)
{
    clear_error();
    if (!out)
        return set_error(MRHS_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(MRHS_SERVER_MIXED | MRHS_SERVER_AMG))
        return set_error(MRHS_EINVAL, "unknown flags 0x%x", flags);
    auto *s = new (std::nothrow) mrhs_server_s(hbm_budget_bytes);
    if (!s)
        return set_error(MRHS_ENOMEM, "host allocation failed");
    s->flags = flags;
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
    // binary32 in the engine: the inner Jacobi solves, or the V-cycle with AMG
    const bool use_amg = (srv->flags & MRHS_SERVER_AMG) != 0;
    const bool f32 = (srv->flags & MRHS_SERVER_MIXED) != 0;
    const uint32_t eflags = f32 ? (use_amg ? kAmgVc32 : MRHS_MIXED) : 0u;
    mrhs_amg H = nullptr;
    if (use_amg) {
        mrhs_status a = amg_create(A, 0.0, 0, 0, &H);
        if (a == MRHS_OK && f32 && (a = amg_make32(H)) != MRHS_OK)
            (void)amg_destroy(H);
        if (a != MRHS_OK)
            return a;  // amg_create / amg_make32 set the message
    }
    const AmgDev *amg = H ? amg_dev_of(H) : nullptr;
    const size_t resident = A->bytes + (H ? amg_bytes_of(H) : 0);
    const size_t eb = engine_bytes(*A, eflags, amg);
    std::string err;
    // the lane owns the hierarchy from here (freed with it, or now if it is refused)
    const mrhs_status st =
        srv->impl.add_lane(std::make_unique<HipDevice>(*A, eflags, H), A->n, resident, eb, matrix_id, &err);
    return st == MRHS_OK ? st : set_error(st, "%s", err.c_str());
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
    std::string err;
    const mrhs_status st = srv->impl.submit(matrix_id, B, k, tol, maxit, ticket, &err);
    return st == MRHS_OK ? st : set_error(st, "%s", err.c_str());
}

MRHS_API mrhs_status solve_server_poll(mrhs_server srv, uint64_t ticket, double *X, mrhs_col_info *info)
{
    clear_error();
    if (!srv)
        return set_error(MRHS_EINVAL, "server handle is NULL");
    std::string err;
    const mrhs_status st = srv->impl.poll(ticket, X, info, &err);
    return st == MRHS_ENOTFOUND ? set_error(st, "%s", err.c_str()) : st;
}

MRHS_API mrhs_status solve_server_stats(mrhs_server srv, mrhs_server_stats *out)
{
    clear_error();
    if (!srv || !out)
        return set_error(MRHS_EINVAL, "NULL argument");
    const sched::Stats s = srv->impl.stats();
    mrhs_server_stats st{};
    st.p50_ms = s.p50_ms;
    st.p99_ms = s.p99_ms;
    st.rhs_per_s = s.rhs_per_s;
    st.submitted = s.submitted;
    st.completed = s.completed;
    st.queued = s.queued;
    st.rhs_completed = s.rhs_completed;
    st.admitted_bytes = s.admitted_bytes;
    *out = st;
    return MRHS_OK;
}

MRHS_API mrhs_status solve_server_destroy(mrhs_server srv)
{
    clear_error();
    if (!srv)
        return MRHS_OK;
    srv->impl.shutdown();
    delete srv;
    return MRHS_OK;
}
