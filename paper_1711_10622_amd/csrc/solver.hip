// Block BiCGStab drivers: binary64, and binary32 inner solves inside binary64
// iterative refinement.  The iteration itself runs entirely on the device
// (ops.h); the host enqueues chunks of iterations and reads the m column
// states once per chunk.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace mrhs {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t ctl, kry64, kry32, tickets, part, gpart;
    size_t v64[5];           // r, r^, p, v, t                 (binary64 solve)
    size_t r64;              // refinement residual            (mixed)
    size_t z[kGcrMax];       // refinement directions z_j      (mixed)
    size_t w[kGcrMax];       // and w_j = A z_j                (mixed)
    size_t v32[6];           // r, r^, p, v, t, y              (mixed, binary32)
    size_t total;
};

int env_int(const char *name, int dflt, int lo, int hi);

// Stored refinement directions (1..kGcrMax; MRHS_GCR_DIRS overrides the default).
int gcr_dirs() { return env_int("MRHS_GCR_DIRS", kGcrMax, 1, kGcrMax); }

Layout layout(int32_t n, int32_t m, uint32_t flags)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.ctl = take(sizeof(Ctl));
    L.kry64 = take(sizeof(Kry<double>));
    L.kry32 = take(sizeof(Kry<float>));
    L.tickets = take(sizeof(unsigned) * (kGroups + 1));
    const size_t V = static_cast<size_t>(kMaxDots) * kMaxM;
    L.part = take(sizeof(double) * V * static_cast<size_t>(max_grid()));
    L.gpart = take(sizeof(double) * V * kGroups);
    const size_t blk64 = sizeof(double) * static_cast<size_t>(n) * m;
    const size_t blk32 = sizeof(float) * static_cast<size_t>(n) * m;
    if (flags & MRHS_MIXED) {
        L.r64 = take(blk64);
        for (int i = 0; i < gcr_dirs(); ++i) {
            L.z[i] = take(blk64);
            L.w[i] = take(blk64);
        }
        for (int i = 0; i < 6; ++i)
            L.v32[i] = take(blk32);
    } else {
        for (int i = 0; i < 5; ++i)
            L.v64[i] = take(blk64);
    }
    L.total = off;
    return L;
}

__global__ void k_fill_u32(unsigned *p, int count, unsigned value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = value;
}

struct Ctx {
    const mrhs_csr_s *A;
    const double *B;
    double *X;
    int32_t n;
    hipStream_t s;
    Ctl *ctl;
    Kry<double> *kry64;
    Kry<float> *kry32;
    RedBufs<double> rb64;
    RedBufs<float> rb32;
    double *r, *rh, *p, *v, *t;
    double *r64;
    GcrBlocks gcr;
    float *r32, *rh32, *p32, *v32, *t32, *y32;
};

#define MRHS_TRY(expr)                    \
    do {                                  \
        hipError_t e_ = (expr);           \
        if (e_ != hipSuccess)             \
            return e_;                    \
    } while (0)

template <int M>
struct Steps {
    static hipError_t f64_setup(Ctx &c, bool x0)
    {
        MRHS_TRY((launch_stream<double, M>(c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl,
                                                             x0 ? SC_IN : SC_ZERO},
                                            c.rb64, c.s)));
        return launch_gspmv<double, M>(view<double>(*c.A, true),
                                       OpResid<M>{c.X, c.B, c.r, c.rh, c.ctl, c.kry64, RES_SETUP},
                                       c.rb64, c.s);
    }
    static hipError_t f64_iterate(Ctx &c, int k)
    {
        const CsrView<double> Ah = view<double>(*c.A, true);
        for (int it = 0; it < k; ++it) {
            MRHS_TRY((launch_stream<double, M>(c.n, OpPUpdate<double, M>{c.p, c.r, c.v, c.ctl, c.kry64},
                                                c.rb64, c.s)));
            MRHS_TRY((launch_gspmv<double, M>(Ah, OpSpmv1<double, M>{c.p, c.v, c.rh, c.ctl, c.kry64},
                                               c.rb64, c.s)));
            MRHS_TRY((launch_gspmv<double, M>(Ah, OpSpmv2<double, M>{c.r, c.v, c.t, c.ctl, c.kry64},
                                               c.rb64, c.s)));
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpXR<double, M>{c.X, c.r, c.p, c.v, c.t, c.rh, c.ctl, c.kry64}, c.rb64, c.s)));
        }
        return hipSuccess;
    }
    static hipError_t f64_check(Ctx &c)
    {
        MRHS_TRY((launch_gspmv<double, M>(view<double>(*c.A, true),
                                           OpResid<M>{c.X, c.B, c.t, nullptr, c.ctl, c.kry64, RES_CHECK},
                                           c.rb64, c.s)));
        return launch_stream<double, M>(c.n, OpRestart<double, M>{c.t, c.r, c.rh, c.ctl}, c.rb64, c.s);
    }
    static hipError_t finish(Ctx &c, bool mixed, bool nullspace)
    {
        MRHS_TRY((launch_stream<double, M>(c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl,
                                                             mixed ? SC_FIX_ZERO : SC_OUT},
                                            c.rb64, c.s)));
        if (nullspace) {
            MRHS_TRY((launch_stream<double, M>(c.n, OpColSum<M>{c.X, c.ctl}, c.rb64, c.s)));
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_SUB_MEAN}, c.rb64, c.s)));
        }
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, nullptr, nullptr, c.ctl, c.kry64, RES_FINAL},
                                       c.rb64, c.s);
    }
    static hipError_t mixed_setup(Ctx &c, bool x0)
    {
        if (!x0)
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_ZERO}, c.rb64, c.s)));
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, c.r64, nullptr, c.ctl, c.kry64, RES_SETUP},
                                       c.rb64, c.s);
    }
    // one refinement step on slot k for every column whose inner solve ended
    static hipError_t mixed_step(Ctx &c, int k)
    {
        MRHS_TRY((launch_stream<double, M>(c.n, OpGcrZ<M>{c.gcr.z[k], c.y32, c.A->dinv, c.ctl}, c.rb64, c.s)));
        MRHS_TRY((launch_gspmv<double, M>(view<double>(*c.A, false), OpStore<double, M>{c.gcr.z[k], c.gcr.w[k]},
                                           c.rb64, c.s)));
        if (k > 0)
            MRHS_TRY((launch_stream<double, M>(c.n, OpGcrDots<M>{c.gcr, k, c.ctl}, c.rb64, c.s)));
        MRHS_TRY((launch_stream<double, M>(c.n, OpGcrOrth<M>{c.gcr, c.r64, k, c.ctl}, c.rb64, c.s)));
        return launch_stream<double, M>(c.n, OpGcrUpdate<M>{c.X, c.r64, c.gcr.z[k], c.gcr.w[k], c.ctl}, c.rb64,
                                        c.s);
    }
    // true residual of columns whose refinement residual met the tolerance
    static hipError_t mixed_check(Ctx &c)
    {
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, c.r64, nullptr, c.ctl, c.kry64, RES_MIXCHECK},
                                       c.rb64, c.s);
    }
    static hipError_t mixed_cast(Ctx &c)
    {
        return launch_stream<float, M>(c.n, OpCast<M>{c.r64, c.r32, c.rh32, c.y32, c.ctl, c.kry32},
                                       c.rb32, c.s);
    }
    static hipError_t inner_iterate(Ctx &c, int k)
    {
        const CsrView<float> Ah = view<float>(*c.A, true);
        for (int it = 0; it < k; ++it) {
            MRHS_TRY((launch_stream<float, M>(
                c.n, OpPUpdate<float, M>{c.p32, c.r32, c.v32, c.ctl, c.kry32}, c.rb32, c.s)));
            MRHS_TRY((launch_gspmv<float, M>(
                Ah, OpSpmv1<float, M>{c.p32, c.v32, c.rh32, c.ctl, c.kry32}, c.rb32, c.s)));
            MRHS_TRY((launch_gspmv<float, M>(
                Ah, OpSpmv2<float, M>{c.r32, c.v32, c.t32, c.ctl, c.kry32}, c.rb32, c.s)));
            MRHS_TRY((launch_stream<float, M>(
                c.n, OpXR<float, M>{c.y32, c.r32, c.p32, c.v32, c.t32, c.rh32, c.ctl, c.kry32}, c.rb32,
                c.s)));
        }
        return hipSuccess;
    }
};

struct StepTable {
    hipError_t (*f64_setup)(Ctx &, bool);
    hipError_t (*f64_iterate)(Ctx &, int);
    hipError_t (*f64_check)(Ctx &);
    hipError_t (*finish)(Ctx &, bool, bool);
    hipError_t (*mixed_setup)(Ctx &, bool);
    hipError_t (*mixed_step)(Ctx &, int);
    hipError_t (*mixed_check)(Ctx &);
    hipError_t (*mixed_cast)(Ctx &);
    hipError_t (*inner_iterate)(Ctx &, int);
};

struct MakeTable {
    template <int M>
    StepTable operator()() const
    {
        return {&Steps<M>::f64_setup, &Steps<M>::f64_iterate, &Steps<M>::f64_check, &Steps<M>::finish,
                &Steps<M>::mixed_setup, &Steps<M>::mixed_step, &Steps<M>::mixed_check, &Steps<M>::mixed_cast,
                &Steps<M>::inner_iterate};
    }
};

int env_int(const char *name, int dflt, int lo, int hi)
{
    const char *v = std::getenv(name);
    if (!v || !*v)
        return dflt;
    const int x = std::atoi(v);
    return std::min(hi, std::max(lo, x));
}

double env_double(const char *name, double dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v)
        return dflt;
    const double x = std::atof(v);
    return x > 0 ? x : dflt;
}

// Pinned host mirror of the control block, one per host thread.
Ctl *host_ctl()
{
    thread_local Ctl *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
            return nullptr;
        p = static_cast<Ctl *>(q);
    }
    return p;
}

struct StatusCount {
    int run = 0, pending = 0, inner_done = 0, outer = 0;
};

StatusCount count(const Ctl &h, int m)
{
    StatusCount c;
    for (int i = 0; i < m; ++i) {
        const int32_t st = h.status[i];
        c.run += st == COL_RUN;
        c.pending += st == COL_PEND_CHECK || st == COL_PEND_BD;
        c.inner_done += st == COL_INNER_DONE;
        c.outer += st == COL_OUTER;
    }
    return c;
}

mrhs_status col_status(int32_t st)
{
    switch (st) {
    case COL_DONE: return MRHS_OK;
    case COL_BREAKDOWN: return MRHS_EBREAKDOWN;
    default: return MRHS_ENOCONV;
    }
}

} // namespace

size_t solve_workspace_bytes(const mrhs_csr_s &A, int32_t m, uint32_t flags)
{
    return layout(A.n, m, flags).total;
}

mrhs_status block_solve(const mrhs_csr_s &A, const double *B, double *X, const SolveParams &p,
                        void *ws, size_t ws_bytes, hipStream_t s, mrhs_col_info *info)
{
    const int m = p.m;
    const bool mixed = (p.flags & MRHS_MIXED) != 0;
    const bool x0 = (p.flags & MRHS_X0_GIVEN) != 0;
    const bool nullspace = (A.flags & MRHS_CSR_NULLSPACE_CONST) != 0;
    const Layout L = layout(A.n, m, p.flags);
    if (ws_bytes < L.total)
        return set_error(MRHS_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                         L.total);
    static const StepTable tables[kMaxM + 1] = {
        {},
        MakeTable{}.operator()<1>(),  MakeTable{}.operator()<2>(),  MakeTable{}.operator()<3>(),
        MakeTable{}.operator()<4>(),  MakeTable{}.operator()<5>(),  MakeTable{}.operator()<6>(),
        MakeTable{}.operator()<7>(),  MakeTable{}.operator()<8>(),  MakeTable{}.operator()<9>(),
        MakeTable{}.operator()<10>(), MakeTable{}.operator()<11>(), MakeTable{}.operator()<12>(),
        MakeTable{}.operator()<13>(), MakeTable{}.operator()<14>(), MakeTable{}.operator()<15>(),
        MakeTable{}.operator()<16>(),
    };
    const StepTable &T = tables[m];

    char *base = static_cast<char *>(ws);
    Ctx c{};
    c.A = &A;
    c.B = B;
    c.X = X;
    c.n = A.n;
    c.s = s;
    c.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    c.kry64 = reinterpret_cast<Kry<double> *>(base + L.kry64);
    c.kry32 = reinterpret_cast<Kry<float> *>(base + L.kry32);
    unsigned *tickets = reinterpret_cast<unsigned *>(base + L.tickets);
    c.rb64 = {reinterpret_cast<double *>(base + L.part), reinterpret_cast<double *>(base + L.gpart), tickets};
    c.rb32 = {reinterpret_cast<float *>(base + L.part), reinterpret_cast<float *>(base + L.gpart), tickets};
    if (mixed) {
        c.r64 = reinterpret_cast<double *>(base + L.r64);
        for (int i = 0; i < gcr_dirs(); ++i) {
            c.gcr.z[i] = reinterpret_cast<double *>(base + L.z[i]);
            c.gcr.w[i] = reinterpret_cast<double *>(base + L.w[i]);
        }
        float **v32[6] = {&c.r32, &c.rh32, &c.p32, &c.v32, &c.t32, &c.y32};
        for (int i = 0; i < 6; ++i)
            *v32[i] = reinterpret_cast<float *>(base + L.v32[i]);
    } else {
        double **v64[5] = {&c.r, &c.rh, &c.p, &c.v, &c.t};
        for (int i = 0; i < 5; ++i)
            *v64[i] = reinterpret_cast<double *>(base + L.v64[i]);
    }

    Ctl *h = host_ctl();
    if (!h)
        return set_error(MRHS_ENOMEM, "pinned host buffer allocation failed");
    std::memset(h, 0, sizeof(Ctl));
    for (int i = 0; i < m; ++i) {
        h->status[i] = COL_RUN;
        h->tol[i] = p.tol;
        h->maxit[i] = p.maxit;
        h->inner_maxit[i] = p.maxit;
    }
    h->mode = mixed ? MODE_INNER : MODE_F64;
    h->tol_in = env_double("MRHS_INNER_TOL", 0.1);
    h->max_outer = env_int("MRHS_MAX_OUTER", 500, 1, 100000);
    h->n = A.n;
    const int chunk = env_int("MRHS_POLL_ITERS", 16, 1, 1024);

    MRHS_HIP(hipMemcpyAsync(c.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, tickets, kGroups + 1, 0u);
    MRHS_HIP(hipGetLastError());

    auto read_status = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(h->status, c.ctl->status, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess)
            return e;
        return hipStreamSynchronize(s);
    };

    if (!mixed) {
        MRHS_HIP(T.f64_setup(c, x0));
        MRHS_HIP(read_status());
        for (;;) {
            const StatusCount sc = count(*h, m);
            if (sc.pending) {
                MRHS_HIP(T.f64_check(c));
                MRHS_HIP(read_status());
                continue;
            }
            if (!sc.run)
                break;
            MRHS_HIP(T.f64_iterate(c, chunk));
            MRHS_HIP(read_status());
        }
    } else {
        // binary32 inner solves, binary64 refinement steps (all columns in
        // step: every inner phase runs until no column is iterating)
        const int ndirs = gcr_dirs();
        int slot = 0;
        MRHS_HIP(T.mixed_setup(c, x0));
        for (;;) {
            MRHS_HIP(read_status());
            const StatusCount sc = count(*h, m);
            if (sc.pending) {
                MRHS_HIP(T.mixed_check(c));
                continue;
            }
            if (!sc.outer)
                break;
            MRHS_HIP(T.mixed_cast(c));
            for (;;) {
                MRHS_HIP(read_status());
                if (!count(*h, m).run)
                    break;
                MRHS_HIP(T.inner_iterate(c, chunk));
            }
            MRHS_HIP(T.mixed_step(c, slot));
            slot = (slot + 1) % ndirs;
        }
    }
    MRHS_HIP(T.finish(c, mixed, nullspace));
    MRHS_HIP(hipMemcpyAsync(h, c.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    MRHS_HIP(hipStreamSynchronize(s));

    mrhs_status worst = MRHS_OK;
    for (int i = 0; i < m; ++i) {
        const mrhs_status cs = col_status(h->status[i]);
        if (info) {
            info[i].iters = mixed ? h->total_iters[i] : h->iters[i];
            info[i].restarts = h->restarts[i];
            info[i].outer = mixed ? h->outer[i] : 0;
            info[i].status = cs;
            info[i].relres = h->relres[i];
        }
        if (cs < worst)
            worst = cs;
    }
    if (worst != MRHS_OK)
        set_error(worst, "not every column converged");
    return worst;
}

} // namespace mrhs
