// Block BiCGStab engine: m column slots sharing one matrix, driven from the
// host in rounds.  Each round reads the column states once and enqueues what
// the columns need next (true-residual checks, refinement steps, a chunk of
// iterations); every decision inside an iteration is taken on the device
// (ops.h).  A one-shot block solve and the solve server both run on it.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace mrhs {

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

int gcr_dirs() { return env_int("MRHS_GCR_DIRS", kGcrMax, 1, kGcrMax); }

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t ctl, kry64, kry32, tickets, part, gpart;
    size_t rv64, p64, t64;  // r and v (one region, see pair_rv), p, t (binary64 solve)
    size_t rv64b, p64b;     // the second r/v region and p of the merged iteration
    size_t sv64, ph64, sh64, vc;  // s, M^-1 p, M^-1 s, V-cycle buffers (AMG preconditioner)
    size_t r64;         // refinement residual             (mixed)
    size_t z[kGcrMax];  // stored directions z_j           (mixed)
    size_t w[kGcrMax];  // and w_j = A z_j                 (mixed)
    size_t znew, wnew;  // the direction being formed      (mixed)
    size_t xacc;        // accumulated correction of x      (mixed)
    // (the mixed-precision binary64 buffers are column-major, one n-vector per column)
    size_t rv32, v32[3];    // r and v (one region), then p, t, y  (mixed, binary32)
    size_t sgn32;       // sign bits of the inner shadow residual (mixed)
    size_t total;
};

// Plain (not interleaved) r and v blocks lie kPairGap bytes further apart
// than their size, for the reason the workspace blocks are staggered (see
// layout).
constexpr size_t kPairGap = 8192;

// r and v share one region of 2 n m elements (+ kPairGap bytes): interleaved
// row by row (v = r + m, row stride 2m) when the matrix has no regular plane
// structure (its gathers visit rows in no particular order, and one line then
// serves both rows of an entry: relabelled cube, m = 8, spmv_omega 601 -> 357
// us binary64 and 553 -> 301 us binary32); else as two plain blocks
// (interleaved, half-line rows made the channel's binary32 passes 4 % slower,
// and whole-line rows its binary64 m = 16 solve 1.2 % slower: spmv_sigma
// 1040 -> 1012 us, spmv_omega 1799 -> 1780 us as plain blocks).
bool pair_rv(const mrhs_csr_s &A)
{
    const int64_t ntiles = (static_cast<int64_t>(A.n) + kTileRows - 1) / kTileRows;
    const int64_t P = (static_cast<int64_t>(A.reach) + kTileRows / 2) / kTileRows;
    const bool planes = P >= 2 * kGroups && ntiles >= 4 * P;
    return !planes;
}

// The binary64 Jacobi iteration runs as two kernels (OpXRSigma, then
// spmv_omega) where that was measured faster: narrow blocks on small and
// mid-size matrices, whose iterations are bound by the kernels' latency
// chains rather than bytes.  Per iteration (ms, three kernels -> two):
// 524k-row channel m = 1 0.083 -> 0.061, m = 4 0.096 -> 0.086, m = 8 0.129 ->
// 0.139; 64^3 Dirichlet m = 4 0.069 -> 0.054, m = 8 0.084 -> 0.080, m = 16
// 0.122 -> 0.140; 12.6M-row channel slower at every m (its gathers of four
// blocks per entry and occupancy 2 cost more than a kernel boundary).
// MRHS_MERGE: 0 never, 1 (default) where faster, 2 always.
bool merged_iteration(int32_t n, int32_t m, uint32_t flags, const AmgDev *amg)
{
    if ((flags & MRHS_MIXED) || amg)
        return false;
    const int mode = env_int("MRHS_MERGE", 1, 0, 2);
    if (mode != 1)
        return mode == 2;
    return (m <= 4 && n <= 600000) || (m <= 8 && n <= 300000);
}

Layout layout(int32_t n, int32_t m, uint32_t flags, const AmgDev *amg = nullptr)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    // block arrays start k * 4 KiB past their predecessor's end (k = 1, 2,
    // ...): with n x m sizes that are multiples of large powers of two the
    // streams of one pass would otherwise sit at the same offset modulo the
    // memory interleave (measured: 128x64x64 channel, m = 16, xr_update 95 ->
    // 92 us on average, binary64 solve -2 %)
    int nblk = 0;
    auto take_blk = [&](size_t bytes) {
        const size_t o = take(bytes);
        off += static_cast<size_t>(4096) * ++nblk;
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
        L.r64 = take_blk(blk64);
        for (int i = 0; i < gcr_dirs(); ++i) {
            L.z[i] = take_blk(blk64);
            L.w[i] = take_blk(blk64);
        }
        L.znew = take_blk(blk64);
        L.wnew = take_blk(blk64);
        L.xacc = take_blk(blk64);
        L.rv32 = take_blk(2 * blk32 + kPairGap);
        for (int i = 0; i < 3; ++i)
            L.v32[i] = take_blk(blk32);
        L.sgn32 = take(static_cast<size_t>(n) * kMaxM);  // n x (lanes per row <= 16) bytes
    } else {
        L.rv64 = take_blk(2 * blk64 + kPairGap);
        L.p64 = take_blk(blk64);
        L.t64 = take_blk(blk64);
        if (merged_iteration(n, m, flags, amg)) {
            L.rv64b = take_blk(2 * blk64 + kPairGap);
            L.p64b = take_blk(blk64);
        }
        if (amg) {
            L.sv64 = take_blk(blk64);
            L.ph64 = take_blk(blk64);
            L.sh64 = take_blk(blk64);
            L.vc = take(amg_vcycle_bytes(*amg, m));
        }
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

// Admission of columns into a block: reset their control state.
__global__ void k_slot_init(Ctl *ctl, uint32_t cmask, SlotInit si)
{
    const int c = threadIdx.x;
    if (c >= kMaxM || !((cmask >> c) & 1u))
        return;
    Ctl &k = *ctl;
    k.status[c] = COL_INIT;
    k.fresh[c] = 1;
    k.flag[c] = 0;
    k.iters[c] = 0;
    k.maxit[c] = si.maxit[c];
    k.restarts[c] = 0;
    k.breakdowns[c] = 0;
    k.bd_run[c] = 0;
    k.outer[c] = 0;
    k.total_iters[c] = 0;
    k.stag_it[c] = 0;
    k.inner_maxit[c] = si.maxit[c];
    k.nb[c] = 0.0;
    k.tol[c] = si.tol[c];
    k.rn[c] = 0.0;
    k.stag_rn[c] = 1.0;
    k.relres[c] = 0.0;
    k.rscale[c] = 0.0;
    k.colsum[c] = 0.0;
    k.kcol[c] = 0;
    k.wnew2[c] = 0.0;
    k.gamma[c] = 0.0;
    for (int j = 0; j < kGcrMax; ++j) {
        k.beta[j][c] = 0.0;
        k.wnorm2[j][c] = 0.0;
    }
}

__global__ void k_ctl_reset(Ctl *ctl, int32_t mode, double tol_in, int32_t max_outer, int32_t n,
                            int32_t stag_window)
{
    if (threadIdx.x == 0) {
        Ctl &k = *ctl;
        for (int c = 0; c < kMaxM; ++c)
            k.status[c] = COL_IDLE;
        k.mode = mode;
        k.tol_in = tol_in;
        k.max_outer = max_outer;
        k.n = n;
        k.stag_window = stag_window;
    }
}

#define MRHS_TRY(expr)          \
    do {                        \
        hipError_t e_ = (expr); \
        if (e_ != hipSuccess)   \
            return e_;          \
    } while (0)

// launches OpColsStore<K> for the K columns listed in cols
struct ColsProduct {
    CsrView<double> A;
    Ctx &c;
    int cols[kMaxM];
    int k;
    template <int K>
    hipError_t operator()() const
    {
        OpColsStore<K> op{};
        const size_t n = static_cast<size_t>(c.n);
        for (int q = 0; q < K; ++q) {
            op.z[q] = c.gcr.znew + static_cast<size_t>(cols[q]) * n;
            op.w[q] = c.gcr.wnew + static_cast<size_t>(cols[q]) * n;
        }
        return launch_gspmv<double, K>(A, op, c.rb64, c.s);
    }
};

template <int M>
struct Steps {
    static hipError_t f64_start(Ctx &c, uint32_t cmask, bool x0)
    {
        MRHS_TRY((launch_stream<double, M>(
            c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, x0 ? SC_IN : SC_ZERO, cmask}, c.rb64, c.s)));
        return launch_gspmv<double, M>(view<double>(*c.A, true),
                                       OpResid<M>{c.X, c.B, c.r, c.p, nullptr, c.ctl, c.kry64, RES_SETUP, 0u, 0, c.ldp64},
                                       c.rb64, c.s);
    }
    static hipError_t f64_iterate(Ctx &c, int k)
    {
        const CsrView<double> Ah = view<double>(*c.A, true);
        if (c.merged) {  // v = Ah p, then (t = Ah s, merged update and next v) k - 1 times, t = Ah s, update
            MRHS_TRY((launch_gspmv<double, M>(Ah, OpSpmv1<double, M>{c.p, c.v, nullptr, c.ctl, c.kry64, c.ldp64},
                                               c.rb64, c.s)));
            for (int it = 0; it < k; ++it) {
                MRHS_TRY((launch_gspmv<double, M>(
                    Ah, OpSpmv2<double, M>{c.r, c.v, nullptr, c.t, c.ctl, c.kry64, c.ldp64}, c.rb64, c.s)));
                if (it + 1 < k) {
                    OpXRSigma<double, M> op{};
                    op.y = c.X;
                    op.r = c.r;
                    op.v = c.v;
                    op.t = c.t;
                    op.p = c.p;
                    op.r2 = c.r2;
                    op.v2 = c.v2;
                    op.p2 = c.p2;
                    op.ctl = c.ctl;
                    op.kry = c.kry64;
                    op.ldp = c.ldp64;
                    MRHS_TRY((launch_gspmv<double, M>(Ah, op, c.rb64, c.s)));
                    std::swap(c.r, c.r2);
                    std::swap(c.v, c.v2);
                    std::swap(c.p, c.p2);
                } else {
                    MRHS_TRY((launch_stream<double, M>(
                        c.n, OpXR<double, M>{c.X, c.r, c.p, c.v, c.t, nullptr, c.ctl, c.kry64, c.ldp64}, c.rb64,
                        c.s)));
                }
            }
            return hipSuccess;
        }
        for (int it = 0; it < k; ++it) {
            MRHS_TRY((launch_gspmv<double, M>(Ah, OpSpmv1<double, M>{c.p, c.v, nullptr, c.ctl, c.kry64, c.ldp64},
                                               c.rb64, c.s)));
            MRHS_TRY((launch_gspmv<double, M>(Ah, OpSpmv2<double, M>{c.r, c.v, nullptr, c.t, c.ctl, c.kry64, c.ldp64},
                                               c.rb64, c.s)));
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpXR<double, M>{c.X, c.r, c.p, c.v, c.t, nullptr, c.ctl, c.kry64, c.ldp64}, c.rb64, c.s)));
        }
        return hipSuccess;
    }
    static hipError_t f64_check(Ctx &c)
    {
        MRHS_TRY((launch_gspmv<double, M>(view<double>(*c.A, true),
                                           OpResid<M>{c.X, c.B, c.t, nullptr, nullptr, c.ctl, c.kry64, RES_CHECK, 0u},
                                           c.rb64, c.s)));
        return launch_stream<double, M>(c.n, OpRestart<double, M>{c.t, c.r, c.p, c.ctl, c.ldp64}, c.rb64, c.s);
    }
    static hipError_t finish(Ctx &c, uint32_t cmask, bool mixed, bool nullspace)
    {
        if (mixed)  // the accumulated corrections into X
            MRHS_TRY((launch_stream<double, M>(c.n, OpFold<M>{c.X, c.gcr.xacc, c.n, FOLD_ADD, cmask}, c.rb64, c.s)));
        MRHS_TRY((launch_stream<double, M>(
            c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, mixed ? SC_FIX_ZERO : SC_OUT, cmask}, c.rb64, c.s)));
        if (nullspace) {
            MRHS_TRY((launch_stream<double, M>(c.n, OpColSum<M>{c.X, c.ctl, cmask}, c.rb64, c.s)));
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_SUB_MEAN, cmask}, c.rb64, c.s)));
        }
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, nullptr, nullptr, nullptr, c.ctl, c.kry64, RES_FINAL, cmask},
                                       c.rb64, c.s);
    }
    static hipError_t mixed_start(Ctx &c, uint32_t cmask, bool x0)
    {
        if (!x0)
            MRHS_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_ZERO, cmask}, c.rb64, c.s)));
        MRHS_TRY((launch_stream<double, M>(c.n, OpFold<M>{c.X, c.gcr.xacc, c.n, FOLD_ZERO, cmask}, c.rb64, c.s)));
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, c.r64, nullptr, nullptr, c.ctl, c.kry64, RES_SETUP, 0u, c.n},
                                       c.rb64, c.s);
    }
    // one refinement step for each column of cmask (their inner solves ended);
    // jmax[c]: directions the column has stored, slot[c]: the slot its new
    // direction goes to (the device's kcol[c], which every step advances)
    static hipError_t mixed_step(Ctx &c, uint32_t cmask, const int32_t *jmax, const int32_t *slot)
    {
        MRHS_TRY((launch_stream<float, M>(c.n, OpGcrZ<M>{c.gcr.znew, c.y32, c.A->dinv, c.ctl, c.n}, c.rb32, c.s)));
        const CsrView<double> A = view<double>(*c.A, false);
        const size_t n = static_cast<size_t>(c.n);
        {  // w = A z for every column of the round in one product
            ColsProduct cp{A, c, {}, 0};
            for (int col = 0; col < M; ++col)
                if ((cmask >> col) & 1u)
                    cp.cols[cp.k++] = col;
            if (cp.k > 0)
                MRHS_TRY(dispatch_m(cp.k, cp));
        }
        for (int col = 0; col < M; ++col) {
            if (!((cmask >> col) & 1u))
                continue;
            const size_t off = static_cast<size_t>(col) * n;
            double *z = c.gcr.znew + off, *w = c.gcr.wnew + off, *r = c.r64 + off;
            OpColDots dots{};
            OpColOrth orth{};
            for (int j = 0; j < kGcrMax; ++j) {
                const bool have = j < c.gcr.ndirs;
                dots.W[j] = orth.W[j] = have ? c.gcr.w[j] + off : nullptr;
                orth.Z[j] = have ? c.gcr.z[j] + off : nullptr;
            }
            dots.w = w;
            dots.jmax = orth.jmax = jmax[col];
            dots.col = orth.col = col;
            dots.ctl = orth.ctl = c.ctl;
            orth.w = w;
            orth.z = z;
            orth.r = r;
            if (jmax[col] > 0)
                MRHS_TRY((launch_stream<double, 1>(c.n, dots, c.rb64, c.s)));
            MRHS_TRY((launch_stream<double, 1>(c.n, orth, c.rb64, c.s)));
            const OpColUpdate upd{c.gcr.xacc + off, r, z, w, c.gcr.z[slot[col]] + off, c.gcr.w[slot[col]] + off,
                                  c.gcr.ndirs, col, c.ctl};
            MRHS_TRY((launch_stream<double, 1>(c.n, upd, c.rb64, c.s)));
        }
        return hipSuccess;
    }
    // true residual of columns whose refinement residual met the tolerance
    // (their accumulated corrections are folded into X first)
    static hipError_t mixed_check(Ctx &c, uint32_t pend)
    {
        MRHS_TRY((launch_stream<double, M>(c.n, OpFold<M>{c.X, c.gcr.xacc, c.n, FOLD_ADD, pend}, c.rb64, c.s)));
        return launch_gspmv<double, M>(view<double>(*c.A, false),
                                       OpResid<M>{c.X, c.B, c.r64, nullptr, nullptr, c.ctl, c.kry64, RES_MIXCHECK, 0u, c.n},
                                       c.rb64, c.s);
    }
    static hipError_t mixed_cast(Ctx &c)
    {
        return launch_stream<float, M>(c.n, OpCast<M>{c.r64, c.r32, c.sgn32, c.y32, c.p32, c.ctl, c.kry32, c.n, c.ldp32}, c.rb32,
                                       c.s);
    }
    static hipError_t inner_iterate(Ctx &c, int k)
    {
        const CsrView<float> Ah = view<float>(*c.A, true);
        for (int it = 0; it < k; ++it) {
            MRHS_TRY((launch_gspmv<float, M>(
                Ah, OpSpmv1<float, M>{c.p32, c.v32, c.sgn32, c.ctl, c.kry32, c.ldp32}, c.rb32, c.s)));
            MRHS_TRY((launch_gspmv<float, M>(
                Ah, OpSpmv2<float, M>{c.r32, c.v32, c.sgn32, c.t32, c.ctl, c.kry32, c.ldp32}, c.rb32, c.s)));
            MRHS_TRY((launch_stream<float, M>(
                c.n, OpXR<float, M>{c.y32, c.r32, c.p32, c.v32, c.t32, c.sgn32, c.ctl, c.kry32, c.ldp32}, c.rb32,
                c.s)));
        }
        return hipSuccess;
    }
};

struct MakeTable {
    template <int M>
    StepTable operator()() const
    {
        return {&Steps<M>::f64_start,   &Steps<M>::f64_iterate, &Steps<M>::f64_check,
                &Steps<M>::finish,      &Steps<M>::mixed_start, &Steps<M>::mixed_step,
                &Steps<M>::mixed_check, &Steps<M>::mixed_cast,  &Steps<M>::inner_iterate};
    }
};

const StepTable &table(int m)
{
    static const StepTable tables[kMaxM + 1] = {
        {},
        MakeTable{}.operator()<1>(),  MakeTable{}.operator()<2>(),  MakeTable{}.operator()<3>(),
        MakeTable{}.operator()<4>(),  MakeTable{}.operator()<5>(),  MakeTable{}.operator()<6>(),
        MakeTable{}.operator()<7>(),  MakeTable{}.operator()<8>(),  MakeTable{}.operator()<9>(),
        MakeTable{}.operator()<10>(), MakeTable{}.operator()<11>(), MakeTable{}.operator()<12>(),
        MakeTable{}.operator()<13>(), MakeTable{}.operator()<14>(), MakeTable{}.operator()<15>(),
        MakeTable{}.operator()<16>(),
    };
    return tables[m];
}

} // namespace

mrhs_status column_status(int32_t st)
{
    switch (st) {
    case COL_DONE: return MRHS_OK;
    case COL_BREAKDOWN: return MRHS_EBREAKDOWN;
    default: return MRHS_ENOCONV;
    }
}

size_t Engine::workspace_bytes(const mrhs_csr_s &A, int32_t m, uint32_t flags, const AmgDev *amg)
{
    return layout(A.n, m, flags, amg).total;
}

Engine::Engine(const mrhs_csr_s &A, int m, uint32_t flags, void *ws, const double *B, double *X, hipStream_t s,
               Ctl *host_ctl, const AmgDev *amg)
    : A_(A), m_(m), mixed_((flags & MRHS_MIXED) != 0), nullspace_((A.flags & MRHS_CSR_NULLSPACE_CONST) != 0),
      s_(s), T_(&table(m)), host_(host_ctl)
{
    const Layout L = layout(A.n, m, flags, amg);
    char *base = static_cast<char *>(ws);
    c_.A = &A;
    c_.B = B;
    c_.X = X;
    c_.n = A.n;
    c_.s = s;
    c_.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    c_.kry64 = reinterpret_cast<Kry<double> *>(base + L.kry64);
    c_.kry32 = reinterpret_cast<Kry<float> *>(base + L.kry32);
    tickets_ = reinterpret_cast<unsigned *>(base + L.tickets);
    c_.rb64 = {reinterpret_cast<double *>(base + L.part), reinterpret_cast<double *>(base + L.gpart), tickets_};
    c_.rb32 = {reinterpret_cast<float *>(base + L.part), reinterpret_cast<float *>(base + L.gpart), tickets_};
    ndirs_ = gcr_dirs();
    if (mixed_) {
        c_.r64 = reinterpret_cast<double *>(base + L.r64);
        for (int i = 0; i < ndirs_; ++i) {
            c_.gcr.z[i] = reinterpret_cast<double *>(base + L.z[i]);
            c_.gcr.w[i] = reinterpret_cast<double *>(base + L.w[i]);
        }
        c_.gcr.znew = reinterpret_cast<double *>(base + L.znew);
        c_.gcr.wnew = reinterpret_cast<double *>(base + L.wnew);
        c_.gcr.xacc = reinterpret_cast<double *>(base + L.xacc);
        c_.gcr.ndirs = ndirs_;
        const bool pair = pair_rv(A);
        c_.r32 = reinterpret_cast<float *>(base + L.rv32);
        c_.v32 = pair ? c_.r32 + m_ : c_.r32 + static_cast<size_t>(A.n) * m_ + kPairGap / sizeof(float);
        c_.ldp32 = pair ? 2 * m_ : m_;
        float **v32[3] = {&c_.p32, &c_.t32, &c_.y32};
        for (int i = 0; i < 3; ++i)
            *v32[i] = reinterpret_cast<float *>(base + L.v32[i]);
        c_.sgn32 = reinterpret_cast<uint8_t *>(base + L.sgn32);
    } else {
        const bool pair = pair_rv(A);
        c_.r = reinterpret_cast<double *>(base + L.rv64);
        c_.v = pair ? c_.r + m_ : c_.r + static_cast<size_t>(A.n) * m_ + kPairGap / sizeof(double);
        c_.ldp64 = pair ? 2 * m_ : m_;
        c_.p = reinterpret_cast<double *>(base + L.p64);
        c_.t = reinterpret_cast<double *>(base + L.t64);
        if (merged_iteration(A.n, m, flags, amg)) {
            c_.merged = true;
            c_.r2 = reinterpret_cast<double *>(base + L.rv64b);
            c_.v2 = pair ? c_.r2 + m_ : c_.r2 + static_cast<size_t>(A.n) * m_ + kPairGap / sizeof(double);
            c_.p2 = reinterpret_cast<double *>(base + L.p64b);
        }
        if (amg) {
            AT_ = &amg_table(m);
            c_.amg = amg;
            c_.sv = reinterpret_cast<double *>(base + L.sv64);
            c_.ph = reinterpret_cast<double *>(base + L.ph64);
            c_.sh = reinterpret_cast<double *>(base + L.sh64);
            c_.vcws = base + L.vc;
            c_.vc32 = (flags & kAmgVc32) != 0;
        }
    }
    chunk_ = env_int("MRHS_POLL_ITERS", 16, 1, 1024);
    tol_in_ = env_double("MRHS_INNER_TOL", 0.2);
    max_outer_ = env_int("MRHS_MAX_OUTER", 500, 1, 100000);
    outer_batch_ = env_double("MRHS_OUTER_BATCH", 1.0);
    outer_wait_ = env_int("MRHS_OUTER_WAIT", 0, 0, 100000);
    mixed_chunk_ = env_int("MRHS_MIXED_POLL", 8, 1, 1024);
    stag_window_ = env_int("MRHS_STAG_WINDOW", kStagWindow, 4, 100000);
    amg_chunk_ = env_int("MRHS_AMG_POLL", 2, 1, 1024);
}

Engine::~Engine()
{
    if (host_ && own_host_)
        (void)hipHostFree(host_);
}

mrhs_status Engine::reset()
{
    if (!host_) {
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
            return set_error(MRHS_ENOMEM, "pinned host buffer allocation failed");
        host_ = static_cast<Ctl *>(q);
        own_host_ = true;
    }
    std::memset(host_, 0, sizeof(Ctl));
    for (int c = 0; c < kMaxM; ++c)
        col_steps_[c] = 0;
    waited_ = 0;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s_, tickets_, kGroups + 1, 0u);
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s_, c_.ctl, mixed_ ? MODE_INNER : MODE_F64, tol_in_,
                       max_outer_, A_.n, stag_window_);
    MRHS_HIP(hipGetLastError());
    return MRHS_OK;
}

mrhs_status Engine::start(uint32_t cmask, const double *tol, const int32_t *maxit, bool x0)
{
    SlotInit si{};
    for (int c = 0; c < kMaxM; ++c) {
        si.tol[c] = c < m_ ? tol[c] : 1.0;
        si.maxit[c] = c < m_ ? maxit[c] : 1;
    }
    cmask &= (1u << m_) - 1u;
    for (int c = 0; c < m_; ++c)
        if ((cmask >> c) & 1u)
            col_steps_[c] = 0;  // the device resets kcol[c] to slot 0
    hipLaunchKernelGGL(k_slot_init, dim3(1), dim3(64), 0, s_, c_.ctl, cmask, si);
    MRHS_HIP(hipGetLastError());
    MRHS_HIP(mixed_ ? T_->mixed_start(c_, cmask, x0)
                    : (AT_ ? AT_->start(c_, cmask, x0) : T_->f64_start(c_, cmask, x0)));
    return MRHS_OK;
}

mrhs_status Engine::read_status()
{
    MRHS_HIP(hipMemcpyAsync(host_->status, c_.ctl->status, sizeof(int32_t) * m_, hipMemcpyDeviceToHost, s_));
    MRHS_HIP(hipStreamSynchronize(s_));
    return MRHS_OK;
}

mrhs_status Engine::read_ctl()
{
    MRHS_HIP(hipMemcpyAsync(host_, c_.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s_));
    MRHS_HIP(hipStreamSynchronize(s_));
    return MRHS_OK;
}

bool Engine::terminal(int32_t st) { return st == COL_DONE || st == COL_NOCONV || st == COL_BREAKDOWN; }

uint32_t Engine::terminal_mask() const
{
    uint32_t mk = 0;
    for (int c = 0; c < m_; ++c)
        if (terminal(host_->status[c]))
            mk |= 1u << c;
    return mk;
}

mrhs_status Engine::advance(bool *busy)
{
    mrhs_status st = read_status();
    if (st != MRHS_OK)
        return st;
    int run = 0, pend = 0, done_in = 0, outer = 0;
    for (int c = 0; c < m_; ++c) {
        const int32_t s = host_->status[c];
        run += s == COL_RUN;
        pend += s == COL_PEND_CHECK || s == COL_PEND_BD;
        done_in += s == COL_INNER_DONE;
        outer += s == COL_OUTER;
    }
    *busy = run || pend || done_in || outer;
    if (!*busy)
        return MRHS_OK;
    if (!mixed_) {
        if (pend)
            MRHS_HIP(AT_ ? AT_->check(c_) : T_->f64_check(c_));
        MRHS_HIP(AT_ ? AT_->iterate(c_, amg_chunk_) : T_->f64_iterate(c_, chunk_));
        return MRHS_OK;
    }
    uint32_t pend_mask = 0, done_mask = 0;
    for (int c = 0; c < m_; ++c) {
        const int32_t s = host_->status[c];
        if (s == COL_PEND_CHECK || s == COL_PEND_BD)
            pend_mask |= 1u << c;
        if (s == COL_INNER_DONE)
            done_mask |= 1u << c;
    }
    if (pend)
        MRHS_HIP(T_->mixed_check(c_, pend_mask));
    // Refinement steps are per column (column-major vectors), but the z
    // formation and the cast back to binary32 pass over the row-interleaved
    // blocks once per round; columns whose inner solve ended may wait for a
    // share outer_batch_ of the active columns, nothing else running, or
    // outer_wait_ iterations.  A column's arithmetic does not depend on when
    // its step comes.
    if (done_in) {
        if (run == 0 || done_in >= outer_batch_ * (run + done_in) || waited_ >= outer_wait_) {
            int32_t jmax[kMaxM], slot[kMaxM];
            for (int c = 0; c < kMaxM; ++c) {
                jmax[c] = std::min(col_steps_[c], ndirs_);
                slot[c] = col_steps_[c] % ndirs_;
            }
            MRHS_HIP(T_->mixed_step(c_, done_mask, jmax, slot));
            for (int c = 0; c < m_; ++c)
                if ((done_mask >> c) & 1u)
                    ++col_steps_[c];
            waited_ = 0;
        } else {
            waited_ += mixed_chunk_;
        }
    }
    MRHS_HIP(T_->mixed_cast(c_));
    MRHS_HIP(T_->inner_iterate(c_, mixed_chunk_));
    return MRHS_OK;
}

mrhs_status Engine::finish(uint32_t cmask)
{
    MRHS_HIP(AT_ ? AT_->finish(c_, cmask, nullspace_) : T_->finish(c_, cmask, mixed_, nullspace_));
    return MRHS_OK;
}

namespace {

// Block width the solver runs at for m right-hand sides.  In binary64 an odd
// m >= 3 runs at m + 1, so every lane moves 16-byte vectors of two columns
// instead of single elements (12.6M-row channel, time per iteration: m = 7
// 3.20 -> 2.83 ms, m = 15 6.42 -> 5.46 ms, m = 9 unchanged); mixed precision
// widens only when m + 1 is a multiple of 4 (binary32 lanes of four columns;
// its m = 10 products are slower than m = 9).  The extra column has a zero
// right-hand side and is finished at admission.  MRHS_PAD_ODD=0 keeps m.
int solve_width(int m, uint32_t flags)
{
    const int pad = env_int("MRHS_PAD_ODD", 1, 0, 1);
    if (!pad || m % 2 == 0 || m < 3 || m >= kMaxM)
        return m;
    if ((flags & MRHS_MIXED) && (m + 1) % 4 != 0)
        return m;
    return m + 1;
}

} // namespace

// Between the caller's blocks (n x m, caller's row numbering) and the
// solver's (n x w, w >= m, row i = the caller's row perm[i], or row i without
// a permutation).  to_solver: sv[i][c] = us[perm[i]][c] for c < m, 0 for
// m <= c < w.  to_user: us[perm[i]][c] = sv[i][c] for c < m.
__global__ void k_to_solver(double *__restrict__ sv, const double *__restrict__ us, const int32_t *__restrict__ perm,
                            int32_t n, int w, int m)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= static_cast<int64_t>(n) * w)
        return;
    const int64_t i = k / w;
    const int c = static_cast<int>(k - i * w);
    const int64_t u = perm ? perm[i] : i;
    sv[k] = c < m ? us[u * m + c] : 0.0;
}

__global__ void k_to_user(double *__restrict__ us, const double *__restrict__ sv, const int32_t *__restrict__ perm,
                          int32_t n, int w, int m)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= static_cast<int64_t>(n) * m)
        return;
    const int64_t i = k / m;
    const int c = static_cast<int>(k - i * m);
    const int64_t u = perm ? perm[i] : i;
    us[u * m + c] = sv[i * w + c];
}

hipError_t to_solver(double *sv, const double *us, const int32_t *perm, int32_t n, int w, int m, hipStream_t s)
{
    const int64_t count = static_cast<int64_t>(n) * w;
    hipLaunchKernelGGL(k_to_solver, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, sv, us, perm,
                       n, w, m);
    return hipGetLastError();
}

hipError_t to_user(double *us, const double *sv, const int32_t *perm, int32_t n, int w, int m, hipStream_t s)
{
    const int64_t count = static_cast<int64_t>(n) * m;
    hipLaunchKernelGGL(k_to_user, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, us, sv, perm, n,
                       w, m);
    return hipGetLastError();
}

size_t padded_block_bytes(int32_t n, int w) { return align_up(sizeof(double) * static_cast<size_t>(n) * w); }

size_t solve_workspace_bytes(const mrhs_csr_s &A, int32_t m, uint32_t flags, const AmgDev *amg)
{
    const int w = solve_width(m, flags);
    const size_t eng = align_up(Engine::workspace_bytes(A, w, flags, amg));
    return (w == m && !A.perm) ? eng : eng + 2 * padded_block_bytes(A.n, w);
}

mrhs_status block_solve(const mrhs_csr_s &A, const double *B, double *X, const SolveParams &p, void *ws,
                        size_t ws_bytes, hipStream_t s, mrhs_col_info *info, Ctl *host_ctl, const AmgDev *amg)
{
    const size_t need = solve_workspace_bytes(A, p.m, p.flags, amg);
    if (ws_bytes < need)
        return set_error(MRHS_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    const int m = solve_width(p.m, p.flags);
    const bool copy = m != p.m || A.perm;
    double *Xw = X;
    const double *Bw = B;
    if (copy) {  // widened and/or renumbered copies of B and X after the engine's workspace
        char *tail = static_cast<char *>(ws) + align_up(Engine::workspace_bytes(A, m, p.flags, amg));
        double *Bp = reinterpret_cast<double *>(tail);
        Xw = reinterpret_cast<double *>(tail + padded_block_bytes(A.n, m));
        MRHS_HIP(to_solver(Bp, B, A.perm, A.n, m, p.m, s));
        if (p.flags & MRHS_X0_GIVEN)
            MRHS_HIP(to_solver(Xw, X, A.perm, A.n, m, p.m, s));
        Bw = Bp;
    }
    Engine e(A, m, p.flags, ws, Bw, Xw, s, host_ctl, amg);
    mrhs_status st = e.reset();
    if (st != MRHS_OK)
        return st;
    double tol[kMaxM];
    int32_t maxit[kMaxM];
    for (int c = 0; c < kMaxM; ++c) {
        tol[c] = p.tol;
        maxit[c] = p.maxit;
    }
    const uint32_t all = (1u << m) - 1u;
    if ((st = e.start(all, tol, maxit, (p.flags & MRHS_X0_GIVEN) != 0)) != MRHS_OK)
        return st;
    bool busy = true;
    while (busy)
        if ((st = e.advance(&busy)) != MRHS_OK)
            return st;
    if ((st = e.finish(all)) != MRHS_OK)
        return st;
    if (copy)
        MRHS_HIP(to_user(X, Xw, A.perm, A.n, m, p.m, s));
    if ((st = e.read_ctl()) != MRHS_OK)
        return st;
    const Ctl &h = e.host();
    const bool mixed = (p.flags & MRHS_MIXED) != 0;
    mrhs_status worst = MRHS_OK;
    for (int i = 0; i < p.m; ++i) {
        const mrhs_status cs = column_status(h.status[i]);
        if (info) {
            info[i].iters = mixed ? h.total_iters[i] : h.iters[i];
            info[i].restarts = h.restarts[i];
            info[i].outer = mixed ? h.outer[i] : 0;
            info[i].status = cs;
            info[i].relres = h.relres[i];
        }
        if (cs < worst)
            worst = cs;
    }
    if (worst != MRHS_OK)
        set_error(worst, "not every column converged");
    return worst;
}

} // namespace mrhs
