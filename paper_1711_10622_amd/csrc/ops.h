// Per-row operations ("ops") plugged into the tile loops of core.h, and the
// per-column control logic of block BiCGStab that runs in the last workgroup
// of a grid reduction.
//
// The solve keeps the right Jacobi preconditioner folded into the matrix:
// with D = diag(A) and Ah = A D^-1 (stored once per matrix), BiCGStab runs on
// Ah y = b and x = D^-1 y.  In exact arithmetic its iterates are those of
// BiCGStab on A x = b with p^ = D^-1 p, s^ = D^-1 s (the right-preconditioned
// form), without a separate preconditioner pass.  Per iteration, for every
// running column (van der Vorst 1992, as cited in Section 1):
//
//   v   = Ah p;   sigma = (r^, v);      alpha = rho / sigma
//   s   = r - alpha v                   (never stored: recomputed where used)
//   t   = Ah s;   omega = (t, s)/(t, t)
//   y  += alpha p + omega s;   r = s - omega t;   rho = (r^, r)
//   p   = r + beta (p - omega v)        beta = (rho_next/rho)(alpha/omega)
//
// with p = r at a (re)start.  The p update is done in the same pass as the
// y and r updates, so beta must be known before that pass: it uses the
// BiCGStab identity (r^, s) = rho - alpha sigma = 0, i.e.
// rho_next = (r^, s - omega t) = -omega (r^, t), summed in the t = Ah s
// pass.  rho itself (for alpha) and ||r|| (for the stopping test) are still
// the directly summed dot products of that update pass.
//
// Each column follows its own control flow (Section 2.2: the m realizations
// are independent systems sharing A):
//   * ||r|| <= tol ||b|| after an iteration, or ||s|| <= tol ||b|| (then the
//     omega half step is skipped), marks the column for a true-residual check;
//     the check either confirms convergence or restarts from r = b - A x.
//   * sigma, omega or rho zero or non-finite is a breakdown: restart from the
//     true residual; the fourth breakdown in a row ends the column.
//   * maxit iterations end the column (restarts count toward maxit).
// The inner solve of mixed-precision refinement runs the same iteration in
// binary32 without restarts; it ends on its relative tolerance, on a
// breakdown, on stagnation (no halving of ||r|| over stag_window iterations,
// 80 by default: shorter windows end inner solves that are still converging,
// 50 cost 13 % more time on the 256x192x256 channel) or on its iteration
// budget.
#pragma once

#include "core.h"
#include "mrhs.h"

namespace mrhs {

enum ColStatus : int32_t {
    COL_IDLE = 0,        // slot not in use
    COL_RUN = 1,         // iterating
    COL_PEND_CHECK = 2,  // recurrence says converged: true residual pending
    COL_PEND_BD = 3,     // breakdown: restart pending
    COL_DONE = 4,        // converged (true residual)
    COL_NOCONV = 5,      // maxit reached
    COL_BREAKDOWN = 6,   // breakdown persisted / non-finite data
    COL_INNER_DONE = 7,  // mixed: inner solve finished, refinement step pending
    COL_OUTER = 8,       // mixed: next inner solve pending (r, ||r|| known)
    COL_INIT = 9,        // admitted: first residual pending
};

enum IterFlag : int32_t { F_SCONV = 1, F_OMEGA_BAD = 2, F_RESTART = 4, F_ZERO_X = 8 };

enum SolveMode : int32_t { MODE_F64 = 0, MODE_INNER = 1 };

constexpr int kMaxBreakdownRestarts = 3;
constexpr int kGcrMax = 8;  // stored refinement directions (mixed precision)
constexpr int kStagWindow = 80;  // default of Ctl::stag_window

struct Ctl {
    int32_t status[kMaxM];
    int32_t fresh[kMaxM];
    int32_t flag[kMaxM];
    int32_t iters[kMaxM];
    int32_t maxit[kMaxM];
    int32_t restarts[kMaxM];
    int32_t breakdowns[kMaxM];
    int32_t bd_run[kMaxM];
    int32_t outer[kMaxM];
    int32_t total_iters[kMaxM];
    int32_t stag_it[kMaxM];
    int32_t inner_maxit[kMaxM];
    double nb[kMaxM];
    double tol[kMaxM];
    double rn[kMaxM];
    double stag_rn[kMaxM];
    double relres[kMaxM];
    double rscale[kMaxM];
    double colsum[kMaxM];
    int32_t kcol[kMaxM];                 // mixed: slot of the column's next stored direction
    double wnew2[kMaxM];                 // mixed: ||w||^2 of the new direction
    double gamma[kMaxM];                 // mixed: step length of the refinement step
    double beta[kGcrMax][kMaxM];         // mixed: projections on the stored directions
    double wnorm2[kGcrMax][kMaxM];       // mixed: ||w_j||^2 of the stored directions
    double tol_in;
    int32_t mode;
    int32_t max_outer;
    int32_t n;
    int32_t stag_window;  // mixed: inner iterations over which ||r|| must halve
};

template <typename T>
struct Kry {
    T rho[kMaxM];
    T rho_old[kMaxM];
    T alpha[kMaxM];
    T omega[kMaxM];
    T nbi[kMaxM];
    T beta[kMaxM];  // for the p update of the current iteration
};

template <typename T>
__device__ __forceinline__ bool bad(T v)
{
    return v == T(0) || !isfinite(v);
}

__device__ __forceinline__ bool pending(int32_t s) { return s == COL_PEND_CHECK || s == COL_PEND_BD; }

// The shadow residual r^ of the binary64 BiCGStab: one vector shared by every
// column, row i holding value number i of the SplitMix64 stream of seed
// MRHS_SHADOW_SEED (Steele, Lea and Flood, OOPSLA 2014) mapped to [-1, 1).
// It is generated where a dot product needs it, never stored, which takes one
// block read out of each of the three passes of an iteration.  The binary32
// inner solves of mixed precision restart at every refinement step, and over
// such short solves a random r^ converges far worse; they take r^ = sign(r0)
// of their own initial residual r0 (entries +-1, +1 for a zero), stored as
// one bit per element: lane g of a row keeps the bits of its VW columns in
// byte i * L + g of the sign array.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__device__ __forceinline__ T shadow(int32_t i);

template <>
__device__ __forceinline__ double shadow<double>(int32_t i)
{
    // top 53 bits scaled to [0, 2) then shifted: exact in binary64
    return static_cast<double>(splitmix64_at(MRHS_SHADOW_SEED, static_cast<uint64_t>(i)) >> 11) * 0x1p-52 - 1.0;
}

template <>
__device__ __forceinline__ float shadow<float>(int32_t i)
{
    // top 24 bits: exact in binary32
    const uint32_t u = static_cast<uint32_t>(splitmix64_at(MRHS_SHADOW_SEED, static_cast<uint64_t>(i)) >> 40);
    return static_cast<float>(u) * 0x1p-23f - 1.0f;
}

// The shadow values of this lane's VW columns of row i: from the sign bits,
// or the generated vector when sgn is null.
template <typename T, int M>
__device__ __forceinline__ void shadow_row(const uint8_t *sgn, int32_t i, int g, T *h)
{
    using S = Shape<T, M>;
    static_assert(S::L <= kMaxM && S::VW <= 8, "a lane's sign bits fit one byte of a row's kMaxM");
    if (sgn) {
        const uint32_t b = sgn[static_cast<size_t>(i) * S::L + g];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            h[q] = ((b >> q) & 1u) ? T(-1) : T(1);
    } else {
        const T s = shadow<T>(i);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            h[q] = s;
    }
}

// ---------------------------------------------------------------------------
// Plain product Y = A X.
template <typename T, int M>
struct OpStore {
    static constexpr const char *kName = "gspmv";
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *X;
    T *Y;
    struct Lane {
        bool on;
    };
    __device__ Lane lane(int) const { return {true}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const
    {
        ld<T, M>(X, c, g, x);
    }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const T *sum,
                                        Acc<T, S::VW, NDOT> &) const
    {
        st<T, M>(Y, i, g, sum);
    }
    __device__ void finish(const T *) const {}
};

// The solver may keep r and v as one interleaved n x 2M block (row i = r_i
// then v_i, so v = r + M): the two rows spmv_omega gathers from one column
// index then share cache lines, which halves the lines fetched per entry when
// rows are visited in no particular order.  Ops take the row stride of r and
// v as ldp (2M when interleaved, else M).

// ---------------------------------------------------------------------------
// Residual R = B - A X with per-column sums of R*R and B*B.  Which columns are
// computed, and what the last workgroup does with the norms, depends on kind.
enum ResidKind : int32_t {
    RES_SETUP = 0,  // first residual of newly admitted (COL_INIT) columns
    RES_CHECK = 1,  // true residual of columns with a pending check/breakdown
    RES_FINAL = 2,  // residual of the returned x (columns in cmask)
    RES_NORM = 4,   // only the norms, into ctl->relres (API use)
    RES_MIXCHECK = 5,  // mixed: true residual of columns whose refinement converged
};

template <int M>
struct OpResid {
    static constexpr const char *kName = "resid";
    using T = double;
    using S = Shape<double, M>;
    static constexpr int NDOT = 3;
    const double *X;
    const double *B;
    double *R;
    double *R2;  // optional second copy of R (may be null)
    double *R3;  // optional third copy of R (may be null)
    Ctl *ctl;
    Kry<double> *kry;
    int32_t kind;
    uint32_t cmask;  // columns of RES_FINAL / RES_NORM
    int32_t rcm;     // > 0: R is column-major with column stride rcm (R2, R3 unused)
    int32_t rld;     // row stride of R when rcm == 0 (0: M; 2M for the r half of an r/v pair)
    struct Lane {
        bool on;
        bool act[S::VW];
    };
    __device__ bool col_on(int c) const
    {
        if (c >= M)
            return false;
        const int32_t st = ctl->status[c];
        switch (kind) {
        case RES_SETUP:
            return st == COL_INIT;
        case RES_CHECK:
        case RES_MIXCHECK:
            return pending(st);
        default:
            return (cmask >> c) & 1u;
        }
    }
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int v = 0; v < S::VW; ++v) {
            ln.act[v] = col_on(g * S::VW + v);
            ln.on = ln.on || ln.act[v];
        }
        return ln;
    }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, double *x) const
    {
        ld<double, M>(X, c, g, x);
    }
    // the row's own b, loaded before its gathers
    struct Pre {
        double b[S::VW];
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<double, M>(B, i, g, pr.b);
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, const double *sum,
                                        Acc<double, S::VW, NDOT> &acc, const Pre &pr) const
    {
        const size_t o = static_cast<size_t>(i) * M + g * S::VW;
        const double *b = pr.b;
        double r[S::VW];
        const bool restart = kind == RES_SETUP || kind == RES_CHECK;
        const double h = restart ? shadow<double>(i) : 0.0;
#pragma unroll
        for (int v = 0; v < S::VW; ++v) {
            r[v] = b[v] - sum[v];
            if (ln.act[v]) {
                acc.a[0][v] += r[v] * r[v];
                acc.a[1][v] += b[v] * b[v];
                acc.a[2][v] += h * r[v];
            }
        }
        if (rcm > 0) {
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                if (ln.act[v] && R)
                    R[static_cast<size_t>(g * S::VW + v) * rcm + i] = r[v];
            return;
        }
        bool all = true;
#pragma unroll
        for (int v = 0; v < S::VW; ++v)
            all = all && ln.act[v];
        if (all) {
            if (R)
                st<double, M>(R, i, g, r, rld ? rld : M);
            if (R2)
                st<double, M>(R2, i, g, r);
            if (R3)
                st<double, M>(R3, i, g, r);
        } else {
            // only the columns this kind owns are written
            const size_t orow = static_cast<size_t>(i) * (rld ? rld : M) + g * S::VW;
#pragma unroll
            for (int v = 0; v < S::VW; ++v) {
                if (!ln.act[v])
                    continue;
                if (R)
                    R[orow + v] = r[v];
                if (R2)
                    R2[o + v] = r[v];
                if (R3)
                    R3[o + v] = r[v];
            }
        }
    }
    __device__ void finish(const double *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || !col_on(c))
            return;
        const double rr = tot[c];
        const double bb = tot[M + c];
        const double hr = tot[2 * M + c];  // (r^, r) of the setup / restart residual
        Ctl &k = *ctl;
        switch (kind) {
        case RES_SETUP: {
            const double nb = sqrt(bb);
            k.nb[c] = nb;
            k.fresh[c] = 1;
            k.flag[c] = 0;
            kry->rho[c] = hr;
            kry->rho_old[c] = kry->alpha[c] = kry->omega[c] = 1.0;
            if (!isfinite(nb)) {
                k.status[c] = COL_BREAKDOWN;
                k.flag[c] = F_ZERO_X;
                k.rn[c] = nb;
            } else if (nb == 0.0) {
                k.status[c] = COL_DONE;
                k.flag[c] = F_ZERO_X;
                k.rn[c] = 0.0;
            } else {
                const double rn = sqrt(rr) / nb;
                const bool mixed = k.mode == MODE_INNER;
                k.rn[c] = rn;
                if (rn <= k.tol[c])
                    k.status[c] = COL_DONE;
                else if (bad(rr))
                    k.status[c] = mixed ? COL_BREAKDOWN : COL_PEND_BD;
                else if (!mixed && bad(hr))
                    k.status[c] = COL_PEND_BD;
                else if (k.iters[c] >= k.maxit[c])
                    k.status[c] = COL_NOCONV;
                else
                    k.status[c] = mixed ? COL_OUTER : COL_RUN;
                k.rscale[c] = sqrt(rr);
            }
            break;
        }
        case RES_CHECK: {
            const int32_t st = k.status[c];
            const double nr = sqrt(rr) / k.nb[c];
            k.flag[c] = 0;
            if (st == COL_PEND_BD) {
                k.breakdowns[c] += 1;
                if (k.bd_run[c] >= kMaxBreakdownRestarts) {
                    k.status[c] = COL_BREAKDOWN;
                    break;
                }
                k.bd_run[c] += 1;
                k.restarts[c] += 1;
            }
            k.rn[c] = nr;
            if (nr <= k.tol[c]) {
                k.status[c] = COL_DONE;
                break;
            }
            if (st == COL_PEND_CHECK)
                k.restarts[c] += 1;
            // restart from the true residual: r = p = b - A x
            kry->rho[c] = hr;
            kry->rho_old[c] = kry->alpha[c] = kry->omega[c] = 1.0;
            k.fresh[c] = 1;
            k.flag[c] = F_RESTART;
            k.status[c] = (k.iters[c] >= k.maxit[c]) ? COL_NOCONV : COL_RUN;
            break;
        }
        case RES_FINAL:
        case RES_NORM:
            k.relres[c] = (k.nb[c] > 0.0) ? sqrt(rr) / k.nb[c] : (k.flag[c] & F_ZERO_X ? 0.0 : sqrt(rr));
            break;
        case RES_MIXCHECK: {
            const double nr = sqrt(rr);
            k.rn[c] = nr / k.nb[c];
            if (!isfinite(nr)) {
                k.status[c] = COL_BREAKDOWN;
            } else if (nr / k.nb[c] <= k.tol[c]) {
                k.status[c] = COL_DONE;
            } else if (k.outer[c] >= ctl->max_outer || k.total_iters[c] >= k.maxit[c]) {
                k.status[c] = COL_NOCONV;
            } else {
                k.restarts[c] += 1;  // continue from the true residual
                k.rscale[c] = nr;
                k.status[c] = COL_OUTER;
            }
            break;
        }
        default:
            break;
        }
    }
};

// ---------------------------------------------------------------------------
// Shared pieces of the Krylov ops: per-lane running flags.
template <typename T, int M>
struct RunLane {
    using S = Shape<T, M>;
    bool on;
    bool act[S::VW];
};

template <typename T, int M>
__device__ __forceinline__ RunLane<T, M> run_lane(const Ctl *ctl, int g)
{
    using S = Shape<T, M>;
    RunLane<T, M> ln;
    ln.on = false;
#pragma unroll
    for (int v = 0; v < S::VW; ++v) {
        ln.act[v] = g * S::VW + v < M && ctl->status[g * S::VW + v] == COL_RUN;
        ln.on = ln.on || ln.act[v];
    }
    return ln;
}

// Column c (running) after its sigma = (r^, v): counts the iteration and
// forms alpha, or marks a breakdown.
template <typename T>
__device__ __forceinline__ void sigma_decide(Ctl &k, Kry<T> *kry, int c, T sigma)
{
    k.iters[c] += 1;
    if (bad(sigma)) {
        k.status[c] = (k.mode == MODE_INNER) ? COL_INNER_DONE : COL_PEND_BD;
        return;
    }
    kry->alpha[c] = kry->rho[c] / sigma;
}

// v = Ah p with sigma = (r^, v); the last workgroup forms alpha.
template <typename T, int M>
struct OpSpmv1 {
    static constexpr const char *kName = "spmv_sigma";
    using S = Shape<T, M>;
    static constexpr int NDOT = 1;
    const T *p;
    T *v;
    const uint8_t *sgn;  // sign bits of the shadow residual, or null: generated
    Ctl *ctl;
    Kry<T> *kry;
    int32_t ldp;  // row stride of v
    using Lane = RunLane<T, M>;
    __device__ Lane lane(int g) const { return run_lane<T, M>(ctl, g); }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const
    {
        ld<T, M>(p, c, g, x);
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, const T *sum,
                                        Acc<T, S::VW, NDOT> &acc) const
    {
        T h[S::VW];
        shadow_row<T, M>(sgn, i, g, h);
        st<T, M>(v, i, g, sum, ldp);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            if (ln.act[q])
                acc.a[0][q] += h[q] * sum[q];
    }
    __device__ void finish(const T *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || ctl->status[c] != COL_RUN)
            return;
        sigma_decide(*ctl, kry, c, tot[c]);
    }
};

// t = Ah s with s = r - alpha v formed on the fly from r and v (s is never
// stored); sums (t,s), (t,t), (s,s).  The last workgroup forms omega.
template <typename T, int M>
struct OpSpmv2 {
    static constexpr const char *kName = "spmv_omega";
    using S = Shape<T, M>;
    static constexpr int NDOT = 4;
#ifndef MRHS_OMEGA_GATHERED
#define MRHS_OMEGA_GATHERED 2
#endif
    static constexpr int GATHERED = MRHS_OMEGA_GATHERED;  // r and v
    const T *r;
    const T *v;
    const uint8_t *sgn;  // sign bits of the shadow residual, or null: generated
    T *t;
    Ctl *ctl;
    Kry<T> *kry;
    int32_t ldp;  // row stride of r and v
    struct Lane {
        bool on;
        bool act[S::VW];
        T alpha[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        const RunLane<T, M> rl = run_lane<T, M>(ctl, g);
        ln.on = rl.on;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            ln.act[q] = rl.act[q];
            ln.alpha[q] = kry->alpha[g * S::VW + q];
        }
        return ln;
    }
    __device__ __forceinline__ void gather(const Lane &ln, int32_t c, int g, T *x) const
    {
        T rr[S::VW], vv[S::VW];
        ld<T, M>(r, c, g, rr, ldp);
        ld<T, M>(v, c, g, vv, ldp);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            x[q] = rr[q] - ln.alpha[q] * vv[q];
    }
    // the row's own s = r - alpha v, loaded before its gathers
    struct Pre {
        T s[S::VW];
    };
    __device__ __forceinline__ Pre pre(const Lane &ln, int32_t i, int g) const
    {
        Pre pr;
        gather(ln, i, g, pr.s);
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, const T *sum,
                                        Acc<T, S::VW, NDOT> &acc, const Pre &pr) const
    {
        const T *s = pr.s;
        T h[S::VW];
        shadow_row<T, M>(sgn, i, g, h);
        st<T, M>(t, i, g, sum);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (ln.act[q]) {
                acc.a[0][q] += sum[q] * s[q];
                acc.a[1][q] += sum[q] * sum[q];
                acc.a[2][q] += s[q] * s[q];
                acc.a[3][q] += h[q] * sum[q];
            }
        }
    }
    __device__ void finish(const T *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || ctl->status[c] != COL_RUN)
            return;
        Ctl &k = *ctl;
        const T ts = tot[c], tt = tot[M + c], ss = tot[2 * M + c], ht = tot[3 * M + c];
        const double nb = (k.mode == MODE_INNER) ? static_cast<double>(kry->nbi[c]) : k.nb[c];
        const double tol = (k.mode == MODE_INNER) ? k.tol_in : k.tol[c];
        int32_t f = 0;
        if (static_cast<double>(sqrt(ss)) / nb <= tol) {
            f = F_SCONV;
        } else {
            const T w = ts / tt;
            if (bad(w)) {
                f = F_OMEGA_BAD;
            } else {
                kry->omega[c] = w;
                // rho_next = -omega (r^, t), so beta = (rho_next/rho)(alpha/omega)
                kry->beta[c] = ((-w * ht) / kry->rho[c]) * (kry->alpha[c] / w);
            }
        }
        k.flag[c] = f;
    }
};

// Column c (running) after its x/r update with sums (r^, r) and (r, r): the
// stopping tests and the next rho.
template <typename T>
__device__ __forceinline__ void xr_decide(Ctl &k, Kry<T> *kry, int c, T rhr, T rr)
{
    const bool inner = k.mode == MODE_INNER;
    const double nb = inner ? static_cast<double>(kry->nbi[c]) : k.nb[c];
    const double tol = inner ? k.tol_in : k.tol[c];
    const double rn = static_cast<double>(sqrt(rr)) / nb;
    k.rn[c] = rn;
    const int32_t f = k.flag[c];
    if (f & F_SCONV) {
        k.status[c] = inner ? COL_INNER_DONE : COL_PEND_CHECK;
        return;
    }
    if (f & F_OMEGA_BAD) {
        k.status[c] = inner ? COL_INNER_DONE : COL_PEND_BD;
        return;
    }
    kry->rho_old[c] = kry->rho[c];
    kry->rho[c] = rhr;
    k.fresh[c] = 0;
    k.bd_run[c] = 0;
    if (rn <= tol) {
        k.status[c] = inner ? COL_INNER_DONE : COL_PEND_CHECK;
    } else if (bad(rhr)) {
        k.status[c] = inner ? COL_INNER_DONE : COL_PEND_BD;
    } else if (inner) {
        if (k.iters[c] >= k.inner_maxit[c]) {
            k.status[c] = COL_INNER_DONE;
        } else if (k.iters[c] - k.stag_it[c] >= k.stag_window) {
            if (rn > 0.5 * k.stag_rn[c])
                k.status[c] = COL_INNER_DONE;
            k.stag_it[c] = k.iters[c];
            k.stag_rn[c] = rn;
        }
    } else if (k.iters[c] >= k.maxit[c]) {
        k.status[c] = COL_NOCONV;
    }
}

// y += alpha p + omega s;  r = s - omega t  (s = r - alpha v); sums (r^, r)
// and (r, r).  The last workgroup updates rho and each column's state.
template <typename T, int M>
struct OpXR {
    static constexpr const char *kName = "xr_update";
    // two workgroups per CU instead of the six that fit: fewer concurrent
    // streams (five read, three written per row) per memory channel; on the
    // 12.6M-row channel 2520 -> 2436 us per launch at m = 16 and 1.2-2.3 %
    // less time per iteration at m = 4, 8, 16 and in mixed solves, the same
    // at m = 1 (full solves; one workgroup per CU is no faster)
    static constexpr int kMaxPerCU = 2;
    using S = Shape<T, M>;
    static constexpr int NDOT = 2;
    T *y;
    T *r;
    T *p;
    const T *v;
    const T *t;
    const uint8_t *sgn;  // sign bits of the shadow residual, or null: generated
    Ctl *ctl;
    Kry<T> *kry;
    int32_t ldp;  // row stride of r and v
    struct Lane {
        bool on;
        bool act[S::VW];
        bool use_w[S::VW];
        T alpha[S::VW], omega[S::VW], beta[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        const RunLane<T, M> rl = run_lane<T, M>(ctl, g);
        ln.on = rl.on;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = rl.act[q];
            ln.use_w[q] = ctl->flag[c] == 0;
            ln.alpha[q] = kry->alpha[c];
            ln.omega[q] = ln.use_w[q] ? kry->omega[c] : T(0);
            ln.beta[q] = kry->beta[c];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<T, S::VW, NDOT> &acc) const
    {
        T yy[S::VW], rr[S::VW], pp[S::VW], vv[S::VW], tt[S::VW];
        ld<T, M>(y, i, g, yy);
        ld<T, M>(r, i, g, rr, ldp);
        ld<T, M>(p, i, g, pp);
        ld<T, M>(v, i, g, vv, ldp);
        ld<T, M>(t, i, g, tt);
        T hh[S::VW];
        shadow_row<T, M>(sgn, i, g, hh);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (ln.act[q]) {
                const T s = rr[q] - ln.alpha[q] * vv[q];
                if (ln.use_w[q]) {
                    yy[q] = yy[q] + (ln.alpha[q] * pp[q] + ln.omega[q] * s);
                    rr[q] = s - ln.omega[q] * tt[q];
                    pp[q] = rr[q] + ln.beta[q] * (pp[q] - ln.omega[q] * vv[q]);
                } else {
                    yy[q] = yy[q] + ln.alpha[q] * pp[q];
                    rr[q] = s;
                }
                acc.a[0][q] += hh[q] * rr[q];
                acc.a[1][q] += rr[q] * rr[q];
            }
        }
        st<T, M>(y, i, g, yy);
        st<T, M>(r, i, g, rr, ldp);
        st<T, M>(p, i, g, pp);
    }
    __device__ void finish(const T *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || ctl->status[c] != COL_RUN)
            return;
        xr_decide(*ctl, kry, c, tot[c], tot[M + c]);
    }
};

// One kernel for the end of an iteration and the start of the next: the
// x/r/p update of OpXR and the product v = Ah p of OpSpmv1 with the new p.
// The new p of a gathered row is formed on the fly from that row's old r, v,
// t and p with the same fused operations as the row's own update, so v is
// exactly Ah times the stored new p.  Other workgroups still gather the old
// r, v, p while a row's new values are written, so those go to a second set
// of blocks (r2, v2, p2; the caller alternates the two sets); y is only read
// and written by its own row and is updated in place.  Sums (r^, r), (r, r)
// and sigma = (r^, v); the last workgroup takes OpXR's decisions and then,
// for columns still running, OpSpmv1's.  The binary64 Jacobi solve uses it
// for narrow blocks on small and mid-size matrices (see merged_iteration).
template <typename T, int M>
struct OpXRSigma {
    static constexpr const char *kName = "xr_sigma";
    using S = Shape<T, M>;
    static constexpr int NDOT = 3;
    static constexpr int GATHERED = 4;  // r, v, t, p
    T *y;
    const T *r, *v, *t, *p;  // this iteration's blocks (r and v with row stride ldp)
    T *r2, *v2, *p2;         // the next iteration's
    Ctl *ctl;
    Kry<T> *kry;
    int32_t ldp;
    struct Lane {
        bool on;
        bool act[S::VW];
        bool use_w[S::VW];
        T alpha[S::VW], omega[S::VW], beta[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        const RunLane<T, M> rl = run_lane<T, M>(ctl, g);
        ln.on = rl.on;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = rl.act[q];
            ln.use_w[q] = c < M && ctl->flag[c] == 0;
            ln.alpha[q] = c < M ? kry->alpha[c] : T(0);
            ln.omega[q] = ln.use_w[q] ? kry->omega[c] : T(0);
            ln.beta[q] = c < M ? kry->beta[c] : T(0);
        }
        return ln;
    }
    // s = r - alpha v; r' = s - omega t; p' = r' + beta (p - omega v) for a
    // column taking the full step, r' = s and p' = p after the half step
    // (s converged, or omega unusable), everything unchanged for a column
    // that is not running
    static __device__ __forceinline__ void step(const Lane &ln, int q, T r, T v, T t, T p, T &s, T &rn, T &pn)
    {
        if (!ln.act[q]) {
            s = r;
            rn = r;
            pn = p;
            return;
        }
        s = __builtin_fma(-ln.alpha[q], v, r);
        if (ln.use_w[q]) {
            rn = __builtin_fma(-ln.omega[q], t, s);
            pn = __builtin_fma(ln.beta[q], __builtin_fma(-ln.omega[q], v, p), rn);
        } else {
            rn = s;
            pn = p;
        }
    }
    __device__ __forceinline__ void gather(const Lane &ln, int32_t c, int g, T *x) const
    {
        T rr[S::VW], vv[S::VW], tt[S::VW], pp[S::VW];
        ld<T, M>(r, c, g, rr, ldp);
        ld<T, M>(v, c, g, vv, ldp);
        ld<T, M>(t, c, g, tt);
        ld<T, M>(p, c, g, pp);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            T s_, r_;
            step(ln, q, rr[q], vv[q], tt[q], pp[q], s_, r_, x[q]);
        }
    }
    struct Pre {
        T y[S::VW], r[S::VW], v[S::VW], t[S::VW], p[S::VW];
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<T, M>(y, i, g, pr.y);
        ld<T, M>(r, i, g, pr.r, ldp);
        ld<T, M>(v, i, g, pr.v, ldp);
        ld<T, M>(t, i, g, pr.t);
        ld<T, M>(p, i, g, pr.p);
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, const T *sum, Acc<T, S::VW, NDOT> &acc,
                                        const Pre &pr) const
    {
        T yy[S::VW], rn[S::VW], pn[S::VW], hh[S::VW];
        shadow_row<T, M>(nullptr, i, g, hh);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            T s;
            step(ln, q, pr.r[q], pr.v[q], pr.t[q], pr.p[q], s, rn[q], pn[q]);
            yy[q] = pr.y[q];
            if (ln.act[q]) {
                yy[q] = ln.use_w[q] ? pr.y[q] + (ln.alpha[q] * pr.p[q] + ln.omega[q] * s)
                                    : pr.y[q] + ln.alpha[q] * pr.p[q];
                acc.a[0][q] += hh[q] * rn[q];
                acc.a[1][q] += rn[q] * rn[q];
                acc.a[2][q] += hh[q] * sum[q];
            }
        }
        st<T, M>(y, i, g, yy);
        st<T, M>(r2, i, g, rn, ldp);
        st<T, M>(p2, i, g, pn);
        st<T, M>(v2, i, g, sum, ldp);
    }
    __device__ void finish(const T *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || ctl->status[c] != COL_RUN)
            return;
        xr_decide(*ctl, kry, c, tot[c], tot[M + c]);
        if (ctl->status[c] == COL_RUN)
            sigma_decide(*ctl, kry, c, tot[2 * M + c]);
    }
};

// After a check: columns restarting take r = r^ = (true residual) rt.
template <typename T, int M>
struct OpRestart {
    static constexpr const char *kName = "restart";
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *rt;
    T *r;
    T *p;
    const Ctl *ctl;
    int32_t ldp;  // row stride of r
    struct Lane {
        bool on;
        bool act[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = c < M && (ctl->flag[c] & F_RESTART) && ctl->status[c] == COL_RUN;
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<T, S::VW, NDOT> &) const
    {
        T a[S::VW], b[S::VW], pp[S::VW];
        ld<T, M>(rt, i, g, a);
        ld<T, M>(r, i, g, b, ldp);
        ld<T, M>(p, i, g, pp);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            if (ln.act[q]) {
                b[q] = a[q];
                pp[q] = a[q];
            }
        st<T, M>(r, i, g, b, ldp);
        st<T, M>(p, i, g, pp);
    }
    __device__ void finish(const T *) const {}
};

// Conversions between y (Ah y = b) and x = D^-1 y, and the null-space
// projection, for every non-idle column.
enum ScaleKind : int32_t {
    SC_IN = 0,        // y = D x          (initial guess given)
    SC_OUT = 1,       // x = D^-1 y, or 0 where F_ZERO_X
    SC_ZERO = 2,      // y = 0
    SC_SUB_MEAN = 3,  // x -= colsum / n
    SC_FIX_ZERO = 4,  // x = 0 where F_ZERO_X
};

template <int M>
struct OpScale {
    static constexpr const char *kName = "scale";
    using S = Shape<double, M>;
    static constexpr int NDOT = 0;
    double *x;
    const double *diag;
    const double *dinv;
    const Ctl *ctl;
    int32_t kind;
    uint32_t cmask;
    struct Lane {
        bool on;
        bool act[S::VW];
        bool zero[S::VW];
        double mean[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = c < M && ((cmask >> c) & 1u);
            ln.zero[q] = (ctl->flag[c] & F_ZERO_X) != 0;
            ln.mean[q] = ctl->colsum[c] / static_cast<double>(ctl->n);
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<double, S::VW, NDOT> &) const
    {
        double a[S::VW];
        ld<double, M>(x, i, g, a);
        const double di = (kind == SC_IN) ? diag[i] : (kind == SC_OUT ? dinv[i] : 1.0);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (!ln.act[q])
                continue;
            if (kind == SC_ZERO)
                a[q] = 0.0;
            else if (kind == SC_SUB_MEAN)
                a[q] = a[q] - ln.mean[q];
            else if ((kind == SC_OUT || kind == SC_FIX_ZERO) && ln.zero[q])
                a[q] = 0.0;
            else if (kind == SC_IN || kind == SC_OUT)
                a[q] = a[q] * di;
        }
        st<double, M>(x, i, g, a);
    }
    __device__ void finish(const double *) const {}
};

// Column sums of x (for the null-space projection).
template <int M>
struct OpColSum {
    static constexpr const char *kName = "colsum";
    using S = Shape<double, M>;
    static constexpr int NDOT = 1;
    const double *x;
    Ctl *ctl;
    uint32_t cmask;
    struct Lane {
        bool on;
        bool act[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            ln.act[q] = g * S::VW + q < M && ((cmask >> (g * S::VW + q)) & 1u);
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<double, S::VW, NDOT> &acc) const
    {
        double a[S::VW];
        ld<double, M>(x, i, g, a);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            if (ln.act[q])
                acc.a[0][q] += a[q];
    }
    __device__ void finish(const double *tot) const
    {
        const int c = threadIdx.x;
        if (c < M && ((cmask >> c) & 1u))
            ctl->colsum[c] = tot[c];
    }
};

// Mixed precision: start an inner solve for each COL_RUN column:
// r32 = p32 = RN32(r64 / ||r64||), r^ = sign(r32) (bits), y32 = 0; sums
// (r32, r32) = (r^, r32)... in binary32: (r32, r32) for the norm and
// (r^, r32) = ||r32||_1 for rho.
template <int M>
struct OpCast {
    static constexpr const char *kName = "cast32";
    using S = Shape<float, M>;
    static constexpr int NDOT = 2;
    const double *r64;  // column-major n x m
    float *r;
    uint8_t *sgn;
    float *y;
    float *p;
    Ctl *ctl;
    Kry<float> *kry;
    int32_t n;
    int32_t ldp;  // row stride of r
    struct Lane {
        bool on;
        bool act[S::VW];
        double scale[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = c < M && ctl->status[c] == COL_OUTER;
            ln.scale[q] = ctl->rscale[c];
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<float, S::VW, NDOT> &acc) const
    {
        float a[S::VW], z[S::VW], pp[S::VW];
        ld<float, M>(r, i, g, a, ldp);
        ld<float, M>(y, i, g, z);
        ld<float, M>(p, i, g, pp);
        uint8_t *sb = sgn + static_cast<size_t>(i) * S::L + g;
        uint32_t bits = *sb;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (ln.act[q]) {
                const float f = static_cast<float>(r64[static_cast<size_t>(g * S::VW + q) * n + i] / ln.scale[q]);
                a[q] = f;
                pp[q] = f;
                z[q] = 0.0f;
                acc.a[0][q] += f * f;
                acc.a[1][q] += fabsf(f);
                bits = (f < 0.0f) ? (bits | (1u << q)) : (bits & ~(1u << q));
            }
        }
        st<float, M>(r, i, g, a, ldp);
        st<float, M>(y, i, g, z);
        st<float, M>(p, i, g, pp);
        *sb = static_cast<uint8_t>(bits);
    }
    __device__ void finish(const float *tot) const
    {
        const int c = threadIdx.x;
        if (c >= M || ctl->status[c] != COL_OUTER)
            return;
        Ctl &k = *ctl;
        k.status[c] = COL_RUN;
        k.inner_maxit[c] = k.maxit[c] - k.total_iters[c];
        const float rr = tot[c];
        kry->rho[c] = tot[M + c];  // (r^, r32) = ||r32||_1
        kry->nbi[c] = sqrtf(rr);
        kry->rho_old[c] = kry->alpha[c] = kry->omega[c] = 1.0f;
        k.fresh[c] = 1;
        k.flag[c] = 0;
        k.iters[c] = 0;
        k.stag_it[c] = 0;
        k.stag_rn[c] = 1.0;
        if (!(rr > 0.0f) || !isfinite(rr))
            k.status[c] = COL_INNER_DONE;
    }
};

// ---------------------------------------------------------------------------
// Mixed precision refinement step (binary64), for every column whose binary32
// inner solve ended.  The inner solve of Ah32 y = r/||r|| gives the correction
// z = ||r|| D^-1 y; with w = A z the step is made minimal-residual over the
// new and the column's stored directions (generalized conjugate residuals,
// truncated to the most recent ndirs directions):
//   w -= sum_j beta_j w_j, z -= sum_j beta_j z_j, beta_j = (w, w_j)/(w_j, w_j)
//   gamma = (r, w)/(w, w);  x += gamma z;  r -= gamma w.
// The refinement vectors are kept per column, column-major (column c's n
// values at offset c * n of an n x m buffer): r, the accumulated correction
// of x, the new direction z, w and the ndirs stored directions (slot kcol[c]
// receives the next one).  A step then streams only its own column's
// vectors, so it runs as soon as that column's inner solve ends; over
// row-interleaved blocks every step would stream all columns' rows.  A
// column's arithmetic never depends on the other columns of the block.
struct GcrBlocks {
    double *z[kGcrMax];  // stored directions z_j
    double *w[kGcrMax];  // and w_j = A z_j
    double *znew;        // the direction being formed
    double *wnew;
    double *xacc;        // accumulated correction of x (folded into X before checks and at the end)
    int32_t ndirs;       // directions kept per column
};

// z_new(:, c) = ||r_c|| D^-1 y32(:, c) for the columns whose inner solve ended
// (row-interleaved binary32 in, column-major binary64 out)
template <int M>
struct OpGcrZ {
    using S = Shape<float, M>;
    static constexpr const char *kName = "gcr_z";
    static constexpr int NDOT = 0;
    double *z;
    const float *y;
    const double *dinv;
    const Ctl *ctl;
    int32_t n;
    struct Lane {
        bool on;
        bool act[S::VW];
        double scale[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = c < M && ctl->status[c] == COL_INNER_DONE;
            ln.scale[q] = ctl->rscale[c];
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<float, S::VW, NDOT> &) const
    {
        float yy[S::VW];
        ld<float, M>(y, i, g, yy);
        const double di = dinv[i];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            if (ln.act[q])
                __builtin_nontemporal_store(ln.scale[q] * (di * static_cast<double>(yy[q])),
                                            z + static_cast<size_t>(g * S::VW + q) * n + i);
    }
    __device__ void finish(const float *) const {}
};

// ---- per-column refinement ops: streams over one column's n-vectors (M = 1)
struct ColLane {
    bool on;
};

// W = A Z for the K refinement columns whose inner solves ended in the same
// round, their vectors column-major (one n-vector per column, so each column
// keeps streaming only its own vectors): one product reads the matrix once
// for all K columns (each column's row sums are those of its own product).
template <int K>
struct OpColsStore {
    static constexpr const char *kName = "gcr_aw";
    using S = Shape<double, K>;
    static constexpr int NDOT = 0;
    const double *z[K];
    double *w[K];
    struct Lane {
        bool on;
    };
    __device__ Lane lane(int) const { return {true}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, double *x) const
    {
#pragma unroll
        for (int v = 0; v < S::VW; ++v) {
            const int q = g * S::VW + v;
            x[v] = q < K ? z[q][c] : 0.0;
        }
    }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const double *sum,
                                        Acc<double, S::VW, NDOT> &) const
    {
#pragma unroll
        for (int v = 0; v < S::VW; ++v) {
            const int q = g * S::VW + v;
            if (q < K)
                __builtin_nontemporal_store(sum[v], w[q] + i);
        }
    }
    __device__ void finish(const double *) const {}
};

// beta_j = (w, w_j) / (w_j, w_j) over the column's stored directions (slot
// kcol[c] is about to be replaced and is left out)
struct OpColDots {
    using S = Shape<double, 1>;
    static constexpr const char *kName = "gcr_dots";
    static constexpr int NDOT = kGcrMax;
    const double *w;
    const double *W[kGcrMax];
    int32_t jmax;
    int32_t col;
    Ctl *ctl;
    using Lane = ColLane;
    __device__ Lane lane(int) const { return {true}; }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int, Acc<double, 1, NDOT> &acc) const
    {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < kGcrMax; ++j)
            if (j < jmax)
                acc.a[j][0] += wi * W[j][i];
    }
    __device__ void finish(const double *tot) const
    {
        if (threadIdx.x != 0)
            return;
        const int c = col;
        for (int j = 0; j < kGcrMax; ++j) {
            const double d = ctl->wnorm2[j][c];
            const bool valid = j < jmax && j != ctl->kcol[c] && d > 0.0 && isfinite(d);
            const double bj = valid ? tot[j] / d : 0.0;
            ctl->beta[j][c] = isfinite(bj) ? bj : 0.0;
        }
    }
};

// w -= sum beta_j w_j, z -= sum beta_j z_j; sums (w, w) and (r, w).  Terms
// with beta_j = 0 are skipped, so slots holding stale data of an earlier
// request in the slot never enter the column's arithmetic.
struct OpColOrth {
    using S = Shape<double, 1>;
    static constexpr const char *kName = "gcr_orth";
    static constexpr int NDOT = 2;
    double *w;
    double *z;
    const double *W[kGcrMax];
    const double *Z[kGcrMax];
    const double *r;
    int32_t jmax;
    int32_t col;
    Ctl *ctl;
    struct Lane {
        bool on;
        double beta[kGcrMax];
    };
    __device__ Lane lane(int) const
    {
        Lane ln;
        ln.on = true;
#pragma unroll
        for (int j = 0; j < kGcrMax; ++j)
            ln.beta[j] = j < jmax ? ctl->beta[j][col] : 0.0;
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int, Acc<double, 1, NDOT> &acc) const
    {
        double wi = w[i], zi = z[i];
#pragma unroll
        for (int j = 0; j < kGcrMax; ++j) {
            if (j < jmax && ln.beta[j] != 0.0) {
                wi -= ln.beta[j] * W[j][i];
                zi -= ln.beta[j] * Z[j][i];
            }
        }
        acc.a[0][0] += wi * wi;
        acc.a[1][0] += r[i] * wi;
        if (jmax > 0) {
            __builtin_nontemporal_store(wi, w + i);
            __builtin_nontemporal_store(zi, z + i);
        }
    }
    __device__ void finish(const double *tot) const
    {
        if (threadIdx.x != 0)
            return;
        const double ww = tot[0], rw = tot[1];
        ctl->wnew2[col] = ww;
        ctl->gamma[col] = (ww > 0.0 && isfinite(ww) && isfinite(rw)) ? rw / ww : 0.0;
    }
};

// x_acc += gamma z;  r -= gamma w; the direction goes to the column's slot
// kcol[c]; sums (r, r).  The last workgroup decides the column's next state.
struct OpColUpdate {
    using S = Shape<double, 1>;
    static constexpr const char *kName = "gcr_update";
    static constexpr int NDOT = 1;
    double *xacc;
    double *r;
    const double *z;
    const double *w;
    double *zslot;
    double *wslot;
    int32_t ndirs;
    int32_t col;
    Ctl *ctl;
    struct Lane {
        bool on;
        double gamma;
    };
    __device__ Lane lane(int) const { return {true, ctl->gamma[col]}; }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int, Acc<double, 1, NDOT> &acc) const
    {
        const double zi = z[i], wi = w[i];
        const double ri = r[i] - ln.gamma * wi;
        __builtin_nontemporal_store(xacc[i] + ln.gamma * zi, xacc + i);
        __builtin_nontemporal_store(ri, r + i);
        __builtin_nontemporal_store(zi, zslot + i);
        __builtin_nontemporal_store(wi, wslot + i);
        acc.a[0][0] += ri * ri;
    }
    __device__ void finish(const double *tot) const
    {
        if (threadIdx.x != 0)
            return;
        const int c = col;
        Ctl &k = *ctl;
        const int slot = k.kcol[c];
        k.wnorm2[slot][c] = k.wnew2[c];
        k.kcol[c] = (slot + 1) % ndirs;
        const double nr = sqrt(tot[0]);
        k.total_iters[c] += k.iters[c];
        k.iters[c] = 0;
        k.outer[c] += 1;
        k.rn[c] = nr / k.nb[c];
        if (!isfinite(nr)) {
            k.status[c] = COL_BREAKDOWN;
        } else if (nr / k.nb[c] <= k.tol[c]) {
            k.status[c] = COL_PEND_CHECK;
        } else if (k.outer[c] >= k.max_outer || k.total_iters[c] >= k.maxit[c]) {
            k.status[c] = COL_NOCONV;
        } else {
            k.rscale[c] = nr;
            k.status[c] = COL_OUTER;
        }
    }
};

// X(:, c) += x_acc(:, c) and x_acc(:, c) = 0 (FOLD), or x_acc(:, c) = 0
// (ZERO), for the columns in cmask.
enum FoldKind : int32_t { FOLD_ADD = 0, FOLD_ZERO = 1 };

template <int M>
struct OpFold {
    using S = Shape<double, M>;
    static constexpr const char *kName = "fold";
    static constexpr int NDOT = 0;
    double *X;
    double *xacc;
    int32_t n;
    int32_t kind;
    uint32_t cmask;
    struct Lane {
        bool on;
        bool act[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        ln.on = false;
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            const int c = g * S::VW + q;
            ln.act[q] = c < M && ((cmask >> c) & 1u);
            ln.on = ln.on || ln.act[q];
        }
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<double, S::VW, NDOT> &) const
    {
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (!ln.act[q])
                continue;
            const int c = g * S::VW + q;
            double *a = xacc + static_cast<size_t>(c) * n + i;
            if (kind == FOLD_ADD) {
                double *xp = X + static_cast<size_t>(i) * M + c;
                *xp = *xp + *a;
            }
            *a = 0.0;
        }
    }
    __device__ void finish(const double *) const {}
};

// Admission of columns into a block: reset their control state.
struct SlotInit {
    double tol[kMaxM];
    int32_t maxit[kMaxM];
};

} // namespace mrhs
