// Classical AMG on the device: the hierarchy built by amg_setup.hip is
// uploaded once per matrix; a V-cycle for an n x m row-interleaved block runs
// level by level as products over the tile loops of core.h, so the m
// right-hand sides share every matrix read of every level; BiCGStab
// preconditioned by it (the paper's solver, Section 4.1) reuses the block
// engine's per-column control (ops.h).
//
// V-cycle at level l for right-hand side b (one l1-Jacobi sweep before and
// after the coarse correction, x = 0 at the start, D = D_l1):
//   r = b - (A D^-1) b          first sweep from x = 0 folded into A D^-1
//   b_c = R r                   restriction
//   x_c = V-cycle at level l+1  (the coarsest level applies its dense inverse)
//   t = D^-1 b + P x_c          first sweep's x plus the coarse correction
//   x = t + D^-1 (b - A t)      post-smoothing
// Four products per level, each reading its matrix once for all m columns.
//
// Preconditioned iteration (right preconditioning, M^-1 = V-cycle): for every
// running column
//   p^ = M^-1 p;  v = A p^;  sigma = (r^, v);  alpha = rho / sigma
//   s = r - alpha v;  s^ = M^-1 s;  t = A s^;  omega = (t, s) / (t, t)
//   x += alpha p^ + omega s^;  r = s - omega t;  p = r + beta (p - omega v)
// with the same fused dots, device-side scalars, stopping tests, true-residual
// checks and restarts as the Jacobi-preconditioned block solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "amg.h"
#include "dict.h"
#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {
namespace {

// Lanes on in a V-cycle product: every column (ctl null) or the running ones.
template <typename T, int M>
__device__ __forceinline__ bool lane_running(const Ctl *ctl, int g)
{
    using S = Shape<T, M>;
    if (!ctl)
        return true;
    bool on = false;
#pragma unroll
    for (int q = 0; q < S::VW; ++q) {
        const int c = g * S::VW + q;
        on = on || (c < M && ctl->status[c] == COL_RUN);
    }
    return on;
}

struct VcLane {
    bool on;
};

// The V-cycle runs in binary64, or in binary32 on binary32 roundings of
// every level's values (MRHS_MIXED with block_bicgstab_amg): the same ops
// over T.

// Y = sum (restriction, coarsest dense inverse)
template <typename T, int M>
struct OpVcStore {
    static constexpr const char *kName = "vc_store";
    static constexpr bool kLongRows = true;
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *X;
    T *Y;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<T, M>(ctl, g)}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const { ld<T, M>(X, c, g, x); }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const T *sum, Acc<T, S::VW, NDOT> &) const
    {
        st<T, M>(Y, i, g, sum);
    }
    __device__ void finish(const T *) const {}
};

// Y = U - sum (residual; with A D^-1 and X = U the residual after the first
// sweep from zero)
template <typename T, int M>
struct OpVcRes {
    static constexpr const char *kName = "vc_resid";
    static constexpr bool kLongRows = true;
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *X, *U;
    T *Y;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<T, M>(ctl, g)}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const { ld<T, M>(X, c, g, x); }
    struct Pre {
        T u[S::VW];
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<T, M>(U, i, g, pr.u);
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const T *sum, Acc<T, S::VW, NDOT> &,
                                        const Pre &pr) const
    {
        T u[S::VW];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            u[q] = pr.u[q] - sum[q];
        st<T, M>(Y, i, g, u);
    }
    __device__ void finish(const T *) const {}
};

// Y = dinv_i U_i + sum (the first sweep's x plus the prolongated correction)
template <typename T, int M>
struct OpVcProl {
    static constexpr const char *kName = "vc_prolong";
    static constexpr bool kLongRows = true;
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *X, *U, *dinv;
    T *Y;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<T, M>(ctl, g)}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const { ld<T, M>(X, c, g, x); }
    struct Pre {
        T u[S::VW];
        T d;
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<T, M>(U, i, g, pr.u);
        pr.d = dinv[i];
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const T *sum, Acc<T, S::VW, NDOT> &,
                                        const Pre &pr) const
    {
        T u[S::VW];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            u[q] = pr.d * pr.u[q] + sum[q];
        st<T, M>(Y, i, g, u);
    }
    __device__ void finish(const T *) const {}
};

// Y = T_i + dinv_i (U_i - sum), sum = (A T)_i (post-smoothing sweep)
template <typename T, int M>
struct OpVcSmooth {
    static constexpr const char *kName = "vc_smooth";
    static constexpr bool kLongRows = true;
    using S = Shape<T, M>;
    static constexpr int NDOT = 0;
    const T *Tv, *U, *dinv;
    T *Y;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<T, M>(ctl, g)}; }
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, T *x) const { ld<T, M>(Tv, c, g, x); }
    struct Pre {
        T t[S::VW], u[S::VW];
        T d;
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<T, M>(Tv, i, g, pr.t);
        ld<T, M>(U, i, g, pr.u);
        pr.d = dinv[i];
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, const T *sum, Acc<T, S::VW, NDOT> &,
                                        const Pre &pr) const
    {
        T t[S::VW];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            t[q] = pr.t[q] + pr.d * (pr.u[q] - sum[q]);
        st<T, M>(Y, i, g, t);
    }
    __device__ void finish(const T *) const {}
};

// Block conversions at the binary32 V-cycle's boundary, in the binary64 lane
// layout: dst = RN32(src) into a binary32 block, and back.
template <int M>
struct OpTo32 {
    static constexpr const char *kName = "amg_to32";
    using S = Shape<double, M>;
    static constexpr int NDOT = 0;
    const double *src;
    float *dst;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<double, M>(ctl, g)}; }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, Acc<double, S::VW, NDOT> &) const
    {
        double v[S::VW];
        float f[S::VW];
        ld<double, M>(src, i, g, v);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            f[q] = static_cast<float>(v[q]);
        Vec<float, S::VW>::store(dst + static_cast<size_t>(i) * M + g * S::VW, f);
    }
    __device__ void finish(const double *) const {}
};

template <int M>
struct OpTo64 {
    static constexpr const char *kName = "amg_to64";
    using S = Shape<double, M>;
    static constexpr int NDOT = 0;
    const float *src;
    double *dst;
    const Ctl *ctl;
    using Lane = VcLane;
    __device__ Lane lane(int g) const { return {lane_running<double, M>(ctl, g)}; }
    __device__ __forceinline__ void row(const Lane &, int32_t i, int g, Acc<double, S::VW, NDOT> &) const
    {
        float f[S::VW];
        double v[S::VW];
        Vec<float, S::VW>::load(src + static_cast<size_t>(i) * M + g * S::VW, f);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            v[q] = static_cast<double>(f[q]);
        st<double, M>(dst, i, g, v);
    }
    __device__ void finish(const double *) const {}
};

// s = r - alpha v for the running columns (the V-cycle's input)
template <int M>
struct OpSForm {
    static constexpr const char *kName = "amg_s";
    using S = Shape<double, M>;
    static constexpr int NDOT = 0;
    const double *r, *v;
    double *s;
    Ctl *ctl;
    Kry<double> *kry;
    int32_t ldp;  // row stride of r and v
    struct Lane {
        bool on;
        double alpha[S::VW];
    };
    __device__ Lane lane(int g) const
    {
        Lane ln;
        const RunLane<double, M> rl = run_lane<double, M>(ctl, g);
        ln.on = rl.on;
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            ln.alpha[q] = g * S::VW + q < M ? kry->alpha[g * S::VW + q] : 0.0;
        return ln;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<double, S::VW, NDOT> &) const
    {
        double rr[S::VW], vv[S::VW];
        ld<double, M>(r, i, g, rr, ldp);
        ld<double, M>(v, i, g, vv, ldp);
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            rr[q] = rr[q] - ln.alpha[q] * vv[q];
        st<double, M>(s, i, g, rr);
    }
    __device__ void finish(const double *) const {}
};

// t = A s^ with s^ = M^-1 s gathered, s read from its block; sums and the
// per-column decisions of the Jacobi iteration's omega pass.
template <int M>
struct OpSpmv2P : OpSpmv2<double, M> {
    static constexpr const char *kName = "amg_omega";
    static constexpr int GATHERED = 1;
    using Base = OpSpmv2<double, M>;
    using S = Shape<double, M>;
    using Lane = typename Base::Lane;
    const double *sh;  // M^-1 s, gathered
    const double *sv;  // s
    __device__ __forceinline__ void gather(const Lane &, int32_t c, int g, double *x) const { ld<double, M>(sh, c, g, x); }
    struct Pre {
        double s[S::VW];
    };
    __device__ __forceinline__ Pre pre(const Lane &, int32_t i, int g) const
    {
        Pre pr;
        ld<double, M>(sv, i, g, pr.s);
        return pr;
    }
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, const double *sum,
                                        Acc<double, S::VW, Base::NDOT> &acc, const Pre &pr) const
    {
        const double *s = pr.s;
        double h[S::VW];
        shadow_row<double, M>(nullptr, i, g, h);
        st<double, M>(this->t, i, g, sum);
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
};

// x += alpha p^ + omega s^;  r = s - omega t;  p = r + beta (p - omega v);
// sums (r^, r), (r, r); the per-column decisions of the Jacobi update pass.
template <int M>
struct OpXRP : OpXR<double, M> {
    static constexpr const char *kName = "amg_xr";
    using Base = OpXR<double, M>;
    using S = Shape<double, M>;
    using Lane = typename Base::Lane;
    const double *ph, *sh, *sv;
    __device__ __forceinline__ void row(const Lane &ln, int32_t i, int g, Acc<double, S::VW, Base::NDOT> &acc) const
    {
        double xx[S::VW], rr[S::VW], pp[S::VW], vv[S::VW], tt[S::VW], a[S::VW], b[S::VW], s[S::VW], hh[S::VW];
        ld<double, M>(this->y, i, g, xx);
        ld<double, M>(this->r, i, g, rr, this->ldp);
        ld<double, M>(this->p, i, g, pp);
        ld<double, M>(this->v, i, g, vv, this->ldp);
        ld<double, M>(this->t, i, g, tt);
        ld<double, M>(ph, i, g, a);
        ld<double, M>(sh, i, g, b);
        ld<double, M>(sv, i, g, s);
        shadow_row<double, M>(nullptr, i, g, hh);
#pragma unroll
        for (int q = 0; q < S::VW; ++q) {
            if (ln.act[q]) {
                rr[q] = s[q];
                if (ln.use_w[q]) {
                    xx[q] = xx[q] + (ln.alpha[q] * a[q] + ln.omega[q] * b[q]);
                    rr[q] = s[q] - ln.omega[q] * tt[q];
                    pp[q] = rr[q] + ln.beta[q] * (pp[q] - ln.omega[q] * vv[q]);
                } else {
                    xx[q] = xx[q] + ln.alpha[q] * a[q];
                }
                acc.a[0][q] += hh[q] * rr[q];
                acc.a[1][q] += rr[q] * rr[q];
            }
        }
        st<double, M>(this->y, i, g, xx);
        st<double, M>(this->r, i, g, rr, this->ldp);
        st<double, M>(this->p, i, g, pp);
    }
};

// ---- V-cycle buffers: for every level but the coarsest r_l and t_l, for
// every level but the finest b_l and x_l, each n_l x m of T; a binary32
// V-cycle also holds its finest level's b and x (the binary64 blocks
// rounded in, and the result before it is widened out).
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <typename T>
struct VcBufs {
    T *r[kAmgMaxLevels], *t[kAmgMaxLevels], *b[kAmgMaxLevels], *x[kAmgMaxLevels];
};

template <typename T>
size_t vc_layout(const AmgDev &H, int32_t m, char *base, VcBufs<T> *out)
{
    size_t off = 0;
    auto take = [&](int32_t n) {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off = align_up(off + sizeof(T) * static_cast<size_t>(n) * m);
        return p;
    };
    VcBufs<T> v{};
    for (int l = 0; l < H.nlev; ++l) {
        const int32_t n = H.lev[l].n;
        if (l + 1 < H.nlev) {
            v.r[l] = take(n);
            v.t[l] = take(n);
        }
        if (l > 0 || !std::is_same<T, double>::value) {
            v.b[l] = take(n);
            v.x[l] = take(n);
        }
    }
    if (out)
        *out = v;
    return off;
}

// The level arrays of the V-cycle's precision.
template <typename T>
struct VcViews;
template <>
struct VcViews<double> {
    static const CsrView<double> &A(const AmgLevelDev &l) { return l.A; }
    static const CsrView<double> &Ah(const AmgLevelDev &l) { return l.Ah; }
    static const CsrView<double> &P(const AmgLevelDev &l) { return l.P; }
    static const CsrView<double> &R(const AmgLevelDev &l) { return l.R; }
    static const double *dinv(const AmgLevelDev &l) { return l.dl1_inv; }
    static const CsrView<double> &cinv(const AmgDev &H) { return H.cinv; }
};
template <>
struct VcViews<float> {
    static const CsrView<float> &A(const AmgLevelDev &l) { return l.A32; }
    static const CsrView<float> &Ah(const AmgLevelDev &l) { return l.Ah32; }
    static const CsrView<float> &P(const AmgLevelDev &l) { return l.P32; }
    static const CsrView<float> &R(const AmgLevelDev &l) { return l.R32; }
    static const float *dinv(const AmgLevelDev &l) { return l.dl1_inv32; }
    static const CsrView<float> &cinv(const AmgDev &H) { return H.cinv32; }
};

// x = V-cycle(b) on blocks of T; b and x are the finest level's blocks
template <typename T, int M>
hipError_t vcycle(const AmgDev &H, const T *b, T *x, const VcBufs<T> &vb, const Ctl *ctl, hipStream_t s)
{
    using V = VcViews<T>;
    VcBufs<T> v = vb;
    const RedBufs<T> none{nullptr, nullptr, nullptr};
    const int L = H.nlev;
    v.b[0] = const_cast<T *>(b);
    v.x[0] = x;
    hipError_t e;
    for (int l = 0; l + 1 < L; ++l) {
        const AmgLevelDev &lv = H.lev[l];
        if ((e = launch_gspmv<T, M>(V::Ah(lv), OpVcRes<T, M>{v.b[l], v.b[l], v.r[l], ctl}, none, s)) != hipSuccess)
            return e;
        if ((e = launch_gspmv<T, M>(V::R(lv), OpVcStore<T, M>{v.r[l], v.b[l + 1], ctl}, none, s)) != hipSuccess)
            return e;
    }
    if ((e = launch_gspmv<T, M>(V::cinv(H), OpVcStore<T, M>{v.b[L - 1], v.x[L - 1], ctl}, none, s)) != hipSuccess)
        return e;
    for (int l = L - 2; l >= 0; --l) {
        const AmgLevelDev &lv = H.lev[l];
        if ((e = launch_gspmv<T, M>(V::P(lv), OpVcProl<T, M>{v.x[l + 1], v.b[l], V::dinv(lv), v.t[l], ctl}, none,
                                    s)) != hipSuccess)
            return e;
        if ((e = launch_gspmv<T, M>(V::A(lv), OpVcSmooth<T, M>{v.t[l], v.b[l], V::dinv(lv), v.x[l], ctl}, none,
                                    s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// x = M^-1 b for binary64 blocks, the V-cycle in binary64 or (vc32) in
// binary32 between a rounding of b and a widening of its result
template <int M>
hipError_t precondition(const AmgDev &H, const double *b, double *x, char *ws, bool vc32, const Ctl *ctl,
                        hipStream_t s)
{
    if (!vc32) {
        VcBufs<double> v;
        vc_layout<double>(H, M, ws, &v);
        return vcycle<double, M>(H, b, x, v, ctl, s);
    }
    VcBufs<float> v;
    vc_layout<float>(H, M, ws, &v);
    const RedBufs<double> none{nullptr, nullptr, nullptr};
    const int32_t n = H.lev[0].n;
    hipError_t e;
    if ((e = launch_stream<double, M>(n, OpTo32<M>{b, v.b[0], ctl}, none, s)) != hipSuccess)
        return e;
    if ((e = vcycle<float, M>(H, v.b[0], v.x[0], v, ctl, s)) != hipSuccess)
        return e;
    return launch_stream<double, M>(n, OpTo64<M>{v.x[0], x, ctl}, none, s);
}

#define AMG_TRY(expr)           \
    do {                        \
        hipError_t e_ = (expr); \
        if (e_ != hipSuccess)   \
            return e_;          \
    } while (0)

template <int M>
struct AmgSteps {
    static CsrView<double> A(const Ctx &c) { return c.amg->lev[0].A; }
    static hipError_t start(Ctx &c, uint32_t cmask, bool x0)
    {
        if (!x0)
            AMG_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_ZERO, cmask}, c.rb64, c.s)));
        return launch_gspmv<double, M>(A(c), OpResid<M>{c.X, c.B, c.r, c.p, nullptr, c.ctl, c.kry64, RES_SETUP, 0u, 0, c.ldp64},
                                       c.rb64, c.s);
    }
    static hipError_t iterate(Ctx &c, int k)
    {
        for (int it = 0; it < k; ++it) {
            AMG_TRY(precondition<M>(*c.amg, c.p, c.ph, c.vcws, c.vc32, c.ctl, c.s));
            AMG_TRY((launch_gspmv<double, M>(A(c), OpSpmv1<double, M>{c.ph, c.v, nullptr, c.ctl, c.kry64, c.ldp64},
                                              c.rb64, c.s)));
            AMG_TRY((launch_stream<double, M>(c.n, OpSForm<M>{c.r, c.v, c.sv, c.ctl, c.kry64, c.ldp64}, c.rb64, c.s)));
            AMG_TRY(precondition<M>(*c.amg, c.sv, c.sh, c.vcws, c.vc32, c.ctl, c.s));
            OpSpmv2P<M> om{};
            om.r = c.r;
            om.v = c.v;
            om.sgn = nullptr;
            om.t = c.t;
            om.ctl = c.ctl;
            om.kry = c.kry64;
            om.ldp = c.ldp64;
            om.sh = c.sh;
            om.sv = c.sv;
            AMG_TRY((launch_gspmv<double, M>(A(c), om, c.rb64, c.s)));
            OpXRP<M> up{};
            up.y = c.X;
            up.r = c.r;
            up.p = c.p;
            up.v = c.v;
            up.t = c.t;
            up.sgn = nullptr;
            up.ctl = c.ctl;
            up.kry = c.kry64;
            up.ldp = c.ldp64;
            up.ph = c.ph;
            up.sh = c.sh;
            up.sv = c.sv;
            AMG_TRY((launch_stream<double, M>(c.n, up, c.rb64, c.s)));
        }
        return hipSuccess;
    }
    static hipError_t check(Ctx &c)
    {
        AMG_TRY((launch_gspmv<double, M>(A(c), OpResid<M>{c.X, c.B, c.t, nullptr, nullptr, c.ctl, c.kry64, RES_CHECK, 0u},
                                          c.rb64, c.s)));
        return launch_stream<double, M>(c.n, OpRestart<double, M>{c.t, c.r, c.p, c.ctl, c.ldp64}, c.rb64, c.s);
    }
    static hipError_t finish(Ctx &c, uint32_t cmask, bool nullspace)
    {
        AMG_TRY((launch_stream<double, M>(
            c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_FIX_ZERO, cmask}, c.rb64, c.s)));
        if (nullspace) {
            AMG_TRY((launch_stream<double, M>(c.n, OpColSum<M>{c.X, c.ctl, cmask}, c.rb64, c.s)));
            AMG_TRY((launch_stream<double, M>(
                c.n, OpScale<M>{c.X, c.A->diag, c.A->dinv, c.ctl, SC_SUB_MEAN, cmask}, c.rb64, c.s)));
        }
        return launch_gspmv<double, M>(A(c), OpResid<M>{c.X, c.B, nullptr, nullptr, nullptr, c.ctl, c.kry64, RES_FINAL, cmask},
                                       c.rb64, c.s);
    }
};

struct MakeAmgTable {
    template <int M>
    AmgStepTable operator()() const
    {
        return {&AmgSteps<M>::start, &AmgSteps<M>::iterate, &AmgSteps<M>::check, &AmgSteps<M>::finish};
    }
};

struct VcLaunch {
    const AmgDev *H;
    const double *b;
    double *x;
    char *ws;
    hipStream_t s;
    template <int M>
    hipError_t operator()() const
    {
        return precondition<M>(*H, b, x, ws, false, nullptr, s);
    }
};

} // namespace

const AmgStepTable &amg_table(int m)
{
    static const AmgStepTable tables[kMaxM + 1] = {
        {},
        MakeAmgTable{}.operator()<1>(),  MakeAmgTable{}.operator()<2>(),  MakeAmgTable{}.operator()<3>(),
        MakeAmgTable{}.operator()<4>(),  MakeAmgTable{}.operator()<5>(),  MakeAmgTable{}.operator()<6>(),
        MakeAmgTable{}.operator()<7>(),  MakeAmgTable{}.operator()<8>(),  MakeAmgTable{}.operator()<9>(),
        MakeAmgTable{}.operator()<10>(), MakeAmgTable{}.operator()<11>(), MakeAmgTable{}.operator()<12>(),
        MakeAmgTable{}.operator()<13>(), MakeAmgTable{}.operator()<14>(), MakeAmgTable{}.operator()<15>(),
        MakeAmgTable{}.operator()<16>(),
    };
    return tables[m];
}

size_t amg_vcycle_bytes(const AmgDev &H, int32_t m)
{
    return std::max(vc_layout<double>(H, m, nullptr, nullptr), vc_layout<float>(H, m, nullptr, nullptr));
}

} // namespace mrhs

// ---- the hierarchy handle ---------------------------------------------------
struct mrhs_amg_s {
    mrhs_csr A = nullptr;
    int device = 0;
    mrhs::AmgDev dev;
    std::mutex mu32;  // serializes the one-time binary32 rounding (amg_make32)
    std::vector<std::vector<int8_t>> cf;  // C/F marks of every level but the coarsest
    std::vector<void *> allocs;
    size_t bytes = 0;
    double op_complexity = 0.0;
};

namespace mrhs {
namespace {

// workspace of one amg_vcycle call: the V-cycle's, plus renumbered copies of
// B and X when the matrix was renumbered
size_t vcycle_call_bytes(const mrhs_amg_s &H, int32_t m)
{
    const size_t v = amg_vcycle_bytes(H.dev, m);
    return H.A->perm ? align_up(v) + 2 * padded_block_bytes(H.A->n, m) : v;
}

constexpr size_t kPadElems = 4;  // zero padding past the nonzeros (whole-vector tile loads)

template <typename T>
T *upload(mrhs_amg_s *H, const T *src, size_t count, size_t pad, hipError_t *err)
{
    void *p = nullptr;
    const size_t bytes = sizeof(T) * (count + pad);
    if (*err != hipSuccess)
        return nullptr;
    if ((*err = hipMalloc(&p, std::max<size_t>(bytes, sizeof(T)))) != hipSuccess)
        return nullptr;
    H->allocs.push_back(p);
    H->bytes += bytes;
    if (pad && (*err = hipMemset(static_cast<T *>(p) + count, 0, sizeof(T) * pad)) != hipSuccess)
        return nullptr;
    if (count && (*err = hipMemcpy(p, src, sizeof(T) * count, hipMemcpyHostToDevice)) != hipSuccess)
        return nullptr;
    return static_cast<T *>(p);
}

int32_t median_reach(const amg::HostCsr &A)
{
    if (A.nr == 0)
        return 0;
    std::vector<int32_t> reach(A.nr, 0);
    for (int32_t i = 0; i < A.nr; ++i)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            reach[i] = std::max(reach[i], A.ci[k] - i);
    std::nth_element(reach.begin(), reach.begin() + A.nr / 2, reach.end());
    return reach[A.nr / 2];
}

// Small levels with long rows (the coarse Galerkin levels, 30-90 nonzeros
// per row, and the coarsest dense inverse) take the one-wave-per-row product:
// the tiled one would run them on a few workgroups with long serial row
// chains.  Large levels keep the tiled product: with ~15 nonzeros per row one
// row per wave leaves most gather slots empty (measured on the 12.6M-row
// channel's first coarse level, 6.3M rows: 1070 -> 1371 us per sweep).
constexpr double kSplitRowNnz = 12.0;
constexpr int32_t kSplitMaxRows = 131072;

CsrView<double> upload_csr(mrhs_amg_s *H, const amg::HostCsr &C, const std::vector<double> *vals, int32_t reach,
                           hipError_t *err)
{
    CsrView<double> v{};
    v.rp = upload(H, C.rp.data(), C.rp.size(), 0, err);
    v.ci = upload(H, C.ci.data(), C.ci.size(), kPadElems, err);
    v.va = upload(H, (vals ? vals : &C.va)->data(), C.va.size(), kPadElems, err);
    v.n = C.nr;
    v.reach = reach;
    v.split = C.nr > 0 && C.nr < kSplitMaxRows && static_cast<double>(C.nnz()) >= kSplitRowNnz * C.nr;
    return v;
}

// The dictionary form (16-bit or column codes, value table) of a level
// operator's binary64 view v with values vals, when it has one; otab: the
// level's offset table on the device (16-bit codes).  The binary32 views
// made later read the plain arrays.
void attach_dict(mrhs_amg_s *H, const amg::HostCsr &C, const std::vector<double> &vals, const dict::Offsets &offs,
                 const int32_t *otab, CsrView<double> &v, hipError_t *err)
{
    if (*err != hipSuccess)
        return;
    const dict::Codes<double> c = dict::codes<double>(C.nr, C.nnz(), C.rp.data(), C.ci.data(), vals.data(), offs);
    if (!c.ok)
        return;
    const double *tab = upload(H, c.tab.data(), c.tab.size(), 0, err);
    if (offs.ok) {
        const uint16_t *code = upload(H, c.code.data(), c.code.size(), 0, err);
        if (*err != hipSuccess)
            return;
        v.code = code;
        v.otab = otab;
        v.noffs = static_cast<int32_t>(offs.set.keys.size());
        v.ob = offs.ob;
    } else {
        const uint32_t *ccode = upload(H, c.ccode.data(), c.ccode.size(), 0, err);
        if (*err != hipSuccess)
            return;
        v.ccode = ccode;
        v.cb = c.cb;
    }
    v.vtab = tab;
    v.nvals = static_cast<int32_t>(c.tab.size());
}

void free_amg(mrhs_amg_s *H)
{
    if (!H)
        return;
    for (void *p : H->allocs)
        (void)hipFree(p);
    delete H;
}

__global__ void k_round32(const double *__restrict__ src, float *__restrict__ dst, int64_t count)
{
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[k] = static_cast<float>(src[k]);
}

// binary32 rounding (nearest even) of count device values, padding included
float *round32(mrhs_amg_s *H, const double *src, int64_t count, hipError_t *err)
{
    void *p = nullptr;
    if (*err != hipSuccess)
        return nullptr;
    const size_t bytes = sizeof(float) * static_cast<size_t>(std::max<int64_t>(count, 1));
    if ((*err = hipMalloc(&p, bytes)) != hipSuccess)
        return nullptr;
    H->allocs.push_back(p);
    H->bytes += bytes;
    if (count > 0) {
        const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
        hipLaunchKernelGGL(k_round32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, nullptr, src,
                           static_cast<float *>(p), count);
        *err = hipGetLastError();
    }
    return static_cast<float *>(p);
}

// The binary32 view of a level operator: its values rounded (nearest even);
// a binary64 dictionary form carries over with its value table rounded the
// same way (equal values round alike, so each entry's code still names its
// rounded value; the table may then hold repeats).
CsrView<float> view32(mrhs_amg_s *H, const CsrView<double> &v, int64_t nnz, hipError_t *err)
{
    CsrView<float> w{v.rp, v.ci, round32(H, v.va, nnz + static_cast<int64_t>(kPadElems), err), v.n, v.reach, v.split};
    if (v.vtab && *err == hipSuccess) {
        const float *tab = round32(H, v.vtab, v.nvals, err);
        if (*err == hipSuccess) {
            w.vtab = tab;
            w.nvals = v.nvals;
            w.code = v.code;
            w.otab = v.otab;
            w.noffs = v.noffs;
            w.ob = v.ob;
            w.ccode = v.ccode;
            w.cb = v.cb;
        }
    }
    return w;
}

} // namespace

const AmgDev *amg_dev_of(mrhs_amg H) { return &H->dev; }
size_t amg_bytes_of(mrhs_amg H) { return H->bytes; }

mrhs_status amg_make32(mrhs_amg H)
{
    std::lock_guard<std::mutex> lk(H->mu32);
    if (H->dev.has32)
        return MRHS_OK;
    (void)hipSetDevice(H->device);
    hipError_t e = hipSuccess;
    AmgDev &D = H->dev;
    const int L = D.nlev;
    for (int l = 0; l < L && e == hipSuccess; ++l) {
        AmgLevelDev &d = D.lev[l];
        d.A32 = view32(H, d.A, d.nnz_a, &e);
        d.dl1_inv32 = round32(H, d.dl1_inv, d.n, &e);
        if (l + 1 < L) {
            d.Ah32 = view32(H, d.Ah, d.nnz_a, &e);
            d.P32 = view32(H, d.P, d.nnz_p, &e);
            d.R32 = view32(H, d.R, d.nnz_p, &e);
        }
    }
    const int64_t nc = D.lev[L - 1].n;
    D.cinv32 = view32(H, D.cinv, nc * nc, &e);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? MRHS_ENOMEM : MRHS_EDEVICE, "binary32 hierarchy failed: %s",
                         hipGetErrorString(e));
    }
    D.has32 = true;
    return MRHS_OK;
}

} // namespace mrhs

using namespace mrhs;

MRHS_API mrhs_status amg_create(mrhs_csr A, double theta, int32_t max_coarse, int32_t max_levels, mrhs_amg *out)
{
    clear_error();
    if (!out)
        return set_error(MRHS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A)
        return set_error(MRHS_EINVAL, "matrix handle is NULL");
    if (A->n == 0)
        return set_error(MRHS_EINVAL, "empty matrix");
    if (A->zero_diag)
        return set_error(MRHS_EINVAL, "the matrix has a zero diagonal entry");
    amg::Params prm;
    if (theta > 0.0) {
        if (!(theta < 1.0))
            return set_error(MRHS_EINVAL, "theta = %g outside (0, 1)", theta);
        prm.theta = theta;
    }
    if (max_coarse > 0)
        prm.max_coarse = max_coarse;
    if (max_levels > 0)
        prm.max_levels = std::min(max_levels, kAmgMaxLevels);
    // the matrix as uploaded (host copy for the setup)
    const int32_t n = A->n;
    std::vector<int32_t> rp(static_cast<size_t>(n) + 1), ci(static_cast<size_t>(A->nnz));
    std::vector<double> va(static_cast<size_t>(A->nnz));
    hipError_t e = hipSuccess;
    if ((e = hipMemcpy(rp.data(), A->rp, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
        (A->nnz && (e = hipMemcpy(ci.data(), A->ci, sizeof(int32_t) * ci.size(), hipMemcpyDeviceToHost)) != hipSuccess) ||
        (A->nnz && (e = hipMemcpy(va.data(), A->val, sizeof(double) * va.size(), hipMemcpyDeviceToHost)) != hipSuccess))
        return set_error(MRHS_EDEVICE, "matrix download failed: %s", hipGetErrorString(e));
    amg::HostHierarchy HH;
    const char *why = nullptr;
    if (!amg::setup(n, rp.data(), ci.data(), va.data(), (A->flags & MRHS_CSR_NULLSPACE_CONST) != 0, prm, &HH, &why))
        return set_error(MRHS_EINVAL, "%s", why ? why : "AMG setup failed");
    rp.clear();
    ci.clear();
    va.clear();
    auto *H = new (std::nothrow) mrhs_amg_s();
    if (!H)
        return set_error(MRHS_ENOMEM, "host allocation failed");
    H->A = A;
    H->device = A->device;
    const bool use_dict = env_int("MRHS_CSR_DICT", 1, 0, 1) != 0;
    const int L = static_cast<int>(HH.levels.size());
    H->dev.nlev = L;
    int64_t nz_all = 0;
    for (int l = 0; l < L; ++l) {
        const amg::HostLevel &hl = HH.levels[l];
        AmgLevelDev &d = H->dev.lev[l];
        d.n = hl.A.nr;
        d.nnz_a = hl.A.nnz();
        nz_all += d.nnz_a;
        const int32_t reach = median_reach(hl.A);
        d.A = upload_csr(H, hl.A, nullptr, reach, &e);
        d.dl1_inv = upload(H, hl.dl1_inv.data(), hl.dl1_inv.size(), 0, &e);
        std::vector<double> vah;
        if (l + 1 < L) {
            vah.resize(hl.A.va.size());
            for (int32_t i = 0; i < hl.A.nr; ++i)
                for (int32_t k = hl.A.rp[i]; k < hl.A.rp[i + 1]; ++k)
                    vah[k] = hl.A.va[k] * hl.dl1_inv[hl.A.ci[k]];
            d.Ah = upload_csr(H, hl.A, &vah, reach, &e);
            d.P = upload_csr(H, hl.P, nullptr, 0, &e);
            d.R = upload_csr(H, hl.R, nullptr, 0, &e);
            d.nnext = hl.P.nc;
            d.nnz_p = hl.P.nnz();
            H->cf.push_back(hl.cf);
        }
        // the tiled products of A_l and A_l D_l1^-1 read codes where the
        // level's operator has a dictionary form (MRHS_CSR_DICT=0: never)
        if (use_dict && !d.A.split && hl.A.nnz() > 0 && e == hipSuccess) {
            dict::Offsets offs;
            dict::offsets(hl.A.nr, hl.A.rp.data(), hl.A.ci.data(), offs);
            std::vector<int32_t> otab(offs.set.keys.begin(), offs.set.keys.end());
            const int32_t *dotab = offs.ok ? upload(H, otab.data(), otab.size(), 0, &e) : nullptr;
            attach_dict(H, hl.A, hl.A.va, offs, dotab, d.A, &e);
            if (l + 1 < L)
                attach_dict(H, hl.A, vah, offs, dotab, d.Ah, &e);
        }
        if (e != hipSuccess)
            break;
    }
    if (e == hipSuccess) {
        const int32_t nc = HH.levels.back().A.nr;
        amg::HostCsr C;
        C.nr = C.nc = nc;
        C.rp.resize(static_cast<size_t>(nc) + 1);
        C.ci.resize(static_cast<size_t>(nc) * nc);
        for (int32_t i = 0; i <= nc; ++i)
            C.rp[i] = i * nc;
        for (int32_t i = 0; i < nc; ++i)
            for (int32_t j = 0; j < nc; ++j)
                C.ci[static_cast<size_t>(i) * nc + j] = j;
        C.va = HH.coarse_inv;
        H->dev.cinv = upload_csr(H, C, nullptr, 0, &e);
    }
    if (e != hipSuccess) {
        free_amg(H);
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? MRHS_ENOMEM : MRHS_EDEVICE, "AMG upload failed: %s",
                         hipGetErrorString(e));
    }
    H->op_complexity = static_cast<double>(nz_all) / static_cast<double>(std::max<int64_t>(HH.levels[0].A.nnz(), 1));
    *out = H;
    return MRHS_OK;
}

MRHS_API mrhs_status amg_destroy(mrhs_amg H)
{
    clear_error();
    if (H) {
        (void)hipDeviceSynchronize();
        free_amg(H);
    }
    return MRHS_OK;
}

MRHS_API mrhs_status amg_info(mrhs_amg H, int32_t *levels, double *operator_complexity, size_t *device_bytes)
{
    clear_error();
    if (!H)
        return set_error(MRHS_EINVAL, "AMG handle is NULL");
    if (levels)
        *levels = H->dev.nlev;
    if (operator_complexity)
        *operator_complexity = H->op_complexity;
    if (device_bytes)
        *device_bytes = H->bytes;
    return MRHS_OK;
}

MRHS_API mrhs_status amg_level(mrhs_amg H, int32_t level, int32_t *rows, int64_t *nnz_a, int64_t *nnz_p)
{
    clear_error();
    if (!H)
        return set_error(MRHS_EINVAL, "AMG handle is NULL");
    if (level < 0 || level >= H->dev.nlev)
        return set_error(MRHS_EINVAL, "level %d outside [0, %d)", level, H->dev.nlev);
    const AmgLevelDev &d = H->dev.lev[level];
    if (rows)
        *rows = d.n;
    if (nnz_a)
        *nnz_a = d.nnz_a;
    if (nnz_p)
        *nnz_p = d.nnz_p;
    return MRHS_OK;
}

MRHS_API mrhs_status amg_level_copy(mrhs_amg H, int32_t level, int32_t what, int32_t *row_ptr, int32_t *col,
                                    double *val)
{
    clear_error();
    if (!H)
        return set_error(MRHS_EINVAL, "AMG handle is NULL");
    if (level < 0 || level >= H->dev.nlev)
        return set_error(MRHS_EINVAL, "level %d outside [0, %d)", level, H->dev.nlev);
    const AmgLevelDev &d = H->dev.lev[level];
    const bool coarsest = level == H->dev.nlev - 1;
    if (what == MRHS_AMG_SPLIT) {
        if (coarsest)
            return set_error(MRHS_EINVAL, "the coarsest level has no C/F splitting");
        if (!col)
            return set_error(MRHS_EINVAL, "col is NULL");
        const std::vector<int8_t> &cf = H->cf[level];
        for (int32_t i = 0; i < d.n; ++i)
            col[i] = cf[i];
        return MRHS_OK;
    }
    if (what != MRHS_AMG_OPERATOR && what != MRHS_AMG_PROLONGATION)
        return set_error(MRHS_EINVAL, "unknown part %d", what);
    if (what == MRHS_AMG_PROLONGATION && coarsest)
        return set_error(MRHS_EINVAL, "the coarsest level has no prolongation");
    if (!row_ptr || !col || !val)
        return set_error(MRHS_EINVAL, "NULL output array");
    const CsrView<double> &v = what == MRHS_AMG_OPERATOR ? d.A : d.P;
    const int64_t nnz = what == MRHS_AMG_OPERATOR ? d.nnz_a : d.nnz_p;
    hipError_t e = hipSuccess;
    if ((e = hipMemcpy(row_ptr, v.rp, sizeof(int32_t) * (static_cast<size_t>(d.n) + 1), hipMemcpyDeviceToHost)) !=
            hipSuccess ||
        (nnz && (e = hipMemcpy(col, v.ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (nnz && (e = hipMemcpy(val, v.va, sizeof(double) * nnz, hipMemcpyDeviceToHost)) != hipSuccess))
        return set_error(MRHS_EDEVICE, "copy failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}

MRHS_API mrhs_status amg_vcycle_workspace_size(mrhs_amg H, int32_t m, size_t *bytes)
{
    clear_error();
    if (!H || !bytes)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    *bytes = vcycle_call_bytes(*H, m);
    return MRHS_OK;
}

MRHS_API mrhs_status amg_vcycle(mrhs_amg H, const double *B, double *X, int32_t m, void *workspace, size_t ws_bytes,
                                void *hip_stream)
{
    clear_error();
    if (!H)
        return set_error(MRHS_EINVAL, "AMG handle is NULL");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    if (!B || !X)
        return set_error(MRHS_EINVAL, "B or X is NULL");
    const size_t need = vcycle_call_bytes(*H, m);
    if (need && (!workspace || ws_bytes < need))
        return set_error(MRHS_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    const size_t blk = sizeof(double) * static_cast<size_t>(H->dev.lev[0].n) * m;
    const uintptr_t b = reinterpret_cast<uintptr_t>(B), x = reinterpret_cast<uintptr_t>(X),
                    w = reinterpret_cast<uintptr_t>(workspace);
    if ((b < x + blk && x < b + blk) || (need && ((w < b + blk && b < w + need) || (w < x + blk && x < w + need))))
        return set_error(MRHS_EINVAL, "B, X and the workspace must not overlap");
    if ((b & 15u) || (x & 15u) || (w & 15u))
        return set_error(MRHS_EINVAL, "B, X and the workspace must be 16-byte aligned");
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t *perm = H->A->perm;
    hipError_t e = hipSuccess;
    if (perm) {  // the hierarchy is of the renumbered matrix: renumber B in, X out
        char *tail = static_cast<char *>(workspace) + align_up(amg_vcycle_bytes(H->dev, m));
        double *Bp = reinterpret_cast<double *>(tail);
        double *Xp = reinterpret_cast<double *>(tail + padded_block_bytes(H->A->n, m));
        if ((e = to_solver(Bp, B, perm, H->A->n, m, m, s)) == hipSuccess &&
            (e = dispatch_m(m, VcLaunch{&H->dev, Bp, Xp, static_cast<char *>(workspace), s})) == hipSuccess)
            e = to_user(X, Xp, perm, H->A->n, m, m, s);
    } else {
        e = dispatch_m(m, VcLaunch{&H->dev, B, X, static_cast<char *>(workspace), s});
    }
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "V-cycle launch failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}

MRHS_API mrhs_status block_bicgstab_amg_workspace_size(mrhs_amg H, int32_t m, size_t *bytes)
{
    clear_error();
    if (!H || !bytes)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    *bytes = solve_workspace_bytes(*H->A, m, 0u, &H->dev);
    return MRHS_OK;
}

MRHS_API mrhs_status block_bicgstab_amg(mrhs_amg H, const double *B, double *X, int32_t m, double tol, int32_t maxit,
                                        uint32_t flags, void *workspace, size_t ws_bytes, void *hip_stream,
                                        mrhs_col_info *info)
{
    clear_error();
    if (!H)
        return set_error(MRHS_EINVAL, "AMG handle is NULL");
    const mrhs_csr_s &A = *H->A;
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    if (!(tol > 0.0) || !std::isfinite(tol))
        return set_error(MRHS_EINVAL, "tol must be positive and finite");
    if (maxit < 1)
        return set_error(MRHS_EINVAL, "maxit must be at least 1");
    if (flags & ~(MRHS_X0_GIVEN | MRHS_MIXED))
        return set_error(MRHS_EINVAL, "unknown flags 0x%x", flags);
    if (!B || !X)
        return set_error(MRHS_EINVAL, "B or X is NULL");
    const size_t blk = static_cast<size_t>(A.n) * m * sizeof(double);
    const uintptr_t b = reinterpret_cast<uintptr_t>(B), x = reinterpret_cast<uintptr_t>(X),
                    w = reinterpret_cast<uintptr_t>(workspace);
    if (b < x + blk && x < b + blk)
        return set_error(MRHS_EINVAL, "B and X overlap");
    if (workspace && ((w < b + blk && b < w + ws_bytes) || (w < x + blk && x < w + ws_bytes)))
        return set_error(MRHS_EINVAL, "the workspace overlaps B or X");
    if ((b & 15u) || (x & 15u) || (w & 15u))
        return set_error(MRHS_EINVAL, "B, X and the workspace must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t need = solve_workspace_bytes(A, m, 0u, &H->dev);
    void *ws = workspace;
    bool own = false;
    if (!ws) {
        if (hipMalloc(&ws, need) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(MRHS_ENOMEM, "workspace allocation of %zu bytes failed", need);
        }
        own = true;
        ws_bytes = need;
    }
    mrhs_status st = MRHS_OK;
    if (flags & MRHS_MIXED)
        st = amg_make32(H);
    const uint32_t sflags = (flags & MRHS_X0_GIVEN) | ((flags & MRHS_MIXED) ? kAmgVc32 : 0u);
    if (st == MRHS_OK)
        st = block_solve(A, B, X, SolveParams{m, tol, maxit, sflags}, ws, ws_bytes, s, info, nullptr, &H->dev);
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
    }
    return st;
}
