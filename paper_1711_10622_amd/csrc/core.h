// Device building blocks shared by every kernel of the library (gfx950).
//
// Work decomposition.  Rows are cut into tiles of kTileRows consecutive rows.
// A workgroup of kBlock = 256 threads (four 64-wide waves) owns a strided set
// of tiles.  The grid is a multiple of kGroups = 8 and workgroup b belongs to
// group b % 8 (the hardware deals workgroups round-robin to the 8 XCDs, so a
// group is one XCD); group x owns the x-th eighth of the tiles, so each XCD
// streams one contiguous stretch of rows and its L2 holds the neighbours'
// block rows that the gather needs.
//
// Lane layout for an n x M row-interleaved block.  Each lane handles VW
// consecutive columns of one row (VW elements = one 8- or 16-byte access), a
// row takes G = M/VW lanes padded to L = next power of two, and a wave holds
// 64/L rows.  A wave-wide access of a block therefore covers 64/L whole rows,
// i.e. contiguous memory.
//
// Reductions (per-column dot products) are deterministic: lanes of one column
// are combined by a fixed xor butterfly inside the wave, waves in fixed order
// inside the workgroup, workgroups of a group by the group's last workgroup in
// fixed order, and the 8 groups by the overall last workgroup in fixed order.
// "Last" is decided by integer tickets; no floating-point atomics are used, so
// every run gives bitwise identical results.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace mrhs {

constexpr int kBlock = 256;
constexpr int kTileRows = 256;
constexpr int kNzCap = 2048;  // staged nonzeros per tile (8 per row on average)
constexpr int kGroups = 8;
constexpr int kMaxM = 16;
constexpr int kMaxDots = 3;

constexpr int next_pow2(int x) { return x <= 1 ? 1 : 2 * next_pow2((x + 1) / 2); }

template <typename T, int M>
struct Shape {
    static constexpr int VW = std::is_same<T, double>::value ? (M % 2 == 0 ? 2 : 1)
                                                             : (M % 4 == 0 ? 4 : (M % 2 == 0 ? 2 : 1));
    static constexpr int G = M / VW;       // lanes that hold data in a row
    static constexpr int L = next_pow2(G); // lanes per row
    static constexpr int RPP = kBlock / L; // rows per pass of the workgroup
    static constexpr int PASSES = kTileRows / RPP;
    static_assert(G * VW == M, "lane width must divide M");
    static_assert(L <= 64, "a row must fit one wave");
};

// ---- 8/16-byte vector access ------------------------------------------------
template <typename T, int VW>
struct Vec;

template <typename T>
struct Vec<T, 1> {
    static __device__ __forceinline__ void load(const T *p, T *v) { v[0] = *p; }
    static __device__ __forceinline__ void store(T *p, const T *v) { *p = v[0]; }
};

template <>
struct Vec<double, 2> {
    typedef double v2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ void load(const double *p, double *v)
    {
        v2 t = *reinterpret_cast<const v2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
    static __device__ __forceinline__ void store(double *p, const double *v)
    {
        v2 t;
        t.x = v[0];
        t.y = v[1];
        *reinterpret_cast<v2 *>(p) = t;
    }
};

template <>
struct Vec<float, 2> {
    typedef float v2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ void load(const float *p, float *v)
    {
        v2 t = *reinterpret_cast<const v2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
    static __device__ __forceinline__ void store(float *p, const float *v)
    {
        v2 t;
        t.x = v[0];
        t.y = v[1];
        *reinterpret_cast<v2 *>(p) = t;
    }
};

template <>
struct Vec<float, 4> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ void load(const float *p, float *v)
    {
        v4 t = *reinterpret_cast<const v4 *>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
    static __device__ __forceinline__ void store(float *p, const float *v)
    {
        v4 t;
        t.x = v[0];
        t.y = v[1];
        t.z = v[2];
        t.w = v[3];
        *reinterpret_cast<v4 *>(p) = t;
    }
};

// ---- tile schedule ------------------------------------------------------------
struct TileRange {
    int64_t first, end, stride;
};

__device__ __forceinline__ TileRange tile_range(int64_t ntiles)
{
    const int b = blockIdx.x;
    const int grp = b % kGroups;
    const int q = b / kGroups;
    const int gx = gridDim.x / kGroups;
    const int64_t lo = ntiles * grp / kGroups;
    const int64_t hi = ntiles * (grp + 1) / kGroups;
    return {lo + q, hi, gx};
}

// ---- matrix view ----------------------------------------------------------------
template <typename T>
struct CsrView {
    const int32_t *__restrict__ rp;
    const int32_t *__restrict__ ci;
    const T *__restrict__ va;
    int32_t n;
};

// One row of the product: sum over the row's entries in storage order of
// val[j] * Xrow(col[j]) for this lane's VW columns.  Four entries are issued
// together so their gathers overlap.
template <typename T, int VW, class Op, typename PI, typename PV>
__device__ __forceinline__ void row_product(PI cis, PV vas, int j0, int j1, int g, const Op &op,
                                            const typename Op::Lane &ln, T *sum)
{
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
        const int32_t c0 = cis[j], c1 = cis[j + 1], c2 = cis[j + 2], c3 = cis[j + 3];
        const T a0 = vas[j], a1 = vas[j + 1], a2 = vas[j + 2], a3 = vas[j + 3];
        T x0[VW], x1[VW], x2[VW], x3[VW];
        op.gather(ln, c0, g, x0);
        op.gather(ln, c1, g, x1);
        op.gather(ln, c2, g, x2);
        op.gather(ln, c3, g, x3);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            sum[v] += a0 * x0[v];
            sum[v] += a1 * x1[v];
            sum[v] += a2 * x2[v];
            sum[v] += a3 * x3[v];
        }
    }
    for (; j < j1; ++j) {
        const int32_t c = cis[j];
        const T a = vas[j];
        T x[VW];
        op.gather(ln, c, g, x);
#pragma unroll
        for (int v = 0; v < VW; ++v)
            sum[v] += a * x[v];
    }
}

// Accumulator of NDOT per-column partial dot products for a lane's columns.
template <typename T, int VW, int NDOT>
struct Acc {
    T a[NDOT > 0 ? NDOT : 1][VW];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int d = 0; d < (NDOT > 0 ? NDOT : 1); ++d)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                a[d][v] = T(0);
    }
};

// Y-side of a generalized SpMV over every tile of this workgroup.  The
// tile's row offsets, column indices and values are first staged in LDS with
// coalesced streaming loads (one pass over HBM, no reuse in cache needed), then
// every lane walks its rows out of LDS and gathers block rows of X through the
// cache hierarchy.  A tile whose nonzeros exceed kNzCap reads them directly.
template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_tiles(const CsrView<T> &A, const Op &op,
                                            Acc<T, Shape<T, M>::VW, Op::NDOT> &acc)
{
    using S = Shape<T, M>;
    __shared__ int32_t s_rp[kTileRows + 1];
    __shared__ int32_t s_ci[kNzCap];
    __shared__ T s_va[kNzCap];
    const int tid = threadIdx.x;
    const int g = tid % S::L;
    const int rl = tid / S::L;
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = g < S::G && ln.on;
    const int64_t ntiles = (static_cast<int64_t>(A.n) + kTileRows - 1) / kTileRows;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
        const int32_t r0 = static_cast<int32_t>(tile * kTileRows);
        const int nr = min(kTileRows, A.n - r0);
        for (int k = tid; k <= nr; k += kBlock)
            s_rp[k] = A.rp[r0 + k];
        __syncthreads();
        const int32_t z0 = s_rp[0];
        const int cnt = s_rp[nr] - z0;
        const bool staged = cnt <= kNzCap;
        if (staged) {
            for (int k = tid; k < cnt; k += kBlock) {
                s_ci[k] = __builtin_nontemporal_load(A.ci + z0 + k);
                s_va[k] = __builtin_nontemporal_load(A.va + z0 + k);
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int p = 0; p < S::PASSES; ++p) {
            const int row_l = p * S::RPP + rl;
            if (lane_on && row_l < nr) {
                const int j0 = s_rp[row_l] - z0;
                const int j1 = s_rp[row_l + 1] - z0;
                T sum[S::VW];
#pragma unroll
                for (int v = 0; v < S::VW; ++v)
                    sum[v] = T(0);
                if (staged)
                    row_product<T, S::VW>(s_ci, s_va, j0, j1, g, op, ln, sum);
                else
                    row_product<T, S::VW>(A.ci + z0, A.va + z0, j0, j1, g, op, ln, sum);
                op.row(ln, r0 + row_l, g, sum, acc);
            }
        }
        __syncthreads();
    }
}

// Elementwise pass over every row of this workgroup's tiles.
template <typename T, int M, class Op>
__device__ __forceinline__ void stream_tiles(int32_t n, const Op &op,
                                             Acc<T, Shape<T, M>::VW, Op::NDOT> &acc)
{
    using S = Shape<T, M>;
    const int tid = threadIdx.x;
    const int g = tid % S::L;
    const int rl = tid / S::L;
    if (g >= S::G)
        return;
    const typename Op::Lane ln = op.lane(g);
    if (!ln.on)
        return;
    const int64_t ntiles = (static_cast<int64_t>(n) + kTileRows - 1) / kTileRows;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
        const int32_t r0 = static_cast<int32_t>(tile * kTileRows);
        const int nr = min(kTileRows, n - r0);
#pragma unroll 2
        for (int p = 0; p < S::PASSES; ++p) {
            const int row_l = p * S::RPP + rl;
            if (row_l < nr)
                op.row(ln, r0 + row_l, g, acc);
        }
    }
}

// ---- deterministic grid reduction ------------------------------------------
// part:    [gridDim.x][NDOT*M]  per-workgroup partial sums
// gpart:   [kGroups][NDOT*M]    per-group sums
// tickets: [kGroups + 1]        zero on entry; reset to zero by the last workgroup
template <typename T>
struct RedBufs {
    T *part;
    T *gpart;
    unsigned int *tickets;
};

// Reduces acc over the whole grid; the very last workgroup then calls
// op.finish(tot) with tot[d*M + c] = total of dot d for column c (in LDS),
// with all threads of that workgroup participating.
template <typename T, int M, int NDOT, class Op>
__device__ __forceinline__ void grid_reduce(Acc<T, Shape<T, M>::VW, NDOT> &acc, const RedBufs<T> &rb,
                                            const Op &op)
{
    using S = Shape<T, M>;
    constexpr int V = NDOT * M;
    constexpr int TPV = (kBlock / V) > 64 ? 64 : (kBlock / V); // threads per value
    __shared__ T s_w[kBlock / 64][V];
    __shared__ T s_k[TPV][V];
    __shared__ T s_tot[V];
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = tid % S::L;

#pragma unroll
    for (int off = S::L; off < 64; off <<= 1)
#pragma unroll
        for (int d = 0; d < NDOT; ++d)
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                acc.a[d][v] += __shfl_xor(acc.a[d][v], off);
    if (lane < S::L && g < S::G) {
#pragma unroll
        for (int d = 0; d < NDOT; ++d)
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                s_w[wave][d * M + g * S::VW + v] = acc.a[d][v];
    }
    __syncthreads();
    const int b = blockIdx.x;
    const int grp = b % kGroups;
    const int gx = gridDim.x / kGroups;
    if (tid < V) {
        T s = s_w[0][tid];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w)
            s += s_w[w][tid];
        rb.part[static_cast<size_t>(b) * V + tid] = s;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0)
        s_flag = atomicAdd(&rb.tickets[grp], 1u) == static_cast<unsigned>(gx - 1);
    __syncthreads();
    if (!s_flag)
        return;
    __threadfence();
    // this workgroup is the last of its group: sum the group's partials
    if (tid < TPV * V) {
        const int v = tid % V;
        const int k = tid / V;
        T s = T(0);
        for (int q = k; q < gx; q += TPV)
            s += rb.part[static_cast<size_t>(grp + q * kGroups) * V + v];
        s_k[k][v] = s;
    }
    __syncthreads();
    if (tid < V) {
        T s = s_k[0][tid];
        for (int k = 1; k < TPV; ++k)
            s += s_k[k][tid];
        rb.gpart[grp * V + tid] = s;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0)
        s_flag = atomicAdd(&rb.tickets[kGroups], 1u) == static_cast<unsigned>(kGroups - 1);
    __syncthreads();
    if (!s_flag)
        return;
    __threadfence();
    if (tid < V) {
        T s = rb.gpart[tid];
#pragma unroll
        for (int x = 1; x < kGroups; ++x)
            s += rb.gpart[x * V + tid];
        s_tot[tid] = s;
    }
    if (tid <= kGroups)
        rb.tickets[tid] = 0u;
    __syncthreads();
    op.finish(s_tot);
}

} // namespace mrhs
