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
// Products over matrices with a long, regular forward reach (a grid operator
// in natural order, whose farthest neighbour is a plane of P tiles away) use
// a plane-interleaved schedule instead: the rows are seen as planes of P
// tiles, group x owns the x-th eighth of every plane and walks the planes in
// order, so the rows a tile gathers from the planes before and after it were
// fetched into the same XCD's L2 by the tiles just before and just after it.
// Wide blocks make a group's eighth of a plane too large for its L2 to keep
// two of them; then every plane is cut into C chunks and the planes are
// walked C times, once per chunk.
//
// Lane layout for an n x M row-interleaved block.  Each lane handles VW
// consecutive columns of one row (VW elements = one 16-byte access when M is
// wide enough), a row takes G = ceil(M/VW) lanes padded to L = next power of
// two, and a wave holds 64/L rows.  A wave-wide access of a block therefore
// covers 64/L whole rows, i.e. contiguous memory.  When VW does not divide M
// the row's last lane holds the remaining TAIL columns and accesses them
// element by element, and the other lanes' vectors are only element-aligned.
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

#ifndef MRHS_TILE_ROWS
#define MRHS_TILE_ROWS 256
#endif
#ifndef MRHS_NZ_PER_ROW
#define MRHS_NZ_PER_ROW 8
#endif
#ifndef MRHS_GATHER_BATCH
#define MRHS_GATHER_BATCH 7  // one batch covers a 7-point stencil row
#endif
#ifndef MRHS_PLANE_CHUNKS
#define MRHS_PLANE_CHUNKS 0  // 0: chosen per product from its block bytes per tile
#endif
#ifndef MRHS_XCD_GROUPS
#define MRHS_XCD_GROUPS 1
#endif

constexpr int kBlock = 256;
constexpr int kTileRows = MRHS_TILE_ROWS;  // rows per tile (at least one pass)
constexpr int kGroups = 8;
constexpr int kMaxM = 16;
constexpr int kMaxDots = 8;  // largest NDOT of any reduction (GCR projections)

constexpr int next_pow2(int x) { return x <= 1 ? 1 : 2 * next_pow2((x + 1) / 2); }

template <typename T, int M>
struct Shape {
    // columns per lane: the widest 8- or 16-byte access that divides the row
    // (a row-end lane holding fewer columns, with element-aligned 16-byte
    // accesses for the others, measured 20 % slower for odd M in binary64)
    static constexpr int VW = std::is_same<T, double>::value ? (M % 2 == 0 ? 2 : 1)
                                                             : (M % 4 == 0 ? 4 : (M % 2 == 0 ? 2 : 1));
    static constexpr int G = (M + VW - 1) / VW;  // lanes that hold data in a row
    static constexpr int TAIL = M - (G - 1) * VW; // columns of the row's last lane (1..VW)
    // lanes per row: the next power of two of G, or G itself for one-element
    // lanes (odd M) and G = 5 when that fits more rows into a wave.  Measured
    // on the 12.6M-row channel: +6..+43 % for odd M; for 16-byte lanes only
    // G = 5 gained (binary32 M = 10: +25 %), G = 3, 6, 7 lost up to 12 %.
    static constexpr bool EXACT = (VW == 1 || G == 5) && 64 / G > 64 / next_pow2(G);
    static constexpr int L = EXACT ? G : next_pow2(G);
    static constexpr bool POW2 = L == next_pow2(L);
    static constexpr int RW = 64 / L;             // rows per wave (lanes past RW*L idle)
    static constexpr int RPP = (kBlock / 64) * RW; // rows per pass of the workgroup
    static constexpr int PASSES = RPP >= kTileRows ? 1 : kTileRows / RPP;
    static constexpr int TR = RPP * PASSES;       // rows per tile
    static constexpr int NZCAP = TR * MRHS_NZ_PER_ROW;  // staged nonzeros per tile
    static_assert(L <= 64, "a row must fit one wave");
    static_assert(L <= kMaxM, "a row's lanes fit the per-row byte arrays");
    // thread -> (lane in row, row in pass); lane_on = false for idle lanes
    static __device__ __forceinline__ int lane_of(int tid) { return (tid & 63) % L; }
    static __device__ __forceinline__ int row_of(int tid) { return (tid >> 6) * RW + (tid & 63) / L; }
    static __device__ __forceinline__ bool used(int tid) { return (tid & 63) < RW * L; }
};

// ---- 8/16-byte vector access ------------------------------------------------
template <typename T, int VW>
struct Vec;

template <typename T>
struct Vec<T, 1> {
    static __device__ __forceinline__ void load(const T *p, T *v) { v[0] = *p; }
    static __device__ __forceinline__ void store(T *p, const T *v) { *p = v[0]; }
    static __device__ __forceinline__ void store_nt(T *p, const T *v) { __builtin_nontemporal_store(v[0], p); }
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
    static __device__ __forceinline__ void store_nt(double *p, const double *v)
    {
        v2 t;
        t.x = v[0];
        t.y = v[1];
        __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(p));
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
    static __device__ __forceinline__ void store_nt(float *p, const float *v)
    {
        v2 t;
        t.x = v[0];
        t.y = v[1];
        __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(p));
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
    static __device__ __forceinline__ void store_nt(float *p, const float *v)
    {
        v4 t;
        t.x = v[0];
        t.y = v[1];
        t.z = v[2];
        t.w = v[3];
        __builtin_nontemporal_store(t, reinterpret_cast<v4 *>(p));
    }
};

// Vectors of VW elements at element (not vector) alignment: the rows of a
// block whose width VW does not divide start at any element.
template <typename T, int VW>
struct VecU {
    typedef T vu __attribute__((ext_vector_type(VW), aligned(sizeof(T))));
    static __device__ __forceinline__ void load(const T *p, T *v)
    {
        const vu t = *reinterpret_cast<const vu *>(p);
#pragma unroll
        for (int q = 0; q < VW; ++q)
            v[q] = t[q];
    }
    static __device__ __forceinline__ void store_nt(T *p, const T *v)
    {
        vu t;
#pragma unroll
        for (int q = 0; q < VW; ++q)
            t[q] = v[q];
        __builtin_nontemporal_store(t, reinterpret_cast<vu *>(p));
    }
    static __device__ __forceinline__ void store(T *p, const T *v)
    {
        vu t;
#pragma unroll
        for (int q = 0; q < VW; ++q)
            t[q] = v[q];
        *reinterpret_cast<vu *>(p) = t;
    }
};

#ifndef MRHS_NT_STORE
#define MRHS_NT_STORE 1
#endif

// Lane g's VW elements of row `row` of an n x M block whose rows lie ld
// elements apart (ld = M, or 2M for a half of an interleaved pair of blocks).
// The last lane of a row whose width VW does not divide reads its TAIL
// elements one by one (the rest of v is zero), so no access leaves the row.
template <typename T, int M>
__device__ __forceinline__ void ld(const T *base, int32_t row, int g, T *v, int32_t ld = M)
{
    using S = Shape<T, M>;
    const T *p = base + static_cast<size_t>(row) * ld + g * S::VW;
    if constexpr (S::TAIL == S::VW) {
        Vec<T, S::VW>::load(p, v);
    } else if (g == S::G - 1) {
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            v[q] = q < S::TAIL ? p[q] : T(0);
    } else {
        VecU<T, S::VW>::load(p, v);
    }
}

// Stores lane g's elements of a row; block outputs use streaming
// (nontemporal) stores: every block is far larger than the caches, and
// keeping written lines out of L2 leaves it to the gathered block rows.
template <typename T, int M>
__device__ __forceinline__ void st(T *base, int32_t row, int g, const T *v, int32_t ld = M)
{
    using S = Shape<T, M>;
    T *p = base + static_cast<size_t>(row) * ld + g * S::VW;
    if constexpr (S::TAIL == S::VW) {
#if MRHS_NT_STORE
        Vec<T, S::VW>::store_nt(p, v);
#else
        Vec<T, S::VW>::store(p, v);
#endif
    } else if (g == S::G - 1) {
#pragma unroll
        for (int q = 0; q < S::TAIL; ++q)
            __builtin_nontemporal_store(v[q], p + q);
    } else {
        VecU<T, S::VW>::store_nt(p, v);
    }
}


// 32-byte lanes: two 16-byte accesses

// ---- tile schedule ------------------------------------------------------------
// Steps s = first, first + stride, ... < end of this workgroup; step s is
// tile s (contiguous mode, P = 0) or, in plane mode with chunks of W = P / C
// tiles and sc = planes * cg steps per chunk, tile
// (s / sc) * W + (t / cg) * P + lo + t % cg with t = s % sc, which may fall
// past the last tile in the final, partial plane (then it is skipped).
struct TileRange {
    int32_t first, end, stride;
    int32_t P, lo, cg;
    int32_t W, sc;  // chunk width in tiles, steps per chunk
    __device__ __forceinline__ int32_t tile(int32_t s) const
    {
        if (!P)
            return s;
        const int32_t c = s / sc, t = s - c * sc;
        return c * W + (t / cg) * P + lo + t % cg;
    }
};

__device__ __forceinline__ TileRange tile_range(int32_t ntiles, int32_t P = 0, int32_t C = 1)
{
#if !MRHS_XCD_GROUPS
    return {static_cast<int32_t>(blockIdx.x), ntiles, static_cast<int32_t>(gridDim.x), 0, 0, 1, 1, 1};
#endif
    const int b = blockIdx.x;
    const int grp = b % kGroups;
    const int q = b / kGroups;
    const int gx = gridDim.x / kGroups;
    if (P) {
        if (P % C != 0 || P / C < 2 * kGroups)
            C = 1;
        const int32_t W = P / C;
        const int32_t lo = W * grp / kGroups;
        const int32_t cg = W * (grp + 1) / kGroups - lo;
        const int32_t planes = (ntiles + P - 1) / P;
        return {q, C * planes * cg, gx, P, lo, cg, W, planes * cg};
    }
    const int32_t lo = static_cast<int32_t>(static_cast<int64_t>(ntiles) * grp / kGroups);
    const int32_t hi = static_cast<int32_t>(static_cast<int64_t>(ntiles) * (grp + 1) / kGroups);
    return {lo + q, hi, gx, 0, 0, 1, 1, 1};
}

// Tiles per plane for the plane-interleaved schedule of a product, or 0 for
// the contiguous one: the matrix's typical forward reach (median over rows of
// the largest column - row offset) rounded to whole tiles, used when every
// group gets at least two tiles of each plane and there are at least four
// planes.
__device__ __forceinline__ int32_t plane_tiles(int32_t reach, int32_t tile_rows, int32_t ntiles)
{
    const int32_t P = (reach + tile_rows / 2) / tile_rows;
    return (P >= 2 * kGroups && ntiles >= 4 * P) ? P : 0;
}

// Chunks per plane: a row gathers from the plane before and the plane after
// its own, so a group's block rows must stay in its L2 while it works through
// about two of its plane shares.  Splitting every plane into C chunks, swept
// one chunk at a time through all planes, divides that share by C.  C is the
// smallest divisor of P that brings the share's block bytes under
// kPlaneShareBytes while leaving at least kMinChunkTiles tiles per chunk, and
// 1 when there is none or when the reach is not a whole number of tiles
// (measured on the 12.6M-row channel: binary64 m = 16 +8 %, m = 8 +2 % with
// whole-tile planes; 4-9 % slower at m = 7, 9, 10, 11, whose 240- and 252-row
// tiles split a plane).
#ifndef MRHS_PLANE_SHARE_KB
#define MRHS_PLANE_SHARE_KB 700
#endif
#ifndef MRHS_PLANE_MIN_CHUNK
#define MRHS_PLANE_MIN_CHUNK 16
#endif
constexpr int32_t kPlaneShareBytes = MRHS_PLANE_SHARE_KB << 10;
constexpr int32_t kMinChunkTiles = MRHS_PLANE_MIN_CHUNK;

__device__ __forceinline__ int32_t plane_chunks(int32_t P, int32_t reach, int32_t tile_rows,
                                                int32_t block_bytes_per_tile)
{
#if MRHS_PLANE_CHUNKS
    return MRHS_PLANE_CHUNKS;
#endif
    if (!P || reach % tile_rows != 0)
        return 1;
    const int64_t share = static_cast<int64_t>((P + kGroups - 1) / kGroups) * block_bytes_per_tile;
    for (int32_t C = static_cast<int32_t>((share + kPlaneShareBytes - 1) / kPlaneShareBytes);
         C > 1 && P / C >= kMinChunkTiles; ++C)
        if (P % C == 0)
            return C;
    return 1;
}

// ---- matrix view ----------------------------------------------------------------
// Dictionary form of a matrix whose entries take few distinct column offsets
// (col - row) and few distinct values, as the finite-difference operators of
// a structured grid do: entry j is one 16-bit code, its column
// row + otab[code & omask] and its value vtab[code >> ob], both exact, so a
// product sums the same values in the same order as from the plain arrays
// and reads 2 bytes per entry instead of 4 + sizeof(T).  A matrix with more
// distinct offsets but few distinct values (a grid operator with its rows
// renumbered) gets 32-bit codes instead: column code & cmask, value
// vtab[code >> cb] (4 bytes per entry).
constexpr int kDictOffs = 32;    // at most this many distinct offsets
constexpr int kDictVals = 2048;  // and this many distinct values per array

template <typename T>
struct CsrView {
    const int32_t *__restrict__ rp;
    const int32_t *__restrict__ ci;
    const T *__restrict__ va;
    int32_t n;
    int32_t reach;  // median over rows of the largest forward column offset
    int32_t split;  // nonzero: long rows, one wave per row (gspmv_rows_split)
    // dictionary form (gspmv_tiles only; null code and ccode: the plain arrays)
    const uint16_t *__restrict__ code = nullptr;   // [nnz + 8]
    const int32_t *__restrict__ otab = nullptr;    // [noffs]
    const uint32_t *__restrict__ ccode = nullptr;  // [nnz + 4] column codes
    const T *__restrict__ vtab = nullptr;          // [nvals]
    int32_t noffs = 0, nvals = 0;
    int32_t ob = 0;  // bits of the offset index in a code
    int32_t cb = 0;  // bits of the column in a column code
};

// One row of the product: sum over the row's entries in storage order of
// val[j] * Xrow(col[j]) for this lane's VW columns.  Entries are taken NB at a
// time and all NB gathers are issued before any is consumed, so a stencil row
// costs one memory round trip.  Slots past the row's end re-read the row's
// last entry (always a valid index, a cache hit) and are not accumulated.
template <typename T, int VW, class Op, typename PI, typename PV>
__device__ __forceinline__ void row_product(PI cis, PV vas, int j0, int j1, int g, const Op &op,
                                            const typename Op::Lane &ln, T *sum)
{
    constexpr int NB = MRHS_GATHER_BATCH;
    for (int j = j0; j < j1; j += NB) {
        int32_t c[NB];
        T a[NB], x[NB][VW];
        bool ok[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            ok[k] = j + k < j1;
            const int jj = ok[k] ? j + k : j1 - 1;
            c[k] = cis[jj];
            a[k] = vas[jj];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k)
            op.gather(ln, c[k], g, x[k]);
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                if (ok[k])
                    sum[v] += a[k] * x[k][v];
    }
}

// row_product over column codes: entry j's column is code & cmask, its value
// vtab[code >> cb] (table in LDS).
template <typename T, int VW, class Op, typename PC>
__device__ __forceinline__ void row_product_cc(PC codes, const T *vtab, int cb, uint32_t cmask, int j0, int j1,
                                               int g, const Op &op, const typename Op::Lane &ln, T *sum)
{
    constexpr int NB = MRHS_GATHER_BATCH;
    for (int j = j0; j < j1; j += NB) {
        int32_t c[NB];
        T a[NB], x[NB][VW];
        bool ok[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            ok[k] = j + k < j1;
            const int jj = ok[k] ? j + k : j1 - 1;
            const uint32_t cd = codes[jj];
            c[k] = static_cast<int32_t>(cd & cmask);
            a[k] = vtab[cd >> cb];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k)
            op.gather(ln, c[k], g, x[k]);
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                if (ok[k])
                    sum[v] += a[k] * x[k][v];
    }
}

// row_product over the dictionary form: entry j's column is
// row + otab[code & omask], its value vtab[code >> ob] (tables in LDS).
template <typename T, int VW, class Op, typename PC>
__device__ __forceinline__ void row_product_dict(PC codes, const int32_t *otab, const T *vtab, int ob,
                                                 uint32_t omask, int32_t row, int j0, int j1, int g, const Op &op,
                                                 const typename Op::Lane &ln, T *sum)
{
    constexpr int NB = MRHS_GATHER_BATCH;
    for (int j = j0; j < j1; j += NB) {
        int32_t c[NB];
        T a[NB], x[NB][VW];
        bool ok[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            ok[k] = j + k < j1;
            const int jj = ok[k] ? j + k : j1 - 1;
            const uint32_t cd = codes[jj];
            c[k] = row + otab[cd & omask];
            a[k] = vtab[cd >> ob];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k)
            op.gather(ln, c[k], g, x[k]);
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int v = 0; v < VW; ++v)
                if (ok[k])
                    sum[v] += a[k] * x[k][v];
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

// Workgroups per CU a streaming op is launched with at most (Op::kMaxPerCU
// when the op defines it; 0: as many as fit).
template <class Op, class = void>
struct max_per_cu {
    static constexpr int value = 0;
};
template <class Op>
struct max_per_cu<Op, std::void_t<decltype(Op::kMaxPerCU)>> {
    static constexpr int value = Op::kMaxPerCU;
};

// Blocks a product gathers per entry (Op::GATHERED when the op defines it).
template <class Op, class = void>
struct gathered_blocks {
    static constexpr int value = 1;
};
template <class Op>
struct gathered_blocks<Op, std::void_t<decltype(Op::GATHERED)>> {
    static constexpr int value = Op::GATHERED;
};

// Ops whose epilogue reads the row's own entries of other blocks may declare
// a type Pre and a method pre(lane, row, g) returning them; the tile loop then
// issues those loads before the row's gathers, so both come back in one
// memory round trip, and passes them to row(..., pre).
template <class Op, class = void>
struct has_pre : std::false_type {};
template <class Op>
struct has_pre<Op, std::void_t<typename Op::Pre>> : std::true_type {};
template <class Op, bool = has_pre<Op>::value>
struct pre_of {
    using type = int;
};
template <class Op>
struct pre_of<Op, true> {
    using type = typename Op::Pre;
};

// Ops that set kLongRows = true may run on the one-wave-per-row product
// (gspmv_rows_split) when their matrix has long rows; the others always use
// the tiled one, which is correct for any matrix.
template <class Op, class = void>
struct long_rows_ok : std::false_type {};
template <class Op>
struct long_rows_ok<Op, std::void_t<decltype(Op::kLongRows)>> : std::integral_constant<bool, Op::kLongRows> {};

// Stages the row offsets of rows r0 .. r0 + nr of A in s_rp, then (when
// they fit NZCAP) the rows' column indices and values in s_ci / s_va with
// coalesced streaming loads.  16-byte loads start at the 4-aligned index
// zb <= z0 = row_ptr[r0] (the matrix arrays carry 4 elements of padding, so
// whole vectors stay in bounds), and every thread issues all of its loads
// before writing any of them to LDS.  Entry z0 + k is then at s_ci[lead + k].
// The caller synchronizes before reading the indices and values.
struct Staged {
    int32_t z0;
    int lead;
    bool staged;
};

template <typename T, int NZCAP>
__device__ __forceinline__ Staged stage_csr(const CsrView<T> &A, int32_t r0, int nr, int32_t *s_rp, int32_t *s_ci,
                                            T *s_va)
{
    const int tid = threadIdx.x;
    for (int k = tid; k <= nr; k += kBlock)
        s_rp[k] = A.rp[r0 + k];
    __syncthreads();
    const int32_t z0 = s_rp[0];
    const int cnt = s_rp[nr] - z0;
    const int32_t zb = z0 & ~3;
    const int lead = z0 - zb;
    const bool staged = cnt + lead <= NZCAP;
    if (staged) {
        using I4 = int __attribute__((ext_vector_type(4)));
        constexpr int VV = 16 / static_cast<int>(sizeof(T));
        using TV = T __attribute__((ext_vector_type(VV)));
        constexpr int CI_PT = ((NZCAP + 4) / 4 + kBlock - 1) / kBlock;
        constexpr int VA_PT = ((NZCAP + 4) / VV + kBlock - 1) / kBlock;
        const int nci = (cnt + lead + 3) / 4;
        const int nva = (cnt + lead + VV - 1) / VV;
        const I4 *gci = reinterpret_cast<const I4 *>(A.ci + zb);
        const TV *gva = reinterpret_cast<const TV *>(A.va + zb);
        I4 bci[CI_PT];
        TV bva[VA_PT];
#pragma unroll
        for (int u = 0; u < CI_PT; ++u) {
            const int k = tid + u * kBlock;
            if (k < nci)
                bci[u] = __builtin_nontemporal_load(gci + k);
        }
#pragma unroll
        for (int u = 0; u < VA_PT; ++u) {
            const int k = tid + u * kBlock;
            if (k < nva)
                bva[u] = __builtin_nontemporal_load(gva + k);
        }
#pragma unroll
        for (int u = 0; u < CI_PT; ++u) {
            const int k = tid + u * kBlock;
            if (k < nci)
                reinterpret_cast<I4 *>(s_ci)[k] = bci[u];
        }
#pragma unroll
        for (int u = 0; u < VA_PT; ++u) {
            const int k = tid + u * kBlock;
            if (k < nva)
                reinterpret_cast<TV *>(s_va)[k] = bva[u];
        }
    }
    return {z0, lead, staged};
}

// Y-side of a generalized SpMV over every tile of this workgroup.  The
// tile's row offsets, column indices and values are first staged in LDS with
// coalesced streaming loads (one pass over HBM, no reuse in cache needed), then
// every lane walks its rows out of LDS and gathers block rows of X through the
// cache hierarchy.  A tile whose nonzeros exceed S::NZCAP reads them directly.
// LDS of a tile: the plain form's indices and values, or the dictionary
// form's codes and tables, in one buffer.
template <typename T, int M>
struct TileLds {
    using S = Shape<T, M>;
    static constexpr int CI_BYTES = (S::NZCAP + 4) * 4;
    // values, or the value table of column codes
    static constexpr int VA_ELEMS = S::NZCAP + 4 > kDictVals ? S::NZCAP + 4 : kDictVals;
    static constexpr int PLAIN = CI_BYTES + VA_ELEMS * static_cast<int>(sizeof(T));
    static constexpr int CODE_BYTES = ((S::NZCAP + 8) * 2 + 15) / 16 * 16;
    static constexpr int VTAB_AT = CODE_BYTES + kDictOffs * 4;
    static constexpr int DICT = VTAB_AT + kDictVals * static_cast<int>(sizeof(T));
    static constexpr int BYTES = PLAIN > DICT ? PLAIN : DICT;
};

// gspmv_tiles over the dictionary form: the tables are loaded into LDS
// once, then every tile stages its codes (16-byte loads of 8 codes from the
// 8-aligned index zb <= z0; the code array carries 8 codes of padding).
template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_tiles_dict(const CsrView<T> &A, const Op &op,
                                                 Acc<T, Shape<T, M>::VW, Op::NDOT> &acc, int32_t *s_rp,
                                                 unsigned char *s_buf)
{
    using S = Shape<T, M>;
    using LD = TileLds<T, M>;
    using I4 = int __attribute__((ext_vector_type(4)));
    uint16_t *s_code = reinterpret_cast<uint16_t *>(s_buf);
    int32_t *s_otab = reinterpret_cast<int32_t *>(s_buf + LD::CODE_BYTES);
    T *s_vtab = reinterpret_cast<T *>(s_buf + LD::VTAB_AT);
    const int tid = threadIdx.x;
    const int g = S::lane_of(tid);
    const int rl = S::row_of(tid);
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = S::used(tid) && g < S::G && ln.on;
    for (int k = tid; k < A.noffs; k += kBlock)
        s_otab[k] = A.otab[k];
    for (int k = tid; k < A.nvals; k += kBlock)
        s_vtab[k] = A.vtab[k];
    // (visible after the first tile's barrier)
    const int ob = A.ob;
    const uint32_t omask = (1u << ob) - 1u;
    const int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(A.n) + S::TR - 1) / S::TR);
    const int32_t P = plane_tiles(A.reach, S::TR, ntiles);
    constexpr int32_t kBlockBytes = (gathered_blocks<Op>::value + 1) * S::TR * M * static_cast<int32_t>(sizeof(T));
    const TileRange tr = tile_range(ntiles, P, plane_chunks(P, A.reach, S::TR, kBlockBytes));
    constexpr int CO_PT = ((S::NZCAP + 8) / 8 + kBlock - 1) / kBlock;
    for (int32_t step = tr.first; step < tr.end; step += tr.stride) {
        const int32_t tile = tr.tile(step);
        if (tile >= ntiles)
            continue;
        const int32_t r0 = tile * S::TR;
        const int nr = min(S::TR, A.n - r0);
        for (int k = tid; k <= nr; k += kBlock)
            s_rp[k] = A.rp[r0 + k];
        __syncthreads();
        const int32_t z0 = s_rp[0];
        const int cnt = s_rp[nr] - z0;
        const int32_t zb = z0 & ~7;
        const int lead = z0 - zb;
        const bool staged = cnt + lead <= S::NZCAP;
        if (staged) {
            const int nco = (cnt + lead + 7) / 8;
            const I4 *gco = reinterpret_cast<const I4 *>(A.code + zb);
            I4 bco[CO_PT];
#pragma unroll
            for (int u = 0; u < CO_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nco)
                    bco[u] = __builtin_nontemporal_load(gco + k);
            }
#pragma unroll
            for (int u = 0; u < CO_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nco)
                    reinterpret_cast<I4 *>(s_code)[k] = bco[u];
            }
        }
        __syncthreads();
        const uint16_t *lco = s_code + lead;
#pragma unroll 1
        for (int p = 0; p < S::PASSES; ++p) {
            const int row_l = p * S::RPP + rl;
            if (lane_on && row_l < nr) {
                const int32_t row = r0 + row_l;
                const int j0 = s_rp[row_l] - z0;
                const int j1 = s_rp[row_l + 1] - z0;
                T sum[S::VW];
#pragma unroll
                for (int v = 0; v < S::VW; ++v)
                    sum[v] = T(0);
                if constexpr (has_pre<Op>::value) {
                    const typename Op::Pre pr = op.pre(ln, row, g);
                    if (staged)
                        row_product_dict<T, S::VW>(lco, s_otab, s_vtab, ob, omask, row, j0, j1, g, op, ln, sum);
                    else
                        row_product_dict<T, S::VW>(A.code + z0, s_otab, s_vtab, ob, omask, row, j0, j1, g, op, ln,
                                                   sum);
                    op.row(ln, row, g, sum, acc, pr);
                } else {
                    if (staged)
                        row_product_dict<T, S::VW>(lco, s_otab, s_vtab, ob, omask, row, j0, j1, g, op, ln, sum);
                    else
                        row_product_dict<T, S::VW>(A.code + z0, s_otab, s_vtab, ob, omask, row, j0, j1, g, op, ln,
                                                   sum);
                    op.row(ln, row, g, sum, acc);
                }
            }
        }
        __syncthreads();
    }
}

// gspmv_tiles over column codes: the value table is loaded into LDS once,
// then every tile stages its 4-byte codes as the plain form stages its
// column indices (the code array carries 4 codes of padding).
template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_tiles_cc(const CsrView<T> &A, const Op &op,
                                               Acc<T, Shape<T, M>::VW, Op::NDOT> &acc, int32_t *s_rp,
                                               unsigned char *s_buf)
{
    using S = Shape<T, M>;
    using LD = TileLds<T, M>;
    using I4 = int __attribute__((ext_vector_type(4)));
    uint32_t *s_cc = reinterpret_cast<uint32_t *>(s_buf);
    T *s_vtab = reinterpret_cast<T *>(s_buf + LD::CI_BYTES);
    const int tid = threadIdx.x;
    const int g = S::lane_of(tid);
    const int rl = S::row_of(tid);
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = S::used(tid) && g < S::G && ln.on;
    for (int k = tid; k < A.nvals; k += kBlock)
        s_vtab[k] = A.vtab[k];
    // (visible after the first tile's barrier)
    const int cb = A.cb;
    const uint32_t cmask = cb >= 32 ? 0xffffffffu : (1u << cb) - 1u;
    const int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(A.n) + S::TR - 1) / S::TR);
    const int32_t P = plane_tiles(A.reach, S::TR, ntiles);
    constexpr int32_t kBlockBytes = (gathered_blocks<Op>::value + 1) * S::TR * M * static_cast<int32_t>(sizeof(T));
    const TileRange tr = tile_range(ntiles, P, plane_chunks(P, A.reach, S::TR, kBlockBytes));
    constexpr int CC_PT = ((S::NZCAP + 4) / 4 + kBlock - 1) / kBlock;
    for (int32_t step = tr.first; step < tr.end; step += tr.stride) {
        const int32_t tile = tr.tile(step);
        if (tile >= ntiles)
            continue;
        const int32_t r0 = tile * S::TR;
        const int nr = min(S::TR, A.n - r0);
        for (int k = tid; k <= nr; k += kBlock)
            s_rp[k] = A.rp[r0 + k];
        __syncthreads();
        const int32_t z0 = s_rp[0];
        const int cnt = s_rp[nr] - z0;
        const int32_t zb = z0 & ~3;
        const int lead = z0 - zb;
        const bool staged = cnt + lead <= S::NZCAP;
        if (staged) {
            const int ncc = (cnt + lead + 3) / 4;
            const I4 *gcc = reinterpret_cast<const I4 *>(A.ccode + zb);
            I4 bcc[CC_PT];
#pragma unroll
            for (int u = 0; u < CC_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < ncc)
                    bcc[u] = __builtin_nontemporal_load(gcc + k);
            }
#pragma unroll
            for (int u = 0; u < CC_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < ncc)
                    reinterpret_cast<I4 *>(s_cc)[k] = bcc[u];
            }
        }
        __syncthreads();
        const uint32_t *lcc = s_cc + lead;
#pragma unroll 1
        for (int p = 0; p < S::PASSES; ++p) {
            const int row_l = p * S::RPP + rl;
            if (lane_on && row_l < nr) {
                const int32_t row = r0 + row_l;
                const int j0 = s_rp[row_l] - z0;
                const int j1 = s_rp[row_l + 1] - z0;
                T sum[S::VW];
#pragma unroll
                for (int v = 0; v < S::VW; ++v)
                    sum[v] = T(0);
                if constexpr (has_pre<Op>::value) {
                    const typename Op::Pre pr = op.pre(ln, row, g);
                    if (staged)
                        row_product_cc<T, S::VW>(lcc, s_vtab, cb, cmask, j0, j1, g, op, ln, sum);
                    else
                        row_product_cc<T, S::VW>(A.ccode + z0, s_vtab, cb, cmask, j0, j1, g, op, ln, sum);
                    op.row(ln, row, g, sum, acc, pr);
                } else {
                    if (staged)
                        row_product_cc<T, S::VW>(lcc, s_vtab, cb, cmask, j0, j1, g, op, ln, sum);
                    else
                        row_product_cc<T, S::VW>(A.ccode + z0, s_vtab, cb, cmask, j0, j1, g, op, ln, sum);
                    op.row(ln, row, g, sum, acc);
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_tiles(const CsrView<T> &A, const Op &op,
                                            Acc<T, Shape<T, M>::VW, Op::NDOT> &acc)
{
    using S = Shape<T, M>;
    __shared__ int32_t s_rp[S::TR + 1];
    __shared__ __align__(16) unsigned char s_buf[TileLds<T, M>::BYTES];
    if (A.code) {
        gspmv_tiles_dict<T, M>(A, op, acc, s_rp, s_buf);
        return;
    }
    if (A.ccode) {
        gspmv_tiles_cc<T, M>(A, op, acc, s_rp, s_buf);
        return;
    }
    int32_t *s_ci = reinterpret_cast<int32_t *>(s_buf);
    T *s_va = reinterpret_cast<T *>(s_buf + TileLds<T, M>::CI_BYTES);
    const int tid = threadIdx.x;
    const int g = S::lane_of(tid);
    const int rl = S::row_of(tid);
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = S::used(tid) && g < S::G && ln.on;
    const int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(A.n) + S::TR - 1) / S::TR);
    const int32_t P = plane_tiles(A.reach, S::TR, ntiles);
    constexpr int32_t kBlockBytes = (gathered_blocks<Op>::value + 1) * S::TR * M * static_cast<int32_t>(sizeof(T));
    const TileRange tr = tile_range(ntiles, P, plane_chunks(P, A.reach, S::TR, kBlockBytes));
    for (int32_t step = tr.first; step < tr.end; step += tr.stride) {
        const int32_t tile = tr.tile(step);
        if (tile >= ntiles)  // past the end of the last, partial plane
            continue;
        const int32_t r0 = tile * S::TR;
        const int nr = min(S::TR, A.n - r0);
        for (int k = tid; k <= nr; k += kBlock)
            s_rp[k] = A.rp[r0 + k];
        __syncthreads();
        const int32_t z0 = s_rp[0];
        const int cnt = s_rp[nr] - z0;
        // 16-byte loads from the 4-aligned index zb <= z0 (the matrix arrays
        // carry 4 elements of padding, so whole vectors stay in bounds); every
        // thread issues all of its loads before writing any of them to LDS
        const int32_t zb = z0 & ~3;
        const int lead = z0 - zb;
        const bool staged = cnt + lead <= S::NZCAP;
        if (staged) {
            using I4 = int __attribute__((ext_vector_type(4)));
            constexpr int VV = 16 / static_cast<int>(sizeof(T));
            using TV = T __attribute__((ext_vector_type(VV)));
            constexpr int CI_PT = ((S::NZCAP + 4) / 4 + kBlock - 1) / kBlock;
            constexpr int VA_PT = ((S::NZCAP + 4) / VV + kBlock - 1) / kBlock;
            const int nci = (cnt + lead + 3) / 4;
            const int nva = (cnt + lead + VV - 1) / VV;
            const I4 *gci = reinterpret_cast<const I4 *>(A.ci + zb);
            const TV *gva = reinterpret_cast<const TV *>(A.va + zb);
            I4 bci[CI_PT];
            TV bva[VA_PT];
#pragma unroll
            for (int u = 0; u < CI_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nci)
                    bci[u] = __builtin_nontemporal_load(gci + k);
            }
#pragma unroll
            for (int u = 0; u < VA_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nva)
                    bva[u] = __builtin_nontemporal_load(gva + k);
            }
#pragma unroll
            for (int u = 0; u < CI_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nci)
                    reinterpret_cast<I4 *>(s_ci)[k] = bci[u];
            }
#pragma unroll
            for (int u = 0; u < VA_PT; ++u) {
                const int k = tid + u * kBlock;
                if (k < nva)
                    reinterpret_cast<TV *>(s_va)[k] = bva[u];
            }
        }
        __syncthreads();
        const int32_t *lci = s_ci + lead;
        const T *lva = s_va + lead;
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
                if constexpr (has_pre<Op>::value) {
                    const typename Op::Pre pr = op.pre(ln, r0 + row_l, g);
                    if (staged)
                        row_product<T, S::VW>(lci, lva, j0, j1, g, op, ln, sum);
                    else
                        row_product<T, S::VW>(A.ci + z0, A.va + z0, j0, j1, g, op, ln, sum);
                    op.row(ln, r0 + row_l, g, sum, acc, pr);
                } else {
                    if (staged)
                        row_product<T, S::VW>(lci, lva, j0, j1, g, op, ln, sum);
                    else
                        row_product<T, S::VW>(A.ci + z0, A.va + z0, j0, j1, g, op, ln, sum);
                    op.row(ln, r0 + row_l, g, sum, acc);
                }
            }
        }
        __syncthreads();
    }
}

// ---- plane march: gathered block rows staged in LDS -------------------------
// For a grid operator in natural order (forward reach R = a whole number of
// march tiles, the plane), a row of plane z gathers from its own tile, the
// tiles next to it in the same plane and the same tile of planes z - 1 and
// z + 1.  A workgroup of the march owns one tile column t of the planes and a
// run of consecutive planes; it walks them in order and keeps the gathered
// block rows of its tile for planes z - 1, z and z + 1 in a ring of three LDS
// windows, each loaded once (with the op's own gather, so a window holds
// exactly the values a gather would return, e.g. s = r - alpha v).  Entries
// whose column falls in a window read LDS; the others (the neighbouring tiles
// of the same plane) gather through the cache as in gspmv_tiles.  Every row's
// sum is formed in the same order from the same values, so the products are
// bitwise those of gspmv_tiles; only the rows' assignment to workgroups (and
// so the order of the per-workgroup partial dot products) differs.
//
// Schedule: group x = b % 8 owns the x-th eighth of the tile columns; its
// workgroups take units u = (run, column) in turn, the columns of one run of
// planes first, so the tiles beside a column are walked by the group's other
// workgroups at about the same time.  The window of plane z + 2 is fetched
// into registers while plane z is computed.
//
// Measured on the 12.6M-row channel (binary64, m = 16) it is slower than
// gspmv_tiles: the 64-row march tiles that keep three windows and four
// workgroups per CU in LDS cost four times the tile-staging round trips of a
// 256-row tile, more than the plane gathers it saves (the GSpMV with every
// gather local takes 840 us against 1003 us, an upper bound on any staging).
// It is selected only by MRHS_MARCH=1.
#ifndef MRHS_MARCH_ROWS
#define MRHS_MARCH_ROWS 64
#endif
template <typename T, int M>
struct MarchShape {
    using S = Shape<T, M>;
    static constexpr int PASSES = S::RPP >= MRHS_MARCH_ROWS ? 1 : MRHS_MARCH_ROWS / S::RPP;
    static constexpr int TR = S::RPP * PASSES;         // rows per march tile
    static constexpr int LDW = S::G * S::VW;            // LDS row stride of a window (elements)
    static constexpr int WIN = TR * LDW;                // elements per window
    static constexpr int NZCAP = TR * MRHS_NZ_PER_ROW;  // staged nonzeros per tile
};

// The three windows of the ring (planes z - 1, z, z + 1): first row, row
// count (0 for a plane that does not exist) and element offset in LDS.
struct MarchWin {
    int32_t bp, np, op;
    int32_t bc, nc, oc;
    int32_t bn, nn, on;
};

template <typename T, int M, class Op>
__device__ __forceinline__ void march_load(const CsrView<T> &A, const Op &op, const typename Op::Lane &ln,
                                           bool lane_on, int g, int rl, int32_t base, int cnt, T *w)
{
    using S = Shape<T, M>;
    using MS = MarchShape<T, M>;
#pragma unroll
    for (int p = 0; p < MS::PASSES; ++p) {
        const int row_l = p * S::RPP + rl;
        if (lane_on && row_l < cnt) {
            T x[S::VW];
            op.gather(ln, base + row_l, g, x);
            Vec<T, S::VW>::store(w + row_l * MS::LDW + g * S::VW, x);
        }
    }
}

// The same rows loaded into registers (issued early, written to LDS a step
// later so their latency hides behind the step's own loads).
template <typename T, int M, class Op>
__device__ __forceinline__ void march_fetch(const Op &op, const typename Op::Lane &ln, bool lane_on, int g, int rl,
                                            int32_t base, int cnt, T (&xr)[MarchShape<T, M>::PASSES][Shape<T, M>::VW])
{
    using S = Shape<T, M>;
    using MS = MarchShape<T, M>;
#pragma unroll
    for (int p = 0; p < MS::PASSES; ++p) {
        const int row_l = p * S::RPP + rl;
        if (lane_on && row_l < cnt)
            op.gather(ln, base + row_l, g, xr[p]);
    }
}

template <typename T, int M>
__device__ __forceinline__ void march_put(bool lane_on, int g, int rl, int cnt,
                                          const T (&xr)[MarchShape<T, M>::PASSES][Shape<T, M>::VW], T *w)
{
    using S = Shape<T, M>;
    using MS = MarchShape<T, M>;
#pragma unroll
    for (int p = 0; p < MS::PASSES; ++p) {
        const int row_l = p * S::RPP + rl;
        if (lane_on && row_l < cnt)
            Vec<T, S::VW>::store(w + row_l * MS::LDW + g * S::VW, xr[p]);
    }
}

// Workgroup barrier that waits for this thread's LDS operations only, so
// global loads issued before it stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// row_product with the windows of the ring: entries in a window read LDS,
// the others gather; all of a batch's loads are issued before any is used.
template <typename T, int M, class Op, typename PI, typename PV>
__device__ __forceinline__ void row_product_march(PI cis, PV vas, int j0, int j1, int g, const Op &op,
                                                  const typename Op::Lane &ln, const T *s_x, const MarchWin &mw,
                                                  T *sum)
{
    using S = Shape<T, M>;
    using MS = MarchShape<T, M>;
    constexpr int NB = MRHS_GATHER_BATCH;
    for (int j = j0; j < j1; j += NB) {
        int32_t c[NB];
        T a[NB], x[NB][S::VW];
        bool ok[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            ok[k] = j + k < j1;
            const int jj = ok[k] ? j + k : j1 - 1;
            c[k] = cis[jj];
            a[k] = vas[jj];
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            int off = -1;
            const int32_t dc = c[k] - mw.bc, dp = c[k] - mw.bp, dn = c[k] - mw.bn;
            if (static_cast<uint32_t>(dc) < static_cast<uint32_t>(mw.nc))
                off = mw.oc + dc * MS::LDW;
            else if (static_cast<uint32_t>(dp) < static_cast<uint32_t>(mw.np))
                off = mw.op + dp * MS::LDW;
            else if (static_cast<uint32_t>(dn) < static_cast<uint32_t>(mw.nn))
                off = mw.on + dn * MS::LDW;
            if (off >= 0)
                Vec<T, S::VW>::load(s_x + off + g * S::VW, x[k]);
            else
                op.gather(ln, c[k], g, x[k]);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                if (ok[k])
                    sum[v] += a[k] * x[k][v];
    }
}

// Rows per plane R = A.reach (a multiple of MS::TR), P = R / MS::TR tile
// columns, runs of ceil(planes / zc) planes.
template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_march(const CsrView<T> &A, const Op &op,
                                            Acc<T, Shape<T, M>::VW, Op::NDOT> &acc, int32_t zc)
{
    using S = Shape<T, M>;
    using MS = MarchShape<T, M>;
    __shared__ int32_t s_rp[MS::TR + 1];
    __shared__ __align__(16) int32_t s_ci[MS::NZCAP + 4];
    __shared__ __align__(16) T s_va[MS::NZCAP + 4];
    __shared__ __align__(16) T s_x[3 * MS::WIN];
    const int tid = threadIdx.x;
    const int g = S::lane_of(tid);
    const int rl = S::row_of(tid);
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = S::used(tid) && g < S::G && ln.on;
    const int32_t R = A.reach;
    const int32_t P = R / MS::TR;
    const int32_t planes = static_cast<int32_t>((static_cast<int64_t>(A.n) + R - 1) / R);
    const int32_t zlen = (planes + zc - 1) / zc;
    const int grp = blockIdx.x % kGroups;
    const int32_t lo = P * grp / kGroups;
    const int32_t cg = P * (grp + 1) / kGroups - lo;
    const int32_t gx = gridDim.x / kGroups;
    // window of plane z for column t: rows [z R + t TR, + TR) within [0, n)
    auto win_base = [&](int32_t z, int32_t t) { return static_cast<int64_t>(z) * R + static_cast<int64_t>(t) * MS::TR; };
    auto win_cnt = [&](int64_t base) {
        return base < A.n ? static_cast<int32_t>(min(static_cast<int64_t>(MS::TR), A.n - base)) : 0;
    };
    for (int32_t u = blockIdx.x / kGroups; u < cg * zc; u += gx) {
        const int32_t t = lo + u % cg;
        const int32_t z0 = (u / cg) * zlen;
        const int32_t z1 = min(planes, z0 + zlen);
        // ring: planes z0 - 1 (when it exists), z0 and z0 + 1 first; at every
        // step plane z + 2 is fetched into registers before the rows are
        // computed and written, after the step, into the slot plane z - 1 held
        MarchWin mw;
        mw.op = 0;
        mw.oc = MS::WIN;
        mw.on = 2 * MS::WIN;
        {
            const int64_t b = win_base(z0 - 1, t);
            mw.bp = z0 > 0 ? static_cast<int32_t>(min(b, static_cast<int64_t>(A.n))) : 0;
            mw.np = z0 > 0 ? win_cnt(b) : 0;
            march_load<T, M>(A, op, ln, lane_on, g, rl, mw.bp, mw.np, s_x + mw.op);
            const int64_t c = win_base(z0, t);
            mw.bc = static_cast<int32_t>(min(c, static_cast<int64_t>(A.n)));
            mw.nc = win_cnt(c);
            march_load<T, M>(A, op, ln, lane_on, g, rl, mw.bc, mw.nc, s_x + mw.oc);
            const int64_t d = win_base(z0 + 1, t);
            mw.bn = static_cast<int32_t>(min(d, static_cast<int64_t>(A.n)));
            mw.nn = z0 + 1 < planes ? win_cnt(d) : 0;
            march_load<T, M>(A, op, ln, lane_on, g, rl, mw.bn, mw.nn, s_x + mw.on);
        }
        T xr[MS::PASSES][S::VW];
        int32_t fb = 0, fn = 0;  // rows of the plane held in xr
        for (int32_t z = z0; z < z1; ++z) {
            const int64_t rb = win_base(z, t);
            if (rb >= A.n)
                break;  // the last, partial plane ends before this column
            const int32_t r0 = static_cast<int32_t>(rb);
            const int nr = min(MS::TR, A.n - r0);
            if (z > z0) {  // plane z + 1, fetched during the previous step
                mw.bn = fb;
                mw.nn = fn;
                march_put<T, M>(lane_on, g, rl, fn, xr, s_x + mw.on);
            }
            const Staged st = stage_csr<T, MS::NZCAP>(A, r0, nr, s_rp, s_ci, s_va);
            {
                const int64_t b = win_base(z + 2, t);
                fb = static_cast<int32_t>(min(b, static_cast<int64_t>(A.n)));
                fn = z + 2 < planes ? win_cnt(b) : 0;
                march_fetch<T, M>(op, ln, lane_on, g, rl, fb, fn, xr);
            }
            lds_barrier();
            const int32_t *lci = s_ci + st.lead;
            const T *lva = s_va + st.lead;
#pragma unroll 1
            for (int p = 0; p < MS::PASSES; ++p) {
                const int row_l = p * S::RPP + rl;
                if (lane_on && row_l < nr) {
                    const int j0 = s_rp[row_l] - st.z0;
                    const int j1 = s_rp[row_l + 1] - st.z0;
                    T sum[S::VW];
#pragma unroll
                    for (int v = 0; v < S::VW; ++v)
                        sum[v] = T(0);
                    if constexpr (has_pre<Op>::value) {
                        const typename Op::Pre pr = op.pre(ln, r0 + row_l, g);
                        if (st.staged)
                            row_product_march<T, M>(lci, lva, j0, j1, g, op, ln, s_x, mw, sum);
                        else
                            row_product_march<T, M>(A.ci + st.z0, A.va + st.z0, j0, j1, g, op, ln, s_x, mw, sum);
                        op.row(ln, r0 + row_l, g, sum, acc, pr);
                    } else {
                        if (st.staged)
                            row_product_march<T, M>(lci, lva, j0, j1, g, op, ln, s_x, mw, sum);
                        else
                            row_product_march<T, M>(A.ci + st.z0, A.va + st.z0, j0, j1, g, op, ln, s_x, mw, sum);
                        op.row(ln, r0 + row_l, g, sum, acc);
                    }
                }
            }
            __syncthreads();
            const int32_t free_slot = mw.op;
            mw.bp = mw.bc;
            mw.np = mw.nc;
            mw.op = mw.oc;
            mw.bc = mw.bn;
            mw.nc = mw.nn;
            mw.oc = mw.on;
            mw.on = free_slot;
        }
    }
}

// Products over matrices with long rows (the Galerkin operators of coarse
// multigrid levels carry 30-90 nonzeros per row): a wave takes one row at a
// time, its RW row slots of L lanes take every RW-th entry of the row (NB at
// a time, all gathers in flight together), a butterfly over the slots adds the
// partial sums, and slot 0 runs the op's epilogue.  Workgroup b belongs to
// XCD group b % 8, which owns a contiguous eighth of the rows.  Only for row
// layouts whose lanes fill the wave (L a power of two).
template <typename T, int M, class Op>
__device__ __forceinline__ void gspmv_rows_split(const CsrView<T> &A, const Op &op,
                                                 Acc<T, Shape<T, M>::VW, Op::NDOT> &acc)
{
    using S = Shape<T, M>;
    static_assert(S::POW2 && S::RW * S::L == 64, "row slots must fill the wave");
    constexpr int NB = MRHS_GATHER_BATCH;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane % S::L;
    const int slot = lane / S::L;
    const typename Op::Lane ln = op.lane(g < S::G ? g : 0);
    const bool lane_on = g < S::G && ln.on;
    const int grp = blockIdx.x % kGroups;
    const int32_t q = blockIdx.x / kGroups, gx = gridDim.x / kGroups;
    const int32_t lo = static_cast<int32_t>(static_cast<int64_t>(A.n) * grp / kGroups);
    const int32_t hi = static_cast<int32_t>(static_cast<int64_t>(A.n) * (grp + 1) / kGroups);
    const int32_t waves = kBlock / 64;
    for (int32_t row = lo + q * waves + (tid >> 6); row < hi; row += gx * waves) {
        const int32_t j0 = A.rp[row], j1 = A.rp[row + 1];
        T sum[S::VW];
#pragma unroll
        for (int v = 0; v < S::VW; ++v)
            sum[v] = T(0);
        [[maybe_unused]] typename pre_of<Op>::type pr{};
        if (lane_on) {
            if constexpr (has_pre<Op>::value) {
                if (slot == 0)
                    pr = op.pre(ln, row, g);
            }
            for (int32_t jb = j0 + slot; jb < j1; jb += S::RW * NB) {
                int32_t c[NB];
                T a[NB], x[NB][S::VW];
                bool ok[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const int32_t j = jb + k * S::RW;
                    ok[k] = j < j1;
                    const int32_t jj = ok[k] ? j : jb;
                    c[k] = A.ci[jj];
                    a[k] = A.va[jj];
                }
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    op.gather(ln, c[k], g, x[k]);
#pragma unroll
                for (int k = 0; k < NB; ++k)
#pragma unroll
                    for (int v = 0; v < S::VW; ++v)
                        if (ok[k])
                            sum[v] += a[k] * x[k][v];
            }
        }
#pragma unroll
        for (int off = S::L; off < 64; off <<= 1)
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                sum[v] += __shfl_xor(sum[v], off);
        if (lane_on && slot == 0) {
            if constexpr (has_pre<Op>::value)
                op.row(ln, row, g, sum, acc, pr);
            else
                op.row(ln, row, g, sum, acc);
        }
    }
}

// Elementwise pass over every row of this workgroup's tiles.
template <typename T, int M, class Op>
__device__ __forceinline__ void stream_tiles(int32_t n, const Op &op,
                                             Acc<T, Shape<T, M>::VW, Op::NDOT> &acc)
{
    using S = Shape<T, M>;
    const int tid = threadIdx.x;
    const int g = S::lane_of(tid);
    const int rl = S::row_of(tid);
    if (!S::used(tid) || g >= S::G)
        return;
    const typename Op::Lane ln = op.lane(g);
    if (!ln.on)
        return;
    const int32_t ntiles = static_cast<int32_t>((static_cast<int64_t>(n) + S::TR - 1) / S::TR);
    const TileRange tr = tile_range(ntiles);
    for (int32_t tile = tr.first; tile < tr.end; tile += tr.stride) {
        const int32_t r0 = tile * S::TR;
        const int nr = min(S::TR, n - r0);
#pragma unroll 2
        for (int p = 0; p < S::PASSES; ++p) {
            const int row_l = p * S::RPP + rl;
            if (row_l < nr)
                op.row(ln, r0 + row_l, g, acc);
        }
    }
}

// ---- cross-workgroup publication without device-wide fences ----------------
// The L2 of each XCD is not coherent with the others, so a device-scope fence
// must write back and invalidate a whole L2: a per-workgroup fence serialises
// badly.  Values that another workgroup must read are instead stored and
// loaded with agent-scope atomics (they bypass the non-coherent caches), and
// ordering against the ticket counter only needs each thread's own memory
// operations to have completed (vmcnt = 0) plus a workgroup-scope fence that
// keeps the compiler from reordering across it.
template <typename T>
struct Bits;
template <>
struct Bits<double> {
    using U = unsigned long long;
};
template <>
struct Bits<float> {
    using U = unsigned int;
};

template <typename T>
__device__ __forceinline__ void publish(T *p, T v)
{
    using U = typename Bits<T>::U;
    __hip_atomic_store(reinterpret_cast<U *>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T fetch_published(const T *p)
{
    using U = typename Bits<T>::U;
    return __builtin_bit_cast(T, __hip_atomic_load(reinterpret_cast<const U *>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT));
}

// vmcnt(0), expcnt/lgkmcnt unconstrained (gfx9 s_waitcnt encoding)
#define MRHS_WAIT_VMEM() __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8))

__device__ __forceinline__ void release_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    MRHS_WAIT_VMEM();
}

__device__ __forceinline__ void acquire_order()
{
    MRHS_WAIT_VMEM();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ unsigned take_ticket(unsigned *t)
{
    return __hip_atomic_fetch_add(t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const int g = S::lane_of(tid);

    // sum the wave's rows lane by lane: a xor butterfly when rows are a power
    // of two of lanes wide, else a fixed shift-down tree over the RW rows
    // (idle lanes past RW*L hold zeros)
    if constexpr (S::POW2) {
#pragma unroll
        for (int off = S::L; off < 64; off <<= 1)
#pragma unroll
            for (int d = 0; d < NDOT; ++d)
#pragma unroll
                for (int v = 0; v < S::VW; ++v)
                    acc.a[d][v] += __shfl_xor(acc.a[d][v], off);
    } else {
#pragma unroll
        for (int off = S::L; off < S::RW * S::L; off <<= 1)
#pragma unroll
            for (int d = 0; d < NDOT; ++d)
#pragma unroll
                for (int v = 0; v < S::VW; ++v) {
                    const T o = __shfl_down(acc.a[d][v], off);
                    if (lane + off < S::RW * S::L)
                        acc.a[d][v] += o;
                }
    }
    if (lane < S::L && g < S::G) {
#pragma unroll
        for (int d = 0; d < NDOT; ++d)
#pragma unroll
            for (int v = 0; v < S::VW; ++v)
                if (g * S::VW + v < M)  // the last lane may hold fewer columns
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
        publish(&rb.part[static_cast<size_t>(b) * V + tid], s);
        release_order();
    }
    __syncthreads();
    if (tid == 0)
        s_flag = take_ticket(&rb.tickets[grp]) == static_cast<unsigned>(gx - 1);
    __syncthreads();
    if (!s_flag)
        return;
    acquire_order();
    // this workgroup is the last of its group: sum the group's partials
    if (tid < TPV * V) {
        const int v = tid % V;
        const int k = tid / V;
        T s = T(0);
        // partials q = k, k + TPV, ... in that order; eight loads in flight
        // at a time (a load-then-add loop waits out one round trip each)
        constexpr int U8 = 8;
        for (int q0 = k; q0 < gx; q0 += U8 * TPV) {
            T w[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                const int q = q0 + u * TPV;
                w[u] = q < gx ? fetch_published(&rb.part[static_cast<size_t>(grp + q * kGroups) * V + v]) : T(0);
            }
#pragma unroll
            for (int u = 0; u < U8; ++u)
                if (q0 + u * TPV < gx)
                    s += w[u];
        }
        s_k[k][v] = s;
    }
    __syncthreads();
    if (tid < V) {
        T s = s_k[0][tid];
        for (int k = 1; k < TPV; ++k)
            s += s_k[k][tid];
        publish(&rb.gpart[grp * V + tid], s);
        release_order();
    }
    __syncthreads();
    if (tid == 0)
        s_flag = take_ticket(&rb.tickets[kGroups]) == static_cast<unsigned>(kGroups - 1);
    __syncthreads();
    if (!s_flag)
        return;
    acquire_order();
    if (tid < V) {
        T s = fetch_published(&rb.gpart[tid]);
#pragma unroll
        for (int x = 1; x < kGroups; ++x)
            s += fetch_published(&rb.gpart[x * V + tid]);
        s_tot[tid] = s;
    }
    if (tid <= kGroups)
        __hip_atomic_store(&rb.tickets[tid], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    op.finish(s_tot);
}

} // namespace mrhs
