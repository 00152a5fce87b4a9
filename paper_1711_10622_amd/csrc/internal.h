// Host-side internals of libmrhs: the matrix handle, error reporting, grid
// sizing and kernel launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>

#include "mrhs.h"
#include "ops.h"

struct mrhs_csr_s {
    int32_t n = 0;
    int64_t nnz = 0;
    uint32_t flags = 0;
    int device = 0;
    bool zero_diag = false;
    int32_t *rp = nullptr;    // [n+1]
    int32_t *ci = nullptr;    // [nnz]
    double *val = nullptr;    // [nnz] A
    double *valh = nullptr;   // [nnz] A D^-1
    float *val32 = nullptr;   // [nnz] RN32(A)
    float *valh32 = nullptr;  // [nnz] RN32(A D^-1)
    double *diag = nullptr;   // [n]
    double *dinv = nullptr;   // [n]
    int32_t reach = 0;        // median over rows of max(col - row), >= 0
    size_t bytes = 0;
    // MRHS_CSR_REORDER: the arrays above hold P A P^T (solver row i is the
    // caller's row perm[i]); the caller's own numbering is kept for gspmv
    int32_t *perm = nullptr;  // [n] device, null without reordering
    int32_t *urp = nullptr, *uci = nullptr;
    double *uval = nullptr;
    float *uval32 = nullptr;
    int32_t ureach = 0;
    // dictionary form of the solver arrays (CsrView): per value array (val,
    // valh, val32, valh32) either 16-bit codes over the offset table (at most
    // kDictOffs distinct offsets) or 32-bit codes holding the column (more
    // offsets), with the array's value table; neither (too many distinct
    // values) means products read the plain arrays
    int32_t *otab = nullptr;
    int32_t noffs = 0, ob = 0;
    uint16_t *code[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t *ccode[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t cbits[4] = {0, 0, 0, 0};
    void *vtab[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t nvals[4] = {0, 0, 0, 0};
};

namespace mrhs {

// Thread-local last-error message; returns s for convenience.
mrhs_status set_error(mrhs_status s, const char *fmt, ...);
void clear_error();

#define MRHS_HIP(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::mrhs::set_error(MRHS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Number of workgroups for a tile-looping kernel over n rows: enough to keep
// every CU at its occupancy limit, never more than there are tiles, rounded
// up to a multiple of kGroups.
int grid_for(const void *kernel, int64_t n, int tile_rows, int max_per_cu = 0);
int max_grid();  // upper bound of grid_for over all kernels (for buffer sizing)

template <typename T>
inline CsrView<T> view(const mrhs_csr_s &A, bool scaled);

// The view of value array k (0 val, 1 valh, 2 val32, 3 valh32), in its
// dictionary form when it has one.
template <typename T>
inline CsrView<T> view_of(const mrhs_csr_s &A, const T *va, int k)
{
    CsrView<T> v{A.rp, A.ci, va, A.n, A.reach, 0};
    if (A.code[k]) {
        v.code = A.code[k];
        v.otab = A.otab;
        v.vtab = static_cast<const T *>(A.vtab[k]);
        v.noffs = A.noffs;
        v.nvals = A.nvals[k];
        v.ob = A.ob;
    } else if (A.ccode[k]) {
        v.ccode = A.ccode[k];
        v.vtab = static_cast<const T *>(A.vtab[k]);
        v.nvals = A.nvals[k];
        v.cb = A.cbits[k];
    }
    return v;
}

template <>
inline CsrView<double> view<double>(const mrhs_csr_s &A, bool scaled)
{
    return scaled ? view_of<double>(A, A.valh, 1) : view_of<double>(A, A.val, 0);
}

template <>
inline CsrView<float> view<float>(const mrhs_csr_s &A, bool scaled)
{
    return scaled ? view_of<float>(A, A.valh32, 3) : view_of<float>(A, A.val32, 2);
}

// The matrix in the caller's numbering (gspmv): the handle's own arrays, or
// the kept originals of a reordered handle.
template <typename T>
inline CsrView<T> user_view(const mrhs_csr_s &A);

template <>
inline CsrView<double> user_view<double>(const mrhs_csr_s &A)
{
    return A.perm ? CsrView<double>{A.urp, A.uci, A.uval, A.n, A.ureach, 0} : view<double>(A, false);
}

template <>
inline CsrView<float> user_view<float>(const mrhs_csr_s &A)
{
    return A.perm ? CsrView<float>{A.urp, A.uci, A.uval32, A.n, A.ureach, 0} : view<float>(A, false);
}

// Reverse Cuthill-McKee permutation of the symmetrized pattern (reorder.hip):
// perm[new] = old.
void rcm_permutation(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *perm);

template <typename T, int M, class Op>
__global__ void __launch_bounds__(kBlock) k_gspmv(CsrView<T> A, Op op, RedBufs<T> rb)
{
    Acc<T, Shape<T, M>::VW, Op::NDOT> acc;
    acc.zero();
    gspmv_tiles<T, M>(A, op, acc);
    if constexpr (Op::NDOT > 0)
        grid_reduce<T, M, Op::NDOT>(acc, rb, op);
}

template <typename T, int M, class Op>
__global__ void __launch_bounds__(kBlock) k_gspmv_march(CsrView<T> A, Op op, RedBufs<T> rb, int32_t runs)
{
    Acc<T, Shape<T, M>::VW, Op::NDOT> acc;
    acc.zero();
    gspmv_march<T, M>(A, op, acc, runs);
    if constexpr (Op::NDOT > 0)
        grid_reduce<T, M, Op::NDOT>(acc, rb, op);
}

// Plane-march plan of a product over n rows with forward reach `reach` in
// tiles of tile_rows rows, for a kernel whose grid_for is `grid`: the number
// of plane runs (>= 1), or 0 when the march does not apply (no whole-tile
// plane of at least 16 tiles, or fewer than 8 planes).  The runs are chosen
// so that each group's (run, column) units fill whole rounds of its
// workgroups, discounted by the extra window each run loads first.
int32_t march_runs(int32_t n, int32_t reach, int tile_rows, int grid);

// MRHS_MARCH=1 runs every product over a grid operator as a plane march
// (measured slower than the tiled products at every block width, so off by
// default; kept to measure LDS staging of the gathered rows).
int march_mode();

template <typename T, int M, class Op>
__global__ void __launch_bounds__(kBlock) k_gspmv_split(CsrView<T> A, Op op, RedBufs<T> rb)
{
    Acc<T, Shape<T, M>::VW, Op::NDOT> acc;
    acc.zero();
    gspmv_rows_split<T, M>(A, op, acc);
    if constexpr (Op::NDOT > 0)
        grid_reduce<T, M, Op::NDOT>(acc, rb, op);
}

template <typename T, int M, class Op>
__global__ void __launch_bounds__(kBlock) k_stream(int32_t n, Op op, RedBufs<T> rb)
{
    Acc<T, Shape<T, M>::VW, Op::NDOT> acc;
    acc.zero();
    stream_tiles<T, M>(n, op, acc);
    if constexpr (Op::NDOT > 0)
        grid_reduce<T, M, Op::NDOT>(acc, rb, op);
}

// ---- optional per-launch timing (mrhs_trace_enable) ---------------------
// When enabled with period k, every k-th launch of each kernel class is
// bracketed by a pair of HIP events on its own stream; mrhs_trace_read
// aggregates the durations per class.  trace_begin returns -1 for launches
// that are not sampled.
extern int g_trace_every;
int trace_begin(hipStream_t s, const char *name, int elem_bytes, int m, int grid, bool windows = false);
void trace_end(int slot, hipStream_t s);

template <typename T, int M, class Op>
inline hipError_t launch_gspmv(const CsrView<T> &A, const Op &op, const RedBufs<T> &rb, hipStream_t s)
{
    if constexpr (Shape<T, M>::POW2 && long_rows_ok<Op>::value) {
        if (A.split) {  // long rows: one wave per row
            const void *fn = reinterpret_cast<const void *>(&k_gspmv_split<T, M, Op>);
            const int grid = grid_for(fn, A.n, kBlock / 64);
            const int slot = g_trace_every ? trace_begin(s, Op::kName, static_cast<int>(sizeof(T)), M, grid) : -1;
            hipLaunchKernelGGL((k_gspmv_split<T, M, Op>), dim3(grid), dim3(kBlock), 0, s, A, op, rb);
            if (slot >= 0)
                trace_end(slot, s);
            return hipGetLastError();
        }
    }
    if (A.reach > 0 && A.reach % MarchShape<T, M>::TR == 0 && march_mode()) {
        const void *fm = reinterpret_cast<const void *>(&k_gspmv_march<T, M, Op>);
        const int grid = grid_for(fm, A.n, MarchShape<T, M>::TR);
        const int32_t runs = march_runs(A.n, A.reach, MarchShape<T, M>::TR, grid);
        if (runs > 0) {
            const int slot =
                g_trace_every ? trace_begin(s, Op::kName, static_cast<int>(sizeof(T)), M, grid, true) : -1;
            hipLaunchKernelGGL((k_gspmv_march<T, M, Op>), dim3(grid), dim3(kBlock), 0, s, A, op, rb, runs);
            if (slot >= 0)
                trace_end(slot, s);
            return hipGetLastError();
        }
    }
    const void *fn = reinterpret_cast<const void *>(&k_gspmv<T, M, Op>);
    const int grid = grid_for(fn, A.n, Shape<T, M>::TR, max_per_cu<Op>::value);
    const int slot = g_trace_every ? trace_begin(s, Op::kName, static_cast<int>(sizeof(T)), M, grid) : -1;
    hipLaunchKernelGGL((k_gspmv<T, M, Op>), dim3(grid), dim3(kBlock), 0, s, A, op, rb);
    if (slot >= 0)
        trace_end(slot, s);
    return hipGetLastError();
}

template <typename T, int M, class Op>
inline hipError_t launch_stream(int32_t n, const Op &op, const RedBufs<T> &rb, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&k_stream<T, M, Op>);
    const int grid = grid_for(fn, n, Shape<T, M>::TR, max_per_cu<Op>::value);
    const int slot = g_trace_every ? trace_begin(s, Op::kName, static_cast<int>(sizeof(T)), M, grid) : -1;
    hipLaunchKernelGGL((k_stream<T, M, Op>), dim3(grid), dim3(kBlock), 0, s, n, op, rb);
    if (slot >= 0)
        trace_end(slot, s);
    return hipGetLastError();
}

// Calls f.template operator()<M>() for the runtime value m in [1, 16].
template <class F>
inline auto dispatch_m(int m, F &&f)
{
    switch (m) {
    case 1: return f.template operator()<1>();
    case 2: return f.template operator()<2>();
    case 3: return f.template operator()<3>();
    case 4: return f.template operator()<4>();
    case 5: return f.template operator()<5>();
    case 6: return f.template operator()<6>();
    case 7: return f.template operator()<7>();
    case 8: return f.template operator()<8>();
    case 9: return f.template operator()<9>();
    case 10: return f.template operator()<10>();
    case 11: return f.template operator()<11>();
    case 12: return f.template operator()<12>();
    case 13: return f.template operator()<13>();
    case 14: return f.template operator()<14>();
    case 15: return f.template operator()<15>();
    default: return f.template operator()<16>();
    }
}

// ---- classical AMG on the device (amg.hip) ------------------------------------
constexpr int kAmgMaxLevels = 25;

// One level of the hierarchy in device memory: A_l, A_l D_l1^-1 (the first
// smoothing sweep from x = 0 folded into the values), the l1-Jacobi
// reciprocals, and the transfers P_l (n_l x n_{l+1}) and R_l = P_l^T.
struct AmgLevelDev {
    int32_t n = 0, nnext = 0;
    int64_t nnz_a = 0, nnz_p = 0;
    CsrView<double> A{}, Ah{}, P{}, R{};
    double *dl1_inv = nullptr;
    // binary32 roundings of the values (same indices), made on first use
    CsrView<float> A32{}, Ah32{}, P32{}, R32{};
    float *dl1_inv32 = nullptr;
};

struct AmgDev {
    int nlev = 0;
    AmgLevelDev lev[kAmgMaxLevels];
    CsrView<double> cinv{};  // dense inverse of the coarsest operator, as a full CRS matrix
    CsrView<float> cinv32{};
    bool has32 = false;
};

// internal solve flag: AMG V-cycle in binary32 (block_bicgstab_amg with MRHS_MIXED)
constexpr uint32_t kAmgVc32 = 1u << 8;

struct Ctx;
struct AmgStepTable {
    hipError_t (*start)(Ctx &, uint32_t, bool);
    hipError_t (*iterate)(Ctx &, int);
    hipError_t (*check)(Ctx &);
    hipError_t (*finish)(Ctx &, uint32_t, bool);
};
const AmgStepTable &amg_table(int m);
// device bytes of the V-cycle's level buffers for an m-column block
size_t amg_vcycle_bytes(const AmgDev &H, int32_t m);

// ---- block solver engine (solver.hip) ---------------------------------------
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
    double *r, *p, *v, *t;
    double *r64;
    GcrBlocks gcr;
    float *r32, *p32, *v32, *t32, *y32;
    int32_t ldp64 = 0, ldp32 = 0;  // row stride of the r/v blocks: 2m interleaved, else m
    uint8_t *sgn32;
    const AmgDev *amg = nullptr;           // AMG-preconditioned iteration (else Jacobi)
    double *sv = nullptr, *ph = nullptr, *sh = nullptr;  // AMG: s, M^-1 p, M^-1 s
    char *vcws = nullptr;                  // AMG: V-cycle level buffers
    bool vc32 = false;                     // AMG: V-cycle in binary32
    bool merged = false;                   // binary64 Jacobi: two kernels per iteration
    double *r2 = nullptr, *v2 = nullptr, *p2 = nullptr;  // merged: the other r/v/p set
};

struct StepTable {
    hipError_t (*f64_start)(Ctx &, uint32_t, bool);
    hipError_t (*f64_iterate)(Ctx &, int);
    hipError_t (*f64_check)(Ctx &);
    hipError_t (*finish)(Ctx &, uint32_t, bool, bool);
    hipError_t (*mixed_start)(Ctx &, uint32_t, bool);
    hipError_t (*mixed_step)(Ctx &, uint32_t, const int32_t *, const int32_t *);
    hipError_t (*mixed_check)(Ctx &, uint32_t);
    hipError_t (*mixed_cast)(Ctx &);
    hipError_t (*inner_iterate)(Ctx &, int);
};

// m column slots over one matrix, with blocks B (right-hand sides) and X
// (solutions) of n x m in device memory and a workspace of workspace_bytes().
// start() admits columns (their B, and X when x0, must be in place), advance()
// runs one round, finish() forms the returned x and its residual for
// finished columns.  Not thread-safe; one engine per host thread.
class Engine {
  public:
    static size_t workspace_bytes(const mrhs_csr_s &A, int32_t m, uint32_t flags, const AmgDev *amg = nullptr);
    // host_ctl: host memory for the mirror of the control block, or null to
    // allocate pinned memory on the first reset(); amg: precondition with
    // this hierarchy's V-cycle instead of Jacobi (binary64 only)
    Engine(const mrhs_csr_s &A, int m, uint32_t flags, void *ws, const double *B, double *X, hipStream_t s,
           Ctl *host_ctl = nullptr, const AmgDev *amg = nullptr);
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;
    mrhs_status reset();
    mrhs_status start(uint32_t cmask, const double *tol, const int32_t *maxit, bool x0);
    mrhs_status advance(bool *busy);  // reads the column states, then enqueues one round
    mrhs_status finish(uint32_t cmask);
    mrhs_status read_status();
    mrhs_status read_ctl();
    const Ctl &host() const { return *host_; }
    uint32_t terminal_mask() const;  // per the last read states
    static bool terminal(int32_t st);
    int m() const { return m_; }

  private:
    const mrhs_csr_s &A_;
    int m_;
    bool mixed_, nullspace_;
    hipStream_t s_;
    const StepTable *T_;
    const AmgStepTable *AT_ = nullptr;
    Ctx c_{};
    unsigned *tickets_ = nullptr;
    Ctl *host_ = nullptr;
    bool own_host_ = false;
    int chunk_ = 16, ndirs_ = kGcrMax, max_outer_ = 500;
    int amg_chunk_ = 2;  // iterations between polls with the AMG preconditioner
    int col_steps_[kMaxM] = {};  // refinement steps of each column since its admission (slot = steps % ndirs)
    double tol_in_ = 0.2;
    double outer_batch_ = 1.0;  // share of a block's active columns that triggers a refinement step
    int outer_wait_ = 0;        // ... or this many iterations waited by a column, whichever first
    int mixed_chunk_ = 8;       // inner iterations between polls (mixed precision)
    int stag_window_ = kStagWindow;
    int waited_ = 0;
};

mrhs_status column_status(int32_t st);
int env_int(const char *name, int dflt, int lo, int hi);
double env_double(const char *name, double dflt);
int gcr_dirs();

struct SolveParams {
    int32_t m;
    double tol;
    int32_t maxit;
    uint32_t flags;
};

// Copies between a caller's n x m block (caller's row numbering) and an
// n x w solver block (w >= m; row i is the caller's row perm[i], or row i
// when perm is NULL; columns m..w-1 zero), and the bytes of such a block
// rounded up to the workspace alignment.
hipError_t to_solver(double *sv, const double *us, const int32_t *perm, int32_t n, int w, int m, hipStream_t s);
hipError_t to_user(double *us, const double *sv, const int32_t *perm, int32_t n, int w, int m, hipStream_t s);
size_t padded_block_bytes(int32_t n, int w);

size_t solve_workspace_bytes(const mrhs_csr_s &A, int32_t m, uint32_t flags, const AmgDev *amg = nullptr);

// The device view and device bytes of a hierarchy (amg.hip); amg_make32
// adds the binary32 roundings of its values once.
const AmgDev *amg_dev_of(mrhs_amg H);
size_t amg_bytes_of(mrhs_amg H);
mrhs_status amg_make32(mrhs_amg H);
// host_ctl and amg as for Engine
mrhs_status block_solve(const mrhs_csr_s &A, const double *B, double *X, const SolveParams &p,
                        void *ws, size_t ws_bytes, hipStream_t s, mrhs_col_info *info, Ctl *host_ctl = nullptr,
                        const AmgDev *amg = nullptr);

} // namespace mrhs
