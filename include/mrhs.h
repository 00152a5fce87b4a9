/*
 * mrhs.h -- block multi-right-hand-side pressure-Poisson solver for MI355X
 * (gfx950).  C ABI of libmrhs.so.
 *
 * Method: B. I. Krasnopolsky, "An Approach for Accelerating Incompressible
 * Turbulent Flow Simulations Based on Simultaneous Modelling of Multiple
 * Ensembles" (arXiv 1711.10622).  m flow realizations share one pressure
 * matrix, so their pressure-Poisson systems form one SLAE with m right-hand
 * sides (Section 2.2); its cost is dominated by the generalized sparse
 * matrix-vector product Y = A X over a block of m vectors (Section 2.3,
 * Figure 1), which reads the matrix once for all m columns.
 *
 * Conventions for every call:
 *  - Every call returns an mrhs_status.  No exception crosses the ABI.  On
 *    failure mrhs_last_error() returns a message for the calling thread.
 *  - A matrix is general CRS: row offsets int32[n+1] (row_ptr[0] == 0,
 *    non-decreasing, row_ptr[n] == nnz), column indices int32[nnz] in
 *    [0, n), values binary64[nnz].  Column order inside a row is free and a
 *    repeated column adds (the Figure 1 loop sums every stored entry); an
 *    empty row yields 0.
 *  - A block X of m vectors is n x m, row-interleaved: X[i*m + l] is row i
 *    of vector l (the m values of a row lie together, the block layout of
 *    Section 2.3).
 *  - 1 <= m <= 16.  Device pointers are HIP device memory of the current
 *    device, 16-byte aligned (EINVAL otherwise); a stream argument of NULL
 *    means the null stream.
 *  - Calls on one matrix handle from several host threads must be
 *    serialised by the caller, except the solve server, which is
 *    thread-safe.
 */
#ifndef MRHS_H
#define MRHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRHS_OK = 0,
    MRHS_EAGAIN = 1,          /* solve_server_poll: not finished yet */
    MRHS_EINVAL = -1,         /* invalid argument or matrix */
    MRHS_ENOMEM = -2,         /* device or host allocation failed */
    MRHS_EDEVICE = -3,        /* a HIP call failed */
    MRHS_ENOCONV = -4,        /* maxit reached; X holds the last iterate */
    MRHS_EBREAKDOWN = -5,     /* BiCGStab breakdown persisted after restarts */
    MRHS_EBUDGET = -6,        /* request can never fit the server's budget */
    MRHS_ESHUTDOWN = -7,      /* server is shutting down */
    MRHS_ENOTFOUND = -8       /* unknown ticket or matrix id */
} mrhs_status;

/* element type of a block (gspmv_ex) */
enum { MRHS_F64 = 0, MRHS_F32 = 1 };

/* csr_create flags */
#define MRHS_CSR_NULLSPACE_CONST 1u /* A*1 = 0 (pure Neumann/periodic): solves
                                       return x with its mean removed */
#define MRHS_CSR_REORDER 2u         /* the solvers work on P A P^T, P the
                                       permutation of csr_reorder_permutation;
                                       every call keeps the caller's numbering */

/* block_bicgstab_ex flags */
#define MRHS_X0_GIVEN 1u   /* X holds the initial guess on entry */
#define MRHS_MIXED 2u      /* FP32 inner BiCGStab inside FP64 refinement */

typedef struct mrhs_csr_s *mrhs_csr;
typedef struct mrhs_server_s *mrhs_server;
typedef struct mrhs_grid_s *mrhs_grid;

/* Per-column outcome of a solve. */
typedef struct {
    int32_t iters;    /* BiCGStab iterations (inner iterations in total for
                         MRHS_MIXED) */
    int32_t restarts; /* restarts from the true residual */
    int32_t outer;    /* refinement steps (MRHS_MIXED), else 0 */
    int32_t status;   /* mrhs_status of this column */
    double relres;    /* ||b - A x||_2 / ||b||_2 in binary64, recomputed from
                         the returned x (0 when b = 0) */
} mrhs_col_info;

typedef struct {
    double p50_ms, p99_ms;   /* request latency, submit to completion */
    double rhs_per_s;        /* completed right-hand sides per second since
                                the first submit */
    int64_t submitted;       /* requests */
    int64_t completed;       /* requests */
    int64_t queued;          /* requests waiting for admission */
    int64_t rhs_completed;   /* right-hand sides */
    size_t admitted_bytes;   /* device bytes held by admitted work */
} mrhs_server_stats;

/* Message describing the last failure on the calling thread ("" if none). */
const char *mrhs_last_error(void);

/* Library version string. */
const char *mrhs_version(void);

/*
 * Upload a CRS matrix (Section 2.3: row, col, val arrays).  The host arrays
 * are copied; the caller keeps ownership.  The handle owns device copies of
 * row_ptr, col_idx and val, plus what the solvers derive from them: the
 * diagonal and its inverse, the column-scaled matrix A D^-1 (the right
 * Jacobi preconditioner folded into the values) and binary32 roundings
 * (round-to-nearest-even) of val and of A D^-1.  With MRHS_CSR_REORDER the
 * solvers' arrays hold P A P^T and the handle also keeps the caller's arrays
 * (gspmv uses those) and the permutation; solves copy B into the solver's
 * numbering and X back (two extra n x m blocks of workspace).
 * EINVAL: n < 0, nnz out of range, a NULL array with n > 0, row_ptr[0] != 0,
 * decreasing row_ptr, row_ptr[n] != nnz, a column outside [0, n), or a
 * non-finite value.  A zero diagonal is accepted here and rejected by the
 * solvers.
 *
 * Dictionary form: for each value array with at most 2048 distinct values
 * the handle also stores one code per entry and the value table: a 16-bit
 * code (offset index and value index, with the offset table) when the
 * solvers' matrix has at most 32 distinct column offsets col - row (a
 * structured grid's stencil), else a 32-bit code (column and value index)
 * when the columns fit beside the value index.  The tiled products then
 * stream 2 or 4 bytes per entry instead of 4 + 8 (binary64) or 4 + 4
 * (binary32) and sum exactly the same values in the same order.  Building it
 * reads the derived arrays back and takes one pass over the entries per
 * array; the environment variable MRHS_CSR_DICT=0 turns it off.  See
 * csr_stream_bytes.
 */
mrhs_status csr_create(int32_t n, int64_t nnz, const int32_t *row_ptr,
                       const int32_t *col_idx, const double *val,
                       uint32_t flags, mrhs_csr *out);

/*
 * The row renumbering MRHS_CSR_REORDER applies, computed on the host with no
 * device involved: reverse Cuthill-McKee on the pattern of A + A^T (each
 * connected component from a pseudo-peripheral row, neighbours by increasing
 * degree, then index; the order reversed).  perm (host, n entries) receives
 * perm[new] = old.  A numbering without locality (randomly permuted rows)
 * makes every gather of a product fetch a cache line of its own; a banded
 * one lets the rows gathered by one tile share lines.  EINVAL for an invalid
 * pattern (as csr_create) or NULL arrays.
 */
mrhs_status csr_reorder_permutation(int32_t n, const int32_t *row_ptr,
                                    const int32_t *col_idx, int32_t *perm);

/* Free the handle and its device memory.  NULL is accepted. */
mrhs_status csr_destroy(mrhs_csr A);

/* Size of the matrix and the device bytes the handle holds. */
mrhs_status csr_info(mrhs_csr A, int32_t *n, int64_t *nnz, size_t *device_bytes);

/*
 * Bytes one tiled product streams from the matrix arrays (Section 2.3: the
 * matrix part of the GSpMV memory traffic): the row offsets plus, per entry,
 * a 2- or 4-byte code in the dictionary form or a 4-byte column index and a
 * value otherwise.  dtype MRHS_F64 or MRHS_F32; scaled != 0 for the solvers'
 * column-scaled matrix A D^-1, 0 for A.  gspmv of a handle made with
 * MRHS_CSR_REORDER reads the caller's arrays in plain form.  EINVAL: NULL
 * handle or output, unknown dtype.
 */
mrhs_status csr_stream_bytes(mrhs_csr A, int32_t dtype, int32_t scaled, int64_t *bytes);

/*
 * Y = A X (Section 2.3, Figure 1) for device blocks X, Y of m binary64
 * vectors on the null stream; returns when the product is enqueued.
 * EINVAL: m outside [1, 16], NULL pointers with n > 0, or X and Y sharing
 * any byte of their n x m blocks.
 */
mrhs_status gspmv(mrhs_csr A, const double *X, double *Y, int32_t m);

/*
 * As gspmv, on a given stream, with the element type dtype: MRHS_F64, or
 * MRHS_F32 (binary32 blocks and the binary32 rounding of val, products
 * accumulated in binary32).
 */
mrhs_status gspmv_ex(mrhs_csr A, int32_t dtype, const void *X, void *Y,
                     int32_t m, void *hip_stream);

/*
 * Solve A X = B for a device block B of m right-hand sides (Section 2.2:
 * one matrix, m independent realizations), each column by BiCGStab with a
 * right Jacobi preconditioner; columns run concurrently and share every
 * matrix read.  Column l stops when ||b_l - A x_l|| <= tol ||b_l|| holds for
 * the recomputed true residual.  Uses the null stream and blocks until done.
 * Returns OK only if every column converged, else the worst column status.
 *
 * The shadow residual r^ of the binary64 iteration (any vector not orthogonal
 * to the initial residual serves) is the same for every column and every
 * restart: row i holds
 * 2 u_i 2^-53 - 1 with u_i the top 53 bits of output number i (counting from
 * 0) of the SplitMix64 generator seeded with MRHS_SHADOW_SEED, i.e. of
 * mix(MRHS_SHADOW_SEED + (i + 1) * 0x9E3779B97F4A7C15).  It is generated
 * where it is used and never stored; i counts the rows the solver works on
 * (those of P A P^T for a matrix created with MRHS_CSR_REORDER).  The binary32 inner solves of MRHS_MIXED
 * (short solves restarted at every refinement step) take r^ = the signs (+1,
 * or -1 for a negative entry) of their own initial residual.
 */
#define MRHS_SHADOW_SEED 17110622ull
mrhs_status block_bicgstab(mrhs_csr A, const double *B, double *X, int32_t m,
                           double tol, int32_t maxit);

/*
 * Full form.  flags: MRHS_X0_GIVEN, MRHS_MIXED.  workspace: device memory of
 * at least block_bicgstab_workspace_size() bytes owned by the caller, or NULL
 * to let the library allocate and free it.  info: host array of m entries or
 * NULL.  Blocks the calling thread until the solve is done.  EINVAL when B
 * and X, or the workspace and either of them, share any byte.
 */
mrhs_status block_bicgstab_ex(mrhs_csr A, const double *B, double *X, int32_t m,
                              double tol, int32_t maxit, uint32_t flags,
                              void *workspace, size_t ws_bytes, void *hip_stream,
                              mrhs_col_info *info);

/* Bytes of device workspace block_bicgstab_ex needs for (A, m, flags). */
mrhs_status block_bicgstab_workspace_size(mrhs_csr A, int32_t m, uint32_t flags,
                                          size_t *bytes);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): block_bicgstab_ex with
 * the workspace taken from a fixed device array of the library,
 * MRHS_NOALLOC_SCRATCH_BYTES long, that every GPU the library runs on holds
 * until the process ends.  The call allocates no device or pinned host memory
 * (with kernel timing, mrhs_trace_enable, off).  B and X are caller-owned
 * device blocks as for block_bicgstab_ex, on the current device, which must
 * be the matrix's; flags and info as there; the call blocks until the solve
 * is done.  EINVAL (nothing launched) when block_bicgstab_workspace_size for
 * (A, m, flags) exceeds MRHS_NOALLOC_SCRATCH_BYTES.  Every call on one GPU
 * uses that GPU's one array: calls that overlap in time on the same GPU (from
 * several threads or streams) race and must be serialised by the caller.
 */
#define MRHS_NOALLOC_SCRATCH_BYTES 67108864u /* 64 MiB */
mrhs_status block_bicgstab_noalloc(mrhs_csr A, const double *B, double *X, int32_t m,
                                   double tol, int32_t maxit, uint32_t flags,
                                   void *hip_stream, mrhs_col_info *info);

/*
 * Solve server: continuous batching of pressure solves from independent
 * ensemble members (Section 2: every realization needs the same operator with
 * its own right-hand side).  Registered matrices stay resident on the device.
 * Each matrix has one block of 16 column slots; submitted right-hand sides
 * join the block as slots free up (between rounds of iterations) and leave it
 * as soon as their column has converged, so requests that arrive while others
 * are being solved share the matrix reads of those already running.  Every
 * column's arithmetic is independent of the other columns in its block.
 * Different matrices are solved by their own host thread on their own stream
 * and overlap on the device.
 *
 * Device memory is admitted against hbm_budget_bytes: registered matrices
 * (their csr_info device bytes) plus the engine of every matrix that has work
 * (its block workspace).  Matrices waiting for engine memory get it in the
 * order they asked; while one waits, the others admit no new columns, finish
 * the ones in flight and give their engine memory back, so under a tight
 * budget the matrices take turns, one batch at a time.  All functions are
 * thread-safe.
 */
#define MRHS_SERVER_MIXED 1u /* binary32 inner solves with binary64 refinement */
#define MRHS_SERVER_AMG 2u   /* BiCGStab with the classical AMG preconditioner
                                (as block_bicgstab_amg); every matrix gets its
                                hierarchy at registration; with
                                MRHS_SERVER_MIXED the V-cycle runs in binary32 */

/* Create a server.  flags: 0 (binary64 Jacobi solves), MRHS_SERVER_MIXED,
 * MRHS_SERVER_AMG or both. */
mrhs_status solve_server_create(size_t hbm_budget_bytes, uint32_t flags,
                                mrhs_server *out);

/*
 * Make matrix A servable; *matrix_id names it in submits.  A must outlive
 * the server.  EBUDGET unless all registered matrices, A, and the largest
 * engine among them (A's included) fit the budget together, which is what
 * lets every matrix run once the other engines are released; EINVAL for an
 * empty matrix or a zero diagonal entry.  With MRHS_SERVER_AMG the matrix's
 * hierarchy is built here (amg_create defaults), counted as resident bytes
 * and freed with the server.
 */
mrhs_status solve_server_register(mrhs_server S, mrhs_csr A, int32_t *matrix_id);

/*
 * Queue k >= 1 right-hand sides B (host memory, n x k row-major: B[i*k + j]
 * is row i of right-hand side j) for matrix_id, each solved to
 * ||b - A x|| <= tol ||b|| within maxit iterations.  B is copied; the caller
 * may free it on return.  *ticket identifies the request.  ENOTFOUND for an
 * unknown matrix id; ESHUTDOWN after solve_server_destroy has begun.
 */
mrhs_status solve_server_submit(mrhs_server S, int32_t matrix_id, const double *B,
                                int32_t k, double tol, int32_t maxit,
                                uint64_t *ticket);

/*
 * EAGAIN while the request is in progress.  When it is complete: copies the
 * solutions into X (host memory, n x k row-major, may be NULL) and the k
 * per-column outcomes into info (may be NULL), forgets the ticket, and
 * returns OK if every column converged, else the worst column status.
 * ENOTFOUND for an unknown (or already collected) ticket.
 */
mrhs_status solve_server_poll(mrhs_server S, uint64_t ticket, double *X,
                              mrhs_col_info *info);

/* Latency percentiles over completed requests, throughput and occupancy. */
mrhs_status solve_server_stats(mrhs_server S, mrhs_server_stats *out);

/* Stop the serving threads (work in progress is abandoned) and free the
 * server.  NULL is accepted. */
mrhs_status solve_server_destroy(mrhs_server S);

/*
 * Ensemble projection step (Section 2.2, eqs. (3)-(4)): m preliminary
 * velocity fields u* on one staggered channel grid give m pressure
 * right-hand sides, solved together by block_bicgstab, and the pressures
 * correct the m fields to divergence-free ones.
 *
 * Grid: nx x ny x nz cells (x fastest), periodic in x and z, walls at the y
 * faces y_faces[0] and y_faces[ny] (host array of ny + 1 strictly increasing
 * coordinates), uniform spacings dx and dz, and optional solid cells
 * (solid: host array of nx*ny*nz bytes, nonzero = solid, or NULL).  Fluid
 * cells carry the pressure unknowns in natural order, as the matching
 * channel pressure matrix numbers its rows: x-faces couple with dy_j dz / dx,
 * y-faces with dx dz / (yc_j - yc_{j-1}), z-faces with dx dy_j / dz (yc the
 * cell centres), so that D G = -A with D and G below.
 *
 * Face blocks (device, row-interleaved, rows x m binary64, 16-byte aligned):
 *   U: nz*ny*nx rows, row (k*ny + j)*nx + i = x-face west of cell (i, j, k);
 *   V: nz*(ny+1)*nx rows, row (k*(ny+1) + j)*nx + i = y-face below cell
 *      (i, j, k), j = 0..ny (rows j = 0 and j = ny lie on the walls);
 *   W: nz*ny*nx rows, row (k*ny + j)*nx + i = z-face behind cell (i, j, k).
 * Faces on a wall or next to a solid cell are closed: no flux passes them,
 * projection_rhs ignores their values and projection_correct leaves them.
 * Cell blocks (B, P): n_fluid rows x m.  The blocks of one call must not
 * share any byte (EINVAL).  Calls are enqueued on hip_stream (NULL = the
 * null stream) and return at once.
 */
mrhs_status grid_create(int32_t nx, int32_t ny, int32_t nz, double dx, double dz,
                        const double *y_faces, const uint8_t *solid, mrhs_grid *out);
mrhs_status grid_destroy(mrhs_grid G);
/* Fluid cells, all cells and y-face rows of the grid (NULL outputs skipped). */
mrhs_status grid_info(mrhs_grid G, int32_t *n_fluid, int64_t *cells, int64_t *v_faces);

/*
 * B = -(1/tau) D(U, V, W) for m fields: D is the volume-integrated discrete
 * divergence, sum over a fluid cell's open faces of area times the outward
 * normal velocity.  tau = -1 gives D itself.  EINVAL for tau = 0.
 */
mrhs_status projection_rhs(mrhs_grid G, const double *U, const double *V, const double *W,
                           double tau, double *B, int32_t m, void *hip_stream);

/*
 * U -= tau G P, V -= tau G P, W -= tau G P on every open face: the pressure
 * difference across the face over the distance between the two cell centres.
 */
mrhs_status projection_correct(mrhs_grid G, double *U, double *V, double *W,
                               const double *P, double tau, int32_t m, void *hip_stream);

/*
 * Classical algebraic multigrid, the preconditioner of the paper's pressure
 * solver (BiCGStab with classical AMG, Section 4.1), for blocks of m
 * right-hand sides: every level's smoothing, restriction and prolongation is
 * a product over an n_l x m row-interleaved block, so the m columns share
 * every matrix read of every level.
 *
 * Construction (Ruge-Stueben): entries sorted and repeated columns summed;
 * j != i is a strong connection of row i when -a_ij >= theta max_{k != i}
 * (-a_ik) > 0; C/F splitting by the first pass of Ruge and Stueben (largest
 * measure first, smallest index on ties); direct interpolation from the strong
 * C neighbours; Galerkin coarse operators P^T A P; levels until at most
 * max_coarse rows, no useful coarsening (none or more than 0.9 of the rows
 * coarse) or max_levels levels; the coarsest level applies the dense inverse
 * of A_c (plus s 1 1^T, s = mean diagonal / n_c, for a matrix created with
 * MRHS_CSR_NULLSPACE_CONST).  V-cycle: one l1-Jacobi sweep
 * (x <- x + D^-1 (b - A x), D = diag of the rows' absolute sums) before and
 * one after the coarse correction, from x = 0.
 */
typedef struct mrhs_amg_s *mrhs_amg;

/* what amg_level_copy copies */
enum { MRHS_AMG_OPERATOR = 0, MRHS_AMG_PROLONGATION = 1, MRHS_AMG_SPLIT = 2 };

/*
 * Build the hierarchy of A on A's device (setup on the host, then upload).
 * theta <= 0, max_coarse <= 0, max_levels <= 0 select the defaults 0.25,
 * 256 and 25 (at most 25).  A must outlive the hierarchy.  For a matrix
 * created with MRHS_CSR_REORDER the hierarchy is that of P A P^T (its levels,
 * as amg_level_copy returns them, are in that numbering); amg_vcycle and
 * block_bicgstab_amg still take and return blocks in the caller's numbering.
 * EINVAL for an
 * empty matrix, a zero diagonal entry, theta >= 1 or a singular coarsest
 * operator; ENOMEM / EDEVICE for device failures.
 */
mrhs_status amg_create(mrhs_csr A, double theta, int32_t max_coarse,
                       int32_t max_levels, mrhs_amg *out);
mrhs_status amg_destroy(mrhs_amg H);
/* Levels, operator complexity (sum of the levels' nonzeros over A's) and the
 * device bytes the hierarchy holds (NULL outputs skipped). */
mrhs_status amg_info(mrhs_amg H, int32_t *levels, double *operator_complexity,
                     size_t *device_bytes);
/* Rows of level l, nonzeros of its operator and of its prolongation (0 on the
 * coarsest level). */
mrhs_status amg_level(mrhs_amg H, int32_t level, int32_t *rows, int64_t *nnz_a,
                      int64_t *nnz_p);
/*
 * Copy part of level l to host arrays sized by amg_level: MRHS_AMG_OPERATOR
 * (row_ptr[rows+1], col[nnz_a], val[nnz_a]), MRHS_AMG_PROLONGATION
 * (row_ptr[rows+1], col[nnz_p], val[nnz_p], columns are coarse rows) or
 * MRHS_AMG_SPLIT (col[rows] = 1 for C rows, 0 for F rows; row_ptr and val
 * unused).  Not for the coarsest level's prolongation or splitting (EINVAL).
 */
mrhs_status amg_level_copy(mrhs_amg H, int32_t level, int32_t what,
                           int32_t *row_ptr, int32_t *col, double *val);
/* Device workspace bytes of amg_vcycle for m columns. */
mrhs_status amg_vcycle_workspace_size(mrhs_amg H, int32_t m, size_t *bytes);
/*
 * X = M^-1 B, one V-cycle from X = 0, for device blocks B, X of m columns
 * (rows x m row-interleaved binary64), enqueued on hip_stream.  workspace:
 * device memory of amg_vcycle_workspace_size bytes.  EINVAL when B, X and the
 * workspace share any byte.
 */
mrhs_status amg_vcycle(mrhs_amg H, const double *B, double *X, int32_t m,
                       void *workspace, size_t ws_bytes, void *hip_stream);
/* Device workspace bytes of block_bicgstab_amg for m columns. */
mrhs_status block_bicgstab_amg_workspace_size(mrhs_amg H, int32_t m, size_t *bytes);
/*
 * block_bicgstab_ex for the hierarchy's matrix with the V-cycle as right
 * preconditioner instead of Jacobi (binary64): per column p^ = M^-1 p,
 * v = A p^, s = r - alpha v, s^ = M^-1 s, t = A s^, x += alpha p^ + omega s^,
 * with the same stopping tests, true-residual checks, restarts, shadow
 * residual and per-column outcomes.  flags: MRHS_X0_GIVEN, and MRHS_MIXED to
 * run the V-cycle in binary32 on binary32 roundings (nearest even) of every
 * level's values, made on the first such call and kept with the hierarchy:
 * p and s are rounded in and M^-1 p, M^-1 s widened out, while the
 * iteration, its products with A and x stay binary64.  workspace NULL:
 * allocated and freed by the call.
 */
mrhs_status block_bicgstab_amg(mrhs_amg H, const double *B, double *X, int32_t m,
                               double tol, int32_t maxit, uint32_t flags,
                               void *workspace, size_t ws_bytes, void *hip_stream,
                               mrhs_col_info *info);

/*
 * Memory ceilings.  Enqueues one streaming pass over a device buffer of
 * `bytes` (a positive multiple of 16, 16-byte aligned buffers) on hip_stream:
 * the attainable HBM rates against which the products and vector passes are
 * judged, since their time is set by the bytes they move (Section 2.3).
 *   MRHS_PROBE_READ / _READ_NT    read src (plain / nontemporal loads); dst
 *                                 is a device word that may be written
 *   MRHS_PROBE_WRITE / _WRITE_NT  write dst (plain / nontemporal stores);
 *                                 src is unused
 *   MRHS_PROBE_COPY / _COPY_NT    dst = src (plain / nontemporal loads and
 *                                 stores); the two must not overlap
 * EINVAL for an unknown kind, a bad size, NULL or misaligned buffers or
 * overlapping copies.  Returns when the pass is enqueued; time it with
 * events on the same stream.
 */
enum {
    MRHS_PROBE_READ = 0,
    MRHS_PROBE_READ_NT = 1,
    MRHS_PROBE_WRITE = 2,
    MRHS_PROBE_WRITE_NT = 3,
    MRHS_PROBE_COPY = 4,
    MRHS_PROBE_COPY_NT = 5
};
mrhs_status mrhs_stream_probe(int32_t kind, const void *src, void *dst, size_t bytes,
                              void *hip_stream);

/*
 * Kernel timing.  mrhs_trace_enable(k), k >= 1, clears the statistics and
 * starts bracketing every k-th launch of each kernel class (counted per
 * class, starting with the first) with a pair of HIP events on the launch's
 * own stream; k = 1 times every launch.  Each event pair adds a few
 * microseconds of idle time on the stream, which sampling keeps small.
 * mrhs_trace_enable(0) stops; k < 0 is EINVAL.  mrhs_trace_read waits for the
 * recorded events and writes a NUL-terminated JSON object
 * {"<kernel>/<f64|f32>/m<M>/g<grid>": {"seen", "launches", "total_ms",
 * "min_ms", "max_ms"}, ...} into buf (cap bytes; the grid is followed by
 * "w" for products that staged their gathered rows in LDS windows, the plane
 * march of grid operators that MRHS_MARCH=1 selects), where "seen" counts all
 * launches of the class and "launches" the timed ones; *len receives the
 * length needed (without the NUL).  EINVAL if the text did not fit (it is
 * truncated).  Not for use while other threads launch library kernels.
 */
mrhs_status mrhs_trace_enable(int every);
mrhs_status mrhs_trace_read(char *buf, size_t cap, size_t *len);

#ifdef __cplusplus
}
#endif

#endif /* MRHS_H */
