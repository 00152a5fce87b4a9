// Classical algebraic multigrid for the block solve: the paper's pressure
// solver is BiCGStab preconditioned by classical AMG (Section 4.1).  The
// hierarchy is built once per matrix on the host (amg_setup.hip); the V-cycle
// and the preconditioned iteration run on the device (amg.hip), every level's
// smoothing, restriction and prolongation as a product over an n_l x m
// row-interleaved block, so the m right-hand sides share every matrix read of
// every level.
//
// Construction (Ruge-Stueben; K. Stueben, "A review of algebraic multigrid",
// J. Comput. Appl. Math. 128, 2001):
//   * rows sorted by column, repeated columns summed;
//   * j != i is a strong connection of row i when -a_ij >= theta * m_i,
//     m_i = max_{k != i}(-a_ik) > 0;
//   * C/F splitting by the first pass of Ruge and Stueben: rows without a
//     strong connection either way are F; then the undecided row of largest
//     measure (the number of rows strongly connected to it that are undecided
//     or became F; smallest index on ties) becomes C, the undecided rows
//     strongly connected to it become F and raise the measure of the
//     undecided rows they are strongly connected to, and the undecided rows
//     it is strongly connected to lower theirs;
//   * direct interpolation from the strong C neighbours, weights
//     -(sum of the row's negative off-diagonals / sum of those to strong C
//     neighbours) a_ik / (a_ii + sum of the row's positive off-diagonals);
//   * Galerkin coarse operators A_c = P^T (A P) with R = P^T stored, every
//     product accumulated row by row in storage order;
//   * until at most max_coarse rows, no useful coarsening (n_c = 0 or
//     n_c > 0.9 n) or max_levels levels; the coarsest level applies the dense
//     inverse of A_c + s 1 1^T (s = mean diagonal / n_c when the operator's
//     null space is the constant vector, else 0);
//   * smoothing by one l1-Jacobi sweep before and one after the coarse
//     correction: x <- x + D_l1^-1 (b - A x), D_l1 = diag(sum_j |a_ij|).
#pragma once

#include <cstdint>
#include <vector>

namespace mrhs {
namespace amg {

constexpr double kTheta = 0.25;
constexpr int kMaxCoarse = 256;
constexpr int kMaxLevels = 25;

struct HostCsr {
    int32_t nr = 0, nc = 0;
    std::vector<int32_t> rp, ci;  // rp has nr + 1 entries
    std::vector<double> va;
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

struct HostLevel {
    HostCsr A;                    // the level's operator
    std::vector<double> dl1_inv;  // 1 / sum_j |a_ij| (0 for an empty row)
    std::vector<int8_t> cf;       // 1 = C row (empty on the coarsest level)
    HostCsr P, R;                 // prolongation n x n_c and R = P^T (empty on the coarsest level)
};

struct HostHierarchy {
    std::vector<HostLevel> levels;
    std::vector<double> coarse_inv;  // dense n_c x n_c, row-major
    double shift = 0.0;
};

struct Params {
    double theta = kTheta;
    int max_coarse = kMaxCoarse;
    int max_levels = kMaxLevels;
};

// Builds the hierarchy of the CRS matrix (row_ptr[0] = 0, columns in [0, n)).
// nullspace_const: the operator's null space is the constant vector.
// Returns false (with a message in err) when the coarsest operator cannot be
// inverted.
bool setup(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val, bool nullspace_const,
           const Params &prm, HostHierarchy *out, const char **err);

} // namespace amg
} // namespace mrhs
