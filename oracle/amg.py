"""Oracle for the classical algebraic multigrid preconditioner (CPU, binary64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the GPU library never does.

The paper's pressure solver is BiCGStab preconditioned by classical algebraic
multigrid (Section 4.1); it names the method, not its parameters.  The reading
implemented here (the classical Ruge-Stueben construction; K. Stueben, "A
review of algebraic multigrid", J. Comput. Appl. Math. 128, 2001):

* Canonical form: entries of a row sorted by column, repeated columns summed.
* Strength: j != i is a strong connection of row i when
  -a_ij >= theta * max_{k != i}(-a_ik) and that maximum is positive
  (theta = 0.25); S_i is the set of strong connections of i, S^T_j the set of
  rows that have j among theirs.
* C/F splitting (the first pass of Ruge and Stueben): rows with no strong
  connection either way are F; then, while undecided rows remain, the
  undecided row i with the largest lambda_i = |S^T_i restricted to undecided
  and F-counted rows| (smallest index on ties) becomes C, every undecided row
  of S^T_i becomes F and raises lambda of the undecided rows of its own S by
  one, and the undecided rows of S_i lower theirs by one.
* Direct interpolation: a C row injects (weight 1 to its coarse index, C rows
  numbered in increasing fine index); an F row i interpolates from
  P_i = S_i intersected with C with w_ik = -(sum_{N_i} a^-) / (sum_{P_i} a^-)
  * a_ik / (a_ii + sum_{N_i} a^+), N_i the off-diagonal entries of row i,
  a^-/a^+ the negative/positive ones (strong connections are negative, so
  P_i has no positive entries and those of N_i are lumped to the diagonal).
  A zero row sum gives weights summing to one: P reproduces constants.
* Galerkin coarse operator A_c = P^T (A P), R = P^T stored explicitly, each
  product accumulated in a fixed order (rows in order, the left factor's
  entries in storage order, the right factor's row in storage order; every
  structurally produced entry is kept, zero or not).
* Levels until the coarse size is at most max_coarse, coarsening stalls
  (n_c > 0.9 n or n_c = 0) or max_levels is reached.  The coarsest level is
  solved with the dense inverse of A_c + s 1 1^T, s = mean(diag A_c) / n_c
  for an operator whose null space is the constant vector (P 1 = 1 keeps it
  at every level), s = 0 otherwise.
* Smoother: l1-Jacobi, x <- x + D_l1^-1 (b - A x), D_l1 = diag(sum_j |a_ij|)
  (Baker, Falgout, Kolev and Yang, SIAM J. Sci. Comput. 33, 2011), applied as
  a product with the stored reciprocals.
* V-cycle for a block of m columns: x = 0, nu pre-smoothing sweeps,
  r = b - A x, coarse correction x += P V(R r), nu post-smoothing sweeps.
  Same number of sweeps before and after: for a symmetric A the cycle is a
  symmetric operator.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

import numpy as np

THETA = 0.25
MAX_COARSE = 256
MAX_LEVELS = 25
SWEEPS = 1


@dataclass
class Csr:
    n_rows: int
    n_cols: int
    rp: np.ndarray   # int64 [n_rows + 1]
    ci: np.ndarray   # int64 [nnz]
    va: np.ndarray   # float64 [nnz]

    @property
    def nnz(self):
        return int(self.rp[-1])

    def to_dense(self):
        D = np.zeros((self.n_rows, self.n_cols))
        for i in range(self.n_rows):
            for k in range(self.rp[i], self.rp[i + 1]):
                D[i, self.ci[k]] += self.va[k]
        return D

    def matvec(self, X):
        """Y = self X, each row summed in storage order (the plain product of
        the oracle), for an (n_cols, m) block."""
        from . import gspmv_rect
        X = np.asarray(X, dtype=np.float64)
        assert X.shape[0] == self.n_cols
        return gspmv_rect(self.n_rows, self.rp, self.ci, self.va, X)


def canonical(n, row_ptr, col, val):
    """Rows sorted by column, repeated columns summed (in storage order)."""
    rp = [0]
    ci, va = [], []
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    for i in range(n):
        acc = {}
        for k in range(row_ptr[i], row_ptr[i + 1]):
            c = int(col[k])
            acc[c] = acc[c] + float(val[k]) if c in acc else float(val[k])
        for c in sorted(acc):
            ci.append(c)
            va.append(acc[c])
        rp.append(len(ci))
    return Csr(n, n, np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int64), np.array(va, dtype=np.float64))


def strength(A: Csr, theta=THETA):
    """S_i as lists: the strong connections of every row."""
    S = []
    for i in range(A.n_rows):
        mx = 0.0
        have = False
        for k in range(A.rp[i], A.rp[i + 1]):
            j = A.ci[k]
            if j != i:
                v = -A.va[k]
                if not have or v > mx:
                    mx = v
                    have = True
        row = []
        if have and mx > 0.0:
            thr = theta * mx
            for k in range(A.rp[i], A.rp[i + 1]):
                j = A.ci[k]
                if j != i and -A.va[k] >= thr:
                    row.append(int(j))
        S.append(row)
    return S


def transpose_sets(S, n):
    ST = [[] for _ in range(n)]
    for i, row in enumerate(S):
        for j in row:
            ST[j].append(i)
    return ST


def rs_split(S, n):
    """C/F splitting, first pass of Ruge and Stueben.  Returns cf (1 = C)."""
    ST = transpose_sets(S, n)
    UND, CPT, FPT = 0, 1, 2
    state = [UND] * n
    lam = [len(ST[i]) for i in range(n)]
    for i in range(n):
        if not S[i] and not ST[i]:
            state[i] = FPT
    heap = [(-lam[i], i) for i in range(n) if state[i] == UND]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != UND or -negl != lam[i]:
            continue  # stale entry
        state[i] = CPT
        for j in ST[i]:
            if state[j] == UND:
                state[j] = FPT
                for k in S[j]:
                    if state[k] == UND:
                        lam[k] += 1
                        heapq.heappush(heap, (-lam[k], k))
        for k in S[i]:
            if state[k] == UND:
                lam[k] -= 1
                heapq.heappush(heap, (-lam[k], k))
    return np.array([1 if s == CPT else 0 for s in state], dtype=np.int8)


def direct_interpolation(A: Csr, S, cf):
    """Prolongation P (n x n_c) by direct interpolation."""
    n = A.n_rows
    cidx = np.cumsum(cf) - 1
    n_c = int(cf.sum())
    rp = [0]
    ci, va = [], []
    for i in range(n):
        if cf[i]:
            ci.append(int(cidx[i]))
            va.append(1.0)
            rp.append(len(ci))
            continue
        strong_c = set(j for j in S[i] if cf[j])
        diag = 0.0
        neg_n = pos_n = neg_p = 0.0
        for k in range(A.rp[i], A.rp[i + 1]):
            j = A.ci[k]
            a = A.va[k]
            if j == i:
                diag += a
            elif a < 0.0:
                neg_n += a
                if j in strong_c:
                    neg_p += a
            elif a > 0.0:
                pos_n += a
        if strong_c and neg_p != 0.0:
            alpha = neg_n / neg_p
            d = diag + pos_n
            for k in range(A.rp[i], A.rp[i + 1]):
                j = A.ci[k]
                if j in strong_c:
                    ci.append(int(cidx[j]))
                    va.append(-(alpha * A.va[k]) / d)
        rp.append(len(ci))
    return Csr(n, n_c, np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int64), np.array(va, dtype=np.float64))


def transpose(P: Csr):
    """R = P^T with rows listing P's rows in increasing order."""
    rows = [[] for _ in range(P.n_cols)]
    for i in range(P.n_rows):
        for k in range(P.rp[i], P.rp[i + 1]):
            rows[P.ci[k]].append((i, P.va[k]))
    rp = [0]
    ci, va = [], []
    for r in rows:
        for (i, v) in r:
            ci.append(i)
            va.append(v)
        rp.append(len(ci))
    return Csr(P.n_cols, P.n_rows, np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int64),
               np.array(va, dtype=np.float64))


def spgemm(L: Csr, Rm: Csr):
    """L Rm, row i accumulated over L's row i in storage order, each term
    spread over Rm's row in storage order; columns of the result sorted."""
    rp = [0]
    ci, va = [], []
    for i in range(L.n_rows):
        acc = {}
        for k in range(L.rp[i], L.rp[i + 1]):
            a = L.va[k]
            l = L.ci[k]
            for q in range(Rm.rp[l], Rm.rp[l + 1]):
                j = int(Rm.ci[q])
                t = a * Rm.va[q]
                acc[j] = acc[j] + t if j in acc else t
        for j in sorted(acc):
            ci.append(j)
            va.append(acc[j])
        rp.append(len(ci))
    return Csr(L.n_rows, Rm.n_cols, np.array(rp, dtype=np.int64), np.array(ci, dtype=np.int64),
               np.array(va, dtype=np.float64))


def l1_inverse(A: Csr):
    out = np.empty(A.n_rows)
    for i in range(A.n_rows):
        s = 0.0
        for k in range(A.rp[i], A.rp[i + 1]):
            s += abs(A.va[k])
        out[i] = 1.0 / s if s > 0.0 else 0.0
    return out


@dataclass
class Level:
    A: Csr
    dl1_inv: np.ndarray
    cf: np.ndarray = None
    P: Csr = None
    R: Csr = None


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    coarse_inv: np.ndarray = None   # dense inverse of the coarsest operator (+ s 1 1^T)
    shift: float = 0.0
    sweeps: int = SWEEPS


def setup(n, row_ptr, col, val, nullspace_const=False, theta=THETA, max_coarse=MAX_COARSE,
          max_levels=MAX_LEVELS, sweeps=SWEEPS):
    """The AMG hierarchy of a CRS matrix (see the module docstring)."""
    H = Hierarchy(sweeps=sweeps)
    A = canonical(n, row_ptr, col, val)
    while True:
        lev = Level(A=A, dl1_inv=l1_inverse(A))
        H.levels.append(lev)
        if A.n_rows <= max_coarse or len(H.levels) >= max_levels:
            break
        S = strength(A, theta)
        cf = rs_split(S, A.n_rows)
        n_c = int(cf.sum())
        if n_c == 0 or n_c > 0.9 * A.n_rows:
            break
        P = direct_interpolation(A, S, cf)
        R = transpose(P)
        lev.cf, lev.P, lev.R = cf, P, R
        A = spgemm(R, spgemm(A, P))
    Ac = H.levels[-1].A.to_dense()
    nc = Ac.shape[0]
    H.shift = float(np.mean(np.diag(Ac))) / nc if (nullspace_const and nc > 0) else 0.0
    H.coarse_inv = np.linalg.inv(Ac + H.shift * np.ones((nc, nc))) if nc else np.zeros((0, 0))
    return H


def smooth(lev: Level, X, B):
    return X + lev.dl1_inv[:, None] * (B - lev.A.matvec(X))


def vcycle(H: Hierarchy, B, level=0):
    """x = M^-1 b for an (n, m) block b (one V-cycle from x = 0)."""
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    if squeeze:
        B = B[:, None]
    if level == len(H.levels) - 1:
        X = H.coarse_inv @ B
    else:
        lev = H.levels[level]
        X = np.zeros_like(B)
        for _ in range(H.sweeps):
            X = smooth(lev, X, B)
        Rr = lev.R.matvec(B - lev.A.matvec(X))
        X = X + lev.P.matvec(vcycle(H, Rr, level + 1))
        for _ in range(H.sweeps):
            X = smooth(lev, X, B)
    return X[:, 0] if squeeze else X


def complexity(H: Hierarchy):
    """Operator complexity (sum of nnz over levels / nnz of the finest) and
    grid complexity (sum of rows / rows of the finest)."""
    nz = sum(l.A.nnz for l in H.levels)
    nr = sum(l.A.n_rows for l in H.levels)
    return nz / H.levels[0].A.nnz, nr / H.levels[0].A.n_rows


def bicgstab(A_rows, H: Hierarchy, b, tol=1e-10, maxit=1000, nullspace_const=False, shadow=None, hist=None):
    """One column of the SLAE by BiCGStab with the V-cycle as right
    preconditioner, in the control flow of the Jacobi oracle: stop when the
    recurrence residual meets tol and the recomputed true residual confirms
    it, else restart from the true residual; x0 = 0; the shadow residual is
    the given vector (kept over restarts) or the initial residual.  A_rows is
    a Csr of the operator (canonical form).  Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    nb = float(np.linalg.norm(b))
    x = np.zeros(n)
    info = {"iters": 0, "restarts": 0, "status": 0}
    if nb == 0.0:
        return x, dict(info, relres=0.0)

    def true_res(x):
        return b - A_rows.matvec(x[:, None])[:, 0]

    r = true_res(x)
    rh = np.array(shadow, dtype=np.float64) if shadow is not None else r.copy()
    rho = float(rh @ r)
    rho_old = alpha = omega = 1.0
    fresh = True
    from_rec = False
    it = 0
    p = np.zeros(n)
    v = np.zeros(n)
    status = -4
    while True:
        rn = float(np.linalg.norm(r)) / nb
        if hist is not None:
            hist.append(rn)
        if rn <= tol:
            if not from_rec:
                status = 0
                break
            r = true_res(x)
            if float(np.linalg.norm(r)) / nb <= tol:
                status = 0
                break
            info["restarts"] += 1
            if shadow is None:
                rh = r.copy()
            rho = float(rh @ r)
            rho_old = alpha = omega = 1.0
            fresh, from_rec = True, False
            continue
        if it >= maxit:
            break
        it += 1
        if fresh:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        ph = vcycle(H, p)
        v = A_rows.matvec(ph[:, None])[:, 0]
        sigma = float(rh @ v)
        if sigma == 0.0 or not np.isfinite(sigma):
            status = -5
            break
        alpha = rho / sigma
        s = r - alpha * v
        if float(np.linalg.norm(s)) / nb <= tol:
            x = x + alpha * ph
            r = s
            from_rec = True
            continue
        sh = vcycle(H, s)
        t = A_rows.matvec(sh[:, None])[:, 0]
        omega = float(t @ s) / float(t @ t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho
        rho = float(rh @ r)
        fresh, from_rec = False, True
    if nullspace_const:
        x = x - x.mean()
    info["iters"] = it
    info["status"] = status
    info["relres"] = float(np.linalg.norm(true_res(x))) / nb
    return x, info
