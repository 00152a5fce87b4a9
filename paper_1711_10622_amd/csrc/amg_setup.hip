// Host construction of the classical AMG hierarchy (see amg.h for the
// method).  Every floating-point sum here runs in a fixed order (rows in
// order, a row's entries in storage order) with no fused multiply-add, so
// the hierarchy is a deterministic function of the matrix.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <thread>
#include <utility>
#include <vector>

#include "amg.h"

#pragma clang fp contract(off)

namespace mrhs {
namespace amg {
namespace {

// Rows are independent in every per-row step below, so they run on host
// threads over contiguous row ranges, each range's rows appended in order to
// its own buffers and the buffers joined in range order: the result is the
// sequential one, bit for bit.
// (MRHS_AMG_THREADS fixes the count, for testing the split on small matrices)
int host_threads(int64_t rows)
{
    if (const char *e = std::getenv("MRHS_AMG_THREADS"))
        return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(std::atoi(e), std::max<int64_t>(rows, 1))));
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t by_size = rows / 32768 + 1;
    return static_cast<int>(std::min<int64_t>({static_cast<int64_t>(hw), 16, by_size}));
}

// fn(lo, hi, t) for T contiguous ranges of [0, n)
template <class F>
void parallel_ranges(int32_t n, int T, F &&fn)
{
    if (T <= 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(static_cast<size_t>(T));
    for (int t = 0; t < T; ++t) {
        const int32_t lo = static_cast<int32_t>(static_cast<int64_t>(n) * t / T);
        const int32_t hi = static_cast<int32_t>(static_cast<int64_t>(n) * (t + 1) / T);
        th.emplace_back([&fn, lo, hi, t] { fn(lo, hi, t); });
    }
    for (auto &x : th)
        x.join();
}

// A CRS matrix of nr rows built by row(i, ci, va, scratch), which appends
// row i's entries; MakeScratch() gives each thread its own scratch;
// reserve(lo, hi) estimates the entries of rows lo..hi-1.
template <class MakeScratch, class Row, class Reserve>
HostCsr build_rows(int32_t nr, int32_t nc, MakeScratch make_scratch, Row row, Reserve reserve)
{
    const int T = host_threads(nr);
    std::vector<std::vector<int32_t>> cis(T), lens(T);
    std::vector<std::vector<double>> vas(T);
    parallel_ranges(nr, T, [&](int32_t lo, int32_t hi, int t) {
        auto scratch = make_scratch();
        std::vector<int32_t> &ci = cis[t], &len = lens[t];
        std::vector<double> &va = vas[t];
        len.reserve(static_cast<size_t>(hi - lo));
        const size_t est = reserve(lo, hi);
        ci.reserve(est);
        va.reserve(est);
        for (int32_t i = lo; i < hi; ++i) {
            const size_t before = ci.size();
            row(i, ci, va, scratch);
            len.push_back(static_cast<int32_t>(ci.size() - before));
        }
    });
    HostCsr C;
    C.nr = nr;
    C.nc = nc;
    C.rp.assign(static_cast<size_t>(nr) + 1, 0);
    size_t total = 0;
    for (int t = 0; t < T; ++t)
        total += cis[t].size();
    C.ci.reserve(total);
    C.va.reserve(total);
    int32_t i = 0;
    for (int t = 0; t < T; ++t) {
        for (int32_t l : lens[t]) {
            C.rp[i + 1] = C.rp[i] + l;
            ++i;
        }
        C.ci.insert(C.ci.end(), cis[t].begin(), cis[t].end());
        C.va.insert(C.va.end(), vas[t].begin(), vas[t].end());
        std::vector<int32_t>().swap(cis[t]);
        std::vector<double>().swap(vas[t]);
    }
    return C;
}

struct NoScratch {};

// Rows sorted by column, repeated columns summed in storage order.
HostCsr canonical(int32_t n, const int32_t *rp, const int32_t *ci, const double *va)
{
    using Row = std::vector<std::pair<int32_t, int32_t>>;  // (column, storage index)
    return build_rows(n, n, [] { return Row(); },
                      [&](int32_t i, std::vector<int32_t> &oci, std::vector<double> &ova, Row &row) {
                          row.clear();
                          for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                              row.emplace_back(ci[k], k);
                          std::sort(row.begin(), row.end());
                          for (size_t q = 0; q < row.size(); ++q) {
                              if (q > 0 && row[q].first == row[q - 1].first) {
                                  ova.back() = ova.back() + va[row[q].second];
                              } else {
                                  oci.push_back(row[q].first);
                                  ova.push_back(va[row[q].second]);
                              }
                          }
                      },
                      [&](int32_t lo, int32_t hi) { return static_cast<size_t>(rp[hi] - rp[lo]); });
}

// Strong connections of every row, as a CRS pattern (columns increasing).
void strength(const HostCsr &A, double theta, std::vector<int32_t> &srp, std::vector<int32_t> &sci)
{
    HostCsr S = build_rows(A.nr, A.nc, [] { return NoScratch{}; },
                           [&](int32_t i, std::vector<int32_t> &oci, std::vector<double> &, NoScratch &) {
                               double mx = 0.0;
                               bool have = false;
                               for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                                   if (A.ci[k] == i)
                                       continue;
                                   const double v = -A.va[k];
                                   if (!have || v > mx) {
                                       mx = v;
                                       have = true;
                                   }
                               }
                               if (have && mx > 0.0) {
                                   const double thr = theta * mx;
                                   for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                                       if (A.ci[k] != i && -A.va[k] >= thr)
                                           oci.push_back(A.ci[k]);
                               }
                           },
                           [&](int32_t lo, int32_t hi) { return static_cast<size_t>(A.rp[hi] - A.rp[lo]); });
    srp.swap(S.rp);
    sci.swap(S.ci);
}

// Max-heap over rows keyed by (measure, -row) with positions, so a row's
// measure can move up or down in place.
class MeasureHeap {
  public:
    explicit MeasureHeap(const std::vector<int32_t> &lam) : lam_(lam), pos_(lam.size(), -1) {}
    void push(int32_t i)
    {
        pos_[i] = static_cast<int32_t>(h_.size());
        h_.push_back(i);
        up(pos_[i]);
    }
    bool empty() const { return h_.empty(); }
    int32_t pop()
    {
        const int32_t top = h_[0];
        remove_at(0);
        return top;
    }
    void remove(int32_t i)
    {
        if (pos_[i] >= 0)
            remove_at(pos_[i]);
    }
    void changed(int32_t i)  // lam[i] moved
    {
        if (pos_[i] < 0)
            return;
        up(pos_[i]);
        down(pos_[i]);
    }

  private:
    bool before(int32_t a, int32_t b) const { return lam_[a] > lam_[b] || (lam_[a] == lam_[b] && a < b); }
    void place(int32_t p, int32_t i)
    {
        h_[p] = i;
        pos_[i] = p;
    }
    void up(int32_t p)
    {
        const int32_t i = h_[p];
        while (p > 0) {
            const int32_t q = (p - 1) / 2;
            if (!before(i, h_[q]))
                break;
            place(p, h_[q]);
            p = q;
        }
        place(p, i);
    }
    void down(int32_t p)
    {
        const int32_t i = h_[p];
        const int32_t n = static_cast<int32_t>(h_.size());
        for (;;) {
            int32_t c = 2 * p + 1;
            if (c >= n)
                break;
            if (c + 1 < n && before(h_[c + 1], h_[c]))
                ++c;
            if (!before(h_[c], i))
                break;
            place(p, h_[c]);
            p = c;
        }
        place(p, i);
    }
    void remove_at(int32_t p)
    {
        const int32_t i = h_[p];
        pos_[i] = -1;
        const int32_t last = h_.back();
        h_.pop_back();
        if (p < static_cast<int32_t>(h_.size())) {
            place(p, last);
            up(p);
            down(pos_[last]);
        }
    }
    const std::vector<int32_t> &lam_;
    std::vector<int32_t> pos_, h_;
};

// First pass of Ruge and Stueben: cf[i] = 1 for C rows.
std::vector<int8_t> split(int32_t n, const std::vector<int32_t> &srp, const std::vector<int32_t> &sci)
{
    // transpose of the strength pattern: the rows strongly connected to j
    std::vector<int32_t> trp(static_cast<size_t>(n) + 1, 0), tci(sci.size());
    for (int32_t j : sci)
        ++trp[j + 1];
    std::partial_sum(trp.begin(), trp.end(), trp.begin());
    {
        std::vector<int32_t> fill(trp.begin(), trp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = srp[i]; k < srp[i + 1]; ++k)
                tci[fill[sci[k]]++] = i;
    }
    enum : int8_t { UND = 0, CPT = 1, FPT = 2 };
    std::vector<int8_t> st(n, UND);
    std::vector<int32_t> lam(n);
    for (int32_t i = 0; i < n; ++i) {
        lam[i] = trp[i + 1] - trp[i];
        if (srp[i + 1] == srp[i] && lam[i] == 0)
            st[i] = FPT;
    }
    MeasureHeap heap(lam);
    for (int32_t i = 0; i < n; ++i)
        if (st[i] == UND)
            heap.push(i);
    while (!heap.empty()) {
        const int32_t i = heap.pop();
        st[i] = CPT;
        for (int32_t q = trp[i]; q < trp[i + 1]; ++q) {
            const int32_t j = tci[q];
            if (st[j] != UND)
                continue;
            st[j] = FPT;
            heap.remove(j);
            for (int32_t k = srp[j]; k < srp[j + 1]; ++k) {
                const int32_t c = sci[k];
                if (st[c] == UND) {
                    ++lam[c];
                    heap.changed(c);
                }
            }
        }
        for (int32_t k = srp[i]; k < srp[i + 1]; ++k) {
            const int32_t c = sci[k];
            if (st[c] == UND) {
                --lam[c];
                heap.changed(c);
            }
        }
    }
    std::vector<int8_t> cf(n);
    for (int32_t i = 0; i < n; ++i)
        cf[i] = st[i] == CPT ? 1 : 0;
    return cf;
}

HostCsr interpolation(const HostCsr &A, const std::vector<int32_t> &srp, const std::vector<int32_t> &sci,
                      const std::vector<int8_t> &cf)
{
    const int32_t n = A.nr;
    std::vector<int32_t> cidx(n, -1);
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (cf[i])
            cidx[i] = nc++;
    // mark[j] == i: j is a strong C neighbour of i
    return build_rows(n, nc, [n] { return std::vector<int32_t>(n, -1); },
                      [&](int32_t i, std::vector<int32_t> &oci, std::vector<double> &ova, std::vector<int32_t> &mark) {
                          if (cf[i]) {
                              oci.push_back(cidx[i]);
                              ova.push_back(1.0);
                              return;
                          }
                          bool any = false;
                          for (int32_t k = srp[i]; k < srp[i + 1]; ++k)
                              if (cf[sci[k]]) {
                                  mark[sci[k]] = i;
                                  any = true;
                              }
                          double diag = 0.0, neg_n = 0.0, pos_n = 0.0, neg_p = 0.0;
                          for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                              const int32_t j = A.ci[k];
                              const double a = A.va[k];
                              if (j == i) {
                                  diag += a;
                              } else if (a < 0.0) {
                                  neg_n += a;
                                  if (mark[j] == i)
                                      neg_p += a;
                              } else if (a > 0.0) {
                                  pos_n += a;
                              }
                          }
                          if (any && neg_p != 0.0) {
                              const double alpha = neg_n / neg_p;
                              const double d = diag + pos_n;
                              for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                                  if (mark[A.ci[k]] == i) {
                                      oci.push_back(cidx[A.ci[k]]);
                                      ova.push_back(-(alpha * A.va[k]) / d);
                                  }
                          }
                      },
                      [&](int32_t lo, int32_t hi) { return static_cast<size_t>(srp[hi] - srp[lo] + (hi - lo)); });
}

HostCsr transpose(const HostCsr &P)
{
    HostCsr R;
    R.nr = P.nc;
    R.nc = P.nr;
    R.rp.assign(static_cast<size_t>(P.nc) + 1, 0);
    for (int32_t c : P.ci)
        ++R.rp[c + 1];
    std::partial_sum(R.rp.begin(), R.rp.end(), R.rp.begin());
    R.ci.resize(P.ci.size());
    R.va.resize(P.va.size());
    std::vector<int32_t> fill(R.rp.begin(), R.rp.end() - 1);
    for (int32_t i = 0; i < P.nr; ++i)
        for (int32_t k = P.rp[i]; k < P.rp[i + 1]; ++k) {
            const int32_t q = fill[P.ci[k]]++;
            R.ci[q] = i;
            R.va[q] = P.va[k];
        }
    return R;
}

// L R: row i sums, over L's row i in storage order, each entry times R's
// row in storage order; result columns increasing.  A row's distinct columns
// are collected in a short list searched linearly (rows of these operators
// have tens of entries, and the list stays in cache where column-indexed
// arrays of the full width would not); a row with more than kShort distinct
// columns moves to the full-width arrays.  Either way each column's terms
// are added in the order they are generated.
struct MulScratch {
    std::vector<double> acc;
    std::vector<int32_t> seen, cols;
    std::vector<std::pair<int32_t, double>> small;
};

HostCsr multiply(const HostCsr &L, const HostCsr &Rm)
{
    constexpr size_t kShort = 64;
    const int32_t nc = Rm.nc;
    return build_rows(
        L.nr, nc, [] { return MulScratch{}; },
        [&](int32_t i, std::vector<int32_t> &oci, std::vector<double> &ova, MulScratch &w) {
            w.small.clear();
            bool wide = false;
            w.cols.clear();
            for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) {
                const double a = L.va[k];
                const int32_t l = L.ci[k];
                for (int32_t q = Rm.rp[l]; q < Rm.rp[l + 1]; ++q) {
                    const int32_t j = Rm.ci[q];
                    const double t = a * Rm.va[q];
                    if (!wide) {
                        size_t e = 0;
                        while (e < w.small.size() && w.small[e].first != j)
                            ++e;
                        if (e < w.small.size()) {
                            w.small[e].second = w.small[e].second + t;
                            continue;
                        }
                        if (w.small.size() < kShort) {
                            w.small.emplace_back(j, t);
                            continue;
                        }
                        // too many columns: continue in the full-width arrays
                        if (w.acc.empty()) {
                            w.acc.assign(nc, 0.0);
                            w.seen.assign(nc, -1);
                        }
                        for (const auto &e2 : w.small) {
                            w.seen[e2.first] = i;
                            w.acc[e2.first] = e2.second;
                            w.cols.push_back(e2.first);
                        }
                        wide = true;
                    }
                    if (w.seen[j] != i) {
                        w.seen[j] = i;
                        w.acc[j] = t;
                        w.cols.push_back(j);
                    } else {
                        w.acc[j] = w.acc[j] + t;
                    }
                }
            }
            if (!wide) {
                std::sort(w.small.begin(), w.small.end(),
                          [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                              return x.first < y.first;
                          });
                for (const auto &e : w.small) {
                    oci.push_back(e.first);
                    ova.push_back(e.second);
                }
                return;
            }
            std::sort(w.cols.begin(), w.cols.end());
            for (int32_t j : w.cols) {
                oci.push_back(j);
                ova.push_back(w.acc[j]);
            }
        },
        [&](int32_t lo, int32_t hi) {
            // about the row count times L's mean row length times Rm's
            const double ln = static_cast<double>(L.rp[hi] - L.rp[lo]);
            const double rn = Rm.nr ? static_cast<double>(Rm.rp[Rm.nr]) / Rm.nr : 0.0;
            return static_cast<size_t>(ln * std::min(rn, 4.0));
        });
}

std::vector<double> l1_inverse(const HostCsr &A)
{
    std::vector<double> out(A.nr);
    parallel_ranges(A.nr, host_threads(A.nr), [&](int32_t lo, int32_t hi, int) {
        for (int32_t i = lo; i < hi; ++i) {
            double s = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                s += std::fabs(A.va[k]);
            out[i] = s > 0.0 ? 1.0 / s : 0.0;
        }
    });
    return out;
}

// Gauss-Jordan inverse with partial pivoting of a dense row-major matrix.
bool invert(std::vector<double> &M, int32_t n)
{
    std::vector<double> inv(static_cast<size_t>(n) * n, 0.0);
    for (int32_t i = 0; i < n; ++i)
        inv[static_cast<size_t>(i) * n + i] = 1.0;
    for (int32_t c = 0; c < n; ++c) {
        int32_t p = c;
        for (int32_t r = c + 1; r < n; ++r)
            if (std::fabs(M[static_cast<size_t>(r) * n + c]) > std::fabs(M[static_cast<size_t>(p) * n + c]))
                p = r;
        const double piv = M[static_cast<size_t>(p) * n + c];
        if (piv == 0.0 || !std::isfinite(piv))
            return false;
        if (p != c)
            for (int32_t k = 0; k < n; ++k) {
                std::swap(M[static_cast<size_t>(p) * n + k], M[static_cast<size_t>(c) * n + k]);
                std::swap(inv[static_cast<size_t>(p) * n + k], inv[static_cast<size_t>(c) * n + k]);
            }
        const double s = 1.0 / piv;
        for (int32_t k = 0; k < n; ++k) {
            M[static_cast<size_t>(c) * n + k] *= s;
            inv[static_cast<size_t>(c) * n + k] *= s;
        }
        for (int32_t r = 0; r < n; ++r) {
            if (r == c)
                continue;
            const double f = M[static_cast<size_t>(r) * n + c];
            if (f == 0.0)
                continue;
            for (int32_t k = 0; k < n; ++k) {
                M[static_cast<size_t>(r) * n + k] -= f * M[static_cast<size_t>(c) * n + k];
                inv[static_cast<size_t>(r) * n + k] -= f * inv[static_cast<size_t>(c) * n + k];
            }
        }
    }
    M.swap(inv);
    return true;
}

} // namespace

bool setup(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val, bool nullspace_const,
           const Params &prm, HostHierarchy *out, const char **err)
{
    HostHierarchy &H = *out;
    H.levels.clear();
    HostCsr A = canonical(n, row_ptr, col, val);
    std::vector<int32_t> srp, sci;
    for (;;) {
        H.levels.emplace_back();
        HostLevel &lev = H.levels.back();
        lev.dl1_inv = l1_inverse(A);
        lev.A = std::move(A);
        if (lev.A.nr <= prm.max_coarse || static_cast<int>(H.levels.size()) >= prm.max_levels)
            break;
        strength(lev.A, prm.theta, srp, sci);
        std::vector<int8_t> cf = split(lev.A.nr, srp, sci);
        int64_t nc = 0;
        for (int8_t c : cf)
            nc += c;
        if (nc == 0 || static_cast<double>(nc) > 0.9 * lev.A.nr)
            break;
        lev.P = interpolation(lev.A, srp, sci, cf);
        lev.R = transpose(lev.P);
        lev.cf = std::move(cf);
        A = multiply(lev.R, multiply(lev.A, lev.P));
    }
    const HostCsr &Ac = H.levels.back().A;
    const int32_t nc = Ac.nr;
    std::vector<double> M(static_cast<size_t>(nc) * nc, 0.0);
    double dsum = 0.0;
    for (int32_t i = 0; i < nc; ++i)
        for (int32_t k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k) {
            M[static_cast<size_t>(i) * nc + Ac.ci[k]] += Ac.va[k];
            if (Ac.ci[k] == i)
                dsum += Ac.va[k];
        }
    H.shift = (nullspace_const && nc > 0) ? (dsum / nc) / nc : 0.0;
    if (H.shift != 0.0)
        for (double &v : M)
            v += H.shift;
    if (nc > 0 && !invert(M, nc)) {
        *err = "the coarsest AMG operator is singular (a null space other than the constants?)";
        return false;
    }
    H.coarse_inv.swap(M);
    return true;
}

} // namespace amg
} // namespace mrhs
