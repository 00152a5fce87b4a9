// C ABI of libmrhs: matrix handles, the generalized SpMV and the block solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "dict.h"
#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {

namespace {
thread_local std::string g_error;
}

mrhs_status set_error(mrhs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

void clear_error() { g_error.clear(); }

namespace {

std::mutex g_grid_mu;
std::unordered_map<const void *, int> g_blocks_per_cu;
int g_num_cu = 0;

int num_cu()
{
    if (g_num_cu == 0) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            g_num_cu = cu;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

} // namespace

int max_grid()
{
    std::lock_guard<std::mutex> lk(g_grid_mu);
    const int g = num_cu() * (2048 / kBlock);
    return (g + kGroups - 1) / kGroups * kGroups;
}

int grid_for(const void *kernel, int64_t n, int tile_rows, int max_per_cu)
{
    int per_cu = 1, cus = 0;
    {
        std::lock_guard<std::mutex> lk(g_grid_mu);
        cus = num_cu();
        auto it = g_blocks_per_cu.find(kernel);
        if (it == g_blocks_per_cu.end()) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1)
                nb = 1;
            nb = std::min(nb, 2048 / kBlock);
            it = g_blocks_per_cu.emplace(kernel, nb).first;
        }
        per_cu = it->second;
    }
    if (max_per_cu > 0)
        per_cu = std::min(per_cu, max_per_cu);
    const int64_t ntiles = (n + tile_rows - 1) / tile_rows;
    int64_t g = std::min<int64_t>(ntiles, static_cast<int64_t>(per_cu) * cus);
    g = std::max<int64_t>(g, 1);
    g = (g + kGroups - 1) / kGroups * kGroups;
    return static_cast<int>(g);
}

int march_mode() { return env_int("MRHS_MARCH", 0, 0, 1); }

int32_t march_runs(int32_t n, int32_t reach, int tile_rows, int grid)
{
    if (reach <= 0 || reach % tile_rows != 0)
        return 0;
    const int32_t P = reach / tile_rows;
    const int32_t planes = static_cast<int32_t>((static_cast<int64_t>(n) + reach - 1) / reach);
    if (P < 2 * kGroups || planes < 8)
        return 0;
    const int64_t cg = (P + kGroups - 1) / kGroups;  // columns of the widest group
    const int64_t gx = std::max(grid / kGroups, 1);
    int32_t best = 1;
    double best_score = -1.0;
    for (int32_t runs = 1; runs <= planes / 8; ++runs) {
        const int64_t units = cg * runs;
        const int64_t rounds = (units + gx - 1) / gx;
        const double fill = static_cast<double>(units) / static_cast<double>(rounds * gx);
        const int32_t zlen = (planes + runs - 1) / runs;
        const double score = fill * zlen / (zlen + 1.0);
        if (score > best_score + 1e-9) {
            best_score = score;
            best = runs;
        }
    }
    return best;
}

// ---- launch tracing ---------------------------------------------------------
int g_trace_every = 0;

namespace {

struct TraceRec {
    hipEvent_t a = nullptr, b = nullptr;
    std::string key;
    bool open = false;
};

struct TraceStat {
    int64_t seen = 0;      // launches of the class since tracing started
    int64_t launches = 0;  // launches timed (every g_trace_every-th)
    double total_ms = 0.0, min_ms = 1e300, max_ms = 0.0;
};

std::mutex g_trace_mu;
std::unordered_map<int, TraceRec> g_trace_recs;  // by slot id
int g_trace_next = 0;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_trace_pool;
std::vector<std::pair<std::string, TraceStat>> g_trace_stats;

TraceStat &trace_stat(const std::string &key)
{
    for (auto &kv : g_trace_stats)
        if (kv.first == key)
            return kv.second;
    g_trace_stats.emplace_back(key, TraceStat{});
    return g_trace_stats.back().second;
}

// Folds every completed record into the statistics (events are synchronised).
void trace_drain_locked()
{
    for (auto it = g_trace_recs.begin(); it != g_trace_recs.end();) {
        TraceRec &r = it->second;
        if (r.open) {
            ++it;
            continue;
        }
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            TraceStat &st = trace_stat(r.key);
            st.launches += 1;
            st.total_ms += ms;
            st.min_ms = std::min<double>(st.min_ms, ms);
            st.max_ms = std::max<double>(st.max_ms, ms);
        }
        g_trace_pool.emplace_back(r.a, r.b);
        it = g_trace_recs.erase(it);
    }
}

} // namespace

int trace_begin(hipStream_t s, const char *name, int elem_bytes, int m, int grid, bool windows)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    char key[128];
    std::snprintf(key, sizeof(key), "%s/%s/m%d/g%d%s", name, elem_bytes == 8 ? "f64" : "f32", m, grid,
                  windows ? "w" : "");
    TraceStat &st = trace_stat(key);
    const int64_t seen = st.seen++;
    if (g_trace_every <= 0 || seen % g_trace_every != 0)
        return -1;
    TraceRec r;
    if (!g_trace_pool.empty()) {
        r.a = g_trace_pool.back().first;
        r.b = g_trace_pool.back().second;
        g_trace_pool.pop_back();
    } else if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
        return -1;
    }
    r.open = true;
    r.key = key;
    (void)hipEventRecord(r.a, s);
    const int slot = g_trace_next;
    g_trace_next = (g_trace_next + 1) & 0x3fffffff;
    g_trace_recs[slot] = r;
    return slot;
}

void trace_end(int slot, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    auto it = g_trace_recs.find(slot);
    if (it == g_trace_recs.end())
        return;
    TraceRec &r = it->second;
    (void)hipEventRecord(r.b, s);
    r.open = false;
    if (g_trace_recs.size() >= 4096)
        trace_drain_locked();
}

namespace {

__global__ void k_derive_rows(int32_t n, const double *__restrict__ diag, double *__restrict__ dinv)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        dinv[i] = diag[i] != 0.0 ? 1.0 / diag[i] : 0.0;
}

// Ah = A D^-1 (column scaling), and binary32 roundings of A and Ah.
__global__ void k_derive_vals(int64_t nnz, const int32_t *__restrict__ ci, const double *__restrict__ val,
                              const double *__restrict__ diag, double *__restrict__ valh,
                              float *__restrict__ val32, float *__restrict__ valh32)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= nnz)
        return;
    const double a = val[j];
    const double d = diag[ci[j]];
    const double h = d != 0.0 ? a / d : 0.0;
    valh[j] = h;
    val32[j] = static_cast<float>(a);
    valh32[j] = static_cast<float>(h);
}

void free_csr(mrhs_csr_s *A)
{
    if (!A)
        return;
    void *ptrs[] = {A->rp,   A->ci,   A->val, A->valh, A->val32, A->valh32, A->diag,
                    A->dinv, A->perm, A->urp, A->uci, A->uval, A->uval32, A->otab,
                    A->code[0], A->code[1], A->code[2], A->code[3],
                    A->ccode[0], A->ccode[1], A->ccode[2], A->ccode[3],
                    A->vtab[0], A->vtab[1], A->vtab[2], A->vtab[3]};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete A;
}

template <typename T>
mrhs_status dev_alloc(T **p, size_t count, size_t &total)
{
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void **>(p), bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(MRHS_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    total += bytes;
    return MRHS_OK;
}

constexpr size_t kPad = 4;  // elements of padding after the nnz entries

// ---- dictionary form (CsrView::code, CsrView::ccode) --------------------------
// Uploads the codes and value table of value array k (host values hv) when
// it has a dictionary form.
template <typename V>
mrhs_status dict_array(mrhs_csr_s *A, const int32_t *rp, const int32_t *ci, const V *hv,
                       const dict::Offsets &offs, int k, size_t &total)
{
    dict::Codes<V> c = dict::codes<V>(A->n, A->nnz, rp, ci, hv, offs);
    if (!c.ok)
        return MRHS_OK;
    V *dtab = nullptr;
    mrhs_status st;
    if ((st = dev_alloc(&dtab, c.tab.size(), total)))
        return st;
    A->vtab[k] = dtab;
    A->nvals[k] = static_cast<int32_t>(c.tab.size());
    hipError_t e = hipMemcpy(dtab, c.tab.data(), sizeof(V) * c.tab.size(), hipMemcpyHostToDevice);
    if (offs.ok) {
        if ((st = dev_alloc(&A->code[k], c.code.size(), total)))
            return st;
        if (e == hipSuccess)
            e = hipMemcpy(A->code[k], c.code.data(), sizeof(uint16_t) * c.code.size(), hipMemcpyHostToDevice);
    } else {
        if ((st = dev_alloc(&A->ccode[k], c.ccode.size(), total)))
            return st;
        A->cbits[k] = c.cb;
        if (e == hipSuccess)
            e = hipMemcpy(A->ccode[k], c.ccode.data(), sizeof(uint32_t) * c.ccode.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "dictionary upload failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}

// Builds the dictionary form of the solver arrays (rp, ci: the solver's
// numbering, sval: its binary64 values on the host; the derived arrays are
// read back from the device, so the tables hold exactly the values the
// products use): 16-bit codes when the matrix has at most kDictOffs distinct
// column offsets, else 32-bit column codes.  MRHS_CSR_DICT=0 turns it off.
mrhs_status build_dict(mrhs_csr_s *A, const int32_t *rp, const int32_t *ci, const double *sval, size_t &total)
{
    if (!env_int("MRHS_CSR_DICT", 1, 0, 1) || A->nnz == 0)
        return MRHS_OK;
    dict::Offsets offs;
    dict::offsets(A->n, rp, ci, offs);
    mrhs_status st;
    hipError_t e;
    if (offs.ok) {
        A->noffs = static_cast<int32_t>(offs.set.keys.size());
        A->ob = offs.ob;
        std::vector<int32_t> otab(offs.set.keys.begin(), offs.set.keys.end());
        if ((st = dev_alloc(&A->otab, otab.size(), total)))
            return st;
        if ((e = hipMemcpy(A->otab, otab.data(), sizeof(int32_t) * otab.size(), hipMemcpyHostToDevice)))
            return set_error(MRHS_EDEVICE, "dictionary upload failed: %s", hipGetErrorString(e));
    }
    const dict::Offsets &po = offs;
    const size_t nnz = static_cast<size_t>(A->nnz);
    if ((st = dict_array<double>(A, rp, ci, sval, po, 0, total)))
        return st;
    {
        std::vector<double> h(nnz);
        if ((e = hipMemcpy(h.data(), A->valh, sizeof(double) * nnz, hipMemcpyDeviceToHost)))
            return set_error(MRHS_EDEVICE, "read-back failed: %s", hipGetErrorString(e));
        if ((st = dict_array<double>(A, rp, ci, h.data(), po, 1, total)))
            return st;
    }
    std::vector<float> h(nnz);
    const float *src[2] = {A->val32, A->valh32};
    for (int k = 0; k < 2; ++k) {
        if ((e = hipMemcpy(h.data(), src[k], sizeof(float) * nnz, hipMemcpyDeviceToHost)))
            return set_error(MRHS_EDEVICE, "read-back failed: %s", hipGetErrorString(e));
        if ((st = dict_array<float>(A, rp, ci, h.data(), po, 2 + k, total)))
            return st;
    }
    return MRHS_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Do the byte ranges [a, a + na) and [b, b + nb) share a byte?
bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

template <typename T>
struct StoreLaunch {
    const mrhs_csr_s *A;
    const void *X;
    void *Y;
    hipStream_t s;
    template <int M>
    hipError_t operator()() const
    {
        return launch_gspmv<T, M>(user_view<T>(*A),
                                  OpStore<T, M>{static_cast<const T *>(X), static_cast<T *>(Y)},
                                  RedBufs<T>{nullptr, nullptr, nullptr}, s);
    }
};

} // namespace
} // namespace mrhs

using namespace mrhs;

MRHS_API const char *mrhs_last_error(void) { return g_error.c_str(); }

MRHS_API const char *mrhs_version(void) { return "mrhs 0.1 (gfx950)"; }

MRHS_API mrhs_status csr_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                const double *val, uint32_t flags, mrhs_csr *out)
{
    clear_error();
    if (!out)
        return set_error(MRHS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0)
        return set_error(MRHS_EINVAL, "n = %d < 0", n);
    if (nnz < 0 || nnz > INT32_MAX)
        return set_error(MRHS_EINVAL, "nnz = %lld outside [0, 2^31)", static_cast<long long>(nnz));
    if (flags & ~(MRHS_CSR_NULLSPACE_CONST | MRHS_CSR_REORDER))
        return set_error(MRHS_EINVAL, "unknown flags 0x%x", flags);
    if (n > 0 && !row_ptr)
        return set_error(MRHS_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && (!col_idx || !val))
        return set_error(MRHS_EINVAL, "col_idx or val is NULL");
    std::vector<double> diag(static_cast<size_t>(n), 0.0);
    std::vector<int32_t> reach(static_cast<size_t>(n), 0);
    if (n > 0) {
        if (row_ptr[0] != 0)
            return set_error(MRHS_EINVAL, "row_ptr[0] = %d, must be 0", row_ptr[0]);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t a = row_ptr[i], b = row_ptr[i + 1];
            if (b < a)
                return set_error(MRHS_EINVAL, "row_ptr decreases at row %d", i);
            if (b > nnz)
                return set_error(MRHS_EINVAL, "row_ptr[%d] = %d exceeds nnz", i + 1, b);
            for (int32_t j = a; j < b; ++j) {
                const int32_t c = col_idx[j];
                if (c < 0 || c >= n)
                    return set_error(MRHS_EINVAL, "col_idx[%d] = %d outside [0, %d)", j, c, n);
                if (!std::isfinite(val[j]))
                    return set_error(MRHS_EINVAL, "val[%d] is not finite", j);
                if (c == i)
                    diag[i] += val[j];
                reach[i] = std::max(reach[i], c - i);
            }
        }
        if (row_ptr[n] != nnz)
            return set_error(MRHS_EINVAL, "row_ptr[n] = %d differs from nnz = %lld", row_ptr[n],
                             static_cast<long long>(nnz));
    } else if (nnz != 0) {
        return set_error(MRHS_EINVAL, "nnz must be 0 when n = 0");
    }

    auto *A = new (std::nothrow) mrhs_csr_s();
    if (!A)
        return set_error(MRHS_ENOMEM, "host allocation failed");
    A->n = n;
    A->nnz = nnz;
    A->flags = flags;
    (void)hipGetDevice(&A->device);
    for (int32_t i = 0; i < n; ++i)
        if (diag[i] == 0.0)
            A->zero_diag = true;
    if (n > 0) {  // the tile schedule of the products uses the median reach
        std::nth_element(reach.begin(), reach.begin() + n / 2, reach.end());
        A->reach = reach[n / 2];
    }
    if (n == 0) {
        *out = A;
        return MRHS_OK;
    }
    // MRHS_CSR_REORDER: the solvers get P A P^T (rows and columns renumbered
    // by reverse Cuthill-McKee), the caller's arrays are kept for gspmv
    std::vector<int32_t> perm, prp, pci;
    std::vector<double> pval, pdiag;
    const int32_t *user_rp = row_ptr, *user_ci = col_idx;  // the caller's numbering
    if (flags & MRHS_CSR_REORDER) {
        perm.resize(n);
        rcm_permutation(n, row_ptr, col_idx, perm.data());
        std::vector<int32_t> iperm(n);
        for (int32_t k = 0; k < n; ++k)
            iperm[perm[k]] = k;
        prp.assign(static_cast<size_t>(n) + 1, 0);
        pci.resize(static_cast<size_t>(nnz));
        pval.resize(static_cast<size_t>(nnz));
        pdiag.resize(n);
        std::vector<int32_t> preach(n, 0);
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t k = 0; k < n; ++k) {
            const int32_t i = perm[k];
            row.clear();
            for (int32_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
                row.emplace_back(iperm[col_idx[j]], val[j]);
            // entries of a row keep their relative order among equal columns
            std::stable_sort(row.begin(), row.end(),
                             [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                                 return a.first < b.first;
                             });
            int32_t w = prp[k];
            for (const auto &e : row) {
                pci[w] = e.first;
                pval[w] = e.second;
                preach[k] = std::max(preach[k], e.first - k);
                ++w;
            }
            prp[k + 1] = w;
            pdiag[k] = diag[i];
        }
        A->ureach = A->reach;
        std::nth_element(preach.begin(), preach.begin() + n / 2, preach.end());
        A->reach = preach[n / 2];
        row_ptr = prp.data();
        col_idx = pci.data();
        diag.swap(pdiag);
    }
    const double *sval = (flags & MRHS_CSR_REORDER) ? pval.data() : val;
    size_t total = 0;
    mrhs_status st = MRHS_OK;
    if ((st = dev_alloc(&A->rp, static_cast<size_t>(n) + 1, total)) ||
        (st = dev_alloc(&A->ci, static_cast<size_t>(nnz) + kPad, total)) ||
        (st = dev_alloc(&A->val, static_cast<size_t>(nnz) + kPad, total)) ||
        (st = dev_alloc(&A->valh, static_cast<size_t>(nnz) + kPad, total)) ||
        (st = dev_alloc(&A->val32, static_cast<size_t>(nnz) + kPad, total)) ||
        (st = dev_alloc(&A->valh32, static_cast<size_t>(nnz) + kPad, total)) ||
        (st = dev_alloc(&A->diag, static_cast<size_t>(n), total)) ||
        (st = dev_alloc(&A->dinv, static_cast<size_t>(n), total))) {
        free_csr(A);
        return st;
    }
    A->bytes = total;
    hipError_t e = hipSuccess;
    // the padding past nnz is read (never used) by whole-vector tile loads
    if ((e = hipMemset(A->ci + nnz, 0, sizeof(int32_t) * kPad)) ||
        (e = hipMemset(A->val + nnz, 0, sizeof(double) * kPad)) ||
        (e = hipMemset(A->valh + nnz, 0, sizeof(double) * kPad)) ||
        (e = hipMemset(A->val32 + nnz, 0, sizeof(float) * kPad)) ||
        (e = hipMemset(A->valh32 + nnz, 0, sizeof(float) * kPad))) {
        free_csr(A);
        return set_error(MRHS_EDEVICE, "padding fill failed: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(A->rp, row_ptr, sizeof(int32_t) * (static_cast<size_t>(n) + 1), hipMemcpyHostToDevice)) ||
        (nnz > 0 && (e = hipMemcpy(A->ci, col_idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice))) ||
        (nnz > 0 && (e = hipMemcpy(A->val, sval, sizeof(double) * nnz, hipMemcpyHostToDevice))) ||
        (e = hipMemcpy(A->diag, diag.data(), sizeof(double) * n, hipMemcpyHostToDevice))) {
        free_csr(A);
        return set_error(MRHS_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    if (flags & MRHS_CSR_REORDER) {
        // the caller's numbering, for gspmv: row offsets, columns, binary64
        // values and their binary32 rounding
        std::vector<float> v32(static_cast<size_t>(nnz));
        for (int64_t j = 0; j < nnz; ++j)
            v32[j] = static_cast<float>(val[j]);  // round to nearest even
        if ((st = dev_alloc(&A->perm, static_cast<size_t>(n), total)) ||
            (st = dev_alloc(&A->urp, static_cast<size_t>(n) + 1, total)) ||
            (st = dev_alloc(&A->uci, static_cast<size_t>(nnz) + kPad, total)) ||
            (st = dev_alloc(&A->uval, static_cast<size_t>(nnz) + kPad, total)) ||
            (st = dev_alloc(&A->uval32, static_cast<size_t>(nnz) + kPad, total))) {
            free_csr(A);
            return st;
        }
        A->bytes = total;
        if ((e = hipMemset(A->uci + nnz, 0, sizeof(int32_t) * kPad)) ||
            (e = hipMemset(A->uval + nnz, 0, sizeof(double) * kPad)) ||
            (e = hipMemset(A->uval32 + nnz, 0, sizeof(float) * kPad)) ||
            (e = hipMemcpy(A->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(A->urp, user_rp, sizeof(int32_t) * (static_cast<size_t>(n) + 1), hipMemcpyHostToDevice)) ||
            (nnz > 0 && (e = hipMemcpy(A->uci, user_ci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice))) ||
            (nnz > 0 && (e = hipMemcpy(A->uval, val, sizeof(double) * nnz, hipMemcpyHostToDevice))) ||
            (nnz > 0 && (e = hipMemcpy(A->uval32, v32.data(), sizeof(float) * nnz, hipMemcpyHostToDevice)))) {
            free_csr(A);
            return set_error(MRHS_EDEVICE, "upload failed: %s", hipGetErrorString(e));
        }
    }
    hipLaunchKernelGGL(k_derive_rows, dim3((n + 255) / 256), dim3(256), 0, 0, n, A->diag, A->dinv);
    if (nnz > 0)
        hipLaunchKernelGGL(k_derive_vals, dim3(static_cast<unsigned>((nnz + 255) / 256)), dim3(256), 0, 0, nnz,
                           A->ci, A->val, A->diag, A->valh, A->val32, A->valh32);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        free_csr(A);
        return set_error(MRHS_EDEVICE, "derive kernels failed: %s", hipGetErrorString(e));
    }
    if ((st = build_dict(A, row_ptr, col_idx, sval, total))) {
        free_csr(A);
        return st;
    }
    A->bytes = total;
    *out = A;
    return MRHS_OK;
}

MRHS_API mrhs_status csr_destroy(mrhs_csr A)
{
    clear_error();
    if (A) {
        (void)hipDeviceSynchronize();
        free_csr(A);
    }
    return MRHS_OK;
}

MRHS_API mrhs_status csr_info(mrhs_csr A, int32_t *n, int64_t *nnz, size_t *device_bytes)
{
    clear_error();
    if (!A)
        return set_error(MRHS_EINVAL, "matrix handle is NULL");
    if (n)
        *n = A->n;
    if (nnz)
        *nnz = A->nnz;
    if (device_bytes)
        *device_bytes = A->bytes;
    return MRHS_OK;
}

MRHS_API mrhs_status csr_stream_bytes(mrhs_csr A, int32_t dtype, int32_t scaled, int64_t *bytes)
{
    clear_error();
    if (!A || !bytes)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (dtype != MRHS_F64 && dtype != MRHS_F32)
        return set_error(MRHS_EINVAL, "unknown dtype %d", dtype);
    const int k = (dtype == MRHS_F64 ? 0 : 2) + (scaled ? 1 : 0);
    const int64_t per = A->code[k] ? 2 : A->ccode[k] ? 4 : 4 + (dtype == MRHS_F64 ? 8 : 4);
    *bytes = 4 * (static_cast<int64_t>(A->n) + 1) + per * A->nnz;
    return MRHS_OK;
}

MRHS_API mrhs_status gspmv_ex(mrhs_csr A, int32_t dtype, const void *X, void *Y, int32_t m, void *hip_stream)
{
    clear_error();
    if (!A)
        return set_error(MRHS_EINVAL, "matrix handle is NULL");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    if (dtype != MRHS_F64 && dtype != MRHS_F32)
        return set_error(MRHS_EINVAL, "unknown dtype %d", dtype);
    if (A->n == 0)
        return MRHS_OK;
    if (!X || !Y)
        return set_error(MRHS_EINVAL, "X or Y is NULL");
    const size_t blk = static_cast<size_t>(A->n) * m * (dtype == MRHS_F64 ? sizeof(double) : sizeof(float));
    if (overlap(X, blk, Y, blk))
        return set_error(MRHS_EINVAL, "X and Y overlap");
    if (!aligned16(X) || !aligned16(Y))
        return set_error(MRHS_EINVAL, "X and Y must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = dtype == MRHS_F64 ? dispatch_m(m, StoreLaunch<double>{A, X, Y, s})
                                     : dispatch_m(m, StoreLaunch<float>{A, X, Y, s});
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "gspmv launch failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}

MRHS_API mrhs_status gspmv(mrhs_csr A, const double *X, double *Y, int32_t m)
{
    return gspmv_ex(A, MRHS_F64, X, Y, m, nullptr);
}

MRHS_API mrhs_status block_bicgstab_workspace_size(mrhs_csr A, int32_t m, uint32_t flags, size_t *bytes)
{
    clear_error();
    if (!A || !bytes)
        return set_error(MRHS_EINVAL, "NULL argument");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    *bytes = solve_workspace_bytes(*A, m, flags);
    return MRHS_OK;
}

MRHS_API mrhs_status block_bicgstab_ex(mrhs_csr A, const double *B, double *X, int32_t m, double tol,
                                       int32_t maxit, uint32_t flags, void *workspace, size_t ws_bytes,
                                       void *hip_stream, mrhs_col_info *info)
{
    clear_error();
    if (!A)
        return set_error(MRHS_EINVAL, "matrix handle is NULL");
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    if (!(tol > 0.0) || !std::isfinite(tol))
        return set_error(MRHS_EINVAL, "tol must be positive and finite");
    if (maxit < 1)
        return set_error(MRHS_EINVAL, "maxit must be at least 1");
    if (flags & ~(MRHS_X0_GIVEN | MRHS_MIXED))
        return set_error(MRHS_EINVAL, "unknown flags 0x%x", flags);
    if (A->n == 0) {
        if (info)
            for (int i = 0; i < m; ++i)
                info[i] = mrhs_col_info{0, 0, 0, MRHS_OK, 0.0};
        return MRHS_OK;
    }
    if (!B || !X)
        return set_error(MRHS_EINVAL, "B or X is NULL");
    const size_t blk = static_cast<size_t>(A->n) * m * sizeof(double);
    if (overlap(B, blk, X, blk))
        return set_error(MRHS_EINVAL, "B and X overlap");
    if (workspace && (overlap(workspace, ws_bytes, B, blk) || overlap(workspace, ws_bytes, X, blk)))
        return set_error(MRHS_EINVAL, "the workspace overlaps B or X");
    if (!aligned16(B) || !aligned16(X) || (workspace && !aligned16(workspace)))
        return set_error(MRHS_EINVAL, "B, X and the workspace must be 16-byte aligned");
    if (A->zero_diag)
        return set_error(MRHS_EINVAL, "the matrix has a zero diagonal entry (Jacobi preconditioner undefined)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t need = solve_workspace_bytes(*A, m, flags);
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
    const mrhs_status st = block_solve(*A, B, X, SolveParams{m, tol, maxit, flags}, ws, ws_bytes, s, info);
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
    }
    return st;
}

MRHS_API mrhs_status block_bicgstab(mrhs_csr A, const double *B, double *X, int32_t m, double tol, int32_t maxit)
{
    return block_bicgstab_ex(A, B, X, m, tol, maxit, 0u, nullptr, 0, nullptr, nullptr);
}

MRHS_API mrhs_status mrhs_trace_enable(int every)
{
    clear_error();
    if (every < 0)
        return set_error(MRHS_EINVAL, "trace period must be >= 0, got %d", every);
    std::lock_guard<std::mutex> lk(g_trace_mu);
    trace_drain_locked();
    if (every)
        g_trace_stats.clear();
    g_trace_every = every;
    return MRHS_OK;
}

MRHS_API mrhs_status mrhs_trace_read(char *buf, size_t cap, size_t *len)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_trace_mu);
    trace_drain_locked();
    std::string out = "{";
    bool first = true;
    for (const auto &kv : g_trace_stats) {
        char item[320];
        std::snprintf(item, sizeof(item),
                      "%s\"%s\": {\"seen\": %lld, \"launches\": %lld, \"total_ms\": %.6f, \"min_ms\": %.6f, "
                      "\"max_ms\": %.6f}",
                      first ? "" : ", ", kv.first.c_str(), static_cast<long long>(kv.second.seen),
                      static_cast<long long>(kv.second.launches), kv.second.total_ms, kv.second.min_ms,
                      kv.second.max_ms);
        out += item;
        first = false;
    }
    out += "}";
    if (len)
        *len = out.size();
    if (buf && cap > 0) {
        const size_t k = std::min(cap - 1, out.size());
        std::memcpy(buf, out.data(), k);
        buf[k] = '\0';
        if (k < out.size())
            return set_error(MRHS_EINVAL, "buffer of %zu bytes too small for %zu", cap, out.size() + 1);
    }
    return MRHS_OK;
}
