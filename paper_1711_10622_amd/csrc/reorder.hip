// Bandwidth-reducing row relabelling for matrices whose numbering has no
// locality (the relabelled cube channel): reverse Cuthill-McKee on the
// symmetrized pattern.  With a banded numbering the rows a product gathers
// for one tile lie close together, so one cache line serves several of them;
// with a random numbering every gather fetches a line of its own.
//
// Reverse Cuthill-McKee (Cuthill and McKee 1969; George 1971): every
// connected component is numbered by a breadth-first search from a
// pseudo-peripheral row (George and Liu 1979: repeated searches from a
// lowest-degree row of the last level while the depth grows), each row's
// unnumbered neighbours taken in order of increasing degree (then index), and
// the whole order is reversed.  Components are started from their
// lowest-degree row, smallest index first.  Host code; deterministic.
#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {

void rcm_permutation(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *perm)
{
    // symmetrized pattern without the diagonal, each neighbour once
    std::vector<int64_t> arp(static_cast<size_t>(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) {
                ++arp[i + 1];
                ++arp[ci[k] + 1];
            }
    std::partial_sum(arp.begin(), arp.end(), arp.begin());
    std::vector<int32_t> adj(static_cast<size_t>(arp[n]));
    {
        std::vector<int64_t> fill(arp.begin(), arp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] != i) {
                    adj[fill[i]++] = ci[k];
                    adj[fill[ci[k]]++] = i;
                }
    }
    std::vector<int64_t> brp(static_cast<size_t>(n) + 1, 0);
    {
        int64_t w = 0;
        for (int32_t i = 0; i < n; ++i) {
            auto b = adj.begin() + arp[i], e = adj.begin() + arp[i + 1];
            std::sort(b, e);
            const int64_t len = std::unique(b, e) - b;
            std::copy(b, b + len, adj.begin() + w);
            w += len;
            brp[i + 1] = w;
        }
        adj.resize(static_cast<size_t>(w));
    }
    auto deg = [&](int32_t i) { return brp[i + 1] - brp[i]; };
    auto lower = [&](int32_t a, int32_t b) { return deg(a) < deg(b) || (deg(a) == deg(b) && a < b); };

    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int8_t> done(n, 0);
    std::vector<int32_t> stamp(n, -1), level(n, 0), queue;
    queue.reserve(n);
    int32_t search = 0;
    // breadth-first search over the rows not yet numbered; returns the depth
    // and leaves the rows reached in queue
    auto bfs = [&](int32_t root) {
        ++search;
        queue.clear();
        queue.push_back(root);
        stamp[root] = search;
        level[root] = 0;
        int32_t depth = 0;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int32_t u = queue[h];
            for (int64_t k = brp[u]; k < brp[u + 1]; ++k) {
                const int32_t v = adj[k];
                if (done[v] || stamp[v] == search)
                    continue;
                stamp[v] = search;
                level[v] = level[u] + 1;
                depth = std::max(depth, level[v]);
                queue.push_back(v);
            }
        }
        return depth;
    };
    std::vector<int32_t> cand(n);
    std::iota(cand.begin(), cand.end(), 0);
    std::sort(cand.begin(), cand.end(), lower);
    std::vector<int32_t> nb;
    for (int32_t start : cand) {
        if (done[start])
            continue;
        int32_t root = start;
        int32_t depth = bfs(root);
        for (int it = 0; it < 8; ++it) {  // pseudo-peripheral row
            int32_t best = -1;
            for (int32_t v : queue)
                if (level[v] == depth && (best < 0 || lower(v, best)))
                    best = v;
            const int32_t d2 = bfs(best);
            if (d2 <= depth)
                break;
            root = best;
            depth = d2;
        }
        // Cuthill-McKee order of the component from root
        const size_t first = order.size();
        order.push_back(root);
        done[root] = 1;
        for (size_t h = first; h < order.size(); ++h) {
            const int32_t u = order[h];
            nb.clear();
            for (int64_t k = brp[u]; k < brp[u + 1]; ++k)
                if (!done[adj[k]])
                    nb.push_back(adj[k]);
            std::sort(nb.begin(), nb.end(), lower);
            for (int32_t v : nb) {
                done[v] = 1;
                order.push_back(v);
            }
        }
    }
    for (int32_t k = 0; k < n; ++k)
        perm[k] = order[n - 1 - k];
}

} // namespace mrhs

using namespace mrhs;

MRHS_API mrhs_status csr_reorder_permutation(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t *perm)
{
    clear_error();
    if (n < 0)
        return set_error(MRHS_EINVAL, "n = %d < 0", n);
    if (n == 0)
        return MRHS_OK;
    if (!row_ptr || !perm || (row_ptr[n] > 0 && !col_idx))
        return set_error(MRHS_EINVAL, "NULL argument");
    if (row_ptr[0] != 0)
        return set_error(MRHS_EINVAL, "row_ptr[0] = %d, must be 0", row_ptr[0]);
    for (int32_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i])
            return set_error(MRHS_EINVAL, "row_ptr decreases at row %d", i);
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] < 0 || col_idx[k] >= n)
                return set_error(MRHS_EINVAL, "col_idx[%d] = %d outside [0, %d)", k, col_idx[k], n);
    }
    rcm_permutation(n, row_ptr, col_idx, perm);
    return MRHS_OK;
}
