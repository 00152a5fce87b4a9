// CPU driver for the library's AMG setup (amg_setup.hip is host-only C++):
// reads a CRS matrix, builds the hierarchy, writes it out, so the test suite
// can compare it with the oracle's without a GPU.  Built and run by
// tests/test_amg_setup_cpu.py.
//
// input  (binary, little endian): int32 n, int64 nnz, int32 nullspace,
//        int32 row_ptr[n+1], int32 col[nnz], float64 val[nnz]
// output: int32 levels; per level: int32 rows, int64 nnz_a, row_ptr, col, val,
//         float64 dl1_inv[rows]; for every level but the coarsest also
//         int8 cf[rows], int32 cols_p, int64 nnz_p, row_ptr, col, val of P;
//         then int32 nc, float64 coarse_inv[nc*nc]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "amg.h"

template <typename T>
static void rd(FILE *f, T *p, size_t n)
{
    if (n && std::fread(p, sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short read\n");
        std::exit(2);
    }
}
template <typename T>
static void wr(FILE *f, const T *p, size_t n)
{
    if (n)
        std::fwrite(p, sizeof(T), n, f);
}

int main(int argc, char **argv)
{
    if (argc != 3)
        return 2;
    FILE *in = std::fopen(argv[1], "rb");
    if (!in)
        return 2;
    int32_t n = 0, ns = 0;
    int64_t nnz = 0;
    rd(in, &n, 1);
    rd(in, &nnz, 1);
    rd(in, &ns, 1);
    std::vector<int32_t> rp(n + 1), ci(nnz);
    std::vector<double> va(nnz);
    rd(in, rp.data(), rp.size());
    rd(in, ci.data(), ci.size());
    rd(in, va.data(), va.size());
    std::fclose(in);
    mrhs::amg::HostHierarchy H;
    const char *err = nullptr;
    if (!mrhs::amg::setup(n, rp.data(), ci.data(), va.data(), ns != 0, mrhs::amg::Params{}, &H, &err)) {
        std::fprintf(stderr, "setup failed: %s\n", err);
        return 1;
    }
    FILE *out = std::fopen(argv[2], "wb");
    const int32_t L = static_cast<int32_t>(H.levels.size());
    wr(out, &L, 1);
    for (int32_t l = 0; l < L; ++l) {
        const auto &lv = H.levels[l];
        const int64_t na = lv.A.nnz();
        wr(out, &lv.A.nr, 1);
        wr(out, &na, 1);
        wr(out, lv.A.rp.data(), lv.A.rp.size());
        wr(out, lv.A.ci.data(), lv.A.ci.size());
        wr(out, lv.A.va.data(), lv.A.va.size());
        wr(out, lv.dl1_inv.data(), lv.dl1_inv.size());
        if (l + 1 < L) {
            const int64_t np = lv.P.nnz();
            wr(out, lv.cf.data(), lv.cf.size());
            wr(out, &lv.P.nc, 1);
            wr(out, &np, 1);
            wr(out, lv.P.rp.data(), lv.P.rp.size());
            wr(out, lv.P.ci.data(), lv.P.ci.size());
            wr(out, lv.P.va.data(), lv.P.va.size());
        }
    }
    const int32_t nc = H.levels.back().A.nr;
    wr(out, &nc, 1);
    wr(out, H.coarse_inv.data(), H.coarse_inv.size());
    std::fclose(out);
    return 0;
}
