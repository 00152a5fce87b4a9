// Ensemble projection step on the staggered channel grid (Section 2.2,
// eqs. (3)-(4)): for m preliminary velocity fields u* at once, the pressure
// right-hand side -(1/tau) D u* and the correction u = u* - tau G p, with D
// the volume-integrated discrete divergence and G the face-normal pressure
// gradient.  Both use the face areas and centre distances of the
// finite-volume pressure operator (x-faces dy_j dz over dx, y-faces dx dz
// over the centre distance, z-faces dx dy_j over dz), so D G = -A for the
// channel pressure matrix A: the block solve of A p = -(1/tau) D u* makes
// D u = 0 up to its residual.
//
// Layout.  Cells (i, j, k), x fastest, nx*ny*nz of them; fluid cells carry
// the pressure unknowns in natural order (solid cells skipped), as the
// channel matrix numbers them.  Face blocks are row-interleaved n_faces x m:
//   U: x-face (i, j, k) = west face of cell (i, j, k), nz*ny*nx rows (periodic);
//   V: y-face (i, j, k) between cells (i, j-1, k) and (i, j, k), j = 0..ny,
//      nz*(ny+1)*nx rows (j = 0 and j = ny are the walls);
//   W: z-face (i, j, k) = back face of cell (i, j, k), nz*ny*nx rows (periodic).
// A face on a wall or touching a solid cell is closed: it carries no flux,
// is ignored by the divergence and never changed by the correction.
//
// Both kernels stream the cells in natural order with the lane layout of the
// products (a lane holds VW consecutive columns of one cell), so every face
// and pressure access of a wave is whole rows; the neighbours' rows (i+1,
// j+1, k+1 / i-1, j-1, k-1) were or will be touched by nearby waves and come
// from cache.  HBM-bound: per cell the divergence moves about three face rows
// in and one pressure row out, the correction one pressure row in and three
// face rows in and out.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

struct mrhs_grid_s {
    int32_t nx = 0, ny = 0, nz = 0;
    int32_t n = 0;            // fluid cells (pressure unknowns)
    int64_t ncell = 0;
    double dx = 0.0, dz = 0.0;
    double *dy = nullptr;     // [ny] cell heights
    double *inv_dyc = nullptr;  // [ny] 1 / (yc_j - yc_{j-1}); entry 0 unused
    int32_t *num = nullptr;   // [ncell] fluid number or -1 for a solid cell
    int device = 0;
    size_t bytes = 0;
};

namespace mrhs {
namespace {

struct ProjGeom {
    int32_t nx, ny, nz;
    int64_t ncell;
    double dx, dz;
    const double *__restrict__ dy;
    const double *__restrict__ inv_dyc;
    const int32_t *__restrict__ num;
};

// Cells of the grid-stride loop of this lane: c = first, first + stride, ...
template <int M>
struct CellLoop {
    using S = Shape<double, M>;
    int64_t first, stride;
    __device__ CellLoop()
        : first(static_cast<int64_t>(blockIdx.x) * S::RPP + S::row_of(threadIdx.x)),
          stride(static_cast<int64_t>(gridDim.x) * S::RPP)
    {
    }
};

// B[fluid(c)] = scale * (D U)_c for every fluid cell c.
template <int M>
__global__ void __launch_bounds__(kBlock) k_proj_rhs(ProjGeom G, const double *__restrict__ U,
                                                    const double *__restrict__ V, const double *__restrict__ W,
                                                    double scale, double *__restrict__ B)
{
    using S = Shape<double, M>;
    const int g = S::lane_of(threadIdx.x);
    if (!S::used(threadIdx.x) || g >= S::G)
        return;
    const CellLoop<M> L;
    const int64_t plane = static_cast<int64_t>(G.nx) * G.ny;
    const int64_t vplane = static_cast<int64_t>(G.nx) * (G.ny + 1);
    for (int64_t c = L.first; c < G.ncell; c += L.stride) {
        const int32_t me = G.num[c];
        if (me < 0)
            continue;
        const int i = static_cast<int>(c % G.nx);
        const int j = static_cast<int>((c / G.nx) % G.ny);
        const int k = static_cast<int>(c / plane);
        const int64_t cw = i == 0 ? c + (G.nx - 1) : c - 1;
        const int64_t ce = i == G.nx - 1 ? c - (G.nx - 1) : c + 1;
        const int64_t cb = k == 0 ? c + (G.nz - 1) * plane : c - plane;
        const int64_t cf = k == G.nz - 1 ? c - (G.nz - 1) * plane : c + plane;
        const bool ow = G.num[cw] >= 0, oe = G.num[ce] >= 0;
        const bool ob = G.num[cb] >= 0, of = G.num[cf] >= 0;
        const bool os = j > 0 && G.num[c - G.nx] >= 0;
        const bool on = j < G.ny - 1 && G.num[c + G.nx] >= 0;
        const int64_t vs = k * vplane + static_cast<int64_t>(j) * G.nx + i;  // south face; north = vs + nx
        const double ax = G.dy[j] * G.dz, ay = G.dx * G.dz, az = G.dx * G.dy[j];
        double uw[S::VW], ue[S::VW], vsv[S::VW], vnv[S::VW], wb[S::VW], wf[S::VW];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            uw[q] = ue[q] = vsv[q] = vnv[q] = wb[q] = wf[q] = 0.0;
        if (ow)
            ld<double, M>(U, static_cast<int32_t>(c), g, uw);
        if (oe)
            ld<double, M>(U, static_cast<int32_t>(ce), g, ue);
        if (os)
            ld<double, M>(V, static_cast<int32_t>(vs), g, vsv);
        if (on)
            ld<double, M>(V, static_cast<int32_t>(vs + G.nx), g, vnv);
        if (ob)
            ld<double, M>(W, static_cast<int32_t>(c), g, wb);
        if (of)
            ld<double, M>(W, static_cast<int32_t>(cf), g, wf);
        double d[S::VW];
#pragma unroll
        for (int q = 0; q < S::VW; ++q)
            d[q] = scale * (ax * (ue[q] - uw[q]) + ay * (vnv[q] - vsv[q]) + az * (wf[q] - wb[q]));
        st<double, M>(B, me, g, d);
    }
}

// U -= tau G P on every open face, each face updated by the cell on its
// upper side (east for x-faces, north for y-faces, front for z-faces).
template <int M>
__global__ void __launch_bounds__(kBlock) k_proj_correct(ProjGeom G, double *__restrict__ U,
                                                        double *__restrict__ V, double *__restrict__ W,
                                                        const double *__restrict__ P, double tau)
{
    using S = Shape<double, M>;
    const int g = S::lane_of(threadIdx.x);
    if (!S::used(threadIdx.x) || g >= S::G)
        return;
    const CellLoop<M> L;
    const int64_t plane = static_cast<int64_t>(G.nx) * G.ny;
    const int64_t vplane = static_cast<int64_t>(G.nx) * (G.ny + 1);
    const double tx = tau / G.dx, tz = tau / G.dz;
    for (int64_t c = L.first; c < G.ncell; c += L.stride) {
        const int32_t me = G.num[c];
        if (me < 0)
            continue;
        const int i = static_cast<int>(c % G.nx);
        const int j = static_cast<int>((c / G.nx) % G.ny);
        const int k = static_cast<int>(c / plane);
        const int64_t cw = i == 0 ? c + (G.nx - 1) : c - 1;
        const int64_t cb = k == 0 ? c + (G.nz - 1) * plane : c - plane;
        const int32_t nw = G.num[cw], nb = G.num[cb];
        const int32_t ns = j > 0 ? G.num[c - G.nx] : -1;
        double p[S::VW], q_[S::VW], f[S::VW];
        ld<double, M>(P, me, g, p);
        if (nw >= 0) {
            ld<double, M>(P, nw, g, q_);
            ld<double, M>(U, static_cast<int32_t>(c), g, f);
#pragma unroll
            for (int q = 0; q < S::VW; ++q)
                f[q] -= tx * (p[q] - q_[q]);
            st<double, M>(U, static_cast<int32_t>(c), g, f);
        }
        if (ns >= 0) {
            const int64_t vs = k * vplane + static_cast<int64_t>(j) * G.nx + i;
            const double ty = tau * G.inv_dyc[j];
            ld<double, M>(P, ns, g, q_);
            ld<double, M>(V, static_cast<int32_t>(vs), g, f);
#pragma unroll
            for (int q = 0; q < S::VW; ++q)
                f[q] -= ty * (p[q] - q_[q]);
            st<double, M>(V, static_cast<int32_t>(vs), g, f);
        }
        if (nb >= 0) {
            ld<double, M>(P, nb, g, q_);
            ld<double, M>(W, static_cast<int32_t>(c), g, f);
#pragma unroll
            for (int q = 0; q < S::VW; ++q)
                f[q] -= tz * (p[q] - q_[q]);
            st<double, M>(W, static_cast<int32_t>(c), g, f);
        }
    }
}

ProjGeom geom(const mrhs_grid_s &G)
{
    return {G.nx, G.ny, G.nz, G.ncell, G.dx, G.dz, G.dy, G.inv_dyc, G.num};
}

template <int M>
unsigned cell_grid(const mrhs_grid_s &G)
{
    const int64_t need = (G.ncell + Shape<double, M>::RPP - 1) / Shape<double, M>::RPP;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(need, 8 * 2048)));
}

struct RhsLaunch {
    const mrhs_grid_s *G;
    const double *U, *V, *W;
    double scale;
    double *B;
    hipStream_t s;
    template <int M>
    hipError_t operator()() const
    {
        hipLaunchKernelGGL(k_proj_rhs<M>, dim3(cell_grid<M>(*G)), dim3(kBlock), 0, s, geom(*G), U, V, W, scale, B);
        return hipGetLastError();
    }
};

struct CorrectLaunch {
    const mrhs_grid_s *G;
    double *U, *V, *W;
    const double *P;
    double tau;
    hipStream_t s;
    template <int M>
    hipError_t operator()() const
    {
        hipLaunchKernelGGL(k_proj_correct<M>, dim3(cell_grid<M>(*G)), dim3(kBlock), 0, s, geom(*G), U, V, W, P, tau);
        return hipGetLastError();
    }
};

void free_grid(mrhs_grid_s *G)
{
    if (!G)
        return;
    void *ptrs[] = {G->dy, G->inv_dyc, G->num};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete G;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

// Checks the face blocks (and one cell block) of a projection call.
mrhs_status check_blocks(const mrhs_grid_s &G, int32_t m, const void *U, const void *V, const void *W,
                         const void *C)
{
    if (m < 1 || m > kMaxM)
        return set_error(MRHS_EINVAL, "m = %d outside [1, 16]", m);
    if (!U || !V || !W || !C)
        return set_error(MRHS_EINVAL, "a block pointer is NULL");
    if (!aligned16(U) || !aligned16(V) || !aligned16(W) || !aligned16(C))
        return set_error(MRHS_EINVAL, "blocks must be 16-byte aligned");
    const size_t row = sizeof(double) * static_cast<size_t>(m);
    const size_t nu = row * static_cast<size_t>(G.ncell);
    const size_t nv = row * static_cast<size_t>(G.nz) * (G.ny + 1) * G.nx;
    const size_t nc = row * static_cast<size_t>(G.n);
    const void *p[4] = {U, V, W, C};
    const size_t sz[4] = {nu, nv, nu, nc};
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (overlap(p[a], sz[a], p[b], sz[b]))
                return set_error(MRHS_EINVAL, "the U, V, W and cell blocks must not overlap");
    return MRHS_OK;
}

} // namespace
} // namespace mrhs

using namespace mrhs;

MRHS_API mrhs_status grid_create(int32_t nx, int32_t ny, int32_t nz, double dx, double dz, const double *y_faces,
                                 const uint8_t *solid, mrhs_grid *out)
{
    clear_error();
    if (!out)
        return set_error(MRHS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 3 || nz < 3 || ny < 1)
        return set_error(MRHS_EINVAL, "need nx >= 3, nz >= 3 (periodic) and ny >= 1, got %d %d %d", nx, ny, nz);
    if (!(dx > 0.0) || !(dz > 0.0) || !std::isfinite(dx) || !std::isfinite(dz))
        return set_error(MRHS_EINVAL, "dx and dz must be positive and finite");
    if (!y_faces)
        return set_error(MRHS_EINVAL, "y_faces is NULL");
    for (int32_t j = 0; j <= ny; ++j)
        if (!std::isfinite(y_faces[j]) || (j > 0 && !(y_faces[j] > y_faces[j - 1])))
            return set_error(MRHS_EINVAL, "y_faces must be finite and strictly increasing (at %d)", j);
    const int64_t ncell = static_cast<int64_t>(nx) * ny * nz;
    const int64_t vrows = static_cast<int64_t>(nx) * (ny + 1) * nz;
    if (vrows > INT32_MAX)
        return set_error(MRHS_EINVAL, "grid of %lld y-faces exceeds 2^31 - 1", static_cast<long long>(vrows));
    std::vector<int32_t> num(static_cast<size_t>(ncell));
    int64_t n = 0;
    for (int64_t c = 0; c < ncell; ++c)
        num[c] = (solid && solid[c]) ? -1 : static_cast<int32_t>(n++);
    std::vector<double> dy(ny), inv_dyc(ny, 0.0);
    for (int32_t j = 0; j < ny; ++j)
        dy[j] = y_faces[j + 1] - y_faces[j];
    for (int32_t j = 1; j < ny; ++j)
        inv_dyc[j] = 1.0 / (0.5 * (y_faces[j] + y_faces[j + 1]) - 0.5 * (y_faces[j - 1] + y_faces[j]));
    auto *G = new (std::nothrow) mrhs_grid_s();
    if (!G)
        return set_error(MRHS_ENOMEM, "host allocation failed");
    G->nx = nx;
    G->ny = ny;
    G->nz = nz;
    G->n = static_cast<int32_t>(n);
    G->ncell = ncell;
    G->dx = dx;
    G->dz = dz;
    (void)hipGetDevice(&G->device);
    const size_t bnum = sizeof(int32_t) * static_cast<size_t>(ncell), by = sizeof(double) * ny;
    if (hipMalloc(reinterpret_cast<void **>(&G->num), bnum) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&G->dy), by) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&G->inv_dyc), by) != hipSuccess) {
        (void)hipGetLastError();
        free_grid(G);
        return set_error(MRHS_ENOMEM, "device allocation of the grid failed");
    }
    G->bytes = bnum + 2 * by;
    hipError_t e = hipSuccess;
    if ((e = hipMemcpy(G->num, num.data(), bnum, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(G->dy, dy.data(), by, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(G->inv_dyc, inv_dyc.data(), by, hipMemcpyHostToDevice))) {
        free_grid(G);
        return set_error(MRHS_EDEVICE, "grid upload failed: %s", hipGetErrorString(e));
    }
    *out = G;
    return MRHS_OK;
}

MRHS_API mrhs_status grid_destroy(mrhs_grid G)
{
    clear_error();
    if (G) {
        (void)hipDeviceSynchronize();
        free_grid(G);
    }
    return MRHS_OK;
}

MRHS_API mrhs_status grid_info(mrhs_grid G, int32_t *n_fluid, int64_t *cells, int64_t *v_faces)
{
    clear_error();
    if (!G)
        return set_error(MRHS_EINVAL, "grid handle is NULL");
    if (n_fluid)
        *n_fluid = G->n;
    if (cells)
        *cells = G->ncell;
    if (v_faces)
        *v_faces = static_cast<int64_t>(G->nx) * (G->ny + 1) * G->nz;
    return MRHS_OK;
}

MRHS_API mrhs_status projection_rhs(mrhs_grid G, const double *U, const double *V, const double *W, double tau,
                                    double *B, int32_t m, void *hip_stream)
{
    clear_error();
    if (!G)
        return set_error(MRHS_EINVAL, "grid handle is NULL");
    if (!(tau != 0.0) || !std::isfinite(tau))
        return set_error(MRHS_EINVAL, "tau must be finite and nonzero");
    mrhs_status st = check_blocks(*G, m, U, V, W, B);
    if (st != MRHS_OK)
        return st;
    const hipError_t e =
        dispatch_m(m, RhsLaunch{G, U, V, W, -1.0 / tau, B, static_cast<hipStream_t>(hip_stream)});
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "projection_rhs launch failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}

MRHS_API mrhs_status projection_correct(mrhs_grid G, double *U, double *V, double *W, const double *P, double tau,
                                        int32_t m, void *hip_stream)
{
    clear_error();
    if (!G)
        return set_error(MRHS_EINVAL, "grid handle is NULL");
    if (!std::isfinite(tau))
        return set_error(MRHS_EINVAL, "tau must be finite");
    mrhs_status st = check_blocks(*G, m, U, V, W, P);
    if (st != MRHS_OK)
        return st;
    const hipError_t e =
        dispatch_m(m, CorrectLaunch{G, U, V, W, P, tau, static_cast<hipStream_t>(hip_stream)});
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "projection_correct launch failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}
