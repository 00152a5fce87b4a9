// block_bicgstab_noalloc: the block solve with its workspace in a fixed
// device array of the library instead of memory allocated per call, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The array `scratch` below lives in the library's code object; every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only stands in for the
// symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept, and the kernels receive that address as the
// solve's workspace, as they receive a caller's workspace in
// block_bicgstab_ex.  The solve clears what must start at zero itself (the
// reduction tickets and the control block, with fill kernels), so what an
// earlier call left in the array does not matter.  All calls on one GPU share
// its array: calls that overlap in time on one GPU race.
#include <cmath>
#include <mutex>

#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

static __device__ __align__(256) unsigned char scratch[MRHS_NOALLOC_SCRATCH_BYTES];

namespace mrhs {
namespace {

constexpr size_t kScratchBytes = static_cast<size_t>(MRHS_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
mrhs_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(MRHS_EDEVICE, "device %d outside the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(MRHS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MRHS_OK;
}

// Host mirror of the control block (no pinned allocation on this path).
thread_local Ctl t_host_ctl;

} // namespace
} // namespace mrhs

using namespace mrhs;

MRHS_API mrhs_status block_bicgstab_noalloc(mrhs_csr A, const double *B, double *X, int32_t m, double tol,
                                            int32_t maxit, uint32_t flags, void *hip_stream, mrhs_col_info *info)
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
    const uintptr_t b = reinterpret_cast<uintptr_t>(B), x = reinterpret_cast<uintptr_t>(X);
    if (b < x + blk && x < b + blk)
        return set_error(MRHS_EINVAL, "B and X overlap");
    if ((b & 15u) || (x & 15u))
        return set_error(MRHS_EINVAL, "B and X must be 16-byte aligned");
    if (A->zero_diag)
        return set_error(MRHS_EINVAL, "the matrix has a zero diagonal entry (Jacobi preconditioner undefined)");
    const size_t need = solve_workspace_bytes(*A, m, flags);
    if (need > kScratchBytes)
        return set_error(MRHS_EINVAL,
                         "this solve needs %zu bytes of workspace, more than the %zu-byte scratch of "
                         "block_bicgstab_noalloc (use block_bicgstab_ex with a workspace)",
                         need, kScratchBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return set_error(MRHS_EDEVICE, "hipGetDevice failed");
    if (dev != A->device)
        return set_error(MRHS_EINVAL, "the matrix lives on device %d, the current device is %d", A->device, dev);
    void *ws = nullptr;
    const mrhs_status st = scratch_address(dev, &ws);
    if (st != MRHS_OK)
        return st;
    const uintptr_t w = reinterpret_cast<uintptr_t>(ws);
    if ((b < w + need && w < b + blk) || (x < w + need && w < x + blk))
        return set_error(MRHS_EINVAL, "B or X overlaps the library's scratch array");
    return block_solve(*A, B, X, SolveParams{m, tol, maxit, flags}, ws, kScratchBytes,
                       static_cast<hipStream_t>(hip_stream), info, &t_host_ctl);
}
