// Streaming kernels that measure the attainable HBM rates of this device
// (read, write and copy of a large buffer), the ceilings against which the
// products and vector passes are judged: their run time is set by the bytes
// they move (Section 2.3).  Each thread moves 16-byte vectors, four in flight
// at a time.  Workgroup b runs on XCD b % 8; the eight groups each stream one
// contiguous eighth of the buffer, their workgroups interleaved 4 KB apart,
// with 16 workgroups per CU.  Measured on 2 GiB against a grid-wide stride
// and against one contiguous range per workgroup, at 4-32 workgroups per CU:
// read 6.8-7.0 TB/s (grid stride 5.7-6.3), write 5.7-6.1 (3.8-4.6), copy
// 5.3-5.5 (4.3-5.0).
#include "internal.h"

#define MRHS_API extern "C" __attribute__((visibility("default")))

namespace mrhs {
namespace {

using V4 = unsigned int __attribute__((ext_vector_type(4)));

// This thread's first vector, end and stride.
__device__ __forceinline__ void xcd_range(int64_t n, int64_t &first, int64_t &end, int64_t &stride)
{
    const int g = blockIdx.x % 8, q = blockIdx.x / 8, gx = gridDim.x / 8;
    const int64_t lo = n * g / 8;
    end = n * (g + 1) / 8;
    stride = static_cast<int64_t>(gx) * blockDim.x;
    first = lo + static_cast<int64_t>(q) * blockDim.x + threadIdx.x;
}

template <bool NT>
__device__ __forceinline__ V4 load16(const V4 *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void store16(V4 *p, V4 v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// XOR of every word read; stored only when it equals a value it cannot be
// expected to take, so the loads stay live without a store per thread.
template <bool NT>
__global__ void __launch_bounds__(256) k_probe_read(const V4 *__restrict__ p, int64_t n, unsigned *sink)
{
    int64_t i, e, stride;
    xcd_range(n, i, e, stride);
    V4 acc = {0u, 0u, 0u, 0u};
    for (; i + 3 * stride < e; i += 4 * stride) {
        const V4 a = load16<NT>(p + i), b = load16<NT>(p + i + stride);
        const V4 c = load16<NT>(p + i + 2 * stride), d = load16<NT>(p + i + 3 * stride);
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < e; i += stride)
        acc ^= load16<NT>(p + i);
    const unsigned x = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (x == 0x9E3779B9u)
        sink[0] = x;
}

template <bool NT>
__global__ void __launch_bounds__(256) k_probe_write(V4 *__restrict__ p, int64_t n)
{
    int64_t i, e, stride;
    xcd_range(n, i, e, stride);
    const V4 v = {static_cast<unsigned>(i), 1u, 2u, 3u};
    for (; i + 3 * stride < e; i += 4 * stride) {
        store16<NT>(p + i, v);
        store16<NT>(p + i + stride, v);
        store16<NT>(p + i + 2 * stride, v);
        store16<NT>(p + i + 3 * stride, v);
    }
    for (; i < e; i += stride)
        store16<NT>(p + i, v);
}

template <bool NT>
__global__ void __launch_bounds__(256) k_probe_copy(const V4 *__restrict__ s, V4 *__restrict__ d, int64_t n)
{
    int64_t i, e, stride;
    xcd_range(n, i, e, stride);
    for (; i + 3 * stride < e; i += 4 * stride) {
        const V4 a = load16<NT>(s + i), b = load16<NT>(s + i + stride);
        const V4 c = load16<NT>(s + i + 2 * stride), f = load16<NT>(s + i + 3 * stride);
        store16<NT>(d + i, a);
        store16<NT>(d + i + stride, b);
        store16<NT>(d + i + 2 * stride, c);
        store16<NT>(d + i + 3 * stride, f);
    }
    for (; i < e; i += stride)
        store16<NT>(d + i, load16<NT>(s + i));
}

} // namespace
} // namespace mrhs

using namespace mrhs;

MRHS_API mrhs_status mrhs_stream_probe(int32_t kind, const void *src, void *dst, size_t bytes, void *hip_stream)
{
    clear_error();
    if (kind < MRHS_PROBE_READ || kind > MRHS_PROBE_COPY_NT)
        return set_error(MRHS_EINVAL, "unknown probe kind %d", kind);
    if (bytes == 0 || bytes % 16 != 0)
        return set_error(MRHS_EINVAL, "bytes = %zu must be a positive multiple of 16", bytes);
    const bool reads = kind != MRHS_PROBE_WRITE && kind != MRHS_PROBE_WRITE_NT;
    const bool writes = kind != MRHS_PROBE_READ && kind != MRHS_PROBE_READ_NT;
    if ((reads && !src) || !dst)
        return set_error(MRHS_EINVAL, "NULL buffer");
    if ((reinterpret_cast<uintptr_t>(src) & 15u) || (reinterpret_cast<uintptr_t>(dst) & 15u))
        return set_error(MRHS_EINVAL, "buffers must be 16-byte aligned");
    if (reads && writes) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        if (a < b + bytes && b < a + bytes)
            return set_error(MRHS_EINVAL, "source and destination overlap");
    }
    const int64_t n = static_cast<int64_t>(bytes / 16);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const int grid = cus * 16 / 8 * 8;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const V4 *in = static_cast<const V4 *>(src);
    V4 *out = static_cast<V4 *>(dst);
    switch (kind) {
    case MRHS_PROBE_READ:
        hipLaunchKernelGGL(k_probe_read<false>, dim3(grid), dim3(256), 0, s, in, n, static_cast<unsigned *>(dst));
        break;
    case MRHS_PROBE_READ_NT:
        hipLaunchKernelGGL(k_probe_read<true>, dim3(grid), dim3(256), 0, s, in, n, static_cast<unsigned *>(dst));
        break;
    case MRHS_PROBE_WRITE:
        hipLaunchKernelGGL(k_probe_write<false>, dim3(grid), dim3(256), 0, s, out, n);
        break;
    case MRHS_PROBE_WRITE_NT:
        hipLaunchKernelGGL(k_probe_write<true>, dim3(grid), dim3(256), 0, s, out, n);
        break;
    case MRHS_PROBE_COPY:
        hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(256), 0, s, in, out, n);
        break;
    default:
        hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(256), 0, s, in, out, n);
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MRHS_EDEVICE, "probe launch failed: %s", hipGetErrorString(e));
    return MRHS_OK;
}
