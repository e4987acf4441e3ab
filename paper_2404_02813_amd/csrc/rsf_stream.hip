// Streaming kernel with a pass's read/write mix, for the achievable HBM
// bandwidth the passes are compared against: n_read float fields are read
// and n_write fields written, each of n floats, out_j[i] = j + sum_k in_k[i].
// Every thread keeps four 16-byte vectors per read field in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "rsf.h"
#include "rsf_internal.hpp"

namespace rsf {

namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;

// One span of kStreamUnroll vectors per thread; GUARD only for the last,
// partial span (a load under a per-lane branch is waited for at once, so
// the whole spans carry no condition and keep all their loads in flight).
template <int NR, int NW, bool GUARD>
__device__ __forceinline__ void stream_span(const float4 *in, float4 *out, int64_t n4,
                                            int64_t base)
{
    float4 v[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kStreamThreads;
            if (!GUARD || i < n4) {
                const float4 a = in[(int64_t)k * n4 + i];
                v[u].x += a.x; v[u].y += a.y; v[u].z += a.z; v[u].w += a.w;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) {
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kStreamThreads;
            if (!GUARD || i < n4) {
                const float o = (float)j;
                out[(int64_t)j * n4 + i] =
                    make_float4(v[u].x + o, v[u].y + o, v[u].z + o, v[u].w + o);
            }
        }
    }
}

template <int NR, int NW>
__global__ __launch_bounds__(kStreamThreads) void stream_kernel(const float4 *in, float4 *out,
                                                                int64_t n4)
{
    constexpr int64_t kBlockSpan = (int64_t)kStreamThreads * kStreamUnroll;
    const int64_t step = (int64_t)gridDim.x * kBlockSpan;
    int64_t b0 = (int64_t)blockIdx.x * kBlockSpan;
    for (; b0 + kBlockSpan <= n4; b0 += step)
        stream_span<NR, NW, false>(in, out, n4, b0 + threadIdx.x);
    if (b0 < n4) stream_span<NR, NW, true>(in, out, n4, b0 + threadIdx.x);
}

template <int NR, int NW>
hipError_t launch_stream_t(const float4 *in, float4 *out, int64_t n4, unsigned blocks,
                           hipStream_t s)
{
    hipLaunchKernelGGL((stream_kernel<NR, NW>), dim3(blocks), dim3(kStreamThreads), 0, s, in, out,
                       n4);
    return hipGetLastError();
}

template <int NR>
hipError_t launch_stream_r(int nw, const float4 *in, float4 *out, int64_t n4, unsigned blocks,
                           hipStream_t s)
{
    switch (nw) {
    case 1: return launch_stream_t<NR, 1>(in, out, n4, blocks, s);
    case 2: return launch_stream_t<NR, 2>(in, out, n4, blocks, s);
    case 3: return launch_stream_t<NR, 3>(in, out, n4, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace rsf

extern "C" rsf_status rsf_stream_probe(const float *in, int n_read, float *out, int n_write,
                                       int64_t n, void *stream)
{
    if (!in || !out || n_read < 1 || n_read > 4 || n_write < 1 || n_write > 3 || n <= 0 ||
        n % 4 != 0 || (reinterpret_cast<uintptr_t>(in) % 16) != 0 ||
        (reinterpret_cast<uintptr_t>(out) % 16) != 0)
        return RSF_ERR_INVALID_ARG;
    const auto *in4 = reinterpret_cast<const float4 *>(in);
    auto *out4 = reinterpret_cast<float4 *>(out);
    const int64_t n4 = n / 4;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return RSF_ERR_DEVICE;
    // enough resident workgroups to keep every CU streaming, no more than
    // the work needs
    const int64_t per_block = (int64_t)rsf::kStreamThreads * rsf::kStreamUnroll;
    const int64_t want = (n4 + per_block - 1) / per_block;
    const unsigned blocks = (unsigned)std::min<int64_t>(want, (int64_t)cus * 8);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipErrorInvalidValue;
    switch (n_read) {
    case 1: e = rsf::launch_stream_r<1>(n_write, in4, out4, n4, blocks, s); break;
    case 2: e = rsf::launch_stream_r<2>(n_write, in4, out4, n4, blocks, s); break;
    case 3: e = rsf::launch_stream_r<3>(n_write, in4, out4, n4, blocks, s); break;
    case 4: e = rsf::launch_stream_r<4>(n_write, in4, out4, n4, blocks, s); break;
    }
    return e == hipSuccess ? RSF_OK : RSF_ERR_DEVICE;
}
