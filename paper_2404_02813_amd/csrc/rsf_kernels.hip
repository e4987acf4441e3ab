// HIP kernels (gfx950) of one RSF level-set iteration.
//
// One iteration = four bandwidth-bound passes plus a tiny reduction:
//   z(H)     : (phi, I) -> Kz*(H I), Kz*H           H = H_eps(phi)      (Sec. 3)
//   xy(fits) : -> A1 = K*(H I), B1 = K*H, with A2 = K*I - A1, B2 = K*1 - B1
//              f1 = A1/B1, f2 = A2/B2, g1 = l1 f1 - l2 f2,
//              g2 = l1 f1^2 - l2 f2^2                                    (Sec. 3)
//   xy(two)  : (g1, g2) -> Kxy*g1, Kxy*g2
//   z(upd)   : Fd = (l1-l2) I^2 K*1 - 2 I K*g1 + K*g2 = l1 e1 - l2 e2,
//              curvature, regulariser, Dirac-weighted explicit update   (Sec. 2-3)
//              and per-block FP64 partial sums of |phi' - phi|
//   reduce   : fixed-order FP64 sum of the partials.
// The separable Gaussian is applied as z passes (each thread marches one
// (x, y) column through a z chunk with a register ring of 2R+1 slices) and xy
// passes (a wave marches a 64-wide strip down a row chunk: rows staged in LDS
// and x-convolved, a register ring of 2R+1 rows for y), so every global
// access is coalesced along x.  Stage 1 runs z first, so H_eps is evaluated
// once per voxel; stage 2 runs z last, so the update sees the z window it
// needs.  Every pass is one launch over a batch of tiles; workgroups are
// numbered so that each of the 8 XCDs works on one contiguous range, keeping
// halo re-reads within one L2.
#include <algorithm>
#include <cmath>

#include "rsf_device.hpp"

namespace rsf {

namespace {

// ---------------------------------------------------------------------------
// Per-tile set-up and reduction (one workgroup per tile)
// ---------------------------------------------------------------------------

// K * 1 = cx[x] cy[y] cz[z]: partial sums of the taps that land inside; the
// tile's flags cleared.
__global__ __launch_bounds__(kThreads) void setup_kernel(Batch bt, Taps t, int R)
{
    const TileDesc &d = bt.tiles[blockIdx.x];
    const Grid3 g = d.g;
    if (threadIdx.x < 2) d.flags[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < g.nx + g.ny + g.nz; i += kThreads) {
        int n, p;
        float *dst;
        if (i < g.nx) { n = g.nx; p = i; dst = d.cx; }
        else if (i < g.nx + g.ny) { n = g.ny; p = i - g.nx; dst = d.cy; }
        else { n = g.nz; p = i - g.nx - g.ny; dst = d.cz; }
        float acc = 0.f;
        for (int k = -R; k <= R; ++k)
            if (p + k >= 0 && p + k < n) acc += t.w[k + R];
        dst[p] = acc;
    }
}

// Fixed-order FP64 sum of one tile's update-pass partials into hist[iters
// run]; sets the tile's stop flag when the tolerance is met.
__global__ __launch_bounds__(kThreads) void reduce_kernel(Batch bt, Coeffs c)
{
    const TileDesc &d = bt.tiles[blockIdx.x];
    if (d.flags[0]) return;
    const int64_t n = u_blocks(d.g, d.sp);
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) acc += d.partials[i];
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int k = d.flags[1];
        if (k < d.hist_cap) d.hist[k] = sh[0];
        *reinterpret_cast<double *>(d.flags + 2) = sh[0];   // last sum, 8-byte aligned
        d.flags[1] = k + 1;
        const double voxels = (double)d.g.nx * d.g.ny * d.g.nz;
        if (c.tol > 0.0 && sh[0] < c.tol * voxels) d.flags[0] = 1;
        else if (k + 1 >= d.hist_cap) d.flags[0] = 2;   // all its iterations done
    }
}

// After the last iteration: a tile whose final iterate n is odd has it in the
// workspace buffer phi[1]; copy it to the caller's phi[0].  Workgroups as in
// the stage-1 z pass.
__global__ __launch_bounds__(kThreads) void finish_kernel(Batch bt)
{
    Where wh;
    if (!locate(bt, wh)) return;
    const TileDesc &d = bt.tiles[wh.t];
    if (!(glb(d.flags)[1] & 1)) return;
    const Grid3 g = d.g;
    const ZCols zt = z_cols(g, d.sp.z, wh.lb);
    if (!zt.active) return;
    const int col = zt.col;
    const gptr<const float> src = glb(d.phi[1]);
    const gptr<float> dst = glb(d.phi[0]);
    for (int z = zt.z0; z < zt.z1; ++z) (dst + (int64_t)z * g.sxy)[col] = (src + (int64_t)z * g.sxy)[col];
}

// ---------------------------------------------------------------------------
// Volume-level driver: gather a sub-volume, merge it back (Sec. 4.1)
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(kThreads) void gather_kernel(const T *src, T *dst, int64_t nx,
                                                          int64_t ny, SubBox b)
{
    const int64_t n = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    const gptr<const T> s = glb(src);
    const gptr<T> d = glb(dst);
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t x = i % b.ext[0], yz = i / b.ext[0];
        const int64_t y = yz % b.ext[1], z = yz / b.ext[1];
        d[i] = s[((z + b.lo[2]) * ny + (y + b.lo[1])) * nx + (x + b.lo[0])];
    }
}

// Weight of a box at volume coordinate c along one axis: 1 inside its core,
// a linear ramp across the 2C voxels straddling each core face it shares
// with a neighbour (the neighbour's ramp is its complement, so the weights
// of all boxes sum to one).
__device__ __forceinline__ float ramp(int c, int core_lo, int core_hi, int nb_lo, int nb_hi, int C)
{
    const float inv = 1.f / (2.f * (float)C);
    if (nb_lo && c < core_lo + C) return ((float)(c - (core_lo - C)) + 0.5f) * inv;
    if (nb_hi && c >= core_hi - C) return ((float)((core_hi + C) - c) - 0.5f) * inv;
    return 1.f;
}

__global__ __launch_bounds__(kThreads) void merge_kernel(float *acc, const float *tile, int64_t nx,
                                                         int64_t ny, SubBox b, int C)
{
    const int64_t n = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    const gptr<float> a = glb(acc);
    const gptr<const float> t = glb(tile);
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int x = (int)(i % b.ext[0]);
        const int64_t yz = i / b.ext[0];
        const int y = (int)(yz % b.ext[1]), z = (int)(yz / b.ext[1]);
        const int gx = x + b.lo[0], gy = y + b.lo[1], gz = z + b.lo[2];
        const float w = ramp(gx, b.core_lo[0], b.core_hi[0], b.nb_lo[0], b.nb_hi[0], C) *
                        ramp(gy, b.core_lo[1], b.core_hi[1], b.nb_lo[1], b.nb_hi[1], C) *
                        ramp(gz, b.core_lo[2], b.core_hi[2], b.nb_lo[2], b.nb_hi[2], C);
        a[((int64_t)gz * ny + gy) * nx + gx] += w * t[i];
    }
}

__global__ __launch_bounds__(kThreads) void fill_kernel(float *dst, int64_t n, float v)
{
    const gptr<float> d = glb(dst);
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        d[i] = v;
}

unsigned stride_grid(int64_t n)
{
    const int64_t g = (n + kThreads - 1) / kThreads;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_gather(const void *src, void *dst, int elem_bytes, int64_t nx, int64_t ny,
                         const SubBox &b, hipStream_t s)
{
    const int64_t n = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    if (elem_bytes == 4)
        hipLaunchKernelGGL(gather_kernel<float>, dim3(stride_grid(n)), dim3(kThreads), 0, s,
                           static_cast<const float *>(src), static_cast<float *>(dst), nx, ny, b);
    else if (elem_bytes == 2)
        hipLaunchKernelGGL(gather_kernel<uint16_t>, dim3(stride_grid(n)), dim3(kThreads), 0, s,
                           static_cast<const uint16_t *>(src), static_cast<uint16_t *>(dst), nx, ny,
                           b);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_merge(float *acc, const float *tile, int64_t nx, int64_t ny, const SubBox &b,
                        int curtain, hipStream_t s)
{
    const int64_t n = (int64_t)b.ext[0] * b.ext[1] * b.ext[2];
    hipLaunchKernelGGL(merge_kernel, dim3(stride_grid(n)), dim3(kThreads), 0, s, acc, tile, nx, ny,
                       b, curtain);
    return hipGetLastError();
}

hipError_t launch_fill(float *dst, int64_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(stride_grid(n)), dim3(kThreads), 0, s, dst, n, v);
    return hipGetLastError();
}

hipError_t launch_setup(const Batch &b, const Taps &t, int R, hipStream_t s)
{
    hipLaunchKernelGGL(setup_kernel, dim3(b.n), dim3(kThreads), 0, s, b, t, R);
    return hipGetLastError();
}

hipError_t launch_reduce(const Batch &b, const Coeffs &c, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(b.n), dim3(kThreads), 0, s, b, c);
    return hipGetLastError();
}

hipError_t launch_finish(const Batch &b, int64_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL(finish_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// dtype codes as in rsf.h
constexpr int F32 = 0, F16 = 1, BF16 = 2, U16 = 3;

bool types_supported(int R, int it, int st)
{
    if (R < 1 || R > kMaxR) return false;
    if (it == F32 && st == F32) return true;
    if (R < kMinRMixed || R > kMaxRMixed) return false;
    return (it == F32 || it == U16) && (st == F32 || st == F16 || st == BF16);
}

// Expand CALL(RR, IT, ST) for the built (radius, image, storage) combination
// matching the runtime (R, it, st).
#define RSF_R_ALL(X, IT, ST) \
    X(1, IT, ST) X(2, IT, ST) X(3, IT, ST) X(4, IT, ST) X(5, IT, ST) X(6, IT, ST) X(7, IT, ST) \
    X(8, IT, ST) X(9, IT, ST) X(10, IT, ST) X(11, IT, ST) X(12, IT, ST) X(13, IT, ST)          \
    X(14, IT, ST) X(15, IT, ST) X(16, IT, ST)
#define RSF_R_MIXED(X, IT, ST) \
    X(4, IT, ST) X(5, IT, ST) X(6, IT, ST) X(7, IT, ST) X(8, IT, ST) X(9, IT, ST) X(10, IT, ST) \
    X(11, IT, ST) X(12, IT, ST)
#define RSF_DISPATCH(CALL)                                                              \
    if (!types_supported(R, it, st)) return hipErrorInvalidValue;                       \
    if (it == F32 && st == F32) {                                                       \
        switch (R) { RSF_R_ALL(CALL, float, float) default: break; }                     \
    } else if (it == U16 && st == F16) {                                                \
        switch (R) { RSF_R_MIXED(CALL, uint16_t, _Float16) default: break; }             \
    } else if (it == U16 && st == BF16) {                                               \
        switch (R) { RSF_R_MIXED(CALL, uint16_t, __bf16) default: break; }               \
    } else if (it == U16 && st == F32) {                                                \
        switch (R) { RSF_R_MIXED(CALL, uint16_t, float) default: break; }                \
    } else if (it == F32 && st == F16) {                                                \
        switch (R) { RSF_R_MIXED(CALL, float, _Float16) default: break; }                \
    } else if (it == F32 && st == BF16) {                                               \
        switch (R) { RSF_R_MIXED(CALL, float, __bf16) default: break; }                  \
    }                                                                                   \
    return hipErrorInvalidValue;

hipError_t launch_xy(int R, int mode, int it, int st, const Batch &b, int64_t blocks,
                     const Taps &t, const Coeffs &c, bool probe, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_xy_r<RR, IT, ST>(mode, b, blocks, t, c, probe, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_plain(int R, int st, const Batch &b, int64_t blocks, const Taps &t,
                          int target, hipStream_t s)
{
    const int it = F32;   // the plain z pass only touches the storage type
#define C(RR, IT, ST) \
    case RR: return launch_z_plain_r<RR, ST>(b, blocks, t, target, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_heaviside(int R, int it, int st, const Batch &b, int64_t blocks,
                              const Taps &t, const Coeffs &c, bool probe, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_z_heaviside_r<RR, IT, ST>(b, blocks, t, c, probe, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_update(int R, int it, int st, const Batch &b, int64_t blocks, const Taps &t,
                           const Coeffs &c, bool probe, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_z_update_r<RR, IT, ST>(b, blocks, t, c, probe, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_update_paper(int it, int st, const Batch &b, int64_t blocks, const Coeffs &c,
                                 bool probe, hipStream_t s)
{
    if (it == F32 && st == F32) return launch_z_update_paper_r<float, float>(b, blocks, c, probe, s);
    if (it == U16 && st == F16) return launch_z_update_paper_r<uint16_t, _Float16>(b, blocks, c, probe, s);
    if (it == U16 && st == BF16) return launch_z_update_paper_r<uint16_t, __bf16>(b, blocks, c, probe, s);
    if (it == U16 && st == F32) return launch_z_update_paper_r<uint16_t, float>(b, blocks, c, probe, s);
    if (it == F32 && st == F16) return launch_z_update_paper_r<float, _Float16>(b, blocks, c, probe, s);
    if (it == F32 && st == BF16) return launch_z_update_paper_r<float, __bf16>(b, blocks, c, probe, s);
    return hipErrorInvalidValue;
}

}  // namespace rsf
