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
// passes (LDS tile with an R halo, x then y), so every global access is
// coalesced along x.  Stage 1 runs z first, so H_eps is evaluated once per
// voxel; stage 2 runs z last, so the update sees the z window it needs.
// Workgroups are handed to tiles so that each of the 8 XCDs works on one
// contiguous range of tiles, keeping halo re-reads within one L2.
#include "rsf_internal.hpp"

namespace rsf {

namespace {

// ---------------------------------------------------------------------------
// Tables and flags
// ---------------------------------------------------------------------------

// K * 1 = cx[x] cy[y] cz[z]: partial sums of the taps that land inside.
__global__ __launch_bounds__(kThreads) void edges_kernel(float *cx, float *cy, float *cz,
                                                         Grid3 g, Taps t, int R)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    int n, p;
    float *dst;
    if (i < g.nx) { n = g.nx; p = i; dst = cx; }
    else if (i < g.nx + g.ny) { n = g.ny; p = i - g.nx; dst = cy; }
    else if (i < g.nx + g.ny + g.nz) { n = g.nz; p = i - g.nx - g.ny; dst = cz; }
    else return;
    float acc = 0.f;
    for (int k = -R; k <= R; ++k)
        if (p + k >= 0 && p + k < n) acc += t.w[k + R];
    dst[p] = acc;
}

// flags[0] = early-stop flag, flags[1] = iterations run.
__global__ void flags_init_kernel(int *flags)
{
    if (threadIdx.x < 2) flags[threadIdx.x] = 0;
}

// Fixed-order FP64 sum of the per-block partials; sets the early-stop flag.
__global__ __launch_bounds__(kThreads) void reduce_kernel(const double *__restrict__ partials,
                                                          int64_t n, double *__restrict__ out,
                                                          int *__restrict__ flags,
                                                          double tol_total)
{
    if (flags[0]) return;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) acc += partials[i];
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = sh[0];
        flags[1] += 1;
        if (tol_total > 0.0 && sh[0] < tol_total) flags[0] = 1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Split n into the fewest chunks giving at least `want` blocks over `cols`
// columns, each chunk at least `least` long; every chunk is non-empty.
static int chunks(int64_t n, int64_t cols, int64_t want_blocks, int64_t least)
{
    int64_t want = (want_blocks + cols - 1) / cols;
    const int64_t most = (n + least - 1) / least;
    if (want > most) want = most;
    if (want < 1) want = 1;
    const int64_t len = (n + want - 1) / want;
    return (int)((n + len - 1) / len);
}

int z_chunks(const Grid3 &g)
{
    const int64_t cols = (int64_t)((g.nx + kZx - 1) / kZx) * ((g.ny + kZy - 1) / kZy);
    return chunks(g.nz, cols, 2048, 8);
}

int64_t z_blocks(const Grid3 &g)
{
    return (int64_t)((g.nx + kZx - 1) / kZx) * ((g.ny + kZy - 1) / kZy) * z_chunks(g);
}

int u_chunks(const Grid3 &g)
{
    const int64_t cols = (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy);
    return chunks(g.nz, cols, 1024, 8);
}

int64_t u_blocks(const Grid3 &g)
{
    return (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy) * u_chunks(g);
}

// xy pass: one wave per (64-wide strip, row chunk, slice); rows per chunk
// >= 8, enough chunks for ~16K waves, no more than needed for 128-row chunks.
int xy_chunks(const Grid3 &g)
{
    const int64_t strips = (g.nx + 63) / 64;
    const int64_t base = (g.ny + 127) / 128;
    int64_t c = chunks(g.ny, strips * g.nz, 16384, 8);
    if (c < base) c = base;
    const int64_t len = (g.ny + c - 1) / c;
    return (int)((g.ny + len - 1) / len);
}

int xy_blocks(const Grid3 &g) { return (int)(((g.nx + 63) / 64) * xy_chunks(g) * g.nz); }

hipError_t launch_edges(float *cx, float *cy, float *cz, Grid3 g, const Taps &t, int R,
                        hipStream_t s)
{
    const int n = g.nx + g.ny + g.nz;
    hipLaunchKernelGGL(edges_kernel, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       cx, cy, cz, g, t, R);
    return hipGetLastError();
}

hipError_t launch_flags_init(int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(flags_init_kernel, dim3(1), dim3(64), 0, s, flags);
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

// Expand F(RR, IT, ST) for every built (radius, image, storage) combination
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

hipError_t launch_xy(int R, int mode, int it, int st, const void *in, void *out, Grid3 g,
                     const Taps &t, const FitArgs *fa, const int *done, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_xy_r<RR, IT, ST>(mode, in, out, g, t, fa, done, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_plain(int R, int st, const void *in, void *out, Grid3 g, const Taps &t,
                          hipStream_t s)
{
    const int it = F32;   // the plain z pass only touches the storage type
#define C(RR, IT, ST) \
    case RR: return launch_z_plain_r<RR, ST>(in, out, g, t, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_heaviside(int R, int it, int st, const float *phi, const void *I,
                              void *pair_out, Grid3 g, const Taps &t, float eps, float *probeH,
                              const int *done, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_z_heaviside_r<RR, IT, ST>(phi, I, pair_out, g, t, eps, probeH, done, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_z_update(int R, int it, int st, const void *pair_in, Grid3 g, const Taps &t,
                           const UpdArgs &ua, const int *done, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_z_update_r<RR, IT, ST>(pair_in, g, t, ua, done, s);
    RSF_DISPATCH(C)
#undef C
}

hipError_t launch_reduce(const double *partials, int64_t n, double *out, int *flags,
                         double tol_total, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, n, out, flags,
                       tol_total);
    return hipGetLastError();
}

}  // namespace rsf
