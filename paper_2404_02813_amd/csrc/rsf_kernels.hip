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

// The tile table of a batch from the kernel argument (one workgroup).
__global__ __launch_bounds__(kThreads) void put_table_kernel(uint32_t *dst, TableBlob blob,
                                                             int words)
{
    for (int i = threadIdx.x; i < words; i += kThreads) dst[i] = blob.w[i];
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

// ---------------------------------------------------------------------------
// Initialisation (Sec. 4.3): determinant-of-Hessian seeds, fast sweeping
// ---------------------------------------------------------------------------

template <class IT>
__global__ __launch_bounds__(kThreads) void smooth_x_kernel(const IT *img, float *out, int64_t nx,
                                                            int64_t n, Taps t, int R)
{
    const gptr<const IT> in = glb(img);
    const gptr<float> o = glb(out);
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t x = i % nx, row = i - x;
        float acc = 0.f;
        for (int k = -R; k <= R; ++k) {
            const int64_t xx = x + k;
            if (xx >= 0 && xx < nx) acc = fmaf(t.w[k + R], to_f(in[row + xx]), acc);
        }
        o[i] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void smooth_y_kernel(const float *src, float *out,
                                                            int64_t nx, int64_t ny, int64_t n,
                                                            Taps t, int R)
{
    const gptr<const float> in = glb(src);
    const gptr<float> o = glb(out);
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t yz = i / nx;
        const int64_t y = yz % ny, base = i - y * nx;   // (z, 0, x)
        float acc = 0.f;
        for (int k = -R; k <= R; ++k) {
            const int64_t yy = y + k;
            if (yy >= 0 && yy < ny) acc = fmaf(t.w[k + R], in[base + yy * nx], acc);
        }
        o[i] = acc;
    }
}

__device__ __forceinline__ int64_t refl(int64_t i, int64_t n)
{
    return i < 0 ? -i : (i > n - 1 ? 2 * (n - 1) - i : i);
}

__global__ __launch_bounds__(kThreads) void hessian_kernel(const float *Lp, float *doh, float *tr,
                                                           float *part, int64_t nx, int64_t ny,
                                                           int64_t n)
{
    const gptr<const float> L = glb(Lp);
    __shared__ float sm[kThreads];
    float best = -kFar;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t x = i % nx, yz = i / nx;
        const int64_t y = yz % ny, base = i - x - y * nx;
        auto at = [&](int64_t xx, int64_t yy) { return L[base + refl(yy, ny) * nx + refl(xx, nx)]; };
        const float c = at(x, y);
        const float lxx = at(x + 1, y) - 2.f * c + at(x - 1, y);
        const float lyy = at(x, y + 1) - 2.f * c + at(x, y - 1);
        const float lxy = (at(x + 1, y + 1) - at(x + 1, y - 1) - at(x - 1, y + 1) +
                           at(x - 1, y - 1)) * 0.25f;
        const float d = lxx * lyy - lxy * lxy;
        glb(doh)[i] = d;
        glb(tr)[i] = lxx + lyy;
        best = fmaxf(best, d);
    }
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) glb(part)[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kThreads) void max_kernel(const float *part, int n, float *out)
{
    __shared__ float sm[kThreads];
    float best = -kFar;
    for (int i = threadIdx.x; i < n; i += kThreads) best = fmaxf(best, glb(part)[i]);
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) glb(out)[0] = sm[0];
}

// A seed is a bright blob (trace < 0) whose determinant exceeds threshold x
// the volume's largest and is a local maximum of its 3x3 in-slice
// neighbourhood: strictly above the neighbours earlier in raster order, at
// least the later ones (so a plateau gives one seed).
__global__ __launch_bounds__(kThreads) void seeds_kernel(const float *dohp, const float *trp,
                                                         const float *maxv, float threshold,
                                                         unsigned char *mask, float *u,
                                                         unsigned *cnt, int64_t nx, int64_t ny,
                                                         int64_t n)
{
    const gptr<const float> doh = glb(dohp);
    __shared__ unsigned sc[kThreads];
    unsigned mine = 0;
    const float thr = threshold * glb(maxv)[0];
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t x = i % nx, yz = i / nx;
        const int64_t y = yz % ny, base = i - x - y * nx;
        const float d = doh[i];
        bool seed = d > thr && glb(trp)[i] < 0.f;
        for (int dy = -1; dy <= 1 && seed; ++dy)
            for (int dx = -1; dx <= 1 && seed; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const int64_t xx = x + dx, yy = y + dy;
                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
                const float nb = doh[base + yy * nx + xx];
                const bool earlier = dy < 0 || (dy == 0 && dx < 0);
                seed = earlier ? d > nb : d >= nb;
            }
        glb(mask)[i] = seed ? 1 : 0;
        glb(u)[i] = seed ? 0.f : kFar;
        mine += seed ? 1u : 0u;
    }
    sc[threadIdx.x] = mine;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sc[threadIdx.x] += sc[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) glb(cnt)[blockIdx.x] = sc[0];
}

// Godunov update of |grad u| = 1 on the unit grid from the smallest
// neighbour value along each axis (a, b, c; kFar when absent).  The roots
// are written in the differences d1 = b - a, d2 = c - a, which are O(1)
// where they are used: the textbook discriminant (a+b+c)^2 - 3(a^2+b^2+c^2-1)
// cancels to O(1) from O(u^2) terms and loses most FP32 digits at large u.
__device__ __forceinline__ float godunov(float a, float b, float c)
{
    float t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    if (a + 1.f <= b) return a + 1.f;
    const float d1 = b - a;
    const float r2 = 0.5f * (d1 + sqrtf(2.f - d1 * d1));
    if (a + r2 <= c) return a + r2;
    const float d2 = c - a, d3 = d2 - d1;
    return a + (d1 + d2 + sqrtf(3.f - (d1 * d1 + d2 * d2 + d3 * d3))) * (1.f / 3.f);
}

// One hyperplane of blocks of a sweep.  In the sweep's orientation
// (i' = i or nx-1-i by its x order, likewise j', k') the volume is cut into
// blocks of kSbx x kSby x kSbz; the blocks with bi' + bj' + bk' = H are
// independent: a block's upwind neighbours (i'-1, j'-1, k'-1 across a face)
// lie in blocks of hyperplane H-1, already swept, and its downwind ones in
// hyperplane H+1, not yet.  One wave loads its block with a one-voxel face
// halo into LDS (absent points as kFar), marches the block's own inner
// hyperplanes in order (lane = one (j', k') line) and writes the block back.
// Every point is thus updated after its upwind neighbours and before its
// downwind ones, which gives exactly the sequential Gauss-Seidel sweep.
// Workgroup g covers bj' = g % nby, bk' = kblo + g / nby.
constexpr int kSbx = 32, kSby = 8, kSbz = 8;
static_assert(kSby * kSbz == 64, "one lane per (j', k') line of a block");
__global__ __launch_bounds__(64) void sweep_block_kernel(float *up, int64_t nx, int64_t ny,
                                                         int64_t nz, int dir, int64_t H,
                                                         int64_t nbx, int64_t nby, int64_t kblo)
{
    constexpr int TX = kSbx + 2, TY = kSby + 2, TZ = kSbz + 2;
    __shared__ float tile[TZ][TY][TX];
    const int64_t gb = blockIdx.x;
    const int64_t bj = gb % nby, bk = kblo + gb / nby;
    const int64_t bi = H - bj - bk;
    if (bi < 0 || bi >= nbx) return;   // the whole workgroup
    const gptr<float> u = glb(up);
    const int lane = threadIdx.x;
    const int64_t i0 = bi * kSbx, j0 = bj * kSby, k0 = bk * kSbz;   // oriented origin
    // global index of oriented point (ip, jp, kp), all inside the volume
    auto gidx = [&](int64_t ip, int64_t jp, int64_t kp) {
        const int64_t i = (dir & 1) ? nx - 1 - ip : ip;
        const int64_t j = (dir & 2) ? ny - 1 - jp : jp;
        const int64_t k = (dir & 4) ? nz - 1 - kp : kp;
        return (k * ny + j) * nx + i;
    };
    // all loads issued before any is used (clamped into the volume, so none
    // sits under a branch), then staged with the absent points set to kFar
    constexpr int NL = (TX * TY * TZ + 63) / 64;
    float v[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int c = min(lane + 64 * r, TX * TY * TZ - 1);
        const int lx = c % TX, ly = (c / TX) % TY, lz = c / (TX * TY);
        const int64_t ip = min(max(i0 - 1 + lx, (int64_t)0), nx - 1);
        const int64_t jp = min(max(j0 - 1 + ly, (int64_t)0), ny - 1);
        const int64_t kp = min(max(k0 - 1 + lz, (int64_t)0), nz - 1);
        v[r] = u[gidx(ip, jp, kp)];
    }
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int c = lane + 64 * r;
        if (c < TX * TY * TZ) {
            const int lx = c % TX, ly = (c / TX) % TY, lz = c / (TX * TY);
            const int64_t ip = i0 - 1 + lx, jp = j0 - 1 + ly, kp = k0 - 1 + lz;
            const bool in = ip >= 0 && ip < nx && jp >= 0 && jp < ny && kp >= 0 && kp < nz;
            (&tile[0][0][0])[c] = in ? v[r] : kFar;
        }
    }
    __syncwarp();
    const int ly = 1 + lane % kSby, lz = 1 + lane / kSby;
    const bool line_in = j0 + ly - 1 < ny && k0 + lz - 1 < nz;
    for (int s = 0; s < kSbx + kSby + kSbz - 2; ++s) {
        const int lx = 1 + s - (ly - 1) - (lz - 1);
        if (line_in && lx >= 1 && lx <= kSbx && i0 + lx - 1 < nx) {
            const float a = fminf(tile[lz][ly][lx - 1], tile[lz][ly][lx + 1]);
            const float b = fminf(tile[lz][ly - 1][lx], tile[lz][ly + 1][lx]);
            const float c = fminf(tile[lz - 1][ly][lx], tile[lz + 1][ly][lx]);
            if (!(a >= kFar && b >= kFar && c >= kFar)) {
                const float v = godunov(a, b, c);
                if (v < tile[lz][ly][lx]) tile[lz][ly][lx] = v;
            }
        }
        __syncwarp();
    }
    for (int c = lane; c < kSbx * kSby * kSbz; c += 64) {
        const int lx = c % kSbx, ly2 = (c / kSbx) % kSby, lz2 = c / (kSbx * kSby);
        const int64_t ip = i0 + lx, jp = j0 + ly2, kp = k0 + lz2;
        if (ip < nx && jp < ny && kp < nz) u[gidx(ip, jp, kp)] = tile[lz2 + 1][ly2 + 1][lx + 1];
    }
}

__global__ __launch_bounds__(kThreads) void offset_kernel(const float *u, float *phi, int64_t n,
                                                          float offset)
{
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        glb(phi)[i] = offset - glb(u)[i];
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

// dtype codes as in rsf.h
constexpr int F32 = 0, F16 = 1, BF16 = 2, U16 = 3;

hipError_t launch_smooth_x(const void *img, int image_dtype, float *out, int64_t nx, int64_t ny,
                           int64_t nz, const Taps &t, int R, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    if (image_dtype == U16)
        hipLaunchKernelGGL(smooth_x_kernel<uint16_t>, dim3(stride_grid(n)), dim3(kThreads), 0, s,
                           static_cast<const uint16_t *>(img), out, nx, n, t, R);
    else
        hipLaunchKernelGGL(smooth_x_kernel<float>, dim3(stride_grid(n)), dim3(kThreads), 0, s,
                           static_cast<const float *>(img), out, nx, n, t, R);
    return hipGetLastError();
}

hipError_t launch_smooth_y(const float *in, float *out, int64_t nx, int64_t ny, int64_t nz,
                           const Taps &t, int R, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    hipLaunchKernelGGL(smooth_y_kernel, dim3(stride_grid(n)), dim3(kThreads), 0, s, in, out, nx, ny,
                       n, t, R);
    return hipGetLastError();
}

hipError_t launch_hessian(const float *L, float *doh, float *tr, float *part, int64_t nx,
                          int64_t ny, int64_t nz, int *blocks, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    const unsigned g = stride_grid(n);
    *blocks = (int)g;
    hipLaunchKernelGGL(hessian_kernel, dim3(g), dim3(kThreads), 0, s, L, doh, tr, part, nx, ny, n);
    return hipGetLastError();
}

hipError_t launch_max(const float *part, int n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(kThreads), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t launch_seeds(const float *doh, const float *tr, const float *maxv, float threshold,
                        unsigned char *mask, float *u, unsigned *cnt, int64_t nx, int64_t ny,
                        int64_t nz, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    hipLaunchKernelGGL(seeds_kernel, dim3(stride_grid(n)), dim3(kThreads), 0, s, doh, tr, maxv,
                       threshold, mask, u, cnt, nx, ny, n);
    return hipGetLastError();
}

int64_t sweep_block_planes(int64_t nx, int64_t ny, int64_t nz)
{
    return (nx + kSbx - 1) / kSbx + (ny + kSby - 1) / kSby + (nz + kSbz - 1) / kSbz - 2;
}

hipError_t launch_sweep_blocks(float *u, int64_t nx, int64_t ny, int64_t nz, int dir, int64_t H,
                               hipStream_t s)
{
    const int64_t nbx = (nx + kSbx - 1) / kSbx, nby = (ny + kSby - 1) / kSby,
                  nbz = (nz + kSbz - 1) / kSbz;
    // bk' runs over the values for which some (bi', bj') completes the plane
    const int64_t klo = std::max<int64_t>(0, H - (nbx - 1) - (nby - 1));
    const int64_t khi = std::min<int64_t>(nbz - 1, H);
    if (khi < klo) return hipSuccess;
    const int64_t g = nby * (khi - klo + 1);
    hipLaunchKernelGGL(sweep_block_kernel, dim3((unsigned)g), dim3(64), 0, s, u, nx, ny, nz, dir,
                       H, nbx, nby, klo);
    return hipGetLastError();
}

hipError_t launch_offset(const float *u, float *phi, int64_t n, float offset, hipStream_t s)
{
    hipLaunchKernelGGL(offset_kernel, dim3(stride_grid(n)), dim3(kThreads), 0, s, u, phi, n, offset);
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

hipError_t launch_put_table(void *dst, const TableBlob &blob, int bytes, hipStream_t s)
{
    if (bytes < 0 || bytes > kTableBlobBytes || bytes % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(put_table_kernel, dim3(1), dim3(kThreads), 0, s,
                       static_cast<uint32_t *>(dst), blob, bytes / 4);
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

hipError_t launch_z_update_fused(int R, int it, int st, const Batch &b, int64_t blocks,
                                 const Taps &t, const Coeffs &c, bool paper, hipStream_t s)
{
#define C(RR, IT, ST) \
    case RR: return launch_z_update_fused_r<RR, IT, ST>(b, blocks, t, c, paper, s);
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
