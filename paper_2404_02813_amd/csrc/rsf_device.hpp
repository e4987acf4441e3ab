// Device helpers shared by every kernel: element conversions, the pair
// layout, reflection, the XCD-aware workgroup numbering, the tile lookup of a
// batched launch and the column/z-chunk decomposition of the z passes.
#pragma once

#include "rsf_internal.hpp"

namespace rsf {

namespace {

constexpr float kTwoPi = 6.28318530717958647693f;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// H_eps(phi) = 1/2 (1 + (2/pi) atan(phi/eps)) (Sec. 3, regularised
// Heaviside).  With a = |phi| and t = min(a, eps)/max(a, eps) in [0, 1],
// q = atan(t)/pi = t P(t^2), and
//   a <= eps:    H = 1/2 + sign(phi) q
//   phi < -eps:  H = q        (= atan(eps/|phi|)/pi: full relative precision
//                              as H -> 0, like atan2(eps, -phi)/pi)
//   phi > eps:   H = 1 - q
// P is the degree-8 polynomial of least maximum relative error for
// atan(sqrt(u))/(pi sqrt(u)) on u in [0, 1] (Remez exchange; 1.5e-8, below
// a quarter FP32 ulp), so H is within about 1e-7 of the exact value: as
// accurate as the library atan2f at a third of its instructions, with one
// reciprocal and no range-reduction branches (csrc/atan_poly.py prints the
// coefficients).
__device__ __forceinline__ float heaviside(float phi, float eps)
{
    const float a = fabsf(phi);
    const float t = fminf(a, eps) * rcp(fmaxf(a, eps));
    const float u = t * t;
    float p = 9.071479804014546e-4f;
    p = fmaf(p, u, -5.114803217655306e-3f);
    p = fmaf(p, u, 1.358913226569387e-2f);
    p = fmaf(p, u, -2.3886911108485072e-2f);
    p = fmaf(p, u, 3.387114486444002e-2f);
    p = fmaf(p, u, -4.521160451520202e-2f);
    p = fmaf(p, u, 6.363848403138736e-2f);
    p = fmaf(p, u, -1.0610246782661932e-1f);
    p = fmaf(p, u, 3.183098813345913e-1f);
    const float q = t * p;
    const float inner = 0.5f + copysignf(q, phi);
    const float outer = phi < 0.f ? q : 1.f - q;
    return a <= eps ? inner : outer;
}

// The tile table hands the kernels generic pointers.  Recasting them to the
// global address space lets the compiler use global instead of flat memory
// instructions: flat ones also count against the LDS wait counter, so every
// LDS wait would also wait for the loads prefetched a step ahead.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> glb(T *p)
{
    return (gptr<T>)p;
}

// Tap k of the 2R + 1 Gaussian taps.  The taps are symmetric by
// construction (w[R + k] = w[R - k]), so only w[0..R] are read and R fewer
// scalar registers hold the kernel.
template <int R>
__device__ __forceinline__ float tap(const Taps &t, int k)
{
    return t.w[k <= R ? k : 2 * R - k];
}

// Buffer-resource access.  The wave-uniform 64-bit base of an array (a
// slice, or any array under 4 GiB) lives in a scalar resource descriptor and
// each lane supplies only a 32-bit byte offset, so no 64-bit address
// arithmetic is done per lane and no 64-bit offsets occupy vector registers.
// Planes are limited so that every in-slice offset fits (kMaxPlane).  The
// descriptor has stride 0 (raw), no range limit and the 32-bit data format
// gfx9 raw buffer instructions expect.  Raw elements are converted only where
// they are used: converting right after the load would make the load's
// consumer wait for it there, and a load issued a step ahead would no longer
// overlap anything.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcFlags = 0x00020000;
__device__ __forceinline__ rsrc_t rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, kRsrcFlags);
}
template <class T>
__device__ __forceinline__ rsrc_t rsrc(gptr<T> base)
{
    return rsrc((const void *)base);
}

// Element i of the array behind r (T of 2, 4 or 8 bytes); `soff` is a
// wave-uniform byte offset added to the lane's.
template <class T>
__device__ __forceinline__ T bld(rsrc_t r, uint32_t i, uint32_t soff = 0)
{
    const uint32_t off = i * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 2) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    } else {
        static_assert(sizeof(T) == 8, "2, 4 or 8-byte elements");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    }
}
template <class T>
__device__ __forceinline__ void bst(rsrc_t r, uint32_t i, T v, uint32_t soff = 0)
{
    const uint32_t off = i * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, soff, 0);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, soff, 0);
    } else {
        static_assert(sizeof(T) == 8, "2, 4 or 8-byte elements");
        using U2 = unsigned int __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, soff, 0);
    }
}

// A wave-uniform element of read-only device data (tables written before the
// kernel starts) through the scalar data cache: one scalar load, no vector
// register.
template <class T>
__device__ __forceinline__ T uniform_ld(const T *p, int i)
{
    return ((__attribute__((address_space(4))) const T *)p)[i];
}

// Storage and image element types: fields may be stored as float, FP16 or
// BF16 (arithmetic is always FP32); the image may be float or uint16, the
// latter normalised to [0, 1] as u / 65535 on load.
__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f(__bf16 v) { return (float)v; }
__device__ __forceinline__ float to_f(uint16_t v) { return (float)v * (1.f / 65535.f); }
template <class T>
__device__ __forceinline__ T from_f(float v) { return (T)v; }   // round to nearest even

// The two fields every pass reads or writes together (Kz*(HI) and Kz*H; g1
// and g2; their xy convolutions) are stored interleaved, so one 4-byte (FP16,
// BF16) or 8-byte (FP32) access per lane moves both.
template <class T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};

// Pair element i as one vector access (4 or 8 bytes per lane).
template <class T>
using Vec2 = T __attribute__((ext_vector_type(2)));

// Pair element i of the array behind r, stored through the descriptor.
template <class T>
__device__ __forceinline__ void bst_pair(rsrc_t r, uint32_t i, float a, float b, uint32_t soff = 0)
{
    Vec2<T> v;
    v.x = from_f<T>(a);
    v.y = from_f<T>(b);
    bst<Vec2<T>>(r, i, v, soff);
}

// Value of lane `src` (wave-uniform) of v.  Lanes past a volume edge store
// the last in-volume lane's value to that lane's own element, so that a store
// needs no per-lane guard: a store under a per-lane branch makes the compiler
// wait for every load in flight at the branch's end.
__device__ __forceinline__ float lane_value(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Make `v` opaque to the optimiser: it must be computed here, so a sum that
// feeds a register ring is not sunk to its distant use (which would keep all
// of its inputs live instead of one value).
__device__ __forceinline__ void pin(float &v) { __asm__ volatile("" : "+v"(v)); }

__device__ __forceinline__ int reflect(int i, int n)
{
    return i < 0 ? -i : (i > n - 1 ? 2 * (n - 1) - i : i);
}

// The tile owning workgroup number gb: the last t with start[t] <= gb.
__device__ __forceinline__ int find_tile(const int *start, int n, int gb)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= gb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// This workgroup's tile and its workgroup number within the tile; false for
// a surplus workgroup (the whole workgroup must then return).
struct Where {
    int t, lb;
};
__device__ __forceinline__ bool locate(const Batch &bt, Where &w)
{
    const int k = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const int gb = bt.xcd[k] + j;
    if (gb >= bt.xcd[k + 1]) return false;
    w.t = find_tile(bt.start, bt.n, gb);
    w.lb = gb - bt.start[w.t];
    return true;
}

// Workgroup lb of a tile in the update pass.
struct ZTile {
    int x, y, z0, z1, tile;
    bool active;
};

// Workgroup lb of a tile covers (TX x TY columns) x (one z chunk), z chunk
// fastest.
template <int TX, int TY>
__device__ __forceinline__ ZTile z_tile_t(const Grid3 &g, int nzc, int lb)
{
    ZTile zt;
    const int tile = lb;
    const int nbx = (g.nx + TX - 1) / TX;
    const int zc = tile % nzc, col = tile / nzc;
    const int lz = (g.nz + nzc - 1) / nzc;
    zt.x = (col % nbx) * TX + (threadIdx.x & (TX - 1));
    zt.y = (col / nbx) * TY + (threadIdx.x / TX);
    zt.z0 = zc * lz;
    zt.z1 = min(zt.z0 + lz, g.nz);
    zt.tile = tile;
    zt.active = zt.x < g.nx && zt.y < g.ny;
    return zt;
}

// Workgroup lb of a tile in the z passes: kThreads consecutive columns
// (y nx + x, so every access is contiguous across row ends) times one z
// chunk, z chunk fastest.
struct ZCols {
    int col, z0, z1;
    bool active;
};
__device__ __forceinline__ ZCols z_cols(const Grid3 &g, int nzc, int lb)
{
    ZCols zc;
    const int c = lb % nzc, cb = lb / nzc;
    const int lz = (g.nz + nzc - 1) / nzc;
    zc.col = cb * kThreads + (int)threadIdx.x;
    zc.z0 = c * lz;
    zc.z1 = min(zc.z0 + lz, g.nz);
    zc.active = zc.col < g.sxy;
    return zc;
}

}  // namespace

}  // namespace rsf
