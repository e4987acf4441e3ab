// Host-side helpers shared by the evolution entry points (rsf_api.hip) and the
// request server (rsf_server.hip): validation, Gaussian taps, coefficients,
// and the per-tile workspace regions.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "rsf.h"
#include "rsf_internal.hpp"

namespace rsf {
namespace host {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline size_t elem_size(int dtype) { return dtype == RSF_F32 ? 4 : 2; }

// Truncation radius of the sampled Gaussian: R = ceil(3 sigma) (Sec. 3).
inline int radius_of(float sigma) { return (int)std::ceil(3.0 * (double)sigma - 1e-9); }

// Sampled, truncated, unit-sum Gaussian (Sec. 3 kernel on the grid).
inline Taps make_taps(float sigma, int R)
{
    Taps t{};
    double w[2 * kMaxR + 1];
    double sum = 0.0;
    for (int k = -R; k <= R; ++k) {
        w[k + R] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
        sum += w[k + R];
    }
    // mirrored, so that the taps are exactly symmetric (the kernels read
    // w[0..R] only)
    for (int k = 0; k <= R; ++k) t.w[R - k] = t.w[R + k] = (float)(w[R + k] / sum);
    return t;
}

inline Coeffs make_coeffs(const rsf_params &p, double tol)
{
    Coeffs c{};
    c.l1 = p.lambda1; c.l2 = p.lambda2; c.nu = p.nu; c.mu = p.mu; c.dt = p.dt;
    c.eps = p.eps;
    c.eps_over_pi = (float)((double)p.eps / M_PI);
    c.eps2 = p.eps * p.eps;
    c.eta = p.eta > 0.f ? p.eta : 1e-10f;
    c.reg = p.regulariser == RSF_REG_SINGLE_WELL ? 1 : 0;
    c.force = p.force;
    c.tol = tol;
    return c;
}

// Each returns nullptr when the argument is valid, else the reason.
inline const char *dims_error(int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 3 || ny < 3 || nz < 3) return "every dimension must be >= 3";
    // in-slice byte offsets of 8-byte elements, y nx + x plus a workgroup's
    // overhang, stay below 2^32 (kernels address a slice with a 32-bit
    // unsigned offset from a 64-bit slice base)
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30) ||
        nx * ny > kMaxPlane || nx * ny > INT64_MAX / nz)
        return "volume too large";
    return nullptr;
}

inline const char *params_error(const rsf_params &p)
{
    const auto fin = [](float v) { return std::isfinite(v); };
    if (!fin(p.sigma) || !fin(p.lambda1) || !fin(p.lambda2) || !fin(p.nu) || !fin(p.mu) ||
        !fin(p.dt) || !fin(p.eps) || !fin(p.eta))
        return "parameters must be finite";
    if (!(p.sigma > 0.f) || radius_of(p.sigma) > kMaxR)
        return "sigma must be > 0 with ceil(3 sigma) <= 16";
    if (!(p.eps > 0.f)) return "eps must be > 0";
    if (!(p.dt > 0.f)) return "dt must be > 0";
    if (p.nu < 0.f || p.mu < 0.f) return "nu and mu must be >= 0";
    if (p.regulariser != RSF_REG_DOUBLE_WELL && p.regulariser != RSF_REG_SINGLE_WELL)
        return "unknown regulariser";
    if (p.storage != RSF_F32 && p.storage != RSF_F16 && p.storage != RSF_BF16)
        return "storage must be RSF_F32, RSF_F16 or RSF_BF16";
    if (p.force != RSF_FORCE_RSF && p.force != RSF_FORCE_PAPER) return "unknown force";
    if (!fin(p.sigma2) || p.sigma2 < 0.f) return "sigma2 must be finite and >= 0";
    if (p.force == RSF_FORCE_PAPER && radius_of(p.sigma2) > kMaxR)
        return "sigma2 must have ceil(3 sigma2) <= 16";
    return nullptr;
}

// The Sec. 4.2 force with sigma2 > 0 needs K2*I and K2*I^2.
inline bool needs_k2(const rsf_params &p) { return p.force == RSF_FORCE_PAPER && p.sigma2 > 0.f; }

inline const char *types_error(float sigma, int image, int storage)
{
    if (image != RSF_F32 && image != RSF_U16) return "volume dtype must be RSF_F32 or RSF_U16";
    if (!types_supported(radius_of(sigma), image, storage))
        return "this image/storage combination is built for ceil(3 sigma) in 4..12 only";
    return nullptr;
}

inline const char *types_error(const rsf_params &p, int image)
{
    if (const char *w = types_error(p.sigma, image, p.storage)) return w;
    if (needs_k2(p) && !types_supported(radius_of(p.sigma2), image, p.storage))
        return "this image/storage combination is built for ceil(3 sigma2) in 4..12 only";
    return nullptr;
}

inline Grid3 grid_of(int64_t nx, int64_t ny, int64_t nz)
{
    return Grid3{(int)nx, (int)ny, (int)nz, nx * ny};
}

// One tile's workspace: the pair fields P and Q and K*I in the storage type,
// the phi ping-pong buffer in float, K*1 edge tables, update partials (sized
// for any valid split), the per-iteration history and the flags.  Offsets are
// relative to the region's start; `total` is its size.
struct TileRegions {
    size_t P, Q, KI, K2I, K2I2, phiB, cx, cy, cz, partials, hist, flags, total;
    bool k2;
};

// k2: also K2*I and K2*I^2 (the Sec. 4.2 force with sigma2 > 0).
inline TileRegions tile_regions(const Grid3 &g, int iters, int storage, bool k2 = false)
{
    TileRegions T{};
    const size_t v = (size_t)g.nx * g.ny * g.nz;
    size_t off = 0;
    T.k2 = k2;
    T.P = off; off += align_up(2 * v * elem_size(storage));
    T.Q = off; off += align_up(2 * v * elem_size(storage));
    T.KI = off; off += align_up(v * elem_size(storage));
    if (k2) {
        T.K2I = off; off += align_up(v * elem_size(storage));
        T.K2I2 = off; off += align_up(v * elem_size(storage));
    }
    T.phiB = off; off += align_up(v * sizeof(float));
    T.cx = off; off += align_up((size_t)g.nx * sizeof(float));
    T.cy = off; off += align_up((size_t)g.ny * sizeof(float));
    T.cz = off; off += align_up((size_t)g.nz * sizeof(float));
    T.partials = off; off += align_up((size_t)u_blocks_max(g) * sizeof(double));
    T.hist = off; off += align_up((size_t)(iters > 0 ? iters : 1) * sizeof(double));
    T.flags = off; off += align_up(4 * sizeof(int));
    T.total = off;
    return T;
}

// Fill a tile descriptor from its region at `base`.  flags: 4 ints (flags[0],
// flags[1], then the last sum |dphi| as a double), 8-byte aligned.
inline TileDesc tile_desc(const Grid3 &g, const Split &sp, const void *volume, float *phi,
                          char *base, const TileRegions &T, int iters, int *flags)
{
    TileDesc d{};
    d.g = g;
    d.sp = sp;
    d.I = volume;
    d.phi[0] = phi;
    d.phi[1] = reinterpret_cast<float *>(base + T.phiB);
    d.P = base + T.P;
    d.Q = base + T.Q;
    d.KI = base + T.KI;
    d.K2I = T.k2 ? base + T.K2I : nullptr;
    d.K2I2 = T.k2 ? base + T.K2I2 : nullptr;
    d.cx = reinterpret_cast<float *>(base + T.cx);
    d.cy = reinterpret_cast<float *>(base + T.cy);
    d.cz = reinterpret_cast<float *>(base + T.cz);
    d.partials = reinterpret_cast<double *>(base + T.partials);
    d.hist = reinterpret_cast<double *>(base + T.hist);
    d.hist_cap = iters > 0 ? iters : 1;
    d.flags = flags ? flags : reinterpret_cast<int *>(base + T.flags);
    return d;
}

// ---------------------------------------------------------------------------
// XCD ranges.  The cost of a workgroup is the rows (xy passes) or slices (z
// and update passes) it marches, counting the halo rows or slices that lie
// inside the tile (those outside are zero padding and never loaded).
// ---------------------------------------------------------------------------

enum PassKind { PASS_XY, PASS_Z, PASS_U };

inline int64_t span_cost(int n, int chunks, int idx, int R)
{
    const int len = (n + chunks - 1) / chunks;
    const int a = idx * len, b = std::min(a + len, n);
    return (int64_t)(b - a) + std::min(R, a) + std::min(R, n - b);
}

inline int64_t blocks_of(PassKind k, const Grid3 &g, const Split &s)
{
    return k == PASS_XY ? xy_blocks(g, s) : (k == PASS_Z ? z_blocks(g, s) : u_blocks(g, s));
}

// Cut the batch's workgroups (tile by tile, each tile in its own workgroup
// order) into kXcds contiguous ranges of about equal total cost, write them
// to b.xcd and return the grid size (kXcds times the longest range).
inline int64_t balance_xcds(Batch &b, PassKind k, const std::vector<Grid3> &g,
                            const std::vector<Split> &sp, int R)
{
    // per-tile: workgroups and the cost of each of its (repeating) chunks
    double total = 0.0;
    int64_t nblocks = 0;
    for (size_t t = 0; t < g.size(); ++t) {
        const int nch = k == PASS_XY ? sp[t].xy : (k == PASS_Z ? sp[t].z : sp[t].u);
        const int n = k == PASS_XY ? g[t].ny : g[t].nz;
        double per = 0.0;   // cost of one full cycle of chunks
        for (int c = 0; c < nch; ++c) per += (double)span_cost(n, nch, c, R);
        const int64_t nb = blocks_of(k, g[t], sp[t]);
        total += per * (double)(nb / nch);
        nblocks += nb;
    }
    // walk the workgroups once, cutting at multiples of total / kXcds
    int cut = 1;
    double acc = 0.0;
    int64_t gb = 0;
    b.xcd[0] = 0;
    for (size_t t = 0; t < g.size() && cut < kXcds; ++t) {
        const int64_t nb = blocks_of(k, g[t], sp[t]);
        const int nch = k == PASS_XY ? sp[t].xy : (k == PASS_Z ? sp[t].z : sp[t].u);
        const int n = k == PASS_XY ? g[t].ny : g[t].nz;
        const int nbx = nbx64(g[t].nx);
        for (int64_t lb = 0; lb < nb && cut < kXcds; ++lb, ++gb) {
            // chunk index of workgroup lb in the tile's workgroup order
            const int c = k == PASS_XY ? (int)((lb / nbx) % nch) : (int)(lb % nch);
            const double w = (double)span_cost(n, nch, c, R);
            // the cut goes before this workgroup if that is nearer the target
            while (cut < kXcds && acc + 0.5 * w >= total * cut / kXcds) b.xcd[cut++] = (int)gb;
            acc += w;
        }
    }
    while (cut <= kXcds) b.xcd[cut++] = (int)nblocks;
    int64_t longest = 0;
    for (int x = 0; x < kXcds; ++x) longest = std::max<int64_t>(longest, b.xcd[x + 1] - b.xcd[x]);
    return longest * kXcds;
}

}  // namespace host
}  // namespace rsf
