// Device templates of the RSF passes (xy and z Gaussian passes with their
// epilogues) and their per-radius launchers.  Included by the translation
// units that instantiate them for a range of radii (rsf_inst_*.hip).
#pragma once

#include <type_traits>

#include "rsf_device.hpp"

namespace rsf {

namespace {

// ---------------------------------------------------------------------------
// xy pass as a march along y.  One wave owns a 64-wide strip of one z slice
// and a chunk of rows.  Each incoming row (with an R halo in x) is staged in
// LDS, convolved along x (one output per lane), and pushed into a per-lane
// register ring of 2R+1 rows, from which the y convolution is taken; x halo
// work is paid only on the chunk's 2R extra rows, never per row.
// ---------------------------------------------------------------------------

// XY_ONE reads the image (IN) and writes one field P (ST), for K*I; XY_FITS
// reads the pair P and K*I and writes the pair Q; XY_TWO reads the pair Q and
// writes the pair P; XY_PAPER reads the pair P, K*I and the image (IMG) and
// writes the force of Sec. 4.2 with sigma2 = 0 to Q as float.
// At least five waves per SIMD (at most 96 registers) where the ring of
// 2R + 2 rows and the stages fit without spilling: radius <= 8, or 9 except
// for the fits of 16-bit storage.  Otherwise, and for the Sec. 4.2 force
// modes (more pointwise inputs), the compiler's own choice (no bound).
template <int R, int MODE, class ST>
constexpr int xy_waves_per_eu =
    (MODE == XY_ONE || MODE == XY_TWO || MODE == XY_FITS) &&
            (R <= 8 || (R == 9 && (std::is_same<ST, float>::value || MODE != XY_FITS)))
        ? 5
        : 1;

template <int R, int MODE, class IN, class ST, class IMG = float>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(xy_waves_per_eu<R, MODE, ST>)))
void xy_kernel(Batch bt, Taps t, Coeffs c)
{
    constexpr bool PAPER_F = MODE == XY_PAPER || MODE == XY_PAPER2;
    constexpr bool FITS = MODE == XY_FITS || PAPER_F;
    constexpr int NF = MODE == XY_ONE ? 1 : 2;
    constexpr int W = 2 * R + 1;
    constexpr int RW = 64 + 2 * R;
    static_assert(RW <= 128, "a staged row is two loads per lane");
    // rows are written whole (128 entries, the tail past RW is never read)
    // so that staging has no branch
    __shared__ float row[2][NF][128];
    // FP16 pairs are staged as they are loaded, both fields in one word, and
    // converted by the x convolution's mixed-precision FMAs (exactly, as a
    // conversion at staging would): half the LDS traffic, no conversions
    constexpr bool PACKROW = NF == 2 && std::is_same<IN, _Float16>::value;
    // Other pairs are staged interleaved, (a, b) per column, so one 64-bit
    // LDS read serves a tap of both fields (and a 128-bit pair read two
    // taps): half the LDS instructions of two separate rows, the same bytes.
    constexpr bool PAIRROW = NF == 2 && !PACKROW;
    __shared__ float2 rowp[2][PAIRROW ? 128 : 1];

    Where wh;
    if (!locate(bt, wh)) return;
    const TileDesc &d = bt.tiles[wh.t];
    if (glb(d.flags)[0]) return;
    const Grid3 g = d.g;
    const int nyc = d.sp.xy;
    const void *__restrict__ in_ = MODE == XY_ONE ? d.I : (FITS ? d.P : d.Q);
    void *__restrict__ out_ = FITS ? d.Q : d.P;
    const int nbx = (g.nx + 63) / 64;
    const int tile = wh.lb;
    const int xs = tile % nbx, rest = tile / nbx;
    const int yc = rest % nyc, z = rest / nyc;
    const int ly = (g.ny + nyc - 1) / nyc;
    const int y0 = yc * ly, y1 = min(y0 + ly, g.ny);
    const int lane = threadIdx.x;
    const int x0 = xs * 64, x = x0 + lane;
    const int64_t zb = (int64_t)z * g.sxy;

    // Raw elements of one row (lanes j and j + 64), converted when staged.
    // The loads are unconditional, with the row and column clamped into the
    // slice; the zero padding is applied when the row is staged.  No load
    // sits under a branch, so waiting for one row leaves later rows in
    // flight.
    struct Raw {
        Vec2<IN> p[2];
        IN s[2];
    };
    // the slice through a buffer descriptor: a row is a uniform byte offset,
    // each lane's column a loop-invariant 32-bit one
    const rsrc_t rin = rsrc(static_cast<const char *>(in_) +
                            zb * (int64_t)(NF == 2 ? sizeof(Pair<IN>) : sizeof(IN)));
    uint32_t gxo[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        // lanes past the staged width load the last staged column: same
        // cache line, no extra traffic
        gxo[h] = (uint32_t)min(max(x0 - R + min(lane + 64 * h, RW - 1), 0), g.nx - 1);
    }
    auto fetch = [&](int y) {
        Raw r;
        const int yy = min(max(y, 0), g.ny - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (NF == 2)
                r.p[h] = bld<Vec2<IN>>(rin, gxo[h], (uint32_t)(yy * g.nx) * (uint32_t)sizeof(Pair<IN>));
            else
                r.s[h] = bld<IN>(rin, gxo[h], (uint32_t)(yy * g.nx) * (uint32_t)sizeof(IN));
        }
        return r;
    };
    // Stage row y (fetched) into LDS slot `slot`, run `between` (work that
    // does not touch the row: the next y convolution, whose two sums it
    // returns), x-convolve the row and return the lane's value.  `between`
    // and the x-convolution's LDS reads share one scheduling region (the
    // wave sync opens it, one `pin` of all four sums closes it), so its FMAs
    // can fill the reads' latency.  Values outside the slice are zeroed by a
    // bit mask, not a branch, so staging opens no new region either.
    auto xrow = [&](const Raw &r, int y, int slot, auto &&between, float2 &yv) -> float2 {
        const bool yok = y >= 0 && y < g.ny;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            const int gx = x0 - R + j;
            const int keep = (yok && gx >= 0 && gx < g.nx) ? -1 : 0;
            auto masked = [&](float v) { return __int_as_float(__float_as_int(v) & keep); };
            if constexpr (PACKROW) {
                const uint32_t bits = __builtin_bit_cast(uint32_t, r.p[h]) & (uint32_t)keep;
                row[slot][0][j] = __builtin_bit_cast(float, bits);
            } else if constexpr (PAIRROW) {
                rowp[slot][j] = make_float2(masked(to_f(r.p[h].x)), masked(to_f(r.p[h].y)));
            } else if (NF == 2) {
                row[slot][0][j] = masked(to_f(r.p[h].x));
                row[slot][NF - 1][j] = masked(to_f(r.p[h].y));
            } else {
                const float v = masked(to_f(r.s[h]));
                row[slot][0][j] = c.square ? v * v : v;
            }
        }
        // the workgroup is one wave: order its LDS writes before the reads
        // (a workgroup barrier's fence would also wait for the global stores
        // and loads in flight)
        __syncwarp();
        yv = between();
        float ca = 0.f, cb = 0.f;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if constexpr (PACKROW) {
                const Vec2<_Float16> v = __builtin_bit_cast(Vec2<_Float16>, row[slot][0][lane + k]);
                ca = fmaf(tap<R>(t, k), (float)v.x, ca);
                cb = fmaf(tap<R>(t, k), (float)v.y, cb);
            } else if constexpr (PAIRROW) {
                const float2 v = rowp[slot][lane + k];
                ca = fmaf(tap<R>(t, k), v.x, ca);
                cb = fmaf(tap<R>(t, k), v.y, cb);
            } else {
                ca = fmaf(tap<R>(t, k), row[slot][0][lane + k], ca);
                if (NF == 2) cb = fmaf(tap<R>(t, k), row[slot][NF - 1][lane + k], cb);
            }
        }
        __asm__ volatile("" : "+v"(ca), "+v"(cb), "+v"(yv.x), "+v"(yv.y));
        return make_float2(ca, cb);
    };
    auto nothing = [] { return make_float2(0.f, 0.f); };

    // Prefetch depth as in the update pass: two stages (a row and the
    // pointwise inputs of one step) alternate by step parity where the
    // registers allow.  The x convolution runs one row ahead of the y
    // convolution: step y x-convolves row y + R + 1 (for the next step) while
    // it y-convolves output y from rows already in the ring, so the LDS reads
    // of the one overlap the FMAs of the other.  The ring therefore holds
    // 2R + 2 rows, and the march is unrolled by M = 2R + 2 (even, as the
    // alternating stages need).
    constexpr int PF = R <= 10 ? 2 : 1;
    constexpr int M = W + 1;
    const int xc = min(x, g.nx - 1);
    const int last = min(63, g.nx - 1 - x0);   // last in-slice lane of the strip
    const rsrc_t rki = rsrc(static_cast<const ST *>(d.KI) + zb);
    const rsrc_t rim = rsrc(static_cast<const IMG *>(d.I) + zb);
    const rsrc_t rk2i = rsrc(static_cast<const ST *>(d.K2I) + zb);
    const rsrc_t rk2q = rsrc(static_cast<const ST *>(d.K2I2) + zb);
    const float cxz = FITS ? glb(d.cx)[xc] * glb(d.cz)[z] : 0.f;
    const float *const cyp = d.cy;   // read once: the loop's stores could alias the table
    // the loads of step y: row y + R + 1 and the fits' pointwise inputs of row y
    struct Stage {
        Raw row;
        ST ki, k2i, k2q;
        IMG im;
        float cy;
    };
    auto stage = [&](int y) {
        Stage st;
        st.row = fetch(y + R + 1);
        if (FITS) {
            const int yy = min(y, g.ny - 1);
            const uint32_t row = (uint32_t)(yy * g.nx);
            st.ki = bld<ST>(rki, (uint32_t)xc, row * (uint32_t)sizeof(ST));
            st.cy = uniform_ld(cyp, yy);   // one value for the wave: a scalar load
            if (MODE == XY_PAPER) st.im = bld<IMG>(rim, (uint32_t)xc, row * (uint32_t)sizeof(IMG));
            if (MODE == XY_PAPER2) {
                st.k2i = bld<ST>(rk2i, (uint32_t)xc, row * (uint32_t)sizeof(ST));
                st.k2q = bld<ST>(rk2q, (uint32_t)xc, row * (uint32_t)sizeof(ST));
            }
        }
        return st;
    };

    // prologue: rows y0 - R .. y0 + R x-convolved into ring slots 0..2R (row
    // y0 - R + j staged in LDS slot j & 1)
    float ra[M], rb[M];
    Stage sa, sb;
    {
        Raw nxt = fetch(y0 - R);
#pragma unroll
        for (int j = 0; j <= 2 * R; ++j) {
            const Raw cur = nxt;
            if (j < 2 * R) {
                nxt = fetch(y0 - R + j + 1);
            } else {
                sa = stage(y0);
                if (PF == 2) sb = stage(y0 + 1);
            }
            float2 unused;
            const float2 v = xrow(cur, y0 - R + j, j & 1, nothing, unused);
            ra[j] = v.x;
            rb[j] = v.y;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const gptr<float> probe_f1 = glb(d.probe_f1), probe_f2 = glb(d.probe_f2),
                      probe_fd = glb(d.probe_Fd);
    // outputs of the slice: one ST field, the pair, or the float force
    const rsrc_t rout = rsrc(static_cast<char *>(out_) +
                             zb * (int64_t)(PAPER_F ? sizeof(float)
                                                    : (NF == 2 ? sizeof(Pair<ST>) : sizeof(ST))));
    // step y (s = its index in the unrolled block) consumes stage `cur` and
    // refills it with the loads of step y + PF
    auto step = [&](Stage &cur, const int s, const int y) {
        const Raw rw = cur.row;
        const ST ki_raw = cur.ki, k2i_raw = cur.k2i, k2q_raw = cur.k2q;
        const IMG im_raw = cur.im;
        const float cyv = cur.cy;
        // Output y from ring rows y - R .. y + R (slots s .. s + 2R), computed
        // while row y + R + 1 is x-convolved for the next step (also on a
        // chunk's last step: no branch; the row is clamped and zero-padded
        // like any other).  That row is the (y - y0 + 2R + 1)-th staged one:
        // LDS slot parity (y - y0 + 1) & 1.
        auto yconv = [&] {
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                a = fmaf(tap<R>(t, k), ra[(s + k) % M], a);
                if (NF == 2) b = fmaf(tap<R>(t, k), rb[(s + k) % M], b);
            }
            return make_float2(a, b);
        };
        float2 acc, xv;
        if constexpr (MODE == XY_PAPER2) {
            // four pointwise inputs per step: interleaving would spill
            float2 unused;
            acc = yconv();
            xv = xrow(rw, y + R + 1, (y - y0 + 1) & 1, nothing, unused);
        } else {
            xv = xrow(rw, y + R + 1, (y - y0 + 1) & 1, yconv, acc);
        }
        const float acc_a = acc.x, acc_b = acc.y;
        ra[(s + 2 * R + 1) % M] = xv.x;
        rb[(s + 2 * R + 1) % M] = xv.y;
        cur = stage(y + PF);
        // every lane stores: one past the slice edge (x >= nx) writes the
        // value of the last in-slice lane to that lane's element (same bits)
        const uint32_t v = (uint32_t)(y * g.nx + xc);   // offset within the slice
        const uint32_t row = (uint32_t)(y * g.nx);
        auto edge = [&](float val) { return x < g.nx ? val : lane_value(val, last); };
        if (FITS) {
            const float ki = to_f(ki_raw);
            // region fits (Sec. 3 local_intensity)
            const float K1 = cxz * cyv;
            const float A2 = ki - acc_a;
            const float B2 = K1 - acc_b;
            const float f1 = acc_a * rcp(acc_b);
            const float f2 = A2 * rcp(B2);
            if (MODE == XY_PAPER) {
                // F+- = (I - r+-)^2 (Sec. 4.2 expansion, sigma2 = 0)
                const float im = to_f(im_raw);
                const float d1 = im - f1, d2 = im - f2;
                const float Fd = edge(c.l1 * d1 * d1 - c.l2 * d2 * d2);
                bst<float>(rout, (uint32_t)xc, Fd, row * 4u);
                if (probe_fd) probe_fd[zb + v] = Fd;
            } else if (MODE == XY_PAPER2) {
                // F+- = K2*I^2 - 2 r+- K2*I + r+-^2 (Sec. 4.2 expansion)
                const float a = to_f(k2i_raw), q = to_f(k2q_raw);
                const float F1 = q - 2.f * f1 * a + f1 * f1;
                const float F2 = q - 2.f * f2 * a + f2 * f2;
                const float Fd = edge(c.l1 * F1 - c.l2 * F2);
                bst<float>(rout, (uint32_t)xc, Fd, row * 4u);
                if (probe_fd) probe_fd[zb + v] = Fd;
            } else {
                // force-convolution inputs g1, g2
                bst_pair<ST>(rout, (uint32_t)xc, edge(c.l1 * f1 - c.l2 * f2),
                             edge(c.l1 * f1 * f1 - c.l2 * f2 * f2),
                             row * (uint32_t)sizeof(Pair<ST>));
            }
            if (probe_f1) probe_f1[zb + v] = edge(f1);
            if (probe_f2) probe_f2[zb + v] = edge(f2);
        } else if (NF == 2) {
            bst_pair<ST>(rout, (uint32_t)xc, edge(acc_a), edge(acc_b),
                         row * (uint32_t)sizeof(Pair<ST>));
        } else {
            bst<ST>(rout, (uint32_t)xc, from_f<ST>(edge(acc_a)), row * (uint32_t)sizeof(ST));
        }
    };
    // whole blocks of M steps with no branch around the steps (as in the
    // update pass), then the rest of the chunk with a per-step check
    int yb = y0;
    for (; yb + M <= y1; yb += M) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            if (PF == 2 && (s & 1)) step(sb, s, yb + s);
            else step(sa, s, yb + s);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (; yb < y1; yb += M) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const int y = yb + s;
            if (y < y1) {
                if (PF == 2 && (s & 1)) step(sb, s, y);
                else step(sa, s, y);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---------------------------------------------------------------------------
// z passes: a thread owns column (x, y) and marches z0..z1 with a ring of the
// 2R+1 slices around z held in registers.  The ring is indexed with
// compile-time slots by unrolling the march in steps of 2R+1.
// ---------------------------------------------------------------------------


// Raw stage-1 inputs of one voxel: phi and the image element.
template <class IT>
struct PhiImg {
    float phi;
    IT img;
};

// Conv ring.  fetch(z) loads the raw inputs of slice z (0 <= z < nz) and
// cook(raw, z) turns them into the two convolved quantities; each slice is
// fetched one step before it is cooked so the load latency overlaps the
// previous step's arithmetic.
template <int R, int NF, typename Fetch, typename Cook, typename Epi>
__device__ __forceinline__ void z_march(int nz, int z0, int z1, const Taps &t, Fetch &&fetch,
                                        Cook &&cook, Epi &&epi)
{
    constexpr int W = 2 * R + 1;
    float ra[W], rb[W];
    // every fetch is unconditional, with the slice clamped into the volume;
    // `use` replaces a slice outside it by the zero padding
    using Raw = decltype(fetch(0));
    auto get = [&](int z) { return fetch(min(max(z, 0), nz - 1)); };
    auto use = [&](const Raw &raw, int z) {
        float2 v = (z >= 0 && z < nz) ? cook(raw, z) : make_float2(0.f, 0.f);
        pin(v.x);
        if (NF == 2) pin(v.y);
        return v;
    };
    Raw nxt = get(z0 - R);
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        const Raw cur = nxt;
        nxt = get(z0 - R + j + 1);
        const float2 v = use(cur, z0 - R + j);
        ra[j] = v.x;
        rb[j] = v.y;
        __builtin_amdgcn_sched_barrier(0);
    }
    auto step = [&](const int s, const int z) {
        const int zn = z + R;
        const auto cur = nxt;
        nxt = get(zn + 1);
        const float2 v = use(cur, zn);
        ra[(s + 2 * R) % W] = v.x;
        rb[(s + 2 * R) % W] = v.y;
        float acc_a = 0.f, acc_b = 0.f;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            acc_a = fmaf(tap<R>(t, k), ra[(s + k) % W], acc_a);
            if (NF == 2) acc_b = fmaf(tap<R>(t, k), rb[(s + k) % W], acc_b);
        }
        epi(z, acc_a, acc_b);
    };
    // Whole blocks of W steps run with no branch around the steps (a step
    // under a branch ends at a join whose register copies wait for the
    // prefetch); the rest of the chunk checks each step.  Each step's work
    // stays inside the step; the one-step prefetch and occupancy hide the
    // latency.
    int zb = z0;
    for (; zb + W <= z1; zb += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            step(s, zb + s);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (; zb < z1; zb += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            if (zb + s < z1) step(s, zb + s);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// K*I: z pass of the field P into KI.
template <int R, class ST>
__global__ __launch_bounds__(kThreads) void z_plain_kernel(Batch bt, Taps t, int target)
{
    Where wh;
    if (!locate(bt, wh)) return;
    const TileDesc &d = bt.tiles[wh.t];
    const Grid3 g = d.g;
    const gptr<const ST> in = glb(static_cast<const ST *>(d.P));
    const gptr<ST> out = glb(static_cast<ST *>(
        target == Z_TO_KI ? d.KI : (target == Z_TO_K2I ? d.K2I : d.K2I2)));
    const ZCols zt = z_cols(g, d.sp.z, wh.lb);
    if (!zt.active) return;
    const uint32_t col = (uint32_t)zt.col;   // nx * ny <= kMaxPlane
    z_march<R, 1>(
        g.nz, zt.z0, zt.z1, t,
        [&](int z) { return bld<ST>(rsrc(in + (int64_t)z * g.sxy), col); },
        [&](ST raw, int) { return make_float2(to_f(raw), 0.f); },
        [&](int z, float va, float) { bst<ST>(rsrc(out + (int64_t)z * g.sxy), col, from_f<ST>(va)); });
}

// Stage-1 z pass: H_eps(phi) and H I formed as slices enter the ring.
template <int R, bool PROBE, class ST, class IT>
__global__ __launch_bounds__(kThreads) void z_heaviside_kernel(Batch bt, Taps t, Coeffs c)
{
    Where wh;
    if (!locate(bt, wh)) return;
    const TileDesc &d = bt.tiles[wh.t];
    if (glb(d.flags)[0]) return;
    const Grid3 g = d.g;
    const gptr<const float> phi = glb(d.phi[glb(d.flags)[1] & 1]);   // iterate n is in phi[n & 1]
    const gptr<const IT> I = glb(static_cast<const IT *>(d.I));
    const gptr<Pair<ST>> tp = glb(static_cast<Pair<ST> *>(d.P));
    const gptr<float> probeH = glb(d.probe_H);
    const float eps = c.eps;
    const ZCols zt = z_cols(g, d.sp.z, wh.lb);
    if (!zt.active) return;
    const uint32_t col = (uint32_t)zt.col;   // nx * ny <= kMaxPlane
    z_march<R, 2>(
        g.nz, zt.z0, zt.z1, t,
        [&](int z) {
            const int64_t zo = (int64_t)z * g.sxy;
            return PhiImg<IT>{bld<float>(rsrc(phi + zo), col), bld<IT>(rsrc(I + zo), col)};
        },
        [&](const PhiImg<IT> &raw, int z) {
            const float H = heaviside(raw.phi, eps);
            if (PROBE && probeH) (probeH + (int64_t)z * g.sxy)[col] = H;
            return make_float2(H * to_f(raw.img), H);
        },
        [&](int z, float va, float vb) {
            if constexpr (!std::is_same<ST, float>::value) {
                // as in the fused update: round the FP32 sums, then convert
                pin(va);
                pin(vb);
            }
            bst_pair<ST>(rsrc(tp + (int64_t)z * g.sxy), col, va, vb);
        });
}

// Unit normal n = g / sqrt(|g|^2 + eta) and regulariser flux V = D(|g|) g,
// D(s) = d_p(s) - 1.  Double well: D = sin(2 pi s)/(2 pi s) - 1 for s <= 1,
// -1/s for s > 1, 0 at s = 0; single well: D = -1/sqrt(|g|^2 + eta).
// v_sin_f32 takes its argument in turns, so it returns sin(2 pi s).
__device__ __forceinline__ void normal_flux(float gx, float gy, float gz, float eta, int reg,
                                            float &nx_, float &ny_, float &nz_, float &vx_,
                                            float &vy_, float &vz_)
{
    const float s2 = gx * gx + gy * gy + gz * gz;
    const float inv_eta = __builtin_amdgcn_rsqf(s2 + eta);
    float D;
    if (reg != 0) {
        D = -inv_eta;
    } else {
        const float rs = __builtin_amdgcn_rsqf(s2);        // inf at s2 = 0
        const float sv = s2 * rs;                           // |g| (NaN at 0)
        const float dw = __builtin_amdgcn_sinf(sv) * rs * (1.f / kTwoPi) - 1.f;
        D = sv > 1.f ? -rs : (s2 > 0.f ? dw : 0.f);
    }
    nx_ = gx * inv_eta; ny_ = gy * inv_eta; nz_ = gz * inv_eta;
    vx_ = D * gx; vy_ = D * gy; vz_ = D * gz;
}

// Stage-2 z pass with the update.  The block's tile is kUx x kUy columns.
// Alongside the per-thread conv ring it keeps in LDS a ring of phi slices
// (tile + 2 halo, 6 slots) and, per slice, the x/y components of the unit
// normal n and of the regulariser flux V = D(|grad phi|) grad phi at the tile
// + 1 halo (3 slots); the z components of the thread's own column stay in
// registers.  Each point's gradient, n and V are computed once and shared by
// the six neighbours whose divergence needs them.
//
// Step z of the march (one barrier per step):
//   store phi(z+3) (fetched one step earlier); barrier;
//   n, V of slice z+2; update of slice z (reads n, V of slices z-1..z+1).
// Slot reuse is safe: phi(z+3) overwrites phi(z-3), last read in step z-2;
// n, V of z+2 overwrite those of z-1, last read in step z-1; a barrier
// separates each pair.
//
// PAPER: the force of Sec. 4.2 was formed by the xy pass and is read
// pointwise (float F_d in Q); there is no stage-2 ring and no image read, and
// R only sets the unroll.
//
// FUSE (every tile marched whole in z): the pass also forms the next
// iteration's stage-1 z Gaussian of (H(phi') I, H(phi')) from the phi' it has
// just computed, in a register ring of radius R, and writes it to P in place
// of the next z_heaviside pass.  At step z it pushes slice z and emits output
// slice z - R; R more steps past the end push the zero padding.  The
// products and the tap order are those of z_heaviside, so P is bitwise the
// same.  With the RSF force P is also this pass's stage-2 input; the z
// Gaussian reads P only in the thread's own column, and slice z - R entered
// the register ring steps before it is overwritten.
template <int R, bool PROBE, class ST, class IT, bool PAPER = false, bool FUSE = false>
__global__ __launch_bounds__(kUThreads, 4) void z_update_kernel(Batch bt, Taps t, Coeffs ua)
{
    static_assert(!(FUSE && PROBE), "probes run the passes separately");
    constexpr int TX = kUx, TY = kUy, NT = kUThreads;
    constexpr int PX = TX + 4, PY = TY + 4;
    constexpr int QX = TX + 2, QY = TY + 2;
    constexpr int QS = QY * QX;
    constexpr int NPHI = 6, NQ = 3;
    constexpr int NLD = (PX * PY + NT - 1) / NT;
    // each slot is padded to NLD * NT entries, so that every thread stores
    // its NLD loaded points with no branch (points past the tile land in
    // the padding, never read)
    __shared__ float sphi[NPHI][NLD * NT];
    __shared__ float sq[NQ][4][QS];   // n_x, V_x, n_y, V_y
    __shared__ double wsum[NT / 64];

    Where wh;
    if (!locate(bt, wh)) return;
    const TileDesc &d = bt.tiles[wh.t];
    // a stopped tile keeps its last iterate where it is (the whole block
    // leaves; its partial is not read)
    if (glb(d.flags)[0]) return;
    const Grid3 g = d.g;
    const gptr<const Pair<ST>> tp = glb(static_cast<const Pair<ST> *>(d.P));
    const int cur = glb(d.flags)[1] & 1;   // iterate n is in phi[n & 1]
    const gptr<const float> phi = glb(d.phi[cur]);
    const gptr<float> phi_out = glb(d.phi[cur ^ 1]);
    const ZTile zt = z_tile_t<TX, TY>(g, d.sp.u, wh.lb);
    const int tid = threadIdx.x;
    const int tx = tid & (TX - 1), ty = tid / TX;
    const int x0 = zt.x - tx, y0 = zt.y - ty;
    double acc = 0.0;

    {
        // phi tile loads: reflected in-slice offsets of this thread's points
        uint32_t loff[NLD];
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int i = tid + r * NT;
            const int px = i % PX, py = i / PX;
            const int gx = reflect(min(x0 - 2 + px, g.nx + 1), g.nx);
            const int gy = reflect(min(y0 - 2 + min(py, PY - 1), g.ny + 1), g.ny);
            loff[r] = (uint32_t)(gy * g.nx + gx);
        }
        struct PhiRaw {
            float v[NLD];
        };
        // Slices used for outputs lie in [-2, nz + 1]; the march also touches
        // up to nz + 4 (prefetch and n, V past the chunk end, never used), so
        // clamp before reflecting to keep every address inside the volume.
        // Lanes past the tile load a reflected in-volume point too and store
        // it to the slot's padding: every prefetch is an unconditional load,
        // so no branch forces a wait on the loads in flight.
        auto fetch_phi = [&](int j) {
            PhiRaw r;
            const gptr<const float> base = phi + (int64_t)reflect(min(j, g.nz + 1), g.nz) * g.sxy;
            const rsrc_t rb = rsrc(base);
#pragma unroll
            for (int k = 0; k < NLD; ++k) r.v[k] = bld<float>(rb, loff[k]);
            return r;
        };
        // Fast form (see `fast` below): slice j is in the volume, and its
        // offset from phi is a 32-bit scalar.
        const rsrc_t r_phi = rsrc(phi);
        const uint32_t sxy = (uint32_t)g.sxy;   // voxels per slice (<= kMaxPlane)
        auto fetch_phi_fast = [&](int j) {
            PhiRaw r;
            const uint32_t so = (uint32_t)j * (sxy * 4u);
#pragma unroll
            for (int k = 0; k < NLD; ++k) r.v[k] = bld<float>(r_phi, loff[k], so);
            return r;
        };
        auto phi_slot = [&](int j) { return sphi[(j + 2 * NPHI) % NPHI]; };
        auto store_phi = [&](const PhiRaw &r, int j) {
            float *dst = phi_slot(j);
#pragma unroll
            for (int k = 0; k < NLD; ++k) dst[tid + k * NT] = r.v[k];
        };
        // n and V at phi-tile point (cx, cy) of slice j
        auto qcalc = [&](int j, int cx, int cy, float &nx_, float &vx_, float &ny_, float &vy_,
                         float &nz_, float &vz_) {
            const float *p0 = phi_slot(j), *pm = phi_slot(j - 1), *pp = phi_slot(j + 1);
            const int c = cy * PX + cx;
            const float gx = 0.5f * (p0[c + 1] - p0[c - 1]);
            const float gy = 0.5f * (p0[c + PX] - p0[c - PX]);
            const float gz = 0.5f * (pp[c] - pm[c]);
            normal_flux(gx, gy, gz, ua.eta, ua.reg, nx_, ny_, nz_, vx_, vy_, vz_);
        };
        // halo points of the normal/flux tile: y halo rows (threads 0..2TX-1),
        // x halo columns (the next 2TY threads)
        int hq = -1;
        if (tid < 2 * TX) hq = (tid < TX ? 0 : QY - 1) * QX + (tid % TX) + 1;
        else if (tid < 2 * TX + 2 * TY) {
            const int k = tid - 2 * TX;
            hq = (k % TY + 1) * QX + (k < TY ? 0 : QX - 1);
        }
        const int own_q = (ty + 1) * QX + tx + 1;
        // n, V of slice j for the own point (z components returned) and halo
        auto q_phase = [&](int j, float &qnz, float &qvz) {
            float qnx, qvx, qny, qvy;
            qcalc(j, tx + 2, ty + 2, qnx, qvx, qny, qvy, qnz, qvz);
            float *q = &sq[(j + 2 * NQ) % NQ][0][0];
            q[0 * QS + own_q] = qnx;
            q[1 * QS + own_q] = qvx;
            q[2 * QS + own_q] = qny;
            q[3 * QS + own_q] = qvy;
            if (hq >= 0) {
                float a0, a1, a2, a3, a4, a5;
                qcalc(j, hq % QX + 1, hq / QX + 1, a0, a1, a2, a3, a4, a5);
                q[0 * QS + hq] = a0;
                q[1 * QS + hq] = a1;
                q[2 * QS + hq] = a2;
                q[3 * QS + hq] = a3;
            }
        };

        const uint32_t col = (uint32_t)(min(zt.y, g.ny - 1) * g.nx + min(zt.x, g.nx - 1));
        const float cxy = glb(d.cx)[min(zt.x, g.nx - 1)] * glb(d.cy)[min(zt.y, g.ny - 1)];
        const gptr<const IT> img = glb(static_cast<const IT *>(d.I));
        auto pair_at = [&](int z) { return bld<Vec2<ST>>(rsrc(tp + (int64_t)z * g.sxy), col); };
        const int z0 = zt.z0;
        // prologue: phi(z0-2..z0+2), then n, V of z0-1, z0, z0+1
#pragma unroll
        for (int j = -2; j <= 2; ++j) store_phi(fetch_phi(z0 + j), z0 + j);
        __syncthreads();
        float nzm, vzm, nz0, vz0, nzp, vzp;
        q_phase(z0 - 1, nzm, vzm);
        q_phase(z0, nz0, vz0);
        q_phase(z0 + 1, nzp, vzp);

        // Prefetch depth: two stages of loads in flight where the registers
        // allow (the conv ring grows with R).  The two stage buffers
        // alternate by step parity, never copied (a copy of registers whose
        // loads are in flight would wait for them), so the march is unrolled
        // by an even count M and the conv ring has M >= 2R + 1 slots.
        constexpr int W = 2 * R + 1;
        // With FP16 storage the stage-2 ring holds the raw pairs, one
        // register per slot, converted where the FMA reads them (the
        // conversion is exact, so the sums are unchanged), which leaves
        // registers for two prefetch stages at every radius and removes the
        // fused update's spills.  (BF16 would pay an extra instruction per
        // tap for its conversion: it keeps the FP32 ring.)  FUSE holds a
        // second (FP32) ring: with the RSF force's stage-2 ring it runs one
        // prefetch stage.
        constexpr bool PACK = std::is_same<ST, _Float16>::value;
        constexpr int PF = FUSE ? (R <= (PAPER ? 9 : 0) ? 2 : 1)
                                : ((PACK || R <= 10) ? 2 : 1);
        constexpr int M = PF == 2 ? W + 1 : W;
        float ra[PACK ? 1 : M], rb[PACK ? 1 : M];
        Vec2<ST> rv[PACK ? M : 1];
        // FUSE: ring of (H(phi') I, H(phi')); slices before the volume are
        // the zero padding (the tile starts at z = 0)
        float ha[FUSE ? M : 1], hb[FUSE ? M : 1];
        if constexpr (FUSE) {
#pragma unroll
            for (int j = 0; j < M; ++j) ha[j] = hb[j] = 0.f;
        }
        const gptr<Pair<ST>> tout = glb(static_cast<Pair<ST> *>(d.P));
        const gptr<const IT> imgp = glb(static_cast<const IT *>(d.I));
        if constexpr (!PAPER) {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) {
                const int z = z0 - R + j;
                const Vec2<ST> v = (z >= 0 && z < g.nz) ? pair_at(z) : Vec2<ST>{};
                if constexpr (PACK) {
                    rv[j] = v;
                } else {
                    ra[j] = to_f(v.x);
                    rb[j] = to_f(v.y);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // A stage holds the loads of one step: the phi slice, the conv
        // inputs, the image (PAPER: the force field instead) and the z edge
        // factor.  The loads are unconditional with indices clamped into the
        // volume (a clamped conv input is replaced by the zero padding when
        // it enters the ring), so no load sits under a branch and the wait
        // for the oldest stage leaves the newer one in flight.
        const int zmax = g.nz - 1;
        const gptr<const float> fdp = glb(static_cast<const float *>(d.Q));
        using IRaw = typename std::conditional<PAPER, float, IT>::type;
        const gptr<const IRaw> ip = PAPER ? (gptr<const IRaw>)fdp : (gptr<const IRaw>)img;
        auto iraw = [&](int z) { return bld<IRaw>(rsrc(ip + (int64_t)z * g.sxy), col); };
        const float *const czp = d.cz;   // read once: the loop's stores could alias the table
        struct Stage {
            PhiRaw phi;    // phi slice z + 3
            Vec2<ST> t;    // conv inputs of slice z + R
            IRaw I;        // image (PAPER: F_d) of slice z
            float cz;      // z edge factor of slice z
            IT img;        // FUSE: image of slice z
        };
        // Fast addressing, for tiles of at most 2^29 voxels (every field then
        // lies within 4 GiB of its base): one descriptor per field, built
        // once, and each slice's byte offset as a 32-bit scalar, instead of a
        // 64-bit slice address and a descriptor per access.  The fast steps
        // also need every slice they load in the volume (no clamp, no
        // reflection): the march uses them for whole blocks away from the
        // volume's far end.
        const bool fast = (uint64_t)g.nz * (uint64_t)g.sxy <= ((uint64_t)1 << 29);
        const rsrc_t r_t = rsrc(tp), r_ip = rsrc(ip), r_img = rsrc(imgp);
        constexpr uint32_t kTB = sizeof(Vec2<ST>), kIB = sizeof(IRaw), kMB = sizeof(IT);
        auto stage = [&](auto fastc, int z) {
            constexpr bool F = decltype(fastc)::value;
            Stage st;
            if constexpr (F) {
                st.phi = fetch_phi_fast(z + 3);
                if constexpr (!PAPER)
                    st.t = bld<Vec2<ST>>(r_t, col, (uint32_t)(z + R) * (sxy * kTB));
                st.I = bld<IRaw>(r_ip, col, (uint32_t)z * (sxy * kIB));
                st.cz = PAPER ? 0.f : uniform_ld(czp, z);
                if constexpr (FUSE && PAPER)
                    st.img = bld<IT>(r_img, col, (uint32_t)z * (sxy * kMB));
            } else {
                st.phi = fetch_phi(z + 3);
                if constexpr (!PAPER) st.t = pair_at(min(z + R, zmax));
                st.I = iraw(min(z, zmax));
                st.cz = PAPER ? 0.f : uniform_ld(czp, min(z, zmax));
                // (RSF force: the image of slice z is already st.I)
                if constexpr (FUSE && PAPER)
                    st.img = bld<IT>(rsrc(imgp + (int64_t)min(z, zmax) * g.sxy), col);
            }
            return st;
        };
        using Fast = std::true_type;
        using Slow = std::false_type;
        Stage sa = stage(Slow{}, z0), sb{};
        if constexpr (PF == 2) sb = stage(Slow{}, z0 + 1);
        // FUSE: push (H I, H) of slice z (s its index in the unrolled block)
        // and write the stage-1 z Gaussian of slice z - R, taps in the order
        // of z_heaviside
        const rsrc_t r_tout = rsrc(tout);
        auto emit = [&](auto fastc, const int s, const int z, float hi, float h) {
            if constexpr (FUSE) {
                pin(hi);
                pin(h);
                ha[(s + 2 * R) % M] = hi;
                hb[(s + 2 * R) % M] = h;
                float acc_a = 0.f, acc_b = 0.f;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    acc_a = fmaf(tap<R>(t, k), ha[(s + k) % M], acc_a);
                    acc_b = fmaf(tap<R>(t, k), hb[(s + k) % M], acc_b);
                }
                // 16-bit storage: opaque sums, so that the compiler cannot
                // merge the last FMA with the conversion (one rounding to 16
                // bits) here and not in z_heaviside, or the reverse
                if constexpr (!std::is_same<ST, float>::value) {
                    pin(acc_a);
                    pin(acc_b);
                }
                if (z >= R && zt.active) {
                    if constexpr (decltype(fastc)::value)
                        bst_pair<ST>(r_tout, col, acc_a, acc_b, (uint32_t)(z - R) * (sxy * kTB));
                    else
                        bst_pair<ST>(rsrc(tout + (int64_t)(z - R) * g.sxy), col, acc_a, acc_b);
                }
            }
        };
        // step z (s = its index in the unrolled block) consumes stage `cur`
        // and refills it with the loads of step z + PF
        const rsrc_t r_out = rsrc(phi_out);
        auto step = [&](auto fastc, Stage &cur, const int s, const int z) {
            constexpr bool F = decltype(fastc)::value;
            float Hs = 0.f, HIs = 0.f;   // FUSE: (H(phi'), H(phi') I) of slice z
            store_phi(cur.phi, z + 3);
            if constexpr (!PAPER) {
                const bool in = z + R < g.nz;   // zero padding past the volume
                if constexpr (PACK) {
                    const uint32_t bits = __builtin_bit_cast(uint32_t, cur.t);
                    rv[(s + 2 * R) % M] = __builtin_bit_cast(Vec2<ST>, in ? bits : 0u);
                } else {
                    ra[(s + 2 * R) % M] = in ? to_f(cur.t.x) : 0.f;
                    rb[(s + 2 * R) % M] = in ? to_f(cur.t.y) : 0.f;
                }
            }
            const IRaw I_cur = cur.I;   // PAPER: F_d of slice z
            const float cz_cur = cur.cz;
            IT img_cur{};
            if constexpr (FUSE) {
                if constexpr (PAPER) img_cur = cur.img;
                else img_cur = I_cur;
            }
            cur = stage(fastc, z + PF);
            __syncthreads();
            float nzpp, vzpp;
            q_phase(z + 2, nzpp, vzpp);
            float KG1 = 0.f, KG2 = 0.f;
            if constexpr (!PAPER) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if constexpr (PACK) {
                        KG1 = fmaf(tap<R>(t, k), to_f(rv[(s + k) % M].x), KG1);
                        KG2 = fmaf(tap<R>(t, k), to_f(rv[(s + k) % M].y), KG2);
                    } else {
                        KG1 = fmaf(tap<R>(t, k), ra[(s + k) % M], KG1);
                        KG2 = fmaf(tap<R>(t, k), rb[(s + k) % M], KG2);
                    }
                }
            }
            if (zt.active) {
                const int64_t zo = (int64_t)z * g.sxy;
                const float *p0 = phi_slot(z), *pm = phi_slot(z - 1), *pp = phi_slot(z + 1);
                const int c = (ty + 2) * PX + tx + 2;
                const float cphi = p0[c];
                const float lap = p0[c + 1] + p0[c - 1] + p0[c + PX] + p0[c - PX] + pp[c] + pm[c] -
                                  6.f * cphi;
                const float *q = &sq[(z + 2 * NQ) % NQ][0][0];
                const int o = own_q;
                const float kappa = 0.5f * (q[o + 1] - q[o - 1]) +
                                    0.5f * (q[2 * QS + o + QX] - q[2 * QS + o - QX]) +
                                    0.5f * (nzp - nzm);
                const float divV = 0.5f * (q[QS + o + 1] - q[QS + o - 1]) +
                                   0.5f * (q[3 * QS + o + QX] - q[3 * QS + o - QX]) +
                                   0.5f * (vzp - vzm);
                const float Iv = to_f(I_cur);
                float Fd;
                if constexpr (PAPER) {
                    Fd = Iv;
                } else {
                    const float K1 = cxy * cz_cur;
                    Fd = (ua.l1 - ua.l2) * Iv * Iv * K1 - 2.f * Iv * KG1 + KG2;
                }
                const float Rt = lap + divV;
                const float delta = ua.eps_over_pi * rcp(ua.eps2 + cphi * cphi);
                const float E = ua.mu * Rt + delta * (ua.nu * kappa - Fd);
                const float nxt = cphi + ua.dt * E;
                if constexpr (F) bst<float>(r_out, col, nxt, (uint32_t)z * (sxy * 4u));
                else bst<float>(rsrc(phi_out + zo), col, nxt);
                acc += fabs((double)nxt - (double)cphi);
                if constexpr (FUSE) {
                    Hs = heaviside(nxt, ua.eps);
                    HIs = Hs * to_f(img_cur);
                }
                if (PROBE) {
                    if (d.probe_Fd) (glb(d.probe_Fd) + zo)[col] = Fd;
                    if (d.probe_kappa) (glb(d.probe_kappa) + zo)[col] = kappa;
                    if (d.probe_lap) (glb(d.probe_lap) + zo)[col] = lap;
                    if (d.probe_R) (glb(d.probe_R) + zo)[col] = Rt;
                    if (d.probe_E) (glb(d.probe_E) + zo)[col] = E;
                }
            }
            nzm = nz0; vzm = vz0; nz0 = nzp; vz0 = vzp; nzp = nzpp; vzp = vzpp;
            if constexpr (FUSE) emit(fastc, s, z, HIs, Hs);
        };
        const int zend = zt.z1 + (FUSE ? R : 0);
        int zb = z0;
        // Whole blocks of M steps inside the chunk run with no branch around
        // the steps: a step under a branch ends at a join that copies the
        // stage registers of the skipped path, and that copy waits for every
        // load in flight, prefetches included.  They use fast addressing
        // where the tile allows it and the registers are there (the fused
        // RSF update, with two rings, spills with it), away from the volume's
        // far end: step z loads up to slice z + PF + max(R, 3).
        constexpr bool kFastAddr = !(FUSE && !PAPER);
        constexpr int kAhead = PF + (R > 3 ? R : 3);
        if constexpr (kFastAddr) {
            if (fast) {
                for (; zb + M <= zt.z1 && zb + M + kAhead <= g.nz; zb += M) {
#pragma unroll
                    for (int s = 0; s < M; ++s) {
                        if (PF == 2 && (s & 1)) step(Fast{}, sb, s, zb + s);
                        else step(Fast{}, sa, s, zb + s);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        } else {
            static_assert(PF == 1, "the fused RSF update runs one prefetch stage");
            for (; zb + M <= zt.z1; zb += M) {
#pragma unroll
                for (int s = 0; s < M; ++s) {
                    step(Slow{}, sa, s, zb + s);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        // the rest of the chunk, then (FUSE) the R steps of zero padding
        for (; zb < zend; zb += M) {
#pragma unroll
            for (int s = 0; s < M; ++s) {
                const int z = zb + s;
                if (z < zt.z1) {
                    if (PF == 2 && (s & 1)) step(Slow{}, sb, s, z);
                    else step(Slow{}, sa, s, z);
                } else if (FUSE && z < zend) {
                    emit(Slow{}, s, z, 0.f, 0.f);   // past the volume: the zero padding
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // Block sum of |dphi| in a fixed order: wave tree, then the waves in order.
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) sum += wsum[w];
        glb(d.partials)[wh.lb] = sum;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Per-radius launchers (explicitly instantiated in rsf_inst_*.hip)
// ---------------------------------------------------------------------------

template <int R, class IT, class ST>
hipError_t launch_xy_r(int mode, const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                       bool, hipStream_t s)
{
    const dim3 grid((unsigned)blocks);
    switch (mode) {
    case XY_ONE:
        hipLaunchKernelGGL((xy_kernel<R, XY_ONE, IT, ST>), grid, dim3(64), 0, s, b, t, c);
        break;
    case XY_TWO:
        hipLaunchKernelGGL((xy_kernel<R, XY_TWO, ST, ST>), grid, dim3(64), 0, s, b, t, c);
        break;
    case XY_FITS:
        hipLaunchKernelGGL((xy_kernel<R, XY_FITS, ST, ST>), grid, dim3(64), 0, s, b, t, c);
        break;
    case XY_PAPER:
        hipLaunchKernelGGL((xy_kernel<R, XY_PAPER, ST, ST, IT>), grid, dim3(64), 0, s, b, t, c);
        break;
    case XY_PAPER2:
        hipLaunchKernelGGL((xy_kernel<R, XY_PAPER2, ST, ST, IT>), grid, dim3(64), 0, s, b, t, c);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R, class ST>
hipError_t launch_z_plain_r(const Batch &b, int64_t blocks, const Taps &t, int target,
                            hipStream_t s)
{
    hipLaunchKernelGGL((z_plain_kernel<R, ST>), dim3((unsigned)blocks), dim3(kThreads), 0, s, b, t,
                       target);
    return hipGetLastError();
}

template <int R, class IT, class ST>
hipError_t launch_z_heaviside_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                                bool probe, hipStream_t s)
{
    const dim3 grid((unsigned)blocks);
    if (probe)
        hipLaunchKernelGGL((z_heaviside_kernel<R, true, ST, IT>), grid, dim3(kThreads), 0, s, b, t,
                           c);
    else
        hipLaunchKernelGGL((z_heaviside_kernel<R, false, ST, IT>), grid, dim3(kThreads), 0, s, b, t,
                           c);
    return hipGetLastError();
}

template <int R, class IT, class ST>
hipError_t launch_z_update_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                             bool probe, hipStream_t s)
{
    const dim3 grid((unsigned)blocks);
    if (probe)
        hipLaunchKernelGGL((z_update_kernel<R, true, ST, IT>), grid, dim3(kUThreads), 0, s, b, t,
                           c);
    else
        hipLaunchKernelGGL((z_update_kernel<R, false, ST, IT>), grid, dim3(kUThreads), 0, s, b, t,
                           c);
    return hipGetLastError();
}

// The update of the Sec. 4.2 force (sigma2 = 0): one instance per type pair.
template <class IT, class ST>
hipError_t launch_z_update_paper_r(const Batch &b, int64_t blocks, const Coeffs &c, bool probe,
                                   hipStream_t s)
{
    const dim3 grid((unsigned)blocks);
    const Taps t{};
    if (probe)
        hipLaunchKernelGGL((z_update_kernel<1, true, ST, IT, true>), grid, dim3(kUThreads), 0, s,
                           b, t, c);
    else
        hipLaunchKernelGGL((z_update_kernel<1, false, ST, IT, true>), grid, dim3(kUThreads), 0, s,
                           b, t, c);
    return hipGetLastError();
}

template <int R, class IT, class ST>
hipError_t launch_z_update_fused_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                                   bool paper, hipStream_t s)
{
    // RSF force: larger radii spill and keep the separate passes
    if (paper) {
        hipLaunchKernelGGL((z_update_kernel<R, false, ST, IT, true, true>), dim3((unsigned)blocks),
                           dim3(kUThreads), 0, s, b, t, c);
    } else {
        if constexpr (R > fuse_max_r_t<ST, IT>) return hipErrorInvalidValue;
        else
            hipLaunchKernelGGL((z_update_kernel<R, false, ST, IT, false, true>),
                               dim3((unsigned)blocks), dim3(kUThreads), 0, s, b, t, c);
    }
    return hipGetLastError();
}

#define RSF_INSTANTIATE_PAPER(IT, ST)                                                      \
    template hipError_t launch_z_update_paper_r<IT, ST>(const Batch &, int64_t, const Coeffs &, \
                                                        bool, hipStream_t);

// Instantiate every pass launcher for radius RR, image type IT, storage ST.
#define RSF_INSTANTIATE(RR, IT, ST)                                                           \
    template hipError_t launch_xy_r<RR, IT, ST>(int, const Batch &, int64_t, const Taps &,    \
                                                const Coeffs &, bool, hipStream_t);           \
    template hipError_t launch_z_plain_r<RR, ST>(const Batch &, int64_t, const Taps &, int,   \
                                                 hipStream_t);                                \
    template hipError_t launch_z_heaviside_r<RR, IT, ST>(const Batch &, int64_t, const Taps &, \
                                                         const Coeffs &, bool, hipStream_t);  \
    template hipError_t launch_z_update_r<RR, IT, ST>(const Batch &, int64_t, const Taps &,   \
                                                      const Coeffs &, bool, hipStream_t);     \
    template hipError_t launch_z_update_fused_r<RR, IT, ST>(const Batch &, int64_t,           \
                                                            const Taps &, const Coeffs &,     \
                                                            bool, hipStream_t);

}  // namespace rsf
