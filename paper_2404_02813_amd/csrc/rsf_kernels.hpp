// Device templates of the RSF passes (xy and z Gaussian passes with their
// epilogues) and their per-radius launchers.  Included by the translation
// units that instantiate them for a range of radii (rsf_inst_*.hip).
#pragma once

#include "rsf_internal.hpp"

namespace rsf {

namespace {


constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kTwoPi = 6.28318530717958647693f;
constexpr int kXcds = 8;

__device__ __forceinline__ float heaviside(float phi, float eps)
{
    // 1/2 (1 + (2/pi) atan(phi/eps)) written as atan2(eps, -phi)/pi, which
    // keeps full relative precision for large negative phi.
    return atan2f(eps, -phi) * kInvPi;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int reflect(int i, int n)
{
    return i < 0 ? -i : (i > n - 1 ? 2 * (n - 1) - i : i);
}

// Workgroup b runs on XCD b % 8.  Give XCD k the contiguous tile range
// [k*per + min(k, rem), ...) so spatial neighbours share an L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int per = n / kXcds, rem = n % kXcds;
    const int x = b % kXcds, local = b / kXcds;
    return x * per + min(x, rem) + local;
}

// ---------------------------------------------------------------------------
// xy pass: LDS tile (kXyTy + 2R) rows x (kXyTx + 2HL) columns (HL = R rounded
// up to 4 so rows load as float4), x convolution into registers, back to
// LDS, y convolution, then the mode's epilogue and a coalesced store.
// ---------------------------------------------------------------------------

template <int R, int MODE>
__global__ __launch_bounds__(kThreads) void xy_kernel(const float *__restrict__ a,
                                                      const float *__restrict__ b,
                                                      float *__restrict__ oa,
                                                      float *__restrict__ ob, Grid3 g, Taps t,
                                                      FitArgs fa, const int *__restrict__ done)
{
    if (done && *done) return;
    constexpr int NF = MODE == XY_ONE ? 1 : 2;
    constexpr int TX = kXyTx, TY = kXyTy;
    constexpr int HL = 4 * ((R + 3) / 4);
    constexpr int LW = TX + 2 * HL;          // loaded columns
    constexpr int PITCH = LW + 4;            // + one float4 the x windows may over-read
    constexpr int OFF = HL - R;
    constexpr int ROWS = TY + 2 * R;
    constexpr int W = 2 * R + 1;
    constexpr int NQ = LW / 4;
    __shared__ __align__(16) float s[NF][ROWS][PITCH];

    const int nbx = (g.nx + TX - 1) / TX, nby = (g.ny + TY - 1) / TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bxi = tile % nbx, rest = tile / nbx;
    const int x0 = bxi * TX, y0 = (rest % nby) * TY, z = rest / nby;
    const int64_t zb = (int64_t)z * g.sxy;
    const int tid = threadIdx.x;
    const bool vec = (g.nx & 3) == 0;

    for (int i = tid; i < ROWS * NQ; i += kThreads) {
        const int r = i / NQ, q = i - r * NQ;
        const int gy = y0 + r - R;
        const int gx = x0 - HL + 4 * q;
        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
        if (gy >= 0 && gy < g.ny) {
            const float *ra = a + zb + (int64_t)gy * g.nx;
            const float *rb = NF == 2 ? b + zb + (int64_t)gy * g.nx : nullptr;
            if (vec && gx >= 0 && gx + 3 < g.nx) {
                va = *reinterpret_cast<const float4 *>(ra + gx);
                if (NF == 2) vb = *reinterpret_cast<const float4 *>(rb + gx);
            } else {
                float ea[4] = {0.f, 0.f, 0.f, 0.f}, eb[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int xx = gx + e;
                    if (xx >= 0 && xx < g.nx) {
                        ea[e] = ra[xx];
                        if (NF == 2) eb[e] = rb[xx];
                    }
                }
                va = make_float4(ea[0], ea[1], ea[2], ea[3]);
                vb = make_float4(eb[0], eb[1], eb[2], eb[3]);
            }
        }
        *reinterpret_cast<float4 *>(&s[0][r][4 * q]) = va;
        if (NF == 2) *reinterpret_cast<float4 *>(&s[NF - 1][r][4 * q]) = vb;
    }
    __syncthreads();

    // x convolution: each lane makes 4 consecutive outputs of one row from a
    // window read with 16-byte LDS loads.
    const int lane = tid & 63, wave = tid >> 6;
    const int xg = lane & 15, rsub = lane >> 4;
    constexpr int NPASS = (ROWS + 15) / 16;
    constexpr int NV = (OFF + 4 + 2 * R + 3) / 4;
    float xr[NF][NPASS][4];
#pragma unroll
    for (int j = 0; j < NPASS; ++j) {
        const int r = wave * 4 + rsub + 16 * j;
        if (r < ROWS) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                float win[4 * NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const float4 q = *reinterpret_cast<const float4 *>(&s[f][r][4 * xg + 4 * v]);
                    win[4 * v + 0] = q.x;
                    win[4 * v + 1] = q.y;
                    win[4 * v + 2] = q.z;
                    win[4 * v + 3] = q.w;
                }
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < W; ++k) acc = fmaf(t.w[k], win[OFF + o + k], acc);
                    xr[f][j][o] = acc;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NPASS; ++j) {
        const int r = wave * 4 + rsub + 16 * j;
        if (r < ROWS) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                *reinterpret_cast<float4 *>(&s[f][r][4 * xg]) =
                    make_float4(xr[f][j][0], xr[f][j][1], xr[f][j][2], xr[f][j][3]);
        }
    }
    __syncthreads();

    // y convolution: lane = column, each wave makes TY/4 consecutive rows.
    constexpr int RPW = TY / 4;
    const int gx = x0 + lane;
    const int rbase = wave * RPW;
    float wa[RPW + 2 * R], wb[RPW + 2 * R];
#pragma unroll
    for (int i = 0; i < RPW + 2 * R; ++i) {
        wa[i] = s[0][rbase + i][lane];
        if (NF == 2) wb[i] = s[NF - 1][rbase + i][lane];
    }
    float cxv = 0.f;
    if (MODE == XY_FITS && gx < g.nx) cxv = fa.cx[gx] * fa.cz[z];
#pragma unroll
    for (int o = 0; o < RPW; ++o) {
        float acc_a = 0.f, acc_b = 0.f;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            acc_a = fmaf(t.w[k], wa[o + k], acc_a);
            if (NF == 2) acc_b = fmaf(t.w[k], wb[o + k], acc_b);
        }
        const int gy = y0 + rbase + o;
        if (gx < g.nx && gy < g.ny) {
            const int64_t v = zb + (int64_t)gy * g.nx + gx;
            if (MODE == XY_FITS) {
                // region fits (Sec. 3 local_intensity) and force-convolution inputs
                const float K1 = cxv * fa.cy[gy];
                const float A2 = fa.KI[v] - acc_a;
                const float B2 = K1 - acc_b;
                const float f1 = acc_a * rcp(acc_b);
                const float f2 = A2 * rcp(B2);
                oa[v] = fa.l1 * f1 - fa.l2 * f2;
                ob[v] = fa.l1 * f1 * f1 - fa.l2 * f2 * f2;
                if (fa.probe_f1) fa.probe_f1[v] = f1;
                if (fa.probe_f2) fa.probe_f2[v] = f2;
            } else {
                oa[v] = acc_a;
                if (NF == 2) ob[v] = acc_b;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// z passes: a thread owns column (x, y) and marches z0..z1 with a ring of the
// 2R+1 slices around z held in registers.  The ring is indexed with
// compile-time slots by unrolling the march in steps of 2R+1.
// ---------------------------------------------------------------------------

struct ZTile {
    int x, y, z0, z1, tile;
    bool active;
};

// Tiles are (kZx x kZy columns) x (one z chunk), z chunk fastest.
__device__ __forceinline__ ZTile z_tile(const Grid3 &g, int nzc)
{
    ZTile zt;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nbx = (g.nx + kZx - 1) / kZx;
    const int zc = tile % nzc, col = tile / nzc;
    const int lz = (g.nz + nzc - 1) / nzc;
    zt.x = (col % nbx) * kZx + (threadIdx.x & (kZx - 1));
    zt.y = (col / nbx) * kZy + (threadIdx.x / kZx);
    zt.z0 = zc * lz;
    zt.z1 = min(zt.z0 + lz, g.nz);
    zt.tile = tile;
    zt.active = zt.x < g.nx && zt.y < g.ny;
    return zt;
}

// Conv ring: ld(z) returns slice z (0 <= z < nz) of the two inputs.
template <int R, int NF, typename Ld, typename Epi>
__device__ __forceinline__ void z_march(int nz, int z0, int z1, const Taps &t, Ld &&ld,
                                        Epi &&epi)
{
    constexpr int W = 2 * R + 1;
    float ra[W], rb[W];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        const int z = z0 - R + j;
        const float2 v = (z >= 0 && z < nz) ? ld(z) : make_float2(0.f, 0.f);
        ra[j] = v.x;
        rb[j] = v.y;
    }
    for (int zb = z0; zb < z1; zb += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int z = zb + s;
            if (z < z1) {
                const int zn = z + R;
                const float2 v = zn < nz ? ld(zn) : make_float2(0.f, 0.f);
                ra[(s + 2 * R) % W] = v.x;
                rb[(s + 2 * R) % W] = v.y;
                float acc_a = 0.f, acc_b = 0.f;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    acc_a = fmaf(t.w[k], ra[(s + k) % W], acc_a);
                    if (NF == 2) acc_b = fmaf(t.w[k], rb[(s + k) % W], acc_b);
                }
                epi(z, acc_a, acc_b);
            }
            // keep each step's loads and math inside the step: occupancy,
            // not hoisting, hides the latency
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int R>
__global__ __launch_bounds__(kThreads) void z_plain_kernel(const float *__restrict__ in,
                                                           float *__restrict__ out, Grid3 g,
                                                           Taps t, int nzc)
{
    const ZTile zt = z_tile(g, nzc);
    if (!zt.active) return;
    const int64_t col = (int64_t)zt.y * g.nx + zt.x;
    z_march<R, 1>(
        g.nz, zt.z0, zt.z1, t,
        [&](int z) { return make_float2(in[col + (int64_t)z * g.sxy], 0.f); },
        [&](int z, float va, float) { out[col + (int64_t)z * g.sxy] = va; });
}

// Stage-1 z pass: H_eps(phi) and H I formed as slices enter the ring.
template <int R, bool PROBE>
__global__ __launch_bounds__(kThreads) void z_heaviside_kernel(
    const float *__restrict__ phi, const float *__restrict__ I, float *__restrict__ t1,
    float *__restrict__ t2, Grid3 g, Taps t, float eps, float *__restrict__ probeH, int nzc,
    const int *__restrict__ done)
{
    if (done && *done) return;
    const ZTile zt = z_tile(g, nzc);
    if (!zt.active) return;
    const int64_t col = (int64_t)zt.y * g.nx + zt.x;
    z_march<R, 2>(
        g.nz, zt.z0, zt.z1, t,
        [&](int z) {
            const int64_t v = col + (int64_t)z * g.sxy;
            const float H = heaviside(phi[v], eps);
            if (PROBE && probeH) probeH[v] = H;
            return make_float2(H * I[v], H);
        },
        [&](int z, float va, float vb) {
            const int64_t v = col + (int64_t)z * g.sxy;
            t1[v] = va;
            t2[v] = vb;
        });
}

// Diffusion-rate excess D(s) = d_p(s) - 1 of the distance regulariser.
// v_sin_f32 takes its argument in turns, so it returns sin(2 pi s).
__device__ __forceinline__ float reg_rate(float s, float s_eta, int reg)
{
    if (reg != 0) return -rcp(s_eta);                       // single well
    const float dw = __builtin_amdgcn_sinf(s) * rcp(kTwoPi * s) - 1.f;
    return s > 1.f ? -rcp(s) : (s > 0.f ? dw : 0.f);
}

// Stage-2 z pass with the update.  The block's tile is kZx x kZy columns.
// Alongside the per-thread conv ring it keeps in LDS a ring of phi slices
// (tile + 2 halo, 5 slots) and, per slice, the x/y components of the unit
// normal n and of the regulariser flux V = D(|grad phi|) grad phi at the tile
// + 1 halo (2 slots); the z components of the thread's own column stay in
// registers.  Each point's gradient, n and V are computed once and shared by
// the six neighbours whose divergence needs them.
template <int R, bool PROBE>
__global__ __launch_bounds__(kThreads) void z_update_kernel(const float *__restrict__ t1,
                                                            const float *__restrict__ t2,
                                                            Grid3 g, Taps t, UpdArgs ua,
                                                            int nzc, const int *__restrict__ done)
{
    constexpr int TX = kZx, TY = kZy;
    constexpr int PX = TX + 4, PY = TY + 4;
    constexpr int QX = TX + 2, QY = TY + 2;
    constexpr int NSLOT = 5;
    constexpr int NLD = (PX * PY + kThreads - 1) / kThreads;
    __shared__ float sphi[NSLOT][PY * PX];
    __shared__ float sq[2][4][QY * QX];   // n_x, V_x, n_y, V_y
    __shared__ double wsum[kThreads / 64];

    const ZTile zt = z_tile(g, nzc);
    const int tid = threadIdx.x;
    const int tx = tid & (TX - 1), ty = tid / TX;
    const int x0 = zt.x - tx, y0 = zt.y - ty;
    const bool stopped = done && *done;
    const float *__restrict__ phi = ua.phi;
    double acc = 0.0;

    if (stopped) {
        if (zt.active) {
            const int64_t col = (int64_t)zt.y * g.nx + zt.x;
            for (int z = zt.z0; z < zt.z1; ++z)
                ua.phi_out[col + (int64_t)z * g.sxy] = phi[col + (int64_t)z * g.sxy];
        }
    } else {
        // phi tile loads: reflected in-slice offsets of this thread's points
        int loff[NLD];
        bool lok[NLD];
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int i = tid + r * kThreads;
            lok[r] = i < PX * PY;
            const int px = i % PX, py = i / PX;
            const int gx = reflect(min(x0 - 2 + px, g.nx + 1), g.nx);
            const int gy = reflect(min(y0 - 2 + py, g.ny + 1), g.ny);
            loff[r] = gy * g.nx + gx;
        }
        auto load_phi = [&](int j) {
            const float *base = phi + (int64_t)reflect(j, g.nz) * g.sxy;
            float *dst = sphi[(j + 2 * NSLOT) % NSLOT];
#pragma unroll
            for (int r = 0; r < NLD; ++r)
                if (lok[r]) dst[tid + r * kThreads] = base[loff[r]];
        };
        // n and V at phi-tile point (cx, cy) of slice j
        auto qcalc = [&](int j, int cx, int cy, float &nx_, float &vx_, float &ny_, float &vy_,
                         float &nz_, float &vz_) {
            const float *p0 = sphi[(j + 2 * NSLOT) % NSLOT];
            const float *pm = sphi[(j - 1 + 2 * NSLOT) % NSLOT];
            const float *pp = sphi[(j + 1 + 2 * NSLOT) % NSLOT];
            const int c = cy * PX + cx;
            const float gx = 0.5f * (p0[c + 1] - p0[c - 1]);
            const float gy = 0.5f * (p0[c + PX] - p0[c - PX]);
            const float gz = 0.5f * (pp[c] - pm[c]);
            const float s2 = gx * gx + gy * gy + gz * gz;
            const float s_eta = __builtin_amdgcn_sqrtf(s2 + ua.eta);
            const float inv = rcp(s_eta);
            const float D = reg_rate(__builtin_amdgcn_sqrtf(s2), s_eta, ua.reg);
            nx_ = gx * inv; ny_ = gy * inv; nz_ = gz * inv;
            vx_ = D * gx; vy_ = D * gy; vz_ = D * gz;
        };
        // halo points of the normal/flux tile: y halo rows (threads 0..127),
        // x halo columns (threads 128..135)
        int hq = -1;
        if (tid < 2 * TX) hq = (tid < TX ? 0 : QY - 1) * QX + (tid % TX) + 1;
        else if (tid < 2 * TX + 2 * TY) {
            const int k = tid - 2 * TX;
            hq = (k % TY + 1) * QX + (k < TY ? 0 : QX - 1);
        }
        const int own_q = (ty + 1) * QX + tx + 1;
        float nzm = 0.f, vzm = 0.f, nz0 = 0.f, vz0 = 0.f, nzp = 0.f, vzp = 0.f;
        auto q_phase = [&](int j) {
            float qnx, qvx, qny, qvy, qnz, qvz;
            qcalc(j, tx + 2, ty + 2, qnx, qvx, qny, qvy, qnz, qvz);
            float *q = &sq[j & 1][0][0];
            q[0 * QY * QX + own_q] = qnx;
            q[1 * QY * QX + own_q] = qvx;
            q[2 * QY * QX + own_q] = qny;
            q[3 * QY * QX + own_q] = qvy;
            nzm = nz0; vzm = vz0; nz0 = nzp; vz0 = vzp; nzp = qnz; vzp = qvz;
            if (hq >= 0) {
                float a0, a1, a2, a3, a4, a5;
                qcalc(j, hq % QX + 1, hq / QX + 1, a0, a1, a2, a3, a4, a5);
                q[0 * QY * QX + hq] = a0;
                q[1 * QY * QX + hq] = a1;
                q[2 * QY * QX + hq] = a2;
                q[3 * QY * QX + hq] = a3;
            }
        };

        const int64_t col = (int64_t)min(zt.y, g.ny - 1) * g.nx + min(zt.x, g.nx - 1);
        const float cxy = ua.cx[min(zt.x, g.nx - 1)] * ua.cy[min(zt.y, g.ny - 1)];
        load_phi(zt.z0 - 2);
        load_phi(zt.z0 - 1);
        for (int j = zt.z0 - 2; j < zt.z0; ++j) {
            load_phi(j + 2);
            __syncthreads();
            q_phase(j + 1);
            __syncthreads();
        }

        constexpr int W = 2 * R + 1;
        float ra[W], rb[W];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            const int z = zt.z0 - R + j;
            const bool ok = z >= 0 && z < g.nz;
            ra[j] = ok ? t1[col + (int64_t)z * g.sxy] : 0.f;
            rb[j] = ok ? t2[col + (int64_t)z * g.sxy] : 0.f;
        }
        for (int zb = zt.z0; zb < zt.z1; zb += W) {
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const int z = zb + s;
                if (z < zt.z1) {
                    load_phi(z + 2);
                    const int zn = z + R;
                    const bool ok = zn < g.nz;
                    ra[(s + 2 * R) % W] = ok ? t1[col + (int64_t)zn * g.sxy] : 0.f;
                    rb[(s + 2 * R) % W] = ok ? t2[col + (int64_t)zn * g.sxy] : 0.f;
                    __syncthreads();
                    q_phase(z + 1);
                    __syncthreads();
                    float KG1 = 0.f, KG2 = 0.f;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        KG1 = fmaf(t.w[k], ra[(s + k) % W], KG1);
                        KG2 = fmaf(t.w[k], rb[(s + k) % W], KG2);
                    }
                    if (zt.active) {
                        const int64_t v = col + (int64_t)z * g.sxy;
                        const float *p0 = sphi[(z + 2 * NSLOT) % NSLOT];
                        const float *pm = sphi[(z - 1 + 2 * NSLOT) % NSLOT];
                        const float *pp = sphi[(z + 1 + 2 * NSLOT) % NSLOT];
                        const int c = (ty + 2) * PX + tx + 2;
                        const float cphi = p0[c];
                        const float lap = p0[c + 1] + p0[c - 1] + p0[c + PX] + p0[c - PX] +
                                          pp[c] + pm[c] - 6.f * cphi;
                        const float *q = &sq[z & 1][0][0];
                        const int o = own_q;
                        const float kappa = 0.5f * (q[o + 1] - q[o - 1]) +
                                            0.5f * (q[2 * QY * QX + o + QX] - q[2 * QY * QX + o - QX]) +
                                            0.5f * (nzp - nzm);
                        const float divV = 0.5f * (q[QY * QX + o + 1] - q[QY * QX + o - 1]) +
                                           0.5f * (q[3 * QY * QX + o + QX] - q[3 * QY * QX + o - QX]) +
                                           0.5f * (vzp - vzm);
                        const float Iv = ua.I[v];
                        const float K1 = cxy * ua.cz[z];
                        const float Fd = (ua.l1 - ua.l2) * Iv * Iv * K1 - 2.f * Iv * KG1 + KG2;
                        const float Rt = lap + divV;
                        const float delta = ua.eps_over_pi * rcp(ua.eps2 + cphi * cphi);
                        const float E = ua.mu * Rt + delta * (ua.nu * kappa - Fd);
                        const float nxt = cphi + ua.dt * E;
                        ua.phi_out[v] = nxt;
                        acc += fabs((double)nxt - (double)cphi);
                        if (PROBE) {
                            if (ua.probe_Fd) ua.probe_Fd[v] = Fd;
                            if (ua.probe_kappa) ua.probe_kappa[v] = kappa;
                            if (ua.probe_lap) ua.probe_lap[v] = lap;
                            if (ua.probe_R) ua.probe_R[v] = Rt;
                            if (ua.probe_E) ua.probe_E[v] = E;
                        }
                    }
                }
            }
        }
    }
    // Block sum of |dphi| in a fixed order: wave tree, then the four waves.
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (tid == 0) ua.partials[zt.tile] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

}  // namespace

// ---------------------------------------------------------------------------
// Per-radius launchers (explicitly instantiated in rsf_inst_*.hip)
// ---------------------------------------------------------------------------

template <int R>
hipError_t launch_xy_r(int mode, const float *a, const float *b, float *oa, float *ob, Grid3 g,
                       const Taps &t, const FitArgs *fa, const int *done, hipStream_t s)
{
    const dim3 grid(xy_blocks(g));
    const FitArgs f = fa ? *fa : FitArgs{};
    switch (mode) {
    case XY_ONE:
        hipLaunchKernelGGL((xy_kernel<R, XY_ONE>), grid, dim3(kThreads), 0, s, a, b, oa, ob, g, t,
                           f, done);
        break;
    case XY_TWO:
        hipLaunchKernelGGL((xy_kernel<R, XY_TWO>), grid, dim3(kThreads), 0, s, a, b, oa, ob, g, t,
                           f, done);
        break;
    case XY_FITS:
        hipLaunchKernelGGL((xy_kernel<R, XY_FITS>), grid, dim3(kThreads), 0, s, a, b, oa, ob, g,
                           t, f, done);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R>
hipError_t launch_z_plain_r(const float *in, float *out, Grid3 g, const Taps &t, hipStream_t s)
{
    hipLaunchKernelGGL((z_plain_kernel<R>), dim3((unsigned)z_blocks(g)), dim3(kThreads), 0, s, in,
                       out, g, t, z_chunks(g));
    return hipGetLastError();
}

template <int R>
hipError_t launch_z_heaviside_r(const float *phi, const float *I, float *t1, float *t2, Grid3 g,
                                const Taps &t, float eps, float *probeH, const int *done,
                                hipStream_t s)
{
    const dim3 grid((unsigned)z_blocks(g));
    if (probeH)
        hipLaunchKernelGGL((z_heaviside_kernel<R, true>), grid, dim3(kThreads), 0, s, phi, I, t1,
                           t2, g, t, eps, probeH, z_chunks(g), done);
    else
        hipLaunchKernelGGL((z_heaviside_kernel<R, false>), grid, dim3(kThreads), 0, s, phi, I, t1,
                           t2, g, t, eps, probeH, z_chunks(g), done);
    return hipGetLastError();
}

template <int R>
hipError_t launch_z_update_r(const float *t1, const float *t2, Grid3 g, const Taps &t,
                             const UpdArgs &ua, const int *done, hipStream_t s)
{
    const dim3 grid((unsigned)z_blocks(g));
    const bool probe = ua.probe_Fd || ua.probe_kappa || ua.probe_lap || ua.probe_R || ua.probe_E;
    if (probe)
        hipLaunchKernelGGL((z_update_kernel<R, true>), grid, dim3(kThreads), 0, s, t1, t2, g, t, ua,
                           z_chunks(g), done);
    else
        hipLaunchKernelGGL((z_update_kernel<R, false>), grid, dim3(kThreads), 0, s, t1, t2, g, t,
                           ua, z_chunks(g), done);
    return hipGetLastError();
}

#define RSF_INSTANTIATE(RR)                                                                     \
    template hipError_t launch_xy_r<RR>(int, const float *, const float *, float *, float *,    \
                                        Grid3, const Taps &, const FitArgs *, const int *,      \
                                        hipStream_t);                                           \
    template hipError_t launch_z_plain_r<RR>(const float *, float *, Grid3, const Taps &,       \
                                             hipStream_t);                                      \
    template hipError_t launch_z_heaviside_r<RR>(const float *, const float *, float *, float *, \
                                                 Grid3, const Taps &, float, float *,           \
                                                 const int *, hipStream_t);                     \
    template hipError_t launch_z_update_r<RR>(const float *, const float *, Grid3, const Taps &, \
                                              const UpdArgs &, const int *, hipStream_t);

}  // namespace rsf
