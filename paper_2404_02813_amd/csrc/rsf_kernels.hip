// HIP kernels (gfx950) of one RSF level-set iteration.
//
// One iteration = four bandwidth-bound passes plus a tiny reduction:
//   xy(H)   : (phi, I) -> Kxy*(H I), Kxy*H          H = H_eps(phi)   (Sec. 3)
//   z(fits) : -> f1 = K*(HI)/K*H, f2 = (K*I - K*(HI))/(K*1 - K*H),
//             g1 = l1 f1 - l2 f2, g2 = l1 f1^2 - l2 f2^2            (Sec. 3)
//   xy(two) : (g1, g2) -> Kxy*g1, Kxy*g2
//   z(upd)  : Fd = (l1-l2) I^2 K*1 - 2 I K*g1 + K*g2 = l1 e1 - l2 e2,
//             curvature, regulariser, Dirac-weighted explicit update  (Sec. 2-3)
//             and per-block FP64 partial sums of |phi' - phi|
//   reduce  : fixed-order FP64 sum of the partials.
// The Gaussian K is separable and applied as an xy pass (LDS tile with an R
// halo, x then y) and a z pass (each thread marches one (x, y) column through
// a z chunk with a register ring of 2R+1 slices), so every global access is
// coalesced along x.  Linearity gives the two missing stage-1 convolutions
// (K*((1-H)I) = K*I - K*(HI), K*(1-H) = K*1 - K*H) and folds e1, e2 into two
// convolutions (of g1 and g2).
#include "rsf_internal.hpp"

namespace rsf {

namespace {

constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kTwoPi = 6.28318530717958647693f;

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

// ---------------------------------------------------------------------------
// xy pass: LDS tile (kXyTy + 2R) x (kXyTx + 2R), x convolution into registers,
// back to LDS, y convolution, coalesced store.
// ---------------------------------------------------------------------------

template <int R, int MODE>
__global__ __launch_bounds__(kThreads) void xy_kernel(const float *__restrict__ a,
                                                      const float *__restrict__ b,
                                                      float *__restrict__ oa,
                                                      float *__restrict__ ob, Grid3 g, Taps t,
                                                      float eps, float *__restrict__ probeH,
                                                      const int *__restrict__ done)
{
    if (done && *done) return;
    constexpr int NF = MODE == XY_ONE ? 1 : 2;
    constexpr int TX = kXyTx, TY = kXyTy;
    constexpr int IW = TX + 2 * R;
    constexpr int ROWS = TY + 2 * R;
    constexpr int PITCH = (IW + 3) & ~3;
    constexpr int W = 2 * R + 1;
    __shared__ __align__(16) float s[NF][ROWS][PITCH];

    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int64_t zb = (int64_t)blockIdx.z * g.sxy;
    const int tid = threadIdx.x;

    for (int i = tid; i < ROWS * IW; i += kThreads) {
        const int r = i / IW, c = i - r * IW;
        const int gx = x0 + c - R, gy = y0 + r - R;
        float va = 0.f, vb = 0.f;
        if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny) {
            const int64_t gi = zb + (int64_t)gy * g.nx + gx;
            if (MODE == XY_HEAVISIDE) {
                const float H = heaviside(a[gi], eps);
                va = H * b[gi];
                vb = H;
                if (probeH && r >= R && r < R + TY && c >= R && c < R + TX) probeH[gi] = H;
            } else {
                va = a[gi];
                if (NF == 2) vb = b[gi];
            }
        }
        s[0][r][c] = va;
        if (NF == 2) s[NF - 1][r][c] = vb;
    }
    __syncthreads();

    // x convolution: each lane makes 4 consecutive outputs of one row from a
    // window read with 16-byte LDS loads.
    const int lane = tid & 63, wave = tid >> 6;
    const int xg = lane & 15, rsub = lane >> 4;
    constexpr int NPASS = (ROWS + 15) / 16;
    constexpr int NV = (4 + 2 * R + 3) / 4;
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
                    for (int k = 0; k < W; ++k) acc = fmaf(t.w[k], win[o + k], acc);
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
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        float win[RPW + 2 * R];
#pragma unroll
        for (int i = 0; i < RPW + 2 * R; ++i) win[i] = s[f][rbase + i][lane];
        float *dst = f == 0 ? oa : ob;
#pragma unroll
        for (int o = 0; o < RPW; ++o) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < W; ++k) acc = fmaf(t.w[k], win[o + k], acc);
            const int gy = y0 + rbase + o;
            if (gx < g.nx && gy < g.ny) dst[zb + (int64_t)gy * g.nx + gx] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// z pass: a thread owns column (x, y) and marches z0..z1 with a ring of the
// 2R+1 slices around z held in registers.  The ring is indexed with
// compile-time slots by unrolling the march in steps of 2R+1.
// ---------------------------------------------------------------------------

template <int R, int NF, typename Epi>
__device__ __forceinline__ void z_march(const float *__restrict__ a, const float *__restrict__ b,
                                        int64_t col, int64_t sxy, int nz, int z0, int z1,
                                        const Taps &t, Epi &&epi)
{
    constexpr int W = 2 * R + 1;
    float ra[W], rb[W];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        const int z = z0 - R + j;
        const bool ok = z >= 0 && z < nz;
        ra[j] = ok ? a[col + (int64_t)z * sxy] : 0.f;
        if (NF == 2) rb[j] = ok ? b[col + (int64_t)z * sxy] : 0.f;
    }
    for (int zb = z0; zb < z1; zb += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int z = zb + s;
            if (z < z1) {
                const int zn = z + R;
                const bool ok = zn < nz;
                ra[(s + 2 * R) % W] = ok ? a[col + (int64_t)zn * sxy] : 0.f;
                if (NF == 2) rb[(s + 2 * R) % W] = ok ? b[col + (int64_t)zn * sxy] : 0.f;
                float acc_a = 0.f, acc_b = 0.f;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    acc_a = fmaf(t.w[k], ra[(s + k) % W], acc_a);
                    if (NF == 2) acc_b = fmaf(t.w[k], rb[(s + k) % W], acc_b);
                }
                epi(z, acc_a, acc_b);
            }
        }
    }
}

struct ZSpan {
    int x, y, z0, z1;
    bool active;
};

__device__ __forceinline__ ZSpan z_span(const Grid3 &g)
{
    ZSpan sp;
    sp.x = blockIdx.x * kZx + (threadIdx.x & (kZx - 1));
    sp.y = blockIdx.y * kZy + (threadIdx.x / kZx);
    const int lz = (g.nz + gridDim.z - 1) / gridDim.z;
    sp.z0 = blockIdx.z * lz;
    sp.z1 = min(sp.z0 + lz, g.nz);
    sp.active = sp.x < g.nx && sp.y < g.ny;
    return sp;
}

template <int R>
__global__ __launch_bounds__(kThreads) void z_plain_kernel(const float *__restrict__ in,
                                                           float *__restrict__ out, Grid3 g,
                                                           Taps t)
{
    const ZSpan sp = z_span(g);
    if (!sp.active) return;
    const int64_t col = (int64_t)sp.y * g.nx + sp.x;
    z_march<R, 1>(in, nullptr, col, g.sxy, g.nz, sp.z0, sp.z1, t,
                  [&](int z, float va, float) { out[col + (int64_t)z * g.sxy] = va; });
}

template <int R, bool PROBE>
__global__ __launch_bounds__(kThreads) void z_fits_kernel(const float *__restrict__ t1,
                                                          const float *__restrict__ t2,
                                                          float *__restrict__ g1,
                                                          float *__restrict__ g2, Grid3 g,
                                                          Taps t, FitArgs fa,
                                                          const int *__restrict__ done)
{
    if (done && *done) return;
    const ZSpan sp = z_span(g);
    if (!sp.active) return;
    const int64_t col = (int64_t)sp.y * g.nx + sp.x;
    const float cxy = fa.cx[sp.x] * fa.cy[sp.y];
    z_march<R, 2>(t1, t2, col, g.sxy, g.nz, sp.z0, sp.z1, t, [&](int z, float A1, float B1) {
        const int64_t v = col + (int64_t)z * g.sxy;
        const float K1 = cxy * fa.cz[z];
        const float A2 = fa.KI[v] - A1;
        const float B2 = K1 - B1;
        const float f1 = A1 * rcp(B1);
        const float f2 = A2 * rcp(B2);
        g1[v] = fa.l1 * f1 - fa.l2 * f2;
        g2[v] = fa.l1 * f1 * f1 - fa.l2 * f2 * f2;
        if (PROBE) {
            if (fa.probe_f1) fa.probe_f1[v] = f1;
            if (fa.probe_f2) fa.probe_f2[v] = f2;
        }
    });
}

// Diffusion-rate excess D(s) = d_p(s) - 1 of the distance regulariser.
__device__ __forceinline__ float reg_rate(float s, float s_eta, int reg)
{
    if (reg != 0) return -rcp(s_eta);
    if (s > 1.f) return -rcp(s);
    if (s == 0.f) return 0.f;
    const float a = kTwoPi * s;
    return sinf(a) / a - 1.f;
}

template <int R, bool PROBE>
__global__ __launch_bounds__(kThreads) void z_update_kernel(const float *__restrict__ t1,
                                                            const float *__restrict__ t2,
                                                            Grid3 g, Taps t, UpdArgs ua,
                                                            const int *__restrict__ done)
{
    const ZSpan sp = z_span(g);
    const int64_t bid =
        blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    const bool stopped = done && *done;
    double acc = 0.0;
    if (sp.active) {
        const int64_t col = (int64_t)sp.y * g.nx + sp.x;
        if (stopped) {
            for (int z = sp.z0; z < sp.z1; ++z)
                ua.phi_out[col + (int64_t)z * g.sxy] = ua.phi[col + (int64_t)z * g.sxy];
        } else {
            // reflected neighbour offsets in x and y (fixed for the column)
            int xo[5], yo[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                xo[k] = reflect(sp.x + k - 2, g.nx);
                yo[k] = reflect(sp.y + k - 2, g.ny) * g.nx;
            }
            const float cxy = ua.cx[sp.x] * ua.cy[sp.y];
            const float *phi = ua.phi;
            z_march<R, 2>(t1, t2, col, g.sxy, g.nz, sp.z0, sp.z1, t,
                          [&](int z, float KG1, float KG2) {
                int64_t zo[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) zo[k] = (int64_t)reflect(z + k - 2, g.nz) * g.sxy;
                auto P = [&](int i, int j, int k) -> float {
                    return phi[zo[k + 2] + yo[j + 2] + xo[i + 2]];
                };
                const int64_t v = col + (int64_t)z * g.sxy;
                const float c = P(0, 0, 0);
                const float I = ua.I[v];
                const float K1 = cxy * ua.cz[z];
                const float Fd = (ua.l1 - ua.l2) * I * I * K1 - 2.f * I * KG1 + KG2;

                const float lap = P(1, 0, 0) + P(-1, 0, 0) + P(0, 1, 0) + P(0, -1, 0) +
                                  P(0, 0, 1) + P(0, 0, -1) - 6.f * c;
                float kappa = 0.f, divV = 0.f;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
                    for (int sg = 1; sg >= -1; sg -= 2) {
                        // gradient at p = v + sg * e_ax
                        const int pi = ax == 0 ? sg : 0, pj = ax == 1 ? sg : 0,
                                  pk = ax == 2 ? sg : 0;
                        const float gx = 0.5f * (P(pi + 1, pj, pk) - P(pi - 1, pj, pk));
                        const float gy = 0.5f * (P(pi, pj + 1, pk) - P(pi, pj - 1, pk));
                        const float gz = 0.5f * (P(pi, pj, pk + 1) - P(pi, pj, pk - 1));
                        const float s2 = gx * gx + gy * gy + gz * gz;
                        const float s_eta = __builtin_amdgcn_sqrtf(s2 + ua.eta);
                        const float ga = ax == 0 ? gx : (ax == 1 ? gy : gz);
                        const float na = ga * rcp(s_eta);
                        const float Da = reg_rate(__builtin_amdgcn_sqrtf(s2), s_eta, ua.reg);
                        kappa += sg > 0 ? 0.5f * na : -0.5f * na;
                        divV += sg > 0 ? 0.5f * Da * ga : -0.5f * Da * ga;
                    }
                }
                const float Rt = lap + divV;
                const float delta = ua.eps_over_pi * rcp(ua.eps2 + c * c);
                const float E = ua.mu * Rt + delta * (ua.nu * kappa - Fd);
                const float nxt = c + ua.dt * E;
                ua.phi_out[v] = nxt;
                acc += fabs((double)nxt - (double)c);
                if (PROBE) {
                    if (ua.probe_Fd) ua.probe_Fd[v] = Fd;
                    if (ua.probe_kappa) ua.probe_kappa[v] = kappa;
                    if (ua.probe_lap) ua.probe_lap[v] = lap;
                    if (ua.probe_R) ua.probe_R[v] = Rt;
                    if (ua.probe_E) ua.probe_E[v] = E;
                }
            });
        }
    }
    // Block sum of |dphi| in a fixed order: wave tree, then the four waves.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double wsum[kThreads / 64];
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) ua.partials[bid] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
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

int z_chunks(const Grid3 &g)
{
    const int64_t cols = (int64_t)((g.nx + kZx - 1) / kZx) * ((g.ny + kZy - 1) / kZy);
    int64_t want = (2048 + cols - 1) / cols;
    const int64_t most = (g.nz + 7) / 8;   // chunks of at least 8 slices
    if (want > most) want = most;
    if (want < 1) want = 1;
    // re-derive so that every chunk is non-empty
    const int lz = (int)((g.nz + want - 1) / want);
    return (g.nz + lz - 1) / lz;
}

int64_t z_blocks(const Grid3 &g)
{
    return (int64_t)((g.nx + kZx - 1) / kZx) * ((g.ny + kZy - 1) / kZy) * z_chunks(g);
}

static dim3 z_grid(const Grid3 &g)
{
    return dim3((g.nx + kZx - 1) / kZx, (g.ny + kZy - 1) / kZy, z_chunks(g));
}

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

#define RSF_R_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_xy(int R, int mode, const float *a, const float *b, float *oa, float *ob,
                     Grid3 g, const Taps &t, float eps, float *probeH, const int *done,
                     hipStream_t s)
{
    const dim3 grid((g.nx + kXyTx - 1) / kXyTx, (g.ny + kXyTy - 1) / kXyTy, g.nz);
    switch (R * 4 + mode) {
#define XY_CASE(RR)                                                                          \
    case RR * 4 + XY_ONE:                                                                    \
        hipLaunchKernelGGL((xy_kernel<RR, XY_ONE>), grid, dim3(kThreads), 0, s, a, b, oa, ob, \
                           g, t, eps, probeH, done);                                         \
        break;                                                                               \
    case RR * 4 + XY_HEAVISIDE:                                                              \
        hipLaunchKernelGGL((xy_kernel<RR, XY_HEAVISIDE>), grid, dim3(kThreads), 0, s, a, b,  \
                           oa, ob, g, t, eps, probeH, done);                                 \
        break;                                                                               \
    case RR * 4 + XY_TWO:                                                                    \
        hipLaunchKernelGGL((xy_kernel<RR, XY_TWO>), grid, dim3(kThreads), 0, s, a, b, oa, ob, \
                           g, t, eps, probeH, done);                                         \
        break;
        RSF_R_CASES(XY_CASE)
#undef XY_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_z_plain(int R, const float *in, float *out, Grid3 g, const Taps &t,
                          hipStream_t s)
{
    switch (R) {
#define ZP_CASE(RR)                                                                        \
    case RR:                                                                               \
        hipLaunchKernelGGL((z_plain_kernel<RR>), z_grid(g), dim3(kThreads), 0, s, in, out, \
                           g, t);                                                          \
        break;
        RSF_R_CASES(ZP_CASE)
#undef ZP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_z_fits(int R, const float *t1, const float *t2, float *g1, float *g2,
                         Grid3 g, const Taps &t, const FitArgs &fa, const int *done,
                         hipStream_t s)
{
    const bool probe = fa.probe_f1 || fa.probe_f2;
    switch (R * 2 + (probe ? 1 : 0)) {
#define ZF_CASE(RR)                                                                     \
    case RR * 2:                                                                        \
        hipLaunchKernelGGL((z_fits_kernel<RR, false>), z_grid(g), dim3(kThreads), 0, s, \
                           t1, t2, g1, g2, g, t, fa, done);                             \
        break;                                                                          \
    case RR * 2 + 1:                                                                    \
        hipLaunchKernelGGL((z_fits_kernel<RR, true>), z_grid(g), dim3(kThreads), 0, s,  \
                           t1, t2, g1, g2, g, t, fa, done);                             \
        break;
        RSF_R_CASES(ZF_CASE)
#undef ZF_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_z_update(int R, const float *t1, const float *t2, Grid3 g, const Taps &t,
                           const UpdArgs &ua, const int *done, hipStream_t s)
{
    const bool probe =
        ua.probe_Fd || ua.probe_kappa || ua.probe_lap || ua.probe_R || ua.probe_E;
    switch (R * 2 + (probe ? 1 : 0)) {
#define ZU_CASE(RR)                                                                       \
    case RR * 2:                                                                          \
        hipLaunchKernelGGL((z_update_kernel<RR, false>), z_grid(g), dim3(kThreads), 0, s, \
                           t1, t2, g, t, ua, done);                                       \
        break;                                                                            \
    case RR * 2 + 1:                                                                      \
        hipLaunchKernelGGL((z_update_kernel<RR, true>), z_grid(g), dim3(kThreads), 0, s,  \
                           t1, t2, g, t, ua, done);                                       \
        break;
        RSF_R_CASES(ZU_CASE)
#undef ZU_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int64_t n, double *out, int *flags,
                         double tol_total, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, n, out, flags,
                       tol_total);
    return hipGetLastError();
}

}  // namespace rsf
