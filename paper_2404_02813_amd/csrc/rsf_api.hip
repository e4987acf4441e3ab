// C ABI of the RSF evolution library (declared in include/rsf.h): argument
// validation, workspace layout, and the per-iteration launch sequence.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "rsf.h"
#include "rsf_internal.hpp"

struct rsf_context {
    int device = 0;
    std::string err;
    void *ws = nullptr;          // owned workspace
    size_t ws_bytes = 0;
    // last evolution, for rsf_get_stats
    hipStream_t last_stream = nullptr;
    const double *last_hist = nullptr;
    const int *last_flags = nullptr;
    int last_iters = 0;
    bool has_last = false;
    // per-pass event timing
    bool prof = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Rec> recs;
};

namespace {

using rsf::Grid3;
using rsf::Taps;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// P, Q: interleaved pairs of the storage type (the stage-1 z-convolved
// fields, then alternately g1/g2 and their xy convolutions); KI: K*I.
struct Layout {
    size_t P, Q, KI, phiB, cx, cy, cz, partials, hist, flags, total;
};

size_t elem_size(int dtype) { return dtype == RSF_F32 ? 4 : 2; }

// Two pair fields and K*I in the storage type, the phi ping-pong buffer in
// float, plus edge tables, partial sums, history and flags.
Layout layout(int64_t nx, int64_t ny, int64_t nz, int iters, int storage)
{
    Layout L{};
    const size_t n = (size_t)nx * ny * nz;
    const size_t field = align_up(n * elem_size(storage));
    const size_t pair = align_up(2 * n * elem_size(storage));
    size_t off = 0;
    L.P = off; off += pair;
    L.Q = off; off += pair;
    L.KI = off; off += field;
    L.phiB = off; off += align_up(n * sizeof(float));
    L.cx = off; off += align_up((size_t)nx * sizeof(float));
    L.cy = off; off += align_up((size_t)ny * sizeof(float));
    L.cz = off; off += align_up((size_t)nz * sizeof(float));
    rsf::Grid3 g{(int)nx, (int)ny, (int)nz, nx * ny};
    L.partials = off; off += align_up((size_t)rsf::u_blocks(g) * sizeof(double));
    L.hist = off; off += align_up((size_t)(iters > 0 ? iters : 1) * sizeof(double));
    L.flags = off; off += align_up(4 * sizeof(int));
    L.total = off;
    return L;
}

int radius_of(float sigma) { return (int)std::ceil(3.0 * (double)sigma - 1e-9); }

// Sampled, truncated, unit-sum Gaussian (Sec. 3 kernel on the grid).
Taps make_taps(float sigma, int R)
{
    Taps t{};
    double w[2 * rsf::kMaxR + 1];
    double sum = 0.0;
    for (int k = -R; k <= R; ++k) {
        w[k + R] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
        sum += w[k + R];
    }
    for (int k = 0; k < 2 * R + 1; ++k) t.w[k] = (float)(w[k] / sum);
    return t;
}

rsf_status fail(rsf_context *ctx, rsf_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

rsf_status hip_fail(rsf_context *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? RSF_ERR_OUT_OF_MEMORY : RSF_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

hipEvent_t take_event(rsf_context *ctx)
{
    if (ctx->ev_used < ctx->ev_pool.size()) return ctx->ev_pool[ctx->ev_used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
    ctx->ev_used = ctx->ev_pool.size();
    return e;
}

// Launch through `fn`, bracketed by events on `s` while profiling is on.
template <class F>
hipError_t timed(rsf_context *ctx, int kind, hipStream_t s, F &&fn)
{
    if (!ctx->prof) return fn();
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return fn();
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e == hipSuccess) ctx->recs.push_back({kind, a, b});
    return e;
}

bool finite(float v) { return std::isfinite(v); }

rsf_status check_dims(rsf_context *ctx, int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 3 || ny < 3 || nz < 3)
        return fail(ctx, RSF_ERR_INVALID_ARG, "every dimension must be >= 3");
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30) || nx * ny > ((int64_t)1 << 31) ||
        nx * ny > INT64_MAX / nz)
        return fail(ctx, RSF_ERR_INVALID_ARG, "volume too large");
    return RSF_OK;
}

rsf_status check_params(rsf_context *ctx, const rsf_params &p)
{
    if (!finite(p.sigma) || !finite(p.lambda1) || !finite(p.lambda2) || !finite(p.nu) ||
        !finite(p.mu) || !finite(p.dt) || !finite(p.eps) || !finite(p.eta))
        return fail(ctx, RSF_ERR_INVALID_ARG, "parameters must be finite");
    if (!(p.sigma > 0.f) || radius_of(p.sigma) > rsf::kMaxR)
        return fail(ctx, RSF_ERR_INVALID_ARG, "sigma must be > 0 with ceil(3 sigma) <= 16");
    if (!(p.eps > 0.f)) return fail(ctx, RSF_ERR_INVALID_ARG, "eps must be > 0");
    if (!(p.dt > 0.f)) return fail(ctx, RSF_ERR_INVALID_ARG, "dt must be > 0");
    if (p.nu < 0.f || p.mu < 0.f) return fail(ctx, RSF_ERR_INVALID_ARG, "nu and mu must be >= 0");
    if (p.regulariser != RSF_REG_DOUBLE_WELL && p.regulariser != RSF_REG_SINGLE_WELL)
        return fail(ctx, RSF_ERR_INVALID_ARG, "unknown regulariser");
    if (p.storage != RSF_F32 && p.storage != RSF_F16 && p.storage != RSF_BF16)
        return fail(ctx, RSF_ERR_INVALID_ARG, "storage must be RSF_F32, RSF_F16 or RSF_BF16");
    return RSF_OK;
}

rsf_status check_types(rsf_context *ctx, float sigma, int image, int storage)
{
    if (image != RSF_F32 && image != RSF_U16)
        return fail(ctx, RSF_ERR_INVALID_ARG, "volume dtype must be RSF_F32 or RSF_U16");
    if (!rsf::types_supported(radius_of(sigma), image, storage))
        return fail(ctx, RSF_ERR_INVALID_ARG,
                    "this image/storage combination is built for ceil(3 sigma) in 4..12 only");
    return RSF_OK;
}

rsf_status set_device(rsf_context *ctx)
{
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    return RSF_OK;
}

// Make sure the context-owned workspace holds `bytes`.
rsf_status ensure_ws(rsf_context *ctx, size_t bytes)
{
    if (ctx->ws_bytes >= bytes) return RSF_OK;
    if (ctx->ws) {
        // the old buffer may still be in use by queued work
        HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
        HIP_TRY(hipFree(ctx->ws), "hipFree");
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, bytes), "hipMalloc(workspace)");
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return RSF_OK;
}

struct Plan {
    Grid3 g;
    int R;
    int image, storage;
    Taps taps;
    Layout L;
    char *base;
    void *P, *Q, *KI;
    float *phiB, *cx, *cy, *cz;
    double *partials, *hist;
    int *flags;
};

Plan make_plan(int64_t nx, int64_t ny, int64_t nz, float sigma, int iters, int image, int storage,
               char *base)
{
    Plan P{};
    P.g = Grid3{(int)nx, (int)ny, (int)nz, nx * ny};
    P.R = radius_of(sigma);
    P.image = image;
    P.storage = storage;
    P.taps = make_taps(sigma, P.R);
    P.L = layout(nx, ny, nz, iters, storage);
    P.base = base;
    auto F = [&](size_t off) { return reinterpret_cast<float *>(base + off); };
    auto V = [&](size_t off) { return static_cast<void *>(base + off); };
    P.P = V(P.L.P); P.Q = V(P.L.Q);
    P.KI = V(P.L.KI); P.phiB = F(P.L.phiB);
    P.cx = F(P.L.cx); P.cy = F(P.L.cy); P.cz = F(P.L.cz);
    P.partials = reinterpret_cast<double *>(base + P.L.partials);
    P.hist = reinterpret_cast<double *>(base + P.L.hist);
    P.flags = reinterpret_cast<int *>(base + P.L.flags);
    return P;
}

// Per-volume set-up: edge tables of K*1, flags, and K*I.
rsf_status prologue(rsf_context *ctx, const Plan &P, const void *I, hipStream_t s)
{
    HIP_TRY(timed(ctx, RSF_PASS_SETUP, s, [&] {
                hipError_t e = rsf::launch_flags_init(P.flags, s);
                if (e == hipSuccess) e = rsf::launch_edges(P.cx, P.cy, P.cz, P.g, P.taps, P.R, s);
                if (e == hipSuccess)
                    e = rsf::launch_xy(P.R, rsf::XY_ONE, P.image, P.storage, I, P.P, P.g, P.taps,
                                       nullptr, nullptr, s);
                if (e == hipSuccess)
                    e = rsf::launch_z_plain(P.R, P.storage, P.P, P.KI, P.g, P.taps, s);
                return e;
            }),
            "setup (K*1 tables, K*I)");
    return RSF_OK;
}

struct Probe {
    float *H = nullptr, *f1 = nullptr, *f2 = nullptr, *Fd = nullptr, *kappa = nullptr,
          *lap = nullptr, *R = nullptr, *E = nullptr;
};

// One iteration phi_cur -> phi_nxt; its sum |dphi| goes to hist_slot.
rsf_status iteration(rsf_context *ctx, const Plan &P, const void *I, const float *cur,
                     float *nxt, const rsf_params &p, double *hist_slot, double tol_total,
                     const Probe &pr, hipStream_t s)
{
    const int *done = P.flags;
    HIP_TRY(timed(ctx, RSF_PASS_Z_HEAVISIDE, s, [&] {
                return rsf::launch_z_heaviside(P.R, P.image, P.storage, cur, I, P.P, P.g, P.taps,
                                               p.eps, pr.H, done, s);
            }),
            "z(H)");
    rsf::FitArgs fa{P.KI, P.cx, P.cy, P.cz, p.lambda1, p.lambda2, pr.f1, pr.f2};
    HIP_TRY(timed(ctx, RSF_PASS_XY_FITS, s, [&] {
                return rsf::launch_xy(P.R, rsf::XY_FITS, P.image, P.storage, P.P, P.Q, P.g,
                                      P.taps, &fa, done, s);
            }),
            "xy(fits)");
    HIP_TRY(timed(ctx, RSF_PASS_XY_FORCE, s, [&] {
                return rsf::launch_xy(P.R, rsf::XY_TWO, P.image, P.storage, P.Q, P.P, P.g,
                                      P.taps, nullptr, done, s);
            }),
            "xy(g)");
    rsf::UpdArgs ua{};
    ua.I = I;
    ua.phi = cur;
    ua.phi_out = nxt;
    ua.cx = P.cx; ua.cy = P.cy; ua.cz = P.cz;
    ua.l1 = p.lambda1; ua.l2 = p.lambda2; ua.nu = p.nu; ua.mu = p.mu; ua.dt = p.dt;
    ua.eps_over_pi = (float)((double)p.eps / M_PI);
    ua.eps2 = p.eps * p.eps;
    ua.eta = p.eta > 0.f ? p.eta : 1e-10f;
    ua.reg = p.regulariser == RSF_REG_SINGLE_WELL ? 1 : 0;
    ua.partials = P.partials;
    ua.probe_Fd = pr.Fd; ua.probe_kappa = pr.kappa; ua.probe_lap = pr.lap;
    ua.probe_R = pr.R; ua.probe_E = pr.E;
    HIP_TRY(timed(ctx, RSF_PASS_Z_UPDATE, s,
                  [&] {
                      return rsf::launch_z_update(P.R, P.image, P.storage, P.P, P.g, P.taps, ua,
                                                  done, s);
                  }),
            "z(update)");
    HIP_TRY(timed(ctx, RSF_PASS_REDUCE, s, [&] {
                return rsf::launch_reduce(P.partials, rsf::u_blocks(P.g), hist_slot, P.flags,
                                          tol_total, s);
            }),
            "reduce");
    return RSF_OK;
}

rsf_status evolve_impl(rsf_context *ctx, const void *volume, int vdt, float *phi, int64_t nx,
                       int64_t ny, int64_t nz, const rsf_params &p, int iters, double tol,
                       void *workspace, size_t ws_bytes, void *stream)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!volume || !phi) return fail(ctx, RSF_ERR_INVALID_ARG, "null volume or phi");
    rsf_status st = check_dims(ctx, nx, ny, nz);
    if (st != RSF_OK) return st;
    st = check_params(ctx, p);
    if (st != RSF_OK) return st;
    st = check_types(ctx, p.sigma, vdt, p.storage);
    if (st != RSF_OK) return st;
    if (iters < 0) return fail(ctx, RSF_ERR_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ctx, RSF_ERR_INVALID_ARG, "tol must be >= 0");
    const Layout L = layout(nx, ny, nz, iters, p.storage);
    if (workspace && ws_bytes < L.total)
        return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    st = set_device(ctx);
    if (st != RSF_OK) return st;
    if (!workspace) {
        st = ensure_ws(ctx, L.total);
        if (st != RSF_OK) return st;
    }
    char *base = static_cast<char *>(workspace ? workspace : ctx->ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Plan P = make_plan(nx, ny, nz, p.sigma, iters, vdt, p.storage, base);
    const void *I = volume;

    st = prologue(ctx, P, I, s);
    if (st != RSF_OK) return st;
    const double tol_total = tol * (double)nx * ny * nz;
    float *cur = phi, *nxt = P.phiB;
    for (int it = 0; it < iters; ++it) {
        st = iteration(ctx, P, I, cur, nxt, p, P.hist + it, tol_total, Probe{}, s);
        if (st != RSF_OK) return st;
        float *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != phi)
        HIP_TRY(hipMemcpyAsync(phi, cur, (size_t)nx * ny * nz * sizeof(float),
                               hipMemcpyDeviceToDevice, s),
                "copy phi");
    ctx->last_stream = s;
    ctx->last_hist = P.hist;
    ctx->last_flags = P.flags;
    ctx->last_iters = iters;
    ctx->has_last = true;
    return RSF_OK;
}

rsf_params default_params(float sigma, float l1, float l2, float nu, float mu, float dt,
                          float eps)
{
    rsf_params p{};
    p.sigma = sigma; p.lambda1 = l1; p.lambda2 = l2; p.nu = nu; p.mu = mu; p.dt = dt;
    p.eps = eps; p.eta = 1e-10f; p.regulariser = RSF_REG_DOUBLE_WELL; p.storage = RSF_F32;
    return p;
}

}  // namespace

extern "C" {

rsf_status rsf_create(rsf_context **out, int device_ordinal)
{
    if (!out) return RSF_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device_ordinal < 0 || device_ordinal >= n)
            return RSF_ERR_INVALID_ARG;
        rsf_context *c = new (std::nothrow) rsf_context();
        if (!c) return RSF_ERR_OUT_OF_MEMORY;
        c->device = device_ordinal;
        *out = c;
        return RSF_OK;
    } catch (...) {
        return RSF_ERR_INTERNAL;
    }
}

void rsf_destroy(rsf_context *ctx)
{
    if (!ctx) return;
    try {
        (void)hipSetDevice(ctx->device);
        if (ctx->ws || !ctx->ev_pool.empty()) (void)hipDeviceSynchronize();
        if (ctx->ws) (void)hipFree(ctx->ws);
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    } catch (...) {
    }
    delete ctx;
}

rsf_status rsf_profile_enable(rsf_context *ctx, int on)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    ctx->prof = on != 0;
    return RSF_OK;
}

rsf_status rsf_profile_read(rsf_context *ctx, rsf_profile *out)
{
    try {
        if (!ctx || !out) return fail(ctx, RSF_ERR_INVALID_ARG, "null argument");
        std::memset(out, 0, sizeof(*out));
        rsf_status st = set_device(ctx);
        if (st != RSF_OK) return st;
        for (const auto &r : ctx->recs) {
            HIP_TRY(hipEventSynchronize(r.b), "hipEventSynchronize");
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
            if (r.kind >= 0 && r.kind < RSF_PASS_COUNT) {
                out->launches[r.kind] += 1;
                out->ms[r.kind] += ms;
            }
        }
        ctx->recs.clear();
        ctx->ev_used = 0;
        return RSF_OK;
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

const char *rsf_last_error(const rsf_context *ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

size_t rsf_workspace_bytes(int64_t nx, int64_t ny, int64_t nz, int iters, int storage)
{
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    if (storage != RSF_F32 && storage != RSF_F16 && storage != RSF_BF16) return 0;
    return layout(nx, ny, nz, iters, storage).total;
}

rsf_status rsf_evolve(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                      int64_t nx, int64_t ny, int64_t nz, float sigma, float lambda1,
                      float lambda2, float nu, float mu, float dt, float eps, int iters,
                      void *stream)
{
    try {
        const rsf_params p = default_params(sigma, lambda1, lambda2, nu, mu, dt, eps);
        return evolve_impl(ctx, volume, volume_dtype, phi, nx, ny, nz, p, iters, 0.0, nullptr, 0,
                           stream);
    } catch (const std::bad_alloc &) {
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_evolve_ex(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                         int64_t nx, int64_t ny, int64_t nz, const rsf_params *params, int iters,
                         double tol, void *workspace, size_t workspace_bytes, void *stream)
{
    try {
        if (!params) return fail(ctx, RSF_ERR_INVALID_ARG, "null params");
        return evolve_impl(ctx, volume, volume_dtype, phi, nx, ny, nz, *params, iters, tol,
                           workspace, workspace_bytes, stream);
    } catch (const std::bad_alloc &) {
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_get_stats(rsf_context *ctx, rsf_stats *out, double *s_hist, int cap)
{
    try {
        if (!ctx || !out) return fail(ctx, RSF_ERR_INVALID_ARG, "null argument");
        if (!ctx->has_last) return fail(ctx, RSF_ERR_INVALID_ARG, "no evolution has run");
        rsf_status st = set_device(ctx);
        if (st != RSF_OK) return st;
        HIP_TRY(hipStreamSynchronize(ctx->last_stream), "hipStreamSynchronize");
        int flags[2] = {0, 0};
        HIP_TRY(hipMemcpy(flags, ctx->last_flags, sizeof(flags), hipMemcpyDeviceToHost),
                "copy flags");
        out->iters_requested = ctx->last_iters;
        out->iters_run = flags[1];
        out->last_sum_abs = 0.0;
        const int n = flags[1];
        if (n > 0) {
            HIP_TRY(hipMemcpy(&out->last_sum_abs, ctx->last_hist + (n - 1), sizeof(double),
                              hipMemcpyDeviceToHost),
                    "copy last sum");
            if (!std::isfinite(out->last_sum_abs))
                (void)fail(ctx, RSF_ERR_NONFINITE, "non-finite sum |dphi|");
        }
        if (s_hist && cap > 0 && n > 0) {
            const int m = cap < n ? cap : n;
            HIP_TRY(hipMemcpy(s_hist, ctx->last_hist, (size_t)m * sizeof(double),
                              hipMemcpyDeviceToHost),
                    "copy history");
        }
        return std::isfinite(out->last_sum_abs) ? RSF_OK : RSF_ERR_NONFINITE;
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_gauss3d(rsf_context *ctx, const float *in, float *out, int64_t nx, int64_t ny,
                       int64_t nz, float sigma, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        if (!in || !out || in == out) return fail(ctx, RSF_ERR_INVALID_ARG, "bad in/out pointers");
        if (nx < 1 || ny < 1 || nz < 1 || nx * ny > ((int64_t)1 << 31))
            return fail(ctx, RSF_ERR_INVALID_ARG, "bad dimensions");
        if (!std::isfinite(sigma) || !(sigma > 0.f) || radius_of(sigma) > rsf::kMaxR)
            return fail(ctx, RSF_ERR_INVALID_ARG, "sigma must be > 0 with ceil(3 sigma) <= 16");
        rsf_status st = set_device(ctx);
        if (st != RSF_OK) return st;
        const size_t need = align_up((size_t)nx * ny * nz * sizeof(float));
        st = ensure_ws(ctx, need);
        if (st != RSF_OK) return st;
        const Grid3 g{(int)nx, (int)ny, (int)nz, nx * ny};
        const int R = radius_of(sigma);
        const Taps t = make_taps(sigma, R);
        float *tmp = static_cast<float *>(ctx->ws);
        hipStream_t s = static_cast<hipStream_t>(stream);
        HIP_TRY(rsf::launch_xy(R, rsf::XY_ONE, RSF_F32, RSF_F32, in, tmp, g, t, nullptr, nullptr,
                               s),
                "xy");
        HIP_TRY(rsf::launch_z_plain(R, RSF_F32, tmp, out, g, t, s), "z");
        return RSF_OK;
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_probe(rsf_context *ctx, const void *volume, int volume_dtype, const float *phi,
                     int64_t nx, int64_t ny, int64_t nz, const rsf_params *params,
                     const rsf_probe_fields *fields, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        if (!volume || !phi || !params || !fields)
            return fail(ctx, RSF_ERR_INVALID_ARG, "null argument");
        rsf_status st = check_dims(ctx, nx, ny, nz);
        if (st != RSF_OK) return st;
        st = check_params(ctx, *params);
        if (st != RSF_OK) return st;
        st = check_types(ctx, params->sigma, volume_dtype, params->storage);
        if (st != RSF_OK) return st;
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        const Layout L = layout(nx, ny, nz, 1, params->storage);
        st = ensure_ws(ctx, L.total);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Plan P = make_plan(nx, ny, nz, params->sigma, 1, volume_dtype, params->storage,
                                 static_cast<char *>(ctx->ws));
        const void *I = volume;
        st = prologue(ctx, P, I, s);
        if (st != RSF_OK) return st;
        Probe pr;
        pr.H = fields->H; pr.f1 = fields->f1; pr.f2 = fields->f2; pr.Fd = fields->Fd;
        pr.kappa = fields->kappa; pr.lap = fields->lap; pr.R = fields->R; pr.E = fields->E;
        float *nxt = fields->phi_next ? fields->phi_next : P.phiB;
        return iteration(ctx, P, I, phi, nxt, *params, P.hist, 0.0, pr, s);
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

}  // extern "C"
