// C ABI of the RSF evolution library (declared in include/rsf.h): argument
// validation, batch planning and workspace layout, and the per-iteration
// launch sequence.  A single volume is evolved as a batch of one tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rsf.h"
#include "rsf_fault.hpp"
#include "rsf_host.hpp"
#include "rsf_internal.hpp"

namespace {

using rsf::Batch;
using rsf::Coeffs;
using rsf::Grid3;
using rsf::Split;
using rsf::Taps;
using rsf::TileDesc;
using rsf::host::align_up;
using rsf::host::kAlign;
using rsf::host::make_coeffs;
using rsf::host::make_taps;
using rsf::host::radius_of;

// Workspace of rsf_evolve_noalloc: one array per GPU, loaded with the
// library's code object and held until the process ends.  In host code the
// name is only a handle: its device address, per device, comes from
// hipGetSymbolAddress at rsf_create and is used everywhere instead.
__device__ __align__(256) char scratch[RSF_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device
// with that device current (the caller's current device is restored).
hipError_t scratch_address(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        e = hipSetDevice(device);
        if (e != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

namespace rsf {
namespace {

// The armed fault: attempts first .. first + count - 1 fail; first 0 when
// disarmed.  Guarded by g_fault_mu (a server's worker thread allocates too).
std::mutex g_fault_mu;
int64_t g_fault_first = 0, g_fault_count = 0, g_fault_seen = 0;
bool g_fault_env_bad = false;

// "alloc_fail:N" or "alloc_fail:N:K" with N, K >= 1; NULL, "" or "off"
// disarms (first = 0).
bool parse_fault(const char *spec, int64_t &first, int64_t &count)
{
    first = count = 0;
    if (!spec || !*spec || std::strcmp(spec, "off") == 0) return true;
    static const char kPrefix[] = "alloc_fail:";
    if (std::strncmp(spec, kPrefix, sizeof(kPrefix) - 1) != 0) return false;
    const char *p = spec + sizeof(kPrefix) - 1;
    char *end = nullptr;
    errno = 0;
    const long long n = std::strtoll(p, &end, 10);
    if (end == p || errno || n < 1) return false;
    long long k = 1;
    if (*end == ':') {
        p = end + 1;
        k = std::strtoll(p, &end, 10);
        if (end == p || errno || k < 1) return false;
    }
    if (*end != '\0') return false;
    first = n;
    count = k;
    return true;
}

// RSF_FAULT is read once, when the library is loaded; a malformed value arms
// nothing and makes rsf_create refuse.
struct FaultFromEnv {
    FaultFromEnv()
    {
        const char *spec = std::getenv("RSF_FAULT");
        if (!parse_fault(spec, g_fault_first, g_fault_count)) {
            g_fault_env_bad = true;
            std::fprintf(stderr, "librsf: malformed RSF_FAULT=%s (expected alloc_fail:N[:K])\n",
                         spec);
        }
    }
} g_fault_from_env;

}  // namespace

bool fault_take_alloc()
{
    std::lock_guard<std::mutex> lock(g_fault_mu);
    if (g_fault_first == 0) return false;
    const int64_t k = ++g_fault_seen;
    return k >= g_fault_first && k - g_fault_first < g_fault_count;
}

}  // namespace rsf

struct rsf_context {
    int device = 0;
    std::string err;
    void *ws = nullptr;          // owned workspace
    size_t ws_bytes = 0;
    // the stream of the last call that used the owned workspace and an event
    // recorded at its end: a call on another stream waits for it on the
    // device before it touches the workspace
    hipStream_t ws_stream = nullptr;
    hipEvent_t ws_ev = nullptr;
    bool ws_pending = false;
    // this device's copy of the no-alloc workspace (`scratch`)
    void *noalloc_ws = nullptr;
    // pinned staging of the tile table, and the event of its last upload
    void *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    // last evolution, for rsf_get_stats / rsf_get_tile_stats
    hipStream_t last_stream = nullptr;
    std::vector<const double *> last_hist;
    std::vector<const int *> last_flags;
    int last_iters = 0;
    bool has_last = false;
    // per-pass event timing
    bool prof = false;
    bool fuse = true;   // fused update + next stage-1 pass where a batch allows it
    // iteration groups replayed from a captured HIP graph (see run_iterations)
    bool graphs = true;
    hipStream_t cap_stream = nullptr;      // capture only: nothing runs on it
    hipGraphExec_t graph_exec = nullptr;   // the last group's executable graph
    std::vector<char> graph_key;           // what it was captured from
    hipEvent_t graph_ev = nullptr;         // recorded after its last launch
    // replaced graphs, destroyed once their last replay has completed
    struct Retired {
        hipGraphExec_t exec;
        hipEvent_t ev;
    };
    std::vector<Retired> retired;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Rec> recs;
    // autotuned splits by tile shape and radius
    std::map<std::vector<int64_t>, Split> tuned;
    // autotuned schedule (fused update or separate passes) by batch: the
    // sorted tile shapes, radius, force, image and storage types
    std::map<std::vector<int64_t>, bool> tuned_fuse;
    int force_schedule = -1;   // autotune trials: -1 none, 0 separate, 1 fused
    // workgroup targets of a batch when no tuned split applies
    rsf::Targets targets = rsf::kDefaultTargets;
};

namespace {

// Batch header (tile table and the three workgroup prefix tables) followed by
// the tiles' regions.
struct TileLayout {
    Grid3 g;
    Split sp;
    size_t base;                 // offset of the tile's region
    rsf::host::TileRegions T;
};

struct BatchLayout {
    size_t descs, start_xy, start_z, start_u, table_bytes;
    std::vector<TileLayout> tiles;
    std::vector<int> pre_xy, pre_z, pre_u;
    size_t total;
};

BatchLayout plan_layout(const rsf_tile *tiles, int n, int iters, int storage,
                        const std::vector<Split> &splits, bool k2 = false)
{
    BatchLayout L;
    size_t off = 0;
    L.descs = off; off += align_up(sizeof(TileDesc) * (size_t)n);
    L.start_xy = off; off += align_up(sizeof(int) * (size_t)(n + 1));
    L.start_z = off; off += align_up(sizeof(int) * (size_t)(n + 1));
    L.start_u = off; off += align_up(sizeof(int) * (size_t)(n + 1));
    L.table_bytes = off;
    L.pre_xy.assign(1, 0);
    L.pre_z.assign(1, 0);
    L.pre_u.assign(1, 0);
    for (int t = 0; t < n; ++t) {
        TileLayout T{};
        T.g = rsf::host::grid_of(tiles[t].nx, tiles[t].ny, tiles[t].nz);
        T.sp = splits[t];
        T.base = off;
        T.T = rsf::host::tile_regions(T.g, iters, storage, k2);
        off += T.T.total;
        L.pre_xy.push_back(L.pre_xy.back() + (int)rsf::xy_blocks(T.g, T.sp));
        L.pre_z.push_back(L.pre_z.back() + (int)rsf::z_blocks(T.g, T.sp));
        L.pre_u.push_back(L.pre_u.back() + (int)rsf::u_blocks(T.g, T.sp));
        L.tiles.push_back(T);
    }
    L.total = off;
    return L;
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

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
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

rsf_status check(rsf_context *ctx, const char *why)
{
    return why ? fail(ctx, RSF_ERR_INVALID_ARG, why) : RSF_OK;
}

rsf_status check_dims(rsf_context *ctx, int64_t nx, int64_t ny, int64_t nz)
{
    return check(ctx, rsf::host::dims_error(nx, ny, nz));
}

rsf_status check_params(rsf_context *ctx, const rsf_params &p)
{
    return check(ctx, rsf::host::params_error(p));
}

rsf_status check_types(rsf_context *ctx, const rsf_params &p, int image)
{
    return check(ctx, rsf::host::types_error(p, image));
}

rsf_status check_tiles(rsf_context *ctx, const rsf_tile *tiles, int n, bool need_pointers)
{
    if (!tiles || n < 1) return fail(ctx, RSF_ERR_INVALID_ARG, "need at least one tile");
    for (int t = 0; t < n; ++t) {
        if (need_pointers && (!tiles[t].volume || !tiles[t].phi))
            return fail(ctx, RSF_ERR_INVALID_ARG, "null volume or phi in tile " + std::to_string(t));
        rsf_status st = check_dims(ctx, tiles[t].nx, tiles[t].ny, tiles[t].nz);
        if (st != RSF_OK) return st;
    }
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
        ctx->has_last = false;   // its statistics lived in the freed buffer
    }
    void *p = nullptr;
    HIP_TRY(rsf::dev_alloc(&p, bytes), "hipMalloc(workspace)");
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return RSF_OK;
}

// Order a call that uses the owned workspace on stream s after the previous
// such call: on another stream, s first waits (on the device) for the event
// recorded at the end of that call.  ws_leave records it.
rsf_status ws_enter(rsf_context *ctx, hipStream_t s)
{
    if (ctx->ws_pending && ctx->ws_stream != s)
        HIP_TRY(hipStreamWaitEvent(s, ctx->ws_ev, 0), "hipStreamWaitEvent(workspace)");
    return RSF_OK;
}

rsf_status ws_leave(rsf_context *ctx, hipStream_t s)
{
    if (!ctx->ws_ev)
        HIP_TRY(hipEventCreateWithFlags(&ctx->ws_ev, hipEventDisableTiming),
                "hipEventCreate(workspace)");
    HIP_TRY(hipEventRecord(ctx->ws_ev, s), "hipEventRecord(workspace)");
    ctx->ws_stream = s;
    ctx->ws_pending = true;
    return RSF_OK;
}

// Pinned staging for the tile table; waits for its previous upload first.
rsf_status ensure_stage(rsf_context *ctx, size_t bytes)
{
    if (ctx->stage_pending) {
        HIP_TRY(hipEventSynchronize(ctx->stage_ev), "hipEventSynchronize(stage)");
        ctx->stage_pending = false;
    }
    if (!ctx->stage_ev)
        HIP_TRY(hipEventCreateWithFlags(&ctx->stage_ev, hipEventDisableTiming),
                "hipEventCreate(stage)");
    if (ctx->stage_bytes >= bytes) return RSF_OK;
    if (ctx->stage) HIP_TRY(hipHostFree(ctx->stage), "hipHostFree");
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    HIP_TRY(rsf::pinned_alloc(&ctx->stage, bytes), "hipHostMalloc(stage)");
    ctx->stage_bytes = bytes;
    return RSF_OK;
}

// A planned batch: device tile table plus the pass views.
struct Plan {
    int n;
    int R;
    int image, storage;
    Taps taps;
    Coeffs c;
    BatchLayout L;
    char *base;
    TileDesc *descs;             // device
    Batch xy, z, u, tile;
    int64_t blocks_xy, blocks_z, blocks_u;   // grid sizes
    bool k2;             // K2*I and K2*I^2 for the Sec. 4.2 force with sigma2 > 0
    int R2;
    Taps taps2;
    // every tile's update marched whole in z: the update also writes the
    // next iteration's stage-1 z pass
    bool fuse;
};

Grid3 grid_of(const rsf_tile &t) { return rsf::host::grid_of(t.nx, t.ny, t.nz); }

// Each tile's share of the batch's voxels.
std::vector<double> shares_of(const rsf_tile *tiles, int n)
{
    double total = 0.0;
    for (int t = 0; t < n; ++t) total += (double)tiles[t].nx * tiles[t].ny * tiles[t].nz;
    std::vector<double> sh;
    for (int t = 0; t < n; ++t)
        sh.push_back((double)tiles[t].nx * tiles[t].ny * tiles[t].nz / total);
    return sh;
}

// Whether an evolution of this batch carries the next stage-1 z pass in its
// update: the context allows it, no probe, and the RSF force's stage-2 ring
// leaves room for the stage-1 ring (radius <= fuse_max_r; the Sec. 4.2 force
// has no stage-2 ring).  Every tile is then marched whole in z (one update
// chunk per column tile).
std::vector<int64_t> schedule_key(const rsf_tile *tiles, int n, const rsf_params &p, int image)
{
    std::vector<std::array<int64_t, 3>> shapes;
    for (int t = 0; t < n; ++t) shapes.push_back({tiles[t].nx, tiles[t].ny, tiles[t].nz});
    std::sort(shapes.begin(), shapes.end());
    std::vector<int64_t> key{radius_of(p.sigma), p.force, image, p.storage};
    for (const auto &a : shapes) key.insert(key.end(), a.begin(), a.end());
    return key;
}

// Whether the force and radius allow the fused update at all (the context's
// switch on, no probe).
bool fusable(const rsf_context *ctx, const rsf_params &p, bool probe, int image)
{
    return ctx && ctx->fuse && !probe &&
           (p.force == RSF_FORCE_PAPER ||
            radius_of(p.sigma) <= rsf::fuse_max_r(p.storage, image));
}

std::vector<Split> splits_for(rsf_context *ctx, const rsf_tile *tiles, int n, int R,
                              bool whole_z = false);

// The schedule of a batch: an autotune trial's forced choice, else the
// autotuned choice for these tile shapes, else fused when the update keeps
// enough parallelism marching every tile whole in z: the tiles' own splits
// already do, or their column tiles alone fill 3/4 of the resident update
// workgroups (small volumes keep the separate passes and their z chunks).
bool decide_fuse(const rsf_context *ctx, const rsf_params &p, bool probe, const rsf_tile *tiles,
                 int n, int image)
{
    if (!fusable(ctx, p, probe, image)) return false;
    if (ctx->force_schedule >= 0) return ctx->force_schedule == 1;
    const auto it = ctx->tuned_fuse.find(schedule_key(tiles, n, p, image));
    if (it != ctx->tuned_fuse.end()) return it->second;
    const int R = radius_of(p.sigma);
    bool whole = true;
    int64_t cols = 0;
    const std::vector<Split> sps = splits_for(const_cast<rsf_context *>(ctx), tiles, n, R, false);
    for (int t = 0; t < n; ++t) {
        whole = whole && sps[t].u == 1;
        cols += (int64_t)((tiles[t].nx + rsf::kUx - 1) / rsf::kUx) *
                ((tiles[t].ny + rsf::kUy - 1) / rsf::kUy);
    }
    return whole || 4 * cols >= 3 * rsf::kResidentU;
}

// Tuned split of the shape if there is one, else the default for its share;
// `whole_z`: one update chunk per tile (the fused update).
// A tile's split when nothing is tuned for it: a single volume with the
// built-in targets is split for the resident capacity, anything else by its
// voxel share of the context's targets.
Split base_split(const rsf_context *ctx, const Grid3 &g, double share, int n, int R)
{
    const rsf::Targets tg = ctx ? ctx->targets : rsf::kDefaultTargets;
    const bool own_targets = tg.xy != rsf::kDefaultTargets.xy ||
                             tg.z != rsf::kDefaultTargets.z || tg.u != rsf::kDefaultTargets.u;
    return n == 1 && !own_targets && R > 0 ? rsf::capacity_split(g, R)
                                           : rsf::default_split(g, share, tg);
}

std::vector<Split> splits_for(rsf_context *ctx, const rsf_tile *tiles, int n, int R,
                              bool whole_z)
{
    const std::vector<double> sh = shares_of(tiles, n);
    std::vector<Split> splits;
    for (int t = 0; t < n; ++t) {
        const Grid3 g = grid_of(tiles[t]);
        Split s = base_split(ctx, g, sh[t], n, R);
        if (ctx) {
            auto it = ctx->tuned.find({g.nx, g.ny, g.nz, R});
            if (it != ctx->tuned.end() && rsf::split_valid(g, it->second)) s = it->second;
        }
        if (whole_z) s.u = 1;
        splits.push_back(s);
    }
    return splits;
}

// Lay out the batch in `base`, upload its tile table, fill the pass views.
// `probe` is for rsf_probe (one tile); `ki_out` for rsf_gauss3d.
rsf_status make_plan(rsf_context *ctx, Plan &P, const rsf_tile *tiles, int n, int image,
                     const rsf_params &p, double tol, int iters, char *base, hipStream_t s,
                     const rsf_probe_fields *probe = nullptr, void *ki_out = nullptr,
                     bool table_by_kernel = false)
{
    P.n = n;
    P.R = radius_of(p.sigma);
    P.image = image;
    P.storage = p.storage;
    P.taps = make_taps(p.sigma, P.R);
    P.c = make_coeffs(p, tol);
    P.k2 = rsf::host::needs_k2(p);
    P.R2 = P.k2 ? radius_of(p.sigma2) : 0;
    if (P.k2) P.taps2 = make_taps(p.sigma2, P.R2);
    const bool fuse = decide_fuse(ctx, p, probe != nullptr, tiles, n, image);
    P.L = plan_layout(tiles, n, iters, p.storage, splits_for(ctx, tiles, n, P.R, fuse), P.k2);
    P.base = base;
    // the table is built on the host: in the pinned staging buffer and
    // copied, or (table_by_kernel) in a kernel argument, allocating nothing
    rsf::TableBlob blob;
    char *h = nullptr;
    if (table_by_kernel) {
        if (P.L.table_bytes > sizeof(blob.w))
            return fail(ctx, RSF_ERR_INVALID_ARG, "tile table too large");
        h = reinterpret_cast<char *>(blob.w);
    } else {
        const rsf_status st = ensure_stage(ctx, P.L.table_bytes);
        if (st != RSF_OK) return st;
        h = static_cast<char *>(ctx->stage);
    }
    std::memset(h, 0, P.L.table_bytes);
    TileDesc *hd = reinterpret_cast<TileDesc *>(h + P.L.descs);
    for (int t = 0; t < n; ++t) {
        const TileLayout &T = P.L.tiles[t];
        TileDesc d = rsf::host::tile_desc(T.g, T.sp, tiles[t].volume, tiles[t].phi,
                                          base + T.base, T.T, iters, nullptr);
        if (ki_out) d.KI = ki_out;
        if (probe) {
            d.probe_H = probe->H; d.probe_f1 = probe->f1; d.probe_f2 = probe->f2;
            d.probe_Fd = probe->Fd; d.probe_kappa = probe->kappa; d.probe_lap = probe->lap;
            d.probe_R = probe->R; d.probe_E = probe->E;
            if (probe->phi_next) d.phi[1] = probe->phi_next;
        }
        hd[t] = d;
    }
    std::memcpy(h + P.L.start_xy, P.L.pre_xy.data(), sizeof(int) * (n + 1));
    std::memcpy(h + P.L.start_z, P.L.pre_z.data(), sizeof(int) * (n + 1));
    std::memcpy(h + P.L.start_u, P.L.pre_u.data(), sizeof(int) * (n + 1));
    if (table_by_kernel) {
        HIP_TRY(rsf::launch_put_table(base, blob, (int)P.L.table_bytes, s), "write tile table");
    } else {
        HIP_TRY(hipMemcpyAsync(base, h, P.L.table_bytes, hipMemcpyHostToDevice, s),
                "upload tile table");
        HIP_TRY(hipEventRecord(ctx->stage_ev, s), "hipEventRecord(stage)");
        ctx->stage_pending = true;
    }
    P.descs = reinterpret_cast<TileDesc *>(base + P.L.descs);
    auto view = [&](size_t start) {
        return Batch{P.descs, reinterpret_cast<const int *>(base + start), n, {}};
    };
    P.xy = view(P.L.start_xy);
    P.z = view(P.L.start_z);
    P.u = view(P.L.start_u);
    P.tile = Batch{P.descs, nullptr, n, {}};
    std::vector<Grid3> gs;
    std::vector<Split> sps;
    for (const TileLayout &T : P.L.tiles) {
        gs.push_back(T.g);
        sps.push_back(T.sp);
    }
    P.blocks_xy = rsf::host::balance_xcds(P.xy, rsf::host::PASS_XY, gs, sps, P.R);
    P.blocks_z = rsf::host::balance_xcds(P.z, rsf::host::PASS_Z, gs, sps, P.R);
    P.blocks_u = rsf::host::balance_xcds(P.u, rsf::host::PASS_U, gs, sps, P.R);
    P.fuse = fuse;
    for (const Split &sp : sps) P.fuse = P.fuse && sp.u == 1;
    return RSF_OK;
}

// Per-batch set-up: K*1 edge tables, flags, K*I, and for the Sec. 4.2 force
// with sigma2 > 0 also K2*I and K2*I^2 (each an xy pass into P, then a z pass).
rsf_status prologue(rsf_context *ctx, const Plan &P, hipStream_t s)
{
    HIP_TRY(timed(ctx, RSF_PASS_SETUP, s, [&] {
                hipError_t e = rsf::launch_setup(P.tile, P.taps, P.R, s);
                if (P.k2) {
                    Coeffs sq = P.c;
                    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
                        sq.square = k;
                        e = rsf::launch_xy(P.R2, rsf::XY_ONE, P.image, P.storage, P.xy,
                                           P.blocks_xy, P.taps2, sq, false, s);
                        if (e == hipSuccess)
                            e = rsf::launch_z_plain(P.R2, P.storage, P.z, P.blocks_z, P.taps2,
                                                    k ? rsf::Z_TO_K2I2 : rsf::Z_TO_K2I, s);
                    }
                }
                if (e == hipSuccess)
                    e = rsf::launch_xy(P.R, rsf::XY_ONE, P.image, P.storage, P.xy, P.blocks_xy,
                                       P.taps, P.c, false, s);
                if (e == hipSuccess)
                    e = rsf::launch_z_plain(P.R, P.storage, P.z, P.blocks_z, P.taps, rsf::Z_TO_KI,
                                            s);
                return e;
            }),
            "setup (K*1 tables, K*I)");
    return RSF_OK;
}

// The stage-1 z pass on its own (each iteration, or once before a fused loop).
rsf_status stage1(rsf_context *ctx, const Plan &P, bool probe, hipStream_t s)
{
    HIP_TRY(timed(ctx, RSF_PASS_Z_HEAVISIDE, s, [&] {
                return rsf::launch_z_heaviside(P.R, P.image, P.storage, P.z, P.blocks_z, P.taps,
                                               P.c, probe, s);
            }),
            "z(H)");
    return RSF_OK;
}

// One iteration of every running tile of the batch.  fused: the stage-1 pass
// of this iteration was written by the previous update (or by stage1 before
// the loop), and this update writes the next one.
rsf_status iteration(rsf_context *ctx, const Plan &P, bool probe, hipStream_t s,
                     bool fused = false)
{
    const Batch &u = P.u;
    if (!fused) {
        const rsf_status st = stage1(ctx, P, probe, s);
        if (st != RSF_OK) return st;
    }
    const bool paper = P.c.force == RSF_FORCE_PAPER;
    HIP_TRY(timed(ctx, RSF_PASS_XY_FITS, s, [&] {
                return rsf::launch_xy(P.R,
                                      paper ? (P.k2 ? rsf::XY_PAPER2 : rsf::XY_PAPER)
                                            : rsf::XY_FITS,
                                      P.image,
                                      P.storage, P.xy, P.blocks_xy, P.taps, P.c, probe, s);
            }),
            "xy(fits)");
    // the Sec. 4.2 force with sigma2 = 0 needs no second Gaussian stage
    if (!paper)
        HIP_TRY(timed(ctx, RSF_PASS_XY_FORCE, s, [&] {
                    return rsf::launch_xy(P.R, rsf::XY_TWO, P.image, P.storage, P.xy,
                                          P.blocks_xy, P.taps, P.c, probe, s);
                }),
                "xy(g)");
    HIP_TRY(timed(ctx, RSF_PASS_Z_UPDATE, s, [&] {
                if (fused)
                    return rsf::launch_z_update_fused(P.R, P.image, P.storage, u, P.blocks_u,
                                                      P.taps, P.c, paper, s);
                return paper ? rsf::launch_z_update_paper(P.image, P.storage, u, P.blocks_u, P.c,
                                                          probe, s)
                             : rsf::launch_z_update(P.R, P.image, P.storage, u, P.blocks_u,
                                                    P.taps, P.c, probe, s);
            }),
            "z(update)");
    HIP_TRY(timed(ctx, RSF_PASS_REDUCE, s, [&] { return rsf::launch_reduce(P.tile, P.c, s); }),
            "reduce");
    return RSF_OK;
}

// Iterations of a planned batch.  Every iteration launches the same kernels
// with the same arguments (each tile's current iterate and stop flag are read
// on the device), so a group of kGraphGroup iterations is captured once into
// a HIP graph and replayed on `s`; the rest of the count launches directly.
// The executable graph is kept and replayed by later calls whose launches are
// the same (same workspace, tile table, taps and coefficients); a different
// one replaces it once its last replay has completed.  The captured region
// holds kernel launches only (no memset, no copy, no event).  Per-pass event
// timing, and the no-alloc form (graph objects are allocations), launch
// every iteration directly.
constexpr int kGraphMinIters = 8;
constexpr int kGraphGroup = 16;

void append_key(std::vector<char> &k, const void *p, size_t n)
{
    const char *c = static_cast<const char *>(p);
    k.insert(k.end(), c, c + n);
}

// Retire the current graph (with the event after its last replay) and
// destroy the retired graphs whose replays have completed; never waits.
rsf_status retire_graph(rsf_context *ctx)
{
    if (ctx->graph_exec) {
        ctx->retired.push_back({ctx->graph_exec, ctx->graph_ev});
        ctx->graph_exec = nullptr;
        ctx->graph_ev = nullptr;
        ctx->graph_key.clear();
    }
    std::vector<rsf_context::Retired> keep;
    for (const auto &r : ctx->retired) {
        if (!r.ev || hipEventQuery(r.ev) == hipSuccess) {
            HIP_TRY(hipGraphExecDestroy(r.exec), "hipGraphExecDestroy");
            if (r.ev) HIP_TRY(hipEventDestroy(r.ev), "hipEventDestroy(graph)");
        } else {
            keep.push_back(r);
        }
    }
    ctx->retired.swap(keep);
    return RSF_OK;
}

rsf_status run_iterations(rsf_context *ctx, const Plan &P, int iters, hipStream_t s, bool fused,
                          bool allow_graph)
{
    int done = 0;
    if (allow_graph && ctx->graphs && !ctx->prof && iters >= kGraphMinIters) {
        const int G = std::min(iters, kGraphGroup);
        std::vector<char> key;
        append_key(key, &G, sizeof(G));
        append_key(key, &fused, sizeof(fused));
        append_key(key, &P.R, sizeof(P.R));
        append_key(key, &P.image, sizeof(P.image));
        append_key(key, &P.storage, sizeof(P.storage));
        append_key(key, &P.taps, sizeof(P.taps));
        append_key(key, &P.c, sizeof(P.c));
        for (const Batch *b : {&P.xy, &P.z, &P.u, &P.tile}) append_key(key, b, sizeof(Batch));
        for (const int64_t *v : {&P.blocks_xy, &P.blocks_z, &P.blocks_u})
            append_key(key, v, sizeof(*v));
        append_key(key, &P.k2, sizeof(P.k2));
        if (!ctx->graph_exec || key != ctx->graph_key) {
            rsf_status st = retire_graph(ctx);
            if (st != RSF_OK) return st;
            if (!ctx->cap_stream)
                HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking),
                        "hipStreamCreate(capture)");
            // A capture or instantiation the runtime refuses leaves the
            // iterations to the direct launches below; a launch error inside
            // the capture is the call's error.
            hipGraphExec_t exec = nullptr;
            if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) ==
                hipSuccess) {
                for (int k = 0; k < G && st == RSF_OK; ++k)
                    st = iteration(ctx, P, false, ctx->cap_stream, fused);
                hipGraph_t graph = nullptr;
                const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
                if (st == RSF_OK && ec == hipSuccess &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                    exec = nullptr;
                if (graph) (void)hipGraphDestroy(graph);
                if (st != RSF_OK) return st;
            }
            (void)hipGetLastError();   // a refused capture leaves no error behind
            ctx->graph_exec = exec;
            if (exec) ctx->graph_key = std::move(key);
        }
        if (ctx->graph_exec) {
            for (; done + G <= iters; done += G)
                HIP_TRY(hipGraphLaunch(ctx->graph_exec, s), "hipGraphLaunch");
            if (!ctx->graph_ev)
                HIP_TRY(hipEventCreateWithFlags(&ctx->graph_ev, hipEventDisableTiming),
                        "hipEventCreate(graph)");
            HIP_TRY(hipEventRecord(ctx->graph_ev, s), "hipEventRecord(graph)");
        }
    }
    for (; done < iters; ++done) {
        const rsf_status st = iteration(ctx, P, false, s, fused);
        if (st != RSF_OK) return st;
    }
    return RSF_OK;
}

// `fixed`: the no-alloc form.  The workspace is the device's `scratch`
// array (in `workspace`), the tile table is written by a kernel, and no
// per-pass events or graphs are made, so nothing is allocated.
rsf_status evolve_impl(rsf_context *ctx, const rsf_tile *tiles, int n, int vdt,
                       const rsf_params &p, int iters, double tol, void *workspace,
                       size_t ws_bytes, void *stream, bool fixed = false)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    ctx->err.clear();
    rsf_status st = check_tiles(ctx, tiles, n, true);
    if (st != RSF_OK) return st;
    st = check_params(ctx, p);
    if (st != RSF_OK) return st;
    st = check_types(ctx, p, vdt);
    if (st != RSF_OK) return st;
    if (iters < 0) return fail(ctx, RSF_ERR_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol))
        return fail(ctx, RSF_ERR_INVALID_ARG, "tol must be >= 0");
    st = set_device(ctx);
    if (st != RSF_OK) return st;
    const size_t need = plan_layout(tiles, n, iters, p.storage,
                                    splits_for(ctx, tiles, n, radius_of(p.sigma)),
                                    rsf::host::needs_k2(p))
                            .total;
    if (fixed && ws_bytes < need)
        return fail(ctx, RSF_ERR_INVALID_ARG,
                    "volume too large for the no-alloc workspace (RSF_NOALLOC_MAX_BYTES)");
    if (workspace && ws_bytes < need) return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (!workspace) {
        st = ensure_ws(ctx, need);
        if (st != RSF_OK) return st;
    }
    char *base = static_cast<char *>(workspace ? workspace : ctx->ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!workspace) {
        st = ws_enter(ctx, s);
        if (st != RSF_OK) return st;
    }
    Plan P;
    st = make_plan(ctx, P, tiles, n, vdt, p, tol, iters, base, s, nullptr, nullptr, fixed);
    if (st != RSF_OK) return st;
    st = prologue(ctx, P, s);
    if (st != RSF_OK) return st;
    const bool fused = P.fuse && iters > 0 && ctx->fuse;
    if (fused) {
        st = stage1(ctx, P, false, s);
        if (st != RSF_OK) return st;
    }
    st = run_iterations(ctx, P, iters, s, fused, !fixed);
    if (st != RSF_OK) return st;
    // tiles that ended on an odd iteration have it in the workspace buffer
    if (iters > 0) HIP_TRY(rsf::launch_finish(P.z, P.blocks_z, s), "finish");
    if (!workspace) {
        st = ws_leave(ctx, s);
        if (st != RSF_OK) return st;
    }
    ctx->last_stream = s;
    ctx->last_hist.clear();
    ctx->last_flags.clear();
    for (int t = 0; t < n; ++t) {
        const TileLayout &T = P.L.tiles[t];
        ctx->last_hist.push_back(reinterpret_cast<const double *>(base + T.base + T.T.hist));
        ctx->last_flags.push_back(reinterpret_cast<const int *>(base + T.base + T.T.flags));
    }
    ctx->last_iters = iters;
    ctx->has_last = true;
    return RSF_OK;
}

// Candidate workgroup targets of the autotuner's coordinate search.
constexpr int64_t kCandXy[] = {2048, 4096, 8192, 16384, 32768};
constexpr int64_t kCandZ[] = {256, 512, 1024, 2048, 4096};
constexpr int64_t kCandU[] = {128, 256, 512, 1024, 2048};

// Device bytes of the autotuner's copies of the tiles' phi.
size_t autotune_copy_bytes(const rsf_tile *tiles, int n)
{
    size_t total = 0;
    for (int t = 0; t < n; ++t)
        total += align_up((size_t)tiles[t].nx * tiles[t].ny * tiles[t].nz * sizeof(float));
    return total;
}

// Batch workspace of the autotuner's largest trial: every split its
// coordinate search can set (each target a candidate or the context's own),
// for trial_iters + 1 iterations.
size_t autotune_trial_ws(rsf_context *ctx, const rsf_tile *tiles, int n, const rsf_params &p,
                         int trial_iters)
{
    const int R = radius_of(p.sigma);
    const std::vector<double> sh = shares_of(tiles, n);
    std::vector<int64_t> xs(std::begin(kCandXy), std::end(kCandXy));
    std::vector<int64_t> zs(std::begin(kCandZ), std::end(kCandZ));
    std::vector<int64_t> us(std::begin(kCandU), std::end(kCandU));
    xs.push_back(ctx->targets.xy);
    zs.push_back(ctx->targets.z);
    us.push_back(ctx->targets.u);
    size_t most = plan_layout(tiles, n, trial_iters + 1, p.storage, splits_for(ctx, tiles, n, R),
                              rsf::host::needs_k2(p))
                      .total;
    std::vector<Split> sp((size_t)n);
    for (int64_t a : xs)
        for (int64_t b : zs)
            for (int64_t c : us) {
                for (int t = 0; t < n; ++t) {
                    const Grid3 g = grid_of(tiles[t]);
                    const auto part = [&](int64_t v) {
                        return (int64_t)std::max(1.0, std::ceil((double)v * sh[t]));
                    };
                    // a candidate the tile cannot take leaves it on its base split
                    const Split c1 = rsf::make_split(g, part(a), part(b), part(c));
                    sp[(size_t)t] = rsf::split_valid(g, c1) ? c1 : base_split(ctx, g, sh[t], n, R);
                }
                most = std::max(most, plan_layout(tiles, n, trial_iters + 1, p.storage, sp,
                                                  rsf::host::needs_k2(p))
                                          .total);
            }
    return most;
}

// Time `iters` iterations of a planned batch (after its prologue) in ms.
rsf_status time_iterations(rsf_context *ctx, const Plan &P, int iters, hipStream_t s, float *ms,
                           bool fused)
{
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(ctx, e, "hipEventCreate");
    }
    rsf_status st = RSF_OK;
    e = hipEventRecord(a, s);
    for (int it = 0; st == RSF_OK && e == hipSuccess && it < iters; ++it)
        st = iteration(ctx, P, false, s, fused);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != RSF_OK) return st;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune timing");
    return RSF_OK;
}

rsf_params default_params(float sigma, float l1, float l2, float nu, float mu, float dt,
                          float eps)
{
    rsf_params p{};
    p.sigma = sigma; p.lambda1 = l1; p.lambda2 = l2; p.nu = nu; p.mu = mu; p.dt = dt;
    p.eps = eps; p.eta = 1e-10f; p.regulariser = RSF_REG_DOUBLE_WELL; p.storage = RSF_F32;
    p.force = RSF_FORCE_RSF; p.sigma2 = 0.f;
    return p;
}

rsf_status tile_stats(rsf_context *ctx, int tile, rsf_stats *out, double *s_hist, int cap)
{
    if (!ctx || !out) return fail(ctx, RSF_ERR_INVALID_ARG, "null argument");
    if (!ctx->has_last) return fail(ctx, RSF_ERR_INVALID_ARG, "no evolution has run");
    if (tile < 0 || tile >= (int)ctx->last_hist.size())
        return fail(ctx, RSF_ERR_INVALID_ARG, "tile index out of range");
    rsf_status st = set_device(ctx);
    if (st != RSF_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->last_stream), "hipStreamSynchronize");
    int flags[2] = {0, 0};
    HIP_TRY(hipMemcpy(flags, ctx->last_flags[tile], sizeof(flags), hipMemcpyDeviceToHost),
            "copy flags");
    out->iters_requested = ctx->last_iters;
    out->iters_run = flags[1];
    out->last_sum_abs = 0.0;
    const int n = flags[1];
    if (n > 0) {
        HIP_TRY(hipMemcpy(&out->last_sum_abs, ctx->last_hist[tile] + (n - 1), sizeof(double),
                          hipMemcpyDeviceToHost),
                "copy last sum");
    }
    if (s_hist && cap > 0 && n > 0) {
        const int m = cap < n ? cap : n;
        HIP_TRY(hipMemcpy(s_hist, ctx->last_hist[tile], (size_t)m * sizeof(double),
                          hipMemcpyDeviceToHost),
                "copy history");
    }
    if (!std::isfinite(out->last_sum_abs))
        return fail(ctx, RSF_ERR_NONFINITE, "non-finite sum |dphi|");
    return RSF_OK;
}

}  // namespace

extern "C" {

rsf_status rsf_create(rsf_context **out, int device_ordinal)
{
    if (!out) return RSF_ERR_INVALID_ARG;
    *out = nullptr;
    if (rsf::g_fault_env_bad) return RSF_ERR_INVALID_ARG;
    try {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device_ordinal < 0 || device_ordinal >= n)
            return RSF_ERR_INVALID_ARG;
        void *sp = nullptr;
        if (scratch_address(device_ordinal, &sp) != hipSuccess) return RSF_ERR_DEVICE;
        rsf_context *c = new (std::nothrow) rsf_context();
        if (!c) return RSF_ERR_OUT_OF_MEMORY;
        c->device = device_ordinal;
        c->noalloc_ws = sp;
        *out = c;
        return RSF_OK;
    } catch (...) {
        return RSF_ERR_INTERNAL;
    }
}

rsf_status rsf_set_fault(const char *spec)
{
    int64_t first = 0, count = 0;
    if (!rsf::parse_fault(spec, first, count)) return RSF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(rsf::g_fault_mu);
    rsf::g_fault_first = first;
    rsf::g_fault_count = count;
    rsf::g_fault_seen = 0;
    return RSF_OK;
}

int64_t rsf_fault_allocations(void)
{
    std::lock_guard<std::mutex> lock(rsf::g_fault_mu);
    return rsf::g_fault_first == 0 ? -1 : rsf::g_fault_seen;
}

void rsf_destroy(rsf_context *ctx)
{
    if (!ctx) return;
    try {
        (void)hipSetDevice(ctx->device);
        if (ctx->ws || !ctx->ev_pool.empty() || ctx->stage || ctx->graph_exec ||
            !ctx->retired.empty())
            (void)hipDeviceSynchronize();
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->stage) (void)hipHostFree(ctx->stage);
        if (ctx->stage_ev) (void)hipEventDestroy(ctx->stage_ev);
        if (ctx->ws_ev) (void)hipEventDestroy(ctx->ws_ev);
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph_ev) (void)hipEventDestroy(ctx->graph_ev);
        for (const auto &r : ctx->retired) {
            (void)hipGraphExecDestroy(r.exec);
            if (r.ev) (void)hipEventDestroy(r.ev);
        }
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    } catch (...) {
    }
    delete ctx;
}

rsf_status rsf_set_fusion(rsf_context *ctx, int on)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    ctx->fuse = on != 0;
    return RSF_OK;
}

rsf_status rsf_set_graphs(rsf_context *ctx, int on)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    ctx->graphs = on != 0;
    return RSF_OK;
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

size_t rsf_batch_workspace_bytes(const rsf_tile *tiles, int n, int iters, int storage)
{
    try {
        if (!tiles || n < 1 || iters < 0) return 0;
        if (storage != RSF_F32 && storage != RSF_F16 && storage != RSF_BF16) return 0;
        for (int t = 0; t < n; ++t)
            if (tiles[t].nx < 3 || tiles[t].ny < 3 || tiles[t].nz < 3) return 0;
        return plan_layout(tiles, n, iters, storage, splits_for(nullptr, tiles, n, 0)).total;
    } catch (...) {
        return 0;
    }
}

size_t rsf_workspace_bytes(int64_t nx, int64_t ny, int64_t nz, int iters, int storage)
{
    rsf_tile t{};
    t.nx = nx; t.ny = ny; t.nz = nz;
    return rsf_batch_workspace_bytes(&t, 1, iters, storage);
}

size_t rsf_batch_workspace_bytes_params(const rsf_tile *tiles, int n, int iters,
                                        const rsf_params *params)
{
    try {
        if (!tiles || n < 1 || iters < 0 || !params) return 0;
        if (rsf::host::params_error(*params)) return 0;
        for (int t = 0; t < n; ++t)
            if (tiles[t].nx < 3 || tiles[t].ny < 3 || tiles[t].nz < 3) return 0;
        return plan_layout(tiles, n, iters, params->storage, splits_for(nullptr, tiles, n, 0),
                           rsf::host::needs_k2(*params))
            .total;
    } catch (...) {
        return 0;
    }
}

size_t rsf_workspace_bytes_params(int64_t nx, int64_t ny, int64_t nz, int iters,
                                  const rsf_params *params)
{
    rsf_tile t{};
    t.nx = nx; t.ny = ny; t.nz = nz;
    return rsf_batch_workspace_bytes_params(&t, 1, iters, params);
}

rsf_status rsf_evolve(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                      int64_t nx, int64_t ny, int64_t nz, float sigma, float lambda1,
                      float lambda2, float nu, float mu, float dt, float eps, int iters,
                      void *stream)
{
    try {
        const rsf_params p = default_params(sigma, lambda1, lambda2, nu, mu, dt, eps);
        rsf_tile t{volume, phi, nx, ny, nz};
        return evolve_impl(ctx, &t, 1, volume_dtype, p, iters, 0.0, nullptr, 0, stream);
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
        rsf_tile t{volume, phi, nx, ny, nz};
        return evolve_impl(ctx, &t, 1, volume_dtype, *params, iters, tol, workspace,
                           workspace_bytes, stream);
    } catch (const std::bad_alloc &) {
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_evolve_noalloc(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                              int64_t nx, int64_t ny, int64_t nz, const rsf_params *params,
                              int iters, double tol, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        if (!params) return fail(ctx, RSF_ERR_INVALID_ARG, "null params");
        if (!ctx->noalloc_ws) return fail(ctx, RSF_ERR_DEVICE, "no-alloc workspace not found");
        rsf_tile t{volume, phi, nx, ny, nz};
        // no per-pass events: creating them could allocate (restored on
        // every exit, exceptions included)
        struct ProfOff {
            rsf_context *c;
            bool was;
            ~ProfOff() { c->prof = was; }
        } off{ctx, ctx->prof};
        ctx->prof = false;
        return evolve_impl(ctx, &t, 1, volume_dtype, *params, iters, tol, ctx->noalloc_ws,
                           RSF_NOALLOC_MAX_BYTES, stream, true);
    } catch (const std::bad_alloc &) {
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_evolve_batch(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                            int volume_dtype, const rsf_params *params, int iters, double tol,
                            void *workspace, size_t workspace_bytes, void *stream)
{
    try {
        if (!params) return fail(ctx, RSF_ERR_INVALID_ARG, "null params");
        return evolve_impl(ctx, tiles, n_tiles, volume_dtype, *params, iters, tol, workspace,
                           workspace_bytes, stream);
    } catch (const std::bad_alloc &) {
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_get_stats(rsf_context *ctx, rsf_stats *out, double *s_hist, int cap)
{
    try {
        return tile_stats(ctx, 0, out, s_hist, cap);
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_get_tile_stats(rsf_context *ctx, int tile, rsf_stats *out, double *s_hist,
                              int cap)
{
    try {
        return tile_stats(ctx, tile, out, s_hist, cap);
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_set_split_targets(rsf_context *ctx, int64_t xy_waves, int64_t z_blocks,
                                 int64_t u_blocks)
{
    if (!ctx) return RSF_ERR_INVALID_ARG;
    if (xy_waves < 0 || z_blocks < 0 || u_blocks < 0 || xy_waves > (1 << 24) ||
        z_blocks > (1 << 24) || u_blocks > (1 << 24))
        return fail(ctx, RSF_ERR_INVALID_ARG, "targets must be in 0..2^24");
    ctx->targets.xy = xy_waves ? xy_waves : rsf::kDefaultTargets.xy;
    ctx->targets.z = z_blocks ? z_blocks : rsf::kDefaultTargets.z;
    ctx->targets.u = u_blocks ? u_blocks : rsf::kDefaultTargets.u;
    return RSF_OK;
}

rsf_status rsf_autotune(rsf_context *ctx, const rsf_tile *tiles, int n_tiles, int volume_dtype,
                        const rsf_params *params, int trial_iters, int64_t *chosen,
                        void *stream)
{
    return rsf_autotune_ex(ctx, tiles, n_tiles, volume_dtype, params, trial_iters, chosen,
                           nullptr, 0, stream);
}

size_t rsf_autotune_workspace_bytes(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                                    const rsf_params *params, int trial_iters)
{
    try {
        if (!ctx || !params || trial_iters < 1) return 0;
        if (check_tiles(nullptr, tiles, n_tiles, false) != RSF_OK) return 0;
        if (check_params(nullptr, *params) != RSF_OK) return 0;
        return autotune_copy_bytes(tiles, n_tiles) +
               autotune_trial_ws(ctx, tiles, n_tiles, *params, trial_iters);
    } catch (...) {
        return 0;
    }
}

rsf_status rsf_autotune_ex(rsf_context *ctx, const rsf_tile *tiles, int n_tiles,
                           int volume_dtype, const rsf_params *params, int trial_iters,
                           int64_t *chosen, void *workspace, size_t workspace_bytes,
                           void *stream)
{
    float *trial_phi = nullptr;   // owned (freed here) unless in the caller's workspace
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        if (!params) return fail(ctx, RSF_ERR_INVALID_ARG, "null params");
        rsf_status st = check_tiles(ctx, tiles, n_tiles, true);
        if (st != RSF_OK) return st;
        st = check_params(ctx, *params);
        if (st != RSF_OK) return st;
        st = check_types(ctx, *params, volume_dtype);
        if (st != RSF_OK) return st;
        if (trial_iters < 1) return fail(ctx, RSF_ERR_INVALID_ARG, "trial_iters must be >= 1");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int R = radius_of(params->sigma);
        // trials evolve copies of phi, never the caller's
        size_t total = 0;
        std::vector<size_t> off;
        for (int t = 0; t < n_tiles; ++t) {
            off.push_back(total);
            total += align_up((size_t)tiles[t].nx * tiles[t].ny * tiles[t].nz * sizeof(float));
        }
        const size_t trial_ws = workspace ? autotune_trial_ws(ctx, tiles, n_tiles, *params,
                                                              trial_iters)
                                          : 0;
        if (workspace && workspace_bytes < total + trial_ws)
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        char *const trial_base = workspace ? static_cast<char *>(workspace) + total : nullptr;
        if (workspace) trial_phi = static_cast<float *>(workspace);
        else HIP_TRY(rsf::dev_alloc(&trial_phi, total), "hipMalloc(autotune trial_phi)");
        auto release = [&] {
            if (!workspace && trial_phi) (void)hipFree(trial_phi);
            trial_phi = nullptr;
        };
        std::vector<rsf_tile> tt(tiles, tiles + n_tiles);
        for (int t = 0; t < n_tiles; ++t) {
            tt[t].phi = reinterpret_cast<float *>(reinterpret_cast<char *>(trial_phi) + off[t]);
            const size_t bytes = (size_t)tiles[t].nx * tiles[t].ny * tiles[t].nz * sizeof(float);
            hipError_t e = hipMemcpyAsync(tt[t].phi, tiles[t].phi, bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) {
                release();
                return hip_fail(ctx, e, "autotune copy");
            }
        }
        // coordinate search over the three per-pass workgroup targets,
        // starting from the context's
        const int64_t *const cand_xy = kCandXy, *const cand_z = kCandZ, *const cand_u = kCandU;
        int64_t best[3] = {ctx->targets.xy, ctx->targets.z, ctx->targets.u};
        // targets are for the whole batch; each tile gets its voxel share
        const std::vector<double> sh = shares_of(tiles, n_tiles);
        auto apply = [&](const int64_t tg[3]) {
            for (int t = 0; t < n_tiles; ++t) {
                const Grid3 g = grid_of(tiles[t]);
                const auto part = [&](int64_t v) {
                    return (int64_t)std::max(1.0, std::ceil((double)v * sh[t]));
                };
                ctx->tuned[{g.nx, g.ny, g.nz, R}] =
                    rsf::make_split(g, part(tg[0]), part(tg[1]), part(tg[2]));
            }
        };
        // time what rsf_evolve_batch would run under the current splits and
        // schedule: one warm-up iteration, then the timed ones
        auto trial = [&](float &ms) -> rsf_status {
            const int runs = trial_iters + 1;
            const size_t need = plan_layout(tt.data(), n_tiles, runs, params->storage,
                                            splits_for(ctx, tt.data(), n_tiles, R),
                                            rsf::host::needs_k2(*params))
                                    .total;
            rsf_status r = RSF_OK;
            if (!workspace) {
                r = ensure_ws(ctx, need);
                if (r == RSF_OK) r = ws_enter(ctx, s);
                if (r != RSF_OK) return r;
                ctx->has_last = false;   // the trials overwrite the workspace
            } else if (need > trial_ws) {
                return fail(ctx, RSF_ERR_INTERNAL, "autotune trial outgrew its workspace");
            }
            Plan P;
            r = make_plan(ctx, P, tt.data(), n_tiles, volume_dtype, *params, 0.0, runs,
                          workspace ? trial_base : static_cast<char *>(ctx->ws), s);
            if (r == RSF_OK) r = prologue(ctx, P, s);
            const bool fused = P.fuse && ctx->fuse;
            if (r == RSF_OK && fused) r = stage1(ctx, P, false, s);
            if (r == RSF_OK) r = iteration(ctx, P, false, s, fused);   // warm-up
            if (r == RSF_OK) r = time_iterations(ctx, P, trial_iters, s, &ms, fused);
            if (r == RSF_OK && !workspace) r = ws_leave(ctx, s);
            return r;
        };
        // The splits are searched with the passes separate (all three
        // targets then matter); then the schedule: the update fused with
        // the next stage-1 pass (each tile one update chunk) against the
        // separate passes, where the force and radius allow fusing.
        const std::vector<int64_t> skey = schedule_key(tiles, n_tiles, *params, volume_dtype);
        ctx->tuned_fuse.erase(skey);
        const bool can_fuse = fusable(ctx, *params, false, volume_dtype);
        ctx->force_schedule = 0;
        float best_ms = -1.f;
        for (int axis = 0; axis < 3; ++axis) {
            const int64_t *cands = axis == 0 ? cand_xy : (axis == 1 ? cand_z : cand_u);
            const int nc = 5;
            int64_t keep = best[axis];
            for (int c = 0; c < nc; ++c) {
                int64_t tg[3] = {best[0], best[1], best[2]};
                tg[axis] = cands[c];
                apply(tg);
                float ms = 0.f;
                st = trial(ms);
                if (st != RSF_OK) break;
                if (best_ms < 0.f || ms < best_ms) {
                    best_ms = ms;
                    keep = cands[c];
                }
            }
            if (st != RSF_OK) break;
            best[axis] = keep;
        }
        int fused_choice = 0;
        if (st == RSF_OK) {
            apply(best);
            if (can_fuse) {
                float sep = 0.f, fus = 0.f;
                st = trial(sep);
                ctx->force_schedule = 1;
                if (st == RSF_OK) st = trial(fus);
                if (st == RSF_OK) {
                    fused_choice = fus < sep ? 1 : 0;
                    ctx->tuned_fuse[skey] = fused_choice == 1;
                }
            }
        }
        ctx->force_schedule = -1;
        if (st == RSF_OK) {
            if (chosen) {
                chosen[0] = best[0];
                chosen[1] = best[1];
                chosen[2] = best[2];
                chosen[3] = fused_choice;
            }
        } else {
            for (int t = 0; t < n_tiles; ++t)
                ctx->tuned.erase({tiles[t].nx, tiles[t].ny, tiles[t].nz, R});
        }
        (void)hipStreamSynchronize(s);
        release();
        return st;
    } catch (...) {
        if (ctx) ctx->force_schedule = -1;
        if (trial_phi && !workspace) (void)hipFree(trial_phi);
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

void rsf_autotune_reset(rsf_context *ctx)
{
    if (!ctx) return;
    ctx->tuned.clear();
    ctx->tuned_fuse.clear();
}

}  // extern "C"

namespace {

// The volume driver's plan: curtained sub-volume boxes, their grouping
// under the budget, and the device memory one call needs (merge buffer,
// sub-volume copies of the largest group, batch workspace of the largest
// group, in that order, each 256-byte aligned).
struct VolPlan {
    int C = 0;
    std::vector<rsf::SubBox> boxes;
    std::vector<std::pair<size_t, size_t>> groups;   // [first, last)
    size_t acc_bytes = 0, copy_bytes = 0, ws_bytes = 0;
    size_t total() const { return acc_bytes + copy_bytes + ws_bytes; }
};

rsf_status volume_plan(rsf_context *ctx, int volume_dtype, int64_t nx, int64_t ny, int64_t nz,
                       int64_t block, int64_t curtain, const rsf_params &p, int iters,
                       size_t budget_bytes, VolPlan &V)
{
    rsf_status st = check_dims(ctx, nx, ny, nz);
    if (st != RSF_OK) return st;
    st = check_params(ctx, p);
    if (st != RSF_OK) return st;
    st = check_types(ctx, p, volume_dtype);
    if (st != RSF_OK) return st;
    if (iters < 0) return fail(ctx, RSF_ERR_INVALID_ARG, "iters must be >= 0");
    if (block < 1) return fail(ctx, RSF_ERR_INVALID_ARG, "block must be >= 1");
    if (curtain < 0) return fail(ctx, RSF_ERR_INVALID_ARG, "curtain must be >= 0");
    V.C = (int)(curtain > 0 ? curtain : std::ceil(3.0 * std::max(p.sigma, p.sigma2) - 1e-9));
    const int C = V.C;
    // near-equal cores per axis; neighbours overlap by 2C around each core face
    const int64_t n3[3] = {nx, ny, nz};
    std::vector<int64_t> cuts[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t nb = (n3[a] + block - 1) / block;
        for (int64_t k = 0; k <= nb; ++k) cuts[a].push_back(k * n3[a] / nb);
        if (nb > 1 && n3[a] / nb < 2 * C)
            return fail(ctx, RSF_ERR_INVALID_ARG,
                        "every core must be at least twice the curtain: raise block or lower "
                        "curtain");
    }
    for (size_t kz = 0; kz + 1 < cuts[2].size(); ++kz)
        for (size_t ky = 0; ky + 1 < cuts[1].size(); ++ky)
            for (size_t kx = 0; kx + 1 < cuts[0].size(); ++kx) {
                rsf::SubBox b{};
                const size_t k[3] = {kx, ky, kz};
                for (int a = 0; a < 3; ++a) {
                    const int64_t c0 = cuts[a][k[a]], c1 = cuts[a][k[a] + 1];
                    const int64_t lo = std::max<int64_t>(0, c0 - C);
                    const int64_t hi = std::min<int64_t>(n3[a], c1 + C);
                    b.lo[a] = (int)lo;
                    b.ext[a] = (int)(hi - lo);
                    b.core_lo[a] = (int)c0;
                    b.core_hi[a] = (int)c1;
                    b.nb_lo[a] = k[a] > 0;
                    b.nb_hi[a] = k[a] + 2 < cuts[a].size();
                }
                V.boxes.push_back(b);
            }
    // group the boxes so each group's copies and workspace fit the budget
    const size_t elem = volume_dtype == RSF_U16 ? 2 : 4;
    auto copies_of = [&](const rsf::SubBox &b) {
        const size_t v = (size_t)b.ext[0] * b.ext[1] * b.ext[2];
        return align_up(v * elem) + align_up(v * 4);
    };
    auto box_bytes = [&](const rsf::SubBox &b) {
        const Grid3 g = rsf::host::grid_of(b.ext[0], b.ext[1], b.ext[2]);
        return copies_of(b) +
               rsf::host::tile_regions(g, iters, p.storage, rsf::host::needs_k2(p)).total +
               2 * kAlign;
    };
    size_t first = 0, sum = 0;
    for (size_t i = 0; i < V.boxes.size(); ++i) {
        const size_t bb = box_bytes(V.boxes[i]);
        if (budget_bytes && bb > budget_bytes)
            return fail(ctx, RSF_ERR_BUDGET, "one sub-volume alone exceeds the budget");
        if (budget_bytes && sum + bb > budget_bytes) {
            V.groups.push_back({first, i});
            first = i;
            sum = 0;
        }
        sum += bb;
    }
    V.groups.push_back({first, V.boxes.size()});
    V.acc_bytes = align_up((size_t)(nx * ny * nz) * sizeof(float));
    const int R = radius_of(p.sigma);
    for (auto &gr : V.groups) {
        size_t c = 0;
        std::vector<rsf_tile> tiles;
        for (size_t i = gr.first; i < gr.second; ++i) {
            c += copies_of(V.boxes[i]);
            const rsf::SubBox &b = V.boxes[i];
            tiles.push_back(rsf_tile{nullptr, nullptr, b.ext[0], b.ext[1], b.ext[2]});
        }
        V.copy_bytes = std::max(V.copy_bytes, c);
        // the batch workspace as evolve_impl sizes it for this context
        const size_t need = plan_layout(tiles.data(), (int)tiles.size(), iters, p.storage,
                                        splits_for(ctx, tiles.data(), (int)tiles.size(), R),
                                        rsf::host::needs_k2(p))
                                .total;
        V.ws_bytes = std::max(V.ws_bytes, align_up(need));
    }
    return RSF_OK;
}

}  // namespace

extern "C" {

size_t rsf_volume_workspace_bytes(rsf_context *ctx, int volume_dtype, int64_t nx, int64_t ny,
                                  int64_t nz, int64_t block, int64_t curtain,
                                  const rsf_params *params, int iters, size_t budget_bytes)
{
    try {
        if (!ctx || !params) return 0;
        VolPlan V;
        if (volume_plan(ctx, volume_dtype, nx, ny, nz, block, curtain, *params, iters,
                        budget_bytes, V) != RSF_OK)
            return 0;
        return V.total();
    } catch (...) {
        return 0;
    }
}

rsf_status rsf_evolve_volume_ex(rsf_context *ctx, const void *volume, int volume_dtype,
                                float *phi, int64_t nx, int64_t ny, int64_t nz, int64_t block,
                                int64_t curtain, const rsf_params *params, int iters,
                                size_t budget_bytes, void *workspace, size_t workspace_bytes,
                                void *stream)
{
    std::vector<void *> owned;
    auto release = [&] {
        for (void *q : owned) (void)hipFree(q);
        owned.clear();
    };
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        if (!volume || !phi || !params) return fail(ctx, RSF_ERR_INVALID_ARG, "null argument");
        VolPlan V;
        rsf_status st = volume_plan(ctx, volume_dtype, nx, ny, nz, block, curtain, *params, iters,
                                    budget_bytes, V);
        if (st != RSF_OK) return st;
        if (workspace && workspace_bytes < V.total())
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int C = V.C;
        const size_t elem = volume_dtype == RSF_U16 ? 2 : 4;
        const int64_t nvox = nx * ny * nz;
        float *acc = nullptr;
        char *copies = nullptr;
        void *batch_ws = nullptr;   // null: the context's own workspace
        if (workspace) {
            char *w = static_cast<char *>(workspace);
            acc = reinterpret_cast<float *>(w);
            copies = w + V.acc_bytes;
            batch_ws = w + V.acc_bytes + V.copy_bytes;
        } else {
            HIP_TRY(rsf::dev_alloc(&acc, (size_t)nvox * sizeof(float)), "hipMalloc(merge accumulator)");
            owned.push_back(acc);
            const hipError_t e = rsf::dev_alloc(&copies, V.copy_bytes);
            if (e != hipSuccess) {
                release();
                return hip_fail(ctx, e, "hipMalloc(sub-volume copies)");
            }
            owned.push_back(copies);
        }
        auto step = [&](hipError_t e, const char *what) -> rsf_status {
            if (e == hipSuccess) return RSF_OK;
            (void)hipStreamSynchronize(s);
            release();
            return hip_fail(ctx, e, what);
        };
        st = step(rsf::launch_fill(acc, nvox, 0.f, s), "fill");
        if (st != RSF_OK) return st;
        for (auto &gr : V.groups) {
            std::vector<rsf_tile> tiles;
            size_t off = 0;
            for (size_t i = gr.first; i < gr.second; ++i) {
                const rsf::SubBox &b = V.boxes[i];
                const size_t v = (size_t)b.ext[0] * b.ext[1] * b.ext[2];
                void *img = copies + off;
                off += align_up(v * elem);
                float *ph = reinterpret_cast<float *>(copies + off);
                off += align_up(v * 4);
                st = step(rsf::launch_gather(volume, img, (int)elem, nx, ny, b, s), "gather image");
                if (st == RSF_OK) st = step(rsf::launch_gather(phi, ph, 4, nx, ny, b, s), "gather phi");
                if (st != RSF_OK) return st;
                tiles.push_back(rsf_tile{img, ph, b.ext[0], b.ext[1], b.ext[2]});
            }
            st = evolve_impl(ctx, tiles.data(), (int)tiles.size(), volume_dtype, *params, iters,
                             0.0, batch_ws, batch_ws ? V.ws_bytes : 0, stream);
            if (st != RSF_OK) {
                (void)hipStreamSynchronize(s);
                release();
                return st;
            }
            for (size_t i = gr.first; i < gr.second; ++i) {
                st = step(rsf::launch_merge(acc, tiles[i - gr.first].phi, nx, ny, V.boxes[i], C, s),
                          "merge");
                if (st != RSF_OK) return st;
            }
        }
        st = step(hipMemcpyAsync(phi, acc, (size_t)nvox * sizeof(float), hipMemcpyDeviceToDevice, s),
                  "copy merged phi");
        if (st != RSF_OK) return st;
        const hipError_t e = hipStreamSynchronize(s);
        release();
        ctx->has_last = false;   // per-tile statistics of the groups are not kept
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
        return RSF_OK;
    } catch (const std::bad_alloc &) {
        release();
        return fail(ctx, RSF_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        release();
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_evolve_volume(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                             int64_t nx, int64_t ny, int64_t nz, int64_t block, int64_t curtain,
                             const rsf_params *params, int iters, size_t budget_bytes, void *stream)
{
    return rsf_evolve_volume_ex(ctx, volume, volume_dtype, phi, nx, ny, nz, block, curtain,
                                params, iters, budget_bytes, nullptr, 0, stream);
}

}  // extern "C"

namespace {

// Device scratch of one call: allocated and freed on every exit, or carved
// (256-byte aligned pieces) from a caller's workspace.
struct Scratch {
    std::vector<void *> p;
    char *arena = nullptr;
    size_t left = 0;
    Scratch() = default;
    Scratch(void *base, size_t bytes) : arena(static_cast<char *>(base)), left(bytes) {}
    ~Scratch()
    {
        for (void *q : p) (void)hipFree(q);
    }
    template <class T>
    hipError_t get(T **out, size_t bytes)
    {
        *out = nullptr;
        if (arena) {
            const size_t b = align_up(bytes ? bytes : 1);
            if (b > left) return hipErrorOutOfMemory;
            *out = reinterpret_cast<T *>(arena);
            arena += b;
            left -= b;
            return hipSuccess;
        }
        void *q = nullptr;
        const hipError_t e = rsf::dev_alloc(&q, bytes ? bytes : 1);
        if (e == hipSuccess) p.push_back(q);
        *out = static_cast<T *>(q);
        return e;
    }
};

// Device bytes of the seed detection's scratch (the pieces Scratch::get
// takes in rsf_seeds: the distance field, then those of seeds_impl), and of
// the initialisation's (rsf_init_phi: the mask first).
size_t seeds_scratch_bytes(int64_t n)
{
    return align_up((size_t)n * 4) + 3 * align_up((size_t)n * 4) + align_up(65536 * 4) +
           align_up(4) + align_up(65536 * 4);
}

size_t init_scratch_bytes(int64_t n) { return align_up((size_t)n) + seeds_scratch_bytes(n); }

rsf_status check_seed_args(rsf_context *ctx, const void *volume, int vdt, int64_t nx, int64_t ny,
                           int64_t nz, float sigma_b, float threshold)
{
    if (!volume) return fail(ctx, RSF_ERR_INVALID_ARG, "null volume");
    rsf_status st = check_dims(ctx, nx, ny, nz);
    if (st != RSF_OK) return st;
    if (nx < 2 || ny < 2) return fail(ctx, RSF_ERR_INVALID_ARG, "seeds need nx, ny >= 2");
    if (ny * nz > (int64_t(1) << 31)) return fail(ctx, RSF_ERR_INVALID_ARG, "ny * nz above 2^31");
    if (vdt != RSF_F32 && vdt != RSF_U16)
        return fail(ctx, RSF_ERR_INVALID_ARG, "volume dtype must be RSF_F32 or RSF_U16");
    if (!std::isfinite(sigma_b) || !(sigma_b > 0.f) || radius_of(sigma_b) > rsf::kMaxR)
        return fail(ctx, RSF_ERR_INVALID_ARG, "sigma_b must be > 0 with ceil(3 sigma_b) <= 16");
    if (!std::isfinite(threshold) || threshold < 0.f || threshold >= 1.f)
        return fail(ctx, RSF_ERR_INVALID_ARG, "threshold must be in [0, 1)");
    return RSF_OK;
}

// Seeds into mask and u (0 at seeds, far elsewhere); the count if asked.
rsf_status seeds_impl(rsf_context *ctx, Scratch &sc, const void *volume, int vdt, int64_t nx,
                      int64_t ny, int64_t nz, float sigma_b, float threshold, unsigned char *mask,
                      float *u, int64_t *n_seeds, hipStream_t s)
{
    const int64_t n = nx * ny * nz;
    const int R = radius_of(sigma_b);
    const Taps t = make_taps(sigma_b, R);
    float *A = nullptr, *B = nullptr, *tr = nullptr, *part = nullptr, *mx = nullptr;
    unsigned *cnt = nullptr;
    HIP_TRY(sc.get(&A, (size_t)n * 4), "hipMalloc(seed scratch)");
    HIP_TRY(sc.get(&B, (size_t)n * 4), "hipMalloc(seed scratch)");
    HIP_TRY(sc.get(&tr, (size_t)n * 4), "hipMalloc(seed scratch)");
    HIP_TRY(sc.get(&part, 65536 * 4), "hipMalloc(seed scratch)");
    HIP_TRY(sc.get(&mx, 4), "hipMalloc(seed scratch)");
    HIP_TRY(sc.get(&cnt, 65536 * 4), "hipMalloc(seed scratch)");
    int blocks = 0;
    // L = 2D Gaussian of each slice (A: x pass, B: y pass); doh into A
    HIP_TRY(timed(ctx, RSF_PASS_INIT_SMOOTH, s,
                  [&] { return rsf::launch_smooth_x(volume, vdt, A, nx, ny, nz, t, R, s); }),
            "smooth x");
    HIP_TRY(timed(ctx, RSF_PASS_INIT_SMOOTH, s,
                  [&] { return rsf::launch_smooth_y(A, B, nx, ny, nz, t, R, s); }),
            "smooth y");
    HIP_TRY(timed(ctx, RSF_PASS_INIT_HESSIAN, s,
                  [&] {
                      const hipError_t e = rsf::launch_hessian(B, A, tr, part, nx, ny, nz, &blocks, s);
                      return e != hipSuccess ? e : rsf::launch_max(part, blocks, mx, s);
                  }),
            "hessian");
    HIP_TRY(timed(ctx, RSF_PASS_INIT_SELECT, s,
                  [&] {
                      return rsf::launch_seeds(A, tr, mx, threshold, mask, u, cnt, nx, ny, nz, s);
                  }),
            "seeds");
    if (n_seeds) {
        std::vector<unsigned> h((size_t)blocks);
        HIP_TRY(hipMemcpyAsync(h.data(), cnt, (size_t)blocks * 4, hipMemcpyDeviceToHost, s),
                "copy counts");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        int64_t total = 0;
        for (unsigned c : h) total += c;
        *n_seeds = total;
    }
    return RSF_OK;
}

rsf_status sweep_impl(rsf_context *ctx, float *u, int64_t nx, int64_t ny, int64_t nz, int rounds,
                      hipStream_t s)
{
    const int64_t planes = rsf::sweep_block_planes(nx, ny, nz);
    for (int r = 0; r < rounds; ++r)
        for (int dir = 0; dir < 8; ++dir)
            for (int64_t h = 0; h < planes; ++h)
                HIP_TRY(timed(ctx, RSF_PASS_INIT_SWEEP, s,
                              [&] { return rsf::launch_sweep_blocks(u, nx, ny, nz, dir, h, s); }),
                        "sweep");
    return RSF_OK;
}

}  // namespace

extern "C" {

rsf_status rsf_seeds(rsf_context *ctx, const void *volume, int volume_dtype, int64_t nx,
                     int64_t ny, int64_t nz, float sigma_b, float threshold, unsigned char *mask,
                     int64_t *n_seeds, void *stream)
{
    return rsf_seeds_ex(ctx, volume, volume_dtype, nx, ny, nz, sigma_b, threshold, mask, n_seeds,
                        nullptr, 0, stream);
}

size_t rsf_seeds_workspace_bytes(int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1 || nx > (int64_t(1) << 40) / ny / nz) return 0;
    return seeds_scratch_bytes(nx * ny * nz);
}

rsf_status rsf_seeds_ex(rsf_context *ctx, const void *volume, int volume_dtype, int64_t nx,
                        int64_t ny, int64_t nz, float sigma_b, float threshold,
                        unsigned char *mask, int64_t *n_seeds, void *workspace,
                        size_t workspace_bytes, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        rsf_status st = check_seed_args(ctx, volume, volume_dtype, nx, ny, nz, sigma_b, threshold);
        if (st != RSF_OK) return st;
        if (!mask) return fail(ctx, RSF_ERR_INVALID_ARG, "null mask");
        if (workspace && workspace_bytes < seeds_scratch_bytes(nx * ny * nz))
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        Scratch sc = workspace ? Scratch(workspace, workspace_bytes) : Scratch();
        float *u = nullptr;
        HIP_TRY(sc.get(&u, (size_t)(nx * ny * nz) * 4), "hipMalloc(seed scratch)");
        st = seeds_impl(ctx, sc, volume, volume_dtype, nx, ny, nz, sigma_b, threshold, mask, u,
                        n_seeds, s);
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        return st;
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

rsf_status rsf_fast_sweep(rsf_context *ctx, float *u, int64_t nx, int64_t ny, int64_t nz,
                          int rounds, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        if (!u) return fail(ctx, RSF_ERR_INVALID_ARG, "null field");
        rsf_status st = check_dims(ctx, nx, ny, nz);
        if (st != RSF_OK) return st;
        if (rounds < 1 || rounds > 64) return fail(ctx, RSF_ERR_INVALID_ARG, "rounds must be in 1..64");
        if (ny * nz > (int64_t(1) << 31)) return fail(ctx, RSF_ERR_INVALID_ARG, "ny * nz above 2^31");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        return sweep_impl(ctx, u, nx, ny, nz, rounds, static_cast<hipStream_t>(stream));
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

size_t rsf_init_workspace_bytes(int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1 || nx > (int64_t(1) << 40) / ny / nz) return 0;
    return init_scratch_bytes(nx * ny * nz);
}

rsf_status rsf_init_phi(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                        int64_t nx, int64_t ny, int64_t nz, float sigma_b, float threshold,
                        float offset, int rounds, int64_t *n_seeds, void *stream)
{
    return rsf_init_phi_ex(ctx, volume, volume_dtype, phi, nx, ny, nz, sigma_b, threshold, offset,
                           rounds, n_seeds, nullptr, 0, stream);
}

rsf_status rsf_init_phi_ex(rsf_context *ctx, const void *volume, int volume_dtype, float *phi,
                           int64_t nx, int64_t ny, int64_t nz, float sigma_b, float threshold,
                           float offset, int rounds, int64_t *n_seeds, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    try {
        if (!ctx) return RSF_ERR_INVALID_ARG;
        ctx->err.clear();
        rsf_status st = check_seed_args(ctx, volume, volume_dtype, nx, ny, nz, sigma_b, threshold);
        if (st != RSF_OK) return st;
        if (!phi) return fail(ctx, RSF_ERR_INVALID_ARG, "null phi");
        if (!std::isfinite(offset)) return fail(ctx, RSF_ERR_INVALID_ARG, "offset must be finite");
        if (rounds < 1 || rounds > 64) return fail(ctx, RSF_ERR_INVALID_ARG, "rounds must be in 1..64");
        const int64_t n = nx * ny * nz;
        if (workspace && workspace_bytes < init_scratch_bytes(n))
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace too small");
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
            return fail(ctx, RSF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        Scratch sc = workspace ? Scratch(workspace, workspace_bytes) : Scratch();
        unsigned char *mask = nullptr;
        float *u = nullptr;
        HIP_TRY(sc.get(&mask, (size_t)n), "hipMalloc(seed scratch)");
        HIP_TRY(sc.get(&u, (size_t)n * 4), "hipMalloc(seed scratch)");
        int64_t count = 0;
        st = seeds_impl(ctx, sc, volume, volume_dtype, nx, ny, nz, sigma_b, threshold, mask, u,
                        &count, s);
        if (st != RSF_OK) return st;
        if (n_seeds) *n_seeds = count;
        if (count == 0) return fail(ctx, RSF_ERR_INVALID_ARG, "no seed found (lower threshold)");
        st = sweep_impl(ctx, u, nx, ny, nz, rounds, s);
        if (st != RSF_OK) return st;
        HIP_TRY(timed(ctx, RSF_PASS_INIT_OFFSET, s,
                      [&] { return rsf::launch_offset(u, phi, n, offset, s); }),
                "offset");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        return RSF_OK;
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
        rsf_status st = check_dims(ctx, nx, ny, nz);
        if (st != RSF_OK) return st;
        if (!std::isfinite(sigma) || !(sigma > 0.f) || radius_of(sigma) > rsf::kMaxR)
            return fail(ctx, RSF_ERR_INVALID_ARG, "sigma must be > 0 with ceil(3 sigma) <= 16");
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        // the K*I prologue of a one-tile batch with I = in and K*I -> out
        rsf_tile t{in, nullptr, nx, ny, nz};
        const rsf_params p = default_params(sigma, 1, 1, 0, 0, 1, 1);
        st = ensure_ws(ctx, plan_layout(&t, 1, 0, RSF_F32,
                                        splits_for(ctx, &t, 1, radius_of(sigma)))
                                .total);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        st = ws_enter(ctx, s);
        if (st != RSF_OK) return st;
        ctx->has_last = false;   // the workspace is reused
        Plan P;
        st = make_plan(ctx, P, &t, 1, RSF_F32, p, 0.0, 0, static_cast<char *>(ctx->ws), s,
                       nullptr, out);
        if (st == RSF_OK) st = prologue(ctx, P, s);
        if (st != RSF_OK) return st;
        return ws_leave(ctx, s);
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
        st = check_types(ctx, *params, volume_dtype);
        if (st != RSF_OK) return st;
        st = set_device(ctx);
        if (st != RSF_OK) return st;
        // phi is only read: the update writes into phi_next (or the workspace)
        rsf_tile t{volume, const_cast<float *>(phi), nx, ny, nz};
        st = ensure_ws(ctx, plan_layout(&t, 1, 1, params->storage,
                                        splits_for(ctx, &t, 1, radius_of(params->sigma)),
                                        rsf::host::needs_k2(*params))
                                .total);
        if (st != RSF_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        st = ws_enter(ctx, s);
        if (st != RSF_OK) return st;
        ctx->has_last = false;   // the workspace is reused
        Plan P;
        st = make_plan(ctx, P, &t, 1, volume_dtype, *params, 0.0, 1,
                       static_cast<char *>(ctx->ws), s, fields);
        if (st == RSF_OK) st = prologue(ctx, P, s);
        if (st == RSF_OK) st = iteration(ctx, P, true, s);
        if (st != RSF_OK) return st;
        return ws_leave(ctx, s);
    } catch (...) {
        return fail(ctx, RSF_ERR_INTERNAL, "internal error");
    }
}

}  // extern "C"
