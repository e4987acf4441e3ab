// Request server (declared in include/rsf.h): continuous batching of
// independent tiles on one device.
//
// A worker thread owns all device work.  Each scheduling chunk it
//   1. admits queued requests in arrival order while their workspaces fit the
//      budget (first-fit arena) and a resident slot is free;
//   2. groups the resident tiles by (radius, types, coefficients);
//   3. per group, uploads a tile table (pinned staging ring), runs the
//      per-tile set-up of newly admitted tiles, up to chunk_iters iterations
//      of every running tile in shared launches (each tile stops on the
//      device at its own iteration count or tolerance), and the finish pass
//      of the tiles that end in this chunk;
//   4. copies the flag slots of all tiles back and records an event.
// Up to kDepth chunks are in flight: the next chunk is planned from host
// bookkeeping while the previous one runs.  A tile's workspace and slot are
// released only when the chunk holding its finish pass has completed, and no
// later chunk refers to it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "rsf.h"
#include "rsf_arena.hpp"
#include "rsf_fault.hpp"
#include "rsf_host.hpp"
#include "rsf_internal.hpp"

namespace {

using rsf::Arena;
using rsf::Batch;
using rsf::Coeffs;
using rsf::Grid3;
using rsf::Split;
using rsf::Taps;
using rsf::TileDesc;
using namespace rsf::host;

constexpr int kDepth = 2;                  // chunks in flight
constexpr int kMaxResident = 4096;
constexpr size_t kSlotBytes = 16;          // flags[0], flags[1], last sum (double)

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Tile {
    uint64_t ticket;
    rsf_request req;
    Grid3 g;
    int R;
    size_t ws_bytes;
    TileRegions T;
    Arena::Block blk;
    char *base = nullptr;
    int slot = -1;
    int remaining = 0;            // iterations not yet launched
    bool started = false;         // set-up launched
    bool stopped = false;         // the device stopped it (tolerance)
    int64_t finish_chunk = -1;    // chunk holding its finish pass
    int64_t chosen = -1;          // last chunk it was picked to iterate in
    double t_submit = 0, t_admit = 0;
};

// Tiles that may share launches: same radius, types and coefficients.
using GroupKey = std::tuple<int, int, int, float, float, float, float, float, float, float, int,
                            double, float, int, float>;

GroupKey key_of(const Tile &t)
{
    const rsf_params &p = t.req.params;
    return GroupKey{t.R,        t.req.volume_dtype, p.storage, p.lambda1, p.lambda2,
                    p.nu,       p.mu,               p.dt,      p.eps,     p.eta,
                    p.regulariser, t.req.tol,       p.sigma,   p.force,   p.sigma2};
}

// One ring entry: pinned staging and device copy of a chunk's tile tables,
// and the pinned copy of the flag slots taken at the chunk's end.
constexpr int kGroupStreams = 3;           // streams for concurrent groups

struct RingEntry {
    void *stage = nullptr;
    void *table = nullptr;
    void *flags_host = nullptr;
    hipEvent_t ev = nullptr;                // chunk done (main stream)
    hipEvent_t up_ev = nullptr;             // table uploaded
    hipEvent_t join_ev[kGroupStreams] = {}; // group streams done
    size_t bytes = 0;
};

struct Chunk {
    int64_t id;
    int ring;
    std::vector<Tile *> ran, finishing;
    int slots_copied = 0;
};

}  // namespace

struct rsf_server {
    rsf_server_config cfg{};
    rsf::Targets targets = rsf::kDefaultTargets;
    hipStream_t stream = nullptr;
    hipStream_t gstream[kGroupStreams] = {};
    int *flags_dev = nullptr;      // kSlotBytes per slot
    RingEntry ring[kDepth];
    Arena arena{0, 0, kAlign};
    std::vector<void *> segments;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Tile>> pending;     // guarded by mu
    std::unordered_map<uint64_t, rsf_result> results;  // done, unread; guarded by mu
    std::unordered_set<uint64_t> live;              // submitted, not done; guarded by mu
    std::string err;                                // guarded by mu
    bool stop = false;                              // guarded by mu
    bool failed = false;                            // guarded by mu
    uint64_t next_ticket = 1;
    uint64_t outstanding = 0;                       // submitted, not done; guarded by mu
    rsf_server_stats stats{};                       // guarded by mu

    // worker-only state
    std::vector<std::unique_ptr<Tile>> resident;
    std::vector<int> free_slots;
    std::deque<Chunk> inflight;
    int64_t next_chunk = 0;
    std::thread worker;
};

namespace {

size_t table_capacity(int max_resident)
{
    // per group: run descs + finish descs and six prefix tables; at most
    // max_resident groups, each table padded to kAlign
    const size_t n = (size_t)max_resident;
    return align_up(2 * n * sizeof(TileDesc)) + 6 * align_up((n + 1) * sizeof(int)) +
           10 * n * kAlign;
}

// Fail every unfinished request (device error); caller holds no lock.
void fail_all(rsf_server *s, const std::string &why)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->failed = true;
    if (s->err.empty()) s->err = why;
    auto finish = [&](Tile &t) {
        rsf_result r{};
        r.status = RSF_ERR_DEVICE;
        r.t_submit = t.t_submit;
        r.t_admit = t.t_admit;
        r.t_done = now_s();
        r.workspace_bytes = t.ws_bytes;
        s->results[t.ticket] = r;
        s->live.erase(t.ticket);
        --s->outstanding;
        ++s->stats.completed;
    };
    for (auto &t : s->resident) finish(*t);
    s->resident.clear();
    for (auto &t : s->pending) finish(*t);
    s->pending.clear();
    s->stats.pending = 0;
    s->stats.resident = 0;
    s->inflight.clear();
    s->cv_done.notify_all();
}

void complete(rsf_server *s, Tile &t, int iters_run, double last)
{
    rsf_result r{};
    r.status = std::isfinite(last) ? RSF_OK : RSF_ERR_NONFINITE;
    r.iters_run = iters_run;
    r.last_sum_abs = last;
    r.t_submit = t.t_submit;
    r.t_admit = t.t_admit;
    r.t_done = now_s();
    r.workspace_bytes = t.ws_bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    s->results[t.ticket] = r;
    s->live.erase(t.ticket);
    --s->outstanding;
    ++s->stats.completed;
    s->stats.voxel_iters += (double)t.g.nx * t.g.ny * t.g.nz * iters_run;
    s->cv_done.notify_all();
}

// Admit queued requests in order while they fit.  Worker thread.
bool admit(rsf_server *s)
{
    bool any = false;
    for (;;) {
        std::unique_ptr<Tile> t;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->pending.empty()) break;
            Tile &head = *s->pending.front();
            if (head.req.iters == 0) {
                t = std::move(s->pending.front());
                s->pending.pop_front();
                s->stats.pending = (int)s->pending.size();
            } else {
                if (s->free_slots.empty()) break;
                if (s->arena.in_use() + s->arena.round(head.ws_bytes) > s->cfg.budget_bytes) break;
                Arena::Block b;
                std::string grow_err;
                const bool ok = s->arena.alloc(head.ws_bytes, b, [&](size_t len) {
                    void *p = nullptr;
                    const hipError_t e = rsf::dev_alloc(&p, len);
                    if (e != hipSuccess) {
                        grow_err = hipGetErrorString(e);
                        return false;
                    }
                    s->segments.push_back(p);
                    return true;
                });
                if (!ok) break;   // wait for resident tiles to leave
                t = std::move(s->pending.front());
                s->pending.pop_front();
                t->blk = b;
                t->base = static_cast<char *>(s->segments[b.seg]) + b.off;
                t->slot = s->free_slots.back();
                s->free_slots.pop_back();
                s->stats.pending = (int)s->pending.size();
                s->stats.bytes_in_use = s->arena.in_use();
                s->stats.peak_bytes = s->arena.peak();
                s->stats.bytes_reserved = s->arena.reserved();
            }
        }
        t->t_admit = now_s();
        if (t->req.iters == 0) {
            complete(s, *t, 0, 0.0);
            continue;
        }
        t->remaining = t->req.iters;
        s->resident.push_back(std::move(t));
        any = true;
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.resident = (int)s->resident.size();
        s->stats.peak_resident = std::max(s->stats.peak_resident, s->stats.resident);
    }
    return any;
}

bool has_work(const rsf_server *s)
{
    for (const auto &t : s->resident)
        if (t->finish_chunk < 0) return true;
    return false;
}

// Table builder over one ring entry's staging buffer.
struct TableWriter {
    char *host;
    char *dev;
    size_t off = 0, cap;
    template <class T>
    size_t put(const T *p, size_t n)
    {
        const size_t at = off;
        const size_t bytes = align_up(n * sizeof(T));
        if (at + bytes > cap) return (size_t)-1;
        std::memcpy(host + at, p, n * sizeof(T));
        off += bytes;
        return at;
    }
};

struct View {
    Batch b;
    int64_t blocks;
};

// Plan and launch one chunk.  Worker thread.  Returns false on a device error
// (with `why` set).
bool launch_chunk(rsf_server *s, std::string &why)
{
    const int64_t id = s->next_chunk++;
    const int ri = (int)(id % kDepth);
    RingEntry &re = s->ring[ri];
    Chunk ch;
    ch.id = id;
    ch.ring = ri;

    // The tiles that iterate in this chunk: all of them, or (with a voxel
    // cap) the first in the configured order until the cap is reached.
    std::vector<Tile *> cand;
    for (auto &t : s->resident)
        if (t->finish_chunk < 0 && t->remaining > 0 && !t->stopped) cand.push_back(t.get());
    if (s->cfg.batch_voxels > 0) {
        auto vox = [](const Tile *t) { return (double)t->g.nx * t->g.ny * t->g.nz; };
        if (s->cfg.order == RSF_ORDER_SHORTEST)
            std::stable_sort(cand.begin(), cand.end(), [&](const Tile *a, const Tile *b) {
                const double wa = vox(a) * a->remaining, wb = vox(b) * b->remaining;
                return wa < wb || (wa == wb && a->ticket < b->ticket);
            });
        else
            std::stable_sort(cand.begin(), cand.end(),
                             [](const Tile *a, const Tile *b) { return a->ticket < b->ticket; });
        double sum = 0.0;
        size_t keep = 0;
        while (keep < cand.size() && (keep == 0 || sum < (double)s->cfg.batch_voxels))
            sum += vox(cand[keep++]);
        cand.resize(keep);
    }
    for (Tile *t : cand) t->chosen = id;

    std::map<GroupKey, std::vector<Tile *>> groups;
    for (auto &t : s->resident)
        if (t->finish_chunk < 0) groups[key_of(*t)].push_back(t.get());

    TableWriter tw{static_cast<char *>(re.stage), static_cast<char *>(re.table), 0, re.bytes};
    struct Launch {
        const Tile *proto;
        int R, image, storage;
        Taps taps;
        bool k2;
        int R2;
        Taps taps2;
        Coeffs c;
        int iters;
        View run_xy, run_z, run_u, run_tile, new_xy, new_z, new_tile, fin_z;
        int n_new, n_run, n_fin;
        bool fuse;
    };
    std::vector<Launch> launches;

    for (auto &kv : groups) {
        std::vector<Tile *> run, fresh, fin;
        for (Tile *t : kv.second)
            if (t->chosen == id) (t->started ? run : fresh).push_back(t);
        const int n_old = (int)run.size();
        run.insert(run.end(), fresh.begin(), fresh.end());
        int iters = 0;
        for (Tile *t : run) iters = std::max(iters, std::min(t->remaining, s->cfg.chunk_iters));
        for (Tile *t : run) t->remaining -= std::min(iters, t->remaining);
        for (Tile *t : kv.second)
            if (t->remaining == 0 || t->stopped) fin.push_back(t);
        if (run.empty() && fin.empty()) continue;

        // The group's update carries the next stage-1 z pass when its force
        // and radius allow it (the RSF force's stage-2 ring leaves room up to
        // radius fuse_max_r); its tiles are then marched whole in z, and one
        // stage-1 pass opens the chunk.
        const Tile *gp = kv.second.front();
        const bool fuse = !s->cfg.separate_passes &&
                          (gp->req.params.force == RSF_FORCE_PAPER ||
                           gp->R <= rsf::fuse_max_r(gp->req.params.storage,
                                                    gp->req.volume_dtype));
        // splits from each tile's share of the group's running voxels
        double vox = 0.0;
        for (Tile *t : run) vox += (double)t->g.nx * t->g.ny * t->g.nz;
        double vox_fin = 0.0;
        for (Tile *t : fin) vox_fin += (double)t->g.nx * t->g.ny * t->g.nz;
        auto desc_of = [&](Tile *t, double total) {
            const double share = (double)t->g.nx * t->g.ny * t->g.nz / total;
            Split sp = rsf::default_split(t->g, share, s->targets);
            if (fuse) sp.u = 1;
            int *flags = reinterpret_cast<int *>(reinterpret_cast<char *>(s->flags_dev) +
                                                 (size_t)t->slot * kSlotBytes);
            return tile_desc(t->g, sp, t->req.volume, t->req.phi, t->base, t->T, t->req.iters,
                             flags);
        };
        std::vector<TileDesc> drun, dfin;
        for (Tile *t : run) drun.push_back(desc_of(t, vox));
        for (Tile *t : fin) dfin.push_back(desc_of(t, vox_fin));
        auto prefix = [](const std::vector<TileDesc> &d, int from, int64_t (*blocks)(const Grid3 &,
                                                                                      const Split &)) {
            std::vector<int> p(1, 0);
            for (int i = from; i < (int)d.size(); ++i)
                p.push_back(p.back() + (int)blocks(d[i].g, d[i].sp));
            return p;
        };
        const std::vector<int> rxy = prefix(drun, 0, rsf::xy_blocks),
                               rz = prefix(drun, 0, rsf::z_blocks),
                               ru = prefix(drun, 0, rsf::u_blocks),
                               nxy = prefix(drun, n_old, rsf::xy_blocks),
                               nz = prefix(drun, n_old, rsf::z_blocks),
                               fz = prefix(dfin, 0, rsf::z_blocks);
        const size_t o_run = drun.empty() ? 0 : tw.put(drun.data(), drun.size());
        const size_t o_fin = dfin.empty() ? 0 : tw.put(dfin.data(), dfin.size());
        const size_t o_rxy = tw.put(rxy.data(), rxy.size()), o_rz = tw.put(rz.data(), rz.size()),
                     o_ru = tw.put(ru.data(), ru.size()), o_nxy = tw.put(nxy.data(), nxy.size()),
                     o_nz = tw.put(nz.data(), nz.size()), o_fz = tw.put(fz.data(), fz.size());
        for (size_t o : {o_run, o_fin, o_rxy, o_rz, o_ru, o_nxy, o_nz, o_fz})
            if (o == (size_t)-1) {
                why = "tile table overflow";
                return false;
            }
        Launch L{};
        Tile *proto = run.empty() ? fin.front() : run.front();
        L.proto = proto;
        L.R = proto->R;
        L.image = proto->req.volume_dtype;
        L.storage = proto->req.params.storage;
        L.taps = make_taps(proto->req.params.sigma, L.R);
        L.k2 = needs_k2(proto->req.params);
        L.R2 = L.k2 ? radius_of(proto->req.params.sigma2) : 0;
        if (L.k2) L.taps2 = make_taps(proto->req.params.sigma2, L.R2);
        L.c = make_coeffs(proto->req.params, proto->req.tol);
        L.iters = iters;
        L.n_run = (int)run.size();
        L.n_new = (int)fresh.size();
        L.n_fin = (int)fin.size();
        L.fuse = fuse;
        const TileDesc *dr = reinterpret_cast<const TileDesc *>(tw.dev + o_run);
        const TileDesc *df = reinterpret_cast<const TileDesc *>(tw.dev + o_fin);
        auto ip = [&](size_t o) { return reinterpret_cast<const int *>(tw.dev + o); };
        // grids and XCD ranges of a view over descriptors [from, to)
        auto view = [&](const TileDesc *dev, const std::vector<TileDesc> &d, int from, size_t o,
                        PassKind k) {
            View v{Batch{dev + from, ip(o), (int)d.size() - from, {}}, 0};
            std::vector<Grid3> gs;
            std::vector<Split> sps;
            for (int i = from; i < (int)d.size(); ++i) {
                gs.push_back(d[i].g);
                sps.push_back(d[i].sp);
            }
            v.blocks = balance_xcds(v.b, k, gs, sps, L.R);
            return v;
        };
        L.run_xy = view(dr, drun, 0, o_rxy, PASS_XY);
        L.run_z = view(dr, drun, 0, o_rz, PASS_Z);
        L.run_u = view(dr, drun, 0, o_ru, PASS_U);
        L.run_tile = View{Batch{dr, nullptr, L.n_run, {}}, L.n_run};
        L.new_xy = view(dr, drun, n_old, o_nxy, PASS_XY);
        L.new_z = view(dr, drun, n_old, o_nz, PASS_Z);
        L.new_tile = View{Batch{dr + n_old, nullptr, L.n_new, {}}, L.n_new};
        L.fin_z = view(df, dfin, 0, o_fz, PASS_Z);
        launches.push_back(L);
        for (Tile *t : run) {
            t->started = true;
            ch.ran.push_back(t);
        }
        for (Tile *t : fin) {
            t->finish_chunk = id;
            ch.finishing.push_back(t);
        }
    }

    hipStream_t st = s->stream;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t r, const char *what) {
        if (r != hipSuccess && e == hipSuccess) {
            e = r;
            why = std::string(what) + ": " + hipGetErrorString(r);
        }
        return e == hipSuccess;
    };
    if (tw.off && !ok(hipMemcpyAsync(re.table, re.stage, tw.off, hipMemcpyHostToDevice, st),
                      "upload tile table"))
        return false;
    // Groups share no tiles: each runs on its own stream (they overlap and
    // fill each other's launch tails), after the table upload; the main
    // stream joins them before copying the flags back.  The next chunk's
    // upload follows that join, so a tile's chunks never overlap.
    const int nstreams = std::min<int>((int)launches.size(), kGroupStreams);
    if (nstreams > 1 && !ok(hipEventRecord(re.up_ev, st), "hipEventRecord(upload)")) return false;
    for (int k = 0; k < nstreams && nstreams > 1; ++k)
        if (!ok(hipStreamWaitEvent(s->gstream[k], re.up_ev, 0), "hipStreamWaitEvent")) return false;
    for (size_t gi = 0; gi < launches.size(); ++gi) {
        const Launch &L = launches[gi];
        hipStream_t st = nstreams > 1 ? s->gstream[gi % kGroupStreams] : s->stream;
        if (L.n_new > 0) {
            if (!ok(rsf::launch_setup(L.new_tile.b, L.taps, L.R, st), "set-up")) return false;
            if (L.k2) {
                Coeffs sq = L.c;
                for (int k = 0; k < 2; ++k) {
                    sq.square = k;
                    if (!ok(rsf::launch_xy(L.R2, rsf::XY_ONE, L.image, L.storage, L.new_xy.b,
                                           L.new_xy.blocks, L.taps2, sq, false, st),
                            "K2*I (xy)") ||
                        !ok(rsf::launch_z_plain(L.R2, L.storage, L.new_z.b, L.new_z.blocks,
                                                L.taps2, k ? rsf::Z_TO_K2I2 : rsf::Z_TO_K2I, st),
                            "K2*I (z)"))
                        return false;
                }
            }
            if (!ok(rsf::launch_xy(L.R, rsf::XY_ONE, L.image, L.storage, L.new_xy.b,
                                   L.new_xy.blocks, L.taps, L.c, false, st),
                    "K*I (xy)"))
                return false;
            if (!ok(rsf::launch_z_plain(L.R, L.storage, L.new_z.b, L.new_z.blocks, L.taps,
                                        rsf::Z_TO_KI, st),
                    "K*I (z)"))
                return false;
        }
        const bool paper = L.c.force == RSF_FORCE_PAPER;
        // fused: one stage-1 pass opens the chunk, each update writes the next
        if (L.fuse && L.iters > 0 &&
            !ok(rsf::launch_z_heaviside(L.R, L.image, L.storage, L.run_z.b, L.run_z.blocks,
                                        L.taps, L.c, false, st),
                "z(H)"))
            return false;
        for (int it = 0; it < L.iters; ++it) {
            if ((!L.fuse && !ok(rsf::launch_z_heaviside(L.R, L.image, L.storage, L.run_z.b,
                                                        L.run_z.blocks, L.taps, L.c, false, st),
                                "z(H)")) ||
                !ok(rsf::launch_xy(L.R,
                                   paper ? (L.k2 ? rsf::XY_PAPER2 : rsf::XY_PAPER) : rsf::XY_FITS,
                                   L.image, L.storage, L.run_xy.b, L.run_xy.blocks, L.taps, L.c,
                                   false, st),
                    "xy(fits)") ||
                (!paper && !ok(rsf::launch_xy(L.R, rsf::XY_TWO, L.image, L.storage, L.run_xy.b,
                                              L.run_xy.blocks, L.taps, L.c, false, st),
                               "xy(g)")) ||
                !ok(L.fuse ? rsf::launch_z_update_fused(L.R, L.image, L.storage, L.run_u.b,
                                                        L.run_u.blocks, L.taps, L.c, paper, st)
                    : paper ? rsf::launch_z_update_paper(L.image, L.storage, L.run_u.b,
                                                         L.run_u.blocks, L.c, false, st)
                            : rsf::launch_z_update(L.R, L.image, L.storage, L.run_u.b,
                                                   L.run_u.blocks, L.taps, L.c, false, st),
                    "z(update)") ||
                !ok(rsf::launch_reduce(L.run_tile.b, L.c, st), "reduce"))
                return false;
        }
        if (L.n_fin > 0 && !ok(rsf::launch_finish(L.fin_z.b, L.fin_z.blocks, st), "finish"))
            return false;
    }
    for (int k = 0; k < nstreams && nstreams > 1; ++k)
        if (!ok(hipEventRecord(re.join_ev[k], s->gstream[k]), "hipEventRecord(join)") ||
            !ok(hipStreamWaitEvent(st, re.join_ev[k], 0), "hipStreamWaitEvent(join)"))
            return false;
    ch.slots_copied = s->cfg.max_resident;
    if (!ok(hipMemcpyAsync(re.flags_host, s->flags_dev, (size_t)ch.slots_copied * kSlotBytes,
                           hipMemcpyDeviceToHost, st),
            "copy flags") ||
        !ok(hipEventRecord(re.ev, st), "hipEventRecord"))
        return false;
    s->inflight.push_back(std::move(ch));
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->stats.chunks;
    return true;
}

// Wait for the oldest chunk and retire what it finished.  Worker thread.
bool retire_chunk(rsf_server *s, std::string &why)
{
    Chunk ch = std::move(s->inflight.front());
    s->inflight.pop_front();
    RingEntry &re = s->ring[ch.ring];
    const hipError_t e = hipEventSynchronize(re.ev);
    if (e != hipSuccess) {
        why = std::string("chunk: ") + hipGetErrorString(e);
        return false;
    }
    const char *fl = static_cast<const char *>(re.flags_host);
    auto slot_flags = [&](const Tile *t) { return reinterpret_cast<const int *>(fl + (size_t)t->slot * kSlotBytes); };
    auto slot_last = [&](const Tile *t) {
        double v;
        std::memcpy(&v, fl + (size_t)t->slot * kSlotBytes + 8, sizeof(double));
        return v;
    };
    // tolerance stops seen in this chunk: finish them in the next one
    for (Tile *t : ch.ran)
        if (t->finish_chunk < 0 && slot_flags(t)[0] == 1) {
            t->stopped = true;
            t->remaining = 0;
        }
    for (Tile *t : ch.finishing) {
        complete(s, *t, slot_flags(t)[1], slot_last(t));
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena.release(t->blk);
        s->free_slots.push_back(t->slot);
        s->stats.bytes_in_use = s->arena.in_use();
    }
    if (!ch.finishing.empty()) {
        auto gone = [&](const std::unique_ptr<Tile> &p) {
            return std::find(ch.finishing.begin(), ch.finishing.end(), p.get()) !=
                   ch.finishing.end();
        };
        s->resident.erase(std::remove_if(s->resident.begin(), s->resident.end(), gone),
                          s->resident.end());
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.resident = (int)s->resident.size();
    }
    return true;
}

void worker_main(rsf_server *s)
{
    if (hipSetDevice(s->cfg.device) != hipSuccess) {
        fail_all(s, "hipSetDevice failed in the server worker");
        return;
    }
    std::string why;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->failed) return;
            // sleep while there is nothing queued, resident or in flight
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->pending.empty() || !s->resident.empty() ||
                       !s->inflight.empty();
            });
            if (s->stop && s->pending.empty() && s->resident.empty() && s->inflight.empty())
                return;
        }
        try {
            admit(s);
            if ((int)s->inflight.size() < kDepth && has_work(s)) {
                if (!launch_chunk(s, why)) {
                    fail_all(s, why);
                    return;
                }
                continue;
            }
            if (!s->inflight.empty()) {
                if (!retire_chunk(s, why)) {
                    fail_all(s, why);
                    return;
                }
                continue;
            }
            // Nothing resident or in flight, yet the head request was not
            // admitted: the arena's segments are too small or fragmented for
            // it and the budget leaves no room to grow.  Start the arena over
            // (no work refers to it now) and retry; if that fails too, the
            // device is out of memory.
            if (!s->pending.empty() && s->resident.empty()) {
                bool reset = false;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    if (s->arena.in_use() == 0 && s->arena.segments() > 0) {
                        for (void *p : s->segments) (void)hipFree(p);
                        s->segments.clear();
                        s->arena = Arena(s->cfg.budget_bytes, align_up(s->cfg.segment_bytes),
                                         kAlign);
                        reset = true;
                    }
                }
                if (reset && admit(s)) continue;
            }
            std::lock_guard<std::mutex> lk(s->mu);
            if (!s->pending.empty() && s->resident.empty()) {
                s->err = "cannot place a request in the arena (device out of memory?)";
                auto t = std::move(s->pending.front());
                s->pending.pop_front();
                rsf_result r{};
                r.status = RSF_ERR_OUT_OF_MEMORY;
                r.t_submit = t->t_submit;
                r.t_done = now_s();
                r.workspace_bytes = t->ws_bytes;
                s->results[t->ticket] = r;
                s->live.erase(t->ticket);
                --s->outstanding;
                ++s->stats.completed;
                s->stats.pending = (int)s->pending.size();
                s->cv_done.notify_all();
            }
        } catch (...) {
            fail_all(s, "internal error in the server worker");
            return;
        }
    }
}

void free_server(rsf_server *s)
{
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (RingEntry &re : s->ring) {
        if (re.stage) (void)hipHostFree(re.stage);
        if (re.flags_host) (void)hipHostFree(re.flags_host);
        if (re.table) (void)hipFree(re.table);
        if (re.ev) (void)hipEventDestroy(re.ev);
        if (re.up_ev) (void)hipEventDestroy(re.up_ev);
        for (hipEvent_t ev : re.join_ev)
            if (ev) (void)hipEventDestroy(ev);
    }
    for (hipStream_t gs : s->gstream)
        if (gs) {
            (void)hipStreamSynchronize(gs);
            (void)hipStreamDestroy(gs);
        }
    for (void *p : s->segments) (void)hipFree(p);
    if (s->flags_dev) (void)hipFree(s->flags_dev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

extern "C" {

rsf_status rsf_server_create(rsf_server **out, const rsf_server_config *cfg)
{
    if (!out) return RSF_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->budget_bytes == 0) return RSF_ERR_INVALID_ARG;
    if (cfg->chunk_iters < 0 || cfg->max_resident < 0 || cfg->max_resident > kMaxResident ||
        cfg->batch_voxels < 0 || (cfg->order != RSF_ORDER_ARRIVAL && cfg->order != RSF_ORDER_SHORTEST) ||
        (cfg->separate_passes != 0 && cfg->separate_passes != 1))
        return RSF_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        if (cfg->split_targets[k] < 0 || cfg->split_targets[k] > (1 << 24)) return RSF_ERR_INVALID_ARG;
    rsf_server *s = nullptr;
    try {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || cfg->device < 0 || cfg->device >= count)
            return RSF_ERR_INVALID_ARG;
        s = new rsf_server;
        s->cfg = *cfg;
        if (s->cfg.chunk_iters == 0) s->cfg.chunk_iters = 4;
        if (s->cfg.max_resident == 0) s->cfg.max_resident = 256;
        if (s->cfg.segment_bytes == 0) s->cfg.segment_bytes = (size_t)8 << 30;
        if (cfg->split_targets[0] > 0) s->targets.xy = cfg->split_targets[0];
        if (cfg->split_targets[1] > 0) s->targets.z = cfg->split_targets[1];
        if (cfg->split_targets[2] > 0) s->targets.u = cfg->split_targets[2];
        s->arena = Arena(s->cfg.budget_bytes, align_up(s->cfg.segment_bytes), kAlign);
        auto bad = [&](hipError_t e) {
            if (e == hipSuccess) return false;
            free_server(s);
            return true;
        };
        if (bad(hipSetDevice(cfg->device))) return RSF_ERR_DEVICE;
        if (bad(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking))) return RSF_ERR_DEVICE;
        for (hipStream_t &gs : s->gstream)
            if (bad(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking))) return RSF_ERR_DEVICE;
        const size_t fbytes = (size_t)s->cfg.max_resident * kSlotBytes;
        if (bad(rsf::dev_alloc(&s->flags_dev, fbytes))) return RSF_ERR_OUT_OF_MEMORY;
        if (bad(hipMemset(s->flags_dev, 0, fbytes))) return RSF_ERR_DEVICE;
        const size_t tbytes = table_capacity(s->cfg.max_resident);
        for (RingEntry &re : s->ring) {
            re.bytes = tbytes;
            if (bad(rsf::pinned_alloc(&re.stage, tbytes)) ||
                bad(rsf::pinned_alloc(&re.flags_host, fbytes)) ||
                bad(rsf::dev_alloc(&re.table, tbytes)) ||
                bad(hipEventCreateWithFlags(&re.ev, hipEventDisableTiming)) ||
                bad(hipEventCreateWithFlags(&re.up_ev, hipEventDisableTiming)))
                return RSF_ERR_OUT_OF_MEMORY;
            for (hipEvent_t &ev : re.join_ev)
                if (bad(hipEventCreateWithFlags(&ev, hipEventDisableTiming))) return RSF_ERR_DEVICE;
        }
        for (int i = s->cfg.max_resident - 1; i >= 0; --i) s->free_slots.push_back(i);
        s->worker = std::thread(worker_main, s);
        *out = s;
        return RSF_OK;
    } catch (...) {
        if (s) free_server(s);
        return RSF_ERR_INTERNAL;
    }
}

rsf_status rsf_server_submit(rsf_server *s, const rsf_request *req, uint64_t *ticket)
{
    if (!s) return RSF_ERR_INVALID_ARG;
    try {
        auto refuse = [&](rsf_status st, const std::string &why) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->err = why;
            return st;
        };
        if (!req || !ticket) return refuse(RSF_ERR_INVALID_ARG, "null argument");
        if (!req->volume || !req->phi) return refuse(RSF_ERR_INVALID_ARG, "null volume or phi");
        if (const char *w = dims_error(req->nx, req->ny, req->nz))
            return refuse(RSF_ERR_INVALID_ARG, w);
        if (const char *w = params_error(req->params)) return refuse(RSF_ERR_INVALID_ARG, w);
        if (const char *w = types_error(req->params, req->volume_dtype))
            return refuse(RSF_ERR_INVALID_ARG, w);
        if (req->iters < 0) return refuse(RSF_ERR_INVALID_ARG, "iters must be >= 0");
        if (!(req->tol >= 0.0) || !std::isfinite(req->tol))
            return refuse(RSF_ERR_INVALID_ARG, "tol must be >= 0");
        auto t = std::make_unique<Tile>();
        t->req = *req;
        t->g = grid_of(req->nx, req->ny, req->nz);
        t->R = radius_of(req->params.sigma);
        t->T = tile_regions(t->g, req->iters, req->params.storage, needs_k2(req->params));
        // charged as rsf_workspace_bytes_params (the region plus a one-tile table)
        t->ws_bytes = rsf_workspace_bytes_params(req->nx, req->ny, req->nz, req->iters,
                                                 &req->params);
        if (t->ws_bytes < t->T.total) return refuse(RSF_ERR_INTERNAL, "workspace size");
        if (t->ws_bytes > s->cfg.budget_bytes)
            return refuse(RSF_ERR_BUDGET, "request workspace exceeds the server budget");
        t->t_submit = now_s();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed) return RSF_ERR_DEVICE;
        if (s->stop) {
            s->err = "server is shutting down";
            return RSF_ERR_INVALID_ARG;
        }
        t->ticket = s->next_ticket++;
        *ticket = t->ticket;
        s->live.insert(t->ticket);
        s->pending.push_back(std::move(t));
        ++s->outstanding;
        ++s->stats.submitted;
        s->stats.pending = (int)s->pending.size();
        s->cv_work.notify_one();
        return RSF_OK;
    } catch (...) {
        return RSF_ERR_INTERNAL;
    }
}

rsf_status rsf_server_wait(rsf_server *s, uint64_t ticket, double timeout_s, rsf_result *out)
{
    if (!s || !out) return RSF_ERR_INVALID_ARG;
    try {
        std::unique_lock<std::mutex> lk(s->mu);
        if (!s->live.count(ticket) && !s->results.count(ticket)) {
            s->err = "unknown ticket (or its result was already read)";
            return RSF_ERR_INVALID_ARG;
        }
        auto ready = [&] { return s->results.count(ticket) != 0; };
        if (timeout_s < 0) s->cv_done.wait(lk, ready);
        else if (timeout_s > 0)
            s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
        auto it = s->results.find(ticket);
        if (it == s->results.end()) return RSF_NOT_READY;
        *out = it->second;
        s->results.erase(it);
        return RSF_OK;
    } catch (...) {
        return RSF_ERR_INTERNAL;
    }
}

rsf_status rsf_server_poll(rsf_server *s, uint64_t ticket, rsf_result *out)
{
    return rsf_server_wait(s, ticket, 0.0, out);
}

rsf_status rsf_server_drain(rsf_server *s)
{
    if (!s) return RSF_ERR_INVALID_ARG;
    try {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
        return s->failed ? RSF_ERR_DEVICE : RSF_OK;
    } catch (...) {
        return RSF_ERR_INTERNAL;
    }
}

rsf_status rsf_server_get_stats(rsf_server *s, rsf_server_stats *out)
{
    if (!s || !out) return RSF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return RSF_OK;
}

const char *rsf_server_last_error(const rsf_server *s)
{
    if (!s) return "null server";
    return s->err.c_str();
}

void rsf_server_destroy(rsf_server *s)
{
    if (!s) return;
    try {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->cv_work.notify_all();
        }
        if (s->worker.joinable()) s->worker.join();
        free_server(s);
    } catch (...) {
    }
}

}  // extern "C"
