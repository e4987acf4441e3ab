// How each pass cuts a tile into workgroups (host code): row chunks of the xy
// passes, z chunks of the z passes and of the update pass.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "rsf_internal.hpp"

namespace rsf {

// The fewest chunks giving at least `want_blocks` over `cols` columns, each
// chunk at least `least` long; re-derived so every chunk is non-empty.
static int chunks(int64_t n, int64_t cols, int64_t want_blocks, int64_t least)
{
    int64_t want = (want_blocks + cols - 1) / cols;
    const int64_t most = (n + least - 1) / least;
    if (want > most) want = most;
    if (want < 1) want = 1;
    const int64_t len = (n + want - 1) / want;
    return (int)((n + len - 1) / len);
}

Split make_split(const Grid3 &g, int64_t xy_waves, int64_t z_target, int64_t u_target)
{
    Split s;
    const int64_t strips = nbx64(g.nx);
    s.xy = chunks(g.ny, strips * g.nz, xy_waves, 8);
    s.z = chunks(g.nz, z_cols(g), z_target, 8);
    s.u = chunks(g.nz, (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy), u_target, 8);
    return s;
}

// A tile holding fraction `share` of a batch's voxels gets that fraction of
// the batch's workgroup targets (by default xy ~16K waves, rows in chunks of
// at most 128; z ~2K workgroups; update ~1K workgroups).  Fewer chunks per tile means fewer
// halo slices re-read, so small tiles in a big batch run unchunked.
Split default_split(const Grid3 &g, double share, const Targets &tg)
{
    const auto part = [&](int64_t n) {
        return (int64_t)std::max(1.0, std::ceil((double)n * share));
    };
    Split s = make_split(g, part(tg.xy), part(tg.z), part(tg.u));
    const int base = (g.ny + 127) / 128;
    if (s.xy < base) {
        const int64_t len = (g.ny + base - 1) / base;
        s.xy = (int)((g.ny + len - 1) / len);
    }
    return s;
}

// z chunks c in 1..ceil(nz/8) for a pass whose workgroups each march a chunk
// plus `halo` extra slices: the cost of c is ceil(groups / resident) x (chunk
// length + halo), the launch's rounds of workgroups.  Among the c that keep at
// least `min_fill` of the resident slots busy, take the fewest chunks whose
// cost is within 3 % of the least (fewer halo re-reads); if none keeps the
// slots that busy, take the most chunks.
static int capacity_chunks(int64_t nz, int64_t cols, int64_t resident, double min_fill,
                           int64_t halo)
{
    const int64_t most = (nz + 7) / 8;
    std::vector<std::pair<int64_t, double>> ok;
    double least = -1.0;
    for (int64_t c = 1; c <= most; ++c) {
        const int64_t len = (nz + c - 1) / c;
        if ((nz + len - 1) / len != c) continue;   // not c non-empty chunks
        const int64_t groups = cols * c;
        if ((double)groups < min_fill * (double)resident) continue;
        const double cost = (double)((groups + resident - 1) / resident) * (double)(len + halo);
        ok.push_back({c, cost});
        if (least < 0.0 || cost < least) least = cost;
    }
    for (const auto &cc : ok)
        if (cc.second <= 1.03 * least) return (int)cc.first;
    const int64_t len = (nz + most - 1) / most;
    return (int)((nz + len - 1) / len);
}

Split capacity_split(const Grid3 &g, int R)
{
    Split s = default_split(g, 1.0, kDefaultTargets);
    // a z-pass chunk primes its ring with 2R slices; an update chunk reads R
    // extra slices of the pair ring on average and 4 of phi
    s.z = capacity_chunks(g.nz, z_cols(g), kResidentZ, 0.5, 2 * R);
    s.u = capacity_chunks(g.nz, (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy),
                          kResidentU, 0.75, R + 2);
    return s;
}

static bool chunks_ok(int n, int c)
{
    if (c < 1 || c > n) return false;
    const int len = (n + c - 1) / c;
    return (c - 1) * len < n;
}

bool split_valid(const Grid3 &g, const Split &s)
{
    return chunks_ok(g.ny, s.xy) && chunks_ok(g.nz, s.z) && chunks_ok(g.nz, s.u) &&
           u_blocks(g, s) <= u_blocks_max(g);
}

}  // namespace rsf
