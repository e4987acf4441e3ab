// Host check of the batched launch geometry: for random batches of tiles and
// splits, the XCD ranges cut by balance_xcds, decoded the way the kernels
// decode them (hardware workgroup b on XCD b % 8, position b / 8 in its
// range, then the tile by binary search of the prefix table), cover every
// workgroup of every tile exactly once, and the ranges' costs are balanced.
// Host code only: nothing runs on a device.
#include <cstdio>
#include <random>
#include <vector>

#include "rsf_host.hpp"

using namespace rsf;
using namespace rsf::host;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static int find_tile_host(const std::vector<int> &start, int n, int gb)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= gb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int main()
{
    std::mt19937 rng(7);
    double worst = 0.0;
    for (int trial = 0; trial < 300; ++trial) {
        const int n = 1 + rng() % 40;
        const int R = 1 + rng() % 16;
        std::vector<Grid3> g;
        std::vector<Split> sp;
        double vol = 0.0;
        for (int t = 0; t < n; ++t) {
            const int big = trial % 3 == 0 ? 400 : 120;
            Grid3 q{3 + (int)(rng() % big), 3 + (int)(rng() % big), 3 + (int)(rng() % big), 0};
            q.sxy = (int64_t)q.nx * q.ny;
            g.push_back(q);
            vol += (double)q.nx * q.ny * q.nz;
        }
        for (int t = 0; t < n; ++t) {
            const double share = (double)g[t].nx * g[t].ny * g[t].nz / vol;
            Split s = trial % 2 ? default_split(g[t], share)
                                : make_split(g[t], 1 + rng() % 40000, 1 + rng() % 5000,
                                             1 + rng() % 3000);
            CHECK(split_valid(g[t], s));
            sp.push_back(s);
        }
        for (PassKind k : {PASS_XY, PASS_Z, PASS_U}) {
            std::vector<int> start(1, 0);
            for (int t = 0; t < n; ++t) start.push_back(start.back() + (int)blocks_of(k, g[t], sp[t]));
            Batch b{nullptr, nullptr, n, {}};
            const int64_t grid = balance_xcds(b, k, g, sp, R);
            CHECK(b.xcd[0] == 0 && b.xcd[kXcds] == start[n]);
            for (int x = 0; x < kXcds; ++x) CHECK(b.xcd[x] <= b.xcd[x + 1]);
            CHECK(grid % kXcds == 0 && grid >= start[n]);
            std::vector<int> seen(start[n], 0);
            std::vector<double> cost(kXcds, 0.0);
            for (int64_t hb = 0; hb < grid; ++hb) {
                const int x = (int)(hb % kXcds), j = (int)(hb / kXcds);
                const int gb = b.xcd[x] + j;
                if (gb >= b.xcd[x + 1]) continue;   // surplus workgroup exits
                CHECK(gb >= 0 && gb < start[n]);
                ++seen[gb];
                const int t = find_tile_host(start, n, gb);
                const int lb = gb - start[t];
                CHECK(t >= 0 && t < n && lb >= 0 && lb < blocks_of(k, g[t], sp[t]));
                const int nch = k == PASS_XY ? sp[t].xy : (k == PASS_Z ? sp[t].z : sp[t].u);
                const int c = k == PASS_XY ? (int)((lb / nbx64(g[t].nx)) % nch) : lb % nch;
                cost[x] += (double)span_cost(k == PASS_XY ? g[t].ny : g[t].nz, nch, c, R);
            }
            for (int v : seen) CHECK(v == 1);
            double mx = 0.0, sum = 0.0, wmax = 0.0;
            for (double c : cost) {
                mx = c > mx ? c : mx;
                sum += c;
            }
            // the imbalance is at most one workgroup's cost per range
            for (int t = 0; t < n; ++t)
                wmax = std::max(wmax, (double)(k == PASS_XY ? g[t].ny : g[t].nz) + 2 * R);
            CHECK(mx <= sum / kXcds + wmax + 1e-9);
            if (start[n] >= 64 * kXcds) worst = std::max(worst, mx / (sum / kXcds));
        }
    }
    std::printf("xcd ok worst %.4f\n", worst);
    return 0;
}
