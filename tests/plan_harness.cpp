// Random blend plans against the bounds the runtime sizes its chunk buffers
// by (blend_plan.h), on the CPU, for every chunk size a plan may take.  Bins
// get list lengths from a heavy-tailed mix; each of a bin's four tiles asks
// for n_chunks(L) records, in 64-tile
// wavefronts taken in a random order, each wavefront reserving a contiguous
// range as the range kernel's atomic does.  Checked per plan: with buffers of
// chunk_bound(K) records every long tile is chunked; with any buffer size
// the records handed out stay inside it and the work items (chunks after the
// first) and re-walk entries (at most one per record) fit it; the chunks of
// a list tile it exactly.  Prints "ok <plans>" or the first failure.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "blend_plan.h"

using namespace v3dg;

static int fail(const char *what, long a, long b)
{
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char **argv)
{
    const int plans = argc > 1 ? std::atoi(argv[1]) : 2000;
    std::mt19937_64 rng(7);
    for (int p = 0; p < plans; ++p) {
        const ChunkPlan cp{kChunkShiftMin + (uint32_t)(p % (kChunkShiftMax - kChunkShiftMin + 1))};
        const uint32_t kFirst = cp.first(), kLater = cp.later();
        const uint32_t n_bins = 1 + (uint32_t)(rng() % 3000);
        std::vector<uint32_t> L(n_bins);
        uint64_t K = 0;
        for (auto &x : L) {
            const uint32_t kind = (uint32_t)(rng() % 10);
            x = kind < 6 ? (uint32_t)(rng() % 2000)                                  // light
                : kind < 9 ? (uint32_t)(kFirst - 3 + rng() % (4 * kLater + 7))  // around the cuts
                           : (uint32_t)(rng() % 200000);                            // very long
            K += x;
        }
        // the chunks of a list tile it exactly
        for (uint32_t b = 0; b < n_bins; ++b) {
            if (L[b] <= kFirst) continue;
            const uint32_t m = cp.n_chunks(L[b]);
            if (cp.begin(0) != 0 || cp.end(0, L[b]) != kFirst || cp.end(m - 1, L[b]) != L[b])
                return fail("cover", L[b], m);
            for (uint32_t c = 0; c < m; ++c) {
                if (!(cp.begin(c) < cp.end(c, L[b]))) return fail("empty chunk", L[b], c);
                if (c > 0 && cp.end(c, L[b]) - cp.begin(c) > kLater) return fail("chunk size", L[b], c);
                if (c + 1 < m && cp.end(c, L[b]) != cp.begin(c + 1)) return fail("gap", L[b], c);
            }
            if ((uint64_t)m * kLater > (uint64_t)L[b]) return fail("records per list", L[b], m);
        }
        const uint64_t bound = chunk_bound(K, cp.shift);
        for (int sz = 0; sz < 3; ++sz) {
            const uint64_t max_chunks = sz == 0 ? bound : sz == 1 ? bound / 3 : rng() % (bound + 1);
            // tiles in 64-wide wavefronts, the wavefronts in a random order
            const uint64_t n_tiles = (uint64_t)n_bins * kTilesPerBin;
            std::vector<uint64_t> waves((n_tiles + 63) / 64);
            for (uint64_t w = 0; w < waves.size(); ++w) waves[w] = w;
            std::shuffle(waves.begin(), waves.end(), rng);
            uint64_t counter = 0, records = 0, items = 0, chunked_long = 0, long_tiles = 0;
            for (uint64_t w : waves) {
                const uint64_t base = counter;
                for (uint64_t t = w * 64; t < std::min(n_tiles, w * 64 + 64); ++t) {
                    const uint32_t l = L[t / kTilesPerBin];
                    const uint32_t m = l > kFirst ? cp.n_chunks(l) : 0u;
                    const uint64_t first = counter;
                    counter += m;
                    if (m) ++long_tiles;
                    if (!plan_fits(first, m, max_chunks)) continue;
                    if (first < base || first + m > max_chunks) return fail("record range", (long)first, m);
                    ++chunked_long;
                    records += m;
                    items += m - 1;
                }
            }
            if (records > max_chunks) return fail("records", (long)records, (long)max_chunks);
            if (items > max_chunks) return fail("items", (long)items, (long)max_chunks);
            if (sz == 0 && chunked_long != long_tiles) return fail("unchunked at the bound", (long)chunked_long,
                                                                    (long)long_tiles);
        }
    }
    std::printf("ok %d\n", plans);
    return 0;
}
