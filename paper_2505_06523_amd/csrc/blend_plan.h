// Long-list chunking of the blend plan: the arithmetic shared by the range
// kernel (which hands out chunk records), the blend kernels (which walk the
// chunks) and the host (which sizes the chunk buffers).  No device calls, so
// the CPU tests compile it on its own.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define V3DG_HD __host__ __device__
#else
#define V3DG_HD
#endif

namespace v3dg {

constexpr uint32_t kTilesPerBin = 4;        // a bin is a 2 x 2 block of tiles; each tile walks the bin's list
constexpr uint32_t kNoChunk = 0xffffffffu;  // chunk base of a tile blended whole

// Chunk sizes of a plan: later chunks of 2^shift keys and a first chunk of
// three of them (the first chunk is longer because most pixels of opaque
// content stop within it).  Smaller chunks shorten the longest walk of a
// frame; larger ones walk fewer pairs speculatively and again, which pays
// when other frames keep the chip busy meanwhile.
constexpr uint32_t kChunkShiftMin = 10, kChunkShiftMax = 12;  // later chunks of 1,024 .. 4,096 keys
constexpr uint32_t kChunkShiftRender = 10;  // v3dg_render: 3,072 / 1,024 keys
constexpr uint32_t kChunkShiftServer = 12;  // the serving loop: 12,288 / 4,096 keys

// A list of L > first() keys is cut into a first chunk of first() keys and
// further chunks of later(): n_chunks(L) chunks, chunk c holding keys
// [begin(c), end(c, L)).
struct ChunkPlan {
    uint32_t shift = kChunkShiftRender;
    V3DG_HD uint32_t later() const { return 1u << shift; }
    V3DG_HD uint32_t first() const { return 3u << shift; }
    V3DG_HD uint32_t n_chunks(uint32_t L) const
    {
        return L <= first() ? 1u : 1u + ((L - first() + later() - 1u) >> shift);
    }
    V3DG_HD uint32_t begin(uint32_t c) const { return c == 0 ? 0u : (c + 2u) << shift; }
    V3DG_HD uint32_t end(uint32_t c, uint32_t L) const
    {
        const uint32_t e = (c + 3u) << shift;
        return e < L ? e : L;
    }
};

// Chunk records a plan over K keys may take: each of the kTilesPerBin tiles
// of a bin with L > first keys takes n_chunks(L) <= 2 + (L - first) / later
// = L / later - 1 records (first = 3 later), so all lists together take at
// most kTilesPerBin K / later.
inline uint64_t chunk_bound(uint64_t K, uint32_t shift)
{
    return (uint64_t)kTilesPerBin * ((K + (1ull << shift) - 1) >> shift) + 1;
}

// Whether a tile given records [first, first + m) of a buffer of max_chunks
// records is chunked (else it is blended whole).
V3DG_HD inline bool plan_fits(uint64_t first, uint32_t m, uint64_t max_chunks)
{
    return m != 0 && first + m <= max_chunks;
}

}  // namespace v3dg
