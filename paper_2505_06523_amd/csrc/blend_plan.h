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
constexpr int kChunk = 1024;                // keys per chunk of a long bin list after the first
constexpr int kChunkFirst = 3072;           // keys of the first chunk (walked by pass 1)
constexpr uint32_t kNoChunk = 0xffffffffu;  // chunk base of a tile blended whole
static_assert(kChunkFirst >= 2 * kChunk, "the chunk bound needs first chunks of at least two later ones");

// A list of L > kChunkFirst keys is cut into a first chunk of kChunkFirst keys
// and further chunks of kChunk: n_chunks(L) chunks, chunk c holding keys
// [chunk_begin(c), chunk_end(c, L)).
V3DG_HD inline uint32_t n_chunks(uint32_t L)
{
    return L <= (uint32_t)kChunkFirst ? 1u : 1u + (L - kChunkFirst + kChunk - 1) / kChunk;
}
V3DG_HD inline uint32_t chunk_begin(uint32_t c) { return c == 0 ? 0u : kChunkFirst + (c - 1) * kChunk; }
V3DG_HD inline uint32_t chunk_end(uint32_t c, uint32_t L)
{
    const uint32_t e = (uint32_t)kChunkFirst + c * (uint32_t)kChunk;
    return e < L ? e : L;
}

// Chunk records a plan over K keys may take: each of the kTilesPerBin tiles
// of a bin with L > kChunkFirst keys takes n_chunks(L) <= 2 + (L - kChunkFirst)
// / kChunk <= L / kChunk records (kChunkFirst >= 2 kChunk), so all lists
// together take at most kTilesPerBin K / kChunk.
inline uint64_t chunk_bound(uint64_t K) { return (uint64_t)kTilesPerBin * ((K + kChunk - 1) / kChunk) + 1; }

// Whether a tile given records [first, first + m) of a buffer of max_chunks
// records is chunked (else it is blended whole).
V3DG_HD inline bool plan_fits(uint64_t first, uint32_t m, uint64_t max_chunks)
{
    return m != 0 && first + m <= max_chunks;
}

}  // namespace v3dg
