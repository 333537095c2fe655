// Binning of splats to 16x16 tiles and the stable radix sorts that order
// every tile's splats front to back.
//
// Two orderings give the same (tile, depth, slot) order:
//   depth-first (default): the slots are radix-sorted by their FP32 depth
//     bits (stable, so equal depths keep slot order); tiles-touched is scanned
//     in that order; one 32-bit tile id is emitted per (slot, tile); a stable
//     radix sort by tile id then leaves each tile's splats in depth order.
//   64-bit keys: one (tile << 32 | depth bits) key per (slot, tile), emitted in
//     slot order and radix-sorted on all significant bits.
// The depth is a positive FP32 (z > near > 0), so its bit pattern orders like
// its value.
//
//   scan_tiles   exclusive scan of tiles-touched (decoupled look-back)
//   emit32/64    keys of every (slot, tile) the support reaches
//   sort_hist    digit histograms of all passes in one read of the keys
//   sort_pass    one onesweep pass: wavefront ballot ranking into LDS, per-digit
//                decoupled look-back across partitions, coalesced scatter
//   tile_ranges  [start, end) of each tile in the sorted keys
#include <algorithm>

#include "v3dg_internal.h"

namespace v3dg {

constexpr uint32_t kSpinLimitSort = 1u << 24;

__device__ __forceinline__ uint64_t wave_incl_scan_u64s(uint64_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t n = __shfl_up(v, o, kWave);
        if (lane >= o) v += n;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = __shfl_up(v, o, kWave);
        if (lane >= o) v += n;
    }
    return v;
}

// Exclusive scan of one u32 per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *s_tmp /* 4 */, uint32_t *total)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane == kWave - 1) s_tmp[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wid) off += s_tmp[w];
        tot += s_tmp[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// lanes of the wavefront holding the same digit of dbits <= 8 bits (among
// valid lanes; dbits is uniform)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, uint32_t dbits = kRadixBits)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        if ((uint32_t)b >= dbits) break;
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

// ---------------------------------------------------------------------------
// scan of tiles-touched
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanThreads) scan_tiles_kernel(const uint32_t *__restrict__ tiles,
                                                                  const uint32_t *__restrict__ order,
                                                                  const uint32_t *__restrict__ n_dev,
                                                                  const uint32_t *__restrict__ n_culled,
                                                                  uint32_t *__restrict__ offsets,
                                                                  uint64_t *__restrict__ status, uint32_t *counters,
                                                                  uint64_t key_cap)
{
    __shared__ uint32_t s_ticket;
    __shared__ uint64_t s_wave[kScanThreads / kWave];
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    // the last *n_culled ranks are culled slots (no keys): not scanned
    const uint32_t n_all = *n_dev, n = n_culled ? n_all - min(n_all, *n_culled) : n_all;
    const uint32_t nparts = (n + kScanPart - 1) / kScanPart;
    if (tid == 0)
        s_ticket = __hip_atomic_fetch_add(&counters[kRenTicketScan], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t p = s_ticket;
    if (p >= nparts) return;
    const uint64_t base = (uint64_t)p * kScanPart + (uint64_t)tid * kScanItems;
    uint32_t v[kScanItems];
    if (order && base + kScanItems <= n) {
        // a whole run: its ranks in 16-byte loads, then the gathers
        const uint4 *src = reinterpret_cast<const uint4 *>(order + base);
        uint32_t o[kScanItems];
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) {
            const uint4 q = src[j];
            o[4 * j] = q.x;
            o[4 * j + 1] = q.y;
            o[4 * j + 2] = q.z;
            o[4 * j + 3] = q.w;
        }
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = tiles[o[j]];
    } else if (order) {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = (base + j < n) ? tiles[order[base + j]] : 0u;
    } else if (base + kScanItems <= n) {
        const uint4 *src = reinterpret_cast<const uint4 *>(tiles + base);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j) {
            const uint4 q = src[j];
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = (base + j < n) ? tiles[base + j] : 0u;
    }
    uint64_t tsum = 0;
    uint32_t nvis = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t x = v[j];
        v[j] = (uint32_t)tsum;  // local exclusive (fits: <= 16 * 2^20 tiles)
        tsum += x;
        nvis += x != 0u;
    }
    nvis = wave_incl_scan_u32(nvis);
    if (lane == kWave - 1) atomicAdd(&counters[kRenVisible], nvis);
    const uint64_t incl = wave_incl_scan_u64s(tsum);
    if (lane == kWave - 1) s_wave[wid] = incl;
    __syncthreads();
    uint64_t wave_off = 0, block_total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        if (w < wid) wave_off += s_wave[w];
        block_total += s_wave[w];
    }
    const uint64_t t_excl = wave_off + incl - tsum;
    if (tid == 0) {
        uint64_t prefix = 0;
        if (p == 0) {
            __hip_atomic_store(&status[0], (kFlagInc << 62) | block_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[p], (kFlagAgg << 62) | block_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)p - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint64_t w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = w >> 62;
                if (flag == 0) {
                    if (++spins > kSpinLimitSort) {
                        atomicOr(&counters[kRenErr], kErrSpin);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += w & ((1ull << 62) - 1);
                if (flag == kFlagInc) break;
                --j;
            }
            __hip_atomic_store(&status[p], (kFlagInc << 62) | (prefix + block_total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix = prefix;
        if (p == nparts - 1) {
            const uint64_t tot = prefix + block_total;
            counters[kRenKeysLo] = (uint32_t)tot;
            counters[kRenKeysHi] = (uint32_t)(tot >> 32);
            // a frame whose keys do not fit leaves holes in the key buffer: it
            // then sorts, bins and blends nothing (and is flagged)
            counters[kRenKeysEff] = (uint32_t)(tot <= key_cap ? tot : 0);
            if (tot > key_cap) atomicOr(&counters[kRenErr], kErrKeyCap);
        }
    }
    __syncthreads();
    const uint64_t b = s_prefix + t_excl;
    if ((b + tsum) >> 32) atomicOr(&counters[kRenErr], kErrOverflow);
    if (base + kScanItems <= n) {
        uint4 *dst = reinterpret_cast<uint4 *>(offsets + base);
#pragma unroll
        for (int j = 0; j < kScanItems / 4; ++j)
            dst[j] = make_uint4((uint32_t)(b + v[4 * j]), (uint32_t)(b + v[4 * j + 1]), (uint32_t)(b + v[4 * j + 2]),
                                (uint32_t)(b + v[4 * j + 3]));
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j)
            if (base + j < n) offsets[base + j] = (uint32_t)(b + v[j]);
    }
}

void launch_scan_tiles(hipStream_t st, const uint32_t *tiles, const uint32_t *order, const uint32_t *n_dev,
                       const uint32_t *n_culled, uint64_t max_n, uint32_t *offsets, uint64_t *status,
                       uint32_t *counters, uint64_t key_cap)
{
    uint64_t blocks = (max_n + kScanPart - 1) / kScanPart;
    if (blocks < 1) blocks = 1;
    if (key_cap > 0xffffffffull) key_cap = 0xffffffffull;
    hipLaunchKernelGGL(scan_tiles_kernel, dim3((uint32_t)blocks), dim3(kScanThreads), 0, st, tiles, order, n_dev,
                       n_culled, offsets, status, counters, key_cap);
}

// ---------------------------------------------------------------------------
// key emission: one key per tile of every row span of the support
// ---------------------------------------------------------------------------
template <bool DEPTH_FIRST>
__global__ void __launch_bounds__(256) emit_kernel(const uint32_t *__restrict__ n_dev, uint32_t max_n,
                                                   const uint32_t *__restrict__ order,
                                                   const uint32_t *__restrict__ tiles,
                                                   const uint32_t *__restrict__ offsets,
                                                   const BinRec *__restrict__ bin,
                                                   const FrameDev *__restrict__ fd, uint64_t key_cap,
                                                   void *__restrict__ keys_v, uint32_t *__restrict__ vals,
                                                   uint32_t *err)
{
    const uint32_t n = min(*n_dev, max_n);
    const uint32_t tiles_x = fd->cam.bins_x;  // keys name bins
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const uint32_t t = DEPTH_FIRST ? order[j] : j;
        const uint32_t nt = tiles[t];
        if (nt == 0) continue;
        uint64_t off = offsets[j];
        if (off + nt > key_cap) {  // the frame's keys exceed the buffers (flagged by the scan too)
            atomicOr(err, kErrKeyCap);
            continue;
        }
        const uint64_t end = off + nt;
        const BinRec b = bin[t];
        uint32_t tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;  // an empty box lists nothing (and is flagged below)
        bin_box(b, fd->cam.width, fd->cam.height, &tx0, &tx1, &ty0, &ty1);
        const uint64_t dbits = __float_as_uint(b.depth);
        for (uint32_t ty = ty0; ty <= ty1; ++ty) {
            uint32_t lo, hi;
            if (!bin_row_span(b, ty, tx0, tx1, &lo, &hi)) continue;
            for (uint32_t tx = lo; tx <= hi && off < end; ++tx) {
                const uint32_t tile = ty * tiles_x + tx;
                if (DEPTH_FIRST)
                    reinterpret_cast<uint32_t *>(keys_v)[off] = tile;
                else
                    reinterpret_cast<uint64_t *>(keys_v)[off] = ((uint64_t)tile << 32) | dbits;
                vals[off] = t;
                ++off;
            }
        }
        if (off != end) atomicOr(err, kErrOverflow);  // counting and emission disagree
    }
}

void launch_emit64(hipStream_t st, const uint32_t *n_dev, uint64_t max_n, const uint32_t *tiles,
                   const uint32_t *offsets, const BinRec *bin, const FrameDev *fd, uint64_t key_cap, uint64_t *keys,
                   uint32_t *vals, uint32_t *err)
{
    if (max_n == 0) return;
    uint64_t blocks = (max_n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(emit_kernel<false>, dim3((uint32_t)blocks), dim3(256), 0, st, n_dev, (uint32_t)max_n,
                       (const uint32_t *)nullptr, tiles, offsets, bin, fd, key_cap, (void *)keys, vals, err);
}

// Depth-first emission.  Every lane takes one depth rank; its keys (one per
// tile its support reaches, row by row) form a contiguous run of the output
// starting at its scanned offset, so a workgroup's 256 ranks fill one
// contiguous range.  Lanes with at most kSmallKeys keys produce their own run;
// larger splats are produced by the whole wavefront, one splat at a time: lane
// r computes the span of tile row r, and lane l then writes keys l, l + 64, ...
// of the splat, finding its row by a binary search over the row prefix sums.
// The first kStage keys of the workgroup's range (up to the first splat left
// to emit_big_kernel) are assembled in LDS and written out with contiguous
// stores; the rest go straight to global memory.  A lane takes its key count
// from consecutive offsets and its bin box from the binning record, so each
// visible splat costs one 32-byte gather.  The digit histograms of the tile
// sort are counted per row span: a span of consecutive tile ids adds one to a
// run of low digits (a difference array over the 256 bins) and to one or two
// higher digits.
constexpr int kEmitThreads = 256;
constexpr uint32_t kSmallKeys = 48;  // measured best of 8..256 on 1080p orbits
// keys assembled in LDS per workgroup: at 3 bytes each (16-bit key, rank),
// 5,120 keys keep the kernel at 7 waves per SIMD
constexpr uint32_t kStage = 5120;

__device__ __forceinline__ void count_span(uint32_t a, uint32_t b, const DigitPlan &dp, uint32_t *s_d0, uint32_t *s_h,
                                           uint32_t *s_all)
{
    // keys a..b (inclusive): every R0 consecutive ids hold each low digit once
    const uint32_t b0 = dp.bits[0], m0 = (1u << b0) - 1u;
    const uint32_t len = b - a + 1;
    if (len > m0) atomicAdd(s_all, len >> b0);
    const uint32_t rem = len & m0;
    if (rem) {
        const uint32_t la = a & m0, lb = (a + rem - 1) & m0;
        atomicAdd(&s_d0[la], 1u);
        atomicAdd(&s_d0[lb + 1], 0xffffffffu);
        if (la > lb) {  // wraps past the last low digit
            atomicAdd(&s_d0[m0 + 1], 0xffffffffu);
            atomicAdd(&s_d0[0], 1u);
        }
    }
    for (int p = 1; p < dp.passes; ++p) {
        const uint32_t sh = dp.shift[p], mp = (1u << dp.bits[p]) - 1u;
        for (uint32_t h = a >> sh; h <= (b >> sh); ++h) {
            const uint32_t lo = max(a, h << sh), hi = min(b, ((h + 1) << sh) - 1);
            atomicAdd(&s_h[(p - 1) * 256 + (h & mp)], hi - lo + 1);
        }
    }
}

template <typename KT>
struct EmitShared {
    uint32_t d0[257];
    uint32_t h[2 * 256];
    uint32_t all;
    uint32_t wlen;                     // at most this many keys go through LDS
    uint64_t lo, hi;                   // the workgroup's output range
    uint32_t pre[kEmitThreads / kWave][kWave];   // per wavefront: row prefix sums
    uint32_t base[kEmitThreads / kWave][kWave];  //   and first tile of each row
    uint32_t slot[kEmitThreads];  // slot of each rank of the workgroup
    KT key[kStage];               // staged keys, and the rank whose slot is
    uint8_t rank[kStage];         //   each key's value
};

// key q of the workgroup's range (output key lo + q), of the splat of rank r
// in the workgroup (slot t): into the LDS stage when q < wlen, else straight
// to global memory
template <typename KT>
__device__ __forceinline__ void put_key(EmitShared<KT> &sh, uint32_t wlen, uint64_t lo, uint32_t q, uint32_t key,
                                        uint32_t r, uint32_t t, KT *__restrict__ keys, uint32_t *__restrict__ vals)
{
    if (q < wlen) {
        sh.key[q] = (KT)key;
        sh.rank[q] = (uint8_t)r;
    } else {
        keys[lo + q] = (KT)key;
        vals[lo + q] = t;
    }
}

// KT: uint16_t when every tile id fits in 16 bits, else uint32_t
// Splats of more than kBigKeys keys are left to emit_big_kernel: the
// emission kernel lists them (their rank j) in big[], counted in *n_big.  A
// workgroup's LDS window ends before the keys of the first splat it lists, so
// the two kernels never write the same keys.
constexpr uint32_t kBigKeys = 2048;

template <typename KT>
__global__ void __launch_bounds__(kEmitThreads) emit32_kernel(
    const uint32_t *__restrict__ n_dev, uint32_t max_n, const uint32_t *__restrict__ order,
    const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ scan_ctr, const BinRec *__restrict__ bin,
    const FrameDev *__restrict__ fd, uint64_t key_cap, DigitPlan dp,
    KT *__restrict__ keys, uint32_t *__restrict__ vals, uint32_t *__restrict__ hist, uint32_t *__restrict__ big,
    uint32_t *n_big, uint32_t *err)
{
    __shared__ EmitShared<KT> sh;
    static_assert(kEmitThreads <= 256, "a rank is stored in one byte");
    // culled slots (no key) sort after every visible one: only the first
    // kRenVisible ranks emit, and the last of them ends at the frame's total
    const uint32_t n = min(min(*n_dev, max_n), scan_ctr[kRenVisible]);
    if (blockIdx.x * kEmitThreads >= n) return;  // whole workgroup past the end
    const uint32_t tiles_x = fd->cam.bins_x;  // keys name bins
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    for (int i = tid; i < 257; i += kEmitThreads) sh.d0[i] = 0u;
    for (int i = tid; i < 2 * 256; i += kEmitThreads) sh.h[i] = 0u;
    if (tid == 0) sh.all = 0u;
    const uint32_t j = blockIdx.x * kEmitThreads + tid;
    const bool valid = j < n;
    const uint32_t t = valid ? order[j] : 0u;
    sh.slot[tid] = t;
    // the offsets are the exclusive scan of the ranks' key counts: rank j has
    // the difference to the next offset (the last rank: to the total), so the
    // count needs no gather by slot
    const uint32_t off32 = valid ? offsets[j] : 0u;
    const uint32_t next = valid ? (j + 1 < n ? offsets[j + 1] : scan_ctr[kRenKeysLo]) : 0u;
    uint32_t nt = next - off32;
    const uint64_t off = off32;
    // output range of the workgroup: from its first rank to its last rank's end
    if (tid == 0) {
        sh.lo = off;
        sh.wlen = kStage;
    }
    if (valid && (j + 1 == n || tid == kEmitThreads - 1)) sh.hi = off + nt;
    if (off + nt > key_cap) {  // the frame's keys exceed the buffers (flagged by the scan too)
        atomicOr(err, kErrKeyCap);
        nt = 0;
    }
    __syncthreads();
    // the keys of a splat listed for emit_big_kernel are written by that
    // kernel: the LDS window ends before the first of them
    if (nt > kBigKeys) atomicMin(&sh.wlen, (uint32_t)(off - sh.lo));
    __syncthreads();
    // keys [lo, lo + wlen) of the workgroup's range are assembled in LDS, the
    // rest go straight to global memory (none when the range passes key_cap)
    const uint64_t wlo = sh.lo;
    const uint32_t wlen = sh.hi <= key_cap ? (uint32_t)min<uint64_t>(sh.hi - wlo, (uint64_t)sh.wlen) : 0u;
    BinRec b{};
    uint32_t tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;  // an empty box lists nothing (and is flagged below)
    if (nt) {
        b = bin[t];
        bin_box(b, fd->cam.width, fd->cam.height, &tx0, &tx1, &ty0, &ty1);
    }
    // small splats: this lane writes its own run
    if (nt && nt <= kSmallKeys) {
        uint32_t left = nt;                    // keys left to write
        uint32_t q = (uint32_t)(off - wlo);    // position in the workgroup's range
        for (uint32_t ty = ty0; ty <= ty1 && left != 0u; ++ty) {
            uint32_t lo, hi;
            if (!bin_row_span(b, ty, tx0, tx1, &lo, &hi)) continue;
            const uint32_t row = ty * tiles_x;
            count_span(row + lo, row + hi, dp, sh.d0, sh.h, &sh.all);
            const uint32_t m = min(hi - lo + 1u, left);
            for (uint32_t i = 0; i < m; ++i) put_key(sh, wlen, wlo, q + i, row + lo + i, (uint32_t)tid, t, keys, vals);
            q += m;
            left -= m;
        }
        if (left != 0u) atomicOr(err, kErrOverflow);  // counting and emission disagree
    }
    // the largest splats: listed for emit_big_kernel
    if (nt > kBigKeys) big[atomicAdd(n_big, 1u)] = j;
    // larger splats: the wavefront writes them one after another
    uint64_t mid = __ballot(nt > kSmallKeys && nt <= kBigKeys);
    while (mid) {
        const int L = __ffsll((unsigned long long)mid) - 1;
        mid &= mid - 1;
        const uint32_t bt = __shfl(t, L, kWave);
        const uint32_t bn = __shfl(nt, L, kWave);
        uint64_t bo = ((uint64_t)__shfl((uint32_t)(off >> 32), L, kWave) << 32) | __shfl((uint32_t)off, L, kWave);
        const uint64_t bend = bo + bn;
        const uint32_t bx0 = __shfl(tx0, L, kWave), bx1 = __shfl(tx1, L, kWave);
        const uint32_t by0 = __shfl(ty0, L, kWave), by1 = __shfl(ty1, L, kWave);
        BinRec bb;
        bb.mx = __shfl(b.mx, L, kWave);
        bb.my = __shfl(b.my, L, kWave);
        bb.sa = __shfl(b.sa, L, kWave);
        bb.sb = __shfl(b.sb, L, kWave);
        bb.sc = __shfl(b.sc, L, kWave);
        bb.det = __shfl(b.det, L, kWave);
        bb.Qm = __shfl(b.Qm, L, kWave);
        bb.depth = __shfl(b.depth, L, kWave);
        for (uint32_t rb = by0; rb <= by1; rb += kWave) {
            const uint32_t ty = rb + (uint32_t)lane;
            uint32_t lo = 0, len = 0;
            if (ty <= by1) {
                uint32_t hi;
                if (bin_row_span(bb, ty, bx0, bx1, &lo, &hi)) {
                    len = hi - lo + 1;
                    count_span(ty * tiles_x + lo, ty * tiles_x + hi, dp, sh.d0, sh.h, &sh.all);
                }
            }
            const uint32_t incl = wave_incl_scan_u32(len);
            const uint32_t pre = incl - len;
            const uint32_t total = __shfl(incl, kWave - 1, kWave);
            sh.pre[wid][lane] = pre;
            sh.base[wid][lane] = ty * tiles_x + lo;
            __builtin_amdgcn_wave_barrier();
            // key q of this block of rows lies in the last row whose prefix is <= q
            for (uint32_t q = (uint32_t)lane; q < total; q += kWave) {
                uint32_t r = 0;
#pragma unroll
                for (uint32_t step = kWave / 2; step > 0; step >>= 1)
                    if (sh.pre[wid][r + step] <= q) r += step;
                const uint64_t o = bo + q;
                if (o < bend)
                    put_key(sh, wlen, wlo, (uint32_t)(o - wlo), sh.base[wid][r] + (q - sh.pre[wid][r]),
                            (uint32_t)(wid * kWave + L), bt, keys, vals);
            }
            __builtin_amdgcn_wave_barrier();
            bo += total;
        }
        if (bo != bend && lane == 0) atomicOr(err, kErrOverflow);  // counting and emission disagree
    }
    __syncthreads();
    for (uint32_t i = tid; i < wlen; i += kEmitThreads) {  // contiguous copy of the assembled keys
        keys[wlo + i] = sh.key[i];
        vals[wlo + i] = sh.slot[sh.rank[i]];
    }
    // digit histograms: prefix of the difference array gives the low-digit counts
    if (tid < kWave) {
        uint32_t run = 0;
        for (int c = 0; c < 4; ++c) {
            const uint32_t v = sh.d0[c * kWave + tid];
            const uint32_t incl = wave_incl_scan_u32(v);
            const uint32_t cntd = run + incl + ((uint32_t)(c * kWave + tid) >> dp.bits[0] == 0u ? sh.all : 0u);
            if (cntd) atomicAdd(&hist[c * kWave + tid], cntd);
            run += __shfl(incl, kWave - 1, kWave);
        }
    }
    for (int p = 1; p < dp.passes; ++p)
        for (int i = tid; i < 256; i += kEmitThreads)
            if (sh.h[(p - 1) * 256 + i]) atomicAdd(&hist[p * 256 + i], sh.h[(p - 1) * 256 + i]);
}

// The listed splats, one workgroup at a time per splat: the threads take its
// tile rows 256 at a time, a workgroup scan of the row lengths places the rows,
// and all threads write the keys (key q lies in the last row whose prefix is
// <= q).  Digit histograms as in emit32_kernel.
template <typename KT>
__global__ void __launch_bounds__(kEmitThreads) emit_big_kernel(
    const uint32_t *__restrict__ n_big, const uint32_t *__restrict__ big, const uint32_t *__restrict__ order,
    const uint32_t *__restrict__ tiles, const uint32_t *__restrict__ offsets, const BinRec *__restrict__ bin,
    const FrameDev *__restrict__ fd, DigitPlan dp, KT *__restrict__ keys,
    uint32_t *__restrict__ vals, uint32_t *__restrict__ hist, uint32_t *err)
{
    __shared__ uint32_t s_d0[257], s_h[2 * 256], s_all, s_tmp[4];
    __shared__ uint32_t s_pre[kEmitThreads], s_base[kEmitThreads];
    const uint32_t nb = *n_big;
    if (blockIdx.x >= nb) return;
    const int tid = threadIdx.x;
    for (int i = tid; i < 257; i += kEmitThreads) s_d0[i] = 0u;
    for (int i = tid; i < 2 * 256; i += kEmitThreads) s_h[i] = 0u;
    if (tid == 0) s_all = 0u;
    __syncthreads();
    const uint32_t tiles_x = fd->cam.bins_x;  // keys name bins
    for (uint32_t e = blockIdx.x; e < nb; e += gridDim.x) {
        const uint32_t j = big[e], t = order[j], nt = tiles[t];
        const uint64_t off = offsets[j];
        const BinRec b = bin[t];
        uint32_t tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;  // an empty box lists nothing (and is flagged below)
        bin_box(b, fd->cam.width, fd->cam.height, &tx0, &tx1, &ty0, &ty1);
        uint64_t o = off;
        for (uint32_t rb = ty0; rb <= ty1; rb += kEmitThreads) {
            const uint32_t ty = rb + (uint32_t)tid;
            uint32_t lo = 0, len = 0;
            if (ty <= ty1) {
                uint32_t hi;
                if (bin_row_span(b, ty, tx0, tx1, &lo, &hi)) {
                    len = hi - lo + 1;
                    count_span(ty * tiles_x + lo, ty * tiles_x + hi, dp, s_d0, s_h, &s_all);
                }
            }
            uint32_t total;
            const uint32_t pre = block_excl_scan_256(len, s_tmp, &total);
            s_pre[tid] = pre;
            s_base[tid] = ty * tiles_x + lo;
            __syncthreads();
            for (uint32_t q = (uint32_t)tid; q < total; q += kEmitThreads) {
                uint32_t r = 0;
#pragma unroll
                for (uint32_t step = kEmitThreads / 2; step > 0; step >>= 1)
                    if (s_pre[r + step] <= q) r += step;
                if (o + q < off + nt) {
                    keys[o + q] = (KT)(s_base[r] + (q - s_pre[r]));
                    vals[o + q] = t;
                }
            }
            __syncthreads();
            o += total;
        }
        if (o != off + nt && tid == 0) atomicOr(err, kErrOverflow);  // counting and emission disagree
    }
    __syncthreads();
    if (tid < kWave) {
        uint32_t run = 0;
        for (int c = 0; c < 4; ++c) {
            const uint32_t v = s_d0[c * kWave + tid];
            const uint32_t incl = wave_incl_scan_u32(v);
            const uint32_t cntd = run + incl + ((uint32_t)(c * kWave + tid) >> dp.bits[0] == 0u ? s_all : 0u);
            if (cntd) atomicAdd(&hist[c * kWave + tid], cntd);
            run += __shfl(incl, kWave - 1, kWave);
        }
    }
    for (int p = 1; p < dp.passes; ++p)
        for (int i = tid; i < 256; i += kEmitThreads)
            if (s_h[(p - 1) * 256 + i]) atomicAdd(&hist[p * 256 + i], s_h[(p - 1) * 256 + i]);
}

template <typename KT>
void launch_emit32(hipStream_t st, const uint32_t *n_dev, uint64_t max_n, const uint32_t *order,
                   const uint32_t *tiles, const uint32_t *offsets, const uint32_t *scan_ctr, const BinRec *bin,
                   const FrameDev *fd, uint64_t key_cap, const DigitPlan &dp, KT *keys, uint32_t *vals, uint32_t *hist,
                   uint32_t *big, uint32_t *n_big, uint32_t *err)
{
    if (max_n == 0) return;
    const uint32_t blocks = (uint32_t)((max_n + kEmitThreads - 1) / kEmitThreads);
    hipLaunchKernelGGL(emit32_kernel<KT>, dim3(blocks), dim3(kEmitThreads), 0, st, n_dev, (uint32_t)max_n, order,
                       offsets, scan_ctr, bin, fd, key_cap, dp, keys, vals, hist, big, n_big, err);
    // a fixed grid walks the list (any number of its slots may be large)
    const uint32_t bblocks = (uint32_t)(max_n < 2048 ? max_n : 2048);
    hipLaunchKernelGGL(emit_big_kernel<KT>, dim3(bblocks), dim3(kEmitThreads), 0, st, n_big, big, order, tiles,
                       offsets, bin, fd, dp, keys, vals, hist, err);
}

// ---------------------------------------------------------------------------
// digit histograms for all passes (one read of the keys).  Lanes holding the
// same digit are matched by ballot and counted by one LDS atomic.
// ---------------------------------------------------------------------------
// 1,024 threads of a workgroup, kHistItems keys each per stride
constexpr int kHistThreads = 1024;
constexpr int kHistItems = 4;

template <typename K>
__global__ void __launch_bounds__(kHistThreads) sort_hist_kernel(const K *__restrict__ keys,
                                                                 const uint32_t *__restrict__ n_dev, uint64_t n_host,
                                                                 int passes, uint32_t *__restrict__ hist,
                                                                 uint32_t *__restrict__ dropped)
{
    __shared__ uint32_t s_h[8 * kRadix];
    __shared__ uint32_t s_drop;
    for (int i = threadIdx.x; i < passes * kRadix; i += blockDim.x) s_h[i] = 0;
    if (threadIdx.x == 0) s_drop = 0u;
    __syncthreads();
    uint32_t my_drop = 0;
    const uint64_t n = n_dev ? min((uint64_t)*n_dev, n_host) : n_host;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // whole wavefronts iterate together so that ballots see every lane; the
    // keys of kHistItems strides are loaded before any is counted, so their
    // loads are in flight together
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n;
         base += stride * kHistItems) {
        K kk[kHistItems];
#pragma unroll
        for (int u = 0; u < kHistItems; ++u) {
            const uint64_t i = base + u * stride + lane;
            kk[u] = i < n ? keys[i] : (K)0;
        }
#pragma unroll
        for (int u = 0; u < kHistItems; ++u) {
            bool valid = base + u * stride + lane < n;
            if (dropped && valid && kk[u] == (K)~(K)0) {  // a dropped key: counted apart
                valid = false;
                ++my_drop;
            }
            // a wavefront whose keys are all dropped (or past the end) counts
            // no digit (uniform: culled slots come in runs, a cluster at a time)
            if (__ballot(valid) == 0) continue;
            for (int p = 0; p < passes; ++p) {
                const uint32_t d = (uint32_t)(kk[u] >> (p * kRadixBits)) & (kRadix - 1);
                const uint64_t peers = match_digit(d, valid);
                if (valid && (peers & lt) == 0) atomicAdd(&s_h[p * kRadix + d], (uint32_t)__popcll(peers));
            }
        }
    }
    if (dropped && my_drop) atomicAdd(&s_drop, my_drop);
    __syncthreads();
    for (int i = threadIdx.x; i < passes * kRadix; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
    if (dropped && threadIdx.x == 0 && s_drop) atomicAdd(dropped, s_drop);
}

template <typename K>
void launch_sort_hist(hipStream_t st, const K *keys, const uint32_t *n_dev, uint64_t n, int passes, uint32_t *hist,
                      uint32_t *dropped)
{
    if (n == 0) return;
    uint64_t blocks = (n + kHistThreads * kHistItems - 1) / (kHistThreads * kHistItems);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(sort_hist_kernel<K>, dim3((uint32_t)blocks), dim3(kHistThreads), 0, st, keys, n_dev, n, passes,
                       hist, dropped);
}

// ---------------------------------------------------------------------------
// one onesweep digit pass
// ---------------------------------------------------------------------------
// look-back word: epoch (30 bits) | flag (2 bits) | count (32 bits)
__device__ __forceinline__ uint64_t lb_word(uint32_t epoch, uint64_t flag, uint32_t v)
{
    return ((uint64_t)epoch << 34) | (flag << 32) | v;
}

// 16-bit keys: three workgroups per CU fit in LDS, so registers are held to
// three waves per SIMD as well
template <typename K, int ITEMS, bool DROP>
__device__ __forceinline__ void sort_pass_body(const K *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
                                               K *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                                               const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
                                               uint32_t dbits, const uint32_t *__restrict__ hist, uint64_t *status,
                                               const uint32_t *__restrict__ epoch_dev, uint32_t epoch_arg,
                                               uint32_t *ticket, uint32_t *err, const uint32_t *__restrict__ dropped,
                                               uint32_t *__restrict__ n_kept)
{
    constexpr int NW = kSortThreads / kWave;           // waves per block
    constexpr int PART = kSortThreads * ITEMS;         // keys of a partition
    constexpr int WAVE_KEYS = PART / NW;               // consecutive keys owned by a wave
    constexpr int ROUNDS = WAVE_KEYS / kWave;          // = ITEMS
    __shared__ K s_keys[PART];
    __shared__ uint32_t s_vals[PART];
    __shared__ uint32_t s_whist[NW][kRadix];
    __shared__ uint32_t s_lstart[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_tmp[4];
    __shared__ uint32_t s_ticket;

    const int wid = (int)threadIdx.x / kWave;
    // DROP: this pass leaves out the keys of all ones (*dropped of them,
    // counted apart by the histogram, which does not count their digits) and
    // writes the count of the others to *n_kept, the key count of the passes
    // after it.  A template parameter: the test costs the other passes
    // registers (the 16-bit pass spilled)
    const uint32_t n = n_dev ? min(*n_dev, n_host) : n_host;
    if constexpr (DROP) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *n_kept = n - min(n, *dropped);
    }
    const uint32_t epoch = epoch_dev ? *epoch_dev + epoch_arg : epoch_arg;
    const uint32_t nparts = (n + PART - 1) / PART;
    const uint32_t dmask = (1u << dbits) - 1u;  // digits d > dmask never occur: no look-back for them
    // Partitions are claimed in ticket order until none is left, so the grid
    // need not match the key count (a bound on it, or far fewer workgroups,
    // both work).  A partition only waits on lower tickets, claimed earlier
    // by running workgroups.
    for (;;) {
    // the thread index, opaque to the compiler once per partition: otherwise
    // the per-item offsets derived from it are hoisted out of the loop and
    // held in about 48 more registers, which costs a workgroup per CU
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & (kWave - 1);
    for (int i = tid; i < NW * kRadix; i += kSortThreads) (&s_whist[0][0])[i] = 0u;
    if (tid == 0) s_ticket = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t p = s_ticket;
    if (p >= nparts) return;  // uniform
    const uint32_t part_base = p * (uint32_t)PART;
    const uint32_t wave_base = part_base + (uint32_t)wid * WAVE_KEYS;
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    K key[ROUNDS];
    uint32_t val[ROUNDS];
    uint32_t dr[ROUNDS];  // digit | rank-in-wave << 8
    // all loads first, so that the partition's 2 x 16 loads per lane are in
    // flight together (ranking round by round would wait for each in turn)
    if (part_base + (uint32_t)PART <= n) {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            key[r] = keys_in[wave_base + r * kWave + lane];
            val[r] = vals_in[wave_base + r * kWave + lane];
        }
    } else {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const uint32_t idx = wave_base + r * kWave + lane;
            key[r] = idx < n ? keys_in[idx] : (K)0;
            val[r] = idx < n ? vals_in[idx] : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t idx = wave_base + r * kWave + lane;
        const bool valid = idx < n && !(DROP && key[r] == (K)~(K)0);
        const K k = key[r];
        const uint32_t d = (uint32_t)(k >> shift) & dmask;
        const uint64_t peers = match_digit(d, valid, dbits);
        const uint32_t rank_in_round = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t old = 0;
        if (valid) old = s_whist[wid][d];
        if (valid && rank_in_round == 0) s_whist[wid][d] = old + cnt;
        dr[r] = d | ((old + rank_in_round) << 8);
    }
    __syncthreads();

    // per-digit totals, wave offsets, look-back (thread d handles digit d)
    const int d = tid;
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t c = s_whist[w][d];
        s_whist[w][d] = total;
        total += c;
    }
    uint64_t *my = status + (uint64_t)p * kRadix + d;
    uint32_t prefix = 0;
    if ((uint32_t)d > dmask) {
        // a digit wider than the pass's: no key holds it, no partition looks it up
    } else if (p == 0) {
        __hip_atomic_store(my, lb_word(epoch, kFlagInc, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(my, lb_word(epoch, kFlagAgg, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t j = (int64_t)p - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            const uint64_t w = __hip_atomic_load(status + (uint64_t)j * kRadix + d, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t flag = ((uint32_t)(w >> 34) == epoch) ? ((w >> 32) & 3ull) : 0ull;
            if (flag == 0) {
                if (++spins > kSpinLimitSort) {
                    atomicOr(err, kErrSpin);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            prefix += (uint32_t)w;
            if (flag == kFlagInc) break;
            --j;
        }
        __hip_atomic_store(my, lb_word(epoch, kFlagInc, prefix + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t tot_all;
    const uint32_t lstart = block_excl_scan_256(total, s_tmp, &tot_all);
    uint32_t hist_tot;
    const uint32_t gstart = block_excl_scan_256(hist[d], s_tmp, &hist_tot);
    s_lstart[d] = lstart;
    s_gbase[d] = gstart + prefix;
    __syncthreads();

    // reorder into LDS by digit (stable: wave order, then round, then lane)
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t idx = wave_base + r * kWave + lane;
        if (idx < n && !(DROP && key[r] == (K)~(K)0)) {
            const uint32_t dd = dr[r] & (kRadix - 1);
            const uint32_t pos = s_lstart[dd] + s_whist[wid][dd] + (dr[r] >> 8);
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();
    // keys of the partition in LDS (those not dropped: tot_all)
    const uint32_t n_here = DROP ? tot_all : ((n - part_base) < (uint32_t)PART ? (n - part_base) : (uint32_t)PART);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t i = tid + r * kSortThreads;
        if (i < n_here) {
            const K k = s_keys[i];
            const uint32_t dd = (uint32_t)(k >> shift) & dmask;
            const uint32_t o = s_gbase[dd] + (i - s_lstart[dd]);
            if (o < n) {  // always true when the histogram and look-back agree
                keys_out[o] = k;
                vals_out[o] = s_vals[i];
            }
        }
    }
    __syncthreads();  // the next partition reuses the LDS arrays and the ticket word
    }
}

// The pass kernel; sort_pass_drop_kernel is the same pass with DROP, a kernel
// of its own so that the extra arguments cost the others nothing.
template <typename K, int ITEMS>
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(sizeof(K) == 2 ? 3 : 1)))
sort_pass_kernel(const K *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, K *__restrict__ keys_out,
                 uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
                 uint32_t dbits, const uint32_t *__restrict__ hist, uint64_t *status,
                 const uint32_t *__restrict__ epoch_dev, uint32_t epoch_arg, uint32_t *ticket, uint32_t *err)
{
    sort_pass_body<K, ITEMS, false>(keys_in, vals_in, keys_out, vals_out, n_dev, n_host, shift, dbits, hist, status,
                                    epoch_dev, epoch_arg, ticket, err, nullptr, nullptr);
}

template <typename K, int ITEMS>
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(sizeof(K) == 2 ? 3 : 1)))
sort_pass_drop_kernel(const K *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, K *__restrict__ keys_out,
                      uint32_t *__restrict__ vals_out, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
                      uint32_t dbits, const uint32_t *__restrict__ hist, uint64_t *status,
                      const uint32_t *__restrict__ epoch_dev, uint32_t epoch_arg, uint32_t *ticket, uint32_t *err,
                      const uint32_t *__restrict__ dropped, uint32_t *__restrict__ n_kept)
{
    sort_pass_body<K, ITEMS, true>(keys_in, vals_in, keys_out, vals_out, n_dev, n_host, shift, dbits, hist, status,
                                   epoch_dev, epoch_arg, ticket, err, dropped, n_kept);
}

// Workgroups of one pass that are resident on the device at once.  A pass
// launches no more than that: its workgroups claim partitions until none is
// left, and a workgroup past the resident set would only be dispatched once
// the work is done, to find nothing (such empty workgroups still cost their
// dispatch, at the end of the pass).
template <typename K, int ITEMS>
static uint32_t sort_pass_resident()
{
    static uint32_t per_dev[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return (uint32_t)kSortMaxGrid;
    if (per_dev[dev] == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sort_pass_kernel<K, ITEMS>, kSortThreads, 0) !=
                hipSuccess ||
            cus <= 0 || per_cu <= 0)
            return (uint32_t)kSortMaxGrid;
        per_dev[dev] = (uint32_t)std::min<uint64_t>((uint64_t)cus * (uint64_t)per_cu, kSortMaxGrid);
    }
    return per_dev[dev];
}

template <typename K>
void launch_sort_pass(hipStream_t st, const K *keys_in, const uint32_t *vals_in, K *keys_out, uint32_t *vals_out,
                      const uint32_t *n_dev, uint64_t n, int pass, const uint32_t *hist, uint64_t *status,
                      const uint32_t *epoch_dev, uint32_t epoch, uint32_t *ticket, uint32_t *err, bool wide, int shift,
                      int dbits, const uint32_t *dropped, uint32_t *n_kept)
{
    if (n == 0) return;
    const int sh = shift < 0 ? pass * kRadixBits : shift;
    const uint32_t db = (uint32_t)(dbits < 1 ? 1 : dbits > kRadixBits ? kRadixBits : dbits);
    // wide partitions (6144 keys) for large 32-bit sorts: fewer partitions to
    // look back over and longer digit runs to store
    if (wide && sizeof(K) <= 4) {
        const uint32_t grid = (uint32_t)std::min<uint64_t>((n + kSortPartWide - 1) / kSortPartWide,
                                                           sort_pass_resident<K, kSortItemsWide>());
        if constexpr (sizeof(K) == 4) {
            if (dropped) {
                hipLaunchKernelGGL((sort_pass_drop_kernel<K, kSortItemsWide>), dim3(grid), dim3(kSortThreads), 0, st,
                                   keys_in, vals_in, keys_out, vals_out, n_dev, (uint32_t)n, sh, db,
                                   hist + pass * kRadix, status, epoch_dev, epoch, ticket, err, dropped, n_kept);
                return;
            }
        }
        hipLaunchKernelGGL((sort_pass_kernel<K, kSortItemsWide>), dim3(grid), dim3(kSortThreads), 0, st, keys_in,
                           vals_in, keys_out, vals_out, n_dev, (uint32_t)n, sh, db, hist + pass * kRadix, status,
                           epoch_dev, epoch, ticket, err);
    } else {
        const uint32_t grid = (uint32_t)std::min<uint64_t>((n + kSortPart - 1) / kSortPart,
                                                           sort_pass_resident<K, kSortItems>());
        if constexpr (sizeof(K) == 4) {
            if (dropped) {
                hipLaunchKernelGGL((sort_pass_drop_kernel<K, kSortItems>), dim3(grid), dim3(kSortThreads), 0, st,
                                   keys_in, vals_in, keys_out, vals_out, n_dev, (uint32_t)n, sh, db,
                                   hist + pass * kRadix, status, epoch_dev, epoch, ticket, err, dropped, n_kept);
                return;
            }
        }
        hipLaunchKernelGGL((sort_pass_kernel<K, kSortItems>), dim3(grid), dim3(kSortThreads), 0, st, keys_in,
                           vals_in, keys_out, vals_out, n_dev, (uint32_t)n, sh, db, hist + pass * kRadix, status,
                           epoch_dev, epoch, ticket, err);
    }
}

// ---------------------------------------------------------------------------
// tile ranges: [lower_bound(t), lower_bound(t + 1)) in the sorted keys, one
// binary search per tile instead of a pass over the keys
// ---------------------------------------------------------------------------
template <typename K>
__device__ __forceinline__ uint32_t lower_bound_tile(const K *__restrict__ keys, uint32_t n, int shift, uint32_t t)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((uint32_t)(keys[mid] >> shift) < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename K>
__global__ void __launch_bounds__(256) tile_ranges_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ n_dev,
                                                          int shift, uint32_t tiles_x, uint32_t n_tiles, uint32_t bins_x,
                                                          uint2 *__restrict__ ranges,
                                                          uint32_t *__restrict__ cbase, uint2 *__restrict__ items,
                                                          uint32_t *__restrict__ rounds, uint32_t rcap,
                                                          uint32_t *__restrict__ order, uint32_t *counters,
                                                          uint32_t max_chunks, ChunkPlan cp,
                                                          const uint32_t *__restrict__ sel_counters,
                                                          FrameRec *rec, uint32_t seq)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (rec && t == 0) {  // every earlier kernel of the frame has set its counters and flags
        rec->keys_lo = counters[kRenKeysLo];
        rec->keys_hi = counters[kRenKeysHi];
        rec->visible = counters[kRenVisible];
        rec->err = counters[kRenErr];
        rec->n_slots = sel_counters[kSelNGaussians];
        rec->n_clusters = sel_counters[kSelNClusters];
        __threadfence_system();
        __hip_atomic_store(&rec->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lt = (1ull << lane) - 1ull;
    const bool in = t < n_tiles;
    uint32_t L = 0;
    if (in) {  // the keys of the tile's bin
        const uint32_t n = *n_dev;
        const uint32_t bin = (t / tiles_x) / 2u * bins_x + (t % tiles_x) / 2u;
        const uint2 r = make_uint2(lower_bound_tile(keys, n, shift, bin), lower_bound_tile(keys, n, shift, bin + 1));
        ranges[t] = r;
        L = r.y - r.x;
    }
    // chunk records and work items, one atomic per wavefront for each
    const uint32_t m = (in && L > cp.first()) ? cp.n_chunks(L) : 0u;
    const uint32_t m_incl = wave_incl_scan_u32(m);
    uint32_t m_base = 0;
    if (lane == kWave - 1 && m_incl) m_base = atomicAdd(&counters[kRenChunks], m_incl);
    const uint32_t first = __shfl(m_base, kWave - 1, kWave) + m_incl - m;
    const bool ok = plan_fits(first, m, max_chunks);
    if (in) cbase[t] = ok ? first : kNoChunk;
    // work items: chunk r of every long tile in round r (r <= kChunkRounds).
    // The workgroup orders its long tiles by their number of rounds nr,
    // largest first (a counting sort in LDS): the tiles of round r are then
    // its first cnt_r tiles, cnt_r = #{nr >= r}, so a tile has one position
    // for all its rounds, and each round takes one range with one atomic.
    static_assert(kChunkRounds == kWave, "one wavefront scans the round counts");
    __shared__ uint32_t hcnt[kChunkRounds + 1], hstart[kChunkRounds + 1], rbase[kChunkRounds];
    const uint32_t nr = ok ? min(m - 1u, (uint32_t)kChunkRounds) : 0u;
    if (threadIdx.x <= kChunkRounds) hcnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t rank = nr ? atomicAdd(&hcnt[nr], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < kWave) {  // lane l takes nr = kChunkRounds - l: suffix counts as a prefix scan
        const uint32_t k = (uint32_t)kChunkRounds - (uint32_t)lane;
        const uint32_t v = hcnt[k], cnt = wave_incl_scan_u32(v);  // cnt = #{nr >= k}
        hstart[k] = cnt - v;
        if (cnt) rbase[k - 1] = atomicAdd(&counters[kRenRound + k - 1], cnt);
    }
    __syncthreads();
    const uint32_t pos = nr ? hstart[nr] + rank : 0u;
    for (uint32_t r = 0; r < nr; ++r) rounds[(uint64_t)r * rcap + rbase[r] + pos] = t;
    const uint32_t it = ok && m - 1u > (uint32_t)kChunkRounds ? m - 1u - (uint32_t)kChunkRounds : 0u;
    const uint32_t it_incl = wave_incl_scan_u32(it);
    uint32_t it_base = 0;
    if (lane == kWave - 1 && it_incl) it_base = atomicAdd(&counters[kRenItems], it_incl);
    const uint32_t it_first = __shfl(it_base, kWave - 1, kWave) + it_incl - it;
    for (uint32_t j = 0; j < it; ++j) items[it_first + j] = make_uint2(t, (uint32_t)kChunkRounds + 1u + j);
    // blend order: full first chunks at the front, the rest from the back
    const bool heavy = in && L >= cp.first();
    const uint64_t hb = __ballot(heavy), lb = __ballot(in && !heavy);
    uint32_t fb = 0, bb = 0;
    if (lane == 0) {
        if (hb) fb = atomicAdd(&counters[kRenFront], (uint32_t)__popcll(hb));
        if (lb) bb = atomicAdd(&counters[kRenBack], (uint32_t)__popcll(lb));
    }
    fb = __shfl(fb, 0, kWave);
    bb = __shfl(bb, 0, kWave);
    if (heavy) order[fb + (uint32_t)__popcll(hb & lt)] = t;
    else if (in) order[n_tiles - 1u - (bb + (uint32_t)__popcll(lb & lt))] = t;
}

template <typename K>
void launch_tile_ranges(hipStream_t st, const K *keys, const uint32_t *n_dev, int shift, uint32_t tiles_x,
                        uint32_t n_tiles, uint32_t bins_x, uint2 *ranges, uint32_t *cbase, uint2 *items,
                        uint32_t *rounds, uint32_t rcap, uint32_t *order, uint32_t *counters, uint64_t max_chunks,
                        const ChunkPlan &cp, const uint32_t *sel_counters, FrameRec *rec, uint32_t seq)
{
    hipLaunchKernelGGL(tile_ranges_kernel<K>, dim3((n_tiles + 255) / 256), dim3(256), 0, st, keys, n_dev, shift,
                       tiles_x, n_tiles, bins_x, ranges, cbase, items, rounds, rcap, order, counters,
                       (uint32_t)(max_chunks < 0xffffffffull ? max_chunks : 0xffffffffull), cp, sel_counters, rec,
                       seq);
}

template void launch_emit32<uint16_t>(hipStream_t, const uint32_t *, uint64_t, const uint32_t *, const uint32_t *,
                                      const uint32_t *, const uint32_t *, const BinRec *, const FrameDev *, uint64_t,
                                      const DigitPlan &, uint16_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t *,
                                      uint32_t *);
template void launch_emit32<uint32_t>(hipStream_t, const uint32_t *, uint64_t, const uint32_t *, const uint32_t *,
                                      const uint32_t *, const uint32_t *, const BinRec *, const FrameDev *, uint64_t,
                                      const DigitPlan &, uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t *,
                                      uint32_t *);
template void launch_sort_hist<uint16_t>(hipStream_t, const uint16_t *, const uint32_t *, uint64_t, int, uint32_t *,
                                      uint32_t *);
template void launch_sort_hist<uint32_t>(hipStream_t, const uint32_t *, const uint32_t *, uint64_t, int, uint32_t *,
                                      uint32_t *);
template void launch_sort_hist<uint64_t>(hipStream_t, const uint64_t *, const uint32_t *, uint64_t, int, uint32_t *,
                                      uint32_t *);
template void launch_sort_pass<uint16_t>(hipStream_t, const uint16_t *, const uint32_t *, uint16_t *, uint32_t *,
                                         const uint32_t *, uint64_t, int, const uint32_t *, uint64_t *,
                                         const uint32_t *, uint32_t, uint32_t *, uint32_t *, bool, int, int,
                                         const uint32_t *, uint32_t *);
template void launch_sort_pass<uint32_t>(hipStream_t, const uint32_t *, const uint32_t *, uint32_t *, uint32_t *,
                                         const uint32_t *, uint64_t, int, const uint32_t *, uint64_t *,
                                         const uint32_t *, uint32_t, uint32_t *, uint32_t *, bool, int, int,
                                         const uint32_t *, uint32_t *);
template void launch_sort_pass<uint64_t>(hipStream_t, const uint64_t *, const uint32_t *, uint64_t *, uint32_t *,
                                         const uint32_t *, uint64_t, int, const uint32_t *, uint64_t *,
                                         const uint32_t *, uint32_t, uint32_t *, uint32_t *, bool, int, int,
                                         const uint32_t *, uint32_t *);
template void launch_tile_ranges<uint16_t>(hipStream_t, const uint16_t *, const uint32_t *, int, uint32_t, uint32_t,
                                          uint32_t, uint2 *, uint32_t *, uint2 *, uint32_t *, uint32_t, uint32_t *,
                                          uint32_t *, uint64_t, const ChunkPlan &, const uint32_t *, FrameRec *,
                                          uint32_t);
template void launch_tile_ranges<uint32_t>(hipStream_t, const uint32_t *, const uint32_t *, int, uint32_t, uint32_t,
                                          uint32_t, uint2 *, uint32_t *, uint2 *, uint32_t *, uint32_t, uint32_t *,
                                          uint32_t *, uint64_t, const ChunkPlan &, const uint32_t *, FrameRec *,
                                          uint32_t);
template void launch_tile_ranges<uint64_t>(hipStream_t, const uint64_t *, const uint32_t *, int, uint32_t, uint32_t,
                                          uint32_t, uint2 *, uint32_t *, uint2 *, uint32_t *, uint32_t, uint32_t *,
                                          uint32_t *, uint64_t, const ChunkPlan &, const uint32_t *, FrameRec *,
                                          uint32_t);

}  // namespace v3dg
