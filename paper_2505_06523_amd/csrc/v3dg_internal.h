// Internal declarations shared by the HIP kernels and the C++ runtime of v3dg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blend_plan.h"

namespace v3dg {

constexpr int kTile = 16;               // edge in pixels of a tile (blended by one workgroup)
constexpr int kBin = 32;                // edge in pixels of a bin (a 2 x 2 block of tiles); keys name bins
static_assert(kBin == 2 * kTile && kTilesPerBin == 4, "a bin is a 2 x 2 block of tiles");
constexpr int kWave = 64;               // CDNA wavefront width

// Gaussian attributes are structure-of-arrays planes with a common stride
// (the row count rounded up to 64): 3 FP32 position planes; 8 "geometry"
// planes (scale x/y/z, quaternion w/x/y/z, opacity) in FP32 or FP16; and
// 3 (d+1)^2 SH planes (coefficient k, channel c at 3k + c) in FP32, BF16 or
// FP16, by storage precision.
constexpr int kGeoSX = 0, kGeoSY = 1, kGeoSZ = 2;
constexpr int kGeoQW = 3, kGeoQX = 4, kGeoQY = 5, kGeoQZ = 6, kGeoOP = 7;
constexpr int kGeoPlanes = 8;

struct Attribs {
    const float *pos;   // 3 planes
    const void *geo;    // 8 planes
    const void *sh;     // 3 (d+1)^2 planes
    uint64_t ps;        // plane stride in elements
};

// Per-instance frame record (64 B): A = fl32(V T) row-major 3x4, the camera
// centre in the asset frame (for view-dependent colour) and the uniform scale.
struct alignas(16) InstRec {
    float A[12];
    float chat[3];
    float s;
};

// Camera constants passed by value to kernels.
struct CamArgs {
    float V[12];
    double cw[3];            // camera centre in world space (FP64)
    float fx, fy, cx, cy;
    float near_plane, far_plane;
    float limx, limy;        // guard band of the EWA Jacobian: 1.3 * tan(half fov)
    float bg[3];
    uint32_t width, height, tiles_x, tiles_y, bins_x, bins_y;
};

// Per-frame state of a render context in device memory.  The first kernel of
// a frame writes it (or, in a replayed graph, the host copies it in before the
// replay); every later kernel of the frame reads camera, image and sort epoch
// from here, so a captured chain of launches serves any camera of its size.
struct FrameDev {
    CamArgs cam;
    float *image;        // H x W x 4 FP32 RGBA, caller-owned
    uint32_t epoch;      // look-back epoch base of the frame's sorts (advanced by kEpochsPerFrame)
    uint32_t pad;
};
constexpr uint32_t kEpochsPerFrame = 8;    // depth sort passes 0..3, tile sort passes 4..7
constexpr uint32_t kEpochLimit = 1u << 30; // width of the epoch field of a sort look-back word

// Look-back status words: two flag bits above the payload.
constexpr uint64_t kFlagAgg = 1ull;
constexpr uint64_t kFlagInc = 2ull;

// The counts of one frame, written by the device into pinned host memory
// once its keys are sorted, so that the host can read them after the frame
// without a copy of its own.
struct FrameRec {
    uint32_t keys_lo, keys_hi, visible, err, n_slots, n_clusters, seq, pad;
};

// Device-side frame counters (u32 words) of a selection.
enum SelCounter : int {
    kSelTicket = 0,
    kSelErr = 1,
    kSelNClusters = 2,
    kSelNGaussians = 3,
    kSelCounters = 8
};

// Device-side frame counters of a render workspace.
enum RenderCounter : int {
    kRenTicketScan = 0,
    kRenErr = 1,
    kRenKeysLo = 2,       // total keys (64-bit, lo/hi)
    kRenKeysHi = 3,
    kRenVisible = 4,      // slots with at least one tile
    kRenChunks = 5,       // chunks of long tiles (blending)
    kRenItems = 6,        // chunk work items (chunks past the first)
    kRenRewalk = 7,       // chunks walked again (they hold a pixel's stop)
    kRenTicketSort = 8,   // 8 passes of the tile (or 64-bit) sort
    kRenTicketDepth = 16, // 4 passes of the depth sort
    kRenFront = 20,       // tiles placed at the front of the blend order (long lists)
    kRenBack = 21,        // tiles placed at its back
    kRenFp64 = 22,        // splats whose 2D covariance was redone in FP64 (det < 1e-6)
    kRenConicClamp = 23,  // splats with a conic entry clamped to +-kConicMax
    kRenCulled = 24,      // slots the projection culled (depth key 0xffffffff; counted by the depth histogram)
    kRenDepthKept = 25,   // slots the depth sort keeps: the visible ones
    kRenHist = 32,        // 8 passes x 256 bins
    kRenHistDepth = 32 + 8 * 256,  // 4 passes x 256 bins
    kRenKeysEff = 32 + 12 * 256,   // keys the frame's buffers hold: min(total, capacity)
    kRenBig = 32 + 12 * 256 + 1,   // splats left to the large-splat emission
    kRenRound = 32 + 12 * 256 + 32,       // kChunkRounds counters: long tiles in round r + 1
    kRenCounters = 32 + 12 * 256 + 32 + 64
};
// Chunks 1 .. kChunkRounds of the long lists are handed out round by round
// (every long tile's chunk 1, then every chunk 2, ...); later chunks after
// them, tile by tile.
constexpr int kChunkRounds = 64;
static_assert(kRenRound + kChunkRounds <= kRenCounters, "round counters out of range");

// Error flag bits
constexpr uint32_t kErrSpin = 1u;       // a bounded look-back wait expired
constexpr uint32_t kErrOverflow = 2u;   // a count did not fit its field, or counting and emission disagreed
constexpr uint32_t kErrKeyCap = 4u;     // the frame's keys exceed its key buffers (capacity-sized launches)

// ---- conservative tile coverage of a splat's support -----------------------
// The support of a splat is {d : d^T Sigma^-1 d <= Q}, Q = 2 ln(255 o), the
// pixels where alpha >= 1/255.  Binning keeps, for every tile row, only the
// tiles that an enlarged support (Qm = 1.05 Q + 0.05, one extra pixel on each
// side) reaches, computed from Sigma = [[sa, sb], [sb, sc]] and its determinant.
// Given dy, the support is an x-interval centred on (sb/sc) dy with half-width
// sqrt((Qm - dy^2/sc) det/sc); its right end is concave in dy and peaks at the
// rightmost point dy_r = sb sqrt(Qm/sa), its left end is convex with minimum at
// -dy_r, so the extreme x over a band of rows is found by clamping dy_r.
// The same function, compiled without contraction, is used to count the
// tiles (projection) and to write them (emission), so both agree bit for bit.
struct BinRec {            // per visible slot, 32 B
    float mx, my, sa, sb;  // mean, Sigma entries
    float sc, det, Qm, depth;
};

// Bins of bin row by (pixel centres kBin by + 0.5 .. + kBin - 0.5) that the
// enlarged support (binning record b) reaches, clipped to [bx_min, bx_max]:
// the x-extent of the ellipse over the row's pixel-centre band (plus one
// pixel each way) is exact, so no bin is listed that the support misses.
__device__ __forceinline__ bool bin_row_span(const BinRec &b, uint32_t by, uint32_t bx_min, uint32_t bx_max,
                                             uint32_t *bx_lo, uint32_t *bx_hi)
{
#pragma clang fp contract(off)
    constexpr float kEdge = (float)kBin, kInv = 1.0f / (float)kBin;  // exact: a power of two
    const float ya = (float)(by * (uint32_t)kBin) + 0.5f, yb = ya + (kEdge - 1.0f);
    const float ymax = sqrtf(b.Qm * b.sc);
    const float lo = fmaxf(ya - 1.0f - b.my, -ymax);
    const float hi = fminf(yb + 1.0f - b.my, ymax);
    if (!(lo <= hi)) return false;
    const float k = b.sb / b.sc;
    const float s2 = b.det / b.sc;
    const float dyr = b.sb * sqrtf(b.Qm / b.sa);
    const float dr = fminf(fmaxf(dyr, lo), hi);
    const float dl = fminf(fmaxf(-dyr, lo), hi);
    const float wr = sqrtf(fmaxf(0.0f, (b.Qm - dr * dr / b.sc) * s2));
    const float wl = sqrtf(fmaxf(0.0f, (b.Qm - dl * dl / b.sc) * s2));
    const float xr = b.mx + k * dr + wr + 1.0f;
    const float xl = b.mx + k * dl - wl - 1.0f;
    // bin bx holds pixel centres kBin bx + 0.5 .. kBin bx + kBin - 0.5
    const float flo = ceilf((xl - (kEdge - 0.5f)) * kInv), fhi = floorf((xr - 0.5f) * kInv);
    const float clo = fmaxf(flo, (float)bx_min), chi = fminf(fhi, (float)bx_max);
    if (!(clo <= chi)) return false;
    *bx_lo = (uint32_t)clo;
    *bx_hi = (uint32_t)chi;
    return true;
}

// Bins [tx0, tx1] x [ty0, ty1] of the box around the enlarged support of
// binning record b (half-extents sqrt(Qm Sxx) + 1 and sqrt(Qm Syy) + 1
// pixels), clipped to the image; false when the box holds no pixel centre.
// Projection counts a splat's keys over this box and emission lists them over
// the same box, so both take it from here.
__device__ __forceinline__ bool bin_box(const BinRec &b, uint32_t width, uint32_t height, uint32_t *tx0,
                                        uint32_t *tx1, uint32_t *ty0, uint32_t *ty1)
{
#pragma clang fp contract(off)
    const float hx = sqrtf(b.Qm * b.sa) + 1.0f, hy = sqrtf(b.Qm * b.sc) + 1.0f;
    const float fx0 = fmaxf(ceilf(b.mx - hx - 0.5f), 0.0f);
    const float fx1 = fminf(floorf(b.mx + hx - 0.5f), (float)(width - 1));
    const float fy0 = fmaxf(ceilf(b.my - hy - 0.5f), 0.0f);
    const float fy1 = fminf(floorf(b.my + hy - 0.5f), (float)(height - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return false;
    *tx0 = (uint32_t)fx0 / kBin;
    *tx1 = (uint32_t)fx1 / kBin;
    *ty0 = (uint32_t)fy0 / kBin;
    *ty1 = (uint32_t)fy1 / kBin;
    return true;
}

// ---- launch wrappers (implemented in the .hip files) ----------------------
// select.hip
// Render set-up: itab from the camera and the instances, clearing of the
// frame's counters and look-back words, and the frame state: with from_fd the
// camera is read from fd (already copied in), otherwise cam/image are written
// there.  bump_epoch advances fd->epoch by kEpochsPerFrame.
void launch_frame_setup(hipStream_t st, const CamArgs &cam, float *image, FrameDev *fd, bool from_fd, bool bump_epoch,
                        const double *T, const float *inst_scale, uint32_t n_inst, InstRec *itab, uint32_t *clear,
                        uint64_t n_clear);
constexpr int kSelThreads = 256;
constexpr int kSelItems = 2;
constexpr int kSelPart = kSelThreads * kSelItems;
// View culling of cut clusters (optional).  A cluster whose rows' means lie
// in the sphere sph (asset frame) and whose scales are at most smax cannot
// reach the image when, for every point of the sphere seen through an
// instance, the enlarged support box of a Gaussian there (half-extent at most
// 3.5 (1 + guard band) f s smax / z + 1 pixels) stays 2 pixels outside the
// image, or the sphere lies behind the near plane.  Each side is a plane test
// on the sphere in camera space (all in FP64).
struct CullRec {
    float4 sph;     // centre and radius of the rows' means
    float smax;     // largest scale of the rows
    float pad[3];
};
struct CullCam {    // plane coefficients of one camera (host-computed in FP64)
    double fx, fy;
    double al, ar, at, ab;   // z coefficients: left/right/top/bottom
    double nl, nr, nt, nb;   // norms of (f, coefficient)
    double kx, ky;           // 3.5 (1 + guard band) f
    double nearp;
};

// One selection request: its asset tables, frame records and outputs.
struct SelReq {
    const float4 *self_sph, *par_sph;
    const uint2 *rowinfo;
    const InstRec *itab;
    uint32_t *gid, *slot_off;
    uint64_t *status;
    uint32_t *counters;       // kSelCounters words
    uint32_t *slot_row, *slot_inst;
    uint32_t NC, n_inst;
    float K, tau;
    uint32_t part_begin;      // first partition of this request in the batch
    uint32_t nparts;
    const CullRec *cull;      // nullptr: no culling
    CullCam cc;
};
// Set-up of a batch of selection requests (frame records + clearing).
struct SelSetup {
    CamArgs cam;
    const double *T;
    const float *inst_scale;
    InstRec *itab;
    uint32_t *clear;
    uint32_t n_inst, n_clear;
};
// one request, ticket in req.counters[kSelTicket]
void launch_select(hipStream_t st, const SelReq &req);
// A batch of requests (device arrays setups[n_req], reqs[n_req]): one set-up
// launch, one persistent selection launch over all their partitions (claimed
// in ticket order from *batch_ticket), and one expansion launch.
void launch_select_batch(hipStream_t st, const SelSetup *setups, const SelReq *reqs, uint32_t n_req,
                         uint32_t total_parts, uint32_t max_inst, uint32_t max_clear, uint32_t *batch_ticket);
void launch_expand(hipStream_t st, const uint32_t *gid, const uint32_t *slot_off, const uint2 *rowinfo,
                   uint32_t n_clusters, const uint32_t *counters, uint32_t max_clusters, uint32_t *slot_row,
                   uint32_t *slot_inst);
// project.hip
struct ProjectOut {
    float4 *splat;      // 3 float4 per slot: (mx,my,A,B) (C,o,r,g) (b,depth,hx,hy)
    float *depth;       // FP32 depth of every slot
    BinRec *bin;        // binning record of visible slots
    uint32_t *tiles;    // tiles the support reaches (0 = culled)
    uint32_t *dkey;     // depth sort key: FP32 depth bits, 0xffffffff when culled
    uint32_t *dval;     // slot index (sort payload)
    uint32_t *counters; // render counters (kRenFp64, kRenConicClamp)
};
// Largest conic entry stored for blending: the conic is scaled by -log2(e)
// when staged, which must stay finite.
constexpr float kConicMax = 1.0e38f;
void launch_project(hipStream_t st, const FrameDev *fd, const Attribs &attr, int precision, int sh_degree,
                    const uint32_t *slot_row, const uint32_t *slot_inst, const uint32_t *n_slots_dev,
                    uint64_t max_slots, const InstRec *itab, ProjectOut out);
// sort.hip
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanPart = kScanThreads * kScanItems;
// exclusive scan of tiles[order[j]] (order may be NULL: identity); the total
// goes to kRenKeysLo/Hi and to kRenKeysEff when it is at most key_cap (else
// kRenKeysEff = 0 and kErrKeyCap is raised: the frame's later steps then
// have no keys to work on).  n_culled (may be NULL): the number of ranks at
// the end that hold culled slots (depth order puts them last), which are
// not scanned; their offsets are not written.
void launch_scan_tiles(hipStream_t st, const uint32_t *tiles, const uint32_t *order, const uint32_t *n_dev,
                       const uint32_t *n_culled, uint64_t max_n, uint32_t *offsets, uint64_t *status,
                       uint32_t *counters, uint64_t key_cap);
constexpr int kRadixBits = 8;
constexpr int kRadix = 256;
// Digits of a radix sort: pass p orders the keys by bits [shift[p], shift[p]
// + bits[p]) (bits[p] <= kRadixBits); digit histograms are kept kRadix apart.
struct DigitPlan {
    int passes = 0;
    uint32_t shift[4] = {0u, 0u, 0u, 0u}, bits[4] = {0u, 0u, 0u, 0u};
};
// key_bits significant bits in the fewest passes of at most kRadixBits bits,
// split as evenly as possible (11-bit bin ids: 6 + 5): narrower digits rank
// with fewer ballots and look back over fewer counts.
inline DigitPlan even_digits(uint32_t key_bits)
{
    DigitPlan d;
    d.passes = (int)((key_bits + kRadixBits - 1) / kRadixBits);
    uint32_t s = 0;
    for (int p = 0; p < d.passes; ++p) {
        const uint32_t left = key_bits - s, rest = (uint32_t)(d.passes - p);
        d.bits[p] = (left + rest - 1) / rest;
        d.shift[p] = s;
        s += d.bits[p];
    }
    return d;
}
// 64-bit keys (bin << 32 | depth bits), slot order
void launch_emit64(hipStream_t st, const uint32_t *n_dev, uint64_t max_n, const uint32_t *tiles,
                   const uint32_t *offsets, const BinRec *bin, const FrameDev *fd, uint64_t key_cap, uint64_t *keys,
                   uint32_t *vals, uint32_t *err);
// Bin-id keys in depth order (order[j] = slot of depth rank j), with the
// digit histograms of the bin sort (digits dp, passes <= 3) accumulated into hist.
// KT = uint16_t for grids of at most kBinKey16Max bins, else uint32_t.
constexpr uint32_t kBinKey16Max = 1u << 16;
// (splats of more than 2048 keys are listed in big[] (n_big: a cleared
// counter; big: max_n entries) and emitted by one workgroup each).  Rank j
// has offsets[j + 1] - offsets[j] keys; scan_ctr (the render counters the
// scan filled) gives the visible ranks, scan_ctr[kRenVisible] (culled slots
// sort last), and the key total, scan_ctr[kRenKeysLo], where the last visible
// rank's keys end.
template <typename KT>
void launch_emit32(hipStream_t st, const uint32_t *n_dev, uint64_t max_n, const uint32_t *order,
                   const uint32_t *tiles, const uint32_t *offsets, const uint32_t *scan_ctr, const BinRec *bin,
                   const FrameDev *fd, uint64_t key_cap, const DigitPlan &dp, KT *keys, uint32_t *vals, uint32_t *hist,
                   uint32_t *big, uint32_t *n_big, uint32_t *err);
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;          // keys per thread
constexpr int kSortPart = kSortThreads * kSortItems;  // partition (also the unit of look-back capacity)
constexpr int kSortItemsWide = 24;      // keys per thread of wide partitions
constexpr int kSortPartWide = kSortThreads * kSortItemsWide;
static_assert(kSortPartWide >= kSortPart, "look-back status is sized for partitions of kSortPart keys");
constexpr uint64_t kSortWideFrom = 1u << 22;  // sorts of at least this many keys use wide partitions
constexpr uint64_t kSortMaxGrid = 4096;       // workgroups of a pass (they claim partitions until none is left)
// Digit histograms of all passes; the key count is n_dev ? *n_dev : n.
template <typename K>
// dropped: when given, keys of all ones are not counted in the digit
// histograms but in *dropped instead (a sort whose first pass drops them).
void launch_sort_hist(hipStream_t st, const K *keys, const uint32_t *n_dev, uint64_t n, int passes, uint32_t *hist,
                      uint32_t *dropped = nullptr);
// One onesweep pass over n_dev ? *n_dev : n keys (grid sized for n); the
// look-back epoch is *epoch_dev + epoch when epoch_dev is given, else epoch.
// wide selects partitions of kSortPartWide keys (keys of at most 32 bits).
template <typename K>
// The pass's digit is bits [shift, shift + dbits) of the key (shift < 0:
// the pass-th 8-bit digit); its histogram is hist + pass * kRadix.
void launch_sort_pass(hipStream_t st, const K *keys_in, const uint32_t *vals_in, K *keys_out, uint32_t *vals_out,
                      const uint32_t *n_dev, uint64_t n, int pass, const uint32_t *hist, uint64_t *status,
                      const uint32_t *epoch_dev, uint32_t epoch, uint32_t *ticket, uint32_t *err, bool wide,
                      int shift = -1, int dbits = kRadixBits, const uint32_t *dropped = nullptr,
                      uint32_t *n_kept = nullptr);
// (dropped, 32-bit keys only: the pass leaves out the keys of all ones, which
// the histogram counted in *dropped instead of their digits, writes the
// others, and stores their count in *n_kept for the passes after it.)
// Per tile t < n_tiles (tiles_x per row): ranges[t] = [first, end) of the
// keys of its bin (bins_x per row) in the sorted keys, and the blend plan.  A
// tile whose bin holds L > cp.first() keys gets cp.n_chunks(L) consecutive
// chunk records from cbase[t] (kNoChunk for other tiles, and for long ones
// beyond max_chunks records, which are then blended whole) and one work item
// (t, c) per chunk c >= 1 (items: counters[kRenItems]).  order is a
// permutation of the tiles with the lists of at least cp.first() keys first,
// so that the longest walks start first.
// With rec (a record in mapped pinned host memory), the kernel also publishes
// the frame's counts there, tagged seq: keys, visible slots and error flags
// from counters, slots and clusters from the selection's sel_counters.
template <typename K>
void launch_tile_ranges(hipStream_t st, const K *keys, const uint32_t *n_dev, int shift, uint32_t tiles_x,
                        uint32_t n_tiles, uint32_t bins_x, uint2 *ranges, uint32_t *cbase, uint2 *items,
                        uint32_t *rounds, uint32_t rcap, uint32_t *order, uint32_t *counters, uint64_t max_chunks,
                        const ChunkPlan &cp, const uint32_t *sel_counters = nullptr, struct FrameRec *rec = nullptr,
                        uint32_t seq = 0);
// blend.hip
constexpr uint32_t kPairSlots = 256;  // spread pair counters (see count_pairs)
// max_items / max_chunks bound the work items and chunks of the plan (grid
// sizes).  rounds (kChunkRounds lists of rcap tiles) and items hold the work
// items as the range kernel lists them; stopm holds 4 words per chunk record
// (the later chunks' stopped pixels), zero on entry and left zero.  pairs (2 kPairSlots counters): with count >= 1 its even entries
// sum the pairs walked, with count 2 its odd entries also sum the pairs taken
// (alpha >= 1/255 at an active pixel); counting slows the walk.  cp: the
// chunk sizes the range kernel planned with.
void launch_blend(hipStream_t st, const FrameDev *fd, uint32_t tiles_x, uint32_t tiles_y, const float4 *splat,
                  const uint32_t *vals, const uint2 *ranges, const uint32_t *cbase, const uint2 *items,
                  const uint32_t *rounds, uint32_t rcap, const uint32_t *order, uint32_t *counters, uint64_t max_items,
                  uint64_t max_chunks, float4 *scratch, uint32_t *pend, uint32_t *need, uint64_t *stopm, uint2 *rewalk,
                  unsigned long long *pairs, int count, ChunkPlan cp);
// Frames whose keys exceeded the key buffers (kErrKeyCap): every tile walks
// the n = counters[kRenVisible] visible slots in depth order (order: the
// depth-sorted slots) and writes its pixels; other frames return at once.
void launch_blend_all(hipStream_t st, const FrameDev *fd, uint32_t n_tiles, const float4 *splat,
                      const uint32_t *order, const uint32_t *counters, unsigned long long *pairs, int count);
// generic fill
void launch_fill_u32(hipStream_t st, uint32_t *p, uint64_t n, uint32_t v);

// build.hip (offline build)
constexpr double kScaleGrowth = 1.122462048309373;  // 2^(1/6): scale growth of a simplified Gaussian
constexpr double kNestSlack = 1.0 + 1.0 / 1024.0;   // parent radius over (distance + child radius)
// One layer of a median split of m items (item ids into pts, x y z per id):
// sets start at start[0..n_sets) and split where splits[s] != 0; writes
// keys (set << 32 | coordinate bits) and vals (items) for the stable sort.
void launch_split_layer(hipStream_t st, const float *pts, const uint32_t *items, uint32_t m, const uint32_t *start,
                        const uint8_t *splits, uint32_t n_sets, uint32_t *box, uint64_t *keys, uint32_t *vals);
// mean[k] = FP64 mean (row order) of the positions of cluster k's rows
// rows[first[k] ..], in FP32; sph4 (optional) = (mean, 0)
void launch_cluster_mean(hipStream_t st, const float *pos, const uint32_t *rows, const uint32_t *first,
                         const uint32_t *count, uint32_t n, float *mean, float *sph4);
// Simplification of n_groups cluster groups into one cluster each: the
// group's rows (ids into the current row store) go to go_rows[g * 128 ..] and
// go_count[g], the kept ones to kept[g * cap ..], their number to out_count[g],
// the group sphere to sph[g], the sphere framing its pseudo-views to vsph[g]
void launch_group(hipStream_t st, const float *pos, const float *scale, const float *opacity, const uint32_t *rows,
                  const uint32_t *first, const uint32_t *count, const float *msph, const uint32_t *perm,
                  const uint32_t *gfirst, const uint32_t *gsize, uint32_t n_groups, uint32_t cap, uint32_t *kept,
                  uint32_t *out_count, float *sph, float *vsph, uint32_t *go_rows, uint32_t *go_count,
                  uint32_t *err);
// The next layer's row store from the kept rows (scales grown once); src
// (nullable: the row id itself) carries the input Gaussian of each row.
void launch_spawn(hipStream_t st, const float *pos, const float *scale, const float *rot, const float *opacity,
                  const float *sh, const uint32_t *src, uint32_t sh_floats, const uint32_t *kept,
                  const uint32_t *count, uint32_t n_groups, uint32_t cap, float *npos, float *nscale, float *nrot,
                  float *nopacity, float *nsh, uint32_t *nsrc, uint32_t *nrows);
// Local splatting of n_groups cluster groups: group g fits the fitted rows
// sfirst[g] .. + scount[g] (<= 64; position, scale, rotation, opacity, dc at
// sdc + stride * row) to its ocount[g] (<= 128) original rows, rows
// orows[ofirst[g] + k] (orows nullable: rows ofirst[g] + k), over views
// dirs[0 .. iters) around sphere[g]; losses (n_groups x iters) and
// grad_first (14 per fitted row) are optional.
void launch_local_splat(hipStream_t st, const uint32_t *ofirst, const uint32_t *ocount, const uint32_t *sfirst,
                        const uint32_t *scount, const float *sphere, const float *opos, const float *oscale,
                        const float *orot, const float *oopacity, const float *odc, uint32_t odc_stride,
                        const uint32_t *orows, float *spos, float *sscale, float *srot, float *sopacity, float *sdc,
                        uint32_t sdc_stride, const float *dirs, uint32_t iters, uint32_t n_groups, float *losses,
                        float *grad_first, uint32_t *err);
// bundle rows of one layer: output row i = row idx[i] of the layer's store
void launch_gather_rows(hipStream_t st, const float *pos, const float *scale, const float *rot, const float *opacity,
                        const float *sh, uint32_t sh_floats, const uint32_t *idx, uint32_t n_rows, float *opos,
                        float *oscale, float *orot, float *oopacity, float *osh);

// stream.hip (cluster streaming): scatter n_up staged page images (layout in
// stream.hip) into the pool planes and point rowinfo[cluster] at each page
void launch_stream_scatter(hipStream_t st, const uint8_t *staging, const uint4 *ups, uint32_t n_up,
                           uint32_t page_bytes, uint32_t geo_bytes, uint32_t sh_bytes, uint32_t n_sh,
                           float *pos_planes, void *geo_planes, void *sh_planes, uint64_t stride, uint2 *rowinfo);

}  // namespace v3dg
