// Front-to-back alpha compositing (paper Sec. 2.1: the splats covering a
// pixel are blended in depth order), one 256-thread workgroup per 16x16 tile.
//
// Each wavefront owns one 8x8 quarter of the tile, one pixel per lane.  A
// tile's depth-sorted splats are staged through LDS in batches of 256 (one
// gather per splat per tile); every wavefront compacts, in order, the batch
// entries whose enlarged support reaches a pixel centre of its quarter (an
// exact ellipse-rectangle test, per 8-row band) and walks only those.
//
// Per (pixel, splat), with d = mean - pixel centre and conic (A, B, C):
//   power = min(0, -1/2 (A dx^2 + C dy^2) - B dx dy),  alpha = min(0.99, o e^power);
//   alpha < 1/255 is skipped;  T' = T (1 - alpha);  T' < 1e-4 ends the pixel
//   without adding this splat;  otherwise C += alpha T rgb, T = T'.
// The quadratic is evaluated in base 2 (conic pre-scaled by log2 e) and the
// 1/255 test is taken on it before the exponential: alpha < 1/255 exactly when
// p < -log2(255 o) with p = log2(e) power.
// Output RGBA: C + T bg, 1 - T.
//
// Long lists.  A few tiles of a near view hold tens of thousands of splats and
// would keep one workgroup busy long after the rest of the frame is done.  A
// list longer than a first chunk is cut into the first chunk and further,
// shorter chunks (the frame's ChunkPlan: most pixels of opaque content stop
// within the first chunk, which leaves the later chunks nothing to do).  The
// tile-range kernel has given every long tile its chunk
// records and listed the work items (tile, chunk >= 1); then
//   blend_kernel  walks chunk 0 of every tile (with the stop rule);
//   chunk_kernel  walks every other chunk in parallel, each from T = 1,
//                 giving per pixel the chunk's colour C_c and transmittance T_c;
//                 a chunk drops the pixels that an earlier chunk of the tile
//                 has already stopped on its own (see ChunkSkip);
//   fold_kernel   folds the chunks in order, C += T C_c, T *= T_c.  Running
//                 transmittance only decreases, so the stopping splat lies in
//                 the first chunk with T T_c < 1e-4 (or that stopped on its own
//                 from T = 1); pixels without one are finished here;
//   rewalk_kernel walks each such chunk again, in parallel over (tile, chunk),
//                 from the folded (T, C) with the stop rule; later chunks are
//                 ignored.
// This is the sequential result up to the association of the FP32 products.
#include "v3dg_internal.h"

namespace v3dg {

constexpr int kBlendThreads = kTile * kTile;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

struct BlendShared {
    float4 P0[kBlendThreads];  // (mx, my, a, b): p = a dx^2 + b dx dy + c dy^2
    float4 P1[kBlendThreads];  // (c, log2 threshold, log2 o, -)
    float4 P2[kBlendThreads];  // (r, g, b, -)
    uint8_t mask[kBlendThreads];
    uint32_t alive;  // byte w: wavefront w has an active pixel
    // per wavefront, its entries in order as byte offsets into P0 / P1 / P2;
    // + one pair read ahead past the last entry
    uint16_t idx[4][kBlendThreads + 2];
};

struct Pix {
    float T, cr, cg, cb;
    bool active;          // still compositing
    uint32_t walked;      // (pixel, splat) pairs walked by the wavefront's active pixels (uniform)
    uint32_t taken;       // of those, pairs with alpha >= 1/255 (composited, or ending the pixel) (uniform)
};

// Pixels that the chunks of a long tile stopped on their own.  When chunk c'
// walked from T = 1 stops pixel p, the sequential walk, which reaches c' with
// T <= 1 and multiplies by the same factors, stops p at or before the same
// splat, so the fold ends p's walk at a chunk <= c' and never reads p's
// summary of a later chunk: a later chunk may drop p, at its start or between
// batches.  Each chunk wavefront publishes the mask of its pixels stopped (or
// dropped) so far in word 4 (record) + wavefront; the fold clears the words
// of the records it has read, so every word is zero when a frame's chunks
// start (the buffer is cleared when it is allocated).  Words are read and written as
// device-scope atomics and no one waits on them: a mask read early only drops
// fewer pixels.
struct ChunkSkip {
    uint64_t *stopm = nullptr;
    uint64_t base = 0;  // the tile's first chunk record
    uint32_t c = 0;     // this chunk
};

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, o, kWave);
        hi |= (uint32_t)__shfl_xor((int)hi, o, kWave);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Stage one batch entry (the splat record of key i) into LDS with its
// quarter mask: bit q when the enlarged support {d : d' S^-1 d <= Qm} (S the
// 2D covariance, Qm = 1.05 Q + 0.05 with alpha >= 1/255 exactly when
// d' S^-1 d <= Q = 2 ln(255 o), enlarged like the binning) reaches a pixel
// centre of quarter q.  Per 8-row band of the tile (offsets [ya, ya + 7] from
// the mean) the support spans x in [k y - w(y), k y + w(y)] with k = Sxy /
// Syy = -B / A and w(y) = sqrt(Qm (1 - y^2 / (Qm Syy)) / A) (A, B the conic's
// entries: Syy / det S = A); its right end peaks at y_r = k Qm Syy /
// sqrt(Qm Sxx) and its left end at -y_r, so the band's x-range comes from
// those points clamped into the band.  A quarter is kept when that range
// meets its pixel centres: exact for the rectangle of centres, with no
// cancellation (no determinant is formed), and a NaN keeps the quarter.
__device__ __forceinline__ void stage_entry(BlendShared &sh, int tid, bool valid, const float4 &f0, const float4 &f1,
                                            const float4 &f2, float bx0, float by0)
{
    uint32_t m = 0;
    if (valid) {
        const float lo = __log2f(f1.y);
        const float l255o = __log2f(255.0f) + lo;
        sh.P0[tid] = make_float4(f0.x, f0.y, -0.5f * kLog2e * f0.z, -kLog2e * f0.w);
        sh.P1[tid] = make_float4(-0.5f * kLog2e * f1.x, -l255o, lo, 0.f);
        sh.P2[tid] = make_float4(f1.z, f1.w, f2.x, 0.f);
        // f2.z, f2.w = sqrt(Qm Sxx), sqrt(Qm Syy) from the projection
        const float Qm = 1.05f * (2.0f * kLn2 * l255o) + 0.05f;
        const float k = -f0.w / f0.z, qa = Qm / f0.z, ymax = f2.w, iym = 1.0f / f2.w;
        const float yr = k * (f2.w * f2.w / f2.z);
        const float X0 = bx0 - f0.x, Y0 = by0 - f0.y;
#pragma unroll
        for (int band = 0; band < 2; ++band) {
            const float ylo = fmaxf(Y0 + 8.0f * (float)band, -ymax), yhi = fminf(Y0 + 8.0f * (float)band + 7.0f, ymax);
            const float dr = fminf(fmaxf(yr, ylo), yhi), dl = fminf(fmaxf(-yr, ylo), yhi);
            const float ur = dr * iym, ul = dl * iym;
            const float xr = fmaf(k, dr, sqrtf(fmaxf(0.0f, (1.0f - ur * ur) * qa)));
            const float xl = fmaf(k, dl, -sqrtf(fmaxf(0.0f, (1.0f - ul * ul) * qa)));
            const bool in_band = !(ylo > yhi);
#pragma unroll
            for (int qx = 0; qx < 2; ++qx) {
                const float xa = X0 + 8.0f * (float)qx;
                m |= (uint32_t)(in_band && !(xl > xa + 7.0f) && !(xr < xa)) << (2 * band + qx);
            }
        }
    }
    sh.mask[tid] = (uint8_t)m;
}

// Orders this wavefront's LDS stores before its later loads (other lanes').
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Record of a staged entry by its byte offset (entry number x 16).
__device__ __forceinline__ float4 rec(const float4 *base, uint32_t off)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// One splat against the lane's pixel, branch-free.  p is its base-2
// quadratic form, log2o = log2 of its opacity, col its colour; take says the
// pixel is active and the splat passes the 1/255 test.  A stopped pixel
// carries its final transmittance negated, so "active" is T > 0 and needs no
// flag of its own.
__device__ __forceinline__ void composite(float p, bool take, float log2o, const float4 &col, float &T, float &cr,
                                          float &cg, float &cb)
{
    // the exponent lies in [log2(1/255), 0]: the hardware exp2 is exact enough
    // min(p, 0) as one integer min on the bit pattern (a negative float is a
    // negative integer, -0 gives the same exponent as 0; a NaN p is never taken)
    const float ex = __builtin_amdgcn_exp2f(__int_as_float(min(__float_as_int(p), 0)) + log2o);
    const float alpha = take ? fminf(0.99f, ex) : 0.0f;
    const float Tn = fmaf(-alpha, T, T);
    // a pixel that does not take the splat keeps Tn = T: >= 1e-4 while
    // active, negative once stopped
    const bool keep = Tn >= 1e-4f;
    const float w = keep ? alpha * T : 0.0f;
    cr = fmaf(w, col.x, cr);
    cg = fmaf(w, col.y, cg);
    cb = fmaf(w, col.z, cb);
    T = keep ? Tn : -fabsf(T);
}

// Composite keys [b, e) of the tile into the lanes' pixels (every thread of
// the workgroup calls this with the same range).  The first batch is loaded
// once a pixel is known to be active; after that the splat records of the
// next batch are gathered while the current one is walked, and the index of
// the batch after that one is read ahead, so no walk waits on global memory.
// kCount 1 counts the pairs walked, 2 also the pairs taken (a few scalar
// operations per pair on the walk's critical path, so only when the profile
// asks for them; 0 counts nothing).  kSkip: a later chunk of a long tile,
// which drops and publishes pixels as ChunkSkip describes.
template <int kCount, bool kSkip>
__device__ void blend_range(uint32_t b, uint32_t e, const float4 *__restrict__ splat,
                            const uint32_t *__restrict__ vals, float bx0, float by0, float pxc, float pyc, int wid,
                            int lane, BlendShared &sh, Pix &px, const ChunkSkip &sk)
{
    const int tid = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0, f2 = f0;
    uint32_t vnext = 0;
    const uint64_t was = __ballot(px.active);
    uint64_t published = 0;
    for (uint32_t start = b; start < e; start += kBlendThreads) {
        if constexpr (kSkip) {
            if (sk.c > 1u && (was & ~published) != 0) {  // uniform
                uint64_t dead = 0;
                for (uint32_t j = 1u + (uint32_t)lane; j < sk.c; j += kWave)
                    dead |= __hip_atomic_load(sk.stopm + (sk.base + j) * 4u + (uint32_t)wid, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                dead = wave_or64(dead);
                if ((dead >> lane) & 1ull) px.active = false;
            }
        }
        // each wavefront notes whether it has an active pixel; the barrier also
        // ends every walk of the previous batch before its records are replaced
        const bool alive = __ballot(px.active) != 0;
        if (lane == 0) reinterpret_cast<uint8_t *>(&sh.alive)[wid] = alive ? 1u : 0u;
        __syncthreads();
        if (sh.alive == 0u) break;
        if (start == b) {
            // the first batch is loaded only once a pixel is known to be active:
            // a later chunk of a tile that its first chunk finished loads nothing
            if (b + tid < e) {
                const float4 *sp = splat + 3 * (uint64_t)vals[b + tid];
                f0 = sp[0];
                f1 = sp[1];
                f2 = sp[2];
            }
            vnext = (b + kBlendThreads + tid < e) ? vals[b + kBlendThreads + tid] : 0u;
        }
        stage_entry(sh, tid, start + tid < e, f0, f1, f2, bx0, by0);
        __syncthreads();
        // read ahead: records of the next batch, index of the one after
        {
            const uint32_t i1 = start + kBlendThreads + tid, i2 = i1 + kBlendThreads;
            if (i1 < e) {
                const float4 *sp = splat + 3 * (uint64_t)vnext;
                f0 = sp[0];
                f1 = sp[1];
                f2 = sp[2];
            }
            vnext = i2 < e ? vals[i2] : 0u;
        }
        // in-order compaction of this quarter's entries
        uint32_t cnt = 0;
#pragma unroll
        for (int c = 0; c < kBlendThreads / kWave; ++c) {
            const bool hit = (sh.mask[c * kWave + lane] >> wid) & 1u;
            const uint64_t bal = __ballot(hit);
            if (hit) sh.idx[wid][cnt + (uint32_t)__popcll(bal & lt)] = (uint16_t)((c * kWave + lane) * sizeof(float4));
            cnt += (uint32_t)__popcll(bal);
        }
        // The entry list is this wavefront's own and the LDS operations of a
        // wavefront complete in order: the walk needs no workgroup barrier,
        // only the compiler must keep the list's stores before its loads.
        wave_sync();
        // an odd last entry is paired with itself (never taken twice), so every
        // record read belongs to this batch
        if ((cnt & 1u) && lane == 0) sh.idx[wid][cnt] = sh.idx[wid][cnt - 1];
        wave_sync();
        uint64_t am = __ballot(px.active);  // active pixels (uniform)
        if (am) {
            // The walk is uniform across the wavefront: entries k, k+1 are the
            // same for every lane; lanes differ only in whether they take them.
            // An entry counts as walked for the pixels active when it is reached.
            float T = px.active ? px.T : -px.T, cr = px.cr, cg = px.cg, cb = px.cb;
            uint32_t walked = 0, taken = 0;
            uint32_t prn = *reinterpret_cast<const uint32_t *>(&sh.idx[wid][0]);
            for (uint32_t k = 0; am != 0 && k < cnt; k += 2) {
                // the next pair's offsets are read one iteration ahead (past the
                // last entry they are stale values of the row and never used)
                const uint32_t pr = prn;
                prn = *reinterpret_cast<const uint32_t *>(&sh.idx[wid][k + 2]);
                const bool two = k + 1 < cnt;
                const uint32_t o0 = pr & 0xffffu, o1 = pr >> 16;
                const float4 a0 = rec(sh.P0, o0), a1 = rec(sh.P0, o1);
                const float4 c0 = rec(sh.P1, o0), c1 = rec(sh.P1, o1);
                const float dx0 = a0.x - pxc, dy0 = a0.y - pyc;
                const float dx1 = a1.x - pxc, dy1 = a1.y - pyc;
                // p = (a dx + b dy) dx + c dy^2
                const float p0 = fmaf(fmaf(a0.z, dx0, a0.w * dy0), dx0, c0.x * dy0 * dy0);
                const float p1 = fmaf(fmaf(a1.z, dx1, a1.w * dy1), dx1, c1.x * dy1 * dy1);
                // alpha >= 1/255; a NaN quadratic form (0 times a clamped conic
                // entry of a needle thinner than FP32 resolves) is not taken
                const bool pass0 = p0 >= c0.y, pass1 = two && p1 >= c1.y;
                uint64_t amid = am;  // active after entry k
                if (__ballot(T > 0.0f && (pass0 || pass1)) != 0) {
                    const float4 col0 = rec(sh.P2, o0), col1 = rec(sh.P2, o1);
                    composite(p0, T > 0.0f && pass0, c0.z, col0, T, cr, cg, cb);
                    const bool act1 = T > 0.0f;
                    amid = __ballot(act1);
                    composite(p1, act1 && pass1, c1.z, col1, T, cr, cg, cb);
                }
                if constexpr (kCount >= 1) walked += (uint32_t)__popcll(am) + (two ? (uint32_t)__popcll(amid) : 0u);
                // the pass masks are the compares' own lane masks: counted on the scalar unit
                if constexpr (kCount >= 2)
                    taken += (uint32_t)__popcll(am & __ballot(pass0)) + (uint32_t)__popcll(amid & __ballot(pass1));
                am = __ballot(T > 0.0f);
            }
            px.walked += walked;
            px.taken += taken;
            px.active = T > 0.0f;
            px.T = fabsf(T);
            px.cr = cr;
            px.cg = cg;
            px.cb = cb;
        }
        if constexpr (kSkip) {
            const uint64_t stopped = was & ~__ballot(px.active);
            if (stopped != published) {  // uniform
                if (lane == 0)
                    __hip_atomic_store(sk.stopm + (sk.base + sk.c) * 4u + (uint32_t)wid, stopped, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                published = stopped;
            }
        }
    }
}

// pairs[2 s]: walked pairs; pairs[2 s + 1]: taken pairs, for s < kPairSlots.
// Wavefronts add to slots spread by workgroup and wavefront: a single
// counter taking every wavefront's add made the blend stage 6 % slower.
__device__ __forceinline__ void count_pairs(const Pix &px, int wid, int lane, unsigned long long *pairs)
{
    const uint32_t slot = (blockIdx.x * (kBlendThreads / kWave) + (uint32_t)wid) % kPairSlots;
    if (lane == 0 && px.walked) atomicAdd(pairs + 2 * slot, (unsigned long long)px.walked);
    if (lane == 0 && px.taken) atomicAdd(pairs + 2 * slot + 1, (unsigned long long)px.taken);
}

struct TileGeo {
    uint32_t x, y, pix;   // pixel, and its index within the tile
    bool inside;
    float pxc, pyc, bx0, by0;
};

__device__ __forceinline__ TileGeo tile_geo(const CamArgs &cam, uint32_t tile, int wid, int lane)
{
    TileGeo g;
    const uint32_t tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const uint32_t col = ((uint32_t)wid & 1u) * 8u + ((uint32_t)lane & 7u);
    const uint32_t row = ((uint32_t)wid >> 1) * 8u + ((uint32_t)lane >> 3);
    g.x = tx * kTile + col;
    g.y = ty * kTile + row;
    g.pix = row * kTile + col;
    g.inside = g.x < cam.width && g.y < cam.height;
    g.pxc = (float)g.x + 0.5f;
    g.pyc = (float)g.y + 0.5f;
    g.bx0 = (float)(tx * kTile) + 0.5f;
    g.by0 = (float)(ty * kTile) + 0.5f;
    return g;
}

__device__ __forceinline__ void write_pixel(const CamArgs &cam, const TileGeo &g, const Pix &px, float4 *image)
{
    if (g.inside)
        image[(uint64_t)g.y * cam.width + g.x] =
            make_float4(px.cr + px.T * cam.bg[0], px.cg + px.T * cam.bg[1], px.cb + px.T * cam.bg[2], 1.0f - px.T);
}

// ---------------------------------------------------------------------------
// pass 1: every tile, up to the end of its first chunk
// ---------------------------------------------------------------------------
// Workgroup b blends tile order[b]: the tiles with the longest first chunks
// come first, so that their walks do not start last and leave the rest of the
// chip idle.
template <int kCount>
__global__ void __launch_bounds__(kBlendThreads) blend_kernel(const FrameDev *__restrict__ fd,
                                                              const float4 *__restrict__ splat,
                                                              const uint32_t *__restrict__ vals,
                                                              const uint2 *__restrict__ ranges,
                                                              const uint32_t *__restrict__ cbase,
                                                              const uint32_t *__restrict__ order,
                                                              float4 *__restrict__ scratch,
                                                              uint32_t *__restrict__ need,
                                                              unsigned long long *__restrict__ pairs, ChunkPlan cp)
{
    __shared__ BlendShared sh;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const CamArgs &cam = fd->cam;
    float4 *image = reinterpret_cast<float4 *>(fd->image);
    const uint32_t tile = order[blockIdx.x];
    const TileGeo g = tile_geo(cam, tile, wid, lane);
    const uint2 rg = ranges[tile];
    Pix px{1.0f, 0.f, 0.f, 0.f, g.inside, 0u, 0u};
    const uint32_t end = rg.y > rg.x ? rg.y : rg.x;
    const uint32_t cb = cbase[tile];  // kNoChunk: blended whole
    const bool long_list = cb != kNoChunk && end - rg.x > cp.first();
    blend_range<kCount, false>(rg.x, long_list ? rg.x + cp.first() : end, splat, vals, g.bx0, g.by0, g.pxc, g.pyc, wid,
                               lane, sh, px, ChunkSkip{});
    if (long_list) {  // state after chunk 0; a negative T marks a finished pixel
        scratch[(uint64_t)cb * kBlendThreads + g.pix] =
            make_float4(px.cr, px.cg, px.cb, px.active ? px.T : -px.T);
        // need[] of chunk 0 (cleared by the fold) notes, one byte per
        // wavefront, whether a pixel is still active: the later chunks of a
        // finished tile do nothing
        const bool any = __ballot(px.active) != 0;
        if (lane == 0) reinterpret_cast<uint8_t *>(need + cb)[wid] = any ? 1u : 0u;
    } else {
        write_pixel(cam, g, px, image);
    }
    count_pairs(px, wid, lane, pairs);
}

// ---------------------------------------------------------------------------
// pass 2: chunks 1.. of long tiles, in parallel, each from T = 1
// ---------------------------------------------------------------------------
// Workgroup i takes work item i, counting first through the rounds (round r:
// chunk r of every long tile with one), then through the items of the chunks
// past the rounds.  Workgroups start in index order, so a later chunk starts
// after the earlier chunks of its tile and finds more of its pixels stopped
// by them (ChunkSkip).
template <int kCount>
__global__ void __launch_bounds__(kBlendThreads) __attribute__((amdgpu_waves_per_eu(7, 7))) chunk_kernel(const FrameDev *__restrict__ fd,
                                                              const float4 *__restrict__ splat,
                                                              const uint32_t *__restrict__ vals,
                                                              const uint2 *__restrict__ ranges,
                                                              const uint32_t *__restrict__ cbase,
                                                              const uint2 *__restrict__ items,
                                                              const uint32_t *__restrict__ rounds, uint32_t rcap,
                                                              const uint32_t *__restrict__ counters,
                                                              float4 *__restrict__ scratch,
                                                              const uint32_t *__restrict__ need,
                                                              uint64_t *__restrict__ stopm,
                                                              unsigned long long *__restrict__ pairs, ChunkPlan cp)
{
    static_assert(kChunkRounds == kWave, "one wavefront scans the round sizes");
    __shared__ BlendShared sh;
    __shared__ uint32_t pre[kChunkRounds];  // inclusive prefix sums of the round sizes
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const CamArgs &cam = fd->cam;
    if (wid == 0) {
        uint32_t v = counters[kRenRound + lane];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t n = (uint32_t)__shfl_up((int)v, o, kWave);
            if (lane >= o) v += n;
        }
        pre[lane] = v;
    }
    __syncthreads();
    const uint32_t in_rounds = pre[kChunkRounds - 1], n_items = in_rounds + counters[kRenItems];
    for (uint32_t t = blockIdx.x; t < n_items; t += gridDim.x) {
        uint32_t tile, c;
        if (t < in_rounds) {
            uint32_t r = 0;  // rounds whose prefix is <= t: t lies in round r + 1
#pragma unroll
            for (uint32_t st = kChunkRounds / 2; st > 0; st >>= 1)
                if (pre[r + st - 1] <= t) r += st;
            tile = rounds[(uint64_t)r * rcap + (t - (r ? pre[r - 1] : 0u))];
            c = r + 1u;
        } else {
            const uint2 item = items[t - in_rounds];
            tile = item.x;
            c = item.y;
        }
        const uint64_t base = cbase[tile];
        if (need[base] != 0u) {  // else every pixel finished in chunk 0 (uniform)
            const TileGeo g = tile_geo(cam, tile, wid, lane);
            const uint2 rg = ranges[tile];
            const float4 s0 = scratch[base * kBlendThreads + g.pix];
            Pix px{1.0f, 0.f, 0.f, 0.f, s0.w > 0.0f, 0u, 0u};
            const bool was = px.active;
            ChunkSkip sk;
            sk.stopm = stopm;
            sk.base = base;
            sk.c = c;
            blend_range<kCount, true>(rg.x + cp.begin(c), rg.x + cp.end(c, rg.y - rg.x), splat, vals, g.bx0, g.by0,
                                      g.pxc, g.pyc, wid, lane, sh, px, sk);
            // the fold reads later chunks only for pixels active after chunk 0 (a
            // dropped pixel's summary is never read)
            if (was)
                scratch[(base + c) * kBlendThreads + g.pix] =
                    make_float4(px.cr, px.cg, px.cb, !px.active ? -px.T : px.T);
            count_pairs(px, wid, lane, pairs);
        }
        __syncthreads();  // the next item reuses the staged batch
    }
}

// ---------------------------------------------------------------------------
// pass 3: fold the chunk summaries of long tiles; list the chunks to walk again
// ---------------------------------------------------------------------------
constexpr uint32_t kNone = 0xffffffffu;

__global__ void __launch_bounds__(kBlendThreads) fold_kernel(const FrameDev *__restrict__ fd,
                                                             const uint2 *__restrict__ ranges,
                                                             const uint32_t *__restrict__ cbase,
                                                             float4 *__restrict__ scratch, uint32_t *__restrict__ pend,
                                                             uint32_t *__restrict__ need, uint64_t *__restrict__ stopm,
                                                             uint2 *__restrict__ rewalk, uint32_t *counters,
                                                             ChunkPlan cp)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const CamArgs &cam = fd->cam;
    const uint32_t tile = blockIdx.x;
    float4 *image = reinterpret_cast<float4 *>(fd->image);
    const uint2 rg = ranges[tile];
    const uint32_t L = rg.y > rg.x ? rg.y - rg.x : 0u;
    if (L <= cp.first() || cbase[tile] == kNoChunk) return;
    const uint32_t m = cp.n_chunks(L);
    const TileGeo g = tile_geo(cam, tile, wid, lane);
    const uint64_t base = cbase[tile];
    for (uint32_t c = tid; c < m; c += kBlendThreads) need[base + c] = 0u;
    // the chunks of this frame are done: clear their stopped-pixel words for
    // the frames after it (every record a chunk can write was assigned to a
    // long tile, and every long tile is folded)
    for (uint32_t w = tid; w < 4u * m; w += kBlendThreads) stopm[4u * base + w] = 0ull;
    __syncthreads();
    const float4 s0 = scratch[base * kBlendThreads + g.pix];
    Pix px{fabsf(s0.w), s0.x, s0.y, s0.z, false, 0u, 0u};
    uint32_t pending = kNone;
    if (s0.w > 0.0f) {
        // four summaries loaded at a time (those past the stop are never used)
        constexpr uint32_t kAhead = 4;
        for (uint32_t c0 = 1; c0 < m && pending == kNone; c0 += kAhead) {
            float4 sc[kAhead];
#pragma unroll
            for (uint32_t k = 0; k < kAhead; ++k)
                sc[k] = c0 + k < m ? scratch[(base + c0 + k) * kBlendThreads + g.pix] : make_float4(0.f, 0.f, 0.f, 1.f);
#pragma unroll
            for (uint32_t k = 0; k < kAhead; ++k) {
                if (pending != kNone || c0 + k >= m) break;
                if (sc[k].w < 0.0f || px.T * sc[k].w < 1e-4f) {
                    pending = c0 + k;
                    break;
                }
                px.cr = fmaf(px.T, sc[k].x, px.cr);
                px.cg = fmaf(px.T, sc[k].y, px.cg);
                px.cb = fmaf(px.T, sc[k].z, px.cb);
                px.T *= sc[k].w;
            }
        }
    }
    if (pending == kNone) {
        write_pixel(cam, g, px, image);
    } else {
        // the folded state goes where chunk 0's was; the chunk to walk again is noted
        scratch[base * kBlendThreads + g.pix] = make_float4(px.cr, px.cg, px.cb, px.T);
        need[base + pending] = 1u;
    }
    pend[base * kBlendThreads + g.pix] = pending;
    __syncthreads();
    for (uint32_t c = tid; c < m; c += kBlendThreads)
        if (need[base + c]) {
            const uint32_t slot = atomicAdd(&counters[kRenRewalk], 1u);
            rewalk[slot] = make_uint2(tile, c);
        }
}

// ---------------------------------------------------------------------------
// pass 4: walk again, with the stop rule, each chunk that holds a stop
// ---------------------------------------------------------------------------
template <int kCount>
__global__ void __launch_bounds__(kBlendThreads) rewalk_kernel(const FrameDev *__restrict__ fd,
                                                               const float4 *__restrict__ splat,
                                                               const uint32_t *__restrict__ vals,
                                                               const uint2 *__restrict__ ranges,
                                                               const uint32_t *__restrict__ cbase,
                                                               const float4 *__restrict__ scratch,
                                                               const uint32_t *__restrict__ pend,
                                                               const uint2 *__restrict__ rewalk,
                                                               const uint32_t *__restrict__ counters,
                                                               unsigned long long *__restrict__ pairs, ChunkPlan cp)
{
    __shared__ BlendShared sh;
    const uint32_t n_items = counters[kRenRewalk];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const CamArgs &cam = fd->cam;
    float4 *image = reinterpret_cast<float4 *>(fd->image);
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint2 item = rewalk[it];
        const uint32_t tile = item.x, c = item.y;
        const TileGeo g = tile_geo(cam, tile, wid, lane);
        const uint2 rg = ranges[tile];
        const uint64_t base = cbase[tile];
        const bool mine = pend[base * kBlendThreads + g.pix] == c;
        const float4 st = scratch[base * kBlendThreads + g.pix];
        Pix px{fabsf(st.w), st.x, st.y, st.z, mine, 0u, 0u};  // a pixel finished before holds -T
        blend_range<kCount, false>(rg.x + cp.begin(c), rg.x + cp.end(c, rg.y - rg.x), splat, vals, g.bx0, g.by0,
                                   g.pxc, g.pyc, wid, lane, sh, px, ChunkSkip{});
        // a pixel that, through rounding of the folded products, does not stop in
        // this chunk keeps T ~ 1e-4: the later chunks would change it by at most that
        if (mine) write_pixel(cam, g, px, image);
        count_pairs(px, wid, lane, pairs);
        __syncthreads();  // the next item reuses the staged batch
    }
}

// ---------------------------------------------------------------------------
// a frame whose keys exceeded its key buffers (kErrKeyCap; its sort and the
// passes above then had no keys and wrote the background): every tile walks
// all visible splats in depth order instead, and the quarter tests of the
// staging keep only those whose support can reach it.  The image is the
// sequential result, only slower to get.
// ---------------------------------------------------------------------------
template <int kCount>
__global__ void __launch_bounds__(kBlendThreads) blend_all_kernel(const FrameDev *__restrict__ fd,
                                                                  const float4 *__restrict__ splat,
                                                                  const uint32_t *__restrict__ order,
                                                                  const uint32_t *__restrict__ counters,
                                                                  unsigned long long *__restrict__ pairs)
{
    if (!(counters[kRenErr] & kErrKeyCap)) return;  // uniform: the frame had room for its keys
    __shared__ BlendShared sh;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const CamArgs &cam = fd->cam;
    float4 *image = reinterpret_cast<float4 *>(fd->image);
    const uint32_t n_vis = counters[kRenVisible];
    for (uint32_t tile = blockIdx.x; tile < cam.tiles_x * cam.tiles_y; tile += gridDim.x) {
        const TileGeo g = tile_geo(cam, tile, wid, lane);
        Pix px{1.0f, 0.f, 0.f, 0.f, g.inside, 0u, 0u};
        blend_range<kCount, false>(0, n_vis, splat, order, g.bx0, g.by0, g.pxc, g.pyc, wid, lane, sh, px, ChunkSkip{});
        write_pixel(cam, g, px, image);
        count_pairs(px, wid, lane, pairs);
        __syncthreads();  // the next tile reuses the staged batch
    }
}

// launched after every frame sized by capacity: a small grid, since it
// returns at once unless the frame's keys did not fit
void launch_blend_all(hipStream_t st, const FrameDev *fd, uint32_t n_tiles, const float4 *splat,
                      const uint32_t *order, const uint32_t *counters, unsigned long long *pairs, int count)
{
    const uint32_t grid = n_tiles < 256u ? n_tiles : 256u;
    if (count >= 2)
        hipLaunchKernelGGL(blend_all_kernel<2>, dim3(grid), dim3(kBlendThreads), 0, st, fd, splat, order, counters, pairs);
    else if (count == 1)
        hipLaunchKernelGGL(blend_all_kernel<1>, dim3(grid), dim3(kBlendThreads), 0, st, fd, splat, order, counters, pairs);
    else
        hipLaunchKernelGGL(blend_all_kernel<0>, dim3(grid), dim3(kBlendThreads), 0, st, fd, splat, order, counters, pairs);
}

template <int kCount>
static void launch_blend_t(hipStream_t st, const FrameDev *fd, uint32_t n_tiles, const float4 *splat,
                           const uint32_t *vals, const uint2 *ranges, const uint32_t *cbase, const uint2 *items,
                           const uint32_t *rounds, uint32_t rcap, const uint32_t *order, uint32_t *counters,
                           uint64_t max_items, uint64_t max_chunks, float4 *scratch, uint32_t *pend, uint32_t *need,
                           uint64_t *stopm, uint2 *rewalk, unsigned long long *pairs, ChunkPlan cp)
{
    // beyond kMaxGrid items workgroups loop over further ones: a capacity-sized
    // bound on the items (frames sized without a host wait) launches no more
    constexpr uint64_t kMaxGrid = 16384;
    hipLaunchKernelGGL(blend_kernel<kCount>, dim3(n_tiles), dim3(kBlendThreads), 0, st, fd, splat, vals, ranges, cbase,
                       order, scratch, need, pairs, cp);
    if (max_items > 0) {
        const uint32_t gi = (uint32_t)(max_items < kMaxGrid ? max_items : kMaxGrid);
        // few chunks hold a stop to walk again: 2048 workgroups loop over them
        // rather than one per chunk of the bound (mostly empty workgroups)
        constexpr uint64_t kRewalkGrid = 2048;
        const uint32_t gc = (uint32_t)(max_chunks < kRewalkGrid ? max_chunks : kRewalkGrid);
        hipLaunchKernelGGL(chunk_kernel<kCount>, dim3(gi), dim3(kBlendThreads), 0, st, fd, splat, vals, ranges, cbase,
                           items, rounds, rcap, counters, scratch, need, stopm, pairs, cp);
        hipLaunchKernelGGL(fold_kernel, dim3(n_tiles), dim3(kBlendThreads), 0, st, fd, ranges, cbase, scratch, pend,
                           need, stopm, rewalk, counters, cp);
        hipLaunchKernelGGL(rewalk_kernel<kCount>, dim3(gc), dim3(kBlendThreads), 0, st, fd, splat, vals, ranges, cbase,
                           scratch, pend, rewalk, counters, pairs, cp);
    }
}

// max_items / max_chunks bound the chunk work items and chunks (grids are
// capped and loop over the device-side counts)
void launch_blend(hipStream_t st, const FrameDev *fd, uint32_t tiles_x, uint32_t tiles_y, const float4 *splat,
                  const uint32_t *vals, const uint2 *ranges, const uint32_t *cbase, const uint2 *items,
                  const uint32_t *rounds, uint32_t rcap, const uint32_t *order, uint32_t *counters, uint64_t max_items,
                  uint64_t max_chunks, float4 *scratch, uint32_t *pend, uint32_t *need, uint64_t *stopm, uint2 *rewalk,
                  unsigned long long *pairs, int count, ChunkPlan cp)
{
    const uint32_t n_tiles = tiles_x * tiles_y;
    if (count >= 2)
        launch_blend_t<2>(st, fd, n_tiles, splat, vals, ranges, cbase, items, rounds, rcap, order, counters, max_items,
                          max_chunks, scratch, pend, need, stopm, rewalk, pairs, cp);
    else if (count == 1)
        launch_blend_t<1>(st, fd, n_tiles, splat, vals, ranges, cbase, items, rounds, rcap, order, counters, max_items,
                          max_chunks, scratch, pend, need, stopm, rewalk, pairs, cp);
    else
        launch_blend_t<0>(st, fd, n_tiles, splat, vals, ranges, cbase, items, rounds, rcap, order, counters, max_items,
                          max_chunks, scratch, pend, need, stopm, rewalk, pairs, cp);
}

}  // namespace v3dg
