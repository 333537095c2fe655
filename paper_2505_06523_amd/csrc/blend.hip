// (e) front-to-back alpha compositing (paper Sec. 2.1: the splats covering a
// pixel are blended in depth order), one 256-thread workgroup per 16x16 tile.
//
// Each wavefront owns one 8x8 quarter of the tile, one pixel per lane.  The
// tile's depth-sorted splats are staged through LDS in batches of 256 (one
// gather per splat per tile); every wavefront then compacts, in order, the
// batch entries whose enlarged support box reaches its quarter and walks only
// those.  A wavefront whose 64 pixels are saturated stops evaluating; the
// workgroup stops once all four are.
//
// Per (pixel, splat), with d = mean - pixel centre and conic (A, B, C):
//   power = min(0, -1/2 (A dx^2 + C dy^2) - B dx dy),  alpha = min(0.99, o e^power);
//   alpha < 1/255 is skipped;  T' = T (1 - alpha);  T' < 1e-4 ends the pixel
//   without adding this splat;  otherwise C += alpha T rgb, T = T'.
// The quadratic is evaluated in base 2 (conic pre-scaled by log2 e) and the
// 1/255 test is taken on it before the exponential: alpha < 1/255 exactly when
// p < -log2(255 o) with p = log2(e) power.
// Output RGBA: C + T bg, 1 - T.
#include "v3dg_internal.h"

namespace v3dg {

constexpr int kBlendThreads = kTile * kTile;
constexpr float kLog2e = 1.4426950408889634f;

__global__ void __launch_bounds__(kBlendThreads) blend_kernel(CamArgs cam, const float4 *__restrict__ splat,
                                                              const uint32_t *__restrict__ vals,
                                                              const uint2 *__restrict__ ranges,
                                                              float4 *__restrict__ image, uint32_t per_xcd,
                                                              unsigned long long *__restrict__ pairs)
{
    __shared__ float4 sP0[kBlendThreads];   // (mx, my, a, b): p = a dx^2 + b dx dy + c dy^2
    __shared__ float4 sP1[kBlendThreads];   // (c, log2 threshold, log2 o, -)
    __shared__ float4 sP2[kBlendThreads];   // (r, g, b, -)
    __shared__ uint8_t sMask[kBlendThreads];
    __shared__ uint8_t sIdx[4][kBlendThreads];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    // workgroups are dealt round-robin to the 8 XCDs: give each XCD a
    // contiguous band of tiles so neighbouring tiles share its L2
    const uint32_t tile = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    if (tile >= n_tiles) return;
    const uint32_t tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const uint32_t qx = (uint32_t)wid & 1u, qy = (uint32_t)wid >> 1;
    const uint32_t x = tx * kTile + qx * 8u + ((uint32_t)lane & 7u), y = ty * kTile + qy * 8u + ((uint32_t)lane >> 3);
    const bool inside = x < cam.width && y < cam.height;
    const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
    // pixel-centre boxes of the four quarters
    const float bx0 = (float)(tx * kTile) + 0.5f, by0 = (float)(ty * kTile) + 0.5f;
    const uint2 rg = ranges[tile];
    float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
    bool done = !inside;
    uint32_t evaluated = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t start = rg.x; start < rg.y; start += kBlendThreads) {
        if (__syncthreads_count(done) == kBlendThreads) break;
        const uint32_t i = start + tid;
        uint32_t m = 0;
        if (i < rg.y) {
            const float4 *sp = splat + 3 * (uint64_t)vals[i];
            const float4 f0 = sp[0], f1 = sp[1], f2 = sp[2];
            const float lo = __log2f(f1.y);
            sP0[tid] = make_float4(f0.x, f0.y, -0.5f * kLog2e * f0.z, -kLog2e * f0.w);
            sP1[tid] = make_float4(-0.5f * kLog2e * f1.x, -(__log2f(255.0f) + lo), lo, 0.f);
            sP2[tid] = make_float4(f1.z, f1.w, f2.x, 0.f);
            const float hx = f2.z + 1.0f, hy = f2.w + 1.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float x0 = bx0 + 8.0f * (float)(q & 1), y0 = by0 + 8.0f * (float)(q >> 1);
                const bool hit = (f0.x + hx >= x0) && (f0.x - hx <= x0 + 7.0f) && (f0.y + hy >= y0) &&
                                 (f0.y - hy <= y0 + 7.0f);
                m |= (uint32_t)hit << q;
            }
        }
        sMask[tid] = (uint8_t)m;
        __syncthreads();
        // in-order compaction of this quarter's entries
        uint32_t cnt = 0;
#pragma unroll
        for (int c = 0; c < kBlendThreads / kWave; ++c) {
            const bool hit = (sMask[c * kWave + lane] >> wid) & 1u;
            const uint64_t bal = __ballot(hit);
            if (hit) sIdx[wid][cnt + (uint32_t)__popcll(bal & lt)] = (uint8_t)(c * kWave + lane);
            cnt += (uint32_t)__popcll(bal);
        }
        __syncthreads();
        if (__ballot(!done)) {
            // the walk is uniform across the wavefront: entry j is the same for
            // every lane; lanes differ only in whether they take the splat
            bool active = !done;
            uint32_t kend = cnt;  // entries this lane evaluated in this batch
            for (uint32_t k = 0; k < cnt; ++k) {
                const uint32_t j = sIdx[wid][k];
                const float4 a = sP0[j];
                const float4 b = sP1[j];
                const float dx = a.x - pxc, dy = a.y - pyc;
                const float p = fmaf(a.z * dx, dx, fmaf(a.w * dx, dy, b.x * dy * dy));
                const bool take = active && !(p < b.y);  // alpha >= 1/255
                if (__ballot(take) == 0) continue;
                // the exponent lies in [log2(1/255), 0]: the hardware exp2 is exact enough
                const float e = __builtin_amdgcn_exp2f((p < 0.0f ? p : 0.0f) + b.z);
                const float alpha = take ? fminf(0.99f, e) : 0.0f;
                const float Tn = T * (1.0f - alpha);
                const bool stop = take && Tn < 1e-4f;
                const bool add = take && !stop;
                const float4 c = sP2[j];
                const float w = add ? alpha * T : 0.0f;
                cr = fmaf(w, c.x, cr);
                cg = fmaf(w, c.y, cg);
                cb = fmaf(w, c.z, cb);
                T = add ? Tn : T;
                if (stop) {
                    active = false;
                    kend = k + 1;
                }
                if (__ballot(active) == 0) break;
            }
            if (!done) evaluated += kend;
            done = !active;
        }
    }
    if (inside)
        image[(uint64_t)y * cam.width + x] =
            make_float4(cr + T * cam.bg[0], cg + T * cam.bg[1], cb + T * cam.bg[2], 1.0f - T);
    // pairs evaluated by this wavefront, one atomic per wavefront
    uint32_t wsum = evaluated;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, kWave);
    if (lane == 0) atomicAdd(pairs, (unsigned long long)wsum);
}

void launch_blend(hipStream_t st, const CamArgs &cam, const float4 *splat, const uint32_t *vals, const uint2 *ranges,
                  float *image, unsigned long long *pairs)
{
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    const uint32_t per_xcd = (n_tiles + 7) / 8;
    hipLaunchKernelGGL(blend_kernel, dim3(per_xcd * 8), dim3(kBlendThreads), 0, st, cam, splat, vals, ranges,
                       reinterpret_cast<float4 *>(image), per_xcd, pairs);
}

}  // namespace v3dg
