// (e) front-to-back alpha compositing, one 256-thread workgroup per 16x16
// tile, one thread per pixel (paper Sec. 2.1: the splats covering a pixel are
// blended in depth order).  The tile's sorted splats are staged through LDS in
// batches of 256; the workgroup stops once every pixel is saturated.
//
// Per (pixel, splat), with d = mean - pixel centre and conic (A, B, C):
//   power = min(0, -1/2 (A dx^2 + C dy^2) - B dx dy),  alpha = min(0.99, o e^power);
//   alpha < 1/255 is skipped;  T' = T (1 - alpha);  T' < 1e-4 ends the pixel
//   without adding this splat;  otherwise C += alpha T rgb, T = T'.
// Output RGBA: C + T bg, 1 - T.
#include "v3dg_internal.h"

namespace v3dg {

constexpr int kBlendThreads = kTile * kTile;

__global__ void __launch_bounds__(kBlendThreads) blend_kernel(CamArgs cam, const float4 *__restrict__ splat,
                                                              const uint32_t *__restrict__ vals,
                                                              const uint2 *__restrict__ ranges,
                                                              float4 *__restrict__ image,
                                                              unsigned long long *__restrict__ pairs)
{
    __shared__ float4 s0[kBlendThreads], s1[kBlendThreads], s2[kBlendThreads];
    const int tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const uint32_t tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const uint32_t x = tx * kTile + (tid & (kTile - 1)), y = ty * kTile + (tid / kTile);
    const bool inside = x < cam.width && y < cam.height;
    const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
    const uint2 rg = ranges[tile];
    float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
    bool done = !inside;
    uint32_t evaluated = 0;
    for (uint32_t start = rg.x; start < rg.y; start += kBlendThreads) {
        if (__syncthreads_count(done) == kBlendThreads) break;
        const uint32_t i = start + tid;
        if (i < rg.y) {
            const float4 *sp = splat + 3 * (uint64_t)vals[i];
            s0[tid] = sp[0];
            s1[tid] = sp[1];
            s2[tid] = sp[2];
        }
        __syncthreads();
        const uint32_t cnt = min((uint32_t)kBlendThreads, rg.y - start);
        if (!done) {
            uint32_t j = 0;
            for (; j < cnt; ++j) {
                const float4 f0 = s0[j];
                const float dx = f0.x - pxc, dy = f0.y - pyc;
                const float4 f1 = s1[j];
                float power = -0.5f * (f0.z * dx * dx + f1.x * dy * dy) - f0.w * dx * dy;
                power = fminf(power, 0.0f);
                const float alpha = fminf(0.99f, f1.y * __expf(power));
                if (alpha < 1.0f / 255.0f) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < 1e-4f) {
                    done = true;
                    ++j;
                    break;
                }
                const float w = alpha * T;
                cr = fmaf(w, f1.z, cr);
                cg = fmaf(w, f1.w, cg);
                cb = fmaf(w, s2[j].x, cb);
                T = Tn;
            }
            evaluated += j;
        }
    }
    // pairs evaluated by this wavefront, one atomic per wavefront
    uint32_t wsum = evaluated;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, kWave);
    if ((tid & (kWave - 1)) == 0) atomicAdd(pairs, (unsigned long long)wsum);
    if (inside)
        image[(uint64_t)y * cam.width + x] =
            make_float4(cr + T * cam.bg[0], cg + T * cam.bg[1], cb + T * cam.bg[2], 1.0f - T);
}

void launch_blend(hipStream_t st, const CamArgs &cam, const float4 *splat, const uint32_t *vals, const uint2 *ranges,
                  float *image, unsigned long long *pairs)
{
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    hipLaunchKernelGGL(blend_kernel, dim3(n_tiles), dim3(kBlendThreads), 0, st, cam, splat, vals, ranges,
                       reinterpret_cast<float4 *>(image), pairs);
}

}  // namespace v3dg
