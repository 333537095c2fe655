// Cluster streaming: page images staged from host memory are scattered into
// the device page pool.
//
// A streamed scene keeps its Gaussian rows in host memory as one page image
// per cluster and holds a pool of pages of 64 rows in device memory, in the
// planar layout the projection reads (plane stride = pool rows).  Selecting a
// cut pages in the clusters it needs that are not resident (the host picks the
// pages and copies their images to a staging buffer in one transfer); this
// kernel then writes every staged image into its page and points the
// cluster's row info at the page.  This is the streaming module the paper's
// conclusion and discussion leaves to future work: selected clusters are
// loaded on demand and pages no longer used are given to others, so the rows
// of a scene need not fit in GPU memory (its cluster tables stay resident).
#include <hip/hip_runtime.h>

#include "v3dg_internal.h"

namespace v3dg {

// Page image layout (bytes): 3 position planes of 64 FP32, then 8 geometry
// planes of 64 elements of geo_bytes, then n_sh planes of 64 elements of
// sh_bytes.  ups[e] = (cluster, destination page, rows, 0).  One workgroup
// of 256 threads per staged image: thread t copies row t % 64 of planes
// t / 64, t / 64 + 4, ...
__global__ void __launch_bounds__(256) stream_scatter_kernel(const uint8_t *__restrict__ staging,
                                                             const uint4 *__restrict__ ups, uint32_t n_up,
                                                             uint32_t page_bytes, uint32_t geo_bytes,
                                                             uint32_t sh_bytes, uint32_t n_sh, float *pos_planes,
                                                             uint8_t *geo_planes, uint8_t *sh_planes,
                                                             uint64_t stride, uint2 *rowinfo)
{
    const uint32_t e = blockIdx.x;
    if (e >= n_up) return;
    const uint4 u = ups[e];
    const uint32_t lane = threadIdx.x & 63u, p0 = threadIdx.x >> 6;
    const uint64_t row = (uint64_t)u.y * 64u + lane;
    const uint8_t *img = staging + (uint64_t)e * page_bytes;
    const uint32_t n_planes = 3u + (uint32_t)kGeoPlanes + n_sh;
    if (lane < u.z) {
        for (uint32_t p = p0; p < n_planes; p += 4) {
            if (p < 3) {
                pos_planes[p * stride + row] = reinterpret_cast<const float *>(img)[p * 64u + lane];
            } else if (p < 3u + (uint32_t)kGeoPlanes) {
                const uint32_t g = p - 3u;
                const uint8_t *src = img + 3u * 256u + (uint64_t)g * 64u * geo_bytes;
                if (geo_bytes == 4)
                    reinterpret_cast<float *>(geo_planes)[g * stride + row] = reinterpret_cast<const float *>(src)[lane];
                else
                    reinterpret_cast<uint16_t *>(geo_planes)[g * stride + row] =
                        reinterpret_cast<const uint16_t *>(src)[lane];
            } else {
                const uint32_t c = p - 3u - (uint32_t)kGeoPlanes;
                const uint8_t *src = img + 3u * 256u + (uint64_t)kGeoPlanes * 64u * geo_bytes + (uint64_t)c * 64u * sh_bytes;
                if (sh_bytes == 4)
                    reinterpret_cast<float *>(sh_planes)[c * stride + row] = reinterpret_cast<const float *>(src)[lane];
                else
                    reinterpret_cast<uint16_t *>(sh_planes)[c * stride + row] =
                        reinterpret_cast<const uint16_t *>(src)[lane];
            }
        }
    }
    if (threadIdx.x == 0) rowinfo[u.x] = make_uint2(u.y * 64u, u.z);
}

void launch_stream_scatter(hipStream_t st, const uint8_t *staging, const uint4 *ups, uint32_t n_up,
                           uint32_t page_bytes, uint32_t geo_bytes, uint32_t sh_bytes, uint32_t n_sh,
                           float *pos_planes, void *geo_planes, void *sh_planes, uint64_t stride, uint2 *rowinfo)
{
    if (n_up == 0) return;
    hipLaunchKernelGGL(stream_scatter_kernel, dim3(n_up), dim3(256), 0, st, staging, ups, n_up, page_bytes, geo_bytes,
                       sh_bytes, n_sh, pos_planes, (uint8_t *)geo_planes, (uint8_t *)sh_planes, stride, rowinfo);
}

}  // namespace v3dg
