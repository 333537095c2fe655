// Offline build of the cluster bundle (paper Sec. 3.1-3.2, Algorithm 1),
// structural part: the binary median split into clusters and cluster groups,
// the halving of every group to the Gaussians with the larger product of
// scale and opacity (scales grown by 2^(1/6)), and the group bounding spheres
// (centre: mean Gaussian position; radius: farthest Gaussian).  The
// local-splatting refinement of the simplified Gaussians is not done here.
//
// Split of a set larger than n (one layer of the split at a time): the axis
// of the largest FP32 bounding-box extent (the first on ties), a stable order
// by that coordinate (-0 and +0 equal), the first ceil(s/2) items to the left.
// A layer is three launches over all sets at once: bounding boxes (atomics on
// order-preserving integer encodings), one 64-bit key per item (set index,
// coordinate bits) and a stable radix sort of (key, item).
//
// Every decision is taken in a fixed arithmetic order, so that the result is
// the same bit for bit on any run: FP32 extents and scores without
// contraction, FP64 means summed in row order, FP64 distances.
#include "v3dg_internal.h"

namespace v3dg {

constexpr int kBuildThreads = 256;

// order-preserving u32 encoding of an FP32 value (and back)
__device__ __forceinline__ uint32_t f2o(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// the set holding position e: the last s with start[s] <= e (start[0] = 0)
__device__ __forceinline__ uint32_t set_of(const uint32_t *__restrict__ start, uint32_t n_sets, uint32_t e)
{
    uint32_t lo = 0, hi = n_sets;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kBuildThreads) split_box_init_kernel(uint32_t *box, uint32_t n_sets)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    for (int a = 0; a < 3; ++a) {
        box[6ull * s + a] = 0xffffffffu;
        box[6ull * s + 3 + a] = 0u;
    }
}

// Bounding boxes of the sets that split: box[s] = (min x, y, z, max x, y, z)
// in the order-preserving encoding.
__global__ void __launch_bounds__(kBuildThreads) split_box_kernel(const float *__restrict__ pts,
                                                                  const uint32_t *__restrict__ items, uint32_t m,
                                                                  const uint32_t *__restrict__ start,
                                                                  const uint8_t *__restrict__ splits, uint32_t n_sets,
                                                                  uint32_t *box)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t s = 0, v[3] = {0u, 0u, 0u};
    bool live = false;
    if (e < m) {
        s = set_of(start, n_sets, e);
        live = splits[s] != 0;
        if (live) {
            const uint32_t it = items[e];
            for (int a = 0; a < 3; ++a) v[a] = f2o(pts[3ull * it + a]);
        }
    }
    const uint64_t act = __ballot(live);
    if (act == 0) return;
    const uint32_t s0 = __shfl(s, __ffsll((unsigned long long)act) - 1, kWave);
    if (__ballot(live && s == s0) == act) {
        // the wavefront's live lanes share one set: reduce, then one lane updates it
        for (int a = 0; a < 3; ++a) {
            uint32_t lo = live ? v[a] : 0xffffffffu, hi = live ? v[a] : 0u;
            for (int o = kWave / 2; o > 0; o >>= 1) {
                lo = min(lo, (uint32_t)__shfl_xor(lo, o, kWave));
                hi = max(hi, (uint32_t)__shfl_xor(hi, o, kWave));
            }
            if (lane == 0) {
                atomicMin(&box[6ull * s0 + a], lo);
                atomicMax(&box[6ull * s0 + 3 + a], hi);
            }
        }
    } else if (live) {
        for (int a = 0; a < 3; ++a) {
            atomicMin(&box[6ull * s + a], v[a]);
            atomicMax(&box[6ull * s + 3 + a], v[a]);
        }
    }
}

// key = set << 32 | coordinate bits along the set's split axis (0 for sets
// that do not split), value = the item
__global__ void __launch_bounds__(kBuildThreads) split_key_kernel(const float *__restrict__ pts,
                                                                  const uint32_t *__restrict__ items, uint32_t m,
                                                                  const uint32_t *__restrict__ start,
                                                                  const uint8_t *__restrict__ splits, uint32_t n_sets,
                                                                  const uint32_t *__restrict__ box,
                                                                  uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint32_t s = set_of(start, n_sets, e);
    const uint32_t it = items[e];
    uint32_t low = 0;
    if (splits[s]) {
        float ext[3];
        for (int a = 0; a < 3; ++a) ext[a] = __fsub_rn(o2f(box[6ull * s + 3 + a]), o2f(box[6ull * s + a]));
        int axis = 0;
        if (ext[1] > ext[axis]) axis = 1;
        if (ext[2] > ext[axis]) axis = 2;
        low = f2o(__fadd_rn(pts[3ull * it + axis], 0.0f));  // -0 and +0 alike
    }
    keys[e] = ((uint64_t)s << 32) | low;
    vals[e] = it;
}

void launch_split_layer(hipStream_t st, const float *pts, const uint32_t *items, uint32_t m, const uint32_t *start,
                        const uint8_t *splits, uint32_t n_sets, uint32_t *box, uint64_t *keys, uint32_t *vals)
{
    const uint32_t g = (m + kBuildThreads - 1) / kBuildThreads;
    hipLaunchKernelGGL(split_box_init_kernel, dim3((n_sets + kBuildThreads - 1) / kBuildThreads), dim3(kBuildThreads),
                       0, st, box, n_sets);
    hipLaunchKernelGGL(split_box_kernel, dim3(g), dim3(kBuildThreads), 0, st, pts, items, m, start, splits, n_sets,
                       box);
    hipLaunchKernelGGL(split_key_kernel, dim3(g), dim3(kBuildThreads), 0, st, pts, items, m, start, splits, n_sets,
                       box, keys, vals);
}

// FP64 mean of a cluster's Gaussian positions, summed in row order, in FP32.
__global__ void __launch_bounds__(kBuildThreads) cluster_mean_kernel(const float *__restrict__ pos,
                                                                     const uint32_t *__restrict__ rows,
                                                                     const uint32_t *__restrict__ first,
                                                                     const uint32_t *__restrict__ count, uint32_t n,
                                                                     float *__restrict__ mean, float *__restrict__ sph4)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double c[3] = {0.0, 0.0, 0.0};
    for (uint32_t i = 0; i < count[k]; ++i) {
        const uint32_t g = rows[first[k] + i];
        for (int a = 0; a < 3; ++a) c[a] = __dadd_rn(c[a], (double)pos[3ull * g + a]);
    }
    for (int a = 0; a < 3; ++a) {
        const float v = (float)__ddiv_rn(c[a], (double)count[k]);
        mean[3ull * k + a] = v;
        if (sph4) sph4[4ull * k + a] = v;
    }
    if (sph4) sph4[4ull * k + 3] = 0.0f;
}

void launch_cluster_mean(hipStream_t st, const float *pos, const uint32_t *rows, const uint32_t *first,
                         const uint32_t *count, uint32_t n, float *mean, float *sph4)
{
    if (n == 0) return;
    hipLaunchKernelGGL(cluster_mean_kernel, dim3((n + kBuildThreads - 1) / kBuildThreads), dim3(kBuildThreads), 0, st,
                       pos, rows, first, count, n, mean, sph4);
}

// smallest FP32 value >= x (x >= 0, finite)
__device__ __forceinline__ float round_up_f32(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, __builtin_huge_valf());
    return f;
}

__device__ __forceinline__ double dist64(const float *p, double cx, double cy, double cz)
{
    const double dx = __dsub_rn((double)p[0], cx), dy = __dsub_rn((double)p[1], cy), dz = __dsub_rn((double)p[2], cz);
    return __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
}

// One workgroup per cluster group (its member clusters are layer positions
// gfirst[g] .. gfirst[g] + gsize[g] - 1 of the permuted layer: perm[pos] is
// the cluster's index before the grouping).  The group's Gaussians G_o are
// the members' rows in member order; the ceil(m/2) with the largest
// ((sx sy) sz) o (current scales: the input's grown gen times; ties to the
// earlier one) are kept in G_o order as the new cluster g's rows at out_rows
// + g * cap.  sph[g] = the group sphere grown over the members' spheres.
constexpr int kGroupMax = 128;

__global__ void __launch_bounds__(kGroupMax) group_kernel(const float *__restrict__ pos,
                                                          const float *__restrict__ scale,
                                                          const float *__restrict__ opacity, uint32_t gen,
                                                          const uint32_t *__restrict__ rows,
                                                          const uint32_t *__restrict__ first,
                                                          const uint32_t *__restrict__ count,
                                                          const float *__restrict__ msph,
                                                          const uint32_t *__restrict__ perm,
                                                          const uint32_t *__restrict__ gfirst,
                                                          const uint32_t *__restrict__ gsize, uint32_t n_groups,
                                                          uint32_t cap, uint32_t *__restrict__ out_rows,
                                                          uint32_t *__restrict__ out_count, float *__restrict__ sph,
                                                          uint32_t *err)
{
    __shared__ float s_score[kGroupMax];
    __shared__ uint32_t s_src[kGroupMax];
    __shared__ double s_r[kGroupMax];
    __shared__ double s_c[3];
    __shared__ uint32_t s_m, s_base[2];
    const uint32_t g = blockIdx.x;
    const int t = threadIdx.x;
    if (g >= n_groups) return;
    if (t == 0) {
        uint32_t m = 0;
        for (uint32_t i = 0; i < gsize[g]; ++i) {
            s_base[i] = m;
            m += count[perm[gfirst[g] + i]];
        }
        s_m = m;
    }
    __syncthreads();
    const uint32_t m = s_m;
    if (m > (uint32_t)kGroupMax || (m + 1) / 2 > cap) {  // never with clusters of at most 64
        if (t == 0) atomicOr(err, 1u);
        return;
    }
    if ((uint32_t)t < m) {
        const uint32_t mi = (gsize[g] > 1 && (uint32_t)t >= s_base[1]) ? 1u : 0u;
        const uint32_t k = perm[gfirst[g] + mi];
        const uint32_t src = rows[first[k] + ((uint32_t)t - s_base[mi])];
        float sx = scale[3ull * src], sy = scale[3ull * src + 1], sz = scale[3ull * src + 2];
        const float grow = (float)kScaleGrowth;
        for (uint32_t j = 0; j < gen; ++j) {
            sx = __fmul_rn(sx, grow);
            sy = __fmul_rn(sy, grow);
            sz = __fmul_rn(sz, grow);
        }
        s_score[t] = __fmul_rn(__fmul_rn(__fmul_rn(sx, sy), sz), opacity[src]);
        s_src[t] = src;
    }
    __syncthreads();
    // rank among the group: larger scores first, the earlier Gaussian on ties
    bool keep = false;
    if ((uint32_t)t < m) {
        const float sc = s_score[t];
        uint32_t rank = 0;
        for (uint32_t q = 0; q < m; ++q) rank += (s_score[q] > sc || (s_score[q] == sc && q < (uint32_t)t)) ? 1u : 0u;
        keep = rank < (m + 1) / 2;
    }
    // kept Gaussians in group order
    {
        const uint64_t b0 = __ballot(keep && t < kWave), b1 = __ballot(keep && t >= kWave);
        __shared__ uint32_t s_cnt[2];
        if ((t & (kWave - 1)) == 0) s_cnt[t / kWave] = (uint32_t)__popcll(t < kWave ? b0 : b1);
        __syncthreads();
        const uint64_t mine = t < kWave ? b0 : b1;
        const uint32_t lane = t & (kWave - 1);
        const uint32_t at = (t < kWave ? 0u : s_cnt[0]) + (uint32_t)__popcll(mine & ((1ull << lane) - 1ull));
        if (keep) out_rows[(uint64_t)g * cap + at] = s_src[t];
        if (t == 0) out_count[g] = (m + 1) / 2;
    }
    // sphere: FP64 mean in G_o order, then the farthest Gaussian
    if (t == 0) {
        double c[3] = {0.0, 0.0, 0.0};
        for (uint32_t q = 0; q < m; ++q)
            for (int a = 0; a < 3; ++a) c[a] = __dadd_rn(c[a], (double)pos[3ull * s_src[q] + a]);
        for (int a = 0; a < 3; ++a) s_c[a] = (double)(float)__ddiv_rn(c[a], (double)m);
    }
    __syncthreads();
    s_r[t] = (uint32_t)t < m ? dist64(pos + 3ull * s_src[t], s_c[0], s_c[1], s_c[2]) : 0.0;
    __syncthreads();
    if (t == 0) {
        double r = 0.0;
        for (uint32_t q = 0; q < m; ++q) r = fmax(r, s_r[q]);
        float rf = round_up_f32(r);
        for (uint32_t i = 0; i < gsize[g]; ++i) {
            const float *cs = msph + 4ull * perm[gfirst[g] + i];
            const double need = __dmul_rn(__dadd_rn(dist64(cs, s_c[0], s_c[1], s_c[2]), (double)cs[3]), kNestSlack);
            rf = fmaxf(rf, round_up_f32(need));
        }
        sph[4ull * g] = (float)s_c[0];
        sph[4ull * g + 1] = (float)s_c[1];
        sph[4ull * g + 2] = (float)s_c[2];
        sph[4ull * g + 3] = rf;
    }
}

void launch_group(hipStream_t st, const float *pos, const float *scale, const float *opacity, uint32_t gen,
                  const uint32_t *rows, const uint32_t *first, const uint32_t *count, const float *msph,
                  const uint32_t *perm, const uint32_t *gfirst, const uint32_t *gsize, uint32_t n_groups, uint32_t cap,
                  uint32_t *out_rows, uint32_t *out_count, float *sph, uint32_t *err)
{
    if (n_groups == 0) return;
    hipLaunchKernelGGL(group_kernel, dim3(n_groups), dim3(kGroupMax), 0, st, pos, scale, opacity, gen, rows, first,
                       count, msph, perm, gfirst, gsize, n_groups, cap, out_rows, out_count, sph, err);
}

// Bundle rows: row i is input Gaussian src[i] with its scales grown gen[i] times.
__global__ void __launch_bounds__(kBuildThreads) bundle_rows_kernel(
    const float *__restrict__ pos, const float *__restrict__ scale, const float *__restrict__ rot,
    const float *__restrict__ opacity, const float *__restrict__ sh, uint32_t sh_floats,
    const uint32_t *__restrict__ src, const uint8_t *__restrict__ gen, uint32_t n_rows, float *__restrict__ opos,
    float *__restrict__ oscale, float *__restrict__ orot, float *__restrict__ oopacity, float *__restrict__ osh)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const uint64_t s = src[i];
    const float grow = (float)kScaleGrowth;
    for (int a = 0; a < 3; ++a) {
        opos[3ull * i + a] = pos[3 * s + a];
        float v = scale[3 * s + a];
        for (uint32_t j = 0; j < gen[i]; ++j) v = __fmul_rn(v, grow);
        oscale[3ull * i + a] = v;
    }
    for (int a = 0; a < 4; ++a) orot[4ull * i + a] = rot[4 * s + a];
    oopacity[i] = opacity[s];
    for (uint32_t a = 0; a < sh_floats; ++a) osh[(uint64_t)sh_floats * i + a] = sh[sh_floats * s + a];
}

void launch_bundle_rows(hipStream_t st, const float *pos, const float *scale, const float *rot, const float *opacity,
                        const float *sh, uint32_t sh_floats, const uint32_t *src, const uint8_t *gen, uint32_t n_rows,
                        float *opos, float *oscale, float *orot, float *oopacity, float *osh)
{
    if (n_rows == 0) return;
    hipLaunchKernelGGL(bundle_rows_kernel, dim3((n_rows + kBuildThreads - 1) / kBuildThreads), dim3(kBuildThreads), 0,
                       st, pos, scale, rot, opacity, sh, sh_floats, src, gen, n_rows, opos, oscale, orot, oopacity,
                       osh);
}

}  // namespace v3dg
