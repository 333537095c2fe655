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
// the members' rows in member order (ids into the layer's row store, written
// to go_rows[g * kGroupMax ..], their number to go_count[g]); the ceil(m/2)
// with the largest ((sx sy) sz) o (the rows' current values; ties to the
// earlier one) are kept in G_o order, their ids at kept + g * cap.  sph[g] =
// the group sphere over G_o, grown over the members' spheres; vsph[g] = its
// centre with the radius that frames the group's pseudo-views: the farthest
// 3-sigma reach |p - c| + 3 max(sx, sy, sz) of a Gaussian of G_o, rounded up.
constexpr int kGroupMax = 128;

__global__ void __launch_bounds__(kGroupMax) group_kernel(const float *__restrict__ pos,
                                                          const float *__restrict__ scale,
                                                          const float *__restrict__ opacity,
                                                          const uint32_t *__restrict__ rows,
                                                          const uint32_t *__restrict__ first,
                                                          const uint32_t *__restrict__ count,
                                                          const float *__restrict__ msph,
                                                          const uint32_t *__restrict__ perm,
                                                          const uint32_t *__restrict__ gfirst,
                                                          const uint32_t *__restrict__ gsize, uint32_t n_groups,
                                                          uint32_t cap, uint32_t *__restrict__ kept,
                                                          uint32_t *__restrict__ out_count, float *__restrict__ sph,
                                                          float *__restrict__ vsph, uint32_t *__restrict__ go_rows,
                                                          uint32_t *__restrict__ go_count, uint32_t *err)
{
    __shared__ float s_score[kGroupMax];
    __shared__ uint32_t s_src[kGroupMax];
    __shared__ double s_r[kGroupMax], s_v[kGroupMax];
    __shared__ float s_ms[kGroupMax];
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
        const float sx = scale[3ull * src], sy = scale[3ull * src + 1], sz = scale[3ull * src + 2];
        s_score[t] = __fmul_rn(__fmul_rn(__fmul_rn(sx, sy), sz), opacity[src]);
        s_ms[t] = fmaxf(fmaxf(sx, sy), sz);
        s_src[t] = src;
        go_rows[(uint64_t)g * kGroupMax + t] = src;
    }
    if (t == 0) go_count[g] = m;
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
        if (keep) kept[(uint64_t)g * cap + at] = s_src[t];
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
    s_v[t] = (uint32_t)t < m ? __dadd_rn(s_r[t], __dmul_rn(3.0, (double)s_ms[t])) : 0.0;
    __syncthreads();
    if (t == 0) {
        double r = 0.0, rv = 0.0;
        for (uint32_t q = 0; q < m; ++q) {
            r = fmax(r, s_r[q]);
            rv = fmax(rv, s_v[q]);
        }
        vsph[4ull * g] = (float)s_c[0];
        vsph[4ull * g + 1] = (float)s_c[1];
        vsph[4ull * g + 2] = (float)s_c[2];
        vsph[4ull * g + 3] = round_up_f32(rv);
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

void launch_group(hipStream_t st, const float *pos, const float *scale, const float *opacity, const uint32_t *rows,
                  const uint32_t *first, const uint32_t *count, const float *msph, const uint32_t *perm,
                  const uint32_t *gfirst, const uint32_t *gsize, uint32_t n_groups, uint32_t cap, uint32_t *kept,
                  uint32_t *out_count, float *sph, float *vsph, uint32_t *go_rows, uint32_t *go_count, uint32_t *err)
{
    if (n_groups == 0) return;
    hipLaunchKernelGGL(group_kernel, dim3(n_groups), dim3(kGroupMax), 0, st, pos, scale, opacity, rows, first, count,
                       msph, perm, gfirst, gsize, n_groups, cap, kept, out_count, sph, vsph, go_rows, go_count, err);
}

// The next layer's row store: slot g * cap + i (i < count[g]) is a copy of
// the kept row kept[g * cap + i] of the current store with its scales grown
// once by float(2^(1/6)); src carries the input Gaussian it descends from
// (the current store's src, or the row id itself for the input); rows[slot]
// = slot.
__global__ void __launch_bounds__(kBuildThreads) spawn_kernel(
    const float *__restrict__ pos, const float *__restrict__ scale, const float *__restrict__ rot,
    const float *__restrict__ opacity, const float *__restrict__ sh, const uint32_t *__restrict__ src,
    uint32_t sh_floats, const uint32_t *__restrict__ kept, const uint32_t *__restrict__ count, uint32_t n_groups,
    uint32_t cap, float *__restrict__ npos, float *__restrict__ nscale, float *__restrict__ nrot,
    float *__restrict__ nopacity, float *__restrict__ nsh, uint32_t *__restrict__ nsrc, uint32_t *__restrict__ nrows)
{
    const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (uint64_t)n_groups * cap) return;
    const uint32_t g = (uint32_t)(slot / cap), i = (uint32_t)(slot % cap);
    if (i >= count[g]) return;
    const uint64_t r = kept[slot];
    const float grow = (float)kScaleGrowth;
    for (int a = 0; a < 3; ++a) {
        npos[3 * slot + a] = pos[3 * r + a];
        nscale[3 * slot + a] = __fmul_rn(scale[3 * r + a], grow);
    }
    for (int a = 0; a < 4; ++a) nrot[4 * slot + a] = rot[4 * r + a];
    nopacity[slot] = opacity[r];
    for (uint32_t a = 0; a < sh_floats; ++a) nsh[(uint64_t)sh_floats * slot + a] = sh[(uint64_t)sh_floats * r + a];
    nsrc[slot] = src ? src[r] : (uint32_t)r;
    nrows[slot] = (uint32_t)slot;
}

void launch_spawn(hipStream_t st, const float *pos, const float *scale, const float *rot, const float *opacity,
                  const float *sh, const uint32_t *src, uint32_t sh_floats, const uint32_t *kept,
                  const uint32_t *count, uint32_t n_groups, uint32_t cap, float *npos, float *nscale, float *nrot,
                  float *nopacity, float *nsh, uint32_t *nsrc, uint32_t *nrows)
{
    const uint64_t n = (uint64_t)n_groups * cap;
    if (n == 0) return;
    hipLaunchKernelGGL(spawn_kernel, dim3((uint32_t)((n + kBuildThreads - 1) / kBuildThreads)), dim3(kBuildThreads), 0,
                       st, pos, scale, rot, opacity, sh, src, sh_floats, kept, count, n_groups, cap, npos, nscale,
                       nrot, nopacity, nsh, nsrc, nrows);
}

// Bundle rows of one layer: output row i is row idx[i] of the layer's store.
__global__ void __launch_bounds__(kBuildThreads) gather_rows_kernel(
    const float *__restrict__ pos, const float *__restrict__ scale, const float *__restrict__ rot,
    const float *__restrict__ opacity, const float *__restrict__ sh, uint32_t sh_floats,
    const uint32_t *__restrict__ idx, uint32_t n_rows, float *__restrict__ opos, float *__restrict__ oscale,
    float *__restrict__ orot, float *__restrict__ oopacity, float *__restrict__ osh)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const uint64_t s = idx[i];
    for (int a = 0; a < 3; ++a) {
        opos[3ull * i + a] = pos[3 * s + a];
        oscale[3ull * i + a] = scale[3 * s + a];
    }
    for (int a = 0; a < 4; ++a) orot[4ull * i + a] = rot[4 * s + a];
    oopacity[i] = opacity[s];
    for (uint32_t a = 0; a < sh_floats; ++a) osh[(uint64_t)sh_floats * i + a] = sh[sh_floats * s + a];
}

void launch_gather_rows(hipStream_t st, const float *pos, const float *scale, const float *rot, const float *opacity,
                        const float *sh, uint32_t sh_floats, const uint32_t *idx, uint32_t n_rows, float *opos,
                        float *oscale, float *orot, float *oopacity, float *osh)
{
    if (n_rows == 0) return;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((n_rows + kBuildThreads - 1) / kBuildThreads), dim3(kBuildThreads), 0,
                       st, pos, scale, rot, opacity, sh, sh_floats, idx, n_rows, opos, oscale, orot, oopacity, osh);
}


// ---------------------------------------------------------------------------
// Local splatting of cluster groups (paper Sec. 3.2): the simplified
// Gaussians of a group are fitted to its original ones.  For every
// pseudo-view (the group centre seen from four radii away along dirs[it]),
// both sets are splatted at 64 x 64 as in the renderer (EWA without
// dilation, guard band 1.3 tan(fov/2), alpha = min(0.99, o e^power), skip
// below 1/255, stop before T falls below 1e-4, background 0), with the
// SH degree-0 colour max(0, C0 dc + 0.5); the loss is mean |rgb - target| +
// 0.1 mean |alpha - target alpha|, and one Adam step (0.9, 0.999, 1e-15)
// updates position, log scale, quaternion, logit opacity and dc with rates
// 1.6e-5, 5e-3, 1e-3, 5e-2, 2.5e-3.
//
// One 1024-thread workgroup per group: 16 wavefronts of 4 image rows each
// (lane = pixel), walking their rows together over the depth-sorted splats
// that reach them.  The backward walk runs over the fitted splats in reverse
// depth order, recovering T by division; each splat's gradient terms are
// summed over a wavefront's rows in every lane, then across the lanes, and
// kept per wavefront, so every sum is taken in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kLsThreads = 1024;
constexpr int kLsRes = 64;
constexpr int kLsMaxO = 128;
constexpr int kLsMaxS = 64;
constexpr int kLsP = 14;  // pos 0-2, log scale 3-5, quaternion 6-9, logit 10, dc 11-13
constexpr float kLsC0 = 0.28209479177387814f;

struct LsShared {
    float prm[kLsMaxS][kLsP], m1[kLsMaxS][kLsP], m2[kLsMaxS][kLsP];
    float opos[kLsMaxO][3], oscl[kLsMaxO][3], oq[kLsMaxO][4], oop[kLsMaxO], orgb[kLsMaxO][3];
    // splats of the current view: originals 0 .. 127, fitted ones 128 .. 191
    float pu[192], pv[192], pca[192], pcb[192], pcc[192], pop[192], prow[192], pz[192], prgb[192][3];
    uint8_t pvalid[192];
    uint8_t ord[192];
    // the view's valid splats in depth order: originals at 0 .., fitted at
    // 128 ..; (u, v, ca, cb), (cc, o, r, g), (b, row limit, -, -)
    float4 sp1[192], sp2[192], sp3[192];
    float acc[kLsThreads / kWave][kLsMaxS][9];  // per wavefront: du dv dca dcb dcc dop dr dg db (per fitted index)
    float cam[12];                                // world-to-camera rows, eye
    float red[kLsThreads / kWave];
};

__device__ __forceinline__ float ls_sigmoid(float x) { return 1.0f / (1.0f + __expf(-x)); }

// trainable forms of scale and opacity; the originals are rendered through
// the same forms, so a set fitted to itself renders bit for bit like its target
__device__ __forceinline__ float ls_logit(float o)
{
    o = fminf(fmaxf(o, 1e-6f), 1.0f - 1e-6f);
    return __logf(o / (1.0f - o));
}

// camera-space point, screen position, conic and Sigma2_yy of a Gaussian
__device__ bool ls_project(const float *cam, const float *p, const float *s, const float *qr, float &u, float &v,
                           float &ca, float &cb, float &cc, float &syy, float &zo)
{
    constexpr float f = 123.93546707863734f;  // 32 / tan(asin(1/4)) = 32 sqrt(15)
    const float dp[3] = {p[0] - cam[9], p[1] - cam[10], p[2] - cam[11]};
    float pc[3];
    for (int r = 0; r < 3; ++r) pc[r] = cam[3 * r] * dp[0] + cam[3 * r + 1] * dp[1] + cam[3 * r + 2] * dp[2];
    zo = pc[2];
    if (!(pc[2] > 0.01f)) return false;
    const float z = pc[2];
    u = f * pc[0] / z + 32.0f;
    v = f * pc[1] / z + 32.0f;
    const float lim = 1.3f * 32.0f / f;
    const float tx = fminf(fmaxf(pc[0] / z, -lim), lim) * z, ty = fminf(fmaxf(pc[1] / z, -lim), lim) * z;
    const float J[2][3] = {{f / z, 0.0f, -f * tx / (z * z)}, {0.0f, f / z, -f * ty / (z * z)}};
    float T[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) T[r][c] = J[r][0] * cam[c] + J[r][1] * cam[3 + c] + J[r][2] * cam[6 + c];
    const float qn = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    const float w = qr[0] / qn, x = qr[1] / qn, y = qr[2] / qn, zq = qr[3] / qn;
    const float R[3][3] = {{1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)},
                           {2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)},
                           {2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)}};
    float TM[2][3];  // T R S
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) TM[r][c] = (T[r][0] * R[0][c] + T[r][1] * R[1][c] + T[r][2] * R[2][c]) * s[c];
    const float a = TM[0][0] * TM[0][0] + TM[0][1] * TM[0][1] + TM[0][2] * TM[0][2];
    const float b = TM[0][0] * TM[1][0] + TM[0][1] * TM[1][1] + TM[0][2] * TM[1][2];
    const float c = TM[1][0] * TM[1][0] + TM[1][1] * TM[1][1] + TM[1][2] * TM[1][2];
    const float det = a * c - b * b;
    if (!(det > 0.0f)) return false;
    ca = c / det;
    cb = -b / det;
    cc = a / det;
    syy = c;
    return true;
}

// Largest squared row distance dy^2 at which a splat still reaches alpha >=
// 1/255 on the row (pixel centre y): the largest power over a row is
// -dy^2 / (2 Sigma2_yy), so dy^2 <= 2 Sigma2_yy ln(255 o), enlarged by 1 %
// and 1e-4 so that the test never drops a contributing splat; -1 when o <
// 1/255 (the splat reaches no row).
__device__ __forceinline__ float ls_row_limit(float syy, float op)
{
    return op * 255.0f >= 1.0f ? 2.0f * syy * __logf(255.0f * op) * 1.01f + 1e-4f : -1.0f;
}

__device__ __forceinline__ float wave_sum(float x)
{
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// value of x in lane k (k uniform across the wavefront)
__device__ __forceinline__ float lane_value(float x, int k)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), k));
}

template <int kCtrl, int kRowMask, int kBankMask>
__device__ __forceinline__ float dpp_from(float x)  // 0 where the source lane is out of range or masked
{
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, kRowMask, kBankMask, false));
}

// Sum over the wavefront by data-parallel moves within rows of 16 lanes and
// row broadcasts (row_shr 1, 2, 4, 8; row_bcast 15, 31): lane 63 ends with
// the total, which is returned to every lane.  The order of the additions is
// fixed, so the sum is deterministic.
__device__ __forceinline__ float wave_total(float x)
{
    x += dpp_from<0x111, 0xf, 0xf>(x);
    x += dpp_from<0x112, 0xf, 0xf>(x);
    x += dpp_from<0x114, 0xf, 0xe>(x);
    x += dpp_from<0x118, 0xf, 0xc>(x);
    x += dpp_from<0x142, 0xa, 0xf>(x);
    x += dpp_from<0x143, 0xc, 0xf>(x);
    return lane_value(x, kWave - 1);
}

__global__ void __launch_bounds__(kLsThreads) local_splat_kernel(
    const uint32_t *__restrict__ ofirst, const uint32_t *__restrict__ ocount, const uint32_t *__restrict__ sfirst,
    const uint32_t *__restrict__ scount, const float *__restrict__ sphere, const float *__restrict__ opos,
    const float *__restrict__ oscale, const float *__restrict__ orot, const float *__restrict__ oopacity,
    const float *__restrict__ odc, uint32_t odc_stride, const uint32_t *__restrict__ orows, float *spos, float *sscale, float *srot, float *sopacity,
    float *sdc, uint32_t sdc_stride, const float *__restrict__ dirs, uint32_t iters, uint32_t n_groups,
    float *__restrict__ losses, float *__restrict__ grad_first, uint32_t *err)
{
    __shared__ LsShared sh;
    const uint32_t g = blockIdx.x;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    if (g >= n_groups) return;
    const uint32_t no = ocount[g], ns = scount[g], of = ofirst[g], sf = sfirst[g];
    if (no > (uint32_t)kLsMaxO || ns > (uint32_t)kLsMaxS) {
        if (t == 0) atomicOr(err, 2u);
        return;
    }
    if (ns == 0) {  // nothing to fit: zero losses
        if (losses)
            for (uint32_t it = (uint32_t)t; it < iters; it += kLsThreads) losses[(uint64_t)g * iters + it] = 0.0f;
        return;
    }
    if ((uint32_t)t < no) {
        const uint64_t r = orows ? orows[of + t] : of + t;
        for (int a = 0; a < 3; ++a) {
            sh.opos[t][a] = opos[3 * r + a];
            sh.oscl[t][a] = __expf(__logf(oscale[3 * r + a]));
            sh.orgb[t][a] = fmaxf(0.0f, kLsC0 * odc[odc_stride * r + a] + 0.5f);
        }
        for (int a = 0; a < 4; ++a) sh.oq[t][a] = orot[4 * r + a];
        sh.oop[t] = ls_sigmoid(ls_logit(oopacity[r]));
    }
    for (int i = t; i < (int)ns * kLsP; i += kLsThreads) {
        const int k = i / kLsP, j = i % kLsP;
        const uint64_t r = sf + k;
        float val;
        if (j < 3) val = spos[3 * r + j];
        else if (j < 6) val = __logf(sscale[3 * r + j - 3]);
        else if (j < 10) val = srot[4 * r + j - 6];
        else if (j == 10) val = ls_logit(sopacity[r]);
        else val = sdc[(uint64_t)sdc_stride * r + j - 11];
        sh.prm[k][j] = val;
        sh.m1[k][j] = 0.0f;
        sh.m2[k][j] = 0.0f;
    }
    for (int i = t; i < kLsThreads / kWave * kLsMaxS * 9; i += kLsThreads) (&sh.acc[0][0][0])[i] = 0.0f;
    const float cx = sphere[4ull * g], cy = sphere[4ull * g + 1], cz = sphere[4ull * g + 2],
                rad = sphere[4ull * g + 3];
    const float wr = 1.0f / (float)(kLsRes * kLsRes * 3), wa = 0.1f / (float)(kLsRes * kLsRes);
    for (uint32_t it = 0; it < iters; ++it) {
        if (t == 0) {  // pseudo-view it (FP64, rounded)
            double d[3] = {dirs[3 * it], dirs[3 * it + 1], dirs[3 * it + 2]};
            const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double eye[3] = {cx + 4.0 * rad * d[0] / dn, cy + 4.0 * rad * d[1] / dn, cz + 4.0 * rad * d[2] / dn};
            const double fw[3] = {-d[0] / dn, -d[1] / dn, -d[2] / dn};
            const double up[3] = {0.0, fabs(d[2] / dn) > 0.99 ? 1.0 : 0.0, fabs(d[2] / dn) > 0.99 ? 0.0 : 1.0};
            double rt[3] = {fw[1] * up[2] - fw[2] * up[1], fw[2] * up[0] - fw[0] * up[2], fw[0] * up[1] - fw[1] * up[0]};
            const double rn = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
            for (int a = 0; a < 3; ++a) rt[a] /= rn;
            const double dw[3] = {fw[1] * rt[2] - fw[2] * rt[1], fw[2] * rt[0] - fw[0] * rt[2],
                                  fw[0] * rt[1] - fw[1] * rt[0]};
            for (int a = 0; a < 3; ++a) {
                sh.cam[a] = (float)rt[a];
                sh.cam[3 + a] = (float)dw[a];
                sh.cam[6 + a] = (float)fw[a];
                sh.cam[9 + a] = (float)eye[a];
            }
        }
        __syncthreads();
        // splats of this view
        if ((uint32_t)t < no || (t >= kLsMaxO && (uint32_t)(t - kLsMaxO) < ns)) {
            const bool orig = t < kLsMaxO;
            const int k = orig ? t : t - kLsMaxO;
            float p[3], s[3], q[4], op;
            if (orig) {
                for (int a = 0; a < 3; ++a) {
                    p[a] = sh.opos[k][a];
                    s[a] = sh.oscl[k][a];
                }
                for (int a = 0; a < 4; ++a) q[a] = sh.oq[k][a];
                op = sh.oop[k];
            } else {
                for (int a = 0; a < 3; ++a) {
                    p[a] = sh.prm[k][a];
                    s[a] = __expf(sh.prm[k][3 + a]);
                }
                for (int a = 0; a < 4; ++a) q[a] = sh.prm[k][6 + a];
                op = ls_sigmoid(sh.prm[k][10]);
            }
            float u = 0, v = 0, ca = 0, cb = 0, cc = 0, syy = 0, z = 0;
            const bool ok = ls_project(sh.cam, p, s, q, u, v, ca, cb, cc, syy, z);
            sh.pu[t] = u;
            sh.pv[t] = v;
            sh.pca[t] = ca;
            sh.pcb[t] = cb;
            sh.pcc[t] = cc;
            sh.prow[t] = ls_row_limit(syy, op);
            sh.pz[t] = z;
            sh.pop[t] = op;
            sh.pvalid[t] = ok ? 1 : 0;
            for (int a = 0; a < 3; ++a)
                sh.prgb[t][a] = orig ? sh.orgb[k][a] : fmaxf(0.0f, kLsC0 * sh.prm[k][11 + a] + 0.5f);
        }
        __syncthreads();
        // depth order of the valid splats of each set (ties: index)
        if ((uint32_t)t < no || (t >= kLsMaxO && (uint32_t)(t - kLsMaxO) < ns)) {
            const bool orig = t < kLsMaxO;
            const int base = orig ? 0 : kLsMaxO, cnt = orig ? (int)no : (int)ns, k = t - base;
            if (sh.pvalid[t]) {
                int rank = 0;
                for (int j = 0; j < cnt; ++j)
                    if (sh.pvalid[base + j] && (sh.pz[base + j] < sh.pz[t] || (sh.pz[base + j] == sh.pz[t] && j < k)))
                        ++rank;
                sh.ord[base + rank] = (uint8_t)k;
                sh.sp1[base + rank] = make_float4(sh.pu[t], sh.pv[t], sh.pca[t], sh.pcb[t]);
                sh.sp2[base + rank] = make_float4(sh.pcc[t], sh.pop[t], sh.prgb[t][0], sh.prgb[t][1]);
                sh.sp3[base + rank] = make_float4(sh.prgb[t][2], sh.prow[t], 0.0f, 0.0f);
            }
        }
        const int n_o = __syncthreads_count((uint32_t)t < no && sh.pvalid[t]);
        const int n_s = __syncthreads_count(t >= kLsMaxO && (uint32_t)(t - kLsMaxO) < ns && sh.pvalid[t]);
        // row tests in registers (lane l: original slots l and 64 + l,
        // fitted slot l); the walks read slot k's parameters from LDS, the
        // same address in every lane
        float oV[2], oR[2];
        for (int h = 0; h < 2; ++h) {
            const int slot = h * kWave + lane;
            oV[h] = slot < n_o ? sh.sp1[slot].y : 0.0f;
            oR[h] = slot < n_o ? sh.sp3[slot].y : -1.0f;
        }
        const int js = lane < n_s ? (int)sh.ord[kLsMaxO + lane] : 0;
        const float sV = lane < n_s ? sh.sp1[kLsMaxO + lane].y : 0.0f, sR = lane < n_s ? sh.sp3[kLsMaxO + lane].y : -1.0f;
        float acc9[9];
        for (int a = 0; a < 9; ++a) acc9[a] = 0.0f;  // gradient sums of fitted depth slot `lane`
        float lsum = 0.0f;
        // the wavefront's kR rows are walked together: a splat's parameters
        // are read once for all of them, and its gradient terms are summed over
        // them in each lane before one wavefront sum
        constexpr int kR = kLsRes / (kLsThreads / kWave);
        const float xc = (float)lane + 0.5f;
        float yc[kR];
        uint64_t mo[kR][2], ms[kR], uo[2] = {0ull, 0ull}, us = 0ull;
#pragma unroll
        for (int r = 0; r < kR; ++r) {  // depth slots whose splat reaches row r, as bit masks
            yc[r] = (float)(wid * kR + r) + 0.5f;
            const float d0 = oV[0] - yc[r], d1 = oV[1] - yc[r], ds = sV - yc[r];
            mo[r][0] = __ballot(d0 * d0 <= oR[0]);
            mo[r][1] = __ballot(d1 * d1 <= oR[1]);
            ms[r] = __ballot(ds * ds <= sR);
            uo[0] |= mo[r][0];
            uo[1] |= mo[r][1];
            us |= ms[r];
        }
        // front-to-back compositing of one splat at one pixel (the renderer's rule)
        auto blend = [&](const float4 &p1, const float4 &p2, const float4 &p3, float yr, float &T, float &c0,
                         float &c1, float &c2, bool &live) -> bool {
            const float dx = p1.x - xc, dy = p1.y - yr;
            const float pw = fminf(0.0f, -0.5f * (p1.z * dx * dx + p2.x * dy * dy) - p1.w * dx * dy);
            const float al = fminf(0.99f, p2.y * __expf(pw));
            const bool take = live && al >= 1.0f / 255.0f;
            const float Tn = T * (1.0f - al);
            const bool stop = take && Tn < 1e-4f;
            if (take && !stop) {
                c0 += al * T * p2.z;
                c1 += al * T * p2.w;
                c2 += al * T * p3.x;
                T = Tn;
            }
            if (stop) live = false;
            return stop;
        };
        float gc0[kR], gc1[kR], gc2[kR], ga[kR], Ts[kR];
        int kstop[kR];  // fitted depth slot where each pixel stopped
        {
            float tg0[kR], tg1[kR], tg2[kR], tga[kR];
            {  // the originals: the target
                float T[kR], c0[kR], c1[kR], c2[kR];
                bool live[kR];
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    T[r] = 1.0f;
                    c0[r] = c1[r] = c2[r] = 0.0f;
                    live[r] = true;
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    uint64_t m = uo[h];
                    while (m) {
                        bool any = false;
#pragma unroll
                        for (int r = 0; r < kR; ++r) any |= live[r];
                        if (__ballot(any) == 0) break;
                        const int k = __builtin_ctzll(m);
                        m &= m - 1;
                        const float4 p1 = sh.sp1[h * kWave + k], p2 = sh.sp2[h * kWave + k], p3 = sh.sp3[h * kWave + k];
#pragma unroll
                        for (int r = 0; r < kR; ++r)
                            if ((mo[r][h] >> k) & 1ull) blend(p1, p2, p3, yc[r], T[r], c0[r], c1[r], c2[r], live[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    tg0[r] = c0[r];
                    tg1[r] = c1[r];
                    tg2[r] = c2[r];
                    tga[r] = 1.0f - T[r];
                }
            }
            {  // the fitted splats
                float T[kR], c0[kR], c1[kR], c2[kR];
                bool live[kR];
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    T[r] = 1.0f;
                    c0[r] = c1[r] = c2[r] = 0.0f;
                    live[r] = true;
                    kstop[r] = n_s;
                }
                uint64_t m = us;
                while (m) {
                    bool any = false;
#pragma unroll
                    for (int r = 0; r < kR; ++r) any |= live[r];
                    if (__ballot(any) == 0) break;
                    const int k = __builtin_ctzll(m);
                    m &= m - 1;
                    const float4 p1 = sh.sp1[kLsMaxO + k], p2 = sh.sp2[kLsMaxO + k], p3 = sh.sp3[kLsMaxO + k];
#pragma unroll
                    for (int r = 0; r < kR; ++r)
                        if (((ms[r] >> k) & 1ull) && blend(p1, p2, p3, yc[r], T[r], c0[r], c1[r], c2[r], live[r]))
                            kstop[r] = k;
                }
#pragma unroll
                for (int r = 0; r < kR; ++r) {  // loss and the gradients of its L1 terms
                    const float d[3] = {c0[r] - tg0[r], c1[r] - tg1[r], c2[r] - tg2[r]};
                    float g[3];
                    for (int a = 0; a < 3; ++a) {
                        g[a] = d[a] > 0.0f ? wr : (d[a] < 0.0f ? -wr : 0.0f);
                        lsum += fabsf(d[a]) * wr;
                    }
                    gc0[r] = g[0];
                    gc1[r] = g[1];
                    gc2[r] = g[2];
                    const float dfa = (1.0f - T[r]) - tga[r];
                    ga[r] = dfa > 0.0f ? wa : (dfa < 0.0f ? -wa : 0.0f);
                    lsum += fabsf(dfa) * wa;
                    Ts[r] = T[r];
                }
            }
        }
        // back-to-front over the fitted splats the rows reach, up to the last
        // slot any pixel of the wavefront blended
        int kmax = kstop[0];
#pragma unroll
        for (int r = 1; r < kR; ++r) kmax = max(kmax, kstop[r]);
        for (int o = kWave / 2; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, kWave));
        {
            float Tc[kR], B0[kR], B1[kR], B2[kR];
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                Tc[r] = Ts[r];
                B0[r] = B1[r] = B2[r] = 0.0f;
            }
            uint64_t m = kmax >= kWave ? us : (us & ((1ull << kmax) - 1ull));
            while (m) {
                const int k = 63 - __builtin_clzll(m);
                m &= ~(1ull << k);
                const float4 p1 = sh.sp1[kLsMaxO + k], p2 = sh.sp2[kLsMaxO + k], p3 = sh.sp3[kLsMaxO + k];
                const float u = p1.x, ca = p1.z, cb = p1.w, cc = p2.x, op = p2.y, q0 = p2.z, q1 = p2.w, q2 = p3.x;
                float s9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                bool any_added = false;
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    if (!((ms[r] >> k) & 1ull)) continue;
                    const float dx = u - xc, dy = p1.y - yc[r];
                    const float raw = -0.5f * (ca * dx * dx + cc * dy * dy) - cb * dx * dy;
                    const float G = __expf(fminf(0.0f, raw));
                    const float ao = op * G;
                    const float al = fminf(0.99f, ao);
                    const bool added = k < kstop[r] && al >= 1.0f / 255.0f;
                    if (added) {
                        const float Tk = Tc[r] / (1.0f - al);
                        const float cg = q0 * gc0[r] + q1 * gc1[r] + q2 * gc2[r];
                        const float bg = B0[r] * gc0[r] + B1[r] * gc1[r] + B2[r] * gc2[r];
                        const float dal = Tk * cg - bg / (1.0f - al) + ga[r] * Ts[r] / (1.0f - al);
                        s9[6] += al * Tk * gc0[r];
                        s9[7] += al * Tk * gc1[r];
                        s9[8] += al * Tk * gc2[r];
                        B0[r] += q0 * al * Tk;
                        B1[r] += q1 * al * Tk;
                        B2[r] += q2 * al * Tk;
                        Tc[r] = Tk;
                        if (ao < 0.99f) {
                            s9[5] += dal * G;
                            const float dpw = raw < 0.0f ? dal * al : 0.0f;
                            s9[0] += -dpw * (ca * dx + cb * dy);
                            s9[1] += -dpw * (cb * dx + cc * dy);
                            s9[2] += -0.5f * dpw * dx * dx;
                            s9[3] += -dpw * dx * dy;
                            s9[4] += -0.5f * dpw * dy * dy;
                        }
                    }
                    any_added |= added;
                }
                if (__ballot(any_added) == 0) continue;
                for (int a = 0; a < 9; ++a) {
                    const float tot = wave_total(s9[a]);
                    if (lane == k) acc9[a] += tot;
                }
            }
        }
        if (lane < n_s)
            for (int a = 0; a < 9; ++a) sh.acc[wid][js][a] = acc9[a];
        const float lw = wave_sum(lsum);
        if (lane == 0) sh.red[wid] = lw;
        __syncthreads();
        if (losses && t == 0) {
            float l = 0.0f;
            for (int w = 0; w < kLsThreads / kWave; ++w) l += sh.red[w];
            losses[(uint64_t)g * iters + it] = l;
        }
        // chain rule and Adam step, one thread per fitted Gaussian
        if ((uint32_t)t < ns) {
            const int k = t, i = kLsMaxO + k;
            float gd[9];
            for (int a = 0; a < 9; ++a) {  // over the wavefronts in order
                gd[a] = 0.0f;
                for (int w = 0; w < kLsThreads / kWave; ++w) {
                    gd[a] += sh.acc[w][k][a];
                    sh.acc[w][k][a] = 0.0f;
                }
            }
            float gp[kLsP];
            for (int a = 0; a < kLsP; ++a) gp[a] = 0.0f;
            const float op = sh.pop[i];
            gp[10] = gd[5] * op * (1.0f - op);
            for (int a = 0; a < 3; ++a) gp[11 + a] = (kLsC0 * sh.prm[k][11 + a] + 0.5f > 0.0f) ? kLsC0 * gd[6 + a] : 0.0f;
            if (sh.pvalid[i]) {
                constexpr float f = 123.93546707863734f;
                const float *cam = sh.cam;
                const float dp[3] = {sh.prm[k][0] - cam[9], sh.prm[k][1] - cam[10], sh.prm[k][2] - cam[11]};
                float pc[3];
                for (int r = 0; r < 3; ++r) pc[r] = cam[3 * r] * dp[0] + cam[3 * r + 1] * dp[1] + cam[3 * r + 2] * dp[2];
                const float z = pc[2];
                const float lim = 1.3f * 32.0f / f;
                const float rx = pc[0] / z, ry = pc[1] / z;
                const bool clx = rx < -lim || rx > lim, cly = ry < -lim || ry > lim;
                const float tx = fminf(fmaxf(rx, -lim), lim) * z, ty = fminf(fmaxf(ry, -lim), lim) * z;
                const float J[2][3] = {{f / z, 0.0f, -f * tx / (z * z)}, {0.0f, f / z, -f * ty / (z * z)}};
                float T[2][3];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 3; ++c) T[r][c] = J[r][0] * cam[c] + J[r][1] * cam[3 + c] + J[r][2] * cam[6 + c];
                const float *qr = &sh.prm[k][6];
                const float qn = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
                const float w = qr[0] / qn, x = qr[1] / qn, y = qr[2] / qn, zq = qr[3] / qn;
                const float R[3][3] = {{1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)},
                                       {2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)},
                                       {2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)}};
                float s[3], M[3][3], S3[3][3];
                for (int a = 0; a < 3; ++a) s[a] = __expf(sh.prm[k][3 + a]);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) M[r][c] = R[r][c] * s[c];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) S3[r][c] = M[r][0] * M[c][0] + M[r][1] * M[c][1] + M[r][2] * M[c][2];
                // conic -> Sigma2 = [[a, b], [b, c]] (b read once, as Sigma2[0][1])
                float TS[2][3];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 3; ++c) TS[r][c] = T[r][0] * S3[0][c] + T[r][1] * S3[1][c] + T[r][2] * S3[2][c];
                const float a2 = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2];
                const float b2 = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
                const float c2 = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2];
                const float det = a2 * c2 - b2 * b2, id2 = 1.0f / (det * det);
                const float dca = gd[2], dcb = gd[3], dcc = gd[4];
                const float da = (-c2 * c2 * dca + b2 * c2 * dcb - b2 * b2 * dcc) * id2;
                const float db = (2.0f * b2 * c2 * dca - (det + 2.0f * b2 * b2) * dcb + 2.0f * a2 * b2 * dcc) * id2;
                const float dc = (-b2 * b2 * dca + a2 * b2 * dcb - a2 * a2 * dcc) * id2;
                const float G2[2][2] = {{da, db}, {0.0f, dc}};
                const float Gs[2][2] = {{2.0f * da, db}, {db, 2.0f * dc}};  // G2 + G2^T
                // dL/dS3 = T^T G2 T ; dL/dT = (G2 + G2^T) T S3
                float G3[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        float acc = 0.0f;
                        for (int m = 0; m < 2; ++m)
                            for (int nn = 0; nn < 2; ++nn) acc += T[m][r] * G2[m][nn] * T[nn][c];
                        G3[r][c] = acc;
                    }
                float dT[2][3];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 3; ++c) dT[r][c] = Gs[r][0] * TS[0][c] + Gs[r][1] * TS[1][c];
                // dL/dJ = dL/dT Rv^T
                float dJ[2][3];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 3; ++c) dJ[r][c] = dT[r][0] * cam[3 * c] + dT[r][1] * cam[3 * c + 1] + dT[r][2] * cam[3 * c + 2];
                // camera-space point: through J and through (u, v)
                float dpc[3] = {0.0f, 0.0f, 0.0f};
                dpc[0] += gd[0] * f / z;
                dpc[1] += gd[1] * f / z;
                dpc[2] += -gd[0] * f * pc[0] / (z * z) - gd[1] * f * pc[1] / (z * z);
                dpc[2] += -(dJ[0][0] + dJ[1][1]) * f / (z * z);
                if (!clx) {
                    dpc[0] += -dJ[0][2] * f / (z * z);
                    dpc[2] += dJ[0][2] * 2.0f * f * pc[0] / (z * z * z);
                } else {
                    dpc[2] += dJ[0][2] * f * (tx / z) / (z * z);
                }
                if (!cly) {
                    dpc[1] += -dJ[1][2] * f / (z * z);
                    dpc[2] += dJ[1][2] * 2.0f * f * pc[1] / (z * z * z);
                } else {
                    dpc[2] += dJ[1][2] * f * (ty / z) / (z * z);
                }
                for (int a = 0; a < 3; ++a) gp[a] = cam[a] * dpc[0] + cam[3 + a] * dpc[1] + cam[6 + a] * dpc[2];
                // S3 = M M^T: dL/dM = (G3 + G3^T) M
                float dM[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        dM[r][c] = (G3[r][0] + G3[0][r]) * M[0][c] + (G3[r][1] + G3[1][r]) * M[1][c] +
                                   (G3[r][2] + G3[2][r]) * M[2][c];
                float dR[3][3];
                for (int c = 0; c < 3; ++c) {
                    const float ds = dM[0][c] * R[0][c] + dM[1][c] * R[1][c] + dM[2][c] * R[2][c];
                    gp[3 + c] = ds * s[c];
                    for (int r = 0; r < 3; ++r) dR[r][c] = dM[r][c] * s[c];
                }
                const float gw = 2.0f * (-zq * dR[0][1] + y * dR[0][2] + zq * dR[1][0] - x * dR[1][2] - y * dR[2][0] +
                                         x * dR[2][1]);
                const float gx = 2.0f * (y * dR[0][1] + zq * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] -
                                         w * dR[1][2] + zq * dR[2][0] + w * dR[2][1] - 2.0f * x * dR[2][2]);
                const float gy = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] +
                                         zq * dR[1][2] - w * dR[2][0] + zq * dR[2][1] - 2.0f * y * dR[2][2]);
                const float gz = 2.0f * (-2.0f * zq * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] -
                                         2.0f * zq * dR[1][1] + y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
                const float dot = w * gw + x * gx + y * gy + zq * gz;
                gp[6] = (gw - w * dot) / qn;
                gp[7] = (gx - x * dot) / qn;
                gp[8] = (gy - y * dot) / qn;
                gp[9] = (gz - zq * dot) / qn;
            }
            if (grad_first && it == 0)
                for (int a = 0; a < kLsP; ++a) grad_first[(uint64_t)kLsP * (sf + k) + a] = gp[a];
            const float b1t = 1.0f - powf(0.9f, (float)(it + 1)), b2t = 1.0f - powf(0.999f, (float)(it + 1));
            for (int a = 0; a < kLsP; ++a) {
                const float lr = a < 3 ? 1.6e-5f : (a < 6 ? 5e-3f : (a < 10 ? 1e-3f : (a == 10 ? 5e-2f : 2.5e-3f)));
                sh.m1[k][a] = 0.9f * sh.m1[k][a] + 0.1f * gp[a];
                sh.m2[k][a] = 0.999f * sh.m2[k][a] + 0.001f * gp[a] * gp[a];
                sh.prm[k][a] -= lr * (sh.m1[k][a] / b1t) / (sqrtf(sh.m2[k][a] / b2t) + 1e-15f);
            }
        }
        __syncthreads();
    }
    // fitted rows back
    if ((uint32_t)t < ns) {
        const int k = t;
        const uint64_t r = sf + k;
        for (int a = 0; a < 3; ++a) {
            spos[3 * r + a] = sh.prm[k][a];
            sscale[3 * r + a] = __expf(sh.prm[k][3 + a]);
            sdc[(uint64_t)sdc_stride * r + a] = sh.prm[k][11 + a];
        }
        const float *qr = &sh.prm[k][6];
        const float qn = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
        for (int a = 0; a < 4; ++a) srot[4 * r + a] = qr[a] / qn;
        sopacity[r] = ls_sigmoid(sh.prm[k][10]);
    }
}

void launch_local_splat(hipStream_t st, const uint32_t *ofirst, const uint32_t *ocount, const uint32_t *sfirst,
                        const uint32_t *scount, const float *sphere, const float *opos, const float *oscale,
                        const float *orot, const float *oopacity, const float *odc, uint32_t odc_stride,
                        const uint32_t *orows, float *spos,
                        float *sscale, float *srot, float *sopacity, float *sdc, uint32_t sdc_stride,
                        const float *dirs, uint32_t iters, uint32_t n_groups, float *losses, float *grad_first,
                        uint32_t *err)
{
    if (n_groups == 0) return;
    hipLaunchKernelGGL(local_splat_kernel, dim3(n_groups), dim3(kLsThreads), 0, st, ofirst, ocount, sfirst, scount,
                       sphere, opos, oscale, orot, oopacity, odc, odc_stride, orows, spos, sscale, srot, sopacity, sdc,
                       sdc_stride, dirs, iters, n_groups, losses, grad_first, err);
}

}  // namespace v3dg
