// C ABI of v3dg: scene residency and validation, selection objects, the
// per-frame kernel chain, and stage timing.  Host code only; every step of the
// frame runs in the HIP kernels of select/project/sort/blend.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/v3dg.h"
#include "v3dg_internal.h"

using namespace v3dg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(x)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fail(V3DG_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dev_alloc(T **p, uint64_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(V3DG_ERR_OOM, "hipMalloc of %llu bytes failed: %s", (unsigned long long)(count * sizeof(T)),
                    hipGetErrorString(e));
    }
    return V3DG_OK;
}

template <class T>
void dev_free(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

bool finite_f(float v) { return std::isfinite(v); }

float round_up_f32(double x)
{
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

// IEEE binary32 -> binary16, round to nearest, ties to even (overflow -> inf)
uint16_t f32_to_half(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t sign = (u >> 16) & 0x8000u, ex = (u >> 23) & 0xffu, man = u & 0x7fffffu;
    if (ex == 0xffu) return (uint16_t)(sign | 0x7c00u | (man ? 0x200u : 0u));
    const int e = (int)ex - 127 + 15;
    if (e >= 31) return (uint16_t)(sign | 0x7c00u);
    if (e <= 0) {  // subnormal half (or zero): unit 2^-24
        if (e < -10) return (uint16_t)sign;
        const uint32_t m = man | 0x800000u;
        const int shift = 14 - e;
        const uint32_t rem = m & ((1u << shift) - 1u), half = 1u << (shift - 1);
        uint32_t hm = m >> shift;
        if (rem > half || (rem == half && (hm & 1u))) ++hm;
        return (uint16_t)(sign | hm);
    }
    uint32_t hm = ((uint32_t)e << 10) | (man >> 13);
    const uint32_t rem = man & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (hm & 1u))) ++hm;  // a carry moves into the exponent
    return (uint16_t)(sign | hm);
}

float half_to_f32(uint16_t h)
{
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16, ex = (h >> 10) & 0x1fu, man = h & 0x3ffu;
    uint32_t u;
    if (ex == 0x1fu) {
        u = sign | 0x7f800000u | (man << 13);
    } else if (ex == 0) {
        const float v = std::ldexp((float)man, -24);
        return sign ? -v : v;
    } else {
        u = sign | ((ex - 15 + 127) << 23) | (man << 13);
    }
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// IEEE binary32 -> bfloat16, round to nearest, ties to even (finite input)
uint16_t f32_to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if (std::isnan(f)) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

float bf16_to_f32(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

uint32_t bits_for(uint32_t n)  // ceil(log2(n)), 0 for n <= 1
{
    uint32_t b = 0;
    while ((1ull << b) < n) ++b;
    return b;
}

}  // namespace

struct ProfRec {
    int stage;
    hipEvent_t a, b;
};

struct v3dg_selection {
    v3dg_scene *scene = nullptr;
    uint64_t cap_tests = 0, cap_slots = 0, n_parts = 0;
    uint32_t *gid = nullptr;
    uint32_t *slot_off = nullptr;
    uint32_t *clear_block = nullptr;  // counters (kSelCounters u32) + look-back words
    uint32_t *counters = nullptr;
    uint64_t *status = nullptr;
    uint32_t *slot_row = nullptr;
    uint32_t *slot_inst = nullptr;
};

struct v3dg_scene {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t NC = 0, n_rows = 0, sh_degree = 0, n_inst = 0;
    uint64_t plane_stride = 0;
    uint32_t precision = V3DG_FP32;
    float *pos_planes = nullptr;  // 3 FP32 planes
    void *geo_planes = nullptr;   // 8 planes, FP32 or FP16
    void *sh_planes = nullptr;    // 3 (d+1)^2 planes, FP32, BF16 or FP16
    float4 *self_sph = nullptr, *par_sph = nullptr;
    uint2 *rowinfo = nullptr;
    double *T_dev = nullptr;
    float *scale_dev = nullptr;
    InstRec *itab = nullptr;
    uint64_t maxcut_rows = 0;
    std::vector<uint32_t> leaf_ids;
    std::vector<uint32_t> h_count;
    // render workspace
    uint64_t cap_slots = 0;
    float4 *splat = nullptr;
    BinRec *bin = nullptr;
    float *depth = nullptr;
    uint2 *rect = nullptr;
    uint32_t *tiles = nullptr;
    uint32_t *offsets = nullptr;
    uint32_t *dkey[2] = {nullptr, nullptr};
    uint32_t *dval[2] = {nullptr, nullptr};
    int sort_mode = V3DG_SORT_DEPTH_FIRST;
    uint32_t *rclear = nullptr;  // counters + scan look-back + tile ranges, cleared every frame
    uint64_t rclear_words = 0;
    uint64_t scan_parts = 0;
    uint32_t tiles_cap = 0;
    uint32_t *rcounters = nullptr;
    uint64_t *scan_status = nullptr;
    uint2 *ranges = nullptr;
    uint64_t cap_keys = 0;
    uint64_t *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    uint64_t *sort_status = nullptr;
    uint64_t sort_status_parts = 0;
    uint32_t *cbase = nullptr;     // per tile: first chunk of a long list
    uint2 *items = nullptr;        // (tile, chunk) work items
    float4 *scratch = nullptr;     // per chunk, per pixel (C, T)
    uint32_t *pend = nullptr;      // per long tile, per pixel: chunk to walk again
    uint32_t *need = nullptr;      // per chunk: walk it again
    uint2 *rewalk = nullptr;       // (tile, chunk) to walk again
    uint64_t cap_chunks = 0;
    uint32_t epoch = 0;
    uint32_t *pinned = nullptr;
    v3dg_frame_stats last{};
    int last_buf = 0;
    v3dg_selection *full = nullptr;
    bool profiling = false;
    v3dg_profile acc{};
    unsigned long long *pairs_dev = nullptr;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
};

namespace {

// ---- profiling --------------------------------------------------------------
struct Stage {
    v3dg_scene *s;
    int stage;
    hipEvent_t b = nullptr;
    Stage(v3dg_scene *sc, int st) : s(sc), stage(st)
    {
        if (!s->profiling) return;
        hipEvent_t a = take();
        b = take();
        (void)hipEventRecord(a, s->stream);
        s->prof.push_back({stage, a, b});
    }
    ~Stage()
    {
        if (b) (void)hipEventRecord(b, s->stream);
    }
    hipEvent_t take()
    {
        if (!s->ev_pool.empty()) {
            hipEvent_t e = s->ev_pool.back();
            s->ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
};

// ---- camera -----------------------------------------------------------------
int make_cam(const v3dg_camera *c, CamArgs *o)
{
    if (!c) return fail(V3DG_ERR_INVALID_ARG, "camera is NULL");
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(V3DG_ERR_INVALID_ARG, "camera size %ux%u outside 1..16384", c->width, c->height);
    const float sc[] = {c->fx, c->fy, c->cx, c->cy, c->near_plane, c->far_plane, c->bg[0], c->bg[1], c->bg[2]};
    for (float v : sc)
        if (!finite_f(v)) return fail(V3DG_ERR_INVALID_ARG, "camera has a non-finite value");
    for (int i = 0; i < 12; ++i)
        if (!finite_f(c->world_to_cam[i])) return fail(V3DG_ERR_INVALID_ARG, "camera matrix has a non-finite value");
    if (!(c->fx > 0.f) || !(c->fy > 0.f)) return fail(V3DG_ERR_INVALID_ARG, "focal lengths must be > 0");
    if (!(c->near_plane > 0.f) || !(c->far_plane > c->near_plane))
        return fail(V3DG_ERR_INVALID_ARG, "need 0 < near_plane < far_plane");
    std::memset(o, 0, sizeof(*o));
    std::memcpy(o->V, c->world_to_cam, sizeof(o->V));
    const float *V = c->world_to_cam;
    for (int k = 0; k < 3; ++k)
        o->cw[k] = -((double)V[0 * 4 + k] * V[0 * 4 + 3] + (double)V[1 * 4 + k] * V[1 * 4 + 3] +
                     (double)V[2 * 4 + k] * V[2 * 4 + 3]);
    o->fx = c->fx;
    o->fy = c->fy;
    o->cx = c->cx;
    o->cy = c->cy;
    o->near_plane = c->near_plane;
    o->far_plane = c->far_plane;
    o->limx = (float)(1.3 * (0.5 * (double)c->width / (double)c->fx));
    o->limy = (float)(1.3 * (0.5 * (double)c->height / (double)c->fy));
    for (int k = 0; k < 3; ++k) o->bg[k] = c->bg[k];
    o->width = c->width;
    o->height = c->height;
    o->tiles_x = (c->width + kTile - 1) / kTile;
    o->tiles_y = (c->height + kTile - 1) / kTile;
    return V3DG_OK;
}

float footprint_K(const v3dg_camera *c)
{
    double k = 3.14159265358979323846 * (double)c->fx;
    k = k * (double)c->fy;
    return (float)k;
}

// ---- instances ----------------------------------------------------------------
int check_instances(const double *T, uint32_t n, std::vector<float> &scale)
{
    if (!T || n == 0) return fail(V3DG_ERR_INVALID_ARG, "need at least one instance");
    scale.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const double *t = T + 12 * (size_t)i;
        for (int j = 0; j < 12; ++j)
            if (!std::isfinite(t[j])) return fail(V3DG_ERR_INVALID_ARG, "instance %u has a non-finite entry", i);
        double s2 = t[0] * t[0];
        s2 = s2 + t[4] * t[4];
        s2 = s2 + t[8] * t[8];
        const double s = std::sqrt(s2);
        if (!(s > 0)) return fail(V3DG_ERR_INVALID_ARG, "instance %u has zero scale", i);
        // columns orthogonal with equal length s: a similarity s R
        const double m[9] = {t[0], t[1], t[2], t[4], t[5], t[6], t[8], t[9], t[10]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = m[0 * 3 + a] * m[0 * 3 + b] + m[1 * 3 + a] * m[1 * 3 + b] + m[2 * 3 + a] * m[2 * 3 + b];
                double want = (a == b) ? s2 : 0.0;
                if (std::fabs(d - want) > 1e-6 * s2)
                    return fail(V3DG_ERR_INVALID_ARG, "instance %u is not a rotation with a uniform scale", i);
            }
        const double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                           m[2] * (m[3] * m[7] - m[4] * m[6]);
        if (!(det > 0)) return fail(V3DG_ERR_INVALID_ARG, "instance %u is a reflection", i);
        scale[i] = (float)s;
    }
    return V3DG_OK;
}

// ---- selection objects ------------------------------------------------------------
void sel_release(v3dg_selection *s)
{
    if (!s) return;
    dev_free(s->gid);
    dev_free(s->slot_off);
    dev_free(s->clear_block);
    dev_free(s->slot_row);
    dev_free(s->slot_inst);
    s->counters = nullptr;
    s->status = nullptr;
}

int sel_alloc(v3dg_scene *sc, v3dg_selection *s)
{
    s->scene = sc;
    s->cap_tests = (uint64_t)sc->NC * sc->n_inst;
    s->cap_slots = sc->cap_slots;
    s->n_parts = (s->cap_tests + kSelPart - 1) / kSelPart;
    int rc;
    if ((rc = dev_alloc(&s->gid, s->cap_tests))) return rc;
    if ((rc = dev_alloc(&s->slot_off, s->cap_tests))) return rc;
    if ((rc = dev_alloc(&s->clear_block, (uint64_t)kSelCounters + 2 * s->n_parts))) return rc;
    s->counters = s->clear_block;
    s->status = reinterpret_cast<uint64_t *>(s->clear_block + kSelCounters);
    if ((rc = dev_alloc(&s->slot_row, s->cap_slots))) return rc;
    if ((rc = dev_alloc(&s->slot_inst, s->cap_slots))) return rc;
    HIP_TRY(hipMemsetAsync(s->clear_block, 0, sizeof(uint32_t) * kSelCounters, sc->stream));
    return V3DG_OK;
}

// ---- render workspace ----------------------------------------------------------------
int ensure_status(v3dg_scene *s, uint64_t parts);

int ensure_slots(v3dg_scene *s)
{
    if (s->splat) return V3DG_OK;
    const uint64_t n = s->cap_slots;
    int rc;
    if ((rc = dev_alloc(&s->splat, 3 * n))) return rc;
    if ((rc = dev_alloc(&s->bin, n))) return rc;
    if ((rc = dev_alloc(&s->depth, n))) return rc;
    if ((rc = dev_alloc(&s->rect, n))) return rc;
    if ((rc = dev_alloc(&s->tiles, n))) return rc;
    if ((rc = dev_alloc(&s->offsets, n))) return rc;
    for (int b = 0; b < 2; ++b) {
        if ((rc = dev_alloc(&s->dkey[b], n))) return rc;
        if ((rc = dev_alloc(&s->dval[b], n))) return rc;
    }
    s->scan_parts = (n + kScanPart - 1) / kScanPart;
    if ((rc = ensure_status(s, (n + kSortPart - 1) / kSortPart))) return rc;
    return V3DG_OK;
}

int ensure_tiles(v3dg_scene *s, uint32_t n_tiles)
{
    if (s->rclear && n_tiles <= s->tiles_cap) return V3DG_OK;
    dev_free(s->rclear);
    s->tiles_cap = std::max<uint32_t>(n_tiles, 8160);
    s->rclear_words = (uint64_t)kRenCounters + 2 * s->scan_parts + 2ull * s->tiles_cap;
    int rc;
    if ((rc = dev_alloc(&s->rclear, s->rclear_words))) return rc;
    s->rcounters = s->rclear;
    s->scan_status = reinterpret_cast<uint64_t *>(s->rclear + kRenCounters);
    s->ranges = reinterpret_cast<uint2 *>(s->rclear + kRenCounters + 2 * s->scan_parts);
    dev_free(s->cbase);
    if ((rc = dev_alloc(&s->cbase, s->tiles_cap))) return rc;
    return V3DG_OK;
}

int ensure_status(v3dg_scene *s, uint64_t parts)
{
    if (parts <= s->sort_status_parts) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    dev_free(s->sort_status);
    const uint64_t np = std::max<uint64_t>(parts + parts / 2, 256);
    int rc;
    if ((rc = dev_alloc(&s->sort_status, np * kRadix))) return rc;
    HIP_TRY(hipMemsetAsync(s->sort_status, 0, np * kRadix * sizeof(uint64_t), s->stream));
    s->sort_status_parts = np;
    s->epoch = 0;
    return V3DG_OK;
}

int ensure_chunks(v3dg_scene *s, uint64_t K, uint32_t n_tiles)
{
    const uint64_t need = (K + kChunk - 1) / kChunk + n_tiles;
    if (need <= s->cap_chunks) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    dev_free(s->items);
    dev_free(s->scratch);
    dev_free(s->pend);
    dev_free(s->need);
    dev_free(s->rewalk);
    const uint64_t cap = need + need / 2;
    int rc;
    if ((rc = dev_alloc(&s->items, cap))) return rc;
    if ((rc = dev_alloc(&s->scratch, cap * 256))) return rc;
    if ((rc = dev_alloc(&s->pend, cap * 256))) return rc;
    if ((rc = dev_alloc(&s->need, cap))) return rc;
    if ((rc = dev_alloc(&s->rewalk, cap))) return rc;
    s->cap_chunks = cap;
    return V3DG_OK;
}

int ensure_keys(v3dg_scene *s, uint64_t K)
{
    const uint64_t parts = (K + kSortPart - 1) / kSortPart;
    if (K > s->cap_keys) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (int b = 0; b < 2; ++b) {
            dev_free(s->keys[b]);
            dev_free(s->vals[b]);
        }
        uint64_t cap = std::max<uint64_t>(K + K / 2, 1u << 20);
        cap = std::min<uint64_t>(cap, 0xffffffffull);
        int rc;
        for (int b = 0; b < 2; ++b) {
            if ((rc = dev_alloc(&s->keys[b], cap))) return rc;
            if ((rc = dev_alloc(&s->vals[b], cap))) return rc;
        }
        s->cap_keys = cap;
    }
    return ensure_status(s, parts);
}

uint32_t next_epoch(v3dg_scene *s)
{
    if (++s->epoch >= (1u << 30)) {  // wrap: old words could alias new epochs
        (void)hipMemsetAsync(s->sort_status, 0, s->sort_status_parts * kRadix * sizeof(uint64_t), s->stream);
        s->epoch = 1;
    }
    return s->epoch;
}

// Stable sort of K (key, value) pairs held in buffer 0 by the low key_bits
// bits of the keys; *out_buf receives the buffer index holding the result.
template <typename KT>
int run_sort(v3dg_scene *s, KT *const kb[2], uint32_t *const vb[2], uint64_t K, uint32_t key_bits, int *out_buf,
             uint32_t *passes_out, bool have_hist)
{
    const int passes = (int)((key_bits + kRadixBits - 1) / kRadixBits);
    *passes_out = (uint32_t)passes;
    int cur = 0;
    if (!have_hist) {
        Stage st(s, V3DG_STAGE_SORT_HIST);
        launch_sort_hist<KT>(s->stream, kb[0], K, passes, s->rcounters + kRenHist);
    }
    for (int p = 0; p < passes; ++p) {
        Stage st(s, V3DG_STAGE_SORT_PASS);
        launch_sort_pass<KT>(s->stream, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], K, p, s->rcounters + kRenHist,
                             s->sort_status, next_epoch(s), s->rcounters + kRenTicketSort + p, s->rcounters + kRenErr);
        cur ^= 1;
    }
    *out_buf = cur;
    return V3DG_OK;
}

int render_impl(v3dg_scene *s, const v3dg_camera *c, const v3dg_selection *sel, float *image)
{
    CamArgs cam;
    int rc = make_cam(c, &cam);
    if (rc) return rc;
    if (!sel || sel->scene != s) return fail(V3DG_ERR_INVALID_ARG, "selection does not belong to this scene");
    if (!image) return fail(V3DG_ERR_INVALID_ARG, "image is NULL");
    HIP_TRY(hipSetDevice(s->device));
    if ((rc = ensure_slots(s))) return rc;
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    if ((rc = ensure_tiles(s, n_tiles))) return rc;
    {
        Stage st(s, V3DG_STAGE_SETUP);
        launch_frame_setup(s->stream, cam, s->T_dev, s->scale_dev, s->n_inst, s->itab, s->rclear,
                           (uint64_t)kRenCounters + 2 * s->scan_parts + 2ull * n_tiles);
    }
    const uint32_t *n_dev = sel->counters + kSelNGaussians;
    ProjectOut po{s->splat, s->depth, s->bin, s->rect, s->tiles, s->dkey[0], s->dval[0]};
    {
        Stage st(s, V3DG_STAGE_PROJECT);
        const Attribs attr{s->pos_planes, s->geo_planes, s->sh_planes, s->plane_stride};
        launch_project(s->stream, cam, attr, (int)s->precision, (int)s->sh_degree, sel->slot_row, sel->slot_inst,
                       n_dev, s->cap_slots, s->itab, po);
    }
    const bool depth_first = s->sort_mode == V3DG_SORT_DEPTH_FIRST;
    if (depth_first) {
        // stable sort of the slots by FP32 depth bits (culled slots last), on
        // the device-side slot count
        {
            Stage st(s, V3DG_STAGE_DEPTH_SORT);
            launch_sort_hist_dev(s->stream, s->dkey[0], n_dev, s->cap_slots, 4, s->rcounters + kRenHistDepth);
        }
        int cur = 0;
        for (int p = 0; p < 4; ++p) {
            Stage st(s, V3DG_STAGE_DEPTH_SORT);
            launch_sort_pass_dev(s->stream, s->dkey[cur], s->dval[cur], s->dkey[cur ^ 1], s->dval[cur ^ 1], n_dev,
                                 s->cap_slots, p, s->rcounters + kRenHistDepth, s->sort_status, next_epoch(s),
                                 s->rcounters + kRenTicketDepth + p, s->rcounters + kRenErr);
            cur ^= 1;
        }
    }
    {
        Stage st(s, V3DG_STAGE_SCAN);
        launch_scan_tiles(s->stream, s->tiles, depth_first ? s->dval[0] : nullptr, n_dev, s->cap_slots, s->offsets,
                          s->scan_status, s->rcounters);
    }
    // one wait per frame: slot and key counts decide the launch sizes below
    HIP_TRY(hipMemcpyAsync(s->pinned, s->rcounters, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(s->pinned + 8, sel->counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const uint32_t err = s->pinned[kRenErr] | s->pinned[8 + kSelErr];
    const uint64_t K = (uint64_t)s->pinned[kRenKeysLo] | ((uint64_t)s->pinned[kRenKeysHi] << 32);
    const uint32_t N = s->pinned[8 + kSelNGaussians];
    const uint32_t n_visible = s->pinned[kRenVisible];
    const uint32_t n_sel_clusters = s->pinned[8 + kSelNClusters];
    if (err & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    if ((err & kErrOverflow) || K >= 0xffffffffull)
        return fail(V3DG_ERR_CAPACITY, "frame needs %llu keys; the limit is 2^32-1", (unsigned long long)K);
    if ((rc = ensure_keys(s, K))) return rc;
    if ((rc = ensure_chunks(s, K, n_tiles))) return rc;
    const uint32_t tile_bits = std::max<uint32_t>(bits_for(n_tiles), 1);
    int buf = 0;
    uint32_t passes = 0;
    uint32_t key_bits;
    if (depth_first) {
        uint32_t *kb[2] = {reinterpret_cast<uint32_t *>(s->keys[0]), reinterpret_cast<uint32_t *>(s->keys[1])};
        key_bits = tile_bits;
        const int tpasses = (int)((key_bits + kRadixBits - 1) / kRadixBits);
        {
            Stage st(s, V3DG_STAGE_EMIT);
            launch_emit32(s->stream, N, s->dval[0], s->tiles, s->offsets, s->rect, s->bin, cam.tiles_x, s->cap_keys,
                          tpasses, kb[0], s->vals[0], s->rcounters + kRenHist, s->rcounters + kRenErr);
        }
        if (K > 0) run_sort<uint32_t>(s, kb, s->vals, K, key_bits, &buf, &passes, true);
        {
            Stage st(s, V3DG_STAGE_RANGES);
            launch_tile_ranges<uint32_t>(s->stream, kb[buf], K, 0, n_tiles, s->ranges);
        }
    } else {
        {
            Stage st(s, V3DG_STAGE_EMIT);
            launch_emit64(s->stream, N, s->tiles, s->offsets, s->rect, s->bin, cam.tiles_x, s->cap_keys, s->keys[0],
                          s->vals[0], s->rcounters + kRenErr);
        }
        key_bits = 32 + tile_bits;
        if (K > 0) run_sort<uint64_t>(s, s->keys, s->vals, K, key_bits, &buf, &passes, false);
        {
            Stage st(s, V3DG_STAGE_RANGES);
            launch_tile_ranges<uint64_t>(s->stream, s->keys[buf], K, 32, n_tiles, s->ranges);
        }
    }
    {
        Stage st(s, V3DG_STAGE_BLEND);
        launch_blend(s->stream, cam, s->splat, s->vals[buf], s->ranges, s->cbase, s->items, s->rcounters,
                     K / kChunk, K / kChunk + n_tiles, s->scratch, s->pend, s->need, s->rewalk, image, s->pairs_dev);
    }
    HIP_TRY(hipGetLastError());
    s->acc.frames += 1;
    s->acc.sel_clusters += n_sel_clusters;
    s->acc.slots += N;
    s->acc.visible += n_visible;
    s->acc.keys += K;
    s->acc.tiles += n_tiles;
    s->acc.pixels += (uint64_t)cam.width * cam.height;
    s->acc.sort_passes += passes;
    if (depth_first) s->acc.depth_sorts += 1;
    s->last.n_slots = N;
    s->last.n_keys = K;
    s->last.n_tiles = n_tiles;
    s->last.key_bits = key_bits;
    s->last.sort_mode = (uint32_t)s->sort_mode;
    s->last.sort_passes = passes;
    s->last_buf = buf;
    return V3DG_OK;
}

int build_full_selection(v3dg_scene *s)
{
    if (s->full) return V3DG_OK;
    auto *sel = new (std::nothrow) v3dg_selection();
    if (!sel) return fail(V3DG_ERR_OOM, "host allocation failed");
    int rc = sel_alloc(s, sel);
    if (rc) {
        sel_release(sel);
        delete sel;
        return rc;
    }
    const uint64_t nl = s->leaf_ids.size();
    std::vector<uint32_t> gid(nl * s->n_inst), off(nl * s->n_inst);
    uint64_t acc = 0;
    for (uint32_t i = 0; i < s->n_inst; ++i)
        for (uint64_t j = 0; j < nl; ++j) {
            const uint64_t q = (uint64_t)i * nl + j;
            gid[q] = i * s->NC + s->leaf_ids[j];
            off[q] = (uint32_t)acc;
            acc += s->h_count[s->leaf_ids[j]];
        }
    uint32_t ctr[kSelCounters] = {0};
    ctr[kSelNClusters] = (uint32_t)gid.size();
    ctr[kSelNGaussians] = (uint32_t)acc;
    HIP_TRY(hipMemcpyAsync(sel->gid, gid.data(), gid.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(sel->slot_off, off.data(), off.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(sel->counters, ctr, sizeof(ctr), hipMemcpyHostToDevice, s->stream));
    launch_expand(s->stream, sel->gid, sel->slot_off, s->rowinfo, s->NC, sel->counters, (uint32_t)gid.size(),
                  sel->slot_row, sel->slot_inst);
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->full = sel;
    return V3DG_OK;
}

void scene_release(v3dg_scene *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->full) {
        sel_release(s->full);
        delete s->full;
        s->full = nullptr;
    }
    dev_free(s->pos_planes);
    dev_free(s->geo_planes);
    dev_free(s->sh_planes);
    dev_free(s->self_sph);
    dev_free(s->par_sph);
    dev_free(s->rowinfo);
    dev_free(s->T_dev);
    dev_free(s->scale_dev);
    dev_free(s->itab);
    dev_free(s->splat);
    dev_free(s->bin);
    dev_free(s->depth);
    for (int b = 0; b < 2; ++b) {
        dev_free(s->dkey[b]);
        dev_free(s->dval[b]);
    }
    dev_free(s->rect);
    dev_free(s->tiles);
    dev_free(s->offsets);
    dev_free(s->rclear);
    for (int b = 0; b < 2; ++b) {
        dev_free(s->keys[b]);
        dev_free(s->vals[b]);
    }
    dev_free(s->sort_status);
    dev_free(s->pairs_dev);
    dev_free(s->cbase);
    dev_free(s->items);
    dev_free(s->scratch);
    dev_free(s->pend);
    dev_free(s->need);
    dev_free(s->rewalk);
    if (s->pinned) (void)hipHostFree(s->pinned);
    s->pinned = nullptr;
    for (auto &r : s->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : s->ev_pool) (void)hipEventDestroy(e);
    s->prof.clear();
    s->ev_pool.clear();
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char *v3dg_last_error(void) { return g_err.c_str(); }

int v3dg_load_hierarchy(const v3dg_hierarchy_desc *d, const double *instances_3x4, uint32_t n_instances,
                        void *hip_stream, uint32_t flags, v3dg_scene **out)
{
    g_err.clear();
    if (!d || !out) return fail(V3DG_ERR_INVALID_ARG, "desc and out must be non-NULL");
    *out = nullptr;
    if (d->precision > V3DG_FP16) return fail(V3DG_ERR_INVALID_ARG, "unknown precision %u", d->precision);
    if (d->sh_degree > 3) return fail(V3DG_ERR_INVALID_ARG, "sh_degree %u > 3", d->sh_degree);
    if (d->n_clusters < 1 || d->n_rows < 1) return fail(V3DG_ERR_INVALID_ARG, "empty hierarchy");
    if (!d->self_sphere || !d->parent_sphere || !d->first_row || !d->count || !d->parent || !d->first_child ||
        !d->n_children || !d->pos || !d->scale || !d->rot || !d->opacity || !d->sh)
        return fail(V3DG_ERR_INVALID_ARG, "a hierarchy array is NULL");
    if (flags & ~V3DG_LOAD_REPAIR_NESTING) return fail(V3DG_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const uint32_t NC = d->n_clusters, NR = d->n_rows;
    std::vector<float> inst_scale;
    int rc = check_instances(instances_3x4, n_instances, inst_scale);
    if (rc) return rc;
    if ((uint64_t)NC * n_instances >= (1ull << 26))
        return fail(V3DG_ERR_CAPACITY, "instances x clusters = %llu exceeds 2^26",
                    (unsigned long long)NC * n_instances);

    // ---- tree structure
    for (uint32_t k = 0; k < NC; ++k) {
        if (d->count[k] < 1 || d->count[k] > 64) return fail(V3DG_ERR_INVALID_ARG, "cluster %u has %u rows", k, d->count[k]);
        if ((uint64_t)d->first_row[k] + d->count[k] > NR)
            return fail(V3DG_ERR_INVALID_ARG, "cluster %u rows out of range", k);
        if (d->n_children[k] > 0) {
            const int64_t fc = d->first_child[k];
            if (fc < 0 || fc + d->n_children[k] > (int64_t)NC)
                return fail(V3DG_ERR_INVALID_ARG, "cluster %u children out of range", k);
            for (int c = 0; c < d->n_children[k]; ++c)
                if (d->parent[fc + c] != (int32_t)k)
                    return fail(V3DG_ERR_INVALID_ARG, "child %lld of cluster %u does not point back",
                                (long long)(fc + c), k);
        }
        if (d->parent[k] < -1 || d->parent[k] >= (int32_t)NC)
            return fail(V3DG_ERR_INVALID_ARG, "cluster %u parent out of range", k);
        if (d->parent[k] >= 0) {
            const int32_t p = d->parent[k];
            const int64_t fc = d->first_child[p];
            if (fc < 0 || (int64_t)k < fc || (int64_t)k >= fc + d->n_children[p])
                return fail(V3DG_ERR_INVALID_ARG, "cluster %u is not among its parent's children", k);
        }
    }
    // reachability from roots; depth order for repair and max-cut
    std::vector<uint32_t> order;
    order.reserve(NC);
    std::vector<uint8_t> seen(NC, 0);
    for (uint32_t k = 0; k < NC; ++k)
        if (d->parent[k] < 0) {
            order.push_back(k);
            seen[k] = 1;
        }
    for (size_t h = 0; h < order.size(); ++h) {
        const uint32_t k = order[h];
        for (int c = 0; c < d->n_children[k]; ++c) {
            const uint32_t ch = (uint32_t)(d->first_child[k] + c);
            if (seen[ch]) return fail(V3DG_ERR_INVALID_ARG, "cluster %u reached twice", ch);
            seen[ch] = 1;
            order.push_back(ch);
        }
    }
    if (order.size() != NC) return fail(V3DG_ERR_INVALID_ARG, "%zu clusters unreachable from a root", NC - order.size());

    // ---- spheres
    std::vector<float> self(d->self_sphere, d->self_sphere + 4 * (size_t)NC);
    std::vector<float> par(d->parent_sphere, d->parent_sphere + 4 * (size_t)NC);
    for (uint32_t k = 0; k < NC; ++k) {
        for (int j = 0; j < 3; ++j)
            if (!finite_f(self[4 * k + j]) || !finite_f(par[4 * k + j]))
                return fail(V3DG_ERR_INVALID_ARG, "cluster %u sphere centre not finite", k);
        const float r = self[4 * k + 3];
        if (d->n_children[k] == 0) {
            if (r != 0.0f) return fail(V3DG_ERR_INVALID_ARG, "leaf cluster %u must have radius 0", k);
        } else if (!(r > 0.0f) || !finite_f(r)) {
            return fail(V3DG_ERR_INVALID_ARG, "cluster %u radius must be finite and > 0", k);
        }
        if (d->parent[k] < 0) {
            if (!std::isinf(par[4 * k + 3]) || par[4 * k + 3] < 0)
                return fail(V3DG_ERR_INVALID_ARG, "root %u needs parent radius +inf", k);
        } else if (std::memcmp(&par[4 * k], &self[4 * (size_t)d->parent[k]], 16) != 0) {
            return fail(V3DG_ERR_INVALID_ARG, "parent_sphere[%u] differs from its parent's own sphere", k);
        }
    }
    for (size_t h = order.size(); h-- > 0;) {  // children before parents
        const uint32_t k = order[h];
        const int32_t p = d->parent[k];
        if (p < 0 || self[4 * k + 3] == 0.0f) continue;
        const double dx = (double)self[4 * p] - self[4 * k], dy = (double)self[4 * p + 1] - self[4 * k + 1],
                     dz = (double)self[4 * p + 2] - self[4 * k + 2];
        const double need = (std::sqrt(dx * dx + dy * dy + dz * dz) + (double)self[4 * k + 3]) * (1.0 + 1.0 / 4096.0);
        if ((double)self[4 * p + 3] < need) {
            if (!(flags & V3DG_LOAD_REPAIR_NESTING))
                return fail(V3DG_ERR_NOT_MONOTONE,
                            "sphere of cluster %d does not nest child %u (r_p = %.9g, needs >= %.9g)", p, k,
                            (double)self[4 * p + 3], need);
            self[4 * p + 3] = round_up_f32((std::sqrt(dx * dx + dy * dy + dz * dz) + (double)self[4 * k + 3]) *
                                               (1.0 + 1.0 / 1024.0) + 1e-6);
        }
    }
    for (uint32_t k = 0; k < NC; ++k)
        if (d->parent[k] >= 0) std::memcpy(&par[4 * k], &self[4 * (size_t)d->parent[k]], 16);

    // ---- Gaussian rows
    for (uint64_t r = 0; r < NR; ++r) {
        const float *q = d->rot + 4 * r;
        const double qn = std::sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
        if (!(std::fabs(qn - 1.0) <= 1e-6)) return fail(V3DG_ERR_INVALID_ARG, "row %llu quaternion not unit", (unsigned long long)r);
        for (int j = 0; j < 3; ++j) {
            if (!finite_f(d->pos[3 * r + j])) return fail(V3DG_ERR_INVALID_ARG, "row %llu position not finite", (unsigned long long)r);
            const float sv = d->scale[3 * r + j];
            if (!(sv > 0.0f) || !finite_f(sv)) return fail(V3DG_ERR_INVALID_ARG, "row %llu scale must be > 0", (unsigned long long)r);
        }
        const float o = d->opacity[r];
        if (!(o > 0.0f) || !(o <= 1.0f)) return fail(V3DG_ERR_INVALID_ARG, "row %llu opacity outside (0, 1]", (unsigned long long)r);
    }
    const int ncoef = (int)((d->sh_degree + 1) * (d->sh_degree + 1));
    for (uint64_t i = 0; i < (uint64_t)NR * ncoef * 3; ++i)
        if (!finite_f(d->sh[i])) return fail(V3DG_ERR_INVALID_ARG, "SH coefficient %llu not finite", (unsigned long long)i);
    // narrow storage: scale and opacity must survive the rounding, SH must stay finite
    if (d->precision != V3DG_FP32) {
        for (uint64_t r = 0; r < NR; ++r) {
            for (int j = 0; j < 3; ++j) {
                const float sv = half_to_f32(f32_to_half(d->scale[3 * r + j]));
                if (!(sv > 0.0f) || !finite_f(sv))
                    return fail(V3DG_ERR_INVALID_ARG, "row %llu scale %g leaves the FP16 range", (unsigned long long)r,
                                (double)d->scale[3 * r + j]);
            }
            if (!(half_to_f32(f32_to_half(d->opacity[r])) > 0.0f))
                return fail(V3DG_ERR_INVALID_ARG, "row %llu opacity %g rounds to 0 in FP16", (unsigned long long)r,
                            (double)d->opacity[r]);
        }
        for (uint64_t i = 0; i < (uint64_t)NR * ncoef * 3; ++i) {
            const float v = d->precision == V3DG_FP16 ? half_to_f32(f32_to_half(d->sh[i])) : bf16_to_f32(f32_to_bf16(d->sh[i]));
            if (!finite_f(v)) return fail(V3DG_ERR_INVALID_ARG, "SH coefficient %llu overflows the storage type", (unsigned long long)i);
        }
    }

    // ---- max cut (bound on slots of any selection) per instance
    std::vector<uint64_t> mc(NC, 0);
    for (size_t h = order.size(); h-- > 0;) {
        const uint32_t k = order[h];
        uint64_t sum = 0;
        for (int c = 0; c < d->n_children[k]; ++c) sum += mc[d->first_child[k] + c];
        mc[k] = std::max<uint64_t>(d->count[k], sum);
    }
    uint64_t maxcut = 0;
    for (uint32_t k = 0; k < NC; ++k)
        if (d->parent[k] < 0) maxcut += mc[k];
    const uint64_t cap_slots = maxcut * n_instances;
    if (cap_slots >= 0xffffffffull) return fail(V3DG_ERR_CAPACITY, "a selection could hold %llu Gaussians (> 2^32)", (unsigned long long)cap_slots);

    // ---- upload
    auto *s = new (std::nothrow) v3dg_scene();
    if (!s) return fail(V3DG_ERR_OOM, "host allocation failed");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(V3DG_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
    s->stream = (hipStream_t)hip_stream;
    s->NC = NC;
    s->n_rows = NR;
    s->sh_degree = d->sh_degree;
    s->n_inst = n_instances;
    s->maxcut_rows = maxcut;
    s->cap_slots = cap_slots;
    s->h_count.assign(d->count, d->count + NC);
    for (uint32_t k = 0; k < NC; ++k)
        if (d->n_children[k] == 0) s->leaf_ids.push_back(k);
    s->plane_stride = ((uint64_t)NR + 63) / 64 * 64;
    s->precision = d->precision;
    const uint64_t ps = s->plane_stride;
    const size_t geo_bytes = d->precision == V3DG_FP32 ? 4 : 2, sh_bytes = geo_bytes;
    auto bail = [&](int code) {
        scene_release(s);
        delete s;
        return code;
    };
    if ((rc = dev_alloc(&s->pos_planes, 3 * ps))) return bail(rc);
    if ((rc = dev_alloc((uint8_t **)&s->geo_planes, kGeoPlanes * ps * geo_bytes))) return bail(rc);
    if ((rc = dev_alloc((uint8_t **)&s->sh_planes, 3ull * ncoef * ps * sh_bytes))) return bail(rc);
    if ((rc = dev_alloc(&s->self_sph, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->par_sph, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->rowinfo, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->T_dev, 12ull * n_instances))) return bail(rc);
    if ((rc = dev_alloc(&s->scale_dev, n_instances))) return bail(rc);
    if ((rc = dev_alloc(&s->itab, n_instances))) return bail(rc);
    if ((rc = dev_alloc(&s->pairs_dev, 1))) return bail(rc);
    if (hipMemset(s->pairs_dev, 0, sizeof(unsigned long long)) != hipSuccess)
        return bail(fail(V3DG_ERR_HIP, "hipMemset failed"));
    if (hipHostMalloc((void **)&s->pinned, 64 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
        return bail(fail(V3DG_ERR_OOM, "pinned allocation failed"));
    {
        std::vector<float> hpos(3 * ps, 0.0f), hgeo(kGeoPlanes * ps, 0.0f), hsh(3ull * ncoef * ps, 0.0f);
        for (uint64_t r = 0; r < NR; ++r) {
            for (int j = 0; j < 3; ++j) {
                hpos[j * ps + r] = d->pos[3 * r + j];
                hgeo[(kGeoSX + j) * ps + r] = d->scale[3 * r + j];
            }
            for (int j = 0; j < 4; ++j) hgeo[(kGeoQW + j) * ps + r] = d->rot[4 * r + j];
            hgeo[kGeoOP * ps + r] = d->opacity[r];
            for (int c = 0; c < 3 * ncoef; ++c) hsh[c * ps + r] = d->sh[(uint64_t)r * 3 * ncoef + c];
        }
        std::vector<uint16_t> ngeo, nsh;
        const void *src_geo = hgeo.data(), *src_sh = hsh.data();
        if (d->precision != V3DG_FP32) {
            ngeo.resize(hgeo.size());
            nsh.resize(hsh.size());
            for (size_t i = 0; i < hgeo.size(); ++i) ngeo[i] = f32_to_half(hgeo[i]);
            for (size_t i = 0; i < hsh.size(); ++i)
                nsh[i] = d->precision == V3DG_FP16 ? f32_to_half(hsh[i]) : f32_to_bf16(hsh[i]);
            src_geo = ngeo.data();
            src_sh = nsh.data();
        }
        std::vector<uint2> ri(NC);
        for (uint32_t k = 0; k < NC; ++k) ri[k] = make_uint2(d->first_row[k], d->count[k]);
        e = hipMemcpy(s->pos_planes, hpos.data(), hpos.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->geo_planes, src_geo, hgeo.size() * geo_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->sh_planes, src_sh, hsh.size() * sh_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->self_sph, self.data(), self.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->par_sph, par.data(), par.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->rowinfo, ri.data(), ri.size() * sizeof(uint2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->T_dev, instances_3x4, 12ull * n_instances * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->scale_dev, inst_scale.data(), n_instances * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(V3DG_ERR_HIP, "upload failed: %s", hipGetErrorString(e)));
    }
    *out = s;
    return V3DG_OK;
}

int v3dg_set_instances(v3dg_scene *s, const double *instances_3x4, uint32_t n)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    if (n != s->n_inst) return fail(V3DG_ERR_INVALID_ARG, "instance count %u != %u", n, s->n_inst);
    std::vector<float> sc;
    int rc = check_instances(instances_3x4, n, sc);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(s->device));
    // the host arrays may be freed on return: copy synchronously on the stream
    HIP_TRY(hipMemcpyAsync(s->T_dev, instances_3x4, 12ull * n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->scale_dev, sc.data(), n * sizeof(float), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return V3DG_OK;
}

int v3dg_select(v3dg_scene *s, const v3dg_camera *c, float tau, v3dg_selection **inout)
{
    g_err.clear();
    if (!s || !inout) return fail(V3DG_ERR_INVALID_ARG, "scene and selection pointer must be non-NULL");
    if (!std::isfinite(tau) || tau < 0.0f) return fail(V3DG_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    CamArgs cam;
    int rc = make_cam(c, &cam);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(s->device));
    v3dg_selection *sel = *inout;
    bool fresh = false;
    if (sel) {
        if (sel->scene != s || sel == s->full) return fail(V3DG_ERR_INVALID_ARG, "selection belongs to another scene");
    } else {
        sel = new (std::nothrow) v3dg_selection();
        if (!sel) return fail(V3DG_ERR_OOM, "host allocation failed");
        if ((rc = sel_alloc(s, sel))) {
            sel_release(sel);
            delete sel;
            return rc;
        }
        fresh = true;
    }
    const float K = footprint_K(c);
    {
        Stage st(s, V3DG_STAGE_SETUP);
        launch_frame_setup(s->stream, cam, s->T_dev, s->scale_dev, s->n_inst, s->itab, sel->clear_block,
                           (uint64_t)kSelCounters + 2 * sel->n_parts);
    }
    {
        Stage st(s, V3DG_STAGE_SELECT);
        launch_select(s->stream, s->self_sph, s->par_sph, s->rowinfo, s->itab, s->NC, s->n_inst, K, tau, sel->gid,
                      sel->slot_off, sel->status, sel->counters);
    }
    {
        Stage st(s, V3DG_STAGE_EXPAND);
        launch_expand(s->stream, sel->gid, sel->slot_off, s->rowinfo, s->NC, sel->counters,
                      (uint32_t)std::min<uint64_t>(sel->cap_tests, 0xffffffffull), sel->slot_row, sel->slot_inst);
    }
    s->acc.selects += 1;
    s->acc.tests += (uint64_t)s->NC * s->n_inst;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        if (fresh) {
            sel_release(sel);
            delete sel;
        }
        return fail(V3DG_ERR_HIP, "select launch failed: %s", hipGetErrorString(e));
    }
    *inout = sel;
    return V3DG_OK;
}

int v3dg_render(v3dg_scene *s, const v3dg_camera *c, const v3dg_selection *sel, float *image)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    return render_impl(s, c, sel, image);
}

int v3dg_render_full(v3dg_scene *s, const v3dg_camera *c, float *image)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    CamArgs cam;
    int rc = make_cam(c, &cam);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(s->device));
    if ((rc = build_full_selection(s))) return rc;
    return render_impl(s, c, s->full, image);
}

int v3dg_selection_info(const v3dg_selection *sel, uint64_t *n_clusters, uint64_t *n_gaussians)
{
    g_err.clear();
    if (!sel || !sel->scene) return fail(V3DG_ERR_INVALID_ARG, "selection is NULL");
    v3dg_scene *s = sel->scene;
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipMemcpyAsync(s->pinned + 8, sel->counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->pinned[8 + kSelErr] & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    if (n_clusters) *n_clusters = s->pinned[8 + kSelNClusters];
    if (n_gaussians) *n_gaussians = s->pinned[8 + kSelNGaussians];
    return V3DG_OK;
}

int v3dg_selection_copy_ids(const v3dg_selection *sel, uint32_t *host_gids, uint64_t cap, uint64_t *n_out)
{
    uint64_t nc = 0, ng = 0;
    int rc = v3dg_selection_info(sel, &nc, &ng);
    if (rc) return rc;
    if (n_out) *n_out = nc;
    if (nc > cap) return fail(V3DG_ERR_CAPACITY, "%llu ids do not fit in %llu", (unsigned long long)nc, (unsigned long long)cap);
    if (nc == 0) return V3DG_OK;
    if (!host_gids) return fail(V3DG_ERR_INVALID_ARG, "host_gids is NULL");
    HIP_TRY(hipMemcpy(host_gids, sel->gid, nc * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return V3DG_OK;
}

int v3dg_selection_copy_slots(const v3dg_selection *sel, uint32_t *host_rows, uint32_t *host_inst, uint64_t cap,
                              uint64_t *n_out)
{
    uint64_t nc = 0, ng = 0;
    int rc = v3dg_selection_info(sel, &nc, &ng);
    if (rc) return rc;
    if (n_out) *n_out = ng;
    if (ng > cap) return fail(V3DG_ERR_CAPACITY, "%llu slots do not fit in %llu", (unsigned long long)ng, (unsigned long long)cap);
    if (ng == 0) return V3DG_OK;
    if (!host_rows || !host_inst) return fail(V3DG_ERR_INVALID_ARG, "output array is NULL");
    HIP_TRY(hipMemcpy(host_rows, sel->slot_row, ng * sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(host_inst, sel->slot_inst, ng * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return V3DG_OK;
}

void v3dg_selection_free(v3dg_selection *sel)
{
    if (!sel) return;
    if (sel->scene && sel == sel->scene->full) return;  // owned by the scene
    if (sel->scene) {
        (void)hipSetDevice(sel->scene->device);
        (void)hipStreamSynchronize(sel->scene->stream);
    }
    sel_release(sel);
    delete sel;
}

void v3dg_scene_free(v3dg_scene *s)
{
    if (!s) return;
    scene_release(s);
    delete s;
}

int v3dg_get_frame_stats(v3dg_scene *s, v3dg_frame_stats *out)
{
    g_err.clear();
    if (!s || !out) return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    uint32_t err = 0;
    if (s->rcounters) HIP_TRY(hipMemcpy(&err, s->rcounters + kRenErr, sizeof(err), hipMemcpyDeviceToHost));
    if (err & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    if (err & kErrOverflow) return fail(V3DG_ERR_DEVICE, "tile counting and key emission disagreed");
    *out = s->last;
    return V3DG_OK;
}

int v3dg_copy_projection(v3dg_scene *s, float *mean2, float *conic, float *rgb, float *opacity, float *depth,
                         uint32_t *tiles, uint64_t cap, uint64_t *n_out)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const uint64_t n = s->last.n_slots;
    if (n_out) *n_out = n;
    if (n > cap) return fail(V3DG_ERR_CAPACITY, "%llu slots do not fit in %llu", (unsigned long long)n, (unsigned long long)cap);
    if (n == 0) return V3DG_OK;
    std::vector<float4> sp(3 * n);
    std::vector<uint32_t> tl(n);
    std::vector<float> dp(n);
    HIP_TRY(hipMemcpy(sp.data(), s->splat, 3 * n * sizeof(float4), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(tl.data(), s->tiles, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dp.data(), s->depth, n * sizeof(float), hipMemcpyDeviceToHost));
    for (uint64_t t = 0; t < n; ++t) {
        const float4 a = sp[3 * t], b = sp[3 * t + 1], c = sp[3 * t + 2];
        if (mean2) { mean2[2 * t] = a.x; mean2[2 * t + 1] = a.y; }
        if (conic) { conic[3 * t] = a.z; conic[3 * t + 1] = a.w; conic[3 * t + 2] = b.x; }
        if (opacity) opacity[t] = b.y;
        if (rgb) { rgb[3 * t] = b.z; rgb[3 * t + 1] = b.w; rgb[3 * t + 2] = c.x; }
        if (depth) depth[t] = dp[t];
        if (tiles) tiles[t] = tl[t];
    }
    return V3DG_OK;
}

int v3dg_copy_attributes(v3dg_scene *s, uint64_t first, uint64_t n, float *pos, float *scale, float *rot,
                         float *opacity, float *sh)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    if (first > s->n_rows || n > s->n_rows - first)
        return fail(V3DG_ERR_INVALID_ARG, "rows [%llu, +%llu) outside the %llu-row table", (unsigned long long)first,
                    (unsigned long long)n, (unsigned long long)s->n_rows);
    if (n == 0) return V3DG_OK;
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const uint64_t ps = s->plane_stride;
    const int ncoef = (int)((s->sh_degree + 1) * (s->sh_degree + 1));
    const size_t eb = s->precision == V3DG_FP32 ? 4 : 2;
    auto widen = [&](const void *base, int plane, bool sh_plane, std::vector<float> &out) -> int {
        std::vector<uint8_t> raw(n * eb);
        HIP_TRY(hipMemcpy(raw.data(), (const uint8_t *)base + (plane * ps + first) * eb, n * eb, hipMemcpyDeviceToHost));
        out.resize(n);
        for (uint64_t i = 0; i < n; ++i) {
            if (eb == 4) {
                std::memcpy(&out[i], &raw[4 * i], 4);
            } else {
                uint16_t h;
                std::memcpy(&h, &raw[2 * i], 2);
                out[i] = (sh_plane && s->precision == V3DG_FP16_BF16SH) ? bf16_to_f32(h) : half_to_f32(h);
            }
        }
        return V3DG_OK;
    };
    std::vector<float> col;
    int rc;
    if (pos)
        for (int j = 0; j < 3; ++j) {
            col.resize(n);
            HIP_TRY(hipMemcpy(col.data(), s->pos_planes + j * ps + first, n * sizeof(float), hipMemcpyDeviceToHost));
            for (uint64_t i = 0; i < n; ++i) pos[3 * i + j] = col[i];
        }
    if (scale)
        for (int j = 0; j < 3; ++j) {
            if ((rc = widen(s->geo_planes, kGeoSX + j, false, col))) return rc;
            for (uint64_t i = 0; i < n; ++i) scale[3 * i + j] = col[i];
        }
    if (rot)
        for (int j = 0; j < 4; ++j) {
            if ((rc = widen(s->geo_planes, kGeoQW + j, false, col))) return rc;
            for (uint64_t i = 0; i < n; ++i) rot[4 * i + j] = col[i];
        }
    if (opacity) {
        if ((rc = widen(s->geo_planes, kGeoOP, false, col))) return rc;
        for (uint64_t i = 0; i < n; ++i) opacity[i] = col[i];
    }
    if (sh)
        for (int c = 0; c < 3 * ncoef; ++c) {
            if ((rc = widen(s->sh_planes, c, true, col))) return rc;
            for (uint64_t i = 0; i < n; ++i) sh[(uint64_t)3 * ncoef * i + c] = col[i];
        }
    return V3DG_OK;
}

int v3dg_copy_sorted_keys(v3dg_scene *s, uint64_t *keys, uint32_t *vals, uint64_t cap, uint64_t *n_out)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const uint64_t n = s->last.n_keys;
    if (n_out) *n_out = n;
    if (n > cap) return fail(V3DG_ERR_CAPACITY, "%llu keys do not fit in %llu", (unsigned long long)n, (unsigned long long)cap);
    if (n == 0) return V3DG_OK;
    std::vector<uint32_t> v(n);
    HIP_TRY(hipMemcpy(v.data(), s->vals[s->last_buf], n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (keys) {
        if (s->last.sort_mode == V3DG_SORT_KEYS64) {
            HIP_TRY(hipMemcpy(keys, s->keys[s->last_buf], n * sizeof(uint64_t), hipMemcpyDeviceToHost));
        } else {  // tile ids; the depth bits come from the slot
            std::vector<uint32_t> tk(n), dp(s->last.n_slots);
            HIP_TRY(hipMemcpy(tk.data(), s->keys[s->last_buf], n * sizeof(uint32_t), hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(dp.data(), s->depth, dp.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
            for (uint64_t i = 0; i < n; ++i) keys[i] = ((uint64_t)tk[i] << 32) | dp[v[i]];
        }
    }
    if (vals) std::memcpy(vals, v.data(), n * sizeof(uint32_t));
    return V3DG_OK;
}

int v3dg_set_sort_mode(v3dg_scene *s, int mode)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    if (mode != V3DG_SORT_DEPTH_FIRST && mode != V3DG_SORT_KEYS64)
        return fail(V3DG_ERR_INVALID_ARG, "unknown sort mode %d", mode);
    s->sort_mode = mode;
    return V3DG_OK;
}

int v3dg_set_profiling(v3dg_scene *s, int on)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    s->profiling = on != 0;
    return V3DG_OK;
}

int v3dg_collect_profile(v3dg_scene *s, v3dg_profile *out)
{
    g_err.clear();
    if (!s || !out) return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    unsigned long long pairs = 0;
    HIP_TRY(hipMemcpy(&pairs, s->pairs_dev, sizeof(pairs), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(s->pairs_dev, 0, sizeof(pairs)));
    v3dg_profile p = s->acc;
    p.pairs = pairs;
    for (int i = 0; i < V3DG_N_STAGES; ++i) {
        p.ms[i] = 0.0;
        p.launches[i] = 0;
    }
    for (auto &r : s->prof) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            p.ms[r.stage] += t;
            p.launches[r.stage] += 1;
        }
        s->ev_pool.push_back(r.a);
        s->ev_pool.push_back(r.b);
    }
    s->prof.clear();
    s->acc = v3dg_profile{};
    *out = p;
    return V3DG_OK;
}

int v3dg_sort_pairs(uint64_t *keys_dev, uint32_t *vals_dev, uint64_t n, uint32_t key_bits, void *hip_stream)
{
    g_err.clear();
    if (key_bits < 1 || key_bits > 64) return fail(V3DG_ERR_INVALID_ARG, "key_bits must be 1..64");
    if (n >= 0xffffffffull) return fail(V3DG_ERR_CAPACITY, "n must be < 2^32");
    if (n == 0) return V3DG_OK;
    if (!keys_dev || !vals_dev) return fail(V3DG_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t st = (hipStream_t)hip_stream;
    const int passes = (int)((key_bits + kRadixBits - 1) / kRadixBits);
    const uint64_t parts = (n + kSortPart - 1) / kSortPart;
    uint64_t *k2 = nullptr, *status = nullptr;
    uint32_t *v2 = nullptr, *ctr = nullptr;
    int rc = dev_alloc(&k2, n);
    if (!rc) rc = dev_alloc(&v2, n);
    if (!rc) rc = dev_alloc(&status, parts * kRadix);
    if (!rc) rc = dev_alloc(&ctr, (uint64_t)kRenCounters);
    if (!rc) {
        launch_fill_u32(st, reinterpret_cast<uint32_t *>(status), 2 * parts * kRadix, 0u);
        launch_fill_u32(st, ctr, kRenCounters, 0u);
        launch_sort_hist<uint64_t>(st, keys_dev, n, passes, ctr + kRenHist);
        uint64_t *kb[2] = {keys_dev, k2};
        uint32_t *vb[2] = {vals_dev, v2};
        int cur = 0;
        for (int p = 0; p < passes; ++p) {
            launch_sort_pass<uint64_t>(st, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, p, ctr + kRenHist, status,
                                       (uint32_t)(p + 1), ctr + kRenTicketSort + p, ctr + kRenErr);
            cur ^= 1;
        }
        if (cur == 1) {
            (void)hipMemcpyAsync(keys_dev, k2, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
            (void)hipMemcpyAsync(vals_dev, v2, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        }
        uint32_t err = 0;
        hipError_t e = hipMemcpyAsync(&err, ctr + kRenErr, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(V3DG_ERR_HIP, "sort failed: %s", hipGetErrorString(e));
        else if (err & kErrSpin) rc = fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    }
    dev_free(k2);
    dev_free(v2);
    dev_free(status);
    dev_free(ctr);
    return rc;
}

}  // extern "C"
