// C ABI of v3dg: scene residency and validation, selection objects, the
// per-frame kernel chain, and stage timing.  Host code only; every step of the
// frame runs in the HIP kernels of select/project/sort/blend.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/v3dg.h"
#include "v3dg_internal.h"
#include "page_lru.h"
#include "page_store.h"

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

// Stream, frame state and render workspace of one frame in flight: the one
// every scene owns (v3dg_render) or one context of a server.
struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    FrameDev *fdev = nullptr;   // camera, image and sort epoch read by the kernels
    uint64_t epoch_host = 0;    // mirror of fdev->epoch
    InstRec *itab = nullptr;
    uint32_t itab_cap = 0;
    uint64_t ws_slots = 0;
    float4 *splat = nullptr;
    BinRec *bin = nullptr;
    float *depth = nullptr;
    uint32_t *tiles = nullptr;
    uint32_t *offsets = nullptr;
    uint32_t *big = nullptr;  // splats emitted by the large-splat kernel
    uint32_t *dkey[2] = {nullptr, nullptr};
    uint32_t *dval[2] = {nullptr, nullptr};
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
    uint32_t *cbase = nullptr;     // per tile: first chunk of a long list; then the blend order (tiles_cap each)
    uint2 *items = nullptr;        // (tile, chunk) work items past the rounds
    uint32_t *rounds = nullptr;    // per round of chunk work, the long tiles (tiles_cap each)
    float4 *scratch = nullptr;     // per chunk, per pixel (C, T)
    uint32_t *pend = nullptr;      // per long tile, per pixel: chunk to walk again
    uint32_t *need = nullptr;      // per chunk: walk it again
    uint64_t *stopm = nullptr;     // per chunk, per wavefront: pixels the chunk stopped
    uint2 *rewalk = nullptr;       // (tile, chunk) to walk again
    uint64_t cap_chunks = 0;
    uint32_t chunk_shift = kChunkShiftRender;  // chunk sizes of long bin lists (ChunkPlan)
    uint32_t *pinned = nullptr;
    v3dg_frame_stats last{};
    int last_buf = 0;
    int sort_mode = V3DG_SORT_DEPTH_FIRST;
    uint32_t profiling = 0;   // stages timed with events (bit per stage)
    int pair_count = 0;       // pairs blending counts: 0 none, 1 walked, 2 walked and taken
    v3dg_profile acc{};
    unsigned long long *pairs_dev = nullptr;  // walked and taken (pixel, splat) pairs, kPairSlots of each
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    // frames sized by capacity publish their counts into a ring of records in
    // mapped pinned memory (FrameRec); the host reads a record once the
    // frame's event has completed
    static constexpr uint32_t kRecRing = 4;  // frames in flight
    FrameRec *rec_h = nullptr, *rec_d = nullptr;
    hipEvent_t rec_ev[kRecRing] = {};
    uint32_t rec_want[kRecRing] = {};  // the tag each record must carry
    uint32_t rec_head = 0, rec_n = 0, rec_seq = 0;
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
    uint64_t stream_frame = 0;  // streamed scenes: the paging frame of the cut
};

// a streamed frame's own copy of its slot count, among the spare render counters
constexpr int kRenSlots = kRenBig + 1;
static_assert(kRenSlots < kRenCounters, "render counter out of range");

struct v3dg_scene : Ctx {
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
    uint64_t maxcut_rows = 0;
    uint64_t cap_slots = 0;       // bound on the slots of any selection
    CullRec *cull_dev = nullptr;  // per cluster: sphere of the rows' means, largest scale
    bool culling = false;         // view culling of cut clusters in v3dg_select
    std::vector<uint32_t> leaf_ids;
    std::vector<uint32_t> h_count;
    v3dg_selection *full = nullptr;
    std::vector<uint32_t> full_gid, full_off;  // the full-detail cut, on the host
    uint32_t full_total = 0;
    // ---- cluster streaming (pool_clusters > 0): the rows live on the host as
    // one page image per cluster; the planes above are a pool of pages of 64
    // rows (plane_stride = 64 pool_clusters); rowinfo[k].x is the first pool
    // row of a resident cluster.  Pages form an LRU list (head: most recent).
    uint32_t pool_clusters = 0, page_bytes = 0, geo_bytes = 4, sh_bytes = 4, n_sh = 0, stage_cap = 0;
    uint64_t stage_stride = 0;  // bytes between staged images (the store's slot)
    PageStore pages;            // page images: host memory or a file
    PageLRU lru;  // which cluster holds which page
    uint8_t *stage_h = nullptr, *stage_d = nullptr;
    uint4 *ups_h = nullptr, *ups_d = nullptr;
    std::vector<uint32_t> cut_gid, cut_off;
    v3dg_stream_stats sstats{};
    // selects of a streamed scene run on sel_stream, after the projection of
    // the frame before (ev_proj) and before the render that follows (ev_sel),
    // so that their read-back and paging overlap that frame's later stages
    hipStream_t sel_stream = nullptr;
    hipEvent_t ev_proj = nullptr, ev_sel = nullptr;
    // v3dg_render without host waits: the first frame of an image size is
    // sized exactly (one wait after the tile scan); later frames of that size
    // run on key buffers sized by capacity (ensure_render_capacity), and
    // their counts come back through FrameRec
    uint32_t rend_tiles = 0;        // tiles of the image size the capacity is set for (0: none)
    uint64_t keys_seen = 0;         // most keys of any frame seen
    uint32_t rend_err = 0;          // error flags of capacity frames read back since the last frame stats
    bool last_keycap = false;       // the last frame's keys exceeded its buffers (blended without them)
    Attribs attribs() const { return Attribs{pos_planes, geo_planes, sh_planes, plane_stride}; }
};

namespace {

// ---- profiling --------------------------------------------------------------
struct Stage {
    Ctx *s;
    int stage;
    hipStream_t q;  // the stream the stage's launches go to
    hipEvent_t b = nullptr;
    Stage(Ctx *sc, int st, hipStream_t on = nullptr) : s(sc), stage(st), q(on ? on : sc->stream)
    {
        if (!(s->profiling >> stage & 1u)) return;
        hipEvent_t a = take();
        b = take();
        (void)hipEventRecord(a, q);
        s->prof.push_back({stage, a, b});
    }
    ~Stage()
    {
        if (b) (void)hipEventRecord(b, q);
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
    o->bins_x = (c->width + kBin - 1) / kBin;
    o->bins_y = (c->height + kBin - 1) / kBin;
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

// buffers for selections of up to cap_tests tests and cap_slots slots
int sel_alloc_caps(v3dg_selection *s, uint64_t cap_tests, uint64_t cap_slots, hipStream_t st)
{
    s->cap_tests = cap_tests;
    s->cap_slots = cap_slots;
    s->n_parts = (s->cap_tests + kSelPart - 1) / kSelPart;
    int rc;
    if ((rc = dev_alloc(&s->gid, s->cap_tests))) return rc;
    if ((rc = dev_alloc(&s->slot_off, s->cap_tests))) return rc;
    if ((rc = dev_alloc(&s->clear_block, (uint64_t)kSelCounters + 2 * s->n_parts))) return rc;
    s->counters = s->clear_block;
    s->status = reinterpret_cast<uint64_t *>(s->clear_block + kSelCounters);
    if ((rc = dev_alloc(&s->slot_row, s->cap_slots))) return rc;
    if ((rc = dev_alloc(&s->slot_inst, s->cap_slots))) return rc;
    HIP_TRY(hipMemsetAsync(s->clear_block, 0, sizeof(uint32_t) * kSelCounters, st));
    return V3DG_OK;
}

int sel_alloc(v3dg_scene *sc, v3dg_selection *s)
{
    s->scene = sc;
    return sel_alloc_caps(s, (uint64_t)sc->NC * sc->n_inst, sc->cap_slots,
                          sc->pool_clusters ? sc->sel_stream : sc->stream);
}

// Plane coefficients of the cluster view cull for one camera (see CullRec).
CullCam make_cullcam(const CamArgs &c)
{
    CullCam cc{};
    cc.fx = c.fx;
    cc.fy = c.fy;
    cc.al = (double)c.cx + 2.5;
    cc.ar = (double)c.cx - (double)c.width - 2.5;
    cc.at = (double)c.cy + 2.5;
    cc.ab = (double)c.cy - (double)c.height - 2.5;
    cc.nl = std::sqrt(cc.fx * cc.fx + cc.al * cc.al);
    cc.nr = std::sqrt(cc.fx * cc.fx + cc.ar * cc.ar);
    cc.nt = std::sqrt(cc.fy * cc.fy + cc.at * cc.at);
    cc.nb = std::sqrt(cc.fy * cc.fy + cc.ab * cc.ab);
    // support half-extent <= sqrt(Qm) |m1| + 1 with Qm <= 1.05 * 2 ln 255 + 0.05 < 3.5^2
    // and |m1| <= (f / z)(1 + guard band) s smax
    cc.kx = 3.5 * (1.0 + (double)c.limx) * cc.fx;
    cc.ky = 3.5 * (1.0 + (double)c.limy) * cc.fy;
    cc.nearp = c.near_plane;
    return cc;
}

// one selection request of scene sc into selection buffers sel
SelReq make_selreq(const v3dg_scene *sc, const InstRec *itab, float K, float tau, v3dg_selection *sel,
                   const CamArgs &cam, bool cull)
{
    SelReq q{};
    q.cull = cull ? sc->cull_dev : nullptr;
    q.cc = make_cullcam(cam);
    q.self_sph = sc->self_sph;
    q.par_sph = sc->par_sph;
    q.rowinfo = sc->rowinfo;
    q.itab = itab;
    q.gid = sel->gid;
    q.slot_off = sel->slot_off;
    q.status = sel->status;
    q.counters = sel->counters;
    q.slot_row = sel->slot_row;
    q.slot_inst = sel->slot_inst;
    q.NC = sc->NC;
    q.n_inst = sc->n_inst;
    q.K = K;
    q.tau = tau;
    q.part_begin = 0;
    q.nparts = (uint32_t)(((uint64_t)sc->NC * sc->n_inst + kSelPart - 1) / kSelPart);
    return q;
}

// ---- render contexts --------------------------------------------------------------
int ctx_init(Ctx *c, int device, hipStream_t stream)
{
    c->device = device;
    c->stream = stream;
    int rc;
    if ((rc = dev_alloc(&c->fdev, 1))) return rc;
    if ((rc = dev_alloc(&c->pairs_dev, 2 * kPairSlots))) return rc;
    HIP_TRY(hipMemset(c->fdev, 0, sizeof(FrameDev)));
    HIP_TRY(hipMemset(c->pairs_dev, 0, 2 * kPairSlots * sizeof(unsigned long long)));
    if (hipHostMalloc((void **)&c->pinned, 64 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        return fail(V3DG_ERR_OOM, "pinned allocation failed");
    }
    if (hipHostMalloc((void **)&c->rec_h, Ctx::kRecRing * sizeof(FrameRec), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        c->rec_h = nullptr;
        return fail(V3DG_ERR_OOM, "pinned allocation failed");
    }
    std::memset(c->rec_h, 0, Ctx::kRecRing * sizeof(FrameRec));
    HIP_TRY(hipHostGetDevicePointer((void **)&c->rec_d, c->rec_h, 0));
    for (uint32_t i = 0; i < Ctx::kRecRing; ++i) HIP_TRY(hipEventCreateWithFlags(&c->rec_ev[i], hipEventDisableTiming));
    return V3DG_OK;
}

void ctx_free_slots(Ctx *c)
{
    dev_free(c->splat);
    dev_free(c->bin);
    dev_free(c->depth);
    for (int b = 0; b < 2; ++b) {
        dev_free(c->dkey[b]);
        dev_free(c->dval[b]);
    }
    dev_free(c->tiles);
    dev_free(c->offsets);
    dev_free(c->big);
    dev_free(c->rclear);
    c->ws_slots = 0;
    c->tiles_cap = 0;
}

void ctx_release(Ctx *c)
{
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    ctx_free_slots(c);
    dev_free(c->fdev);
    dev_free(c->itab);
    for (int b = 0; b < 2; ++b) {
        dev_free(c->keys[b]);
        dev_free(c->vals[b]);
    }
    dev_free(c->sort_status);
    dev_free(c->pairs_dev);
    dev_free(c->cbase);
    dev_free(c->rounds);
    dev_free(c->items);
    dev_free(c->scratch);
    dev_free(c->pend);
    dev_free(c->need);
    dev_free(c->stopm);
    dev_free(c->rewalk);
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    if (c->rec_h) (void)hipHostFree(c->rec_h);
    c->rec_h = c->rec_d = nullptr;
    for (uint32_t i = 0; i < Ctx::kRecRing; ++i)
        if (c->rec_ev[i]) (void)hipEventDestroy(c->rec_ev[i]);
    for (auto &r : c->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    c->prof.clear();
    c->ev_pool.clear();
}

int ensure_status(Ctx *c, uint64_t parts);

int ensure_itab(Ctx *c, uint32_t n)
{
    if (n <= c->itab_cap) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dev_free(c->itab);
    int rc;
    if ((rc = dev_alloc(&c->itab, n))) return rc;
    c->itab_cap = n;
    return V3DG_OK;
}

int ensure_slots(Ctx *c, uint64_t n)
{
    if (n <= c->ws_slots && c->splat) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    ctx_free_slots(c);
    int rc;
    if ((rc = dev_alloc(&c->splat, 3 * n))) return rc;
    if ((rc = dev_alloc(&c->bin, n))) return rc;
    if ((rc = dev_alloc(&c->depth, n))) return rc;
    if ((rc = dev_alloc(&c->tiles, n))) return rc;
    if ((rc = dev_alloc(&c->offsets, n))) return rc;
    if ((rc = dev_alloc(&c->big, n))) return rc;
    for (int b = 0; b < 2; ++b) {
        if ((rc = dev_alloc(&c->dkey[b], n))) return rc;
        if ((rc = dev_alloc(&c->dval[b], n))) return rc;
    }
    c->ws_slots = n;
    c->scan_parts = (n + kScanPart - 1) / kScanPart;
    if ((rc = ensure_status(c, (n + kSortPart - 1) / kSortPart))) return rc;
    return V3DG_OK;
}

int ensure_tiles(Ctx *c, uint32_t n_tiles)
{
    if (c->rclear && n_tiles <= c->tiles_cap) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dev_free(c->rclear);
    c->tiles_cap = std::max<uint32_t>(n_tiles, 8160);
    c->rclear_words = (uint64_t)kRenCounters + 2 * c->scan_parts + 2ull * c->tiles_cap;
    int rc;
    if ((rc = dev_alloc(&c->rclear, c->rclear_words))) return rc;
    c->rcounters = c->rclear;
    c->scan_status = reinterpret_cast<uint64_t *>(c->rclear + kRenCounters);
    c->ranges = reinterpret_cast<uint2 *>(c->rclear + kRenCounters + 2 * c->scan_parts);
    dev_free(c->cbase);
    if ((rc = dev_alloc(&c->cbase, 2ull * c->tiles_cap))) return rc;
    dev_free(c->rounds);
    if ((rc = dev_alloc(&c->rounds, (uint64_t)kChunkRounds * c->tiles_cap))) return rc;
    return V3DG_OK;
}

int ensure_status(Ctx *c, uint64_t parts)
{
    if (parts <= c->sort_status_parts) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dev_free(c->sort_status);
    const uint64_t np = std::max<uint64_t>(parts + parts / 2, 256);
    int rc;
    if ((rc = dev_alloc(&c->sort_status, np * kRadix))) return rc;
    HIP_TRY(hipMemsetAsync(c->sort_status, 0, np * kRadix * sizeof(uint64_t), c->stream));
    c->sort_status_parts = np;
    return V3DG_OK;
}

// chunk buffers for frames of up to K keys (chunk_bound of the context's plan)
int ensure_chunks(Ctx *c, uint64_t K)
{
    const uint64_t need = chunk_bound(K, c->chunk_shift);
    if (need <= c->cap_chunks) return V3DG_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    dev_free(c->items);
    dev_free(c->scratch);
    dev_free(c->pend);
    dev_free(c->need);
    dev_free(c->stopm);
    dev_free(c->rewalk);
    const uint64_t cap = need + need / 2;
    int rc;
    if ((rc = dev_alloc(&c->items, cap))) return rc;
    if ((rc = dev_alloc(&c->scratch, cap * 256))) return rc;
    if ((rc = dev_alloc(&c->pend, cap * 256))) return rc;
    if ((rc = dev_alloc(&c->need, cap))) return rc;
    if ((rc = dev_alloc(&c->stopm, cap * 4))) return rc;
    // the blend keeps these words zero between frames (see launch_blend)
    HIP_TRY(hipMemsetAsync(c->stopm, 0, cap * 4 * sizeof(uint64_t), c->stream));
    if ((rc = dev_alloc(&c->rewalk, cap))) return rc;
    c->cap_chunks = cap;
    return V3DG_OK;
}

// key buffers for at least K keys (exact_cap: exactly max(K, 1))
int ensure_keys(Ctx *c, uint64_t K, bool exact_cap = false)
{
    const uint64_t parts = (K + kSortPart - 1) / kSortPart;
    if (K > c->cap_keys) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int b = 0; b < 2; ++b) {
            dev_free(c->keys[b]);
            dev_free(c->vals[b]);
        }
        uint64_t cap = exact_cap ? std::max<uint64_t>(K, 1) : std::max<uint64_t>(K + K / 2, 1u << 20);
        cap = std::min<uint64_t>(cap, 0xffffffffull);
        int rc;
        for (int b = 0; b < 2; ++b) {
            if ((rc = dev_alloc(&c->keys[b], cap))) return rc;
            if ((rc = dev_alloc(&c->vals[b], cap))) return rc;
        }
        c->cap_keys = cap;
    }
    return ensure_status(c, parts);
}

// Every frame takes kEpochsPerFrame look-back epochs; before the 30-bit field
// wraps, the look-back words and the epoch start again from zero.
void epoch_advance(Ctx *c)
{
    if (c->epoch_host + 2 * kEpochsPerFrame >= kEpochLimit) {
        if (c->sort_status) launch_fill_u32(c->stream, reinterpret_cast<uint32_t *>(c->sort_status),
                                            2 * c->sort_status_parts * kRadix, 0u);
        launch_fill_u32(c->stream, &c->fdev->epoch, 1, 0u);
        c->epoch_host = 0;
    }
    c->epoch_host += kEpochsPerFrame;
}

// Stable sort of K (key, value) pairs held in buffer 0 by the low key_bits
// bits; n_dev, when given, is the device-side count (K then bounds it).
// have_hist: the digit histograms of plan dp were counted by emission;
// otherwise the keys are sorted by 8-bit digits with their own histogram pass.
template <typename KT>
void run_sort(Ctx *c, KT *const kb[2], uint32_t *const vb[2], const uint32_t *n_dev, uint64_t K, uint32_t key_bits,
              uint32_t epoch_base, int *out_buf, uint32_t *passes_out, bool have_hist, const DigitPlan *dp = nullptr)
{
    const int passes = have_hist && dp ? dp->passes : (int)((key_bits + kRadixBits - 1) / kRadixBits);
    *passes_out = (uint32_t)passes;
    int cur = 0;
    if (!have_hist) {
        Stage st(c, V3DG_STAGE_SORT_HIST);
        launch_sort_hist<KT>(c->stream, kb[0], n_dev, K, passes, c->rcounters + kRenHist);
    }
    for (int p = 0; p < passes; ++p) {
        Stage st(c, V3DG_STAGE_SORT_PASS);
        const int shift = have_hist && dp ? (int)dp->shift[p] : -1;
        const int dbits = have_hist && dp ? (int)dp->bits[p] : kRadixBits;
        launch_sort_pass<KT>(c->stream, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n_dev, K, p, c->rcounters + kRenHist,
                             c->sort_status, &c->fdev->epoch, epoch_base + (uint32_t)p,
                             c->rcounters + kRenTicketSort + p, c->rcounters + kRenErr, K >= kSortWideFrom, shift,
                             dbits);
        cur ^= 1;
    }
    *out_buf = cur;
}

// Depth-first binning: tile-id keys of type KT in depth order, their stable
// sort, and the tile ranges with the blend plan.
// Where a frame publishes its counts (capacity-sized frames of v3dg_render)
struct FramePub {
    const uint32_t *sel_counters = nullptr;
    FrameRec *rec = nullptr;  // device address of the record, nullptr: none
    uint32_t seq = 0;
    bool fallback = false;    // blend the frame from all visible splats when its keys do not fit
};

template <typename KT>
void tile_keys(Ctx *c, const uint32_t *n_dev, uint64_t S, const uint32_t *k_dev, uint64_t KL, uint32_t key_bits,
               uint32_t tiles_x, uint32_t n_tiles, uint32_t bins_x, uint64_t max_chunks, int *buf, uint32_t *passes,
               const FramePub &pub)
{
    KT *kb[2] = {reinterpret_cast<KT *>(c->keys[0]), reinterpret_cast<KT *>(c->keys[1])};
    const DigitPlan dp = even_digits(key_bits);
    {
        Stage st(c, V3DG_STAGE_EMIT);
        launch_emit32<KT>(c->stream, n_dev, S, c->dval[0], c->tiles, c->offsets, c->rcounters, c->bin,
                          c->fdev, c->cap_keys, dp, kb[0], c->vals[0], c->rcounters + kRenHist, c->big,
                          c->rcounters + kRenBig, c->rcounters + kRenErr);
    }
    if (KL > 0) run_sort<KT>(c, kb, c->vals, k_dev, KL, key_bits, 4, buf, passes, true, &dp);
    {
        Stage st(c, V3DG_STAGE_RANGES);
        launch_tile_ranges<KT>(c->stream, kb[*buf], c->rcounters + kRenKeysEff, 0, tiles_x, n_tiles, bins_x,
                               c->ranges, c->cbase, c->items, c->rounds, c->tiles_cap, c->cbase + c->tiles_cap,
                               c->rcounters, max_chunks, ChunkPlan{c->chunk_shift}, pub.sel_counters, pub.rec,
                               pub.seq);
    }
}

struct SelView {
    const uint32_t *counters;  // kSelNGaussians holds the slot count
    const uint32_t *slot_row, *slot_inst;
};

// What one frame's launches were sized for.
struct FrameInfo {
    uint64_t K = 0;            // keys (host-sized frames only)
    uint32_t n_tiles = 0, n_bins = 0, key_bits = 0, passes = 0, N = 0, n_visible = 0, n_sel_clusters = 0;
    int buf = 0;
    bool depth_first = true;
};

// Enqueue one frame of scene sc on context c.
//   capacity == false: the counts are read back once after the tile scan
//     (one host wait), buffers grow to fit and every later launch is sized
//     exactly.  Used by v3dg_render.
//   capacity == true: no host wait; launches are sized by the context's
//     capacities, kernels read every count from device memory and a frame
//     that needs more keys than cap_keys raises kErrOverflow (its image is
//     then incomplete).  The caller ensures capacities first; from_fd says
//     the camera and image were copied into c->fdev.  Capturable in a graph.
int enqueue_frame(Ctx *c, v3dg_scene *sc, const CamArgs &cam, float *image, const SelView &sel, bool capacity,
                  bool from_fd, FrameInfo *fi, const FramePub &pub = FramePub{})
{
    int rc;
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    fi->n_tiles = n_tiles;
    fi->n_bins = cam.bins_x * cam.bins_y;
    if (!capacity) {
        if ((rc = ensure_itab(c, sc->n_inst))) return rc;
        if ((rc = ensure_slots(c, sc->cap_slots))) return rc;
        if ((rc = ensure_tiles(c, n_tiles))) return rc;
        epoch_advance(c);
    }
    const uint64_t S = sc->cap_slots;  // grid bound of the per-slot kernels
    const uint32_t *n_dev = sel.counters + kSelNGaussians;
    {
        Stage st(c, V3DG_STAGE_SETUP);
        launch_frame_setup(c->stream, cam, image, c->fdev, from_fd, true, sc->T_dev, sc->scale_dev, sc->n_inst,
                           c->itab, c->rclear, (uint64_t)kRenCounters + 2 * c->scan_parts + 2ull * n_tiles);
    }
    if (sc->pool_clusters) {  // streamed: the next select may rewrite the selection once projection is done
        HIP_TRY(hipMemcpyAsync(c->rcounters + kRenSlots, n_dev, sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
        n_dev = c->rcounters + kRenSlots;
    }
    ProjectOut po{c->splat, c->depth, c->bin, c->tiles, c->dkey[0], c->dval[0], c->rcounters};
    {
        Stage st(c, V3DG_STAGE_PROJECT);
        launch_project(c->stream, c->fdev, sc->attribs(), (int)sc->precision, (int)sc->sh_degree, sel.slot_row,
                       sel.slot_inst, n_dev, S, c->itab, po);
    }
    if (sc->pool_clusters) HIP_TRY(hipEventRecord(sc->ev_proj, c->stream));
    const bool depth_first = capacity || c->sort_mode == V3DG_SORT_DEPTH_FIRST;
    fi->depth_first = depth_first;
    if (depth_first) {
        // stable sort of the visible slots by FP32 depth bits: the culled ones
        // (key 0xffffffff) are counted by the histogram and left out by the
        // first pass, so the later passes and every step after them take the
        // first n - culled ranks only
        {
            Stage st(c, V3DG_STAGE_DEPTH_SORT);
            launch_sort_hist<uint32_t>(c->stream, c->dkey[0], n_dev, S, 4, c->rcounters + kRenHistDepth,
                                       c->rcounters + kRenCulled);
        }
        int cur = 0;
        for (int p = 0; p < 4; ++p) {
            Stage st(c, V3DG_STAGE_DEPTH_SORT);
            launch_sort_pass<uint32_t>(c->stream, c->dkey[cur], c->dval[cur], c->dkey[cur ^ 1], c->dval[cur ^ 1],
                                       p == 0 ? n_dev : c->rcounters + kRenDepthKept, S, p,
                                       c->rcounters + kRenHistDepth, c->sort_status, &c->fdev->epoch, (uint32_t)p,
                                       c->rcounters + kRenTicketDepth + p, c->rcounters + kRenErr, S >= kSortWideFrom,
                                       -1, kRadixBits, p == 0 ? c->rcounters + kRenCulled : nullptr,
                                       p == 0 ? c->rcounters + kRenDepthKept : nullptr);
            cur ^= 1;
        }
    }
    {
        Stage st(c, V3DG_STAGE_SCAN);
        // the depth sort left the culled slots out (the histogram counted them)
        const uint32_t *n_culled = depth_first ? c->rcounters + kRenCulled : nullptr;
        launch_scan_tiles(c->stream, c->tiles, depth_first ? c->dval[0] : nullptr, n_dev, n_culled, S, c->offsets,
                          c->scan_status, c->rcounters, capacity ? c->cap_keys : 0xffffffffull);
    }
    uint64_t KL;  // key bound of the launches below
    if (!capacity) {
        // one wait per frame: slot and key counts decide the launch sizes below
        HIP_TRY(hipMemcpyAsync(c->pinned, c->rcounters, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(c->pinned + 8, sel.counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        const uint32_t err = c->pinned[kRenErr] | c->pinned[8 + kSelErr];
        const uint64_t K = (uint64_t)c->pinned[kRenKeysLo] | ((uint64_t)c->pinned[kRenKeysHi] << 32);
        fi->N = c->pinned[8 + kSelNGaussians];
        fi->n_visible = c->pinned[kRenVisible];
        fi->n_sel_clusters = c->pinned[8 + kSelNClusters];
        if (err & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
        if ((err & (kErrOverflow | kErrKeyCap)) || K >= 0xffffffffull)
            return fail(V3DG_ERR_CAPACITY, "frame needs %llu keys; the limit is 2^32-1", (unsigned long long)K);
        if ((rc = ensure_keys(c, K))) return rc;
        if ((rc = ensure_chunks(c, K))) return rc;
        fi->K = K;
        KL = K;
    } else {
        KL = c->cap_keys;
    }
    const uint32_t *k_dev = capacity ? c->rcounters + kRenKeysEff : nullptr;
    // chunk records the plan may use (each tile of a bin walks the bin's list)
    const uint64_t max_chunks = capacity ? c->cap_chunks : chunk_bound(KL, c->chunk_shift);
    const ChunkPlan cp{c->chunk_shift};
    const uint32_t n_bins = cam.bins_x * cam.bins_y;
    const uint32_t bin_bits = std::max<uint32_t>(bits_for(n_bins), 1);
    int buf = 0;
    uint32_t passes = 0;
    uint32_t key_bits;
    if (depth_first) {
        key_bits = bin_bits;
        if (n_bins <= kBinKey16Max)
            tile_keys<uint16_t>(c, n_dev, S, k_dev, KL, key_bits, cam.tiles_x, n_tiles, cam.bins_x, max_chunks, &buf,
                                &passes, pub);
        else
            tile_keys<uint32_t>(c, n_dev, S, k_dev, KL, key_bits, cam.tiles_x, n_tiles, cam.bins_x, max_chunks, &buf,
                                &passes, pub);
    } else {
        {
            Stage st(c, V3DG_STAGE_EMIT);
            launch_emit64(c->stream, n_dev, S, c->tiles, c->offsets, c->bin, c->fdev, c->cap_keys, c->keys[0],
                          c->vals[0], c->rcounters + kRenErr);
        }
        key_bits = 32 + bin_bits;
        if (KL > 0) run_sort<uint64_t>(c, c->keys, c->vals, k_dev, KL, key_bits, 0, &buf, &passes, false);
        {
            Stage st(c, V3DG_STAGE_RANGES);
            launch_tile_ranges<uint64_t>(c->stream, c->keys[buf], c->rcounters + kRenKeysEff, 32, cam.tiles_x,
                                         n_tiles, cam.bins_x, c->ranges, c->cbase, c->items, c->rounds,
                                         c->tiles_cap, c->cbase + c->tiles_cap, c->rcounters, max_chunks, cp);
        }
    }
    {
        Stage st(c, V3DG_STAGE_BLEND);
        launch_blend(c->stream, c->fdev, cam.tiles_x, cam.tiles_y, c->splat, c->vals[buf], c->ranges, c->cbase,
                     c->items, c->rounds, c->tiles_cap, c->cbase + c->tiles_cap, c->rcounters, max_chunks, max_chunks,
                     c->scratch, c->pend,
                     c->need, c->stopm, c->rewalk, c->pairs_dev, c->pair_count, cp);
        // a frame whose keys did not fit is blended from its depth-sorted slots
        if (pub.fallback && depth_first)
            launch_blend_all(c->stream, c->fdev, n_tiles, c->splat, c->dval[0], c->rcounters, c->pairs_dev,
                             c->pair_count);
    }
    HIP_TRY(hipGetLastError());
    fi->key_bits = key_bits;
    fi->passes = passes;
    fi->buf = buf;
    return V3DG_OK;
}

void record_frame(Ctx *c, const FrameInfo &fi, uint64_t pixels)
{
    c->acc.frames += 1;
    c->acc.sel_clusters += fi.n_sel_clusters;
    c->acc.slots += fi.N;
    c->acc.visible += fi.n_visible;
    c->acc.keys += fi.K;
    c->acc.tiles += fi.n_tiles;
    c->acc.pixels += pixels;
    c->acc.sort_passes += fi.passes;
    if (fi.depth_first) c->acc.depth_sorts += 1;
    c->last.n_slots = fi.N;
    c->last.n_keys = fi.K;
    c->last.n_tiles = fi.n_tiles;
    c->last.n_bins = fi.n_bins;
    c->last.key_bits = fi.key_bits;
    c->last.sort_mode = fi.depth_first ? V3DG_SORT_DEPTH_FIRST : V3DG_SORT_KEYS64;
    c->last.sort_passes = fi.passes;
    c->last_buf = fi.buf;
}

// Reads the records of finished capacity-sized frames, oldest first (all of
// them, waiting, when block is set): their counts go to the profile and the
// frame stats, and the most keys seen decides the next capacity.
int drain_records(v3dg_scene *s, bool block)
{
    while (s->rec_n > 0) {
        const uint32_t slot = s->rec_head;
        if (block) {
            HIP_TRY(hipEventSynchronize(s->rec_ev[slot]));
        } else {
            const hipError_t q = hipEventQuery(s->rec_ev[slot]);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return fail(V3DG_ERR_HIP, "frame failed: %s", hipGetErrorString(q));
        }
        const volatile FrameRec &r = s->rec_h[slot];
        if (r.seq != s->rec_want[slot]) return fail(V3DG_ERR_DEVICE, "a frame did not publish its counts");
        const uint64_t K = (uint64_t)r.keys_lo | ((uint64_t)r.keys_hi << 32);
        s->keys_seen = std::max(s->keys_seen, K);
        s->acc.keys += K;
        s->acc.visible += r.visible;
        s->acc.slots += r.n_slots;
        s->acc.sel_clusters += r.n_clusters;
        s->last.n_keys = K;
        s->last.n_slots = r.n_slots;
        s->last_keycap = (r.err & kErrKeyCap) != 0;
        s->rend_err |= r.err & (kErrSpin | kErrOverflow);
        s->rec_head = (slot + 1) % Ctx::kRecRing;
        s->rec_n -= 1;
    }
    return V3DG_OK;
}

// Key buffers (and chunk records) for frames of n_tiles tiles sized by
// capacity: twice the most keys seen, and at least kRenderKeysPerPixel keys
// per pixel up to kRenderKeysFloorMax keys.  Grows only (a growth waits for
// the frames in flight).
constexpr uint64_t kRenderKeysPerPixel = 48;
constexpr uint64_t kRenderKeysFloorMax = 1ull << 27;
int ensure_render_capacity(v3dg_scene *s, uint32_t n_tiles, uint64_t pixels)
{
    const uint64_t floor = std::min(kRenderKeysPerPixel * pixels, kRenderKeysFloorMax);
    const uint64_t want = std::min<uint64_t>(std::max(2 * s->keys_seen, floor), 0xfffff000ull);
    int rc;
    if (want > s->cap_keys && (rc = ensure_keys(s, want, true))) return rc;
    return ensure_chunks(s, s->cap_keys);
}

int render_impl(v3dg_scene *s, const v3dg_camera *c, const v3dg_selection *sel, float *image)
{
    CamArgs cam;
    int rc = make_cam(c, &cam);
    if (rc) return rc;
    if (!sel || sel->scene != s) return fail(V3DG_ERR_INVALID_ARG, "selection does not belong to this scene");
    if (!image) return fail(V3DG_ERR_INVALID_ARG, "image is NULL");
    if (s->pool_clusters && sel->stream_frame <= s->lru.max_evicted_stamp)
        return fail(V3DG_ERR_INVALID_ARG, "the selection's clusters were paged out by a later select: select again");
    HIP_TRY(hipSetDevice(s->device));
    const uint32_t n_tiles = cam.tiles_x * cam.tiles_y;
    const uint64_t pixels = (uint64_t)cam.width * cam.height;
    FrameInfo fi;
    const SelView sv{sel->counters, sel->slot_row, sel->slot_inst};
    if ((rc = drain_records(s, false))) return rc;
    if (s->sort_mode != V3DG_SORT_DEPTH_FIRST || s->rend_tiles != n_tiles) {
        // the first frame of an image size (or a 64-bit-key frame): sized
        // exactly after one host wait; it sets the capacity of later frames
        if ((rc = drain_records(s, true))) return rc;
        if ((rc = enqueue_frame(s, s, cam, image, sv, false, false, &fi))) return rc;
        record_frame(s, fi, pixels);
        s->last_keycap = false;
        s->keys_seen = std::max(s->keys_seen, fi.K);
        // the next frame of this size grows the buffers before it runs (not
        // now: this frame's sorted keys stay readable until then)
        if (s->sort_mode == V3DG_SORT_DEPTH_FIRST) s->rend_tiles = n_tiles;
        return V3DG_OK;
    }
    // later frames: no host wait; launches are sized by the capacity and the
    // kernels read their counts on the device
    if ((rc = ensure_render_capacity(s, n_tiles, pixels))) return rc;
    if (s->rec_n == Ctx::kRecRing) {  // a ring of frames in flight: wait for the oldest
        const uint32_t keep = s->rec_n;
        while (s->rec_n == keep)
            if ((rc = drain_records(s, true))) return rc;
    }
    if ((rc = ensure_itab(s, s->n_inst))) return rc;
    if ((rc = ensure_slots(s, s->cap_slots))) return rc;
    if ((rc = ensure_tiles(s, n_tiles))) return rc;
    epoch_advance(s);
    const uint32_t slot = (s->rec_head + s->rec_n) % Ctx::kRecRing;
    FramePub pub;
    pub.sel_counters = sel->counters;
    pub.rec = s->rec_d + slot;
    pub.seq = ++s->rec_seq;
    pub.fallback = true;
    s->rec_want[slot] = pub.seq;
    if ((rc = enqueue_frame(s, s, cam, image, sv, true, false, &fi, pub))) return rc;
    HIP_TRY(hipEventRecord(s->rec_ev[slot], s->stream));
    s->rec_n += 1;
    // counts that the host knows now; keys, slots and visible come with the record
    s->acc.frames += 1;
    s->acc.tiles += fi.n_tiles;
    s->acc.pixels += pixels;
    s->acc.sort_passes += fi.passes;
    s->acc.depth_sorts += 1;
    s->last.n_tiles = fi.n_tiles;
    s->last.n_bins = fi.n_bins;
    s->last.key_bits = fi.key_bits;
    s->last.sort_mode = V3DG_SORT_DEPTH_FIRST;
    s->last.sort_passes = fi.passes;
    s->last_buf = fi.buf;
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
    s->full_gid = gid;
    s->full_off = off;
    s->full_total = (uint32_t)acc;
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

// ---- cluster streaming ----------------------------------------------------
// Pages in every cluster with slots in a cut (gid, slot offsets, n clusters,
// total slots; host arrays) as a new paging frame: the page-replacement plan
// (PageLRU) assigns pages to the missing clusters; their page images are
// staged and copied in one transfer per stage_cap clusters and scattered into
// their pages on stream st.  V3DG_ERR_CAPACITY (nothing paged) when the cut
// needs more pages than the pool holds.
int page_in(v3dg_scene *s, hipStream_t st, const uint32_t *gid, const uint32_t *off, uint32_t n, uint32_t total)
{
    std::vector<uint32_t> ks, miss;
    ks.reserve(n);
    for (uint32_t c = 0; c < n; ++c)
        if ((c + 1 < n ? off[c + 1] : total) != off[c]) ks.push_back(gid[c] % s->NC);
    uint32_t touched = 0;
    if (!s->lru.plan(ks.data(), ks.size(), miss, touched))
        return fail(V3DG_ERR_CAPACITY, "the cut needs more resident clusters than the pool's %u", s->pool_clusters);
    std::vector<uint32_t> chunk;
    for (size_t i = 0; i < miss.size(); i += s->stage_cap) {
        const uint32_t m = (uint32_t)std::min<size_t>(s->stage_cap, miss.size() - i);
        // ascending clusters: a run of neighbours is one read from a page file
        chunk.assign(miss.begin() + i, miss.begin() + i + m);
        std::sort(chunk.begin(), chunk.end());
        for (uint32_t j = 0; j < m; ++j) s->ups_h[j] = make_uint4(chunk[j], s->lru.page_of(chunk[j]), s->h_count[chunk[j]], 0u);
        std::string ioerr;
        hipError_t e = hipSuccess;
        if (!s->pages.get(chunk.data(), m, s->stage_h, &ioerr)) {
            for (size_t q = i; q < miss.size(); ++q) s->lru.release(miss[q]);
            return fail(V3DG_ERR_IO, "paging in clusters failed: %s", ioerr.c_str());
        }
        e = hipMemcpyAsync(s->stage_d, s->stage_h, (uint64_t)m * s->stage_stride, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s->ups_d, s->ups_h, m * sizeof(uint4), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            launch_stream_scatter(st, s->stage_d, s->ups_d, m, s->stage_stride, s->geo_bytes, s->sh_bytes,
                                  s->n_sh, s->pos_planes, s->geo_planes, s->sh_planes, s->plane_stride, s->rowinfo);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // the staging buffers are reused
        if (e != hipSuccess) {  // the pages of this chunk and the rest hold nothing valid: free them
            for (size_t q = i; q < miss.size(); ++q) s->lru.release(miss[q]);
            return fail(V3DG_ERR_HIP, "paging in clusters failed: %s", hipGetErrorString(e));
        }
    }
    s->sstats.frames += 1;
    s->sstats.pages_in += miss.size();
    s->sstats.bytes_in += (uint64_t)miss.size() * s->page_bytes;
    s->sstats.evictions = s->lru.evictions;
    s->sstats.last_pages_in = miss.size();
    s->sstats.last_resident_used = touched + (uint32_t)miss.size();
    s->sstats.file_reads = s->pages.reads();
    return V3DG_OK;
}

void scene_release(v3dg_scene *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->sel_stream) (void)hipStreamSynchronize(s->sel_stream);
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
    dev_free(s->cull_dev);
    dev_free(s->stage_d);
    dev_free(s->ups_d);
    if (s->ev_proj) (void)hipEventDestroy(s->ev_proj);
    if (s->ev_sel) (void)hipEventDestroy(s->ev_sel);
    if (s->sel_stream) (void)hipStreamDestroy(s->sel_stream);
    if (s->stage_h) (void)hipHostFree(s->stage_h);
    if (s->ups_h) (void)hipHostFree(s->ups_h);
    s->pages.close();
    ctx_release(s);
}

}  // namespace

namespace {

// ---- sort primitive ---------------------------------------------------------
// Stable LSD sort of n (key, value) pairs by the low key_bits bits through the
// given temporaries: k2 / v2 (n entries each), status (look-back words for
// ceil(n / kSortPart) partitions) and ctr (kRenCounters words); status and
// ctr are cleared here by fill kernels.  Synchronises to read the error flag.
int sort_pairs_in(hipStream_t st, uint64_t *keys_dev, uint32_t *vals_dev, uint64_t n, uint32_t key_bits, uint64_t *k2,
                  uint32_t *v2, uint64_t *status, uint32_t *ctr)
{
    const int passes = (int)((key_bits + kRadixBits - 1) / kRadixBits);
    const uint64_t parts = (n + kSortPart - 1) / kSortPart;
    launch_fill_u32(st, reinterpret_cast<uint32_t *>(status), 2 * parts * kRadix, 0u);
    launch_fill_u32(st, ctr, kRenCounters, 0u);
    launch_sort_hist<uint64_t>(st, keys_dev, nullptr, n, passes, ctr + kRenHist);
    uint64_t *kb[2] = {keys_dev, k2};
    uint32_t *vb[2] = {vals_dev, v2};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        launch_sort_pass<uint64_t>(st, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], nullptr, n, p, ctr + kRenHist, status,
                                   nullptr, (uint32_t)(p + 1), ctr + kRenTicketSort + p, ctr + kRenErr, false);
        cur ^= 1;
    }
    if (cur == 1) {
        HIP_TRY(hipMemcpyAsync(keys_dev, k2, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(vals_dev, v2, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(&err, ctr + kRenErr, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(V3DG_ERR_HIP, "sort failed: %s", hipGetErrorString(e));
    if (err & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    return V3DG_OK;
}

// ---- scratch of the allocation-free sort --------------------------------------
// One fixed device array per GPU, laid out as the sort's temporaries for
// V3DG_SORT_NOALLOC_MAX pairs: alternate keys, alternate values, look-back
// words and counters.  Its device address is looked up once per device (the
// name itself is a host-side stand-in) and kept; every call on that device
// shares the array.
constexpr uint64_t kNaMaxParts = (V3DG_SORT_NOALLOC_MAX + kSortPart - 1) / kSortPart;
constexpr uint64_t kNaKeysOff = 0;
constexpr uint64_t kNaValsOff = kNaKeysOff + 8ull * V3DG_SORT_NOALLOC_MAX;
constexpr uint64_t kNaStatusOff = (kNaValsOff + 4ull * V3DG_SORT_NOALLOC_MAX + 255) / 256 * 256;
constexpr uint64_t kNaCtrOff = kNaStatusOff + 8ull * kNaMaxParts * kRadix;
constexpr uint64_t kNaBytes = (kNaCtrOff + 4ull * kRenCounters + 255) / 256 * 256;
static_assert(kNaBytes <= (16ull << 20), "the allocation-free sort's scratch stays below 16 MiB");

}  // namespace

static __device__ __align__(256) uint8_t scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
uint8_t *g_na_ptr[kNaMaxDevices] = {};

int noalloc_scratch(uint8_t **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(V3DG_ERR_INVALID_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(V3DG_ERR_HIP, "scratch address lookup failed: %s", hipGetErrorString(e));
        g_na_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_na_ptr[dev];
    return V3DG_OK;
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
    return v3dg_load_hierarchy_streamed(d, instances_3x4, n_instances, hip_stream, flags, 0, out);
}

int v3dg_load_hierarchy_streamed(const v3dg_hierarchy_desc *d, const double *instances_3x4, uint32_t n_instances,
                                 void *hip_stream, uint32_t flags, uint32_t pool_clusters, v3dg_scene **out)
{
    return v3dg_load_hierarchy_streamed_file(d, instances_3x4, n_instances, hip_stream, flags, pool_clusters, nullptr,
                                             0, out);
}

int v3dg_load_hierarchy_streamed_file(const v3dg_hierarchy_desc *d, const double *instances_3x4,
                                      uint32_t n_instances, void *hip_stream, uint32_t flags, uint32_t pool_clusters,
                                      const char *page_file, uint32_t file_flags, v3dg_scene **out)
{
    g_err.clear();
    if (!d || !out) return fail(V3DG_ERR_INVALID_ARG, "desc and out must be non-NULL");
    if (pool_clusters >= (1u << 26)) return fail(V3DG_ERR_INVALID_ARG, "pool_clusters must be < 2^26");
    if (page_file && (!page_file[0] || pool_clusters == 0))
        return fail(V3DG_ERR_INVALID_ARG, "a page file needs a non-empty path and pool_clusters > 0");
    if (file_flags & ~(V3DG_PAGE_FILE_DIRECT | V3DG_PAGE_FILE_KEEP))
        return fail(V3DG_ERR_INVALID_ARG, "unknown page file flags 0x%x", file_flags);
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
    const uint64_t ps = ((uint64_t)NR + 63) / 64 * 64;  // host plane stride
    s->precision = d->precision;
    const size_t geo_bytes = d->precision == V3DG_FP32 ? 4 : 2, sh_bytes = geo_bytes;
    auto bail = [&](int code) {
        scene_release(s);
        delete s;
        return code;
    };
    s->pool_clusters = std::min(pool_clusters, NC);
    const bool streamed = s->pool_clusters > 0;
    s->plane_stride = streamed ? 64ull * s->pool_clusters : ps;
    const uint64_t dps = s->plane_stride;
    if ((rc = dev_alloc(&s->pos_planes, 3 * dps))) return bail(rc);
    if ((rc = dev_alloc((uint8_t **)&s->geo_planes, kGeoPlanes * dps * geo_bytes))) return bail(rc);
    if ((rc = dev_alloc((uint8_t **)&s->sh_planes, 3ull * ncoef * dps * sh_bytes))) return bail(rc);
    if ((rc = dev_alloc(&s->self_sph, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->par_sph, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->rowinfo, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->cull_dev, NC))) return bail(rc);
    if ((rc = dev_alloc(&s->T_dev, 12ull * n_instances))) return bail(rc);
    if ((rc = dev_alloc(&s->scale_dev, n_instances))) return bail(rc);
    if ((rc = ctx_init(s, s->device, s->stream))) return bail(rc);
    if ((rc = ensure_itab(s, n_instances))) return bail(rc);
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
        for (uint32_t k = 0; k < NC; ++k) ri[k] = make_uint2(streamed ? 0u : d->first_row[k], d->count[k]);
        if (streamed) {  // page images of the clusters; an empty pool
            s->geo_bytes = (uint32_t)geo_bytes;
            s->sh_bytes = (uint32_t)sh_bytes;
            s->n_sh = 3u * (uint32_t)ncoef;
            s->page_bytes = 3u * 256u + (uint32_t)kGeoPlanes * 64u * s->geo_bytes + s->n_sh * 64u * s->sh_bytes;
            std::string ioerr;
            if (page_file) {
                if (!s->pages.init_file(page_file, NC, s->page_bytes, (file_flags & V3DG_PAGE_FILE_DIRECT) != 0,
                                        (file_flags & V3DG_PAGE_FILE_KEEP) != 0, &ioerr))
                    return bail(fail(V3DG_ERR_IO, "page file %s: %s", page_file, ioerr.c_str()));
            } else {
                s->pages.init_memory(NC, s->page_bytes);
            }
            s->stage_stride = s->pages.stride();
            s->sstats.tier = s->pages.tier();
            std::vector<uint8_t> image(s->page_bytes);
            for (uint32_t k = 0; k < NC; ++k) {
                uint8_t *img = image.data();
                std::memset(img, 0, image.size());
                const uint64_t r0 = d->first_row[k], cnt = d->count[k];
                for (int j = 0; j < 3; ++j) std::memcpy(img + 256u * j, &hpos[j * ps + r0], cnt * 4);
                uint8_t *g = img + 768;
                for (int j = 0; j < kGeoPlanes; ++j)
                    std::memcpy(g + (uint64_t)j * 64 * geo_bytes, (const uint8_t *)src_geo + (j * ps + r0) * geo_bytes,
                                cnt * geo_bytes);
                uint8_t *h = g + (uint64_t)kGeoPlanes * 64 * geo_bytes;
                for (uint32_t j = 0; j < s->n_sh; ++j)
                    std::memcpy(h + (uint64_t)j * 64 * sh_bytes, (const uint8_t *)src_sh + (j * ps + r0) * sh_bytes,
                                cnt * sh_bytes);
                if (!s->pages.put(k, img, &ioerr)) return bail(fail(V3DG_ERR_IO, "%s", ioerr.c_str()));
            }
            if (!s->pages.seal(&ioerr)) return bail(fail(V3DG_ERR_IO, "%s", ioerr.c_str()));
            const uint32_t P = s->pool_clusters;
            s->lru.init(NC, P);
            s->stage_cap = std::min<uint32_t>(P, 2048u);
            s->sstats.pool_clusters = P;
            if (hipHostMalloc((void **)&s->stage_h, (uint64_t)s->stage_cap * s->stage_stride, hipHostMallocDefault) !=
                    hipSuccess ||
                hipHostMalloc((void **)&s->ups_h, s->stage_cap * sizeof(uint4), hipHostMallocDefault) != hipSuccess) {
                return bail(fail(V3DG_ERR_OOM, "pinned staging allocation failed"));
            }
            if ((rc = dev_alloc(&s->stage_d, (uint64_t)s->stage_cap * s->stage_stride))) return bail(rc);
            if ((rc = dev_alloc(&s->ups_d, s->stage_cap))) return bail(rc);
            // non-blocking: no implicit wait for work on the null stream (the
            // scene's stream may be it); ordering is by the two events alone
            if (hipStreamCreateWithFlags(&s->sel_stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->ev_proj, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s->ev_sel, hipEventDisableTiming) != hipSuccess)
                return bail(fail(V3DG_ERR_HIP, "stream or event creation failed"));
        }
        // view-cull table: sphere of each cluster's row means (FP64, radius
        // rounded up) and its largest scale (enlarged to cover FP16 storage)
        std::vector<CullRec> cr(NC);
        for (uint32_t k = 0; k < NC; ++k) {
            const uint64_t r0 = d->first_row[k], n = d->count[k];
            double c[3] = {0, 0, 0}, smax = 0.0;
            for (uint64_t r = r0; r < r0 + n; ++r)
                for (int j = 0; j < 3; ++j) {
                    c[j] += d->pos[3 * r + j];
                    smax = std::max(smax, (double)d->scale[3 * r + j]);
                }
            for (int j = 0; j < 3; ++j) c[j] /= (double)std::max<uint64_t>(n, 1);
            const float cf[3] = {(float)c[0], (float)c[1], (float)c[2]};
            double rad = 0.0;
            for (uint64_t r = r0; r < r0 + n; ++r) {
                double q = 0.0;
                for (int j = 0; j < 3; ++j) {
                    const double dd = (double)d->pos[3 * r + j] - (double)cf[j];
                    q += dd * dd;
                }
                rad = std::max(rad, std::sqrt(q));
            }
            cr[k].sph = make_float4(cf[0], cf[1], cf[2], round_up_f32(rad * (1.0 + 1e-6) + 1e-7));
            cr[k].smax = round_up_f32(smax * (1.0 + 1.0 / 1024.0));
        }
        e = hipSuccess;
        if (!streamed) {
            e = hipMemcpy(s->pos_planes, hpos.data(), hpos.size() * sizeof(float), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(s->geo_planes, src_geo, hgeo.size() * geo_bytes, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(s->sh_planes, src_sh, hsh.size() * sh_bytes, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipMemcpy(s->self_sph, self.data(), self.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->par_sph, par.data(), par.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->rowinfo, ri.data(), ri.size() * sizeof(uint2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->cull_dev, cr.data(), cr.size() * sizeof(CullRec), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->T_dev, instances_3x4, 12ull * n_instances * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->scale_dev, inst_scale.data(), n_instances * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(V3DG_ERR_HIP, "upload failed: %s", hipGetErrorString(e)));
    }
    *out = s;
    return V3DG_OK;
}

int v3dg_get_stream_stats(const v3dg_scene *s, v3dg_stream_stats *out)
{
    g_err.clear();
    if (!s || !out) return fail(V3DG_ERR_INVALID_ARG, "scene and out must be non-NULL");
    *out = s->sstats;
    out->resident = s->pool_clusters ? s->lru.resident() : 0u;
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

// Streamed scenes: read a selected cut back (synchronises) and page it in.
static int stream_cut(v3dg_scene *s, v3dg_selection *sel)
{
    HIP_TRY(hipMemcpyAsync(s->pinned + 8, sel->counters, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s->sel_stream));
    HIP_TRY(hipStreamSynchronize(s->sel_stream));
    if (s->pinned[8 + kSelErr] & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    const uint32_t n = s->pinned[8 + kSelNClusters], total = s->pinned[8 + kSelNGaussians];
    s->cut_gid.resize(n);
    s->cut_off.resize(n);
    if (n) {  // on the select stream only: the previous render's later stages go on meanwhile
        HIP_TRY(hipMemcpyAsync(s->cut_gid.data(), sel->gid, n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s->sel_stream));
        HIP_TRY(hipMemcpyAsync(s->cut_off.data(), sel->slot_off, n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               s->sel_stream));
        HIP_TRY(hipStreamSynchronize(s->sel_stream));
    }
    const int rc = page_in(s, s->sel_stream, s->cut_gid.data(), s->cut_off.data(), n, total);
    if (rc) return rc;
    sel->stream_frame = s->lru.frame;
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
    // a streamed scene selects on its own stream, once the frame before has
    // been projected (it rewrites the instance table, the selection and pages)
    const hipStream_t qs = s->pool_clusters ? s->sel_stream : s->stream;
    if (s->pool_clusters) HIP_TRY(hipStreamWaitEvent(qs, s->ev_proj, 0));
    {
        Stage st(s, V3DG_STAGE_SETUP, qs);
        launch_frame_setup(qs, cam, nullptr, nullptr, false, false, s->T_dev, s->scale_dev, s->n_inst, s->itab,
                           sel->clear_block, (uint64_t)kSelCounters + 2 * sel->n_parts);
    }
    {
        Stage st(s, V3DG_STAGE_SELECT, qs);
        launch_select(qs, make_selreq(s, s->itab, K, tau, sel, cam, s->culling));
    }
    if (s->pool_clusters) {  // streamed: read the cut back, page in what it lacks
        rc = stream_cut(s, sel);
        if (rc) {
            sel->stream_frame = 0;  // its cut is not expanded: never renderable
            (void)hipStreamSynchronize(s->sel_stream);
            if (fresh) {
                sel_release(sel);
                delete sel;
            }
            return rc;
        }
    }
    {
        Stage st(s, V3DG_STAGE_EXPAND, qs);
        launch_expand(qs, sel->gid, sel->slot_off, s->rowinfo, s->NC, sel->counters,
                      (uint32_t)std::min<uint64_t>(sel->cap_tests, 0xffffffffull), sel->slot_row, sel->slot_inst);
    }
    if (s->pool_clusters) {  // whatever comes next on the scene's stream waits for this select
        HIP_TRY(hipEventRecord(s->ev_sel, qs));
        HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_sel, 0));
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
    if (s->pool_clusters) {  // streamed: page in every leaf, then place the slots on the pages
        v3dg_selection *f = s->full;
        if ((rc = page_in(s, s->stream, s->full_gid.data(), s->full_off.data(), (uint32_t)s->full_gid.size(),
                          s->full_total)))
            return rc;
        f->stream_frame = s->lru.frame;
        launch_expand(s->stream, f->gid, f->slot_off, s->rowinfo, s->NC, f->counters, (uint32_t)s->full_gid.size(),
                      f->slot_row, f->slot_inst);
        HIP_TRY(hipGetLastError());
    }
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
        if (sel->scene->sel_stream) (void)hipStreamSynchronize(sel->scene->sel_stream);
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
    int rc = drain_records(s, true);
    if (rc) return rc;
    static_assert(kRenErr < 32 && kRenFp64 < 32 && kRenConicClamp < 32, "frame stats read the first 32 counters");
    uint32_t ctr[32] = {0};
    if (s->rcounters) HIP_TRY(hipMemcpy(ctr, s->rcounters, sizeof(ctr), hipMemcpyDeviceToHost));
    const uint32_t err = ctr[kRenErr] | s->rend_err;
    s->rend_err = 0;
    if (err & kErrSpin) return fail(V3DG_ERR_DEVICE, "a look-back wait expired on the device");
    if (err & kErrOverflow) return fail(V3DG_ERR_DEVICE, "tile counting and key emission disagreed");
    *out = s->last;
    out->n_fp64_conics = ctr[kRenFp64];
    out->n_conics_clamped = ctr[kRenConicClamp];
    return V3DG_OK;
}

int v3dg_copy_projection(v3dg_scene *s, float *mean2, float *conic, float *rgb, float *opacity, float *depth,
                         uint32_t *tiles, uint64_t cap, uint64_t *n_out)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    int rc = drain_records(s, true);
    if (rc) return rc;
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
    if (s->pool_clusters) return fail(V3DG_ERR_INVALID_ARG, "a streamed scene keeps its rows on the host");
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
    int rc = drain_records(s, true);
    if (rc) return rc;
    if (s->last_keycap)
        return fail(V3DG_ERR_CAPACITY, "the last frame's keys exceeded its key buffers: it was blended without them");
    const uint64_t n = s->last.n_keys;
    if (n_out) *n_out = n;
    if (n > cap) return fail(V3DG_ERR_CAPACITY, "%llu keys do not fit in %llu", (unsigned long long)n, (unsigned long long)cap);
    if (n == 0) return V3DG_OK;
    std::vector<uint32_t> v(n);
    HIP_TRY(hipMemcpy(v.data(), s->vals[s->last_buf], n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (keys) {
        if (s->last.sort_mode == V3DG_SORT_KEYS64) {
            HIP_TRY(hipMemcpy(keys, s->keys[s->last_buf], n * sizeof(uint64_t), hipMemcpyDeviceToHost));
        } else {  // bin ids (16 bits on grids of at most kBinKey16Max bins); the depth bits come from the slot
            std::vector<uint32_t> tk(n), dp(s->last.n_slots);
            if (s->last.n_bins <= kBinKey16Max) {
                std::vector<uint16_t> t16(n);
                HIP_TRY(hipMemcpy(t16.data(), s->keys[s->last_buf], n * sizeof(uint16_t), hipMemcpyDeviceToHost));
                for (uint64_t i = 0; i < n; ++i) tk[i] = t16[i];
            } else {
                HIP_TRY(hipMemcpy(tk.data(), s->keys[s->last_buf], n * sizeof(uint32_t), hipMemcpyDeviceToHost));
            }
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

namespace {
// log2 of a later-chunk size: a power of two of 2^kChunkShiftMin ..
// 2^kChunkShiftMax keys
bool chunk_shift_of(uint32_t keys, uint32_t *shift)
{
    for (uint32_t k = kChunkShiftMin; k <= kChunkShiftMax; ++k)
        if (keys == (1u << k)) {
            *shift = k;
            return true;
        }
    return false;
}
}  // namespace

int v3dg_set_chunk_keys(v3dg_scene *s, uint32_t keys)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    uint32_t shift = 0;
    if (!chunk_shift_of(keys, &shift))
        return fail(V3DG_ERR_INVALID_ARG, "chunk_keys must be 1024, 2048 or 4096 (got %u)", keys);
    s->chunk_shift = shift;
    return V3DG_OK;
}

int v3dg_set_culling(v3dg_scene *s, int on)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    s->culling = on != 0;
    return V3DG_OK;
}

constexpr size_t kEventPoolWarm = 512;  // two events per timed stage and frame: 256 frames of one stage

int v3dg_set_profiling(v3dg_scene *s, int stage_mask)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "scene is NULL");
    s->profiling = (uint32_t)stage_mask & V3DG_PROFILE_ALL;
    s->pair_count = (stage_mask & V3DG_PROFILE_PAIR_AUDIT) ? 2 : (stage_mask & V3DG_PROFILE_PAIRS) ? 1 : 0;
    // events for the timed stages are created here rather than inside the
    // frames being timed (creating one costs far more than recording it)
    if (s->profiling || s->pair_count) {
        HIP_TRY(hipSetDevice(s->device));
        while (s->ev_pool.size() < kEventPoolWarm) {
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreate(&e));
            s->ev_pool.push_back(e);
        }
    }
    return V3DG_OK;
}

int v3dg_collect_profile(v3dg_scene *s, v3dg_profile *out)
{
    g_err.clear();
    if (!s || !out) return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipStreamSynchronize(s->stream));
    int rc = drain_records(s, true);
    if (rc) return rc;
    unsigned long long pairs[2 * kPairSlots] = {0};
    HIP_TRY(hipMemcpy(pairs, s->pairs_dev, sizeof(pairs), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(s->pairs_dev, 0, sizeof(pairs)));
    v3dg_profile p = s->acc;
    p.pairs = p.pairs_taken = 0;
    for (uint32_t k = 0; k < kPairSlots; ++k) {
        p.pairs += pairs[2 * k];
        p.pairs_taken += pairs[2 * k + 1];
    }
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
    const uint64_t parts = (n + kSortPart - 1) / kSortPart;
    uint64_t *k2 = nullptr, *status = nullptr;
    uint32_t *v2 = nullptr, *ctr = nullptr;
    int rc = dev_alloc(&k2, n);
    if (!rc) rc = dev_alloc(&v2, n);
    if (!rc) rc = dev_alloc(&status, parts * kRadix);
    if (!rc) rc = dev_alloc(&ctr, (uint64_t)kRenCounters);
    if (!rc) rc = sort_pairs_in((hipStream_t)hip_stream, keys_dev, vals_dev, n, key_bits, k2, v2, status, ctr);
    dev_free(k2);
    dev_free(v2);
    dev_free(status);
    dev_free(ctr);
    return rc;
}

int v3dg_sort_pairs_noalloc(uint64_t *keys_dev, uint32_t *vals_dev, uint64_t n, uint32_t key_bits, void *hip_stream)
{
    g_err.clear();
    if (key_bits < 1 || key_bits > 64) return fail(V3DG_ERR_INVALID_ARG, "key_bits must be 1..64");
    if (n > V3DG_SORT_NOALLOC_MAX)
        return fail(V3DG_ERR_CAPACITY, "%llu pairs exceed the %u this entry point sorts without allocating",
                    (unsigned long long)n, (unsigned)V3DG_SORT_NOALLOC_MAX);
    if (n == 0) return V3DG_OK;
    if (!keys_dev || !vals_dev) return fail(V3DG_ERR_INVALID_ARG, "NULL buffer");
    uint8_t *base = nullptr;
    int rc = noalloc_scratch(&base);
    if (rc) return rc;
    uint64_t *k2 = reinterpret_cast<uint64_t *>(base + kNaKeysOff);
    uint32_t *v2 = reinterpret_cast<uint32_t *>(base + kNaValsOff);
    uint64_t *status = reinterpret_cast<uint64_t *>(base + kNaStatusOff);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(base + kNaCtrOff);
    return sort_pairs_in((hipStream_t)hip_stream, keys_dev, vals_dev, n, key_bits, k2, v2, status, ctr);
}

}  // extern "C"

// =============================================================================
// serving: render contexts, admission under an HBM budget, batched selection
// =============================================================================
namespace {

double now_ms(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct SrvReq {
    uint64_t ticket = 0;
    uint32_t scene = 0;
    CamArgs cam{};
    float K = 0.f, tau = 0.f;
    float *image = nullptr;
    double submit_ms = 0.0, admit_ms = 0.0;
    uint32_t retries = 0;
    bool full = false;  // every leaf, no selection (v3dg_server_submit_full)
};

using ShapeKey = std::tuple<uint32_t, uint32_t, uint32_t, bool>;  // scene, width, height, full detail

struct SrvCtx : Ctx {
    v3dg_selection sel;                 // selection buffers for the largest scene
    bool busy = false;
    SrvReq req;
    hipEvent_t done = nullptr;
    FrameDev *stage = nullptr;          // pinned staging of the frame header
    uint64_t generation = 0;            // advanced whenever a buffer is reallocated
    std::map<ShapeKey, std::pair<hipGraphExec_t, uint64_t>> graphs;
    uint64_t bytes = 0;                 // device memory held
};

struct BatchSlot {
    SelSetup *h_setup = nullptr;
    SelReq *h_req = nullptr;
    SelSetup *d_setup = nullptr;
    SelReq *d_req = nullptr;
    uint32_t *d_ticket = nullptr;
    hipEvent_t ev = nullptr;            // recorded after the batch's launches
    bool used = false;
};

constexpr int kBatchRing = 8;

}  // namespace

struct v3dg_server {
    int device = 0;
    std::vector<v3dg_scene *> scenes;
    v3dg_server_config cfg{};
    uint32_t chunk_shift = kChunkShiftServer;  // chunk sizes of the contexts' plans
    hipStream_t sched = nullptr;        // batched selection
    std::vector<SrvCtx *> ctx;
    std::deque<SrvReq> queue;
    BatchSlot ring[kBatchRing];
    int ring_next = 0;
    uint64_t next_ticket = 1;
    uint64_t max_tests = 0, max_slots = 0;
    uint32_t max_inst = 0;
    std::map<ShapeKey, uint64_t> keys_seen;
    std::chrono::steady_clock::time_point t0;
    v3dg_server_stats st{};
};

namespace {

// device bytes per slot: splat record 48, binning record 32, depth 4, bins
// touched 4, key offset 4, large-splat list 4, depth-sort keys and values 16
constexpr uint64_t kSlotBytes = 48 + 32 + 4 + 4 + 4 + 4 + 16;

uint64_t ctx_bytes(const SrvCtx *c)
{
    uint64_t b = c->ws_slots * kSlotBytes;
    b += (uint64_t)c->itab_cap * sizeof(InstRec) + sizeof(FrameDev) + 8;
    b += c->rclear_words * 4 + (uint64_t)c->tiles_cap * (8 + 4 * kChunkRounds);
    b += c->cap_keys * 24 + c->sort_status_parts * kRadix * 8;
    b += c->cap_chunks * (8 + 256 * 16 + 256 * 4 + 4 + 32 + 8);
    b += c->sel.cap_tests * 8 + ((uint64_t)kSelCounters + 2 * c->sel.n_parts) * 4 + c->sel.cap_slots * 8;
    return b;
}

// bytes of a context before any image size or key count is provisioned
uint64_t ctx_base_bytes(const SrvCtx *c)
{
    return c->ws_slots * kSlotBytes + (uint64_t)c->itab_cap * sizeof(InstRec) +
           sizeof(FrameDev) + 8 + c->sel.cap_tests * 8 + ((uint64_t)kSelCounters + 2 * c->sel.n_parts) * 4 +
           c->sel.cap_slots * 8;
}

// bytes context c (nullptr: a new one) would add to hold K keys over n_tiles tiles
uint64_t growth_bytes(const SrvCtx *c, uint64_t K, uint32_t n_tiles, uint32_t chunk_shift)
{
    const uint64_t keys = c ? c->cap_keys : 0, tiles = c ? c->tiles_cap : 0, chunks = c ? c->cap_chunks : 0;
    uint64_t g = 0;
    const uint64_t K2 = std::max(K, keys);
    g += (K2 - keys) * 24 + ((K2 - keys + kSortPart - 1) / kSortPart) * 3 / 2 * kRadix * 8;
    const uint64_t T2 = std::max<uint64_t>(std::max<uint64_t>(n_tiles, 8160), tiles);
    g += (T2 - tiles) * (16 + 4 * kChunkRounds);
    const uint64_t ch = chunk_bound(K2, chunk_shift);
    if (ch > chunks) g += (ch + ch / 2 - chunks) * (8 + 256 * 16 + 256 * 4 + 4 + 32 + 8);
    return g;
}

void srv_account(v3dg_server *s)
{
    uint64_t tot = 0;
    for (auto *c : s->ctx) {
        c->bytes = ctx_bytes(c);
        tot += c->bytes;
    }
    s->st.workspace_bytes = tot;
    s->st.peak_workspace_bytes = std::max(s->st.peak_workspace_bytes, tot);
}

void drop_graphs(SrvCtx *c)
{
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second.first);
    c->graphs.clear();
}

void srv_ctx_free(SrvCtx *c)
{
    drop_graphs(c);
    sel_release(&c->sel);
    if (c->done) (void)hipEventDestroy(c->done);
    if (c->stage) (void)hipHostFree(c->stage);
    ctx_release(c);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// key capacity to provision for a request shape
uint64_t keys_estimate(v3dg_server *s, const ShapeKey &k, uint64_t pixels)
{
    auto it = s->keys_seen.find(k);
    const uint64_t kpp = s->cfg.keys_per_pixel ? s->cfg.keys_per_pixel : 24;
    uint64_t e = it != s->keys_seen.end() ? it->second + it->second / 4 : pixels * kpp;
    e = std::max<uint64_t>(e, 1u << 16);
    return std::min<uint64_t>(e, 0xfffff000ull);
}

// Grow c to serve a frame of n_tiles tiles with K keys.  Returns 1 when a
// buffer was reallocated (captured graphs of c are then stale).
int srv_provision(SrvCtx *c, uint32_t n_inst, uint32_t n_tiles, uint64_t K, bool *changed)
{
    const uint64_t before[4] = {c->itab_cap, c->tiles_cap, c->cap_keys, c->cap_chunks};
    const uint64_t parts_before = c->sort_status_parts;
    int rc;
    if ((rc = ensure_itab(c, n_inst))) return rc;
    if ((rc = ensure_tiles(c, n_tiles))) return rc;
    if ((rc = ensure_keys(c, K, true))) return rc;
    if ((rc = ensure_chunks(c, c->cap_keys))) return rc;
    const uint64_t after[4] = {c->itab_cap, c->tiles_cap, c->cap_keys, c->cap_chunks};
    *changed = std::memcmp(before, after, sizeof(before)) != 0 || parts_before != c->sort_status_parts;
    if (*changed) {
        ++c->generation;
        drop_graphs(c);
    }
    return V3DG_OK;
}

int srv_new_ctx(v3dg_server *s, SrvCtx **out)
{
    auto *c = new (std::nothrow) SrvCtx();
    if (!c) return fail(V3DG_ERR_OOM, "host allocation failed");
    c->chunk_shift = s->chunk_shift;
    hipStream_t st = nullptr;
    int rc = V3DG_OK;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) rc = fail(V3DG_ERR_HIP, "stream creation failed");
    if (!rc) rc = ctx_init(c, s->device, st);
    if (!rc) rc = sel_alloc_caps(&c->sel, s->max_tests, s->max_slots, st);
    if (!rc) rc = ensure_itab(c, s->max_inst);
    if (!rc) rc = ensure_slots(c, s->max_slots);
    if (!rc && hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess)
        rc = fail(V3DG_ERR_HIP, "event creation failed");
    if (!rc && hipHostMalloc((void **)&c->stage, sizeof(FrameDev), hipHostMallocDefault) != hipSuccess) {
        c->stage = nullptr;
        rc = fail(V3DG_ERR_OOM, "pinned allocation failed");
    }
    if (!rc) rc = hipStreamSynchronize(st) == hipSuccess ? V3DG_OK : fail(V3DG_ERR_HIP, "stream sync failed");
    if (rc) {
        srv_ctx_free(c);
        return rc;
    }
    *out = c;
    return V3DG_OK;
}

// the render chain of one request on its context, as a replayed graph or as
// direct launches (the selection has been written into c->sel)
int srv_launch(v3dg_server *s, SrvCtx *c, hipEvent_t sel_done)
{
    v3dg_scene *sc = s->scenes[c->req.scene];
    const CamArgs &cam = c->req.cam;
    // a full-detail request renders the scene's own list of every leaf (built
    // at submit, read-only, shared by the contexts)
    const v3dg_selection *src = c->req.full ? sc->full : &c->sel;
    const SelView sv{src->counters, src->slot_row, src->slot_inst};
    hipGraphExec_t exec = nullptr;
    if (s->cfg.use_graphs) {
        const ShapeKey key{c->req.scene, cam.width, cam.height, c->req.full};
        auto it = c->graphs.find(key);
        if (it != c->graphs.end() && it->second.second == c->generation) {
            exec = it->second.first;
        } else {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
            FrameInfo fi;
            const int rc = enqueue_frame(c, sc, cam, nullptr, sv, true, true, &fi);
            const hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (rc) return rc;
            if (e != hipSuccess) return fail(V3DG_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
            const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e2 != hipSuccess) return fail(V3DG_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e2));
            if (it != c->graphs.end()) (void)hipGraphExecDestroy(it->second.first);
            c->graphs[key] = {exec, c->generation};
            ++s->st.graph_captures;
        }
    }
    HIP_TRY(hipStreamWaitEvent(c->stream, sel_done, 0));
    c->stage->cam = cam;
    c->stage->image = c->req.image;
    HIP_TRY(hipMemcpyAsync(c->fdev, c->stage, offsetof(FrameDev, epoch), hipMemcpyHostToDevice, c->stream));
    epoch_advance(c);
    if (exec) {
        HIP_TRY(hipGraphLaunch(exec, c->stream));
        ++s->st.graph_launches;
    } else {
        FrameInfo fi;
        int rc = enqueue_frame(c, sc, cam, nullptr, sv, true, true, &fi);
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(c->pinned, c->rcounters, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->pinned + 8, src->counters, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipEventRecord(c->done, c->stream));
    c->busy = true;
    return V3DG_OK;
}

// one batched selection for the requests just admitted into ctxs[], then
// their render chains
int srv_dispatch(v3dg_server *s, const std::vector<SrvCtx *> &batch)
{
    if (batch.empty()) return V3DG_OK;
    BatchSlot &b = s->ring[s->ring_next];
    s->ring_next = (s->ring_next + 1) % kBatchRing;
    if (b.used) HIP_TRY(hipEventSynchronize(b.ev));  // its descriptors may be reused now
    uint32_t parts = 0, max_clear = 0, n = 0;
    for (size_t i = 0; i < batch.size(); ++i) {
        SrvCtx *c = batch[i];
        if (c->req.full) continue;  // renders the scene's list of leaves: nothing to select
        v3dg_scene *sc = s->scenes[c->req.scene];
        SelReq q = make_selreq(sc, c->itab, c->req.K, c->req.tau, &c->sel, c->req.cam, s->cfg.cull != 0);
        q.part_begin = parts;
        parts += q.nparts;
        b.h_req[n] = q;
        SelSetup su{};
        su.cam = c->req.cam;
        su.T = sc->T_dev;
        su.inst_scale = sc->scale_dev;
        su.itab = c->itab;
        su.clear = c->sel.clear_block;
        su.n_inst = sc->n_inst;
        su.n_clear = (uint32_t)(kSelCounters + 2 * q.nparts);
        max_clear = std::max(max_clear, su.n_clear);
        b.h_setup[n++] = su;
    }
    if (n > 0) {
        HIP_TRY(hipMemcpyAsync(b.d_setup, b.h_setup, n * sizeof(SelSetup), hipMemcpyHostToDevice, s->sched));
        HIP_TRY(hipMemcpyAsync(b.d_req, b.h_req, n * sizeof(SelReq), hipMemcpyHostToDevice, s->sched));
        launch_select_batch(s->sched, b.d_setup, b.d_req, n, parts, s->max_inst, max_clear, b.d_ticket);
        HIP_TRY(hipGetLastError());
        s->st.batches += 1;
        s->st.batched_requests += n;
    }
    HIP_TRY(hipEventRecord(b.ev, s->sched));
    b.used = true;
    for (SrvCtx *c : batch) {
        int rc = srv_launch(s, c, b.ev);
        if (rc) return rc;
    }
    return V3DG_OK;
}

}  // namespace

extern "C" {

int v3dg_server_create(v3dg_scene *const *scenes, uint32_t n_scenes, const v3dg_server_config *cfg,
                       v3dg_server **out)
{
    g_err.clear();
    if (!scenes || n_scenes == 0 || !cfg || !out) return fail(V3DG_ERR_INVALID_ARG, "NULL argument or no scenes");
    if (cfg->n_contexts < 1 || cfg->n_contexts > 64 || cfg->max_batch < 1 || cfg->max_batch > 64)
        return fail(V3DG_ERR_INVALID_ARG, "n_contexts and max_batch must be 1..64");
    uint32_t chunk_shift = kChunkShiftServer;
    if (cfg->chunk_keys != 0 && !chunk_shift_of(cfg->chunk_keys, &chunk_shift))
        return fail(V3DG_ERR_INVALID_ARG, "chunk_keys must be 0, 1024, 2048 or 4096 (got %u)", cfg->chunk_keys);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto *s = new (std::nothrow) v3dg_server();
    if (!s) return fail(V3DG_ERR_OOM, "host allocation failed");
    s->device = dev;
    s->cfg = *cfg;
    s->chunk_shift = chunk_shift;
    s->t0 = std::chrono::steady_clock::now();
    for (uint32_t i = 0; i < n_scenes; ++i) {
        v3dg_scene *sc = scenes[i];
        if (!sc || sc->device != dev) {
            delete s;
            return fail(V3DG_ERR_INVALID_ARG, "scene %u is NULL or on another device", i);
        }
        if (sc->pool_clusters) {
            delete s;
            return fail(V3DG_ERR_INVALID_ARG, "scene %u is streamed; the server takes resident scenes", i);
        }
        (void)hipStreamSynchronize(sc->stream);
        s->scenes.push_back(sc);
        s->max_tests = std::max<uint64_t>(s->max_tests, (uint64_t)sc->NC * sc->n_inst);
        s->max_slots = std::max<uint64_t>(s->max_slots, sc->cap_slots);
        s->max_inst = std::max(s->max_inst, sc->n_inst);
    }
    int rc = V3DG_OK;
    if (hipStreamCreateWithFlags(&s->sched, hipStreamNonBlocking) != hipSuccess)
        rc = fail(V3DG_ERR_HIP, "stream creation failed");
    for (int r = 0; r < kBatchRing && !rc; ++r) {
        BatchSlot &b = s->ring[r];
        if (hipHostMalloc((void **)&b.h_setup, cfg->max_batch * sizeof(SelSetup), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&b.h_req, cfg->max_batch * sizeof(SelReq), hipHostMallocDefault) != hipSuccess)
            rc = fail(V3DG_ERR_OOM, "pinned allocation failed");
        if (!rc) rc = dev_alloc(reinterpret_cast<uint8_t **>(&b.d_setup), cfg->max_batch * sizeof(SelSetup));
        if (!rc) rc = dev_alloc(reinterpret_cast<uint8_t **>(&b.d_req), cfg->max_batch * sizeof(SelReq));
        if (!rc) rc = dev_alloc(&b.d_ticket, 1);
        if (!rc && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess)
            rc = fail(V3DG_ERR_HIP, "event creation failed");
    }
    if (!rc) {  // the first context must fit the budget
        SrvCtx *c = nullptr;
        rc = srv_new_ctx(s, &c);
        if (!rc) {
            s->ctx.push_back(c);
            srv_account(s);
            if (s->st.workspace_bytes > cfg->hbm_budget_bytes)
                rc = fail(V3DG_ERR_OOM, "one render context needs %llu bytes; the budget is %llu",
                          (unsigned long long)s->st.workspace_bytes, (unsigned long long)cfg->hbm_budget_bytes);
        }
    }
    if (rc) {
        v3dg_server_free(s);
        return rc;
    }
    *out = s;
    return V3DG_OK;
}

int v3dg_server_submit(v3dg_server *s, uint32_t scene, const v3dg_camera *cam, float tau, float *image_dev,
                       uint64_t *ticket)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "server is NULL");
    if (scene >= s->scenes.size()) return fail(V3DG_ERR_INVALID_ARG, "scene %u out of range", scene);
    if (!image_dev) return fail(V3DG_ERR_INVALID_ARG, "image is NULL");
    if (!std::isfinite(tau) || tau < 0.0f) return fail(V3DG_ERR_INVALID_ARG, "tolerance must be finite and >= 0");
    SrvReq r;
    int rc = make_cam(cam, &r.cam);
    if (rc) return rc;
    r.ticket = s->next_ticket++;
    r.scene = scene;
    r.K = footprint_K(cam);
    r.tau = tau;
    r.image = image_dev;
    r.submit_ms = now_ms(s->t0);
    s->queue.push_back(r);
    s->st.submitted += 1;
    if (ticket) *ticket = r.ticket;
    return V3DG_OK;
}

int v3dg_server_submit_full(v3dg_server *s, uint32_t scene, const v3dg_camera *cam, float *image_dev,
                            uint64_t *ticket)
{
    g_err.clear();
    if (!s) return fail(V3DG_ERR_INVALID_ARG, "server is NULL");
    if (scene >= s->scenes.size()) return fail(V3DG_ERR_INVALID_ARG, "scene %u out of range", scene);
    if (!image_dev) return fail(V3DG_ERR_INVALID_ARG, "image is NULL");
    SrvReq r;
    int rc = make_cam(cam, &r.cam);
    if (rc) return rc;
    v3dg_scene *sc = s->scenes[scene];
    HIP_TRY(hipSetDevice(sc->device));
    if ((rc = build_full_selection(sc))) return rc;  // once per scene, on its stream (synchronised)
    r.ticket = s->next_ticket++;
    r.scene = scene;
    r.full = true;
    r.image = image_dev;
    r.submit_ms = now_ms(s->t0);
    s->queue.push_back(r);
    s->st.submitted += 1;
    if (ticket) *ticket = r.ticket;
    return V3DG_OK;
}

int v3dg_server_poll(v3dg_server *s, int wait, v3dg_request_done *done, uint32_t cap, uint32_t *n_done)
{
    g_err.clear();
    if (!s || !n_done || (cap && !done)) return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    if (wait && cap == 0) return fail(V3DG_ERR_INVALID_ARG, "a waiting poll needs room for one record (cap >= 1)");
    HIP_TRY(hipSetDevice(s->device));
    *n_done = 0;
    // ---- retire
    for (;;) {
        bool any_busy = false;
        for (SrvCtx *c : s->ctx) {
            if (!c->busy) continue;
            any_busy = true;
            if (*n_done >= cap) break;
            const hipError_t q = hipEventQuery(c->done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return fail(V3DG_ERR_HIP, "frame failed: %s", hipGetErrorString(q));
            c->busy = false;
            const uint32_t err = c->pinned[kRenErr] | c->pinned[8 + kSelErr];
            const uint64_t K = (uint64_t)c->pinned[kRenKeysLo] | ((uint64_t)c->pinned[kRenKeysHi] << 32);
            const ShapeKey key{c->req.scene, c->req.cam.width, c->req.cam.height, c->req.full};
            uint64_t &seen = s->keys_seen[key];
            seen = std::max(seen, K);
            int status = V3DG_OK;
            if (err & kErrSpin) {
                status = V3DG_ERR_DEVICE;
            } else if (K > c->cap_keys) {
                if (K >= 0xfffff000ull) {
                    status = V3DG_ERR_CAPACITY;
                } else {  // render it again once the context holds K keys
                    SrvReq r = c->req;
                    r.retries += 1;
                    s->st.retries += 1;
                    s->queue.push_front(r);
                    continue;
                }
            } else if (err & kErrOverflow) {
                status = V3DG_ERR_DEVICE;  // counting and emission disagreed
            }
            v3dg_request_done &d = done[(*n_done)++];
            d.ticket = c->req.ticket;
            d.status = status;
            d.retries = c->req.retries;
            d.n_slots = c->pinned[8 + kSelNGaussians];
            d.n_keys = K;
            d.submit_ms = c->req.submit_ms;
            d.admit_ms = c->req.admit_ms;
            d.done_ms = now_ms(s->t0);
            if (status) s->st.failed += 1;
            else s->st.completed += 1;
        }
        if (!wait || *n_done > 0 || !any_busy) break;
        // block on the oldest frame in flight
        SrvCtx *oldest = nullptr;
        for (SrvCtx *c : s->ctx)
            if (c->busy && (!oldest || c->req.admit_ms < oldest->req.admit_ms)) oldest = c;
        if (oldest) HIP_TRY(hipEventSynchronize(oldest->done));
    }
    // ---- admit: a free context that needs the least growth, else a new
    // context, while the budget holds what the front request would add
    std::vector<SrvCtx *> batch;
    while (!s->queue.empty() && batch.size() < s->cfg.max_batch) {
        SrvReq &r = s->queue.front();
        v3dg_scene *sc = s->scenes[r.scene];
        const uint32_t n_tiles = r.cam.tiles_x * r.cam.tiles_y;
        const ShapeKey key{r.scene, r.cam.width, r.cam.height, r.full};
        const uint64_t Kneed = keys_estimate(s, key, (uint64_t)r.cam.width * r.cam.height);
        SrvCtx *c = nullptr;
        uint64_t cost = 0;
        for (SrvCtx *x : s->ctx) {
            if (x->busy || std::find(batch.begin(), batch.end(), x) != batch.end()) continue;
            const uint64_t g = growth_bytes(x, Kneed, n_tiles, s->chunk_shift);
            if (!c || g < cost) {
                c = x;
                cost = g;
            }
        }
        const bool create = !c && s->ctx.size() < s->cfg.n_contexts;
        if (create) cost = ctx_base_bytes(s->ctx[0]) + growth_bytes(nullptr, Kneed, n_tiles, s->chunk_shift);
        if (!c && !create) break;  // every context is busy
        if (s->st.workspace_bytes + cost > s->cfg.hbm_budget_bytes) {
            bool busy = !batch.empty();
            for (SrvCtx *x : s->ctx) busy |= x->busy;
            if (busy) break;  // admit it once frames in flight have finished
            if (!c) break;
            // alone on the device and still over the budget: the request fails
            if (*n_done >= cap) break;
            v3dg_request_done &d = done[(*n_done)++];
            std::memset(&d, 0, sizeof(d));
            d.ticket = r.ticket;
            d.status = V3DG_ERR_OOM;
            d.submit_ms = r.submit_ms;
            d.done_ms = now_ms(s->t0);
            s->st.failed += 1;
            s->queue.pop_front();
            continue;
        }
        if (create) {
            int rc = srv_new_ctx(s, &c);
            if (rc) return rc;
            s->ctx.push_back(c);
        }
        bool changed = false;
        int rc = srv_provision(c, sc->n_inst, n_tiles, Kneed, &changed);
        if (rc) return rc;
        srv_account(s);
        c->req = r;
        c->req.admit_ms = now_ms(s->t0);
        s->queue.pop_front();
        batch.push_back(c);
    }
    int rc = srv_dispatch(s, batch);
    if (rc) return rc;
    s->st.queued = (uint32_t)s->queue.size();
    s->st.contexts_live = (uint32_t)s->ctx.size();
    return V3DG_OK;
}

int v3dg_server_get_stats(v3dg_server *s, v3dg_server_stats *out)
{
    g_err.clear();
    if (!s || !out) return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    s->st.queued = (uint32_t)s->queue.size();
    s->st.contexts_live = (uint32_t)s->ctx.size();
    *out = s->st;
    return V3DG_OK;
}

void v3dg_server_free(v3dg_server *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    for (SrvCtx *c : s->ctx) srv_ctx_free(c);
    s->ctx.clear();
    if (s->sched) (void)hipStreamSynchronize(s->sched);
    for (auto &b : s->ring) {
        if (b.h_setup) (void)hipHostFree(b.h_setup);
        if (b.h_req) (void)hipHostFree(b.h_req);
        dev_free(b.d_setup);
        dev_free(b.d_req);
        dev_free(b.d_ticket);
        if (b.ev) (void)hipEventDestroy(b.ev);
    }
    if (s->sched) (void)hipStreamDestroy(s->sched);
    delete s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Offline build (paper Sec. 3.1-3.2, Algorithm 1), structural part
// ---------------------------------------------------------------------------
struct v3dg_bundle {
    uint32_t n_clusters = 0, n_rows = 0, n_leaf = 0, n_layers = 0, sh_floats = 0, fit_iters = 0;
    std::vector<float> fit_loss;  // per coarse layer and view: the mean loss over the layer's groups
    std::vector<float> pos, scale, rot, opacity, sh, self_sphere, parent_sphere;
    std::vector<uint32_t> first_row, src;
    std::vector<uint8_t> count, level, n_children, gen;
    std::vector<int32_t> parent, first_child;
};

namespace {

// Sets of a median split of m items into sets of at most n, layer by layer:
// starts[l], splits[l] describe the sets entering layer l of the split, and
// the final sets are (fstart, fsize).  The sizes depend on m and n only.
struct SplitPlan {
    std::vector<std::vector<uint32_t>> starts;
    std::vector<std::vector<uint8_t>> splits;
    std::vector<uint32_t> fstart, fsize;
};

SplitPlan plan_split(uint32_t m, uint32_t n)
{
    SplitPlan p;
    std::vector<uint32_t> st{0}, sz{m};
    for (;;) {
        bool any = false;
        for (uint32_t z : sz) any |= z > n;
        if (!any) break;
        std::vector<uint8_t> sp(sz.size());
        std::vector<uint32_t> nst, nsz;
        for (size_t i = 0; i < sz.size(); ++i) {
            sp[i] = sz[i] > n ? 1 : 0;
            if (sp[i]) {
                const uint32_t h = (sz[i] + 1) / 2;
                nst.push_back(st[i]);
                nsz.push_back(h);
                nst.push_back(st[i] + h);
                nsz.push_back(sz[i] - h);
            } else {
                nst.push_back(st[i]);
                nsz.push_back(sz[i]);
            }
        }
        p.starts.push_back(st);
        p.splits.push_back(sp);
        st.swap(nst);
        sz.swap(nsz);
    }
    p.fstart = st;
    p.fsize = sz;
    return p;
}

struct DevBuf {  // a device allocation freed on scope exit (movable, not copyable)
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p) { o.p = nullptr; }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        std::swap(p, o.p);
        return *this;
    }
    ~DevBuf() { dev_free(p); }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

template <class T>
int dev_make(DevBuf &b, uint64_t count)
{
    T *q = nullptr;
    const int rc = dev_alloc(&q, count);
    b.p = q;
    return rc;
}

template <class T>
int upload(DevBuf &b, const T *h, uint64_t count)
{
    int rc = dev_make<T>(b, count);
    if (rc) return rc;
    if (count) HIP_TRY(hipMemcpy(b.p, h, count * sizeof(T), hipMemcpyHostToDevice));
    return V3DG_OK;
}

// device-to-host copy after the stream's work so far
int d2h(void *dst, const void *src, uint64_t bytes, hipStream_t st)
{
    if (bytes == 0) return V3DG_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return V3DG_OK;
}

uint32_t bits_of(uint64_t v)  // bits to hold 0 .. v
{
    uint32_t b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

// Median split of the m items in *items (device, current order, replaced by
// the split order) by their points (x y z per item id) into sets of at most n.
int device_split(hipStream_t st, const float *pts, DevBuf &items, DevBuf &spare, uint32_t m, uint32_t n,
                 std::vector<uint32_t> *fstart, std::vector<uint32_t> *fsize)
{
    const SplitPlan plan = plan_split(m, n);
    DevBuf keys, box, d_start, d_split;
    int rc;
    if ((rc = dev_make<uint64_t>(keys, m))) return rc;
    for (size_t l = 0; l < plan.starts.size(); ++l) {
        const uint32_t ns = (uint32_t)plan.starts[l].size();
        DevBuf a, b, c;
        if ((rc = upload(a, plan.starts[l].data(), ns))) return rc;
        if ((rc = upload(b, plan.splits[l].data(), ns))) return rc;
        if ((rc = dev_make<uint32_t>(c, 6ull * ns))) return rc;
        launch_split_layer(st, pts, items.as<uint32_t>(), m, a.as<uint32_t>(), b.as<uint8_t>(), ns, c.as<uint32_t>(),
                           keys.as<uint64_t>(), spare.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        if ((rc = v3dg_sort_pairs(keys.as<uint64_t>(), spare.as<uint32_t>(), m, 32 + std::max<uint32_t>(bits_of(ns - 1), 1),
                                  st)))
            return rc;
        std::swap(items.p, spare.p);
    }
    *fstart = plan.fstart;
    *fsize = plan.fsize;
    return V3DG_OK;
}

// One layer of the bundle during the build: its clusters (in the order they
// were made), their rows (ids into the layer's row store), own spheres,
// children (positions in the previous layer's grouping order) and the
// grouping order.  Layers above C_0 own their row store (slot g * cap + i of
// cluster g); C_0's store is the input.
struct BuildLayer {
    DevBuf rows, first, count, sph;
    DevBuf pos, scale, rot, op, sh, src;
    std::vector<uint32_t> h_first, h_count, h_rows, perm;
    std::vector<float> h_sph;
    std::vector<uint32_t> child_first, child_n;
};

struct RowStore {
    const float *pos, *scale, *rot, *op, *sh;
    const uint32_t *src;  // input Gaussian of each row; NULL: the row id itself
};

int build_impl(const float *pos, const float *scale, const float *rot, const float *opacity, const float *sh,
               uint32_t n, uint32_t sh_degree, uint32_t cap, uint32_t iters, const float *dirs, hipStream_t st,
               v3dg_bundle *B)
{
    const uint32_t shf = 3u * (sh_degree + 1u) * (sh_degree + 1u);
    DevBuf d_pos, d_scale, d_rot, d_opacity, d_sh, d_dirs, spare, err;
    int rc;
    if ((rc = upload(d_pos, pos, 3ull * n))) return rc;
    if ((rc = upload(d_scale, scale, 3ull * n))) return rc;
    if ((rc = upload(d_rot, rot, 4ull * n))) return rc;
    if ((rc = upload(d_opacity, opacity, (uint64_t)n))) return rc;
    if ((rc = upload(d_sh, sh, (uint64_t)shf * n))) return rc;
    if (iters && (rc = upload(d_dirs, dirs, 3ull * iters))) return rc;
    if ((rc = dev_make<uint32_t>(err, 1))) return rc;
    HIP_TRY(hipMemset(err.p, 0, sizeof(uint32_t)));
    auto store_of = [&](const BuildLayer &ly, bool input) {
        if (input)
            return RowStore{d_pos.as<float>(), d_scale.as<float>(), d_rot.as<float>(), d_opacity.as<float>(),
                            d_sh.as<float>(), nullptr};
        return RowStore{ly.pos.as<float>(), ly.scale.as<float>(), ly.rot.as<float>(), ly.op.as<float>(),
                        ly.sh.as<float>(), ly.src.as<uint32_t>()};
    };

    std::vector<BuildLayer> L(1);
    {  // layer C_0: the split of the Gaussians
        std::vector<uint32_t> iota(n);
        for (uint32_t i = 0; i < n; ++i) iota[i] = i;
        if ((rc = upload(L[0].rows, iota.data(), (uint64_t)n))) return rc;
        if ((rc = dev_make<uint32_t>(spare, n))) return rc;
        if ((rc = device_split(st, d_pos.as<float>(), L[0].rows, spare, n, cap, &L[0].h_first, &L[0].h_count)))
            return rc;
        const uint32_t C = (uint32_t)L[0].h_first.size();
        if ((rc = upload(L[0].first, L[0].h_first.data(), C))) return rc;
        if ((rc = upload(L[0].count, L[0].h_count.data(), C))) return rc;
        if ((rc = dev_make<float>(L[0].sph, 4ull * C))) return rc;
        DevBuf mean;
        if ((rc = dev_make<float>(mean, 3ull * C))) return rc;
        launch_cluster_mean(st, d_pos.as<float>(), L[0].rows.as<uint32_t>(), L[0].first.as<uint32_t>(),
                            L[0].count.as<uint32_t>(), C, mean.as<float>(), L[0].sph.as<float>());
        HIP_TRY(hipGetLastError());
        L[0].child_first.assign(C, 0);
        L[0].child_n.assign(C, 0);
    }
    // coarser layers while a layer holds two clusters or more
    for (uint32_t gen = 0;; ++gen) {
        BuildLayer &cur = L.back();
        const RowStore S = store_of(cur, gen == 0);
        const uint32_t C = (uint32_t)cur.h_first.size();
        if (C < 2) {
            cur.perm.assign(C, 0);
            for (uint32_t k = 0; k < C; ++k) cur.perm[k] = k;
            break;
        }
        if (gen >= 250) return fail(V3DG_ERR_DEVICE, "offline build: too many layers");
        DevBuf mean, gitems, gspare, d_gfirst, d_gsize, kept, go_rows, go_count, go_first, losses, vsph;
        if ((rc = dev_make<float>(mean, 3ull * C))) return rc;
        launch_cluster_mean(st, S.pos, cur.rows.as<uint32_t>(), cur.first.as<uint32_t>(), cur.count.as<uint32_t>(), C,
                            mean.as<float>(), nullptr);
        HIP_TRY(hipGetLastError());
        std::vector<uint32_t> iota(C), gfirst, gsize;
        for (uint32_t k = 0; k < C; ++k) iota[k] = k;
        if ((rc = upload(gitems, iota.data(), C))) return rc;
        if ((rc = dev_make<uint32_t>(gspare, C))) return rc;
        if ((rc = device_split(st, mean.as<float>(), gitems, gspare, C, 2, &gfirst, &gsize))) return rc;
        cur.perm.resize(C);
        if ((rc = d2h(cur.perm.data(), gitems.p, C * sizeof(uint32_t), st))) return rc;
        const uint32_t G = (uint32_t)gfirst.size();
        const uint64_t slots = (uint64_t)G * cap;
        if ((rc = upload(d_gfirst, gfirst.data(), G))) return rc;
        if ((rc = upload(d_gsize, gsize.data(), G))) return rc;
        BuildLayer nx;
        if ((rc = dev_make<uint32_t>(kept, slots)) || (rc = dev_make<uint32_t>(go_rows, 128ull * G)) ||
            (rc = dev_make<uint32_t>(go_count, G)) || (rc = dev_make<uint32_t>(nx.rows, slots)) ||
            (rc = dev_make<uint32_t>(nx.count, G)) || (rc = dev_make<float>(nx.sph, 4ull * G)) ||
            (rc = dev_make<float>(vsph, 4ull * G)) ||
            (rc = dev_make<float>(nx.pos, 3 * slots)) || (rc = dev_make<float>(nx.scale, 3 * slots)) ||
            (rc = dev_make<float>(nx.rot, 4 * slots)) || (rc = dev_make<float>(nx.op, slots)) ||
            (rc = dev_make<float>(nx.sh, shf * slots)) || (rc = dev_make<uint32_t>(nx.src, slots)))
            return rc;
        launch_group(st, S.pos, S.scale, S.op, cur.rows.as<uint32_t>(), cur.first.as<uint32_t>(),
                     cur.count.as<uint32_t>(), cur.sph.as<float>(), gitems.as<uint32_t>(), d_gfirst.as<uint32_t>(),
                     d_gsize.as<uint32_t>(), G, cap, kept.as<uint32_t>(), nx.count.as<uint32_t>(), nx.sph.as<float>(),
                     vsph.as<float>(), go_rows.as<uint32_t>(), go_count.as<uint32_t>(), err.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        launch_spawn(st, S.pos, S.scale, S.rot, S.op, S.sh, S.src, shf, kept.as<uint32_t>(), nx.count.as<uint32_t>(),
                     G, cap, nx.pos.as<float>(), nx.scale.as<float>(), nx.rot.as<float>(), nx.op.as<float>(),
                     nx.sh.as<float>(), nx.src.as<uint32_t>(), nx.rows.as<uint32_t>());
        HIP_TRY(hipGetLastError());
        nx.h_first.resize(G);
        for (uint32_t g = 0; g < G; ++g) nx.h_first[g] = g * cap;
        if ((rc = upload(nx.first, nx.h_first.data(), G))) return rc;
        if (iters) {  // local splatting of every group (Sec. 3.2)
            std::vector<uint32_t> gof(G);
            for (uint32_t g = 0; g < G; ++g) gof[g] = 128u * g;
            if ((rc = upload(go_first, gof.data(), G))) return rc;
            if ((rc = dev_make<float>(losses, (uint64_t)G * iters))) return rc;
            launch_local_splat(st, go_first.as<uint32_t>(), go_count.as<uint32_t>(), nx.first.as<uint32_t>(),
                               nx.count.as<uint32_t>(), vsph.as<float>(), S.pos, S.scale, S.rot, S.op, S.sh, shf,
                               go_rows.as<uint32_t>(), nx.pos.as<float>(), nx.scale.as<float>(), nx.rot.as<float>(),
                               nx.op.as<float>(), nx.sh.as<float>(), shf, d_dirs.as<float>(), iters, G,
                               losses.as<float>(), nullptr, err.as<uint32_t>());
            HIP_TRY(hipGetLastError());
            std::vector<float> h((uint64_t)G * iters);
            if ((rc = d2h(h.data(), losses.p, h.size() * sizeof(float), st))) return rc;
            for (uint32_t it = 0; it < iters; ++it) {
                double acc = 0.0;
                for (uint32_t g = 0; g < G; ++g) acc += h[(uint64_t)g * iters + it];
                B->fit_loss.push_back((float)(acc / G));
            }
        }
        nx.h_count.resize(G);
        if ((rc = d2h(nx.h_count.data(), nx.count.p, G * sizeof(uint32_t), st))) return rc;
        nx.child_first = gfirst;
        nx.child_n = gsize;
        L.push_back(std::move(nx));
    }
    uint32_t e = 0;
    if ((rc = d2h(&e, err.p, sizeof(uint32_t), st))) return rc;
    if (e) return fail(V3DG_ERR_DEVICE, "offline build: a cluster group exceeded its bounds");

    // ids (layer-major, grouping order), rows, links
    const uint32_t NL = (uint32_t)L.size();
    std::vector<uint32_t> base(NL + 1, 0);
    for (uint32_t l = 0; l < NL; ++l) base[l + 1] = base[l] + (uint32_t)L[l].h_first.size();
    const uint32_t C = base[NL];
    B->n_clusters = C;
    B->n_leaf = base[1];
    B->n_layers = NL;
    B->sh_floats = shf;
    B->fit_iters = iters;
    B->first_row.assign(C, 0);
    B->count.assign(C, 0);
    B->level.assign(C, 0);
    B->parent.assign(C, -1);
    B->first_child.assign(C, -1);
    B->n_children.assign(C, 0);
    B->self_sphere.assign(4ull * C, 0.f);
    B->parent_sphere.assign(4ull * C, 0.f);
    std::vector<std::vector<uint32_t>> idx(NL);  // per layer: store row of each bundle row
    uint64_t row = 0;
    for (uint32_t l = 0; l < NL; ++l) {
        BuildLayer &ly = L[l];
        const uint32_t Cl = (uint32_t)ly.h_first.size();
        ly.h_sph.resize(4ull * Cl);
        if ((rc = d2h(ly.h_sph.data(), ly.sph.p, 4ull * Cl * sizeof(float), st))) return rc;
        uint64_t store = 0;
        for (uint32_t k = 0; k < Cl; ++k) store = std::max<uint64_t>(store, (uint64_t)ly.h_first[k] + ly.h_count[k]);
        ly.h_rows.resize(store);
        if ((rc = d2h(ly.h_rows.data(), ly.rows.p, store * sizeof(uint32_t), st))) return rc;
        std::vector<uint32_t> lsrc;
        if (l > 0) {
            lsrc.resize(store);
            if ((rc = d2h(lsrc.data(), ly.src.p, store * sizeof(uint32_t), st))) return rc;
        }
        for (uint32_t p = 0; p < Cl; ++p) {
            const uint32_t k = ly.perm[p], id = base[l] + p;
            B->first_row[id] = (uint32_t)row;
            B->count[id] = (uint8_t)ly.h_count[k];
            B->level[id] = (uint8_t)l;
            for (int a = 0; a < 4; ++a) B->self_sphere[4ull * id + a] = ly.h_sph[4ull * k + a];
            if (l > 0) {
                B->first_child[id] = (int32_t)(base[l - 1] + ly.child_first[k]);
                B->n_children[id] = (uint8_t)ly.child_n[k];
                for (uint32_t i = 0; i < ly.child_n[k]; ++i) B->parent[base[l - 1] + ly.child_first[k] + i] = (int32_t)id;
            }
            for (uint32_t i = 0; i < ly.h_count[k]; ++i) {
                const uint32_t r = ly.h_rows[ly.h_first[k] + i];
                idx[l].push_back(r);
                B->src.push_back(l == 0 ? r : lsrc[r]);
                B->gen.push_back((uint8_t)l);
            }
            row += ly.h_count[k];
        }
    }
    for (uint32_t id = 0; id < C; ++id) {
        const int32_t par = B->parent[id];
        for (int a = 0; a < 4; ++a)
            B->parent_sphere[4ull * id + a] = par < 0 ? (a == 3 ? INFINITY : B->self_sphere[4ull * id + a])
                                                      : B->self_sphere[4ull * par + a];
    }
    // rows: gathered layer by layer from the row stores on the device
    const uint32_t R = (uint32_t)row;
    B->n_rows = R;
    DevBuf o_pos, o_scale, o_rot, o_op, o_sh;
    if ((rc = dev_make<float>(o_pos, 3ull * R))) return rc;
    if ((rc = dev_make<float>(o_scale, 3ull * R))) return rc;
    if ((rc = dev_make<float>(o_rot, 4ull * R))) return rc;
    if ((rc = dev_make<float>(o_op, R))) return rc;
    if ((rc = dev_make<float>(o_sh, (uint64_t)shf * R))) return rc;
    uint64_t r0 = 0;
    std::vector<DevBuf> d_idx(NL);
    for (uint32_t l = 0; l < NL; ++l) {
        const uint32_t nr = (uint32_t)idx[l].size();
        if ((rc = upload(d_idx[l], idx[l].data(), nr))) return rc;
        const RowStore S = store_of(L[l], l == 0);
        launch_gather_rows(st, S.pos, S.scale, S.rot, S.op, S.sh, shf, d_idx[l].as<uint32_t>(), nr,
                           o_pos.as<float>() + 3 * r0, o_scale.as<float>() + 3 * r0, o_rot.as<float>() + 4 * r0,
                           o_op.as<float>() + r0, o_sh.as<float>() + (uint64_t)shf * r0);
        HIP_TRY(hipGetLastError());
        r0 += nr;
    }
    B->pos.resize(3ull * R);
    B->scale.resize(3ull * R);
    B->rot.resize(4ull * R);
    B->opacity.resize(R);
    B->sh.resize((uint64_t)shf * R);
    HIP_TRY(hipMemcpyAsync(B->pos.data(), o_pos.p, 3ull * R * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(B->scale.data(), o_scale.p, 3ull * R * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(B->rot.data(), o_rot.p, 4ull * R * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(B->opacity.data(), o_op.p, (uint64_t)R * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(B->sh.data(), o_sh.p, (uint64_t)shf * R * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return V3DG_OK;
}

// unit-length-able view directions: finite and not zero
bool dirs_ok(const float *d, uint32_t n)
{
    for (uint64_t i = 0; i < n; ++i) {
        const double x = d[3 * i], y = d[3 * i + 1], z = d[3 * i + 2], q = x * x + y * y + z * z;
        if (!std::isfinite(q) || !(q > 1e-12)) return false;
    }
    return true;
}

}  // namespace

extern "C" {

int v3dg_build_bundle(const float *pos, const float *scale, const float *rot, const float *opacity, const float *sh,
                      uint32_t n, uint32_t sh_degree, uint32_t cluster_size, uint32_t fit_iters,
                      const float *view_dirs, v3dg_bundle **out)
{
    g_err.clear();
    if (!out) return fail(V3DG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!pos || !scale || !rot || !opacity || !sh) return fail(V3DG_ERR_INVALID_ARG, "NULL input array");
    if (n == 0 || n >= (1u << 31)) return fail(V3DG_ERR_INVALID_ARG, "n must be 1 .. 2^31-1");
    if (sh_degree > 3) return fail(V3DG_ERR_INVALID_ARG, "sh_degree must be 0..3");
    if (cluster_size < 2 || cluster_size > 64) return fail(V3DG_ERR_INVALID_ARG, "cluster_size must be 2..64");
    if (fit_iters > (1u << 20)) return fail(V3DG_ERR_INVALID_ARG, "fit_iters must be at most 2^20");
    if (fit_iters && (!view_dirs || !dirs_ok(view_dirs, fit_iters)))
        return fail(V3DG_ERR_INVALID_ARG, "view_dirs must hold fit_iters finite non-zero directions");
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreate(&st));  // blocking: the synchronous uploads are ordered with its work
    v3dg_bundle *B = new v3dg_bundle();
    const int rc = build_impl(pos, scale, rot, opacity, sh, n, sh_degree, cluster_size, fit_iters, view_dirs, st, B);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (rc) {
        delete B;
        return rc;
    }
    *out = B;
    return V3DG_OK;
}

int v3dg_bundle_sizes(const v3dg_bundle *b, uint32_t *n_clusters, uint32_t *n_rows, uint32_t *n_leaf_clusters,
                      uint32_t *n_layers)
{
    g_err.clear();
    if (!b) return fail(V3DG_ERR_INVALID_ARG, "bundle is NULL");
    if (n_clusters) *n_clusters = b->n_clusters;
    if (n_rows) *n_rows = b->n_rows;
    if (n_leaf_clusters) *n_leaf_clusters = b->n_leaf;
    if (n_layers) *n_layers = b->n_layers;
    return V3DG_OK;
}

int v3dg_bundle_copy(const v3dg_bundle *b, float *pos, float *scale, float *rot, float *opacity, float *sh,
                     float *self_sphere, float *parent_sphere, uint32_t *first_row, uint8_t *count, uint8_t *level,
                     int32_t *parent, int32_t *first_child, uint8_t *n_children, uint32_t *src, uint8_t *gen)
{
    g_err.clear();
    if (!b) return fail(V3DG_ERR_INVALID_ARG, "bundle is NULL");
    auto cp = [](void *dst, const void *from, size_t bytes) {
        if (dst && bytes) std::memcpy(dst, from, bytes);
    };
    cp(pos, b->pos.data(), b->pos.size() * 4);
    cp(scale, b->scale.data(), b->scale.size() * 4);
    cp(rot, b->rot.data(), b->rot.size() * 4);
    cp(opacity, b->opacity.data(), b->opacity.size() * 4);
    cp(sh, b->sh.data(), b->sh.size() * 4);
    cp(self_sphere, b->self_sphere.data(), b->self_sphere.size() * 4);
    cp(parent_sphere, b->parent_sphere.data(), b->parent_sphere.size() * 4);
    cp(first_row, b->first_row.data(), b->first_row.size() * 4);
    cp(count, b->count.data(), b->count.size());
    cp(level, b->level.data(), b->level.size());
    cp(parent, b->parent.data(), b->parent.size() * 4);
    cp(first_child, b->first_child.data(), b->first_child.size() * 4);
    cp(n_children, b->n_children.data(), b->n_children.size());
    cp(src, b->src.data(), b->src.size() * 4);
    cp(gen, b->gen.data(), b->gen.size());
    return V3DG_OK;
}

int v3dg_bundle_fit_loss(const v3dg_bundle *b, float *loss)
{
    g_err.clear();
    if (!b) return fail(V3DG_ERR_INVALID_ARG, "bundle is NULL");
    if (loss && !b->fit_loss.empty()) std::memcpy(loss, b->fit_loss.data(), b->fit_loss.size() * sizeof(float));
    return V3DG_OK;
}

void v3dg_bundle_free(v3dg_bundle *b) { delete b; }

int v3dg_local_splat(uint32_t n_groups, const uint32_t *orig_first, const uint32_t *orig_count,
                     const uint32_t *fit_first, const uint32_t *fit_count, const float *sphere, const float *orig_pos,
                     const float *orig_scale, const float *orig_rot, const float *orig_opacity, const float *orig_dc,
                     uint32_t n_orig, float *fit_pos, float *fit_scale, float *fit_rot, float *fit_opacity,
                     float *fit_dc, uint32_t n_fit, const float *view_dirs, uint32_t iters, float *losses,
                     float *grad_first)
{
    g_err.clear();
    if (n_groups == 0) return V3DG_OK;
    if (!orig_first || !orig_count || !fit_first || !fit_count || !sphere || !orig_pos || !orig_scale || !orig_rot ||
        !orig_opacity || !orig_dc || !fit_pos || !fit_scale || !fit_rot || !fit_opacity || !fit_dc ||
        (iters && !view_dirs))
        return fail(V3DG_ERR_INVALID_ARG, "NULL argument");
    if (iters && !dirs_ok(view_dirs, iters))
        return fail(V3DG_ERR_INVALID_ARG, "view_dirs must hold iters finite non-zero directions");
    for (uint32_t g = 0; g < n_groups; ++g) {
        if (orig_count[g] > 128 || fit_count[g] > 64)
            return fail(V3DG_ERR_INVALID_ARG, "group %u: at most 128 original and 64 fitted Gaussians", g);
        if ((uint64_t)orig_first[g] + orig_count[g] > n_orig || (uint64_t)fit_first[g] + fit_count[g] > n_fit)
            return fail(V3DG_ERR_INVALID_ARG, "group %u: rows out of range", g);
        if (!(sphere[4ull * g + 3] > 0.0f)) return fail(V3DG_ERR_INVALID_ARG, "group %u: radius must be > 0", g);
    }
    DevBuf of, oc, ff, fc, sp, op, os, orr, oo, od, fp, fs, fr, fo, fd, dr, lo, gf, err;
    int rc;
    if ((rc = upload(of, orig_first, n_groups)) || (rc = upload(oc, orig_count, n_groups)) ||
        (rc = upload(ff, fit_first, n_groups)) || (rc = upload(fc, fit_count, n_groups)) ||
        (rc = upload(sp, sphere, 4ull * n_groups)) || (rc = upload(op, orig_pos, 3ull * n_orig)) ||
        (rc = upload(os, orig_scale, 3ull * n_orig)) || (rc = upload(orr, orig_rot, 4ull * n_orig)) ||
        (rc = upload(oo, orig_opacity, (uint64_t)n_orig)) || (rc = upload(od, orig_dc, 3ull * n_orig)) ||
        (rc = upload(fp, fit_pos, 3ull * n_fit)) || (rc = upload(fs, fit_scale, 3ull * n_fit)) ||
        (rc = upload(fr, fit_rot, 4ull * n_fit)) || (rc = upload(fo, fit_opacity, (uint64_t)n_fit)) ||
        (rc = upload(fd, fit_dc, 3ull * n_fit)) || (rc = upload(dr, view_dirs, 3ull * iters)) ||
        (rc = dev_make<float>(lo, (uint64_t)n_groups * iters)) || (rc = dev_make<float>(gf, 14ull * n_fit)) ||
        (rc = dev_make<uint32_t>(err, 1)))
        return rc;
    HIP_TRY(hipMemset(err.p, 0, sizeof(uint32_t)));
    launch_local_splat(nullptr, of.as<uint32_t>(), oc.as<uint32_t>(), ff.as<uint32_t>(), fc.as<uint32_t>(),
                       sp.as<float>(), op.as<float>(), os.as<float>(), orr.as<float>(), oo.as<float>(),
                       od.as<float>(), 3, nullptr, fp.as<float>(), fs.as<float>(), fr.as<float>(), fo.as<float>(),
                       fd.as<float>(), 3, dr.as<float>(), iters, n_groups, lo.as<float>(), gf.as<float>(),
                       err.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    uint32_t e = 0;
    HIP_TRY(hipMemcpy(&e, err.p, sizeof(e), hipMemcpyDeviceToHost));
    if (e) return fail(V3DG_ERR_DEVICE, "local splatting: group bounds exceeded");
    HIP_TRY(hipMemcpy(fit_pos, fp.p, 3ull * n_fit * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(fit_scale, fs.p, 3ull * n_fit * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(fit_rot, fr.p, 4ull * n_fit * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(fit_opacity, fo.p, (uint64_t)n_fit * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(fit_dc, fd.p, 3ull * n_fit * 4, hipMemcpyDeviceToHost));
    if (losses && iters) HIP_TRY(hipMemcpy(losses, lo.p, (uint64_t)n_groups * iters * 4, hipMemcpyDeviceToHost));
    if (grad_first && iters) HIP_TRY(hipMemcpy(grad_first, gf.p, 14ull * n_fit * 4, hipMemcpyDeviceToHost));
    return V3DG_OK;
}

}  // extern "C"
