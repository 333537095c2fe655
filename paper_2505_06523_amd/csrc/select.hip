// Parallel cluster selection with single-pass compaction, expansion of
// the chosen clusters into the slot stream, and the per-frame instance set-up.
//
// Selection rule (paper Sec. 3.4): cluster k of instance i is drawn iff its own
// footprint fits the tolerance and its parent's does not, F_c <= tau < F_p,
// with F = pi r^2 fx fy / z^2 the pixel area of the cluster group's bounding
// sphere (Sec. 3.3).  Every (instance, cluster) test is independent; the chosen
// gids are compacted in ascending order by a decoupled look-back scan over
// partitions claimed with an atomic ticket.
#include "v3dg_internal.h"

#pragma clang fp contract(off)

namespace v3dg {

// ---------------------------------------------------------------------------
// per-frame set-up: A_i = fl32(V T_i) in FP64 (left-to-right sums, one final
// rounding), the camera centre in each asset frame, and clearing of the
// frame's counters / look-back words.
// ---------------------------------------------------------------------------
__device__ InstRec make_instrec(const CamArgs &cam, const double *__restrict__ t, float s)
{
    InstRec r;
#pragma unroll
    for (int row = 0; row < 3; ++row) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = __dmul_rn((double)cam.V[row * 4 + 0], t[0 * 4 + c]);
            acc = __dadd_rn(acc, __dmul_rn((double)cam.V[row * 4 + 1], t[1 * 4 + c]));
            acc = __dadd_rn(acc, __dmul_rn((double)cam.V[row * 4 + 2], t[2 * 4 + c]));
            if (c == 3) acc = __dadd_rn(acc, (double)cam.V[row * 4 + 3]);
            r.A[row * 4 + c] = __double2float_rn(acc);
        }
    }
    // camera centre in the asset frame: M^{-1} (cw - t) via the adjugate
    const double m0 = t[0], m1 = t[1], m2 = t[2], m3 = t[4], m4 = t[5], m5 = t[6], m6 = t[8], m7 = t[9], m8 = t[10];
    const double d0 = cam.cw[0] - t[3], d1 = cam.cw[1] - t[7], d2 = cam.cw[2] - t[11];
    const double a0 = m4 * m8 - m5 * m7, a1 = m2 * m7 - m1 * m8, a2 = m1 * m5 - m2 * m4;
    const double a3 = m5 * m6 - m3 * m8, a4 = m0 * m8 - m2 * m6, a5 = m2 * m3 - m0 * m5;
    const double a6 = m3 * m7 - m4 * m6, a7 = m1 * m6 - m0 * m7, a8 = m0 * m4 - m1 * m3;
    const double inv = 1.0 / (m0 * a0 + m1 * a3 + m2 * a6);
    r.chat[0] = (float)((a0 * d0 + a1 * d1 + a2 * d2) * inv);
    r.chat[1] = (float)((a3 * d0 + a4 * d1 + a5 * d2) * inv);
    r.chat[2] = (float)((a6 * d0 + a7 * d1 + a8 * d2) * inv);
    r.s = s;
    return r;
}

__global__ void __launch_bounds__(256) frame_setup_kernel(CamArgs cam_val, float *image, FrameDev *fd, int from_fd,
                                                          int bump_epoch, const double *__restrict__ T,
                                                          const float *__restrict__ inst_scale, uint32_t n_inst,
                                                          InstRec *__restrict__ itab, uint32_t *__restrict__ clear,
                                                          uint64_t n_clear)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = i; j < n_clear; j += stride) clear[j] = 0u;
    if (i == 0 && fd) {
        if (!from_fd) {
            fd->cam = cam_val;
            fd->image = image;
        }
        if (bump_epoch) fd->epoch += kEpochsPerFrame;
    }
    if (i >= n_inst) return;
    itab[i] = make_instrec(from_fd ? fd->cam : cam_val, T + 12 * i, inst_scale[i]);
}

void launch_frame_setup(hipStream_t st, const CamArgs &cam, float *image, FrameDev *fd, bool from_fd, bool bump_epoch,
                        const double *T, const float *inst_scale, uint32_t n_inst, InstRec *itab, uint32_t *clear,
                        uint64_t n_clear)
{
    uint64_t blocks = (n_inst + 255) / 256;          // one thread per instance
    uint64_t clear_blocks = (n_clear + 255) / 256;   // grid-stride over the words to clear
    if (clear_blocks > 1024) clear_blocks = 1024;
    if (blocks < clear_blocks) blocks = clear_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(frame_setup_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, cam, image, fd, (int)from_fd,
                       (int)bump_epoch, T, inst_scale, n_inst, itab, clear, n_clear);
}

// set-up of a batch: block row r serves request r; block (0, 0) clears the
// batch ticket
__global__ void __launch_bounds__(256) select_setup_batch_kernel(const SelSetup *__restrict__ setups,
                                                                 uint32_t *__restrict__ batch_ticket)
{
    const SelSetup &su = setups[blockIdx.y];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (i == 0 && blockIdx.y == 0) *batch_ticket = 0u;
    for (uint32_t j = i; j < su.n_clear; j += stride) su.clear[j] = 0u;
    for (uint32_t j = i; j < su.n_inst; j += stride)
        su.itab[j] = make_instrec(su.cam, su.T + 12 * (uint64_t)j, su.inst_scale[j]);
}

// ---------------------------------------------------------------------------
// selection
// ---------------------------------------------------------------------------

// "fits" = F <= tau for a sphere (c, r) seen through row 2 of A.  Operation
// order is fixed (no contraction, no division) so that every implementation
// of the rule takes the same decisions: z = ((a0 cx + a1 cy) + a2 cz) + a3;
// r' = r s; r' == 0 fits (a leaf has no own group); |z| <= r' does not fit
// (the camera plane cuts the sphere); else (r' r') K <= tau (z z).
__device__ __forceinline__ bool sel_fits(float4 sp, float a0, float a1, float a2, float a3, float s, float K,
                                         float tau)
{
    const float r = __fmul_rn(sp.w, s);
    if (r == 0.0f) return true;
    float z = __fmul_rn(a0, sp.x);
    z = __fadd_rn(z, __fmul_rn(a1, sp.y));
    z = __fadd_rn(z, __fmul_rn(a2, sp.z));
    z = __fadd_rn(z, a3);
    if (fabsf(z) <= r) return false;
    const float lhs = __fmul_rn(__fmul_rn(r, r), K);
    const float rhs = __fmul_rn(tau, __fmul_rn(z, z));
    return lhs <= rhs;
}

// true when no Gaussian of the cluster can reach the image through this
// instance (the planes of CullCam; see CullRec)
__device__ __forceinline__ bool cull_cluster(const CullRec &cr, const InstRec &ir, const CullCam &cc)
{
    const double cx = cr.sph.x, cy = cr.sph.y, cz = cr.sph.z;
    const double x = (double)ir.A[0] * cx + (double)ir.A[1] * cy + (double)ir.A[2] * cz + (double)ir.A[3];
    const double y = (double)ir.A[4] * cx + (double)ir.A[5] * cy + (double)ir.A[6] * cz + (double)ir.A[7];
    const double z = (double)ir.A[8] * cx + (double)ir.A[9] * cy + (double)ir.A[10] * cz + (double)ir.A[11];
    const double s = ir.s;
    const double r = (double)cr.sph.w * s * (1.0 + 1e-5) + 1e-5 * (1.0 + fabs(z));
    if (z + r <= cc.nearp) return true;
    const double e = (double)cr.smax * s;
    const double kx = cc.kx * e, ky = cc.ky * e;
    if (cc.fx * x + cc.al * z + r * cc.nl + kx < 0.0) return true;
    if (cc.fx * x + cc.ar * z - r * cc.nr - kx > 0.0) return true;
    if (cc.fy * y + cc.at * z + r * cc.nt + ky < 0.0) return true;
    if (cc.fy * y + cc.ab * z - r * cc.nb - ky > 0.0) return true;
    return false;
}

// packed scan payload: selected clusters in bits 36..61, Gaussians in 0..35
constexpr int kSelGBits = 36;
constexpr uint64_t kSelGMask = (1ull << kSelGBits) - 1;
constexpr uint64_t kPayload62 = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t n = __shfl_up(v, o, kWave);
        if (lane >= o) v += n;
    }
    return v;
}

// One partition (kSelPart consecutive tests) of request q: evaluate, scan,
// look back across the request's earlier partitions, write the chosen gids.
__device__ __forceinline__ void select_part(const SelReq &q, uint32_t p, uint64_t *s_wave, uint64_t *s_prefix)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const uint32_t NC = q.NC;
    const uint32_t n_tests = NC * q.n_inst;
    const uint32_t g0 = p * (uint32_t)kSelPart + (uint32_t)tid * kSelItems;
    uint64_t *status = q.status;
    uint32_t *counters = q.counters;

    uint64_t v[kSelItems];
    uint32_t inst = g0 / NC, k = g0 - inst * NC;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, s = 1.f;
    uint32_t cur_inst = 0xffffffffu;
    uint64_t tsum = 0;
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
        const uint32_t g = g0 + j;
        uint64_t val = 0;
        if (g < n_tests) {
            if (inst != cur_inst) {
                const InstRec &ir = q.itab[inst];
                a0 = ir.A[8];
                a1 = ir.A[9];
                a2 = ir.A[10];
                a3 = ir.A[11];
                s = ir.s;
                cur_inst = inst;
            }
            const bool sel = sel_fits(q.self_sph[k], a0, a1, a2, a3, s, q.K, q.tau) &&
                             !sel_fits(q.par_sph[k], a0, a1, a2, a3, s, q.K, q.tau);
            // a culled cluster stays in the cut but contributes no slots
            if (sel) val = (1ull << kSelGBits) |
                           ((q.cull && cull_cluster(q.cull[k], q.itab[inst], q.cc)) ? 0ull : (uint64_t)q.rowinfo[k].y);
        }
        v[j] = tsum;
        tsum += val;
        if (++k == NC) {
            k = 0;
            ++inst;
        }
    }
    // block exclusive scan of the per-thread sums
    const uint64_t incl = wave_incl_scan_u64(tsum);
    if (lane == kWave - 1) s_wave[wid] = incl;
    __syncthreads();
    uint64_t wave_off = 0, block_total = 0;
#pragma unroll
    for (int w = 0; w < kSelThreads / kWave; ++w) {
        if (w < wid) wave_off += s_wave[w];
        block_total += s_wave[w];
    }
    const uint64_t t_excl = wave_off + incl - tsum;

    if (tid == 0) {
        uint64_t prefix = 0;
        if (p == 0) {
            __hip_atomic_store(&status[0], (kFlagInc << 62) | block_total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[p], (kFlagAgg << 62) | block_total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)p - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint64_t w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = w >> 62;
                if (flag == 0) {
                    if (++spins > kSpinLimit) {
                        atomicOr(&counters[kSelErr], kErrSpin);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += w & kPayload62;
                if (flag == kFlagInc) break;
                --j;
            }
            __hip_atomic_store(&status[p], (kFlagInc << 62) | (prefix + block_total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        *s_prefix = prefix;
        if (p == q.nparts - 1) {
            const uint64_t tot = prefix + block_total;
            counters[kSelNClusters] = (uint32_t)(tot >> kSelGBits);
            counters[kSelNGaussians] = (uint32_t)(tot & kSelGMask);
            if ((tot & kSelGMask) >> 32) atomicOr(&counters[kSelErr], kErrOverflow);
        }
    }
    __syncthreads();
    const uint64_t base = *s_prefix + t_excl;
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
        // v[j] is the running sum before item j; a selected item adds at least
        // 1 << 36, so it is selected exactly when the sum after it differs
        const uint64_t next = (j + 1 < kSelItems) ? v[j + 1] : tsum;
        if (next != v[j]) {
            const uint64_t at = base + v[j];
            const uint32_t pos = (uint32_t)(at >> kSelGBits);
            q.gid[pos] = g0 + j;
            q.slot_off[pos] = (uint32_t)(at & kSelGMask);
        }
    }
}

// Workgroups claim partitions by ticket until all are taken.  A partition
// waits only on partitions of its own request with smaller tickets, which
// were claimed earlier by running workgroups, so the look-back always ends.
// With reqs == nullptr the single request `one` is served.
__global__ void __launch_bounds__(kSelThreads) select_kernel(SelReq one, const SelReq *__restrict__ reqs,
                                                             uint32_t n_req, uint32_t total_parts, uint32_t *ticket)
{
    __shared__ uint32_t s_ticket, s_req;
    __shared__ uint64_t s_wave[kSelThreads / kWave];
    __shared__ uint64_t s_prefix;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t r = 0;
            if (reqs && t < total_parts) {  // last request whose first partition is <= t
                uint32_t lo = 0, hi = n_req - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (reqs[mid].part_begin <= t) lo = mid;
                    else hi = mid - 1;
                }
                r = lo;
            }
            s_ticket = t;
            s_req = r;
        }
        __syncthreads();
        const uint32_t t = s_ticket;
        if (t >= total_parts) return;
        const SelReq q = reqs ? reqs[s_req] : one;
        select_part(q, t - q.part_begin, s_wave, &s_prefix);
        __syncthreads();
    }
}

void launch_select(hipStream_t st, const SelReq &req)
{
    if (req.nparts == 0) return;
    hipLaunchKernelGGL(select_kernel, dim3(req.nparts), dim3(kSelThreads), 0, st, req, (const SelReq *)nullptr, 1u,
                       req.nparts, req.counters + kSelTicket);
}

// ---------------------------------------------------------------------------
// expansion: one wavefront per selected cluster, one lane per Gaussian row
// (a cluster holds at most 64 rows).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) expand_kernel(const uint32_t *__restrict__ gid,
                                                     const uint32_t *__restrict__ slot_off,
                                                     const uint2 *__restrict__ rowinfo, uint32_t NC,
                                                     const uint32_t *__restrict__ counters,
                                                     uint32_t *__restrict__ slot_row, uint32_t *__restrict__ slot_inst)
{
    const uint32_t n = counters[kSelNClusters], total = counters[kSelNGaussians];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t nwaves = (gridDim.x * blockDim.x) / kWave;
    for (uint32_t c = wave; c < n; c += nwaves) {
        const uint32_t g = gid[c];
        const uint32_t inst = g / NC;
        const uint32_t k = g - inst * NC;
        const uint2 ri = rowinfo[k];
        const uint32_t off = slot_off[c];
        // the slot count is what the scan gave the cluster (0 when culled)
        const uint32_t cnt = (c + 1 < n ? slot_off[c + 1] : total) - off;
        if (lane < cnt) {
            slot_row[off + lane] = ri.x + lane;
            slot_inst[off + lane] = inst;
        }
    }
}

void launch_expand(hipStream_t st, const uint32_t *gid, const uint32_t *slot_off, const uint2 *rowinfo,
                   uint32_t n_clusters, const uint32_t *counters, uint32_t max_clusters, uint32_t *slot_row,
                   uint32_t *slot_inst)
{
    uint32_t blocks = (max_clusters + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(expand_kernel, dim3(blocks), dim3(256), 0, st, gid, slot_off, rowinfo, n_clusters, counters,
                       slot_row, slot_inst);
}

__global__ void __launch_bounds__(256) expand_batch_kernel(const SelReq *__restrict__ reqs, uint32_t n_req)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t nwaves = (gridDim.x * blockDim.x) / kWave;
    for (uint32_t r = 0; r < n_req; ++r) {
        const SelReq &q = reqs[r];
        const uint32_t n = q.counters[kSelNClusters], total = q.counters[kSelNGaussians];
        for (uint32_t c = wave; c < n; c += nwaves) {
            const uint32_t g = q.gid[c];
            const uint32_t inst = g / q.NC;
            const uint2 ri = q.rowinfo[g - inst * q.NC];
            const uint32_t off = q.slot_off[c];
            const uint32_t cnt = (c + 1 < n ? q.slot_off[c + 1] : total) - off;
            if (lane < cnt) {
                q.slot_row[off + lane] = ri.x + lane;
                q.slot_inst[off + lane] = inst;
            }
        }
    }
}

void launch_select_batch(hipStream_t st, const SelSetup *setups, const SelReq *reqs, uint32_t n_req,
                         uint32_t total_parts, uint32_t max_inst, uint32_t max_clear, uint32_t *batch_ticket)
{
    if (n_req == 0) return;
    uint32_t bx = (max(max_inst, max_clear) + 255) / 256;
    if (bx > 64) bx = 64;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(select_setup_batch_kernel, dim3(bx, n_req), dim3(256), 0, st, setups, batch_ticket);
    if (total_parts) {
        const uint32_t grid = total_parts < 2048u ? total_parts : 2048u;  // persistent: 8 per CU at most
        SelReq none{};
        hipLaunchKernelGGL(select_kernel, dim3(grid), dim3(kSelThreads), 0, st, none, reqs, n_req, total_parts,
                           batch_ticket);
    }
    hipLaunchKernelGGL(expand_batch_kernel, dim3(2048), dim3(256), 0, st, reqs, n_req);
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

void launch_fill_u32(hipStream_t st, uint32_t *p, uint64_t n, uint32_t v)
{
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
}

}  // namespace v3dg
