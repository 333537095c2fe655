// (a) parallel cluster selection with single-pass compaction, (b) expansion of
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
__global__ void __launch_bounds__(256) frame_setup_kernel(CamArgs cam, const double *__restrict__ T,
                                                          const float *__restrict__ inst_scale, uint32_t n_inst,
                                                          InstRec *__restrict__ itab, uint32_t *__restrict__ clear,
                                                          uint64_t n_clear)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = i; j < n_clear; j += stride) clear[j] = 0u;
    if (i >= n_inst) return;
    const double *t = T + 12 * i;
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
    r.s = inst_scale[i];
    itab[i] = r;
}

void launch_frame_setup(hipStream_t st, const CamArgs &cam, const double *T, const float *inst_scale,
                        uint32_t n_inst, InstRec *itab, uint32_t *clear, uint64_t n_clear)
{
    uint64_t blocks = (n_inst + 255) / 256;          // one thread per instance
    uint64_t clear_blocks = (n_clear + 255) / 256;   // grid-stride over the words to clear
    if (clear_blocks > 1024) clear_blocks = 1024;
    if (blocks < clear_blocks) blocks = clear_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(frame_setup_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, cam, T, inst_scale, n_inst, itab,
                       clear, n_clear);
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

__global__ void __launch_bounds__(kSelThreads) select_kernel(const float4 *__restrict__ self_sph,
                                                             const float4 *__restrict__ par_sph,
                                                             const uint2 *__restrict__ rowinfo,
                                                             const InstRec *__restrict__ itab, uint32_t NC,
                                                             uint32_t n_inst, float K, float tau,
                                                             uint32_t *__restrict__ gid_out,
                                                             uint32_t *__restrict__ slot_off_out,
                                                             uint64_t *__restrict__ status, uint32_t *counters,
                                                             uint32_t nparts)
{
    __shared__ uint32_t s_ticket;
    __shared__ uint64_t s_wave[kSelThreads / kWave];
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    if (tid == 0) s_ticket = __hip_atomic_fetch_add(&counters[kSelTicket], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t p = s_ticket;
    if (p >= nparts) return;
    const uint32_t n_tests = NC * n_inst;
    const uint32_t g0 = p * (uint32_t)kSelPart + (uint32_t)tid * kSelItems;

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
                const InstRec &ir = itab[inst];
                a0 = ir.A[8];
                a1 = ir.A[9];
                a2 = ir.A[10];
                a3 = ir.A[11];
                s = ir.s;
                cur_inst = inst;
            }
            const bool sel = sel_fits(self_sph[k], a0, a1, a2, a3, s, K, tau) &&
                             !sel_fits(par_sph[k], a0, a1, a2, a3, s, K, tau);
            if (sel) val = (1ull << kSelGBits) | (uint64_t)rowinfo[k].y;
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
        s_prefix = prefix;
        if (p == nparts - 1) {
            const uint64_t tot = prefix + block_total;
            counters[kSelNClusters] = (uint32_t)(tot >> kSelGBits);
            counters[kSelNGaussians] = (uint32_t)(tot & kSelGMask);
            if ((tot & kSelGMask) >> 32) atomicOr(&counters[kSelErr], kErrOverflow);
        }
    }
    __syncthreads();
    const uint64_t base = s_prefix + t_excl;
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
        // v[j] is the running sum before item j; a selected item adds at least
        // 1 << 36, so it is selected exactly when the sum after it differs
        const uint64_t next = (j + 1 < kSelItems) ? v[j + 1] : tsum;
        if (next != v[j]) {
            const uint64_t at = base + v[j];
            const uint32_t pos = (uint32_t)(at >> kSelGBits);
            gid_out[pos] = g0 + j;
            slot_off_out[pos] = (uint32_t)(at & kSelGMask);
        }
    }
}

void launch_select(hipStream_t st, const float4 *self_sph, const float4 *par_sph, const uint2 *rowinfo,
                   const InstRec *itab, uint32_t n_clusters, uint32_t n_inst, float K, float tau,
                   uint32_t *gid_out, uint32_t *slot_off_out, uint64_t *status, uint32_t *counters)
{
    const uint64_t n_tests = (uint64_t)n_clusters * n_inst;
    const uint32_t nparts = (uint32_t)((n_tests + kSelPart - 1) / kSelPart);
    if (nparts == 0) return;
    hipLaunchKernelGGL(select_kernel, dim3(nparts), dim3(kSelThreads), 0, st, self_sph, par_sph, rowinfo, itab,
                       n_clusters, n_inst, K, tau, gid_out, slot_off_out, status, counters, nparts);
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
    const uint32_t n = counters[kSelNClusters];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t nwaves = (gridDim.x * blockDim.x) / kWave;
    for (uint32_t c = wave; c < n; c += nwaves) {
        const uint32_t g = gid[c];
        const uint32_t inst = g / NC;
        const uint32_t k = g - inst * NC;
        const uint2 ri = rowinfo[k];
        const uint32_t off = slot_off[c];
        if (lane < ri.y) {
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
