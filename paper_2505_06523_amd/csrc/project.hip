// Projection of every slot's Gaussian to a 2D splat.
//
// A 3D Gaussian (p, s, q, o, SH colour) is splatted to the image plane with
// the EWA local affine approximation and no 2D dilation (paper Sec. 2.1 and
// Sec. 5.1).  With M = J W R(q) diag(s) (2x3), the 2D covariance is M M^T, so
// its entries are dot products of M's rows and its determinant is the squared
// length of their cross product: no cancellation in det even for thin splats.
// Splats with det below 1e-6 are redone in FP64 (counted per frame).
//
// Outputs per slot: the splat record read by blending, the FP32 depth used as
// the sort key, the binning record of the support {alpha >= 1/255} (ellipse
// d^T Sigma^-1 d <= 2 ln(255 o), enlarged) and the number of bins it reaches.
#include <hip/hip_fp16.h>

#include "v3dg_internal.h"

namespace v3dg {

// Real spherical harmonics up to degree 3 (Condon-Shortley phase, m = -l..l),
// normalisation K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), written as
// polynomials of the unit view direction.
constexpr float sqrtc(double x)
{
    // Newton iteration in double, for compile-time constants only
    double r = x > 1 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return (float)r;
}
constexpr double kPiD = 3.14159265358979323846;
constexpr float kY00 = sqrtc(1.0 / (4.0 * kPiD));
constexpr float kY1 = sqrtc(3.0 / (4.0 * kPiD));
constexpr float kY2a = sqrtc(15.0 / (4.0 * kPiD));   // xy, yz, xz
constexpr float kY2b = sqrtc(5.0 / (16.0 * kPiD));   // 3z^2-1 = 2z^2-x^2-y^2
constexpr float kY2c = sqrtc(15.0 / (16.0 * kPiD));  // x^2-y^2
constexpr float kY3a = sqrtc(35.0 / (32.0 * kPiD));  // y(3x^2-y^2), x(x^2-3y^2)
constexpr float kY3b = sqrtc(105.0 / (4.0 * kPiD));  // xyz
constexpr float kY3c = sqrtc(21.0 / (32.0 * kPiD));  // y(4z^2-x^2-y^2), x(...)
constexpr float kY3d = sqrtc(7.0 / (16.0 * kPiD));   // z(2z^2-3x^2-3y^2)
constexpr float kY3e = sqrtc(105.0 / (16.0 * kPiD)); // z(x^2-y^2)

template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y)
{
    Y[0] = kY00;
    if (D >= 1) {
        Y[1] = -kY1 * y;
        Y[2] = kY1 * z;
        Y[3] = -kY1 * x;
    }
    if (D >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kY2a * x * y;
        Y[5] = -kY2a * y * z;
        Y[6] = kY2b * (2.f * zz - xx - yy);
        Y[7] = -kY2a * x * z;
        Y[8] = kY2c * (xx - yy);
        if (D >= 3) {
            Y[9] = -kY3a * y * (3.f * xx - yy);
            Y[10] = kY3b * x * y * z;
            Y[11] = -kY3c * y * (4.f * zz - xx - yy);
            Y[12] = kY3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
            Y[13] = -kY3c * x * (4.f * zz - xx - yy);
            Y[14] = kY3e * z * (xx - yy);
            Y[15] = -kY3a * x * (xx - 3.f * yy);
        }
    }
}

// FP32 depth of a mean, the cull decision and the sort key:
// z = ((a20 px + a21 py) + a22 pz) + a23, each product and sum rounded on its
// own (no contraction), so that every implementation gets the same bits.
__device__ __forceinline__ float depth_z(const float *A, float px, float py, float pz)
{
#pragma clang fp contract(off)
    float z = A[8] * px;
    z = z + A[9] * py;
    z = z + A[10] * pz;
    z = z + A[11];
    return z;
}

// FP64 redo of the 2D covariance for near-degenerate splats: (a, b, c) of
// Sigma2 and its determinant.  Every argument is a value or a pointer to
// global memory (no local array has its address taken, so nothing spills).
struct Cov2d {
    double a, b, c, det;
};
constexpr double kBinEps2 = 1e-12;

__device__ __noinline__ Cov2d cov2_fp64(const InstRec *__restrict__ ir, const FrameDev *__restrict__ fd, float px,
                                        float py, float pz, float4 q4, float sx, float sy, float sz)
{
    const float *A = ir->A;
    const CamArgs &cam = fd->cam;
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float s[3] = {sx, sy, sz};
    const double x = (double)A[0] * px + (double)A[1] * py + (double)A[2] * pz + (double)A[3];
    const double y = (double)A[4] * px + (double)A[5] * py + (double)A[6] * pz + (double)A[7];
    const double z = (double)A[8] * px + (double)A[9] * py + (double)A[10] * pz + (double)A[11];
    const double qn = 1.0 / sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    const double qw = q[0] * qn, qx = q[1] * qn, qy = q[2] * qn, qz = q[3] * qn;
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[i * 3 + j] = ((double)A[i * 4 + 0] * R[0 * 3 + j] + (double)A[i * 4 + 1] * R[1 * 3 + j] +
                            (double)A[i * 4 + 2] * R[2 * 3 + j]) *
                           (double)s[j];
    double ux = x / z, uy = y / z;
    ux = fmin(fmax(ux, -(double)cam.limx), (double)cam.limx);
    uy = fmin(fmax(uy, -(double)cam.limy), (double)cam.limy);
    const double j00 = cam.fx / z, j02 = -cam.fx * ux / z, j11 = cam.fy / z, j12 = -cam.fy * uy / z;
    double m1[3], m2[3];
    for (int j = 0; j < 3; ++j) {
        m1[j] = j00 * M[0 * 3 + j] + j02 * M[2 * 3 + j];
        m2[j] = j11 * M[1 * 3 + j] + j12 * M[2 * 3 + j];
    }
    Cov2d r;
    r.a = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
    r.b = m1[0] * m2[0] + m1[1] * m2[1] + m1[2] * m2[2];
    r.c = m2[0] * m2[0] + m2[1] * m2[1] + m2[2] * m2[2];
    const double c0 = m1[1] * m2[2] - m1[2] * m2[1];
    const double c1 = m1[2] * m2[0] - m1[0] * m2[2];
    const double c2 = m1[0] * m2[1] - m1[1] * m2[0];
    r.det = c0 * c0 + c1 * c1 + c2 * c2;
    return r;
}

// attribute loads by storage precision: 0 FP32; 1 FP16 geometry + BF16 SH;
// 2 FP16 geometry + FP16 SH
template <int P>
__device__ __forceinline__ float load_geo(const Attribs &at, int plane, uint32_t row)
{
    if (P == 0) return static_cast<const float *>(at.geo)[plane * at.ps + row];
    return __half2float(static_cast<const __half *>(at.geo)[plane * at.ps + row]);
}

template <int P>
__device__ __forceinline__ float load_sh(const Attribs &at, int plane, uint32_t row)
{
    if (P == 0) return static_cast<const float *>(at.sh)[plane * at.ps + row];
    if (P == 1) return __uint_as_float((uint32_t) static_cast<const uint16_t *>(at.sh)[plane * at.ps + row] << 16);
    return __half2float(static_cast<const __half *>(at.sh)[plane * at.ps + row]);
}

template <int D, int P>
__global__ void __launch_bounds__(256) project_kernel(const FrameDev *__restrict__ fd, Attribs at,
                                                      const uint32_t *__restrict__ slot_row,
                                                      const uint32_t *__restrict__ slot_inst,
                                                      const uint32_t *__restrict__ n_dev,
                                                      const InstRec *__restrict__ itab, ProjectOut out)
{
    const uint64_t ps = at.ps;
    const CamArgs cam = fd->cam;
    constexpr int NCOEF = (D + 1) * (D + 1);
    const uint32_t n = *n_dev;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint32_t row = slot_row[t];
        const uint32_t inst = slot_inst[t];
        float A[12];
        {
            const float4 *ir = reinterpret_cast<const float4 *>(itab + inst);
            const float4 r0 = ir[0], r1 = ir[1], r2 = ir[2];
            A[0] = r0.x; A[1] = r0.y; A[2] = r0.z; A[3] = r0.w;
            A[4] = r1.x; A[5] = r1.y; A[6] = r1.z; A[7] = r1.w;
            A[8] = r2.x; A[9] = r2.y; A[10] = r2.z; A[11] = r2.w;
        }
        const float px = at.pos[0 * ps + row];
        const float py = at.pos[1 * ps + row];
        const float pz = at.pos[2 * ps + row];
        const float op = load_geo<P>(at, kGeoOP, row);
        const float z = depth_z(A, px, py, pz);
        out.depth[t] = z;
        out.dval[t] = t;
        out.dkey[t] = 0xffffffffu;  // culled slots sort last and emit nothing
        out.tiles[t] = 0u;
        // alpha = min(0.99, o e^power) <= o, so o < 1/255 never contributes
        if (!(z > cam.near_plane) || !(z < cam.far_plane) || !(op >= 1.0f / 255.0f)) continue;
        const float x = fmaf(A[0], px, fmaf(A[1], py, fmaf(A[2], pz, A[3])));
        const float y = fmaf(A[4], px, fmaf(A[5], py, fmaf(A[6], pz, A[7])));
        float q[4], s[3];
        q[0] = load_geo<P>(at, kGeoQW, row);
        q[1] = load_geo<P>(at, kGeoQX, row);
        q[2] = load_geo<P>(at, kGeoQY, row);
        q[3] = load_geo<P>(at, kGeoQZ, row);
        s[0] = load_geo<P>(at, kGeoSX, row);
        s[1] = load_geo<P>(at, kGeoSY, row);
        s[2] = load_geo<P>(at, kGeoSZ, row);
        // rotation of the normalised quaternion (narrow storage leaves |q| off 1 by ~1e-3)
        const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float qw = q[0] * qn, qx = q[1] * qn, qy = q[2] * qn, qz = q[3] * qn;
        const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                            2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                            2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
        // M = W R diag(s)
        float M[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                M[i * 3 + j] = (A[i * 4 + 0] * R[0 * 3 + j] + A[i * 4 + 1] * R[1 * 3 + j] + A[i * 4 + 2] * R[2 * 3 + j]) *
                               s[j];
        const float rz = 1.0f / z;
        const float ux = fminf(fmaxf(x * rz, -cam.limx), cam.limx);
        const float uy = fminf(fmaxf(y * rz, -cam.limy), cam.limy);
        const float j00 = cam.fx * rz, j02 = -cam.fx * ux * rz;
        const float j11 = cam.fy * rz, j12 = -cam.fy * uy * rz;
        float m1[3], m2[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            m1[j] = j00 * M[0 * 3 + j] + j02 * M[2 * 3 + j];
            m2[j] = j11 * M[1 * 3 + j] + j12 * M[2 * 3 + j];
        }
        float a = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
        float b = m1[0] * m2[0] + m1[1] * m2[1] + m1[2] * m2[2];
        float c = m2[0] * m2[0] + m2[1] * m2[1] + m2[2] * m2[2];
        const float c0 = m1[1] * m2[2] - m1[2] * m2[1];
        const float c1 = m1[2] * m2[0] - m1[0] * m2[2];
        const float c2 = m1[0] * m2[1] - m1[1] * m2[0];
        const float det = c0 * c0 + c1 * c1 + c2 * c2;
        float ca, cb, cc, det_s = det;
        if (det >= 1e-6f) {
            const float inv = 1.0f / det;
            ca = c * inv;
            cb = -b * inv;
            cc = a * inv;
        } else {
            const Cov2d r = cov2_fp64(itab + inst, fd, px, py, pz, make_float4(q[0], q[1], q[2], q[3]), s[0], s[1], s[2]);
            if (!(r.det > 0.0)) continue;
            atomicAdd(&out.counters[kRenFp64], 1u);
            const double inv = 1.0 / r.det;
            ca = (float)(r.c * inv);
            cb = (float)(-r.b * inv);
            cc = (float)(r.a * inv);
            // The binning record takes Sigma + eps I (eps = 1e-12 px^2): its
            // support contains this splat's, and every entry and the
            // determinant stay normal FP32 numbers, so the per-row tile spans
            // keep full precision even for a needle of subnormal width.
            a = (float)(r.a + kBinEps2);
            b = (float)r.b;
            c = (float)(r.c + kBinEps2);
            det_s = (float)(r.det + kBinEps2 * (r.a + r.c) + kBinEps2 * kBinEps2);
        }
        // A conic entry beyond +-kConicMax (a splat thinner than ~1e-19 px
        // across, or one overflowing FP32) is clamped: blending then still
        // draws an axis-aligned needle on the pixel row or column it runs
        // through, and elsewhere its quadratic form overflows (no contribution).
        if (!(fabsf(ca) <= kConicMax && fabsf(cb) <= kConicMax && fabsf(cc) <= kConicMax)) {
            atomicAdd(&out.counters[kRenConicClamp], 1u);
            ca = fminf(fmaxf(ca, -kConicMax), kConicMax);
            cb = fminf(fmaxf(cb, -kConicMax), kConicMax);
            cc = fminf(fmaxf(cc, -kConicMax), kConicMax);
        }
        const float mx = cam.fx * (x * rz) + cam.cx;
        const float my = cam.fy * (y * rz) + cam.cy;
        // view-dependent colour in the asset frame
        const float *ch = itab[inst].chat;
        float dx = px - ch[0], dy = py - ch[1], dz = pz - ch[2];
        const float il = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= il;
        dy *= il;
        dz *= il;
        float Y[NCOEF];
        sh_basis<D>(dx, dy, dz, Y);
        float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < NCOEF; ++k)
#pragma unroll
            for (int cch = 0; cch < 3; ++cch) col[cch] = fmaf(load_sh<P>(at, 3 * k + cch, row), Y[k], col[cch]);
        // tile coverage of the (enlarged) support
        const float Q = 2.0f * __logf(255.0f * op);
        BinRec br;
        br.mx = mx;
        br.my = my;
        br.sa = a;
        br.sb = b;
        br.sc = c;
        br.det = det_s;
        br.Qm = 1.05f * Q + 0.05f;
        br.depth = z;
        uint32_t tx0, tx1, ty0, ty1;
        if (!bin_box(br, cam.width, cam.height, &tx0, &tx1, &ty0, &ty1)) continue;
        uint32_t ntiles = 0;  // bins touched
        for (uint32_t ty = ty0; ty <= ty1; ++ty) {
            uint32_t lo, hi;
            if (bin_row_span(br, ty, tx0, tx1, &lo, &hi)) ntiles += hi - lo + 1;
        }
        if (ntiles == 0) continue;
        out.tiles[t] = ntiles;
        out.dkey[t] = __float_as_uint(z);
        out.bin[t] = br;
        float4 *sp = out.splat + 3 * (uint64_t)t;
        sp[0] = make_float4(mx, my, ca, cb);
        sp[1] = make_float4(cc, op, fmaxf(col[0], 0.f), fmaxf(col[1], 0.f));
        // support half-extents (enlarged like the binning), used to cull per 8x8 block
        sp[2] = make_float4(fmaxf(col[2], 0.f), z, sqrtf(br.Qm * a), sqrtf(br.Qm * c));
    }
}

template <int D>
static void launch_project_d(hipStream_t st, dim3 g, dim3 b, const FrameDev *cam, const Attribs &at, int precision,
                             const uint32_t *slot_row, const uint32_t *slot_inst, const uint32_t *n_dev,
                             const InstRec *itab, const ProjectOut &out)
{
    switch (precision) {
    case 0: hipLaunchKernelGGL((project_kernel<D, 0>), g, b, 0, st, cam, at, slot_row, slot_inst, n_dev, itab, out); break;
    case 1: hipLaunchKernelGGL((project_kernel<D, 1>), g, b, 0, st, cam, at, slot_row, slot_inst, n_dev, itab, out); break;
    default: hipLaunchKernelGGL((project_kernel<D, 2>), g, b, 0, st, cam, at, slot_row, slot_inst, n_dev, itab, out); break;
    }
}

void launch_project(hipStream_t st, const FrameDev *cam, const Attribs &attr, int precision, int sh_degree,
                    const uint32_t *slot_row, const uint32_t *slot_inst, const uint32_t *n_slots_dev,
                    uint64_t max_slots, const InstRec *itab, ProjectOut out)
{
    uint64_t blocks = (max_slots + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    dim3 g((uint32_t)blocks), b(256);
    switch (sh_degree) {
    case 0: launch_project_d<0>(st, g, b, cam, attr, precision, slot_row, slot_inst, n_slots_dev, itab, out); break;
    case 1: launch_project_d<1>(st, g, b, cam, attr, precision, slot_row, slot_inst, n_slots_dev, itab, out); break;
    case 2: launch_project_d<2>(st, g, b, cam, attr, precision, slot_row, slot_inst, n_slots_dev, itab, out); break;
    default: launch_project_d<3>(st, g, b, cam, attr, precision, slot_row, slot_inst, n_slots_dev, itab, out); break;
    }
}

}  // namespace v3dg
