/*
 * CPU oracle for the V3DG per-frame path.  TEST INFRASTRUCTURE ONLY (see the
 * header): plain, slow, obviously correct.  Built with -O2 -ffp-contract=off
 * so every FP32 decision below is evaluated exactly in the order written.
 *
 * Paper passages followed:
 *   Sec. 3.3 (footprint figure and text): the bounding sphere of a cluster
 *     group and F = pi r^2 fx fy / z_v^2, the pixel area it covers;
 *   Sec. 3.4: each cluster stores its own (c_c, r_c) and its parent's
 *     (c_p, r_p); a cluster is rendered iff F_c <= tau < F_p;
 *   Sec. 2.1: a 3D Gaussian (p, s, q, o, c) is splatted to the image plane
 *     (EWA) and the splats covering a pixel are alpha-blended;
 *   Sec. 5.1: no 2D dilation (eps2d = 0), pinhole camera;
 *   Sec. 4.2 and Appendix A.2/A.3: many instances of one asset, each with its
 *     own rigid (or uniformly scaled) transform, re-selected every frame.
 * Readings where the paper is silent (tolerance unit, leaf/root spheres,
 * camera inside a sphere, support of a splat, ties) are listed with the
 * function that takes them.
 */
#include "v3dg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define AMBIG_REL (1.0 / 16384.0) /* 2^-14: a threshold decision this close is ambiguous */

/* ------------------------------------------------------------------------ */
/* Frame set-up: compose the instance transform into the camera.            */
/* ------------------------------------------------------------------------ */

/* A = fl32(V * T) with T the instance's 3x4 affine (implicit last row 0 0 0 1),
 * every entry summed left to right in FP64 and rounded once to FP32.  The
 * uniform scale s of a similarity T = [s R | t] is the length of the first
 * column of its 3x3 part, in FP64, rounded to FP32.  K = fl32(pi * fx * fy). */
void orc_frame_setup(uint32_t n_inst, const double *T, const orc_camera *cam,
                     float *A_out, float *s_out, double *chat_out, float *K_out)
{
    const float *V = cam->V;
    /* camera centre in world space: -R^T t */
    double cw[3];
    for (int c = 0; c < 3; ++c)
        cw[c] = -((double)V[0 * 4 + c] * V[0 * 4 + 3] + (double)V[1 * 4 + c] * V[1 * 4 + 3] +
                  (double)V[2 * 4 + c] * V[2 * 4 + 3]);
    for (uint32_t i = 0; i < n_inst; ++i) {
        const double *t = T + 12 * (size_t)i;
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 4; ++c) {
                double acc = (double)V[r * 4 + 0] * t[0 * 4 + c];
                acc = acc + (double)V[r * 4 + 1] * t[1 * 4 + c];
                acc = acc + (double)V[r * 4 + 2] * t[2 * 4 + c];
                if (c == 3) acc = acc + (double)V[r * 4 + 3];
                A_out[12 * (size_t)i + r * 4 + c] = (float)acc;
            }
        }
        double s2 = t[0] * t[0];
        s2 = s2 + t[4] * t[4];
        s2 = s2 + t[8] * t[8];
        s_out[i] = (float)sqrt(s2);
        /* chat = M^{-1} (cw - t_T) via the adjugate of the 3x3 part M */
        double m[9] = {t[0], t[1], t[2], t[4], t[5], t[6], t[8], t[9], t[10]};
        double d[3] = {cw[0] - t[3], cw[1] - t[7], cw[2] - t[11]};
        double adj[9];
        adj[0] = m[4] * m[8] - m[5] * m[7];
        adj[1] = m[2] * m[7] - m[1] * m[8];
        adj[2] = m[1] * m[5] - m[2] * m[4];
        adj[3] = m[5] * m[6] - m[3] * m[8];
        adj[4] = m[0] * m[8] - m[2] * m[6];
        adj[5] = m[2] * m[3] - m[0] * m[5];
        adj[6] = m[3] * m[7] - m[4] * m[6];
        adj[7] = m[1] * m[6] - m[0] * m[7];
        adj[8] = m[0] * m[4] - m[1] * m[3];
        double det = m[0] * adj[0] + m[1] * adj[3] + m[2] * adj[6];
        for (int r = 0; r < 3; ++r)
            chat_out[3 * (size_t)i + r] = (adj[r * 3 + 0] * d[0] + adj[r * 3 + 1] * d[1] + adj[r * 3 + 2] * d[2]) / det;
    }
    double k = ORC_PI * (double)cam->fx;
    k = k * (double)cam->fy;
    *K_out = (float)k;
}

/* ------------------------------------------------------------------------ */
/* Footprint predicate (Sec. 3.3/3.4).                                      */
/* ------------------------------------------------------------------------ */

/* "fits" means F <= tau for the sphere (c, r) seen through the instance.
 * Readings: tau is in the paper's unit of F, a pixel AREA.  A sphere of radius
 * 0 (a leaf's own sphere: leaves are not simplified from anything) has F = 0.
 * When the camera's z-plane cuts the sphere (|z| <= r) F is taken as +inf
 * (does not fit).  The comparison F <= tau is evaluated without division as
 * (r*r)*K <= tau*(z*z), K = fl32(pi fx fy), in FP32 in exactly this order;
 * z = ((a0*cx + a1*cy) + a2*cz) + a3 with row 2 of A.  r is scaled by the
 * instance's uniform scale first: r_eff = fl32(r * s). */
static int orc_fits(const float *sph, const float *a2, float s, float K, float tau)
{
    float r = sph[3] * s;
    if (r == 0.0f) return 1;
    float z = a2[0] * sph[0];
    z = z + a2[1] * sph[1];
    z = z + a2[2] * sph[2];
    z = z + a2[3];
    if (fabsf(z) <= r) return 0;
    float lhs = r * r;
    lhs = lhs * K;
    float rhs = z * z;
    rhs = tau * rhs;
    return lhs <= rhs;
}

double orc_footprint(const float sphere[4], const float A_row2[4], float s, float fx, float fy)
{
    double r = (double)sphere[3] * s;
    double z = (double)A_row2[0] * sphere[0] + (double)A_row2[1] * sphere[1] + (double)A_row2[2] * sphere[2] + A_row2[3];
    if (fabs(z) <= r) return INFINITY;
    return ORC_PI * r * r * (double)fx * (double)fy / (z * z);
}

typedef struct {
    const orc_asset *a;
    const float *a2; /* row 2 of this instance's A */
    float s, K, tau;
    uint8_t *mask;   /* this instance's n_clusters bytes */
    uint64_t n;
} walk_ctx;

static void orc_visit(walk_ctx *w, int32_t k)
{
    if (orc_fits(w->a->self_sphere + 4 * (size_t)k, w->a2, w->s, w->K, w->tau)) {
        w->mask[k] = 1;
        w->n++;
        return;
    }
    int32_t c0 = w->a->first_child[k];
    for (int32_t c = 0; c < (int32_t)w->a->n_children[k]; ++c) orc_visit(w, c0 + c);
}

uint64_t orc_select_walk(const orc_asset *a, uint32_t n_inst, const double *T,
                         const orc_camera *cam, float tau, uint8_t *out_mask)
{
    float *A = (float *)malloc(sizeof(float) * 12 * (n_inst ? n_inst : 1));
    float *s = (float *)malloc(sizeof(float) * (n_inst ? n_inst : 1));
    double *ch = (double *)malloc(sizeof(double) * 3 * (n_inst ? n_inst : 1));
    float K;
    orc_frame_setup(n_inst, T, cam, A, s, ch, &K);
    memset(out_mask, 0, (size_t)n_inst * a->n_clusters);
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        walk_ctx w = {a, A + 12 * (size_t)i + 8, s[i], K, tau, out_mask + (size_t)i * a->n_clusters, 0};
        for (uint32_t k = 0; k < a->n_clusters; ++k)
            if (a->parent[k] < 0) orc_visit(&w, (int32_t)k);
        total += w.n;
    }
    free(A);
    free(s);
    free(ch);
    return total;
}

uint64_t orc_select_predicate(const orc_asset *a, uint32_t n_inst, const double *T,
                              const orc_camera *cam, float tau, uint8_t *out_mask)
{
    float *A = (float *)malloc(sizeof(float) * 12 * (n_inst ? n_inst : 1));
    float *s = (float *)malloc(sizeof(float) * (n_inst ? n_inst : 1));
    double *ch = (double *)malloc(sizeof(double) * 3 * (n_inst ? n_inst : 1));
    float K;
    orc_frame_setup(n_inst, T, cam, A, s, ch, &K);
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const float *a2 = A + 12 * (size_t)i + 8;
        for (uint32_t k = 0; k < a->n_clusters; ++k) {
            int sel = orc_fits(a->self_sphere + 4 * (size_t)k, a2, s[i], K, tau) &&
                      !orc_fits(a->parent_sphere + 4 * (size_t)k, a2, s[i], K, tau);
            out_mask[(size_t)i * a->n_clusters + k] = (uint8_t)sel;
            total += (uint64_t)sel;
        }
    }
    free(A);
    free(s);
    free(ch);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics from the associated Legendre functions.          */
/* ------------------------------------------------------------------------ */

static double orc_fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* P_l^m(x), m >= 0, with the Condon-Shortley phase (-1)^m. */
static double orc_legendre(int l, int m, double x)
{
    double pmm = 1.0;
    double sx = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * sx;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

/* Y_l^m for m = -l..l at index l*l + l + m:  K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
 * m > 0: sqrt2 K cos(m phi) P_l^m;  m < 0: sqrt2 K sin(|m| phi) P_l^|m|;  m = 0: K P_l^0. */
void orc_sh_basis(int degree, const double dir[3], double *out)
{
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
    double phi = atan2(y, x);
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * orc_fact(l - am) / orc_fact(l + am));
            double P = orc_legendre(l, am, z);
            double v;
            if (m > 0) v = sqrt(2.0) * K * cos(am * phi) * P;
            else if (m < 0) v = sqrt(2.0) * K * sin(am * phi) * P;
            else v = K * P;
            out[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Slots and projection.                                                     */
/* ------------------------------------------------------------------------ */

uint64_t orc_count_slots(const orc_asset *a, uint64_t n_gids, const uint32_t *gids)
{
    uint64_t n = 0;
    for (uint64_t g = 0; g < n_gids; ++g) n += a->count[gids[g] % a->n_clusters];
    return n;
}

/* slot t -> (instance, row); gids are ascending, rows of a cluster in stored order */
static void orc_build_slots(const orc_asset *a, uint64_t n_gids, const uint32_t *gids,
                            uint32_t *inst, uint32_t *row)
{
    uint64_t t = 0;
    for (uint64_t g = 0; g < n_gids; ++g) {
        uint32_t i = gids[g] / a->n_clusters, k = gids[g] % a->n_clusters;
        for (uint32_t j = 0; j < a->count[k]; ++j) {
            inst[t] = i;
            row[t] = a->first_row[k] + j;
            ++t;
        }
    }
}

typedef struct {
    uint8_t valid;
    float depth;
    double mx, my, ca, cb, cc, r, g, b, o, sxx, sxy, syy;
} orc_splat;

/* One Gaussian through one instance (Sec. 2.1, EWA splatting); the colour
 * is computed by orc_colour_one:
 *   camera-space mean m = A p; the cull and the sort key use the FP32 depth
 *   z32 = ((a20*px + a21*py) + a22*pz) + a23 (near < z32 < far);
 *   Sigma = R(q) diag(s^2) R(q)^T;  Sigma_cam = W Sigma W^T, W = A's 3x3;
 *   J = [[fx/z, 0, -fx tx/z^2], [0, fy/z, -fy ty/z^2]] with tx = z clamp(x/z, +-1.3 W/(2fx))
 *   (and the same for y): the 3DGS guard band;  Sigma2 = J Sigma_cam J^T with no
 *   dilation (Sec. 5.1); cull when det(Sigma2) <= 0;  conic = Sigma2^{-1};
 *   mean2 = (fx x/z + cx, fy y/z + cy);
 *   colour = max(0, sum_lm sh_lm Y_lm(d) + 0.5), d = normalise(p - chat), the
 *   view direction in the asset's frame. */
static void orc_project_one(const orc_asset *a, const float *A, const double *chat,
                            const orc_camera *cam, uint32_t row, orc_splat *o)
{
    const float *p = a->pos + 3 * (size_t)row;
    memset(o, 0, sizeof(*o));
    float z32 = A[8] * p[0];
    z32 = z32 + A[9] * p[1];
    z32 = z32 + A[10] * p[2];
    z32 = z32 + A[11];
    o->depth = z32;
    if (!(z32 > cam->near_plane) || !(z32 < cam->far_plane)) return;
    double x = (double)A[0] * p[0] + (double)A[1] * p[1] + (double)A[2] * p[2] + (double)A[3];
    double y = (double)A[4] * p[0] + (double)A[5] * p[1] + (double)A[6] * p[2] + (double)A[7];
    double z = (double)A[8] * p[0] + (double)A[9] * p[1] + (double)A[10] * p[2] + (double)A[11];
    const float *q = a->rot + 4 * (size_t)row;
    /* rotation matrix of the normalised quaternion */
    double qn = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    double qw = q[0] / qn, qx = q[1] / qn, qy = q[2] / qn, qz = q[3] / qn;
    double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                   2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                   2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    const float *s = a->scale + 3 * (size_t)row;
    double S2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    double Sig[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[i * 3 + k] * S2[k] * R[j * 3 + k];
            Sig[i * 3 + j] = acc;
        }
    double W[9] = {A[0], A[1], A[2], A[4], A[5], A[6], A[8], A[9], A[10]};
    double WS[9], Sc[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += W[i * 3 + k] * Sig[k * 3 + j];
            WS[i * 3 + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += WS[i * 3 + k] * W[j * 3 + k];
            Sc[i * 3 + j] = acc;
        }
    double fx = cam->fx, fy = cam->fy;
    double limx = 1.3 * (0.5 * (double)cam->width / fx);
    double limy = 1.3 * (0.5 * (double)cam->height / fy);
    double ux = x / z, uy = y / z;
    if (ux < -limx) ux = -limx;
    if (ux > limx) ux = limx;
    if (uy < -limy) uy = -limy;
    if (uy > limy) uy = limy;
    double tx = z * ux, ty = z * uy;
    double J[6] = {fx / z, 0.0, -fx * tx / (z * z), 0.0, fy / z, -fy * ty / (z * z)};
    double JS[6], S2d[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[i * 3 + k] * Sc[k * 3 + j];
            JS[i * 3 + j] = acc;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += JS[i * 3 + k] * J[j * 3 + k];
            S2d[i * 2 + j] = acc;
        }
    double sa = S2d[0], sb = 0.5 * (S2d[1] + S2d[2]), sc = S2d[3];
    double det = sa * sc - sb * sb;
    if (!(det > 0.0)) return;
    o->valid = 1;
    o->ca = sc / det;
    o->cb = -sb / det;
    o->cc = sa / det;
    o->sxx = sa;
    o->sxy = sb;
    o->syy = sc;
    o->mx = fx * x / z + (double)cam->cx;
    o->my = fy * y / z + (double)cam->cy;
    o->o = a->opacity[row];
}

/* The colour of a valid splat (see orc_project_one). */
static void orc_colour_one(const orc_asset *a, const double *chat, uint32_t row, orc_splat *o)
{
    const float *p = a->pos + 3 * (size_t)row;
    int deg = (int)a->sh_degree, nc = (deg + 1) * (deg + 1);
    double dir[3] = {(double)p[0] - chat[0], (double)p[1] - chat[1], (double)p[2] - chat[2]};
    double Y[16];
    orc_sh_basis(deg, dir, Y);
    const float *c = a->sh + (size_t)row * nc * 3;
    double rgb[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nc; ++k)
        for (int ch = 0; ch < 3; ++ch) rgb[ch] += (double)c[k * 3 + ch] * Y[k];
    o->r = fmax(0.0, rgb[0] + 0.5);
    o->g = fmax(0.0, rgb[1] + 0.5);
    o->b = fmax(0.0, rgb[2] + 0.5);
}

typedef struct {
    uint64_t n_slots, n_valid;
    orc_splat *sp;       /* per slot */
    uint64_t n_order;    /* entries of order[] */
    uint64_t *order;     /* valid slots (with the index: those whose box meets the image), by (depth, slot) */
    /* bucket index */
    uint32_t bw, bh, nbx, nby;
    uint64_t *bstart;    /* nbx*nby+1 */
    uint64_t *blist;     /* positions into order[] */
} orc_frame;

static const orc_splat *g_sort_sp; /* qsort has no context argument */

static int orc_cmp(const void *pa, const void *pb)
{
    uint64_t ia = *(const uint64_t *)pa, ib = *(const uint64_t *)pb;
    float da = g_sort_sp[ia].depth, db = g_sort_sp[ib].depth;
    if (da < db) return -1;
    if (da > db) return 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* Support of a splat: the pixels where alpha >= 1/255, i.e. d^T conic d <= Q with
 * Q = 2 ln(255 o).  Its bounding box half-extents are sqrt(Q Sigma2_xx) and
 * sqrt(Q Sigma2_yy); widened here so that every decision that could be
 * ambiguous lies inside.  Pixel centres are at (x+0.5, y+0.5). */
static int orc_box(const orc_splat *s, const orc_camera *cam, int *x0, int *x1, int *y0, int *y1)
{
    if (!s->valid || !(255.0 * s->o >= 1.0 - AMBIG_REL)) return 0;
    double Q = 2.0 * log(fmax(255.0 * s->o, 1.0)) + 1e-3;
    double hx = sqrt(Q * s->sxx) * (1.0 + 1.0 / 1024.0) + 2.0;
    double hy = sqrt(Q * s->syy) * (1.0 + 1.0 / 1024.0) + 2.0;
    double fx0 = ceil(s->mx - hx - 0.5), fx1 = floor(s->mx + hx - 0.5);
    double fy0 = ceil(s->my - hy - 0.5), fy1 = floor(s->my + hy - 0.5);
    if (fx1 < 0 || fy1 < 0 || fx0 > (double)cam->width - 1 || fy0 > (double)cam->height - 1) return 0;
    *x0 = fx0 < 0 ? 0 : (int)fx0;
    *y0 = fy0 < 0 ? 0 : (int)fy0;
    *x1 = fx1 > cam->width - 1 ? (int)cam->width - 1 : (int)fx1;
    *y1 = fy1 > cam->height - 1 ? (int)cam->height - 1 : (int)fy1;
    return 1;
}

static int orc_prepare(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
                       uint64_t n_gids, const uint32_t *gids, int use_index, orc_frame *f)
{
    memset(f, 0, sizeof(*f));
    uint32_t ni = n_inst ? n_inst : 1;
    float *A = (float *)malloc(sizeof(float) * 12 * ni);
    float *sc = (float *)malloc(sizeof(float) * ni);
    double *ch = (double *)malloc(sizeof(double) * 3 * ni);
    float K;
    orc_frame_setup(n_inst, T, cam, A, sc, ch, &K);
    uint64_t n = orc_count_slots(a, n_gids, gids);
    f->n_slots = n;
    uint32_t *inst = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *row = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    orc_build_slots(a, n_gids, gids, inst, row);
    uint64_t nv = 0, nvalid = 0;
    if (!use_index) {
        f->sp = (orc_splat *)malloc(sizeof(orc_splat) * (n ? n : 1));
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < (int64_t)n; ++t) {
            const double *cht = ch + 3 * (size_t)inst[t];
            orc_project_one(a, A + 12 * (size_t)inst[t], cht, cam, row[t], &f->sp[t]);
            if (f->sp[t].valid) orc_colour_one(a, cht, row[t], &f->sp[t]);
        }
        f->order = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
        for (uint64_t t = 0; t < n; ++t)
            if (f->sp[t].valid) f->order[nv++] = t;
        nvalid = nv;
    } else {
        /* With the index, a slot whose box misses the image is in no pixel's
         * bucket list, so it is left out altogether: its record is not kept
         * and it is not sorted.  The kept records are stored in slot order
         * (their positions order them as their slots do), so the same pixels
         * visit the same splats in the same order.  Two passes over fixed
         * blocks of slots: count the kept ones, then store them. */
        const uint64_t blk = 1u << 16, nb = (n + blk - 1) / blk;
        uint64_t *bcnt = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
        uint64_t *bval = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < (int64_t)nb; ++b) {
            uint64_t kept = 0, valid = 0;
            for (uint64_t t = (uint64_t)b * blk; t < n && t < (uint64_t)(b + 1) * blk; ++t) {
                orc_splat sp;
                int x0, x1, y0, y1;
                orc_project_one(a, A + 12 * (size_t)inst[t], ch + 3 * (size_t)inst[t], cam, row[t], &sp);
                valid += sp.valid;
                kept += (uint64_t)orc_box(&sp, cam, &x0, &x1, &y0, &y1);
            }
            bcnt[b + 1] = kept;
            bval[b + 1] = valid;
        }
        for (uint64_t b = 0; b < nb; ++b) {
            bcnt[b + 1] += bcnt[b];
            nvalid += bval[b + 1];
        }
        nv = bcnt[nb];
        f->sp = (orc_splat *)malloc(sizeof(orc_splat) * (nv ? nv : 1));
        f->order = (uint64_t *)malloc(sizeof(uint64_t) * (nv ? nv : 1));
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < (int64_t)nb; ++b) {
            uint64_t j = bcnt[b];
            for (uint64_t t = (uint64_t)b * blk; t < n && t < (uint64_t)(b + 1) * blk; ++t) {
                orc_splat sp;
                int x0, x1, y0, y1;
                const double *cht = ch + 3 * (size_t)inst[t];
                orc_project_one(a, A + 12 * (size_t)inst[t], cht, cam, row[t], &sp);
                if (!orc_box(&sp, cam, &x0, &x1, &y0, &y1)) continue;
                orc_colour_one(a, cht, row[t], &sp);
                f->sp[j] = sp;
                f->order[j] = j;
                ++j;
            }
        }
        free(bcnt);
        free(bval);
    }
    free(inst);
    free(row);
    free(A);
    free(sc);
    free(ch);
    f->n_valid = nvalid;
    f->n_order = nv;
    /* stable order by FP32 depth; equal depths keep slot order */
    g_sort_sp = f->sp;
    qsort(f->order, nv, sizeof(uint64_t), orc_cmp);
    if (use_index) {
        f->bw = 32;
        f->bh = 32;
        f->nbx = (cam->width + f->bw - 1) / f->bw;
        f->nby = (cam->height + f->bh - 1) / f->bh;
        uint64_t nb = (uint64_t)f->nbx * f->nby;
        f->bstart = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
        for (uint64_t j = 0; j < nv; ++j) {
            int x0, x1, y0, y1;
            if (!orc_box(&f->sp[f->order[j]], cam, &x0, &x1, &y0, &y1)) continue;
            for (int by = y0 / (int)f->bh; by <= y1 / (int)f->bh; ++by)
                for (int bx = x0 / (int)f->bw; bx <= x1 / (int)f->bw; ++bx) f->bstart[(size_t)by * f->nbx + bx + 1]++;
        }
        for (uint64_t b = 0; b < nb; ++b) f->bstart[b + 1] += f->bstart[b];
        f->blist = (uint64_t *)malloc(sizeof(uint64_t) * (f->bstart[nb] ? f->bstart[nb] : 1));
        uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * (nb ? nb : 1));
        memcpy(fill, f->bstart, sizeof(uint64_t) * nb);
        for (uint64_t j = 0; j < nv; ++j) {
            int x0, x1, y0, y1;
            if (!orc_box(&f->sp[f->order[j]], cam, &x0, &x1, &y0, &y1)) continue;
            for (int by = y0 / (int)f->bh; by <= y1 / (int)f->bh; ++by)
                for (int bx = x0 / (int)f->bw; bx <= x1 / (int)f->bw; ++bx) f->blist[fill[(size_t)by * f->nbx + bx]++] = j;
        }
        free(fill);
    }
    return 0;
}

static void orc_frame_free(orc_frame *f)
{
    free(f->sp);
    free(f->order);
    free(f->bstart);
    free(f->blist);
}

static int orc_near(double v, double thr) { return fabs(v - thr) <= AMBIG_REL * thr; }

/* Front-to-back compositing of one pixel (Sec. 2.1), FP64:
 *   power = min(0, -1/2 (A dx^2 + C dy^2) - B dx dy);  alpha = min(0.99, o e^power);
 *   alpha < 1/255 contributes nothing;  T' = T (1 - alpha); when T' < 1e-4 the
 *   pixel is finished and this splat is not added;  C += alpha T rgb;  T = T'.
 *   Output RGB = C + T bg, A = 1 - T. */
static void orc_pixel(const orc_frame *f, const orc_camera *cam, int px, int py, int use_index,
                      double *out4, uint8_t *amb, uint64_t *pairs, uint64_t *hits)
{
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    double pcx = px + 0.5, pcy = py + 0.5;
    uint64_t j0, j1;
    const uint64_t *lst = NULL;
    if (use_index) {
        uint64_t b = (uint64_t)(py / (int)f->bh) * f->nbx + (uint64_t)(px / (int)f->bw);
        j0 = f->bstart[b];
        j1 = f->bstart[b + 1];
        lst = f->blist;
    } else {
        j0 = 0;
        j1 = f->n_order;
    }
    uint8_t ambiguous = 0;
    uint64_t np = 0, nh = 0;
    for (uint64_t jj = j0; jj < j1; ++jj) {
        uint64_t j = lst ? lst[jj] : jj;
        const orc_splat *s = &f->sp[f->order[j]];
        double dx = s->mx - pcx, dy = s->my - pcy;
        double power = -0.5 * (s->ca * dx * dx + s->cc * dy * dy) - s->cb * dx * dy;
        if (power > 0.0) power = 0.0;
        double alpha = s->o * exp(power);
        if (alpha > 0.99) alpha = 0.99;
        ++np;
        if (orc_near(alpha, 1.0 / 255.0)) ambiguous = 1;
        if (alpha < 1.0 / 255.0) continue;
        ++nh; /* this splat is composited, or it ends the pixel */
        double Tn = T * (1.0 - alpha);
        if (orc_near(Tn, 1e-4)) ambiguous = 1;
        if (Tn < 1e-4) break;
        C[0] += alpha * T * s->r;
        C[1] += alpha * T * s->g;
        C[2] += alpha * T * s->b;
        T = Tn;
    }
    out4[0] = C[0] + T * cam->bg[0];
    out4[1] = C[1] + T * cam->bg[1];
    out4[2] = C[2] + T * cam->bg[2];
    out4[3] = 1.0 - T;
    if (amb) *amb = ambiguous;
    *pairs += np;
    *hits += nh;
}

void orc_project(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
                 uint64_t n_gids, const uint32_t *gids,
                 uint8_t *valid, float *depth, double *mean2, double *conic,
                 double *rgb, double *opac, double *cov2)
{
    orc_frame f;
    orc_prepare(a, n_inst, T, cam, n_gids, gids, 0, &f);
    for (uint64_t t = 0; t < f.n_slots; ++t) {
        const orc_splat *s = &f.sp[t];
        valid[t] = s->valid;
        depth[t] = s->depth;
        mean2[2 * t] = s->mx;
        mean2[2 * t + 1] = s->my;
        conic[3 * t] = s->ca;
        conic[3 * t + 1] = s->cb;
        conic[3 * t + 2] = s->cc;
        rgb[3 * t] = s->r;
        rgb[3 * t + 1] = s->g;
        rgb[3 * t + 2] = s->b;
        opac[t] = s->o;
        cov2[3 * t] = s->sxx;
        cov2[3 * t + 1] = s->sxy;
        cov2[3 * t + 2] = s->syy;
    }
    orc_frame_free(&f);
}

int orc_render(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
               uint64_t n_gids, const uint32_t *gids, int use_index, int n_threads,
               double *rgba_out, uint8_t *ambiguous_out, orc_stats *stats)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    orc_frame f;
    orc_prepare(a, n_inst, T, cam, n_gids, gids, use_index, &f);
    uint64_t pairs = 0, hits = 0, namb = 0;
    int W = (int)cam->width, H = (int)cam->height;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : pairs, hits, namb)
    for (int py = 0; py < H; ++py) {
        for (int px = 0; px < W; ++px) {
            uint8_t amb = 0;
            size_t idx = (size_t)py * W + px;
            orc_pixel(&f, cam, px, py, use_index, rgba_out + 4 * idx, &amb, &pairs, &hits);
            if (ambiguous_out) ambiguous_out[idx] = amb;
            namb += amb;
        }
    }
    if (stats) {
        stats->n_slots = f.n_slots;
        stats->n_valid = f.n_valid;
        stats->n_ambiguous = namb;
        stats->n_pairs = pairs;
        stats->n_hits = hits;
    }
    orc_frame_free(&f);
    return 0;
}

int orc_render_pixels(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
                      uint64_t n_gids, const uint32_t *gids, uint64_t n_pix, const uint32_t *pix_xy,
                      int n_threads, double *rgba_out, uint8_t *ambiguous_out, orc_stats *stats)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    orc_frame f;
    orc_prepare(a, n_inst, T, cam, n_gids, gids, 1, &f);
    uint64_t pairs = 0, hits = 0, namb = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : pairs, hits, namb)
    for (int64_t i = 0; i < (int64_t)n_pix; ++i) {
        uint8_t amb = 0;
        orc_pixel(&f, cam, (int)pix_xy[2 * i], (int)pix_xy[2 * i + 1], 1, rgba_out + 4 * i, &amb, &pairs, &hits);
        if (ambiguous_out) ambiguous_out[i] = amb;
        namb += amb;
    }
    if (stats) {
        stats->n_slots = f.n_slots;
        stats->n_valid = f.n_valid;
        stats->n_ambiguous = namb;
        stats->n_pairs = pairs;
        stats->n_hits = hits;
    }
    orc_frame_free(&f);
    return 0;
}
