/*
 * CPU oracle for the V3DG per-frame path.  TEST INFRASTRUCTURE ONLY: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code, header or constant with the HIP library.
 *
 * What it computes, and from which passage of the paper:
 *   - footprint F = pi r^2 fx fy / z_v^2 of a cluster-group bounding sphere
 *     (Sec. 3.3, footprint figure) and the selection rule F_c <= tau < F_p
 *     (Sec. 3.4), evaluated as a literal recursive walk of the cluster tree;
 *   - the 3DGS splat of each selected Gaussian (Sec. 2.1; rasterised with
 *     the original splatting algorithm, Sec. 3 overview and Sec. 5.1, with
 *     no 2D dilation) in FP64;
 *   - front-to-back alpha compositing of every pixel over every depth-sorted
 *     splat in FP64 (Sec. 2.1).
 * Decision quantities that pick integers (the FP32 depth used for the cull
 * and the sort, the footprint predicate) are evaluated in FP32 in the fixed
 * operation order that defines them; everything else is FP64.
 */
#ifndef V3DG_ORACLE_H
#define V3DG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t n_clusters, n_rows, sh_degree, pad0;
    const float *self_sphere;     /* n_clusters x 4 (cx,cy,cz,r); r = 0 leaf */
    const float *parent_sphere;   /* n_clusters x 4; r = +inf root           */
    const uint32_t *first_row;    /* n_clusters */
    const uint8_t *count;         /* n_clusters */
    const int32_t *parent;        /* n_clusters, -1 root */
    const int32_t *first_child;   /* n_clusters, -1 leaf */
    const uint8_t *n_children;    /* n_clusters */
    const float *pos;             /* n_rows x 3 */
    const float *scale;           /* n_rows x 3 (linear) */
    const float *rot;             /* n_rows x 4 (w,x,y,z) */
    const float *opacity;         /* n_rows */
    const float *sh;              /* n_rows x (deg+1)^2 x 3 */
} orc_asset;

typedef struct {
    uint32_t width, height;
    float fx, fy, cx, cy;
    float V[12];                  /* world->camera 3x4 row-major, OpenCV axes */
    float near_plane, far_plane;
    float bg[3];
    float pad0;
} orc_camera;

/* n_pairs: (pixel, splat) pairs visited (the bucket's splats up to the
 * pixel's end); n_hits: of those, the splats with alpha >= 1/255, i.e. the
 * ones composited plus the one that ends the pixel. */
typedef struct {
    uint64_t n_slots, n_valid, n_ambiguous, n_pairs, n_hits;
} orc_stats;

/* Per-instance frame quantities: A = fl32(V T) composed in FP64, s = fl32 of
 * the instance's uniform scale, chat = T^{-1}(camera centre) in FP64.
 * T is n_inst x 12 (3x4 row-major, FP64). */
void orc_frame_setup(uint32_t n_inst, const double *T, const orc_camera *cam,
                     float *A_out, float *s_out, double *chat_out, float *K_out);

/* Literal recursive walk (Sec. 3.4): for each instance and each root, a
 * cluster is emitted when its own footprint fits tau, otherwise its children
 * are visited.  out_mask is n_inst x n_clusters bytes.  Returns the number of
 * selected clusters. */
uint64_t orc_select_walk(const orc_asset *a, uint32_t n_inst, const double *T,
                         const orc_camera *cam, float tau, uint8_t *out_mask);

/* The parallel predicate F_c <= tau < F_p evaluated for every (instance,
 * cluster), used by the tests to check the walk against it. */
uint64_t orc_select_predicate(const orc_asset *a, uint32_t n_inst, const double *T,
                              const orc_camera *cam, float tau, uint8_t *out_mask);

/* Footprint of one sphere seen through row 2 of A with scale s; +inf when the
 * camera plane is within the sphere (|z| <= r). FP64, for reporting. */
double orc_footprint(const float sphere[4], const float A_row2[4], float s, float fx, float fy);

/* Real spherical harmonics (Condon-Shortley phase, m = -l..l per band) from
 * the associated Legendre definition, FP64, up to degree 3. */
void orc_sh_basis(int degree, const double dir[3], double *out);

/* Per-slot projection of the gids' rows (slot order: ascending gid, rows in
 * stored order).  Arrays are n_slots long (x2, x3 where noted). */
uint64_t orc_count_slots(const orc_asset *a, uint64_t n_gids, const uint32_t *gids);
void orc_project(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
                 uint64_t n_gids, const uint32_t *gids,
                 uint8_t *valid, float *depth, double *mean2 /*x2*/, double *conic /*x3*/,
                 double *rgb /*x3*/, double *opac, double *cov2 /*x3*/);

/* Full render: slots from gids, FP64 projection, stable (depth, slot) order,
 * per-pixel FP64 compositing.  use_index = 0 is brute force over every
 * splat for every pixel; 1 uses an exact bucket index.  rgba_out is
 * H x W x 4 (FP64), ambiguous_out is H x W bytes (may be NULL). */
int orc_render(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
               uint64_t n_gids, const uint32_t *gids, int use_index, int n_threads,
               double *rgba_out, uint8_t *ambiguous_out, orc_stats *stats);

/* Render only the listed pixels (x,y pairs) with the exact index; for
 * sampled parity checks on large frames. */
int orc_render_pixels(const orc_asset *a, uint32_t n_inst, const double *T, const orc_camera *cam,
                      uint64_t n_gids, const uint32_t *gids, uint64_t n_pix, const uint32_t *pix_xy,
                      int n_threads, double *rgba_out, uint8_t *ambiguous_out, orc_stats *stats);

#ifdef __cplusplus
}
#endif
#endif
