/*
 * v3dg — per-frame hot path of Virtualized 3D Gaussians on MI355X (gfx950).
 *
 * The library keeps one asset's cluster hierarchy and Gaussians resident in
 * HBM together with a table of rigid instances, and per frame
 *   1. tests every (instance, cluster) footprint against a tolerance and
 *       compacts the cut (paper Sec. 3.4, selection run in parallel over
 *       the discrete clusters; footprint of Sec. 3.3),
 *   2. compacts the chosen clusters' Gaussians into a slot stream,
 *   3. projects each Gaussian to a 2D conic and colour (3D Gaussian splat of
 *       Sec. 2.1, no 2D dilation as in Sec. 5.1),
 *   4. bins the splats to 32x32-pixel bins and puts every bin's splats in
 *       depth order: a stable radix sort of the slots by FP32 depth, then bin
 *       ids emitted in that order (16-bit up to 65,536 bins, else 32-bit) and
 *       stably radix-sorted (the same order as 64-bit (bin, depth) keys, which
 *       remain selectable with v3dg_set_sort_mode),
 *   5. alpha-composites every 16x16-pixel tile front to back (Sec. 2.1) from
 *       its bin's list, each 8x8 quarter walking the splats that reach it.
 * All device work runs as HIP kernels on the stream given at load time.
 *
 * Conventions for every entry point:
 *   - return 0 (V3DG_OK) or a negative V3DG_ERR_* code; the message of the last
 *     failure on the calling thread is available from v3dg_last_error();
 *   - nothing is written to caller memory when a call fails;
 *   - calls are asynchronous on the scene's stream unless marked "synchronises";
 *     the first v3dg_render of an image size also waits once, mid-frame, for
 *     the device-side key count (later frames of that size do not wait);
 *   - host arrays passed in are only read during the call; device pointers
 *     (the image) stay owned by the caller.
 */
#ifndef V3DG_H
#define V3DG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define V3DG_OK 0
#define V3DG_ERR_INVALID_ARG (-1)  /* bad pointer, size, non-finite value, malformed tree */
#define V3DG_ERR_OOM (-2)          /* device or host allocation failed                    */
#define V3DG_ERR_HIP (-3)          /* a HIP runtime call failed                            */
#define V3DG_ERR_NOT_MONOTONE (-4) /* parent sphere does not nest its child (see load)     */
#define V3DG_ERR_CAPACITY (-5)     /* a frame exceeds a 32-bit count                       */
#define V3DG_ERR_DEVICE (-6)       /* a kernel raised its error flag (bounded wait expired)*/
#define V3DG_ERR_IO (-7)           /* a page file could not be written or read            */

/* Storage precision of the Gaussian attributes (positions always stay FP32;
 * arithmetic is FP32 in every case).  The library rounds the FP32 input of
 * v3dg_load_hierarchy to nearest-even:
 *   V3DG_FP32         everything FP32                          (236 B/row at SH3)
 *   V3DG_FP16_BF16SH  scale, rotation, opacity FP16; SH BF16   (124 B/row at SH3)
 *   V3DG_FP16         scale, rotation, opacity and SH FP16     (124 B/row at SH3) */
#define V3DG_FP32 0u
#define V3DG_FP16_BF16SH 1u
#define V3DG_FP16 2u
/* load flags */
#define V3DG_LOAD_REPAIR_NESTING 1u /* inflate parent radii bottom-up instead of failing */

typedef struct v3dg_scene v3dg_scene;         /* opaque; library-owned */
typedef struct v3dg_selection v3dg_selection; /* opaque; library-owned */

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  Pixel (x, y) has
 * its centre at (x + 0.5, y + 0.5).  Requirements: 1 <= width, height <= 16384;
 * fx, fy > 0; every value finite; 0 < near_plane < far_plane. */
typedef struct {
    uint32_t width, height;
    float fx, fy, cx, cy;
    float world_to_cam[12]; /* 3x4 row-major [R | t] */
    float near_plane, far_plane;
    float bg[3];            /* background added as T * bg */
    float pad0;
} v3dg_camera;

/* One asset: clusters and Gaussian rows as structure-of-arrays host arrays.
 * Cluster k owns rows first_row[k] .. first_row[k] + count[k] - 1 (1 <= count <= 64).
 * Children of k are first_child[k] .. first_child[k] + n_children[k] - 1; leaves
 * have n_children = 0; roots have parent = -1.
 * self_sphere[k] = (cx, cy, cz, r) is the bounding sphere of the cluster group
 * k was simplified from (paper Sec. 3.3: centre = mean Gaussian position,
 * r = farthest Gaussian); leaves have r = 0.  parent_sphere[k] must equal
 * self_sphere[parent[k]] bit for bit, and r = +inf for roots (Sec. 3.4).
 * Gaussian rows: pos (x,y,z), scale (linear, > 0), rot unit quaternion
 * (w,x,y,z) within 1e-6, opacity in (0, 1], sh row-major
 * [(sh_degree+1)^2][3] real-SH coefficients (sh_degree 0..3).  All arrays
 * are FP32; `precision` (V3DG_FP32, V3DG_FP16_BF16SH, V3DG_FP16) selects how
 * the library stores them.  In the narrow tiers scale and opacity must stay
 * positive and finite after rounding. */
typedef struct {
    uint32_t n_clusters, n_rows, sh_degree, precision;
    const float *self_sphere;   /* n_clusters x 4 */
    const float *parent_sphere; /* n_clusters x 4 */
    const uint32_t *first_row;  /* n_clusters */
    const uint8_t *count;       /* n_clusters */
    const int32_t *parent;      /* n_clusters */
    const int32_t *first_child; /* n_clusters */
    const uint8_t *n_children;  /* n_clusters */
    const float *pos;           /* n_rows x 3 */
    const float *scale;         /* n_rows x 3 */
    const float *rot;           /* n_rows x 4 */
    const float *opacity;       /* n_rows */
    const float *sh;            /* n_rows x (sh_degree+1)^2 x 3 */
} v3dg_hierarchy_desc;

/* How each bin's splats are put in front-to-back order (same result):
 * DEPTH_FIRST sorts the slots by FP32 depth, emits bin ids in that order
 * (16-bit on grids of up to 65,536 bins, 32-bit beyond) and stably sorts them
 * by bin; KEYS64 emits (bin << 32 | depth bits) keys in slot order and sorts
 * all their significant bits. */
#define V3DG_SORT_DEPTH_FIRST 0
#define V3DG_SORT_KEYS64 1

/* Counters of the last frame rendered on a scene. */
typedef struct {
    uint64_t n_slots;    /* Gaussians in the rendered selection            */
    uint64_t n_keys;     /* (bin, splat) pairs sorted                      */
    uint32_t n_tiles;    /* 16x16-pixel tiles in the image (blended)       */
    uint32_t key_bits;   /* significant bits of the (last) sort key        */
    uint32_t sort_passes;/* radix passes of the bin / 64-bit key sort      */
    uint32_t sort_mode;  /* V3DG_SORT_*                                    */
    uint32_t n_fp64_conics;    /* splats whose 2D covariance determinant fell below
                                  1e-6 px^4 and was redone in FP64               */
    uint32_t n_conics_clamped; /* splats with a conic entry beyond 1e38 in
                                  magnitude, stored as +-1e38 (thinner than
                                  ~1e-19 px across: an axis-aligned needle still
                                  covers the pixel centres it runs through)      */
    uint32_t n_bins;     /* 32x32-pixel bins of the image (keys name bins)  */
} v3dg_frame_stats;

/* Kernel stages timed when profiling is on (v3dg_set_profiling). */
#define V3DG_STAGE_SETUP 0
#define V3DG_STAGE_SELECT 1
#define V3DG_STAGE_EXPAND 2
#define V3DG_STAGE_PROJECT 3
#define V3DG_STAGE_SCAN 4
#define V3DG_STAGE_EMIT 5
#define V3DG_STAGE_SORT_HIST 6
#define V3DG_STAGE_SORT_PASS 7
#define V3DG_STAGE_RANGES 8
#define V3DG_STAGE_BLEND 9
#define V3DG_STAGE_DEPTH_SORT 10 /* histogram + passes of the depth sort */
#define V3DG_N_STAGES 11

/* Upload an asset and its instances to HBM and validate it.
 * Validation (paper Sec. 3.4 keeps r_p > r_c so that a cluster and its parent
 * are never both selected; this library requires the stronger nesting that
 * makes the per-cluster test exact for every camera): for every non-root
 * cluster with r_c > 0, r_p >= (|c_p - c_c| + r_c) (1 + 2^-12).  A violation
 * returns V3DG_ERR_NOT_MONOTONE unless V3DG_LOAD_REPAIR_NESTING is set, in
 * which case parent radii are enlarged bottom-up (and the copies in
 * parent_sphere updated) on the library's copy.
 * instances_3x4: n_instances x 12 doubles, each [s R | t] with R a rotation
 * and s > 0 a uniform scale (paper Sec. 4.2 / Appendix A.2); 1 <= n_instances.
 * hip_stream: the hipStream_t every later call runs on (NULL = default).
 * On success *out receives a new scene; free it with v3dg_scene_free. */
int v3dg_load_hierarchy(const v3dg_hierarchy_desc *desc, const double *instances_3x4, uint32_t n_instances,
                        void *hip_stream, uint32_t flags, v3dg_scene **out);

/* Streamed load (the streaming module the paper's conclusion and discussion
 * leaves to future work): as v3dg_load_hierarchy, but the Gaussian rows stay
 * in host memory as one page image per cluster, and device memory holds a
 * pool of pool_clusters pages of 64 rows (1 <= pool_clusters < 2^26; a
 * larger pool than the scene's cluster count is cut to it; 0 loads the rows
 * resident, as v3dg_load_hierarchy).  Cluster tables, spheres and instances
 * stay resident.  v3dg_select runs on a stream of the scene's own, once the
 * previous render has projected its Gaussians; it reads the cut back (waiting
 * for that stream only, so the previous render's later stages go on), keeps
 * the resident clusters it uses, and pages in the others in place of the
 * least recently used pages that this cut does not use: the page images are
 * staged in pinned host memory, copied in one transfer per 2048 clusters and
 * scattered into their pages.  Work enqueued on the scene's stream after the
 * select waits for it on the device.  Images equal those of
 * the resident scene bit for bit.  A cut that needs more clusters than the
 * pool holds fails with V3DG_ERR_CAPACITY and pages nothing.  A selection is
 * renderable until a later select pages out one of its clusters; rendering it
 * after that fails with V3DG_ERR_INVALID_ARG.  Slot rows name pool rows.
 * v3dg_render_full pages in every leaf.  v3dg_copy_attributes and the server
 * take resident scenes only. */
int v3dg_load_hierarchy_streamed(const v3dg_hierarchy_desc *desc, const double *instances_3x4,
                                 uint32_t n_instances, void *hip_stream, uint32_t flags, uint32_t pool_clusters,
                                 v3dg_scene **out);

/* The same with the page images in a file on disk instead of host memory
 * (the tier below host memory).  The library creates (or truncates) page_file,
 * writes every cluster's image at a 4 KiB-aligned slot during the load, and
 * each select reads the images it pages in with positioned reads, one per
 * run of consecutive clusters, into the pinned stage.  file_flags:
 * V3DG_PAGE_FILE_DIRECT asks for reads that bypass the operating system's page
 * cache (O_DIRECT; where the file system refuses it the reads are buffered,
 * see v3dg_stream_stats.tier); V3DG_PAGE_FILE_KEEP keeps the file when the
 * scene is freed (it is removed otherwise).  pool_clusters must be > 0.  A
 * failed write or read returns V3DG_ERR_IO (a failed read pages nothing).
 * Images equal those of the resident scene bit for bit. */
#define V3DG_PAGE_FILE_DIRECT 1u
#define V3DG_PAGE_FILE_KEEP 2u
int v3dg_load_hierarchy_streamed_file(const v3dg_hierarchy_desc *desc, const double *instances_3x4,
                                      uint32_t n_instances, void *hip_stream, uint32_t flags, uint32_t pool_clusters,
                                      const char *page_file, uint32_t file_flags, v3dg_scene **out);

/* Paging counters of a streamed scene (zeros for a resident one). */
typedef struct {
    uint64_t frames;            /* cuts paged in (selects and full renders)          */
    uint64_t pages_in;          /* clusters copied into the pool                     */
    uint64_t bytes_in;          /* host-to-device bytes of those page images         */
    uint64_t evictions;         /* resident clusters whose page was given to another */
    uint64_t last_pages_in;     /* clusters paged in by the latest cut               */
    uint32_t last_resident_used;/* resident clusters the latest cut uses             */
    uint32_t pool_clusters;     /* pages in the pool                                 */
    uint32_t resident;          /* clusters resident now                             */
    uint32_t tier;              /* where the page images live: 0 host memory, 1 a
                                   file read through the page cache, 2 a file read
                                   directly (O_DIRECT)                              */
    uint64_t file_reads;        /* positioned reads of the page file so far          */
} v3dg_stream_stats;
int v3dg_get_stream_stats(const v3dg_scene *scene, v3dg_stream_stats *out);

/* Replace the instance transforms (same count), e.g. every frame of a dynamic
 * scene of rigid objects (paper Appendix A.3). */
int v3dg_set_instances(v3dg_scene *scene, const double *instances_3x4, uint32_t n_instances);

/* Parallel selection (paper Sec. 3.4): cluster k of instance i is selected iff
 * F(own sphere) <= tolerance < F(parent sphere), F = pi r^2 fx fy / z^2 the
 * pixel area of the sphere (Sec. 3.3).  tolerance is in the unit of F (pixel
 * area), finite and >= 0.  The exact FP32 predicate: z = ((a0 cx + a1 cy) +
 * a2 cz) + a3 with row 2 of A = fl32(V T_i); r' = r s_i; "fits" is r' == 0, or
 * |z| > r' and (r' r') K <= tolerance (z z) with K = fl32(pi fx fy).
 * Also expands the chosen clusters into the slot stream (one slot per
 * Gaussian, ascending gid = i * n_clusters + k, rows in stored order).
 * *inout: NULL to get a new selection object, or an existing one of this
 * scene to overwrite (its buffers are reused). */
int v3dg_select(v3dg_scene *scene, const v3dg_camera *cam, float tolerance, v3dg_selection **inout);

/* Render a selection: project, bin, sort, blend.  image_rgba_dev is a device
 * buffer of height x width x 4 floats (RGB = sum + T bg, A = 1 - T), written
 * completely.  The first frame of an image size (and every frame in the
 * 64-bit-key sort mode) synchronises once mid-frame to size the key buffers
 * exactly.  Later frames of that size run without any host wait: their
 * launches are sized by a key capacity of at least 2^20 keys, 48 keys per
 * pixel (up to 2^27 keys) and twice the most keys any frame needed, the kernels read their counts on the
 * device, and each frame publishes its counts to pinned host memory, read
 * when a later call finds the frame finished.  A frame that needs more keys
 * than the capacity is still rendered exactly, by every tile walking all
 * visible splats in depth order (slower); the capacity then grows for the
 * frames after.  Such a frame's sorted keys are not available
 * (v3dg_copy_sorted_keys fails with V3DG_ERR_CAPACITY). */
int v3dg_render(v3dg_scene *scene, const v3dg_camera *cam, const v3dg_selection *sel, float *image_rgba_dev);

/* Full-detail baseline: every leaf cluster of every instance (no selection). */
int v3dg_render_full(v3dg_scene *scene, const v3dg_camera *cam, float *image_rgba_dev);

/* Selected cluster and Gaussian counts (synchronises). */
int v3dg_selection_info(const v3dg_selection *sel, uint64_t *n_clusters, uint64_t *n_gaussians);

/* Copy the ascending gid list to host memory (synchronises).  Fails with
 * V3DG_ERR_CAPACITY when cap is smaller than the count. */
int v3dg_selection_copy_ids(const v3dg_selection *sel, uint32_t *host_gids, uint64_t cap, uint64_t *n_out);

/* Copy the slot stream (row and instance of every selected Gaussian). */
int v3dg_selection_copy_slots(const v3dg_selection *sel, uint32_t *host_rows, uint32_t *host_inst, uint64_t cap,
                              uint64_t *n_out);

void v3dg_selection_free(v3dg_selection *sel);
void v3dg_scene_free(v3dg_scene *scene);

/* Counters of the last frame rendered on this scene (synchronises). */
int v3dg_get_frame_stats(v3dg_scene *scene, v3dg_frame_stats *out);

/* Per-slot results of the last frame's projection (synchronises), for
 * parity checks.  Arrays of cap entries: mean2 x2, conic x3, rgb x3; depth;
 * opacity; tiles = bins touched (0 = culled). */
int v3dg_copy_projection(v3dg_scene *scene, float *mean2, float *conic, float *rgb, float *opacity, float *depth,
                         uint32_t *tiles, uint64_t cap, uint64_t *n_out);

/* The stored Gaussian attributes of rows [first, first + n), widened to FP32
 * (synchronises): what the projection reads in the scene's precision tier.
 * Layouts as in v3dg_hierarchy_desc (pos x3, scale x3, rot x4, opacity,
 * sh 3 (d+1)^2); any pointer may be NULL.  V3DG_ERR_INVALID_ARG when the
 * range leaves the table. */
int v3dg_copy_attributes(v3dg_scene *scene, uint64_t first, uint64_t n, float *pos, float *scale, float *rot,
                         float *opacity, float *sh);

/* The last frame's sorted keys as (bin << 32 | depth bits) and values
 * (slot), whatever the sort mode (synchronises). */
int v3dg_copy_sorted_keys(v3dg_scene *scene, uint64_t *keys, uint32_t *vals, uint64_t cap, uint64_t *n_out);

/* Work done and time spent since the previous v3dg_collect_profile. */
typedef struct {
    double ms[V3DG_N_STAGES];          /* summed kernel time per stage (profiling on) */
    uint64_t launches[V3DG_N_STAGES];  /* timed launches per stage                    */
    uint64_t frames;                   /* renders                                     */
    uint64_t selects, tests;           /* selections, (instance, cluster) tests       */
    uint64_t sel_clusters;             /* selected clusters of the rendered selections*/
    uint64_t slots, visible;           /* Gaussians projected / with a bin            */
    uint64_t keys, tiles, pixels;      /* sorted keys, image tiles, image pixels      */
    uint64_t sort_passes;              /* digit passes of the bin / 64-bit key sort   */
    uint64_t depth_sorts;              /* frames that sorted slots by depth first     */
    uint64_t pairs;                    /* (pixel, splat) pairs evaluated by blending: for
                                          each splat of a quarter's list, the quarter's
                                          pixels still compositing when it is reached.
                                          Counted only with V3DG_PROFILE_PAIRS (or
                                          PAIR_AUDIT), else 0                            */
    uint64_t pairs_taken;              /* of those, pairs with alpha >= 1/255 (composited,
                                          or ending the pixel); later chunks of long bin
                                          lists are walked from T = 1 and count pairs a
                                          sequential walk would not reach.  Counted only
                                          with V3DG_PROFILE_PAIR_AUDIT, else 0            */
} v3dg_profile;

/* View culling of the cut (default off).  When on, v3dg_select still returns
 * the paper's cut (v3dg_selection_copy_ids is unchanged) but gives no slots
 * to an (instance, cluster) that provably cannot reach the image: behind the
 * near plane, or with every Gaussian's enlarged support box (half-extent
 * bounded from the cluster's largest scale) at least 2 pixels outside it.
 * Images are unchanged bit for bit; fewer Gaussians are projected, sorted
 * and binned. */
int v3dg_set_culling(v3dg_scene *scene, int on);

/* Chunk sizes of long bin lists for later renders of this scene (default
 * 1024).  Blending composites each bin's depth-sorted list front to back
 * (Sec. 2.1); a list longer than 3 * keys is walked as a first chunk of
 * 3 * keys and further chunks of `keys`, in parallel, folded in order and
 * walked again where a pixel stops (the sequential result up to the
 * association of FP32 products).  Smaller chunks shorten a frame's longest
 * walk; larger ones walk fewer pairs twice, which pays when several frames
 * share the device (the serving loop's default is 4096).  keys: 1024, 2048
 * or 4096, else V3DG_ERR_INVALID_ARG.  Images of different chunk sizes may
 * differ in the last bits. */
int v3dg_set_chunk_keys(v3dg_scene *scene, uint32_t keys);

/* Select the sort strategy for later renders of this scene (default
 * V3DG_SORT_DEPTH_FIRST).  Both give bit-identical images. */
int v3dg_set_sort_mode(v3dg_scene *scene, int mode);

/* Stage timing with hipEvents on the scene's stream.  stage_mask selects the
 * stages whose launches are bracketed by events (bit s for stage s,
 * V3DG_PROFILE_ALL for every stage, 0 for none).  Work counters are kept
 * either way.  v3dg_collect_profile synchronises, fills *out with the totals
 * since the previous collect, and clears them. */
#define V3DG_PROFILE_ALL 0x7ff
/* Added to stage_mask: blending counts the (pixel, splat) pairs it walks
 * (v3dg_profile.pairs, otherwise 0); with PAIR_AUDIT also the pairs it takes
 * (v3dg_profile.pairs_taken).  Counting costs a few scalar operations per
 * pair on the walk's critical path (about 4 % of the blend stage for pairs),
 * so both are off by default. */
#define V3DG_PROFILE_PAIR_AUDIT 0x800
#define V3DG_PROFILE_PAIRS 0x1000
int v3dg_set_profiling(v3dg_scene *scene, int stage_mask);
int v3dg_collect_profile(v3dg_scene *scene, v3dg_profile *out);

/* Stable LSD radix sort of n (key, value) pairs in device memory by the low
 * key_bits bits of the keys (1..64), the primitive behind binning.  Synchronises;
 * allocates its own temporary buffers. */
int v3dg_sort_pairs(uint64_t *keys_dev, uint32_t *vals_dev, uint64_t n, uint32_t key_bits, void *hip_stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): v3dg_sort_pairs
 * without any allocation.  Its temporaries (alternate keys and values,
 * look-back words, counters) live in one fixed device array per GPU, about
 * 12.6 MB, held until the process ends; the array is looked up (not
 * allocated) on the first call on a device.  n <= V3DG_SORT_NOALLOC_MAX, else
 * V3DG_ERR_CAPACITY with nothing sorted.  Same arguments, result and errors
 * as v3dg_sort_pairs; synchronises.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other host threads, other streams)
 * race and must be serialised by the caller. */
#define V3DG_SORT_NOALLOC_MAX (1u << 20)
int v3dg_sort_pairs_noalloc(uint64_t *keys_dev, uint32_t *vals_dev, uint64_t n, uint32_t key_bits,
                            void *hip_stream);

/* ---- serving ----------------------------------------------------------------
 * A server renders camera requests against several resident scenes with
 * several frames in flight (continuous batching).  Requests queue on the host;
 * each v3dg_server_poll retires finished frames and admits queued requests
 * into free render contexts while the contexts' workspaces fit the HBM
 * budget.  The requests admitted in one poll are selected together: one
 * set-up launch, one persistent selection launch over all their (instance,
 * cluster) tests and one expansion launch.  Each context then renders its
 * request on its own stream, by replaying a captured HIP graph of the render
 * chain (one per scene and image size) or by direct launches.  Frames run
 * without host waits: launches are sized by the context's capacities and
 * the kernels read every count from device memory; a frame that needs more
 * keys than its context holds is detected on completion and rendered again
 * after the context grows.  Images equal those of v3dg_select +
 * v3dg_render bit for bit.  Single-threaded: one host thread drives a
 * server; all its scenes must live on the current device. */
typedef struct v3dg_server v3dg_server;

typedef struct {
    uint32_t n_contexts;        /* render contexts (frames in flight), 1..64              */
    uint32_t max_batch;         /* requests admitted per batched selection, 1..64          */
    uint64_t hbm_budget_bytes;  /* device memory the contexts' workspaces may hold in total */
    uint32_t use_graphs;        /* 1: replay captured graphs, 0: launch directly          */
    uint32_t keys_per_pixel;    /* key capacity first provisioned per pixel of an image size
                                   not seen yet (0: 24); later frames of a size get 1.25 x the
                                   most keys seen                                          */
    uint32_t cull;              /* 1: view culling of the cut, as v3dg_set_culling          */
    uint32_t chunk_keys;        /* keys per later chunk of long bin lists, as
                                   v3dg_set_chunk_keys (0: 4096)                           */
} v3dg_server_config;

typedef struct {
    uint64_t ticket;            /* from v3dg_server_submit                                */
    int32_t status;             /* V3DG_OK or a negative error code                       */
    uint32_t retries;           /* renders repeated after a key-capacity overflow         */
    uint64_t n_slots, n_keys;   /* Gaussians projected and keys sorted                    */
    double submit_ms, admit_ms, done_ms;  /* host clock (ms since server creation):
                                             queued, admitted, completion seen by poll  */
} v3dg_request_done;

typedef struct {
    uint64_t submitted, completed, failed, retries;
    uint64_t batches, batched_requests;  /* selection launches and the requests they served  */
    uint64_t graph_captures, graph_launches;
    uint64_t workspace_bytes;            /* device memory the contexts hold now            */
    uint64_t peak_workspace_bytes;
    uint32_t contexts_live, queued;
} v3dg_server_stats;

/* Create a server over n_scenes loaded scenes (not owned: free the server
 * first).  Errors: V3DG_ERR_INVALID_ARG for a bad configuration or scene,
 * V3DG_ERR_OOM when not even one context fits the budget. */
int v3dg_server_create(v3dg_scene *const *scenes, uint32_t n_scenes, const v3dg_server_config *cfg,
                       v3dg_server **out);

/* Queue a request: render scene `scene` from `cam` at tolerance `tau` into
 * image_dev (caller-owned device memory, H x W x 4 FP32, untouched by the
 * caller until the request completes).  Nothing is launched until the next
 * poll.  *ticket identifies the request in v3dg_request_done. */
int v3dg_server_submit(v3dg_server *srv, uint32_t scene, const v3dg_camera *cam, float tau, float *image_dev,
                       uint64_t *ticket);

/* Queue a full-detail request: every leaf of scene `scene`, no selection
 * (v3dg_render_full through the serving loop; the paper's comparison with
 * vanilla 3DGS, Sec. 5).  The first such request of a scene builds the
 * scene's list of leaves (one synchronisation of the scene's stream).  Same
 * image contract and errors as v3dg_server_submit. */
int v3dg_server_submit_full(v3dg_server *srv, uint32_t scene, const v3dg_camera *cam, float *image_dev,
                            uint64_t *ticket);

/* Retire finished frames (up to cap records into done[], count in *n_done),
 * then admit and launch queued requests.  wait != 0 blocks until at least one
 * frame has finished when any is in flight; it needs cap >= 1
 * (V3DG_ERR_INVALID_ARG otherwise). */
int v3dg_server_poll(v3dg_server *srv, int wait, v3dg_request_done *done, uint32_t cap, uint32_t *n_done);

int v3dg_server_get_stats(v3dg_server *srv, v3dg_server_stats *out);

/* Waits for the frames in flight, then frees every context. */
void v3dg_server_free(v3dg_server *srv);

/* ---- Offline build (paper Sec. 3.1-3.2, Algorithm 1), on the GPU -------------
 * Builds the cluster bundle of an asset from its n Gaussians: a binary median
 * split into clusters of at most cluster_size Gaussians (layer C_0); then,
 * while a layer holds two clusters or more, the same split pairs its clusters
 * into cluster groups, every group is halved to the ceil(m/2) Gaussians with
 * the largest ((sx sy) sz) opacity (ties: the earlier one in the group), whose
 * scales grow by float(2^(1/6)), and these form one cluster of the next layer.
 * The group's bounding sphere (centre: FP64 mean of its Gaussians' positions,
 * rounded to FP32; radius: the farthest of them, rounded up) is the new
 * cluster's own sphere and its members' parent sphere; it is grown to
 * (|c_p - c_c| + r_c)(1 + 2^-10) over every member so that spheres nest.
 * Leaves have radius 0 (centre: their mean); the root's parent radius is +inf.
 * Split of a set larger than the limit: the axis of the largest FP32 extent
 * (the first on ties), a stable order along it, ceil(s/2) items to the left.
 * Every coarser layer is made from the current rows of the layer below it:
 * means, spheres and halving scores use them as they stand.
 *
 * With fit_iters > 0, every group's kept Gaussians are refined right after
 * the halving by local splatting (Sec. 3.2, as v3dg_local_splat: the group's
 * Gaussians are the originals; the pseudo-views face the group centre from
 * four times the group's reach, the largest |p - c| + 3 max(sx, sy, sz) of
 * its Gaussians (FP64, rounded up to FP32), so that they frame the Gaussians'
 * 3-sigma extents; view i looks along view_dirs[3i .. 3i+2], the same
 * directions for every group);
 * with fit_iters = 0 the rows of a layer are plain copies of rows below
 * (structural build).  view_dirs: host, 3 x fit_iters finite non-zero floats
 * (normalised here), may be NULL when fit_iters = 0; fit_iters <= 2^20.
 *
 * Inputs are host arrays: pos, scale (n x 3), rot (n x 4), opacity (n), sh
 * (n x (sh_degree+1)^2 x 3), all FP32; 1 <= n < 2^31, sh_degree <= 3,
 * 2 <= cluster_size <= 64.  The result (cluster ids layer-major, within a layer
 * in grouping order; rows in cluster order) is owned by *out until
 * v3dg_bundle_free and is loadable with v3dg_load_hierarchy.  Synchronises.
 * Errors: V3DG_ERR_INVALID_ARG, V3DG_ERR_OOM, V3DG_ERR_HIP, V3DG_ERR_DEVICE. */
typedef struct v3dg_bundle v3dg_bundle;
int v3dg_build_bundle(const float *pos, const float *scale, const float *rot, const float *opacity, const float *sh,
                      uint32_t n, uint32_t sh_degree, uint32_t cluster_size, uint32_t fit_iters,
                      const float *view_dirs, v3dg_bundle **out);

/* Sizes of a built bundle: clusters, rows, leaf clusters (ids 0 .. n_leaf-1)
 * and layers. */
int v3dg_bundle_sizes(const v3dg_bundle *b, uint32_t *n_clusters, uint32_t *n_rows, uint32_t *n_leaf_clusters,
                      uint32_t *n_layers);

/* Copy a built bundle into caller arrays sized by v3dg_bundle_sizes (any may
 * be NULL): rows as in v3dg_hierarchy_desc, clusters likewise plus level[k];
 * src[i] is the input Gaussian row i descends from and gen[i] the
 * simplifications it went through (in a structural build its scales are the
 * input's grown gen[i] times, the rest of it a copy). */
int v3dg_bundle_copy(const v3dg_bundle *b, float *pos, float *scale, float *rot, float *opacity, float *sh,
                     float *self_sphere, float *parent_sphere, uint32_t *first_row, uint8_t *count, uint8_t *level,
                     int32_t *parent, int32_t *first_child, uint8_t *n_children, uint32_t *src, uint8_t *gen);

/* Mean local-splatting loss of a built bundle: loss[(l - 1) * fit_iters + i]
 * is the mean over the groups that made layer l (1 .. n_layers - 1) of their
 * loss at view i, before its step; (n_layers - 1) x fit_iters floats, none
 * when fit_iters = 0. */
int v3dg_bundle_fit_loss(const v3dg_bundle *b, float *loss);

void v3dg_bundle_free(v3dg_bundle *b);

/* Local splatting of cluster groups (paper Sec. 3.2), on the GPU.  Group g
 * fits its simplified ("fitted") Gaussians, rows fit_first[g] .. +
 * fit_count[g] - 1 (at most 64), to its original Gaussians, rows orig_first[g]
 * .. + orig_count[g] - 1 (at most 128): for view i < iters, both sets are
 * splatted at 64 x 64 from c + 4 r d_i towards the centre c of sphere[g] =
 * (cx, cy, cz, r > 0), with d_i = view_dirs[3i .. 3i+2] (normalised here; up
 * = +z unless |d_z| > 0.99, then +y; focal 32 / tan(asin(1/4))).  Splatting
 * is the renderer's (no dilation, alpha = min(0.99, o e^power), skip below
 * 1/255, stop before T < 1e-4, background 0) with colour max(0, C0 dc + 0.5)
 * from the degree-0 SH term dc.  Loss: mean |rgb - target| + 0.1 mean |alpha -
 * target alpha|; one Adam step (0.9, 0.999, eps 1e-15) per view on position,
 * log scale, quaternion, logit opacity and dc with learning rates 1.6e-5 (the
 * paper's), 5e-3, 1e-3, 5e-2, 2.5e-3.  Rows are host arrays: pos, scale (x 3),
 * rot (x 4, w x y z), opacity, dc (x 3); the fitted rows are updated in place
 * (quaternions returned unit).  losses (n_groups x iters, before each step)
 * and grad_first (14 per fitted row: the gradients of the first view) may be
 * NULL.  Synchronises.  Errors: V3DG_ERR_INVALID_ARG, V3DG_ERR_OOM,
 * V3DG_ERR_HIP, V3DG_ERR_DEVICE. */
int v3dg_local_splat(uint32_t n_groups, const uint32_t *orig_first, const uint32_t *orig_count,
                     const uint32_t *fit_first, const uint32_t *fit_count, const float *sphere, const float *orig_pos,
                     const float *orig_scale, const float *orig_rot, const float *orig_opacity, const float *orig_dc,
                     uint32_t n_orig, float *fit_pos, float *fit_scale, float *fit_rot, float *fit_opacity,
                     float *fit_dc, uint32_t n_fit, const float *view_dirs, uint32_t iters, float *losses,
                     float *grad_first);

/* Message of the last failure on this thread ("" if none). */
const char *v3dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
