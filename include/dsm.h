/*
 * dsm.h -- C ABI of the MI355X (gfx950) library for differentiable
 * pre-filtered shadow mapping (Worchel & Alexa, "Differentiable Shadow
 * Mapping for Efficient Inverse Graphics", CVPR 2023).
 *
 * The library renders Lambert-shaded images whose shadows come from
 * variance shadow maps (Sec. 3: moments of a filtered shadow map and the
 * one-sided Chebyshev bound; Alg. 1 RenderShadowMap, Alg. 2
 * ComputeVisibility) and computes the reverse-mode gradient of a loss on
 * those images with respect to vertex positions, light parameters and
 * albedo (Sec. 4, derivatives of the moments and of the visibility).
 * Borders of primitives are antialiased in both the light and the camera
 * view; that smoothing is what carries gradients across silhouettes and
 * shadow borders (Sec. 4; Sec. 5, optimization without smoothed shadow map).
 *
 * Conventions for every call:
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors); every other pointer is host memory read during the call only.
 *  - Arrays are dense row-major, float32 unless stated; vertices [V,3],
 *    faces [F,3] int32 with scene-local vertex indices, images [H,W,C].
 *  - All device work is enqueued on `stream` (a hipStream_t; NULL = the
 *    default stream).  Calls return once the work is enqueued; outputs are
 *    valid after the stream reaches that point.  A plan must not be used
 *    from two streams at once: every forward and backward rewrites the
 *    plan's per-view constants (the light cameras) on the device.
 *  - Every call returns a dsm_status.  Arguments are validated on the host
 *    before anything is enqueued; on an error nothing is enqueued and
 *    outputs are left untouched.  No exception or abort crosses the ABI.
 *  - Gradient outputs are overwritten, never accumulated.
 *  - Thread safety: distinct plans may be used from distinct host threads.
 */
#ifndef DSM_H
#define DSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSM_ABI_VERSION 2

typedef enum {
    DSM_OK = 0,
    DSM_ERR_INVALID_ARG = 1,          /* a null pointer, size or index out of range       */
    DSM_ERR_OUT_OF_MEMORY = 2,        /* plan-owned device memory could not be allocated  */
    DSM_ERR_WORKSPACE_TOO_SMALL = 3,  /* caller workspace smaller than the plan requires  */
    DSM_ERR_UNSUPPORTED = 4,          /* valid request this build does not implement      */
    DSM_ERR_NO_DEVICE = 5,            /* no HIP device                                    */
    DSM_ERR_HIP = 6,                  /* a HIP runtime call failed                         */
    DSM_ERR_DEVICE_FAULT = 7          /* device-side invariant violated (see dsm_get_stats) */
} dsm_status;

enum { DSM_LIGHT_DIRECTIONAL = 0, DSM_LIGHT_POINT = 1, DSM_LIGHT_SPOT = 2, DSM_LIGHT_CUBE_FACE = 3 };
enum { DSM_FILTER_BOX = 0, DSM_FILTER_GAUSSIAN = 1 };

/* Limits checked by every entry point. */
#define DSM_MAX_RESOLUTION 8192      /* shadow-map side and camera width/height        */
#define DSM_MAX_KERNEL 31            /* odd filter size k, 1 <= k <= 31, and k <= S    */
#define DSM_MAX_LIGHTS_PER_RENDER 16

typedef void *dsm_stream;            /* hipStream_t */
typedef struct dsm_plan dsm_plan;

/*
 * One light and its shadow map (Sec. 3 light model; one map per light,
 * Sec. 5).  The light camera is built on the device from the differentiable
 * light parameter (position for point/spot lights, travel direction for
 * directional lights) passed to dsm_forward:
 *   directional: orthographic, eye = -dir_distance * w (w = unit travel
 *                direction) looking at the origin, half-extent ortho_half;
 *                distance d(x) = (x - eye) . w, a plane outside the scene;
 *   point, spot: perspective at the position looking at `target`, vertical
 *                field of view fov_deg, aspect 1; d(x) = |x - position|.
 *                A spot light lights only the cone of half-angle fov_deg/2
 *                around its axis (hard mask, no gradient through it).
 *   cube face:   one of the six faces of an omnidirectional point light's
 *                cube shadow map (Sec. 3: rays parameterized over several
 *                planes arranged as a box; Sec. 5: omnidirectional lights
 *                by several shadow maps).  Face f = cube_face in 0..5
 *                looks along +x, -x, +y, -y, +z, -z from the position
 *                through a square 90 degree frustum (target, up and fov_deg
 *                are ignored; the library picks the face's up vector), and
 *                lights only the points x whose direction x - position has
 *                its largest |component| on the face's axis with the face's
 *                sign (ties go to the lower axis; hard mask, no gradient
 *                through it), so six faces with one position light every
 *                direction exactly once.  Each face is a light of its own
 *                with its own map and parameter slot; the gradient for the
 *                shared position is the sum of the six.  The six faces of
 *                one cube light are consecutive lights with cube_face 0..5
 *                in order and equal scene, resolution, filter, k and sigma
 *                (else DSM_ERR_INVALID_ARG); their parameters should hold
 *                the same position.  Each face's map is padded with
 *                (k - 1) / 2 + 1 texels sampled from its neighbours across
 *                the cube's edges (bilinear, along the direction of each
 *                padded texel with the face's plane continued) before
 *                filtering, so the filter and the bilinear fetch continue
 *                across the seams.
 * Depths are stored as z = d / zfar.  `k` is the odd filter size of the
 * moment filter (box or Gaussian with std. dev. sigma in texels; sigma <= 0
 * means (k-1)/3).  min_variance floors sigma^2 = m2 - m1^2.
 *
 * Alternative pre-filtered maps (Sec. 3 lists pre-warps g(f) such as exp;
 * light bleeding, supplementary limitations):
 *   warp_exponent c > 0 stores exp(c z) and exp(2 c z) instead of z and z^2
 *   (background exp(c), exp(2c)); the lookup compares exp(c d / zfar) with
 *   the filtered first moment and floors sigma^2 at
 *   min_variance * (c exp(c d / zfar))^2.  0 <= c <= 40 (larger values
 *   overflow float32 in the floor); 0 keeps plain variance maps.
 *   bleed_reduction a in [0, 1) maps the visibility v to
 *   clamp((v - a) / (1 - a), 0, 1), cutting light bleeding where occluders
 *   at several depths share a filter window; 0 leaves v unchanged.
 */
typedef struct {
    int32_t type;          /* DSM_LIGHT_*                                   */
    int32_t scene;         /* scene index the light shadows                 */
    float target[3];       /* point/spot look-at target                     */
    float up[3];           /* up vector of the light camera                 */
    float fov_deg;         /* point/spot field of view (spot: cone angle)   */
    float dir_distance;    /* directional: eye distance from the origin     */
    float ortho_half;      /* directional: orthographic half-extent         */
    float znear, zfar;
    float intensity;
    int32_t resolution;    /* shadow-map side S                             */
    int32_t filter;        /* DSM_FILTER_*                                  */
    int32_t k;
    float sigma;
    float min_variance;
    int32_t antialias;     /* smooth the light view at primitive borders    */
    int32_t cube_face;     /* DSM_LIGHT_CUBE_FACE: face 0..5; else ignored  */
    float warp_exponent;   /* exponential maps: c in [0, 40]; 0 = plain     */
    float bleed_reduction; /* light-bleeding reduction amount in [0, 1)     */
} dsm_light_desc;

/* A perspective viewer camera (fixed; no gradient). */
typedef struct {
    float eye[3], target[3], up[3];
    float fov_deg;         /* vertical field of view, aspect = width/height */
    float znear, zfar;
    int32_t width, height;
    int32_t scene;
} dsm_camera_desc;

/* One rendered image: a camera and a set of lights whose Lambert terms are
 * summed (deferred shading over any number of lights). */
typedef struct {
    int32_t camera;        /* index into cameras                           */
    int32_t light_begin;   /* range into render_light_list                 */
    int32_t light_count;
} dsm_render_desc;

/*
 * A batch: scenes of uneven size concatenated (CSR offsets), each with any
 * number of lights and cameras, and renders pairing them.  Everything here is
 * host memory, copied by dsm_plan_create.
 */
typedef struct {
    int32_t num_scenes;
    const int32_t *vert_offsets;       /* [num_scenes+1] into the vertex array        */
    const int32_t *face_offsets;       /* [num_scenes+1] into the face array          */
    const int32_t *faces;              /* [F_total,3] scene-local vertex indices      */
    const int32_t *pose_counts;        /* [num_scenes] or NULL: posed vertex prefix   */
    const float *pose_centers;         /* [num_scenes,3] or NULL                      */
    int32_t num_lights;
    const dsm_light_desc *lights;
    int32_t num_cameras;
    const dsm_camera_desc *cameras;
    int32_t num_renders;
    const dsm_render_desc *renders;
    const int32_t *render_light_list;  /* light indices referenced by the renders     */
    int32_t channels;                  /* 1 or 3 colour channels                      */
    int32_t camera_antialias;          /* smooth the shaded images at borders         */
} dsm_batch_desc;

/* Sizes a caller needs, filled by dsm_plan_info. */
typedef struct {
    int64_t total_vertices;
    int64_t total_faces;
    int64_t image_floats;        /* sum over renders of H*W*C                          */
    int64_t saved_bytes;         /* forward state kept for the backward pass (depth
                                    keys, triangle setup, maps, images before smoothing,
                                    the tile bins and the forward's counters)           */
    int64_t scratch_bytes;       /* temporaries of one forward or backward call; nothing
                                    in it outlives the call, so any scratch of this size
                                    serves any call                                     */
    int64_t map_floats;          /* sum over lights of 2*S*S                           */
    int32_t tile_size;           /* raster tile side in pixels                         */
    int32_t bin_capacity_scale;  /* bin capacity = scale * (triangles + tiles) / 4     */
    int64_t forward_scratch_bytes; /* the part of scratch a forward pass uses (at most
                                    scratch_bytes); dsm_forward_static_scratch needs it
                                    to be at most DSM_STATIC_SCRATCH_BYTES              */
} dsm_plan_info;

/* Counters of a forward pass, kept in its saved buffer (read back on demand). */
typedef struct {
    uint64_t culled_triangles;   /* dropped by the w > 0 / near / guard-band tests     */
    uint64_t binned_pairs;       /* (triangle, tile) pairs requested                    */
    uint64_t overflow_triangles; /* rasterized by the overflow path (bins full)         */
    uint64_t bad_indices;        /* faces referencing vertices outside their scene      */
} dsm_stats;

const char *dsm_version(void);
const char *dsm_status_string(dsm_status status);

/*
 * Build a plan for a batch: validates the description, uploads faces, builds
 * the edge adjacency used for silhouette tests, lays out every buffer.
 * tile_size: raster tile side (8, 16 or 32; 0 = library default 8);
 * bin_capacity_scale: the tile bins hold bin_capacity_scale * (triangles +
 * tiles) / 4 (triangle, tile) pairs over all views (1..1024; 0 = default 32).
 * Triangles whose pairs do not fit are rasterized by a slower overflow path
 * with identical results.
 * The plan owns only mesh-static device data (faces, adjacency, layout),
 * allocated on the HIP device current at this call; later calls with the
 * plan run with that device current.
 */
dsm_status dsm_plan_create(const dsm_batch_desc *desc, int32_t tile_size, int32_t bin_capacity_scale,
                           dsm_plan **out_plan);
dsm_status dsm_plan_info_get(const dsm_plan *plan, dsm_plan_info *out);
void dsm_plan_destroy(dsm_plan *plan);

/*
 * Forward pass (Alg. 1 for every light, then Alg. 2 and Lambert shading for
 * every render).
 *   verts_dev        [V_total,3] world-space vertex positions
 *   light_params_dev [L,3] position (point/spot) or travel direction (dir.)
 *   albedo_dev       [F_total,C] per-face albedo
 *   saved_dev        saved_bytes of caller memory, written here, read by
 *                    dsm_backward (keep it alive and unmodified in between)
 *   scratch_dev      scratch_bytes of caller memory, used only during this
 *                    call (its contents on return are unspecified)
 *   images_dev       [image_floats]: render r's [H,W,C] image at the offset
 *                    sum_{r'<r} H W C
 */
dsm_status dsm_forward(dsm_plan *plan, const float *verts_dev, const float *light_params_dev,
                       const float *albedo_dev, void *saved_dev, size_t saved_bytes,
                       void *scratch_dev, size_t scratch_bytes, float *images_dev, dsm_stream stream);

/*
 * dsm_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc): the same
 * kernels and results, with the forward's temporaries in a library-owned
 * device array of DSM_STATIC_SCRATCH_BYTES per GPU (held from the library's
 * load until the process ends) instead of a caller scratch buffer.  The
 * caller still owns verts, light_params, albedo, saved and images, with the
 * meanings and layouts of dsm_forward; dsm_backward then takes any scratch
 * buffer of scratch_bytes, as after dsm_forward.  The call allocates nothing.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (two streams, two host threads) race: order them on one stream.
 * Errors: DSM_ERR_WORKSPACE_TOO_SMALL when the plan's forward_scratch_bytes
 * exceed DSM_STATIC_SCRATCH_BYTES or saved_bytes is below the plan's;
 * DSM_ERR_INVALID_ARG for null or misaligned buffers, or when the current
 * device is not the one the plan was created on; otherwise as dsm_forward.
 */
#define DSM_STATIC_SCRATCH_BYTES (64ull << 20)
dsm_status dsm_forward_static_scratch(dsm_plan *plan, const float *verts_dev, const float *light_params_dev,
                                      const float *albedo_dev, void *saved_dev, size_t saved_bytes,
                                      float *images_dev, dsm_stream stream);

/*
 * Reverse pass of dsm_forward for upstream image gradient grad_images_dev
 * (same layout as images).  Outputs (overwritten):
 *   grad_verts_dev        [V_total,3]
 *   grad_light_params_dev [L,3]
 *   grad_albedo_dev       [F_total,C] or NULL
 * verts/light_params/albedo/saved must be those of the matching forward;
 * scratch_dev is any scratch_bytes of caller memory (it need not be the
 * forward's: backward reads only what saved holds).
 */
dsm_status dsm_backward(dsm_plan *plan, const float *verts_dev, const float *light_params_dev,
                        const float *albedo_dev, const void *saved_dev, size_t saved_bytes,
                        void *scratch_dev, size_t scratch_bytes, const float *grad_images_dev,
                        float *grad_verts_dev, float *grad_light_params_dev, float *grad_albedo_dev,
                        dsm_stream stream);

/*
 * Rigid pose of the first pose_counts[s] vertices of each scene:
 * world = R(r) v + center + t, pose [num_scenes,6] = (axis-angle r, t).
 * Vertices past the prefix are copied unchanged.  pose_backward turns the
 * world-vertex gradient into [num_scenes,6] pose gradients (overwritten).
 */
dsm_status dsm_pose_forward(dsm_plan *plan, const float *local_verts_dev, const float *poses_dev,
                            float *world_verts_dev, dsm_stream stream);
dsm_status dsm_pose_backward(dsm_plan *plan, const float *local_verts_dev, const float *poses_dev,
                             const float *grad_world_dev, float *grad_poses_dev, dsm_stream stream);

/*
 * Capture one forward + backward (+ pose forward/backward when poses_dev is
 * not NULL) with the given pointers into a HIP graph owned by the plan, and
 * replay it with dsm_graph_launch.  Pointers must stay valid and unchanged
 * for as long as the graph is replayed; a new capture replaces the old one.
 */
dsm_status dsm_graph_capture(dsm_plan *plan, const float *local_verts_dev, const float *poses_dev,
                             float *verts_dev, const float *light_params_dev, const float *albedo_dev,
                             void *saved_dev, size_t saved_bytes, void *scratch_dev, size_t scratch_bytes,
                             float *images_dev, const float *grad_images_dev, float *grad_verts_dev,
                             float *grad_light_params_dev, float *grad_albedo_dev, float *grad_poses_dev,
                             dsm_stream stream);
dsm_status dsm_graph_launch(dsm_plan *plan, dsm_stream stream);

/*
 * Stage outputs of the last forward, copied out of `saved` (parity checks).
 *  dsm_get_view_keys: 64-bit depth|triangle keys of view v (lights first,
 *      then cameras; ~0 = background) -> [H,W] uint64.
 *  dsm_get_light_maps: which = 0 unsmoothed (z, z^2), 1 smoothed, 2 filtered
 *      moments (m1, m2) -> [2,S,S], of z = d / zfar (exponential maps:
 *      exp(c z), exp(2 c z)).  Internally the maps hold the same quantities
 *      of z - zc, zc a per-light reference depth (the depth of the light's
 *      look-at point; 0 for cube faces) kept in saved, which leaves
 *      m2 - m1^2 and d - m1 unchanged and keeps more float32 digits of the
 *      variance; the getter converts back.  saved is needed for every
 *      `which`; which = 1 also needs scratch of the forward still intact
 *      (it is not part of the saved state).
 *  dsm_get_render_image0: shaded image of render r before border smoothing.
 */
dsm_status dsm_get_view_keys(const dsm_plan *plan, const void *saved_dev, int32_t view,
                             uint64_t *keys_dev, dsm_stream stream);
dsm_status dsm_get_light_maps(const dsm_plan *plan, const void *saved_dev, const void *scratch_dev,
                              int32_t light, int32_t which, float *out_dev, dsm_stream stream);
dsm_status dsm_get_render_image0(const dsm_plan *plan, const void *saved_dev, int32_t render,
                                 float *out_dev, dsm_stream stream);
/* Counters of the forward that wrote saved_dev; synchronizes `stream`. */
dsm_status dsm_get_stats(const dsm_plan *plan, const void *saved_dev, dsm_stats *out, dsm_stream stream);

/*
 * Moment filter on its own (Eq. moment1 and moment2: m = G f~ for both
 * channels): n_maps maps of 2 channels, [n_maps,2,S,S].  adjoint = 0 applies
 * G (horizontal then vertical pass, clamp-to-edge); adjoint = 1 applies G^T
 * (the transpose, with out-of-range taps folded onto the border texels).
 * in_dev and out_dev must not overlap.
 */
dsm_status dsm_filter_moments(int32_t S, int32_t n_maps, int32_t filter, int32_t k, float sigma,
                              const float *in_dev, float *out_dev, int32_t adjoint, dsm_stream stream);

/*
 * Stage timing (instrumentation, not part of the method).  The pipeline's
 * stages in launch order; a stage's time runs from its first launch to the
 * end of its last launch on the stream.
 */
typedef enum {
    DSM_STAGE_SETUP = 0,        /* zero fills, light frames, transform, triangle setup, silhouette masks */
    DSM_STAGE_BIN,              /* (triangle, tile) pair scan and tile binning */
    DSM_STAGE_RASTER,           /* tile raster of every light and camera view (a2-a3, a7) */
    DSM_STAGE_RESOLVE,          /* light-view moment resolve (z, z^2) */
    DSM_STAGE_LIGHT_AA,         /* light-view edge smoothing */
    DSM_STAGE_FILTER,           /* moment filter G (Alg. 1) */
    DSM_STAGE_LOOKUP,           /* Chebyshev visibility + Lambert shading (Alg. 2) */
    DSM_STAGE_CAMERA_AA,        /* camera-view edge smoothing */
    DSM_STAGE_BWD_SETUP,        /* zero fills, light frames */
    DSM_STAGE_CAMERA_AA_ADJ,    /* camera-view smoothing^T */
    DSM_STAGE_LOOKUP_ADJ,       /* lookup + shading^T, map-gradient scatter, per-(triangle, tile) sums */
    DSM_STAGE_FILTER_ADJ,       /* G^T */
    DSM_STAGE_LIGHT_ADJ,        /* light-view smoothing^T + resolve^T */
    DSM_STAGE_VERTEX_GRAD,      /* per-triangle reduction, vertex and albedo gathers */
    DSM_STAGE_LIGHT_GRAD,       /* light partial reduction and light-parameter chain */
    DSM_STAGE_COUNT
} dsm_stage;
#define DSM_MAX_TIMING_REPS 1000

/*
 * Runs dsm_forward + dsm_backward `reps` times on `stream` (arguments as
 * there) with a HIP event at the start and at the end of every stage, waits
 * for the stream, and writes each stage's mean duration in milliseconds to
 * ms_out (host, [DSM_STAGE_COUNT]).  flush_dev (nullable): flush_bytes of
 * device memory that the timer overwrites after every stage ends and before
 * the next starts (outside the timed intervals), so that each stage starts
 * with cold caches (give it more than the GPU's last-level cache, e.g.
 * 1 GiB); NULL times the stages back to back, each finding what the
 * previous one left in the caches.  `stream` must be a non-null stream that
 * is not being captured.  Outputs are those of the last repetition.  Errors:
 * DSM_ERR_INVALID_ARG for a null plan/ms_out/stream, reps outside
 * [1, DSM_MAX_TIMING_REPS], or a flush buffer that is misaligned or under 4
 * bytes; buffer errors as dsm_forward; DSM_ERR_HIP when an event cannot be
 * created, recorded or read.
 */
dsm_status dsm_time_stages(dsm_plan *plan, const float *verts_dev, const float *light_params_dev,
                           const float *albedo_dev, void *saved_dev, size_t saved_bytes, void *scratch_dev,
                           size_t scratch_bytes, float *images_dev, const float *grad_images_dev,
                           float *grad_verts_dev, float *grad_light_params_dev, float *grad_albedo_dev,
                           int32_t reps, void *flush_dev, size_t flush_bytes, float *ms_out, dsm_stream stream);

/*
 * Autotuner for the plan's tile side and bin depth (dsm_plan_create's
 * tile_size and bin_capacity_scale).  For every candidate (tile side 8, 16,
 * 32; bin capacity scale 8, 32) it builds a plan for `desc`, runs one
 * untimed and `reps` timed dsm_forward + dsm_backward passes on the given
 * inputs (same layouts as there; grad_images_dev has the plan's
 * image_floats) on `stream`, and returns the fastest choice in
 * *tile_size_out / *bin_capacity_scale_out and its mean milliseconds per
 * forward + backward in *ms_out (nullable).  The device work is timed with
 * HIP events; the call waits for `stream` and allocates and frees its own
 * device buffers.  cache_path (nullable) names a text file of earlier
 * decisions, one "key tile scale ms" line each, keyed by a hash of the
 * batch's shape (counts, mesh sizes, map and image sizes, filters) and the
 * device: a hit returns the stored choice without timing, a miss appends the
 * new one.  Errors: DSM_ERR_INVALID_ARG for null required pointers or reps
 * outside [1, DSM_MAX_TIMING_REPS], or a description dsm_plan_create
 * rejects; DSM_ERR_NO_DEVICE without a device; DSM_ERR_OUT_OF_MEMORY when
 * no candidate fits in device memory; DSM_ERR_HIP on a failed HIP call.
 */
dsm_status dsm_autotune(const dsm_batch_desc *desc, const float *verts_dev, const float *light_params_dev,
                        const float *albedo_dev, const float *grad_images_dev, int32_t reps,
                        const char *cache_path, dsm_stream stream, int32_t *tile_size_out,
                        int32_t *bin_capacity_scale_out, float *ms_out);

#ifdef __cplusplus
}
#endif
#endif /* DSM_H */
