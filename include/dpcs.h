/*
 * dpcs.h -- C ABI of the MI355X (gfx950) DPCS project-and-capture renderer.
 *
 * The library renders the camera image a projector-camera system captures when a
 * projector input image is projected onto a textured triangle-mesh surface, and the
 * vector-Jacobian product of that map (paper Sec. 3):
 *
 *   forward rendering   I_c = R(I_p, theta)                       (Eq. 7)
 *   inverse rendering   {I_p, theta} = R^-1(I_c) by gradients      (Eq. 8, 9, 13)
 *   training objective  L1 data term, map regulariser L(m), denoiser D (Eq. 9, 11)
 *
 * with the projector response E_p = g_p M I_p^gamma_p (Eq. 1; M = I gives Eq. 1
 * exactly), a pinhole projector emitter (Eq. 2, 6), multi-bounce Monte-Carlo light
 * transport with importance sampling (Eq. 3, 10), per-sample radiance clipping
 * min(L, k / min(w)) (Eq. 12), a box-filtered pixel mean (Eq. 4) and the camera
 * response I_c = (g_c w E_c)^gamma_c (Eq. 5).
 *
 * Conventions (every entry point):
 *  - Images and maps are float32, contiguous, row-major HWC (H rows, W columns,
 *    C channels); albedo H x W x 3, roughness and specular H x W.
 *  - Unless stated otherwise, pointers passed to render / VJP / server calls are
 *    DEVICE pointers on the context's device; the caller owns them and keeps them
 *    valid until the context's stream has passed the call.  Mesh inputs of
 *    dpcs_scene_create are HOST pointers and are copied.
 *  - Every render call is asynchronous on the context's HIP stream; nothing syncs
 *    the host except dpcs_scene_create, dpcs_context_synchronize and the server.
 *    Inside a call, large waves run their shadow rays on a second stream the context
 *    owns (default priority, made on first use), forked from the context's stream and
 *    joined back into it by events within the same call: when the context's stream has
 *    passed a call, all of its work is done.
 *  - Argument checks happen before any launch and return DPCS_E_INVALID with a
 *    message for dpcs_last_error().  Device faults are sticky: the next call on the
 *    context returns DPCS_E_DEVICE.
 *  - Pinhole devices map a world point x to device coordinates R x + t (OpenCV axes,
 *    +z forward) and to pixel coordinates (K (R x + t)).xy / z; pixel (i, j) covers
 *    [i, i+1) x [j, j+1).
 */
#ifndef DPCS_H
#define DPCS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define DPCS_API __attribute__((visibility("default")))
#else
#define DPCS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DPCS_OK = 0,
    DPCS_E_INVALID = -1,      /* bad argument; nothing was launched */
    DPCS_E_OOM = -2,          /* scratch limit or device memory exhausted; outputs undefined */
    DPCS_E_DEVICE = -3,       /* a HIP call or kernel failed (sticky on the context) */
    DPCS_E_UNSUPPORTED = -4,  /* valid request the library cannot serve (e.g. BVH too deep) */
    DPCS_E_BUSY = -5,         /* object still referenced by queued work */
    DPCS_E_REJECTED = -6      /* server: the request can never fit the memory budget */
} dpcs_status;

enum { DPCS_BRDF_LAMBERT = 0, DPCS_BRDF_GGX = 1 };

typedef struct dpcs_context_s* dpcs_context;
typedef struct dpcs_scene_s* dpcs_scene;
typedef struct dpcs_server_s* dpcs_server;

/* ---------------------------------------------------------------- context */

/* One device, one HIP stream (hip_stream may be NULL: the null stream) and a scratch
 * pool that grows up to scratch_limit_bytes (0: no limit). */
DPCS_API dpcs_status dpcs_context_create(int32_t device, void* hip_stream, size_t scratch_limit_bytes,
                                dpcs_context* out);
DPCS_API void dpcs_context_destroy(dpcs_context ctx);
/* Text of the last error on ctx (valid until the next call on ctx); "" if none. */
DPCS_API const char* dpcs_last_error(dpcs_context ctx);
/* Waits for the context's stream; reports DPCS_E_DEVICE if queued work failed. */
DPCS_API dpcs_status dpcs_context_synchronize(dpcs_context ctx);
/* Samples per launch wave (in-flight path capacity, >= 1).  Results do not depend on it. */
DPCS_API dpcs_status dpcs_context_set_capacity(dpcs_context ctx, int64_t paths);

/* ------------------------------------------------------------------ scene */

/* Triangle mesh of the projection surface (paper Sec. 3.1: the surface x_s the
 * projector lights and the camera sees).  HOST pointers, copied. */
typedef struct {
    const float* positions;     /* num_vertices x 3 */
    int32_t num_vertices;
    const int32_t* triangles;   /* num_triangles x 3 vertex indices */
    int32_t num_triangles;
    const float* corner_uvs;    /* num_triangles x 3 x 2 texture coordinates */
    const float* emission;      /* NULL, or num_triangles x 3 surface radiance (test scenes) */
    int32_t bvh_kind;           /* DPCS_BVH_LBVH (0): radix tree over Morton codes;
                                   DPCS_BVH_SAH (1): top-down binned SAH (32 bins, the
                                   fewest node visits per ray);
                                   DPCS_BVH_PLOC (2): locally-ordered clustering over the
                                   Morton order (between the two).  All are built on the
                                   device and collapsed there to the 4-wide traversal
                                   tree; DPCS_E_UNSUPPORTED for a tree deeper than 64. */
} dpcs_mesh_desc;

enum { DPCS_BVH_LBVH = 0, DPCS_BVH_SAH = 1, DPCS_BVH_PLOC = 2 };

typedef struct {
    int32_t num_triangles;
    int32_t num_nodes;          /* binary BVH internal nodes */
    int32_t max_depth;          /* deepest leaf */
    int32_t wide_nodes;         /* nodes of the 4-wide BVH the renderer traverses (0: binary) */
    int64_t device_bytes;       /* resident bytes (BVH + triangle records + attributes) */
    double build_ms;            /* wall time of the device build (sort, hierarchy, leaf
                                   records, 4-wide collapse and checks), uploads excluded */
    float bbox_lo[3], bbox_hi[3];
    float tmin;                 /* ray epsilon: 1e-5 x bounding-box diagonal */
} dpcs_scene_info;

/* Uploads the mesh and builds its BVH on the device (Morton codes, radix sort, then the
 * binary radix tree with bottom-up bounds or clustering, then the 4-wide collapse); the
 * tree never leaves the device.  Synchronises the context's stream. */
DPCS_API dpcs_status dpcs_scene_create(dpcs_context ctx, const dpcs_mesh_desc* mesh, dpcs_scene* out);
DPCS_API dpcs_status dpcs_scene_get_info(dpcs_scene s, dpcs_scene_info* out);
/* Frees the scene after the context's stream has drained; DPCS_E_BUSY while a server
 * still holds requests on it. */
DPCS_API dpcs_status dpcs_scene_destroy(dpcs_scene s);
/* Moves the scene's vertices (Sec. 4.4: editing the mesh simulates projection on a moving
 * surface, and compensation for it, frame by frame).  positions: DEVICE pointer,
 * num_vertices x 3 float32, same triangles and texture coordinates.  The BVH keeps its
 * topology: its boxes are refitted bottom-up on the device (binary and 4-wide) and the
 * leaf records rewritten, asynchronously on the context's stream, with no host copy.
 * The ray epsilon and the reported bounds stay those of creation; traversal slows as
 * the shape departs from the one the tree was built for (create a new scene for large
 * changes).  Non-finite positions are the caller's to avoid.  DPCS_E_BUSY while a
 * server holds requests on the scene. */
DPCS_API dpcs_status dpcs_scene_refit(dpcs_context ctx, dpcs_scene s, const float* positions);

/* ----------------------------------------------------------------- render */

typedef struct {
    double K[9];                /* intrinsics, row-major */
    double R[9];                /* world -> device rotation, row-major */
    double t[3];                /* world -> device translation */
    int32_t width, height;
} dpcs_pinhole;

/* Scalar parameters of theta that the VJP differentiates, in this order. */
enum { DPCS_NUM_SCALARS = 18 };  /* gamma_p[3], M[9] row-major, gamma_c[3], w[3] */

typedef struct {
    dpcs_pinhole camera, projector;       /* Eq. 6 */
    int32_t brdf;                         /* DPCS_BRDF_LAMBERT or DPCS_BRDF_GGX */
    const float* albedo;                  /* tex_h x tex_w x 3 (device) */
    const float* roughness;               /* tex_h x tex_w (device; GGX only, else may be NULL) */
    const float* specular;                /* tex_h x tex_w (device; GGX only, else may be NULL) */
    int32_t tex_w, tex_h;
    float prf_gamma[3];                   /* gamma_p (Eq. 1) */
    float prf_gain;                       /* g_p (Eq. 1; folds phi of Eq. 2) */
    float prf_mix[9];                     /* M, row-major; identity for Eq. 1 */
    float crf_gamma[3];                   /* gamma_c (Eq. 5) */
    float crf_gain;                       /* g_c (Eq. 5) */
    float white_balance[3];               /* w (Eq. 5, Eq. 12) */
    const float* device_scalars;          /* NULL, or device[18] overriding the five fields
                                             gamma_p, M, gamma_c, w above (same order) */
    float env_radiance[3];                /* constant environment radiance (0: dark room) */
    int32_t clip_enable;                  /* Eq. 12 on/off */
    float clip_k;                         /* k of Eq. 12 */
    int32_t spp;                          /* camera samples per pixel, >= 1 */
    int32_t max_depth;                    /* surface vertices per path, 1..64 (1: direct only) */
    uint64_t seed;                        /* Philox key */
    uint32_t sample_offset;               /* added to the sample index of every counter */
    /* The principled BRDF's further maps (Sec. 3.2: theta holds the BRDF maps and the
     * normal map v_n; Sec. 4.3: base colour, roughness, metallic, normal map), tex_h x
     * tex_w, both optional:
     *   metallic    (GGX only; NULL: 0) blends the dielectric specular colour 0.08 x
     *               specular into the base colour, F0 = (1 - mu) 0.08 sp + mu a, and
     *               scales the diffuse lobe by (1 - mu);
     *   normal_map  (x 3, NULL: none) values v in [0, 1] decode to t = 2 v - 1 in the
     *               tangent frame T = dP/du (the triangle's texture parameterisation,
     *               orthogonal to the two-sided geometric normal n), B = n x T, and tilt
     *               the shading normal to ns = (t_x T + t_y B + t_z n) / |t|; (0.5, 0.5, 1)
     *               changes nothing.  The BRDF, the rendering equation's cosine and the
     *               sampled directions are taken about ns; a direction counts only above
     *               both ns and the geometric surface.
     * With either map dpcs_render_vjp needs path records (its own or the caller's): the
     * re-tracing mode and the request loop return DPCS_E_UNSUPPORTED. */
    const float* metallic;
    const float* normal_map;
} dpcs_render_params;

/* Optional per-call outputs of dpcs_render (any field may be NULL). */
typedef struct {
    float* linear;              /* Hc x Wc x 3: E_c before the CRF */
    float* sample_radiance;     /* Hc x Wc x spp x 3: unclipped radiance of every camera sample */
    int32_t* hit_prims;         /* Hc x Wc x spp x max_depth: triangle hit per vertex,
                                   -1 escaped, -2 path ended earlier */
    uint32_t* path_records;     /* Hc x Wc x spp x max_depth: opaque replay records for
                                   dpcs_render_vjp (which leaf each vertex hit, which of its
                                   shadow rays were unoccluded); words past a path's end are
                                   left as they were.  4 bytes per (sample, depth).  Setting
                                   it makes the forward trace shadow rays whose contribution
                                   is zero too (their visibility carries gradient). */
} dpcs_render_aux;

/* I_c = R(I_p, theta) (Eq. 7).  proj_image: Hp x Wp x 3, out_image: Hc x Wc x 3. */
DPCS_API dpcs_status dpcs_render(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                        const float* proj_image, float* out_image, const dpcs_render_aux* aux);

/* dpcs_render for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, same
 * checks and the same results bit for bit (the same samples, summed in the same order);
 * the call itself allocates nothing: E_p, the packed maps and the launch wave's queues
 * (with the traversal's stack spill space) are carved from a static device array of
 * DPCS_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds from context
 * creation until the process ends, and each wave holds as many paths as fit (at most
 * the context's capacity).  Profiling is suspended during the call.
 * Limit: 16 bytes per projector pixel + 16 bytes per map texel (32 with the metallic or
 * normal map) + 508 bytes per camera sample of one pixel must fit in the array, else
 * DPCS_E_INVALID before any launch.
 * Every call on a device shares that device's array and leaves its contents there (all
 * of it is written before it is read, nothing has to start at zero): calls on one device
 * whose work overlaps on the GPU (different streams, e.g. two contexts) race; order them
 * on one stream or synchronise between them.  DPCS_E_DEVICE if the array's address could
 * not be looked up when the context was created. */
enum { DPCS_NOALLOC_SCRATCH_BYTES = 64 << 20 };
DPCS_API dpcs_status dpcs_render_noalloc(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                         const float* proj_image, float* out_image, const dpcs_render_aux* aux);

/* Gradient buffers of dpcs_render_vjp (device pointers, OVERWRITTEN, any may be NULL). */
typedef struct {
    float* d_proj_image;        /* Hp x Wp x 3 */
    float* d_albedo;            /* tex_h x tex_w x 3 */
    float* d_roughness;         /* tex_h x tex_w */
    float* d_specular;          /* tex_h x tex_w */
    float* d_scalars;           /* DPCS_NUM_SCALARS, layout of device_scalars */
    float* d_metallic;          /* tex_h x tex_w (needs params->metallic) */
    float* d_normal_map;        /* tex_h x tex_w x 3, of the stored values v (needs params->normal_map) */
    float* d_camera;            /* 12: d/dR_c (row-major 3 x 3) then d/dt_c of the camera pose (Sec. 3.2:
                                   R_c, t_c refined with theta).  The interior part: per camera
                                   sample, the first vertex's radiance differentiated w.r.t. its hit
                                   point and viewing direction with every visibility decision, the
                                   sampled directions and the rest of the path held; plus, when
                                   camera_edge_density > 0, the boundary part below.  Needs path
                                   records: with sample_radiance alone DPCS_E_UNSUPPORTED; not in
                                   the server. */
    double camera_edge_density; /* boundary part of d_camera (0: none; needs d_camera; <= 1e6):
                                   points per pixel of image length on the images of the mesh edges
                                   where the first surface seen jumps (vertices of triangles at one
                                   position are one vertex, faces of no area are left out, and
                                   overlapping edges of different vertices each count; edges of one
                                   face or of three or more,
                                   faces not coplanar -- creases and all silhouettes --, faces folded
                                   flat, texture-coordinate and emission seams), clipped to the
                                   image and in front of the camera.  Each point adds (f- - f+) times
                                   the edge's normal speed in the image times its share of the
                                   edge's length, f-/+ the clipped radiance of two paths 0.01 pixel
                                   to either side that share the point's random numbers (their own
                                   key: seed XOR 0x9E3779B97F4A7C15), weighted by its pixel's
                                   cotangent.  Shadow and projector-frustum boundaries on surfaces
                                   are not included.  The edge table is built on the host on first
                                   use and after each refit; DPCS_E_UNSUPPORTED above 2^32 points. */
} dpcs_grads;

/* Vector-Jacobian product of dpcs_render at the same params (same seed: the same
 * sample paths are replayed): given grad_image = dLoss/dI_c (Hc x Wc x 3), writes
 * dLoss/d{I_p, albedo, roughness, specular, gamma_p, M, gamma_c, w} (Eq. 9, 13).
 * sample_radiance and path_records (optional) are aux outputs of a forward call with
 * the same scene, params and proj_image:
 *   both NULL           the forward samples and their path records are recomputed
 *                       here, wave by wave (scratch: 4 B x spp x max_depth per pixel
 *                       of a wave), then replayed without tracing;
 *   both given          replay from the caller's records, no tracing;
 *   sample_radiance     replay that traces every bounce and shadow ray again.
 *   only
 * path_records without sample_radiance is DPCS_E_INVALID.
 * The same inputs give the same gradient bits on every call (map cotangents are summed
 * in exact fixed point, scalar sums in a fixed order); maps larger than 1024 x 1024 fall
 * back to float atomics, whose summation order varies. */
DPCS_API dpcs_status dpcs_render_vjp(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                            const float* proj_image, const float* grad_image,
                            const float* sample_radiance, const uint32_t* path_records,
                            const dpcs_grads* grads);

/* -------------------------------------------------- training objective */

/* Eq. 9 fits theta by minimising the mean L1 distance between denoised renderings and
 * captures plus lambda_reg L(m); Eq. 11 denoises the rendering with a cross-bilateral
 * filter D first.  The paper fixes neither D's window and weights nor L's formula; the
 * library's readings are stated with each call.  All buffers below are DEVICE pointers
 * owned by the caller; every call is asynchronous on the context's stream. */

enum { DPCS_DENOISE_MAX_GUIDE = 8, DPCS_DENOISE_MAX_RADIUS = 8 };

typedef struct {
    int32_t width, height;      /* image size, 1..16384 each */
    int32_t guide_channels;     /* G, 0..DPCS_DENOISE_MAX_GUIDE */
    int32_t radius;             /* r: the window is (2r+1) x (2r+1), 0..DPCS_DENOISE_MAX_RADIUS */
    float spatial;              /* a_s = 1 / (2 sigma_s^2) in 1/pixel^2, >= 0 */
    float guide[DPCS_DENOISE_MAX_GUIDE]; /* a_k = 1 / (2 sigma_k^2) per guide channel, >= 0 */
} dpcs_denoise_params;

/* D of Eq. 11 on an H x W x 3 image steered by an H x W x G guide (G = 0: guide may be
 * NULL):  out_p = sum_q w(p,q) image_q / sum_q w(p,q) over the window around p clipped
 * to the image, w(p,q) = exp(-a_s |p - q|^2 - sum_k a_k (guide_k(p) - guide_k(q))^2).
 * The centre weight is 1, so the sum never vanishes.  Guide values must be finite.
 * out must not overlap image.  FP32 arithmetic. */
DPCS_API dpcs_status dpcs_denoise(dpcs_context ctx, const dpcs_denoise_params* p, const float* image,
                                  const float* guide, float* out);
/* VJP of dpcs_denoise with the same p and guide (the guide is a constant of D, so D is
 * linear): grad_image_q = sum_p w(p,q) grad_out_p / sum_q' w(p,q'), OVERWRITTEN.
 * Uses an H x W x 4 float scratch buffer of the context.  grad_image must not overlap
 * grad_out. */
DPCS_API dpcs_status dpcs_denoise_vjp(dpcs_context ctx, const dpcs_denoise_params* p, const float* grad_out,
                                      const float* guide, float* grad_image);

/* Guide features for dpcs_denoise: one camera ray through the centre of each pixel
 * (Eq. 6 inverted, no jitter), closest hit on the scene.  gbuffer (Hc x Wc x 8 float):
 * albedo rgb at the hit (bilinear lookup of params->albedo), unit geometric normal
 * turned toward the camera (xyz), hit distance along the unit ray, 1; all eight are 0
 * where the ray escapes.  params must be valid as for dpcs_render (no projector image is
 * needed); the call uses its camera and BRDF maps.  gbuffer must be 16-byte aligned. */
DPCS_API dpcs_status dpcs_render_gbuffer(dpcs_context ctx, dpcs_scene scene, const dpcs_render_params* params,
                                         float* gbuffer);

/* L(m) of Eq. 9 for one h x w x c map (c = 1 for roughness or specular, 3 for albedo),
 * read as the anisotropic L1 total variation:  mean |m(y+1,x) - m(y,x)| over the
 * c (h-1) w vertical pairs plus mean |m(y,x+1) - m(y,x)| over the c h (w-1) horizontal
 * pairs (a direction without pairs adds 0).  Sums in FP64 in a fixed order (the result
 * does not vary between runs); loss (device, 1 float) is written.  h, w, c >= 1,
 * h w c < 2^31. */
DPCS_API dpcs_status dpcs_tv_loss(dpcs_context ctx, const float* map, int32_t h, int32_t w, int32_t c,
                                  float* loss);
/* grad_map = grad_loss[0] * dL/dm (h x w x c, OVERWRITTEN), with d|x|/dx = sign(x) and
 * sign(0) = 0; grad_loss is a device scalar (the loss's cotangent). */
DPCS_API dpcs_status dpcs_tv_vjp(dpcs_context ctx, const float* map, int32_t h, int32_t w, int32_t c,
                                 const float* grad_loss, float* grad_map);

/* Data term of Eq. 9 for one image pair: loss = mean |a - b| over n values (FP64 sums
 * in a fixed order; 1 float written).  1 <= n < 2^31. */
DPCS_API dpcs_status dpcs_l1_loss(dpcs_context ctx, const float* a, const float* b, int64_t n, float* loss);
/* grad_a = grad_loss[0] * sign(a - b) / n (OVERWRITTEN; sign(0) = 0). */
DPCS_API dpcs_status dpcs_l1_vjp(dpcs_context ctx, const float* a, const float* b, int64_t n,
                                 const float* grad_loss, float* grad_a);

/* ------------------------------------------------------------ debug/test */

/* Hits of n rays (device: rays n x 8 = o.xyz, d.xyz, tmax, skip prim as float).
 * use_bvh: 0 closest hit by brute force over all triangles, 1 closest hit through the
 * BVH the renderer traverses (4-wide when built), 2 closest hit through the binary
 * BVH, 3 any hit (shadow query) through the renderer's BVH, 4 any hit by brute force.
 * Output device arrays: prim (n, -1 on a miss), t/b1/b2 (n each; may be NULL). */
DPCS_API dpcs_status dpcs_debug_intersect(dpcs_context ctx, dpcs_scene scene, const float* rays, int64_t n,
                                 int32_t use_bvh, int32_t* prim, float* t, float* b1, float* b2);
/* Philox4x32-10 of n counters (device: ctr n x 4, out n x 4). */
DPCS_API dpcs_status dpcs_debug_philox(dpcs_context ctx, uint64_t seed, const uint32_t* ctr, int64_t n,
                              uint32_t* out);
/* The surface reflectance f_r of the rendering equation (Sec. 3.2, Eq. 3) as this
 * library models it (brdf: DPCS_BRDF_LAMBERT, or Lambert + GGX microfacet lobe), its
 * derivatives, and the bounce sampler with its density, evaluated by the same device
 * code the renderer and the VJP use, for n rows of FP64 input.
 * in  (device, n x 17): normal xyz, outgoing direction xyz, incoming direction xyz (all
 *     unit), albedo rgb, roughness, specular, sampler numbers (lobe, u1, u2) in [0, 1).
 * out (device, n x 11): f rgb, d(specular term)/d roughness, d(specular term)/d specular,
 *     density of sampling the incoming direction, a direction sampled from the three
 *     numbers (xyz) and its density, and f.r as the forward (non-derivative) evaluation
 *     computes it.  The caller owns both buffers; DPCS_E_INVALID on a bad kind or null
 *     pointer with n > 0. */
DPCS_API dpcs_status dpcs_debug_brdf(dpcs_context ctx, int32_t brdf, const double* in, int64_t n, double* out);

/* -------------------------------------------------------------- profiling */

/* Per-stage kernel timing for benchmarks.  mode 0: off.  mode 1: every launch of a
 * stage is bracketed by HIP events on the context's stream and its work-item count
 * (queue size) is copied to pinned host memory.  mode 2: as 1, and the traversal
 * kernels also count visited BVH nodes and tested triangles (slower; use it to measure
 * the traversal byte model, not to time).  Enabling or disabling clears the record. */
enum {
    DPCS_STAGE_RAYGEN = 0, DPCS_STAGE_TRACE = 1, DPCS_STAGE_SHADE = 2, DPCS_STAGE_SHADOW = 3,
    DPCS_STAGE_FINALIZE = 4, DPCS_STAGE_ADJ_PIXEL = 5, DPCS_STAGE_ADJ_SHADE = 6, DPCS_STAGE_ADJ_SHADOW = 7,
    DPCS_STAGE_OTHER = 8, DPCS_NUM_STAGES = 9
};
typedef struct {
    int64_t launches[DPCS_NUM_STAGES];
    double ms[DPCS_NUM_STAGES];        /* sum of event-measured launch durations */
    int64_t items[DPCS_NUM_STAGES];    /* rays / paths / pixels processed */
    int64_t nodes[DPCS_NUM_STAGES];    /* mode 2: BVH nodes visited (TRACE, SHADOW, ADJ_SHADOW) */
    int64_t tris[DPCS_NUM_STAGES];     /* mode 2: triangles tested */
} dpcs_profile;
DPCS_API dpcs_status dpcs_context_set_profiling(dpcs_context ctx, int32_t mode);
/* Synchronises the stream, returns the totals since profiling was enabled and clears them. */
DPCS_API dpcs_status dpcs_context_get_profile(dpcs_context ctx, dpcs_profile* out);

/* ----------------------------------------------------------------- server */

/* Continuous-batching request loop on ctx's device: requests are admitted while the
 * device-memory estimate of all admitted requests stays within memory_budget_bytes and
 * fewer than max_slots are active; every launch wave mixes camera samples of all active
 * requests in shared path queues. */
DPCS_API dpcs_status dpcs_server_create(dpcs_context ctx, size_t memory_budget_bytes, int32_t max_slots,
                               dpcs_server* out);

typedef struct {
    dpcs_scene scene;
    dpcs_render_params params;  /* copied at submit; device pointers must stay valid */
    const float* proj_image;    /* Hp x Wp x 3 */
    float* out_image;           /* Hc x Wc x 3 */
    /* compensation step (fwd + VJP), when grads != NULL: the cotangent is grad_image, or,
       if grad_image is NULL and target is not, the gradient of the L2 loss
       sum((I_c - target)^2) / (Hc Wc 3) */
    const float* grad_image;
    const float* target;
    const dpcs_grads* grads;
    uint64_t request_id;
    void* input_stream;         /* HIP stream on which the caller produced the request's inputs
                                   (projector image, maps, device scalars, target or cotangent);
                                   NULL: the context's stream.  The request's first launch waits
                                   for all work queued on it before the submit call. */
} dpcs_request;

/* Non-blocking.  DPCS_E_REJECTED if the request alone exceeds the budget.  Waves hold
 * at most 2^21 paths, so a newcomer waits for short waves only. */
DPCS_API dpcs_status dpcs_server_submit(dpcs_server srv, const dpcs_request* req);
/* Non-blocking: up to max finished requests (ids, statuses, latency in ms from submit
 * to completion on the device; latency_ms may be NULL).  Returns the count. */
DPCS_API int32_t dpcs_server_poll(dpcs_server srv, uint64_t* done_ids, int32_t* done_status, double* latency_ms,
                         int32_t max);
/* Counters (out: 14 int64 on the host): [0] submitted, [1] completed, [2] rejected,
 * [3] active, [4] queued, [5] launch waves, [6] samples traced, [7] peak admitted bytes,
 * [8] waves whose compensation segments replayed path records, [9] waves whose
 * compensation segments re-traced (their paths did not fit the wave's records), the
 * latency of the completed requests summed in microseconds, in three parts: [10] submit
 * to admission (queued for memory or a slot), [11] admission to the launch of the
 * request's first wave, [12] from there to completion on the device; [13] waves whose
 * compensation paths, all of one request, binned their map cotangents (sorted by tile,
 * summed in fixed point) instead of scattering them with atomics. */
DPCS_API dpcs_status dpcs_server_stats(dpcs_server srv, int64_t* out14);
/* Waits for every admitted request, then stops the loop. */
DPCS_API dpcs_status dpcs_server_destroy(dpcs_server srv);

#ifdef __cplusplus
}
#endif

#endif /* DPCS_H */
