/*
 * grtx.h -- C ABI of the MI355X (gfx950) Gaussian ray tracer.
 *
 * The library renders 3D Gaussian scenes by ray tracing (3DGRT pipeline, Sec. III-A:
 * build an acceleration structure over the Gaussians, generate rays, traverse, sort
 * hits by distance, alpha-blend). Each Gaussian is a unit sphere after its own affine
 * ray transform (GRTX-SW, Sec. IV-A); hits are gathered k at a time into a k-buffer
 * (Sec. III-A, Listing 1) and each round resumes from a per-ray traversal checkpoint
 * (deferred nodes and evicted hits, GRTX-HW, Sec. IV-B) instead of the root.
 *
 * Conventions for every entry point:
 *   - All functions return grtx_status. On any status other than GRTX_OK the
 *     out-parameters are left untouched and grtx_last_error() returns a message
 *     (thread-local; valid until the next call on the same thread).
 *   - Arguments are validated on the host before any launch.
 *   - Pointers named "device" must point to device memory of the current HIP device
 *     (hipMalloc or an equivalent allocator such as PyTorch's). Host pointers are
 *     named "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work is
 *     enqueued asynchronously on it; the caller synchronises.
 *   - No exception crosses the ABI.
 */
#ifndef GRTX_H
#define GRTX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRTX_VERSION 5

typedef enum grtx_status {
  GRTX_OK = 0,
  GRTX_ERR_INVALID_ARG = 1,   /* bad argument; nothing was enqueued */
  GRTX_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed */
  GRTX_ERR_DEVICE = 3,        /* a HIP call failed; the HIP message is in grtx_last_error() */
  GRTX_ERR_CAPACITY = 4,      /* a request can never fit the configured budget */
  GRTX_ERR_NOT_READY = 5,     /* asynchronous result not available yet */
  GRTX_ERR_INTERNAL = 6
} grtx_status;

/* Kind of acceleration structure.
 * SPHERE_INSTANCE: one leaf per Gaussian holding its world->unit-sphere transform; the
 *   leaf test is "transform the ray, intersect the unit sphere" (Sec. IV-A, bounding
 *   primitive 1). This is the method's structure.
 * PROXY20: one leaf per triangle of a bounding icosahedron per Gaussian (20N leaves),
 *   the monolithic triangle-mesh BVH of the baseline (Sec. III-C, Observation I;
 *   Sec. IV-A). Hits are ordered by the entry distance through the icosahedron.
 * ICO_INSTANCE: one leaf per Gaussian holding its transform, like SPHERE_INSTANCE, but
 *   the leaf test is the shared icosahedron (inradius 1) in the unit frame: the
 *   instanced-mesh configuration between the two (Sec. IV-A, one BLAS shared by all
 *   instances; Sec. V's intermediate design). Keys and images equal PROXY20's. */
typedef enum grtx_bvh_kind {
  GRTX_BVH_SPHERE_INSTANCE = 0,
  GRTX_BVH_PROXY20 = 1,
  GRTX_BVH_ICO_INSTANCE = 2
} grtx_bvh_kind;

/* Tracing mode.
 * CHECKPOINT: multi-round k-buffer tracing where each round resumes from the previous
 *   round's deferred nodes and evicted hits (Sec. IV-B, traversal checkpointing and
 *   replay; Listing 1).
 * RESTART: each round restarts from the root with t_min = the last blended hit
 *   (Sec. III-A; the multi-round baseline). Both modes give identical outputs. */
typedef enum grtx_mode {
  GRTX_MODE_CHECKPOINT = 0,
  GRTX_MODE_RESTART = 1,
  /* SINGLE_ROUND: the single-round alternative the paper weighs against multi-round
   *   tracing (Sec. III-C, Observation II): one traversal collects all of a ray's hits,
   *   unsorted, into a list of collect_capacity entries (no early termination during the
   *   traversal), which is then sorted and blended with early termination. k is not used.
   *   A ray with more hits than the list holds gets an incomplete result (the first hits
   *   in traversal order) and its GRTX_STAT_FALLBACKS counter set to 1; otherwise it
   *   blends the hits the other modes blend, in the same order, with colour and depth
   *   equal up to rounding (its accumulation runs in a kernel of its own). SPHERE_INSTANCE
   *   structures, unbounded rays without a starting transmittance; not available through
   *   grtx_trace_noalloc. */
  GRTX_MODE_SINGLE_ROUND = 2
} grtx_mode;

/* Scene parameters (Sec. II-B). All device pointers, float32, C-contiguous:
 *   means [count,3]; scales [count,3] linear standard deviation per axis;
 *   quats [count,4] (w,x,y,z), normalised inside; opacities [count];
 *   sh [count,(sh_degree+1)^2,3] real SH coefficients, band-major, m=-l..l, RGB last.
 * The library copies what it derives (transforms, boxes, nodes) and BORROWS opacities
 * and sh: they must stay alive and unchanged until grtx_bvh_destroy. */
typedef struct grtx_gaussians {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  int64_t count;     /* >= 0; 0 gives an empty scene */
  int32_t sh_degree; /* 0..3 */
  int32_t reserved;
} grtx_gaussians;

/* alpha_min: each Gaussian is bounded by the ellipsoid on which o*G = alpha_min, i.e.
 * Mahalanobis radius rho = sqrt(2 ln(o/alpha_min)); Gaussians with o <= alpha_min are
 * never hit. Must be in (0, 1).
 * plain_lbvh: nonzero keeps the radix tree exactly as the LBVH construction gives it (the
 * topology grtx_bvh_export_topology then reports is the plain Karras tree of the sorted
 * Morton codes); 0 (default) rebuilds small treelets of it bottom-up into the topology of
 * least surface-area cost. Leaves keep their sorted order either way, and traced results
 * are identical; only the internal nodes, and so the work per ray, differ.
 * max_depth: the deepest tree the build keeps, in internal nodes on a root-to-leaf path
 * (0 = GRTX_MAX_TREE_DEPTH, the depth the trace's traversal stack is sized for; at most
 * that). The plain radix tree over distinct 95-bit (Morton code, position) keys is never
 * deeper than 96; a restructured tree that comes out deeper is replaced on the device by
 * the plain one (grtx_bvh_info reports which). */
typedef struct grtx_build_params {
  float alpha_min;
  int32_t plain_lbvh;
  int32_t max_depth;
  int32_t reserved;
} grtx_build_params;

/* Deepest tree the trace supports: its per-lane stack holds 3 * GRTX_MAX_TREE_DEPTH + 16
 * entries, and a four-wide record leaves at most three entries pending per level. */
#define GRTX_MAX_TREE_DEPTH 96

typedef struct grtx_bvh grtx_bvh;

typedef struct grtx_bvh_info {
  int64_t gaussians;
  int64_t leaves;         /* gaussians (SPHERE_INSTANCE, ICO_INSTANCE) or 20*gaussians (PROXY20) */
  int64_t internal_nodes; /* leaves - 1 (0 for fewer than two leaves) */
  int64_t device_bytes;   /* bytes the handle owns on the device */
  int32_t kind;
  int32_t sh_degree;
  float alpha_min;
  float root_lo[3];       /* filled only after the build has completed on its stream */
  float root_hi[3];
  int32_t depth;          /* internal nodes on the longest root-to-leaf path (0: < 2 leaves) */
  int32_t restructured;   /* 1: treelet-restructured tree; 0: plain radix tree (asked for,
                             or the restructured tree exceeded max_depth) */
} grtx_bvh_info;

/* Rays: device origins [count,3] and unit-length directions [count,3], float32.
 * t_near >= 0: hits need an entry distance > t_near. image_width > 0 declares rays
 * image_begin..count-1 to be a row-major image of that width (image_begin = 0: all of
 * them); the kernel then schedules those in 8x8 pixel tiles, after the rays before
 * image_begin, which form no image. One launch thus traces an image together with a
 * set of other rays, and the image's cheaper tiles fill the end of the launch. Results
 * are unaffected. image_begin must lie in 0..count, and be 0 when image_width is 0; a
 * trace launch takes at most 2^31-1 rays, counting an image's 8x8 tiles whole.
 * Optional, for ray paths traced in segments (secondary rays, below):
 *   t_far [count] float32 (NULL = unbounded): the ray ends on a surface at that distance;
 *     hits need a key distance < t_far, and a bounded ray (t_far < +inf) gets no
 *     background, which the surface hides.
 *   transmittance [count] float32 (NULL = 1): the transmittance the ray starts with, the
 *     light an earlier segment of its path left; blending weights scale with it, and
 *     early termination compares the running transmittance with T_min.
 *   next_origins, next_dirs [count,3], path [count], kind [count] (all four or none; the
 *     outputs of grtx_object_rays; needs t_far and t_near = 0): a ray whose kind is MIRROR
 *     or GLASS and which reaches its t_far with transmittance >= T_min goes on, in the same
 *     launch, along its continuation ray (unbounded). The outputs are then those of the
 *     whole path, as grtx_continue_rays, a trace and grtx_continue_composite give them
 *     (equal up to rounding order), and hit_ids lists both segments' hits in order. */
typedef struct grtx_rays {
  const float* origins;
  const float* dirs;
  int64_t count;
  float t_near;
  int32_t image_width;
  const float* t_far;
  const float* transmittance;
  const float* next_origins;
  const float* next_dirs;
  const float* path;
  const int32_t* kind;
  int64_t image_begin;
} grtx_rays;

/* k: k-buffer size, 1..64 (Sec. III-A). T_min: a ray stops after the hit that brings
 * its transmittance below T_min (early ray termination, Sec. III-A), in [0, 1).
 * mode: grtx_mode. bg: background colour added with the remaining transmittance.
 * defer_capacity / evict_capacity: per-ray entries of the checkpoint lists (0 = the
 * defaults: 256 deferred nodes and 128 evicted hits, or 12288 and 3072 for structures of
 * more than a million leaves, where grtx_trace_noalloc takes 2048 and 512), rounded up
 * to a multiple of 8. A nearly full list is compacted: its nearer entries stay and the
 * ray's distance limit comes down to where the dropped ones begin; the ray falls back to
 * a restart-from-root round only if its blending reaches that limit. Results are the same
 * for every capacity. The lists live in a per-stream pool of
 * 512 B x (288 + 2 x defer + 2 x evict + k) per wave in flight (3072 waves at k <= 32:
 * about 1.7 GB with 256/128, 49 GB with 12288/3072), kept for later calls on the stream;
 * RESTART keeps no lists and takes 512 B x (288 + k) per wave. */
typedef struct grtx_trace_params {
  int32_t k;
  float T_min;
  int32_t mode;
  float bg[3];
  int32_t defer_capacity;
  int32_t evict_capacity;
  int32_t collect_capacity; /* SINGLE_ROUND: hits listed per ray, 0 = 2048, at most 8192 */
  int32_t reserved;
} grtx_trace_params;

/* Per-ray counters written to grtx_trace_outputs.stats. They count the work a ray took.
 * Where a checkpoint list fills and is compacted, the point at which that happens follows
 * the launch's scheduling, so the counts of entries written and of the work after it can
 * differ between launches, and so can the rounds of a ray that then restarts from the
 * root (GRTX_STAT_FALLBACKS); the blended count, like the outputs, cannot. */
enum {
  GRTX_STAT_NODES = 0,      /* internal nodes fetched and tested */
  GRTX_STAT_LEAVES = 1,     /* leaf primitives fetched and tested */
  GRTX_STAT_ROUNDS = 2,     /* tracing rounds */
  GRTX_STAT_BLENDED = 3,    /* hits blended */
  GRTX_STAT_DEFERRED = 4,   /* checkpoint entries written (node deferrals and copies) */
  GRTX_STAT_FETCH_FREE = 5, /* checkpoint entries carried forward without a fetch */
  GRTX_STAT_EVICTED = 6,    /* hits written to the eviction list */
  GRTX_STAT_FALLBACKS = 7,  /* rounds restarted from the root after a list overflow */
  GRTX_STAT_STACK_DROPS = 8, /* traversal-stack entries lost to a full stack; zero for every
                                tree the build keeps (depth <= GRTX_MAX_TREE_DEPTH) */
  GRTX_STATS_FIELDS = 9
};

/* Outputs, all caller-owned device memory:
 *   rgb [count,3], depth [count] (sum of w_i t_alpha_i), opacity [count] (1 - T).
 *   stats: optional [count, GRTX_STATS_FIELDS] uint32.
 *   hit_ids: optional [count, hit_capacity] int32: ids of the blended Gaussians in blend
 *     order (the first hit_capacity of them); hit_counts: optional [count] int32, the
 *     number of blended hits (may exceed hit_capacity). */
typedef struct grtx_trace_outputs {
  float* rgb;
  float* depth;
  float* opacity;
  uint32_t* stats;
  int32_t* hit_ids;
  int32_t* hit_counts;
  int32_t hit_capacity;
  int32_t reserved;
} grtx_trace_outputs;

/* Pinhole camera (ray generation, Sec. III-A): forward = normalise(target - eye),
 * right = normalise(forward x up), true up = right x forward; pixel (x, y), row 0 at
 * the top, sampled at its centre; vertical field of view in degrees. */
typedef struct grtx_camera {
  float eye[3];
  float target[3];
  float up[3];
  float fov_y_deg;
  int32_t width;
  int32_t height;
} grtx_camera;

/* Build the acceleration structure (LBVH: Morton codes of the means, stable radix
 * sort, radix tree, bottom-up refit, then, unless p->plain_lbvh, bottom-up passes of
 * treelet restructuring: one, three above 2^20 leaves) over `g`. Enqueued on `stream`; the handle may be
 * used for grtx_trace on the same stream right away. On success *out receives a new
 * handle (free it with grtx_bvh_destroy). */
grtx_status grtx_build(const grtx_gaussians* g, grtx_bvh_kind kind, const grtx_build_params* p,
                       void* stream, grtx_bvh** out);

/* Sizes, bounds and depth of a built structure (host out-param). Synchronises `bvh`'s
 * build stream to read the root bounds and the depth. */
grtx_status grtx_bvh_get_info(const grtx_bvh* bvh, grtx_bvh_info* out);

/* Copy the topology into caller-owned DEVICE buffers (each may be NULL to skip):
 *   child  [internal_nodes,2] uint32: bit 31 set = leaf, low bits = sorted leaf position;
 *          otherwise an internal node index (0 = root);
 *   parent [internal_nodes + leaves] uint32: internal nodes first, then leaves in sorted
 *          order; the root's parent is 0xFFFFFFFF;
 *   morton [leaves] uint64: sorted Morton codes;
 *   perm   [leaves] uint32: sorted position -> primitive index (Gaussian index, or
 *          20*gaussian + face for PROXY20);
 *   boxes  [internal_nodes + leaves, 6] float32: (lo xyz, hi xyz) of every node, same
 *          order as parent.
 * Enqueued on `stream`. */
grtx_status grtx_bvh_export_topology(const grtx_bvh* bvh, uint32_t* child, uint32_t* parent, uint64_t* morton,
                                     uint32_t* perm, float* boxes, void* stream);

/* Release a handle and its device memory. NULL is accepted. The caller must make sure
 * that no enqueued work still uses it. */
grtx_status grtx_bvh_destroy(grtx_bvh* bvh);

/* Generate width*height pinhole rays into caller-owned device buffers origins/dirs
 * [width*height,3] float32, row-major from the top row. */
grtx_status grtx_pinhole_rays(const grtx_camera* cam, float* origins, float* dirs, void* stream);

/* Render `rays` against `bvh` (Sec. III-A pipeline with Sec. IV-B checkpointing).
 * Deterministic: the same inputs give bit-identical colour, depth, opacity and hit lists,
 * in either mode, for any k and whatever the scheduling (see the counters above). The library keeps a per-(device, stream) pool of per-ray checkpoint storage and
 * grows it on demand (GRTX_ERR_OUT_OF_MEMORY if it cannot). Calls on one stream are
 * ordered; calls on different streams use different pools. */
grtx_status grtx_trace(const grtx_bvh* bvh, const grtx_rays* rays, const grtx_trace_params* p,
                       const grtx_trace_outputs* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): grtx_trace with the same arguments,
 * conventions and results (bit-identical outputs), except that it calls no allocator.
 * Its working memory (the work counters and the per-wave checkpoint lists and stack spill)
 * is a static array of GRTX_NOALLOC_SCRATCH_MB MiB that each device running the library
 * holds from the library's first use on it until the process ends. As many persistent
 * workgroups run as their lists fit in it (about 2.1 MiB per workgroup at k = 16 with
 * the 256/128 default capacities, 11 MiB with 2048/512), so throughput can be below
 * grtx_trace's; image rays are taken in row-major tile order and other rays in the
 * caller's order (grtx_trace orders both by estimated cost). GRTX_ERR_CAPACITY when not
 * even one workgroup's lists fit (lower defer_capacity / evict_capacity). Every call on a
 * device uses that device's one array: calls that overlap on one device (different
 * streams or threads without ordering between them) race and give wrong results; calls
 * ordered on one stream are safe (each call resets the counters it uses). */
#define GRTX_NOALLOC_SCRATCH_MB 512
grtx_status grtx_trace_noalloc(const grtx_bvh* bvh, const grtx_rays* rays, const grtx_trace_params* p,
                               const grtx_trace_outputs* out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Secondary rays: ray continuation at a surface (Sec. II-A), with the two objects of the
 * paper's secondary-ray experiment, a glass sphere and a rectangular mirror placed in
 * the scene (Sec. VI). A path is traced in segments. grtx_object_rays finds where each
 * ray meets an object and the ray that continues from there; grtx_trace renders the
 * segment up to that surface (rays.t_far); grtx_continue_rays gathers the continuation
 * rays of the segments that reached their surface; grtx_trace renders those, starting
 * from the transmittance left (rays.transmittance); grtx_continue_composite adds their
 * results to the segments they continue. Repeating the steps follows further bounces.
 * ------------------------------------------------------------------------------------- */

/* Glass sphere: centre, radius (<= 0: none), index of refraction relative to the
 * surroundings (> 0). Mirror: the parallelogram centre + x u + y v, |x| <= 1, |y| <= 1,
 * u and v orthogonal half-axes (u x v = 0: none). Object hits need a distance
 * > t_near + surface_eps (0 = 1e-4), so that a continuation ray does not meet the
 * surface it starts on. */
typedef struct grtx_objects {
  float sphere_center[3];
  float sphere_radius;
  float sphere_ior;
  float mirror_center[3];
  float mirror_u[3];
  float mirror_v[3];
  float surface_eps;
} grtx_objects;

/* What a ray met (grtx_object_rays kind). */
typedef enum grtx_object_kind {
  GRTX_OBJECT_NONE = 0,
  GRTX_OBJECT_MIRROR = 1,
  GRTX_OBJECT_GLASS = 2,
  GRTX_OBJECT_GLASS_TRAPPED = 3 /* still inside after 8 chords of total internal reflection */
} grtx_object_kind;

/* For each ray of `rays` (origins, dirs, count, t_near; t_far and transmittance are not
 * read): t_far [count], the distance to the first object surface (+inf if none); the
 * continuation ray next_origins / next_dirs [count,3] (unit direction; zeros where there
 * is none); path [count], the length of the bent path from the ray origin to the
 * continuation origin; kind [count] (grtx_object_kind). Mirror: two-sided, perfect
 * reflection d - 2 (d.n) n. Glass: solid (no Gaussian inside it is seen); Snell
 * refraction in, along the chord, refraction out; total internal reflection follows
 * further chords, at most 8. All light follows the one continuation ray (no Fresnel
 * split, no absorption). Outputs are caller-owned device arrays. Enqueued on `stream`.
 * ERR_INVALID_ARG for a non-positive index, or mirror half-axes that are not orthogonal
 * (|u.v| > 1e-4 |u||v|). */
grtx_status grtx_object_rays(const grtx_objects* obj, const grtx_rays* rays, float* t_far, float* next_origins,
                             float* next_dirs, float* path, int32_t* kind, void* stream);

/* Gather continuation rays: ray i continues if kind[i] is MIRROR or GLASS and its
 * segment reached the surface, i.e. it left transmittance T = 1 - opacity[i] >= T_min
 * (early termination did not stop it). For the continuing rays in increasing i, writes
 * cont_origins / cont_dirs [n,3] (copies of next_origins / next_dirs), cont_transmittance
 * [n] = T and cont_index [n] = i into caller-owned device buffers of `count` entries, and
 * n into *n_cont (host memory). count <= 2^24. Enqueued on `stream`; the call waits once
 * on `stream` to read n. Scratch of 8 B per ray is allocated and freed in stream order. */
grtx_status grtx_continue_rays(int64_t count, const int32_t* kind, const float* opacity, float T_min,
                               const float* next_origins, const float* next_dirs, float* cont_origins,
                               float* cont_dirs, float* cont_transmittance, int32_t* cont_index, int64_t* n_cont,
                               void* stream);

/* Add the results of n continuation rays (cont_rgb [n,3], cont_depth [n], cont_opacity
 * [n], the outputs of grtx_trace over the gathered rays with their transmittance) to the
 * segments they continue, in place, for i = cont_index[j]:
 *   rgb[i]     += cont_rgb[j]
 *   depth[i]   += cont_depth[j] + path[i] * (cont_transmittance[j] - (1 - cont_opacity[j]))
 *   opacity[i]  = cont_opacity[j]
 * so depth sums distances along the bent path and opacity is one minus the path's final
 * transmittance. cont_index entries must be distinct. Enqueued on `stream`. */
grtx_status grtx_continue_composite(int64_t n, const int32_t* cont_index, const float* cont_transmittance,
                                    const float* path, const float* cont_rgb, const float* cont_depth,
                                    const float* cont_opacity, float* rgb, float* depth, float* opacity,
                                    void* stream);

/* Gradients of the Gaussian parameters, caller-owned DEVICE arrays shaped like the inputs
 * of grtx_gaussians (means [N,3], scales [N,3], quats [N,4], opacities [N],
 * sh [N,(L+1)^2,3]). grtx_trace_backward ADDS into them (it never zeroes). */
typedef struct grtx_gaussian_grads {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
} grtx_gaussian_grads;

/* Backward of grtx_trace (differentiation of Eq. 1 with Eq. 2 alphas and SH colours;
 * the paper's method is forward-only). `g` must be the parameters `bvh` was built from
 * and `rays`/`p` those of the forward call. `fwd` holds the forward outputs:
 *   - with fwd->hit_ids (and hit_counts, hit_capacity > 0): rgb, depth and opacity are
 *     required too, and the blended hits are read from the list;
 *   - with fwd->hit_ids NULL: the rays are traced again (grtx_trace with `p`, which is
 *     deterministic and so gives the forward's outputs) into internal lists of
 *     fwd->hit_capacity entries per ray (0 = 256); fwd's other fields are not read.
 * grad_rgb [R,3] is dL/drgb; grad_depth [R] and grad_opacity [R] are optional (NULL =
 * zero). For each ray the blended hits are replayed in order; the per-hit contributions
 * are grouped by Gaussian (sorted, ray order kept) and summed in a fixed order, then
 * added to `grads` (which the caller zeroes): results are deterministic. Rays with more
 * blended hits than the list holds contribute only their first hit_capacity hits; their
 * number is written to the optional device counter `truncated_rays` (uint32, may be
 * NULL). Enqueued on `stream` without any host wait: the number of hit records stays on
 * the device, and scratch of about 88 B x rays x hit_capacity is taken from the
 * stream's pool and released in stream order. ERR_INVALID_ARG when rays x hit_capacity
 * reaches 2^32, or for rays with t_far or transmittance (the backward pass covers
 * unbounded rays that start with transmittance 1 and have no continuation). */
grtx_status grtx_trace_backward(const grtx_bvh* bvh, const grtx_gaussians* g, const grtx_rays* rays,
                                const grtx_trace_params* p, const grtx_trace_outputs* fwd, const float* grad_rgb,
                                const float* grad_depth, const float* grad_opacity, const grtx_gaussian_grads* grads,
                                uint32_t* truncated_rays, void* stream);

/* ---------------------------------------------------------------------------------------
 * Serving: render requests over several device-resident scenes, traced by one persistent
 * kernel fed from a work queue (an extension of the method to a serving workload; each
 * ray is traced as in grtx_trace, Sec. III-A and IV-B).
 * A worker thread admits queued requests first come, first served while their outputs
 * fit the memory budget and publishes each admitted request to a queue in host memory.
 * One kernel launch, resident on all but a few CUs, takes the published requests' 8x8
 * pixel tiles as its lanes fall idle, generates each pixel's ray from the request's
 * camera, and flags the request in host memory when its last pixel is written; a request
 * published while the kernel runs joins it. The launch ends once no work has been taken
 * for `idle_exit_us` (freeing the device for other work) and the next publication starts
 * another. Results are identical to tracing each request alone with grtx_pinhole_rays +
 * grtx_trace on its scene.
 * ------------------------------------------------------------------------------------- */
typedef struct grtx_server grtx_server;

/* memory_budget: device bytes the server may hold (the serving kernel's checkpoint pool,
 *   about 8.3 GB at k <= 32 for 2048 deferred nodes and 512 evicted hits per lane,
 *   the scene set copy, and per admitted request its outputs until released; the outputs
 *   live in an arena grown in chunks of at least 1 GiB within the budget).
 * k, T_min, mode, bg: as in grtx_trace_params, for every request (mode CHECKPOINT or
 *   RESTART).
 * max_request_rays: pixels per request (0 = 2^22, also the largest accepted); larger
 *   requests are refused.
 * idle_exit_us: how long the kernel waits for new work before it ends (0 = 2000). */
typedef struct grtx_serve_config {
  int64_t memory_budget;
  int32_t k;
  float T_min;
  int32_t mode;
  int32_t max_request_rays;
  float bg[3];
  int32_t idle_exit_us;
} grtx_serve_config;

/* A render request: pinhole camera (as grtx_camera) on scene `scene_id`. */
typedef struct grtx_request {
  int32_t scene_id;
  int32_t width;
  int32_t height;
  float eye[3];
  float target[3];
  float up[3];
  float fov_y_deg;
} grtx_request;

/* Result of a finished request: device arrays rgb [H*W,3], depth [H*W], opacity [H*W]
 * (row-major pixels), owned by the server until grtx_serve_release; timestamps in
 * seconds since the server was created: submitted, admitted (outputs placed and the
 * request published to the kernel; t_launch is the same moment), finished (seen by the
 * worker). */
typedef struct grtx_request_result {
  const float* rgb;
  const float* depth;
  const float* opacity;
  int32_t width;
  int32_t height;
  double t_submit;
  double t_admit;
  double t_launch;
  double t_done;
} grtx_request_result;

/* Latency percentiles over finished requests (submission to completion), throughput
 * over the span from the first publication to the last completion, the budget's use
 * (bytes held by admitted requests, bytes the budget leaves for outputs, bytes of arena
 * allocated) and the number of kernel launches so far. */
typedef struct grtx_serve_stats {
  int64_t submitted;
  int64_t completed;
  int64_t rays_completed;
  int64_t bytes_in_use;
  int64_t bytes_available;
  int64_t bytes_arena;
  int64_t launches;
  double p50_ms;
  double p99_ms;
  double mean_ms;
  double max_ms;
  double busy_s;
  double mrays_per_s;
} grtx_serve_stats;

/* Device bytes a request holds while admitted (host-only; no device needed). */
grtx_status grtx_serve_request_bytes(const grtx_request* r, int64_t* bytes);

/* Create a server on the current device. GRTX_ERR_CAPACITY if the budget cannot even
 * hold the serving kernel's checkpoint pool. */
grtx_status grtx_serve_create(const grtx_serve_config* cfg, grtx_server** out);

/* Register a built SPHERE_INSTANCE structure (all scenes share one SH degree) before the
 * first request; its device data is copied into the server's scene set at the first
 * submit. *scene_id receives the index requests use. The handle may be destroyed after
 * the first submit. */
grtx_status grtx_serve_add_scene(grtx_server* s, const grtx_bvh* bvh, int32_t* scene_id);

/* Queue a request; *ticket identifies it. GRTX_ERR_CAPACITY if it can never fit the
 * budget or max_request_rays. Thread-safe. */
grtx_status grtx_serve_submit(grtx_server* s, const grtx_request* r, uint64_t* ticket);

/* GRTX_OK with *res filled once the request has finished, GRTX_ERR_NOT_READY while it
 * is queued or in flight, GRTX_ERR_DEVICE if its launch failed. Thread-safe. */
grtx_status grtx_serve_poll(grtx_server* s, uint64_t ticket, grtx_request_result* res);

/* Copy a finished request's outputs into caller-owned DEVICE arrays (rgb [H*W,3],
 * depth [H*W], opacity [H*W]; each may be NULL), enqueued on `stream`. */
grtx_status grtx_serve_copy_result(grtx_server* s, uint64_t ticket, float* rgb, float* depth, float* opacity,
                                   void* stream);

/* Free a finished request's outputs (and its share of the budget), or withdraw a
 * request that is still queued; GRTX_ERR_NOT_READY while it is in flight. */
grtx_status grtx_serve_release(grtx_server* s, uint64_t ticket);

grtx_status grtx_serve_get_stats(grtx_server* s, grtx_serve_stats* st);

/* Stop: the kernel finishes the published requests, queued ones are dropped, and
 * everything is freed. NULL is accepted. */
grtx_status grtx_serve_destroy(grtx_server* s);

/* Message of the last failure on the calling thread ("" if none). */
const char* grtx_last_error(void);

/* GRTX_VERSION of the loaded library. */
int32_t grtx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRTX_H */
