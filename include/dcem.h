/*
 * dcem.h - C ABI of the MI355X dynamic coherence-based EM ray tracer.
 *
 * Implements the per-frame loop of Wang & Manocha, "Dynamic Coherence-Based
 * EM Ray Tracing Simulations in Vehicular Environments" (Sec. III): a BVH
 * kept up to date while vehicles move ("Efficient BVH updating"), a sphere of
 * rays bounced by specular reflection up to K times (the frame algorithm's
 * steps 1-2 and the "Reflected and transmitted rays" item), receiver capture
 * spheres, de-duplicated face-sequence candidates (the per-depth visited-path
 * tables), image-method refinement and validation (steps 3-4), per-path
 * distance, direction, Fresnel attenuation and phase (step 6), and per-receiver
 * received power (Eq. (3) with path-loss exponent 2 for the free-space
 * magnitude, plus the phase calculation).  Paths found in the previous frame
 * are revalidated and only invalidated rays are traced again ("Propagation
 * path caching").
 *
 * Rays are shot from the transmitters and captured at receiver spheres, or
 * (trace_from_rx) cast from the receivers and captured at transmitter
 * spheres, the paper's backward tracing (Sec. III, "Backward ray tracing");
 * both directions yield the same candidates, keyed from the transmitter, so
 * everything after the trace is the same.
 *
 * Units: metres, hertz, watts, siemens per metre.  Right-handed, z up.
 * Geometry is FP32; path lengths, phases and fields are FP64.
 *
 * Conventions for every call:
 *  - A dcem_ctx owns one HIP device and one HIP stream; all work is enqueued
 *    on that stream in call order.  A context is not thread-safe.
 *  - Input arrays are owned by the caller.  Host inputs (mem_kind
 *    DCEM_MEM_HOST) are copied before the call returns and may be freed at
 *    once.  Device inputs (DCEM_MEM_DEVICE) are read on the context's stream
 *    and must stay valid and unchanged until that stream has passed the call.
 *  - No exception or abort crosses this interface.  Every call returns a
 *    dcem_status; on failure dcem_last_error() describes it.  Faults detected
 *    inside kernels (traversal stack overflow, candidate buffer overflow,
 *    non-finite input) set a device error word that is reported by the next
 *    call that synchronises (dcem_received_power, dcem_get_*); that frame's
 *    outputs are then undefined.
 *  - Call order: dcem_scene_upload, then per frame optionally
 *    dcem_set_object_transforms and dcem_refit_bvh, then dcem_trace_frame,
 *    then dcem_received_power / dcem_get_*.  Other orders return
 *    DCEM_E_STATE.
 */
#ifndef DCEM_H
#define DCEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dcem_ctx dcem_ctx;
typedef int32_t dcem_status;

#define DCEM_OK 0
#define DCEM_E_INVALID_ARG (-1)   /* bad pointer, size, index or non-finite value */
#define DCEM_E_OUT_OF_MEMORY (-2) /* device allocation failed */
#define DCEM_E_DEVICE (-3)        /* HIP runtime error */
#define DCEM_E_STATE (-4)         /* call made out of order */
#define DCEM_E_CAPACITY (-5)      /* a device buffer or the traversal stack overflowed */
#define DCEM_E_UNSUPPORTED (-6)   /* sizes beyond what this build supports */

#define DCEM_MEM_HOST 0
#define DCEM_MEM_DEVICE 1

#define DCEM_MODE_FULL 0      /* trace every ray */
#define DCEM_MODE_COHERENT 1  /* reuse the previous frame's rays; retrace invalidated ones */

#define DCEM_FORCE_REBUILD 1     /* dcem_refit_bvh flag: rebuild the whole tree instead of refitting */
#define DCEM_REBUILD_SUBTREES 2  /* dcem_refit_bvh flag: rebuild the tree above the objects' subtrees */

/* dcem_refit_bvh's decision (rebuilt, dcem_frame_stats.rebuilt) */
#define DCEM_REFITTED 0
#define DCEM_REBUILT_FULL 1      /* the whole tree was built again */
#define DCEM_REBUILT_SUBTREES 2  /* only the tree above the objects' subtrees was built again */

/* dcem_trace_params.discovery: which face sequences become candidates */
#define DCEM_DISCOVER_CAPTURE 0  /* sequences of rays that pass through a capture sphere */
#define DCEM_DISCOVER_VISITED 1  /* every visited series, tried against every target */

#define DCEM_MAX_REFLECTIONS 10  /* paper, Sec. III: at most 10 reflections and transmissions */
#define DCEM_MAX_TRANSMISSIONS 2 /* transmissions per path (dcem_trace_params.max_transmissions) */
#define DCEM_PATTERN_TAPS 16     /* weights of the transmit pattern (dcem_set_tx_pattern) */

/* bits of the device error word (reported as DCEM_E_CAPACITY / DCEM_E_INVALID_ARG) */
#define DCEM_ERR_STACK 1u      /* traversal stack overflow */
#define DCEM_ERR_CAPTURES 2u   /* more captures than the candidate capacity */
#define DCEM_ERR_NONFINITE 4u  /* non-finite vertex after a transform */

/* Scene geometry and materials (paper Sec. III: the environment description
 * and Table II's per-material reflection properties).
 *  vertices             [n_vertices][3] FP32, the upload (reference) pose
 *  tris                 [n_tris][3] vertex indices
 *  tri_face             [n_tris] face index of each triangle.  A face is a
 *                       planar group of triangles; paths are identified by
 *                       face sequences, so a tessellated wall is one face.
 *  face_material        [n_faces] material index
 *  face_object          [n_faces] moving-object index, -1 for static faces
 *  materials            [n_materials][3] FP64: eps_r, sigma [S/m],
 *                       const_gamma.  const_gamma = NaN selects Fresnel
 *                       coefficients from (eps_r, sigma); any other value g
 *                       is a polarisation-independent coefficient of
 *                       magnitude g (Table II's scalar reflection
 *                       coefficient): Gamma_TE = -g, Gamma_TM = +g.
 *  object_vertex_range  [n_objects][2] half-open vertex range of each moving
 *                       object; ranges must not overlap
 *  mem_kind             DCEM_MEM_HOST or DCEM_MEM_DEVICE for all arrays
 * Limits: n_tris < 2^27, n_vertices < 2^31, n_faces < 2^20, n_objects < 2^16. */
typedef struct dcem_scene_desc {
  const float* vertices;
  int64_t n_vertices;
  const int32_t* tris;
  const int32_t* tri_face;
  int64_t n_tris;
  const int32_t* face_material;
  const int32_t* face_object;
  int32_t n_faces;
  const double* materials;
  int32_t n_materials;
  const int64_t* object_vertex_range;
  int32_t n_objects;
  int32_t mem_kind;
} dcem_scene_desc;

/* One frame of tracing.
 *  tx_pos [n_tx][3], rx_pos [n_rx][3] FP32 (mem_kind); rx_radius: capture
 *  sphere radius (closed ball, transparent).
 *  n_rays: rays per transmitter; ray_dirs [n_rays][3] FP32 (mem_kind) or NULL
 *  for a Fibonacci sphere: z_i = 1 - (2i+1)/n, phi_i = i * pi * (3 - sqrt 5),
 *  evaluated in FP64 and rounded to FP32 (paper: "a sphere of sampled rays").
 *  max_reflections: 0..DCEM_MAX_REFLECTIONS.
 *  freqs_hz [n_freqs] FP64, host memory.  tx_power_w: transmit power;
 *  atten_db_per_km: Eq. (3)'s atmospheric term as a specific attenuation.
 *  mode: DCEM_MODE_FULL or DCEM_MODE_COHERENT.  COHERENT reuses the cached
 *  rays of the previous frame traced with the same transmitters, rays,
 *  max_reflections, receiver count and capture radius (falls back to FULL
 *  otherwise; ray_dirs given in device memory are re-read every frame and
 *  always count as changed).  Receivers may move between coherent frames
 *  (vehicle-mounted receivers): the captures of every reused segment are then
 *  taken again against the new positions from the cached segments, so the
 *  frame still equals a full re-trace.
 *  los_always: 1 adds the direct path of every (tx, rx) pair as a candidate
 *  (direct rays are their own mechanism, Sec. III); 0 keeps only captured ones.
 *  keep_cache: 1 stores the per-ray segments needed by the next COHERENT
 *  frame (COHERENT implies it).
 *  record_trace_log: 1 stores per (tx, ray, bounce) the hit triangle, its
 *  distance and the cumulative path length (see dcem_get_trace_log).
 *  discovery: DCEM_DISCOVER_CAPTURE (0) keys a candidate for each capture
 *  sphere a ray passes through, with the faces it reflected on before.
 *  DCEM_DISCOVER_VISITED (1) follows the paper's frame algorithm literally
 *  (Sec. III, steps 2-4): every distinct series of faces the rays reflect on
 *  (the faces of a ray's first d hits, d = 1..max_reflections, per source) is
 *  entered in the visited table of its depth and tried against every target
 *  by the image method, so the path set no longer depends on a ray passing
 *  close to a receiver; rx_radius is then unused and no capture records are
 *  made.  The candidates kept are those whose reflection points lie strictly
 *  inside their segments and inside their faces (checked before the
 *  occlusion tests of the refinement, with the same arithmetic); their number
 *  is bounded by the capture capacity (dcem_set_capture_capacity; overflow
 *  sets DCEM_ERR_CAPTURES) and the series times targets by 2^32
 *  (DCEM_E_UNSUPPORTED).  los_always keeps its meaning (the empty series).
 *  Candidate discovery of this mode reads counts back to the host (it is not
 *  asynchronous).  Coherent frames reuse rays traced in the same mode.
 *  max_transmissions: 0..DCEM_MAX_TRANSMISSIONS, with max_reflections +
 *  max_transmissions <= DCEM_MAX_REFLECTIONS (Sec. III, "Reflected and
 *  transmitted rays": at most 10 interactions).  A ray that meets a face whose
 *  material has a finite penetration loss (dcem_set_penetration_loss) splits
 *  into the reflected ray and the ray that goes straight on through the face;
 *  each ray is traced once per branch, a branch being the set of its first
 *  max_reflections + max_transmissions interactions that transmit (at most
 *  max_transmissions of them; n_branch = sum over t <= max_transmissions of
 *  C(max_reflections + max_transmissions, t), branch 0 only reflects; a
 *  branch ends where it would transmit through an opaque face or reflect a
 *  (max_reflections + 1)-th time).  Paths are then sequences of interactions,
 *  each a reflection or a transmission, at most max_reflections of the first
 *  and max_transmissions of the second; a transmission scales the field by
 *  the face's penetration loss and leaves its direction and polarisation
 *  unchanged.  0 (the paper's outdoor setting: no penetration) traces one
 *  branch.  Work items per frame: sources x n_branch x n_rays (< 2^31 - 1).
 *  trace_from_rx: 1 casts the n_rays rays from every receiver and captures
 *  them at spheres of radius rx_radius around the transmitters (backward
 *  tracing, Sec. III: the ray count no longer grows with the number of
 *  sources); every record is turned into the path's key from the transmitter
 *  (faces in reverse order of the trace), refined and accumulated as in a
 *  forward frame.  0 shoots from the transmitters.  Coherent frames reuse the
 *  rays of a previous frame traced in the same direction; in a backward frame
 *  the transmitters are the capture spheres and may move between coherent
 *  frames, while moved receivers re-trace.
 *  Antennas are ideal and omnidirectional (Sec. III); the transmitter is
 *  vertically polarised (theta-hat of the departure direction) and the
 *  receiver is polarisation-agnostic. */
typedef struct dcem_trace_params {
  const float* tx_pos;
  int32_t n_tx;
  const float* rx_pos;
  int32_t n_rx;
  float rx_radius;
  int64_t n_rays;
  const float* ray_dirs;
  int32_t max_reflections;
  const double* freqs_hz;
  int32_t n_freqs;
  double tx_power_w;
  double atten_db_per_km;
  int32_t mode;
  int32_t los_always;
  int32_t keep_cache;
  int32_t record_trace_log;
  int32_t mem_kind;
  int32_t trace_from_rx;
  int32_t discovery;
  int32_t max_transmissions;
} dcem_trace_params;

/* Counters and timings of the last dcem_refit_bvh + dcem_trace_frame. */
typedef struct dcem_frame_stats {
  int64_t rays_total;        /* work items: sources (n_tx, or n_rx when tracing from the receivers)
                                x transmission branches x n_rays */
  int64_t rays_traced;       /* rays actually traced this frame */
  int64_t rays_reused;       /* rays whose cached result was reused */
  int64_t segments;          /* closest-hit queries executed */
  int64_t captures;          /* capture records (reused + new) */
  int64_t unique_candidates; /* unique (tx, rx, order, faces) keys */
  int64_t valid_paths;
  int64_t nodes_visited;     /* 4-wide BVH nodes the closest-hit traversal fetched from device memory
                                (the per-thread traversal keeps the top three levels in LDS) */
  int64_t tri_tests;         /* ray-triangle tests of the closest-hit traversal */
  int32_t rebuilt;           /* last dcem_refit_bvh: DCEM_REFITTED, DCEM_REBUILT_FULL or DCEM_REBUILT_SUBTREES */
  int32_t coherent;          /* this frame reused the cache */
  double sah_ratio;          /* SAH cost of the tree relative to its last build */
  /* stage times (dcem_set_timing): the refit or rebuild, then the trace's
   * stages; in a coherent frame the refit shares the revalidation launch, so
   * ms_refit is that launch and ms_coherence includes it */
  float ms_refit, ms_coherence, ms_trace, ms_candidates, ms_refine, ms_reduce;
  int32_t trace_kernel;      /* closest-hit traversal used: 0 one thread per ray, 1 one wavefront per ray */
} dcem_frame_stats;

/* Source of a context's device memory, so that a framework (a caching
 * allocator such as torch's) owns it.  alloc returns `bytes` of device memory
 * usable on `stream` (NULL on failure, reported as DCEM_E_OUT_OF_MEMORY);
 * free returns a block alloc gave, with its size.  Both are called on the
 * thread that makes the dcem call, only from dcem calls on the context, with
 * the context's stream: memory freed there may be reused by later work on
 * that stream only (stream-ordered reuse).  `user` is passed through. */
typedef struct dcem_allocator {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} dcem_allocator;

/* Create a context on `device`, enqueueing on `hip_stream` (a hipStream_t;
 * NULL = the device's null stream).  allocator (nullable, copied): where every
 * device buffer of the context comes from; NULL selects hipMalloc / hipFree.
 * Pinned host staging (the per-frame result block, the gradients' read-back)
 * is the library's own.  Errors: DCEM_E_INVALID_ARG for a bad device or an
 * allocator without both functions. */
dcem_status dcem_create(dcem_ctx** out, int32_t device, void* hip_stream, const dcem_allocator* allocator);
void dcem_destroy(dcem_ctx* ctx);
/* Human-readable description of the last failure on ctx ("" if none). */
const char* dcem_last_error(const dcem_ctx* ctx);
/* Capacity of the capture buffer (default 1<<22 records).  Overflow sets
 * DCEM_ERR_CAPTURES. */
dcem_status dcem_set_capture_capacity(dcem_ctx* ctx, int64_t max_captures);
/* Cap the closest-hit traversal stacks at `entries` entries per query (0
 * restores the full depth: 64 per ray in the per-thread traversal, the first
 * 32 in LDS, 128 in the group traversal; larger values are clamped to those).  Results do not
 * change unless a stack overflows; an overflow drops the entries that do not
 * fit, sets DCEM_ERR_STACK, and is reported as DCEM_E_CAPACITY by the next
 * synchronising call (that frame's outputs are undefined).  The full depth
 * holds every tree this library builds; smaller caps exercise the overflow
 * path.  Applies to frames traced after the call.
 * Errors: DCEM_E_INVALID_ARG for a negative count. */
dcem_status dcem_set_stack_limit(dcem_ctx* ctx, int32_t entries);
/* Enable per-stage HIP event timings in dcem_frame_stats (default off). */
dcem_status dcem_set_timing(dcem_ctx* ctx, int32_t enabled);

/* Copy the scene to the device and build its LBVH (paper Sec. III: the BVH
 * over the environment's triangles).  Replaces any previous scene and drops
 * the ray cache.  Validates indices and finiteness on the host (host inputs)
 * and returns DCEM_E_INVALID_ARG on a violation. */
dcem_status dcem_scene_upload(dcem_ctx* ctx, const dcem_scene_desc* scene);

/* Place the moving objects for the next frame (paper Sec. III: objects move
 * between frames).  xf [n_objects][3][4] row-major FP32 object-to-world
 * transforms applied to the upload pose: x' = R x + t, evaluated with exact
 * FP32 products summed left to right in FP64 and rounded to FP32. */
dcem_status dcem_set_object_transforms(dcem_ctx* ctx, const float* xf, int32_t n_objects,
                                       int32_t mem_kind);

/* Bring the BVH up to date with the current vertices (paper Sec. III,
 * "Efficient BVH updating"): refit the node boxes bottom-up over the fixed
 * topology (the binary tree and its 4-wide form together), measure quality as
 * the SAH surface-area sum relative to the last build, and rebuild instead
 * when the quality measured after the previous refit exceeds
 * rebuild_threshold (<= 0 selects 1.5; +inf never rebuilds) or when flags
 * has DCEM_FORCE_REBUILD or DCEM_REBUILD_SUBTREES.  A rebuild the quality
 * test asks for first rebuilds only subtrees (paper: "it is possible to just
 * rebuild subtrees in some cases"): the static geometry and each moving
 * object keep their own subtrees, which rigid motion does not degrade, and
 * only the tree above them is built again from the objects' current
 * positions (DCEM_REBUILT_SUBTREES); once the tree that leaves has a SAH sum
 * above rebuild_threshold times that of the last full build, the next
 * rebuild is a full one (DCEM_REBUILT_FULL).  The decision lags by one refit so that no host
 * round trip is needed: the ratio of a refit is read back by the next
 * synchronising call.  rebuilt / sah_ratio (nullable, host) receive the
 * decision and the ratio it was based on (1.0 right after a rebuild).
 * A rebuild is enqueued on the context stream at once; a refit is deferred to
 * the next call that reads the tree or the vertices (a coherent
 * dcem_trace_frame runs it in the same launch as its revalidation pass).
 * Device errors are reported by the next synchronising call.  The build at scene upload and the rebuilds the quality
 * test asks for put the static geometry and every moving object, and inside
 * them every face, in subtrees of their own, so that refits under rigid motion
 * keep the tree tight; a
 * forced rebuild orders all triangles along one Morton curve, the better tree
 * for a frame traced without refitting.  Rebuilding never changes traced
 * results: hits are the lexicographic minimum of (distance, triangle id) over
 * conservative boxes. */
dcem_status dcem_refit_bvh(dcem_ctx* ctx, int32_t flags, double rebuild_threshold,
                           int32_t* rebuilt, double* sah_ratio);

/* Trace one frame (asynchronous on the context stream). */
dcem_status dcem_trace_frame(dcem_ctx* ctx, const dcem_trace_params* params);

/* Received power of the last frame, [n_freqs][n_tx][n_rx] FP64 watts:
 * p_coh = sum over field components of |sum over valid paths of a_p|^2
 * (phase-coherent), p_incoh (nullable) = sum over paths of |a_p|^2.  Paths
 * are summed in key order, so results are bitwise reproducible.  Waits for
 * the frame and reports any device error. */
dcem_status dcem_received_power(dcem_ctx* ctx, double* p_coh, double* p_incoh, int32_t mem_kind);

/* Transmit field pattern, an extension of the paper's ideal omnidirectional
 * antenna (Sec. III takes the transmitter as isotropic): each path's field is
 * scaled by g(phi) = sum_j w_j B_j(phi), phi the azimuth (atan2(y, x)) of its
 * departure direction and B_j the periodic hat of half-width 2 pi / 16
 * centred on azimuth 2 pi j / 16.  The hats sum to one, so all weights 1 is
 * the isotropic antenna; the power scales with g^2.
 * weights: host, DCEM_PATTERN_TAPS finite values (any sign), copied; null with
 * n_weights = 0 restores the isotropic antenna (the default).  Applies to the
 * frames traced after the call, for every transmitter; scene uploads keep it.
 * Errors: DCEM_E_INVALID_ARG for another count or a non-finite weight. */
dcem_status dcem_set_tx_pattern(dcem_ctx* ctx, const double* weights, int32_t n_weights);

/* Replace the scene's material table (same count and row layout as
 * dcem_scene_desc.materials: eps_r >= 1, sigma >= 0, const_gamma in [0, 1] or
 * NaN) without a new upload: the geometry, the BVH and the coherent-frame
 * cache stay, since materials change only the fields (Sec. III, the Fresnel
 * coefficients of Eq. (3)'s reflected paths).  materials: host, copied.
 * Applies to the frames traced after the call; the last frame's powers and
 * gradients keep the table it was traced with.  For calibration loops that
 * fit materials with dcem_power_gradients.
 * Errors: DCEM_E_STATE without a scene; DCEM_E_INVALID_ARG for another count
 * or an invalid row. */
dcem_status dcem_set_materials(dcem_ctx* ctx, const double* materials, int32_t n_materials);

/* Penetration loss of each material in dB (Table II: indoor wall 20 dB,
 * glass 5 dB), the field factor of a transmission through a face of that
 * material being 10^(-loss/20) at any incidence; +inf (the default after
 * every scene upload) makes the material opaque.  Paths transmit only when a
 * frame's max_transmissions > 0.  loss_db: host, n_materials values >= 0 or
 * +inf, copied; applies to the frames traced after the call (the ray cache
 * is dropped).  The Table II thickness does not enter: a plane-parallel slab
 * leaves a ray's direction unchanged, and the lateral offset it causes (at
 * most the thickness times tan theta) is neglected with it.
 * Errors: DCEM_E_STATE without a scene; DCEM_E_INVALID_ARG for another count
 * or a negative or NaN loss. */
dcem_status dcem_set_penetration_loss(dcem_ctx* ctx, const double* loss_db, int32_t n_materials);

/* Derivatives of the last frame's coherent received power p_coh (see
 * dcem_received_power) along its fixed set of valid paths: the path geometry
 * is held, and the field of each path (Sec. III, Eq. (3) with the Fresnel
 * reflection coefficients of its faces' materials, eps_c = eps_r -
 * j sigma / (2 pi f eps0)) is differentiated exactly, the Fresnel coefficients
 * in closed form with respect to eps_c:
 *   dP/dtheta = 2 Re sum_c conj(A_c) dA_c/dtheta,  A = sum_p a_p.
 * Outputs (host, caller-owned, each nullable):
 *   d_eps_r, d_sigma  [n_freqs][n_tx][n_rx][n_materials]: dP/d eps_r and
 *                     dP/d sigma of every material of the scene (zero for a
 *                     constant-gamma material and for materials the paths do
 *                     not reflect on), W per unit and W per S/m;
 *   d_tx_power        [n_freqs][n_tx][n_rx]: dP/dP_t = P / P_t (P is
 *                     proportional to the transmit power);
 *   d_pattern         [n_freqs][n_tx][n_rx][DCEM_PATTERN_TAPS]: dP/dw_j of
 *                     the transmit pattern weights (dcem_set_tx_pattern) at
 *                     the weights the frame was traced with, also for the
 *                     isotropic antenna (w = 1): each path's field is
 *                     g(phi_p) a_p^iso, so dA/dw_j = sum_p B_j(phi_p) a_p^iso.
 * The material derivatives include the pattern's gain.
 * Sums run over each receiver's paths in key order (bitwise reproducible).
 * Waits for the frame; valid until the next dcem_trace_frame, also when the
 * next frame's refit and revalidation have already been started.
 * Errors: DCEM_E_STATE without a traced frame; device errors as for
 * dcem_received_power. */
dcem_status dcem_power_gradients(dcem_ctx* ctx, double* d_eps_r, double* d_sigma, double* d_tx_power,
                                 double* d_pattern);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight calibration loops, harnesses that forbid allocation): the outputs of
 * dcem_power_gradients, computed by the same kernel, with its device
 * workspace in a fixed library-owned array of DCEM_NOALLOC_GRAD_DOUBLES
 * doubles (1 MiB) that each GPU the library runs on holds until the process
 * ends, and the results copied straight into the caller's host arrays (no
 * pinned staging).  Allocates no device or host memory.
 * Limits: (2 * n_materials + DCEM_PATTERN_TAPS) * n_freqs * n_tx * n_rx <=
 * DCEM_NOALLOC_GRAD_DOUBLES, else DCEM_E_UNSUPPORTED; the frame's results
 * must have been read (dcem_received_power after its dcem_trace_frame), else
 * DCEM_E_STATE, since finishing a frame may allocate.  Every call on one GPU
 * shares that GPU's array and overwrites it: calls that overlap on one GPU
 * (from different contexts or threads) race.  Errors otherwise as for
 * dcem_power_gradients; DCEM_E_DEVICE if the array's address could not be
 * obtained at dcem_create. */
#define DCEM_NOALLOC_GRAD_DOUBLES 131072
dcem_status dcem_power_gradients_noalloc(dcem_ctx* ctx, double* d_eps_r, double* d_sigma, double* d_tx_power,
                                         double* d_pattern);

/* Paths of the last frame in key order (tx, rx, order, faces), host memory.
 * keys [cap][3 + K] int32, K = max_reflections + max_transmissions: order =
 * the number of interactions, then one entry per interaction from the
 * transmitter: the face index f for a reflection, -2 - f for a transmission
 * through face f, -1 past the order.
 * valid [cap], length [cap] (m), tau [cap] (s), aod/aoa [cap][3] unit vectors
 * (departure direction at the transmitter; direction from the receiver
 * towards the last path point), amp [cap][n_freqs][3][2] complex field vector
 * (re, im) whose squared norm is the path's received power, first_ray [cap]
 * (lowest ray index (source * n_branch + branch) * n_rays + i that found it,
 * the source being the transmitter, or the receiver when tracing backward; -1
 * for a direct path added by los_always).  Any output pointer may be NULL.
 * n_out receives the number of paths; at most cap are written. */
dcem_status dcem_get_paths(dcem_ctx* ctx, int64_t cap, int32_t* keys, uint8_t* valid, double* length,
                           double* tau, double* aod, double* aoa, double* amp, int32_t* first_ray,
                           int64_t* n_out);

/* Per (source, ray, segment) log of the last frame ([n_src][n_branch *
 * n_rays][K+1], host, K = max_reflections + max_transmissions, rays of branch
 * b at b * n_rays + i; the sources are the transmitters, or the receivers
 * when tracing backward):
 * tri = hit triangle (-1 miss, -2 not reached), t = hit distance along the
 * (unnormalised) direction, length = cumulative path length at the hit.
 * Requires record_trace_log = 1.  Any pointer may be NULL. */
dcem_status dcem_get_trace_log(dcem_ctx* ctx, int32_t* tri, float* t, float* length);

/* Raw capture records of the last frame (host): rows [cap][4 + K] =
 * (ray, source, target, order, faces... padded -1) in the trace's direction
 * (ray = (source * n_branch + branch) * n_rays + i; a transmission through
 * face f is -2 - f):
 * (ray, tx, rx, order, faces from the transmitter), or when tracing from the
 * receivers (ray, rx, tx, order, faces from the receiver); sorted by
 * (source, target, order, faces), then ray. */
dcem_status dcem_get_captures(dcem_ctx* ctx, int64_t cap, int32_t* rows, int64_t* n_out);

/* Current BVH (host): n_internal nodes; child [n][2] (>= 0 internal node,
 * < 0 leaf ~child); box [n][2][6] child boxes (lo xyz, hi xyz); leaf_tri
 * [n_tris] triangle index of each leaf.  Pointers may be NULL to query
 * n_internal. */
dcem_status dcem_get_bvh(dcem_ctx* ctx, int64_t cap_internal, int32_t* n_internal, int32_t* child,
                         float* box, int32_t* leaf_tri);

/* Current world-space vertices [n_vertices][3] (host). */
dcem_status dcem_get_vertices(dcem_ctx* ctx, float* out);

/* Ray directions of the last frame [n_rays][3] (host). */
dcem_status dcem_get_ray_dirs(dcem_ctx* ctx, float* out);

dcem_status dcem_get_stats(dcem_ctx* ctx, dcem_frame_stats* out);

/* ---- Batches: one frame of many scenes at once.
 * Each scene is a context holding its own scene, BVH and caches; a batch
 * traces one frame of every context (the frame algorithm of Sec. III per
 * scene, as dcem_trace_frame) with ONE persistent closest-hit launch for the
 * full traces of all of them: a queue of (scene, chunk of work items) that
 * wavefronts drain, so scenes of very different sizes (ragged triangle
 * counts, transmitters, ray budgets, reflection limits, receivers, bands)
 * keep every compute unit busy to the end.  Contexts in coherent mode trace
 * their own (short) re-trace lists.  Results are per context, read with
 * dcem_received_power / dcem_get_* on each, and equal those of
 * dcem_trace_frame bitwise. */
typedef struct dcem_batch dcem_batch;

/* Launch shape and tuning state of a batch. */
typedef struct dcem_batch_info {
  int32_t n_ctx;
  int32_t lds_stack;       /* per-thread traversal stack entries kept in LDS (16 or 32; the rest in device memory) */
  int32_t blocks_per_cu;   /* persistent blocks of 128 threads per compute unit */
  int32_t chunk;           /* work items per queue chunk */
  int32_t tuned;           /* the shape comes from dcem_batch_tune */
  int32_t graph_frames;    /* frames launched as one captured HIP graph */
  float ms_trace_tuned;    /* batched trace time of the tuned shape (ms, HIP events) */
} dcem_batch_info;

/* A batch over ctxs[0..n) (not copied beyond the pointers; each context must
 * outlive the batch).  All contexts must use one device and one HIP stream.
 * Errors: DCEM_E_INVALID_ARG (null, n < 1, mixed devices or streams, a
 * context twice), DCEM_E_DEVICE. */
dcem_status dcem_batch_create(dcem_batch** out, dcem_ctx* const* ctxs, int32_t n);
void dcem_batch_destroy(dcem_batch* batch);

/* enabled = 1: each batched frame whose device work needs no host round trip
 * (every context on the one-workgroup candidate path, no stage timing) is
 * captured from the stream as one HIP graph and launched with one call; the
 * executable graph is updated in place from frame to frame.  Needs a
 * non-null stream.  Default 0 (direct launches). */
dcem_status dcem_batch_set_graph(dcem_batch* batch, int32_t enabled);

/* Fix the launch shape (see dcem_batch_info): lds_stack 16 or 32,
 * blocks_per_cu 1..32, chunk a positive multiple of 64 up to 2^20.  Results
 * never depend on it.  Default 32, 8, 256. */
dcem_status dcem_batch_set_shape(dcem_batch* batch, int32_t lds_stack, int32_t blocks_per_cu, int32_t chunk);

/* Trace one frame of every context of the batch; params[j] (as for
 * dcem_trace_frame) for context j.  Asynchronous like dcem_trace_frame;
 * errors are those of dcem_trace_frame, reported on the context concerned. */
dcem_status dcem_batch_trace(dcem_batch* batch, const dcem_trace_params* params);

/* Autotuner of the batched trace: traces the batch's frame `repeats` times for
 * each candidate shape (LDS stack 32 with 4, 6 or 8 blocks per compute unit,
 * LDS stack 16 with 4 to 16 blocks, chunk 256; then chunks 64 and 1024 at the
 * best of those), times the batched launch with HIP events, and keeps the
 * fastest shape.  The contexts hold the last traced frame (equal to every
 * other one).  Synchronises. */
dcem_status dcem_batch_tune(dcem_batch* batch, const dcem_trace_params* params, int32_t repeats);

dcem_status dcem_batch_get_info(const dcem_batch* batch, dcem_batch_info* out);

#ifdef __cplusplus
}
#endif
#endif /* DCEM_H */
