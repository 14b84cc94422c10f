// Internal declarations shared by the HIP translation units of libdcem.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dcem.h"

namespace dcem {

constexpr int kWave = 64;
constexpr float kTMin = 1e-4f;           // hits closer than this to a segment start are ignored
constexpr double kTMinD = 1e-4;
constexpr int kStackLds = 32;            // per-thread traversal stack entries kept in LDS
constexpr int kStackSpill = 32;          // further entries per thread in device memory (rarely reached)
constexpr int kStackSize = kStackLds + kStackSpill;
constexpr int kTopNodes = 21;            // 4-wide nodes of the top three levels, kept in LDS
constexpr int kTraceBlock = 128;         // threads per trace block
constexpr uint32_t kNoRay = 0xffffffffu;
constexpr int32_t kTransmit = 1 << 30;   // decoded face entry: the interaction transmits through the face
constexpr int32_t kFaceMask = kTransmit - 1;

// BVH2 internal node, 64 bytes: both child boxes plus links.
//   b0 = (lo0.x, lo0.y, lo0.z, hi0.x)   b1 = (hi0.y, hi0.z, lo1.x, lo1.y)
//   b2 = (lo1.z, hi1.x, hi1.y, hi1.z)   c  = (child0, child1, parent*2+slot, 0)
// child >= 0 is an internal node, child < 0 is leaf ~child; parent -1 at the root.
struct __align__(16) Node {
  float4 b0, b1, b2;
  int4 c;
};

// One child slot of a 4-wide node, 32 bytes: the child's box, the child
// entry (>= 0 node, < 0 leaf ~entry, kEmpty unused) and, for a child node, its
// leaf-slot mask (bit j set: slot j of that child is a leaf).
struct __align__(16) Slot4 {
  float lx, ly, lz;
  int child;
  float hx, hy, hz;
  uint32_t mask;
};

// 4-wide node used by the traversals, 128 bytes.  Built by collapsing every
// other level of the binary tree; nodes are stored in breadth-first order so
// the top of the tree is a prefix of the array.  A traversal that knows a
// node's leaf-slot mask before reading it (from the parent's slot, or the
// tree-info word for the root) can fetch the node and its leaf triangles at
// the same time.
struct __align__(16) Node4 {
  Slot4 s[4];
};
constexpr int kEmpty = (int)0x80000000;

// Stack entry of the group traversals: node index | leaf-slot mask << kNodeBits
// (node indices stay below 2^27: at most 2^27 - 1 triangles).
constexpr int kNodeBits = 27;
constexpr uint32_t kNoEntry = 0xffffffffu;   // no child to push
constexpr int kGroup = 16;                   // lanes per query in the group traversals: one DPP row
constexpr int kGroupStack = 128;             // stack entries per group
constexpr int kRxCols = 64;                  // x columns of the receivers (group re-trace capture test)

// Order LDS accesses of the lanes of one wavefront.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Leaf triangle, 48 bytes: vertices with the triangle id, its face id and 1
// if the face belongs to a moving object (else 0) in the w components (as
// integer bits).  Stored in slot order, [n4][4] with the leaf in slot e of
// 4-wide node q at 4q + e (other slots unused); leaf_slot maps each sorted
// leaf of the binary tree to its slot.
struct __align__(16) Leaf {
  float4 v0, v1, v2;
};

// Packed capture record: ray work item (src * n_rays + position) and
// (src * n_tgt + tgt) << 4 | order, in the trace's direction (source and
// target are the transmitter and receiver, swapped in a backward frame).
struct Capture {
  uint32_t work;
  uint32_t pair_order;
};

// Frame-invariant description of the current trace configuration, used to
// decide whether the coherence cache still applies.
// Transmit field pattern: gain sum_j w[j] B_j(azimuth of the departure
// direction), B_j the periodic hat of half-width 2 pi / 16 centred on azimuth
// 2 pi j / 16.  on == 0: the isotropic antenna (gain 1).  Passed to kernels by
// value, so a launch keeps the weights it was given.
constexpr int kPatternTaps = 16;
struct TxPattern {
  double w[kPatternTaps];
  int on;
};

// The trace side of a frame: rays start at the sources and are captured by
// spheres around the targets (forward: transmitters and receivers; a backward
// frame swaps them).
struct TraceConfig {
  int32_t n_src = 0, n_tgt = 0, K = -1, T = 0;
  bool backward = false;
  bool visited = false;   // candidates by visited-series discovery
  int64_t n_rays = 0;
  float rx_radius = 0.f;
  std::vector<float> src, tgt;
  bool dirs_fib = true;
  const void* dirs_ptr = nullptr;
  std::vector<float> dirs_host;
};

// Where a context's device memory comes from: the caller's allocator
// (dcem_allocator, e.g. a framework's caching allocator) or, without one,
// hipMalloc / hipFree.  Allocations and frees are ordered on `stream`.
struct Allocator {
  dcem_allocator fn{};
  bool user = false;
  hipStream_t stream = nullptr;
};

// Growable device allocation owned by the context (its allocator set when the
// context is created).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const Allocator* al = nullptr;
};

}  // namespace dcem

struct dcem_ctx {
  int device = 0;
  int n_cus = 0;                                     // compute units of the device (0: not queried yet)
  hipStream_t stream = nullptr;
  dcem::Allocator alloc;                             // source of every DevBuf below
  // A refit is enqueued lazily: by the next trace, in one launch with the
  // revalidation pass of a coherent frame (which does not read the tree), or
  // by the first call that reads the tree or the vertices.
  bool refit_pending = false;
  // Going ahead: once a frame's results are in and a refit is pending, the
  // next frame is begun (capture list switched, counters cleared) and its
  // revalidation enqueued with the refit; a coherent trace with the same
  // configuration then starts at the re-trace.
  bool frame_begun = false;
  bool revalidated_ahead = false;
  // the going-ahead launch was enqueued before the last frame's results were
  // read, guarded by that frame's fallback flag (it did nothing if that frame
  // needs its candidates redone)
  bool early_ahead = false;
  // host state before the first early launch, restored when it did nothing
  int early_caps = 0;
  bool early_begun = false;
  bool early_list_clear = false;
  bool list_clear = false;   // kCntList of the current frame block is zero (its last frame's reduction ran)
  bool last_los = true;
  hipEvent_t ev_copy = nullptr;   // the last traced frame's results have reached host_block
  bool copy_pending = false;
  std::string err;
  bool timing = false;
  int64_t cap_capacity = int64_t(1) << 22;
  int32_t stack_limit = 0;   // traversal stack cap (dcem_set_stack_limit); 0 = full depth
  double* scratch = nullptr;  // this device's fixed gradient workspace (dcem_power_gradients_noalloc)

  // -- scene
  bool has_scene = false;
  int64_t nv = 0, nt = 0;
  int32_t nf = 0, nm = 0, no = 0;
  float pad = 0.f;          // absolute padding of leaf boxes (conservative traversal)
  dcem::DevBuf ref_vertices, vertices, tris, tri_face, face_material, face_object, materials,
      obj_range, face_tri_off, face_tris, face_ref_tri, xf, obj_box, face_plane;
  // per entry of face_tris: the slot of that triangle in the slot triangle
  // array (set by each build), so the refinement's face test reads the
  // vertices the tree holds (the refit's, not a later transform's)
  dcem::DevBuf tri_slot, face_slots;
  std::vector<int32_t> h_face_object, h_face_material;
  // penetration loss per material in dB (+inf: opaque), for the next traced
  // frame (dcem_set_penetration_loss); uploaded as per-face flags and
  // per-material amplitude factors
  std::vector<double> pen_next;
  bool pen_pending = false;
  dcem::DevBuf face_pen, mat_pen;   // uint8 [n_faces] 1 = penetrable; double [n_materials] 10^(-dB/20)

  // -- BVH
  bool has_bvh = false;
  int32_t n_internal = 0;
  double sah_build = 0.0, sah_last = 1.0;
  int32_t last_rebuilt = 0;
  int32_t last_trace_kernel = 0;                     // traversal of the last frame (0 per thread, 1 per wavefront)
  dcem::DevBuf nodes, leaf_slot, leaf_tri, leaf_parent, refit_cnt, morton, sort_tmp, sah_part, scene_box,
      node_range;
  dcem::DevBuf nodes4, bvh2_of4, map4, depth_key;   // 4-wide tree and its mapping from the binary one
  dcem::DevBuf slot4;                                // per binary child slot: the 4-wide slot holding its box, or -1
  dcem::DevBuf cross;                                // refit: nodes spanning refit blocks (index, list, parents, slots)
  dcem::DevBuf tree_info;                            // uint32 [0]: 4-wide nodes, [1]: root leaf-slot mask,
                                                     // [2]: cross nodes, [3], [4]: refit list length and block ticket
  dcem::DevBuf tri4;                                 // leaf triangles in slot order (Leaf [n4][4])
  dcem::DevBuf face_build;                           // build scratch: face boxes, keys, order and ranks
  int face_bits = 0;                                 // bits of a face's rank among its group's faces
  // the last full build's keys (in `morton`): grouped by object, and their layout
  bool keys_grouped = false;
  int key_words_built = 1, key_rank_bits = 0, key_face_bits = 0;
  double subtree_ratio = 1.0;                        // SAH of the last build relative to the last full build

  // -- rays and cache
  dcem::TraceConfig cfg;
  bool cache_valid = false;
  bool geometry_moved = true;   // transforms changed since the cached frame
  // ray origins and capture-sphere centres of the trace (transmitters and
  // receivers; receivers and transmitters in a backward frame)
  int32_t n_src = 0, n_tgt = 0;
  bool backward = false;
  // rx_nodes, rx_cols: the capture spheres (the targets) as a tree and by x column
  dcem::DevBuf dirs, ray_order, src_pos, tgt_pos, freqs, rx_nodes;
  // targets ordered by x column: [n_tgt] float4 (x, y, z, target index
  // bits), then kRxCols + 1 int32 column starts; column of x:
  // clamp(floor((x - rx_col_x0) * rx_col_scale), 0, kRxCols - 1)
  dcem::DevBuf rx_cols;
  dcem::DevBuf grad_buf;   // power gradients: [2][freq][pair][material], then [freq][pair][16]
  void* grad_host = nullptr;   // pinned copy of grad_buf, read back in one transfer
  size_t grad_host_bytes = 0;
  float rx_col_x0 = 0.0f, rx_col_scale = 0.0f;
  std::vector<double> freqs_host;
  int32_t n_rx_nodes = 0;
  dcem::DevBuf face_log;     // [K+1][n_work] int32 face hit per bounce (-1 miss)
  dcem::DevBuf ray_state;    // [n_work] uint8: segments (low 4 bits), bit 7 = hit a moving face
  dcem::DevBuf seg_o, seg_d; // [K+1][n_work] float4: origin + t_end, direction
  dcem::DevBuf log_tri, log_t, log_len;  // parity log [n_work][K+1]
  dcem::DevBuf caps[2];      // double-buffered capture lists
  int cur_caps = 0;
  dcem::DevBuf work_list, invalid_flag;   // re-trace list; per-ray first invalid segment (255 = valid)
  dcem::DevBuf stack_spill;  // per-thread traversal stack entries beyond the LDS part (kStackSpill each)
  // One device block holding everything the host reads after a frame, copied
  // in one transfer to pinned host memory: counters (128 B), error word
  // (128 B), SAH values (256 B), then p_coh and p_inc.
  dcem::DevBuf frame_block;
  void* host_block = nullptr;
  size_t host_block_bytes = 0;
  int64_t n_pow_cap = 0;
  uint32_t* cnt_dev = nullptr;
  uint32_t* err_dev = nullptr;
  double* sah_dev = nullptr;     // SAH sums: [0] of the last build, [1] of the last refit, [2] of the last full build
  double* pcoh_dev = nullptr;
  double* pinc_dev = nullptr;
  uint32_t last_cnt[32] = {};    // counters as of the last synchronisation
  bool counts_current = false;   // last_cnt reflects the last traced frame
  bool refit_since_build = false;
  double pending_ratio = 1.0;    // quality ratio measured after the last refit
  bool refit_pending_timing = false;

  // -- candidates / paths
  // n_tx, n_rx: the paths' transmitters and receivers (either direction).
  // K: interactions per path at most (max_reflections + max_transmissions),
  // the length of every face sequence; max_refl, max_trans: the two limits.
  // A ray is traced once per branch (n_branch; branch_set holds each
  // branch's set of interaction indices that transmit, bit j = interaction j).
  int32_t key_words = 0, K = 0, n_freqs = 0, n_tx = 0, n_rx = 0;
  int32_t max_refl = 0, max_trans = 0, n_branch = 1;
  dcem::DevBuf branch_set;
  int64_t n_rays = 0;
  int bits_tx = 0, bits_rx = 0, bits_face = 0;
  dcem::DevBuf cand_keys, cand_perm, cand_tmp, uniq_idx, first_ray;
  dcem::DevBuf path_valid, path_len, path_tau, path_aod, path_aoa, path_amp;
  dcem::DevBuf pair_range, path_order, path_faces, path_pts;
  int64_t key_stride = 1;        // stride of the candidate key words
  int64_t path_cap = 0;          // bound on the number of unique paths of the frame
  bool small_path = false;       // candidates de-duplicated without a host round trip
  dcem::DevBuf sort_hist;
  // visited-series discovery: the sorted unique series (source, order, faces,
  // lowest ray) with per-source starts, and the expansion's survivor masks
  bool visited = false;
  dcem::DevBuf series_buf, expand_buf;
  int64_t n_caps_host = 0;
  double sqrt_pt = 0.0, atten_db_per_km = 0.0;
  // transmit pattern: the weights of the next traced frame, and those the
  // last traced frame used (its paths' fields, and its gradients)
  dcem::TxPattern pattern_next{}, pattern_frame{};
  // material table set after the scene upload, uploaded by the next traced frame
  std::vector<double> mat_next;
  bool mat_pending = false;
  bool bvh_stale = false;     // transforms changed since the last refit
  bool has_frame = false;
  int32_t record_log = 0;
  dcem_frame_stats stats{};
  hipEvent_t ev[9] = {};   // stage boundaries of a frame (timing on): see dcem_get_stats

  // Every device buffer of the context (given its allocator at creation,
  // released at destruction).
  std::vector<dcem::DevBuf*> buffers() {
    return {&ref_vertices, &vertices, &tris, &tri_face, &face_material, &face_object, &materials, &obj_range,
            &face_tri_off, &face_tris, &face_ref_tri, &xf, &obj_box, &face_plane, &tri_slot, &face_slots,
            &nodes, &leaf_slot, &leaf_tri, &leaf_parent, &refit_cnt, &morton, &sort_tmp, &sah_part, &scene_box,
            &node_range, &nodes4, &bvh2_of4, &map4, &depth_key, &slot4, &cross, &tree_info, &tri4, &face_build,
            &dirs, &ray_order, &src_pos, &tgt_pos, &freqs, &rx_nodes, &rx_cols, &grad_buf, &face_log, &ray_state,
            &seg_o, &seg_d, &log_tri, &log_t, &log_len, &caps[0], &caps[1], &work_list, &invalid_flag, &stack_spill,
            &frame_block, &cand_keys, &cand_perm, &cand_tmp, &uniq_idx, &first_ray, &path_valid, &path_len,
            &path_tau, &path_aod, &path_aoa, &path_amp, &pair_range, &path_order, &path_faces, &path_pts,
            &sort_hist, &series_buf, &expand_buf, &face_pen, &mat_pen, &branch_set};
  }
};

namespace dcem {

// counters in ctx->counters
enum : int {
  kCntCaptures = 0,   // capture records in the current list
  kCntWork = 1,       // work items to trace
  kCntQueue = 2,      // persistent-thread queue head
  kCntUnique = 3,     // unique candidates
  kCntSegments = 4,   // closest-hit queries executed
  kCntValid = 5,      // valid paths
  kCntNodes = 6,      // BVH nodes visited by the trace kernel (64-bit, slots 6-7)
  kCntTris = 8,       // triangle tests of the trace kernel (64-bit, slots 8-9)
  kCntFallback = 10,  // the small de-duplication path saw more captures than it holds
  kCntList = 11,      // rays the revalidation listed for the re-trace (the trace copies it to kCntWork);
                      // zeroed at the end of each frame, so the next frame's revalidation may start
                      // before that frame's other counters are reset
  kCntSlots = 12,     // number of counter words cleared per frame
};

hipError_t ensure(DevBuf& b, size_t bytes);
void release(DevBuf& b);
// Set n 32-bit words at p to v on stream s (a kernel: no memset node, so the
// work can be captured in a graph).
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);

template <class T>
T* ptr(DevBuf& b) { return static_cast<T*>(b.p); }

// ---- launchers (bvh.hip)
// Transform the moving objects' vertices by xf ([n_objects][3][4], device).
void launch_xform(dcem_ctx* c, const float* xf);
// Build the binary and 4-wide trees.  `separate_objects`: every moving object
// (and the static geometry) in a subtree of its own, for a tree that will be
// refitted; otherwise one Morton order over all triangles.
hipError_t build_lbvh(dcem_ctx* c, bool separate_objects);
// Rebuild the part of the tree above the groups (the static geometry and each
// moving object): the groups are ordered again by their current centres and
// every group's subtree keeps its structure (its triangles keep their keys
// below the group prefix).  Needs a last full build with separated objects,
// else does one.
hipError_t rebuild_subtrees(dcem_ctx* c);
// Refit the binary tree (`wide`: and the 4-wide tree in place, no collapse
// needed), write the SAH ratio to sah_out and the face planes.
void launch_refit(dcem_ctx* c, bool wide, double* sah_out);
void launch_collapse(dcem_ctx* c);

// ---- radix sort (sort.hip)
// Stable LSD sort of n items by `bits` low bits of a multi-word key stored
// word-major ([W][stride], word W-1 least significant; stride -1: n_max),
// producing a permutation.  The item count is min(*n_dev, n_max), read on the
// device.  Only the low `low_bits` bits of word W-1 are sorted on (the others
// are zero in every key).
hipError_t radix_sort_perm(dcem_ctx* c, const uint32_t* keys, int W, int bits, const uint32_t* n_dev,
                           int64_t n_max, uint32_t* perm, uint32_t* perm_tmp, hipStream_t s, int64_t stride = -1,
                           int low_bits = 32);
// The sort's histogram space for up to n_max items (sized before a frame that
// a graph may capture).
hipError_t prepare_sort(dcem_ctx* c, int64_t n_max);

// ---- trace (trace.hip)
void launch_fibonacci(dcem_ctx* c);
// Trace all rays, or (coherent frame) the listed ones after keeping the
// previous frame's still-valid captures.  Returns the traversal launched:
// 0 one thread per ray, 1 one group of lanes per ray; -1 when its stack
// space could not be allocated (nothing launched).
int launch_trace(dcem_ctx* c, bool all_rays, bool keep_cache, int64_t expected, uint32_t n_prev_caps);
void launch_coherence(dcem_ctx* c);
// Coherent frame with moved receivers: captures of the kept segments of every
// cached ray against the current receivers (after the revalidation pass).
void launch_recapture(dcem_ctx* c);
// The pending refit of the 4-wide tree and the revalidation pass in one launch
// (skip, nullable: a device word that, nonzero at launch, cancels the launch).
void launch_refit_coherence(dcem_ctx* c, bool begin, const uint32_t* skip = nullptr);
// Clear the frame counters and seed the capture list with the LoS candidates.
void launch_frame_begin(dcem_ctx* c, bool los, const uint32_t* skip = nullptr);
hipError_t build_ray_order(dcem_ctx* c);
// Buffers a frame's trace needs (the per-thread stack's spill space), sized
// before anything of the frame is enqueued.
hipError_t prepare_trace(dcem_ctx* c);
// Launch configuration of a batched trace (several contexts' full frames in
// one persistent launch): per-thread stack entries kept in LDS, blocks per
// compute unit, work items per queue chunk.
struct BatchShape {
  int lds_stack = 32;
  int blocks_per_cu = 8;
  int chunk = 256;
};
// Bytes of spill space a batched trace of this shape needs.
size_t batch_spill_bytes(const dcem_ctx* c, const BatchShape& shape);
// One persistent launch tracing every ray of the given contexts (full frames
// on one stream; keep_cache[j]: context j stores its segment cache).  `table`
// holds the per-context arguments and the chunk table (staged through pinned
// `host_table`), `spill` the stack spill space.
hipError_t launch_trace_batch(dcem_ctx* const* cs, const uint8_t* keep_cache, int n, const BatchShape& shape,
                              DevBuf& table, void* host_table, size_t host_table_bytes, DevBuf& spill, hipStream_t s);
size_t batch_table_bytes(int n);

// ---- candidates, refinement and accumulation (refine.hip)
hipError_t build_candidates(dcem_ctx* c, bool small, int64_t hint = 0);
// Buffers of the sort-based de-duplication sized for n captures.
hipError_t prepare_sorted_candidates(dcem_ctx* c, int64_t n);
// Visited-series discovery: every distinct series of faces the frame's rays
// reflect on (per source, up to K), tried against every target; the
// candidates whose image-method points lie inside their segments and faces
// become the frame's paths (host round trips for the counts).
hipError_t build_visited_candidates(dcem_ctx* c, bool los, bool& too_many);
// Buffers of the one-workgroup de-duplication path and of its paths.
hipError_t prepare_small_candidates(dcem_ctx* c);
bool small_path_fits(const dcem_ctx* c);
int64_t small_path_capacity();
hipError_t ensure_paths(dcem_ctx* c, int64_t n);
void launch_refine(dcem_ctx* c);
void launch_reduce(dcem_ctx* c);
void launch_power_grad(dcem_ctx* c, uint32_t n_unique, double* g_eps, double* g_sig, double* g_pat);

}  // namespace dcem
