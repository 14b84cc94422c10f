// Ray shooting: Fibonacci ray sphere, closest-hit BVH traversal with a
// watertight ray-triangle test, receiver-sphere capture and specular
// reflection, plus the frame-to-frame coherence pass.
//
// Paper, Sec. III: the frame algorithm casts a sphere of sampled rays (step 1)
// and records their reflections up to a bounce limit (step 2; at most 10);
// propagation-path caching re-checks the previous frame's paths at the start
// of each frame so that fewer rays are cast.  Here a ray is reused unchanged
// when none of its segments can meet moved geometry; only the others are
// traced again, which reproduces the full re-trace exactly.
#include "dcem_internal.h"
#include "refit.h"

#include <cfloat>

namespace dcem {
namespace {

__device__ inline float comp(const float3& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

__device__ inline uint32_t ordered_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

struct Ray {
  float3 o, d, inv;   // origin, direction (not normalised), 1 / direction (zeros replaced)
  float sx, sy, sz;   // shear constants of the watertight test
  int kx, ky, kz;     // axis permutation of the watertight test
};

__device__ inline void setup_ray(Ray& r) {
  const float ax = fabsf(r.d.x), ay = fabsf(r.d.y), az = fabsf(r.d.z);
  int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(r.d, kz) < 0.0f) { int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  const float tiny = 1e-30f;
  r.inv = make_float3(__fdiv_rn(1.0f, r.d.x != 0.0f ? r.d.x : tiny), __fdiv_rn(1.0f, r.d.y != 0.0f ? r.d.y : tiny),
                      __fdiv_rn(1.0f, r.d.z != 0.0f ? r.d.z : tiny));
  // shear constants from the reciprocal of the dominant component (never
  // zero for a nonzero direction): one division per axis in all
  r.sz = comp(r.inv, kz);
  r.sx = comp(r.d, kx) * r.sz;
  r.sy = comp(r.d, ky) * r.sz;
}

// Watertight ray-triangle intersection (Woop, Benthin and Wald, JCGT 2013):
// vertices are translated to the ray origin and sheared so the ray runs along
// +z; the 2D edge functions decide the hit, with an FP64 re-evaluation when
// one is exactly zero.  Edge functions are evaluated without FMA contraction
// so that two triangles sharing an edge compute exactly opposite values.
// Returns the hit distance t (IEEE division) or -1.  The axis permutation is
// read through a policy: the ray's axis indices (per-thread traversal) or
// per-lane select masks precomputed once per segment (group traversal); the
// arithmetic is the same.
struct RayAxes {
  int kx, ky, kz;
  __device__ float x(const float3& v) const { return comp(v, kx); }
  __device__ float y(const float3& v) const { return comp(v, ky); }
  __device__ float z(const float3& v) const { return comp(v, kz); }
};

// Component selection by bit masks (all ones for the chosen component), so
// that lanes tracing different rays need no branches.
struct MaskAxes {
  uint32_t x0, x1, x2, y0, y1, y2, z0, z1, z2;
  __device__ static float pick(const float3& v, uint32_t m0, uint32_t m1, uint32_t m2) {
    return __uint_as_float((__float_as_uint(v.x) & m0) | (__float_as_uint(v.y) & m1) | (__float_as_uint(v.z) & m2));
  }
  __device__ float x(const float3& v) const { return pick(v, x0, x1, x2); }
  __device__ float y(const float3& v) const { return pick(v, y0, y1, y2); }
  __device__ float z(const float3& v) const { return pick(v, z0, z1, z2); }
};

template <class Axes>
__device__ inline float watertight_axes(const Ray& r, const Axes& ax, const float4& p0, const float4& p1,
                                        const float4& p2) {
#pragma clang fp contract(off)
  const float3 A = make_float3(p0.x - r.o.x, p0.y - r.o.y, p0.z - r.o.z);
  const float3 B = make_float3(p1.x - r.o.x, p1.y - r.o.y, p1.z - r.o.z);
  const float3 C = make_float3(p2.x - r.o.x, p2.y - r.o.y, p2.z - r.o.z);
  const float Az = ax.z(A), Bz = ax.z(B), Cz = ax.z(C);
  const float Ax = ax.x(A) - r.sx * Az, Ay = ax.y(A) - r.sy * Az;
  const float Bx = ax.x(B) - r.sx * Bz, By = ax.y(B) - r.sy * Bz;
  const float Cx = ax.x(C) - r.sx * Cz, Cy = ax.y(C) - r.sy * Cz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return -1.0f;
  const float det = U + V + W;
  if (det == 0.0f) return -1.0f;
  const float T = U * (r.sz * Az) + V * (r.sz * Bz) + W * (r.sz * Cz);
  return __fdiv_rn(T, det);
}

__device__ inline float watertight(const Ray& r, const float4& p0, const float4& p1, const float4& p2) {
  return watertight_axes(r, RayAxes{r.kx, r.ky, r.kz}, p0, p1, p2);
}

// Conservative slab test against a box given as (lo, hi) over (t0, tmax].
__device__ inline bool slab(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz, float tmax,
                            float& tnear) {
  const float ox = r.o.x * r.inv.x, oy = r.o.y * r.inv.y, oz = r.o.z * r.inv.z;
  const float ax = fmaf(lx, r.inv.x, -ox), bx = fmaf(hx, r.inv.x, -ox);
  const float ay = fmaf(ly, r.inv.y, -oy), by = fmaf(hy, r.inv.y, -oy);
  const float az = fmaf(lz, r.inv.z, -oz), bz = fmaf(hz, r.inv.z, -oz);
  const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
  const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tmax));
  tnear = tn;
  return tn <= tf * 1.0000004f;
}

struct Hit {
  float t;
  int tri;    // original triangle id, -1 none
  int leaf;   // slot of the triangle in the slot triangle array, -1 none
  int face;
};

__device__ inline void test_leaf(const Ray& r, const Leaf* __restrict__ tri4, int li, int excl, Hit& h) {
  const float4 p0 = tri4[li].v0, p1 = tri4[li].v1, p2 = tri4[li].v2;
  const int face = __float_as_int(p1.w);
  if (face == excl) return;
  const float t = watertight(r, p0, p1, p2);
  if (!(t > kTMin)) return;
  const int tri = __float_as_int(p0.w);
  if (t < h.t || (t == h.t && tri < h.tri)) {
    h.t = t;
    h.tri = tri;
    h.leaf = li;
    h.face = face;
  }
}

__device__ inline void cswap(float& ta, int& ca, float& tb, int& cb) {
  if (tb < ta) {
    const float t = ta; ta = tb; tb = t;
    const int c = ca; ca = cb; cb = c;
  }
}

// Per-thread traversal stack: the first kStackLds entries in LDS (strided by
// the block size), deeper ones in this thread's region of device memory.  A
// 4-wide traversal pushes at most three entries per level, so the spill part
// is reached only by rays in unusually deep parts of a tree.
struct ThreadStack {
  int* lds;
  int* spill;           // this thread's first spill entry
  size_t spill_stride;  // threads of the grid
  int cap;              // entries usable (<= kStackSize)
  int lds_entries = kStackLds;
  __device__ void put(int i, int v) {
    if (i < lds_entries) lds[i * kTraceBlock] = v;
    else spill[(size_t)(i - lds_entries) * spill_stride] = v;
  }
  __device__ int get(int i) const {
    return i < lds_entries ? lds[i * kTraceBlock] : spill[(size_t)(i - lds_entries) * spill_stride];
  }
};

typedef __attribute__((address_space(3))) const Node4 LdsNode4;      // a node in LDS
typedef __attribute__((address_space(1))) const Node4 GlobalNode4;   // a node in device memory
// Node i of an array known to live in LDS / in device memory (address-space
// casts need C-style casts).
__device__ inline Node4 node_in_lds(const Node4* a, int i) { return *(const Node4*)((const LdsNode4*)a + i); }
__device__ inline Node4 node_in_memory(const Node4* a, int i) { return *(const Node4*)((const GlobalNode4*)a + i); }

// Closest hit: lexicographic minimum of (t, triangle id) over all triangles
// with t > t_min outside face `excl`, by a stack traversal of the 4-wide tree
// (nearest child first; the top levels are read from LDS).  The result does
// not depend on the tree shape: boxes are conservative and nodes are pruned
// only when their entry distance exceeds the current best (ties are visited).
__device__ Hit closest_hit(const Ray& r, const Node4* __restrict__ nodes, const Node4* top, int n_top, int n4,
                           const Leaf* __restrict__ tri4, int excl, ThreadStack& stack, bool& overflow,
                           uint32_t& n_nodes, uint32_t& n_tris) {
  Hit h{FLT_MAX, -1, -1, -1};
  if (n4 == 0) return h;
  int node = 0, sp = 0;
  // a sound tree visits each node at most once per query; the bound only
  // guarantees termination
  for (int64_t guard = (int64_t)n4 + 2;; --guard) {
    if (guard == 0) { overflow = true; break; }
    // read through address-space-typed pointers, in two branches: a select
    // of the two pointers would make every node read a generic load that
    // waits on both the LDS and the memory counters
    Node4 nd;
    if (node < n_top) nd = node_in_lds(top, node);
    else nd = node_in_memory(nodes, node);
    if (node >= n_top) ++n_nodes;   // fetched from memory (the top levels sit in LDS)
    float t[4];
    int c[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      t[e] = INFINITY;
      c[e] = kEmpty;
      const Slot4& sl = nd.s[e];
      const int ch = sl.child;
      if (ch == kEmpty) continue;
      float tn;
      if (!slab(r, sl.lx, sl.ly, sl.lz, sl.hx, sl.hy, sl.hz, h.t, tn)) continue;
      if (ch < 0) {
        test_leaf(r, tri4, 4 * node + e, excl, h);
        ++n_tris;
      } else {
        t[e] = tn;
        c[e] = ch;
      }
    }
    cswap(t[0], c[0], t[1], c[1]);
    cswap(t[2], c[2], t[3], c[3]);
    cswap(t[0], c[0], t[2], c[2]);
    cswap(t[1], c[1], t[3], c[3]);
    cswap(t[1], c[1], t[2], c[2]);
    if (c[0] == kEmpty) {
      if (sp == 0) break;
      node = stack.get(--sp);
      continue;
    }
#pragma unroll
    for (int e = 3; e >= 1; --e) {
      if (c[e] == kEmpty) continue;
      if (sp < stack.cap) stack.put(sp++, c[e]);
      else overflow = true;
    }
    node = c[0];
  }
  return h;
}

// Fibonacci sphere in FP64, plain evaluation (no fused multiply-add), rounded to FP32.
__global__ void k_fibonacci(float* __restrict__ dirs, int64_t n) {
#pragma clang fp contract(off)
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double golden = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  const double z = 1.0 - (2.0 * (double)i + 1.0) / (double)n;
  const double rho = sqrt(1.0 - z * z);
  const double phi = (double)i * golden;
  double s, c;
  sincos(phi, &s, &c);
  dirs[3 * i] = (float)(rho * c);
  dirs[3 * i + 1] = (float)(rho * s);
  dirs[3 * i + 2] = (float)z;
}

struct TraceArgs {
  const Node4* nodes4;
  const Leaf* tri4;           // leaf triangles in slot order
  const uint32_t* n4_dev;     // number of 4-wide nodes (null: empty scene)
  const float* dirs;
  const uint32_t* ray_order;  // traversal position -> ray (directions sorted along a space-filling curve);
                              // per-ray device state is indexed by position: neighbouring directions share
                              // cache lines
  // ray origins [n_src][3] and capture-sphere centres [n_rx][3]: the
  // transmitters and receivers, or in a backward frame the receivers and
  // transmitters (records then name (receiver, transmitter) pairs)
  const float* tx;
  const float* rx;
  int n_rx;
  int capture;          // 0: no capture tests (candidates come from the visited series)
  const Node* rx_nodes; // BVH over the capture spheres (boxes padded), leaves = sphere ids
  int n_rx_nodes;
  float r2;
  float rx_zlo, rx_zhi; // z range of all capture spheres
  float rx_cull;        // xy margin of the group kernel's receiver cull (radius plus slack)
  const float4* rx_cols;      // receivers by x column, then the column starts (see dcem_ctx::rx_cols)
  float rx_col_x0, rx_col_scale;
  const uint8_t* restart;     // work-list mode: first segment to trace again
  int64_t n_rays;             // rays per source and branch
  int n_work;
  const uint32_t* work_list;  // null: all work items
  int K;                      // interactions at most (segments 0..K)
  // Transmission (the "Reflected and transmitted rays" item of Sec. III):
  // each ray is traced once per branch; branch b transmits at the
  // interactions in branch_set[b] (bit j: interaction j) and reflects at the
  // others, at most max_refl times.  Work item (src, b, position) is
  // (src * n_branch + b) * n_rays + position.  A branch stops where it would
  // transmit through a face that is not penetrable (face_pen[face] == 0).
  int max_refl;
  int n_branch;
  const uint32_t* branch_set;
  const uint8_t* face_pen;
  const int32_t* face_object;
  uint32_t* counters;
  int32_t* face_log;          // [K+1][n_work]
  uint8_t* ray_state;         // [n_work]
  float4* seg_o;              // [K+1][n_work] or null
  float4* seg_d;
  int32_t* log_tri;           // [n_work][K+1] or null
  float* log_t;
  float* log_len;
  Capture* caps;
  int64_t cap_capacity;
  uint32_t* err;
  const Capture* prev_caps;   // coherent frames: the previous frame's captures to filter
  uint32_t n_prev;
  int* stack_spill;           // [kStackSpill][grid threads] per-thread stack entries beyond the LDS part
  int stack_thread;           // stack entries a per-thread traversal may use (<= kStackSize)
  int stack_group;            // stack entries a group traversal may use (<= kRayStack)
};

// Coherent frames: keep each capture of the previous frame made before its
// ray's first re-traced segment (those after it are found again by the
// re-trace).  Appended with one atomic per wavefront; run by every block of
// the trace kernel, block b taking the records of position `blk` (b, or the
// blocks in reverse order when the last blocks of the launch trace nothing).
__device__ void keep_previous_captures(const TraceArgs& a, bool& cap_over, uint32_t blk) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blk * blockDim.x + (threadIdx.x - lane); base < a.n_prev; base += stride) {
    const uint32_t i = base + lane;
    bool keep = false;
    Capture c{};
    if (i < a.n_prev) {
      c = a.prev_caps[i];
      keep = c.work != kNoRay && (c.pair_order & 15u) < a.restart[c.work];
    }
    const uint64_t m = __ballot(keep);
    uint32_t b = 0;
    if (lane == 0 && m) b = atomicAdd(&a.counters[kCntCaptures], (uint32_t)__popcll(m));
    b = __shfl(b, 0);
    if (keep) {
      const uint32_t slot = b + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (slot < a.cap_capacity) a.caps[slot] = c;
      else cap_over = true;
    }
  }
}

// Per-segment arithmetic shared by both trace kernels.  Contraction into fused
// multiply-adds is disabled (fused operations are written out) so that every
// kernel computes bitwise the same values: a reused ray must equal a re-traced one.

// Capture test of one segment [o, o + tend d] against one sphere: closest
// approach of the segment to the centre within the radius (FP32).
__device__ inline bool captured(const Ray& r, float tend, float dd, float cx, float cy, float cz, float r2) {
#pragma clang fp contract(off)
  const float wx = cx - r.o.x, wy = cy - r.o.y, wz = cz - r.o.z;
  float s = __fdiv_rn(wx * r.d.x + wy * r.d.y + wz * r.d.z, dd);
  s = fminf(fmaxf(s, 0.0f), tend);
  const float px = fmaf(s, r.d.x, -wx), py = fmaf(s, r.d.y, -wy), pz = fmaf(s, r.d.z, -wz);
  return px * px + py * py + pz * pz <= r2;
}

__device__ inline float dot_dd(const Ray& r) {
#pragma clang fp contract(off)
  return r.d.x * r.d.x + r.d.y * r.d.y + r.d.z * r.d.z;
}

// Specular reflection off the plane of triangle (p0, p1, p2) at parameter t.
__device__ inline void reflect_ray(Ray& r, float t, const float4& p0, const float4& p1, const float4& p2) {
#pragma clang fp contract(off)
  const float ex = p1.x - p0.x, ey = p1.y - p0.y, ez = p1.z - p0.z;
  const float fx = p2.x - p0.x, fy = p2.y - p0.y, fz = p2.z - p0.z;
  float nx = ey * fz - ez * fy, ny = ez * fx - ex * fz, nz = ex * fy - ey * fx;
  const float rl = __fdiv_rn(1.0f, __fsqrt_rn(nx * nx + ny * ny + nz * nz));
  nx = nx * rl;
  ny = ny * rl;
  nz = nz * rl;
  const float dn2 = 2.0f * (r.d.x * nx + r.d.y * ny + r.d.z * nz);
  r.o = make_float3(__fmaf_rn(t, r.d.x, r.o.x), __fmaf_rn(t, r.d.y, r.o.y), __fmaf_rn(t, r.d.z, r.o.z));
  r.d = make_float3(r.d.x - dn2 * nx, r.d.y - dn2 * ny, r.d.z - dn2 * nz);
  setup_ray(r);
}

// Continue straight on from the hit at parameter t (transmission), with the
// origin computed as a reflection computes it.
__device__ inline void transmit_ray(Ray& r, float t) {
  r.o = make_float3(__fmaf_rn(t, r.d.x, r.o.x), __fmaf_rn(t, r.d.y, r.o.y), __fmaf_rn(t, r.d.z, r.o.z));
  setup_ray(r);
}

// Captures of one segment [o, o + tend d] (tend infinite on a miss; th its
// hit distance): receivers whose padded box the segment meets, by the
// receiver tree, then the exact closest-approach test; records appended to
// the frame's capture list.
__device__ void capture_segment(const TraceArgs& a, const Ray& r, bool hit, float th, float tend, float dd,
                                uint32_t work, uint32_t txi, int k, ThreadStack& stack, bool& overflow,
                                bool& cap_over) {
  if (!a.capture) return;
  const float za = r.o.z;
  const float zb = hit ? __fmaf_rn(th, r.d.z, r.o.z) : (r.d.z > 0 ? INFINITY : (r.d.z < 0 ? -INFINITY : r.o.z));
  if (fmaxf(za, zb) >= a.rx_zlo && fminf(za, zb) <= a.rx_zhi) {
    int node = 0, sp = 0;
    for (int guard = 2 * a.n_rx_nodes + 2; guard > 0; --guard) {
      const Node nd = a.rx_nodes[node];
      float t0, t1;
      bool h0 = slab(r, nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y, tend, t0);
      bool h1 = slab(r, nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w, tend, t1);
      const int c0 = nd.c.x, c1 = nd.c.y;
      for (int side = 0; side < 2; ++side) {
        const int cc = side ? c1 : c0;
        const bool hh = side ? h1 : h0;
        if (!(hh && cc < 0) || (side == 1 && c1 == c0)) continue;   // a lone sphere fills both slots
        const int c = ~cc;
        if (captured(r, tend, dd, a.rx[3 * c], a.rx[3 * c + 1], a.rx[3 * c + 2], a.r2)) {
          const uint32_t slot = atomicAdd(&a.counters[kCntCaptures], 1u);
          if (slot < a.cap_capacity) {
            Capture cp;
            cp.work = work;
            cp.pair_order = ((txi * (uint32_t)a.n_rx + (uint32_t)c) << 4) | (uint32_t)k;
            a.caps[slot] = cp;
          } else {
            cap_over = true;
          }
        }
      }
      h0 = h0 && c0 >= 0;
      h1 = h1 && c1 >= 0;
      if (h0 && h1) {
        if (sp < stack.cap) stack.put(sp++, c1);
        else overflow = true;
        node = c0;
      } else if (h0) {
        node = c0;
      } else if (h1) {
        node = c1;
      } else {
        if (sp == 0) break;
        node = stack.get(--sp);
      }
    }
  }
}

// Per-thread tracing of one work item (a ray, from its first segment or, in
// work-list mode, from its restart segment): closest hits, captures,
// reflections, the per-bounce face log and segment cache.
struct ItemCounts {
  uint32_t seg = 0, node = 0, tri = 0;
  bool overflow = false, cap_over = false;
};

__device__ void trace_item(const TraceArgs& a, uint32_t wi, const Node4* top, int n_top, int n4, ThreadStack& stack,
                           ItemCounts& ic) {
  uint32_t& seg_count = ic.seg;
  uint32_t& node_count = ic.node;
  uint32_t& tri_count = ic.tri;
  bool& overflow = ic.overflow;
  bool& cap_over = ic.cap_over;
  // work: the ray's traversal position (its index in the face log, the
  // caches and the capture records); rid: its ray id (the parity log)
  const uint32_t work = a.work_list ? a.work_list[wi] : wi;
  const uint32_t vsrc = (uint32_t)(work / (uint64_t)a.n_rays);   // src * n_branch + branch
  const uint32_t ray = a.ray_order[work - (uint64_t)vsrc * a.n_rays];
  const uint32_t rid = vsrc * (uint32_t)a.n_rays + ray;
  const uint32_t txi = vsrc / (uint32_t)a.n_branch;
  // the branch's transmitting interactions; segments up to its last one are
  // those of the branch without it, which records their captures
  const uint32_t tset = a.branch_set[vsrc - txi * (uint32_t)a.n_branch];
  const int last_t = tset ? 31 - __builtin_clz(tset) : -1;
  int k = a.restart ? (int)a.restart[work] : 0;
  Ray r;
  int excl = -1;
  float L = 0.0f;
  if (k == 0) {
    r.o = make_float3(a.tx[3 * txi], a.tx[3 * txi + 1], a.tx[3 * txi + 2]);
    r.d = make_float3(a.dirs[3 * ray], a.dirs[3 * ray + 1], a.dirs[3 * ray + 2]);
  } else {
    const float4 so = a.seg_o[(size_t)k * a.n_work + work];
    const float4 sd = a.seg_d[(size_t)k * a.n_work + work];
    r.o = make_float3(so.x, so.y, so.z);
    r.d = make_float3(sd.x, sd.y, sd.z);
    L = sd.w;
    excl = a.face_log[(size_t)(k - 1) * a.n_work + work];
  }
  setup_ray(r);
  uint32_t state = 0;
  for (; k <= a.K; ++k) {
    Hit h = closest_hit(r, a.nodes4, top, n_top, n4, a.tri4, excl, stack, overflow, node_count, tri_count);
    ++seg_count;
    const bool hit = h.tri >= 0;
    const float tend = hit ? h.t : INFINITY;
    a.face_log[(size_t)k * a.n_work + work] = hit ? h.face : -1;
    if (hit && a.face_object[h.face] >= 0) state |= 0x80u;
    if (a.seg_o) {
      a.seg_o[(size_t)k * a.n_work + work] = make_float4(r.o.x, r.o.y, r.o.z, tend);
      a.seg_d[(size_t)k * a.n_work + work] = make_float4(r.d.x, r.d.y, r.d.z, L);
    }
    const float dd = dot_dd(r);
    const float L_hit = __fmaf_rn(h.t, __fsqrt_rn(dd), L);
    if (a.log_tri) {
      const size_t li = (size_t)rid * (a.K + 1) + k;
      a.log_tri[li] = h.tri;
      a.log_t[li] = hit ? h.t : INFINITY;
      a.log_len[li] = hit ? L_hit : INFINITY;
    }
    if (k > last_t) capture_segment(a, r, hit, h.t, tend, dd, work, txi, k, stack, overflow, cap_over);
    if (!hit || k == a.K) { ++k; break; }
    if ((tset >> k) & 1u) {
      // transmission: straight on through a penetrable face
      if (!a.face_pen[h.face]) { ++k; break; }
      L = L_hit;
      transmit_ray(r, h.t);
    } else {
      // specular reflection off the hit triangle's plane, unless the branch
      // has reflected max_refl times
      if (k - __popc(tset & ((1u << k) - 1u)) == a.max_refl) { ++k; break; }
      L = L_hit;
      reflect_ray(r, h.t, a.tri4[h.leaf].v0, a.tri4[h.leaf].v1, a.tri4[h.leaf].v2);
    }
    excl = h.face;
  }
  // mark the remaining bounces as not reached
  for (int j = k; j <= a.K; ++j) {
    a.face_log[(size_t)j * a.n_work + work] = -2;
    if (a.log_tri) {
      const size_t li = (size_t)rid * (a.K + 1) + j;
      a.log_tri[li] = -2;
      a.log_t[li] = INFINITY;
      a.log_len[li] = INFINITY;
    }
  }
  a.ray_state[work] = (uint8_t)(state | (uint32_t)k);
}

// Wavefront-wide sums of a block's item counts, added to the frame counters
// (one atomic per wavefront), and its error flags.
__device__ void flush_counts(const TraceArgs& a, ItemCounts& ic) {
  uint32_t seg_count = ic.seg, node_count = ic.node, tri_count = ic.tri;
  for (int off = 32; off > 0; off >>= 1) {
    seg_count += __shfl_xor(seg_count, off);
    node_count += __shfl_xor(node_count, off);
    tri_count += __shfl_xor(tri_count, off);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicAdd(&a.counters[kCntSegments], seg_count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntNodes]), (unsigned long long)node_count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntTris]), (unsigned long long)tri_count);
  }
  if (ic.overflow) atomicOr(a.err, DCEM_ERR_STACK);
  if (ic.cap_over) atomicOr(a.err, DCEM_ERR_CAPTURES);
  ic = ItemCounts{};
}

// Persistent trace kernel: each wavefront takes 64 consecutive work items from
// a global queue and traces them through all bounces.  In work-list mode a ray
// restarts at its first invalidated segment from the cached segment state.
__global__ __launch_bounds__(kTraceBlock) void k_trace(TraceArgs a) {
  __shared__ int stack_mem[kStackLds * kTraceBlock];
  __shared__ Node4 top[kTopNodes];
  ThreadStack stack{stack_mem + threadIdx.x, a.stack_spill + blockIdx.x * (size_t)kTraceBlock + threadIdx.x,
                    (size_t)gridDim.x * kTraceBlock, a.stack_thread};
  const int n4 = a.n4_dev ? (int)*a.n4_dev : 0;
  const int n_top = min(kTopNodes, n4);
  for (int i = threadIdx.x; i < n_top; i += blockDim.x) top[i] = a.nodes4[i];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t n_work = a.work_list ? a.counters[kCntList] : (uint32_t)a.n_work;
  if (a.work_list && blockIdx.x == 0 && threadIdx.x == 0) a.counters[kCntWork] = n_work;
  ItemCounts ic;
  while (true) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&a.counters[kCntQueue], (uint32_t)kWave);
    base = __shfl(base, 0);
    if (base >= n_work) break;
    const uint32_t wi = base + lane;
    if (wi < n_work) trace_item(a, wi, top, n_top, n4, stack, ic);
  }
  keep_previous_captures(a, ic.cap_over, blockIdx.x);
  flush_counts(a, ic);
}

// Coherent frames whose receivers moved: the captures of every kept segment
// (each segment before its ray's first re-traced one, all segments of a
// reused ray) against the receivers' current positions, from the cached
// segment origins, directions and ends, with the arithmetic of the trace
// kernels (a re-trace would capture exactly these).  The re-trace that
// follows captures its own segments.
__global__ __launch_bounds__(kTraceBlock) void k_recapture(TraceArgs a) {
  __shared__ int stack_mem[kStackLds * kTraceBlock];
  ThreadStack stack{stack_mem + threadIdx.x, a.stack_spill + blockIdx.x * (size_t)kTraceBlock + threadIdx.x,
                    (size_t)gridDim.x * kTraceBlock, a.stack_thread};
  bool overflow = false, cap_over = false;
  const uint32_t n_work = (uint32_t)a.n_work;
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < n_work; w += gridDim.x * blockDim.x) {
    const int nseg = (int)(a.ray_state[w] & 0x0fu);
    const int stop = min(nseg, (int)a.restart[w]);
    const uint32_t vsrc = (uint32_t)(w / (uint64_t)a.n_rays);
    const uint32_t txi = vsrc / (uint32_t)a.n_branch;
    const uint32_t tset = a.branch_set[vsrc - txi * (uint32_t)a.n_branch];
    // a branch records the captures of its segments after its last transmission
    for (int k = tset ? 32 - __builtin_clz(tset) : 0; k < stop; ++k) {
      const float4 so = a.seg_o[(size_t)k * a.n_work + w];
      const float4 sd = a.seg_d[(size_t)k * a.n_work + w];
      Ray r;
      r.o = make_float3(so.x, so.y, so.z);
      r.d = make_float3(sd.x, sd.y, sd.z);
      setup_ray(r);
      const bool hit = so.w < INFINITY;
      capture_segment(a, r, hit, so.w, so.w, dot_dd(r), w, txi, k, stack, overflow, cap_over);
    }
  }
  if (overflow) atomicOr(a.err, DCEM_ERR_STACK);
  if (cap_over) atomicOr(a.err, DCEM_ERR_CAPTURES);
}

// Full traces of several scenes in one persistent launch.  args[j] describes
// scene j's frame (all rays, no work list); its items are cut into chunks of
// `chunk` consecutive work items, chunk_start[j] the first chunk of scene j in
// one queue over all scenes (chunk_start[n] the total).  A wavefront takes the
// next chunk, finds its scene and traces the chunk's items, 64 at a time;
// counts and errors go to that scene's frame.  The per-thread stack keeps its
// first S entries in LDS.  No top-level node cache: consecutive chunks may
// belong to different scenes.
template <int S>
__global__ __launch_bounds__(kTraceBlock) void k_trace_batch(const TraceArgs* __restrict__ args,
                                                             const uint32_t* __restrict__ chunk_start, int n_scene,
                                                             uint32_t chunk, uint32_t* __restrict__ queue,
                                                             int* __restrict__ spill) {
  __shared__ int stack_mem[S * kTraceBlock];
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t total = chunk_start[n_scene];
  while (true) {
    uint32_t g = 0;
    if (lane == 0) g = atomicAdd(queue, 1u);
    g = __builtin_amdgcn_readfirstlane(g);   // uniform: the scene's arguments load as scalars
    if (g >= total) break;
    int lo = 0, hi = n_scene - 1;   // the last scene whose first chunk is <= g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (chunk_start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const TraceArgs a = args[lo];
    ThreadStack stack{stack_mem + threadIdx.x, spill + blockIdx.x * (size_t)kTraceBlock + threadIdx.x,
                      (size_t)gridDim.x * kTraceBlock, a.stack_thread};
    stack.lds_entries = S;
    const int n4 = a.n4_dev ? (int)*a.n4_dev : 0;
    const uint32_t base = (g - chunk_start[lo]) * chunk;
    const uint32_t end = min(base + chunk, (uint32_t)a.n_work);
    ItemCounts ic;
    for (uint32_t b = base; b < end; b += kWave)
      if (b + lane < end) trace_item(a, b + lane, nullptr, 0, n4, stack, ic);
    flush_counts(a, ic);
  }
}

// Group-per-ray tracing for short work lists (the rays a coherent frame
// re-traces).  A ray is traced by a group of 16 lanes (one DPP row), four rays
// per wavefront, one tree level per step: a group pops up to four entries of
// its stack in LDS and each lane takes one slot of one popped 4-wide node.  A
// stack entry carries its node's leaf-slot mask, so a lane fetches its slot's
// leaf triangle or child box directly (one memory round trip per step); hit
// child nodes are pushed with their entry distance, and after every step the
// group's best hits are reduced to the lexicographic minimum of (t, triangle
// id).  Entries whose distance exceeds the current best are skipped.  When a
// group's stack empties it finishes the segment (logs, receivers, reflection)
// and continues with the next segment or ray while the other groups keep
// traversing.  Every triangle the per-thread traversal tests is tested here
// too (leaf triangles without their boxes, which only drops a conservative
// filter), with the same arithmetic, so the hit is the same.
// Lanes per ray: one DPP row.  (Measured on the re-trace of the urban
// workload: 8 and 32 lanes per ray take 1.7x and 1.1x as long.)
constexpr int kRayLanes = kGroup;
constexpr int kGroups = kWave / kRayLanes;  // rays per wavefront
constexpr int kRayStack = kRayLanes == 64 ? 256 : kGroupStack;   // stack entries per ray
constexpr int kWaves = 4;                   // wavefronts per block
constexpr int kWaveBlock = kWaves * kWave;
constexpr int kWaveRx = 512;                // receivers cached in LDS (more are read from memory)
constexpr int kCapStage = 256;              // new captures a block stages in LDS
constexpr int64_t kWaveTraceMax = 1 << 16;  // longest list traced by groups

__device__ inline bool hit_less(float ta, int ia, float tb, int ib) { return ta < tb || (ta == tb && ia < ib); }

// (t, triangle id) as one key ordered lexicographically: hit distances are
// positive, so their bit patterns order like the values; no hit is all ones.
__device__ inline uint64_t hit_key(float t, int tri) {
  return tri < 0 ? ~0ull : ((uint64_t)__float_as_uint(t) << 32) | (uint32_t)tri;
}

// A 64-bit value from another lane of the same row (DPP control CTRL).
template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const uint32_t nlo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const uint32_t nhi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return ((uint64_t)nhi << 32) | nlo;
}

struct SlotHit {
  float t;
  int tri;    // original triangle id, -1 none
  int slot;   // index into the slot triangle array
  int face;
  int moving; // the face belongs to a moving object
  float3 v0, v1, v2;   // the triangle (for the reflection)
};

// Minimum over each group of kRayLanes lanes: swaps within pairs and quads,
// then the mirrored halves of each 8-lane half-row and of each row, then
// across rows.
__device__ inline uint64_t group_min_u64(uint64_t v) {
  uint64_t o = dpp_u64<0xb1>(v);   // quad_perm [1, 0, 3, 2]
  v = o < v ? o : v;
  o = dpp_u64<0x4e>(v);            // quad_perm [2, 3, 0, 1]
  v = o < v ? o : v;
  if (kRayLanes >= 8) {
    o = dpp_u64<0x141>(v);         // row_half_mirror
    v = o < v ? o : v;
  }
  if (kRayLanes >= 16) {
    o = dpp_u64<0x140>(v);         // row_mirror
    v = o < v ? o : v;
  }
  if (kRayLanes >= 32) {
    o = __shfl_xor(v, 16);
    v = o < v ? o : v;
  }
  if (kRayLanes == 64) {
    o = __shfl_xor(v, 32);
    v = o < v ? o : v;
  }
  return v;
}

__device__ inline MaskAxes mask_axes(const Ray& r) {
  auto m = [](int k, int j) { return k == j ? 0xffffffffu : 0u; };
  return MaskAxes{m(r.kx, 0), m(r.kx, 1), m(r.kx, 2), m(r.ky, 0), m(r.ky, 1),
                  m(r.ky, 2), m(r.kz, 0), m(r.kz, 1), m(r.kz, 2)};
}


__global__ __launch_bounds__(kWaveBlock) void k_trace_wave(TraceArgs a) {
  __shared__ float4 rxs[kWaveRx];             // receivers by x column (x, y, z, index bits)
  __shared__ int32_t rx_col[kRxCols + 1];       // column starts
  __shared__ Capture scap[kCapStage];          // the block's new captures, appended at the end
  __shared__ uint32_t scap_n, scap_base;
  __shared__ uint32_t stk_e[kWaves * kGroups][kRayStack];
  __shared__ float stk_t[kWaves * kGroups][kRayStack];
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / kRayLanes, gl = lane & (kRayLanes - 1), jl = gl >> 2, el = gl & 3;
  const int leader = lane & ~(kRayLanes - 1);
  const uint64_t gmask = kRayLanes == kWave ? ~0ull : ((1ull << (kRayLanes % kWave)) - 1ull) << (kRayLanes * g);
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t* se = stk_e[threadIdx.x / kRayLanes];
  float* st = stk_t[threadIdx.x / kRayLanes];
  // the block's receivers, loaded into registers first (stored to LDS below,
  // once the group's first ray has been loaded alongside)
  const bool rx_lds = a.n_rx <= kWaveRx;
  float4 rx_pre[kWaveRx / kWaveBlock];
#pragma unroll
  for (int q = 0; q < kWaveRx / kWaveBlock; ++q) {
    const int i = threadIdx.x + q * kWaveBlock;
    rx_pre[q] = rx_lds && i < a.n_rx ? a.rx_cols[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int32_t* col_start = reinterpret_cast<const int32_t*>(a.rx_cols + a.n_rx);
  static_assert(kRxCols < kWaveBlock, "one column start per thread");
  const int32_t col_pre = threadIdx.x <= kRxCols ? col_start[threadIdx.x] : 0;
  const int n4 = a.n4_dev ? (int)a.n4_dev[0] : 0;
  const uint32_t root = n4 > 0 ? a.n4_dev[1] << kNodeBits : 0u;
  const uint32_t n_work = a.counters[kCntList];
  // the group's first list entry, read within the list's capacity (used
  // only when it is in the list)
  const uint32_t item0 = (blockIdx.x * kWaves + threadIdx.x / kWave) * kGroups + g;
  const uint32_t work0 = item0 < (uint64_t)a.n_work ? a.work_list[item0] : 0u;
  auto rx_column = [&](float x) {
    return (int)fminf(fmaxf(floorf((x - a.rx_col_x0) * a.rx_col_scale), 0.0f), (float)(kRxCols - 1));
  };
  if (blockIdx.x == 0 && threadIdx.x == 0) a.counters[kCntWork] = n_work;
  uint32_t seg_count = 0, node_count = 0, tri_count = 0;
  bool overflow = false, cap_over = false;

  // this group's ray (equal on its lanes)
  bool busy = false;
  uint32_t work = 0, rid = 0, txi = 0, state = 0;   // traversal position, ray id, transmitter
  int k = 0, excl = -1, guard = 0, sp = 0;
  float L = 0.0f, best_t = INFINITY;
  Ray r;
  MaskAxes ax;
  SlotHit h{FLT_MAX, -1, -1, -1, 0, {}, {}, {}};
  uint64_t best = ~0ull;   // the group's lexicographic minimum of (t, triangle)

  auto begin_segment = [&]() {
    h = SlotHit{FLT_MAX, -1, -1, -1, 0, {}, {}, {}};
    best_t = INFINITY;
    best = ~0ull;
    guard = n4 + 2;
    sp = 0;
    if (n4 > 0) {
      if (gl == 0) {
        se[0] = root;
        st[0] = 0.0f;
      }
      sp = 1;
    }
    ax = mask_axes(r);
  };
  auto start_ray = [&](uint32_t item, bool first) {
    busy = item < n_work;
    if (!busy) return;
    work = first ? work0 : a.work_list[item];
    txi = (uint32_t)(work / (uint64_t)a.n_rays);
    const uint32_t ray = a.ray_order[work - (uint64_t)txi * a.n_rays];
    rid = txi * (uint32_t)a.n_rays + ray;
    k = (int)a.restart[work];
    excl = -1;
    L = 0.0f;
    if (k == 0) {
      r.o = make_float3(a.tx[3 * txi], a.tx[3 * txi + 1], a.tx[3 * txi + 2]);
      r.d = make_float3(a.dirs[3 * ray], a.dirs[3 * ray + 1], a.dirs[3 * ray + 2]);
    } else {
      const float4 so = a.seg_o[(size_t)k * a.n_work + work];
      const float4 sd = a.seg_d[(size_t)k * a.n_work + work];
      r.o = make_float3(so.x, so.y, so.z);
      r.d = make_float3(sd.x, sd.y, sd.z);
      L = sd.w;
      excl = a.face_log[(size_t)(k - 1) * a.n_work + work];
    }
    setup_ray(r);
    state = 0;
    begin_segment();
  };

  // the previous frame's captures that stay, copied by the last blocks of
  // the launch first (sized for a quarter more rays than listed, they have
  // none to trace), so the blocks that trace start at once
  keep_previous_captures(a, cap_over, gridDim.x - 1 - blockIdx.x);
  // first item by position, then from the shared queue
  start_ray(item0, true);
#pragma unroll
  for (int q = 0; q < kWaveRx / kWaveBlock; ++q) {
    const int i = threadIdx.x + q * kWaveBlock;
    if (rx_lds && i < a.n_rx) rxs[i] = rx_pre[q];
  }
  if (threadIdx.x <= kRxCols) rx_col[threadIdx.x] = col_pre;
  if (threadIdx.x == 0) scap_n = 0;
  __syncthreads();
  const uint32_t n_static = gridDim.x * kWaves * kGroups;
  while (true) {
    wave_sync();
    if (__ballot(busy) == 0) break;
    // ---- one traversal step of every group whose stack is not empty
    const int n_pop = busy ? min(kRayLanes / 4, sp) : 0;
    bool act = jl < n_pop;
    uint32_t ent = 0;
    float tn = 0.0f;
    if (act) {
      ent = se[sp - 1 - jl];
      tn = st[sp - 1 - jl];
    }
    wave_sync();
    sp -= n_pop;
    act = act && tn <= best_t;
    const int node = (int)(ent & ((1u << kNodeBits) - 1));
    const bool leaf = act && ((ent >> (kNodeBits + el)) & 1u);
    const bool inner = act && !leaf;
    // this lane's slot, 48 bytes in one load: the leaf triangle, or the
    // child's box and entry (and 16 bytes of the next slot, unused)
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
    if (act) {
      const float4* src = leaf ? reinterpret_cast<const float4*>(a.tri4 + 4 * (size_t)node + el)
                               : reinterpret_cast<const float4*>(&a.nodes4[node].s[el]);
      q0 = src[0];
      q1 = src[1];
      q2 = src[2];
    }
    uint32_t push = kNoEntry;
    float pt = 0.0f;
    bool improved = false;
    if (leaf) {
      const int face = __float_as_int(q1.w);
      if (face != excl) {
        const float t = watertight_axes(r, ax, q0, q1, q2);
        const int tri = __float_as_int(q0.w);
        if (t > kTMin && hit_less(t, tri, h.t, h.tri)) {
          improved = true;
          h.t = t;
          h.tri = tri;
          h.slot = 4 * node + el;
          h.face = face;
          h.moving = __float_as_int(q2.w);
          h.v0 = make_float3(q0.x, q0.y, q0.z);
          h.v1 = make_float3(q1.x, q1.y, q1.z);
          h.v2 = make_float3(q2.x, q2.y, q2.z);
        }
      }
      ++tri_count;
    } else if (inner) {
      const int ch = __float_as_int(q0.w);
      float te;
      if (ch != kEmpty && slab(r, q0.x, q0.y, q0.z, q1.x, q1.y, q1.z, fminf(h.t, best_t), te)) {
        push = (uint32_t)ch | (__float_as_uint(q1.w) << kNodeBits);
        pt = te;
      }
    }
    if (act && el == 0) ++node_count;
    // push each group's hit children in lane order
    const uint64_t want = __ballot(push != kNoEntry) & gmask;
    const int total = __popcll(want);
    const int pos = sp + __popcll(want & below);
    if (push != kNoEntry && pos < a.stack_group) {
      se[pos] = push;
      st[pos] = pt;
    }
    if (sp + total > a.stack_group) overflow = true;
    sp = min(sp + total, a.stack_group);
    if (n_pop > 0 && --guard <= 0 && sp > 0) {   // only a malformed tree gets here
      overflow = true;
      sp = 0;
    }
    if (__ballot(improved)) {   // the groups' minima change only where a lane found a nearer hit
      best = group_min_u64(hit_key(h.t, h.tri));
      best_t = best == ~0ull ? INFINITY : __uint_as_float((uint32_t)(best >> 32));
    }
    if (!(busy && sp == 0)) continue;
    // ---- this group's traversal ended: finish the segment
    const uint64_t own = __ballot(best != ~0ull && hit_key(h.t, h.tri) == best) & gmask;
    const bool hit = own != 0;
    const int src = hit ? __ffsll((unsigned long long)own) - 1 : leader;
    const int face = __shfl(h.face, src), moving = __shfl(h.moving, src);
    const float th = hit ? __uint_as_float((uint32_t)(best >> 32)) : FLT_MAX;
    const int tri = hit ? (int)(uint32_t)best : -1;
    const bool more = hit && k < a.K;
    // the reflecting triangle, from the lane that found it
    const float4 w0 = make_float4(__shfl(h.v0.x, src), __shfl(h.v0.y, src), __shfl(h.v0.z, src), 0.0f);
    const float4 w1 = make_float4(__shfl(h.v1.x, src), __shfl(h.v1.y, src), __shfl(h.v1.z, src), 0.0f);
    const float4 w2 = make_float4(__shfl(h.v2.x, src), __shfl(h.v2.y, src), __shfl(h.v2.z, src), 0.0f);
    const float tend = hit ? th : INFINITY;
    if (hit && moving) state |= 0x80u;
    const float dd = dot_dd(r);
    const float L_hit = __fmaf_rn(th, __fsqrt_rn(dd), L);
    if (gl == 0) {
      ++seg_count;
      a.face_log[(size_t)k * a.n_work + work] = hit ? face : -1;
      a.seg_o[(size_t)k * a.n_work + work] = make_float4(r.o.x, r.o.y, r.o.z, tend);
      a.seg_d[(size_t)k * a.n_work + work] = make_float4(r.d.x, r.d.y, r.d.z, L);
      if (a.log_tri) {
        const size_t li = (size_t)rid * (a.K + 1) + k;
        a.log_tri[li] = tri;
        a.log_t[li] = hit ? th : INFINITY;
        a.log_len[li] = hit ? L_hit : INFINITY;
      }
    }
    // capture: the group's lanes share the receivers
    const float za = r.o.z;
    const float zb = hit ? __fmaf_rn(th, r.d.z, r.o.z) : (r.d.z > 0 ? INFINITY : (r.d.z < 0 ? -INFINITY : r.o.z));
    if (a.capture && fmaxf(za, zb) >= a.rx_zlo && fminf(za, zb) <= a.rx_zhi) {
      // cull by the xy bounds of the segment's part inside the receivers' z
      // band: a sphere the segment meets has its centre within a radius of
      // that part (rx_cull adds slack far above the rounding here)
      float bx0 = -INFINITY, bx1 = INFINITY, by0 = -INFINITY, by1 = INFINITY;
      float s0 = 0.0f, s1 = tend;
      if (fabsf(r.d.z) > 1e-20f) {
        const float rz = __builtin_amdgcn_rcpf(r.d.z);
        const float a0 = (a.rx_zlo - r.o.z) * rz, a1 = (a.rx_zhi - r.o.z) * rz;
        s0 = fmaxf(s0, fminf(a0, a1));
        s1 = fminf(s1, fmaxf(a0, a1));
      }
      if (s1 < 1e30f) {
        const float xa = fmaf(s0, r.d.x, r.o.x), xb = fmaf(s1, r.d.x, r.o.x);
        const float ya = fmaf(s0, r.d.y, r.o.y), yb = fmaf(s1, r.d.y, r.o.y);
        bx0 = fminf(xa, xb) - a.rx_cull;
        bx1 = fmaxf(xa, xb) + a.rx_cull;
        by0 = fminf(ya, yb) - a.rx_cull;
        by1 = fmaxf(ya, yb) + a.rx_cull;
      }
      // receivers of the columns the box covers (one more on each side)
      int c0 = 0, c1 = a.n_rx;
      if (bx1 < INFINITY) {
        c0 = rx_col[max(rx_column(bx0) - 1, 0)];
        c1 = rx_col[min(rx_column(bx1) + 1, kRxCols - 1) + 1];
      }
      auto test_rx = [&](const float4 q) {
        if (q.x < bx0 || q.x > bx1 || q.y < by0 || q.y > by1) return;
        if (captured(r, tend, dd, q.x, q.y, q.z, a.r2)) {
          Capture cp;
          cp.work = work;
          cp.pair_order = ((txi * (uint32_t)a.n_rx + (uint32_t)__float_as_int(q.w)) << 4) | (uint32_t)k;
          const uint32_t p = atomicAdd(&scap_n, 1u);
          if (p < (uint32_t)kCapStage) {
            scap[p] = cp;
          } else {
            const uint32_t cs = atomicAdd(&a.counters[kCntCaptures], 1u);
            if (cs < a.cap_capacity) a.caps[cs] = cp;
            else cap_over = true;
          }
        }
      };
      // two loops (the condition is uniform): a load that may read either
      // LDS or device memory would wait for this segment's log stores
      if (rx_lds) {
        for (int c = c0 + gl; c < c1; c += kRayLanes) test_rx(rxs[c]);
      } else {
        for (int c = c0 + gl; c < c1; c += kRayLanes) test_rx(a.rx_cols[c]);
      }
    }
    ++k;
    if (more) {
      // specular reflection (identical arithmetic on the group's lanes)
      L = L_hit;
      reflect_ray(r, th, w0, w1, w2);
      excl = face;
      begin_segment();
      continue;
    }
    if (gl == 0) {
      for (int j = k; j <= a.K; ++j) {
        a.face_log[(size_t)j * a.n_work + work] = -2;
        if (a.log_tri) {
          const size_t li = (size_t)rid * (a.K + 1) + j;
          a.log_tri[li] = -2;
          a.log_t[li] = INFINITY;
          a.log_len[li] = INFINITY;
        }
      }
      a.ray_state[work] = (uint8_t)(state | (uint32_t)k);
    }
    // the next item from the shared queue, unless the first items covered
    // every ray (no atomic round trip then)
    uint32_t next = n_work;
    if (n_static < n_work) {
      if (gl == 0) next = n_static + atomicAdd(&a.counters[kCntQueue], 1u);
      next = __shfl(next, leader);
    }
    start_ray(next, false);
  }
  // append the block's staged captures with one atomic
  __syncthreads();
  const uint32_t ns = min(scap_n, (uint32_t)kCapStage);
  if (threadIdx.x == 0 && ns) scap_base = atomicAdd(&a.counters[kCntCaptures], ns);
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < ns; j += kWaveBlock) {
    const uint32_t slot = scap_base + j;
    if (slot < a.cap_capacity) a.caps[slot] = scap[j];
    else cap_over = true;
  }
  for (int off = 32; off > 0; off >>= 1) {
    seg_count += __shfl_xor(seg_count, off);
    node_count += __shfl_xor(node_count, off);
    tri_count += __shfl_xor(tri_count, off);
  }
  if (lane == 0) {
    atomicAdd(&a.counters[kCntSegments], seg_count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntNodes]), (unsigned long long)node_count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[kCntTris]), (unsigned long long)tri_count);
  }
  if (overflow) atomicOr(a.err, DCEM_ERR_STACK);
  if (cap_over) atomicOr(a.err, DCEM_ERR_CAPTURES);
}

// Start of a frame's lists: the counters reset (the revalidation's list
// counter kept when `keep_list`: a revalidation in the same launch appends to
// it) and one line-of-sight record per (tx, rx) pair at the head of the
// capture list.  Threads `t` of `nt` share the records.
struct FrameBegin {
  uint32_t* counters;
  Capture* caps;
  int n_los;
  int64_t cap_capacity;
  uint32_t* err;
  // nullable: a nonzero word here (read at launch; the last frame's candidate
  // fallback flag) makes the launch do nothing: that frame's candidates must
  // be redone on the tree it was traced with before the next frame begins
  const uint32_t* skip;
};

__device__ inline void frame_begin_part(const FrameBegin& f, int t, int nt, bool keep_list) {
  if (t < kCntSlots && !(keep_list && t == kCntList)) f.counters[t] = t == kCntCaptures ? f.n_los : 0;
  for (int p = t; p < f.n_los; p += nt) {
    if (p < f.cap_capacity) {
      Capture c;
      c.work = kNoRay;
      c.pair_order = (uint32_t)p << 4;
      f.caps[p] = c;
    } else if (p == f.cap_capacity) {
      atomicOr(f.err, DCEM_ERR_CAPTURES);
    }
  }
}

__global__ void k_frame_begin(FrameBegin f) {
  if (f.skip && *f.skip) return;
  frame_begin_part(f, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, false);
}

// Coherence pass.  Segment k of a cached ray is still valid iff no earlier
// segment is invalid, its hit in the cached frame was not on a moving face, and
// it (unbounded on a miss) does not meet the padded box of any moving object
// now.  A ray whose segments are all valid would be traced to exactly the same
// hits and captures, so it is reused as it is; otherwise it is listed for
// re-tracing from its first invalid segment (wavefront-aggregated append).
// Each block bins the moving-object boxes on a 32 x 32 grid over their xy
// extent in LDS, one bit per object and cell, so a segment tests only the
// boxes of the cells its xy bounds cover (up to kCohGridObjects objects; more
// are tested one by one).
constexpr int kCohBlock = 256;
constexpr int kCohGrid = 32;
constexpr int kCohGridObjects = 256;
constexpr int kCohMaxCells = 16;   // wider xy bounds test every box
constexpr int kCohBatch = 5;       // cached segments loaded at once
constexpr int kCohList = 4096;     // invalid rays a block collects before one list append

struct CohArgs {
  const uint8_t* ray_state;
  const float4* seg_o;
  const float4* seg_d;
  const int32_t* face_log;
  const int32_t* face_object;
  const float* obj_box;
  int n_obj;
  int n_work;
  const float* tx;
  int64_t n_rays;
  float margin;
  uint8_t* restart;
  uint32_t* list;
  uint32_t* counters;
  int list_cap;   // invalid rays a block collects in LDS (dynamic, after the grid)
};

// One block of the revalidation pass: block cb of n_cb, blockDim.x threads.
__device__ __forceinline__ void coherence_block(const CohArgs& args, int cb, int n_cb) {
  const uint8_t* __restrict__ ray_state = args.ray_state;
  const float4* __restrict__ seg_o = args.seg_o;
  const float4* __restrict__ seg_d = args.seg_d;
  const int32_t* __restrict__ face_log = args.face_log;
  const int32_t* __restrict__ face_object = args.face_object;
  const float* __restrict__ obj_box = args.obj_box;
  const int n_obj = args.n_obj, n_work = args.n_work;
  const float* __restrict__ tx = args.tx;
  const int64_t n_rays = args.n_rays;
  const float margin = args.margin;
  uint8_t* __restrict__ restart = args.restart;
  uint32_t* __restrict__ list = args.list;
  uint32_t* counters = args.counters;
  const int nth = blockDim.x;
  // dynamic LDS (grid mode): cell bits [cell][word], then the boxes [6][n_obj]
  extern __shared__ unsigned long long coh_lds[];
  __shared__ uint32_t ext[6];   // ordered bits: min x, min y, min z, max x, max y, max z
  // the block's invalid rays (dynamic LDS after the grid), appended to the
  // global list with one atomic at the end (a counter shared by every
  // wavefront of the grid would serialise)
  __shared__ uint32_t bcount, bbase;
  const int kList = args.list_cap;
  if (threadIdx.x == 0) bcount = 0;
  const bool grid = n_obj <= kCohGridObjects;
  const int words = (n_obj + 63) / 64;
  unsigned long long* cell = coh_lds;
  float* blf = reinterpret_cast<float*>(coh_lds + (grid ? kCohGrid * kCohGrid * words : 0));
  uint32_t* blist = reinterpret_cast<uint32_t*>(blf + (grid ? 6 * n_obj : 0));
  auto bl = [&](int a, int b) -> float& { return blf[a * n_obj + b]; };
  if (threadIdx.x < 6) ext[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;
  if (grid)
    for (int c = threadIdx.x; c < kCohGrid * kCohGrid * words; c += nth) cell[c] = 0ull;
  __syncthreads();
  // the objects' extent: each wavefront loads its boxes at once and reduces
  // them before one set of LDS atomics (atomics with lane-varying values on
  // one address would be serialised over the lanes)
  const int lane0 = threadIdx.x & (kWave - 1);
  for (int w0 = threadIdx.x - lane0; w0 < n_obj; w0 += nth) {   // uniform over the wavefront
    const int b = w0 + lane0;
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    if (b < n_obj) {
      float v[6];
      for (int k = 0; k < 6; ++k) v[k] = obj_box[6 * b + k];
      if (grid)
        for (int k = 0; k < 6; ++k) bl(k, b) = v[k];
      for (int a = 0; a < 3; ++a) {
        mn[a] = ordered_bits(v[a]);
        mx[a] = ordered_bits(v[3 + a]);
      }
    }
    for (int off = kWave / 2; off > 0; off >>= 1)
      for (int a = 0; a < 3; ++a) {
        mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], off));
        mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], off));
      }
    if (lane0 == 0)
      for (int a = 0; a < 3; ++a) {
        atomicMin(&ext[a], mn[a]);
        atomicMax(&ext[3 + a], mx[a]);
      }
  }
  __syncthreads();
  const float gx0 = from_ordered(ext[0]), gy0 = from_ordered(ext[1]);
  const float zlo = n_obj ? from_ordered(ext[2]) - margin : INFINITY;
  const float zhi = n_obj ? from_ordered(ext[5]) + margin : -INFINITY;
  const float sx = kCohGrid / fmaxf(from_ordered(ext[3]) - gx0, 1e-6f);
  const float sy = kCohGrid / fmaxf(from_ordered(ext[4]) - gy0, 1e-6f);
  // cell index of a coordinate, clamped to the grid (infinite bounds included):
  // monotonic, so overlapping ranges share a cell
  auto cell_of = [](float u) { return (int)fminf(fmaxf(floorf(u), 0.0f), (float)(kCohGrid - 1)); };
  auto cx = [&](float x) { return cell_of((x - gx0) * sx); };
  auto cy = [&](float y) { return cell_of((y - gy0) * sy); };
  if (grid) {
    for (int b = threadIdx.x; b < n_obj; b += nth) {
      const int x0 = cx(bl(0, b)), x1 = cx(bl(3, b)), y0 = cy(bl(1, b)), y1 = cy(bl(4, b));
      for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) atomicOr(&cell[(y * kCohGrid + x) * words + (b >> 6)], 1ull << (b & 63));
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  // blocks stride over the rays (the grid above is built once per block)
  // each thread checks rays i, i + stride, ...: the next ray's state byte is
  // loaded while the current ray's segments are, so a ray costs one round trip
  const int64_t stride = (int64_t)n_cb * nth;
  uint32_t st_next = (int64_t)cb * nth + threadIdx.x < n_work ? ray_state[cb * nth + threadIdx.x] : 0u;
  for (int64_t base0 = (int64_t)cb * nth; base0 < n_work; base0 += stride) {
    const int64_t i = base0 + threadIdx.x;
    int first = 255;
    const uint32_t w = (uint32_t)i;
    const uint32_t st_cur = st_next;
    if (i + stride < n_work) st_next = ray_state[i + stride];
    if (i < n_work) {
      const uint32_t st = st_cur;
      const int nseg = (int)(st & 0x0fu);
      const bool moving_hit = (st & 0x80u) != 0;
      // does the cached segment (o, d) meet a moving object's box now?
      // Does the cached segment (o, d) meet a moving object's box now?  The
      // answer only has to be conservative (a ray listed without need is traced
      // again to the same result), so reciprocals are the hardware's (about one
      // ulp) and every bound is widened by `margin`, far above those errors.
      auto meets_moving = [&](const float4& o, const float4& d) {
        // cull: the part of the segment inside the moving objects' z range, and
        // its xy bounds
        float s0 = 0.0f, s1 = o.w;
        if (d.z != 0.0f) {
          const float rz = __builtin_amdgcn_rcpf(d.z);
          const float a0 = (zlo - o.z) * rz, a1 = (zhi - o.z) * rz;
          s0 = fmaxf(s0, fminf(a0, a1));
          s1 = fminf(s1, fmaxf(a0, a1));
        } else if (o.z < zlo || o.z > zhi) {
          return false;
        }
        if (!(s0 <= s1)) return false;
        const float xa = fmaf(s0, d.x, o.x), xb = fmaf(s1, d.x, o.x);
        const float ya = fmaf(s0, d.y, o.y), yb = fmaf(s1, d.y, o.y);
        const float bx0 = fminf(xa, xb) - margin, bx1 = fmaxf(xa, xb) + margin;
        const float by0 = fminf(ya, yb) - margin, by1 = fmaxf(ya, yb) + margin;
        Ray r;
        r.o = make_float3(o.x, o.y, o.z);
        r.d = make_float3(d.x, d.y, d.z);
        const float tiny = 1e-30f;
        r.inv = make_float3(__builtin_amdgcn_rcpf(r.d.x != 0.0f ? r.d.x : tiny),
                            __builtin_amdgcn_rcpf(r.d.y != 0.0f ? r.d.y : tiny),
                            __builtin_amdgcn_rcpf(r.d.z != 0.0f ? r.d.z : tiny));
        auto meets = [&](float lx, float ly, float lz, float hx, float hy, float hz) {
          if (hx < bx0 || lx > bx1 || hy < by0 || ly > by1) return false;
          float tn;
          return slab(r, lx - margin, ly - margin, lz - margin, hx + margin, hy + margin, hz + margin, o.w, tn);
        };
        if (!grid) {
          for (int b = 0; b < n_obj; ++b) {
            const float* bx = obj_box + 6 * b;
            if (meets(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5])) return true;
          }
          return false;
        }
        // candidate objects: the union of the covered cells' bits
        const int x0 = cx(bx0), x1 = cx(bx1), y0 = cy(by0), y1 = cy(by1);
        const bool all = (x1 - x0 + 1) * (y1 - y0 + 1) > kCohMaxCells;
        for (int wd = 0; wd < words; ++wd) {
          unsigned long long m = 0;
          if (all) {
            m = ~0ull;
          } else {
            for (int y = y0; y <= y1; ++y)
              for (int x = x0; x <= x1; ++x) m |= cell[(y * kCohGrid + x) * words + wd];
          }
          while (m) {
            const int b = 64 * wd + __ffsll(m) - 1;
            m &= m - 1;
            if (b >= n_obj) break;
            if (meets(bl(0, b), bl(1, b), bl(2, b), bl(3, b), bl(4, b), bl(5, b))) return true;
          }
        }
        return false;
      };
      // The ray's polyline: its transmitter, then the origin of each later
      // segment (a reflection starts exactly at the previous segment's end
      // point), then the last segment's direction and extent.  Segment k < last
      // runs from origin k to origin k + 1.  Origins are loaded in batches, so
      // a ray of n >= 2 segments reads n cached 16-byte records.
      const int last = nseg - 1;
      const uint32_t txi = (uint32_t)(w / (uint64_t)n_rays);
      float4 prev = make_float4(tx[3 * txi], tx[3 * txi + 1], tx[3 * txi + 2], 0.0f);   // origin of segment k0
      if (last == 0) prev.w = seg_o[w].w;   // the one segment's extent
      for (int k0 = 0; k0 <= last && first == 255; k0 += kCohBatch) {
        float4 nxt[kCohBatch];   // origin of segment k0 + j + 1 (its extent in w)
        int bf[kCohBatch];
        float4 dl = make_float4(0.f, 0.f, 0.f, 0.f);
        const bool has_last = last < k0 + kCohBatch;
#pragma unroll
        for (int j = 0; j < kCohBatch; ++j) {
          const int k = k0 + j;
          bf[j] = -1;
          if (k + 1 <= last) nxt[j] = seg_o[(size_t)(k + 1) * n_work + w];
          if (k <= last && moving_hit) bf[j] = face_log[(size_t)k * n_work + w];
        }
        if (has_last) dl = seg_d[(size_t)last * n_work + w];
#pragma unroll
        for (int j = 0; j < kCohBatch; ++j) {
          const int k = k0 + j;
          if (k > last || first != 255) break;
          float4 o = prev, d;
          if (k < last) {
            o.w = 1.0f;
            d = make_float4(nxt[j].x - prev.x, nxt[j].y - prev.y, nxt[j].z - prev.z, 0.0f);
            prev = nxt[j];
          } else {
            d = dl;
          }
          if ((bf[j] >= 0 && face_object[bf[j]] >= 0) || meets_moving(o, d)) first = k;
        }
      }
      restart[w] = (uint8_t)first;
    }
    const bool bad = first != 255;
    const uint64_t m = __ballot(bad);
    if (m) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&bcount, (uint32_t)__popcll(m));
      base = __shfl(base, 0);
      if (bad) {
        const uint32_t p = base + __popcll(m & ((1ull << lane) - 1ull));
        if (p < (uint32_t)kList) blist[p] = w;
        else list[atomicAdd(&counters[kCntList], 1u)] = w;   // only when a block is given more rays
      }
    }
  }
  __syncthreads();
  const uint32_t nb = min(bcount, (uint32_t)kList);
  if (threadIdx.x == 0 && nb) bbase = atomicAdd(&counters[kCntList], nb);
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < nb; j += nth) list[bbase + j] = blist[j];
}

__global__ __launch_bounds__(kCohBlock) void k_coherence(CohArgs a) { coherence_block(a, blockIdx.x, gridDim.x); }

// A coherent frame's refit and revalidation in one launch: blocks [0, n_rb)
// refit the tree, the others revalidate the cached rays (which do not read the
// tree), so the latency-bound refit overlaps the revalidation.
// With `begin`, the first revalidation block also starts the frame's lists
// (all but the list counter the revalidation appends to, which the previous
// frame's reduction zeroed).
__global__ __launch_bounds__(kRefitBlock) void k_refit_coherence(RefitArgs ra, CohArgs ca, int n_rb, FrameBegin fb,
                                                                 int begin) {
  // with a skip word set (the last frame needs its candidates redone) nothing
  // runs; the word only turns from nonzero to zero inside this launch (the
  // frame start clears it) if it was zero already, so every block agrees
  if (fb.skip && *fb.skip) return;
  if ((int)blockIdx.x < n_rb) {
    refit_block(ra, blockIdx.x, n_rb);
  } else {
    if (begin && (int)blockIdx.x == n_rb) frame_begin_part(fb, threadIdx.x, blockDim.x, true);
    coherence_block(ca, blockIdx.x - n_rb, gridDim.x - n_rb);
  }
}


// Spatial key of a direction: octahedral map to the unit square, 16 bits per
// axis, interleaved.  Sorting rays by it groups neighbouring directions in a
// wavefront.
__device__ inline uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__global__ void k_dir_keys(const float* __restrict__ dirs, int64_t n, uint32_t* __restrict__ key) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x = dirs[3 * i], y = dirs[3 * i + 1], z = dirs[3 * i + 2];
  const float l1 = fabsf(x) + fabsf(y) + fabsf(z);
  float u = 0.f, v = 0.f;
  if (l1 > 0.f) {
    x /= l1; y /= l1; z /= l1;
    if (z >= 0.f) { u = x; v = y; }
    else { u = (1.f - fabsf(y)) * (x >= 0.f ? 1.f : -1.f); v = (1.f - fabsf(x)) * (y >= 0.f ? 1.f : -1.f); }
  }
  const uint32_t qu = (uint32_t)fminf(fmaxf((u * 0.5f + 0.5f) * 65535.f, 0.f), 65535.f);
  const uint32_t qv = (uint32_t)fminf(fmaxf((v * 0.5f + 0.5f) * 65535.f, 0.f), 65535.f);
  key[i] = (spread16(qu) << 1) | spread16(qv);
}

int cu_count(dcem_ctx* c) {
  if (c->n_cus == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->n_cus = prop.multiProcessorCount;
    if (c->n_cus <= 0) c->n_cus = 256;
  }
  return c->n_cus;
}

int trace_grid(dcem_ctx* c) {
  return cu_count(c) * 8;   // 16 KB of LDS stack and 2.7 KB of top nodes per block: eight blocks per CU
}

}  // namespace

void launch_fibonacci(dcem_ctx* c) {
  const int64_t n = c->n_rays;
  hipLaunchKernelGGL(k_fibonacci, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, ptr<float>(c->dirs), n);
}

// Trace all work items (all_rays) or those listed by the coherence pass.  The
// persistent grid is sized for `expected` work items (any size is correct:
// blocks drain a shared queue).
namespace {

// Arguments of a context's trace launch.
TraceArgs trace_args(dcem_ctx* c, bool all_rays, bool keep_cache, uint32_t n_prev_caps) {
  const int64_t n_work = (int64_t)c->n_src * c->n_branch * c->n_rays;
  TraceArgs a;
  a.nodes4 = ptr<Node4>(c->nodes4);
  a.tri4 = ptr<Leaf>(c->tri4);
  a.n4_dev = c->nt > 0 ? ptr<uint32_t>(c->tree_info) : nullptr;
  a.dirs = ptr<float>(c->dirs);
  a.ray_order = ptr<uint32_t>(c->ray_order);
  a.tx = ptr<float>(c->src_pos);
  a.rx = ptr<float>(c->tgt_pos);
  a.n_rx = c->n_tgt;
  a.capture = c->visited ? 0 : 1;
  a.rx_nodes = ptr<Node>(c->rx_nodes);
  a.n_rx_nodes = c->n_rx_nodes;
  a.restart = all_rays ? nullptr : ptr<uint8_t>(c->invalid_flag);
  a.r2 = c->cfg.rx_radius * c->cfg.rx_radius;
  float zlo = FLT_MAX, zhi = -FLT_MAX;
  for (int i = 0; i < c->n_tgt; ++i) {
    zlo = fminf(zlo, c->cfg.tgt[3 * i + 2]);
    zhi = fmaxf(zhi, c->cfg.tgt[3 * i + 2]);
  }
  // widen the culling slab well beyond rounding so it never changes a decision
  const float rr = c->cfg.rx_radius * 1.001f + 1e-3f;
  a.rx_zlo = zlo - rr;
  a.rx_zhi = zhi + rr;
  a.rx_cull = c->cfg.rx_radius * 1.001f + 1e-2f;
  a.rx_cols = ptr<float4>(c->rx_cols);
  a.rx_col_x0 = c->rx_col_x0;
  a.rx_col_scale = c->rx_col_scale;
  a.n_rays = c->n_rays;
  a.n_work = (int)n_work;
  a.work_list = all_rays ? nullptr : ptr<uint32_t>(c->work_list);
  a.K = c->K;
  a.max_refl = c->max_refl;
  a.n_branch = c->n_branch;
  a.branch_set = ptr<uint32_t>(c->branch_set);
  a.face_pen = ptr<uint8_t>(c->face_pen);
  a.face_object = ptr<int32_t>(c->face_object);
  a.counters = c->cnt_dev;
  a.face_log = ptr<int32_t>(c->face_log);
  a.ray_state = ptr<uint8_t>(c->ray_state);
  a.seg_o = keep_cache ? ptr<float4>(c->seg_o) : nullptr;
  a.seg_d = keep_cache ? ptr<float4>(c->seg_d) : nullptr;
  a.log_tri = c->record_log ? ptr<int32_t>(c->log_tri) : nullptr;
  a.log_t = c->record_log ? ptr<float>(c->log_t) : nullptr;
  a.log_len = c->record_log ? ptr<float>(c->log_len) : nullptr;
  a.caps = ptr<Capture>(c->caps[c->cur_caps]);
  a.cap_capacity = c->cap_capacity;
  a.err = c->err_dev;
  a.prev_caps = ptr<Capture>(c->caps[c->cur_caps ^ 1]);
  a.n_prev = all_rays ? 0u : n_prev_caps;
  a.stack_spill = nullptr;
  a.stack_thread = c->stack_limit > 0 ? std::min(c->stack_limit, kStackSize) : kStackSize;
  a.stack_group = c->stack_limit > 0 ? std::min(c->stack_limit, kRayStack) : kRayStack;
  return a;
}

}  // namespace

int launch_trace(dcem_ctx* c, bool all_rays, bool keep_cache, int64_t expected, uint32_t n_prev_caps) {
  TraceArgs a = trace_args(c, all_rays, keep_cache, n_prev_caps);
  if (!all_rays && expected <= kWaveTraceMax && c->n_branch == 1) {
    // short re-trace list: one wavefront per ray
    const int64_t want = (expected + expected / 4 + kWaves * kGroups - 1) / (kWaves * kGroups) + 1;
    const int grid = (int)std::max<int64_t>(16, std::min<int64_t>((int64_t)cu_count(c) * 8, want));
    hipLaunchKernelGGL(k_trace_wave, dim3(grid), dim3(kWaveBlock), 0, c->stream, a);
    return 1;
  }
  const int64_t want = (expected + expected / 4 + kTraceBlock - 1) / kTraceBlock;
  const int grid = (int)std::max<int64_t>(16, std::min<int64_t>(trace_grid(c), want));
  if (prepare_trace(c) != hipSuccess) {   // sized already by the frame's setup
    (void)hipGetLastError();
    return -1;
  }
  a.stack_spill = ptr<int>(c->stack_spill);
  hipLaunchKernelGGL(k_trace, dim3(grid), dim3(kTraceBlock), 0, c->stream, a);
  return 0;
}

size_t batch_table_bytes(int n) {
  return ((sizeof(TraceArgs) * (size_t)n + 255) / 256) * 256 + sizeof(uint32_t) * ((size_t)n + 1) + 256;
}

size_t batch_spill_bytes(const dcem_ctx* c, const BatchShape& shape) {
  const int grid = std::max(1, cu_count(const_cast<dcem_ctx*>(c)) * shape.blocks_per_cu);
  return sizeof(int) * (size_t)(kStackSize - shape.lds_stack) * kTraceBlock * (size_t)grid;
}

hipError_t launch_trace_batch(dcem_ctx* const* cs, const uint8_t* keep_cache, int n, const BatchShape& shape,
                              DevBuf& table, void* host_table, size_t host_table_bytes, DevBuf& spill, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t args_bytes = ((sizeof(TraceArgs) * (size_t)n + 255) / 256) * 256;
  if (host_table_bytes < batch_table_bytes(n) || table.bytes < batch_table_bytes(n)) return hipErrorInvalidValue;
  if (spill.bytes < batch_spill_bytes(cs[0], shape)) return hipErrorInvalidValue;
  // per-context arguments and the chunk table, staged in pinned memory
  char* h = static_cast<char*>(host_table);
  TraceArgs* ha = reinterpret_cast<TraceArgs*>(h);
  uint32_t* hc = reinterpret_cast<uint32_t*>(h + args_bytes);
  uint64_t total = 0;
  for (int j = 0; j < n; ++j) {
    ha[j] = trace_args(cs[j], true, keep_cache[j] != 0, 0u);
    hc[j] = (uint32_t)total;
    total += ((uint64_t)ha[j].n_work + shape.chunk - 1) / shape.chunk;
  }
  hc[n] = (uint32_t)total;
  if (total >= (uint64_t)1 << 32) return hipErrorInvalidValue;
  uint32_t* queue = reinterpret_cast<uint32_t*>(static_cast<char*>(table.p) + args_bytes + sizeof(uint32_t) * (n + 1));
  hipError_t e = hipMemcpyAsync(table.p, host_table, args_bytes + sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  fill_u32(queue, 0u, 1, s);
  const TraceArgs* dargs = static_cast<const TraceArgs*>(table.p);
  const uint32_t* dchunk = reinterpret_cast<const uint32_t*>(static_cast<char*>(table.p) + args_bytes);
  const int want = (int)std::min<uint64_t>((total * shape.chunk + kTraceBlock - 1) / kTraceBlock + 1,
                                           (uint64_t)cu_count(cs[0]) * shape.blocks_per_cu);
  const int grid = std::max(1, want);
  int* sp = ptr<int>(spill);
  if (shape.lds_stack == 16)
    hipLaunchKernelGGL(k_trace_batch<16>, dim3(grid), dim3(kTraceBlock), 0, s, dargs, dchunk, n,
                       (uint32_t)shape.chunk, queue, sp);
  else if (shape.lds_stack == 32)
    hipLaunchKernelGGL(k_trace_batch<32>, dim3(grid), dim3(kTraceBlock), 0, s, dargs, dchunk, n,
                       (uint32_t)shape.chunk, queue, sp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

void launch_recapture(dcem_ctx* c) {
  TraceArgs a = trace_args(c, false, true, 0u);
  a.stack_spill = ptr<int>(c->stack_spill);
  const int64_t n_work = (int64_t)c->n_src * c->n_branch * c->n_rays;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(trace_grid(c), (n_work + kTraceBlock - 1) / kTraceBlock));
  hipLaunchKernelGGL(k_recapture, dim3(grid), dim3(kTraceBlock), 0, c->stream, a);
}

hipError_t prepare_trace(dcem_ctx* c) {
  // spill space for the largest grid, so it never changes from frame to frame
  return ensure(c->stack_spill, sizeof(int) * kStackSpill * kTraceBlock * (size_t)std::max(trace_grid(c), 16));
}

FrameBegin frame_begin_args(dcem_ctx* c, bool los) {
  return FrameBegin{c->cnt_dev, ptr<Capture>(c->caps[c->cur_caps]), los ? c->n_src * c->n_tgt : 0, c->cap_capacity,
                    c->err_dev, nullptr};
}

void launch_frame_begin(dcem_ctx* c, bool los, const uint32_t* skip) {
  FrameBegin f = frame_begin_args(c, los);
  f.skip = skip;
  hipLaunchKernelGGL(k_frame_begin, dim3((unsigned)std::max(1, (f.n_los + 255) / 256)), dim3(256), 0, c->stream, f);
}

CohArgs coherence_args(dcem_ctx* c) {
  CohArgs a;
  a.ray_state = ptr<uint8_t>(c->ray_state);
  a.seg_o = ptr<float4>(c->seg_o);
  a.seg_d = ptr<float4>(c->seg_d);
  a.face_log = ptr<int32_t>(c->face_log);
  a.face_object = ptr<int32_t>(c->face_object);
  a.obj_box = ptr<float>(c->obj_box);
  a.n_obj = c->no;
  a.n_work = (int)((int64_t)c->n_src * c->n_branch * c->n_rays);
  a.tx = ptr<float>(c->src_pos);
  a.n_rays = c->n_rays * c->n_branch;   // work items per source (the segment-0 origin)
  a.margin = 1e-3f + c->pad;
  a.restart = ptr<uint8_t>(c->invalid_flag);
  a.list = ptr<uint32_t>(c->work_list);
  a.counters = c->cnt_dev;
  return a;
}

// dynamic LDS of the revalidation: the object grid and boxes (none beyond
// kCohGridObjects objects, which are then tested one by one), then the
// block's list of invalid rays
size_t coherence_lds(const dcem_ctx* c, int list_cap) {
  return (c->no <= kCohGridObjects
              ? sizeof(unsigned long long) * kCohGrid * kCohGrid * ((c->no + 63) / 64) + sizeof(float) * 6 * c->no
              : 0) +
         sizeof(uint32_t) * list_cap;
}

void launch_coherence(dcem_ctx* c) {
  CohArgs a = coherence_args(c);
  a.list_cap = kCohList;
  // four blocks per compute unit (each thread then checks several rays), and
  // at most kCohList rays per block
  const int blocks = (int)std::max<int64_t>(
      std::min<int64_t>((a.n_work + kCohBlock - 1) / kCohBlock, (int64_t)cu_count(c) * 4),
      (a.n_work + kCohList - 1) / kCohList);
  hipLaunchKernelGGL(k_coherence, dim3(std::max(blocks, 1)), dim3(kCohBlock), coherence_lds(c, a.list_cap), c->stream,
                     a);
}

void launch_refit_coherence(dcem_ctx* c, bool begin, const uint32_t* skip) {
  CohArgs ca = coherence_args(c);
  ca.list_cap = 2 * kCohList;
  const int n_rb = refit_blocks(c);
  // one revalidation block per compute unit the refit leaves free (the
  // refit's LDS allows one block of either kind per unit), at most
  // list_cap rays per block
  const int cb = (int)std::max<int64_t>(
      std::min<int64_t>((ca.n_work + kRefitBlock - 1) / kRefitBlock, std::max(cu_count(c) - n_rb, 1)),
      (ca.n_work + ca.list_cap - 1) / ca.list_cap);
  RefitArgs ra = make_refit_args(c, true, c->sah_dev + 1);
  ra.skip = skip;
  FrameBegin fb = frame_begin_args(c, c->last_los);
  fb.skip = skip;
  hipLaunchKernelGGL(k_refit_coherence, dim3(n_rb + std::max(cb, 1)), dim3(kRefitBlock),
                     coherence_lds(c, ca.list_cap), c->stream, ra, ca, n_rb, fb, begin ? 1 : 0);
  if (ra.cross_kernel) launch_refit_cross(c, ra, n_rb);
}

hipError_t build_ray_order(dcem_ctx* c) {
  const int64_t n = c->n_rays;
  hipError_t e;
  if ((e = ensure(c->ray_order, sizeof(uint32_t) * 3 * std::max<int64_t>(n, 1) + 16)) != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  uint32_t* order = ptr<uint32_t>(c->ray_order);
  uint32_t* tmp = order + n;
  uint32_t* key = tmp + n;
  uint32_t* n_dev = key + n;
  hipLaunchKernelGGL(k_dir_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, ptr<float>(c->dirs), n,
                     key);
  const uint32_t n32 = (uint32_t)n;
  if ((e = hipMemcpyAsync(n_dev, &n32, 4, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return e;
  if ((e = radix_sort_perm(c, key, 1, 32, n_dev, n, order, tmp, c->stream)) != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

}  // namespace dcem
