// Bottom-up refit of the binary and the 4-wide tree, shared by the refit
// kernel and the frame kernel that runs it beside the revalidation pass.
#pragma once

#include "dcem_internal.h"

#include <cfloat>
#include <type_traits>

namespace dcem {

struct RefitArgs {
  const float* V;
  const int32_t* T;
  const int32_t* tri_face;
  const int32_t* face_object;
  const int32_t* leaf_tri;
  const int32_t* leaf_parent;
  Node* nodes;
  uint32_t* cnt;              // device-wide arrival counters (cross nodes, when not two-phase)
  float* root_box;
  int n;                      // leaves
  int n_internal;
  float pad;
  bool wide;                  // also update the 4-wide tree
  const int32_t* slot4;
  const int32_t* leaf_slot;
  Node4* nodes4;
  Leaf* tri4;
  const int32_t* cross_index; // [n_internal]
  const int32_t* cross_list;  // [n_cross]
  const int32_t* cross_parent;
  uint32_t* entries;          // binary slots of cross nodes filled by the block pass
  uint32_t* info;             // [2] cross nodes, [3] entries, [4] finished blocks
  double* part;               // per-block surface-area sums
  double* sah_out;            // SAH ratio of the refitted tree
  const int32_t* face_ref_tri;
  int nf;
  double4* plane;             // per face: unit normal and offset
  bool cross_kernel;          // the cross nodes and the SAH sum are finished by k_refit_cross (large trees)
  const uint32_t* skip;       // nullable: a nonzero word here (read at launch) makes the launch do nothing
};

// Trees with more leaves than this finish their cross nodes in a launch of
// their own (one block; cross nodes beyond the LDS capacity climb through
// device memory with workgroup-scope arrivals) instead of in the refit's last
// block, which would otherwise fall back to device-scope arrivals.
constexpr int64_t kCrossKernelLeaves = 512 * 1024;

// Arguments of a refit of the current tree (`wide`: also the 4-wide tree in
// place), its SAH ratio written to sah_out.
RefitArgs make_refit_args(dcem_ctx* c, bool wide, double* sah_out);
// Refit blocks of the current tree.
int refit_blocks(const dcem_ctx* c);
// The cross-node pass of a large tree's refit (a.cross_kernel), after the
// launch that ran its block pass: its listed slots climb on the threads of
// several blocks, and the last block to finish sums the SAH areas.
void launch_refit_cross(dcem_ctx* c, const RefitArgs& a, int n_rb);

namespace {

__device__ inline float3 load_v(const float* v, int i) { return make_float3(v[3 * i], v[3 * i + 1], v[3 * i + 2]); }


// Binary slot 0 is floats 0-5 of the node (b0, b1.xy), slot 1 floats 6-11
// (b1.zw, b2): two vector stores each.
__device__ inline void store_slot(Node* nd, int slot, const float* lo, const float* hi) {
  if (slot == 0) {
    nd->b0 = make_float4(lo[0], lo[1], lo[2], hi[0]);
    *reinterpret_cast<float2*>(&nd->b1.x) = make_float2(hi[1], hi[2]);
  } else {
    *reinterpret_cast<float2*>(&nd->b1.z) = make_float2(lo[0], lo[1]);
    nd->b2 = make_float4(lo[2], hi[0], hi[1], hi[2]);
  }
}

__device__ inline void load_slot_coherent(Node* nd, int slot, float* lo, float* hi) {
  float* f = reinterpret_cast<float*>(nd);
  const int base = slot * 6;
  for (int a = 0; a < 3; ++a) {
    lo[a] = __hip_atomic_load(f + base + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hi[a] = __hip_atomic_load(f + base + 3 + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

constexpr int kRefitBlock = 1024;

// Leaf record of triangle `tri` (vertices; id, face and moving flag in w).
__device__ inline Leaf leaf_record(const float* __restrict__ V, const int32_t* __restrict__ T,
                                   const int32_t* __restrict__ tri_face, const int32_t* __restrict__ face_object,
                                   int tri) {
  const float3 a = load_v(V, T[3 * tri]), b = load_v(V, T[3 * tri + 1]), c = load_v(V, T[3 * tri + 2]);
  const int face = tri_face[tri];
  Leaf L;
  L.v0 = make_float4(a.x, a.y, a.z, __int_as_float(tri));
  L.v1 = make_float4(b.x, b.y, b.z, __int_as_float(face));
  L.v2 = make_float4(c.x, c.y, c.z, __int_as_float(face_object[face] >= 0 ? 1 : 0));
  return L;
}

__device__ inline void store_box4(Slot4* sl, const float* lo, const float* hi) {
  *reinterpret_cast<float3*>(&sl->lx) = make_float3(lo[0], lo[1], lo[2]);
  *reinterpret_cast<float3*>(&sl->hx) = make_float3(hi[0], hi[1], hi[2]);
}

__device__ inline double box_area(const float* lo, const float* hi) {
  double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
  return 2.0 * (dx * dy + dy * dz + dz * dx);
}

// Unit normal n and offset n . a of the plane through a, b, c (FP64:
// n = (b - a) x (c - a) normalised).
__device__ inline double4 plane_of(const float3& a, const float3& b, const float3& c) {
  const double ax = a.x, ay = a.y, az = a.z;
  const double ux = (double)b.x - ax, uy = (double)b.y - ay, uz = (double)b.z - az;
  const double vx = (double)c.x - ax, vy = (double)c.y - ay, vz = (double)c.z - az;
  double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  const double l = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= l;
  ny /= l;
  nz /= l;
  return make_double4(nx, ny, nz, nx * ax + ny * ay + nz * az);
}

// The plane of face f, from the face's reference triangle t.
__device__ inline void face_plane(const float* __restrict__ V, const int32_t* __restrict__ T, int t,
                                  double4* __restrict__ plane, int f) {
  plane[f] = plane_of(load_v(V, T[3 * t]), load_v(V, T[3 * t + 1]), load_v(V, T[3 * t + 2]));
}


// A child box of binary node `p2 >> 1` (slot p2 & 1): in the binary tree and,
// refitting a collapsed tree, in the 4-wide slot d that holds it (slot4[p2]).
__device__ inline void put_child_box(const RefitArgs& a, int p2, int d, const float* lo, const float* hi) {
  store_slot(&a.nodes[p2 >> 1], p2 & 1, lo, hi);
  if (a.wide && d >= 0) store_box4(&a.nodes4[d >> 2].s[d & 3], lo, hi);
}

constexpr int kMaxCross = 1024;   // cross nodes finished in LDS by the last block

// Arrival at a node whose two child boxes meet in LDS: the count of earlier
// arrivals.  The boxes are exchanged through LDS only, so the ordering is an
// LDS-only release and acquire (no wait for the global box stores of the
// level, which only the last block reads, after the device-scope ticket).
__device__ inline uint32_t lds_arrive(uint32_t* cnt) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  const uint32_t old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  return old;
}

// Sum of v over the block (kRefitBlock threads), valid in thread 0, in a fixed
// order: butterflies within each wavefront, then the wavefronts' sums in order.
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();   // red may still be read by an earlier sum
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kRefitBlock / kWave; ++w) t += red[w];
  return t;
}

// The links of cross node k (fixed between builds): its parent entry, its
// binary node, that node's children and their 4-wide slots.
struct CrossLinks {
  int par, node;
  int2 kid, s4;
};

__device__ inline CrossLinks cross_links(const RefitArgs& a, uint32_t k) {
  CrossLinks x;
  x.par = a.cross_parent[k];
  x.node = a.cross_list[k];
  x.kid = make_int2(a.nodes[x.node].c.x, a.nodes[x.node].c.y);
  x.s4 = a.wide ? make_int2(a.slot4[2 * x.node], a.slot4[2 * x.node + 1]) : make_int2(-1, -1);
  return x;
}

// Last-block pass of the refit: finish the cross nodes in LDS, from the slots
// the block pass listed up to the root.  With `have`, pre holds this thread's
// first cross node's links (loaded ahead).
__device__ __forceinline__ void finish_cross_nodes(const RefitArgs& a, uint32_t n_cross, float (*lbox)[12], uint32_t* lcnt,
                                   int32_t* lpar, int32_t* lnode, int2* lslot4, int2* lkid, bool have,
                                   const CrossLinks& pre) {
  const int tid = threadIdx.x;
  const uint32_t n_ent = __hip_atomic_load(&a.info[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t k = tid; k < n_cross; k += kRefitBlock) {
    const CrossLinks x = have && k == (uint32_t)tid ? pre : cross_links(a, k);
    lcnt[k] = 0;
    lpar[k] = x.par;
    lnode[k] = x.node;
    lkid[k] = x.kid;
    if (a.wide) lslot4[k] = x.s4;
  }
  __syncthreads();
  if (tid == 0) a.info[3] = 0;   // ready for the next refit
  for (uint32_t e = tid; e < n_ent; e += kRefitBlock) {
    const int p2 = (int)__hip_atomic_load(&a.entries[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int k = a.cross_index[p2 >> 1], slot = p2 & 1;
    float lo[3], hi[3];
    load_slot_coherent(&a.nodes[p2 >> 1], slot, lo, hi);
    int kp = lpar[k];
    for (uint32_t guard = n_cross + 1; guard > 0; --guard) {
      // the parent's links (written before the climb, never by it) are read
      // while this level's box is stored and the arrival counted
      int kpp = -1, pnode = 0;
      int2 ds = make_int2(-1, -1);
      if (kp >= 0) {
        kpp = lpar[kp >> 1];
        pnode = lnode[kp >> 1];
        if (a.wide) ds = lslot4[kp >> 1];
      }
      float* bx = lbox[k] + 6 * slot;
      for (int q = 0; q < 3; ++q) { bx[q] = lo[q]; bx[3 + q] = hi[q]; }
      const uint32_t old = lds_arrive(&lcnt[k]);
      if (old == 0) break;
      const float* sb = lbox[k] + 6 * (slot ^ 1);
      for (int q = 0; q < 3; ++q) {
        lo[q] = fminf(lo[q], sb[q]);
        hi[q] = fmaxf(hi[q], sb[3 + q]);
      }
      if (kp < 0) {
        for (int q = 0; q < 3; ++q) { a.root_box[q] = lo[q]; a.root_box[3 + q] = hi[q]; }
        break;
      }
      k = kp >> 1;
      slot = kp & 1;
      put_child_box(a, (pnode << 1) | slot, slot ? ds.y : ds.x, lo, hi);
      kp = kpp;
    }
  }
}

// Cross nodes finished in device memory by the blocks of the cross pass:
// every slot the block pass listed climbs through the cross nodes above it
// (the slots spread over the launch's threads); the second arrival at a node
// (device-scope counter) forms the union and writes it into the parent's
// slot.  Arrival counters are reset for the next refit.
__device__ __forceinline__ void climb_cross_global(const RefitArgs& a) {
  const uint32_t n_ent = __hip_atomic_load(&a.info[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // a thread's listed slots are loaded ahead: while one climbs, the next
  // one's box (written by the block pass, never by this climb) and the one
  // after's slot index are in flight
  const uint32_t step = gridDim.x * blockDim.x;
  const uint32_t e0 = blockIdx.x * blockDim.x + threadIdx.x;
  int p2_cur = 0, p2_next = 0;
  float lo_cur[3] = {0.f, 0.f, 0.f}, hi_cur[3] = {0.f, 0.f, 0.f};
  if (e0 < n_ent) p2_cur = (int)a.entries[e0];
  if (e0 + step < n_ent) p2_next = (int)a.entries[e0 + step];
  if (e0 < n_ent) load_slot_coherent(&a.nodes[p2_cur >> 1], p2_cur & 1, lo_cur, hi_cur);
  for (uint32_t e = e0; e < n_ent; e += step) {
    int p2 = p2_cur;
    float lo[3] = {lo_cur[0], lo_cur[1], lo_cur[2]}, hi[3] = {hi_cur[0], hi_cur[1], hi_cur[2]};
    if (e + step < n_ent) load_slot_coherent(&a.nodes[p2_next >> 1], p2_next & 1, lo_cur, hi_cur);
    p2_cur = p2_next;
    if (e + 2 * step < n_ent) p2_next = (int)a.entries[e + 2 * step];
    for (int guard = a.n_internal + 1; guard > 0; --guard) {
      const int node = p2 >> 1, slot = p2 & 1;
      // the parent link (fixed between builds) is read while the arrival is counted
      const int pp = a.nodes[node].c.z;
      const uint32_t old = __hip_atomic_fetch_add(&a.cnt[node], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (old == 0) break;
      a.cnt[node] = 0;
      float slo[3], shi[3];
      load_slot_coherent(&a.nodes[node], slot ^ 1, slo, shi);
      for (int k = 0; k < 3; ++k) {
        lo[k] = fminf(lo[k], slo[k]);
        hi[k] = fmaxf(hi[k], shi[k]);
      }
      if (pp < 0) {
        for (int k = 0; k < 3; ++k) { a.root_box[k] = lo[k]; a.root_box[3 + k] = hi[k]; }
        break;
      }
      put_child_box(a, pp, a.wide ? a.slot4[pp] : -1, lo, hi);
      p2 = pp;
    }
  }
}

__device__ __forceinline__ void refit_tail(const RefitArgs& a, int n_rb, bool lds, uint32_t n_cross,
                                           float (*lbox)[12], int2* lkid, double* red);

// Bottom-up refit over a fixed topology, in two passes of one kernel.
// Block pass: one thread per leaf writes its padded box into its parent's
// slot; the second thread to arrive at a node forms the union and climbs on.
// An internal node covers a contiguous range of sorted leaves and is one end
// of it, so a node whose range lies inside this block's 1024 leaves has both
// children here: its boxes, arrival counter and parent link live in LDS.  A
// thread stops at the first cross node (range spanning blocks), leaving its
// box in that node's slot and the slot in a list.  Last-block pass: the last
// block to finish finishes every cross node the same way in LDS, from the
// listed slots up to the root.  (With more cross nodes than LDS holds, cross
// nodes use device-wide arrival counters in the block pass instead.)  Boxes
// are min/max of FP32 values: the result does not depend on the order of
// arrival.  With `wide` (a refit of a collapsed tree) every child box stored
// in a binary slot is also stored in the 4-wide slot that holds it and the leaf
// thread writes its triangle to its slot, so no separate collapse is needed.
// The same kernel measures the tree: the surface areas of the internal nodes
// below the root (each node's internal children), summed per block in a fixed
// order and over blocks by the last block, over the root's area (sah_out); and
// it computes every face's plane (used by the refinement's image method).
// rb and n_rb: this block's index among the refit blocks and their number (the
// refit may share a launch with other work).
__device__ __forceinline__ void refit_block(const RefitArgs& a, int rb, int n_rb) {
  // block pass: slot boxes, counters, parent links and cross flags of the
  // block's nodes; last-block pass: the same for the cross nodes
  __shared__ float lbox[kRefitBlock][12];
  __shared__ uint32_t lcnt[kRefitBlock];
  __shared__ int32_t lpar[kRefitBlock];
  __shared__ int32_t lnode[kRefitBlock];
  __shared__ int2 lslot4[kRefitBlock];   // the 4-wide slots of the node's two child boxes
  __shared__ int2 lkid[kRefitBlock];     // child entries (>= 0: internal)
  __shared__ double red[kRefitBlock / kWave];
  __shared__ bool last;
  const int b0 = rb * kRefitBlock;
  const int tid = threadIdx.x;
  const uint32_t n_cross = a.info[2];
  const bool two_phase = a.cross_kernel || n_cross <= (uint32_t)kMaxCross;   // cross slots listed
  // Thread tid of the block holds node, leaf and face b0 + tid.  Their three
  // dependent gathers (index, vertex indices, vertices) are issued together,
  // so the climb starts three memory round trips after the launch instead of
  // seven.
  const int node = b0 + tid, i = b0 + tid, f = b0 + tid;
  const bool ok = node < a.n_internal, has_leaf = i < a.n, has_face = f < a.nf;
  const int lt = has_leaf ? a.leaf_tri[i] : 0;
  const int ls = has_leaf && a.wide ? a.leaf_slot[i] : 0;
  const int ft = has_face ? a.face_ref_tri[f] : 0;
  const int4 nc = ok ? a.nodes[node].c : make_int4(-1, -1, -1, 0);
  const bool local_node = ok && a.cross_index[node] < 0;
  const int2 s4 = a.wide && ok ? make_int2(a.slot4[2 * node], a.slot4[2 * node + 1]) : make_int2(-1, -1);
  int lv[3] = {0, 0, 0}, fv[3] = {0, 0, 0}, lface = 0;
  if (has_leaf) {
    for (int k = 0; k < 3; ++k) lv[k] = a.T[3 * lt + k];
    lface = a.tri_face[lt];
  }
  if (has_face)
    for (int k = 0; k < 3; ++k) fv[k] = a.T[3 * ft + k];
  float3 lp[3], fp[3];
  int lmoving = 0;
  for (int k = 0; k < 3; ++k) {
    lp[k] = has_leaf ? load_v(a.V, lv[k]) : make_float3(0.f, 0.f, 0.f);
    fp[k] = has_face ? load_v(a.V, fv[k]) : make_float3(0.f, 0.f, 0.f);
  }
  if (has_leaf) lmoving = a.face_object[lface] >= 0 ? 1 : 0;
  // the cross nodes' links, loaded by every block with its own gathers: the
  // block that finishes last has them at once
  const bool have_links = two_phase && !a.cross_kernel && (uint32_t)tid < n_cross;
  const CrossLinks links = have_links ? cross_links(a, tid) : CrossLinks{0, 0, make_int2(-1, -1), make_int2(-1, -1)};
  lcnt[tid] = 0;
  lpar[tid] = ok ? nc.z : -1;
  lnode[tid] = local_node;   // block-local
  lkid[tid] = ok ? make_int2(nc.x, nc.y) : make_int2(-1, -1);
  if (a.wide && ok) lslot4[tid] = s4;
  if (has_face) a.plane[f] = plane_of(fp[0], fp[1], fp[2]);
  // faces beyond one per thread (none when the refit has a thread per
  // triangle: every face holds a triangle)
  for (int g = f + n_rb * kRefitBlock; g < a.nf; g += n_rb * kRefitBlock)
    face_plane(a.V, a.T, a.face_ref_tri[g], a.plane, g);
  __syncthreads();
  if (has_leaf) {
    Leaf L;
    L.v0 = make_float4(lp[0].x, lp[0].y, lp[0].z, __int_as_float(lt));
    L.v1 = make_float4(lp[1].x, lp[1].y, lp[1].z, __int_as_float(lface));
    L.v2 = make_float4(lp[2].x, lp[2].y, lp[2].z, __int_as_float(lmoving));
    if (a.wide) a.tri4[ls] = L;
    float lo[3] = {fminf(L.v0.x, fminf(L.v1.x, L.v2.x)) - a.pad, fminf(L.v0.y, fminf(L.v1.y, L.v2.y)) - a.pad,
                   fminf(L.v0.z, fminf(L.v1.z, L.v2.z)) - a.pad};
    float hi[3] = {fmaxf(L.v0.x, fmaxf(L.v1.x, L.v2.x)) + a.pad, fmaxf(L.v0.y, fmaxf(L.v1.y, L.v2.y)) + a.pad,
                   fmaxf(L.v0.z, fmaxf(L.v1.z, L.v2.z)) + a.pad};
    if (a.n == 1) {   // the root holds the one leaf in both slots
      put_child_box(a, 0, 0, lo, hi);
      put_child_box(a, 1, 1, lo, hi);
      if (a.wide) a.tri4[1] = L;
      for (int k = 0; k < 3; ++k) { a.root_box[k] = lo[k]; a.root_box[3 + k] = hi[k]; }
    } else {
      // the climb, compiled apart for the two-phase case (the usual one), so
      // that its in-block levels contain no global load to wait for
      auto climb = [&](auto two_phase_t) {
        constexpr bool kTwoPhase = decltype(two_phase_t)::value;
        int p2 = a.leaf_parent[i];
        // the leaf's loads are complete before the loop (vmcnt 0): otherwise
        // the wait for them sits at the loop head and every level would wait
        // for the previous level's box stores as well
        if (kTwoPhase) __builtin_amdgcn_s_waitcnt(0x0f70);
        for (int guard = a.n; guard > 0; --guard) {   // depth < n in a sound tree
          const int node = p2 >> 1, slot = p2 & 1;
          // the node's links in LDS (written before the climb, never by it),
          // read together
          const bool in_block = node >= b0 && node < b0 + kRefitBlock;
          const int li = in_block ? node - b0 : 0;
          const bool local = in_block && lnode[li];
          const int2 ds = lslot4[li];
          const int par = lpar[li];
          float slo[3], shi[3];
          if (local) {
            put_child_box(a, p2, a.wide ? (slot ? ds.y : ds.x) : -1, lo, hi);
            float* bx = lbox[node - b0] + 6 * slot;
            for (int k = 0; k < 3; ++k) { bx[k] = lo[k]; bx[3 + k] = hi[k]; }
            if (lds_arrive(&lcnt[node - b0]) == 0) break;
            const float* sb = lbox[node - b0] + 6 * (slot ^ 1);
            for (int k = 0; k < 3; ++k) { slo[k] = sb[k]; shi[k] = sb[3 + k]; }
          } else if (kTwoPhase) {
            // a cross node: its slot, listed, is finished by the last block
            put_child_box(a, p2, a.wide ? a.slot4[p2] : -1, lo, hi);
            a.entries[atomicAdd(&a.info[3], 1u)] = (uint32_t)p2;
            break;
          } else {
            put_child_box(a, p2, a.wide ? a.slot4[p2] : -1, lo, hi);
            const uint32_t old = __hip_atomic_fetch_add(&a.cnt[node], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (old == 0) break;
            a.cnt[node] = 0;
            load_slot_coherent(&a.nodes[node], slot ^ 1, slo, shi);
          }
          for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], slo[k]);
            hi[k] = fmaxf(hi[k], shi[k]);
          }
          if (kTwoPhase) p2 = par;   // local here
          else p2 = local ? par : a.nodes[node].c.z;
          if (p2 < 0) {
            for (int k = 0; k < 3; ++k) { a.root_box[k] = lo[k]; a.root_box[3 + k] = hi[k]; }
            break;
          }
        }
      };
      if (two_phase) climb(std::true_type{});
      else climb(std::false_type{});
    }
  }
  __syncthreads();
  // areas of the internal children of this block's local nodes
  {
    double ar = 0.0;
    if (lnode[tid]) {
      if (lkid[tid].x >= 0) ar += box_area(lbox[tid], lbox[tid] + 3);
      if (lkid[tid].y >= 0) ar += box_area(lbox[tid] + 6, lbox[tid] + 9);
    }
    ar = block_sum(ar, red);
    if (a.cross_kernel) {   // k_refit_cross finishes, after this launch
      if (tid == 0) a.part[rb] = ar;
      return;
    }
    if (tid == 0) {
      __hip_atomic_store(&a.part[rb], ar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&a.info[4], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)n_rb - 1;
    }
    __syncthreads();
  }
  if (!last) return;
  // ---- the last block to finish completes the cross nodes and the SAH sum
  if (tid == 0) a.info[4] = 0;   // ready for the next refit
  if (two_phase && n_cross > 0)
    finish_cross_nodes(a, n_cross, lbox, lcnt, lpar, lnode, lslot4, lkid, have_links, links);
  __syncthreads();
  refit_tail(a, n_rb, two_phase, n_cross, lbox, lkid, red);
}

// The cross nodes and the SAH ratio of a large tree, after the refit's block
// pass: in LDS by block 0 when they fit, else climbed by every block in device
// memory, the SAH sum then by the last block to finish.
__device__ __forceinline__ void refit_cross_block(const RefitArgs& a, int n_rb) {
  __shared__ float lbox[kRefitBlock][12];
  __shared__ uint32_t lcnt[kRefitBlock];
  __shared__ int32_t lpar[kRefitBlock];
  __shared__ int32_t lnode[kRefitBlock];
  __shared__ int2 lslot4[kRefitBlock];
  __shared__ int2 lkid[kRefitBlock];
  __shared__ double red[kRefitBlock / kWave];
  __shared__ bool last;
  const uint32_t n_cross = a.info[2];
  const bool lds = n_cross <= (uint32_t)kMaxCross;
  if (lds) {
    if (blockIdx.x != 0) return;   // uniform
    if (n_cross > 0) finish_cross_nodes(a, n_cross, lbox, lcnt, lpar, lnode, lslot4, lkid, false, CrossLinks{});
  } else {
    climb_cross_global(a);
    __threadfence();   // this thread's box stores before the block's ticket
    __syncthreads();
    if (threadIdx.x == 0)
      last = __hip_atomic_fetch_add(&a.info[4], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;   // uniform
    __threadfence();     // every block's climbs before the sums
    if (threadIdx.x == 0) {
      a.info[3] = 0;   // ready for the next refit
      a.info[4] = 0;
    }
  }
  __syncthreads();
  refit_tail(a, n_rb, lds, n_cross, lbox, lkid, red);
}

// SAH ratio of a refitted tree: areas of the cross nodes' internal children
// (from LDS when `lds`, else from the binary nodes) plus the blocks' sums,
// over the root's area; written by thread 0.
__device__ __forceinline__ void refit_tail(const RefitArgs& a, int n_rb, bool lds, uint32_t n_cross,
                                           float (*lbox)[12], int2* lkid, double* red) {
  const int tid = threadIdx.x;
  const bool two_phase = lds;
  // areas of the cross nodes' internal children (in LDS after the two-phase
  // pass, else in the binary nodes), plus the blocks' sums
  double ar = 0.0;
  for (uint32_t k = tid; k < n_cross; k += kRefitBlock) {
    if (two_phase) {
      if (lkid[k].x >= 0) ar += box_area(lbox[k], lbox[k] + 3);
      if (lkid[k].y >= 0) ar += box_area(lbox[k] + 6, lbox[k] + 9);
      continue;
    }
    const int node = a.cross_list[k];
    float lo[3], hi[3];
    if (a.nodes[node].c.x >= 0) {
      load_slot_coherent(&a.nodes[node], 0, lo, hi);
      ar += box_area(lo, hi);
    }
    if (a.nodes[node].c.y >= 0) {
      load_slot_coherent(&a.nodes[node], 1, lo, hi);
      ar += box_area(lo, hi);
    }
  }
  for (unsigned b = tid; b < (unsigned)n_rb; b += kRefitBlock)
    ar += __hip_atomic_load(&a.part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double t = block_sum(ar, red);
  if (tid != 0) return;
  float rlo[3], rhi[3];
  for (int q = 0; q < 3; ++q) {
    rlo[q] = __hip_atomic_load(&a.root_box[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    rhi[q] = __hip_atomic_load(&a.root_box[3 + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const double root = box_area(rlo, rhi);
  *a.sah_out = root > 0 ? (t + root) / root : 1.0;
}

}  // namespace
}  // namespace dcem
