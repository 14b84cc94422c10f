// Moving-object transforms, LBVH construction and bottom-up refit.
//
// The paper keeps a BVH over the scene and updates it every frame, rebuilding
// only when its quality has degraded (Sec. III, "Efficient BVH updating").
// Here the tree is a linear BVH (Morton-ordered triangles, hierarchy from the
// longest common prefixes of the sorted codes, one thread per internal node),
// refit bottom-up with arrival counters, and scored by the SAH surface-area
// sum relative to the last build.
#include "dcem_internal.h"
#include "refit.h"

#include <cfloat>

namespace dcem {
namespace {

__device__ inline uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// x' = R x + t for one row: the FP32 x FP32 products are exact in FP64 and are
// summed left to right, then rounded once to FP32.
__device__ inline float xform_row(const float* m, float x, float y, float z) {
  double r = (double)m[0] * (double)x;
  r = r + (double)m[1] * (double)y;
  r = r + (double)m[2] * (double)z;
  r = r + (double)m[3];
  return (float)r;
}

// One block per moving object: transform its vertex range and reduce its
// world-space box (padded by `pad`, used by the coherence test).
__global__ void k_xform(const float* __restrict__ ref, float* __restrict__ out,
                        const int64_t* __restrict__ range, const float* __restrict__ xf,
                        float* __restrict__ obj_box, float pad, uint32_t* err) {
  const int o = blockIdx.x;
  const int64_t b = range[2 * o], e = range[2 * o + 1];
  const float* m = xf + 12 * o;
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  bool bad = false;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    float x = ref[3 * i], y = ref[3 * i + 1], z = ref[3 * i + 2];
    float w[3] = {xform_row(m, x, y, z), xform_row(m + 4, x, y, z), xform_row(m + 8, x, y, z)};
    for (int a = 0; a < 3; ++a) {
      out[3 * i + a] = w[a];
      lo[a] = fminf(lo[a], w[a]);
      hi[a] = fmaxf(hi[a], w[a]);
      bad |= !isfinite(w[a]);
    }
  }
  if (bad) atomicOr(err, DCEM_ERR_NONFINITE);
  __shared__ float red[6][256];
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) {
    float v = red[threadIdx.x][0];
    obj_box[6 * o + threadIdx.x] = threadIdx.x < 3 ? v - pad : v + pad;
  }
}

// Clear the centroid bounds (ordered bits) and store the item count next to them.
__global__ void k_box_init(uint32_t* box, uint32_t n) {
  if (threadIdx.x < 3) box[threadIdx.x] = 0xffffffffu;
  else if (threadIdx.x < 6) box[threadIdx.x] = 0u;
  else if (threadIdx.x == 6) box[6] = n;
}

__global__ void k_set2(uint32_t* p, uint32_t a, uint32_t* q, uint32_t b) {
  if (threadIdx.x == 0) {
    *p = a;
    *q = b;
  }
}

// Bounds of the triangle centroids (exact min/max through order-preserving bits).
__global__ void k_centroid_bounds(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nt,
                                  uint32_t* box) {
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nt; i += (int64_t)gridDim.x * blockDim.x) {
    float3 a = load_v(V, T[3 * i]), b = load_v(V, T[3 * i + 1]), c = load_v(V, T[3 * i + 2]);
    float cx = (a.x + b.x + c.x) * (1.0f / 3.0f), cy = (a.y + b.y + c.y) * (1.0f / 3.0f),
          cz = (a.z + b.z + c.z) * (1.0f / 3.0f);
    lo[0] = fminf(lo[0], cx); lo[1] = fminf(lo[1], cy); lo[2] = fminf(lo[2], cz);
    hi[0] = fmaxf(hi[0], cx); hi[1] = fmaxf(hi[1], cy); hi[2] = fmaxf(hi[2], cz);
  }
  // wave reduction, then block reduction, then one set of atomics per block
  // (device-scope atomics on six addresses: fewer of them contend less)
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], off));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off));
    }
  }
  __shared__ float wred[6][1024 / 64];
  const int nw = (int)blockDim.x / 64, wv = (int)threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      wred[a][wv] = lo[a];
      wred[3 + a][wv] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w)
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], wred[a][w]);
        hi[a] = fmaxf(hi[a], wred[3 + a][w]);
      }
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[a], ordered_bits(lo[a]));
      atomicMax(&box[3 + a], ordered_bits(hi[a]));
    }
  }
}

__device__ inline uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton code of point p inside the box (lo, lo + ext).
__device__ inline uint32_t morton30(const float* p, const float* lo, const float* ext) {
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    float u = (p[k] - lo[k]) / ext[k];
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    q[k] = (uint32_t)fminf(u * 1024.0f, 1023.0f);
  }
  return (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

__device__ inline void bounds_of(const uint32_t* box, float* lo, float* ext) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = from_ordered(box[a]);
    const float h = from_ordered(box[3 + a]);
    ext[a] = h > lo[a] ? h - lo[a] : 1.0f;
  }
}

// Morton code of each moving object's box centre in the centroid bounds.
__global__ void k_object_codes(const float* __restrict__ obj_box, int no, const uint32_t* __restrict__ box,
                               uint32_t* __restrict__ ocode) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= no) return;
  float lo[3], ext[3], p[3];
  bounds_of(box, lo, ext);
  for (int a = 0; a < 3; ++a) p[a] = 0.5f * (obj_box[6 * o + a] + obj_box[6 * o + 3 + a]);
  ocode[o] = morton30(p, lo, ext);
}

// Rank of each moving object in the order of its code (ties by object id).
__global__ void k_object_rank(const uint32_t* __restrict__ ocode, int no, int32_t* __restrict__ rank) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= no) return;
  const uint32_t mine = ocode[o];
  int r = 0;
  for (int j = 0; j < no; ++j) {
    const uint32_t cj = ocode[j];
    r += (cj < mine || (cj == mine && j < o)) ? 1 : 0;
  }
  rank[o] = r;
}

// Group of a face: its moving object, or -1 for static geometry (and for
// every face when the objects are not separated: orank null).  Group prefix:
// 0 for group -1, else 1 << rank_bits | the object's spatial rank.
__device__ inline int face_group(const int32_t* face_object, const int32_t* orank, int f) {
  return orank ? face_object[f] : -1;
}
__device__ inline uint32_t group_prefix(const int32_t* face_object, const int32_t* orank, int rank_bits, int f) {
  const int obj = face_group(face_object, orank, f);
  return obj < 0 ? 0u : ((1u << rank_bits) | (uint32_t)orank[obj]);
}

// Box of each face (its triangles' vertices) and its sort key within the
// faces: group prefix << 30 | Morton code of the box centre in the group's box
// (the centroid bounds for static faces, the object's box for moving ones),
// as two words.  Thread 0 also stores the face count for the sort.
__global__ void k_face_keys(const float* __restrict__ V, const int32_t* __restrict__ T,
                            const int32_t* __restrict__ face_tri_off, const int32_t* __restrict__ face_tris, int nf,
                            const int32_t* __restrict__ face_object, const float* __restrict__ obj_box,
                            const int32_t* __restrict__ orank, int rank_bits, const uint32_t* __restrict__ box,
                            float* __restrict__ fbox, uint32_t* __restrict__ fkey_hi, uint32_t* __restrict__ fkey_lo,
                            uint32_t* __restrict__ n_faces) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f == 0) *n_faces = (uint32_t)nf;
  if (f >= nf) return;
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int k = face_tri_off[f]; k < face_tri_off[f + 1]; ++k) {
    const int t = face_tris[k];
    for (int v = 0; v < 3; ++v) {
      const float3 p = load_v(V, T[3 * t + v]);
      lo[0] = fminf(lo[0], p.x); lo[1] = fminf(lo[1], p.y); lo[2] = fminf(lo[2], p.z);
      hi[0] = fmaxf(hi[0], p.x); hi[1] = fmaxf(hi[1], p.y); hi[2] = fmaxf(hi[2], p.z);
    }
  }
  float glo[3], gext[3], c[3];
  bounds_of(box, glo, gext);
  const int obj = face_group(face_object, orank, f);
  if (obj >= 0)
    for (int k = 0; k < 3; ++k) {
      glo[k] = obj_box[6 * obj + k];
      const float h = obj_box[6 * obj + 3 + k];
      gext[k] = h > glo[k] ? h - glo[k] : 1.0f;
    }
  for (int k = 0; k < 3; ++k) {
    fbox[6 * f + k] = lo[k];
    fbox[6 * f + 3 + k] = hi[k];
    c[k] = lo[k] <= hi[k] ? 0.5f * (lo[k] + hi[k]) : glo[k];   // a face without triangles sorts first
  }
  const uint64_t key = ((uint64_t)group_prefix(face_object, orank, rank_bits, f) << 30) | morton30(c, glo, gext);
  fkey_hi[f] = (uint32_t)(key >> 32);
  fkey_lo[f] = (uint32_t)key;
}

// First sorted position of each group's faces.
__global__ void k_face_first(const uint32_t* __restrict__ fperm, int nf, const int32_t* __restrict__ face_object,
                             const int32_t* __restrict__ orank, int32_t* __restrict__ first) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nf) return;
  const int g = face_group(face_object, orank, (int)fperm[q]);
  if (q == 0 || face_group(face_object, orank, (int)fperm[q - 1]) != g) first[g + 1] = q;
}

// Rank of each face among its group's faces, in sorted order.
__global__ void k_face_rank(const uint32_t* __restrict__ fperm, int nf, const int32_t* __restrict__ face_object,
                            const int32_t* __restrict__ orank, const int32_t* __restrict__ first,
                            int32_t* __restrict__ frank) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nf) return;
  const int f = (int)fperm[q];
  frank[f] = q - first[face_group(face_object, orank, f) + 1];
}

// Sort key of each triangle.  key_hi null: the 30-bit Morton code of its
// centroid in the centroid bounds.  Otherwise the key is, from the most
// significant bit, the group prefix of its face (static geometry 0, a moving
// object 1 << rank_bits | the object's spatial rank; no prefix when the
// objects are not separated), the face's rank among its group's faces
// (face_bits bits, frank null: none) and the Morton code of the centroid in
// the face's box (frank null: in the object's box, or the centroid bounds).
// The hierarchy built from these keys holds the static geometry, every moving
// object and, inside those, every face in subtrees of their own: rigid motion
// leaves the objects' subtrees tight under refitting, and a planar face's
// triangles sit under a flat box.  Keys are stored as two words, key_hi (bits
// 63..32) and key_lo (bits 31..0).
__global__ void k_morton(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nt,
                         const uint32_t* __restrict__ box, const int32_t* __restrict__ tri_face,
                         const int32_t* __restrict__ face_object, const int32_t* __restrict__ orank, int rank_bits,
                         const int32_t* __restrict__ frank, int face_bits, const float* __restrict__ fbox,
                         const float* __restrict__ obj_box, uint32_t* __restrict__ key_hi,
                         uint32_t* __restrict__ key_lo) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nt) return;
  float lo[3], ext[3];
  bounds_of(box, lo, ext);
  float3 a = load_v(V, T[3 * i]), b = load_v(V, T[3 * i + 1]), c = load_v(V, T[3 * i + 2]);
  float p[3] = {(a.x + b.x + c.x) * (1.0f / 3.0f), (a.y + b.y + c.y) * (1.0f / 3.0f),
                (a.z + b.z + c.z) * (1.0f / 3.0f)};
  if (!key_hi) {
    key_lo[i] = morton30(p, lo, ext);
    return;
  }
  const int f = tri_face[i];
  const int obj = face_group(face_object, orank, f);
  const float* fb = fbox ? fbox + 6 * f : nullptr;   // without the face level: the object's box
  if (fb || obj >= 0) {
    if (!fb) fb = obj_box + 6 * obj;
    for (int k = 0; k < 3; ++k) {
      lo[k] = fb[k];
      ext[k] = fb[3 + k] > lo[k] ? fb[3 + k] - lo[k] : 1.0f;
    }
  }
  const uint64_t key = ((((uint64_t)group_prefix(face_object, orank, rank_bits, f) << face_bits) |
                         (uint64_t)(frank ? frank[f] : 0)) << 30) | morton30(p, lo, ext);
  key_hi[i] = (uint32_t)(key >> 32);
  key_lo[i] = (uint32_t)key;
}

// Longest common prefix of the sorted keys i and j (ties broken by index).
__device__ inline int lcp(const uint32_t* __restrict__ key_hi, const uint32_t* __restrict__ key_lo,
                          const uint32_t* __restrict__ perm, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t pi = perm[i], pj = perm[j];
  uint64_t a = key_lo[pi], b = key_lo[pj];
  if (key_hi) {
    a |= (uint64_t)key_hi[pi] << 32;
    b |= (uint64_t)key_hi[pj] << 32;
  }
  if (a != b) return __clzll((long long)(a ^ b));
  return 64 + __clz((uint32_t)(i ^ j));
}

// Hierarchy from the sorted Morton codes, one thread per internal node
// (Karras, "Maximizing parallelism in the construction of BVHs", 2012).
__global__ void k_karras(const uint32_t* __restrict__ key_hi, const uint32_t* __restrict__ key_lo,
                         const uint32_t* __restrict__ perm, int n,
                         Node* __restrict__ nodes, int32_t* __restrict__ leaf_parent,
                         int32_t* __restrict__ leaf_tri, int2* __restrict__ range) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) leaf_tri[i] = (int32_t)perm[i];
  if (i >= n - 1) return;
  int d = (lcp(key_hi, key_lo, perm, n, i, i + 1) - lcp(key_hi, key_lo, perm, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = lcp(key_hi, key_lo, perm, n, i, i - d);
  int lmax = 2;
  while (lcp(key_hi, key_lo, perm, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (lcp(key_hi, key_lo, perm, n, i, i + (l + t) * d) > dmin) l += t;
  int j = i + l * d;
  int dnode = lcp(key_hi, key_lo, perm, n, i, j);
  int s = 0;
  int t = l;
  do {
    t = (t + 1) >> 1;
    if (lcp(key_hi, key_lo, perm, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int gamma = i + s * d + min(d, 0);
  int lo = min(i, j), hi = max(i, j);
  range[i] = make_int2(lo, hi);
  int left = (lo == gamma) ? ~gamma : gamma;
  int right = (hi == gamma + 1) ? ~(gamma + 1) : gamma + 1;
  nodes[i].c.x = left;
  nodes[i].c.y = right;
  nodes[i].c.w = 0;
  if (left < 0) leaf_parent[~left] = 2 * i;
  else nodes[left].c.z = 2 * i;
  if (right < 0) leaf_parent[~right] = 2 * i + 1;
  else nodes[right].c.z = 2 * i + 1;
  if (i == 0) nodes[0].c.z = -1;
}

// Binary nodes whose leaf range spans several refit blocks ("cross" nodes):
// listed once per build with their list index per node (-1 otherwise) and the
// list index and slot of their parent (the parent of a cross node is one too).
__global__ void k_cross_mark(const int2* __restrict__ range, int n_internal, int32_t* __restrict__ cross_index,
                             int32_t* __restrict__ cross_list, uint32_t* __restrict__ n_cross) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_internal) return;
  const int2 rg = range[i];
  if (rg.x / kRefitBlock == rg.y / kRefitBlock) {
    cross_index[i] = -1;
    return;
  }
  const uint32_t k = atomicAdd(n_cross, 1u);
  cross_index[i] = (int32_t)k;
  cross_list[k] = i;
}

__global__ void k_cross_parent(const Node* __restrict__ nodes, const int32_t* __restrict__ cross_index,
                               const int32_t* __restrict__ cross_list, const uint32_t* __restrict__ n_cross,
                               int n_internal, int32_t* __restrict__ cross_parent) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_internal || k >= (int)*n_cross) return;
  const int p2 = nodes[cross_list[k]].c.z;
  cross_parent[k] = p2 < 0 ? -1 : (cross_index[p2 >> 1] << 1) | (p2 & 1);
}

__global__ __launch_bounds__(kRefitBlock) void k_refit(RefitArgs a) { refit_block(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kRefitBlock) void k_refit_cross(RefitArgs a, int n_rb) {
  if (a.skip && *a.skip) return;   // uniform: the word does not change during the launch
  refit_cross_block(a, n_rb);
}





// scene_box layout: root box (6 floats, 2 spare), then the refit blocks'
// surface-area sums.
double* sah_parts(dcem_ctx* c) { return reinterpret_cast<double*>(ptr<char>(c->scene_box) + 8 * sizeof(float)); }

// Depth of each binary internal node (steps to the root) as a sort key: nodes
// at even depth become 4-wide nodes and are ordered by (depth, index), i.e.
// breadth-first; odd-depth nodes sort to the end.
__global__ void k_depth_keys(const Node* __restrict__ nodes, int n_internal, uint32_t* __restrict__ key,
                             uint32_t* __restrict__ n_even) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_internal) return;
  int d = 0, p2 = nodes[i].c.z;
  while (p2 >= 0 && d < n_internal) {
    ++d;
    p2 = nodes[p2 >> 1].c.z;
  }
  const bool even = (d & 1) == 0;
  key[i] = even ? ((uint32_t)d << 26) | (uint32_t)i : 0xffffffffu;
  if (even) atomicAdd(n_even, 1u);
}

// 4-wide node of each even-depth binary node (-1 for odd depth).
__global__ void k_map4(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ n4_dev, int n_internal,
                       int32_t* __restrict__ bvh2_of, int32_t* __restrict__ map4) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_internal) return;
  const int p = (int)perm[q];
  if (q < (int)*n4_dev) {
    bvh2_of[q] = p;
    map4[p] = q;
  } else {
    map4[p] = -1;
  }
}

// Leaf-slot mask of the 4-wide node made from binary node p: its slots are,
// in order, each leaf child of p, or the two children of each internal child
// of p; bit j is set when slot j is a leaf.
__device__ inline uint32_t slot_leaf_mask(const Node* __restrict__ nodes, int p) {
  uint32_t m = 0;
  int s = 0;
  const int cp[2] = {nodes[p].c.x, nodes[p].c.y};
  for (int i = 0; i < 2; ++i) {
    if (cp[i] < 0) {
      m |= 1u << s++;
    } else {
      if (nodes[cp[i]].c.x < 0) m |= 1u << s;
      ++s;
      if (nodes[cp[i]].c.y < 0) m |= 1u << s;
      ++s;
    }
  }
  return m;
}

// Fill every 4-wide node from its binary node p (after a build): a leaf child
// of p is one entry (box from p's slot); an internal child c of p contributes
// its two children (boxes from c's slots).  Also stores the leaf-slot masks of
// the node's child nodes (and the root's own mask in info[1]), the leaf
// triangles in slot order and, per sorted leaf, its slot (where refits write
// the moved triangle).
__global__ void k_collapse(const Node* __restrict__ nodes, const float* __restrict__ V,
                           const int32_t* __restrict__ T, const int32_t* __restrict__ tri_face,
                           const int32_t* __restrict__ face_object, const int32_t* __restrict__ leaf_tri,
                           const int32_t* __restrict__ bvh2_of, const int32_t* __restrict__ map4,
                           uint32_t* __restrict__ info, Node4* __restrict__ out, Leaf* __restrict__ tri4,
                           int32_t* __restrict__ leaf_slot, int32_t* __restrict__ slot4) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int)info[0]) return;
  const int p = bvh2_of[q];
  float lo[4][3], hi[4][3];
  int ch[4];
  int m = 0;
  uint32_t own = 0, kids = 0;   // leaf-slot masks of this node and (4 bits per slot) of its child nodes
  const float* fp = reinterpret_cast<const float*>(&nodes[p]);
  const int cp[2] = {nodes[p].c.x, nodes[p].c.y};
  for (int s = 0; s < 2; ++s) {
    const int c = cp[s];
    if (c < 0) {
      for (int a = 0; a < 3; ++a) { lo[m][a] = fp[6 * s + a]; hi[m][a] = fp[6 * s + 3 + a]; }
      own |= 1u << m;
      slot4[2 * p + s] = 4 * q + m;
      ch[m++] = c;
    } else {
      const float* fc = reinterpret_cast<const float*>(&nodes[c]);
      const int cc[2] = {nodes[c].c.x, nodes[c].c.y};
      slot4[2 * p + s] = -1;   // an internal child's box is not kept in the 4-wide tree
      for (int t = 0; t < 2; ++t) {
        slot4[2 * c + t] = 4 * q + m;
        for (int a = 0; a < 3; ++a) { lo[m][a] = fc[6 * t + a]; hi[m][a] = fc[6 * t + 3 + a]; }
        if (cc[t] < 0) {
          own |= 1u << m;
          ch[m++] = cc[t];
        } else {
          kids |= slot_leaf_mask(nodes, cc[t]) << (4 * m);
          ch[m++] = map4[cc[t]];
        }
      }
    }
  }
  for (int e = 0; e < m; ++e) {
    if (ch[e] >= 0) continue;
    tri4[4 * (size_t)q + e] = leaf_record(V, T, tri_face, face_object, leaf_tri[~ch[e]]);
    leaf_slot[~ch[e]] = 4 * q + e;
  }
  Node4 n;
  for (int e = 0; e < 4; ++e) {
    Slot4& sl = n.s[e];
    if (e < m) {
      sl.lx = lo[e][0]; sl.ly = lo[e][1]; sl.lz = lo[e][2];
      sl.hx = hi[e][0]; sl.hy = hi[e][1]; sl.hz = hi[e][2];
      sl.child = ch[e];
      sl.mask = (kids >> (4 * e)) & 15u;
    } else {
      sl.lx = sl.ly = sl.lz = sl.hx = sl.hy = sl.hz = 0.0f;
      sl.child = kEmpty;
      sl.mask = 0;
    }
  }
  if (q == 0) info[1] = own;
  out[q] = n;
}

}  // namespace

void launch_xform(dcem_ctx* c, const float* xf) {
  if (c->no == 0) return;
  hipLaunchKernelGGL(k_xform, dim3(c->no), dim3(256), 0, c->stream, ptr<float>(c->ref_vertices),
                     ptr<float>(c->vertices), ptr<int64_t>(c->obj_range), xf,
                     ptr<float>(c->obj_box), c->pad, c->err_dev);
}

// Build the binary LBVH and its 4-wide collapse, entirely on the stream (no
// host round trip).  The SAH sum ratio of the new tree goes to sah_dev[0].
__global__ void k_tri_slot(const int32_t* __restrict__ leaf_tri, const int32_t* __restrict__ leaf_slot, int n,
                           int32_t* __restrict__ tri_slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) tri_slot[leaf_tri[i]] = leaf_slot[i];
}

__global__ void k_face_slots(const int32_t* __restrict__ face_tris, const int32_t* __restrict__ tri_slot, int n,
                             int32_t* __restrict__ face_slots) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) face_slots[k] = tri_slot[face_tris[k]];
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// Replace the group prefix of every triangle's stored key (the group's
// spatial rank) and keep the rest (the face rank and the Morton code inside
// the group), so the keys order the groups by their current centres while
// each group's triangles keep their order.
__global__ void k_regroup_keys(const int32_t* __restrict__ tri_face, const int32_t* __restrict__ face_object,
                               const int32_t* __restrict__ orank, int rank_bits, int low_bits, int64_t nt,
                               uint32_t* __restrict__ key_hi, uint32_t* __restrict__ key_lo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const uint64_t low = (((uint64_t)key_hi[i] << 32) | key_lo[i]) & ((1ull << low_bits) - 1ull);
  const uint64_t key = ((uint64_t)group_prefix(face_object, orank, rank_bits, tri_face[i]) << low_bits) | low;
  key_hi[i] = (uint32_t)(key >> 32);
  key_lo[i] = (uint32_t)key;
}

hipError_t tree_from_keys(dcem_ctx* c, int key_words, int key_bits);

hipError_t rebuild_subtrees(dcem_ctx* c) {
  if (!c->keys_grouped || c->nt < 2) return build_lbvh(c, true);
  const int64_t nt = c->nt;
  const int no = c->no;
  const int key_words = c->key_words_built;
  uint32_t* code = ptr<uint32_t>(c->morton);
  uint32_t* key_hi = code;
  uint32_t* key_lo = code + (size_t)nt;
  uint32_t* nbox = code + (key_words + 2) * (size_t)nt;   // the last full build's centroid bounds
  uint32_t* ocode = nbox + 8;
  int32_t* orank = reinterpret_cast<int32_t*>(ocode + no);
  c->refit_since_build = false;
  c->pending_ratio = 1.0;
  hipLaunchKernelGGL(k_object_codes, dim3((no + 255) / 256), dim3(256), 0, c->stream, ptr<float>(c->obj_box), no,
                     nbox, ocode);
  hipLaunchKernelGGL(k_object_rank, dim3((no + 255) / 256), dim3(256), 0, c->stream, ocode, no, orank);
  const int low_bits = c->key_face_bits + 30;
  hipLaunchKernelGGL(k_regroup_keys, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, c->stream,
                     ptr<int32_t>(c->tri_face), ptr<int32_t>(c->face_object), orank, c->key_rank_bits, low_bits, nt,
                     key_hi, key_lo);
  return tree_from_keys(c, key_words, c->key_rank_bits + 1 + low_bits);
}

hipError_t build_lbvh(dcem_ctx* c, bool separate_objects) {
  const int64_t nt = c->nt;
  hipError_t e;
  c->n_internal = nt > 1 ? (int32_t)(nt - 1) : (nt == 1 ? 1 : 0);
  c->refit_since_build = false;
  c->pending_ratio = 1.0;
  if (nt == 0) {
    c->has_bvh = true;
    return hipSuccess;
  }
  const int ni = c->n_internal;
  if ((e = ensure(c->nodes, sizeof(Node) * ni)) != hipSuccess) return e;
  if ((e = ensure(c->leaf_slot, sizeof(int32_t) * nt)) != hipSuccess) return e;
  if ((e = ensure(c->leaf_tri, sizeof(int32_t) * nt)) != hipSuccess) return e;
  if ((e = ensure(c->leaf_parent, sizeof(int32_t) * nt)) != hipSuccess) return e;
  if ((e = ensure(c->refit_cnt, sizeof(uint32_t) * ni)) != hipSuccess) return e;
  // cross-node index, list, parents and the listed slots of a refit
  if ((e = ensure(c->cross, sizeof(int32_t) * 5 * (size_t)ni)) != hipSuccess) return e;
  if ((e = ensure(c->node_range, sizeof(int2) * ni)) != hipSuccess) return e;
  // sort keys (two words with the object or face level), permutation,
  // scratch, bounds, then the objects' codes and ranks
  const int no = c->no;
  const bool objects = separate_objects && no > 0;
  int rank_bits = 1;
  while ((1 << rank_bits) < no) ++rank_bits;
  const int prefix_bits = objects ? rank_bits + 1 : 0;
  // the face level (with separated objects): a face's rank among its group's faces
  const bool faces = objects && prefix_bits + c->face_bits + 30 <= 64;
  const int key_words = objects || faces ? 2 : 1;
  if ((e = ensure(c->morton, sizeof(uint32_t) * ((key_words + 2) * nt + 8 + 2 * (size_t)no))) != hipSuccess)
    return e;
  const int64_t refit_blocks = (nt + kRefitBlock - 1) / kRefitBlock;
  if ((e = ensure(c->scene_box, sizeof(float) * 8 + sizeof(double) * (refit_blocks + 2))) != hipSuccess) return e;
  // one spare node: the re-trace reads 48 bytes from a 32-byte slot
  if ((e = ensure(c->nodes4, sizeof(Node4) * (ni + 1))) != hipSuccess) return e;
  if ((e = ensure(c->tri4, sizeof(Leaf) * 4 * (size_t)ni)) != hipSuccess) return e;
  if ((e = ensure(c->bvh2_of4, sizeof(int32_t) * ni)) != hipSuccess) return e;
  if ((e = ensure(c->map4, sizeof(int32_t) * ni)) != hipSuccess) return e;
  if ((e = ensure(c->slot4, sizeof(int32_t) * 2 * (size_t)ni)) != hipSuccess) return e;
  if ((e = ensure(c->depth_key, sizeof(uint32_t) * (3 * (size_t)ni + 8))) != hipSuccess) return e;
  if ((e = ensure(c->tree_info, 64)) != hipSuccess) return e;
  uint32_t* code = ptr<uint32_t>(c->morton);   // [key_words][nt]
  uint32_t* key_hi = key_words == 2 ? code : nullptr;
  uint32_t* key_lo = code + (key_words - 1) * (size_t)nt;
  uint32_t* perm = code + key_words * (size_t)nt;
  uint32_t* perm_tmp = perm + nt;
  uint32_t* nbox = perm_tmp + nt;   // 6 ordered-bit words, then n
  uint32_t* ocode = nbox + 8;
  int32_t* orank = objects ? reinterpret_cast<int32_t*>(ocode + no) : nullptr;
  hipLaunchKernelGGL(k_box_init, dim3(1), dim3(64), 0, c->stream, nbox, (uint32_t)nt);
  const int nb = (int)std::min<int64_t>((nt + 255) / 256, 1024);
  hipLaunchKernelGGL(k_centroid_bounds, dim3(nb), dim3(256), 0, c->stream, ptr<float>(c->vertices),
                     ptr<int32_t>(c->tris), nt, nbox);
  if (objects) {
    hipLaunchKernelGGL(k_object_codes, dim3((no + 255) / 256), dim3(256), 0, c->stream, ptr<float>(c->obj_box), no,
                       nbox, ocode);
    hipLaunchKernelGGL(k_object_rank, dim3((no + 255) / 256), dim3(256), 0, c->stream, ocode, no, orank);
  }
  int32_t* frank = nullptr;
  float* fbox = nullptr;
  int fbits = 0;
  if (faces) {
    // faces in their groups' spatial order: boxes and keys, sort, ranks
    const int nf = c->nf;
    if ((e = ensure(c->face_build, sizeof(uint32_t) * (12 * (size_t)nf + (size_t)no + 16))) != hipSuccess) return e;
    fbox = ptr<float>(c->face_build);
    uint32_t* fkey = reinterpret_cast<uint32_t*>(fbox + 6 * (size_t)nf);   // [2][nf]
    uint32_t* fperm = fkey + 2 * (size_t)nf;
    uint32_t* ftmp = fperm + nf;
    frank = reinterpret_cast<int32_t*>(ftmp + nf);
    int32_t* ffirst = frank + nf;                                           // [no + 1]
    uint32_t* fn = reinterpret_cast<uint32_t*>(ffirst + no + 1);
    const int fb = (nf + 255) / 256;
    hipLaunchKernelGGL(k_face_keys, dim3(fb), dim3(256), 0, c->stream, ptr<float>(c->vertices), ptr<int32_t>(c->tris),
                       ptr<int32_t>(c->face_tri_off), ptr<int32_t>(c->face_tris), nf, ptr<int32_t>(c->face_object),
                       ptr<float>(c->obj_box), orank, rank_bits, nbox, fbox, fkey, fkey + nf, fn);
    if ((e = radix_sort_perm(c, fkey, 2, 30 + prefix_bits, fn, nf, fperm, ftmp, c->stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_face_first, dim3(fb), dim3(256), 0, c->stream, fperm, nf, ptr<int32_t>(c->face_object),
                       orank, ffirst);
    hipLaunchKernelGGL(k_face_rank, dim3(fb), dim3(256), 0, c->stream, fperm, nf, ptr<int32_t>(c->face_object),
                       orank, ffirst, frank);
    fbits = c->face_bits;
  }
  hipLaunchKernelGGL(k_morton, dim3((nt + 255) / 256), dim3(256), 0, c->stream, ptr<float>(c->vertices),
                     ptr<int32_t>(c->tris), nt, nbox, ptr<int32_t>(c->tri_face), ptr<int32_t>(c->face_object),
                     orank, rank_bits, frank, fbits, fbox, ptr<float>(c->obj_box), key_hi, key_lo);
  const int key_bits = key_words == 2 ? prefix_bits + fbits + 30 : 30;
  // what a subtree rebuild needs of these keys
  c->keys_grouped = objects;
  c->key_words_built = key_words;
  c->key_rank_bits = rank_bits;
  c->key_face_bits = fbits;
  if ((e = tree_from_keys(c, key_words, key_bits)) != hipSuccess) return e;
  // the SAH of a full build: the reference of later subtree rebuilds
  hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(64), 0, c->stream, c->sah_dev + 0, c->sah_dev + 2);
  return hipGetLastError();
}

// The binary tree of the sorted keys (code [key_words][nt] per triangle,
// key_bits significant), its refit, the 4-wide tree and the face slots.
hipError_t tree_from_keys(dcem_ctx* c, int key_words, int key_bits) {
  const int64_t nt = c->nt;
  const int ni = c->n_internal;
  hipError_t e;
  uint32_t* code = ptr<uint32_t>(c->morton);   // [key_words][nt]
  uint32_t* key_hi = key_words == 2 ? code : nullptr;
  uint32_t* key_lo = code + (key_words - 1) * (size_t)nt;
  uint32_t* perm = code + key_words * (size_t)nt;
  uint32_t* perm_tmp = perm + nt;
  uint32_t* nbox = perm_tmp + nt;
  if ((e = radix_sort_perm(c, code, key_words, key_bits, nbox + 6, nt, perm, perm_tmp, c->stream)) != hipSuccess)
    return e;
  fill_u32(ptr<uint32_t>(c->refit_cnt), 0u, (size_t)ni, c->stream);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nt == 1) {
    Node root{};
    root.c = make_int4(~0, ~0, -1, 0);
    if ((e = hipMemcpyAsync(c->nodes.p, &root, sizeof(Node), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return e;
    int32_t zero = 0, lp = 0;
    const int2 rg = make_int2(0, 0);
    if ((e = hipMemcpyAsync(c->leaf_tri.p, &zero, 4, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(c->leaf_parent.p, &lp, 4, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(c->node_range.p, &rg, sizeof rg, hipMemcpyHostToDevice, c->stream)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_karras, dim3((nt + 255) / 256), dim3(256), 0, c->stream, key_hi, key_lo, perm, (int)nt,
                       ptr<Node>(c->nodes), ptr<int32_t>(c->leaf_parent), ptr<int32_t>(c->leaf_tri),
                       ptr<int2>(c->node_range));
  }
  uint32_t* info = ptr<uint32_t>(c->tree_info);
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, c->stream, info + 2, 0u, info + 3, 0u);
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, c->stream, info + 4, 0u, info + 4, 0u);
  int32_t* cross = ptr<int32_t>(c->cross);
  hipLaunchKernelGGL(k_cross_mark, dim3((ni + 255) / 256), dim3(256), 0, c->stream, ptr<int2>(c->node_range), ni,
                     cross, cross + ni, info + 2);
  hipLaunchKernelGGL(k_cross_parent, dim3((ni + 255) / 256), dim3(256), 0, c->stream, ptr<Node>(c->nodes), cross,
                     cross + ni, info + 2, ni, cross + 2 * (size_t)ni);
  launch_refit(c, false, c->sah_dev + 0);
  // 4-wide tree: binary nodes at even depth, breadth-first
  uint32_t* dkey = ptr<uint32_t>(c->depth_key);
  uint32_t* dperm = dkey + ni;
  uint32_t* dtmp = dperm + ni;
  uint32_t* dn = dtmp + ni;   // item count for the sort
  uint32_t* n4 = ptr<uint32_t>(c->tree_info);   // [0] = 4-wide node count
  hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, c->stream, n4, 0u, dn, (uint32_t)ni);
  hipLaunchKernelGGL(k_depth_keys, dim3((ni + 255) / 256), dim3(256), 0, c->stream, ptr<Node>(c->nodes), ni, dkey, n4);
  if ((e = radix_sort_perm(c, dkey, 1, 32, dn, ni, dperm, dtmp, c->stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_map4, dim3((ni + 255) / 256), dim3(256), 0, c->stream, dperm, n4, ni,
                     ptr<int32_t>(c->bvh2_of4), ptr<int32_t>(c->map4));
  launch_collapse(c);
  // slot of every face triangle, for the refinement's face test (face_tris
  // lists every triangle once, grouped by face)
  const int64_t nft = nt;
  if ((e = ensure(c->tri_slot, sizeof(int32_t) * nt)) != hipSuccess) return e;
  if ((e = ensure(c->face_slots, sizeof(int32_t) * std::max<int64_t>(nft, 1))) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_slot, dim3((nt + 255) / 256), dim3(256), 0, c->stream, ptr<int32_t>(c->leaf_tri),
                     ptr<int32_t>(c->leaf_slot), (int)nt, ptr<int32_t>(c->tri_slot));
  if (nft > 0)
    hipLaunchKernelGGL(k_face_slots, dim3((unsigned)((nft + 255) / 256)), dim3(256), 0, c->stream,
                       ptr<int32_t>(c->face_tris), ptr<int32_t>(c->tri_slot), (int)nft, ptr<int32_t>(c->face_slots));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  c->has_bvh = true;
  return hipSuccess;
}

void launch_collapse(dcem_ctx* c) {
  if (c->nt == 0) return;
  hipLaunchKernelGGL(k_collapse, dim3((c->n_internal + 255) / 256), dim3(256), 0, c->stream, ptr<Node>(c->nodes),
                     ptr<float>(c->vertices), ptr<int32_t>(c->tris), ptr<int32_t>(c->tri_face),
                     ptr<int32_t>(c->face_object), ptr<int32_t>(c->leaf_tri), ptr<int32_t>(c->bvh2_of4),
                     ptr<int32_t>(c->map4), ptr<uint32_t>(c->tree_info), ptr<Node4>(c->nodes4),
                     ptr<Leaf>(c->tri4), ptr<int32_t>(c->leaf_slot), ptr<int32_t>(c->slot4));
}

RefitArgs make_refit_args(dcem_ctx* c, bool wide, double* sah_out) {
  const int ni = c->n_internal;
  int32_t* cross = ptr<int32_t>(c->cross);
  RefitArgs a;
  a.skip = nullptr;
  a.V = ptr<float>(c->vertices);
  a.T = ptr<int32_t>(c->tris);
  a.tri_face = ptr<int32_t>(c->tri_face);
  a.face_object = ptr<int32_t>(c->face_object);
  a.leaf_tri = ptr<int32_t>(c->leaf_tri);
  a.leaf_parent = ptr<int32_t>(c->leaf_parent);
  a.nodes = ptr<Node>(c->nodes);
  a.cnt = ptr<uint32_t>(c->refit_cnt);
  a.root_box = ptr<float>(c->scene_box);
  a.n = (int)c->nt;
  a.n_internal = ni;
  a.pad = c->pad;
  a.wide = wide;
  a.slot4 = ptr<int32_t>(c->slot4);
  a.leaf_slot = ptr<int32_t>(c->leaf_slot);
  a.nodes4 = ptr<Node4>(c->nodes4);
  a.tri4 = ptr<Leaf>(c->tri4);
  a.cross_index = cross;
  a.cross_list = cross + ni;
  a.cross_parent = cross + 2 * (size_t)ni;
  a.entries = reinterpret_cast<uint32_t*>(cross + 3 * (size_t)ni);
  a.info = ptr<uint32_t>(c->tree_info);
  a.part = sah_parts(c);
  a.sah_out = sah_out;
  a.face_ref_tri = ptr<int32_t>(c->face_ref_tri);
  a.nf = c->nf;
  a.plane = ptr<double4>(c->face_plane);
  a.cross_kernel = c->nt > kCrossKernelLeaves;
  return a;
}

int refit_blocks(const dcem_ctx* c) { return (int)((c->nt + kRefitBlock - 1) / kRefitBlock); }

void launch_refit(dcem_ctx* c, bool wide, double* sah_out) {
  if (c->nt == 0) return;
  const RefitArgs a = make_refit_args(c, wide, sah_out);
  hipLaunchKernelGGL(k_refit, dim3((unsigned)refit_blocks(c)), dim3(kRefitBlock), 0, c->stream, a);
  if (a.cross_kernel) launch_refit_cross(c, a, refit_blocks(c));
}

void launch_refit_cross(dcem_ctx* c, const RefitArgs& a, int n_rb) {
  // about a dozen listed slots per refit block: a thread per slot for up to
  // 32 per block (more are taken in turn by the same threads)
  const int blocks = std::min(std::max((n_rb * 32 + kRefitBlock - 1) / kRefitBlock, 1), 512);
  hipLaunchKernelGGL(k_refit_cross, dim3(blocks), dim3(kRefitBlock), 0, c->stream, a, n_rb);
}


}  // namespace dcem
