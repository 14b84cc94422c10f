// Moving-object transforms, LBVH construction and bottom-up refit.
//
// The paper keeps a BVH over the scene and updates it every frame, rebuilding
// only when its quality has degraded (Sec. III, "Efficient BVH updating").
// Here the tree is a linear BVH (Morton-ordered triangles, hierarchy from the
// longest common prefixes of the sorted codes, one thread per internal node),
// refit bottom-up with arrival counters, and scored by the SAH surface-area
// sum relative to the last build.
#include "dcem_internal.h"

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

__device__ inline float3 load_v(const float* v, int i) { return make_float3(v[3 * i], v[3 * i + 1], v[3 * i + 2]); }

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
  // wave reduction, then one atomic per wave
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], off));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off));
    }
  }
  if ((threadIdx.x & 63) == 0) {
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

__device__ inline double box_area(const float* lo, const float* hi) {
  double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
  return 2.0 * (dx * dy + dy * dz + dz * dx);
}

// Unit normal n and offset n . a of the plane of face f (FP64, from the
// face's reference triangle a, b, c: n = (b - a) x (c - a) normalised).
__device__ inline void face_plane(const float* __restrict__ V, const int32_t* __restrict__ T, int t,
                                  double4* __restrict__ plane, int f) {
  const int ia = T[3 * t], ib = T[3 * t + 1], ic = T[3 * t + 2];
  const double ax = V[3 * ia], ay = V[3 * ia + 1], az = V[3 * ia + 2];
  const double ux = V[3 * ib] - ax, uy = V[3 * ib + 1] - ay, uz = V[3 * ib + 2] - az;
  const double vx = V[3 * ic] - ax, vy = V[3 * ic + 1] - ay, vz = V[3 * ic + 2] - az;
  double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
  const double l = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= l;
  ny /= l;
  nz /= l;
  plane[f] = make_double4(nx, ny, nz, nx * ax + ny * ay + nz * az);
}

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
};

// A child box of binary node `p2 >> 1` (slot p2 & 1): in the binary tree and,
// refitting a collapsed tree, in the 4-wide slot d that holds it (slot4[p2]).
__device__ inline void put_child_box(const RefitArgs& a, int p2, int d, const float* lo, const float* hi) {
  store_slot(&a.nodes[p2 >> 1], p2 & 1, lo, hi);
  if (a.wide && d >= 0) store_box4(&a.nodes4[d >> 2].s[d & 3], lo, hi);
}

constexpr int kMaxCross = 1024;   // cross nodes finished in LDS by the last block

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

// Last-block pass of the refit: finish the cross nodes in LDS, from the slots
// the block pass listed up to the root.
__device__ __forceinline__ void finish_cross_nodes(const RefitArgs& a, uint32_t n_cross, float (*lbox)[12], uint32_t* lcnt,
                                   int32_t* lpar, int32_t* lnode, int2* lslot4, int2* lkid) {
  const int tid = threadIdx.x;
  const uint32_t n_ent = __hip_atomic_load(&a.info[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t k = tid; k < n_cross; k += kRefitBlock) {
    lcnt[k] = 0;
    lpar[k] = a.cross_parent[k];
    const int node = a.cross_list[k];
    lnode[k] = node;
    lkid[k] = make_int2(a.nodes[node].c.x, a.nodes[node].c.y);
    if (a.wide) lslot4[k] = make_int2(a.slot4[2 * node], a.slot4[2 * node + 1]);
  }
  __syncthreads();
  if (tid == 0) a.info[3] = 0;   // ready for the next refit
  for (uint32_t e = tid; e < n_ent; e += kRefitBlock) {
    const int p2 = (int)__hip_atomic_load(&a.entries[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int k = a.cross_index[p2 >> 1], slot = p2 & 1;
    float lo[3], hi[3];
    load_slot_coherent(&a.nodes[p2 >> 1], slot, lo, hi);
    for (uint32_t guard = n_cross + 1; guard > 0; --guard) {
      float* bx = lbox[k] + 6 * slot;
      for (int q = 0; q < 3; ++q) { bx[q] = lo[q]; bx[3 + q] = hi[q]; }
      const uint32_t old = __hip_atomic_fetch_add(&lcnt[k], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      const float* sb = lbox[k] + 6 * (slot ^ 1);
      for (int q = 0; q < 3; ++q) {
        lo[q] = fminf(lo[q], sb[q]);
        hi[q] = fmaxf(hi[q], sb[3 + q]);
      }
      const int kp = lpar[k];
      if (kp < 0) {
        for (int q = 0; q < 3; ++q) { a.root_box[q] = lo[q]; a.root_box[3 + q] = hi[q]; }
        break;
      }
      k = kp >> 1;
      slot = kp & 1;
      const int2 ds = a.wide ? lslot4[k] : make_int2(-1, -1);
      put_child_box(a, (lnode[k] << 1) | slot, slot ? ds.y : ds.x, lo, hi);
    }
  }
}

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
__global__ __launch_bounds__(kRefitBlock) void k_refit(RefitArgs a) {
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
  for (int f = blockIdx.x * kRefitBlock + threadIdx.x; f < a.nf; f += gridDim.x * kRefitBlock)
    face_plane(a.V, a.T, a.face_ref_tri[f], a.plane, f);
  const int b0 = blockIdx.x * kRefitBlock;
  const int tid = threadIdx.x;
  const uint32_t n_cross = a.info[2];
  const bool two_phase = n_cross <= (uint32_t)kMaxCross;
  {
    const int node = b0 + tid;
    lcnt[tid] = 0;
    const bool ok = node < a.n_internal;
    lpar[tid] = ok ? a.nodes[node].c.z : -1;
    lnode[tid] = ok && a.cross_index[node] < 0;   // block-local
    lkid[tid] = ok ? make_int2(a.nodes[node].c.x, a.nodes[node].c.y) : make_int2(-1, -1);
    if (a.wide && ok) lslot4[tid] = make_int2(a.slot4[2 * node], a.slot4[2 * node + 1]);
  }
  __syncthreads();
  const int i = b0 + tid;
  if (i < a.n) {
    const Leaf L = leaf_record(a.V, a.T, a.tri_face, a.face_object, a.leaf_tri[i]);
    if (a.wide) a.tri4[a.leaf_slot[i]] = L;
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
      int p2 = a.leaf_parent[i];
      for (int guard = a.n; guard > 0; --guard) {   // depth < n in a sound tree
        const int node = p2 >> 1, slot = p2 & 1;
        const bool local = node >= b0 && node < b0 + kRefitBlock && lnode[node - b0];
        int d = -1;
        if (a.wide) {
          if (local) {
            const int2 ds = lslot4[node - b0];
            d = slot ? ds.y : ds.x;
          } else {
            d = a.slot4[p2];
          }
        }
        put_child_box(a, p2, d, lo, hi);
        float slo[3], shi[3];
        if (local) {
          float* bx = lbox[node - b0] + 6 * slot;
          for (int k = 0; k < 3; ++k) { bx[k] = lo[k]; bx[3 + k] = hi[k]; }
          const uint32_t old = __hip_atomic_fetch_add(&lcnt[node - b0], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
          if (old == 0) break;
          const float* sb = lbox[node - b0] + 6 * (slot ^ 1);
          for (int k = 0; k < 3; ++k) { slo[k] = sb[k]; shi[k] = sb[3 + k]; }
        } else if (two_phase) {
          a.entries[atomicAdd(&a.info[3], 1u)] = (uint32_t)p2;
          break;
        } else {
          const uint32_t old = __hip_atomic_fetch_add(&a.cnt[node], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
          if (old == 0) break;
          a.cnt[node] = 0;
          load_slot_coherent(&a.nodes[node], slot ^ 1, slo, shi);
        }
        for (int k = 0; k < 3; ++k) {
          lo[k] = fminf(lo[k], slo[k]);
          hi[k] = fmaxf(hi[k], shi[k]);
        }
        p2 = local ? lpar[node - b0] : a.nodes[node].c.z;
        if (p2 < 0) {
          for (int k = 0; k < 3; ++k) { a.root_box[k] = lo[k]; a.root_box[3 + k] = hi[k]; }
          break;
        }
      }
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
    if (tid == 0) {
      __hip_atomic_store(&a.part[blockIdx.x], ar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&a.info[4], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    }
    __syncthreads();
  }
  if (!last) return;
  // ---- the last block to finish completes the cross nodes and the SAH sum
  if (tid == 0) a.info[4] = 0;   // ready for the next refit
  if (two_phase && n_cross > 0) finish_cross_nodes(a, n_cross, lbox, lcnt, lpar, lnode, lslot4, lkid);
  __syncthreads();
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
  for (unsigned b = tid; b < gridDim.x; b += kRefitBlock)
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
  if ((e = radix_sort_perm(c, code, key_words, key_bits, nbox + 6, nt, perm, perm_tmp, c->stream)) != hipSuccess)
    return e;
  if ((e = hipMemsetAsync(c->refit_cnt.p, 0, sizeof(uint32_t) * ni, c->stream)) != hipSuccess) return e;
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
  launch_refit(c, false, c->sah_dev + 0, c->stream);
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

void launch_refit(dcem_ctx* c, bool wide, double* sah_out, hipStream_t s) {
  if (c->nt == 0) return;
  const int ni = c->n_internal;
  int32_t* cross = ptr<int32_t>(c->cross);
  RefitArgs a;
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
  hipLaunchKernelGGL(k_refit, dim3((unsigned)((c->nt + kRefitBlock - 1) / kRefitBlock)), dim3(kRefitBlock), 0, s, a);
}


}  // namespace dcem
