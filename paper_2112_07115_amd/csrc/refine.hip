// Candidate de-duplication, image-method refinement in FP64 and per-receiver
// accumulation.
//
// Paper, Sec. III: visited propagation paths are kept in one table per
// reflection depth (step 2); each new sequence of faces yields images of the
// source through the face planes (step 3) and is validated (step 4); every
// valid path gets its total length, direction, attenuation and phase (step 6).
// Candidates here are keys (tx, rx, order, face sequence) sorted
// lexicographically, so the per-receiver sums are taken in a fixed order.
#include "dcem_internal.h"

#include <cfloat>

namespace dcem {
namespace {

constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxK = DCEM_MAX_REFLECTIONS;

struct KeyLayout {
  int W;       // 32-bit words per key
  int bits;    // significant bits
  int bt, br, bf, K;           // bf: bits per interaction field (face << tb | transmits)
  int tb;                      // 1 when interactions may transmit (the field's low bit), else 0
  int n_branch;                // branches per ray (work item (src * n_branch + b) * n_rays + position)
  const uint32_t* branch_set;  // transmitting interactions of each branch (bit j: interaction j)
  int n_rx;                    // receivers of the paths
  int n_tgt;                   // capture spheres of the trace (pairs of a record: src * n_tgt + tgt)
  bool backward;               // records traced from the receivers: (src, tgt) = (rx, tx), faces reversed
  const uint32_t* ray_order;   // traversal position -> ray within its source's block
  int64_t n_rays;
};

// Captures, the face log and the ray caches are indexed by traversal position
// (tx * n_rays + rank of the ray's direction along the sort curve); the ray
// id tx * n_rays + ray of position p:
__device__ inline uint32_t ray_of(uint32_t p, const KeyLayout& L) {
  if (p == kNoRay) return kNoRay;
  const uint32_t tx = (uint32_t)(p / (uint64_t)L.n_rays);
  return tx * (uint32_t)L.n_rays + L.ray_order[p - (uint64_t)tx * L.n_rays];
}

// Place `nbits` of `v` at bit offset `pos` (from the least significant end of
// the W-word key, word W-1 holding bits 0..31).
__device__ inline void put_bits(uint32_t* w, int W, int pos, int nbits, uint32_t v) {
  while (nbits > 0) {
    const int word = W - 1 - pos / 32, off = pos % 32;
    const int take = min(nbits, 32 - off);
    const uint32_t mask = take == 32 ? 0xffffffffu : ((1u << take) - 1u);
    w[word] |= (v & mask) << off;
    v = take == 32 ? 0 : (v >> take);
    nbits -= take;
    pos += take;
  }
}

// Sort key of a capture: (tx, rx, order, f1..fK) packed most significant
// first, faces read from the per-bounce face log of the capturing ray.  A
// record traced from a receiver names (rx, tx) and meets the faces in reverse
// path order; its key is the path's, from the transmitter.  Returns the
// path's pair tx * n_rx + rx.
__device__ inline uint32_t capture_key(const Capture& c, const int32_t* __restrict__ face_log, int64_t n_work,
                                       const KeyLayout& L, uint32_t* w) {
  const uint32_t tpair = c.pair_order >> 4, order = c.pair_order & 15u;
  const uint32_t src = tpair / (uint32_t)L.n_tgt, tgt = tpair - src * (uint32_t)L.n_tgt;
  const uint32_t tx = L.backward ? tgt : src, rx = L.backward ? src : tgt;
  const uint32_t tset =
      (order > 0 && L.n_branch > 1) ? L.branch_set[(c.work / (uint64_t)L.n_rays) % (uint32_t)L.n_branch] : 0u;
  // the ray's faces in bounce order, loaded together (one round trip)
  int32_t fl[kMaxK];
#pragma unroll
  for (int b = 0; b < kMaxK; ++b) {
    fl[b] = 0;
    if (b >= L.K) break;   // uniform
    if ((uint32_t)b < order) fl[b] = face_log[(size_t)b * n_work + c.work];
  }
  for (int k = 0; k < 8; ++k) w[k] = 0;
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) {
    if (j >= L.K) break;   // uniform
    uint32_t f = 0;
    if ((uint32_t)j < order) {
      int bounce = j;
      int32_t fb = fl[j];
      if (L.backward) {   // uniform: faces in reverse order, picked without indexing the array
        bounce = (int)order - 1 - j;
#pragma unroll
        for (int b = 0; b < kMaxK; ++b)
          if (b == bounce) fb = fl[b];
      }
      f = ((uint32_t)fb << L.tb) | ((tset >> bounce) & (uint32_t)L.tb);
    }
    put_bits(w, L.W, (L.K - 1 - j) * L.bf, L.bf, f);
  }
  int pos = L.K * L.bf;
  put_bits(w, L.W, pos, 4, order);
  pos += 4;
  put_bits(w, L.W, pos, L.br, rx);
  pos += L.br;
  put_bits(w, L.W, pos, L.bt, tx);
  return tx * (uint32_t)L.n_rx + rx;
}

// Item counts of the sort-based path are read on the device: min(*n_dev, n_max).
__global__ void k_keys(const Capture* __restrict__ caps, const uint32_t* __restrict__ n_dev, uint32_t n_max,
                       const int32_t* __restrict__ face_log, int64_t n_work, KeyLayout L, uint32_t* __restrict__ keys,
                       int64_t stride) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= min(*n_dev, n_max)) return;
  uint32_t w[8];
  capture_key(caps[i], face_log, n_work, L, w);
  for (int k = 0; k < L.W; ++k) keys[k * stride + i] = w[k];
}

// De-duplication of a small capture list (n <= kSmallN, read on the device)
// in one workgroup, without a sort of the captures:
//  1. every capture's key goes into LDS and, by linear probing, into a hash
//     table of capture indices, so equal keys meet in one slot; the slot
//     keeps the capture with the lowest (ray, index) of its key;
//  2. the occupied slots (the unique keys) are bucketed by their (tx, rx)
//     pair, the key's most significant field (pairs >> shift, a monotone map);
//  3. a key's position in sorted order is its bucket's start plus the number
//     of smaller keys in its bucket.
// Output, per unique key u in ascending key order: perm[u] = the chosen
// capture (its key words stay in `keys_out`, its ray is the lowest ray that
// found the candidate); uniq_pos is the identity, so each unique key's
// capture range [uniq_pos[u], uniq_pos[u + 1]) holds that one capture; and
// the decoded candidate (see UniqueOut).  The set of keys, their order and
// the lowest ray per key equal those of a stable sort of all captures
// followed by run heads.
constexpr int kSmallN = 2048;
constexpr int kSmallW = 3;
constexpr int kCandBlock = 1024;
constexpr int kCandPer = kSmallN / kCandBlock;   // captures per thread
constexpr int kHashSlots = 2 * kSmallN;          // load factor <= 1/2
constexpr int kSlotsPer = kHashSlots / kCandBlock;
constexpr int kBuckets = 2048;
constexpr int kBucketsPer = kBuckets / kCandBlock;
constexpr uint32_t kEmptySlot = 0xffffffffu;

__device__ inline uint32_t key_hash(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u ^ (c + 0x165667B1u) * 0xC2B2AE3Du;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return h & (kHashSlots - 1);
}

// A unique candidate, decoded from its key: (tx, rx) pair, reflection order,
// face sequence (-1 past the order) and the lowest ray that captured it (-1:
// only the line-of-sight record).  Written per unique key in key order; the
// refinement reads it.
struct UniqueOut {
  int32_t* pair;
  uint8_t* order;
  int32_t* faces;   // [n][K]
  int32_t* first_ray;
};

__device__ inline uint32_t key_bits(const uint32_t* w, int W, int pos, int nbits) {
  uint32_t v = 0;
  int got = 0;
  while (got < nbits) {
    const int word = W - 1 - pos / 32, off = pos % 32;
    const int take = min(nbits - got, 32 - off);
    const uint32_t mask = take == 32 ? 0xffffffffu : ((1u << take) - 1u);
    v |= ((w[word] >> off) & mask) << got;
    got += take;
    pos += take;
  }
  return v;
}

// Decoded face entry of an interaction field: the face, with kTransmit when
// the interaction transmits.
__device__ inline int32_t field_face(uint32_t field, int tb) {
  return (int32_t)(field >> tb) | ((field & (uint32_t)tb) ? kTransmit : 0);
}

__device__ inline void write_unique(const UniqueOut& o, const KeyLayout& L, uint32_t u, const uint32_t* w,
                                    uint32_t first_work) {
  int pos = L.K * L.bf;
  const uint32_t order = key_bits(w, L.W, pos, 4);
  pos += 4;
  const uint32_t rx = key_bits(w, L.W, pos, L.br);
  pos += L.br;
  const uint32_t tx = key_bits(w, L.W, pos, L.bt);
  o.pair[u] = (int32_t)(tx * (uint32_t)L.n_rx + rx);
  o.order[u] = (uint8_t)order;
  for (int j = 0; j < L.K; ++j)
    o.faces[(size_t)u * L.K + j] = (uint32_t)j < order ? field_face(key_bits(w, L.W, (L.K - 1 - j) * L.bf, L.bf), L.tb) : -1;
  o.first_ray[u] = first_work == kNoRay ? -1 : (int32_t)first_work;
}

__device__ inline bool key_less(const uint4& a, const uint4& b) {
  return a.x < b.x || (a.x == b.x && (a.y < b.y || (a.y == b.y && a.z < b.z)));
}

__global__ __launch_bounds__(kCandBlock) void k_small_candidates(
    const Capture* __restrict__ caps, const uint32_t* __restrict__ n_dev, uint32_t capacity,
    const int32_t* __restrict__ face_log, int64_t n_work, KeyLayout L, int pair_shift,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ perm_out, uint32_t* __restrict__ uniq_pos,
    UniqueOut out, uint32_t* __restrict__ n_unique, uint32_t* __restrict__ fallback) {
  __shared__ uint32_t kk[kSmallW][kSmallN];              // key words per capture
  __shared__ uint32_t cpair[kSmallN];                    // (tx, rx) pair per capture
  __shared__ uint32_t cwork[kSmallN];                    // lowest ray of the key, at its chosen capture
  __shared__ uint32_t slot_idx[kHashSlots];              // a capture of the slot's key
  __shared__ unsigned long long slot_best[kHashSlots];   // min (ray << 32 | capture) of the key
  __shared__ uint32_t bstart[kBuckets];                  // counts, then exclusive starts
  __shared__ uint32_t wsum[kCandBlock / kWave + 1];
  uint4* bkey = reinterpret_cast<uint4*>(slot_best);     // after step 2: unique keys by bucket
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  // the records are loaded while their count is (every record below the
  // buffer's capacity is readable; those past the count go unused)
  Capture cr[kCandPer];
#pragma unroll
  for (int q = 0; q < kCandPer; ++q) {
    const uint32_t i = tid + q * kCandBlock;
    cr[q] = i < capacity ? caps[i] : Capture{kNoRay, 0u};
  }
  // the counter keeps counting past the buffer when captures overflow (the
  // trace kernel flags that); only the stored records are read
  const uint32_t n = min(*n_dev, capacity);
  if (n > (uint32_t)kSmallN) {   // uniform: the host redoes this frame's candidates the exact way
    if (tid == 0) {
      *fallback = 1;
      *n_unique = 0;
    }
    return;
  }
  for (int q = 0; q < kSlotsPer; ++q) {
    slot_idx[tid + q * kCandBlock] = kEmptySlot;
    slot_best[tid + q * kCandBlock] = ~0ull;
  }
  for (int q = 0; q < kBucketsPer; ++q) bstart[tid + q * kCandBlock] = 0;
  uint32_t work[kCandPer];
#pragma unroll
  for (int q = 0; q < kCandPer; ++q) {
    const uint32_t i = tid + q * kCandBlock;
    work[q] = 0;
    if (i < n) {
      const Capture c = cr[q];
      uint32_t w[8];
      const uint32_t pair = capture_key(c, face_log, n_work, L, w);
      for (int k = 0; k < L.W; ++k) keys_out[k * (int64_t)kSmallN + i] = w[k];
      for (int k = 0; k < kSmallW; ++k) kk[k][i] = k < L.W ? w[k] : 0u;
      cpair[i] = pair;
      work[q] = ray_of(c.work, L);
    }
  }
  __syncthreads();
  // ---- 1. hash insertion: a slot, once claimed, names a capture whose key
  // is already in LDS; at most n < kHashSlots slots are ever claimed
#pragma unroll
  for (int q = 0; q < kCandPer; ++q) {
    const uint32_t i = tid + q * kCandBlock;
    if (i >= n) continue;
    const uint32_t k0 = kk[0][i], k1 = kk[1][i], k2 = kk[2][i];
    uint32_t h = key_hash(k0, k1, k2);
    while (true) {
      const uint32_t prev = atomicCAS(&slot_idx[h], kEmptySlot, i);
      if (prev == kEmptySlot || (kk[0][prev] == k0 && kk[1][prev] == k1 && kk[2][prev] == k2)) break;
      h = (h + 1) & (kHashSlots - 1);
    }
    atomicMin(&slot_best[h], ((unsigned long long)work[q] << 32) | i);
  }
  __syncthreads();
  // ---- 2. bucket the unique keys by pair
  uint32_t rep[kSlotsPer], bpos[kSlotsPer], bkt[kSlotsPer];
#pragma unroll
  for (int q = 0; q < kSlotsPer; ++q) {
    const int j = tid + q * kCandBlock;
    rep[q] = kEmptySlot;
    if (slot_idx[j] != kEmptySlot) {
      const unsigned long long best = slot_best[j];
      rep[q] = (uint32_t)best;
      cwork[rep[q]] = (uint32_t)(best >> 32);
      bkt[q] = cpair[rep[q]] >> pair_shift;
      bpos[q] = atomicAdd(&bstart[bkt[q]], 1u);
    }
  }
  __syncthreads();
  // exclusive scan of the bucket counts (kBucketsPer consecutive per thread)
  uint32_t cnt[kBucketsPer], local = 0;
#pragma unroll
  for (int q = 0; q < kBucketsPer; ++q) {
    cnt[q] = bstart[tid * kBucketsPer + q];
    local += cnt[q];
  }
  uint32_t incl = local;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int v = 0; v < kCandBlock / kWave; ++v) {
      const uint32_t x = wsum[v];
      wsum[v] = run;
      run += x;
    }
    wsum[kCandBlock / kWave] = run;
  }
  __syncthreads();
  uint32_t run = wsum[wave] + incl - local;
#pragma unroll
  for (int q = 0; q < kBucketsPer; ++q) {
    bstart[tid * kBucketsPer + q] = run;
    run += cnt[q];
  }
  const uint32_t nu = wsum[kCandBlock / kWave];
  __syncthreads();   // slot_best is read no more: bkey may overwrite it
#pragma unroll
  for (int q = 0; q < kSlotsPer; ++q)
    if (rep[q] != kEmptySlot) bkey[bstart[bkt[q]] + bpos[q]] = make_uint4(kk[0][rep[q]], kk[1][rep[q]], kk[2][rep[q]], rep[q]);
  __syncthreads();
  // ---- 3. rank within the bucket (keys are distinct)
  for (uint32_t p = tid; p < nu; p += kCandBlock) {
    const uint4 me = bkey[p];
    const uint32_t b = cpair[me.w] >> pair_shift;
    const uint32_t b0 = bstart[b], b1 = b + 1 < (uint32_t)kBuckets ? bstart[b + 1] : nu;
    uint32_t r = b0;
    for (uint32_t v = b0; v < b1; ++v) r += key_less(bkey[v], me) ? 1u : 0u;
    perm_out[r] = me.w;
    uniq_pos[r] = r;
    const uint32_t w[kSmallW] = {me.x, me.y, me.z};
    write_unique(out, L, r, w, cwork[me.w]);
  }
  if (tid == 0) {
    *n_unique = nu;
    uniq_pos[nu] = nu;
  }
}

UniqueOut unique_out(dcem_ctx* c) {
  return UniqueOut{ptr<int32_t>(c->pair_range), ptr<uint8_t>(c->path_order), ptr<int32_t>(c->path_faces),
                   ptr<int32_t>(c->first_ray)};
}

// De-duplication of a small list in one launch.
void launch_small_dedupe(dcem_ctx* c, const KeyLayout& L, int64_t n_work) {
  uint32_t* cnt = c->cnt_dev;
  const uint32_t n_pairs = (uint32_t)c->n_tx * (uint32_t)c->n_rx;
  int shift = 0;
  while (n_pairs > 0 && ((n_pairs - 1) >> shift) >= (uint32_t)kBuckets) ++shift;
  hipLaunchKernelGGL(k_small_candidates, dim3(1), dim3(kCandBlock), 0, c->stream,
                     ptr<Capture>(c->caps[c->cur_caps]), cnt + kCntCaptures, (uint32_t)c->cap_capacity,
                     ptr<int32_t>(c->face_log), n_work, L, shift, ptr<uint32_t>(c->cand_keys),
                     ptr<uint32_t>(c->cand_perm), ptr<uint32_t>(c->uniq_idx), unique_out(c), cnt + kCntUnique,
                     cnt + kCntFallback);
}

__global__ __launch_bounds__(256) void k_heads(const uint32_t* __restrict__ keys, int64_t stride, int W,
                                               const uint32_t* __restrict__ perm, const uint32_t* __restrict__ n_dev,
                                               uint32_t n_max, uint8_t* __restrict__ head,
                                               uint32_t* __restrict__ block_cnt, uint32_t* __restrict__ run_min) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = min(*n_dev, n_max);
  bool h = false;
  if (run_min && i < n) run_min[i] = kNoRay;   // nullable: per-run lowest ray ids, filled by k_compact
  if (i < n) {
    h = i == 0;
    if (!h) {
      const uint32_t a = perm[i], b = perm[i - 1];
      for (int k = 0; k < W && !h; ++k) h = keys[k * stride + a] != keys[k * stride + b];
    }
    head[i] = h ? 1 : 0;
  }
  const uint64_t m = __ballot(h);
  __shared__ uint32_t wc[4];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(1024) void k_scan_small(uint32_t* __restrict__ v, int n, uint32_t* __restrict__ total) {
  __shared__ uint32_t part[1024];
  const int per = (n + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t x = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int i = b; i < e; ++i) {
    uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  if (threadIdx.x == 1023) *total = part[1023];
}

// Positions of the run heads (uniq_pos), and with run_min (nullable) the
// lowest ray id of every run: each capture of the sorted list enters its
// ray into its run's minimum (atomic, so a long run costs no serial walk).
__global__ __launch_bounds__(256) void k_compact(const uint8_t* __restrict__ head,
                                                 const uint32_t* __restrict__ block_off,
                                                 const uint32_t* __restrict__ n_dev, uint32_t n_max,
                                                 const uint32_t* __restrict__ n_unique,
                                                 uint32_t* __restrict__ uniq_pos, uint32_t* __restrict__ run_min,
                                                 const uint32_t* __restrict__ perm, const Capture* __restrict__ caps,
                                                 KeyLayout L) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = min(*n_dev, n_max);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool h = i < n && head[i];
  uint32_t ray = kNoRay;
  if (run_min && i < n) ray = ray_of(caps[perm[i]].work, L);   // loaded while the heads are counted
  const uint64_t m = __ballot(h);
  __shared__ uint32_t wc[4];
  if (lane == 0) wc[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t off = block_off[blockIdx.x];
  for (int w = 0; w < wave; ++w) off += wc[w];
  if (h) uniq_pos[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
  // run index of position i: the heads at or before it, less one
  if (run_min && i < n) atomicMin(&run_min[off + __popcll(m & ((2ull << lane) - 1ull)) - 1], ray);
  if (i == 0) uniq_pos[*n_unique] = n;
}

// Decoded candidate of every unique key of the sorted list: its key from the
// first capture of its run, its lowest ray over the run (from k_compact).
__global__ __launch_bounds__(256) void k_unique_info(const uint32_t* __restrict__ keys, int64_t stride, KeyLayout L,
                                                     const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ uniq_pos,
                                                     const uint32_t* __restrict__ n_unique,
                                                     const uint32_t* __restrict__ run_min, UniqueOut out) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= *n_unique) return;
  const uint32_t h = uniq_pos[u];
  const uint32_t fr = run_min[u];
  uint32_t w[8];
  const uint32_t idx = perm[h];
  for (int k = 0; k < L.W; ++k) w[k] = keys[k * stride + idx];
  write_unique(out, L, u, w, fr);
}


struct D3 {
  double x, y, z;
};
__device__ inline D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double len(D3 a) { return sqrt(dot(a, a)); }
__device__ inline D3 normed(D3 a) { return (1.0 / len(a)) * a; }
__device__ inline D3 fvec(const float* v, int i) { return {(double)v[3 * i], (double)v[3 * i + 1], (double)v[3 * i + 2]}; }

struct Cx {
  double re, im;
};
__device__ inline Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cx cscl(double s, Cx a) { return {s * a.re, s * a.im}; }
__device__ inline Cx cdiv(Cx a, Cx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
// principal square root for Re z >= 0 (the case eps_c - sin^2 with eps_r >= 1)
__device__ inline Cx csqrt_p(Cx z) {
  const double r = hypot(z.re, z.im);
  double re = sqrt(0.5 * (r + z.re));
  if (re == 0.0) return {0.0, sqrt(0.5 * (r - z.re)) * (z.im < 0 ? -1.0 : 1.0)};
  return {re, z.im / (2.0 * re)};
}

// Reflection coefficients of a plane interface with relative permittivity
// eps_c = eps_r - j sigma / (2 pi f eps0) (time factor e^{+j w t}); TE with
// E normal to the plane of incidence, TM with E in it.  const_gamma g (not
// NaN) is a polarisation-independent mirror: TE = -g, TM = +g.
__device__ inline void fresnel_coeffs(const double* mat, double freq, double cos_t, Cx& te, Cx& tm) {
  const double g = mat[2];
  if (!isnan(g)) {
    te = {-g, 0.0};
    tm = {g, 0.0};
    return;
  }
  const Cx ec = {mat[0], -mat[1] / (2.0 * kPi * freq * kEps0)};
  const Cx root = csqrt_p({ec.re - (1.0 - cos_t * cos_t), ec.im});
  const Cx ct = {cos_t, 0.0};
  te = cdiv(csub(ct, root), cadd(ct, root));
  const Cx ecc = cscl(cos_t, ec);
  tm = cdiv(csub(ecc, root), cadd(ecc, root));
}

__device__ inline double vol(D3 a, D3 b, D3 c, D3 d) { return dot(b - a, cross(c - a, d - a)); }

// Derivatives of the Fresnel coefficients with respect to the complex
// permittivity eps_c (both are analytic in it): with r = sqrt(eps_c - sin^2)
// and c = cos(theta), dr/deps_c = 1 / (2 r), so
//   dGamma_TE/deps_c = -c / (r (c + r)^2),
//   dGamma_TM/deps_c = 2 c (r - eps_c / (2 r)) / (eps_c c + r)^2;
// zero for a constant-gamma material.
__device__ inline void fresnel_deps(const double* mat, double freq, double cos_t, Cx& dte, Cx& dtm) {
  if (!isnan(mat[2])) {
    dte = dtm = Cx{0.0, 0.0};
    return;
  }
  const Cx ec = {mat[0], -mat[1] / (2.0 * kPi * freq * kEps0)};
  const Cx r = csqrt_p({ec.re - (1.0 - cos_t * cos_t), ec.im});
  const Cx ctr = cadd(Cx{cos_t, 0.0}, r);
  dte = cdiv(Cx{-cos_t, 0.0}, cmul(r, cmul(ctr, ctr)));
  const Cx den = cadd(cscl(cos_t, ec), r);
  const Cx num = cscl(2.0 * cos_t, csub(r, cdiv(ec, cscl(2.0, r))));
  dtm = cdiv(num, cmul(den, den));
}

// Azimuth cell of a departure direction u: the pattern taps j and j + 1
// (mod 16) around its azimuth and the fraction t in [0, 1) of the way to j + 1,
// so B_j = 1 - t, B_{j+1} = t and every other hat is zero there.
__device__ inline void pattern_cell(D3 u, int& j, double& t) {
  double x = atan2(u.y, u.x) * (kPatternTaps / (2.0 * kPi));   // [-8, 8]
  if (x < 0.0) x += kPatternTaps;
  const double fl = floor(x);
  t = x - fl;
  j = (int)fl & (kPatternTaps - 1);   // x = 16 after the wrap is tap 0
}

// Gain of the pattern at u, as w_j + t (w_{j+1} - w_j): exactly 1 when all
// weights are 1.
__device__ inline double pattern_gain(const TxPattern& p, D3 u) {
  if (!p.on) return 1.0;
  int j;
  double t;
  pattern_cell(u, j, t);
  const double w0 = p.w[j], w1 = p.w[(j + 1) & (kPatternTaps - 1)];
  return w0 + t * (w1 - w0);
}

struct RefineArgs {
  int K;                     // maximum reflection order (row length of faces)
  int n_rx;
  const uint32_t* n_unique;
  const float* tx;
  const float* rx;
  const double4* plane;
  const int32_t* face_tri_off;
  const int32_t* face_tris;
  const int32_t* face_slots;   // slot triangle of each face_tris entry
  const int32_t* face_material;
  const double* materials;
  const double* mat_pen;    // per material: field factor of a transmission, 10^(-loss dB / 20)
  const Node4* nodes4;
  const Leaf* tri4;         // leaf triangles in slot order
  const uint32_t* n4_dev;   // null: empty scene; [1] root leaf-slot mask
  const double* freqs;
  int n_freqs;
  double sqrt_pt;
  double atten_db_per_km;
  TxPattern pat;
  int64_t n_rays;
  uint8_t* valid;
  double* length;
  double* tau;
  double* aod;
  double* aoa;
  double* amp;       // [n][n_freqs][3][2]
  const int32_t* pair;      // decoded candidates (written by the de-duplication)
  const uint8_t* order;     // [n] reflection order
  const int32_t* faces;     // [n][K] face sequence
  double* pts;       // [n][K+2][3] transmitter, reflection points, receiver
  uint32_t* counters;
  uint32_t* err;
};

// Is point p inside one of the triangles k0, k0 + step, ... of face f
// (inclusive)?  2D edge functions on the plane projection that drops the
// normal's dominant axis.  (k0 = 0, step = 1: inside the face.)
__device__ bool in_face(const RefineArgs& a, int f, D3 p, D3 n, int k0 = 0, int step = 1) {
  const double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
  const int drop = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  auto pr = [drop](D3 v, double& u, double& w) {
    if (drop == 0) { u = v.y; w = v.z; }
    else if (drop == 1) { u = v.z; w = v.x; }
    else { u = v.x; w = v.y; }
  };
  double pu, pw;
  pr(p, pu, pw);
  for (int k = a.face_tri_off[f] + k0; k < a.face_tri_off[f + 1]; k += step) {
    const Leaf L = a.tri4[a.face_slots[k]];
    const D3 A = {L.v0.x, L.v0.y, L.v0.z}, B = {L.v1.x, L.v1.y, L.v1.z}, C = {L.v2.x, L.v2.y, L.v2.z};
    double au, aw, bu, bw, cu, cw;
    pr(A, au, aw);
    pr(B, bu, bw);
    pr(C, cu, cw);
    const double e0 = (bu - au) * (pw - aw) - (bw - aw) * (pu - au);
    const double e1 = (cu - bu) * (pw - bw) - (cw - bw) * (pu - bu);
    const double e2 = (au - cu) * (pw - cw) - (aw - cw) * (pu - cu);
    if ((e0 >= 0 && e1 >= 0 && e2 >= 0) || (e0 <= 0 && e1 <= 0 && e2 <= 0)) return true;
  }
  return false;
}

// Any triangle (outside faces fa, fb) crossed by the open segment p -> q,
// keeping t_min away from both ends?  FP64 orientation tests at the leaves;
// 4-wide tree boxes (FP32, padded) tested in FP64.  Traversed by a group of
// kCheckLanes lanes, one tree level per step: each lane takes one slot of up
// to kCheckLanes / 4 popped nodes (a stack entry carries its node's leaf-slot
// mask, so leaf triangles come straight from the slot array).  The answer does
// not depend on the order: the first occluder found ends the query, and an
// unoccluded segment visits every box it meets, so a wide group takes few
// steps.
constexpr int kCheckLanes = kWave;              // lanes per occlusion query
constexpr int kCheckStack = 256;                // stack entries per query

__device__ bool group_occluded(const RefineArgs& a, D3 p, D3 q, int fa, int fb, uint32_t* se, int lane,
                               uint64_t gmask, bool& fault) {
  const int n4 = a.n4_dev ? (int)a.n4_dev[0] : 0;
  if (n4 == 0) return false;
  const D3 dv = q - p;
  const double L = len(dv);
  const double tlo = kTMinD / L, thi = 1.0 - kTMinD / L;
  if (!(tlo < thi)) return false;
  const double big = 1e300;
  const double ix = dv.x != 0 ? 1.0 / dv.x : big, iy = dv.y != 0 ? 1.0 / dv.y : big,
               iz = dv.z != 0 ? 1.0 / dv.z : big;
  const int gl = lane & (kCheckLanes - 1), jl = gl >> 2, el = gl & 3;
  const uint64_t below = (1ull << lane) - 1ull;
  if (gl == 0) se[0] = a.n4_dev[1] << kNodeBits;
  int sp = 1;
  wave_sync();
  for (int guard = n4 + 2; sp > 0; --guard) {
    if (guard == 0) {
      fault = true;
      return false;
    }
    const int n_pop = min(kCheckLanes / 4, sp);
    const bool act = jl < n_pop;
    const uint32_t ent = act ? se[sp - 1 - jl] : 0u;
    wave_sync();
    sp -= n_pop;
    const int node = (int)(ent & ((1u << kNodeBits) - 1));
    const bool leaf = act && ((ent >> (kNodeBits + el)) & 1u);
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
    if (act) {
      const float4* src = leaf ? reinterpret_cast<const float4*>(a.tri4 + 4 * (size_t)node + el)
                               : reinterpret_cast<const float4*>(&a.nodes4[node].s[el]);
      q0 = src[0];
      q1 = src[1];
      q2 = src[2];
    }
    bool hit = false;
    uint32_t push = kNoEntry;
    if (leaf) {
      const int face = __float_as_int(q1.w);
      if (face != fa && face != fb) {
        const D3 A = {q0.x, q0.y, q0.z}, B = {q1.x, q1.y, q1.z}, C = {q2.x, q2.y, q2.z};
        const double op = vol(A, B, C, p), oq = vol(A, B, C, q);
        if (op != oq) {
          const double t = op / (op - oq);
          if (t > tlo && t < thi) {
            const double s0 = vol(p, q, A, B), s1 = vol(p, q, B, C), s2 = vol(p, q, C, A);
            hit = (s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0);
          }
        }
      }
    } else if (act && __float_as_int(q0.w) != kEmpty) {
      const double ax = (q0.x - p.x) * ix, bx = (q1.x - p.x) * ix;
      const double ay = (q0.y - p.y) * iy, by = (q1.y - p.y) * iy;
      const double az = (q0.z - p.z) * iz, bz = (q1.z - p.z) * iz;
      const double tn = fmax(fmax(fmin(ax, bx), fmin(ay, by)), fmax(fmin(az, bz), 0.0));
      const double tf = fmin(fmin(fmax(ax, bx), fmax(ay, by)), fmin(fmax(az, bz), 1.0));
      if (tn <= tf * (1.0 + 1e-12)) push = (uint32_t)__float_as_int(q0.w) | (__float_as_uint(q1.w) << kNodeBits);
    }
    if (__ballot(hit) & gmask) return true;
    const uint64_t want = __ballot(push != kNoEntry) & gmask;
    const int pos = sp + __popcll(want & below);
    if (push != kNoEntry && pos < kCheckStack) se[pos] = push;
    if (sp + __popcll(want) > kCheckStack) fault = true;
    sp = min(sp + __popcll(want), kCheckStack);
    wave_sync();
  }
  return false;
}

// The image of point im in plane pl (unit normal xyz, offset w), with
// contraction off: the refinement and the visited-series expansion both
// compute images with this function.
__device__ inline D3 reflect_image(D3 im, double4 pl) {
#pragma clang fp contract(off)
  const double h = 2.0 * ((im.x * pl.x + im.y * pl.y + im.z * pl.z) - pl.w);
  return D3{im.x - h * pl.x, im.y - h * pl.y, im.z - h * pl.z};
}

// Image-method geometry of a candidate (Sec. III step 3): image(j) gives the
// image of T through the planes of interactions 1..j in turn (reflect_image
// for each reflection; a transmission leaves the image where it is: the ray
// goes straight on), plane(j) interaction j + 1's plane; the interaction
// points are walked back from R towards the images, each on its plane, and
// visit(j, P) receives point j (j = order..1) and may stop the walk by
// returning false; d receives the distance from R to the last image (the path
// length).  False when a walk is parallel to its plane, a point falls outside
// its open segment, or visit stops.  Contraction is off, so the refinement
// and the visited-series expansion, which share this code, take the same
// decisions.
template <class Image, class Plane, class Visit>
__device__ inline bool image_walk(D3 R, int order, Image image, Plane plane, Visit visit, double& d) {
#pragma clang fp contract(off)
  const D3 last = image(order);
  const D3 rl = {R.x - last.x, R.y - last.y, R.z - last.z};
  d = sqrt(rl.x * rl.x + rl.y * rl.y + rl.z * rl.z);
  D3 Q = R;
  for (int j = order; j >= 1; --j) {
    const double4 pl = plane(j - 1);
    const D3 n = {pl.x, pl.y, pl.z};
    const D3 im = j == order ? last : image(j);
    const D3 D = {im.x - Q.x, im.y - Q.y, im.z - Q.z};
    const double den = D.x * n.x + D.y * n.y + D.z * n.z;
    if (den == 0.0) return false;
    const double s = (pl.w - (Q.x * n.x + Q.y * n.y + Q.z * n.z)) / den;
    if (!(s > 0.0 && s < 1.0)) return false;
    Q = D3{Q.x + s * D.x, Q.y + s * D.y, Q.z + s * D.z};
    if (!visit(j, Q)) return false;
  }
  return true;
}

// Does the candidate transmit through a face whose material is opaque (a
// zero transmission factor)?  No path does.
__device__ inline bool through_opaque(const RefineArgs& a, const int* faces, int order, uint32_t tmask) {
  for (int j = 0; j < order; ++j)
    if (((tmask >> j) & 1u) && a.mat_pen[a.face_material[faces[j]]] == 0.0) return true;
  return false;
}

// Refinement of one unique candidate u by one block of four wavefronts (one
// per SIMD, so four blocks share a compute unit; blocks of more wavefronts
// place two on the same SIMD and only two of them fit).
//  1. Geometry (wavefront 0: lane j loads face j's plane, lane 0 walks):
//     decode the key, image sources through the face planes and reflection
//     points walked back from the receiver, each strictly inside its segment
//     (Sec. III step 3).
//  2. One validation task per sub-segment j = 0..order: the sub-segment must
//     be unoccluded (every triangle outside its end faces), and for j >= 1
//     reflection point j must lie in its face, the face's triangles spread
//     over the lanes (Sec. III step 4).
//  3. The field task (lane f for frequency f): length, delay, directions and
//     the field: theta-hat of the departure direction carried through each
//     reflection by the Fresnel coefficients, times sqrt(Pt) lambda /
//     (4 pi d), the specific attenuation and the phase e^{-j k0 d} (Eq. (3)
//     with n = 2, Sec. III step 6).
// The tasks are drawn in a fixed order from an LDS counter (wavefront w
// starts with position w): the sub-segments longest first, the field at
// position 1, so wavefront 1 computes it and then writes the outputs once
// every task is done (a path found invalid is zeroed then).
constexpr int kRefineWaves = 4;

__global__ __launch_bounds__(kRefineWaves * kWave) __attribute__((amdgpu_waves_per_eu(4)))
void k_refine(RefineArgs a) {
  __shared__ double sP[(kMaxK + 2) * 3];      // transmitter, reflection points, receiver
  __shared__ D3 simg[kMaxK + 1];             // images of the transmitter
  __shared__ int sfaces[kMaxK];              // face ids (transmission flag cleared)
  __shared__ uint32_t stmask;                 // bit j - 1: interaction j transmits
  __shared__ int sorder, sok, sfail;
  __shared__ double sd;
  __shared__ double4 spl[kMaxK];              // planes of the faces
  __shared__ uint32_t stk[kRefineWaves][kCheckStack];   // each wavefront's occlusion stack
  __shared__ int snext;                                   // next free task
  __shared__ int stask[kMaxK + 2];                        // the tasks in the order they are drawn
  const uint32_t u = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int K = a.K;
  // the decoded candidate (pair, order, faces: written by the
  // de-duplication) is loaded while the count is; the arrays hold an entry
  // for every block, and entries past the count are never used
  int order0 = 0, pair = 0, face = -1;
  if (w == 0) {
    order0 = a.order[u];
    pair = a.pair[u];
    if (lane < K) face = a.faces[(size_t)u * K + lane];
  }
  if (u >= *a.n_unique) return;   // uniform over the block
  // ---- 1. geometry: lane j takes face j and loads its plane, lane 0 then
  // runs the image method on LDS copies
  if (w == 0) {
    const uint64_t tm = __ballot(lane < order0 && (face & kTransmit));
    if (lane < order0) {
      sfaces[lane] = face & kFaceMask;
      spl[lane] = a.plane[face & kFaceMask];
    }
    wave_sync();
    if (lane == 0) {
      const int tx = pair / a.n_rx, rx = pair - tx * a.n_rx;
      const D3 T = fvec(a.tx, tx), R = fvec(a.rx, rx);
      stmask = (uint32_t)tm;
      sP[0] = T.x; sP[1] = T.y; sP[2] = T.z;
      sP[3 * (order0 + 1)] = R.x; sP[3 * (order0 + 1) + 1] = R.y; sP[3 * (order0 + 1) + 2] = R.z;
      // the images, forward once (reflect_image), kept in LDS for the walk
      D3 im = T;
      simg[0] = im;
      for (int j = 1; j <= order0; ++j) {
        if (!((tm >> (j - 1)) & 1ull)) im = reflect_image(im, spl[j - 1]);
        simg[j] = im;
      }
      bool ok = image_walk(
          R, order0, [&](int j) { return simg[j]; }, [&](int j) { return spl[j]; },
          [&](int j, D3 q) {
            sP[3 * j] = q.x; sP[3 * j + 1] = q.y; sP[3 * j + 2] = q.z;
            return true;
          },
          sd);
      ok = ok && !through_opaque(a, sfaces, order0, (uint32_t)tm);
      double* P = a.pts + (size_t)u * (K + 2) * 3;
      for (int j = 0; j < 3 * (order0 + 2); ++j) P[j] = sP[j];
      a.length[u] = sd;
      sorder = order0;
      sok = ok ? 1 : 0;
      sfail = 0;
      // the task order: the sub-segments longest first (an occlusion query's
      // cost grows with the length it crosses), the field second, so that
      // wavefront 1 always computes it; tasks 0..3 go to wavefronts 0..3
      int n_seg = 0;
      double seg_len[kMaxK + 1];
      for (int j = 0; j <= order0; ++j) {
        const double dx = sP[3 * j + 3] - sP[3 * j], dy = sP[3 * j + 4] - sP[3 * j + 1],
                     dz = sP[3 * j + 5] - sP[3 * j + 2];
        const double l2 = dx * dx + dy * dy + dz * dz;
        int i = n_seg++;
        for (; i > 0 && seg_len[i - 1] < l2; --i) {
          seg_len[i] = seg_len[i - 1];
          stask[i + (i >= 1 ? 1 : 0)] = stask[i - 1 + (i - 1 >= 1 ? 1 : 0)];
        }
        seg_len[i] = l2;
        stask[i + (i >= 1 ? 1 : 0)] = j;
      }
      stask[1] = order0 + 1;
      snext = kRefineWaves;
    }
  }
  __syncthreads();
  const int order = sorder;
  bool ok = sok != 0;
  auto pt = [&](int j) { return D3{sP[3 * j], sP[3 * j + 1], sP[3 * j + 2]}; };
  // task positions are drawn in increasing order, each once: position 1 is
  // the field (wavefront 1 first), the others are sub-segments
  const int n_tasks = ok ? order + 2 : 0;
  int t = w;   // uniform over the wavefront
  auto draw = [&]() {
    int next = 0;
    if (lane == 0) next = atomicAdd(&snext, 1);
    t = __shfl(next, 0);
  };
  if (t == 1 && n_tasks > 1) {
    // ---- 3. the field, one lane per frequency (a path found invalid is
    // zeroed once every task is done)
    const double d = sd;
    const D3 aod = normed(pt(1) - pt(0));
    const double rho = sqrt(aod.x * aod.x + aod.y * aod.y);
    const D3 e0 = rho > 0 ? D3{aod.z * aod.x / rho, aod.z * aod.y / rho, -rho} : D3{aod.z, 0.0, 0.0};
    const double gain = pattern_gain(a.pat, aod);
    for (int fi = lane; fi < a.n_freqs; fi += kWave) {
      const double f = a.freqs[fi];
      double* out = a.amp + ((size_t)u * a.n_freqs + fi) * 6;
      Cx E[3] = {{e0.x, 0}, {e0.y, 0}, {e0.z, 0}};
      for (int j = 1; j <= order; ++j) {
        if ((stmask >> (j - 1)) & 1u) {
          // transmission: the penetration loss of the face's material
          // (Table II), polarisation and direction unchanged
          const double tf = a.mat_pen[a.face_material[sfaces[j - 1]]];
          for (int c = 0; c < 3; ++c) E[c] = cscl(tf, E[c]);
          continue;
        }
        const double4 pl = spl[j - 1];
        const D3 n = {pl.x, pl.y, pl.z};
        const D3 ki = normed(pt(j) - pt(j - 1));
        const D3 kr = normed(pt(j + 1) - pt(j));
        const double cos_t = fabs(dot(ki, n));
        D3 s = cross(ki, n);
        const double sl = len(s);
        if (sl < 1e-12) {
          const D3 ax = fabs(ki.x) < 0.9 ? D3{1, 0, 0} : D3{0, 1, 0};
          s = normed(cross(ki, ax));
        } else {
          s = (1.0 / sl) * s;
        }
        const D3 pin = cross(s, ki), pout = cross(s, kr);
        Cx te, tm;
        fresnel_coeffs(a.materials + 3 * a.face_material[sfaces[j - 1]], f, cos_t, te, tm);
        const Cx es = cadd(cadd(cscl(s.x, E[0]), cscl(s.y, E[1])), cscl(s.z, E[2]));
        const Cx ep = cadd(cadd(cscl(pin.x, E[0]), cscl(pin.y, E[1])), cscl(pin.z, E[2]));
        const Cx cs = cmul(te, es), cp = cmul(tm, ep);
        E[0] = cadd(cscl(s.x, cs), cscl(pout.x, cp));
        E[1] = cadd(cscl(s.y, cs), cscl(pout.y, cp));
        E[2] = cadd(cscl(s.z, cs), cscl(pout.z, cp));
      }
      const double lam = kC0 / f;
      const double k0 = 2.0 * kPi * f / kC0;
      const double mag = a.sqrt_pt * lam / (4.0 * kPi * d) * pow(10.0, -a.atten_db_per_km * d / 20000.0) * gain;
      double sn, cs;
      sincos(k0 * d, &sn, &cs);
      const Cx ph = {mag * cs, -mag * sn};
      for (int c = 0; c < 3; ++c) {
        const Cx v = cmul(ph, E[c]);
        out[2 * c] = v.re;
        out[2 * c + 1] = v.im;
      }
    }
    draw();
  }
  while (t < n_tasks) {
    // ---- 2. validation of sub-segment j: for j >= 1 also reflection point j
    // against its face
    const int j = stask[t];
    const uint64_t all = ~0ull;
    bool fail = false, fault = false;
    if (j >= 1) {
      const int f = sfaces[j - 1];
      const double4 pl = spl[j - 1];
      const bool inside = in_face(a, f, pt(j), D3{pl.x, pl.y, pl.z}, lane, kWave);
      fail = __ballot(inside) == 0;
    }
    const int fa = j >= 1 ? sfaces[j - 1] : -1;
    const int fb = j + 1 <= order ? sfaces[j] : -1;
    if (!fail && group_occluded(a, pt(j), pt(j + 1), fa, fb, stk[w], lane, all, fault)) fail = true;
    if (fail && lane == 0) sfail = 1;
    if (fault && lane == 0) atomicOr(a.err, DCEM_ERR_STACK);
    draw();
  }
  __syncthreads();
  // the outputs, by the wavefront that wrote the field (wavefront 0 when
  // there was none)
  if (w != (ok ? 1 : 0)) return;
  ok = ok && sfail == 0;
  D3 aod = {0, 0, 0}, aoa = {0, 0, 0};
  if (ok) {
    aod = normed(pt(1) - pt(0));
    aoa = normed(pt(order) - pt(order + 1));
  }
  if (lane == 0) {
    a.valid[u] = ok ? 1 : 0;
    a.tau[u] = ok ? sd / kC0 : 0.0;
    if (!ok) a.length[u] = 0.0;
    a.aod[3 * u] = aod.x; a.aod[3 * u + 1] = aod.y; a.aod[3 * u + 2] = aod.z;
    a.aoa[3 * u] = aoa.x; a.aoa[3 * u + 1] = aoa.y; a.aoa[3 * u + 2] = aoa.z;
  }
  if (!ok)
    for (int fi = lane; fi < a.n_freqs; fi += kWave)
      for (int k = 0; k < 6; ++k) a.amp[((size_t)u * a.n_freqs + fi) * 6 + k] = 0.0;
}


// ---- Visited-series discovery (Sec. III, the frame algorithm's steps 2-4:
// each new series of faces a ray visits is entered in the visited table of its
// depth and generates images, which are checked for a valid path; no capture
// sphere decides which series are tried).
//
// 1. Items: for every ray, the series of its first d hits for d = 1..(its
//    leading hits, at most K), plus the empty series of every source (the
//    direct paths).  Item key: words 0..W-1 hold (source, order, faces in path
//    order) in a candidate key's layout without the receiver field; word W
//    holds the item's ray id (kNoRay for an empty series), so after one sort
//    the head of each run of equal series carries the lowest ray visiting it.
// 2. Sort, run heads, compaction: the unique series, sorted, and per source
//    the start of its series.
// 3. Expansion: candidate u of the S x n_tgt (series, target) pairs, numbered
//    in the order of its path key (forward: source-major, then target, then
//    series; backward: target-major, then series), survives when its
//    image-method points lie strictly inside their segments and inside their
//    faces (the refinement's first checks, with the same code); survivors are
//    compacted in order into the decoded-candidate arrays.
__global__ __launch_bounds__(256) void k_series_items(const int32_t* __restrict__ face_log,
                                                      const uint8_t* __restrict__ ray_state, int64_t n_work,
                                                      int n_src, int los, KeyLayout S, uint32_t* __restrict__ keys,
                                                      int64_t stride, uint32_t* __restrict__ count, uint32_t cap) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  // the series of work item i: its interactions d = d0..depth (a branch
  // adds those through its last transmission; shorter ones are its parent's)
  int d0 = 1, depth = 0;
  uint32_t tset = 0, src = 0;
  if (i < (uint64_t)n_work) {
    depth = (int)(ray_state[i] & 0x0fu) - 1;   // interactions performed: segments - 1
    tset = S.branch_set[(i / (uint64_t)S.n_rays) % (uint32_t)S.n_branch];
    if (tset) d0 = 32 - __builtin_clz(tset);   // last transmission + 1
    src = (uint32_t)(i / ((uint64_t)S.n_rays * S.n_branch));
  }
  // interaction fields in bounce order (face, transmit bit)
  uint32_t fld[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j)
    fld[j] = j < depth ? ((uint32_t)face_log[(size_t)j * n_work + i] << S.tb) | ((tset >> j) & (uint32_t)S.tb) : 0u;
  // Neighbouring positions are rays of neighbouring directions and mostly
  // visit the same series: within a wavefront, a run of consecutive items
  // with the same series of length d enters it once, with the run's lowest
  // ray id (the sort below keeps the lowest over all entries, so the result
  // is the same).
  const uint32_t rid = i < (uint64_t)n_work ? ray_of(i, S) : kNoRay;
  const uint32_t psrc = __shfl_up(src, 1);
  const int pdepth = __shfl_up(depth, 1), pd0 = __shfl_up(d0, 1);
  uint32_t enter = 0;        // bit d - 1: this item enters its series of length d
  uint32_t run_min[kMaxK];   // the lowest ray id of that run
  bool eq = lane > 0 && psrc == src;
#pragma unroll
  for (int d = 1; d <= kMaxK; ++d) {
    run_min[d - 1] = kNoRay;
    if (d > S.K) continue;   // uniform
    eq = eq && __shfl_up(fld[d - 1], 1) == fld[d - 1];
    const bool has = d >= d0 && d <= depth;
    const bool same = has && eq && d >= pd0 && d <= pdepth;
    // runs: each starts at an item that does not continue its predecessor's
    const uint64_t starts = __ballot(!same);
    const uint64_t above = lane == kWave - 1 ? 0ull : starts & ~((2ull << lane) - 1ull);
    const int last = above ? __ffsll((unsigned long long)above) - 2 : kWave - 1;   // this lane's run ends here
    uint32_t m = has ? rid : kNoRay;
    for (int step = 1; step < kWave; step <<= 1) {   // suffix minimum within the run
      const uint32_t o = __shfl_down(m, step);
      if (lane + step <= last) m = min(m, o);
    }
    if (has && !same) {
      enter |= 1u << (d - 1);
      run_min[d - 1] = m;
    }
  }
  const bool empty_series = los && i < (uint32_t)n_src;
  const int n_items = __popc(enter) + (empty_series ? 1 : 0);
  // one append per block: wave scans, then the wave totals in LDS
  __shared__ uint32_t wsum[256 / kWave], bbase;
  const int wave = threadIdx.x / kWave;
  int incl = n_items;
  for (int off = 1; off < kWave; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == kWave - 1) wsum[wave] = (uint32_t)incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int v = 0; v < 256 / kWave; ++v) {
      const uint32_t x = wsum[v];
      wsum[v] = t;
      t += x;
    }
    bbase = t > 0 ? atomicAdd(count, t) : 0u;
  }
  __syncthreads();
  uint32_t slot = bbase + wsum[wave] + (uint32_t)(incl - n_items);
#pragma unroll
  for (int d = 1; d <= kMaxK; ++d) {
    if (!((enter >> (d - 1)) & 1u)) continue;
    if (slot < cap) {   // the host sizes cap for every item
      uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < d; ++j) put_bits(w, S.W, (S.K - 1 - j) * S.bf, S.bf, fld[S.backward ? d - 1 - j : j]);
      put_bits(w, S.W, S.K * S.bf, 4, (uint32_t)d);
      put_bits(w, S.W, S.K * S.bf + 4, S.bt, src);
      for (int k = 0; k < S.W; ++k) keys[k * stride + slot] = w[k];
      keys[S.W * stride + slot] = run_min[d - 1];
    }
    ++slot;
  }
  if (empty_series && slot < cap) {
    uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    put_bits(w, S.W, S.K * S.bf + 4, S.bt, i);
    for (int k = 0; k < S.W; ++k) keys[k * stride + slot] = w[k];
    keys[S.W * stride + slot] = kNoRay;
  }
}

// The unique series: per unique run s (heads in uniq_pos), its source, order,
// faces [K] (path order, -1 past the order) and lowest ray id (-1: the empty
// series).
struct SeriesOut {
  int32_t* src;
  int32_t* order;
  int32_t* first;
  int32_t* faces;
};

__global__ __launch_bounds__(256) void k_series_info(const uint32_t* __restrict__ keys, int64_t stride, KeyLayout S,
                                                     const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ uniq_pos,
                                                     const uint32_t* __restrict__ n_series, SeriesOut o) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *n_series) return;
  const uint32_t idx = perm[uniq_pos[s]];
  uint32_t w[8];
  for (int k = 0; k < S.W; ++k) w[k] = keys[k * stride + idx];
  const uint32_t order = key_bits(w, S.W, S.K * S.bf, 4);
  o.src[s] = (int32_t)key_bits(w, S.W, S.K * S.bf + 4, S.bt);
  o.order[s] = (int32_t)order;
  const uint32_t rid = keys[S.W * stride + idx];
  o.first[s] = rid == kNoRay ? -1 : (int32_t)rid;
  for (int j = 0; j < S.K; ++j)
    o.faces[(size_t)s * S.K + j] = (uint32_t)j < order ? field_face(key_bits(w, S.W, (S.K - 1 - j) * S.bf, S.bf), S.tb) : -1;
}

// start[src] = first unique series of source src (lower bound), start[n_src] = S.
__global__ __launch_bounds__(256) void k_series_starts(const int32_t* __restrict__ ser_src,
                                                       const uint32_t* __restrict__ n_series, int n_src,
                                                       uint32_t* __restrict__ start) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > n_src) return;
  uint32_t lo = 0, hi = *n_series;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ser_src[mid] < q) lo = mid + 1;
    else hi = mid;
  }
  start[q] = lo;
}

// Bounds of each face's vertices (as the tree holds them), for the
// expansion's pre-test of its in-face checks: [nf][6] lo xyz, hi xyz as
// order-preserving integer bits (min and max by integer atomics), one thread
// per face triangle; box must hold 0xffffffff in the lo words and 0 in the hi
// words.
__device__ inline uint32_t ordered_u32(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered_u32(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ __launch_bounds__(256) void k_face_boxes(const int32_t* __restrict__ face_tris,
                                                    const int32_t* __restrict__ tri_face,
                                                    const int32_t* __restrict__ face_slots,
                                                    const Leaf* __restrict__ tri4, int64_t nt, uint32_t* __restrict__ box) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const bool ok = k < nt;
  int f = -1;
  uint32_t b[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};   // ordered bits: lo x y z, hi x y z
  if (ok) {
    f = tri_face[face_tris[k]];
    const Leaf L = tri4[face_slots[k]];
    const float4 v[3] = {L.v0, L.v1, L.v2};
    for (int q = 0; q < 3; ++q) {
      const uint32_t o[3] = {ordered_u32(v[q].x), ordered_u32(v[q].y), ordered_u32(v[q].z)};
      for (int a = 0; a < 3; ++a) {
        b[a] = min(b[a], o[a]);
        b[3 + a] = max(b[3 + a], o[a]);
      }
    }
  }
  // a face's triangles are consecutive: each run of one face in the
  // wavefront is reduced first and enters the face's box with one set of
  // atomics (a face of many triangles would otherwise serialise on them)
  const bool head = ok && (lane == 0 || __shfl_up(f, 1) != f);
  const uint64_t starts = __ballot(!ok || head);
  const uint64_t above = lane == kWave - 1 ? 0ull : starts & ~((2ull << lane) - 1ull);
  const int last = above ? __ffsll((unsigned long long)above) - 2 : kWave - 1;
  for (int step = 1; step < kWave; step <<= 1) {
    uint32_t o[6];
    for (int a = 0; a < 6; ++a) o[a] = __shfl_down(b[a], step);
    if (lane + step <= last) {
      for (int a = 0; a < 3; ++a) {
        b[a] = min(b[a], o[a]);
        b[3 + a] = max(b[3 + a], o[3 + a]);
      }
    }
  }
  if (head) {
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[6 * f + a], b[a]);
      atomicMax(&box[6 * f + 3 + a], b[3 + a]);
    }
  }
}

__global__ void k_face_box_init(uint32_t* __restrict__ box, int nf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 6 * nf) box[i] = (i % 6) < 3 ? 0xffffffffu : 0u;
}

// May p lie in face f?  The two coordinates in_face keeps (the normal's
// dominant axis dropped) against the face's bounds: a point in_face accepts
// always passes (it lies in a triangle's projection, inside the bounds of its
// vertices), so this only skips checks that would fail.
__device__ inline bool in_face_bounds(const uint32_t* __restrict__ box, int f, D3 p, D3 n) {
  const double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
  const int drop = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  const uint32_t* b = box + 6 * f;
  auto inside = [&](double u, int a) {
    return u >= (double)from_ordered_u32(b[a]) && u <= (double)from_ordered_u32(b[3 + a]);
  };
  return (drop == 0 || inside(p.x, 0)) && (drop == 1 || inside(p.y, 1)) && (drop == 2 || inside(p.z, 2));
}

struct ExpandArgs {
  SeriesOut ser;
  const uint32_t* start;   // [n_src + 1]
  uint32_t n_series;
  uint64_t n_cand;         // n_series * n_tgt
  int n_src, n_tgt, n_rx, K;
  bool backward;
  const float* src_pos;
  const float* tgt_pos;
  RefineArgs ra;           // faces: planes, triangles (in_face)
  const uint32_t* face_box;   // [nf][6] face bounds as ordered bits (k_face_boxes)
  uint64_t* mask;          // [ceil(n_cand / 64)] survivors, one bit per candidate
  uint32_t* block_cnt;     // survivors per block, then (scanned) their offsets
  uint32_t capacity;       // decoded-candidate entries available
  uint32_t* err;           // DCEM_ERR_CAPTURES when survivors exceed the capacity
  UniqueOut out;
};

// (series, target) of candidate u, in path-key order.
__device__ inline void expand_index(const ExpandArgs& e, uint64_t u, uint32_t& s, uint32_t& tgt) {
  if (e.backward) {
    tgt = (uint32_t)(u / e.n_series);
    s = (uint32_t)(u - (uint64_t)tgt * e.n_series);
    return;
  }
  // the source whose block [start * n_tgt, start' * n_tgt) holds u
  int lo = 0, hi = e.n_src - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint64_t)e.start[mid] * e.n_tgt <= u) lo = mid;
    else hi = mid - 1;
  }
  const uint64_t local = u - (uint64_t)e.start[lo] * e.n_tgt;
  const uint32_t cnt = e.start[lo + 1] - e.start[lo];
  tgt = (uint32_t)(local / cnt);
  s = e.start[lo] + (uint32_t)(local - (uint64_t)tgt * cnt);
}

// write = 0: survivor mask and per-block counts; write = 1: the survivors'
// decoded candidates at the scanned block offsets.
__global__ __launch_bounds__(256) void k_expand(ExpandArgs e, int write) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  __shared__ uint32_t wcnt[256 / kWave];
  bool keep = false;
  uint32_t s = 0, tgt = 0;
  if (u < e.n_cand) {
    if (write) {
      keep = (e.mask[u / kWave] >> lane) & 1ull;
      if (keep) expand_index(e, u, s, tgt);
    } else {
      expand_index(e, u, s, tgt);
      const int order = e.ser.order[s];
      const uint32_t src = (uint32_t)e.ser.src[s];
      const uint32_t txi = e.backward ? tgt : src, rxi = e.backward ? src : tgt;
      const D3 T = fvec(e.backward ? e.tgt_pos : e.src_pos, (int)txi);
      const D3 R = fvec(e.backward ? e.src_pos : e.tgt_pos, (int)rxi);
      const int32_t* fs = e.ser.faces + (size_t)s * e.K;
      uint32_t tmask = 0;
      bool opaque = false;
      for (int j = 0; j < order; ++j) {
        const int32_t fe = fs[j];
        if (fe & kTransmit) {
          tmask |= 1u << j;
          opaque = opaque || e.ra.mat_pen[e.ra.face_material[fe & kFaceMask]] == 0.0;
        }
      }
      double d;
      // each point is tested against its face as soon as the walk reaches it
      auto plane = [&](int j) { return e.ra.plane[fs[j] & kFaceMask]; };
      // images recomputed when the walk needs them (no arrays), with the
      // refinement's reflect_image
      auto image = [&](int j) {
        D3 im = T;
        for (int q = 1; q <= j; ++q)
          if (!((tmask >> (q - 1)) & 1u)) im = reflect_image(im, plane(q - 1));
        return im;
      };
      keep = !opaque && image_walk(
                            R, order, image, plane,
                            [&](int j, D3 q) {
                              const int f = fs[j - 1] & kFaceMask;
                              const double4 pl = e.ra.plane[f];
                              const D3 n = {pl.x, pl.y, pl.z};
                              return in_face_bounds(e.face_box, f, q, n) && in_face(e.ra, f, q, n);
                            },
                            d);
    }
  }
  const uint64_t m = __ballot(keep);
  if (!write) {
    if (lane == 0 && u < e.n_cand) e.mask[u / kWave] = m;
    if (lane == 0) wcnt[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int v = 0; v < 256 / kWave; ++v) t += wcnt[v];
      e.block_cnt[blockIdx.x] = t;
    }
    return;
  }
  if (lane == 0) wcnt[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t pos = e.block_cnt[blockIdx.x];
  for (int v = 0; v < wave; ++v) pos += wcnt[v];
  pos += (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
  if (!keep) return;
  if (pos >= e.capacity) {
    atomicOr(e.err, DCEM_ERR_CAPTURES);
    return;
  }
  const int order = e.ser.order[s];
  const uint32_t src = (uint32_t)e.ser.src[s];
  const uint32_t txi = e.backward ? tgt : src, rxi = e.backward ? src : tgt;
  e.out.pair[pos] = (int32_t)(txi * (uint32_t)e.n_rx + rxi);
  e.out.order[pos] = (uint8_t)order;
  for (int j = 0; j < e.K; ++j) e.out.faces[(size_t)pos * e.K + j] = e.ser.faces[(size_t)s * e.K + j];
  e.out.first_ray[pos] = e.ser.first[s];
}

// The run of `key` in the sorted array a[0, n): [start, end) with a[i] == key,
// by one wavefront (all lanes call it with the same arguments): 64-way splits
// of both bounds at once, each round one load per lane and bound, so the run
// is found in log64(n) memory round trips instead of 2 log2(n).
__device__ inline void wave_run(const int32_t* __restrict__ a, int n, int key, int lane, int& start, int& end) {
  int lo0 = 0, hi0 = n, lo1 = 0, hi1 = n;   // first index with a[i] >= key, with a[i] > key
  while (lo0 < hi0 || lo1 < hi1) {          // uniform over the wavefront
    const int s0 = max((hi0 - lo0 + kWave - 1) / kWave, 1), s1 = max((hi1 - lo1 + kWave - 1) / kWave, 1);
    const int q0 = lo0 + lane * s0, q1 = lo1 + lane * s1;
    const bool b0 = q0 < hi0 && a[q0] < key;    // a prefix of the lanes (a is sorted)
    const bool b1 = q1 < hi1 && a[q1] <= key;
    const int c0 = __popcll(__ballot(b0)), c1 = __popcll(__ballot(b1));
    if (lo0 < hi0) {
      if (c0 == 0) {
        hi0 = lo0;
      } else {
        const int nl = lo0 + (c0 - 1) * s0 + 1;
        hi0 = min(hi0, lo0 + c0 * s0);
        lo0 = nl;
      }
    }
    if (lo1 < hi1) {
      if (c1 == 0) {
        hi1 = lo1;
      } else {
        const int nl = lo1 + (c1 - 1) * s1 + 1;
        hi1 = min(hi1, lo1 + c1 * s1);
        lo1 = nl;
      }
    }
  }
  start = lo0;
  end = lo1;
}

// One wavefront per (tx, rx): sum the valid paths of that pair (contiguous in
// key order) with a fixed lane assignment and butterfly, so the result is
// bitwise reproducible.
__global__ __launch_bounds__(256) void k_reduce(const int32_t* __restrict__ pair, const uint8_t* __restrict__ valid,
                                                const double* __restrict__ amp, const uint32_t* __restrict__ n_unique,
                                                int n_pairs, int n_freqs, double* __restrict__ p_coh,
                                                double* __restrict__ p_inc, uint32_t* __restrict__ counters) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  // the re-trace has read this frame's list length: zero it for the next
  // frame's revalidation (which may start before that frame's lists are reset)
  if (blockIdx.x == 0 && threadIdx.x == 0) counters[kCntList] = 0;
  __shared__ uint32_t nvalid;   // valid paths of the block's pairs
  if (threadIdx.x == 0) nvalid = 0;
  __syncthreads();
  if (wave < n_pairs) {
    const int n = (int)*n_unique;
    int start, end;
    wave_run(pair, n, wave, lane, start, end);
    uint32_t nv = 0;
    for (int u = start + lane; u < end; u += 64) nv += valid[u] ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
    if (lane == 0 && nv) atomicAdd(&nvalid, nv);
    for (int fi = 0; fi < n_freqs; ++fi) {
      double acc[6] = {0, 0, 0, 0, 0, 0};
      double inc = 0.0;
      for (int u = start + lane; u < end; u += 64) {
        if (!valid[u]) continue;
        const double* v = amp + ((size_t)u * n_freqs + fi) * 6;
        for (int k = 0; k < 6; ++k) {
          acc[k] += v[k];
          inc += v[k] * v[k];
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        for (int k = 0; k < 6; ++k) acc[k] += __shfl_xor(acc[k], off);
        inc += __shfl_xor(inc, off);
      }
      if (lane == 0) {
        double pc = 0.0;
        for (int k = 0; k < 6; ++k) pc += acc[k] * acc[k];
        p_coh[(size_t)fi * n_pairs + wave] = pc;
        p_inc[(size_t)fi * n_pairs + wave] = inc;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && nvalid) atomicAdd(&counters[kCntValid], nvalid);
}

// Power gradients along the frame's paths, one wavefront per (tx, rx) pair:
// the coherent field A = sum_p a_p per frequency (fixed butterfly), then, one
// lane per (path, material) item, the derivative of the path's amplitude with
// respect to the material's eps_c, carried forward through its reflections (E -> Gamma_TE (E.s) s
// + Gamma_TM (E.p_in) p_out, plus the map with the Gammas' derivatives at a
// face of material m), and dP/dtheta = 2 Re sum_c conj(A_c) dA_c/dtheta with
// d/deps_r = d/deps_c and d/dsigma = -j / (2 pi f eps0) d/deps_c.  Each
// reflection's normal is taken from the path itself (along k_out - k_in), so
// the pass reads only the frame's path arrays.  Out: [freq][pair][material]
// (g_eps null: skipped).  With the transmit pattern, a_p = g(phi_p) a_p^iso:
// the material derivatives carry the gain, and g_pat (nullable) receives
// dP/dw_j = 2 Re sum_c conj(A_c) sum_p B_j(phi_p) a_pc^iso, [freq][pair][16].
__global__ __launch_bounds__(256) void k_power_grad(const int32_t* __restrict__ pair, const uint8_t* __restrict__ valid,
                                                    const double* __restrict__ amp, const double* __restrict__ pts,
                                                    const uint8_t* __restrict__ order, const int32_t* __restrict__ faces,
                                                    const double* __restrict__ length, uint32_t n_unique, int K,
                                                    int n_pairs, const double* __restrict__ freqs, int n_freqs,
                                                    const int32_t* __restrict__ face_material,
                                                    const double* __restrict__ materials,
                                                    const double* __restrict__ mat_pen, int n_mat, double sqrt_pt,
                                                    double atten_db_per_km, TxPattern pat, double* __restrict__ g_eps,
                                                    double* __restrict__ g_sig, double* __restrict__ g_pat) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= n_pairs) return;   // uniform per wavefront
  const int n = (int)n_unique;
  int start, end;
  wave_run(pair, n, wave, lane, start, end);
  auto butterfly = [](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
  };
  auto departure = [&](int u) {
    const double* P = pts + (size_t)u * (K + 2) * 3;
    return normed(D3{P[3] - P[0], P[4] - P[1], P[5] - P[2]});
  };
  // Field of path u at frequency f through its reflection chain (unit
  // magnitude and phase), and with m >= 0 its forward-mode derivative with
  // respect to material m's eps_c.
  auto walk = [&](int u, double f, int m, Cx* E, Cx* dE) {
    const int ord = order[u];
    const double* P = pts + (size_t)u * (K + 2) * 3;
    auto pt = [&](int j) { return D3{P[3 * j], P[3 * j + 1], P[3 * j + 2]}; };
    const D3 aod = normed(pt(1) - pt(0));
    const double rho = sqrt(aod.x * aod.x + aod.y * aod.y);
    const D3 e0 = rho > 0 ? D3{aod.z * aod.x / rho, aod.z * aod.y / rho, -rho} : D3{aod.z, 0.0, 0.0};
    E[0] = {e0.x, 0};
    E[1] = {e0.y, 0};
    E[2] = {e0.z, 0};
    for (int c = 0; c < 3; ++c) dE[c] = {0, 0};
    for (int j = 1; j <= ord; ++j) {
      const int32_t fe = faces[(size_t)u * K + j - 1];
      const int mat = face_material[fe & kFaceMask];
      if (fe & kTransmit) {
        // a transmission scales the field (and its derivatives) by its loss,
        // which no material parameter here changes
        const double tf = mat_pen[mat];
        for (int c = 0; c < 3; ++c) {
          E[c] = cscl(tf, E[c]);
          dE[c] = cscl(tf, dE[c]);
        }
        continue;
      }
      const D3 ki = normed(pt(j) - pt(j - 1));
      const D3 kr = normed(pt(j + 1) - pt(j));
      const D3 dk = kr - ki;   // along the normal (zero only at grazing incidence)
      const double dkl = len(dk);
      const D3 nrm = dkl > 0.0 ? (1.0 / dkl) * dk : D3{0.0, 0.0, 1.0};
      const double cos_t = fabs(dot(ki, nrm));
      D3 sv = cross(ki, nrm);
      const double sl = len(sv);
      if (sl < 1e-12) {
        const D3 ax = fabs(ki.x) < 0.9 ? D3{1, 0, 0} : D3{0, 1, 0};
        sv = normed(cross(ki, ax));
      } else {
        sv = (1.0 / sl) * sv;
      }
      const D3 pin = cross(sv, ki), pout = cross(sv, kr);
      Cx te, tm;
      fresnel_coeffs(materials + 3 * mat, f, cos_t, te, tm);
      auto apply = [&](const Cx* X, Cx a, Cx b, Cx* Y) {   // Y = a (X.s) s + b (X.p_in) p_out
        const Cx xs = cadd(cadd(cscl(sv.x, X[0]), cscl(sv.y, X[1])), cscl(sv.z, X[2]));
        const Cx xp = cadd(cadd(cscl(pin.x, X[0]), cscl(pin.y, X[1])), cscl(pin.z, X[2]));
        const Cx cs = cmul(a, xs), cp = cmul(b, xp);
        Y[0] = cadd(cscl(sv.x, cs), cscl(pout.x, cp));
        Y[1] = cadd(cscl(sv.y, cs), cscl(pout.y, cp));
        Y[2] = cadd(cscl(sv.z, cs), cscl(pout.z, cp));
      };
      Cx nd[3], ne[3];
      if (m >= 0) {
        apply(dE, te, tm, nd);
        if (mat == m) {
          Cx dte, dtm, extra[3];
          fresnel_deps(materials + 3 * mat, f, cos_t, dte, dtm);
          apply(E, dte, dtm, extra);
          for (int c = 0; c < 3; ++c) nd[c] = cadd(nd[c], extra[c]);
        }
        for (int c = 0; c < 3; ++c) dE[c] = nd[c];
      }
      apply(E, te, tm, ne);
      for (int c = 0; c < 3; ++c) E[c] = ne[c];
    }
  };
  const int nme = g_eps ? n_mat : 0;                // material tasks
  const int T = nme + (g_pat ? 1 : 0);               // tasks per path
  const int n_items = (end - start) * T;
  for (int fi = 0; fi < n_freqs; ++fi) {
    const double f = freqs[fi];
    double A[6] = {0, 0, 0, 0, 0, 0};
    for (int u = start + lane; u < end; u += 64) {
      if (!valid[u]) continue;
      const double* v = amp + ((size_t)u * n_freqs + fi) * 6;
      for (int k = 0; k < 6; ++k) A[k] += v[k];
    }
    for (int k = 0; k < 6; ++k) A[k] = butterfly(A[k]);
    const double lam = kC0 / f, k0 = 2.0 * kPi * f / kC0;
    const Cx dsig = {0.0, -1.0 / (2.0 * kPi * f * kEps0)};
    // magnitude and phase of path u without the pattern's gain
    auto phase = [&](int u) {
      const double d = length[u];
      const double mag = sqrt_pt * lam / (4.0 * kPi * d) * pow(10.0, -atten_db_per_km * d / 20000.0);
      double sn, cs;
      sincos(k0 * d, &sn, &cs);
      return Cx{mag * cs, -mag * sn};
    };
    // Items (path, task) over the lanes, task < nme: material task, task ==
    // nme: the pattern; each round's per-task sums by fixed butterflies, the
    // rounds added in order by lane 0 (bitwise reproducible).
    for (int base = 0; base < max(n_items, 1); base += 64) {   // uniform per wavefront
      const int it = base + lane;
      int task = -1, jt = 0;
      double v0 = 0.0, v1 = 0.0;
      if (it < n_items) {
        const int u = start + it / T;
        task = it % T;
        const int m = task < nme ? task : -1;
        bool act = valid[u] != 0;
        if (act && m >= 0) {
          bool uses = false;
          for (int j = 0; j < order[u]; ++j) {
            const int32_t fe = faces[(size_t)u * K + j];
            uses = uses || (!(fe & kTransmit) && face_material[fe & kFaceMask] == m);
          }
          act = uses;
        }
        if (act) {
          Cx E[3], dE[3];
          walk(u, f, m, E, dE);
          const Cx ph = phase(u);
          if (m >= 0) {
            const Cx phg = cscl(pattern_gain(pat, departure(u)), ph);
            for (int c = 0; c < 3; ++c) {
              const Cx da = cmul(phg, dE[c]);             // d a_c / d eps_c
              const Cx ds = cmul(dsig, da);               // d a_c / d sigma
              const Cx Ac = {A[2 * c], -A[2 * c + 1]};    // conj(A_c)
              v0 += 2.0 * cmul(Ac, da).re;
              v1 += 2.0 * cmul(Ac, ds).re;
            }
          } else {
            // a_p = g(phi_p) a_p^iso: d a_p / d w_j = B_j(phi_p) a_p^iso, nonzero
            // for the two taps around the departure azimuth
            for (int c = 0; c < 3; ++c) v0 += 2.0 * cmul(Cx{A[2 * c], -A[2 * c + 1]}, cmul(ph, E[c])).re;
            pattern_cell(departure(u), jt, v1);
          }
        }
      }
      const size_t row = (size_t)fi * n_pairs + wave;
      for (int m = 0; m < nme; ++m) {
        const double e = butterfly(task == m ? v0 : 0.0);
        const double sg = butterfly(task == m ? v1 : 0.0);
        if (lane == 0) {
          g_eps[row * n_mat + m] = (base ? g_eps[row * n_mat + m] : 0.0) + e;
          g_sig[row * n_mat + m] = (base ? g_sig[row * n_mat + m] : 0.0) + sg;
        }
      }
      if (g_pat) {
        const bool ip = task == nme;
        const int j1 = (jt + 1) & (kPatternTaps - 1);
#pragma unroll
        for (int q = 0; q < kPatternTaps; ++q) {
          const double cq = ip ? (q == jt ? (1.0 - v1) * v0 : 0.0) + (q == j1 ? v1 * v0 : 0.0) : 0.0;
          const double v = butterfly(cq);
          if (lane == 0) g_pat[row * kPatternTaps + q] = (base ? g_pat[row * kPatternTaps + q] : 0.0) + v;
        }
      }
    }
  }
}

int bits_for(int64_t n_values) {
  int b = 0;
  while (((int64_t)1 << b) < n_values) ++b;
  return b;
}

KeyLayout key_layout(const dcem_ctx* c) {
  KeyLayout L;
  L.bt = bits_for(c->n_tx);
  L.br = bits_for(c->n_rx);
  L.tb = c->max_trans > 0 ? 1 : 0;
  L.bf = std::max(1, bits_for(c->nf)) + L.tb;
  L.K = c->K;
  L.n_branch = c->n_branch;
  L.branch_set = static_cast<const uint32_t*>(c->branch_set.p);
  L.n_rx = c->n_rx;
  L.n_tgt = c->n_tgt;
  L.backward = c->backward;
  L.ray_order = static_cast<const uint32_t*>(c->ray_order.p);
  L.n_rays = std::max<int64_t>(c->n_rays, 1);
  L.bits = L.bt + L.br + 4 + L.K * L.bf;
  L.W = (L.bits + 31) / 32;
  return L;
}

}  // namespace

bool small_path_fits(const dcem_ctx* c) { return key_layout(c).W <= kSmallW; }
int64_t small_path_capacity() { return kSmallN; }

hipError_t ensure_paths(dcem_ctx* c, int64_t n) {
  hipError_t e;
  n = std::max<int64_t>(n, 1);
  if ((e = ensure(c->path_valid, n)) != hipSuccess) return e;
  if ((e = ensure(c->path_len, 8 * n)) != hipSuccess) return e;
  if ((e = ensure(c->path_tau, 8 * n)) != hipSuccess) return e;
  if ((e = ensure(c->path_aod, 24 * n)) != hipSuccess) return e;
  if ((e = ensure(c->path_aoa, 24 * n)) != hipSuccess) return e;
  if ((e = ensure(c->path_amp, 48 * n * (size_t)c->n_freqs)) != hipSuccess) return e;
  if ((e = ensure(c->first_ray, 4 * n)) != hipSuccess) return e;
  if ((e = ensure(c->pair_range, 4 * n)) != hipSuccess) return e;
  if ((e = ensure(c->path_order, n)) != hipSuccess) return e;
  if ((e = ensure(c->path_faces, 4 * n * (size_t)std::max(c->K, 1))) != hipSuccess) return e;
  if ((e = ensure(c->path_pts, 24 * n * (size_t)(c->K + 2))) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t prepare_small_candidates(dcem_ctx* c) {
  hipError_t e;
  const KeyLayout L = key_layout(c);
  if ((e = ensure(c->cand_keys, sizeof(uint32_t) * L.W * kSmallN)) != hipSuccess) return e;
  if ((e = ensure(c->cand_perm, sizeof(uint32_t) * kSmallN)) != hipSuccess) return e;
  if ((e = ensure(c->uniq_idx, sizeof(uint32_t) * (kSmallN + 1))) != hipSuccess) return e;
  return ensure_paths(c, kSmallN);
}

// Buffers of the sort-based de-duplication for n captures (keys, permutation,
// run heads and block counts, unique positions, paths, the sort's histograms).
hipError_t prepare_sorted_candidates(dcem_ctx* c, int64_t n) {
  hipError_t e;
  n = std::max<int64_t>(n, 1);
  const KeyLayout L = key_layout(c);
  const int64_t nb = (n + 255) / 256;
  if ((e = ensure(c->cand_keys, sizeof(uint32_t) * L.W * n)) != hipSuccess) return e;
  if ((e = ensure(c->cand_perm, sizeof(uint32_t) * 2 * n)) != hipSuccess) return e;
  if ((e = ensure(c->cand_tmp, n + 16 + sizeof(uint32_t) * (nb + 8))) != hipSuccess) return e;
  if ((e = ensure(c->uniq_idx, sizeof(uint32_t) * (n + 1))) != hipSuccess) return e;
  if ((e = ensure_paths(c, n)) != hipSuccess) return e;
  return prepare_sort(c, n);
}

namespace {

// Size-hinted path: more captures than the buffers were sized for leave the
// frame's candidates to the host's exact redo (as the one-workgroup path does).
__global__ void k_fit_check(const uint32_t* __restrict__ n_caps, uint32_t n_max, uint32_t* __restrict__ n_unique,
                            uint32_t* __restrict__ fallback) {
  if (threadIdx.x == 0 && *n_caps > n_max) {
    *fallback = 1;
    *n_unique = 0;
  }
}

}  // namespace

// Candidate keys, sort and unique.  `small`: one workgroup de-duplicates up to
// kSmallN captures whose count it reads on the device (no host round trip; a
// larger count raises the fallback counter and the host redoes the frame's
// candidates exactly).  `hint` > 0: the sort-based path with every size taken
// from `hint` and the capture count read on the device (no host round trip;
// more captures than `hint` fall back the same way).  Otherwise the capture
// count is read back first.
hipError_t build_candidates(dcem_ctx* c, bool small, int64_t hint) {
  hipError_t e;
  // the de-duplication writes each unique candidate's decoded record into
  // the path arrays
  uint32_t* cnt = c->cnt_dev;
  const KeyLayout L = key_layout(c);
  c->key_words = L.W;
  c->bits_tx = L.bt;
  c->bits_rx = L.br;
  c->bits_face = L.bf;
  const int64_t n_work = (int64_t)c->n_src * c->n_branch * c->n_rays;
  if (small) {
    if ((e = ensure(c->cand_keys, sizeof(uint32_t) * L.W * kSmallN)) != hipSuccess) return e;
    if ((e = ensure(c->cand_perm, sizeof(uint32_t) * kSmallN)) != hipSuccess) return e;
    if ((e = ensure(c->uniq_idx, sizeof(uint32_t) * (kSmallN + 1))) != hipSuccess) return e;
    c->key_stride = kSmallN;
    c->path_cap = kSmallN;
    c->small_path = true;
    if ((e = ensure_paths(c, c->path_cap)) != hipSuccess) return e;
    launch_small_dedupe(c, L, n_work);
    return hipGetLastError();
  }
  c->small_path = false;
  const bool device_count = hint > 0;
  uint32_t n_max = 0;
  if (device_count) {
    n_max = (uint32_t)std::min<int64_t>(hint, c->cap_capacity);
  } else {
    uint32_t n_caps = 0;
    if ((e = hipMemcpyAsync(&n_caps, cnt + kCntCaptures, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    if (n_caps > c->cap_capacity) n_caps = (uint32_t)c->cap_capacity;
    c->n_caps_host = n_caps;
    if (n_caps <= (uint32_t)kSmallN && L.W <= kSmallW) {
      c->path_cap = n_caps;
      if ((e = ensure_paths(c, std::max<int64_t>(n_caps, 1))) != hipSuccess) return e;
      if ((e = ensure(c->cand_keys, sizeof(uint32_t) * L.W * kSmallN)) != hipSuccess) return e;
      if ((e = ensure(c->cand_perm, sizeof(uint32_t) * kSmallN)) != hipSuccess) return e;
      if ((e = ensure(c->uniq_idx, sizeof(uint32_t) * (kSmallN + 1))) != hipSuccess) return e;
      c->key_stride = kSmallN;
      launch_small_dedupe(c, L, n_work);
      return hipGetLastError();
    }
    n_max = n_caps;
  }
  const int64_t n = std::max<int64_t>(n_max, 1);
  c->path_cap = n_max;
  c->key_stride = n;
  if ((e = prepare_sorted_candidates(c, n)) != hipSuccess) return e;
  if (n_max == 0) return hipSuccess;   // the unique counter was cleared at frame start
  const int nb = (int)((n + 255) / 256);
  uint32_t* keys = ptr<uint32_t>(c->cand_keys);
  uint32_t* perm = ptr<uint32_t>(c->cand_perm);
  uint8_t* head = ptr<uint8_t>(c->cand_tmp);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(ptr<uint8_t>(c->cand_tmp) + ((n + 15) / 16) * 16);
  const uint32_t* n_dev = cnt + kCntCaptures;
  hipLaunchKernelGGL(k_keys, dim3(nb), dim3(256), 0, c->stream, ptr<Capture>(c->caps[c->cur_caps]), n_dev, n_max,
                     ptr<int32_t>(c->face_log), n_work, L, keys, (int64_t)n);
  if ((e = radix_sort_perm(c, keys, L.W, L.bits, n_dev, n, perm, perm + n, c->stream)) != hipSuccess) return e;
  // the sort's second permutation buffer is free after the sort: the runs'
  // lowest ray ids
  uint32_t* run_min = perm + n;
  hipLaunchKernelGGL(k_heads, dim3(nb), dim3(256), 0, c->stream, keys, (int64_t)n, L.W, perm, n_dev, n_max, head, bcnt,
                     run_min);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, c->stream, bcnt, nb, cnt + kCntUnique);
  hipLaunchKernelGGL(k_compact, dim3(nb), dim3(256), 0, c->stream, head, bcnt, n_dev, n_max, cnt + kCntUnique,
                     ptr<uint32_t>(c->uniq_idx), run_min, perm, ptr<Capture>(c->caps[c->cur_caps]), L);
  hipLaunchKernelGGL(k_unique_info, dim3(nb), dim3(256), 0, c->stream, keys, (int64_t)n, L, perm,
                     ptr<uint32_t>(c->uniq_idx), cnt + kCntUnique, run_min, unique_out(c));
  if (device_count)
    hipLaunchKernelGGL(k_fit_check, dim3(1), dim3(64), 0, c->stream, n_dev, n_max, cnt + kCntUnique,
                       cnt + kCntFallback);
  return hipGetLastError();
}

hipError_t build_visited_candidates(dcem_ctx* c, bool los, bool& too_many) {
  hipError_t e;
  too_many = false;
  c->small_path = false;
  c->path_cap = 0;
  // the series key: a candidate key's layout with the source in the
  // transmitter field and no receiver field, then the ray id word
  KeyLayout S = key_layout(c);
  S.bt = bits_for(c->n_src);
  S.br = 0;
  S.bits = S.bt + 4 + S.K * S.bf;
  S.W = (S.bits + 31) / 32;
  const int Wt = S.W + 1;
  const int64_t n_work = (int64_t)c->n_src * c->n_branch * c->n_rays;
  const int64_t cap = (los ? c->n_src : 0) + n_work * c->K;
  if (cap == 0) return hipSuccess;   // no series: no candidates (the unique counter was cleared)
  if (cap >= ((int64_t)1 << 32) - 1) {
    too_many = true;
    return hipSuccess;
  }
  const int nb = (int)((cap + 255) / 256);
  if ((e = ensure(c->cand_keys, sizeof(uint32_t) * Wt * cap)) != hipSuccess) return e;
  if ((e = ensure(c->cand_perm, sizeof(uint32_t) * 2 * cap)) != hipSuccess) return e;
  if ((e = ensure(c->cand_tmp, cap + 16 + sizeof(uint32_t) * (nb + 8))) != hipSuccess) return e;
  if ((e = ensure(c->uniq_idx, sizeof(uint32_t) * (cap + 1))) != hipSuccess) return e;
  // series_buf: [0] item count, [1] series count (256 B), then the series
  // arrays (source, order, lowest ray, faces [K]) and the per-source starts
  const size_t K = (size_t)std::max(c->K, 1);
  const size_t ser_bytes = 256 + sizeof(int32_t) * (size_t)cap * (3 + K) + sizeof(uint32_t) * ((size_t)c->n_src + 1);
  if ((e = ensure(c->series_buf, ser_bytes)) != hipSuccess) return e;
  uint32_t* sc = ptr<uint32_t>(c->series_buf);
  SeriesOut so;
  so.src = reinterpret_cast<int32_t*>(ptr<char>(c->series_buf) + 256);
  so.order = so.src + cap;
  so.first = so.order + cap;
  so.faces = so.first + cap;
  uint32_t* start = reinterpret_cast<uint32_t*>(so.faces + (size_t)cap * K);
  uint32_t* keys = ptr<uint32_t>(c->cand_keys);
  uint32_t* perm = ptr<uint32_t>(c->cand_perm);
  uint8_t* head = ptr<uint8_t>(c->cand_tmp);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(ptr<uint8_t>(c->cand_tmp) + ((cap + 15) / 16) * 16);
  fill_u32(sc, 0u, 2, c->stream);
  const int64_t n_thr = std::max<int64_t>(n_work, c->n_src);
  hipLaunchKernelGGL(k_series_items, dim3((unsigned)((n_thr + 255) / 256)), dim3(256), 0, c->stream,
                     ptr<int32_t>(c->face_log), ptr<uint8_t>(c->ray_state), n_work, c->n_src, los ? 1 : 0, S, keys,
                     cap, sc, (uint32_t)cap);
  uint32_t n_items = 0;
  if ((e = hipMemcpyAsync(&n_items, sc, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  if (n_items == 0) return hipSuccess;
  n_items = std::min<uint32_t>(n_items, (uint32_t)cap);
  // sized by the items there are (read above), on the bits of ray ids there are
  if ((e = radix_sort_perm(c, keys, Wt, 32 + S.bits, sc, n_items, perm, perm + cap, c->stream, cap,
                           bits_for(n_work))) != hipSuccess)
    return e;
  const int nbi = (int)((n_items + 255) / 256);
  hipLaunchKernelGGL(k_heads, dim3(nbi), dim3(256), 0, c->stream, keys, (int64_t)cap, S.W, perm, sc, n_items, head,
                     bcnt, nullptr);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, c->stream, bcnt, nbi, sc + 1);
  hipLaunchKernelGGL(k_compact, dim3(nbi), dim3(256), 0, c->stream, head, bcnt, sc, n_items, sc + 1,
                     ptr<uint32_t>(c->uniq_idx), nullptr, nullptr, nullptr, S);
  hipLaunchKernelGGL(k_series_info, dim3(nbi), dim3(256), 0, c->stream, keys, (int64_t)cap, S, perm,
                     ptr<uint32_t>(c->uniq_idx), sc + 1, so);
  hipLaunchKernelGGL(k_series_starts, dim3((c->n_src + 1 + 255) / 256), dim3(256), 0, c->stream, so.src, sc + 1,
                     c->n_src, start);
  uint32_t n_series = 0;
  if ((e = hipMemcpyAsync(&n_series, sc + 1, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  const uint64_t n_cand = (uint64_t)n_series * (uint64_t)c->n_tgt;
  if (n_cand == 0) return hipSuccess;
  if (n_cand >= ((uint64_t)1 << 32) - 256) {
    too_many = true;
    return hipSuccess;
  }
  const uint32_t nbe = (uint32_t)((n_cand + 255) / 256);
  const size_t mask_words = (size_t)nbe * 4;
  const size_t box_floats = 6 * (size_t)std::max(c->nf, 1);
  if ((e = ensure(c->expand_buf, sizeof(uint64_t) * mask_words + sizeof(uint32_t) * ((size_t)nbe + 8) +
                                     sizeof(float) * box_floats)) != hipSuccess)
    return e;
  ExpandArgs x;
  x.ser = so;
  x.start = start;
  x.n_series = n_series;
  x.n_cand = n_cand;
  x.n_src = c->n_src;
  x.n_tgt = c->n_tgt;
  x.n_rx = c->n_rx;
  x.K = c->K;
  x.backward = c->backward;
  x.src_pos = ptr<float>(c->src_pos);
  x.tgt_pos = ptr<float>(c->tgt_pos);
  x.ra = RefineArgs{};
  x.ra.plane = ptr<double4>(c->face_plane);
  x.ra.face_tri_off = ptr<int32_t>(c->face_tri_off);
  x.ra.face_tris = ptr<int32_t>(c->face_tris);
  x.ra.face_slots = ptr<int32_t>(c->face_slots);
  x.ra.tri4 = ptr<Leaf>(c->tri4);
  x.ra.face_material = ptr<int32_t>(c->face_material);
  x.ra.mat_pen = ptr<double>(c->mat_pen);
  x.mask = ptr<uint64_t>(c->expand_buf);
  x.block_cnt = reinterpret_cast<uint32_t*>(x.mask + mask_words);
  uint32_t* fbox = x.block_cnt + nbe + 8;
  x.face_box = fbox;
  if (c->nf > 0 && c->nt > 0) {
    hipLaunchKernelGGL(k_face_box_init, dim3((6 * c->nf + 255) / 256), dim3(256), 0, c->stream, fbox, c->nf);
    hipLaunchKernelGGL(k_face_boxes, dim3((unsigned)((c->nt + 255) / 256)), dim3(256), 0, c->stream,
                       ptr<int32_t>(c->face_tris), ptr<int32_t>(c->tri_face), ptr<int32_t>(c->face_slots),
                       ptr<Leaf>(c->tri4), c->nt, fbox);
  }
  x.capacity = 0;
  x.err = c->err_dev;
  x.out = unique_out(c);
  hipLaunchKernelGGL(k_expand, dim3(nbe), dim3(256), 0, c->stream, x, 0);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, c->stream, x.block_cnt, (int)nbe,
                     c->cnt_dev + kCntUnique);
  uint32_t n_keep = 0;
  if ((e = hipMemcpyAsync(&n_keep, c->cnt_dev + kCntUnique, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  const uint32_t capacity = (uint32_t)std::min<int64_t>(n_keep, c->cap_capacity);
  if (n_keep > capacity) fill_u32(c->cnt_dev + kCntUnique, capacity, 1, c->stream);
  c->path_cap = capacity;
  if ((e = ensure_paths(c, c->path_cap)) != hipSuccess) return e;
  x.capacity = capacity;
  x.out = unique_out(c);
  if (n_keep > 0) hipLaunchKernelGGL(k_expand, dim3(nbe), dim3(256), 0, c->stream, x, 1);
  return hipGetLastError();
}

void launch_refine(dcem_ctx* c) {
  const int64_t n = c->path_cap;
  if (n == 0) return;
  RefineArgs a;
  a.K = c->K;
  a.n_rx = c->n_rx;
  a.n_unique = c->cnt_dev + kCntUnique;
  a.tx = ptr<float>(c->backward ? c->tgt_pos : c->src_pos);
  a.rx = ptr<float>(c->backward ? c->src_pos : c->tgt_pos);
  a.plane = ptr<double4>(c->face_plane);
  a.face_tri_off = ptr<int32_t>(c->face_tri_off);
  a.face_tris = ptr<int32_t>(c->face_tris);
  a.face_slots = ptr<int32_t>(c->face_slots);
  a.face_material = ptr<int32_t>(c->face_material);
  a.materials = ptr<double>(c->materials);
  a.mat_pen = ptr<double>(c->mat_pen);
  a.nodes4 = ptr<Node4>(c->nodes4);
  a.tri4 = ptr<Leaf>(c->tri4);
  a.n4_dev = c->nt > 0 ? ptr<uint32_t>(c->tree_info) : nullptr;
  a.freqs = ptr<double>(c->freqs);
  a.n_freqs = c->n_freqs;
  a.sqrt_pt = c->sqrt_pt;
  a.atten_db_per_km = c->atten_db_per_km;
  a.pat = c->pattern_frame;
  a.n_rays = c->n_rays;
  a.valid = ptr<uint8_t>(c->path_valid);
  a.length = ptr<double>(c->path_len);
  a.tau = ptr<double>(c->path_tau);
  a.aod = ptr<double>(c->path_aod);
  a.aoa = ptr<double>(c->path_aoa);
  a.amp = ptr<double>(c->path_amp);
  a.pair = ptr<int32_t>(c->pair_range);
  a.order = ptr<uint8_t>(c->path_order);
  a.faces = ptr<int32_t>(c->path_faces);
  a.pts = ptr<double>(c->path_pts);
  a.counters = c->cnt_dev;
  a.err = c->err_dev;
  hipLaunchKernelGGL(k_refine, dim3((unsigned)n), dim3(kRefineWaves * kWave), 0, c->stream, a);
}

void launch_power_grad(dcem_ctx* c, uint32_t n_unique, double* g_eps, double* g_sig, double* g_pat) {
  const int n_pairs = c->n_tx * c->n_rx;
  hipLaunchKernelGGL(k_power_grad, dim3((n_pairs * 64 + 255) / 256), dim3(256), 0, c->stream,
                     ptr<int32_t>(c->pair_range), ptr<uint8_t>(c->path_valid), ptr<double>(c->path_amp),
                     ptr<double>(c->path_pts), ptr<uint8_t>(c->path_order), ptr<int32_t>(c->path_faces),
                     ptr<double>(c->path_len), n_unique, c->K, n_pairs, ptr<double>(c->freqs),
                     c->n_freqs, ptr<int32_t>(c->face_material), ptr<double>(c->materials), ptr<double>(c->mat_pen),
                     c->nm, c->sqrt_pt,
                     c->atten_db_per_km, c->pattern_frame, g_eps, g_sig, g_pat);
}

void launch_reduce(dcem_ctx* c) {
  const int n_pairs = c->n_tx * c->n_rx;
  hipLaunchKernelGGL(k_reduce, dim3((n_pairs * 64 + 255) / 256), dim3(256), 0, c->stream,
                     ptr<int32_t>(c->pair_range), ptr<uint8_t>(c->path_valid), ptr<double>(c->path_amp),
                     c->cnt_dev + kCntUnique, n_pairs, c->n_freqs, c->pcoh_dev,
                     c->pinc_dev, c->cnt_dev);
}

}  // namespace dcem
