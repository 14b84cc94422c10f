// Stable LSD radix sort of multi-word keys into a permutation.
//
// Each 8-bit pass has three kernels: per-tile digit histograms, an exclusive
// scan in (digit, tile) order, and a stable scatter.  Inside a tile, items are
// ranked 256 at a time with wavefront ballots: the lanes holding the same digit
// are found by intersecting one ballot per digit bit, and a lane's rank is the
// number of such peers below it.  Keys are read through the source
// permutation; only the permutation moves.
#include "dcem_internal.h"

namespace dcem {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 8;
constexpr int kTile = kThreads * kRounds;
constexpr int kWaves = kThreads / kWave;
constexpr int kSmallScan = 1 << 14;   // histogram entries the one-block scan takes alone

__device__ inline uint32_t digit_of(const uint32_t* __restrict__ keys, int64_t stride, int word, int shift,
                                    uint32_t idx) {
  return (keys[word * stride + idx] >> shift) & 0xffu;
}

__global__ __launch_bounds__(kThreads) void k_hist(const uint32_t* __restrict__ keys, int64_t stride, int word,
                                                   int shift, const uint32_t* __restrict__ src,
                                                   const uint32_t* __restrict__ n_dev, uint32_t n_max,
                                                   uint32_t* __restrict__ hist, int n_tiles) {
  __shared__ uint32_t cnt[256];
  const uint32_t n = min(*n_dev, n_max);
  const int tile = blockIdx.x;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)tile * kTile;
  if (base < n) {
    for (int r = 0; r < kRounds; ++r) {
      int64_t i = base + r * kThreads + threadIdx.x;
      if (i < n) {
        uint32_t idx = src ? src[i] : (uint32_t)i;
        atomicAdd(&cnt[digit_of(keys, stride, word, shift, idx)], 1u);
      }
    }
  }
  __syncthreads();
  hist[threadIdx.x * n_tiles + tile] = cnt[threadIdx.x];
}

// Exclusive scan of hist[256 * n_tiles] in place (single block).
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ hist, int total) {
  __shared__ uint32_t part[1024];
  const int per = (total + 1023) / 1024;
  const int b = threadIdx.x * per;
  const int e = min(total, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += hist[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int i = b; i < e; ++i) {
    uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
}

// Larger histograms: a three-kernel scan.  Block g owns the contiguous
// segment [g * seg, (g + 1) * seg) of hist: k_scan_sums reduces it into
// sums[g], k_scan (one block) scans the sums, and k_scan_down scans the
// segment again, 256 coalesced entries at a time, from its block's offset.
constexpr int kScanBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_scan_sums(const uint32_t* __restrict__ hist, int total, int seg,
                                                       uint32_t* __restrict__ sums) {
  __shared__ uint32_t ws[kWaves];
  const int b = blockIdx.x * seg, e = min(total, b + seg);
  uint32_t s = 0;
  for (int i = b + (int)threadIdx.x; i < e; i += kThreads) s += hist[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_down(uint32_t* __restrict__ hist, int total, int seg,
                                                       const uint32_t* __restrict__ offs) {
  __shared__ uint32_t ws[kWaves];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int b = blockIdx.x * seg, e = min(total, b + seg);
  uint32_t run = offs[blockIdx.x];
  for (int c = b; c < e; c += kThreads) {
    const int i = c + (int)threadIdx.x;
    const uint32_t v = i < e ? hist[i] : 0u;
    uint32_t incl = v;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) ws[wave] = incl;
    __syncthreads();
    uint32_t before = run;
    for (int w = 0; w < wave; ++w) before += ws[w];
    uint32_t chunk = 0;
    for (int w = 0; w < kWaves; ++w) chunk += ws[w];
    if (i < e) hist[i] = before + incl - v;
    run += chunk;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_scatter(const uint32_t* __restrict__ keys, int64_t stride, int word,
                                                      int shift, const uint32_t* __restrict__ src,
                                                      uint32_t* __restrict__ dst, const uint32_t* __restrict__ n_dev,
                                                      uint32_t n_max, const uint32_t* __restrict__ hist, int n_tiles) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const uint32_t n = min(*n_dev, n_max);
  const int tile = blockIdx.x;
  const int64_t base = (int64_t)tile * kTile;
  if (base >= n) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  running[threadIdx.x] = hist[threadIdx.x * n_tiles + tile];
  for (int r = 0; r < kRounds; ++r) {
    for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = base + r * kThreads + threadIdx.x;
    const bool valid = i < n;
    uint32_t idx = 0, d = 0;
    if (valid) {
      idx = src ? src[i] : (uint32_t)i;
      d = digit_of(keys, stride, word, shift, idx);
    }
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint64_t below = peers & ((1ull << lane) - 1ull);
    const uint32_t rank = (uint32_t)__popcll(below);
    if (valid && below == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      dst[pos] = idx;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][threadIdx.x];
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

hipError_t prepare_sort(dcem_ctx* c, int64_t n_max) {
  const int64_t n_tiles = std::max<int64_t>((n_max + kTile - 1) / kTile, 1);
  return ensure(c->sort_hist, sizeof(uint32_t) * (256 * (size_t)n_tiles + kScanBlocks));
}

hipError_t radix_sort_perm(dcem_ctx* c, const uint32_t* keys, int W, int bits, const uint32_t* n_dev,
                           int64_t n_max, uint32_t* perm, uint32_t* perm_tmp, hipStream_t s, int64_t stride,
                           int low_bits) {
  if (n_max <= 0) return hipSuccess;
  if (stride < 0) stride = n_max;
  const int n_tiles = (int)((n_max + kTile - 1) / kTile);
  const int total = 256 * n_tiles;
  // histograms of more entries than the one-block scan handles quickly are
  // scanned by kScanBlocks blocks (their sums after the histogram)
  const int seg = (total + kScanBlocks - 1) / kScanBlocks;
  hipError_t e = ensure(c->sort_hist, sizeof(uint32_t) * ((size_t)total + kScanBlocks));
  if (e != hipSuccess) return e;
  uint32_t* hist = ptr<uint32_t>(c->sort_hist);
  uint32_t* sums = hist + total;
  // digit passes from the least significant bit, without the digits of word
  // W-1 above low_bits (zero in every key)
  auto used = [&](int b) { return b >= 32 || b < low_bits; };
  int passes = 0;
  for (int b = 0; b < bits; b += 8) passes += used(b) ? 1 : 0;
  const uint32_t* src = nullptr;
  for (int b = 0, p = 0; b < bits; b += 8) {
    if (!used(b)) continue;
    const int word = W - 1 - b / 32;
    const int shift = b % 32;
    uint32_t* dst = ((passes - 1 - p) % 2 == 0) ? perm : perm_tmp;
    ++p;
    hipLaunchKernelGGL(k_hist, dim3(n_tiles), dim3(kThreads), 0, s, keys, stride, word, shift, src, n_dev,
                       (uint32_t)n_max, hist, n_tiles);
    if (total <= kSmallScan) {
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, hist, total);
    } else {
      hipLaunchKernelGGL(k_scan_sums, dim3(kScanBlocks), dim3(kThreads), 0, s, hist, total, seg, sums);
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, sums, kScanBlocks);
      hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(kThreads), 0, s, hist, total, seg, sums);
    }
    hipLaunchKernelGGL(k_scatter, dim3(n_tiles), dim3(kThreads), 0, s, keys, stride, word, shift, src, dst, n_dev,
                       (uint32_t)n_max, hist, n_tiles);
    src = dst;
  }
  return hipGetLastError();
}

}  // namespace dcem
