// Host side of the C ABI: argument checks, device buffers, call order and the
// per-frame schedule of kernels on the context's stream.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>

#include "dcem_internal.h"

using namespace dcem;

namespace dcem {

namespace {

hipError_t dev_free(const Allocator* al, void* p, size_t bytes) {
  if (al->user) {
    al->fn.free(p, bytes, al->stream, al->fn.user);
    return hipSuccess;
  }
  return hipFree(p);
}

}  // namespace

namespace {
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
}  // namespace

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, v, n);
}

hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return hipSuccess;
  if (!b.al) return hipErrorInvalidValue;   // a buffer outside dcem_ctx::buffers()
  if (b.p) {
    hipError_t e = dev_free(b.al, b.p, b.bytes);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  if (b.al->user) {
    b.p = b.al->fn.alloc(want, b.al->stream, b.al->fn.user);
    if (!b.p) return hipErrorOutOfMemory;
  } else {
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      b.p = nullptr;
      return e;
    }
  }
  b.bytes = want;
  return hipSuccess;
}

void release(DevBuf& b) {
  if (b.p && b.al) (void)dev_free(b.al, b.p, b.bytes);
  b.p = nullptr;
  b.bytes = 0;
}

}  // namespace dcem

namespace {

// Device workspace of dcem_power_gradients_noalloc: a fixed array that every
// GPU the library runs on holds once (a module variable: one copy per device,
// at its own address).  Host code never uses its name as an address: the
// pointer comes from hipGetSymbolAddress, looked up once per device with that
// device current, and is passed to the kernels like any buffer.
__device__ __align__(256) double scratch[DCEM_NOALLOC_GRAD_DOUBLES];
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// This device's array (the device must be current).
hipError_t scratch_of(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

dcem_status fail(dcem_ctx* c, dcem_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
dcem_status fail(dcem_ctx* c, dcem_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

dcem_status hip_fail(dcem_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? DCEM_E_OUT_OF_MEMORY : DCEM_E_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(c, e_, what); \
  } while (0)

// Copy n elements of T from caller memory (host or device) into a host vector.
template <class T>
hipError_t fetch(std::vector<T>& out, const T* src, size_t n, int mem_kind, hipStream_t s) {
  out.resize(n);
  if (n == 0) return hipSuccess;
  if (mem_kind == DCEM_MEM_DEVICE) {
    hipError_t e = hipMemcpyAsync(out.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  std::memcpy(out.data(), src, n * sizeof(T));
  return hipSuccess;
}

template <class T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  hipError_t e = ensure(b, std::max<size_t>(v.size() * sizeof(T), 16));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

bool mem_kind_ok(int k) { return k == DCEM_MEM_HOST || k == DCEM_MEM_DEVICE; }

// Binary tree over the capture spheres (median split on the longest axis of the
// centres), in the scene BVH's node layout; leaves are receiver ids and every
// box is the sphere box grown by `grow`, so the box test is conservative.
struct RxTree {
  std::vector<Node> nodes;
  const std::vector<float>* rx;
  float r;

  void box_of(const std::vector<int>& ids, int b, int e, float* lo, float* hi) const {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int i = b; i < e; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], (*rx)[3 * ids[i] + a] - r);
        hi[a] = std::max(hi[a], (*rx)[3 * ids[i] + a] + r);
      }
  }
  static void set_slot(Node& n, int slot, const float* lo, const float* hi) {
    float* f = reinterpret_cast<float*>(&n);
    for (int a = 0; a < 3; ++a) { f[6 * slot + a] = lo[a]; f[6 * slot + 3 + a] = hi[a]; }
  }
  int build(std::vector<int>& ids, int b, int e) {
    if (e - b == 1) return ~ids[b];
    const int me = (int)nodes.size();
    nodes.push_back(Node{});
    float lo[3], hi[3];
    box_of(ids, b, e, lo, hi);
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    const int mid = (b + e) / 2;
    std::nth_element(ids.begin() + b, ids.begin() + mid, ids.begin() + e, [&](int x, int y) {
      const float px = (*rx)[3 * x + ax], py = (*rx)[3 * y + ax];
      return px < py || (px == py && x < y);
    });
    const int l = build(ids, b, mid), rr = build(ids, mid, e);
    float llo[3], lhi[3], rlo[3], rhi[3];
    box_of(ids, b, mid, llo, lhi);
    box_of(ids, mid, e, rlo, rhi);
    set_slot(nodes[me], 0, llo, lhi);
    set_slot(nodes[me], 1, rlo, rhi);
    nodes[me].c = make_int4(l, rr, -1, 0);
    return me;
  }
};

// Receivers counting-sorted into kRxCols columns of equal x width (stable in
// receiver index), for the capture test of the group re-trace: a segment
// scans only the columns its xy extent covers.  The device evaluates the same
// column formula in the same FP32 operations.
hipError_t upload_rx_columns(dcem_ctx* c, const std::vector<float>& rx) {
  const int n = (int)(rx.size() / 3);
  float x0 = INFINITY, x1 = -INFINITY;
  for (int i = 0; i < n; ++i) {
    x0 = std::min(x0, rx[3 * i]);
    x1 = std::max(x1, rx[3 * i]);
  }
  const float scale = x1 > x0 ? (float)kRxCols / (x1 - x0) : 0.0f;
  auto col = [&](float x) {
    const float v = std::floor((x - x0) * scale);
    return (int)std::min(std::max(v, 0.0f), (float)(kRxCols - 1));
  };
  std::vector<int32_t> start(kRxCols + 1, 0);
  for (int i = 0; i < n; ++i) ++start[col(rx[3 * i]) + 1];
  for (int k = 0; k < kRxCols; ++k) start[k + 1] += start[k];
  std::vector<float> rec(4 * (size_t)n + (kRxCols + 1));
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  for (int i = 0; i < n; ++i) {
    const int at = fill[col(rx[3 * i])]++;
    rec[4 * at] = rx[3 * i];
    rec[4 * at + 1] = rx[3 * i + 1];
    rec[4 * at + 2] = rx[3 * i + 2];
    std::memcpy(&rec[4 * at + 3], &i, 4);
  }
  std::memcpy(&rec[4 * (size_t)n], start.data(), sizeof(int32_t) * (kRxCols + 1));
  c->rx_col_x0 = x0;
  c->rx_col_scale = scale;
  return upload(c->rx_cols, rec, c->stream);
}

std::vector<Node> build_rx_tree(const std::vector<float>& rx, float radius) {
  RxTree t;
  t.rx = &rx;
  double R = 1.0;
  for (float v : rx) R = std::max(R, (double)std::fabs(v));
  t.r = (float)(radius * (1.0 + 1e-5) + 1e-3 + 4e-6 * (2.0 * R + 1.0));
  const int n = (int)(rx.size() / 3);
  std::vector<int> ids(n);
  for (int i = 0; i < n; ++i) ids[i] = i;
  if (n == 1) {
    Node root{};
    float lo[3], hi[3];
    t.box_of(ids, 0, 1, lo, hi);
    RxTree::set_slot(root, 0, lo, hi);
    RxTree::set_slot(root, 1, lo, hi);
    root.c = make_int4(~0, ~0, -1, 0);
    return {root};
  }
  t.build(ids, 0, n);
  return t.nodes;
}

void ev_record(dcem_ctx* c, int i) {
  if (c->timing) (void)hipEventRecord(c->ev[i], c->stream);
}

// Enqueue a pending refit by itself (before anything that reads the tree or
// the vertices, or when no revalidation pass can take it along).
hipError_t flush_refit(dcem_ctx* c) {
  if (!c->refit_pending) return hipSuccess;
  c->refit_pending = false;
  ev_record(c, 6);
  launch_refit(c, true, c->sah_dev + 1);
  ev_record(c, 7);
  return hipGetLastError();
}

float ev_ms(dcem_ctx* c, int a, int b) {
  float ms = 0.f;
  if (c->timing && hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) == hipSuccess) return ms;
  return 0.f;
}

// Frame block layout (bytes): counters [0, 128), error word [128, 256),
// SAH values [256, 512), p_coh and p_inc from 512.
constexpr size_t kBlockHead = 512;

hipError_t ensure_frame_block(dcem_ctx* c, int64_t n_pow) {
  n_pow = std::max<int64_t>(n_pow, 1);
  if (n_pow <= c->n_pow_cap && c->frame_block.p) return hipSuccess;
  hipError_t je = flush_refit(c);   // a pending refit writes its SAH value here
  if (je != hipSuccess) return je;
  const size_t bytes = kBlockHead + 2 * sizeof(double) * (size_t)n_pow;
  c->list_clear = false;   // the new block's counters start undefined
  // a revalidation enqueued ahead left its list count and the frame's start
  // in the old block: the frame starts over in the new one (which the
  // allocator may well place at the old address)
  c->revalidated_ahead = false;
  // keep the head (SAH values of the current tree) across a reallocation
  double sah_keep[3] = {1.0, 1.0, 1.0};
  const bool had = c->frame_block.p != nullptr;
  hipError_t e;
  if (had) {
    if ((e = hipMemcpyAsync(sah_keep, c->sah_dev, sizeof sah_keep, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
  }
  e = ensure(c->frame_block, bytes);
  if (e != hipSuccess) return e;
  if (c->host_block) (void)hipHostFree(c->host_block);
  c->host_block = nullptr;
  if ((e = hipHostMalloc(&c->host_block, c->frame_block.bytes, hipHostMallocDefault)) != hipSuccess) return e;
  c->host_block_bytes = c->frame_block.bytes;
  char* b = ptr<char>(c->frame_block);
  c->cnt_dev = reinterpret_cast<uint32_t*>(b);
  c->err_dev = reinterpret_cast<uint32_t*>(b + 128);
  c->sah_dev = reinterpret_cast<double*>(b + 256);
  c->pcoh_dev = reinterpret_cast<double*>(b + kBlockHead);
  c->pinc_dev = c->pcoh_dev + n_pow;
  c->n_pow_cap = n_pow;
  fill_u32(reinterpret_cast<uint32_t*>(b), 0u, c->frame_block.bytes / 4, c->stream);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipMemcpyAsync(c->sah_dev, sah_keep, sizeof sah_keep, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

dcem_status finish_candidates(dcem_ctx* c);

// Begin the next frame and enqueue its revalidation with the pending refit,
// once nothing of the last frame remains to be read back (see frame_begun).
// While the last frame's results are still on their way, the launches go
// ahead at once, each guarded on the device by that frame's fallback flag:
// a frame whose candidates must be redone (on the tree it was traced with)
// turns them into no-ops, and sync_frame restores the host state.  (Not with
// stage timings on: the events would be recorded over before they are read.)
void go_ahead(dcem_ctx* c) {
  if (!c->refit_pending || c->revalidated_ahead || !c->has_frame || !c->cache_valid) return;
  const bool early = !c->counts_current;
  if (early && (!c->copy_pending || c->timing)) return;
  const uint32_t* skip = early ? c->cnt_dev + kCntFallback : nullptr;
  if (early && !c->early_ahead) {
    c->early_ahead = true;
    c->early_caps = c->cur_caps;
    c->early_begun = c->frame_begun;
    c->early_list_clear = c->list_clear;
  }
  if (!c->frame_begun) {
    c->cur_caps ^= 1;
    c->frame_begun = true;
  }
  // the last frame's reduction zeroed the list counter: the revalidation's
  // launch also starts the frame (one launch instead of two), unless an
  // earlier early start of this frame appended to it
  const bool fresh = c->list_clear;
  ev_record(c, 0);
  if (!fresh) launch_frame_begin(c, c->last_los, skip);
  c->refit_pending = false;
  ev_record(c, 6);
  launch_refit_coherence(c, fresh, skip);
  c->list_clear = false;
  ev_record(c, 7);
  ev_record(c, 1);
  c->revalidated_ahead = true;
}

size_t frame_block_bytes(const dcem_ctx* c) {
  return kBlockHead + 2 * sizeof(double) * (size_t)std::max<int64_t>(c->n_pow_cap, 1);
}

// Wait for the stream and read the frame block in one transfer: counters,
// device error word, SAH values and powers.  Redoes a frame's candidates when
// the small de-duplication path overflowed.  Reports device errors.
dcem_status sync_frame(dcem_ctx* c) {
  if (c->copy_pending) {
    // the frame's own copy, enqueued right behind its last kernel: later work
    // on the stream (the next frame's transforms and refit) is not waited for
    c->copy_pending = false;
    HIP_TRY(hipEventSynchronize(c->ev_copy), "synchronize");
  } else if (c->frame_begun) {
    // the next frame has begun on the device: host_block keeps the last one
  } else {
    HIP_TRY(flush_refit(c), "refit");   // a pending refit writes its SAH value into the block
    HIP_TRY(hipMemcpyAsync(c->host_block, c->frame_block.p, frame_block_bytes(c), hipMemcpyDeviceToHost, c->stream),
            "read results");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  }
  const char* hb = static_cast<const char*>(c->host_block);
  if (c->has_frame && !c->frame_begun && c->timing) {
    // the frame's stage events have all completed: its revalidation (0..1,
    // begun early or not), re-trace (8..2), candidates, refinement, reduction
    dcem_frame_stats& s = c->stats;
    if (c->refit_pending_timing) {
      s.ms_refit = ev_ms(c, 6, 7);
      c->refit_pending_timing = false;
    }
    s.ms_coherence = ev_ms(c, 0, 1);
    s.ms_trace = ev_ms(c, 8, 2);
    s.ms_candidates = ev_ms(c, 2, 3);
    s.ms_refine = ev_ms(c, 3, 4);
    s.ms_reduce = ev_ms(c, 4, 5);
  }
  std::memcpy(c->last_cnt, hb, sizeof(uint32_t) * kCntSlots);
  uint32_t err = 0;
  std::memcpy(&err, hb + 128, 4);
  double sah[3];
  std::memcpy(sah, hb + 256, sizeof sah);
  if (c->refit_since_build && sah[0] > 0) c->pending_ratio = sah[1] / sah[0];
  c->subtree_ratio = sah[2] > 0 ? sah[0] / sah[2] : 1.0;
  c->sah_last = c->pending_ratio;
  if (c->has_frame) {
    c->n_caps_host = std::min<int64_t>(c->last_cnt[kCntCaptures], c->cap_capacity);
    c->counts_current = true;
    if (c->early_ahead) {
      c->early_ahead = false;
      if (c->last_cnt[kCntFallback]) {
        // the launches that went ahead did nothing: the refit is pending again
        c->cur_caps = c->early_caps;
        c->frame_begun = c->early_begun;
        c->list_clear = c->early_list_clear;
        c->revalidated_ahead = false;
        c->refit_pending = true;
      } else if (err) {
        // they ran, but an error they raised would be cleared with this
        // frame's: the next frame starts over from its lists
        c->revalidated_ahead = false;
      }
    }
    if (c->last_cnt[kCntFallback] && !err) {
      // more captures than the small path holds: redo the candidates exactly
      const uint32_t zero = 0;
      HIP_TRY(hipMemcpyAsync(c->cnt_dev + kCntFallback, &zero, 4, hipMemcpyHostToDevice, c->stream), "reset");
      dcem_status st = finish_candidates(c);
      if (st != DCEM_OK) return st;
      return sync_frame(c);
    }
  }
  if (err) {
    fill_u32(c->err_dev, 0u, 1, c->stream);
    HIP_TRY(hipGetLastError(), "clear error word");
    if (err & DCEM_ERR_NONFINITE) return fail(c, DCEM_E_INVALID_ARG, "non-finite vertex after a transform");
    return fail(c, DCEM_E_CAPACITY, "device capacity exceeded (%s%s)",
                (err & DCEM_ERR_STACK) ? "traversal stack " : "", (err & DCEM_ERR_CAPTURES) ? "capture buffer" : "");
  }
  return DCEM_OK;
}

dcem_status check_device_error(dcem_ctx* c) { return sync_frame(c); }

// Candidates (exact count), refinement and accumulation of the current frame.
dcem_status finish_candidates(dcem_ctx* c) {
  HIP_TRY(build_candidates(c, false), "candidates");
  HIP_TRY(ensure_paths(c, c->path_cap), "alloc paths");
  launch_refine(c);
  launch_reduce(c);
  HIP_TRY(hipGetLastError(), "refine kernels");
  return DCEM_OK;
}

}  // namespace

extern "C" {

dcem_status dcem_create(dcem_ctx** out, int32_t device, void* hip_stream, const dcem_allocator* allocator) {
  if (!out) return DCEM_E_INVALID_ARG;
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) return DCEM_E_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DCEM_E_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return DCEM_E_DEVICE;
  dcem_ctx* c = new dcem_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->alloc.stream = c->stream;
  if (allocator) {
    c->alloc.fn = *allocator;
    c->alloc.user = true;
  }
  for (DevBuf* b : c->buffers()) b->al = &c->alloc;
  // the no-allocation gradient call's workspace on this device (null if the
  // lookup fails: that call then reports DCEM_E_DEVICE, nothing else needs it)
  if (scratch_of(device, &c->scratch) != hipSuccess) {
    c->scratch = nullptr;
    (void)hipGetLastError();
  }
  if (ensure_frame_block(c, 1) != hipSuccess) {
    release(c->frame_block);
    if (c->host_block) (void)hipHostFree(c->host_block);
    delete c;
    return DCEM_E_OUT_OF_MEMORY;
  }
  for (auto& e : c->ev) (void)hipEventCreate(&e);
  if (hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming) != hipSuccess) {
    dcem_destroy(c);
    return DCEM_E_DEVICE;
  }
  *out = c;
  return DCEM_OK;
}

void dcem_destroy(dcem_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : c->buffers()) release(*b);
  if (c->host_block) (void)hipHostFree(c->host_block);
  if (c->grad_host) (void)hipHostFree(c->grad_host);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->ev_copy) (void)hipEventDestroy(c->ev_copy);
  delete c;
}

const char* dcem_last_error(const dcem_ctx* c) { return c ? c->err.c_str() : "null context"; }

dcem_status dcem_set_capture_capacity(dcem_ctx* c, int64_t max_captures) {
  if (!c) return DCEM_E_INVALID_ARG;
  if (max_captures < 1 || max_captures > (int64_t(1) << 31))
    return fail(c, DCEM_E_INVALID_ARG, "capture capacity must be in [1, 2^31]");
  c->cap_capacity = max_captures;
  c->cache_valid = false;
  return DCEM_OK;
}

dcem_status dcem_set_stack_limit(dcem_ctx* c, int32_t entries) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (entries < 0) return fail(c, DCEM_E_INVALID_ARG, "stack limit must be >= 0");
  c->stack_limit = entries;
  return DCEM_OK;
}

dcem_status dcem_set_timing(dcem_ctx* c, int32_t enabled) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->timing = enabled != 0;
  return DCEM_OK;
}

// Material rows (eps_r, sigma, const_gamma): DCEM_E_INVALID_ARG for the first bad one.
dcem_status check_materials(dcem_ctx* c, const double* M, int32_t n) {
  for (int32_t m = 0; m < n; ++m) {
    const double er = M[3 * m], sg = M[3 * m + 1], g = M[3 * m + 2];
    if (!std::isfinite(er) || !std::isfinite(sg) || er < 1.0 || sg < 0.0 || (!std::isnan(g) && !(g >= 0.0 && g <= 1.0)))
      return fail(c, DCEM_E_INVALID_ARG, "material %d: need eps_r >= 1, sigma >= 0, const_gamma in [0,1] or NaN", m);
  }
  return DCEM_OK;
}

dcem_status dcem_scene_upload(dcem_ctx* c, const dcem_scene_desc* s) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!s) return fail(c, DCEM_E_INVALID_ARG, "null scene");
  if (!mem_kind_ok(s->mem_kind)) return fail(c, DCEM_E_INVALID_ARG, "bad mem_kind");
  if (s->n_vertices < 0 || s->n_tris < 0 || s->n_faces < 0 || s->n_materials < 0 || s->n_objects < 0)
    return fail(c, DCEM_E_INVALID_ARG, "negative size");
  if (s->n_tris >= (int64_t(1) << 27) || s->n_vertices >= (int64_t(1) << 31))
    return fail(c, DCEM_E_UNSUPPORTED, "at most 2^27 - 1 triangles and 2^31 - 1 vertices");
  if (s->n_faces >= (1 << 20)) return fail(c, DCEM_E_UNSUPPORTED, "at most 2^20 - 1 faces");
  if (s->n_objects >= (1 << 16)) return fail(c, DCEM_E_UNSUPPORTED, "at most 2^16 - 1 objects");
  if (s->n_tris > 0 && s->n_faces == 0) return fail(c, DCEM_E_INVALID_ARG, "triangles without faces");
  if (s->n_faces > 0 && s->n_materials == 0) return fail(c, DCEM_E_INVALID_ARG, "faces without materials");
  if ((s->n_vertices && !s->vertices) || (s->n_tris && (!s->tris || !s->tri_face)) ||
      (s->n_faces && (!s->face_material || !s->face_object)) || (s->n_materials && !s->materials) ||
      (s->n_objects && !s->object_vertex_range))
    return fail(c, DCEM_E_INVALID_ARG, "null array with nonzero size");
  HIP_TRY(hipSetDevice(c->device), "set device");
  c->refit_pending = false;   // the new scene is built from scratch
  c->frame_begun = false;
  c->revalidated_ahead = false;
  c->early_ahead = false;
  std::vector<float> V;
  std::vector<int32_t> T, TF, FM, FO;
  std::vector<double> M;
  std::vector<int64_t> OR;
  HIP_TRY(fetch(V, s->vertices, 3 * (size_t)s->n_vertices, s->mem_kind, c->stream), "read vertices");
  HIP_TRY(fetch(T, s->tris, 3 * (size_t)s->n_tris, s->mem_kind, c->stream), "read tris");
  HIP_TRY(fetch(TF, s->tri_face, (size_t)s->n_tris, s->mem_kind, c->stream), "read tri_face");
  HIP_TRY(fetch(FM, s->face_material, (size_t)s->n_faces, s->mem_kind, c->stream), "read face_material");
  HIP_TRY(fetch(FO, s->face_object, (size_t)s->n_faces, s->mem_kind, c->stream), "read face_object");
  HIP_TRY(fetch(M, s->materials, 3 * (size_t)s->n_materials, s->mem_kind, c->stream), "read materials");
  HIP_TRY(fetch(OR, s->object_vertex_range, 2 * (size_t)s->n_objects, s->mem_kind, c->stream), "read objects");
  double R = 0.0;
  for (size_t i = 0; i < V.size(); ++i) {
    if (!std::isfinite(V[i])) return fail(c, DCEM_E_INVALID_ARG, "non-finite vertex coordinate %zu", i / 3);
    R = std::max(R, (double)std::fabs(V[i]));
  }
  for (size_t i = 0; i < T.size(); ++i)
    if (T[i] < 0 || T[i] >= s->n_vertices) return fail(c, DCEM_E_INVALID_ARG, "triangle %zu: vertex index out of range", i / 3);
  for (size_t i = 0; i < TF.size(); ++i)
    if (TF[i] < 0 || TF[i] >= s->n_faces) return fail(c, DCEM_E_INVALID_ARG, "triangle %zu: face out of range", i);
  for (int32_t f = 0; f < s->n_faces; ++f) {
    if (FM[f] < 0 || FM[f] >= s->n_materials) return fail(c, DCEM_E_INVALID_ARG, "face %d: material out of range", f);
    if (FO[f] < -1 || FO[f] >= s->n_objects) return fail(c, DCEM_E_INVALID_ARG, "face %d: object out of range", f);
  }
  {
    const dcem_status ms = check_materials(c, M.data(), s->n_materials);
    if (ms != DCEM_OK) return ms;
  }
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int32_t o = 0; o < s->n_objects; ++o) {
    const int64_t b = OR[2 * o], e = OR[2 * o + 1];
    if (b < 0 || e < b || e > s->n_vertices) return fail(c, DCEM_E_INVALID_ARG, "object %d: bad vertex range", o);
    ranges.push_back({b, e});
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) return fail(c, DCEM_E_INVALID_ARG, "object vertex ranges overlap");
  // faces: triangle lists (CSR) and the largest triangle (plane reference)
  const int nf = s->n_faces;
  std::vector<int32_t> off(nf + 1, 0), ftris(T.size() / 3), ref(nf, -1);
  std::vector<double> best(nf, -1.0);
  for (size_t t = 0; t < TF.size(); ++t) off[TF[t] + 1]++;
  for (int f = 0; f < nf; ++f) off[f + 1] += off[f];
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (size_t t = 0; t < TF.size(); ++t) {
      const int f = TF[t];
      ftris[fill[f]++] = (int32_t)t;
      const float* a = &V[3 * T[3 * t]];
      const float* b = &V[3 * T[3 * t + 1]];
      const float* cc = &V[3 * T[3 * t + 2]];
      const double ux = b[0] - (double)a[0], uy = b[1] - (double)a[1], uz = b[2] - (double)a[2];
      const double vx = cc[0] - (double)a[0], vy = cc[1] - (double)a[1], vz = cc[2] - (double)a[2];
      const double nx = uy * vz - uz * vy, ny = uz * vx - ux * vz, nz = ux * vy - uy * vx;
      const double ar = std::sqrt(nx * nx + ny * ny + nz * nz);
      if (ar > best[f]) {
        best[f] = ar;
        ref[f] = (int32_t)t;
      }
    }
  }
  for (int f = 0; f < nf; ++f) {
    if (ref[f] < 0) return fail(c, DCEM_E_INVALID_ARG, "face %d has no triangle", f);
    if (!(best[f] > 0.0)) return fail(c, DCEM_E_INVALID_ARG, "face %d has only degenerate triangles", f);
  }
  c->nv = s->n_vertices;
  c->nt = s->n_tris;
  c->nf = nf;
  c->nm = s->n_materials;
  c->mat_pending = false;
  // every material opaque until dcem_set_penetration_loss says otherwise
  c->pen_next.assign((size_t)s->n_materials, std::numeric_limits<double>::infinity());
  c->pen_pending = true;
  c->h_face_material = FM;
  c->no = s->n_objects;
  c->pad = (float)(4e-6 * (2.0 * R + 1.0));
  c->h_face_object = FO;
  {
    // faces per group (the static geometry, each moving object): the sort
    // keys of the build hold a face's rank within its group
    std::vector<int32_t> per((size_t)c->no + 1, 0);
    for (int32_t o : FO) ++per[(size_t)(o + 1)];
    int32_t most = 1;
    for (int32_t v : per) most = std::max(most, v);
    c->face_bits = 0;
    while ((int64_t(1) << c->face_bits) < most) ++c->face_bits;
  }
  HIP_TRY(upload(c->ref_vertices, V, c->stream), "upload vertices");
  HIP_TRY(upload(c->vertices, V, c->stream), "upload vertices");
  HIP_TRY(upload(c->tris, T, c->stream), "upload tris");
  HIP_TRY(upload(c->tri_face, TF, c->stream), "upload tri_face");
  HIP_TRY(upload(c->face_material, FM, c->stream), "upload face_material");
  HIP_TRY(upload(c->face_object, FO, c->stream), "upload face_object");
  HIP_TRY(upload(c->materials, M, c->stream), "upload materials");
  HIP_TRY(upload(c->obj_range, OR, c->stream), "upload objects");
  HIP_TRY(upload(c->face_tri_off, off, c->stream), "upload faces");
  HIP_TRY(upload(c->face_tris, ftris, c->stream), "upload faces");
  HIP_TRY(upload(c->face_ref_tri, ref, c->stream), "upload faces");
  HIP_TRY(ensure(c->face_plane, sizeof(double) * 4 * std::max(nf, 1)), "alloc planes");
  std::vector<float> ident(12 * (size_t)c->no, 0.f);
  for (int o = 0; o < c->no; ++o) ident[12 * o] = ident[12 * o + 5] = ident[12 * o + 10] = 1.f;
  HIP_TRY(upload(c->xf, ident, c->stream), "upload transforms");
  HIP_TRY(ensure(c->obj_box, sizeof(float) * 6 * std::max(c->no, 1)), "alloc object boxes");
  launch_xform(c, ptr<float>(c->xf));
  HIP_TRY(hipGetLastError(), "transform kernel");
  HIP_TRY(build_lbvh(c, true), "build BVH");
  c->has_scene = true;
  c->cache_valid = false;
  c->has_frame = false;
  c->bvh_stale = false;
  c->sah_last = 1.0;
  c->last_rebuilt = 1;
  return check_device_error(c);
}

dcem_status dcem_set_object_transforms(dcem_ctx* c, const float* xf, int32_t n_objects, int32_t mem_kind) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  if (n_objects != c->no) return fail(c, DCEM_E_INVALID_ARG, "scene has %d objects, got %d", c->no, n_objects);
  if (!mem_kind_ok(mem_kind)) return fail(c, DCEM_E_INVALID_ARG, "bad mem_kind");
  if (n_objects == 0) return DCEM_OK;
  if (!xf) return fail(c, DCEM_E_INVALID_ARG, "null transforms");
  c->revalidated_ahead = false;   // it saw the old object boxes (the frame stays begun)
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (c->refit_pending && c->copy_pending) {
    // the pending refit is about to change the tree an unread frame may still
    // need (see dcem_refit_bvh): finish that frame first
    const dcem_status st = sync_frame(c);
    if (st != DCEM_OK) return st;
  }
  HIP_TRY(flush_refit(c), "refit");
  if (mem_kind == DCEM_MEM_HOST) {
    for (int i = 0; i < 12 * n_objects; ++i)
      if (!std::isfinite(xf[i])) return fail(c, DCEM_E_INVALID_ARG, "non-finite transform entry %d", i);
    HIP_TRY(hipMemcpyAsync(c->xf.p, xf, sizeof(float) * 12 * n_objects, hipMemcpyHostToDevice, c->stream), "copy xf");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    launch_xform(c, ptr<float>(c->xf));
  } else {
    launch_xform(c, xf);   // read in place: device inputs stay valid until the stream reaches the kernel
  }
  HIP_TRY(hipGetLastError(), "transform kernel");
  c->bvh_stale = true;
  return DCEM_OK;
}

dcem_status dcem_refit_bvh(dcem_ctx* c, int32_t flags, double threshold, int32_t* rebuilt, double* sah_ratio) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  if (std::isnan(threshold)) return fail(c, DCEM_E_INVALID_ARG, "threshold is NaN");
  if (threshold <= 0.0) threshold = 1.5;
  HIP_TRY(hipSetDevice(c->device), "set device");
  // a refit still pending reads the same vertices as this one: it is kept (or dropped by a rebuild)
  // the decision uses the quality measured after the previous refit (read at
  // the last synchronisation), so no host round trip is needed here
  const double measured = c->pending_ratio;
  int32_t rb = 0;
  // a quality-driven rebuild first rebuilds only the tree above the groups
  // (static geometry, each moving object), whose subtrees moved rigidly;
  // once the tree that leaves is itself worse than the threshold relative to
  // the last full build, the whole tree is rebuilt
  const bool subtrees = (flags & DCEM_REBUILD_SUBTREES) ||
                        (!(flags & DCEM_FORCE_REBUILD) && c->keys_grouped && c->subtree_ratio <= threshold);
  if ((flags & (DCEM_FORCE_REBUILD | DCEM_REBUILD_SUBTREES)) || measured > threshold) {
    // a frame whose results are still unread may have to redo its candidates
    // (more captures than the device path holds), which reads the tree it
    // was traced with: finish it before the tree is rebuilt
    if (c->copy_pending) {
      const dcem_status st = sync_frame(c);
      if (st != DCEM_OK) return st;
    }
    c->refit_pending = false;
    ev_record(c, 6);
    // a forced rebuild serves the frame at hand; one the quality test asks
    // for keeps the objects apart for the refits that follow
    if (subtrees && !(flags & DCEM_FORCE_REBUILD) && c->keys_grouped) {
      HIP_TRY(rebuild_subtrees(c), "rebuild BVH subtrees");
      rb = DCEM_REBUILT_SUBTREES;
    } else {
      HIP_TRY(build_lbvh(c, !(flags & DCEM_FORCE_REBUILD)), "rebuild BVH");
      rb = DCEM_REBUILT_FULL;
    }
    ev_record(c, 7);
  } else {
    // enqueued by the next call that needs the tree (a coherent trace runs
    // it in one launch with its revalidation pass), or at once with the next
    // frame's revalidation when the last frame's results are already in
    c->refit_pending = true;
    c->refit_since_build = true;
    go_ahead(c);
    HIP_TRY(hipGetLastError(), "revalidation");
  }
  c->bvh_stale = false;
  c->last_rebuilt = rb;
  c->refit_pending_timing = true;
  if (rebuilt) *rebuilt = rb;
  if (sah_ratio) *sah_ratio = rb ? 1.0 : measured;
  return DCEM_OK;
}

}  // extern "C"

namespace {

// The branches of a ray when up to max_t of its first `slots` interactions
// may transmit: every set of at most max_t interaction indices, as a bit mask
// (bit j: interaction j transmits), by size, then lexicographically (the
// empty set first: the ray that only reflects).
std::vector<uint32_t> branch_sets(int slots, int max_t) {
  std::vector<uint32_t> out{0u};
  for (int t = 1; t <= max_t; ++t) {
    std::vector<int> idx(t);
    for (int j = 0; j < t; ++j) idx[j] = j;
    while (true) {
      uint32_t m = 0;
      for (int j : idx) m |= 1u << j;
      out.push_back(m);
      int j = t - 1;
      while (j >= 0 && idx[j] == slots - t + j) --j;
      if (j < 0) break;
      ++idx[j];
      for (int q = j + 1; q < t; ++q) idx[q] = idx[q - 1] + 1;
    }
  }
  return out;
}

// What the device part of a frame does, decided by its host part.
struct FramePlan {
  bool coherent = false;    // reuse the cached rays, re-trace the listed ones
  bool keep_cache = false;  // store the segment cache for the next coherent frame
  bool small = false;       // one-workgroup candidate de-duplication
  bool ahead = false;       // the frame's start and revalidation are already enqueued
  bool los = true;
  bool recapture = false;   // coherent frame whose receivers moved: kept segments captured again
  bool visited = false;     // candidates from the visited series, not from capture spheres
  bool seed_los = true;     // direct-path records seeded into the capture list at the frame's start
  int64_t hint = 0;         // > 0: sort-based candidates sized for this many captures, counts read on the device
  int64_t n_work = 0;       // n_tx * n_rays
  int64_t expected = 0;     // work items the trace is sized for
  uint32_t n_prev = 0;      // captures of the previous frame (kept by a coherent frame)
};

// Host part of a frame: argument checks, the unread previous frame, the
// configuration, uploads and buffers.  Enqueues nothing of the frame itself
// beyond the uploads (and, when the rays changed, their directions and order).
dcem_status frame_setup(dcem_ctx* c, const dcem_trace_params* p, FramePlan& plan) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  if (c->bvh_stale) return fail(c, DCEM_E_STATE, "objects moved: call dcem_refit_bvh before tracing");
  if (!p) return fail(c, DCEM_E_INVALID_ARG, "null params");
  if (!mem_kind_ok(p->mem_kind)) return fail(c, DCEM_E_INVALID_ARG, "bad mem_kind");
  if (p->n_tx < 1 || p->n_rx < 1 || !p->tx_pos || !p->rx_pos) return fail(c, DCEM_E_INVALID_ARG, "need >= 1 tx and rx");
  if (p->n_rays < 0) return fail(c, DCEM_E_INVALID_ARG, "negative ray count");
  if (p->max_reflections < 0 || p->max_reflections > DCEM_MAX_REFLECTIONS)
    return fail(c, DCEM_E_INVALID_ARG, "max_reflections must be in [0, %d]", DCEM_MAX_REFLECTIONS);
  if (p->n_freqs < 1 || p->n_freqs > 64 || !p->freqs_hz) return fail(c, DCEM_E_INVALID_ARG, "need 1..64 frequencies");
  for (int i = 0; i < p->n_freqs; ++i)
    if (!(p->freqs_hz[i] > 0.0) || !std::isfinite(p->freqs_hz[i])) return fail(c, DCEM_E_INVALID_ARG, "bad frequency");
  if (!(p->rx_radius >= 0.0f) || !std::isfinite(p->rx_radius)) return fail(c, DCEM_E_INVALID_ARG, "bad rx_radius");
  if (!(p->tx_power_w >= 0.0) || !std::isfinite(p->tx_power_w)) return fail(c, DCEM_E_INVALID_ARG, "bad tx_power_w");
  if (!std::isfinite(p->atten_db_per_km)) return fail(c, DCEM_E_INVALID_ARG, "bad atten_db_per_km");
  if (p->mode != DCEM_MODE_FULL && p->mode != DCEM_MODE_COHERENT) return fail(c, DCEM_E_INVALID_ARG, "bad mode");
  if (p->trace_from_rx != 0 && p->trace_from_rx != 1) return fail(c, DCEM_E_INVALID_ARG, "trace_from_rx must be 0 or 1");
  if (p->discovery != DCEM_DISCOVER_CAPTURE && p->discovery != DCEM_DISCOVER_VISITED)
    return fail(c, DCEM_E_INVALID_ARG, "bad discovery mode");
  const bool visited = p->discovery == DCEM_DISCOVER_VISITED;
  if (p->max_transmissions < 0 || p->max_transmissions > DCEM_MAX_TRANSMISSIONS)
    return fail(c, DCEM_E_INVALID_ARG, "max_transmissions must be in [0, %d]", DCEM_MAX_TRANSMISSIONS);
  if (p->max_reflections + p->max_transmissions > DCEM_MAX_REFLECTIONS)
    return fail(c, DCEM_E_INVALID_ARG, "max_reflections + max_transmissions must be <= %d", DCEM_MAX_REFLECTIONS);
  const int32_t slots = p->max_reflections + p->max_transmissions;   // interactions per path at most
  const std::vector<uint32_t> bsets = branch_sets(slots, p->max_transmissions);
  const int32_t n_branch = (int32_t)bsets.size();
  const bool backward = p->trace_from_rx == 1;
  const int32_t n_src = backward ? p->n_rx : p->n_tx, n_tgt = backward ? p->n_tx : p->n_rx;
  const int64_t n_work = (int64_t)n_src * n_branch * p->n_rays;
  if (n_work >= (int64_t(1) << 31) - 1)
    return fail(c, DCEM_E_UNSUPPORTED, "work items per frame (sources x branches x n_rays) must be < 2^31 - 1");
  if ((int64_t)p->n_tx * p->n_rx >= (int64_t(1) << 27)) return fail(c, DCEM_E_UNSUPPORTED, "too many tx x rx pairs");
  {
    int bt = 0, br = 0, bf = 0;
    while ((int64_t(1) << bt) < p->n_tx) ++bt;
    while ((int64_t(1) << br) < p->n_rx) ++br;
    while ((int64_t(1) << bf) < c->nf) ++bf;
    if (bt + br + 4 + slots * (std::max(bf, 1) + (p->max_transmissions > 0 ? 1 : 0)) > 256)
      return fail(c, DCEM_E_UNSUPPORTED, "candidate key exceeds 256 bits");
  }
  HIP_TRY(hipSetDevice(c->device), "set device");
  // An unread previous frame is finished before anything of this frame
  // replaces its configuration or buffers: its results land in the frame
  // block this call may reallocate, its captures and counters are what a
  // coherent frame reuses, and a candidate redo (more captures than the
  // device path holds) must run with that frame's layout.
  if (c->has_frame && !c->counts_current) {
    const dcem_status st = sync_frame(c);
    if (st != DCEM_OK) return st;
  }
  // -- configuration and cache applicability
  std::vector<float> txh, rxh;
  HIP_TRY(fetch(txh, p->tx_pos, 3 * (size_t)p->n_tx, p->mem_kind, c->stream), "read tx");
  HIP_TRY(fetch(rxh, p->rx_pos, 3 * (size_t)p->n_rx, p->mem_kind, c->stream), "read rx");
  for (float v : txh) if (!std::isfinite(v)) return fail(c, DCEM_E_INVALID_ARG, "non-finite tx position");
  for (float v : rxh) if (!std::isfinite(v)) return fail(c, DCEM_E_INVALID_ARG, "non-finite rx position");
  const bool fib = p->ray_dirs == nullptr;
  std::vector<float> dirh;
  if (!fib && p->mem_kind == DCEM_MEM_HOST) {
    dirh.assign(p->ray_dirs, p->ray_dirs + 3 * (size_t)p->n_rays);
    for (float v : dirh) if (!std::isfinite(v)) return fail(c, DCEM_E_INVALID_ARG, "non-finite ray direction");
  }
  TraceConfig& cfg = c->cfg;
  // the trace's sources and targets (the receivers and transmitters when
  // tracing backward)
  std::vector<float>& srch = backward ? rxh : txh;
  std::vector<float>& tgth = backward ? txh : rxh;
  // the cached rays stay valid while the sources, the rays and the bounce
  // limit stay; targets may move (their captures are then taken again from
  // the cached segments)
  const bool same_geom = cfg.n_src == n_src && cfg.n_tgt == n_tgt && cfg.backward == backward &&
                         cfg.visited == visited &&
                         cfg.K == p->max_reflections && cfg.T == p->max_transmissions && cfg.n_rays == p->n_rays &&
                         cfg.rx_radius == p->rx_radius && !c->pen_pending &&
                         cfg.src == srch && cfg.dirs_fib == fib &&
                         (fib || (p->mem_kind == DCEM_MEM_HOST && cfg.dirs_host == dirh));
  const bool rx_moved = cfg.tgt != tgth;
  const bool coherent = p->mode == DCEM_MODE_COHERENT && c->cache_valid && same_geom;
  const bool keep_cache = p->keep_cache != 0 || p->mode == DCEM_MODE_COHERENT;
  plan.recapture = coherent && rx_moved && !visited;   // visited series are tried against the current targets
  // -- device inputs
  const bool need_dirs = !same_geom || !c->has_frame;
  const bool need_rx = need_dirs || rx_moved;
  cfg.n_src = n_src;
  cfg.n_tgt = n_tgt;
  cfg.backward = backward;
  cfg.visited = visited;
  cfg.K = p->max_reflections;
  cfg.T = p->max_transmissions;
  cfg.n_rays = p->n_rays;
  cfg.rx_radius = p->rx_radius;
  cfg.src = srch;
  cfg.tgt = tgth;
  cfg.dirs_fib = fib;
  cfg.dirs_ptr = p->ray_dirs;
  cfg.dirs_host = dirh;
  c->n_tx = p->n_tx;
  c->n_rx = p->n_rx;
  c->n_src = n_src;
  c->n_tgt = n_tgt;
  c->backward = backward;
  c->visited = visited;
  c->n_rays = p->n_rays;
  c->K = slots;
  c->max_refl = p->max_reflections;
  c->max_trans = p->max_transmissions;
  c->n_branch = n_branch;
  c->n_freqs = p->n_freqs;
  c->sqrt_pt = std::sqrt(p->tx_power_w);
  c->atten_db_per_km = p->atten_db_per_km;
  c->pattern_frame = c->pattern_next;
  if (c->mat_pending) {   // stream-ordered after the last frame's field and gradient kernels
    HIP_TRY(upload(c->materials, c->mat_next, c->stream), "upload materials");
    c->mat_pending = false;
  }
  c->record_log = p->record_trace_log != 0;
  if (need_dirs) HIP_TRY(upload(c->src_pos, srch, c->stream), "upload sources");   // sources or rays changed
  if (need_rx) {
    HIP_TRY(upload(c->tgt_pos, tgth, c->stream), "upload targets");
    std::vector<Node> rt = build_rx_tree(tgth, p->rx_radius);
    c->n_rx_nodes = (int32_t)rt.size();
    HIP_TRY(upload(c->rx_nodes, rt, c->stream), "upload capture-sphere tree");
    HIP_TRY(upload_rx_columns(c, tgth), "upload capture-sphere columns");
  }
  {
    std::vector<double> fv(p->freqs_hz, p->freqs_hz + p->n_freqs);
    if (fv != c->freqs_host || need_dirs || c->freqs_host.empty()) {
      HIP_TRY(upload(c->freqs, fv, c->stream), "upload freqs");
      c->freqs_host = fv;
    }
  }
  if (need_dirs) {
    HIP_TRY(ensure(c->dirs, sizeof(float) * 3 * std::max<int64_t>(p->n_rays, 1)), "alloc dirs");
    if (fib) {
      if (p->n_rays > 0) launch_fibonacci(c);
    } else if (p->mem_kind == DCEM_MEM_HOST) {
      HIP_TRY(upload(c->dirs, dirh, c->stream), "upload dirs");
    } else if (p->n_rays > 0) {
      HIP_TRY(hipMemcpyAsync(c->dirs.p, p->ray_dirs, sizeof(float) * 3 * p->n_rays, hipMemcpyDeviceToDevice, c->stream),
              "copy dirs");
    }
    HIP_TRY(build_ray_order(c), "ray order");
  }
  if (need_dirs) HIP_TRY(upload(c->branch_set, bsets, c->stream), "upload branches");
  if (c->pen_pending || c->face_pen.p == nullptr) {
    // per-face flags and per-material factors of the penetration losses
    std::vector<uint8_t> fp((size_t)std::max(c->nf, 1), 0);
    std::vector<double> mp((size_t)std::max(c->nm, 1), 0.0);
    for (int m = 0; m < c->nm; ++m) mp[m] = std::isfinite(c->pen_next[m]) ? std::pow(10.0, -c->pen_next[m] / 20.0) : 0.0;
    for (int f = 0; f < c->nf; ++f) fp[f] = std::isfinite(c->pen_next[c->h_face_material[f]]) ? 1 : 0;
    HIP_TRY(upload(c->face_pen, fp, c->stream), "upload penetration flags");
    HIP_TRY(upload(c->mat_pen, mp, c->stream), "upload penetration losses");
    c->pen_pending = false;
  }
  const size_t nw = (size_t)std::max<int64_t>(n_work, 1), K1 = (size_t)slots + 1;
  HIP_TRY(ensure(c->face_log, sizeof(int32_t) * K1 * nw), "alloc face log");
  HIP_TRY(ensure(c->ray_state, nw), "alloc ray state");
  if (keep_cache) {
    HIP_TRY(ensure(c->seg_o, sizeof(float4) * K1 * nw), "alloc segment log");
    HIP_TRY(ensure(c->seg_d, sizeof(float4) * K1 * nw), "alloc segment log");
  }
  if (c->record_log) {
    HIP_TRY(ensure(c->log_tri, sizeof(int32_t) * K1 * nw), "alloc trace log");
    HIP_TRY(ensure(c->log_t, sizeof(float) * K1 * nw), "alloc trace log");
    HIP_TRY(ensure(c->log_len, sizeof(float) * K1 * nw), "alloc trace log");
  }
  HIP_TRY(ensure(c->caps[0], sizeof(Capture) * (size_t)c->cap_capacity), "alloc captures");
  HIP_TRY(ensure(c->caps[1], sizeof(Capture) * (size_t)c->cap_capacity), "alloc captures");
  HIP_TRY(ensure(c->work_list, sizeof(uint32_t) * nw), "alloc work list");
  HIP_TRY(ensure(c->invalid_flag, nw), "alloc flags");
  HIP_TRY(ensure_frame_block(c, (int64_t)p->n_freqs * p->n_tx * p->n_rx), "alloc results");
  // counts of the previous frame (read above): its capture list (reused by a
  // coherent frame), its re-trace count (sizes the persistent grid) and its
  // capture count (picks the de-duplication path)
  // moved receivers: captures taken again; visited series: no captures
  plan.n_prev = (plan.recapture || visited) ? 0u : (uint32_t)c->n_caps_host;
  plan.n_work = n_work;
  plan.expected = coherent ? ((c->has_frame && c->stats.coherent) ? (int64_t)c->last_cnt[kCntWork] : n_work) : n_work;
  plan.small = !visited && c->has_frame && same_geom && c->n_caps_host <= small_path_capacity() * 3 / 4 &&
               small_path_fits(c);
  plan.visited = visited;
  // more captures than the one workgroup holds: the sort-based path, sized
  // from the last frame's count with room to grow, so the frame needs no
  // host round trip (a larger count is redone exactly when read)
  if (!plan.small && !visited && c->has_frame && same_geom)
    plan.hint = std::min<int64_t>(c->cap_capacity, 2 * c->n_caps_host + 4096);
  plan.coherent = coherent;
  plan.keep_cache = keep_cache;
  plan.los = p->los_always != 0;
  plan.seed_los = plan.los && !visited;   // visited discovery: the empty series gives the direct paths
  // a revalidation enqueued ahead (go_ahead) serves a coherent frame with the
  // same configuration, as long as the result block stayed in place (a
  // reallocation clears revalidated_ahead)
  plan.ahead = c->revalidated_ahead && coherent && plan.seed_los == c->last_los;
  if (plan.small) HIP_TRY(prepare_small_candidates(c), "alloc candidates");
  if (plan.hint > 0) HIP_TRY(prepare_sorted_candidates(c, plan.hint), "alloc candidates");
  HIP_TRY(prepare_trace(c), "alloc traversal stack");
  return DCEM_OK;
}

// Device part of a frame up to the trace: the frame's start (counters, line
// of sight records), the pending refit, the revalidation pass.
dcem_status frame_front(dcem_ctx* c, const FramePlan& plan) {
  if (!plan.ahead) {
    ev_record(c, 0);
    if (!c->frame_begun) c->cur_caps ^= 1;
    launch_frame_begin(c, plan.seed_los);
    if (plan.coherent && c->refit_pending) {
      // the revalidation does not read the tree: one launch with the refit
      c->refit_pending = false;
      ev_record(c, 6);
      launch_refit_coherence(c, false);
      ev_record(c, 7);
    } else {
      HIP_TRY(flush_refit(c), "refit");
      if (plan.coherent) launch_coherence(c);
    }
    c->list_clear = false;
    ev_record(c, 1);
  }
  c->frame_begun = false;
  c->revalidated_ahead = false;
  c->last_los = plan.seed_los;
  HIP_TRY(hipGetLastError(), "frame start");
  return DCEM_OK;
}

// The frame's own closest-hit launch.
dcem_status frame_trace(dcem_ctx* c, const FramePlan& plan) {
  ev_record(c, 8);
  if (plan.recapture && plan.n_work > 0) launch_recapture(c);
  const int traversal =
      plan.n_work > 0 ? launch_trace(c, !plan.coherent, plan.keep_cache, plan.expected, plan.n_prev) : 0;
  if (traversal < 0) return fail(c, DCEM_E_OUT_OF_MEMORY, "alloc traversal stack");
  c->last_trace_kernel = traversal;
  ev_record(c, 2);
  HIP_TRY(hipGetLastError(), "trace kernels");
  return DCEM_OK;
}

// Device part after the trace: candidates, refinement, reduction, and the
// copy of the frame block to pinned host memory behind them.
dcem_status frame_back(dcem_ctx* c, const FramePlan& plan) {
  if (plan.visited) {
    bool too_many = false;
    HIP_TRY(build_visited_candidates(c, plan.los, too_many), "visited-series candidates");
    if (too_many) return fail(c, DCEM_E_UNSUPPORTED, "visited series x targets must be < 2^32");
  } else {
    HIP_TRY(build_candidates(c, plan.small, plan.hint), "candidates");
  }
  ev_record(c, 3);
  HIP_TRY(ensure_paths(c, c->path_cap), "alloc paths");
  launch_refine(c);
  ev_record(c, 4);
  launch_reduce(c);
  c->list_clear = true;
  ev_record(c, 5);
  HIP_TRY(hipGetLastError(), "refine kernels");
  HIP_TRY(hipMemcpyAsync(c->host_block, c->frame_block.p, frame_block_bytes(c), hipMemcpyDeviceToHost, c->stream),
          "read results");
  return DCEM_OK;
}

// Host state once a frame's work is enqueued: its results are on their way.
dcem_status frame_done(dcem_ctx* c, const FramePlan& plan) {
  HIP_TRY(hipEventRecord(c->ev_copy, c->stream), "read results");
  c->copy_pending = true;
  c->cache_valid = plan.keep_cache;
  c->has_frame = true;
  c->counts_current = false;
  c->stats.coherent = plan.coherent ? 1 : 0;
  c->stats.rays_total = plan.n_work;
  return DCEM_OK;
}

}  // namespace

extern "C" {

dcem_status dcem_trace_frame(dcem_ctx* c, const dcem_trace_params* p) {
  FramePlan plan;
  dcem_status st = frame_setup(c, p, plan);
  if (st == DCEM_OK) st = frame_front(c, plan);
  if (st == DCEM_OK) st = frame_trace(c, plan);
  if (st == DCEM_OK) st = frame_back(c, plan);
  if (st == DCEM_OK) st = frame_done(c, plan);
  return st;
}

dcem_status dcem_received_power(dcem_ctx* c, double* p_coh, double* p_inc, int32_t mem_kind) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  if (!p_coh || !mem_kind_ok(mem_kind)) return fail(c, DCEM_E_INVALID_ARG, "bad output");
  HIP_TRY(hipSetDevice(c->device), "set device");
  dcem_status st = sync_frame(c);
  if (st != DCEM_OK) return st;
  const size_t n = (size_t)c->n_freqs * c->n_tx * c->n_rx;
  const double* hp = reinterpret_cast<const double*>(static_cast<const char*>(c->host_block) + kBlockHead);
  if (mem_kind == DCEM_MEM_HOST) {
    std::memcpy(p_coh, hp, sizeof(double) * n);
    if (p_inc) std::memcpy(p_inc, hp + c->n_pow_cap, sizeof(double) * n);
  } else {
    HIP_TRY(hipMemcpyAsync(p_coh, c->pcoh_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream), "copy power");
    if (p_inc)
      HIP_TRY(hipMemcpyAsync(p_inc, c->pinc_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream), "copy power");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  }
  go_ahead(c);   // a refit requested before these powers were read: start the next frame
  HIP_TRY(hipGetLastError(), "revalidation");
  return DCEM_OK;
}

dcem_status dcem_set_tx_pattern(dcem_ctx* c, const double* weights, int32_t n_weights) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!weights) {
    if (n_weights != 0) return fail(c, DCEM_E_INVALID_ARG, "null weights need n_weights = 0");
    c->pattern_next = TxPattern{};
    return DCEM_OK;
  }
  if (n_weights != kPatternTaps) return fail(c, DCEM_E_INVALID_ARG, "need %d pattern weights", kPatternTaps);
  for (int j = 0; j < kPatternTaps; ++j)
    if (!std::isfinite(weights[j])) return fail(c, DCEM_E_INVALID_ARG, "non-finite pattern weight");
  TxPattern p{};
  for (int j = 0; j < kPatternTaps; ++j) p.w[j] = weights[j];
  p.on = 1;
  c->pattern_next = p;
  return DCEM_OK;
}

dcem_status dcem_set_materials(dcem_ctx* c, const double* materials, int32_t n_materials) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  if (n_materials != c->nm) return fail(c, DCEM_E_INVALID_ARG, "the scene has %d materials", c->nm);
  if (n_materials > 0 && !materials) return fail(c, DCEM_E_INVALID_ARG, "null materials");
  const dcem_status ms = check_materials(c, materials, n_materials);
  if (ms != DCEM_OK) return ms;
  c->mat_next.assign(materials, materials + 3 * (size_t)n_materials);
  c->mat_pending = true;
  return DCEM_OK;
}

dcem_status dcem_set_penetration_loss(dcem_ctx* c, const double* loss_db, int32_t n_materials) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  if (n_materials != c->nm) return fail(c, DCEM_E_INVALID_ARG, "the scene has %d materials", c->nm);
  if (n_materials > 0 && !loss_db) return fail(c, DCEM_E_INVALID_ARG, "null losses");
  for (int m = 0; m < n_materials; ++m)
    if (!(loss_db[m] >= 0.0)) return fail(c, DCEM_E_INVALID_ARG, "material %d: loss must be >= 0 dB or +inf", m);
  c->pen_next.assign(loss_db, loss_db + n_materials);
  c->pen_pending = true;
  return DCEM_OK;
}

dcem_status dcem_power_gradients(dcem_ctx* c, double* d_eps_r, double* d_sigma, double* d_tx_power,
                                 double* d_pattern) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  HIP_TRY(hipSetDevice(c->device), "set device");
  dcem_status st = sync_frame(c);
  if (st != DCEM_OK) return st;
  const size_t n = (size_t)c->n_freqs * c->n_tx * c->n_rx;
  if (d_tx_power) {
    // P is proportional to the transmit power
    const double* hp = reinterpret_cast<const double*>(static_cast<const char*>(c->host_block) + kBlockHead);
    const double pt = c->sqrt_pt * c->sqrt_pt;
    for (size_t i = 0; i < n; ++i) d_tx_power[i] = pt > 0 ? hp[i] / pt : 0.0;
  }
  const size_t ng = n * (size_t)std::max(c->nm, 0);
  const size_t np = n * kPatternTaps;
  const bool want_mat = (d_eps_r || d_sigma) && ng > 0;
  if (want_mat || d_pattern) {
    HIP_TRY(ensure(c->grad_buf, sizeof(double) * (2 * ng + np)), "alloc gradients");
    double* g = ptr<double>(c->grad_buf);
    // the frame's unique candidates (its path arrays stay until the next
    // frame's trace, also when that frame has begun)
    const uint32_t nu = c->last_cnt[kCntUnique];
    launch_power_grad(c, nu, want_mat ? g : nullptr, g + ng, d_pattern ? g + 2 * ng : nullptr);
    HIP_TRY(hipGetLastError(), "gradient kernel");
    // one transfer into pinned memory, then host copies into the caller's arrays
    const size_t lo = want_mat ? 0 : 2 * ng, hi = d_pattern ? 2 * ng + np : 2 * ng;
    const size_t bytes = sizeof(double) * (2 * ng + np);
    if (c->grad_host_bytes < bytes) {
      if (c->grad_host) (void)hipHostFree(c->grad_host);
      c->grad_host = nullptr;
      c->grad_host_bytes = 0;
      HIP_TRY(hipHostMalloc(&c->grad_host, bytes, hipHostMallocDefault), "alloc pinned gradients");
      c->grad_host_bytes = bytes;
    }
    double* h = static_cast<double*>(c->grad_host);
    HIP_TRY(hipMemcpyAsync(h + lo, g + lo, sizeof(double) * (hi - lo), hipMemcpyDeviceToHost, c->stream), "copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
    if (d_eps_r && want_mat) std::memcpy(d_eps_r, h, sizeof(double) * ng);
    if (d_sigma && want_mat) std::memcpy(d_sigma, h + ng, sizeof(double) * ng);
    if (d_pattern) std::memcpy(d_pattern, h + 2 * ng, sizeof(double) * np);
  }
  return DCEM_OK;
}

dcem_status dcem_power_gradients_noalloc(dcem_ctx* c, double* d_eps_r, double* d_sigma, double* d_tx_power,
                                         double* d_pattern) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  // the frame must be finished (its results read): finishing it could
  // allocate (a candidate redo when its captures overflowed the device path)
  if (!c->counts_current) return fail(c, DCEM_E_STATE, "the frame's results are unread: call dcem_received_power");
  if (!c->scratch) return fail(c, DCEM_E_DEVICE, "no gradient workspace on device %d", c->device);
  const size_t n = (size_t)c->n_freqs * c->n_tx * c->n_rx;
  const size_t ng = n * (size_t)std::max(c->nm, 0);
  const size_t np = n * kPatternTaps;
  if (2 * ng + np > (size_t)DCEM_NOALLOC_GRAD_DOUBLES)
    return fail(c, DCEM_E_UNSUPPORTED, "gradients need %zu doubles of workspace, the fixed array holds %d",
                2 * ng + np, DCEM_NOALLOC_GRAD_DOUBLES);
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (d_tx_power) {
    const double* hp = reinterpret_cast<const double*>(static_cast<const char*>(c->host_block) + kBlockHead);
    const double pt = c->sqrt_pt * c->sqrt_pt;
    for (size_t i = 0; i < n; ++i) d_tx_power[i] = pt > 0 ? hp[i] / pt : 0.0;
  }
  const bool want_mat = (d_eps_r || d_sigma) && ng > 0;
  if (want_mat || d_pattern) {
    double* g = c->scratch;   // the array's address on this device, never its host-side name
    const uint32_t nu = c->last_cnt[kCntUnique];
    launch_power_grad(c, nu, want_mat ? g : nullptr, g + ng, d_pattern ? g + 2 * ng : nullptr);
    HIP_TRY(hipGetLastError(), "gradient kernel");
    // straight into the caller's arrays (no pinned staging)
    if (d_eps_r && want_mat)
      HIP_TRY(hipMemcpyAsync(d_eps_r, g, sizeof(double) * ng, hipMemcpyDeviceToHost, c->stream), "copy");
    if (d_sigma && want_mat)
      HIP_TRY(hipMemcpyAsync(d_sigma, g + ng, sizeof(double) * ng, hipMemcpyDeviceToHost, c->stream), "copy");
    if (d_pattern)
      HIP_TRY(hipMemcpyAsync(d_pattern, g + 2 * ng, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream), "copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  }
  return DCEM_OK;
}

dcem_status dcem_get_stats(dcem_ctx* c, dcem_frame_stats* out) {
  if (!c || !out) return DCEM_E_INVALID_ARG;
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  dcem_status st = sync_frame(c);
  if (st != DCEM_OK) return st;
  const uint32_t* cnt = c->last_cnt;
  dcem_frame_stats& s = c->stats;
  s.rays_traced = s.coherent ? (int64_t)cnt[kCntWork] : s.rays_total;
  s.rays_reused = s.rays_total - s.rays_traced;
  s.segments = cnt[kCntSegments];
  s.captures = c->n_caps_host;
  s.unique_candidates = cnt[kCntUnique];
  s.valid_paths = cnt[kCntValid];
  uint64_t nodes = 0, tris = 0;
  std::memcpy(&nodes, &cnt[kCntNodes], 8);
  std::memcpy(&tris, &cnt[kCntTris], 8);
  s.nodes_visited = (int64_t)nodes;
  s.tri_tests = (int64_t)tris;
  s.rebuilt = c->last_rebuilt;
  s.trace_kernel = c->last_trace_kernel;
  s.sah_ratio = c->sah_last;
  *out = s;   // stage times: taken when the frame's results arrived (sync_frame)
  return DCEM_OK;
}

dcem_status dcem_get_paths(dcem_ctx* c, int64_t cap, int32_t* keys, uint8_t* valid, double* length, double* tau,
                           double* aod, double* aoa, double* amp, int32_t* first_ray, int64_t* n_out) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  if (cap < 0) return fail(c, DCEM_E_INVALID_ARG, "negative capacity");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  dcem_status st = check_device_error(c);
  if (st != DCEM_OK) return st;
  const uint32_t nu = c->last_cnt[kCntUnique];   // cleared at each frame's start
  if (n_out) *n_out = nu;
  const int64_t n = std::min<int64_t>(nu, cap);
  if (n == 0) return DCEM_OK;
  auto get = [&](void* dst, DevBuf& b, size_t bytes) -> hipError_t {
    if (!dst) return hipSuccess;
    return hipMemcpy(dst, b.p, bytes, hipMemcpyDeviceToHost);
  };
  HIP_TRY(get(valid, c->path_valid, n), "copy valid");
  HIP_TRY(get(length, c->path_len, 8 * n), "copy length");
  HIP_TRY(get(tau, c->path_tau, 8 * n), "copy tau");
  HIP_TRY(get(aod, c->path_aod, 24 * n), "copy aod");
  HIP_TRY(get(aoa, c->path_aoa, 24 * n), "copy aoa");
  HIP_TRY(get(amp, c->path_amp, 48 * n * (size_t)c->n_freqs), "copy amp");
  HIP_TRY(get(first_ray, c->first_ray, 4 * n), "copy first ray");
  if (keys) {
    // the decoded candidates (pair, order, faces) the de-duplication or the
    // visited-series expansion wrote, in key order
    std::vector<int32_t> pair((size_t)n), faces((size_t)n * std::max(c->K, 1));
    std::vector<uint8_t> order((size_t)n);
    HIP_TRY(hipMemcpy(pair.data(), c->pair_range.p, 4 * (size_t)n, hipMemcpyDeviceToHost), "copy pairs");
    HIP_TRY(hipMemcpy(order.data(), c->path_order.p, (size_t)n, hipMemcpyDeviceToHost), "copy orders");
    if (c->K > 0)
      HIP_TRY(hipMemcpy(faces.data(), c->path_faces.p, 4 * (size_t)n * c->K, hipMemcpyDeviceToHost), "copy faces");
    const int K = c->K;
    for (int64_t u = 0; u < n; ++u) {
      int32_t* row = keys + u * (3 + K);
      row[0] = pair[u] / c->n_rx;
      row[1] = pair[u] % c->n_rx;
      row[2] = order[u];
      for (int j = 0; j < K; ++j) {
        const int32_t fe = faces[(size_t)u * K + j];
        // a transmission through face f is reported as -2 - f
        row[3 + j] = j >= order[u] ? -1 : ((fe & kTransmit) ? -2 - (fe & kFaceMask) : fe);
      }
    }
  }
  return DCEM_OK;
}

dcem_status dcem_get_trace_log(dcem_ctx* c, int32_t* tri, float* t, float* length) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  if (!c->record_log) return fail(c, DCEM_E_STATE, "trace log not recorded (record_trace_log = 0)");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  dcem_status st = check_device_error(c);
  if (st != DCEM_OK) return st;
  const size_t n = (size_t)c->n_src * c->n_branch * c->n_rays * (c->K + 1);
  if (tri) HIP_TRY(hipMemcpy(tri, c->log_tri.p, 4 * n, hipMemcpyDeviceToHost), "copy log");
  if (t) HIP_TRY(hipMemcpy(t, c->log_t.p, 4 * n, hipMemcpyDeviceToHost), "copy log");
  if (length) HIP_TRY(hipMemcpy(length, c->log_len.p, 4 * n, hipMemcpyDeviceToHost), "copy log");
  return DCEM_OK;
}

dcem_status dcem_get_captures(dcem_ctx* c, int64_t cap, int32_t* rows, int64_t* n_out) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  if (cap < 0) return fail(c, DCEM_E_INVALID_ARG, "negative capacity");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  dcem_status st = check_device_error(c);
  if (st != DCEM_OK) return st;
  const int64_t nc = c->n_caps_host;
  if (n_out) *n_out = nc;
  if (!rows || nc == 0) return DCEM_OK;
  std::vector<Capture> cp(nc);
  const int list = c->frame_begun ? c->cur_caps ^ 1 : c->cur_caps;   // the last traced frame's
  HIP_TRY(hipMemcpy(cp.data(), c->caps[list].p, sizeof(Capture) * nc, hipMemcpyDeviceToHost), "copy caps");
  const int64_t n_work = (int64_t)c->n_src * c->n_branch * c->n_rays;
  // records and the face log are indexed by traversal position; rows name the ray
  std::vector<uint32_t> order((size_t)std::max<int64_t>(c->n_rays, 1));
  if (c->n_rays > 0)
    HIP_TRY(hipMemcpy(order.data(), c->ray_order.p, 4 * (size_t)c->n_rays, hipMemcpyDeviceToHost), "copy order");
  // the ray column: (source * n_branch + branch) * n_rays + ray (branch 0 only reflects)
  auto ray_of = [&](uint32_t p) -> int32_t {
    const int64_t vs = p / c->n_rays;
    return (int32_t)(vs * c->n_rays + order[(size_t)(p - vs * c->n_rays)]);
  };
  std::vector<uint32_t> bsets((size_t)c->n_branch);
  HIP_TRY(hipMemcpy(bsets.data(), c->branch_set.p, 4 * bsets.size(), hipMemcpyDeviceToHost), "copy branches");
  const int K = c->K;
  std::vector<int32_t> flog((size_t)(K + 1) * std::max<int64_t>(n_work, 1));
  if (n_work > 0)
    HIP_TRY(hipMemcpy(flog.data(), c->face_log.p, 4 * flog.size(), hipMemcpyDeviceToHost), "copy face log");
  std::vector<std::vector<int32_t>> out;
  out.reserve(nc);
  for (const Capture& x : cp) {
    std::vector<int32_t> r(4 + K, -1);
    const uint32_t pair = x.pair_order >> 4, order = x.pair_order & 15u;
    r[0] = x.work == kNoRay ? -1 : ray_of(x.work);
    r[1] = (int32_t)(pair / c->n_tgt);
    r[2] = (int32_t)(pair % c->n_tgt);
    r[3] = (int32_t)order;
    const uint32_t tset = x.work == kNoRay ? 0u : bsets[(x.work / c->n_rays) % c->n_branch];
    for (uint32_t j = 0; j < order; ++j) {
      const int32_t f = flog[(size_t)j * n_work + x.work];
      r[4 + j] = ((tset >> j) & 1u) ? -2 - f : f;
    }
    out.push_back(std::move(r));
  }
  std::sort(out.begin(), out.end(), [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
    if (a[1] != b[1]) return a[1] < b[1];
    if (a[2] != b[2]) return a[2] < b[2];
    if (a[3] != b[3]) return a[3] < b[3];
    for (size_t j = 4; j < a.size(); ++j)
      if (a[j] != b[j]) return a[j] < b[j];
    return a[0] < b[0];
  });
  const int64_t n = std::min<int64_t>(nc, cap);
  for (int64_t i = 0; i < n; ++i) std::memcpy(rows + i * (4 + K), out[i].data(), sizeof(int32_t) * (4 + K));
  return DCEM_OK;
}

dcem_status dcem_get_bvh(dcem_ctx* c, int64_t cap_internal, int32_t* n_internal, int32_t* child, float* box,
                         int32_t* leaf_tri) {
  if (!c) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  const int32_t ni = c->nt > 0 ? c->n_internal : 0;
  if (n_internal) *n_internal = ni;
  if (ni == 0) return DCEM_OK;
  if ((child || box) && cap_internal < ni) return fail(c, DCEM_E_INVALID_ARG, "capacity below node count");
  std::vector<Node> nodes(ni);
  HIP_TRY(hipMemcpy(nodes.data(), c->nodes.p, sizeof(Node) * ni, hipMemcpyDeviceToHost), "copy nodes");
  for (int32_t i = 0; i < ni; ++i) {
    if (child) {
      child[2 * i] = nodes[i].c.x;
      child[2 * i + 1] = nodes[i].c.y;
    }
    if (box) std::memcpy(box + 12 * i, &nodes[i], 12 * sizeof(float));
  }
  if (leaf_tri) HIP_TRY(hipMemcpy(leaf_tri, c->leaf_tri.p, 4 * c->nt, hipMemcpyDeviceToHost), "copy leaves");
  return DCEM_OK;
}

dcem_status dcem_get_vertices(dcem_ctx* c, float* out) {
  if (!c || !out) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_scene) return fail(c, DCEM_E_STATE, "no scene uploaded");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  if (c->nv) HIP_TRY(hipMemcpy(out, c->vertices.p, sizeof(float) * 3 * c->nv, hipMemcpyDeviceToHost), "copy vertices");
  return check_device_error(c);
}

dcem_status dcem_get_ray_dirs(dcem_ctx* c, float* out) {
  if (!c || !out) return DCEM_E_INVALID_ARG;
  c->err.clear();
  if (!c->has_frame) return fail(c, DCEM_E_STATE, "no frame traced");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(flush_refit(c), "refit");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronize");
  if (c->n_rays) HIP_TRY(hipMemcpy(out, c->dirs.p, sizeof(float) * 3 * c->n_rays, hipMemcpyDeviceToHost), "copy dirs");
  return DCEM_OK;
}

}  // extern "C"

// ---- batches: one frame of several contexts with one persistent trace launch

struct dcem_batch {
  std::vector<dcem_ctx*> ctx;
  int device = 0;
  hipStream_t stream = nullptr;
  dcem::DevBuf table, spill;          // per-context trace arguments + chunk table; stack spill space
  void* host_table = nullptr;         // pinned staging of `table`
  size_t host_table_bytes = 0;
  dcem::BatchShape shape;
  bool tuned = false;
  bool use_graph = false;
  hipGraphExec_t exec = nullptr;      // the last captured frame, updated in place when its topology holds
  int graph_frames = 0;               // frames launched as one graph
  hipEvent_t ev[2] = {};
  float ms_trace = 0.f;               // the last directly launched batch trace (or graph frame)
};

namespace {

dcem_status batch_fail(dcem_batch* b, dcem_status s, const char* msg) {
  for (dcem_ctx* c : b->ctx) c->err = msg;
  return s;
}

// Buffers of a batch launch of `shape` (from the first context's allocator).
hipError_t batch_buffers(dcem_batch* b, const dcem::BatchShape& shape) {
  hipError_t e;
  const size_t tb = batch_table_bytes((int)b->ctx.size());
  if ((e = ensure(b->table, tb)) != hipSuccess) return e;
  if ((e = ensure(b->spill, batch_spill_bytes(b->ctx[0], shape))) != hipSuccess) return e;
  if (b->host_table_bytes < tb) {
    if (b->host_table) (void)hipHostFree(b->host_table);
    b->host_table = nullptr;
    b->host_table_bytes = 0;
    if ((e = hipHostMalloc(&b->host_table, tb, hipHostMallocDefault)) != hipSuccess) return e;
    b->host_table_bytes = tb;
  }
  return hipSuccess;
}

// One batched frame: every context's host part, then the device work of all
// of them (frame starts and refits, the full traces in one persistent launch
// (coherent contexts trace their own re-trace lists), candidates, refinement,
// reductions and read-backs), captured as one HIP graph when asked for and
// possible.  `timed`: HIP events around the batched trace (direct launch).
dcem_status batch_frame(dcem_batch* b, const dcem_trace_params* params, const dcem::BatchShape& shape, bool timed) {
  const int n = (int)b->ctx.size();
  std::vector<FramePlan> plan(n);
  for (int j = 0; j < n; ++j) {
    const dcem_status st = frame_setup(b->ctx[j], &params[j], plan[j]);
    if (st != DCEM_OK) return st;
  }
  dcem_ctx* c = b->ctx[0];   // for HIP_TRY's messages
  HIP_TRY(hipSetDevice(b->device), "set device");
  if (batch_buffers(b, shape) != hipSuccess) return batch_fail(b, DCEM_E_OUT_OF_MEMORY, "alloc batch buffers");
  std::vector<dcem_ctx*> full;
  std::vector<uint8_t> full_cache;   // the full trace stores the segment cache (a coherent frame follows)
  bool capturable = b->use_graph && b->stream != nullptr && !timed;
  for (int j = 0; j < n; ++j) {
    dcem_ctx* cj = b->ctx[j];
    if (!plan[j].coherent && plan[j].n_work > 0) {
      full.push_back(cj);
      full_cache.push_back(plan[j].keep_cache ? 1 : 0);
    }
    // device-side decisions only (no host round trip, no timing events)
    capturable = capturable && (plan[j].small || plan[j].hint > 0) && !cj->timing;
  }
  if (capturable) HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed), "begin capture");
  dcem_status st = DCEM_OK;
  for (int j = 0; j < n && st == DCEM_OK; ++j) st = frame_front(b->ctx[j], plan[j]);
  if (st == DCEM_OK && timed) (void)hipEventRecord(b->ev[0], b->stream);
  if (st == DCEM_OK && !full.empty()) {
    for (dcem_ctx* f : full) ev_record(f, 8);
    const hipError_t e = launch_trace_batch(full.data(), full_cache.data(), (int)full.size(), shape, b->table,
                                            b->host_table, b->host_table_bytes, b->spill, b->stream);
    if (e != hipSuccess) st = hip_fail(c, e, "batched trace");
    for (dcem_ctx* f : full) {
      f->last_trace_kernel = 0;
      ev_record(f, 2);
    }
  }
  if (st == DCEM_OK && timed) (void)hipEventRecord(b->ev[1], b->stream);
  for (int j = 0; j < n && st == DCEM_OK; ++j)
    if (plan[j].coherent) st = frame_trace(b->ctx[j], plan[j]);
  for (int j = 0; j < n && st == DCEM_OK; ++j) st = frame_back(b->ctx[j], plan[j]);
  if (capturable) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != DCEM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_TRY(e, "end capture");
    bool updated = false;
    if (b->exec) {
      hipGraphExecUpdateResult res;
      hipGraphNode_t bad = nullptr;
      updated = hipGraphExecUpdate(b->exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
      if (!updated) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
      }
    }
    if (!updated) {
      const hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->exec = nullptr;
        return hip_fail(c, ie, "instantiate graph");
      }
    }
    (void)hipGraphDestroy(g);
    HIP_TRY(hipGraphLaunch(b->exec, b->stream), "launch graph");
    ++b->graph_frames;
  }
  if (st != DCEM_OK) return st;
  for (int j = 0; j < n; ++j) {
    st = frame_done(b->ctx[j], plan[j]);
    if (st != DCEM_OK) return st;
  }
  return DCEM_OK;
}

}  // namespace

extern "C" {

dcem_status dcem_batch_create(dcem_batch** out, dcem_ctx* const* ctxs, int32_t n) {
  if (!out) return DCEM_E_INVALID_ARG;
  *out = nullptr;
  if (!ctxs || n < 1) return DCEM_E_INVALID_ARG;
  for (int32_t j = 0; j < n; ++j) {
    if (!ctxs[j]) return DCEM_E_INVALID_ARG;
    if (ctxs[j]->device != ctxs[0]->device || ctxs[j]->stream != ctxs[0]->stream)
      return fail(ctxs[j], DCEM_E_INVALID_ARG, "batched contexts must share one device and one stream");
    for (int32_t k = 0; k < j; ++k)
      if (ctxs[k] == ctxs[j]) return fail(ctxs[j], DCEM_E_INVALID_ARG, "a context appears twice in the batch");
  }
  dcem_batch* b = new dcem_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->device = ctxs[0]->device;
  b->stream = ctxs[0]->stream;
  b->table.al = b->spill.al = &ctxs[0]->alloc;
  if (hipSetDevice(b->device) != hipSuccess || hipEventCreate(&b->ev[0]) != hipSuccess ||
      hipEventCreate(&b->ev[1]) != hipSuccess) {
    dcem_batch_destroy(b);
    return DCEM_E_DEVICE;
  }
  *out = b;
  return DCEM_OK;
}

void dcem_batch_destroy(dcem_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  release(b->table);
  release(b->spill);
  if (b->host_table) (void)hipHostFree(b->host_table);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  delete b;
}

dcem_status dcem_batch_set_graph(dcem_batch* b, int32_t enabled) {
  if (!b) return DCEM_E_INVALID_ARG;
  b->use_graph = enabled != 0;
  return DCEM_OK;
}

dcem_status dcem_batch_set_shape(dcem_batch* b, int32_t lds_stack, int32_t blocks_per_cu, int32_t chunk) {
  if (!b) return DCEM_E_INVALID_ARG;
  if ((lds_stack != 16 && lds_stack != 32) || blocks_per_cu < 1 || blocks_per_cu > 32 || chunk < 64 ||
      chunk % 64 != 0 || chunk > (1 << 20))
    return batch_fail(b, DCEM_E_INVALID_ARG, "shape: lds_stack 16 or 32, 1..32 blocks per CU, chunk a multiple of 64");
  b->shape.lds_stack = lds_stack;
  b->shape.blocks_per_cu = blocks_per_cu;
  b->shape.chunk = chunk;
  return DCEM_OK;
}

dcem_status dcem_batch_trace(dcem_batch* b, const dcem_trace_params* params) {
  if (!b) return DCEM_E_INVALID_ARG;
  if (!params) return batch_fail(b, DCEM_E_INVALID_ARG, "null params");
  return batch_frame(b, params, b->shape, false);
}

dcem_status dcem_batch_tune(dcem_batch* b, const dcem_trace_params* params, int32_t repeats) {
  if (!b) return DCEM_E_INVALID_ARG;
  if (!params || repeats < 1) return batch_fail(b, DCEM_E_INVALID_ARG, "null params or repeats < 1");
  // block shape and LDS stack depth first (chunk 256), then the chunk
  std::vector<dcem::BatchShape> cand;
  for (int lds : {32, 16})
    for (int bpc : {4, 6, 8, 12, 16}) {
      if (lds == 32 && bpc > 8) continue;   // 16 KB of LDS stack per block: at most 9 blocks per CU
      cand.push_back(dcem::BatchShape{lds, bpc, 256});
    }
  auto time_shape = [&](const dcem::BatchShape& sh, float* best_ms) -> dcem_status {
    float sum = 0.f;
    for (int r = 0; r < repeats; ++r) {
      dcem_status st = batch_frame(b, params, sh, true);
      if (st != DCEM_OK) return st;
      dcem_ctx* c = b->ctx[0];
      HIP_TRY(hipEventSynchronize(b->ev[1]), "synchronize");
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]), "elapsed");
      sum += ms;
    }
    *best_ms = sum / repeats;
    return DCEM_OK;
  };
  float best = INFINITY;
  dcem::BatchShape best_shape = b->shape;
  for (const auto& sh : cand) {
    float ms = 0.f;
    const dcem_status st = time_shape(sh, &ms);
    if (st != DCEM_OK) return st;
    if (ms < best) {
      best = ms;
      best_shape = sh;
    }
  }
  for (int chunk : {64, 1024}) {
    dcem::BatchShape sh = best_shape;
    sh.chunk = chunk;
    float ms = 0.f;
    const dcem_status st = time_shape(sh, &ms);
    if (st != DCEM_OK) return st;
    if (ms < best) {
      best = ms;
      best_shape = sh;
    }
  }
  b->shape = best_shape;
  b->tuned = true;
  b->ms_trace = best;
  return DCEM_OK;
}

dcem_status dcem_batch_get_info(const dcem_batch* b, dcem_batch_info* out) {
  if (!b || !out) return DCEM_E_INVALID_ARG;
  out->n_ctx = (int32_t)b->ctx.size();
  out->lds_stack = b->shape.lds_stack;
  out->blocks_per_cu = b->shape.blocks_per_cu;
  out->chunk = b->shape.chunk;
  out->tuned = b->tuned ? 1 : 0;
  out->graph_frames = b->graph_frames;
  out->ms_trace_tuned = b->ms_trace;
  return DCEM_OK;
}

}  // extern "C"
