// kdt_api.hip -- C ABI entry points for tree construction and inspection,
// error reporting and the cache of device-resident build schedules.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kdt_debug.h"
#include "kdt_query.h"

static thread_local std::string g_error;

void kdt_set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}

void kdt_clear_error() { g_error.clear(); }

extern "C" const char* kdt_last_error(void) { return g_error.c_str(); }

namespace kdt {

namespace {
struct ScratchKey {
  int device;
  hipStream_t stream;
  int slot;
  bool operator<(const ScratchKey& o) const {
    if (device != o.device) return device < o.device;
    if (stream != o.stream) return stream < o.stream;
    return slot < o.slot;
  }
};
struct ScratchBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_scratch_mu;
// never destroyed: device memory is not released from static destructors
std::map<ScratchKey, ScratchBuf>* g_scratch = new std::map<ScratchKey, ScratchBuf>();
}  // namespace

namespace {
std::atomic<int64_t> g_fail_after{-1};
}  // namespace

bool alloc_should_fail() {
  int64_t v = g_fail_after.load();
  while (v > 0) {
    if (g_fail_after.compare_exchange_weak(v, v - 1)) return v == 1;
  }
  return false;
}

unsigned long long* visit_counters() {
#ifdef KDT_COUNT_VISITS
  static unsigned long long* buf = nullptr;
  static std::once_flag once;
  std::call_once(once, [] {
    const size_t bytes = sizeof(unsigned long long) * kVisitSlots * kVisitShards;
    if (hipMalloc((void**)&buf, bytes) != hipSuccess || hipMemset(buf, 0, bytes) != hipSuccess)
      buf = nullptr;
  });
  return buf;
#else
  return nullptr;
#endif
}

void* stream_scratch(hipStream_t stream, int slot, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchBuf& b = (*g_scratch)[ScratchKey{dev, stream, slot}];
  if (b.ptr && b.bytes >= bytes) return b.ptr;
  if (b.ptr) (void)hipFreeAsync(b.ptr, stream);
  b.ptr = nullptr;
  b.bytes = 0;
  // grow by a quarter beyond the request, so slowly growing calls settle
  const size_t want = std::max<size_t>(256, bytes + bytes / 4);
  if (dev_alloc(&b.ptr, want, stream) != hipSuccess) {
    b.ptr = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.ptr;
}

extern "C" kdt_status kdt_stream_release(hipStream_t stream) {
  kdt_clear_error();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    kdt_set_error("kdt_stream_release: no current device");
    return KDT_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  kdt_status st = KDT_OK;
  for (auto it = g_scratch->begin(); it != g_scratch->end();) {
    if (it->first.device == dev && it->first.stream == stream) {
      if (it->second.ptr && hipFreeAsync(it->second.ptr, stream) != hipSuccess) {
        kdt_set_error("kdt_stream_release: hipFreeAsync failed");
        st = KDT_EDEVICE;
      }
      it = g_scratch->erase(it);
    } else {
      ++it;
    }
  }
  return st;
}


// Build schedules depend only on (device, n, d, leaf); repeated builds of the
// same shape reuse the uploaded tables.
// The device tables are released with the last reference (hipFree waits for
// the device, so a build still reading them finishes first).
struct CachedPlan {
  int device;
  int64_t n;
  int d, leaf;
  Plan plan;
  PlanDev dev;
  CachedPlan() = default;
  CachedPlan(const CachedPlan&) = delete;
  CachedPlan& operator=(const CachedPlan&) = delete;
  ~CachedPlan() { plan_release(dev); }
};

static std::mutex g_plan_mu;
// Never destroyed: releasing device memory from static destructors at process
// exit could run after the HIP runtime has shut down.
static std::list<std::shared_ptr<CachedPlan>>& g_plans =
    *new std::list<std::shared_ptr<CachedPlan>>();
constexpr size_t kPlanCache = 512;

static kdt_status get_plan(int device, int64_t n, int d, int leaf, hipStream_t stream,
                           std::shared_ptr<CachedPlan>& out) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
    if ((*it)->device == device && (*it)->n == n && (*it)->d == d && (*it)->leaf == leaf) {
      out = *it;
      g_plans.splice(g_plans.begin(), g_plans, it);
      return KDT_OK;
    }
  }
  auto cp = std::make_shared<CachedPlan>();
  cp->device = device;
  cp->n = n;
  cp->d = d;
  cp->leaf = leaf;
  int64_t offs[2] = {0, n};
  std::string err;
  if (!make_plan(offs, 1, d, &leaf, cp->plan, err)) {
    kdt_set_error("%s", err.c_str());
    return KDT_EINVAL;
  }
  kdt_status st = plan_upload(cp->plan, cp->dev, stream);
  if (st != KDT_OK) return st;
  g_plans.push_front(cp);
  // the oldest plans leave the cache; one still held by a running build is
  // released when that build drops it
  while (g_plans.size() > kPlanCache) g_plans.pop_back();
  out = cp;
  return KDT_OK;
}

static bool dim_ok(int d) { return d == 2 || d == 3 || d == 4 || d == 8 || d == 16; }

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_build(const float* d_pts, int64_t n, int32_t d,
                                const kdt_build_opts* opts, hipStream_t stream, kdt_tree** out) {
  kdt_clear_error();
  if (!out) {
    kdt_set_error("kdt_build: out is NULL");
    return KDT_EINVAL;
  }
  *out = nullptr;
  if (!d_pts || n < 1 || n > INT32_MAX) {
    kdt_set_error("kdt_build: NULL points or n=%lld outside [1, 2^31-1]", (long long)n);
    return KDT_EINVAL;
  }
  if (!dim_ok(d)) {
    kdt_set_error("kdt_build: dimension %d is not one of 2, 3, 4, 8, 16", d);
    return KDT_EUNSUPPORTED;
  }
  int leaf = 0, check = 1, rule = 0, tune_k = 0;  // check: 0 none, 1 wait, 2 deferred
  if (opts) {
    leaf = opts->leaf_size;
    check = opts->check_finite;
    rule = opts->split_rule;
    tune_k = opts->tune_k;
  }
  if (tune_k < 0) {
    kdt_set_error("kdt_build: tune_k %d is negative", tune_k);
    return KDT_EINVAL;
  }
  if (leaf == 0) leaf = tuned(d, n, tune_k ? tune_k : 32).leaf;
  if (leaf < 2 || leaf > 256) {
    kdt_set_error("kdt_build: leaf_size %d outside [2, 256]", leaf);
    return KDT_EINVAL;
  }
  if (check < 0 || check > 2) {
    kdt_set_error("kdt_build: check_finite %d is not 0, 1 or 2", check);
    return KDT_EINVAL;
  }
  if (rule != 0 && rule != 1) {
    kdt_set_error("kdt_build: split_rule %d is not 0 (median) or 1 (sliding midpoint)", rule);
    return KDT_EINVAL;
  }
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) {
    kdt_set_error("kdt_build: no HIP device");
    return KDT_EDEVICE;
  }
  if (rule == 1) {
    kdt_tree* t = new (std::nothrow) kdt_tree();
    if (!t) {
      kdt_set_error("kdt_build: out of host memory");
      return KDT_ENOMEM;
    }
    t->device = device;
    t->stream = stream;
    t->n = n;
    t->d = d;
    t->leaf = leaf;
    t->stride = rec_stride(d);
    const kdt_status st = build_midpoint(d_pts, n, d, leaf, check != 0, stream, t);
    if (st != KDT_OK) {
      if (t->rec) (void)hipFreeAsync(t->rec, stream);
      delete t;
      return st;
    }
    *out = t;
    return KDT_OK;
  }
  std::shared_ptr<CachedPlan> cp;
  kdt_status st = get_plan(device, n, d, leaf, stream, cp);
  if (st != KDT_OK) return st;
  const Plan& plan = cp->plan;

  kdt_tree* t = new (std::nothrow) kdt_tree();
  if (!t) {
    kdt_set_error("kdt_build: out of host memory");
    return KDT_ENOMEM;
  }
  t->device = device;
  t->stream = stream;
  t->n = n;
  t->d = d;
  t->leaf = leaf;
  t->levels = plan.sets[0].levels;
  t->stride = rec_stride(d);
  t->n_nodes = plan.n_nodes;
  const size_t b_rec = sizeof(float) * (size_t)n * t->stride;
  const size_t b_box = sizeof(float) * (size_t)t->n_nodes * 2 * pad4(d);
  const size_t b_perm = sizeof(int32_t) * (size_t)n;
  const size_t b_axis = sizeof(int32_t) * (size_t)t->n_nodes;
  const size_t b_split = sizeof(float) * (size_t)t->n_nodes;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  void* block = nullptr;
  // + 256 B for the deferred finiteness flag
  if (dev_alloc(&block, up(b_rec) + up(b_box) + up(b_perm) + up(b_axis) + up(b_split) + 256,
                stream) != hipSuccess) {
    delete t;
    kdt_set_error("kdt_build: cannot allocate the tree (%lld points)", (long long)n);
    return KDT_ENOMEM;
  }
  unsigned char* bp = static_cast<unsigned char*>(block);
  t->rec = reinterpret_cast<float*>(bp);
  t->box = reinterpret_cast<float*>(bp + up(b_rec));
  t->perm = reinterpret_cast<int32_t*>(bp + up(b_rec) + up(b_box));
  t->axis = reinterpret_cast<int32_t*>(bp + up(b_rec) + up(b_box) + up(b_perm));
  t->split = reinterpret_cast<float*>(bp + up(b_rec) + up(b_box) + up(b_perm) + up(b_axis));

  BuildScratch w;
  st = build_scratch_alloc(plan, cp->dev, w, stream);
  if (st != KDT_OK) {
    (void)hipFreeAsync(block, stream);
    delete t;
    return st;
  }
  BuildOut o{t->rec, t->box, t->perm, t->axis, t->split};
  st = build_launch(plan, cp->dev, d_pts, w, o, 0, stream);
  if (st == KDT_OK && check == 2) {
    // deferred: the flag moves into the tree, kdt_tree_check reads it later
    t->flag = reinterpret_cast<int32_t*>(bp + up(b_rec) + up(b_box) + up(b_perm) + up(b_axis) +
                                         up(b_split));
    if (hipMemcpyAsync(t->flag, w.bad, sizeof(int32_t), hipMemcpyDeviceToDevice, stream) !=
        hipSuccess) {
      kdt_set_error("kdt_build: keeping the input check failed");
      st = KDT_EDEVICE;
    }
  } else if (st == KDT_OK && check) {
    int32_t bad = 0;
    if (hipMemcpyAsync(&bad, w.bad, sizeof(bad), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      kdt_set_error("kdt_build: reading the input check failed");
      st = KDT_EDEVICE;
    } else if (bad) {
      kdt_set_error("kdt_build: the points contain NaN or infinite coordinates");
      st = KDT_EINVAL;
    }
  }
  if (st == KDT_OK) st = build_launch(plan, cp->dev, d_pts, w, o, 1, stream);
  build_scratch_free(w, stream);
  if (st != KDT_OK) {
    (void)hipFreeAsync(block, stream);
    delete t;
    return st;
  }
  *out = t;
  return KDT_OK;
}

extern "C" kdt_status kdt_free(kdt_tree* tree) {
  kdt_clear_error();
  if (!tree) return KDT_OK;
  hipError_t e = hipStreamSynchronize(tree->stream);
  if (tree->rec) (void)hipFreeAsync(tree->rec, tree->stream);
  if (tree->f64_block) (void)hipFreeAsync(tree->f64_block, tree->stream);
  delete tree;
  if (e != hipSuccess) {
    kdt_set_error("kdt_free: waiting for the tree's stream failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_tree_check(const kdt_tree* tree, hipStream_t stream) {
  kdt_clear_error();
  if (!tree) {
    kdt_set_error("kdt_tree_check: NULL tree");
    return KDT_EINVAL;
  }
  if (!tree->flag) return KDT_OK;  // checked while building, or not asked for
  int32_t bad = 0;
  if (hipMemcpyAsync(&bad, tree->flag, sizeof(bad), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_tree_check: reading the input check failed");
    return KDT_EDEVICE;
  }
  if (bad) {
    kdt_set_error("kdt_tree_check: the points contain NaN or infinite coordinates");
    return KDT_EINVAL;
  }
  return KDT_OK;
}

namespace {
// Rows of W 4-byte elements (W = 0: the runtime width w) between input and
// tree order: gather out[t] = in[perm[t]], scatter out[perm[t]] = in[t].  One
// thread per element, consecutive threads on consecutive tree-order
// elements, so the tree-order side is read or written as whole lines.
template <int W, bool SCATTER>
__global__ void k_tree_permute(const int32_t* __restrict__ perm, int64_t n, int w,
                               const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  const int64_t width = W > 0 ? W : w;
  const int64_t total = n * width;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += step) {
    const int64_t t = e / width, c = e - t * width;
    const int64_t i = perm[t];
    if (SCATTER)
      out[i * width + c] = in[e];
    else
      out[e] = in[i * width + c];
  }
}

kdt_status tree_permute(const kdt_tree* tree, const void* d_in, int32_t width, void* d_out,
                        hipStream_t stream, bool scatter, const char* who) {
  if (!tree || width < 1 || width > 4096 || (tree->n > 0 && (!d_in || !d_out)) ||
      (tree->n > 0 && d_in == d_out)) {
    kdt_set_error("%s: NULL tree or arrays, width outside [1, 4096], or in == out", who);
    return KDT_EINVAL;
  }
  if (tree->n == 0) return KDT_OK;
  const int64_t total = tree->n * (int64_t)width;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  const auto* in = static_cast<const uint32_t*>(d_in);
  auto* out = static_cast<uint32_t*>(d_out);
#define KDT_PERMUTE(WW)                                                                  \
  (scatter ? (k_tree_permute<WW, true><<<grid, 256, 0, stream>>>(tree->perm, tree->n, width, \
                                                                 in, out))               \
           : (k_tree_permute<WW, false><<<grid, 256, 0, stream>>>(tree->perm, tree->n, width, \
                                                                  in, out)))
  if (width == 1)
    KDT_PERMUTE(1);
  else if (width == 3)
    KDT_PERMUTE(3);
  else
    KDT_PERMUTE(0);
#undef KDT_PERMUTE
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("%s: kernel launch failed", who);
    return KDT_EDEVICE;
  }
  return KDT_OK;
}
}  // namespace

extern "C" kdt_status kdt_tree_gather(const kdt_tree* tree, const void* d_in, int32_t width,
                                      void* d_out, hipStream_t stream) {
  kdt_clear_error();
  return tree_permute(tree, d_in, width, d_out, stream, false, "kdt_tree_gather");
}

extern "C" kdt_status kdt_tree_scatter(const kdt_tree* tree, const void* d_in, int32_t width,
                                       void* d_out, hipStream_t stream) {
  kdt_clear_error();
  return tree_permute(tree, d_in, width, d_out, stream, true, "kdt_tree_scatter");
}

extern "C" kdt_status kdt_tree_get_info(const kdt_tree* tree, kdt_tree_info* info) {
  kdt_clear_error();
  if (!tree || !info) {
    kdt_set_error("kdt_tree_get_info: NULL argument");
    return KDT_EINVAL;
  }
  info->n = tree->n;
  info->d = tree->d;
  info->leaf_size = tree->leaf;
  info->levels = tree->levels;
  info->stride = tree->stride;
  info->n_nodes = tree->n_nodes;
  return KDT_OK;
}

extern "C" const int32_t* kdt_tree_perm(const kdt_tree* tree) { return tree ? tree->perm : nullptr; }

extern "C" kdt_status kdt_tree_nodes(const kdt_tree* tree, int32_t* h_left, int32_t* h_begin,
                                     int32_t* h_end, int32_t* h_level, hipStream_t stream) {
  kdt_clear_error();
  if (!tree) {
    kdt_set_error("kdt_tree_nodes: NULL tree");
    return KDT_EINVAL;
  }
  const int64_t m = tree->n_nodes;
  std::vector<int4> rec((size_t)m);
  if (tree->nodes) {
    hipError_t e = hipMemcpyAsync(rec.data(), tree->nodes, sizeof(int4) * (size_t)m,
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      kdt_set_error("kdt_tree_nodes: copy failed: %s", hipGetErrorString(e));
      return KDT_EDEVICE;
    }
  } else {
    // the implicit median layout, written out
    for (int64_t v = 0; v < m; ++v) {
      int lev = 0;
      while ((int64_t(2) << lev) - 1 <= v) ++lev;
      const int64_t j = v - ((int64_t(1) << lev) - 1);
      const bool leaf = lev == tree->levels;
      rec[(size_t)v] = make_int4(leaf ? -1 : (int)(2 * v + 1), (int)node_begin(tree->n, lev, j),
                                 (int)node_begin(tree->n, lev, j + 1), lev);
    }
  }
  for (int64_t v = 0; v < m; ++v) {
    if (h_left) h_left[v] = rec[(size_t)v].x;
    if (h_begin) h_begin[v] = rec[(size_t)v].y;
    if (h_end) h_end[v] = rec[(size_t)v].z;
    if (h_level) h_level[v] = rec[(size_t)v].w;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_tree_export(const kdt_tree* tree, float* h_pts, int32_t* h_perm,
                                      float* h_lo, float* h_hi, int32_t* h_axis, float* h_split,
                                      hipStream_t stream) {
  kdt_clear_error();
  if (!tree) {
    kdt_set_error("kdt_tree_export: NULL tree");
    return KDT_EINVAL;
  }
  const int d = tree->d, S = tree->stride, P = pad4(d);
  std::vector<float> rec((size_t)tree->n * S);
  std::vector<float> box((size_t)tree->n_nodes * 2 * P);
  hipError_t e = hipMemcpyAsync(rec.data(), tree->rec, sizeof(float) * rec.size(),
                                hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(box.data(), tree->box, sizeof(float) * box.size(), hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess && h_perm)
    e = hipMemcpyAsync(h_perm, tree->perm, sizeof(int32_t) * tree->n, hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess && h_axis)
    e = hipMemcpyAsync(h_axis, tree->axis, sizeof(int32_t) * tree->n_nodes,
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && h_split)
    e = hipMemcpyAsync(h_split, tree->split, sizeof(float) * tree->n_nodes,
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    kdt_set_error("kdt_tree_export: copy failed: %s", hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  for (int64_t i = 0; h_pts && i < tree->n; ++i)
    for (int a = 0; a < d; ++a) h_pts[i * d + a] = rec[(size_t)i * S + a];
  for (int64_t v = 0; v < tree->n_nodes; ++v)
    for (int a = 0; a < d; ++a) {
      if (h_lo) h_lo[v * d + a] = box[(size_t)v * 2 * P + a];
      if (h_hi) h_hi[v * d + a] = box[(size_t)v * 2 * P + P + a];
    }
  return KDT_OK;
}

extern "C" kdt_status kdt_debug_fail_alloc(int64_t after) {
  kdt_clear_error();
  g_fail_after.store(after > 0 ? after : -1);
  return KDT_OK;
}

extern "C" kdt_status kdt_debug_visits(uint64_t* h_counts, int32_t reset) {
  kdt_clear_error();
  unsigned long long* d = visit_counters();
  if (!d) {
    kdt_set_error("kdt_debug_visits: this library was built without work counters");
    return KDT_EUNSUPPORTED;
  }
  unsigned long long h[kVisitSlots * kVisitShards];
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
      (reset && hipMemset(d, 0, sizeof(h)) != hipSuccess)) {
    kdt_set_error("kdt_debug_visits: reading the counters failed");
    return KDT_EDEVICE;
  }
  if (h_counts)
    for (int s = 0; s < kVisitSlots; ++s) {
      uint64_t sum = 0;
      for (int k = 0; k < kVisitShards; ++k) sum += h[s * kVisitShards + k];
      h_counts[s] = sum;
    }
  return KDT_OK;
}

namespace {
// Eight independent multiply-add chains per lane (each a separate multiply and
// add: the library is built without contraction or packed float32): a kernel
// that does nothing but issue VALU instructions, for calibrating the VALU
// issue rate that the counters of the other kernels are read against.
__global__ __launch_bounds__(256) void k_valu_probe(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = (float)(threadIdx.x + j) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = a[j] * 0.9999f + 1e-4f;
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  if (s == 12345.678f) out[blockIdx.x] = s;  // keeps the chains live; never true
}
}  // namespace

extern "C" kdt_status kdt_debug_valu_probe(float* d_out, int32_t blocks, int32_t iters,
                                           hipStream_t stream) {
  kdt_clear_error();
  if (!d_out || blocks < 1 || iters < 1) {
    kdt_set_error("kdt_debug_valu_probe: NULL output or non-positive size");
    return KDT_EINVAL;
  }
  k_valu_probe<<<blocks, 256, 0, stream>>>(d_out, iters);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_debug_valu_probe: launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}
