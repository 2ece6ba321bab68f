// kdt_internal.h -- shared device helpers and host-side structures of the
// HIP k-d tree library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "kdt.h"

namespace kdt {

constexpr int kWave = 64;

// Floats per node bounding-box half (lo or hi), padded so a node's box is
// two aligned runs of float4.
__host__ __device__ constexpr int pad4(int d) { return (d + 3) & ~3; }
// Floats per tree-ordered point record: d coordinates, then the original index
// (int32 bits), padded to a multiple of 4 so records load as float4.
__host__ __device__ constexpr int rec_stride(int d) { return (d + 1 + 3) & ~3; }

// Order-preserving map of float32 onto uint32 (total order; -0 sorts below +0).
__device__ __forceinline__ uint32_t fkey(float f) {
  uint32_t b = __float_as_uint(f);
  return b ^ ((b & 0x80000000u) ? 0xFFFFFFFFu : 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(uint32_t u) {
  uint32_t b = u ^ ((u & 0x80000000u) ? 0x80000000u : 0xFFFFFFFFu);
  return __uint_as_float(b);
}

// Point range [begin, end) of node (level, j) of a balanced tree over n points.
__host__ __device__ __forceinline__ int64_t node_begin(int64_t n, int level, int64_t j) {
  return (j * n) >> level;
}

// Level of heap node id v (root 0, children 2v+1, 2v+2).
__device__ __forceinline__ int node_level(uint32_t v) { return 31 - __clz(v + 1); }

// Memory-model helpers for data written by other workgroups in the same launch.
__device__ __forceinline__ uint32_t ld_acquire_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_agent_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Orders LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups are handed to the 8 XCDs round robin (workgroup b to XCD b % 8),
// and each XCD has its own L2.  Kernels whose neighbouring workgroups touch
// the same data (queries sorted along the tree) renumber themselves so that
// runs of R consecutive logical workgroups go to one XCD: neighbours then
// share an L2, while work that varies in space still spreads over all XCDs
// every 8 R workgroups.  R = 0 gives each XCD one contiguous eighth of the
// grid.  A bijection of [0, gridDim.x) for any grid size.
template <int R>
__device__ __forceinline__ int64_t xcd_block() {
  constexpr int64_t kXcd = 8;
  const int64_t g = gridDim.x, b = blockIdx.x;
  const int64_t span = R > 0 ? kXcd * R : g;
  const int64_t base = b / span * span, r = b - base;
  const int64_t size = g - base < span ? g - base : span;
  const int64_t per = size / kXcd, rem = size % kXcd, x = r % kXcd;
  return base + x * per + (x < rem ? x : rem) + r / kXcd;
}

// Run lengths per kernel family, measured on 2^24 clustered points (R = 1 is
// the plain round robin).  Per-lane kNN gains most from whole eighths
// (9.4 -> 8.3 ms for 2^22 queries, 26.3 -> 21.6 ms for all points, k = 32);
// grouping, whose cost is concentrated in the halos, balances better with
// runs of 16 (19.5 -> 18.4 ms; whole eighths: 27 ms); wave-packet ball
// counts gain nothing.
constexpr int kXcdRunLane = 0;    // per-lane kNN and ball queries
constexpr int kXcdRunPacket = 1;  // wave-packet kNN and ball queries
constexpr int kXcdRunFof = 16;    // grouping
constexpr int kXcdRunP2M = 64;    // particle passes of the deposit and its adjoint

// Number of set lanes of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// ---------------------------------------------------------------------------
// Host-side structures
// ---------------------------------------------------------------------------

// One tree of a forest (a single tree is a forest of one set).
struct SetDesc {
  int64_t off;        // first row of the set in the concatenated point array
  int64_t n;          // points in the set
  int64_t node_base;  // first node id of the set
  int32_t levels;     // L
  int32_t glevels;    // levels split by the multi-workgroup path
};

// A node split by the multi-workgroup path at one level.
struct SegEntry {
  int64_t b, e, m;      // global rows [b, e), first right row m
  int64_t node;         // global node id
  int64_t child;        // global node id of the left child (right = child + 1)
  int32_t first_chunk;  // chunk ids [first_chunk, first_chunk + n_chunks)
  int32_t n_chunks;
  // Where the partial boxes of this node's points were left: the root pass
  // chunks [src_first, src_first + src_count) (src_side < 0) or the chunks of
  // the parent at the previous level, left (0) or right (1) side.
  int32_t src_first;
  int32_t src_count;
  int32_t src_side;
  int32_t pad;
};

struct ChunkEntry {
  int64_t b, e;  // rows
  int32_t seg;   // segment index within the level (or set index for the root pass)
  int32_t sole;  // 1 when the chunk is its segment's only one
};

// A node finished inside one workgroup's LDS, with its whole subtree.
struct SubEntry {
  int64_t j;      // index of the node within its level
  int32_t set;
  int32_t level;
};

// Selection state of one segment during the radix-select passes.
struct SegState {
  uint32_t prefix;   // resolved high bits of the pivot key
  int32_t rank;      // rank of the pivot among the keys that match prefix
  int32_t hb;        // highest unresolved bit, -1 when the pivot is known
  int32_t axis;
  int32_t n_eq_left; // keys equal to the pivot that go left
  int32_t pad[3];
};

struct Plan {
  int d = 0, leaf = 0;
  int64_t total = 0;
  std::vector<SetDesc> sets;
  int64_t n_nodes = 0;
  int n_glevels = 0;
  // per global level: segment and chunk tables
  std::vector<std::vector<SegEntry>> segs;
  std::vector<std::vector<ChunkEntry>> chunks;
  std::vector<ChunkEntry> root_chunks;  // seg field = set index
  std::vector<char> multi_chunk;        // per global level: some node owns several chunks
  std::vector<SubEntry> subs;
  int lds_cap = 0;  // largest node finished in LDS
  int sub_max = 1;  // largest node that is finished in LDS in this plan
};

// Builds the static schedule of a forest from host-known sizes.
// leaves: N_leaf of each set (n_sets entries); plan.leaf is the largest.
bool make_plan(const int64_t* offsets, int n_sets, int d, const int* leaves, Plan& plan,
               std::string& err);

int levels_for(int64_t n, int leaf);

// Stable LSD radix sort of (key, value) pairs on key bits [begin_bit, end_bit)
// (kdt_sort.hip), 8 bits per pass, ping-ponging between keys[0]/keys[1] and
// vals[0]/vals[1] (input in [0]); returns the index of the pair of arrays
// holding the result.  scratch: radix_sort_scratch_bytes(n) device bytes.
size_t radix_sort_scratch_bytes(int64_t n);
int radix_sort_pairs(uint32_t* keys[2], int32_t* vals[2], int64_t n, int begin_bit, int end_bit,
                     void* scratch, hipStream_t stream);

// Exclusive running sum of n int32 values into out (kdt_sort.hip), 64-bit
// sums; the total is written to *total_at (device) when total_at is not
// NULL (for CSR offsets: total_at = out + n).  scratch: scan_scratch_bytes(n)
// device bytes.
size_t scan_scratch_bytes(int64_t n);
template <typename Out>
kdt_status exclusive_scan(const int32_t* in, Out* out, int64_t n, int64_t* total_at,
                          void* scratch, hipStream_t stream);

// Sorts every row of a CSR list ascending (kdt_rowsort.hip): row r is
// in[off[r], off[r + 1]) and goes to the same range of out (in != out; off
// device, nq + 1 entries, total = off[nq]; every entry in [0, key_limit)).
// Scratch from the stream-ordered pool; waits on `stream` once, twice when
// rows above 16384 entries occur.  KDT_ENOMEM, KDT_EUNSUPPORTED (total
// above 2^31 - 1), KDT_EDEVICE, with the error set.
kdt_status sort_list_rows(const int32_t* in, int32_t* out, const int64_t* off, int64_t nq,
                          int64_t total, int64_t key_limit, hipStream_t stream);

// *out (device) <- the number of i in [0, n) with labels[i] == i: the groups
// of a friends-of-friends labelling (kdt_sort.hip).  scratch:
// scan_scratch_bytes(n) device bytes.
kdt_status count_roots(const int32_t* labels, int64_t n, int64_t* out, void* scratch,
                       hipStream_t stream);

// The tuning table (kdt_tuning.hip): N_leaf and queries per traversal (1 or
// 64) measured fastest for the nearest shape of dimension d.
struct Tuning {
  int leaf;
  int qpw;
};
Tuning tuned(int d, int64_t n, int k);
int lds_capacity(int d);

// Device copies of a plan's tables (one allocation).
struct PlanDev {
  SetDesc* sets = nullptr;
  ChunkEntry* root_chunks = nullptr;
  std::vector<SegEntry*> segs;
  std::vector<ChunkEntry*> chunks;
  SubEntry* subs = nullptr;
  void* block = nullptr;
  size_t max_segs = 0, max_chunks = 0;
};

// Scratch of one build (stream-ordered allocations).
struct BuildScratch {
  float* x[2] = {nullptr, nullptr};
  int32_t* p[2] = {nullptr, nullptr};
  uint32_t* pbox = nullptr;   // partial boxes of the root pass, [root chunk][2][d]
  uint32_t* cbox = nullptr;   // partial child boxes, [chunk][side][2][d]
  SegState* st = nullptr;
  uint32_t* chist = nullptr;  // per-chunk digit histograms, [chunk][256]
  int32_t* cnt = nullptr;     // per-chunk (below, equal) pivot counts
  int32_t* bad = nullptr;
};

// Where a build writes the tree.
struct BuildOut {
  float* rec;
  float* box;
  int32_t* perm;
  int32_t* axis;
  float* split;
};

kdt_status plan_upload(const Plan& p, PlanDev& pd, hipStream_t stream);
void plan_release(PlanDev& pd);
// Passing kPlainAlloc as the stream allocates with hipMalloc instead of the
// stream-ordered pool (used by batch plans, whose buffers live in a graph).
static const hipStream_t kPlainAlloc = reinterpret_cast<hipStream_t>(~uintptr_t(0));
kdt_status build_scratch_alloc(const Plan& p, const PlanDev& pd, BuildScratch& w,
                               hipStream_t stream);
// Sets kernel attributes once (must run outside any graph capture).
void build_init_once();
void build_scratch_free(BuildScratch& w, hipStream_t stream);
// phase 0: ingest and root boxes; phase 1: everything after.
kdt_status build_launch(const Plan& p, const PlanDev& pd, const float* d_pts,
                        const BuildScratch& w, const BuildOut& o, int phase, hipStream_t stream);
// Stream-ordered device allocation from the default pool (kept cached).
// Fails on purpose when the allocation-failure hook (kdt_debug_fail_alloc)
// says so.
hipError_t dev_alloc(void** ptr, size_t bytes, hipStream_t stream);
// True if the allocation-failure hook wants this allocation to fail.
bool alloc_should_fail();
// The device counters of the instrumented build (KDT_COUNT_VISITS), else
// NULL; traversal views carry them.
unsigned long long* visit_counters();

// Scratch that an entry point keeps on its stream from one call to the next:
// slot `slot` of (current device, stream) holds at least `bytes` bytes,
// grown (stream-ordered free and allocation) when a call needs more, never
// shrunk, held until the process ends.  The deposit uses it: its host part
// waits on the stream anyway, and freeing its large buffers back to the
// pool on every call cost milliseconds of host time.  Calls that share a
// stream must not run their host parts concurrently (they already share the
// stream's order).  NULL if the allocation fails.
void* stream_scratch(hipStream_t stream, int slot, size_t bytes);

// Stream-ordered scratch buffers of one call, released in stream order when
// the holder goes out of scope -- on every return path, errors included.
class PoolBuffers {
 public:
  explicit PoolBuffers(hipStream_t s) : stream_(s) {}
  PoolBuffers(const PoolBuffers&) = delete;
  PoolBuffers& operator=(const PoolBuffers&) = delete;
  ~PoolBuffers() { release(); }
  // Returns every held buffer to the pool now, in stream order (work queued
  // before this call still sees them).  A call that waits on its stream at
  // the end releases first: a free can block the host for milliseconds, and
  // queued behind the stream's work it costs no GPU time.
  void release() {
    for (void*& q : held_)
      if (q) {
        (void)hipFreeAsync(q, stream_);
        q = nullptr;
      }
  }
  // count elements of T (at least one); false if the pool is exhausted
  template <typename T>
  bool get(T** p, size_t count) {
    void* q = nullptr;
    if (dev_alloc(&q, (count > 0 ? count : 1) * sizeof(T), stream_) != hipSuccess) return false;
    held_.push_back(q);
    *p = static_cast<T*>(q);
    return true;
  }
  // Hands a buffer over to the caller: it is no longer released here.
  void keep(const void* p) {
    for (void*& q : held_)
      if (q == p) q = nullptr;
  }

 private:
  hipStream_t stream_;
  std::vector<void*> held_;
};

}  // namespace kdt

// Library-owned tree.
struct kdt_tree {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int d = 0, leaf = 0, levels = 0, stride = 0;
  int64_t n_nodes = 0;
  float* rec = nullptr;      // [n][stride]
  float* box = nullptr;      // [n_nodes][2 * pad4(d)]
  int32_t* perm = nullptr;   // [n]
  int32_t* axis = nullptr;   // [n_nodes]
  float* split = nullptr;    // [n_nodes]
  // sliding-midpoint trees (split_rule 1): [n_nodes] (left child or -1, first
  // point, end point, level), nodes numbered level by level; NULL for the
  // implicit median layout
  int4* nodes = nullptr;
  // float64 trees (kdt_build_f64): coordinates in tree order [n][d] and the
  // tight float64 node boxes [n_nodes][2][d], one allocation (f64_block);
  // NULL for float32 trees
  double* rec64 = nullptr;
  double* box64 = nullptr;
  void* f64_block = nullptr;
  // deferred finiteness check (check_finite 2): nonzero if a coordinate was
  // NaN or infinite; inside the tree's allocation.  NULL otherwise.
  int32_t* flag = nullptr;
};

namespace kdt {
// The sliding-midpoint build (Sec. 2.1); fills t (levels, n_nodes and the
// arrays, one allocation starting at t->rec) from d_pts [n][d].
kdt_status build_midpoint(const float* d_pts, int64_t n, int d, int leaf, bool check,
                          hipStream_t stream, kdt_tree* t);
}  // namespace kdt

// Error reporting shared by every entry point.
void kdt_set_error(const char* fmt, ...);
void kdt_clear_error();

// The float32 query entry points refuse a tree built from float64
// coordinates (its float32 copy only steers the shape): true (and the error
// set) if t is one.
inline bool refuse_f64(const kdt_tree* t, const char* who) {
  if (t && t->rec64) {
    kdt_set_error("%s: the tree holds float64 coordinates; use the _f64 entry points", who);
    return true;
  }
  return false;
}

// The rows of self queries (d_q NULL).  opts->tree_rows 0: row i belongs to
// input point i; 1: row t belongs to the tree's t-th point (tree order).
// The query kernels take, for self queries, a non-NULL order argument as the
// request for tree-order rows (it is never read): *rows gets t->perm then,
// else NULL.  KDT_EINVAL (error set) for another value, or tree_rows with
// external queries.
inline kdt_status self_rows(const kdt_tree* t, const void* d_q, const kdt_query_opts* opts,
                            const char* who, const int32_t** rows) {
  const int32_t tr = opts ? opts->tree_rows : 0;
  *rows = nullptr;
  if (tr != 0 && tr != 1) {
    kdt_set_error("%s: tree_rows must be 0 or 1", who);
    return KDT_EINVAL;
  }
  if (tr && d_q) {
    kdt_set_error("%s: tree_rows applies to self queries (NULL queries) only", who);
    return KDT_EINVAL;
  }
  if (tr) *rows = t->perm;
  return KDT_OK;
}

// Entry points whose kernels use the median tree's implicit layout refuse a
// sliding-midpoint tree: true (and the error set) if t is one.
inline bool refuse_stored(const kdt_tree* t, const char* who) {
  if (t && t->nodes) {
    kdt_set_error("%s: not available on a sliding-midpoint tree (split_rule 1)", who);
    return true;
  }
  return false;
}
