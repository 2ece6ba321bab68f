// kdt_fof.hip -- friends-of-friends grouping (Sec. 4.1) on gfx950.
//
// Every point runs a ball query of radius l over the tree (in tree order, so
// the lanes of a wave search neighbouring space) and links itself to every
// friend at a later tree position (nodes that end at or before its own are
// never entered: the other end of each such pair links it) through a
// lock-free union-find: roots
// always hang under the smaller root (compare-and-swap), so the root of each
// component is its smallest input index.  Finding a root halves the path as
// it goes.  A final pass points every element at its root, which is the
// canonical group label.
#include <hip/hip_runtime.h>

#include "kdt_query.h"

namespace kdt {

constexpr int kFBlock = 128;

template <int D>
__global__ void k_fof_clique_mark(const float* __restrict__ box, int64_t n_nodes, float l2,
                                  uint32_t* __restrict__ conn) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n_nodes) fof_mark_clique<D>(box, v, l2, conn);
}

template <int D>
__global__ void k_fof_clique_join(TreeView t, int32_t* __restrict__ parent,
                                  const uint32_t* __restrict__ conn) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= t.n) return;
  constexpr int S = rec_stride(D);
  fof_join_clique<D>(t, s, __float_as_int(t.rec[s * S + D]), 0, parent, conn);
}

template <int D>
__global__ __launch_bounds__(kFBlock) void k_fof_link(TreeView t, float l2,
                                                      int32_t* __restrict__ parent,
                                                      uint32_t* __restrict__ conn) {
  __shared__ uint32_t stk[kMaxDepth][kFBlock];
  const int64_t s = xcd_block<kXcdRunFof>() * kFBlock + threadIdx.x;
  if (s >= t.n) return;
  float p[D];
  int32_t me = 0;
  load_rec<D>(t.rec, s, p, me);
  fof_point<D>(t, p, s, me, l2, 0, parent, conn, &stk[0][threadIdx.x], kFBlock);
}

// The same links over a sliding-midpoint tree: its depth is data-dependent,
// so the stack (levels + 2 entries per lane) is sized at launch.
template <int D>
__global__ __launch_bounds__(kFBlock) void k_fof_link_stored(TreeView t, float l2,
                                                             int32_t* __restrict__ parent,
                                                             uint32_t* __restrict__ conn) {
  extern __shared__ uint32_t stk_fof[];
  const int64_t s = xcd_block<kXcdRunFof>() * kFBlock + threadIdx.x;
  if (s >= t.n) return;
  float p[D];
  int32_t me = 0;
  load_rec<D>(t.rec, s, p, me);
  fof_point<D, StoredShape>(t, p, s, me, l2, 0, parent, conn, stk_fof + threadIdx.x, kFBlock);
}

__global__ void k_fill_conn(uint32_t* __restrict__ conn, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) conn[i] = 0u;
}

// Returns the status of the launches (the packet launch checks its own and
// clears the runtime's error, so it is passed on from here).
template <int D>
static kdt_status fof_launch(const TreeView& v, int leaf, int64_t n_nodes, float l2,
                             int32_t* labels, uint32_t* conn, hipStream_t stream) {
  const unsigned gn = (unsigned)((n_nodes + 255) / 256);
  const unsigned gp = (unsigned)((v.n + 255) / 256);
  const unsigned gl = (unsigned)((v.n + kFBlock - 1) / kFBlock);
  if (v.nodes) {
    // a sliding-midpoint tree: every friend pair is linked by the search (no
    // one-component node flags, which join through the implicit layout)
    k_fill_conn<<<gn, 256, 0, stream>>>(conn, n_nodes);
    const size_t smem = sizeof(uint32_t) * (size_t)(v.levels + 2) * kFBlock;
    k_fof_link_stored<D><<<gl, kFBlock, smem, stream>>>(v, l2, labels, conn);
    return KDT_OK;
  }
  k_fof_clique_mark<D><<<gn, 256, 0, stream>>>(v.box, n_nodes, l2, conn);
  k_fof_clique_join<D><<<gp, 256, 0, stream>>>(v, labels, conn);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_fof: clique kernel launch failed");
    return KDT_EDEVICE;
  }
  if (leaf <= 64) return fof_packet_launch<D>(v, leaf, l2, labels, conn, stream);
  k_fof_link<D><<<gl, kFBlock, 0, stream>>>(v, l2, labels, conn);
  return KDT_OK;
}

__global__ void k_fof_init(int32_t* __restrict__ parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) parent[i] = (int32_t)i;
}

// Points every element at its root.  No path shortcuts here: each element is
// written by its own lane only, so no lane can overwrite a finished label with
// an intermediate ancestor.
__global__ void k_fof_final(int32_t* __restrict__ parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    uf_st(parent + i, uf_root(parent, (int32_t)i));
  }
}

static TreeView view_of(const kdt_tree* t) {
  TreeView v;
  v.rec = t->rec;
  v.box = t->box;
  v.n = t->n;
  v.levels = t->levels;
  v.nodes = t->nodes;
  return v;
}

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_fof(const kdt_tree* tree, float l, int32_t* d_labels, int64_t* n_groups,
                              hipStream_t stream) {
  kdt_clear_error();
  if (refuse_f64(tree, "kdt_fof")) return KDT_EUNSUPPORTED;
  if (!tree || !d_labels || !(l >= 0.0f) || !std::isfinite(l)) {
    kdt_set_error("kdt_fof: NULL tree or labels, or linking length not finite and >= 0");
    return KDT_EINVAL;
  }
  const int64_t n = tree->n;
  const unsigned g = (unsigned)((n + 255) / 256);
  k_fof_init<<<g, 256, 0, stream>>>(d_labels, n);
  const TreeView v = view_of(tree);
  const float l2 = l * l;
  uint32_t* conn = nullptr;
  if (dev_alloc((void**)&conn, sizeof(uint32_t) * tree->n_nodes, stream) != hipSuccess) {
    kdt_set_error("kdt_fof: device allocation failed");
    return KDT_ENOMEM;
  }
  kdt_status st = KDT_OK;
  switch (tree->d) {
    case 2: st = fof_launch<2>(v, tree->leaf, tree->n_nodes, l2, d_labels, conn, stream); break;
    case 3: st = fof_launch<3>(v, tree->leaf, tree->n_nodes, l2, d_labels, conn, stream); break;
    case 4: st = fof_launch<4>(v, tree->leaf, tree->n_nodes, l2, d_labels, conn, stream); break;
    case 8: st = fof_launch<8>(v, tree->leaf, tree->n_nodes, l2, d_labels, conn, stream); break;
    case 16: st = fof_launch<16>(v, tree->leaf, tree->n_nodes, l2, d_labels, conn, stream); break;
    default:
      (void)hipFreeAsync(conn, stream);
      kdt_set_error("kdt_fof: unsupported dimension %d", tree->d);
      return KDT_EUNSUPPORTED;
  }
  (void)hipFreeAsync(conn, stream);
  if (st != KDT_OK) return st;
  k_fof_final<<<g, 256, 0, stream>>>(d_labels, n);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_fof: kernel launch failed");
    return KDT_EDEVICE;
  }
  if (n_groups) {
    PoolBuffers buf(stream);
    int64_t* d_out = nullptr;
    char* tmp = nullptr;
    if (!buf.get(&d_out, 1) || !buf.get(&tmp, scan_scratch_bytes(n))) {
      kdt_set_error("kdt_fof: device allocation failed");
      return KDT_ENOMEM;
    }
    int64_t h = 0;
    if (count_roots(d_labels, n, d_out, tmp, stream) != KDT_OK ||
        hipMemcpyAsync(&h, d_out, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      kdt_set_error("kdt_fof: counting groups failed");
      return KDT_EDEVICE;
    }
    *n_groups = h;
  }
  return KDT_OK;
}
