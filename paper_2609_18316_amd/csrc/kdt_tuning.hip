// The tuning table behind leaf_size = 0 and traversal = 0: for a workload
// shape (dimension, number of points, k) the leaf size N_leaf and the number
// of queries a traversal serves (1: one per lane, 64: one shared by a wave)
// that the autotuner measured fastest.  The paper tunes N_leaf by hand
// (Sec. 2.1 and App. A: the best value moves with N and D); here the choice is
// measured on the GPU by paper_2609_18316_amd/autotune.py, compiled in from
// the table that tool writes (kdt_tuning.inc), and can be replaced at run time
// through kdt_tuning_set with values measured in the calling process.
//
// A lookup takes the entry of the same dimension nearest in (log2 n, log2 k):
// one step of log2 n counts as much as one step of log2 k; ties go to the
// run-time entry, then to the earlier compiled-in one.  A dimension with no
// entry gets leaf 32 and one query per lane up to d = 8, wave packets above.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "kdt.h"
#include "kdt_internal.h"

namespace kdt {
namespace {

struct TuneEntry {
  int d;
  int log2n;  // log2 of the point count, rounded
  int k;
  int leaf;
  int qpw;    // queries per traversal: 1 or 64
};

const TuneEntry kBuiltin[] = {
#include "kdt_tuning.inc"
};

std::mutex g_mu;
std::map<std::tuple<int, int, int>, TuneEntry>* g_runtime = new std::map<std::tuple<int, int, int>, TuneEntry>();

int log2_round(int64_t n) { return (int)std::lround(std::log2((double)std::max<int64_t>(n, 1))); }

double distance(const TuneEntry& e, int log2n, int k) {
  return std::fabs((double)(e.log2n - log2n)) +
         std::fabs(std::log2((double)std::max(e.k, 1)) - std::log2((double)std::max(k, 1)));
}

}  // namespace

Tuning tuned(int d, int64_t n, int k) {
  const int l2 = log2_round(n);
  const TuneEntry* best = nullptr;
  double bd = 0.0;
  TuneEntry rt{};
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& kv : *g_runtime) {
      const TuneEntry& e = kv.second;
      if (e.d != d) continue;
      const double dist = distance(e, l2, k);
      if (!best || dist < bd) {
        rt = e;
        best = &rt;
        bd = dist;
      }
    }
  }
  for (const TuneEntry& e : kBuiltin) {
    if (e.d != d) continue;
    const double dist = distance(e, l2, k);
    if (!best || dist < bd) {
      best = &e;
      bd = dist;
    }
  }
  if (!best) return Tuning{32, d <= 8 ? 1 : 64};
  return Tuning{best->leaf, best->qpw};
}

}  // namespace kdt

using kdt::Tuning;

extern "C" kdt_status kdt_tuning_set(int32_t d, int64_t n, int32_t k, int32_t leaf_size,
                                     int32_t queries_per_wave) {
  kdt_clear_error();
  const bool erase = leaf_size == 0 && queries_per_wave == 0;
  if ((d != 2 && d != 3 && d != 4 && d != 8 && d != 16) || n < 1 || k < 1 ||
      (!erase && (leaf_size < 2 || leaf_size > 256 ||
                  (queries_per_wave != 1 && queries_per_wave != 64)))) {
    kdt_set_error("kdt_tuning_set: d in {2,3,4,8,16}, n >= 1, k >= 1, leaf_size in [2, 256] "
                  "and queries_per_wave 1 or 64 are required");
    return KDT_EINVAL;
  }
  const int l2 = kdt::log2_round(n);
  std::lock_guard<std::mutex> lock(kdt::g_mu);
  if (erase)
    kdt::g_runtime->erase(std::make_tuple(d, l2, k));
  else
    (*kdt::g_runtime)[std::make_tuple(d, l2, k)] =
        kdt::TuneEntry{d, l2, k, leaf_size, queries_per_wave};
  return KDT_OK;
}

extern "C" kdt_status kdt_tuning_get(int32_t d, int64_t n, int32_t k, int32_t* leaf_size,
                                     int32_t* queries_per_wave, int32_t* stack_depth) {
  kdt_clear_error();
  if ((d != 2 && d != 3 && d != 4 && d != 8 && d != 16) || n < 1 || k < 1) {
    kdt_set_error("kdt_tuning_get: d in {2,3,4,8,16}, n >= 1 and k >= 1 are required");
    return KDT_EINVAL;
  }
  const Tuning t = kdt::tuned(d, n, k);
  if (leaf_size) *leaf_size = t.leaf;
  if (queries_per_wave) *queries_per_wave = t.qpw;
  if (stack_depth) *stack_depth = kdt::levels_for(n, t.leaf) + 1;
  return KDT_OK;
}
