/*
 * kdt_debug.h -- test and measurement hooks of the k-d tree library.  Not
 * for production use; every call is cheap and allocates nothing.
 */
#ifndef KDT_DEBUG_H
#define KDT_DEBUG_H

#include "kdt.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Makes the `after`-th next device allocation of the library (counting
 * from 1, process-wide) fail as if the device were out of memory, so that
 * tests can check the KDT_ENOMEM paths; after <= 0 disarms the hook.
 * Allocations of batched plans (plain hipMalloc at plan creation) are not
 * covered.
 */
kdt_status kdt_debug_fail_alloc(int64_t after);

/*
 * Work counters of the instrumented build of the library (compiled with
 * KDT_COUNT_VISITS; the product build returns KDT_EUNSUPPORTED): waits for
 * the device, then writes 8 uint64 totals to h_counts (host, may be NULL)
 * and zeroes the counters if `reset`.  Slots: 0 nodes visited (node boxes
 * tested) and 1 leaf point records scanned by the traversals with one query
 * per lane, 2 records read again to insert a kNN candidate, 3 node boxes and
 * 4 leaf points read by the wave-shared traversals (once per wave), 5 boxes
 * read again when a node leaves a per-lane stack; 6-7 unused.  They give the traversal term of the algorithmic bytes of a call:
 * points x record bytes + nodes x box bytes.
 */
kdt_status kdt_debug_visits(uint64_t *h_counts, int32_t reset);

/*
 * Launches a kernel of `blocks` workgroups of 256 threads that only issues
 * VALU instructions (eight independent multiply-add chains per lane, `iters`
 * rounds, 16 float32 instructions per round), asynchronously on `stream`.
 * Profiled with the same counters as the library's kernels, it gives the
 * chip's VALU issue rate that their instruction counts are read against.
 * d_out [blocks] float32 (device) is never written in practice.
 */
kdt_status kdt_debug_valu_probe(float *d_out, int32_t blocks, int32_t iters,
                                hipStream_t stream);

/*
 * The library's radix sort (the one that orders queries): sorts n pairs
 * (d_keys [n] uint32, d_vals [n] int32, device, in place) by the key bits
 * [begin_bit, end_bit), stably, asynchronously on `stream`.  For testing the
 * sort against a reference.  Errors: KDT_EINVAL, KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_debug_radix_sort(uint32_t *d_keys, int32_t *d_vals, int64_t n, int32_t begin_bit,
                                int32_t end_bit, hipStream_t stream);

/*
 * Exclusive running sum of the n int32 values d_in (device) into d_out
 * (device), the library's scan of the CSR list offsets and of the sliding
 * midpoint build's ranks.  out_bits = 64: d_out holds n + 1 int64 values,
 * the last the total; out_bits = 32: d_out holds n int32 values (NULL
 * allowed when n = 0; sums below 2^31 assumed).  Asynchronous on `stream`.
 * For testing the scan against a reference.  Errors: KDT_EINVAL,
 * KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_debug_exclusive_scan(const int32_t *d_in, void *d_out, int64_t n, int32_t out_bits,
                                    hipStream_t stream);

/*
 * Sorts every row of a CSR list ascending, as the ball and box lists are:
 * row r of d_in [total] int32 (device) is [d_off[r], d_off[r + 1]) (d_off
 * [nq + 1] int64, device, d_off[nq] = total) and goes to the same range of
 * d_out (not d_in).  Waits on `stream`.  For testing the row sort against a
 * reference.  Errors: KDT_EINVAL, KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_debug_sort_rows(const int32_t *d_in, int32_t *d_out, const int64_t *d_off,
                               int64_t nq, int64_t total, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* KDT_DEBUG_H */
