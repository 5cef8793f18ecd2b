/*
 * cc_bench.h -- memory-system microbenchmarks that give the roofline
 * denominators for the connectivity kernels of cc.h.
 *
 * Bulk-Update and Bulk-Query are random-access bound: per edge they stream
 * 8 bytes of ids and chase parent pointers, i.e. random 4-byte reads of the
 * parent array (Section 4: each edge needs a find on both endpoints).  These
 * kernels measure what the device can do for each ingredient in isolation,
 * so that a connectivity kernel's throughput can be stated as a fraction of
 * a measured bound rather than of a datasheet figure.  They are not part of
 * the connectivity method.
 *
 * All calls are asynchronous on `stream` (a hipStream_t, NULL = null stream);
 * the caller times them (e.g. with events on the same stream).  All pointers
 * are DEVICE pointers owned by the caller.  Return 0 on success, -1 for a
 * bad argument (nothing enqueued), -4 if the launch failed.
 */
#ifndef CC_BENCH_H
#define CC_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random gathers: `count` reads table[h(seed, i) mod n_table] of int32, with
 * h a 32-bit integer hash computed in registers (no index stream); the
 * xor of all values read goes to *sink (one uint32).  n_table must be a
 * power of two, 1 <= n_table <= 2^31. */
int ccb_gather(const int32_t* table, int64_t n_table, int64_t count, uint32_t seed, uint32_t* sink,
               void* stream);

/* Streaming read of `bytes` (a multiple of 16) from buf; xor of all words to
 * *sink. */
int ccb_stream_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream);

/* Plain copy of `bytes` (a multiple of 16) from src to dst (used to calibrate
 * hardware traffic counters against a known byte count). */
int ccb_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Random compare-and-swaps: `count` device-scope compare-and-swaps on
 * table[j], j = h(seed, i) mod n_table, each expecting the value j and
 * writing j xor 1 (so the table's contents change).  n_table a power of two. */
int ccb_cas(int32_t* table, int64_t n_table, int64_t count, uint32_t seed, void* stream);

/* Timing events for measurement code.  A HIP event created with
 * hipEventDisableSystemFence: recording it writes a timestamp between the
 * work before and after it on `stream` without the cache writeback and
 * invalidation of a default event (about 3.6 us per record on MI355X, which
 * on a stream of short kernels inflates what is measured).  The event only
 * orders timing; it makes no memory visible to the host.
 *   ccb_event_create   *ev receives the handle (owned by the caller, released
 *                      with ccb_event_destroy)
 *   ccb_event_record   enqueue on `stream` (a hipStream_t, NULL = null stream)
 *   ccb_event_elapsed_ms  waits for `stop`, then *ms = stop - start
 * Return 0 on success, -1 for a bad argument, -4 if a HIP call failed. */
int ccb_event_create(void** ev);
int ccb_event_record(void* ev, void* stream);
int ccb_event_elapsed_ms(void* start, void* stop, float* ms);
int ccb_event_destroy(void* ev);

#ifdef __cplusplus
}
#endif

#endif /* CC_BENCH_H */
