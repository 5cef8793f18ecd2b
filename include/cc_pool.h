/*
 * cc_pool.h -- many independent graph streams on one GPU.
 *
 * A pool holds many graphs of the bulk incremental connectivity problem
 * (Simsiri et al., Section 1, Model) in one device arena, and runs a list of
 * Bulk-Update / Bulk-Query operations over many graphs with one kernel launch
 * per round instead of one launch per graph.  Each graph keeps the paper's
 * rule that a bulk operation completes before the next begins (Section 1):
 * operations on the same graph take effect in list order; operations on
 * different graphs are independent and may run at the same time.  Results are
 * exactly those of a cc_graph (include/cc.h) fed the same calls.
 *
 * Memory: the arena holds `capacity` int32 parent entries; a graph of n
 * vertices occupies n consecutive entries (first fit).  Adding a graph fails
 * with CC_ENOMEM when no gap is large enough: the caller (e.g. a serving loop
 * with a memory budget) then saves and removes an idle graph.
 *
 * Conventions are those of cc.h: asynchronous, ordered on the pool's stream;
 * device pointers owned by the caller stay valid until the stream has run the
 * call; out-of-range ids are skipped and reported once by cc_pool_sync as
 * CC_ERANGE; argument errors return CC_EINVAL with nothing enqueued.  A pool
 * handle is not thread safe.
 */
#ifndef CC_POOL_H
#define CC_POOL_H

#include <stdint.h>

#include "cc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc_pool cc_pool;

/* One operation of a cc_pool_run list.  kind 0 = Bulk-Update: `items` holds
 * count edges, device int32[count][2] (8-byte aligned), graph-local ids.  kind 1 = Bulk-Query:
 * `items` holds count pairs and `out` receives count uint8 answers (device),
 * in input order. */
typedef struct {
  int32_t graph;
  int32_t kind;
  int64_t count;
  const int32_t* items;
  uint8_t* out;
} cc_op;

/* Create a pool with room for `capacity` vertices in total and at most
 * max_graphs graphs, on the current device and the null stream.  NULL on
 * failure (cc_last_error()). */
cc_pool* cc_pool_create(int64_t capacity, int32_t max_graphs);
int cc_pool_destroy(cc_pool* p);  /* waits for the stream */
int cc_pool_set_stream(cc_pool* p, void* stream);
/* Options of enum cc_option that apply to the pool: CC_OPT_BLOCK,
 * CC_OPT_ITEMS, CC_OPT_QUERY_HALVING, CC_OPT_HOOK 0, 1 or 2 (set before
 * adding graphs, CC_EINVAL once a graph exists; under 2, union by rank,
 * cc_pool_add refuses graphs of more than 2^27 vertices), CC_OPT_GRID_CAP,
 * CC_OPT_COMPRESS_LINKED, CC_OPT_SPIN_LIMIT, CC_OPT_ONE_LAUNCH, and
 * CC_OPT_FILTER 0 or 1 (any other value: CC_EINVAL).  CC_OPT_FILTER 1 is a
 * membership filter per graph (an anchor vertex and one bit per slot of the
 * arena, capacity / 8 bytes, allocated when first turned on; CC_ENOMEM if
 * that fails): before an update round on a graph updated since its marks
 * were last renewed, one pass over the graph's slots marks the vertices
 * known to be connected to the anchor, and an edge or query pair with both
 * ends marked is settled without a parent read.  The one-launch form renews
 * the marks inside its launch, between two device-wide barriers.  Turning
 * it on clears every mark; reset, reset_all, add and load clear the graph's
 * own.  No option changes a result. */
int cc_pool_set_option(cc_pool* p, int key, int64_t value);

/* Add a graph on vertices [0, n), every vertex alone; *id receives its
 * handle.  CC_ENOMEM if no gap of n entries (or no free handle) is left. */
int cc_pool_add(cc_pool* p, int64_t n, int32_t* id);
/* Remove a graph and free its entries (stream ordered: later work may reuse
 * them only after earlier work on the stream). */
int cc_pool_remove(cc_pool* p, int32_t id);
/* Restore a graph to every vertex alone. */
int cc_pool_reset(cc_pool* p, int32_t id);
/* Restore every graph of the pool to every vertex alone (one launch). */
int cc_pool_reset_all(cc_pool* p);
int64_t cc_pool_graph_vertices(const cc_pool* p, int32_t id);   /* 0 if no such graph */
int64_t cc_pool_free_vertices(const cc_pool* p);               /* total free entries */
int64_t cc_pool_largest_gap(const cc_pool* p);                 /* largest addable n */
/* Arena offset of graph `id` (-1 if no such graph), and the free ranges:
 * up to max (base, length) pairs in ascending base order; returns how many
 * free ranges there are.  For callers that plan admissions and evictions. */
int64_t cc_pool_graph_base(const cc_pool* p, int32_t id);
int32_t cc_pool_gaps(const cc_pool* p, int64_t* bases, int64_t* lengths, int32_t max);

/* Run the operations: those on one graph in list order, different graphs
 * together, with one kernel launch per round (round r holds every graph's
 * r-th operation).  Operations with count 0 are skipped.  Every graph id and
 * kind is checked before anything is enqueued (CC_EINVAL). */
int cc_pool_run(cc_pool* p, const cc_op* ops, int32_t num_ops);

/* out[v] = smallest id of v's component in graph `id` (device int32[n]). */
int cc_pool_labels(cc_pool* p, int32_t id, int32_t* out);
/* Components of graph `id`, counting isolated vertices.  Waits. */
int cc_pool_num_components(cc_pool* p, int32_t id, int64_t* out);
/* Wait; report a latched CC_ERANGE / CC_ECORRUPT once, as cc_sync. */
int cc_pool_sync(cc_pool* p);

/* State image of one graph in the cc_save layout (int64 n, int64 links,
 * int32 parent[n] with graph-local ids), so images move freely between pool
 * slots and standalone graphs.  Save waits; load checks the image as cc_load
 * does (CC_ECORRUPT, graph unchanged) and waits for the copy. */
int64_t cc_pool_state_bytes(const cc_pool* p, int32_t id);
int cc_pool_save(cc_pool* p, int32_t id, void* host_buf);
int cc_pool_load(cc_pool* p, int32_t id, const void* host_buf);

#ifdef __cplusplus
}
#endif

#endif /* CC_POOL_H */
