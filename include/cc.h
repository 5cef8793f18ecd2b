/*
 * cc.h -- bulk-parallel incremental graph connectivity on one AMD MI355X.
 *
 * The problem is the one of Simsiri, Tangwongsan, Tirthapura and Wu,
 * "Work-Efficient Parallel and Incremental Graph Connectivity", Section 1
 * (Model): a fixed vertex set V = {0, ..., n-1} receives a stream of edge
 * minibatches A_1, A_2, ...; after A_t the graph is G_t = (V, A_1 u ... u A_t).
 * Two bulk operations act on it:
 *   - Bulk-Update(A_i) adds a minibatch of edges;
 *   - Bulk-Query(pairs) answers, for each vertex pair, whether the pair is
 *     connected in the edges seen so far.
 * A bulk operation completes before the next begins (Section 1).  Here that
 * order is the order of calls on the graph's HIP stream: every call is
 * asynchronous and stream ordered, and no call waits for the device unless
 * its comment says so.
 *
 * State is one int32 union-find parent array of n entries in device memory
 * (O(n) words, Theorem 1 of Section 4), owned by the graph handle.
 *
 * Conventions for every call:
 *   - Vertex ids are int32 in [0, n).  Edge and pair arrays are int32[k][2]
 *     (u0, v0, u1, v1, ...), 8-byte aligned, in DEVICE memory owned by the
 *     caller; they must stay valid until the stream has run the call.
 *   - An edge or pair holding an id outside [0, n) is skipped: the edge is
 *     not applied, the pair's answer is 0.  All other items are processed as
 *     usual.  The skip is latched on the device and reported once by the next
 *     cc_sync() as CC_ERANGE.
 *   - Argument errors (NULL handle or pointer with a nonzero count, negative
 *     count) return CC_EINVAL at once and enqueue nothing.
 *   - A count of 0 is a no-op.
 *   - A handle is not thread safe; different handles are independent.
 *   - Return codes are CC_OK or one of the negative CC_E* codes; the text of
 *     the last failure in the calling thread is available from
 *     cc_last_error().
 */
#ifndef CC_H
#define CC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc_graph cc_graph;

enum cc_status {
  CC_OK = 0,
  CC_EINVAL = -1,   /* bad argument; nothing was enqueued */
  CC_ENOMEM = -2,   /* device or host allocation failed */
  CC_ERANGE = -3,   /* an id outside [0, n) was skipped (reported by cc_sync) */
  CC_EDEVICE = -4,  /* a HIP runtime call failed */
  CC_ECORRUPT = -5  /* a find exceeded n steps (the parent array holds a cycle),
                       or a state image given to cc_load is not a valid forest */
};

/* Tuning options (cc_set_option).  None changes any result. */
enum cc_option {
  /* Bulk-Update schedule.  0 = fused: one kernel finds both roots and links
   * them with a compare-and-swap in place.  1 = split: a filter kernel
   * relabels edges by their roots and compacts the pairs with distinct roots
   * (the relabel and filter of Algorithm 2) into a live list, a link kernel joins the live
   * root pairs, a compress kernel points the linked roots at their new root;
   * at most 2^31 - 1 edges per call.
   * 2 = contracting: Algorithm 2 with its connected-components step done on
   * the contracted edge list A'' by rounds of hooking and shortcutting (one
   * cooperative launch; 8 bytes of scratch per edge of the largest
   * minibatch; each round's work is linear in the surviving root pairs, not
   * in the minibatch; the open question of Section 7 about very large
   * minibatches).  Id and hashed orders only, not available during capture,
   * at most 2^31 - 1 edges per call.
   * Union by rank (CC_OPT_HOOK 2) takes schedules 0 and 1.  Default 0. */
  CC_OPT_UPDATE_MODE = 1,
  CC_OPT_BLOCK = 2,          /* threads per block, multiple of 64 in [64, 1024]; default 256 */
  CC_OPT_ITEMS = 3,          /* edges (or pairs) per thread: 1, 2, 4 or 8, or 0 = chosen per
                                call from the item count (default 0) */
  CC_OPT_QUERY_HALVING = 4,  /* 1: query finds also halve paths (default); 0: read-only */
  CC_OPT_COMPRESS_EVERY = 5, /* k > 0: after every k-th update point every vertex at its
                                root (full pass over n); 0 = never (default) */
  CC_OPT_HOOK = 6,           /* linking order: 0 = by vertex id, the smaller id becomes
                                the root (default); 1 = by a hashed priority (fmix32);
                                2 = union by rank (the balanced linking of Section 4
                                with ranks in place of sizes; a root's rank sits in
                                bits 27-31 of its word, so n <= 2^27).  Can change
                                only while the graph has had no update since its
                                creation or the last cc_reset (CC_EINVAL otherwise);
                                a load keeps the order it was checked against. */
  CC_OPT_GRID_CAP = 7,       /* upper bound on blocks per launch (grid-stride beyond it);
                                default 4096 */
  /* Fused schedule: 1 = record the roots each update links and afterwards
   * point every vertex on their paths straight at the root (the "pragmatic"
   * path compression of Section 6.1, limited to what the minibatch changed);
   * 0 = rely on path halving alone.  Default 1. */
  CC_OPT_COMPRESS_LINKED = 8,
  /* cc_bulk_stream: how many sleeps (about 60 ns each) a block waits at a
   * device-wide barrier before it gives up, raises the timeout condition
   * (reported by cc_sync as CC_EDEVICE) and makes every block leave the
   * kernel.  Default 2^24 (about one second). */
  CC_OPT_SPIN_LIMIT = 9,
  /* How finds are done.  0 = every endpoint walks to its root on its own
   * (with path halving; default).  1 = Bulk-Find (Section 5, Algorithm 4):
   * all endpoints of a Bulk-Update or Bulk-Query are resolved together, flows
   * that meet are merged, and every traversed vertex is pointed at its root;
   * Phase II by pointer jumping over the traversed vertices.  2 = Bulk-Find
   * with Phase II as the paper's top-down distribution through the response
   * distributor (Section 5.1: the traversed parent pointers sorted by a hash
   * of the parent into 3x as many buckets, then handed the root level by
   * level from the roots; about 52 more bytes per traversal bound entry,
   * 2 * (vertices + items), at most 2^31 - 1 of them).  Two launches per
   * bulk operation: level 0 (every item read once) as an ordinary launch,
   * then Phases I and II in one cooperative launch of at most 256 blocks;
   * scratch of about 8 bytes per vertex plus 8 bytes per item of the
   * largest bulk operation; not available during capture. */
  CC_OPT_FIND = 10,
  /* Pools only (cc_pool_run): 1 = all rounds of a run in one cooperative
   * launch, separated by device-wide barriers, instead of one launch per
   * round; no linked-root compression in that form.  Default 0. */
  CC_OPT_ONE_LAUNCH = 11,
  /* Membership filter of the largest component: two bitmaps of n bits each
   * (n / 4 bytes of device memory).  The membership bitmap holds vertices
   * proven connected to an anchor vertex, chosen as the root most sampled
   * minibatch endpoints lead to; the touched bitmap holds both ends of every
   * link.  1 = under the fused schedule an edge whose endpoints are both
   * members is dropped without a find (it could only join a component with
   * itself); 2 = that, and Bulk-Query answers without a find a pair of two
   * members (1) and, while every update since the last reset went through
   * the filtered fused schedule or filtered Bulk-Find, a pair with an end
   * outside the touched bitmap (0: that vertex never had an edge); its finds
   * also add the endpoints they prove connected.  cc_labels uses the bitmaps
   * whenever they exist.  Bits are set only from proofs, so results are
   * unchanged.  Choosing the anchor costs one single-block launch and one
   * launch that refills the membership bitmap when the anchor changes (a
   * pass over the parent array), before update calls 0, 1, 2, 4, 8, ... and
   * every 64th call after a reset or load.  With CC_OPT_FIND 1 or 2,
   * Bulk-Find settles the same items before its climb and keeps the touched
   * bitmap; it sets no membership bits itself, so the bitmap is also
   * refilled before a Bulk-Update once n / 8 edges have gone in since the
   * last refill.  The split and contracting schedules and cc_bulk_stream
   * neither use nor update the bitmaps.  Default 0. */
  CC_OPT_FILTER = 12,
  /* Pairs per thread of Bulk-Query: 1, 2, 4 or 8, or 0 = as CC_OPT_ITEMS
   * (default), for when queries and updates want different amounts of work
   * in flight per thread. */
  CC_OPT_QUERY_ITEMS = 13,
  /* Compaction threshold of the fused schedule (CC_OPT_UPDATE_MODE 0), a
   * percentage in [0, 100].  t > 0: an update whose minibatch is expected to
   * keep fewer than t% of its edges live (edges whose endpoints' roots
   * differ, the contracted edge list A'' of Algorithm 2) runs the split
   * schedule, which compacts the live edges before linking them; the others
   * run fused.  The estimate is the fraction of edges that linked in the
   * latest earlier updates whose link counts have reached the host: after
   * each such update the library copies its link counters to pinned host
   * memory asynchronously and reads them at a later call once the copy has
   * finished, so no call waits for the device.  The first update after
   * creation or a reset runs fused.  During capture the schedule of the last
   * eager decision is recorded.  0 = always fused (default). */
  CC_OPT_SPLIT_BELOW = 14
};

/* Create a graph on vertices [0, n), 1 <= n <= 2^31 - 1, every vertex its own
 * component (parent[v] = v).  Uses the current HIP device and the null
 * stream until cc_set_stream.  Waits for the initialisation to finish.
 * Returns NULL on failure (see cc_last_error()).  Ownership: the caller
 * releases the handle with cc_destroy. */
cc_graph* cc_create(int64_t n);

/* Release the handle and its device memory.  Waits for the graph's stream. */
int cc_destroy(cc_graph* g);

/* Issue all later work of g on `stream` (a hipStream_t; NULL = null stream).
 * The caller keeps ownership of the stream and must not destroy it while g
 * uses it. */
int cc_set_stream(cc_graph* g, void* stream);

/* Set a tuning option (enum cc_option).  CC_EINVAL for an unknown key or a
 * value out of range. */
int cc_set_option(cc_graph* g, int key, int64_t value);
int cc_get_option(cc_graph* g, int key, int64_t* value);

/* Pre-size the scratch used by the split update schedule (or by the
 * contracting schedule, when that is the schedule set at the time of the
 * call) for minibatches of up to max_batch edges, so that no later call
 * allocates.  Waits for the
 * stream if an existing buffer is replaced. */
int cc_reserve(cc_graph* g, int64_t max_batch);

/* Restore the initial state (every vertex alone) without reallocating. */
int cc_reset(cc_graph* g);

/* Bulk-Update (Section 1; Algorithm 2 of Section 4.2 computes the same
 * connectivity): add the m edges of `edges` (device int32[m][2]).  Edges are
 * undirected; self-loops and repeated edges are allowed and change nothing.
 * The order of edges within the minibatch does not matter (Section 4.2,
 * correctness of Simple-Bulk-Update).  May allocate split-schedule scratch if
 * m exceeds the reserved size (see cc_reserve). */
int cc_bulk_update(cc_graph* g, const int32_t* edges, int64_t m);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Bulk-Update as cc_bulk_update, with the same results, that allocates
 * nothing.  It always runs the fused schedule with linked-root compression,
 * whatever CC_OPT_UPDATE_MODE, CC_OPT_FIND, CC_OPT_FILTER and
 * CC_OPT_COMPRESS_LINKED say (any linking order; the filter's bitmaps, if
 * they exist, are marked incomplete as after any unfiltered update).  Its
 * scratch (the list of roots the call links and two counters) is a
 * fixed-size array in the library's device code, one copy per device, held
 * until the process ends; the call clears what must start at zero with a
 * kernel, so it can be captured.  Limit: at most 2^22 edges per call
 * (CC_EINVAL beyond, nothing enqueued).  Every call on a device shares that
 * device's array: calls that overlap on one device (different streams,
 * different graphs) race and must be ordered by the caller, e.g. on one
 * stream. */
int cc_bulk_update_noalloc(cc_graph* g, const int32_t* edges, int64_t m);

/* Bulk-Query (Algorithm 1, Simple-Bulk-Query): out[i] = 1 if pairs[i] are
 * connected by the edges of all earlier updates on g, else 0.  pairs is
 * device int32[q][2], out is device uint8[q], written in input order.  A pair
 * (u, u) answers 1. */
int cc_bulk_query(cc_graph* g, const int32_t* pairs, int64_t q, uint8_t* out);

/* A whole stream in one launch: for k = 0 .. batches-1, Bulk-Update of edges
 * [eoff[k], eoff[k+1]) and then Bulk-Query of pairs [qoff[k], qoff[k+1]) with
 * answers out[qoff[k] ..], exactly as the same sequence of cc_bulk_update and
 * cc_bulk_query calls (each bulk operation completes before the next begins,
 * Section 1).  edges and pairs are device int32[][2]; eoff and qoff are
 * DEVICE int64[batches+1] item offsets into them; out is device uint8 indexed
 * like pairs.  max_items (>= 1) bounds the items of any one operation and
 * sizes the grid: ceil(max_items / CC_OPT_BLOCK) blocks of CC_OPT_BLOCK
 * threads, at most CC_OPT_GRID_CAP, 1024 and what can be resident with one
 * block per compute unit to spare.  The operations are separated by device-wide barriers
 * inside one cooperative launch, for streams of many small minibatches whose
 * separate launches would cost mostly launch latency.  Not available during
 * capture.  A barrier that waits past CC_OPT_SPIN_LIMIT ends the kernel and
 * is reported by cc_sync as CC_EDEVICE. */
int cc_bulk_stream(cc_graph* g, int64_t batches, const int32_t* edges, const int64_t* eoff,
                   const int32_t* pairs, const int64_t* qoff, uint8_t* out, int64_t max_items);

/* Canonical component labels: out[v] = the smallest vertex id connected to v
 * (the paper's find returns "an identifier" of the component, Section 4;
 * this fixes it to the minimum).  out is device int32[n].  Every vertex
 * whose label takes a walk to its root is also pointed directly at the root;
 * vertices that the membership filter's bitmaps settle (CC_OPT_FILTER: a
 * member of the anchor's component, or a vertex proven alone) are not
 * walked. */
int cc_labels(cc_graph* g, int32_t* out);

/* Number of connected components of G_t, counting isolated vertices
 * (n minus the number of successful links).  Waits for the stream;
 * *out is a host int64. */
int cc_num_components(cc_graph* g, int64_t* out);

/* Number of roots (vertices v with parent[v] == v), counted by a pass over
 * the parent array.  Equals cc_num_components; kept as an independent check.
 * Waits for the stream. */
int cc_count_roots(cc_graph* g, int64_t* out);

/* State of the membership filter (CC_OPT_FILTER), for checks.  *anchor gets
 * the anchor vertex (-1 if none, or if the filter has not run since the
 * last reset or load).  *touched_complete gets 1 while every update since
 * the last reset went through the filtered fused form or filtered
 * Bulk-Find, so that the touched bitmap is complete, else 0.  Unless bits
 * is NULL, it gets 2 * ceil(n / 32) HOST uint32 words: the membership
 * bitmap, then the touched bitmap, vertex v at bit v % 32 of word v / 32 of
 * each (all zero if the filter has never run).  Every vertex in the membership bitmap is connected to the anchor;
 * while touched_complete is 1, every vertex in neither bitmap is alone in
 * its component.  Waits for the stream. */
int cc_filter_state(cc_graph* g, int32_t* anchor, int32_t* touched_complete, uint32_t* bits);

/* Wait for all work issued on g's stream; then report, once, a skipped id
 * (CC_ERANGE) or a corrupt forest (CC_ECORRUPT) latched since the last
 * cc_sync, and clear it.  CC_EDEVICE if the stream failed. */
int cc_sync(cc_graph* g);

/* State image for checkpoint and restore: cc_state_bytes(g) bytes laid out as
 * int64 n, int64 successful links, int32 parent[n].  cc_save writes it to a
 * caller-owned HOST buffer and waits for the stream; cc_load reads it back
 * (same n), checks that it is a forest under g's linking order (else
 * CC_ECORRUPT and g is unchanged), and waits for the copy. */
int64_t cc_state_bytes(const cc_graph* g);
int cc_save(cc_graph* g, void* host_buf);
int cc_load(cc_graph* g, const void* host_buf);

/* Capture and replay with a HIP graph, for streams of many small minibatches
 * whose cost is dominated by launch overhead.  Between cc_capture_begin(g)
 * and cc_capture_end(g, &x) the calls cc_reset, cc_bulk_update, cc_bulk_query
 * and cc_labels on g are recorded instead of run; cc_exec_launch(x) then runs
 * the whole recorded sequence, in order, with one launch on g's stream,
 * reading and writing the same caller buffers each time (their contents may
 * change between launches).  g's stream must not be the null stream.  During
 * capture, calls that wait for the device (cc_num_components, cc_count_roots,
 * cc_sync, cc_save, cc_load, cc_reserve, cc_destroy) return CC_EINVAL, and so
 * does a split-schedule update larger than the size reserved before the
 * capture.  The recorded work uses no memset nodes.  Ownership: the caller
 * releases x with cc_exec_destroy, before destroying g. */
typedef struct cc_exec cc_exec;
int cc_capture_begin(cc_graph* g);
int cc_capture_end(cc_graph* g, cc_exec** out);
int cc_exec_launch(cc_exec* x);
int cc_exec_destroy(cc_exec* x);

/* Vertex count of g (0 for NULL). */
int64_t cc_num_vertices(const cc_graph* g);

/* Text of a status code, and of the last failure in the calling thread. */
const char* cc_strerror(int code);
const char* cc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CC_H */
