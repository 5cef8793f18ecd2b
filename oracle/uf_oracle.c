/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, obviously correct union-find that defines what the bulk
 * incremental connectivity library must return.  Only tests, the smoke check
 * and the benchmark's CPU-baseline leg load this file; the product path never
 * does, and the two share no code.
 *
 * What it computes (Simsiri, Tangwongsan, Tirthapura, Wu, "Work-Efficient
 * Parallel and Incremental Graph Connectivity"):
 *   - Section 1 (Model): a stream of minibatches A_1, A_2, ...; after A_t the
 *     graph is G_t = (V, union of A_1..A_t).  Bulk-Update adds a minibatch,
 *     Bulk-Query answers "connected in G_t?" for each pair; each bulk call
 *     completes before the next starts.
 *   - Section 4 (union-find preamble): find(u) returns the root of u's tree,
 *     and find(u) == find(v) exactly when u and v are connected; union links
 *     two roots.  The paper links by size and notes that union by rank works
 *     as well; this oracle links by rank (ties: the smaller id stays root and
 *     its rank grows), which keeps every tree's height at most floor(log2 n)
 *     (the sequential union-find lemma of Section 4).
 *   - Section 6.1 baseline "UF with path compression": every find re-points
 *     the nodes of its path at the root (two passes, iterative).
 *   - Algorithm 1 (Simple-Bulk-Query): answer i is find(u_i) == find(v_i), in
 *     input order.
 *   - Bulk-Update here is the sequential counterpart the paper compares
 *     against (Section 6.2, "Baseline"): a union per edge, in input order.
 *     By the correctness lemma of Section 4.2 the connectivity after a
 *     minibatch does not depend on the order the unions are applied in, so
 *     this defines the unique answers any parallel method must reproduce.
 *   - Component identifier: the smallest vertex id of the component (a
 *     canonical choice; the paper only asks for "an identifier").
 *
 * Ids are int32 in [0, n).  An edge or pair with an id outside that range is
 * skipped (an edge is not applied, a query answers 0) and counted.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  int32_t* parent;
  uint8_t* rank;
  int64_t unions;
  int64_t invalid;
} uf_t;

uf_t* uf_create(int64_t n) {
  if (n < 1 || n > INT32_MAX) return NULL;
  uf_t* u = (uf_t*)calloc(1, sizeof(uf_t));
  if (!u) return NULL;
  u->n = n;
  u->parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  u->rank = (uint8_t*)calloc((size_t)n, 1);
  if (!u->parent || !u->rank) {
    free(u->parent);
    free(u->rank);
    free(u);
    return NULL;
  }
  for (int64_t i = 0; i < n; ++i) u->parent[i] = (int32_t)i;
  return u;
}

void uf_destroy(uf_t* u) {
  if (!u) return;
  free(u->parent);
  free(u->rank);
  free(u);
}

/* Root of x, with full path compression (walk up, then re-walk pointing every
 * node at the root).  Iterative: paths may be long before compression. */
static int32_t uf_find(uf_t* u, int32_t x) {
  int32_t r = x;
  while (u->parent[r] != r) r = u->parent[r];
  while (u->parent[x] != r) {
    int32_t next = u->parent[x];
    u->parent[x] = r;
    x = next;
  }
  return r;
}

static int in_range(const uf_t* u, int32_t x) { return x >= 0 && (int64_t)x < u->n; }

/* Union by rank of the trees of a and b.  Returns 1 if they were distinct. */
static int uf_union(uf_t* u, int32_t a, int32_t b) {
  int32_t ra = uf_find(u, a), rb = uf_find(u, b);
  if (ra == rb) return 0;
  if (u->rank[ra] < u->rank[rb] || (u->rank[ra] == u->rank[rb] && rb < ra)) {
    int32_t t = ra;
    ra = rb;
    rb = t;
  }
  /* ra is the new root: higher rank, or equal rank and smaller id */
  u->parent[rb] = ra;
  if (u->rank[ra] == u->rank[rb]) u->rank[ra]++;
  u->unions++;
  return 1;
}

/* Bulk-Update: edges is int32[m][2]; returns the number of skipped edges. */
int64_t uf_bulk_update(uf_t* u, const int32_t* edges, int64_t m) {
  int64_t bad = 0;
  for (int64_t i = 0; i < m; ++i) {
    int32_t a = edges[2 * i], b = edges[2 * i + 1];
    if (!in_range(u, a) || !in_range(u, b)) {
      bad++;
      continue;
    }
    uf_union(u, a, b);
  }
  u->invalid += bad;
  return bad;
}

/* Bulk-Query: out[i] = 1 iff pairs[i] are connected; returns skipped count. */
int64_t uf_bulk_query(uf_t* u, const int32_t* pairs, int64_t q, uint8_t* out) {
  int64_t bad = 0;
  for (int64_t i = 0; i < q; ++i) {
    int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    if (!in_range(u, a) || !in_range(u, b)) {
      out[i] = 0;
      bad++;
      continue;
    }
    out[i] = uf_find(u, a) == uf_find(u, b) ? 1 : 0;
  }
  u->invalid += bad;
  return bad;
}

/* label[v] = smallest id in v's component: scanning v upwards, the first
 * vertex met in a tree is that tree's minimum. */
int uf_labels(uf_t* u, int32_t* out) {
  int32_t* first = (int32_t*)malloc((size_t)u->n * sizeof(int32_t));
  if (!first) return -1;
  for (int64_t i = 0; i < u->n; ++i) first[i] = -1;
  for (int64_t v = 0; v < u->n; ++v) {
    int32_t r = uf_find(u, (int32_t)v);
    if (first[r] < 0) first[r] = (int32_t)v;
    out[v] = first[r];
  }
  free(first);
  return 0;
}

int64_t uf_num_components(const uf_t* u) { return u->n - u->unions; }
int64_t uf_unions(const uf_t* u) { return u->unions; }
int64_t uf_invalid(const uf_t* u) { return u->invalid; }

/* Number of roots (parent[v] == v), counted directly. */
int64_t uf_count_roots(const uf_t* u) {
  int64_t c = 0;
  for (int64_t v = 0; v < u->n; ++v) c += u->parent[v] == v;
  return c;
}

/* Height of the tallest tree (edges on the longest node-to-root path),
 * measured without compressing. */
int32_t uf_max_height(const uf_t* u) {
  int32_t h = 0;
  for (int64_t v = 0; v < u->n; ++v) {
    int32_t d = 0, x = (int32_t)v;
    while (u->parent[x] != x) {
      x = u->parent[x];
      d++;
    }
    if (d > h) h = d;
  }
  return h;
}

/* Copy of the parent array (for tests of the oracle's own invariants). */
void uf_parents(const uf_t* u, int32_t* out) { memcpy(out, u->parent, (size_t)u->n * 4); }
