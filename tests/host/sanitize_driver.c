/* Host-only driver for the C code of the oracle and of the input generators,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (every report
 * aborts).  It runs both through small and degenerate cases: n = 1, empty
 * batches, ids out of range, repeated edges, every generator at tiny sizes.
 * Exit status 0 means no sanitizer report and every check held. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void* uf_create(int64_t n);
void uf_destroy(void* u);
int64_t uf_bulk_update(void* u, const int32_t* edges, int64_t m);
int64_t uf_bulk_query(void* u, const int32_t* pairs, int64_t q, uint8_t* out);
int uf_labels(void* u, int32_t* out);
int64_t uf_num_components(const void* u);
int64_t uf_count_roots(const void* u);
int64_t uf_invalid(const void* u);
int32_t uf_max_height(const void* u);
void uf_parents(const void* u, int32_t* out);

uint64_t sg_key(uint64_t seed, uint64_t stream, uint64_t purpose);
void sg_uniform_pairs(uint64_t key, int64_t start, int64_t count, int64_t n, int32_t* out);
void sg_rmat_edges(uint64_t key, int64_t start, int64_t count, int scale, double a, double b, double c, int64_t n,
                   const int32_t* perm, int32_t* out);
void sg_permutation(uint64_t key, int64_t n, int32_t* out);
void sg_shuffle_pairs(uint64_t key, int64_t count, int32_t* pairs);
int64_t sg_grid_edge_count(int64_t W, int64_t H);
int64_t sg_grid_stream(int64_t W, int64_t H, int64_t extra, uint64_t lkey, uint64_t skey, int32_t* out);
int64_t sg_grid3d_edge_count(int64_t L);
int64_t sg_grid3d_stream(int64_t L, uint64_t skey, int32_t* out);
void sg_local_pairs(uint64_t key, int64_t start, int64_t count, int64_t n, double lg, int32_t* out);
void sg_lognormal_counts(uint64_t key, int64_t count, double mu, double sigma, int64_t lo, int64_t hi, int64_t* out);
void sg_poisson_arrivals(uint64_t key, int64_t count, double lam, double* out);

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                     \
    }                                                               \
  } while (0)

static int oracle_cases(void) {
  /* n = 1: only the self-loop exists */
  void* u = uf_create(1);
  CHECK(u);
  int32_t e1[4] = {0, 0, 0, 0};
  uint8_t a1[2];
  CHECK(uf_bulk_update(u, e1, 2) == 0);
  CHECK(uf_bulk_query(u, e1, 2, a1) == 0 && a1[0] == 1 && a1[1] == 1); /* returns the skipped count */
  int32_t lab1[1];
  CHECK(uf_labels(u, lab1) == 0 && lab1[0] == 0);
  CHECK(uf_num_components(u) == 1 && uf_count_roots(u) == 1);
  uf_destroy(u);

  /* invalid ids, empty batches, repeated edges, a long chain */
  const int64_t n = 1000;
  u = uf_create(n);
  CHECK(uf_bulk_update(u, NULL, 0) == 0);
  int32_t bad[8] = {-1, 3, 5, (int32_t)n, 7, 7, 2147483647, -2147483647 - 1};
  uf_bulk_update(u, bad, 4);
  CHECK(uf_invalid(u) == 3);
  int32_t* chain = (int32_t*)malloc(sizeof(int32_t) * 2 * (n - 1));
  for (int64_t i = 0; i < n - 1; ++i) {
    chain[2 * i] = (int32_t)(n - 1 - i);
    chain[2 * i + 1] = (int32_t)(n - 2 - i);
  }
  uf_bulk_update(u, chain, n - 1);
  uf_bulk_update(u, chain, n - 1); /* repeats change nothing */
  CHECK(uf_num_components(u) == 1 && uf_count_roots(u) == 1);
  int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * n);
  int32_t* par = (int32_t*)malloc(sizeof(int32_t) * n);
  CHECK(uf_labels(u, lab) == 0);
  for (int64_t v = 0; v < n; ++v) CHECK(lab[v] == 0);
  uf_parents(u, par);
  CHECK(uf_max_height(u) <= 10);
  uint8_t* ans = (uint8_t*)malloc(n - 1);
  CHECK(uf_bulk_query(u, chain, n - 1, ans) == 0);
  for (int64_t i = 0; i < n - 1; ++i) CHECK(ans[i] == 1);
  free(chain);
  free(lab);
  free(par);
  free(ans);
  uf_destroy(u);
  return 0;
}

static int generator_cases(void) {
  const uint64_t k = sg_key(0x16020523u, 3, 7);
  int32_t pairs[2 * 64];
  sg_uniform_pairs(k, 0, 64, 1, pairs);
  for (int i = 0; i < 128; ++i) CHECK(pairs[i] == 0);
  sg_uniform_pairs(k, 5, 0, 10, pairs);
  int32_t perm[1 << 6];
  sg_permutation(k, 1 << 6, perm);
  int seen[1 << 6];
  memset(seen, 0, sizeof(seen));
  for (int i = 0; i < (1 << 6); ++i) {
    CHECK(perm[i] >= 0 && perm[i] < (1 << 6));
    seen[perm[i]]++;
  }
  for (int i = 0; i < (1 << 6); ++i) CHECK(seen[i] == 1);
  sg_rmat_edges(k, 0, 64, 6, 0.57, 0.19, 0.19, 1 << 6, perm, pairs);
  for (int i = 0; i < 128; ++i) CHECK(pairs[i] >= 0 && pairs[i] < (1 << 6));
  sg_rmat_edges(k, 0, 64, 6, 0.57, 0.19, 0.19, 37, NULL, pairs); /* n not a power of two: redraws */
  for (int i = 0; i < 128; ++i) CHECK(pairs[i] >= 0 && pairs[i] < 37);
  sg_shuffle_pairs(k, 64, pairs);
  sg_shuffle_pairs(k, 1, pairs);
  for (int64_t W = 1; W <= 5; ++W)
    for (int64_t H = 1; H <= 5; ++H) {
      const int64_t m = sg_grid_edge_count(W, H), extra = 3;
      int32_t* g = (int32_t*)malloc(sizeof(int32_t) * 2 * (m + extra) + 8);
      CHECK(sg_grid_stream(W, H, extra, k, k + 1, g) == m + extra);
      for (int64_t i = 0; i < 2 * (m + extra); ++i) CHECK(g[i] >= 0 && g[i] < W * H);
      free(g);
    }
  for (int64_t L = 1; L <= 4; ++L) {
    const int64_t m = sg_grid3d_edge_count(L);
    int32_t* g = (int32_t*)malloc(sizeof(int32_t) * 2 * m + 8);
    CHECK(sg_grid3d_stream(L, k, g) == m);
    for (int64_t i = 0; i < 2 * m; ++i) CHECK(g[i] >= 0 && g[i] < L * L * L);
    free(g);
  }
  sg_local_pairs(k, 0, 64, 1, 0.0, pairs);
  for (int i = 0; i < 128; ++i) CHECK(pairs[i] == 0);
  sg_local_pairs(k, 0, 64, 100, 10.0, pairs);
  for (int i = 0; i < 128; ++i) CHECK(pairs[i] >= 0 && pairs[i] < 100);
  int64_t counts[32];
  sg_lognormal_counts(k, 32, 14.0, 2.0, 1 << 10, 1 << 20, counts);
  for (int i = 0; i < 32; ++i) CHECK(counts[i] >= (1 << 10) && counts[i] <= (1 << 20));
  double t[32];
  sg_poisson_arrivals(k, 32, 1000.0, t);
  for (int i = 1; i < 32; ++i) CHECK(t[i] >= t[i - 1]);
  return 0;
}

int main(void) {
  if (oracle_cases()) return 1;
  if (generator_cases()) return 1;
  printf("sanitized host checks passed\n");
  return 0;
}
