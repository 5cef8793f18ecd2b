/*
 * Seeded synthetic graph streams for the bulk incremental connectivity
 * library and its oracle.
 *
 * This module holds no part of the connectivity method: it only produces
 * inputs (edge lists, query pairs, batch sizes, permutations, arrival times).
 * Both the CPU oracle side and the GPU side draw their inputs from here, so a
 * given (seed, stream, purpose, index) always yields the same bytes.
 *
 * Random numbers are counter based: draw(key, i) is the (i+1)-th output of
 * Vigna's splitmix64 generator started at state `key`, i.e. the splitmix64
 * finaliser applied to key + (i+1) * 0x9e3779b97f4a7c15.  Any slice of any
 * stream can therefore be regenerated independently and in parallel, and the
 * output does not depend on the number of threads.
 *
 * Workload shapes follow the paper's evaluation (Section 6.2, Table 1):
 * uniform random graphs, power-law R-MAT graphs (Chakrabarti, Zhan and
 * Faloutsos' recursive matrix model) and high-diameter meshes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SG_GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t sg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Key of one named random stream: (seed, stream, purpose) -> 64-bit state. */
uint64_t sg_key(uint64_t seed, uint64_t stream, uint64_t purpose) {
  uint64_t k = sg_mix(seed + SG_GOLDEN);
  k = sg_mix(k ^ ((stream + 1) * 0xd1b54a32d192ed03ULL));
  k = sg_mix(k ^ ((purpose + 1) * 0x8cb92ba72f3d8dd7ULL));
  return k;
}

/* i-th (0-based) output of splitmix64 started at state `key`. */
uint64_t sg_draw(uint64_t key, uint64_t i) {
  return sg_mix(key + (i + 1) * SG_GOLDEN);
}

/* Uniform integer in [0, n) by Lemire's multiply-high mapping. */
static inline int64_t sg_below(uint64_t r, uint64_t n) {
  return (int64_t)(((unsigned __int128)r * n) >> 64);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double sg_unit(uint64_t r) {
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

/* Raw draws out[k] = draw(key, start + k). */
void sg_draws(uint64_t key, int64_t start, int64_t count, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = sg_draw(key, (uint64_t)(start + k));
}

/* Uniform doubles in [0, 1). */
void sg_unit_doubles(uint64_t key, int64_t start, int64_t count, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = sg_unit(sg_draw(key, (uint64_t)(start + k)));
}

/*
 * Uniform vertex pairs: pair i = (draw(key, 2i) mod* n, draw(key, 2i+1) mod* n)
 * where mod* is the multiply-high mapping.  Self-loops and repeats are kept.
 * Used for Erdos-Renyi edges and for query pairs.  out is int32[count][2].
 */
void sg_uniform_pairs(uint64_t key, int64_t start, int64_t count, int64_t n, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    uint64_t i = (uint64_t)(start + k);
    out[2 * k] = (int32_t)sg_below(sg_draw(key, 2 * i), (uint64_t)n);
    out[2 * k + 1] = (int32_t)sg_below(sg_draw(key, 2 * i + 1), (uint64_t)n);
  }
}

/*
 * R-MAT edges.  Edge i descends `scale` levels of the adjacency matrix; at
 * each level one draw picks the quadrant: top-left with probability a (both
 * id bits 0), top-right b (v bit 1), bottom-left c (u bit 1), bottom-right
 * 1-a-b-c.  Level 0 sets the most significant bit.  If either endpoint is
 * >= n (n not a power of two) the whole edge is redrawn from a derived key,
 * up to 64 attempts, after which ids are folded by the multiply-high map.
 * If perm is non-NULL both ids are mapped through it afterwards.
 */
void sg_rmat_edges(uint64_t key, int64_t start, int64_t count, int scale, double a, double b,
                   double c, int64_t n, const int32_t* perm, int32_t* out) {
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    uint64_t i = (uint64_t)(start + k);
    int64_t u = 0, v = 0;
    for (int attempt = 0; attempt < 64; ++attempt) {
      uint64_t akey = attempt == 0 ? key : sg_mix(key ^ ((uint64_t)attempt * 0xa0761d6478bd642fULL));
      u = 0;
      v = 0;
      for (int lvl = 0; lvl < scale; ++lvl) {
        double x = sg_unit(sg_draw(akey, i * 32 + (uint64_t)lvl));
        int ub = 0, vb = 0;
        if (x < a) {
        } else if (x < ab) {
          vb = 1;
        } else if (x < abc) {
          ub = 1;
        } else {
          ub = 1;
          vb = 1;
        }
        u = (u << 1) | ub;
        v = (v << 1) | vb;
      }
      if (u < n && v < n) break;
      if (attempt == 63) {
        u = sg_below((uint64_t)u * SG_GOLDEN, (uint64_t)n);
        v = sg_below((uint64_t)v * SG_GOLDEN, (uint64_t)n);
      }
    }
    if (perm) {
      u = perm[u];
      v = perm[v];
    }
    out[2 * k] = (int32_t)u;
    out[2 * k + 1] = (int32_t)v;
  }
}

/* Seeded Fisher-Yates permutation of [0, n): swap i with j = below(draw(key, i), i+1). */
void sg_permutation(uint64_t key, int64_t n, int32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = sg_below(sg_draw(key, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

/* Seeded Fisher-Yates shuffle of count int32 pairs in place. */
void sg_shuffle_pairs(uint64_t key, int64_t count, int32_t* pairs) {
  int64_t* p = (int64_t*)pairs; /* one pair = 8 bytes */
  for (int64_t i = count - 1; i > 0; --i) {
    int64_t j = sg_below(sg_draw(key, (uint64_t)i), (uint64_t)(i + 1));
    int64_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
}

/* Number of edges of a W x H 4-neighbour mesh. */
int64_t sg_grid_edge_count(int64_t W, int64_t H) { return H * (W - 1) + (H - 1) * W; }

/*
 * W x H mesh, row-major ids r*W + c: horizontal edges (r,c)-(r,c+1) first,
 * then vertical edges (r,c)-(r+1,c); then `extra` uniform random pairs drawn
 * with purpose key `lkey`; then the whole list shuffled with `skey`.
 * out must hold sg_grid_edge_count(W,H) + extra pairs.  Returns the count.
 */
int64_t sg_grid_stream(int64_t W, int64_t H, int64_t extra, uint64_t lkey, uint64_t skey,
                       int32_t* out) {
  const int64_t nh = H * (W - 1), nv = (H - 1) * W;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nh; ++k) {
    int64_t r = k / (W - 1), c = k % (W - 1);
    out[2 * k] = (int32_t)(r * W + c);
    out[2 * k + 1] = (int32_t)(r * W + c + 1);
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nv; ++k) {
    int64_t r = k / W, c = k % W;
    out[2 * (nh + k)] = (int32_t)(r * W + c);
    out[2 * (nh + k) + 1] = (int32_t)((r + 1) * W + c);
  }
  sg_uniform_pairs(lkey, 0, extra, W * H, out + 2 * (nh + nv));
  sg_shuffle_pairs(skey, nh + nv + extra, out);
  return nh + nv + extra;
}

/* Number of edges of an L x L x L 6-neighbour mesh. */
int64_t sg_grid3d_edge_count(int64_t L) { return 3 * L * L * (L - 1); }

/*
 * L x L x L mesh, ids x + L*(y + L*z): edges along x, then y, then z, each
 * joining a vertex to its +1 neighbour on that axis; then shuffled with skey.
 * out must hold sg_grid3d_edge_count(L) pairs.
 */
int64_t sg_grid3d_stream(int64_t L, uint64_t skey, int32_t* out) {
  const int64_t per = L * L * (L - 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < per; ++k) {
    /* k indexes (a, b, c) with a in [0, L-1) the step coordinate */
    const int64_t a = k % (L - 1), r = k / (L - 1), b = r % L, c = r / L;
    /* axis x: (a, b, c)-(a+1, b, c) */
    out[2 * k] = (int32_t)(a + L * (b + L * c));
    out[2 * k + 1] = (int32_t)(a + 1 + L * (b + L * c));
    /* axis y: (b, a, c)-(b, a+1, c) */
    out[2 * (per + k)] = (int32_t)(b + L * (a + L * c));
    out[2 * (per + k) + 1] = (int32_t)(b + L * (a + 1 + L * c));
    /* axis z: (b, c, a)-(b, c, a+1) */
    out[2 * (2 * per + k)] = (int32_t)(b + L * (c + L * a));
    out[2 * (2 * per + k) + 1] = (int32_t)(b + L * (c + L * (a + 1)));
  }
  sg_shuffle_pairs(skey, 3 * per, out);
  return 3 * per;
}

/*
 * Locality-biased random edges (small separators): edge i joins
 * u = below(draw(key, 3i), n) and v = (u + s * d) mod n with
 * d = floor(2^(U * lg)) for U = unit(draw(key, 3i+1)), lg = log2(window),
 * and s = +1 or -1 from draw(key, 3i+2): most edges are short, a few span
 * up to `window` ids.
 */
void sg_local_pairs(uint64_t key, int64_t start, int64_t count, int64_t n, double lg, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    const uint64_t i = (uint64_t)(start + k);
    const int64_t u = sg_below(sg_draw(key, 3 * i), (uint64_t)n);
    const int64_t d = (int64_t)floor(exp2(sg_unit(sg_draw(key, 3 * i + 1)) * lg));
    const int64_t sgn = (sg_draw(key, 3 * i + 2) >> 63) ? 1 : -1;
    int64_t v = (u + sgn * (d % n)) % n;
    if (v < 0) v += n;
    out[2 * k] = (int32_t)u;
    out[2 * k + 1] = (int32_t)v;
  }
}

/* Map both ids of count pairs through perm, in place. */
void sg_apply_perm(const int32_t* perm, int64_t count, int32_t* pairs) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < 2 * count; ++k) pairs[k] = perm[pairs[k]];
}

/*
 * Log-normal vertex counts: X = mu + sigma * Z (Z standard normal by the
 * Box-Muller transform of draws 2k, 2k+1), out[k] = clip(round(2^X), lo, hi).
 */
void sg_lognormal_counts(uint64_t key, int64_t count, double mu, double sigma, int64_t lo,
                         int64_t hi, int64_t* out) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t k = 0; k < count; ++k) {
    double u1 = 1.0 - sg_unit(sg_draw(key, 2 * (uint64_t)k)); /* (0, 1] */
    double u2 = sg_unit(sg_draw(key, 2 * (uint64_t)k + 1));
    double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    double x = mu + sigma * z;
    int64_t v = (int64_t)llround(exp2(x));
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    out[k] = v;
  }
}

/* Poisson arrival times at rate lam: cumulative sums of -ln(1-U)/lam. */
void sg_poisson_arrivals(uint64_t key, int64_t count, double lam, double* out) {
  double t = 0.0;
  for (int64_t k = 0; k < count; ++k) {
    double u = sg_unit(sg_draw(key, (uint64_t)k));
    t += -log1p(-u) / lam;
    out[k] = t;
  }
}
