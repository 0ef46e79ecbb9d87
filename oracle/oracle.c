/*
 * Plain CPU oracle for the restless-path / restless-motif sieve fingerprint.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library. Written for a
 * reader holding the paper (arXiv 2010.08423); every function names the
 * passage it follows. Slow on purpose: no blocking, no fusion, no reordering
 * beyond what the recurrence itself states.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* x^64 = x^4 + x^3 + x + 1 in the field (the low part of the modulus). */
#define ORC_POLY_LOW 0x1Bull
#define ORC_GOLDEN 0x9E3779B97F4A7C15ull

/* ---------------------------------------------------------------------------
 * GF(2^64). An element is a polynomial over GF(2) of degree < 64; bit i holds
 * the coefficient of x^i (Sec. 4.2: an element of GF(2^b) is a b-bit vector;
 * Sec. 5.1: b = 64). Addition is XOR.
 * ------------------------------------------------------------------------ */

/* Product by definition: carry-less schoolbook product of degree <= 126,
 * then reduction from the top bit down using x^64 = x^4 + x^3 + x + 1. */
uint64_t orc_gf_mul(uint64_t a, uint64_t b) {
  u128 acc = 0;
  for (int i = 0; i < 64; i++)
    if ((b >> i) & 1) acc ^= (u128)a << i;
  for (int i = 127; i >= 64; i--)
    if ((acc >> i) & 1) acc ^= ((u128)1 << i) ^ ((u128)ORC_POLY_LOW << (i - 64));
  return (uint64_t)acc;
}

/* a * x mod the field polynomial. */
static uint64_t orc_mul_x(uint64_t a) { return (a << 1) ^ ((a >> 63) ? ORC_POLY_LOW : 0); }

/* Second formulation: tab[v] = v(x) * b for the 16 polynomials v of degree
 * < 4, then Horner over the 16 base-16 digits of a, most significant first. */
uint64_t orc_gf_mul_nibble(uint64_t a, uint64_t b) {
  uint64_t tab[16];
  tab[0] = 0;
  tab[1] = b;
  for (int v = 2; v < 16; v++) tab[v] = (v & 1) ? (tab[v - 1] ^ b) : orc_mul_x(tab[v / 2]);
  uint64_t acc = 0;
  for (int i = 15; i >= 0; i--) {
    for (int s = 0; s < 4; s++) acc = orc_mul_x(acc);
    acc ^= tab[(a >> (4 * i)) & 15];
  }
  return acc;
}

uint64_t orc_gf_pow(uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = orc_gf_mul_nibble(r, a);
    a = orc_gf_mul_nibble(a, a);
    e >>= 1;
  }
  return r;
}

/* The multiplicative group has order 2^64 - 1, so a^(2^64-2) = a^(-1). */
uint64_t orc_gf_inv(uint64_t a) { return orc_gf_pow(a, 0xFFFFFFFFFFFFFFFEull); }

/* ---------------------------------------------------------------------------
 * Counter-based randomness. The paper draws y from a pseudorandom number
 * generator (Sec. 5.1) and z, gamma, omega uniformly from the field
 * (Sec. 4.3, 4.4); the generator is unspecified there. This project fixes a
 * keyed hash built on the SplitMix64 output finalizer (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).
 * ------------------------------------------------------------------------ */
uint64_t orc_mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

uint64_t orc_hash(uint64_t seed, uint64_t tag, const uint64_t* w, int nw) {
  uint64_t h = orc_mix64(seed + tag * ORC_GOLDEN);
  for (int i = 0; i < nw; i++) h = orc_mix64(h ^ (w[i] + ORC_GOLDEN));
  return h;
}

static uint64_t orc_key1(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  uint64_t w = (a & 0xFFFFFFFFull) | (b << 32);
  return orc_hash(seed, tag, &w, 1);
}

/* y_{e,p}: the variable of edge e = (src, dst, t) at walk position p
 * (App. C: one y per temporal edge and position). */
static uint64_t orc_y(uint64_t seed, uint32_t src, uint32_t dst, uint32_t t, uint32_t p) {
  uint64_t w[2];
  w[0] = (uint64_t)src | ((uint64_t)dst << 32);
  w[1] = (uint64_t)t | ((uint64_t)p << 32);
  return orc_hash(seed, 'Y', w, 2);
}

/* ---------------------------------------------------------------------------
 * Substitution table z_{u,j}, j = 1..k.
 * Path mode: z_{u,j} uniform in the field (Sec. 4.3, before the multilinear
 * sieving lemma). Motif mode (Sec. 4.4, Eq. multilinear:3): colour s owns
 * mu(s) shades; z_{u,j} = sum over shades d of c(u) of gamma_{u,d} omega_{d,j}.
 * Shades are numbered 0..k-1, contiguous per colour, colours ascending.
 * ------------------------------------------------------------------------ */
int orc_z_table(uint32_t n, const uint8_t* colour, uint32_t n_colours, uint32_t k,
                const uint8_t* motif_count, uint64_t seed, uint64_t* z_out) {
  if (k < 1 || !z_out) return -1;
  if (!motif_count) {
    for (uint32_t u = 0; u < n; u++)
      for (uint32_t j = 1; j <= k; j++) z_out[(uint64_t)u * k + (j - 1)] = orc_key1(seed, 'Z', u, j);
    return 0;
  }
  if (!colour || n_colours == 0 || n_colours > 256) return -1;
  uint32_t total = 0;
  uint32_t off[257];
  for (uint32_t s = 0; s < n_colours; s++) {
    off[s] = total;
    total += motif_count[s];
  }
  if (total != k) return -1;
  for (uint32_t u = 0; u < n; u++) {
    uint32_t s = colour[u];
    if (s >= n_colours) return -1;
    for (uint32_t j = 1; j <= k; j++) {
      uint64_t acc = 0;
      for (uint32_t r = 0; r < motif_count[s]; r++) {
        uint32_t d = off[s] + r;
        acc ^= orc_gf_mul_nibble(orc_key1(seed, 'G', u, d), orc_key1(seed, 'W', d, j));
      }
      z_out[(uint64_t)u * k + (j - 1)] = acc;
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Temporal graph (Sec. 2): E is a set of triples (u, v, j), j >= 1. Duplicates
 * collapse; self-loops are removed (a self-loop repeats its vertex, so it is
 * on no path, and every walk through it cancels in the sieve).
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t src, dst, t;
} orc_edge;

static int orc_edge_cmp(const void* pa, const void* pb) {
  const orc_edge* a = (const orc_edge*)pa;
  const orc_edge* b = (const orc_edge*)pb;
  if (a->dst != b->dst) return a->dst < b->dst ? -1 : 1;
  if (a->t != b->t) return a->t < b->t ? -1 : 1;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  return 0;
}

static int orc_canon(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                     const uint32_t* t, orc_edge** out, uint64_t* m_out) {
  orc_edge* e = (orc_edge*)malloc(sizeof(orc_edge) * (m ? m : 1));
  if (!e) return -2;
  uint64_t c = 0;
  for (uint64_t i = 0; i < m; i++) {
    if (src[i] >= n || dst[i] >= n || t[i] < 1) {
      free(e);
      return -1;
    }
    if (src[i] == dst[i]) continue;
    e[c].src = src[i];
    e[c].dst = dst[i];
    e[c].t = t[i];
    c++;
  }
  qsort(e, c, sizeof(orc_edge), orc_edge_cmp);
  uint64_t w = 0;
  for (uint64_t i = 0; i < c; i++)
    if (w == 0 || orc_edge_cmp(&e[w - 1], &e[i]) != 0) e[w++] = e[i];
  *out = e;
  *m_out = w;
  return 0;
}

static int orc_check_query(uint32_t n, const uint8_t* colour, uint32_t n_colours, uint32_t k,
                           const uint32_t* delta, const uint8_t* motif_count) {
  if (k < 2 || k > 24 || !delta) return -1;
  if (motif_count) {
    if (!colour || n_colours == 0 || n_colours > 256) return -1;
    uint32_t s = 0;
    for (uint32_t c = 0; c < n_colours; c++) s += motif_count[c];
    if (s != k) return -1;
    for (uint32_t u = 0; u < n; u++)
      if (colour[u] >= n_colours) return -1;
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * The sieve (Alg. 1 with the readings fixed in the header):
 *   for every subset L of [k] (iteration index i <-> L):
 *     z^L_u = sum_{j in L} z_{u,j}
 *     chi_{u,2,i}   = z^L_u * sum_{v in N_i(u)} y_{(v,u,i),1} * z^L_v
 *     chi_{u,l,i}   = z^L_u * sum_{v in N_i(u)} y_{(v,u,i),l-1}
 *                            * sum_{j = 0..delta(v), i-j >= 1} chi_{v,l-1,i-j}
 *     f_L = sum over (u, i) of chi_{u,k,i}
 *   F = sum over L of f_L.
 * This is Eq. (poly-enc:1) with y taken per (edge, position) as App. C and
 * Sec. 5.1 define it, level 1 counted once per start vertex, and the
 * per-(u, i) tests of Alg. 1 aggregated into one sum. Values chi_{v,l,i} are
 * stored only for the (v, i) that have an arriving edge; every other value is
 * zero, so skipping them leaves each sum unchanged.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n;
  uint64_t m;
  orc_edge* e;         /* sorted by (dst, t, src) */
  uint64_t n_slots;    /* distinct (dst, t) pairs */
  uint64_t* v_off;     /* [n+1] slot range of each vertex */
  uint32_t* slot_t;    /* [n_slots] arrival time of the slot */
  uint64_t* slot_e;    /* [n_slots+1] edge range of the slot */
} orc_graph;

static void orc_graph_free(orc_graph* g) {
  free(g->e);
  free(g->v_off);
  free(g->slot_t);
  free(g->slot_e);
}

static int orc_graph_build(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                           const uint32_t* t, orc_graph* g) {
  memset(g, 0, sizeof(*g));
  g->n = n;
  int rc = orc_canon(n, m, src, dst, t, &g->e, &g->m);
  if (rc) return rc;
  uint64_t ns = 0;
  for (uint64_t i = 0; i < g->m; i++)
    if (i == 0 || g->e[i].dst != g->e[i - 1].dst || g->e[i].t != g->e[i - 1].t) ns++;
  g->n_slots = ns;
  g->v_off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  g->slot_t = (uint32_t*)malloc(sizeof(uint32_t) * (ns ? ns : 1));
  g->slot_e = (uint64_t*)malloc(sizeof(uint64_t) * (ns + 1));
  if (!g->v_off || !g->slot_t || !g->slot_e) {
    orc_graph_free(g);
    return -2;
  }
  uint64_t s = 0;
  for (uint64_t i = 0; i < g->m; i++) {
    if (i == 0 || g->e[i].dst != g->e[i - 1].dst || g->e[i].t != g->e[i - 1].t) {
      g->slot_t[s] = g->e[i].t;
      g->slot_e[s] = i;
      g->v_off[g->e[i].dst + 1]++;
      s++;
    }
  }
  g->slot_e[ns] = g->m;
  for (uint32_t u = 0; u < n; u++) g->v_off[u + 1] += g->v_off[u];
  return 0;
}

/* Sum over j = 0..delta(v) with i - j >= 1 of chi_{v,l-1,i-j}. The terms at
 * times where v has no arrival are zero, so the sum runs over the arrival
 * slots of v whose time lies in [max(1, i - delta(v)), i]. */
static uint64_t orc_window(const orc_graph* g, const uint64_t* chi, uint32_t v, uint32_t i,
                           uint32_t dv) {
  int64_t first = (int64_t)i - (int64_t)dv;
  if (first < 1) first = 1;
  /* locate the first slot of v with time >= first */
  uint64_t lo = g->v_off[v], hi = g->v_off[v + 1];
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if ((int64_t)g->slot_t[mid] < first)
      lo = mid + 1;
    else
      hi = mid;
  }
  uint64_t acc = 0;
  for (uint64_t s = lo; s < g->v_off[v + 1] && g->slot_t[s] <= i; s++) acc ^= chi[s];
  return acc;
}

/* chi_{u,k,i} for every slot (u, i), for one subset L (bit j-1 of L <-> j in
 * L): levels 1..k of Eq. (poly-enc:1). With source_mask != NULL only the
 * vertices u with source_mask[u] != 0 carry a level-1 term (chi_{u,1,i} =
 * z^L_u for them, 0 for every other vertex), so only walks that start in
 * that set are generated: the source constraint of the reachability problems
 * of Sec. 3. Returns the array (chi_a or chi_b) that holds level k. */
static uint64_t* orc_levels_L(const orc_graph* g, const uint64_t* z, uint32_t k, const uint32_t* delta,
                              const uint8_t* source_mask, uint64_t seed, uint64_t L, uint64_t* zL,
                              uint64_t* chi_a, uint64_t* chi_b) {
  uint64_t* chi_prev = chi_a;
  uint64_t* chi_cur = chi_b;
  for (uint32_t u = 0; u < g->n; u++) {
    uint64_t s = 0;
    for (uint32_t j = 1; j <= k; j++)
      if ((L >> (j - 1)) & 1) s ^= z[(uint64_t)u * k + (j - 1)];
    zL[u] = s;
  }
  /* level 2 */
  for (uint32_t u = 0; u < g->n; u++) {
    for (uint64_t sl = g->v_off[u]; sl < g->v_off[u + 1]; sl++) {
      uint64_t acc = 0;
      for (uint64_t ei = g->slot_e[sl]; ei < g->slot_e[sl + 1]; ei++) {
        const orc_edge* e = &g->e[ei];
        if (source_mask && !source_mask[e->src]) continue; /* chi_{src,1,.} = 0 */
        acc ^= orc_gf_mul_nibble(orc_y(seed, e->src, e->dst, e->t, 1), zL[e->src]);
      }
      chi_prev[sl] = orc_gf_mul_nibble(zL[u], acc);
    }
  }
  /* levels 3..k */
  for (uint32_t l = 3; l <= k; l++) {
    for (uint32_t u = 0; u < g->n; u++) {
      for (uint64_t sl = g->v_off[u]; sl < g->v_off[u + 1]; sl++) {
        uint64_t acc = 0;
        for (uint64_t ei = g->slot_e[sl]; ei < g->slot_e[sl + 1]; ei++) {
          const orc_edge* e = &g->e[ei];
          uint64_t w = orc_window(g, chi_prev, e->src, e->t, delta[e->src]);
          acc ^= orc_gf_mul_nibble(orc_y(seed, e->src, e->dst, e->t, l - 1), w);
        }
        chi_cur[sl] = orc_gf_mul_nibble(zL[u], acc);
      }
    }
    uint64_t* tmp = chi_prev;
    chi_prev = chi_cur;
    chi_cur = tmp;
  }
  return chi_prev;
}

/* f_L for one subset L: the sum of chi_{u,k,i} over all slots (u, i), or,
 * with target_mask != NULL, over the slots of the vertices u with
 * target_mask[u] != 0 (paths ending in that set: the destination of the
 * problems of Sec. 3). */
static uint64_t orc_eval_L(const orc_graph* g, const uint64_t* z, uint32_t k, const uint32_t* delta,
                           const uint8_t* source_mask, const uint8_t* target_mask, uint64_t seed, uint64_t L,
                           uint64_t* zL, uint64_t* chi_a, uint64_t* chi_b) {
  const uint64_t* chi = orc_levels_L(g, z, k, delta, source_mask, seed, L, zL, chi_a, chi_b);
  uint64_t f = 0;
  for (uint32_t u = 0; u < g->n; u++) {
    if (target_mask && !target_mask[u]) continue;
    for (uint64_t sl = g->v_off[u]; sl < g->v_off[u + 1]; sl++) f ^= chi[sl];
  }
  return f;
}

int orc_sieve(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
              const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
              uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
              uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
              uint64_t* F_out, uint64_t* per_it) {
  return orc_sieve_ex(n, m, src, dst, t, colour, n_colours, k, delta, motif_count, NULL, NULL, seed, it_begin,
                      it_end, threads, F_out, per_it);
}

int orc_sieve_ex(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                 const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                 uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                 const uint8_t* source_mask, const uint8_t* target_mask,
                 uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
                 uint64_t* F_out, uint64_t* per_it) {
  if (!F_out) return -1;
  int rc = orc_check_query(n, colour, n_colours, k, delta, motif_count);
  if (rc) return rc;
  uint64_t total = 1ull << k;
  if (it_begin == 0 && it_end == 0) it_end = total;
  if (it_begin > it_end || it_end > total) return -1;
  orc_graph g;
  rc = orc_graph_build(n, m, src, dst, t, &g);
  if (rc) return rc;
  uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n * k + 1));
  if (!z) {
    orc_graph_free(&g);
    return -2;
  }
  rc = orc_z_table(n, colour, n_colours, k, motif_count, seed, z);
  if (rc) {
    free(z);
    orc_graph_free(&g);
    return rc;
  }
  uint64_t F = 0;
  int nthr = threads > 1 ? threads : 1;
  int failed = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthr) reduction(^ : F) reduction(| : failed)
#endif
  {
    uint64_t* zL = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n + 1));
    uint64_t* c0 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
    uint64_t* c1 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
    if (!zL || !c0 || !c1) {
      failed = 1;
    } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
      for (int64_t it = (int64_t)it_begin; it < (int64_t)it_end; it++) {
        uint64_t f = orc_eval_L(&g, z, k, delta, source_mask, target_mask, seed, (uint64_t)it, zL, c0, c1);
        if (per_it) per_it[(uint64_t)it - it_begin] = f;
        F ^= f;
      }
    }
    free(zL);
    free(c0);
    free(c1);
  }
  free(z);
  orc_graph_free(&g);
  if (failed) return -2;
  *F_out = F;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Fine-grained oracle (Alg. 1, FineGrainedOracle): per slot (u, i), the sum
 * over L of chi_{u,k,i}, i.e. zeta_{u,k,i}, without summing over (u, i).
 * zeta_{u,k,i} != 0 says a restless path with k vertices ending at u at time
 * i exists (Sec. 4.5); R_u is the least such i and D the vertices that have
 * one. zeta_edge (may be NULL; m entries) receives, for each canonical edge
 * (deduplicated, self-loops dropped, sorted by (dst, t, src)) in that order,
 * the zeta of its slot (dst, t); *m_canon_out its number of edges. reach_out
 * (n entries) receives R_u, or 0xFFFFFFFF where no slot of u is non-zero.
 * F_out (may be NULL) receives the sum of zeta over the slots of the target
 * vertices (all vertices when target_mask is NULL), which equals the
 * orc_sieve_ex fingerprint of the same query.
 * ------------------------------------------------------------------------ */
int orc_fine_grained(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                     const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                     uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                     const uint8_t* source_mask, const uint8_t* target_mask, uint64_t seed,
                     uint64_t it_begin, uint64_t it_end, int threads, uint64_t* zeta_edge,
                     uint64_t* m_canon_out, uint32_t* reach_out, uint64_t* F_out) {
  if (!reach_out) return -1;
  int rc = orc_check_query(n, colour, n_colours, k, delta, motif_count);
  if (rc) return rc;
  uint64_t total = 1ull << k;
  if (it_begin == 0 && it_end == 0) it_end = total;
  if (it_begin > it_end || it_end > total) return -1;
  orc_graph g;
  rc = orc_graph_build(n, m, src, dst, t, &g);
  if (rc) return rc;
  uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n * k + 1));
  uint64_t* zeta = (uint64_t*)calloc(g.n_slots + 1, sizeof(uint64_t));
  if (!z || !zeta) {
    free(z);
    free(zeta);
    orc_graph_free(&g);
    return -2;
  }
  rc = orc_z_table(n, colour, n_colours, k, motif_count, seed, z);
  int nthr = threads > 1 ? threads : 1;
  int failed = 0;
  if (!rc) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nthr) reduction(| : failed)
#endif
    {
      uint64_t* zL = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n + 1));
      uint64_t* c0 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
      uint64_t* c1 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
      uint64_t* mine = (uint64_t*)calloc(g.n_slots + 1, sizeof(uint64_t));
      if (!zL || !c0 || !c1 || !mine) {
        failed = 1;
      } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t it = (int64_t)it_begin; it < (int64_t)it_end; it++) {
          const uint64_t* chi = orc_levels_L(&g, z, k, delta, source_mask, seed, (uint64_t)it, zL, c0, c1);
          for (uint64_t sl = 0; sl < g.n_slots; sl++) mine[sl] ^= chi[sl];
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        for (uint64_t sl = 0; sl < g.n_slots; sl++) zeta[sl] ^= mine[sl];
      }
      free(zL);
      free(c0);
      free(c1);
      free(mine);
    }
  }
  if (!rc && !failed) {
    uint64_t F = 0;
    for (uint32_t u = 0; u < n; u++) {
      reach_out[u] = 0xFFFFFFFFu;
      for (uint64_t sl = g.v_off[u]; sl < g.v_off[u + 1]; sl++) {
        if (target_mask && !target_mask[u]) zeta[sl] = 0; /* only paths ending at a target count */
        F ^= zeta[sl];
        if (zeta[sl] && g.slot_t[sl] < reach_out[u]) reach_out[u] = g.slot_t[sl];
      }
    }
    if (zeta_edge)
      for (uint64_t sl = 0; sl < g.n_slots; sl++)
        for (uint64_t ei = g.slot_e[sl]; ei < g.slot_e[sl + 1]; ei++) zeta_edge[ei] = zeta[sl];
    if (m_canon_out) *m_canon_out = g.m;
    if (F_out) *F_out = F;
  }
  free(z);
  free(zeta);
  orc_graph_free(&g);
  if (rc) return rc;
  return failed ? -2 : 0;
}

/* ---------------------------------------------------------------------------
 * Literal reading of Eq. (poly-enc:1): the y variable of a window term is
 * indexed by the edge's end points, the level and the predecessor's arrival
 * time i - j (y_{uv, l-1, i-j}), not by the edge's own time, and level 1 is
 * x_u at every time i in [tau], so a path also takes a term for each time it
 * may have waited at its first vertex. Each window term has its own y, so an
 * edge-update costs delta(v) + 1 products (the evaluation-cost lemma of
 * Sec. 4.3). Two paths that differ only in the time of their last edge share
 * every variable, so their terms cancel in a sum over end times; each slot
 * (u, i) is therefore tested on its own (Alg. 1's per-slot test).
 * ------------------------------------------------------------------------ */

/* y_{uv, l, p}: the literal variable of the edge from v (src) to u (dst) at
 * level l for a predecessor that arrived at v at time p. */
static uint64_t orc_y_literal(uint64_t seed, uint32_t src, uint32_t dst, uint32_t p, uint32_t l) {
  uint64_t w[2];
  w[0] = (uint64_t)src | ((uint64_t)dst << 32);
  w[1] = (uint64_t)p | ((uint64_t)l << 32);
  return orc_hash(seed, 'P', w, 2);
}

/* chi_{v,l,p} of a level >= 2: the value of slot (v, p), or 0 when v has no
 * arrival at time p. */
static uint64_t orc_chi_at(const orc_graph* g, const uint64_t* chi, uint32_t v, uint32_t p) {
  uint64_t lo = g->v_off[v], hi = g->v_off[v + 1];
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (g->slot_t[mid] < p)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < g->v_off[v + 1] && g->slot_t[lo] == p) ? chi[lo] : 0;
}

/* chi_{u,k,i} for every slot (u, i), for one subset L, by the literal
 * recurrence: for each in-edge from v at time i and each j = 0..delta(v) with
 * i - j > 0, the term y_{uv,l-1,i-j} chi_{v,l-1,i-j}; level 1 is z^L_v at
 * every time. Returns the array that holds level k. */
static uint64_t* orc_literal_levels_L(const orc_graph* g, const uint64_t* z, uint32_t k, const uint32_t* delta,
                                      uint64_t seed, uint64_t L, uint64_t* zL, uint64_t* chi_a, uint64_t* chi_b) {
  uint64_t* chi_prev = chi_a;
  uint64_t* chi_cur = chi_b;
  for (uint32_t u = 0; u < g->n; u++) {
    uint64_t s = 0;
    for (uint32_t j = 1; j <= k; j++)
      if ((L >> (j - 1)) & 1) s ^= z[(uint64_t)u * k + (j - 1)];
    zL[u] = s;
  }
  for (uint32_t l = 2; l <= k; l++) {
    for (uint32_t u = 0; u < g->n; u++) {
      for (uint64_t sl = g->v_off[u]; sl < g->v_off[u + 1]; sl++) {
        const uint32_t i = g->slot_t[sl];
        uint64_t acc = 0;
        for (uint64_t ei = g->slot_e[sl]; ei < g->slot_e[sl + 1]; ei++) {
          const uint32_t v = g->e[ei].src;
          for (uint32_t j = 0; j <= delta[v] && j < i; j++) {
            const uint64_t prev = l == 2 ? zL[v] : orc_chi_at(g, chi_prev, v, i - j);
            acc ^= orc_gf_mul_nibble(orc_y_literal(seed, v, u, i - j, l - 1), prev);
          }
        }
        chi_cur[sl] = orc_gf_mul_nibble(zL[u], acc);
      }
    }
    uint64_t* tmp = chi_prev;
    chi_prev = chi_cur;
    chi_cur = tmp;
  }
  return chi_prev;
}

int orc_fine_literal(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const uint32_t* t,
                     const uint8_t* colour, uint32_t n_colours, uint32_t k, const uint32_t* delta,
                     const uint8_t* motif_count, uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
                     uint64_t* zeta_edge, uint64_t* m_canon_out, uint32_t* reach_out) {
  if (!reach_out) return -1;
  int rc = orc_check_query(n, colour, n_colours, k, delta, motif_count);
  if (rc) return rc;
  uint64_t total = 1ull << k;
  if (it_begin == 0 && it_end == 0) it_end = total;
  if (it_begin > it_end || it_end > total) return -1;
  orc_graph g;
  rc = orc_graph_build(n, m, src, dst, t, &g);
  if (rc) return rc;
  uint64_t* z = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n * k + 1));
  uint64_t* zeta = (uint64_t*)calloc(g.n_slots + 1, sizeof(uint64_t));
  if (!z || !zeta) {
    free(z);
    free(zeta);
    orc_graph_free(&g);
    return -2;
  }
  rc = orc_z_table(n, colour, n_colours, k, motif_count, seed, z);
  int nthr = threads > 1 ? threads : 1;
  int failed = 0;
  if (!rc) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nthr) reduction(| : failed)
#endif
    {
      uint64_t* zL = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n + 1));
      uint64_t* c0 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
      uint64_t* c1 = (uint64_t*)malloc(sizeof(uint64_t) * (g.n_slots + 1));
      uint64_t* mine = (uint64_t*)calloc(g.n_slots + 1, sizeof(uint64_t));
      if (!zL || !c0 || !c1 || !mine) {
        failed = 1;
      } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t it = (int64_t)it_begin; it < (int64_t)it_end; it++) {
          const uint64_t* chi = orc_literal_levels_L(&g, z, k, delta, seed, (uint64_t)it, zL, c0, c1);
          for (uint64_t sl = 0; sl < g.n_slots; sl++) mine[sl] ^= chi[sl];
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        for (uint64_t sl = 0; sl < g.n_slots; sl++) zeta[sl] ^= mine[sl];
      }
      free(zL);
      free(c0);
      free(c1);
      free(mine);
    }
  }
  if (!rc && !failed) {
    for (uint32_t u = 0; u < n; u++) {
      reach_out[u] = 0xFFFFFFFFu;
      for (uint64_t sl = g.v_off[u]; sl < g.v_off[u + 1]; sl++)
        if (zeta[sl] && g.slot_t[sl] < reach_out[u]) reach_out[u] = g.slot_t[sl];
    }
    if (zeta_edge)
      for (uint64_t sl = 0; sl < g.n_slots; sl++)
        for (uint64_t ei = g.slot_e[sl]; ei < g.slot_e[sl + 1]; ei++) zeta_edge[ei] = zeta[sl];
    if (m_canon_out) *m_canon_out = g.m;
  }
  free(z);
  free(zeta);
  orc_graph_free(&g);
  if (rc) return rc;
  return failed ? -2 : 0;
}

/* ---------------------------------------------------------------------------
 * Determinants over GF(2^64).
 * ------------------------------------------------------------------------ */
uint64_t orc_gf_det(const uint64_t* a, int k) {
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(k * k + 1));
  memcpy(w, a, sizeof(uint64_t) * (size_t)(k * k));
  uint64_t det = 1;
  for (int c = 0; c < k; c++) {
    int p = -1;
    for (int r = c; r < k; r++)
      if (w[r * k + c]) {
        p = r;
        break;
      }
    if (p < 0) {
      free(w);
      return 0;
    }
    if (p != c)
      for (int j = 0; j < k; j++) {
        uint64_t x = w[p * k + j];
        w[p * k + j] = w[c * k + j];
        w[c * k + j] = x;
      }
    det = orc_gf_mul(det, w[c * k + c]);
    uint64_t inv = orc_gf_inv(w[c * k + c]);
    for (int r = c + 1; r < k; r++) {
      uint64_t f = orc_gf_mul(w[r * k + c], inv);
      if (!f) continue;
      for (int j = c; j < k; j++) w[r * k + j] ^= orc_gf_mul(f, w[c * k + j]);
    }
  }
  free(w);
  return det;
}

static uint64_t orc_leibniz_rec(const uint64_t* a, int k, int row, uint32_t used, uint64_t prod) {
  if (row == k) return prod;
  uint64_t s = 0;
  for (int c = 0; c < k; c++)
    if (!((used >> c) & 1)) s ^= orc_leibniz_rec(a, k, row + 1, used | (1u << c), orc_gf_mul(prod, a[row * k + c]));
  return s;
}

uint64_t orc_gf_det_leibniz(const uint64_t* a, int k) {
  if (k < 0 || k > 8) return 0;
  return orc_leibniz_rec(a, k, 0, 0, 1);
}

/* ---------------------------------------------------------------------------
 * Restless path enumeration (Sec. 2 definitions; the exhaustive temporal DFS
 * of Sec. 5.3): vertices v_1..v_k distinct, edges e_p = (v_p, v_{p+1}, t_p),
 * 0 <= t_{p+1} - t_p <= delta(v_{p+1}).
 * ------------------------------------------------------------------------ */
typedef struct {
  const orc_graph* g;
  uint64_t* out_off; /* [n+1] */
  uint64_t* out_e;   /* edge ids grouped by source */
  uint32_t k;
  const uint32_t* delta;
  const uint8_t* colour;
  const uint8_t* motif;
  uint32_t n_colours;
  const uint64_t* z; /* closed form only */
  uint64_t seed;
  const uint8_t* source_mask; /* NULL = any start vertex */
  const uint8_t* target_mask; /* NULL = any end vertex */
  uint64_t* acc_edge;         /* NULL, or per canonical edge: sum of the paths whose last edge it is */
  uint64_t* cnt_edge;         /* NULL, or per canonical edge: number of those paths */
  uint32_t path_v[32];
  uint64_t path_e[32];
  uint64_t count;
  uint64_t F;
  int closed;
} orc_dfs;

static int orc_colours_agree(const orc_dfs* d) {
  uint32_t cnt[256];
  memset(cnt, 0, sizeof(cnt));
  for (uint32_t p = 0; p < d->k; p++) cnt[d->colour[d->path_v[p]]]++;
  for (uint32_t s = 0; s < d->n_colours; s++)
    if (cnt[s] != d->motif[s]) return 0;
  for (uint32_t s = d->n_colours; s < 256; s++)
    if (cnt[s]) return 0;
  return 1;
}

static void orc_dfs_record(orc_dfs* d) {
  if (d->target_mask && !d->target_mask[d->path_v[d->k - 1]]) return;
  const uint64_t last = d->path_e[d->k - 2];
  if (!d->closed) {
    if (!d->motif || orc_colours_agree(d)) {
      d->count++;
      if (d->cnt_edge) d->cnt_edge[last]++;
    }
    return;
  }
  d->count++;
  if (d->cnt_edge && (!d->motif || orc_colours_agree(d))) d->cnt_edge[last]++;
  uint64_t Y = 1;
  for (uint32_t p = 1; p < d->k; p++) {
    const orc_edge* e = &d->g->e[d->path_e[p - 1]];
    Y = orc_gf_mul(Y, orc_y(d->seed, e->src, e->dst, e->t, p));
  }
  uint64_t Z[32 * 32];
  for (uint32_t p = 0; p < d->k; p++)
    for (uint32_t j = 0; j < d->k; j++) Z[p * d->k + j] = d->z[(uint64_t)d->path_v[p] * d->k + j];
  const uint64_t term = orc_gf_mul(Y, orc_gf_det(Z, (int)d->k));
  d->F ^= term;
  if (d->acc_edge) d->acc_edge[last] ^= term;
}

static void orc_dfs_extend(orc_dfs* d, uint32_t depth, uint32_t last_t) {
  /* depth = number of vertices on the path so far */
  if (depth == d->k) {
    orc_dfs_record(d);
    return;
  }
  uint32_t v = d->path_v[depth - 1];
  for (uint64_t i = d->out_off[v]; i < d->out_off[v + 1]; i++) {
    const orc_edge* e = &d->g->e[d->out_e[i]];
    if (depth >= 2) {
      if (e->t < last_t) continue;
      if ((uint64_t)e->t - last_t > d->delta[v]) continue;
    }
    int seen = 0;
    for (uint32_t p = 0; p < depth; p++)
      if (d->path_v[p] == e->dst) seen = 1;
    if (seen) continue;
    d->path_v[depth] = e->dst;
    d->path_e[depth - 1] = d->out_e[i];
    orc_dfs_extend(d, depth + 1, e->t);
  }
}

static int orc_enumerate(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                         const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                         uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                         const uint8_t* source_mask, const uint8_t* target_mask,
                         uint64_t seed, int closed, uint64_t* F_out, uint64_t* count_out,
                         uint64_t* zeta_edge, uint64_t* count_edge, uint64_t* m_canon_out) {
  int rc = orc_check_query(n, colour, n_colours, k, delta, motif_count);
  if (rc) return rc;
  if (k > 32) return -1;
  orc_graph g;
  rc = orc_graph_build(n, m, src, dst, t, &g);
  if (rc) return rc;
  orc_dfs d;
  memset(&d, 0, sizeof(d));
  d.g = &g;
  d.k = k;
  d.delta = delta;
  d.colour = colour;
  d.motif = motif_count;
  d.n_colours = n_colours;
  d.seed = seed;
  d.closed = closed;
  d.source_mask = source_mask;
  d.target_mask = target_mask;
  d.out_off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  d.out_e = (uint64_t*)malloc(sizeof(uint64_t) * (g.m ? g.m : 1));
  if (zeta_edge) d.acc_edge = (uint64_t*)calloc(g.m + 1, sizeof(uint64_t));
  if (count_edge) d.cnt_edge = (uint64_t*)calloc(g.m + 1, sizeof(uint64_t));
  uint64_t* z = NULL;
  if (closed) {
    z = (uint64_t*)malloc(sizeof(uint64_t) * ((uint64_t)n * k + 1));
    rc = orc_z_table(n, colour, n_colours, k, motif_count, seed, z);
    d.z = z;
  }
  if (!rc) {
    for (uint64_t i = 0; i < g.m; i++) d.out_off[g.e[i].src + 1]++;
    for (uint32_t v = 0; v < n; v++) d.out_off[v + 1] += d.out_off[v];
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    memcpy(fill, d.out_off, sizeof(uint64_t) * ((size_t)n + 1));
    for (uint64_t i = 0; i < g.m; i++) d.out_e[fill[g.e[i].src]++] = i;
    free(fill);
    for (uint32_t v = 0; v < n; v++) {
      if (source_mask && !source_mask[v]) continue;
      d.path_v[0] = v;
      orc_dfs_extend(&d, 1, 0);
    }
    if (F_out) *F_out = d.F;
    if (count_out) *count_out = d.count;
    /* per slot (dst, t): the sum (count) over the slot's edges, stored at each of them */
    for (uint64_t sl = 0; sl < g.n_slots; sl++) {
      uint64_t zs = 0, cs = 0;
      for (uint64_t ei = g.slot_e[sl]; ei < g.slot_e[sl + 1]; ei++) {
        if (d.acc_edge) zs ^= d.acc_edge[ei];
        if (d.cnt_edge) cs += d.cnt_edge[ei];
      }
      for (uint64_t ei = g.slot_e[sl]; ei < g.slot_e[sl + 1]; ei++) {
        if (zeta_edge) zeta_edge[ei] = zs;
        if (count_edge) count_edge[ei] = cs;
      }
    }
    if (m_canon_out) *m_canon_out = g.m;
  }
  free(z);
  free(d.out_off);
  free(d.out_e);
  free(d.acc_edge);
  free(d.cnt_edge);
  orc_graph_free(&g);
  return rc;
}

int orc_closed_form(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                    const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                    uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                    uint64_t seed, uint64_t* F_out, uint64_t* n_paths_out) {
  return orc_enumerate(n, m, src, dst, t, colour, n_colours, k, delta, motif_count, NULL, NULL, seed, 1, F_out,
                       n_paths_out, NULL, NULL, NULL);
}

int orc_closed_form_ex(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                       const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                       uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                       const uint8_t* source_mask, const uint8_t* target_mask, uint64_t seed,
                       uint64_t* F_out, uint64_t* n_paths_out, uint64_t* zeta_edge, uint64_t* count_edge,
                       uint64_t* m_canon_out) {
  return orc_enumerate(n, m, src, dst, t, colour, n_colours, k, delta, motif_count, source_mask, target_mask, seed,
                       1, F_out, n_paths_out, zeta_edge, count_edge, m_canon_out);
}

int orc_count_paths(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                    const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                    uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                    uint64_t* count_out) {
  return orc_enumerate(n, m, src, dst, t, colour, n_colours, k, delta, motif_count, NULL, NULL, 0, 0, NULL,
                       count_out, NULL, NULL, NULL);
}
