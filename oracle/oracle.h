/*
 * Plain CPU oracle for the restless-path / restless-motif sieve fingerprint.
 *
 * TEST INFRASTRUCTURE ONLY. This header and oracle.c are the slow, obviously
 * correct reference the GPU library is checked against. Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it. It shares
 * no code, header, table or constant generator with the GPU library, and the
 * GPU library never calls it.
 *
 * What is computed (Thejaswi, Lauri, Gionis, "Restless reachability problems
 * in temporal graphs", arXiv 2010.08423):
 *   - GF(2^64) arithmetic (Sec. 4.2 and Sec. 5.1 fix b = 64; the reduction
 *     polynomial x^64 + x^4 + x^3 + x + 1 is this project's choice).
 *   - the restless-walk generating function, Eq. (poly-enc:1) of Sec. 4.3,
 *     evaluated at one point per sieve subset L;
 *   - multilinear sieving, Eq. (multilinear:1), and its colour-constrained
 *     form with shades, Eq. (multilinear:3) and Eq. (multilinear:2), Sec. 4.4;
 *   - the sum over subsets L of Alg. 1 (FineGrainedOracle), aggregated over
 *     all end vertices and end times into one fingerprint F.
 *   - brute-force restless-path enumeration (the exhaustive temporal DFS the
 *     paper uses as its baseline, Sec. 5.3) and the closed form
 *     F = XOR over restless paths P of (prod_p y_{e_p,p}) * det Z_P.
 *
 * Conventions shared with the GPU library only by specification (each side
 * implements them independently):
 *   - element bit i = coefficient of x^i; addition = XOR;
 *   - mix64 = SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014);
 *     H(seed, tag, w_1..w_r): h = mix64(seed + tag * G);
 *     h = mix64(h ^ (w_i + G)) for each word; result h; G = 0x9E3779B97F4A7C15.
 *   - z_{u,j} = H(seed,'Z', u | j<<32), j = 1..k      (path mode)
 *     gamma_{u,d} = H(seed,'G', u | d<<32), d = 0..k-1 (shade ids)
 *     omega_{d,j} = H(seed,'W', d | j<<32)
 *     y_{e,p} = H(seed,'Y', src | dst<<32, t | p<<32), p = 1..k-1
 *   - iteration i in [0, 2^k) <-> L(i) = { j : bit j-1 of i set }.
 *
 * Every function returns 0 on success, a negative value on invalid input.
 */
#ifndef RESTLESS_ORACLE_H
#define RESTLESS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* GF(2^64): definition-level product (shift-and-add, then reduce). */
uint64_t orc_gf_mul(uint64_t a, uint64_t b);
/* GF(2^64): second, independent formulation (Horner over 4-bit digits of a
 * with a table of reduced multiples of b); used by the sieve for speed and
 * cross-checked against orc_gf_mul. */
uint64_t orc_gf_mul_nibble(uint64_t a, uint64_t b);
uint64_t orc_gf_pow(uint64_t a, uint64_t e);
/* a^(2^64 - 2); the inverse for a != 0, 0 for a == 0. */
uint64_t orc_gf_inv(uint64_t a);

uint64_t orc_mix64(uint64_t x);
uint64_t orc_hash(uint64_t seed, uint64_t tag, const uint64_t* w, int nw);

/* z table, row-major [n][k], entry (u, j-1) = z_{u,j} (path mode) or the
 * shade sum of Eq. (multilinear:3) (motif mode, motif_count != NULL). */
int orc_z_table(uint32_t n, const uint8_t* colour, uint32_t n_colours, uint32_t k,
                const uint8_t* motif_count, uint64_t seed, uint64_t* z_out);

/* Sieve fingerprint over iterations [it_begin, it_end) (both 0 -> all 2^k).
 * delta: per-vertex resting time, length n.
 * per_it (may be NULL): receives f_L for each iteration of the range.
 * threads: 1 = single thread; >1 = OpenMP over iterations. */
int orc_sieve(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
              const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
              uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
              uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
              uint64_t* F_out, uint64_t* per_it);

/* As orc_sieve, with the source and destination constraints of the problems
 * of Sec. 3: source_mask (n bytes, NULL = every vertex) keeps only the walks
 * that start at a vertex u with source_mask[u] != 0 (the level-1 terms of
 * Eq. poly-enc:1 of every other vertex are 0); target_mask (n bytes, NULL =
 * every vertex) sums the last level only over the end vertices u with
 * target_mask[u] != 0. */
int orc_sieve_ex(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                 const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                 uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                 const uint8_t* source_mask, const uint8_t* target_mask,
                 uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
                 uint64_t* F_out, uint64_t* per_it);

/* Fine-grained oracle (Alg. 1, FineGrainedOracle; Sec. 4.5): zeta_{u,k,i},
 * the sum over the iterations of [it_begin, it_end) of the last level's value
 * at slot (u, i), kept per slot. Outputs, for the canonical edge list
 * (deduplicated, self-loops dropped, sorted by (dst, t, src); *m_canon_out
 * edges): zeta_edge[e] = zeta of the slot (dst(e), t(e)) (NULL = not wanted;
 * caller sizes it to m); reach_out[u] = least time i with zeta_{u,k,i} != 0,
 * 0xFFFFFFFF if none (D = the vertices with a finite R_u); F_out (may be NULL)
 * = the sum of all zeta, which is the orc_sieve_ex fingerprint. Masks as in
 * orc_sieve_ex (slots of non-target vertices are 0). */
int orc_fine_grained(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                     const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                     uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                     const uint8_t* source_mask, const uint8_t* target_mask, uint64_t seed,
                     uint64_t it_begin, uint64_t it_end, int threads, uint64_t* zeta_edge,
                     uint64_t* m_canon_out, uint32_t* reach_out, uint64_t* F_out);

/* Fine-grained outputs under the literal reading of Eq. (poly-enc:1): y of
 * a window term indexed by (v, u, level, predecessor arrival time i - j),
 * level 1 = z^L at every time, delta(v) + 1 products per edge-update. Outputs
 * as orc_fine_grained (no masks, no aggregate: the sum over end times cancels
 * paths that differ only in their last edge's time). */
int orc_fine_literal(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const uint32_t* t,
                     const uint8_t* colour, uint32_t n_colours, uint32_t k, const uint32_t* delta,
                     const uint8_t* motif_count, uint64_t seed, uint64_t it_begin, uint64_t it_end, int threads,
                     uint64_t* zeta_edge, uint64_t* m_canon_out, uint32_t* reach_out);

/* Closed form: XOR over all restless paths P with k vertices (motif mode:
 * z from the shade sum, so colour-mismatched paths contribute det = 0) of
 * (prod_p y_{e_p,p}) * det Z_P. n_paths_out counts the paths enumerated
 * (before colour filtering). */
int orc_closed_form(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                    const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                    uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                    uint64_t seed, uint64_t* F_out, uint64_t* n_paths_out);

/* Closed form per slot, with the masks of orc_sieve_ex (paths that start at a
 * source and end at a target): zeta_edge[e] (may be NULL; sized m) = XOR of
 * (prod_p y) det Z_P over the paths whose last edge arrives at the slot
 * (dst(e), t(e)); count_edge[e] (may be NULL) = the number of such paths
 * (colour-agreeing ones in motif mode), for every edge of that slot. */
int orc_closed_form_ex(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                       const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                       uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                       const uint8_t* source_mask, const uint8_t* target_mask, uint64_t seed,
                       uint64_t* F_out, uint64_t* n_paths_out, uint64_t* zeta_edge, uint64_t* count_edge,
                       uint64_t* m_canon_out);

/* Exhaustive temporal DFS: number of restless paths with k vertices whose
 * colours agree with the motif (all paths when motif_count == NULL). */
int orc_count_paths(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                    const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                    uint32_t k, const uint32_t* delta, const uint8_t* motif_count,
                    uint64_t* count_out);

/* det over GF(2^64) of a k x k row-major matrix by Gaussian elimination. */
uint64_t orc_gf_det(const uint64_t* a, int k);
/* Leibniz sum over all permutations (= permanent = determinant in
 * characteristic 2); k <= 8. */
uint64_t orc_gf_det_leibniz(const uint64_t* a, int k);

#ifdef __cplusplus
}
#endif
#endif
