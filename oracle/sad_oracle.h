/*
 * CPU oracle for the Sample-Align-D data-parallel core (Saeed & Khokhar,
 * arXiv 0901.2742).  TEST INFRASTRUCTURE ONLY: this library is the slow,
 * plain reference that the tests, the smoke check and the benchmark's CPU
 * baseline compare the HIP library against.  It shares no code, header or
 * table with the HIP library and must never be called from the product path.
 *
 * All arrays are host memory owned by the caller.  Every function returns one
 * of the status codes below and writes nothing it does not document.
 *
 * Parity status: every step is pinned by tests (brute force, invariants,
 * library special cases); the end-to-end result has no printed example in the
 * paper, so whole-pipeline outputs are pinned only through those invariants.
 */
#ifndef SAD_ORACLE_H
#define SAD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SADREF_OK = 0,
  SADREF_E_INVAL = -1,
  SADREF_E_CAPACITY = -2,
  SADREF_E_OVERFLOW = -3,
};

/* Op codes of an alignment between profile P1 (rows i) and P2 (columns j). */
enum { SADREF_OP_M = 0, SADREF_OP_X = 1, SADREF_OP_Y = 2 };

/* Sorted unique k-mer list of one sequence (Section 2, k-mer counts nx(tau)).
 * taus/counts must hold L-k+1 entries; returns the number of unique k-mers in
 * *n_unique.  tau = sum_u x[t+u] * A^(k-1-u). */
/* Threads for the loops over independent items (sequences, chunks,
 * buckets, refinement alignments); 1 (the default) runs everything on the
 * calling thread.  Results do not depend on it. */
void sadref_set_threads(int32_t threads);

int sadref_kmer_list(const uint8_t* x, int64_t L, int A, int k,
                     int32_t* taus, int32_t* counts, int64_t* n_unique);

/* c = sum_tau min(n_i(tau), n_j(tau)) (numerator of r_ij, Section 2). */
int64_t sadref_common_kmers(const uint8_t* xi, int64_t Li, const uint8_t* xj, int64_t Lj,
                            int A, int k);

/* Fixed-point similarity floor(c * 2^31 / d), d = min(Li, Lj) - k + 1, and 0
 * when either sequence is shorter than k. */
uint32_t sadref_fhat(const uint8_t* xi, int64_t Li, const uint8_t* xj, int64_t Lj, int A, int k);

/* Step 1 of the algorithm (local rank, samples, globalised rank; Sections 2
 * and 2.3.1).  key[i] = sum over samples s of F(i,s).  sample_ids receives the
 * p * k_s sample ids (chunk-major). */
/* Rank of rows against a sample list (all n when samples is NULL: the
 * centralised rank); rows NULL: all rows. */
int sadref_rank_against(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                        int32_t kmer_k, const int32_t* samples, int32_t n_samples,
                        const int32_t* rows, int32_t nrows, uint64_t* key);

int sadref_kmer_rank(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                     int32_t kmer_k, int32_t p, int32_t s_max,
                     uint64_t* key, int32_t* sample_ids, int32_t sample_cap,
                     int32_t* n_samples);

/* Regular-sampling splitters and buckets (Section 2.3.2). */
int sadref_partition(int32_t n, const uint64_t* key, int32_t p,
                     uint64_t* pivot_key, int32_t* pivot_id,
                     int32_t* bucket, int32_t* bucket_off, int32_t* members);

/* UPGMA on an n x n fixed-point similarity matrix F (row-major, uint32).
 * merges receives (n-1) pairs (a, b), a < b, of cluster ids; leaves are 0..n-1
 * and the cluster made at step t has id n + t. */
int sadref_upgma(int32_t n, const uint32_t* F, int32_t* merges);

/* Profile-profile affine-gap alignment (Section 2.3.3).  C1 is W1 x A and C2
 * is W2 x A residue counts (row-major, uint16); n1, n2 are the row counts.
 * ops receives the alignment (forward order, codes SADREF_OP_*), capacity
 * W1 + W2; *score receives its score. */
int sadref_profile_align(const uint16_t* C1, int32_t W1, int32_t n1,
                         const uint16_t* C2, int32_t W2, int32_t n2,
                         int32_t A, const int8_t* S, int32_t go, int32_t ge,
                         uint8_t* ops, int32_t* n_ops, int64_t* score);

/* Independent alignment of every bucket (Sections 2.3.2-2.3.3).
 * colmap[sum L]: column of each residue in its bucket's alignment;
 * width[p]; merge_score/merge_cells[n]: bucket b's merges at
 * [bucket_off[b], bucket_off[b] + n_b - 1); merge_list[2n] likewise (pairs);
 * *cells: total DP cells.  ops/ops_off are optional (NULL to skip): the op
 * strings of every merge, concatenated, with ops_off[n+1] offsets indexed
 * like merge_score (capacity given by ops_cap). */
int sadref_align_buckets(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                         int32_t p, const int32_t* bucket_off, const int32_t* members,
                         int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge,
                         int32_t* colmap, int32_t* width, int64_t* merge_score,
                         int32_t* merge_list, int64_t* merge_cells, int64_t* cells,
                         uint8_t* ops, int64_t ops_cap, int64_t* ops_off);

/* Consensus of an alignment given by its W x A column counts and row count n:
 * column c is kept iff 2 * residues(c) >= n; the kept residue is the most
 * frequent (smallest code on ties).  out needs W entries. */
int sadref_consensus(const uint16_t* counts, int32_t W, int32_t n, int32_t A,
                     uint8_t* out, int32_t* out_len);

/* Global ancestor and ancestor-constrained refinement + glue (Section 2.3.3).
 * ga[ga_cap] receives the global ancestor; colmap_g[sum L] the column of each
 * residue in the glued alignment, *width_g its width.  merge_score_g and
 * merge_cells_g (capacity 2p): the ancestor alignment's q-1 merges followed by
 * the q refinement alignments (q = non-empty buckets); merge_list_g[2p]. */
/* Refinement against a chosen template: tmpl 0 = GA as one row (what
 * sadref_refine does), 1 = the ancestors' alignment as a profile of q rows. */
int sadref_refine_template(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                           int32_t p, const int32_t* bucket_off, const int32_t* members,
                           const int32_t* colmap_b, const int32_t* width_b,
                           int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge, int32_t tmpl,
                           uint8_t* ga, int32_t ga_cap, int32_t* ga_len,
                           int32_t* colmap_g, int32_t* width_g,
                           int64_t* merge_score_g, int32_t* merge_list_g, int64_t* merge_cells_g,
                           int32_t* n_merges_g, int64_t* cells);
/* sadref_refine_template that also returns the refinement op strings:
 * bucket u's (u-th non-empty bucket) ops at rf_ops[rf_ops_off[u] ..
 * rf_ops_off[u+1]) (rf_ops_off has q + 1 entries; SADREF_E_CAPACITY when
 * rf_ops_cap is too small) and the template's width in *tmpl_width. */
int sadref_refine_template_ops(int32_t n, int32_t A, const uint8_t* codes,
                               const int64_t* offsets, int32_t p, const int32_t* bucket_off,
                               const int32_t* members, const int32_t* colmap_b,
                               const int32_t* width_b, int32_t kmer_k, const int8_t* S,
                               int32_t go, int32_t ge, int32_t tmpl, uint8_t* ga, int32_t ga_cap,
                               int32_t* ga_len, int32_t* colmap_g, int32_t* width_g,
                               int64_t* merge_score_g, int32_t* merge_list_g,
                               int64_t* merge_cells_g, int32_t* n_merges_g, int64_t* cells,
                               uint8_t* rf_ops, int64_t rf_ops_cap, int64_t* rf_ops_off,
                               int32_t* tmpl_width);
/* The glue of step 15 on its own: q refined bucket alignments given as op
 * strings (M, X, Y) against a template of TW columns -> the glued column of
 * every bucket column (to_g, buckets one after another) and the glued width.
 * SADREF_E_INVAL when an op string does not span its bucket and the template. */
int sadref_glue(int32_t q, int32_t TW, const uint8_t* ops, const int64_t* ops_off,
                const int32_t* width_u, int32_t* to_g, int32_t* width_g);
int sadref_refine(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                  int32_t p, const int32_t* bucket_off, const int32_t* members,
                  const int32_t* colmap_b, const int32_t* width_b,
                  int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge,
                  uint8_t* ga, int32_t ga_cap, int32_t* ga_len,
                  int32_t* colmap_g, int32_t* width_g,
                  int64_t* merge_score_g, int32_t* merge_list_g, int64_t* merge_cells_g,
                  int32_t* n_merges_g, int64_t* cells);

#ifdef __cplusplus
}
#endif
/* Tree-dependent refinement of the glued alignment: every edge of the
 * ancestors' guide tree (tree: the q - 1 merges, leaves = non-empty buckets
 * in bucket order) splits the sequences in two; the two parts are re-aligned
 * as profiles and the result kept iff its profile score is higher.  Per step
 * (node, old score, new score) is recorded while rec_cap allows. */
int sadref_refine_tree(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                       int32_t p, const int32_t* bucket_off, const int32_t* members,
                       const int32_t* colmap_in, int32_t width_in, const int32_t* tree,
                       int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge, int32_t passes,
                       int32_t* colmap_out, int32_t* width_out, int32_t* n_steps,
                       int32_t* rec_node, int64_t* rec_old, int64_t* rec_new, int32_t rec_cap,
                       int32_t* n_accepted);

#endif
