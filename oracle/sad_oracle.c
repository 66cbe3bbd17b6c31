/*
 * CPU oracle for the Sample-Align-D data-parallel core (Saeed & Khokhar,
 * arXiv 0901.2742).  TEST INFRASTRUCTURE ONLY -- see sad_oracle.h.
 *
 * Plain C.  Each function follows one step of the method in the order the
 * paper states it; where the paper leaves a choice open, the reading used is
 * stated next to the code.  All arithmetic is integer: scores in int64, k-mer
 * similarities as exact rationals c/d turned into the fixed point
 * floor(c * 2^31 / d).  Single-threaded by default; sadref_set_threads(t)
 * spreads loops over independent items (sequences, chunks, buckets, the
 * refinement alignments) over t threads, each item computed exactly as in
 * the single-threaded loop and written to its own outputs.
 */
#include "sad_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* loops over independent items                                        */
/* ------------------------------------------------------------------ */

static int g_threads = 1;

void sadref_set_threads(int32_t threads) { g_threads = threads < 1 ? 1 : threads; }

typedef void (*item_fn)(void* ctx, int64_t i);

typedef struct {
  item_fn fn;
  void* ctx;
  int64_t n;
  int64_t next; /* next unclaimed item, taken with an atomic add */
} item_loop_t;

/* set while a thread runs items: loops nested in an item run on its thread */
static __thread int t_in_items = 0;

static void* item_worker(void* arg) {
  item_loop_t* L = (item_loop_t*)arg;
  t_in_items = 1;
  for (;;) {
    int64_t i = __atomic_fetch_add(&L->next, 1, __ATOMIC_RELAXED);
    if (i >= L->n) break;
    L->fn(L->ctx, i);
  }
  return NULL;
}

/* fn(ctx, i) for i = 0..n-1, on up to g_threads threads (the caller's one
 * included); items must not write to shared state. */
static void for_items(int64_t n, item_fn fn, void* ctx) {
  int64_t t = g_threads < n ? g_threads : n;
  if (t <= 1 || t_in_items) {
    for (int64_t i = 0; i < n; ++i) fn(ctx, i);
    return;
  }
  item_loop_t L = {fn, ctx, n, 0};
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)(t - 1));
  int64_t started = 0;
  for (int64_t k = 0; k < t - 1; ++k)
    if (pthread_create(&th[k], NULL, item_worker, &L) == 0) started = k + 1;
    else break;
  item_worker(&L);
  t_in_items = 0;
  for (int64_t k = 0; k < started; ++k) pthread_join(th[k], NULL);
  free(th);
}

#define NEG_INF (INT64_MIN / 4)

/* ------------------------------------------------------------------ */
/* input validation                                                    */
/* ------------------------------------------------------------------ */

/* A^k, or -1 if it exceeds 2^16 (k-mer codes are kept below 2^16). */
static int64_t kmer_space(int A, int k) {
  int64_t v = 1;
  for (int u = 0; u < k; ++u) {
    v *= A;
    if (v > 65536) return -1;
  }
  return v;
}

static int validate_seqs(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                         int32_t k) {
  if (n < 0 || (A != 4 && A != 20) || k < 1 || kmer_space(A, k) < 0) return SADREF_E_INVAL;
  if (!offsets || offsets[0] != 0) return SADREF_E_INVAL;
  for (int32_t i = 0; i < n; ++i) {
    int64_t L = offsets[i + 1] - offsets[i];
    if (L < k) return SADREF_E_INVAL;
    for (int64_t t = offsets[i]; t < offsets[i + 1]; ++t)
      if (codes[t] >= A) return SADREF_E_INVAL;
  }
  return SADREF_OK;
}

/* ------------------------------------------------------------------ */
/* k-mer counts and the fractional common k-mer similarity (Section 2)  */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

int sadref_kmer_list(const uint8_t* x, int64_t L, int A, int k,
                     int32_t* taus, int32_t* counts, int64_t* n_unique) {
  *n_unique = 0;
  if (L < k) return SADREF_OK;
  int64_t m = L - k + 1;
  int32_t* all = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  for (int64_t t = 0; t < m; ++t) {
    int32_t tau = 0;
    for (int u = 0; u < k; ++u) tau = tau * A + x[t + u];
    all[t] = tau;
  }
  qsort(all, (size_t)m, sizeof(int32_t), cmp_i32);
  int64_t u = 0;
  for (int64_t t = 0; t < m; ++t) {
    if (u > 0 && taus[u - 1] == all[t]) {
      counts[u - 1] += 1;
    } else {
      taus[u] = all[t];
      counts[u] = 1;
      ++u;
    }
  }
  free(all);
  *n_unique = u;
  return SADREF_OK;
}

typedef struct {
  int64_t len;      /* sequence length */
  int64_t nu;       /* unique k-mers */
  int32_t* tau;
  int32_t* cnt;
} kmer_list_t;

static void build_list(kmer_list_t* kl, const uint8_t* x, int64_t L, int A, int k) {
  int64_t m = L >= k ? L - k + 1 : 1;
  kl->len = L;
  kl->tau = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  kl->cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  sadref_kmer_list(x, L, A, k, kl->tau, kl->cnt, &kl->nu);
}

static void free_list(kmer_list_t* kl) {
  free(kl->tau);
  free(kl->cnt);
}

/* sum_tau min(n_i(tau), n_j(tau)) by a merge of two sorted lists */
static int64_t common_lists(const kmer_list_t* a, const kmer_list_t* b) {
  int64_t c = 0, u = 0, v = 0;
  while (u < a->nu && v < b->nu) {
    if (a->tau[u] < b->tau[v]) {
      ++u;
    } else if (a->tau[u] > b->tau[v]) {
      ++v;
    } else {
      c += a->cnt[u] < b->cnt[v] ? a->cnt[u] : b->cnt[v];
      ++u;
      ++v;
    }
  }
  return c;
}

/* Reading of the garbled r_ij formula: the leading "tau ." is dropped, so
 * r_ij = c_ij / d_ij with d_ij = min(|x_i|, |x_j|) - k + 1, a similarity in
 * [0, 1].  Its fixed point is floor(c * 2^31 / d). */
static uint32_t fhat_lists(const kmer_list_t* a, const kmer_list_t* b, int k) {
  int64_t L = a->len < b->len ? a->len : b->len;
  if (L < k) return 0;
  int64_t d = L - k + 1;
  int64_t c = common_lists(a, b);
  return (uint32_t)(((uint64_t)c << 31) / (uint64_t)d);
}

int64_t sadref_common_kmers(const uint8_t* xi, int64_t Li, const uint8_t* xj, int64_t Lj,
                            int A, int k) {
  kmer_list_t a, b;
  build_list(&a, xi, Li, A, k);
  build_list(&b, xj, Lj, A, k);
  int64_t c = common_lists(&a, &b);
  free_list(&a);
  free_list(&b);
  return c;
}

uint32_t sadref_fhat(const uint8_t* xi, int64_t Li, const uint8_t* xj, int64_t Lj, int A, int k) {
  kmer_list_t a, b;
  build_list(&a, xi, Li, A, k);
  build_list(&b, xj, Lj, A, k);
  uint32_t f = fhat_lists(&a, &b, k);
  free_list(&a);
  free_list(&b);
  return f;
}

/* ------------------------------------------------------------------ */
/* composite keys (K_i, i) and chunks                                  */
/* ------------------------------------------------------------------ */

typedef struct {
  uint64_t key;
  int32_t id;
} ckey_t;

static int cmp_ckey(const void* a, const void* b) {
  const ckey_t* x = (const ckey_t*)a;
  const ckey_t* y = (const ckey_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int ckey_less(ckey_t a, ckey_t b) { return cmp_ckey(&a, &b) < 0; }

/* The paper places N/p sequences on each of p processors; here processor c
 * holds the contiguous chunk [floor(c N / p), floor((c+1) N / p)). */
static int32_t chunk_lo(int32_t n, int32_t p, int32_t c) {
  return (int32_t)(((int64_t)c * n) / p);
}

/* ------------------------------------------------------------------ */
/* Step 1: local rank, samples, globalised rank (Sections 2, 2.3.1)     */
/* ------------------------------------------------------------------ */

typedef struct {
  kmer_list_t* kl;
  const uint8_t* codes;
  const int64_t* offsets;
  int A, k;
} lists_ctx_t;

static void list_item(void* ctx, int64_t i) {
  lists_ctx_t* c = (lists_ctx_t*)ctx;
  build_list(&c->kl[i], c->codes + c->offsets[i], c->offsets[i + 1] - c->offsets[i], c->A, c->k);
}

static void build_lists(kmer_list_t* kl, int32_t n, const uint8_t* codes, const int64_t* offsets,
                        int A, int k) {
  lists_ctx_t c = {kl, codes, offsets, A, k};
  for_items(n, list_item, &c);
}

/* one chunk c: local ranks over the chunk, its order by (rank, id), its ks
 * samples (buf[lo..hi) is the chunk's own part of the buffer) */
typedef struct {
  const kmer_list_t* kl;
  ckey_t* buf;
  int32_t* sample_ids;
  int32_t n, p, ks, k;
} local_ctx_t;

static void local_chunk(void* ctx, int64_t c64) {
  local_ctx_t* L = (local_ctx_t*)ctx;
  const int32_t c = (int32_t)c64;
  int32_t lo = chunk_lo(L->n, L->p, c), hi = chunk_lo(L->n, L->p, c + 1), w = hi - lo;
  ckey_t* b = L->buf + lo;
  for (int32_t i = lo; i < hi; ++i) {
    uint64_t s = 0;
    for (int32_t j = lo; j < hi; ++j) s += fhat_lists(&L->kl[i], &L->kl[j], L->k);
    b[i - lo].key = s;
    b[i - lo].id = i;
  }
  qsort(b, (size_t)w, sizeof(ckey_t), cmp_ckey);
  for (int32_t t = 1; t <= L->ks; ++t)
    L->sample_ids[c * L->ks + (t - 1)] = b[((int64_t)t * w) / (L->ks + 1)].id;
}

/* one row t: key[t] = sum over the samples s of F(row, s); samples == NULL
 * means all sequences 0..ns-1, rows == NULL row t itself */
typedef struct {
  const kmer_list_t* kl;
  const int32_t* samples;
  int32_t ns;
  const int32_t* rows;
  uint64_t* key;
  int k;
} against_ctx_t;

static void against_row(void* ctx, int64_t t) {
  against_ctx_t* G = (against_ctx_t*)ctx;
  const int32_t i = G->rows ? G->rows[t] : (int32_t)t;
  uint64_t sum = 0;
  for (int32_t u = 0; u < G->ns; ++u)
    sum += fhat_lists(&G->kl[i], &G->kl[G->samples ? G->samples[u] : u], G->k);
  G->key[t] = sum;
}

int sadref_kmer_rank(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                     int32_t kmer_k, int32_t p, int32_t s_max,
                     uint64_t* key, int32_t* sample_ids, int32_t sample_cap,
                     int32_t* n_samples) {
  int st = validate_seqs(n, A, codes, offsets, kmer_k);
  if (st) return st;
  if (p < 1 || s_max < 1 || n < 2 * p) return SADREF_E_INVAL;

  kmer_list_t* kl = (kmer_list_t*)malloc(sizeof(kmer_list_t) * (size_t)(n > 0 ? n : 1));
  build_lists(kl, n, codes, offsets, A, kmer_k);

  /* samples per processor: k = p - 1 as in Section 2.3.2, capped so that the
   * whole sample stays within s_max and each chunk keeps a non-sampled item */
  int32_t w_min = n;
  for (int32_t c = 0; c < p; ++c) {
    int32_t w = chunk_lo(n, p, c + 1) - chunk_lo(n, p, c);
    if (w < w_min) w_min = w;
  }
  int32_t ks = p - 1;
  int32_t cap = s_max / p;
  if (cap < 1) cap = 1;
  if (ks > cap) ks = cap;
  if (ks > w_min - 1) ks = w_min - 1;
  int32_t S = p * ks;
  *n_samples = S;
  if (S > sample_cap) {
    for (int32_t i = 0; i < n; ++i) free_list(&kl[i]);
    free(kl);
    return SADREF_E_CAPACITY;
  }

  /* local k-mer rank: K_loc(i) = sum over j in i's chunk (self included) of
   * F(i, j); the chunk is sorted by (K_loc, i) and ks evenly spaced items are
   * sampled at positions floor(t w / (ks + 1)), t = 1..ks */
  ckey_t* buf = (ckey_t*)malloc(sizeof(ckey_t) * (size_t)(n > 0 ? n : 1));
  local_ctx_t lc = {kl, buf, sample_ids, n, p, ks, kmer_k};
  for_items(p, local_chunk, &lc);

  /* globalised rank: every sequence against all k*p samples (self included
   * when the sequence is itself a sample) */
  against_ctx_t gc = {kl, sample_ids, S, NULL, key, kmer_k};
  for_items(n, against_row, &gc);

  free(buf);
  for (int32_t i = 0; i < n; ++i) free_list(&kl[i]);
  free(kl);
  return SADREF_OK;
}

/* ------------------------------------------------------------------ */
/* Regular sampling, pivots and buckets (Section 2.3.2)                 */
/* ------------------------------------------------------------------ */

/* Rank of listed rows against a listed sample (Section 2.3.1): for each row i
 * in rows[0..nrows), key[t] = sum over the samples s of F(i, s), self
 * included when i is itself a sample.  samples == NULL takes all n sequences
 * (the centralised rank, every sequence against all N); rows == NULL takes
 * rows 0..n-1.  Sample and row ids outside [0, n) are rejected. */
int sadref_rank_against(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                        int32_t kmer_k, const int32_t* samples, int32_t n_samples,
                        const int32_t* rows, int32_t nrows, uint64_t* key) {
  int st = validate_seqs(n, A, codes, offsets, kmer_k);
  if (st) return st;
  if (samples == NULL) n_samples = n;
  if (rows == NULL) nrows = n;
  if (n_samples < 0 || nrows < 0) return SADREF_E_INVAL;
  for (int32_t t = 0; samples && t < n_samples; ++t)
    if (samples[t] < 0 || samples[t] >= n) return SADREF_E_INVAL;
  for (int32_t t = 0; rows && t < nrows; ++t)
    if (rows[t] < 0 || rows[t] >= n) return SADREF_E_INVAL;
  kmer_list_t* kl = (kmer_list_t*)malloc(sizeof(kmer_list_t) * (size_t)(n > 0 ? n : 1));
  build_lists(kl, n, codes, offsets, A, kmer_k);
  against_ctx_t gc = {kl, samples, n_samples, rows, key, kmer_k};
  for_items(nrows, against_row, &gc);
  for (int32_t i = 0; i < n; ++i) free_list(&kl[i]);
  free(kl);
  return SADREF_OK;
}

int sadref_partition(int32_t n, const uint64_t* key, int32_t p,
                     uint64_t* pivot_key, int32_t* pivot_id,
                     int32_t* bucket, int32_t* bucket_off, int32_t* members) {
  if (p < 1 || n < 2 * p) return SADREF_E_INVAL;
  int64_t ny = (int64_t)p * (p - 1);
  ckey_t* Y = (ckey_t*)malloc(sizeof(ckey_t) * (size_t)(ny > 0 ? ny : 1));
  ckey_t* buf = (ckey_t*)malloc(sizeof(ckey_t) * (size_t)n);

  /* each chunk sorted by (K_i, i); p - 1 evenly spaced keys at positions
   * floor(t w / p), t = 1..p-1 (repeats allowed when w < p) */
  for (int32_t c = 0; c < p; ++c) {
    int32_t lo = chunk_lo(n, p, c), hi = chunk_lo(n, p, c + 1), w = hi - lo;
    for (int32_t i = lo; i < hi; ++i) {
      buf[i - lo].key = key[i];
      buf[i - lo].id = i;
    }
    qsort(buf, (size_t)w, sizeof(ckey_t), cmp_ckey);
    for (int32_t t = 1; t <= p - 1; ++t)
      Y[(int64_t)c * (p - 1) + (t - 1)] = buf[((int64_t)t * w) / p];
  }

  /* sort the p(p-1) gathered keys; pivots Y_{p/2}, Y_{p+p/2}, ...,
   * Y_{(p-2)p+p/2} (1-based) -- p - 1 of them */
  qsort(Y, (size_t)ny, sizeof(ckey_t), cmp_ckey);
  for (int32_t t = 1; t <= p - 1; ++t) {
    ckey_t y = Y[p / 2 + (int64_t)(t - 1) * p - 1];
    pivot_key[t - 1] = y.key;
    pivot_id[t - 1] = y.id;
  }

  /* bucket(i) = number of pivots strictly below (K_i, i): a key equal to a
   * pivot stays in the lower bucket */
  for (int32_t b = 0; b <= p; ++b) bucket_off[b] = 0;
  for (int32_t i = 0; i < n; ++i) {
    ckey_t me = {key[i], i};
    int32_t b = 0;
    for (int32_t t = 0; t < p - 1; ++t) {
      ckey_t y = {pivot_key[t], pivot_id[t]};
      if (ckey_less(y, me)) ++b;
    }
    bucket[i] = b;
    bucket_off[b + 1] += 1;
  }
  for (int32_t b = 0; b < p; ++b) bucket_off[b + 1] += bucket_off[b];
  int32_t* fill = (int32_t*)calloc((size_t)p, sizeof(int32_t));
  for (int32_t i = 0; i < n; ++i) {
    int32_t b = bucket[i];
    members[bucket_off[b] + fill[b]++] = i;
  }
  free(fill);
  free(buf);
  free(Y);
  return SADREF_OK;
}

/* ------------------------------------------------------------------ */
/* UPGMA guide tree on the fixed-point similarities                    */
/* ------------------------------------------------------------------ */

/* Pick the active pair with the largest average similarity
 * S_AB / (|A| |B|); compared exactly by cross-multiplication in 128 bits;
 * ties go to the lexicographically smallest (min id, max id). */
typedef struct {
  const uint64_t* S;
  const int32_t* id;
  const int64_t* sz;
  const char* active;
  int32_t n, parts;
  int32_t* part_a;
  int32_t* part_b;
} upgma_scan_t;

/* pair (a, b) comes before pair (c, d) in the merge order */
static int pair_before(const upgma_scan_t* U, int32_t a, int32_t b, int32_t c, int32_t d) {
  const int32_t n = U->n;
  unsigned __int128 lhs = (unsigned __int128)U->S[(size_t)a * n + b] *
                          (unsigned __int128)(U->sz[c] * U->sz[d]);
  unsigned __int128 rhs = (unsigned __int128)U->S[(size_t)c * n + d] *
                          (unsigned __int128)(U->sz[a] * U->sz[b]);
  if (lhs != rhs) return lhs > rhs;
  int32_t lo1 = U->id[a] < U->id[b] ? U->id[a] : U->id[b];
  int32_t hi1 = U->id[a] < U->id[b] ? U->id[b] : U->id[a];
  int32_t lo2 = U->id[c] < U->id[d] ? U->id[c] : U->id[d];
  int32_t hi2 = U->id[c] < U->id[d] ? U->id[d] : U->id[c];
  return lo1 < lo2 || (lo1 == lo2 && hi1 < hi2);
}

/* the first active pair (a, b), a < b, among the rows a = part, part +
 * parts, ... (the order is strict, so splitting the rows cannot change the
 * overall first) */
static void upgma_scan_part(void* ctx, int64_t part) {
  upgma_scan_t* U = (upgma_scan_t*)ctx;
  int32_t ba = -1, bb = -1;
  for (int32_t a = (int32_t)part; a < U->n; a += U->parts) {
    if (!U->active[a]) continue;
    for (int32_t b = a + 1; b < U->n; ++b) {
      if (!U->active[b]) continue;
      if (ba < 0 || pair_before(U, a, b, ba, bb)) {
        ba = a;
        bb = b;
      }
    }
  }
  U->part_a[part] = ba;
  U->part_b[part] = bb;
}

int sadref_upgma(int32_t n, const uint32_t* F, int32_t* merges) {
  if (n <= 1) return SADREF_OK;
  uint64_t* S = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n * (size_t)n);
  int32_t* id = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* sz = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  char* active = (char*)malloc((size_t)n);
  for (int32_t a = 0; a < n; ++a) {
    for (int32_t b = 0; b < n; ++b) S[(size_t)a * n + b] = F[(size_t)a * n + b];
    id[a] = a;
    sz[a] = 1;
    active[a] = 1;
  }
  const int32_t max_parts = g_threads > 1 ? 4 * g_threads : 1;
  int32_t* part_a = (int32_t*)malloc(sizeof(int32_t) * (size_t)max_parts);
  int32_t* part_b = (int32_t*)malloc(sizeof(int32_t) * (size_t)max_parts);
  upgma_scan_t U = {S, id, sz, active, n, 1, part_a, part_b};
  for (int32_t step = 0; step < n - 1; ++step) {
    /* rows split over threads while enough clusters remain */
    U.parts = n - step >= 256 ? max_parts : 1;
    for_items(U.parts, upgma_scan_part, &U);
    int32_t ba = -1, bb = -1;
    for (int32_t t = 0; t < U.parts; ++t) {
      if (part_a[t] < 0) continue;
      if (ba < 0 || pair_before(&U, part_a[t], part_b[t], ba, bb)) {
        ba = part_a[t];
        bb = part_b[t];
      }
    }
    int32_t ia = id[ba], ib = id[bb];
    merges[2 * step] = ia < ib ? ia : ib;
    merges[2 * step + 1] = ia < ib ? ib : ia;
    /* the union takes slot ba: S(new, C) = S(A, C) + S(B, C) */
    for (int32_t c = 0; c < n; ++c) {
      if (!active[c] || c == ba || c == bb) continue;
      uint64_t v = S[(size_t)ba * n + c] + S[(size_t)bb * n + c];
      S[(size_t)ba * n + c] = v;
      S[(size_t)c * n + ba] = v;
    }
    sz[ba] += sz[bb];
    id[ba] = n + step;
    active[bb] = 0;
  }
  free(S);
  free(id);
  free(sz);
  free(active);
  free(part_a);
  free(part_b);
  return SADREF_OK;
}

/* ------------------------------------------------------------------ */
/* Profile-profile affine-gap alignment (Section 2.3.3)                */
/* ------------------------------------------------------------------ */

/* Tie bits recorded per cell: which ops attain H, and which predecessor
 * attains X and Y. */
#define B_HM 1
#define B_HX 2
#define B_HY 4
#define B_XO 8
#define B_XE 16
#define B_YO 32
#define B_YE 64

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* Column score s(i, j) = sum_a sum_b C1[i][a] S[a][b] C2[j][b]: every pair of
 * rows (one from each profile) with residues in both columns contributes its
 * substitution score.  U = C1 * S is formed first (a plain matrix product). */
static int64_t* column_scores(const uint16_t* C1, int32_t W1, const uint16_t* C2, int32_t W2,
                              int32_t A, const int8_t* S) {
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * (size_t)(W1 > 0 ? W1 : 1) * (size_t)A);
  for (int32_t i = 0; i < W1; ++i)
    for (int32_t b = 0; b < A; ++b) {
      int64_t u = 0;
      for (int32_t a = 0; a < A; ++a) u += (int64_t)C1[(size_t)i * A + a] * S[a * A + b];
      U[(size_t)i * A + b] = u;
    }
  int64_t* sc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(W1 > 0 ? W1 : 1) *
                                 (size_t)(W2 > 0 ? W2 : 1));
  for (int32_t i = 0; i < W1; ++i)
    for (int32_t j = 0; j < W2; ++j) {
      int64_t s = 0;
      for (int32_t b = 0; b < A; ++b) s += U[(size_t)i * A + b] * C2[(size_t)j * A + b];
      sc[(size_t)i * W2 + j] = s;
    }
  free(U);
  return sc;
}

/* Reading of the profile gap model (the paper only names the method of its
 * reference [12]): affine run cost g(l) = o + (l - 1) e with o = n1 n2 go and
 * e = n1 n2 ge, terminal gaps charged like internal ones.  Recurrences
 * (Gotoh):
 *   M(i,j) = H(i-1,j-1) + s(i,j)
 *   X(i,j) = max(X(i-1,j) - e, H(i-1,j) - o)      column i of P1 vs a gap
 *   Y(i,j) = max(Y(i,j-1) - e, H(i,j-1) - o)      column j of P2 vs a gap
 *   H(i,j) = max(M, X, Y)
 * Among optimal alignments the one returned has the lexicographically smallest
 * op string read backwards from (W1, W2), with M < X < Y. */
int sadref_profile_align(const uint16_t* C1, int32_t W1, int32_t n1,
                         const uint16_t* C2, int32_t W2, int32_t n2,
                         int32_t A, const int8_t* S, int32_t go, int32_t ge,
                         uint8_t* ops, int32_t* n_ops, int64_t* score) {
  if (W1 < 0 || W2 < 0 || n1 < 0 || n2 < 0 || go < ge || ge < 0) return SADREF_E_INVAL;
  int64_t G = (int64_t)n1 * n2;
  int64_t o = G * go, e = G * ge;
  int64_t smax = 1;
  for (int32_t a = 0; a < A * A; ++a) {
    int64_t v = S[a] < 0 ? -(int64_t)S[a] : S[a];
    if (v > smax) smax = v;
  }
  int64_t unit = smax > go ? smax : go;
  /* static bound of every DP value: (W1 + W2 + 2) * G * max(|S|, go) */
  if ((double)(W1 + W2 + 2) * (double)G * (double)unit >= 2.0e18) return SADREF_E_OVERFLOW;

  int64_t* sc = column_scores(C1, W1, C2, W2, A, S);
  size_t R = (size_t)W1 + 1, C = (size_t)W2 + 1;
  int64_t* H = (int64_t*)malloc(sizeof(int64_t) * R * C);
  int64_t* X = (int64_t*)malloc(sizeof(int64_t) * R * C);
  int64_t* Y = (int64_t*)malloc(sizeof(int64_t) * R * C);
  uint8_t* bits = (uint8_t*)calloc(R * C, 1);
#define AT(M_, i_, j_) M_[(size_t)(i_) * C + (size_t)(j_)]

  AT(H, 0, 0) = 0;
  AT(X, 0, 0) = NEG_INF;
  AT(Y, 0, 0) = NEG_INF;
  for (int32_t i = 1; i <= W1; ++i) {
    AT(H, i, 0) = -(o + (int64_t)(i - 1) * e);
    AT(X, i, 0) = AT(H, i, 0);
    AT(Y, i, 0) = NEG_INF;
  }
  for (int32_t j = 1; j <= W2; ++j) {
    AT(H, 0, j) = -(o + (int64_t)(j - 1) * e);
    AT(Y, 0, j) = AT(H, 0, j);
    AT(X, 0, j) = NEG_INF;
  }
  for (int32_t i = 1; i <= W1; ++i) {
    for (int32_t j = 1; j <= W2; ++j) {
      int64_t m = AT(H, i - 1, j - 1) + sc[(size_t)(i - 1) * W2 + (j - 1)];
      int64_t xo = AT(H, i - 1, j) - o;
      int64_t xe = AT(X, i - 1, j) - e;
      int64_t x = max2(xo, xe);
      int64_t yo = AT(H, i, j - 1) - o;
      int64_t ye = AT(Y, i, j - 1) - e;
      int64_t y = max2(yo, ye);
      int64_t h = max2(m, max2(x, y));
      uint8_t bt = 0;
      if (m == h) bt |= B_HM;
      if (x == h) bt |= B_HX;
      if (y == h) bt |= B_HY;
      if (xo == x) bt |= B_XO;
      if (xe == x) bt |= B_XE;
      if (yo == y) bt |= B_YO;
      if (ye == y) bt |= B_YE;
      AT(H, i, j) = h;
      AT(X, i, j) = x;
      AT(Y, i, j) = y;
      AT(bits, i, j) = bt;
    }
  }
  *score = AT(H, W1, W2);

  /* Traceback, greedy from the end: at every step the next op back is the
   * smallest one that still admits an optimal completion.  In state H the
   * candidates are the ops attaining H; in state X the run either extends
   * (xExt) or was opened from H(i-1, j), whose attaining ops then follow
   * (an X never directly precedes an opened X run unless o == e, in which
   * case the extension covers it); likewise for Y. */
  int32_t i = W1, j = W2, k = 0;
  int state = 0; /* 0 = H, 1 = X, 2 = Y */
  uint8_t* rev = (uint8_t*)malloc((size_t)W1 + (size_t)W2 + 1);
  while (i > 0 && j > 0) {
    uint8_t bt = AT(bits, i, j);
    if (state == 0) {
      if (bt & B_HM) {
        rev[k++] = SADREF_OP_M;
        --i;
        --j;
      } else if (bt & B_HX) {
        state = 1;
      } else {
        state = 2;
      }
    } else if (state == 1) {
      rev[k++] = SADREF_OP_X;
      --i;
      int prev_m = (i > 0 && j > 0) ? (AT(bits, i, j) & B_HM) != 0 : 0;
      if ((bt & B_XO) && prev_m) state = 0;
      else if (bt & B_XE) state = 1;
      else state = 0;
    } else {
      rev[k++] = SADREF_OP_Y;
      --j;
      int prev_mx = (i > 0 && j > 0) ? (AT(bits, i, j) & (B_HM | B_HX)) != 0 : 0;
      if ((bt & B_YO) && prev_mx) state = 0;
      else if (bt & B_YE) state = 2;
      else state = 0;
    }
  }
  /* on the border the rest of the path is forced */
  while (i > 0) {
    rev[k++] = SADREF_OP_X;
    --i;
  }
  while (j > 0) {
    rev[k++] = SADREF_OP_Y;
    --j;
  }
  for (int32_t t = 0; t < k; ++t) ops[t] = rev[k - 1 - t];
  *n_ops = k;
#undef AT
  free(rev);
  free(sc);
  free(H);
  free(X);
  free(Y);
  free(bits);
  return SADREF_OK;
}

/* ------------------------------------------------------------------ */
/* Progressive alignment along the guide tree                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t W;        /* columns */
  int32_t n;        /* rows */
  uint16_t* cnt;    /* W x A counts */
  int32_t* up;      /* column in the parent, W entries (NULL for the root) */
  int32_t parent;
} node_t;

static int check_count(int64_t v) { return v <= 65535; }

/* Aligns n leaf sequences progressively along the UPGMA tree of their
 * k-mer similarities.  Outputs: root node index, per-merge scores, cells, op
 * strings.  nodes[] must hold 2n - 1 entries. */
static int progressive(int32_t n, const uint8_t* const* seq, const int64_t* len, int32_t A,
                       int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge,
                       node_t* nodes, int32_t* merges, int64_t* mscore, int64_t* mcells,
                       uint8_t* ops_out, int64_t ops_cap, int64_t* ops_off, int64_t* ops_pos) {
  /* leaves: one-row profiles */
  for (int32_t a = 0; a < n; ++a) {
    node_t* nd = &nodes[a];
    nd->W = (int32_t)len[a];
    nd->n = 1;
    nd->cnt = (uint16_t*)calloc((size_t)(nd->W > 0 ? nd->W : 1) * (size_t)A, sizeof(uint16_t));
    for (int32_t c = 0; c < nd->W; ++c) nd->cnt[(size_t)c * A + seq[a][c]] = 1;
    nd->up = NULL;
    nd->parent = -1;
  }
  if (n <= 1) return SADREF_OK;

  /* pairwise fixed-point similarities, then UPGMA */
  kmer_list_t* kl = (kmer_list_t*)malloc(sizeof(kmer_list_t) * (size_t)n);
  for (int32_t a = 0; a < n; ++a) build_list(&kl[a], seq[a], len[a], A, kmer_k);
  uint32_t* F = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n * (size_t)n);
  for (int32_t a = 0; a < n; ++a)
    for (int32_t b = 0; b < n; ++b) F[(size_t)a * n + b] = fhat_lists(&kl[a], &kl[b], kmer_k);
  for (int32_t a = 0; a < n; ++a) free_list(&kl[a]);
  free(kl);
  sadref_upgma(n, F, merges);
  free(F);

  int st = SADREF_OK;
  for (int32_t t = 0; t < n - 1 && st == SADREF_OK; ++t) {
    /* P1 = the child with the smaller id */
    node_t* p1 = &nodes[merges[2 * t]];
    node_t* p2 = &nodes[merges[2 * t + 1]];
    node_t* nd = &nodes[n + t];
    int32_t cap = p1->W + p2->W;
    uint8_t* ops = (uint8_t*)malloc((size_t)(cap > 0 ? cap : 1));
    int32_t nops = 0;
    int64_t sc = 0;
    st = sadref_profile_align(p1->cnt, p1->W, p1->n, p2->cnt, p2->W, p2->n, A, S, go, ge,
                              ops, &nops, &sc);
    if (st) {
      free(ops);
      break;
    }
    mscore[t] = sc;
    mcells[t] = (int64_t)p1->W * p2->W;
    if (ops_out) {
      ops_off[t] = *ops_pos;
      if (*ops_pos + nops > ops_cap) {
        st = SADREF_E_CAPACITY;
      } else {
        memcpy(ops_out + *ops_pos, ops, (size_t)nops);
        *ops_pos += nops;
      }
    }
    /* merged alignment: P1's rows then P2's rows; column counts add */
    nd->W = nops;
    nd->n = p1->n + p2->n;
    nd->cnt = (uint16_t*)calloc((size_t)(nops > 0 ? nops : 1) * (size_t)A, sizeof(uint16_t));
    nd->up = NULL;
    nd->parent = -1;
    p1->up = (int32_t*)malloc(sizeof(int32_t) * (size_t)(p1->W > 0 ? p1->W : 1));
    p2->up = (int32_t*)malloc(sizeof(int32_t) * (size_t)(p2->W > 0 ? p2->W : 1));
    p1->parent = n + t;
    p2->parent = n + t;
    int32_t i = 0, j = 0;
    for (int32_t c = 0; c < nops; ++c) {
      if (ops[c] != SADREF_OP_Y) {
        for (int32_t a = 0; a < A; ++a) {
          int64_t v = (int64_t)nd->cnt[(size_t)c * A + a] + p1->cnt[(size_t)i * A + a];
          if (!check_count(v)) st = SADREF_E_OVERFLOW;
          nd->cnt[(size_t)c * A + a] = (uint16_t)v;
        }
        p1->up[i++] = c;
      }
      if (ops[c] != SADREF_OP_X) {
        for (int32_t a = 0; a < A; ++a) {
          int64_t v = (int64_t)nd->cnt[(size_t)c * A + a] + p2->cnt[(size_t)j * A + a];
          if (!check_count(v)) st = SADREF_E_OVERFLOW;
          nd->cnt[(size_t)c * A + a] = (uint16_t)v;
        }
        p2->up[j++] = c;
      }
    }
    free(ops);
  }
  return st;
}

static void free_nodes(node_t* nodes, int32_t m) {
  for (int32_t a = 0; a < m; ++a) {
    free(nodes[a].cnt);
    free(nodes[a].up);
  }
}

/* column of residue r of leaf a in the root's alignment */
static int32_t root_column(const node_t* nodes, int32_t a, int32_t r) {
  int32_t c = r;
  while (nodes[a].parent >= 0) {
    c = nodes[a].up[c];
    a = nodes[a].parent;
  }
  return c;
}

/* one bucket's progressive alignment and its column map; ops (when given)
 * are appended at *ops_pos, so buckets with ops run one after another */
typedef struct {
  int32_t A, kmer_k, go, ge;
  const uint8_t* codes;
  const int64_t* offsets;
  const int32_t *bucket_off, *members;
  const int8_t* S;
  int32_t *colmap, *width, *merge_list;
  int64_t *merge_score, *merge_cells;
  uint8_t* ops;
  int64_t ops_cap;
  int64_t* ops_off;
  int64_t* ops_pos;
  int* status; /* per bucket */
} bucket_ctx_t;

static void align_one_bucket(void* ctx, int64_t b64) {
  bucket_ctx_t* B = (bucket_ctx_t*)ctx;
  const int32_t b = (int32_t)b64;
  int32_t lo = B->bucket_off[b], nb = B->bucket_off[b + 1] - lo;
  B->status[b] = SADREF_OK;
  if (nb <= 0) {
    B->width[b] = 0;
    if (nb < 0) B->status[b] = SADREF_E_INVAL;
    return;
  }
  const uint8_t** seq = (const uint8_t**)malloc(sizeof(uint8_t*) * (size_t)nb);
  int64_t* len = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
  for (int32_t a = 0; a < nb; ++a) {
    int32_t id = B->members[lo + a];
    seq[a] = B->codes + B->offsets[id];
    len[a] = B->offsets[id + 1] - B->offsets[id];
  }
  node_t* nodes = (node_t*)calloc((size_t)(2 * nb - 1), sizeof(node_t));
  int st = progressive(nb, seq, len, B->A, B->kmer_k, B->S, B->go, B->ge, nodes,
                       B->merge_list + 2 * (int64_t)lo, B->merge_score + lo,
                       B->merge_cells + lo, B->ops, B->ops_cap,
                       B->ops ? B->ops_off + lo : NULL, B->ops_pos);
  /* the bucket's last slot holds no merge: its offset closes the previous
   * op string, so merge t always ends at ops_off[t + 1] */
  if (B->ops && st == SADREF_OK) B->ops_off[lo + nb - 1] = *B->ops_pos;
  if (st == SADREF_OK) {
    int32_t root = 2 * nb - 2;
    B->width[b] = nodes[root].W;
    for (int32_t a = 0; a < nb; ++a) {
      int32_t id = B->members[lo + a];
      for (int64_t r = 0; r < len[a]; ++r)
        B->colmap[B->offsets[id] + r] = root_column(nodes, a, (int32_t)r);
    }
  }
  B->status[b] = st;
  free_nodes(nodes, 2 * nb - 1);
  free(nodes);
  free(seq);
  free(len);
}

int sadref_align_buckets(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                         int32_t p, const int32_t* bucket_off, const int32_t* members,
                         int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge,
                         int32_t* colmap, int32_t* width, int64_t* merge_score,
                         int32_t* merge_list, int64_t* merge_cells, int64_t* cells,
                         uint8_t* ops, int64_t ops_cap, int64_t* ops_off) {
  int st = validate_seqs(n, A, codes, offsets, kmer_k);
  if (st) return st;
  if (p < 1 || go < ge || ge < 0) return SADREF_E_INVAL;
  if (bucket_off[0] != 0 || bucket_off[p] != n) return SADREF_E_INVAL;
  for (int32_t b = 0; b < p; ++b)
    if (bucket_off[b + 1] < bucket_off[b]) return SADREF_E_INVAL;
  *cells = 0;
  int64_t ops_pos = 0;
  int* status = (int*)calloc((size_t)p, sizeof(int));
  bucket_ctx_t bc = {A, kmer_k, go, ge, codes, offsets, bucket_off, members, S, colmap, width,
                     merge_list, merge_score, merge_cells, ops, ops_cap, ops_off, &ops_pos,
                     status};
  if (ops) {
    /* op strings are appended bucket by bucket: in order, up to the first
     * failure */
    for (int32_t b = 0; b < p && st == SADREF_OK; ++b) {
      align_one_bucket(&bc, b);
      st = status[b];
    }
  } else {
    for_items(p, align_one_bucket, &bc);
    for (int32_t b = 0; b < p && st == SADREF_OK; ++b) st = status[b];
  }
  for (int32_t b = 0; b < p && st == SADREF_OK; ++b)
    for (int32_t t = bucket_off[b]; t < bucket_off[b + 1] - 1; ++t) *cells += merge_cells[t];
  if (ops && st == SADREF_OK) ops_off[n] = ops_pos;
  free(status);
  return st;
}

/* ------------------------------------------------------------------ */
/* Ancestors, global ancestor, refinement and glue (Section 2.3.3)      */
/* ------------------------------------------------------------------ */

/* Reading of "local ancestor": the majority consensus of the alignment. */
int sadref_consensus(const uint16_t* counts, int32_t W, int32_t n, int32_t A,
                     uint8_t* out, int32_t* out_len) {
  int32_t m = 0;
  for (int32_t c = 0; c < W; ++c) {
    int64_t tot = 0;
    int32_t best = 0;
    for (int32_t a = 0; a < A; ++a) {
      tot += counts[(size_t)c * A + a];
      if (counts[(size_t)c * A + a] > counts[(size_t)c * A + best]) best = a;
    }
    if (2 * tot >= n) out[m++] = (uint8_t)best;
  }
  *out_len = m;
  return SADREF_OK;
}

/* Glue of the refined bucket alignments (Section 2.3.3, step 15; the
 * paper only says they are joined).  Bucket u (u = 0..q-1, non-empty buckets
 * in bucket order) was aligned against the template of TW columns by the op
 * string ops[ops_off[u] .. ops_off[u+1]): M pairs its next column with the
 * next template column, X places its next column against a gap, Y places a
 * gap against the next template column.  Layout: before template column j
 * (j = 0..TW; slot TW follows the last column) an insert slot holds the
 * X-columns of every bucket that fall there, bucket 0's first, each bucket's
 * in its own order, each in a column of its own; then comes the shared column
 * j, holding each bucket's M-column of j or a gap.  Columns that hold no
 * residue (shared columns every bucket skips) are dropped.  Output: to_g, for
 * bucket u at to_g[col_off[u] ..] (col_off = prefix sums of width_u), the glued
 * column of each of its columns; *width_g. */
int sadref_glue(int32_t q, int32_t TW, const uint8_t* ops, const int64_t* ops_off,
                const int32_t* width_u, int32_t* to_g, int32_t* width_g) {
  if (q < 0 || TW < 0) return SADREF_E_INVAL;
  int64_t slots = (int64_t)TW + 1;
  int64_t* ins = (int64_t*)calloc((size_t)(q * slots > 0 ? q * slots : 1), sizeof(int64_t));
  char* shared_used = (char*)calloc((size_t)(TW > 0 ? TW : 1), 1);
  int st = SADREF_OK;
  for (int32_t u = 0; u < q && st == SADREF_OK; ++u) {
    int32_t i = 0, j = 0;
    for (int64_t t = ops_off[u]; t < ops_off[u + 1]; ++t) {
      uint8_t op = ops[t];
      if (op == SADREF_OP_X) {
        ins[(int64_t)u * slots + j] += 1;
        ++i;
      } else if (op == SADREF_OP_M || op == SADREF_OP_Y) {
        if (j >= TW) { st = SADREF_E_INVAL; break; }
        if (op == SADREF_OP_M) { shared_used[j] = 1; ++i; }
        ++j;
      } else {
        st = SADREF_E_INVAL;
        break;
      }
    }
    if (st == SADREF_OK && (i != width_u[u] || j != TW)) st = SADREF_E_INVAL;
  }
  /* start index of each (slot, bucket) block and each kept shared column */
  int64_t* blk = (int64_t*)malloc(sizeof(int64_t) * (size_t)(q * slots > 0 ? q * slots : 1));
  int64_t* shared_at = (int64_t*)malloc(sizeof(int64_t) * (size_t)(TW > 0 ? TW : 1));
  int64_t pos = 0;
  if (st == SADREF_OK) {
    for (int64_t j = 0; j < slots; ++j) {
      for (int32_t u = 0; u < q; ++u) {
        blk[(int64_t)u * slots + j] = pos;
        pos += ins[(int64_t)u * slots + j];
      }
      if (j < TW) {
        shared_at[j] = shared_used[j] ? pos : -1;
        if (shared_used[j]) ++pos;
      }
    }
    *width_g = (int32_t)pos;
    int64_t base = 0;
    for (int32_t u = 0; u < q; ++u) {
      int32_t i = 0, j = 0;
      int64_t k_in = 0;
      for (int64_t t = ops_off[u]; t < ops_off[u + 1]; ++t) {
        uint8_t op = ops[t];
        if (op == SADREF_OP_X) {
          to_g[base + i++] = (int32_t)(blk[(int64_t)u * slots + j] + k_in);
          ++k_in;
        } else {
          if (op == SADREF_OP_M) to_g[base + i++] = (int32_t)shared_at[j];
          ++j;
          k_in = 0;
        }
      }
      base += width_u[u];
    }
  }
  free(ins);
  free(shared_used);
  free(blk);
  free(shared_at);
  return st;
}

/* Refinement with a choice of template (Section 2.3.3, steps 12-15):
 * tmpl 0 aligns every bucket with GA as a one-row profile (the consensus of
 * the ancestors' alignment); tmpl 1 aligns every bucket with the ancestors'
 * alignment itself, a profile of q rows (the richer template the paper leaves
 * to future work).  With one non-empty bucket both are the bucket's own
 * ancestor as one row. */
/* refinement alignment u: bucket u's profile against the template */
typedef struct {
  const int32_t *nonempty, *width_b, *bucket_off;
  uint16_t* const* prof;
  const uint16_t* tprof;
  int32_t TW, tn, A;
  const int8_t* S;
  int32_t go, ge;
  uint8_t** bops;
  int32_t* bnops;
  int64_t *score, *cells;
  int32_t* list;
  int* status;
} refine_ctx_t;

static void refine_one_bucket(void* ctx, int64_t u64) {
  refine_ctx_t* R = (refine_ctx_t*)ctx;
  const int32_t u = (int32_t)u64;
  int32_t b = R->nonempty[u];
  int32_t W = R->width_b[b], nb = R->bucket_off[b + 1] - R->bucket_off[b];
  R->bops[u] = (uint8_t*)malloc((size_t)(W + R->TW > 0 ? W + R->TW : 1));
  int64_t sc = 0;
  R->status[u] = sadref_profile_align(R->prof[b], W, nb, R->tprof, R->TW, R->tn, R->A, R->S,
                                      R->go, R->ge, R->bops[u], &R->bnops[u], &sc);
  R->score[u] = sc;
  R->cells[u] = (int64_t)W * R->TW;
  R->list[2 * u] = b;
  R->list[2 * u + 1] = -1;
}

int sadref_refine_template_ops(int32_t n, int32_t A, const uint8_t* codes,
                               const int64_t* offsets, int32_t p, const int32_t* bucket_off,
                               const int32_t* members, const int32_t* colmap_b,
                               const int32_t* width_b, int32_t kmer_k, const int8_t* S,
                               int32_t go, int32_t ge, int32_t tmpl, uint8_t* ga, int32_t ga_cap,
                               int32_t* ga_len, int32_t* colmap_g, int32_t* width_g,
                               int64_t* merge_score_g, int32_t* merge_list_g,
                               int64_t* merge_cells_g, int32_t* n_merges_g, int64_t* cells,
                               uint8_t* rf_ops, int64_t rf_ops_cap, int64_t* rf_ops_off,
                               int32_t* tmpl_width) {
  int st = validate_seqs(n, A, codes, offsets, kmer_k);
  if (st) return st;
  if (p < 1 || go < ge || ge < 0 || tmpl < 0 || tmpl > 1) return SADREF_E_INVAL;
  if (bucket_off[0] != 0 || bucket_off[p] != n) return SADREF_E_INVAL;

  /* bucket alignments as column-count profiles */
  int32_t q = 0;
  int32_t* nonempty = (int32_t*)malloc(sizeof(int32_t) * (size_t)p);
  uint16_t** prof = (uint16_t**)calloc((size_t)p, sizeof(uint16_t*));
  for (int32_t b = 0; b < p; ++b) {
    int32_t lo = bucket_off[b], nb = bucket_off[b + 1] - lo;
    if (nb <= 0) continue;
    nonempty[q++] = b;
    int32_t W = width_b[b];
    prof[b] = (uint16_t*)calloc((size_t)(W > 0 ? W : 1) * (size_t)A, sizeof(uint16_t));
    for (int32_t a = 0; a < nb; ++a) {
      int32_t id = members[lo + a];
      for (int64_t r = offsets[id]; r < offsets[id + 1]; ++r) {
        int32_t c = colmap_b[r];
        if (c < 0 || c >= W) {
          st = SADREF_E_INVAL;
          continue;
        }
        prof[b][(size_t)c * A + codes[r]] += 1;
      }
    }
  }

  /* local ancestors */
  uint8_t** anc = (uint8_t**)calloc((size_t)(q > 0 ? q : 1), sizeof(uint8_t*));
  int64_t* anc_len = (int64_t*)calloc((size_t)(q > 0 ? q : 1), sizeof(int64_t));
  for (int32_t u = 0; u < q && st == SADREF_OK; ++u) {
    int32_t b = nonempty[u];
    int32_t W = width_b[b], len = 0;
    anc[u] = (uint8_t*)malloc((size_t)(W > 0 ? W : 1));
    sadref_consensus(prof[b], W, bucket_off[b + 1] - bucket_off[b], A, anc[u], &len);
    anc_len[u] = len;
  }

  /* global ancestor: the consensus of the ancestors aligned along their own
   * guide tree (leaves in bucket order) */
  int32_t nm = 0;
  *cells = 0;
  uint8_t* GA = NULL;
  int32_t GL = 0;
  /* the template profile: TW columns of counts over tn rows */
  uint16_t* tprof = NULL;
  int32_t TW = 0, tn = 1;
  if (st == SADREF_OK) {
    if (q == 1) {
      GL = (int32_t)anc_len[0];
      GA = (uint8_t*)malloc((size_t)(GL > 0 ? GL : 1));
      memcpy(GA, anc[0], (size_t)GL);
    } else {
      node_t* nodes = (node_t*)calloc((size_t)(2 * q - 1), sizeof(node_t));
      st = progressive(q, (const uint8_t* const*)anc, anc_len, A, kmer_k, S, go, ge, nodes,
                       merge_list_g, merge_score_g, merge_cells_g, NULL, 0, NULL, NULL);
      if (st == SADREF_OK) {
        node_t* root = &nodes[2 * q - 2];
        GA = (uint8_t*)malloc((size_t)(root->W > 0 ? root->W : 1));
        sadref_consensus(root->cnt, root->W, root->n, A, GA, &GL);
        if (tmpl == 1) {
          TW = root->W;
          tn = root->n;
          tprof = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(TW > 0 ? TW : 1) * (size_t)A);
          memcpy(tprof, root->cnt, sizeof(uint16_t) * (size_t)TW * (size_t)A);
        }
        nm = q - 1;
        for (int32_t t = 0; t < nm; ++t) *cells += merge_cells_g[t];
      }
      free_nodes(nodes, 2 * q - 1);
      free(nodes);
    }
  }
  if (st == SADREF_OK) {
    *ga_len = GL;
    if (GL > ga_cap) st = SADREF_E_CAPACITY;
    else memcpy(ga, GA, (size_t)GL);
  }

  /* refinement: every bucket alignment against GA as a one-row profile; the
   * bucket's own columns stay together (only all-gap columns are inserted) */
  uint8_t** bops = (uint8_t**)calloc((size_t)(q > 0 ? q : 1), sizeof(uint8_t*));
  int32_t* bnops = (int32_t*)calloc((size_t)(q > 0 ? q : 1), sizeof(int32_t));
  if (st == SADREF_OK && tprof == NULL) {
    /* GA as a one-row profile */
    TW = GL;
    tn = 1;
    tprof = (uint16_t*)calloc((size_t)(GL > 0 ? GL : 1) * (size_t)A, sizeof(uint16_t));
    for (int32_t c = 0; c < GL; ++c) tprof[(size_t)c * A + GA[c]] = 1;
  }
  if (st == SADREF_OK) {
    int* rst = (int*)calloc((size_t)(q > 0 ? q : 1), sizeof(int));
    refine_ctx_t rc = {nonempty, width_b, bucket_off, prof, tprof, TW, tn, A, S, go, ge, bops,
                       bnops, merge_score_g + nm, merge_cells_g + nm, merge_list_g + 2 * nm,
                       rst};
    for_items(q, refine_one_bucket, &rc);
    for (int32_t u = 0; u < q && st == SADREF_OK; ++u) {
      st = rst[u];
      if (st == SADREF_OK) *cells += merge_cells_g[nm + u];
    }
    free(rst);
  }

  /* the refinement op strings, for callers that check the glue */
  if (st == SADREF_OK && rf_ops_off) {
    int64_t tot = 0;
    for (int32_t u = 0; u < q; ++u) {
      rf_ops_off[u] = tot;
      if (rf_ops && tot + bnops[u] <= rf_ops_cap) memcpy(rf_ops + tot, bops[u], (size_t)bnops[u]);
      tot += bnops[u];
    }
    rf_ops_off[q] = tot;
    if (tmpl_width) *tmpl_width = TW;
    if (rf_ops && tot > rf_ops_cap) st = SADREF_E_CAPACITY;
  }

  /* glue: the bucket columns' places in the joined alignment */
  if (st == SADREF_OK) {
    int64_t* ooff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(q + 1));
    int32_t* wu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(q > 0 ? q : 1));
    int64_t tot_ops = 0, tot_w = 0;
    for (int32_t u = 0; u < q; ++u) {
      ooff[u] = tot_ops;
      tot_ops += bnops[u];
      wu[u] = width_b[nonempty[u]];
      tot_w += wu[u];
    }
    ooff[q] = tot_ops;
    uint8_t* allops = (uint8_t*)malloc((size_t)(tot_ops > 0 ? tot_ops : 1));
    for (int32_t u = 0; u < q; ++u) memcpy(allops + ooff[u], bops[u], (size_t)bnops[u]);
    int32_t* to_g = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tot_w > 0 ? tot_w : 1));
    st = sadref_glue(q, TW, allops, ooff, wu, to_g, width_g);
    int64_t base = 0;
    for (int32_t u = 0; u < q && st == SADREF_OK; ++u) {
      int32_t b = nonempty[u];
      int32_t lo = bucket_off[b], nb = bucket_off[b + 1] - lo;
      for (int32_t a = 0; a < nb; ++a) {
        int32_t id = members[lo + a];
        for (int64_t r = offsets[id]; r < offsets[id + 1]; ++r)
          colmap_g[r] = to_g[base + colmap_b[r]];
      }
      base += wu[u];
    }
    free(ooff);
    free(wu);
    free(allops);
    free(to_g);
  }
  *n_merges_g = nm + q;

  for (int32_t u = 0; u < q; ++u) {
    free(anc[u]);
    free(bops[u]);
  }
  for (int32_t b = 0; b < p; ++b) free(prof[b]);
  free(prof);
  free(anc);
  free(anc_len);
  free(bops);
  free(bnops);
  free(tprof);
  free(GA);
  free(nonempty);
  return st;
}

int sadref_refine_template(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                           int32_t p, const int32_t* bucket_off, const int32_t* members,
                           const int32_t* colmap_b, const int32_t* width_b,
                           int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge, int32_t tmpl,
                           uint8_t* ga, int32_t ga_cap, int32_t* ga_len,
                           int32_t* colmap_g, int32_t* width_g,
                           int64_t* merge_score_g, int32_t* merge_list_g, int64_t* merge_cells_g,
                           int32_t* n_merges_g, int64_t* cells) {
  return sadref_refine_template_ops(n, A, codes, offsets, p, bucket_off, members, colmap_b,
                                    width_b, kmer_k, S, go, ge, tmpl, ga, ga_cap, ga_len,
                                    colmap_g, width_g, merge_score_g, merge_list_g,
                                    merge_cells_g, n_merges_g, cells, NULL, 0, NULL, NULL);
}

int sadref_refine(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                  int32_t p, const int32_t* bucket_off, const int32_t* members,
                  const int32_t* colmap_b, const int32_t* width_b,
                  int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge,
                  uint8_t* ga, int32_t ga_cap, int32_t* ga_len,
                  int32_t* colmap_g, int32_t* width_g,
                  int64_t* merge_score_g, int32_t* merge_list_g, int64_t* merge_cells_g,
                  int32_t* n_merges_g, int64_t* cells) {
  return sadref_refine_template(n, A, codes, offsets, p, bucket_off, members, colmap_b, width_b,
                                kmer_k, S, go, ge, 0, ga, ga_cap, ga_len, colmap_g, width_g,
                                merge_score_g, merge_list_g, merge_cells_g, n_merges_g, cells);
}

/* ------------------------------------------------------------------------
 * Tree-dependent refinement of the glued alignment (the refinement of the
 * global alignment that the paper's closing section asks for, in the manner
 * of MUSCLE's tree-dependent stage): every edge of the ancestors' guide tree
 * splits the buckets into two groups; the two groups' parts of the current
 * alignment (all-gap columns dropped) are re-aligned as two profiles, and the
 * result replaces the alignment iff its profile score beats the score of the
 * alignment the two parts already have.  Edges are visited deepest first
 * (ties by node id); the root's second child is skipped (same split as its
 * first); passes repeat until one accepts nothing or `passes` are done. */

/* score of aligning the two column profiles by the op string `ops`: column
 * scores of M ops minus (go + (l - 1) ge) n1 n2 per maximal X run and per
 * maximal Y run (terminal runs included) */
static int64_t ops_score(const uint16_t* C1, int32_t n1, const uint16_t* C2, int32_t n2,
                         int32_t A, const int8_t* S, int32_t go, int32_t ge, const uint8_t* ops,
                         int32_t nops) {
  const int64_t G = (int64_t)n1 * n2;
  int64_t total = 0;
  int32_t i = 0, j = 0, prev = -1;
  for (int32_t t = 0; t < nops; ++t) {
    const int op = ops[t];
    if (op == SADREF_OP_M) {
      int64_t sc = 0;
      for (int32_t a = 0; a < A; ++a)
        for (int32_t b = 0; b < A; ++b)
          sc += (int64_t)C1[(size_t)i * A + a] * S[a * A + b] * (int64_t)C2[(size_t)j * A + b];
      total += sc;
      ++i;
      ++j;
    } else if (op == SADREF_OP_X) {
      total -= (prev == SADREF_OP_X ? (int64_t)ge : (int64_t)go) * G;
      ++i;
    } else {
      total -= (prev == SADREF_OP_Y ? (int64_t)ge : (int64_t)go) * G;
      ++j;
    }
    prev = op;
  }
  return total;
}

int sadref_refine_tree(int32_t n, int32_t A, const uint8_t* codes, const int64_t* offsets,
                       int32_t p, const int32_t* bucket_off, const int32_t* members,
                       const int32_t* colmap_in, int32_t width_in, const int32_t* tree,
                       int32_t kmer_k, const int8_t* S, int32_t go, int32_t ge, int32_t passes,
                       int32_t* colmap_out, int32_t* width_out, int32_t* n_steps,
                       int32_t* rec_node, int64_t* rec_old, int64_t* rec_new, int32_t rec_cap,
                       int32_t* n_accepted) {
  int st = validate_seqs(n, A, codes, offsets, kmer_k);
  if (st) return st;
  if (p < 1 || go < ge || ge < 0 || passes < 0 || width_in < 0) return SADREF_E_INVAL;
  if (bucket_off[0] != 0 || bucket_off[p] != n) return SADREF_E_INVAL;
  if (n > 65535) return SADREF_E_CAPACITY; /* column counts are 16-bit */
  const int64_t total = offsets[n];
  /* leaf u of the ancestor tree = the u-th non-empty bucket */
  int32_t q = 0;
  int32_t* seq_u = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t b = 0; b < p; ++b) {
    if (bucket_off[b + 1] - bucket_off[b] <= 0) continue;
    for (int32_t t = bucket_off[b]; t < bucket_off[b + 1]; ++t) seq_u[members[t]] = q;
    ++q;
  }
  for (int64_t r = 0; r < total; ++r) {
    if (colmap_in[r] < 0 || colmap_in[r] >= width_in) st = SADREF_E_INVAL;
    colmap_out[r] = colmap_in[r];
  }
  int32_t W = width_in;
  *n_steps = 0;
  *n_accepted = 0;
  const int32_t nn = q >= 2 ? 2 * q - 1 : 1;
  int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)nn);
  char* in1 = (char*)malloc((size_t)(q > 0 ? q : 1));
  int32_t nsplit = 0;
  if (st == SADREF_OK && q >= 2) {
    for (int32_t v = 0; v < nn; ++v) parent[v] = -1;
    for (int32_t t = 0; t < q - 1; ++t) {
      const int32_t a = tree[2 * t], b = tree[2 * t + 1];
      if (a < 0 || b < 0 || a >= q + t || b >= q + t || parent[a] >= 0 || parent[b] >= 0 ||
          a == b) {
        st = SADREF_E_INVAL;
        break;
      }
      parent[a] = q + t;
      parent[b] = q + t;
    }
    if (st == SADREF_OK) {
      /* depths from the root (node 2q - 2, the last merge), then the visiting
       * order: deeper first, smaller id first among equals */
      for (int32_t v = nn - 1; v >= 0; --v) depth[v] = parent[v] < 0 ? 0 : depth[parent[v]] + 1;
      const int32_t skip = tree[2 * (q - 2) + 1];
      for (int32_t v = 0; v < nn - 1; ++v)
        if (v != skip) order[nsplit++] = v;
      for (int32_t x = 1; x < nsplit; ++x) {  /* insertion sort by (-depth, id) */
        const int32_t v = order[x];
        int32_t y = x - 1;
        while (y >= 0 && (depth[order[y]] < depth[v] ||
                          (depth[order[y]] == depth[v] && order[y] > v))) {
          order[y + 1] = order[y];
          --y;
        }
        order[y + 1] = v;
      }
    }
  }
  for (int32_t pass = 0; pass < passes && st == SADREF_OK && q >= 2; ++pass) {
    int32_t accepted = 0;
    for (int32_t x = 0; x < nsplit && st == SADREF_OK; ++x) {
      const int32_t v = order[x];
      /* group 1: the sequences of the buckets (leaves) under v */
      for (int32_t u = 0; u < q; ++u) {
        int32_t w = u;
        while (w >= 0 && w != v) w = parent[w];
        in1[u] = w == v;
      }
      /* per column: counts of each group */
      uint16_t* cnt = (uint16_t*)calloc((size_t)2 * (size_t)(W > 0 ? W : 1) * (size_t)A,
                                        sizeof(uint16_t));
      int32_t n1 = 0, n2 = 0;
      for (int32_t i = 0; i < n; ++i) {
        const int g = in1[seq_u[i]] ? 0 : 1;
        if (g == 0) ++n1;
        else ++n2;
        for (int64_t r = offsets[i]; r < offsets[i + 1]; ++r)
          cnt[((size_t)g * W + colmap_out[r]) * A + codes[r]] += 1;
      }
      /* the two parts as profiles (columns with a residue of the group) and
       * the op string of their present alignment */
      int32_t* idx1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(W > 0 ? W : 1));
      int32_t* idx2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(W > 0 ? W : 1));
      uint16_t* C1 = (uint16_t*)calloc((size_t)(W > 0 ? W : 1) * A, sizeof(uint16_t));
      uint16_t* C2 = (uint16_t*)calloc((size_t)(W > 0 ? W : 1) * A, sizeof(uint16_t));
      uint8_t* old_ops = (uint8_t*)malloc((size_t)(W > 0 ? W : 1));
      int32_t W1 = 0, W2 = 0;
      for (int32_t c = 0; c < W; ++c) {
        int h1 = 0, h2 = 0;
        for (int32_t a = 0; a < A; ++a) {
          h1 |= cnt[((size_t)0 * W + c) * A + a] > 0;
          h2 |= cnt[((size_t)1 * W + c) * A + a] > 0;
        }
        idx1[c] = h1 ? W1 : -1;
        idx2[c] = h2 ? W2 : -1;
        if (h1) memcpy(C1 + (size_t)W1++ * A, cnt + ((size_t)0 * W + c) * A, sizeof(uint16_t) * A);
        if (h2) memcpy(C2 + (size_t)W2++ * A, cnt + ((size_t)1 * W + c) * A, sizeof(uint16_t) * A);
        old_ops[c] = h1 && h2 ? SADREF_OP_M : (h1 ? SADREF_OP_X : SADREF_OP_Y);
        if (!h1 && !h2) st = SADREF_E_INVAL; /* an all-gap column */
      }
      const int64_t s_old = ops_score(C1, n1, C2, n2, A, S, go, ge, old_ops, W);
      uint8_t* ops = (uint8_t*)malloc((size_t)(W1 + W2 > 0 ? W1 + W2 : 1));
      int32_t nops = 0;
      int64_t s_new = 0;
      if (st == SADREF_OK)
        st = sadref_profile_align(C1, W1, n1, C2, W2, n2, A, S, go, ge, ops, &nops, &s_new);
      if (st == SADREF_OK) {
        if (*n_steps < rec_cap) {
          rec_node[*n_steps] = v;
          rec_old[*n_steps] = s_old;
          rec_new[*n_steps] = s_new;
        }
        ++*n_steps;
        if (s_new > s_old) {
          /* lay the residues out by the new op string */
          int32_t* map1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(W1 > 0 ? W1 : 1));
          int32_t* map2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(W2 > 0 ? W2 : 1));
          int32_t i = 0, j = 0;
          for (int32_t t = 0; t < nops; ++t) {
            if (ops[t] != SADREF_OP_Y) map1[i++] = t;
            if (ops[t] != SADREF_OP_X) map2[j++] = t;
          }
          for (int32_t s = 0; s < n; ++s) {
            const int g1 = in1[seq_u[s]];
            for (int64_t r = offsets[s]; r < offsets[s + 1]; ++r)
              colmap_out[r] = g1 ? map1[idx1[colmap_out[r]]] : map2[idx2[colmap_out[r]]];
          }
          W = nops;
          ++accepted;
          ++*n_accepted;
          free(map1);
          free(map2);
        }
      }
      free(cnt);
      free(idx1);
      free(idx2);
      free(C1);
      free(C2);
      free(old_ops);
      free(ops);
    }
    if (accepted == 0) break;
  }
  *width_out = W;
  free(seq_u);
  free(parent);
  free(depth);
  free(order);
  free(in1);
  return st;
}
