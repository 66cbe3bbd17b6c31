/*
 * sad.h -- C-ABI of the MI355X (gfx950) library for the data-parallel core of
 * Sample-Align-D (F. Saeed, A. Khokhar, "Sample-Align-D: A High Performance
 * Multiple Sequence Alignment System using Phylogenetic Sampling and Domain
 * Decomposition", arXiv 0901.2742).
 *
 * Problem statement (Section 2, algorithm box; Section 2.2): given N
 * sequences, insert gaps so that all rows have equal length and the sum-of-
 * pairs score of the result is high.  The method sample-sorts the sequences
 * into p buckets by k-mer rank, aligns every bucket independently, and glues
 * the bucket alignments through a global ancestor.  The four calls below are
 * the four stages of that pipeline, in order.
 *
 * Conventions for every call
 *  - Pointers named d_* are device pointers (HBM of the current HIP device);
 *    everything else is host memory.  All arrays are owned by the caller; the
 *    library never frees or keeps them.  Inputs are read-only.
 *  - Device workspace of the four stage calls is caller-owned: each call takes
 *    (d_ws, ws_bytes), a 256-byte aligned device block that it uses only
 *    while it runs (nothing in it survives the call), sized by the call's
 *    sad_*_workspace query.  A block that turns out too small gives
 *    SAD_E_CAPACITY, and sad_workspace_needed() then returns a size that
 *    suffices.  d_ws = NULL (ws_bytes = 0) lets the library use its own
 *    per-device workspace instead (grown on demand, kept until sad_release());
 *    the other calls always do.  Besides workspaces the library keeps, per
 *    device, a status word, pinned host staging, the alignment engine's
 *    boundary-row areas (zeroed once; tags in them must only grow) and the
 *    autotuner's cache, for the life of the process.
 *  - Work is enqueued on `stream`; each call synchronises that stream before
 *    it returns so that it can report device-side errors in its status
 *    (except sad_partition_noalloc).
 *  - Residue codes are 0..A-1 (A = 20 proteins, A = 4 DNA).  A k-mer tau of
 *    a sequence x at position t is sum_u x[t+u] * A^(k-1-u); A^k <= 65536.
 *  - Limits: sequence length <= 8192; profile width <= 4096 columns; at most
 *    8000 sequences per bucket and 8000 buckets; DP values must stay within
 *    the bound described at sad_align_buckets (otherwise SAD_E_OVERFLOW).
 *  - Status codes are returned; no exception crosses the ABI.  On error the
 *    contents of the outputs are unspecified.  sad_last_error() gives a
 *    message for the calling thread's last failure.
 */
#ifndef SAD_H
#define SAD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SAD_OK 0
#define SAD_E_INVAL (-1)        /* bad code, L < k, N < 2p, go < ge, bad alphabet, bad k */
#define SAD_E_CAPACITY (-2)     /* a caller capacity or a library limit is too small */
#define SAD_E_OVERFLOW (-3)     /* a DP value bound exceeds the 64-bit DP's range */
#define SAD_E_DEVICE (-4)       /* HIP runtime failure */
#define SAD_E_UNIMPLEMENTED (-5)

/* mode flags (sad_params.mode) */
#define SAD_PLAIN 0u            /* column scores on the vector ALUs */
#define SAD_BATCHED_MFMA 1u     /* column scores on int8 matrix cores (same results) */

/* refinement templates (sad_refine_template) */
#define SAD_TEMPLATE_GA 0       /* GA, the consensus of the ancestors' alignment, as one row */
#define SAD_TEMPLATE_GA_MSA 1   /* the ancestors' alignment itself, q rows */

/* N sequences: residue codes of sequence i are d_codes[d_offsets[i] ..
 * d_offsets[i+1]).  total_len must equal d_offsets[n]; max_len must be >= every
 * length (both are checked on the device). */
typedef struct sad_seqs {
  int32_t n;
  int32_t alphabet;            /* 20 or 4 */
  const uint8_t* d_codes;      /* [total_len] */
  const int64_t* d_offsets;    /* [n + 1], d_offsets[0] == 0 */
  int64_t total_len;
  int32_t max_len;
} sad_seqs;

/* Method parameters.  subst is a host pointer to the A x A int8 substitution
 * matrix (row-major, symmetric).  Gap runs of length l cost
 * gap_open + (l - 1) * gap_extend (gap_open >= gap_extend >= 0). */
typedef struct sad_params {
  int32_t kmer_k;              /* k-mer length of the similarity (Section 2) */
  int32_t p;                   /* number of buckets ("processors") */
  int32_t s_max;               /* cap on the number of global samples (1024) */
  const int8_t* subst;         /* host, A x A */
  int32_t gap_open;
  int32_t gap_extend;
  uint32_t mode;               /* SAD_PLAIN or SAD_BATCHED_MFMA */
} sad_params;

/* Alignment results (device arrays, caller-allocated). */
typedef struct sad_msa {
  int32_t* d_colmap;           /* [total_len]: column of each residue */
  int32_t* d_width;            /* per bucket [p] (bucket alignments) or [1] (glued) */
  int64_t* d_merge_score;      /* per alignment step (see each call) */
  int32_t* d_merge_list;       /* pairs of cluster ids per alignment step */
  int64_t* d_merge_cells;      /* DP cells W1 * W2 per alignment step */
  int64_t* d_cells;            /* [1]: total DP cells */
} sad_msa;

/*
 * Stage 1 -- k-mer rank (Section 2 "k-mer Rank", Section 2.3.1, steps 1-6 of
 * the algorithm box).  Processor c of the paper holds the contiguous chunk
 * [floor(c N / p), floor((c+1) N / p)).  With F(i,j) = floor(c_ij 2^31 / d_ij),
 * c_ij = sum_tau min(n_i(tau), n_j(tau)) and d_ij = min(L_i, L_j) - k + 1:
 *   local rank  K_loc(i) = sum_{j in chunk(i)} F(i,j)  (self included);
 *   each chunk is sorted by (K_loc(i), i) and k_s = min(p-1, max(1, s_max/p),
 *   w_min - 1) samples are taken at positions floor(t w / (k_s+1)), t=1..k_s;
 *   globalised rank d_key[i] = sum over all p k_s samples s of F(i,s).
 * Outputs: d_key[n] (uint64), d_sample_ids[p k_s] (chunk-major), *n_samples
 * (host).  SAD_E_CAPACITY (with *n_samples set) if p k_s > sample_cap.
 */
int32_t sad_kmer_rank(const sad_seqs* seqs, const sad_params* prm, uint64_t* d_key,
                      int32_t* d_sample_ids, int32_t sample_cap, int32_t* n_samples,
                      void* d_ws, size_t ws_bytes, hipStream_t stream);
/* Workspace of sad_kmer_rank (exact): k-mer lists of every sequence, local
 * ranks and the chunk order; about 4 total_len + 16 n bytes. */
int32_t sad_kmer_rank_workspace(const sad_seqs* seqs, const sad_params* prm, size_t* ws_bytes);

/*
 * Rank against a given sample (Section 2.3.1, Table 1): d_key[i] = sum over
 * the n_samples ids s in d_sample_ids of F(i, s) for every sequence i (self
 * included when i is listed), the globalised rank's formula with the sample
 * chosen by the caller.  d_sample_ids == NULL takes all n sequences: the
 * centralised rank, each sequence against the whole set, which the sampled
 * (globalised) rank of sad_kmer_rank approximates.  Inputs: seqs as for
 * sad_kmer_rank, kmer_k >= 1, d_sample_ids[n_samples] (device, ids in [0, n))
 * or NULL.  Output: d_key[n] (device uint64, caller-owned).  SAD_E_INVAL for
 * a bad sequence set, k, count or id (ids are checked on the device; an id
 * out of range is never dereferenced).
 */
int32_t sad_rank_against(const sad_seqs* seqs, int32_t kmer_k, const int32_t* d_sample_ids,
                         int32_t n_samples, uint64_t* d_key, hipStream_t stream);

/*
 * Stage 2 -- regular-sampling partition (Section 2.3.2, steps 7-10).  Each chunk
 * is sorted by the composite key (key_i, i); p-1 keys are taken at positions
 * floor(t w / p), t = 1..p-1; the p(p-1) gathered keys Y are sorted and the
 * pivots are Y at 1-based positions floor(p/2) + (t-1) p, t = 1..p-1.
 * bucket(i) = number of pivots strictly below (key_i, i).
 * Outputs (device): d_pivot_key/d_pivot_id[p-1], d_bucket[n],
 * d_bucket_off[p+1] (exclusive prefix of bucket sizes), d_members[n] (ids of
 * each bucket, ascending).
 */
int32_t sad_partition(const sad_seqs* seqs, const uint64_t* d_key, const sad_params* prm,
                      uint64_t* d_pivot_key, int32_t* d_pivot_id, int32_t* d_bucket,
                      int32_t* d_bucket_off, int32_t* d_members, void* d_ws, size_t ws_bytes,
                      hipStream_t stream);
/* Workspace of sad_partition (exact): the chunk order, the p(p-1) regular
 * samples and their sorted copy, per-block bucket counts; about
 * 4n + 24 p(p-1) + 4 p ceil(n/256) bytes. */
int32_t sad_partition_workspace(const sad_seqs* seqs, const sad_params* prm, size_t* ws_bytes);

/*
 * sad_partition without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, checks and outputs as sad_partition
 * (bit-identical results); its scratch is a static device array of 32 MiB per
 * device (enough for 200000 ids in 1024 buckets), held from the library's
 * load until the process ends.  SAD_E_CAPACITY when the partition needs more
 * (about 4n + 24 p(p-1) + 4 p ceil(n/256) bytes).  The call only enqueues
 * kernels on `stream` and returns without synchronising (launch failures are
 * SAD_E_DEVICE); it calls no allocator.  Every call on one device shares the
 * one scratch array: calls that overlap in time on a device (different
 * streams, or host threads) race and must be serialised by the caller, e.g.
 * by issuing them on one stream.
 */
int32_t sad_partition_noalloc(const sad_seqs* seqs, const uint64_t* d_key,
                              const sad_params* prm, uint64_t* d_pivot_key, int32_t* d_pivot_id,
                              int32_t* d_bucket, int32_t* d_bucket_off, int32_t* d_members,
                              hipStream_t stream);

/*
 * Stage 3 -- independent alignment of every bucket (Section 2.3.3, step 11; the
 * sequential aligner is k-mer similarity + UPGMA + progressive profile-profile
 * alignment):
 *   - UPGMA on F among the bucket's members (leaves in d_members order) merges
 *     the active pair with the largest average similarity, compared exactly;
 *     ties go to the smallest (min id, max id); cluster t gets id n_b + t;
 *   - each merge aligns P1 = child with the smaller id against P2 with affine
 *     gaps: column score s(i,j) = sum_ab C1[i][a] S[a][b] C2[j][b]; a gap run
 *     of length l costs G (go + (l-1) ge), G = n1 n2; terminal gaps charged;
 *     among optimal alignments the one whose op string read backwards is
 *     lexicographically smallest (M < X < Y) is taken; rows of P1 then P2.
 * Outputs (device, out): d_colmap[total_len]: column of each residue in its
 * bucket's alignment; d_width[p]; bucket b's merges occupy slots
 * [d_bucket_off[b], d_bucket_off[b] + n_b - 1) of d_merge_score[n],
 * d_merge_cells[n] and d_merge_list[2n] (local cluster ids); d_cells[1].
 * Value bound: a merge whose (W1 + W2 + 2) n1 n2 max(|S|, go) is below 2^29
 * runs the 32-bit DP, up to 2 * 10^18 the 64-bit DP (same results); beyond
 * that, or if n1 n2 max|S| reaches 2^31 (column scores are 32-bit), the call
 * fails with SAD_E_OVERFLOW.
 */
int32_t sad_align_buckets(const sad_seqs* seqs, const int32_t* d_bucket_off,
                          const int32_t* d_members, const sad_params* prm, sad_msa* out,
                          void* d_ws, size_t ws_bytes, hipStream_t stream);
/* Workspace of sad_align_buckets that suffices for any input with these
 * buckets, under any schedule (reads the p+1 offsets, synchronising
 * `stream`): k-mer lists, the bucket similarity matrices and UPGMA sums
 * (12 sum n_b^2 bytes), and the alignment engine sized for the worst case:
 * profile pools for every merge of W1 + W2 <= min(8192, (leaves below) *
 * max_len) columns, tie bytes and boundary rows for 4096-column profiles per
 * persistent workgroup.  Typical inputs use a small part of it; the engine's
 * pools take whatever space the other buffers leave, so a smaller block
 * often suffices (else SAD_E_CAPACITY, see sad_workspace_needed). */
int32_t sad_align_buckets_workspace(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                    const sad_params* prm, size_t* ws_bytes, hipStream_t stream);

/*
 * Stage 4 -- global ancestor, ancestor-constrained refinement and glue
 * (Section 2.3.3, steps 12-15).  The local ancestor of a bucket is the
 * majority consensus of its alignment (column kept iff 2 residues >= rows;
 * most frequent residue, smallest code on ties).  The q non-empty buckets'
 * ancestors are aligned like a bucket (leaves in bucket order); GA is the
 * consensus of that alignment (GA = the ancestor when q = 1).  Each bucket
 * alignment is then aligned against GA as a one-row profile (G = n_b); its own
 * columns stay together.  Glue: before GA position j (and after the last) an
 * insert slot holds the bucket columns aligned to gaps there, bucket by
 * bucket; then the shared column j; all-gap columns are dropped.
 * Inputs: the stage-3 outputs d_colmap/d_width of `buckets`.
 * Outputs: d_ga[ga_cap] and *ga_len (host; SAD_E_CAPACITY if too small);
 * global_out: d_colmap[total_len], d_width[1]; d_merge_score/d_merge_cells
 * [2p] and d_merge_list[4p]: the q-1 ancestor merges then the q refinement
 * alignments (pairs (bucket, -1)); *n_steps (host) = 2q - 1; d_cells[1].
 */
int32_t sad_refine(const sad_seqs* seqs, const int32_t* d_bucket_off, const int32_t* d_members,
                   const sad_msa* buckets, const sad_params* prm, uint8_t* d_ga,
                   int32_t ga_cap, int32_t* ga_len, sad_msa* global_out, int32_t* n_steps,
                   void* d_ws, size_t ws_bytes, hipStream_t stream);
/* Workspace of sad_refine and sad_refine_template (either template) that
 * suffices for these stage-3 results (reads the p+1 offsets and p widths of
 * `buckets`, synchronising `stream`): bucket profiles, ancestors, GA and the
 * refinement's op strings and glue tables for a template of up to
 * min(4096, sum of widths) columns, then the larger of the ancestors' stage
 * (similarity matrix, guide tree, engine at its worst-case size) and the
 * refinement engine. */
int32_t sad_refine_workspace(const sad_seqs* seqs, const int32_t* d_bucket_off,
                             const sad_msa* buckets, const sad_params* prm, size_t* ws_bytes,
                             hipStream_t stream);

/*
 * Stage 4 with a choice of template.  SAD_TEMPLATE_GA is sad_refine.
 * SAD_TEMPLATE_GA_MSA aligns each bucket alignment against the ancestors'
 * alignment as a profile of q rows (the richer template that the paper's
 * future-work section asks for; Section 2.3.3 speaks of the global ancestor
 * "profile"): column scores sum over its q rows and gap costs scale with
 * G = n_b q; the glue runs over its columns instead of GA's.  GA (the
 * consensus) is still returned in d_ga.  With q = 1 both templates are the
 * bucket's own ancestor as one row.  Merge cells of the refinement steps are
 * W_b times the template's width.  SAD_E_INVAL for an unknown template; the
 * value bound of sad_align_buckets applies to every refinement alignment.
 */
int32_t sad_refine_template(const sad_seqs* seqs, const int32_t* d_bucket_off,
                            const int32_t* d_members, const sad_msa* buckets,
                            const sad_params* prm, int32_t tmpl, uint8_t* d_ga, int32_t ga_cap,
                            int32_t* ga_len, sad_msa* global_out, int32_t* n_steps,
                            void* d_ws, size_t ws_bytes, hipStream_t stream);

/*
 * Tree-dependent refinement of the glued alignment (the refinement of the
 * global alignment for divergent families that the paper's closing section
 * asks for, in the manner of MUSCLE's tree-dependent stage).  Every edge of
 * the ancestors' guide tree splits the sequences into the buckets below it
 * and the rest; edges are visited deeper first (smaller node id first among
 * equals; the root's second child is skipped, it splits like the first).  At
 * each edge the two groups' parts of the current alignment (all-gap columns
 * dropped) become two profiles; their present alignment is scored with the
 * profile objective of sad_align_buckets (column scores C1 S C2^T, affine gap
 * runs scaled by n1 n2, terminal gaps charged), the profiles are re-aligned
 * optimally, and the new layout replaces the alignment iff its score is
 * higher.  Passes over all edges repeat until one changes nothing or
 * `passes` have run.  Each group's own rows keep their alignment.
 * Inputs: seqs, d_bucket_off/d_members as for sad_refine; `glued` = the
 * output of sad_refine / sad_refine_template: d_colmap[total_len], d_width[1]
 * and d_merge_list, whose first q - 1 pairs are the ancestors' merges (leaves
 * 0..q-1 = non-empty buckets in bucket order, merge t makes node q + t).
 * Outputs: out->d_colmap[total_len], out->d_width[1] (device, may not alias
 * glued's); *n_steps and *n_accepted (host); rec (host, rec_cap x 3 int64,
 * may be NULL when rec_cap = 0): per step (tree node, present score, new
 * score).  SAD_E_INVAL for a malformed tree or an alignment with an all-gap
 * column; SAD_E_CAPACITY beyond 65535 sequences or a width above 4096; the
 * value bound of sad_align_buckets applies to every re-alignment.
 */
int32_t sad_refine_tree(const sad_seqs* seqs, const int32_t* d_bucket_off,
                        const int32_t* d_members, const sad_msa* glued, const sad_params* prm,
                        int32_t passes, sad_msa* out, int32_t* n_steps, int32_t* n_accepted,
                        int64_t* rec, int32_t rec_cap, hipStream_t stream);

/* Autotuner for sad_align_buckets (batching of the bucket merges, Section
 * 2.3.3 step 11).  Runs the call on the given buckets under each candidate
 * schedule, once to warm up and three times timed (the fastest counts), with
 * HIP events on `stream`.  Batched mode, one persistent launch over every
 * bucket's merge DAG: column scores as int8 MFMA tiles with a grid of 1, 3/4
 * or 1/2 workgroup per CU, guide trees built inside the launch (buckets of up
 * to 600 members) or by a separate kernel, and cooperative merges (a merge's
 * 4-strip groups spread over idle workgroups) on or off -- 12 schedules; or
 * column scores as vector-ALU dot products (the plain kernel, whose registers
 * and LDS allow several workgroups per CU) with 1, 2 or 3 workgroups per CU
 * and the guide trees inside the launch or separate -- 6 schedules; then the
 * fastest MFMA schedule once more with a shape of its DP strips changed:
 * 16-step chunks instead of 32 (a strip trails the one above by 63 + chunk
 * steps, and each chunk costs a boundary-row check and a tie-word store).
 * Plain mode: 1, 2 or 3 workgroups per CU for the per-level
 * launches.  The fastest is kept in a process-wide cache keyed by (alphabet,
 * n, p, mode, largest bucket, total length) and used by later
 * sad_align_buckets calls with that key; results never depend on the
 * schedule.  `out` receives the last run's (identical) results.  *grid_out =
 * chosen workgroup count (0 = default), *fuse_out = 1 trees in the launch, 0
 * separate, *flags_out: bit 0 cooperative merges, bit 1 MFMA column scores,
 * bit 2 16-step chunks (any of them may be NULL).  The environment variable
 * SAD_SCHEDULE="grid,fuse[,coop[,mfma[,chunk]]]" imposes one schedule on
 * every call instead (for tests that check each candidate). */
int32_t sad_tune(const sad_seqs* seqs, const int32_t* d_bucket_off, const int32_t* d_members,
                 const sad_params* prm, sad_msa* out, int32_t* grid_out, int32_t* fuse_out,
                 int32_t* flags_out, hipStream_t stream);

/* Kernel timing for measurement tools.  on & 1: every launch of the
 * alignment engine kernel (the DP + traceback + merge kernel that dominates
 * stages 3 and 4) is bracketed by HIP events on the call's stream (a replayed
 * launch too: the engine is a graph of its own); the accumulated time and
 * launch count are read (and optionally reset) with sad_profile_read.  on & 2: per-job phase
 * ticks and per-job records as well (sad_profile_phases, sad_profile_jobs;
 * this turns the graph replay of sad_align_buckets off).  Disabled by
 * default. */
int32_t sad_profile_enable(int32_t on);
int32_t sad_profile_read(double* engine_ms, int64_t* engine_launches, int32_t reset);
/* Alignment quality against a known homology (Section 4, the Q measure: the
 * correctly aligned residue pairs over the residue pairs of the reference).
 * The reference is given as homology classes: residues r and r' form a
 * reference pair iff d_class[r] == d_class[r'] (a class holds at most one
 * residue of each sequence, so the two lie in different sequences); the pair
 * is aligned iff d_colmap[r] == d_colmap[r'] (e.g. the glued column map of
 * sad_refine).  Inputs (device): d_colmap[total], d_class[total] with classes
 * 0..nclass-1.  Outputs (host): *aligned_pairs, *true_pairs; Q = aligned /
 * true.  SAD_E_INVAL for a class id out of range (checked on the device),
 * total outside 0..2^31-1 or nclass < 1.  Device workspace: the library's. */
int32_t sad_quality(const int32_t* d_colmap, const int32_t* d_class, int64_t total,
                    int32_t nclass, uint64_t* aligned_pairs, uint64_t* true_pairs,
                    hipStream_t stream);

/* Per-job phase times of the alignment engine while profiling is enabled,
 * summed over jobs (milliseconds): ms_out[0] waiting for a ready job,
 * [1] DP, [2] traceback, [3] merge, [4] publication (device-scope fence and
 * queue hand-off); *jobs = jobs timed.  ms_out needs 5 entries. */
int32_t sad_profile_phases(double* ms_out, int64_t* jobs, int32_t reset);
/* Per-job records of the most recent engine launch made while profiling was
 * enabled: 8 int64 per job slot (slots without a job are all zero), {W1, W2, ops, fetch, start, DP end,
 * traceback end, merge end}; the first word also carries, in bit 32, whether the
 * merge ran cooperatively and, in bits 40..47, how many strip groups its owner
 * ran itself.  Times in nanoseconds from the launch's first job
 * fetch (fetch = the workgroup asked the queue; start = the job was handed
 * to it).  Copies min(cap, n) records to host memory `out` (may be NULL);
 * *njobs = n. */
int32_t sad_profile_jobs(int64_t* out, int64_t cap, int64_t* njobs);

/* Graphs: in batched mode with the guide trees built inside the engine
 * launch, sad_align_buckets records its device work (k-mer lists, similarity
 * matrices, engine set-up, the persistent launch, result kernels) into a
 * hipGraph after a successful eager call and replays it on later calls whose
 * baked-in arguments (buffers, sizes, parameters, stream) are unchanged;
 * SAD_GRAPHS=0 in the environment disables this. */

/* Graph captures and replays of sad_align_buckets since the last reset. */
int32_t sad_profile_graphs(int64_t* captured, int64_t* replayed, int32_t reset);

/* After a stage call on this thread returned SAD_E_CAPACITY because its
 * caller workspace was too small: a workspace size that suffices for the
 * same call (0 otherwise). */
size_t sad_workspace_needed(void);

/* Message for the calling thread's last non-OK status (static storage). */
const char* sad_last_error(void);

/* Frees the library's device workspaces on every device. */
void sad_release(void);

/* Library version string. */
const char* sad_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SAD_H */
