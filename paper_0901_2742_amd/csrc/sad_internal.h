// Internal declarations of the gfx950 library: device status word, workspace
// arena, and the launchers each translation unit exports to the host API.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/sad.h"

namespace sad {

// ------------------------------------------------------------------ limits
constexpr int kMaxLen = 8192;        // longest accepted sequence
constexpr int kMaxWidth = 4096;      // widest profile a DP accepts
// cooperative merges: strips per group, helper tickets per merge, and the
// layout of a workgroup's boundary-row area (a head of 32-bit words, word 0
// the workgroup's tag counter, then per group boundary an H row and an X row
// of kMaxWidth + 1 tagged 64-bit words)
constexpr int kCoopGroupStrips = 4;
constexpr int kMaxHelpers = 3;
constexpr int kCoopMaxGroups = kMaxWidth / 64 / kCoopGroupStrips;
constexpr int kCoopHeadWords = 64;
constexpr int kCoopRowLen = kMaxWidth + 1;
constexpr int64_t kCoopWordsPerWG =
    kCoopHeadWords + (int64_t)(kCoopMaxGroups - 1) * 2 * kCoopRowLen * 2;
// a workgroup's own tagged rows: the same head, then 4 H/X row pairs
constexpr int64_t kTagRowWordsPerWG = kCoopHeadWords + (int64_t)4 * 2 * kCoopRowLen * 2;
constexpr int32_t kHelperTicket = 1 << 30;
constexpr int kMaxAlpha = 20;
constexpr int kMaxGroup = 8000;      // largest bucket (UPGMA keeps 5 ints per member in LDS)
constexpr int32_t kNeg32 = -(1 << 30);  // "minus infinity" of the 32-bit DP

// ------------------------------------------------------------------ device status
// st[0]: first error code (0 = none); st[1]: detail (e.g. needed capacity, low
// 32 bits); st[2]: detail high bits; st[3]: which kernel raised it.
struct DevStatus {
  int32_t code;
  int32_t detail_lo;
  int32_t detail_hi;
  int32_t where;
};

__device__ inline void raise_error(DevStatus* st, int32_t code, int64_t detail, int32_t where) {
  if (atomicCAS(&st->code, 0, code) == 0) {
    st->detail_lo = (int32_t)(detail & 0xffffffff);
    st->detail_hi = (int32_t)(detail >> 32);
    st->where = where;
  }
}

// where-codes for error reports
enum Where : int32_t {
  W_VALIDATE = 1, W_KMER = 2, W_RANK = 3, W_PART = 4, W_UPGMA = 5, W_ENGINE = 6,
  W_ENGINE_POOL = 7, W_ENGINE_TB = 8, W_ENGINE_WIDTH = 9, W_ENGINE_BOUND = 10,
  W_ENGINE_WAIT = 11, W_REFINE = 12, W_ENGINE_LINK = 13, W_QUALITY = 14,
};

// ------------------------------------------------------------------ arena
// Bump allocator over one device block; reset per call.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  void reset() { used = 0; }
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// ------------------------------------------------------------------ k-mer lists
// Entry = (tau << 16) | count, sorted by tau; the list of sequence i starts at
// its residue offset off[i] and holds nu[i] entries.
struct KmerLists {
  const uint32_t* entries;
  const int64_t* off;
  const int32_t* nu;
  const int64_t* seq_off;  // sequence offsets (lengths)
};

// ------------------------------------------------------------------ launchers
// kmer.hip
void launch_validate(const sad_seqs& s, int k, DevStatus* st, hipStream_t stream);
void launch_kmer_lists(const uint8_t* codes, const int64_t* offsets, int n, int A, int k,
                       uint32_t* entries, int64_t* kl_off, int32_t* nu, DevStatus* st,
                       hipStream_t stream);
// Pair sums over k-mer lists: for every "row" sequence r (given by row_ids or
// 0..nrows-1), sum F(r, c) over the column set, or write F rows.
void launch_rowsum_chunk(const KmerLists& kl, int n, int p, int k, int kspace,
                         uint64_t* out, hipStream_t stream);
void launch_rowsum_list(const KmerLists& kl, int n, const int32_t* cols, int ncols, int k,
                        int kspace, uint64_t* out, DevStatus* st, hipStream_t stream);
// (max_group: the largest group; every group's n_g x n_g matrix is written)
void launch_fmatrix_groups(const KmerLists& kl, const int32_t* group_off, const int32_t* ids,
                           int ngroups, int max_group, const int64_t* fm_off, int k, int kspace,
                           uint32_t* F, hipStream_t stream);
void launch_chunk_sort(const uint64_t* key, int n, int p, int32_t* sorted, hipStream_t stream);
void launch_pick_samples(const int32_t* sorted, int n, int p, int ks, int32_t* sample_ids,
                         hipStream_t stream);

// partition.hip
void launch_partition(const uint64_t* key, int n, int p, const int32_t* sorted,
                      uint64_t* Ykey, int32_t* Yid, uint64_t* Ysorted_key, int32_t* Ysorted_id,
                      uint64_t* pivot_key, int32_t* pivot_id, int32_t* bucket,
                      int32_t* blk_cnt, int32_t* total, int32_t* bucket_off, int32_t* members,
                      hipStream_t stream);
struct PartitionScratch {
  int32_t* sorted;          // [n] ids in (key, id) order within each chunk
  uint64_t *Yk, *Ysk;       // [p (p - 1)] regular samples, then sorted
  int32_t *Yi, *Ysi;
  int32_t* blk;             // [blocks x p] per-block bucket counts
  int32_t* total;           // [p]
};
size_t partition_scratch(int n, int p, char* base, PartitionScratch* ps);
// chunk sort + partition of n ids with keys `key` into p buckets
void launch_partition_keys(const uint64_t* key, int n, int p, const PartitionScratch& ps,
                           uint64_t* pivot_key, int32_t* pivot_id, int32_t* bucket,
                           int32_t* bucket_off, int32_t* members, hipStream_t stream);
// records a failure for sad_last_error() and returns code (api.hip)
int32_t report_error(int32_t code, const std::string& msg);

// upgma.hip: one workgroup per group; F given per group at fm_off (n_g x n_g).
// alignment quality against homology classes (quality.hip): sums[0] aligned
// pairs, sums[1] true pairs; cnt/cursor nclass, off nclass + 1, cols total
void launch_quality(const int32_t* colmap, const int32_t* cls, int64_t total, int32_t nclass,
                    int32_t* cnt, int32_t* off, int32_t* cursor, int32_t* cols,
                    unsigned long long* sums, DevStatus* st, hipStream_t stream);
void launch_upgma(const uint32_t* F, const int64_t* fm_off, const int32_t* group_off,
                  int ngroups, int max_n, uint64_t* Swork, int32_t* merges_out,
                  const int32_t* merge_base, DevStatus* st, hipStream_t stream);

// engine.hip: progressive alignment engine (see engine.hip for the layout)
struct EngineArgs {
  // nodes
  int32_t* node_W;
  int32_t* node_n;
  int64_t* node_prof;     // offset in profile pool (uint16 units)
  int64_t* node_up;       // offset in up pool (int32 units)
  int32_t* node_parent;   // parent node or -1
  uint16_t* prof_pool;
  int32_t* up_pool;
  unsigned long long* prof_top;  // bump pointers
  unsigned long long* up_top;
  int64_t prof_cap;
  int64_t up_cap;
  // jobs
  int32_t njobs;
  int32_t* job_a;         // P1 node (smaller id)
  int32_t* job_b;         // P2 node
  int32_t* job_out;       // output node
  int32_t* job_next;      // job waiting on this one's output node, or -1
  int32_t* job_pending;   // unfinished children per job
  int64_t* job_score;
  int64_t* job_cells;
  int64_t* job_ops_off;   // where to write the op string (or -1)
  uint8_t* ops_out;
  // queue
  int32_t* queue;
  int32_t* queue_flag;
  int32_t* queue_head;
  int32_t* queue_tail;
  // DP scratch (per workgroup)
  uint32_t* tb;           // tie bytes, packed four per word
  int64_t tb_words_per_wg;
  int32_t* bnd;           // strip boundary rows: link_rows x {H, X} x link_stride ints
  int64_t link_words_per_wg;
  int32_t link_rows;
  int32_t link_stride;
  // scoring
  int32_t A;
  int8_t S[kMaxAlpha * kMaxAlpha];
  int32_t go, ge;
  int32_t smax;           // max |S|
  uint32_t mode;
  int32_t chunk;          // steps per chunk of the MFMA kernel's 32-bit strips: 32 or 16
  int64_t wait_ticks;     // queue wait limit in s_memrealtime ticks
  unsigned long long* phase_acc;  // optional: ticks in queue wait, DP, traceback, merge; jobs
  long long* job_rec;  // optional: per job slot W1, W2, ops and five phase timestamps (8 words)
  int32_t nrec;        // job slots in job_rec
  int32_t no_push;     // 1: finished jobs do not queue their parents (level-by-level launches)
  // Per job slot: hand-off word between a finished job and its parent's
  // creation (0 neither yet, 1 the job finished first, 2 the parent exists):
  // whichever comes second releases the job's share of the parent's count.
  int32_t* job_link;
  // Fused guide trees (up_ngroups > 0): workgroups first build the UPGMA
  // trees of groups claimed from *up_next, creating each merge's job as soon
  // as it is decided; leaves are nodes group_off[g] + x, internal nodes
  // up_N + slot.
  const uint32_t* up_F;
  const int64_t* up_fm_off;
  uint64_t* up_Sw;        // pair sums of groups above the in-LDS size (F's offsets)
  const int32_t* up_group_off;
  int32_t up_ngroups, up_N;
  int32_t* up_merges;
  int32_t* up_next;
  // Cooperative merges (batched kernel, 32-bit DP): a merge of more than 4
  // strips is cut into groups of 4 consecutive strips; its owner and helper
  // workgroups (queued as tickets job | kHelperTicket while workgroups wait
  // idle) claim the groups in order.  Boundary rows between groups pass
  // through coop_buf (uncached memory, one area per owner workgroup: a tag
  // counter, then tagged H and X rows per group boundary), the owner's
  // tie-byte scratch receives every strip.
  int32_t queue_cap;        // tickets the queue holds
  int32_t* jobs_done;       // merges finished; the last one sets *finished
  int32_t* finished;
  int32_t* wait_sites;      // bit w set when a wait of site w ran out of time
  int32_t* coop_next;       // per job slot: next group to claim
  int32_t* coop_strips;     // per job slot: strips finished
  int32_t* coop_owner;      // per job slot: owner workgroup + 1
  int32_t* coop_tag;        // per job slot: tag of its group boundary rows
  int64_t* coop_score;      // per job slot: H(W1, W2)
  int32_t* coop_buf;
  int64_t coop_words_per_wg;
  int32_t coop_wgs;         // owner workgroups coop_buf has room for (0: no cooperation)
  // Boundary rows of the 32-bit strips inside a workgroup (batched kernel):
  // per workgroup a tag counter, then 4 tagged H/X row pairs (zeroed once,
  // kept for the process)
  int32_t* trow;
  int64_t trow_words_per_wg;
  DevStatus* st;
};
void launch_engine(const EngineArgs& a, int nwg, hipStream_t stream);
int engine_workgroups();
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t stream);

// Leaf r is sequence ids[r] (or r when ids is null): node node_base + r, its
// one-hot profile at offsets[id] * A and its column map at offsets[id].
void launch_make_leaves(const uint8_t* codes, const int64_t* offsets, const int32_t* ids,
                        int nleaves, int A, int32_t node_base, int32_t* node_W, int32_t* node_n,
                        int64_t* node_prof, int64_t* node_up, int32_t* node_parent,
                        uint16_t* prof_pool, int64_t total_len, hipStream_t stream);
// Jobs from UPGMA merge lists (one group per bucket, slots = member positions).
int engine_fused_max_group();  // largest group the engine builds its guide tree for
int engine_fused_lds_group();  // largest such group whose pair sums stay in LDS
void launch_make_jobs(const int32_t* merges, const int32_t* group_off, int ngroups, int nslots,
                      int32_t internal_base, int32_t* node_parent, int32_t* job_a, int32_t* job_b,
                      int32_t* job_out, int32_t* job_next, int32_t* job_pending, int32_t* job_link,
                      int32_t* queue, int32_t* queue_flag, int32_t* queue_tail,
                      hipStream_t stream);
// Reorders the ready jobs queue[0..nready) (leaf-leaf merges, as make_jobs
// queued them) by estimated path to their tree's root, longest first.  prio:
// nslots ints, cnt: kPrioBins ints of scratch.
constexpr int kPrioBins = 4096;
void launch_job_priorities(const int32_t* merges, const int32_t* group_off, int ngroups,
                           int max_group, int nslots, const int32_t* node_W, int32_t* prio,
                           int32_t* cnt, int32_t* queue, DevStatus* st, hipStream_t stream);
void launch_colmap(const int64_t* offsets, const int32_t* ids, int nleaves,
                   const int32_t* node_parent, const int64_t* node_up, const int32_t* up_pool,
                   int32_t* colmap, DevStatus* st, hipStream_t stream);
void launch_widths(const int32_t* group_off, int ngroups, int32_t internal_base,
                   const int32_t* node_W, int32_t* width, hipStream_t stream);
void launch_job_results(const int32_t* job_a, const int64_t* job_score, const int64_t* job_cells,
                        int nslots, int64_t* score_out, int64_t* cells_out, int64_t* cells_total,
                        hipStream_t stream);

// refine.hip
void launch_rebuild_profiles(const uint8_t* codes, const int64_t* offsets, const int32_t* members,
                             const int32_t* bucket_off, int p, int n, const int32_t* colmap,
                             const int32_t* uidx, const int64_t* wo, const int32_t* width, int A,
                             uint32_t* cnt32, int64_t cnt_len, uint16_t* out16, DevStatus* st,
                             hipStream_t stream);
void launch_consensus(const int32_t* list, int nlist, const int32_t* node_W, const int32_t* node_n,
                      const int64_t* node_prof, const uint16_t* pool, int A, uint8_t* out,
                      const int64_t* out_off, int32_t* out_len, hipStream_t stream);
void launch_compact(const uint8_t* stage, const int64_t* st_off, const int32_t* len, int q,
                    int64_t* off, uint8_t* out, hipStream_t stream);
void launch_glue(const uint8_t* ops, const int64_t* ops_off, const int32_t* nops, int q, int GL,
                 int32_t* ins, int32_t* used, int32_t* slot_total, int32_t* slot_start,
                 int32_t* shared_at, int32_t* width, const int64_t* wo, int32_t* to_g,
                 const int64_t* offsets, const int32_t* members, const int32_t* bucket_off, int p,
                 int n, const int32_t* uidx, const int32_t* colmap_b, int32_t* colmap_g,
                 hipStream_t stream);
void launch_refine_jobs(int q, const int64_t* ops_off, int32_t* job_a, int32_t* job_b,
                        int32_t* job_out, int32_t* job_next, int32_t* job_pending,
                        int64_t* job_ops_off, int32_t* queue, int32_t* queue_flag,
                        int32_t* queue_tail, int32_t* node_parent, hipStream_t stream);
void launch_refine_nodes(int q, const int64_t* wo, const int32_t* width_u, const int32_t* rows_u,
                         int64_t ga_prof, int64_t ga_up, const int32_t* ga_len, int ga_n, int A,
                         int64_t up_base, int32_t* node_W, int32_t* node_n, int64_t* node_prof,
                         int64_t* node_up, hipStream_t stream);
void launch_copy_node_profile(const int32_t* node_W, const int64_t* node_prof,
                              const uint16_t* pool, int root, int A, uint16_t* dst, int64_t cap,
                              int32_t* w_out, DevStatus* st, hipStream_t stream);
void launch_seq_leaf(const int32_t* bucket_off, int p, const int32_t* members,
                     const int32_t* uidx, int n, int32_t* seq_u, hipStream_t stream);
void launch_split_step(const uint8_t* codes, const int64_t* offsets, int n, const int32_t* colmap,
                       const int32_t* seq_u, const int8_t* in1, int W, int A, uint32_t* cnt,
                       int32_t* idx1, int32_t* idx2, uint8_t* ops, int32_t* wid, uint16_t* prof,
                       int64_t off1, int64_t off2, const int32_t* S, int64_t o, int64_t e,
                       unsigned long long* s_old, DevStatus* st, hipStream_t stream);
void launch_split_result(const unsigned long long* s_old, const int64_t* job_score,
                         const int32_t* node_W, int out_node, int64_t* out, hipStream_t stream);
void launch_split_apply(const uint8_t* ops, const int32_t* nops, int32_t* map1, int32_t* map2,
                        const int64_t* offsets, int n, const int32_t* seq_u, const int8_t* in1,
                        const int32_t* idx1, const int32_t* idx2, const int32_t* colmap_in,
                        int32_t* colmap_out, hipStream_t stream);
void launch_onehot_seq(const uint8_t* codes, const int32_t* len, int maxlen, int A,
                       uint16_t* prof, hipStream_t stream);

}  // namespace sad
