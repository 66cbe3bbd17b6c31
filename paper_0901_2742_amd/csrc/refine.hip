// Ancestors, global ancestor and ancestor-constrained refinement + glue
// (paper Section 2.3.3, steps 12-15 of the algorithm box).
//  - profiles of the bucket alignments are rebuilt from the column maps;
//  - local ancestor = majority consensus (column kept iff 2 residues >= rows,
//    most frequent residue, smallest code on ties);
//  - after each bucket alignment is aligned against GA (a one-row profile),
//    the glue lays out, for every GA position j, an insert slot (the bucket
//    columns aligned to gaps before j, bucket by bucket) and then the shared
//    column j, dropping shared columns no bucket matched.
#include "sad_internal.h"

namespace sad {

__device__ inline int find_group(const int32_t* off, int ngroups, int r) {
  int lo = 0, hi = ngroups;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= r) lo = mid;
    else hi = mid;
  }
  return lo;
}

// cnt32[(wo[u] + col) * A + code] += 1 for every residue of bucket b (u = uidx[b])
__global__ void rebuild_counts_kernel(const uint8_t* __restrict__ codes,
                                      const int64_t* __restrict__ offsets,
                                      const int32_t* __restrict__ members,
                                      const int32_t* __restrict__ bucket_off, int p,
                                      const int32_t* __restrict__ colmap,
                                      const int32_t* __restrict__ uidx,
                                      const int64_t* __restrict__ wo,
                                      const int32_t* __restrict__ width, int A,
                                      uint32_t* __restrict__ cnt32, DevStatus* st) {
  const int r = blockIdx.x;
  const int b = find_group(bucket_off, p, r);
  const int u = uidx[b];
  const int W = width[b];
  const int id = members[r];
  const int64_t o = offsets[id];
  const int L = (int)(offsets[id + 1] - o);
  for (int x = threadIdx.x; x < L; x += blockDim.x) {
    const int c = colmap[o + x];
    if (c < 0 || c >= W) {
      raise_error(st, SAD_E_INVAL, o + x, W_REFINE);
      continue;
    }
    atomicAdd(&cnt32[(wo[u] + c) * A + codes[o + x]], 1u);
  }
}

__global__ void narrow_counts_kernel(const uint32_t* __restrict__ in, int64_t n,
                                     uint16_t* __restrict__ out) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
    out[t] = (uint16_t)in[t];
}

void launch_rebuild_profiles(const uint8_t* codes, const int64_t* offsets, const int32_t* members,
                             const int32_t* bucket_off, int p, int n, const int32_t* colmap,
                             const int32_t* uidx, const int64_t* wo, const int32_t* width, int A,
                             uint32_t* cnt32, int64_t cnt_len, uint16_t* out16, DevStatus* st,
                             hipStream_t stream) {
  if (n > 0)
    rebuild_counts_kernel<<<n, 128, 0, stream>>>(codes, offsets, members, bucket_off, p, colmap,
                                                 uidx, wo, width, A, cnt32, st);
  int64_t blocks = (cnt_len + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  narrow_counts_kernel<<<(int)blocks, 256, 0, stream>>>(cnt32, cnt_len, out16);
}

// Consensus of node list[u]: codes to out + out_off[u]; length to out_len[u].
constexpr int kConsThreads = 256;
__global__ __launch_bounds__(kConsThreads) void consensus_kernel(
    const int32_t* __restrict__ list, const int32_t* __restrict__ node_W,
    const int32_t* __restrict__ node_n, const int64_t* __restrict__ node_prof,
    const uint16_t* __restrict__ pool, int A, uint8_t* __restrict__ out,
    const int64_t* __restrict__ out_off, int32_t* __restrict__ out_len) {
  __shared__ int32_t seg[kConsThreads + 1];
  const int u = blockIdx.x;
  const int node = list[u];
  const int W = node_W[node], n = node_n[node];
  const uint16_t* P = pool + node_prof[node];
  const int per = (W + kConsThreads - 1) / kConsThreads;
  const int s0 = min(W, (int)threadIdx.x * per), s1 = min(W, s0 + per);
  int kept = 0;
  for (int c = s0; c < s1; ++c) {
    int tot = 0;
    for (int b = 0; b < A; ++b) tot += P[(int64_t)c * A + b];
    kept += (2 * tot >= n);
  }
  seg[threadIdx.x] = kept;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < kConsThreads; ++w) {
      int v = seg[w];
      seg[w] = acc;
      acc += v;
    }
    out_len[u] = acc;
  }
  __syncthreads();
  int k = seg[threadIdx.x];
  uint8_t* dst = out + out_off[u];
  for (int c = s0; c < s1; ++c) {
    int tot = 0, best = 0, bv = -1;
    for (int b = 0; b < A; ++b) {
      const int v = P[(int64_t)c * A + b];
      tot += v;
      if (v > bv) {
        bv = v;
        best = b;
      }
    }
    if (2 * tot >= n) dst[k++] = (uint8_t)best;
  }
}

void launch_consensus(const int32_t* list, int nlist, const int32_t* node_W, const int32_t* node_n,
                      const int64_t* node_prof, const uint16_t* pool, int A, uint8_t* out,
                      const int64_t* out_off, int32_t* out_len, hipStream_t stream) {
  if (nlist <= 0) return;
  consensus_kernel<<<nlist, kConsThreads, 0, stream>>>(list, node_W, node_n, node_prof, pool, A,
                                                       out, out_off, out_len);
}

// exclusive scan of q lengths into off[q + 1] (single thread; q <= a few thousand)
__global__ void scan_lengths_kernel(const int32_t* __restrict__ len, int q,
                                    int64_t* __restrict__ off) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t acc = 0;
  for (int u = 0; u < q; ++u) {
    off[u] = acc;
    acc += len[u];
  }
  off[q] = acc;
}

__global__ void compact_kernel(const uint8_t* __restrict__ stage, const int64_t* __restrict__ st_off,
                               const int32_t* __restrict__ len, const int64_t* __restrict__ off,
                               uint8_t* __restrict__ out) {
  const int u = blockIdx.x;
  for (int x = threadIdx.x; x < len[u]; x += blockDim.x) out[off[u] + x] = stage[st_off[u] + x];
}

void launch_compact(const uint8_t* stage, const int64_t* st_off, const int32_t* len, int q,
                    int64_t* off, uint8_t* out, hipStream_t stream) {
  scan_lengths_kernel<<<1, 1, 0, stream>>>(len, q, off);
  if (q > 0) compact_kernel<<<q, 128, 0, stream>>>(stage, st_off, len, off, out);
}

// ------------------------------------------------------------------ glue

// Block-wide scans of one value per thread (NT threads, Hillis-Steele in LDS):
// the exclusive prefix sum (total in *total) and the exclusive prefix maximum
// (identity `lo`).
constexpr int kGlueThreads = 256;

template <int NT>
__device__ inline int block_excl_sum(int v, int* sh, int* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int d = 1; d < NT; d <<= 1) {
    const int x = tid >= d ? sh[tid - d] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[NT - 1];
  __syncthreads();
  return incl - v;
}

template <int NT>
__device__ inline int block_excl_max(int v, int lo, int* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int d = 1; d < NT; d <<= 1) {
    const int x = tid >= d ? sh[tid - d] : lo;
    __syncthreads();
    sh[tid] = max(sh[tid], x);
    __syncthreads();
  }
  const int r = tid > 0 ? sh[tid - 1] : lo;
  __syncthreads();
  return r;
}

// Bucket u's op string against the template (TL columns): op t lies in slot
// j(t) = the number of non-X ops before it; an X op is the kin(t)-th of the run
// of X ops in its slot, kin(t) = t - 1 - (the last non-X op before t).  One
// workgroup per bucket, the ops in chunks of kGlueThreads.  Count pass: the
// last X op of each run stores the run length as the slot's insert count;
// M ops flag their template column.
__global__ __launch_bounds__(kGlueThreads) void glue_count_kernel(
    const uint8_t* __restrict__ ops, const int64_t* __restrict__ ops_off,
    const int32_t* __restrict__ nops, int q, int GL, int32_t* __restrict__ ins,
    int32_t* __restrict__ used) {
  __shared__ int sh[kGlueThreads];
  const int u = blockIdx.x;
  const uint8_t* o = ops + ops_off[u];
  int32_t* row = ins + (int64_t)u * (GL + 1);
  const int m = nops[u];
  int cj = 0, clast = -1;
  for (int t0 = 0; t0 < m; t0 += kGlueThreads) {
    const int t = t0 + (int)threadIdx.x;
    const int op = t < m ? o[t] : 3;
    const int nonx = (t < m && op != 1) ? 1 : 0;
    int tot = 0;
    const int j = cj + block_excl_sum<kGlueThreads>(nonx, sh, &tot);
    const int lastc = block_excl_max<kGlueThreads>(nonx ? t : -1, -1, sh);
    const int last = max(clast, lastc);
    if (t < m) {
      if (op == 1) {
        const bool run_end = t + 1 == m || o[t + 1] != 1;
        if (run_end) row[j] = t - last;
      } else if (op == 0) {
        used[j] = 1;
      }
    }
    cj += tot;
    // the last non-X op of this chunk, for the next one
    if ((int)threadIdx.x == kGlueThreads - 1) sh[0] = max(lastc, nonx ? t : -1);
    __syncthreads();
    clast = max(clast, sh[0]);
    __syncthreads();
  }
}

// per slot j: exclusive prefix over buckets (in place) and slot total
__global__ void glue_slot_kernel(int32_t* __restrict__ ins, int q, int GL,
                                 int32_t* __restrict__ slot_total) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > GL) return;
  int acc = 0;
  for (int u = 0; u < q; ++u) {
    const int v = ins[(int64_t)u * (GL + 1) + j];
    ins[(int64_t)u * (GL + 1) + j] = acc;
    acc += v;
  }
  slot_total[j] = acc;
}

// Glued positions: slot j starts after every earlier slot and every earlier
// kept template column; template column j follows its slot (one workgroup).
__global__ __launch_bounds__(kGlueThreads) void glue_scan_kernel(
    const int32_t* __restrict__ slot_total, const int32_t* __restrict__ used, int GL,
    int32_t* __restrict__ slot_start, int32_t* __restrict__ shared_at,
    int32_t* __restrict__ width) {
  __shared__ int sh[kGlueThreads];
  int base = 0;
  for (int j0 = 0; j0 <= GL; j0 += kGlueThreads) {
    const int j = j0 + (int)threadIdx.x;
    const int st = j <= GL ? slot_total[j] : 0;
    const int us = j < GL ? (used[j] ? 1 : 0) : 0;
    int tot = 0;
    const int pre = base + block_excl_sum<kGlueThreads>(st + us, sh, &tot);
    if (j <= GL) {
      slot_start[j] = pre;
      if (j < GL) shared_at[j] = us ? pre + st : -1;
    }
    base += tot;
  }
  if (threadIdx.x == 0) width[0] = base;
}

// Map pass: bucket column i(t) (the number of M and X ops before t) goes to
// slot_start[j] + (earlier buckets' inserts in slot j) + kin(t) for an X op,
// to the template column's glued position for an M op.
__global__ __launch_bounds__(kGlueThreads) void glue_map_kernel(
    const uint8_t* __restrict__ ops, const int64_t* __restrict__ ops_off,
    const int32_t* __restrict__ nops, int q, int GL, const int32_t* __restrict__ ins,
    const int32_t* __restrict__ slot_start, const int32_t* __restrict__ shared_at,
    const int64_t* __restrict__ wo, int32_t* __restrict__ to_g) {
  __shared__ int sh[kGlueThreads];
  const int u = blockIdx.x;
  const uint8_t* o = ops + ops_off[u];
  const int32_t* row = ins + (int64_t)u * (GL + 1);
  int32_t* dst = to_g + wo[u];
  const int m = nops[u];
  int ci = 0, cj = 0, clast = -1;
  for (int t0 = 0; t0 < m; t0 += kGlueThreads) {
    const int t = t0 + (int)threadIdx.x;
    const int op = t < m ? o[t] : 3;
    const int nonx = (t < m && op != 1) ? 1 : 0;
    const int cons = (t < m && op != 2) ? 1 : 0;
    int tj = 0, ti = 0;
    const int j = cj + block_excl_sum<kGlueThreads>(nonx, sh, &tj);
    const int i = ci + block_excl_sum<kGlueThreads>(cons, sh, &ti);
    const int lastc = block_excl_max<kGlueThreads>(nonx ? t : -1, -1, sh);
    const int last = max(clast, lastc);
    if (t < m) {
      if (op == 1) dst[i] = slot_start[j] + row[j] + (t - last - 1);
      else if (op == 0) dst[i] = shared_at[j];
    }
    cj += tj;
    ci += ti;
    if ((int)threadIdx.x == kGlueThreads - 1) sh[0] = max(lastc, nonx ? t : -1);
    __syncthreads();
    clast = max(clast, sh[0]);
    __syncthreads();
  }
}

__global__ void glue_colmap_kernel(const int64_t* __restrict__ offsets,
                                   const int32_t* __restrict__ members,
                                   const int32_t* __restrict__ bucket_off, int p,
                                   const int32_t* __restrict__ uidx, const int64_t* __restrict__ wo,
                                   const int32_t* __restrict__ colmap_b,
                                   const int32_t* __restrict__ to_g, int32_t* __restrict__ colmap_g) {
  const int r = blockIdx.x;
  const int b = find_group(bucket_off, p, r);
  const int u = uidx[b];
  const int id = members[r];
  const int64_t o = offsets[id];
  const int L = (int)(offsets[id + 1] - o);
  for (int x = threadIdx.x; x < L; x += blockDim.x) colmap_g[o + x] = to_g[wo[u] + colmap_b[o + x]];
}

void launch_glue(const uint8_t* ops, const int64_t* ops_off, const int32_t* nops, int q, int GL,
                 int32_t* ins, int32_t* used, int32_t* slot_total, int32_t* slot_start,
                 int32_t* shared_at, int32_t* width, const int64_t* wo, int32_t* to_g,
                 const int64_t* offsets, const int32_t* members, const int32_t* bucket_off, int p,
                 int n, const int32_t* uidx, const int32_t* colmap_b, int32_t* colmap_g,
                 hipStream_t stream) {
  if (q <= 0) return;
  glue_count_kernel<<<q, kGlueThreads, 0, stream>>>(ops, ops_off, nops, q, GL, ins, used);
  glue_slot_kernel<<<(GL + 1 + 255) / 256, 256, 0, stream>>>(ins, q, GL, slot_total);
  glue_scan_kernel<<<1, kGlueThreads, 0, stream>>>(slot_total, used, GL, slot_start, shared_at,
                                                   width);
  glue_map_kernel<<<q, kGlueThreads, 0, stream>>>(ops, ops_off, nops, q, GL, ins, slot_start,
                                                   shared_at, wo, to_g);
  if (n > 0)
    glue_colmap_kernel<<<n, 128, 0, stream>>>(offsets, members, bucket_off, p, uidx, wo, colmap_b,
                                              to_g, colmap_g);
}

// refinement jobs: job u aligns node u (bucket) against node q (GA) into node
// q + 1 + u; every job is ready at once.
__global__ void refine_jobs_kernel(int q, const int64_t* __restrict__ ops_off, int32_t* job_a,
                                   int32_t* job_b, int32_t* job_out, int32_t* job_next,
                                   int32_t* job_pending, int64_t* job_ops_off, int32_t* queue,
                                   int32_t* queue_flag, int32_t* queue_tail, int32_t* node_parent) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= q) return;
  job_a[u] = u;
  job_b[u] = q;
  job_out[u] = q + 1 + u;
  job_next[u] = -1;
  job_pending[u] = 0;
  job_ops_off[u] = ops_off[u];
  node_parent[u] = q + 1 + u;
  queue[u] = u;
  queue_flag[u] = 1;
  if (u == 0) *queue_tail = q;
}

void launch_refine_jobs(int q, const int64_t* ops_off, int32_t* job_a, int32_t* job_b,
                        int32_t* job_out, int32_t* job_next, int32_t* job_pending,
                        int64_t* job_ops_off, int32_t* queue, int32_t* queue_flag,
                        int32_t* queue_tail, int32_t* node_parent, hipStream_t stream) {
  if (q <= 0) return;
  refine_jobs_kernel<<<(q + 63) / 64, 64, 0, stream>>>(q, ops_off, job_a, job_b, job_out, job_next,
                                                       job_pending, job_ops_off, queue, queue_flag,
                                                       queue_tail, node_parent);
}

// nodes 0..q-1 = bucket profiles at prof offsets wo[u] * A; node q = GA
__global__ void refine_nodes_kernel(int q, const int64_t* __restrict__ wo,
                                    const int32_t* __restrict__ width_u,
                                    const int32_t* __restrict__ rows_u, int64_t ga_prof,
                                    int64_t ga_up, const int32_t* __restrict__ ga_len, int ga_n,
                                    int A, int64_t up_base, int32_t* node_W, int32_t* node_n,
                                    int64_t* node_prof, int64_t* node_up) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u > q) return;
  if (u < q) {
    node_W[u] = width_u[u];
    node_n[u] = rows_u[u];
    node_prof[u] = wo[u] * A;
    node_up[u] = up_base + wo[u];
  } else {
    node_W[u] = *ga_len;
    node_n[u] = ga_n;
    node_prof[u] = ga_prof;
    node_up[u] = ga_up;
  }
}

void launch_refine_nodes(int q, const int64_t* wo, const int32_t* width_u, const int32_t* rows_u,
                         int64_t ga_prof, int64_t ga_up, const int32_t* ga_len, int ga_n, int A,
                         int64_t up_base, int32_t* node_W, int32_t* node_n, int64_t* node_prof,
                         int64_t* node_up, hipStream_t stream) {
  refine_nodes_kernel<<<(q + 1 + 63) / 64, 64, 0, stream>>>(q, wo, width_u, rows_u, ga_prof, ga_up,
                                                            ga_len, ga_n, A, up_base, node_W,
                                                            node_n, node_prof, node_up);
}

// The profile of node `root` (W x A counts) copied out of an engine's pool;
// *w_out = W.  A profile wider than the destination is reported.
__global__ void copy_node_profile_kernel(const int32_t* __restrict__ node_W,
                                         const int64_t* __restrict__ node_prof,
                                         const uint16_t* __restrict__ pool, int root, int A,
                                         uint16_t* __restrict__ dst, int64_t cap,
                                         int32_t* __restrict__ w_out, DevStatus* st) {
  const int W = node_W[root];
  const int64_t n = (int64_t)W * A;
  if (n > cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_error(st, SAD_E_CAPACITY, n, W_REFINE);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *w_out = W;
  const uint16_t* src = pool + node_prof[root];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

void launch_copy_node_profile(const int32_t* node_W, const int64_t* node_prof,
                              const uint16_t* pool, int root, int A, uint16_t* dst, int64_t cap,
                              int32_t* w_out, DevStatus* st, hipStream_t stream) {
  copy_node_profile_kernel<<<64, 256, 0, stream>>>(node_W, node_prof, pool, root, A, dst, cap,
                                                   w_out, st);
}

__global__ void onehot_seq_kernel(const uint8_t* __restrict__ codes, const int32_t* __restrict__ len,
                                  int A, uint16_t* __restrict__ prof) {
  const int L = *len;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x)
    for (int b = 0; b < A; ++b) prof[(int64_t)t * A + b] = (uint16_t)(b == codes[t]);
}

void launch_onehot_seq(const uint8_t* codes, const int32_t* len, int maxlen, int A,
                       uint16_t* prof, hipStream_t stream) {
  int blocks = (maxlen + 255) / 256;
  if (blocks < 1) blocks = 1;
  onehot_seq_kernel<<<blocks, 256, 0, stream>>>(codes, len, A, prof);
}

}  // namespace sad
