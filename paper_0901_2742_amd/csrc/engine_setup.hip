// Setup and result kernels of the alignment engine: leaf nodes from
// sequences, jobs from UPGMA merge lists, column maps of every residue in its
// tree's root, per-group widths and per-job results.
#include "sad_internal.h"

namespace sad {

// ------------------------------------------------------------------ setup kernels

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_i32_kernel<<<(int)blocks, 256, 0, stream>>>(p, v, n);
}

// Leaf r: sequence ids[r]; its profile and column map live at the sequence's
// residue offset (offsets[id] * A in the profile pool, offsets[id] in the map
// pool), so the first total_len * A / total_len entries of the pools hold the
// leaves.
__global__ void make_leaves_kernel(const int64_t* __restrict__ offsets,
                                   const int32_t* __restrict__ ids, int nleaves, int A,
                                   int32_t node_base, int32_t* node_W, int32_t* node_n,
                                   int64_t* node_prof, int64_t* node_up, int32_t* node_parent) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nleaves) return;
  const int id = ids ? ids[r] : r;
  const int64_t o = offsets[id];
  node_W[node_base + r] = (int32_t)(offsets[id + 1] - o);
  node_n[node_base + r] = 1;
  node_prof[node_base + r] = o * A;
  node_up[node_base + r] = o;
  node_parent[node_base + r] = -1;
}

__global__ void onehot_kernel(const uint8_t* __restrict__ codes, int64_t total, int A,
                              uint16_t* __restrict__ prof) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int c = codes[t];
    for (int b = 0; b < A; ++b) prof[t * A + b] = (uint16_t)(b == c);
  }
}

void launch_make_leaves(const uint8_t* codes, const int64_t* offsets, const int32_t* ids,
                        int nleaves, int A, int32_t node_base, int32_t* node_W, int32_t* node_n,
                        int64_t* node_prof, int64_t* node_up, int32_t* node_parent,
                        uint16_t* prof_pool, int64_t total_len, hipStream_t stream) {
  if (nleaves <= 0) return;
  make_leaves_kernel<<<(nleaves + 255) / 256, 256, 0, stream>>>(
      offsets, ids, nleaves, A, node_base, node_W, node_n, node_prof, node_up, node_parent);
  int64_t blocks = (total_len + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  onehot_kernel<<<(int)blocks, 256, 0, stream>>>(codes, total_len, A, prof_pool);
}

// Jobs of UPGMA trees.  Group g has members group_off[g]..group_off[g+1]; its
// leaves are nodes group_off[g] + x and its cluster n_g + t is node
// internal_base + group_off[g] + t, made by the job in slot group_off[g] + t.
__global__ void make_jobs_kernel(const int32_t* __restrict__ merges,
                                 const int32_t* __restrict__ group_off, int ngroups, int nslots,
                                 int32_t internal_base, int32_t* node_parent, int32_t* job_a,
                                 int32_t* job_b, int32_t* job_out, int32_t* job_next,
                                 int32_t* job_pending, int32_t* job_link, int32_t* queue,
                                 int32_t* queue_flag, int32_t* queue_tail) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  int lo = 0, hi = ngroups;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (group_off[mid] <= s) lo = mid;
    else hi = mid;
  }
  const int g0 = group_off[lo], ng = group_off[lo + 1] - g0;
  const int t = s - g0;
  if (t >= ng - 1) {
    job_a[s] = -1;
    return;
  }
  const int la = merges[2 * s], lb = merges[2 * s + 1];
  const int a = la < ng ? g0 + la : internal_base + g0 + (la - ng);
  const int b = lb < ng ? g0 + lb : internal_base + g0 + (lb - ng);
  job_a[s] = a;
  job_b[s] = b;
  job_out[s] = internal_base + s;
  node_parent[a] = internal_base + s;
  node_parent[b] = internal_base + s;
  int pending = 0;
  // parents exist before any job runs: every child's hand-off word says so
  if (la >= ng) {
    job_next[g0 + (la - ng)] = s;
    job_link[g0 + (la - ng)] = 2;
    ++pending;
  }
  if (lb >= ng) {
    job_next[g0 + (lb - ng)] = s;
    job_link[g0 + (lb - ng)] = 2;
    ++pending;
  }
  job_pending[s] = pending;
  if (pending == 0) {
    const int pos = atomicAdd(queue_tail, 1);
    queue[pos] = s;
    queue_flag[pos] = 1;
  }
}

void launch_make_jobs(const int32_t* merges, const int32_t* group_off, int ngroups, int nslots,
                      int32_t internal_base, int32_t* node_parent, int32_t* job_a, int32_t* job_b,
                      int32_t* job_out, int32_t* job_next, int32_t* job_pending, int32_t* job_link,
                      int32_t* queue, int32_t* queue_flag, int32_t* queue_tail,
                      hipStream_t stream) {
  if (nslots <= 0) return;
  make_jobs_kernel<<<(nslots + 255) / 256, 256, 0, stream>>>(
      merges, group_off, ngroups, nslots, internal_base, node_parent, job_a, job_b, job_out,
      job_next, job_pending, job_link, queue, queue_flag, queue_tail);
}

// Column of every residue in its tree's root: leaf node of member position r
// is r; follow column maps up to the root.
__global__ void colmap_kernel(const int64_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                              int nleaves, const int32_t* __restrict__ node_parent,
                              const int64_t* __restrict__ node_up,
                              const int32_t* __restrict__ up_pool, int32_t* __restrict__ colmap,
                              DevStatus* st) {
  const int r = blockIdx.x;
  const int id = ids ? ids[r] : r;
  const int64_t o = offsets[id];
  const int L = (int)(offsets[id + 1] - o);
  for (int x = threadIdx.x; x < L; x += blockDim.x) {
    int c = x, node = r, depth = 0;
    // a tree over n leaves has depth < n; the bound guards a malformed one
    while (node_parent[node] >= 0 && depth < nleaves) {
      c = up_pool[node_up[node] + c];
      node = node_parent[node];
      ++depth;
    }
    if (depth >= nleaves) raise_error(st, SAD_E_DEVICE, r, W_ENGINE);
    colmap[o + x] = c;
  }
}

void launch_colmap(const int64_t* offsets, const int32_t* ids, int nleaves,
                   const int32_t* node_parent, const int64_t* node_up, const int32_t* up_pool,
                   int32_t* colmap, DevStatus* st, hipStream_t stream) {
  if (nleaves <= 0) return;
  colmap_kernel<<<nleaves, 128, 0, stream>>>(offsets, ids, nleaves, node_parent, node_up, up_pool,
                                             colmap, st);
}

// width of group g's root node
__global__ void widths_kernel(const int32_t* __restrict__ group_off, int ngroups,
                              int32_t internal_base, const int32_t* __restrict__ node_W,
                              int32_t* __restrict__ width) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int g0 = group_off[g], ng = group_off[g + 1] - g0;
  if (ng == 0) width[g] = 0;
  else if (ng == 1) width[g] = node_W[g0];
  else width[g] = node_W[internal_base + g0 + ng - 2];
}

void launch_widths(const int32_t* group_off, int ngroups, int32_t internal_base,
                   const int32_t* node_W, int32_t* width, hipStream_t stream) {
  if (ngroups <= 0) return;
  widths_kernel<<<(ngroups + 255) / 256, 256, 0, stream>>>(group_off, ngroups, internal_base,
                                                           node_W, width);
}

// per-slot results copied to the caller's arrays (slots without a job untouched)
__global__ void job_results_kernel(const int32_t* __restrict__ job_a,
                                   const int64_t* __restrict__ job_score,
                                   const int64_t* __restrict__ job_cells, int nslots,
                                   int64_t* score_out, int64_t* cells_out,
                                   unsigned long long* cells_total) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots || job_a[s] < 0) return;
  score_out[s] = job_score[s];
  cells_out[s] = job_cells[s];
  atomicAdd(cells_total, (unsigned long long)job_cells[s]);
}

void launch_job_results(const int32_t* job_a, const int64_t* job_score, const int64_t* job_cells,
                        int nslots, int64_t* score_out, int64_t* cells_out, int64_t* cells_total,
                        hipStream_t stream) {
  if (nslots <= 0) return;
  job_results_kernel<<<(nslots + 255) / 256, 256, 0, stream>>>(
      job_a, job_score, job_cells, nslots, score_out, cells_out,
      reinterpret_cast<unsigned long long*>(cells_total));
}

// ---------------------------------------------------------------- job priorities
// Order of the initially ready jobs (leaf-leaf merges) of the persistent
// launch: the longest estimated remaining path to the tree root first, so
// that the chains that bound the launch start before short ones.  A job's
// estimate is W1 W2 DP cells plus per-column and per-job terms, with a node's
// width estimated as its wider child's (leaves: sequence lengths); its path
// adds the estimates of its ancestors.  The order only schedules the work:
// results never depend on it.  Ready jobs are placed by a counting sort on
// the path's log2 in steps of 1/128 (kPrioBins bins; ties in any order).

// One workgroup per group: the group's leaf widths and its merges (a chunk at
// a time) are staged in LDS, where the first thread walks the merges in order
// (each internal node's width, parent and path estimate, kept as float: the
// bins need far less precision); then prio[s] = the bin of ready job s
// (highest path first), -1 for the group's other jobs.
constexpr int kPrioChunk = 1024;
__global__ __launch_bounds__(256) void prio_paths_kernel(const int32_t* __restrict__ merges,
                                                         const int32_t* __restrict__ group_off,
                                                         const int32_t* __restrict__ node_W,
                                                         int32_t* __restrict__ prio,
                                                         DevStatus* st) {
  extern __shared__ int32_t prio_sh[];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int g0 = group_off[g], n = group_off[g + 1] - g0;
  if (n <= 1) return;
  const int m = n - 1;
  float* path = reinterpret_cast<float*>(prio_sh);
  int32_t* width = prio_sh + m;
  int32_t* parent = width + m;
  int32_t* leafw = parent + m;
  int32_t* mch = leafw + n;  // 2 kPrioChunk
  for (int x = tid; x < n; x += blockDim.x) leafw[x] = node_W[g0 + x];
  for (int t = tid; t < m; t += blockDim.x) parent[t] = -1;
  for (int c0 = 0; c0 < m; c0 += kPrioChunk) {
    const int cn = min(kPrioChunk, m - c0);
    __syncthreads();
    for (int q = tid; q < 2 * cn; q += blockDim.x) mch[q] = merges[2 * (int64_t)(g0 + c0) + q];
    __syncthreads();
    if (tid == 0) {
      for (int t = c0; t < c0 + cn; ++t) {
        int w[2];
        for (int q = 0; q < 2; ++q) {
          int x = mch[2 * (t - c0) + q];
          if (x < 0 || x >= n + t) {  // not a leaf or an earlier cluster
            raise_error(st, SAD_E_INVAL, g0 + t, W_ENGINE);
            x = 0;
          }
          if (x < n) {
            w[q] = leafw[x];
          } else {
            w[q] = width[x - n];
            parent[x - n] = t;
          }
        }
        width[t] = max(w[0], w[1]);
        path[t] = (float)((int64_t)w[0] * w[1] + 64 * (int64_t)(w[0] + w[1]) + 16384);
      }
    }
  }
  __syncthreads();
  // parents come after their children in merge order
  if (tid == 0)
    for (int t = m - 1; t >= 0; --t)
      if (parent[t] >= 0) path[t] += path[parent[t]];
  __syncthreads();
  for (int t = tid; t < m; t += blockDim.x) {
    const int la = merges[2 * (int64_t)(g0 + t)], lb = merges[2 * (int64_t)(g0 + t) + 1];
    int bin = -1;
    if (la >= 0 && la < n && lb >= 0 && lb < n) {
      // path >= 2^14; bins of 1/128 octave above it, highest path in bin 0
      const int b = (int)((__log2f(path[t]) - 14.0f) * 128.0f);
      bin = kPrioBins - 1 - min(max(b, 0), kPrioBins - 1);
    }
    prio[g0 + t] = bin;
  }
}

__global__ void prio_count_kernel(const int32_t* __restrict__ prio, int nslots,
                                  int32_t* __restrict__ cnt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslots && prio[s] >= 0 && prio[s] < kPrioBins) atomicAdd(&cnt[prio[s]], 1);
}

// cnt[b] <- first queue position of bin b (exclusive scan, one workgroup of
// 1024 threads, four bins each).
__global__ __launch_bounds__(1024) void prio_scan_kernel(int32_t* __restrict__ cnt) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  int v[4], sum = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = cnt[4 * t + q];
    sum += v[q];
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int add = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int q = 0; q < 4; ++q) {
    cnt[4 * t + q] = run;
    run += v[q];
  }
}

__global__ void prio_scatter_kernel(const int32_t* __restrict__ prio, int nslots,
                                    int32_t* __restrict__ cnt, int32_t* __restrict__ queue) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslots && prio[s] >= 0 && prio[s] < kPrioBins) queue[atomicAdd(&cnt[prio[s]], 1)] = s;
}

void launch_job_priorities(const int32_t* merges, const int32_t* group_off, int ngroups,
                           int max_group, int nslots, const int32_t* node_W, int32_t* prio,
                           int32_t* cnt, int32_t* queue, DevStatus* st, hipStream_t stream) {
  if (ngroups <= 0 || nslots <= 0 || max_group <= 1) return;
  static_assert(kPrioBins == 4 * 1024, "the scan takes four bins per thread");
  // path, width, parent of the internal nodes, the leaf widths, a merge chunk
  const size_t lds = ((size_t)3 * (max_group - 1) + max_group + 2 * kPrioChunk) * sizeof(int32_t);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)prio_paths_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  launch_fill_i32(cnt, 0, kPrioBins, stream);
  launch_fill_i32(prio, -1, nslots, stream);
  prio_paths_kernel<<<ngroups, 256, lds, stream>>>(merges, group_off, node_W, prio, st);
  const int blocks = (nslots + 255) / 256;
  prio_count_kernel<<<blocks, 256, 0, stream>>>(prio, nslots, cnt);
  prio_scan_kernel<<<1, 1024, 0, stream>>>(cnt);
  prio_scatter_kernel<<<blocks, 256, 0, stream>>>(prio, nslots, cnt, queue);
}

}  // namespace sad
