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

}  // namespace sad
