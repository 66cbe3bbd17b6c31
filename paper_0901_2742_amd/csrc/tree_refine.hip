// Tree-dependent refinement of the glued alignment: the device side of one
// step.  A step takes one edge of the ancestors' guide tree, which splits the
// sequences into group 1 (the buckets below the edge) and group 2 (the rest),
// and
//   1. counts, per column of the current alignment, the residues of each
//      group by code (split_counts_kernel);
//   2. keeps the columns that hold a residue of a group as that group's
//      profile, in order, and records the present alignment of the two
//      profiles as ops: M where a column holds both groups, X (group 1 only)
//      or Y (group 2 only) (split_scan_kernel, one workgroup);
//   3. writes the two profiles into the alignment engine's pool
//      (split_profiles_kernel) and scores the present alignment with the
//      engine's objective: column scores C1 S C2^T of M columns, minus
//      (go + (l - 1) ge) n1 n2 per maximal X or Y run (split_score_kernel);
//   4. after the engine has re-aligned the two profiles, and only if its
//      score is higher, lays every residue out by the new ops
//      (split_map_kernel, split_remap_kernel).
// The host (sad_refine_tree) orders the edges and decides acceptance.
#include "sad_internal.h"

namespace sad {

constexpr int kSplitThreads = 256;
constexpr int kSplitScanThreads = 1024;

// leaf of the ancestor tree of every sequence: the index u of its bucket
// among the non-empty buckets (uidx[b]), found by binary search on bucket_off
__global__ void seq_leaf_kernel(const int32_t* __restrict__ bucket_off, int p,
                                const int32_t* __restrict__ members,
                                const int32_t* __restrict__ uidx, int n,
                                int32_t* __restrict__ seq_u) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int lo = 0, hi = p;  // bucket_off[lo] <= t < bucket_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (bucket_off[mid] <= t) lo = mid;
    else hi = mid;
  }
  seq_u[members[t]] = uidx[lo];
}

// cnt[(g W + c) A + a] += residues of group g with code a in column c; one
// workgroup per sequence
__global__ __launch_bounds__(kSplitThreads) void split_counts_kernel(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ colmap, const int32_t* __restrict__ seq_u,
    const int8_t* __restrict__ in1, int W, int A, uint32_t* __restrict__ cnt) {
  const int s = blockIdx.x;
  const int g = in1[seq_u[s]] ? 0 : 1;
  uint32_t* base = cnt + (int64_t)g * W * A;
  for (int64_t r = offsets[s] + threadIdx.x; r < offsets[s + 1]; r += kSplitThreads)
    atomicAdd(&base[(int64_t)colmap[r] * A + codes[r]], 1u);
}

// Per column: which groups it holds; the exclusive scans give each group's
// profile column (idx = -1 where the group has none) and the widths
// wid[0] = W1, wid[1] = W2; ops[c] is the present alignment's op.  A column
// with neither group is reported (the alignment must have no all-gap column).
__global__ __launch_bounds__(kSplitScanThreads) void split_scan_kernel(
    const uint32_t* __restrict__ cnt, int W, int A, int32_t* __restrict__ idx1,
    int32_t* __restrict__ idx2, uint8_t* __restrict__ ops, int32_t* __restrict__ wid,
    DevStatus* st) {
  __shared__ int32_t s1[kSplitScanThreads], s2[kSplitScanThreads];
  __shared__ int32_t base1, base2;
  const int tid = threadIdx.x;
  if (tid == 0) {
    base1 = 0;
    base2 = 0;
  }
  __syncthreads();
  for (int c0 = 0; c0 < W; c0 += kSplitScanThreads) {
    const int c = c0 + tid;
    int h1 = 0, h2 = 0;
    if (c < W) {
      const uint32_t* a1 = cnt + (int64_t)c * A;
      const uint32_t* a2 = cnt + ((int64_t)W + c) * A;
      for (int a = 0; a < A; ++a) {
        h1 |= a1[a] != 0u;
        h2 |= a2[a] != 0u;
      }
      if (!h1 && !h2) raise_error(st, SAD_E_INVAL, c, W_REFINE);
    }
    s1[tid] = h1;
    s2[tid] = h2;
    __syncthreads();
    // inclusive scans (Hillis-Steele)
    for (int d = 1; d < kSplitScanThreads; d <<= 1) {
      const int v1 = tid >= d ? s1[tid - d] : 0, v2 = tid >= d ? s2[tid - d] : 0;
      __syncthreads();
      s1[tid] += v1;
      s2[tid] += v2;
      __syncthreads();
    }
    if (c < W) {
      idx1[c] = h1 ? base1 + s1[tid] - 1 : -1;
      idx2[c] = h2 ? base2 + s2[tid] - 1 : -1;
      ops[c] = (uint8_t)(h1 && h2 ? 0 : (h1 ? 1 : 2));
    }
    __syncthreads();
    if (tid == kSplitScanThreads - 1) {
      base1 += s1[tid];
      base2 += s2[tid];
    }
    __syncthreads();
  }
  if (tid == 0) {
    wid[0] = base1;
    wid[1] = base2;
  }
}

// group 1's profile at prof + off1, group 2's at prof + off2 (u16 counts)
__global__ void split_profiles_kernel(const uint32_t* __restrict__ cnt, int W, int A,
                                      const int32_t* __restrict__ idx1,
                                      const int32_t* __restrict__ idx2, uint16_t* __restrict__ prof,
                                      int64_t off1, int64_t off2) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)W * A) return;
  const int c = (int)(t / A), a = (int)(t % A);
  if (idx1[c] >= 0) prof[off1 + (int64_t)idx1[c] * A + a] = (uint16_t)cnt[t];
  if (idx2[c] >= 0) prof[off2 + (int64_t)idx2[c] * A + a] = (uint16_t)cnt[(int64_t)W * A + t];
}

// out[0] += score of the present alignment of the two profiles (columns of
// the current alignment in order: M columns add C1 S C2^T, a run of X or Y
// costs go n1 n2 at its first column and ge n1 n2 at each further one)
__global__ __launch_bounds__(kSplitThreads) void split_score_kernel(
    const uint32_t* __restrict__ cnt, int W, int A, const uint8_t* __restrict__ ops,
    const int32_t* __restrict__ S, int64_t o, int64_t e, unsigned long long* __restrict__ out) {
  __shared__ long long red[kSplitThreads / 64];
  long long part = 0;
  for (int c = blockIdx.x * kSplitThreads + threadIdx.x; c < W; c += gridDim.x * kSplitThreads) {
    const int op = ops[c];
    if (op == 0) {
      const uint32_t* a1 = cnt + (int64_t)c * A;
      const uint32_t* a2 = cnt + ((int64_t)W + c) * A;
      long long sc = 0;
      for (int a = 0; a < A; ++a) {
        if (!a1[a]) continue;
        long long row = 0;
        for (int b = 0; b < A; ++b) row += (long long)S[a * A + b] * (long long)a2[b];
        sc += (long long)a1[a] * row;
      }
      part += sc;
    } else {
      const bool ext = c > 0 && ops[c - 1] == op;
      part -= ext ? e : o;
    }
  }
  for (int m = 32; m > 0; m >>= 1) part += __shfl_xor(part, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < kSplitThreads / 64; ++w) s += red[w];
    atomicAdd(out, (unsigned long long)s);
  }
}

// map1[i] / map2[j]: the new column of group 1's i-th / group 2's j-th
// profile column under the op string ops[0..*nops) (one workgroup)
__global__ __launch_bounds__(kSplitScanThreads) void split_map_kernel(
    const uint8_t* __restrict__ ops, const int32_t* __restrict__ nops_p,
    int32_t* __restrict__ map1, int32_t* __restrict__ map2) {
  __shared__ int32_t s1[kSplitScanThreads], s2[kSplitScanThreads];
  __shared__ int32_t base1, base2;
  const int tid = threadIdx.x;
  const int nops = *nops_p;
  if (tid == 0) {
    base1 = 0;
    base2 = 0;
  }
  __syncthreads();
  for (int t0 = 0; t0 < nops; t0 += kSplitScanThreads) {
    const int t = t0 + tid;
    const int op = t < nops ? ops[t] : -1;
    const int c1 = op == 0 || op == 1, c2 = op == 0 || op == 2;
    s1[tid] = c1;
    s2[tid] = c2;
    __syncthreads();
    for (int d = 1; d < kSplitScanThreads; d <<= 1) {
      const int v1 = tid >= d ? s1[tid - d] : 0, v2 = tid >= d ? s2[tid - d] : 0;
      __syncthreads();
      s1[tid] += v1;
      s2[tid] += v2;
      __syncthreads();
    }
    if (c1) map1[base1 + s1[tid] - 1] = t;
    if (c2) map2[base2 + s2[tid] - 1] = t;
    __syncthreads();
    if (tid == kSplitScanThreads - 1) {
      base1 += s1[tid];
      base2 += s2[tid];
    }
    __syncthreads();
  }
}

// every residue moves to its group's new column; one workgroup per sequence
__global__ __launch_bounds__(kSplitThreads) void split_remap_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ seq_u,
    const int8_t* __restrict__ in1, const int32_t* __restrict__ idx1,
    const int32_t* __restrict__ idx2, const int32_t* __restrict__ map1,
    const int32_t* __restrict__ map2, const int32_t* __restrict__ colmap_in,
    int32_t* __restrict__ colmap_out) {
  const int s = blockIdx.x;
  const bool g1 = in1[seq_u[s]] != 0;
  for (int64_t r = offsets[s] + threadIdx.x; r < offsets[s + 1]; r += kSplitThreads) {
    const int c = colmap_in[r];
    colmap_out[r] = g1 ? map1[idx1[c]] : map2[idx2[c]];
  }
}

// out[0] = present score, out[1] = the engine's score, out[2] = new width
__global__ void split_result_kernel(const unsigned long long* __restrict__ s_old,
                                    const int64_t* __restrict__ job_score,
                                    const int32_t* __restrict__ node_W, int out_node,
                                    int64_t* __restrict__ out) {
  out[0] = (int64_t)*s_old;
  out[1] = job_score[0];
  out[2] = node_W[out_node];
}

void launch_seq_leaf(const int32_t* bucket_off, int p, const int32_t* members,
                     const int32_t* uidx, int n, int32_t* seq_u, hipStream_t stream) {
  if (n <= 0) return;
  seq_leaf_kernel<<<(n + 255) / 256, 256, 0, stream>>>(bucket_off, p, members, uidx, n, seq_u);
}

void launch_split_step(const uint8_t* codes, const int64_t* offsets, int n, const int32_t* colmap,
                       const int32_t* seq_u, const int8_t* in1, int W, int A, uint32_t* cnt,
                       int32_t* idx1, int32_t* idx2, uint8_t* ops, int32_t* wid, uint16_t* prof,
                       int64_t off1, int64_t off2, const int32_t* S, int64_t o, int64_t e,
                       unsigned long long* s_old, DevStatus* st, hipStream_t stream) {
  launch_fill_i32(reinterpret_cast<int32_t*>(cnt), 0, 2 * (int64_t)W * A, stream);
  launch_fill_i32(reinterpret_cast<int32_t*>(s_old), 0, 2, stream);
  split_counts_kernel<<<n, kSplitThreads, 0, stream>>>(codes, offsets, colmap, seq_u, in1, W, A,
                                                       cnt);
  split_scan_kernel<<<1, kSplitScanThreads, 0, stream>>>(cnt, W, A, idx1, idx2, ops, wid, st);
  const int64_t cells = (int64_t)W * A;
  split_profiles_kernel<<<(unsigned)((cells + 255) / 256), 256, 0, stream>>>(cnt, W, A, idx1, idx2,
                                                                          prof, off1, off2);
  const int blocks = std::max(1, std::min((W + kSplitThreads - 1) / kSplitThreads, 256));
  split_score_kernel<<<blocks, kSplitThreads, 0, stream>>>(cnt, W, A, ops, S, o, e, s_old);
}

void launch_split_result(const unsigned long long* s_old, const int64_t* job_score,
                         const int32_t* node_W, int out_node, int64_t* out, hipStream_t stream) {
  split_result_kernel<<<1, 1, 0, stream>>>(s_old, job_score, node_W, out_node, out);
}

void launch_split_apply(const uint8_t* ops, const int32_t* nops, int32_t* map1, int32_t* map2,
                        const int64_t* offsets, int n, const int32_t* seq_u, const int8_t* in1,
                        const int32_t* idx1, const int32_t* idx2, const int32_t* colmap_in,
                        int32_t* colmap_out, hipStream_t stream) {
  split_map_kernel<<<1, kSplitScanThreads, 0, stream>>>(ops, nops, map1, map2);
  split_remap_kernel<<<n, kSplitThreads, 0, stream>>>(offsets, seq_u, in1, idx1, idx2, map1, map2,
                                                      colmap_in, colmap_out);
}

}  // namespace sad
