// Regular-sampling partition (paper Section 2.3.2): per-chunk picks of p-1
// composite keys (K_i, i), a stable merge of the p sorted runs into Y, the
// pivots Y_{p/2 + (t-1)p}, bucket ids by binary search over the pivots, and a
// stable scatter of ids into buckets.
#include <algorithm>

#include "sad_internal.h"

namespace sad {

__device__ inline bool ck_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Y[c (p-1) + t - 1] = key of sorted chunk c at floor(t w / p)
__global__ void y_pick_kernel(const uint64_t* __restrict__ key, const int32_t* __restrict__ sorted,
                              int n, int p, uint64_t* __restrict__ Yk, int32_t* __restrict__ Yi) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= p * (p - 1)) return;
  int c = q / (p - 1), t = q % (p - 1) + 1;
  int lo = (int)(((int64_t)c * n) / p), hi = (int)(((int64_t)(c + 1) * n) / p);
  int id = sorted[lo + (int)(((int64_t)t * (hi - lo)) / p)];
  Yk[q] = key[id];
  Yi[q] = id;
}

// number of entries of run [r0, r0 + len) strictly below (k, i)
__device__ inline int run_lower(const uint64_t* Yk, const int32_t* Yi, int r0, int len, uint64_t k,
                                int32_t i) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ck_less(Yk[r0 + mid], Yi[r0 + mid], k, i)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One round of the pairwise merge of Y's sorted runs of `len` entries (the
// last may be shorter): runs 2m and 2m + 1 merge into one.  Entry x of run j
// lands at the start of its pair plus its index in its run plus the number of
// entries of the partner run below it (an entry without a partner run keeps
// its place).  The composite keys (K_i, i) are distinct, so after the last
// round the entries are in (K, i) order, whatever the merge order.
__global__ void y_merge_round_kernel(const uint64_t* __restrict__ Ik,
                                     const int32_t* __restrict__ Ii, int ny, int len,
                                     uint64_t* __restrict__ Ok, int32_t* __restrict__ Oi) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ny) return;
  const int j = x / len;
  const int start = j * len;
  const int ps = (j ^ 1) * len;  // partner run
  const uint64_t k = Ik[x];
  const int32_t i = Ii[x];
  int below = 0;
  if (ps < ny) below = run_lower(Ik, Ii, ps, min(len, ny - ps), k, i);
  const int to = (j & ~1) * len + (x - start) + below;
  Ok[to] = k;
  Oi[to] = i;
}

__global__ void pivot_kernel(const uint64_t* __restrict__ Sk, const int32_t* __restrict__ Si, int p,
                             uint64_t* __restrict__ pk, int32_t* __restrict__ pi) {
  int t = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (t > p - 1) return;
  int idx = p / 2 + (t - 1) * p - 1;
  pk[t - 1] = Sk[idx];
  pi[t - 1] = Si[idx];
}

constexpr int kScatterBlock = 256;

// bucket(i) = #pivots strictly below (K_i, i); per-block bucket counts.
__global__ __launch_bounds__(kScatterBlock) void bucket_kernel(
    const uint64_t* __restrict__ key, int n, int p, const uint64_t* __restrict__ pk,
    const int32_t* __restrict__ pi, int32_t* __restrict__ bucket, int32_t* __restrict__ blk_cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = key[i];
  int lo = 0, hi = p - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ck_less(pk[mid], pi[mid], k, i)) lo = mid + 1;
    else hi = mid;
  }
  bucket[i] = lo;
  atomicAdd(&blk_cnt[(int64_t)blockIdx.x * p + lo], 1);
}

// per bucket: exclusive prefix over blocks (in place) and total
__global__ void bucket_scan_blocks_kernel(int32_t* __restrict__ blk_cnt, int nblk, int p,
                                          int32_t* __restrict__ total) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p) return;
  int acc = 0;
  for (int q = 0; q < nblk; ++q) {
    int v = blk_cnt[(int64_t)q * p + b];
    blk_cnt[(int64_t)q * p + b] = acc;
    acc += v;
  }
  total[b] = acc;
}

__global__ void bucket_offsets_kernel(const int32_t* __restrict__ total, int p,
                                      int32_t* __restrict__ off) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int acc = 0;
  for (int b = 0; b < p; ++b) {
    off[b] = acc;
    acc += total[b];
  }
  off[p] = acc;
}

__global__ __launch_bounds__(kScatterBlock) void bucket_scatter_kernel(
    const int32_t* __restrict__ bucket, int n, int p, const int32_t* __restrict__ blk_cnt,
    const int32_t* __restrict__ off, int32_t* __restrict__ members) {
  __shared__ int32_t bk[kScatterBlock];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int b = i < n ? bucket[i] : -1;
  bk[threadIdx.x] = b;
  __syncthreads();
  if (i >= n) return;
  int before = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) before += (bk[t] == b);
  members[off[b] + blk_cnt[(int64_t)blockIdx.x * p + b] + before] = i;
}

void launch_partition(const uint64_t* key, int n, int p, const int32_t* sorted, uint64_t* Ykey,
                      int32_t* Yid, uint64_t* Ysorted_key, int32_t* Ysorted_id,
                      uint64_t* pivot_key, int32_t* pivot_id, int32_t* bucket, int32_t* blk_cnt,
                      int32_t* total, int32_t* bucket_off, int32_t* members, hipStream_t stream) {
  const int ny = p * (p - 1);
  if (ny > 0) {
    y_pick_kernel<<<(ny + 255) / 256, 256, 0, stream>>>(key, sorted, n, p, Ykey, Yid);
    // the p runs (each chunk's picks, in its order) merged pairwise, ping-pong
    // between the two buffers
    uint64_t *ik = Ykey, *ok = Ysorted_key;
    int32_t *ii = Yid, *oi = Ysorted_id;
    for (int len = p - 1; len < ny; len *= 2) {
      y_merge_round_kernel<<<(ny + 255) / 256, 256, 0, stream>>>(ik, ii, ny, len, ok, oi);
      std::swap(ik, ok);
      std::swap(ii, oi);
    }
    pivot_kernel<<<(p - 1 + 255) / 256, 256, 0, stream>>>(ik, ii, p, pivot_key, pivot_id);
  }
  const int nblk = (n + kScatterBlock - 1) / kScatterBlock;
  // cleared by a kernel (no memset node when a caller captures the launches)
  launch_fill_i32(blk_cnt, 0, (int64_t)nblk * p, stream);
  bucket_kernel<<<nblk, kScatterBlock, 0, stream>>>(key, n, p, pivot_key, pivot_id, bucket,
                                                    blk_cnt);
  bucket_scan_blocks_kernel<<<(p + 255) / 256, 256, 0, stream>>>(blk_cnt, nblk, p, total);
  bucket_offsets_kernel<<<1, 1, 0, stream>>>(total, p, bucket_off);
  bucket_scatter_kernel<<<nblk, kScatterBlock, 0, stream>>>(bucket, n, p, blk_cnt, bucket_off,
                                                            members);
}

// Scratch of the partition of n ids into p buckets: the chunk order, the
// p(p-1) regular samples and their sorted copy, per-block bucket counts and
// bucket totals, each 256-byte aligned.  Returns the bytes; carves them from
// base when it is not null.
size_t partition_scratch(int n, int p, char* base, PartitionScratch* ps) {
  const size_t ny = (size_t)p * (size_t)(p - 1);
  const size_t nblk = ((size_t)n + kScatterBlock - 1) / kScatterBlock;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += (std::max(bytes, (size_t)1) + 255) & ~(size_t)255;
    return q;
  };
  char* sorted = take(sizeof(int32_t) * (size_t)n);
  char* yk = take(sizeof(uint64_t) * ny);
  char* yi = take(sizeof(int32_t) * ny);
  char* ysk = take(sizeof(uint64_t) * ny);
  char* ysi = take(sizeof(int32_t) * ny);
  char* blk = take(sizeof(int32_t) * nblk * (size_t)p);
  char* total = take(sizeof(int32_t) * (size_t)p);
  if (base && ps) {
    ps->sorted = reinterpret_cast<int32_t*>(sorted);
    ps->Yk = reinterpret_cast<uint64_t*>(yk);
    ps->Yi = reinterpret_cast<int32_t*>(yi);
    ps->Ysk = reinterpret_cast<uint64_t*>(ysk);
    ps->Ysi = reinterpret_cast<int32_t*>(ysi);
    ps->blk = reinterpret_cast<int32_t*>(blk);
    ps->total = reinterpret_cast<int32_t*>(total);
  }
  return off;
}

void launch_partition_keys(const uint64_t* key, int n, int p, const PartitionScratch& ps,
                           uint64_t* pivot_key, int32_t* pivot_id, int32_t* bucket,
                           int32_t* bucket_off, int32_t* members, hipStream_t stream) {
  launch_chunk_sort(key, n, p, ps.sorted, stream);
  launch_partition(key, n, p, ps.sorted, ps.Yk, ps.Yi, ps.Ysk, ps.Ysi, pivot_key, pivot_id,
                   bucket, ps.blk, ps.total, bucket_off, members, stream);
}

}  // namespace sad
