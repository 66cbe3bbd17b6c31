// Alignment quality against known homology: the Q measure of Section 4 (the
// number of correctly aligned residue pairs over the number of residue pairs
// of the reference), with the reference given as homology classes: two
// residues are a reference pair iff they belong to the same class (ids are
// unique within a sequence, so the two lie in different sequences), and the
// pair is correctly aligned iff the alignment puts both in one column.
//
//   true pairs    = sum over classes of m (m - 1) / 2      (m = class size)
//   aligned pairs = sum over classes of the pairs of members in one column
//
// Kernels: class sizes (atomics), their exclusive scan (one workgroup), the
// members' columns scattered by class (CSR), then one wave per class counts
// equal columns among its members.
#include "sad_internal.h"

namespace sad {

constexpr int kQualThreads = 256;
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kQualThreads) void class_count_kernel(const int32_t* __restrict__ cls,
                                                                   int64_t total, int32_t nclass,
                                                                   int32_t* __restrict__ cnt,
                                                                   DevStatus* st) {
  for (int64_t r = blockIdx.x * (int64_t)kQualThreads + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kQualThreads) {
    const int32_t c = cls[r];
    if (c < 0 || c >= nclass) {
      raise_error(st, SAD_E_INVAL, r, W_QUALITY);
      continue;
    }
    atomicAdd(&cnt[c], 1);
  }
}

// off[c] = sum of cnt[0..c), off[nclass] = total; cursor = off (one workgroup).
__global__ __launch_bounds__(kScanThreads) void class_scan_kernel(const int32_t* __restrict__ cnt,
                                                                  int32_t nclass,
                                                                  int32_t* __restrict__ off,
                                                                  int32_t* __restrict__ cursor) {
  __shared__ int32_t part[kScanThreads];
  const int tid = threadIdx.x;
  const int per = (nclass + kScanThreads - 1) / kScanThreads;
  const int lo = min(nclass, tid * per), hi = min(nclass, lo + per);
  int32_t s = 0;
  for (int c = lo; c < hi; ++c) s += cnt[c];
  part[tid] = s;
  __syncthreads();
  // inclusive scan of the per-thread sums (Hillis-Steele)
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int32_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - s;
  for (int c = lo; c < hi; ++c) {
    off[c] = run;
    cursor[c] = run;
    run += cnt[c];
  }
  if (tid == kScanThreads - 1) off[nclass] = part[tid];
}

__global__ __launch_bounds__(kQualThreads) void class_scatter_kernel(
    const int32_t* __restrict__ cls, const int32_t* __restrict__ colmap, int64_t total,
    int32_t nclass, int32_t* __restrict__ cursor, int32_t* __restrict__ cols) {
  for (int64_t r = blockIdx.x * (int64_t)kQualThreads + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kQualThreads) {
    const int32_t c = cls[r];
    if (c < 0 || c >= nclass) continue;  // reported by the count kernel
    cols[atomicAdd(&cursor[c], 1)] = colmap[r];
  }
}

// One wave per class: lane l takes members l, l + 64, ... and compares each
// with the members after it.  sums[0] += aligned pairs, sums[1] += true pairs.
__global__ __launch_bounds__(kQualThreads) void class_pairs_kernel(
    const int32_t* __restrict__ off, const int32_t* __restrict__ cols, int32_t nclass,
    unsigned long long* __restrict__ sums) {
  const int lane = threadIdx.x & 63;
  const int waves = (int)(gridDim.x * (kQualThreads / 64));
  const int w0 = (int)(blockIdx.x * (kQualThreads / 64) + (threadIdx.x >> 6));
  unsigned long long aligned = 0, truep = 0;
  for (int c = w0; c < nclass; c += waves) {
    const int b = off[c], m = off[c + 1] - b;
    if (lane == 0) truep += (unsigned long long)m * (unsigned long long)(m - 1) / 2;
    for (int i = lane; i < m; i += 64) {
      const int32_t ci = cols[b + i];
      for (int j = i + 1; j < m; ++j) aligned += cols[b + j] == ci ? 1ull : 0ull;
    }
  }
  // wave sums, then one atomic per wave
  for (int o = 32; o > 0; o >>= 1) {
    aligned += __shfl_xor(aligned, o, 64);
    truep += __shfl_xor(truep, o, 64);
  }
  if (lane == 0) {
    atomicAdd(&sums[0], aligned);
    atomicAdd(&sums[1], truep);
  }
}

void launch_quality(const int32_t* colmap, const int32_t* cls, int64_t total, int32_t nclass,
                    int32_t* cnt, int32_t* off, int32_t* cursor, int32_t* cols,
                    unsigned long long* sums, DevStatus* st, hipStream_t stream) {
  launch_fill_i32(cnt, 0, nclass, stream);
  launch_fill_i32(reinterpret_cast<int32_t*>(sums), 0, 4, stream);
  if (total > 0) {
    const int blocks = (int)std::min<int64_t>((total + kQualThreads - 1) / kQualThreads, 4096);
    class_count_kernel<<<blocks, kQualThreads, 0, stream>>>(cls, total, nclass, cnt, st);
    class_scan_kernel<<<1, kScanThreads, 0, stream>>>(cnt, nclass, off, cursor);
    class_scatter_kernel<<<blocks, kQualThreads, 0, stream>>>(cls, colmap, total, nclass, cursor,
                                                               cols);
    const int pblocks = std::max(1, std::min((nclass + 3) / 4, 4096));
    class_pairs_kernel<<<pblocks, kQualThreads, 0, stream>>>(off, cols, nclass, sums);
  }
}

}  // namespace sad
