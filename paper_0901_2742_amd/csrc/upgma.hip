// UPGMA guide trees on the fixed-point k-mer similarities, one workgroup per
// group (bucket).  Each step merges the active pair with the largest average
// similarity S_AB / (|A| |B|), compared exactly by 128-bit cross products;
// ties go to the smallest (min id, max id).  The union keeps the slot of its
// first member and S(A u B, C) = S(A, C) + S(B, C).
#include "sad_internal.h"

namespace sad {

constexpr int kUpgmaThreads = 256;

struct Cand {
  uint64_t s;     // summed similarity
  uint64_t prod;  // |A| |B|
  uint64_t key;   // (min id << 32) | max id; all ones = no candidate
  int32_t a, b;   // slots
};

// 128-bit compare of s1 * p2 against s2 * p1
__device__ inline int cmp_avg(uint64_t s1, uint64_t p1, uint64_t s2, uint64_t p2) {
  uint64_t lo1 = s1 * p2, hi1 = __umul64hi(s1, p2);
  uint64_t lo2 = s2 * p1, hi2 = __umul64hi(s2, p1);
  if (hi1 != hi2) return hi1 > hi2 ? 1 : -1;
  if (lo1 != lo2) return lo1 > lo2 ? 1 : -1;
  return 0;
}

__device__ inline bool better(const Cand& x, const Cand& y) {
  if (x.key == ~0ull) return false;
  if (y.key == ~0ull) return true;
  int c = cmp_avg(x.s, x.prod, y.s, y.prod);
  if (c != 0) return c > 0;
  return x.key < y.key;
}

__global__ __launch_bounds__(kUpgmaThreads) void upgma_kernel(
    const uint32_t* __restrict__ F, const int64_t* __restrict__ fm_off,
    const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw,
    int32_t* __restrict__ merges_out, const int32_t* __restrict__ merge_base, DevStatus* st) {
  extern __shared__ int32_t sh[];
  __shared__ Cand red[kUpgmaThreads];
  const int g = blockIdx.x;
  const int n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  int32_t* id = sh;
  int32_t* sz = sh + n;
  int32_t* active = sh + 2 * n;
  const uint32_t* Fg = F + fm_off[g];
  uint64_t* S = Sw + fm_off[g];
  int32_t* mo = merges_out + 2 * (int64_t)merge_base[g];
  const int tid = threadIdx.x;
  for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaThreads) S[q] = Fg[q];
  for (int a = tid; a < n; a += kUpgmaThreads) {
    id[a] = a;
    sz[a] = 1;
    active[a] = 1;
  }
  __syncthreads();
  for (int step = 0; step < n - 1; ++step) {
    Cand best;
    best.key = ~0ull;
    best.s = 0;
    best.prod = 1;
    best.a = best.b = -1;
    // rows a = tid, tid + T, ...; columns b > a
    for (int a = tid; a < n; a += kUpgmaThreads) {
      if (!active[a]) continue;
      const int ia = id[a];
      const uint64_t sa = (uint64_t)sz[a];
      const uint64_t* Srow = S + (int64_t)a * n;
      for (int b = a + 1; b < n; ++b) {
        if (!active[b]) continue;
        Cand c;
        c.s = Srow[b];
        c.prod = sa * (uint64_t)sz[b];
        const int ib = id[b];
        const uint32_t lo = (uint32_t)min(ia, ib), hi = (uint32_t)max(ia, ib);
        c.key = ((uint64_t)lo << 32) | hi;
        c.a = a;
        c.b = b;
        if (better(c, best)) best = c;
      }
    }
    red[tid] = best;
    __syncthreads();
    for (int w = kUpgmaThreads / 2; w > 0; w >>= 1) {
      if (tid < w && better(red[tid + w], red[tid])) red[tid] = red[tid + w];
      __syncthreads();
    }
    const int ba = red[0].a, bb = red[0].b;
    if (ba < 0) {
      if (tid == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return;
    }
    if (tid == 0) {
      const int ia = id[ba], ib = id[bb];
      mo[2 * step] = min(ia, ib);
      mo[2 * step + 1] = max(ia, ib);
    }
    // S(new, c) = S(a, c) + S(b, c) for the remaining active clusters
    for (int c = tid; c < n; c += kUpgmaThreads) {
      if (!active[c] || c == ba || c == bb) continue;
      uint64_t v = S[(int64_t)ba * n + c] + S[(int64_t)bb * n + c];
      S[(int64_t)ba * n + c] = v;
      S[(int64_t)c * n + ba] = v;
    }
    __syncthreads();
    if (tid == 0) {
      sz[ba] += sz[bb];
      id[ba] = n + step;
      active[bb] = 0;
    }
    __threadfence_block();
    __syncthreads();
  }
}

void launch_upgma(const uint32_t* F, const int64_t* fm_off, const int32_t* group_off,
                        int ngroups, int max_n, uint64_t* Swork, int32_t* merges_out,
                        const int32_t* merge_base, DevStatus* st, hipStream_t stream) {
  if (ngroups <= 0 || max_n <= 1) return;
  size_t lds = (size_t)3 * max_n * sizeof(int32_t);
  if (lds > 64 * 1024) {
    hipFuncSetAttribute((const void*)upgma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
  }
  upgma_kernel<<<ngroups, kUpgmaThreads, lds, stream>>>(F, fm_off, group_off, Swork, merges_out,
                                                         merge_base, st);
}

}  // namespace sad
