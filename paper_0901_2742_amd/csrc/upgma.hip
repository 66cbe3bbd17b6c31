// UPGMA guide trees on the fixed-point k-mer similarities, one workgroup per
// group (bucket); the steps are in upgma_core.h.  The pair sums live in LDS
// (upper triangle, 64-bit) when the group is small enough, otherwise in a
// global n x n work array.
#include "upgma_core.h"

namespace sad {

// The whole workgroup loads the sums and finds every cluster's best partner;
// wave 0 then runs the merge steps.  With the sums in LDS the merges are
// listed in LDS (ml) and copied to mo at the end, so that a step makes no
// global access; with global sums (ml == nullptr) they go to mo directly.
template <bool W64, typename St>
__device__ inline void upgma_run(const St& S, int n, int32_t* id, int32_t* sz, int32_t* active,
                                 int32_t* best, int32_t* rec, int32_t* ml, int32_t* mo, int g,
                                 DevStatus* st) {
  upgma_init_best<W64>(S, n, id, sz, active, best);
  __syncthreads();
  if ((threadIdx.x >> 6) == 0) {
    int32_t* dst = ml ? ml : mo;
    upgma_steps<W64, 4>(S, n, id, sz, active, best, rec, g, st, [&](int step, int ia, int ib) {
      dst[2 * step] = ia;
      dst[2 * step + 1] = ib;
    });
  }
  __syncthreads();
  if (ml)
    for (int q = threadIdx.x; q < 2 * (n - 1); q += kUpgmaThreads) mo[q] = ml[q];
}

__global__ __launch_bounds__(kUpgmaThreads) void upgma_kernel(
    const uint32_t* __restrict__ F, const int64_t* __restrict__ fm_off,
    const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw,
    int32_t* __restrict__ merges_out, const int32_t* __restrict__ merge_base, int lds_n,
    DevStatus* st) {
  extern __shared__ __attribute__((aligned(16))) uint64_t shq[];
  const int g = blockIdx.x;
  const int n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  const bool in_lds = n <= lds_n;
  // LDS: [triangle of lds_n (lds_n - 1) / 2 u64][5 lds_n-or-n i32]
  //      [merge list, 2 lds_n i32, when the sums are in LDS]
  int32_t* sh = reinterpret_cast<int32_t*>(shq + (in_lds ? (int64_t)lds_n * (lds_n - 1) / 2 : 0));
  int32_t* id = sh;
  int32_t* sz = sh + n;
  int32_t* active = sh + 2 * n;
  int32_t* best = sh + 3 * n;
  int32_t* rec = sh + 4 * n;
  int32_t* ml = in_lds ? sh + 5 * lds_n : nullptr;
  const uint32_t* Fg = F + fm_off[g];
  int32_t* mo = merges_out + 2 * (int64_t)merge_base[g];
  const int tid = threadIdx.x;
  for (int a = tid; a < n; a += kUpgmaThreads) {
    id[a] = a;
    sz[a] = 1;
    active[a] = 1;
  }
  const bool w64 = n <= kUpgmaW64MaxN;
  if (in_lds) {
    const TriS S{shq, n};
    for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaThreads) {
      const int a = (int)(q / n), b = (int)(q % n);
      if (a < b) shq[a * n - a * (a + 1) / 2 + b - a - 1] = Fg[q];
    }
    __threadfence_block();
    __syncthreads();
    if (w64)
      upgma_run<true>(S, n, id, sz, active, best, rec, ml, mo, g, st);
    else
      upgma_run<false>(S, n, id, sz, active, best, rec, ml, mo, g, st);
  } else {
    const FullS S{Sw + fm_off[g], n};
    for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaThreads) S.t[q] = Fg[q];
    __threadfence_block();
    __syncthreads();
    if (w64)
      upgma_run<true>(S, n, id, sz, active, best, rec, nullptr, mo, g, st);
    else
      upgma_run<false>(S, n, id, sz, active, best, rec, nullptr, mo, g, st);
  }
}

// Large groups: one workgroup of kUpgmaWideThreads per group, pair sums in
// the global n x n work array, the steps split over all its waves.
__global__ __launch_bounds__(kUpgmaWideThreads) void upgma_wide_kernel(
    const uint32_t* __restrict__ F, const int64_t* __restrict__ fm_off,
    const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw,
    int32_t* __restrict__ merges_out, const int32_t* __restrict__ merge_base, DevStatus* st) {
  extern __shared__ int32_t shw[];
  __shared__ WideScratch ws;
  const int g = blockIdx.x;
  const int n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  int32_t* id = shw;
  int32_t* sz = shw + n;
  int32_t* active = shw + 2 * n;
  int32_t* best = shw + 3 * n;
  int32_t* rec = shw + 4 * n;
  const uint32_t* Fg = F + fm_off[g];
  int32_t* mo = merges_out + 2 * (int64_t)merge_base[g];
  const int tid = threadIdx.x;
  for (int a = tid; a < n; a += kUpgmaWideThreads) {
    id[a] = a;
    sz[a] = 1;
    active[a] = 1;
  }
  const FullS S{Sw + fm_off[g], n};
  for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaWideThreads) S.t[q] = Fg[q];
  __syncthreads();
  auto rec_merge = [&](int step, int ia, int ib) {
    mo[2 * step] = ia;
    mo[2 * step + 1] = ib;
  };
  if (n <= kUpgmaW64MaxN) {
    wide_init_best<true>(S, n, id, sz, active, best, &ws);
    upgma_steps_wide<true>(S, n, id, sz, active, best, rec, &ws, g, st, rec_merge);
  } else {
    wide_init_best<false>(S, n, id, sz, active, best, &ws);
    upgma_steps_wide<false>(S, n, id, sz, active, best, rec, &ws, g, st, rec_merge);
  }
}

void launch_upgma(const uint32_t* F, const int64_t* fm_off, const int32_t* group_off,
                  int ngroups, int max_n, uint64_t* Swork, int32_t* merges_out,
                  const int32_t* merge_base, DevStatus* st, hipStream_t stream) {
  if (ngroups <= 0 || max_n <= 1) return;
  if (max_n >= kUpgmaWideMinN) {
    // a large group: its O(n) step phases on a workgroup of 16 waves
    const size_t lds = (size_t)5 * max_n * sizeof(int32_t);
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)upgma_wide_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    upgma_wide_kernel<<<ngroups, kUpgmaWideThreads, lds, stream>>>(F, fm_off, group_off, Swork,
                                                                   merges_out, merge_base, st);
    return;
  }
  // groups up to lds_n keep their sums in LDS; the per-cluster arrays take
  // 5 max(n) words either way
  const int lds_n = std::min(max_n, kUpgmaLdsN);
  const size_t tri = (size_t)lds_n * (lds_n - 1) / 2 * sizeof(uint64_t);
  // (the merge lists of groups kept in LDS follow their 5 lds_n words)
  size_t lds = tri + (size_t)std::max(5 * max_n, 7 * lds_n) * sizeof(int32_t);
  int use_lds_n = lds_n;
  if (lds > 160 * 1024 - 1024) {
    // large groups present: all groups use the global sums
    use_lds_n = 0;
    lds = (size_t)5 * max_n * sizeof(int32_t);
  }
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)upgma_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  upgma_kernel<<<ngroups, kUpgmaThreads, lds, stream>>>(F, fm_off, group_off, Swork, merges_out,
                                                         merge_base, use_lds_n, st);
}

}  // namespace sad
