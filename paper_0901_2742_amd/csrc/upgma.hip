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
    // sums in the global work array; each cluster's best pair sum cached in
    // LDS after the cluster arrays (groups here are below kUpgmaWideMinN
    // members, so 64-bit cross products are exact)
    const FullS S{Sw + fm_off[g], n};
    if (lds_n > 0) {  // (with lds_n == 0 every group was widened beforehand)
      for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaThreads) S.t[q] = Fg[q];
      __threadfence_block();
    }
    __syncthreads();
    static_assert(kUpgmaWideMinN - 1 <= kUpgmaW64MaxN, "64-bit cross products");
    uint64_t* bsum = reinterpret_cast<uint64_t*>(sh + ((5 * n + 1) & ~1));
    upgma_init_best<true>(S, n, id, sz, active, best);
    __syncthreads();
    if ((tid >> 6) == 0)
      upgma_steps_hbm<true, 4>(S, n, id, sz, active, best, bsum, rec, g, st,
                               [&](int step, int ia, int ib) {
                                 mo[2 * step] = ia;
                                 mo[2 * step + 1] = ib;
                               });
  }
}

// Sw <- F widened to 64 bits, group by group (the two share their layout):
// blockIdx.y is the group, the blocks along x stride over its n^2 entries.
__global__ void widen_sums_kernel(const uint32_t* __restrict__ F,
                                  const int64_t* __restrict__ fm_off,
                                  const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw) {
  const int g = blockIdx.y;
  const int64_t n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  const int64_t m = n * n, o = fm_off[g];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += stride)
    Sw[o + q] = F[o + q];
}

// Large groups: one workgroup of kUpgmaWideThreads per group, pair sums in
// the global n x n work array, the steps split over all its waves.  LDS: id,
// size (0 = inactive), best partner, rescan list (4 n words) and, up to
// kUpgmaWideLdsN members, the best pair sums (n 64-bit words; larger groups
// keep them on the array's diagonal).
__global__ __launch_bounds__(kUpgmaWideThreads) void upgma_wide_kernel(
    const int64_t* __restrict__ fm_off,
    const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw,
    int32_t* __restrict__ merges_out, const int32_t* __restrict__ merge_base, DevStatus* st) {
  extern __shared__ uint64_t shw[];
  __shared__ WideScratch ws;
  const int g = blockIdx.x;
  const int n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  const bool lds_best = n <= kUpgmaWideLdsN;
  int32_t* id = reinterpret_cast<int32_t*>(shw + (lds_best ? n : 0));
  int32_t* sz = id + n;
  int32_t* best = id + 2 * n;
  int32_t* rec = id + 3 * n;
  int32_t* mo = merges_out + 2 * (int64_t)merge_base[g];
  const int tid = threadIdx.x;
  for (int a = tid; a < n; a += kUpgmaWideThreads) {
    id[a] = a;
    sz[a] = 1;
  }
  // (the sums were widened from F by widen_sums_kernel)
  const FullS S{Sw + fm_off[g], n};
  __syncthreads();
  auto rec_merge = [&](int step, int ia, int ib) {
    mo[2 * step] = ia;
    mo[2 * step + 1] = ib;
  };
  if (n <= kUpgmaW64MaxN)
    upgma_steps_wide<true, true>(S, n, id, sz, best, LdsBest{shw}, rec, &ws, g, st, rec_merge);
  else if (lds_best)
    upgma_steps_wide<false, true>(S, n, id, sz, best, LdsBest{shw}, rec, &ws, g, st, rec_merge);
  else if (n <= kUpgmaRow64MaxN)
    upgma_steps_wide<false, true>(S, n, id, sz, best, DiagBest{S.t, n}, rec, &ws, g, st,
                                  rec_merge);
  else
    upgma_steps_wide<false, false>(S, n, id, sz, best, DiagBest{S.t, n}, rec, &ws, g, st,
                                   rec_merge);
}

void launch_upgma(const uint32_t* F, const int64_t* fm_off, const int32_t* group_off,
                  int ngroups, int max_n, uint64_t* Swork, int32_t* merges_out,
                  const int32_t* merge_base, DevStatus* st, hipStream_t stream) {
  if (ngroups <= 0 || max_n <= 1) return;
  if (max_n >= kUpgmaWideMinN) {
    // a large group: its O(n) step phases on a workgroup of 4 waves
    // (a group of up to kUpgmaWideLdsN members also keeps its best sums in
    // LDS, whatever the largest group's size)
    const size_t lds = std::max((size_t)max_n * 4 * sizeof(int32_t),
                                (size_t)std::min(max_n, kUpgmaWideLdsN) *
                                    (4 * sizeof(int32_t) + sizeof(uint64_t)));
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)upgma_wide_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int bx = (int)std::min<int64_t>(64, ((int64_t)max_n * max_n + 255) / 256);
    widen_sums_kernel<<<dim3(bx, ngroups), 256, 0, stream>>>(F, fm_off, group_off, Swork);
    upgma_wide_kernel<<<ngroups, kUpgmaWideThreads, lds, stream>>>(fm_off, group_off, Swork,
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
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (lds > 160 * 1024 - 1024 || ngroups > cus) {
    // large groups present, or more groups than CUs (the LDS triangle allows
    // one workgroup per CU, so they would take several rounds): all groups
    // keep their sums in HBM, widened from F by one grid-wide pass
    use_lds_n = 0;
    lds = 0;
    const int bx = (int)std::min<int64_t>(64, ((int64_t)max_n * max_n + 255) / 256);
    widen_sums_kernel<<<dim3(bx, ngroups), 256, 0, stream>>>(F, fm_off, group_off, Swork);
  }
  // a group with global sums: 5 n words of cluster arrays, then n best sums
  lds = std::max(lds, ((size_t)7 * max_n + 2) * sizeof(int32_t));
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)upgma_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  upgma_kernel<<<ngroups, kUpgmaThreads, lds, stream>>>(F, fm_off, group_off, Swork, merges_out,
                                                         merge_base, use_lds_n, st);
}

}  // namespace sad
