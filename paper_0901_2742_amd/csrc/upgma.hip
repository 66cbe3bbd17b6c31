// UPGMA guide trees on the fixed-point k-mer similarities, one workgroup per
// group (bucket).  Each step merges the active pair with the largest average
// similarity S_AB / (|A| |B|), compared exactly by 128-bit cross products;
// ties go to the smallest (min id, max id).  The union keeps the slot of its
// first member and S(A u B, C) = S(A, C) + S(B, C).
//
// Every active cluster keeps its best partner under that same total order, so
// the global choice is a reduction over clusters.  After a merge, pairs not
// involving the two merged clusters are unchanged: a cluster whose best partner
// was one of them is rescanned (one wave per cluster), every other cluster only
// compares its best with the new union.
#include "sad_internal.h"

namespace sad {

constexpr int kUpgmaThreads = 256;
constexpr int kUpgmaWaves = kUpgmaThreads / 64;

struct Cand {
  uint64_t s;     // summed similarity
  uint64_t prod;  // |A| |B|
  uint64_t key;   // (min id << 32) | max id; all ones = no candidate
  int32_t a, b;   // slots
};

// 128-bit compare of s1 * p2 against s2 * p1
__device__ inline int cmp_avg(uint64_t s1, uint64_t p1, uint64_t s2, uint64_t p2) {
  const uint64_t lo1 = s1 * p2, hi1 = __umul64hi(s1, p2);
  const uint64_t lo2 = s2 * p1, hi2 = __umul64hi(s2, p1);
  if (hi1 != hi2) return hi1 > hi2 ? 1 : -1;
  if (lo1 != lo2) return lo1 > lo2 ? 1 : -1;
  return 0;
}

__device__ inline bool better(uint64_t s1, uint64_t p1, uint64_t k1, uint64_t s2, uint64_t p2,
                              uint64_t k2) {
  if (k1 == ~0ull) return false;
  if (k2 == ~0ull) return true;
  const int c = cmp_avg(s1, p1, s2, p2);
  if (c != 0) return c > 0;
  return k1 < k2;
}

__device__ inline uint64_t pair_key(int ia, int ib) {
  const uint32_t lo = (uint32_t)min(ia, ib), hi = (uint32_t)max(ia, ib);
  return ((uint64_t)lo << 32) | hi;
}

// best partner of slot r among active slots (whole wave; result in every lane)
__device__ inline int wave_best_partner(const uint64_t* S, int n, int r, const int32_t* id,
                                        const int32_t* sz, const int32_t* active) {
  const int lane = threadIdx.x & 63;
  uint64_t bs = 0, bp = 1, bk = ~0ull;
  int bb = -1;
  const uint64_t sr = (uint64_t)sz[r];
  const int ir = id[r];
  const uint64_t* Sr = S + (int64_t)r * n;
  for (int b = lane; b < n; b += 64) {
    if (b == r || !active[b]) continue;
    const uint64_t s = Sr[b], p = sr * (uint64_t)sz[b], k = pair_key(ir, id[b]);
    if (better(s, p, k, bs, bp, bk)) {
      bs = s;
      bp = p;
      bk = k;
      bb = b;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t os = __shfl_xor(bs, o, 64), op = __shfl_xor(bp, o, 64),
                   ok = __shfl_xor(bk, o, 64);
    const int ob = __shfl_xor(bb, o, 64);
    if (better(os, op, ok, bs, bp, bk)) {
      bs = os;
      bp = op;
      bk = ok;
      bb = ob;
    }
  }
  return bb;
}

__global__ __launch_bounds__(kUpgmaThreads) void upgma_kernel(
    const uint32_t* __restrict__ F, const int64_t* __restrict__ fm_off,
    const int32_t* __restrict__ group_off, uint64_t* __restrict__ Sw,
    int32_t* __restrict__ merges_out, const int32_t* __restrict__ merge_base, DevStatus* st) {
  extern __shared__ int32_t sh[];
  __shared__ Cand red[kUpgmaThreads];
  __shared__ int32_t nrec;
  const int g = blockIdx.x;
  const int n = group_off[g + 1] - group_off[g];
  if (n <= 1) return;
  int32_t* id = sh;
  int32_t* sz = sh + n;
  int32_t* active = sh + 2 * n;
  int32_t* best = sh + 3 * n;
  int32_t* rec = sh + 4 * n;
  const uint32_t* Fg = F + fm_off[g];
  uint64_t* S = Sw + fm_off[g];
  int32_t* mo = merges_out + 2 * (int64_t)merge_base[g];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int64_t q = tid; q < (int64_t)n * n; q += kUpgmaThreads) S[q] = Fg[q];
  for (int a = tid; a < n; a += kUpgmaThreads) {
    id[a] = a;
    sz[a] = 1;
    active[a] = 1;
  }
  __threadfence_block();
  __syncthreads();
  for (int r = wave; r < n; r += kUpgmaWaves) {
    const int b = wave_best_partner(S, n, r, id, sz, active);
    if (lane == 0) best[r] = b;
  }
  __syncthreads();
  for (int step = 0; step < n - 1; ++step) {
    // the best pair is the best of the clusters' best pairs
    Cand c0;
    c0.key = ~0ull;
    c0.s = 0;
    c0.prod = 1;
    c0.a = c0.b = -1;
    for (int a = tid; a < n; a += kUpgmaThreads) {
      const int b = best[a];
      if (!active[a] || b < 0) continue;
      const uint64_t s = S[(int64_t)a * n + b], p = (uint64_t)sz[a] * (uint64_t)sz[b];
      const uint64_t k = pair_key(id[a], id[b]);
      if (better(s, p, k, c0.s, c0.prod, c0.key)) {
        c0.s = s;
        c0.prod = p;
        c0.key = k;
        c0.a = min(a, b);
        c0.b = max(a, b);
      }
    }
    red[tid] = c0;
    __syncthreads();
    for (int w = kUpgmaThreads / 2; w > 0; w >>= 1) {
      if (tid < w) {
        const Cand& x = red[tid + w];
        const Cand& y = red[tid];
        if (better(x.s, x.prod, x.key, y.s, y.prod, y.key)) red[tid] = x;
      }
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
      nrec = 0;
    }
    // S(new, c) = S(a, c) + S(b, c) for the remaining active clusters
    for (int c = tid; c < n; c += kUpgmaThreads) {
      if (!active[c] || c == ba || c == bb) continue;
      const uint64_t v = S[(int64_t)ba * n + c] + S[(int64_t)bb * n + c];
      S[(int64_t)ba * n + c] = v;
      S[(int64_t)c * n + ba] = v;
    }
    __threadfence_block();
    __syncthreads();
    if (tid == 0) {
      sz[ba] += sz[bb];
      id[ba] = n + step;
      active[bb] = 0;
    }
    __syncthreads();
    if (step == n - 2) break;
    // best partners: rescan clusters that pointed at a merged cluster,
    // otherwise compare with the union
    for (int c = tid; c < n; c += kUpgmaThreads) {
      if (!active[c]) continue;
      const int b = best[c];
      if (c == ba || b == ba || b == bb) {
        rec[atomicAdd(&nrec, 1)] = c;
      } else {
        const uint64_t sb = S[(int64_t)c * n + b], pb = (uint64_t)sz[c] * (uint64_t)sz[b];
        const uint64_t sn = S[(int64_t)c * n + ba], pn = (uint64_t)sz[c] * (uint64_t)sz[ba];
        if (better(sn, pn, pair_key(id[c], id[ba]), sb, pb, pair_key(id[c], id[b]))) best[c] = ba;
      }
    }
    __syncthreads();
    const int nr = nrec;
    for (int q = wave; q < nr; q += kUpgmaWaves) {
      const int r = rec[q];
      const int b = wave_best_partner(S, n, r, id, sz, active);
      if (lane == 0) best[r] = b;
    }
    __syncthreads();
  }
}

void launch_upgma(const uint32_t* F, const int64_t* fm_off, const int32_t* group_off,
                  int ngroups, int max_n, uint64_t* Swork, int32_t* merges_out,
                  const int32_t* merge_base, DevStatus* st, hipStream_t stream) {
  if (ngroups <= 0 || max_n <= 1) return;
  const size_t lds = (size_t)5 * max_n * sizeof(int32_t);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)upgma_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  upgma_kernel<<<ngroups, kUpgmaThreads, lds, stream>>>(F, fm_off, group_off, Swork, merges_out,
                                                         merge_base, st);
}

}  // namespace sad
