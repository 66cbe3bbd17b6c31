// UPGMA core shared by the standalone guide-tree kernel and the alignment
// engine's fused tree phase (device code only).
//
// Each step merges the active pair with the largest average similarity
// S_AB / (|A| |B|), compared exactly by 128-bit cross products; ties go to
// the smallest (min id, max id).  The union keeps the slot of its first member
// and S(A u B, C) = S(A, C) + S(B, C).  Every active cluster keeps its best
// partner under that same order, so the global choice is a reduction over
// clusters; after a merge only clusters whose best partner was one of the two
// merged ones are rescanned (one wave each), the others compare their best
// with the union.
#pragma once
#include "sad_internal.h"

namespace sad {

constexpr int kUpgmaThreads = 256;
constexpr int kUpgmaWaves = kUpgmaThreads / 64;
// largest group whose upper triangle of 64-bit sums fits in LDS next to the
// per-cluster arrays
constexpr int kUpgmaLdsN = 190;

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

__device__ inline void cand_take_if_better(Cand& c, const Cand& o) {
  if (better(o.s, o.prod, o.key, c.s, c.prod, c.key)) c = o;
}

// wave-wide best candidate (every lane ends with it)
__device__ inline Cand wave_best(Cand c) {
  for (int o = 32; o > 0; o >>= 1) {
    Cand x;
    x.s = __shfl_xor(c.s, o, 64);
    x.prod = __shfl_xor(c.prod, o, 64);
    x.key = __shfl_xor(c.key, o, 64);
    x.a = __shfl_xor(c.a, o, 64);
    x.b = __shfl_xor(c.b, o, 64);
    cand_take_if_better(c, x);
  }
  return c;
}

// Pair sums in LDS: upper triangle, a < b at a n - a (a + 1) / 2 + b - a - 1.
struct TriS {
  uint64_t* t;
  int n;
  __device__ uint64_t get(int a, int b) const {
    const int lo = min(a, b), hi = max(a, b);
    return t[lo * n - lo * (lo + 1) / 2 + hi - lo - 1];
  }
  __device__ void set(int a, int b, uint64_t v) const {
    const int lo = min(a, b), hi = max(a, b);
    t[lo * n - lo * (lo + 1) / 2 + hi - lo - 1] = v;
  }
};

// Pair sums in a global n x n array (both halves kept).
struct FullS {
  uint64_t* t;
  int n;
  __device__ uint64_t get(int a, int b) const { return t[(int64_t)a * n + b]; }
  __device__ void set(int a, int b, uint64_t v) const {
    t[(int64_t)a * n + b] = v;
    t[(int64_t)b * n + a] = v;
  }
};

// best partner of slot r among active slots (whole wave; result in every lane)
template <typename St>
__device__ inline int wave_best_partner(const St& S, int n, int r, const int32_t* id,
                                        const int32_t* sz, const int32_t* active) {
  const int lane = threadIdx.x & 63;
  Cand c;
  c.s = 0;
  c.prod = 1;
  c.key = ~0ull;
  c.a = r;
  c.b = -1;
  const uint64_t sr = (uint64_t)sz[r];
  const int ir = id[r];
  for (int b = lane; b < n; b += 64) {
    if (b == r || !active[b]) continue;
    Cand x;
    x.s = S.get(r, b);
    x.prod = sr * (uint64_t)sz[b];
    x.key = pair_key(ir, id[b]);
    x.a = r;
    x.b = b;
    cand_take_if_better(c, x);
  }
  return wave_best(c).b;
}

template <typename St, typename OnMerge>
__device__ void upgma_group(const St& S, int n, int32_t* id, int32_t* sz, int32_t* active,
                            int32_t* best, int32_t* rec, int32_t* nrec, Cand* red, int32_t* mo,
                            int g, DevStatus* st, OnMerge&& on_merge) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int r = wave; r < n; r += kUpgmaWaves) {
    const int b = wave_best_partner(S, n, r, id, sz, active);
    if (lane == 0) best[r] = b;
  }
  __syncthreads();
  for (int step = 0; step < n - 1; ++step) {
    // the best pair is the best of the clusters' best pairs
    Cand c;
    c.key = ~0ull;
    c.s = 0;
    c.prod = 1;
    c.a = c.b = -1;
    for (int a = tid; a < n; a += kUpgmaThreads) {
      const int b = best[a];
      if (!active[a] || b < 0) continue;
      Cand x;
      x.s = S.get(a, b);
      x.prod = (uint64_t)sz[a] * (uint64_t)sz[b];
      x.key = pair_key(id[a], id[b]);
      x.a = min(a, b);
      x.b = max(a, b);
      cand_take_if_better(c, x);
    }
    c = wave_best(c);
    if (lane == 0) red[(step & 1) * kUpgmaWaves + wave] = c;
    __syncthreads();
    // (red alternates halves between steps, so no barrier is needed before
    // the next step's writes)
    Cand w = red[(step & 1) * kUpgmaWaves];
#pragma unroll
    for (int q = 1; q < kUpgmaWaves; ++q) cand_take_if_better(w, red[(step & 1) * kUpgmaWaves + q]);
    const int ba = w.a, bb = w.b;
    if (ba < 0) {
      if (tid == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return;
    }
    if (tid == 0) {
      const int ia = id[ba], ib = id[bb];
      mo[2 * step] = min(ia, ib);
      mo[2 * step + 1] = max(ia, ib);
      on_merge(step, min(ia, ib), max(ia, ib));
    }
    // S(new, c) = S(a, c) + S(b, c) for the remaining active clusters
    for (int q = tid; q < n; q += kUpgmaThreads) {
      if (!active[q] || q == ba || q == bb) continue;
      S.set(ba, q, S.get(ba, q) + S.get(bb, q));
    }
    __threadfence_block();
    __syncthreads();
    if (tid == 0) {
      sz[ba] += sz[bb];
      id[ba] = n + step;
      active[bb] = 0;
      *nrec = 0;
    }
    __syncthreads();
    if (step == n - 2) break;
    // best partners: rescan clusters that pointed at a merged cluster,
    // otherwise compare with the union
    for (int q = tid; q < n; q += kUpgmaThreads) {
      if (!active[q]) continue;
      const int b = best[q];
      if (q == ba || b == ba || b == bb) {
        rec[atomicAdd(nrec, 1)] = q;
      } else {
        const uint64_t sb = S.get(q, b), pb = (uint64_t)sz[q] * (uint64_t)sz[b];
        const uint64_t sn = S.get(q, ba), pn = (uint64_t)sz[q] * (uint64_t)sz[ba];
        if (better(sn, pn, pair_key(id[q], id[ba]), sb, pb, pair_key(id[q], id[b]))) best[q] = ba;
      }
    }
    __syncthreads();
    const int nr = *nrec;
    for (int q = wave; q < nr; q += kUpgmaWaves) {
      const int r = rec[q];
      const int b = wave_best_partner(S, n, r, id, sz, active);
      if (lane == 0) best[r] = b;
    }
    __syncthreads();
  }
}


}  // namespace sad
