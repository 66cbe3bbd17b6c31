// UPGMA core shared by the standalone guide-tree kernel and the alignment
// engine's fused tree phase (device code only).
//
// Each step merges the active pair with the largest average similarity
// S_AB / (|A| |B|), compared exactly by cross products; ties go to the
// smallest (min id, max id).  The union keeps the slot of its first member
// and S(A u B, C) = S(A, C) + S(B, C).  Every active cluster keeps its best
// partner under that same order, so the global choice is a reduction over
// clusters; after a merge only clusters whose best partner was one of the two
// merged ones are rescanned, the others compare their best with the union.
//
// The steps run on one wave: a step is a few wave-wide reductions (DPP within
// rows, two swizzles across them) with no workgroup barrier.  While a group
// has at most kUpgmaW64MaxN members the cross products fit 64 bits: a pair
// sum is at most |A| |B| 2^31 with |A| |B| <= n^2 / 4, so s1 p2 < 2^64 when
// n^4 / 16 * 2^31 < 2^64, i.e. n < 608.  Larger groups compare 128-bit
// products.
#pragma once
#include "sad_internal.h"

namespace sad {

constexpr int kUpgmaThreads = 256;
constexpr int kUpgmaWaves = kUpgmaThreads / 64;
// largest group whose upper triangle of 64-bit sums fits in LDS next to the
// per-cluster arrays
constexpr int kUpgmaLdsN = 190;
constexpr int kUpgmaW64MaxN = 600;

// A candidate pair: summed similarity, |A| |B|, the pair of ids packed as
// (min << 16) | max (ids < 2 kMaxGroup < 2^16; all ones = no candidate) and
// the pair of slots packed as a | b << 16.
struct WCand {
  uint64_t s;
  uint64_t p;
  uint32_t key;
  uint32_t ab;
};

__device__ inline uint32_t pair_key16(int ia, int ib) {
  return ((uint32_t)min(ia, ib) << 16) | (uint32_t)max(ia, ib);
}

// sign of s1 p2 - s2 p1
template <bool W64>
__device__ inline int cmp_avg(uint64_t s1, uint64_t p1, uint64_t s2, uint64_t p2) {
  if constexpr (W64) {
    const uint64_t l = s1 * p2, r = s2 * p1;
    return l > r ? 1 : (l < r ? -1 : 0);
  } else {
    const uint64_t lo1 = s1 * p2, hi1 = __umul64hi(s1, p2);
    const uint64_t lo2 = s2 * p1, hi2 = __umul64hi(s2, p1);
    if (hi1 != hi2) return hi1 > hi2 ? 1 : -1;
    if (lo1 != lo2) return lo1 > lo2 ? 1 : -1;
    return 0;
  }
}

// x comes before y in the merge order
template <bool W64>
__device__ inline bool wc_better(const WCand& x, const WCand& y) {
  if (x.key == ~0u) return false;
  if (y.key == ~0u) return true;
  const int c = cmp_avg<W64>(x.s, x.p, y.s, y.p);
  if (c != 0) return c > 0;
  return x.key < y.key;
}

__device__ inline WCand wc_none() {
  WCand c;
  c.s = 0;
  c.p = 1;
  c.key = ~0u;
  c.ab = 0;
  return c;
}

template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline uint64_t dpp64(uint64_t v) {
  return (uint64_t)dpp32<CTRL>((uint32_t)v) | ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL>
__device__ inline WCand wc_dpp(const WCand& c) {
  WCand x;
  x.s = dpp64<CTRL>(c.s);
  x.p = dpp64<CTRL>(c.p);
  x.key = dpp32<CTRL>(c.key);
  x.ab = dpp32<CTRL>(c.ab);
  return x;
}
__device__ inline WCand wc_xor(const WCand& c, int m) {
  WCand x;
  x.s = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)c.s, m, 64) |
        ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(c.s >> 32), m, 64) << 32);
  x.p = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)c.p, m, 64) |
        ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(c.p >> 32), m, 64) << 32);
  x.key = (uint32_t)__shfl_xor((int)c.key, m, 64);
  x.ab = (uint32_t)__shfl_xor((int)c.ab, m, 64);
  return x;
}

// The first candidate of the wave in the merge order, in every lane (all 64
// lanes active).  Pairings: lanes ^1 and ^2 within a quad, the mirrored quad
// of each half row, the mirrored half of each row, then rows ^16 and ^32;
// after each stage every lane of the group holds the group's first.
template <bool W64>
__device__ inline WCand wave_first(WCand c) {
  WCand x;
  x = wc_dpp<0xB1>(c);  // quad_perm [1, 0, 3, 2]
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x4E>(c);  // quad_perm [2, 3, 0, 1]
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x141>(c);  // row_half_mirror
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x140>(c);  // row_mirror
  if (wc_better<W64>(x, c)) c = x;
  x = wc_xor(c, 16);
  if (wc_better<W64>(x, c)) c = x;
  x = wc_xor(c, 32);
  if (wc_better<W64>(x, c)) c = x;
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

// Makes one lane's earlier LDS / global writes visible to the wave's later
// reads (and keeps the compiler from moving accesses across).
__device__ inline void wave_sync() {
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}

// Best partner of slot r among the active slots (whole wave; -1 if none).
template <bool W64, typename St>
__device__ inline int wave_best_partner(const St& S, int n, int r, const int32_t* id,
                                        const int32_t* sz, const int32_t* active) {
  const int lane = threadIdx.x & 63;
  WCand c = wc_none();
  const uint64_t sr = (uint64_t)sz[r];
  const int ir = id[r];
  for (int b = lane; b < n; b += 64) {
    if (b == r || !active[b]) continue;
    WCand x;
    x.s = S.get(r, b);
    x.p = sr * (uint64_t)sz[b];
    x.key = pair_key16(ir, id[b]);
    x.ab = (uint32_t)b;
    if (wc_better<W64>(x, c)) c = x;
  }
  c = wave_first<W64>(c);
  return c.key == ~0u ? -1 : (int)c.ab;
}

// Best partners of every slot (the whole workgroup, kUpgmaWaves waves).
template <bool W64, typename St>
__device__ inline void upgma_init_best(const St& S, int n, const int32_t* id, const int32_t* sz,
                                       const int32_t* active, int32_t* best) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = wave; r < n; r += kUpgmaWaves) {
    const int b = wave_best_partner<W64>(S, n, r, id, sz, active);
    if (lane == 0) best[r] = b;
  }
}

// The n - 1 merge steps, run by one wave after upgma_init_best.  mo receives
// the merges (min id, max id); on_merge(step, min id, max id) is called by
// lane 0 as soon as a merge is decided.  rec: scratch of n slots.  Returns
// false (after raising an error) if a step finds no pair.
template <bool W64, typename St, typename OnMerge>
__device__ bool upgma_steps(const St& S, int n, int32_t* id, int32_t* sz, int32_t* active,
                            int32_t* best, int32_t* rec, int32_t* mo, int g, DevStatus* st,
                            OnMerge&& on_merge) {
  const int lane = threadIdx.x & 63;
  for (int step = 0; step < n - 1; ++step) {
    // the best pair is the first of the clusters' best pairs
    WCand c = wc_none();
    for (int r = lane; r < n; r += 64) {
      const int b = best[r];
      if (!active[r] || b < 0) continue;
      WCand x;
      x.s = S.get(r, b);
      x.p = (uint64_t)sz[r] * (uint64_t)sz[b];
      x.key = pair_key16(id[r], id[b]);
      x.ab = (uint32_t)min(r, b) | ((uint32_t)max(r, b) << 16);
      if (wc_better<W64>(x, c)) c = x;
    }
    c = wave_first<W64>(c);
    if (c.key == ~0u) {
      if (lane == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return false;
    }
    const int ba = (int)(c.ab & 0xffffu), bb = (int)(c.ab >> 16);
    if (lane == 0) {
      const int ia = id[ba], ib = id[bb];
      mo[2 * step] = min(ia, ib);
      mo[2 * step + 1] = max(ia, ib);
      on_merge(step, min(ia, ib), max(ia, ib));
    }
    // S(new, c) = S(a, c) + S(b, c) for the remaining active clusters
    for (int q = lane; q < n; q += 64) {
      if (!active[q] || q == ba || q == bb) continue;
      S.set(ba, q, S.get(ba, q) + S.get(bb, q));
    }
    wave_sync();
    if (lane == 0) {
      sz[ba] += sz[bb];
      id[ba] = n + step;
      active[bb] = 0;
    }
    wave_sync();
    if (step == n - 2) break;
    // best partners: clusters that pointed at a merged cluster are listed
    // for a rescan, the others compare their best with the union
    int nrec = 0;
    for (int q0 = 0; q0 < n; q0 += 64) {
      const int q = q0 + lane;
      bool again = false;
      if (q < n && active[q]) {
        const int b = best[q];
        if (q == ba || b == ba || b == bb) {
          again = true;
        } else {
          WCand cur, uni;
          cur.s = S.get(q, b);
          cur.p = (uint64_t)sz[q] * (uint64_t)sz[b];
          cur.key = pair_key16(id[q], id[b]);
          uni.s = S.get(q, ba);
          uni.p = (uint64_t)sz[q] * (uint64_t)sz[ba];
          uni.key = pair_key16(id[q], id[ba]);
          if (wc_better<W64>(uni, cur)) best[q] = ba;
        }
      }
      const uint64_t m = __ballot(again);
      if (again) rec[nrec + (int)__popcll(m & ((1ull << lane) - 1ull))] = q;
      nrec += (int)__popcll(m);
    }
    wave_sync();
    for (int t = 0; t < nrec; ++t) {
      const int r = rec[t];
      const int b = wave_best_partner<W64>(S, n, r, id, sz, active);
      if (lane == 0) best[r] = b;
    }
    wave_sync();
  }
  return true;
}

}  // namespace sad
