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
// rows, row broadcasts across them) with no workgroup barrier.  While a group
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

// A candidate pair: summed similarity, |A| |B| (at most (kMaxGroup / 2)^2 <
// 2^32) and the pair of ids packed as (min << 16) | max (ids < 2 kMaxGroup <
// 2^16; all ones = no candidate).  The key names the pair, so the slots of the
// winner of a wave reduction are read from the lane whose own candidate has
// the winning key (winner_lane) instead of travelling with it.
struct WCand {
  uint64_t s;
  uint32_t p;
  uint32_t key;
};

__device__ inline uint32_t pair_key16(int ia, int ib) {
  return ((uint32_t)min(ia, ib) << 16) | (uint32_t)max(ia, ib);
}

// x comes before y in the merge order: the larger average s / p (compared by
// the cross products x.s y.p and y.s x.p, 64 x 32 bits), then the smaller
// key.  "No candidate" (s 0, p 1, key all ones) comes after every pair under
// this same order (a pair's key is below all ones and its average is at least
// 0), so it needs no test of its own.  Both comparisons are evaluated in every
// lane and combined without branches.
template <bool W64>
__device__ inline bool wc_better(const WCand& x, const WCand& y) {
  const bool key_first = x.key < y.key;
  if constexpr (W64) {
    const uint64_t l = x.s * (uint64_t)y.p, r = y.s * (uint64_t)x.p;
    return (l > r) | ((l == r) & key_first);
  } else {
    const uint64_t lo1 = x.s * (uint64_t)y.p, hi1 = __umul64hi(x.s, (uint64_t)y.p);
    const uint64_t lo2 = y.s * (uint64_t)x.p, hi2 = __umul64hi(y.s, (uint64_t)x.p);
    return (hi1 > hi2) | ((hi1 == hi2) & ((lo1 > lo2) | ((lo1 == lo2) & key_first)));
  }
}

__device__ inline WCand wc_none() {
  WCand c;
  c.s = 0;
  c.p = 1;
  c.key = ~0u;
  return c;
}

// First lane whose own candidate has the wave's winning key wk (-1 if none).
__device__ inline int winner_lane(uint32_t mine_key, uint32_t wk) {
  const uint64_t m = __ballot(wk != ~0u && mine_key == wk);
  return m ? __ffsll((unsigned long long)m) - 1 : -1;
}

// A lane's candidate moved by a DPP pattern; rows outside ROWS keep their own
// (with every row written, no lane keeps its old value: a plain DPP move).
template <int CTRL, int ROWS = 0xf>
__device__ inline uint32_t dpp32(uint32_t v) {
  if constexpr (ROWS == 0xf)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ inline uint64_t dpp64(uint64_t v) {
  return (uint64_t)dpp32<CTRL, ROWS>((uint32_t)v) |
         ((uint64_t)dpp32<CTRL, ROWS>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL, int ROWS = 0xf>
__device__ inline WCand wc_dpp(const WCand& c) {
  WCand x;
  x.s = dpp64<CTRL, ROWS>(c.s);
  x.p = dpp32<CTRL, ROWS>(c.p);
  x.key = dpp32<CTRL, ROWS>(c.key);
  return x;
}

// The key of the wave's first candidate in the merge order (all ones if no
// lane has one), wave-uniform; all 64 lanes active.  Within each row of 16
// lanes: lanes ^1 and ^2 of a quad, the mirrored quad of each half row, the
// mirrored half of the row (after each stage every lane of the group holds
// the group's first).  Across rows, by row broadcasts: lane 15 of rows 0 and
// 2 into rows 1 and 3, then lane 31 into rows 2 and 3, which leaves the
// wave's first in lane 63.
template <bool W64>
__device__ inline uint32_t wave_first_key(WCand c) {
  WCand x;
  x = wc_dpp<0xB1>(c);  // quad_perm [1, 0, 3, 2]
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x4E>(c);  // quad_perm [2, 3, 0, 1]
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x141>(c);  // row_half_mirror
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x140>(c);  // row_mirror
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x142, 0xa>(c);  // row_bcast:15 into rows 1 and 3
  if (wc_better<W64>(x, c)) c = x;
  x = wc_dpp<0x143, 0xc>(c);  // row_bcast:31 into rows 2 and 3
  if (wc_better<W64>(x, c)) c = x;
  return (uint32_t)__builtin_amdgcn_readlane((int)c.key, 63);
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

// The step loops take UB slots per lane at a time and load all their pair
// sums before using any (with the sums in global memory each load is a round
// trip: the standalone kernel uses UB = 4; the engine's tree phase, sums in
// LDS, uses 1).  A slot that is out of range or the row itself reads a valid
// stand-in pair whose value is ignored.

__device__ inline int other_slot(int r) { return r == 0 ? 1 : 0; }

// Best partner of slot r among the active slots (whole wave; -1 if none).
template <bool W64, int UB, typename St>
__device__ inline int wave_best_partner(const St& S, int n, int r, const int32_t* id,
                                        const int32_t* sz, const int32_t* active) {
  const int lane = threadIdx.x & 63;
  WCand c = wc_none();
  int cb = -1;
  const uint32_t sr = (uint32_t)sz[r];
  const int ir = id[r];
  for (int b0 = lane; b0 < n; b0 += 64 * UB) {
    uint64_t sv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = b0 + 64 * u;
      sv[u] = S.get(r, (b < n && b != r) ? b : other_slot(r));
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int b = b0 + 64 * u;
      if (b >= n || b == r || !active[b]) continue;
      WCand x;
      x.s = sv[u];
      x.p = sr * (uint32_t)sz[b];
      x.key = pair_key16(ir, id[b]);
      if (wc_better<W64>(x, c)) {
        c = x;
        cb = b;
      }
    }
  }
  const int src = winner_lane(c.key, wave_first_key<W64>(c));
  return src < 0 ? -1 : __builtin_amdgcn_readlane(cb, src);
}

// Best partners of every slot (the whole workgroup, kUpgmaWaves waves).
template <bool W64, int UB, typename St>
__device__ inline void upgma_init_best(const St& S, int n, const int32_t* id, const int32_t* sz,
                                       const int32_t* active, int32_t* best) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = wave; r < n; r += kUpgmaWaves) {
    const int b = wave_best_partner<W64, UB>(S, n, r, id, sz, active);
    if (lane == 0) best[r] = b;
  }
}

// The n - 1 merge steps, run by one wave after upgma_init_best.
// on_merge(step, min id, max id) is called by lane 0 as soon as a merge is
// decided and records it (the caller keeps the merge list: with the sums in
// LDS a step then touches no global memory, so its wave-local fences cost no
// memory round trip).  rec: scratch of n slots.  Returns false (after raising
// an error) if a step finds no pair.
template <bool W64, int UB, typename St, typename OnMerge>
__device__ bool upgma_steps(const St& S, int n, int32_t* id, int32_t* sz, int32_t* active,
                            int32_t* best, int32_t* rec, int g, DevStatus* st,
                            OnMerge&& on_merge) {
  const int lane = threadIdx.x & 63;
  for (int step = 0; step < n - 1; ++step) {
    // the best pair is the first of the clusters' best pairs
    WCand c = wc_none();
    uint32_t cab = 0;
    for (int r0 = lane; r0 < n; r0 += 64 * UB) {
      int bs[UB];
      uint64_t sv[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int r = r0 + 64 * u;
        bs[u] = r < n && active[r] ? best[r] : -1;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int r = r0 + 64 * u;
        sv[u] = bs[u] >= 0 ? S.get(r, bs[u]) : 0;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int r = r0 + 64 * u, b = bs[u];
        if (b < 0) continue;
        WCand x;
        x.s = sv[u];
        x.p = (uint32_t)sz[r] * (uint32_t)sz[b];
        x.key = pair_key16(id[r], id[b]);
        if (wc_better<W64>(x, c)) {
          c = x;
          cab = (uint32_t)min(r, b) | ((uint32_t)max(r, b) << 16);
        }
      }
    }
    const int src = winner_lane(c.key, wave_first_key<W64>(c));
    if (src < 0) {
      if (lane == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return false;
    }
    const uint32_t ab = (uint32_t)__builtin_amdgcn_readlane((int)cab, src);
    const int ba = (int)(ab & 0xffffu), bb = (int)(ab >> 16);
    if (lane == 0) {
      const int ia = id[ba], ib = id[bb];
      on_merge(step, min(ia, ib), max(ia, ib));
    }
    // S(new, c) = S(a, c) + S(b, c) for the remaining active clusters
    for (int q0 = lane; q0 < n; q0 += 64 * UB) {
      uint64_t va[UB], vb[UB];
      bool on[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int q = q0 + 64 * u;
        on[u] = q < n && active[q] && q != ba && q != bb;
        va[u] = on[u] ? S.get(ba, q) : 0;
        vb[u] = on[u] ? S.get(bb, q) : 0;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (on[u]) S.set(ba, q0 + 64 * u, va[u] + vb[u]);
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
    for (int q0 = 0; q0 < n; q0 += 64 * UB) {
      int bs[UB];
      bool cmp[UB], again[UB];
      uint64_t vc[UB], vu[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int q = q0 + 64 * u + lane;
        const bool on = q < n && active[q];
        bs[u] = on ? best[q] : -1;
        again[u] = on && (q == ba || bs[u] == ba || bs[u] == bb);
        cmp[u] = on && !again[u];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int q = q0 + 64 * u + lane;
        vc[u] = cmp[u] ? S.get(q, bs[u]) : 0;
        vu[u] = cmp[u] ? S.get(q, ba) : 0;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int q = q0 + 64 * u + lane;
        if (cmp[u]) {
          const int b = bs[u];
          WCand cur, uni;
          cur.s = vc[u];
          cur.p = (uint32_t)sz[q] * (uint32_t)sz[b];
          cur.key = pair_key16(id[q], id[b]);
          uni.s = vu[u];
          uni.p = (uint32_t)sz[q] * (uint32_t)sz[ba];
          uni.key = pair_key16(id[q], id[ba]);
          if (wc_better<W64>(uni, cur)) best[q] = ba;
        }
        // rescans listed in slot order
        const uint64_t m = __ballot(again[u]);
        if (again[u]) rec[nrec + (int)__popcll(m & ((1ull << lane) - 1ull))] = q;
        nrec += (int)__popcll(m);
      }
    }
    wave_sync();
    for (int t = 0; t < nrec; ++t) {
      const int r = rec[t];
      const int b = wave_best_partner<W64, UB>(S, n, r, id, sz, active);
      if (lane == 0) best[r] = b;
    }
    wave_sync();
  }
  return true;
}

}  // namespace sad
