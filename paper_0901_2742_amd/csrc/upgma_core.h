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

// The keys of the wave's first candidates in the merge order of RB
// independent reductions (all ones where no lane has one), wave-uniform; all
// 64 lanes active.  Within each row of 16 lanes: lanes ^1 and ^2 of a quad,
// the mirrored quad of each half row, the mirrored half of the row (after
// each stage every lane of the group holds the group's first).  Across rows,
// by row broadcasts: lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
// into rows 2 and 3, which leaves the wave's first in lane 63.  The RB
// reductions advance stage by stage together, so that their dependency chains
// overlap.
template <int CTRL, int ROWS, bool W64, int RB>
__device__ inline void wc_stage(WCand (&c)[RB]) {
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const WCand x = wc_dpp<CTRL, ROWS>(c[j]);
    if (wc_better<W64>(x, c[j])) c[j] = x;
  }
}
template <bool W64, int RB>
__device__ inline void wave_first_keys(WCand (&c)[RB], uint32_t (&wk)[RB]) {
  wc_stage<0xB1, 0xf, W64>(c);   // quad_perm [1, 0, 3, 2]
  wc_stage<0x4E, 0xf, W64>(c);   // quad_perm [2, 3, 0, 1]
  wc_stage<0x141, 0xf, W64>(c);  // row_half_mirror
  wc_stage<0x140, 0xf, W64>(c);  // row_mirror
  wc_stage<0x142, 0xa, W64>(c);  // row_bcast:15 into rows 1 and 3
  wc_stage<0x143, 0xc, W64>(c);  // row_bcast:31 into rows 2 and 3
#pragma unroll
  for (int j = 0; j < RB; ++j) wk[j] = (uint32_t)__builtin_amdgcn_readlane((int)c[j].key, 63);
}
template <bool W64>
__device__ inline uint32_t wave_first_key(const WCand& c) {
  WCand cc[1] = {c};
  uint32_t wk[1];
  wave_first_keys<W64, 1>(cc, wk);
  return wk[0];
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
// LDS, uses 1); the best-partner scans get the same effect from scanning
// several rows at once.  A slot that is out of range or the row itself reads
// a valid stand-in pair whose value is ignored.

__device__ inline int other_slot(int r) { return r == 0 ? 1 : 0; }

// Best partners of the slots r[0..RB) among the active slots (whole wave; -1
// where none).  The rows share the loads of the slot arrays; their pair sums
// are all loaded before any is used, and their reductions run together.
template <bool W64, int RB, typename St>
__device__ inline void wave_best_partners(const St& S, int n, const int (&r)[RB],
                                          const int32_t* id, const int32_t* sz,
                                          const int32_t* active, int (&out)[RB]) {
  const int lane = threadIdx.x & 63;
  WCand c[RB];
  int cb[RB], ir[RB];
  uint32_t sr[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    c[j] = wc_none();
    cb[j] = -1;
    sr[j] = (uint32_t)sz[r[j]];
    ir[j] = id[r[j]];
  }
  for (int b = lane; b < n; b += 64) {
    uint64_t sv[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) sv[j] = S.get(r[j], b != r[j] ? b : other_slot(r[j]));
    const bool on = active[b] != 0;
    const uint32_t zb = (uint32_t)sz[b];
    const int ib = id[b];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (!on || b == r[j]) continue;
      WCand x;
      x.s = sv[j];
      x.p = sr[j] * zb;
      x.key = pair_key16(ir[j], ib);
      if (wc_better<W64>(x, c[j])) {
        c[j] = x;
        cb[j] = b;
      }
    }
  }
  uint32_t mine[RB], wk[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) mine[j] = c[j].key;
  wave_first_keys<W64, RB>(c, wk);
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const int src = winner_lane(mine[j], wk[j]);
    out[j] = src < 0 ? -1 : __builtin_amdgcn_readlane(cb[j], src);
  }
}

// Rows per batch of best-partner scans.
constexpr int kScanBatch = 4;

// Best partners of the slots rows[0..m) (whole wave), written to best[] by
// lane 0: batches of up to kScanBatch rows (a short last batch runs as 2 or
// 1 rows).
template <bool W64, typename St>
__device__ inline void scan_rows(const St& S, int n, const int32_t* rows, int m,
                                 const int32_t* id, const int32_t* sz, const int32_t* active,
                                 int32_t* best) {
  const int lane = threadIdx.x & 63;
  int t = 0;
  for (; t + kScanBatch <= m; t += kScanBatch) {
    int rr[kScanBatch], bb[kScanBatch];
#pragma unroll
    for (int j = 0; j < kScanBatch; ++j) rr[j] = rows[t + j];
    wave_best_partners<W64, kScanBatch>(S, n, rr, id, sz, active, bb);
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < kScanBatch; ++j) best[rr[j]] = bb[j];
  }
  if (m - t >= 2) {
    int rr[2] = {rows[t], rows[t + 1]}, bb[2];
    wave_best_partners<W64, 2>(S, n, rr, id, sz, active, bb);
    if (lane == 0) {
      best[rr[0]] = bb[0];
      best[rr[1]] = bb[1];
    }
    t += 2;
  }
  if (t < m) {
    int rr[1] = {rows[t]}, bb[1];
    wave_best_partners<W64, 1>(S, n, rr, id, sz, active, bb);
    if (lane == 0) best[rr[0]] = bb[0];
  }
}

// Best partners of every slot (the whole workgroup, kUpgmaWaves waves; wave w
// scans the slots w, w + kUpgmaWaves, ..., kScanBatch at a time).
template <bool W64, typename St>
__device__ inline void upgma_init_best(const St& S, int n, const int32_t* id, const int32_t* sz,
                                       const int32_t* active, int32_t* best) {
  const int wave = threadIdx.x >> 6;
  const int m = wave < n ? (n - wave + kUpgmaWaves - 1) / kUpgmaWaves : 0;
  for (int t = 0; t < m; t += kScanBatch) {
    const int k = min(kScanBatch, m - t);
    int rr[kScanBatch], bb[kScanBatch];
#pragma unroll
    for (int j = 0; j < kScanBatch; ++j) rr[j] = wave + kUpgmaWaves * (t + min(j, k - 1));
    wave_best_partners<W64, kScanBatch>(S, n, rr, id, sz, active, bb);
    if ((threadIdx.x & 63) == 0)
      for (int j = 0; j < k; ++j) best[rr[j]] = bb[j];
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
    scan_rows<W64>(S, n, rec, nrec, id, sz, active, best);
    wave_sync();
  }
  return true;
}

}  // namespace sad

namespace sad {

// ---------------------------------------------------------------- wide steps
// The same steps for large groups, run by a workgroup of kUpgmaWideThreads
// threads (one wave per SIMD), with each cluster's best pair sum cached
// (bs[r] = S(r, best[r]); in LDS up to kUpgmaWideLdsN members).  A step: the
// first of the best pairs (a reduction over the workgroup: a thread's own
// candidates in registers, then DPP across the wave, then across the waves
// through LDS); one pass over the clusters that forms the union's sums and
// compares each cluster's best with the union; the union's size and id; the
// rescans of the clusters that pointed at a merged one, spread over the
// waves, each row scanned by one wave.  Every reduction keeps the order of
// upgma_steps, so the merges are the same.
constexpr int kUpgmaWideThreads = 256;
constexpr int kUpgmaWideWaves = kUpgmaWideThreads / 64;
constexpr int kUpgmaWideMinN = 257;    // smaller groups keep the one-wave steps
constexpr int kUpgmaWideLdsN = 4096;   // larger groups keep the best sums in HBM
constexpr int kWideRB = 2;             // rows per wave and rescan batch
// Comparisons within one row r (its rescans, its best against the union)
// share the factor |r| in both cross products, so they compare s |b'| with
// s' |b|: s <= 2^31 |r| |b| and |r| + |b| + |b'| <= n give products of at most
// 2^31 (n / 3)^3, below 2^64 while n < 6144.
constexpr int kUpgmaRow64MaxN = 6143;

// Where the best pair sums live: LDS, or the unused diagonal of the n x n
// pair-sum array.
struct LdsBest {
  uint64_t* b;
  __device__ uint64_t get(int r) const { return b[r]; }
  __device__ void set(int r, uint64_t v) const { b[r] = v; }
};
struct DiagBest {
  uint64_t* t;
  int n;
  __device__ uint64_t get(int r) const { return t[(int64_t)r * (n + 1)]; }
  __device__ void set(int r, uint64_t v) const { t[(int64_t)r * (n + 1)] = v; }
};

// Per-wave winners of the workgroup reductions (one at a time), in LDS.
struct WideScratch {
  uint64_t s[1][kUpgmaWideWaves];
  uint32_t p[1][kUpgmaWideWaves];
  uint32_t key[1][kUpgmaWideWaves];
  int32_t arg[1][kUpgmaWideWaves];
  int32_t nrec;
};

// The workgroup's first candidate of RB reductions: every wave reduces its
// lanes' candidates c[j] (argument a[j]), lane 0 of each wave publishes, and
// after a barrier every thread compares the published ones in turn; out[j] is the
// winner's argument (-1 if no candidate) and outs[j] its sum.  The caller
// places a barrier before the next call (the published winners are read until
// then).
template <bool W64, int RB>
__device__ inline void wg_first(WCand (&c)[RB], const int (&a)[RB], WideScratch* ws,
                                int (&out)[RB], uint64_t (&outs)[RB]) {
  static_assert(RB == 1, "one workgroup reduction at a time");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t mine[RB], wk[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) mine[j] = c[j].key;
  wave_first_keys<W64, RB>(c, wk);
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const int src = winner_lane(mine[j], wk[j]);
    // after the reduction lane 63 holds the wave's first candidate
    const uint64_t s = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c[j].s, 63) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(c[j].s >> 32), 63)
                        << 32);
    const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)c[j].p, 63);
    const int arg = src < 0 ? -1 : __builtin_amdgcn_readlane(a[j], src);
    if (lane == 0) {
      ws->s[j][wave] = src < 0 ? 0 : s;
      ws->p[j][wave] = src < 0 ? 1u : p;
      ws->key[j][wave] = wk[j];
      ws->arg[j][wave] = arg;
    }
  }
  __syncthreads();
  // the waves' winners in wave order (a pair published twice carries the
  // same argument either time)
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    WCand d;
    d.s = ws->s[j][0];
    d.p = ws->p[j][0];
    d.key = ws->key[j][0];
    int da = ws->arg[j][0];
#pragma unroll
    for (int w = 1; w < kUpgmaWideWaves; ++w) {
      WCand x;
      x.s = ws->s[j][w];
      x.p = ws->p[j][w];
      x.key = ws->key[j][w];
      if (wc_better<W64>(x, d)) {
        d = x;
        da = ws->arg[j][w];
      }
    }
    out[j] = d.key == ~0u ? -1 : da;
    outs[j] = d.s;
  }
}

// Best partners of the rows r[0..RB) among the active slots (sz > 0), one
// wave scanning them all (kWideU slots per lane at a time, their sums loaded
// before any is compared; a candidate's p is the partner's size alone, R64
// when 64-bit products are exact); out[j] is the partner (-1 if none),
// outs[j] its pair sum, both wave-uniform.
constexpr int kWideU = 16;
template <bool R64, int RB, typename St, int U = kWideU>
__device__ inline void wave_rescan(const St& S, int n, const int (&r)[RB], const int32_t* id,
                                   const int32_t* sz, int (&out)[RB], uint64_t (&outs)[RB]) {
  const int lane = threadIdx.x & 63;
  WCand c[RB];
  int cb[RB], ir[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    c[j] = wc_none();
    cb[j] = -1;
    ir[j] = id[r[j]];
  }
  for (int b0 = lane; b0 < n; b0 += 64 * U) {
    uint64_t sv[U][RB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = min(b0 + 64 * u, n - 1);
#pragma unroll
      for (int j = 0; j < RB; ++j) sv[u][j] = S.get(r[j], b != r[j] ? b : other_slot(r[j]));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + 64 * u;
      const uint32_t zb = b < n ? (uint32_t)sz[b] : 0u;
      const int ib = b < n ? id[b] : 0;
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        if (zb == 0 || b == r[j]) continue;
        WCand x;
        x.s = sv[u][j];
        x.p = zb;
        x.key = pair_key16(ir[j], ib);
        if (wc_better<R64>(x, c[j])) {
          c[j] = x;
          cb[j] = b;
        }
      }
    }
  }
  uint32_t mine[RB], wk[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) mine[j] = c[j].key;
  wave_first_keys<R64, RB>(c, wk);
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const int src = winner_lane(mine[j], wk[j]);
    out[j] = src < 0 ? -1 : __builtin_amdgcn_readlane(cb[j], src);
    // after the reduction lane 63 holds the first candidate
    outs[j] = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c[j].s, 63) |
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(c[j].s >> 32), 63) << 32);
  }
}

// Rescans of the rows rows[0..m) (m the same in every thread): wave w takes
// the rows w, w + kUpgmaWideWaves, ..., kWideRB at a time, and its lane 0
// stores their best[] and bs[].  Ends with a barrier.
template <bool R64, typename St, typename BS>
__device__ inline void wide_rescan_rows(const St& S, int n, const int32_t* rows, int m,
                                        const int32_t* id, const int32_t* sz, int32_t* best,
                                        const BS& bs) {
  constexpr int RB = kWideRB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mine = m > wave ? (m - wave + kUpgmaWideWaves - 1) / kUpgmaWideWaves : 0;
  for (int t = 0; t < mine; t += RB) {
    const int k = min(RB, mine - t);
    int rr[RB], out[RB];
    uint64_t outs[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) rr[j] = rows[wave + kUpgmaWideWaves * (t + min(j, k - 1))];
    wave_rescan<R64, RB>(S, n, rr, id, sz, out, outs);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < k) {
          best[rr[j]] = out[j];
          bs.set(rr[j], outs[j]);
        }
    }
  }
  __syncthreads();
}

// The n - 1 merge steps on the whole workgroup.  sz[r] == 0 marks an
// inactive slot.  on_merge(step, min id, max id) runs on thread 0.  Returns
// false (after raising an error) if a step finds no pair; every thread
// returns the same.  rec: scratch of n slots.
template <bool W64, bool R64, typename St, typename BS, typename OnMerge>
__device__ bool upgma_steps_wide(const St& S, int n, int32_t* id, int32_t* sz, int32_t* best,
                                 const BS& bs, int32_t* rec, WideScratch* ws, int g,
                                 DevStatus* st, OnMerge&& on_merge) {
  const int tid = threadIdx.x;
  // every cluster's best partner and pair sum
  for (int r = tid; r < n; r += kUpgmaWideThreads) rec[r] = r;
  __syncthreads();
  wide_rescan_rows<R64>(S, n, rec, n, id, sz, best, bs);
  for (int step = 0; step < n - 1; ++step) {
    // the first of the clusters' best pairs (cached sums)
    WCand c[1] = {wc_none()};
    int cab[1] = {0};
    for (int r = tid; r < n; r += kUpgmaWideThreads) {
      const int b = sz[r] ? best[r] : -1;
      if (b < 0) continue;
      WCand x;
      x.s = bs.get(r);
      x.p = (uint32_t)sz[r] * (uint32_t)sz[b];
      x.key = pair_key16(id[r], id[b]);
      if (wc_better<W64>(x, c[0])) {
        c[0] = x;
        cab[0] = min(r, b) | (max(r, b) << 16);
      }
    }
    int win[1];
    uint64_t wins[1];
    wg_first<W64, 1>(c, cab, ws, win, wins);
    if (win[0] < 0) {
      if (tid == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return false;
    }
    const int ba = win[0] & 0xffff, bb = win[0] >> 16;
    const uint32_t szu = (uint32_t)(sz[ba] + sz[bb]);
    const int idu = n + step;
    if (tid == 0) {
      on_merge(step, min(id[ba], id[bb]), max(id[ba], id[bb]));
      rec[0] = ba;  // the union's own row is rescanned
      ws->nrec = 1;
    }
    __syncthreads();
    // the union's sums S(new, q) = S(a, q) + S(b, q); each other cluster
    // compares its best pair with the union, or is listed for a rescan if its
    // best partner was a merged cluster
    for (int q = tid; q < n; q += kUpgmaWideThreads) {
      if (!sz[q] || q == ba || q == bb) continue;
      const uint64_t v = S.get(ba, q) + S.get(bb, q);
      S.set(ba, q, v);
      const int b = best[q];
      if (b == ba || b == bb) {
        rec[atomicAdd(&ws->nrec, 1)] = q;
        continue;
      }
      WCand cur, uni;
      cur.s = bs.get(q);
      cur.p = (uint32_t)sz[b];  // (the common factor |q| dropped)
      cur.key = pair_key16(id[q], id[b]);
      uni.s = v;
      uni.p = szu;
      uni.key = pair_key16(id[q], idu);
      if (wc_better<R64>(uni, cur)) {
        best[q] = ba;
        bs.set(q, v);
      }
    }
    __syncthreads();
    if (tid == 0) {
      sz[ba] = (int32_t)szu;
      id[ba] = idu;
      sz[bb] = 0;
    }
    __syncthreads();
    if (step == n - 2) break;
    wide_rescan_rows<R64>(S, n, rec, ws->nrec, id, sz, best, bs);
  }
  return true;
}

// ---------------------------------------------------------------- one wave, sums in HBM
// The steps on one wave for a group whose pair sums live in the global work
// array (below kUpgmaRow64MaxN members): each cluster's best pair sum cached
// in LDS (bsum), the union's sums formed and compared with every cluster's
// best in one pass (QC slots per lane at a time, their loads first), then the
// rescans of the union and of the clusters that pointed at a merged one, two
// rows at a time.  A merged-away slot gets size 0 besides active = 0 (the
// rescans skip slots of size 0).  Comparisons within a row drop the row's own
// size (exact in 64 bits below kUpgmaRow64MaxN members).  Called by one wave
// after upgma_init_best; the merges are those of upgma_steps.
template <bool W64, int QC, typename St, typename OnMerge>
__device__ bool upgma_steps_hbm(const St& S, int n, int32_t* id, int32_t* sz, int32_t* active,
                                int32_t* best, uint64_t* bsum, int32_t* rec, int g,
                                DevStatus* st, OnMerge&& on_merge) {
  // (callers hold groups below kUpgmaRow64MaxN: row comparisons in 64 bits)
  const int lane = threadIdx.x & 63;
  for (int r = lane; r < n; r += 64) bsum[r] = S.get(r, best[r]);
  wave_sync();
  for (int step = 0; step < n - 1; ++step) {
    // the first of the clusters' best pairs (LDS only)
    WCand c = wc_none();
    uint32_t cab = 0;
    for (int r = lane; r < n; r += 64) {
      if (!active[r]) continue;
      const int b = best[r];
      WCand x;
      x.s = bsum[r];
      x.p = (uint32_t)sz[r] * (uint32_t)sz[b];
      x.key = pair_key16(id[r], id[b]);
      if (wc_better<W64>(x, c)) {
        c = x;
        cab = (uint32_t)min(r, b) | ((uint32_t)max(r, b) << 16);
      }
    }
    const int src = winner_lane(c.key, wave_first_key<W64>(c));
    if (src < 0) {
      if (lane == 0) raise_error(st, SAD_E_INVAL, g, W_UPGMA);
      return false;
    }
    const uint32_t ab = (uint32_t)__builtin_amdgcn_readlane((int)cab, src);
    const int ba = (int)(ab & 0xffffu), bb = (int)(ab >> 16);
    const uint32_t szu = (uint32_t)(sz[ba] + sz[bb]);
    const int idu = n + step;
    if (lane == 0) on_merge(step, min(id[ba], id[bb]), max(id[ba], id[bb]));
    // S(new, q) = S(a, q) + S(b, q), QC slots per lane at a time with their
    // loads first; each other cluster compares its best with the union or is
    // listed for a rescan
    if (lane == 0) rec[0] = ba;
    int nrec = 1;
    for (int q0 = lane; q0 < 64 * ((n + 63) / 64); q0 += 64 * QC) {
      uint64_t va[QC], vb[QC];
      bool on[QC];
#pragma unroll
      for (int u = 0; u < QC; ++u) {
        const int q = q0 + 64 * u;
        on[u] = q < n && active[q] && q != ba && q != bb;
        va[u] = on[u] ? S.get(ba, q) : 0;
        vb[u] = on[u] ? S.get(bb, q) : 0;
      }
#pragma unroll
      for (int u = 0; u < QC; ++u) {
        const int q = q0 + 64 * u;
        bool again = false;
        if (on[u]) {
          const uint64_t v = va[u] + vb[u];
          S.set(ba, q, v);
          const int b = best[q];
          again = b == ba || b == bb;
          if (!again) {
            WCand cur, uni;
            cur.s = bsum[q];
            cur.p = (uint32_t)sz[b];  // (the common factor |q| dropped)
            cur.key = pair_key16(id[q], id[b]);
            uni.s = v;
            uni.p = szu;
            uni.key = pair_key16(id[q], idu);
            if (wc_better<true>(uni, cur)) {
              best[q] = ba;
              bsum[q] = v;
            }
          }
        }
        const uint64_t m = __ballot(again);
        if (again) rec[nrec + (int)__popcll(m & ((1ull << lane) - 1ull))] = q;
        nrec += (int)__popcll(m);
      }
    }
    wave_sync();
    if (lane == 0) {
      sz[ba] = (int32_t)szu;
      id[ba] = idu;
      active[bb] = 0;
      sz[bb] = 0;
    }
    wave_sync();
    if (step == n - 2) break;
    for (int t = 0; t < nrec; t += 2) {
      const int k = min(2, nrec - t);
      int rr[2] = {rec[t], rec[t + k - 1]}, out[2];
      uint64_t outs[2];
      wave_rescan<true, 2, St, QC>(S, n, rr, id, sz, out, outs);
      if (lane == 0) {
        best[rr[0]] = out[0];
        bsum[rr[0]] = outs[0];
        if (k == 2) {
          best[rr[1]] = out[1];
          bsum[rr[1]] = outs[1];
        }
      }
    }
    wave_sync();
  }
  return true;
}

}  // namespace sad
