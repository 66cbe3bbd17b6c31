// Progressive profile-profile alignment engine (paper Section 2.3.3: each
// bucket is aligned by a sequential aligner; here UPGMA-guided progressive
// alignment with affine gaps).
//
// Work model: a DAG of jobs.  A job aligns two nodes (profiles) P1, P2 and
// writes a new node; a job becomes ready when its children's jobs are done.
// A persistent grid pops ready jobs from a device queue; each workgroup (four
// waves) runs one job at a time:
//   1. DP over 64-row strips of P1, strips dealt round-robin to the waves.  In
//      a strip, lane l owns row i = 64 s + l + 1 and at step t computes column
//      j = t - l + 1 (an anti-diagonal wavefront); the row above arrives from
//      lane l-1 through a DPP wave shift.  Strip s reads the last row of strip
//      s-1 from a per-link buffer, one 64-column chunk behind its producer, so
//      the waves work on consecutive strips at the same time.  Column scores
//      s(i,j) = U[i] . C2[j] with U = C1 S use packed 16-bit dot products
//      against P2 columns staged in a per-wave LDS ring.  Per cell one byte of
//      tie information is stored (the smallest op attaining H, and for X and
//      Y whether the open and/or the extend predecessor attains them).
//   2. Traceback from (W1, W2) by one wave in lockstep, staging 4 KB blocks of
//      tie bytes in LDS.  The greedy rule picks the smallest op still admitting
//      an optimal completion, which yields the optimal alignment whose op
//      string read backwards is lexicographically smallest (M < X < Y).
//   3. Merge by the whole workgroup: the op string is scanned to lay out the
//      new profile's columns (counts add) and each child's column map.
//
// Memory layout: node profiles are W x A uint16 counts in one pool; column
// maps (node column -> parent column) are W int32 in another.  Internal nodes
// are bump-allocated with W1 + W2 columns.
#include <cstdlib>
#include <type_traits>

#include "sad_internal.h"
#include "upgma_core.h"

namespace sad {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kColRing = 128;   // staged P2 columns per wave (power of two)
// Slots kColRing .. kColRing + 63 repeat slots 0 .. 63, so that a lane reads
// the 64 columns of a chunk at one base plus constant offsets (no wrap).
constexpr int kColRingPad = 64;
constexpr int kStageT4 = 16;    // traceback staging: 16 x 64 words (64 steps of a strip)
constexpr int kMaxStrips = kMaxWidth / 64;
constexpr int kEngineWGPerCU = 1;

// 32-bit words per staged P2 column: counts as packed u16 pairs, padded so a
// protein column is three 16-byte LDS reads
template <int A>
struct ColWords {
  static constexpr int value = A == 20 ? 12 : (A + 1) / 2;
};

__device__ inline int32_t shr1(int32_t old_lane0, int32_t v) {
  // lane l receives lane l-1's v; lane 0 keeps old_lane0
  return __builtin_amdgcn_update_dpp(old_lane0, v, 0x138, 0xf, 0xf, false);
}
__device__ inline int32_t shl1(int32_t old_lane63, int32_t v) {
  // lane l receives lane l+1's v; lane 63 keeps old_lane63
  return __builtin_amdgcn_update_dpp(old_lane63, v, 0x130, 0xf, 0xf, false);
}
// 64-bit DP values (merges whose score bound does not fit 32 bits) move
// between lanes as two 32-bit halves.
__device__ inline int64_t shr1(int64_t old_lane0, int64_t v) {
  const int32_t lo = shr1((int32_t)(uint32_t)old_lane0, (int32_t)(uint32_t)v);
  const int32_t hi = shr1((int32_t)(old_lane0 >> 32), (int32_t)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline int64_t shl1(int64_t old_lane63, int64_t v) {
  const int32_t lo = shl1((int32_t)(uint32_t)old_lane63, (int32_t)(uint32_t)v);
  const int32_t hi = shl1((int32_t)(old_lane63 >> 32), (int32_t)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// "minus infinity" of the DP in each value type: far enough below every
// reachable value that subtracting gap costs cannot wrap
template <typename T>
struct DpNeg;
template <>
struct DpNeg<int32_t> {
  static constexpr int32_t value = kNeg32;
};
template <>
struct DpNeg<int64_t> {
  static constexpr int64_t value = -(1ll << 62);
};
// Largest static bound of a 64-bit merge (the same limit as the CPU oracle's).
constexpr int64_t kBound64 = 2000000000000000000ll;

// Per-workgroup scratch (tie words, strip boundary rows) is written and read
// by the waves of one workgroup, i.e. one CU, whose vector L1 is write-through
// and sees its own stores: plain loads after workgroup-scope synchronisation.
template <typename V>
__device__ inline V load_wg(const V* p) {
  return *p;
}

// -1, 0 or 1 for d < 0, d == 0, d > 0 (one v_med3_i32)
__device__ inline int32_t sign3(int32_t d) {
  int32_t r;
  asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(d));
  return r;
}
__device__ inline int32_t sign3(int64_t d) { return (int32_t)(d > 0) - (int32_t)(d < 0); }

__device__ inline int32_t dot2(uint32_t a, uint32_t b, int32_t c) {
  typedef short v2s __attribute__((ext_vector_type(2)));
  v2s x = __builtin_bit_cast(v2s, a), y = __builtin_bit_cast(v2s, b);
  return __builtin_amdgcn_sdot2(x, y, c, false);
}

struct JobInfo {
  int32_t job, slot;
  int32_t na, nb, out;
  int32_t W1, W2, n1, n2;
  int64_t o, e;          // gap costs scaled by n1 n2
  int32_t err, abort, packed;
  int32_t wide;           // 1: DP values in 64 bits
  int32_t nstrips, nchunks;
  int64_t final_score;
  int32_t nops;
  int32_t nd_u, nd_c;  // digits of U and of the counts in the MFMA tile products
  int32_t coop, helper, owner;  // cooperative merge; this workgroup only helps; owner workgroup
  uint32_t tag;                 // tag of the merge's group boundary rows
  uint32_t ltag;                // first of 16 tags of this workgroup's own rows
  long long prof_off, up_off;
};

// Bounded waits of the engine, by site: a wait that runs out of time sets the
// site's bit in *wait_sites (kept even when an earlier error holds the status)
// and raises SAD_E_DEVICE with the site in the detail's high word.
enum WaitSite : int {
  WS_QUEUE = 0, WS_LINK = 1, WS_PROGRESS = 2, WS_ROW = 3, WS_GROUP = 4, WS_COOP = 5,
  WS_STRIP = 6, WS_LOADER = 7, WS_TREE = 8,
};
__device__ inline void wait_expired(DevStatus* st, int32_t* sites, int site, int64_t detail) {
  if (sites) atomicOr(sites, 1 << site);
  raise_error(st, SAD_E_DEVICE, ((int64_t)site << 32) | (uint32_t)detail, W_ENGINE_WAIT);
}

// Waits until link L has `need` columns; false on abort or time-out.
__device__ inline bool wait_link(const EngineArgs& a, JobInfo& J, const int32_t* prog, int L,
                                 int need) {
  if (__hip_atomic_load(&prog[L], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= need)
    return true;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  while (__hip_atomic_load(&prog[L], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
    if (__hip_atomic_load(&J.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
    __builtin_amdgcn_s_sleep(1);
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
      __hip_atomic_store(&J.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if ((threadIdx.x & 63) == 0) wait_expired(a.st, a.wait_sites, WS_LINK, L);
      return false;
    }
  }
  return true;
}

// Progress of a strip boundary row of this workgroup (an LDS counter).
__device__ inline int32_t link_progress(const int32_t* lds) {
  return __hip_atomic_load(lds, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until the boundary row has `need` columns; false on abort or time-out.
__device__ inline bool wait_progress(const EngineArgs& a, JobInfo& J, const int32_t* lds,
                                     int need) {
  if (link_progress(lds) >= need) return true;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  while (link_progress(lds) < need) {
    if (__hip_atomic_load(&J.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
    __builtin_amdgcn_s_sleep(1);
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
      __hip_atomic_store(&J.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if ((threadIdx.x & 63) == 0) wait_expired(a.st, a.wait_sites, WS_PROGRESS, need);
      return false;
    }
  }
  return true;
}

// A word of a boundary row, written by another wave of this workgroup or (in
// a cooperative merge) by another workgroup: agent-scope atomic stores and
// loads, which go past the CU's vector L1 (so a polling loop never sees a
// stale line) and are never merged or hoisted by the compiler.
template <typename T>
__device__ inline T load_link(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where a strip's boundary rows come from and go to (64-bit DP): the row
// above (H and X of the previous strip's last row) under its progress
// counter, this strip's last row and the counter to publish (null when no
// strip follows), and where H(W1, W2) goes if this strip holds row W1.
template <typename T>
struct StripLinks {
  const T* inH;
  const T* inX;
  const int32_t* in_lds;
  T* outH;
  T* outX;
  int32_t* out_lds;
  int64_t* score;
};

// Boundary rows of a 32-bit strip are tagged instead: each column is a 64-bit
// word, value in the low half and a tag in the high half, written once per tag
// with no fence; the reader loads a column until its tag matches.  The rows
// live in memory that holds nothing but such words (zeroed once, tags never
// reused), so a stale word never carries the tag a reader waits for.
struct TagLinks {
  const uint64_t* inH;  // row above (strip 0: a row of this workgroup, read
  const uint64_t* inX;  // but unused)
  bool has_in;          // the strip has a row above
  uint64_t* outH;       // this strip's last row (null for the last strip)
  uint64_t* outX;
  uint32_t in_tag, out_tag;
  int64_t* score;       // H(W1, W2) goes here if this strip holds row W1
};

__device__ inline uint64_t tag_word(int32_t v, uint32_t tag) {
  return (uint64_t)(uint32_t)v | ((uint64_t)tag << 32);
}
__device__ inline uint32_t tag_of(uint64_t w) { return (uint32_t)(w >> 32); }

// The row above a strip during one chunk: H and X of the previous strip's
// last row at the column each step's lane 0 computes.  RegRow keeps them in
// two registers (lane m: step m's column) shifted one lane per step; LdsRow
// reads them from the wave's LDS pairs at a wave-uniform address (a broadcast
// read, no shifts), put there by put_row.
template <typename T>
struct RegRow {
  T bhv, bxv;
  __device__ __forceinline__ T h(int) const { return bhv; }
  __device__ __forceinline__ T x(int) const { return bxv; }
  __device__ __forceinline__ void next() {
    bhv = shl1(bhv, bhv);
    bxv = shl1(bxv, bxv);
  }
};
template <typename T>
struct LdsRow {
  const T* p;  // step k: H at p[2 k], X at p[2 k + 1]
  __device__ __forceinline__ T h(int k) const { return p[2 * k]; }
  __device__ __forceinline__ T x(int k) const { return p[2 * k + 1]; }
  __device__ __forceinline__ void next() {}
};
// The chunk's row above read from the wave's LDS pairs into registers at the
// chunk's start, all K steps at once (the reads are in flight while the
// chunk's scores are read; read one by one next to their steps, each exposes
// the LDS latency to a wave that has its SIMD to itself).
template <typename T, int K>
struct ArrRow {
  T hv[K], xv[K];
  __device__ __forceinline__ void load(const T* p) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      hv[k] = p[2 * k];
      xv[k] = p[2 * k + 1];
    }
  }
  __device__ __forceinline__ T h(int k) const { return hv[k]; }
  __device__ __forceinline__ T x(int k) const { return xv[k]; }
  __device__ __forceinline__ void next() {}
};
// Lane m stores the row above of step m (lanes past the chunk's steps store
// values no step reads).  The wave's LDS operations run in order, so the
// chunk's reads that follow see these stores, and the next chunk's stores
// come after them.
template <typename T>
__device__ __forceinline__ void put_row(T* p, int lane, T h, T x) {
  p[2 * lane] = h;
  p[2 * lane + 1] = x;
  __builtin_amdgcn_wave_barrier();
}

// The strip's last row (lane 63's H and X after each step), collected for the
// next strip by shifting it into two registers: after K steps lane 64 - K + m
// holds step m.  (Storing each step's pair to LDS instead takes fewer
// instructions, but the stores share the in-order LDS counter with the
// row-above reads, and waiting for a read then waits for the stores too.)
template <typename T>
struct RegOut {
  T oh = 0, ox = 0;
  __device__ __forceinline__ void put(int, T h, T x) {
    oh = shl1(h, oh);
    ox = shl1(x, ox);
  }
};

template <int A, bool PACK>
struct RingScore;
// M = H_diag + s(i, j) of step k: the 32-bit vector-ALU strips fold H_diag
// into their dot products; other scores are added.
template <typename Score, typename T>
__device__ __forceinline__ T diag_plus_score(const Score& score, int k, int j, T h) {
  return h + (T)score(k, j);
}
template <int A, bool PACK>
__device__ __forceinline__ int32_t diag_plus_score(const RingScore<A, PACK>& score, int k, int,
                                                   int32_t h) {
  return score.plus(k, h);
}

// DP steps K0..K1-1 (K0 a multiple of 4) of the 64 steps of one chunk of a
// strip.  MASK: some cells of the chunk lie outside 1 <= j <= W2 and must
// leave H/X/Y untouched.  score(k, j) gives s(i, j) of this lane's row at step
// k.  R gives the row above the strip at lane 0 (RegRow or LdsRow); O
// collects the strip's last row.
// The gap states are carried plus the gap-open cost: X and Y here (and in
// every boundary row) are X + o and Y + o, so that X's update
// max(H_up - o, X_up - e) becomes max(H_up, X_up - e) + o, and
// open - extend = H_up - (X_up - e) in the same terms; H = max(M, max(X, Y) - o)
// is unchanged.  Integer identities, so every value and tie is the same.
template <bool MASK, int K0, int K1, typename T, typename Score, typename Row, typename Out>
__device__ __forceinline__ void dp_steps(int t0, int lane, int W2, T o, T e, Score&& score, T& H,
                                         T& X, T& Y, T& Hprev, Row& R, Out& O,
                                         uint32_t (&tw)[16]) {
  static_assert(K0 % 4 == 0 && K1 % 4 == 0, "tie words hold 4 steps");
  uint32_t word = 0;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    const int j = t0 + k - lane + 1;
    const T Hup = shr1(R.h(k), H);
    const T Xup = shr1(R.x(k), X);
    R.next();
    const T Hdiag = Hprev;
    Hprev = Hup;
    const T M = diag_plus_score(score, k, j, Hdiag);
    const T xe = Xup - e;
    const T Xn = max(Hup, xe);
    const T ye = Y - e;
    const T Yn = max(H, ye);
    const T t2 = max(Xn, Yn) - o;
    const T Hn = max(M, t2);
    const uint32_t hc = (M >= t2) ? 0u : ((Xn >= Yn) ? 1u : 2u);
    // tie byte hc | xc << 2 | yc << 4 with xc, yc = sign(open - extend) + 1
    // (0 extend only, 1 both, 2 open only), accumulated as hc + 4 sign + 16
    // sign; the + 4 + 16 of every byte is added once per word (each byte of
    // the exact sum lies in 0..42, so none carries into the next)
    const int32_t v = (int32_t)hc + 4 * sign3(Hup - xe) + 16 * sign3(H - ye);
    if (!MASK || (j >= 1 && j <= W2)) {
      H = Hn;
      X = Xn;
      Y = Yn;
    }
    word += (uint32_t)v << (8 * (k & 3));
    if ((k & 3) == 3) {
      tw[k >> 2] = word + 0x14141414u;
      word = 0;
    }
    O.put(k, H, X);
  }
}

// All 64 DP steps of one chunk of a strip.
template <bool MASK, typename T, typename Score, typename Row, typename Out>
__device__ __forceinline__ void dp_chunk(int t0, int lane, int W2, T o, T e, Score&& score, T& H,
                                         T& X, T& Y, T& Hprev, Row R, Out& O,
                                         uint32_t (&tw)[16]) {
  dp_steps<MASK, 0, 64>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
}

// Column score from a P2 column staged in the wave's LDS ring: packed 16-bit
// dot products (PACK) or 32-bit products.  base is this lane's slot of the
// chunk's first step (column t0 - lane + 1 at slot (t0 - lane) mod kColRing);
// step k reads slot base + k, past kColRing in the repeated slots.
template <int A, bool PACK>
struct RingScore {
  const uint32_t* base;
  const uint32_t* Up;
  const int32_t* U;
  __device__ __forceinline__ int32_t operator()(int k, int) const { return plus(k, 0); }
  // h + s(i, j) of step k: the dot products accumulate onto h (modulo 2^32,
  // exact because the sum fits in 32 bits)
  __device__ __forceinline__ int32_t plus(int k, int32_t h) const {
    constexpr int CW = ColWords<A>::value;
    const uint32_t* col = base + k * CW;
    int32_t sc = h;
    if constexpr (PACK) {
      if constexpr (A == 20) {
        const uint4 c0 = *reinterpret_cast<const uint4*>(col);
        const uint4 c1 = *reinterpret_cast<const uint4*>(col + 4);
        const uint2 c2 = *reinterpret_cast<const uint2*>(col + 8);
        sc = dot2(Up[0], c0.x, sc);
        sc = dot2(Up[1], c0.y, sc);
        sc = dot2(Up[2], c0.z, sc);
        sc = dot2(Up[3], c0.w, sc);
        sc = dot2(Up[4], c1.x, sc);
        sc = dot2(Up[5], c1.y, sc);
        sc = dot2(Up[6], c1.z, sc);
        sc = dot2(Up[7], c1.w, sc);
        sc = dot2(Up[8], c2.x, sc);
        sc = dot2(Up[9], c2.y, sc);
      } else {
#pragma unroll
        for (int m = 0; m < CW; ++m) sc = dot2(Up[m], col[m], sc);
      }
    } else {
#pragma unroll
      for (int m = 0; m < (A + 1) / 2; ++m) {
        const uint32_t w = col[m];
        sc = (int32_t)((uint32_t)sc + (uint32_t)(U[2 * m] * (int32_t)(w & 0xffffu)));
        if (2 * m + 1 < A)
          sc = (int32_t)((uint32_t)sc + (uint32_t)(U[2 * m + 1] * (int32_t)(w >> 16)));
      }
    }
    return sc;
  }
};

// One strip of the DP (run by one wave).  Returns false if the job aborted.
// PACK: U fits in 16 bits, so column scores use packed dot products.
template <int A, bool PACK, typename T>
__device__ bool dp_strip(const EngineArgs& a, JobInfo& J, int s, int lane, uint32_t* ring,
                         int32_t* prog, uint32_t* tbw, int32_t* links, const int32_t* Ssh,
                         const uint16_t* P1, const uint16_t* P2, T* rowl) {
  constexpr int CW = ColWords<A>::value;
  const int W1 = J.W1, W2 = J.W2, nchunks = J.nchunks, nstrips = J.nstrips;
  const T o = (T)J.o, e = (T)J.e;
  const int i = 64 * s + lane + 1;
  const int ie = min(i, W1);
  int32_t U[PACK ? 1 : A];
  uint32_t Up[PACK ? (A + 1) / 2 : 1];
  {
    // U = C1[i] S, one row of S at a time (keeps few values live)
    int32_t Uf[A];
#pragma unroll
    for (int b = 0; b < A; ++b) Uf[b] = 0;
    const uint16_t* crow = P1 + (int64_t)(ie - 1) * A;
#pragma unroll 1
    for (int q = 0; q < A; ++q) {
      const int32_t cq = (i <= W1) ? (int32_t)crow[q] : 0;
      const int32_t* Srow = Ssh + q * A;
#pragma unroll
      for (int b = 0; b < A; ++b) Uf[b] += cq * Srow[b];
    }
    if constexpr (PACK) {
#pragma unroll
      for (int m = 0; m < (A + 1) / 2; ++m) {
        const uint32_t lo = (uint32_t)Uf[2 * m] & 0xffffu;
        const uint32_t hi = (2 * m + 1 < A) ? ((uint32_t)Uf[2 * m + 1] << 16) : 0u;
        Up[m] = lo | hi;
      }
    } else {
#pragma unroll
      for (int b = 0; b < A; ++b) U[b] = Uf[b];
    }
  }
  T H = -(o + (T)(ie - 1) * e);
  const T neg = DpNeg<T>::value + o;  // minus infinity of the offset gap states
  T X = neg, Y = neg;
  T Hprev = (s == 0) ? (T)0 : -(o + (T)(64 * s - 1) * e);
  uint32_t* tbs = tbw + (int64_t)s * nchunks * 16 * 64;
  // boundary rows: H and X of each strip's last row, link_stride 32-bit
  // words per row (half as many 64-bit values)
  const int stride = a.link_stride / (int)(sizeof(T) / 4);
  T* lk = reinterpret_cast<T*>(links);
  const T* inH = lk + (int64_t)(s - 1) * 2 * stride;
  const T* inX = inH + stride;
  T* outH = lk + (int64_t)s * 2 * stride;
  T* outX = outH + stride;
  // the next chunk's P2 columns and boundary row are loaded during the current
  // chunk (the boundary only if its producer is already far enough)
  constexpr int NW = (A + 1) / 2;
  uint32_t pcol[NW];
  T pbh = 0, pbx = neg;
  bool have_link = (s == 0);
  auto prefetch = [&](int c, bool block) -> bool {
    const int jn = 64 * c + 1 + lane;
    if (jn <= W2) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(P2 + (int64_t)(jn - 1) * A);
#pragma unroll
      for (int m = 0; m < NW; ++m) pcol[m] = src[m];
    }
    if (s == 0) {
      pbh = jn <= W2 ? -(o + (T)(jn - 1) * e) : (T)0;
      pbx = neg;
      have_link = true;
      return true;
    }
    const int need = min(W2, 64 * c + 64);
    if (block) {
      if (!wait_link(a, J, prog, s - 1, need)) return false;
    } else if (__hip_atomic_load(&prog[s - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <
               need) {
      have_link = false;
      return true;
    }
    if (jn <= W2) {
      pbh = load_wg(inH + jn);
      pbx = load_wg(inX + jn);
    }
    have_link = true;
    return true;
  };
  if (!prefetch(0, true)) return false;
  for (int c = 0; c < nchunks; ++c) {
    const int t0 = 64 * c;
    const int jn = t0 + 1 + lane;
    if (!have_link) {
      if (!wait_link(a, J, prog, s - 1, min(W2, t0 + 64))) return false;
      if (jn <= W2) {
        pbh = load_wg(inH + jn);
        pbx = load_wg(inX + jn);
      }
    }
    const T bh = pbh, bx = pbx;
    if (jn <= W2) {
      const int slot = (jn - 1) & (kColRing - 1);
      uint32_t* dst = ring + slot * CW;
#pragma unroll
      for (int m = 0; m < NW; ++m) dst[m] = pcol[m];
#pragma unroll
      for (int m = NW; m < CW; ++m) dst[m] = 0u;
      if (slot < kColRingPad) {
        uint32_t* rep = dst + kColRing * CW;
#pragma unroll
        for (int m = 0; m < NW; ++m) rep[m] = pcol[m];
#pragma unroll
        for (int m = NW; m < CW; ++m) rep[m] = 0u;
      }
    }
    put_row(rowl, lane, bh, bx);
    __threadfence_block();
    if (c + 1 < nchunks) prefetch(c + 1, false);
    RegOut<T> O;
    const bool mask = (c == 0) || (t0 + 64 > W2);
    const RingScore<A, PACK> score{ring + ((t0 - lane) & (kColRing - 1)) * CW, Up, U};
    const LdsRow<T> R{rowl};
    uint32_t tw[16];
    if (mask)
      dp_chunk<true>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    else
      dp_chunk<false>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    if (s + 1 < nstrips) {
      // lane m holds the last row's value of step t0 + m, i.e. column t0 + m - 62
      const int jo = t0 + lane - 62;
      if (jo >= 1 && jo <= W2) {
        outH[jo] = O.oh;
        outX[jo] = O.ox;
      }
      const int done = (c + 1 == nchunks) ? W2 : min(W2, t0 + 1);
      __builtin_amdgcn_s_waitcnt(0);  // the link stores have reached L2
      __hip_atomic_store(&prog[s], done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // tie words after the release, so that the wait above covers only the
    // link stores (and this chunk's loads)
#pragma unroll
    for (int q = 0; q < 16; ++q) tbs[(t0 / 4 + q) * 64 + lane] = tw[q];
  }
  if (s == ((W1 - 1) >> 6) && lane == ((W1 - 1) & 63)) J.final_score = H;
  return true;
}

// ------------------------------------------------- DP strip, MFMA column scores
// The scores of a 64 x 64 tile (this strip's rows, 64 columns of P2) are one
// int8 matrix product on the matrix cores: s = U C2^T with U = C1 S.  U is
// split into signed base-256 digits and the counts into base-128 digits, so
// every partial product is exact in int32 and s = sum 2^(8a + 7b) U_a C2_b^T
// (mod 2^32, where s itself fits).  The tile is stored in a per-wave LDS ring
// skewed along anti-diagonals: cell (row l, column j) sits in row l at slot
// (l + j - 1) mod 128, so the scores lane l needs during one chunk are 64
// consecutive words of its row.  Tile c is written before chunk c; chunk c
// reads tile c for k >= l and tile c - 1 otherwise (its slots were written one
// chunk earlier and are not overwritten until chunk c + 1).
constexpr int kScPitch = 129;             // words per ring row (odd: no bank conflicts)
constexpr int kScWords = 64 * kScPitch;   // per wave
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned v16u __attribute__((ext_vector_type(16)));

template <int A>
struct Tile {
  static constexpr int KS = A > 16 ? 2 : 1;  // 16-deep K steps (K padded to 16 KS)
};

__device__ inline long pack_bytes8(const int32_t (&v)[8]) {
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    lo |= ((uint32_t)v[e] & 0xffu) << (8 * e);
    hi |= ((uint32_t)v[4 + e] & 0xffu) << (8 * e);
  }
  return (long)(((uint64_t)hi << 32) | lo);
}

// 8 counts held as four packed u16 pairs -> 8 bytes (bytes 0 and 2 of each word)
__device__ inline long pack_counts8(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
  const uint32_t lo = __builtin_amdgcn_perm(w1, w0, 0x06040200u);
  const uint32_t hi = __builtin_amdgcn_perm(w3, w2, 0x06040200u);
  return (long)(((uint64_t)hi << 32) | lo);
}

// Raw counts of tile columns for this lane's MFMA B operand: column
// 64 c + 32 cb + (lane & 31), counts 16 ks + 8 h + 0..7 (h = lane / 32).
template <int A>
__device__ inline void tile_load_counts(uint32_t (&bw)[2][Tile<A>::KS][4], const uint16_t* P2,
                                        int W2, int c, int lane) {
  const int n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int col = 64 * c + 32 * cb + n;
    const bool ok = col < W2;
    const uint2* src = reinterpret_cast<const uint2*>(P2 + (int64_t)(ok ? col : 0) * A);
#pragma unroll
    for (int ks = 0; ks < Tile<A>::KS; ++ks) {
      // words [8 ks + 4 h, +4) of the column, where they exist
      const int w0 = 8 * ks + 4 * h;
      uint2 x = make_uint2(0u, 0u), y = make_uint2(0u, 0u);
      if (ok && 2 * w0 < A) x = src[w0 / 2];
      if (ok && 2 * w0 + 4 < A) y = src[w0 / 2 + 1];
      bw[cb][ks][0] = x.x;
      bw[cb][ks][1] = x.y;
      bw[cb][ks][2] = y.x;
      bw[cb][ks][3] = y.y;
    }
  }
}

// Computes tile c and stores it in the wave's score ring.
template <int A>
__device__ inline void tile_scores(const long (&ua)[3][2][Tile<A>::KS],
                                   const uint32_t (&bw)[2][Tile<A>::KS][4], int nd_u, int nd_c,
                                   uint32_t* ring, int c, int lane) {
  constexpr int KS = Tile<A>::KS;
  const int n = lane & 31, h = lane >> 5;
  long bd[3][2][KS];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint32_t* w = bw[cb][ks];
      bd[0][cb][ks] = pack_counts8(w[0] & 0x007f007fu, w[1] & 0x007f007fu, w[2] & 0x007f007fu,
                                   w[3] & 0x007f007fu);
      bd[1][cb][ks] = pack_counts8((w[0] >> 7) & 0x007f007fu, (w[1] >> 7) & 0x007f007fu,
                                   (w[2] >> 7) & 0x007f007fu, (w[3] >> 7) & 0x007f007fu);
      bd[2][cb][ks] = pack_counts8((w[0] >> 14) & 0x00030003u, (w[1] >> 14) & 0x00030003u,
                                   (w[2] >> 14) & 0x00030003u, (w[3] >> 14) & 0x00030003u);
    }
  const int base = 64 * (c & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      v16u tot = {};
#pragma unroll
      for (int ad = 0; ad < 3; ++ad)
#pragma unroll
        for (int bdg = 0; bdg < 3; ++bdg) {
          if (ad >= nd_u || bdg >= nd_c) continue;
          v16i acc = {};
#pragma unroll
          for (int ks = 0; ks < KS; ++ks)
            acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(ua[ad][rb][ks], bd[bdg][cb][ks], acc, 0, 0,
                                                         0);
          tot += __builtin_bit_cast(v16u, acc) << (uint32_t)(8 * ad + 7 * bdg);
        }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + (r & 3) + 8 * (r >> 2) + 4 * h;
        const int slot = (base + row + 32 * cb + n) & 127;
        ring[row * kScPitch + slot] = tot[r];
      }
    }
}

// A operands of the tile products of strip s: U rows 64 s + 32 rb + (lane & 31),
// K entries 16 ks + 8 h + 0..7, as signed base-256 digits.
template <int A>
__device__ inline void tile_rows(long (&ua)[3][2][Tile<A>::KS], const uint16_t* P1,
                                 const int32_t* S32, int W1, int s, int lane) {
  constexpr int KS = Tile<A>::KS;
  const int m = lane & 31, h = lane >> 5;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const int row = 64 * s + 32 * rb + m;
    const bool ok = row < W1;
    const uint16_t* crow = P1 + (int64_t)(ok ? row : 0) * A;
    int32_t u[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int q = 0; q < 8; ++q) u[ks][q] = 0;
#pragma unroll 1
    for (int q = 0; q < A; ++q) {
      const int32_t cq = ok ? (int32_t)crow[q] : 0;
      const int32_t* Sq = S32 + q * 32 + 8 * h;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int x = 0; x < 8; ++x) u[ks][x] += cq * Sq[16 * ks + x];
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      int32_t d0[8], d1[8], d2[8];
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        const int32_t v = u[ks][x];
        const int32_t a0 = (int32_t)((uint32_t)v << 24) >> 24;
        const int32_t v1 = (v - a0) >> 8;
        const int32_t a1 = (int32_t)((uint32_t)v1 << 24) >> 24;
        d0[x] = a0;
        d1[x] = a1;
        d2[x] = (v1 - a1) >> 8;
      }
      ua[0][rb][ks] = pack_bytes8(d0);
      ua[1][rb][ks] = pack_bytes8(d1);
      ua[2][rb][ks] = pack_bytes8(d2);
    }
  }
}

// One strip of a 64-bit DP with MFMA tile scores (run by one wave), boundary
// rows a chunk at a time under LDS counters.  Returns false if the job
// aborted.
template <int A, typename T>
__device__ __forceinline__ bool dp_strip_mfma(const EngineArgs& a, JobInfo& J, int s, int lane, uint32_t* ring,
                              uint32_t* tbw, const StripLinks<T>& L, const int32_t* S32,
                              const uint16_t* P1, const uint16_t* P2) {
  constexpr int KS = Tile<A>::KS;
  const int W1 = J.W1, W2 = J.W2, nchunks = J.nchunks, nstrips = J.nstrips;
  const int nd_u = J.nd_u, nd_c = J.nd_c;
  const T o = (T)J.o, e = (T)J.e;
  const int i = 64 * s + lane + 1;
  const int ie = min(i, W1);
  long ua[3][2][KS];
  tile_rows<A>(ua, P1, S32, W1, s, lane);
  T H = -(o + (T)(ie - 1) * e);
  const T neg = DpNeg<T>::value + o;  // minus infinity of the offset gap states
  T X = neg, Y = neg;
  T Hprev = (s == 0) ? (T)0 : -(o + (T)(64 * s - 1) * e);
  uint32_t* tbs = tbw + (int64_t)s * nchunks * 16 * 64;
  const int ntiles = (W2 + 63) >> 6;
  uint32_t bw[2][KS][4];
  T pbh = 0, pbx = neg;
  bool have_link = (s == 0);
  auto link_fetch = [&](int c, bool block) -> bool {
    const int jn = 64 * c + 1 + lane;
    if (s == 0) {
      pbh = jn <= W2 ? -(o + (T)(jn - 1) * e) : (T)0;
      pbx = neg;
      have_link = true;
      return true;
    }
    const int need = min(W2, 64 * c + 64);
    if (block) {
      if (!wait_progress(a, J, L.in_lds, need)) return false;
    } else if (link_progress(L.in_lds) < need) {
      have_link = false;
      return true;
    }
    if (jn <= W2) {
      pbh = load_link(L.inH + jn);
      pbx = load_link(L.inX + jn);
    }
    have_link = true;
    return true;
  };
  tile_load_counts<A>(bw, P2, W2, 0, lane);
  if (!link_fetch(0, true)) return false;
  for (int c = 0; c < nchunks; ++c) {
    const int t0 = 64 * c;
    const int jn = t0 + 1 + lane;
    if (!have_link && !link_fetch(c, true)) return false;
    const T bh = pbh, bx = pbx;
    if (c < ntiles) tile_scores<A>(ua, bw, nd_u, nd_c, ring, c, lane);
    int32_t scv[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) scv[k] = (int32_t)ring[lane * kScPitch + (t0 & 127) + k];
    if (c + 1 < ntiles) tile_load_counts<A>(bw, P2, W2, c + 1, lane);
    if (c + 1 < nchunks) link_fetch(c + 1, false);
    RegOut<T> O;
    const bool mask = (c == 0) || (t0 + 64 > W2);
    auto score = [&](int k, int) -> int32_t { return scv[k]; };
    const RegRow<T> R{bh, bx};
    uint32_t tw[16];
    if (mask)
      dp_chunk<true>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    else
      dp_chunk<false>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    // lane m holds the last row's value of step t0 + m, i.e. column t0 + m - 62
    const int jo = t0 + lane - 62;
    if (L.outH) {
      if (jo >= 1 && jo <= W2) {
        L.outH[jo] = O.oh;
        L.outX[jo] = O.ox;
      }
      const int done = (c + 1 == nchunks) ? W2 : min(W2, t0 + 1);
      __builtin_amdgcn_s_waitcnt(0);  // the link stores are complete
      __hip_atomic_store(L.out_lds, done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // tie words after the release, so that the wait above covers only the
    // link stores (and this chunk's loads)
#pragma unroll
    for (int q = 0; q < 16; ++q) tbs[(t0 / 4 + q) * 64 + lane] = tw[q];
  }
  if (s == ((W1 - 1) >> 6) && lane == ((W1 - 1) & 63)) *L.score = (int64_t)H;
  return true;
}

// Boundary rows of strip s of the current merge (64-bit DP): rows of the
// workgroup's link buffer (indexed by strip) under LDS counters.  Every field
// is chosen by a select and written once, so that the struct stays in
// registers.
template <typename T>
__device__ inline StripLinks<T> strip_links(const EngineArgs& a, JobInfo& J, int s, int32_t* prog,
                                            int32_t* links) {
  const int ns = J.nstrips;
  const int stride = a.link_stride / (int)(sizeof(T) / 4);
  T* lk = reinterpret_cast<T*>(links);
  const bool has_in = s > 0, has_out = s + 1 < ns;
  T* lin = lk + (int64_t)(s - 1) * 2 * stride;
  T* lout = lk + (int64_t)s * 2 * stride;
  StripLinks<T> L;
  L.inH = has_in ? lin : nullptr;
  L.inX = has_in ? lin + stride : nullptr;
  L.in_lds = has_in ? &prog[s - 1] : nullptr;
  L.outH = has_out ? lout : nullptr;
  L.outX = has_out ? lout + stride : nullptr;
  L.out_lds = has_out ? &prog[s] : nullptr;
  L.score = &J.final_score;
  return L;
}

// One strip of a 32-bit DP with MFMA tile scores and tagged boundary rows
// (run by one wave), in chunks of CW steps (32 or 16, a shape the autotuner
// picks): a chunk needs CW columns of the row above, so the next strip trails
// this one by 63 + CW steps rather than 63 + 64; shorter chunks shorten that
// lag on chains of dependent merges and cost more per-chunk work.  The
// 64 x 64 score tile of columns 64 m + 1 .. 64 m + 64 is made at the start of
// chunk (64 / CW) m; the chunks of tile m read only tiles m - 1 and m, and
// tile m + 1 overwrites their ring slots only at the chunk after them.  The
// row above is read a chunk ahead, and again until every column carries the
// tag; the strip's last row is written at the end of each chunk with no
// fence, so the wave never waits for its own stores.  False when the job
// aborted.
template <int A, int CW>
__device__ __forceinline__ bool dp_strip_tagged(const EngineArgs& a, JobInfo& J, int s, int lane, uint32_t* ring,
                                uint32_t* tbw, const TagLinks& L, const int32_t* S32,
                                const uint16_t* P1, const uint16_t* P2, int32_t* rowl) {
  using T = int32_t;
  constexpr int KS = Tile<A>::KS;
  static_assert(CW == 16 || CW == 32, "chunks of 16 or 32 steps");
  constexpr int CPT = 64 / CW;  // chunks per score tile
  const int W1 = J.W1, W2 = J.W2;
  const int nch = (W2 + 63 + CW - 1) / CW;  // chunks of CW steps
  const int nd_u = J.nd_u, nd_c = J.nd_c;
  const T o = (T)J.o, e = (T)J.e;
  const int i = 64 * s + lane + 1;
  const int ie = min(i, W1);
  long ua[3][2][KS];
  tile_rows<A>(ua, P1, S32, W1, s, lane);
  T H = -(o + (T)(ie - 1) * e);
  const T neg = DpNeg<T>::value + o;  // minus infinity of the offset gap states
  T X = neg, Y = neg;
  T Hprev = (s == 0) ? (T)0 : -(o + (T)(64 * s - 1) * e);
  // tie words: the strip's block of J.nchunks x 16 x 64 words, word (t / 4, lane)
  uint32_t* tbs = tbw + (int64_t)s * J.nchunks * 16 * 64;
  const int ntiles = (W2 + 63) >> 6;
  uint32_t bw[2][KS][4];
  // above-row words of the next chunk (lanes 0..CW-1), loaded one chunk ahead
  // (strip 0's row above is the DP's boundary row, selected at the check: no
  // path writes these registers other than by the loads)
  // The loads are unconditional (no branch in the middle of a chunk): every
  // lane reads a column of the row, clamped to 1..W2 (strip 0 reads a row of
  // this workgroup and ignores it).
  const bool has_in = L.has_in;
  uint64_t nh = 0, nx = 0;
  auto fetch = [&](int c) {
    const int jn = min(max(CW * min(c, nch - 1) + 1 + lane, 1), W2);
    nh = load_link(L.inH + jn);
    nx = load_link(L.inX + jn);
  };
  // Loads and stores share one in-order counter, so waiting for a load also
  // waits for every store issued before it.  The row above of chunk c + 1 is
  // therefore read before chunk c's stores and checked right after them, in
  // the same iteration (the loop is rotated: the check of chunk c + 1 ends
  // iteration c), so that the wait covers that read and the count loads
  // before it but leaves the stores in flight; the poll only runs when a tag
  // is missing.
  T bh = 0, bx = 0;
  auto check = [&](int c) -> bool {
    const int jn = CW * c + 1 + lane;
    const bool need = has_in && lane < CW && jn <= W2;
    if (!__all(!need || (tag_of(nh) == L.in_tag && tag_of(nx) == L.in_tag))) {
      const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
      do {
        if (__hip_atomic_load(&J.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
          return false;
        __builtin_amdgcn_s_sleep(1);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
          __hip_atomic_store(&J.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (lane == 0) wait_expired(a.st, a.wait_sites, WS_ROW, jn);
          return false;
        }
        fetch(c);
      } while (!__all(!need || (tag_of(nh) == L.in_tag && tag_of(nx) == L.in_tag)));
    }
    bh = has_in ? (T)(int32_t)(uint32_t)nh : (jn <= W2 ? -(o + (T)(jn - 1) * e) : (T)0);
    bx = has_in ? (T)(int32_t)(uint32_t)nx : neg;
    return true;
  };
  tile_load_counts<A>(bw, P2, W2, 0, lane);
  fetch(0);
  if (!check(0)) return false;
  for (int c = 0; c < nch; ++c) {
    const int t0 = CW * c;
    const int m = c / CPT;
    if (c % CPT == 0 && m < ntiles) {
      tile_scores<A>(ua, bw, nd_u, nd_c, ring, m, lane);
      if (m + 1 < ntiles) tile_load_counts<A>(bw, P2, W2, m + 1, lane);
    }
    put_row(rowl, lane, bh, bx);
    ArrRow<T, CW> R;
    R.load(rowl);
    int32_t scv[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) scv[k] = (int32_t)ring[lane * kScPitch + (t0 & 127) + k];
    // (the reads above stay ahead of the steps)
    __builtin_amdgcn_sched_barrier(0);
    RegOut<T> O;
    const bool mask = (t0 < 63) || (t0 + CW > W2);
    auto score = [&](int k, int) -> int32_t { return scv[k]; };
    uint32_t tw[16];
    // the next chunk's row above is read half-way through this one: early
    // enough to arrive by the check, late enough that a strip trailing its
    // producer as closely as it can still finds it written
    constexpr int KF = CW / 2;
    if (mask) {
      dp_steps<true, 0, KF>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
      fetch(c + 1);
      dp_steps<true, KF, CW>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    } else {
      dp_steps<false, 0, KF>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
      fetch(c + 1);
      dp_steps<false, KF, CW>(t0, lane, W2, o, e, score, H, X, Y, Hprev, R, O, tw);
    }
    if (L.outH) {
      // lanes 64 - CW .. 63 hold the last row's values of steps t0 .. t0 + CW - 1,
      // i.e. columns t0 + lane - (64 - CW) - 62
      const int jo = t0 + lane - (64 - CW) - 62;
      const T oh = O.oh, ox = O.ox;
      if (lane >= 64 - CW && jo >= 1 && jo <= W2) {
        __hip_atomic_store(L.outH + jo, tag_word(oh, L.out_tag), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(L.outX + jo, tag_word(ox, L.out_tag), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
#pragma unroll
    for (int q = 0; q < CW / 4; ++q) tbs[(t0 / 4 + q) * 64 + lane] = tw[q];
    if (c + 1 < nch && !check(c + 1)) return false;
  }
  if (s == ((W1 - 1) >> 6) && lane == ((W1 - 1) & 63)) *L.score = (int64_t)H;
  return true;
}

// Rows of a 32-bit strip s in the k-th group this workgroup runs.  Rows inside
// a group are the workgroup's own (row s mod 4, tag ltag + k).  Rows between
// groups: in a cooperative merge the owner's uncached area (row of the group
// boundary, the merge's tag); otherwise the workgroup's row 3 (tag ltag + the
// group of the writing strip).
__device__ inline TagLinks tag_links(const EngineArgs& a, JobInfo& J, int s, int k) {
  const int ns = J.nstrips;
  constexpr int64_t R2 = 2 * (int64_t)kCoopRowLen;  // an H row and an X row
  uint64_t* lrows =
      reinterpret_cast<uint64_t*>(a.trow + (int64_t)blockIdx.x * a.trow_words_per_wg +
                                  kCoopHeadWords);
  uint64_t* crows =
      reinterpret_cast<uint64_t*>(a.coop_buf + (int64_t)J.owner * a.coop_words_per_wg +
                                  kCoopHeadWords);
  const bool has_in = s > 0, has_out = s + 1 < ns;
  const bool grp_in = s % kCoopGroupStrips == 0;
  const bool grp_out = s % kCoopGroupStrips == kCoopGroupStrips - 1;
  const int g = s / kCoopGroupStrips;
  uint64_t* rin = grp_in ? (J.coop ? crows + (int64_t)(g - 1) * R2 : lrows + 3 * R2)
                         : lrows + (int64_t)((s - 1) % kCoopGroupStrips) * R2;
  uint64_t* rout = grp_out ? (J.coop ? crows + (int64_t)g * R2 : lrows + 3 * R2)
                           : lrows + (int64_t)(s % kCoopGroupStrips) * R2;
  TagLinks L;
  L.has_in = has_in;
  L.inH = has_in ? rin : lrows;
  L.inX = has_in ? rin + kCoopRowLen : lrows + kCoopRowLen;
  L.outH = has_out ? rout : nullptr;
  L.outX = has_out ? rout + kCoopRowLen : nullptr;
  L.in_tag = grp_in ? (J.coop ? J.tag : J.ltag + (uint32_t)(k - 1)) : J.ltag + (uint32_t)k;
  L.out_tag = (grp_out && J.coop) ? J.tag : J.ltag + (uint32_t)k;
  L.score = J.coop ? &a.coop_score[J.job] : &J.final_score;
  return L;
}

// The 32-bit DP of a merge on this workgroup.  The strips form groups of 4;
// wave w runs strip 4 g + w of each group g the workgroup takes.  Alone, the
// workgroup takes every group in order.  In a cooperative merge the groups
// are claimed in increasing order from the merge's counter (the owner starts
// with group 0); wave 0 claims the next group when it reaches it, so the
// groups of one workgroup overlap as the strips of one merge do, and every
// finished strip makes its tie bytes (and H(W1, W2)) visible device-wide,
// then counts itself.
template <int A, int CW>
__device__ __forceinline__ bool tagged_dp(const EngineArgs& a, JobInfo& J, int wave, int lane, uint32_t* myring,
                          const int32_t* S32, const uint16_t* P1, const uint16_t* P2,
                          int32_t* glist, int32_t* gstate, int32_t* rowl) {
  const int ns = J.nstrips;
  const int ngroups = (ns + kCoopGroupStrips - 1) / kCoopGroupStrips;
  uint32_t* tbw = a.tb + (int64_t)J.owner * a.tb_words_per_wg;
  for (int k = 0;; ++k) {
    int g = k;
    if (J.coop) {
      if (wave == 0 && lane == 0 &&
          k >= __hip_atomic_load(&gstate[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
        const int c = atomicAdd(&a.coop_next[J.job], 1);
        if (c < ngroups) {
          glist[k] = c;
          __hip_atomic_store(&gstate[0], k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          __hip_atomic_store(&gstate[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      int have = 0;
      const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        have = __hip_atomic_load(&gstate[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (have > k) break;
        if (__hip_atomic_load(&gstate[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) {
          have = __hip_atomic_load(&gstate[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          break;
        }
        if (__hip_atomic_load(&J.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
          return false;
        __builtin_amdgcn_s_sleep(1);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
          __hip_atomic_store(&J.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (lane == 0) wait_expired(a.st, a.wait_sites, WS_GROUP, k);
          return false;
        }
      }
      if (have <= k) break;
      g = glist[k];
    } else if (g >= ngroups) {
      break;
    }
    const int s = g * kCoopGroupStrips + wave;
    if (s < ns) {
      const TagLinks L = tag_links(a, J, s, k);
      if (!dp_strip_tagged<A, CW>(a, J, s, lane, myring, tbw, L, S32, P1, P2, rowl))
        return false;
      if (J.coop) {
        __builtin_amdgcn_s_waitcnt(0);
        __threadfence();
        if (lane == 0) atomicAdd(&a.coop_strips[J.job], 1);
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------- traceback
// The path visits strips from the last to the first and, inside a strip,
// steps t = j - 1 + l that decrease by one or two per op: a staged block of
// 16 x 64 tie words in LDS serves about 30 ops before it is reloaded.
struct Stage {
  int s, t4a;
};

// Makes the staged block of strip s cover tie words t4lo..t4hi (t4hi - t4lo
// < kStageT4); the block is placed with t4hi at its top because the path
// moves towards smaller t.
__device__ inline void stage_cover(const uint32_t* tbw, uint32_t* tbst, Stage& st, int stride_s,
                                   int T4, int lane, int s, int t4lo, int t4hi) {
  if (s == st.s && t4lo >= st.t4a && t4hi < st.t4a + kStageT4) return;
  const int t4a = max(0, t4hi - (kStageT4 - 1));
  __builtin_amdgcn_wave_barrier();
  __threadfence_block();
  // all loads in flight before the first LDS store (addresses clamped to the
  // strip, out-of-strip words zeroed afterwards)
  const uint32_t* base = tbw + (int64_t)s * stride_s + lane;
  uint32_t v[kStageT4];
#pragma unroll
  for (int r = 0; r < kStageT4; ++r) v[r] = load_wg(base + (int64_t)min(t4a + r, T4 - 1) * 64);
#pragma unroll
  for (int r = 0; r < kStageT4; ++r) tbst[r * 64 + lane] = (t4a + r < T4) ? v[r] : 0u;
  st.s = s;
  st.t4a = t4a;
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}

// The traceback enters a cell in one of 7 states: 0 = H, 1 + c = after an X
// op whose cell had open/extend code c, 4 + c = after a Y op likewise.  The op
// taken at the cell depends only on the state and the cell's tie byte:
//   after X: H if the run was opened (c >= 1) and M attains H here, else X if
//            it could be extended (c <= 1), else H;
//   after Y: H if opened and M or X attains H here, else Y if extendable, else H;
//   in H: the smallest op attaining H.
// The state after the op determines the op (0: M, 1-3: X, 4-6: Y) and, with
// the cell's X or Y code, the next entry state.  next_table packs, for each of
// the 7 entry states, the next state in a 4-bit field, so one v_readlane and
// one bit-field extract advance the walk by one op.
__device__ inline uint32_t next_table(uint32_t b) {
  const uint32_t hc = b & 3u, xc = (b >> 2) & 3u, yc = (b >> 4) & 3u;
  const uint32_t nx = 1u + xc, ny = 4u + yc;
  const uint32_t n0 = 0u, n1 = nx, n2 = ny;
  const uint32_t nh = hc == 0u ? n0 : (hc == 1u ? n1 : n2);
  uint32_t t = nh;
#pragma unroll
  for (uint32_t c = 0; c < 3; ++c) {
    const uint32_t ox = (c >= 1u && hc == 0u) ? 0u : (c <= 1u ? 1u : hc);
    const uint32_t oy = (c >= 1u && hc <= 1u) ? hc : (c <= 1u ? 2u : hc);
    const uint32_t sx = ox == 0u ? n0 : (ox == 1u ? n1 : n2);
    const uint32_t sy = oy == 0u ? n0 : (oy == 1u ? n1 : n2);
    t |= sx << (4 * (1 + c));
    t |= sy << (4 * (4 + c));
  }
  return t;
}

// Window step per next state: M moves (-1, -1), X (-1, 0), Y (0, -1); in the
// window's lane numbering (lane q = cell (i - q / 8, j - q % 8)) that is +9,
// +8 or +1.  One 4-bit field per state.
constexpr uint32_t kWindowStep = 0x1118889u;
// Ops per window: after at most 7 ops the offset (di, dj) is still below 8 in
// both coordinates, so the lane index identifies it and no bound is checked.
constexpr int kWindowOps = 7;

__device__ inline int state_op(int sg) { return sg == 0 ? 0 : (sg <= 3 ? 1 : 2); }

// Entry states are shifted into a register one per op (the newest in lane 63)
// and stored as ops when 56 or more are pending: the q-th op from the end goes
// to ops[cap - 1 - q].
__device__ inline void ops_store(uint8_t* ops, int cap, int lane, int32_t acc, int k, int kst) {
  const int pend = k - kst;
  if (lane >= 64 - pend) ops[cap - 1 - (k - 64 + lane)] = (uint8_t)state_op(acc);
}

// Tie words of the strip the walk is on, from 16 x 64-word blocks staged in
// LDS on demand.
struct StageSource {
  const uint32_t* tbw;
  uint32_t* tbst;
  Stage st;
  int stride_s, T4;
  __device__ void cover(int lane, int s, int t4lo, int t4hi) {
    stage_cover(tbw, tbst, st, stride_s, T4, lane, s, t4lo, t4hi);
  }
  __device__ uint32_t word(int, int t4, int lc) const { return tbst[(t4 - st.t4a) * 64 + lc]; }
  __device__ void finish() {}
};

// Whole strips in LDS, copied by a helper wave (strip_loader) while the walk
// proceeds: strip s goes to buffer s & 1.  The walk waits for ready[b] == s
// and, leaving a strip, sets consumed[b] to it so the buffer can be refilled.
struct StripSource {
  const uint32_t* buf;
  int words;  // per strip
  int32_t* ready;
  int32_t* consumed;
  int32_t* fin;
  int64_t wait_ticks;
  int cur;
  DevStatus* st;
  int32_t* wsites;
  __device__ void cover(int, int s, int, int) {
    if (s == cur) return;
    if (cur >= 0)
      __hip_atomic_store(&consumed[cur & 1], cur, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    cur = s;
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(&ready[s & 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != s) {
      __builtin_amdgcn_s_sleep(1);
      // the loader always makes progress; the limit only guards a broken wait
      if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > wait_ticks) {
        if ((threadIdx.x & 63) == 0) wait_expired(st, wsites, WS_STRIP, s);
        break;
      }
    }
  }
  __device__ uint32_t word(int s, int t4, int lc) const {
    return buf[(s & 1) * words + t4 * 64 + lc];
  }
  __device__ void finish() {
    __hip_atomic_store(fin, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Helper wave of StripSource: copies strips sL, sL - 1, ... (each nchunks x
// 4 KB, contiguous) into the two LDS buffers with direct-to-LDS loads.
__device__ __forceinline__ void strip_loader(const uint32_t* tbw, uint32_t* buf, int words, int sL,
                             int32_t* ready, int32_t* consumed, int32_t* fin, int64_t wait_ticks,
                             DevStatus* st, int32_t* wsites, int lane) {
  for (int s = sL; s >= 0; --s) {
    const int b = s & 1;
    if (s <= sL - 2) {
      const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&consumed[b], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) !=
             s + 2) {
        if (__hip_atomic_load(fin, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
        __builtin_amdgcn_s_sleep(1);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > wait_ticks) {
          if (lane == 0) wait_expired(st, wsites, WS_LOADER, s);
          return;
        }
      }
    } else if (__hip_atomic_load(fin, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) {
      return;
    }
    const uint32_t* src = tbw + (int64_t)s * words + lane * 4;
    uint32_t* dst = buf + b * words;
    for (int q = 0; q < words; q += 256)
      __builtin_amdgcn_global_load_lds(src + q, (__attribute__((address_space(3))) void*)(dst + q),
                                       16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(&ready[b], s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Writes the op string to ops[cap - n .. cap); returns n.  Whole wave.
template <typename Src>
__device__ __forceinline__ int traceback(Src& src, uint8_t* ops, int W1, int W2, int lane) {
  const int cap = W1 + W2;
  int32_t acc = 0;
  int k = 0, kst = 0;
  int i = W1, j = W2;
  int sg = 0;
  const int qi = lane >> 3, qj = lane & 7;
  while (i > 0 && j > 0) {
    // window of the cells (i - qi, j - qj) of this strip, from the staged block
    const int s = (i - 1) >> 6;
    const int lo = 64 * s + 1, l = (i - 1) & 63;
    const int ilow = max(lo, i - 7);
    const int t_hi = j - 1 + l;
    const int t_lo = max(0, j - 8) + ((ilow - 1) & 63);
    src.cover(lane, s, t_lo >> 2, t_hi >> 2);
    const int ci = i - qi, cj = j - qj;
    uint32_t byte = 0;
    if (ci >= lo && cj >= 1) {
      const int lc = (ci - 1) & 63, t = cj - 1 + lc;
      const uint32_t word = src.word(s, t >> 2, lc);
      byte = (word >> (8 * (t & 3))) & 0xffu;
    }
    const int32_t v = (int32_t)next_table(byte);
    if (k - kst > 64 - kWindowOps) {
      ops_store(ops, cap, lane, acc, k, kst);
      kst = k;
    }
    // the window's cells outside the strip or left of column 1 are never
    // reached: at most l + 1 row steps and j column steps
    const int n = min(kWindowOps, min(l + 1, j));
    // the window's states are collected in a scalar, 3 bits per op, and
    // appended to acc once: its lanes move down by n and lanes 64 - n .. 63
    // take the n new states (the newest in lane 63)
    int idx = 0;
    uint32_t packed = 0;
    auto walk = [&](int r) {
      const uint32_t tab = (uint32_t)__builtin_amdgcn_readlane(v, idx);
      sg = (int)((tab >> (4 * sg)) & 7u);
      idx += (int)((kWindowStep >> (4 * sg)) & 15u);
      packed |= (uint32_t)sg << (3 * r);
    };
    if (n == kWindowOps) {
      // a full window (the common case) needs no per-op count test
#pragma unroll
      for (int r = 0; r < kWindowOps; ++r) walk(r);
    } else {
#pragma unroll
      for (int r = 0; r < kWindowOps; ++r) {
        if (r >= n) break;
        walk(r);
      }
    }
    {
      const int32_t moved = __builtin_amdgcn_ds_bpermute(min(lane + n, 63) << 2, acc);
      const int rr = lane - (64 - n);
      acc = rr >= 0 ? (int32_t)((packed >> (3 * rr)) & 7u) : moved;
    }
    k += n;
    i -= idx >> 3;
    j -= idx & 7;
  }
  src.finish();
  for (; i > 0; --i) {
    if (k - kst == 64) {
      ops_store(ops, cap, lane, acc, k, kst);
      kst = k;
    }
    acc = __builtin_amdgcn_update_dpp(1, acc, 0x130, 0xf, 0xf, false);
    ++k;
  }
  for (; j > 0; --j) {
    if (k - kst == 64) {
      ops_store(ops, cap, lane, acc, k, kst);
      kst = k;
    }
    acc = __builtin_amdgcn_update_dpp(4, acc, 0x130, 0xf, 0xf, false);
    ++k;
  }
  ops_store(ops, cap, lane, acc, k, kst);
  return k;
}

// ---------------------------------------------------------------- merge
// Column q of the new profile is P1[ii] + P2[jj] (the parts its op consumes),
// where ii and jj count the earlier ops that consume a P1 / P2 column.  The
// counts come from one ballot per 64 ops and a scan over those groups; then
// each lane writes one whole column (rows are 8-byte aligned: A u16 counts
// at a multiple of A elements, A in {4, 20}).
template <int A>
struct MergeRow {
  static constexpr int NW = A / 4;  // uint2 words per column
  uint2 a[NW], b[NW];
  int q, ii, jj;
  bool c1, c2;
};

template <int A>
__device__ inline void merge_load(MergeRow<A>& r, const uint8_t* ops, int base, int nops, int g,
                                  const int32_t* gcnt, const uint2* __restrict__ P1,
                                  const uint2* __restrict__ P2, int lane) {
  constexpr int NW = MergeRow<A>::NW;
  r.q = 64 * g + lane;
  const bool in = r.q < nops;
  const int op = in ? ops[base + r.q] : 3;
  r.c1 = in && op != 2;
  r.c2 = in && op != 1;
  const uint64_t b1 = __ballot(r.c1), b2 = __ballot(r.c2);
  const uint64_t below = (1ull << lane) - 1ull;
  const int pre = gcnt[g];
  r.ii = (pre & 0xffff) + __popcll(b1 & below);
  r.jj = (pre >> 16) + __popcll(b2 & below);
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    r.a[m] = r.c1 ? P1[(int64_t)r.ii * NW + m] : make_uint2(0u, 0u);
    r.b[m] = r.c2 ? P2[(int64_t)r.jj * NW + m] : make_uint2(0u, 0u);
  }
}

template <int A>
__device__ inline void merge_store(const MergeRow<A>& r, int nops, uint2* __restrict__ Pout,
                                   int32_t* up1, int32_t* up2) {
  constexpr int NW = MergeRow<A>::NW;
  if (r.q < nops) {
    // counts add per 16-bit half without carries (n1 + n2 < 65536)
#pragma unroll
    for (int m = 0; m < NW; ++m)
      Pout[(int64_t)r.q * NW + m] = make_uint2(r.a[m].x + r.b[m].x, r.a[m].y + r.b[m].y);
  }
  if (r.c1 && up1) up1[r.ii] = r.q;
  if (r.c2 && up2) up2[r.jj] = r.q;
}

template <int A>
__device__ __forceinline__ void merge(const uint8_t* ops, int base, int nops, const uint16_t* P1,
                      const uint16_t* P2, uint16_t* Pout, int32_t* up1, int32_t* up2,
                      int32_t* gcnt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ng = (nops + 63) >> 6;
  for (int g = wave; g < ng; g += kWaves) {
    const int q = 64 * g + lane;
    const int op = q < nops ? ops[base + q] : 3;
    const uint64_t b1 = __ballot(q < nops && op != 2), b2 = __ballot(q < nops && op != 1);
    if (lane == 0) gcnt[g] = __popcll(b1) | (__popcll(b2) << 16);
  }
  __syncthreads();
  if (wave == 0) {
    // exclusive scan of the packed (P1, P2) counts; halves stay below 2^16
    int carry = 0;
    for (int g0 = 0; g0 < ng; g0 += 64) {
      const int g = g0 + lane;
      const int v = g < ng ? gcnt[g] : 0;
      int x = v;
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      if (g < ng) gcnt[g] = carry + x - v;
      carry += __shfl(x, 63, 64);
    }
  }
  __syncthreads();
  const uint2* p1 = reinterpret_cast<const uint2*>(P1);
  const uint2* p2 = reinterpret_cast<const uint2*>(P2);
  uint2* po = reinterpret_cast<uint2*>(Pout);
  for (int g = wave; g < ng; g += 2 * kWaves) {
    MergeRow<A> r0, r1;
    merge_load<A>(r0, ops, base, nops, g, gcnt, p1, p2, lane);
    const bool two = g + kWaves < ng;
    if (two) merge_load<A>(r1, ops, base, nops, g + kWaves, gcnt, p1, p2, lane);
    merge_store<A>(r0, nops, po, up1, up2);
    if (two) merge_store<A>(r1, nops, po, up1, up2);
  }
}

// ---------------------------------------------------------------- job hand-off
// Appends ready job j to the queue (one thread).
__device__ inline void push_job(const EngineArgs& a, int j) {
  __threadfence();
  const int pos = atomicAdd(a.queue_tail, 1);
  if (pos >= a.queue_cap) {  // cannot happen: at most 1 + kMaxHelpers tickets per merge
    raise_error(a.st, SAD_E_CAPACITY, pos, W_ENGINE);
    return;
  }
  __hip_atomic_store(&a.queue[pos], j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();
  __hip_atomic_store(&a.queue_flag[pos], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// A finished job releases its share of its parent's count if the parent
// already exists; otherwise the parent's creation does it (one thread).  If
// this release makes the parent ready and `keep` is set, the parent is
// returned for the caller to run next instead of being queued (else -1).
__device__ inline int job_finished(const EngineArgs& a, int job, bool keep) {
  const int old = atomicCAS(&a.job_link[job], 0, 1);
  if (old != 2) return -1;
  __threadfence();
  const int nx = __hip_atomic_load(&a.job_next[job], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (atomicSub(&a.job_pending[nx], 1) == 1) {
    if (keep) return nx;
    push_job(a, nx);
  }
  return -1;
}

// Creates the job of merge `step` of group g (cluster ids ia < ib, leaves
// below n) as soon as UPGMA decides it (one thread).  Its count starts at one
// per internal child plus one for the creation itself.
__device__ inline void create_job(const EngineArgs& a, int g0, int n, int step, int ia, int ib) {
  const int N = a.up_N;
  const int s = g0 + step;
  const int na = ia < n ? g0 + ia : N + g0 + (ia - n);
  const int nb = ib < n ? g0 + ib : N + g0 + (ib - n);
  a.job_a[s] = na;
  a.job_b[s] = nb;
  a.job_out[s] = N + s;
  a.node_parent[na] = N + s;
  a.node_parent[nb] = N + s;
  __hip_atomic_store(&a.job_pending[s], 1 + (ia >= n) + (ib >= n), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();
  const int kids[2] = {ia, ib};
  for (int q = 0; q < 2; ++q) {
    if (kids[q] < n) continue;
    const int c = g0 + (kids[q] - n);
    __hip_atomic_store(&a.job_next[c], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    if (atomicCAS(&a.job_link[c], 0, 2) == 1) atomicSub(&a.job_pending[s], 1);
  }
  if (atomicSub(&a.job_pending[s], 1) == 1) push_job(a, s);
}

// In the MFMA kernel, groups up to kFusedLdsN keep the triangle of 64-bit pair
// sums in the score ring's LDS and the five cluster arrays in the traceback
// staging block; larger ones, up to kFusedMaxN, and every group of the
// vector-ALU kernel (whose ring is too small for the triangle) keep the sums
// in their n x n area of the global work array (a.up_Sw at the group's matrix
// offset), the cluster arrays and each cluster's best pair sum in `big` (the
// MFMA kernel's ring, or an LDS block of their own).  The merge list
// (2 (n - 1) ints) fits the op buffer.
constexpr int kFusedLdsN = 182;
constexpr int kFusedMaxN = 600;
static_assert(kFusedMaxN <= kUpgmaW64MaxN, "in-launch trees compare 64-bit cross products");

// The steps of the tree of group g on wave 0, the jobs of its merges made by
// wave 1 as they are decided (see fused_tree).  Sums in LDS (TriS): the
// one-wave steps; in HBM (FullS, bsum non-null): the steps with cached best
// sums.
template <typename St>
__device__ void fused_tree_steps(const EngineArgs& a, int g, int g0, int n, const St& S, int32_t* id,
                                 int32_t* sz, int32_t* active, int32_t* best, int32_t* rec,
                                 uint64_t* bsum, int32_t* mlist, int32_t* mcount) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // (kFusedMaxN <= kUpgmaW64MaxN: 64-bit cross products are exact)
  upgma_init_best<true>(S, n, id, sz, active, best);
  __syncthreads();
  if (wave == 0) {
    // the merge steps; each decided merge is listed for wave 1
    auto listed = [&](int step, int ia, int ib) {
      mlist[2 * step] = ia;
      mlist[2 * step + 1] = ib;
      __hip_atomic_store(mcount, step + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    bool ok;
    if constexpr (std::is_same<St, FullS>::value)
      ok = upgma_steps_hbm<true, 4>(S, n, id, sz, active, best, bsum, rec, g, a.st, listed);
    else
      ok = upgma_steps<true, 1>(S, n, id, sz, active, best, rec, g, a.st, listed);
    if (!ok && lane == 0)
      __hip_atomic_store(mcount, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else if (wave == 1) {
    // jobs for the listed merges, up to 64 at a time (one lane each), so that
    // their fences and atomics are paid once per batch
    int k0 = 0;
    uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    while (k0 < n - 1) {
      const int avail = __hip_atomic_load(mcount, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (avail < 0) break;
      if (avail == k0) {
        __builtin_amdgcn_s_sleep(1);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
          if (lane == 0) wait_expired(a.st, a.wait_sites, WS_TREE, g);
          break;
        }
        continue;
      }
      const int kb = min(avail, k0 + 64);
      const int k = k0 + lane;
      if (k < kb) {
        const int ia = mlist[2 * k], ib = mlist[2 * k + 1];
        // the merge list output (kept off the tree wave's path)
        a.up_merges[2 * ((int64_t)g0 + k)] = ia;
        a.up_merges[2 * ((int64_t)g0 + k) + 1] = ib;
        create_job(a, g0, n, k, ia, ib);
      }
      k0 = kb;
      t_start = __builtin_amdgcn_s_memrealtime();
    }
  }
  __syncthreads();
}

// UPGMA of group g by the whole workgroup.
template <bool MFMA>
__device__ __forceinline__ void fused_tree(const EngineArgs& a, int g, uint32_t* ring, uint32_t* tbst,
                           int32_t* big, int32_t* mlist, int32_t* mcount) {
  const int g0 = a.up_group_off[g], n = a.up_group_off[g + 1] - g0;
  if (n <= 1) return;
  const int tid = threadIdx.x;
  const bool in_lds = MFMA && n <= kFusedLdsN;
  int32_t* id = in_lds ? reinterpret_cast<int32_t*>(tbst) : big;
  int32_t* sz = id + n;
  int32_t* active = id + 2 * n;
  int32_t* best = id + 3 * n;
  int32_t* rec = id + 4 * n;
  // the best pair sums of the HBM branch, 8-byte aligned after the arrays
  uint64_t* bsum = reinterpret_cast<uint64_t*>(big + ((5 * n + 1) & ~1));
  for (int x = tid; x < n; x += kThreads) {
    id[x] = x;
    sz[x] = 1;
    active[x] = 1;
  }
  const uint32_t* Fg = a.up_F + a.up_fm_off[g];
  if (tid == 0) *mcount = 0;
  if (!in_lds) {
    // sums in the group's area of the global work array (both halves)
    const FullS S{a.up_Sw + a.up_fm_off[g], n};
    for (int64_t q = tid; q < (int64_t)n * n; q += kThreads) S.t[q] = Fg[q];
    __threadfence_block();
    __syncthreads();
    fused_tree_steps(a, g, g0, n, S, id, sz, active, best, rec, bsum, mlist, mcount);
    return;
  }
  if constexpr (!MFMA) return;  // (every group of this kernel takes the branch above)
  uint64_t* tri = reinterpret_cast<uint64_t*>(ring);
  for (int64_t q = tid; q < (int64_t)n * n; q += kThreads) {
    const int x = (int)(q / n), y = (int)(q % n);
    if (x < y) tri[x * n - x * (x + 1) / 2 + y - x - 1] = Fg[q];
  }
  __threadfence_block();
  __syncthreads();
  fused_tree_steps(a, g, g0, n, TriS{tri, n}, id, sz, active, best, rec, nullptr, mlist, mcount);
}


// ---------------------------------------------------------------- kernel
template <int A, bool MFMA>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MFMA ? 1 : 2))) void
engine_kernel(EngineArgs a) {
  constexpr int CW = ColWords<A>::value;
  constexpr int kRingWords = MFMA ? kScWords : (kColRing + kColRingPad) * CW;  // per wave
  __shared__ __attribute__((aligned(16))) uint32_t ring[kWaves * kRingWords];
  __shared__ int32_t S32[MFMA ? A * 32 : 1];
  __shared__ uint32_t tbst[kStageT4 * 64];
  __shared__ __attribute__((aligned(16))) uint8_t ops[2 * kMaxWidth];
  __shared__ int32_t Ssh[A * A];
  __shared__ int32_t prog[kMaxStrips];
  __shared__ int32_t gcnt[2 * kMaxWidth / 64];
  __shared__ int32_t tbctl[5];  // strip staging: ready[2], consumed[2], fin
  __shared__ int32_t glist[kCoopMaxGroups];  // groups of a cooperative merge claimed here
  __shared__ int32_t gstate[2];              // groups claimed, no group left
  // per wave: the row above of the current chunk, (H, X) per step (the MFMA
  // kernel's 32-bit strips put 64 lanes' pairs of 32-bit values, the other
  // kernel's strips up to 64 pairs of 64-bit values)
  constexpr int kRowWords = MFMA ? 128 : 256;
  __shared__ __attribute__((aligned(16))) int32_t rowbuf[kWaves * kRowWords];
  __shared__ JobInfo J;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  for (int q = tid; q < A * A; q += kThreads) Ssh[q] = a.S[q];
  if constexpr (MFMA) {
    // S with its columns zero-padded to 32 (the K extent of the tile products)
    for (int q = tid; q < A * 32; q += kThreads) S32[q] = (q % 32) < A ? a.S[(q / 32) * A + q % 32] : 0;
  }
  uint32_t* tbw = a.tb + (int64_t)blockIdx.x * a.tb_words_per_wg;
  int32_t* links = a.bnd + (int64_t)blockIdx.x * a.link_words_per_wg;
  uint32_t* myring = ring + wave * kRingWords;
  int32_t* myrow = rowbuf + wave * kRowWords;
  __syncthreads();

  if constexpr (MFMA) {
    static_assert(5 * kFusedLdsN <= kStageT4 * 64, "cluster arrays fit the staging block");
    static_assert((int64_t)kFusedLdsN * (kFusedLdsN - 1) / 2 * 8 <=
                      (int64_t)kWaves * kRingWords * 4, "pair sums fit the score ring");
    static_assert(7 * kFusedMaxN + 2 <= kWaves * kRingWords,
                  "cluster arrays and best sums fit the score ring");
  }
  static_assert(kUpgmaThreads == kThreads, "tree phase uses the engine's workgroup shape");
  static_assert(2 * (kFusedMaxN - 1) * 4 <= 2 * kMaxWidth, "merge list fits the ops buffer");
  // the vector-ALU kernel's cluster arrays and best sums of an in-launch tree
  __shared__ __attribute__((aligned(8))) int32_t tree_arrays[MFMA ? 1 : 7 * kFusedMaxN + 2];
  __shared__ int32_t umcount, ugrp;
  // guide trees first; their merges become jobs for the other workgroups
  if (a.up_ngroups > 0) {
    int32_t* big = MFMA ? reinterpret_cast<int32_t*>(ring) : tree_arrays;
    for (;;) {
      if (tid == 0) ugrp = atomicAdd(a.up_next, 1);
      __syncthreads();
      const int g = ugrp;
      __syncthreads();
      if (g >= a.up_ngroups) break;
      fused_tree<MFMA>(a, g, ring, tbst, big, reinterpret_cast<int32_t*>(ops), &umcount);
    }
  }
  uint64_t tk0 = 0, tk1 = 0, tk2 = 0, tk3 = 0, tk35 = 0;  // phase timestamps (thread 0)
  // (thread 0) a merge that this workgroup's last job made ready: it runs
  // next without a trip through the queue.  Only in the batched kernel, whose
  // idle workgroups leave on the `finished` flag rather than on a count of
  // queued jobs.
  int keep_job = -1;
  for (;;) {
    // ---- fetch a ready job (thread 0) and describe it to the workgroup
    if (tid == 0) {
      tk0 = __builtin_amdgcn_s_memrealtime();
      J.job = -1;
      J.helper = 0;
      // the batched kernel's queue also carries helper tickets, so its slots
      // outnumber the merges: workgroups leave when every merge is done
      const int bound = MFMA ? a.queue_cap : a.njobs;
      const int slot = keep_job >= 0 ? -1 : atomicAdd(a.queue_head, 1);
      J.slot = slot;
      if (keep_job >= 0) {
        // the other child's results were released before its count was
        // (fence, then the count); this fence orders the reads after ours
        __threadfence();
        J.job = keep_job;
        keep_job = -1;
      } else if (slot < bound) {
        const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
        bool ok = true;
        // relaxed polls (an agent-scope acquire invalidates cache lines that
        // the working workgroups use); the fence below orders the job's reads
        while (__hip_atomic_load(&a.queue_flag[slot], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) == 0) {
          if (MFMA && __hip_atomic_load(a.finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
          if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
            wait_expired(a.st, a.wait_sites, WS_QUEUE, slot);
            ok = false;
            break;
          }
        }
        if (ok) {
          __threadfence();
          const int ticket =
              __hip_atomic_load(&a.queue[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          J.job = ticket & (kHelperTicket - 1);
          J.helper = (ticket & kHelperTicket) ? 1 : 0;
        }
      }
      const int job = J.job;
      if (job >= 0) {
        const int na = a.job_a[job], nb = a.job_b[job];
        J.na = na;
        J.nb = nb;
        J.out = a.job_out[job];
        const int W1 = a.node_W[na], W2 = a.node_W[nb];
        const int n1 = a.node_n[na], n2 = a.node_n[nb];
        J.W1 = W1;
        J.W2 = W2;
        J.n1 = n1;
        J.n2 = n2;
        const int64_t G = (int64_t)n1 * n2;
        const int64_t unit = max((int64_t)max(a.smax, a.go), (int64_t)1);
        // static bound of every DP value; 32-bit DP below 2^29, 64-bit DP up
        // to kBound64 (beyond it the merge is rejected, as by the oracle)
        const bool over64 =
            (double)(W1 + W2 + 2) * (double)G * (double)unit >= (double)kBound64;
        const int64_t bound = over64 ? kBound64 : (int64_t)(W1 + W2 + 2) * G * unit;
        const int wide = bound >= (1ll << 29) ? 1 : 0;
        // column scores are int32 (|s| <= n1 n2 max|S|); the tile products need
        // |U| <= n1 max|S| within three signed base-256 digits
        const bool score_over = (double)G * (double)max(a.smax, 1) >= 2147483647.0 ||
                                (int64_t)n1 * a.smax > 8355711;
        const int nstrips = (W1 + 63) >> 6;
        const int nchunks = (W2 + 63 + 63) >> 6;
        J.nstrips = nstrips;
        J.nchunks = nchunks;
        const int64_t tb_need = (int64_t)nstrips * nchunks * 16 * 64;
        const int cap = W1 + W2;
        int err = 0;
        if (J.helper) {
          // a helper only runs strips; its owner checked the merge already
        } else if (W1 > kMaxWidth || W2 > kMaxWidth) {
          err = 1;
          raise_error(a.st, SAD_E_CAPACITY, cap, W_ENGINE_WIDTH);
        } else if (over64 || score_over) {
          err = 1;
          raise_error(a.st, SAD_E_OVERFLOW, bound, W_ENGINE_BOUND);
        } else if (tb_need > a.tb_words_per_wg) {
          err = 1;
          raise_error(a.st, SAD_E_CAPACITY, tb_need, W_ENGINE_TB);
        } else if (nstrips > a.link_rows + 1 || (W2 + 1) * (wide ? 2 : 1) > a.link_stride) {
          err = 1;
          raise_error(a.st, SAD_E_CAPACITY, (int64_t)max(W1, W2), W_ENGINE_LINK);
        } else if (n1 + n2 > 65535) {
          err = 1;
          raise_error(a.st, SAD_E_CAPACITY, n1 + n2, W_ENGINE);
        }
        long long prof_off = 0, up_off = 0;
        if (!err && !J.helper) {
          prof_off = (long long)atomicAdd(a.prof_top, (unsigned long long)cap * A);
          up_off = (long long)atomicAdd(a.up_top, (unsigned long long)cap);
          if (prof_off + (long long)cap * A > a.prof_cap) {
            raise_error(a.st, SAD_E_CAPACITY, prof_off + (long long)cap * A, W_ENGINE_POOL);
            err = 1;
          } else if (up_off + cap > a.up_cap) {
            raise_error(a.st, SAD_E_CAPACITY, up_off + cap, W_ENGINE_POOL);
            err = 1;
          }
        }
        J.prof_off = prof_off;
        J.up_off = up_off;
        J.err = err;
        J.abort = 0;
        J.o = G * a.go;
        J.e = G * a.ge;
        J.wide = wide;
        J.packed = ((int64_t)n1 * a.smax <= 32767 && n2 <= 32767) ? 1 : 0;
        // signed base-256 digits of U (|U| <= n1 smax), base-128 digits of counts
        const int64_t umax = (int64_t)n1 * a.smax;
        J.nd_u = umax <= 127 ? 1 : (umax <= 32639 ? 2 : 3);
        J.nd_c = n2 <= 127 ? 1 : (n2 <= 16383 ? 2 : 3);
        J.final_score = 0;
        J.coop = 0;
        J.owner = (int)blockIdx.x;
        J.tag = 0;
        J.ltag = 0;
        if constexpr (MFMA) {
          if (!err && !wide) {
            // 16 fresh tags for this workgroup's own rows (only its thread 0
            // touches its counter)
            int32_t* head = a.trow + (int64_t)blockIdx.x * a.trow_words_per_wg;
            J.ltag = (uint32_t)head[0] + 1u;
            head[0] = (int32_t)(J.ltag + 15u);
          }
          const int ngroups = (nstrips + kCoopGroupStrips - 1) / kCoopGroupStrips;
          // workgroups waiting for a ticket that no merge has filled yet
          const int idle = __hip_atomic_load(a.queue_head, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) -
                           __hip_atomic_load(a.queue_tail, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
          if (J.helper) {
            J.coop = 1;
            J.owner = __hip_atomic_load(&a.coop_owner[job], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) - 1;
            J.tag = (uint32_t)__hip_atomic_load(&a.coop_tag[job], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            gstate[0] = 0;
            gstate[1] = 0;
          } else if (!err && !wide && W1 > 0 && W2 > 0 && ngroups > 1 && idle > 0 &&
                     (int)blockIdx.x < a.coop_wgs) {
            // cooperative merge while workgroups wait idle: a fresh tag for
            // its boundary rows, its group and strip counters, then helper
            // tickets (the owner runs group 0 and claims further groups like
            // any helper)
            J.coop = 1;
            int32_t* area = a.coop_buf + (int64_t)blockIdx.x * a.coop_words_per_wg;
            // only this workgroup's thread 0 touches its counter: no RMW
            // atomic on uncached memory needed
            J.tag = (uint32_t)__hip_atomic_load(&area[0], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) + 1u;
            __hip_atomic_store(&area[0], (int32_t)J.tag, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            a.coop_tag[job] = (int32_t)J.tag;
            a.coop_next[job] = 1;
            a.coop_strips[job] = 0;
            a.coop_owner[job] = (int)blockIdx.x + 1;
            glist[0] = 0;
            gstate[0] = 1;
            gstate[1] = 0;
            __builtin_amdgcn_s_waitcnt(0);
            __threadfence();
            const int nh = min(min(ngroups - 1, kMaxHelpers), idle);
            for (int h = 0; h < nh; ++h) push_job(a, job | kHelperTicket);
          }
        }
      }
    }
    __syncthreads();
    const int job = J.job;
    if (job < 0) break;
    if (tid == 0) tk1 = __builtin_amdgcn_s_memrealtime();
    const int na = J.na, nb = J.nb, out = J.out;
    const int W1 = J.W1, W2 = J.W2;
    const uint16_t* P1 = a.prof_pool + a.node_prof[na];
    const uint16_t* P2 = a.prof_pool + a.node_prof[nb];
    int32_t* up1 = a.up_pool + a.node_up[na];
    int32_t* up2 = a.up_pool + a.node_up[nb];
    const int64_t oo = a.job_ops_off[job];

    if (!J.err) {
      for (int L = tid; L < kMaxStrips; L += kThreads) prog[L] = 0;
      if (tid < 5) tbctl[tid] = tid < 4 ? -1 : 0;
      __syncthreads();
      if (W1 > 0 && W2 > 0) {
        if constexpr (MFMA) {
          if (J.wide) {
            for (int s = wave; s < J.nstrips; s += kWaves) {
              const StripLinks<int64_t> L = strip_links<int64_t>(a, J, s, prog, links);
              if (!dp_strip_mfma<A, int64_t>(a, J, s, lane, myring, tbw, L, S32, P1, P2)) break;
            }
          } else {
            // alone or cooperative (the tagged rows hold 32-bit values)
            if (a.chunk == 16)
              tagged_dp<A, 16>(a, J, wave, lane, myring, S32, P1, P2, glist, gstate, myrow);
            else
              tagged_dp<A, 32>(a, J, wave, lane, myring, S32, P1, P2, glist, gstate, myrow);
          }
        } else if (J.wide) {
          for (int s = wave; s < J.nstrips; s += kWaves)
            if (!dp_strip<A, false, int64_t>(a, J, s, lane, myring, prog, tbw, links, Ssh, P1, P2,
                                             reinterpret_cast<int64_t*>(myrow)))
              break;
        } else if (J.packed) {
          for (int s = wave; s < J.nstrips; s += kWaves)
            if (!dp_strip<A, true, int32_t>(a, J, s, lane, myring, prog, tbw, links, Ssh, P1, P2,
                                            myrow))
              break;
        } else {
          for (int s = wave; s < J.nstrips; s += kWaves)
            if (!dp_strip<A, false, int32_t>(a, J, s, lane, myring, prog, tbw, links, Ssh, P1, P2,
                                             myrow))
              break;
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // tie bytes stored before the barrier
      __threadfence_block();
      __syncthreads();
      if (J.abort) {
        if (tid == 0) J.err = 1;
        __syncthreads();
      }
    }
    // a helper's part ends with its strips; the rest is the owner's
    if (!J.helper) {
      if (J.coop && !J.err) {
        // every strip of the merge done (some on other workgroups), their tie
        // bytes and H(W1, W2) visible here
        if (tid == 0) {
          const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
          while (__hip_atomic_load(&a.coop_strips[job], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) < J.nstrips) {
            __builtin_amdgcn_s_sleep(2);
            if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
              wait_expired(a.st, a.wait_sites, WS_COOP, job);
              J.err = 1;
              break;
            }
          }
          __threadfence();
          J.final_score =
              __hip_atomic_load(&a.coop_score[job], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
      }
      if (tid == 0) tk2 = __builtin_amdgcn_s_memrealtime();
      if (!J.err) {
        const int nchunks = J.nchunks;
        const int sw = nchunks * 16 * 64;  // tie words per strip
        bool strips_in_lds = false;
        if constexpr (MFMA) strips_in_lds = 2 * sw <= kWaves * kRingWords;
        if (strips_in_lds) {
          // wave 1 streams whole strips into the (idle) score ring
          if (wave == 0) {
            StripSource src{ring, sw, tbctl, tbctl + 2, tbctl + 4, a.wait_ticks, -1, a.st,
                            a.wait_sites};
            const int n = traceback(src, ops, W1, W2, lane);
            if (lane == 0) J.nops = n;
          } else if (wave == 1) {
            strip_loader(tbw, ring, sw, (W1 - 1) >> 6, tbctl, tbctl + 2, tbctl + 4, a.wait_ticks,
                         a.st, a.wait_sites, lane);
          }
        } else if (wave == 0) {
          StageSource src{tbw, tbst, Stage{-1, 0}, sw, nchunks * 16};
          const int n = traceback(src, ops, W1, W2, lane);
          if (lane == 0) J.nops = n;
        }
        __syncthreads();
        if (tid == 0) tk3 = __builtin_amdgcn_s_memrealtime();
        const int nops = J.nops;
        const int base = W1 + W2 - nops;
        // jobs that export their op string (refinement) leave the column maps
        // alone: several of them share the same second node
        merge<A>(ops, base, nops, P1, P2, a.prof_pool + J.prof_off, oo >= 0 ? nullptr : up1,
                 oo >= 0 ? nullptr : up2, gcnt);
        if (oo >= 0)
          for (int q = tid; q < nops; q += kThreads) a.ops_out[oo + q] = ops[base + q];
        if (tid == 0) {
          int64_t score = J.final_score;
          if (W1 == 0 || W2 == 0) {
            const int w = W1 + W2;
            score = w == 0 ? 0 : -(J.o + (int64_t)(w - 1) * J.e);
          }
          a.node_W[out] = nops;
          a.node_n[out] = J.n1 + J.n2;
          a.node_prof[out] = J.prof_off;
          a.node_up[out] = J.up_off;
          a.job_score[job] = score;
          a.job_cells[job] = (int64_t)W1 * W2;
        }
      } else {
        // keep the DAG consistent and every later access in bounds
        if (oo < 0) {
          for (int q = tid; q < W1; q += kThreads) up1[q] = 0;
          for (int q = tid; q < W2; q += kThreads) up2[q] = 0;
        }
        if (tid == 0) {
          a.node_W[out] = 0;
          a.node_n[out] = J.n1 + J.n2;
          a.node_prof[out] = 0;
          a.node_up[out] = 0;
          a.job_score[job] = 0;
          a.job_cells[job] = (int64_t)W1 * W2;
        }
      }
      __syncthreads();
      if (tid == 0) tk35 = __builtin_amdgcn_s_memrealtime();
      __threadfence();
      __syncthreads();
      if (tid == 0 && a.phase_acc) {
        const uint64_t tk4 = __builtin_amdgcn_s_memrealtime();
        if (tk3 < tk2) tk3 = tk2;
        atomicAdd(&a.phase_acc[0], (unsigned long long)(tk1 - tk0));
        atomicAdd(&a.phase_acc[1], (unsigned long long)(tk2 - tk1));
        atomicAdd(&a.phase_acc[2], (unsigned long long)(tk3 - tk2));
        atomicAdd(&a.phase_acc[3], (unsigned long long)(tk35 - tk3));
        atomicAdd(&a.phase_acc[4], 1ull);
        atomicAdd(&a.phase_acc[5], (unsigned long long)(tk4 - tk35));
        if (a.job_rec && job < a.nrec) {
          long long* r = a.job_rec + (int64_t)job * 8;
          // W1; cooperative flag; groups the owner ran itself (LDS claim count)
          r[0] = (long long)W1 | ((long long)J.coop << 32) |
                 ((long long)(J.coop ? gstate[0] : 0) << 40);
          r[1] = W2;
          r[2] = J.err ? 0 : J.nops;
          r[3] = (long long)tk0;
          r[4] = (long long)tk1;
          r[5] = (long long)tk2;
          r[6] = (long long)tk3;
          r[7] = (long long)tk35;
        }
      }
      if (tid == 0 && !a.no_push) keep_job = job_finished(a, job, MFMA);
      if constexpr (MFMA) {
        if (tid == 0 && atomicAdd(a.jobs_done, 1) == a.njobs - 1)
          __hip_atomic_store(a.finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }  // owner
    __syncthreads();
  }
}

int engine_fused_max_group() { return kFusedMaxN; }
int engine_fused_lds_group() { return kFusedLdsN; }

int engine_workgroups() {
  int per_cu = kEngineWGPerCU;
  if (const char* env = getenv("SAD_ENGINE_WGS_PER_CU")) {
    const int v = atoi(env);
    if (v >= 1 && v <= 8) per_cu = v;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  if (cus <= 0) cus = 256;
  return cus * per_cu;
}

void launch_engine(const EngineArgs& a, int nwg, hipStream_t stream) {
  if (a.njobs <= 0 || nwg <= 0) return;
  const bool mfma = a.mode == SAD_BATCHED_MFMA;
  if (a.A == 20) {
    if (mfma) engine_kernel<20, true><<<nwg, kThreads, 0, stream>>>(a);
    else engine_kernel<20, false><<<nwg, kThreads, 0, stream>>>(a);
  } else {
    if (mfma) engine_kernel<4, true><<<nwg, kThreads, 0, stream>>>(a);
    else engine_kernel<4, false><<<nwg, kThreads, 0, stream>>>(a);
  }
}

}  // namespace sad
