// k-mer stage kernels (paper Section 2 "k-mer Rank" and Section 2.3.1):
// input validation, per-sequence sorted k-mer lists, pair sums
// c_ij = sum_tau min(n_i(tau), n_j(tau)) against an LDS-resident histogram,
// the fixed point F = floor(c 2^31 / d), and the per-chunk rank sort.
#include "sad_internal.h"

namespace sad {

// ------------------------------------------------------------------ validation

__global__ void validate_lengths_kernel(const int64_t* __restrict__ off, int n, int64_t total,
                                        int max_len, int k, DevStatus* st) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    if (off[0] != 0 || off[n] != total) raise_error(st, SAD_E_INVAL, off[n], W_VALIDATE);
  }
  if (i >= n) return;
  int64_t L = off[i + 1] - off[i];
  if (L < k || L > max_len || L > kMaxLen) raise_error(st, SAD_E_INVAL, i, W_VALIDATE);
}

__global__ void validate_codes_kernel(const uint8_t* __restrict__ codes, int64_t total, int A,
                                      DevStatus* st) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride)
    if (codes[t] >= A) raise_error(st, SAD_E_INVAL, t, W_VALIDATE);
}

void launch_validate(const sad_seqs& s, int k, DevStatus* st, hipStream_t stream) {
  int n = s.n;
  validate_lengths_kernel<<<(n + 256) / 256, 256, 0, stream>>>(s.d_offsets, n, s.total_len,
                                                              s.max_len, k, st);
  int64_t blocks = (s.total_len + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  validate_codes_kernel<<<(int)blocks, 256, 0, stream>>>(s.d_codes, s.total_len, s.alphabet, st);
}

// ------------------------------------------------------------------ k-mer lists
// One 256-thread workgroup per sequence: k-mer codes into LDS, bitonic sort,
// run-length compaction to (tau << 16 | count) entries in ascending tau.

constexpr int kListThreads = 256;

__global__ __launch_bounds__(kListThreads) void kmer_list_kernel(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ off, int A, int k,
    uint32_t* __restrict__ entries, int32_t* __restrict__ nu) {
  __shared__ uint32_t keys[kMaxLen];
  __shared__ int32_t seg_base[kListThreads + 1];
  const int seq = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t base = off[seq];
  const int L = (int)(off[seq + 1] - base);
  const int m = L - k + 1;
  if (m <= 0) {
    if (tid == 0) nu[seq] = 0;
    return;
  }
  int P = 1;
  while (P < m) P <<= 1;
  for (int t = tid; t < P; t += kListThreads) {
    uint32_t tau = 0xffffffffu;
    if (t < m) {
      tau = 0;
      for (int u = 0; u < k; ++u) tau = tau * (uint32_t)A + codes[base + t + u];
    }
    keys[t] = tau;
  }
  __syncthreads();
  // bitonic sort of keys[0..P)
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P / 2; t += kListThreads) {
        int lo = 2 * t - (t & (stride - 1));
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        uint32_t a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  // run starts: each thread owns a contiguous segment of positions
  const int per = (m + kListThreads - 1) / kListThreads;
  const int s0 = tid * per;
  const int s1 = min(m, s0 + per);
  int cnt = 0;
  for (int t = s0; t < s1; ++t)
    if (t == 0 || keys[t] != keys[t - 1]) ++cnt;
  seg_base[tid] = cnt;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < kListThreads; ++w) {
      int c = seg_base[w];
      seg_base[w] = acc;
      acc += c;
    }
    seg_base[kListThreads] = acc;
    nu[seq] = acc;
  }
  __syncthreads();
  int u = seg_base[tid];
  for (int t = s0; t < s1; ++t) {
    if (t == 0 || keys[t] != keys[t - 1]) {
      int e = t + 1;
      while (e < m && keys[e] == keys[t]) ++e;
      entries[base + u] = (keys[t] << 16) | (uint32_t)(e - t);
      ++u;
    }
  }
}

void launch_kmer_lists(const uint8_t* codes, const int64_t* offsets, int n, int A, int k,
                       uint32_t* entries, int64_t* /*kl_off*/, int32_t* nu, DevStatus* /*st*/,
                       hipStream_t stream) {
  if (n <= 0) return;
  kmer_list_kernel<<<n, kListThreads, 0, stream>>>(codes, offsets, A, k, entries, nu);
}

// ------------------------------------------------------------------ pair sums
// One 256-thread workgroup per row sequence r: its counts go to a dense u16
// histogram in LDS; each wave streams one column sequence's list at a time
// (64 consecutive entries per load) and sums min(count, H[tau]).

constexpr int kPairThreads = 256;
// Workgroups of the pair kernels whose histogram leaves room for only one
// workgroup per CU (above 64 KB: 4^8 k-mers) take four times the waves, so
// that more column lists are in flight against the one histogram.
constexpr int kPairThreadsMax = 1024;

// F = floor(c 2^31 / d), d = min(Li, Lj) - k + 1.  The numerator is below
// 2^44 (c <= d <= 8192), so the double quotient is within one of the floor
// and one integer correction makes it exact.
__device__ inline uint32_t fhat_of(int64_t c, int64_t Li, int64_t Lj, int k) {
  int64_t L = Li < Lj ? Li : Lj;
  if (L < k) return 0u;
  const uint64_t d = (uint64_t)(L - k + 1);
  const uint64_t num = (uint64_t)c << 31;
  uint64_t qt = (uint64_t)((double)num / (double)d);
  if (qt * d > num) --qt;
  else if ((qt + 1) * d <= num) ++qt;
  return (uint32_t)qt;
}

// Loads row r's list into the histogram (hist must be zero).
__device__ inline void hist_load(uint16_t* hist, const KmerLists& kl, int r) {
  const uint32_t* e = kl.entries + kl.off[r];
  const int nr = kl.nu[r];
  for (int t = threadIdx.x; t < nr; t += blockDim.x) {
    uint32_t v = e[t];
    hist[v >> 16] = (uint16_t)(v & 0xffff);
  }
}

__device__ inline void hist_clear(uint16_t* hist, int kspace) {
  uint32_t* h32 = reinterpret_cast<uint32_t*>(hist);
  for (int t = threadIdx.x; t < (kspace + 1) / 2; t += blockDim.x) h32[t] = 0;
}

// Sum over the wave (all 64 lanes active), wave-uniform: prefix sums within
// each row of 16 lanes by DPP row shifts (lanes past a row's start read 0),
// then lane 15 of rows 0 and 2 into rows 1 and 3 and lane 31 into rows 2 and
// 3 by row broadcasts, which leaves the total in lane 63.
template <int CTRL, int ROWS = 0xf>
__device__ inline int32_t dpp_in(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
__device__ inline int32_t wave_sum32(int32_t v) {
  v += dpp_in<0x111>(v);  // row_shr:1
  v += dpp_in<0x112>(v);  // row_shr:2
  v += dpp_in<0x114>(v);  // row_shr:4
  v += dpp_in<0x118>(v);  // row_shr:8
  v += dpp_in<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_in<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __builtin_amdgcn_readlane(v, 63);
}

// c between the histogram's row and NC column sequences cs[0..NC) (wave-wide;
// cs[q] < 0: none).  Four entries per lane and column are loaded before any
// is used, so NC lists of up to 256 entries cost one round trip.  Lanes past
// a list's end read the entry 0 (count 0, adds nothing).
template <int NC>
__device__ inline void wave_common_n(const uint16_t* hist, const KmerLists& kl, const int* cs,
                                     int32_t* res) {
  const uint32_t* e[NC];
  int nl[NC];
  int nmax = 0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    e[q] = kl.entries + kl.off[cs[q] >= 0 ? cs[q] : cs[0]];
    nl[q] = cs[q] >= 0 ? kl.nu[cs[q]] : 0;
    nmax = nl[q] > nmax ? nl[q] : nmax;
  }
  const int lane = threadIdx.x & 63;
  int32_t acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = 0;
  for (int t0 = 0; t0 < nmax; t0 += 256) {
    uint32_t v[NC][4];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + 64 * u + lane;
        v[q][u] = t < nl[q] ? e[q][t] : 0u;
      }
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t h = hist[v[q][u] >> 16], k = v[q][u] & 0xffffu;
        acc[q] += (int32_t)(k < h ? k : h);
      }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) res[q] = wave_sum32(acc[q]);
}

// columns per wave pass in the pair-sum kernels
constexpr int kPairCols = 8;

// The NC column results of a pass (wave-uniform) one per lane, so that their
// quotients are computed side by side: lane q < NC takes column q's count,
// sequence and position (the other lanes: sequence -1).
template <int NC>
__device__ inline void lane_column(const int32_t* cc, const int* cs, int lane, int32_t& c, int& j,
                                   int& q_of_lane) {
  c = 0;
  j = -1;
  q_of_lane = 0;
#pragma unroll
  for (int q = 0; q < NC; ++q)
    if (lane == q) {
      c = cc[q];
      j = cs[q];
      q_of_lane = q;
    }
}

// Sum over the wave of a 64-bit value (once per workgroup).
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1)
    v += (uint64_t)__shfl_xor((unsigned long long)v, o, 64);
  return v;
}

__device__ inline int64_t seq_len(const KmerLists& kl, int i) {
  return kl.seq_off[i + 1] - kl.seq_off[i];
}

// Block reduction of per-wave partial sums held by lane 0 of each wave.
__device__ inline uint64_t block_sum_waves(uint64_t v, uint64_t* red) {
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  uint64_t s = 0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  return s;
}

// ------------------------------------------------------------------ row groups
// A workgroup takes kRowGroup consecutive rows that share their column set
// (rows of one chunk, of the listed rows, of one group).  Their counts go to
// one histogram as 4-bit fields (row g in bits 4g..4g+3 of the k-mer's 16-bit
// word): each streamed column entry then serves every row of the group.  A
// count above 15 (the field's range) anywhere in the group sends the group
// down the one-row path instead (a full 16-bit count per k-mer, one row at a
// time), so the sums are exact either way.
constexpr int kRowGroup = 4;

// Loads the lists of rows[0..kRowGroup) (-1: none) as 4-bit fields; sets
// *over if a count does not fit.  hist and *over must be zero.
__device__ __forceinline__ void hist_load_packed(uint16_t* hist, const KmerLists& kl,
                                        const int* rows, int32_t* over) {
  uint32_t* h32 = reinterpret_cast<uint32_t*>(hist);
#pragma unroll
  for (int g = 0; g < kRowGroup; ++g) {
    if (rows[g] < 0) continue;
    const uint32_t* e = kl.entries + kl.off[rows[g]];
    const int nr = kl.nu[rows[g]];
    for (int t = threadIdx.x; t < nr; t += blockDim.x) {
      const uint32_t v = e[t], tau = v >> 16, cnt = v & 0xffffu;
      if (cnt > 15u) *over = 1;
      else if (cnt) atomicOr(&h32[tau >> 1], cnt << (4 * g + 16 * (tau & 1u)));
    }
  }
}

// c between every row of the packed histogram and NC column sequences
// cs[0..NC) (wave-wide; cs[q] < 0: none): res[q][g] for row g.  The loads are
// those of wave_common_n; each entry adds min(count, field g) for every g.
template <int NC>
__device__ __forceinline__ void wave_common_packed(const uint16_t* hist, const KmerLists& kl, const int* cs,
                                          int32_t (&res)[NC][kRowGroup]) {
  const uint32_t* e[NC];
  int nl[NC];
  int nmax = 0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    e[q] = kl.entries + kl.off[cs[q] >= 0 ? cs[q] : cs[0]];
    nl[q] = cs[q] >= 0 ? kl.nu[cs[q]] : 0;
    nmax = nl[q] > nmax ? nl[q] : nmax;
  }
  const int lane = threadIdx.x & 63;
  int32_t acc[NC][kRowGroup];
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int g = 0; g < kRowGroup; ++g) acc[q][g] = 0;
  for (int t0 = 0; t0 < nmax; t0 += 256) {
    uint32_t v[NC][4];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + 64 * u + lane;
        v[q][u] = t < nl[q] ? e[q][t] : 0u;
      }
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t h = hist[v[q][u] >> 16], k = v[q][u] & 0xffffu;
#pragma unroll
        for (int g = 0; g < kRowGroup; ++g) {
          const uint32_t f = (h >> (4 * g)) & 15u;
          acc[q][g] += (int32_t)(k < f ? k : f);
        }
      }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int g = 0; g < kRowGroup; ++g) res[q][g] = wave_sum32(acc[q][g]);
}

// The NC x kRowGroup results of a packed pass one per lane: lane q
// kRowGroup + g takes column q's count for row g (lanes past them: column -1).
template <int NC>
__device__ __forceinline__ void lane_pair(const int32_t (&cc)[NC][kRowGroup], const int* cs, int lane,
                                 int32_t& c, int& j, int& q_of_lane) {
  c = 0;
  j = -1;
  q_of_lane = 0;
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int g = 0; g < kRowGroup; ++g)
      if (lane == q * kRowGroup + g) {
        c = cc[q][g];
        j = cs[q];
        q_of_lane = q;
      }
}

// Per-row sums of the workgroup's lanes (row g = lane % kRowGroup, lanes
// below NC kRowGroup): thread 0 gets sums[g].
__device__ __forceinline__ void block_sum_rows(uint64_t part, uint64_t* red, uint64_t* sums) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int g = 0; g < kRowGroup; ++g) {
    const uint64_t v = wave_sum_u64((lane % kRowGroup) == g ? part : 0ull);
    if (lane == 0) red[g * (kPairThreadsMax / 64) + w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int g = 0; g < kRowGroup; ++g) {
      uint64_t t = 0;
      for (int q = 0; q < nw; ++q) t += red[g * (kPairThreadsMax / 64) + q];
      sums[g] = t;
    }
}

// Column passes of the group's rows over the columns col(x), x in [0, ncol)
// (col(x) < 0: skip).  packed: all rows at once against the 4-bit histogram,
// cb(x, g, c) for every column and row with its count c; otherwise only row
// `one` against the 16-bit histogram, cb(x, one, c).  cb runs on the lane that
// holds the result.
template <typename Col, typename Cb>
__device__ __forceinline__ void column_passes(const uint16_t* hist, const KmerLists& kl, int ncol, bool packed,
                                     int one, Col&& col, Cb&& cb) {
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  for (int x0 = wave; x0 < ncol; x0 += kPairCols * nw) {
    int cs[kPairCols], xs[kPairCols];
    bool any = false;
#pragma unroll
    for (int q = 0; q < kPairCols; ++q) {
      const int x = x0 + q * nw;
      xs[q] = x;
      cs[q] = x < ncol ? col(x) : -1;
      any = any || cs[q] >= 0;
    }
    if (!any) continue;
    // the first column must be valid (it names the stand-in list)
    if (cs[0] < 0)
#pragma unroll
      for (int q = 1; q < kPairCols; ++q)
        if (cs[0] < 0 && cs[q] >= 0) {
          cs[0] = cs[q];
          xs[0] = xs[q];
          cs[q] = -1;
        }
    int32_t cl;
    int jl, ql;
    if (packed) {
      int32_t cc[kPairCols][kRowGroup];
      wave_common_packed<kPairCols>(hist, kl, cs, cc);
      lane_pair<kPairCols>(cc, cs, lane, cl, jl, ql);
    } else {
      int32_t cc[kPairCols];
      wave_common_n<kPairCols>(hist, kl, cs, cc);
      lane_column<kPairCols>(cc, cs, lane, cl, jl, ql);
    }
    int xl = xs[0];
#pragma unroll
    for (int q = 0; q < kPairCols; ++q)
      if (q == ql) xl = xs[q];
    if (jl >= 0) cb(xl, packed ? lane % kRowGroup : one, jl, cl);
  }
}

// The shared body of the pair kernels: rows[0..kRowGroup) (-1: none) against
// the columns col(x); cb(x, g, column sequence, c) on the lane holding each
// result (g = the row's index in rows); done(g) by every thread after the
// columns of row g (one-row path) or of all rows (packed, g = -1).  Clears
// and loads the histogram.
template <typename Col, typename Cb, typename Done>
__device__ __forceinline__ void pair_rows(uint16_t* hist, int kspace, const KmerLists& kl,
                                 const int* rows, int ncol, int32_t* over, Col&& col,
                                 Cb&& cb, Done&& done) {
  hist_clear(hist, kspace);
  if (threadIdx.x == 0) *over = 0;
  __syncthreads();
  hist_load_packed(hist, kl, rows, over);
  __syncthreads();
  if (!*over) {
    // lanes of absent rows (a group's last rows) produce no result
    column_passes(hist, kl, ncol, true, -1, col, [&](int x, int g, int j, int32_t c) {
      if (rows[g] >= 0) cb(x, g, j, c);
    });
    done(-1);
    return;
  }
  for (int g = 0; g < kRowGroup; ++g) {
    const int rg = rows[g];
    if (rg < 0) continue;
    __syncthreads();
    hist_clear(hist, kspace);
    __syncthreads();
    hist_load(hist, kl, rg);
    __syncthreads();
    column_passes(hist, kl, ncol, false, g, col, cb);
    done(g);
  }
}

// Row sums of the pair kernels: the packed path's per-row lanes, or one row's
// lanes; thread 0 writes out[rows[g]].  Resets part.
__device__ __forceinline__ void store_row_sums(int g, uint64_t& part, uint64_t* red, uint64_t* sums,
                                      const int* rows, uint64_t* out) {
  if (g < 0) {
    block_sum_rows(part, red, sums);
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < kRowGroup; ++q)
        if (rows[q] >= 0) out[rows[q]] = sums[q];
  } else {
    const uint64_t s = block_sum_waves(wave_sum_u64(part), red);
    if (threadIdx.x == 0) out[rows[g]] = s;
  }
  part = 0;
  __syncthreads();
}

// K_loc(r) = sum over j in chunk(r) of F(r, j).  Workgroup (x, c) runs rows
// 4x .. 4x + 3 of chunk c.
__global__ __launch_bounds__(kPairThreadsMax) void rowsum_chunk_kernel(KmerLists kl, int n, int p,
                                                                     int k, int kspace,
                                                                     uint64_t* __restrict__ out) {
  extern __shared__ uint16_t hist[];
  __shared__ uint64_t red[kRowGroup * (kPairThreadsMax / 64)];
  __shared__ uint64_t sums[kRowGroup];
  __shared__ int32_t over;
  const int c = blockIdx.y;
  const int lo = (int)(((int64_t)c * n) / p), hi = (int)(((int64_t)(c + 1) * n) / p);
  const int r = lo + kRowGroup * (int)blockIdx.x;
  if (r >= hi) return;
  // the group's rows and lengths in LDS (read with lane-dependent indices)
  __shared__ int rows[kRowGroup];
  __shared__ int64_t Lr[kRowGroup];
  if (threadIdx.x < kRowGroup) {
    const int g = threadIdx.x;
    rows[g] = r + g < hi ? r + g : -1;
    Lr[g] = rows[g] >= 0 ? seq_len(kl, rows[g]) : 0;
  }
  __syncthreads();
  uint64_t part = 0;
  pair_rows(hist, kspace, kl, rows, hi - lo, &over, [&](int x) { return lo + x; },
            [&](int, int g, int j, int32_t cnt) {
              part += fhat_of(cnt, Lr[g], seq_len(kl, j), k);
            },
            [&](int g) { store_row_sums(g, part, red, sums, rows, out); });
}

// out(r) = sum over the listed columns of F(r, col); cols == nullptr lists
// all n sequences.  A listed id outside [0, n) is reported and skipped.
// Workgroup b runs rows 4b .. 4b + 3.
__global__ __launch_bounds__(kPairThreadsMax) void rowsum_list_kernel(KmerLists kl, int n,
                                                                    const int32_t* __restrict__ cols,
                                                                    int ncols, int k, int kspace,
                                                                    uint64_t* __restrict__ out,
                                                                    DevStatus* st) {
  extern __shared__ uint16_t hist[];
  __shared__ uint64_t red[kRowGroup * (kPairThreadsMax / 64)];
  __shared__ uint64_t sums[kRowGroup];
  __shared__ int32_t over;
  const int r = kRowGroup * (int)blockIdx.x;
  __shared__ int rows[kRowGroup];
  __shared__ int64_t Lr[kRowGroup];
  if (threadIdx.x < kRowGroup) {
    const int g = threadIdx.x;
    rows[g] = r + g < n ? r + g : -1;
    Lr[g] = rows[g] >= 0 ? seq_len(kl, rows[g]) : 0;
  }
  __syncthreads();
  uint64_t part = 0;
  pair_rows(hist, kspace, kl, rows, ncols, &over,
            [&](int x) {
              const int j = cols ? cols[x] : x;
              if (j < 0 || j >= n) {
                if (r == 0 && (threadIdx.x & 63) == 0) raise_error(st, SAD_E_INVAL, x, W_RANK);
                return -1;
              }
              return j;
            },
            [&](int, int g, int j, int32_t cnt) {
              part += fhat_of(cnt, Lr[g], seq_len(kl, j), k);
            },
            [&](int g) { store_row_sums(g, part, red, sums, rows, out); });
}

// F rows inside groups: group g's members are ids[group_off[g] ..
// group_off[g+1]); its matrix starts at fm_off[g] (n_g x n_g, row-major).
// Workgroup (x, g) writes the rows of members 4x .. 4x + 3 of group g.
__global__ __launch_bounds__(kPairThreadsMax) void fmatrix_kernel(KmerLists kl,
                                                                const int32_t* __restrict__ group_off,
                                                                const int32_t* __restrict__ ids,
                                                                int ngroups,
                                                                const int64_t* __restrict__ fm_off,
                                                                int k, int kspace,
                                                                uint32_t* __restrict__ F) {
  extern __shared__ uint16_t hist[];
  __shared__ int32_t over;
  const int g = blockIdx.y;
  const int g0 = group_off[g], ng = group_off[g + 1] - g0;
  const int a = kRowGroup * (int)blockIdx.x;
  if (a >= ng) return;
  const int row = g0 + a;
  __shared__ int rows[kRowGroup];
  __shared__ int64_t Lr[kRowGroup];
  if (threadIdx.x < kRowGroup) {
    const int q = threadIdx.x;
    rows[q] = a + q < ng ? ids[row + q] : -1;
    Lr[q] = rows[q] >= 0 ? seq_len(kl, rows[q]) : 0;
  }
  __syncthreads();
  uint32_t* Fg = F + fm_off[g] + (int64_t)a * ng;
  pair_rows(hist, kspace, kl, rows, ng, &over, [&](int x) { return ids[g0 + x]; },
            [&](int x, int q, int j, int32_t cnt) {
              Fg[(int64_t)q * ng + x] = fhat_of(cnt, Lr[q], seq_len(kl, j), k);
            },
            [&](int) {});
}

static size_t hist_bytes(int kspace) { return (size_t)((kspace + 1) / 2) * 4; }

static int pair_threads(int kspace) {
  return hist_bytes(kspace) > 64 * 1024 ? kPairThreadsMax : kPairThreads;
}

// Histograms above 64 KB (4^8 k-mers) need the larger dynamic-LDS limit.
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_rowsum_chunk(const KmerLists& kl, int n, int p, int k, int kspace, uint64_t* out,
                         hipStream_t stream) {
  if (n <= 0) return;
  allow_lds((const void*)rowsum_chunk_kernel, hist_bytes(kspace));
  const int wmax = (n + p - 1) / p;  // largest chunk
  const dim3 grid((wmax + kRowGroup - 1) / kRowGroup, p);
  rowsum_chunk_kernel<<<grid, pair_threads(kspace), hist_bytes(kspace), stream>>>(kl, n, p, k,
                                                                                kspace, out);
}

void launch_rowsum_list(const KmerLists& kl, int n, const int32_t* cols, int ncols, int k,
                        int kspace, uint64_t* out, DevStatus* st, hipStream_t stream) {
  if (n <= 0) return;
  allow_lds((const void*)rowsum_list_kernel, hist_bytes(kspace));
  rowsum_list_kernel<<<(n + kRowGroup - 1) / kRowGroup, pair_threads(kspace), hist_bytes(kspace),
                       stream>>>(kl, n, cols, ncols, k, kspace, out, st);
}

void launch_fmatrix_groups(const KmerLists& kl, const int32_t* group_off, const int32_t* ids,
                           int ngroups, int max_group, const int64_t* fm_off, int k, int kspace,
                           uint32_t* F, hipStream_t stream) {
  if (ngroups <= 0 || max_group <= 0) return;
  allow_lds((const void*)fmatrix_kernel, hist_bytes(kspace));
  const dim3 grid((max_group + kRowGroup - 1) / kRowGroup, ngroups);
  fmatrix_kernel<<<grid, pair_threads(kspace), hist_bytes(kspace), stream>>>(
      kl, group_off, ids, ngroups, fm_off, k, kspace, F);
}

// ------------------------------------------------------------------ chunk sort
// sorted[lo(c) + rank] = i, rank = #{j in chunk(i) : (key_j, j) < (key_i, i)}.

__global__ void chunk_rank_kernel(const uint64_t* __restrict__ key, int n, int p,
                                  int32_t* __restrict__ sorted) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = (int)(((int64_t)i * p) / n);
  while (c + 1 <= p && (((int64_t)(c + 1) * n) / p) <= i) ++c;
  while ((((int64_t)c * n) / p) > i) --c;
  const int lo = (int)(((int64_t)c * n) / p), hi = (int)(((int64_t)(c + 1) * n) / p);
  const uint64_t ki = key[i];
  int rank = 0;
  for (int j = lo; j < hi; ++j) {
    uint64_t kj = key[j];
    rank += (kj < ki) || (kj == ki && j < i);
  }
  sorted[lo + rank] = i;
}

void launch_chunk_sort(const uint64_t* key, int n, int p, int32_t* sorted, hipStream_t stream) {
  if (n <= 0) return;
  chunk_rank_kernel<<<(n + 255) / 256, 256, 0, stream>>>(key, n, p, sorted);
}

// sample t (1..ks) of chunk c: sorted[lo + floor(t w / (ks + 1))]
__global__ void pick_samples_kernel(const int32_t* __restrict__ sorted, int n, int p, int ks,
                                    int32_t* __restrict__ sample_ids) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= p * ks) return;
  int c = q / ks, t = q % ks + 1;
  int lo = (int)(((int64_t)c * n) / p), hi = (int)(((int64_t)(c + 1) * n) / p);
  int w = hi - lo;
  sample_ids[q] = sorted[lo + (int)(((int64_t)t * w) / (ks + 1))];
}

void launch_pick_samples(const int32_t* sorted, int n, int p, int ks, int32_t* sample_ids,
                         hipStream_t stream) {
  int tot = p * ks;
  if (tot <= 0) return;
  pick_samples_kernel<<<(tot + 255) / 256, 256, 0, stream>>>(sorted, n, p, ks, sample_ids);
}

}  // namespace sad
