// Progressive profile-profile alignment engine (paper Section 2.3.3: each
// bucket is aligned by a sequential aligner; here UPGMA-guided progressive
// alignment with affine gaps).
//
// Work model: a DAG of jobs.  A job aligns two nodes (profiles) P1, P2 and
// writes a new node; a job becomes ready when its children's jobs are done.
// A persistent grid pops ready jobs from a device queue; each workgroup is one
// wave (64 lanes) that runs the whole job:
//   1. DP over 64-row strips of P1: lane l owns row i = 64 s + l + 1 and at
//      step t computes column j = t - l + 1 (an anti-diagonal wavefront).  The
//      row above arrives from lane l-1 through a DPP wave shift; lane 0 reads
//      the previous strip's last row from a boundary buffer.  Per cell a byte
//      of tie information is stored (which of M/X/Y is the smallest op
//      attaining H; which predecessor attains X and Y).
//   2. Traceback from (W1, W2): the whole wave walks the path in lockstep,
//      staging 4 KB blocks of tie bytes in LDS.  The greedy rule picks the
//      smallest op still admitting an optimal completion, which yields the
//      optimal alignment whose op string read backwards is lexicographically
//      smallest (M < X < Y).
//   3. Merge: the op string is scanned across lanes to lay out the new
//      profile's columns (counts add) and each child's column map.
//
// Memory layout: node profiles are W x A uint16 counts in one pool; column
// maps (node column -> parent column) are W int32 in another.  Internal nodes
// are bump-allocated with W1 + W2 columns.
#include "sad_internal.h"

namespace sad {

constexpr int kRing = 256;     // columns of P2 staged in LDS (power of two)
constexpr int kStageT4 = 16;   // traceback staging: 16 x 64 words
constexpr int kEngineWavesPerCU = 7;

__device__ inline int32_t shr1(int32_t old_lane0, int32_t v) {
  // lane l receives lane l-1's v; lane 0 keeps old_lane0
  return __builtin_amdgcn_update_dpp(old_lane0, v, 0x138, 0xf, 0xf, false);
}

__device__ inline int32_t shl1(int32_t old_lane63, int32_t v) {
  // lane l receives lane l+1's v; lane 63 keeps old_lane63
  return __builtin_amdgcn_update_dpp(old_lane63, v, 0x130, 0xf, 0xf, false);
}

__device__ inline int readl(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

template <int A>
struct Engine {
  const EngineArgs& a;
  uint16_t* ring;
  uint32_t* tbst;
  uint8_t* ops;
  const int32_t* Ssh;
  int lane;

  __device__ Engine(const EngineArgs& args, uint16_t* r, uint32_t* t, uint8_t* o,
                    const int32_t* s)
      : a(args), ring(r), tbst(t), ops(o), Ssh(s), lane(threadIdx.x) {}

  // ---------------------------------------------------------------- DP
  // Fills the tie bytes of the whole (W1 x W2) matrix; returns H(W1, W2).
  __device__ int32_t dp(const uint16_t* P1, int W1, const uint16_t* P2, int W2, int32_t o,
                        int32_t e, uint32_t* tbw, int T4, int32_t* Hb, int32_t* Xb) {
    const int T = W2 + 63;
    for (int j = lane; j <= W2; j += 64) {
      Hb[j] = (j == 0) ? 0 : -(o + (j - 1) * e);
      Xb[j] = kNeg32;
    }
    __threadfence();
    __syncthreads();
    int32_t final_score = 0;
    const int nstrips = (W1 + 63) >> 6;
    for (int s = 0; s < nstrips; ++s) {
      const int i = 64 * s + lane + 1;
      int32_t U[A];
      {
        uint16_t c1[A];
        const bool rowv = i <= W1;
#pragma unroll
        for (int q = 0; q < A; ++q) c1[q] = rowv ? P1[(int64_t)(i - 1) * A + q] : (uint16_t)0;
#pragma unroll
        for (int b = 0; b < A; ++b) {
          int32_t u = 0;
#pragma unroll
          for (int q = 0; q < A; ++q) u += (int32_t)c1[q] * Ssh[q * A + b];
          U[b] = u;
        }
      }
      int32_t H = -(o + (min(i, W1) - 1) * e);
      int32_t X = kNeg32, Y = kNeg32;
      int32_t Hprev = Hb[0];
      uint32_t word = 0;
      uint32_t* tbs = tbw + (int64_t)s * T4 * 64;
      for (int t0 = 0; t0 < T; t0 += 64) {
        const int jn = t0 + 1 + lane;
        int32_t bh = 0, bx = 0;
        if (jn <= W2) {
          const uint16_t* src = P2 + (int64_t)(jn - 1) * A;
          uint16_t* dst = ring + ((jn - 1) & (kRing - 1)) * A;
#pragma unroll
          for (int q = 0; q < A; ++q) dst[q] = src[q];
          bh = Hb[jn];
          bx = Xb[jn];
        }
        __syncthreads();
        int32_t oh = 0, ox = 0;
        const int kend = min(64, T - t0);
        for (int k = 0; k < kend; ++k) {
          const int t = t0 + k;
          const int j = t - lane + 1;
          const int32_t Hup = shr1(readl(bh, k), H);
          const int32_t Xup = shr1(readl(bx, k), X);
          const int32_t Hdiag = Hprev;
          Hprev = Hup;
          int32_t sc = 0;
          if (j >= 1 && j <= W2) {
            const uint16_t* col = ring + ((j - 1) & (kRing - 1)) * A;
#pragma unroll
            for (int b = 0; b < A; ++b) sc += U[b] * (int32_t)col[b];
          }
          const int32_t M = Hdiag + sc;
          const int32_t xo = Hup - o, xe = Xup - e;
          const int32_t Xn = max(xo, xe);
          const int32_t yo = H - o, ye = Y - e;
          const int32_t Yn = max(yo, ye);
          const int32_t Hn = max(M, max(Xn, Yn));
          uint32_t bits = (M == Hn) ? 0u : ((Xn == Hn) ? 1u : 2u);
          bits |= ((uint32_t)(xo == Xn) << 2) | ((uint32_t)(xe == Xn) << 3) |
                  ((uint32_t)(yo == Yn) << 4) | ((uint32_t)(ye == Yn) << 5);
          if (j >= 1) {
            H = Hn;
            X = Xn;
            Y = Yn;
          }
          if (j == W2 && i == W1) final_score = Hn;
          word |= bits << (8 * (t & 3));
          if ((t & 3) == 3) {
            tbs[(int64_t)(t >> 2) * 64 + lane] = word;
            word = 0;
          }
          // lane 63's row shifts in from the right: after kend steps lane m
          // holds the value of step m - (64 - kend)
          oh = shl1(H, oh);
          ox = shl1(X, ox);
        }
        const int kk = lane - (64 - kend);
        const int jo = t0 + kk - 62;
        if (kk >= 0 && jo >= 1 && jo <= W2) {
          Hb[jo] = oh;
          Xb[jo] = ox;
        }
        __syncthreads();
      }
      if (T & 3) tbs[(int64_t)(T >> 2) * 64 + lane] = word;
      if (lane == 0) Hb[0] = -(o + (64 * (s + 1) - 1) * e);
      __threadfence();
      __syncthreads();
    }
    return readl(final_score, (W1 - 1) & 63);
  }

  // ---------------------------------------------------------------- traceback
  int st_s, st_t4a;

  __device__ uint32_t fetch(const uint32_t* tbw, int T4, int i, int j) {
    const int s = (i - 1) >> 6, l = (i - 1) & 63, t = j - 1 + l, t4 = t >> 2;
    if (s != st_s || t4 < st_t4a || t4 >= st_t4a + kStageT4) {
      st_s = s;
      st_t4a = max(0, t4 - (kStageT4 - 1));
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kStageT4; ++r) {
        const int tt = st_t4a + r;
        tbst[r * 64 + lane] = (tt < T4) ? tbw[((int64_t)s * T4 + tt) * 64 + lane] : 0u;
      }
      __syncthreads();
    }
    const uint32_t w = tbst[(t4 - st_t4a) * 64 + l];
    return (w >> (8 * (t & 3))) & 0xffu;
  }

  // Writes the op string to ops[cap - n .. cap); returns n.
  __device__ int traceback(const uint32_t* tbw, int T4, int W1, int W2) {
    st_s = -1;
    st_t4a = 0;
    const int cap = W1 + W2;
    int i = W1, j = W2, state = 0, k = 0;
    while (i > 0 && j > 0) {
      const uint32_t b = fetch(tbw, T4, i, j);
      if (state == 0) {
        const uint32_t hc = b & 3u;
        if (hc == 0) {
          if (lane == 0) ops[cap - 1 - k] = 0;
          ++k;
          --i;
          --j;
        } else {
          state = (int)hc;
        }
      } else if (state == 1) {
        if (lane == 0) ops[cap - 1 - k] = 1;
        ++k;
        const bool xo = (b >> 2) & 1u, xe = (b >> 3) & 1u;
        --i;
        bool pm = false;
        if (i > 0) pm = (fetch(tbw, T4, i, j) & 3u) == 0;
        state = (xo && pm) ? 0 : (xe ? 1 : 0);
      } else {
        if (lane == 0) ops[cap - 1 - k] = 2;
        ++k;
        const bool yo = (b >> 4) & 1u, ye = (b >> 5) & 1u;
        --j;
        bool pmx = false;
        if (j > 0) pmx = (fetch(tbw, T4, i, j) & 3u) <= 1u;
        state = (yo && pmx) ? 0 : (ye ? 2 : 0);
      }
    }
    for (; i > 0; --i, ++k)
      if (lane == 0) ops[cap - 1 - k] = 1;
    for (; j > 0; --j, ++k)
      if (lane == 0) ops[cap - 1 - k] = 2;
    __syncthreads();
    return k;
  }

  // ---------------------------------------------------------------- merge
  __device__ void merge(const uint16_t* P1, const uint16_t* P2, int base, int nops,
                        uint16_t* Pout, int32_t* up1, int32_t* up2) {
    const int per = (nops + 63) / 64;
    const int s0 = min(nops, lane * per), s1 = min(nops, s0 + per);
    int ci = 0, cj = 0;
    for (int q = s0; q < s1; ++q) {
      const uint8_t op = ops[base + q];
      ci += (op != 2);
      cj += (op != 1);
    }
    int ii = ci, jj = cj;
    for (int d = 1; d < 64; d <<= 1) {
      const int vi = __shfl_up(ii, d, 64), vj = __shfl_up(jj, d, 64);
      if (lane >= d) {
        ii += vi;
        jj += vj;
      }
    }
    ii -= ci;
    jj -= cj;
    for (int q = s0; q < s1; ++q) {
      const uint8_t op = ops[base + q];
#pragma unroll
      for (int b = 0; b < A; ++b) {
        uint32_t v = 0;
        if (op != 2) v += P1[(int64_t)ii * A + b];
        if (op != 1) v += P2[(int64_t)jj * A + b];
        Pout[(int64_t)q * A + b] = (uint16_t)v;
      }
      if (op != 2) {
        if (up1) up1[ii] = q;
        ++ii;
      }
      if (op != 1) {
        if (up2) up2[jj] = q;
        ++jj;
      }
    }
  }
};

template <int A>
__global__ __launch_bounds__(64) void engine_kernel(EngineArgs a) {
  __shared__ uint16_t ring[kRing * A];
  __shared__ uint32_t tbst[kStageT4 * 64];
  __shared__ uint8_t ops[2 * kMaxWidth];
  __shared__ int32_t Ssh[A * A];
  const int lane = threadIdx.x;
  for (int q = lane; q < A * A; q += 64) Ssh[q] = a.S[q];
  __syncthreads();
  Engine<A> eng(a, ring, tbst, ops, Ssh);
  uint32_t* tbw = a.tb + (int64_t)blockIdx.x * a.tb_words_per_wg;
  int32_t* Hb = a.bnd + (int64_t)blockIdx.x * 2 * (kMaxWidth + 1);
  int32_t* Xb = Hb + (kMaxWidth + 1);

  for (;;) {
    int slot = 0;
    if (lane == 0) slot = atomicAdd(a.queue_head, 1);
    slot = __shfl(slot, 0, 64);
    if (slot >= a.njobs) break;
    int ok = 1;
    if (lane == 0) {
      const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&a.queue_flag[slot], __ATOMIC_ACQUIRE,
                               __HIP_MEMORY_SCOPE_AGENT) == 0) {
        __builtin_amdgcn_s_sleep(8);
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t_start) > a.wait_ticks) {
          raise_error(a.st, SAD_E_DEVICE, slot, W_ENGINE_WAIT);
          ok = 0;
          break;
        }
      }
    }
    ok = __shfl(ok, 0, 64);
    if (!ok) break;
    __threadfence();
    const int job = __hip_atomic_load(&a.queue[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    const int na = a.job_a[job], nb = a.job_b[job], out = a.job_out[job];
    const int W1 = a.node_W[na], W2 = a.node_W[nb];
    const int n1 = a.node_n[na], n2 = a.node_n[nb];
    const uint16_t* P1 = a.prof_pool + a.node_prof[na];
    const uint16_t* P2 = a.prof_pool + a.node_prof[nb];
    int32_t* up1 = a.up_pool + a.node_up[na];
    int32_t* up2 = a.up_pool + a.node_up[nb];

    const int64_t G = (int64_t)n1 * n2;
    const int64_t unit = max((int64_t)max(a.smax, a.go), (int64_t)1);
    const int64_t bound = (int64_t)(W1 + W2 + 2) * G * unit;
    const int nstrips = (W1 + 63) >> 6;
    const int T4 = (W2 + 63 + 3) >> 2;
    const int64_t tb_need = (int64_t)nstrips * T4 * 64;
    const int cap = W1 + W2;
    int err = 0;
    if (W1 > kMaxWidth || W2 > kMaxWidth) {
      err = 1;
      if (lane == 0) raise_error(a.st, SAD_E_CAPACITY, cap, W_ENGINE_WIDTH);
    } else if (bound >= (1ll << 29)) {
      err = 1;
      if (lane == 0) raise_error(a.st, SAD_E_OVERFLOW, bound, W_ENGINE_BOUND);
    } else if (tb_need > a.tb_words_per_wg) {
      err = 1;
      if (lane == 0) raise_error(a.st, SAD_E_CAPACITY, tb_need, W_ENGINE_TB);
    } else if (n1 + n2 > 65535) {
      err = 1;
      if (lane == 0) raise_error(a.st, SAD_E_CAPACITY, n1 + n2, W_ENGINE);
    }
    long long prof_off = 0, up_off = 0;
    if (!err) {
      if (lane == 0) {
        prof_off = (long long)atomicAdd(a.prof_top, (unsigned long long)cap * A);
        up_off = (long long)atomicAdd(a.up_top, (unsigned long long)cap);
        if (prof_off + (long long)cap * A > a.prof_cap) {
          raise_error(a.st, SAD_E_CAPACITY, prof_off + (long long)cap * A, W_ENGINE_POOL);
          prof_off = -1;
        }
        if (up_off + cap > a.up_cap) {
          raise_error(a.st, SAD_E_CAPACITY, up_off + cap, W_ENGINE_POOL);
          up_off = -1;
        }
      }
      prof_off = __shfl(prof_off, 0, 64);
      up_off = __shfl(up_off, 0, 64);
      if (prof_off < 0 || up_off < 0) err = 1;
    }

    if (err) {
      // keep the DAG consistent and every later access in bounds
      for (int q = lane; q < W1; q += 64) up1[q] = 0;
      for (int q = lane; q < W2; q += 64) up2[q] = 0;
      if (lane == 0) {
        a.node_W[out] = 0;
        a.node_n[out] = n1 + n2;
        a.node_prof[out] = 0;
        a.node_up[out] = 0;
        a.job_score[job] = 0;
        a.job_cells[job] = (int64_t)W1 * W2;
      }
    } else {
      const int32_t o = (int32_t)(G * a.go), e = (int32_t)(G * a.ge);
      int32_t score;
      if (W1 == 0 || W2 == 0) {
        const int w = W1 + W2;
        score = w == 0 ? 0 : -(o + (w - 1) * e);
      } else {
        score = eng.dp(P1, W1, P2, W2, o, e, tbw, T4, Hb, Xb);
      }
      const int nops = eng.traceback(tbw, T4, W1, W2);
      const int base = cap - nops;
      uint16_t* Pout = a.prof_pool + prof_off;
      const int64_t oo = a.job_ops_off[job];
      // jobs that export their op string (refinement) leave the column maps
      // alone: several of them share the same second node
      eng.merge(P1, P2, base, nops, Pout, oo >= 0 ? nullptr : up1, oo >= 0 ? nullptr : up2);
      if (oo >= 0)
        for (int q = lane; q < nops; q += 64) a.ops_out[oo + q] = ops[base + q];
      if (lane == 0) {
        a.node_W[out] = nops;
        a.node_n[out] = n1 + n2;
        a.node_prof[out] = prof_off;
        a.node_up[out] = up_off;
        a.job_score[job] = score;
        a.job_cells[job] = (int64_t)W1 * W2;
      }
    }
    __threadfence();
    __syncthreads();
    if (lane == 0) {
      const int nx = a.job_next[job];
      if (nx >= 0) {
        const int prev = atomicSub(&a.job_pending[nx], 1);
        if (prev == 1) {
          __threadfence();
          const int pos = atomicAdd(a.queue_tail, 1);
          __hip_atomic_store(&a.queue[pos], nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __threadfence();
          __hip_atomic_store(&a.queue_flag[pos], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }
}

int engine_workgroups() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  if (cus <= 0) cus = 256;
  return cus * kEngineWavesPerCU;
}

void launch_engine(const EngineArgs& a, int nwg, hipStream_t stream) {
  if (a.njobs <= 0 || nwg <= 0) return;
  if (a.A == 20) engine_kernel<20><<<nwg, 64, 0, stream>>>(a);
  else engine_kernel<4><<<nwg, 64, 0, stream>>>(a);
}

// ------------------------------------------------------------------ setup kernels

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_i32_kernel<<<(int)blocks, 256, 0, stream>>>(p, v, n);
}

// Leaf r: sequence ids[r]; its profile and column map live at the sequence's
// residue offset (offsets[id] * A in the profile pool, offsets[id] in the map
// pool), so the first total_len * A / total_len entries of the pools hold the
// leaves.
__global__ void make_leaves_kernel(const int64_t* __restrict__ offsets,
                                   const int32_t* __restrict__ ids, int nleaves, int A,
                                   int32_t node_base, int32_t* node_W, int32_t* node_n,
                                   int64_t* node_prof, int64_t* node_up, int32_t* node_parent) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nleaves) return;
  const int id = ids ? ids[r] : r;
  const int64_t o = offsets[id];
  node_W[node_base + r] = (int32_t)(offsets[id + 1] - o);
  node_n[node_base + r] = 1;
  node_prof[node_base + r] = o * A;
  node_up[node_base + r] = o;
  node_parent[node_base + r] = -1;
}

__global__ void onehot_kernel(const uint8_t* __restrict__ codes, int64_t total, int A,
                              uint16_t* __restrict__ prof) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int c = codes[t];
    for (int b = 0; b < A; ++b) prof[t * A + b] = (uint16_t)(b == c);
  }
}

void launch_make_leaves(const uint8_t* codes, const int64_t* offsets, const int32_t* ids,
                        int nleaves, int A, int32_t node_base, int32_t* node_W, int32_t* node_n,
                        int64_t* node_prof, int64_t* node_up, int32_t* node_parent,
                        uint16_t* prof_pool, int64_t total_len, hipStream_t stream) {
  if (nleaves <= 0) return;
  make_leaves_kernel<<<(nleaves + 255) / 256, 256, 0, stream>>>(
      offsets, ids, nleaves, A, node_base, node_W, node_n, node_prof, node_up, node_parent);
  int64_t blocks = (total_len + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  onehot_kernel<<<(int)blocks, 256, 0, stream>>>(codes, total_len, A, prof_pool);
}

// Jobs of UPGMA trees.  Group g has members group_off[g]..group_off[g+1]; its
// leaves are nodes group_off[g] + x and its cluster n_g + t is node
// internal_base + group_off[g] + t, made by the job in slot group_off[g] + t.
__global__ void make_jobs_kernel(const int32_t* __restrict__ merges,
                                 const int32_t* __restrict__ group_off, int ngroups, int nslots,
                                 int32_t internal_base, int32_t* node_parent, int32_t* job_a,
                                 int32_t* job_b, int32_t* job_out, int32_t* job_next,
                                 int32_t* job_pending, int32_t* queue, int32_t* queue_flag,
                                 int32_t* queue_tail) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  int lo = 0, hi = ngroups;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (group_off[mid] <= s) lo = mid;
    else hi = mid;
  }
  const int g0 = group_off[lo], ng = group_off[lo + 1] - g0;
  const int t = s - g0;
  if (t >= ng - 1) {
    job_a[s] = -1;
    return;
  }
  const int la = merges[2 * s], lb = merges[2 * s + 1];
  const int a = la < ng ? g0 + la : internal_base + g0 + (la - ng);
  const int b = lb < ng ? g0 + lb : internal_base + g0 + (lb - ng);
  job_a[s] = a;
  job_b[s] = b;
  job_out[s] = internal_base + s;
  node_parent[a] = internal_base + s;
  node_parent[b] = internal_base + s;
  int pending = 0;
  if (la >= ng) {
    job_next[g0 + (la - ng)] = s;
    ++pending;
  }
  if (lb >= ng) {
    job_next[g0 + (lb - ng)] = s;
    ++pending;
  }
  job_pending[s] = pending;
  if (pending == 0) {
    const int pos = atomicAdd(queue_tail, 1);
    queue[pos] = s;
    queue_flag[pos] = 1;
  }
}

void launch_make_jobs(const int32_t* merges, const int32_t* group_off, int ngroups, int nslots,
                      int32_t internal_base, int32_t* node_parent, int32_t* job_a, int32_t* job_b,
                      int32_t* job_out, int32_t* job_next, int32_t* job_pending, int32_t* queue,
                      int32_t* queue_flag, int32_t* queue_tail, hipStream_t stream) {
  if (nslots <= 0) return;
  make_jobs_kernel<<<(nslots + 255) / 256, 256, 0, stream>>>(
      merges, group_off, ngroups, nslots, internal_base, node_parent, job_a, job_b, job_out,
      job_next, job_pending, queue, queue_flag, queue_tail);
}

// Column of every residue in its tree's root: leaf node of member position r
// is r; follow column maps up to the root.
__global__ void colmap_kernel(const int64_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                              int nleaves, const int32_t* __restrict__ node_parent,
                              const int64_t* __restrict__ node_up,
                              const int32_t* __restrict__ up_pool, int32_t* __restrict__ colmap,
                              DevStatus* st) {
  const int r = blockIdx.x;
  const int id = ids ? ids[r] : r;
  const int64_t o = offsets[id];
  const int L = (int)(offsets[id + 1] - o);
  for (int x = threadIdx.x; x < L; x += blockDim.x) {
    int c = x, node = r, depth = 0;
    // a tree over n leaves has depth < n; the bound guards a malformed one
    while (node_parent[node] >= 0 && depth < nleaves) {
      c = up_pool[node_up[node] + c];
      node = node_parent[node];
      ++depth;
    }
    if (depth >= nleaves) raise_error(st, SAD_E_DEVICE, r, W_ENGINE);
    colmap[o + x] = c;
  }
}

void launch_colmap(const int64_t* offsets, const int32_t* ids, int nleaves,
                   const int32_t* node_parent, const int64_t* node_up, const int32_t* up_pool,
                   int32_t* colmap, DevStatus* st, hipStream_t stream) {
  if (nleaves <= 0) return;
  colmap_kernel<<<nleaves, 128, 0, stream>>>(offsets, ids, nleaves, node_parent, node_up, up_pool,
                                             colmap, st);
}

// width of group g's root node
__global__ void widths_kernel(const int32_t* __restrict__ group_off, int ngroups,
                              int32_t internal_base, const int32_t* __restrict__ node_W,
                              int32_t* __restrict__ width) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int g0 = group_off[g], ng = group_off[g + 1] - g0;
  if (ng == 0) width[g] = 0;
  else if (ng == 1) width[g] = node_W[g0];
  else width[g] = node_W[internal_base + g0 + ng - 2];
}

void launch_widths(const int32_t* group_off, int ngroups, int32_t internal_base,
                   const int32_t* node_W, int32_t* width, hipStream_t stream) {
  if (ngroups <= 0) return;
  widths_kernel<<<(ngroups + 255) / 256, 256, 0, stream>>>(group_off, ngroups, internal_base,
                                                           node_W, width);
}

// per-slot results copied to the caller's arrays (slots without a job untouched)
__global__ void job_results_kernel(const int32_t* __restrict__ job_a,
                                   const int64_t* __restrict__ job_score,
                                   const int64_t* __restrict__ job_cells, int nslots,
                                   int64_t* score_out, int64_t* cells_out,
                                   unsigned long long* cells_total) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots || job_a[s] < 0) return;
  score_out[s] = job_score[s];
  cells_out[s] = job_cells[s];
  atomicAdd(cells_total, (unsigned long long)job_cells[s]);
}

void launch_job_results(const int32_t* job_a, const int64_t* job_score, const int64_t* job_cells,
                        int nslots, int64_t* score_out, int64_t* cells_out, int64_t* cells_total,
                        hipStream_t stream) {
  if (nslots <= 0) return;
  job_results_kernel<<<(nslots + 255) / 256, 256, 0, stream>>>(
      job_a, job_score, job_cells, nslots, score_out, cells_out,
      reinterpret_cast<unsigned long long*>(cells_total));
}

}  // namespace sad
