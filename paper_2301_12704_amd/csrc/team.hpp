// A "team" of G co-resident workgroups (NT threads each) working on one dense task, with
// team-wide barriers through a counter in device memory.  G == 1 is a plain workgroup and its
// barrier is __syncthreads().  Team routines distribute their work over the G * NT team
// threads and end with a team barrier, so results are visible to every member on return.
//
// Every output element is computed in one fixed order whatever G is: by one MFMA tile of one
// wave (the dense products), by one group of 16 lanes in the fixed chain-and-tree order below
// (the row sums of the pivoted QR and the Q formation), or by one thread (copies).
#pragma once
#include "dense_wg.hpp"

namespace aifmm {

// Candidate of one team member for the pivot rule of t_cpqr: its largest trailing norm mv,
// the lowest position p among its columns within a relative 1e-11 of mv, and that column's
// norm nv (p = INT_MAX when the member has no live column).
struct Cand {
  double mv, nv;
  int p, pad;
};

// Pivot candidate state for one pass over the live columns: the largest norm mx, the lowest
// position p among the columns whose norm is >= keep * mx, that column's norm nv, and amb set
// when merging lost the information needed to know p exactly (a column within the band of a
// smaller maximum that may or may not reach the band of the larger one).  Merging is
// associative; when amb is clear, p is exactly the pivot of the two-pass rule.
struct PivState {
  double mx, nv;
  int p, amb;
};
// Barrier counters of concurrent teams sit CTR_STRIDE words (256 bytes) apart, so the teams'
// atomics and polls do not contend for one cache line.
constexpr int CTR_STRIDE = 64;
// The members' exchange slots sit CAND_STRIDE entries (192 bytes) apart for the same reason.
constexpr int CAND_STRIDE = 8;

// Device-scope (all compute units) stores and loads: relaxed atomics at agent scope, which
// write through to and read from the device's point of coherence.
template <class T_>
__device__ __attribute__((always_inline)) inline void st_dev(T_* p, T_ v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T_>
__device__ __attribute__((always_inline)) inline T_ ld_dev(const T_* p) {
  return __hip_atomic_load(const_cast<T_*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT>
struct Team {
  int member = 0, G = 1;      // this workgroup's index in the team, team size
  int gtid = 0, GT = NT;      // team thread index and count
  int cid = 0;                // column-interleaved team thread index: member + G * thread
  unsigned* ctr = nullptr;    // barrier counter (zero at launch)
  Cand* part = nullptr;       // 2 x G exchange slots, CAND_STRIDE apart (double-buffered)
  int* abort = nullptr;       // set when a barrier waited too long; every later barrier returns
  unsigned epoch = 0;
  unsigned xep = 0;           // exchanges by flags so far (exchange_merge)
  int slot = 0;
  bool bad = false;           // the abort flag was seen at the last barrier: data exchanged through
                              // the team may be stale, so callers stop using it and exit

  __device__ __attribute__((always_inline)) void init(int member_, int G_, unsigned* ctr_, Cand* part_, int* abort_) {
    member = member_;
    G = G_;
    gtid = member * NT + (int)threadIdx.x;
    GT = G * NT;
    cid = member + G * (int)threadIdx.x;
    ctr = ctr_;
    part = part_;
    abort = abort_;
  }

  // Wait for every member.  The workgroup barrier orders this workgroup's writes before thread
  // 0's agent-scope release; thread 0's acquire after the wait makes the other members' writes
  // visible to the whole workgroup.  The wait is bounded (max_spins polls, a few seconds by
  // default): on expiry the abort flag is raised and the team falls through, so every
  // workgroup still runs to its end and the host reports the failure.  Thread 0 reads the flag
  // after the wait and the workgroup takes its value through LDS, so bad is uniform over the
  // workgroup (members of a team may see the flag at different barriers; once raised it stays
  // raised, so every later barrier of every member falls through and sets bad).
  __device__ __attribute__((always_inline)) void sync(unsigned max_spins = 1u << 24) {
    __shared__ int s_bad;
    __syncthreads();
    if (G == 1) return;
    if (threadIdx.x == 0) {
      ++epoch;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(ctr, 1u);
      unsigned target = epoch * (unsigned)G;
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        // the abort flag (one word every team polls) is read every 64th poll
        if ((spins & 63) == 63 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(2);
        if (++spins > max_spins) {
          atomicExch(abort, 1);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_bad = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    bad = s_bad != 0;
  }

  // Publish one value per member and return all G of them (the same array on every thread;
  // member q's value at q CAND_STRIDE).
  __device__ __attribute__((always_inline)) const Cand* exchange(const Cand& c) {
    Cand* p = part + (size_t)slot * G * CAND_STRIDE;
    if (threadIdx.x == 0) p[member * CAND_STRIDE] = c;
    sync();
    slot ^= 1;
    return p;
  }

  // Publish one candidate state per member and return the merge of all G of them (the same
  // on every thread), without a team barrier: every thread waits for its own device-scope
  // publication stores, the workgroup synchronises, thread 0 stores the member's state
  // (device scope) into the exchange slot, waits for it, and then raises the member's flag
  // (the member's count of such exchanges, in the unused part of its slot-0 entry; zero at
  // launch).  Lane q of the first wave waits for member q's flag to reach this exchange's count
  // and reads member q's state; the wave merges them by a tree.  Data read after a member's
  // flag (its state, its publication slot) is read with device-scope loads.  A slot is
  // rewritten two exchanges later, which no member reaches before every member has raised its
  // flag for the exchange in between, so double-buffered slots suffice.  The wait is bounded
  // like sync(); on expiry, or with the abort flag raised, bad is set.
  template <class R, class Merge, class WaveMerge>
  __device__ __attribute__((always_inline)) PivState exchange_merge(const Cand& c, R keep, PivState* shres,
                                                                   Merge merge, WaveMerge wmerge,
                                                                   unsigned max_spins = 1u << 24) {
    __shared__ int s_bad;
    ++xep;
    Cand* p = part + (size_t)slot * G * CAND_STRIDE;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's publication stores are done
    __syncthreads();
    if (threadIdx.x == 0) {
      Cand* q = p + member * CAND_STRIDE;
      st_dev(&q->mv, c.mv);
      st_dev(&q->nv, c.nv);
      st_dev(&q->p, c.p);
      st_dev(&q->pad, c.pad);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      st_dev((unsigned*)(part + (size_t)member * CAND_STRIDE + 1), xep);
    }
    if (threadIdx.x < WAVE) {
      PivState g{-1.0, -1.0, INT_MAX, 0};
      int ok = 1;
      for (int q = (int)threadIdx.x; q < G && ok; q += WAVE) {
        const unsigned* fq = (const unsigned*)(part + (size_t)q * CAND_STRIDE + 1);
        unsigned spins = 0;
        while (ld_dev(fq) < xep) {
          if ((spins & 63) == 63 && ld_dev(abort)) {
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          if (++spins > max_spins) {
            atomicExch(abort, 1);
            ok = 0;
            break;
          }
        }
        if (!ok) break;
        asm volatile("" ::: "memory");
        const Cand* cq = p + q * CAND_STRIDE;
        g = merge(g, PivState{ld_dev(&cq->mv), ld_dev(&cq->nv), ld_dev(&cq->p), ld_dev(&cq->pad)});
      }
      const int allok = __all(ok);
      g = wmerge(g);
      if (threadIdx.x == 0) {
        shres[0] = g;
        s_bad = !allok || ld_dev(abort) != 0;
      }
    }
    __syncthreads();
    bad = s_bad != 0;
    slot ^= 1;
    return shres[0];
  }

  // Team-wide argmax (ties to the lowest index); the same value on every thread of the team.
  __device__ __attribute__((always_inline)) ValIdx argmax(ValIdx x, ValIdx* shv) {
    ValIdx r = wg_argmax<NT>(x, shv);
    if (G == 1) return r;
    const Cand* all = exchange(Cand{r.v, 0.0, r.i, 0});
    ValIdx b{-1.0, INT_MAX};
    for (int q = 0; q < G; ++q) {
      ValIdx c{all[q * CAND_STRIDE].mv, all[q * CAND_STRIDE].p};
      if (vi_better(c, b)) b = c;
    }
    return b;
  }
};

template <int NT, class TS, class TD>
__device__ inline void t_copy(Team<NT>& T, int M, int N, const TS* __restrict__ A, int lda, TD* __restrict__ C, int ldc) {
  for (int idx = T.gtid; idx < M * N; idx += T.GT) {
    int r = idx / N, c = idx - r * N;
    C[(size_t)r * ldc + c] = (TD)A[(size_t)r * lda + c];
  }
  T.sync();
}
template <int NT, class TD>
__device__ inline void t_zero(Team<NT>& T, int M, int N, TD* C, int ldc) {
  for (int idx = T.gtid; idx < M * N; idx += T.GT) {
    int r = idx / N, c = idx - r * N;
    C[(size_t)r * ldc + c] = (TD)0;
  }
  T.sync();
}
// C = alpha op(A) op(B) + beta C, each element accumulated from zero in ascending k in the
// precision of the operands, then scaled and added in C's precision.  The team's waves take
// 16 x 16 output tiles on MFMA 16x16x4.  All-FP64 products use FP64 MFMA, which adds its four
// products one fused multiply-add at a time in ascending k (the slots past K add exact zeros
// at the end of the chain), so the results are those of the sequential chains; products with
// an FP32 operand or result (the precision form) use FP32 MFMA with FP32 accumulation, in the
// hardware's order inside an MFMA.
template <int NT, class TA, class TB, class TC>
__device__ inline void t_gemm(Team<NT>& T, int M, int N, int K, double alpha, const TA* __restrict__ A, int lda,
                              bool ta, const TB* __restrict__ B, int ldb, bool tb, double beta, TC* C, int ldc) {
  if constexpr (sizeof(TA) == 4 || sizeof(TB) == 4 || sizeof(TC) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int KC = 8;
    const int lane = (int)threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
    const int wid = T.member * (NT / WAVE) + (int)threadIdx.x / WAVE, nwv = T.G * (NT / WAVE);
    const int tm = (M + 15) / 16, tn = (N + 15) / 16, nsteps = (K + 3) / 4;
    const size_t ai = ta ? 1 : (size_t)lda, ak = ta ? (size_t)lda : 1;
    const size_t bk = tb ? 1 : (size_t)ldb, bj = tb ? (size_t)ldb : 1;
    for (int tile = wid; tile < tm * tn; tile += nwv) {
      const int R0 = (tile / tn) * 16, C0 = (tile % tn) * 16;
      const bool aok = R0 + fr < M, bok = C0 + fr < N;
      const TA* Ar = A + (size_t)(R0 + fr) * ai;
      const TB* Bc = B + (size_t)(C0 + fr) * bj;
      auto fa = [&](int s) {
        int k = 4 * s + fk;
        return (aok && k < K) ? (float)Ar[(size_t)k * ak] : 0.0f;
      };
      auto fb = [&](int s) {
        int k = 4 * s + fk;
        return (bok && k < K) ? (float)Bc[(size_t)k * bk] : 0.0f;
      };
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      float pa[KC], pb[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        pa[u] = u < nsteps ? fa(u) : 0.0f;
        pb[u] = u < nsteps ? fb(u) : 0.0f;
      }
      for (int s0 = 0; s0 < nsteps; s0 += KC) {
        float ca[KC], cb[KC];
#pragma unroll
        for (int u = 0; u < KC; ++u) {
          ca[u] = pa[u];
          cb[u] = pb[u];
        }
        if (s0 + KC < nsteps) {
#pragma unroll
          for (int u = 0; u < KC; ++u) {
            int s = s0 + KC + u;
            pa[u] = s < nsteps ? fa(s) : 0.0f;
            pb[u] = s < nsteps ? fb(s) : 0.0f;
          }
        }
#pragma unroll
        for (int u = 0; u < KC; ++u)
          if (s0 + u < nsteps) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[u], cb[u], acc, 0, 0, 0);
      }
      // output (lane, q): row R0 + 4 (lane / 16) + q, column C0 + lane % 16 (FP32 MFMA layout)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = R0 + 4 * fk + q, c = C0 + fr;
        if (r < M && c < N) {
          TC v = (TC)((float)alpha * acc[q]);
          if (beta != 0.0) v += (TC)beta * C[(size_t)r * ldc + c];
          C[(size_t)r * ldc + c] = v;
        }
      }
    }
  } else {
    static_assert(sizeof(TA) == 8 && sizeof(TB) == 8 && sizeof(TC) == 8, "FP64 or FP32 products only");
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int KC = 8;
    const int lane = (int)threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
    const int wid = T.member * (NT / WAVE) + (int)threadIdx.x / WAVE, nwv = T.G * (NT / WAVE);
    const int tm = (M + 15) / 16, tn = (N + 15) / 16, nsteps = (K + 3) / 4;
    const size_t ai = ta ? 1 : (size_t)lda, ak = ta ? (size_t)lda : 1;
    const size_t bk = tb ? 1 : (size_t)ldb, bj = tb ? (size_t)ldb : 1;
    for (int tile = wid; tile < tm * tn; tile += nwv) {
      const int R0 = (tile / tn) * 16, C0 = (tile % tn) * 16;
      const bool aok = R0 + fr < M, bok = C0 + fr < N;
      const TA* Ar = A + (size_t)(R0 + fr) * ai;
      const TB* Bc = B + (size_t)(C0 + fr) * bj;
      auto fa = [&](int s) {
        int k = 4 * s + fk;
        return (aok && k < K) ? (double)Ar[(size_t)k * ak] : 0.0;
      };
      auto fb = [&](int s) {
        int k = 4 * s + fk;
        return (bok && k < K) ? (double)Bc[(size_t)k * bk] : 0.0;
      };
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      double pa[KC], pb[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        pa[u] = u < nsteps ? fa(u) : 0.0;
        pb[u] = u < nsteps ? fb(u) : 0.0;
      }
      for (int s0 = 0; s0 < nsteps; s0 += KC) {
        double ca[KC], cb[KC];
#pragma unroll
        for (int u = 0; u < KC; ++u) {
          ca[u] = pa[u];
          cb[u] = pb[u];
        }
        if (s0 + KC < nsteps) {
#pragma unroll
          for (int u = 0; u < KC; ++u) {
            int s = s0 + KC + u;
            pa[u] = s < nsteps ? fa(s) : 0.0;
            pb[u] = s < nsteps ? fb(s) : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < KC; ++u)
          if (s0 + u < nsteps) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u], cb[u], acc, 0, 0, 0);
      }
      // output (lane, q): row R0 + lane / 16 + 4 q, column C0 + lane % 16
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = R0 + fk + 4 * q, c = C0 + fr;
        if (r < M && c < N) {
          double v = alpha * acc[q];
          if (beta != 0.0) v += beta * (double)C[(size_t)r * ldc + c];
          C[(size_t)r * ldc + c] = (TC)v;
        }
      }
    }
  }
  T.sync();
}

// A value of another lane of the same 16-lane DPP row (v_mov_b32_dpp with control CTRL, all
// rows and banks); 64-bit values move as two halves.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <class R>
__device__ inline PivState piv_merge(const PivState& a, const PivState& b, R keep) {
  PivState r;
  r.mx = fmax(a.mx, b.mx);
  r.p = INT_MAX;
  r.nv = -1.0;
  r.amb = a.amb | b.amb;
  const double thr = (double)((R)r.mx * keep);
  const PivState* s[2] = {&a, &b};
  for (int q = 0; q < 2; ++q) {
    const PivState& x = *s[q];
    if (x.p == INT_MAX || x.mx < thr) continue;
    if (x.nv >= thr) {
      if (x.p < r.p) { r.p = x.p; r.nv = x.nv; }
    } else {
      r.amb = 1;
    }
  }
  return r;
}
// Merges of candidate states.  The merge is commutative and associative, so any pairing gives
// the same state: inside each 16-lane row the partners come through DPP moves (lane ^ 1,
// lane ^ 2, the other quad, the other half row, as in lane_sum16), then across the wave's four
// rows through two lane exchanges.
template <int CTRL>
__device__ inline PivState dpp_piv(const PivState& x) {
  PivState o;
  o.mx = dpp_mov<CTRL>(x.mx);
  o.nv = dpp_mov<CTRL>(x.nv);
  o.p = __builtin_amdgcn_mov_dpp(x.p, CTRL, 0xF, 0xF, false);
  o.amb = __builtin_amdgcn_mov_dpp(x.amb, CTRL, 0xF, 0xF, false);
  return o;
}
// Wave-wide merge (the same state on every lane of the wave).
template <class R>
__device__ inline PivState wave_pivmerge(PivState x, R keep) {
  x = piv_merge(x, dpp_piv<0xB1>(x), keep);
  x = piv_merge(x, dpp_piv<0x4E>(x), keep);
  x = piv_merge(x, dpp_piv<0x141>(x), keep);
  x = piv_merge(x, dpp_piv<0x140>(x), keep);
  for (int off = 16; off < WAVE; off <<= 1) {
    PivState o;
    o.mx = __shfl_xor(x.mx, off, WAVE);
    o.nv = __shfl_xor(x.nv, off, WAVE);
    o.p = __shfl_xor(x.p, off, WAVE);
    o.amb = __shfl_xor(x.amb, off, WAVE);
    x = piv_merge(x, o, keep);
  }
  return x;
}
// Workgroup-wide maximum of a double and minimum of an int (the same value on every thread):
// DPP moves inside each 16-lane row, two lane exchanges across the rows, then the waves' values
// through LDS (sh: NT / 64 entries, not read again before the next __syncthreads).  Maxima and
// minima do not depend on the order of the operands.
template <int NT>
__device__ inline double wg_max(double x, double* sh) {
  x = fmax(x, dpp_mov<0xB1>(x));
  x = fmax(x, dpp_mov<0x4E>(x));
  x = fmax(x, dpp_mov<0x141>(x));
  x = fmax(x, dpp_mov<0x140>(x));
  x = fmax(x, __shfl_xor(x, 16, WAVE));
  x = fmax(x, __shfl_xor(x, 32, WAVE));
  if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = x;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int q = 1; q < NT / WAVE; ++q) r = fmax(r, sh[q]);
  return r;
}
template <int NT>
__device__ inline int wg_min(int x, int* sh) {
  x = min(x, __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false));
  x = min(x, __shfl_xor(x, 16, WAVE));
  x = min(x, __shfl_xor(x, 32, WAVE));
  if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = x;
  __syncthreads();
  int r = sh[0];
#pragma unroll
  for (int q = 1; q < NT / WAVE; ++q) r = min(r, sh[q]);
  return r;
}

// Row sums of the pivoted QR and of the Q formation are taken in one fixed order: sixteen
// partial fused multiply-add chains over the rows, chain q holding the rows i = q (mod 16) in
// ascending order, then the pairwise tree ((t0 + t1) + (t2 + t3)) + ... over the chains.  A
// group of PL = 16 lanes (one DPP row of the wave) owns a column: lane q runs chain q, and
// lane_sum16 leaves the tree's sum on all 16 lanes.  Each level adds the value of the partner
// lane through a DPP move within the row: lane ^ 1 and lane ^ 2 (quad permutations), then the
// other quad of the half row (half-row mirror) and the other half row (row mirror); after a
// level every lane of a pair, quad or half row holds the same value (IEEE addition is
// commutative), so the mirrors pair exactly the subtrees of the tree.  A column's dependent
// chain is m / 16 terms long instead of m.
constexpr int PL = 16;
template <class R>
__device__ inline R lane_sum16(R t) {
  t = t + dpp_mov<0xB1>(t);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  t = t + dpp_mov<0x4E>(t);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  t = t + dpp_mov<0x141>(t);  // row_half_mirror: the other quad of the half row
  t = t + dpp_mov<0x140>(t);  // row_mirror: the other half row
  return t;
}
// loads in flight per lane in the column passes: LDS columns, and workspace columns (which
// come from L2 at a much longer latency)
constexpr int COL_B = 4, COL_BG = 16;

// The passes of one column by its 16-lane group; lane r0 % 16 takes the rows r0, r0 + 16, ...
// below m, B loads in flight.  grp_dot: the lane's partial chain of sum v_i a_i.
template <int B, class R>
__device__ inline R grp_dot(const R* col, const R* v, int r0, int m) {
  R acc = 0;
  for (int i0 = r0; i0 < m; i0 += PL * B) {
    R a[B], b[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      int i = i0 + PL * u;
      a[u] = i < m ? col[i] : R(0);
      b[u] = i < m ? v[i] : R(0);
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (i0 + PL * u < m) acc = fma(b[u], a[u], acc);
  }
  return acc;
}
// a_i -= w v_i; returns the lane's partial chain of sum a_i^2 over the rows above s (with
// norm), else 0
template <int B, bool NORM, class R>
__device__ inline R grp_axpy(R* col, const R* v, int r0, int m, int s, R w) {
  R t = 0;
  for (int i0 = r0; i0 < m; i0 += PL * B) {
    R a[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      int i = i0 + PL * u;
      a[u] = i < m ? col[i] : R(0);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      int i = i0 + PL * u;
      if (i < m) {
        R x = fma(-w, v[i], a[u]);
        col[i] = x;
        if (NORM && i > s) t = fma(x, x, t);
      }
    }
  }
  return t;
}

// Column storage of the pivoted QR and the Q formation.  A member's own columns are numbered
// lc = 0, 1, ... (column c = member + G lc of the matrix, or c0 + member + G lc of Q); lane group
// lc mod (NT / 16) runs column lc.  The first (NT / 16) NS own columns live in registers (slot
// lc / (NT / 16) of that lane group; lane q holds the rows q, q + 16, ..., RMAX of them, so the
// tier needs m <= 16 RMAX); the next lcols in the member's LDS (lcol, column at
// lcol + (lc - (NT / 16) NS) (m | 1)); the rest in the workspace gcol.  RMAX = 0 turns the
// register tier off.
//
// reflector entries read ahead by the register tier's row loops (a scheduling barrier between
// groups keeps the compiler from issuing all RMAX loads at once)
constexpr int REG_CHUNK = 8;
// reflectors the register-tier Q formation stages in LDS at a time
constexpr int FQ_RB = 8;
// Register slots a lane group holds (RMAX rows each): 64 FP64 values a lane (at least one
// slot), or up to 4 slots of FP32, the same for the pivoted QR and the Q formation.  Larger
// tiers make the compiler spill slots in the pivot-step loop (the kernel holds 512 threads, so
// a lane has 256 registers).
template <int RMAX, class R>
__host__ __device__ constexpr int reg_slots() {
  return RMAX == 0 ? 0 : sizeof(R) == 8 ? (64 / RMAX > 1 ? 64 / RMAX : 1) : (128 / RMAX < 4 ? 128 / RMAX : 4);
}

// Each value passes through an empty asm statement, so the compiler cannot merge the slots'
// branches into one load of ra at the runtime index k (which would keep ra in scratch memory).
// DEV: device-scope stores (a team's publication slot), else plain stores (LDS).
template <int RMAX, int NS, bool DEV, class R>
__device__ __attribute__((always_inline)) inline void reg_put(const R (&ra)[NS][RMAX], int k, int lane, R* dst) {
#pragma unroll
  for (int kk = 0; kk < NS; ++kk)
    if (kk == k) {
#pragma unroll
      for (int u = 0; u < RMAX; ++u) {
        R x = ra[kk][u];
        asm volatile("" : "+v"(x));
        if constexpr (DEV) st_dev(dst + lane + PL * u, x);
        else dst[lane + PL * u] = x;
      }
    }
}

// Householder QR with column pivoting of the m x n row-major M, truncated at the first step
// whose pivot column norm is <= tol times the first one (RRQR with threshold eps_A of
// Sec. 3.2.1).  Pivot: the lowest-position column whose trailing norm is within a relative
// band (1e-11 in FP64, 2e-6 in FP32) of the largest, so norms equal in exact arithmetic
// (orthonormal basis columns) tie whatever the rounding.  Trailing norms are recomputed every
// step as row sums (formed while the previous reflector is applied; never downdated).
// Columns stay where they are: column c is owned by member c mod G and, inside it, by the
// lane group (c / G) mod (NT / 16); its pivot-order position is tracked in pos / at (LDS of
// every member, n entries each), so a swap of positions s and p is the column exchange of the
// textbook algorithm.  M is read once, into the column storage above (registers, LDS lcol,
// workspace gcol with column c at gcol + c m).  In a team each member publishes its candidate
// column in pub before the exchange (2 G slots of m entries, of 16 RMAX with the register
// tier); a lone workgroup stages a register column in vsh.  The pivot column is read by every
// member to form the reflector (vsh: LDS of max(m, 16 RMAX) entries).
// Reflector s is written to row s of V (ldv) with V[s][s] = 1, its scale to tau[s]; lnr (LDS,
// n / G entries) holds the member's own columns' trailing norms (column c at lnr[c / G]), and
// nrm (device memory, 2 entries) passes the pivot's norm after an ambiguous merge.  M is left
// unchanged (R is not formed).  Returns the rank; ratio (if given) receives |R_kk| / (tol |R_11|)
// of the last kept and of the first rejected pivot.
template <int NT, int RMAX, class R>
__device__ inline int t_cpqr(Team<NT>& T, int m, int n, const R* M, int ldm, double tol, R* V, int ldv, R* tau,
                             R* nrm, R* lnr, ValIdx* shv, R* vsh, int* pos, int* at, double* ratio, R* lcol,
                             int lcols, R* pub, R* gcol) {
  __shared__ double shmx[NT / WAVE];
  __shared__ int shmn[NT / WAVE];
  __shared__ PivState psres[1];
  constexpr int NGW = NT / PL;  // lane groups per workgroup
  constexpr int NS = reg_slots<RMAX, R>();
  constexpr int NREG = NGW * NS;  // own columns in registers
  // loads in flight a lane for the columns outside registers (fewer beside more register slots)
  constexpr int GB = NS == 0 ? COL_BG : NS >= 3 ? 2 : 8;
  const int PS = NS > 0 ? PL * RMAX : m;  // entries of a publication slot
  // pivot ties: norms within a relative band of the largest (1e-11 in FP64, 2e-6 in FP32)
  const R keep = sizeof(R) == 4 ? R(1.0 - 2e-6) : R(1.0 - 1e-11);
  const R tolr = (R)tol;
  const int lstride = m | 1;  // odd column stride: the groups of a wave start on distinct banks
  // a column outside the register tier: LDS, then workspace
  auto colp = [&](int lc, int c) -> R* {
    const int l = lc - NREG;
    return l < lcols ? lcol + (size_t)l * lstride : gcol + (size_t)c * m;
  };
  const int lane = (int)threadIdx.x & (PL - 1), grp = (int)threadIdx.x / PL;
  const int nloc = (n - T.member + T.G - 1) / T.G;  // own columns: c = member + G lc
  double kept = 0.0, next = 0.0;
  int smax = m < n ? m : n;
  R r11 = 0;
  R ra[NS > 0 ? NS : 1][RMAX > 0 ? RMAX : 1];
  // own columns into column storage, with their norms
  if constexpr (NS > 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int lc = grp + NGW * k;
      const int c = T.member + T.G * lc;
      const bool own = lc < nloc;
      R t = 0;
#pragma unroll
      for (int u = 0; u < RMAX; ++u) {
        const int i = lane + PL * u;
        const R a = (own && i < m) ? M[(size_t)i * ldm + c] : R(0);
        ra[k][u] = a;
        if (i < m) t = fma(a, a, t);
      }
      t = lane_sum16(t);
      if (own && lane == 0) lnr[lc] = sqrt(t);
    }
  }
  for (int lc = NREG + grp; lc < nloc; lc += NGW) {
    const int c = T.member + T.G * lc;
    R* d = colp(lc, c);
    R t = 0;
    for (int i0 = lane; i0 < m; i0 += PL * GB) {
      R a[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        int i = i0 + PL * u;
        a[u] = i < m ? M[(size_t)i * ldm + c] : R(0);
      }
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        int i = i0 + PL * u;
        if (i < m) {
          d[i] = a[u];
          t = fma(a[u], a[u], t);
        }
      }
    }
    t = lane_sum16(t);
    if (lane == 0) lnr[lc] = sqrt(t);
  }
  for (int c = threadIdx.x; c < n; c += NT) {
    pos[c] = c;
    at[c] = c;
  }
  // the register tier runs every row of its slots: the rows m .. 16 RMAX - 1 hold zeros in
  // the columns and in vsh, whose entries below s are zero too, so those rows add exact zeros
  // to the row sums and leave the column values as they are
  for (int i = m + (int)threadIdx.x; i < PL * RMAX; i += NT) vsh[i] = R(0);
  __syncthreads();
  // the rows s..m-1 of own column cc (lc = cc / G) into dst: by its lane group from registers
  // (all 16 RMAX rows of the slot; the rows below s are not read), else by the whole
  // workgroup; device-scope stores into a team's publication slot (dev), plain ones into LDS
  auto publish = [&](int cc, R* dst, int s, bool dev) {
    const int lc = cc / T.G;
    if (lc < NREG) {
      if constexpr (NS > 0)
        if (grp == lc % NGW) {
          if (dev) reg_put<RMAX, NS, true>(ra, lc / NGW, lane, dst);
          else reg_put<RMAX, NS, false>(ra, lc / NGW, lane, dst);
        }
    } else {
      const R* src = colp(lc, cc);
      if (dev)
        for (int i = s + threadIdx.x; i < m; i += NT) st_dev(dst + i, src[i]);
      else
        for (int i = s + threadIdx.x; i < m; i += NT) dst[i] = src[i];
    }
  };
  int s = 0;
  for (; s < smax; ++s) {
    // the member's exact pivot (the largest live norm of its columns, then the lowest position
    // within the tie band of it), then one exchange across the team that merges the members'
    // states; the exact two-pass selection over the team runs only when the merge reports an
    // ambiguity
    double mxl = -1.0;
    for (int c = T.cid; c < n; c += T.GT)
      if (pos[c] >= s) mxl = fmax(mxl, (double)lnr[c / T.G]);
    const double mxw = wg_max<NT>(mxl, shmx);
    const R thrw = (R)mxw * keep;
    int pl = INT_MAX;
    for (int c = T.cid; c < n; c += T.GT)
      if (pos[c] >= s && lnr[c / T.G] >= thrw && pos[c] < pl) pl = pos[c];
    const int pw = wg_min<NT>(pl, shmn);
    PivState ps{mxw, pw != INT_MAX ? (double)lnr[at[pw] / T.G] : -1.0, pw, 0};
    // a team: each member publishes its candidate column (rows s..m-1) before the exchange, in
    // a buffer alternating with the step parity
    R* slot = pub + ((size_t)(s & 1) * T.G + T.member) * PS;
    if (T.G > 1 && ps.p != INT_MAX) publish(at[ps.p], slot, s, true);
    if (T.G > 1) {
      // the members' states through their flags: lane q of the first wave takes members q,
      // q + 64, ..., then a tree across the wave (any pairing gives the same state)
      ps = T.exchange_merge(Cand{ps.mx, ps.nv, ps.p, ps.amb}, keep, psres,
                            [&](const PivState& a, const PivState& b) { return piv_merge(a, b, keep); },
                            [&](const PivState& a) { return wave_pivmerge(a, keep); });
      if (T.bad) break;  // the members' candidates may be stale: no pivot is taken from them
    }
    int pp = ps.p;
    bool amb = ps.amb != 0;
    if (amb) {  // exact rule: team maximum, then the lowest position within its band
      ValIdx mx{-1.0, INT_MAX};
      for (int c = T.cid; c < n; c += T.GT)
        if (pos[c] >= s) {
          ValIdx x{(double)lnr[c / T.G], pos[c]};
          if (vi_better(x, mx)) mx = x;
        }
      mx = T.argmax(mx, shv);
      R thr = (R)mx.v * keep;
      ValIdx b2{-1.0, INT_MAX};
      for (int c = T.cid; c < n; c += T.GT)
        if (pos[c] >= s && lnr[c / T.G] >= thr && pos[c] < b2.i) b2 = ValIdx{0.0, pos[c]};
      pp = T.argmax(b2, shv).i;
      if (T.bad) break;
    }
    if (pp < s || pp >= n) break;  // no live column (cannot happen while s < min(m, n))
    const int cp = at[pp];
    // the pivot's norm: carried by the merged candidate state (its nv is the norm of the column
    // at position p); after the exact fallback the owner publishes it (nrm, alternating with
    // the step parity) with the column
    R bv = (R)ps.nv;
    // where the pivot column is read from: the owner's publication slot (a team), the LDS
    // staging copy in vsh (a lone workgroup's register column), or its storage
    const R* pcol;
    bool staged = false;
    if (T.G > 1) {
      const int owner = cp % T.G;
      R* oslot = pub + ((size_t)(s & 1) * T.G + owner) * PS;
      if (amb) {  // the chosen column may not be its owner's candidate: publish it
        if (T.member == owner) {
          publish(cp, oslot, s, true);
          if (threadIdx.x == 0) nrm[s & 1] = lnr[cp / T.G];
        }
        T.sync();
        if (T.bad) break;
        bv = nrm[s & 1];
      }
      pcol = oslot;
    } else {
      if (amb) bv = lnr[cp / T.G];
      pcol = nullptr;
    }
    if (s == 0) {
      r11 = bv;
      if (r11 == R(0)) break;
    } else if (bv <= tolr * r11) {
      next = (double)bv / ((double)tolr * (double)r11);
      break;
    }
    kept = (double)bv / ((double)tolr * (double)r11);
    if (T.G == 1) {
      if (cp < NREG) {
        publish(cp, vsh, s, false);
        staged = true;
        pcol = vsh;
      } else {
        pcol = colp(cp, cp);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int cs = at[s];
      at[s] = cp;
      at[pp] = cs;
      pos[cp] = s;
      pos[cs] = pp;
    }
    // the thread's rows of the pivot column are read together with x0 (one memory latency);
    // a team's publication slot with device-scope loads
    const bool pdev = T.G > 1;
    auto pget = [&](int i) -> R { return pdev ? ld_dev(pcol + i) : pcol[i]; };
    constexpr int PV = 2;
    R pv[PV];
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int i = (int)threadIdx.x + k * NT;
      pv[k] = (i > s && i < m) ? pget(i) : R(0);
    }
    R x0 = pget(s);
    R beta = x0 >= R(0) ? -bv : bv;
    R scale = x0 - beta;
    R tv = (beta - x0) / beta;
    if (staged) __syncthreads();  // pcol read by every thread before vsh is overwritten in place
#pragma unroll
    for (int k = 0; k < PV; ++k) {
      const int i = (int)threadIdx.x + k * NT;
      if (i < m) {
        R v = 0;
        if (i == s) v = 1;
        else if (i > s) v = pv[k] / scale;
        vsh[i] = v;
        if (T.member == 0 && i >= s) V[(size_t)s * ldv + i] = v;
      }
    }
    for (int i = (int)threadIdx.x + PV * NT; i < m; i += NT) {
      R v = 0;
      if (i == s) v = 1;
      else if (i > s) v = pget(i) / scale;
      vsh[i] = v;
      if (T.member == 0 && i >= s) V[(size_t)s * ldv + i] = v;
    }
    if (T.member == 0 && threadIdx.x == 0) tau[s] = tv;
    __syncthreads();
    // apply the reflector to the own live columns: w = tau v^T a over rows s..m-1, a -= w v,
    // and the new trailing norm over rows s+1..m-1
    if constexpr (NS > 0) {
      // every row of every slot: a column no longer live (a pivot already taken) is not read
      // again, so it may be updated as well; only its norm is not stored
      R acc[NS], w[NS], t[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        acc[k] = 0;
        t[k] = 0;
      }
#pragma unroll
      for (int u = 0; u < RMAX; ++u) {
        if (u % REG_CHUNK == 0) __builtin_amdgcn_sched_barrier(0);
        const R vv = vsh[lane + PL * u];
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] = fma(vv, ra[k][u], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) w[k] = lane_sum16(acc[k]) * tv;
      // vsh is read again rather than kept: its RMAX values would double the tier's registers
      asm volatile("" ::: "memory");
#pragma unroll
      for (int u = 0; u < RMAX; ++u) {
        if (u % REG_CHUNK == 0) __builtin_amdgcn_sched_barrier(0);
        const R vv = vsh[lane + PL * u];
        const bool below = lane + PL * u > s;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const R x = fma(-w[k], vv, ra[k][u]);
          ra[k][u] = x;
          const R xs = below ? x : R(0);
          t[k] = fma(xs, xs, t[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const R tt = lane_sum16(t[k]);
        const int lc = grp + NGW * k;
        if (lane == 0 && lc < nloc && pos[T.member + T.G * lc] > s) lnr[lc] = sqrt(tt);
      }
    }
    const int r0 = s + ((lane - s) & (PL - 1));  // this lane's first row >= s
    for (int lc = NREG + grp; lc < nloc; lc += NGW) {
      const int c = T.member + T.G * lc;
      if (pos[c] <= s) continue;
      R* col = colp(lc, c);
      R acc, t;
      if constexpr (NS > 0) {  // one path for LDS and workspace columns, few registers
        acc = grp_dot<GB>(col, vsh, r0, m);
        const R w = lane_sum16(acc) * tv;
        t = grp_axpy<GB, true>(col, vsh, r0, m, s, w);
      } else {
        const bool inl = lc - NREG < lcols;
        acc = inl ? grp_dot<COL_B>(col, vsh, r0, m) : grp_dot<COL_BG>(col, vsh, r0, m);
        const R w = lane_sum16(acc) * tv;
        t = inl ? grp_axpy<COL_B, true>(col, vsh, r0, m, s, w) : grp_axpy<COL_BG, true>(col, vsh, r0, m, s, w);
      }
      t = lane_sum16(t);
      if (lane == 0) lnr[lc] = sqrt(t);
    }
    __syncthreads();
  }
  if (ratio && T.gtid == 0) {
    ratio[0] = kept;
    ratio[1] = next;
  }
  T.sync();
  return s;
}

// Columns c0 .. q-1 of Q = H_0 ... H_{rank-1} [I; 0] (m x q, ldq); columns below c0 are left
// as they are (already formed).  Reflector s is row s of V (ldv), as t_cpqr writes it.  Column
// j is owned by member (j - c0) mod G (own index lj = (j - c0) / G) and formed by one lane
// group through all reflectors (row sums in the fixed order of lane_sum16), then written to
// Q, so members only synchronise at the end.  With the register tier (RMAX > 0) the columns
// are independent, so the member forms them in passes of (NT / 16) NS register columns, with
// the reflectors staged in lcol (FQ_RB 16 RMAX entries, which the host reserves); without it a
// column lives in the member's LDS (lcol, lcols columns of stride m | 1) or the workspace gcol
// (column j at gcol + (j - c0) m).
template <int NT, int RMAX, class R>
__device__ inline void t_formq(Team<NT>& T, int m, int rank, int q, const R* V, int ldv, const R* tau, R* Q, int ldq,
                               R* vsh, int c0, R* lcol, int lcols, R* gcol) {
  if (q <= c0) return;  // nothing to form (uniform over the team)
  constexpr int NGW = NT / PL;
  constexpr int NS = reg_slots<RMAX, R>();
  const int lane = (int)threadIdx.x & (PL - 1), grp = (int)threadIdx.x / PL;
  const int nloc = (q - c0 - T.member + T.G - 1) / T.G;  // own columns: j = c0 + member + G lj
  if constexpr (NS > 0) {
    constexpr int NREG = NGW * NS;
    // every row of every slot, with the reflector zero outside the rows s..m-1: the columns
    // hold exact zeros beyond row m, and the rows of a column that a reflector does not reach
    // are +0 or the 1 of e_j, which adding exact zeros leaves as they are.  The reflectors are
    // staged FQ_RB at a time in the member's LDS column region (free here: FQ_RB rows of
    // 16 RMAX entries) and applied one after another, in descending order, without a barrier
    // between them (the columns are independent and the staged rows read-only).
    constexpr int RR = PL * RMAX;
    R* vb = lcol;
    __shared__ R tb[FQ_RB];
    for (int p0 = 0; p0 < nloc; p0 += NREG) {
      R ra[NS][RMAX];
      // the first own column of the pass through an empty asm statement: the compiler cannot
      // form the pass's columns ahead of their use (above earlier loops), where they would
      // hold registers
      int jp = c0 + T.member + T.G * p0;
      asm volatile("" : "+v"(jp));
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int j = jp + T.G * (grp + NGW * k);
#pragma unroll
        for (int u = 0; u < RMAX; ++u) ra[k][u] = (lane + PL * u == j) ? R(1) : R(0);
      }
      for (int sb = rank - 1; sb >= 0; sb -= FQ_RB) {
        const int nb = sb + 1 < FQ_RB ? sb + 1 : FQ_RB;  // reflectors sb, sb - 1, .., sb - nb + 1
        __syncthreads();
        for (int idx = threadIdx.x; idx < nb * RR; idx += NT) {
          const int b = idx / RR, i = idx - b * RR, s = sb - b;
          vb[idx] = (i >= s && i < m) ? V[(size_t)s * ldv + i] : R(0);
        }
        if ((int)threadIdx.x < nb) tb[threadIdx.x] = tau[sb - (int)threadIdx.x];
        __syncthreads();
        // a wave whose lane groups hold none of the pass's columns (its first, p0 + its first
        // group, is past the member's columns) skips the arithmetic; there is no barrier in it
        if (p0 + (int)(threadIdx.x / WAVE) * (WAVE / PL) >= nloc) continue;
        for (int b = 0; b < nb; ++b) {
          const R* vr = vb + b * RR;
          const R tv = tb[b];
          R acc[NS], w[NS];
#pragma unroll
          for (int k = 0; k < NS; ++k) acc[k] = 0;
#pragma unroll
          for (int u = 0; u < RMAX; ++u) {
            if (u % REG_CHUNK == 0) __builtin_amdgcn_sched_barrier(0);
            const R vv = vr[lane + PL * u];
#pragma unroll
            for (int k = 0; k < NS; ++k) acc[k] = fma(vv, ra[k][u], acc[k]);
          }
#pragma unroll
          for (int k = 0; k < NS; ++k) w[k] = lane_sum16(acc[k]) * tv;
          // the row is read again rather than kept: its RMAX values would double the tier's
          // registers
          asm volatile("" ::: "memory");
#pragma unroll
          for (int u = 0; u < RMAX; ++u) {
            if (u % REG_CHUNK == 0) __builtin_amdgcn_sched_barrier(0);
            const R vv = vr[lane + PL * u];
#pragma unroll
            for (int k = 0; k < NS; ++k) ra[k][u] = fma(-w[k], vv, ra[k][u]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int lj = p0 + grp + NGW * k;
        if (lj < nloc) {
          const int j = c0 + T.member + T.G * lj;
#pragma unroll
          for (int u = 0; u < RMAX; ++u) {
            const int i = lane + PL * u;
            if (i < m) Q[(size_t)i * ldq + j] = ra[k][u];
          }
        }
      }
    }
  } else {
    const int lstride = m | 1;
    auto colp = [&](int lj, int j) -> R* {
      return lj < lcols ? lcol + (size_t)lj * lstride : gcol + (size_t)(j - c0) * m;
    };
    for (int lj = grp; lj < nloc; lj += NGW) {
      const int j = c0 + T.member + T.G * lj;
      R* col = colp(lj, j);
      for (int i = lane; i < m; i += PL) col[i] = (i == j) ? R(1) : R(0);
    }
    for (int s = rank - 1; s >= 0; --s) {
      R tv = tau[s];
      __syncthreads();
      for (int i = s + threadIdx.x; i < m; i += NT) vsh[i] = V[(size_t)s * ldv + i];
      __syncthreads();
      const int j0 = c0 > s ? c0 : s;
      const int r0 = s + ((lane - s) & (PL - 1));
      // a column is still e_j while s > j, so the reflector leaves it unchanged
      for (int lj = grp; lj < nloc; lj += NGW) {
        const int j = c0 + T.member + T.G * lj;
        if (j < j0) continue;
        R* col = colp(lj, j);
        const bool inl = lj < lcols;
        const R acc = inl ? grp_dot<COL_B>(col, vsh, r0, m) : grp_dot<COL_BG>(col, vsh, r0, m);
        const R w = lane_sum16(acc) * tv;
        if (inl) grp_axpy<COL_B, false>(col, vsh, r0, m, s, w);
        else grp_axpy<COL_BG, false>(col, vsh, r0, m, s, w);
      }
    }
    __syncthreads();
    for (int lj = grp; lj < nloc; lj += NGW) {
      const int j = c0 + T.member + T.G * lj;
      const R* col = colp(lj, j);
      for (int i = lane; i < m; i += PL) Q[(size_t)i * ldq + j] = col[i];
    }
  }
  T.sync();
}

// LU with row partial pivoting of the m x m row-major A (ties to the lowest row; ipiv[k] = the
// row swapped with row k at step k), blocked in NB-column panels over a team of 256-thread
// workgroups.  Every element receives its updates a = fma(-l, u, a) one at a time in ascending
// step order and every pivot is chosen from the fully updated column, so the factors are bit
// for bit those of the textbook elimination.  Member 0 factors each panel (in its LDS panel
// buffer pl, m (NB + 1) doubles, when use_pl) and leaves the panel and its pivots in A and
// ipiv; after a team barrier every member applies the panel's row swaps, in step order, to
// its share of the other columns and solves their U12 rows with the panel's unit-lower L11;
// after another the members take the 64 x 64 tiles of the trailing update in turn (FP64
// MFMA accumulating onto the current entries in ascending step order); a third barrier ends
// the panel.  sh: LDS of NB + 64 (NB + 1) + 65 NB doubles; ipv: NB ints of LDS.  status
// (device memory) carries member 0's result (0, or 1 + the step of an exactly zero pivot) to
// the team; the return value is the same on every member.
template <int NB>
__device__ inline int t_lu_blocked(Team<WG>& T, int m, double* A, int lda, int* ipiv, ValIdx* shv, double* sh,
                                   int* ipv, double* pl, bool use_pl, int* status) {
  constexpr int NT = WG;
  const int tid = threadIdx.x;
  double* prow = sh;
  double* Ls = sh + NB;                // [64][NB + 1]
  double* Us = Ls + 64 * (NB + 1);     // [NB][65]
  if (T.member == 0 && tid == 0) *status = 0;
  for (int k0 = 0; k0 < m; k0 += NB) {
    const int nb = min(NB, m - k0);
    if (T.member == 0) {
      const bool lp = use_pl;  // a flag, not a null test of the LDS pointer
      auto el = [&](int i, int j) -> double* {
        return lp ? pl + (size_t)(i - k0) * (NB + 1) + j : A + (size_t)i * lda + k0 + j;
      };
      if (lp) {
        for (int idx = tid; idx < (m - k0) * nb; idx += NT) {
          int r = idx / nb, j = idx - r * nb;
          pl[(size_t)r * (NB + 1) + j] = A[(size_t)(k0 + r) * lda + k0 + j];
        }
        __syncthreads();
      }
      int bad = 0;
      for (int s = 0; s < nb; ++s) {
        const int k = k0 + s;
        ValIdx best{-1.0, INT_MAX};
        for (int i = k + tid; i < m; i += NT) {
          ValIdx c{fabs(*el(i, s)), i};
          if (vi_better(c, best)) best = c;
        }
        best = wg_argmax<NT>(best, shv);
        if (best.v == 0.0) {
          bad = 1 + k;
          break;
        }
        const int p = best.i;
        if (tid == 0) ipiv[k] = p;
        if (p != k)
          for (int j = tid; j < nb; j += NT) {
            double t = *el(k, j);
            *el(k, j) = *el(p, j);
            *el(p, j) = t;
          }
        __syncthreads();
        for (int j = tid; j < nb; j += NT) prow[j] = *el(k, j);
        __syncthreads();
        const double piv = prow[s];
        for (int i = k + 1 + tid; i < m; i += NT) {
          double* row = el(i, 0);
          double as = row[s];
          double v[NB];
#pragma unroll
          for (int j = 0; j < NB; ++j) v[j] = (j > s && j < nb) ? row[j] : 0.0;
          double l = as / piv;
          row[s] = l;
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j > s && j < nb) row[j] = fma(-l, prow[j], v[j]);
        }
        __syncthreads();
      }
      if (bad) {
        if (tid == 0) *status = bad;
      } else if (lp) {
        for (int idx = tid; idx < (m - k0) * nb; idx += NT) {
          int r = idx / nb, j = idx - r * nb;
          A[(size_t)(k0 + r) * lda + k0 + j] = pl[(size_t)r * (NB + 1) + j];
        }
      }
    }
    T.sync();
    if (T.bad) return 1;  // member 0's status and pivots may be stale
    const int st = *(volatile int*)status;
    if (st) return st;
    // the panel's row swaps on every other column, in step order, then the U12 rows of the
    // columns right of the panel (unit-lower L11 from the panel)
    for (int s = tid; s < nb; s += NT) ipv[s] = ipiv[k0 + s];
    const int c1 = k0 + nb;
    for (int idx = tid; idx < nb * nb; idx += NT) {
      int r = idx / nb, t = idx - r * nb;
      Ls[r * (NB + 1) + t] = A[(size_t)(k0 + r) * lda + k0 + t];
    }
    __syncthreads();
    for (int c = T.gtid; c < m; c += T.GT) {
      if (c >= k0 && c < c1) continue;
      for (int s = 0; s < nb; ++s) {
        int r = k0 + s, p = ipv[s];
        if (p != r) {
          double t = A[(size_t)r * lda + c];
          A[(size_t)r * lda + c] = A[(size_t)p * lda + c];
          A[(size_t)p * lda + c] = t;
        }
      }
      if (c >= c1) {
        double u[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) u[t] = t < nb ? A[(size_t)(k0 + t) * lda + c] : 0.0;
#pragma unroll
        for (int r = 1; r < NB; ++r)
#pragma unroll
          for (int t = 0; t < r; ++t)
            if (r < nb) u[r] = fma(-Ls[r * (NB + 1) + t], u[t], u[r]);
#pragma unroll
        for (int t = 1; t < NB; ++t)
          if (t < nb) A[(size_t)(k0 + t) * lda + c] = u[t];
      }
    }
    T.sync();
    if (T.bad) return 1;
    if (c1 >= m) break;
    // A22 -= L21 U12 in 64 x 64 tiles (taken by the members in turn), each wave a 32 x 32
    // quarter as 2 x 2 FP64 MFMA 16x16x4 blocks accumulating onto the current entries
    const int rem = m - c1;
    const int tiles = (rem + 63) / 64;
    const int lane = tid % WAVE, wv = tid / WAVE;
    const int wr = (wv / 2) * 32, wc = (wv % 2) * 32;
    const int fr = lane % 16, fk = lane / 16;
    for (int tt = T.member; tt < tiles * tiles; tt += T.G) {
      int r0 = c1 + (tt / tiles) * 64, cc0 = c1 + (tt % tiles) * 64;
      __syncthreads();
      for (int idx = tid; idx < 64 * NB; idx += NT) {
        int r = idx / NB, t = idx - r * NB;
        int gr = r0 + r;
        Ls[r * (NB + 1) + t] = (gr < m && t < nb) ? -A[(size_t)gr * lda + k0 + t] : 0.0;
      }
      for (int idx = tid; idx < NB * 64; idx += NT) {
        int t = idx / 64, c = idx - t * 64;
        int gc = cc0 + c;
        Us[t * 65 + c] = (gc < m && t < nb) ? A[(size_t)(k0 + t) * lda + gc] : 0.0;
      }
      __syncthreads();
      lu_dbl4 acc[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int gr = r0 + wr + 16 * i + fk + 4 * q, gc = cc0 + wc + 16 * j + fr;
            acc[i][j][q] = (gr < m && gc < m) ? A[(size_t)gr * lda + gc] : 0.0;
          }
#pragma unroll
      for (int k4 = 0; k4 < NB; k4 += 4) {
        double a0 = Ls[(wr + fr) * (NB + 1) + k4 + fk], a1 = Ls[(wr + 16 + fr) * (NB + 1) + k4 + fk];
        double b0 = Us[(k4 + fk) * 65 + wc + fr], b1 = Us[(k4 + fk) * 65 + wc + 16 + fr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int gr = r0 + wr + 16 * i + fk + 4 * q, gc = cc0 + wc + 16 * j + fr;
            if (gr < m && gc < m) A[(size_t)gr * lda + gc] = acc[i][j][q];
          }
    }
    T.sync();
    if (T.bad) return 1;
  }
  return 0;
}

}  // namespace aifmm
