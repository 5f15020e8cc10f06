// A "team" of G co-resident workgroups (NT threads each) working on one dense task, with
// team-wide barriers through a counter in device memory.  G == 1 is a plain workgroup and its
// barrier is __syncthreads().  Team routines distribute their work over the G * NT team
// threads and end with a team barrier, so results are visible to every member on return.
//
// The arithmetic of every output element is done by one thread in the same order as the
// single-workgroup routines of dense_wg.hpp, so results do not depend on G.
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

template <int NT>
struct Team {
  int member = 0, G = 1;      // this workgroup's index in the team, team size
  int gtid = 0, GT = NT;      // team thread index and count
  int cid = 0;                // column-interleaved team thread index: member + G * thread
  unsigned* ctr = nullptr;    // barrier counter (zero at launch)
  Cand* part = nullptr;       // 2 x G exchange slots (double-buffered)
  int* abort = nullptr;       // set when a barrier waited too long; every later barrier returns
  unsigned epoch = 0;
  int slot = 0;

  __device__ void init(int member_, int G_, unsigned* ctr_, Cand* part_, int* abort_) {
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
  // visible to the whole workgroup.  The wait is bounded (a few seconds of polling): on expiry
  // the abort flag is raised and the team falls through, so every workgroup still runs to its
  // end and the host reports the failure.
  __device__ void sync() {
    __syncthreads();
    if (G == 1) return;
    if (threadIdx.x == 0) {
      ++epoch;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(ctr, 1u);
      unsigned target = epoch * (unsigned)G;
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 24)) {
          atomicExch(abort, 1);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  }

  // Publish one value per member and return all G of them (the same array on every thread).
  __device__ const Cand* exchange(const Cand& c) {
    Cand* p = part + slot * G;
    if (threadIdx.x == 0) p[member] = c;
    sync();
    slot ^= 1;
    return p;
  }

  // Team-wide argmax (ties to the lowest index); the same value on every thread of the team.
  __device__ ValIdx argmax(ValIdx x, ValIdx* shv) {
    ValIdx r = wg_argmax<NT>(x, shv);
    if (G == 1) return r;
    const Cand* all = exchange(Cand{r.v, 0.0, r.i, 0});
    ValIdx b{-1.0, INT_MAX};
    for (int q = 0; q < G; ++q) {
      ValIdx c{all[q].mv, all[q].p};
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
// C = alpha op(A) op(B) + beta C, each element accumulated in ascending k in the precision of
// C (as wg_gemm).
template <int NT, class TA, class TB, class TC>
__device__ inline void t_gemm(Team<NT>& T, int M, int N, int K, double alpha, const TA* __restrict__ A, int lda,
                              bool ta, const TB* __restrict__ B, int ldb, bool tb, double beta, TC* C, int ldc) {
  for (int idx = T.gtid; idx < M * N; idx += T.GT) {
    int r = idx / N, c = idx - r * N;
    const TA* pa = ta ? A + r : A + (size_t)r * lda;
    const TB* pb = tb ? B + (size_t)c * ldb : B + c;
    size_t sa = ta ? (size_t)lda : 1, sb = tb ? 1 : (size_t)ldb;
    TC acc = seq_dot(K, [&](int k) { return (TC)pa[k * sa]; }, [&](int k) { return (TC)pb[k * sb]; }, (TC)0);
    TC v = (TC)alpha * acc;
    if (beta != 0.0) v += (TC)beta * C[(size_t)r * ldc + c];
    C[(size_t)r * ldc + c] = v;
  }
  T.sync();
}

// Pivot candidate state for one pass over the live columns: the largest norm mx, the lowest
// position p among the columns whose norm is >= keep * mx, that column's norm nv, and amb set
// when merging lost the information needed to know p exactly (a column within the band of a
// smaller maximum that may or may not reach the band of the larger one).  Merging is
// associative; when amb is clear, p is exactly the pivot of the two-pass rule.
struct PivState {
  double mx, nv;
  int p, amb;
};
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
// Workgroup-wide merge of the per-thread states (the same result on every thread).
template <int NT, class R>
__device__ inline PivState wg_pivmerge(PivState x, R keep, PivState* sh) {
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    PivState o;
    o.mx = __shfl_down(x.mx, off, WAVE);
    o.nv = __shfl_down(x.nv, off, WAVE);
    o.p = __shfl_down(x.p, off, WAVE);
    o.amb = __shfl_down(x.amb, off, WAVE);
    x = piv_merge(x, o, keep);
  }
  int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    PivState b = sh[0];
    for (int q = 1; q < NT / WAVE; ++q) b = piv_merge(b, sh[q], keep);
    sh[NT / WAVE] = b;
  }
  __syncthreads();
  PivState r = sh[NT / WAVE];
  return r;
}

// Householder QR with column pivoting of the m x n row-major M, truncated at the first step
// whose pivot column norm is <= tol times the first one (RRQR with threshold eps_A of
// Sec. 3.2.1).  Pivot: the lowest-position column whose trailing norm is within a relative
// band (1e-11 in FP64, 2e-6 in FP32) of the largest, so norms equal in exact arithmetic
// (orthonormal basis columns) tie whatever the rounding.  Trailing norms are recomputed every
// step as sums over the rows in ascending order (formed while the previous reflector is
// applied; never downdated).  Columns stay where they are: column c is owned by member c mod G
// (columns interleave across members), and its pivot-order position is tracked in pos / at
// (LDS of every member, n entries each), so a swap of positions s and p is the column exchange
// of the textbook algorithm.  The pivot column is read by every member to form the reflector
// (vsh: m entries of LDS).  Reflector s is written to column s of V (ldv) with V[s][s] = 1, its
// scale to tau[s]; nrm (device memory, n) holds each column's trailing norm.  M's pivot columns
// are left as they were when chosen (R is not formed).  Returns the rank; ratio (if given)
// receives |R_kk| / (tol |R_11|) of the last kept and of the first rejected pivot.
// column passes of the pivoted QR and Q formation keep this many loads in flight per thread
constexpr int COL_B = SEQ_B;
template <int NT, class R>
__device__ inline int t_cpqr(Team<NT>& T, int m, int n, R* M, int ldm, double tol, R* V, int ldv, R* tau, R* nrm,
                             ValIdx* shv, R* vsh, int* pos, int* at, double* ratio, R* lcol, R* pub) {
  __shared__ PivState psh[NT / WAVE + 1];
  // pivot ties: norms within a relative band of the largest (1e-11 in FP64, 2e-6 in FP32)
  const R keep = sizeof(R) == 4 ? R(1.0 - 2e-6) : R(1.0 - 1e-11);
  const R tolr = (R)tol;
  // column storage: with lcol the member's own columns are copied to its LDS (column c at
  // lcol + (c / G) m, rows contiguous) and M is only read once; otherwise M in place
  const bool lds = lcol != nullptr;
  const int lstride = m | 1;  // odd column stride: the lanes of a wave hit distinct LDS banks
  auto cptr = [&](int c) -> R* { return lds ? lcol + (size_t)(c / T.G) * lstride : M + c; };
  const size_t cst = lds ? 1 : (size_t)ldm;
  double kept = 0.0, next = 0.0;
  int smax = m < n ? m : n;
  R r11 = 0;
  if (lds)
    for (int c = T.cid; c < n; c += T.GT) {
      R* d = cptr(c);
      const R* g = M + c;
      int i = 0;
      for (; i + SEQ_B <= m; i += SEQ_B) {
        R a[SEQ_B];
#pragma unroll
        for (int u = 0; u < SEQ_B; ++u) a[u] = g[(size_t)(i + u) * ldm];
#pragma unroll
        for (int u = 0; u < SEQ_B; ++u) d[i + u] = a[u];
      }
      for (; i < m; ++i) d[i] = g[(size_t)i * ldm];
    }
  for (int c = T.cid; c < n; c += T.GT) {
    const R* col = cptr(c);
    R t = seq_dot<COL_B>(m, [&](int i) { return col[i * cst]; }, [&](int i) { return col[i * cst]; }, R(0));
    nrm[c] = sqrt(t);
  }
  for (int c = threadIdx.x; c < n; c += NT) {
    pos[c] = c;
    at[c] = c;
  }
  __syncthreads();
  int s = 0;
  for (; s < smax; ++s) {
    // one merged pass per workgroup, then one exchange across the team: the largest live norm
    // and the lowest position within the tie band of it; the exact two-pass selection runs
    // only when a merge reports an ambiguity
    PivState ps{-1.0, -1.0, INT_MAX, 0};
    for (int c = T.cid; c < n; c += T.GT)
      if (pos[c] >= s) ps = piv_merge(ps, PivState{(double)nrm[c], (double)nrm[c], pos[c], 0}, keep);
    ps = wg_pivmerge<NT>(ps, keep, psh);
    // LDS columns of a team: each member publishes its candidate column (rows s..m-1) before
    // the exchange, in a buffer alternating with the step parity
    R* slot = pub + ((size_t)(s & 1) * T.G + T.member) * m;
    if (lds && T.G > 1 && ps.p != INT_MAX) {
      const R* src = cptr(at[ps.p]);
      for (int i = s + threadIdx.x; i < m; i += NT) slot[i] = src[i];
    }
    if (T.G > 1) {
      const Cand* all = T.exchange(Cand{ps.mx, ps.nv, ps.p, ps.amb});
      PivState g{-1.0, -1.0, INT_MAX, 0};
      for (int q = 0; q < T.G; ++q) g = piv_merge(g, PivState{all[q].mv, all[q].nv, all[q].p, all[q].pad}, keep);
      ps = g;
    }
    int pp = ps.p;
    bool amb = ps.amb != 0;
    if (amb) {  // exact rule: team maximum, then the lowest position within its band
      ValIdx mx{-1.0, INT_MAX};
      for (int c = T.cid; c < n; c += T.GT)
        if (pos[c] >= s) {
          ValIdx x{(double)nrm[c], pos[c]};
          if (vi_better(x, mx)) mx = x;
        }
      mx = T.argmax(mx, shv);
      R thr = (R)mx.v * keep;
      ValIdx b2{-1.0, INT_MAX};
      for (int c = T.cid; c < n; c += T.GT)
        if (pos[c] >= s && nrm[c] >= thr && pos[c] < b2.i) b2 = ValIdx{0.0, pos[c]};
      pp = T.argmax(b2, shv).i;
    }
    const int cp = at[pp];
    const R bv = nrm[cp];
    if (s == 0) {
      r11 = bv;
      if (r11 == R(0)) break;
    } else if (bv <= tolr * r11) {
      next = (double)bv / ((double)tolr * (double)r11);
      break;
    }
    kept = (double)bv / ((double)tolr * (double)r11);
    // where the pivot column is read from
    const R* pcol = M + cp;
    size_t pst = (size_t)ldm;
    if (lds) {
      pst = 1;
      if (T.G == 1) {
        pcol = cptr(cp);
      } else {
        const int owner = cp % T.G;
        R* oslot = pub + ((size_t)(s & 1) * T.G + owner) * m;
        if (amb) {  // the chosen column may not be its owner's candidate: publish it
          if (T.member == owner) {
            const R* src = cptr(cp);
            for (int i = s + threadIdx.x; i < m; i += NT) oslot[i] = src[i];
          }
          T.sync();
        }
        pcol = oslot;
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
    R x0 = pcol[(size_t)s * pst];
    R beta = x0 >= R(0) ? -bv : bv;
    R scale = x0 - beta;
    R tv = (beta - x0) / beta;
    for (int i = threadIdx.x; i < m; i += NT) {
      R v = 0;
      if (i == s) v = 1;
      else if (i > s) v = pcol[(size_t)i * pst] / scale;
      vsh[i] = v;
      if (T.member == 0) V[(size_t)i * ldv + s] = v;
    }
    if (T.member == 0 && threadIdx.x == 0) tau[s] = tv;
    __syncthreads();
    const int len = m - s;
    const R* vv = vsh + s;
    for (int c = T.cid; c < n; c += T.GT) {
      if (pos[c] <= s) continue;
      R* col = cptr(c) + (size_t)s * cst;
      R w = seq_dot<COL_B>(len, [&](int i) { return vv[i]; }, [&](int i) { return col[i * cst]; }, R(0));
      w *= tv;
      col[0] = fma(-w, vv[0], col[0]);
      R t = 0;
      int i = 1;
      for (; i + COL_B <= len; i += COL_B) {
        R a[COL_B];
#pragma unroll
        for (int u = 0; u < COL_B; ++u) a[u] = col[(i + u) * cst];
#pragma unroll
        for (int u = 0; u < COL_B; ++u) {
          a[u] = fma(-w, vv[i + u], a[u]);
          col[(i + u) * cst] = a[u];
          t = fma(a[u], a[u], t);
        }
      }
      for (; i < len; ++i) {
        R a = fma(-w, vv[i], col[i * cst]);
        col[i * cst] = a;
        t = fma(a, a, t);
      }
      nrm[c] = sqrt(t);
    }
  }
  if (ratio && T.gtid == 0) {
    ratio[0] = kept;
    ratio[1] = next;
  }
  T.sync();
  return s;
}

// Columns c0 .. q-1 of Q = H_0 ... H_{rank-1} [I; 0] (m x q, ldq); columns below c0 are left
// as they are (already formed).  Every column is
// formed by one team thread through all reflectors, so members only synchronise at the end.
template <int NT, class R>
__device__ inline void t_formq(Team<NT>& T, int m, int rank, int q, const R* V, int ldv, const R* tau, R* Q, int ldq,
                               R* vsh, int c0, R* lcol) {
  // with lcol every column is formed in the member's LDS (column j at lcol + ((j - c0) / G) m)
  // and written to Q at the end
  if (q <= c0) return;  // nothing to form (uniform over the team)
  const bool lds = lcol != nullptr;
  const int lstride = m | 1;
  auto cptr = [&](int j) -> R* { return lds ? lcol + (size_t)((j - c0) / T.G) * lstride : Q + j; };
  const size_t cst = lds ? 1 : (size_t)ldq;
  for (int j = c0 + T.cid; j < q; j += T.GT) {
    R* col = cptr(j);
    for (int r = 0; r < m; ++r) col[r * cst] = (r == j) ? R(1) : R(0);
  }
  for (int s = rank - 1; s >= 0; --s) {
    R tv = tau[s];
    __syncthreads();
    for (int i = s + threadIdx.x; i < m; i += NT) vsh[i] = V[(size_t)i * ldv + s];
    __syncthreads();
    int len = m - s;
    const R* vv = vsh + s;
    int j0 = c0 > s ? c0 : s;
    // a column is still e_j while s > j, so the reflector leaves it unchanged
    for (int j = c0 + T.cid; j < q; j += T.GT) {
      if (j < j0) continue;
      R* col = cptr(j) + (size_t)s * cst;
      R w = seq_dot<COL_B>(len, [&](int i) { return vv[i]; }, [&](int i) { return col[i * cst]; }, R(0));
      w *= tv;
      int i = 0;
      for (; i + COL_B <= len; i += COL_B) {
        R a[COL_B];
#pragma unroll
        for (int u = 0; u < COL_B; ++u) a[u] = col[(i + u) * cst];
#pragma unroll
        for (int u = 0; u < COL_B; ++u) col[(i + u) * cst] = fma(-w, vv[i + u], a[u]);
      }
      for (; i < len; ++i) col[i * cst] = fma(-w, vv[i], col[i * cst]);
    }
  }
  if (lds)
    for (int j = c0 + T.cid; j < q; j += T.GT) {
      const R* col = cptr(j);
      for (int r = 0; r < m; ++r) Q[(size_t)r * ldq + j] = col[r];
    }
  T.sync();
}

}  // namespace aifmm
