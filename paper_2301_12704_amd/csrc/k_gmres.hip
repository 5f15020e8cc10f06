// Exact FP64 matrix-vector product with the kernel matrix and right-preconditioned flexible
// GMRES with the AIFMM factorization as preconditioner (the paper uses AIFMM as a GMRES
// preconditioner in Sec. 4, Experiment 5, with the relative residual ||A x - b|| / ||b|| as
// stopping rule, Table of notations).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "dense_wg.hpp"
#include "system.hpp"

namespace aifmm {

// 1 / sqrt(x) for x > 0: the hardware estimate refined by two Newton steps on 1 - x y^2
// (about one ulp; the operator's entries need not match the factorization's bit for bit).
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

typedef double mv_dbl4 __attribute__((ext_vector_type(4)));
__device__ inline mv_dbl4 mv_mfma(double a, double b, mv_dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// y[i, c] = sum_j A_ij x[j, c] for the points in tree order; x, y row-major (N x nr).
// Every entry is evaluated once: a wave owns 16 targets and a block of MV_R right-hand sides;
// lane (fr, fk) evaluates the entry of target fr and source 4 s + fk as the A operand of one FP64
// MFMA 16x16x4 per step s, the staged right-hand sides of the four sources are the B operand.
// The MFMA adds its four products one fused multiply-add at a time in ascending k, so every
// output is the ascending fused multiply-add chain over the sources, as a sequential loop.
// KIND and the dimension D are template arguments.
constexpr int MV_T = 256, MV_S = 256, MV_R = 16;
template <int KIND, int D>
__global__ void __launch_bounds__(MV_T) k_matvec(KernelDesc K, const double* __restrict__ pts, int64_t N,
                                                 const double* __restrict__ x, int nr, double* __restrict__ y) {
  __shared__ double sp[MV_S * D];
  __shared__ double sx[MV_S * MV_R];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, fr = lane % 16, fk = lane / 16;
  const int64_t tile0 = (int64_t)blockIdx.x * (MV_T / WAVE * 16) + wv * 16;
  const int64_t i = tile0 + fr;  // the target of this lane's A rows
  const int c0 = blockIdx.y * MV_R;
  const int nc = min(MV_R, nr - c0);
  double pi[D];
#pragma unroll
  for (int t = 0; t < D; ++t) pi[t] = i < N ? pts[i * D + t] : 0.0;
  const double s2 = K.scale * K.scale;
  mv_dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t j0 = 0; j0 < N; j0 += MV_S) {
    const int cnt = (int)std::min<int64_t>(MV_S, N - j0);
    __syncthreads();
    for (int q = threadIdx.x; q < cnt * D; q += MV_T) sp[q] = pts[j0 * D + q];
    for (int q = threadIdx.x; q < MV_S * MV_R; q += MV_T) {  // rows past cnt are zero
      const int jj = q / MV_R, c = q % MV_R;
      sx[q] = (jj < cnt && c < nc) ? x[(j0 + jj) * nr + c0 + c] : 0.0;
    }
    __syncthreads();
    const int steps = (cnt + 3) / 4;
#pragma unroll 4
    for (int st = 0; st < steps; ++st) {
      const int jj = 4 * st + fk;
      double v = 0.0;
      if (jj < cnt && i < N) {
        double r2 = 0.0;
#pragma unroll
        for (int t = 0; t < D; ++t) {
          const double z = pi[t] - sp[jj * D + t];
          r2 = fma(z, z, r2);
        }
        v = KIND == 0 ? dexp(-sqrt(r2) / K.scale) : rsqrt_nr(r2 + s2);
        if (j0 + jj == i) v += K.shift;
      }
      acc = mv_mfma(v, sx[jj * MV_R + fr], acc);
    }
  }
  // output (lane, q): target tile0 + fk + 4 q, column c0 + fr
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t t = tile0 + fk + 4 * q;
    if (t < N && fr < nc) y[t * nr + c0 + fr] = acc[q];
  }
}

// ------------------------------------------------------------------------------------------
// NNCA-based H^2 product (Sec. 2.3, the operator table; the paper's GMRES operator in Sec. 4):
// far field through the nested NNCA operators of every interaction-list pair, near field of
// the leaf neighbours evaluated exactly.  u = v and a symmetric kernel give V = U, so the
// upward pass applies U^T (P2M at the leaf, M2M above) and the downward pass U (L2L, L2P).
// Vectors are row-major (row, column) in tree order: the points at the leaf, the NNCA ranks of
// the boxes in box order above (the rows of a box's U are the points of the box at the leaf and
// the stacked incoming pivots of its children above, so the rows of box b start at T_off[b]
// in both the level's input and the children's rank vector).
// ------------------------------------------------------------------------------------------

// The per-box products below are 16 x 16 output tiles on FP64 MFMA 16x16x4 (16 rows of the
// result, 16 right-hand sides), one wave per tile, the tiles of a box spread over the waves of
// blockIdx.y; K runs in steps of 4 (terms past K are exact zeros).

// P2M / M2M: q[koff[b] + j] = sum_r U_b[r][j] src[T_off[b] + r].
__global__ void __launch_bounds__(WG) k_h2_up(const double* __restrict__ U, const int64_t* __restrict__ U_off,
                                             const int* __restrict__ T_off, const int* __restrict__ k,
                                             const int64_t* __restrict__ koff, const double* __restrict__ src,
                                             double* __restrict__ q, int nr) {
  const int b = blockIdx.x, kb = k[b];
  if (kb == 0) return;
  const int t0 = T_off[b], m = T_off[b + 1] - t0;
  const double* Ub = U + U_off[b];
  const int lane = threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
  const int tr = (kb + 15) / 16, tc = (nr + 15) / 16;
  for (int t = blockIdx.y * (WG / WAVE) + threadIdx.x / WAVE; t < tr * tc; t += gridDim.y * (WG / WAVE)) {
    const int R0 = (t / tc) * 16, C0 = (t % tc) * 16;
    const bool rok = R0 + fr < kb, cok = C0 + fr < nr;
    mv_dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < m; k0 += 4) {
      const int r = k0 + fk;
      const double a = (rok && r < m) ? Ub[(size_t)r * kb + R0 + fr] : 0.0;
      const double bb = (cok && r < m) ? src[(size_t)(t0 + r) * nr + C0 + fr] : 0.0;
      acc = mv_mfma(a, bb, acc);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = R0 + fk + 4 * u, c = C0 + fr;
      if (j < kb && c < nr) q[(size_t)(koff[b] + j) * nr + c] = acc[u];
    }
  }
}

// M2L: loc[koff[b] + j] (+)= sum over D in IL(b) of sum_i A_bD[j][i] q[koff[D] + i].
__global__ void __launch_bounds__(WG) k_h2_m2l(const double* __restrict__ M, const int64_t* __restrict__ M_off,
                                              const int* __restrict__ il_off, const int* __restrict__ il,
                                              const int* __restrict__ k, const int64_t* __restrict__ koff,
                                              const double* __restrict__ q, double* __restrict__ loc, int nr, int add) {
  const int b = blockIdx.x, kb = k[b];
  if (kb == 0) return;
  const int lane = threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
  const int tr = (kb + 15) / 16, tc = (nr + 15) / 16;
  for (int t = blockIdx.y * (WG / WAVE) + threadIdx.x / WAVE; t < tr * tc; t += gridDim.y * (WG / WAVE)) {
    const int R0 = (t / tc) * 16, C0 = (t % tc) * 16;
    const bool rok = R0 + fr < kb, cok = C0 + fr < nr;
    mv_dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int e = il_off[b]; e < il_off[b + 1]; ++e) {
      const int D = il[e], kd = k[D];
      const double* Me = M + M_off[e] + (size_t)(R0 + fr) * kd;
      const double* qd = q + (size_t)koff[D] * nr + C0 + fr;
#pragma unroll 4
      for (int k0 = 0; k0 < kd; k0 += 4) {
        const int i = k0 + fk;
        const double a = (rok && i < kd) ? Me[i] : 0.0;
        const double bb = (cok && i < kd) ? qd[(size_t)i * nr] : 0.0;
        acc = mv_mfma(a, bb, acc);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = R0 + fk + 4 * u, c = C0 + fr;
      if (j < kb && c < nr) {
        double* o = loc + (size_t)(koff[b] + j) * nr + c;
        *o = add ? *o + acc[u] : acc[u];
      }
    }
  }
}

// L2L / L2P: out[T_off[b] + r] = sum_j U_b[r][j] loc[koff[b] + j] for every row r of box b (the
// children's locals above the leaf, the points of the leaf at the leaf); rows of a box of rank
// 0 get 0.
__global__ void __launch_bounds__(WG) k_h2_down(const double* __restrict__ U, const int64_t* __restrict__ U_off,
                                               const int* __restrict__ T_off, const int* __restrict__ k,
                                               const int64_t* __restrict__ koff, const double* __restrict__ loc,
                                               double* __restrict__ out, int nr) {
  const int b = blockIdx.x, kb = k[b];
  const int t0 = T_off[b], m = T_off[b + 1] - t0;
  const double* Ub = U + U_off[b];
  const int lane = threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
  const int tr = (m + 15) / 16, tc = (nr + 15) / 16;
  for (int t = blockIdx.y * (WG / WAVE) + threadIdx.x / WAVE; t < tr * tc; t += gridDim.y * (WG / WAVE)) {
    const int R0 = (t / tc) * 16, C0 = (t % tc) * 16;
    const bool rok = R0 + fr < m, cok = C0 + fr < nr;
    const double* Ur = Ub + (size_t)(R0 + fr) * kb;
    mv_dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < kb; k0 += 4) {
      const int j = k0 + fk;
      const double a = (rok && j < kb) ? Ur[j] : 0.0;
      const double bb = (cok && j < kb) ? loc[(size_t)(koff[b] + j) * nr + C0 + fr] : 0.0;
      acc = mv_mfma(a, bb, acc);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = R0 + fk + 4 * u, c = C0 + fr;
      if (r < m && c < nr) out[(size_t)(t0 + r) * nr + c] = acc[u];
    }
  }
}

// P2P: y[p] += sum over X in N(b) of sum over the points s of X of A_ps x[s], every entry
// evaluated (one wave per leaf box; a lane per target point, the sources of a neighbour staged
// through LDS in tiles, the right-hand sides in blocks of MV_R columns).
constexpr int P2P_T = 64;
template <int KIND, int D>
__global__ void __launch_bounds__(P2P_T) k_h2_p2p(KernelDesc K, const double* __restrict__ pts,
                                                 const int* __restrict__ box_off, const int* __restrict__ nbr_off,
                                                 const int* __restrict__ nbr, const double* __restrict__ x,
                                                 double* __restrict__ y, int nr) {
  __shared__ double sp[P2P_T * D];
  __shared__ double sx[P2P_T * MV_R];
  const int b = blockIdx.x;
  const int p0 = box_off[b], np = box_off[b + 1] - p0;
  const double s2 = K.scale * K.scale;
  for (int r0 = 0; r0 < np; r0 += P2P_T) {
    const int i = p0 + r0 + (int)threadIdx.x;
    const bool live = r0 + (int)threadIdx.x < np;
    double pi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) pi[t] = live ? pts[(size_t)i * D + t] : 0.0;
    for (int c0 = 0; c0 < nr; c0 += MV_R) {
      const int nc = min(MV_R, nr - c0);
      double acc[MV_R];
#pragma unroll
      for (int c = 0; c < MV_R; ++c) acc[c] = 0.0;
      for (int e = nbr_off[b]; e < nbr_off[b + 1]; ++e) {
        const int X = nbr[e];
        const int q0 = box_off[X], nq = box_off[X + 1] - q0;
        for (int s0 = 0; s0 < nq; s0 += P2P_T) {
          const int cnt = min(P2P_T, nq - s0);
          __syncthreads();
          for (int u = threadIdx.x; u < cnt * D; u += P2P_T) sp[u] = pts[(size_t)(q0 + s0) * D + u];
          for (int u = threadIdx.x; u < cnt * MV_R; u += P2P_T) {
            const int jj = u / MV_R, c = u - jj * MV_R;
            sx[u] = c < nc ? x[(size_t)(q0 + s0 + jj) * nr + c0 + c] : 0.0;
          }
          __syncthreads();
          if (live) {
            const int dj = i - (q0 + s0);  // the diagonal when the target is in this tile
            for (int jj = 0; jj < cnt; ++jj) {
              double r2 = 0.0;
#pragma unroll
              for (int t = 0; t < D; ++t) {
                const double z = pi[t] - sp[jj * D + t];
                r2 = fma(z, z, r2);
              }
              double v = KIND == 0 ? dexp(-sqrt(r2) / K.scale) : rsqrt_nr(r2 + s2);
              if (jj == dj) v += K.shift;
#pragma unroll
              for (int c = 0; c < MV_R; ++c) acc[c] = fma(v, sx[jj * MV_R + c], acc[c]);
            }
          }
        }
      }
      if (live)
        for (int c = 0; c < nc; ++c) y[(size_t)i * nr + c0 + c] += acc[c];
    }
  }
}

__global__ void k_zero_vec(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// column dot products: out[c] = sum_i a[i, c] b[i, c]  (row-major N x nr), partial sums per block
__global__ void k_coldot(const double* a, const double* b, int64_t N, int nr, double* part) {
  __shared__ double sh[WG / WAVE + 1];
  for (int c = 0; c < nr; ++c) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < N; i += (int64_t)gridDim.x * WG) s = fma(a[i * nr + c], b[i * nr + c], s);
    s = wg_sum<WG>(s, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * nr + c] = s;
  }
}
// y[:, c] += alpha[c] x[:, c]
__global__ void k_axpy_cols(int64_t N, int nr, const double* alpha, const double* x, double* y) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * nr) return;
  int c = (int)(q % nr);
  y[q] = fma(alpha[c], x[q], y[q]);
}
// y[:, c] = x[:, c] * alpha[c]
__global__ void k_scale_cols(int64_t N, int nr, const double* alpha, const double* x, double* y) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * nr) return;
  y[q] = x[q] * alpha[q % nr];
}
__global__ void k_perm_rows_in(const double* b, int64_t ldb, const int64_t* perm, int64_t N, int nr, double* out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * nr) return;
  int64_t i = q / nr;
  int c = (int)(q - i * nr);
  out[q] = b[c * ldb + perm[i]];
}
__global__ void k_perm_rows_out(const double* xs, const int64_t* perm, int64_t N, int nr, double* x, int64_t ldx) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * nr) return;
  int64_t i = q / nr;
  int c = (int)(q - i * nr);
  x[c * ldx + perm[i]] = xs[q];
}

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// y = A x for tree-ordered row-major vectors
void matvec_tree(aifmm_system& s, const double* x, int nr, double* y) {
  dim3 grid(cdiv(s.N, MV_T / WAVE * 16), cdiv(nr, MV_R));
  auto kern = s.K.kind == 0 ? (s.d == 2 ? k_matvec<0, 2> : k_matvec<0, 3>) : (s.d == 2 ? k_matvec<1, 2> : k_matvec<1, 3>);
  hipLaunchKernelGGL(kern, grid, dim3(MV_T), 0, s.stream, s.K, s.d_pts.p, s.N, x, nr, y);
  AIFMM_HIP(hipGetLastError());
}

// y = A~ x with the H^2 operator of s (its matvec-tolerance NNCA when it has one, else its own)
// for tree-ordered row-major vectors.  Kernels only on s's stream; the q / l work vectors are
// the operator's (kept across calls).
void h2_matvec_tree(aifmm_system& s, const double* x, int nr, double* y, hipStream_t st) {
  aifmm_system& S = s.op ? *s.op : s;
  const int L = S.L;
  H2Cache& hc = S.hc;
  if (nr > hc.nr_cap) {
    hc.q.clear();
    hc.loc.clear();
    hc.q.resize(L + 1);
    hc.loc.resize(L + 1);
    for (int l = 2; l <= L; ++l) {
      int64_t K = std::max<int64_t>(1, S.lev[l].koff_nn.back());
      hc.q[l].alloc((size_t)K * nr);
      hc.loc[l].alloc((size_t)K * nr);
    }
    hc.nr_cap = nr;
  }
  // tile groups per box (four tiles of 16 x 16 each): enough workgroups at the coarse levels
  auto groups = [&](int rows) {
    int64_t t = (int64_t)((rows + 15) / 16) * ((nr + 15) / 16);
    return (unsigned)std::max<int64_t>(1, (t + 3) / 4);
  };
  for (int l = L; l >= 2; --l) {  // upward pass: P2M at the leaf, M2M above
    LevelDev& lv = S.lev[l];
    const double* src = l == L ? x : hc.q[l + 1].p;
    int kmax = 0;
    for (int kb : lv.knn) kmax = std::max(kmax, kb);
    hipLaunchKernelGGL(k_h2_up, dim3(lv.nb, groups(kmax)), dim3(WG), 0, st, lv.d_Unn.p, lv.d_Unn_off.p, lv.d_T_off.p,
                       lv.d_knn.p, lv.d_koff_nn.p, src, hc.q[l].p, nr);
  }
  for (int l = 2; l <= L; ++l) {  // M2L, then L2L into the children (downward pass)
    LevelDev& lv = S.lev[l];
    int kmax = 0, mmax = 0;
    for (int b = 0; b < lv.nb; ++b) {
      kmax = std::max(kmax, lv.knn[b]);
      mmax = std::max(mmax, lv.T_off[b + 1] - lv.T_off[b]);
    }
    // level 2 starts the locals; below it they already hold the parent's L2L contribution
    hipLaunchKernelGGL(k_h2_m2l, dim3(lv.nb, groups(kmax)), dim3(WG), 0, st, lv.d_m2l_nn.p, lv.d_m2l_nn_off.p,
                       lv.d_il_off.p, lv.d_il.p, lv.d_knn.p, lv.d_koff_nn.p, hc.q[l].p, hc.loc[l].p, nr, l > 2 ? 1 : 0);
    double* out = l < L ? hc.loc[l + 1].p : y;  // L2L writes the children's locals, L2P writes y
    hipLaunchKernelGGL(k_h2_down, dim3(lv.nb, groups(mmax)), dim3(WG), 0, st, lv.d_Unn.p, lv.d_Unn_off.p,
                       lv.d_T_off.p, lv.d_knn.p, lv.d_koff_nn.p, hc.loc[l].p, out, nr);
  }
  LevelDev& lf = S.lev[L];  // P2P near field of the leaf neighbours
  auto kern = S.K.kind == 0 ? (S.d == 2 ? k_h2_p2p<0, 2> : k_h2_p2p<0, 3>) : (S.d == 2 ? k_h2_p2p<1, 2> : k_h2_p2p<1, 3>);
  hipLaunchKernelGGL(kern, dim3(lf.nb), dim3(P2P_T), 0, st, S.K, S.d_pts.p, lf.d_T_off.p, lf.d_nbr_off.p, lf.d_nbr.p, x,
                     y, nr);
  AIFMM_HIP(hipGetLastError());
}

static std::vector<double> coldots(aifmm_system& s, const double* a, const double* b, int nr, DBuf<double>& part) {
  int nblk = 256;
  if (part.n < (size_t)nblk * nr) part.alloc((size_t)nblk * nr);
  hipLaunchKernelGGL(k_coldot, dim3(nblk), dim3(WG), 0, s.stream, a, b, s.N, nr, part.p);
  std::vector<double> h = part.download(s.stream, (size_t)nblk * nr);
  std::vector<double> out(nr, 0.0);
  for (int q = 0; q < nblk; ++q)
    for (int c = 0; c < nr; ++c) out[c] += h[(size_t)q * nr + c];
  return out;
}

void matvec_system(aifmm_system& s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy, bool x_dev,
                   bool y_dev) {
  hipStream_t st = s.stream;
  int nr = (int)nrhs;
  int64_t N = s.N;
  DBuf<double> xin, xt, yt, yout;
  const double* xs = x;
  int64_t ldxs = ldx;
  if (!x_dev) {  // host x: its N rows per column staged compactly
    xin.alloc((size_t)N * nr);
    h2d_cols(xin.p, x, ldx, N, nr, st);
    xs = xin.p;
    ldxs = N;
  }
  xt.alloc((size_t)N * nr);
  yt.alloc((size_t)N * nr);
  hipLaunchKernelGGL(k_perm_rows_in, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, xs, ldxs, s.d_perm.p, N, nr, xt.p);
  matvec_tree(s, xt.p, nr, yt.p);
  if (y_dev) {
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, yt.p, s.d_perm.p, N, nr, y, ldy);
  } else {
    yout.alloc((size_t)N * nr);
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, yt.p, s.d_perm.p, N, nr, yout.p, N);
    d2h_cols(y, ldy, yout.p, N, nr, st);
  }
  AIFMM_HIP(hipStreamSynchronize(st));
}

void h2_matvec_system(aifmm_system& s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy, bool x_dev,
                      bool y_dev) {
  hipStream_t st = s.stream;
  int nr = (int)nrhs;
  int64_t N = s.N;
  DBuf<double> xin, xt, yt, yout;
  const double* xs = x;
  int64_t ldxs = ldx;
  if (!x_dev) {
    xin.alloc((size_t)N * nr);
    h2d_cols(xin.p, x, ldx, N, nr, st);
    xs = xin.p;
    ldxs = N;
  }
  xt.alloc((size_t)N * nr);
  yt.alloc((size_t)N * nr);
  hipLaunchKernelGGL(k_perm_rows_in, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, xs, ldxs, s.d_perm.p, N, nr, xt.p);
  h2_matvec_tree(s, xt.p, nr, yt.p, st);
  if (y_dev) {
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, yt.p, s.d_perm.p, N, nr, y, ldy);
  } else {
    yout.alloc((size_t)N * nr);
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, yt.p, s.d_perm.p, N, nr, yout.p, N);
    d2h_cols(y, ldy, yout.p, N, nr, st);
  }
  AIFMM_HIP(hipStreamSynchronize(st));
}

// Right-preconditioned flexible GMRES(m) with modified Gram-Schmidt, all right-hand sides
// advanced together (each with its own Hessenberg matrix), from x = 0: the preconditioner is the
// AIFMM solve of s in tree order, the operator apply(); column c stops once its residual
// b - A x (recomputed from x at every restart and at the end) is <= tgt[c].  rhs, x: tree-ordered
// row-major device vectors (N x nr).  its[c] accumulates the iterations; res[c] gets the final
// residual norms.  Returns the iterations used (the largest over the columns).
template <class Apply>
static int fgmres_tree(aifmm_system& s, Apply apply, const double* rhs, int nr, const std::vector<double>& tgt,
                       int restart, int maxit, double* x, std::vector<int>& its, std::vector<double>& res) {
  hipStream_t st = s.stream;
  const int m = std::max(1, restart);
  const int64_t N = s.N;
  const size_t vec = (size_t)N * nr;
  GmresCache& G = s.gc;
  DBuf<double>&r = G.r, &w = G.w, &part = G.part, &dalpha = G.dalpha;
  std::vector<DBuf<double>>&V = G.V, &Z = G.Z;
  auto set_alpha = [&](const std::vector<double>& a) {
    AIFMM_HIP(hipMemcpyAsync(dalpha.p, a.data(), sizeof(double) * nr, hipMemcpyHostToDevice, st));
    AIFMM_HIP(hipStreamSynchronize(st));  // the host vector may go out of scope
  };
  auto axpy = [&](const std::vector<double>& a, const double* xx, double* yy) {
    set_alpha(a);
    hipLaunchKernelGGL(k_axpy_cols, dim3(cdiv(vec, WG)), dim3(WG), 0, st, N, nr, dalpha.p, xx, yy);
  };
  auto scale = [&](const std::vector<double>& a, const double* xx, double* yy) {
    set_alpha(a);
    hipLaunchKernelGGL(k_scale_cols, dim3(cdiv(vec, WG)), dim3(WG), 0, st, N, nr, dalpha.p, xx, yy);
  };
  hipLaunchKernelGGL(k_zero_vec, dim3(cdiv(vec, WG)), dim3(WG), 0, st, x, (int64_t)vec);
  std::vector<int> done(nr, 0);
  int total = 0;
  bool x_zero = true;  // x is still the zero start, so A x = 0 and r = rhs exactly
  while (true) {
    AIFMM_HIP(hipMemcpyAsync(r.p, rhs, sizeof(double) * vec, hipMemcpyDeviceToDevice, st));
    if (!x_zero) {
      apply(x, w.p);
      axpy(std::vector<double>(nr, -1.0), w.p, r.p);
    }
    std::vector<double> beta = coldots(s, r.p, r.p, nr, part);
    bool all = true;
    for (int c = 0; c < nr; ++c) {
      beta[c] = std::sqrt(beta[c]);
      res[c] = beta[c];
      done[c] = beta[c] <= tgt[c];
      all = all && done[c];
    }
    if (all || total >= maxit) break;
    std::vector<double> inv(nr);
    for (int c = 0; c < nr; ++c) inv[c] = (done[c] || beta[c] == 0.0) ? 0.0 : 1.0 / beta[c];
    scale(inv, r.p, V[0].p);
    std::vector<std::vector<double>> H((size_t)(m + 1) * m, std::vector<double>(nr, 0.0));
    std::vector<std::vector<double>> cs(m, std::vector<double>(nr)), sn(m, std::vector<double>(nr));
    std::vector<std::vector<double>> g(m + 1, std::vector<double>(nr, 0.0));
    for (int c = 0; c < nr; ++c) g[0][c] = done[c] ? 0.0 : beta[c];
    int j = 0;
    for (; j < m && total < maxit; ++j, ++total) {
      solve_tree(s, V[j].p, nr, Z[j].p);  // Z_j = M^{-1} V_j
      apply(Z[j].p, w.p);
      for (int i = 0; i <= j; ++i) {
        std::vector<double> h = coldots(s, V[i].p, w.p, nr, part);
        for (int c = 0; c < nr; ++c) H[(size_t)i * m + j][c] = h[c];
        std::vector<double> neg(nr);
        for (int c = 0; c < nr; ++c) neg[c] = -h[c];
        axpy(neg, V[i].p, w.p);
      }
      std::vector<double> hn = coldots(s, w.p, w.p, nr, part);
      std::vector<double> inv2(nr);
      for (int c = 0; c < nr; ++c) {
        hn[c] = std::sqrt(hn[c]);
        H[(size_t)(j + 1) * m + j][c] = hn[c];
        inv2[c] = hn[c] > 0 ? 1.0 / hn[c] : 0.0;
      }
      scale(inv2, w.p, V[j + 1].p);
      bool conv = true;
      for (int c = 0; c < nr; ++c) {
        for (int i = 0; i < j; ++i) {
          double a = H[(size_t)i * m + j][c], bb = H[(size_t)(i + 1) * m + j][c];
          H[(size_t)i * m + j][c] = cs[i][c] * a + sn[i][c] * bb;
          H[(size_t)(i + 1) * m + j][c] = -sn[i][c] * a + cs[i][c] * bb;
        }
        double a = H[(size_t)j * m + j][c], bb = H[(size_t)(j + 1) * m + j][c];
        double rr = std::hypot(a, bb);
        cs[j][c] = rr > 0 ? a / rr : 1.0;
        sn[j][c] = rr > 0 ? bb / rr : 0.0;
        H[(size_t)j * m + j][c] = rr;
        H[(size_t)(j + 1) * m + j][c] = 0.0;
        g[j + 1][c] = -sn[j][c] * g[j][c];
        g[j][c] = cs[j][c] * g[j][c];
        if (!done[c]) {
          ++its[c];
          if (std::fabs(g[j + 1][c]) > 0.5 * tgt[c]) conv = false;
        }
      }
      if (conv) { ++j; ++total; break; }
    }
    // x += Z y with H y = g (upper triangular, per column)
    for (int c = 0; c < nr; ++c) {
      std::vector<double> y(j, 0.0);
      for (int i = j - 1; i >= 0; --i) {
        double v = g[i][c];
        for (int t = i + 1; t < j; ++t) v -= H[(size_t)i * m + t][c] * y[t];
        y[i] = H[(size_t)i * m + i][c] != 0.0 ? v / H[(size_t)i * m + i][c] : 0.0;
      }
      for (int i = 0; i < j; ++i) H[(size_t)i * m][c] = y[i];  // reuse column 0 as storage
    }
    for (int i = 0; i < j; ++i) {
      std::vector<double> a(nr);
      for (int c = 0; c < nr; ++c) a[c] = done[c] ? 0.0 : H[(size_t)i * m][c];
      axpy(a, Z[i].p, x);
    }
    if (j > 0) x_zero = false;
  }
  return total;
}

// FGMRES to relative residual rtol (module comment above fgmres_tree) with the H^2 product of op
// as the operator (the exact product of s when op is null; op's tree is s's tree: same points
// and options).  With an H^2 operator the result is then checked with the exact product: the H^2
// product carries an error of about eps_G |A|, which FGMRES cannot see, so while the exact
// residual of a column is above rtol the exact residual is solved for (FGMRES with the same
// operator) and added, at most three times.  relres reports the exact residual of each column.
void gmres_op_system(aifmm_system* op, aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double rtol,
                     int restart, int maxit, double* x, int64_t ldx, int32_t* iters, double* relres, bool b_dev,
                     bool x_dev) {
  hipStream_t st = s.stream;
  int nr = (int)nrhs, m = std::max(1, restart);
  int64_t N = s.N;
  size_t vec = (size_t)N * nr;
  GmresCache& G = s.gc;
  if (nr > G.nr_cap || m > G.m_cap) {
    int nc = std::max(nr, G.nr_cap), mc = std::max(m, G.m_cap);
    size_t v2 = (size_t)N * nc;
    G.bt.alloc(v2);
    G.xt.alloc(v2);
    G.r.alloc(v2);
    G.w.alloc(v2);
    G.rx.alloc(v2);
    G.cx.alloc(v2);
    G.dalpha.alloc(nc);
    G.V.clear();
    G.Z.clear();
    G.V.resize(mc + 1);
    G.Z.resize(mc);
    for (auto& v : G.V) v.alloc(v2);
    for (auto& z : G.Z) z.alloc(v2);
    G.nr_cap = nc;
    G.m_cap = mc;
  }
  DBuf<double>&bt = G.bt, &xt = G.xt, &part = G.part;
  const double* bs = b;
  int64_t ldbs = ldb;
  if (!b_dev) {  // host b: its N rows per column staged compactly
    if ((int64_t)G.bin.n < N * nr) G.bin.alloc((size_t)N * nr);
    h2d_cols(G.bin.p, b, ldb, N, nr, st);
    bs = G.bin.p;
    ldbs = N;
  }
  hipLaunchKernelGGL(k_perm_rows_in, dim3(cdiv(vec, WG)), dim3(WG), 0, st, bs, ldbs, s.d_perm.p, N, nr, bt.p);
  std::vector<double> bnorm = coldots(s, bt.p, bt.p, nr, part);
  for (auto& v : bnorm) v = std::sqrt(v);
  std::vector<int> its(nr, 0);
  std::vector<double> res(nr, 0.0), tgt(nr), rel(nr, 0.0);
  for (int c = 0; c < nr; ++c) tgt[c] = rtol * bnorm[c];
  auto apply_op = [&](const double* xx, double* yy) {
    if (op) h2_matvec_tree(*op, xx, nr, yy, st);
    else matvec_tree(s, xx, nr, yy);
  };
  int total = fgmres_tree(s, apply_op, bt.p, nr, tgt, restart, maxit, xt.p, its, res);
  for (int c = 0; c < nr; ++c) rel[c] = bnorm[c] > 0 ? res[c] / bnorm[c] : 0.0;
  if (op) {
    for (int round = 0;; ++round) {
      // exact residual rx = b - A x
      matvec_tree(s, xt.p, nr, G.w.p);
      AIFMM_HIP(hipMemcpyAsync(G.rx.p, bt.p, sizeof(double) * vec, hipMemcpyDeviceToDevice, st));
      std::vector<double> neg(nr, -1.0);
      AIFMM_HIP(hipMemcpyAsync(G.dalpha.p, neg.data(), sizeof(double) * nr, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_axpy_cols, dim3(cdiv(vec, WG)), dim3(WG), 0, st, N, nr, G.dalpha.p, G.w.p, G.rx.p);
      std::vector<double> rn = coldots(s, G.rx.p, G.rx.p, nr, part);
      bool ok = true;
      std::vector<double> t2(nr);
      for (int c = 0; c < nr; ++c) {
        rn[c] = std::sqrt(rn[c]);
        rel[c] = bnorm[c] > 0 ? rn[c] / bnorm[c] : 0.0;
        // the correction solve stops at half the allowed residual (columns already within
        // rtol get a zero correction)
        t2[c] = rel[c] <= rtol ? rn[c] : 0.5 * tgt[c];
        ok = ok && rel[c] <= rtol;
      }
      if (ok || round >= 3 || total >= maxit) break;
      std::vector<double> res2(nr, 0.0);
      total += fgmres_tree(s, apply_op, G.rx.p, nr, t2, restart, maxit - total, G.cx.p, its, res2);
      std::vector<double> one(nr, 1.0);
      AIFMM_HIP(hipMemcpyAsync(G.dalpha.p, one.data(), sizeof(double) * nr, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_axpy_cols, dim3(cdiv(vec, WG)), dim3(WG), 0, st, N, nr, G.dalpha.p, G.cx.p, xt.p);
      AIFMM_HIP(hipStreamSynchronize(st));
    }
  }
  for (int c = 0; c < nr; ++c) {
    if (iters) iters[c] = its[c];
    if (relres) relres[c] = rel[c];
  }
  if (x_dev) {
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(vec, WG)), dim3(WG), 0, st, xt.p, s.d_perm.p, N, nr, x, ldx);
  } else {
    DBuf<double>& xo = G.xo;
    if (xo.n < (size_t)N * nr) xo.alloc((size_t)N * nr);
    hipLaunchKernelGGL(k_perm_rows_out, dim3(cdiv(vec, WG)), dim3(WG), 0, st, xt.p, s.d_perm.p, N, nr, xo.p, N);
    d2h_cols(x, ldx, xo.p, N, nr, st);
  }
  AIFMM_HIP(hipStreamSynchronize(st));
  bool ok = true;
  for (int c = 0; c < nr; ++c) ok = ok && rel[c] <= rtol;
  if (!ok) throw Error{AIFMM_ERR_NOCONV, "GMRES did not reach the requested residual within maxit"};
}

// FGMRES with the system's own operator: its H^2 product when it was built with a matvec
// tolerance, else the exact product.
void gmres_system(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double rtol, int restart, int maxit,
                  double* x, int64_t ldx, int32_t* iters, double* relres, bool b_dev, bool x_dev) {
  gmres_op_system(s.op ? &s : nullptr, s, b, nrhs, ldb, rtol, restart, maxit, x, ldx, iters, relres, b_dev, x_dev);
}

}  // namespace aifmm
