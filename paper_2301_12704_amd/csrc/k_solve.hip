// Solve phase (Sec. 3.4, Algorithm "Back Substitution", with the right-hand-side Schur
// operations of the elimination): forward sweep in elimination order, dense solve of the
// level-2 multipoles, backward sweep in reverse order.  Right-hand sides are stored per
// level row-major (row, rhs) so every box touches contiguous rows.
#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>

#include "dense_wg.hpp"
#include "system.hpp"

namespace aifmm {

// Y tile = A tile B for one task (at most 64 rows of A, K columns; B is K x nr, row-major)
// on FP64 MFMA 16x16x4: the task's rows are the A operand (row tiles of 16; for a fixed step
// the four lanes of a row read 32 contiguous bytes of it), 16 right-hand-side columns the B
// operand.  Row tile rt runs on the waves w with w mod RT = rt (RT row tiles), which split the
// K range; their partial tiles are added in wave order, so the result does not depend on
// scheduling.  The summation order differs from the oracle's (the solve is not on the
// rank-deciding path).  NT: 16-column tiles per pass over the right-hand sides.
typedef double sdbl4 __attribute__((ext_vector_type(4)));
template <int NT, int MODE>
__global__ void __launch_bounds__(WG) k_rows_mfma(const STask* __restrict__ tasks, const double* __restrict__ fslab,
                                                 const double* __restrict__ Bbuf, double* Y0buf, double* Y1buf,
                                                 const double* __restrict__ Yinit, int nr) {
  __shared__ double red[WG / WAVE][NT][4][WAVE];
  const STask T = tasks[blockIdx.x];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
  const int RT = max(1, (T.rows + 15) / 16);
  const int KP = (WG / WAVE) / RT;
  const int rt = w % RT, kp = w / RT;
  const bool active = kp < KP;
  const int ksteps = (T.K + 3) / 4;
  const int per = (ksteps + KP - 1) / KP;
  const int s0 = kp * per, s1 = min(ksteps, s0 + per);
  const int row = rt * 16 + fr;
  const bool rok = active && row < T.rows;
  const double* Ar = fslab + T.a + (size_t)(rok ? row : 0) * T.lda;
  const double* B = Bbuf + (size_t)T.b * nr;
  constexpr int KU = 8;  // MFMA steps whose operands are loaded together
  for (int cb = 0; cb < nr; cb += 16 * NT) {
    sdbl4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = sdbl4{0.0, 0.0, 0.0, 0.0};
    if (active)
      for (int s = s0; s < s1; s += KU) {
        double a[KU], bb[NT][KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const int k = 4 * (s + u) + fk;
          const bool kok = s + u < s1 && k < T.K;
          a[u] = (rok && kok) ? Ar[k] : 0.0;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int col = cb + 16 * t + fr;
            bb[t][u] = (kok && col < nr) ? B[(size_t)k * nr + col] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[t][u], acc[t], 0, 0, 0);
      }
    if (KP > 1) {  // the row tile's partial tiles, added in wave order by its first wave
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[w][t][q][lane] = acc[t][q];
      __syncthreads();
      if (active && kp == 0)
        for (int p = 1; p < KP; ++p)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[t][q] += red[rt + RT * p][t][q][lane];
    }
    // output (lane, q) of tile t: row rt 16 + lane / 16 + 4 q, column cb + 16 t + lane % 16
    if (active && kp == 0)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = rt * 16 + fk + 4 * q, col = cb + 16 * t + fr;
          if (r >= T.rows || col >= nr) continue;
          const double v = acc[t][q];
          if (MODE == 0) {  // w = Piv^{-1}[rhs(X_b); 0]; rows from sel on are also rhs(Z_b)
            Y0buf[(size_t)(T.y + r) * nr + col] = v;
            if (r >= T.sel) Y1buf[(size_t)(T.z + r) * nr + col] = v;
          } else if (MODE == 1) {  // rhs(rows(p)) -= A[rows(p), x_b] w_x
            double* Y = T.sel ? Y1buf : Y0buf;
            Y[(size_t)(T.y + r) * nr + col] -= v;
          } else {  // sol(x_b) = w_x - W sol(O_c)
            Y0buf[(size_t)(T.y + r) * nr + col] = Yinit[(size_t)(T.y0 + r) * nr + col] - v;
          }
        }
    __syncthreads();
  }
}

// B of the backward products: the solution segments of the coupled columns, gathered into one
// contiguous block per box (one workgroup per segment; sel 1 = x of this level, 0 = y).
__global__ void __launch_bounds__(WG) k_gather_seg(const STask* __restrict__ segs, const double* ys, const double* xs,
                                                  double* g, int nr) {
  STask T = segs[blockIdx.x];
  const double* src = (T.sel ? xs : ys) + (size_t)T.b * nr;
  double* dst = g + (size_t)T.y * nr;
  for (int idx = threadIdx.x; idx < T.rows * nr; idx += WG) dst[idx] = src[idx];
}

// Top (level-2 multipole) system, Sec. 3.2: y = U^{-1} L^{-1} P rhs with the dense LU of the
// top matrix.  The solves are blocked by 64 rows: one workgroup solves the block's triangle
// (the block and its right-hand sides staged in LDS, one column per thread), then the rows
// beyond the block are updated by a tiled product (k_rows_mfma), block after block.
constexpr int TB = 64;
__global__ void k_top_perm(const double* __restrict__ B, const int* __restrict__ perm, int K, int nr, double* X) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * nr) return;
  int r = (int)(idx / nr), c = (int)(idx - (int64_t)r * nr);
  X[idx] = B[(size_t)perm[r] * nr + c];
}
__global__ void __launch_bounds__(WG) k_top_diag(const double* __restrict__ A, int K, int b0, int bw, double* X, int nr,
                                                 int lower) {
  __shared__ double Ab[TB][TB + 1];
  __shared__ double Xb[TB][TB + 1];
  for (int idx = threadIdx.x; idx < bw * bw; idx += WG) {
    int r = idx / bw, c = idx - r * bw;
    Ab[r][c] = A[(size_t)(b0 + r) * K + b0 + c];
  }
  for (int c0 = 0; c0 < nr; c0 += TB) {
    int nc = min(TB, nr - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < bw * nc; idx += WG) {
      int r = idx / nc, c = idx - r * nc;
      Xb[r][c] = X[(size_t)(b0 + r) * nr + c0 + c];
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      int c = threadIdx.x;
      if (lower) {
        for (int r = 1; r < bw; ++r) {
          double v = Xb[r][c];
          for (int t = 0; t < r; ++t) v = fma(-Ab[r][t], Xb[t][c], v);
          Xb[r][c] = v;
        }
      } else {
        for (int r = bw - 1; r >= 0; --r) {
          double v = Xb[r][c];
          for (int t = r + 1; t < bw; ++t) v = fma(-Ab[r][t], Xb[t][c], v);
          Xb[r][c] = v / Ab[r][r];
        }
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < bw * nc; idx += WG) {
      int r = idx / nc, c = idx - r * nc;
      X[(size_t)(b0 + r) * nr + c0 + c] = Xb[r][c];
    }
  }
}

__global__ void k_zero(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// b (N x nrhs column-major, original order) -> rhs rows in tree order (row-major)
__global__ void k_perm_in(const double* b, int64_t ldb, const int64_t* perm, int64_t N, int nr, double* out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nr) return;
  int64_t i = idx / nr;
  int c = (int)(idx - i * nr);
  out[idx] = b[c * ldb + perm[i]];
}
__global__ void k_perm_out(const double* xs, const int64_t* perm, int64_t N, int nr, double* x, int64_t ldx) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nr) return;
  int64_t i = idx / nr;
  int c = (int)(idx - i * nr);
  x[c * ldx + perm[i]] = xs[idx];
}

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
static void launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{AIFMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

// Task lists of the solve sweeps (static after the factorization): per level and colour,
// the row tiles of the forward products, of the forward updates, of the backward products and
// the gather segments.
static void build_solve_plan(aifmm_system& s) {
  SolveCache& sc = s.sc;
  int L = s.L;
  double solve_bytes = 0.0;  // factor-store bytes the products of one solve read
  sc.lev.clear();
  sc.lev.resize(L + 1);
  hipStream_t st = s.stream;
  for (int l = 2; l <= L; ++l) {
    LevelDev& lv = s.lev[l];
    LevelPlan& P = s.plan[l];
    SolveLevel& sl = sc.lev[l];
    std::vector<STask> fw, fu, bw, gs;
    sl.fw_off = {0};
    sl.fu_off = {0};
    sl.bw_off = {0};
    sl.gs_off = {0};
    sl.woff.assign(lv.nb + 1, 0);
    for (int b = 0; b < lv.nb; ++b) sl.woff[b + 1] = sl.woff[b] + lv.n[b] + lv.kfin[b];
    int64_t gmax = 0;
    for (size_t c = 0; c + 1 < P.col_off.size(); ++c) {
      int64_t go = 0;
      for (int q = P.col_off[c]; q < P.col_off[c + 1]; ++q) {
        int b = P.order[q];
        int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
        int n = lv.n[b], k = lv.kfin[b], m = n + k;
        auto dim = [&](int g) {
          if (g == G - 1) return k;
          int p = P.grp_box[g0 + g];
          return P.grp_elim[g0 + g] ? lv.kfin[p] : lv.n[p];
        };
        int C = 0;
        for (int g = 0; g < G; ++g) C += dim(g);
        int ldw = C + n;
        for (int r0 = 0; r0 < m; r0 += WAVE) {
          STask t{};
          t.a = lv.fW[b] + C + (int64_t)r0 * ldw;
          t.lda = ldw;
          t.K = n;
          t.rows = std::min(WAVE, m - r0);
          t.b = lv.xoff[b];
          t.y = sl.woff[b] + r0;
          t.sel = n - r0;
          t.z = lv.koff[b] + r0 - n;
          fw.push_back(t);
        }
        int ro = 0;
        for (int g = 0; g < G - 1; ++g) {
          int p = P.grp_box[g0 + g], e = P.grp_elim[g0 + g];
          int rd = dim(g);
          for (int r0 = 0; r0 < rd; r0 += WAVE) {
            STask t{};
            t.a = lv.fC[b] + (int64_t)(ro + r0) * n;
            t.lda = n;
            t.K = n;
            t.rows = std::min(WAVE, rd - r0);
            t.b = sl.woff[b];
            t.y = (e ? lv.koff[p] : lv.xoff[p]) + r0;
            t.sel = e;
            fu.push_back(t);
          }
          ro += rd;
        }
        int co = 0;
        for (int g = 0; g < G; ++g) {
          int p = P.grp_box[g0 + g], e = P.grp_elim[g0 + g];
          int cd = dim(g);
          if (cd > 0) {
            STask t{};
            t.y = go + co;
            t.rows = cd;
            if (g == G - 1) { t.b = lv.koff[b]; t.sel = 0; }
            else if (e) { t.b = lv.koff[p]; t.sel = 0; }
            else { t.b = lv.xoff[p]; t.sel = 1; }
            gs.push_back(t);
          }
          co += cd;
        }
        for (int r0 = 0; r0 < n; r0 += WAVE) {
          STask t{};
          t.a = lv.fW[b] + (int64_t)r0 * ldw;
          t.lda = ldw;
          t.K = C;
          t.rows = std::min(WAVE, n - r0);
          t.b = go;
          t.y = lv.xoff[b] + r0;
          t.y0 = sl.woff[b] + r0;
          bw.push_back(t);
        }
        go += C;
      }
      gmax = std::max(gmax, go);
      sl.fw_off.push_back((int)fw.size());
      sl.fu_off.push_back((int)fu.size());
      sl.bw_off.push_back((int)bw.size());
      sl.gs_off.push_back((int)gs.size());
    }
    sl.grows = gmax;
    for (auto* v : {&fw, &fu, &bw})
      for (const STask& t : *v) solve_bytes += 8.0 * t.rows * t.K;
    sl.fw.upload(fw, st);
    sl.fu.upload(fu, st);
    sl.bw.upload(bw, st);
    sl.gs.upload(gs, st);
  }
  // top system: the row order of its LU pivoting and the block-update tiles
  int K = s.Ktop;
  if (K > 0) {
    std::vector<int> piv = s.d_top_piv.download(st, K), perm(K);
    for (int r = 0; r < K; ++r) perm[r] = r;
    for (int r = 0; r < K; ++r) std::swap(perm[r], perm[piv[r]]);
    sc.top_perm.upload(perm, st);
    std::vector<STask> fw, bw;
    sc.top_fw_off = {0};
    sc.top_bw_off = {0};
    int nblk = (K + TB - 1) / TB;
    for (int bi = 0; bi < nblk; ++bi) {  // forward: rows below block bi
      int b0 = bi * TB, w = std::min(TB, K - b0);
      for (int r0 = b0 + w; r0 < K; r0 += TB) {
        STask t{};
        t.a = (int64_t)r0 * K + b0;
        t.lda = K;
        t.K = w;
        t.rows = std::min(TB, K - r0);
        t.b = b0;
        t.y = r0;
        fw.push_back(t);
      }
      sc.top_fw_off.push_back((int)fw.size());
    }
    for (int bi = nblk - 1; bi >= 0; --bi) {  // backward: rows above block bi
      int b0 = bi * TB, w = std::min(TB, K - b0);
      for (int r0 = 0; r0 < b0; r0 += TB) {
        STask t{};
        t.a = (int64_t)r0 * K + b0;
        t.lda = K;
        t.K = w;
        t.rows = std::min(TB, b0 - r0);
        t.b = b0;
        t.y = r0;
        bw.push_back(t);
      }
      sc.top_bw_off.push_back((int)bw.size());
    }
    sc.top_fw.upload(fw, st);
    sc.top_bw.upload(bw, st);
  }
  solve_bytes += 8.0 * (double)K * K;  // the top system's LU factors, once over both sweeps
  s.stats.solve_bytes = solve_bytes;
  sc.nr_cap = 0;
  sc.built = true;
}

// Work buffers of one solve of nr columns: per level l the right-hand sides of the Z rows
// (R[l-1]), the solution of the y / x variables (X[l-1], X[l] for l < L), the forward results
// w = Piv^{-1} rhs of every box (W[l]) and the gathered coupled-column segments (G).
struct SolveBufs {
  std::vector<double*> R, X, W;
  double* G = nullptr;
};

// Doubles of each work buffer for nr columns (R and X by level l - 1, W by level l), and G.
static void solve_buf_sizes(aifmm_system& s, int nr, std::vector<int64_t>& rsz, std::vector<int64_t>& wsz,
                            int64_t& gsz) {
  int L = s.L;
  rsz.assign(L + 1, 0);
  wsz.assign(L + 1, 0);
  for (int l = L; l >= 2; --l) {
    rsz[l - 1] = std::max<int64_t>(1, s.lev[l].koff[s.lev[l].nb]) * nr;
    wsz[l] = std::max<int64_t>(1, s.sc.lev[l].woff.back()) * nr;
  }
  int64_t gmax = 1;
  for (int l = 2; l <= L; ++l) gmax = std::max(gmax, s.sc.lev[l].grows);
  gsz = gmax * nr;
}

static void ensure_solve_buffers(aifmm_system& s, int nr) {
  SolveCache& sc = s.sc;
  if (!sc.built) build_solve_plan(s);
  if (nr <= sc.nr_cap) return;
  int L = s.L;
  sc.R.clear();
  sc.X.clear();
  sc.R.resize(L + 1);
  sc.X.resize(L + 1);
  sc.W.clear();
  sc.W.resize(L + 1);
  std::vector<int64_t> rsz, wsz;
  int64_t gsz = 0;
  solve_buf_sizes(s, nr, rsz, wsz, gsz);
  for (int l = L; l >= 2; --l) {
    sc.R[l - 1].alloc((size_t)rsz[l - 1]);
    sc.X[l - 1].alloc((size_t)rsz[l - 1]);
    sc.W[l].alloc((size_t)wsz[l]);
  }
  sc.G.alloc((size_t)gsz);
  sc.nr_cap = nr;
}

template <int MODE>
static void launch_rows(int ntask, const STask* t, const double* fslab, const double* B, double* Y0, double* Y1,
                        const double* Yi, int nr, hipStream_t st) {
  if (ntask <= 0) return;
  dim3 g(ntask), blk(WG);
  if (nr <= 16) hipLaunchKernelGGL((k_rows_mfma<1, MODE>), g, blk, 0, st, t, fslab, B, Y0, Y1, Yi, nr);
  else if (nr <= 32) hipLaunchKernelGGL((k_rows_mfma<2, MODE>), g, blk, 0, st, t, fslab, B, Y0, Y1, Yi, nr);
  else hipLaunchKernelGGL((k_rows_mfma<4, MODE>), g, blk, 0, st, t, fslab, B, Y0, Y1, Yi, nr);
}

static SolveBufs cache_bufs(aifmm_system& s) {
  SolveCache& sc = s.sc;
  SolveBufs B;
  B.R.assign(s.L + 1, nullptr);
  B.X.assign(s.L + 1, nullptr);
  B.W.assign(s.L + 1, nullptr);
  for (int l = 0; l <= s.L; ++l) {
    B.R[l] = sc.R[l].p;
    B.X[l] = sc.X[l].p;
    B.W[l] = sc.W[l].p;
  }
  B.G = sc.G.p;
  return B;
}

// Solve with tree-ordered row-major right-hand sides (N x nr) on the device; x may be rhs
// itself (then the solve runs in place), otherwise it aliases nothing.  The launch sequence of
// one solve (buffers sized for nr): kernels and at most one device-to-device copy, so it can
// also be captured into a graph.
static void solve_tree_launch(aifmm_system& s, const double* rhs, int nr, double* x, const SolveBufs& B) {
  hipStream_t st = s.stream;
  int L = s.L;
  int64_t N = s.N;
  SolveCache& sc = s.sc;
  // rhs of the X rows of level L is the input; rhs of Z rows of level l = X rows of level l-1
  if (x != rhs) AIFMM_HIP(hipMemcpyAsync(x, rhs, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, st));
  auto Xrows = [&](int l) { return l == L ? x : B.R[l]; };   // rhs, overwritten in place
  for (int l = L; l >= 2; --l) {
    int64_t K = s.lev[l].koff[s.lev[l].nb];
    if (K > 0) hipLaunchKernelGGL(k_zero, dim3(cdiv(K * nr, WG)), dim3(WG), 0, st, B.R[l - 1], K * nr);
  }
  // the forward sweep keeps rhs(X^{(L)}) in x; the backward sweep overwrites x with sol(x^{(L)})
  // box by box after every read of rhs(X_b) (the forward sweep has finished by then)
  for (int l = L; l >= 2; --l) {
    LevelDev& lv = s.lev[l];
    SolveLevel& sl = sc.lev[l];
    double* Xr = Xrows(l);
    double* Zr = B.R[l - 1];
    for (size_t c = 0; c + 1 < sl.fw_off.size(); ++c) {
      launch_rows<0>(sl.fw_off[c + 1] - sl.fw_off[c], sl.fw.p + sl.fw_off[c], lv.fslab.p, Xr, B.W[l], Zr, nullptr,
                     nr, st);
      launch_rows<1>(sl.fu_off[c + 1] - sl.fu_off[c], sl.fu.p + sl.fu_off[c], lv.fslab.p, B.W[l], Xr, Zr, nullptr,
                     nr, st);
    }
  }
  launch_check("forward sweep");
  // level-2 multipoles: y^{(2)} = Top^{-1} rhs(Z^{(2)})
  if (s.Ktop > 0) {
    int K = s.Ktop, nblk = (K + TB - 1) / TB;
    double* Xt = B.X[1];
    hipLaunchKernelGGL(k_top_perm, dim3(cdiv((int64_t)K * nr, WG)), dim3(WG), 0, st, B.R[1], sc.top_perm.p, K, nr, Xt);
    for (int bi = 0; bi < nblk; ++bi) {
      int b0 = bi * TB, w = std::min(TB, K - b0);
      hipLaunchKernelGGL(k_top_diag, dim3(1), dim3(WG), 0, st, s.d_top.p, K, b0, w, Xt, nr, 1);
      launch_rows<1>(sc.top_fw_off[bi + 1] - sc.top_fw_off[bi], sc.top_fw.p + sc.top_fw_off[bi], s.d_top.p, Xt, Xt,
                     nullptr, nullptr, nr, st);
    }
    for (int q = 0; q < nblk; ++q) {
      int bi = nblk - 1 - q;
      int b0 = bi * TB, w = std::min(TB, K - b0);
      hipLaunchKernelGGL(k_top_diag, dim3(1), dim3(WG), 0, st, s.d_top.p, K, b0, w, Xt, nr, 0);
      launch_rows<1>(sc.top_bw_off[q + 1] - sc.top_bw_off[q], sc.top_bw.p + sc.top_bw_off[q], s.d_top.p, Xt, Xt,
                     nullptr, nullptr, nr, st);
    }
  }
  for (int l = 2; l <= L; ++l) {
    LevelDev& lv = s.lev[l];
    SolveLevel& sl = sc.lev[l];
    double* xs = l == L ? x : B.X[l];
    const double* ys = B.X[l - 1];
    for (size_t c = sl.bw_off.size() - 1; c-- > 0;) {
      int ng = sl.gs_off[c + 1] - sl.gs_off[c];
      if (ng > 0)
        hipLaunchKernelGGL(k_gather_seg, dim3(ng), dim3(WG), 0, st, sl.gs.p + sl.gs_off[c], ys, xs, B.G, nr);
      launch_rows<2>(sl.bw_off[c + 1] - sl.bw_off[c], sl.bw.p + sl.bw_off[c], lv.fslab.p, B.G, xs, nullptr,
                     B.W[l], nr, st);
    }
  }
  launch_check("backward sweep");
}

void solve_tree(aifmm_system& s, const double* rhs, int nr, double* x) {
  ensure_solve_buffers(s, nr);
  solve_tree_launch(s, rhs, nr, x, cache_bufs(s));
  AIFMM_HIP(hipStreamSynchronize(s.stream));
}

static bool graphs_off() {
  const char* v = getenv("AIFMM_NO_GRAPH");
  return v && *v && *v != '0';
}

void solve_system(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx, bool b_dev,
                  bool x_dev) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  int nr = (int)nrhs;
  int64_t N = s.N;
  // staging buffers are the system's (kept across calls)
  GmresCache& G = s.gc;
  if ((int64_t)G.bt.n < N * nr) G.bt.alloc((size_t)N * nr);
  if ((int64_t)G.xt.n < N * nr) G.xt.alloc((size_t)N * nr);
  const double* bsrc = b;
  int64_t ldbs = ldb;
  if (!b_dev) {  // host b: its N rows per column staged compactly
    if ((int64_t)G.bin.n < N * nr) G.bin.alloc((size_t)N * nr);
    h2d_cols(G.bin.p, b, ldb, N, nr, st);
    bsrc = G.bin.p;
    ldbs = N;
  }
  hipLaunchKernelGGL(k_perm_in, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, bsrc, ldbs, s.d_perm.p, N, nr, G.bt.p);
  ensure_solve_buffers(s, nr);
  SolveCache& sc = s.sc;
  const SolveBufs bufs = cache_bufs(s);
  if (graphs_off() || st == nullptr) {  // the legacy default stream cannot be captured
    solve_tree_launch(s, G.bt.p, nr, G.xt.p, bufs);
  } else {
    // the solve's few hundred launches replayed from one graph, captured for this column count
    // and these buffers (recaptured when either changes; a factorization resets it)
    if (!sc.graph.exec || sc.graph.nr != nr || sc.graph.in != G.bt.p || sc.graph.out != G.xt.p ||
        sc.graph.cap != sc.nr_cap) {
      sc.graph.reset();
      hipGraph_t g = nullptr;
      AIFMM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        solve_tree_launch(s, G.bt.p, nr, G.xt.p, bufs);
      } catch (...) {
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      AIFMM_HIP(hipStreamEndCapture(st, &g));
      sc.graph.graph = g;
      AIFMM_HIP(hipGraphInstantiate(&sc.graph.exec, g, nullptr, nullptr, 0));
      sc.graph.nr = nr;
      sc.graph.in = G.bt.p;
      sc.graph.out = G.xt.p;
      sc.graph.cap = sc.nr_cap;
    }
    AIFMM_HIP(hipGraphLaunch(sc.graph.exec, st));
  }
  if (x_dev) {
    hipLaunchKernelGGL(k_perm_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, G.xt.p, s.d_perm.p, N, nr, x, ldx);
  } else {
    if ((int64_t)G.xo.n < N * nr) G.xo.alloc((size_t)N * nr);
    hipLaunchKernelGGL(k_perm_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, G.xt.p, s.d_perm.p, N, nr, G.xo.p, N);
    d2h_cols(x, ldx, G.xo.p, N, nr, st);
  }
  AIFMM_HIP(hipStreamSynchronize(st));
  launch_check("solve");
  s.stats.solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// The solve's task lists, built right after a factorization so that later solves (including
// the allocation-free one) find them ready.
void prepare_solve(aifmm_system& s) {
  if (!s.sc.built) build_solve_plan(s);
  AIFMM_HIP(hipStreamSynchronize(s.stream));
}

// ---- allocation-free solve --------------------------------------------------------------
// Work buffers of aifmm_solve_noalloc: one static array per device (the loader places a copy
// on every GPU the library runs on).  In host code the array's name is only a stand-in: its
// device address is looked up once per device with hipGetSymbolAddress and used from then on.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;  // by device ordinal, nullptr until looked up

// The scratch array's device address on the current device (looked up on its first use there).
static double* scratch_on_current_device() {
  int dev = 0;
  AIFMM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{AIFMM_ERR_DEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}

size_t noalloc_max_bytes() { return kNoAllocBytes; }

// Bytes of scratch a solve of nr columns needs: the tree-ordered solution (N x nr) and the work
// buffers, each region rounded up to 256 bytes.
size_t noalloc_need_bytes(aifmm_system& s, int nr) {
  std::vector<int64_t> rsz, wsz;
  int64_t gsz = 0;
  solve_buf_sizes(s, nr, rsz, wsz, gsz);
  auto up = [](int64_t n) { return (size_t)((n + 31) & ~int64_t(31)); };
  size_t tot = up(s.N * nr) + up(gsz);
  for (int l = 2; l <= s.L; ++l) tot += 2 * up(rsz[l - 1]) + up(wsz[l]);
  return tot * sizeof(double);
}

// aifmm_solve on device buffers with every work buffer carved from the scratch array: kernels
// only (no allocation, no graph); b and x are device memory.
void solve_system_noalloc(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  int nr = (int)nrhs;
  int64_t N = s.N;
  if (!s.sc.built) throw Error{AIFMM_ERR_STATE, "solve plan missing (factor first)"};
  size_t need = noalloc_need_bytes(s, nr);
  if (need > kNoAllocBytes)
    throw Error{AIFMM_ERR_CAPACITY, "allocation-free solve needs " + std::to_string(need) + " bytes of scratch for " +
                                        std::to_string(nr) + " columns; the maximum is " +
                                        std::to_string(kNoAllocBytes)};
  double* base = scratch_on_current_device();
  std::vector<int64_t> rsz, wsz;
  int64_t gsz = 0;
  solve_buf_sizes(s, nr, rsz, wsz, gsz);
  size_t off = 0;
  auto take = [&](int64_t n) {
    double* p = base + off;
    off += (size_t)((n + 31) & ~int64_t(31));
    return p;
  };
  double* xt = take(N * nr);
  SolveBufs B;
  B.R.assign(s.L + 1, nullptr);
  B.X.assign(s.L + 1, nullptr);
  B.W.assign(s.L + 1, nullptr);
  for (int l = s.L; l >= 2; --l) {
    B.R[l - 1] = take(rsz[l - 1]);
    B.X[l - 1] = take(rsz[l - 1]);
    B.W[l] = take(wsz[l]);
  }
  B.G = take(gsz);
  hipLaunchKernelGGL(k_perm_in, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, b, ldb, s.d_perm.p, N, nr, xt);
  solve_tree_launch(s, xt, nr, xt, B);
  hipLaunchKernelGGL(k_perm_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, xt, s.d_perm.p, N, nr, x, ldx);
  AIFMM_HIP(hipStreamSynchronize(st));
  launch_check("allocation-free solve");
  s.stats.solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace aifmm
