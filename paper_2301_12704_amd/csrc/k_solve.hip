// Solve phase (Sec. 3.4, Algorithm "Back Substitution", with the right-hand-side Schur
// operations of the elimination): forward sweep in elimination order, dense solve of the
// level-2 multipoles, backward sweep in reverse order.  Right-hand sides are stored per
// level row-major (row, rhs) so every box touches contiguous rows.
#include <algorithm>
#include <chrono>

#include "dense_wg.hpp"
#include "system.hpp"

namespace aifmm {

struct SolvePtrs {
  int nrhs;
  const int* n;
  const int* k;
  const int* grp_off;
  const int* grp_box;
  const int* grp_elim;
  const double* fslab;
  const int64_t* fC;
  const int64_t* fW;
  const int64_t* xoff;   // per box, rows of x / X at this level
  const int64_t* koff;   // per box, rows of y / z / Z at this level
  double* Xr;            // rhs of X rows (level l)
  double* Zr;            // rhs of Z rows (level l) == rhs of X rows of level l-1
  double* xs;            // solution x (level l)
  const double* ys;      // solution y (level l) == solution x of level l-1
  double* wsave;         // per box m x nrhs
  const int64_t* woff;
};

__device__ inline int grp_dim(const SolvePtrs& S, int g, int G, int b, int q, int e) {
  if (g == G - 1) return S.k[b];
  return e ? S.k[q] : S.n[q];
}

// w = Piv^{-1} [rhs(X_b); 0] = Px rhs(X_b); rhs(rows(p)) -= A[rows(p), x_b] w_x; rhs(Z_b) = w_z
__global__ void __launch_bounds__(WG) k_fwd(SolvePtrs S, const int* __restrict__ boxes) {
  int b = boxes[blockIdx.x];
  int g0 = S.grp_off[b], G = S.grp_off[b + 1] - g0;
  int n = S.n[b], k = S.k[b], m = n + k, nr = S.nrhs;
  int C = 0;
  for (int g = 0; g < G; ++g) C += grp_dim(S, g, G, b, S.grp_box[g0 + g], S.grp_elim[g0 + g]);
  int ldw = C + n;
  const double* W = S.fslab + S.fW[b];
  const double* Px = W + C;  // columns C .. C+n of the extended W
  const double* rx = S.Xr + S.xoff[b] * nr;
  double* w = S.wsave + S.woff[b];
  for (int idx = threadIdx.x; idx < m * nr; idx += WG) {
    int r = idx / nr, c = idx - r * nr;
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += Px[(size_t)r * ldw + t] * rx[(size_t)t * nr + c];
    w[idx] = acc;
  }
  __syncthreads();
  const double* Cb = S.fslab + S.fC[b];
  int ro = 0;
  for (int g = 0; g < G - 1; ++g) {
    int p = S.grp_box[g0 + g], e = S.grp_elim[g0 + g];
    int rd = e ? S.k[p] : S.n[p];
    double* dst = e ? S.Zr + S.koff[p] * nr : S.Xr + S.xoff[p] * nr;
    for (int idx = threadIdx.x; idx < rd * nr; idx += WG) {
      int r = idx / nr, c = idx - r * nr;
      double acc = 0.0;
      for (int t = 0; t < n; ++t) acc += Cb[(size_t)(ro + r) * n + t] * w[(size_t)t * nr + c];
      dst[idx] -= acc;
    }
    ro += rd;
  }
  double* zb = S.Zr + S.koff[b] * nr;
  for (int idx = threadIdx.x; idx < k * nr; idx += WG) zb[idx] = w[(size_t)n * nr + idx];
}

// sol(x_b; z_b) = w - W sol(O_c);  only x_b is needed further (z never couples forward)
__global__ void __launch_bounds__(WG) k_bwd(SolvePtrs S, const int* __restrict__ boxes) {
  int b = boxes[blockIdx.x];
  int g0 = S.grp_off[b], G = S.grp_off[b + 1] - g0;
  int n = S.n[b], nr = S.nrhs;
  int C = 0;
  for (int g = 0; g < G; ++g) C += grp_dim(S, g, G, b, S.grp_box[g0 + g], S.grp_elim[g0 + g]);
  int ldw = C + n;
  const double* W = S.fslab + S.fW[b];
  const double* w = S.wsave + S.woff[b];
  double* xb = S.xs + S.xoff[b] * nr;
  for (int idx = threadIdx.x; idx < n * nr; idx += WG) {
    int r = idx / nr, c = idx - r * nr;
    double acc = w[idx];
    int co = 0;
    for (int g = 0; g < G; ++g) {
      int q = S.grp_box[g0 + g], e = S.grp_elim[g0 + g];
      int cd = grp_dim(S, g, G, b, q, e);
      const double* src = (g == G - 1) ? S.ys + S.koff[b] * nr : (e ? S.ys + S.koff[q] * nr : S.xs + S.xoff[q] * nr);
      for (int t = 0; t < cd; ++t) acc -= W[(size_t)r * ldw + co + t] * src[(size_t)t * nr + c];
      co += cd;
    }
    xb[idx] = acc;
  }
}

// dense LU solve of the level-2 system, columns of the right-hand side in parallel
__global__ void __launch_bounds__(WG) k_top_solve(const double* A, const int* ipiv, int K, double* X, int nr) {
  for (int r = 0; r < K; ++r) {
    int p = ipiv[r];
    if (p != r)
      for (int c = threadIdx.x; c < nr; c += WG) {
        double t = X[(size_t)r * nr + c];
        X[(size_t)r * nr + c] = X[(size_t)p * nr + c];
        X[(size_t)p * nr + c] = t;
      }
    __syncthreads();
  }
  // forward: x_r -= L[r, 0:r] x   (column-oriented updates)
  for (int t = 0; t < K; ++t) {
    for (int idx = threadIdx.x; idx < (K - t - 1) * nr; idx += WG) {
      int r = t + 1 + idx / nr, c = idx % nr;
      X[(size_t)r * nr + c] -= A[(size_t)r * K + t] * X[(size_t)t * nr + c];
    }
    __syncthreads();
  }
  for (int t = K - 1; t >= 0; --t) {
    for (int c = threadIdx.x; c < nr; c += WG) X[(size_t)t * nr + c] /= A[(size_t)t * K + t];
    __syncthreads();
    for (int idx = threadIdx.x; idx < t * nr; idx += WG) {
      int r = idx / nr, c = idx % nr;
      X[(size_t)r * nr + c] -= A[(size_t)r * K + t] * X[(size_t)t * nr + c];
    }
    __syncthreads();
  }
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

// Solve with tree-ordered row-major right-hand sides (N x nr) on the device; x may alias nothing.
void solve_tree(aifmm_system& s, const double* rhs, int nr, double* x) {
  hipStream_t st = s.stream;
  int L = s.L;
  int64_t N = s.N;
  // buffers: rhs per level (X rows of level l; Z rows of level l == X rows of level l-1)
  std::vector<DBuf<double>> R(L + 2), X(L + 2);  // R[l]: rhs of X rows at level l; X[l]: solution x at level l
  R[L].alloc((size_t)N * nr);
  AIFMM_HIP(hipMemcpyAsync(R[L].p, rhs, sizeof(double) * N * nr, hipMemcpyDeviceToDevice, st));
  for (int l = L; l >= 2; --l) {
    int64_t K = s.lev[l].koff[s.lev[l].nb];
    R[l - 1].alloc((size_t)std::max<int64_t>(1, K) * nr);
    R[l - 1].zero(st);
    X[l - 1].alloc((size_t)std::max<int64_t>(1, K) * nr);
  }
  // per level device offsets and w storage
  std::vector<DBuf<int64_t>> dx(L + 1), dk(L + 1), dwo(L + 1);
  std::vector<DBuf<double>> wsv(L + 1);
  for (int l = 2; l <= L; ++l) {
    LevelDev& lv = s.lev[l];
    dx[l].upload(lv.xoff, st);
    dk[l].upload(lv.koff, st);
    std::vector<int64_t> wo(lv.nb);
    int64_t o = 0;
    for (int bx = 0; bx < lv.nb; ++bx) { wo[bx] = o; o += (int64_t)(lv.n[bx] + lv.kfin[bx]) * nr; }
    dwo[l].upload(wo, st);
    wsv[l].alloc(std::max<int64_t>(1, o));
  }
  auto sp = [&](int l) {
    LevelDev& lv = s.lev[l];
    SolvePtrs S;
    S.nrhs = nr;
    S.n = lv.d_n.p;
    S.k = lv.d_k.p;
    S.grp_off = lv.d_grp_off.p;
    S.grp_box = lv.d_grp_box.p;
    S.grp_elim = lv.d_grp_elim.p;
    S.fslab = lv.fslab.p;
    S.fC = lv.d_fC.p;
    S.fW = lv.d_fW.p;
    S.xoff = dx[l].p;
    S.koff = dk[l].p;
    S.Xr = R[l].p;
    S.Zr = R[l - 1].p;
    S.xs = l == L ? x : X[l].p;
    S.ys = X[l - 1].p;
    S.wsave = wsv[l].p;
    S.woff = dwo[l].p;
    return S;
  };
  for (int l = L; l >= 2; --l) {
    SolvePtrs S = sp(l);
    LevelPlan& P = s.plan[l];
    for (size_t c = 0; c + 1 < P.col_off.size(); ++c) {
      int nbox = P.col_off[c + 1] - P.col_off[c];
      hipLaunchKernelGGL(k_fwd, dim3(nbox), dim3(WG), 0, st, S, s.lev[l].d_order.p + P.col_off[c]);
    }
  }
  launch_check("forward sweep");
  // level-2 multipoles: y^{(2)} = Top^{-1} rhs(Z^{(2)})
  if (s.Ktop > 0) {
    AIFMM_HIP(hipMemcpyAsync(X[1].p, R[1].p, sizeof(double) * s.Ktop * nr, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_top_solve, dim3(1), dim3(WG), 0, st, s.d_top.p, s.d_top_piv.p, s.Ktop, X[1].p, nr);
  }
  for (int l = 2; l <= L; ++l) {
    SolvePtrs S = sp(l);
    LevelPlan& P = s.plan[l];
    for (size_t c = P.col_off.size() - 1; c-- > 0;) {
      int nbox = P.col_off[c + 1] - P.col_off[c];
      // boxes of one colour are independent; reverse order inside the colour is not needed
      hipLaunchKernelGGL(k_bwd, dim3(nbox), dim3(WG), 0, st, S, s.lev[l].d_order.p + P.col_off[c]);
    }
  }
  launch_check("backward sweep");
  AIFMM_HIP(hipStreamSynchronize(st));
}

void solve_system(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx, bool b_dev,
                  bool x_dev) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  int nr = (int)nrhs;
  int64_t N = s.N;
  DBuf<double> bdev, rt, xt;
  const double* bsrc = b;
  if (!b_dev) {
    bdev.alloc((size_t)ldb * nr);
    AIFMM_HIP(hipMemcpyAsync(bdev.p, b, sizeof(double) * ldb * nr, hipMemcpyHostToDevice, st));
    bsrc = bdev.p;
  }
  rt.alloc((size_t)N * nr);
  xt.alloc((size_t)N * nr);
  hipLaunchKernelGGL(k_perm_in, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, bsrc, ldb, s.d_perm.p, N, nr, rt.p);
  solve_tree(s, rt.p, nr, xt.p);
  if (x_dev) {
    hipLaunchKernelGGL(k_perm_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, xt.p, s.d_perm.p, N, nr, x, ldx);
  } else {
    DBuf<double> xd;
    xd.alloc((size_t)ldx * nr);
    xd.zero(st);
    hipLaunchKernelGGL(k_perm_out, dim3(cdiv(N * nr, WG)), dim3(WG), 0, st, xt.p, s.d_perm.p, N, nr, xd.p, ldx);
    AIFMM_HIP(hipMemcpyAsync(x, xd.p, sizeof(double) * ldx * nr, hipMemcpyDeviceToHost, st));
  }
  AIFMM_HIP(hipStreamSynchronize(st));
  launch_check("solve");
  s.stats.solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace aifmm
