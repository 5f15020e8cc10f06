// Build phase on the device: uniform tree (Sec. 2.1), NNCA pivots and operators (Sec. 2.3)
// and the leaf level of the extended sparse system (Sec. 3.1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "dense_wg.hpp"
#include "system.hpp"

namespace aifmm {

// ------------------------------------------------------------------------------------------
// Tree: bounding box, leaf Morton codes, stable counting sort of the points by leaf
// ------------------------------------------------------------------------------------------
__global__ void k_bbox(const double* __restrict__ pts, int64_t n, int d, double* out /* 6 */) {
  __shared__ double sh[WG / WAVE + 1];
  for (int t = 0; t < d; ++t) {
    double lo = 1e300, hi = -1e300;
    for (int64_t i = threadIdx.x; i < n; i += WG) {
      double v = pts[i * d + t];
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
    // min via -max(-x)
    for (int off = WAVE / 2; off > 0; off >>= 1) {
      lo = fmin(lo, __shfl_down(lo, off, WAVE));
      hi = fmax(hi, __shfl_down(hi, off, WAVE));
    }
    __syncthreads();
    if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = lo;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = sh[0];
      for (int q = 1; q < WG / WAVE; ++q) m = fmin(m, sh[q]);
      out[t] = m;
    }
    __syncthreads();
    if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = sh[0];
      for (int q = 1; q < WG / WAVE; ++q) m = fmax(m, sh[q]);
      out[3 + t] = m;
    }
    __syncthreads();
  }
}

// Leaf of every point: the smallest hypercube holding the points, centred on the bounding
// box, side = largest extent, divided uniformly into 2^L cells per axis.
__global__ void k_leaf_code(const double* __restrict__ pts, int64_t n, int d, int L, const double* __restrict__ bb,
                            int* __restrict__ code, int* __restrict__ count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double side = 0.0;
  for (int t = 0; t < d; ++t) side = fmax(side, bb[3 + t] - bb[t]);
  if (side == 0.0) side = 1.0;
  int64_t nside = (int64_t)1 << L;
  int m = 0;
  for (int t = 0; t < d; ++t) {
    double base = (bb[t] + bb[3 + t]) * 0.5 - side * 0.5;
    double f = floor(__dmul_rn(__ddiv_rn(__dsub_rn(pts[i * d + t], base), side), (double)nside));
    int64_t q = (int64_t)f;
    q = q < 0 ? 0 : (q > nside - 1 ? nside - 1 : q);
    for (int bit = 0; bit < L; ++bit) m |= (int)((q >> bit) & 1) << (bit * d + t);
  }
  code[i] = m;
  atomicAdd(&count[m], 1);
}

__global__ void k_scatter(const int* __restrict__ code, int64_t n, int* __restrict__ cursor, int64_t* __restrict__ order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int pos = atomicAdd(&cursor[code[i]], 1);
  order[pos] = i;
}

// Sort each leaf's point indices ascending (rank sort; leaves are small).
__global__ void k_leaf_sort(int64_t* __restrict__ order, const int* __restrict__ off, int64_t* __restrict__ tmp) {
  int b = blockIdx.x;
  int lo = off[b], hi = off[b + 1], m = hi - lo;
  for (int t = threadIdx.x; t < m; t += WG) {
    int64_t v = order[lo + t];
    int r = 0;
    for (int u = 0; u < m; ++u) r += order[lo + u] < v;
    tmp[lo + r] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m; t += WG) order[lo + t] = tmp[lo + t];
}

__global__ void k_gather_pts(const double* __restrict__ pts, const int64_t* __restrict__ order, int64_t n, int d,
                             double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int t = 0; t < d; ++t) out[i * d + t] = pts[order[i] * d + t];
}

// ------------------------------------------------------------------------------------------
// NNCA: ACA with partial pivoting of A[T_b, F_b] per box (one workgroup per box).
// T_b: leaf points, or the children's incoming pivots above the leaf.  F_b: the points of
// the interaction-list boxes (search space of the far-field pivots).
// ------------------------------------------------------------------------------------------
struct AcaArgs {
  KernelDesc K;
  const double* pts;
  int d;
  double tol;
  const int* T;          // row sets
  const int* T_off;      // nb + 1
  const int* il_off;     // IL CSR of the level
  const int* il;
  const int* box_off;    // point offsets of the level's boxes in tree order (nb + 1)
  const int64_t* F_off;  // per box: start of its column workspace (sum of |F|)
  const int64_t* ws_off; // per box: start of U/V workspace in doubles
  double* ws;
  unsigned char* cused;  // |F| per box
  unsigned char* rused;  // |T| per box (at T_off)
  int* piv_r;            // per box at T_off: pivot row positions (tree positions)
  int* piv_c;
  int* rank;             // k_b
  int* flag;             // [3] capacity flag
  int b0;                // first box of the launch (workgroup x takes box b0 + x); ws starts at its ws_off
};

__global__ void __launch_bounds__(WG) k_aca(AcaArgs a) {
  int b = a.b0 + blockIdx.x;
  int t0 = a.T_off[b], m = a.T_off[b + 1] - t0;
  int64_t fbase = a.F_off[b];
  int n = (int)(a.F_off[b + 1] - fbase);
  if (threadIdx.x == 0) a.rank[b] = 0;
  if (m == 0 || n == 0) return;
  const int* T = a.T + t0;
  int kmax = m < n ? m : n;
  double* U = a.ws + (a.ws_off[b] - a.ws_off[a.b0]);  // kmax x m
  double* V = U + (size_t)kmax * m;        // kmax x n
  double* r = V + (size_t)kmax * n;        // n  (residual row)
  double* du = r + n;                      // kmax
  double* dvw = du + kmax;                 // kmax
  unsigned char* cused = a.cused + fbase;
  unsigned char* rused = a.rused + t0;
  __shared__ ValIdx shv[WG / WAVE + 1];
  __shared__ double shd[WG / WAVE + 1];
  for (int t = threadIdx.x; t < m; t += WG) rused[t] = 0;
  for (int j = threadIdx.x; j < n; j += WG) cused[j] = 0;
  __syncthreads();
  int il0 = a.il_off[b], il1 = a.il_off[b + 1];
  int i = 0, k = 0;
  double nrm2 = 0.0;
  while (k < kmax) {
    // residual row i: r_j = A[T_i, F_j] - sum_l U_l[i] V_l[j]   (l in order)
    ValIdx best{-1.0, INT_MAX};
    int Ti = T[i];
    int j0 = 0;
    for (int e = il0; e < il1; ++e) {
      int D = a.il[e];
      int p0 = a.box_off[D], cnt = a.box_off[D + 1] - p0;
      for (int t = threadIdx.x; t < cnt; t += WG) {
        int j = j0 + t;
        double v = kernel_entry(a.K, a.pts, a.d, Ti, p0 + t);
        for (int l = 0; l < k; ++l) v = fma(-U[(size_t)l * m + i], V[(size_t)l * n + j], v);
        r[j] = v;
        if (!cused[j]) {
          ValIdx c{fabs(v), j};
          if (vi_better(c, best)) best = c;
        }
      }
      j0 += cnt;
    }
    best = wg_argmax(best, shv);
    if (threadIdx.x == 0) rused[i] = 1;
    __syncthreads();
    if (best.i == INT_MAX) break;
    if (best.v == 0.0) {  // exactly zero residual row: take the lowest unused row
      ValIdx lo{-1.0, INT_MAX};
      for (int t = threadIdx.x; t < m; t += WG)
        if (!rused[t]) { ValIdx c{0.0, t}; if (vi_better(c, lo)) lo = c; }
      lo = wg_argmax(lo, shv);
      if (lo.i == INT_MAX) break;
      i = lo.i;
      continue;
    }
    int jb = best.i;
    double delta = r[jb];
    for (int j = threadIdx.x; j < n; j += WG) V[(size_t)k * n + j] = r[j] / delta;
    // column jb: u_t = A[T_t, F_jb] - sum_l V_l[jb] U_l[t]
    int Fjb = 0;
    {
      int jj = jb;
      for (int e = il0; e < il1; ++e) {
        int D = a.il[e];
        int cnt = a.box_off[D + 1] - a.box_off[D];
        if (jj < cnt) { Fjb = a.box_off[D] + jj; break; }
        jj -= cnt;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += WG) {
      double v = kernel_entry(a.K, a.pts, a.d, T[t], Fjb);
      for (int l = 0; l < k; ++l) v = fma(-V[(size_t)l * n + jb], U[(size_t)l * m + t], v);
      U[(size_t)k * m + t] = v;
    }
    if (threadIdx.x == 0) {
      cused[jb] = 1;
      a.piv_r[t0 + k] = T[i];
      a.piv_c[t0 + k] = Fjb;
    }
    __syncthreads();
    // |u|^2, |v|^2 and the cross terms (U_l . u)(V_l . v) of the Frobenius-norm update
    double su = 0.0, sv = 0.0;
    for (int t = threadIdx.x; t < m; t += WG) { double x = U[(size_t)k * m + t]; su += x * x; }
    for (int j = threadIdx.x; j < n; j += WG) { double x = V[(size_t)k * n + j]; sv += x * x; }
    double uu = wg_sum(su, shd);
    double vv = wg_sum(sv, shd);
    for (int l = threadIdx.x; l < k; l += WG) {
      double s = 0.0;
      for (int t = 0; t < m; ++t) s += U[(size_t)l * m + t] * U[(size_t)k * m + t];
      du[l] = s;
    }
    int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    for (int l = wave; l < k; l += WG / WAVE) {
      double s = 0.0;
      for (int j = lane; j < n; j += WAVE) s += V[(size_t)l * n + j] * V[(size_t)k * n + j];
      for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_down(s, off, WAVE);
      if (lane == 0) dvw[l] = s;
    }
    __syncthreads();
    double cr = 0.0;
    for (int l = threadIdx.x; l < k; l += WG) cr += du[l] * dvw[l];
    double cross = wg_sum(cr, shd);
    nrm2 += 2.0 * cross + uu * vv;
    ++k;
    if (sqrt(uu * vv) <= a.tol * sqrt(nrm2)) break;
    ValIdx nb{-1.0, INT_MAX};
    for (int t = threadIdx.x; t < m; t += WG)
      if (!rused[t]) { ValIdx c{fabs(U[(size_t)(k - 1) * m + t]), t}; if (vi_better(c, nb)) nb = c; }
    nb = wg_argmax(nb, shv);
    if (nb.i == INT_MAX) break;
    i = nb.i;
  }
  if (threadIdx.x == 0) a.rank[b] = k;
}

// Operators of one box (one workgroup): C = A[t_i, s_i], U_B = A[T_B, s_i] C^{-1}.
struct OpArgs {
  KernelDesc K;
  const double* pts;
  int d;
  const int* T;
  const int* T_off;
  const int* piv_r;
  const int* piv_c;
  const int* rank;
  const int64_t* U_off;
  double* U;
  double* ws;        // per block k_cap^2 + k_cap
  int kcap;
  int* ipivws;
  int* flag;
};

__global__ void __launch_bounds__(WG) k_nnca_ops(OpArgs a) {
  int b = blockIdx.x;
  int k = a.rank[b];
  if (k == 0) return;
  int t0 = a.T_off[b], m = a.T_off[b + 1] - t0;
  double* C = a.ws + (size_t)b * a.kcap * a.kcap;
  int* ipiv = a.ipivws + (size_t)b * a.kcap;
  __shared__ ValIdx shv[WG / WAVE + 1];
  // C^T with C = A[t_i, s_i]; U_B^T solves C^T U_B^T = A[T_B, s_i]^T through the LU of C^T
  for (int idx = threadIdx.x; idx < k * k; idx += WG) {
    int r = idx / k, c = idx - r * k;
    C[idx] = kernel_entry(a.K, a.pts, a.d, a.piv_r[t0 + c], a.piv_c[t0 + r]);
  }
  __syncthreads();
  int st = wg_lu(k, C, k, ipiv, shv);
  if (st) {
    if (threadIdx.x == 0) { a.flag[0] = 1; a.flag[1] = b; }
    return;
  }
  double* Ub = a.U + a.U_off[b];
  for (int t = threadIdx.x; t < m; t += WG) {
    double* x = Ub + (size_t)t * k;
    int Tt = a.T[t0 + t];
    for (int c = 0; c < k; ++c) x[c] = kernel_entry(a.K, a.pts, a.d, Tt, a.piv_c[t0 + c]);
    for (int j = 0; j < k; ++j) {
      int p = ipiv[j];
      if (p != j) { double tmp = x[j]; x[j] = x[p]; x[p] = tmp; }
    }
    for (int i = 1; i < k; ++i)
      for (int j = 0; j < i; ++j) x[i] = fma(-C[(size_t)i * k + j], x[j], x[i]);
    for (int i = k - 1; i >= 0; --i) {
      for (int j = i + 1; j < k; ++j) x[i] = fma(-C[(size_t)i * k + j], x[j], x[i]);
      x[i] /= C[(size_t)i * k + i];
    }
  }
}

// M2L operators A_BD = A[t^{B,i}, t^{D,i}] for every IL entry (one workgroup per entry).
__global__ void k_nnca_m2l(KernelDesc K, const double* pts, int d, const int* il_box, const int* il, const int* T_off,
                           const int* piv_r, const int* rank, const int64_t* off, double* out) {
  int e = blockIdx.x;
  int B = il_box[e], D = il[e];
  int kb = rank[B], kd = rank[D];
  double* o = out + off[e];
  for (int idx = threadIdx.x; idx < kb * kd; idx += WG) {
    int r = idx / kd, c = idx - r * kd;
    o[idx] = kernel_entry(K, pts, d, piv_r[T_off[B] + r], piv_r[T_off[D] + c]);
  }
}

// Parent row set: concatenation of the children's incoming pivots in child order.
__global__ void k_gather_T(const int* __restrict__ child_piv, const int* __restrict__ child_T_off,
                           const int* __restrict__ child_rank, const int* __restrict__ T_off, int nch, int* __restrict__ T) {
  int b = blockIdx.x;
  int o = T_off[b];
  for (int ch = 0; ch < nch; ++ch) {
    int c = b * nch + ch;
    int k = child_rank[c];
    for (int t = threadIdx.x; t < k; t += WG) T[o + t] = child_piv[child_T_off[c] + t];
    o += k;
  }
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

static void launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{AIFMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

void build_system(aifmm_system& s, const double* pts_in, bool on_device) {
  auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = s.stream;
  int d = s.d, L = s.L;
  int64_t N = s.N;
  DBuf<double> d_raw;
  d_raw.alloc((size_t)N * d);
  AIFMM_HIP(hipMemcpyAsync(d_raw.p, pts_in, sizeof(double) * N * d,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  s.d_flag.alloc(8);
  s.d_flag.zero(st);
  // tree
  DBuf<double> bb;
  bb.alloc(6);
  hipLaunchKernelGGL(k_bbox, dim3(1), dim3(WG), 0, st, d_raw.p, N, d, bb.p);
  int nleaf = 1 << (d * L);
  DBuf<int> code, count;
  code.alloc(N);
  count.alloc(nleaf);
  count.zero(st);
  hipLaunchKernelGGL(k_leaf_code, dim3(cdiv(N, WG)), dim3(WG), 0, st, d_raw.p, N, d, L, bb.p, code.p, count.p);
  launch_check("leaf codes");
  std::vector<int> cnt = count.download(st);
  s.leaf_off.assign(nleaf + 1, 0);
  for (int b = 0; b < nleaf; ++b) s.leaf_off[b + 1] = s.leaf_off[b] + cnt[b];
  DBuf<int> cursor, d_leaf_off;
  cursor.upload(std::vector<int>(s.leaf_off.begin(), s.leaf_off.end() - 1), st);
  d_leaf_off.upload(s.leaf_off, st);
  DBuf<int64_t> tmp;
  s.d_perm.alloc(N);
  tmp.alloc(N);
  hipLaunchKernelGGL(k_scatter, dim3(cdiv(N, WG)), dim3(WG), 0, st, code.p, N, cursor.p, s.d_perm.p);
  hipLaunchKernelGGL(k_leaf_sort, dim3(nleaf), dim3(WG), 0, st, s.d_perm.p, d_leaf_off.p, tmp.p);
  s.d_pts.alloc((size_t)N * d);
  hipLaunchKernelGGL(k_gather_pts, dim3(cdiv(N, WG)), dim3(WG), 0, st, d_raw.p, s.d_perm.p, N, d, s.d_pts.p);
  launch_check("tree");

  // plans and per-level sizes
  s.plan.assign(L + 1, LevelPlan());
  s.lev.clear();
  s.lev.resize(L + 1);
  for (int l = 2; l <= L; ++l) plan_level(s.plan[l], d, l);
  plan_level(s.plan[1], d, 1);
  for (int l = 2; l <= L; ++l) {
    LevelDev& lv = s.lev[l];
    LevelPlan& P = s.plan[l];
    lv.l = l;
    lv.nb = P.nb;
    lv.d_nbr_off.upload(P.nbr_off, st);
    lv.d_nbr.upload(P.nbr, st);
    lv.d_il_off.upload(P.il_off, st);
    lv.d_il.upload(P.il, st);
    lv.d_il_tr.upload(P.il_tr, st);
    lv.d_p2_off.upload(P.p2_off, st);
    lv.d_p2.upload(P.p2, st);
    lv.d_grp_off.upload(P.grp_off, st);
    lv.d_grp_box.upload(P.grp_box, st);
    lv.d_grp_elim.upload(P.grp_elim, st);
  }

  // NNCA bottom-up
  for (int l = L; l >= 2; --l) {
    LevelDev& lv = s.lev[l];
    LevelPlan& P = s.plan[l];
    int nb = lv.nb;
    int shift = d * (L - l);
    std::vector<int> box_off(nb + 1);
    for (int b = 0; b <= nb; ++b) box_off[b] = s.leaf_off[(size_t)b << shift];
    DBuf<int> d_box_off;
    d_box_off.upload(box_off, st);
    // row sets
    lv.T_off.assign(nb + 1, 0);
    if (l == L) {
      for (int b = 0; b < nb; ++b) lv.T_off[b + 1] = box_off[b + 1];
      std::vector<int> T(N);
      for (int64_t i = 0; i < N; ++i) T[i] = (int)i;
      lv.d_T.upload(T, st);
    } else {
      LevelDev& dn = s.lev[l + 1];
      int nch = 1 << d;
      for (int b = 0; b < nb; ++b) {
        int sum = 0;
        for (int ch = 0; ch < nch; ++ch) sum += dn.knn[b * nch + ch];
        lv.T_off[b + 1] = lv.T_off[b] + sum;
      }
      lv.d_T.alloc(std::max(1, lv.T_off[nb]));
      DBuf<int> d_Toff_tmp;
      d_Toff_tmp.upload(lv.T_off, st);
      hipLaunchKernelGGL(k_gather_T, dim3(nb), dim3(WG), 0, st, dn.d_piv_r.p, dn.d_T_off.p, dn.d_k.p, d_Toff_tmp.p, nch,
                         lv.d_T.p);
    }
    lv.d_T_off.upload(lv.T_off, st);
    // column search spaces and ACA workspace
    std::vector<int64_t> F_off(nb + 1, 0), ws_off(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      int64_t f = 0;
      for (int e = P.il_off[b]; e < P.il_off[b + 1]; ++e) f += box_off[P.il[e] + 1] - box_off[P.il[e]];
      int64_t m = lv.T_off[b + 1] - lv.T_off[b];
      int64_t km = std::min<int64_t>(m, f);
      F_off[b + 1] = F_off[b] + f;
      ws_off[b + 1] = ws_off[b] + km * m + km * f + f + 2 * km + 8;
    }
    DBuf<int64_t> d_F_off, d_ws_off;
    d_F_off.upload(F_off, st);
    d_ws_off.upload(ws_off, st);
    // boxes in launches whose U/V workspaces together stay within a budget (half the free
    // device memory, at most 32 GiB): in 3D a box's column space is every point of its ~189
    // interaction-list boxes, so the whole level's workspace can exceed the device
    int64_t budget = (int64_t)32 << 27;  // doubles
    {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = std::min<int64_t>(budget, (int64_t)(fr / 2 / sizeof(double)));
    }
    std::vector<int> chunk{0};
    int64_t wmax = 0;
    for (int b = 0; b < nb; ++b) {
      if (ws_off[b + 1] - ws_off[chunk.back()] > budget && b > chunk.back()) chunk.push_back(b);
      wmax = std::max(wmax, ws_off[b + 1] - ws_off[chunk.back()]);
    }
    chunk.push_back(nb);
    DBuf<double> acaws;
    acaws.alloc(std::max<int64_t>(1, wmax));
    DBuf<unsigned char> cused, rused;
    cused.alloc(std::max<int64_t>(1, F_off[nb]));
    rused.alloc(std::max<int64_t>(1, lv.T_off[nb]));
    lv.d_piv_r.alloc(std::max(1, lv.T_off[nb]));
    lv.d_piv_c.alloc(std::max(1, lv.T_off[nb]));
    lv.d_k.alloc(nb);
    lv.d_kn.alloc(nb);
    for (size_t c = 0; c + 1 < chunk.size(); ++c) {
      AcaArgs aa{s.K, s.d_pts.p, d, s.tol, lv.d_T.p, lv.d_T_off.p, lv.d_il_off.p, lv.d_il.p, d_box_off.p,
                 d_F_off.p, d_ws_off.p, acaws.p, cused.p, rused.p, lv.d_piv_r.p, lv.d_piv_c.p, lv.d_k.p, s.d_flag.p,
                 chunk[c]};
      hipLaunchKernelGGL(k_aca, dim3(chunk[c + 1] - chunk[c]), dim3(WG), 0, st, aa);
      launch_check("aca");
    }
    lv.knn = lv.d_k.download(st);
    lv.d_knn.upload(lv.knn, st);
    if (const char* v = getenv("AIFMM_VERBOSE"); v && *v && *v != '0')
      fprintf(stderr, "[aifmm] build level %d: cross approximation in %zu launch(es), workspace %.2f GB, max rank %d, at %.3f s\n",
              l, chunk.size() - 1, wmax * 8e-9, *std::max_element(lv.knn.begin(), lv.knn.end()),
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
    lv.koff_nn.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) lv.koff_nn[b + 1] = lv.koff_nn[b] + lv.knn[b];
    lv.d_koff_nn.upload(lv.koff_nn, st);
    std::vector<int> flag = s.d_flag.download(st);
    if (flag[3]) throw Error{AIFMM_ERR_CAPACITY, "ACA row set or rank above the workgroup capacity at level " + std::to_string(l)};
    acaws.release();
    cused.release();
    // operators
    lv.Unn_off.assign(nb + 1, 0);
    int kcap = 1;
    for (int b = 0; b < nb; ++b) {
      lv.Unn_off[b + 1] = lv.Unn_off[b] + (int64_t)(lv.T_off[b + 1] - lv.T_off[b]) * lv.knn[b];
      kcap = std::max(kcap, lv.knn[b]);
    }
    lv.d_Unn.alloc(std::max<int64_t>(1, lv.Unn_off[nb]));
    lv.d_Unn_off.upload(lv.Unn_off, st);
    DBuf<double> opws;
    opws.alloc((size_t)nb * kcap * kcap);
    DBuf<int> ipws;
    ipws.alloc((size_t)nb * kcap);
    OpArgs oa{s.K, s.d_pts.p, d, lv.d_T.p, lv.d_T_off.p, lv.d_piv_r.p, lv.d_piv_c.p, lv.d_k.p, lv.d_Unn_off.p,
              lv.d_Unn.p, opws.p, kcap, ipws.p, s.d_flag.p};
    hipLaunchKernelGGL(k_nnca_ops, dim3(nb), dim3(WG), 0, st, oa);
    launch_check("nnca operators");
    flag = s.d_flag.download(st);
    if (flag[0]) throw Error{AIFMM_ERR_SINGULAR, "singular NNCA cross matrix at level " + std::to_string(l) + " box " + std::to_string(flag[1])};
    // M2L
    std::vector<int> il_box(P.il.size());
    lv.m2l_nn_off.assign(P.il.size() + 1, 0);
    for (int b = 0; b < nb; ++b)
      for (int e = P.il_off[b]; e < P.il_off[b + 1]; ++e) {
        il_box[e] = b;
        lv.m2l_nn_off[e + 1] = lv.m2l_nn_off[e] + (int64_t)lv.knn[b] * lv.knn[P.il[e]];
      }
    DBuf<int> d_il_box;
    d_il_box.upload(il_box, st);
    lv.d_m2l_nn_off.upload(lv.m2l_nn_off, st);
    lv.d_m2l_nn.alloc(std::max<int64_t>(1, lv.m2l_nn_off.back()));
    if (!P.il.empty())
      hipLaunchKernelGGL(k_nnca_m2l, dim3((unsigned)P.il.size()), dim3(WG), 0, st, s.K, s.d_pts.p, d, d_il_box.p,
                         lv.d_il.p, lv.d_T_off.p, lv.d_piv_r.p, lv.d_k.p, lv.d_m2l_nn_off.p, lv.d_m2l_nn.p);
    launch_check("nnca m2l");
    AIFMM_HIP(hipStreamSynchronize(st));
  }
  s.stats.build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
}

}  // namespace aifmm
