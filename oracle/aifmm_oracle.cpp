// AIFMM CPU oracle — TEST INFRASTRUCTURE ONLY (loaded by tests/, the smoke entry and
// the benchmark's CPU-baseline leg; never by the product path).
//
// Plain FP64, textbook loops, no BLAS/LAPACK, single-threaded.  Every step follows the
// paper "Algebraic Inverse Fast Multipole Method" (Gujjula & Ambikasaran, arXiv 2301.12704)
// in its order and notation; where the paper is silent the reading used is stated next to
// the code (the same readings are listed in the design notes of the repository).
//
// Parity pins: tests/test_oracle_*.py pin every function here against closed forms,
// brute force and textbook identities (see each test's docstring).
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace {

// ----------------------------------------------------------------------------------------
// Dense helpers (row-major)
// ----------------------------------------------------------------------------------------
struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() {}
  Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& at(int i, int j) { return a[(size_t)i * c + j]; }
  double at(int i, int j) const { return a[(size_t)i * c + j]; }
};

double g_flops[5];

// Arithmetic and ordering choices that the paper leaves open (see oracle.h, ORACLE_MODE_*):
// the default follows the device's choices; the textbook mode takes the plainest reading of
// each.  Set from the system's mode at the start of every call that computes.
int g_mode = 0;
enum { MODE_STD_EXP = 1, MODE_ASC_SUMS = 2, MODE_ASC_BACK = 4, MODE_SEQUENTIAL = 8 };

Mat mul(const Mat& A, const Mat& B, int counter = -1) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      double aik = A.at(i, k);
      if (aik == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C.at(i, j) = std::fma(aik, B.at(k, j), C.at(i, j));
    }
  if (counter >= 0) g_flops[counter] += 2.0 * A.r * A.c * B.c;
  return C;
}
Mat tr(const Mat& A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T.at(j, i) = A.at(i, j);
  return T;
}
Mat eye(int k, double s) {
  Mat I(k, k);
  for (int i = 0; i < k; ++i) I.at(i, i) = s;
  return I;
}
Mat hcat(const Mat& A, const Mat& B) {  // [A | B], same row count
  Mat C(A.r, A.c + B.c);
  for (int i = 0; i < A.r; ++i) {
    for (int j = 0; j < A.c; ++j) C.at(i, j) = A.at(i, j);
    for (int j = 0; j < B.c; ++j) C.at(i, A.c + j) = B.at(i, j);
  }
  return C;
}

// Textbook LU with row partial pivoting (ties go to the lowest row).  Returns 0 or 1+k for
// an exactly zero pivot at step k.
int lu_factor(Mat& A, std::vector<int>& perm) {
  int n = A.r;
  perm.resize(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A.at(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A.at(i, k)) > best) { best = std::fabs(A.at(i, k)); p = i; }
    if (best == 0.0) return 1 + k;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A.at(k, j), A.at(p, j));
      std::swap(perm[k], perm[p]);
    }
    double piv = A.at(k, k);
    for (int i = k + 1; i < n; ++i) {
      double l = A.at(i, k) / piv;
      A.at(i, k) = l;
      for (int j = k + 1; j < n; ++j) A.at(i, j) = std::fma(-l, A.at(k, j), A.at(i, j));
    }
  }
  g_flops[0] += 2.0 * n * n * n / 3.0;
  return 0;
}
// Solve (LU) X = P B in place on B (n x m); perm from lu_factor (row i of PA = row perm[i] of A).
// Forward substitution sums each row's terms in ascending column order.  Backward substitution
// sums them in ascending column order, or with back_desc in descending column order (the
// column-oriented back substitution (the paper fixes no order), used for the pivot blocks of the
// elimination).
Mat lu_solve(const Mat& LU, const std::vector<int>& perm, const Mat& B, int counter = 1, bool back_desc = false) {
  int n = LU.r, m = B.c;
  Mat X(n, m);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) X.at(i, j) = B.at(perm[i], j);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) {
      double l = LU.at(i, k);
      if (l == 0.0) continue;
      for (int j = 0; j < m; ++j) X.at(i, j) = std::fma(-l, X.at(k, j), X.at(i, j));
    }
  for (int i = n - 1; i >= 0; --i) {
    for (int q = i + 1; q < n; ++q) {
      int k = back_desc ? n + i - q : q;
      double u = LU.at(i, k);
      if (u == 0.0) continue;
      for (int j = 0; j < m; ++j) X.at(i, j) = std::fma(-u, X.at(k, j), X.at(i, j));
    }
    double d = LU.at(i, i);
    for (int j = 0; j < m; ++j) X.at(i, j) /= d;
  }
  if (counter >= 0) g_flops[counter] += 2.0 * n * n * m;
  return X;
}

// Householder QR with column pivoting (the reading taken of the RRQR with threshold eps_A,
// Sec. 3.2.1): trailing column norms recomputed exactly every step, ties (within a relative
// 1e-11) to the lowest column, stop at the smallest k with |R_{k+1,k+1}| <= tol |R_11|.
// Norms and reflector products are row sums in the order of rowsum16.
struct Cpqr {
  int rank = 0;
  int m = 0;
  std::vector<std::vector<double>> v;  // reflector vectors (length m, zeros above s)
  std::vector<double> tau;
  std::vector<int> perm;
  Mat R;               // rank x n (pivoted column order)
  double kept = 0.0;   // |R_kk| / (tol |R_11|) of the last kept pivot
  double next = 0.0;   // |R_{k+1,k+1}| / (tol |R_11|) of the first rejected pivot (0 if none)
};

const double kTieTol = 1e-11;

// Sum over the rows i = a .. m-1 of x(i) y(i) in one fixed order, the device's too (the paper
// fixes no order): sixteen partial fused multiply-add chains, chain q taking the rows i = q (mod 16)
// in ascending order, then the pairwise tree ((t0 + t1) + (t2 + t3)) + ... over the chains.
// Every row sum of the pivoted QR and of the Q formation is taken this way.
template <class X, class Y>
double rowsum16(int a, int m, X x, Y y) {
  if (g_mode & MODE_ASC_SUMS) {  // textbook order: one chain, ascending rows
    double t = 0.0;
    for (int i = a; i < m; ++i) t = std::fma(x(i), y(i), t);
    return t;
  }
  double t[16] = {0.0};
  for (int i = a; i < m; ++i) t[i % 16] = std::fma(x(i), y(i), t[i % 16]);
  for (int d = 1; d < 16; d *= 2)
    for (int q = 0; q < 16; q += 2 * d) t[q] = t[q] + t[q + d];
  return t[0];
}

Cpqr cpqr(const Mat& M, double tol) {
  Cpqr out;
  int m = M.r, n = M.c;
  out.m = m;
  Mat A = M;
  out.perm.resize(n);
  for (int j = 0; j < n; ++j) out.perm[j] = j;
  double r11 = 0.0;
  int s = 0;
  int smax = std::min(m, n);
  for (; s < smax; ++s) {
    // pivot: the lowest-index column whose trailing norm is within a relative 1e-11 of the
    // largest (norms that equal in exact arithmetic, as the columns of an orthonormal basis
    // block, count as ties whatever their rounding)
    std::vector<double> nrm(n, 0.0);
    double mx = -1.0;
    for (int j = s; j < n; ++j) {
      double t = rowsum16(s, m, [&](int i) { return A.at(i, j); }, [&](int i) { return A.at(i, j); });
      nrm[j] = std::sqrt(t);
      mx = std::max(mx, nrm[j]);
    }
    int p = s;
    for (int j = s; j < n; ++j)
      if (nrm[j] >= mx * (1.0 - kTieTol)) { p = j; break; }
    double best = nrm[p];
    if (s == 0) {
      r11 = best;
      if (r11 == 0.0) break;
    } else if (best <= tol * r11) {
      out.next = best / (tol * r11);
      break;
    }
    out.kept = best / (tol * r11);
    if (p != s) {
      for (int i = 0; i < m; ++i) std::swap(A.at(i, s), A.at(i, p));
      std::swap(out.perm[s], out.perm[p]);
    }
    // reflector H = I - tau v v^T mapping A[s:,s] to beta e_1
    double x0 = A.at(s, s);
    double alpha = best;
    double beta = (x0 >= 0.0) ? -alpha : alpha;
    std::vector<double> v(m, 0.0);
    double tau = 0.0;
    if (alpha != 0.0) {
      double scale = x0 - beta;
      v[s] = 1.0;
      for (int i = s + 1; i < m; ++i) v[i] = A.at(i, s) / scale;
      tau = (beta - x0) / beta;
    }
    for (int j = s + 1; j < n; ++j) {
      double w = rowsum16(s, m, [&](int i) { return v[i]; }, [&](int i) { return A.at(i, j); });
      w *= tau;
      for (int i = s; i < m; ++i) A.at(i, j) = std::fma(-w, v[i], A.at(i, j));
    }
    A.at(s, s) = beta;
    for (int i = s + 1; i < m; ++i) A.at(i, s) = 0.0;
    out.v.push_back(v);
    out.tau.push_back(tau);
    g_flops[3] += 4.0 * (m - s) * (n - s);
  }
  out.rank = (int)out.v.size();
  out.R = Mat(out.rank, n);
  for (int i = 0; i < out.rank; ++i)
    for (int j = i; j < n; ++j) out.R.at(i, j) = A.at(i, j);
  return out;
}
// First q columns of Q = H_1 H_2 ... H_rank (m x q).  Columns beyond the rank are the
// further columns of the same orthogonal Householder Q (the paper leaves them open).
Mat cpqr_q(const Cpqr& f, int q) {
  int m = f.m;
  Mat Q(m, q);
  for (int j = 0; j < q && j < m; ++j) Q.at(j, j) = 1.0;
  for (int s = f.rank - 1; s >= 0; --s) {
    const std::vector<double>& v = f.v[s];
    double tau = f.tau[s];
    for (int j = 0; j < q; ++j) {
      double w = rowsum16(s, m, [&](int i) { return v[i]; }, [&](int i) { return Q.at(i, j); });
      w *= tau;
      for (int i = s; i < m; ++i) Q.at(i, j) = std::fma(-w, v[i], Q.at(i, j));
    }
  }
  g_flops[3] += 4.0 * m * q * f.rank;
  return Q;
}

// e^x by Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2 (ln2 split in a high part with
// trailing zero bits and a low correction), the Taylor series of e^r to degree 13 in Horner
// form (truncation below 4e-18 relative on the reduced range) and an exact scaling by 2^k.
double kexp(double x) {
  if (x < -745.0) return 0.0;
  double kd = std::rint(x * 1.4426950408889634);
  double r = std::fma(-kd, 6.93147180369123816490e-01, x);
  r = std::fma(-kd, 1.90821492927058770002e-10, r);
  double p = 1.6059043836821613e-10;
  p = std::fma(p, r, 2.08767569878681e-09);
  p = std::fma(p, r, 2.505210838544172e-08);
  p = std::fma(p, r, 2.755731922398589e-07);
  p = std::fma(p, r, 2.7557319223985893e-06);
  p = std::fma(p, r, 2.48015873015873e-05);
  p = std::fma(p, r, 0.0001984126984126984);
  p = std::fma(p, r, 0.001388888888888889);
  p = std::fma(p, r, 0.008333333333333333);
  p = std::fma(p, r, 0.041666666666666664);
  p = std::fma(p, r, 0.16666666666666666);
  p = std::fma(p, r, 0.5);
  p = std::fma(p, r, 1.0);
  p = std::fma(p, r, 1.0);
  return std::ldexp(p, (int)kd);
}

// ----------------------------------------------------------------------------------------
// Kernel matrix A_ij = kappa(|p_i - p_j|) + shift * delta_ij  (the N-body matrix of Sec. 2)
// ----------------------------------------------------------------------------------------
struct Kern {
  const double* pts;
  int d, kind;
  double scale, shift;
  double operator()(int64_t i, int64_t j) const {
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
      double z = pts[i * d + t] - pts[j * d + t];
      r2 += z * z;
    }
    double v;
    if (kind == 0) v = (g_mode & MODE_STD_EXP) ? std::exp(-std::sqrt(r2) / scale) : kexp(-std::sqrt(r2) / scale);
    else v = 1.0 / std::sqrt(r2 + scale * scale);
    if (i == j) v += shift;
    return v;
  }
};

// ACA with partial pivoting (the reading taken of the NNCA pivot search, Sec. 2.3).  Works on an
// implicitly given m x n matrix; returns pivots in selection order and the factors.
struct AcaOut {
  std::vector<int> I, J;
  std::vector<std::vector<double>> U, V;  // U[k] length m, V[k] length n
  double stop_margin = 1e300;             // |log(|u||v| / (tol |S|))| at the last two tests
  double gap = 1e300;                     // min relative gap between best and second argmax
};
template <class F>
AcaOut aca_pp(int m, int n, const F& M, double tol) {
  AcaOut o;
  std::vector<char> rused(m, 0), cused(n, 0);
  int kmax = std::min(m, n);
  if (kmax == 0) return o;
  int i = 0;
  double nrm2 = 0.0;
  std::vector<double> r(n), u(m);
  while ((int)o.I.size() < kmax) {
    int k = (int)o.I.size();
    for (int j = 0; j < n; ++j) {
      double a = M(i, j);
      for (int l = 0; l < k; ++l) a = std::fma(-o.U[l][i], o.V[l][j], a);
      r[j] = a;
    }
    rused[i] = 1;
    int jb = -1;
    double best = -1.0, second = -1.0;
    for (int j = 0; j < n; ++j) {
      if (cused[j]) continue;
      double t = std::fabs(r[j]);
      if (t > best) { second = best; best = t; jb = j; }
      else if (t > second) second = t;
    }
    if (jb < 0) break;
    if (best == 0.0) {  // exactly zero residual row: skip it, take the lowest unused row
      int ni = -1;
      for (int t = 0; t < m; ++t)
        if (!rused[t]) { ni = t; break; }
      if (ni < 0) break;
      i = ni;
      continue;
    }
    if (second >= 0.0) o.gap = std::min(o.gap, (best - second) / best);
    double delta = r[jb];
    std::vector<double> v(n);
    for (int j = 0; j < n; ++j) v[j] = r[j] / delta;
    for (int t = 0; t < m; ++t) {
      double a = M(t, jb);
      for (int l = 0; l < k; ++l) a = std::fma(-o.V[l][jb], o.U[l][t], a);
      u[t] = a;
    }
    cused[jb] = 1;
    double uu = 0.0, vv = 0.0, cross = 0.0;
    for (int t = 0; t < m; ++t) uu += u[t] * u[t];
    for (int j = 0; j < n; ++j) vv += v[j] * v[j];
    for (int l = 0; l < k; ++l) {
      double du = 0.0, dv = 0.0;
      for (int t = 0; t < m; ++t) du += o.U[l][t] * u[t];
      for (int j = 0; j < n; ++j) dv += o.V[l][j] * v[j];
      cross += du * dv;
    }
    nrm2 += 2.0 * cross + uu * vv;
    o.I.push_back(i);
    o.J.push_back(jb);
    o.U.push_back(u);
    o.V.push_back(v);
    double lhs = std::sqrt(uu * vv), rhs = tol * std::sqrt(nrm2);
    if (rhs > 0.0) o.stop_margin = std::min(o.stop_margin, std::fabs(std::log(lhs / rhs)));
    if (lhs <= rhs) break;
    int ib = -1;
    double ub = -1.0;
    for (int t = 0; t < m; ++t) {
      if (rused[t]) continue;
      double a = std::fabs(u[t]);
      if (a > ub) { ub = a; ib = t; }
    }
    if (ib < 0) break;
    i = ib;  // ties and the all-zero case both give the lowest unused row
  }
  return o;
}

// ----------------------------------------------------------------------------------------
// Sparse block store of the extended system (Sec. 3.1): blocks keyed by (row var, col var)
// ----------------------------------------------------------------------------------------
enum VK { VX = 0, VY = 1, VZ = 2, Vx = 3, Vz = 4, Vy = 5 };
inline int64_t var(int kind, int level, int box) {
  return ((int64_t)kind << 40) | ((int64_t)level << 32) | (int64_t)(uint32_t)box;
}
inline int vkind(int64_t v) { return (int)(v >> 40); }
inline int vlevel(int64_t v) { return (int)((v >> 32) & 0xff); }
inline int vbox(int64_t v) { return (int)(v & 0xffffffff); }

struct Store {
  std::map<std::pair<int64_t, int64_t>, Mat> blk;
  std::map<int64_t, std::set<int64_t>> rows, cols;
  std::map<int64_t, int> dim;
  int d(int64_t v) const {
    auto it = dim.find(v);
    return it == dim.end() ? 0 : it->second;
  }
  Mat* find(int64_t r, int64_t c) {
    auto it = blk.find({r, c});
    return it == blk.end() ? nullptr : &it->second;
  }
  Mat get(int64_t r, int64_t c) {  // zero block if absent
    Mat* p = find(r, c);
    if (p) return *p;
    return Mat(d(r), d(c));
  }
  void set(int64_t r, int64_t c, const Mat& m) {
    if (m.r == 0 || m.c == 0) { erase(r, c); return; }
    blk[{r, c}] = m;
    rows[r].insert(c);
    cols[c].insert(r);
  }
  void erase(int64_t r, int64_t c) {
    blk.erase({r, c});
    auto it = rows.find(r);
    if (it != rows.end()) it->second.erase(c);
    auto jt = cols.find(c);
    if (jt != cols.end()) jt->second.erase(r);
  }
  std::vector<int64_t> row_cols(int64_t r) {
    auto it = rows.find(r);
    if (it == rows.end()) return {};
    return std::vector<int64_t>(it->second.begin(), it->second.end());
  }
  std::vector<int64_t> col_rows(int64_t c) {
    auto it = cols.find(c);
    if (it == cols.end()) return {};
    return std::vector<int64_t>(it->second.begin(), it->second.end());
  }
};

struct Factor {
  int level = 0, box = 0;
  std::vector<int64_t> PR, PC, Or, Oc;
  std::vector<int> dPR, dPC, dOr, dOc;
  Mat LU;
  std::vector<int> perm;
  Mat Cb, W;
};

struct Level {
  int nb = 0;
  std::vector<std::array<int, 3>> coord;
  std::vector<std::vector<int>> nbr, il;
  std::vector<std::vector<int64_t>> pts;   // t^B = s^B (u = v), ascending original index
  std::vector<std::vector<int64_t>> ti;    // incoming pivots t^{B,i}
  std::vector<std::vector<int64_t>> si;    // s^{B,i}
  std::vector<int> knn;                    // NNCA rank
  std::vector<Mat> U, Vs;                  // leaf L2P U_B (n x k) and P2M V_B^* (k x n)
  std::vector<Mat> Ud, Vds;                // L2L U^dagger_B (k_B x k_P), M2M V^dagger*_B (k_P x k_B)
  std::vector<std::vector<Mat>> m2l;       // per box, per IL entry: A_BD (k_B x k_D)
  std::vector<int> order;                  // elimination order: colour-major, Morton inside a colour
  std::vector<int> kfin, nfin;             // rank and x-size at elimination
};

}  // namespace

struct oracle_sys {
  int64_t N = 0;
  int d = 2, L = 2, leaf = 64;
  Kern K{};
  double tol = 1e-10;
  std::vector<double> pts;
  std::vector<Level> lev;  // index by level 0..L
  Store S;
  std::vector<Factor> fac;
  Mat top;
  std::vector<int> top_perm;
  std::vector<int64_t> top_vars;  // Z^{(2)} row vars == y^{(2)} col vars (boxes)
  std::vector<int> top_dims;
  bool factored = false;
  std::string err;
  std::vector<std::array<int, 4>> trace;
  std::vector<std::array<int, 6>> trace_ranks;     // r1..r4 (P2P) or r5, r6, then k_i', k_j'
  std::vector<std::array<double, 8>> trace_ratio;  // per RRQR: kept, next ratio
  int64_t far_fill = 0;
  int mode = 0;
  // rows whose right-hand side may be nonzero at this point of the elimination (the X rows of
  // every level, and every row an elimination has updated); compressions must not transform them
  std::set<int64_t> rhs_rows;
  int64_t rhs_violations = 0;
  double cpqr_margin = 1e300, aca_stop = 1e300, aca_gap = 1e300;
  double flops[5] = {0, 0, 0, 0, 0};
  Mat dense_ext;  // built on demand
};

namespace {

// Morton code with coordinate 0 in the lowest bit of every d-bit group; the children of
// box P are (P << d) | ch.
int64_t morton(const int* c, int d, int l) {
  int64_t m = 0;
  for (int b = 0; b < l; ++b)
    for (int t = 0; t < d; ++t) m |= (int64_t)((c[t] >> b) & 1) << (b * d + t);
  return m;
}
void demorton(int64_t m, int d, int l, int* c) {
  for (int t = 0; t < d; ++t) c[t] = 0;
  for (int b = 0; b < l; ++b)
    for (int t = 0; t < d; ++t) c[t] |= (int)((m >> (b * d + t)) & 1) << b;
}
int cheb(const std::array<int, 3>& a, const std::array<int, 3>& b, int d) {
  int m = 0;
  for (int t = 0; t < d; ++t) m = std::max(m, std::abs(a[t] - b[t]));
  return m;
}

// Sec. 2.1: smallest hypercube holding the points (centred at the bounding-box
// midpoint, side = largest extent), uniform subdivision to depth
// L = max(2, ceil(log_{2^d}(N / n_max))).
void build_tree(oracle_sys& s) {
  int d = s.d;
  double lo[3], hi[3];
  for (int t = 0; t < d; ++t) { lo[t] = 1e300; hi[t] = -1e300; }
  for (int64_t i = 0; i < s.N; ++i)
    for (int t = 0; t < d; ++t) {
      lo[t] = std::min(lo[t], s.pts[i * d + t]);
      hi[t] = std::max(hi[t], s.pts[i * d + t]);
    }
  double side = 0.0;
  for (int t = 0; t < d; ++t) side = std::max(side, hi[t] - lo[t]);
  if (side == 0.0) side = 1.0;
  double base[3];
  for (int t = 0; t < d; ++t) base[t] = (lo[t] + hi[t]) * 0.5 - side * 0.5;
  int L = s.L;
  int64_t nside = (int64_t)1 << L;
  s.lev.assign(L + 1, Level());
  for (int l = 0; l <= L; ++l) {
    Level& lv = s.lev[l];
    lv.nb = 1 << (d * l);
    lv.coord.resize(lv.nb);
    lv.pts.assign(lv.nb, {});
    for (int b = 0; b < lv.nb; ++b) {
      int c[3] = {0, 0, 0};
      demorton(b, d, l, c);
      lv.coord[b] = {c[0], c[1], c[2]};
    }
  }
  for (int64_t i = 0; i < s.N; ++i) {
    int c[3] = {0, 0, 0};
    for (int t = 0; t < d; ++t) {
      double f = std::floor((s.pts[i * d + t] - base[t]) / side * (double)nside);
      int64_t q = (int64_t)f;
      if (q < 0) q = 0;
      if (q > nside - 1) q = nside - 1;
      c[t] = (int)q;
    }
    int64_t leaf = morton(c, d, L);
    s.lev[L].pts[leaf].push_back(i);
  }
  // a coarser box lists its points in tree order: children in Morton order, each child's
  // points in its own order (ascending original index at the leaf)
  for (int l = L - 1; l >= 0; --l)
    for (int b = 0; b < s.lev[l].nb; ++b)
      for (int ch = 0; ch < (1 << d); ++ch) {
        const std::vector<int64_t>& t = s.lev[l + 1].pts[(b << d) | ch];
        s.lev[l].pts[b].insert(s.lev[l].pts[b].end(), t.begin(), t.end());
      }
}

// Sec. 2.2, neighbour / interaction-list table (i in N(i); admissible iff integer
// Chebyshev distance >= 2, which is the eta = sqrt(d) condition on the box geometry).
void build_lists(oracle_sys& s) {
  int d = s.d;
  for (int l = 0; l <= s.L; ++l) {
    Level& lv = s.lev[l];
    lv.nbr.assign(lv.nb, {});
    lv.il.assign(lv.nb, {});
    for (int b = 0; b < lv.nb; ++b)
      for (int q = 0; q < lv.nb; ++q)
        if (cheb(lv.coord[b], lv.coord[q], d) <= 1) lv.nbr[b].push_back(q);
    if (l < 2) continue;
    Level& up = s.lev[l - 1];
    for (int b = 0; b < lv.nb; ++b) {
      int P = b >> d;
      std::vector<int> cand;
      for (int Q : up.nbr[P])
        for (int ch = 0; ch < (1 << d); ++ch) cand.push_back((Q << d) | ch);
      std::sort(cand.begin(), cand.end());
      for (int q : cand)
        if (cheb(lv.coord[b], lv.coord[q], d) >= 2) lv.il[b].push_back(q);
    }
  }
}

// Solve X C = B for X (C k x k, B r x k) through an LU of C^T (never an explicit inverse).
Mat right_solve(const Mat& C, const Mat& B) {
  Mat Ct = tr(C);
  std::vector<int> perm;
  if (lu_factor(Ct, perm)) return Mat();
  Mat Xt = lu_solve(Ct, perm, tr(B), -1);
  return tr(Xt);
}
// Solve C X = B for X
Mat left_solve(const Mat& C, const Mat& B) {
  Mat LU = C;
  std::vector<int> perm;
  if (lu_factor(LU, perm)) return Mat();
  return lu_solve(LU, perm, B, -1);
}
Mat kblock(const oracle_sys& s, const std::vector<int64_t>& r, const std::vector<int64_t>& c) {
  Mat M((int)r.size(), (int)c.size());
  for (size_t i = 0; i < r.size(); ++i)
    for (size_t j = 0; j < c.size(); ++j) M.at((int)i, (int)j) = s.K(r[i], c[j]);
  return M;
}

// Sec. 2.3: NNCA, bottom-up.  Row set T = t^B at the leaf and the children's incoming
// pivots above it; column search space F^{B,i} = sources of IL(B) (eq. Fj).  Outgoing
// pivots are the incoming ones swapped (u = v and a symmetric kernel).
bool build_nnca(oracle_sys& s) {
  int d = s.d, L = s.L;
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    lv.ti.assign(lv.nb, {});
    lv.si.assign(lv.nb, {});
    lv.knn.assign(lv.nb, 0);
    for (int B = 0; B < lv.nb; ++B) {
      std::vector<int64_t> T;
      if (l == L) T = lv.pts[B];
      else
        for (int ch = 0; ch < (1 << d); ++ch) {
          const std::vector<int64_t>& t = s.lev[l + 1].ti[(B << d) | ch];
          T.insert(T.end(), t.begin(), t.end());
        }
      std::vector<int64_t> F;
      for (int D : lv.il[B]) F.insert(F.end(), lv.pts[D].begin(), lv.pts[D].end());
      const Kern& K = s.K;
      auto M = [&](int i, int j) { return K(T[i], F[j]); };
      AcaOut a = aca_pp((int)T.size(), (int)F.size(), M, s.tol);
      s.aca_stop = std::min(s.aca_stop, a.stop_margin);
      s.aca_gap = std::min(s.aca_gap, a.gap);
      for (size_t q = 0; q < a.I.size(); ++q) {
        lv.ti[B].push_back(T[a.I[q]]);
        lv.si[B].push_back(F[a.J[q]]);
      }
      lv.knn[B] = (int)a.I.size();
    }
    // operators of the table following eq. NCA
    lv.m2l.assign(lv.nb, {});
    if (l == L) { lv.U.assign(lv.nb, Mat()); lv.Vs.assign(lv.nb, Mat()); }
    for (int B = 0; B < lv.nb; ++B) {
      int k = lv.knn[B];
      // t^{B,o} := s^{B,i}, s^{B,o} := t^{B,i}
      const std::vector<int64_t>& to = lv.si[B];
      const std::vector<int64_t>& so = lv.ti[B];
      Mat C = kblock(s, lv.ti[B], lv.si[B]);   // A_{t^{B,i} s^{B,i}}
      Mat Co = kblock(s, to, so);              // A_{t^{B,o} s^{B,o}}
      if (l == L) {
        // L2P U_B = A_{t^B s^{B,i}} (A_{t^{B,i} s^{B,i}})^{-1};  P2M V_B^* = (A_{t^{B,o}s^{B,o}})^{-1} A_{t^{B,o} s^B}
        if (k > 0) {
          lv.U[B] = right_solve(C, kblock(s, lv.pts[B], lv.si[B]));
          lv.Vs[B] = left_solve(Co, kblock(s, to, lv.pts[B]));
          if (lv.U[B].r == 0 || lv.Vs[B].r == 0) {
            s.err = "singular NNCA cross matrix at level " + std::to_string(l) + " box " + std::to_string(B);
            return false;
          }
        } else {
          lv.U[B] = Mat((int)lv.pts[B].size(), 0);
          lv.Vs[B] = Mat(0, (int)lv.pts[B].size());
        }
      }
      // M2L A_BD = A_{t^{B,i} s^{D,o}} for D in IL(B)
      for (int D : lv.il[B]) lv.m2l[B].push_back(kblock(s, lv.ti[B], lv.ti[D]));
      // children's L2L / M2M (operators of level l+1 boxes towards their parent B)
      if (l < L) {
        Level& dn = s.lev[l + 1];
        if (dn.Ud.empty()) { dn.Ud.assign(dn.nb, Mat()); dn.Vds.assign(dn.nb, Mat()); }
        for (int ch = 0; ch < (1 << d); ++ch) {
          int c = (B << d) | ch;
          int kc = dn.knn[c];
          if (k > 0 && kc > 0) {
            dn.Ud[c] = right_solve(C, kblock(s, dn.ti[c], lv.si[B]));   // A_{t^{c,i} s^{B,i}} C^{-1}
            dn.Vds[c] = left_solve(Co, kblock(s, to, dn.ti[c]));        // (A_{t^{B,o}s^{B,o}})^{-1} A_{t^{B,o} s^{c,o}}
            if (dn.Ud[c].r == 0 || dn.Vds[c].r == 0) {
              s.err = "singular NNCA cross matrix at level " + std::to_string(l) + " box " + std::to_string(B);
              return false;
            }
          } else {
            dn.Ud[c] = Mat(kc, k);
            dn.Vds[c] = Mat(k, kc);
          }
        }
      }
    }
  }
  return true;
}

// Sec. 3.1: the extended sparse system (equations X: K x + U z = b, Y: V^T x - y = 0,
// Z: U^dagger z_P + sum A y - z = 0).
void assemble(oracle_sys& s) {
  int d = s.d, L = s.L;
  Store& S = s.S;
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    for (int b = 0; b < lv.nb; ++b) {
      int k = lv.knn[b];
      S.dim[var(VY, l, b)] = k;
      S.dim[var(VZ, l, b)] = k;
      S.dim[var(Vz, l, b)] = k;
      S.dim[var(Vy, l, b)] = k;
      if (l == L) {
        int n = (int)lv.pts[b].size();
        S.dim[var(VX, l, b)] = n;
        S.dim[var(Vx, l, b)] = n;
      }
    }
  }
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    for (int b = 0; b < lv.nb; ++b) {
      int k = lv.knn[b];
      if (l == L) {
        // Equation X_b: sum_{q in N(b)} K_bq x_q + U_b z_b = b_b
        for (int q : lv.nbr[b]) S.set(var(VX, l, b), var(Vx, l, q), kblock(s, lv.pts[b], lv.pts[q]));
        S.set(var(VX, l, b), var(Vz, l, b), lv.U[b]);
        // Equation Y_b: V_b^* x_b - y_b = 0
        S.set(var(VY, l, b), var(Vx, l, b), lv.Vs[b]);
      }
      S.set(var(VY, l, b), var(Vy, l, b), eye(k, -1.0));
      // Equation Z_b: U^dagger_b z_P + sum_{D in IL(b)} A_bD y_D - z_b = 0
      S.set(var(VZ, l, b), var(Vz, l, b), eye(k, -1.0));
      for (size_t q = 0; q < lv.il[b].size(); ++q) S.set(var(VZ, l, b), var(Vy, l, lv.il[b][q]), lv.m2l[b][q]);
      if (l > 2) {
        int P = b >> d;
        S.set(var(VZ, l, b), var(Vz, l - 1, P), lv.Ud[b]);
        // Y_P row: M2M of the child, part of the parent's P2M (Table of non-leaf operators)
        S.set(var(VY, l - 1, P), var(Vy, l, b), lv.Vds[b]);
      }
    }
  }
}

// Colour-major order, colour = (c_1 mod 5, ..., c_d mod 5) lexicographic, Morton inside.
void build_order(oracle_sys& s) {
  int d = s.d;
  for (int l = 2; l <= s.L; ++l) {
    Level& lv = s.lev[l];
    std::vector<std::pair<int64_t, int>> key;
    for (int b = 0; b < lv.nb; ++b) {
      int64_t col = 0;
      for (int t = 0; t < d; ++t) col = col * 5 + (lv.coord[b][t] % 5);
      key.push_back({col * (int64_t)lv.nb + b, b});
    }
    std::sort(key.begin(), key.end());
    lv.order.clear();
    for (auto& kv : key) lv.order.push_back(kv.second);
  }
}

// Level transition (eq. particleAtNonLeafLevel and the X^{(l)} form): x_b^{(l)} stacks the
// children's y^{(l+1)}, row X_b^{(l)} stacks the children's Z^{(l+1)} rows.
void merge_level(oracle_sys& s, int l) {
  int d = s.d;
  Store& S = s.S;
  Level& lv = s.lev[l];
  int nch = 1 << d;
  // offsets of the children inside the parent's stacked vector
  std::vector<std::vector<int>> off(lv.nb, std::vector<int>(nch + 1, 0));
  for (int b = 0; b < lv.nb; ++b) {
    for (int ch = 0; ch < nch; ++ch) off[b][ch + 1] = off[b][ch] + S.d(var(Vy, l + 1, (b << d) | ch));
    S.dim[var(VX, l, b)] = off[b][nch];
    S.dim[var(Vx, l, b)] = off[b][nch];
  }
  std::map<std::pair<int64_t, int64_t>, Mat> merged;
  auto tgt = [&](int64_t r, int64_t c) -> Mat& {
    auto it = merged.find({r, c});
    if (it == merged.end()) it = merged.emplace(std::make_pair(r, c), Mat(S.d(r), S.d(c))).first;
    return it->second;
  };
  std::vector<std::pair<int64_t, int64_t>> kill;
  for (auto& kv : S.blk) {
    int64_t r = kv.first.first, c = kv.first.second;
    bool rz = vkind(r) == VZ && vlevel(r) == l + 1;
    bool cy = vkind(c) == Vy && vlevel(c) == l + 1;
    if (!rz && !cy) continue;
    int64_t R = r, C = c;
    int ro = 0, co = 0;
    if (rz) { int cb = vbox(r); R = var(VX, l, cb >> d); ro = off[cb >> d][cb & (nch - 1)]; }
    if (cy) { int cb = vbox(c); C = var(Vx, l, cb >> d); co = off[cb >> d][cb & (nch - 1)]; }
    Mat& T = tgt(R, C);
    const Mat& B = kv.second;
    for (int i = 0; i < B.r; ++i)
      for (int j = 0; j < B.c; ++j) T.at(ro + i, co + j) += B.at(i, j);
    kill.push_back(kv.first);
  }
  for (auto& k : kill) S.erase(k.first, k.second);
  for (auto& kv : merged) S.set(kv.first.first, kv.first.second, kv.second);
}

void set_basis(oracle_sys& s, int l, int b, const Mat& U, const Mat& V) {
  Store& S = s.S;
  // the new row Y_b is the old one transformed by the change of multipole basis
  if (s.rhs_rows.count(var(VY, l, b))) ++s.rhs_violations;
  int k = U.c;
  S.dim[var(VY, l, b)] = k;
  S.dim[var(VZ, l, b)] = k;
  S.dim[var(Vz, l, b)] = k;
  S.dim[var(Vy, l, b)] = k;
  S.set(var(VX, l, b), var(Vz, l, b), U);
  S.set(var(VY, l, b), var(Vx, l, b), tr(V));
  S.set(var(VY, l, b), var(Vy, l, b), eye(k, -1.0));
  S.set(var(VZ, l, b), var(Vz, l, b), eye(k, -1.0));
}

void note_cpqr(oracle_sys& s, const Cpqr& f) {
  if (f.rank > 0 && f.kept > 0) s.cpqr_margin = std::min(s.cpqr_margin, std::fabs(std::log(f.kept)));
  if (f.next > 0) s.cpqr_margin = std::min(s.cpqr_margin, std::fabs(std::log(f.next)));
}

// Left-multiply every block of row Z_b except the -I and the listed pair block by Lb; the
// L2L block and all M2L blocks of the row are covered (eq. for A_ic := L_i A_ic and the L2L
// update), at non-leaf levels too.
void row_update(oracle_sys& s, int l, int b, const Mat& Lb, int64_t skip_col) {
  Store& S = s.S;
  int64_t R = var(VZ, l, b);
  if (s.rhs_rows.count(R)) ++s.rhs_violations;  // a row operation on a row with a right-hand side
  for (int64_t c : S.row_cols(R)) {
    if (c == var(Vz, l, b) || c == skip_col) continue;
    Mat* B = S.find(R, c);
    S.set(R, c, mul(Lb, *B, 4));
  }
}
// Right-multiply every block of column y_b except the -I and the pair block by Rb^T (the
// A_dj := A_dj R_j^* and M2M updates).
void col_update(oracle_sys& s, int l, int b, const Mat& Rb, int64_t skip_row) {
  Store& S = s.S;
  int64_t C = var(Vy, l, b);
  Mat Rt = tr(Rb);
  for (int64_t r : S.col_rows(C)) {
    if (r == var(VY, l, b) || r == skip_row) continue;
    Mat* B = S.find(r, C);
    S.set(r, C, mul(*B, Rt, 4));
  }
}

// Result of one compression: new bases, the coefficient matrices L, R of the boxes whose
// bases change and the new values of the two pair blocks.
struct Comp {
  int kind = 0, i = 0, j = 0;  // P2P: pair (i, j); P2L: box i and eliminated box r = j
  Mat Uin, Vin, Ujn, Vjn, Li, Ri, Lj, Rj;
  Mat A1, A2;  // P2P: (Z_i, y_j), (Z_j, y_i); P2L: (Z_i, y_r), (Z_r, y_i)
};

// Sec. 3.2.1: compression and redirection of the P2P fill-in pair (P2P_ij, P2P_ji), with the
// Readings of Sec. 3.2.1-3.2.3 (four RRQRs, per-box rank = max of its U-side and V-side ranks,
// coefficients by projection onto the final orthonormal bases).
Comp compress_p2p(oracle_sys& s, int l, int i, int j) {
  Store& S = s.S;
  Comp c;
  c.kind = 0; c.i = i; c.j = j;
  int64_t Xi = var(VX, l, i), Xj = var(VX, l, j), xi = var(Vx, l, i), xj = var(Vx, l, j);
  Mat Ui = S.get(Xi, var(Vz, l, i)), Uj = S.get(Xj, var(Vz, l, j));
  Mat Vi = tr(S.get(var(VY, l, i), xi)), Vj = tr(S.get(var(VY, l, j), xj));
  Mat Fij = S.get(Xi, xj), Fji = S.get(Xj, xi);
  double tol = s.tol;
  Cpqr f1 = cpqr(hcat(Ui, Fij), tol);   // [U_i | P2P_ij] = U~_i L_ij
  Cpqr f2 = cpqr(hcat(Uj, Fji), tol);   // [U_j | P2P_ji] = U~_j L_ji
  Mat Q1r = cpqr_q(f1, f1.rank), Q2r = cpqr_q(f2, f2.rank);
  Cpqr f3 = cpqr(hcat(Vj, mul(tr(Fij), Q1r, 4)), tol);  // [V_j | L~_ij^*] = V~_j R_ij
  Cpqr f4 = cpqr(hcat(Vi, mul(tr(Fji), Q2r, 4)), tol);  // [V_i | L~_ji^*] = V~_i R_ji
  note_cpqr(s, f1); note_cpqr(s, f2); note_cpqr(s, f3); note_cpqr(s, f4);
  int ki = std::max(f1.rank, f4.rank), kj = std::max(f2.rank, f3.rank);
  s.trace_ranks.push_back({f1.rank, f2.rank, f3.rank, f4.rank, ki, kj});
  s.trace_ratio.push_back({f1.kept, f1.next, f2.kept, f2.next, f3.kept, f3.next, f4.kept, f4.next});
  c.Uin = cpqr_q(f1, ki); c.Vin = cpqr_q(f4, ki); c.Ujn = cpqr_q(f2, kj); c.Vjn = cpqr_q(f3, kj);
  c.Li = mul(tr(c.Uin), Ui, 4); c.Ri = mul(tr(c.Vin), Vi, 4);   // U_i = U~_i L_i, V_i = V~_i R_i
  c.Lj = mul(tr(c.Ujn), Uj, 4); c.Rj = mul(tr(c.Vjn), Vj, 4);
  Mat Ltij = mul(tr(c.Uin), Fij, 4);        // P2P_ij = U~_i L~_ij
  Mat Rtij = mul(tr(c.Vjn), tr(Ltij), 4);   // L~_ij^* = V~_j R~_ij
  Mat Ltji = mul(tr(c.Ujn), Fji, 4);
  Mat Rtji = mul(tr(c.Vin), tr(Ltji), 4);
  int64_t Zi = var(VZ, l, i), Zj = var(VZ, l, j), yi = var(Vy, l, i), yj = var(Vy, l, j);
  // A_ij := L_i A_ij R_j^* + R~_ij^*
  c.A1 = mul(mul(c.Li, S.get(Zi, yj), 4), tr(c.Rj), 4);
  Mat Rt1 = tr(Rtij);
  for (size_t q = 0; q < c.A1.a.size(); ++q) c.A1.a[q] += Rt1.a[q];
  c.A2 = mul(mul(c.Lj, S.get(Zj, yi), 4), tr(c.Ri), 4);
  Mat Rt2 = tr(Rtji);
  for (size_t q = 0; q < c.A2.a.size(); ++q) c.A2.a[q] += Rt2.a[q];
  return c;
}

// Sec. 3.2.2 and 3.2.3: compression of P2L_ri (row Z_r, column x_i) and M2P_ir (row X_i,
// column y_r), r eliminated, i about to be eliminated.  Box r's bases are frozen (bases of
// eliminated boxes never change).
Comp compress_p2l(oracle_sys& s, int l, int r, int i) {
  Store& S = s.S;
  Comp c;
  c.kind = 1; c.i = i; c.j = r;
  int64_t Xi = var(VX, l, i), xi = var(Vx, l, i), Zr = var(VZ, l, r), yr = var(Vy, l, r);
  int64_t Zi = var(VZ, l, i), yi = var(Vy, l, i);
  Mat Ui = S.get(Xi, var(Vz, l, i));
  Mat Vi = tr(S.get(var(VY, l, i), xi));
  Mat P2L = S.get(Zr, xi), M2P = S.get(Xi, yr);
  double tol = s.tol;
  Cpqr f5 = cpqr(hcat(Vi, tr(P2L)), tol);   // [V_i | P2L_ri^*] = V~_i R_ri
  Cpqr f6 = cpqr(hcat(Ui, M2P), tol);       // [U_i | M2P_ir]  = U~_i L_ir
  note_cpqr(s, f5); note_cpqr(s, f6);
  int ki = std::max(f5.rank, f6.rank);
  s.trace_ranks.push_back({f5.rank, f6.rank, 0, 0, ki, 0});
  s.trace_ratio.push_back({f5.kept, f5.next, f6.kept, f6.next, 0, 0, 0, 0});
  c.Vin = cpqr_q(f5, ki); c.Uin = cpqr_q(f6, ki);
  c.Ri = mul(tr(c.Vin), Vi, 4); c.Li = mul(tr(c.Uin), Ui, 4);
  // A_ir := L_i A_ir + L~_ir  with L~_ir = U~_i^* M2P_ir
  c.A1 = mul(c.Li, S.get(Zi, yr), 4);
  Mat add2 = mul(tr(c.Uin), M2P, 4);
  for (size_t q = 0; q < c.A1.a.size(); ++q) c.A1.a[q] += add2.a[q];
  // A_ri := A_ri R_i^* + R~_ri^*  with R~_ri^* = (V~_i^* P2L_ri^*)^* = P2L_ri V~_i
  c.A2 = mul(S.get(Zr, yi), tr(c.Ri), 4);
  Mat add1 = mul(P2L, c.Vin, 4);
  for (size_t q = 0; q < c.A2.a.size(); ++q) c.A2.a[q] += add1.a[q];
  return c;
}

// The other M2L, L2L and M2M blocks of the rows Z and columns y whose bases changed
// ("Other M2L updates", M2M and L2L updates): left factors first, for every compression of
// the round, then the right factors.
void comp_rows(oracle_sys& s, int l, const Comp& c) {
  row_update(s, l, c.i, c.Li, var(Vy, l, c.j));
  if (c.kind == 0) row_update(s, l, c.j, c.Lj, var(Vy, l, c.i));
}
void comp_cols(oracle_sys& s, int l, const Comp& c) {
  col_update(s, l, c.i, c.Ri, var(VZ, l, c.j));
  if (c.kind == 0) col_update(s, l, c.j, c.Rj, var(VZ, l, c.i));
}
// New bases, the redirected pair blocks, and the compressed fill-ins removed.
void comp_commit(oracle_sys& s, int l, const Comp& c) {
  Store& S = s.S;
  int i = c.i, j = c.j;
  if (c.kind == 0) {
    S.erase(var(VX, l, i), var(Vx, l, j));
    S.erase(var(VX, l, j), var(Vx, l, i));
    set_basis(s, l, i, c.Uin, c.Vin);
    set_basis(s, l, j, c.Ujn, c.Vjn);
  } else {
    S.erase(var(VZ, l, j), var(Vx, l, i));
    S.erase(var(VX, l, i), var(Vy, l, j));
    set_basis(s, l, i, c.Uin, c.Vin);
  }
  S.set(var(VZ, l, i), var(Vy, l, j), c.A1);
  S.set(var(VZ, l, j), var(Vy, l, i), c.A2);
}

// Algorithm "Efficient Elimination", the elimination step: pivot rows (X_i, Y_i) and columns
// (x_i, z_i) of eq. X2 / Y, LU with partial pivoting, Schur update of every coupled block.
bool eliminate(oracle_sys& s, int l, int i) {
  Store& S = s.S;
  Level& lv = s.lev[l];
  Factor F;
  F.level = l;
  F.box = i;
  for (int64_t v : {var(VX, l, i), var(VY, l, i)})
    if (S.d(v) > 0) { F.PR.push_back(v); F.dPR.push_back(S.d(v)); }
  for (int64_t v : {var(Vx, l, i), var(Vz, l, i)})
    if (S.d(v) > 0) { F.PC.push_back(v); F.dPC.push_back(S.d(v)); }
  lv.kfin[i] = S.d(var(Vz, l, i));
  lv.nfin[i] = S.d(var(Vx, l, i));
  int m = 0, mc = 0;
  for (int x : F.dPR) m += x;
  for (int x : F.dPC) mc += x;
  if (m != mc) {
    s.err = "non-square pivot block at level " + std::to_string(l) + " box " + std::to_string(i);
    return false;
  }
  std::set<int64_t> orset, ocset;
  for (int64_t c : F.PC)
    for (int64_t r : S.col_rows(c))
      if (std::find(F.PR.begin(), F.PR.end(), r) == F.PR.end()) orset.insert(r);
  for (int64_t r : F.PR)
    for (int64_t c : S.row_cols(r))
      if (std::find(F.PC.begin(), F.PC.end(), c) == F.PC.end()) ocset.insert(c);
  F.Or.assign(orset.begin(), orset.end());
  F.Oc.assign(ocset.begin(), ocset.end());
  // O8 check: every coupled variable belongs to a box of N(i) at this level (or the parent
  // locals/multipoles never appear here).
  auto near = [&](int64_t v) {
    if (vlevel(v) != l) return false;
    return cheb(lv.coord[vbox(v)], lv.coord[i], s.d) <= 1;
  };
  for (int64_t v : F.Or) if (!near(v)) s.far_fill++;
  for (int64_t v : F.Oc) if (!near(v)) s.far_fill++;
  for (int64_t v : F.Or) F.dOr.push_back(S.d(v));
  for (int64_t v : F.Oc) F.dOc.push_back(S.d(v));
  int R = 0, C = 0;
  for (int x : F.dOr) R += x;
  for (int x : F.dOc) C += x;
  // gather
  Mat Piv(m, m), Cb(R, m), Rb(m, C);
  {
    int ro = 0;
    for (size_t a = 0; a < F.PR.size(); ++a) {
      int co = 0;
      for (size_t b = 0; b < F.PC.size(); ++b) {
        Mat* B = S.find(F.PR[a], F.PC[b]);
        if (B) for (int x = 0; x < B->r; ++x) for (int y = 0; y < B->c; ++y) Piv.at(ro + x, co + y) = B->at(x, y);
        co += F.dPC[b];
      }
      co = 0;
      for (size_t b = 0; b < F.Oc.size(); ++b) {
        Mat* B = S.find(F.PR[a], F.Oc[b]);
        if (B) for (int x = 0; x < B->r; ++x) for (int y = 0; y < B->c; ++y) Rb.at(ro + x, co + y) = B->at(x, y);
        co += F.dOc[b];
      }
      ro += F.dPR[a];
    }
    ro = 0;
    for (size_t a = 0; a < F.Or.size(); ++a) {
      int co = 0;
      for (size_t b = 0; b < F.PC.size(); ++b) {
        Mat* B = S.find(F.Or[a], F.PC[b]);
        if (B) for (int x = 0; x < B->r; ++x) for (int y = 0; y < B->c; ++y) Cb.at(ro + x, co + y) = B->at(x, y);
        co += F.dPC[b];
      }
      ro += F.dOr[a];
    }
  }
  F.LU = Piv;
  int st = lu_factor(F.LU, F.perm);
  if (st) {
    s.err = "singular self-block at level " + std::to_string(l) + " box " + std::to_string(i);
    return false;
  }
  if (g_mode & MODE_ASC_BACK) {
    // textbook: substitution on the right-hand sides, ascending back substitution
    F.W = lu_solve(F.LU, F.perm, Rb, 1, false);
  } else {
    // W = Piv^{-1} [rhs] as the product of the explicit inverse of the pivot block (formed by
    // substitution on the identity's columns, column-oriented back substitution) with the
    // right-hand sides, each element summed in ascending k
    Mat Pinv = lu_solve(F.LU, F.perm, eye(m, 1.0), -1, true);
    F.W = mul(Pinv, Rb, 1);
    g_flops[1] += 2.0 * m * m * m;
  }
  Mat Upd = mul(Cb, F.W, 2);
  // scatter: A[O_r, O_c] -= A[O_r, (x_i, z_i)] Piv^{-1} A[(X_i, Y_i), O_c]
  {
    int ro = 0;
    for (size_t a = 0; a < F.Or.size(); ++a) {
      int co = 0;
      for (size_t b = 0; b < F.Oc.size(); ++b) {
        Mat T = S.get(F.Or[a], F.Oc[b]);
        for (int x = 0; x < T.r; ++x)
          for (int y = 0; y < T.c; ++y) T.at(x, y) -= Upd.at(ro + x, co + y);
        S.set(F.Or[a], F.Oc[b], T);
        co += F.dOc[b];
      }
      ro += F.dOr[a];
    }
  }
  for (int64_t r : F.Or) s.rhs_rows.insert(r);  // the elimination's right-hand-side updates
  for (int64_t r : F.PR)
    for (int64_t c : S.row_cols(r)) S.erase(r, c);
  for (int64_t c : F.PC)
    for (int64_t r : S.col_rows(c)) S.erase(r, c);
  F.Cb = Cb;
  s.fac.push_back(std::move(F));
  return true;
}

bool factor(oracle_sys& s) {
  int d = s.d, L = s.L;
  Store& S = s.S;
  s.rhs_rows.clear();
  s.rhs_violations = 0;
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    if (l < L) merge_level(s, l);
    for (int b = 0; b < lv.nb; ++b) s.rhs_rows.insert(var(VX, l, b));  // b on X^(L), stacked Z rows above
    lv.kfin.assign(lv.nb, 0);
    lv.nfin.assign(lv.nb, 0);
    std::vector<char> elim(lv.nb, 0);
    std::vector<int> pos(lv.nb, 0);
    for (int q = 0; q < lv.nb; ++q) pos[lv.order[q]] = q;
    std::set<std::pair<int, int>> vP2P;   // unordered (min, max)
    std::set<std::pair<int, int>> vP2L;   // ordered (eliminated, not eliminated)
    // colour batches of the order: the compressions of one batch touch disjoint rows and
    // columns except for commuting left/right factors on shared M2L blocks, and an
    // elimination never touches another box of its batch, so every batch runs as: the
    // r-th compression of each of its boxes for r = 0, 1, ... (left factors of the round,
    // then right factors), then the eliminations.  In the sequential mode every batch is one
    // box: its compressions one after the other, then its elimination.
    for (int q0 = 0; q0 < lv.nb;) {
      auto colour = [&](int b) {
        int64_t c = 0;
        for (int t = 0; t < d; ++t) c = c * 5 + (lv.coord[b][t] % 5);
        return c;
      };
      int q1 = q0;
      if (g_mode & MODE_SEQUENTIAL) q1 = q0 + 1;  // the Algorithm's order: one box after the other
      else
        while (q1 < lv.nb && colour(lv.order[q1]) == colour(lv.order[q0])) ++q1;
      std::vector<std::vector<std::pair<int, int>>> ops(q1 - q0);  // (kind, partner)
      size_t rounds = 0;
      for (int q = q0; q < q1; ++q) {
        int i = lv.order[q];
        // pending P2P pairs containing i, by increasing partner position
        std::vector<std::pair<int, int>> todo;
        for (auto& pr : vP2P)
          if (pr.first == i || pr.second == i) {
            int j = pr.first == i ? pr.second : pr.first;
            todo.push_back({pos[j], j});
          }
        std::sort(todo.begin(), todo.end());
        for (auto& t : todo) {
          ops[q - q0].push_back({0, t.second});
          vP2P.erase({std::min(i, t.second), std::max(i, t.second)});
        }
        todo.clear();
        for (auto& pr : vP2L)
          if (pr.second == i) todo.push_back({pos[pr.first], pr.first});
        std::sort(todo.begin(), todo.end());
        for (auto& t : todo) {
          ops[q - q0].push_back({1, t.second});
          vP2L.erase({t.second, i});
        }
        rounds = std::max(rounds, ops[q - q0].size());
      }
      for (size_t r = 0; r < rounds; ++r) {
        std::vector<Comp> res;
        for (int q = q0; q < q1; ++q) {
          if (r >= ops[q - q0].size()) continue;
          int i = lv.order[q];
          auto op = ops[q - q0][r];
          if (op.first == 0) res.push_back(compress_p2p(s, l, i, op.second));
          else res.push_back(compress_p2l(s, l, op.second, i));
          s.trace.push_back({l, i, op.first, op.second});
        }
        for (auto& c : res) comp_rows(s, l, c);
        for (auto& c : res) comp_cols(s, l, c);
        for (auto& c : res) comp_commit(s, l, c);
      }
      for (int q = q0; q < q1; ++q) {
        int i = lv.order[q];
        if (!eliminate(s, l, i)) return false;
        elim[i] = 1;
        // record the well-separated fill-ins created among N(i) (Algorithm, push steps)
        for (int p : lv.nbr[i])
          for (int r : lv.nbr[i]) {
            if (p == r || p == i || r == i) continue;
            if (cheb(lv.coord[p], lv.coord[r], d) < 2) continue;
            if (elim[p] && elim[r]) continue;
            if (elim[p]) vP2L.insert({p, r});
            else if (elim[r]) vP2L.insert({r, p});
            else vP2P.insert({std::min(p, r), std::max(p, r)});
          }
      }
      q0 = q1;
    }
    if (!vP2P.empty() || !vP2L.empty()) {
      s.err = "pending fill-ins left at the end of level " + std::to_string(l);
      return false;
    }
  }
  // the level-2 multipole system, solved directly at the end of the elimination (Sec. 3.2):
  // dense partial-pivot LU
  Level& l2 = s.lev[2];
  s.top_vars.clear();
  s.top_dims.clear();
  int Kt = 0;
  std::vector<int> toff;
  for (int b = 0; b < l2.nb; ++b) {
    int k = S.d(var(Vy, 2, b));
    toff.push_back(Kt);
    s.top_vars.push_back(b);
    s.top_dims.push_back(k);
    Kt += k;
  }
  s.top = Mat(Kt, Kt);
  for (int a = 0; a < l2.nb; ++a)
    for (int b = 0; b < l2.nb; ++b) {
      Mat* B = S.find(var(VZ, 2, a), var(Vy, 2, b));
      if (!B) continue;
      for (int x = 0; x < B->r; ++x)
        for (int y = 0; y < B->c; ++y) s.top.at(toff[a] + x, toff[b] + y) = B->at(x, y);
    }
  if (Kt > 0 && lu_factor(s.top, s.top_perm)) {
    s.err = "singular top-level system";
    return false;
  }
  return true;
}

bool solve(oracle_sys& s, const double* b, int64_t nrhs, double* x) {
  int d = s.d, L = s.L;
  int m = (int)nrhs;
  std::map<int64_t, Mat> rhs, sol;
  std::map<int64_t, int> dims;
  auto dimv = [&](int64_t v) { return s.S.d(v); };
  Level& lL = s.lev[L];
  for (int bx = 0; bx < lL.nb; ++bx) {
    const std::vector<int64_t>& t = lL.pts[bx];
    if (t.empty()) continue;
    Mat R((int)t.size(), m);
    for (size_t q = 0; q < t.size(); ++q)
      for (int c = 0; c < m; ++c) R.at((int)q, c) = b[c * s.N + t[q]];
    rhs[var(VX, L, bx)] = R;
  }
  auto getr = [&](int64_t v, int dm) -> Mat& {
    auto it = rhs.find(v);
    if (it == rhs.end()) it = rhs.emplace(v, Mat(dm, m)).first;
    return it->second;
  };
  std::vector<Mat> wsave(s.fac.size());
  size_t fi = 0;
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    if (l < L) {  // rhs of X_b^{(l)} = stacked rhs of the children's Z rows
      for (int bx = 0; bx < lv.nb; ++bx) {
        int n = lv.nfin[bx];
        if (n == 0) continue;
        Mat R(n, m);
        int o = 0;
        for (int ch = 0; ch < (1 << d); ++ch) {
          int c = (bx << d) | ch;
          int k = s.lev[l + 1].kfin[c];
          if (k == 0) continue;
          Mat& zc = getr(var(VZ, l + 1, c), k);
          for (int q = 0; q < k; ++q)
            for (int cc = 0; cc < m; ++cc) R.at(o + q, cc) = zc.at(q, cc);
          o += k;
        }
        rhs[var(VX, l, bx)] = R;
      }
    }
    for (; fi < s.fac.size() && s.fac[fi].level == l; ++fi) {
      Factor& F = s.fac[fi];
      int mm = F.LU.r;
      Mat rr(mm, m);
      int o = 0;
      for (size_t a = 0; a < F.PR.size(); ++a) {
        Mat& src = getr(F.PR[a], F.dPR[a]);
        for (int q = 0; q < F.dPR[a]; ++q)
          for (int c = 0; c < m; ++c) rr.at(o + q, c) = src.at(q, c);
        o += F.dPR[a];
      }
      Mat w = lu_solve(F.LU, F.perm, rr, -1);
      Mat up = mul(F.Cb, w);
      o = 0;
      for (size_t a = 0; a < F.Or.size(); ++a) {
        Mat& dst = getr(F.Or[a], F.dOr[a]);
        for (int q = 0; q < F.dOr[a]; ++q)
          for (int c = 0; c < m; ++c) dst.at(q, c) -= up.at(o + q, c);
        o += F.dOr[a];
      }
      wsave[fi] = w;
    }
  }
  // top solve for y^{(2)}
  {
    int Kt = s.top.r;
    Mat rt(Kt, m);
    int o = 0;
    for (size_t a = 0; a < s.top_vars.size(); ++a) {
      int k = s.top_dims[a];
      if (k) {
        Mat& src = getr(var(VZ, 2, s.top_vars[a]), k);
        for (int q = 0; q < k; ++q)
          for (int c = 0; c < m; ++c) rt.at(o + q, c) = src.at(q, c);
      }
      o += k;
    }
    Mat y2 = Kt ? lu_solve(s.top, s.top_perm, rt, -1) : Mat(0, m);
    o = 0;
    for (size_t a = 0; a < s.top_vars.size(); ++a) {
      int k = s.top_dims[a];
      Mat v(k, m);
      for (int q = 0; q < k; ++q)
        for (int c = 0; c < m; ++c) v.at(q, c) = y2.at(o + q, c);
      sol[var(Vy, 2, s.top_vars[a])] = v;
      o += k;
    }
  }
  (void)dims;
  (void)dimv;
  auto gets = [&](int64_t v, int dm) -> Mat& {
    auto it = sol.find(v);
    if (it == sol.end()) it = sol.emplace(v, Mat(dm, m)).first;
    return it->second;
  };
  // back substitution, levels 2..L, boxes in reverse elimination order
  size_t end = s.fac.size();
  for (int l = 2; l <= L; ++l) {
    Level& lv = s.lev[l];
    size_t beg = end;
    while (beg > 0 && s.fac[beg - 1].level == l) --beg;
    for (size_t q = end; q > beg; --q) {
      Factor& F = s.fac[q - 1];
      int C = F.W.c;
      Mat so(C, m);
      int o = 0;
      for (size_t a = 0; a < F.Oc.size(); ++a) {
        Mat& src = gets(F.Oc[a], F.dOc[a]);
        for (int t = 0; t < F.dOc[a]; ++t)
          for (int c = 0; c < m; ++c) so.at(o + t, c) = src.at(t, c);
        o += F.dOc[a];
      }
      Mat corr = mul(F.W, so);
      Mat v = wsave[q - 1];
      for (size_t t = 0; t < v.a.size(); ++t) v.a[t] -= corr.a[t];
      o = 0;
      for (size_t a = 0; a < F.PC.size(); ++a) {
        Mat part(F.dPC[a], m);
        for (int t = 0; t < F.dPC[a]; ++t)
          for (int c = 0; c < m; ++c) part.at(t, c) = v.at(o + t, c);
        sol[F.PC[a]] = part;
        o += F.dPC[a];
      }
    }
    end = beg;
    // y^{(l+1)} of the children from x^{(l)} (eq. particleAtNonLeafLevel)
    if (l < L) {
      for (int bx = 0; bx < lv.nb; ++bx) {
        if (lv.nfin[bx] == 0) continue;
        Mat& xv = gets(var(Vx, l, bx), lv.nfin[bx]);
        int o = 0;
        for (int ch = 0; ch < (1 << d); ++ch) {
          int c = (bx << d) | ch;
          int k = s.lev[l + 1].kfin[c];
          Mat yv(k, m);
          for (int t = 0; t < k; ++t)
            for (int cc = 0; cc < m; ++cc) yv.at(t, cc) = xv.at(o + t, cc);
          sol[var(Vy, l + 1, c)] = yv;
          o += k;
        }
      }
    }
  }
  for (int bx = 0; bx < lL.nb; ++bx) {
    const std::vector<int64_t>& t = lL.pts[bx];
    if (t.empty()) continue;
    Mat& xv = gets(var(Vx, L, bx), (int)t.size());
    for (size_t q = 0; q < t.size(); ++q)
      for (int c = 0; c < m; ++c) x[c * s.N + t[q]] = xv.at((int)q, c);
  }
  return true;
}

// NNCA-based H^2 product y = A~ x (Sec. 2.3, the operator table): the far field of every
// interaction-list pair (B, D) at every level through the nested operators, the near field of
// the leaf neighbours exactly.  Upward pass: multipoles q_B = V_B^* x_B at the leaf (P2M) and
// q_P = sum over children c of V^dagger*_c q_c above (M2M); M2L: l_B = sum over D in IL(B) of
// A_BD q_D; downward pass: l_c += U^dagger_c l_P (L2L), then y_B = U_B l_B (L2P) plus
// sum over X in N(B) of K_BX x_X (P2P).  x, y: N x nrhs column-major, original point order.
void h2_matvec(oracle_sys& s, const double* x, int nrhs, double* y) {
  int d = s.d, L = s.L;
  std::vector<std::vector<Mat>> q(L + 1), loc(L + 1);
  for (int l = L; l >= 2; --l) {
    Level& lv = s.lev[l];
    q[l].assign(lv.nb, Mat());
    loc[l].assign(lv.nb, Mat());
    for (int b = 0; b < lv.nb; ++b) {
      int k = lv.knn[b];
      loc[l][b] = Mat(k, nrhs);
      if (l == L) {
        const std::vector<int64_t>& t = lv.pts[b];
        Mat xb((int)t.size(), nrhs);
        for (size_t r = 0; r < t.size(); ++r)
          for (int c = 0; c < nrhs; ++c) xb.at((int)r, c) = x[c * s.N + t[r]];
        q[l][b] = k > 0 ? mul(lv.Vs[b], xb) : Mat(0, nrhs);
      } else {
        Level& dn = s.lev[l + 1];
        Mat acc(k, nrhs);
        for (int ch = 0; ch < (1 << d); ++ch) {
          int c = (b << d) | ch;
          if (k == 0 || dn.knn[c] == 0) continue;
          Mat t = mul(dn.Vds[c], q[l + 1][c]);
          for (size_t u = 0; u < t.a.size(); ++u) acc.a[u] += t.a[u];
        }
        q[l][b] = acc;
      }
    }
  }
  for (int l = 2; l <= L; ++l) {
    Level& lv = s.lev[l];
    for (int b = 0; b < lv.nb; ++b) {
      if (lv.knn[b] == 0) continue;
      for (size_t e = 0; e < lv.il[b].size(); ++e) {
        int D = lv.il[b][e];
        if (lv.knn[D] == 0) continue;
        Mat t = mul(lv.m2l[b][e], q[l][D]);
        for (size_t u = 0; u < t.a.size(); ++u) loc[l][b].a[u] += t.a[u];
      }
      if (l < L) {
        Level& dn = s.lev[l + 1];
        for (int ch = 0; ch < (1 << d); ++ch) {
          int c = (b << d) | ch;
          if (dn.knn[c] == 0) continue;
          Mat t = mul(dn.Ud[c], loc[l][b]);
          for (size_t u = 0; u < t.a.size(); ++u) loc[l + 1][c].a[u] += t.a[u];
        }
      }
    }
  }
  Level& lv = s.lev[L];
  for (int64_t q0 = 0; q0 < s.N * nrhs; ++q0) y[q0] = 0.0;
  for (int b = 0; b < lv.nb; ++b) {
    const std::vector<int64_t>& t = lv.pts[b];
    if (t.empty()) continue;
    Mat yb((int)t.size(), nrhs);
    if (lv.knn[b] > 0) yb = mul(lv.U[b], loc[L][b]);
    for (int X : lv.nbr[b]) {
      const std::vector<int64_t>& u = lv.pts[X];
      for (size_t r = 0; r < t.size(); ++r)
        for (size_t j = 0; j < u.size(); ++j) {
          double a = s.K(t[r], u[j]);
          for (int c = 0; c < nrhs; ++c) yb.at((int)r, c) += a * x[c * s.N + u[j]];
        }
    }
    for (size_t r = 0; r < t.size(); ++r)
      for (int c = 0; c < nrhs; ++c) y[c * s.N + t[r]] = yb.at((int)r, c);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// C API
// ------------------------------------------------------------------------------------------
extern "C" {

void oracle_kernel_block(const double* pts, int d, int kind, double scale, double shift,
                         const int64_t* rows, int64_t nr, const int64_t* cols, int64_t nc, double* out) {
  g_mode = 0;  // unit routines and the brute-force product take the default readings
  Kern K{pts, d, kind, scale, shift};
  for (int64_t i = 0; i < nr; ++i)
    for (int64_t j = 0; j < nc; ++j) out[i * nc + j] = K(rows[i], cols[j]);
}

void oracle_matvec_rows(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                        const int64_t* rows, int64_t nsel, const double* x, int64_t nrhs, double* y) {
  g_mode = 0;  // unit routines and the brute-force product take the default readings
  Kern K{pts, d, kind, scale, shift};
  std::vector<double> acc(nrhs);
  for (int64_t r = 0; r < nsel; ++r) {
    std::fill(acc.begin(), acc.end(), 0.0);
    for (int64_t j = 0; j < n; ++j) {
      double a = K(rows[r], j);
      for (int64_t c = 0; c < nrhs; ++c) acc[c] += a * x[c * n + j];
    }
    for (int64_t c = 0; c < nrhs; ++c) y[c * nsel + r] = acc[c];
  }
}

void oracle_matvec(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                   const double* x, int64_t nrhs, double* y) {
  std::vector<int64_t> rows(n);
  for (int64_t i = 0; i < n; ++i) rows[i] = i;
  oracle_matvec_rows(pts, n, d, kind, scale, shift, rows.data(), n, x, nrhs, y);
}

int oracle_dense_solve(int64_t n, const double* A, int64_t nrhs, const double* B, double* X) {
  Mat M((int)n, (int)n);
  for (int64_t q = 0; q < n * n; ++q) M.a[q] = A[q];
  std::vector<int> perm;
  int st = lu_factor(M, perm);
  if (st) return st;
  Mat Bm((int)n, (int)nrhs);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < nrhs; ++c) Bm.at((int)i, (int)c) = B[c * n + i];
  Mat Xm = lu_solve(M, perm, Bm, -1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < nrhs; ++c) X[c * n + i] = Xm.at((int)i, (int)c);
  return 0;
}

int oracle_aca(const double* M, int m, int n, double tol, int* I, int* J, double* U, double* V) {
  g_mode = 0;  // unit routines and the brute-force product take the default readings
  auto f = [&](int i, int j) { return M[(size_t)i * n + j]; };
  AcaOut a = aca_pp(m, n, f, tol);
  int k = (int)a.I.size();
  for (int q = 0; q < k; ++q) {
    I[q] = a.I[q];
    J[q] = a.J[q];
    for (int i = 0; i < m; ++i) U[(size_t)q * m + i] = a.U[q][i];
    for (int j = 0; j < n; ++j) V[(size_t)q * n + j] = a.V[q][j];
  }
  return k;
}

int oracle_cpqr(const double* M, int m, int n, double tol, int qcols, double* Q, int* perm, double* R) {
  g_mode = 0;  // unit routines and the brute-force product take the default readings
  Mat A(m, n);
  for (size_t q = 0; q < (size_t)m * n; ++q) A.a[q] = M[q];
  Cpqr f = cpqr(A, tol);
  if (Q && qcols > 0) {
    Mat Qm = cpqr_q(f, qcols);
    for (size_t q = 0; q < Qm.a.size(); ++q) Q[q] = Qm.a[q];
  }
  if (perm) for (int j = 0; j < n; ++j) perm[j] = f.perm[j];
  if (R) for (size_t q = 0; q < f.R.a.size(); ++q) R[q] = f.R.a[q];
  return f.rank;
}

oracle_sys* oracle_create(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                          double tol, int leaf_size, int depth) {
  return oracle_create_mode(pts, n, d, kind, scale, shift, tol, leaf_size, depth, 0);
}

oracle_sys* oracle_create_mode(const double* pts, int64_t n, int d, int kind, double scale, double shift,
                               double tol, int leaf_size, int depth, int mode) {
  g_mode = mode;
  oracle_sys* s = new oracle_sys();
  s->mode = mode;
  for (int q = 0; q < 5; ++q) g_flops[q] = 0;
  s->N = n;
  s->d = d;
  s->tol = tol;
  s->leaf = leaf_size;
  s->pts.assign(pts, pts + n * d);
  s->K = Kern{s->pts.data(), d, kind, scale, shift};
  if (depth > 0) s->L = depth;
  else {
    // depth rule: L = max(2, ceil(log_{2^d}(N / n_max)))
    int L = 0;
    double cap = (double)leaf_size;
    while ((double)n > cap) { cap *= (double)(1 << d); ++L; }
    s->L = std::max(2, L);
  }
  if (d < 2 || d > 3 || n <= 0) { s->err = "bad arguments"; return s; }
  build_tree(*s);
  build_lists(*s);
  if (!build_nnca(*s)) return s;
  build_order(*s);
  assemble(*s);
  return s;
}

const char* oracle_error(oracle_sys* s) { return s->err.c_str(); }
int oracle_depth(oracle_sys* s) { return s->L; }

int oracle_box_count(oracle_sys* s, int level, int* nb) {
  if (level < 0 || level > s->L) return -1;
  Level& lv = s->lev[level];
  for (int b = 0; b < lv.nb; ++b) nb[b] = (int)lv.pts[b].size();
  return lv.nb;
}
int oracle_nnca_ranks(oracle_sys* s, int level, int* k) {
  if (level < 2 || level > s->L) return -1;
  Level& lv = s->lev[level];
  for (int b = 0; b < lv.nb; ++b) k[b] = lv.knn[b];
  return lv.nb;
}
int oracle_final_ranks(oracle_sys* s, int level, int* k) {
  if (level < 2 || level > s->L || !s->factored) return -1;
  Level& lv = s->lev[level];
  for (int b = 0; b < lv.nb; ++b) k[b] = lv.kfin[b];
  return lv.nb;
}
int oracle_xsize(oracle_sys* s, int level, int* n) {
  if (level < 2 || level > s->L || !s->factored) return -1;
  Level& lv = s->lev[level];
  for (int b = 0; b < lv.nb; ++b) n[b] = lv.nfin[b];
  return lv.nb;
}
int oracle_pivots(oracle_sys* s, int level, int box, int64_t* t_i, int64_t* s_i) {
  if (level < 2 || level > s->L) return -1;
  Level& lv = s->lev[level];
  int k = lv.knn[box];
  for (int q = 0; q < k; ++q) {
    if (t_i) t_i[q] = lv.ti[box][q];
    if (s_i) s_i[q] = lv.si[box][q];
  }
  return k;
}
int oracle_nnca_U(oracle_sys* s, int level, int box, double* out) {
  // U_B = A[T_B, s^{B,i}] (A[t^{B,i}, s^{B,i}])^{-1}: L2P at the leaf, stacked children's L2L above
  if (level < 2 || level > s->L) return -1;
  Level& lv = s->lev[level];
  int k = lv.knn[box];
  if (level == s->L) {
    const Mat& U = lv.U[box];
    for (size_t q = 0; q < U.a.size(); ++q) out[q] = U.a[q];
    return U.r;
  }
  Level& dn = s->lev[level + 1];
  int o = 0;
  for (int ch = 0; ch < (1 << s->d); ++ch) {
    const Mat& U = dn.Ud[(box << s->d) | ch];
    for (int i = 0; i < U.r; ++i)
      for (int j = 0; j < k; ++j) out[(size_t)(o + i) * k + j] = U.at(i, j);
    o += U.r;
  }
  return o;
}
int oracle_perm(oracle_sys* s, int64_t* perm) {
  int64_t o = 0;
  Level& lv = s->lev[s->L];
  for (int b = 0; b < lv.nb; ++b)
    for (int64_t p : lv.pts[b]) perm[o++] = p;
  return 0;
}
int oracle_elim_order(oracle_sys* s, int level, int* order) {
  if (level < 2 || level > s->L) return -1;
  Level& lv = s->lev[level];
  for (int b = 0; b < lv.nb; ++b) order[b] = lv.order[b];
  return lv.nb;
}

int oracle_dense_extended(oracle_sys* s, int64_t* dim, double* out, int64_t* xcols) {
  // row order: X^{(L)}, then per level L..2: Y, Z; column order x^{(L)}, then z, y per level
  if (s->factored) return -1;
  Store& S = s->S;
  std::vector<int64_t> rv, cv;
  int L = s->L;
  for (int b = 0; b < s->lev[L].nb; ++b) { rv.push_back(var(VX, L, b)); cv.push_back(var(Vx, L, b)); }
  for (int l = L; l >= 2; --l)
    for (int b = 0; b < s->lev[l].nb; ++b) {
      rv.push_back(var(VY, l, b)); rv.push_back(var(VZ, l, b));
      cv.push_back(var(Vz, l, b)); cv.push_back(var(Vy, l, b));
    }
  std::map<int64_t, int64_t> ro, co;
  int64_t nr = 0, nc = 0;
  for (int64_t v : rv) { ro[v] = nr; nr += S.d(v); }
  for (int64_t v : cv) { co[v] = nc; nc += S.d(v); }
  if (nr != nc) return -2;
  *dim = nr;
  if (!out) return 0;
  std::fill(out, out + nr * nr, 0.0);
  for (auto& kv : S.blk) {
    int64_t r0 = ro[kv.first.first], c0 = co[kv.first.second];
    const Mat& B = kv.second;
    for (int i = 0; i < B.r; ++i)
      for (int j = 0; j < B.c; ++j) out[(r0 + i) * nr + c0 + j] = B.at(i, j);
  }
  if (xcols) {
    for (int b = 0; b < s->lev[L].nb; ++b) {
      int64_t c0 = co[var(Vx, L, b)];
      const std::vector<int64_t>& t = s->lev[L].pts[b];
      for (size_t q = 0; q < t.size(); ++q) xcols[t[q]] = c0 + (int64_t)q;
    }
  }
  return 0;
}

int oracle_factor(oracle_sys* s) {
  g_mode = s->mode;
  if (!s->err.empty()) return 4;
  if (s->factored) return 4;
  for (int q = 0; q < 5; ++q) g_flops[q] = 0;
  bool ok = factor(*s);
  for (int q = 0; q < 5; ++q) s->flops[q] = g_flops[q];
  if (!ok) return 3;
  s->factored = true;
  return 0;
}

int oracle_solve(oracle_sys* s, const double* b, int64_t nrhs, double* x) {
  g_mode = s->mode;
  if (!s->factored) return 4;
  return solve(*s, b, nrhs, x) ? 0 : 3;
}

int64_t oracle_trace(oracle_sys* s, int* out, int64_t cap) {
  int64_t n = (int64_t)s->trace.size();
  if (out)
    for (int64_t q = 0; q < n && q < cap; ++q)
      for (int t = 0; t < 4; ++t) out[q * 4 + t] = s->trace[q][t];
  return n;
}
int64_t oracle_trace_ranks(oracle_sys* s, int* ranks, double* ratio, int64_t cap) {
  int64_t n = (int64_t)s->trace_ranks.size();
  for (int64_t q = 0; q < n && q < cap; ++q) {
    for (int t = 0; t < 6; ++t) ranks[q * 6 + t] = s->trace_ranks[q][t];
    for (int t = 0; t < 8; ++t) ratio[q * 8 + t] = s->trace_ratio[q][t];
  }
  return n;
}
int oracle_h2_matvec(oracle_sys* s, const double* x, int64_t nrhs, double* y) {
  g_mode = s->mode;
  if (!s->err.empty() || s->lev.empty() || s->lev[s->L].U.empty()) return 4;
  h2_matvec(*s, x, (int)nrhs, y);
  return 0;
}
int64_t oracle_far_fill_count(oracle_sys* s) { return s->far_fill; }
int64_t oracle_rhs_violations(oracle_sys* s) { return s->rhs_violations; }
int oracle_row_set(oracle_sys* s, int level, int box, int64_t* out) {
  // T_B: the box's points at the leaf, the children's incoming pivots (child order) above
  if (level < 2 || level > s->L) return -1;
  std::vector<int64_t> T;
  if (level == s->L) T = s->lev[level].pts[box];
  else
    for (int ch = 0; ch < (1 << s->d); ++ch) {
      const std::vector<int64_t>& t = s->lev[level + 1].ti[(box << s->d) | ch];
      T.insert(T.end(), t.begin(), t.end());
    }
  if (out) for (size_t q = 0; q < T.size(); ++q) out[q] = T[q];
  return (int)T.size();
}
void oracle_kexp(const double* x, int64_t n, double* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = kexp(x[q]);
}
int oracle_lists(oracle_sys* s, int level, int box, int* nbr, int* il) {
  if (level < 0 || level > s->L) return -1;
  Level& lv = s->lev[level];
  for (size_t q = 0; q < lv.nbr[box].size(); ++q) nbr[q] = lv.nbr[box][q];
  for (size_t q = 0; q < lv.il[box].size(); ++q) il[q] = lv.il[box][q];
  return (int)lv.nbr[box].size() * 1000 + (int)lv.il[box].size();
}
void oracle_margins(oracle_sys* s, double* a, double* b, double* c) {
  *a = s->cpqr_margin;
  *b = s->aca_stop;
  *c = s->aca_gap;
}
void oracle_flops(oracle_sys* s, double* f5) {
  for (int q = 0; q < 5; ++q) f5[q] = s->flops[q];
}
void oracle_destroy(oracle_sys* s) { delete s; }

}  // extern "C"
