// Internal structures of the MI355X AIFMM library (host planner + device block store).
//
// Terminology follows the paper (arXiv 2301.12704): boxes of a uniform 2^d tree, neighbours
// N(b) and interaction list IL(b) (Sec. 2.2), particles x, locals z and multipoles y of every
// box at levels 2..L (Sec. 3.1), rows X / Y / Z of the extended system (equations X, Y, Z).
//
// Device block store of one level l (the "live" extended system while level l is being
// eliminated):
//   near slot  (p,q), dist_inf(p,q) <= 1 : the live block rows(p) x cols(q), where
//              rows(p) = X_p before p is eliminated and Z_p after; cols(q) = x_q / y_q.
//   fill slot  (p,q), dist_inf(p,q) == 2 : the accumulated P2P / P2L / M2P fill-in.
//   M2L slot   (p,q), q in IL(p)         : A_pq = block (Z_p, y_q).
//   per box    U_b (X_b, z_b), V_b (transpose of (Y_b, x_b)), L2L (Z_b, z_parent) and
//              M2M (transpose of (Y_parent, y_b)).
// Every slot (p,q) is row-major with capacity n_p x n_q and leading dimension n_q; a box's
// rank never exceeds n_b, so every live shape fits.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/aifmm.h"

namespace aifmm {

struct Error {
  aifmm_status st;
  std::string msg;
};

#define AIFMM_HIP(x)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw ::aifmm::Error{AIFMM_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// While a factorization runs on this thread, buffers released are only collected here and
// freed when it ends: hipFree waits for the whole device, which would stall the other systems'
// streams in a batched factorization.
inline thread_local std::vector<void*>* g_defer_free = nullptr;

// Device buffer owned by the system (hipMalloc / hipFree).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) {
      if (g_defer_free) g_defer_free->push_back((void*)p);
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    if (hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error{AIFMM_ERR_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void zero(hipStream_t s) { if (p) AIFMM_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) AIFMM_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s, size_t count = (size_t)-1) const {
    if (count == (size_t)-1) count = n;
    std::vector<T> h(count);
    if (count) AIFMM_HIP(hipMemcpyAsync(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    AIFMM_HIP(hipStreamSynchronize(s));
    return h;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Host N x nr column-major array with leading dimension ld (>= N) to or from a compact device
// array (leading dimension N).  Only the N rows of each column are touched on the host side, so
// the caller's padding rows and anything past the last column stay as they are.
inline void h2d_cols(double* dst, const double* src, int64_t ld, int64_t N, int64_t nr, hipStream_t st) {
  if (ld == N)
    AIFMM_HIP(hipMemcpyAsync(dst, src, sizeof(double) * N * nr, hipMemcpyHostToDevice, st));
  else
    AIFMM_HIP(hipMemcpy2DAsync(dst, sizeof(double) * N, src, sizeof(double) * ld, sizeof(double) * N, nr,
                               hipMemcpyHostToDevice, st));
}
inline void d2h_cols(double* dst, int64_t ld, const double* src, int64_t N, int64_t nr, hipStream_t st) {
  if (ld == N)
    AIFMM_HIP(hipMemcpyAsync(dst, src, sizeof(double) * N * nr, hipMemcpyDeviceToHost, st));
  else
    AIFMM_HIP(hipMemcpy2DAsync(dst, sizeof(double) * ld, src, sizeof(double) * N, sizeof(double) * N, nr,
                               hipMemcpyDeviceToHost, st));
}

struct KernelDesc {
  int kind;      // 0: exp(-r/scale), 1: 1/sqrt(r^2 + scale^2)
  double scale;  // > 0
  double shift;  // added when i == j
};

// One compression of the static schedule (Algorithm "Efficient Elimination", the loops over
// vP2P / vP2L before eliminating box i).
struct PairOp {
  int i;        // box about to be eliminated
  int kind;     // 0 = P2P pair (i, j), 1 = P2L pair (r eliminated, i)
  int partner;  // j (P2P) or r (P2L)
};

// Host plan of one level: lists, elimination order, colours, compression rounds and the
// coupled-block tables of every box's elimination.
struct LevelPlan {
  int l = 0, nb = 0;
  std::vector<int> coord;                 // nb * 3
  std::vector<int> nbr_off, nbr;          // N(b), self included, Morton order
  std::vector<int> il_off, il;            // IL(b), Morton order
  std::vector<int> il_tr;                 // for entry e of IL(b)=d: entry index of b in IL(d)
  std::vector<int> p2_off, p2;            // distance-2 partners, Morton order
  std::vector<int> p2_tr;                 // transpose index inside the p2 CSR
  std::vector<int> order, pos;            // elimination order and position of every box
  std::vector<int> col_off;               // colour batches: order[col_off[c] .. col_off[c+1])
  std::vector<std::vector<std::vector<PairOp>>> rounds;  // [colour][round] -> compressions
  // coupled groups of each box elimination: G = |N(b)| entries; entries 0..G-2 are the
  // neighbours other than b (Morton order), entry G-1 is b itself (rows Z_b / column y_b).
  std::vector<int> grp_off;               // nb+1 (offsets into grp_box / grp_elim)
  std::vector<int> grp_box, grp_elim;     // elim: 1 if eliminated before b
};

int cheb(const int* a, const int* b, int d);

// Build the host plan of level l (lists from Sec. 2.2, colour order, compression schedule).
void plan_level(LevelPlan& P, int d, int l);

// Per-level device data.
struct LevelDev {
  int l = 0, nb = 0;
  std::vector<int> n;          // x sizes n_b (host copy)
  std::vector<int> knn;        // NNCA ranks
  std::vector<int> kfin;       // ranks at elimination (host copy after factor)
  std::vector<int64_t> xoff;   // prefix of n (rhs / solution offsets of x and X)
  std::vector<int64_t> koff;   // prefix of final k (rhs / solution offsets of y, z, Y, Z)
  DBuf<int> d_n, d_k, d_kn;    // n_b, current rank, next rank
  // plan tables on device
  DBuf<int> d_nbr_off, d_nbr, d_il_off, d_il, d_il_tr, d_p2_off, d_p2, d_grp_off, d_grp_box, d_grp_elim;
  // NNCA outputs (compact, valid for the whole factorization)
  std::vector<int> T_off;      // row set sizes prefix: ACA rows of box b
  DBuf<int> d_T;               // row sets (tree positions), |T_b| per box
  DBuf<int> d_T_off;
  DBuf<int> d_piv_r, d_piv_c;  // pivot rows / cols (tree positions), capacity |T_b| per box
  DBuf<double> d_Unn;          // U_B = A[T_B, s_i] C^{-1}, |T_B| x k_B row-major
  std::vector<int64_t> Unn_off;
  DBuf<int64_t> d_Unn_off;
  DBuf<double> d_m2l_nn;       // A_BD, k_B x k_D, one per IL entry
  std::vector<int64_t> m2l_nn_off;
  DBuf<int64_t> d_m2l_nn_off;
  DBuf<int> d_knn;             // NNCA ranks on the device (d_k changes during the factorization)
  std::vector<int64_t> koff_nn;  // prefix of the NNCA ranks (rows of the H^2 product's q and l)
  DBuf<int64_t> d_koff_nn;
  // live block store (allocated when the level is eliminated)
  DBuf<double> slab;
  DBuf<int64_t> d_near_slot, d_p2_slot, d_il_slot;   // per CSR entry
  DBuf<int64_t> d_U_off, d_V_off, d_l2l_off, d_m2m_off;  // per box
  DBuf<int> d_kP;              // NNCA rank of the parent (columns of L2L / M2M), 0 at level 2
  DBuf<int64_t> d_tslot;       // per box: Gmax x Gmax target offsets (Schur scatter)
  DBuf<int> d_grc;             // per box 2 x 28: row / column offsets of the coupled groups
  // factor store (kept for the solve)
  DBuf<double> fslab;
  DBuf<int64_t> d_fLU, d_fPx, d_fC, d_fW;  // per box offsets into fslab
  DBuf<int> d_order;           // elimination order on the device
  DBuf<int> d_fpiv;            // ipiv, capacity 2 n_b per box
  DBuf<int64_t> d_fpiv_off;
  std::vector<int64_t> fLU, fPx, fC, fW;   // host copies of the offsets
  std::vector<int> Rcap, Ccap;
  int nmax = 0, Rmax = 0, Cmax = 0, Gmax = 0;
};

// decision log of one compression (static schedule entry plus the ranks it decided)
struct TraceRec {
  int level, i, kind, partner;
  int r[6];
  double ratio[8];
};

// One tile of at most 64 rows of a solve-sweep product Y (rows x nr) = A (rows x K, row-major
// lda) B (K x nr, row-major); how Y is written depends on the kernel.  Offsets are in elements
// of the factor store (a) and in rows of the right-hand-side buffers (b, y, y0, z).
struct STask {
  int64_t a, b, y, y0, z;
  int lda, K, rows, sel;
};

// Static task lists of the solve sweeps of one level (per colour offsets) and buffers.
struct SolveLevel {
  DBuf<STask> fw, fu, bw, gs;
  std::vector<int> fw_off, fu_off, bw_off, gs_off;
  std::vector<int64_t> woff;  // rows of w = Piv^{-1} rhs per box
  int64_t grows = 0;          // rows of the largest gathered colour
};
// A captured solve (graph and its executable), released with the cache.
struct SolveGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int nr = 0, cap = 0;
  const double* in = nullptr;
  const double* out = nullptr;
  SolveGraph() = default;
  SolveGraph(const SolveGraph&) = delete;
  SolveGraph& operator=(const SolveGraph&) = delete;
  SolveGraph(SolveGraph&& o) noexcept { *this = std::move(o); }
  SolveGraph& operator=(SolveGraph&& o) noexcept {
    if (this != &o) {
      reset();
      graph = o.graph; exec = o.exec; nr = o.nr; cap = o.cap; in = o.in; out = o.out;
      o.graph = nullptr; o.exec = nullptr;
    }
    return *this;
  }
  ~SolveGraph() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    nr = 0;
  }
};

struct SolveCache {
  bool built = false;
  SolveGraph graph;
  int nr_cap = 0;
  // blocked triangular solves of the top system: row permutation of its LU, and the update
  // tiles of every 64-row block step (forward below the block, backward above it)
  DBuf<int> top_perm;
  DBuf<STask> top_fw, top_bw;
  std::vector<int> top_fw_off, top_bw_off;
  std::vector<SolveLevel> lev;
  std::vector<DBuf<double>> R, X, W;
  DBuf<double> G;
};

// Work vectors of the H^2 product (multipoles q and locals l of every level), grown to the
// largest right-hand-side count seen.
struct H2Cache {
  int nr_cap = 0;
  std::vector<DBuf<double>> q, loc;
};

// FGMRES workspace kept across calls (grown to the largest right-hand-side count seen), so a
// served system allocates nothing per request once warm.
struct GmresCache {
  int nr_cap = 0, m_cap = 0;
  int64_t ld_cap = 0;
  DBuf<double> bin, bt, xt, r, w, part, dalpha, xo;
  DBuf<double> rx, cx;  // exact residual and correction of the refinement with an H^2 operator
  std::vector<DBuf<double>> V, Z;
};

// Figures of one level's factorization (device times are HIP-event times of the launches).
struct LevelStats {
  double factor_s = 0;                    // wall time of the level
  double schur_flops = 0, schur_bytes = 0;  // Schur update: 2 R n C flops, 8 (R n + n C + 2 R C) bytes per box
  double trsm_flops = 0;                  // pivot-block solve, algorithmic 2 m^2 C per box
  double trsm_flops_impl = 0;             // as executed, 2 m^2 (C + n) (W also holds Piv^{-1}[:, x_b])
  double lu_flops = 0;                    // (2/3) m^3 per box
  double schur_s = 0, trsm_s = 0, compress_s = 0;
  double compress_flops = 0;              // pivoted QRs, Q formations and coefficient products as executed
  double compressions = 0, rounds = 0;
  double crit_steps = 0;                  // sum over rounds of the longest pivot-step chain of the round
  double pivot_steps = 0;                 // all pivot steps of the level's pivoted QRs
  double boxes = 0;
};

struct Stats {
  std::vector<LevelStats> lvl;            // by level (2..L used)
  double build_s = 0, factor_s = 0, solve_s = 0;
  double schur_flops = 0, schur_bytes = 0, trsm_flops = 0, lu_flops = 0;
  double schur_kernel_s = 0, compress_kernel_s = 0;   // event-timed device time of the last factor
  double schur_launches = 0, compress_launches = 0;
  double trsm_kernel_s = 0, trsm_launches = 0;
  double gmres_s = 0, gmres_iters = 0;
  double solve_bytes = 0;                 // factor-store bytes one solve's products read (any nrhs)
};

}  // namespace aifmm

struct aifmm_system {
  int d = 2, L = 2, leaf = 64, device = 0;
  int64_t N = 0;
  aifmm::KernelDesc K{};
  double tol = 1e-10;
  int prec = 0;                   // AIFMM_FP64 or AIFMM_FP32 (arithmetic of Schur update and compression)
  hipStream_t stream = nullptr;
  bool factored = false;
  std::string err;
  std::mutex use;                  // held by every call that runs work on the system
  // tree
  aifmm::DBuf<double> d_pts;      // points in tree order, N x d
  aifmm::DBuf<int64_t> d_perm;    // tree position -> original index
  std::vector<int> leaf_off;      // nb_L + 1, point offsets of leaves in tree order
  std::vector<aifmm::LevelPlan> plan;   // by level, 0..L
  std::vector<aifmm::LevelDev> lev;     // by level, 0..L (2..L used)
  // top-level multipole system
  int Ktop = 0;
  aifmm::DBuf<double> d_top;
  aifmm::DBuf<int> d_top_piv;
  // workspaces
  aifmm::DBuf<double> ws;         // compression / transform / elimination scratch
  aifmm::DBuf<int> d_flag;        // [0] singular flag, [1] box, [2] level, [3] capacity flag
  aifmm::DBuf<int> d_rounds;      // scratch upload area for round lists
  aifmm::Stats stats;
  aifmm::SolveCache sc;           // solve task lists and buffers (rebuilt after every factor)
  aifmm::GmresCache gc;           // FGMRES vectors
  std::vector<aifmm::TraceRec> trace;
  size_t device_bytes = 0;
  // the H^2 operator: NNCA of the same points at the matvec tolerance (absent: this system's own
  // NNCA at tol is the operator)
  std::unique_ptr<aifmm_system> op;
  double matvec_tol = 0.0;
  aifmm::H2Cache hc;
};

namespace aifmm {
template <class T>
inline size_t buf_bytes(const DBuf<T>& b) { return b.p ? b.n * sizeof(T) : 0; }
template <class T>
inline size_t buf_bytes(const std::vector<DBuf<T>>& v) {
  size_t t = 0;
  for (auto& b : v) t += buf_bytes(b);
  return t;
}
// Device bytes a system holds in the workspaces that grow with the number of right-hand sides
// (solve buffers, FGMRES vectors, H^2 work vectors, and those of its operator system); they
// are kept between calls, so a served system keeps them while it is resident.
inline size_t rhs_workspace_bytes(const aifmm_system& s) {
  size_t t = buf_bytes(s.sc.R) + buf_bytes(s.sc.X) + buf_bytes(s.sc.W) + buf_bytes(s.sc.G);
  const GmresCache& g = s.gc;
  t += buf_bytes(g.bin) + buf_bytes(g.bt) + buf_bytes(g.xt) + buf_bytes(g.r) + buf_bytes(g.w) + buf_bytes(g.part) +
       buf_bytes(g.dalpha) + buf_bytes(g.xo) + buf_bytes(g.rx) + buf_bytes(g.cx) + buf_bytes(g.V) + buf_bytes(g.Z);
  t += buf_bytes(s.hc.q) + buf_bytes(s.hc.loc);
  if (s.op) t += rhs_workspace_bytes(*s.op);
  return t;
}
// build.hip
void build_system(aifmm_system& s, const double* pts_host_or_dev, bool on_device);
// factor.hip
void factor_system(aifmm_system& s);
// several systems of one device, precision and stream, in lockstep (k_factor.hip)
void factor_systems(const std::vector<aifmm_system*>& S);
// solve.hip
void solve_system(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx,
                  bool b_dev, bool x_dev);
void solve_tree(aifmm_system& s, const double* rhs, int nr, double* x);
void prepare_solve(aifmm_system& s);
size_t noalloc_max_bytes();
size_t noalloc_need_bytes(aifmm_system& s, int nr);
void solve_system_noalloc(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx);
// k_gmres.hip
void matvec_tree(aifmm_system& s, const double* x, int nr, double* y);
void h2_matvec_tree(aifmm_system& s, const double* x, int nr, double* y, hipStream_t st);
void h2_matvec_system(aifmm_system& s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy, bool x_dev,
                      bool y_dev);
void gmres_op_system(aifmm_system* op, aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double rtol,
                     int restart, int maxit, double* x, int64_t ldx, int32_t* iters, double* relres, bool b_dev,
                     bool x_dev);
void matvec_system(aifmm_system& s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy, bool x_dev,
                   bool y_dev);
void gmres_system(aifmm_system& s, const double* b, int64_t nrhs, int64_t ldb, double rtol, int restart, int maxit,
                  double* x, int64_t ldx, int32_t* iters, double* relres, bool b_dev, bool x_dev);
}  // namespace aifmm
