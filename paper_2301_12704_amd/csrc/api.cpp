// C ABI of the library (declarations and contracts in include/aifmm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "system.hpp"

namespace {
thread_local std::string g_err;

aifmm_status fail(aifmm_system* s, aifmm_status st, const std::string& msg) {
  g_err = msg;
  if (s) s->err = msg;
  return st;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

template <class F>
aifmm_status guarded(aifmm_system* s, F&& f) {
  try {
    f();
    return AIFMM_OK;
  } catch (const aifmm::Error& e) {
    return fail(s, e.st, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(s, AIFMM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(s, AIFMM_ERR_DEVICE, "unexpected failure");
  }
}
}  // namespace

extern "C" {

aifmm_status aifmm_options_default(aifmm_options* opt) {
  if (!opt) return fail(nullptr, AIFMM_ERR_ARG, "opt is NULL");
  opt->dim = 2;
  opt->leaf_size = 64;
  opt->depth = 0;
  opt->device = 0;
  opt->stream = nullptr;
  opt->prec = AIFMM_FP64;
  opt->matvec_tol = 0.0;
  return AIFMM_OK;
}

aifmm_status aifmm_build(const double* points, int64_t n, aifmm_kernel kernel, double tol, const aifmm_options* opt,
                         aifmm_system** out) {
  if (!out) return fail(nullptr, AIFMM_ERR_ARG, "out is NULL");
  *out = nullptr;
  aifmm_options o;
  aifmm_options_default(&o);
  if (opt) o = *opt;
  if (!points || n <= 0) return fail(nullptr, AIFMM_ERR_ARG, "points is NULL or n <= 0");
  if (o.dim != 2 && o.dim != 3) return fail(nullptr, AIFMM_ERR_ARG, "dim must be 2 or 3");
  if (o.leaf_size <= 0 || o.depth < 0 || o.depth > (o.dim == 2 ? 10 : 7))
    return fail(nullptr, AIFMM_ERR_ARG, "bad leaf_size or depth");
  if (kernel.kind != AIFMM_K_EXP && kernel.kind != AIFMM_K_INVMQ) return fail(nullptr, AIFMM_ERR_ARG, "bad kernel kind");
  if (o.prec != AIFMM_FP64 && o.prec != AIFMM_FP32) return fail(nullptr, AIFMM_ERR_ARG, "bad precision");
  if (!(kernel.scale > 0.0) || !std::isfinite(kernel.shift)) return fail(nullptr, AIFMM_ERR_ARG, "bad kernel scale/shift");
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(nullptr, AIFMM_ERR_ARG, "tol must be in (0, 1)");
  if (!(o.matvec_tol >= 0.0) || !(o.matvec_tol < 1.0)) return fail(nullptr, AIFMM_ERR_ARG, "matvec_tol must be in [0, 1)");
  if (n > (int64_t)1 << 30) return fail(nullptr, AIFMM_ERR_ARG, "n too large");
  aifmm_system* s = new (std::nothrow) aifmm_system();
  if (!s) return fail(nullptr, AIFMM_ERR_NOMEM, "host allocation failed");
  s->d = o.dim;
  s->N = n;
  s->leaf = o.leaf_size;
  s->device = o.device;
  s->stream = (hipStream_t)o.stream;
  s->tol = tol;
  s->prec = o.prec;
  s->K = aifmm::KernelDesc{(int)kernel.kind, kernel.scale, kernel.shift};
  if (o.depth > 0) {
    s->L = o.depth;
  } else {
    int L = 0;
    double cap = (double)o.leaf_size;
    while ((double)n > cap) { cap *= (double)(1 << o.dim); ++L; }
    s->L = L < 2 ? 2 : L;
  }
  if (s->L > (o.dim == 2 ? 10 : 7)) { delete s; return fail(nullptr, AIFMM_ERR_ARG, "tree too deep"); }
  aifmm_status st = guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    bool dev = is_device_ptr(points);
    aifmm::build_system(*s, points, dev);
    if (o.matvec_tol > 0.0 && o.matvec_tol != tol) {
      // the H^2 operator: the same tree with its own NNCA at the matvec tolerance
      std::unique_ptr<aifmm_system> op(new aifmm_system());
      op->d = s->d;
      op->N = s->N;
      op->leaf = s->leaf;
      op->L = s->L;
      op->device = s->device;
      op->stream = s->stream;
      op->tol = o.matvec_tol;
      op->prec = AIFMM_FP64;
      op->K = s->K;
      aifmm::build_system(*op, points, dev);
      s->stats.build_s += op->stats.build_s;
      s->op = std::move(op);
    }
    s->matvec_tol = o.matvec_tol > 0.0 ? o.matvec_tol : tol;
  });
  if (st != AIFMM_OK) {
    g_err = s->err;
    delete s;
    return st;
  }
  *out = s;
  return AIFMM_OK;
}

aifmm_status aifmm_factor(aifmm_system* s) {
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "system is NULL");
  std::lock_guard<std::mutex> lk(s->use);
  if (s->factored) return fail(s, AIFMM_ERR_STATE, "already factored");
  aifmm_status st = guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    aifmm::factor_system(*s);
    aifmm::prepare_solve(*s);
  });
  if (st == AIFMM_OK) s->factored = true;
  return st;
}

// Independent systems factored concurrently: nstreams worker threads, each with a stream of
// its own, take the systems in order; each system runs on its worker's stream and gets its
// previous stream back.  Returns the first failing status (every system is still attempted;
// aifmm_last_error of a system tells its own error).
aifmm_status aifmm_factor_batch(aifmm_system* const* systems, int32_t n, int32_t group) {
  if (!systems || n <= 0 || group <= 0) return fail(nullptr, AIFMM_ERR_ARG, "bad systems / n / group");
  for (int i = 0; i < n; ++i) {
    if (!systems[i]) return fail(nullptr, AIFMM_ERR_ARG, "a system is NULL");
    if (systems[i]->factored) return fail(systems[i], AIFMM_ERR_STATE, "already factored");
    for (int j = 0; j < i; ++j)
      if (systems[j] == systems[i]) return fail(nullptr, AIFMM_ERR_ARG, "a system is listed twice");
  }
  // systems of one device and precision, in the given order, in groups of up to `group`
  std::vector<std::vector<aifmm_system*>> groups;
  {
    std::vector<bool> taken(n, false);
    for (int i = 0; i < n; ++i) {
      if (taken[i]) continue;
      std::vector<aifmm_system*> g;
      for (int j = i; j < n && (int)g.size() < group; ++j)
        if (!taken[j] && systems[j]->device == systems[i]->device && systems[j]->prec == systems[i]->prec) {
          g.push_back(systems[j]);
          taken[j] = true;
        }
      groups.push_back(std::move(g));
    }
  }
  aifmm_status first = AIFMM_OK;
  for (auto& g : groups) {
    // every system of the group is locked (in address order) and runs on the first one's stream
    std::vector<aifmm_system*> order(g);
    std::sort(order.begin(), order.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (aifmm_system* s : order) locks.emplace_back(s->use);
    std::vector<hipStream_t> old;
    for (aifmm_system* s : g) old.push_back(s->stream);
    for (aifmm_system* s : g) s->stream = g[0]->stream;
    aifmm_status st = guarded(g[0], [&] {
      AIFMM_HIP(hipSetDevice(g[0]->device));
      aifmm::factor_systems(g);
    });
    for (size_t q = 0; q < g.size(); ++q) g[q]->stream = old[q];
    for (aifmm_system* s : g) {
      if (st != AIFMM_OK) {
        if (s != g[0]) fail(s, st, g[0]->err);
        continue;
      }
      aifmm_status sp = guarded(s, [&] {
        AIFMM_HIP(hipSetDevice(s->device));
        aifmm::prepare_solve(*s);
      });
      if (sp == AIFMM_OK) s->factored = true;
      else if (first == AIFMM_OK) first = sp;
    }
    if (st != AIFMM_OK && first == AIFMM_OK) first = st;
  }
  return first;
}

aifmm_status aifmm_solve(aifmm_system* s, const double* b, int64_t nrhs, int64_t ldb, double* x, int64_t ldx) {
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "system is NULL");
  std::lock_guard<std::mutex> lk(s->use);
  if (!s->factored) return fail(s, AIFMM_ERR_STATE, "solve before factor");
  if (!b || !x || nrhs <= 0 || ldb < s->N || ldx < s->N) return fail(s, AIFMM_ERR_ARG, "bad b/x/nrhs/ld");
  if (nrhs > 4096) return fail(s, AIFMM_ERR_ARG, "nrhs too large");
  return guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    aifmm::solve_system(*s, b, nrhs, ldb, x, ldx, is_device_ptr(b), is_device_ptr(x));
  });
}

aifmm_status aifmm_solve_noalloc(aifmm_system* s, const double* b, int64_t nrhs, int64_t ldb, double* x,
                                 int64_t ldx) {
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "system is NULL");
  std::lock_guard<std::mutex> lk(s->use);
  if (!s->factored) return fail(s, AIFMM_ERR_STATE, "solve before factor");
  if (!b || !x || nrhs <= 0 || ldb < s->N || ldx < s->N) return fail(s, AIFMM_ERR_ARG, "bad b/x/nrhs/ld");
  if (nrhs > 4096) return fail(s, AIFMM_ERR_ARG, "nrhs too large");
  return guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    if (!is_device_ptr(b) || !is_device_ptr(x))
      throw aifmm::Error{AIFMM_ERR_ARG, "the allocation-free solve takes device pointers only"};
    aifmm::solve_system_noalloc(*s, b, nrhs, ldb, x, ldx);
  });
}

aifmm_status aifmm_matvec(aifmm_system* s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy) {
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "system is NULL");
  std::lock_guard<std::mutex> lk(s->use);
  if (!x || !y || nrhs <= 0 || ldx < s->N || ldy < s->N || nrhs > 4096) return fail(s, AIFMM_ERR_ARG, "bad x/y/nrhs/ld");
  return guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    aifmm::matvec_system(*s, x, nrhs, ldx, y, ldy, is_device_ptr(x), is_device_ptr(y));
  });
}

aifmm_status aifmm_matvec_h2(aifmm_system* s, const double* x, int64_t nrhs, int64_t ldx, double* y, int64_t ldy) {
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "system is NULL");
  std::lock_guard<std::mutex> lk(s->use);
  if (!x || !y || nrhs <= 0 || ldx < s->N || ldy < s->N || nrhs > 4096) return fail(s, AIFMM_ERR_ARG, "bad x/y/nrhs/ld");
  return guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    aifmm::h2_matvec_system(*s, x, nrhs, ldx, y, ldy, is_device_ptr(x), is_device_ptr(y));
  });
}

aifmm_status aifmm_gmres(aifmm_system* op, aifmm_system* prec, const double* b, int64_t nrhs, int64_t ldb, double rtol,
                         int32_t restart, int32_t maxit, double* x, int64_t ldx, int32_t* iters, double* relres) {
  aifmm_system* s = prec;
  if (!s) return fail(nullptr, AIFMM_ERR_ARG, "preconditioner system is NULL");
  std::unique_lock<std::mutex> la(s->use, std::defer_lock), lb;
  if (op && op != s) {
    lb = std::unique_lock<std::mutex>(op->use, std::defer_lock);
    std::lock(la, lb);
  } else {
    la.lock();
  }
  if (!s->factored) return fail(s, AIFMM_ERR_STATE, "gmres before factor");
  if (!b || !x || nrhs <= 0 || ldb < s->N || ldx < s->N || nrhs > 4096 || !(rtol > 0.0) || restart <= 0 || maxit <= 0)
    return fail(s, AIFMM_ERR_ARG, "bad b/x/nrhs/ld/rtol/restart/maxit");
  if (op && op != s &&
      (op->N != s->N || op->d != s->d || op->L != s->L || op->leaf_off != s->leaf_off || op->K.kind != s->K.kind ||
       op->K.scale != s->K.scale || op->K.shift != s->K.shift || op->device != s->device))
    return fail(s, AIFMM_ERR_ARG, "operator and preconditioner systems differ (points, tree, kernel or device)");
  auto t0 = std::chrono::steady_clock::now();
  aifmm_status st = guarded(s, [&] {
    AIFMM_HIP(hipSetDevice(s->device));
    if (op && op != s && op->d_perm.download(op->stream) != s->d_perm.download(s->stream))
      throw aifmm::Error{AIFMM_ERR_ARG, "operator and preconditioner systems order the points differently"};
    aifmm::gmres_op_system(op, *s, b, nrhs, ldb, rtol, restart, maxit, x, ldx, iters, relres, is_device_ptr(b),
                           is_device_ptr(x));
  });
  s->stats.gmres_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

aifmm_status aifmm_get_depth(const aifmm_system* s, int32_t* L) {
  if (!s || !L) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  *L = s->L;
  return AIFMM_OK;
}

aifmm_status aifmm_get_ranks(const aifmm_system* s, int32_t level, int32_t* ranks) {
  if (!s || !ranks) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  if (level < 2 || level > s->L) return fail(nullptr, AIFMM_ERR_ARG, "level out of range");
  const aifmm::LevelDev& lv = s->lev[level];
  const std::vector<int>& k = s->factored ? lv.kfin : lv.knn;
  for (int b = 0; b < lv.nb; ++b) ranks[b] = k[b];
  return AIFMM_OK;
}

aifmm_status aifmm_get_stats(const aifmm_system* s, double* stats) {
  if (!s || !stats) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  for (int q = 0; q < AIFMM_STAT_COUNT; ++q) stats[q] = 0.0;
  stats[AIFMM_STAT_BUILD_S] = s->stats.build_s;
  stats[AIFMM_STAT_FACTOR_S] = s->stats.factor_s;
  stats[AIFMM_STAT_SOLVE_S] = s->stats.solve_s;
  stats[AIFMM_STAT_SCHUR_FLOPS] = s->stats.schur_flops;
  stats[AIFMM_STAT_SCHUR_BYTES] = s->stats.schur_bytes;
  stats[AIFMM_STAT_TRSM_FLOPS] = s->stats.trsm_flops;
  stats[AIFMM_STAT_LU_FLOPS] = s->stats.lu_flops;
  double bytes = 0;
  for (const auto& lv : s->lev) bytes += (double)lv.fslab.bytes() + (double)lv.slab.bytes() + (double)lv.d_Unn.bytes();
  stats[AIFMM_STAT_DEVICE_BYTES] = bytes;
  stats[AIFMM_STAT_SCHUR_KERNEL_S] = s->stats.schur_kernel_s;
  stats[AIFMM_STAT_SCHUR_LAUNCHES] = s->stats.schur_launches;
  stats[AIFMM_STAT_COMPRESS_KERNEL_S] = s->stats.compress_kernel_s;
  stats[AIFMM_STAT_COMPRESS_LAUNCHES] = s->stats.compress_launches;
  stats[AIFMM_STAT_GMRES_S] = s->stats.gmres_s;
  stats[AIFMM_STAT_TRSM_KERNEL_S] = s->stats.trsm_kernel_s;
  stats[AIFMM_STAT_TRSM_LAUNCHES] = s->stats.trsm_launches;
  stats[AIFMM_STAT_SOLVE_BYTES] = s->stats.solve_bytes;
  return AIFMM_OK;
}

aifmm_status aifmm_get_level_stats(const aifmm_system* s, int32_t level, double* out) {
  if (!s || !out) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  if (!s->factored) return fail(nullptr, AIFMM_ERR_STATE, "no factorization");
  if (level < 2 || level > s->L || level >= (int)s->stats.lvl.size()) return fail(nullptr, AIFMM_ERR_ARG, "level out of range");
  const aifmm::LevelStats& v = s->stats.lvl[level];
  for (int q = 0; q < AIFMM_LSTAT_COUNT; ++q) out[q] = 0.0;
  out[AIFMM_LSTAT_FACTOR_S] = v.factor_s;
  out[AIFMM_LSTAT_SCHUR_FLOPS] = v.schur_flops;
  out[AIFMM_LSTAT_SCHUR_BYTES] = v.schur_bytes;
  out[AIFMM_LSTAT_TRSM_FLOPS] = v.trsm_flops;
  out[AIFMM_LSTAT_TRSM_FLOPS_IMPL] = v.trsm_flops_impl;
  out[AIFMM_LSTAT_LU_FLOPS] = v.lu_flops;
  out[AIFMM_LSTAT_SCHUR_KERNEL_S] = v.schur_s;
  out[AIFMM_LSTAT_TRSM_KERNEL_S] = v.trsm_s;
  out[AIFMM_LSTAT_COMPRESS_KERNEL_S] = v.compress_s;
  out[AIFMM_LSTAT_COMPRESS_FLOPS] = v.compress_flops;
  out[AIFMM_LSTAT_COMPRESSIONS] = v.compressions;
  out[AIFMM_LSTAT_ROUNDS] = v.rounds;
  out[AIFMM_LSTAT_CRIT_STEPS] = v.crit_steps;
  out[AIFMM_LSTAT_PIVOT_STEPS] = v.pivot_steps;
  out[AIFMM_LSTAT_BOXES] = v.boxes;
  return AIFMM_OK;
}

aifmm_status aifmm_get_trace(const aifmm_system* s, int32_t* rec, double* ratio, int64_t cap, int64_t* count) {
  if (!s || !count) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  if (!s->factored) return fail(nullptr, AIFMM_ERR_STATE, "no factorization");
  *count = (int64_t)s->trace.size();
  for (int64_t q = 0; q < *count && q < cap; ++q) {
    const aifmm::TraceRec& t = s->trace[q];
    if (rec) {
      int32_t* o = rec + q * 10;
      o[0] = t.level; o[1] = t.i; o[2] = t.kind; o[3] = t.partner;
      for (int a = 0; a < 6; ++a) o[4 + a] = t.r[a];
    }
    if (ratio)
      for (int a = 0; a < 8; ++a) ratio[q * 8 + a] = t.ratio[a];
  }
  return AIFMM_OK;
}

aifmm_status aifmm_get_nnca(const aifmm_system* s, int32_t level, int32_t box, int64_t* t_i, int64_t* s_i, double* U,
                            int32_t* k, int32_t* rows) {
  if (!s || !k || !rows) return fail(nullptr, AIFMM_ERR_ARG, "NULL argument");
  if (level < 2 || level > s->L) return fail(nullptr, AIFMM_ERR_ARG, "level out of range");
  const aifmm::LevelDev& lv = s->lev[level];
  if (box < 0 || box >= lv.nb) return fail(nullptr, AIFMM_ERR_ARG, "box out of range");
  return guarded(const_cast<aifmm_system*>(s), [&] {
    hipStream_t st = s->stream;
    int kb = lv.knn[box];
    int t0 = lv.T_off[box], m = lv.T_off[box + 1] - t0;
    *k = kb;
    *rows = m;
    std::vector<int64_t> perm = s->d_perm.download(st);
    std::vector<int> pr = lv.d_piv_r.download(st), pc = lv.d_piv_c.download(st);
    for (int q = 0; q < kb; ++q) {
      if (t_i) t_i[q] = perm[pr[t0 + q]];
      if (s_i) s_i[q] = perm[pc[t0 + q]];
    }
    if (U && kb > 0 && m > 0)
      AIFMM_HIP(hipMemcpy(U, lv.d_Unn.p + lv.Unn_off[box], sizeof(double) * (size_t)m * kb, hipMemcpyDeviceToHost));
  });
}

const char* aifmm_last_error(const aifmm_system* s) {
  if (s) return s->err.c_str();
  return g_err.c_str();
}

void aifmm_destroy(aifmm_system* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  delete s;
}

}  // extern "C"
