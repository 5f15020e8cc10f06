// Workgroup-cooperative dense building blocks for gfx950 (wave64, 256-thread workgroups).
// Used by the NNCA, compression and elimination kernels.  Every routine is called by all
// threads of a workgroup and ends with a barrier, so results are visible on return.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "system.hpp"

namespace aifmm {

constexpr int WG = 256;
constexpr int WAVE = 64;

// e^x: Cody-Waite reduction x = k ln2 + r with |r| <= ln2/2 (ln2 split in a high part with
// trailing zero bits and a low correction), Taylor series of e^r to degree 13 in Horner form
// with fused multiply-adds (truncation below 4e-18 relative), exact scaling by 2^k.
__device__ inline double dexp(double x) {
  if (x < -745.0) return 0.0;
  double kd = rint(x * 1.4426950408889634);
  double r = fma(-kd, 6.93147180369123816490e-01, x);
  r = fma(-kd, 1.90821492927058770002e-10, r);
  double p = 1.6059043836821613e-10;
  p = fma(p, r, 2.08767569878681e-09);
  p = fma(p, r, 2.505210838544172e-08);
  p = fma(p, r, 2.755731922398589e-07);
  p = fma(p, r, 2.7557319223985893e-06);
  p = fma(p, r, 2.48015873015873e-05);
  p = fma(p, r, 0.0001984126984126984);
  p = fma(p, r, 0.001388888888888889);
  p = fma(p, r, 0.008333333333333333);
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)kd);
}

// Kernel entry A_ij = kappa(|p_i - p_j|) + shift * delta_ij on tree positions i, j.  The
// squared distance is formed without fused multiply-add so the value is the correctly
// rounded sequence of IEEE operations.
__device__ inline double kernel_entry(const KernelDesc& K, const double* __restrict__ pts, int d, int i, int j) {
  double r2 = 0.0;
  for (int t = 0; t < d; ++t) {
    double z = __dsub_rn(pts[i * d + t], pts[j * d + t]);
    r2 = __dadd_rn(r2, __dmul_rn(z, z));
  }
  double v;
  if (K.kind == 0) v = dexp(-sqrt(r2) / K.scale);
  else v = 1.0 / sqrt(__dadd_rn(r2, __dmul_rn(K.scale, K.scale)));
  if (i == j) v += K.shift;
  return v;
}

struct ValIdx {
  double v;
  int i;
};
__device__ inline bool vi_better(const ValIdx& a, const ValIdx& b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}

// Workgroup-wide reductions for NT threads (NT a multiple of 64).  sh needs NT/64 + 1 slots.
// argmax: ties to the lowest index; invalid lanes pass v = -1, i = INT_MAX.
template <int NT = WG>
__device__ inline ValIdx wg_argmax(ValIdx x, ValIdx* sh) {
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    ValIdx o;
    o.v = __shfl_down(x.v, off, WAVE);
    o.i = __shfl_down(x.i, off, WAVE);
    if (vi_better(o, x)) x = o;
  }
  int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    ValIdx b = sh[0];
    for (int q = 1; q < NT / WAVE; ++q)
      if (vi_better(sh[q], b)) b = sh[q];
    sh[NT / WAVE] = b;
  }
  __syncthreads();
  ValIdx r = sh[NT / WAVE];
  __syncthreads();
  return r;
}

template <int NT = WG>
__device__ inline double wg_sum(double x, double* sh) {
  for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_down(x, off, WAVE);
  int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < NT / WAVE; ++q) s += sh[q];
    sh[NT / WAVE] = s;
  }
  __syncthreads();
  double r = sh[NT / WAVE];
  __syncthreads();
  return r;
}

// In-place LU with row partial pivoting (ties to the lowest row) of the m x m row-major A;
// ipiv[k] is the row swapped with k at step k.  Returns 0 or 1+k for an exactly zero pivot.
template <int NT = WG>
__device__ inline int wg_lu(int m, double* A, int lda, int* ipiv, ValIdx* shv) {
  for (int k = 0; k < m; ++k) {
    ValIdx best{-1.0, INT_MAX};
    for (int i = k + (int)threadIdx.x; i < m; i += NT) {
      ValIdx c{fabs(A[(size_t)i * lda + k]), i};
      if (vi_better(c, best)) best = c;
    }
    best = wg_argmax<NT>(best, shv);
    if (best.v == 0.0) return 1 + k;
    int p = best.i;
    if (threadIdx.x == 0) ipiv[k] = p;
    if (p != k) {
      for (int j = threadIdx.x; j < m; j += NT) {
        double a = A[(size_t)k * lda + j];
        A[(size_t)k * lda + j] = A[(size_t)p * lda + j];
        A[(size_t)p * lda + j] = a;
      }
    }
    __syncthreads();
    double piv = A[(size_t)k * lda + k];
    int rem = m - k - 1;
    for (int i = threadIdx.x; i < rem; i += NT) A[(size_t)(k + 1 + i) * lda + k] /= piv;
    __syncthreads();
    for (int idx = threadIdx.x; idx < rem * rem; idx += NT) {
      int i = k + 1 + idx / rem, j = k + 1 + idx % rem;
      A[(size_t)i * lda + j] = fma(-A[(size_t)i * lda + k], A[(size_t)k * lda + j], A[(size_t)i * lda + j]);
    }
    __syncthreads();
  }
  return 0;
}


// FP64 MFMA accumulator of the blocked LU (t_lu_blocked)
typedef double lu_dbl4 __attribute__((ext_vector_type(4)));

}  // namespace aifmm
