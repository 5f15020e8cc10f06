// Factorization (Sec. 3.2-3.3, Algorithm "Efficient Elimination") on the device.
//
// Per level l = L..2 and per colour batch of the colour-major order:
//   1. compression rounds: round r compresses the r-th pending pair of every box of the
//      colour (P2P pairs by four RRQRs, P2L/M2P pairs by two, Sec. 3.2.1-3.2.3), then the
//      basis changes of the other blocks of the touched rows Z and columns y are applied
//      (left factors L in one launch, right factors R^* in the next, so no block element is
//      written twice in a launch);
//   2. elimination of every box of the colour: gather of the pivot block
//      [[K_ii, U_i], [V_i^*, 0]] and of the coupled blocks, pivoted LU, triangular solves
//      W = Piv^{-1} A[(X_i,Y_i), O_c], Schur update A[O_r, O_c] -= A[O_r, x_i] W_x and the
//      new rows Z_i = W_z.
// Between levels the remaining Z^{(l)} x y^{(l)} blocks become the next level's particle
// blocks (eq. particleAtNonLeafLevel), and after level 2 the level-2 multipole system is
// factored densely (it is solved directly at the end of the elimination, Sec. 3.2).
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>

#include "dense_wg.hpp"
#include "team.hpp"
#include "system.hpp"

namespace aifmm {

struct RoundEntry {
  int i, kind, partner;
  int e_ij, e_ji;  // M2L slot entries: (i, partner) and (partner, i)
  int f_ij, f_ji;  // fill slot entries: (i, partner) and (partner, i)
  int sys, tidx;   // the system (index into the launch's level tables) and its trace record
};
struct XformEntry {
  int x, skip, pair, side;
  int sys;
};

struct LevelPtrs {
  int l, nb, d;
  const int* n;
  int* k;
  int* kn;
  const int* nbr_off;
  const int* nbr;
  const int* il_off;
  const int* il;
  const int* il_tr;
  const int* p2_off;
  const int* p2;
  const int* grp_off;
  const int* grp_box;
  const int* grp_elim;
  double* slab;
  const int64_t* near_slot;
  const int64_t* p2_slot;
  const int64_t* il_slot;
  const int64_t* U_off;
  const int64_t* V_off;
  const int64_t* l2l_off;
  const int64_t* m2m_off;
  const int* kP;
  const int64_t* tslot;
  int* grc;          // per box 2 x 28 ints: row and column offsets of the coupled groups
  int Gmax;
  double* fslab;
  const int64_t* fLU;
  const int64_t* fC;
  const int64_t* fW;
  int* fpiv;
  const int64_t* fpiv_off;
  int* trace;        // per compression: r1 r2 r3 r4 k_i' k_j'
  double* trace_ratio;  // per compression: 4 x (kept, next) decision ratios
  int* flag;         // the system's flags ([0] singular, [1] box, [2] level)
  double tol;        // the system's eps_A
};

// Every factorization kernel reads the level tables of the system its work item belongs to:
// PP holds one LevelPtrs per system of the launch (one system: PP[0]), and box lists come with
// bsys, the system of each listed box (nullptr: every box of system 0).
__device__ inline const LevelPtrs& sys_ptrs(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys, int item) {
  return PP[bsys ? bsys[item] : 0];
}

// ------------------------------------------------------------------------------------------
// compression of one pending pair per workgroup (CT threads)
// ------------------------------------------------------------------------------------------
constexpr int CT = 512;

// R: arithmetic of the compression (double, or float in the precision form); the block store
// stays FP64 and operands are converted on load / store.
template <class RT, int RMAX>
__global__ void __launch_bounds__(CT) k_compress(const LevelPtrs* __restrict__ PP, const RoundEntry* __restrict__ ent,
                                                 int nent, double* ws, int64_t wsz, int cap, int G, unsigned* ctr,
                                                 Cand* part, int* abort, int lds_cols, double* pubbuf) {
  int e = blockIdx.x / G;
  if (e >= nent) return;
  Team<CT> T;
  T.init(blockIdx.x - e * G, G, ctr + (size_t)e * CTR_STRIDE, part + (size_t)e * 4 * G * CAND_STRIDE, abort);
  // a team of two or more runs the independent pivoted QRs of the compression concurrently on
  // its two halves (sub-teams A: members 0 .. GA-1 and B: the rest), each with its own barrier
  // counter, exchange slots, publication slots and workspace, and joins them with a team barrier
  const bool split = G > 1;
  const int GA = G / 2;
  const bool inA = T.member < GA;
  // the team that runs a chain: the half-team when split, else the lone workgroup (G == 1, whose
  // barrier keeps no state); one object initialised from selected values, so it stays in
  // registers
  Team<CT> C;
  if (split)
    C.init(inA ? T.member : T.member - GA, inA ? GA : G - GA, ctr + (size_t)(nent + 2 * e + (inA ? 0 : 1)) * CTR_STRIDE,
           part + ((size_t)e * 4 * G + 2 * G + (inA ? 0 : 2 * GA)) * CAND_STRIDE, abort);
  else
    C.init(0, 1, ctr + (size_t)e * CTR_STRIDE, part + (size_t)e * 4 * G * CAND_STRIDE, abort);
  RoundEntry R = ent[e];
  const LevelPtrs& P = PP[R.sys];
  const double tol = P.tol;
  int* tr = P.trace + (size_t)R.tidx * 6;
  double* trr = P.trace_ratio + (size_t)R.tidx * 8;
  __shared__ ValIdx shv[CT / WAVE + 1];
  extern __shared__ double shm[];  // one reflector (cap), pivot positions (2 x 2cap ints), own norms (2cap)
  // vsh: the reflector, with the register tier's rows up to 16 RMAX
  constexpr int RROWS = 16 * RMAX;
  const int vlen = cap > RROWS ? cap : RROWS;
  RT* vsh = (RT*)shm;
  int* pos = (int*)(vsh + vlen);
  int* at = pos + 2 * cap;
  // columns of the pivoted QRs and Q formations: the register tier (RMAX rows per lane), then
  // lds_cols per member in LDS, then the workspace; the members' candidate pivot columns
  // published in pub (2 x G x vlen entries per compression)
  RT* lnr = (RT*)(at + 2 * cap);  // the member's own columns' norms (2 cap entries)
  RT* lcol = lnr + 2 * cap;
  RT* pub = (RT*)pubbuf + (size_t)e * 2 * G * vlen;
  RT* pubS = pub + (split && !inA ? (size_t)2 * GA * vlen : 0);  // the sub-team's publication slots
  RT* w = (RT*)(ws + (size_t)e * wsz);
  size_t c2 = (size_t)cap * cap;
  RT* Lb_i = w;
  RT* Rb_i = w + c2;
  RT* Lb_j = w + 2 * c2;
  RT* Rb_j = w + 3 * c2;
  RT* M = w + 4 * c2;        // cap x 2cap
  RT* V1 = w + 6 * c2;
  RT* V2 = w + 7 * c2;
  RT* V3 = w + 8 * c2;
  RT* V4 = w + 9 * c2;
  RT* nU = w + 10 * c2;      // new bases, cap x cap, ld cap
  RT* nV = w + 11 * c2;
  RT* nUj = w + 12 * c2;
  RT* nVj = w + 13 * c2;
  RT* t1 = w + 14 * c2;      // cap x 2cap; column storage of the QRs without LDS columns
  RT* t2 = w + 16 * c2;
  RT* tau = w + 17 * c2;     // 4 * cap
  RT* nrm = tau + 4 * cap;   // 2 * cap
  RT* Mb = nrm + 2 * cap;    // sub-team B: input matrix (cap x 2cap), column storage, norms
  RT* t1b = Mb + 2 * c2;
  RT* nrmb = t1b + 2 * c2;
  const double* U_i = P.slab + P.U_off[R.i];
  const double* V_i = P.slab + P.V_off[R.i];
  int i = R.i, ni = P.n[i], ki = P.k[i];
  int ki1 = ki > 0 ? ki : 1;
  if (R.kind == 0) {
    int j = R.partner, nj = P.n[j], kj = P.k[j];
    int kj1 = kj > 0 ? kj : 1;
    const double* U_j = P.slab + P.U_off[j];
    const double* V_j = P.slab + P.V_off[j];
    double* Fij = P.slab + P.p2_slot[R.f_ij];  // (X_i, x_j): ni x nj, ld nj
    double* Fji = P.slab + P.p2_slot[R.f_ji];  // (X_j, x_i): nj x ni, ld ni
    double* Aij = P.slab + P.il_slot[R.e_ij];  // (Z_i, y_j): ki x kj, ld nj
    double* Aji = P.slab + P.il_slot[R.e_ji];  // (Z_j, y_i): kj x ki, ld ni
    // two chains: RRQR1 -> Q1 -> RRQR3 and RRQR2 -> Q2 -> RRQR4 (sub-teams A and B, or one
    // after the other on a lone workgroup)
    int r1 = 0, r2 = 0, r3 = 0, r4 = 0;
    if (!split || inA) {
      // RRQR1: [U_i | P2P_ij] = U~_i L_ij
      int ld = ki + nj;
      t_copy(C, ni, ki, U_i, ni, M, ld);
      t_copy(C, ni, nj, Fij, nj, M + ki, ld);
      r1 = t_cpqr<CT, RMAX>(C, ni, ld, M, ld, tol, V1, cap, tau, nrm, lnr, shv, vsh, pos, at, trr, lcol, lds_cols, pubS, t1);
      // RRQR3: [V_j | L~_ij^*] with L~_ij = Q1_{r1}^* P2P_ij  (Q1_{r1} = first r1 columns of U~_i)
      t_formq<CT, RMAX>(C, ni, r1, r1, V1, cap, tau, nU, cap, vsh, 0, lcol, lds_cols, t1);
      ld = kj + r1;
      t_copy(C, nj, kj, V_j, nj, M, ld);
      t_gemm(C, nj, r1, ni, 1.0, Fij, nj, true, nU, cap, false, 0.0, M + kj, ld);
      r3 = t_cpqr<CT, RMAX>(C, nj, ld, M, ld, tol, V3, cap, tau + 2 * cap, nrm, lnr, shv, vsh, pos, at, trr + 4, lcol, lds_cols, pubS, t1);
      if (C.gtid == 0) {
        tr[0] = r1;
        tr[2] = r3;
      }
    }
    if (!split || !inA) {
      RT* Mc = split ? Mb : M;
      RT* gc = split ? t1b : t1;
      RT* nc = split ? nrmb : nrm;
      // RRQR2: [U_j | P2P_ji] = U~_j L_ji
      int ld = kj + ni;
      t_copy(C, nj, kj, U_j, nj, Mc, ld);
      t_copy(C, nj, ni, Fji, ni, Mc + kj, ld);
      r2 = t_cpqr<CT, RMAX>(C, nj, ld, Mc, ld, tol, V2, cap, tau + cap, nc, lnr, shv, vsh, pos, at, trr + 2, lcol, lds_cols, pubS, gc);
      // RRQR4: [V_i | L~_ji^*]
      t_formq<CT, RMAX>(C, nj, r2, r2, V2, cap, tau + cap, nUj, cap, vsh, 0, lcol, lds_cols, gc);
      ld = ki + r2;
      t_copy(C, ni, ki, V_i, ni, Mc, ld);
      t_gemm(C, ni, r2, nj, 1.0, Fji, ni, true, nUj, cap, false, 0.0, Mc + ki, ld);
      r4 = t_cpqr<CT, RMAX>(C, ni, ld, Mc, ld, tol, V4, cap, tau + 3 * cap, nc, lnr, shv, vsh, pos, at, trr + 6, lcol, lds_cols, pubS, gc);
      if (C.gtid == 0) {
        tr[1] = r2;
        tr[3] = r4;
      }
    }
    if (split) {  // join (waits for a whole chain: a longer bound); every member takes the ranks
      T.sync(1u << 28);
      if (T.bad) return;  // the other half's ranks may be stale: the host reports the failure
      r1 = tr[0];
      r2 = tr[1];
      r3 = tr[2];
      r4 = tr[3];
    }
    int kin = r1 > r4 ? r1 : r4, kjn = r2 > r3 ? r2 : r3;
    // new orthonormal bases: columns beyond a tolerance rank are further columns of the same
    // Householder Q (the first r1 / r2 columns of U~_i / U~_j are already formed), then the
    // coefficients by projection, U_i = U~_i L_i, V_i = V~_i R_i, ...: the i side on half A,
    // the j side on half B
    if (!split || inA) {
      t_formq<CT, RMAX>(C, ni, r1, kin, V1, cap, tau, nU, cap, vsh, r1, lcol, lds_cols, t1);
      t_formq<CT, RMAX>(C, ni, r4, kin, V4, cap, tau + 3 * cap, nV, cap, vsh, 0, lcol, lds_cols, t1);
      t_gemm(C, kin, ki, ni, 1.0, nU, cap, true, U_i, ni, false, 0.0, Lb_i, ki1);
      t_gemm(C, kin, ki, ni, 1.0, nV, cap, true, V_i, ni, false, 0.0, Rb_i, ki1);
    }
    if (!split || !inA) {
      RT* gc = split ? t1b : t1;
      t_formq<CT, RMAX>(C, nj, r2, kjn, V2, cap, tau + cap, nUj, cap, vsh, r2, lcol, lds_cols, gc);
      t_formq<CT, RMAX>(C, nj, r3, kjn, V3, cap, tau + 2 * cap, nVj, cap, vsh, 0, lcol, lds_cols, gc);
      t_gemm(C, kjn, kj, nj, 1.0, nUj, cap, true, U_j, nj, false, 0.0, Lb_j, kj1);
      t_gemm(C, kjn, kj, nj, 1.0, nVj, cap, true, V_j, nj, false, 0.0, Rb_j, kj1);
    }
    if (split) {
      T.sync(1u << 28);
      if (T.bad) return;
    }
    int nj1 = nj > 0 ? nj : 1, ni1 = ni > 0 ? ni : 1;
    if (!split || inA) {
      // A_ij := L_i A_ij R_j^* + R~_ij^*,  L~_ij = U~_i^* P2P_ij (kin x nj), R~_ij = V~_j^* L~_ij^*
      t_gemm(C, kin, nj, ni, 1.0, nU, cap, true, Fij, nj, false, 0.0, t1, nj1);
      t_gemm(C, kjn, kin, nj, 1.0, nVj, cap, true, t1, nj1, true, 0.0, t2, cap);   // R~_ij
      t_gemm(C, kin, kj, ki, 1.0, Lb_i, ki1, false, Aij, nj, false, 0.0, t1, kj1);  // L_i A_ij
      for (int idx = C.gtid; idx < kin * kjn; idx += C.GT) {
        int r = idx / kjn, c = idx - r * kjn;
        Aij[(size_t)r * nj + c] = t2[(size_t)c * cap + r];
      }
      C.sync();
      t_gemm(C, kin, kjn, kj, 1.0, t1, kj1, false, Rb_j, kj1, true, 1.0, Aij, nj);
    }
    if (!split || !inA) {
      // A_ji := L_j A_ji R_i^* + R~_ji^*  (half B: temporaries in its own workspace)
      RT* u1 = split ? t1b : t1;
      RT* u2 = split ? Mb : t2;
      t_gemm(C, kjn, ni, nj, 1.0, nUj, cap, true, Fji, ni, false, 0.0, u1, ni1);
      t_gemm(C, kin, kjn, ni, 1.0, nV, cap, true, u1, ni1, true, 0.0, u2, cap);    // R~_ji
      t_gemm(C, kjn, ki, kj, 1.0, Lb_j, kj1, false, Aji, ni, false, 0.0, u1, ki1);
      for (int idx = C.gtid; idx < kjn * kin; idx += C.GT) {
        int r = idx / kin, c = idx - r * kin;
        Aji[(size_t)r * ni + c] = u2[(size_t)c * cap + r];
      }
      C.sync();
      t_gemm(C, kjn, kin, ki, 1.0, u1, ki1, false, Rb_i, ki1, true, 1.0, Aji, ni);
    }
    if (split) {
      T.sync(1u << 28);
      if (T.bad) return;
    }
    // bases, fill-ins, ranks
    t_copy(T, ni, kin, nU, cap, (double*)U_i, ni);
    t_copy(T, ni, kin, nV, cap, (double*)V_i, ni);
    t_copy(T, nj, kjn, nUj, cap, (double*)U_j, nj);
    t_copy(T, nj, kjn, nVj, cap, (double*)V_j, nj);
    t_zero(T, ni, nj, Fij, nj);
    t_zero(T, nj, ni, Fji, ni);
    if (T.gtid == 0) {
      P.kn[i] = kin;
      P.kn[j] = kjn;
      tr[0] = r1; tr[1] = r2; tr[2] = r3; tr[3] = r4; tr[4] = kin; tr[5] = kjn;
    }
  } else {
    int r = R.partner, nr = P.n[r], kr = P.k[r];
    int kr1 = kr > 0 ? kr : 1;
    double* M2P = P.slab + P.p2_slot[R.f_ij];  // (X_i, y_r): ni x kr, ld nr
    double* P2L = P.slab + P.p2_slot[R.f_ji];  // (Z_r, x_i): kr x ni, ld ni
    double* Air = P.slab + P.il_slot[R.e_ij];  // (Z_i, y_r): ki x kr, ld nr
    double* Ari = P.slab + P.il_slot[R.e_ji];  // (Z_r, y_i): kr x ki, ld ni
    int ld = ki + kr;
    int r5 = 0, r6 = 0;
    if (!split || inA) {
      // RRQR: [V_i | P2L_ri^*] = V~_i R_ri
      t_copy(C, ni, ki, V_i, ni, M, ld);
      for (int idx = C.gtid; idx < ni * kr; idx += C.GT) {
        int a = idx / kr, c = idx - a * kr;
        M[(size_t)a * ld + ki + c] = P2L[(size_t)c * ni + a];
      }
      C.sync();
      r5 = t_cpqr<CT, RMAX>(C, ni, ld, M, ld, tol, V1, cap, tau, nrm, lnr, shv, vsh, pos, at, trr, lcol, lds_cols, pubS, t1);
      if (C.gtid == 0) tr[0] = r5;
    }
    if (!split || !inA) {
      RT* Mc = split ? Mb : M;
      // RRQR: [U_i | M2P_ir] = U~_i L_ir
      t_copy(C, ni, ki, U_i, ni, Mc, ld);
      t_copy(C, ni, kr, M2P, nr, Mc + ki, ld);
      // column storage of the chain: t1b, never t1, which holds the new A_ri below when both
      // chains run on one workgroup
      r6 = t_cpqr<CT, RMAX>(C, ni, ld, Mc, ld, tol, V2, cap, tau + cap, split ? nrmb : nrm, lnr, shv, vsh, pos, at, trr + 2,
                  lcol, lds_cols, pubS, t1b);
      if (C.gtid == 0) tr[1] = r6;
    }
    if (split) {
      T.sync(1u << 28);
      if (T.bad) return;
      r5 = tr[0];
      r6 = tr[1];
    }
    int kin = r5 > r6 ? r5 : r6;
    // the V side (A_ri) on half A, the U side (A_ir) on half B
    if (!split || inA) {
      t_formq<CT, RMAX>(C, ni, r5, kin, V1, cap, tau, nV, cap, vsh, 0, lcol, lds_cols, t1);
      t_gemm(C, kin, ki, ni, 1.0, nV, cap, true, V_i, ni, false, 0.0, Rb_i, ki1);
      // A_ri := A_ri R_i^* + P2L_ri V~_i
      t_gemm(C, kr, kin, ki, 1.0, Ari, ni, false, Rb_i, ki1, true, 0.0, t1, cap);
      t_gemm(C, kr, kin, ni, 1.0, P2L, ni, false, nV, cap, false, 1.0, t1, cap);
    }
    if (!split || !inA) {
      t_formq<CT, RMAX>(C, ni, r6, kin, V2, cap, tau + cap, nU, cap, vsh, 0, lcol, lds_cols, t1b);  // t1 holds A_ri here
      t_gemm(C, kin, ki, ni, 1.0, nU, cap, true, U_i, ni, false, 0.0, Lb_i, ki1);
      // A_ir := L_i A_ir + U~_i^* M2P_ir
      t_gemm(C, kin, kr, ki, 1.0, Lb_i, ki1, false, Air, nr, false, 0.0, t2, kr1);
      t_gemm(C, kin, kr, ni, 1.0, nU, cap, true, M2P, nr, false, 1.0, t2, kr1);
    }
    if (split) {
      T.sync(1u << 28);
      if (T.bad) return;
    }
    t_copy(T, kr, kin, t1, cap, Ari, ni);
    t_copy(T, kin, kr, t2, kr1, Air, nr);
    t_copy(T, ni, kin, nU, cap, (double*)U_i, ni);
    t_copy(T, ni, kin, nV, cap, (double*)V_i, ni);
    t_zero(T, nr, ni, P2L, ni);
    t_zero(T, ni, nr, M2P, nr);
    if (T.gtid == 0) {
      P.kn[i] = kin;
      tr[0] = r5; tr[1] = r6; tr[2] = 0; tr[3] = 0; tr[4] = kin; tr[5] = 0;
      trr[4] = trr[5] = trr[6] = trr[7] = 0.0;
    }
  }
}

__global__ void k_commit(const LevelPtrs* __restrict__ PP, const XformEntry* __restrict__ xe, int nx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nx) {
    const LevelPtrs& P = PP[xe[t].sys];
    P.k[xe[t].x] = P.kn[xe[t].x];
  }
}

// ------------------------------------------------------------------------------------------
// elimination of the boxes of one colour
// ------------------------------------------------------------------------------------------
__device__ inline int grp_rows(const LevelPtrs& P, int g, int G, int b, int gb, int ge) {
  if (g == G - 1) return P.k[b];
  return ge ? P.k[gb] : P.n[gb];
}
__device__ inline int64_t near_entry(const LevelPtrs& P, int p, int q) {
  for (int e = P.nbr_off[p]; e < P.nbr_off[p + 1]; ++e)
    if (P.nbr[e] == q) return P.near_slot[e];
  return -1;
}

// Pivot block [[K_bb, U_b],[V_b^*, 0]] (into the factor store), right-hand sides
// [A[X_b, O_c] | E | I] (into the colour's workspace, ld C + n) and the coupled column blocks
// A[O_r, x_b] of box b (GS workgroups per box).
constexpr int GS = 16;  // workgroups per box of k_elim_gather
__global__ void __launch_bounds__(WG) k_elim_gather(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys,
                                                   const int* __restrict__ boxes, double* rws, int64_t rstride) {
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.x);
  int b = boxes[blockIdx.x];
  int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
  int n = P.n[b], k = P.k[b], m = n + k;
  double* Piv = P.fslab + P.fLU[b];
  double* W = rws + (size_t)blockIdx.x * rstride;  // the right-hand sides [A[X_b, O_c] | E | I]
  double* Cb = P.fslab + P.fC[b];
  // column (co) and coupled-row (ro) offsets of the groups, the group sizes and source blocks
  __shared__ int co[29], ro[29], cdim[28];
  __shared__ int64_t src_bq[28], src_qb[28];
  __shared__ int ldq[28];
  if (threadIdx.x == 0) {
    int r0 = 0, c0 = 0;
    for (int g = 0; g < G; ++g) {
      int q = P.grp_box[g0 + g];
      int cd = grp_rows(P, g, G, b, q, P.grp_elim[g0 + g]);
      co[g] = c0;
      ro[g] = r0;
      cdim[g] = cd;
      if (g < G - 1) {
        src_bq[g] = near_entry(P, b, q);  // (X_b, x_q | y_q), ld n_q
        src_qb[g] = near_entry(P, q, b);  // (X_q | Z_q, x_b), ld n_b
        ldq[g] = P.n[q];
        r0 += cd;
      }
      c0 += cd;
    }
    co[G] = c0;
    ro[G] = r0;
    if (blockIdx.y == 0) {  // group offsets for the Schur update: rows (all but y_b's group), columns
      int* rc = P.grc + (size_t)b * 56;
      for (int g = 0; g <= G; ++g) {
        rc[g] = ro[g];
        rc[28 + g] = co[g];
      }
    }
  }
  __syncthreads();
  const int C = co[G], ldw = C + n;
  const double* Kbb = P.slab + near_entry(P, b, b);
  const double* Ub = P.slab + P.U_off[b];
  const double* Vb = P.slab + P.V_off[b];
  const int gt = blockIdx.y * WG + threadIdx.x;
  for (int idx = gt; idx < m * m; idx += GS * WG) {
    int r = idx / m, c = idx - r * m;
    double v = 0.0;
    if (r < n) v = c < n ? Kbb[(size_t)r * n + c] : Ub[(size_t)r * n + (c - n)];
    else if (c < n) v = Vb[(size_t)c * n + (r - n)];
    Piv[idx] = v;
  }
  // every element of W written once: one wave per (row, segment); segments g < G are the
  // column groups, segment G the extension columns C .. C+n-1 (Piv^{-1}[:, x_b])
  const int lane = threadIdx.x % WAVE;
  const int wid = blockIdx.y * (WG / WAVE) + threadIdx.x / WAVE, nwv = GS * (WG / WAVE);
  for (int it = wid; it < m * (G + 1); it += nwv) {
    const int r = it / (G + 1), g = it - r * (G + 1);
    double* Wr = W + (size_t)r * ldw;
    if (g == G) {
      for (int c = lane; c < n; c += WAVE) Wr[C + c] = (r < n && c == r) ? 1.0 : 0.0;
    } else if (g == G - 1) {  // (Y_b, y_b) = -I
      for (int c = lane; c < cdim[g]; c += WAVE) Wr[co[g] + c] = (r >= n && c == r - n) ? -1.0 : 0.0;
    } else {
      const double* Bbq = P.slab + src_bq[g] + (size_t)r * ldq[g];
      for (int c = lane; c < cdim[g]; c += WAVE) Wr[co[g] + c] = r < n ? Bbq[c] : 0.0;
    }
  }
  // coupled column blocks A[O_r, x_b]: one wave per row
  const int R = ro[G > 0 ? G - 1 : 0];
  for (int rr = wid; rr < R; rr += nwv) {
    int g = 0;
    while (ro[g + 1] <= rr) ++g;
    const double* Bqb = P.slab + src_qb[g] + (size_t)(rr - ro[g]) * n;
    for (int c = lane; c < n; c += WAVE) Cb[(size_t)rr * n + c] = Bqb[c];
  }
}

constexpr int LU_NB = 16;
// Pivot-block LU of every box of a colour, G workgroups per box (a team, co-resident through a
// cooperative launch when G > 1; ctr, status: one barrier counter, zero at launch, and one
// status word per box).
__global__ void __launch_bounds__(WG) k_elim_lu(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys,
                                                const int* __restrict__ boxes, int64_t dyn_bytes, int G, unsigned* ctr,
                                                int* status, int* abort) {
  const int e = blockIdx.x / G;
  const LevelPtrs& P = sys_ptrs(PP, bsys, e);
  int* flag = P.flag;
  int b = boxes[e];
  int m = P.n[b] + P.k[b];
  Team<WG> T;
  T.init(blockIdx.x - e * G, G, ctr + (size_t)e * CTR_STRIDE, nullptr, abort);
  __shared__ ValIdx shv[WG / WAVE + 1];
  __shared__ double sh[LU_NB + 64 * (LU_NB + 1) + LU_NB * 65];
  __shared__ int ipv[LU_NB];
  // dynamic LDS (dyn_bytes): the panels of the factorization when m (LU_NB + 1) doubles fit,
  // afterwards 2 m ints: the row swaps, then the row permutation
  extern __shared__ double dyn[];
  int* pm = (int*)dyn;
  int* piv = P.fpiv + P.fpiv_off[b];
  const bool lp = (int64_t)m * (LU_NB + 1) * (int64_t)sizeof(double) <= dyn_bytes;
  int st = t_lu_blocked<LU_NB>(T, m, P.fslab + P.fLU[b], m, piv, shv, sh, ipv, dyn, lp, status + e);
  __syncthreads();
  if (T.member != 0) return;
  if (st) {
    if (threadIdx.x == 0) {
      flag[0] = 1;
      flag[1] = b;
      flag[2] = P.l;
    }
    return;
  }
  // the row swaps of the pivoting, applied in order, as one permutation: row i of P Piv is row
  // perm[i] of Piv; it replaces the swaps in fpiv
  __syncthreads();
  int* sw = pm + m;
  for (int i = threadIdx.x; i < m; i += WG) {
    pm[i] = i;
    sw[i] = piv[i];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int r = 0; r < m; ++r) {
      int p = sw[r];
      if (p != r && p > r && p < m) {
        int t = pm[r];
        pm[r] = pm[p];
        pm[p] = t;
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += WG) piv[i] = pm[i];
}

// Schur update of the coupled blocks: T[p, q] -= A[rows(p), x_b] W_x[:, cols(q)], with the
// column y_b written (not accumulated).  One ST x ST output tile per workgroup; each wave owns
// an (ST/2) x (ST/2) quarter as BL x BL blocks of FP64 MFMA 16x16x4.  The MFMA adds its four
// products to the accumulator one fused multiply-add at a time in ascending k, so every output
// is the ascending-k fused multiply-add sum, exactly as the sequential product.  The tiles of
// the next k chunk are loaded into registers while the current chunk is multiplied from LDS.
// In the precision form (F32) the tiles are converted to FP32 and multiplied with FP32 MFMA
// 16x16x4 (FP32 accumulation); the FP64 block store receives the FP32 products.  K chunks of
// 16 keep the register use low enough for five workgroups per CU, whose prologues, barriers
// and scatter epilogues then overlap the others' MFMA streams.
constexpr int ST = 64, SK = 16, BL = ST / 32;
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
__device__ inline dbl4 mfma16(double a, double b, dbl4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline flt4 mfma16(float a, float b, flt4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
template <bool F32> struct MfmaT { using T = double; using T4 = dbl4; };
template <> struct MfmaT<true> { using T = float; using T4 = flt4; };
template <bool F32>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5)))
k_elim_schur(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys, const int* __restrict__ boxes, int tiles_c) {
  using TT = typename MfmaT<F32>::T;
  using TT4 = typename MfmaT<F32>::T4;
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.y);
  if (P.flag[0]) return;
  int b = boxes[blockIdx.y];
  int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
  int n = P.n[b];
  __shared__ int rstart[28], cstart[28];
  __shared__ TT As[ST][SK + 1];
  __shared__ TT Bs[SK][ST + 1];
  const int* rc = P.grc + (size_t)b * 56;
  if (threadIdx.x <= G) rstart[threadIdx.x] = rc[threadIdx.x];
  else if (threadIdx.x >= 64 && threadIdx.x <= 64 + G) cstart[threadIdx.x - 64] = rc[28 + threadIdx.x - 64];
  __syncthreads();
  int R = rstart[G - 1], C = cstart[G];
  // XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs, so workgroup x
  // runs on XCD x % 8; each XCD takes a contiguous range of this box's tiles, walked in groups
  // of SG tile rows column by column, so the A strips of a group and the W strip of a column
  // stay in that XCD's L2 while they are reused.
  int tiles_r = (R + ST - 1) / ST, tcn = (C + ST - 1) / ST;
  int nt = tiles_r * tcn, per = (nt + 7) / 8;
  int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (blockIdx.x >= 8 * per || t >= nt) return;
  constexpr int SG = 8;
  int grp = t / (SG * tcn), rem = t - grp * SG * tcn;
  int gh = min(SG, tiles_r - grp * SG);
  int tr = grp * SG + rem % gh, tc = rem / gh;
  int r0 = tr * ST, c0 = tc * ST;
  (void)tiles_c;
  int ldw = C + n;
  const double* Cb = P.fslab + P.fC[b];
  const double* W = P.fslab + P.fW[b];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int wr = (wv / 2) * (ST / 2), wc = (wv % 2) * (ST / 2);
  const int fr = lane % 16, fk = lane / 16;
  TT4 acc[BL][BL];
#pragma unroll
  for (int i = 0; i < BL; ++i)
#pragma unroll
    for (int j = 0; j < BL; ++j) acc[i][j] = TT4{0, 0, 0, 0};
  constexpr int NA = ST * SK / WG, NBv = SK * ST / WG;
  TT ra[NA], rb[NBv];
  // A chunk: row r = idx / SK, k = idx % SK; B chunk: k = idx / ST, column = idx % ST
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int idx = threadIdx.x + u * WG;
      int gr = r0 + idx / SK, gk = k0 + idx % SK;
      ra[u] = (gr < R && gk < n) ? (TT)Cb[(size_t)gr * n + gk] : (TT)0;
    }
#pragma unroll
    for (int u = 0; u < NBv; ++u) {
      int idx = threadIdx.x + u * WG;
      int gk = k0 + idx / ST, gc = c0 + idx % ST;
      rb[u] = (gk < n && gc < C) ? (TT)W[(size_t)gk * ldw + gc] : (TT)0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += SK) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int idx = threadIdx.x + u * WG;
      As[idx / SK][idx % SK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NBv; ++u) {
      int idx = threadIdx.x + u * WG;
      Bs[idx / ST][idx % ST] = rb[u];
    }
    __syncthreads();
    if (k0 + SK < n) fetch(k0 + SK);
#pragma unroll
    for (int k4 = 0; k4 < SK; k4 += 4) {
      TT a[BL], bb[BL];
#pragma unroll
      for (int i = 0; i < BL; ++i) a[i] = As[wr + 16 * i + fr][k4 + fk];
#pragma unroll
      for (int j = 0; j < BL; ++j) bb[j] = Bs[k4 + fk][wc + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < BL; ++i)
#pragma unroll
        for (int j = 0; j < BL; ++j) acc[i][j] = mfma16(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  const int64_t* ts = P.tslot + (size_t)b * P.Gmax * P.Gmax;
  // output (lane, q) of block (i, j): column wc + 16 j + lane % 16; row wr + 16 i + lane / 16 + 4 q
  // (FP64 MFMA) or wr + 16 i + 4 (lane / 16) + q (FP32 MFMA)
#pragma unroll
  for (int j = 0; j < BL; ++j) {
    int c = c0 + wc + 16 * j + fr;
    if (c >= C) continue;
    int gc = 0;
    while (cstart[gc + 1] <= c) ++gc;
    int lc = c - cstart[gc];
    int q = P.grp_box[g0 + gc];
    int ldq = P.n[q];
    bool last = gc == G - 1;
#pragma unroll
    for (int i = 0; i < BL; ++i)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        int r = r0 + wr + 16 * i + (F32 ? 4 * fk + qq : fk + 4 * qq);
        if (r >= R) continue;
        int gr = 0;
        while (rstart[gr + 1] <= r) ++gr;
        int lr = r - rstart[gr];
        double* T = P.slab + ts[gr * P.Gmax + gc];
        size_t addr = (size_t)lr * ldq + lc;
        double v = (double)acc[i][j][qq];
        if (last) T[addr] = -v;
        else T[addr] -= v;
      }
  }
}

// W = Piv^{-1} [rhs] for every box of a colour: (m x m, ld m, from k_elim_trsm) times the
// right-hand sides (m x (C + n), ld C + n, from k_elim_gather) into the factor store's W.  The
// tiles of the Schur update: 64 x 64 per workgroup, 2 x 2 blocks of FP64 MFMA 16x16x4 per wave, K
// chunks of 16 through LDS with the next chunk prefetched into registers, XCD-aware tile order;
// every element is the ascending fused multiply-add chain over k from zero.
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5)))
k_elim_wgemm(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys, const int* __restrict__ boxes,
             const double* __restrict__ pws, int64_t pstride, const double* __restrict__ rws, int64_t rstride) {
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.y);
  if (P.flag[0]) return;
  const int b = boxes[blockIdx.y];
  const int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
  const int n = P.n[b], m = n + P.k[b];
  int C = 0;
  for (int g = 0; g < G; ++g) C += grp_rows(P, g, G, b, P.grp_box[g0 + g], P.grp_elim[g0 + g]);
  const int ldw = C + n;
  __shared__ double As[ST][SK + 1];
  __shared__ double Bs[SK][ST + 1];
  const int tiles_r = (m + ST - 1) / ST, tcn = (ldw + ST - 1) / ST;
  const int nt = tiles_r * tcn, per = (nt + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (m == 0 || blockIdx.x >= 8 * per || t >= nt) return;
  constexpr int SG = 8;
  const int grp = t / (SG * tcn), rem = t - grp * SG * tcn;
  const int gh = min(SG, tiles_r - grp * SG);
  const int r0 = (grp * SG + rem % gh) * ST, c0 = (rem / gh) * ST;
  const double* Pinv = pws + (size_t)blockIdx.y * pstride + pstride / 2;
  const double* R = rws + (size_t)blockIdx.y * rstride;
  double* W = P.fslab + P.fW[b];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int wr = (wv / 2) * (ST / 2), wc = (wv % 2) * (ST / 2);
  const int fr = lane % 16, fk = lane / 16;
  dbl4 acc[BL][BL];
#pragma unroll
  for (int i = 0; i < BL; ++i)
#pragma unroll
    for (int j = 0; j < BL; ++j) acc[i][j] = dbl4{0, 0, 0, 0};
  constexpr int NA = ST * SK / WG, NBv = SK * ST / WG;
  double ra[NA], rb[NBv];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int idx = threadIdx.x + u * WG;
      int gr = r0 + idx / SK, gk = k0 + idx % SK;
      ra[u] = (gr < m && gk < m) ? Pinv[(size_t)gr * m + gk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NBv; ++u) {
      int idx = threadIdx.x + u * WG;
      int gk = k0 + idx / ST, gc = c0 + idx % ST;
      rb[u] = (gk < m && gc < ldw) ? R[(size_t)gk * ldw + gc] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += SK) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      int idx = threadIdx.x + u * WG;
      As[idx / SK][idx % SK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NBv; ++u) {
      int idx = threadIdx.x + u * WG;
      Bs[idx / ST][idx % ST] = rb[u];
    }
    __syncthreads();
    if (k0 + SK < m) fetch(k0 + SK);
#pragma unroll
    for (int k4 = 0; k4 < SK; k4 += 4) {
      double a[BL], bb[BL];
#pragma unroll
      for (int i = 0; i < BL; ++i) a[i] = As[wr + 16 * i + fr][k4 + fk];
#pragma unroll
      for (int j = 0; j < BL; ++j) bb[j] = Bs[k4 + fk][wc + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < BL; ++i)
#pragma unroll
        for (int j = 0; j < BL; ++j) acc[i][j] = mfma16(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  // output (lane, q) of block (i, j): row wr + 16 i + lane / 16 + 4 q, column wc + 16 j + lane % 16
#pragma unroll
  for (int i = 0; i < BL; ++i)
#pragma unroll
    for (int j = 0; j < BL; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr + 16 * i + fk + 4 * q, c = c0 + wc + 16 * j + fr;
        if (r < m && c < ldw) W[(size_t)r * ldw + c] = acc[i][j][q];
      }
}

// Piv^{-1} for the pivot block of every box of a colour, with the LU factors of k_elim_lu (row
// permutation in fpiv): the substitution on the columns of the identity, Piv^{-1} =
// U^{-1} L^{-1} P.  One wave owns 16 columns and walks the rows in blocks of 16, left-looking.
// Forward (unit lower L): a block's rows start from the permuted identity, take the terms of
// every earlier row through FP64 MFMA 16x16x4 in ascending column order, then the in-block terms
// one at a time (16 lanes, one column each), so every element is the ascending fused
// multiply-add chain of the forward substitution; the result goes to the workspace X.  Backward
// (upper U): a block's rows take the terms of every later row through MFMA in descending column
// order (four columns per MFMA, highest first), then the in-block terms in descending order and
// the division by the diagonal: the column-oriented back substitution, element by element; the
// result is the inverse, m x m with ld m, after X in the box's workspace.  The wave's stores are
// fenced before its later blocks read them; waves share nothing, so the workgroup never
// synchronises.  W = Piv^{-1} [rhs] is then one product (k_elim_wgemm).
constexpr int TW = 4;  // waves per workgroup
__global__ void __launch_bounds__(TW * WAVE) k_elim_trsm(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys,
                                                         const int* __restrict__ boxes, double* pws, int64_t pstride) {
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.y);
  if (P.flag[0]) return;
  const int b = boxes[blockIdx.y];
  const int n = P.n[b], k = P.k[b], m = n + k;
  const int ldw = m;  // the identity's columns
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int c0 = (blockIdx.x * TW + wv) * 16;
  if (c0 >= ldw || m == 0) return;  // the whole wave
  const int fr = lane % 16, fk = lane / 16;
  const int col = c0 + fr;
  const bool cok = col < ldw;
  const double* A = P.fslab + P.fLU[b];
  const int* perm = P.fpiv + P.fpiv_off[b];
  double* X = pws + (size_t)blockIdx.y * pstride;  // forward results, m x m
  double* W = X + pstride / 2;                     // the inverse, m x m
  __shared__ double xs_all[TW][16][17], ls_all[TW][16][17];
  double(*xs)[17] = xs_all[wv];
  double(*ls)[17] = ls_all[wv];
  const int nblk = (m + 15) / 16;
  // nsteps MFMA steps onto acc; operands of step s from fa(s) / fb(s), eight steps loaded ahead
  constexpr int KC = 8;
  auto gemm = [&](dbl4& acc, int nsteps, auto fa, auto fb) {
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
        if (s0 + u < nsteps) acc = mfma16(ca[u], cb[u], acc);
    }
  };
  // the block's rows and the diagonal 16 x 16 block of the factors, staged in the wave's LDS
  auto stage = [&](const dbl4& acc, int R0, int nr) {
#pragma unroll
    for (int q = 0; q < 4; ++q) xs[fk + 4 * q][fr] = acc[q];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = lane + WAVE * u, i = idx / 16, t = idx % 16;
      ls[i][t] = (i < nr && t < nr) ? A[(size_t)(R0 + i) * m + R0 + t] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
  };
  for (int j = 0; j < nblk; ++j) {
    const int R0 = 16 * j, nr = min(16, m - R0);
    dbl4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int r = R0 + fk + 4 * q;
      acc[q] = (r < m && cok && perm[r] == col) ? 1.0 : 0.0;  // row perm[r] of the identity
    }
    const bool aok = R0 + fr < m;
    const double* Ar = A + (size_t)(R0 + fr) * m;
    // earlier rows t = 0 .. R0-1: step s, slot fk takes t = 4 s + fk
    gemm(acc, R0 / 4, [&](int s) { return aok ? -Ar[4 * s + fk] : 0.0; },
         [&](int s) { return cok ? X[(size_t)(4 * s + fk) * ldw + col] : 0.0; });
    stage(acc, R0, nr);
    if (lane < 16) {
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = xs[r][lane];
#pragma unroll
      for (int r = 1; r < 16; ++r)
#pragma unroll
        for (int t = 0; t < r; ++t)
          if (r < nr) x[r] = fma(-ls[r][t], x[t], x[r]);
      if (cok)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (r < nr) X[(size_t)(R0 + r) * ldw + col] = x[r];
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
  for (int j = nblk - 1; j >= 0; --j) {
    const int R0 = 16 * j, R1 = min(R0 + 16, m), nr = R1 - R0;
    dbl4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int r = R0 + fk + 4 * q;
      acc[q] = (r < m && cok) ? X[(size_t)r * ldw + col] : 0.0;
    }
    const bool aok = R0 + fr < m;
    const double* Ar = A + (size_t)(R0 + fr) * m;
    // later rows t = m-1 down to R1: step s, slot fk takes t = m - 1 - 4 s - fk
    gemm(acc, (m - R1 + 3) / 4,
         [&](int s) {
           int t = m - 1 - 4 * s - fk;
           return (aok && t >= R1) ? -Ar[t] : 0.0;
         },
         [&](int s) {
           int t = m - 1 - 4 * s - fk;
           return (cok && t >= R1) ? W[(size_t)t * ldw + col] : 0.0;
         });
    stage(acc, R0, nr);
    if (lane < 16) {
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = xs[r][lane];
#pragma unroll
      for (int r = 15; r >= 0; --r)
        if (r < nr) {
          double v = x[r];
#pragma unroll
          for (int t = 15; t > r; --t)
            if (t < nr) v = fma(-ls[r][t], x[t], v);
          x[r] = v / ls[r][r];
        }
      if (cok)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (r < nr) W[(size_t)(R0 + r) * ldw + col] = x[r];
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// The same inverse, right-looking: a workgroup of NW waves owns a strip of 16 columns of the
// identity and keeps all of the strip's rows in FP64 MFMA accumulators, row block i (16 rows)
// in wave i mod NW (PMB blocks per wave, so m <= 256 NW).  Forward, block by block: the owner of
// block j, whose rows have taken the terms of every earlier block, adds the in-block terms one
// at a time (16 lanes, one column each) and publishes the finished block in LDS; after one
// workgroup barrier every wave adds the block's terms to its later blocks through MFMA, four
// columns per MFMA in ascending order.  Backward likewise from the last block, with the terms
// of later blocks in descending column order and the division by the diagonal at the end of
// each element's chain; the finished blocks are the rows of the inverse.  Every element thus
// receives exactly the fused multiply-add sequence of the column-oriented substitution (the
// MFMA slots past the matrix add exact zeros), the same as k_elim_trsm, while a strip's chain
// of dependent steps is spread over NW waves and the factors are read once per strip.
// Accumulators are indexed by constants only: a wave's array is rotated by one position each
// time it finishes a block, so the block it works on next is always in position 0 (position p
// holds the wave's block (p + rot) mod PMB).  PMB (blocks per wave) sets the register footprint:
// the host takes the shape with the fewest registers that holds the level's largest block.
template <int NW, int PMB>
__global__ void __launch_bounds__(NW * WAVE) k_elim_pinv(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys,
                                                         const int* __restrict__ boxes, double* pws, int64_t pstride) {
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.y);
  if (P.flag[0]) return;
  const int b = boxes[blockIdx.y];
  const int m = P.n[b] + P.k[b];
  const int c0 = blockIdx.x * 16;
  if (c0 >= m) return;  // the whole workgroup
  const int wv = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int fr = lane % 16, fk = lane / 16;
  const int col = c0 + fr;
  const bool cok = col < m;
  const double* A = P.fslab + P.fLU[b];
  const int* perm = P.fpiv + P.fpiv_off[b];
  double* W = pws + (size_t)blockIdx.y * pstride + pstride / 2;  // the inverse, m x m, ld m
  const int nblk = (m + 15) / 16;
  if (nblk > PMB * NW) return;      // the host sizes the launch so that this never happens
  constexpr int HC = PMB < 8 ? PMB : 8;  // blocks whose factor operands are loaded together
  __shared__ double xs[2][16][17];  // the finished block of the step, alternating with its parity
  __shared__ double ts[16][17];     // the owner's block before its in-block terms
  __shared__ double ls[16][17];     // the diagonal 16 x 16 block of the factors
  dbl4 acc[PMB];
  int rot = 0;
  auto rot_left = [&]() {
    dbl4 t = acc[0];
#pragma unroll
    for (int u = 0; u + 1 < PMB; ++u) acc[u] = acc[u + 1];
    acc[PMB - 1] = t;
    rot = rot + 1 == PMB ? 0 : rot + 1;
  };
  auto rot_right = [&]() {
    dbl4 t = acc[PMB - 1];
#pragma unroll
    for (int u = PMB - 1; u > 0; --u) acc[u] = acc[u - 1];
    acc[0] = t;
    rot = rot == 0 ? PMB - 1 : rot - 1;
  };
  // forward: the rows of the permuted identity (row r holds e_{perm[r]})
#pragma unroll
  for (int u = 0; u < PMB; ++u) {
    const int i = wv + NW * u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * i + fk + 4 * q;
      acc[u][q] = (i < nblk && r < m && cok && perm[r] == col) ? 1.0 : 0.0;
    }
  }
  // the owner's block (position 0) and the diagonal block of the factors into LDS
  auto stage = [&](int R0, int nr) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ts[fk + 4 * q][fr] = acc[0][q];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int idx = lane + WAVE * v, i = idx / 16, t = idx % 16;
      ls[i][t] = (i < nr && t < nr) ? A[(size_t)(R0 + i) * m + R0 + t] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
  };
  int step = 0;
  for (int j = 0; j < nblk; ++j, ++step) {
    const int R0 = 16 * j, nr = min(16, m - R0), p = step & 1;
    if (wv == j % NW) {
      stage(R0, nr);
      if (lane < 16) {
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = ts[r][lane];
#pragma unroll
        for (int r = 1; r < 16; ++r)
#pragma unroll
          for (int t = 0; t < r; ++t)
            if (r < nr) x[r] = fma(-ls[r][t], x[t], x[r]);
#pragma unroll
        for (int r = 0; r < 16; ++r) xs[p][r][lane] = x[r];
      }
      __builtin_amdgcn_wave_barrier();
      // the finished rows stay in the accumulators for the backward pass
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[0][q] = xs[p][fk + 4 * q][fr];
      rot_left();
    }
    __syncthreads();
    double bx[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bx[s] = xs[p][4 * s + fk][fr];
    // later blocks i > j: slot fk of MFMA s takes column R0 + 4 s + fk of the factors
#pragma unroll
    for (int h = 0; h < PMB; h += HC) {
      double la[HC][4];
#pragma unroll
      for (int u = h; u < h + HC; ++u) {
        const int uu = u + rot < PMB ? u + rot : u + rot - PMB;
        const int i = wv + NW * uu, row = 16 * i + fr;
        const bool on = i > j && i < nblk && row < m;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int t = R0 + 4 * s + fk;
          la[u - h][s] = (on && t < m) ? -A[(size_t)row * m + t] : 0.0;
        }
      }
#pragma unroll
      for (int u = h; u < h + HC; ++u) {
        const int uu = u + rot < PMB ? u + rot : u + rot - PMB;
        const int i = wv + NW * uu;
        if (i > j && i < nblk)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[u] = mfma16(la[u - h][s], bx[s], acc[u]);
      }
    }
  }
  // the wave's blocks in descending order: its block u sits in position 0 once rot == u
  for (int j = nblk - 1; j >= 0; --j, ++step) {
    const int R0 = 16 * j, nr = min(16, m - R0), p = step & 1;
    if (wv == j % NW) {
      while (rot != j / NW) rot_right();
      stage(R0, nr);
      if (lane < 16) {
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = ts[r][lane];
#pragma unroll
        for (int r = 15; r >= 0; --r)
          if (r < nr) {
            double v = x[r];
#pragma unroll
            for (int t = 15; t > r; --t)
              if (t < nr) v = fma(-ls[r][t], x[t], v);
            x[r] = v / ls[r][r];
          }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          xs[p][r][lane] = x[r];
          if (cok && r < nr) W[(size_t)(R0 + r) * m + col] = x[r];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (j == 0) break;
    // earlier blocks i < j: slot fk of MFMA s takes column R0 + 15 - 4 s - fk (descending)
    double bx[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bx[s] = xs[p][15 - 4 * s - fk][fr];
#pragma unroll
    for (int h = 0; h < PMB; h += HC) {
      double la[HC][4];
#pragma unroll
      for (int u = h; u < h + HC; ++u) {
        const int uu = u + rot < PMB ? u + rot : u + rot - PMB;
        const int i = wv + NW * uu, row = 16 * i + fr;
        const bool on = i < j && row < m;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int t = R0 + 15 - 4 * s - fk;
          la[u - h][s] = (on && t < m) ? -A[(size_t)row * m + t] : 0.0;
        }
      }
#pragma unroll
      for (int u = h; u < h + HC; ++u) {
        const int uu = u + rot < PMB ? u + rot : u + rot - PMB;
        const int i = wv + NW * uu;
        if (i < j)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[u] = mfma16(la[u - h][s], bx[s], acc[u]);
      }
    }
  }
}

// One 16-wide output slab of an in-place product on MFMA 16x16x4 of precision RT: out = opA opB
// (M x N, K terms), element (i, k) of opA at A[i ai + k ak] and (k, j) of opB at B[k bk + j bj],
// operands converted to RT.  In FP64 every element is the ascending fused multiply-add chain
// from zero over k (the slots past K add exact zeros at its end); in FP32 (the precision
// form) the order inside an MFMA is the hardware's.  The wave computes columns 16 s .. 16 s + 15
// (colslab) or rows 16 s .. 16 s + 15 of out and writes them to dst (ldd, FP64): with up to 8
// tiles of 16 from registers after one pass over K, else tile by tile through its workspace
// tmp (16 max(M, N) entries).  dst may be the operand the slab came from: each output column
// (colslab) or row depends only on the same column or row of that operand, and every read has
// been consumed before the first write.
template <class RT, class TA, class TB>
__device__ inline void wave_xform_slab(int M, int N, int K, const TA* A, int64_t ai, int64_t ak, const TB* B, int64_t bk,
                                       int64_t bj, bool colslab, int s, RT* tmp, double* dst, int64_t ldd) {
  using RT4 = typename MfmaT<sizeof(RT) == 4>::T4;
  const int lane = threadIdx.x % WAVE, fr = lane % 16, fk = lane / 16;
  const int nt = colslab ? (M + 15) / 16 : (N + 15) / 16;
  const int nsteps = (K + 3) / 4;
  constexpr int XT = 8;
  if (nt <= XT) {
    // up to 8 tiles: one pass over K for all of them (the slab's operand read once a step,
    // each tile's accumulator in registers), then the results straight to dst.  Each tile's
    // chain runs over the same steps in the same order as below.
    constexpr int KQ = 4;
    RT4 acc[XT];
#pragma unroll
    for (int t = 0; t < XT; ++t) acc[t] = RT4{0, 0, 0, 0};
    const int RS = 16 * s;  // first row (or column) of the slab
    for (int s0 = 0; s0 < nsteps; s0 += KQ) {
      RT sl[KQ], ot[XT][KQ];
#pragma unroll
      for (int u = 0; u < KQ; ++u) {
        const int k = 4 * (s0 + u) + fk;
        const bool kin = s0 + u < nsteps && k < K;
        // the slab's own operand: B's columns RS.. (colslab) or A's rows RS..
        if (colslab) sl[u] = (kin && RS + fr < N) ? (RT)B[(int64_t)k * bk + (int64_t)(RS + fr) * bj] : (RT)0;
        else sl[u] = (kin && RS + fr < M) ? (RT)A[(int64_t)(RS + fr) * ai + (int64_t)k * ak] : (RT)0;
#pragma unroll
        for (int t = 0; t < XT; ++t)
          if (t < nt) {
            const int o = 16 * t + fr;
            if (colslab) ot[t][u] = (kin && o < M) ? (RT)A[(int64_t)o * ai + (int64_t)k * ak] : (RT)0;
            else ot[t][u] = (kin && o < N) ? (RT)B[(int64_t)k * bk + (int64_t)o * bj] : (RT)0;
          }
      }
#pragma unroll
      for (int u = 0; u < KQ; ++u)
        if (s0 + u < nsteps) {
#pragma unroll
          for (int t = 0; t < XT; ++t)
            if (t < nt) acc[t] = colslab ? mfma16(ot[t][u], sl[u], acc[t]) : mfma16(sl[u], ot[t][u], acc[t]);
        }
    }
    // every read of the slab has been consumed: write it in place
#pragma unroll
    for (int t = 0; t < XT; ++t)
      if (t < nt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = sizeof(RT) == 4 ? 4 * fk + q : fk + 4 * q;
          const int r = (colslab ? 16 * t : RS) + rr, c = (colslab ? RS : 16 * t) + fr;
          if (r < M && c < N) dst[(int64_t)r * ldd + c] = (double)acc[t][q];
        }
      }
    return;
  }
  constexpr int KC = 8;
  for (int t = 0; t < nt; ++t) {
    const int R0 = colslab ? 16 * t : 16 * s, C0 = colslab ? 16 * s : 16 * t;
    const bool aok = R0 + fr < M, bok = C0 + fr < N;
    const TA* Ar = A + (int64_t)(R0 + fr) * ai;
    const TB* Bc = B + (int64_t)(C0 + fr) * bj;
    auto fa = [&](int st) {
      int k = 4 * st + fk;
      return (aok && k < K) ? (RT)Ar[(int64_t)k * ak] : (RT)0;
    };
    auto fb = [&](int st) {
      int k = 4 * st + fk;
      return (bok && k < K) ? (RT)Bc[(int64_t)k * bk] : (RT)0;
    };
    RT4 acc = {0, 0, 0, 0};
    RT pa[KC], pb[KC];
#pragma unroll
    for (int u = 0; u < KC; ++u) {
      pa[u] = u < nsteps ? fa(u) : (RT)0;
      pb[u] = u < nsteps ? fb(u) : (RT)0;
    }
    for (int s0 = 0; s0 < nsteps; s0 += KC) {
      RT ca[KC], cb[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        ca[u] = pa[u];
        cb[u] = pb[u];
      }
      if (s0 + KC < nsteps) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
          int st = s0 + KC + u;
          pa[u] = st < nsteps ? fa(st) : (RT)0;
          pb[u] = st < nsteps ? fb(st) : (RT)0;
        }
      }
#pragma unroll
      for (int u = 0; u < KC; ++u)
        if (s0 + u < nsteps) acc = mfma16(ca[u], cb[u], acc);
    }
    // output (lane, q): row R0 + lane / 16 + 4 q (FP64) or R0 + 4 (lane / 16) + q (FP32),
    // column C0 + lane % 16
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int rr = sizeof(RT) == 4 ? 4 * fk + q : fk + 4 * q;
      int r = R0 + rr, c = C0 + fr;
      if (r < M && c < N) tmp[colslab ? r * 16 + fr : c * 16 + rr] = acc[q];
    }
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  if (colslab) {
    const int w = min(16, N - 16 * s);
    for (int idx = lane; idx < M * 16; idx += WAVE) {
      int f = idx / 16, u = idx % 16;
      if (u < w) dst[(int64_t)f * ldd + 16 * s + u] = (double)tmp[f * 16 + u];
    }
  } else {
    const int w = min(16, M - 16 * s);
    for (int idx = lane; idx < w * N; idx += WAVE) {
      int u = idx / N, f = idx % N;
      dst[(int64_t)(16 * s + u) * ldd + f] = (double)tmp[f * 16 + u];
    }
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}

// The basis changes of a round (rows Z_x: L_x * block; columns y_x: block * R_x^* and the M2M
// block R_x * block), in the precision RT of the compression, one 16-wide slab of one block
// per wave, through wave_xform_slab.  Work items (entry, block, slab group: the slabs g,
// g + sgroups, ...) are spread over all waves of the grid; wstride is each wave's workspace
// (doubles).
template <class RT>
__global__ void __launch_bounds__(WG) k_xform(const LevelPtrs* __restrict__ PP, const XformEntry* __restrict__ xe, int nx, const double* ws,
                                              int64_t wsz, int cap, int maxblk, int sgroups, int cols_side,
                                              double* scratch, int64_t wstride) {
  const int64_t gw = (int64_t)blockIdx.x * (WG / WAVE) + threadIdx.x / WAVE;
  const int64_t nw = (int64_t)gridDim.x * (WG / WAVE);
  RT* tmp = (RT*)(scratch + gw * wstride);
  const size_t c2 = (size_t)cap * cap;
  const int64_t total = (int64_t)nx * maxblk * sgroups;
  for (int64_t item = gw; item < total; item += nw) {
    const int g = (int)(item % sgroups);  // this item's slabs: g, g + sgroups, ...
    const int64_t task = item / sgroups;
    const int t = (int)(task / maxblk), q = (int)(task - (int64_t)t * maxblk);
    const XformEntry X = xe[t];
    const LevelPtrs& P = PP[X.sys];
    const int x = X.x;
    const int nil = P.il_off[x + 1] - P.il_off[x];
    if (q > nil || (q == nil && P.l == 2)) continue;
    const int kold = P.k[x], knew = P.kn[x];
    const int kold1 = kold > 0 ? kold : 1;
    if (!cols_side) {
      const RT* Lm = (const RT*)(ws + (size_t)X.pair * wsz) + (X.side ? 2 * c2 : 0);
      double* B;
      int cols, ld;
      if (q < nil) {
        int c = P.il[P.il_off[x] + q];
        if (c == X.skip) continue;
        B = P.slab + P.il_slot[P.il_off[x] + q];
        cols = P.k[c];
        ld = P.n[c];
      } else {
        B = P.slab + P.l2l_off[x];
        cols = P.kP[x];
        ld = cols;
      }
      for (int s = g; 16 * s < cols; s += sgroups)
        wave_xform_slab<RT>(knew, cols, kold, Lm, kold1, 1, B, ld, 1, true, s, tmp, B, ld);
    } else {
      const RT* Rm = (const RT*)(ws + (size_t)X.pair * wsz) + (X.side ? 3 * c2 : c2);
      if (q < nil) {
        int dbox = P.il[P.il_off[x] + q];
        if (dbox == X.skip) continue;
        double* B = P.slab + P.il_slot[P.il_tr[P.il_off[x] + q]];
        int rows = P.kn[dbox], ld = P.n[x];
        for (int s = g; 16 * s < rows; s += sgroups)
          wave_xform_slab<RT>(rows, knew, kold, B, ld, 1, Rm, 1, kold1, false, s, tmp, B, ld);
      } else {
        double* B = P.slab + P.m2m_off[x];
        int cols = P.kP[x];
        for (int s = g; 16 * s < cols; s += sgroups)
          wave_xform_slab<RT>(knew, cols, kold, Rm, kold1, 1, B, cols, 1, true, s, tmp, B, cols);
      }
    }
  }
}

// New rows Z_b: (Z_b, cols(q)) = W_z[:, cols(q)] for every coupled column group.
__global__ void __launch_bounds__(WG) k_elim_zrow(const LevelPtrs* __restrict__ PP, const int* __restrict__ bsys,
                                                 const int* __restrict__ boxes) {
  const LevelPtrs& P = sys_ptrs(PP, bsys, blockIdx.x);
  if (P.flag[0]) return;
  int b = boxes[blockIdx.x];
  int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
  int n = P.n[b], k = P.k[b];
  int C = 0;
  for (int g = 0; g < G; ++g) C += grp_rows(P, g, G, b, P.grp_box[g0 + g], P.grp_elim[g0 + g]);
  int ldw = C + n;
  const double* W = P.fslab + P.fW[b];
  int co = 0;
  for (int g = 0; g < G; ++g) {
    int q = P.grp_box[g0 + g];
    int cd = grp_rows(P, g, G, b, q, P.grp_elim[g0 + g]);
    double* T = P.slab + near_entry(P, b, q);
    int ldq = P.n[q];
    for (int idx = threadIdx.x; idx < k * cd; idx += WG) {
      int r = idx / cd, c = idx - r * cd;
      T[(size_t)r * ldq + c] = W[(size_t)(n + r) * ldw + co + c];
    }
    co += cd;
  }
}

// ------------------------------------------------------------------------------------------
// Leaf level of the extended system: P2P near blocks, U_b = V_b, L2L / M2M, M2L
// ------------------------------------------------------------------------------------------
__global__ void k_fill_near(KernelDesc K, const double* pts, int d, const int* nbr_off, const int* nbr,
                            const int* box_off, const int* n, const int64_t* slot, double* slab) {
  int b = blockIdx.y;
  int e = nbr_off[b] + blockIdx.x;
  if (e >= nbr_off[b + 1]) return;
  int q = nbr[e];
  int np = n[b], nq = n[q];
  double* o = slab + slot[e];
  int p0 = box_off[b], q0 = box_off[q];
  for (int idx = threadIdx.x; idx < np * nq; idx += WG) {
    int r = idx / nq, c = idx - r * nq;
    o[idx] = kernel_entry(K, pts, d, p0 + r, q0 + c);
  }
}

// copy a compact k_r x k_c block into a slot with leading dimension ld
__global__ void k_copy_blocks(const double* src, const int64_t* src_off, const int* rows, const int* cols,
                              const int64_t* dst_off, const int* ld, double* dst) {
  int e = blockIdx.x;
  int R = rows[e], C = cols[e], L = ld[e];
  const double* s = src + src_off[e];
  double* o = dst + dst_off[e];
  for (int idx = threadIdx.x; idx < R * C; idx += WG) {
    int r = idx / C, c = idx - r * C;
    o[(size_t)r * L + c] = s[idx];
  }
}

// ------------------------------------------------------------------------------------------
// level activation: near blocks of level l-1 from the Z^{(l)} x y^{(l)} blocks of level l
// ------------------------------------------------------------------------------------------
struct RepackArgs {
  int d;
  // destination level
  const int* nbr_off;
  const int* nbr;
  const int* n;          // n_P
  const int64_t* near_slot;
  double* slab;
  // source level (children)
  const int* ck;         // final child ranks
  const int* cn;
  const int* cnbr_off;
  const int* cnbr;
  const int64_t* cnear_slot;
  const int* cil_off;
  const int* cil;
  const int64_t* cil_slot;
  const double* cslab;
};

__global__ void __launch_bounds__(WG) k_repack_near(RepackArgs a) {
  int Pb = blockIdx.y;
  int e = a.nbr_off[Pb] + blockIdx.x;
  if (e >= a.nbr_off[Pb + 1]) return;
  int Q = a.nbr[e];
  int nch = 1 << a.d;
  double* out = a.slab + a.near_slot[e];
  int ldo = a.n[Q];
  int ro = 0;
  for (int ci = 0; ci < nch; ++ci) {
    int c = Pb * nch + ci;
    int kc = a.ck[c];
    int co = 0;
    for (int ei = 0; ei < nch; ++ei) {
      int f = Q * nch + ei;
      int kf = a.ck[f];
      const double* src = nullptr;
      int lds = a.cn[f];
      for (int t = a.cnbr_off[c]; t < a.cnbr_off[c + 1]; ++t)
        if (a.cnbr[t] == f) { src = a.cslab + a.cnear_slot[t]; break; }
      if (!src)
        for (int t = a.cil_off[c]; t < a.cil_off[c + 1]; ++t)
          if (a.cil[t] == f) { src = a.cslab + a.cil_slot[t]; break; }
      if (src)
        for (int idx = threadIdx.x; idx < kc * kf; idx += WG) {
          int r = idx / kf, cc = idx - r * kf;
          out[(size_t)(ro + r) * ldo + co + cc] = src[(size_t)r * lds + cc];
        }
      co += kf;
    }
    ro += kc;
  }
}

// stacked U_P / V_P from the children's L2L / M2M blocks
__global__ void k_stack_basis(int d, const int* ck, const int* kPc /* child's kP */, const int64_t* cl2l, const int64_t* cm2m,
                              const double* cslab, const int* n, const int64_t* U_off, const int64_t* V_off, double* slab) {
  int Pb = blockIdx.x;
  int nch = 1 << d;
  int nP = n[Pb];
  int ro = 0;
  for (int ci = 0; ci < nch; ++ci) {
    int c = Pb * nch + ci;
    int kc = ck[c], kp = kPc[c];
    const double* L2 = cslab + cl2l[c];
    const double* M2 = cslab + cm2m[c];
    for (int idx = threadIdx.x; idx < kc * kp; idx += WG) {
      int r = idx / kp, cc = idx - r * kp;
      slab[U_off[Pb] + (size_t)(ro + r) * nP + cc] = L2[(size_t)r * kp + cc];
      slab[V_off[Pb] + (size_t)(ro + r) * nP + cc] = M2[(size_t)r * kp + cc];
    }
    ro += kc;
  }
}

__global__ void k_gather_top(int nb, const int* k, const int* n, const int* koff, const int* nbr_off, const int* nbr,
                             const int64_t* near_slot, const int* il_off, const int* il, const int64_t* il_slot,
                             const double* slab, double* top, int K) {
  int a = blockIdx.x, bq = blockIdx.y;
  int ka = k[a], kb = k[bq];
  const double* src = nullptr;
  for (int t = nbr_off[a]; t < nbr_off[a + 1]; ++t)
    if (nbr[t] == bq) { src = slab + near_slot[t]; break; }
  if (!src)
    for (int t = il_off[a]; t < il_off[a + 1]; ++t)
      if (il[t] == bq) { src = slab + il_slot[t]; break; }
  int ld = n[bq];
  for (int idx = threadIdx.x; idx < ka * kb; idx += WG) {
    int r = idx / kb, c = idx - r * kb;
    top[(size_t)(koff[a] + r) * K + koff[bq] + c] = src ? src[(size_t)r * ld + c] : 0.0;
  }
}

// Blocked LU with row partial pivoting of the dense level-2 system.  Every element receives
// its updates fma(-l_ik, u_kj, a_ij) in ascending k, exactly as in the unblocked algorithm,
// so the factors equal those of a column-by-column elimination.
constexpr int PT = 1024, PNB = 64;
__global__ void __launch_bounds__(PT) k_lu_panel(double* A, int K, int k0, int nb, int* ipiv, int* flag) {
  __shared__ ValIdx shv[PT / WAVE + 1];
  if (flag[0]) return;
  for (int k = k0; k < k0 + nb; ++k) {
    ValIdx best{-1.0, INT_MAX};
    for (int i = k + (int)threadIdx.x; i < K; i += PT) {
      ValIdx c{fabs(A[(size_t)i * K + k]), i};
      if (vi_better(c, best)) best = c;
    }
    best = wg_argmax<PT>(best, shv);
    if (best.v == 0.0) {
      if (threadIdx.x == 0) { flag[0] = 1; flag[1] = -1; flag[2] = 1; }
      return;
    }
    int p = best.i;
    if (threadIdx.x == 0) ipiv[k] = p;
    if (p != k)
      for (int j = k0 + (int)threadIdx.x; j < k0 + nb; j += PT) {
        double a = A[(size_t)k * K + j];
        A[(size_t)k * K + j] = A[(size_t)p * K + j];
        A[(size_t)p * K + j] = a;
      }
    __syncthreads();
    double piv = A[(size_t)k * K + k];
    for (int i = k + 1 + (int)threadIdx.x; i < K; i += PT) A[(size_t)i * K + k] /= piv;
    __syncthreads();
    int w = k0 + nb - k - 1;
    if (w > 0)
      for (int idx = threadIdx.x; idx < (K - k - 1) * w; idx += PT) {
        int i = k + 1 + idx / w, j = k + 1 + idx % w;
        A[(size_t)i * K + j] = fma(-A[(size_t)i * K + k], A[(size_t)k * K + j], A[(size_t)i * K + j]);
      }
    __syncthreads();
  }
}
// row swaps of the panel applied to the columns outside it
__global__ void k_lu_swaps(double* A, int K, int k0, int nb, const int* ipiv, const int* flag) {
  if (flag[0]) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K || (j >= k0 && j < k0 + nb)) return;
  for (int k = k0; k < k0 + nb; ++k) {
    int p = ipiv[k];
    if (p != k) {
      double a = A[(size_t)k * K + j];
      A[(size_t)k * K + j] = A[(size_t)p * K + j];
      A[(size_t)p * K + j] = a;
    }
  }
}
// U12 = L11^{-1} A12 (unit lower), one column per thread
__global__ void k_lu_u12(double* A, int K, int k0, int nb, const int* flag) {
  if (flag[0]) return;
  int j = k0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  for (int k = k0; k < k0 + nb; ++k) {
    double u = A[(size_t)k * K + j];
    for (int i = k + 1; i < k0 + nb; ++i) A[(size_t)i * K + j] = fma(-A[(size_t)i * K + k], u, A[(size_t)i * K + j]);
  }
}
// A22 -= L21 U12, each element accumulating the panel's updates in ascending k
__global__ void __launch_bounds__(256) k_lu_a22(double* A, int K, int k0, int nb, const int* flag) {
  if (flag[0]) return;
  __shared__ double Ls[64][PNB + 1];
  __shared__ double Us[PNB][64 + 1];
  int r0 = k0 + nb + blockIdx.y * 64, c0 = k0 + nb + blockIdx.x * 64;
  int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  for (int idx = threadIdx.x; idx < 64 * nb; idx += 256) {
    int r = idx / nb, kk = idx % nb;
    Ls[r][kk] = (r0 + r < K) ? A[(size_t)(r0 + r) * K + k0 + kk] : 0.0;
  }
  for (int idx = threadIdx.x; idx < nb * 64; idx += 256) {
    int kk = idx / 64, c = idx % 64;
    Us[kk][c] = (c0 + c < K) ? A[(size_t)(k0 + kk) * K + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int a = 0; a < 4; ++a) {
    int r = r0 + ty * 4 + a;
    if (r >= K) continue;
    for (int b = 0; b < 4; ++b) {
      int c = c0 + tx * 4 + b;
      if (c >= K) continue;
      double acc = A[(size_t)r * K + c];
      for (int kk = 0; kk < nb; ++kk) acc = fma(-Ls[ty * 4 + a][kk], Us[kk][tx * 4 + b], acc);
      A[(size_t)r * K + c] = acc;
    }
  }
}

static void top_lu(double* A, int K, int* ipiv, int* flag, hipStream_t st) {
  for (int k0 = 0; k0 < K; k0 += PNB) {
    int nb = std::min(PNB, K - k0);
    hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(PT), 0, st, A, K, k0, nb, ipiv, flag);
    hipLaunchKernelGGL(k_lu_swaps, dim3((K + 255) / 256), dim3(256), 0, st, A, K, k0, nb, ipiv, flag);
    int rest = K - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_lu_u12, dim3((rest + 255) / 256), dim3(256), 0, st, A, K, k0, nb, flag);
      unsigned t = (unsigned)((rest + 63) / 64);
      hipLaunchKernelGGL(k_lu_a22, dim3(t, t), dim3(256), 0, st, A, K, k0, nb, flag);
    }
  }
}

// ------------------------------------------------------------------------------------------
// host orchestration
// ------------------------------------------------------------------------------------------
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
static void launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{AIFMM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

static LevelPtrs ptrs(aifmm_system& s, int l) {
  LevelDev& v = s.lev[l];
  LevelPtrs P;
  P.l = l;
  P.nb = v.nb;
  P.d = s.d;
  P.n = v.d_n.p;
  P.k = v.d_k.p;
  P.kn = v.d_kn.p;
  P.nbr_off = v.d_nbr_off.p;
  P.nbr = v.d_nbr.p;
  P.il_off = v.d_il_off.p;
  P.il = v.d_il.p;
  P.il_tr = v.d_il_tr.p;
  P.p2_off = v.d_p2_off.p;
  P.p2 = v.d_p2.p;
  P.grp_off = v.d_grp_off.p;
  P.grp_box = v.d_grp_box.p;
  P.grp_elim = v.d_grp_elim.p;
  P.slab = v.slab.p;
  P.near_slot = v.d_near_slot.p;
  P.p2_slot = v.d_p2_slot.p;
  P.il_slot = v.d_il_slot.p;
  P.U_off = v.d_U_off.p;
  P.V_off = v.d_V_off.p;
  P.l2l_off = v.d_l2l_off.p;
  P.m2m_off = v.d_m2m_off.p;
  P.kP = v.d_kP.p;
  P.tslot = v.d_tslot.p;
  P.Gmax = v.Gmax;
  P.fslab = v.fslab.p;
  P.fLU = v.d_fLU.p;
  P.fC = v.d_fC.p;
  P.fW = v.d_fW.p;
  P.fpiv = v.d_fpiv.p;
  P.fpiv_off = v.d_fpiv_off.p;
  P.grc = v.d_grc.p;
  return P;
}

static int find_in(const std::vector<int>& off, const std::vector<int>& val, int b, int q) {
  auto beg = val.begin() + off[b], end = val.begin() + off[b + 1];
  auto it = std::lower_bound(beg, end, q);
  if (it == end || *it != q) return -1;
  return (int)(it - val.begin());
}

// Allocate and fill the live block store of level l.
static void activate_level(aifmm_system& s, int l) {
  hipStream_t st = s.stream;
  int d = s.d, L = s.L;
  LevelDev& lv = s.lev[l];
  LevelPlan& P = s.plan[l];
  int nb = lv.nb;
  // sizes
  lv.n.assign(nb, 0);
  if (l == L) {
    for (int b = 0; b < nb; ++b) lv.n[b] = s.leaf_off[b + 1] - s.leaf_off[b];
  } else {
    LevelDev& dn = s.lev[l + 1];
    for (int b = 0; b < nb; ++b)
      for (int ch = 0; ch < (1 << d); ++ch) lv.n[b] += dn.kfin[(b << d) | ch];
  }
  for (int b = 0; b < nb; ++b)
    if (lv.knn[b] > lv.n[b])
      throw Error{AIFMM_ERR_CAPACITY, "NNCA rank " + std::to_string(lv.knn[b]) + " above box size " +
                                          std::to_string(lv.n[b]) + " at level " + std::to_string(l) + " box " +
                                          std::to_string(b)};
  lv.d_n.upload(lv.n, st);
  lv.nmax = 1;
  for (int b = 0; b < nb; ++b) lv.nmax = std::max(lv.nmax, lv.n[b]);
  std::vector<int> kP(nb, 0);
  if (l > 2)
    for (int b = 0; b < nb; ++b) kP[b] = s.lev[l - 1].knn[b >> d];
  lv.d_kP.upload(kP, st);
  // slab layout
  int64_t off = 0;
  auto take = [&](int64_t cnt) { int64_t o = off; off += (cnt + 1) & ~int64_t(1); return o; };
  std::vector<int64_t> near(P.nbr.size()), p2s(P.p2.size()), ils(P.il.size()), Uo(nb), Vo(nb), l2l(nb), m2m(nb);
  for (int b = 0; b < nb; ++b) {
    for (int e = P.nbr_off[b]; e < P.nbr_off[b + 1]; ++e) near[e] = take((int64_t)lv.n[b] * lv.n[P.nbr[e]]);
    for (int e = P.p2_off[b]; e < P.p2_off[b + 1]; ++e) p2s[e] = take((int64_t)lv.n[b] * lv.n[P.p2[e]]);
    for (int e = P.il_off[b]; e < P.il_off[b + 1]; ++e) ils[e] = take((int64_t)lv.n[b] * lv.n[P.il[e]]);
    Uo[b] = take((int64_t)lv.n[b] * lv.n[b]);
    Vo[b] = take((int64_t)lv.n[b] * lv.n[b]);
    l2l[b] = take((int64_t)lv.n[b] * kP[b]);
    m2m[b] = take((int64_t)lv.n[b] * kP[b]);
  }
  lv.slab.alloc(off);
  lv.slab.zero(st);
  lv.d_near_slot.upload(near, st);
  lv.d_p2_slot.upload(p2s, st);
  lv.d_il_slot.upload(ils, st);
  lv.d_U_off.upload(Uo, st);
  lv.d_V_off.upload(Vo, st);
  lv.d_l2l_off.upload(l2l, st);
  lv.d_m2m_off.upload(m2m, st);
  // Schur target table
  lv.Gmax = 1;
  for (int b = 0; b < nb; ++b) lv.Gmax = std::max(lv.Gmax, P.grp_off[b + 1] - P.grp_off[b]);
  int Gm = lv.Gmax;
  std::vector<int64_t> ts((size_t)nb * Gm * Gm, -1);
  for (int b = 0; b < nb; ++b) {
    int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
    for (int gr = 0; gr < G; ++gr)
      for (int gc = 0; gc < G; ++gc) {
        int p = P.grp_box[g0 + gr], q = P.grp_box[g0 + gc];
        int dist = cheb(&P.coord[p * 3], &P.coord[q * 3], d);
        int64_t o = -1;
        int ix;
        if (dist <= 1) { ix = find_in(P.nbr_off, P.nbr, p, q); if (ix >= 0) o = near[ix]; }
        else if (P.grp_elim[g0 + gr] && P.grp_elim[g0 + gc]) { ix = find_in(P.il_off, P.il, p, q); if (ix >= 0) o = ils[ix]; }
        else { ix = find_in(P.p2_off, P.p2, p, q); if (ix >= 0) o = p2s[ix]; }
        if (o < 0) throw Error{AIFMM_ERR_STATE, "missing Schur target slot"};
        ts[((size_t)b * Gm + gr) * Gm + gc] = o;
      }
  }
  lv.d_tslot.upload(ts, st);
  lv.d_grc.alloc((size_t)nb * 56);
  // factor store
  lv.fLU.assign(nb, 0);
  lv.fPx.assign(nb, 0);
  lv.fC.assign(nb, 0);
  lv.fW.assign(nb, 0);
  lv.Rcap.assign(nb, 0);
  lv.Ccap.assign(nb, 0);
  std::vector<int64_t> fpo(nb);
  int64_t fo = 0, po = 0;
  lv.Rmax = lv.Cmax = 0;
  for (int b = 0; b < nb; ++b) {
    int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
    int Rc = 0;
    for (int g = 0; g < G - 1; ++g) Rc += lv.n[P.grp_box[g0 + g]];
    int Cc = Rc + lv.n[b];
    int mc = 2 * lv.n[b];
    lv.Rcap[b] = Rc;
    lv.Ccap[b] = Cc;
    lv.Rmax = std::max(lv.Rmax, Rc);
    lv.Cmax = std::max(lv.Cmax, Cc + lv.n[b]);
    lv.fLU[b] = fo; fo += ((int64_t)mc * mc + 1) & ~int64_t(1);
    lv.fC[b] = fo; fo += ((int64_t)Rc * lv.n[b] + 1) & ~int64_t(1);
    lv.fW[b] = fo; fo += ((int64_t)mc * (Cc + lv.n[b]) + 1) & ~int64_t(1);
    fpo[b] = po; po += mc;
  }
  lv.fslab.alloc(fo);
  lv.d_fLU.upload(lv.fLU, st);
  lv.d_fC.upload(lv.fC, st);
  lv.d_fW.upload(lv.fW, st);
  lv.d_fpiv_off.upload(fpo, st);
  lv.d_fpiv.alloc(std::max<int64_t>(1, po));
  // ranks: the NNCA ranks
  lv.d_kn.upload(lv.knn, st);
  lv.d_k.upload(lv.knn, st);

  // contents
  if (l == L) {
    std::vector<int> box_off(nb + 1);
    for (int b = 0; b <= nb; ++b) box_off[b] = s.leaf_off[b];
    DBuf<int> d_box_off;
    d_box_off.upload(box_off, st);
    int maxn = 0;
    for (int b = 0; b < nb; ++b) maxn = std::max(maxn, P.nbr_off[b + 1] - P.nbr_off[b]);
    hipLaunchKernelGGL(k_fill_near, dim3(maxn, nb), dim3(WG), 0, st, s.K, s.d_pts.p, d, lv.d_nbr_off.p, lv.d_nbr.p,
                       d_box_off.p, lv.d_n.p, lv.d_near_slot.p, lv.slab.p);
    launch_check("fill near");
    AIFMM_HIP(hipStreamSynchronize(st));
  } else {
    LevelDev& dn = s.lev[l + 1];
    RepackArgs ra{d, lv.d_nbr_off.p, lv.d_nbr.p, lv.d_n.p, lv.d_near_slot.p, lv.slab.p, dn.d_k.p, dn.d_n.p,
                  dn.d_nbr_off.p, dn.d_nbr.p, dn.d_near_slot.p, dn.d_il_off.p, dn.d_il.p, dn.d_il_slot.p, dn.slab.p};
    int maxn = 0;
    for (int b = 0; b < nb; ++b) maxn = std::max(maxn, P.nbr_off[b + 1] - P.nbr_off[b]);
    hipLaunchKernelGGL(k_repack_near, dim3(maxn, nb), dim3(WG), 0, st, ra);
    hipLaunchKernelGGL(k_stack_basis, dim3(nb), dim3(WG), 0, st, d, dn.d_k.p, dn.d_kP.p, dn.d_l2l_off.p, dn.d_m2m_off.p,
                       dn.slab.p, lv.d_n.p, lv.d_U_off.p, lv.d_V_off.p, lv.slab.p);
    launch_check("repack");
  }
  // M2L blocks from NNCA
  {
    int ne = (int)P.il.size();
    if (ne) {
      std::vector<int> rows(ne), cols(ne), ld(ne);
      for (int b = 0; b < nb; ++b)
        for (int e = P.il_off[b]; e < P.il_off[b + 1]; ++e) {
          rows[e] = lv.knn[b];
          cols[e] = lv.knn[P.il[e]];
          ld[e] = lv.n[P.il[e]];
        }
      DBuf<int> dr, dc, dl;
      dr.upload(rows, st);
      dc.upload(cols, st);
      dl.upload(ld, st);
      hipLaunchKernelGGL(k_copy_blocks, dim3(ne), dim3(WG), 0, st, lv.d_m2l_nn.p, lv.d_m2l_nn_off.p, dr.p, dc.p,
                         lv.d_il_slot.p, dl.p, lv.slab.p);
      launch_check("m2l copy");
      AIFMM_HIP(hipStreamSynchronize(st));
    }
  }
  // leaf bases U = V from NNCA; L2L / M2M rows from the parent's NNCA operator
  {
    std::vector<int64_t> so, dof;
    std::vector<int> rows, cols, ld;
    if (l == L)
      for (int b = 0; b < nb; ++b) {
        so.push_back(lv.Unn_off[b]); dof.push_back(Uo[b]); rows.push_back(lv.n[b]); cols.push_back(lv.knn[b]); ld.push_back(lv.n[b]);
        so.push_back(lv.Unn_off[b]); dof.push_back(Vo[b]); rows.push_back(lv.n[b]); cols.push_back(lv.knn[b]); ld.push_back(lv.n[b]);
      }
    if (!so.empty()) {
      DBuf<int64_t> dso, ddo;
      DBuf<int> dr, dc, dl;
      dso.upload(so, st); ddo.upload(dof, st); dr.upload(rows, st); dc.upload(cols, st); dl.upload(ld, st);
      hipLaunchKernelGGL(k_copy_blocks, dim3((unsigned)so.size()), dim3(WG), 0, st, lv.d_Unn.p, dso.p, dr.p, dc.p, ddo.p,
                         dl.p, lv.slab.p);
      launch_check("leaf bases");
      AIFMM_HIP(hipStreamSynchronize(st));
    }
    if (l > 2) {
      LevelDev& up = s.lev[l - 1];
      so.clear(); dof.clear(); rows.clear(); cols.clear(); ld.clear();
      for (int b = 0; b < nb; ++b) {
        int Pb = b >> d;
        int ro = 0;
        for (int ch = 0; ch < (b & ((1 << d) - 1)); ++ch) ro += lv.knn[(Pb << d) | ch];
        int64_t src = up.Unn_off[Pb] + (int64_t)ro * up.knn[Pb];
        so.push_back(src); dof.push_back(l2l[b]); rows.push_back(lv.knn[b]); cols.push_back(kP[b]); ld.push_back(kP[b]);
        so.push_back(src); dof.push_back(m2m[b]); rows.push_back(lv.knn[b]); cols.push_back(kP[b]); ld.push_back(kP[b]);
      }
      DBuf<int64_t> dso, ddo;
      DBuf<int> dr, dc, dl;
      dso.upload(so, st); ddo.upload(dof, st); dr.upload(rows, st); dc.upload(cols, st); dl.upload(ld, st);
      hipLaunchKernelGGL(k_copy_blocks, dim3((unsigned)so.size()), dim3(WG), 0, st, up.d_Unn.p, dso.p, dr.p, dc.p, ddo.p,
                         dl.p, lv.slab.p);
      launch_check("l2l/m2m");
      AIFMM_HIP(hipStreamSynchronize(st));
    }
  }
  AIFMM_HIP(hipStreamSynchronize(st));
}

// Algorithmic work of the level's compressions from the decision log (launch order; ranks
// before each compression replayed from the NNCA ranks), and the pivot-step chains of its
// rounds: a P2P compression runs the chains RRQR1 -> RRQR3 and RRQR2 -> RRQR4, a P2L one RRQR5
// and RRQR6, on two half-teams when the team is split (else one after the other).
static void count_compress(aifmm_system& s, int l, const std::vector<int64_t>& r_off, size_t t0) {
  LevelDev& lv = s.lev[l];
  LevelStats& ls = s.stats.lvl[l];
  std::vector<int> k(lv.knn);
  auto rrqr = [](double m, double n, double r) {
    double f = 0;
    for (double q = 0; q < r; ++q) f += 4.0 * (m - q) * (n - q);
    return f;
  };
  auto formq = [](double m, double r, double q) { return 4.0 * m * q * r; };
  auto gemm = [](double a, double b, double c) { return 2.0 * a * b * c; };
  for (size_t round = 0; round + 1 < r_off.size(); ++round) {
    double crit = 0;
    for (int64_t q = r_off[round]; q < r_off[round + 1]; ++q) {
      const TraceRec& t = s.trace[t0 + q];
      const int i = t.i, j = t.partner;
      const double ni = lv.n[i], nj = lv.n[j], ki = k[i], kj = k[j];
      const double r1 = t.r[0], r2 = t.r[1], r3 = t.r[2], r4 = t.r[3], kin = t.r[4], kjn = t.r[5];
      double f = 0, ca, cb;
      if (t.kind == 0) {
        f += rrqr(ni, ki + nj, r1) + rrqr(nj, kj + ni, r2) + rrqr(nj, kj + r1, r3) + rrqr(ni, ki + r2, r4);
        f += formq(ni, r1, r1) + formq(nj, r2, r2) + formq(ni, r1, kin - r1) + formq(ni, r4, kin);
        f += formq(nj, r2, kjn - r2) + formq(nj, r3, kjn);
        f += gemm(nj, r1, ni) + gemm(ni, r2, nj);
        f += 2 * gemm(kin, ki, ni) + 2 * gemm(kjn, kj, nj);
        f += gemm(kin, nj, ni) + gemm(kjn, kin, nj) + gemm(kin, kj, ki) + gemm(kin, kjn, kj);
        f += gemm(kjn, ni, nj) + gemm(kin, kjn, ni) + gemm(kjn, ki, kj) + gemm(kjn, kin, ki);
        ca = r1 + r3;
        cb = r2 + r4;
        k[i] = (int)kin;
        k[j] = (int)kjn;
      } else {
        const double kr = kj;  // the eliminated partner's rank (frozen)
        f += rrqr(ni, ki + kr, r1) + rrqr(ni, ki + kr, r2) + formq(ni, r1, kin) + formq(ni, r2, kin);
        f += 2 * gemm(kin, ki, ni) + gemm(kr, kin, ki) + gemm(kr, kin, ni) + gemm(kin, kr, ki) + gemm(kin, kr, ni);
        ca = r1;
        cb = r2;
        k[i] = (int)kin;
      }
      ls.compress_flops += f;
      ls.pivot_steps += ca + cb;
      crit = std::max(crit, std::max(ca, cb));  // the two chains overlap on split teams
    }
    ls.crit_steps += crit;
    ls.rounds += 1;
  }
  ls.compressions += (double)(r_off.back() - r_off.front());
}

static void count_flops(aifmm_system& s, int l) {
  LevelDev& lv = s.lev[l];
  LevelPlan& P = s.plan[l];
  LevelStats& ls = s.stats.lvl[l];
  ls.boxes = lv.nb;
  for (int b = 0; b < lv.nb; ++b) {
    int g0 = P.grp_off[b], G = P.grp_off[b + 1] - g0;
    double R = 0, C = 0;
    for (int g = 0; g < G; ++g) {
      int q = P.grp_box[g0 + g];
      double dm = (g == G - 1) ? lv.kfin[b] : (P.grp_elim[g0 + g] ? lv.kfin[q] : lv.n[q]);
      if (g < G - 1) R += dm;
      C += dm;
    }
    double n = lv.n[b], m = lv.n[b] + lv.kfin[b];
    s.stats.schur_flops += 2.0 * R * n * C;
    s.stats.schur_bytes += 8.0 * (R * n + n * C + 2.0 * R * C);
    s.stats.trsm_flops += 2.0 * m * m * m + 2.0 * m * m * (C + n);
    s.stats.lu_flops += 2.0 * m * m * m / 3.0;
    ls.schur_flops += 2.0 * R * n * C;
    ls.schur_bytes += 8.0 * (R * n + n * C + 2.0 * R * C);
    ls.trsm_flops += 2.0 * m * m * C;
    ls.trsm_flops_impl += 2.0 * m * m * m + 2.0 * m * m * (C + n);
    ls.lu_flops += 2.0 * m * m * m / 3.0;
  }
}

// largest half-team of a compression (a whole team has at most 128 members)
static int team_max() {
  const char* v = getenv("AIFMM_TEAM_MAX");
  int g = v && *v ? atoi(v) : 64;
  return std::max(1, std::min(64, g));
}

// largest team of workgroups factoring one pivot block
static int lu_team_max() {
  const char* v = getenv("AIFMM_LU_TEAM_MAX");
  int g = v && *v ? atoi(v) : 64;
  return std::max(1, std::min(256, g));
}

// rows per lane of the compression's register column tier for boxes of up to cap rows: the
// smallest compiled size holding cap rows in a 16-lane group, 0 (no register tier) beyond
// 1024 rows or when switched off
static int reg_rows(int cap) {
  const char* v = getenv("AIFMM_NO_REG_COLUMNS");
  if (v && *v && *v != '0') return 0;
  for (int r : {16, 32, 40, 64})
    if (16 * r >= cap) return r;
  return 0;
}

template <class RT>
static const void* compress_fn(int rmax) {
  switch (rmax) {
    case 16: return (const void*)k_compress<RT, 16>;
    case 32: return (const void*)k_compress<RT, 32>;
    case 40: return (const void*)k_compress<RT, 40>;
    case 64: return (const void*)k_compress<RT, 64>;
    default: return (const void*)k_compress<RT, 0>;
  }
}
// register slots of the pivoted QR's tier for rmax rows a lane
template <class RT>
static int reg_slots_of(int rmax) {
  switch (rmax) {
    case 16: return reg_slots<16, RT>();
    case 32: return reg_slots<32, RT>();
    case 40: return reg_slots<40, RT>();
    case 64: return reg_slots<64, RT>();
    default: return 0;
  }
}

static bool lds_off() {
  const char* v = getenv("AIFMM_NO_LDS_COLUMNS");
  return v && *v && *v != '0';
}

static bool team_off() {
  const char* v = getenv("AIFMM_NO_TEAMS");
  return v && *v && *v != '0';
}

// pivot-block LU panels factored in place in device memory, never staged in LDS
static bool lu_panels_off() {
  const char* v = getenv("AIFMM_NO_LDS_PANELS");
  return v && *v && *v != '0';
}

// Shape of the right-looking pivot-block inverse for pivot blocks of up to maxmc rows and
// `strips` strips of 16 columns: nw waves per workgroup and pb row blocks per wave (16 pb nw >=
// maxmc); nw = 0 selects the left-looking kernel (blocks of 513 to 1024 or above 2048 rows, or
// the test switch AIFMM_PINV_LEFT).  AIFMM_PINV_SHAPE=<nw>x<pb> forces one of the compiled shapes.
static void pinv_shape(int maxmc, int64_t strips, int& nw, int& pb) {
  nw = pb = 0;
  const char* v = getenv("AIFMM_PINV_LEFT");
  if ((v && *v && *v != '0') || maxmc > 2048) return;
  static const int shapes[][2] = {{1, 16}, {2, 16}, {4, 16}, {8, 16}, {2, 8}, {4, 8}, {8, 8}, {4, 4}, {8, 4}, {16, 4}};
  const char* f = getenv("AIFMM_PINV_SHAPE");
  if (f && *f) {
    int a = 0, c = 0;
    if (sscanf(f, "%dx%d", &a, &c) == 2)
      for (auto& sh : shapes)
        if (sh[0] == a && sh[1] == c && 16 * a * c >= maxmc) {
          nw = a;
          pb = c;
          return;
        }
  }
  // blocks of 513 to 1024 rows: the left-looking kernel (measured faster there, where a level has
  // many boxes per colour); otherwise the fewest blocks per wave that hold the block with at most
  // 8 waves (fewer registers, more workgroups per compute unit), then more waves per strip while
  // the grid stays within about one pass over the device's wave slots
  if (maxmc > 512 && maxmc <= 1024) return;
  const int nblk = (maxmc + 15) / 16;
  for (int c : {4, 8, 16}) {
    int a = 1;
    while (a < 8 && 16 * a * c < maxmc) a *= 2;
    if (16 * a * c < maxmc) continue;
    while (a < (c == 4 ? 16 : 8) && 2 * a <= nblk && strips * 2 * a <= 4096) a *= 2;
    for (auto& sh : shapes)
      if (sh[0] == a && sh[1] == c) {
        nw = a;
        pb = c;
        return;
      }
  }
}

// test switch: raise the team abort flag from the host before a level's first launch
static bool debug_abort() {
  const char* v = getenv("AIFMM_DEBUG_ABORT");
  return v && *v && *v != '0';
}

static bool verbose() {
  const char* v = getenv("AIFMM_VERBOSE");
  return v && *v && *v != '0';
}

static void factor_levels_multi(const std::vector<aifmm_system*>& S);

// Factorization of one or more systems.  Several systems (same device and precision) are
// factored in lockstep: step t handles level L_s - t of every system s that still has one, and
// every launch of the step (a round of compressions, its basis changes and commits, the
// elimination phases of a colour) carries the work of all of those systems at once, each work
// item reading its own system's level tables.  Every element of every system is computed by
// the same operations as when the system is factored alone, so the results are the same.
void factor_systems(const std::vector<aifmm_system*>& S) {
  // buffers released during the factorization are freed after its last synchronization
  struct Defer {
    std::vector<void*> ptrs;
    std::vector<void*>* prev;
    hipStream_t st;
    Defer(hipStream_t s_) : prev(g_defer_free), st(s_) { g_defer_free = &ptrs; }
    ~Defer() {
      g_defer_free = prev;
      (void)hipStreamSynchronize(st);
      for (void* p : ptrs) (void)hipFree(p);
    }
  } defer(S[0]->stream);
  factor_levels_multi(S);
}

void factor_system(aifmm_system& s) { factor_systems({&s}); }

static void factor_levels_multi(const std::vector<aifmm_system*>& S) {
  auto t0 = std::chrono::steady_clock::now();
  auto since = [&](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  };
  hipStream_t st = S[0]->stream;
  const bool f32 = S[0]->prec == AIFMM_FP32;
  int Lmax = 0;
  for (aifmm_system* sp : S) {
    aifmm_system& s = *sp;
    if (s.stream != st || s.prec != S[0]->prec || s.device != S[0]->device)
      throw Error{AIFMM_ERR_ARG, "systems factored together need one stream, device and precision"};
    s.stats.schur_flops = s.stats.schur_bytes = s.stats.trsm_flops = s.stats.lu_flops = 0;
    s.stats.schur_kernel_s = s.stats.compress_kernel_s = s.stats.schur_launches = s.stats.compress_launches = 0;
    s.stats.trsm_kernel_s = s.stats.trsm_launches = 0;
    s.stats.lvl.assign(s.L + 1, LevelStats{});
    s.trace.clear();
    s.sc = SolveCache{};
    s.d_flag.zero(st);
    Lmax = std::max(Lmax, s.L);
  }
  const bool multi = S.size() > 1;
  // per system of a step: its level, its own schedule lists and its trace buffers
  struct Run {
    aifmm_system* s = nullptr;
    int l = 0;
    std::vector<RoundEntry> rent;
    std::vector<XformEntry> xent;
    std::vector<int64_t> r_off, x_off;  // per (colour, round)
    std::vector<int> nrounds;           // per colour
    std::vector<int64_t> rix0;          // per colour: index of its first round in r_off
    DBuf<int> d_tr;
    DBuf<double> d_trr;
    std::chrono::steady_clock::time_point tl;
  };
  for (int step = 0; step + 2 <= Lmax; ++step) {
    std::vector<Run> runs;
    for (aifmm_system* sp : S)
      if (sp->L - step >= 2) {
        runs.emplace_back();
        runs.back().s = sp;
        runs.back().l = sp->L - step;
      }
    const int na = (int)runs.size();
    std::vector<LevelPtrs> hP(na);
    int cap = 1, maxblk = 1, kPmax = 1, maxmc = 1, Cmax = 0, Rmax = 0, ncol = 0;
    int64_t tstride = 2;
    for (int q = 0; q < na; ++q) {
      Run& R = runs[q];
      aifmm_system& s = *R.s;
      const int l = R.l;
      R.tl = std::chrono::steady_clock::now();
      activate_level(s, l);
      if (verbose() && !multi) fprintf(stderr, "[aifmm] level %d activated in %.3f s\n", l, since(R.tl));
      LevelDev& lv = s.lev[l];
      LevelPlan& Pl = s.plan[l];
      if (l < s.L) s.lev[l + 1].slab.release();
      cap = std::max(cap, lv.nmax);
      for (int b = 0; b < lv.nb; ++b) {
        maxblk = std::max(maxblk, Pl.il_off[b + 1] - Pl.il_off[b] + 1);
        tstride = std::max(tstride, (int64_t)2 * lv.n[b] * (lv.Ccap[b] + lv.n[b]));
        maxmc = std::max(maxmc, 2 * lv.n[b]);
        if (l > 2) kPmax = std::max(kPmax, s.lev[l - 1].knn[b >> s.d]);
      }
      Cmax = std::max(Cmax, lv.Cmax);
      Rmax = std::max(Rmax, lv.Rmax);
      ncol = std::max(ncol, (int)Pl.col_off.size() - 1);
      lv.d_order.upload(Pl.order, st);
      // the system's static round and transform lists (pair: the entry's index in its round)
      for (size_t c = 0; c + 1 < Pl.col_off.size(); ++c) {
        R.nrounds.push_back((int)Pl.rounds[c].size());
        R.rix0.push_back((int64_t)R.r_off.size());
        for (auto& round : Pl.rounds[c]) {
          R.r_off.push_back((int64_t)R.rent.size());
          R.x_off.push_back((int64_t)R.xent.size());
          int pi = 0;
          for (auto& op : round) {
            RoundEntry E;
            E.i = op.i;
            E.kind = op.kind;
            E.partner = op.partner;
            E.e_ij = find_in(Pl.il_off, Pl.il, op.i, op.partner);
            E.e_ji = find_in(Pl.il_off, Pl.il, op.partner, op.i);
            E.f_ij = find_in(Pl.p2_off, Pl.p2, op.i, op.partner);
            E.f_ji = find_in(Pl.p2_off, Pl.p2, op.partner, op.i);
            if (E.e_ij < 0 || E.e_ji < 0 || E.f_ij < 0 || E.f_ji < 0)
              throw Error{AIFMM_ERR_STATE, "inconsistent compression schedule"};
            E.sys = q;
            E.tidx = (int)R.rent.size();
            R.rent.push_back(E);
            R.xent.push_back({op.i, op.partner, pi, 0, q});
            if (op.kind == 0) R.xent.push_back({op.partner, op.i, pi, 1, q});
            ++pi;
          }
        }
      }
      R.r_off.push_back((int64_t)R.rent.size());
      R.x_off.push_back((int64_t)R.xent.size());
      R.d_tr.alloc(R.rent.size() * 6 + 6);
      R.d_trr.alloc(R.rent.size() * 8 + 8);
      R.d_tr.zero(st);
      R.d_trr.zero(st);
      hP[q] = ptrs(s, l);
      hP[q].trace = R.d_tr.p;
      hP[q].trace_ratio = R.d_trr.p;
      hP[q].flag = s.d_flag.p;
      hP[q].tol = s.tol;
    }
    DBuf<LevelPtrs> dPP;
    dPP.upload(hP, st);
    const LevelPtrs* PP = dPP.p;
    // the step's merged lists: per colour and round the entries of every system (an entry's
    // pair index becomes its index in the merged round), per colour the boxes of every system
    std::vector<RoundEntry> mrent;
    std::vector<XformEntry> mxent;
    std::vector<int64_t> mr_off, mx_off, mb_off;
    std::vector<int> mnr(ncol, 0), mbox, mbsys;
    int maxcol = 1;
    for (int c = 0; c < ncol; ++c) {
      for (auto& R : runs)
        if (c < (int)R.nrounds.size()) mnr[c] = std::max(mnr[c], R.nrounds[c]);
      for (int r = 0; r < mnr[c]; ++r) {
        mr_off.push_back((int64_t)mrent.size());
        mx_off.push_back((int64_t)mxent.size());
        for (auto& R : runs) {
          if (c >= (int)R.nrounds.size() || r >= R.nrounds[c]) continue;
          const int64_t rix = R.rix0[c] + r;
          const int base_pair = (int)(mrent.size() - mr_off.back());
          for (int64_t e = R.r_off[rix]; e < R.r_off[rix + 1]; ++e) mrent.push_back(R.rent[e]);
          for (int64_t x = R.x_off[rix]; x < R.x_off[rix + 1]; ++x) {
            XformEntry X = R.xent[x];
            X.pair += base_pair;
            mxent.push_back(X);
          }
        }
      }
      mb_off.push_back((int64_t)mbox.size());
      int nbc = 0;
      for (int q = 0; q < na; ++q) {
        LevelPlan& Pl = runs[q].s->plan[runs[q].l];
        if (c + 1 >= (int)Pl.col_off.size()) continue;
        for (int i = Pl.col_off[c]; i < Pl.col_off[c + 1]; ++i) {
          mbox.push_back(Pl.order[i]);
          mbsys.push_back(q);
          ++nbc;
        }
      }
      maxcol = std::max(maxcol, nbc);
    }
    mr_off.push_back((int64_t)mrent.size());
    mx_off.push_back((int64_t)mxent.size());
    mb_off.push_back((int64_t)mbox.size());
    DBuf<RoundEntry> d_rent;
    DBuf<XformEntry> d_xent;
    DBuf<int> d_mbox, d_mbsys;
    d_rent.upload(mrent, st);
    d_xent.upload(mxent, st);
    d_mbox.upload(mbox, st);
    d_mbsys.upload(mbsys, st);
    const int* bsys_all = multi ? d_mbsys.p : nullptr;
    const int64_t wsz = 22 * (int64_t)cap * cap + 10 * cap + 16;
    const int XG = 1024;
    // basis changes: 16-wide slabs, each wave with a workspace of 16 x maxdim
    const int maxdim = std::max(cap, kPmax);
    const int nslab = cdiv(maxdim, 16);
    const int64_t wstride = (int64_t)16 * maxdim;
    DBuf<double> ws, scratch;
    ws.alloc((size_t)maxcol * wsz);
    scratch.alloc((size_t)XG * (WG / WAVE) * wstride);
    // the right-hand sides of the pivot-block solves of one colour (a W-sized block per box),
    // the forward results and inverses of the pivot blocks (two m x m blocks per box), and the
    // LDS of the row permutation of each pivot-block LU
    DBuf<double> tws, pws;
    tws.alloc((size_t)maxcol * tstride);
    const int64_t pstride = (int64_t)2 * maxmc * maxmc;
    pws.alloc((size_t)maxcol * pstride);
    // LU: LDS panels where they fit (up to 140 KB beside the kernel's static LDS), and the
    // permutation
    const size_t lu_perm = (size_t)2 * maxmc * sizeof(int);
    if (lu_perm > 128 * 1024) throw Error{AIFMM_ERR_CAPACITY, "pivot block too large for the LU kernel"};
    const size_t lu_shm = std::max(lu_perm, std::min<size_t>(140 * 1024, (size_t)maxmc * (LU_NB + 1) * sizeof(double)));
    AIFMM_HIP(hipFuncSetAttribute((const void*)k_elim_lu, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lu_shm));
    int lu_coop = 0;  // co-resident LU workgroups on the device (0: no cooperative launch)
    {
      int dev = 0, coop = 0, ncu = 0, per = 0;
      AIFMM_HIP(hipGetDevice(&dev));
      AIFMM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
      AIFMM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      AIFMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_elim_lu, WG, lu_shm));
      if (coop && !team_off()) lu_coop = per * ncu;
    }
    DBuf<unsigned> d_luctr;
    DBuf<int> d_lust;
    d_luctr.alloc((size_t)std::max(1, maxcol) * CTR_STRIDE);
    d_lust.alloc(std::max(1, maxcol));
    // the compressions of a round are spread over teams of G workgroups each (cooperative
    // launch, so every team is co-resident); a member keeps its share of a pivoted QR's columns
    // in registers (rows up to 16 RMAX), then in LDS, then in the workspace
    const size_t rs = f32 ? sizeof(float) : sizeof(double);
    const int rmax = reg_rows(cap);
    const void* kcomp = f32 ? compress_fn<float>(rmax) : compress_fn<double>(rmax);
    const int nreg = (CT / 16) * (f32 ? reg_slots_of<float>(rmax) : reg_slots_of<double>(rmax));  // per member
    // reflector (rows up to the register tier's 16 RMAX), pivot positions, own column norms
    const int vlen = std::max(cap, 16 * rmax);
    const size_t base = (size_t)vlen * rs + (size_t)4 * cap * sizeof(int) + (size_t)2 * cap * rs;
    const size_t lds_max = 152 * 1024;
    if (base > lds_max) throw Error{AIFMM_ERR_CAPACITY, "box size too large for the compression kernel"};
    const size_t colb = (size_t)(cap | 1) * rs;
    const int ldsc = lds_off() ? 0 : (int)((lds_max - base) / colb);  // LDS columns per member
    AIFMM_HIP(hipFuncSetAttribute(kcomp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
    constexpr int GMAX = 128;
    int coop_c = 0;  // co-resident compression workgroups (0: no cooperative launch)
    {
      int dev = 0, coop = 0, ncu = 0, per = 0;
      AIFMM_HIP(hipGetDevice(&dev));
      AIFMM_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
      AIFMM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      AIFMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kcomp, CT, lds_max));
      if (coop && !team_off()) coop_c = per * ncu;
    }
    // the smallest even team whose halves (one pivoted QR each) hold their columns on chip, at
    // most team_max members a half and as many as the co-resident workgroups allow; columns
    // beyond the chip's share go to the workspace
    auto team_shape = [&](int ne, int& G, int& lcols, size_t& shm) {
      const int need = 2 * cap;  // columns of one pivoted QR
      int h = cdiv(need, std::max(1, nreg + ldsc));
      h = std::max(1, std::min({h, team_max(), GMAX / 2}));
      G = 1;
      if (coop_c > 0 && (int64_t)ne * 2 <= coop_c) G = 2 * std::min<int64_t>(h, coop_c / (2 * (int64_t)ne));
      const int share = G > 1 ? cdiv(need, G / 2) : need;  // a member's columns of one QR
      lcols = std::min(ldsc, std::max(0, share - nreg));
      // the register tier's Q formation stages FQ_RB reflectors of 16 RMAX entries there too
      shm = base + std::max((size_t)lcols * colb, rmax > 0 ? (size_t)FQ_RB * 16 * rmax * rs : (size_t)0);
    };
    std::map<std::pair<int, int>, int> team_hist;  // (team size, LDS columns a member) -> rounds
    DBuf<unsigned> d_ctr;
    DBuf<Cand> d_part;
    DBuf<int> d_abort;
    DBuf<double> d_pub;
    // a team's counter, then two per compression for its halves, CTR_STRIDE apart
    d_ctr.alloc((size_t)3 * std::max(1, maxcol) * CTR_STRIDE);
    d_part.alloc((size_t)std::max(1, maxcol) * 4 * GMAX * CAND_STRIDE);
    d_pub.alloc((size_t)std::max(1, maxcol) * 2 * GMAX * vlen);
    d_abort.alloc(1);
    d_part.zero(st);
    if (debug_abort()) {  // the abort flag raised before the first launch: every team barrier of
      const int one = 1;  // the step falls through at once and the step reports the failure
      AIFMM_HIP(hipMemcpyAsync(d_abort.p, &one, sizeof(int), hipMemcpyHostToDevice, st));
      AIFMM_HIP(hipStreamSynchronize(st));
    } else {
      d_abort.zero(st);
    }
    std::vector<std::pair<hipEvent_t, hipEvent_t>> sch_ev, cmp_ev, trs_ev;
    auto ev_pair = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
      hipEvent_t a, b;
      AIFMM_HIP(hipEventCreate(&a));
      AIFMM_HIP(hipEventCreate(&b));
      v.push_back({a, b});
      return v.back();
    };
    size_t rix = 0;
    for (int c = 0; c < ncol; ++c) {
      for (int r = 0; r < mnr[c]; ++r, ++rix) {
        int ne = (int)(mr_off[rix + 1] - mr_off[rix]);
        int nx = (int)(mx_off[rix + 1] - mx_off[rix]);
        if (ne == 0) continue;
        const RoundEntry* er = d_rent.p + mr_off[rix];
        const XformEntry* ex = d_xent.p + mx_off[rix];
        auto ce = ev_pair(cmp_ev);
        AIFMM_HIP(hipEventRecord(ce.first, st));
        int G = 1, lcols = 0;
        size_t shm = base;
        team_shape(ne, G, lcols, shm);
        if (verbose()) ++team_hist[{G, lcols}];
        if (G > 1) {
          AIFMM_HIP(hipMemsetAsync(d_ctr.p, 0, sizeof(unsigned) * 3 * ne * CTR_STRIDE, st));
          // exchange slots and the members' exchange flags start at zero in every launch
          AIFMM_HIP(hipMemsetAsync(d_part.p, 0, sizeof(Cand) * (size_t)ne * 4 * G * CAND_STRIDE, st));
        }
        {
          Cand* partp = d_part.p;
          unsigned* ctrp = d_ctr.p;
          int* abortp = d_abort.p;
          double* wsp = ws.p;
          double* pubp = d_pub.p;
          int64_t wszv = wsz;
          void* args[] = {(void*)&PP, (void*)&er, &ne, &wsp, &wszv, &cap, &G, &ctrp, &partp, &abortp, &lcols, &pubp};
          if (G > 1)
            AIFMM_HIP(hipLaunchCooperativeKernel(kcomp, dim3(ne * G), dim3(CT), args, shm, st));
          else
            AIFMM_HIP(hipLaunchKernel(kcomp, dim3(ne), dim3(CT), args, shm, st));
        }
        AIFMM_HIP(hipEventRecord(ce.second, st));
        {
          // an item is a block and every sgroups-th of its slabs, with sgroups chosen so the
          // items about fill the resident waves: each item reads its block's tables once
          const int64_t blocks = std::max<int64_t>(1, (int64_t)nx * maxblk);
          const int sgroups = (int)std::max<int64_t>(1, std::min<int64_t>(nslab, (int64_t)XG * (WG / WAVE) / blocks));
          int64_t items = blocks * sgroups;
          int g64 = (int)std::min<int64_t>(XG, std::max<int64_t>(1, cdiv(items, WG / WAVE)));
          if (f32) {
            hipLaunchKernelGGL(k_xform<float>, dim3(g64), dim3(WG), 0, st, PP, ex, nx, ws.p, wsz, cap, maxblk, sgroups, 0,
                               scratch.p, wstride);
            hipLaunchKernelGGL(k_xform<float>, dim3(g64), dim3(WG), 0, st, PP, ex, nx, ws.p, wsz, cap, maxblk, sgroups, 1,
                               scratch.p, wstride);
          } else {
            hipLaunchKernelGGL(k_xform<double>, dim3(g64), dim3(WG), 0, st, PP, ex, nx, ws.p, wsz, cap, maxblk, sgroups, 0,
                               scratch.p, wstride);
            hipLaunchKernelGGL(k_xform<double>, dim3(g64), dim3(WG), 0, st, PP, ex, nx, ws.p, wsz, cap, maxblk, sgroups, 1,
                               scratch.p, wstride);
          }
        }
        hipLaunchKernelGGL(k_commit, dim3(cdiv(nx, WG)), dim3(WG), 0, st, PP, ex, nx);
      }
      int nbox = (int)(mb_off[c + 1] - mb_off[c]);
      if (nbox == 0) continue;
      const int* boxes = d_mbox.p + mb_off[c];
      const int* bsys = bsys_all ? bsys_all + mb_off[c] : nullptr;
      hipLaunchKernelGGL(k_elim_gather, dim3(nbox, GS), dim3(WG), 0, st, PP, bsys, boxes, tws.p, tstride);
      {
        // teams of up to lu_team_max co-resident workgroups per pivot block
        const int Gl = (lu_coop > 0) ? std::max(1, std::min(lu_team_max(), lu_coop / std::max(1, nbox))) : 1;
        int64_t dynb = lu_panels_off() ? 0 : (int64_t)lu_shm;  // bytes the panels may use
        unsigned* lctr = d_luctr.p;
        int* lst = d_lust.p;
        int* abortp = d_abort.p;
        if (Gl > 1) {
          AIFMM_HIP(hipMemsetAsync(d_luctr.p, 0, sizeof(unsigned) * nbox * CTR_STRIDE, st));
          int Glv = Gl;
          void* args[] = {(void*)&PP, (void*)&bsys, (void*)&boxes, &dynb, &Glv, &lctr, &lst, &abortp};
          AIFMM_HIP(hipLaunchCooperativeKernel((const void*)k_elim_lu, dim3(nbox * Gl), dim3(WG), args, lu_shm, st));
        } else {
          hipLaunchKernelGGL(k_elim_lu, dim3(nbox), dim3(WG), lu_shm, st, PP, bsys, boxes, dynb, 1, lctr, lst, abortp);
        }
      }
      auto te = ev_pair(trs_ev);
      AIFMM_HIP(hipEventRecord(te.first, st));
      {
        // right-looking inverse on strips of 16 columns (shape from pinv_shape), else the
        // left-looking kernel
        const int nblk = cdiv(maxmc, 16);
        int nw = 0, pb = 0;
        pinv_shape(maxmc, nblk * nbox, nw, pb);
        const dim3 pg(nblk, nbox);
#define AIFMM_PINV(NW_, PB_)                                                                            \
  else if (nw == NW_ && pb == PB_) hipLaunchKernelGGL((k_elim_pinv<NW_, PB_>), pg, dim3(NW_ * WAVE), 0, st, PP, \
                                                      bsys, boxes, pws.p, pstride);
        if (nw == 0)
          hipLaunchKernelGGL(k_elim_trsm, dim3(cdiv(maxmc, 16 * TW), nbox), dim3(TW * WAVE), 0, st, PP, bsys, boxes,
                             pws.p, pstride);
        AIFMM_PINV(1, 16) AIFMM_PINV(2, 16) AIFMM_PINV(4, 16) AIFMM_PINV(8, 16)
        AIFMM_PINV(2, 8) AIFMM_PINV(4, 8) AIFMM_PINV(8, 8)
        AIFMM_PINV(4, 4) AIFMM_PINV(8, 4) AIFMM_PINV(16, 4)
#undef AIFMM_PINV
        else throw Error{AIFMM_ERR_STATE, "no pivot-inverse kernel of the chosen shape"};
      }
      {
        const int wt = (int)(cdiv(maxmc, ST) * (int64_t)cdiv(Cmax, ST));
        hipLaunchKernelGGL(k_elim_wgemm, dim3(8 * cdiv(wt, 8), nbox), dim3(WG), 0, st, PP, bsys, boxes, pws.p, pstride,
                           tws.p, tstride);
      }
      AIFMM_HIP(hipEventRecord(te.second, st));
      int tiles_c = cdiv(Cmax, ST), tiles_r = cdiv(std::max(1, Rmax), ST);
      int tiles_x = 8 * cdiv((int64_t)tiles_r * tiles_c, 8);
      auto se = ev_pair(sch_ev);
      AIFMM_HIP(hipEventRecord(se.first, st));
      if (f32)
        hipLaunchKernelGGL(k_elim_schur<true>, dim3(tiles_x, nbox), dim3(WG), 0, st, PP, bsys, boxes, tiles_c);
      else
        hipLaunchKernelGGL(k_elim_schur<false>, dim3(tiles_x, nbox), dim3(WG), 0, st, PP, bsys, boxes, tiles_c);
      AIFMM_HIP(hipEventRecord(se.second, st));
      hipLaunchKernelGGL(k_elim_zrow, dim3(nbox), dim3(WG), 0, st, PP, bsys, boxes);
      launch_check("elimination");
    }
    for (auto& R : runs) R.s->lev[R.l].kfin = R.s->lev[R.l].d_k.download(st);
    AIFMM_HIP(hipStreamSynchronize(st));
    if (d_abort.download(st)[0]) {
      std::string what = multi ? "level " + std::to_string(step) + " from the leaves"
                               : "level " + std::to_string(runs[0].l);
      throw Error{AIFMM_ERR_DEVICE, what + ": a team barrier timed out"};
    }
    // kernel times of the step's launches (shared by the systems of a merged step)
    double t_sch = 0, t_trs = 0, t_cmp = 0;
    auto drain = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& acc) {
      for (auto& pr : v) {
        float ms = 0;
        AIFMM_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        acc += ms * 1e-3;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
    };
    drain(sch_ev, t_sch);
    drain(trs_ev, t_trs);
    drain(cmp_ev, t_cmp);
    for (int q = 0; q < na; ++q) {
      Run& R = runs[q];
      aifmm_system& s = *R.s;
      const int l = R.l;
      LevelDev& lv = s.lev[l];
      double sch_before = s.stats.schur_kernel_s;
      LevelStats& ls = s.stats.lvl[l];
      s.stats.schur_kernel_s += t_sch;
      ls.schur_s += t_sch;
      s.stats.schur_launches += (double)sch_ev.size();
      s.stats.trsm_kernel_s += t_trs;
      ls.trsm_s += t_trs;
      s.stats.trsm_launches += (double)trs_ev.size();
      s.stats.compress_kernel_s += t_cmp;
      ls.compress_s += t_cmp;
      s.stats.compress_launches += (double)cmp_ev.size();
      if (verbose()) {
        fprintf(stderr,
                "[aifmm] level %d factored in %.3f s (%zu compressions), cap %d, %d register columns of %d rows a "
                "member, coop %d; rounds by team (G, LDS columns):",
                l, since(R.tl), R.rent.size(), cap, nreg, 16 * rmax, coop_c);
        for (auto& kv : team_hist) fprintf(stderr, " G%d+L%d:%d", kv.first.first, kv.first.second, kv.second);
        if (multi) fprintf(stderr, " (merged with %d systems)", na);
        fprintf(stderr, "\n");
      }
      const size_t trace0 = s.trace.size();
      {
        std::vector<int> tr = R.d_tr.download(st, R.rent.size() * 6);
        std::vector<double> trr = R.d_trr.download(st, R.rent.size() * 8);
        for (size_t e = 0; e < R.rent.size(); ++e) {
          TraceRec t;
          t.level = l;
          t.i = R.rent[e].i;
          t.kind = R.rent[e].kind;
          t.partner = R.rent[e].partner;
          for (int a = 0; a < 6; ++a) t.r[a] = tr[e * 6 + a];
          for (int a = 0; a < 8; ++a) t.ratio[a] = trr[e * 8 + a];
          s.trace.push_back(t);
        }
      }
      std::vector<int> flag = s.d_flag.download(st);
      if (flag[0])
        throw Error{AIFMM_ERR_SINGULAR, "singular self-block at level " + std::to_string(flag[2]) + " box " + std::to_string(flag[1])};
      for (int b = 0; b < lv.nb; ++b)
        if (lv.kfin[b] > lv.n[b]) throw Error{AIFMM_ERR_CAPACITY, "rank above box size"};
      count_compress(s, l, R.r_off, trace0);
      {
        double f0 = s.stats.schur_flops;
        count_flops(s, l);
        if (verbose())
          fprintf(stderr, "[aifmm] level %d Schur %.3e flop in %.4f s (%.2f TFLOP/s)\n", l, s.stats.schur_flops - f0,
                  s.stats.schur_kernel_s - sch_before,
                  (s.stats.schur_flops - f0) / std::max(1e-12, s.stats.schur_kernel_s - sch_before) * 1e-12);
      }
      lv.xoff.assign(lv.nb + 1, 0);
      lv.koff.assign(lv.nb + 1, 0);
      for (int b = 0; b < lv.nb; ++b) {
        lv.xoff[b + 1] = lv.xoff[b] + lv.n[b];
        lv.koff[b + 1] = lv.koff[b] + lv.kfin[b];
      }
      ls.factor_s = since(R.tl);
      if (l == 2) {
        // top-level multipole system
        LevelDev& l2 = s.lev[2];
        s.Ktop = (int)l2.koff[l2.nb];
        int K = std::max(1, s.Ktop);
        s.d_top.alloc((size_t)K * K);
        s.d_top_piv.alloc(K);
        std::vector<int> koff32(l2.nb);
        for (int b = 0; b < l2.nb; ++b) koff32[b] = (int)l2.koff[b];
        DBuf<int> d_koff;
        d_koff.upload(koff32, st);
        if (s.Ktop > 0) {
          hipLaunchKernelGGL(k_gather_top, dim3(l2.nb, l2.nb), dim3(WG), 0, st, l2.nb, l2.d_k.p, l2.d_n.p, d_koff.p,
                             l2.d_nbr_off.p, l2.d_nbr.p, l2.d_near_slot.p, l2.d_il_off.p, l2.d_il.p, l2.d_il_slot.p,
                             l2.slab.p, s.d_top.p, s.Ktop);
          top_lu(s.d_top.p, s.Ktop, s.d_top_piv.p, s.d_flag.p, st);
          launch_check("top");
        }
        std::vector<int> tflag = s.d_flag.download(st);
        if (verbose()) fprintf(stderr, "[aifmm] top system K=%d factored at %.3f s\n", s.Ktop, since(t0));
        if (tflag[0]) throw Error{AIFMM_ERR_SINGULAR, "singular level-2 multipole system"};
        l2.slab.release();
      }
    }
  }
  AIFMM_HIP(hipStreamSynchronize(st));
  for (aifmm_system* sp : S) sp->stats.factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace aifmm
