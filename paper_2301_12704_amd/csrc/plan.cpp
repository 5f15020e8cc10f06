// Host planner: per-level lists, colour-major elimination order and the static compression
// schedule of the efficient elimination algorithm (Sec. 3.3).  Everything here depends only
// on the geometry of the uniform tree, never on matrix values, so it is computed once at
// build time and the device kernels read it from tables.
#include <algorithm>
#include <set>

#include "system.hpp"

namespace aifmm {

int cheb(const int* a, const int* b, int d) {
  int m = 0;
  for (int t = 0; t < d; ++t) m = std::max(m, std::abs(a[t] - b[t]));
  return m;
}

static int morton_of(const int* c, int d, int l) {
  int m = 0;
  for (int bit = 0; bit < l; ++bit)
    for (int t = 0; t < d; ++t) m |= ((c[t] >> bit) & 1) << (bit * d + t);
  return m;
}

static void csr_from(const std::vector<std::vector<int>>& lists, std::vector<int>& off, std::vector<int>& val) {
  off.assign(lists.size() + 1, 0);
  for (size_t b = 0; b < lists.size(); ++b) off[b + 1] = off[b] + (int)lists[b].size();
  val.clear();
  val.reserve(off.back());
  for (auto& v : lists) val.insert(val.end(), v.begin(), v.end());
}

static void transpose_index(const std::vector<int>& off, const std::vector<int>& val, std::vector<int>& tr) {
  tr.assign(val.size(), -1);
  int nb = (int)off.size() - 1;
  for (int b = 0; b < nb; ++b)
    for (int e = off[b]; e < off[b + 1]; ++e) {
      int q = val[e];
      auto beg = val.begin() + off[q], end = val.begin() + off[q + 1];
      auto it = std::lower_bound(beg, end, b);
      if (it != end && *it == b) tr[e] = (int)(it - val.begin());
    }
}

void plan_level(LevelPlan& P, int d, int l) {
  P.l = l;
  P.nb = 1 << (d * l);
  int side = 1 << l;
  int nb = P.nb;
  P.coord.assign((size_t)nb * 3, 0);
  for (int b = 0; b < nb; ++b)
    for (int bit = 0; bit < l; ++bit)
      for (int t = 0; t < d; ++t) P.coord[b * 3 + t] |= ((b >> (bit * d + t)) & 1) << bit;
  std::vector<std::vector<int>> nbr(nb), il(nb), p2(nb);
  for (int b = 0; b < nb; ++b) {
    const int* c = &P.coord[b * 3];
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int t = 0; t < d; ++t) { lo[t] = std::max(0, c[t] - 2); hi[t] = std::min(side - 1, c[t] + 2); }
    int q[3] = {0, 0, 0};
    for (q[0] = lo[0]; q[0] <= hi[0]; ++q[0])
      for (q[1] = lo[1]; q[1] <= hi[1]; ++q[1])
        for (q[2] = lo[2]; q[2] <= (d == 3 ? hi[2] : 0); ++q[2]) {
          int dist = cheb(c, q, d);
          int m = morton_of(q, d, l);
          if (dist <= 1) nbr[b].push_back(m);
          else if (dist == 2) p2[b].push_back(m);
        }
    std::sort(nbr[b].begin(), nbr[b].end());
    std::sort(p2[b].begin(), p2[b].end());
    // IL(b): children of the parent's neighbours that are not neighbours of b (Sec. 2.2)
    if (l >= 2) {
      int pc[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
      int pside = side >> 1;
      int r[3] = {0, 0, 0};
      for (r[0] = std::max(0, pc[0] - 1); r[0] <= std::min(pside - 1, pc[0] + 1); ++r[0])
        for (r[1] = std::max(0, pc[1] - 1); r[1] <= std::min(pside - 1, pc[1] + 1); ++r[1])
          for (r[2] = (d == 3 ? std::max(0, pc[2] - 1) : 0); r[2] <= (d == 3 ? std::min(pside - 1, pc[2] + 1) : 0); ++r[2])
            for (int ch = 0; ch < (1 << d); ++ch) {
              int cc[3] = {2 * r[0] + (ch & 1), 2 * r[1] + ((ch >> 1) & 1), d == 3 ? 2 * r[2] + ((ch >> 2) & 1) : 0};
              if (cheb(c, cc, d) >= 2) il[b].push_back(morton_of(cc, d, l));
            }
      std::sort(il[b].begin(), il[b].end());
    }
  }
  csr_from(nbr, P.nbr_off, P.nbr);
  csr_from(il, P.il_off, P.il);
  csr_from(p2, P.p2_off, P.p2);
  transpose_index(P.il_off, P.il, P.il_tr);
  transpose_index(P.p2_off, P.p2, P.p2_tr);

  // colour-major order: colour = (c_1 mod 5, ..., c_d mod 5) lexicographic, Morton within.
  // Boxes of one colour are >= 5 apart, so their neighbourhoods, their distance-2 partners
  // and the rows / columns touched by their compressions are disjoint.
  std::vector<std::pair<int64_t, int>> key(nb);
  for (int b = 0; b < nb; ++b) {
    int64_t col = 0;
    for (int t = 0; t < d; ++t) col = col * 5 + (P.coord[b * 3 + t] % 5);
    key[b] = {col * (int64_t)nb + b, b};
  }
  std::sort(key.begin(), key.end());
  P.order.resize(nb);
  P.pos.resize(nb);
  P.col_off.clear();
  int64_t prev_col = -1;
  for (int q = 0; q < nb; ++q) {
    P.order[q] = key[q].second;
    P.pos[key[q].second] = q;
    int64_t col = key[q].first / nb;
    if (col != prev_col) { P.col_off.push_back(q); prev_col = col; }
  }
  P.col_off.push_back(nb);

  // Static schedule of Algorithm "Efficient Elimination": replay the elimination order and
  // the fill-in bookkeeping (pending P2P pairs unordered, pending P2L pairs ordered as
  // (eliminated, not eliminated)); before box i: its P2P pairs, then its P2L pairs, each by
  // increasing elimination position of the partner.
  std::vector<char> elim(nb, 0);
  std::vector<std::set<int>> pend_p2p(nb), pend_p2l(nb);
  std::vector<std::vector<PairOp>> ops(nb);
  for (int q = 0; q < nb; ++q) {
    int i = P.order[q];
    std::vector<std::pair<int, int>> t;
    for (int j : pend_p2p[i]) t.push_back({P.pos[j], j});
    std::sort(t.begin(), t.end());
    for (auto& pj : t) {
      ops[i].push_back({i, 0, pj.second});
      pend_p2p[pj.second].erase(i);
    }
    pend_p2p[i].clear();
    t.clear();
    for (int r : pend_p2l[i]) t.push_back({P.pos[r], r});
    std::sort(t.begin(), t.end());
    for (auto& pr : t) ops[i].push_back({i, 1, pr.second});
    pend_p2l[i].clear();
    elim[i] = 1;
    for (int e1 = P.nbr_off[i]; e1 < P.nbr_off[i + 1]; ++e1)
      for (int e2 = P.nbr_off[i]; e2 < P.nbr_off[i + 1]; ++e2) {
        int p = P.nbr[e1], r = P.nbr[e2];
        if (p == r || p == i || r == i) continue;
        if (cheb(&P.coord[p * 3], &P.coord[r * 3], d) != 2) continue;
        if (elim[p] && elim[r]) continue;
        if (elim[p]) pend_p2l[r].insert(p);
        else if (elim[r]) pend_p2l[p].insert(r);
        else { pend_p2p[p].insert(r); pend_p2p[r].insert(p); }
      }
  }
  int ncol = (int)P.col_off.size() - 1;
  P.rounds.assign(ncol, {});
  for (int c = 0; c < ncol; ++c) {
    size_t smax = 0;
    for (int q = P.col_off[c]; q < P.col_off[c + 1]; ++q) smax = std::max(smax, ops[P.order[q]].size());
    P.rounds[c].assign(smax, {});
    for (int q = P.col_off[c]; q < P.col_off[c + 1]; ++q) {
      int i = P.order[q];
      for (size_t r = 0; r < ops[i].size(); ++r) P.rounds[c][r].push_back(ops[i][r]);
    }
  }
  // coupled groups of every elimination (Appendix-style reading of eq. X2 / Y): the other
  // neighbours in Morton order, then the box itself
  P.grp_off.assign(nb + 1, 0);
  P.grp_box.clear();
  P.grp_elim.clear();
  for (int b = 0; b < nb; ++b) {
    for (int e = P.nbr_off[b]; e < P.nbr_off[b + 1]; ++e) {
      int p = P.nbr[e];
      if (p == b) continue;
      P.grp_box.push_back(p);
      P.grp_elim.push_back(P.pos[p] < P.pos[b] ? 1 : 0);
    }
    P.grp_box.push_back(b);
    P.grp_elim.push_back(0);
    P.grp_off[b + 1] = (int)P.grp_box.size();
  }
}

}  // namespace aifmm
