// Host-side decision rules of the doubling (plain C++, no device code): the
// truncation rule, the sweep schedule and its gauge, the S^z charge
// bookkeeping of the U(1) route and the merge of the singular values of
// charge blocks.  The library calls them on the values and charges it reads
// back from the device.
#pragma once

#include <algorithm>
#include <limits>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

namespace xtrg_host {

// Number of kept singular values (truncation by the number of kept states,
// Sec. II.D).  S descending; values <= max(floor * S[0], abs_floor) count
// as zero; at most D are kept, backed off to the largest k >= D/2 whose gap
// S[k-1] - S[k] exceeds deg_rtol * S[k-1] + abs_floor, so that a degenerate
// multiplet is not split (deg_rtol = 0: cut at exactly D).
inline int keep_count(const std::vector<double>& S, int D, double deg_rtol, double floor, double abs_floor) {
  if (S.empty() || !(S[0] > 0)) return 1;
  const double f = std::max(floor * S[0], abs_floor);
  int r = 0;
  for (double v : S)
    if (v > f) ++r;
  r = std::max(r, 1);
  if (r <= D) return r;
  // a gap separates two multiplets only if it exceeds deg_rtol * S[k-1]
  // plus the absolute rounding noise abs_floor of the values themselves
  if (!(deg_rtol > 0)) return D;
  const int lo = std::max(1, (D + 1) / 2);
  for (int k = D; k >= lo; --k)
    if (S[k - 1] - S[k] > deg_rtol * S[k - 1] + abs_floor) return k;
  return D;
}

// The bonds a doubling visits (App. D.1: variational two-site sweeps):
// n_sweeps full sweeps, each a left-to-right half-sweep over bonds 0 .. n-2
// (from 1 after the first) and a right-to-left one over n-3 .. 0, so the
// bond that ends a half-sweep is not optimised twice in a row.
struct Step {
  int bond;
  int dir;        // +1 left-to-right, -1 right-to-left
  bool last;      // last bond of its half-sweep
};

inline std::vector<Step> schedule(int n, int n_sweeps) {
  std::vector<Step> out;
  for (int h = 0; h < 2 * n_sweeps; ++h) {
    std::vector<int> bonds;
    if (h % 2 == 0)
      for (int b = (h == 0 ? 0 : 1); b <= n - 2; ++b) bonds.push_back(b);
    else
      for (int b = n - 3; b >= 0; --b) bonds.push_back(b);
    for (size_t j = 0; j < bonds.size(); ++j)
      out.push_back({bonds[j], h % 2 == 0 ? 1 : -1, j + 1 == bonds.size()});
  }
  return out;
}

// Which side of a step keeps the isometry: the left site (the sweep moves
// right) unless the step ends its half-sweep, where the gauge turns; the
// final step of the doubling leaves the centre at site 0 (right side
// isometric), where the result is normalised.
inline bool gauge_right(const Step& sp, bool final_step) { return final_step ? false : (sp.dir > 0) != sp.last; }

// U(1) charge sectors (Sec. II.A: the XXZ models conserve S^z_tot; App.
// B.2).  Site index 0 is up; the entry W[a][s][s'][b] of a site tensor
// [Dl][2][2][Dr] multiplies |s><s'|, which raises S^z by s' - s, so in a
// charge-definite basis it is non-zero only if q_b = q_a + (s' - s).

// Charges of the rows (c, s, s'') of a site matrix or two-site tensor from
// the charges q of its left bond: q_c + (s'' - s).
inline std::vector<int> row_charges(const std::vector<int>& q) {
  std::vector<int> out(q.size() * 4);
  for (size_t c = 0; c < q.size(); ++c)
    for (int s = 0; s < 2; ++s)
      for (int u = 0; u < 2; ++u) out[c * 4 + s * 2 + u] = q[c] + (u - s);
  return out;
}

// Charge a left index must carry to connect to the column (t, t'', c) of a
// site matrix or two-site tensor: q_c - (t'' - t).
inline std::vector<int> col_charges(const std::vector<int>& q) {
  const size_t D = q.size();
  std::vector<int> out(4 * D);
  for (int t = 0; t < 2; ++t)
    for (int u = 0; u < 2; ++u)
      for (size_t c = 0; c < D; ++c) out[(t * 2 + u) * D + c] = q[c] - (u - t);
  return out;
}

// Charges of every bond index from the non-zero entries of the sites, from
// q = 0 at the left end.  An index that no non-zero entry reaches from an
// index of known charge contributes nothing to the operator; it gets charge
// 0.  Throws std::invalid_argument if an index would need two charges.
inline std::vector<std::vector<int>> infer_charges(const std::vector<std::vector<double>>& W,
                                                   const std::vector<int>& dims) {
  const int L = (int)W.size();
  std::vector<std::vector<int>> q(L + 1);
  q[0].assign(dims[0], 0);
  std::vector<char> known(dims[0], 1);
  for (int i = 0; i < L; ++i) {
    const int Dl = dims[i], Dr = dims[i + 1];
    std::vector<int> lo(Dr, std::numeric_limits<int>::max()), hi(Dr, std::numeric_limits<int>::min());
    for (int a = 0; a < Dl; ++a) {
      if (!known[a]) continue;
      for (int st = 0; st < 4; ++st) {
        const double* row = W[i].data() + ((size_t)a * 4 + st) * Dr;
        const int v = q[i][a] + ((st & 1) - (st >> 1));
        for (int b = 0; b < Dr; ++b)
          if (row[b] != 0.0) {
            lo[b] = std::min(lo[b], v);
            hi[b] = std::max(hi[b], v);
          }
      }
    }
    q[i + 1].assign(Dr, 0);
    known.assign(Dr, 0);
    for (int b = 0; b < Dr; ++b) {
      if (hi[b] < lo[b]) continue;
      if (hi[b] != lo[b])
        throw std::invalid_argument("site " + std::to_string(i) + ": a bond index carries two S^z charges");
      known[b] = 1;
      q[i + 1][b] = lo[b];
    }
  }
  return q;
}

// The charge blocks of a matrix whose rows carry the charges ql and columns
// qp: for every charge present on both sides (increasing), its rows and
// columns in increasing index order.
struct ChargeBlock {
  int q;
  std::vector<int> rows, cols;
};

inline std::vector<ChargeBlock> charge_blocks(const std::vector<int>& ql, const std::vector<int>& qp) {
  std::map<int, std::pair<std::vector<int>, std::vector<int>>> g;
  for (int r = 0; r < (int)ql.size(); ++r) g[ql[r]].first.push_back(r);
  for (int j = 0; j < (int)qp.size(); ++j) g[qp[j]].second.push_back(j);
  std::vector<ChargeBlock> out;
  for (auto& kv : g)
    if (!kv.second.first.empty() && !kv.second.second.empty())
      out.push_back({kv.first, std::move(kv.second.first), std::move(kv.second.second)});
  return out;
}

// The singular values of the charge blocks of one matrix merged into one
// descending list.  Blocks come in increasing charge, each block's values
// descending; a stable sort by value keeps both orders among equal values
// (equal values in increasing charge).  For every merged value: its
// charge, its block and its rank in the block.
struct Merged {
  std::vector<double> S;
  std::vector<int> qs, from, rank;
};

inline Merged merge_block_values(const std::vector<int>& q, const std::vector<std::vector<double>>& S) {
  struct E {
    double v;
    int q, blk, rank;
  };
  std::vector<E> e;
  for (size_t t = 0; t < S.size(); ++t)
    for (size_t j = 0; j < S[t].size(); ++j) e.push_back({S[t][j], q[t], (int)t, (int)j});
  std::stable_sort(e.begin(), e.end(), [](const E& a, const E& b) { return a.v > b.v; });
  Merged m;
  for (const E& x : e) {
    m.S.push_back(x.v);
    m.qs.push_back(x.q);
    m.from.push_back(x.blk);
    m.rank.push_back(x.rank);
  }
  return m;
}

}  // namespace xtrg_host
