// C entry points over the library's host-side rules (host_rules.h) for the
// CPU tests, which compare them with the oracle.  Test infrastructure only.
#include <cstring>
#include <vector>

#include "host_rules.h"

extern "C" {

int hr_keep_count(const double* S, int n, int D, double deg_rtol, double floor, double abs_floor) {
  return xtrg_host::keep_count(std::vector<double>(S, S + n), D, deg_rtol, floor, abs_floor);
}

// sites: the L site tensors [dims[i]][2][2][dims[i+1]] one after the other;
// out: the charges of bonds 0..L one after the other.  0, or -1 if refused.
int hr_infer_charges(int L, const int* dims, const double* sites, int* out) {
  std::vector<std::vector<double>> W(L);
  std::vector<int> d(dims, dims + L + 1);
  size_t o = 0;
  for (int i = 0; i < L; ++i) {
    const size_t n = (size_t)dims[i] * 4 * dims[i + 1];
    W[i].assign(sites + o, sites + o + n);
    o += n;
  }
  try {
    const auto q = xtrg_host::infer_charges(W, d);
    size_t k = 0;
    for (const auto& b : q)
      for (int v : b) out[k++] = v;
    return 0;
  } catch (const std::invalid_argument&) {
    return -1;
  }
}

// nb blocks of charges q, with r[t] values each (concatenated in vals);
// out: the merged values, their charges, blocks and ranks.
void hr_merge(int nb, const int* q, const int* r, const double* vals, double* S, int* qs, int* from, int* rank) {
  std::vector<int> qb(q, q + nb);
  std::vector<std::vector<double>> Sb(nb);
  size_t o = 0;
  for (int t = 0; t < nb; ++t) {
    Sb[t].assign(vals + o, vals + o + r[t]);
    o += r[t];
  }
  const auto m = xtrg_host::merge_block_values(qb, Sb);
  for (size_t j = 0; j < m.S.size(); ++j) {
    S[j] = m.S[j];
    qs[j] = m.qs[j];
    from[j] = m.from[j];
    rank[j] = m.rank[j];
  }
}

// The steps of a doubling of n sites with n_sweeps sweeps (arrays of
// (n - 1) * 2 * n_sweeps entries at most); returns their count.
int hr_schedule(int n, int n_sweeps, int* bond, int* dir, int* last, int* gauge) {
  const auto sc = xtrg_host::schedule(n, n_sweeps);
  for (size_t j = 0; j < sc.size(); ++j) {
    bond[j] = sc[j].bond;
    dir[j] = sc[j].dir;
    last[j] = sc[j].last ? 1 : 0;
    gauge[j] = xtrg_host::gauge_right(sc[j], j + 1 == sc.size()) ? 1 : 0;
  }
  return (int)sc.size();
}

// The charge blocks of rows ql (nl) and columns qp (np): their charges,
// sizes, and the rows and columns one block after the other; returns the
// number of blocks.
int hr_charge_blocks(int nl, const int* ql, int np, const int* qp, int* q, int* nr, int* nc, int* rows, int* cols) {
  const auto cb = xtrg_host::charge_blocks(std::vector<int>(ql, ql + nl), std::vector<int>(qp, qp + np));
  int orr = 0, oc = 0;
  for (size_t t = 0; t < cb.size(); ++t) {
    q[t] = cb[t].q;
    nr[t] = (int)cb[t].rows.size();
    nc[t] = (int)cb[t].cols.size();
    for (int r : cb[t].rows) rows[orr++] = r;
    for (int c : cb[t].cols) cols[oc++] = c;
  }
  return (int)cb.size();
}

}  // extern "C"
