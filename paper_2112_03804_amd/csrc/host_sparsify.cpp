// Technique B's explicit factors of a river endgame's payoff matrix (host).
//
// Proposition 1 writes A, in hand-major order (row h1 * S1 + s1, column
// h2 * S2 + s2), as C (x) F + (L1 W L2) (x) S with L_i = diag(lambda_i),
// lambda_i = mu_i / sqrt(beta), C = lambda1 lambda2^T - L1 Hx L2 (Hx: the
// pairs of hands that share a card), W the showdown outcome and F, S the fold
// payoffs and showdown stakes over sequence pairs.  Technique B (Section 4)
// sorts Player 1's hands by strength and writes W = D^-1 Y, with D lower
// bidiagonal (1 on the diagonal, -1 below) and Y = D W the differences of
// consecutive outcome rows; then
//   A = Ahat + U M^-1 V^T,   Ahat = -(L1 Hx L2) (x) F,
//   U = [L1 (x) I | lambda1 (x) I],   M = blockdiag(D (x) I, I),
//   V = [(L2 Y^T) (x) S^T | lambda2 (x) F^T]
// (lambda in the rank-one and U, V blocks, the reading under which the
// product is A).  The Postprocessing subsection drops the identically zero
// columns of V: with M unit lower triangular, the unknown of such a column is
// minus the combination its row of M gives, and it is substituted into the
// other rows of M and into U.  Sizes are stored nonzeros (Table 1's metric).
//
// The factors are also emitted for the GPU path: CSR forms of Ahat, U and V
// (and their transposes) indexed by the library's vector elements, and the
// postprocessed M as chains (every row and column of M holds at most one
// off-diagonal entry), solved by pointer jumping.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

namespace pmx {

namespace {

struct Triplet {
  int64_t r, c;
  double v;
};

void to_csr(std::vector<Triplet> t, int64_t rows, int64_t cols, TbCsr& out) {
  std::sort(t.begin(), t.end(), [](const Triplet& a, const Triplet& b) { return a.r < b.r || (a.r == b.r && a.c < b.c); });
  out.rows = rows;
  out.cols = cols;
  out.ptr.assign(rows + 1, 0);
  out.idx.clear();
  out.val.clear();
  for (size_t i = 0; i < t.size();) {
    size_t j = i;
    double s = 0.0;
    while (j < t.size() && t[j].r == t[i].r && t[j].c == t[i].c) s += t[j++].v;
    if (s != 0.0) {
      out.idx.push_back(t[i].c);
      out.val.push_back(s);
      ++out.ptr[t[i].r + 1];
    }
    i = j;
  }
  for (int64_t r = 0; r < rows; ++r) out.ptr[r + 1] += out.ptr[r];
}

std::vector<Triplet> transpose(const std::vector<Triplet>& t) {
  std::vector<Triplet> o(t.size());
  for (size_t i = 0; i < t.size(); ++i) o[i] = {t[i].c, t[i].r, t[i].v};
  return o;
}

}  // namespace

int build_tb_factors(const HostGame& hg, TbHost& out, std::string& msg) {
  out = TbHost();
  if (hg.inst.size() != 1) {
    msg = "the explicit factors are built for games of one instance";
    return PMX_EINVAL;
  }
  const Built& b = hg.inst[0];
  const Instance& in = b.inst;
  if (in.two_rounds()) {
    msg = "the explicit factors are built for river endgames (one final board)";
    return PMX_EINVAL;
  }
  const int S1 = b.sf.n_seq[0], S2 = b.sf.n_seq[1];
  const int N1 = in.n[0], N2 = in.n[1];
  const int64_t st0 = b.stride[0], st1 = b.stride[1];
  const std::vector<double>& lam1 = b.lam[0];
  const std::vector<double>& lam2 = b.lam[1];
  // fold payoffs and showdown stakes over sequence pairs
  std::vector<double> F((size_t)S1 * S2, 0.0), S((size_t)S1 * S2, 0.0);
  for (const Terminal& t : b.sf.terms) {
    const size_t k = (size_t)t.seq[0] * S2 + t.seq[1];
    if (t.kind == PMX_SHOWDOWN) S[k] += t.c1;
    else F[k] += t.kind == PMX_FOLD_P1 ? -t.c1 : t.c2;
  }
  // Player 1's hands by increasing strength (ties keep list order)
  std::vector<int> order(N1);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return in.strength[0][a] < in.strength[0][c]; });
  auto shares = [&](int h1, int h2) {
    for (int a = 0; a < in.cph; ++a)
      for (int c = 0; c < in.cph; ++c)
        if (in.cards[0][(size_t)h1 * in.cph + a] == in.cards[1][(size_t)h2 * in.cph + c]) return true;
    return false;
  };
  auto outcome = [&](int h1, int h2) {
    if (shares(h1, h2)) return 0.0;
    const int32_t a = in.strength[0][h1], c = in.strength[1][h2];
    return a > c ? 1.0 : (a < c ? -1.0 : 0.0);
  };
  // nonzeros of A: fold pairs x compatible pairs + showdown pairs x decided pairs
  {
    int64_t nf = 0, ns = 0, nc = 0, nw = 0;
    for (size_t k = 0; k < F.size(); ++k) {
      nf += F[k] != 0.0;
      ns += S[k] != 0.0;
    }
    for (int h1 = 0; h1 < N1; ++h1)
      for (int h2 = 0; h2 < N2; ++h2) {
        const double pi = lam1[h1] * lam2[h2];
        if (pi == 0.0) continue;
        nc += !shares(h1, h2);
        nw += outcome(h1, h2) != 0.0;
      }
    out.nnz_A = nf * nc + ns * nw;
  }
  const int64_t n_m = (int64_t)N1 * S1 + S1;   // the solve's dimension before postprocessing
  // internal indices: Player 1 row pos * S1 + s1 (pos: strength position),
  // Player 2 row h2 * S2 + s2
  std::vector<Triplet> ahat, U, V;
  std::vector<std::map<int64_t, double>> ucol(n_m), mrow(n_m);
  std::vector<std::set<int64_t>> mcol(n_m);
  std::vector<double> Yrow(N2), Wprev(N2, 0.0), Wcur(N2);
  for (int pos = 0; pos < N1; ++pos) {
    const int h1 = order[pos];
    for (int h2 = 0; h2 < N2; ++h2) {
      Wcur[h2] = outcome(h1, h2);
      Yrow[h2] = Wcur[h2] - (pos > 0 ? Wprev[h2] : 0.0);
    }
    Wprev = Wcur;
    for (int s1 = 0; s1 < S1; ++s1) {
      const int64_t row = (int64_t)pos * S1 + s1;
      // Ahat = -(L1 Hx L2) (x) F
      for (int s2 = 0; s2 < S2; ++s2) {
        const double f = F[(size_t)s1 * S2 + s2];
        if (f == 0.0) continue;
        for (int h2 = 0; h2 < N2; ++h2)
          if (shares(h1, h2)) {
            const double v = -lam1[h1] * lam2[h2] * f;
            if (v != 0.0) ahat.push_back({row, (int64_t)h2 * S2 + s2, v});
          }
      }
      // U = [L1 (x) I | lambda1 (x) I]
      if (lam1[h1] != 0.0) {
        ucol[row][row] = lam1[h1];
        ucol[(int64_t)N1 * S1 + s1][row] = lam1[h1];
      }
      // M = D (x) I on the first block: -1 below the diagonal
      if (pos > 0) {
        mrow[row][row - S1] = -1.0;
        mcol[row - S1].insert(row);
      }
      // V first block: (L2 Y^T) (x) S^T
      for (int s2 = 0; s2 < S2; ++s2) {
        const double sv = S[(size_t)s1 * S2 + s2];
        if (sv == 0.0) continue;
        for (int h2 = 0; h2 < N2; ++h2) {
          const double v = lam2[h2] * Yrow[h2] * sv;
          if (v != 0.0) V.push_back({(int64_t)h2 * S2 + s2, row, v});
        }
      }
    }
  }
  // V second block: lambda2 (x) F^T
  for (int s1 = 0; s1 < S1; ++s1)
    for (int s2 = 0; s2 < S2; ++s2) {
      const double f = F[(size_t)s1 * S2 + s2];
      if (f == 0.0) continue;
      for (int h2 = 0; h2 < N2; ++h2) {
        const double v = lam2[h2] * f;
        if (v != 0.0) V.push_back({(int64_t)h2 * S2 + s2, (int64_t)N1 * S1 + s1, v});
      }
    }
  auto count_u = [&]() {
    int64_t n = 0;
    for (const auto& c : ucol)
      for (const auto& kv : c) n += kv.second != 0.0;
    return n;
  };
  auto count_m = [&](const std::vector<char>& alive) {
    int64_t n = 0;
    for (int64_t k = 0; k < n_m; ++k) {
      if (!alive[k]) continue;
      ++n;
      for (const auto& kv : mrow[k]) n += kv.second != 0.0;
    }
    return n;
  };
  std::vector<char> vcol_nz(n_m, 0), alive(n_m, 1);
  for (const Triplet& t : V) vcol_nz[t.c] = 1;
  out.m_dim = n_m;
  out.nnz[0] = (int64_t)ahat.size();
  out.nnz[1] = count_u();
  out.nnz[2] = count_m(alive);
  out.nnz[3] = (int64_t)V.size();
  // postprocessing: substitute the unknowns of V's zero columns, in order
  for (int64_t j = 0; j < n_m; ++j) {
    if (vcol_nz[j]) continue;
    const std::map<int64_t, double> a = mrow[j];   // y_j = -sum_i a_i y_i
    for (const auto& ai : a) {
      for (const auto& ru : ucol[j]) ucol[ai.first][ru.first] -= ai.second * ru.second;
      mcol[ai.first].erase(j);
    }
    for (int64_t k : mcol[j]) {
      const double mkj = mrow[k][j];
      mrow[k].erase(j);
      for (const auto& ai : a) {
        mrow[k][ai.first] -= mkj * ai.second;
        mcol[ai.first].insert(k);
      }
    }
    ucol[j].clear();
    mrow[j].clear();
    mcol[j].clear();
    alive[j] = 0;
  }
  std::vector<int64_t> newpos(n_m, -1);
  int64_t m2 = 0;
  for (int64_t j = 0; j < n_m; ++j)
    if (alive[j]) newpos[j] = m2++;
  out.m_dim_pp = m2;
  out.nnz_pp[0] = out.nnz[0];
  out.nnz_pp[1] = count_u();
  out.nnz_pp[2] = count_m(alive);
  out.nnz_pp[3] = out.nnz[3];
  // M after postprocessing as chains: one parent (the row's off-diagonal
  // entry) and at most one child per unknown
  out.par.assign(m2, -1);
  out.chi.assign(m2, -1);
  out.cpar.assign(m2, 0.0);
  out.cchi.assign(m2, 0.0);
  for (int64_t k = 0; k < n_m; ++k) {
    if (!alive[k]) continue;
    int cnt = 0;
    for (const auto& kv : mrow[k]) {
      if (kv.second == 0.0) continue;
      if (++cnt > 1) {
        msg = "M has a row with two off-diagonal entries (not a set of chains)";
        return PMX_EINVAL;
      }
      const int64_t kk = newpos[k], ii = newpos[kv.first];
      if (out.chi[ii] >= 0) {
        msg = "M has a column with two off-diagonal entries (not a set of chains)";
        return PMX_EINVAL;
      }
      // z_k + M[k, i] z_i = r_k: z_k = r_k - M[k, i] z_i, and in M^T w = r,
      // w_i = r_i - M[k, i] w_k
      out.par[kk] = (int32_t)ii;
      out.cpar[kk] = -kv.second;
      out.chi[ii] = (int32_t)kk;
      out.cchi[ii] = -kv.second;
    }
  }
  int depth = 0;
  for (int64_t k = 0; k < m2; ++k) {
    if (out.par[k] >= 0) continue;   // the head of a chain
    int d = 1;
    for (int64_t c = out.chi[k]; c >= 0; c = out.chi[c]) ++d;
    depth = std::max(depth, d);
  }
  out.depth = depth;
  // device forms over the library's vector elements
  auto own_el = [&](int64_t r) {   // internal Player 1 index -> element
    const int pos = (int)(r / S1), s1 = (int)(r % S1);
    return b.vec_off[0] + (int64_t)s1 * st0 + order[pos];
  };
  auto opp_el = [&](int64_t c) {   // internal Player 2 index -> element
    const int h2 = (int)(c / S2), s2 = (int)(c % S2);
    return b.vec_off[1] + (int64_t)s2 * st1 + h2;
  };
  const int64_t E0 = hg.elems[0], E1 = hg.elems[1];
  std::vector<Triplet> A_el, U_el, V_el;
  A_el.reserve(ahat.size());
  for (const Triplet& t : ahat) A_el.push_back({own_el(t.r), opp_el(t.c), t.v});
  for (int64_t j = 0; j < n_m; ++j) {
    if (!alive[j]) continue;
    for (const auto& ru : ucol[j])
      if (ru.second != 0.0) U_el.push_back({own_el(ru.first), newpos[j], ru.second});
  }
  V_el.reserve(V.size());
  for (const Triplet& t : V) V_el.push_back({opp_el(t.r), newpos[t.c], t.v});
  to_csr(A_el, E0, E1, out.ahat);
  to_csr(transpose(A_el), E1, E0, out.ahat_t);
  to_csr(U_el, E0, m2, out.u);
  to_csr(transpose(U_el), m2, E0, out.u_t);
  to_csr(V_el, E1, m2, out.v);
  to_csr(transpose(V_el), m2, E1, out.v_t);
  return PMX_OK;
}

}  // namespace pmx
