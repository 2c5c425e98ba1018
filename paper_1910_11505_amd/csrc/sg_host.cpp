// Host set-up mathematics of the SG solver: chaos index sets, Hermite triple
// products, the KL eigenproblem and the field-split groupings.  Written
// independently of any reference implementation: own enumeration, own
// Cholesky + cyclic Jacobi eigensolver, no LAPACK.
#include <algorithm>
#include <cmath>
#include <functional>

#include "sg_internal.h"

namespace sg {

// J(p) = {alpha in N^M : |alpha| <= p} (Sec. 2.2), graded by |alpha|; inside
// one degree the tuples come in descending lexicographic order, which is what
// a depth-first enumeration taking the largest first entry first produces.
std::vector<std::vector<int>> total_degree_set(int M, int p) {
  std::vector<std::vector<int>> out;
  std::vector<int> cur(M, 0);
  std::function<void(int, int)> rec = [&](int pos, int left) {
    if (pos == M - 1) {
      cur[pos] = left;
      out.push_back(cur);
      return;
    }
    for (int v = left; v >= 0; --v) {
      cur[pos] = v;
      rec(pos + 1, left - v);
    }
  };
  for (int d = 0; d <= p; ++d) rec(0, d);
  return out;
}

static double factorial(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= i;
  return f;
}

// E[psi_a psi_b psi_c] for orthonormal probabilists' Hermite polynomials:
// nonzero only when a+b+c is even and the half-sum s is at least each index,
// then sqrt(a! b! c!) / ((s-a)! (s-b)! (s-c)!).
double hermite_triple(int a, int b, int c) {
  int tot = a + b + c;
  if (tot & 1) return 0.0;
  int s = tot / 2;
  if (s < a || s < b || s < c) return 0.0;
  return std::sqrt(factorial(a) * factorial(b) * factorial(c)) /
         (factorial(s - a) * factorial(s - b) * factorial(s - c));
}

// All nonzero [G_k]_{ij} = prod_n t(i_n, j_n, k_n) (Sec. 2.2), ordered by
// (k, i, j).  A nonzero needs |i_n - j_n| <= k_n <= i_n + j_n in every
// variable, which prunes the k loop per (i, j).
std::vector<Triple> triple_list(const std::vector<std::vector<int>>& Jp,
                                const std::vector<std::vector<int>>& Jq) {
  std::vector<Triple> out;
  const int M = Jp.empty() ? 0 : (int)Jp[0].size();
  for (int k = 0; k < (int)Jq.size(); ++k) {
    for (int i = 0; i < (int)Jp.size(); ++i) {
      for (int j = 0; j < (int)Jp.size(); ++j) {
        double v = 1.0;
        for (int m = 0; m < M && v != 0.0; ++m) v *= hermite_triple(Jp[i][m], Jp[j][m], Jq[k][m]);
        if (v != 0.0) out.push_back({k, i, j, v});
      }
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// KL expansion (Sec. 2.1).  1D Galerkin with P1 hats on the n-element grid:
// C e = lambda M e, C_ij = int int c(x,x') phi_i phi_j with 4-point
// Gauss-Legendre on every element pair, M the exact P1 mass.  Reduced to a
// standard symmetric problem with the Cholesky factor of the tridiagonal M
// and solved by cyclic Jacobi rotations.
// ---------------------------------------------------------------------------
namespace {

double kernel1d(int cov, double corr_len, double d) {
  if (cov == SG_COV_EXP_L1) return std::exp(-std::fabs(d) / corr_len);
  return std::exp(-(d * d) / (corr_len * corr_len));
}

// cyclic Jacobi on a dense symmetric matrix A (row-major, m x m); on return
// A's diagonal holds eigenvalues and Q (row-major) the eigenvectors in columns
void jacobi_eigen(std::vector<double>& A, int m, std::vector<double>& Q) {
  Q.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * m + j]; };
  double fro = 0.0;
  for (double x : A) fro += x * x;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += at(i, j) * at(i, j);
    if (std::sqrt(off) <= 1e-17 * fro) break;
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        double apq = at(p, q);
        if (apq == 0.0) continue;
        double app = at(p, p), aqq = at(q, q);
        if (sweep > 3 && std::fabs(app) + 100.0 * std::fabs(apq) == std::fabs(app) &&
            std::fabs(aqq) + 100.0 * std::fabs(apq) == std::fabs(aqq)) {
          at(p, q) = at(q, p) = 0.0;  // below rounding of both diagonal entries
          continue;
        }
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < m; ++r) {
          double arp = at(r, p), arq = at(r, q);
          at(r, p) = c * arp - s * arq;
          at(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < m; ++r) {
          double apr = at(p, r), aqr = at(q, r);
          at(p, r) = c * apr - s * aqr;
          at(q, r) = s * apr + c * aqr;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        for (int r = 0; r < m; ++r) {
          double qrp = Q[(size_t)r * m + p], qrq = Q[(size_t)r * m + q];
          Q[(size_t)r * m + p] = c * qrp - s * qrq;
          Q[(size_t)r * m + q] = s * qrp + c * qrq;
        }
      }
    }
  }
}

}  // namespace

KL karhunen_loeve(int n, int cov, double corr_len, double sigma, int M) {
  const int m = n + 1;
  const double h = 1.0 / n;
  // 4-point Gauss-Legendre on [0,1]
  const double gx[4] = {0.5 * (1.0 - 0.8611363115940526), 0.5 * (1.0 - 0.3399810435848563),
                        0.5 * (1.0 + 0.3399810435848563), 0.5 * (1.0 + 0.8611363115940526)};
  const double gw[4] = {0.5 * 0.3478548451374538, 0.5 * 0.6521451548625461,
                        0.5 * 0.6521451548625461, 0.5 * 0.3478548451374538};
  std::vector<double> C((size_t)m * m, 0.0);
  for (int e = 0; e < n; ++e) {
    for (int f = 0; f < n; ++f) {
      for (int a = 0; a < 4; ++a) {
        double x = (e + gx[a]) * h, wa = gw[a] * h;
        double pe[2] = {1.0 - gx[a], gx[a]};
        for (int b = 0; b < 4; ++b) {
          double y = (f + gx[b]) * h, wb = gw[b] * h;
          double pf[2] = {1.0 - gx[b], gx[b]};
          double kv = kernel1d(cov, corr_len, x - y) * wa * wb;
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) C[(size_t)(e + i) * m + (f + j)] += kv * pe[i] * pf[j];
        }
      }
    }
  }
  // symmetrise against rounding in the accumulation order
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      double s = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
      C[(size_t)i * m + j] = C[(size_t)j * m + i] = s;
    }
  // Cholesky of the tridiagonal mass: diag d (h/3 at ends, 2h/3 inside), off h/6
  std::vector<double> Ld(m), Lo(m, 0.0);  // L = bidiagonal, Lo[i] = L(i, i-1)
  for (int i = 0; i < m; ++i) {
    double dii = (i == 0 || i == m - 1) ? h / 3.0 : 2.0 * h / 3.0;
    if (i > 0) {
      Lo[i] = (h / 6.0) / Ld[i - 1];
      dii -= Lo[i] * Lo[i];
    }
    Ld[i] = std::sqrt(dii);
  }
  // B = L^{-1} C L^{-T}: forward substitution on columns, then on rows
  auto fsolve = [&](std::vector<double>& X, bool rows) {
    for (int c = 0; c < m; ++c) {
      for (int i = 0; i < m; ++i) {
        double& xi = rows ? X[(size_t)c * m + i] : X[(size_t)i * m + c];
        double prev = (i > 0) ? (rows ? X[(size_t)c * m + i - 1] : X[(size_t)(i - 1) * m + c]) : 0.0;
        xi = (xi - (i > 0 ? Lo[i] * prev : 0.0)) / Ld[i];
      }
    }
  };
  std::vector<double> B = C;
  fsolve(B, false);  // L^{-1} C
  fsolve(B, true);   // (L^{-1} C) L^{-T}
  std::vector<double> Q;
  jacobi_eigen(B, m, Q);
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::vector<double> ev(m);
  for (int i = 0; i < m; ++i) ev[i] = B[(size_t)i * m + i];
  std::sort(order.begin(), order.end(), [&](int a, int b) { return ev[a] > ev[b]; });
  const int R = std::min(m, M + 1);
  std::vector<double> lam1(R);
  std::vector<std::vector<double>> E(R, std::vector<double>(m));
  for (int r = 0; r < R; ++r) {
    int c = order[r];
    lam1[r] = ev[c];
    // e = L^{-T} q  (back substitution with the bidiagonal L^T)
    std::vector<double>& e = E[r];
    for (int i = m - 1; i >= 0; --i) {
      double v = Q[(size_t)i * m + c];
      if (i < m - 1) v -= Lo[i + 1] * e[i + 1];
      e[i] = v / Ld[i];
    }
    double mx = 0.0;
    for (double x : e) mx = std::max(mx, std::fabs(x));
    int idx = 0;
    if (std::fabs(e[0]) < 1e-12 * mx)
      while (idx < m && std::fabs(e[idx]) < 1e-12 * mx) ++idx;
    if (e[idx] < 0)
      for (double& x : e) x = -x;
  }
  // leading tensor pairs: descending symmetric key min*max; a run of keys
  // within 1e-10 of its first key is a tie, broken by smaller max(r,s), then
  // r > s first, then smaller min(r,s)
  struct Cand { double key; int r, s; };
  std::vector<Cand> cand;
  for (int r = 0; r < R; ++r)
    for (int s = 0; s < R; ++s)
      cand.push_back({std::min(lam1[r], lam1[s]) * std::max(lam1[r], lam1[s]), r, s});
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.key > b.key; });
  std::vector<Cand> chosen;
  for (size_t i = 0; i < cand.size() && (int)chosen.size() < M;) {
    size_t j = i + 1;
    while (j < cand.size() && std::fabs(cand[i].key - cand[j].key) <= 1e-10 * std::fabs(cand[i].key)) ++j;
    std::vector<Cand> run(cand.begin() + i, cand.begin() + j);
    std::sort(run.begin(), run.end(), [](const Cand& a, const Cand& b) {
      int ma = std::max(a.r, a.s), mb = std::max(b.r, b.s);
      if (ma != mb) return ma < mb;
      int ga = a.r > a.s ? 0 : 1, gb = b.r > b.s ? 0 : 1;
      if (ga != gb) return ga < gb;
      return std::min(a.r, a.s) < std::min(b.r, b.s);
    });
    for (auto& c : run) chosen.push_back(c);
    i = j;
  }
  chosen.resize(M);
  KL kl;
  kl.e1 = E;
  const int Nq = 4 * n * n;
  kl.gq.assign((size_t)M * Nq, 0.0);
  const double g0 = 0.5 * (1.0 - 1.0 / std::sqrt(3.0)), g1 = 0.5 * (1.0 + 1.0 / std::sqrt(3.0));
  const double gp[2] = {g0, g1};
  for (int t = 0; t < M; ++t) {
    int r = chosen[t].r, s = chosen[t].s;
    double lam = sigma * sigma * lam1[r] * lam1[s];
    kl.lam.push_back(lam);
    kl.pairs.push_back({r, s});
    double sq = std::sqrt(lam);
    for (int ey = 0; ey < n; ++ey)
      for (int ex = 0; ex < n; ++ex)
        for (int qy = 0; qy < 2; ++qy)
          for (int qx = 0; qx < 2; ++qx) {
            double bx = (1.0 - gp[qx]) * E[r][ex] + gp[qx] * E[r][ex + 1];
            double by = (1.0 - gp[qy]) * E[s][ey] + gp[qy] * E[s][ey + 1];
            kl.gq[(size_t)t * Nq + 4 * ((size_t)ey * n + ex) + 2 * qy + qx] = sq * bx * by;
          }
  }
  return kl;
}

// Field-split groupings (Sec. 3, eqs. P_preconditioner / P_group).
std::vector<std::vector<int>> make_splits(const std::vector<std::vector<int>>& J, int grouping) {
  const int P = (int)J.size(), M = (int)J[0].size();
  std::vector<std::vector<int>> out;
  if (grouping == SG_GROUP_PERMODE) {
    for (int i = 0; i < P; ++i) out.push_back({i});
    return out;
  }
  if (grouping == SG_GROUP_ALL) {
    out.emplace_back(P);
    for (int i = 0; i < P; ++i) out[0][i] = i;
    return out;
  }
  if (grouping == SG_GROUP_KLVAR || grouping == SG_GROUP_KLVAR_MEANSEP) {
    std::vector<std::vector<int>> byvar(M);
    std::vector<int> mean;
    for (int i = 0; i < P; ++i) {
      int first = -1;
      for (int m = 0; m < M; ++m)
        if (J[i][m] != 0) { first = m; break; }
      if (first < 0) mean.push_back(i); else byvar[first].push_back(i);
    }
    if (grouping == SG_GROUP_KLVAR_MEANSEP) out.push_back(mean);
    else byvar[0].insert(byvar[0].begin(), mean.begin(), mean.end());
    for (auto& g : byvar)
      if (!g.empty()) out.push_back(g);
    if (out.empty() || out[0].empty()) out.erase(out.begin());
    return out;
  }
  if (grouping == SG_GROUP_FG) {
    int p = 0;
    for (auto& a : J) {
      int s = 0;
      for (int x : a) s += x;
      p = std::max(p, s);
    }
    for (int g = 0; g <= p; ++g) {
      std::vector<int> mem;
      for (int i = 0; i < P; ++i)
        if (J[i][0] == g) mem.push_back(i);
      if (mem.empty()) continue;
      bool opens = (M * g <= p);   // (g, ..., g) is in J(p)
      if (opens || out.empty()) out.push_back(mem);
      else out.back().insert(out.back().end(), mem.begin(), mem.end());
    }
    return out;
  }
  throw Error(SG_ERR_INVALID_ARG, "unknown grouping");
}

}  // namespace sg
