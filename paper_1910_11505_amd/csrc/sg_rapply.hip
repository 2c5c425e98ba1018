// Register-resident factored SG apply for small chaos spaces (P <= 35).
//
// The same operator as the factored tile kernel (sum_k a_k G_k = a_min I +
// w T T^T, exact for q >= 2p; see FRowSetDev), with the chaos structure of
// J(M, p) generated at compile time: every multi-index, monomial recursion
// and (gamma <= alpha) pair is a constant, so the per-point contraction runs
// entirely in registers with no index arithmetic.  One wavefront per
// 4 x 4-element tile, one Gauss point per lane:
//   1. nodal values of the tile (5 x 5 nodes, every mode) -> LDS;
//   2. per lane: scaled gradients G^_alpha = s_alpha grad U_alpha for the
//      column modes (zero for the others), w(x_q), scaled monomials
//      m_delta = g^delta / delta!;
//   3. step 1 in place, gamma in graded order: Vbar_gamma = s_gamma^-2
//      sum_{alpha >= gamma} m_(alpha-gamma) G^_alpha (only alpha of higher
//      degree or gamma itself are read, none of them overwritten yet);
//   4. step 2 for the output rows: flux_beta = s_beta w sum_{gamma <= beta}
//      m_(beta-gamma) Vbar_gamma + a_min grad U_beta (column rows only); the
//      four corner contributions (1/4) grad phi_a . flux of each element are
//      reduce-scattered over the element's four lanes -> LDS;
//   5. the tile's 25 node sums per row, in a fixed order -> out (owned nodes)
//      and the edge buffer (right/top edge, corner) for the fixup.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int rc_binom(int n, int k) {
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

template <int M, int p>
constexpr int rc_pairs() {
  // number of (gamma <= alpha) pairs over J(p): sum over alpha of prod (alpha_n + 1)
  // (enumerated below; counted the same way)
  int cnt = 0;
  int cur[M] = {};
  for (int d = 0; d <= p; ++d) {
    for (int n = 0; n < M; ++n) cur[n] = 0;
    cur[0] = d;
    for (;;) {
      int prod = 1;
      for (int n = 0; n < M; ++n) prod *= cur[n] + 1;
      cnt += prod;
      int i = M - 2;
      while (i >= 0 && cur[i] == 0) --i;
      if (i < 0) break;
      int rest = 0;
      for (int n = i + 1; n < M; ++n) rest += cur[n];
      cur[i]--;
      cur[i + 1] = rest + 1;
      for (int n = i + 2; n < M; ++n) cur[n] = 0;
    }
  }
  return cnt;
}

template <int M, int p>
struct RTab {
  static constexpr int P = rc_binom(M + p, p);
  static constexpr int NT = rc_pairs<M, p>();
  int J[P][M] = {};
  int par[P] = {}, var[P] = {};
  double inv[P] = {}, s[P] = {}, is2[P] = {};
  // step 1, grouped by gamma: alpha and delta of every pair
  int p1[P + 1] = {}, a1[NT] = {}, d1[NT] = {};
  // step 2, grouped by beta: gamma and delta of every pair
  int p2[P + 1] = {}, g2[NT] = {}, d2[NT] = {};
};

template <int M, int p>
constexpr RTab<M, p> rc_make() {
  RTab<M, p> T{};
  constexpr int P = RTab<M, p>::P;
  // J(p): graded, descending lexicographic inside a degree
  int k = 0;
  int cur[M] = {};
  for (int d = 0; d <= p; ++d) {
    for (int n = 0; n < M; ++n) cur[n] = 0;
    cur[0] = d;
    for (;;) {
      for (int n = 0; n < M; ++n) T.J[k][n] = cur[n];
      ++k;
      int i = M - 2;
      while (i >= 0 && cur[i] == 0) --i;
      if (i < 0) break;
      int rest = 0;
      for (int n = i + 1; n < M; ++n) rest += cur[n];
      cur[i]--;
      cur[i + 1] = rest + 1;
      for (int n = i + 2; n < M; ++n) cur[n] = 0;
    }
  }
  auto find = [&](const int* v) {
    for (int i = 0; i < P; ++i) {
      bool eq = true;
      for (int n = 0; n < M; ++n) eq = eq && T.J[i][n] == v[n];
      if (eq) return i;
    }
    return -1;
  };
  // sqrt(k!) for k <= 6
  const double sq[7] = {1.0, 1.0, 1.4142135623730951, 2.449489742783178, 4.898979485566356,
                        10.954451150103322, 26.832815729997478};
  for (int i = 0; i < P; ++i) {
    double s = 1.0;
    for (int n = 0; n < M; ++n) s *= sq[T.J[i][n]];
    T.s[i] = s;
    T.is2[i] = 1.0 / (s * s);
    int n = 0;
    while (n < M && T.J[i][n] == 0) ++n;
    if (n == M) continue;
    int pv[M] = {};
    for (int t = 0; t < M; ++t) pv[t] = T.J[i][t];
    pv[n]--;
    T.par[i] = find(pv);
    T.var[i] = n;
    T.inv[i] = 1.0 / T.J[i][n];
  }
  // pairs gamma <= alpha
  int t1 = 0;
  for (int gm = 0; gm < P; ++gm) {
    T.p1[gm] = t1;
    for (int a = 0; a < P; ++a) {
      bool le = true;
      int de[M] = {};
      for (int n = 0; n < M; ++n) {
        le = le && T.J[gm][n] <= T.J[a][n];
        de[n] = T.J[a][n] - T.J[gm][n];
      }
      if (!le) continue;
      T.a1[t1] = a;
      T.d1[t1] = find(de);
      ++t1;
    }
  }
  T.p1[P] = t1;
  int t2 = 0;
  for (int b = 0; b < P; ++b) {
    T.p2[b] = t2;
    for (int gm = 0; gm < P; ++gm) {
      bool le = true;
      int de[M] = {};
      for (int n = 0; n < M; ++n) {
        le = le && T.J[gm][n] <= T.J[b][n];
        de[n] = T.J[b][n] - T.J[gm][n];
      }
      if (!le) continue;
      T.g2[t2] = gm;
      T.d2[t2] = find(de);
      ++t2;
    }
  }
  T.p2[P] = t2;
  return T;
}

template <int M, int p>
struct RTabHolder {
  static constexpr RTab<M, p> v = rc_make<M, p>();
};

__device__ __forceinline__ double r_gauss_pt(int i) {
  return i ? 0.78867513459481288225 : 0.21132486540518711775;
}

inline int r_cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

template <int M, int p>
__device__ __forceinline__ void rapply_tile(double* smem, int tile, int n, double mu,
                                            double a_min, const double* __restrict__ g,
                                            const RApplyRows& rr, const double* __restrict__ U,
                                            int64_t Nh, const double* __restrict__ rin,
                                            double beta, double sgn, double* __restrict__ out,
                                            double* __restrict__ edge) {
  constexpr const RTab<M, p>& T = RTabHolder<M, p>::v;
  constexpr int P = RTab<M, p>::P;
  double* sN = smem;             // [P][25] nodal values
  double* sC = smem + P * 25;    // [nrows][64] corner contributions
  const int nt = n / kTileE, ntiles = nt * nt;
  const int tx = tile % nt, ty = tile / nt;
  const int x0 = tx * kTileE, y0 = ty * kTileE;
  const int lane = threadIdx.x;
  const int m = n - 1;
  const int64_t Nq = (int64_t)4 * n * n;
  const uint64_t colmask = rr.colmask, rowmask = rr.rowmask;

  // 1. nodal values of the column modes (all loads in flight at once)
  constexpr int NL = (P * 25 + 63) / 64;
  double v[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = lane + 64 * u;
    const int c = min(idx / 25, P - 1), nd = idx - (idx / 25) * 25;
    const int gx = x0 + nd % 5, gy = y0 + nd / 5;
    const bool ok = idx < P * 25 && ((colmask >> c) & 1) && gx >= 1 && gx <= m && gy >= 1 && gy <= m;
    v[u] = ok ? U[(int64_t)c * Nh + (int64_t)(gy - 1) * m + (gx - 1)] : 0.0;
  }
  double gv[M];
#pragma unroll
  for (int nn = 0; nn < M; ++nn) gv[nn] = g[(int64_t)nn * Nq + (int64_t)tile * kTileQ + lane];
#pragma unroll
  for (int u = 0; u < NL; ++u)
    if (lane + 64 * u < P * 25) sN[lane + 64 * u] = v[u];
  __syncthreads();

  // 2. gradients, w, monomials
  const int el = lane >> 2, ql = lane & 3;
  const int ex = el & 3, ey = el >> 2;
  const double xi = r_gauss_pt(ql & 1), eta = r_gauss_pt(ql >> 1);
  double G[P][2];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    if (!((colmask >> a) & 1)) {  // not a column of this block
      G[a][0] = G[a][1] = 0.0;
      continue;
    }
    const double* u = sN + a * 25;
    const double u00 = u[ey * 5 + ex], u10 = u[ey * 5 + ex + 1];
    const double u01 = u[(ey + 1) * 5 + ex], u11 = u[(ey + 1) * 5 + ex + 1];
    G[a][0] = T.s[a] * ((1.0 - eta) * (u10 - u00) + eta * (u11 - u01));
    G[a][1] = T.s[a] * ((1.0 - xi) * (u01 - u00) + xi * (u11 - u10));
  }
  double s2 = 0.0;
#pragma unroll
  for (int nn = 0; nn < M; ++nn) s2 = fma(gv[nn], gv[nn], s2);
  const double w = exp(mu + 0.5 * s2);
  double mono[P];
  mono[0] = 1.0;
#pragma unroll
  for (int d = 1; d < P; ++d) mono[d] = mono[T.par[d]] * gv[T.var[d]] * T.inv[d];

  // 3. step 1 in place
  // gamma outside the block's set: never read by step 2, or zero (then no column
  // lies above it, so its slot already holds zero)
  const uint64_t gammask = rr.gammask;
#pragma unroll
  for (int gm = 0; gm < P; ++gm) {
    if (!((gammask >> gm) & 1)) continue;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int t = T.p1[gm]; t < T.p1[gm + 1]; ++t) {
      sx = fma(mono[T.d1[t]], G[T.a1[t]][0], sx);
      sy = fma(mono[T.d1[t]], G[T.a1[t]][1], sy);
    }
    G[gm][0] = sx * T.is2[gm];
    G[gm][1] = sy * T.is2[gm];
  }

  // 4. step 2 and the corner contributions of every output row
  double gpx[4], gpy[4];
#pragma unroll
  for (int a4 = 0; a4 < 4; ++a4) {
    const int ax = a4 & 1, ay = a4 >> 1;
    gpx[a4] = 0.25 * (ax ? 1.0 : -1.0) * (ay ? eta : 1.0 - eta);
    gpy[a4] = 0.25 * (ay ? 1.0 : -1.0) * (ax ? xi : 1.0 - xi);
  }
#pragma unroll
  for (int b = 0; b < P; ++b) {
    if (!((rowmask >> b) & 1)) continue;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int t = T.p2[b]; t < T.p2[b + 1]; ++t) {
      sx = fma(mono[T.d2[t]], G[T.g2[t]][0], sx);
      sy = fma(mono[T.d2[t]], G[T.g2[t]][1], sy);
    }
    const double sr = T.s[b] * w;
    double fx = sr * sx, fy = sr * sy;
    if ((colmask >> b) & 1) {
      // a_min grad U_beta from the nodal values (the gradient slot now holds Vbar)
      const double* u = sN + b * 25;
      const double u00 = u[ey * 5 + ex], u10 = u[ey * 5 + ex + 1];
      const double u01 = u[(ey + 1) * 5 + ex], u11 = u[(ey + 1) * 5 + ex + 1];
      fx = fma(a_min, (1.0 - eta) * (u10 - u00) + eta * (u11 - u01), fx);
      fy = fma(a_min, (1.0 - xi) * (u01 - u00) + xi * (u11 - u10), fy);
    }
    double t4[4];
#pragma unroll
    for (int a4 = 0; a4 < 4; ++a4) t4[a4] = gpx[a4] * fx + gpy[a4] * fy;
    // reduce-scatter over the element's four lanes: lane ql ends with corner ql
    const bool hi2 = (ql & 2) != 0, hi1 = (ql & 1) != 0;
    double k0 = hi2 ? t4[2] : t4[0], k1 = hi2 ? t4[3] : t4[1];
    const double x0v = hi2 ? t4[0] : t4[2], x1v = hi2 ? t4[1] : t4[3];
    k0 += __shfl_xor(x0v, 2);
    k1 += __shfl_xor(x1v, 2);
    double kk = hi1 ? k1 : k0;
    kk += __shfl_xor(hi1 ? k0 : k1, 1);
    sC[rr.slot[b] * 64 + lane] = kk;
  }
  __syncthreads();

  // 5. node sums: corner 3 of (x-1, y-1), 2 of (x, y-1), 1 of (x-1, y), 0 of (x, y)
  const int nrows = rr.nrows;
  for (int idx = lane; idx < nrows * 25; idx += 64) {
    const int slot = idx / 25, nd = idx - slot * 25;
    const int nx = nd % 5, ny = nd / 5;
    const double* c = sC + slot * 64;
    double sum = 0.0;
    if (nx >= 1 && ny >= 1) sum += c[((ny - 1) * 4 + nx - 1) * 4 + 3];
    if (nx <= 3 && ny >= 1) sum += c[((ny - 1) * 4 + nx) * 4 + 2];
    if (nx >= 1 && ny <= 3) sum += c[(ny * 4 + nx - 1) * 4 + 1];
    if (nx <= 3 && ny <= 3) sum += c[(ny * 4 + nx) * 4 + 0];
    if (nx <= 3 && ny <= 3) {
      const int gx = x0 + nx, gy = y0 + ny;
      if (gx >= 1 && gy >= 1) {
        const int64_t node = (int64_t)(gy - 1) * m + (gx - 1);
        double base = 0.0;
        if (beta != 0.0) base = beta * rin[(int64_t)rr.mode[slot] * Nh + node];
        out[(int64_t)slot * Nh + node] = base + sgn * sum;
      }
    } else {
      const int e = (nx == 4 && ny == 4) ? 8 : (nx == 4 ? ny : 4 + nx);
      edge[((int64_t)slot * ntiles + tile) * kEdgeVals + e] = sum;
    }
  }
}

template <int M, int p>
__global__ __launch_bounds__(64) void rapply_kernel(int n, double mu, double a_min,
                                                    const double* __restrict__ g, RApplyRows rr,
                                                    const double* __restrict__ U, int64_t Nh,
                                                    const double* __restrict__ rin, double beta,
                                                    double sgn, double* __restrict__ out,
                                                    double* __restrict__ edge) {
  extern __shared__ double smem[];
  const int nt = n / kTileE;
  rapply_tile<M, p>(smem, xcd_tile(blockIdx.x, nt * nt), n, mu, a_min, g, rr, U, Nh, rin, beta,
                    sgn, out, edge);
}

// (instance, tile) items of instances sharing one (M, p)
template <int M, int p>
__global__ __launch_bounds__(64) void brapply_kernel(const BInst* __restrict__ Is,
                                                     const BState* __restrict__ Ss,
                                                     const BItem* __restrict__ items, int nitems,
                                                     int rowset, int src, int rin, int dst,
                                                     double beta, double sgn, int gate) {
  extern __shared__ double smem[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) continue;
    __syncthreads();  // the previous item is done with the LDS
    const RApplyRows& rr = rowset == 0 ? I.rfull : I.rpart[rowset];
    rapply_tile<M, p>(smem, w.local, I.n, I.mu, I.amin, I.gq, rr, bbuf(I, S, src), I.Nh,
                      rin >= 0 ? bbuf(I, S, rin) : nullptr, beta, sgn, bbuf(I, S, dst), I.edge);
  }
}

size_t rapply_lds_bytes(int P, int nrows) { return 8 * ((size_t)P * 25 + (size_t)nrows * 64); }

#define SG_RAPPLY_LIST(X) \
  X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(3, 1) X(3, 2) X(3, 3) \
  X(3, 4) X(4, 1) X(4, 2) X(4, 3) X(5, 1) X(5, 2) X(6, 1) X(6, 2)

bool rapply_supported(int M, int p) {
#define SG_RAPPLY_SUP(MM, PP) if (M == MM && p == PP) return true;
  SG_RAPPLY_LIST(SG_RAPPLY_SUP)
#undef SG_RAPPLY_SUP
  return false;
}

template <int M, int p>
static bool rapply_check(const std::vector<std::vector<int>>& Jp) {
  constexpr const RTab<M, p>& T = RTabHolder<M, p>::v;
  if ((int)Jp.size() != RTab<M, p>::P) return false;
  for (int i = 0; i < RTab<M, p>::P; ++i)
    for (int nn = 0; nn < M; ++nn)
      if (Jp[i][nn] != T.J[i][nn]) return false;
  return true;
}

bool rapply_matches(int M, int p, const std::vector<std::vector<int>>& Jp) {
#define SG_RAPPLY_CHK(MM, PP) if (M == MM && p == PP) return rapply_check<MM, PP>(Jp);
  SG_RAPPLY_LIST(SG_RAPPLY_CHK)
#undef SG_RAPPLY_CHK
  return false;
}

void launch_rapply(hipStream_t s, int M, int p, int n, double mu, double a_min, const double* g,
                   const RApplyRows& rr, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge) {
  const int nt = n / kTileE, ntiles = nt * nt;
  const int P = (int)rc_binom(M + p, p);
  if (rr.nrows < 1 || rr.nrows > P) throw Error(SG_ERR_INTERNAL, "register apply: bad rows");
  const size_t lds = rapply_lds_bytes(P, rr.nrows);
#define SG_RAPPLY_LAUNCH(MM, PP)                                                               \
  if (M == MM && p == PP) {                                                                    \
    hipLaunchKernelGGL((rapply_kernel<MM, PP>), dim3(ntiles), dim3(64), lds, s, n, mu, a_min, \
                       g, rr, U, Nh, rin, beta, sgn, out, edge);                               \
  } else
  SG_RAPPLY_LIST(SG_RAPPLY_LAUNCH) { throw Error(SG_ERR_INTERNAL, "register apply: (M, p)"); }
#undef SG_RAPPLY_LAUNCH
  launch_apply_fixup(s, n, rr.nrows, sgn, edge, out, Nh);
}

void launch_brapply(hipStream_t s, int M, int p, size_t lds, const BInst* I, const BState* st,
                    const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                    double beta, double sgn, int gate) {
  if (nitems <= 0) return;
  const int grid = std::min(nitems, 256 * 8);
#define SG_BRAPPLY_LAUNCH(MM, PP)                                                             \
  if (M == MM && p == PP) {                                                                   \
    hipLaunchKernelGGL((brapply_kernel<MM, PP>), dim3(grid), dim3(64), lds, s, I, st, items, \
                       nitems, rowset, src, rin, dst, beta, sgn, gate);                       \
  } else
  SG_RAPPLY_LIST(SG_BRAPPLY_LAUNCH) { throw Error(SG_ERR_INTERNAL, "batched register apply: (M, p)"); }
#undef SG_BRAPPLY_LAUNCH
}

}  // namespace sg
