// Register-resident factored SG apply: every chaos space with M <= 6, p <= 4
// (rapply_tile for P <= 35 as described here; rapply_stream_tile, further
// down, for 35 < P <= 210).
//
// The same operator as the factored tile kernel (sum_k a_k G_k = a_min I +
// w T T^T, exact for q >= 2p; see FRowSetDev), with the chaos structure of
// J(M, p) generated at compile time: every multi-index, monomial recursion
// and (gamma <= alpha) pair is a constant, so the per-point contraction runs
// entirely in registers with no index arithmetic.  One workgroup of two
// wavefronts per 4 x 4-element tile, one Gauss point per lane; both steps are
// linear and act on each gradient component separately, so wavefront c
// carries component c of every gradient:
//   1. nodal values of the tile (5 x 5 nodes, every mode) -> LDS;
//   2. per lane: component c of the scaled gradients G^_alpha = s_alpha grad
//      U_alpha for the column modes (zero for the others), w(x_q), scaled
//      monomials m_delta = g^delta / delta!;
//   3. step 1 in place, gamma in graded order: Vbar_gamma = s_gamma^-2
//      sum_{alpha >= gamma} m_(alpha-gamma) G^_alpha (only alpha of higher
//      degree or gamma itself are read, none of them overwritten yet);
//   4. step 2 for the output rows: flux_beta = s_beta w sum_{gamma <= beta}
//      m_(beta-gamma) Vbar_gamma + a_min grad U_beta (column rows only); the
//      four corner contributions (1/4) d_c phi_a flux_c of each element are
//      reduce-scattered over the element's four lanes (quad permutations) ->
//      LDS, one array per component (the nodal values are dead by then);
//   5. the tile's 25 node sums per row (both components, fixed order) -> out
//      (owned nodes) and the edge buffer (right/top edge, corner) for the fixup.
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

// position of multi-index a in J(p) ordered by degree, descending
// lexicographic inside a degree: the indices of lower degree, then for each
// position i those of the same degree that agree before i and are larger at i
// (compositions of the remainder over the later positions)
constexpr int rc_rank(const int* a, int M) {
  int d = 0;
  for (int n = 0; n < M; ++n) d += a[n];
  int idx = d == 0 ? 0 : rc_binom(M + d - 1, d - 1);
  int rem = d;
  for (int i = 0; i < M - 1; ++i) {
    const int k = M - i - 1;
    for (int v = a[i] + 1; v <= rem; ++v) idx += rc_binom(rem - v + k - 1, k - 1);
    rem -= a[i];
  }
  return idx;
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
  auto find = [&](const int* v) { return rc_rank(v, M); };
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

// Step-1 pairs (gamma, delta) of each degree-p mode alpha with gamma of degree
// below p, grouped by alpha (the pairs of the gamma-grouped table with that
// alpha, in the same gamma order).
template <int M, int p>
struct RTabTop {
  static constexpr int P = RTab<M, p>::P;
  static constexpr int PN = rc_binom(M + p - 1, p - 1);  // modes of degree below p
  static constexpr int NT = RTab<M, p>::NT;
  int pq[P - PN + 1] = {}, qg[NT] = {}, qd[NT] = {};
};

template <int M, int p>
constexpr RTabTop<M, p> rc_make_top() {
  constexpr const RTab<M, p>& T = RTabHolder<M, p>::v;
  RTabTop<M, p> Q{};
  constexpr int P = RTabTop<M, p>::P, PN = RTabTop<M, p>::PN;
  int k = 0;
  for (int a = PN; a < P; ++a) {
    Q.pq[a - PN] = k;
    for (int gm = 0; gm < PN; ++gm)
      for (int t = T.p1[gm]; t < T.p1[gm + 1]; ++t)
        if (T.a1[t] == a) {
          Q.qg[k] = gm;
          Q.qd[k] = T.d1[t];
          ++k;
        }
  }
  Q.pq[P - PN] = k;
  return Q;
}

template <int M, int p>
struct RTabTopHolder {
  static constexpr RTabTop<M, p> v = rc_make_top<M, p>();
};

__device__ __forceinline__ double r_gauss_pt(int i) {
  return i ? 0.78867513459481288225 : 0.21132486540518711775;
}

}  // namespace

// value of lane (lane ^ K) of the lane's quad, K = 1 or 2 (DPP quad permutation;
// every lane of the wavefront active)
template <int K>
__device__ __forceinline__ double quad_xor(double v) {
  constexpr int ctrl = K == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

constexpr int kRThreads = 128;  // two wavefronts per tile

// Quadrature point, within its element, carried by a lane of wavefront c: lane
// bit 0 is the xi index and bit 1 the eta index for c = 0, the other way round
// for c = 1.  The contribution of a point's flux f to corner (ax, ay) of its
// element is s E f / 4, with (component x) s = -1, +1 for ax = 0, 1 and E =
// 1 - eta, eta for ay = 0, 1 (component y: x and y swapped), so a corner sum
// is a sign times one of two partial sums.  With this lane order both
// components build the partial sum with the lane two apart and apply the sign
// difference with the neighbour lane.
__device__ __forceinline__ int r_lane_qp(int lane, int comp) {
  const int q = lane & 3;
  return comp ? ((q & 1) << 1) | (q >> 1) : q;
}
// weights of a lane's flux: wc for the corner the lane ends up holding, wo for
// the one its partner two apart holds
__device__ __forceinline__ void r_corner_weights(int comp, int ql, double xi, double eta,
                                                 double& wc, double& wo) {
  const int qx = ql & 1, qy = ql >> 1;
  const double s4 = 0.25 * ((comp ? qy : qx) ? 1.0 : -1.0);
  wc = s4 * (comp ? (qx ? xi : 1.0 - xi) : (qy ? eta : 1.0 - eta));
  wo = s4 * (comp ? (qx ? 1.0 - xi : xi) : (qy ? 1.0 - eta : eta));
}

// Gradient component c at a lane's Gauss point from one nodal value per lane.
// Each lane of an element reads the corner (qx, qy) of its own point; in the
// lane order of r_lane_qp the neighbour lane then holds the other end of the
// lane's element edge along direction c, and the lane two apart the parallel
// edge, so with d = u - u[lane ^ 1]
//   x: (1 - eta)(u10 - u00) + eta (u11 - u01) = ga d + gb d[lane ^ 2]
//   y: (1 - xi)(u01 - u00) + xi (u11 - u10)   = ga d + gb d[lane ^ 2]
// with the edge weights and the sign of d folded into ga and gb.
struct RGrad {
  int oc;  // the lane's corner in the tile's 5x5 node block
  double ga, gb;
};
__device__ __forceinline__ RGrad r_grad_setup(int comp, int ql, int el, double xi, double eta) {
  const int qx = ql & 1, qy = ql >> 1;
  RGrad r;
  r.oc = (el >> 2) * 5 + (el & 3) + qx + 5 * qy;
  const double s = (comp ? qy : qx) ? 1.0 : -1.0;
  r.ga = s * (comp ? (qx ? xi : 1.0 - xi) : (qy ? eta : 1.0 - eta));
  r.gb = s * (comp ? (qx ? 1.0 - xi : xi) : (qy ? 1.0 - eta : eta));
  return r;
}
__device__ __forceinline__ double r_grad(const RGrad& r, const double* u) {
  const double v = u[r.oc];
  const double d = v - quad_xor<1>(v);
  return r.ga * d + r.gb * quad_xor<2>(d);
}

// Corner buffers: one row of 64 corner slots per output row, rows kCS apart
// and slot s at cpos(s), so that the node sums' reads (the same corner of
// elements four apart, the same slot of neighbouring rows) fall in different
// LDS banks.  cpos keeps the four slots of an element adjacent.
constexpr int kCS = 66;
__device__ __forceinline__ int cpos(int s) { return s + (s >> 5); }

// One of a tile's 25 nodes in the node sums: the lanes of the corner slots it
// adds (corner 3 of element (x-1, y-1), 2 of (x, y-1), 1 of (x-1, y), 0 of
// (x, y); -1 where the element lies outside the tile; the y part holds corners
// 1 and 2 swapped, see r_lane_qp), and where the sum goes: an owned node of
// the output, or a right/top edge or corner value of the edge buffer.
struct RNode {
  int i3, i2, i1, i0;
  bool owned, write;
  int64_t node;
  int e;
};
__device__ __forceinline__ RNode r_node(int nd, int x0, int y0, int m) {
  const int nx = nd % 5, ny = nd / 5;
  RNode q;
  q.i3 = nx >= 1 && ny >= 1 ? cpos(((ny - 1) * 4 + nx - 1) * 4 + 3) : -1;
  q.i2 = nx <= 3 && ny >= 1 ? cpos(((ny - 1) * 4 + nx) * 4 + 2) : -1;
  q.i1 = nx >= 1 && ny <= 3 ? cpos((ny * 4 + nx - 1) * 4 + 1) : -1;
  q.i0 = nx <= 3 && ny <= 3 ? cpos((ny * 4 + nx) * 4) : -1;
  q.owned = nx <= 3 && ny <= 3;
  const int gx = x0 + nx, gy = y0 + ny;
  q.write = q.owned && gx >= 1 && gy >= 1;
  q.node = (int64_t)(gy - 1) * m + (gx - 1);
  q.e = (nx == 4 && ny == 4) ? 8 : (nx == 4 ? ny : 4 + nx);
  return q;
}
// the node's sum over its corners in a fixed order, each the x part plus the y
// part; all eight reads are issued (absent corners read slot 0 and add +0.0,
// which leaves the sum's bits unchanged), so they wait once, not per corner
__device__ __forceinline__ double r_node_sum(const RNode& q, const double* c, const double* cy) {
  const int j3 = q.i3 >= 0 ? q.i3 : 0, j2 = q.i2 >= 0 ? q.i2 : 1;
  const int j1 = q.i1 >= 0 ? q.i1 : 0, j0 = q.i0 >= 0 ? q.i0 : 0;
  const double a3 = c[j3] + cy[j3], a2 = c[j2] + cy[j2 - 1];
  const double a1 = c[j1] + cy[j1 + 1], a0 = c[j0] + cy[j0];
  double sum = 0.0;
  sum += q.i3 >= 0 ? a3 : 0.0;
  sum += q.i2 >= 0 ? a2 : 0.0;
  sum += q.i1 >= 0 ? a1 : 0.0;
  sum += q.i0 >= 0 ? a0 : 0.0;
  return sum;
}

// output rows per corner-sum chunk of the streamed tile: the most that keep
// the tiles per CU the registers allow.  P = 56 and 84 fit six tiles (three
// wavefronts per SIMD) with 14 and 9 rows (26 KB of LDS each; 16 rows at
// P = 84 left two wavefronts per SIMD: 0.140 against 0.122 ms per 256x256
// apply); P = 70 is held to two wavefronts per SIMD by its registers and
// takes 16 rows, the larger spaces (one wavefront per SIMD) 24.  Fewer chunks
// mean fewer barriers and fuller node-sum passes (125 threads, five rows
// each): against 8 rows (16 above P = 84), 2% at P = 56, 1% at P = 70, 3.6%
// at P = 210 on 128x128, the same at P = 84.
constexpr int rchunk(int P) { return P == 84 ? 9 : P == 56 ? 14 : P == 70 ? 16 : P > 84 ? 24 : 8; }
constexpr int kRFence = 4;   // rows between its scheduling fences

// Field-split blocks known at compile time.  With the splits taken by the
// first KL variable a mode depends on (the mean with variable 0), the block of
// split V >= 1 has the modes whose first variable is V as rows and those whose
// first variable is below V as columns; which gammas it reads (below a row and
// below a column) follows.  A block kernel built on these tables drops every
// pair, gradient and row chunk the block does not need at compile time, where
// run-time masks can only skip whole modes.
// (internal linkage like the other tables, so that device code folds their
// reads instead of loading a symbol the host could rewrite)
namespace {
template <int M, int p>
struct RSel {
  static constexpr int P = RTab<M, p>::P;
  static constexpr int NT = RTab<M, p>::NT;
  int row[P] = {}, col[P] = {}, gam[P] = {};
  int chunk[(P + rchunk(P) - 1) / rchunk(P)] = {};
  // the block's own pair lists (the whole operator's, filtered):
  // step 1a: each gamma below p that the block reads, with its column alphas below p
  int n1 = 0, g1[P] = {}, p1[P + 1] = {}, a1[NT] = {}, d1[NT] = {};
  // step 1b: each column mode of degree p, with the gammas the block reads below it
  int nq = 0, qa[P] = {}, pq[P + 1] = {}, qg[NT] = {}, qd[NT] = {};
  // step 2: each row, with the gammas below p the block reads
  int p2[P + 1] = {}, g2[NT] = {}, d2[NT] = {};
};

template <int M, int p, int V>
constexpr RSel<M, p> rc_make_sel() {
  const RTab<M, p>& T = RTabHolder<M, p>::v;
  constexpr int P = RTab<M, p>::P;
  RSel<M, p> S{};
  int first[P] = {};
  for (int i = 0; i < P; ++i) {
    first[i] = 0;
    for (int n = M - 1; n >= 0; --n)
      if (T.J[i][n] != 0) first[i] = n;
  }
  for (int i = 0; i < P; ++i) {
    S.row[i] = first[i] == V;
    S.col[i] = first[i] < V;
    if (S.row[i]) S.chunk[i / rchunk(P)] = 1;
  }
  for (int g = 0; g < P; ++g) {
    bool br = false, bc = false;
    for (int i = 0; i < P; ++i) {
      bool le = true;
      for (int n = 0; n < M; ++n) le = le && T.J[g][n] <= T.J[i][n];
      if (le) {
        br = br || S.row[i];
        bc = bc || S.col[i];
      }
    }
    S.gam[g] = br && bc;
  }
  const RTabTop<M, p>& Q = RTabTopHolder<M, p>::v;
  constexpr int PN = RTabTop<M, p>::PN;
  int k = 0;
  for (int g = 0; g < PN; ++g) {
    if (!S.gam[g]) continue;
    S.g1[S.n1] = g;
    S.p1[S.n1] = k;
    for (int t = T.p1[g]; t < T.p1[g + 1]; ++t)
      if (T.a1[t] < PN && S.col[T.a1[t]]) {
        S.a1[k] = T.a1[t];
        S.d1[k] = T.d1[t];
        ++k;
      }
    ++S.n1;
  }
  S.p1[S.n1] = k;
  k = 0;
  for (int a = PN; a < P; ++a) {
    if (!S.col[a]) continue;
    S.qa[S.nq] = a;
    S.pq[S.nq] = k;
    for (int t = Q.pq[a - PN]; t < Q.pq[a - PN + 1]; ++t)
      if (S.gam[Q.qg[t]]) {
        S.qg[k] = Q.qg[t];
        S.qd[k] = Q.qd[t];
        ++k;
      }
    ++S.nq;
  }
  S.pq[S.nq] = k;
  k = 0;
  for (int b = 0; b < P; ++b) {
    S.p2[b] = k;
    if (!S.row[b]) continue;
    for (int t = T.p2[b]; t < T.p2[b + 1]; ++t)
      if (T.g2[t] < PN && S.gam[T.g2[t]]) {
        S.g2[k] = T.g2[t];
        S.d2[k] = T.d2[t];
        ++k;
      }
  }
  S.p2[P] = k;
  return S;
}

template <int M, int p, int V>
struct RSelHolder {
  static constexpr RSel<M, p> v = rc_make_sel<M, p, V>();
};
}  // namespace

// FULL: every mode is a row and a column, in order (the whole operator); the
// masks and slot tables are then compile-time constants.
template <int M, int p, bool FULL = false, int V = 0>
__device__ __forceinline__ void rapply_tile(double* smem, int tile, int n, double mu,
                                            double a_min, const double* __restrict__ g,
                                            const RApplyRows& rr, const double* __restrict__ U,
                                            int64_t Nh, const double* __restrict__ rin,
                                            double beta, double sgn, double* __restrict__ out,
                                            double* __restrict__ edge) {
  constexpr const RTab<M, p>& T = RTabHolder<M, p>::v;
  constexpr int P = RTab<M, p>::P;
  static_assert(P <= 64, "one mask word");
  constexpr uint64_t kAll = P >= 64 ? ~0ull : ((1ull << P) - 1);
  const int nrows = FULL ? P : rr.nrows;
  double* sN = smem;  // [P][25] nodal values (steps 1-2)
  double* sC = smem;  // [2][nrows][kCS] corner contributions (steps 4-5)
  const int nt = n / kTileE, ntiles = nt * nt;
  const int tx = tile % nt, ty = tile / nt;
  const int x0 = tx * kTileE, y0 = ty * kTileE;
  const int tid = threadIdx.x, lane = tid & 63;
  const int comp = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qp = r_lane_qp(lane, comp), pt = (lane & ~3) | qp;  // the lane's Gauss point
  const int m = n - 1;
  const int64_t Nq = (int64_t)4 * n * n;
  // (the column and gamma masks stay run-time values: known, the unrolled
  // gradient and step-1 code is scheduled with more values live than fit)
  const uint64_t colmask = rr.colmask[0], rowmask = FULL ? kAll : rr.rowmask[0];
  // output slot of each row, read once as whole words (uniform registers)
  uint32_t slotw[(P + 3) / 4];
#pragma unroll
  for (int k = 0; k < (P + 3) / 4; ++k)
    slotw[k] = FULL ? 0u : reinterpret_cast<const uint32_t*>(rr.slot)[k];
  auto slot_of = [&](int b) {
    return FULL ? b : (int)((slotw[b >> 2] >> (8 * (b & 3))) & 0xFFu);
  };

  // 1. nodal values of the column modes (all loads in flight at once)
  constexpr int NL = (P * 25 + kRThreads - 1) / kRThreads;
  double v[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = tid + kRThreads * u;
    const int c = min(idx / 25, P - 1), nd = idx - (idx / 25) * 25;
    const int gx = x0 + nd % 5, gy = y0 + nd / 5;
    const bool ok = idx < P * 25 && ((colmask >> c) & 1) && gx >= 1 && gx <= m && gy >= 1 && gy <= m;
    v[u] = ok ? U[(int64_t)c * Nh + (int64_t)(gy - 1) * m + (gx - 1)] : 0.0;
  }
  double gv[M];
#pragma unroll
  for (int nn = 0; nn < M; ++nn) gv[nn] = g[(int64_t)nn * Nq + (int64_t)tile * kTileQ + pt];
#pragma unroll
  for (int u = 0; u < NL; ++u)
    if (tid + kRThreads * u < P * 25) sN[tid + kRThreads * u] = v[u];
  __syncthreads();

  // 2. gradient component c (r_grad), w, monomials
  const int el = lane >> 2, ql = qp;
  const double xi = r_gauss_pt(ql & 1), eta = r_gauss_pt(ql >> 1);
  const RGrad rg = r_grad_setup(comp, ql, el, xi, eta);
  // V > 0: the field-split block of split V, rows, columns and gammas known at
  // compile time (RSel); its rows are never its columns
  static_assert(V >= 0 && (V == 0 || (V < M && !FULL)), "block selector");
  constexpr bool SEL = V > 0;
  constexpr const RSel<M, p>& S = RSelHolder<M, p, V>::v;
  double G[P], Gc[P];  // Gc: unscaled component, for the a_min term of column rows
  // no test of the run-time column mask: the nodal values of other modes were
  // stored as zeros, so their gradients are zero, and no branch separates the
  // modes' reads
#pragma unroll
  for (int a = 0; a < P; ++a) {
    const double d = (!SEL || S.col[a]) ? r_grad(rg, sN + a * 25) : 0.0;
    G[a] = T.s[a] * d;
    Gc[a] = d;
  }
  double s2 = 0.0;
#pragma unroll
  for (int nn = 0; nn < M; ++nn) s2 = fma(gv[nn], gv[nn], s2);
  const double w = exp(mu + 0.5 * s2);
  double mono[P];
  mono[0] = 1.0;
#pragma unroll
  for (int d = 1; d < P; ++d) mono[d] = mono[T.par[d]] * gv[T.var[d]] * T.inv[d];
  __syncthreads();  // both wavefronts are done with the nodal values

  // 3. step 1 in place
  // gamma outside the block's set: never read by step 2, or zero (then no column
  // lies above it, so its slot already holds zero)
  const uint64_t gammask = rr.gammask[0];
#pragma unroll
  for (int gm = 0; gm < P; ++gm) {
    if (SEL ? !S.gam[gm] : !((gammask >> gm) & 1)) continue;
    double sx = 0.0;
#pragma unroll
    for (int t = T.p1[gm]; t < T.p1[gm + 1]; ++t)
      if (!SEL || S.col[T.a1[t]]) sx = fma(mono[T.d1[t]], G[T.a1[t]], sx);
    G[gm] = sx * T.is2[gm];
  }
  // keep the scheduler from interleaving the phases (register pressure)
  __builtin_amdgcn_sched_barrier(0);

  // 4. step 2 and the corner contributions of every output row: the partial
  // sum with the lane two apart, then the signed sum with the neighbour lane
  // (see r_lane_qp); lane j of an element ends with its corner r_lane_qp(j, c)
  double wc, wo;
  r_corner_weights(comp, ql, xi, eta, wc, wo);
  double* sCc = sC + comp * nrows * kCS;
  const int lpos = cpos(lane);
#pragma unroll
  for (int b = 0; b < P; ++b) {
    if (SEL ? !S.row[b] : !((rowmask >> b) & 1)) continue;
    double sx = 0.0;
#pragma unroll
    for (int t = T.p2[b]; t < T.p2[b + 1]; ++t)
      if (!SEL || S.gam[T.g2[t]]) sx = fma(mono[T.d2[t]], G[T.g2[t]], sx);
    const double sr = T.s[b] * w;
    double f = sr * sx;
    if (FULL || (!SEL && ((colmask >> b) & 1))) f = fma(a_min, Gc[b], f);
    const double t = wc * f + quad_xor<2>(wo * f);
    sCc[slot_of(b) * kCS + lpos] = t - quad_xor<1>(t);
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();

  // 5. node sums: thread t takes node t % 25 of slots t / 25, t / 25 + 5, ...
  // (threads 125-127 have none), so a node's geometry is worked out once
  if (tid < 125) {
    const RNode q = r_node(tid % 25, x0, y0, m);
#pragma unroll
    for (int k = 0; k < (P + 4) / 5; ++k) {
      const int slot = tid / 25 + 5 * k;
      if (slot >= nrows) break;
      const double* c = sC + slot * kCS;
      const double sum = r_node_sum(q, c, c + nrows * kCS);
      if (q.owned) {
        if (q.write) {
          double base = 0.0;
          if (beta != 0.0) base = beta * rin[(int64_t)(FULL ? slot : rr.mode[slot]) * Nh + q.node];
          out[(int64_t)slot * Nh + q.node] = base + sgn * sum;
        }
      } else {
        edge[((int64_t)slot * ntiles + tile) * kEdgeVals + q.e] = sum;
      }
    }
  }
}

template <int M, int p, bool FULL, int V = 0>
__global__ __launch_bounds__(kRThreads, 2) void rapply_kernel(int n, double mu, double a_min,
                                                    const double* __restrict__ g, RApplyRows rr,
                                                    const double* __restrict__ U, int64_t Nh,
                                                    const double* __restrict__ rin, double beta,
                                                    double sgn, double* __restrict__ out,
                                                    double* __restrict__ edge) {
  extern __shared__ double smem[];
  const int nt = n / kTileE;
  rapply_tile<M, p, FULL, V>(smem, xcd_tile(blockIdx.x, nt * nt), n, mu, a_min, g, rr, U, Nh, rin,
                          beta, sgn, out, edge);
}

// (instance, tile) items of instances sharing one (M, p)
template <int M, int p>
__global__ __launch_bounds__(kRThreads) void brapply_kernel(const BInst* __restrict__ Is,
                                                     const BState* __restrict__ Ss,
                                                     const BItem* __restrict__ items, int nitems,
                                                     int rowset, int src, int rin, int dst,
                                                     double beta, double sgn, int gate) {
  extern __shared__ double smem[];
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) return;
    // read in place: the tile code loads the masks and slot words once into
    // uniform registers, the mode table only in the node sums
    const RApplyRows& rr = rowset == 0 ? I.rfull : I.rpart[rowset];
    rapply_tile<M, p>(smem, w.local, I.n, I.mu, I.amin, gptr(I.gq), rr, bbuf(I, S, src), I.Nh,
                      rin >= 0 ? bbuf(I, S, rin) : nullptr, beta, sgn, bbuf(I, S, dst),
                      gptr(I.edge));
  }
}

// ---------------------------------------------------------------------------
// The same operator for larger chaos spaces (35 < P <= 210), where the P
// gradients and P monomials of a point no longer fit a lane together.  It
// rests on the degree structure of the contraction: a step-1 output gamma of
// degree d needs m_delta with |delta| <= p - d, and a step-2 row beta needs a
// degree-p monomial only for its gamma = 0 term, so a degree-p mode alpha
// enters step 1 only through the Vbar_gamma below it and step 2 only through
// its own row (Vbar_alpha is its scaled gradient alone).
//  - Only the modes of degree below p keep their gradient (then Vbar) in
//    registers, and only the monomials of degree below p - 1; degree p - 1
//    and p monomials are formed where used from their parents (the same
//    products, in the same order, as the recurrence).
//  - Step 1 first sums the pairs with alpha of degree below p in place, then
//    streams the degree-p modes: each one's gradient is recomputed from the
//    nodal values (one read and two DPP exchanges) and added to every
//    Vbar_gamma below it (the pairs grouped by alpha, RTabTop).
//  - Step 2 recomputes a degree-p row's gradient for its gamma = beta term
//    and, for every row, the a_min term's gradient, through an offset the
//    compiler cannot equate with the gradient loop's; its monomials come from
//    copies of g it cannot equate with step 1's (either way it would keep
//    step-1 values alive through step 2 and spill).
//  - Output rows go in chunks of rchunk(P): corner sums to LDS, barrier, node
//    sums, barrier.  For the whole operator the rows carry no branches and are
//    scheduled kRFence at a time between fences.
// ---------------------------------------------------------------------------


template <int M, int p, bool FULL, int V = 0>
__device__ __forceinline__ void rapply_stream_tile(double* smem, int tile, int n, double mu,
                                                 double a_min, const double* __restrict__ g,
                                                 const RApplyRows& rr,
                                                 const double* __restrict__ U, int64_t Nh,
                                                 const double* __restrict__ rin, double beta,
                                                 double sgn, double* __restrict__ out,
                                                 double* __restrict__ edge) {
  constexpr const RTab<M, p>& T = RTabHolder<M, p>::v;
  constexpr const RTabTop<M, p>& Q = RTabTopHolder<M, p>::v;
  constexpr int P = RTab<M, p>::P;
  constexpr int PN = RTabTop<M, p>::PN;           // modes of degree below p
  constexpr int PL = rc_binom(M + p - 2, p - 2);  // monomials of degree below p - 1
  static_assert(P <= kRMax && p >= 2, "mask words, degree");
  static_assert(V >= 0 && V < M && !(FULL && V > 0), "block selector");
  // V > 0: the block of split V, rows, columns and gammas known at compile time
  constexpr bool SEL = V > 0;
  constexpr const RSel<M, p>& S = RSelHolder<M, p, V>::v;
  constexpr int SN1 = S.n1, SNQ = S.nq;
  double* sN = smem;            // [P][25] nodal values
  constexpr int kRChunk = rchunk(P);
  double* sC = sN + P * 25;     // [2][kRChunk][kCS] corner contributions of a row chunk
  const int nt = n / kTileE, ntiles = nt * nt;
  const int tx = tile % nt, ty = tile / nt;
  const int x0 = tx * kTileE, y0 = ty * kTileE;
  const int tid = threadIdx.x, lane = tid & 63;
  const int comp = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qp = r_lane_qp(lane, comp), pt = (lane & ~3) | qp;  // the lane's Gauss point
  const int m = n - 1;
  const int64_t Nq = (int64_t)4 * n * n;
  // Masks: the column and gamma masks stay run-time values (known, they let
  // the compiler move step-1 arithmetic into step 2 and spill), the row side is
  // compile-time for the whole operator.  They are read once into uniform
  // registers, not per test, where the compiler would narrow each test to an
  // unaligned vector load of the descriptor.  A block skips the degree-p modes
  // that are not columns (their nodal values, hence gradients, are zero) and
  // the step-1a sums of gammas no output row reads; their registers keep
  // values nothing uses.
  uint64_t cm[kRMaskW], rm[kRMaskW], gmk[kRMaskW];
#pragma unroll
  for (int k = 0; k < kRMaskW; ++k) {
    cm[k] = rr.colmask[k];
    rm[k] = rr.rowmask[k];
    gmk[k] = rr.gammask[k];
  }
  auto col = [&](int a) { return FULL || rbit(cm, a); };
  auto row = [&](int b) { return FULL || rbit(rm, b); };

  // 1. nodal values of the column modes (zeros elsewhere), in two halves so
  // that at most half of them are in flight per thread
  constexpr int NL = (P * 25 + kRThreads - 1) / kRThreads;
  constexpr int NLH = (NL + 1) / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double v[NLH];
#pragma unroll
    for (int u = 0; u < NLH; ++u) {
      const int idx = tid + kRThreads * (h * NLH + u);
      const int c = min(idx / 25, P - 1), nd = idx - (idx / 25) * 25;
      const int gx = x0 + nd % 5, gy = y0 + nd / 5;
      const bool ok = idx < P * 25 && col(c) && gx >= 1 && gx <= m && gy >= 1 && gy <= m;
      v[u] = ok ? U[(int64_t)c * Nh + (int64_t)(gy - 1) * m + (gx - 1)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NLH; ++u) {
      const int idx = tid + kRThreads * (h * NLH + u);
      if (idx < P * 25) sN[idx] = v[u];
    }
  }
  double gv[M];
#pragma unroll
  for (int nn = 0; nn < M; ++nn) gv[nn] = g[(int64_t)nn * Nq + (int64_t)tile * kTileQ + pt];

  // 2. monomials of degree below p - 1 (graded order: the first PL); degree
  // p - 1 (indices PL .. PN-1) and p (PN ..) formed from their parents, the
  // same products in the same order as the recurrence
  double mono[PL];
  mono[0] = 1.0;
#pragma unroll
  for (int d = 1; d < PL; ++d) mono[d] = mono[T.par[d]] * gv[T.var[d]] * T.inv[d];
  auto mono_of = [&](int d, const double* gg) {
    if (d < PL) return mono[d];
    if (d < PN) return mono[T.par[d]] * gg[T.var[d]] * T.inv[d];
    const int q = T.par[d];
    return mono[T.par[q]] * gg[T.var[q]] * T.inv[q] * gg[T.var[d]] * T.inv[d];
  };
  __syncthreads();
  const int el = lane >> 2, ql = qp;
  const double xi = r_gauss_pt(ql & 1), eta = r_gauss_pt(ql >> 1);
  const RGrad rg = r_grad_setup(comp, ql, el, xi, eta);
  double G[PN];
#pragma unroll
  for (int a = 0; a < PN; ++a) G[a] = (!SEL || S.col[a]) ? T.s[a] * r_grad(rg, sN + a * 25) : 0.0;
  double s2 = 0.0;
#pragma unroll
  for (int nn = 0; nn < M; ++nn) s2 = fma(gv[nn], gv[nn], s2);
  const double w = exp(mu + 0.5 * s2);

  // 3a. step 1 over the pairs with alpha of degree below p, in place (unscaled)
  if constexpr (SEL) {
    // the block's gammas in ascending order: each reads only G[alpha],
    // alpha >= gamma, not yet overwritten
#pragma unroll
    for (int i = 0; i < SN1; ++i) {
      double sx = 0.0;
#pragma unroll
      for (int t = S.p1[i]; t < S.p1[i + 1]; ++t) sx = fma(mono_of(S.d1[t], gv), G[S.a1[t]], sx);
      G[S.g1[i]] = sx;
    }
  } else {
#pragma unroll
    for (int gm = 0; gm < PN; ++gm) {
      if (!FULL && !rbit(gmk, gm)) continue;
      double sx = 0.0;
#pragma unroll
      for (int t = T.p1[gm]; t < T.p1[gm + 1]; ++t)
        if (T.a1[t] < PN) sx = fma(mono_of(T.d1[t], gv), G[T.a1[t]], sx);
      G[gm] = sx;
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  // 3b. the degree-p modes, one at a time
  if constexpr (SEL) {
#pragma unroll
    for (int i = 0; i < SNQ; ++i) {
      const double ga = T.s[S.qa[i]] * r_grad(rg, sN + S.qa[i] * 25);
#pragma unroll
      for (int k = S.pq[i]; k < S.pq[i + 1]; ++k)
        G[S.qg[k]] = fma(mono_of(S.qd[k], gv), ga, G[S.qg[k]]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < SN1; ++i) G[S.g1[i]] *= T.is2[S.g1[i]];
  } else {
#pragma unroll
    for (int a = PN; a < P; ++a) {
      if (!col(a)) continue;
      const double ga = T.s[a] * r_grad(rg, sN + a * 25);
#pragma unroll
      for (int k = Q.pq[a - PN]; k < Q.pq[a - PN + 1]; ++k)
        G[Q.qg[k]] = fma(mono_of(Q.qd[k], gv), ga, G[Q.qg[k]]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int gm = 0; gm < PN; ++gm) G[gm] *= T.is2[gm];
  }

  // 4. step 2 by chunks of rows; corner sums as in rapply_tile
  double wc, wo;
  r_corner_weights(comp, ql, xi, eta, wc, wo);
  int opq = 0;
  asm volatile("" : "+v"(opq));
  RGrad rg2 = rg;
  rg2.oc += opq;
  double gv2[M];
#pragma unroll
  for (int nn = 0; nn < M; ++nn) {
    gv2[nn] = gv[nn];
    asm volatile("" : "+v"(gv2[nn]));
  }
  double* sCc = sC + comp * kRChunk * kCS;
  const double* sCy = sC + kRChunk * kCS;
  const int lpos = cpos(lane);
  const RNode nq = r_node(tid % 25, x0, y0, m);
#pragma unroll
  for (int b0 = 0; b0 < P; b0 += kRChunk) {
    if (SEL && !S.chunk[b0 / kRChunk]) continue;
#pragma unroll
    for (int b = b0; b < (b0 + kRChunk < P ? b0 + kRChunk : P); ++b) {
      if (SEL ? !S.row[b] : !row(b)) continue;
      double sx = 0.0;
      if constexpr (SEL) {
#pragma unroll
        for (int t = S.p2[b]; t < S.p2[b + 1]; ++t) sx = fma(mono_of(S.d2[t], gv2), G[S.g2[t]], sx);
      } else {
#pragma unroll
        for (int t = T.p2[b]; t < T.p2[b + 1]; ++t)
          if (T.g2[t] < PN) sx = fma(mono_of(T.d2[t], gv2), G[T.g2[t]], sx);
      }
      double f;
      if constexpr (SEL) {
        // a compile-time block's rows are never its columns: no a_min term,
        // and a degree-p row's own Vbar (its gradient) is zero
        f = (T.s[b] * w) * sx;
      } else {
        // the unscaled gradient of the row's mode: the a_min term, and for a
        // degree-p row its own Vbar (gamma = beta, the list's last pair)
        const double db = r_grad(rg2, sN + b * 25);
        if (b >= PN) sx += (T.is2[b] * T.s[b]) * db;
        f = (T.s[b] * w) * sx;
        if (FULL || col(b)) f = fma(a_min, db, f);
      }
      const double t = wc * f + quad_xor<2>(wo * f);
      sCc[(b - b0) * kCS + lpos] = t - quad_xor<1>(t);
      if ((!FULL && !SEL) || b % kRFence == kRFence - 1) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (tid < 125)
#pragma unroll
      for (int k = 0; k < (kRChunk + 4) / 5; ++k) {
        const int bl = tid / 25 + 5 * k, b = b0 + bl;
        if (bl >= kRChunk || b >= P) break;
        if (!row(b)) continue;
        const int slot = FULL ? b : rr.slot[b];
        const double sum = r_node_sum(nq, sC + bl * kCS, sCy + bl * kCS);
        if (nq.owned) {
          if (nq.write) {
            double base = 0.0;
            if (beta != 0.0) base = beta * rin[(int64_t)(FULL ? slot : rr.mode[slot]) * Nh + nq.node];
            out[(int64_t)slot * Nh + nq.node] = base + sgn * sum;
          }
        } else {
          edge[((int64_t)slot * ntiles + tile) * kEdgeVals + nq.e] = sum;
        }
      }
    __syncthreads();  // the next chunk reuses the corner buffer
  }
}

template <int M, int p, bool FULL, int V = 0>
__global__ __launch_bounds__(kRThreads) void rapply_stream_kernel(
    int n, double mu, double a_min, const double* __restrict__ g, RApplyRows rr,
    const double* __restrict__ U, int64_t Nh, const double* __restrict__ rin, double beta,
    double sgn, double* __restrict__ out, double* __restrict__ edge) {
  extern __shared__ double smem[];
  const int nt = n / kTileE;
  rapply_stream_tile<M, p, FULL, V>(smem, xcd_tile(blockIdx.x, nt * nt), n, mu, a_min, g, rr, U, Nh,
                               rin, beta, sgn, out, edge);
}

template <int M, int p>
__global__ __launch_bounds__(kRThreads) void brapply_stream_kernel(
    const BInst* __restrict__ Is, const BState* __restrict__ Ss, const BItem* __restrict__ items,
    int nitems, int rowset, int src, int rin, int dst, double beta, double sgn, int gate) {
  extern __shared__ double smem[];
  const int it = blockIdx.x;  // one workgroup per item (grid = nitems)
  if (it >= nitems) return;
  const BItem w = items[it];
  const BInst& I = Is[w.inst];
  const BState& S = Ss[w.inst];
  if (gated(S, gate)) return;
  const RApplyRows& rr = rowset == 0 ? I.rfull : I.rpart[rowset];
  rapply_stream_tile<M, p, false>(smem, w.local, I.n, I.mu, I.amin, gptr(I.gq), rr,
                                bbuf(I, S, src), I.Nh, rin >= 0 ? bbuf(I, S, rin) : nullptr,
                                beta, sgn, bbuf(I, S, dst), gptr(I.edge));
}

// The compile-time block kernel of split kv (1 <= kv < M) of one (M, p).  Each
// (M, p) is instantiated in a translation unit of its own (sg_rapply_blocks_*)
// so that the block kernels compile beside the rest of the library.
template <int M, int p, int V = 1>
void launch_rblock(hipStream_t s, int kv, int n, double mu, double a_min, const double* g,
                   const RApplyRows& rr, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge) {
  if constexpr (V < M) {
    if (kv != V) {
      launch_rblock<M, p, V + 1>(s, kv, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);
      return;
    }
    const int nt = n / kTileE;
    constexpr int P = RTab<M, p>::P;
    if constexpr (P > kRSmall) {
      const size_t lds = 8 * ((size_t)25 * P + 2 * rchunk(P) * kCS);
      static const bool attr_ok =
          hipFuncSetAttribute((const void*)rapply_stream_kernel<M, p, false, V>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
      if (!attr_ok) throw Error(SG_ERR_HIP, "register apply: LDS size attribute");
      hipLaunchKernelGGL((rapply_stream_kernel<M, p, false, V>), dim3(nt * nt), dim3(kRThreads),
                         lds, s, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);
    } else {
      const size_t lds = 8 * (size_t)std::max(25 * P, 2 * rr.nrows * kCS);
      hipLaunchKernelGGL((rapply_kernel<M, p, false, V>), dim3(nt * nt), dim3(kRThreads), lds, s,
                         n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);
    }
  } else {
    throw Error(SG_ERR_INTERNAL, "register apply: block split");
  }
}

#define SG_RBLOCK_DECL(MM, PP)                                                                  \
  template void launch_rblock<MM, PP, 1>(hipStream_t, int, int, double, double, const double*,  \
                                         const RApplyRows&, const double*, int64_t,             \
                                         const double*, double, double, double*, double*);

#define SG_RAPPLY_STREAM_LIST(X) X(5, 3) X(4, 4) X(6, 3) X(5, 4) X(6, 4)
#define SG_RAPPLY_LIST(X) \
  X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(3, 1) X(3, 2) X(3, 3) \
  X(3, 4) X(4, 1) X(4, 2) X(4, 3) X(5, 1) X(5, 2) X(6, 1) X(6, 2)

#ifndef SG_RAPPLY_BLOCK_TU
#define SG_RBLOCK_EXTERN(MM, PP) extern SG_RBLOCK_DECL(MM, PP)
SG_RAPPLY_STREAM_LIST(SG_RBLOCK_EXTERN)
SG_RAPPLY_LIST(SG_RBLOCK_EXTERN)
#undef SG_RBLOCK_EXTERN

size_t rapply_stream_lds_bytes(int P) {
  return 8 * ((size_t)P * 25 + (size_t)2 * rchunk(P) * kCS);
}

// P <= kRSmall: the nodal values and, after them, the corner contributions of
// both components; above, the layout of rapply_stream_tile
size_t rapply_lds_bytes(int P, int nrows) {
  if (P > kRSmall) return rapply_stream_lds_bytes(P);
  return 8 * std::max((size_t)P * 25, (size_t)2 * nrows * kCS);
}


bool rapply_supported(int M, int p) {
#define SG_RAPPLY_SUP(MM, PP) if (M == MM && p == PP) return true;
  SG_RAPPLY_LIST(SG_RAPPLY_SUP)
  SG_RAPPLY_STREAM_LIST(SG_RAPPLY_SUP)
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
  SG_RAPPLY_STREAM_LIST(SG_RAPPLY_CHK)
#undef SG_RAPPLY_CHK
  return false;
}

void launch_rapply(hipStream_t s, int M, int p, int n, double mu, double a_min, const double* g,
                   const RApplyRows& rr, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge, bool fixup, int kv) {
  const int nt = n / kTileE, ntiles = nt * nt;
  const int P = (int)rc_binom(M + p, p);
  if (rr.nrows < 1 || rr.nrows > P) throw Error(SG_ERR_INTERNAL, "register apply: bad rows");
  if (P > kRMax) throw Error(SG_ERR_INTERNAL, "register apply: P");
  bool full = rr.nrows == P;
  for (int b = 0; full && b < P; ++b)
    full = rbit(rr.colmask, b) && rbit(rr.rowmask, b) && rbit(rr.gammask, b) && rr.slot[b] == b &&
           rr.mode[b] == b;
#define SG_RAPPLY_STREAM_LAUNCH(MM, PP)                                                          \
  if (M == MM && p == PP) {                                                                    \
    const size_t blds = rapply_stream_lds_bytes(P);                                               \
    static const bool attr_ok =                                                                \
        hipFuncSetAttribute((const void*)rapply_stream_kernel<MM, PP, true>,                     \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)blds) == hipSuccess && \
        hipFuncSetAttribute((const void*)rapply_stream_kernel<MM, PP, false>,                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)blds) == hipSuccess; \
    if (!attr_ok) throw Error(SG_ERR_HIP, "register apply: LDS size attribute");               \
    if (!full && kv > 0)                                                                       \
      launch_rblock<MM, PP>(s, kv, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);     \
    else if (full)                                                                             \
      hipLaunchKernelGGL((rapply_stream_kernel<MM, PP, true>), dim3(ntiles), dim3(kRThreads),   \
                         blds, s, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);      \
    else                                                                                       \
      hipLaunchKernelGGL((rapply_stream_kernel<MM, PP, false>), dim3(ntiles), dim3(kRThreads),  \
                         blds, s, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);      \
    if (fixup) launch_apply_fixup(s, n, rr.nrows, sgn, edge, out, Nh);                         \
    return;                                                                                    \
  }
  SG_RAPPLY_STREAM_LIST(SG_RAPPLY_STREAM_LAUNCH)
#undef SG_RAPPLY_STREAM_LAUNCH
  const size_t lds = rapply_lds_bytes(P, rr.nrows);
#define SG_RAPPLY_LAUNCH(MM, PP)                                                              \
  if (M == MM && p == PP) {                                                                   \
    if (full)                                                                                 \
      hipLaunchKernelGGL((rapply_kernel<MM, PP, true>), dim3(ntiles), dim3(kRThreads), lds, s, \
                         n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);              \
    else if (kv > 0)                                                                          \
      launch_rblock<MM, PP>(s, kv, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);    \
    else                                                                                      \
      hipLaunchKernelGGL((rapply_kernel<MM, PP, false>), dim3(ntiles), dim3(kRThreads), lds,  \
                         s, n, mu, a_min, g, rr, U, Nh, rin, beta, sgn, out, edge);           \
  } else
  SG_RAPPLY_LIST(SG_RAPPLY_LAUNCH) { throw Error(SG_ERR_INTERNAL, "register apply: (M, p)"); }
#undef SG_RAPPLY_LAUNCH
  if (fixup) launch_apply_fixup(s, n, rr.nrows, sgn, edge, out, Nh);
}

void launch_brapply(hipStream_t s, int M, int p, size_t lds, const BInst* I, const BState* st,
                    const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                    double beta, double sgn, int gate) {
  if (nitems <= 0) return;
  const int grid = nitems;  // one workgroup per item, as in a single-instance launch
#define SG_BRAPPLY_STREAM_LAUNCH(MM, PP)                                                         \
  if (M == MM && p == PP) {                                                                    \
    static const bool attr_ok =                                                                \
        hipFuncSetAttribute((const void*)brapply_stream_kernel<MM, PP>,                          \
                            hipFuncAttributeMaxDynamicSharedMemorySize,                         \
                            (int)rapply_stream_lds_bytes(rc_binom(MM + PP, PP))) == hipSuccess;   \
    if (!attr_ok) throw Error(SG_ERR_HIP, "batched register apply: LDS size attribute");      \
    hipLaunchKernelGGL((brapply_stream_kernel<MM, PP>), dim3(grid), dim3(kRThreads), lds, s, I,  \
                       st, items, nitems, rowset, src, rin, dst, beta, sgn, gate);             \
    return;                                                                                    \
  }
  SG_RAPPLY_STREAM_LIST(SG_BRAPPLY_STREAM_LAUNCH)
#undef SG_BRAPPLY_STREAM_LAUNCH
#define SG_BRAPPLY_LAUNCH(MM, PP)                                                             \
  if (M == MM && p == PP) {                                                                   \
    hipLaunchKernelGGL((brapply_kernel<MM, PP>), dim3(grid), dim3(kRThreads), lds, s, I, st, items, \
                       nitems, rowset, src, rin, dst, beta, sgn, gate);                       \
  } else
  SG_RAPPLY_LIST(SG_BRAPPLY_LAUNCH) { throw Error(SG_ERR_INTERNAL, "batched register apply: (M, p)"); }
#undef SG_BRAPPLY_LAUNCH
}

#endif  // SG_RAPPLY_BLOCK_TU

}  // namespace sg
