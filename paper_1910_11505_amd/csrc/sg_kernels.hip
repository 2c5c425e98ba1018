// HIP kernels (gfx950) of the stochastic-Galerkin solver.
//
//  * set-up: coefficient chaos modes a_k at the Gauss points, the mean
//    stiffness stencil and its Galerkin coarse stencils, the load vector;
//  * the matrix-free SG operator W = sum_k vec(A_k U G_k^T) (Sec. 2.2);
//  * geometric-multigrid pieces on the 9-point mean stiffness, batched over
//    stochastic modes (inner solver of the preconditioners of Sec. 3);
//  * FP64 Krylov helpers with fixed-order (deterministic) reductions.
//
// No floating-point atomics are used: every output element is written by one
// thread and every sum is taken in a fixed order, so results are bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "sg_internal.h"

namespace sg {

namespace {

// 2-point Gauss-Legendre abscissae on [0, 1]
__device__ __forceinline__ double gauss_pt(int i) {
  return i ? 0.78867513459481288225 : 0.21132486540518711775;
}

// reference gradient of the bilinear hat of local node a = (ax, ay) at (xi, eta)
__device__ __forceinline__ void ref_grad(int a, double xi, double eta, double& gx, double& gy) {
  const int ax = a & 1, ay = a >> 1;
  const double fy = ay ? eta : 1.0 - eta;
  const double fx = ax ? xi : 1.0 - xi;
  gx = (ax ? 1.0 : -1.0) * fy;
  gy = (ay ? 1.0 : -1.0) * fx;
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// a_k(x_q) = a_min [k=0] + exp(mu + sum_m g_m^2 / 2) prod_m g_m^{k_m} / sqrt(k_m!)
// (eq. dataProjection evaluated in closed form through the Hermite generating
// function).  One thread per Gauss point, a slice of modes per block row.
// ---------------------------------------------------------------------------
__global__ void coeff_kernel(int64_t Nq, int M, int na, int kper, const double* __restrict__ g,
                             const int* __restrict__ Jq, const double* __restrict__ isf,
                             double mu, double a_min, double* __restrict__ a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Nq) return;
  double gv[16];
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    gv[m] = (m < M) ? g[(int64_t)m * Nq + q] : 0.0;
    s += gv[m] * gv[m];
  }
  const double E = exp(mu + 0.5 * s);
  const int k0 = blockIdx.y * kper;
  const int k1 = min(na, k0 + kper);
  for (int k = k0; k < k1; ++k) {
    double prod = 1.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      if (m < M) {
        const int e = Jq[k * M + m];
        for (int t = 0; t < e; ++t) prod *= gv[m];
      }
    }
    double v = E * isf[k] * prod;
    if (k == 0) v += a_min;
    a[(int64_t)k * Nq + q] = v;
  }
}

void launch_coeff(hipStream_t s, int n, int M, int na, const double* g, const int* Jq,
                  const double* isf, double mu, double a_min, double* a) {
  const int64_t Nq = (int64_t)4 * n * n;
  const int kper = 32;
  dim3 grid(cdiv(Nq, 256), cdiv(na, kper));
  hipLaunchKernelGGL(coeff_kernel, grid, dim3(256), 0, s, Nq, M, na, kper, g, Jq, isf, mu,
                     a_min, a);
}

// ---------------------------------------------------------------------------
// Mean stiffness stencil (eq. A_q with coefficient a_0): for every interior
// node, the 9 couplings summed over its 4 elements; couplings to Dirichlet
// nodes are dropped.  Stencil entry s = 3(dy+1) + (dx+1), SoA layout.
// ---------------------------------------------------------------------------
__global__ void fine_stencil_kernel(int n, const double* __restrict__ a0, double* __restrict__ S) {
  const int m = n - 1;
  const int64_t N = (int64_t)m * m;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int ix = (int)(node % m) + 1, iy = (int)(node / m) + 1;
  double st[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) st[t] = 0.0;
  for (int de = 0; de < 4; ++de) {
    const int ex = ix - 1 + (de & 1), ey = iy - 1 + (de >> 1);
    // local index of this node inside element (ex, ey)
    const int la = (ix - ex) + 2 * (iy - ey);
    double ke[4] = {0.0, 0.0, 0.0, 0.0};
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi = gauss_pt(qx), eta = gauss_pt(qy);
        const double c = 0.25 * a0[tiled_q(n, ex, ey, qx, qy)];
        double gax, gay;
        ref_grad(la, xi, eta, gax, gay);
        for (int b = 0; b < 4; ++b) {
          double gbx, gby;
          ref_grad(b, xi, eta, gbx, gby);
          ke[b] += c * (gax * gbx + gay * gby);
        }
      }
    for (int b = 0; b < 4; ++b) {
      const int jx = ex + (b & 1), jy = ey + (b >> 1);
      st[3 * (jy - iy + 1) + (jx - ix + 1)] += ke[b];
    }
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int jx = ix + (t % 3) - 1, jy = iy + (t / 3) - 1;
    const bool inside = jx >= 1 && jx <= m && jy >= 1 && jy <= m;
    S[(int64_t)t * N + node] = inside ? st[t] : 0.0;
  }
}

void launch_fine_stencil(hipStream_t s, int n, const double* a0, double* S) {
  const int64_t N = (int64_t)(n - 1) * (n - 1);
  hipLaunchKernelGGL(fine_stencil_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, n, a0, S);
}

// 1D interpolation weight of coarse node I at fine node i (fine interior
// numbering 1..nf-1, coarse 1..nc-1): 1 at i = 2I, 1/2 at i = 2I +- 1
__device__ __forceinline__ double pw(int i, int I) {
  const int d = i - 2 * I;
  return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0);
}

// Galerkin coarse stencil A_c = P^T A_f P for bilinear interpolation P.
__global__ void rap_kernel(int nf, const double* __restrict__ Sf, double* __restrict__ Sc) {
  const int mf = nf - 1, nc = nf / 2, mc = nc - 1;
  const int64_t Nf = (int64_t)mf * mf, Nc = (int64_t)mc * mc;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= Nc) return;
  const int I = (int)(node % mc) + 1, J = (int)(node / mc) + 1;
  double st[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) st[t] = 0.0;
  for (int fy = 2 * J - 1; fy <= 2 * J + 1; ++fy)
    for (int fx = 2 * I - 1; fx <= 2 * I + 1; ++fx) {
      const double wf = pw(fx, I) * pw(fy, J);
      const int64_t f = (int64_t)(fy - 1) * mf + (fx - 1);
      for (int t = 0; t < 9; ++t) {
        const int gx = fx + (t % 3) - 1, gy = fy + (t / 3) - 1;
        if (gx < 1 || gx > mf || gy < 1 || gy > mf) continue;
        const double afg = Sf[(int64_t)t * Nf + f];
        if (afg == 0.0) continue;
        // coarse nodes that interpolate to fine node g
        for (int cy = J - 1; cy <= J + 1; ++cy)
          for (int cx = I - 1; cx <= I + 1; ++cx) {
            if (cx < 1 || cx > mc || cy < 1 || cy > mc) continue;
            const double w = pw(gx, cx) * pw(gy, cy);
            if (w != 0.0) st[3 * (cy - J + 1) + (cx - I + 1)] += wf * afg * w;
          }
      }
    }
#pragma unroll
  for (int t = 0; t < 9; ++t) Sc[(int64_t)t * Nc + node] = st[t];
}

void launch_rap(hipStream_t s, int nf, const double* Sf, double* Sc) {
  const int64_t Nc = (int64_t)(nf / 2 - 1) * (nf / 2 - 1);
  hipLaunchKernelGGL(rap_kernel, dim3(cdiv(Nc, 128)), dim3(128), 0, s, nf, Sf, Sc);
}

// F = e_0 (x) M_h f_h: consistent Q1 mass on the nodal forcing, mode 0 only.
__global__ void rhs_kernel(int n, const double* __restrict__ f, double* __restrict__ F,
                           int64_t total) {
  const int m = n - 1;
  const int64_t N = (int64_t)m * m;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  if (idx >= N) {
    F[idx] = 0.0;
    return;
  }
  const int ix = (int)(idx % m) + 1, iy = (int)(idx / m) + 1;
  const double h = 1.0 / n;
  double acc = 0.0;
  for (int de = 0; de < 4; ++de) {
    const int ex = ix - 1 + (de & 1), ey = iy - 1 + (de >> 1);
    const int la = (ix - ex) + 2 * (iy - ey);
    for (int b = 0; b < 4; ++b) {
      const int jx = ex + (b & 1), jy = ey + (b >> 1);
      const int same = (la == b), opposite = ((la ^ b) == 3);
      const double w = same ? 4.0 : (opposite ? 1.0 : 2.0);
      acc += w * f[(int64_t)jy * (n + 1) + jx];
    }
  }
  F[idx] = acc * (h * h / 36.0);
}

void launch_rhs(hipStream_t s, int n, const double* f, double* F, int64_t total) {
  hipLaunchKernelGGL(rhs_kernel, dim3(cdiv(total, 256)), dim3(256), 0, s, n, f, F, total);
}

// ---------------------------------------------------------------------------
// SG operator apply.  One tile = 4x4 elements (64 Gauss points, one per lane),
// four wavefronts splitting the output rows.  For each pass over a slice of
// the input columns (all columns in one pass unless their gradients exceed
// LDS):
//   1. stage the tile's 5x5 nodal values of the pass's input modes in LDS;
//   2. reference gradients of those modes at the 64 points -> LDS;
//   3. stream the coefficient modes a_k in chunks of kc modes through LDS
//      (each value read from HBM once per pass, coalesced 512-byte rows,
//      prefetched into registers one chunk ahead) together with the chunk's
//      (k, j, value) records, and per output row accumulate
//      flux_i(q) += a_k(q) [G_k]_{ij} grad U_j(q);
// then per row: element-node contributions (1/4) grad phi_a . flux, summed over
// the element's four lanes, then node sums in fixed order; nodes owned by the
// tile are written, the right/top edge and corner go to a small edge buffer
// folded in by the fixup step.
// out[slot] = beta * rin[row] + sgn * (K_sub U)[row].
// ---------------------------------------------------------------------------
template <int RMAX>
__device__ __forceinline__ void apply_tile(double* smem, int tile, int n, int na,
                                           const double* __restrict__ a, const RowSetDev& rs,
                                           const double* __restrict__ U, int64_t Nh,
                                           const double* __restrict__ rin, double beta,
                                           double sgn, double* __restrict__ out,
                                           double* __restrict__ edge) {
  const int nt = n / kTileE;
  const int ntiles = nt * nt;
  const int tx = tile % nt, ty = tile / nt;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t Nq = (int64_t)4 * n * n;
  const int m = n - 1;
  const int kc = rs.kc, nchunk = rs.nchunk, nrows = rs.nrows;
  double2* sG = reinterpret_cast<double2*>(smem);
  double* sA = smem + 2 * rs.maxcols * kTileQ;
  const int sa_len = (max(max(kc * kTileQ, rs.maxcols * 25), kApplyWaves * kTileQ) + 1) & ~1;
  Entry* sEnt = reinterpret_cast<Entry*>(sA + sa_len);
  const int x0 = tx * kTileE, y0 = ty * kTileE;

  double ax[RMAX], ay[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) ax[r] = ay[r] = 0.0;
  // RMAX is the compiled bound; the row set's own per-wave stride is rs.rmax <= RMAX
  const int* wrows = rs.wrows + wave * rs.rmax;
  constexpr int kPre = kMaxChunk * kTileQ / 256;
  double pre[kPre];
  auto prefetch = [&](int ch) {
    const int k0 = ch * kc;
    const int cnt = min(kc, na - k0) * kTileQ;
    const double* src = a + (int64_t)k0 * Nq + (int64_t)tile * kTileQ;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int idx = tid + u * 256;
      pre[u] = (idx < cnt) ? src[(int64_t)(idx >> 6) * Nq + (idx & 63)] : 0.0;
    }
  };

  for (int pass = 0; pass < rs.npass; ++pass) {
    const int c0 = rs.cpass[pass];
    const int ncols = rs.cpass[pass + 1] - c0;
    prefetch(0);
    // 1. nodal values of the pass's modes on the tile's 5x5 nodes (batched loads)
    for (int base = tid; base < ncols * 25; base += 256 * 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = base + u * 256;
        v[u] = 0.0;
        if (idx < ncols * 25) {
          const int c = idx / 25, nd = idx - c * 25;
          const int gx = x0 + nd % 5, gy = y0 + nd / 5;
          if (gx >= 1 && gx <= m && gy >= 1 && gy <= m)
            v[u] = U[(int64_t)rs.cols[c0 + c] * Nh + (int64_t)(gy - 1) * m + (gx - 1)];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (base + u * 256 < ncols * 25) sA[base + u * 256] = v[u];
    }
    __syncthreads();
    // 2. reference gradients at the Gauss points
    for (int idx = tid; idx < ncols * kTileQ; idx += 256) {
      const int c = idx >> 6, lq = idx & 63;
      const int el = lq >> 2, ql = lq & 3;
      const int elx = el & 3, ely = el >> 2;
      const double xi = gauss_pt(ql & 1), eta = gauss_pt(ql >> 1);
      const double* u = sA + c * 25;
      const double u00 = u[ely * 5 + elx], u10 = u[ely * 5 + elx + 1];
      const double u01 = u[(ely + 1) * 5 + elx], u11 = u[(ely + 1) * 5 + elx + 1];
      sG[idx] = make_double2((1.0 - eta) * (u10 - u00) + eta * (u11 - u01),
                             (1.0 - xi) * (u01 - u00) + xi * (u11 - u10));
    }
    __syncthreads();
    // 3. flux accumulation over the coefficient chunks
    const int* pptr = rs.ptr + (int64_t)pass * nchunk * (nrows + 1);
    for (int ch = 0; ch < nchunk; ++ch) {
      const int cnt = min(kc, na - ch * kc) * kTileQ;
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        if (tid + u * 256 < cnt) sA[tid + u * 256] = pre[u];
      const int cb = pptr[ch * (nrows + 1)];
      const int ce = pptr[ch * (nrows + 1) + nrows];
      const int4* esrc = reinterpret_cast<const int4*>(rs.ent + cb);
      int4* edst = reinterpret_cast<int4*>(sEnt);
      for (int base = tid; base < ce - cb; base += 256 * 4) {
        int4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (base + u * 256 < ce - cb) v[u] = esrc[base + u * 256];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (base + u * 256 < ce - cb) edst[base + u * 256] = v[u];
      }
      __syncthreads();
      if (ch + 1 < nchunk) prefetch(ch + 1);
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int slot = (r < rs.rmax) ? wrows[r] : -1;
        if (slot >= 0) {
          const int b = pptr[ch * (nrows + 1) + slot] - cb;
          const int e = pptr[ch * (nrows + 1) + slot + 1] - cb;
          double sx = ax[r], sy = ay[r];
          for (int t = b; t < e; t += kEntryUnroll) {
            Entry en[kEntryUnroll];
#pragma unroll
            for (int u = 0; u < kEntryUnroll; ++u) en[u] = sEnt[t + u];
            double av[kEntryUnroll];
            double2 gg[kEntryUnroll];
#pragma unroll
            for (int u = 0; u < kEntryUnroll; ++u) {
              av[u] = sA[(en[u].kj & 0xffff) * kTileQ + lane];
              gg[u] = sG[(en[u].kj >> 16) * kTileQ + lane];
            }
#pragma unroll
            for (int u = 0; u < kEntryUnroll; ++u) {
              const double c = av[u] * en[u].v;
              sx = fma(c, gg[u].x, sx);
              sy = fma(c, gg[u].y, sy);
            }
          }
          ax[r] = sx;
          ay[r] = sy;
        }
      }
      __syncthreads();
    }
  }

  // 4. node contributions, row by row
  const int ql = lane & 3;
  const double xi = gauss_pt(ql & 1), eta = gauss_pt(ql >> 1);
  double gpx[4], gpy[4];
#pragma unroll
  for (int a4 = 0; a4 < 4; ++a4) ref_grad(a4, xi, eta, gpx[a4], gpy[a4]);
  double* sE = sA + wave * kTileQ;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int slot = (r < rs.rmax) ? wrows[r] : -1;
    if (slot >= 0) {
      double c[4];
#pragma unroll
      for (int a4 = 0; a4 < 4; ++a4) c[a4] = 0.25 * (gpx[a4] * ax[r] + gpy[a4] * ay[r]);
#pragma unroll
      for (int a4 = 0; a4 < 4; ++a4) {
        c[a4] += __shfl_xor(c[a4], 1);
        c[a4] += __shfl_xor(c[a4], 2);
      }
      const double mine = (ql == 0) ? c[0] : (ql == 1) ? c[1] : (ql == 2) ? c[2] : c[3];
      sE[lane] = mine;
    }
    __syncthreads();
    if (slot >= 0 && lane < 25) {
      const int nx = lane % 5, ny = lane / 5;
      double sum = 0.0;
      // fixed order: NE of (nx-1,ny-1), NW of (nx,ny-1), SE of (nx-1,ny), SW of (nx,ny)
      if (nx >= 1 && ny >= 1) sum += sE[((ny - 1) * 4 + (nx - 1)) * 4 + 3];
      if (nx <= 3 && ny >= 1) sum += sE[((ny - 1) * 4 + nx) * 4 + 2];
      if (nx >= 1 && ny <= 3) sum += sE[(ny * 4 + (nx - 1)) * 4 + 1];
      if (nx <= 3 && ny <= 3) sum += sE[(ny * 4 + nx) * 4 + 0];
      if (nx <= 3 && ny <= 3) {
        const int gx = x0 + nx, gy = y0 + ny;
        if (gx >= 1 && gy >= 1) {
          const int64_t node = (int64_t)(gy - 1) * m + (gx - 1);
          double base = 0.0;
          if (beta != 0.0) base = beta * rin[(int64_t)rs.rows[slot] * Nh + node];
          out[(int64_t)slot * Nh + node] = base + sgn * sum;
        }
      } else {
        const int idx = (nx == 4 && ny == 4) ? 8 : (nx == 4 ? ny : 4 + nx);
        edge[((int64_t)slot * ntiles + tile) * kEdgeVals + idx] = sum;
      }
    }
    __syncthreads();
  }
}

template <int RMAX>
__global__ __launch_bounds__(256) void apply_kernel(int n, int na, const double* __restrict__ a,
                                                    RowSetDev rs, const double* __restrict__ U,
                                                    int64_t Nh, const double* __restrict__ rin,
                                                    double beta, double sgn,
                                                    double* __restrict__ out,
                                                    double* __restrict__ edge) {
  extern __shared__ double smem[];
  apply_tile<RMAX>(smem, blockIdx.x, n, na, a, rs, U, Nh, rin, beta, sgn, out, edge);
}

// Folds the edge contributions of the left, bottom and diagonal neighbour
// tiles into the nodes on a tile's left column and bottom row (item gid of
// nrows * ntiles * 7).
__device__ __forceinline__ void apply_fixup_item(int64_t gid, int n, double sgn,
                                                 const double* __restrict__ edge,
                                                 double* __restrict__ out, int64_t Nh) {
  // item counts stay below 2^31 (checked at launch): 32-bit unsigned division
  const int nt = n / kTileE, ntiles = nt * nt, m = n - 1;
  const unsigned g = (unsigned)gid;
  const int j = (int)(g % 7u);
  const unsigned rt = g / 7u;
  const int tile = (int)(rt % (unsigned)ntiles);
  const int slot = (int)(rt / (unsigned)ntiles);
  const int tx = tile % nt, ty = tile / nt;
  const int nx = j < 4 ? 0 : j - 3;  // (0,0..3) then (1..3,0)
  const int ny = j < 4 ? j : 0;
  const int gx = tx * kTileE + nx, gy = ty * kTileE + ny;
  if (gx < 1 || gy < 1) return;
  const int64_t node = (int64_t)(gy - 1) * m + (gx - 1);
  const double* eb = edge + (int64_t)slot * ntiles * kEdgeVals;
  double v = out[(int64_t)slot * Nh + node];
  if (nx == 0) v += sgn * eb[(int64_t)(tile - 1) * kEdgeVals + ny];
  if (ny == 0) v += sgn * eb[(int64_t)(tile - nt) * kEdgeVals + 4 + nx];
  if (nx == 0 && ny == 0) v += sgn * eb[(int64_t)(tile - nt - 1) * kEdgeVals + 8];
  out[(int64_t)slot * Nh + node] = v;
}

__global__ void apply_fixup_kernel(int n, int nrows, double sgn, const double* __restrict__ edge,
                                   double* __restrict__ out, int64_t Nh) {
  const int nt = n / kTileE;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nrows * nt * nt * 7) return;
  apply_fixup_item(gid, n, sgn, edge, out, Nh);
}

void launch_apply_fixup(hipStream_t s, int n, int nrows, double sgn, const double* edge,
                        double* out, int64_t Nh) {
  const int nt = n / kTileE;
  const int64_t total = (int64_t)nrows * nt * nt * 7;
  if (total >= (int64_t)1 << 31) throw Error(SG_ERR_UNSUPPORTED, "apply fixup: too many edge values");
  hipLaunchKernelGGL(apply_fixup_kernel, dim3(cdiv(total, 256)), dim3(256), 0, s, n, nrows, sgn,
                     edge, out, Nh);
}

size_t apply_lds_bytes(int maxcols, int kc, int maxent) {
  size_t sa = std::max<size_t>({(size_t)kc * kTileQ, (size_t)maxcols * 25, (size_t)kApplyWaves * kTileQ});
  sa = (sa + 1) & ~size_t(1);  // keeps the entry records 16-byte aligned
  return 8 * (2 * (size_t)maxcols * kTileQ + sa) + sizeof(Entry) * (size_t)maxent;
}

void launch_apply(hipStream_t s, int n, int na, const double* a, const RowSetDev& rs,
                  const double* U, int64_t Nh, const double* rin, double beta, double sgn,
                  double* out, double* edge, bool fixup) {
  const int nt = n / kTileE;
  const int ntiles = nt * nt;
  const size_t lds = apply_lds_bytes(rs.maxcols, rs.kc, rs.maxent);
  dim3 grid(ntiles), block(256);
#define SG_APPLY_CASE(R)                                                                     \
  case R:                                                                                    \
    hipLaunchKernelGGL(apply_kernel<R>, grid, block, lds, s, n, na, a, rs, U, Nh, rin, beta, \
                       sgn, out, edge);                                                      \
    break;
  switch (rs.rmax) {
    SG_APPLY_CASE(1)
    SG_APPLY_CASE(2)
    SG_APPLY_CASE(4)
    SG_APPLY_CASE(8)
    SG_APPLY_CASE(16)
    SG_APPLY_CASE(32)
    SG_APPLY_CASE(64)
    default:
      throw Error(SG_ERR_INTERNAL, "apply: unsupported rows per wavefront");
  }
#undef SG_APPLY_CASE
  if (fixup) launch_apply_fixup(s, n, rs.nrows, sgn, edge, out, Nh);
}

// ---------------------------------------------------------------------------
// Factored SG operator apply, exact when the coefficient degree q >= 2p.
//
// With y ~ N(0, I), shifting the Gaussian measure by g(x) and the Hermite
// addition formula give, for the orthonormal chaos,
//   sum_k a_k(x) [G_k]_{beta,alpha} = E[a psi_beta psi_alpha]
//     = a_min delta_{beta,alpha} + w(x) sum_gamma T_{beta,gamma} T_{alpha,gamma},
//   w = exp(mu + |g|^2 / 2),  T_{alpha,gamma} = prod_n sqrt(alpha_n!/gamma_n!)
//                                             g_n^(alpha_n-gamma_n) / (alpha_n-gamma_n)!
// for gamma <= alpha componentwise (zero otherwise).  The chaos projection of
// eq. dataProjection is exact up to degree 2p, so this is the same matrix K.
// Only g_n(x_q) (M values per Gauss point) is read instead of n_a coefficient
// modes, and the per-point contraction costs 2 nnz(T) products instead of
// nnz(G).  The factorials are folded into scaled gradients and monomials (see
// FRowSetDev), so a record is one 32-bit (slot, monomial) word.
//
// One workgroup per 4x4-element tile; its 64 Gauss points are taken in
// sub-batches of QB points (64: the whole tile, 32: 4x2 elements, 16: 2x2,
// 8: 2x1).  Thread t handles point t % QB of the sub-batch for the rows of
// row group t / QB.  Per sub-batch:
//   1. nodal values of the column modes and g_n at the points -> LDS (loaded
//      into registers during the previous sub-batch);
//   2. scaled gradients G^_alpha, w(x_q), scaled monomials m_delta;
//   3. step 1: Vbar_gamma -> LDS;
//   4. step 2: flux_beta, then the element-node contributions (1/4) grad phi_a .
//      flux_beta, summed over the element's four points by lane shuffles.
// With QB = 64 a row group is one wavefront holding the whole tile: its
// records are wave-uniform (scalar loads), and the 25 node sums of a row are
// gathered across lanes and written at once (owned nodes to out, the right/
// top edge and corner to the edge buffer for the fixup).  With smaller
// sub-batches the node sums accumulate in LDS over the sub-batches in a fixed
// order (sub-batch, then local corner of the element) and are written at the
// end of the tile.
// ---------------------------------------------------------------------------
namespace {
template <int QB>
struct FaGeom {
  static constexpr int SW = QB <= 16 ? 2 : 4;  // elements per sub-batch row
  static constexpr int SH = QB / (4 * SW);     // element rows per sub-batch
  static constexpr int NND = (SW + 1) * (SH + 1);
  static constexpr int NSUB = kTileQ / QB;
  static constexpr int SUBS_X = kTileE / SW;
  static constexpr int LOG = QB == 8 ? 3 : QB == 16 ? 4 : QB == 32 ? 5 : 6;
};
__host__ __device__ inline int fa_nodes(int qb) {
  const int sw = qb <= 16 ? 2 : 4, sh = qb / (4 * sw);
  return (sw + 1) * (sh + 1);
}
__host__ __device__ inline int fa_even(int x) { return (x + 1) & ~1; }
constexpr int kFPre = 10;  // prefetch registers per thread (nodal values + g of a sub-batch)

// LDS layout, in doubles: tables | node sums (QB < 64) | G^ [ncols][QB] |
// Vbar [ngam][QB] (nodal values alias it) | m [P + 1][QB] | w [QB] | g [M][QB]
struct FaLds {
  int node, grad, vgam, mono, w, g, total;
};
__host__ __device__ inline FaLds fa_layout(int qb, int nrows, int ncols, int ngam, int nmono,
                                           int M, int nblob) {
  FaLds L;
  L.node = fa_even(nblob) / 2;
  L.grad = L.node + (qb == 64 ? 0 : fa_even(nrows * 25));
  L.vgam = L.grad + (ncols > 1 ? ncols : 1) * qb * 2;
  const int vsz = (ngam > 1 ? ngam : 1) * qb * 2, nsz = fa_even(ncols * fa_nodes(qb));
  L.mono = L.vgam + (vsz > nsz ? vsz : nsz);
  L.w = L.mono + fa_even((nmono + 1) * qb);
  L.g = L.w + qb;
  L.total = L.g + fa_even(M * qb);
  return L;
}
}  // namespace

size_t fapply_lds_bytes(int qb, int nrows, int ncols, int ngam, int nmono, int M, int nblob) {
  return 8 * (size_t)fa_layout(qb, nrows, ncols, ngam, nmono, M, nblob).total;
}

template <int QB>
__device__ __forceinline__ void fapply_tile(double* smem, int tile, int n, double mu,
                                            double a_min, const double* __restrict__ g,
                                            const FRowSetDev& rs, const int* __restrict__ blob,
                                            const double* __restrict__ U, int64_t Nh,
                                            const double* __restrict__ rin, double beta,
                                            double sgn, double* __restrict__ out,
                                            double* __restrict__ edge) {
  using Geo = FaGeom<QB>;
  constexpr int SW = Geo::SW, SH = Geo::SH, NND = Geo::NND, LOG = Geo::LOG;
  const int nt = n / kTileE;
  const int ntiles = nt * nt;
  const int tx = tile % nt, ty = tile / nt;
  const int x0 = tx * kTileE, y0 = ty * kTileE;
  const int tid = threadIdx.x;
  const int q = tid & (QB - 1);
  const int grp = QB == 64 ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> LOG;
  const int64_t Nq = (int64_t)4 * n * n;
  const int m = n - 1;
  const int M = rs.M, ncols = rs.ncols, nrows = rs.nrows, rmax = rs.rmax, P = rs.nmono;

  const FaLds L = fa_layout(QB, nrows, ncols, rs.ngam, P, M, rs.nblob);
  int* sB = reinterpret_cast<int*>(smem);
  double* sNode = smem + L.node;                               // [nrows][25], QB < 64
  double2* sG = reinterpret_cast<double2*>(smem + L.grad);     // [ncols][QB]
  double2* sV = reinterpret_cast<double2*>(smem + L.vgam);     // [ngam][QB]
  double* sN = smem + L.vgam;                                  // nodal values [ncols][NND]
  double* sM = smem + L.mono;                                  // [P + 1][QB]
  double* sW = smem + L.w;                                     // [QB]
  double* sg = smem + L.g;                                     // [M][QB]

  const int* tcols = sB + rs.o_cols;
  const int* tmpar = sB + rs.o_mpar;
  const int* tmvar = sB + rs.o_mvar;
  const int* tmdeg = sB + rs.o_mdeg;
  const double* tcs = reinterpret_cast<const double*>(sB + rs.o_cs);
  const double* tgs = reinterpret_cast<const double*>(sB + rs.o_gs);
  const double* trs = reinterpret_cast<const double*>(sB + rs.o_rs);
  const double* tra = reinterpret_cast<const double*>(sB + rs.o_ra);
  const double* tminv = reinterpret_cast<const double*>(sB + rs.o_minv);
  // row lists and records: wave-uniform global reads for QB = 64, LDS otherwise
  const int2* rr1 = reinterpret_cast<const int2*>((QB == 64 ? blob : sB) + rs.o_r1) + grp * rmax;
  const int2* rr2 = reinterpret_cast<const int2*>((QB == 64 ? blob : sB) + rs.o_r2) + grp * rmax;
  const int* rdcol = (QB == 64 ? blob : sB) + rs.o_dcol;
  const int4* re1 = reinterpret_cast<const int4*>((QB == 64 ? blob : sB) + rs.o_e1);
  const int4* re2 = reinterpret_cast<const int4*>((QB == 64 ? blob : sB) + rs.o_e2);

  // nodal values of the column modes, then g_n at the points, of sub-batch sb
  const int nnod = ncols * NND, nitems = nnod + M * QB;
  auto fetch = [&](const int* __restrict__ cols, int sb, int base, double* v) {
    const int ex0 = (sb % Geo::SUBS_X) * SW, ey0 = (sb / Geo::SUBS_X) * SH;
#pragma unroll
    for (int u = 0; u < kFPre; ++u) {
      const int idx = base + tid + u * 256;
      double x = 0.0;
      if (idx < nnod) {
        const int c = idx / NND, nd = idx - c * NND;
        const int gx = x0 + ex0 + nd % (SW + 1), gy = y0 + ey0 + nd / (SW + 1);
        if (gx >= 1 && gx <= m && gy >= 1 && gy <= m)
          x = U[(int64_t)cols[c] * Nh + (int64_t)(gy - 1) * m + (gx - 1)];
      } else if (idx < nitems) {
        const int j = idx - nnod, nn = j >> LOG, qq = j & (QB - 1);
        const int el = qq >> 2;
        const int elx = ex0 + el % SW, ely = ey0 + el / SW;
        x = g[(int64_t)nn * Nq + (int64_t)tile * kTileQ + (ely * kTileE + elx) * 4 + (qq & 3)];
      }
      v[u] = x;
    }
  };
  auto store = [&](int base, const double* v) {
#pragma unroll
    for (int u = 0; u < kFPre; ++u) {
      const int idx = base + tid + u * 256;
      if (idx < nnod) sN[idx] = v[u];
      else if (idx < nitems) sg[idx - nnod] = v[u];
    }
  };
  const bool prefetch = nitems <= kFPre * 256;
  double pre[kFPre];
  // the first sub-batch's loads overlap the table staging (column ids from global)
  if (prefetch) fetch(blob + rs.o_cols, 0, 0, pre);
  // tables -> LDS with 16-byte loads, eight in flight per thread (nblob % 4 == 0)
  {
    const int n4 = rs.nblob >> 2;
    const int4* src = reinterpret_cast<const int4*>(blob);
    int4* dst = reinterpret_cast<int4*>(sB);
    for (int base = tid; base < n4; base += 256 * 8) {
      int4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[min(base + u * 256, n4 - 1)];  // clamped, no branch
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (base + u * 256 < n4) dst[base + u * 256] = v[u];
    }
  }
  if (QB < 64)
    for (int i = tid; i < nrows * 25; i += 256) sNode[i] = 0.0;
  for (int i = tid; i < QB; i += 256) sM[P * QB + i] = 0.0;
  __syncthreads();

  const int ql = q & 3;
  const double xi = gauss_pt(ql & 1), eta = gauss_pt(ql >> 1);
  double gpx[4], gpy[4];
#pragma unroll
  for (int a4 = 0; a4 < 4; ++a4) ref_grad(a4, xi, eta, gpx[a4], gpy[a4]);
  // QB = 64: lane l < 25 gathers node (l % 5, l / 5) from the lanes holding the
  // corner contributions of its (up to) four elements
  const int gnx = tid % 5, gny = (tid & 63) / 5;
  int src[4];
  bool has[4];
#pragma unroll
  for (int a4 = 0; a4 < 4; ++a4) {
    const int ex = gnx - (a4 & 1), ey = gny - (a4 >> 1);
    has[a4] = (tid & 63) < 25 && ex >= 0 && ex < 4 && ey >= 0 && ey < 4;
    src[a4] = has[a4] ? ((ey * 4 + ex) * 4 + a4) * 4 : 0;  // byte index for ds_bpermute
  }

  for (int sb = 0; sb < Geo::NSUB; ++sb) {
    const int ex0 = (sb % Geo::SUBS_X) * SW, ey0 = (sb / Geo::SUBS_X) * SH;
    if (sb > 0) __syncthreads();  // the previous sub-batch is done with sV, sM and sg
    if (prefetch) {
      store(0, pre);
    } else {
      for (int base = 0; base < nitems; base += kFPre * 256) {
        double v[kFPre];
        fetch(tcols, sb, base, v);
        store(base, v);
      }
    }
    __syncthreads();
    if (prefetch && sb + 1 < Geo::NSUB) fetch(tcols, sb + 1, 0, pre);  // in flight meanwhile
    // scaled gradients, w, monomials of degree 0 and 1
    for (int idx = tid; idx < ncols * QB; idx += 256) {
      const int c = idx >> LOG, qq = idx & (QB - 1);
      const int el = qq >> 2, qp = qq & 3;
      const int lx = el % SW, ly = el / SW;
      const double xq = gauss_pt(qp & 1), yq = gauss_pt(qp >> 1);
      const double* u = sN + c * NND;
      const double u00 = u[ly * (SW + 1) + lx], u10 = u[ly * (SW + 1) + lx + 1];
      const double u01 = u[(ly + 1) * (SW + 1) + lx], u11 = u[(ly + 1) * (SW + 1) + lx + 1];
      const double s = tcs[c];
      sG[idx] = make_double2(s * ((1.0 - yq) * (u10 - u00) + yq * (u11 - u01)),
                             s * ((1.0 - xq) * (u01 - u00) + xq * (u11 - u10)));
    }
    if (tid < QB) {
      double s2 = 0.0;
      for (int nn = 0; nn < M; ++nn) s2 = fma(sg[nn * QB + tid], sg[nn * QB + tid], s2);
      sW[tid] = exp(mu + 0.5 * s2);
    }
    for (int idx = tid; idx < tmdeg[2] * QB; idx += 256) {
      const int d = idx >> LOG, qq = idx & (QB - 1);
      sM[idx] = d == 0 ? 1.0 : sg[tmvar[d] * QB + qq];
    }
    for (int deg = 2; deg <= rs.pdeg; ++deg) {
      __syncthreads();
      const int d0 = tmdeg[deg], cnt = (tmdeg[deg + 1] - d0) * QB;
      for (int idx = tid; idx < cnt; idx += 256) {
        const int d = d0 + (idx >> LOG), qq = idx & (QB - 1);
        sM[d * QB + qq] = sM[tmpar[d] * QB + qq] * sg[tmvar[d] * QB + qq] * tminv[d];
      }
    }
    __syncthreads();
    const double* mq = sM + q;
    const double2* gq = sG + q;
    double2* vq = sV + q;
    // sum over records [4 b, 4 e) of m_(record) * X_(record slot) at this point;
    // up to four record groups are loaded before the first is used
    // (four independent accumulator pairs, one per record position of a group,
    // summed in a fixed order at the end: FP64 FMA chains are latency-bound)
    auto contract = [&](const int4* __restrict__ rec, const double2* __restrict__ xq, int b,
                        int e, double& sx, double& sy) {
      double ax[4] = {0.0, 0.0, 0.0, 0.0}, ay[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = b; t < e; t += 4) {
        int4 E[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) E[u] = rec[min(t + u, e - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (t + u < e) {
            const int ks[4] = {E[u].x, E[u].y, E[u].z, E[u].w};
            double mv[4];
            double2 xv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              mv[k] = mq[(ks[k] >> 16) << LOG];
              xv[k] = xq[(ks[k] & 0xffff) << LOG];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              ax[k] = fma(mv[k], xv[k].x, ax[k]);
              ay[k] = fma(mv[k], xv[k].y, ay[k]);
            }
          }
        }
      }
      sx = (ax[0] + ax[1]) + (ax[2] + ax[3]);
      sy = (ay[0] + ay[1]) + (ay[2] + ay[3]);
    };
    // step 1: Vbar for this group's gamma rows (overwrites the nodal values)
    for (int r = 0; r < rmax; ++r) {
      const int2 rw = rr1[r];
      if (rw.x < 0) break;
      double sx = 0.0, sy = 0.0;
      contract(re1, gq, rw.y & 0xffff, (unsigned)rw.y >> 16, sx, sy);
      const double sc = tgs[rw.x];
      vq[rw.x << LOG] = make_double2(sx * sc, sy * sc);
    }
    __syncthreads();
    // step 2 and the node contributions, row by row
    const double w = sW[q];
    const int el = q >> 2;
    const int nloc = (ey0 + el / SW + (ql >> 1)) * 5 + ex0 + el % SW + (ql & 1);
    for (int r = 0; r < rmax; ++r) {
      const int2 rw = rr2[r];
      if (rw.x < 0) break;
      const int s2 = rw.x;
      double sx = 0.0, sy = 0.0;
      contract(re2, vq, rw.y & 0xffff, (unsigned)rw.y >> 16, sx, sy);
      const double sr = trs[s2] * w;
      double flx = sr * sx, fly = sr * sy;
      const int dc = rdcol[s2];
      if (dc >= 0) {
        const double2 gu = gq[dc << LOG];
        const double am = a_min * tra[s2];
        flx = fma(am, gu.x, flx);
        fly = fma(am, gu.y, fly);
      }
      double c4[4];
#pragma unroll
      for (int a4 = 0; a4 < 4; ++a4) c4[a4] = 0.25 * (gpx[a4] * flx + gpy[a4] * fly);
#pragma unroll
      for (int a4 = 0; a4 < 4; ++a4) {
        c4[a4] += __shfl_xor(c4[a4], 1);
        c4[a4] += __shfl_xor(c4[a4], 2);
      }
      const double mine = (ql == 0) ? c4[0] : (ql == 1) ? c4[1] : (ql == 2) ? c4[2] : c4[3];
      if (QB == 64) {
        // node (gnx, gny) = corner 3 of element (x-1, y-1) + corner 2 of (x, y-1)
        //                 + corner 1 of (x-1, y) + corner 0 of (x, y), in that order
        const long long bits = __double_as_longlong(mine);
        const int lo = (int)bits, hi = (int)(bits >> 32);
        double sum = 0.0;
#pragma unroll
        for (int k = 3; k >= 0; --k) {
          const int l2 = __builtin_amdgcn_ds_bpermute(src[k], lo);
          const int h2 = __builtin_amdgcn_ds_bpermute(src[k], hi);
          const double v = __longlong_as_double(((long long)h2 << 32) | (unsigned)l2);
          if (has[k]) sum += v;
        }
        if ((tid & 63) < 25) {
          if (gnx <= 3 && gny <= 3) {
            const int gx = x0 + gnx, gy = y0 + gny;
            if (gx >= 1 && gy >= 1) {
              const int64_t node = (int64_t)(gy - 1) * m + (gx - 1);
              double base = 0.0;
              if (beta != 0.0) base = beta * rin[(int64_t)blob[rs.o_rows + s2] * Nh + node];
              out[(int64_t)s2 * Nh + node] = base + sgn * sum;
            }
          } else {
            const int ei = (gnx == 4 && gny == 4) ? 8 : (gnx == 4 ? gny : 4 + gnx);
            edge[((int64_t)s2 * ntiles + tile) * kEdgeVals + ei] = sum;
          }
        }
      } else {
        double* dst = sNode + s2 * 25 + nloc;
        // the same local corner of distinct elements is a distinct node, so one
        // phase per corner gives a fixed summation order without atomics; a row
        // belongs to one group, whose lanes all sit in one wavefront
#pragma unroll
        for (int a4 = 0; a4 < 4; ++a4) {
          if (ql == a4) *dst += mine;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
    }
  }
  if (QB == 64) return;
  __syncthreads();
  // tile nodes: owned -> out, right/top edge and corner -> edge buffer
  const int* trows = sB + rs.o_rows;
  for (int idx = tid; idx < nrows * 25; idx += 256) {
    const int slot = idx / 25, nd = idx - slot * 25;
    const int nx = nd % 5, ny = nd / 5;
    const double sum = sNode[idx];
    if (nx <= 3 && ny <= 3) {
      const int gx = x0 + nx, gy = y0 + ny;
      if (gx >= 1 && gy >= 1) {
        const int64_t node = (int64_t)(gy - 1) * m + (gx - 1);
        double base = 0.0;
        if (beta != 0.0) base = beta * rin[(int64_t)trows[slot] * Nh + node];
        out[(int64_t)slot * Nh + node] = base + sgn * sum;
      }
    } else {
      const int e = (nx == 4 && ny == 4) ? 8 : (nx == 4 ? ny : 4 + nx);
      edge[((int64_t)slot * ntiles + tile) * kEdgeVals + e] = sum;
    }
  }
}

template <int QB>
__global__ __launch_bounds__(256) void fapply_kernel(int n, double mu, double a_min,
                                                     const double* __restrict__ g, FRowSetDev rs,
                                                     const int* __restrict__ blob,
                                                     const double* __restrict__ U, int64_t Nh,
                                                     const double* __restrict__ rin, double beta,
                                                     double sgn, double* __restrict__ out,
                                                     double* __restrict__ edge) {
  extern __shared__ double smem[];
  const int nt = n / kTileE;
  fapply_tile<QB>(smem, xcd_tile(blockIdx.x, nt * nt), n, mu, a_min, g, rs, blob, U, Nh, rin,
                  beta, sgn, out, edge);
}

void launch_fapply(hipStream_t s, int n, double mu, double a_min, const double* g,
                   const FRowSetDev& rs, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge, bool fixup) {
  const int nt = n / kTileE;
  const int ntiles = nt * nt;
  const size_t lds =
      fapply_lds_bytes(rs.qb, rs.nrows, rs.ncols, rs.ngam, rs.nmono, rs.M, rs.nblob);
  if (lds > 160 * 1024 || rs.ncols < 1 || rs.ncols > 65535 || rs.ngam > 65535 || rs.nblob % 4)
    throw Error(SG_ERR_INTERNAL, "factored apply: bad sub-batch plan");
  switch (rs.qb) {
#define SG_FAPPLY_CASE(Q)                                                                    \
  case Q:                                                                                    \
    hipLaunchKernelGGL(fapply_kernel<Q>, dim3(ntiles), dim3(256), lds, s, n, mu, a_min, g,   \
                       rs, rs.blob, U, Nh, rin, beta, sgn, out, edge);                       \
    break;
    SG_FAPPLY_CASE(8)
    SG_FAPPLY_CASE(16)
    SG_FAPPLY_CASE(32)
    SG_FAPPLY_CASE(64)
#undef SG_FAPPLY_CASE
    default:
      throw Error(SG_ERR_INTERNAL, "factored apply: bad sub-batch size");
  }
  if (fixup) launch_apply_fixup(s, n, rs.nrows, sgn, edge, out, Nh);
}

// ---------------------------------------------------------------------------
// Mode gather/scatter for the field-split groups.
// ---------------------------------------------------------------------------
__global__ void gather_modes_kernel(int modes, const int* __restrict__ idx, int64_t Nh,
                                    const double* __restrict__ src, double* __restrict__ dst,
                                    int scatter) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Nh * modes) return;
  const int64_t node = gid % Nh;
  const int t = (int)(gid / Nh);
  const int64_t full = (int64_t)idx[t] * Nh + node;
  if (scatter) dst[full] = src[gid];
  else dst[gid] = src[full];
}

void launch_gather_modes(hipStream_t s, int modes, const int* idx, int64_t Nh, const double* src,
                         double* dst) {
  hipLaunchKernelGGL(gather_modes_kernel, dim3(cdiv(Nh * modes, 256)), dim3(256), 0, s, modes, idx,
                     Nh, src, dst, 0);
}

void launch_scatter_modes(hipStream_t s, int modes, const int* idx, int64_t Nh, const double* src,
                          double* dst) {
  hipLaunchKernelGGL(gather_modes_kernel, dim3(cdiv(Nh * modes, 256)), dim3(256), 0, s, modes, idx,
                     Nh, src, dst, 1);
}

__global__ void zero_kernel(double* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

void launch_zero(hipStream_t s, double* x, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, x, n);
}

// ---------------------------------------------------------------------------
// Krylov helpers.  Dots: every block reduces a fixed contiguous slice in a
// fixed tree, partials are summed by one wavefront in block order.
// ---------------------------------------------------------------------------
constexpr int kDotThreads = 256;

int dot_blocks(int64_t N) {
  int64_t b = (N + 4 * kDotThreads - 1) / (4 * kDotThreads);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  // wavefront tree then across the block's four wavefronts
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[l * nblk + block] = sum over the block's slice of V_l . w
__global__ __launch_bounds__(kDotThreads) void multidot_kernel(
    const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ w, int64_t N,
    double* __restrict__ partial, int nblk) {
  __shared__ double red[4];
  const int64_t per = (N + nblk - 1) / nblk;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = std::min<int64_t>(N, lo + per);
  for (int l = 0; l < nv; ++l) {
    const double* v = V + (int64_t)l * ldv;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kDotThreads) acc = fma(v[i], w[i], acc);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)l * nblk + blockIdx.x] = s;
  }
}

void launch_multidot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* w,
                     int64_t N, double* partial, int nblk) {
  hipLaunchKernelGGL(multidot_kernel, dim3(nblk), dim3(kDotThreads), 0, s, V, ldv, nv, w, N,
                     partial, nblk);
}

// out[l] = sum_b partial[l * nblk + b], one wavefront per l
__global__ void reduce_kernel(const double* __restrict__ partial, int nblk, int nv,
                              double* __restrict__ out) {
  const int l = blockIdx.x;
  if (l >= nv) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += partial[(int64_t)l * nblk + b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (threadIdx.x == 0) out[l] = acc;
}

void launch_reduce(hipStream_t s, const double* partial, int nblk, int nv, double* out) {
  hipLaunchKernelGGL(reduce_kernel, dim3(nv), dim3(64), 0, s, partial, nblk, nv, out);
}

// w += sign * sum_l h[l] V_l
__global__ void update_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                              const double* __restrict__ h, double* __restrict__ w, int64_t N,
                              double sign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int l = 0; l < nv; ++l) acc = fma(h[l], V[(int64_t)l * ldv + i], acc);
  w[i] += sign * acc;
}

void launch_update(hipStream_t s, const double* V, int64_t ldv, int nv, const double* h, double* w,
                   int64_t N, double sign) {
  hipLaunchKernelGGL(update_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, V, ldv, nv, h, w, N, sign);
}

// ---------------------------------------------------------------------------
// Register-blocked Gram-Schmidt passes.  One element per thread (block b,
// thread t: element b * kDotThreads + t), all of a thread's basis loads in
// flight at once, and one reduction per block at the end instead of one per
// basis vector.  Per-block partial sums go to partial[l * nblk + b] with
// nblk = ceil(N / kDotThreads) and are summed by reduce_wide_kernel.
// ---------------------------------------------------------------------------
int gs_blocks(int64_t N) { return (int)std::max<int64_t>(1, cdiv(N, kDotThreads)); }

// Sums NVB (a power of two <= 64) per-lane values over a wavefront and writes
// the NVB totals to red[0..NVB).  A butterfly: at each exchange step a lane
// keeps half of its values and adds the partner lane's copy of that half, so
// the NVB sums cost NVB - 1 exchanges; after log2(NVB) steps lane L holds the
// sum for index L >> (6 - log2 NVB) over its lane group, finished by plain
// exchanges over the remaining lane bits.
template <int HALF, int OFF, int NVB>
__device__ __forceinline__ void wave_fold(double (&a)[NVB], int lane) {
  if constexpr (HALF >= 1) {
    const bool hi = (lane & OFF) != 0;
#pragma unroll
    for (int j = 0; j < HALF; ++j) {
      const double send = hi ? a[j] : a[j + HALF];
      const double keep = hi ? a[j + HALF] : a[j];
      a[j] = keep + __shfl_xor(send, OFF);
    }
    wave_fold<HALF / 2, OFF / 2, NVB>(a, lane);
  }
}

template <int NVB>
__device__ __forceinline__ void wave_sums(double (&a)[NVB], double* __restrict__ red) {
  constexpr int kShift = NVB == 1 ? 6 : NVB == 2 ? 5 : NVB == 4 ? 4 : NVB == 8 ? 3 : NVB == 16 ? 2 : NVB == 32 ? 1 : 0;
  static_assert((1 << (6 - kShift)) == NVB, "NVB must be a power of two <= 64");
  const int lane = threadIdx.x & 63;
  wave_fold<NVB / 2, 32, NVB>(a, lane);
  double v = a[0];
#pragma unroll
  for (int off = (1 << kShift) >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((lane & ((1 << kShift) - 1)) == 0) red[lane >> kShift] = v;
}

// Combines the four wavefronts' totals (red[w * 64 + l]) into the block's partials.
__device__ __forceinline__ void block_partials(const double* __restrict__ red, int nv,
                                               double* __restrict__ partial, int nblk, int l0) {
  __syncthreads();
  const int l = threadIdx.x;
  if (l < nv)
    partial[(int64_t)(l0 + l) * nblk + blockIdx.x] = (red[l] + red[64 + l]) + (red[128 + l] + red[192 + l]);
}

// partial[(l0 + l) * nblk + b] = block b's part of V_{l0+l} . w, l < min(64, nv - l0),
// with l0 = 64 * blockIdx.y
template <int NVB>
__global__ __launch_bounds__(kDotThreads) void gs_dot_kernel(const double* __restrict__ V,
                                                            int64_t ldv, int nv,
                                                            const double* __restrict__ w,
                                                            int64_t N, double* __restrict__ partial,
                                                            int nblk, EdgeFix ef) {
  __shared__ double red[4 * 64];
  const int l0 = 64 * blockIdx.y;
  const int cnt = min(nv - l0, NVB);
  const int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  const bool in = i < N;
  const double wi = in ? w_fixed(w, i, ef) : 0.0;
  const double* Vb = V + (int64_t)l0 * ldv + i;
  double a[NVB];
#pragma unroll
  for (int l = 0; l < NVB; ++l) a[l] = (l < cnt && in) ? Vb[(int64_t)l * ldv] : 0.0;
#pragma unroll
  for (int l = 0; l < NVB; ++l) a[l] *= wi;
  wave_sums<NVB>(a, red + 64 * (threadIdx.x >> 6));
  block_partials(red, cnt, partial, nblk, l0);
}

// w <- w + sign * sum_l h[l] V_l, then partial[l * nblk + b] = block b's part of
// V_l . w (the new w), nv <= NVB <= 32: the basis values stay in registers
// between the update and the dots, so V is read once for both.
template <int NVB>
__global__ __launch_bounds__(kDotThreads) void gs_update_dot_kernel(
    const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
    double* __restrict__ w, int64_t N, double sign, double* __restrict__ partial, int nblk,
    EdgeFix ef) {
  __shared__ double red[4 * 64];
  const int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  const bool in = i < N;
  double a[NVB];
#pragma unroll
  for (int l = 0; l < NVB; ++l) a[l] = (l < nv && in) ? V[(int64_t)l * ldv + i] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < NVB; ++l)
    if (l < nv) acc = fma(h[l], a[l], acc);
  double wi = 0.0;
  if (in) {
    wi = w_fixed(w, i, ef) + sign * acc;
    w[i] = wi;
  }
#pragma unroll
  for (int l = 0; l < NVB; ++l) a[l] *= wi;
  wave_sums<NVB>(a, red + 64 * (threadIdx.x >> 6));
  block_partials(red, nv, partial, nblk, 0);
}

// partial[(l0 + l) * gridDim.x + b] = block b's part of V_{l0+l} . w with
// l0 = kStreamVecs * blockIdx.y: a grid-stride loop over at most kStreamBlocks
// blocks keeps kStreamVecs dot products per thread in registers, so a block
// reduces once over many elements and the partials to sum are few.  Used for
// nv > kStreamVecs, where it moves more bytes per second than one element per
// thread with all nv values in registers.
constexpr int kStreamBlocks = 512;
constexpr int kStreamVecs = 16;
__global__ __launch_bounds__(kDotThreads) void gs_dot_stream_kernel(
    const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ w, int64_t N,
    double* __restrict__ partial, EdgeFix ef) {
  __shared__ double red[4 * 64];
  const int l0 = kStreamVecs * blockIdx.y;
  const int cnt = min(nv - l0, kStreamVecs);
  const double* Vb = V + (int64_t)l0 * ldv;
  double acc[kStreamVecs];
#pragma unroll
  for (int l = 0; l < kStreamVecs; ++l) acc[l] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kDotThreads) {
    const double wi = w_fixed(w, i, ef);
    double a[kStreamVecs];
#pragma unroll
    for (int l = 0; l < kStreamVecs; ++l) a[l] = l < cnt ? Vb[(int64_t)l * ldv + i] : 0.0;
#pragma unroll
    for (int l = 0; l < kStreamVecs; ++l) acc[l] = fma(a[l], wi, acc[l]);
  }
  wave_sums<kStreamVecs>(acc, red + 64 * (threadIdx.x >> 6));
  block_partials(red, cnt, partial, gridDim.x, l0);
}

// The update-and-dots pass for 32 < nv <= 64 with each element shared by a lane
// pair: the even lane holds V_0..V_31, the odd lane V_32..V_63, so a lane keeps
// 32 basis values in registers rather than 64 and three times as many
// wavefronts stay resident.  The two halves of sum_l h[l] V_l meet in one
// exchange (a + b and b + a round alike, so both lanes hold the same new w);
// a five-step butterfly over the other lane bits leaves lane L with the block
// wavefront's sum for basis vector 32 * (L & 1) + (L >> 1).  A block of
// 2 * kDotThreads threads covers kDotThreads elements, so the partials keep the
// one-lane layout partial[l * nblk + b], nblk = gs_blocks(N).
constexpr int kPairThreads = 2 * kDotThreads;
__global__ __launch_bounds__(kPairThreads) void gs_update_dot_pair_kernel(
    const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
    double* __restrict__ w, int64_t N, double sign, double* __restrict__ partial, int nblk,
    EdgeFix ef) {
  __shared__ double red[8 * 64];
  const int lane = threadIdx.x & 63;
  const int q = lane & 1;
  const int lb = 32 * q;
  const int64_t i = (int64_t)blockIdx.x * kDotThreads + (threadIdx.x >> 1);
  const bool in = i < N;
  double a[32];
#pragma unroll
  for (int l = 0; l < 32; ++l) a[l] = (lb + l < nv && in) ? V[(int64_t)(lb + l) * ldv + i] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < 32; ++l) {
    const double h0 = h[l];
    const double h1 = 32 + l < nv ? h[32 + l] : 0.0;
    acc = fma(q ? h1 : h0, a[l], acc);
  }
  acc += __shfl_xor(acc, 1);
  double wi = 0.0;
  if (in) {
    wi = w_fixed(w, i, ef) + sign * acc;
    if (q == 0) w[i] = wi;
  }
#pragma unroll
  for (int l = 0; l < 32; ++l) a[l] *= wi;
  wave_fold<16, 32, 32>(a, lane);
  red[64 * (threadIdx.x >> 6) + 32 * q + (lane >> 1)] = a[0];
  __syncthreads();
  const int l = threadIdx.x;
  if (l < nv)
    partial[(int64_t)l * nblk + blockIdx.x] = ((red[l] + red[64 + l]) + (red[128 + l] + red[192 + l])) +
                                              ((red[256 + l] + red[320 + l]) + (red[384 + l] + red[448 + l]));
}

// w <- w + sign * sum_l h[l] V_l, then partial[b] = block b's part of w . w;
// a grid-stride loop over at most kNormBlocks blocks, so the norm's partials
// are few enough for every block of the scaling kernel to sum them itself
constexpr int kNormBlocks = 1024;
__global__ __launch_bounds__(kDotThreads) void gs_update_norm_kernel(
    const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ h,
    double* __restrict__ w, int64_t N, double sign, double* __restrict__ partial) {
  __shared__ double red[4 * 64];
  double a[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kDotThreads) {
    double acc = 0.0;
#pragma unroll 8
    for (int l = 0; l < nv; ++l) acc = fma(h[l], V[(int64_t)l * ldv + i], acc);
    const double wi = w[i] + sign * acc;
    w[i] = wi;
    a[0] = fma(wi, wi, a[0]);
  }
  wave_sums<1>(a, red + 64 * (threadIdx.x >> 6));
  block_partials(red, 1, partial, gridDim.x, 0);
}

// v = w / |w| with |w|^2 = sum_b partial[b] (b < nblk), summed by every block
// in the same fixed order; block 0 stores |w|^2 in *nrm2
__global__ __launch_bounds__(kDotThreads) void scale_norm_kernel(const double* __restrict__ w,
                                                                const double* __restrict__ partial,
                                                                int nblk, double* __restrict__ nrm2,
                                                                double* __restrict__ v, int64_t N) {
  __shared__ double red[4];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * kDotThreads < nblk; b += 4 * kDotThreads) {
    a0 += partial[b];
    a1 += partial[b + kDotThreads];
    a2 += partial[b + 2 * kDotThreads];
    a3 += partial[b + 3 * kDotThreads];
  }
  for (; b < nblk; b += kDotThreads) a0 += partial[b];
  const double nn2 = block_sum((a0 + a1) + (a2 + a3), red);
  if (blockIdx.x == 0 && threadIdx.x == 0) *nrm2 = nn2;
  const double nn = sqrt(nn2);
  const int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  if (i < N) v[i] = nn > 0.0 ? w[i] / nn : 0.0;
}

// out[l] = sum_b partial[l * nblk + b]: one block per l, four fixed strided
// accumulators per thread, then the block tree
__global__ __launch_bounds__(kDotThreads) void reduce_wide_kernel(const double* __restrict__ partial,
                                                                 int nblk, double* __restrict__ out) {
  __shared__ double red[4];
  const double* p = partial + (int64_t)blockIdx.x * nblk;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * kDotThreads < nblk; b += 4 * kDotThreads) {
    a0 += p[b];
    a1 += p[b + kDotThreads];
    a2 += p[b + 2 * kDotThreads];
    a3 += p[b + 3 * kDotThreads];
  }
  for (; b < nblk; b += kDotThreads) a0 += p[b];
  const double v = block_sum((a0 + a1) + (a2 + a3), red);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

void launch_gs_dot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                   double* partial, double* out, const EdgeFix& ef) {
  if (nv > kStreamVecs) {
    const int nb = std::min(gs_blocks(N), kStreamBlocks);
    hipLaunchKernelGGL(gs_dot_stream_kernel, dim3(nb, cdiv(nv, kStreamVecs)), dim3(kDotThreads), 0,
                       s, V, ldv, nv, w, N, partial, ef);
    hipLaunchKernelGGL(reduce_wide_kernel, dim3(nv), dim3(kDotThreads), 0, s, partial, nb, out);
    return;
  }
  const int nblk = gs_blocks(N);
  const int top = std::min(nv, 64);
  dim3 grid(nblk, cdiv(nv, 64)), block(kDotThreads);
#define SG_GS_DOT(B)                                                                          \
  if (top <= B) {                                                                             \
    hipLaunchKernelGGL(gs_dot_kernel<B>, grid, block, 0, s, V, ldv, nv, w, N, partial, nblk, ef); \
  } else
  SG_GS_DOT(1) SG_GS_DOT(2) SG_GS_DOT(4) SG_GS_DOT(8) SG_GS_DOT(16) {}
#undef SG_GS_DOT
  hipLaunchKernelGGL(reduce_wide_kernel, dim3(nv), block, 0, s, partial, nblk, out);
}

void launch_gs_update_dot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* h,
                          double* w, int64_t N, double sign, double* partial, double* out,
                          const EdgeFix& ef) {
  if (nv > 64) {
    if (ef.edge) launch_apply_fixup(s, 4 * ef.nt, (int)(N / ef.Nh), ef.sgn, ef.edge, w, ef.Nh);
    launch_update(s, V, ldv, nv, h, w, N, sign);
    launch_gs_dot(s, V, ldv, nv, w, N, partial, out);
    return;
  }
  const int nblk = gs_blocks(N);
  dim3 grid(nblk), block(kDotThreads);
  if (nv > 32) {
    hipLaunchKernelGGL(gs_update_dot_pair_kernel, grid, dim3(kPairThreads), 0, s, V, ldv, nv, h, w,
                       N, sign, partial, nblk, ef);
    hipLaunchKernelGGL(reduce_wide_kernel, dim3(nv), block, 0, s, partial, nblk, out);
    return;
  }
#define SG_GS_UD(B)                                                                          \
  if (nv <= B) {                                                                             \
    hipLaunchKernelGGL(gs_update_dot_kernel<B>, grid, block, 0, s, V, ldv, nv, h, w, N, sign, \
                       partial, nblk, ef);                                                   \
  } else
  SG_GS_UD(1) SG_GS_UD(2) SG_GS_UD(4) SG_GS_UD(8) SG_GS_UD(16) SG_GS_UD(32) {}
#undef SG_GS_UD
  hipLaunchKernelGGL(reduce_wide_kernel, dim3(nv), block, 0, s, partial, nblk, out);
}

void launch_gs_update_norm_scale(hipStream_t s, const double* V, int64_t ldv, int nv,
                                 const double* h, double* w, int64_t N, double sign,
                                 double* partial, double* nrm2, double* vnext) {
  const int nb = std::min(gs_blocks(N), kNormBlocks);
  hipLaunchKernelGGL(gs_update_norm_kernel, dim3(nb), dim3(kDotThreads), 0, s, V, ldv, nv, h, w, N,
                     sign, partial);
  hipLaunchKernelGGL(scale_norm_kernel, dim3(gs_blocks(N)), dim3(kDotThreads), 0, s, w, partial, nb,
                     nrm2, vnext, N);
}

// ---------------------------------------------------------------------------
// Gram-Schmidt with the second projection delayed by one step (two passes over
// the basis per Arnoldi step instead of three).  At step j the basis holds
// orthonormal q_0..q_{j-1} and, in slot j, u_j: the previous step's vector
// after one projection.  With w the operator applied to u_j:
//   pass A   s = Q^T u_j, t = Q^T w, u_j.u_j, u_j.w, w.w      (one read of Q)
//   coefs    nu = |u_j - Q s|, c_j = q_j . w, rho = |w - Q_{0..j} c| / nu
//            (by Pythagoras, with c = (t, c_j))
//   pass B   q_j = (u_j - Q s) / nu            (slot j, in place)
//            u_{j+1} = (w - Q t - c_j q_j) / (nu rho)       (slot j + 1)
// so q_j receives its second projection one step late, and u_{j+1} its first.
// The host keeps the Arnoldi relation exact by expressing each step in the
// vectors it actually applied the operator to (u_j = nu_j q_j + Q s_j).
// ---------------------------------------------------------------------------
constexpr int kPassVecs = 16;

// Shape of pass A for nv <= kPassVecs basis vectors (one block row): VB
// vectors per block, U elements per thread and loop iteration, at most
// `blocks` blocks.  Few basis vectors leave a thread few loads per iteration,
// so those shapes take more elements per iteration and more blocks.
struct Gs2Shape {
  int vb, u, blocks;
};
Gs2Shape gs2_shape(int nv) {
  if (nv <= 4) return {4, 4, 2048};
  if (nv <= 8) return {8, 2, 1024};
  return {16, 1, 1024};
}

// Above kPassVecs basis vectors pass A runs gs2_dotc_kernel: each block owns
// E kDotThreads consecutive elements, E <= 4 chosen so that a vector fills at
// least about 2048 blocks.
constexpr int kChunkMinBlocks = 2048;
int gs2_chunk(int64_t N) {
  int e = 4;
  while (e > 1 && N < (int64_t)e * kDotThreads * kChunkMinBlocks) e >>= 1;
  return e;
}
int gs2_dot_blocks(int nv, int64_t N) {
  if (nv > kPassVecs) return (int)std::max<int64_t>(1, cdiv(N, (int64_t)gs2_chunk(N) * kDotThreads));
  return std::min(gs_blocks(N), gs2_shape(nv).blocks);
}

int gs2_dot_slots(int nv, bool with_w) { return with_w ? 2 * nv + 3 : nv + 1; }
size_t gs2_partial_doubles(int max_nv, int64_t N) {
  size_t most = 0;
  for (int nv = 0; nv <= max_nv; ++nv)
    most = std::max(most, (size_t)gs2_dot_slots(nv, true) * gs2_dot_blocks(nv, N));
  return most;
}

// Block partials of Q_l . u (slot l < nv), Q_l . w (slot nv + l) and, from the
// first row of blocks, u.u, u.w, w.w (slots 2 nv .. 2 nv + 2; without w only
// Q_l . u and u.u at slot nv).  Grid-stride over elements, VB basis vectors
// per block row, U elements per iteration.
template <int VB, int U>
__global__ __launch_bounds__(kDotThreads) void gs2_dot_kernel(
    const double* __restrict__ Q, int64_t ldq, int nv, const double* __restrict__ u,
    const double* __restrict__ w, int64_t N, double* __restrict__ partial, EdgeFix ef) {
  constexpr int NA = 2 * VB + 3 <= 16 ? 16 : 2 * VB + 3 <= 32 ? 32 : 64;
  __shared__ double red[4 * 64];
  const int l0 = VB * blockIdx.y;
  const int cnt = max(0, min(nv - l0, VB));
  const bool extras = blockIdx.y == 0;
  const bool hasw = w != nullptr;
  const double* Qb = Q + (int64_t)l0 * ldq;
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kDotThreads;
  for (int64_t i0 = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i0 < N; i0 += U * stride) {
    double ui[U], wi[U], a[U][VB];
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const int64_t i = i0 + e * stride;
      const bool in = i < N;
      ui[e] = in ? u[i] : 0.0;
      wi[e] = in && hasw ? w_fixed(w, i, ef) : 0.0;
#pragma unroll
      for (int l = 0; l < VB; ++l) a[e][l] = in && l < cnt ? Qb[(int64_t)l * ldq + i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < U; ++e) {
#pragma unroll
      for (int l = 0; l < VB; ++l) {
        acc[l] = fma(a[e][l], ui[e], acc[l]);
        acc[VB + l] = fma(a[e][l], wi[e], acc[VB + l]);
      }
      if (extras) {
        acc[2 * VB] = fma(ui[e], ui[e], acc[2 * VB]);
        acc[2 * VB + 1] = fma(ui[e], wi[e], acc[2 * VB + 1]);
        acc[2 * VB + 2] = fma(wi[e], wi[e], acc[2 * VB + 2]);
      }
    }
  }
  wave_sums<NA>(acc, red + 64 * (threadIdx.x >> 6));
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= NA) return;
  int slot = -1;
  if (k < VB) {
    if (k < cnt) slot = l0 + k;
  } else if (k < 2 * VB) {
    if (hasw && k - VB < cnt) slot = nv + l0 + (k - VB);
  } else if (extras && k < 2 * VB + 3) {
    const int e = k - 2 * VB;
    if (e == 0 || hasw) slot = (hasw ? 2 * nv : nv) + e;
  }
  if (slot >= 0)
    partial[(int64_t)slot * gridDim.x + blockIdx.x] = (red[k] + red[64 + k]) + (red[128 + k] + red[192 + k]);
}

// Pass A for more than kPassVecs basis vectors, with the slots of
// gs2_dot_kernel.  A block owns elements [b E T, (b + 1) E T) (T =
// kDotThreads), keeps their u and w (pending edge sums added once) in
// registers and runs over the basis in groups of eight vectors, writing each
// group's block partials before the next: u and w are read once whatever nv
// is, and the basis once.  (Groups of 16, eight elements per thread, or
// per-wavefront partials without the barriers measured 2-5% slower.)
template <int E>
__global__ __launch_bounds__(kDotThreads) void gs2_dotc_kernel(
    const double* __restrict__ Q, int64_t ldq, int nv, const double* __restrict__ u,
    const double* __restrict__ w, int64_t N, double* __restrict__ partial, EdgeFix ef) {
  constexpr int VB = 8;
  __shared__ double red[4 * 64];
  const bool hasw = w != nullptr;
  const int64_t i0 = (int64_t)blockIdx.x * (E * kDotThreads) + threadIdx.x;
  double ui[E], wi[E];
  double ex[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = i0 + (int64_t)e * kDotThreads;
    const bool in = i < N;
    ui[e] = in ? u[i] : 0.0;
    wi[e] = in && hasw ? w_fixed(w, i, ef) : 0.0;
    ex[0] = fma(ui[e], ui[e], ex[0]);
    ex[1] = fma(ui[e], wi[e], ex[1]);
    ex[2] = fma(wi[e], wi[e], ex[2]);
  }
  double* redw = red + 64 * (threadIdx.x >> 6);
  const int k = threadIdx.x;
  for (int l0 = 0; l0 < nv; l0 += VB) {
    const int cnt = min(nv - l0, VB);
    const double* Qb = Q + (int64_t)l0 * ldq;
    double acc[2 * VB];
#pragma unroll
    for (int l = 0; l < 2 * VB; ++l) acc[l] = 0.0;
#pragma unroll 1
    for (int e = 0; e < E; ++e) {
      const int64_t i = i0 + (int64_t)e * kDotThreads;
      const bool in = i < N;
      double a[VB];
#pragma unroll
      for (int l = 0; l < VB; ++l) a[l] = in && l < cnt ? Qb[(int64_t)l * ldq + i] : 0.0;
#pragma unroll
      for (int l = 0; l < VB; ++l) {
        acc[l] = fma(a[l], ui[e], acc[l]);
        acc[VB + l] = fma(a[l], wi[e], acc[VB + l]);
      }
    }
    wave_sums<2 * VB>(acc, redw);
    __syncthreads();
    int slot = -1;
    if (k < VB) {
      if (k < cnt) slot = l0 + k;
    } else if (k < 2 * VB) {
      if (hasw && k - VB < cnt) slot = nv + l0 + (k - VB);
    }
    if (slot >= 0)
      partial[(int64_t)slot * gridDim.x + blockIdx.x] = (red[k] + red[64 + k]) + (red[128 + k] + red[192 + k]);
    __syncthreads();  // red is rewritten by the next group
  }
  wave_sums<4>(ex, redw);
  __syncthreads();
  if (k < 3 && (k == 0 || hasw))
    partial[(int64_t)((hasw ? 2 * nv : nv) + k) * gridDim.x + blockIdx.x] =
        (red[k] + red[64 + k]) + (red[128 + k] + red[192 + k]);
}

void launch_gs2_dot(hipStream_t s, const double* Q, int64_t ldq, int nv, const double* u,
                    const double* w, int64_t N, double* partial, double* out, const EdgeFix& ef) {
  if (nv > kPassVecs) {
    const int nb = gs2_dot_blocks(nv, N);
    const dim3 grid(nb), block(kDotThreads);
    switch (gs2_chunk(N)) {
      case 4:
        hipLaunchKernelGGL(gs2_dotc_kernel<4>, grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
        break;
      case 2:
        hipLaunchKernelGGL(gs2_dotc_kernel<2>, grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
        break;
      default:
        hipLaunchKernelGGL(gs2_dotc_kernel<1>, grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
    }
    hipLaunchKernelGGL(reduce_wide_kernel, dim3(gs2_dot_slots(nv, w != nullptr)), block, 0, s,
                       partial, nb, out);
    return;
  }
  const Gs2Shape sh = gs2_shape(nv);
  const int nb = gs2_dot_blocks(nv, N);
  const int ny = std::max(1, cdiv(nv, sh.vb));
  const dim3 grid(nb, ny), block(kDotThreads);
  if (sh.vb == 4)
    hipLaunchKernelGGL((gs2_dot_kernel<4, 4>), grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
  else if (sh.vb == 8)
    hipLaunchKernelGGL((gs2_dot_kernel<8, 2>), grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
  else
    hipLaunchKernelGGL((gs2_dot_kernel<16, 1>), grid, block, 0, s, Q, ldq, nv, u, w, N, partial, ef);
  hipLaunchKernelGGL(reduce_wide_kernel, dim3(gs2_dot_slots(nv, w != nullptr)), block, 0, s,
                     partial, nb, out);
}

// coef[0] = nu, coef[1] = c_j, coef[2] = rho, coef[3] = |w - Q c|^2 before the
// floor, from dots = (s, t, u.u, u.w, w.w) of pass A; the sums run in index
// order.  rho^2 is floored at 1e-28 w.w / nu^2 so that a cancelled Pythagorean
// difference only mis-scales u_{j+1} (the next step measures its norm).
__global__ void gs2_coef_kernel(int nv, const double* __restrict__ dots, double* __restrict__ coef) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double* sv = dots;
  const double* tv = dots + nv;
  double ss = 0.0, st = 0.0, tt = 0.0;
  for (int l = 0; l < nv; ++l) {
    ss = fma(sv[l], sv[l], ss);
    st = fma(sv[l], tv[l], st);
    tt = fma(tv[l], tv[l], tt);
  }
  const double uu = dots[2 * nv], uw = dots[2 * nv + 1], ww = dots[2 * nv + 2];
  const double nu = sqrt(uu - ss);
  const double cj = (uw - st) / nu;
  const double r2 = ww - tt - cj * cj;
  const double rho = sqrt(fmax(r2, 1e-28 * ww)) / nu;
  coef[0] = nu;
  coef[1] = cj;
  coef[2] = rho;
  coef[3] = r2;
}

void launch_gs2_coef(hipStream_t s, int nv, const double* dots, double* coef) {
  hipLaunchKernelGGL(gs2_coef_kernel, dim3(1), dim3(64), 0, s, nv, dots, coef);
}

// pass B, one element per thread: q_j = (u_j - Q s) / nu in place of u_j, then
// u_{j+1} = (w - Q t - c_j q_j) / (nu rho); the basis values of a chunk of
// kPassVecs vectors are loaded together and serve both sums
__global__ __launch_bounds__(kDotThreads) void gs2_update_kernel(
    const double* __restrict__ Q, int64_t ldq, int nv, const double* __restrict__ sv,
    const double* __restrict__ tv, const double* __restrict__ coef, double* __restrict__ uq,
    const double* __restrict__ w, double* __restrict__ unext, int64_t N, EdgeFix ef) {
  const int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  if (i >= N) return;
  double as = 0.0, at = 0.0;
  for (int l0 = 0; l0 < nv; l0 += kPassVecs) {
    const int cnt = min(nv - l0, kPassVecs);
    double a[kPassVecs];
#pragma unroll
    for (int l = 0; l < kPassVecs; ++l) a[l] = l < cnt ? Q[(int64_t)(l0 + l) * ldq + i] : 0.0;
#pragma unroll
    for (int l = 0; l < kPassVecs; ++l) {
      if (l < cnt) {
        as = fma(sv[l0 + l], a[l], as);
        at = fma(tv[l0 + l], a[l], at);
      }
    }
  }
  const double nu = coef[0], cj = coef[1], rho = coef[2];
  const double q = (uq[i] - as) / nu;
  uq[i] = q;
  unext[i] = (w_fixed(w, i, ef) - at - cj * q) / (nu * rho);
}

void launch_gs2_update(hipStream_t s, const double* Q, int64_t ldq, int nv, const double* sv,
                       const double* tv, const double* coef, double* uq, const double* w,
                       double* unext, int64_t N, const EdgeFix& ef) {
  hipLaunchKernelGGL(gs2_update_kernel, dim3(gs_blocks(N)), dim3(kDotThreads), 0, s, Q, ldq, nv,
                     sv, tv, coef, uq, w, unext, N, ef);
}

// out = sum_l y[l] V_l
__global__ void combine_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                               const double* __restrict__ y, double* __restrict__ out, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int l = 0; l < nv; ++l) acc = fma(y[l], V[(int64_t)l * ldv + i], acc);
  out[i] = acc;
}

void launch_combine(hipStream_t s, const double* V, int64_t ldv, int nv, const double* y,
                    double* out, int64_t N) {
  hipLaunchKernelGGL(combine_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, V, ldv, nv, y, out, N);
}

// v = w / sqrt(nrm2[0]) (v = 0 when the norm vanishes: breakdown)
__global__ void scale_kernel(const double* __restrict__ w, const double* __restrict__ nrm2,
                             double* __restrict__ v, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double nn = sqrt(nrm2[0]);
  v[i] = nn > 0.0 ? w[i] / nn : 0.0;
}

void launch_scale_by_inv_norm(hipStream_t s, const double* w, const double* nrm2, double* v,
                              int64_t N) {
  hipLaunchKernelGGL(scale_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, w, nrm2, v, N);
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b,
                             double* __restrict__ y, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, int64_t N) {
  hipLaunchKernelGGL(axpby_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, a, x, b, y, N);
}

__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = a[i] - b[i];
}

void launch_sub(hipStream_t s, const double* a, const double* b, double* out, int64_t N) {
  hipLaunchKernelGGL(sub_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, a, b, out, N);
}

// out_t = b_t - B_t x_t for m modes stored compactly (entry t*N + node), B_t
// the 9-point stencil of id smode[t] (0: the mean stiffness A_0; i+1: the
// diagonal block K_ii) on the finest level, planes s = 3(dy+1) + (dx+1)
__global__ void stencil_residual_kernel(int n, const double* __restrict__ S,
                                        const int* __restrict__ smode,
                                        const double* __restrict__ b,
                                        const double* __restrict__ x, double* __restrict__ out,
                                        int64_t N) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (node >= N) return;
  const int m = n - 1;
  const int ix = (int)(node % m), iy = (int)(node / m);
  const double* St = S + (int64_t)(smode ? smode[t] : 0) * 9 * N;
  const double* xt = x + (int64_t)t * N;
  double acc = 0.0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int jx = ix + dx, jy = iy + dy;
      if (jx < 0 || jx >= m || jy < 0 || jy >= m) continue;
      acc = fma(St[(int64_t)(3 * (dy + 1) + (dx + 1)) * N + node], xt[(int64_t)jy * m + jx], acc);
    }
  out[(int64_t)t * N + node] = b[(int64_t)t * N + node] - acc;
}

void launch_stencil_residual(hipStream_t s, int n, const double* S, const int* smode, int m,
                             const double* b, const double* x, double* out) {
  const int64_t N = (int64_t)(n - 1) * (n - 1);
  hipLaunchKernelGGL(stencil_residual_kernel, dim3(cdiv(N, 256), m), dim3(256), 0, s, n, S, smode,
                     b, x, out, N);
}

// The learned stage's step weight: alpha = dots[0] / dots[1] (<r, Kc> / ||Kc||^2)
// when both are finite and dots[1] > 0, else 0 (dots[2] receives alpha); then
// z += alpha c and, when w is given, w += alpha Kc.  With alpha = 0 nothing is
// written, so a non-finite prediction leaves z (and w) as they were.
__global__ void stage_alpha_kernel(double* __restrict__ dots, const double* __restrict__ c,
                                   const double* __restrict__ kc, double* __restrict__ z,
                                   double* __restrict__ w, int64_t N) {
  const double num = dots[0], den = dots[1];
  const double alpha = (isfinite(num) && isfinite(den) && den > 0.0) ? num / den : 0.0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) dots[2] = alpha;
  if (alpha == 0.0 || i >= N) return;
  z[i] = fma(alpha, c[i], z[i]);
  if (w) w[i] = fma(alpha, kc[i], w[i]);
}

void launch_stage_alpha(hipStream_t s, double* dots, const double* c, const double* kc, double* z,
                        double* w, int64_t N) {
  hipLaunchKernelGGL(stage_alpha_kernel, dim3(cdiv(N, 256)), dim3(256), 0, s, dots, c, kc, z, w, N);
}


// ===========================================================================
// Fused multigrid V-cycle kernels.
//
// Fine levels run as two kernels each, on tiles of TC x TC coarse nodes (the
// fine nodes 2I-1 and 2I of coarse slot I are owned by that slot's tile; slot
// nc owns the last fine node):
//   vdown: x1 = w D^-1 b, x2 = x1 + w D^-1 (b - A x1), r = b - A x2, b_c = P^T r
//          (halo 2 recomputed per tile), writes x2 and b_c;
//   vup:   x3 = x2 + P x_c, x4, x5 = two more damped Jacobi sweeps, writes x5.
// Levels with n <= kCoarseN run inside one workgroup per mode (vcoarse), with
// every vector and stencil of those levels resident in LDS.
// Each mode may use its own stencil: stencil id smode[t] (0 if smode is null),
// at S + id * 9 * N on every level.
// ===========================================================================
namespace {

constexpr int kTC = 8;                     // coarse nodes per tile side
constexpr int kDE = 2 * kTC + 5;           // fine extent incl. halo 2 (down)
constexpr int kUE = 2 * kTC + 4;           // fine extent incl. halo 2 (up)
constexpr int kCE = kTC + 4;               // coarse extent (up)

__device__ __forceinline__ const double* sel_stencil(const double* S, int64_t N,
                                                     const int* smode, int t) {
  return S + (smode ? (int64_t)smode[t] * 9 * N : 0);
}

}  // namespace

struct VDownLds {
  double sb[kDE * kDE], sd[kDE * kDE], sx1[kDE * kDE], sx2[kDE * kDE], sr[kDE * kDE];
};

// One (tile, mode) item of the down sweep; ends with a barrier, so a workgroup
// may go on to another item with the same LDS.
__device__ __forceinline__ void vdown_tile(VDownLds& L, int tile, int mode,
                                           const double* __restrict__ Sbase, int nf, int64_t Nf,
                                           int64_t Nc, const int* smode, const int* bmap,
                                           const double* __restrict__ bglob,
                                           double* __restrict__ x2out,
                                           double* __restrict__ bcout, double omega,
                                           const EdgeFix& ef = EdgeFix{}) {
  double* sb = L.sb;
  double* sd = L.sd;
  double* sx1 = L.sx1;
  double* sx2 = L.sx2;
  double* sr = L.sr;
  const int mf = nf - 1, nc = nf / 2, mc = nc - 1;
  const int tpr = (nc + kTC - 1) / kTC;
  const int tx = tile % tpr, ty = tile / tpr;
  const double* S = sel_stencil(Sbase, Nf, smode, mode);
  const double* b = bglob + (int64_t)(bmap ? bmap[mode] : mode) * Nf;
  const int I0 = 1 + tx * kTC, J0 = 1 + ty * kTC;
  const int ox = 2 * I0 - 3, oy = 2 * J0 - 3;  // fine index of LDS (0,0)
  const int tid = threadIdx.x;
  auto inside = [&](int fx, int fy) { return fx >= 1 && fx <= mf && fy >= 1 && fy <= mf; };
  auto gidx = [&](int fx, int fy) { return (int64_t)(fy - 1) * mf + (fx - 1); };
  // a thread keeps the same local points (e = tid + 256 p) in every phase: their
  // right-hand side and stencil rows are loaded once, all in flight together
  constexpr int kNP = (kDE * kDE + 255) / 256;
  double sv[kNP][9], bv[kNP];
  int64_t gp[kNP];
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kDE, ly = e / kDE, fx = ox + lx, fy = oy + ly;
    const bool in = e < kDE * kDE && inside(fx, fy);
    gp[p] = in ? gidx(fx, fy) : -1;
    bv[p] = in ? b[gp[p]] : 0.0;
    if (in && ef.edge) bv[p] = edge_fixed(bv[p], ef, mode, fx, fy);
#pragma unroll
    for (int t = 0; t < 9; ++t) sv[p][t] = in ? S[t * Nf + gp[p]] : (t == 4 ? 1.0 : 0.0);
  }
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p;
    if (e < kDE * kDE) {
      sb[e] = bv[p];
      sd[e] = sv[p][4];
      sx1[e] = gp[p] >= 0 ? omega * bv[p] / sv[p][4] : 0.0;
    }
  }
  __syncthreads();
  // x2 on [1, kDE-2)^2 local
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kDE, ly = e / kDE;
    if (e >= kDE * kDE) continue;
    double v = 0.0;
    if (lx >= 1 && lx < kDE - 1 && ly >= 1 && ly < kDE - 1 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx1[(ly + t / 3 - 1) * kDE + (lx + t % 3 - 1)];
      v = sx1[e] + omega * (sb[e] - ax) / sd[e];
    }
    sx2[e] = v;
  }
  __syncthreads();
  // r on [2, kDE-2)^2 local; owned x2 written out
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kDE, ly = e / kDE;
    if (e >= kDE * kDE) continue;
    double v = 0.0;
    if (lx >= 2 && lx < kDE - 2 && ly >= 2 && ly < kDE - 2 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx2[(ly + t / 3 - 1) * kDE + (lx + t % 3 - 1)];
      v = sb[e] - ax;
      if (lx < kDE - 3 && ly < kDE - 3) x2out[(int64_t)mode * Nf + gp[p]] = sx2[e];
    }
    sr[e] = v;
  }
  __syncthreads();
  // restriction to the tile's coarse nodes
  if (tid < kTC * kTC) {
    const int I = I0 + tid % kTC, J = J0 + tid / kTC;
    if (I <= mc && J <= mc) {
      double acc = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const double w = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0);
          acc += w * sr[(2 * J + dy - oy) * kDE + (2 * I + dx - ox)];
        }
      bcout[(int64_t)mode * Nc + (int64_t)(J - 1) * mc + (I - 1)] = acc;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void vdown_kernel(const double* __restrict__ Sbase, int nf,
                                                    int64_t Nf, int64_t Nc, const int* smode,
                                                    const int* bmap,
                                                    const double* __restrict__ bglob,
                                                    double* __restrict__ x2out,
                                                    double* __restrict__ bcout, double omega,
                                                    EdgeFix ef) {
  __shared__ VDownLds L;
  vdown_tile(L, blockIdx.x, blockIdx.y, Sbase, nf, Nf, Nc, smode, bmap, bglob, x2out, bcout,
             omega, ef);
}

struct VUpLds {
  double sb[kUE * kUE], sd[kUE * kUE], sx3[kUE * kUE], sx4[kUE * kUE], sc[kCE * kCE];
};

// One (tile, mode) item of the up sweep; ends with a barrier.
__device__ __forceinline__ void vup_tile(VUpLds& L, int tile, int mode,
                                         const double* __restrict__ Sbase, int nf, int64_t Nf,
                                         int64_t Nc, const int* smode, const int* bmap,
                                         const int* xmap, const double* __restrict__ bglob,
                                         const double* __restrict__ x2glob,
                                         const double* __restrict__ xcglob,
                                         double* __restrict__ xout, double omega,
                                         int64_t xcslab = 0, const EdgeFix& ef = EdgeFix{}) {
  double* sb = L.sb;
  double* sd = L.sd;
  double* sx3 = L.sx3;
  double* sx4 = L.sx4;
  double* sc = L.sc;
  const int mf = nf - 1, nc = nf / 2, mc = nc - 1;
  const int tpr = (nc + kTC - 1) / kTC;
  const int tx = tile % tpr, ty = tile / tpr;
  const double* S = sel_stencil(Sbase, Nf, smode, mode);
  const double* b = bglob + (int64_t)(bmap ? bmap[mode] : mode) * Nf;
  const double* x2 = x2glob + (int64_t)mode * Nf;
  const double* xc = xcglob + (int64_t)mode * Nc;
  const int I0 = 1 + tx * kTC, J0 = 1 + ty * kTC;
  const int ox = 2 * I0 - 3, oy = 2 * J0 - 3;  // fine index of LDS (0,0)
  const int cx0 = I0 - 2, cy0 = J0 - 2;        // coarse index of sc(0,0)
  const int tid = threadIdx.x;
  auto inside = [&](int fx, int fy) { return fx >= 1 && fx <= mf && fy >= 1 && fy <= mf; };
  auto gidx = [&](int fx, int fy) { return (int64_t)(fy - 1) * mf + (fx - 1); };
  // the coarse correction, and for the thread's local points (e = tid + 256 p,
  // the same in every phase) the right-hand side, the pre-smoothed x2 and the
  // stencil rows, all loaded at once
  constexpr int kNP = (kUE * kUE + 255) / 256;
  static_assert(kCE * kCE <= 256, "one coarse value per thread");
  double cv = 0.0;
  {
    const int cx = cx0 + tid % kCE, cy = cy0 + tid / kCE;
    if (tid < kCE * kCE && cx >= 1 && cx <= mc && cy >= 1 && cy <= mc) {
      const int64_t g = (int64_t)(cy - 1) * mc + (cx - 1);
      cv = xc[g];
      if (xcslab) cv = (cv + xc[g + xcslab]) + (xc[g + 2 * xcslab] + xc[g + 3 * xcslab]);
    }
  }
  double sv[kNP][9], bv[kNP], xv[kNP];
  int64_t gp[kNP];
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kUE, ly = e / kUE, fx = ox + lx, fy = oy + ly;
    const bool in = e < kUE * kUE && inside(fx, fy);
    gp[p] = in ? gidx(fx, fy) : -1;
    bv[p] = in ? b[gp[p]] : 0.0;
    if (in && ef.edge) bv[p] = edge_fixed(bv[p], ef, mode, fx, fy);
    xv[p] = in ? x2[gp[p]] : 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) sv[p][t] = in ? S[t * Nf + gp[p]] : (t == 4 ? 1.0 : 0.0);
  }
  if (tid < kCE * kCE) sc[tid] = cv;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kUE, ly = e / kUE, fx = ox + lx, fy = oy + ly;
    if (e >= kUE * kUE) continue;
    double x3 = 0.0;
    if (gp[p] >= 0) {
      // bilinear interpolation from the coarse neighbours
      const int Ia = fx >> 1, Ib = (fx + 1) >> 1, Ja = fy >> 1, Jb = (fy + 1) >> 1;
      auto C = [&](int I, int J) { return sc[(J - cy0) * kCE + (I - cx0)]; };
      double pr;
      if (fx & 1) {
        if (fy & 1) pr = 0.25 * C(Ia, Ja) + 0.25 * C(Ib, Ja) + 0.25 * C(Ia, Jb) + 0.25 * C(Ib, Jb);
        else pr = 0.5 * C(Ia, Ja) + 0.5 * C(Ib, Ja);
      } else {
        if (fy & 1) pr = 0.5 * C(Ia, Ja) + 0.5 * C(Ia, Jb);
        else pr = C(Ia, Ja);
      }
      x3 = xv[p] + pr;
    }
    sb[e] = bv[p];
    sd[e] = sv[p][4];
    sx3[e] = x3;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kUE, ly = e / kUE;
    if (e >= kUE * kUE) continue;
    double v = 0.0;
    if (lx >= 1 && lx < kUE - 1 && ly >= 1 && ly < kUE - 1 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx3[(ly + t / 3 - 1) * kUE + (lx + t % 3 - 1)];
      v = sx3[e] + omega * (sb[e] - ax) / sd[e];
    }
    sx4[e] = v;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kNP; ++p) {
    const int e = tid + 256 * p, lx = e % kUE, ly = e / kUE;
    if (e >= kUE * kUE) continue;
    if (lx >= 2 && lx < kUE - 2 && ly >= 2 && ly < kUE - 2 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx4[(ly + t / 3 - 1) * kUE + (lx + t % 3 - 1)];
      xout[(int64_t)(xmap ? xmap[mode] : mode) * Nf + gp[p]] = sx4[e] + omega * (sb[e] - ax) / sd[e];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void vup_kernel(const double* __restrict__ Sbase, int nf,
                                                  int64_t Nf, int64_t Nc, const int* smode,
                                                  const int* bmap, const int* xmap,
                                                  const double* __restrict__ bglob,
                                                  const double* __restrict__ x2glob,
                                                  const double* __restrict__ xcglob,
                                                  double* __restrict__ xout, double omega,
                                                  int64_t xcslab, EdgeFix ef) {
  __shared__ VUpLds L;
  vup_tile(L, blockIdx.x, blockIdx.y, Sbase, nf, Nf, Nc, smode, bmap, xmap, bglob, x2glob, xcglob,
           xout, omega, xcslab, ef);
}

// ---------------------------------------------------------------------------
// Two fine levels of the V-cycle in one pass each way (levels l and l+1, the
// mean stiffness).  A workgroup takes the T2 x T2 nodes of one level-(l+2)
// tile and recomputes the halos it needs instead of reading them from a
// neighbour, so every value it produces is the one the one-level kernels
// produce (same formulas, same order):
//   down: level l on (4 T2 + 15)^2 nodes (its (4 T2)^2 own nodes plus the halo
//         whose residual restricts onto the (2 T2 + 5)^2 level-(l+1) nodes),
//         then level l+1 as vdown_kernel does, writing level l's pre-smoothed
//         x, level l+1's right-hand side and pre-smoothed x, and level l+2's
//         right-hand side;
//   up:   level l+1's prolong-add and post-smoothing on (2 T2 + 7)^2 nodes (own
//         nodes plus the halo that level l interpolates from), then level l's
//         on (4 T2 + 4)^2 nodes, writing level l's (4 T2)^2 own nodes.
// ---------------------------------------------------------------------------
template <int T2, int NT>
struct V2Geom {
  static constexpr int kT2 = T2;            // level-(l+2) nodes per tile side
  static constexpr int kD1 = 2 * T2 + 5;    // level-(l+1) extent, down
  static constexpr int kD0 = 2 * kD1 + 5;   // level-l extent, down
  static constexpr int kU0 = 4 * T2 + 4;    // level-l extent, up
  static constexpr int kU1 = 2 * T2 + 7;    // level-(l+1) extent, up
  static constexpr int kU2 = T2 + 5;        // level-(l+2) extent, up
  static constexpr int kV2Threads = NT;
  static constexpr size_t down_lds() { return 8 * (5 * (size_t)kD0 * kD0 + 5 * (size_t)kD1 * kD1); }
  static constexpr size_t up_lds() {
    return 8 * (4 * (size_t)kU0 * kU0 + 5 * (size_t)kU1 * kU1 + (size_t)kU2 * kU2);
  }
};

template <int T2, int NT>
__global__ __launch_bounds__(NT) void vdown2_kernel(
    const double* __restrict__ S0, const double* __restrict__ S1, int n0, int64_t N0, int64_t N1,
    int64_t N2, const int* bmap, const double* __restrict__ bglob, double* __restrict__ x2out0,
    double* __restrict__ b1out, double* __restrict__ x2out1, double* __restrict__ b2out,
    double omega, EdgeFix ef) {
  using Gm = V2Geom<T2, NT>;
  constexpr int kT2 = Gm::kT2, kD0 = Gm::kD0, kD1 = Gm::kD1, kV2Threads = NT;
  extern __shared__ double smem[];
  constexpr int A0 = kD0 * kD0, A1 = kD1 * kD1;
  double* sb0 = smem;
  double* sd0 = sb0 + A0;
  double* sx1 = sd0 + A0;
  double* sx2 = sx1 + A0;
  double* sr0 = sx2 + A0;
  double* sb1 = sr0 + A0;
  double* sd1 = sb1 + A1;
  double* sy1 = sd1 + A1;
  double* sy2 = sy1 + A1;
  double* sr1 = sy2 + A1;
  const int mode = blockIdx.y, tid = threadIdx.x;
  const int m0 = n0 - 1, m1 = n0 / 2 - 1, n2 = n0 / 4, m2 = n2 - 1;
  const int tpr = (n2 + kT2 - 1) / kT2;
  const int tx = blockIdx.x % tpr, ty = blockIdx.x / tpr;
  const int I0 = 1 + tx * kT2, J0 = 1 + ty * kT2;       // level l+2, first node
  const int o1x = 2 * I0 - 3, o1y = 2 * J0 - 3;          // level l+1 index of local (0,0)
  const int o0x = 2 * o1x - 3, o0y = 2 * o1y - 3;        // level l index of local (0,0)
  const double* b = bglob + (int64_t)(bmap ? bmap[mode] : mode) * N0;
  auto in0 = [&](int x, int y) { return x >= 1 && x <= m0 && y >= 1 && y <= m0; };
  auto in1 = [&](int x, int y) { return x >= 1 && x <= m1 && y >= 1 && y <= m1; };
  // every global load of both levels at once: level l's right-hand side and
  // stencil rows for the thread's points (e = tid + 512 p), level l+1's rows
  constexpr int kP0 = (A0 + kV2Threads - 1) / kV2Threads;
  static_assert(A1 <= kV2Threads, "one level-(l+1) point per thread");
  double sv[kP0][9], bv[kP0], tv[9];
  int64_t gp[kP0];
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kD0, ly = e / kD0;
    const int fx = o0x + lx, fy = o0y + ly;
    const bool in = e < A0 && in0(fx, fy);
    gp[p] = in ? (int64_t)(fy - 1) * m0 + (fx - 1) : -1;
    bv[p] = in ? b[gp[p]] : 0.0;
    if (in && ef.edge) bv[p] = edge_fixed(bv[p], ef, mode, fx, fy);
#pragma unroll
    for (int t = 0; t < 9; ++t) sv[p][t] = in ? S0[t * N0 + gp[p]] : (t == 4 ? 1.0 : 0.0);
  }
  const int l1x = tid % kD1, l1y = tid / kD1;
  const int k1x = o1x + l1x, k1y = o1y + l1y;
  const bool p1 = tid < A1, inp1 = p1 && in1(k1x, k1y);
  const int64_t g1 = inp1 ? (int64_t)(k1y - 1) * m1 + (k1x - 1) : -1;
#pragma unroll
  for (int t = 0; t < 9; ++t) tv[t] = inp1 ? S1[t * N1 + g1] : (t == 4 ? 1.0 : 0.0);
  // level l: x1 = omega b / d
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p;
    if (e < A0) {
      sb0[e] = bv[p];
      sd0[e] = sv[p][4];
      sx1[e] = gp[p] >= 0 ? omega * bv[p] / sv[p][4] : 0.0;
    }
  }
  __syncthreads();
  // level l: x2 on [1, kD0-1)^2
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kD0, ly = e / kD0;
    if (e >= A0) continue;
    double v = 0.0;
    if (lx >= 1 && lx < kD0 - 1 && ly >= 1 && ly < kD0 - 1 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx1[(ly + t / 3 - 1) * kD0 + (lx + t % 3 - 1)];
      v = sx1[e] + omega * (sb0[e] - ax) / sd0[e];
    }
    sx2[e] = v;
  }
  __syncthreads();
  // level l: residual on [2, kD0-2)^2; own x2 (local [6, 38)^2) written out
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kD0, ly = e / kD0;
    if (e >= A0) continue;
    double v = 0.0;
    if (lx >= 2 && lx < kD0 - 2 && ly >= 2 && ly < kD0 - 2 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx2[(ly + t / 3 - 1) * kD0 + (lx + t % 3 - 1)];
      v = sb0[e] - ax;
      if (lx >= 6 && lx < 6 + 4 * kT2 && ly >= 6 && ly < 6 + 4 * kT2)
        x2out0[(int64_t)mode * N0 + gp[p]] = sx2[e];
    }
    sr0[e] = v;
  }
  __syncthreads();
  // level l+1: right-hand side by restriction, then x1 = omega b / d; own
  // right-hand side (local [2, 18)^2) written out
  if (p1) {
    double bb = 0.0;
    if (inp1) {
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const double wgt = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0);
          bb += wgt * sr0[(2 * k1y + dy - o0y) * kD0 + (2 * k1x + dx - o0x)];
        }
      if (l1x >= 2 && l1x < 2 + 2 * kT2 && l1y >= 2 && l1y < 2 + 2 * kT2)
        b1out[(int64_t)mode * N1 + g1] = bb;
    }
    sb1[tid] = bb;
    sd1[tid] = tv[4];
    sy1[tid] = inp1 ? omega * bb / tv[4] : 0.0;
  }
  __syncthreads();
  if (p1) {
    double v = 0.0;
    if (l1x >= 1 && l1x < kD1 - 1 && l1y >= 1 && l1y < kD1 - 1 && inp1) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += tv[t] * sy1[(l1y + t / 3 - 1) * kD1 + (l1x + t % 3 - 1)];
      v = sy1[tid] + omega * (sb1[tid] - ax) / sd1[tid];
    }
    sy2[tid] = v;
  }
  __syncthreads();
  if (p1) {
    double v = 0.0;
    if (l1x >= 2 && l1x < kD1 - 2 && l1y >= 2 && l1y < kD1 - 2 && inp1) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += tv[t] * sy2[(l1y + t / 3 - 1) * kD1 + (l1x + t % 3 - 1)];
      v = sb1[tid] - ax;
      if (l1x < kD1 - 3 && l1y < kD1 - 3) x2out1[(int64_t)mode * N1 + g1] = sy2[tid];
    }
    sr1[tid] = v;
  }
  __syncthreads();
  // level l+2: right-hand side of the tile's nodes
  if (tid < kT2 * kT2) {
    const int I = I0 + tid % kT2, J = J0 + tid / kT2;
    if (I <= m2 && J <= m2) {
      double acc = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const double wgt = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0);
          acc += wgt * sr1[(2 * J + dy - o1y) * kD1 + (2 * I + dx - o1x)];
        }
      b2out[(int64_t)mode * N2 + (int64_t)(J - 1) * m2 + (I - 1)] = acc;
    }
  }
}

template <int T2, int NT>
__global__ __launch_bounds__(NT) void vup2_kernel(
    const double* __restrict__ S0, const double* __restrict__ S1, int n0, int64_t N0, int64_t N1,
    int64_t N2, const int* bmap, const int* xmap, const double* __restrict__ bglob,
    const double* __restrict__ x2in0, const double* __restrict__ b1in,
    const double* __restrict__ x2in1, const double* __restrict__ xc2, int64_t xcslab,
    double* __restrict__ xout, double omega, EdgeFix ef) {
  using Gm = V2Geom<T2, NT>;
  constexpr int kT2 = Gm::kT2, kU0 = Gm::kU0, kU1 = Gm::kU1, kU2 = Gm::kU2, kV2Threads = NT;
  extern __shared__ double smem[];
  constexpr int A0 = kU0 * kU0, A1 = kU1 * kU1, A2 = kU2 * kU2;
  double* sb0 = smem;
  double* sd0 = sb0 + A0;
  double* sx3 = sd0 + A0;
  double* sx4 = sx3 + A0;
  double* sb1 = sx4 + A0;
  double* sd1 = sb1 + A1;
  double* sy3 = sd1 + A1;
  double* sy4 = sy3 + A1;
  double* sy5 = sy4 + A1;
  double* sc = sy5 + A1;
  const int mode = blockIdx.y, tid = threadIdx.x;
  const int m0 = n0 - 1, m1 = n0 / 2 - 1, n2 = n0 / 4, m2 = n2 - 1;
  const int tpr = (n2 + kT2 - 1) / kT2;
  const int tx = blockIdx.x % tpr, ty = blockIdx.x / tpr;
  const int I0 = 1 + tx * kT2, J0 = 1 + ty * kT2;
  const int o0x = 4 * I0 - 5, o0y = 4 * J0 - 5;          // level l index of local (0,0)
  const int o1x = 2 * I0 - 5, o1y = 2 * J0 - 5;          // level l+1
  const int o2x = I0 - 3, o2y = J0 - 3;                  // level l+2
  const double* b = bglob + (int64_t)(bmap ? bmap[mode] : mode) * N0;
  const double* x20 = x2in0 + (int64_t)mode * N0;
  const double* b1 = b1in + (int64_t)mode * N1;
  const double* x21 = x2in1 + (int64_t)mode * N1;
  const double* xc = xc2 + (int64_t)mode * N2;
  auto in0 = [&](int x, int y) { return x >= 1 && x <= m0 && y >= 1 && y <= m0; };
  auto in1 = [&](int x, int y) { return x >= 1 && x <= m1 && y >= 1 && y <= m1; };
  static_assert(A2 <= kV2Threads, "one coarse value per thread");
  // every global load at once: the coarse correction, level l+1's and level
  // l's right-hand sides, pre-smoothed values and stencil rows
  double cv = 0.0;
  {
    const int cx = o2x + tid % kU2, cy = o2y + tid / kU2;
    if (tid < A2 && cx >= 1 && cx <= m2 && cy >= 1 && cy <= m2) {
      const int64_t g = (int64_t)(cy - 1) * m2 + (cx - 1);
      cv = xc[g];
      if (xcslab) cv = (cv + xc[g + xcslab]) + (xc[g + 2 * xcslab] + xc[g + 3 * xcslab]);
    }
  }
  constexpr int kP1 = (A1 + kV2Threads - 1) / kV2Threads;
  constexpr int kP0 = (A0 + kV2Threads - 1) / kV2Threads;
  double tv[kP1][9], b1v[kP1], x1v[kP1];
  int64_t g1p[kP1];
#pragma unroll
  for (int p = 0; p < kP1; ++p) {
    const int e = tid + kV2Threads * p, kx = o1x + e % kU1, ky = o1y + e / kU1;
    const bool in = e < A1 && in1(kx, ky);
    g1p[p] = in ? (int64_t)(ky - 1) * m1 + (kx - 1) : -1;
    b1v[p] = in ? b1[g1p[p]] : 0.0;
    x1v[p] = in ? x21[g1p[p]] : 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) tv[p][t] = in ? S1[t * N1 + g1p[p]] : (t == 4 ? 1.0 : 0.0);
  }
  double sv[kP0][9], bv[kP0], xv[kP0];
  int64_t gp[kP0];
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, fx = o0x + e % kU0, fy = o0y + e / kU0;
    const bool in = e < A0 && in0(fx, fy);
    gp[p] = in ? (int64_t)(fy - 1) * m0 + (fx - 1) : -1;
    bv[p] = in ? b[gp[p]] : 0.0;
    if (in && ef.edge) bv[p] = edge_fixed(bv[p], ef, mode, fx, fy);
    xv[p] = in ? x20[gp[p]] : 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) sv[p][t] = in ? S0[t * N0 + gp[p]] : (t == 4 ? 1.0 : 0.0);
  }
  if (tid < A2) sc[tid] = cv;
  __syncthreads();
  // bilinear interpolation from a coarser level held in LDS (origin ocx, ocy)
  auto interp = [&](const double* c, int ext, int ocx, int ocy, int fx, int fy) {
    const int Ia = fx >> 1, Ib = (fx + 1) >> 1, Ja = fy >> 1, Jb = (fy + 1) >> 1;
    auto C = [&](int I, int J) { return c[(J - ocy) * ext + (I - ocx)]; };
    double pr;
    if (fx & 1) {
      if (fy & 1) pr = 0.25 * C(Ia, Ja) + 0.25 * C(Ib, Ja) + 0.25 * C(Ia, Jb) + 0.25 * C(Ib, Jb);
      else pr = 0.5 * C(Ia, Ja) + 0.5 * C(Ib, Ja);
    } else {
      if (fy & 1) pr = 0.5 * C(Ia, Ja) + 0.5 * C(Ia, Jb);
      else pr = C(Ia, Ja);
    }
    return pr;
  };
  // level l+1: prolong-add, then two post-smoothing sweeps
#pragma unroll
  for (int p = 0; p < kP1; ++p) {
    const int e = tid + kV2Threads * p;
    if (e >= A1) continue;
    const int kx = o1x + e % kU1, ky = o1y + e / kU1;
    sb1[e] = b1v[p];
    sd1[e] = tv[p][4];
    sy3[e] = g1p[p] >= 0 ? x1v[p] + interp(sc, kU2, o2x, o2y, kx, ky) : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kP1; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kU1, ly = e / kU1;
    if (e >= A1) continue;
    double v = 0.0;
    if (lx >= 1 && lx < kU1 - 1 && ly >= 1 && ly < kU1 - 1 && g1p[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += tv[p][t] * sy3[(ly + t / 3 - 1) * kU1 + (lx + t % 3 - 1)];
      v = sy3[e] + omega * (sb1[e] - ax) / sd1[e];
    }
    sy4[e] = v;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kP1; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kU1, ly = e / kU1;
    if (e >= A1) continue;
    double v = 0.0;
    if (lx >= 2 && lx < kU1 - 2 && ly >= 2 && ly < kU1 - 2 && g1p[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += tv[p][t] * sy4[(ly + t / 3 - 1) * kU1 + (lx + t % 3 - 1)];
      v = sy4[e] + omega * (sb1[e] - ax) / sd1[e];
    }
    sy5[e] = v;  // level l+1's correction (zero outside the domain)
  }
  __syncthreads();
  // level l: prolong-add from level l+1, then two post-smoothing sweeps
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p;
    if (e >= A0) continue;
    const int fx = o0x + e % kU0, fy = o0y + e / kU0;
    sb0[e] = bv[p];
    sd0[e] = sv[p][4];
    sx3[e] = gp[p] >= 0 ? xv[p] + interp(sy5, kU1, o1x, o1y, fx, fy) : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kU0, ly = e / kU0;
    if (e >= A0) continue;
    double v = 0.0;
    if (lx >= 1 && lx < kU0 - 1 && ly >= 1 && ly < kU0 - 1 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx3[(ly + t / 3 - 1) * kU0 + (lx + t % 3 - 1)];
      v = sx3[e] + omega * (sb0[e] - ax) / sd0[e];
    }
    sx4[e] = v;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kP0; ++p) {
    const int e = tid + kV2Threads * p, lx = e % kU0, ly = e / kU0;
    if (e >= A0) continue;
    if (lx >= 2 && lx < kU0 - 2 && ly >= 2 && ly < kU0 - 2 && gp[p] >= 0) {
      double ax = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) ax += sv[p][t] * sx4[(ly + t / 3 - 1) * kU0 + (lx + t % 3 - 1)];
      xout[(int64_t)(xmap ? xmap[mode] : mode) * N0 + gp[p]] = sx4[e] + omega * (sb0[e] - ax) / sd0[e];
    }
  }
}

// The two-level kernels pay off where a one-level launch is latency-bound:
// few workgroups, each waiting on its own chain of barriers.  The tile size
// follows the launch's size in 8 x 8 tiles (W8 workgroups): below 128, 4 x 4
// tiles (31^2 level-l nodes per 256-thread workgroup down, 20^2 up: four times
// the workgroups, shorter chains); below 512, 8 x 8 tiles (47^2 and 36^2, 512
// threads); from 512 on the one-level kernels, which compute no halo twice,
// are faster (measured at 128x128: W8 = 48, 96 / 160, 256 / 560).
namespace {
int64_t two_level_w8(const Level& L2, int modes) {
  const int t8 = (L2.n + 7) / 8;
  return (int64_t)t8 * t8 * modes;
}
}  // namespace

bool two_level_pays(const Level& L2, int modes) { return two_level_w8(L2, modes) < 512; }

void launch_vdown2(hipStream_t s, const Level& L0, const Level& L1, const Level& L2, int modes,
                   const double* b, double* x2_0, double* b1, double* x2_1, double* b2,
                   double omega, const int* bmap, const EdgeFix& ef) {
  if (L0.n % 4 || L1.n * 2 != L0.n || L2.n * 4 != L0.n)
    throw Error(SG_ERR_INTERNAL, "two-level V-cycle: grid sizes");
  if (two_level_w8(L2, modes) < 128) {
    const int tpr = (L2.n + 3) / 4;
    const size_t lds = V2Geom<4, 256>::down_lds();
    hipLaunchKernelGGL((vdown2_kernel<4, 256>), dim3(tpr * tpr, modes), dim3(256), lds, s, L0.S,
                       L1.S, L0.n, L0.N, L1.N, L2.N, bmap, b, x2_0, b1, x2_1, b2, omega, ef);
  } else {
    const int tpr = (L2.n + 7) / 8;
    const size_t lds = V2Geom<8, 512>::down_lds();
    hipLaunchKernelGGL((vdown2_kernel<8, 512>), dim3(tpr * tpr, modes), dim3(512), lds, s, L0.S,
                       L1.S, L0.n, L0.N, L1.N, L2.N, bmap, b, x2_0, b1, x2_1, b2, omega, ef);
  }
}

void launch_vup2(hipStream_t s, const Level& L0, const Level& L1, const Level& L2, int modes,
                 const double* b, const double* x2_0, const double* b1, const double* x2_1,
                 const double* xc2, int xc_slices, double* x, double omega, const int* bmap,
                 const int* xmap, const EdgeFix& ef) {
  if (L0.n % 4 || L1.n * 2 != L0.n || L2.n * 4 != L0.n)
    throw Error(SG_ERR_INTERNAL, "two-level V-cycle: grid sizes");
  if (xc_slices != 1 && xc_slices != kDenseSlices) throw Error(SG_ERR_INTERNAL, "vup2: slices");
  const int64_t xcslab = xc_slices == 1 ? 0 : (int64_t)modes * L2.N;
  if (two_level_w8(L2, modes) < 128) {
    const int tpr = (L2.n + 3) / 4;
    const size_t lds = V2Geom<4, 256>::up_lds();
    hipLaunchKernelGGL((vup2_kernel<4, 256>), dim3(tpr * tpr, modes), dim3(256), lds, s, L0.S,
                       L1.S, L0.n, L0.N, L1.N, L2.N, bmap, xmap, b, x2_0, b1, x2_1, xc2, xcslab,
                       x, omega, ef);
  } else {
    const int tpr = (L2.n + 7) / 8;
    const size_t lds = V2Geom<8, 512>::up_lds();
    hipLaunchKernelGGL((vup2_kernel<8, 512>), dim3(tpr * tpr, modes), dim3(512), lds, s, L0.S,
                       L1.S, L0.n, L0.N, L1.N, L2.N, bmap, xmap, b, x2_0, b1, x2_1, xc2, xcslab,
                       x, omega, ef);
  }
}

// bmap / xmap (device, may be null): mode t reads b from vector bmap[t] and
// writes x to vector xmap[t] of the full-length arrays (the field split's
// gather and scatter folded into the finest level)
void launch_vdown(hipStream_t s, const Level& Lf, const Level& Lc, int modes, const int* smode,
                  const double* b, double* x2, double* bc, double omega, const int* bmap,
                  const EdgeFix& ef) {
  const int tpr = (Lf.n / 2 + kTC - 1) / kTC;
  hipLaunchKernelGGL(vdown_kernel, dim3(tpr * tpr, modes), dim3(256), 0, s, Lf.S, Lf.n, Lf.N, Lc.N,
                     smode, bmap, b, x2, bc, omega, ef);
}

void launch_vup(hipStream_t s, const Level& Lf, const Level& Lc, int modes, const int* smode,
                const double* b, const double* x2, const double* xc, double* x, double omega,
                const int* bmap, const int* xmap, int xc_slices, const EdgeFix& ef) {
  if (xc_slices != 1 && xc_slices != kDenseSlices) throw Error(SG_ERR_INTERNAL, "vup: slices");
  const int tpr = (Lf.n / 2 + kTC - 1) / kTC;
  const int64_t xcslab = xc_slices == 1 ? 0 : (int64_t)modes * Lc.N;
  hipLaunchKernelGGL(vup_kernel, dim3(tpr * tpr, modes), dim3(256), 0, s, Lf.S, Lf.n, Lf.N, Lc.N,
                     smode, bmap, xmap, b, x2, xc, x, omega, xcslab, ef);
}

// ---- coarse levels in LDS, one workgroup per mode --------------------------
namespace {

__device__ __forceinline__ double lds_stencil(const double* S, int N, int m, int node,
                                              const double* x) {
  const int ix = node % m, iy = node / m;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int jx = ix + (t % 3) - 1, jy = iy + (t / 3) - 1;
    if (jx >= 0 && jx < m && jy >= 0 && jy < m) acc += S[t * N + node] * x[jy * m + jx];
  }
  return acc;
}

}  // namespace

// One mode of the LDS-resident coarse V-cycle; ends with a barrier.
__device__ __forceinline__ void vcoarse_mode(double* lds, int mode, const CoarseLevels& cl,
                                             const int* smode, const double* __restrict__ bglob,
                                             double* __restrict__ xglob, double omega) {
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  int off[kMaxCoarseLevels];
  int tot = 0;
#pragma unroll
  for (int l = 0; l < kMaxCoarseLevels; ++l) {
    off[l] = tot;
    if (l < cl.nl) tot += (int)cl.N[l];
  }
  double* S = lds;                 // 9 x tot
  double* B = S + 9 * tot;
  double* X = B + tot;
  double* T = X + tot;
  double* R = T + tot;
  // stencils of every coarse level and the right-hand side -> LDS as one flat
  // range, eight loads in flight per thread
  {
    const double* src[kMaxCoarseLevels];
#pragma unroll
    for (int l = 0; l < kMaxCoarseLevels; ++l)
      src[l] = l < cl.nl ? sel_stencil(cl.S[l], cl.N[l], smode, mode) : cl.S[0];
    const int N0 = (int)cl.N[0];
    const int tot9 = 9 * tot, all = tot9 + N0;
    for (int base = tid; base < all; base += nth * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(base + u * nth, all - 1);
        if (e >= tot9) {
          v[u] = bglob[(int64_t)mode * N0 + (e - tot9)];
        } else {
          const double* p = src[0];
          int o = 0;
#pragma unroll
          for (int l = 1; l < kMaxCoarseLevels; ++l)
            if (l < cl.nl && e >= 9 * off[l]) {
              p = src[l];
              o = 9 * off[l];
            }
          v[u] = p[e - o];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * nth;
        if (e < tot9) S[e] = v[u];
        else if (e < all) B[e - tot9] = v[u];
      }
    }
  }
  __syncthreads();
  // descend
  for (int l = 0; l < cl.nl; ++l) {
    const int N = (int)cl.N[l], m = cl.n[l] - 1;
    const double* Sl = S + 9 * off[l];
    double *b = B + off[l], *x = X + off[l], *t = T + off[l], *r = R + off[l];
    if (l == cl.nl - 1) {
      for (int e = tid; e < N; e += nth) x[e] = b[e] / Sl[4 * N + e];
      __syncthreads();
      break;
    }
    for (int e = tid; e < N; e += nth) t[e] = omega * b[e] / Sl[4 * N + e];
    __syncthreads();
    for (int e = tid; e < N; e += nth)
      x[e] = t[e] + omega * (b[e] - lds_stencil(Sl, N, m, e, t)) / Sl[4 * N + e];
    __syncthreads();
    for (int e = tid; e < N; e += nth) r[e] = b[e] - lds_stencil(Sl, N, m, e, x);
    __syncthreads();
    const int mc = cl.n[l + 1] - 1;
    double* bc = B + off[l + 1];
    for (int e = tid; e < mc * mc; e += nth) {
      const int I = e % mc + 1, J = e / mc + 1;
      double acc = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
          acc += (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * r[(2 * J + dy - 1) * m + (2 * I + dx - 1)];
      bc[e] = acc;
    }
    __syncthreads();
  }
  // ascend
  for (int l = cl.nl - 2; l >= 0; --l) {
    const int N = (int)cl.N[l], m = cl.n[l] - 1, mc = cl.n[l + 1] - 1;
    const double* Sl = S + 9 * off[l];
    double *b = B + off[l], *x = X + off[l], *t = T + off[l];
    const double* xc = X + off[l + 1];
    for (int e = tid; e < N; e += nth) {
      const int i = e % m + 1, j = e / m + 1;
      const int Ia = i >> 1, Ib = (i + 1) >> 1, Ja = j >> 1, Jb = (j + 1) >> 1;
      auto C = [&](int I, int J) {
        return (I >= 1 && I <= mc && J >= 1 && J <= mc) ? xc[(J - 1) * mc + (I - 1)] : 0.0;
      };
      double p;
      if (i & 1) {
        if (j & 1) p = 0.25 * C(Ia, Ja) + 0.25 * C(Ib, Ja) + 0.25 * C(Ia, Jb) + 0.25 * C(Ib, Jb);
        else p = 0.5 * C(Ia, Ja) + 0.5 * C(Ib, Ja);
      } else {
        if (j & 1) p = 0.5 * C(Ia, Ja) + 0.5 * C(Ia, Jb);
        else p = C(Ia, Ja);
      }
      x[e] += p;
    }
    __syncthreads();
    for (int e = tid; e < N; e += nth)
      t[e] = x[e] + omega * (b[e] - lds_stencil(Sl, N, m, e, x)) / Sl[4 * N + e];
    __syncthreads();
    for (int e = tid; e < N; e += nth)
      x[e] = t[e] + omega * (b[e] - lds_stencil(Sl, N, m, e, t)) / Sl[4 * N + e];
    __syncthreads();
  }
  {
    const int N = (int)cl.N[0];
    for (int e = tid; e < N; e += nth) xglob[(int64_t)mode * N + e] = X[e];
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void vcoarse_kernel(CoarseLevels cl, const int* smode,
                                                      const double* __restrict__ bglob,
                                                      double* __restrict__ xglob, double omega) {
  extern __shared__ double lds[];
  vcoarse_mode(lds, blockIdx.x, cl, smode, bglob, xglob, omega);
}

// ---------------------------------------------------------------------------
// Coarse part of the V-cycle as a dense operator.  From a level with
// n <= kDenseN down, one V(2,2) cycle with zero initial guess is a fixed linear
// map x = C b of the level's (n-1)^2 unknowns; C is built once by running the
// cycle's own kernels on unit vectors and then applied to a batch of modes as
// X = C B (C, B, X column-major, leading dimension N).  One workgroup per
// 16 x 16 output tile; the tile's 16 columns of B are staged in LDS; the four
// wavefronts split the inner index and their partial tiles are summed in a
// fixed order.
// ---------------------------------------------------------------------------
__global__ void unit_columns_kernel(int N, int j0, int m, double* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)N * m) return;
  const int k = (int)(gid / N), i = (int)(gid - (int64_t)k * N);
  out[gid] = (i == j0 + k) ? 1.0 : 0.0;
}

void launch_unit_columns(hipStream_t s, int N, int j0, int m, double* out) {
  hipLaunchKernelGGL(unit_columns_kernel, dim3(cdiv((int64_t)N * m, 256)), dim3(256), 0, s, N, j0,
                     m, out);
}

// One 512-thread workgroup per 16 x 16 output tile and slice of the inner
// index: the slice's rows of the tile's 16 columns of B (zero past N) are
// staged in LDS, each of the 8 wavefronts takes NB batches of 32 inner indices
// (the next batch of matrix loads in flight while one is used), and the 8
// partial tiles are summed in a fixed order.  With one slice (NB = 4, all
// kDenseK inner indices) the tile goes to X; with four (NB = 1) slice z writes
// its partial tile to X + z * xslab, and the four partial results are summed,
// in slice order, by the kernel that reads X.
template <int NB>
__global__ __launch_bounds__(512) void dense_coarse_kernel(int N, int m,
                                                           const double* __restrict__ C,
                                                           const double* __restrict__ B,
                                                           double* __restrict__ X, int64_t xslab,
                                                           const int* bmap, const int* xmap) {
  constexpr int D = 32;            // matrix loads per batch
  constexpr int KW = NB * D;       // inner indices per wavefront
  constexpr int KB = 8 * KW;       // inner indices per workgroup
  extern __shared__ double smem[];
  double* Bs = smem;               // [KB][16]
  double* red = smem + (size_t)KB * 16;  // [8][256]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r0 = blockIdx.x * 16, k0 = blockIdx.y * 16, ncol = min(16, m - k0);
  const int kbase = blockIdx.z * KB;
  const int r = lane & 15, cg = (lane >> 4) * 4;
  const double* Cr = C + min(r0 + r, N - 1);
  const int jw = kbase + wave * KW;
  double a[D], an[D];
#pragma unroll
  for (int u = 0; u < D; ++u) a[u] = Cr[(int64_t)min(jw + u, N - 1) * N];  // clamped
  {
    // thread t stages column t % 16, slice rows t / 16 + 32 s
    const int c = tid & 15, j0 = tid >> 4;
    const int bc = k0 + min(c, ncol - 1);
    const double* Bc = B + (int64_t)(bmap ? bmap[bc] : bc) * N;
    double v[KB / 32];
#pragma unroll
    for (int u = 0; u < KB / 32; ++u) v[u] = Bc[min(kbase + j0 + 32 * u, N - 1)];
#pragma unroll
    for (int u = 0; u < KB / 32; ++u) {
      const int j = j0 + 32 * u;
      Bs[j * 16 + c] = (c < ncol && kbase + j < N) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  // two accumulator sets (even / odd inner index): eight independent FMA chains
  double acc2[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  const double* Bw = Bs + (jw - kbase) * 16 + cg;
#pragma unroll
  for (int bt = 0; bt < NB; ++bt) {
    if (bt + 1 < NB) {
#pragma unroll
      for (int u = 0; u < D; ++u) an[u] = Cr[(int64_t)min(jw + (bt + 1) * D + u, N - 1) * N];
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const double2 b01 = *reinterpret_cast<const double2*>(Bw + (bt * D + u) * 16);
      const double2 b23 = *reinterpret_cast<const double2*>(Bw + (bt * D + u) * 16 + 2);
      double* ac = acc2[u & 1];
      ac[0] = fma(a[u], b01.x, ac[0]);
      ac[1] = fma(a[u], b01.y, ac[1]);
      ac[2] = fma(a[u], b23.x, ac[2]);
      ac[3] = fma(a[u], b23.y, ac[3]);
    }
    if (bt + 1 < NB) {
#pragma unroll
      for (int u = 0; u < D; ++u) a[u] = an[u];
    }
  }
  double acc[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = acc2[0][v] + acc2[1][v];
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave * 256 + v * 64 + lane] = acc[v];
  __syncthreads();
  if (wave == 0) {
    double* Xz = X + (int64_t)blockIdx.z * xslab;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double x = red[v * 64 + lane];
#pragma unroll
      for (int w = 1; w < 8; ++w) x += red[w * 256 + v * 64 + lane];
      const int c = cg + v;
      if (r0 + r < N && c < ncol) Xz[(int64_t)(xmap ? xmap[k0 + c] : k0 + c) * N + r0 + r] = x;
    }
  }
}

void launch_dense_coarse(hipStream_t s, int N, int m, const double* C, const double* B,
                         double* X, const int* bmap, const int* xmap, int slices) {
  if (N < 1 || N > kDenseK || m < 1) throw Error(SG_ERR_INTERNAL, "dense coarse operator: size");
  const int64_t xslab = (int64_t)m * N;
  if (slices == 1) {
    const size_t lds = 8 * ((size_t)kDenseK * 16 + 8 * 256);
    hipLaunchKernelGGL(dense_coarse_kernel<4>, dim3(cdiv(N, 16), cdiv(m, 16), 1), dim3(512), lds,
                       s, N, m, C, B, X, xslab, bmap, xmap);
  } else if (slices == kDenseSlices && !xmap) {
    const size_t lds = 8 * ((size_t)(kDenseK / kDenseSlices) * 16 + 8 * 256);
    hipLaunchKernelGGL(dense_coarse_kernel<1>, dim3(cdiv(N, 16), cdiv(m, 16), kDenseSlices),
                       dim3(512), lds, s, N, m, C, B, X, xslab, bmap, xmap);
  } else {
    throw Error(SG_ERR_INTERNAL, "dense coarse operator: slices");
  }
}

size_t vcoarse_lds_bytes(const CoarseLevels& cl) {
  size_t tot = 0;
  for (int l = 0; l < cl.nl; ++l) tot += cl.N[l];
  return 8 * 13 * tot;
}

void launch_vcoarse(hipStream_t s, const CoarseLevels& cl, int modes, const int* smode,
                    const double* b, double* x, double omega) {
  hipLaunchKernelGGL(vcoarse_kernel, dim3(modes), dim3(256), vcoarse_lds_bytes(cl), s, cl, smode,
                     b, x, omega);
}

// c[q] = sum over the (k, v) list of v * a_k(q): the coefficient of a diagonal
// block K_ii = sum_k [G_k]_{ii} A_k
__global__ void diag_coeff_kernel(int64_t Nq, int cnt, const int* __restrict__ ks,
                                  const double* __restrict__ vs, const double* __restrict__ a,
                                  double* __restrict__ c) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Nq) return;
  double acc = 0.0;
  for (int t = 0; t < cnt; ++t) acc += vs[t] * a[(int64_t)ks[t] * Nq + q];
  c[q] = acc;
}

void launch_diag_coeff(hipStream_t s, int n, int cnt, const int* ks, const double* vs,
                       const double* a, double* c) {
  const int64_t Nq = (int64_t)4 * n * n;
  hipLaunchKernelGGL(diag_coeff_kernel, dim3(cdiv(Nq, 256)), dim3(256), 0, s, Nq, cnt, ks, vs, a, c);
}

}  // namespace sg

// ===========================================================================
// Batched versions for many instances in one launch.  Every kernel runs one
// workgroup per entry of a table of (instance, local item) work items (each
// item's arithmetic is fixed, so results do not depend on scheduling), reads
// the instance's descriptor, and skips instances that are gated off (finished,
// or out of the current Arnoldi cycle).  A persistent form, fewer workgroups
// looping over the table, ran the shared tile code 1.5-2x slower: the loop's
// state stayed live across it and the compiler spilled scalar registers.  Per-instance
// solver state (the Arnoldi index j, the Givens rotations, the convergence
// flags) lives on the device, so one Arnoldi step of every instance is a fixed
// launch sequence that can be captured once in a HIP graph and replayed.
// ===========================================================================
namespace sg {

namespace {

}  // namespace

template <int RMAX>
__global__ __launch_bounds__(256) void bapply_kernel(const BInst* __restrict__ Is,
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
    // a copy, so the tile code reads the descriptor from registers, not memory
    RowSetDev rs = rowset == 0 ? I.full : I.part[rowset];
    rs.rows = gptr(rs.rows);
    rs.cols = gptr(rs.cols);
    rs.cpass = gptr(rs.cpass);
    rs.wrows = gptr(rs.wrows);
    rs.ptr = gptr(rs.ptr);
    rs.ent = gptr(rs.ent);
    apply_tile<RMAX>(smem, w.local, I.n, I.na, gptr(I.a), rs, bbuf(I, S, src), I.Nh,
                     rin >= 0 ? bbuf(I, S, rin) : nullptr, beta, sgn, bbuf(I, S, dst),
                     gptr(I.edge));
  }
}

void launch_bapply(hipStream_t s, int rmax, size_t lds, const BInst* I, const BState* st,
                   const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                   double beta, double sgn, int gate) {
  if (nitems <= 0) return;
  // one workgroup per item (the loop in the kernel is then a single pass): the
  // hardware schedules the tiles exactly as in a single-instance launch
  const int grid = nitems;
#define SG_BAPPLY(R)                                                                       \
  case R:                                                                                  \
    hipLaunchKernelGGL(bapply_kernel<R>, dim3(grid), dim3(256), lds, s, I, st, items, nitems, \
                       rowset, src, rin, dst, beta, sgn, gate);                            \
    break;
  switch (rmax) {
    SG_BAPPLY(1) SG_BAPPLY(2) SG_BAPPLY(4) SG_BAPPLY(8) SG_BAPPLY(16) SG_BAPPLY(32) SG_BAPPLY(64)
    default: throw Error(SG_ERR_INTERNAL, "batched apply: unsupported rows per wavefront");
  }
#undef SG_BAPPLY
}

// factored apply over (instance, tile) items of instances sharing one sub-batch size
template <int QB>
__global__ __launch_bounds__(256) void bfapply_kernel(const BInst* __restrict__ Is,
                                                      const BState* __restrict__ Ss,
                                                      const BItem* __restrict__ items, int nitems,
                                                      int rowset, int src, int rin, int dst,
                                                      double beta, double sgn, int gate) {
  // one workgroup per item (grid = nitems)
  extern __shared__ double smem[];
  if ((int)blockIdx.x >= nitems) return;
  const BItem w = items[blockIdx.x];
  const BInst& I = Is[w.inst];
  const BState& S = Ss[w.inst];
  if (gated(S, gate)) return;
  // a copy, so the tile code reads the descriptor from registers, not memory
  const FRowSetDev rs = rowset == 0 ? I.ffull : I.fpart[rowset];
  fapply_tile<QB>(smem, w.local, I.n, I.mu, I.amin, gptr(I.gq), rs, gptr(rs.blob),
                  bbuf(I, S, src), I.Nh, rin >= 0 ? bbuf(I, S, rin) : nullptr, beta, sgn,
                  bbuf(I, S, dst), gptr(I.edge));
}

void launch_bfapply(hipStream_t s, int qb, size_t lds, const BInst* I, const BState* st,
                    const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                    double beta, double sgn, int gate) {
  if (nitems <= 0) return;
  if (lds > 160 * 1024) throw Error(SG_ERR_INTERNAL, "batched factored apply: LDS");
  // one workgroup per item (the loop in the kernel is then a single pass): the
  // hardware schedules the tiles exactly as in a single-instance launch
  const int grid = nitems;
  switch (qb) {
#define SG_BFAPPLY(Q)                                                                          \
  case Q:                                                                                      \
    hipLaunchKernelGGL(bfapply_kernel<Q>, dim3(grid), dim3(256), lds, s, I, st, items, nitems, \
                       rowset, src, rin, dst, beta, sgn, gate);                                \
    break;
    SG_BFAPPLY(8) SG_BFAPPLY(16) SG_BFAPPLY(32) SG_BFAPPLY(64)
#undef SG_BFAPPLY
    default: throw Error(SG_ERR_INTERNAL, "batched factored apply: sub-batch size");
  }
}

// fixup items: local = chunk of kVecChunk fixup points of the row set
__global__ void bfixup_kernel(const BInst* __restrict__ Is, const BState* __restrict__ Ss,
                              const BItem* __restrict__ items, int nitems, int rowset, int dst,
                              double sgn, int gate) {
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) return;
    const RowSetDev& rs = rowset == 0 ? I.full : I.part[rowset];
    const int nt = I.n / kTileE;
    const int64_t total = (int64_t)rs.nrows * nt * nt * 7;
    const int64_t g0 = (int64_t)w.local * kVecChunk;
    for (int64_t g = g0 + threadIdx.x; g < std::min<int64_t>(total, g0 + kVecChunk); g += blockDim.x)
      apply_fixup_item(g, I.n, sgn, gptr(I.edge), bbuf(I, S, dst), I.Nh);
  }
}

void launch_bfixup(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                   int rowset, int dst, double sgn, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bfixup_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, rowset, dst, sgn, gate);
}

// V-cycle items: local = tile * m + mode on the instance's level `depth`
__global__ __launch_bounds__(256) void bvdown_kernel(const BInst* __restrict__ Is,
                                                     const BState* __restrict__ Ss,
                                                     const BItem* __restrict__ items, int nitems,
                                                     int depth, int split, int gate) {
  __shared__ VDownLds L;
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    if (gated(Ss[w.inst], gate)) return;
    const int m = I.split_m[split];
    const Level& Lf = I.L[depth];
    const Level& Lc = I.L[depth + 1];
    const double* b = gptr(depth == 0 ? I.fsT : I.mg_b[depth]);
    vdown_tile(L, w.local / m, w.local % m, gptr(Lf.S), Lf.n, Lf.N, Lc.N, nullptr, nullptr, b,
               gptr(I.mg_xa[depth]), gptr(I.mg_b[depth + 1]), 8.0 / 9.0);
  }
}

__global__ __launch_bounds__(256) void bvup_kernel(const BInst* __restrict__ Is,
                                                   const BState* __restrict__ Ss,
                                                   const BItem* __restrict__ items, int nitems,
                                                   int depth, int split, int gate) {
  __shared__ VUpLds L;
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    if (gated(Ss[w.inst], gate)) return;
    const int m = I.split_m[split];
    const Level& Lf = I.L[depth];
    const Level& Lc = I.L[depth + 1];
    const double* b = gptr(depth == 0 ? I.fsT : I.mg_b[depth]);
    double* x = gptr(depth == 0 ? I.fsX : I.mg_x[depth]);
    vup_tile(L, w.local / m, w.local % m, gptr(Lf.S), Lf.n, Lf.N, Lc.N, nullptr, nullptr, nullptr,
             b, gptr(I.mg_xa[depth]), gptr(I.mg_x[depth + 1]), x, 8.0 / 9.0);
  }
}

void launch_bvdown(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                   int depth, int split, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bvdown_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, depth, split, gate);
}

void launch_bvup(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                 int depth, int split, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bvup_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, depth, split, gate);
}

// coarse items: local = mode
__global__ __launch_bounds__(256) void bvcoarse_kernel(const BInst* __restrict__ Is,
                                                       const BState* __restrict__ Ss,
                                                       const BItem* __restrict__ items,
                                                       int nitems, int split, int gate) {
  extern __shared__ double lds[];
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    if (gated(Ss[w.inst], gate)) return;
    CoarseLevels cl{};
    cl.nl = I.nlev - I.nfine;
#pragma unroll
    for (int l = 0; l < kMaxCoarseLevels; ++l)
      if (l < cl.nl) {
        cl.n[l] = I.L[I.nfine + l].n;
        cl.N[l] = I.L[I.nfine + l].N;
        cl.S[l] = gptr(I.L[I.nfine + l].S);
      }
    const double* b = gptr(I.nfine == 0 ? I.fsT : I.mg_b[I.nfine]);
    double* x = gptr(I.nfine == 0 ? I.fsX : I.mg_x[I.nfine]);
    vcoarse_mode(lds, w.local, cl, nullptr, b, x, 8.0 / 9.0);
  }
}

void launch_bvcoarse(hipStream_t s, size_t lds, const BInst* I, const BState* st,
                     const BItem* items, int nitems, int split, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bvcoarse_kernel, dim3(nitems), dim3(256), lds, s, I, st,
                     items, nitems, split, gate);
}

// gather (scatter = 0): fsT[t][node] = buf[idx[t]][node]; scatter: buf[idx[t]] = fsX[t]
// items: local = chunk of kVecChunk elements of m * N_h
__global__ void bgather_kernel(const BInst* __restrict__ Is, const BState* __restrict__ Ss,
                               const BItem* __restrict__ items, int nitems, int split, int buf,
                               int scatter, int gate) {
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) return;
    const int64_t total = (int64_t)I.split_m[split] * I.Nh;
    const int* idx = gptr(I.split_idx[split]);
    double* full = bbuf(I, S, buf);
    const int64_t g0 = (int64_t)w.local * kVecChunk;
    for (int64_t g = g0 + threadIdx.x; g < std::min<int64_t>(total, g0 + kVecChunk); g += blockDim.x) {
      const int t = (int)(g / I.Nh);
      const int64_t f = (int64_t)idx[t] * I.Nh + (g - (int64_t)t * I.Nh);
      if (scatter) full[f] = gptr(I.fsX)[g];
      else gptr(I.fsT)[g] = full[f];
    }
  }
}

void launch_bgather(hipStream_t s, const BInst* I, const BState* st, const BItem* items,
                    int nitems, int split, int buf, int scatter, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bgather_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, split, buf, scatter, gate);
}

// vector operations on N_v-long vectors, items: local = chunk of kVecChunk
__global__ void bvec_kernel(const BInst* __restrict__ Is, const BState* __restrict__ Ss,
                            const BItem* __restrict__ items, int nitems, int op, int xb, int yb,
                            int ob, double a, double b, int gate) {
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) return;
    const int64_t g0 = (int64_t)w.local * kVecChunk;
    const int64_t g1 = std::min<int64_t>(I.Nv, g0 + kVecChunk);
    const int m = I.m;
    if (op == BV_AXPBY) {
      const double* x = bbuf(I, S, xb);
      const double* y = bbuf(I, S, yb);
      double* o = bbuf(I, S, ob);
      for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x)
        o[g] = (b == 0.0) ? (a == 0.0 ? 0.0 : a * x[g]) : a * x[g] + b * y[g];
    } else if (op == BV_UPDATE1 || op == BV_UPDATE2) {
      const double* h = gptr(I.hv + (op == BV_UPDATE1 ? 0 : m + 1));
      const double* V = gptr(I.V);
      double* wv = gptr(I.w);
      for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
        double acc = 0.0;
        for (int l = 0; l <= S.j; ++l) acc = fma(h[l], V[(int64_t)l * I.Nv + g], acc);
        wv[g] -= acc;
      }
    } else if (op == BV_SCALE_NEXT) {
      const double nn = sqrt(gptr(I.hv)[2 * m + 2]);
      double* v = gptr(I.V + (int64_t)(S.j + 1) * I.Nv);
      const double* wv = gptr(I.w);
      for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) v[g] = nn > 0.0 ? wv[g] / nn : 0.0;
    } else if (op == BV_COMBINE) {
      const double* y = gptr(I.y);
      const double* V = gptr(I.V);
      double* t = gptr(I.t);
      for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
        double acc = 0.0;
        for (int l = 0; l < S.kdone; ++l) acc = fma(y[l], V[(int64_t)l * I.Nv + g], acc);
        t[g] = acc;
      }
    } else {  // BV_START: V_0 = t / beta
      double* V = gptr(I.V);
      const double* t = gptr(I.t);
      for (int64_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) V[g] = t[g] / S.beta;
    }
  }
}

void launch_bvec(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                 int op, int x, int y, int out, double a, double b, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bvec_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, op, x, y, out, a, b, gate);
}

// dots: items (inst, block b < nblk); self_buf < 0: V_l . w for l <= j, else buf . buf
// partial[l * nblk + b] = item b's slice of V_l . x (x = w, l <= j), or of x . x
// for a named buffer.  The basis is taken 16 vectors at a time: for each
// element of the slice the 16 loads are in flight together, and the 16 sums
// are reduced once per chunk (wavefront butterfly, then the four wavefronts).
__global__ __launch_bounds__(256) void bmultidot_kernel(const BInst* __restrict__ Is,
                                                        const BState* __restrict__ Ss,
                                                        const BItem* __restrict__ items,
                                                        int nitems, int self_buf, int gate) {
  constexpr int C = 16;
  __shared__ double red[4 * 64];
  // one workgroup per item (grid = nitems)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    const BItem w = items[it];
    const BInst& I = Is[w.inst];
    const BState& S = Ss[w.inst];
    if (gated(S, gate)) return;
    const int nblk = I.nblk;
    const int64_t per = (I.Nv + nblk - 1) / nblk;
    const int64_t lo = (int64_t)w.local * per;
    const int64_t hi = std::min<int64_t>(I.Nv, lo + per);
    const double* x = self_buf >= 0 ? bbuf(I, S, self_buf) : gptr(I.w);
    const double* Vb = self_buf >= 0 ? x : gptr(I.V);
    const int nv = self_buf >= 0 ? 1 : S.j + 1;
    for (int l0 = 0; l0 < nv; l0 += C) {
      const int cnt = min(C, nv - l0);
      double acc[C];
#pragma unroll
      for (int l = 0; l < C; ++l) acc[l] = 0.0;
      for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double xi = x[i];
        double v[C];
#pragma unroll
        for (int l = 0; l < C; ++l) v[l] = l < cnt ? Vb[(int64_t)(l0 + l) * I.Nv + i] : 0.0;
#pragma unroll
        for (int l = 0; l < C; ++l) acc[l] = fma(v[l], xi, acc[l]);
      }
      wave_sums<C>(acc, red + 64 * (threadIdx.x >> 6));
      __syncthreads();
      if (threadIdx.x < cnt) {
        const int l = threadIdx.x;
        gptr(I.partial)[(int64_t)(l0 + l) * nblk + w.local] =
            (red[l] + red[64 + l]) + (red[128 + l] + red[192 + l]);
      }
      __syncthreads();  // red is reused
    }
  }
}

void launch_bmultidot(hipStream_t s, const BInst* I, const BState* st, const BItem* items,
                      int nitems, int self_buf, int gate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(bmultidot_kernel, dim3(nitems), dim3(256), 0, s, I, st, items,
                     nitems, self_buf, gate);
}

// which: 0 -> h1[0..j], 1 -> h2[0..j], 2 -> nrm (one value); one workgroup per instance
__global__ void breduce_kernel(const BInst* __restrict__ Is, const BState* __restrict__ Ss,
                               int which, int gate) {
  const BInst& I = Is[blockIdx.x];
  const BState& S = Ss[blockIdx.x];
  if (gated(S, gate)) return;
  const int m = I.m;
  const int nv = which == 2 ? 1 : S.j + 1;
  double* out = gptr(I.hv + (which == 0 ? 0 : which == 1 ? m + 1 : 2 * m + 2));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int l = wave; l < nv; l += blockDim.x / 64) {
    double acc = 0.0;
    for (int b = lane; b < I.nblk; b += 64) acc += gptr(I.partial)[(int64_t)l * I.nblk + b];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) out[l] = acc;
  }
}

void launch_breduce(hipStream_t s, const BInst* I, const BState* st, int count, int which,
                    int gate) {
  hipLaunchKernelGGL(breduce_kernel, dim3(count), dim3(256), 0, s, I, st, which, gate);
}

// Hessenberg column, Givens rotations and the residual estimate of step j
__global__ void bgivens_kernel(const BInst* __restrict__ Is, BState* __restrict__ Ss, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const BInst& I = Is[k];
  BState& S = Ss[k];
  if (!S.active) return;
  const int m = I.m, j = S.j;
  double* H = I.H;  // (m + 1) x m, row-major
  for (int i = 0; i <= j; ++i) H[i * m + j] = I.hv[i] + I.hv[m + 1 + i];
  H[(j + 1) * m + j] = sqrt(I.hv[2 * m + 2]);
  if (!isfinite(H[(j + 1) * m + j])) {
    S.status = SG_BREAKDOWN;
    S.kdone = j;
    S.active = 0;
    return;
  }
  for (int i = 0; i < j; ++i) {
    const double t = I.cs[i] * H[i * m + j] + I.sn[i] * H[(i + 1) * m + j];
    H[(i + 1) * m + j] = -I.sn[i] * H[i * m + j] + I.cs[i] * H[(i + 1) * m + j];
    H[i * m + j] = t;
  }
  const double a = H[j * m + j], b = H[(j + 1) * m + j];
  double c = 1.0, sn = 0.0;
  if (b != 0.0) {
    const double r = hypot(a, b);
    c = a / r;
    sn = b / r;
  }
  I.cs[j] = c;
  I.sn[j] = sn;
  H[j * m + j] = c * a + sn * b;
  H[(j + 1) * m + j] = 0.0;
  I.g[j + 1] = -sn * I.g[j];
  I.g[j] = c * I.g[j];
  S.it += 1;
  S.est = fabs(I.g[j + 1]);
  S.kdone = j + 1;
  S.j = j + 1;
  if (H[j * m + j] == 0.0) {
    S.status = SG_BREAKDOWN;
    S.kdone = j;
    S.active = 0;
  } else if (S.est <= S.target || S.it >= S.max_it || j + 1 == m) {
    S.active = 0;
  }
}

void launch_bgivens(hipStream_t s, const BInst* I, BState* st, int count) {
  hipLaunchKernelGGL(bgivens_kernel, dim3((count + 63) / 64), dim3(64), 0, s, I, st, count);
}

// back substitution H y = g over the cycle's kdone columns
__global__ void bsolve_kernel(const BInst* __restrict__ Is, const BState* __restrict__ Ss,
                              int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const BInst& I = Is[k];
  const BState& S = Ss[k];
  if (S.done) return;
  const int m = I.m;
  for (int i = S.kdone - 1; i >= 0; --i) {
    double acc = I.g[i];
    for (int l = i + 1; l < S.kdone; ++l) acc -= I.H[i * m + l] * I.y[l];
    I.y[i] = acc / I.H[i * m + i];
  }
}

void launch_bsolve(hipStream_t s, const BInst* I, const BState* st, int count) {
  hipLaunchKernelGGL(bsolve_kernel, dim3((count + 63) / 64), dim3(64), 0, s, I, st, count);
}

// cycle start: beta = ||t|| (norm squared in hv[2m+2]); finish or reset the cycle
__global__ void binit_kernel(const BInst* __restrict__ Is, BState* __restrict__ Ss, int count,
                             int first, double tol) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const BInst& I = Is[k];
  BState& S = Ss[k];
  if (S.done) return;
  const int m = I.m;
  const double beta = sqrt(I.hv[2 * m + 2]);
  if (first) {
    S.nF = beta;
    S.target = tol * beta;
    S.it = 0;
    S.restarts = 0;
    S.status = SG_NOT_CONVERGED;
  } else {
    S.restarts += 1;
  }
  S.beta = beta;
  S.kdone = 0;
  S.j = 0;
  const bool broke = S.status == SG_BREAKDOWN;
  if (S.nF == 0.0 || beta <= S.target) {
    S.status = SG_CONVERGED;
    S.done = 1;
    S.active = 0;
  } else if (!isfinite(beta) || broke || S.it >= S.max_it) {
    S.status = (!isfinite(beta) || broke) ? SG_BREAKDOWN : SG_NOT_CONVERGED;
    S.done = 1;
    S.active = 0;
  } else {
    for (int i = 0; i <= m; ++i) I.g[i] = 0.0;
    I.g[0] = beta;
    S.active = 1;
  }
}

void launch_binit(hipStream_t s, const BInst* I, BState* st, int count, int first, double tol) {
  hipLaunchKernelGGL(binit_kernel, dim3((count + 63) / 64), dim3(64), 0, s, I, st, count, first, tol);
}

}  // namespace sg
