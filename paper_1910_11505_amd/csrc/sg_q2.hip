// HIP kernels (gfx950) of the SG operator apply on biquadratic (Q2) elements
// (Sec. 2.2; eq. A_q with 3 x 3 Gauss points per element, the coefficient
// of block (i, j) taken through the Hermite translation factorisation
// sum_k a_k(x) [G_k]_{ij} = a_min delta_ij + exp(mu + |g(x)|^2 / 2) (T T^T)_{ij},
// exact when q >= 2p).  Four passes, each one thread per output value, all
// HBM-streaming (no atomics, every sum in a fixed order):
//  1. gradients of every mode at every Gauss point of its element;
//  2. per mode and Gauss point, y_beta = sum_alpha' T_{alpha' beta} grad_alpha';
//  3. per mode and Gauss point, flux_alpha = a_min grad_alpha
//       + exp(mu + |g|^2/2) sum_beta T_{alpha beta} y_beta, written over the
//     gradients;
//  4. per element and mode, in four colours of elements that share no node,
//     the weighted sums of grad phi_node . flux over the element's Gauss
//     points, added to the output (zeroed first).
// Index layout is described in sg_q2.h.
#include <hip/hip_runtime.h>

#include "sg_internal.h"
#include "sg_q2.h"

namespace sg {

namespace {

constexpr int kQ2Threads = 256;

// 3-point Gauss-Legendre on [0, 1]: 1/2 -+ sqrt(3/5)/2, weights 5/18, 8/18, 5/18
__device__ __forceinline__ double q2_pt(int i) {
  return i == 0 ? 0.11270166537925831 : i == 1 ? 0.5 : 0.88729833462074169;
}
__device__ __forceinline__ double q2_wt(int i) { return i == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }
// quadratic Lagrange polynomials through 0, 1/2, 1 and their derivatives
__device__ __forceinline__ double lag(int a, double s) {
  return a == 0 ? 2.0 * (s - 0.5) * (s - 1.0) : a == 1 ? 4.0 * s * (1.0 - s) : 2.0 * s * (s - 0.5);
}
__device__ __forceinline__ double dlag(int a, double s) {
  return a == 0 ? 4.0 * s - 3.0 : a == 1 ? 4.0 - 8.0 * s : 4.0 * s - 1.0;
}

// pass 1: thread (mode i, element e); the 9 nodal values of the element
// (zero on the Dirichlet boundary), gradients at its 9 points
__global__ __launch_bounds__(kQ2Threads) void q2_grad_kernel(int n2, int P,
                                                             const double* __restrict__ U,
                                                             double* __restrict__ grad) {
  const int64_t E = (int64_t)n2 * n2, Nq = 9 * E;
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid >= (int64_t)P * E) return;
  const int i = (int)(gid / E);
  const int64_t e = gid - (int64_t)i * E;
  const int ey = (int)(e / n2), ex = (int)(e - (int64_t)ey * n2);
  const int m = 2 * n2 - 1;
  const int64_t Nh = (int64_t)m * m;
  const double* Ui = U + (int64_t)i * Nh;
  double u[3][3];
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int X = 2 * ex + ax, Y = 2 * ey + ay;
      const bool in = X >= 1 && X <= m && Y >= 1 && Y <= m;
      u[ay][ax] = in ? Ui[(int64_t)(Y - 1) * m + (X - 1)] : 0.0;
    }
  double* gx = grad + (int64_t)(2 * i) * Nq + e;
  double* gy = grad + (int64_t)(2 * i + 1) * Nq + e;
#pragma unroll
  for (int qy = 0; qy < 3; ++qy)
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
      const double sx = q2_pt(qx), sy = q2_pt(qy);
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          vx += dlag(ax, sx) * lag(ay, sy) * u[ay][ax];
          vy += lag(ax, sx) * dlag(ay, sy) * u[ay][ax];
        }
      gx[(3 * qy + qx) * E] = vx;
      gy[(3 * qy + qx) * E] = vy;
    }
}

// g^(packed exponents), 4 bits per KL variable; variables past the highest
// nonzero exponent are skipped (code runs out)
__device__ __forceinline__ double q2_mono(const double (&g)[kQ2MaxM], uint64_t code) {
  double v = 1.0;
#pragma unroll
  for (int k = 0; k < kQ2MaxM; ++k) {
    if (code == 0) break;
    const int ek = (int)(code & 15u);
    code >>= 4;
    for (int t = 0; t < ek; ++t) v *= g[k];
  }
  return v;
}

// the KL values of Gauss point q (zero past M)
__device__ __forceinline__ void q2_point(const double* __restrict__ g, int64_t Nq, int M,
                                         int64_t q, double (&gv)[kQ2MaxM]) {
#pragma unroll
  for (int k = 0; k < kQ2MaxM; ++k) gv[k] = k < M ? g[(int64_t)k * Nq + q] : 0.0;
}

// pass 2: thread (mode beta, Gauss point q), y_beta = sum_alpha T_{alpha beta} grad_alpha
// (one thread per output keeps many independent loads in flight; consecutive
// threads take consecutive points of one mode, so a wavefront's table walk
// is uniform)
__global__ __launch_bounds__(kQ2Threads) void q2_ty_kernel(int64_t Nq, int M, int P,
                                                           const double* __restrict__ g, Q2TDev T,
                                                           const double* __restrict__ grad,
                                                           double* __restrict__ y) {
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid >= (int64_t)P * Nq) return;
  const int b = (int)(gid / Nq);
  const int64_t q = gid - (int64_t)b * Nq;
  double gv[kQ2MaxM];
  q2_point(g, Nq, M, q, gv);
  double yx = 0.0, yy = 0.0;
  for (int t = T.ptr1[b]; t < T.ptr1[b + 1]; ++t) {
    const int a = T.idx1[t];
    const double tv = T.c1[t] * q2_mono(gv, T.e1[t]);
    yx += tv * grad[(int64_t)(2 * a) * Nq + q];
    yy += tv * grad[(int64_t)(2 * a + 1) * Nq + q];
  }
  y[(int64_t)(2 * b) * Nq + q] = yx;
  y[(int64_t)(2 * b + 1) * Nq + q] = yy;
}

// pass 3: thread (mode alpha, Gauss point q),
// flux_alpha = a_min grad_alpha + exp(mu + |g|^2/2) sum_beta T_{alpha beta} y_beta,
// written over grad_alpha (read by this thread only)
__global__ __launch_bounds__(kQ2Threads) void q2_tflux_kernel(int64_t Nq, int M, int P, double mu,
                                                              double a_min,
                                                              const double* __restrict__ g,
                                                              Q2TDev T, double* __restrict__ grad,
                                                              const double* __restrict__ y) {
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid >= (int64_t)P * Nq) return;
  const int a = (int)(gid / Nq);
  const int64_t q = gid - (int64_t)a * Nq;
  double gv[kQ2MaxM];
  q2_point(g, Nq, M, q, gv);
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < kQ2MaxM; ++k) g2 += gv[k] * gv[k];
  const double sc = exp(mu + 0.5 * g2);
  double fx = 0.0, fy = 0.0;
  for (int t = T.ptr2[a]; t < T.ptr2[a + 1]; ++t) {
    const int b = T.idx2[t];
    const double tv = T.c2[t] * q2_mono(gv, T.e2[t]);
    fx += tv * y[(int64_t)(2 * b) * Nq + q];
    fy += tv * y[(int64_t)(2 * b + 1) * Nq + q];
  }
  double* px = grad + (int64_t)(2 * a) * Nq + q;
  double* py = grad + (int64_t)(2 * a + 1) * Nq + q;
  *px = a_min * *px + sc * fx;
  *py = a_min * *py + sc * fy;
}

// pass 4, in four colours: thread (mode i, element of colour (ex & 1) + 2 (ey & 1));
// the element's 9 node sums from its 9 Gauss points are added to W (zeroed
// first).  Two elements of one colour are two element rows or columns apart
// and share no node, so a colour's threads never touch the same entry; each
// entry receives its elements' sums in colour order.  Each flux value is
// read once.
__global__ __launch_bounds__(kQ2Threads) void q2_scatter_kernel(int n2, int P, int colour,
                                                                const double* __restrict__ flux,
                                                                double* __restrict__ W) {
  const int m = 2 * n2 - 1;
  const int h2 = n2 / 2;  // elements of one colour per row (n2 is even)
  const int64_t Ec = (int64_t)h2 * h2, E = (int64_t)n2 * n2, Nq = 9 * E;
  const int64_t Nh = (int64_t)m * m;
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid >= (int64_t)P * Ec) return;
  const int i = (int)(gid / Ec);
  const int64_t k = gid - (int64_t)i * Ec;
  const int ey = 2 * (int)(k / h2) + (colour >> 1), ex = 2 * (int)(k % h2) + (colour & 1);
  const int64_t el = (int64_t)ey * n2 + ex;
  const double* fx = flux + (int64_t)(2 * i) * Nq + el;
  const double* fy = flux + (int64_t)(2 * i + 1) * Nq + el;
  double fxq[9], fyq[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    fxq[q] = fx[q * E];
    fyq[q] = fy[q * E];
  }
  double* Wi = W + (int64_t)i * Nh;
#pragma unroll
  for (int ay = 0; ay < 3; ++ay)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int X = 2 * ex + ax, Y = 2 * ey + ay;
      if (X < 1 || X > m || Y < 1 || Y > m) continue;
      double acc = 0.0;
#pragma unroll
      for (int qy = 0; qy < 3; ++qy)
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
          const double sx = q2_pt(qx), sy = q2_pt(qy);
          const double w = q2_wt(qx) * q2_wt(qy);
          acc += w * (dlag(ax, sx) * lag(ay, sy) * fxq[3 * qy + qx] +
                      lag(ax, sx) * dlag(ay, sy) * fyq[3 * qy + qx]);
        }
      Wi[(int64_t)(Y - 1) * m + (X - 1)] += acc;
    }
}

__global__ __launch_bounds__(kQ2Threads) void q2_zero_kernel(double* __restrict__ W, int64_t n) {
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid < n) W[gid] = 0.0;
}

// F(node) for mode 0: sum over the node's elements of h^2 (M1 (x) M1)_{a b} f_b,
// M1 = [[4, 2, -1], [2, 16, 2], [-1, 2, 4]] / 30 (exact Q2 mass)
__device__ __forceinline__ double mass1(int a, int b) {
  const int s = a + b;
  if (a == 1 && b == 1) return 16.0 / 30.0;
  if (s == 1 || s == 3) return 2.0 / 30.0;
  if (a == b) return 4.0 / 30.0;
  return -1.0 / 30.0;  // (0, 2) and (2, 0)
}

__global__ __launch_bounds__(kQ2Threads) void q2_rhs_kernel(int n2, int P,
                                                            const double* __restrict__ f,
                                                            double* __restrict__ F) {
  const int m = 2 * n2 - 1, mf = 2 * n2 + 1;
  const int64_t Nh = (int64_t)m * m;
  const int64_t gid = (int64_t)blockIdx.x * kQ2Threads + threadIdx.x;
  if (gid >= (int64_t)P * Nh) return;
  if (gid >= Nh) {
    F[gid] = 0.0;
    return;
  }
  const int Y = (int)(gid / m) + 1, X = (int)(gid - (int64_t)(Y - 1) * m) + 1;
  const int nx = (X & 1) ? 1 : 2, ny = (Y & 1) ? 1 : 2;
  const int ex0 = (X & 1) ? (X - 1) / 2 : X / 2 - 1, ax0 = (X & 1) ? 1 : 2;
  const int ey0 = (Y & 1) ? (Y - 1) / 2 : Y / 2 - 1, ay0 = (Y & 1) ? 1 : 2;
  const double h = 1.0 / n2;
  double acc = 0.0;
  for (int jy = 0; jy < ny; ++jy) {
    const int ey = ey0 + jy, ay = jy ? 0 : ay0;
    for (int jx = 0; jx < nx; ++jx) {
      const int ex = ex0 + jx, ax = jx ? 0 : ax0;
      for (int by = 0; by < 3; ++by)
        for (int bx = 0; bx < 3; ++bx)
          acc += mass1(ay, by) * mass1(ax, bx) * f[(int64_t)(2 * ey + by) * mf + 2 * ex + bx];
    }
  }
  F[gid] = h * h * acc;
}

inline unsigned q2_blocks(int64_t work) {
  return (unsigned)((work + kQ2Threads - 1) / kQ2Threads);
}

}  // namespace

void launch_q2_apply(hipStream_t s, int n2, int M, int P, double mu, double a_min,
                     const double* g, const Q2TDev& T, const double* U, double* W, double* grad,
                     double* y) {
  const int64_t E = (int64_t)n2 * n2, Nq = 9 * E, Nh = (int64_t)(2 * n2 - 1) * (2 * n2 - 1);
  hipLaunchKernelGGL(q2_grad_kernel, dim3(q2_blocks(P * E)), dim3(kQ2Threads), 0, s, n2, P, U,
                     grad);
  hipLaunchKernelGGL(q2_ty_kernel, dim3(q2_blocks(P * Nq)), dim3(kQ2Threads), 0, s, Nq, M, P, g,
                     T, grad, y);
  hipLaunchKernelGGL(q2_tflux_kernel, dim3(q2_blocks(P * Nq)), dim3(kQ2Threads), 0, s, Nq, M, P,
                     mu, a_min, g, T, grad, y);
  hipLaunchKernelGGL(q2_zero_kernel, dim3(q2_blocks(P * Nh)), dim3(kQ2Threads), 0, s, W, P * Nh);
  const int64_t Ec = (int64_t)(n2 / 2) * (n2 / 2);
  for (int colour = 0; colour < 4; ++colour)
    hipLaunchKernelGGL(q2_scatter_kernel, dim3(q2_blocks(P * Ec)), dim3(kQ2Threads), 0, s, n2, P,
                       colour, grad, W);
}

void launch_q2_rhs(hipStream_t s, int n2, int P, const double* f, double* F) {
  const int64_t Nh = (int64_t)(2 * n2 - 1) * (2 * n2 - 1);
  hipLaunchKernelGGL(q2_rhs_kernel, dim3(q2_blocks(P * Nh)), dim3(kQ2Threads), 0, s, n2, P, f, F);
}

}  // namespace sg
