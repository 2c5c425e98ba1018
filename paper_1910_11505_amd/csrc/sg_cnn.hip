// Mode-channel CNN of the learned preconditioner stage (gfx950 HIP).
//
// The network maps a residual field (P stochastic modes on the n x n pixel
// grid of interior nodes, pixel (x, y) = node (x+1, y+1), the last row and
// column zero, plus a constant sigma channel) to an approximate error field.
// Nine 3x3 'same' convolutions over four resolution levels (average pooling
// down, nearest upsampling plus a skip tensor up), ReLU after all but the
// last layer.  Activations are NHWC bfloat16, weights bfloat16 copies of FP32
// master weights, every convolution an implicit GEMM on the 16x16x32 BF16
// matrix cores with FP32 accumulation.  Backward: data gradients reuse the
// forward kernel with flipped, transposed weights; weight gradients are an
// MFMA reduction over pixels with fixed-order split-K partial sums.  Adam
// updates the FP32 master weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sg_internal.h"
#include "sg_learned.h"

namespace sg {

namespace {

typedef unsigned short bf16_t;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline bf16_t f2bf(float f) {
  unsigned u = __builtin_bit_cast(unsigned, f);
  u = u + 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t b) {
  return __builtin_bit_cast(float, ((unsigned)b) << 16);
}

inline int cdivl(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Target scale kappa = 2 pi^2: the smallest eigenvalue of the unit-square
// Laplacian, so that the smoothest error of a unit residual maps to O(1).
constexpr double kTargetScale = 19.739208802178716;

__device__ __forceinline__ f32x4 mfma32(short8 a, short8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

}  // namespace

// ---------------------------------------------------------------------------
// 3x3 convolution, implicit GEMM.  One workgroup = 64 PT consecutive pixels of
// the batch (four wavefronts of PT tiles of 16), all output channels.  Per tap
// and 32 input channels: B = 32 channels x 16 output channels (one 16-byte
// weight load per lane and output block, shared by the wavefront's PT tiles),
// A = 16 pixels x 32 channels per tile (one 16-byte load per lane).  Zero
// padding at the image border.  Every tile's accumulators see the same
// products in the same order for any PT.
//   MODE 0: + bias, ReLU, bf16 out;  1: + bias, fp32 out;  2: fp32 out.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int MODE, int PT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const bf16_t* __restrict__ X,
                                                       const bf16_t* __restrict__ W,
                                                       const float* __restrict__ bias,
                                                       void* __restrict__ Yv, int S, int npix) {
  // pixels are numbered over the whole batch (gp = b * S * S + y * S + x), so
  // coarse levels with fewer than 64 pixels per image still fill the tiles
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int SS = S * S;
  const int row = lane & 15, kg = lane >> 4;
  const int wbase = blockIdx.x * (64 * PT) + wave * (16 * PT);
  constexpr int NB = COUT / 16;
  f32x4 acc[PT][NB];
  const bf16_t* Xb[PT];
  int py[PT], px[PT];
  bool valid[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[t][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int gp = wbase + 16 * t + row;
    valid[t] = gp < npix;
    const int b = valid[t] ? gp / SS : 0;
    const int p = gp - b * SS;
    py[t] = p / S;
    px[t] = p - py[t] * S;
    Xb[t] = X + (size_t)b * SS * CIN;
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
    for (int cb = 0; cb < CIN / 32; ++cb) {
      short8 w[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        w[nb] = *reinterpret_cast<const short8*>(
            W + (size_t)(tap * COUT + nb * 16 + row) * CIN + cb * 32 + kg * 8);
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int qx = px[t] + tap % 3 - 1, qy = py[t] + tap / 3 - 1;
        const bool in = valid[t] && (unsigned)qx < (unsigned)S && (unsigned)qy < (unsigned)S;
        short8 a = short8{0, 0, 0, 0, 0, 0, 0, 0};
        if (in) a = *reinterpret_cast<const short8*>(Xb[t] + (size_t)(qy * S + qx) * CIN + kg * 8 + cb * 32);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[t][nb] = mfma32(a, w[nb], acc[t][nb]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < PT; ++t) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pix = wbase + 16 * t + kg * 4 + i;
        if (pix >= npix) continue;
        const int co = nb * 16 + row;
        float v = acc[t][nb][i];
        if (MODE < 2) v += bias[co];
        const size_t o = (size_t)pix * COUT + co;
        if (MODE == 0) reinterpret_cast<bf16_t*>(Yv)[o] = f2bf(fmaxf(v, 0.f));
        else reinterpret_cast<float*>(Yv)[o] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient dW[tap][co][ci] = sum over pixels of G[p][co] X[p + off][ci]:
// one workgroup per (pixel chunk, tap); 32-pixel slabs of G and of the shifted
// X are staged in LDS and contracted on the matrix cores; each workgroup writes
// its partial sum, reduced afterwards in chunk order.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_bwdw_kernel(const bf16_t* __restrict__ X,
                                                        const bf16_t* __restrict__ G,
                                                        float* __restrict__ partial, int S,
                                                        int chunk, int npix) {
  constexpr int LG = COUT + 8, LX = CIN + 8;  // padded LDS rows (bank spread)
  __shared__ __attribute__((aligned(16))) bf16_t sG[32 * LG];
  __shared__ __attribute__((aligned(16))) bf16_t sX[32 * LX];
  const int c = blockIdx.x, tap = blockIdx.y;
  const int dx = tap % 3 - 1, dy = tap / 3 - 1;
  const int SS = S * S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kg = lane >> 4;
  constexpr int NCI = CIN / 16, T = (COUT / 16) * NCI, TPW = (T + 3) / 4;
  f32x4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int k_begin = c * chunk, k_end = min(npix, k_begin + chunk);
  for (int k0 = k_begin; k0 < k_end; k0 += 32) {
    // stage 32 pixel rows of G (COUT) and of the shifted X (CIN) as 16-byte vectors
    for (int e = threadIdx.x; e < 32 * (COUT / 8); e += 256) {
      const int r = e / (COUT / 8), v8 = e % (COUT / 8);
      short8 v = short8{0, 0, 0, 0, 0, 0, 0, 0};
      if (k0 + r < k_end) v = *reinterpret_cast<const short8*>(G + (size_t)(k0 + r) * COUT + v8 * 8);
      *reinterpret_cast<short8*>(&sG[r * LG + v8 * 8]) = v;
    }
    for (int e = threadIdx.x; e < 32 * (CIN / 8); e += 256) {
      const int r = e / (CIN / 8), v8 = e % (CIN / 8);
      const int gp = k0 + r;
      const int bimg = gp / SS, pp = gp - bimg * SS;
      const int py = pp / S, px = pp - py * S;
      const int qx = px + dx, qy = py + dy;
      short8 v = short8{0, 0, 0, 0, 0, 0, 0, 0};
      if (gp < k_end && (unsigned)qx < (unsigned)S && (unsigned)qy < (unsigned)S)
        v = *reinterpret_cast<const short8*>(X + ((size_t)bimg * SS + qy * S + qx) * CIN + v8 * 8);
      *reinterpret_cast<short8*>(&sX[r * LX + v8 * 8]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = wave + 4 * tt;
      if (t < T) {
        const int mb = t / NCI, nb = t % NCI;
        short8 a, bb;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          a[i] = (short)sG[(kg * 8 + i) * LG + mb * 16 + row];
          bb[i] = (short)sX[(kg * 8 + i) * LX + nb * 16 + row];
        }
        acc[tt] = mfma32(a, bb, acc[tt]);
      }
    }
    __syncthreads();
  }
  float* out = partial + ((size_t)c * 9 + tap) * COUT * CIN;
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    const int t = wave + 4 * tt;
    if (t < T) {
      const int mb = t / NCI, nb = t % NCI;
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(mb * 16 + kg * 4 + i) * CIN + nb * 16 + row] = acc[tt][i];
    }
  }
}

// dst[i] (+)= sum over chunks of partial[chunk * len + i], chunk order fixed
__global__ void chunk_reduce_kernel(const float* __restrict__ partial, int nchunks, int64_t len,
                                    float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * len + i];
  dst[i] = s;
}

// bias gradient partials: per chunk of pixels, the column sums of G
__global__ void bias_partial_kernel(const bf16_t* __restrict__ G, int C, int chunk, int npix,
                                    float* __restrict__ partial) {
  const int c = blockIdx.x;
  for (int co = threadIdx.x; co < C; co += blockDim.x) {
    float s = 0.f;
    const int k1 = min(npix, (c + 1) * chunk);
    for (int k = c * chunk; k < k1; ++k) s += bf2f(G[(size_t)k * C + co]);
    partial[(size_t)c * C + co] = s;
  }
}

// 2x2 average pooling, bf16 -> bf16 (S = fine size)
__global__ void pool_kernel(const bf16_t* __restrict__ X, bf16_t* __restrict__ Y, int S, int C,
                            int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int Sc = S / 2;
  const int c = (int)(i % C);
  const int64_t pc = i / C;
  const int x = (int)(pc % Sc), y = (int)((pc / Sc) % Sc);
  const int64_t b = pc / ((int64_t)Sc * Sc);
  const bf16_t* base = X + (size_t)b * S * S * C;
  const float s = bf2f(base[((size_t)(2 * y) * S + 2 * x) * C + c]) +
                  bf2f(base[((size_t)(2 * y) * S + 2 * x + 1) * C + c]) +
                  bf2f(base[((size_t)(2 * y + 1) * S + 2 * x) * C + c]) +
                  bf2f(base[((size_t)(2 * y + 1) * S + 2 * x + 1) * C + c]);
  Y[i] = f2bf(0.25f * s);
}

// Y = nearest-upsample(Xc) + skip, bf16 (S = fine size)
__global__ void upadd_kernel(const bf16_t* __restrict__ Xc, const bf16_t* __restrict__ skip,
                             bf16_t* __restrict__ Y, int S, int C, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % C);
  const int64_t p = i / C;
  const int x = (int)(p % S), y = (int)((p / S) % S);
  const int64_t b = p / ((int64_t)S * S);
  const int Sc = S / 2;
  const float v = bf2f(Xc[(((size_t)b * Sc + y / 2) * Sc + x / 2) * C + c]) + bf2f(skip[i]);
  Y[i] = f2bf(v);
}

// G = bf16(g * [act > 0]) (act may be null: no activation)
__global__ void mask_kernel(const float* __restrict__ g, const bf16_t* __restrict__ act,
                            bf16_t* __restrict__ G, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float v = g[i];
  if (act && !(bf2f(act[i]) > 0.f)) v = 0.f;
  G[i] = f2bf(v);
}

// gf += pool^T(gc) = gc / 4 on each fine pixel (S = fine size)
__global__ void pool_back_add_kernel(const float* __restrict__ gc, float* __restrict__ gf, int S,
                                     int C, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % C);
  const int64_t p = i / C;
  const int x = (int)(p % S), y = (int)((p / S) % S);
  const int64_t b = p / ((int64_t)S * S);
  const int Sc = S / 2;
  gf[i] += 0.25f * gc[(((size_t)b * Sc + y / 2) * Sc + x / 2) * C + c];
}

// gc = upsample^T(gf): sum of the four fine pixels (S = fine size)
__global__ void up_back_kernel(const float* __restrict__ gf, float* __restrict__ gc, int S, int C,
                               int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int Sc = S / 2;
  const int c = (int)(i % C);
  const int64_t pc = i / C;
  const int x = (int)(pc % Sc), y = (int)((pc / Sc) % Sc);
  const int64_t b = pc / ((int64_t)Sc * Sc);
  const float* base = gf + (size_t)b * S * S * C;
  gc[i] = base[((size_t)(2 * y) * S + 2 * x) * C + c] + base[((size_t)(2 * y) * S + 2 * x + 1) * C + c] +
          base[((size_t)(2 * y + 1) * S + 2 * x) * C + c] +
          base[((size_t)(2 * y + 1) * S + 2 * x + 1) * C + c];
}

// Batch input and target from stored pairs: X0[b][y][x][c] (bf16, CI0 channels:
// P modes, sigma, zeros) and T[b][y][x][c] (fp32, CO channels)
__global__ void assemble_kernel(const bf16_t* __restrict__ R, const bf16_t* __restrict__ Tp,
                                const float* __restrict__ sig, const int* __restrict__ idx, int P,
                                int n, int CI0, int CO, bf16_t* __restrict__ X0,
                                float* __restrict__ T, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;  // total = B * n * n
  const int x = (int)(i % n), y = (int)((i / n) % n);
  const int b = (int)(i / ((int64_t)n * n));
  const int m = n - 1;
  const int64_t Nh = (int64_t)m * m;
  const int64_t pr = idx[b];
  const bool valid = x < m && y < m;
  const int64_t node = (int64_t)y * m + x;
  bf16_t* xo = X0 + i * CI0;
  for (int c = 0; c < CI0; ++c) {
    bf16_t v = 0;
    if (c < P && valid) v = R[(pr * P + c) * Nh + node];
    else if (c == P) v = f2bf(sig[pr]);
    xo[c] = v;
  }
  if (T) {
    float* to = T + i * CO;
    for (int c = 0; c < CO; ++c) to[c] = (c < P && valid) ? bf2f(Tp[(pr * P + c) * Nh + node]) : 0.f;
  }
}

// Relative squared error partial sums: acc[b][block] = (sum (Y-T)^2, sum T^2) over
// valid pixels and channels < P
__global__ void loss_partial_kernel(const float* __restrict__ Y, const float* __restrict__ T, int P,
                                    int n, int CO, int nblk, double* __restrict__ acc) {
  __shared__ double r1[256], r2[256];
  const int b = blockIdx.y;
  const int64_t per = ((int64_t)n * n + nblk - 1) / nblk;
  const int64_t lo = blockIdx.x * per, hi = std::min<int64_t>((int64_t)n * n, lo + per);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) {
    const int x = (int)(p % n), y = (int)(p / n);
    if (x >= n - 1 || y >= n - 1) continue;
    const float* yp = Y + ((size_t)b * n * n + p) * CO;
    const float* tp = T + ((size_t)b * n * n + p) * CO;
    for (int c = 0; c < P; ++c) {
      const double d = (double)yp[c] - (double)tp[c];
      s1 += d * d;
      s2 += (double)tp[c] * (double)tp[c];
    }
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[((size_t)b * nblk + blockIdx.x) * 2] = r1[0];
    acc[((size_t)b * nblk + blockIdx.x) * 2 + 1] = r2[0];
  }
}

// per-sample sums -> loss (sum over samples of ratio / B) and den[b] = sum T^2
__global__ void loss_final_kernel(const double* __restrict__ acc, int B, int nblk,
                                  double* __restrict__ den, double* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double L = 0.0;
  for (int b = 0; b < B; ++b) {
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nblk; ++k) {
      s1 += acc[((size_t)b * nblk + k) * 2];
      s2 += acc[((size_t)b * nblk + k) * 2 + 1];
    }
    den[b] = s2;
    L += (s2 > 0.0 ? s1 / s2 : 0.0) / B;
  }
  loss[0] = L;
}

// dL/dY = 2 (Y - T) / den[b] / B on valid entries
__global__ void loss_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, int P,
                                 int n, int CO, int B, const double* __restrict__ den,
                                 float* __restrict__ dY, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % CO);
  const int64_t p = i / CO;
  const int x = (int)(p % n), y = (int)((p / n) % n);
  const int b = (int)(p / ((int64_t)n * n));
  float g = 0.f;
  if (c < P && x < n - 1 && y < n - 1 && den[b] > 0.0)
    g = (float)(2.0 * ((double)Y[i] - (double)T[i]) / den[b] / B);
  dY[i] = g;
}

// Adam on FP32 master weights (bias-corrected), in place
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 working copies of one layer: Wq[tap][co][ci] and the flipped transpose
// Wf[tap'][ci][co] = W[8 - tap'][co][ci] used by the data-gradient convolution
__global__ void cast_weights_kernel(const float* __restrict__ W, bf16_t* __restrict__ Wq,
                                    bf16_t* __restrict__ Wf, int co, int ci) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)9 * co * ci;
  if (i >= tot) return;
  const int c_i = (int)(i % ci);
  const int c_o = (int)((i / ci) % co);
  const int tap = (int)(i / ((int64_t)ci * co));
  const bf16_t q = f2bf(W[i]);
  Wq[i] = q;
  Wf[((int64_t)(8 - tap) * ci + c_i) * co + c_o] = q;
}

// SG vector (FP64, P x N_h mode-major) -> one network input image, scaled by
// s = sqrt(P N_h) / ||v|| (the norm squared is nrm2[0])
__global__ void sg_to_image_kernel(const double* __restrict__ v, const double* __restrict__ nrm2,
                                   double sigma, int P, int n, int CI0, bf16_t* __restrict__ X0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  const int x = (int)(i % n), y = (int)(i / n);
  const int m = n - 1;
  const int64_t Nh = (int64_t)m * m;
  const double s = sqrt((double)P * Nh) / sqrt(nrm2[0]);
  bf16_t* xo = X0 + i * CI0;
  for (int c = 0; c < CI0; ++c) {
    bf16_t q = 0;
    if (c < P && x < m && y < m) q = f2bf((float)(v[(int64_t)c * Nh + (int64_t)y * m + x] * s));
    else if (c == P) q = f2bf((float)sigma);
    xo[c] = q;
  }
}

// network output image -> SG vector c = Y ||v|| n^2 / (sqrt(P N_h) kappa)
__global__ void image_to_sg_kernel(const float* __restrict__ Y, const double* __restrict__ nrm2,
                                   int P, int n, int CO, double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = n - 1;
  const int64_t Nh = (int64_t)m * m;
  if (i >= (int64_t)P * Nh) return;
  const int mode = (int)(i / Nh);
  const int64_t node = i - (int64_t)mode * Nh;
  const int x = (int)(node % m), y = (int)(node / m);
  const double s = sqrt(nrm2[0]) * (double)n * n / (sqrt((double)P * Nh) * kTargetScale);
  c[i] = (double)Y[((int64_t)y * n + x) * CO + mode] * s;
}

// batch slot of the network output -> SG vector (no scaling; the stage
// objective is scale-free): c[mode * N_h + node] = Y[slot][y][x][mode]
__global__ void slot_to_sg_kernel(const float* __restrict__ Y, int slot, int P, int n, int CO,
                                  double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = n - 1;
  const int64_t Nh = (int64_t)m * m;
  if (i >= (int64_t)P * Nh) return;
  const int mode = (int)(i / Nh);
  const int64_t node = i - (int64_t)mode * Nh;
  const int x = (int)(node % m), y = (int)(node / m);
  c[i] = (double)Y[(((int64_t)slot * n + y) * n + x) * CO + mode];
}

// stored bf16 pair residual -> FP64 SG vector
__global__ void pair_to_sg_kernel(const bf16_t* __restrict__ R, int64_t len, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) r[i] = (double)bf2f(R[i]);
}

// output gradient of one batch slot from an SG vector: dY[slot][y][x][c] =
// scale[0] g[c * N_h + node] on interior pixels and the first P channels,
// zero elsewhere in the slot
__global__ void sg_to_slot_grad_kernel(const double* __restrict__ g, const double* __restrict__ scale,
                                       int slot, int P, int n, int CO, float* __restrict__ dY) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n * CO) return;
  const int c = (int)(i % CO);
  const int64_t px = i / CO;
  const int x = (int)(px % n), y = (int)(px / n);
  const int m = n - 1;
  float v = 0.f;
  if (c < P && x < m && y < m) v = (float)(scale[0] * g[(int64_t)c * m * m + (int64_t)y * m + x]);
  dY[(int64_t)slot * n * n * CO + i] = v;
}

// one training pair from FP64 SG vectors: residual r and error e = ustar - u;
// R = bf16(r s), T = bf16(e s kappa / n^2), s = sqrt(P N_h) / ||r||
__global__ void make_pair_kernel(const double* __restrict__ r, const double* __restrict__ ustar,
                                 const double* __restrict__ u, const double* __restrict__ nrm2,
                                 int n, int64_t len, bf16_t* __restrict__ R,
                                 bf16_t* __restrict__ T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double s = sqrt((double)len) / sqrt(nrm2[0]);
  R[i] = f2bf((float)(r[i] * s));
  T[i] = f2bf((float)((ustar[i] - u[i]) * s * kTargetScale / ((double)n * n)));
}

// ===========================================================================
// host side
// ===========================================================================
struct CnnLayer {
  int ci, co, relu, level;
  size_t woff, boff;  // offsets in the concatenated weight / bias arrays
};

struct sg_cnn_impl {
  int P, n, c0, c1, maxB, CI0, CO;
  std::vector<CnnLayer> L;
  size_t nw = 0, nb = 0;
  bool bound = false;
  // device
  float *W = nullptr, *Wm = nullptr, *Wv = nullptr, *dW = nullptr;
  float *Bs = nullptr, *Bm = nullptr, *Bv = nullptr, *dB = nullptr;
  bf16_t *Wq = nullptr, *Wf = nullptr;
  bf16_t* act[20] = {};
  float* Y = nullptr;
  float* T = nullptr;
  float *g0 = nullptr, *g1 = nullptr, *gs0 = nullptr, *gs1 = nullptr, *gs2 = nullptr;
  bf16_t* Gm = nullptr;
  float* partial = nullptr;
  double *lacc = nullptr, *lden = nullptr, *lval = nullptr, *nrm = nullptr, *dscr = nullptr;
  int* idx = nullptr;
  int nchunk_max = 0;
  size_t partial_len = 0;
  std::vector<double> host_loss;
};

}  // namespace sg

// ---------------------------------------------------------------------------
namespace {

using namespace sg;

constexpr int kChunk = 2048;   // pixels per weight-gradient workgroup
// convolutions over at least kConvWidePix pixels (the finest levels at full
// batch) take kConvTiles 16-pixel tiles per wavefront, so that each weight
// fragment a wavefront loads serves that many tiles
constexpr int kConvTiles = 4;
constexpr int kConvWidePix = 64 * kConvTiles * 512;
constexpr int kLossBlk = 16;

template <class T>
T* carve_take(char*& base, size_t& off, size_t count) {
  T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
  off += (count * sizeof(T) + 255) & ~size_t(255);
  return p;
}

// buffer indices in act[]: 0 X0, then per layer l: in_l (1+2l) and out_l (2+2l)
enum { A_X0 = 0 };
inline int A_IN(int l) { return 1 + 2 * l; }
inline int A_OUT(int l) { return 2 + 2 * l; }

int level_size(const sg_cnn_impl& C, int lvl) { return C.n >> lvl; }

size_t layout(sg_cnn_impl& C, char* base) {
  size_t off = 0;
  C.W = carve_take<float>(base, off, C.nw);
  C.Wm = carve_take<float>(base, off, C.nw);
  C.Wv = carve_take<float>(base, off, C.nw);
  C.dW = carve_take<float>(base, off, C.nw);
  C.Bs = carve_take<float>(base, off, C.nb);
  C.Bm = carve_take<float>(base, off, C.nb);
  C.Bv = carve_take<float>(base, off, C.nb);
  C.dB = carve_take<float>(base, off, C.nb);
  C.Wq = carve_take<bf16_t>(base, off, C.nw);
  C.Wf = carve_take<bf16_t>(base, off, C.nw);
  const size_t B = C.maxB;
  auto px = [&](int lvl) { size_t s = level_size(C, lvl); return B * s * s; };
  C.act[A_X0] = carve_take<bf16_t>(base, off, px(0) * C.CI0);
  size_t gmax = 0;
  for (size_t l = 0; l < C.L.size(); ++l) {
    const CnnLayer& ly = C.L[l];
    if (l > 0) C.act[A_IN(l)] = carve_take<bf16_t>(base, off, px(ly.level) * ly.ci);
    if (l + 1 < C.L.size()) C.act[A_OUT(l)] = carve_take<bf16_t>(base, off, px(ly.level) * ly.co);
    gmax = std::max(gmax, px(ly.level) * (size_t)std::max(ly.ci, ly.co));
  }
  C.Y = carve_take<float>(base, off, px(0) * C.CO);
  C.T = carve_take<float>(base, off, px(0) * C.CO);
  C.g0 = carve_take<float>(base, off, gmax);
  C.g1 = carve_take<float>(base, off, gmax);
  C.gs0 = carve_take<float>(base, off, px(0) * C.c0);
  C.gs1 = carve_take<float>(base, off, px(1) * C.c1);
  C.gs2 = carve_take<float>(base, off, px(2) * C.c1);
  C.Gm = carve_take<bf16_t>(base, off, gmax);
  C.nchunk_max = cdivl((int64_t)px(0), kChunk);
  C.partial_len = (size_t)C.nchunk_max * 9 * 64 * 64;
  C.partial = carve_take<float>(base, off, C.partial_len);
  C.lacc = carve_take<double>(base, off, 2 * B * kLossBlk);
  C.lden = carve_take<double>(base, off, B);
  C.lval = carve_take<double>(base, off, 4);
  C.nrm = carve_take<double>(base, off, 4);
  C.dscr = carve_take<double>(base, off, 1024);
  C.idx = carve_take<int>(base, off, B);
  return off;
}

void check_last() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SG_ERR_HIP, std::string("cnn kernel launch: ") + hipGetErrorString(e));
}

void conv_forward(hipStream_t s, const sg_cnn_impl& C, int l, const bf16_t* X, void* Y, int B,
                  int mode) {
  const CnnLayer& ly = C.L[l];
  const int S = level_size(C, ly.level);
  const int npix = B * S * S;
  const bool wide = npix >= kConvWidePix;
  dim3 grid(cdivl(npix, wide ? 64 * kConvTiles : 64));
  const bf16_t* W = C.Wq + ly.woff;
  const float* bias = C.Bs + ly.boff;
#define SG_CONV(CI, CO_, M)                                                                   \
  if (ly.ci == CI && ly.co == CO_ && mode == M) {                                             \
    if (wide)                                                                                 \
      hipLaunchKernelGGL((conv_fwd_kernel<CI, CO_, M, kConvTiles>), grid, dim3(256), 0, s, X, W, \
                         bias, Y, S, npix);                                                   \
    else                                                                                      \
      hipLaunchKernelGGL((conv_fwd_kernel<CI, CO_, M, 1>), grid, dim3(256), 0, s, X, W, bias, Y, \
                         S, npix);                                                            \
    return;                                                                                   \
  }
  SG_CONV(32, 32, 0) SG_CONV(64, 32, 0) SG_CONV(32, 64, 0) SG_CONV(64, 64, 0)
  SG_CONV(32, 32, 1) SG_CONV(32, 64, 1) SG_CONV(64, 32, 1) SG_CONV(64, 64, 1)
#undef SG_CONV
  throw Error(SG_ERR_UNSUPPORTED, "cnn: unsupported layer shape");
}

// dX (fp32) = data gradient of layer l from the masked output gradient G (bf16)
void conv_backward_data(hipStream_t s, const sg_cnn_impl& C, int l, const bf16_t* G, float* dX,
                        int B) {
  const CnnLayer& ly = C.L[l];
  const int S = level_size(C, ly.level);
  const int npix = B * S * S;
  const bool wide = npix >= kConvWidePix;
  dim3 grid(cdivl(npix, wide ? 64 * kConvTiles : 64));
  const bf16_t* Wf = C.Wf + ly.woff;
#define SG_CONVT(CO_, CI)                                                                       \
  if (ly.co == CO_ && ly.ci == CI) {                                                            \
    if (wide)                                                                                   \
      hipLaunchKernelGGL((conv_fwd_kernel<CO_, CI, 2, kConvTiles>), grid, dim3(256), 0, s, G, Wf, \
                         nullptr, dX, S, npix);                                                 \
    else                                                                                        \
      hipLaunchKernelGGL((conv_fwd_kernel<CO_, CI, 2, 1>), grid, dim3(256), 0, s, G, Wf, nullptr, \
                         dX, S, npix);                                                          \
    return;                                                                                     \
  }
  SG_CONVT(32, 32) SG_CONVT(32, 64) SG_CONVT(64, 32) SG_CONVT(64, 64)
#undef SG_CONVT
  throw Error(SG_ERR_UNSUPPORTED, "cnn: unsupported layer shape (backward)");
}

void conv_backward_weight(hipStream_t s, sg_cnn_impl& C, int l, const bf16_t* X, const bf16_t* G,
                          int B) {
  const CnnLayer& ly = C.L[l];
  const int S = level_size(C, ly.level);
  const int npix = B * S * S;
  const int nch = cdivl(npix, kChunk);
  dim3 grid(nch, 9);
#define SG_BWDW(CI, CO_)                                                                         \
  if (ly.ci == CI && ly.co == CO_) {                                                             \
    hipLaunchKernelGGL((conv_bwdw_kernel<CI, CO_>), grid, dim3(256), 0, s, X, G, C.partial, S,  \
                       kChunk, npix);                                                            \
  } else
  SG_BWDW(32, 32) SG_BWDW(64, 32) SG_BWDW(32, 64) SG_BWDW(64, 64) {
    throw Error(SG_ERR_UNSUPPORTED, "cnn: unsupported layer shape (weight gradient)");
  }
#undef SG_BWDW
  const int64_t len = (int64_t)9 * ly.co * ly.ci;
  hipLaunchKernelGGL(chunk_reduce_kernel, dim3(cdivl(len, 256)), dim3(256), 0, s, C.partial, nch,
                     len, C.dW + ly.woff);
  hipLaunchKernelGGL(bias_partial_kernel, dim3(nch), dim3(64), 0, s, G, ly.co, kChunk, npix,
                     C.partial);
  hipLaunchKernelGGL(chunk_reduce_kernel, dim3(1), dim3(64), 0, s, C.partial, nch,
                     (int64_t)ly.co, C.dB + ly.boff);
}

template <class K, class... A>
void launch1d(hipStream_t s, K k, int64_t total, A... args) {
  hipLaunchKernelGGL(k, dim3(cdivl(total, 256)), dim3(256), 0, s, args..., total);
}

// full forward from act[A_X0]; output Y (fp32)
void forward(hipStream_t s, sg_cnn_impl& C, int B) {
  auto px = [&](int lvl) { int64_t S = level_size(C, lvl); return (int64_t)B * S * S; };
  const bf16_t* x = C.act[A_X0];
  for (size_t l = 0; l < C.L.size(); ++l) {
    const CnnLayer& ly = C.L[l];
    const int S = level_size(C, ly.level);
    bf16_t* in = (l == 0) ? const_cast<bf16_t*>(x) : C.act[A_IN(l)];
    if (l == 2 || l == 3 || l == 4) {
      // pooled output of the previous layer (the skip tensor one level up)
      launch1d(s, pool_kernel, px(ly.level) * ly.ci, C.act[A_OUT(l - 1)], in, 2 * S, ly.ci);
    } else if (l == 5 || l == 6 || l == 7) {
      const int skip_layer = (l == 5) ? 3 : (l == 6) ? 2 : 1;
      launch1d(s, upadd_kernel, px(ly.level) * ly.ci, C.act[A_OUT(l - 1)],
               C.act[A_OUT(skip_layer)], in, S, ly.ci);
    } else if (l == 1 || l == 8) {
      in = C.act[A_OUT(l - 1)];
    }
    if (l + 1 < C.L.size()) conv_forward(s, C, (int)l, in, C.act[A_OUT(l)], B, 0);
    else conv_forward(s, C, (int)l, in, C.Y, B, 1);
  }
  check_last();
}

const bf16_t* layer_input(const sg_cnn_impl& C, size_t l) {
  if (l == 0) return C.act[A_X0];
  if (l == 1 || l == 8) return C.act[A_OUT(l - 1)];
  return C.act[A_IN(l)];
}

// backward from dY = C.g0 (fp32, B x n x n x CO); fills C.dW, C.dB
void backward(hipStream_t s, sg_cnn_impl& C, int B) {
  auto px = [&](int lvl) { int64_t S = level_size(C, lvl); return (int64_t)B * S * S; };
  float* g = C.g0;     // gradient w.r.t. the current layer's output
  float* gx = C.g1;    // scratch for data gradients
  auto layer_back = [&](int l, const float* gout, float* dX) {
    const CnnLayer& ly = C.L[l];
    const bf16_t* act = (l + 1 < (int)C.L.size()) ? C.act[A_OUT(l)] : nullptr;
    launch1d(s, mask_kernel, px(ly.level) * ly.co, gout, act, C.Gm);
    conv_backward_weight(s, C, l, layer_input(C, l), C.Gm, B);
    if (dX) conv_backward_data(s, C, l, C.Gm, dX, B);
  };
  const int S0 = level_size(C, 0), S1 = level_size(C, 1), S2 = level_size(C, 2);
  // layer 8: input = out7
  layer_back(8, g, gx);                          // gx = d out7
  layer_back(7, gx, C.gs0);                      // gs0 = d in7 (skip part)
  launch1d(s, up_back_kernel, px(1) * C.c0, C.gs0, g, S0, C.c0);      // g = d out6
  layer_back(6, g, C.gs1);                       // gs1 = d in6
  launch1d(s, up_back_kernel, px(2) * C.c1, C.gs1, g, S1, C.c1);      // g = d out5
  layer_back(5, g, C.gs2);                       // gs2 = d in5
  launch1d(s, up_back_kernel, px(3) * C.c1, C.gs2, g, S2, C.c1);      // g = d out4
  layer_back(4, g, gx);                          // gx = d pool(out3)
  launch1d(s, pool_back_add_kernel, px(2) * C.c1, gx, C.gs2, S2, C.c1);  // gs2 = d out3
  layer_back(3, C.gs2, gx);                      // gx = d pool(out2)
  launch1d(s, pool_back_add_kernel, px(1) * C.c1, gx, C.gs1, S1, C.c1);  // gs1 = d out2
  layer_back(2, C.gs1, gx);                      // gx = d pool(out1)
  launch1d(s, pool_back_add_kernel, px(0) * C.c0, gx, C.gs0, S0, C.c0);  // gs0 = d out1
  layer_back(1, C.gs0, gx);                      // gx = d out0
  layer_back(0, gx, nullptr);
  check_last();
}

void cast_all(hipStream_t s, sg_cnn_impl& C) {
  for (const CnnLayer& ly : C.L) {
    const int64_t tot = (int64_t)9 * ly.co * ly.ci;
    hipLaunchKernelGGL(cast_weights_kernel, dim3(cdivl(tot, 256)), dim3(256), 0, s, C.W + ly.woff,
                       C.Wq + ly.woff, C.Wf + ly.woff, ly.co, ly.ci);
  }
}

thread_local std::string g_cnn_err;

int cfail(int code, const std::string& m) {
  g_cnn_err = m;
  return code;
}

}  // namespace

// ===========================================================================
struct sg_cnn : sg::sg_cnn_impl {};

namespace sg {

// z-free inference on an SG vector: c = N(v) in SG units (stream-ordered)
void cnn_apply_sg(sg_cnn* C, hipStream_t s, const double* v, double sigma, double* c,
                  double* scratch_partial, int nblk) {
  const int64_t Nv = (int64_t)C->P * (C->n - 1) * (C->n - 1);
  launch_multidot(s, v, Nv, 1, v, Nv, scratch_partial, nblk);
  launch_reduce(s, scratch_partial, nblk, 1, C->nrm);
  const int64_t npx = (int64_t)C->n * C->n;
  hipLaunchKernelGGL(sg_to_image_kernel, dim3(cdivl(npx, 256)), dim3(256), 0, s, v, C->nrm, sigma,
                     C->P, C->n, C->CI0, C->act[A_X0]);
  forward(s, *C, 1);
  hipLaunchKernelGGL(image_to_sg_kernel, dim3(cdivl(Nv, 256)), dim3(256), 0, s, C->Y, C->nrm, C->P,
                     C->n, C->CO, c);
}

void cnn_slot_to_sg(sg_cnn* C, hipStream_t s, int slot, double* c) {
  const int64_t Nv = (int64_t)C->P * (C->n - 1) * (C->n - 1);
  hipLaunchKernelGGL(slot_to_sg_kernel, dim3(cdivl(Nv, 256)), dim3(256), 0, s, C->Y, slot, C->P,
                     C->n, C->CO, c);
}

void cnn_pair_to_sg(sg_cnn* C, hipStream_t s, const uint16_t* R, int64_t pair, double* r) {
  const int64_t Nv = (int64_t)C->P * (C->n - 1) * (C->n - 1);
  hipLaunchKernelGGL(pair_to_sg_kernel, dim3(cdivl(Nv, 256)), dim3(256), 0, s,
                     reinterpret_cast<const bf16_t*>(R) + pair * Nv, Nv, r);
}

void cnn_slot_grad_from_sg(sg_cnn* C, hipStream_t s, int slot, const double* g,
                           const double* scale) {
  const int64_t tot = (int64_t)C->n * C->n * C->CO;
  hipLaunchKernelGGL(sg_to_slot_grad_kernel, dim3(cdivl(tot, 256)), dim3(256), 0, s, g, scale,
                     slot, C->P, C->n, C->CO, C->g0);
}

int cnn_max_batch(const sg_cnn* C) { return C->maxB; }

__global__ void stage_objective_coef_kernel(double* __restrict__ d, int batch) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double a = d[0], b = d[1], rho = d[2];
  const bool ok = b > 0.0 && rho > 0.0;
  d[3] = ok ? a / b : 0.0;
  d[4] = ok ? 2.0 * a / (rho * b * batch) : 0.0;
  d[5] = ok ? 1.0 - a * a / (rho * b) : 0.0;
}

__global__ void stage_objective_vec_kernel(const double* __restrict__ d, const double* __restrict__ Kc,
                                           const double* __restrict__ r, double* __restrict__ v,
                                           int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] = d[3] * Kc[i] - r[i];
}

void launch_stage_objective(hipStream_t s, double* dots, int batch, const double* Kc,
                            const double* r, double* v, int64_t N) {
  hipLaunchKernelGGL(stage_objective_coef_kernel, dim3(1), dim3(64), 0, s, dots, batch);
  hipLaunchKernelGGL(stage_objective_vec_kernel, dim3(cdivl(N, 256)), dim3(256), 0, s, dots, Kc, r,
                     v, N);
}

int cnn_modes(const sg_cnn* C) { return C->P; }
int cnn_grid(const sg_cnn* C) { return C->n; }
bool cnn_bound(const sg_cnn* C) { return C && C->bound; }

}  // namespace sg

extern "C" {

const char* sg_cnn_last_error(void) { return g_cnn_err.c_str(); }

int sg_cnn_create(int32_t P, int32_t n, int32_t c0, int32_t c1, int32_t max_batch, sg_cnn** out) {
  if (!out) return cfail(SG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (P < 1 || P > 63) return cfail(SG_ERR_UNSUPPORTED, "P must be in [1, 63] for the network");
  if (n < 16 || n > 1024 || (n & (n - 1))) return cfail(SG_ERR_INVALID_ARG, "n must be a power of two in [16, 1024]");
  if ((c0 != 32 && c0 != 64) || c1 != 64)
    return cfail(SG_ERR_UNSUPPORTED, "hidden widths: first level 32 or 64, coarser levels 64");
  if (max_batch < 1 || max_batch > 256) return cfail(SG_ERR_INVALID_ARG, "max_batch in [1, 256]");
  sg_cnn* C = new sg_cnn();
  C->P = P;
  C->n = n;
  C->c0 = c0;
  C->c1 = c1;
  C->maxB = max_batch;
  C->CI0 = ((P + 1 + 31) / 32) * 32;
  C->CO = ((P + 31) / 32) * 32;
  const int tab[9][4] = {{C->CI0, c0, 1, 0}, {c0, c0, 1, 0}, {c0, c1, 1, 1}, {c1, c1, 1, 2},
                         {c1, c1, 1, 3},     {c1, c1, 1, 2}, {c1, c0, 1, 1}, {c0, c0, 1, 0},
                         {c0, C->CO, 0, 0}};
  for (auto& t : tab) {
    CnnLayer ly{t[0], t[1], t[2], t[3], C->nw, C->nb};
    C->nw += (size_t)9 * ly.ci * ly.co;
    C->nb += ly.co;
    C->L.push_back(ly);
  }
  *out = C;
  return SG_OK;
}

int sg_cnn_param_counts(const sg_cnn* C, int64_t* nweights, int64_t* nbias) {
  if (!C) return cfail(SG_ERR_INVALID_ARG, "null handle");
  if (nweights) *nweights = (int64_t)C->nw;
  if (nbias) *nbias = (int64_t)C->nb;
  return SG_OK;
}

size_t sg_cnn_workspace_bytes(const sg_cnn* C) {
  if (!C) return 0;
  sg_cnn tmp = *C;
  return layout(tmp, nullptr);
}

int sg_cnn_bind(sg_cnn* C, void* ws, size_t bytes, void* stream) {
  if (!C || !ws) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (bytes < sg_cnn_workspace_bytes(C)) return cfail(SG_ERR_WORKSPACE, "CNN workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return cfail(SG_ERR_WORKSPACE, "CNN workspace must be 256-byte aligned");
  layout(*C, static_cast<char*>(ws));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemsetAsync(ws, 0, sg_cnn_workspace_bytes(C), s) != hipSuccess)
    return cfail(SG_ERR_HIP, "memset failed");
  if (hipStreamSynchronize(s) != hipSuccess) return cfail(SG_ERR_HIP, "sync failed");
  C->bound = true;
  return SG_OK;
}

// W: concatenated per-layer (9, co, ci) FP32 weights; b: concatenated biases (host)
int sg_cnn_set_params(sg_cnn* C, const float* W, const float* b, void* stream) {
  if (!C || !W || !b) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(C->W, W, C->nw * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(C->Bs, b, C->nb * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(C->Wm, 0, C->nw * 4, s) != hipSuccess ||
        hipMemsetAsync(C->Wv, 0, C->nw * 4, s) != hipSuccess ||
        hipMemsetAsync(C->Bm, 0, C->nb * 4, s) != hipSuccess ||
        hipMemsetAsync(C->Bv, 0, C->nb * 4, s) != hipSuccess)
      return cfail(SG_ERR_HIP, "copy failed");
    cast_all(s, *C);
    check_last();
    if (hipStreamSynchronize(s) != hipSuccess) return cfail(SG_ERR_HIP, "sync failed");
    return SG_OK;
  } catch (const Error& e) {
    return cfail(e.code, e.what());
  }
}

int sg_cnn_get_params(sg_cnn* C, float* W, float* b) {
  if (!C || !W || !b) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(W, C->W, C->nw * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(b, C->Bs, C->nb * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return cfail(SG_ERR_HIP, "copy failed");
  return SG_OK;
}

// Adam moments (first and second, weights then biases) out and in, so that a
// training run can be stopped and resumed: together with the parameters and
// the step number the caller passes, they are the whole optimiser state
int sg_cnn_get_adam(sg_cnn* C, float* wm, float* wv, float* bm, float* bv) {
  if (!C || !wm || !wv || !bm || !bv) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(wm, C->Wm, C->nw * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(wv, C->Wv, C->nw * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(bm, C->Bm, C->nb * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(bv, C->Bv, C->nb * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return cfail(SG_ERR_HIP, "copy failed");
  return SG_OK;
}

int sg_cnn_set_adam(sg_cnn* C, const float* wm, const float* wv, const float* bm, const float* bv,
                    void* stream) {
  if (!C || !wm || !wv || !bm || !bv) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(C->Wm, wm, C->nw * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(C->Wv, wv, C->nw * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(C->Bm, bm, C->nb * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(C->Bv, bv, C->nb * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return cfail(SG_ERR_HIP, "copy failed");
  return SG_OK;
}

// One training pair from device FP64 SG vectors: residual r, reference solution
// ustar and iterate u (error ustar - u); R_out, T_out are P*N_h bf16
int sg_cnn_make_pair(sg_cnn* C, const double* r, const double* ustar, const double* u,
                     uint16_t* R_out, uint16_t* T_out, void* stream) {
  if (!C || !r || !ustar || !u || !R_out || !T_out) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t len = (int64_t)C->P * (C->n - 1) * (C->n - 1);
  const int nblk = dot_blocks(len);
  launch_multidot(s, r, len, 1, r, len, C->dscr, nblk);
  launch_reduce(s, C->dscr, nblk, 1, C->nrm);
  hipLaunchKernelGGL(make_pair_kernel, dim3(cdivl(len, 256)), dim3(256), 0, s, r, ustar, u, C->nrm,
                     C->n, len, reinterpret_cast<bf16_t*>(R_out), reinterpret_cast<bf16_t*>(T_out));
  return hipGetLastError() == hipSuccess ? SG_OK : cfail(SG_ERR_HIP, "launch failed");
}

// Forward (and optionally backward) on a batch of stored pairs.
//   R, Tp: pair arrays (npairs x P x N_h bf16, device); sig: npairs floats (device);
//   idx: batch indices (host, `batch` entries); Y_out (nullable, device): the
//   network output B x n x n x CO fp32; loss (nullable, host).
//   mode 0: forward only; 1: forward + gradients; 2: 1 + Adam step with lr.
int sg_cnn_run(sg_cnn* C, const uint16_t* R, const uint16_t* Tp, const float* sig,
               const int32_t* idx, int32_t batch, int32_t mode, float lr, int32_t step,
               float* Y_out, double* loss, void* stream) {
  if (!C || !R || !sig || !idx) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  if (batch < 1 || batch > C->maxB) return cfail(SG_ERR_INVALID_ARG, "batch out of range");
  if (mode < 0 || mode > 2) return cfail(SG_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
  if (mode > 0 && !Tp) return cfail(SG_ERR_INVALID_ARG, "targets needed for gradients");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(C->idx, idx, batch * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess)
      return cfail(SG_ERR_HIP, "copy failed");
    const int64_t npx = (int64_t)batch * C->n * C->n;
    hipLaunchKernelGGL(assemble_kernel, dim3(cdivl(npx, 256)), dim3(256), 0, s,
                       reinterpret_cast<const bf16_t*>(R), reinterpret_cast<const bf16_t*>(Tp),
                       sig, C->idx, C->P, C->n, C->CI0, C->CO, C->act[A_X0], Tp ? C->T : nullptr,
                       npx);
    forward(s, *C, batch);
    if (Y_out)
      if (hipMemcpyAsync(Y_out, C->Y, npx * C->CO * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return cfail(SG_ERR_HIP, "copy failed");
    if (Tp) {
      hipLaunchKernelGGL(loss_partial_kernel, dim3(kLossBlk, batch), dim3(256), 0, s, C->Y, C->T,
                         C->P, C->n, C->CO, kLossBlk, C->lacc);
      hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, C->lacc, batch, kLossBlk,
                         C->lden, C->lval);
    }
    if (mode >= 1) {
      launch1d(s, loss_grad_kernel, npx * C->CO, C->Y, C->T, C->P, C->n, C->CO, batch, C->lden,
               C->g0);
      backward(s, *C, batch);
    }
    if (mode == 2) {
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
      hipLaunchKernelGGL(adam_kernel, dim3(cdivl(C->nw, 256)), dim3(256), 0, s, C->W, C->Wm, C->Wv,
                         C->dW, (int64_t)C->nw, lr, b1, b2, 1e-8f, c1, c2);
      hipLaunchKernelGGL(adam_kernel, dim3(cdivl(C->nb, 256)), dim3(256), 0, s, C->Bs, C->Bm, C->Bv,
                         C->dB, (int64_t)C->nb, lr, b1, b2, 1e-8f, c1, c2);
      cast_all(s, *C);
    }
    check_last();
    if (loss && Tp) {
      double lv = 0.0;
      if (hipMemcpyAsync(&lv, C->lval, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return cfail(SG_ERR_HIP, "copy failed");
      *loss = lv;
    }
    return SG_OK;
  } catch (const Error& e) {
    return cfail(e.code, e.what());
  }
}

// Gradients of the last sg_cnn_run with mode >= 1 (host copies)
int sg_cnn_get_grads(sg_cnn* C, float* dW, float* dB) {
  if (!C || !dW || !dB) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(dW, C->dW, C->nw * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(dB, C->dB, C->nb * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return cfail(SG_ERR_HIP, "copy failed");
  return SG_OK;
}

// Gradients (and, with adam != 0, one Adam step) from the output gradient the
// caller's sg_cnn_stage_grad calls left in the network for the batch of the
// last forward (sg_cnn_run)
int sg_cnn_backward(sg_cnn* C, int32_t batch, int32_t adam, float lr, int32_t step, void* stream) {
  if (!C) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  if (batch < 1 || batch > C->maxB) return cfail(SG_ERR_INVALID_ARG, "batch out of range");
  if (adam && step < 1) return cfail(SG_ERR_INVALID_ARG, "Adam step numbers start at 1");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    backward(s, *C, batch);
    if (adam) {
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
      hipLaunchKernelGGL(adam_kernel, dim3(cdivl(C->nw, 256)), dim3(256), 0, s, C->W, C->Wm, C->Wv,
                         C->dW, (int64_t)C->nw, lr, b1, b2, 1e-8f, c1, c2);
      hipLaunchKernelGGL(adam_kernel, dim3(cdivl(C->nb, 256)), dim3(256), 0, s, C->Bs, C->Bm, C->Bv,
                         C->dB, (int64_t)C->nb, lr, b1, b2, 1e-8f, c1, c2);
      cast_all(s, *C);
    }
    check_last();
    return SG_OK;
  } catch (const Error& e) {
    return cfail(e.code, e.what());
  }
}

// Inference in SG units: c = ||v|| n^2 / sqrt(P N_h) * N(v sqrt(P N_h) / ||v||, sigma)
int sg_cnn_apply(sg_cnn* C, const double* v, double sigma, double* c, void* stream) {
  if (!C || !v || !c) return cfail(SG_ERR_INVALID_ARG, "null argument");
  if (!C->bound) return cfail(SG_ERR_NOT_BOUND, "CNN not bound");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    cnn_apply_sg(C, s, v, sigma, c, C->dscr, dot_blocks((int64_t)C->P * (C->n - 1) * (C->n - 1)));
    check_last();
    return SG_OK;
  } catch (const Error& e) {
    return cfail(e.code, e.what());
  }
}

void sg_cnn_destroy(sg_cnn* C) { delete C; }

}  // extern "C"
