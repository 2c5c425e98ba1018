// HIP kernels (gfx950) of the multigrid V-cycle on the full stochastic-
// Galerkin system (Sec. 3: multigrid on K with the field-split level
// iteration of eq. level_solver as the smoother, the G-M-F-I / G-M-Fg-I
// family).  Every level carries the whole SG operator, applied by the
// operator-apply kernels on that level's grid; these kernels add:
//  * the nodal split blocks: probe vectors for the apply (one mode, one of
//    four node colours), the gather of the probed columns, and the in-place
//    inversion of every node's |g| x |g| block;
//  * the smoother's block step dz_{g}(node) = omega D_node^{-1} t(node);
//  * the transfers (bilinear prolongation, restriction by its transpose) for
//    all modes at once, and the dense solve of the coarsest level.
// Vectors are mode-major (entry i*N + node, node = (iy-1)(n-1) + (ix-1)).
// Nodal blocks are stored pair-major (a thread per node reads consecutive
// addresses): the probed blocks in full, entry (a*m + b)*N + node, their
// inverses as the upper triangle of the block padded to a compiled size,
// packed row by row.  No atomics: every output is
// written by one thread, every sum in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sg_internal.h"

namespace sg {

namespace {

inline int mg_cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
// the most modes one split's nodal blocks may hold (the largest inversion
// kernel below)
constexpr int kMgMaxSplit = 128;

// colour of an interior node: (ix mod 2) + 2 (iy mod 2); two nodes of one
// colour are at least two grid steps apart in x or in y, so the 9-point
// couplings of K never join them
__device__ __forceinline__ int node_colour(int64_t node, int m) {
  const int ix = (int)(node % m) + 1, iy = (int)(node / m) + 1;
  return (ix & 1) + 2 * (iy & 1);
}

__global__ void mg_mark_kernel(double* __restrict__ u, int m, int colour, double val, int64_t N) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node < N && node_colour(node, m) == colour) u[node] = val;
}

// D[(a*mm + b)*N + node] = W[modes[a]*N + node] for the nodes of one colour
__global__ void mg_gather_kernel(const double* __restrict__ W, int m, int colour,
                                 const int* __restrict__ modes, int mm, int b,
                                 double* __restrict__ D, int64_t N) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (node >= N || node_colour(node, m) != colour) return;
  D[((int64_t)a * mm + b) * N + node] = W[(int64_t)modes[a] * N + node];
}

// index of pair (a, b), a <= b < MP, in the row-by-row packing of an MP x MP
// upper triangle
template <int MP>
__host__ __device__ constexpr int64_t packed_pair(int a, int b) {
  return (int64_t)a * MP - (int64_t)a * (a - 1) / 2 + (b - a);
}

// Inverse of every node's mm x mm block (symmetric positive definite:
// Gauss-Jordan without pivoting), padded to MP x MP with the identity.  Reads
// the full block, entry (a*mm + b)*N + node, and writes the inverse's upper
// triangle packed into the same array.  One
// workgroup per node, thread i holds row i in registers; step k broadcasts
// the scaled pivot row through LDS.  Steps past mm leave the identity padding
// unchanged, so only mm steps run.
template <int MP>
__global__ __launch_bounds__(MP < 64 ? 64 : MP) __attribute__((amdgpu_waves_per_eu(1, 2))) void mg_invert_kernel(double* __restrict__ D,
                                                                     int mm, int64_t N) {
  __shared__ double prow[MP];
  const int64_t node = blockIdx.x;
  const int i = threadIdx.x;
  double a[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j)
    a[j] = (i < mm && j < mm) ? D[((int64_t)i * mm + j) * N + node] : (i == j ? 1.0 : 0.0);
  // the step loop stays rolled; a[k] is picked by selects over the unrolled
  // column loop, so the row never leaves the registers
#pragma unroll 1
  for (int k = 0; k < mm; ++k) {
    double f = 0.0;
#pragma unroll
    for (int j = 0; j < MP; ++j) f = (j == k) ? a[j] : f;
    if (i == k) {
      const double piv = 1.0 / f;
#pragma unroll
      for (int j = 0; j < MP; ++j) {
        a[j] = (j == k) ? piv : a[j] * piv;
        prow[j] = a[j];
      }
    }
    __syncthreads();
    if (i != k && i < MP) {
#pragma unroll
      for (int j = 0; j < MP; ++j) a[j] = (j == k ? 0.0 : a[j]) - f * prow[j];
    }
    __syncthreads();
  }
  // the inverse is symmetric: row i keeps its entries j >= i, packed row by
  // row over the padded size (pair (i, j) at packed_pair<MP>(i, j)); the
  // padding rows hold the identity
  if (i < MP) {
#pragma unroll
    for (int j = 0; j < MP; ++j)
      if (j >= i) D[packed_pair<MP>(i, j) * N + node] = a[j];
  }
}


// dz[modes[a]*N + node] = omega * sum_b Dinv_ab(node) t_b(node), Dinv the
// symmetric inverse, its upper triangle packed over the padded size mp
// (pair-major); t_b = t[(tmap ? tmap[b] : b)*N + node].  One thread per (node,
// output row a), 256 nodes per workgroup.  Every pair is read by two rows (a
// and b); to give the second read a chance in L2 (measured on 256x256 with
// one split of 84 modes: about a quarter of them avoid memory):
//  - row a takes its pairs in the order b = (s - a) mod mm, s = 0, 1, ...,
//    so rows a and b read pair {a, b} at the same step s;
//  - the rows of one node block run on one XCD, back to back: workgroups go
//    to the XCDs in turn (id mod 8), and the r-th workgroup of XCD x takes
//    node block 8 (r / mm) + x, row r mod mm (the node blocks padded to a
//    multiple of 8; the padding's workgroups have no nodes).
__global__ __launch_bounds__(256) void mg_block_kernel(const double* __restrict__ Dinv, int mm, int mp,
                                                       const double* __restrict__ t,
                                                       const int* __restrict__ tmap,
                                                       const int* __restrict__ modes, double omega,
                                                       double* __restrict__ dz, int64_t N) {
  const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
  const int a = r % mm, nb = 8 * (r / mm) + x;
  const int64_t node = (int64_t)nb * 256 + threadIdx.x;
  // the input map in LDS (splits hold at most kMgMaxSplit modes), so that a
  // group's input rows are known without a wait per step
  __shared__ int smap[kMgMaxSplit];
  for (int i = threadIdx.x; i < mm; i += blockDim.x) smap[i] = tmap ? tmap[i] : i;
  __syncthreads();
  if (node >= N) return;
  auto pair = [&](int bb) {
    const int lo = min(a, bb), hi = max(a, bb);
    return (int64_t)lo * mp - (int64_t)lo * (lo - 1) / 2 + (hi - lo);
  };
  // steps in groups of kU: the group's map entries, pairs and inputs are all
  // requested before the first product, so a wavefront waits once per group
  // (even steps add into acc0, odd ones into acc1, as one step at a time)
  constexpr int kU = 8;
  double acc0 = 0.0, acc1 = 0.0;
  int b = a == 0 ? 0 : mm - a;  // (0 - a) mod mm
  int st = 0;
  for (; st + kU <= mm; st += kU) {
    double dv[kU], tv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int bb = b + u < mm ? b + u : b + u - mm;
      tv[u] = t[(int64_t)smap[bb] * N + node];
      dv[u] = Dinv[pair(bb) * N + node];
    }
#pragma unroll
    for (int u = 0; u < kU; u += 2) {
      acc0 = fma(dv[u], tv[u], acc0);
      acc1 = fma(dv[u + 1], tv[u + 1], acc1);
    }
    b = b + kU < mm ? b + kU : b + kU - mm;
  }
  for (; st < mm; ++st) {
    const double tb = t[(int64_t)smap[b] * N + node];
    if (st & 1) acc1 = fma(Dinv[pair(b) * N + node], tb, acc1);
    else acc0 = fma(Dinv[pair(b) * N + node], tb, acc0);
    if (++b == mm) b = 0;
  }
  dz[(int64_t)modes[a] * N + node] = omega * (acc0 + acc1);
}

// rc = R rf, R = P^T of bilinear interpolation: each interior coarse node
// gathers its fine counterpart (weight 1), the four edge neighbours (1/2) and
// the four diagonal neighbours (1/4); all nine are interior fine nodes
__global__ void mg_restrict_kernel(const double* __restrict__ rf, double* __restrict__ rc, int nf,
                                   int64_t Nc, int64_t Nf) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mode = blockIdx.y;
  if (c >= Nc) return;
  const int mc = nf / 2 - 1, mf = nf - 1;
  const int X = (int)(c % mc) + 1, Y = (int)(c / mc) + 1;
  const double* r = rf + (int64_t)mode * Nf;
  double acc = 0.0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    const double wy = dy ? 0.5 : 1.0;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const double w = wy * (dx ? 0.5 : 1.0);
      acc = fma(w, r[(int64_t)(2 * Y + dy - 1) * mf + (2 * X + dx - 1)], acc);
    }
  }
  rc[(int64_t)mode * Nc + c] = acc;
}

// zf += P zc: bilinear interpolation of the coarse interior values (boundary
// values zero)
__global__ void mg_prolong_add_kernel(const double* __restrict__ zc, double* __restrict__ zf,
                                      int nf, int64_t Nc, int64_t Nf) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mode = blockIdx.y;
  if (f >= Nf) return;
  const int mc = nf / 2 - 1, mf = nf - 1;
  const int fx = (int)(f % mf) + 1, fy = (int)(f / mf) + 1;
  const double* z = zc + (int64_t)mode * Nc;
  // 1D stencils: even fine index -> one coarse node, odd -> its two neighbours
  int xs[2], ys[2];
  double wx[2], wy[2];
  int nx, ny;
  if (fx & 1) { xs[0] = (fx - 1) / 2; xs[1] = (fx + 1) / 2; wx[0] = wx[1] = 0.5; nx = 2; }
  else { xs[0] = fx / 2; wx[0] = 1.0; nx = 1; }
  if (fy & 1) { ys[0] = (fy - 1) / 2; ys[1] = (fy + 1) / 2; wy[0] = wy[1] = 0.5; ny = 2; }
  else { ys[0] = fy / 2; wy[0] = 1.0; ny = 1; }
  double acc = 0.0;
  for (int b = 0; b < ny; ++b) {
    if (ys[b] < 1 || ys[b] > mc) continue;
    for (int a = 0; a < nx; ++a) {
      if (xs[a] < 1 || xs[a] > mc) continue;
      acc = fma(wy[b] * wx[a], z[(int64_t)(ys[b] - 1) * mc + (xs[a] - 1)], acc);
    }
  }
  zf[(int64_t)mode * Nf + f] += acc;
}

// x = C b, C column-major Nc x Nc (the coarsest level's inverse): a
// workgroup takes 64 rows, its 16 wavefronts split the columns, partial sums
// meet in LDS in a fixed order
constexpr int kDenseSplit = 16;
__global__ __launch_bounds__(64 * kDenseSplit) void mg_dense_kernel(const double* __restrict__ C,
                                                                   const double* __restrict__ b,
                                                                   double* __restrict__ x, int Nc) {
  __shared__ double part[kDenseSplit][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int per = (Nc + kDenseSplit - 1) / kDenseSplit;
  const int j0 = w * per, j1 = min(Nc, j0 + per);
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  if (i < Nc) {
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      acc0 = fma(C[(int64_t)j * Nc + i], b[j], acc0);
      acc1 = fma(C[(int64_t)(j + 1) * Nc + i], b[j + 1], acc1);
      acc2 = fma(C[(int64_t)(j + 2) * Nc + i], b[j + 2], acc2);
      acc3 = fma(C[(int64_t)(j + 3) * Nc + i], b[j + 3], acc3);
    }
    for (; j < j1; ++j) acc0 = fma(C[(int64_t)j * Nc + i], b[j], acc0);
  }
  part[w][lane] = (acc0 + acc1) + (acc2 + acc3);
  __syncthreads();
  if (w == 0 && i < Nc) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kDenseSplit; ++k) s += part[k][lane];
    x[i] = s;
  }
}

__global__ void mg_unit_kernel(double* __restrict__ u, int64_t n, int64_t idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[i] = (i == idx) ? 1.0 : 0.0;
}

__global__ void mg_axpy_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

}  // namespace

void launch_mg_mark(hipStream_t s, double* u, int n, int colour, double val) {
  const int64_t N = (int64_t)(n - 1) * (n - 1);
  hipLaunchKernelGGL(mg_mark_kernel, dim3(mg_cdiv(N, 256)), dim3(256), 0, s, u, n - 1, colour, val, N);
}

void launch_mg_gather(hipStream_t s, const double* W, int n, int colour, const int* modes, int mm,
                      int b, double* D) {
  const int64_t N = (int64_t)(n - 1) * (n - 1);
  hipLaunchKernelGGL(mg_gather_kernel, dim3(mg_cdiv(N, 256), mm), dim3(256), 0, s, W, n - 1, colour,
                     modes, mm, b, D, N);
}

int mg_block_pad(int mm) {
  for (int mp : {16, 32, 35, 48, 56, 64, 70, 84, 96, 128})
    if (mm <= mp) return mp;
  return 0;
}

size_t mg_block_doubles(int mm) {
  const size_t mp = (size_t)mg_block_pad(mm);
  return std::max((size_t)mm * mm, mp * (mp + 1) / 2);
}

void launch_mg_invert(hipStream_t s, double* D, int mm, int64_t N) {
  const int mp = mg_block_pad(mm);
  const int threads = std::max(64, mp);
  switch (mp) {
#define SG_MG_INV(MP)                                                                        \
  case MP:                                                                                   \
    hipLaunchKernelGGL(mg_invert_kernel<MP>, dim3((unsigned)N), dim3(threads), 0, s, D, mm, N); \
    return;
    SG_MG_INV(16) SG_MG_INV(32) SG_MG_INV(35) SG_MG_INV(48) SG_MG_INV(56) SG_MG_INV(64)
    SG_MG_INV(70) SG_MG_INV(84) SG_MG_INV(96) SG_MG_INV(128)
#undef SG_MG_INV
    default:
      throw Error(SG_ERR_UNSUPPORTED, "full-system multigrid: a split of more than 128 modes");
  }
}

void launch_mg_block(hipStream_t s, const double* Dinv, int mm, int64_t N, const double* t,
                     const int* tmap, const int* modes, double omega, double* dz) {
  if (mm < 1 || mm > kMgMaxSplit)
    throw Error(SG_ERR_UNSUPPORTED, "full-system multigrid: a split of more than 128 modes");
  const int64_t nblk8 = (mg_cdiv(N, 256) + 7) / 8 * 8;
  hipLaunchKernelGGL(mg_block_kernel, dim3((unsigned)(mm * nblk8)), dim3(256), 0, s, Dinv, mm,
                     mg_block_pad(mm), t, tmap, modes, omega, dz, N);
}

void launch_mg_restrict(hipStream_t s, const double* rf, double* rc, int nf, int P) {
  const int64_t Nf = (int64_t)(nf - 1) * (nf - 1), Nc = (int64_t)(nf / 2 - 1) * (nf / 2 - 1);
  hipLaunchKernelGGL(mg_restrict_kernel, dim3(mg_cdiv(Nc, 256), P), dim3(256), 0, s, rf, rc, nf, Nc, Nf);
}

void launch_mg_prolong_add(hipStream_t s, const double* zc, double* zf, int nf, int P) {
  const int64_t Nf = (int64_t)(nf - 1) * (nf - 1), Nc = (int64_t)(nf / 2 - 1) * (nf / 2 - 1);
  hipLaunchKernelGGL(mg_prolong_add_kernel, dim3(mg_cdiv(Nf, 256), P), dim3(256), 0, s, zc, zf, nf,
                     Nc, Nf);
}

void launch_mg_dense(hipStream_t s, const double* C, const double* b, double* x, int Nc) {
  hipLaunchKernelGGL(mg_dense_kernel, dim3(mg_cdiv(Nc, 64)), dim3(64 * kDenseSplit), 0, s, C, b, x,
                     Nc);
}

void launch_mg_unit(hipStream_t s, double* u, int64_t n, int64_t idx) {
  hipLaunchKernelGGL(mg_unit_kernel, dim3(mg_cdiv(n, 256)), dim3(256), 0, s, u, n, idx);
}

void launch_mg_axpy(hipStream_t s, const double* x, double* y, int64_t n) {
  hipLaunchKernelGGL(mg_axpy_kernel, dim3(mg_cdiv(n, 256)), dim3(256), 0, s, x, y, n);
}

}  // namespace sg
