// Internal declarations shared by the host set-up, the ABI layer and the HIP
// kernels of the stochastic-Galerkin solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sg.h"

namespace sg {

// ---- fixed geometry of the apply kernel -----------------------------------
// Elements are processed in 4x4 tiles: 16 elements, 64 Gauss points, one
// point per lane of a 64-wide wavefront.  Coefficient modes are stored
// tile-major so that a tile's 64 values of one mode are 512 contiguous bytes.
constexpr int kTileE = 4;            // elements per tile side
constexpr int kTileQ = 64;           // Gauss points per tile
constexpr int kApplyWaves = 4;       // wavefronts per apply workgroup
constexpr int kEdgeVals = 9;         // right edge 4, top edge 4, corner 1
constexpr int kMaxP = 256;
constexpr int kMaxRestart = 200;
constexpr int kCoarseN = 16;  // levels with n <= kCoarseN run in one LDS kernel
constexpr int kDenseSlices = 4;  // inner-index slices of the dense operator below the finest level
constexpr int kDenseN = 32;   // levels with n <= kDenseN: V-cycle applied as a dense operator
constexpr int kMaxCoarseLevels = 8;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ---- host set-up (sg_host.cpp) ---------------------------------------------
std::vector<std::vector<int>> total_degree_set(int M, int p);
double hermite_triple(int a, int b, int c);

struct Triple { int k, i, j; double v; };
std::vector<Triple> triple_list(const std::vector<std::vector<int>>& Jp,
                                const std::vector<std::vector<int>>& Jq);

struct KL {
  std::vector<double> lam;               // M eigenvalues (with sigma^2)
  std::vector<std::pair<int, int>> pairs;
  std::vector<double> gq;                // M x Nq, canonical q order
  std::vector<std::vector<double>> e1;   // 1D eigenvectors (n+1 nodal values) of the pairs' factors
};
KL karhunen_loeve(int n, int cov, double corr_len, double sigma, int M);

std::vector<std::vector<int>> make_splits(const std::vector<std::vector<int>>& J, int grouping);

// canonical Gauss point index q = 4e + 2qy + qx  ->  tile-major index
__host__ __device__ inline int64_t tiled_q(int n, int ex, int ey, int qx, int qy) {
  int nt = n / kTileE;
  int64_t t = (int64_t)(ey / kTileE) * nt + (ex / kTileE);
  int el = (ey % kTileE) * kTileE + (ex % kTileE);
  return t * kTileQ + el * 4 + qy * 2 + qx;
}

// Workgroup index -> tile index for one-tile-per-workgroup launches: the
// hardware deals workgroups round-robin over the 8 XCDs (each with its own
// L2), so consecutive workgroup ids are spread to give every XCD a contiguous
// band of tiles, whose shared halo rows then stay in that XCD's L2.
__host__ __device__ inline int xcd_tile(int wg, int ntiles) {
  if (ntiles % 8) return wg;
  return (wg & 7) * (ntiles >> 3) + (wg >> 3);
}

// ---- device-side descriptors -----------------------------------------------
// A row set of the operator: output modes `rows`, their nonzero triple
// products bucketed by coefficient-mode chunk, and the input columns whose
// gradients are needed.
// one nonzero triple product of a row: (k - chunk base) | (column slot << 16), value
struct alignas(16) Entry {
  int kj;
  int pad;
  double v;
};
constexpr int kEntryUnroll = 4;  // row segments are padded to this many entries
constexpr int kMaxChunk = 64;    // coefficient modes staged per chunk at most

struct RowSetHost {
  int nrows = 0, ncols = 0, rmax = 0, maxent = 0;
  int kc = 0, nchunk = 0, npass = 1, maxcols = 0;
  std::vector<int> rows;        // mode index of each output row
  std::vector<int> cols;        // mode index of each gradient column, pass by pass
  std::vector<int> cpass;       // npass + 1 column offsets of the passes
  std::vector<int> wrows;       // kApplyWaves x rmax, row slot per wave (-1 pad)
  std::vector<int> ptr;         // npass x nchunk x (nrows+1): row segments
  std::vector<Entry> ent;       // zero-valued padding entries point at (0, 0)
};

struct RowSetDev {
  int nrows, ncols, rmax, maxent;
  int kc, nchunk, npass, maxcols;
  const int* rows;
  const int* cols;
  const int* cpass;
  const int* wrows;
  const int* ptr;
  const Entry* ent;
};

// Factored apply (exact when q >= 2p): sum_k a_k(x) G_k = a_min I + w(x) T T^T with
// w = exp(mu + |g|^2 / 2) and T_{alpha,gamma} = (s_alpha / s_gamma) g^delta / delta!,
// delta = alpha - gamma >= 0, s_alpha = prod_n sqrt(alpha_n!).  With scaled
// gradients G^_alpha = s_alpha grad U_alpha and scaled monomials m_delta = g^delta / delta!:
//   step 1: Vbar_gamma = (1 / s_gamma^2) sum_alpha m_(alpha-gamma) G^_alpha  (column modes),
//   step 2: flux_beta  = s_beta w sum_gamma m_(beta-gamma) Vbar_gamma + (a_min / s_beta) G^_beta.
// All tables of a row set live in one int32 blob (staged in LDS by every tile); the
// o_* fields are word offsets into it, the o_cs.. fields point at FP64 values.
// Records are (slot | monomial << 16); padding records name monomial nmono, a row
// of zeros.
struct FRowSetDev {
  int nrows, ncols, ngam;  // output rows, input columns, intermediate gamma slots
  int qb, rmax;            // Gauss points per sub-batch (8/16/32/64), row slots per row group
  int nmono, pdeg, M;      // monomials (= |J(p)|), chaos degree p, KL terms
  int nblob;               // int32 words of the blob
  int o_r1, o_r2;          // int2 [groups][rmax]: (row slot or -1, first | end << 16) in
                           // units of 4 records; step 1 rows are gamma slots, step 2 output rows
  int o_e1, o_e2;          // records (16-byte aligned, row segments padded to 4)
  int o_dcol;              // [nrows] column slot of the output mode, or -1
  int o_cols, o_rows;      // input / output mode ids
  int o_mpar, o_mvar, o_mdeg;  // monomial recursion: parent, KL variable, first of each degree
  int o_cs, o_gs, o_rs, o_ra, o_minv;  // FP64: s_col, 1/s_gam^2, s_row, 1/s_row, 1/delta_var
  const int* blob;
};

// Rows of the register-resident factored apply: column modes, output modes
// and the intermediate gamma set as bit masks over J(p); slot[beta] is the
// output slot of mode beta (compact output layout; 0xFF: not an output row),
// mode[slot] its mode id.
constexpr int kRMax = 256;            // modes of the register-resident apply
constexpr int kRMaskW = kRMax / 64;   // mask words
constexpr int kRSmall = 35;  // ... whose gradients and monomials all stay in registers
struct RApplyRows {
  uint64_t colmask[kRMaskW], rowmask[kRMaskW];
  uint64_t gammask[kRMaskW];  // gamma <= some column and <= some output row (step-1 rows that matter)
  int nrows;
  unsigned char slot[kRMax];
  unsigned char mode[kRMax];
};
static_assert(offsetof(RApplyRows, slot) % 4 == 0, "slot table read as 32-bit words");
__host__ __device__ inline bool rbit(const uint64_t (&m)[kRMaskW], int i) {
  return ((m[i >> 6] >> (i & 63)) & 1) != 0;
}
__host__ inline void rset(uint64_t (&m)[kRMaskW], int i) { m[i >> 6] |= uint64_t(1) << (i & 63); }

struct Level {
  int n;          // elements per side on this level
  int64_t N;      // (n-1)^2
  double* S;      // 9 x N stencil
};

// launch wrappers (sg_kernels.hip)
void launch_coeff(hipStream_t s, int n, int M, int na, const double* g, const int* Jq,
                  const double* inv_sqrt_fact, double mu, double a_min, double* a);
void launch_fine_stencil(hipStream_t s, int n, const double* a0, double* S);
void launch_rap(hipStream_t s, int nf, const double* Sf, double* Sc);
void launch_rhs(hipStream_t s, int n, const double* f_nodal, double* F, int64_t total);
// Edge sums of a tile-based operator apply not yet added to its output
// (edge null: none pending).  A tile owns its 4 x 4 lower-left nodes; its
// right/top edge and corner sums (kEdgeVals per tile and output vector) belong
// to the neighbouring tiles' nodes.  The apply kernels either add them in a
// fixup kernel or leave them to the kernel that reads the output next, which
// adds them for output vector slot at interior node (gx, gy) (1-based) in the
// fixup kernel's order, so both give the same bits.
struct EdgeFix {
  const double* edge = nullptr;
  int nt = 0;         // tiles per side
  double sgn = 1.0;   // sign the sums enter the output with
  int64_t Nh = 0;     // vector length (node count) of one output vector
  int m = 0;          // interior nodes per side
  uint64_t rNh = 0;   // recip64(Nh) and recip64(m), for w_fixed's divisions
  uint64_t rm = 0;
};

// ceil(2^64 / d) for 2 <= d < 2^32 (2^(64 - t) when d = 2^t): with it the high
// 64 bits of x * recip64(d) equal x / d for every x < 2^32 (with
// recip64(d) d = 2^64 + e, 0 <= e < d, the product overshoots x / d by
// x e / (d 2^64) < 1 / d, too little to reach the next integer)
inline uint64_t recip64(uint64_t d) { return ~uint64_t(0) / d + 1; }

__device__ __forceinline__ double edge_fixed(double v, const EdgeFix& f, int slot, int gx, int gy) {
  const int nx = gx & 3, ny = gy & 3;
  if (nx && ny) return v;
  const int nt = f.nt, tile = (gy >> 2) * nt + (gx >> 2);
  const double* eb = f.edge + (int64_t)slot * nt * nt * kEdgeVals;
  if (nx == 0) v += f.sgn * eb[(int64_t)(tile - 1) * kEdgeVals + ny];
  if (ny == 0) v += f.sgn * eb[(int64_t)(tile - nt) * kEdgeVals + 4 + nx];
  if (nx == 0 && ny == 0) v += f.sgn * eb[(int64_t)(tile - nt - 1) * kEdgeVals + 8];
  return v;
}

// element i of a vector of output vectors (vector i / Nh, node i % Nh) with
// its pending edge sums added; i < P N_h < 2^32 (P <= 256, N_h < 4096^2)
__device__ __forceinline__ double w_fixed(const double* __restrict__ w, int64_t i, const EdgeFix& f) {
  double v = w[i];
  if (f.edge) {
    const uint64_t ii = (uint64_t)i;
    const uint64_t slot = __umul64hi(ii, f.rNh), node = ii - slot * (uint64_t)f.Nh;
    const uint64_t gy = __umul64hi(node, f.rm), gx = node - gy * (uint64_t)f.m;
    v = edge_fixed(v, f, (int)slot, (int)gx + 1, (int)gy + 1);
  }
  return v;
}

// The apply launchers end with the edge fixup unless fixup is false (the
// caller then hands the pending sums to the next reader as an EdgeFix).
void launch_apply(hipStream_t s, int n, int na, const double* a, const RowSetDev& rs,
                  const double* U, int64_t Nh, const double* rin, double beta, double sgn,
                  double* out, double* edge, bool fixup = true);
size_t apply_lds_bytes(int maxcols, int kc, int maxent);
constexpr int kDenseK = 1024;  // padded inner index of the dense coarse operator (>= 31^2)
void launch_dense_coarse(hipStream_t s, int N, int m, const double* C, const double* B, double* X,
                         const int* bmap = nullptr, const int* xmap = nullptr, int slices = 1);
void launch_unit_columns(hipStream_t s, int N, int j0, int m, double* out);
bool rapply_supported(int M, int p);
bool rapply_matches(int M, int p, const std::vector<std::vector<int>>& Jp);
// kv > 0: rr is block kv of the field split by first KL variable (rows the modes
// whose first variable is kv, columns those below it; checked by the caller),
// which a kernel with that block's pairs compiled in serves
void launch_rapply(hipStream_t s, int M, int p, int n, double mu, double a_min, const double* g,
                   const RApplyRows& rr, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge, bool fixup = true,
                   int kv = 0);
void launch_apply_fixup(hipStream_t s, int n, int nrows, double sgn, const double* edge,
                        double* out, int64_t Nh);
size_t fapply_lds_bytes(int qb, int nrows, int ncols, int ngam, int nmono, int M, int nblob);
void launch_fapply(hipStream_t s, int n, double mu, double a_min, const double* g,
                   const FRowSetDev& rs, const double* U, int64_t Nh, const double* rin,
                   double beta, double sgn, double* out, double* edge, bool fixup = true);
void launch_zero(hipStream_t s, double* x, int64_t n);
void launch_gather_modes(hipStream_t s, int m, const int* modes, int64_t Nh, const double* src,
                         double* dst);
void launch_scatter_modes(hipStream_t s, int m, const int* modes, int64_t Nh, const double* src,
                          double* dst);
// fused multigrid
struct CoarseLevels {
  int nl;
  int n[kMaxCoarseLevels];
  int64_t N[kMaxCoarseLevels];
  const double* S[kMaxCoarseLevels];
};
void launch_vdown(hipStream_t s, const Level& Lf, const Level& Lc, int modes, const int* smode,
                  const double* b, double* x2, double* bc, double omega,
                  const int* bmap = nullptr, const EdgeFix& ef = EdgeFix{});
void launch_vup(hipStream_t s, const Level& Lf, const Level& Lc, int modes, const int* smode,
                const double* b, const double* x2, const double* xc, double* x, double omega,
                const int* bmap = nullptr, const int* xmap = nullptr, int xc_slices = 1,
                const EdgeFix& ef = EdgeFix{});
// Levels l and l+1 of the cycle in one kernel each way (mean stiffness,
// L0.n a multiple of 4; L1, L2 the next two levels), used where
// two_level_pays(L2, modes).  down writes level l's
// pre-smoothed x2_0, level l+1's right-hand side b1 and pre-smoothed x2_1, and
// level l+2's right-hand side b2; up reads those and level l+2's correction
// (xc_slices partial results) and writes level l's corrected x.
bool two_level_pays(const Level& L2, int modes);
void launch_vdown2(hipStream_t s, const Level& L0, const Level& L1, const Level& L2, int modes,
                   const double* b, double* x2_0, double* b1, double* x2_1, double* b2,
                   double omega, const int* bmap = nullptr, const EdgeFix& ef = EdgeFix{});
void launch_vup2(hipStream_t s, const Level& L0, const Level& L1, const Level& L2, int modes,
                 const double* b, const double* x2_0, const double* b1, const double* x2_1,
                 const double* xc2, int xc_slices, double* x, double omega,
                 const int* bmap = nullptr, const int* xmap = nullptr,
                 const EdgeFix& ef = EdgeFix{});
void launch_vcoarse(hipStream_t s, const CoarseLevels& cl, int modes, const int* smode,
                    const double* b, double* x, double omega);
size_t vcoarse_lds_bytes(const CoarseLevels& cl);
void launch_diag_coeff(hipStream_t s, int n, int cnt, const int* ks, const double* vs,
                       const double* a, double* c);
// Krylov helpers
int dot_blocks(int64_t N);
void launch_multidot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* w,
                     int64_t N, double* partial, int nblk);
void launch_reduce(hipStream_t s, const double* partial, int nblk, int nv, double* out);
void launch_update(hipStream_t s, const double* V, int64_t ldv, int nv, const double* h,
                   double* w, int64_t N, double sign);
// Gram-Schmidt passes (one element per thread, partial sized nv * gs_blocks(N));
// each ends with the reduction into out[0..nv) (out[0] for the norm)
int gs_blocks(int64_t N);
// (ef: pending edge sums of the apply that wrote w, added as w is read)
void launch_gs_dot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                   double* partial, double* out, const EdgeFix& ef = EdgeFix{});
void launch_gs_update_dot(hipStream_t s, const double* V, int64_t ldv, int nv, const double* h,
                          double* w, int64_t N, double sign, double* partial, double* out,
                          const EdgeFix& ef = EdgeFix{});
// w <- w + sign V h, |w|^2 -> *nrm2 and vnext = w / |w| (zero when |w| = 0)
void launch_gs_update_norm_scale(hipStream_t s, const double* V, int64_t ldv, int nv,
                                 const double* h, double* w, int64_t N, double sign,
                                 double* partial, double* nrm2, double* vnext);
// Gram-Schmidt with the second projection delayed by one step: pass A
// (out = Q^T u, Q^T w, u.u, u.w, w.w over nv basis vectors; without w:
// Q^T u, u.u), its coefficients (nu, c_j, rho, raw |w - Q c|^2), pass B
// (q_j in place of u_j, u_{j+1}); partial sized gs2_partial_doubles(nv, N)
int gs2_dot_slots(int nv, bool with_w);
size_t gs2_partial_doubles(int max_nv, int64_t N);
void launch_gs2_dot(hipStream_t s, const double* Q, int64_t ldq, int nv, const double* u,
                    const double* w, int64_t N, double* partial, double* out,
                    const EdgeFix& ef = EdgeFix{});
void launch_gs2_coef(hipStream_t s, int nv, const double* dots, double* coef);
void launch_gs2_update(hipStream_t s, const double* Q, int64_t ldq, int nv, const double* sv,
                       const double* tv, const double* coef, double* uq, const double* w,
                       double* unext, int64_t N, const EdgeFix& ef = EdgeFix{});
void launch_combine(hipStream_t s, const double* V, int64_t ldv, int nv, const double* y,
                    double* out, int64_t N);
void launch_scale_by_inv_norm(hipStream_t s, const double* w, const double* nrm2, double* v,
                              int64_t N);
void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, int64_t N);
void launch_sub(hipStream_t s, const double* a, const double* b, double* out, int64_t N);
void launch_stencil_residual(hipStream_t s, int n, const double* S, const int* smode, int m,
                             const double* b, const double* x, double* out);
void launch_stage_alpha(hipStream_t s, double* dots, const double* c, const double* kc, double* z,
                        double* w, int64_t N);
// multigrid on the full SG system (sg_mg.hip)
void launch_mg_mark(hipStream_t s, double* u, int n, int colour, double val);
void launch_mg_gather(hipStream_t s, const double* W, int n, int colour, const int* modes, int mm,
                      int b, double* D);
int mg_block_pad(int mm);  // padded block size of the inversion kernel, 0 if mm > 128
size_t mg_block_doubles(int mm);  // doubles per node of one split's block storage
void launch_mg_invert(hipStream_t s, double* D, int mm, int64_t N);
void launch_mg_block(hipStream_t s, const double* Dinv, int mm, int64_t N, const double* t,
                     const int* tmap, const int* modes, double omega, double* dz);
void launch_mg_restrict(hipStream_t s, const double* rf, double* rc, int nf, int P);
void launch_mg_prolong_add(hipStream_t s, const double* zc, double* zf, int nf, int P);
void launch_mg_dense(hipStream_t s, const double* C, const double* b, double* x, int Nc);
void launch_mg_axpy(hipStream_t s, const double* x, double* y, int64_t n);
void launch_mg_unit(hipStream_t s, double* u, int64_t n, int64_t idx);

// ---- batched solves (sg_batch.cpp, batched kernels in sg_kernels.hip) ------
constexpr int kMaxSplitsB = 12;
constexpr int kMaxLevelsB = 12;

// buffers a batched kernel can address by id (resolved per instance on device)
enum BufId { BUF_F = 0, BUF_U, BUF_VJ, BUF_VJ1, BUF_V0, BUF_W, BUF_Z, BUF_T, BUF_FST, BUF_FSX };

struct BInst {  // one instance of a batch, device-resident
  int n, P, na, nlev, nfine, nsplit, m, nblk;
  int64_t Nh, Nv;
  const double* a;
  RowSetDev full;
  RowSetDev part[kMaxSplitsB];
  int form;                        // apply: 0 triple products, 1 factored tiles, 2 factored registers
  int M, pdeg;
  double mu, amin;
  const double* gq;                // KL values at the Gauss points (tile order)
  FRowSetDev ffull, fpart[kMaxSplitsB];
  RApplyRows rfull, rpart[kMaxSplitsB];
  const int* split_idx[kMaxSplitsB];
  int split_m[kMaxSplitsB];
  Level L[kMaxLevelsB];
  double* mg_b[kMaxLevelsB];
  double* mg_x[kMaxLevelsB];
  double* mg_xa[kMaxLevelsB];
  double *edge, *fsT, *fsX;
  const double* F;
  double *u, *V, *w, *z, *t;
  double *partial, *H, *cs, *sn, *g, *y, *hv;  // hv: h1 (m+1), h2 (m+1), nrm
};

struct BState {  // per-instance solver state, device-resident
  int j, active, done, kdone, it, restarts, status, max_it;
  double beta, nF, est, target;
};

struct BItem {  // one work item (one workgroup) of a batched kernel
  int inst, local;
};

// device helpers of the batched kernels: gate test and buffer-id resolution
__device__ inline bool gated(const BState& S, int gate) {
  return gate == 0 ? (S.active == 0) : (S.done != 0);
}

// A pointer into device memory read from a descriptor table.  Such pointers
// are generic, so the compiler would access them with flat instructions, whose
// waits also cover LDS traffic; obtained this way (an integer to a
// global-address-space pointer, which no cast round trip folds away) the
// accesses through it are global loads and stores.
template <class T>
__device__ __forceinline__ T* gptr(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ inline double* bbuf(const BInst& I, const BState& S, int id) {
  switch (id) {
    case BUF_F: return gptr(const_cast<double*>(I.F));
    case BUF_U: return gptr(I.u);
    case BUF_VJ: return gptr(I.V + (int64_t)S.j * I.Nv);
    case BUF_VJ1: return gptr(I.V + (int64_t)(S.j + 1) * I.Nv);
    case BUF_V0: return gptr(I.V);
    case BUF_W: return gptr(I.w);
    case BUF_Z: return gptr(I.z);
    case BUF_T: return gptr(I.t);
    case BUF_FST: return gptr(I.fsT);
    default: return gptr(I.fsX);
  }
}


// gate: 0 = instances still in the current Arnoldi cycle, 1 = instances not done
constexpr int kVecChunk = 4096;     // elements per item of the batched vector kernels
void launch_bapply(hipStream_t s, int rmax, size_t lds, const BInst* I, const BState* st,
                   const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                   double beta, double sgn, int gate);
void launch_bfapply(hipStream_t s, int qb, size_t lds, const BInst* I, const BState* st,
                    const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                    double beta, double sgn, int gate);
void launch_brapply(hipStream_t s, int M, int p, size_t lds, const BInst* I, const BState* st,
                    const BItem* items, int nitems, int rowset, int src, int rin, int dst,
                    double beta, double sgn, int gate);
size_t rapply_lds_bytes(int P, int nrows);
void launch_bfixup(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                   int rowset, int dst, double sgn, int gate);
void launch_bvdown(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                   int depth, int split, int gate);
void launch_bvup(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                 int depth, int split, int gate);
void launch_bvcoarse(hipStream_t s, size_t lds, const BInst* I, const BState* st,
                     const BItem* items, int nitems, int split, int gate);
void launch_bgather(hipStream_t s, const BInst* I, const BState* st, const BItem* items,
                    int nitems, int split, int buf, int scatter, int gate);
void launch_bvec(hipStream_t s, const BInst* I, const BState* st, const BItem* items, int nitems,
                 int op, int x, int y, int out, double a, double b, int gate);
void launch_bmultidot(hipStream_t s, const BInst* I, const BState* st, const BItem* items,
                      int nitems, int self_buf, int gate);
void launch_breduce(hipStream_t s, const BInst* I, const BState* st, int count, int which,
                    int gate);
void launch_bgivens(hipStream_t s, const BInst* I, BState* st, int count);
void launch_bsolve(hipStream_t s, const BInst* I, const BState* st, int count);
void launch_binit(hipStream_t s, const BInst* I, BState* st, int count, int first, double tol);
enum BVecOp { BV_AXPBY = 0, BV_UPDATE1, BV_UPDATE2, BV_SCALE_NEXT, BV_COMBINE, BV_START };

// learned stage (sg_cnn.hip)
void cnn_apply_sg(sg_cnn* C, hipStream_t s, const double* v, double sigma, double* c,
                  double* scratch_partial, int nblk);
int cnn_modes(const sg_cnn* C);
int cnn_grid(const sg_cnn* C);
bool cnn_bound(const sg_cnn* C);

}  // namespace sg
