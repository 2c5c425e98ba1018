// C ABI of the SG solver: handle life cycle, workspace layout, operator and
// preconditioner applies, and the restarted GMRES driver.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <numeric>
#include <string>
#include <vector>

#include "sg_internal.h"
#include "sg_learned.h"
#include "sg_q2.h"

using namespace sg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define SG_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw Error(SG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

constexpr double kOmega = 8.0 / 9.0;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Host plan of a factored row set (see FRowSetDev): gamma slots, the two
// record lists, the rows of every row group, and the packed table blob.
struct FRowSetHost {
  int nrows = 0, ncols = 0, ngam = 0, qb = 0, rmax = 0;
  std::vector<int> rows, cols, gam, l1, l2, dcol, p1, p2, e1, e2;
  std::vector<int> blob;
  FRowSetDev off{};  // sizes and blob offsets (pointer filled at bind)
};

// capacity of the per-group row tables (groups * rmax <= kMaxP + 32 for every plan)
constexpr int kFGroupCap = kMaxP + 32;

struct FSHost {
  std::vector<std::vector<int>> splits;
  std::vector<RowSetHost> partial;    // partial[s] for s >= 1 (index 0 unused)
  std::vector<FRowSetHost> fpartial;  // the same blocks in factored form
  std::vector<std::vector<int>> sid;  // stencil ids (mode + 1) of each split
};

struct FSDev {
  std::vector<int*> split_idx;
  std::vector<int*> split_sid;   // stencil id (mode + 1) of every mode of a split
  std::vector<RowSetDev> partial;
  std::vector<FRowSetDev> fpartial;
};

// every device pointer inside the bound workspace
struct DevPtrs {
  double *a = nullptr, *g = nullptr, *isf = nullptr, *f = nullptr;
  int* Jq = nullptr;
  std::vector<Level> L;
  RowSetDev full{};
  FRowSetDev ffull{};
  FSDev fs[SG_GROUP_COUNT];
  double* edge = nullptr;
  std::vector<double*> mg_b, mg_x, mg_xa, mg_r;
  double *fsT = nullptr, *fsX = nullptr;
  double *fsR = nullptr, *fsD = nullptr;  // inner iterations of the diagonal blocks
  int* all_sid = nullptr;        // mode + 1 for every mode
  int* diag_k = nullptr;         // (k, v) lists of the diagonal blocks
  double* diag_v = nullptr;
  double* cdiag = nullptr;       // one coefficient field (set-up scratch)
  double* Cd = nullptr;          // dense coarse V-cycle operator, N x N column-major
  double* stage = nullptr;       // learned stage of sg_precond_apply: dot partials, 4 scalars
  // biquadratic handles: KL values at the Q2 Gauss points, the apply's two
  // per-point buffers, and the translation-matrix lists
  double *q2g = nullptr, *q2grad = nullptr, *q2y = nullptr;
  Q2TDev q2t{};
};

// bump allocator over the caller's workspace (or a dry run to size it)
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align256(count * sizeof(T));
    return p;
  }
};

}  // namespace

// Multigrid on the full SG system (sg_mg_bind): per level its grid, KL values
// and coefficient modes at its Gauss points and edge buffer (level 0: the
// handle's own), right-hand side and correction (level 0: the caller's), work
// vectors, and the inverted nodal blocks of every split; the coarsest level's
// dense inverse.
struct MGLevel {
  int n = 0;
  int64_t N = 0;
  double *g = nullptr, *a = nullptr, *edge = nullptr, *b = nullptr, *z = nullptr;
  double *res = nullptr, *dz = nullptr, *t = nullptr;
  std::vector<double*> Dinv;
};
struct MGState {
  bool bound = false;
  int grouping = -1;
  std::vector<MGLevel> L;
  double* Cinv = nullptr;  // coarsest level: K^{-1}, column-major Nc x Nc
  int Nc = 0;
};

struct sg_handle {
  sg_problem prob{};
  int n = 0, M = 0, P = 0, na = 0, nt = 0, ntiles = 0;
  int64_t Nh = 0, Nq = 0;
  std::vector<std::vector<int>> Jp, Jq;
  std::vector<Triple> G;
  KL kl;
  std::vector<double> f_nodal, g_tiled, isf;
  std::vector<int> Jq_flat;
  RowSetHost full;
  FRowSetHost ffull;
  std::vector<int> mpar, mvar, mdeg;  // monomial recursion over J(p)
  std::vector<double> minv, sfac;     // 1/delta_n of the recursion; s_alpha = prod sqrt(alpha_n!)
  bool factored_ok = false;           // q >= 2p: the factored apply is exact
  bool use_factored = false;          // apply form in use: factored ...
  bool use_rapply = false;            // ... in registers (else the LDS tile kernel)
  bool rapply_ok = false;             // register form compiled for (M, p) and P <= 64
  int fqb = 0;                        // forced sub-batch size (0: planner's choice)
  RApplyRows rfull{};                 // register-form rows: whole operator
  std::vector<RApplyRows> rpart[SG_GROUP_COUNT];  // and the field-split blocks (index 0 unused)
  std::vector<int> rkv[SG_GROUP_COUNT];         // block index of the first-variable split, else 0
  FSHost fs[SG_GROUP_COUNT];
  std::vector<int> level_n;
  std::vector<int> diag_ptr, diag_k, diag_sid;  // per mode i: [G_k]_{ii} != 0 entries
  std::vector<double> diag_v;
  int nfine = 0;                                // levels with n > kCoarseN
  int ldense = -1;                              // first level with n <= kDenseN
  bool dense_ready = false;                     // dense coarse operator built

  // device state
  bool bound = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  DevPtrs d;
  double* host_pinned = nullptr;  // small staging for Krylov scalars
  hipEvent_t fetched = nullptr;   // marks the Krylov scalars' copy to host_pinned
  sg_cnn* cnn = nullptr;          // attached learned stage (not owned)
  double cnn_sigma = 0.0;
  MGState mg;                     // full-system multigrid (sg_mg_bind)
  // biquadratic elements (sg_setup_q2): n2 elements per side; everything above
  // describes the Q1 operator of the refined grid (2 n2 elements per side,
  // the same nodes), which the preconditioners use
  bool q2 = false;
  int n2 = 0;
  int64_t Nq2 = 0;
  std::vector<double> q2g;                      // M x 9 n2^2 KL values
  std::vector<int> q2p1, q2i1, q2p2, q2i2;      // T by column, by row
  std::vector<double> q2c1, q2c2;
  std::vector<uint64_t> q2e1, q2e2;

  ~sg_handle() {
    if (host_pinned) (void)hipHostFree(host_pinned);
    if (fetched) (void)hipEventDestroy(fetched);
  }
};

namespace {

// Groups a row set's nonzero triple products by column pass and coefficient
// chunk of kc modes: pass-major, then chunk-major, and inside a chunk row by
// row, every row segment padded to kEntryUnroll entries.  Column slots are
// relative to the pass.  Returns the largest entry count of one (pass, chunk).
int layout_entries(const sg_handle& H, RowSetHost& rs, int kc, const std::vector<int>& rslot,
                   const std::vector<int>& cslot) {
  const int nchunk = (H.na + kc - 1) / kc;
  const int np = rs.npass;
  std::vector<int> cpass_of(rs.ncols);
  for (int p = 0; p < np; ++p)
    for (int c = rs.cpass[p]; c < rs.cpass[p + 1]; ++c) cpass_of[c] = p;
  std::vector<std::vector<std::vector<std::pair<int, double>>>> bucket(
      (size_t)np * nchunk, std::vector<std::vector<std::pair<int, double>>>(rs.nrows));
  for (const Triple& tr : H.G) {
    int r = rslot[tr.i], c = cslot[tr.j];
    if (r < 0 || c < 0) continue;
    const int p = cpass_of[c];
    const int ch = tr.k / kc;
    bucket[(size_t)p * nchunk + ch][r].push_back({(tr.k - ch * kc) | ((c - rs.cpass[p]) << 16), tr.v});
  }
  rs.ent.clear();
  rs.ptr.assign((size_t)np * nchunk * (rs.nrows + 1), 0);
  int maxent = 0;
  for (int pc = 0; pc < np * nchunk; ++pc) {
    const int base = (int)rs.ent.size();
    for (int r = 0; r < rs.nrows; ++r) {
      rs.ptr[(size_t)pc * (rs.nrows + 1) + r] = (int)rs.ent.size();
      for (auto& e : bucket[pc][r]) rs.ent.push_back(Entry{e.first, 0, e.second});
      while (rs.ent.size() % kEntryUnroll) rs.ent.push_back(Entry{0, 0, 0.0});
    }
    rs.ptr[(size_t)pc * (rs.nrows + 1) + rs.nrows] = (int)rs.ent.size();
    maxent = std::max(maxent, (int)rs.ent.size() - base);
  }
  return maxent;
}

RowSetHost build_rowset(const sg_handle& H, const std::vector<int>& rows,
                        const std::vector<int>& cols, int force_kc = 0) {
  RowSetHost rs;
  rs.rows = rows;
  rs.cols = cols;
  rs.nrows = (int)rows.size();
  rs.ncols = (int)cols.size();
  std::vector<int> rslot(H.P, -1), cslot(H.P, -1);
  for (int t = 0; t < rs.nrows; ++t) rslot[rows[t]] = t;
  for (int t = 0; t < rs.ncols; ++t) cslot[cols[t]] = t;
  // kc: coefficient modes staged per chunk.  Prefer three workgroups per CU
  // (<= 53 KB of LDS) with chunks of >= 32 modes, then two, then one; when the
  // gradients of all columns do not fit, split the columns into passes.
  const int cands[] = {64, 48, 32, 24, 16, 12, 8, 6, 4, 3, 2, 1};
  static_assert(kMaxChunk == 64, "candidate list starts at kMaxChunk");
  const struct { size_t budget; int minkc; } tiers[] = {{53 * 1024, 32}, {80 * 1024, 16},
                                                         {160 * 1024, 1}};
  int kc = 0;
  for (int np = 1; np <= 8 && !kc; ++np) {
    rs.npass = np;
    rs.cpass.assign(np + 1, 0);
    for (int p = 0; p <= np; ++p) rs.cpass[p] = (int)((int64_t)rs.ncols * p / np);
    rs.maxcols = 1;
    for (int p = 0; p < np; ++p) rs.maxcols = std::max(rs.maxcols, rs.cpass[p + 1] - rs.cpass[p]);
    for (auto& tier : tiers) {
      if (np > 1 && tier.budget < 160 * 1024) continue;
      for (int c : cands) {
        if (force_kc > 0 && c != force_kc) continue;
        const int kcc = std::min(c, H.na);
        if (kcc < std::min(np > 1 ? 16 : tier.minkc, H.na)) break;
        const int maxent = layout_entries(H, rs, kcc, rslot, cslot);
        if (apply_lds_bytes(rs.maxcols, kcc, maxent) <= tier.budget) {
          kc = kcc;
          rs.maxent = maxent;
          break;
        }
      }
      if (kc) break;
    }
  }
  if (!kc)
    throw Error(SG_ERR_UNSUPPORTED, "apply: the gradients of " + std::to_string(rs.ncols) +
                                        " modes do not fit in LDS");
  const int nchunk = (H.na + kc - 1) / kc;
  rs.kc = kc;
  rs.nchunk = nchunk;
  std::vector<long> load(rs.nrows, 0);
  for (int pc = 0; pc < rs.npass * nchunk; ++pc)
    for (int r = 0; r < rs.nrows; ++r)
      load[r] += rs.ptr[(size_t)pc * (rs.nrows + 1) + r + 1] - rs.ptr[(size_t)pc * (rs.nrows + 1) + r];
  // rows to wavefronts: longest rows first onto the least loaded wavefront
  const int need = std::max(1, (rs.nrows + kApplyWaves - 1) / kApplyWaves);
  int rmax = 1;
  while (rmax < need) rmax *= 2;
  if (rmax > 64) throw Error(SG_ERR_UNSUPPORTED, "apply: too many rows per wavefront");
  rs.rmax = rmax;
  rs.wrows.assign((size_t)kApplyWaves * rmax, -1);
  std::vector<int> order(rs.nrows);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[a] > load[b]; });
  std::vector<long> wl(kApplyWaves, 0);
  std::vector<int> wc(kApplyWaves, 0);
  for (int r : order) {
    int best = -1;
    for (int w = 0; w < kApplyWaves; ++w)
      if (wc[w] < need && (best < 0 || wl[w] < wl[best])) best = w;
    rs.wrows[(size_t)best * rmax + wc[best]] = r;
    wc[best]++;
    wl[best] += load[r];
  }
  // one zero group past the end (reads of a padded group never leave the array)
  for (int u = 0; u < kEntryUnroll; ++u) rs.ent.push_back(Entry{0, 0, 0.0});
  return rs;
}

// Pairs gamma <= alpha (componentwise) of J(p) with the coefficient
// c_{alpha,gamma} = prod_n sqrt(alpha_n!/gamma_n!) / (alpha_n - gamma_n)! and the
// J(p) index of delta = alpha - gamma (the monomial g^delta).
struct TPair {
  int a, gm, d;
  double c;
};

std::vector<TPair> t_pairs(const sg_handle& H) {
  std::map<std::vector<int>, int> idx;
  for (int i = 0; i < H.P; ++i) idx[H.Jp[i]] = i;
  auto fact = [](int k) {
    double f = 1.0;
    for (int t = 2; t <= k; ++t) f *= t;
    return f;
  };
  std::vector<TPair> out;
  for (int a = 0; a < H.P; ++a) {
    const std::vector<int>& al = H.Jp[a];
    std::vector<int> gm(H.M, 0), de(H.M);
    for (;;) {
      double c = 1.0;
      for (int n = 0; n < H.M; ++n) {
        de[n] = al[n] - gm[n];
        c *= std::sqrt(fact(al[n]) / fact(gm[n])) / fact(de[n]);
      }
      out.push_back({a, idx.at(gm), idx.at(de), c});
      int n = 0;
      while (n < H.M && ++gm[n] > al[n]) gm[n++] = 0;
      if (n == H.M) break;
    }
  }
  return out;
}

// Monomial recursion over J(p): m_delta = m_(delta - e_n) g_n / delta_n with n
// the first nonzero index of delta, so m_delta = g^delta / delta!; mdeg[d] is
// the first index of degree d (J(p) is graded), padded with P up to index p + 2.
void monomial_tables(sg_handle& H) {
  std::map<std::vector<int>, int> idx;
  for (int i = 0; i < H.P; ++i) idx[H.Jp[i]] = i;
  const int p = H.prob.p;
  H.mpar.assign(H.P, 0);
  H.mvar.assign(H.P, 0);
  H.minv.assign(H.P, 1.0);
  H.mdeg.assign(p + 3, H.P);
  H.sfac.assign(H.P, 1.0);
  for (int i = H.P - 1; i >= 0; --i) {
    const std::vector<int>& d = H.Jp[i];
    const int deg = std::accumulate(d.begin(), d.end(), 0);
    H.mdeg[deg] = i;
    for (int e : d)
      for (int t = 2; t <= e; ++t) H.sfac[i] *= std::sqrt((double)t);
    if (deg == 0) continue;
    int n = 0;
    while (d[n] == 0) ++n;
    std::vector<int> par = d;
    par[n]--;
    H.mpar[i] = idx.at(par);
    H.mvar[i] = n;
    H.minv[i] = 1.0 / d[n];
  }
}

// record buckets -> CSR, every row segment padded to 4 records naming the zero
// monomial row `pad`
void layout_records(const std::vector<std::vector<int>>& b, int pad, std::vector<int>& ptr,
                    std::vector<int>& rec) {
  ptr.assign(b.size() + 1, 0);
  rec.clear();
  for (size_t r = 0; r < b.size(); ++r) {
    ptr[r] = (int)rec.size();
    for (int e : b[r]) rec.push_back(e);
    while (rec.size() % 4) rec.push_back(pad << 16);
  }
  ptr[b.size()] = (int)rec.size();
}

// rows of one step to row groups: longest first onto the least loaded group
// with a free slot
void assign_groups(const std::vector<int>& ptr, int groups, int rmax, std::vector<int>& lst) {
  const int cnt = (int)ptr.size() - 1;
  lst.assign((size_t)groups * rmax, -1);
  std::vector<int> order(cnt);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b];
  });
  std::vector<long> load(groups, 0);
  std::vector<int> used(groups, 0);
  for (int r : order) {
    int best = -1;
    for (int gi = 0; gi < groups; ++gi)
      if (used[gi] < rmax && (best < 0 || load[gi] < load[best])) best = gi;
    lst[(size_t)best * rmax + used[best]++] = r;
    load[best] += ptr[r + 1] - ptr[r];
  }
}

// Packs every table of the row set into one int32 blob (layout independent of
// the sub-batch plan: the group tables are reserved at kFGroupCap).
void pack_frowset(const sg_handle& H, FRowSetHost& f) {
  std::vector<int>& B = f.blob;
  B.clear();
  auto put = [&](const std::vector<int>& v, size_t cap, int align) {
    while (B.size() % align) B.push_back(0);
    const int o = (int)B.size();
    B.insert(B.end(), v.begin(), v.end());
    B.resize(o + std::max(cap, v.size()), -1);
    return o;
  };
  auto putd = [&](const std::vector<double>& v) {
    while (B.size() % 2) B.push_back(0);
    const int o = (int)B.size();
    B.resize(o + 2 * v.size());
    if (!v.empty()) std::memcpy(B.data() + o, v.data(), v.size() * sizeof(double));
    return o;
  };
  FRowSetDev& d = f.off;
  d.nrows = f.nrows;
  d.ncols = f.ncols;
  d.ngam = f.ngam;
  d.qb = f.qb;
  d.rmax = f.rmax;
  d.nmono = H.P;
  d.pdeg = H.prob.p;
  d.M = H.M;
  d.o_e1 = put(f.e1, 0, 4);
  d.o_e2 = put(f.e2, 0, 4);
  // per group and row: (slot, first record group | end record group << 16)
  auto rowtab = [&](const std::vector<int>& lst, const std::vector<int>& ptr) {
    std::vector<int> t(2 * (size_t)kFGroupCap, -1);
    for (size_t i = 0; i < lst.size(); ++i) {
      const int sl = lst[i];
      if (sl < 0) continue;
      const int b4 = ptr[sl] / 4, e4 = ptr[sl + 1] / 4;
      if (e4 > 0xffff) throw Error(SG_ERR_UNSUPPORTED, "factored apply: too many records");
      t[2 * i] = sl;
      t[2 * i + 1] = b4 | (e4 << 16);
    }
    return t;
  };
  d.o_r1 = put(rowtab(f.l1, f.p1), 0, 2);
  d.o_r2 = put(rowtab(f.l2, f.p2), 0, 2);
  d.o_dcol = put(f.dcol, 0, 1);
  d.o_cols = put(f.cols, 0, 1);
  d.o_rows = put(f.rows, 0, 1);
  d.o_mpar = put(H.mpar, 0, 1);
  d.o_mvar = put(H.mvar, 0, 1);
  d.o_mdeg = put(H.mdeg, 0, 1);
  std::vector<double> cs(f.ncols), gs(f.ngam), rsv(f.nrows), ra(f.nrows);
  for (int c = 0; c < f.ncols; ++c) cs[c] = H.sfac[f.cols[c]];
  for (int gi = 0; gi < f.ngam; ++gi) gs[gi] = 1.0 / (H.sfac[f.gam[gi]] * H.sfac[f.gam[gi]]);
  for (int r = 0; r < f.nrows; ++r) {
    rsv[r] = H.sfac[f.rows[r]];
    ra[r] = 1.0 / H.sfac[f.rows[r]];
  }
  d.o_cs = putd(cs);
  d.o_gs = putd(gs);
  d.o_rs = putd(rsv);
  d.o_ra = putd(ra);
  d.o_minv = putd(H.minv);
  while (B.size() % 4) B.push_back(0);  // staged with 16-byte loads
  d.nblob = (int)B.size();
  d.blob = nullptr;
}

// Sub-batch size: forced, else the largest of 64/32/16/8 whose LDS allows two
// workgroups per CU, else the largest that fits at all.
void plan_frowset(const sg_handle& H, FRowSetHost& f, int force_qb) {
  int qb = 0;
  const int cands[] = {64, 32, 16, 8};
  const int nblob = (int)f.blob.size();
  for (size_t budget : {(size_t)80 * 1024, (size_t)160 * 1024}) {
    for (int c : cands) {
      if (force_qb && c != force_qb) continue;
      if (fapply_lds_bytes(c, f.nrows, f.ncols, f.ngam, H.P, H.M, nblob) <= budget) {
        qb = c;
        break;
      }
    }
    if (qb) break;
  }
  if (!qb)
    throw Error(SG_ERR_UNSUPPORTED, "factored apply: no sub-batch size fits in LDS" +
                                        std::string(force_qb ? " (forced)" : ""));
  const int groups = 256 / qb;
  const int rmax = std::max({1, (f.ngam + groups - 1) / groups, (f.nrows + groups - 1) / groups});
  if (groups * rmax > kFGroupCap) throw Error(SG_ERR_INTERNAL, "factored apply: group table");
  f.qb = qb;
  f.rmax = rmax;
  assign_groups(f.p1, groups, rmax, f.l1);
  assign_groups(f.p2, groups, rmax, f.l2);
  pack_frowset(H, f);
}

FRowSetHost build_frowset(const sg_handle& H, const std::vector<TPair>& T,
                          const std::vector<int>& rows, const std::vector<int>& cols,
                          int force_qb) {
  FRowSetHost f;
  f.rows = rows;
  f.cols = cols;
  f.nrows = (int)rows.size();
  f.ncols = (int)cols.size();
  std::vector<int> rslot(H.P, -1), cslot(H.P, -1), gslot(H.P, -1);
  for (int t = 0; t < f.nrows; ++t) rslot[rows[t]] = t;
  for (int t = 0; t < f.ncols; ++t) cslot[cols[t]] = t;
  // gamma couples a column to a row only if gamma <= some column and <= some row
  std::vector<char> fromc(H.P, 0), fromr(H.P, 0);
  for (const TPair& t : T) {
    if (cslot[t.a] >= 0) fromc[t.gm] = 1;
    if (rslot[t.a] >= 0) fromr[t.gm] = 1;
  }
  for (int gm = 0; gm < H.P; ++gm)
    if (fromc[gm] && fromr[gm]) {
      gslot[gm] = (int)f.gam.size();
      f.gam.push_back(gm);
    }
  f.ngam = (int)f.gam.size();
  std::vector<std::vector<int>> b1(f.ngam), b2(f.nrows);
  for (const TPair& t : T) {
    if (gslot[t.gm] < 0) continue;
    if (cslot[t.a] >= 0) b1[gslot[t.gm]].push_back(cslot[t.a] | (t.d << 16));
    if (rslot[t.a] >= 0) b2[rslot[t.a]].push_back(gslot[t.gm] | (t.d << 16));
  }
  layout_records(b1, H.P, f.p1, f.e1);
  layout_records(b2, H.P, f.p2, f.e2);
  f.dcol.resize(f.nrows);
  for (int r = 0; r < f.nrows; ++r) f.dcol[r] = cslot[rows[r]];
  // the blob's size does not depend on the plan: pack once to size it
  f.l1.assign(kFGroupCap, -1);
  f.l2.assign(kFGroupCap, -1);
  pack_frowset(H, f);
  plan_frowset(H, f, force_qb);
  return f;
}

void validate(const sg_problem& p) {
  auto bad = [](const std::string& m) { throw Error(SG_ERR_INVALID_ARG, m); };
  if (p.n < 4 || p.n > 4096 || (p.n & (p.n - 1))) bad("n must be a power of two in [4, 4096]");
  if (p.M < 1 || p.M > 12) bad("M must be in [1, 12]");
  if (p.p < 0 || p.q < 0 || p.q > 16) bad("p >= 0 and 0 <= q <= 16 required");
  if (p.cov != SG_COV_EXP_L1 && p.cov != SG_COV_SQEXP) bad("unknown covariance");
  if (!(p.sigma >= 0.0) || !(p.corr_len > 0.0) || !(p.a_min >= 0.0) || !std::isfinite(p.mu) ||
      !std::isfinite(p.sigma) || !std::isfinite(p.corr_len) || !std::isfinite(p.a_min))
    bad("need sigma >= 0, corr_len > 0, a_min >= 0, all finite");
}

// workspace layout: carved identically for sizing (base = nullptr) and binding
void carve(const sg_handle& H, DevPtrs& D, Carver& c) {
  D.a = c.take<double>((size_t)H.na * H.Nq);
  D.g = c.take<double>((size_t)H.M * H.Nq);
  D.isf = c.take<double>(H.na);
  D.Jq = c.take<int>((size_t)H.na * H.M);
  D.f = c.take<double>((size_t)(H.n + 1) * (H.n + 1));
  D.L.clear();
  for (int ln : H.level_n) {
    Level lv;
    lv.n = ln;
    lv.N = (int64_t)(ln - 1) * (ln - 1);
    lv.S = c.take<double>(9 * (size_t)lv.N * (1 + H.P));  // A_0, then K_ii per mode
    D.L.push_back(lv);
  }
  auto put_rowset = [&](const RowSetHost& rs, RowSetDev& d) {
    d.nrows = rs.nrows;
    d.ncols = rs.ncols;
    d.rmax = rs.rmax;
    d.maxent = rs.maxent;
    d.kc = rs.kc;
    d.nchunk = rs.nchunk;
    d.npass = rs.npass;
    d.maxcols = rs.maxcols;
    d.rows = c.take<int>(rs.rows.size());
    d.cols = c.take<int>(std::max<size_t>(rs.cols.size(), 1));
    d.cpass = c.take<int>(rs.cpass.size());
    d.wrows = c.take<int>(rs.wrows.size());
    d.ptr = c.take<int>(rs.ptr.size());
    d.ent = c.take<Entry>(std::max<size_t>(rs.ent.size(), 1));
  };
  put_rowset(H.full, D.full);
  auto put_frowset = [&](const FRowSetHost& f, FRowSetDev& d) {
    d = f.off;
    d.blob = c.take<int>(f.blob.size());
  };
  if (H.factored_ok) put_frowset(H.ffull, D.ffull);
  for (int g = 0; g < SG_GROUP_COUNT; ++g) {
    const FSHost& fh = H.fs[g];
    FSDev& fd = D.fs[g];
    fd.split_idx.assign(fh.splits.size(), nullptr);
    fd.split_sid.assign(fh.splits.size(), nullptr);
    fd.partial.assign(fh.splits.size(), RowSetDev{});
    fd.fpartial.assign(fh.splits.size(), FRowSetDev{});
    for (size_t s = 0; s < fh.splits.size(); ++s) {
      fd.split_idx[s] = c.take<int>(fh.splits[s].size());
      fd.split_sid[s] = c.take<int>(fh.splits[s].size());
      if (s >= 1) put_rowset(fh.partial[s], fd.partial[s]);
      if (s >= 1 && H.factored_ok) put_frowset(fh.fpartial[s], fd.fpartial[s]);
    }
  }
  D.edge = c.take<double>((size_t)H.P * H.ntiles * kEdgeVals);
  const size_t nl = D.L.size();
  D.mg_b.assign(nl, nullptr);
  D.mg_x.assign(nl, nullptr);
  D.mg_xa.assign(nl, nullptr);
  D.mg_r.assign(nl, nullptr);
  for (size_t l = 0; l < nl; ++l) {
    const size_t sz = (size_t)H.P * D.L[l].N;
    if (l > 0) {
      D.mg_b[l] = c.take<double>(sz);
      // the dense operator below the finest level writes kDenseSlices partial results
      D.mg_x[l] = c.take<double>((int)l == H.ldense ? kDenseSlices * sz : sz);
    }
    D.mg_xa[l] = c.take<double>(sz);
    D.mg_r[l] = c.take<double>(sz);
  }
  D.fsT = c.take<double>((size_t)H.P * H.Nh);
  D.fsX = c.take<double>((size_t)H.P * H.Nh);
  D.fsR = c.take<double>((size_t)H.P * H.Nh);
  D.fsD = c.take<double>((size_t)H.P * H.Nh);
  D.all_sid = c.take<int>(H.P);
  D.diag_k = c.take<int>(std::max<size_t>(H.diag_k.size(), 1));
  D.diag_v = c.take<double>(std::max<size_t>(H.diag_v.size(), 1));
  D.cdiag = c.take<double>(H.Nq);
  {
    const int64_t Nv = (int64_t)H.P * H.Nh;
    D.stage = c.take<double>((size_t)std::max(dot_blocks(Nv), gs_blocks(Nv)) + 4);
  }
  if (H.ldense >= 0) {
    const size_t Nd = (size_t)(H.level_n[H.ldense] - 1) * (H.level_n[H.ldense] - 1);
    D.Cd = c.take<double>(Nd * Nd);
  }
  if (H.q2) {
    D.q2g = c.take<double>((size_t)H.M * H.Nq2);
    D.q2grad = c.take<double>((size_t)2 * H.P * H.Nq2);
    D.q2y = c.take<double>((size_t)2 * H.P * H.Nq2);
    D.q2t.ptr1 = c.take<int>(H.q2p1.size());
    D.q2t.idx1 = c.take<int>(H.q2i1.size());
    D.q2t.c1 = c.take<double>(H.q2c1.size());
    D.q2t.e1 = c.take<uint64_t>(H.q2e1.size());
    D.q2t.ptr2 = c.take<int>(H.q2p2.size());
    D.q2t.idx2 = c.take<int>(H.q2i2.size());
    D.q2t.c2 = c.take<double>(H.q2c2.size());
    D.q2t.e2 = c.take<uint64_t>(H.q2e2.size());
  }
}

template <class T>
void upload(hipStream_t s, const T* dst, const std::vector<T>& src) {
  if (!src.empty())
    SG_HIP(hipMemcpyAsync(const_cast<T*>(dst), src.data(), src.size() * sizeof(T),
                          hipMemcpyHostToDevice, s));
}

void upload_rowset(hipStream_t s, const RowSetHost& h, const RowSetDev& d) {
  upload(s, d.rows, h.rows);
  upload(s, d.cols, h.cols);
  upload(s, d.cpass, h.cpass);
  upload(s, d.wrows, h.wrows);
  upload(s, d.ptr, h.ptr);
  upload(s, d.ent, h.ent);
}

void upload_frowset(hipStream_t s, const FRowSetHost& h, FRowSetDev& d) {
  const int* blob = d.blob;
  d = h.off;
  d.blob = blob;
  upload(s, d.blob, h.blob);
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// One V(2,2) cycle for m modes starting at level l0: b and x hold m compact
// vectors of that level; smode (device, may be null) gives each mode's stencil id.
// bmap / xmap (device, may be null; l0 must be a fused fine level): mode t reads
// vector bmap[t] of b and writes vector xmap[t] of x.
void vcycle_levels(sg_handle& H, hipStream_t s, int l0, int m, const int* smode, const double* b,
                   double* x, const int* bmap = nullptr, const int* xmap = nullptr,
                   const EdgeFix& ef = EdgeFix{}) {
  DevPtrs& D = H.d;
  const int nf = H.nfine;
  const int nl = (int)D.L.size();
  if ((bmap || xmap || ef.edge) && l0 >= nf)
    throw Error(SG_ERR_INTERNAL, "mode maps and edge sums need a fused level");
  std::vector<const double*> bl(nl);
  std::vector<double*> xl(nl);
  for (int l = l0 + 1; l < nl; ++l) {
    bl[l] = D.mg_b[l];
    xl[l] = D.mg_x[l];
  }
  bl[l0] = b;
  xl[l0] = x;
  const int c0 = std::max(nf, l0);
  for (int l = l0; l < nf; ++l)
    launch_vdown(s, D.L[l], D.L[l + 1], m, smode, bl[l], D.mg_xa[l], D.mg_b[l + 1], kOmega,
                 l == l0 ? bmap : nullptr, l == l0 ? ef : EdgeFix{});
  CoarseLevels cl{};
  cl.nl = nl - c0;
  for (int l = 0; l < cl.nl; ++l) {
    cl.n[l] = D.L[c0 + l].n;
    cl.N[l] = D.L[c0 + l].N;
    cl.S[l] = D.L[c0 + l].S;
  }
  launch_vcoarse(s, cl, m, smode, bl[c0], xl[c0], kOmega);
  for (int l = nf - 1; l >= l0; --l)
    launch_vup(s, D.L[l], D.L[l + 1], m, smode, bl[l], D.mg_xa[l], xl[l + 1], xl[l], kOmega,
               l == l0 ? bmap : nullptr, l == l0 ? xmap : nullptr, 1, l == l0 ? ef : EdgeFix{});
}

// Whether vcycle() can read and write through mode maps (the finest level is a
// fused kernel pair or the dense operator).
bool vcycle_maps_ok(const sg_handle& H, const int* smode) {
  return H.nfine > 0 || (!smode && H.dense_ready);
}

// Whether vcycle()'s finest level is a vdown / vup pair, which can add an
// apply's pending edge sums to the right-hand side as it reads it.
bool vcycle_edges_ok(const sg_handle& H, const int* smode) {
  return (!smode && H.dense_ready) ? H.ldense > 0 : H.nfine > 0;
}

// One V(2,2) cycle on the finest level.  With the mean stiffness (smode null)
// the levels from H.ldense down are one precomputed dense operator (the same
// linear map, built by vcycle_levels on unit vectors at bind).
void vcycle(sg_handle& H, hipStream_t s, int m, const int* smode, const double* b, double* x,
            const int* bmap = nullptr, const int* xmap = nullptr, const EdgeFix& ef = EdgeFix{}) {
  if (smode || !H.dense_ready) {
    vcycle_levels(H, s, 0, m, smode, b, x, bmap, xmap, ef);
    return;
  }
  if (ef.edge && H.ldense == 0) throw Error(SG_ERR_INTERNAL, "edge sums need a fused level");
  DevPtrs& D = H.d;
  const int ld = H.ldense;
  auto bl = [&](int l) -> const double* { return l == 0 ? b : D.mg_b[l]; };
  auto xl = [&](int l) -> double* { return l == 0 ? x : D.mg_x[l]; };
  // the two finest levels in one kernel each way when both are above the dense
  // operator and the launches are small enough to be latency-bound
  const bool two = ld >= 2 && H.n % 4 == 0 && two_level_pays(D.L[2], m);
  const int lf = two ? 2 : 0;  // first level run by the one-level kernels
  if (two)
    launch_vdown2(s, D.L[0], D.L[1], D.L[2], m, b, D.mg_xa[0], D.mg_b[1], D.mg_xa[1], D.mg_b[2],
                  kOmega, bmap, ef);
  for (int l = lf; l < ld; ++l)
    launch_vdown(s, D.L[l], D.L[l + 1], m, nullptr, bl(l), D.mg_xa[l], D.mg_b[l + 1], kOmega,
                 l == 0 ? bmap : nullptr, l == 0 ? ef : EdgeFix{});
  // below the finest level the operator runs in kDenseSlices inner-index
  // slices whose partial results the next finer vup sums
  const int slices = ld == 0 ? 1 : kDenseSlices;
  launch_dense_coarse(s, (int)D.L[ld].N, m, D.Cd, bl(ld), xl(ld), ld == 0 ? bmap : nullptr,
                      ld == 0 ? xmap : nullptr, slices);
  for (int l = ld - 1; l >= lf; --l)
    launch_vup(s, D.L[l], D.L[l + 1], m, nullptr, bl(l), D.mg_xa[l], xl(l + 1), xl(l), kOmega,
               l == 0 ? bmap : nullptr, l == 0 ? xmap : nullptr, l == ld - 1 ? slices : 1,
               l == 0 ? ef : EdgeFix{});
  if (two)
    launch_vup2(s, D.L[0], D.L[1], D.L[2], m, b, D.mg_xa[0], D.mg_b[1], D.mg_xa[1], xl(2),
                ld == 2 ? slices : 1, x, kOmega, bmap, xmap, ef);
}

// The edge sums an apply with sign sgn leaves pending in H.d.edge.
EdgeFix pending_edges(const sg_handle& H, double sgn) {
  EdgeFix f;
  f.edge = H.d.edge;
  f.nt = H.n / kTileE;
  f.sgn = sgn;
  f.Nh = H.Nh;
  f.m = H.n - 1;
  f.rNh = recip64((uint64_t)f.Nh);
  f.rm = recip64((uint64_t)f.m);
  return f;
}

// W = K U; with fixup false the edge sums stay pending (pending_edges(H, 1.0)).
// `edge` (default: the handle's own) receives the tiles' edge sums, P * ntiles
// * kEdgeVals values, every one written by the apply before the fixup reads it.
void do_apply(sg_handle& H, hipStream_t s, const double* U, double* W, bool fixup = true,
              double* edge = nullptr) {
  if (H.q2) {
    // complete on return: no edge sums are left pending
    launch_q2_apply(s, H.n2, H.M, H.P, H.prob.mu, H.prob.a_min, H.d.q2g, H.d.q2t, U, W,
                    H.d.q2grad, H.d.q2y);
    return;
  }
  if (!edge) edge = H.d.edge;
  if (H.use_factored && H.use_rapply)
    launch_rapply(s, H.M, H.prob.p, H.n, H.prob.mu, H.prob.a_min, H.d.g, H.rfull, U, H.Nh,
                  nullptr, 0.0, 1.0, W, edge, fixup);
  else if (H.use_factored)
    launch_fapply(s, H.n, H.prob.mu, H.prob.a_min, H.d.g, H.d.ffull, U, H.Nh, nullptr, 0.0, 1.0,
                  W, edge, fixup);
  else
    launch_apply(s, H.n, H.na, H.d.a, H.d.full, U, H.Nh, nullptr, 0.0, 1.0, W, edge, fixup);
}

// ---- the apply without allocation ------------------------------------------
// sg_apply_noalloc keeps the apply's edge sums (its only scratch) in this
// file-scope device array instead of the handle's workspace.  Each device holds
// its own copy until the process ends.  In host code `scratch` names a host
// stand-in, not device memory: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on first use there).
double* noalloc_scratch() {
  int dev = 0;
  SG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    throw Error(SG_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw Error(SG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}

// ---- multigrid on the full SG system ----------------------------------------
// (Sec. 3: one V-cycle on K preconditions GMRES; every level carries the whole
// SG operator, the smoother is the field-split level iteration of eq.
// level_solver, the coarsest level is solved directly.)  Levels n, n/2, ..., 4
// are rediscretised: the operator-apply kernels run on each level's grid with
// the KL values at that level's Gauss points.  The smoother's split blocks are
// the nodal blocks of K restricted to each split's modes, inverted exactly.
constexpr int kMGPre = 1, kMGPost = 1;
constexpr int kMGCoarseN = 4;

// g_m at the Gauss points of the nl-element grid, tile order: the 1D
// eigenvectors of the finest grid (P1) interpolated linearly at the level's
// Gauss abscissae, g_m = sqrt(lambda_m) e_r(x_1) e_s(x_2).
std::vector<double> mg_level_g(const sg_handle& H, int nl) {
  const int n = H.n, ratio = n / nl;
  const int64_t Nq = (int64_t)4 * nl * nl;
  const double gp[2] = {0.5 * (1.0 - 1.0 / std::sqrt(3.0)), 0.5 * (1.0 + 1.0 / std::sqrt(3.0))};
  std::vector<double> out((size_t)H.M * Nq);
  auto e_at = [&](const std::vector<double>& e, int el, int q) {
    const double t = (el + gp[q]) * ratio;
    const int i = std::min((int)std::floor(t), n - 1);
    const double f = t - i;
    return (1.0 - f) * e[i] + f * e[i + 1];
  };
  for (int m = 0; m < H.M; ++m) {
    const auto& er = H.kl.e1[H.kl.pairs[m].first];
    const auto& es = H.kl.e1[H.kl.pairs[m].second];
    const double sq = std::sqrt(H.kl.lam[m]);
    for (int ey = 0; ey < nl; ++ey)
      for (int ex = 0; ex < nl; ++ex)
        for (int qy = 0; qy < 2; ++qy)
          for (int qx = 0; qx < 2; ++qx)
            out[(size_t)m * Nq + tiled_q(nl, ex, ey, qx, qy)] = sq * e_at(es, ey, qy) * e_at(er, ex, qx);
  }
  return out;
}

// Carves (or, with base == nullptr, sizes) the multigrid workspace.
size_t mg_layout(const sg_handle& H, int grouping, MGState& st, char* base) {
  Carver c{base};
  const auto& splits = H.fs[grouping].splits;
  size_t maxm = 0;
  for (const auto& g : splits) maxm = std::max(maxm, g.size());
  st.L.clear();
  for (int nl = H.n;; nl /= 2) {
    MGLevel L;
    L.n = nl;
    L.N = (int64_t)(nl - 1) * (nl - 1);
    const size_t PN = (size_t)H.P * L.N;
    const bool last = nl <= kMGCoarseN;
    if (nl != H.n) {
      L.g = c.take<double>((size_t)H.M * 4 * nl * nl);
      // the triple-product form's coefficient modes (either form may be selected later)
      L.a = c.take<double>((size_t)H.na * 4 * nl * nl);
      L.edge = c.take<double>((size_t)H.P * (nl / kTileE) * (nl / kTileE) * kEdgeVals);
      L.b = c.take<double>(PN);
      L.z = c.take<double>(PN);
    }
    L.res = c.take<double>(PN);
    L.dz = c.take<double>(PN);
    L.t = c.take<double>(maxm * L.N);
    if (!last)
      for (const auto& g : splits) L.Dinv.push_back(c.take<double>(mg_block_doubles((int)g.size()) * L.N));
    st.L.push_back(L);
    if (last) break;
  }
  st.Nc = (int)(H.P * st.L.back().N);
  st.Cinv = c.take<double>((size_t)st.Nc * st.Nc);
  return c.off;
}

// out = beta rin + sgn K_l U on level l (the whole operator)
void mg_apply(sg_handle& H, hipStream_t s, int l, const double* U, const double* rin, double beta,
              double sgn, double* out) {
  const MGLevel& L = H.mg.L[l];
  const double* g = l ? L.g : H.d.g;
  double* edge = l ? L.edge : H.d.edge;
  if (H.use_factored && H.use_rapply)
    launch_rapply(s, H.M, H.prob.p, L.n, H.prob.mu, H.prob.a_min, g, H.rfull, U, L.N, rin, beta,
                  sgn, out, edge, true);
  else if (H.use_factored)
    launch_fapply(s, L.n, H.prob.mu, H.prob.a_min, g, H.d.ffull, U, L.N, rin, beta, sgn, out, edge,
                  true);
  else
    launch_apply(s, L.n, H.na, l ? L.a : H.d.a, H.d.full, U, L.N, rin, beta, sgn, out, edge, true);
}

// out (the split's rows, compact) = rin_{g_sp} - K_{g_sp, g_<sp} U on level l
void mg_partial(sg_handle& H, hipStream_t s, int l, int sp, const double* U, const double* rin,
                double* out) {
  const MGLevel& L = H.mg.L[l];
  const int gr = H.mg.grouping;
  const double* g = l ? L.g : H.d.g;
  double* edge = l ? L.edge : H.d.edge;
  if (H.use_factored && H.use_rapply)
    launch_rapply(s, H.M, H.prob.p, L.n, H.prob.mu, H.prob.a_min, g, H.rpart[gr][sp], U, L.N, rin,
                  1.0, -1.0, out, edge, true, H.rkv[gr][sp]);
  else if (H.use_factored)
    launch_fapply(s, L.n, H.prob.mu, H.prob.a_min, g, H.d.fs[gr].fpartial[sp], U, L.N, rin, 1.0,
                  -1.0, out, edge, true);
  else
    launch_apply(s, L.n, H.na, l ? L.a : H.d.a, H.d.fs[gr].partial[sp], U, L.N, rin, 1.0, -1.0,
                 out, edge, true);
}

// One level iteration z <- z + P_FS^{-1}(b - K z) (eq. level_solver); with
// zero_start the residual is b itself and the correction is written to z.
void mg_smooth(sg_handle& H, hipStream_t s, int l, const double* b, double* z, bool zero_start) {
  const MGLevel& L = H.mg.L[l];
  const FSHost& fh = H.fs[H.mg.grouping];
  const FSDev& fd = H.d.fs[H.mg.grouping];
  const double* res = b;
  double* dz = z;
  if (!zero_start) {
    mg_apply(H, s, l, z, b, 1.0, -1.0, L.res);
    res = L.res;
    dz = L.dz;
  }
  for (size_t sp = 0; sp < fh.splits.size(); ++sp) {
    const int mm = (int)fh.splits[sp].size();
    if (sp == 0) {
      launch_mg_block(s, L.Dinv[0], mm, L.N, res, fd.split_idx[0], fd.split_idx[0], kOmega, dz);
    } else {
      mg_partial(H, s, l, (int)sp, dz, res, L.t);
      launch_mg_block(s, L.Dinv[sp], mm, L.N, L.t, nullptr, fd.split_idx[sp], kOmega, dz);
    }
  }
  if (!zero_start) launch_mg_axpy(s, L.dz, z, (int64_t)H.P * L.N);
}

// z = V(b) on level l (V(kMGPre, kMGPost) from z = 0)
void mg_vcycle(sg_handle& H, hipStream_t s, int l, const double* b, double* z) {
  const int last = (int)H.mg.L.size() - 1;
  if (l == last) {
    launch_mg_dense(s, H.mg.Cinv, b, z, H.mg.Nc);
    return;
  }
  MGLevel& L = H.mg.L[l];
  MGLevel& C = H.mg.L[l + 1];
  for (int k = 0; k < kMGPre; ++k) mg_smooth(H, s, l, b, z, k == 0);
  mg_apply(H, s, l, z, b, 1.0, -1.0, L.res);
  launch_mg_restrict(s, L.res, C.b, L.n, H.P);
  mg_vcycle(H, s, l + 1, C.b, C.z);
  launch_mg_prolong_add(s, C.z, z, L.n, H.P);
  for (int k = 0; k < kMGPost; ++k) mg_smooth(H, s, l, b, z, false);
}

// In-place inverse of a dense n x n column-major matrix (Gauss-Jordan with
// partial pivoting; element (i, j) at A[j*n + i]); false when singular.
bool dense_inverse(std::vector<double>& A, int n) {
  std::vector<int> piv(n);
  std::vector<double> f(n);
  for (int k = 0; k < n; ++k) {
    double* ck = &A[(size_t)k * n];
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(ck[i]) > std::fabs(ck[p])) p = i;
    if (ck[p] == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)j * n + k], A[(size_t)j * n + p]);
    const double d = 1.0 / ck[k];
    ck[k] = 1.0;
    for (int j = 0; j < n; ++j) A[(size_t)j * n + k] *= d;   // row k
    for (int i = 0; i < n; ++i) f[i] = (i == k) ? 0.0 : ck[i];
    for (int i = 0; i < n; ++i)
      if (i != k) ck[i] = 0.0;
    for (int j = 0; j < n; ++j) {
      double* cj = &A[(size_t)j * n];
      const double akj = cj[k];
      if (akj == 0.0) continue;
      for (int i = 0; i < n; ++i) cj[i] -= f[i] * akj;
    }
  }
  // undo the row swaps as column swaps, in reverse order
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k)
      for (int i = 0; i < n; ++i) std::swap(A[(size_t)k * n + i], A[(size_t)piv[k] * n + i]);
  return true;
}

// x = B_t^{-1}-approximation of the compact block right-hand side b for the m
// modes of a split: `inner` Richardson steps x <- x + V(b - B x) from x = 0
// (eq. level_solver on each diagonal block), B the A_0 or K_ii stencil.
void block_solve(sg_handle& H, hipStream_t s, int m, const int* smode, int inner, const double* b,
                 double* x) {
  vcycle(H, s, m, smode, b, x);
  for (int k = 1; k < inner; ++k) {
    launch_stencil_residual(s, H.n, H.d.L[0].S, smode, m, b, x, H.d.fsR);
    vcycle(H, s, m, smode, H.d.fsR, H.d.fsD);
    launch_axpby(s, 1.0, H.d.fsD, 1.0, x, (int64_t)m * H.Nh);
  }
}

void do_precond(sg_handle& H, hipStream_t s, int pc, int grouping, const double* r, double* z) {
  const int64_t Nv = (int64_t)H.P * H.Nh;
  const bool kii = (pc & SG_PC_DIAG_KII) != 0;
  const int inner = std::max(1, (pc >> SG_PC_INNER_SHIFT) & 0xff);
  const int kind = pc & 0xff;
  if (inner > 1 && (kind == SG_PC_MEAN || kind == SG_PC_FS)) {
    // the blocks' inner iterations run on compact copies of each split
    const int g = kind == SG_PC_MEAN ? -1 : grouping;
    if (g >= SG_GROUP_COUNT) throw Error(SG_ERR_INVALID_ARG, "unknown grouping");
    if (g < 0) {
      block_solve(H, s, H.P, kii ? H.d.all_sid : nullptr, inner, r, z);
      return;
    }
    const FSHost& fh = H.fs[g];
    const FSDev& fd = H.d.fs[g];
    for (size_t sp = 0; sp < fh.splits.size(); ++sp) {
      const int m = (int)fh.splits[sp].size();
      if (sp == 0)
        launch_gather_modes(s, m, fd.split_idx[0], H.Nh, r, H.d.fsT);
      else if (H.use_factored && H.use_rapply)
        launch_rapply(s, H.M, H.prob.p, H.n, H.prob.mu, H.prob.a_min, H.d.g, H.rpart[g][sp], z,
                      H.Nh, r, 1.0, -1.0, H.d.fsT, H.d.edge, true, H.rkv[g][sp]);
      else if (H.use_factored)
        launch_fapply(s, H.n, H.prob.mu, H.prob.a_min, H.d.g, fd.fpartial[sp], z, H.Nh, r, 1.0,
                      -1.0, H.d.fsT, H.d.edge, true);
      else
        launch_apply(s, H.n, H.na, H.d.a, fd.partial[sp], z, H.Nh, r, 1.0, -1.0, H.d.fsT,
                     H.d.edge, true);
      block_solve(H, s, m, kii ? fd.split_sid[sp] : nullptr, inner, H.d.fsT, H.d.fsX);
      launch_scatter_modes(s, m, fd.split_idx[sp], H.Nh, H.d.fsX, z);
    }
    return;
  }
  if (kind == SG_PC_NONE) {
    SG_HIP(hipMemcpyAsync(z, r, Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    return;
  }
  if (kind == SG_PC_MEAN) {
    vcycle(H, s, H.P, kii ? H.d.all_sid : nullptr, r, z);
    return;
  }
  if (kind == SG_PC_MG) {
    if (!H.mg.bound) throw Error(SG_ERR_NOT_BOUND, "full-system multigrid not bound (sg_mg_bind)");
    if (grouping != H.mg.grouping)
      throw Error(SG_ERR_INVALID_ARG, "grouping differs from the one the multigrid was bound with");
    mg_vcycle(H, s, 0, r, z);
    return;
  }
  if (kind != SG_PC_FS) throw Error(SG_ERR_INVALID_ARG, "unknown preconditioner");
  if (grouping < 0 || grouping >= SG_GROUP_COUNT) throw Error(SG_ERR_INVALID_ARG, "unknown grouping");
  const FSHost& fh = H.fs[grouping];
  const FSDev& fd = H.d.fs[grouping];
  for (size_t sp = 0; sp < fh.splits.size(); ++sp) {
    const int m = (int)fh.splits[sp].size();
    const int* smode = kii ? fd.split_sid[sp] : nullptr;
    const bool maps = vcycle_maps_ok(H, smode);
    // the off-diagonal apply's edge sums are added by the cycle's finest level
    const bool defer = maps && vcycle_edges_ok(H, smode);
    if (sp == 0) {
      // the gather is folded into the cycle's finest level when it can be
      if (maps) {
        vcycle(H, s, m, smode, r, z, fd.split_idx[0], fd.split_idx[0]);
        continue;
      }
      launch_gather_modes(s, m, fd.split_idx[0], H.Nh, r, H.d.fsT);
    } else {
      if (H.use_factored && H.use_rapply)
        launch_rapply(s, H.M, H.prob.p, H.n, H.prob.mu, H.prob.a_min, H.d.g, H.rpart[grouping][sp],
                      z, H.Nh, r, 1.0, -1.0, H.d.fsT, H.d.edge, !defer, H.rkv[grouping][sp]);
      else if (H.use_factored)
        launch_fapply(s, H.n, H.prob.mu, H.prob.a_min, H.d.g, fd.fpartial[sp], z, H.Nh, r, 1.0,
                      -1.0, H.d.fsT, H.d.edge, !defer);
      else
        launch_apply(s, H.n, H.na, H.d.a, fd.partial[sp], z, H.Nh, r, 1.0, -1.0, H.d.fsT,
                     H.d.edge, !defer);
    }
    if (maps) {
      vcycle(H, s, m, smode, H.d.fsT, z, nullptr, fd.split_idx[sp],
             defer ? pending_edges(H, -1.0) : EdgeFix{});
    } else {
      vcycle(H, s, m, smode, H.d.fsT, H.d.fsX);
      launch_scatter_modes(s, m, fd.split_idx[sp], H.Nh, H.d.fsX, z);
    }
  }
}

// One application of the learned stage (the network is not part of the paper):
//   z0 = P_FS^{-1} v (fs_pc: the field split, with or without K_ii blocks),
//   r1 = v - K z0, c = N(r1) (the attached network's error prediction),
//   z = z0 + alpha c with alpha = <r1, K c> / ||K c||^2, the step that
//   minimises ||v - K z|| along c; alpha = 0 (z = z0) when the prediction is
//   not finite.  The field split is thus both the fallback and the judge: the
//   stage's residual never exceeds the field split's.
// Scratch: r1, c, kc (vectors), partial (dot partials), dots (3 scalars; dots[2]
// receives alpha).  w (nullable) receives K z (for the Arnoldi step).
void learned_stage(sg_handle& H, hipStream_t s, int fs_pc, int grouping, const double* v, double* z,
                   double* w, double* r1, double* c, double* kc, double* partial, int nblk,
                   double* dots) {
  const int64_t Nv = (int64_t)H.P * H.Nh;
  do_precond(H, s, fs_pc, grouping, v, z);
  double* kz = w ? w : kc;
  do_apply(H, s, z, kz);
  launch_sub(s, v, kz, r1, Nv);
  cnn_apply_sg(H.cnn, s, r1, H.cnn_sigma, c, partial, nblk);
  do_apply(H, s, c, kc);
  launch_gs_dot(s, r1, Nv, 1, kc, Nv, partial, dots);
  launch_gs_dot(s, kc, Nv, 1, kc, Nv, partial, dots + 1);
  launch_stage_alpha(s, dots, c, kc, z, w, Nv);
}

// allow_solve: the flags of a whole solve (the learned stage, the switch to
// K_ii cycles) are allowed too
bool valid_pc(int pc, bool allow_learned = false, bool allow_solve = false) {
  const int kind = pc & 0xff, inner = (pc >> SG_PC_INNER_SHIFT) & 0xff;
  const int flags = pc & ~0xff & ~(0xff << SG_PC_INNER_SHIFT);
  if (kind < SG_PC_NONE || kind > SG_PC_MG) return false;
  if (kind == SG_PC_LEARNED && !allow_learned) return false;
  if (pc < 0 || (inner > 1 && kind != SG_PC_MEAN && kind != SG_PC_FS && kind != SG_PC_LEARNED))
    return false;
  if (flags & ~(SG_PC_DIAG_KII | SG_PC_SWITCH_KII)) return false;
  if ((flags & SG_PC_SWITCH_KII) &&
      (!allow_solve || (kind != SG_PC_MEAN && kind != SG_PC_FS) || (flags & SG_PC_DIAG_KII)))
    return false;
  if (kind == SG_PC_MG && flags) return false;
  return true;
}

constexpr double kSwitchRatio = 0.2;  // SG_PC_SWITCH_KII: least reduction of a cycle

}  // namespace

// ===========================================================================
extern "C" {

const char* sg_last_error(void) { return g_last_error.c_str(); }

namespace {
int setup_impl(const sg_problem* prob, const double* f_nodal, int force_kc, sg_handle** out);
}

int sg_setup(const sg_problem* prob, const double* f_nodal, sg_handle** out) {
  return setup_impl(prob, f_nodal, 0, out);
}

int sg_setup_q2(const sg_problem* prob, const double* f_nodal, sg_handle** out) {
  if (!prob || !out) return fail(SG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (prob->n < 4 || prob->n > 2048 || (prob->n & (prob->n - 1)))
    return fail(SG_ERR_INVALID_ARG, "n must be a power of two in [4, 2048] for Q2 elements");
  if (prob->p < 0 || prob->q < 2 * prob->p)
    return fail(SG_ERR_UNSUPPORTED, "the Q2 apply is the factored form: q >= 2p required");
  if (prob->p > 15) return fail(SG_ERR_UNSUPPORTED, "the Q2 apply packs exponents below 16: p <= 15");
  sg_problem r = *prob;
  r.n = 2 * prob->n;
  sg_handle* raw = nullptr;
  const int rc = setup_impl(&r, f_nodal, 0, &raw);
  if (rc != SG_OK) return rc;
  std::unique_ptr<sg_handle> H(raw);
  try {
    H->q2 = true;
    H->n2 = prob->n;
    const int n2 = H->n2, nr = H->n, M = H->M, P = H->P;
    H->Nq2 = (int64_t)9 * n2 * n2;
    // the apply's launches take one work-item per (mode, Gauss point)
    if ((int64_t)P * H->Nq2 >= (int64_t(1) << 31))
      return fail(SG_ERR_UNSUPPORTED, "Q2: P * 9 n^2 must stay below 2^31");
    // KL values at the 3 x 3 Gauss points: the refined grid's 1D eigenvectors,
    // linear in each coordinate within a refined cell
    const double gp[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
    H->q2g.assign((size_t)M * H->Nq2, 0.0);
    auto lin = [&](const std::vector<double>& e, int el, int qi) {
      const double X = 2.0 * (el + gp[qi]);
      const int c = std::min((int)std::floor(X), nr - 1);
      const double t = X - c;
      return (1.0 - t) * e[c] + t * e[c + 1];
    };
    for (int m = 0; m < M; ++m) {
      const auto& er = H->kl.e1[H->kl.pairs[m].first];
      const auto& es = H->kl.e1[H->kl.pairs[m].second];
      const double sq = std::sqrt(H->kl.lam[m]);
      for (int ey = 0; ey < n2; ++ey)
        for (int ex = 0; ex < n2; ++ex)
          for (int qy = 0; qy < 3; ++qy)
            for (int qx = 0; qx < 3; ++qx)
              H->q2g[(size_t)m * H->Nq2 + (size_t)(3 * qy + qx) * n2 * n2 + (size_t)ey * n2 + ex] =
                  sq * lin(er, ex, qx) * lin(es, ey, qy);
    }
    // T_{alpha beta} = prod_m sqrt(alpha_m! / beta_m!) g_m^(alpha_m - beta_m) / (alpha_m - beta_m)!
    // for beta <= alpha, listed by column and by row
    auto fact = [](int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; };
    struct Ent { int a, b; double c; uint64_t e; };
    std::vector<Ent> ent;
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b) {
        bool le = true;
        for (int m = 0; m < M; ++m) le = le && H->Jp[b][m] <= H->Jp[a][m];
        if (!le) continue;
        double c = 1.0;
        uint64_t code = 0;
        for (int m = 0; m < M; ++m) {
          const int am = H->Jp[a][m], bm = H->Jp[b][m];
          c *= std::sqrt(fact(am) / fact(bm)) / fact(am - bm);
          code |= (uint64_t)(am - bm) << (4 * m);
        }
        ent.push_back({a, b, c, code});
      }
    auto lists = [&](bool by_col, std::vector<int>& ptr, std::vector<int>& idx,
                     std::vector<double>& cv, std::vector<uint64_t>& ev) {
      std::vector<Ent> v = ent;
      std::stable_sort(v.begin(), v.end(), [&](const Ent& x, const Ent& y) {
        return by_col ? (x.b != y.b ? x.b < y.b : x.a < y.a) : (x.a != y.a ? x.a < y.a : x.b < y.b);
      });
      ptr.assign(P + 1, 0);
      for (const Ent& x : v) {
        ptr[(by_col ? x.b : x.a) + 1]++;
        idx.push_back(by_col ? x.a : x.b);
        cv.push_back(x.c);
        ev.push_back(x.e);
      }
      for (int i = 0; i < P; ++i) ptr[i + 1] += ptr[i];
    };
    lists(true, H->q2p1, H->q2i1, H->q2c1, H->q2e1);
    lists(false, H->q2p2, H->q2i2, H->q2c2, H->q2e2);
    *out = H.release();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

namespace {
int setup_impl(const sg_problem* prob, const double* f_nodal, int force_kc, sg_handle** out) {
  if (!prob || !out) return fail(SG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  try {
    validate(*prob);
    auto H = std::make_unique<sg_handle>();
    H->prob = *prob;
    H->n = prob->n;
    H->M = prob->M;
    H->Nh = (int64_t)(H->n - 1) * (H->n - 1);
    H->Nq = (int64_t)4 * H->n * H->n;
    H->nt = H->n / kTileE;
    H->ntiles = H->nt * H->nt;
    H->Jp = total_degree_set(prob->M, prob->p);
    H->Jq = total_degree_set(prob->M, prob->q);
    H->P = (int)H->Jp.size();
    H->na = (int)H->Jq.size();
    if (H->P > kMaxP) throw Error(SG_ERR_UNSUPPORTED, "P exceeds 256 modes");
    if (H->na > 65535) throw Error(SG_ERR_UNSUPPORTED, "too many coefficient modes");
    H->G = triple_list(H->Jp, H->Jq);
    H->kl = karhunen_loeve(H->n, prob->cov, prob->corr_len, prob->sigma, prob->M);
    // tile-major copy of g_m(x_q)
    H->g_tiled.assign((size_t)H->M * H->Nq, 0.0);
    for (int m = 0; m < H->M; ++m)
      for (int ey = 0; ey < H->n; ++ey)
        for (int ex = 0; ex < H->n; ++ex)
          for (int qy = 0; qy < 2; ++qy)
            for (int qx = 0; qx < 2; ++qx) {
              size_t canon = 4 * ((size_t)ey * H->n + ex) + 2 * qy + qx;
              H->g_tiled[(size_t)m * H->Nq + tiled_q(H->n, ex, ey, qx, qy)] =
                  H->kl.gq[(size_t)m * H->Nq + canon];
            }
    for (auto& k : H->Jq) {
      double f = 1.0;
      for (int e : k) {
        double fac = 1.0;
        for (int t = 2; t <= e; ++t) fac *= t;
        f /= std::sqrt(fac);
      }
      H->isf.push_back(f);
      for (int e : k) H->Jq_flat.push_back(e);
    }
    const size_t nn = (size_t)(H->n + 1) * (H->n + 1);
    if (f_nodal) H->f_nodal.assign(f_nodal, f_nodal + nn);
    else H->f_nodal.assign(nn, 1.0);
    for (double v : H->f_nodal)
      if (!std::isfinite(v)) throw Error(SG_ERR_INVALID_ARG, "non-finite forcing");
    std::vector<int> all(H->P);
    std::iota(all.begin(), all.end(), 0);
    H->full = build_rowset(*H, all, all, force_kc);
    H->factored_ok = prob->q >= 2 * prob->p;
    H->use_factored = H->factored_ok;
    for (int g = 0; g < SG_GROUP_COUNT; ++g) {
      FSHost& fh = H->fs[g];
      fh.splits = make_splits(H->Jp, g);
      fh.partial.assign(fh.splits.size(), RowSetHost{});
      fh.fpartial.assign(fh.splits.size(), FRowSetHost{});
      fh.sid.assign(fh.splits.size(), {});
      for (size_t sp = 0; sp < fh.splits.size(); ++sp)
        for (int i : fh.splits[sp]) fh.sid[sp].push_back(i + 1);
      std::vector<int> prev;
      for (size_t s = 0; s < fh.splits.size(); ++s) {
        if (s >= 1) fh.partial[s] = build_rowset(*H, fh.splits[s], prev);
        prev.insert(prev.end(), fh.splits[s].begin(), fh.splits[s].end());
      }
    }
    if (H->factored_ok) {
      // a mode count whose tables do not fit in LDS keeps the triple-product form
      try {
        std::vector<TPair> T = t_pairs(*H);
        monomial_tables(*H);
        H->ffull = build_frowset(*H, T, all, all, 0);
        for (int g = 0; g < SG_GROUP_COUNT; ++g) {
          FSHost& fh = H->fs[g];
          std::vector<int> prev = fh.splits[0];
          for (size_t s = 1; s < fh.splits.size(); ++s) {
            fh.fpartial[s] = build_frowset(*H, T, fh.splits[s], prev, 0);
            prev.insert(prev.end(), fh.splits[s].begin(), fh.splits[s].end());
          }
        }
      } catch (const Error& e) {
        if (e.code != SG_ERR_UNSUPPORTED) throw;
        H->factored_ok = H->use_factored = false;
      }
    }
    // register form: the compiled chaos table must be this handle's J(p)
    H->rapply_ok = H->factored_ok && H->P <= kRMax && rapply_supported(H->M, prob->p) &&
                   rapply_matches(H->M, prob->p, H->Jp);
    H->use_rapply = H->rapply_ok;
    if (H->rapply_ok) {
      auto rows = [&](const std::vector<int>& outm, const std::vector<int>& colm) {
        RApplyRows r{};
        for (int c : colm) rset(r.colmask, c);
        std::memset(r.slot, 0xFF, sizeof(r.slot));
        for (size_t t = 0; t < outm.size(); ++t) {
          rset(r.rowmask, outm[t]);
          r.slot[outm[t]] = (unsigned char)t;
          r.mode[t] = (unsigned char)outm[t];
        }
        r.nrows = (int)outm.size();
        // gamma matters iff it lies below some column and below some output row
        for (int gm = 0; gm < H->P; ++gm) {
          auto below = [&](const std::vector<int>& set) {
            for (int a : set) {
              bool le = true;
              for (int k = 0; k < H->M; ++k) le = le && H->Jp[gm][k] <= H->Jp[a][k];
              if (le) return true;
            }
            return false;
          };
          if (below(colm) && below(outm)) rset(r.gammask, gm);
        }
        return r;
      };
      H->rfull = rows(all, all);
      for (int g = 0; g < SG_GROUP_COUNT; ++g) {
        FSHost& fh = H->fs[g];
        H->rpart[g].assign(fh.splits.size(), RApplyRows{});
        H->rkv[g].assign(fh.splits.size(), 0);
        std::vector<int> prev = fh.splits[0];
        for (size_t sp = 1; sp < fh.splits.size(); ++sp) {
          H->rpart[g][sp] = rows(fh.splits[sp], prev);
          prev.insert(prev.end(), fh.splits[sp].begin(), fh.splits[sp].end());
          // the compiled block of split sp serves it iff its rows are the modes
          // whose first variable is sp and its columns those below (the mean
          // counting as variable 0)
          const RApplyRows& r = H->rpart[g][sp];
          bool same = (int)sp < H->M;
          for (int i = 0; same && i < H->P; ++i) {
            int first = 0;
            for (int k = H->M - 1; k >= 0; --k)
              if (H->Jp[i][k] != 0) first = k;
            same = rbit(r.rowmask, i) == (first == (int)sp) && rbit(r.colmask, i) == (first < (int)sp);
          }
          if (same) H->rkv[g][sp] = (int)sp;
        }
      }
    }
    for (int ln = H->n; ln >= 2; ln /= 2) {
      if (ln <= kDenseN && H->ldense < 0) H->ldense = (int)H->level_n.size();
      H->level_n.push_back(ln);
      if (ln > kCoarseN) H->nfine++;
    }
    if ((int)H->level_n.size() - H->nfine > kMaxCoarseLevels)
      throw Error(SG_ERR_INTERNAL, "too many coarse levels");
    H->diag_ptr.assign(1, 0);
    for (int i = 0; i < H->P; ++i) {
      for (const Triple& t : H->G)
        if (t.i == i && t.j == i) {
          H->diag_k.push_back(t.k);
          H->diag_v.push_back(t.v);
        }
      H->diag_ptr.push_back((int)H->diag_k.size());
      H->diag_sid.push_back(i + 1);
    }
    *out = H.release();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

}  // namespace

int sg_sizes(const sg_handle* h, int64_t* P, int64_t* N_h, int64_t* n_a, int64_t* nnz_G) {
  if (!h) return fail(SG_ERR_INVALID_ARG, "null handle");
  if (P) *P = h->P;
  if (N_h) *N_h = h->Nh;
  if (n_a) *n_a = h->na;
  if (nnz_G) *nnz_G = (int64_t)h->G.size();
  return SG_OK;
}

size_t sg_workspace_bytes(const sg_handle* h) {
  if (!h) return 0;
  DevPtrs dry;
  Carver c{nullptr};
  carve(*h, dry, c);
  return c.off;
}

int sg_bind(sg_handle* h, void* dev_workspace, size_t bytes, void* stream) {
  if (!h || !dev_workspace) return fail(SG_ERR_INVALID_ARG, "null argument");
  try {
    const size_t need = sg_workspace_bytes(h);
    if (bytes < need)
      return fail(SG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
      return fail(SG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    sg_handle& H = *h;
    H.ws = static_cast<char*>(dev_workspace);
    H.ws_bytes = bytes;
    Carver c{H.ws};
    carve(H, H.d, c);
    DevPtrs& D = H.d;
    upload(s, D.g, H.g_tiled);
    upload(s, D.isf, H.isf);
    upload(s, D.Jq, H.Jq_flat);
    upload(s, D.f, H.f_nodal);
    upload_rowset(s, H.full, D.full);
    if (H.factored_ok) upload_frowset(s, H.ffull, D.ffull);
    for (int g = 0; g < SG_GROUP_COUNT; ++g)
      for (size_t sp = 0; sp < H.fs[g].splits.size(); ++sp) {
        upload(s, D.fs[g].split_idx[sp], H.fs[g].splits[sp]);
        upload(s, D.fs[g].split_sid[sp], H.fs[g].sid[sp]);
        if (sp >= 1) upload_rowset(s, H.fs[g].partial[sp], D.fs[g].partial[sp]);
        if (sp >= 1 && H.factored_ok)
          upload_frowset(s, H.fs[g].fpartial[sp], D.fs[g].fpartial[sp]);
      }
    upload(s, D.all_sid, H.diag_sid);
    upload(s, D.diag_k, H.diag_k);
    upload(s, D.diag_v, H.diag_v);
    if (H.q2) {
      upload(s, D.q2g, H.q2g);
      upload(s, D.q2t.ptr1, H.q2p1);
      upload(s, D.q2t.idx1, H.q2i1);
      upload(s, D.q2t.c1, H.q2c1);
      upload(s, D.q2t.e1, H.q2e1);
      upload(s, D.q2t.ptr2, H.q2p2);
      upload(s, D.q2t.idx2, H.q2i2);
      upload(s, D.q2t.c2, H.q2c2);
      upload(s, D.q2t.e2, H.q2e2);
    }
    launch_coeff(s, H.n, H.M, H.na, D.g, D.Jq, D.isf, H.prob.mu, H.prob.a_min, D.a);
    // stencil 0: mean stiffness A_0; stencil i+1: diagonal block K_ii
    for (int id = 0; id <= H.P; ++id) {
      const double* coef = D.a;
      if (id > 0) {
        const int b0 = H.diag_ptr[id - 1], b1 = H.diag_ptr[id];
        launch_diag_coeff(s, H.n, b1 - b0, D.diag_k + b0, D.diag_v + b0, D.a, D.cdiag);
        coef = D.cdiag;
      }
      launch_fine_stencil(s, H.n, coef, D.L[0].S + (int64_t)id * 9 * D.L[0].N);
      for (size_t l = 1; l < D.L.size(); ++l)
        launch_rap(s, D.L[l - 1].n, D.L[l - 1].S + (int64_t)id * 9 * D.L[l - 1].N,
                   D.L[l].S + (int64_t)id * 9 * D.L[l].N);
    }
    // dense coarse operator: the cycle from level ldense applied to unit vectors,
    // P columns at a time
    if (H.ldense >= 0) {
      H.dense_ready = false;
      const int Nd = (int)D.L[H.ldense].N;
      for (int j0 = 0; j0 < Nd; j0 += H.P) {
        const int m = std::min(H.P, Nd - j0);
        launch_unit_columns(s, Nd, j0, m, D.fsT);
        vcycle_levels(H, s, H.ldense, m, nullptr, D.fsT, D.fsX);
        SG_HIP(hipMemcpyAsync(D.Cd + (size_t)j0 * Nd, D.fsX, sizeof(double) * m * Nd,
                              hipMemcpyDeviceToDevice, s));
      }
      H.dense_ready = true;
    }
    check_launch();
    if (!H.host_pinned)
      SG_HIP(hipHostMalloc((void**)&H.host_pinned, sizeof(double) * (4 * (kMaxRestart + 2) + 8),
                           hipHostMallocDefault));
    if (!H.fetched) SG_HIP(hipEventCreateWithFlags(&H.fetched, hipEventDisableTiming));
    SG_HIP(hipStreamSynchronize(s));
    H.bound = true;
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

int sg_rhs(sg_handle* h, double* F, void* stream) {
  if (!h || !F) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  try {
    if (h->q2)
      launch_q2_rhs(reinterpret_cast<hipStream_t>(stream), h->n2, h->P, h->d.f, F);
    else
      launch_rhs(reinterpret_cast<hipStream_t>(stream), h->n, h->d.f, F, (int64_t)h->P * h->Nh);
    check_launch();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_apply_form(const sg_handle* h, int* form, int* points_per_batch) {
  if (!h || !form || !points_per_batch) return fail(SG_ERR_INVALID_ARG, "null argument");
  *form = h->q2 ? 3 : !h->use_factored ? 0 : h->use_rapply ? 2 : 1;
  *points_per_batch = *form == 1 ? h->ffull.qb : 0;
  return SG_OK;
}

int sg_set_apply(sg_handle* h, int kind, int points_per_batch, void* stream) {
  if (!h) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (h->q2) return fail(SG_ERR_UNSUPPORTED, "a Q2 handle has one apply form");
  if (kind < SG_APPLY_AUTO || kind > SG_APPLY_FACTORED)
    return fail(SG_ERR_INVALID_ARG, "unknown apply form");
  const int qb = points_per_batch;
  if (qb != 0 && qb != 8 && qb != 16 && qb != 32 && qb != 64)
    return fail(SG_ERR_INVALID_ARG, "points_per_batch must be 0, 8, 16, 32 or 64");
  sg_handle& H = *h;
  if (kind == SG_APPLY_FACTORED && !H.factored_ok)
    return fail(SG_ERR_UNSUPPORTED, "the factored apply needs q >= 2p");
  try {
    if (H.factored_ok && qb != H.fqb) {
      // plan on copies first: a size that does not fit leaves the old plan in place
      FRowSetHost full = H.ffull;
      plan_frowset(H, full, qb);
      std::vector<std::vector<FRowSetHost>> parts(SG_GROUP_COUNT);
      for (int g = 0; g < SG_GROUP_COUNT; ++g) {
        parts[g] = H.fs[g].fpartial;
        for (size_t sp = 1; sp < parts[g].size(); ++sp) plan_frowset(H, parts[g][sp], qb);
      }
      H.ffull = std::move(full);
      for (int g = 0; g < SG_GROUP_COUNT; ++g) H.fs[g].fpartial = std::move(parts[g]);
      H.fqb = qb;
      if (H.bound) {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        upload_frowset(s, H.ffull, H.d.ffull);
        for (int g = 0; g < SG_GROUP_COUNT; ++g)
          for (size_t sp = 1; sp < H.fs[g].fpartial.size(); ++sp)
            upload_frowset(s, H.fs[g].fpartial[sp], H.d.fs[g].fpartial[sp]);
        SG_HIP(hipStreamSynchronize(s));
      }
    }
    H.use_factored = kind == SG_APPLY_AUTO ? H.factored_ok : kind == SG_APPLY_FACTORED;
    // the register form unless a sub-batch size of the LDS tile kernel was asked for
    H.use_rapply = H.use_factored && H.rapply_ok && qb == 0;
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

int sg_apply(sg_handle* h, const double* U, double* W, void* stream) {
  if (!h || !U || !W) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (U == W) return fail(SG_ERR_INVALID_ARG, "U and W must not alias");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  try {
    do_apply(*h, reinterpret_cast<hipStream_t>(stream), U, W);
    check_launch();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_apply_noalloc(sg_handle* h, const double* U, double* W, void* stream) {
  if (!h || !U || !W) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (U == W) return fail(SG_ERR_INVALID_ARG, "U and W must not alias");
  if (h->q2) return fail(SG_ERR_UNSUPPORTED, "sg_apply_noalloc: Q1 handles only");
  const size_t need = (size_t)h->P * h->ntiles * kEdgeVals * sizeof(double);
  if (need > kNoAllocScratchBytes)
    return fail(SG_ERR_UNSUPPORTED, "sg_apply_noalloc: the edge sums need " + std::to_string(need) +
                                        " bytes, above the fixed scratch of " +
                                        std::to_string(kNoAllocScratchBytes) + " bytes");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  try {
    double* edge = noalloc_scratch();
    do_apply(*h, reinterpret_cast<hipStream_t>(stream), U, W, true, edge);
    check_launch();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_residual(sg_handle* h, const double* F, const double* u, double* r, void* stream) {
  if (!h || !F || !u || !r) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (r == F || r == u) return fail(SG_ERR_INVALID_ARG, "r must not alias F or u");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    do_apply(*h, s, u, r);
    launch_axpby(s, 1.0, F, -1.0, r, (int64_t)h->P * h->Nh);
    check_launch();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_precond_apply(sg_handle* h, int pc, int grouping, const double* r, double* z,
                     void* stream) {
  if (!h || !r || !z) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (r == z) return fail(SG_ERR_INVALID_ARG, "r and z must not alias");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  if (!valid_pc(pc, true)) return fail(SG_ERR_INVALID_ARG, "unknown preconditioner");
  if (grouping < 0 || grouping >= SG_GROUP_COUNT) return fail(SG_ERR_INVALID_ARG, "unknown grouping");
  const bool learned = (pc & 0xff) == SG_PC_LEARNED;
  if (learned && !h->cnn) return fail(SG_ERR_INVALID_ARG, "learned stage needs an attached network");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (learned) {
      // the preconditioner's own scratch is free once z0 is formed
      sg_handle& H = *h;
      const int64_t Nv = (int64_t)H.P * H.Nh;
      const int nb = std::max(dot_blocks(Nv), gs_blocks(Nv));
      learned_stage(H, s, (pc & ~0xff) | SG_PC_FS, grouping, r, z, nullptr, H.d.fsT, H.d.fsX,
                    H.d.mg_xa[0], H.d.stage, dot_blocks(Nv), H.d.stage + nb);
      check_launch();
      return SG_OK;
    }
    do_precond(*h, s, pc, grouping, r, z);
    check_launch();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

size_t sg_mg_workspace_bytes(const sg_handle* h, int grouping) {
  if (!h || grouping < 0 || grouping >= SG_GROUP_COUNT) return 0;
  MGState st;
  return mg_layout(*h, grouping, st, nullptr);
}

int sg_mg_bind(sg_handle* h, int grouping, void* ws, size_t bytes, void* stream) {
  if (!h || !ws) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  if (grouping < 0 || grouping >= SG_GROUP_COUNT) return fail(SG_ERR_INVALID_ARG, "unknown grouping");
  for (const auto& g : h->fs[grouping].splits)
    if (mg_block_pad((int)g.size()) == 0)
      return fail(SG_ERR_UNSUPPORTED, "full-system multigrid: a split of more than 128 modes");
  if (bytes < sg_mg_workspace_bytes(h, grouping)) return fail(SG_ERR_WORKSPACE, "multigrid workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(SG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  try {
    sg_handle& H = *h;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    H.mg.bound = false;
    mg_layout(H, grouping, H.mg, static_cast<char*>(ws));
    H.mg.grouping = grouping;
    const auto& splits = H.fs[grouping].splits;
    const FSDev& fd = H.d.fs[grouping];
    std::vector<int> split_of(H.P), pos_of(H.P);
    for (size_t sp = 0; sp < splits.size(); ++sp)
      for (size_t a = 0; a < splits[sp].size(); ++a) {
        split_of[splits[sp][a]] = (int)sp;
        pos_of[splits[sp][a]] = (int)a;
      }
    for (size_t l = 1; l < H.mg.L.size(); ++l) {
      MGLevel& L = H.mg.L[l];
      upload(s, L.g, mg_level_g(H, L.n));
      launch_coeff(s, L.n, H.M, H.na, L.g, H.d.Jq, H.d.isf, H.prob.mu, H.prob.a_min, L.a);
    }
    const int last = (int)H.mg.L.size() - 1;
    // nodal blocks: apply K to one mode on one node colour at a time
    for (int l = 0; l < last; ++l) {
      MGLevel& L = H.mg.L[l];
      double* U = L.res;
      double* W = L.dz;
      launch_zero(s, U, (int64_t)H.P * L.N);
      for (int colour = 0; colour < 4; ++colour)
        for (int j = 0; j < H.P; ++j) {
          launch_mg_mark(s, U + (int64_t)j * L.N, L.n, colour, 1.0);
          mg_apply(H, s, l, U, nullptr, 0.0, 1.0, W);
          const int sp = split_of[j];
          launch_mg_gather(s, W, L.n, colour, fd.split_idx[sp], (int)splits[sp].size(), pos_of[j],
                           L.Dinv[sp]);
          launch_mg_mark(s, U + (int64_t)j * L.N, L.n, colour, 0.0);
        }
      for (size_t sp = 0; sp < splits.size(); ++sp)
        launch_mg_invert(s, L.Dinv[sp], (int)splits[sp].size(), L.N);
      check_launch();
    }
    // coarsest level: K column by column, inverted on the host
    {
      MGLevel& L = H.mg.L[last];
      const int Nc = H.mg.Nc;
      for (int col = 0; col < Nc; ++col) {
        launch_mg_unit(s, L.res, Nc, col);
        mg_apply(H, s, last, L.res, nullptr, 0.0, 1.0, H.mg.Cinv + (int64_t)col * Nc);
      }
      check_launch();
      std::vector<double> A((size_t)Nc * Nc);
      SG_HIP(hipMemcpyAsync(A.data(), H.mg.Cinv, A.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      SG_HIP(hipStreamSynchronize(s));
      if (!dense_inverse(A, Nc)) throw Error(SG_ERR_INTERNAL, "coarsest multigrid level is singular");
      SG_HIP(hipMemcpyAsync(H.mg.Cinv, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    SG_HIP(hipStreamSynchronize(s));
    H.mg.bound = true;
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

namespace {
struct KrylovWS {
  double *V, *Z, *w, *z, *t, *x2, *partial, *hdev, *ydev;
  int nblk;
};

size_t krylov_layout(const sg_handle* h, int restart, bool flexible, KrylovWS* k, char* base) {
  const int64_t Nv = (int64_t)h->P * h->Nh;
  Carver c{base};
  KrylovWS tmp;
  KrylovWS& K = k ? *k : tmp;
  K.nblk = dot_blocks(Nv);
  K.V = c.take<double>((size_t)(restart + 1) * Nv);
  K.Z = flexible ? c.take<double>((size_t)restart * Nv) : nullptr;
  K.w = c.take<double>(Nv);
  K.z = c.take<double>(Nv);
  K.t = c.take<double>(Nv);
  K.x2 = c.take<double>(Nv);
  K.partial = c.take<double>(std::max((size_t)std::max(K.nblk, gs_blocks(Nv)) * (restart + 1),
                                       gs2_partial_doubles(restart, Nv)));
  K.hdev = c.take<double>(3 * (size_t)(restart + 1) + 16);
  K.ydev = c.take<double>(restart + 1);
  return c.off;
}

bool is_learned(const sg_solve_opts* o) { return (o->pc & 0xff) == SG_PC_LEARNED; }
}  // namespace

size_t sg_gmres_workspace_bytes(const sg_handle* h, const sg_solve_opts* o) {
  if (!h || !o || o->restart < 1 || o->restart > kMaxRestart) return 0;
  return krylov_layout(h, o->restart, is_learned(o), nullptr, nullptr);
}

size_t sg_cnn_stage_work_doubles(const sg_handle* h) {
  if (!h) return 0;
  const int64_t Nv = (int64_t)h->P * h->Nh;
  return (size_t)(5 * Nv + 16 + gs_blocks(Nv));
}

// The learned stage's own objective for one stored pair: with c the network's
// output for the pair (batch slot `slot` of the last forward) and r its
// residual, the stage's step z0 + alpha c leaves the fraction
// L = 1 - (r.Kc)^2 / (|r|^2 |Kc|^2) of the residual (squared); this writes
// dL/dc / batch = 2a / (rho b batch) K((a/b) Kc - r), a = r.Kc, b = |Kc|^2,
// rho = |r|^2 (K symmetric), into the network's output gradient of that slot.
int sg_cnn_stage_grad(sg_handle* h, sg_cnn* c, const uint16_t* R, int64_t pair, int32_t slot,
                      int32_t batch, double* work, double* loss, void* stream) {
  if (!h || !c || !R || !work) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  if (!cnn_bound(c)) return fail(SG_ERR_NOT_BOUND, "network not bound");
  if (cnn_modes(c) != h->P || cnn_grid(c) != h->n)
    return fail(SG_ERR_INVALID_ARG, "network P / n do not match the problem");
  if (batch < 1 || batch > cnn_max_batch(c) || slot < 0 || slot >= batch || pair < 0)
    return fail(SG_ERR_INVALID_ARG, "slot, batch or pair out of range");
  try {
    sg_handle& H = *h;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t Nv = (int64_t)H.P * H.Nh;
    double* cv = work;
    double* r = work + Nv;
    double* Kc = work + 2 * Nv;
    double* v = work + 3 * Nv;
    double* Kv = work + 4 * Nv;
    double* d = work + 5 * Nv;
    double* partial = d + 16;
    cnn_slot_to_sg(c, s, slot, cv);
    cnn_pair_to_sg(c, s, R, pair, r);
    do_apply(H, s, cv, Kc);
    launch_gs_dot(s, r, Nv, 1, Kc, Nv, partial, d);
    launch_gs_dot(s, Kc, Nv, 1, Kc, Nv, partial, d + 1);
    launch_gs_dot(s, r, Nv, 1, r, Nv, partial, d + 2);
    launch_stage_objective(s, d, batch, Kc, r, v, Nv);
    do_apply(H, s, v, Kv);
    cnn_slot_grad_from_sg(c, s, slot, Kv, d + 4);
    check_launch();
    if (loss) {
      SG_HIP(hipMemcpyAsync(loss, d + 5, sizeof(double), hipMemcpyDeviceToHost, s));
      SG_HIP(hipStreamSynchronize(s));
    }
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_attach_cnn(sg_handle* h, sg_cnn* c, double sigma) {
  if (!h) return fail(SG_ERR_INVALID_ARG, "null handle");
  if (c) {
    if (h->q2) return fail(SG_ERR_UNSUPPORTED, "the learned stage serves Q1 handles only");
    if (!cnn_bound(c)) return fail(SG_ERR_NOT_BOUND, "network not bound");
    if (cnn_modes(c) != h->P || cnn_grid(c) != h->n)
      return fail(SG_ERR_INVALID_ARG, "network P / n do not match the problem");
    if (!std::isfinite(sigma)) return fail(SG_ERR_INVALID_ARG, "sigma must be finite");
  }
  h->cnn = c;
  h->cnn_sigma = sigma;
  return SG_OK;
}

int sg_gmres_solve(sg_handle* h, const sg_solve_opts* o, const double* F, double* u,
                   void* krylov_ws, size_t ws_bytes, double* resid_hist, int32_t hist_len,
                   sg_solve_info* info, void* stream) {
  if (!h || !o || !F || !u || !krylov_ws || !info) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!h->bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
  if (o->restart < 1 || o->restart > kMaxRestart) return fail(SG_ERR_INVALID_ARG, "restart out of range");
  if (o->max_it < 1) return fail(SG_ERR_INVALID_ARG, "max_it must be positive");
  if (!(o->tol > 0.0)) return fail(SG_ERR_INVALID_ARG, "tol must be positive");
  if (!valid_pc(o->pc, true, true)) return fail(SG_ERR_INVALID_ARG, "unknown preconditioner");
  if (is_learned(o) && !h->cnn) return fail(SG_ERR_INVALID_ARG, "learned stage needs an attached network");
  if (o->grouping < 0 || o->grouping >= SG_GROUP_COUNT) return fail(SG_ERR_INVALID_ARG, "unknown grouping");
  if (ws_bytes < sg_gmres_workspace_bytes(h, o)) return fail(SG_ERR_WORKSPACE, "Krylov workspace too small");
  if (reinterpret_cast<uintptr_t>(krylov_ws) % 256) return fail(SG_ERR_WORKSPACE, "Krylov workspace must be 256-byte aligned");
  try {
    sg_handle& H = *h;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int m = o->restart;
    const int64_t Nv = (int64_t)H.P * H.Nh;
    KrylovWS K;
    const bool learned = is_learned(o);
    krylov_layout(h, m, learned, &K, static_cast<char*>(krylov_ws));
    const int fs_pc = (o->pc & ~0xff) | SG_PC_FS;
    // the preconditioner in use (SG_PC_SWITCH_KII may add SG_PC_DIAG_KII at a restart)
    int pc = o->pc & ~SG_PC_SWITCH_KII;
    int switches = 0;
    int fallbacks = 0;
    double* hp = H.host_pinned;
    auto norm2 = [&](const double* x, double* dst) {
      launch_gs_dot(s, x, Nv, 1, x, Nv, K.partial, dst);
    };
    auto fetch = [&](const double* src, int count) {
      SG_HIP(hipMemcpyAsync(hp, src, count * sizeof(double), hipMemcpyDeviceToHost, s));
      SG_HIP(hipStreamSynchronize(s));
    };
    norm2(F, K.hdev);
    fetch(K.hdev, 1);
    const double nF = std::sqrt(hp[0]);
    std::memset(info, 0, sizeof(*info));
    int hist_n = 0;
    auto push_hist = [&](double v) {
      if (resid_hist && hist_n < hist_len) resid_hist[hist_n] = v;
      hist_n++;
    };
    if (nF == 0.0 || !std::isfinite(nF)) {
      launch_zero(s, u, Nv);
      SG_HIP(hipStreamSynchronize(s));
      info->status = nF == 0.0 ? SG_CONVERGED : SG_BREAKDOWN;
      push_hist(0.0);
      return SG_OK;
    }
    const double target = o->tol * nF;
    double beta;
    if (o->use_x0) {
      do_apply(H, s, u, K.w);
      launch_sub(s, F, K.w, K.t, Nv);
      norm2(K.t, K.hdev);
      fetch(K.hdev, 1);
      beta = std::sqrt(hp[0]);
    } else {
      launch_zero(s, u, Nv);
      SG_HIP(hipMemcpyAsync(K.t, F, Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
      beta = nF;
    }
    push_hist(beta / nF);
    std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hat = [&](int i, int j) -> double& { return Hm[(size_t)i * m + j]; };
    int it = 0, restarts = 0;
    bool broke = false;
    double est = beta;
    // Rotates column j of Hat by the rotations 0..j-1, forms rotation j and
    // applies it to g.
    auto rotate_column = [&](int j) {
      for (int i = 0; i < j; ++i) {
        double tmp = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
        Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
        Hat(i, j) = tmp;
      }
      double a = Hat(j, j), b = Hat(j + 1, j);
      if (b == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        double r = std::hypot(a, b);
        cs[j] = a / r;
        sn[j] = b / r;
      }
      Hat(j, j) = cs[j] * a + sn[j] * b;
      Hat(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
    };
    // Linear preconditioners: Gram-Schmidt with the second projection delayed
    // by one step (launch_gs2_*, two passes over the basis per step).  Step j
    // applies the operator B = K M^{-1} to u_j, the previous step's vector after
    // one projection, u_j = nu_j q_j + Q s_j.  Pass A/B give
    //   B u_j = Q_{0..j} c_j + a_j u_{j+1},  a_j = nu_j rho_j,
    // so in the vectors the operator was applied to, B U = Q H~ with column j
    // of H~ equal to (c_j + a_j s_{j+1}, a_j nu_{j+1}): complete one step later,
    // once s_{j+1} and nu_{j+1} are known.  GMRES minimises |beta nu_0 e_1 -
    // H~ y| and corrects x by M^{-1} U y = M^{-1} Q (S y), S the upper
    // triangle with columns (s_j, nu_j).  The residual estimate of step j
    // takes column j with s_{j+1} = 0, nu_{j+1} = 1; when it meets the
    // tolerance, and at the end of a cycle, one more dot pass completes it.
    std::vector<double> Ht(learned ? 0 : (size_t)(m + 1) * m), Sm(learned ? 0 : (size_t)m * m),
        av(m), col(m + 1);
    auto Htt = [&](int i, int j) -> double& { return Ht[(size_t)i * m + j]; };
    auto Smm = [&](int i, int j) -> double& { return Sm[(size_t)i * m + j]; };
    const int kCoef = 2 * (m + 1) + 2;  // offsets into hdev and hp
    const int kFin = kCoef + 4;
    int nfinal = 0;
    // completes column j from s_{j+1} (j + 1 values) and nu_{j+1}
    auto finish_column = [&](int j, const double* s1, double nu1) {
      for (int i = 0; i <= j; ++i) Htt(i, j) += av[j] * s1[i];
      Htt(j + 1, j) = av[j] * nu1;
      for (int i = 0; i <= j + 1; ++i) Hat(i, j) = Htt(i, j);
      rotate_column(j);
      nfinal = j + 1;
    };
    // |g_{j+1}| with column j completed by s_{j+1} = 0, nu_{j+1} = 1
    auto provisional = [&](int j) {
      for (int i = 0; i <= j; ++i) col[i] = Htt(i, j);
      double b = av[j];
      for (int i = 0; i < j; ++i) {
        double tmp = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = tmp;
      }
      const double r = std::hypot(col[j], b);
      return r > 0.0 ? std::fabs(g[j]) * std::fabs(b) / r : std::fabs(g[j]);
    };
    // The operator apply leaves its edge sums pending (no apply_fixup_kernel):
    // both passes add them as they read w, each once per element.
    auto linear_cycle = [&]() -> int {
      nfinal = 0;
      std::fill(Ht.begin(), Ht.end(), 0.0);
      std::fill(Sm.begin(), Sm.end(), 0.0);
      // the next step's preconditioner and operator apply (which need only
      // u_{j+1}, already on the device) are queued before the host waits for
      // step j's scalars; wasted once, when step j ends the solve
      bool queued = false;
      for (int j = 0; j < m; ++j) {
        double* uj = K.V + (int64_t)j * Nv;
        double* un = K.V + (int64_t)(j + 1) * Nv;
        if (!queued) {
          do_precond(H, s, pc, o->grouping, uj, K.z);
          do_apply(H, s, K.z, K.w, false);
        }
        queued = false;
        const EdgeFix ef = H.q2 ? EdgeFix{} : pending_edges(H, 1.0);
        launch_gs2_dot(s, K.V, Nv, j, uj, K.w, Nv, K.partial, K.hdev, ef);
        launch_gs2_coef(s, j, K.hdev, K.hdev + kCoef);
        launch_gs2_update(s, K.V, Nv, j, K.hdev, K.hdev + j, K.hdev + kCoef, uj, K.w, un, Nv, ef);
        check_launch();
        SG_HIP(hipMemcpyAsync(hp, K.hdev, (kCoef + 4) * sizeof(double), hipMemcpyDeviceToHost, s));
        SG_HIP(hipEventRecord(H.fetched, s));
        if (j + 1 < m && it + 1 < o->max_it) {
          do_precond(H, s, pc, o->grouping, un, K.z);
          do_apply(H, s, K.z, K.w, false);
          queued = true;
        }
        SG_HIP(hipEventSynchronize(H.fetched));
        const double nu = hp[kCoef], cj = hp[kCoef + 1], rho = hp[kCoef + 2];
        if (!std::isfinite(nu)) {
          broke = true;
          return nfinal;
        }
        // u_j = nu_j q_j + Q s_j completes column j - 1 (r = beta u_0 = beta nu_0 q_0)
        if (j == 0)
          g[0] = beta * nu;
        else if (nfinal == j - 1)
          finish_column(j - 1, hp, nu);
        if (j > 0) {
          est = std::fabs(g[j]);
          if (Hat(j - 1, j - 1) == 0.0) {
            broke = true;
            return nfinal;
          }
        }
        // nu_j = 0: u_j lies in the span of the basis, the space is exhausted
        if (nu == 0.0) {
          if (j == 0) broke = true;
          return nfinal;
        }
        if (!std::isfinite(cj) || !std::isfinite(rho)) {
          broke = true;
          return nfinal;
        }
        for (int i = 0; i < j; ++i) Smm(i, j) = hp[i];
        Smm(j, j) = nu;
        for (int i = 0; i < j; ++i) Htt(i, j) = hp[j + i];
        Htt(j, j) = cj;
        av[j] = nu * rho;
        ++it;
        est = provisional(j);
        push_hist(est / nF);
        if (est <= target || j + 1 == m || it >= o->max_it) {
          // complete column j: s_{j+1} = Q_{0..j}^T u_{j+1} and |u_{j+1}|^2
          launch_gs2_dot(s, K.V, Nv, j + 1, un, nullptr, Nv, K.partial, K.hdev + kFin);
          check_launch();
          SG_HIP(hipMemcpyAsync(hp + kFin, K.hdev + kFin, (j + 2) * sizeof(double),
                                hipMemcpyDeviceToHost, s));
          SG_HIP(hipStreamSynchronize(s));
          double ss = 0.0;
          for (int i = 0; i <= j; ++i) ss = std::fma(hp[kFin + i], hp[kFin + i], ss);
          const double nu1 = std::sqrt(hp[kFin + j + 1] - ss);
          if (!std::isfinite(nu1)) {
            broke = true;
            return nfinal;
          }
          finish_column(j, hp + kFin, nu1);
          est = std::fabs(g[j + 1]);
          if (resid_hist && hist_n - 1 < hist_len) resid_hist[hist_n - 1] = est / nF;
          if (Hat(j, j) == 0.0) broke = true;
          if (broke || est <= target || j + 1 == m || it >= o->max_it) return nfinal;
          // not met after all: go on (the next step's pass A recomputes
          // s_{j+1}, and column j is not completed twice)
        }
      }
      return nfinal;
    };
    while (beta > target && it < o->max_it && !broke) {
      std::fill(Hm.begin(), Hm.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      launch_axpby(s, 1.0 / beta, K.t, 0.0, K.V, Nv);
      int kdone = 0;
      if (!learned) {
        kdone = linear_cycle();
      } else {
        // flexible GMRES (the learned stage is nonlinear): classical
        // Gram-Schmidt with both projections in the same step
        for (int j = 0; j < m; ++j) {
          double* vj = K.V + (int64_t)j * Nv;
          // field split first, then the network's prediction c of the error
          // left in the field-split residual r = v - K P_FS^{-1} v, weighted by
          // alpha = <r, K c> / ||K c||^2 (the residual-minimising step), so the
          // stage's residual never exceeds the field split's; alpha = 0 (plain
          // field split) when the prediction is not finite
          double* zj = K.Z + (int64_t)j * Nv;
          learned_stage(H, s, fs_pc, o->grouping, vj, zj, K.w, K.x2, K.z, K.t, K.partial, K.nblk,
                        K.hdev + 2 * (m + 1) + 1);
          double* h1 = K.hdev;
          double* h2 = K.hdev + (m + 1);
          double* nrm = K.hdev + 2 * (m + 1);
          // CGS2: h1 = V^T w, w -= V h1, h2 = V^T w (fused with that update),
          // w -= V h2 and |w|^2 (fused with the second update), v_{j+1} = w / |w|
          launch_gs_dot(s, K.V, Nv, j + 1, K.w, Nv, K.partial, h1);
          launch_gs_update_dot(s, K.V, Nv, j + 1, h1, K.w, Nv, -1.0, K.partial, h2);
          launch_gs_update_norm_scale(s, K.V, Nv, j + 1, h2, K.w, Nv, -1.0, K.partial, nrm,
                                      K.V + (int64_t)(j + 1) * Nv);
          check_launch();
          // the Hessenberg column and the norm; for the learned stage also its alpha
          SG_HIP(hipMemcpyAsync(hp, K.hdev, (2 * (m + 1) + 4) * sizeof(double),
                                hipMemcpyDeviceToHost, s));
          SG_HIP(hipEventRecord(H.fetched, s));
          SG_HIP(hipEventSynchronize(H.fetched));
          if (hp[2 * (m + 1) + 3] == 0.0) ++fallbacks;
          for (int i = 0; i <= j; ++i) Hat(i, j) = hp[i] + hp[m + 1 + i];
          Hat(j + 1, j) = std::sqrt(hp[2 * (m + 1)]);
          if (!std::isfinite(Hat(j + 1, j))) {
            broke = true;
            break;
          }
          rotate_column(j);
          ++it;
          kdone = j + 1;
          est = std::fabs(g[j + 1]);
          push_hist(est / nF);
          if (est <= target || it >= o->max_it) break;
          if (Hat(j, j) == 0.0) {
            broke = true;
            break;
          }
        }
      }
      if (kdone == 0) break;
      for (int i = kdone - 1; i >= 0; --i) {
        double acc = g[i];
        for (int l = i + 1; l < kdone; ++l) acc -= Hat(i, l) * y[l];
        y[i] = acc / Hat(i, i);
      }
      if (learned) {
        for (int i = 0; i < kdone; ++i) hp[i] = y[i];
      } else {
        // the correction in the vectors the operator was applied to: U y = Q (S y)
        for (int i = 0; i < kdone; ++i) {
          double acc = 0.0;
          for (int l = i; l < kdone; ++l) acc += Smm(i, l) * y[l];
          hp[i] = acc;
        }
      }
      SG_HIP(hipMemcpyAsync(K.ydev, hp, kdone * sizeof(double), hipMemcpyHostToDevice, s));
      if (learned) {
        launch_combine(s, K.Z, Nv, kdone, K.ydev, K.t, Nv);
        launch_axpby(s, 1.0, K.t, 1.0, u, Nv);
      } else {
        launch_combine(s, K.V, Nv, kdone, K.ydev, K.t, Nv);
        do_precond(H, s, pc, o->grouping, K.t, K.z);
        launch_axpby(s, 1.0, K.z, 1.0, u, Nv);
      }
      do_apply(H, s, u, K.w);
      launch_sub(s, F, K.w, K.t, Nv);
      norm2(K.t, K.hdev);
      fetch(K.hdev, 1);
      const double beta_prev = beta;
      beta = std::sqrt(hp[0]);
      ++restarts;
      if (!std::isfinite(beta)) broke = true;
      if ((o->pc & SG_PC_SWITCH_KII) && !(pc & SG_PC_DIAG_KII) && beta > target &&
          beta > kSwitchRatio * beta_prev) {
        pc |= SG_PC_DIAG_KII;
        ++switches;
      }
    }
    info->iterations = it;
    info->restarts = restarts;
    info->fallbacks = fallbacks + switches;
    info->relres = beta / nF;
    info->relres_est = est / nF;
    info->status = (beta <= target) ? SG_CONVERGED : (broke ? SG_BREAKDOWN : SG_NOT_CONVERGED);
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

int sg_export(sg_handle* h, int what, int level, double* out, size_t count) {
  if (!h || !out) return fail(SG_ERR_INVALID_ARG, "null argument");
  try {
    sg_handle& H = *h;
    auto need = [&](size_t c) {
      if (count < c) throw Error(SG_ERR_INVALID_ARG, "output buffer too small: need " + std::to_string(c));
    };
    switch (what) {
      case SG_EXPORT_KL:
        need(H.kl.lam.size());
        std::copy(H.kl.lam.begin(), H.kl.lam.end(), out);
        return SG_OK;
      case SG_EXPORT_GQ:
        need(H.kl.gq.size());
        std::copy(H.kl.gq.begin(), H.kl.gq.end(), out);
        return SG_OK;
      case SG_EXPORT_GROUPS: {
        if (level < 0 || level >= SG_GROUP_COUNT) throw Error(SG_ERR_INVALID_ARG, "grouping out of range");
        std::vector<double> v;
        v.push_back((double)H.fs[level].splits.size());
        for (auto& sp : H.fs[level].splits) {
          v.push_back((double)sp.size());
          for (int i : sp) v.push_back(i);
        }
        need(v.size());
        std::copy(v.begin(), v.end(), out);
        return SG_OK;
      }
      case SG_EXPORT_BLOCKS: {
        if (level < 0 || level >= SG_GROUP_COUNT) throw Error(SG_ERR_INVALID_ARG, "grouping out of range");
        const size_t S = H.fs[level].splits.size();
        need(1 + S);
        out[0] = (double)S;
        for (size_t sp = 0; sp < S; ++sp)
          out[1 + sp] = (H.use_factored && H.use_rapply && sp < H.rkv[level].size())
                            ? (double)H.rkv[level][sp]
                            : 0.0;
        return SG_OK;
      }
      case SG_EXPORT_COEFF: {
        if (!H.bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
        need((size_t)H.na * H.Nq);
        std::vector<double> tiled((size_t)H.na * H.Nq);
        SG_HIP(hipMemcpy(tiled.data(), H.d.a, tiled.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int k = 0; k < H.na; ++k)
          for (int ey = 0; ey < H.n; ++ey)
            for (int ex = 0; ex < H.n; ++ex)
              for (int qy = 0; qy < 2; ++qy)
                for (int qx = 0; qx < 2; ++qx)
                  out[(size_t)k * H.Nq + 4 * ((size_t)ey * H.n + ex) + 2 * qy + qx] =
                      tiled[(size_t)k * H.Nq + tiled_q(H.n, ex, ey, qx, qy)];
        return SG_OK;
      }
      case SG_EXPORT_STENCIL: {
        if (!H.bound) return fail(SG_ERR_NOT_BOUND, "handle not bound");
        if (level < 0 || level >= (int)H.d.L.size()) throw Error(SG_ERR_INVALID_ARG, "level out of range");
        need(9 * (size_t)H.d.L[level].N);
        SG_HIP(hipMemcpy(out, H.d.L[level].S, 9 * H.d.L[level].N * sizeof(double), hipMemcpyDeviceToHost));
        return SG_OK;
      }
      default:
        return fail(SG_ERR_INVALID_ARG, "unknown export");
    }
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

void sg_destroy(sg_handle* h) { delete h; }

}  // extern "C"

// ===========================================================================
// Batched solves: many instances of uneven size advanced in lockstep by
// kernels over device work-item tables (one launch per step kernel covers every
// instance); one Arnoldi step of every instance and the restart step are each
// captured once in a HIP graph.
// ===========================================================================
#include <fstream>
#include <map>
#include <sstream>

namespace {

struct KPtr {
  double *V, *w, *z, *t, *partial, *H, *cs, *sn, *g, *y, *hv;
  int* ident;
  int nblk;
};

struct LaunchRec {
  int kind;       // BK_*
  int64_t off;    // offset of the work items in the item array
  int count;      // work items
  int gate;       // 0: instances in the current cycle, 1: instances not done
  int a0, a1, a2, a3, a4;
  double d0, d1;
  size_t lds;
};

enum {
  BK_APPLY = 0, BK_FIXUP, BK_VDOWN, BK_VUP, BK_VCOARSE, BK_GATHER, BK_VEC, BK_DOT, BK_REDUCE,
  BK_GIVENS, BK_SOLVE, BK_INIT, BK_FAPPLY, BK_RAPPLY
};

struct Plan {
  std::vector<BItem> items;
  std::vector<LaunchRec> step, restart, start;
  std::vector<BInst> inst;
  hipGraphExec_t gstep = nullptr, grestart = nullptr;
};

}  // namespace

struct sg_batch {
  std::vector<sg_handle*> h;
  int count = 0, restart = 0;
  bool bound = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<int64_t> voff;
  std::vector<KPtr> kp;
  BInst* dI = nullptr;
  BState* dS = nullptr;
  BItem* dItems = nullptr;
  size_t item_cap = 0;
  BState* hS = nullptr;  // pinned
  char* solo_ws = nullptr;  // Krylov workspaces (kSoloStreams of solo_bytes) of the
                            // instances solved one at a time
  size_t solo_bytes = 0;
  char* tail_ws = nullptr;  // ... of the lockstep instances that finish one at a time
  size_t tail_bytes = 0;
  std::map<int, Plan> plans;
  ~sg_batch() {
    for (auto& kv : plans) {
      if (kv.second.gstep) (void)hipGraphExecDestroy(kv.second.gstep);
      if (kv.second.grestart) (void)hipGraphExecDestroy(kv.second.grestart);
    }
    for (auto* x : h) sg_destroy(x);
    if (hS) (void)hipHostFree(hS);
  }
};

namespace {

constexpr size_t kBatchItemCap = 1 << 24;  // work items of all tables of one plan
constexpr int kBatchTail = 4;  // instances left when a solve continues them one at a time
// instances with at least this many unknowns fill the chip with their own
// kernels: a batched solve on a stream runs them through the single-instance
// solver beside the lockstep batch of the others, kSoloStreams at a time
// (their kernels are short enough that one instance alone leaves the chip
// idle between launches)
constexpr int64_t kBatchSoloUnknowns = int64_t(1) << 20;
constexpr int kSoloStreams = 3;

int cdivi(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

size_t batch_layout(sg_batch& B, char* base) {
  Carver c{base};
  B.kp.assign(B.count, KPtr{});
  for (int i = 0; i < B.count; ++i) {
    sg_handle& H = *B.h[i];
    const size_t hb = sg_workspace_bytes(&H);
    char* hbase = c.take<char>(hb);
    if (base) {
      H.ws = hbase;
      H.ws_bytes = hb;
    }
  }
  for (int i = 0; i < B.count; ++i) {
    const sg_handle& H = *B.h[i];
    const int64_t Nv = (int64_t)H.P * H.Nh;
    const int m = B.restart;
    KPtr& k = B.kp[i];
    k.nblk = dot_blocks(Nv);
    k.V = c.take<double>((size_t)(m + 1) * Nv);
    k.w = c.take<double>(Nv);
    k.z = c.take<double>(Nv);
    k.t = c.take<double>(Nv);
    k.partial = c.take<double>((size_t)k.nblk * (m + 1));
    k.H = c.take<double>((size_t)(m + 1) * m);
    k.cs = c.take<double>(m);
    k.sn = c.take<double>(m);
    k.g = c.take<double>(m + 1);
    k.y = c.take<double>(m + 1);
    k.hv = c.take<double>(2 * (size_t)(m + 1) + 2);
    k.ident = c.take<int>(H.P);
  }
  B.dI = c.take<BInst>(B.count);
  B.dS = c.take<BState>(B.count);
  B.dItems = c.take<BItem>(kBatchItemCap);
  B.item_cap = kBatchItemCap;
  // Krylov workspaces for the instances a solve runs one at a time: the
  // largest instance's need, and the largest below the solo size (the tail of
  // the lockstep batch, which may run beside the solo instances)
  size_t solo = 0, tail = 0;
  for (int i = 0; i < B.count; ++i) {
    const size_t kb = krylov_layout(B.h[i], B.restart, false, nullptr, nullptr);
    solo = std::max(solo, kb);
    if ((int64_t)B.h[i]->P * B.h[i]->Nh < kBatchSoloUnknowns) tail = std::max(tail, kb);
  }
  solo = (solo + 255) & ~size_t(255);  // each of the kSoloStreams areas 256-byte aligned
  char* sw = c.take<char>(solo * kSoloStreams);
  char* tw = c.take<char>(tail);
  if (base) {
    B.solo_ws = sw;
    B.solo_bytes = solo;
    B.tail_ws = tw;
    B.tail_bytes = tail;
  }
  return c.off;
}

// Builds the descriptors, work-item tables and launch sequences for one
// preconditioner (mean-based, or field split with a grouping).
// apply form of an instance in batched solves: 2 register-resident, 1 factored
// in LDS tiles, 0 triple products
int batch_form(const sg_handle& H) {
  if (!H.use_factored) return 0;
  return H.use_rapply ? 2 : 1;
}

// live (may be null): instances whose work items the plan holds; the others'
// descriptors stay (items name instances by index) but none of their work is
// launched, which is what their device gates would skip anyway
Plan build_plan(sg_batch& B, int pc_kind, int grouping, const double* F, double* u,
                const std::vector<char>* live = nullptr) {
  Plan pl;
  auto skip = [&](int i) { return live && !(*live)[i]; };
  const int m = B.restart;
  int maxS = 0, maxfine = 0;
  pl.inst.resize(B.count);
  for (int i = 0; i < B.count; ++i) {
    sg_handle& H = *B.h[i];
    const DevPtrs& D = H.d;
    const KPtr& k = B.kp[i];
    BInst& I = pl.inst[i];
    std::memset(&I, 0, sizeof(I));
    I.n = H.n;
    I.P = H.P;
    I.na = H.na;
    I.nlev = (int)D.L.size();
    I.nfine = H.nfine;
    I.m = m;
    I.nblk = k.nblk;
    I.Nh = H.Nh;
    I.Nv = (int64_t)H.P * H.Nh;
    I.a = D.a;
    I.full = D.full;
    I.form = batch_form(H);
    I.M = H.M;
    I.pdeg = H.prob.p;
    I.mu = H.prob.mu;
    I.amin = H.prob.a_min;
    I.gq = D.g;
    if (H.factored_ok) I.ffull = D.ffull;
    if (H.rapply_ok) I.rfull = H.rfull;
    if (I.nlev > kMaxLevelsB) throw Error(SG_ERR_UNSUPPORTED, "batch: too many grid levels");
    for (int l = 0; l < I.nlev; ++l) {
      I.L[l] = D.L[l];
      I.mg_b[l] = D.mg_b[l];
      I.mg_x[l] = D.mg_x[l];
      I.mg_xa[l] = D.mg_xa[l];
    }
    if (pc_kind == SG_PC_MEAN) {
      I.nsplit = 1;
      I.split_idx[0] = k.ident;
      I.split_m[0] = H.P;
    } else {
      const FSHost& fh = H.fs[grouping];
      I.nsplit = (int)fh.splits.size();
      if (I.nsplit > kMaxSplitsB) throw Error(SG_ERR_UNSUPPORTED, "batch: too many splits");
      for (int s = 0; s < I.nsplit; ++s) {
        I.split_idx[s] = D.fs[grouping].split_idx[s];
        I.split_m[s] = (int)fh.splits[s].size();
        if (s >= 1) I.part[s] = D.fs[grouping].partial[s];
        if (s >= 1 && H.factored_ok) I.fpart[s] = D.fs[grouping].fpartial[s];
        if (s >= 1 && H.rapply_ok) I.rpart[s] = H.rpart[grouping][s];
      }
    }
    I.edge = D.edge;
    I.fsT = D.fsT;
    I.fsX = D.fsX;
    I.F = F + B.voff[i];
    I.u = u + B.voff[i];
    I.V = k.V;
    I.w = k.w;
    I.z = k.z;
    I.t = k.t;
    I.partial = k.partial;
    I.H = k.H;
    I.cs = k.cs;
    I.sn = k.sn;
    I.g = k.g;
    I.y = k.y;
    I.hv = k.hv;
    maxS = std::max(maxS, I.nsplit);
    maxfine = std::max(maxfine, I.nfine);
  }
  auto rec = [&](int kind, const std::vector<BItem>& t, int gate) {
    LaunchRec r{};
    r.kind = kind;
    r.off = (int64_t)pl.items.size();
    r.count = (int)t.size();
    r.gate = gate;
    pl.items.insert(pl.items.end(), t.begin(), t.end());
    return r;
  };
  std::vector<BItem> tvec, tdot;
  for (int i = 0; i < B.count; ++i) {
    if (skip(i)) continue;
    const BInst& I = pl.inst[i];
    for (int c = 0; c < cdivi(I.Nv, kVecChunk); ++c) tvec.push_back({i, c});
    for (int b = 0; b < I.nblk; ++b) tdot.push_back({i, b});
  }
  // operator launches for a row set (0 = full, s = partial of split s): one
  // launch per rows-per-wavefront class, then the edge fixup
  auto apply_recs = [&](int rowset, int src, int rin, int dst, double beta, double sgn, int gate,
                        std::vector<LaunchRec>& out) {
    // class of an instance: (form, rows per wavefront | sub-batch size | M * 16 + p)
    std::map<std::pair<int, int>, std::pair<std::vector<BItem>, size_t>> classes;
    std::vector<BItem> tfix;
    for (int i = 0; i < B.count; ++i) {
      const BInst& I = pl.inst[i];
      if (skip(i) || (rowset > 0 && rowset >= I.nsplit)) continue;
      const RowSetDev& rs = rowset == 0 ? I.full : I.part[rowset];
      std::pair<int, int> key;
      size_t lds;
      if (I.form == 2) {
        const RApplyRows& rr = rowset == 0 ? I.rfull : I.rpart[rowset];
        key = {2, I.M * 16 + I.pdeg};
        lds = rapply_lds_bytes(I.P, rr.nrows);
      } else if (I.form == 1) {
        const FRowSetDev& f = rowset == 0 ? I.ffull : I.fpart[rowset];
        key = {1, f.qb};
        lds = fapply_lds_bytes(f.qb, f.nrows, f.ncols, f.ngam, f.nmono, f.M, f.nblob);
      } else {
        key = {0, rs.rmax};
        lds = apply_lds_bytes(rs.maxcols, rs.kc, rs.maxent);
      }
      auto& cl = classes[key];
      const int nt = I.n / kTileE;
      // XCD-aware order: workgroup w runs on XCD w mod 8 and per-instance tile
      // counts are multiples of 8 at the workload sizes, so each XCD walks a
      // contiguous band of tiles and their shared halo lines stay in one L2
      for (int t = 0; t < nt * nt; ++t) cl.first.push_back({i, xcd_tile(t, nt * nt)});
      cl.second = std::max(cl.second, lds);
      const int64_t fixn = (int64_t)rs.nrows * nt * nt * 7;
      for (int c = 0; c < cdivi(fixn, kVecChunk); ++c) tfix.push_back({i, c});
    }
    for (auto& kv : classes) {
      const int kind = kv.first.first == 0 ? BK_APPLY : kv.first.first == 1 ? BK_FAPPLY : BK_RAPPLY;
      LaunchRec r = rec(kind, kv.second.first, gate);
      r.a0 = kv.first.second;
      r.a1 = rowset;
      r.a2 = src;
      r.a3 = rin;
      r.a4 = dst;
      r.d0 = beta;
      r.d1 = sgn;
      r.lds = kv.second.second;
      out.push_back(r);
    }
    LaunchRec fx = rec(BK_FIXUP, tfix, gate);
    fx.a0 = rowset;
    fx.a1 = dst;
    fx.d0 = sgn;
    out.push_back(fx);
  };
  size_t coarse_lds = 0;
  for (int i = 0; i < B.count; ++i) {
    const BInst& I = pl.inst[i];
    CoarseLevels cl{};
    cl.nl = I.nlev - I.nfine;
    for (int l = 0; l < cl.nl; ++l) cl.N[l] = I.L[I.nfine + l].N;
    coarse_lds = std::max(coarse_lds, vcoarse_lds_bytes(cl));
  }
  // preconditioner src -> dst: forward block Gauss-Seidel over the splits
  auto fs_recs = [&](int src, int dst, int gate, std::vector<LaunchRec>& out) {
    for (int s = 0; s < maxS; ++s) {
      std::vector<BItem> tsplit, tcoarse;
      std::vector<std::vector<BItem>> tdepth(maxfine);
      for (int i = 0; i < B.count; ++i) {
        const BInst& I = pl.inst[i];
        if (skip(i) || s >= I.nsplit) continue;
        const int ms = I.split_m[s];
        for (int c = 0; c < cdivi((int64_t)ms * I.Nh, kVecChunk); ++c) tsplit.push_back({i, c});
        for (int md = 0; md < ms; ++md) tcoarse.push_back({i, md});
        for (int d = 0; d < I.nfine; ++d) {
          const int tpr = (I.L[d].n / 2 + 7) / 8;
          for (int t = 0; t < tpr * tpr * ms; ++t) tdepth[d].push_back({i, t});
        }
      }
      if (s == 0) {
        LaunchRec g = rec(BK_GATHER, tsplit, gate);
        g.a0 = s;
        g.a1 = src;
        g.a2 = 0;
        out.push_back(g);
      } else {
        apply_recs(s, dst, src, BUF_FST, 1.0, -1.0, gate, out);
      }
      for (int d = 0; d < maxfine; ++d) {
        LaunchRec r = rec(BK_VDOWN, tdepth[d], gate);
        r.a0 = d;
        r.a1 = s;
        out.push_back(r);
      }
      LaunchRec c = rec(BK_VCOARSE, tcoarse, gate);
      c.a0 = s;
      c.lds = coarse_lds;
      out.push_back(c);
      for (int d = maxfine - 1; d >= 0; --d) {
        LaunchRec r = rec(BK_VUP, tdepth[d], gate);
        r.a0 = d;
        r.a1 = s;
        out.push_back(r);
      }
      LaunchRec g = rec(BK_GATHER, tsplit, gate);
      g.a0 = s;
      g.a1 = dst;
      g.a2 = 1;
      out.push_back(g);
    }
  };
  auto vec = [&](int op, int x, int y, int o, double a, double b, int gate) {
    LaunchRec r = rec(BK_VEC, tvec, gate);
    r.a0 = op;
    r.a1 = x;
    r.a2 = y;
    r.a3 = o;
    r.d0 = a;
    r.d1 = b;
    return r;
  };
  auto dot = [&](int self_buf, int gate) {
    LaunchRec r = rec(BK_DOT, tdot, gate);
    r.a0 = self_buf;
    return r;
  };
  auto reduce = [&](int which, int gate) {
    LaunchRec r = rec(BK_REDUCE, {}, gate);
    r.a0 = which;
    return r;
  };
  auto simple = [&](int kind, int a0) {
    LaunchRec r = rec(kind, {}, 0);
    r.a0 = a0;
    return r;
  };
  // first start: u = 0, t = F, beta = ||F||, V_0 = t / beta
  pl.start.push_back(vec(BV_AXPBY, BUF_U, BUF_U, BUF_U, 0.0, 0.0, 1));
  pl.start.push_back(vec(BV_AXPBY, BUF_F, BUF_F, BUF_T, 1.0, 0.0, 1));
  pl.start.push_back(dot(BUF_T, 1));
  pl.start.push_back(reduce(2, 1));
  pl.start.push_back(simple(BK_INIT, 1));
  pl.start.push_back(vec(BV_START, 0, 0, 0, 0, 0, 0));
  // one Arnoldi step: z = P^{-1} v_j, w = K z, CGS2, Givens
  fs_recs(BUF_VJ, BUF_Z, 0, pl.step);
  apply_recs(0, BUF_Z, -1, BUF_W, 0.0, 1.0, 0, pl.step);
  pl.step.push_back(dot(-1, 0));
  pl.step.push_back(reduce(0, 0));
  pl.step.push_back(vec(BV_UPDATE1, 0, 0, 0, 0, 0, 0));
  pl.step.push_back(dot(-1, 0));
  pl.step.push_back(reduce(1, 0));
  pl.step.push_back(vec(BV_UPDATE2, 0, 0, 0, 0, 0, 0));
  pl.step.push_back(dot(BUF_W, 0));
  pl.step.push_back(reduce(2, 0));
  pl.step.push_back(vec(BV_SCALE_NEXT, 0, 0, 0, 0, 0, 0));
  pl.step.push_back(simple(BK_GIVENS, 0));
  // restart: y, u += P^{-1}(V y), t = F - K u, beta, next cycle
  pl.restart.push_back(simple(BK_SOLVE, 0));
  pl.restart.push_back(vec(BV_COMBINE, 0, 0, 0, 0, 0, 1));
  fs_recs(BUF_T, BUF_Z, 1, pl.restart);
  pl.restart.push_back(vec(BV_AXPBY, BUF_Z, BUF_U, BUF_U, 1.0, 1.0, 1));
  apply_recs(0, BUF_U, -1, BUF_W, 0.0, 1.0, 1, pl.restart);
  pl.restart.push_back(vec(BV_AXPBY, BUF_F, BUF_W, BUF_T, 1.0, -1.0, 1));
  pl.restart.push_back(dot(BUF_T, 1));
  pl.restart.push_back(reduce(2, 1));
  pl.restart.push_back(simple(BK_INIT, 0));
  pl.restart.push_back(vec(BV_START, 0, 0, 0, 0, 0, 0));
  if (pl.items.size() > B.item_cap) throw Error(SG_ERR_UNSUPPORTED, "batch: too many work items");
  return pl;
}

void run_recs(sg_batch& B, hipStream_t s, const std::vector<LaunchRec>& recs, double tol) {
  for (const LaunchRec& r : recs) {
    const BItem* it = B.dItems + r.off;
    switch (r.kind) {
      case BK_APPLY:
        launch_bapply(s, r.a0, r.lds, B.dI, B.dS, it, r.count, r.a1, r.a2, r.a3, r.a4, r.d0, r.d1,
                      r.gate);
        break;
      case BK_FAPPLY:
        launch_bfapply(s, r.a0, r.lds, B.dI, B.dS, it, r.count, r.a1, r.a2, r.a3, r.a4, r.d0,
                       r.d1, r.gate);
        break;
      case BK_RAPPLY:
        launch_brapply(s, r.a0 / 16, r.a0 % 16, r.lds, B.dI, B.dS, it, r.count, r.a1, r.a2,
                       r.a3, r.a4, r.d0, r.d1, r.gate);
        break;
      case BK_FIXUP: launch_bfixup(s, B.dI, B.dS, it, r.count, r.a0, r.a1, r.d0, r.gate); break;
      case BK_VDOWN: launch_bvdown(s, B.dI, B.dS, it, r.count, r.a0, r.a1, r.gate); break;
      case BK_VUP: launch_bvup(s, B.dI, B.dS, it, r.count, r.a0, r.a1, r.gate); break;
      case BK_VCOARSE: launch_bvcoarse(s, r.lds, B.dI, B.dS, it, r.count, r.a0, r.gate); break;
      case BK_GATHER: launch_bgather(s, B.dI, B.dS, it, r.count, r.a0, r.a1, r.a2, r.gate); break;
      case BK_VEC:
        launch_bvec(s, B.dI, B.dS, it, r.count, r.a0, r.a1, r.a2, r.a3, r.d0, r.d1, r.gate);
        break;
      case BK_DOT: launch_bmultidot(s, B.dI, B.dS, it, r.count, r.a0, r.gate); break;
      case BK_REDUCE: launch_breduce(s, B.dI, B.dS, B.count, r.a0, r.gate); break;
      case BK_GIVENS: launch_bgivens(s, B.dI, B.dS, B.count); break;
      case BK_SOLVE: launch_bsolve(s, B.dI, B.dS, B.count); break;
      case BK_INIT: launch_binit(s, B.dI, B.dS, B.count, r.a0, tol); break;
      default: throw Error(SG_ERR_INTERNAL, "batch: unknown launch");
    }
  }
}

hipGraphExec_t capture(sg_batch& B, hipStream_t s, const std::vector<LaunchRec>& recs,
                       double tol) {
  hipGraph_t g = nullptr;
  SG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  try {
    run_recs(B, s, recs, tol);
  } catch (...) {
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  SG_HIP(hipStreamEndCapture(s, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess)
    throw Error(SG_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return ex;
}

// ---- autotuner: the apply form and tile shape of each problem class --------
// Candidates are the forms the batched step kernels run for an instance:
//   kTuneRegister          the register-resident factored kernel (one tile of
//                          4x4 elements per workgroup, every mode in registers)
//   kTuneTile + qb         the factored LDS tile kernel with qb Gauss points
//                          per sub-batch (qb = 8, 16, 32, 64)
//   kTuneTriple + kc       the triple-product form streaming kc coefficient
//                          modes per chunk (kc = 16, 32, 48, 64)
// A class is (device, M, p, q); it is timed on a grid of min(n, 128) elements
// per side (1024 tiles: the kernels' relative speed at full occupancy, in
// milliseconds per candidate), 10 applies per candidate.
constexpr int kTuneRegister = 1, kTuneTile = 100, kTuneTriple = 200;

std::string tune_cache_path() {
  const char* p = getenv("SG_AUTOTUNE_CACHE");
  if (p && *p) return p;
  const char* home = getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.sgfs_autotune.txt";
}

std::map<std::string, int> tune_load() {
  std::map<std::string, int> m;
  std::ifstream f(tune_cache_path());
  std::string key;
  int code;
  while (f >> key >> code) m[key] = code;
  return m;
}

void tune_store(const std::map<std::string, int>& m) {
  std::ofstream f(tune_cache_path());
  for (auto& kv : m) f << kv.first << ' ' << kv.second << '\n';
}

std::string tune_key(const sg_problem& p) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ':' || c == ' ') c = '_';
  std::ostringstream o;
  o << arch << "_M" << p.M << "_p" << p.p << "_q" << p.q << "_form";
  return o.str();
}

// Puts an unbound handle's apply in the form of a tuner code; false when the
// form does not exist for this problem (the handle's form is then unchanged).
bool set_form(sg_handle* h, int code) {
  if (code == kTuneRegister)
    return sg_set_apply(h, SG_APPLY_FACTORED, 0, nullptr) == SG_OK && h->use_rapply;
  if (code > kTuneTile && code < kTuneTriple)
    return sg_set_apply(h, SG_APPLY_FACTORED, code - kTuneTile, nullptr) == SG_OK;
  if (code > kTuneTriple)
    return h->full.kc == code - kTuneTriple && sg_set_apply(h, SG_APPLY_TRIPLE, 0, nullptr) == SG_OK;
  return false;
}

// The tuner code of the form a handle's apply uses.
int form_code(const sg_handle& H) {
  if (H.use_factored && H.use_rapply) return kTuneRegister;
  if (H.use_factored) return kTuneTile + H.ffull.qb;
  return kTuneTriple + H.full.kc;
}

// Times one apply of every candidate form on scratch device memory; returns
// the fastest candidate's code (0 if none could be timed).
int tune_apply(const sg_problem& prob, float* best_ms_out) {
  sg_problem tp = prob;
  tp.n = std::min(prob.n, 128);
  std::vector<int> cands = {kTuneRegister};
  for (int qb : {64, 32, 16, 8}) cands.push_back(kTuneTile + qb);
  for (int kc : {16, 32, 48, 64}) cands.push_back(kTuneTriple + kc);
  int best = 0;
  float best_ms = 1e30f;
  for (int code : cands) {
    sg_handle* h = nullptr;
    const int kc = code > kTuneTriple ? code - kTuneTriple : 0;
    if (setup_impl(&tp, nullptr, kc, &h) != SG_OK) continue;
    std::unique_ptr<sg_handle> hold(h);
    if (!set_form(h, code)) continue;
    const size_t wb = sg_workspace_bytes(h);
    const int64_t Nv = (int64_t)h->P * h->Nh;
    void* ws = nullptr;
    double* v = nullptr;
    if (hipMalloc(&ws, wb + 256) != hipSuccess) continue;
    if (hipMalloc((void**)&v, 2 * Nv * sizeof(double)) != hipSuccess) {
      (void)hipFree(ws);
      continue;
    }
    char* aligned =
        reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
    float ms = 1e30f;
    if (sg_bind(h, aligned, wb, nullptr) == SG_OK &&
        hipMemset(v, 0, 2 * Nv * sizeof(double)) == hipSuccess) {
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        (void)sg_apply(h, v, v + Nv, nullptr);
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < 10; ++r) (void)sg_apply(h, v, v + Nv, nullptr);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
      }
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(v);
    (void)hipFree(ws);
    if (ms < best_ms) {
      best_ms = ms;
      best = code;
    }
  }
  if (best_ms_out) *best_ms_out = best_ms / 10;
  return best;
}

}  // namespace

extern "C" {

int sg_autotune_apply(const sg_problem* prob, int32_t* best_form, float* best_ms) {
  if (!prob || !best_form) return fail(SG_ERR_INVALID_ARG, "null argument");
  try {
    validate(*prob);
    *best_form = tune_apply(*prob, best_ms);
    if (*best_form <= 0) return fail(SG_ERR_HIP, "no candidate could be timed");
    std::map<std::string, int> cache = tune_load();
    cache[tune_key(*prob)] = *best_form;
    tune_store(cache);
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_batch_create(int32_t count, const sg_problem* probs, const double* const* f_nodal,
                    int32_t autotune, sg_batch** out) {
  if (!probs || !out || count < 1) return fail(SG_ERR_INVALID_ARG, "need count >= 1 and problems");
  *out = nullptr;
  try {
    auto B = std::make_unique<sg_batch>();
    B->count = count;
    std::map<std::string, int> cache;
    bool dirty = false;
    if (autotune) cache = tune_load();
    for (int i = 0; i < count; ++i) {
      validate(probs[i]);
      int code = 0;
      if (autotune) {
        const std::string key = tune_key(probs[i]);
        auto itc = cache.find(key);
        if (itc != cache.end()) {
          code = itc->second;
        } else {
          code = tune_apply(probs[i], nullptr);
          cache[key] = code;
          dirty = true;
        }
      }
      sg_handle* h = nullptr;
      const double* f = f_nodal ? f_nodal[i] : nullptr;
      const int kc = code > kTuneTriple ? code - kTuneTriple : 0;
      int rc = setup_impl(&probs[i], f, kc, &h);
      if (rc != SG_OK && kc != 0) rc = setup_impl(&probs[i], f, 0, &h);
      if (rc != SG_OK) return rc;
      // the tuned form where it exists for this instance, else the default
      if (code && !set_form(h, code)) (void)sg_set_apply(h, SG_APPLY_AUTO, 0, nullptr);
      B->h.push_back(h);
    }
    if (dirty) tune_store(cache);
    B->voff.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) B->voff[i + 1] = B->voff[i] + (int64_t)B->h[i]->P * B->h[i]->Nh;
    *out = B.release();
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_batch_layout(const sg_batch* b, int64_t* offsets, int32_t* form) {
  if (!b || !offsets) return fail(SG_ERR_INVALID_ARG, "null argument");
  for (int i = 0; i <= b->count; ++i) offsets[i] = b->voff[i];
  if (form)
    for (int i = 0; i < b->count; ++i) form[i] = form_code(*b->h[i]);
  return SG_OK;
}

size_t sg_batch_workspace_bytes(const sg_batch* b, int32_t restart) {
  if (!b || restart < 1 || restart > kMaxRestart) return 0;
  sg_batch& B = const_cast<sg_batch&>(*b);
  const int keep = B.restart;
  std::vector<KPtr> kp = B.kp;
  B.restart = restart;
  const size_t n = batch_layout(B, nullptr);
  B.restart = keep;
  B.kp = kp;
  return n;
}

int sg_batch_bind(sg_batch* b, int32_t restart, void* ws, size_t bytes, void* stream) {
  if (!b || !ws) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (restart < 1 || restart > kMaxRestart) return fail(SG_ERR_INVALID_ARG, "restart out of range");
  if (bytes < sg_batch_workspace_bytes(b, restart))
    return fail(SG_ERR_WORKSPACE, "batch workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(SG_ERR_WORKSPACE, "batch workspace must be 256-byte aligned");
  try {
    sg_batch& B = *b;
    for (auto& kv : B.plans) {
      if (kv.second.gstep) (void)hipGraphExecDestroy(kv.second.gstep);
      if (kv.second.grestart) (void)hipGraphExecDestroy(kv.second.grestart);
    }
    B.plans.clear();
    B.restart = restart;
    B.ws = static_cast<char*>(ws);
    B.ws_bytes = bytes;
    batch_layout(B, B.ws);
    for (int i = 0; i < B.count; ++i) {
      int rc = sg_bind(B.h[i], B.h[i]->ws, B.h[i]->ws_bytes, stream);
      if (rc != SG_OK) return rc;
      std::vector<int> ident(B.h[i]->P);
      std::iota(ident.begin(), ident.end(), 0);
      SG_HIP(hipMemcpy(B.kp[i].ident, ident.data(), ident.size() * sizeof(int),
                       hipMemcpyHostToDevice));
    }
    if (!B.hS) SG_HIP(hipHostMalloc((void**)&B.hS, sizeof(BState) * B.count, hipHostMallocDefault));
    B.bound = true;
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int sg_batch_rhs(sg_batch* b, double* F, void* stream) {
  if (!b || !F) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!b->bound) return fail(SG_ERR_NOT_BOUND, "batch not bound");
  for (int i = 0; i < b->count; ++i) {
    int rc = sg_rhs(b->h[i], F + b->voff[i], stream);
    if (rc != SG_OK) return rc;
  }
  return SG_OK;
}

int sg_batch_handle(sg_batch* b, int32_t i, sg_handle** h) {
  if (!b || !h || i < 0 || i >= b->count) return fail(SG_ERR_INVALID_ARG, "index out of range");
  *h = b->h[i];
  return SG_OK;
}

int sg_batch_solve(sg_batch* b, const sg_solve_opts* o, const double* F, double* u,
                   sg_solve_info* infos, void* stream) {
  if (!b || !o || !F || !u || !infos) return fail(SG_ERR_INVALID_ARG, "null argument");
  if (!b->bound) return fail(SG_ERR_NOT_BOUND, "batch not bound");
  if (o->restart != b->restart) return fail(SG_ERR_INVALID_ARG, "restart must match the bound value");
  const int kind = o->pc & 0xff;
  if ((kind != SG_PC_MEAN && kind != SG_PC_FS) || (o->pc & ~(0xff | SG_PC_SWITCH_KII)))
    return fail(SG_ERR_UNSUPPORTED, "batched solves take the mean-based or field-split preconditioner");
  if (o->grouping < 0 || o->grouping >= SG_GROUP_COUNT) return fail(SG_ERR_INVALID_ARG, "unknown grouping");
  if (o->use_x0) return fail(SG_ERR_UNSUPPORTED, "batched solves start from zero");
  if (!(o->tol > 0.0) || o->max_it < 1) return fail(SG_ERR_INVALID_ARG, "need tol > 0 and max_it >= 1");
  try {
    sg_batch& B = *b;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int key = kind * 16 + (kind == SG_PC_FS ? o->grouping : 0);
    auto itp = B.plans.find(key);
    // a plan is rebuilt when the buffers or an instance's apply form changed
    auto forms_changed = [&](const Plan& pl) {
      for (int i = 0; i < B.count; ++i) {
        const sg_handle& Hi = *B.h[i];
        const int f = batch_form(Hi);
        if (pl.inst[i].form != f || (f == 1 && pl.inst[i].ffull.qb != Hi.d.ffull.qb)) return true;
      }
      return false;
    };
    if (itp != B.plans.end() && (itp->second.inst[0].F != F || itp->second.inst[0].u != u ||
                                 forms_changed(itp->second))) {
      if (itp->second.gstep) (void)hipGraphExecDestroy(itp->second.gstep);
      if (itp->second.grestart) (void)hipGraphExecDestroy(itp->second.grestart);
      B.plans.erase(itp);
      itp = B.plans.end();
    }
    if (itp == B.plans.end())
      itp = B.plans.emplace(key, build_plan(B, kind, o->grouping, F, u)).first;
    Plan& pl = itp->second;
    // descriptors and work items, stream-ordered before any use
    SG_HIP(hipMemcpyAsync(B.dI, pl.inst.data(), pl.inst.size() * sizeof(BInst),
                          hipMemcpyHostToDevice, s));
    SG_HIP(hipMemcpyAsync(B.dItems, pl.items.data(), pl.items.size() * sizeof(BItem),
                          hipMemcpyHostToDevice, s));
    // one Arnoldi step and the restart are captured once per plan (needs a
    // non-null stream; on the null stream the same sequences run eagerly)
    const bool graphs = (s != nullptr);
    // instances whose kernels fill the chip run one at a time through the
    // single-instance solver on a second stream, beside the lockstep batch of
    // the others (on a stream only; all of them, if every instance is large)
    std::vector<char> solo(B.count, 0);
    int nsolo = 0;
    if (graphs)
      for (int i = 0; i < B.count; ++i)
        if ((int64_t)B.h[i]->P * B.h[i]->Nh >= kBatchSoloUnknowns) nsolo += (solo[i] = 1);
    for (int i = 0; i < B.count; ++i) {
      BState st{};
      st.max_it = o->max_it;
      if (solo[i]) {  // gated off in every batched kernel
        st.done = 1;
        st.status = SG_NOT_CONVERGED;
      }
      B.hS[i] = st;
    }
    SG_HIP(hipMemcpyAsync(B.dS, B.hS, sizeof(BState) * B.count, hipMemcpyHostToDevice, s));
    SG_HIP(hipStreamSynchronize(s));
    // the solo instances' solves: up to kSoloStreams host threads, each with
    // a stream (default priority) and a Krylov area of its own, take the
    // instances largest first from a shared counter (joined on every way out
    // of this call)
    std::vector<sg_solve_info> solo_info(B.count);
    std::atomic<int> solo_rc{SG_OK};
    std::atomic<int> solo_next{0};
    std::mutex solo_mu;
    std::string solo_err;
    std::vector<int> solo_order;
    for (int i = 0; i < B.count; ++i)
      if (solo[i]) solo_order.push_back(i);
    std::stable_sort(solo_order.begin(), solo_order.end(), [&](int a, int b) {
      return (int64_t)B.h[a]->P * B.h[a]->Nh > (int64_t)B.h[b]->P * B.h[b]->Nh;
    });
    std::vector<hipStream_t> s2;
    std::vector<std::thread> solo_threads;
    struct Joiner {
      std::vector<std::thread>& t;
      std::vector<hipStream_t>& st;
      ~Joiner() {
        for (auto& th : t)
          if (th.joinable()) th.join();
        for (hipStream_t x : st) (void)hipStreamDestroy(x);
      }
    } joiner{solo_threads, s2};
    const int nthreads = std::min(nsolo, kSoloStreams);
    for (int k = 0; k < nthreads; ++k) {
      hipStream_t x = nullptr;
      SG_HIP(hipStreamCreate(&x));
      s2.push_back(x);
    }
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    for (int k = 0; k < nthreads; ++k) {
      solo_threads.emplace_back([&, k]() {
        if (hipSetDevice(dev) != hipSuccess) {
          solo_rc = SG_ERR_HIP;
          return;
        }
        char* ws = B.solo_ws + (size_t)k * B.solo_bytes;
        for (;;) {
          const int t = solo_next.fetch_add(1);
          if (t >= nsolo || solo_rc.load() != SG_OK) return;
          const int i = solo_order[t];
          sg_solve_opts oi = *o;
          oi.use_x0 = 0;
          const int rc = sg_gmres_solve(B.h[i], &oi, F + B.voff[i], u + B.voff[i], ws,
                                        B.solo_bytes, nullptr, 0, &solo_info[i], s2[k]);
          if (rc != SG_OK) {
            std::lock_guard<std::mutex> lk(solo_mu);
            if (solo_rc.load() == SG_OK) solo_err = sg_last_error();
            solo_rc = rc;
            return;
          }
        }
      });
    }
    // Once a quarter of the instances still running at the last (re)build
    // have finished, the step and restart are rebuilt over the remaining ones
    // (items uploaded, graphs captured again), so the step kernels stop
    // walking the work of finished instances.  The full plan stays cached for
    // the next solve, which uploads its items again.  With solo instances the
    // lockstep starts from such a plan over the others.
    Plan* cur = &pl;
    std::unique_ptr<Plan> compact;
    auto drop_compact = [&]() {
      if (!compact) return;
      if (compact->gstep) (void)hipGraphExecDestroy(compact->gstep);
      if (compact->grestart) (void)hipGraphExecDestroy(compact->grestart);
      compact.reset();
    };
    struct Dropper {
      std::function<void()> f;
      ~Dropper() { f(); }
    } dropper{drop_compact};
    std::vector<char> inbatch(B.count);
    for (int i = 0; i < B.count; ++i) inbatch[i] = !solo[i];
    int live_at_build = B.count - nsolo;
    if (nsolo > 0 && nsolo < B.count) {
      compact.reset(new Plan(build_plan(B, kind, o->grouping, F, u, &inbatch)));
      SG_HIP(hipMemcpyAsync(B.dItems, compact->items.data(), compact->items.size() * sizeof(BItem),
                            hipMemcpyHostToDevice, s));
      SG_HIP(hipStreamSynchronize(s));
      compact->gstep = capture(B, s, compact->step, o->tol);
      compact->grestart = capture(B, s, compact->restart, o->tol);
      cur = compact.get();
    } else if (graphs && !pl.gstep) {
      pl.gstep = capture(B, s, pl.step, o->tol);
      pl.grestart = capture(B, s, pl.restart, o->tol);
    }
    if (nsolo < B.count) run_recs(B, s, cur->start, o->tol);
    check_launch();
    std::vector<sg_solve_info> tail_info(B.count);
    std::vector<char> handed(B.count, 0);
    const int m = B.restart;
    const int max_cycles = o->max_it + 1;
    for (int cycle = 0; cycle < max_cycles && nsolo < B.count; ++cycle) {
      for (int j = 0; j < m; ++j) {
        if (graphs) SG_HIP(hipGraphLaunch(cur->gstep, s));
        else run_recs(B, s, cur->step, o->tol);
        if ((j + 1) % 10 == 0 && j + 1 < m) {
          SG_HIP(hipMemcpyAsync(B.hS, B.dS, sizeof(BState) * B.count, hipMemcpyDeviceToHost, s));
          SG_HIP(hipStreamSynchronize(s));
          bool any = false;
          for (int i = 0; i < B.count; ++i) any = any || B.hS[i].active;
          if (!any) break;
        }
      }
      if (graphs) SG_HIP(hipGraphLaunch(cur->grestart, s));
      else run_recs(B, s, cur->restart, o->tol);
      SG_HIP(hipMemcpyAsync(B.hS, B.dS, sizeof(BState) * B.count, hipMemcpyDeviceToHost, s));
      SG_HIP(hipStreamSynchronize(s));
      check_launch();
      std::vector<char> live(B.count);
      int nlive = 0;
      for (int i = 0; i < B.count; ++i) nlive += (live[i] = !solo[i] && !B.hS[i].done);
      if (nlive == 0) break;
      // The last few instances continue one at a time with the single-instance
      // solver from their current iterate (a restart boundary, so the same
      // method): with so few left, lockstep launches cost more than their own
      // kernels.
      if (nlive <= kBatchTail && nlive < B.count - nsolo) {
        for (int i = 0; i < B.count; ++i) {
          if (!live[i] || o->max_it - B.hS[i].it < 1) continue;
          sg_solve_opts oi = *o;
          oi.use_x0 = 1;
          oi.max_it = o->max_it - B.hS[i].it;
          // (the solo instances' Krylov area, unless they are running)
          char* kws = nsolo > 0 ? B.tail_ws : B.solo_ws;
          const size_t kbytes = nsolo > 0 ? B.tail_bytes : B.solo_bytes;
          const int rc = sg_gmres_solve(B.h[i], &oi, F + B.voff[i], u + B.voff[i], kws, kbytes,
                                        nullptr, 0, &tail_info[i], stream);
          if (rc != SG_OK) return rc;
          handed[i] = 1;
        }
        break;
      }
      if (graphs && 4 * nlive <= 3 * live_at_build) {
        std::unique_ptr<Plan> next(new Plan(build_plan(B, kind, o->grouping, F, u, &live)));
        SG_HIP(hipMemcpyAsync(B.dItems, next->items.data(), next->items.size() * sizeof(BItem),
                              hipMemcpyHostToDevice, s));
        SG_HIP(hipStreamSynchronize(s));
        next->gstep = capture(B, s, next->step, o->tol);
        next->grestart = capture(B, s, next->restart, o->tol);
        drop_compact();
        compact = std::move(next);
        cur = compact.get();
        live_at_build = nlive;
      }
    }
    for (auto& th : solo_threads)
      if (th.joinable()) th.join();
    if (solo_rc.load() != SG_OK) return fail(solo_rc.load(), "solo instance: " + solo_err);
    for (int i = 0; i < B.count; ++i) {
      const BState& st = B.hS[i];
      sg_solve_info& inf = infos[i];
      std::memset(&inf, 0, sizeof(inf));
      if (solo[i]) {
        inf = solo_info[i];
        continue;
      }
      if (handed[i]) {  // lockstep part, then the one-at-a-time part
        inf = tail_info[i];
        inf.iterations += st.it;
        inf.restarts += st.restarts;
        continue;
      }
      inf.status = st.done ? st.status : SG_NOT_CONVERGED;
      inf.iterations = st.it;
      inf.restarts = st.restarts;
      inf.relres = st.nF > 0 ? st.beta / st.nF : 0.0;
      inf.relres_est = st.nF > 0 ? st.est / st.nF : 0.0;
    }
    return SG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(SG_ERR_INTERNAL, e.what());
  }
}

void sg_batch_destroy(sg_batch* b) { delete b; }

}  // extern "C"
