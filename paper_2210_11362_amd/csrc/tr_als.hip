// Host runtime of the TR-ALS library: context, per-mode plans, workspace, the
// Gauss-Seidel sweep driver (Alg. 2 / Alg. 3) and the C ABI of tr_als.h.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>

#include "common.h"
#include "runtime.h"

namespace {

// How mode m's subchain G^{!=m} is split into two partial-subchain tables and
// how the contraction index k (the other modes, memory order) maps onto them.
struct Plan {
  int64_t I = 0, K = 0, L = 1;
  int layout = 0;
  std::vector<int> f1c, f2c;  // cores (0-based, chain order) of each factor
  int64_t K1 = 1, K2 = 1, d1 = 1, m1 = 1, d2 = 1, m2 = 1;
  int Rb = 1, Rmid = 1, Ra = 1;
  // two-stage MTTSP (regime 1): stage-1 group of modes and the stage-2 steps
  int regime = 2;
  int nn = 1;                 // 1: group = slowest modes, 0: fastest modes
  std::vector<int> gcores;    // group cores in chain (= memory) order
  int64_t gK = 1, gM = 1;     // group size and rows of the intermediate
  int gC = 1, gRu = 1, gRc = 1;
  bool reuse_prev = false;    // same group table as the previous mode of the sweep
  // slab contraction (order 3, large ranks; k_slab.hip): mode contracted on
  // MFMA against its core, slab mode absorbed per slab, and the case
  bool slab = false;
  int sk_mode = 0, sl_mode = 0, slab_caseB = 0;
  bool reuse_y = false;       // and the same reduced stage-1 result, still in Y0
  struct Step { int64_t lo, I, hi; int Ru, Rc, core, side; };
  std::vector<Step> steps;
};

}  // namespace

struct tr_als_ctx {
  int N = 0;
  int64_t dims[TR_MAXN] = {0};
  int R[TR_MAXN + 1] = {0};
  int variant = TR_NE;
  int xdt = TR_F32;
  const void* X = nullptr;
  int64_t numel = 0;
  std::vector<double*> user_cores;
  hipStream_t stream = nullptr;
  hipStream_t stream2 = nullptr;             // coefficient-matrix branch (default priority)
  hipStream_t cap_stream = nullptr;          // private stream the sweep graphs are captured on
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* Sinv = nullptr;
  // solve of the mode update: TR_SOLVE_FACTOR (SPD inverse / Cholesky, or the
  // triangular substitution of Alg. 3) or TR_SOLVE_PINV (pseudo-inverse by the
  // Jacobi SVD, singular values <= rcond * max dropped)
  int solve = TR_SOLVE_FACTOR;
  double rcond = 0.0;
  double* pinvw = nullptr;
  double* blkw = nullptr;   // workspace of the blocked SPD inverse (R_n R_{n+1} > 112)
  double* rdiag = nullptr;                   // reciprocal pivots of the Cholesky factor
  // QR variant state (Alg. 3): per-core Q_j (I_j x r_j) and R-cores
  // (R_j x r_j x R_{j+1}), r_j = min(I_j, R_j R_{j+1}); workspace
  double* qQ[TR_MAXN] = {nullptr};
  double* qR[TR_MAXN] = {nullptr};
  int64_t qr_r[TR_MAXN] = {0};
  double *qA = nullptr, *qV = nullptr, *qtau = nullptr, *qRt = nullptr;
  double *qT = nullptr, *qV2 = nullptr, *qQa = nullptr, *qQb = nullptr, *qY0 = nullptr, *qY1 = nullptr, *qW = nullptr;
  // Multi-TTM part shared by a pair of modes within a sweep (see multi_ttm_y)
  double* qZ = nullptr;
  int z_pair = -1, z_prec = -1;
  int64_t z_cd[TR_MAXN] = {};
  double *qG = nullptr, *qL[3] = {nullptr, nullptr, nullptr}, *qLT = nullptr, *qRi = nullptr, *qLp = nullptr,
         *qLt = nullptr, *qshift = nullptr, *qpart = nullptr;
  int64_t qpart_elems = 0;
  // R_n R_{n+1} > 128 (QR-based variants): the large plain FP64 products
  // (Gram of V_n[2], the triangular passes of the Cholesky-QR, Y_[n] Q_0 and
  // the substitution with R_[2]) go through rocBLAS
  rocblas_handle blas = nullptr;
  // captured sweeps, one per (precision, refinement steps)
  hipGraphExec_t graphs[4][5] = {{nullptr}};
  std::string graph_note;   // why the last sweep capture was abandoned (empty if none)
  bool graphs_ok = true;
  double* cores[TR_MAXN] = {nullptr};
  double* gram[TR_MAXN] = {nullptr};
  Plan plan[TR_MAXN];
  // workspace
  std::vector<void*> allocs;
  // workspace carved from a caller-supplied region (serving) or only sized
  char* region = nullptr;
  size_t region_cap = 0, region_off = 0;
  bool measure = false;
  bool own_stream2 = true;
  bool bf16_ready = false, fp8_ready = false;
  double *F1 = nullptr, *F2 = nullptr, *T0 = nullptr, *T1 = nullptr;
  double *M = nullptr, *S = nullptr, *W0 = nullptr, *W1 = nullptr, *Lf = nullptr, *LTf = nullptr, *cholw = nullptr;
  double* Wpre[2] = {nullptr, nullptr};   // ring prefix of mode m in Wpre[m & 1] within a sweep (order >= 4)
  int64_t w_cap = 0;        // elements of W0, W1 and Wpre
  // TR_ALS_CANARY=1: every workspace buffer is followed by a guard band filled
  // with a byte pattern, checked when the context is destroyed
  bool canary = false;
  std::vector<std::pair<char*, int>> guards;   // (guard band, allocation index)
  size_t guards_filled = 0;
  int nalloc = 0;
  double *Gn = nullptr, *G0u = nullptr, *LinvT = nullptr, *Tsol = nullptr;
  double *Y0 = nullptr, *Y1 = nullptr;   // stage-2 intermediates
  void* Bt = nullptr;                    // stage-1 table, transposed, operand type
  size_t bt_bytes = 0;
  void* partial = nullptr;
  size_t partial_bytes = 0;
  double* dpart = nullptr;
  float* fpart = nullptr;
  double* dscal = nullptr;   // [0] ||X||^2, [1] fit sum, [2] table max 1, [3] table max 2
  float* fscal = nullptr;    // [0] |X| max, [1] fp8 scale
  int* status = nullptr;
  void* xbf16 = nullptr;
  void* xfp8 = nullptr;
  // transposed BF16/FP8 shadows for the two-stage modes that contract the
  // slowest modes at split t_gK (0: none)
  void* xbf16t = nullptr;
  void* xfp8t = nullptr;
  int64_t t_gK = 0;
  float fp8_scale = 1.0f;
  double xnorm2 = 0.0;
  int nred = 1024;
  std::string err;
  // profiling of the X-stream kernel
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  double prof_bytes = 0.0;
};

namespace {

int fail(tr_als_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, TR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

constexpr size_t GUARD_BYTES = 4096;
constexpr unsigned char GUARD_BYTE = 0xA5;
std::atomic<int> g_overruns{0};

int alloc(tr_als_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  const size_t guard = c->canary ? GUARD_BYTES : 0;
  bytes = trx_round(bytes) + guard;
  const int idx = c->nalloc++;
  auto note = [&]() {
    if (guard && !c->measure) c->guards.push_back({(char*)*p + bytes - guard, idx});
  };
  if (c->measure || c->region) {
    const size_t b = trx_round(bytes);
    if (c->region && c->region_off + b > c->region_cap) {
      *p = nullptr;
      return fail(c, TR_ENOMEM, "workspace region of " + std::to_string(c->region_cap) + " bytes exhausted");
    }
    // sizing only: a distinct, never dereferenced, aligned placeholder
    *p = c->region ? (void*)(c->region + c->region_off) : (void*)(TRX_ALIGN + c->region_off);
    c->region_off += b;
    note();
    return TR_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, TR_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(*p);
  note();
  return TR_OK;
}

// Guard bands: filled in stream order after their allocation (never inside a
// graph capture: allocation happens before), checked at destruction.
void fill_guards(tr_als_ctx* c, hipStream_t s) {
  for (; c->guards_filled < c->guards.size(); ++c->guards_filled)
    (void)hipMemsetAsync(c->guards[c->guards_filled].first, GUARD_BYTE, GUARD_BYTES, s);
}

void check_guards(tr_als_ctx* c) {
  std::vector<unsigned char> h(GUARD_BYTES);
  for (auto& g : c->guards) {
    if (hipMemcpy(h.data(), g.first, GUARD_BYTES, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    for (size_t q = 0; q < GUARD_BYTES; ++q)
      if (h[q] != GUARD_BYTE) {
        g_overruns++;
        fprintf(stderr, "tr_als: workspace buffer %d overrun (guard byte %zu written)\n", g.second, q);
        break;
      }
  }
}

int64_t prod(const int64_t* d, int a, int b) {  // prod of dims[a..b)
  int64_t p = 1;
  for (int j = a; j < b; ++j) p *= d[j];
  return p;
}

// Build the plan of mode m (0-based).
Plan make_plan(const tr_als_ctx* c, int m) {
  const int N = c->N;
  const int* R = c->R;  // R[N] == R[0]
  Plan p;
  p.I = c->dims[m];
  p.K = c->numel / p.I;
  p.Ra = R[m];
  p.Rb = R[m + 1];
  if (m == 0) {
    p.layout = 0;
    p.L = 1;
    if (N == 2) {
      p.f1c = {1};
      p.Rmid = R[2];
    } else {
      int best = -1;
      int64_t bestT = 0;
      for (int q = 1; q <= N - 2; ++q) {  // F1 = cores 1..q, F2 = cores q+1..N-1
        const int64_t T1 = prod(c->dims, 1, q + 1), T2 = prod(c->dims, q + 1, N);
        const int rm = R[q + 1];
        const int64_t tb = std::max(T1, T2);
        if (best < 0 || rm < R[best + 1] || (rm == R[best + 1] && tb < bestT)) { best = q; bestT = tb; }
      }
      for (int j = 1; j <= best; ++j) p.f1c.push_back(j);
      for (int j = best + 1; j <= N - 1; ++j) p.f2c.push_back(j);
      p.Rmid = R[best + 1];
    }
    p.K1 = 1;
    for (int j : p.f1c) p.K1 *= c->dims[j];
    p.K2 = 1;
    for (int j : p.f2c) p.K2 *= c->dims[j];
    p.d1 = 1; p.m1 = p.K1; p.d2 = p.K1; p.m2 = p.K2;
  } else if (m == N - 1) {
    p.layout = 1;
    p.L = p.K;
    if (N == 2) {
      p.f1c = {0};
      p.Rmid = R[1];
    } else {
      int best = -1;
      int64_t bestT = 0;
      for (int q = 1; q <= N - 2; ++q) {  // F1 = cores 0..q-1, F2 = cores q..N-2
        const int64_t T1 = prod(c->dims, 0, q), T2 = prod(c->dims, q, N - 1);
        const int rm = R[q];
        const int64_t tb = std::max(T1, T2);
        if (best < 0 || rm < R[best] || (rm == R[best] && tb < bestT)) { best = q; bestT = tb; }
      }
      for (int j = 0; j < best; ++j) p.f1c.push_back(j);
      for (int j = best; j <= N - 2; ++j) p.f2c.push_back(j);
      p.Rmid = R[best];
    }
    p.K1 = 1;
    for (int j : p.f1c) p.K1 *= c->dims[j];
    p.K2 = 1;
    for (int j : p.f2c) p.K2 *= c->dims[j];
    p.d1 = 1; p.m1 = p.K1; p.d2 = p.K1; p.m2 = p.K2;
  } else {
    p.layout = 1;
    p.L = prod(c->dims, 0, m);
    for (int j = m + 1; j < N; ++j) p.f1c.push_back(j);
    for (int j = 0; j < m; ++j) p.f2c.push_back(j);
    p.Rmid = R[0];
    p.K1 = prod(c->dims, m + 1, N);
    p.K2 = p.L;
    p.d1 = p.L; p.m1 = p.K1; p.d2 = 1; p.m2 = p.L;
  }
  // Two-stage MTTSP: contract X over the contiguous group of modes that keeps
  // both the group's partial-subchain table (#K x C) and the intermediate
  // (numel/#K x C) small; taken when their sum is at most a tenth of X.
  double bestc = -1;
  int bnn = 1, bp = -1;
  for (int q = m + 1; q < N; ++q) {  // slowest modes q..N-1
    const int64_t K = prod(c->dims, q, N);
    const int C = R[q] * R[0];
    const double cost = ((double)K + (double)c->numel / K) * C;
    if (C <= 1024 && (bestc < 0 || cost < bestc)) { bestc = cost; bnn = 1; bp = q; }
  }
  for (int q = 0; q < m; ++q) {      // fastest modes 0..q
    const int64_t K = prod(c->dims, 0, q + 1);
    const int C = R[0] * R[q + 1];
    const double cost = ((double)K + (double)c->numel / K) * C;
    if (C <= 1024 && (bestc < 0 || cost < bestc)) { bestc = cost; bnn = 0; bp = q; }
  }
  // TR_ALS_FORCE_REGIME=1|2 pins the choice (used by the tests to run both
  // kernels on every shape)
  const char* fr = getenv("TR_ALS_FORCE_REGIME");
  const int force = fr ? atoi(fr) : 0;
  const bool take = bp >= 0 && (force == 1 || (force != 2 && bestc <= 0.1 * (double)c->numel));
  if (take) {
    p.regime = 1;
    p.nn = bnn;
    if (bnn) {
      for (int j = bp; j < N; ++j) p.gcores.push_back(j);
      p.gK = prod(c->dims, bp, N);
      p.gRu = R[bp]; p.gRc = R[0];
      int Ru = p.gRu, Rc = p.gRc;
      for (int j = bp - 1; j > m; --j) {   // slow side, next to bond u
        p.steps.push_back({prod(c->dims, 0, j), c->dims[j], 1, Ru, Rc, j, 0});
        Ru = R[j];
      }
      for (int j = 0; j < m; ++j) {        // fast side, next to bond c
        p.steps.push_back({1, c->dims[j], prod(c->dims, j + 1, m + 1), Ru, Rc, j, 1});
        Rc = R[j + 1];
      }
    } else {
      for (int j = 0; j <= bp; ++j) p.gcores.push_back(j);
      p.gK = prod(c->dims, 0, bp + 1);
      p.gRu = R[0]; p.gRc = R[bp + 1];
      int Ru = p.gRu, Rc = p.gRc;
      for (int j = bp + 1; j < m; ++j) {   // fast side, next to bond c
        p.steps.push_back({1, c->dims[j], prod(c->dims, j + 1, N), Ru, Rc, j, 1});
        Rc = R[j + 1];
      }
      for (int j = N - 1; j > m; --j) {    // slow side, next to bond u
        p.steps.push_back({prod(c->dims, m, j), c->dims[j], 1, Ru, Rc, j, 0});
        Ru = R[j];
      }
    }
    p.gC = p.gRu * p.gRc;
    p.gM = c->numel / p.gK;
  }
  // Order 3 outside the two-stage regime with R_n R_{n+1} > 128: the fused
  // kernel would form R^3 subchain values per k for many column tiles; the
  // slab kernel contracts one mode against its core on MFMA and absorbs the
  // other per slab instead (TR_ALS_NO_SLAB=1 keeps the fused kernel).
  const bool no_slab = getenv("TR_ALS_NO_SLAB") && getenv("TR_ALS_NO_SLAB")[0] == '1';
  if (N == 3 && p.regime == 2 && !no_slab && (int64_t)R[m] * R[m + 1] > 128) {
    const int c1 = (m + 1) % 3, c2 = (m + 2) % 3;
    // the contracted mode must leave a 2-D slab with unit stride along the rows or along k
    const int kappa = m == 0 ? c1 : 0;
    const int caseB = kappa == c2 ? 1 : 0;
    const int Rm = R[c2];
    const int Ro = caseB ? R[m + 1] : R[m];
    if (xslab_group(Rm, Ro) > 0) {
      p.slab = true;
      p.sk_mode = kappa;
      p.sl_mode = caseB ? c1 : c2;
      p.slab_caseB = caseB;
    }
  }
  return p;
}

int64_t table_elems(const tr_als_ctx* c, const std::vector<int>& cl, int Rdefault) {
  if (cl.empty()) return (int64_t)Rdefault * Rdefault;
  int64_t K = 1;
  for (int j : cl) K *= c->dims[j];
  return K * c->R[cl.front()] * c->R[cl.back() + 1];
}

// Intermediate sizes of building a table chain (for the ping-pong buffers).
int64_t table_build_max(const tr_als_ctx* c, const std::vector<int>& cl) {
  int64_t mx = 0, J = 1;
  for (size_t s = 0; s < cl.size(); ++s) {
    J *= c->dims[cl[s]];
    mx = std::max(mx, J * c->R[cl.front()] * c->R[cl[s] + 1]);
  }
  return mx;
}

// Table of the partial subchain of cores `cl` (chain order, first index
// fastest); `cores`/`dims` default to the context's TR-cores (the QR variant
// passes its R-cores and their middle sizes).
int build_table_ex(tr_als_ctx* c, const std::vector<int>& cl, int Rid, double* out, double* const* cores,
                   const int64_t* dims, double* t0, double* t1) {
  hipStream_t s = c->stream;
  if (cl.empty()) {
    HIPCHK(c, launch_identity_table(Rid, out, s));
    return TR_OK;
  }
  const int Rl = c->R[cl.front()];
  double* cur = (cl.size() == 1) ? out : t0;
  HIPCHK(c, launch_core_to_table(cores[cl[0]], Rl, dims[cl[0]], c->R[cl[0] + 1], cur, s));
  int64_t J = dims[cl[0]];
  for (size_t q = 1; q < cl.size(); ++q) {
    const int k = cl[q];
    double* nxt = (q + 1 == cl.size()) ? out : (cur == t0 ? t1 : t0);
    HIPCHK(c, launch_chain_step(cur, J, Rl, c->R[k], cores[k], dims[k], c->R[k + 1], nxt, s));
    J *= dims[k];
    cur = nxt;
  }
  return TR_OK;
}

int build_table(tr_als_ctx* c, const std::vector<int>& cl, int Rid, double* out) {
  return build_table_ex(c, cl, Rid, out, c->cores, c->dims, c->T0, c->T1);
}

struct XsCfg {
  XsArgs a;
  int kt = 64, wlay = 0;
  size_t lds = 0;
};

// Tile / split configuration of the X-stream kernel for mode m in precision prec.
XsCfg xs_config(const tr_als_ctx* c, int m, int prec) {
  const Plan& p = c->plan[m];
  XsCfg x;
  XsArgs& a = x.a;
  a.I = p.I; a.K = p.K; a.L = p.L; a.layout = p.layout;
  a.F1 = c->F1; a.F2 = c->F2;
  a.d1 = p.d1; a.m1 = p.m1; a.d2 = p.d2; a.m2 = p.m2;
  a.Rb = p.Rb; a.Rmid = p.Rmid; a.Ra = p.Ra;
  a.tmax = nullptr;
  a.partial = c->partial;
  if (p.I <= 128) { a.MT = (int)((p.I + 15) / 16 * 16); a.n_mt = 1; }
  else { a.MT = 128; a.n_mt = (int)((p.I + 127) / 128); }
  if (p.Ra * p.Rb <= 128) { a.NTb = p.Rb; a.NT = (p.Ra * p.Rb + 15) / 16 * 16; a.n_nt = 1; }
  else {
    a.NTb = std::max(4, (128 / p.Ra) / 4 * 4);
    a.NT = (p.Ra * a.NTb + 15) / 16 * 16;
    a.n_nt = (p.Rb + a.NTb - 1) / a.NTb;
  }
  // K tile: the largest that leaves room for >= 3 workgroups per CU, else the
  // largest that fits the 160 KB of LDS (x.lds == 0 marks "does not fit")
  const int cand_f64[2] = {32, 16}, cand_lo[2] = {64, 32};
  const int* cand = (prec == TR_F64) ? cand_f64 : cand_lo;
  x.kt = 0;
  for (int pass = 0; pass < 2 && x.kt == 0; ++pass)
    for (int q = 0; q < 2; ++q)
      if (xstream_lds_bytes(a, prec, cand[q]) <= (pass == 0 ? 52u : 160u) * 1024u) { x.kt = cand[q]; break; }
  x.lds = x.kt ? xstream_lds_bytes(a, prec, x.kt) : 0;
  if (!x.kt) x.kt = cand[1];
  // wave arrangement
  const int MB = a.MT / 16, NB = a.NT / 16;
  struct Opt { int wgm, wgn, wm, wn, lay; } opts[3] = {{2, 2, 4, 4, 0}, {1, 4, 8, 2, 1}, {4, 1, 2, 8, 2}};
  int best = -1, bestv = 1 << 30;
  for (int o = 0; o < 3; ++o) {
    const int pm = (MB + opts[o].wgm - 1) / opts[o].wgm, pn = (NB + opts[o].wgn - 1) / opts[o].wgn;
    if (pm > opts[o].wm || pn > opts[o].wn) continue;
    const int v = pm * pn;
    if (v < bestv) { bestv = v; best = o; }
  }
  a.wgm = opts[best].wgm; a.wgn = opts[best].wgn; x.wlay = opts[best].lay;
  // split-K
  const int64_t ktiles = (p.K + x.kt - 1) / x.kt;
  const int64_t ntiles = (int64_t)a.n_mt * a.n_nt;
  int64_t nsplit = std::max<int64_t>(1, (768 + ntiles - 1) / ntiles);
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, ktiles / 4));
  const int64_t tps = (ktiles + nsplit - 1) / nsplit;
  a.k_per_split = tps * x.kt;
  a.nsplit = (int)((p.K + a.k_per_split - 1) / a.k_per_split);
  return x;
}

// Slab-kernel configuration of mode m (order 3): strides, ranks, groups and
// the split over slabs (about two workgroups per CU in flight).
XslabArgs xslab_config(const tr_als_ctx* c, int m, const void* X) {
  const Plan& p = c->plan[m];
  XslabArgs a;
  const int64_t stride[3] = {1, c->dims[0], c->dims[0] * c->dims[1]};
  a.X = X;
  a.In = c->dims[m]; a.Ik = c->dims[p.sk_mode]; a.Il = c->dims[p.sl_mode];
  a.sn = stride[m]; a.sk = stride[p.sk_mode]; a.sl = stride[p.sl_mode];
  a.caseB = p.slab_caseB;
  a.Gl = c->cores[p.sl_mode];
  const int c2 = (m + 2) % 3;
  a.Rm = c->R[c2];
  a.Rn = c->R[m];
  a.Rg = a.caseB ? c->R[m] : c->R[m + 1];
  a.Ro = a.caseB ? c->R[m + 1] : c->R[m];
  a.NG = xslab_group(a.Rm, a.Ro);
  a.TWg = (a.NG * a.Rm + 15) / 16 * 16;
  a.OWg = a.NG * a.Ro;
  a.n_g = (a.Rg + a.NG - 1) / a.NG;
  a.n_mt = (int)((a.In + xslab_rows() - 1) / xslab_rows());
  a.ldb = 0;                 // set per precision by the caller (k tile)
  const int64_t tiles = (int64_t)a.n_mt * a.n_g;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(a.Il, (512 + tiles - 1) / tiles));
  a.l_per_split = (a.Il + ns - 1) / ns;
  a.nsplit = (int)((a.Il + a.l_per_split - 1) / a.l_per_split);
  a.Bt = c->Bt;
  a.partial = c->partial;
  return a;
}

size_t xslab_partial_bytes(const XslabArgs& a, int prec) {
  return (size_t)a.nsplit * a.n_mt * a.n_g * xslab_rows() * a.OWg * (prec == TR_F64 ? 8 : 4);
}

size_t xslab_bt_bytes(const XslabArgs& a, int prec) {   // BF16: hi and lo parts
  const int kt = xslab_kt(prec);
  const int64_t ldb = (a.Ik + kt - 1) / kt * kt;
  return (size_t)a.n_g * a.TWg * ldb * (prec == TR_F64 ? 8 : prec == TR_F32 ? 4 : 4);
}

XgArgs xg_config(const tr_als_ctx* c, int m, int prec, const void* X, int esize, bool transposed = false,
                 int mt_override = 0) {
  const Plan& p = c->plan[m];
  XgArgs g;
  g.X = X;
  g.M = p.gM; g.K = p.gK; g.C = p.gC; g.nn = transposed ? 0 : p.nn;
  // 16-byte aligned starts of the contiguous runs of A: rows (fastest-modes
  // group) or columns (slowest-modes group, BF16 row-vector loads)
  g.vec_ok = ((((g.nn ? p.gM : p.gK) * esize) % 16 == 0) && (((uintptr_t)X) % 16 == 0)) ? 1 : 0;
  // Row tile and split-K target (workgroups per launch); measured best on the
  // 100^4 rank-10 workload with X streamed from HBM (not the last-level
  // cache): 128 rows, ~448 workgroups for BF16 (6 splits: 59.7 us against
  // 65-75 us for 5 or 7-13 splits), ~1024 for FP32 (MFMA-bound).
  // TR_ALS_XG_MT / TR_ALS_XG_WGS override (read at every call, so a test can
  // run the 128-row tiles on a small shape; the buffers are sized for both).
  g.MT = p.gM > 8192 ? 128 : 64;
  const int env_mt = getenv("TR_ALS_XG_MT") ? atoi(getenv("TR_ALS_XG_MT")) : 0;
  const int env_wgs = getenv("TR_ALS_XG_WGS") ? atoi(getenv("TR_ALS_XG_WGS")) : 0;
  if (env_mt == 64 || env_mt == 128) g.MT = env_mt;
  if (mt_override) g.MT = mt_override;
  const int64_t target_wgs = env_wgs > 0 ? env_wgs : ((prec == TR_F32 || prec == TR_F64) ? 1024 : 448);
  g.n_mt = (int)((p.gM + g.MT - 1) / g.MT);
  if (p.gC <= 128) { g.NT = (p.gC + 15) / 16 * 16; g.n_nt = 1; }
  else { g.NT = 128; g.n_nt = (p.gC + 127) / 128; }
  const int kt = xgemm_kt(prec);
  g.ldb = (p.gK + kt - 1) / kt * kt;
  const int64_t ktiles = g.ldb / kt;
  const int64_t tiles = (int64_t)g.n_mt * g.n_nt;
  int64_t ns = std::max<int64_t>(1, (target_wgs + tiles - 1) / tiles);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, ktiles / 2));
  // XCD-aware mapping (TR_ALS_XG_XCD=1) when there are enough splits: a
  // multiple of 8 of them.  It brings the fetched bytes of the 100^4 rank-10
  // launch down to the algorithmic ones (202-213 MB instead of 240-294 MB) but
  // measured ~6% slower, so it is off by default.
  static const bool env_xcd = getenv("TR_ALS_XG_XCD") && getenv("TR_ALS_XG_XCD")[0] == '1';
  g.xcd_map = 0;
  if (env_xcd && ns >= 6 && ktiles >= 16) {
    const int64_t ns8 = std::max<int64_t>(8, (ns + 4) / 8 * 8);
    const int64_t tps8 = (ktiles + ns8 - 1) / ns8;
    if ((ktiles + tps8 - 1) / tps8 == ns8) {   // every one of the ns8 splits has work
      ns = ns8;
      g.xcd_map = 1;
    }
  }
  const int64_t tps = (ktiles + ns - 1) / ns;
  g.k_per_split = tps * kt;
  g.nsplit = (int)((p.gK + g.k_per_split - 1) / g.k_per_split);
  if (g.xcd_map && g.nsplit != ns) g.xcd_map = 0;
  g.Bt = c->Bt;
  g.tmax = nullptr;
  g.partial = c->partial;
  return g;
}

size_t xg_partial_bytes(const XgArgs& g, int prec) {
  return (size_t)g.nsplit * g.n_mt * g.n_nt * g.MT * g.NT * (prec == TR_F64 ? 8 : 4);
}

size_t xg_bt_bytes(const XgArgs& g, int prec) {   // FP8: hi and lo parts
  const size_t es = prec == TR_F64 ? 8 : prec == TR_F32 ? 4 : prec == TR_BF16 ? 2 : 2;
  return (size_t)g.n_nt * g.NT * g.ldb * es;
}

size_t partial_bytes_needed(const XsCfg& x, int prec) {
  return (size_t)x.a.nsplit * x.a.n_mt * x.a.n_nt * x.a.MT * x.a.NT * (prec == TR_F64 ? 8 : 4);
}

int ensure_shadow(tr_als_ctx* c, int prec) {
  hipStream_t s = c->stream;
  struct Fill {   // guard bands of shadows allocated here, in stream order
    tr_als_ctx* c; hipStream_t s;
    ~Fill() { if (c->canary) fill_guards(c, s); }
  } fill{c, s};
  if (prec == TR_BF16 && !c->bf16_ready) {
    if (!c->xbf16) {
      int rc = alloc(c, &c->xbf16, (size_t)c->numel * 2);
      if (rc) return rc;
    }
    HIPCHK(c, launch_to_bf16(c->X, c->xdt, c->numel, c->xbf16, s));
    if (c->t_gK) {
      if (!c->xbf16t) {
        int rc = alloc(c, &c->xbf16t, (size_t)c->numel * 2);
        if (rc) return rc;
      }
      HIPCHK(c, launch_to_lowp_t(c->X, c->xdt, c->numel / c->t_gK, c->t_gK, nullptr, TR_BF16, c->xbf16t, s));
    }
    c->bf16_ready = true;
  }
  if (prec == TR_FP8 && !c->fp8_ready) {
    if (!c->xfp8) {
      int rc = alloc(c, &c->xfp8, (size_t)c->numel);
      if (rc) return rc;
    }
    c->fp8_ready = true;
    HIPCHK(c, launch_absmax(c->X, c->xdt, c->numel, c->fpart, c->nred, c->fscal, s));
    HIPCHK(c, launch_to_fp8(c->X, c->xdt, c->numel, c->fscal, c->fscal + 1, c->xfp8, s));
    if (c->t_gK) {
      if (!c->xfp8t) {
        int rc = alloc(c, &c->xfp8t, (size_t)c->numel);
        if (rc) return rc;
      }
      HIPCHK(c, launch_to_lowp_t(c->X, c->xdt, c->numel / c->t_gK, c->t_gK, c->fscal, TR_FP8, c->xfp8t, s));
    }
    HIPCHK(c, hipMemcpyAsync(&c->fp8_scale, c->fscal + 1, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  return TR_OK;
}

// Two-stage M_n: group table -> transposed operand table -> stage-1 GEMM over
// X -> ordered reduction -> stage-2 absorptions.
// `after_main` (may be empty) is enqueued right after the X-contraction
// launch: the NE update forks its coefficient branch there, so that a graph
// built from the sweep releases the contraction before the branch.
using Hook = std::function<int()>;

// Stage 2: absorb the remaining cores into the reduced stage-1 result `cur`
// (Y0), ping-ponging through Y1 / Y0, the last step writing M.
int absorb_steps(tr_als_ctx* c, const Plan& p, double* cur, double* Mout, hipStream_t s) {
  for (size_t q = 0; q < p.steps.size(); ++q) {
    const Plan::Step& st = p.steps[q];
    const bool last = q + 1 == p.steps.size();
    double* nxt = last ? Mout : (cur == c->Y0 ? c->Y1 : c->Y0);
    HIPCHK(c, launch_absorb(cur, st.lo, st.I, st.hi, st.Ru, st.Rc, c->cores[st.core], c->R[st.core],
                            c->R[st.core + 1], st.side, last ? 1 : 0, nxt, (double*)c->partial, c->partial_bytes,
                            s));
    cur = nxt;
  }
  return TR_OK;
}

int compute_mttsp_two_stage(tr_als_ctx* c, int m, int prec, double* Mout, bool in_sweep, const Hook& after_main) {
  hipStream_t s = c->stream;
  const Plan& p = c->plan[m];
  const bool reuse = in_sweep && p.reuse_prev;
  if (reuse && p.reuse_y) {
    // the previous mode contracted X with this same group table and left the
    // reduced result in Y0 (identical bits): only the absorptions differ
    if (after_main) {
      const int hr = after_main();
      if (hr) return hr;
    }
    return absorb_steps(c, p, c->Y0, Mout, s);
  }
  // groups of one or two cores: operand table straight from the cores
  const bool direct = prec != TR_FP8 && (p.gcores.size() == 1 || p.gcores.size() == 2) && c->R[p.gcores[0]] <= 24;
  int rc = (reuse || direct) ? TR_OK : build_table(c, p.gcores, 1, c->F1);
  if (rc) return rc;
  rc = ensure_shadow(c, prec);
  if (rc) return rc;
  // the slowest-modes group reads the transposed shadow as a fastest-modes one
  const bool use_t = p.nn && c->t_gK == p.gK && ((prec == TR_BF16 && c->xbf16t) || (prec == TR_FP8 && c->xfp8t));
  const void* X = use_t ? (prec == TR_BF16 ? c->xbf16t : c->xfp8t)
                        : prec == TR_BF16 ? c->xbf16 : prec == TR_FP8 ? c->xfp8 : c->X;
  const int esize = prec == TR_BF16 ? 2 : prec == TR_FP8 ? 1 : (c->xdt == TR_F64 ? 8 : 4);
  XgArgs g = xg_config(c, m, prec, X, esize, use_t);
  if (xg_partial_bytes(g, prec) > c->partial_bytes || xg_bt_bytes(g, prec) > c->bt_bytes)
    return fail(c, TR_EHIP, "internal: stage-1 buffers too small");
  double out_scale = 1.0;
  if (prec == TR_FP8 && !reuse) {
    // the table's scale is derived on the device from its max (no host round
    // trip: the sweep stays capturable); the reduction undoes it
    HIPCHK(c, launch_table_absmax(c->F1, p.gK * p.gC, c->dscal + 2, s));
  }
  if (prec == TR_FP8) {
    g.tmax = c->dscal + 2;
    out_scale = 1.0 / (double)c->fp8_scale;
  }
  if (!reuse && direct) {
    const int g0 = p.gcores[0], two = p.gcores.size() == 2;
    const int g1 = two ? p.gcores[1] : g0;
    HIPCHK(c, launch_group_bt(c->cores[g0], c->R[g0], c->dims[g0], c->R[g0 + 1], c->cores[g1], c->dims[g1], two, p.gK,
                              p.gC, g.n_nt * g.NT, g.ldb, prec, c->Bt, s));
  } else if (!reuse) {
    HIPCHK(c, launch_table_to_bt(c->F1, p.gK, p.gC, g.n_nt * g.NT, g.ldb, prec, 1.0, c->Bt, s, c->dscal + 2));
  }
  const bool prof = c->prof;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) {
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, s));
  }
  HIPCHK(c, launch_xgemm(g, prec, (prec == TR_F64 || prec == TR_F32) ? c->xdt : prec, s));
  if (prof) {
    HIPCHK(c, hipEventRecord(e1, s));
    c->evs.push_back({e0, e1});
    c->prof_bytes = (double)esize * (double)c->numel;
  }
  if (after_main) {
    const int hr = after_main();
    if (hr) return hr;
  }
  double* cur = p.steps.empty() ? c->Y1 : c->Y0;
  HIPCHK(c, launch_xg_reduce(g, prec, out_scale, cur, c->status, s));
  if (p.steps.empty()) {
    HIPCHK(c, launch_bond_to_M(cur, p.I, p.gRu, p.gRc, Mout, s));
    return TR_OK;
  }
  return absorb_steps(c, p, cur, Mout, s);
}

// M_n = X_[n] G^{!=n}_[2] for the context's current cores (tables + X stream +
// ordered split-K reduction).
// M_n by the slab kernel (order 3, large ranks): table of the contracted
// mode's core in the operand type, the slab pass over X, ordered reduction.
int compute_mttsp_slab(tr_als_ctx* c, int m, int prec, double* Mout, const Hook& after_main) {
  hipStream_t s = c->stream;
  const Plan& p = c->plan[m];
  int rc = ensure_shadow(c, prec);
  if (rc) return rc;
  const void* X = prec == TR_BF16 ? c->xbf16 : c->X;
  XslabArgs a = xslab_config(c, m, X);
  const int kt = xslab_kt(prec);
  a.ldb = (a.Ik + kt - 1) / kt * kt;
  if (xslab_partial_bytes(a, prec) > c->partial_bytes || xslab_bt_bytes(a, prec) > c->bt_bytes)
    return fail(c, TR_EHIP, "internal: slab buffers too small");
  HIPCHK(c, launch_xslab_table(a, c->cores[p.sk_mode], prec, c->Bt, s));
  const bool prof = c->prof;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) {
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, s));
  }
  HIPCHK(c, launch_xslab(a, prec, (prec == TR_F64 || prec == TR_F32) ? c->xdt : prec, xslab_lds_bytes(a, prec), s));
  if (prof) {
    HIPCHK(c, hipEventRecord(e1, s));
    c->evs.push_back({e0, e1});
    c->prof_bytes = (double)c->numel * (prec == TR_BF16 ? 2 : (c->xdt == TR_F64 ? 8 : 4));
  }
  if (after_main) {
    const int hr = after_main();
    if (hr) return hr;
  }
  HIPCHK(c, launch_xslab_reduce(a, prec, 1.0, Mout, c->status, s));
  return TR_OK;
}

int compute_mttsp(tr_als_ctx* c, int m, int prec, double* Mout, bool in_sweep = false, const Hook& after_main = Hook()) {
  hipStream_t s = c->stream;
  const Plan& p = c->plan[m];
  if (p.regime == 1) return compute_mttsp_two_stage(c, m, prec, Mout, in_sweep, after_main);
  // the slab kernel's BF16 form loads 8 consecutive elements at a time: every
  // mode size a multiple of 8 (else BF16 takes the fused kernel); FP8 always
  // takes the fused kernel
  const bool slab_bf16_ok = c->N == 3 && c->dims[0] % 8 == 0 && c->dims[1] % 8 == 0 && c->dims[2] % 8 == 0;
  if (p.slab && prec != TR_FP8 && (prec != TR_BF16 || slab_bf16_ok))
    return compute_mttsp_slab(c, m, prec, Mout, after_main);
  int rc = build_table(c, p.f1c, p.Rmid, c->F1);
  if (rc) return rc;
  rc = build_table(c, p.f2c, p.Rmid, c->F2);
  if (rc) return rc;
  rc = ensure_shadow(c, prec);
  if (rc) return rc;
  XsCfg x = xs_config(c, m, prec);
  if (x.lds == 0) return fail(c, TR_EINVAL, "ranks too large for the LDS tiles of the X stream");
  if (partial_bytes_needed(x, prec) > c->partial_bytes) return fail(c, TR_EHIP, "internal: partial buffer too small");
  double out_scale = 1.0;
  if (prec == TR_BF16) x.a.X = c->xbf16;
  else if (prec == TR_FP8) {
    x.a.X = c->xfp8;
    // the generated subchain rows are scaled into the E4M3 range by a power of
    // two derived on the device from max|F1 F2| <= Rmid max|F1| max|F2| (no
    // host round trip); the reduction undoes it
    const int64_t n1 = table_elems(c, p.f1c, p.Rmid), n2 = table_elems(c, p.f2c, p.Rmid);
    HIPCHK(c, launch_table_absmax(c->F1, n1, c->dscal + 2, s));
    HIPCHK(c, launch_table_absmax(c->F2, n2, c->dscal + 3, s));
    x.a.tmax = c->dscal + 2;
    out_scale = 1.0 / (double)c->fp8_scale;
  } else x.a.X = c->X;
  const bool prof = c->prof;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) {
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, s));
  }
  HIPCHK(c, launch_xstream(x.a, prec, (prec == TR_F64 || prec == TR_F32) ? c->xdt : prec, x.kt, x.wlay, x.lds, s));
  if (prof) {
    HIPCHK(c, hipEventRecord(e1, s));
    c->evs.push_back({e0, e1});
    const double eb = prec == TR_F64 ? (c->xdt == TR_F64 ? 8 : 4) : prec == TR_F32 ? (c->xdt == TR_F64 ? 8 : 4)
                    : prec == TR_BF16 ? 2 : 1;
    c->prof_bytes = eb * (double)c->numel;
  }
  if (after_main) {
    const int hr = after_main();
    if (hr) return hr;
  }
  HIPCHK(c, launch_xs_reduce(x.a, prec, out_scale, Mout, c->status, s));
  return TR_OK;
}

// S_n<2> from the Gram ring: W = K_{m+1} K_{m+2} ... K_{m-1} (Kronecker-order
// Grams), then realigned.
// Ring product of Prop. 3.1 for mode m: W = K_{m+1} K_{m+2} ... K_{m-1} over
// the Kronecker-form Gram views, then realigned into S_m.  Within a sweep of
// order >= 4 the prefix K_{m+1} ... K_{m-2} (it excludes the cores of modes
// m-1 and m) is formed by the previous mode's branch (ring_prefix), so only
// the last factor, refreshed by that mode, is multiplied here.
// With S_out the last GEMM stores its result realigned into S_out (mode m),
// in one launch with the independent product *pair when one is given.
int ring_gemms(tr_als_ctx* c, const std::vector<int>& chain, MatView W, int64_t rows, double* last_out,
               hipStream_t s, double* S_out = nullptr, int m = 0, const Gemm64Desc* pair = nullptr) {
  auto gview = [&](int k) {
    MatView v;
    v.p = c->gram[k]; v.ld = 0; v.kind = 1; v.Rl = c->R[k]; v.Rr = c->R[k + 1];
    return v;
  };
  double* bufs[2] = {c->W0, c->W1};
  int cur = 0;
  for (size_t q = 0; q < chain.size(); ++q) {
    const int k = chain[q];
    const int64_t inner = (int64_t)c->R[k] * c->R[k];
    const int64_t cols = (int64_t)c->R[k + 1] * c->R[k + 1];
    const bool last = q + 1 == chain.size();
    if (last && S_out) {   // W (R_{m+1}^2 x R_m^2) straight into S_m<2>
      if (pair) HIPCHK(c, launch_gemm64_pair(gemm64_realign_desc(inner, W, gview(k), c->R[m], c->R[m + 1], S_out),
                                             *pair, s));
      else HIPCHK(c, launch_gemm64_realign(inner, W, gview(k), c->R[m], c->R[m + 1], S_out, s));
      break;
    }
    double* out = (last && last_out) ? last_out : bufs[cur];
    if (rows * cols > c->w_cap) return fail(c, TR_EINVAL, "internal: ring workspace too small");
    HIPCHK(c, launch_gemm64(rows, cols, inner, 1.0, W, gview(k), 0.0, nullptr, 0, out, rows, s));
    W.p = out; W.ld = rows; W.kind = 0;
    cur ^= 1;
  }
  return TR_OK;
}

MatView ring_first(const tr_als_ctx* c, int k) {
  MatView v;
  v.p = c->gram[k]; v.ld = 0; v.kind = 1; v.Rl = c->R[k]; v.Rr = c->R[k + 1];
  return v;
}

int compute_coef(tr_als_ctx* c, int m, double* Sout, hipStream_t s, bool use_prefix = false,
                 const Gemm64Desc* pair = nullptr) {
  const int N = c->N;
  const int64_t rows = (int64_t)c->R[(m + 1) % N] * c->R[(m + 1) % N];
  MatView W;
  std::vector<int> rest;
  if (use_prefix) {   // Wpre[m & 1] = K_{m+1} ... K_{m-2}
    W.p = c->Wpre[m & 1]; W.ld = rows; W.kind = 0; W.Rl = 0; W.Rr = 0;
    rest.push_back((m + N - 1) % N);
  } else {
    W = ring_first(c, (m + 1) % N);
    for (int k = 2; k < N; ++k) rest.push_back((m + k) % N);
  }
  if (!rest.empty()) return ring_gemms(c, rest, W, rows, nullptr, s, Sout, m, pair);   // last GEMM realigns
  HIPCHK(c, launch_realign_S(W, c->R[m], c->R[m + 1], Sout, s));
  return TR_OK;
}

// Prefix K_{m+1} ... K_{m-2} of mode m's ring, into Wpre[m & 1] (order >= 4).
int ring_prefix(tr_als_ctx* c, int m, hipStream_t s) {
  const int N = c->N;
  const int64_t rows = (int64_t)c->R[(m + 1) % N] * c->R[(m + 1) % N];
  std::vector<int> rest;
  for (int k = 2; k <= N - 2; ++k) rest.push_back((m + k) % N);
  return ring_gemms(c, rest, ring_first(c, (m + 1) % N), rows, c->Wpre[m & 1], s);
}

// Order 4: mode m's prefix is the one product K_{m+1} K_{m+2}; its descriptor
// (false when it is more than one product or does not fit the workspace).
bool ring_prefix_single(const tr_als_ctx* c, int m, Gemm64Desc* d) {
  const int N = c->N;
  if (N != 4) return false;
  const int k0 = (m + 1) % N, k1 = (m + 2) % N;
  const int64_t rows = (int64_t)c->R[k0] * c->R[k0], inner = (int64_t)c->R[k1] * c->R[k1];
  const int64_t cols = (int64_t)c->R[k1 + 1] * c->R[k1 + 1];
  if (rows * cols > c->w_cap) return false;
  MatView B;
  B.p = c->gram[k1]; B.ld = 0; B.kind = 1; B.Rl = c->R[k1]; B.Rr = c->R[k1 + 1];
  *d = Gemm64Desc{rows, cols, inner, 1.0, ring_first(c, k0), B, 0.0, nullptr, 0, c->Wpre[m & 1], rows, 0, 0};
  return true;
}

// S^{-1} of an SPD matrix larger than the one-workgroup inverse takes
// (R_n R_{n+1} > 112), from a blocked Cholesky factor: with S = [A C; C^T D],
// A = L_A L_A^T (LDS Cholesky of a block of at most 112), L_21 = C^T L_A^{-T}
// (triangular solves on the rows of C^T), the Schur complement
// D - L_21 L_21^T (FP64 MFMA) factored the same way, and the inverse factor
// L^{-1} = [L_A^{-1} 0; -L_D^{-1} L_21 L_A^{-1}  L_D^{-1}]; then
// S^{-1} = L^{-T} L^{-1}.  A non-positive pivot latches ST_SINGULAR.  S
// (ld ldS) may be a sub-block; Linv (ld ldo) receives L^{-1}; ws holds
// chol_inv_blocked_ws(n) doubles.
int chol_inv_blocked(tr_als_ctx* c, const double* S, int64_t ldS, int n, double* Linv, int64_t ldo, double* ws,
                     hipStream_t s) {
  constexpr int b = 112;
  const int nb = std::min(n, b);
  double* Ac = ws;                       // nb x nb
  double* L = Ac + nb * nb;              // nb x nb
  double* LT = L + nb * nb;              // nb x nb
  double* G = LT + nb * nb;              // nb x nb: L_A^{-T}
  double* rd = G + nb * nb;              // 256 reciprocal pivots
  double* rest = rd + 256;
  HIPCHK(c, launch_copy_block(S, ldS, nb, nb, Ac, nb, s));
  HIPCHK(c, launch_chol_lds(Ac, nb, L, LT, rd, c->status, s));
  HIPCHK(c, launch_trsm_rhs(L, rd, nb, nullptr, nb, G, 0, c->status, s, 1));          // G = L_A^{-T}
  HIPCHK(c, launch_copy_block(G, nb, nb, nb, Linv, ldo, s, 1));                       // L_A^{-1} = G^T
  if (n <= b) return TR_OK;
  const int m = n - b;
  double* Ct = rest;                     // m x b: C^T = S[b:n, 0:b]
  double* L21 = Ct + (int64_t)m * b;     // m x b
  double* Sc = L21 + (int64_t)m * b;     // m x m
  double* T1 = Sc + (int64_t)m * m;      // m x b
  double* next = T1 + (int64_t)m * b;
  HIPCHK(c, launch_copy_block(S + b, ldS, m, b, Ct, m, s));
  HIPCHK(c, launch_trsm_rhs(L, rd, b, Ct, m, L21, 0, c->status, s, 1));             // L21 L_A^T = C^T
  const MatView vL21{L21, m, 0, 0, 0}, vL21t{L21, m, 2, 0, 0};
  HIPCHK(c, launch_gemm64(m, m, b, -1.0, vL21, vL21t, 1.0, S + b + ldS * b, ldS, Sc, m, s));   // D - L21 L21^T
  double* Linv22 = Linv + b + ldo * b;
  int rc = chol_inv_blocked(c, Sc, m, m, Linv22, ldo, next, s);
  if (rc) return rc;
  const MatView vGt{G, b, 2, 0, 0}, vT1{T1, m, 0, 0, 0}, vLi22{Linv22, ldo, 0, 0, 0};
  HIPCHK(c, launch_gemm64(m, b, b, 1.0, vL21, vGt, 0.0, nullptr, 0, T1, m, s));                // L21 L_A^{-1}
  HIPCHK(c, launch_gemm64(m, b, m, -1.0, vLi22, vT1, 0.0, nullptr, 0, Linv + b, ldo, s));      // -L_D^{-1} (.)
  HIPCHK(c, launch_copy_block(nullptr, 0, b, m, Linv + ldo * b, ldo, s));                      // upper block 0
  return TR_OK;
}

int64_t chol_inv_blocked_ws(int n) {
  int64_t tot = 0;
  while (true) {
    const int64_t nb = std::min(n, 112);
    tot += 4 * nb * nb + 256;
    if (n <= 112) break;
    const int64_t m = n - 112;
    tot += 3 * m * 112 + m * m;
    n = (int)m;
  }
  return tot;
}

int spd_inverse_blocked(tr_als_ctx* c, const double* S, int n, double* Sinv, double* ws, hipStream_t s) {
  double* Linv = ws;
  int rc = chol_inv_blocked(c, S, n, n, Linv, n, ws + (int64_t)n * n, s);
  if (rc) return rc;
  const MatView vLt{Linv, n, 2, 0, 0}, vL{Linv, n, 0, 0, 0};
  HIPCHK(c, launch_gemm64(n, n, n, 1.0, vLt, vL, 0.0, nullptr, 0, Sinv, n, s));                // L^{-T} L^{-1}
  return TR_OK;
}

int64_t spd_inverse_blocked_ws(int n) { return (int64_t)n * n + chol_inv_blocked_ws(n); }

// Cut-off of the pseudo-inverse of S_n: the caller's rcond, else n * eps
// (relative to the largest singular value of S_n, which squares those of
// G^{!=n}_[2]).
double pinv_rcond(const tr_als_ctx* c, int n) { return c->rcond > 0.0 ? c->rcond : n * 2.220446049250313e-16; }

// One NE mode update.  The coefficient branch (Gram ring -> S_n -> Cholesky ->
// S_n^{-1}) does not depend on X and runs on a second stream concurrently with
// the MTTSP; the solve is then G = M S^{-1} with iterative refinement
// G += (M - G S) S^{-1}, all on FP64 MFMA.
int update_mode_ne(tr_als_ctx* c, int m, int prec, int refine, bool in_sweep) {
  hipStream_t s = c->stream, s2 = c->stream2;
  const Plan& p = c->plan[m];
  const int n = p.Ra * p.Rb;
  HIPCHK(c, hipEventRecord(c->ev_fork, s));
  // coefficient branch on the second stream, forked after the X-contraction
  // launch (it needs only the Grams, which are ready at the fork)
  // within a sweep of order >= 4 the previous mode formed this mode's ring
  // prefix (mode 1 of a sweep starts from scratch: nothing crosses sweeps)
  const bool prefix = in_sweep && c->N >= 4;
  auto branch = [&]() -> int {
    HIPCHK(c, hipStreamWaitEvent(s2, c->ev_fork, 0));
    // order 4: the next mode's prefix K_{m+2} K_{m+3} is one product of Grams
    // that are final here; it goes into the same launch as this mode's last
    // ring GEMM (its ring has at least one GEMM at order 4)
    Gemm64Desc pd;
    const bool pair = prefix && m + 1 < c->N && ring_prefix_single(c, m + 1, &pd);
    const int r = compute_coef(c, m, c->S, s2, prefix && m > 0, pair ? &pd : nullptr);
    if (r) return r;
    if (c->solve == TR_SOLVE_PINV) {
      HIPCHK(c, launch_pinv(c->S, n, pinv_rcond(c, n), c->Sinv, c->pinvw, c->status, s2));
    } else if (spd_inverse_fits(n)) {
      HIPCHK(c, launch_spd_inverse(c->S, n, c->Sinv, c->status, s2));
    } else {
      const int r2 = spd_inverse_blocked(c, c->S, n, c->Sinv, c->blkw, s2);
      if (r2) return r2;
    }
    HIPCHK(c, hipEventRecord(c->ev_join, s2));
    // after the join: the next mode's prefix excludes this mode's core
    if (prefix && m + 1 < c->N && !pair) return ring_prefix(c, m + 1, s2);
    return TR_OK;
  };
  int rc = compute_mttsp(c, m, prec, c->M, in_sweep, branch);
  if (rc) return rc;
  HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
  // G = M S^{-1} with refinement; the apply latches any non-finite entry, and
  // the commit keeps the old core (and its Gram) when the status word is set
  HIPCHK(c, launch_ne_apply(c->M, p.I, n, c->S, c->Sinv, refine, c->Gn, c->status, s));
  HIPCHK(c, launch_commit_gram(c->Gn, p.I, p.Ra, p.Rb, c->cores[m], c->gram[m], c->status, s));
  return TR_OK;
}

// rocBLAS on the context's stream (handle created at the first use).
int blas_on(tr_als_ctx* c, hipStream_t s) {
  if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success) {
    c->blas = nullptr;
    return fail(c, TR_EHIP, "rocblas_create_handle failed");
  }
  if (rocblas_set_stream(c->blas, s) != rocblas_status_success) return fail(c, TR_EHIP, "rocblas_set_stream failed");
  return TR_OK;
}

#define BLASCHK(c, x)                                                                              \
  do {                                                                                             \
    const rocblas_status st_ = (x);                                                                \
    if (st_ != rocblas_status_success)                                                             \
      return fail(c, TR_EHIP, std::string("rocBLAS: ") + rocblas_status_to_string(st_) + " in " #x); \
  } while (0)

// Lower Cholesky factor L (n x n, ld n, strict upper triangle zero) of the SPD
// matrix whose lower triangle is in G (ld n), right-looking by 112-column
// blocks: LDS factor of the diagonal block, triangular solve for the panel
// below it, rank-k update of the trailing matrix (both triangles; only the
// lower one is read later).  A non-positive
// pivot latches ST_SINGULAR.  ws holds 3 * 112^2 doubles.
int chol_lower_blocked(tr_als_ctx* c, const double* G, int n, double* L, double* ws, hipStream_t s) {
  constexpr int b = 112;
  const double one = 1.0, mone = -1.0;
  HIPCHK(c, launch_copy_block(G, n, n, n, L, n, s));
  for (int j = 0; j < n; j += b) {
    const int nb = std::min(b, n - j), m = n - j - nb;
    double* Ajj = L + j + (int64_t)n * j;
    HIPCHK(c, launch_copy_block(Ajj, n, nb, nb, ws, nb, s));
    HIPCHK(c, launch_chol_lds(ws, nb, ws + b * b, ws + 2 * b * b, c->rdiag, c->status, s));
    HIPCHK(c, launch_copy_block(ws + b * b, nb, nb, nb, Ajj, n, s));
    if (j > 0) HIPCHK(c, launch_copy_block(nullptr, 0, j, nb, L + (int64_t)n * j, n, s));   // above the block
    if (m > 0) {
      BLASCHK(c, rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                               rocblas_diagonal_non_unit, m, nb, &one, Ajj, n, Ajj + nb, n));
      BLASCHK(c, rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_transpose, m, m, nb, &mone, Ajj + nb,
                               n, Ajj + nb, n, &one, Ajj + nb + (int64_t)n * nb, n));
    }
  }
  return TR_OK;
}

// C (P x Q) = op(A) B over a long inner dimension K, split into chunks whose
// products (one strided-batched rocBLAS call, plus one for the remainder) are
// summed in chunk order: rocBLAS runs such reduction-shaped products (small
// C, K up to 10^6) as one long serial sweep otherwise.  trans_a: A is K x P
// (ld lda), C = A^T B; else A is P x K (ld lda), C = A B.  B is K x Q (ld ldb).
int blas_long_product(tr_als_ctx* c, bool trans_a, const double* A, int64_t lda, const double* B, int64_t ldb,
                      int64_t K, int P, int Q, double* C, hipStream_t s) {
  const int64_t pq = (int64_t)P * Q;
  int64_t nch = std::min<int64_t>({64, c->qpart_elems / pq - 1, std::max<int64_t>(1, K / 256)});
  if (nch < 1) return fail(c, TR_EHIP, "internal: chunk buffer too small");
  const int64_t kc = K / nch, rem = K - nch * kc;
  const double one = 1.0, zero = 0.0;
  const rocblas_operation ta = trans_a ? rocblas_operation_transpose : rocblas_operation_none;
  const int64_t sa = trans_a ? kc : kc * lda;   // start of chunk q of A: row q kc (A^T) or column q kc
  BLASCHK(c, rocblas_dgemm_strided_batched(c->blas, ta, rocblas_operation_none, P, Q, (int)kc, &one, A, (int)lda, sa, B,
                                           (int)ldb, kc, &zero, c->qpart, P, pq, (int)nch));
  if (rem > 0)
    BLASCHK(c, rocblas_dgemm(c->blas, ta, rocblas_operation_none, P, Q, (int)rem, &one, A + nch * sa, (int)lda,
                             B + nch * kc, (int)ldb, &zero, c->qpart + nch * pq, P));
  HIPCHK(c, launch_sum_chunks(c->qpart, (int)(nch + (rem > 0 ? 1 : 0)), pq, C, s));
  return TR_OK;
}

// W = Y_[n] B (I_n x Q) for the Multi-TTM result Y with extents cd (mode n of
// size I_n between L = prod cd[0..n) and T = prod cd(n..N)) and B (L T x Q,
// rows in Y's order, ld ldb).  For a middle mode the slices of Y are
// transposed first into tmp (L I T doubles), so that Y_[n] is I_n x (L T).
int blas_mode_product(tr_als_ctx* c, const double* Y, const int64_t* cd, int m, const double* B, int64_t ldb, int Q,
                      double* W, double* tmp, hipStream_t s) {
  const int64_t L = prod(cd, 0, m), I = c->dims[m], T = prod(cd, m + 1, c->N);
  if (T == 1) return blas_long_product(c, true, Y, L, B, ldb, L, (int)I, Q, W, s);
  if (L > 1) {
    HIPCHK(c, launch_slice_transpose(Y, L, I, T, tmp, s));
    Y = tmp;
  }
  return blas_long_product(c, false, Y, I, B, ldb, L * T, (int)I, Q, W, s);
}

// Mode-2 QR of core k (Definition of the mode-n QR): Q_k and the R-core.
// A tall unfolding with more than 128 columns (I_k >= R_k R_{k+1} > 128) is
// factored by the shifted Cholesky-QR (three passes, as for V_n[2]) on
// rocBLAS: Q_k = A L_1^{-T} L_2^{-T} L_3^{-T}, R = (L_1 L_2 L_3)^T.  The
// factors can differ from Householder's by the signs of matching columns of Q
// and rows of R, which leaves every product Q_k R the same.
int qr_core(tr_als_ctx* c, int k) {
  hipStream_t s = c->stream;
  const int Ra = c->R[k], Rb = c->R[k + 1], n = Ra * Rb;
  const int64_t I = c->dims[k], r = c->qr_r[k];
  HIPCHK(c, launch_core_unfold(c->cores[k], Ra, I, Rb, c->qA, s));
  if (n > 128 && I >= n) {
    int rc = blas_on(c, s);
    if (rc) return rc;
    const double one = 1.0;
    for (int it = 0; it < 3; ++it) {
      rc = blas_long_product(c, true, c->qA, I, c->qA, I, I, n, n, c->qG, s);
      if (rc) return rc;
      if (it == 0) HIPCHK(c, launch_shift_and_add(c->qG, n, I, c->qshift, s));
      rc = chol_lower_blocked(c, c->qG, n, c->qL[it], c->qLT, s);
      if (rc) return rc;
      BLASCHK(c, rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                               rocblas_diagonal_non_unit, (int)I, n, &one, c->qL[it], n, c->qA, (int)I));
    }
    MatView L1{c->qL[0], n, 0, 0, 0}, L2{c->qL[1], n, 0, 0, 0}, L3{c->qL[2], n, 0, 0, 0}, Lp{c->qLp, n, 0, 0, 0};
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, L1, L2, 0.0, nullptr, 0, c->qLp, n, s));
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, Lp, L3, 0.0, nullptr, 0, c->qLt, n, s));
    HIPCHK(c, hipMemcpyAsync(c->qQ[k], c->qA, (size_t)I * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, launch_transpose(c->qLt, n, n, c->qRt, s));
  } else if (n > 128 && I < n && householder_in_registers(I, 16)) {
    // a wide unfolding (Q_k square): Householder on panels of w columns in
    // one workgroup's registers, each panel's factor Q_p taken out of the
    // columns to its right by block Gram-Schmidt applied twice (the second
    // pass restores orthogonality to rounding), so Q = [Q_1 ... Q_p] and
    // R = [R_pp on the diagonal, Q_p^T A on its right, zeros below]
    int w = 128;
    while (!householder_in_registers(I, w)) w /= 2;
    const int ni = (int)I;
    double* T1 = c->qV;    // w x (n - w) at most: within I x n
    double* T2 = c->qRi;   // within n x n
    HIPCHK(c, launch_copy_block(nullptr, 0, (int)r, n, c->qRt, r, s));
    for (int c0 = 0; c0 < (int)r; c0 += w) {
      const int wp = std::min<int>(w, (int)r - c0), rest = n - c0 - wp;
      double* Qp = c->qQ[k] + (int64_t)c0 * I;
      double* Ar = c->qA + (int64_t)(c0 + wp) * I;   // the columns right of the panel
      HIPCHK(c, launch_householder_qr(c->qA + (int64_t)c0 * I, I, wp, c->qV, c->qtau, Qp, c->qLT, s));
      HIPCHK(c, launch_copy_block(c->qLT, wp, wp, wp, c->qRt + c0 + r * c0, r, s));
      if (rest == 0) continue;
      const MatView Qt{Qp, I, 2, 0, 0}, Qv{Qp, I, 0, 0, 0};
      for (int pass = 0; pass < 2; ++pass) {
        double* T = pass == 0 ? T1 : T2;
        const MatView Av{Ar, I, 0, 0, 0}, Tv{T, wp, 0, 0, 0};
        HIPCHK(c, launch_gemm64(wp, rest, ni, 1.0, Qt, Av, 0.0, nullptr, 0, T, wp, s));        // T = Q_p^T A_r
        HIPCHK(c, launch_gemm64(ni, rest, wp, -1.0, Qv, Tv, 1.0, Ar, I, Ar, I, s));          // A_r -= Q_p T
      }
      HIPCHK(c, launch_copy_block(T2, wp, wp, rest, T1, wp, s, 0, true));
      HIPCHK(c, launch_copy_block(T1, wp, wp, rest, c->qRt + c0 + r * (c0 + wp), r, s));
    }
  } else {
    HIPCHK(c, launch_householder_qr(c->qA, I, n, c->qV, c->qtau, c->qQ[k], c->qRt, s));
  }
  HIPCHK(c, launch_core_fold(c->qRt, r, Ra, Rb, c->qR[k], s));
  return TR_OK;
}

// One mode product out = cur x_j Q_j^T of the Multi-TTM (cd: the extents of
// cur, updated); cur is in type ctype, scaled by scale on the way in.
int ttm_step(tr_als_ctx* c, const void* cur, int ctype, double scale, int j, int64_t* cd, double* out) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const int64_t L = prod(cd, 0, j), T = prod(cd, j + 1, N);
  const int64_t I = c->dims[j], R = c->qr_r[j];
  if (ctype == TR_F64 && scale == 1.0 && (I > 112 || R > 112)) {
    // out(l, r, t) = sum_i in(l + L (i + I t)) Q(i, r): Q^T in_[j] per slice t
    int rc = blas_on(c, s);
    if (rc) return rc;
    const double one = 1.0, zero = 0.0;
    const double* in = (const double*)cur;
    if (L == 1) {
      BLASCHK(c, rocblas_dgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)R, (int)T, (int)I,
                               &one, c->qQ[j], (int)I, in, (int)I, &zero, out, (int)R));
    } else {
      BLASCHK(c, rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none, (int)L,
                                               (int)R, (int)I, &one, in, (int)L, L * I, c->qQ[j], (int)I, 0, &zero,
                                               out, (int)L, L * R, (int)T));
    }
  } else {
    HIPCHK(c, launch_ttm(cur, ctype, L, I, T, c->qQ[j], (int)R, scale, out, s));
  }
  cd[j] = c->qr_r[j];
  return TR_OK;
}

// Multi-TTM Y = X x_{j!=m} Q_j^T of the QR-based variants (Alg. 3 and 4), the
// most compressing mode first: the first TTM reads X in the contraction type
// (the BF16/FP8 shadows), the rest run in FP64 on the compressed tensor.  *Y
// is one of the ping-pong buffers; cd receives the extents of Y.
// Within a sweep (tree) the modes go in pairs (p, p+1), p even: mode p forms
// Z = X x_{j not in {p, p+1}} Q_j^T once, keeps it, and takes Y = Z x_{p+1}
// Q_{p+1}^T; mode p+1 takes Y = Z x_p Q_p^T with the Q_p of its update.  Z's
// factors do not change between the two updates, so both Y are those of the
// definition (the products taken in another order), with one TTM pass in
// place of two at order 4.
int multi_ttm_y(tr_als_ctx* c, int m, int prec, bool tree, const double** Y, int64_t* cd) {
  const int N = c->N;
  const int p = m & ~1;
  const bool paired = tree && N >= 3 && p + 1 < N && c->qZ;
  if (paired && m == p + 1 && c->z_pair == p && c->z_prec == prec) {
    for (int j = 0; j < N; ++j) cd[j] = c->z_cd[j];
    c->z_pair = -1;
    int rc = ttm_step(c, c->qZ, TR_F64, 1.0, p, cd, c->qY0);
    if (rc) return rc;
    *Y = c->qY0;
    return TR_OK;
  }
  c->z_pair = -1;
  std::vector<int> order;
  for (int k = 1; k < N; ++k) {
    const int j = (m + k) % N;
    if (!(paired && m == p && j == p + 1)) order.push_back(j);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)c->qr_r[a] / c->dims[a] < (double)c->qr_r[b] / c->dims[b];
  });
  for (int j = 0; j < N; ++j) cd[j] = c->dims[j];
  int rc = ensure_shadow(c, prec);
  if (rc) return rc;
  const void* cur = prec == TR_BF16 ? c->xbf16 : prec == TR_FP8 ? c->xfp8 : c->X;
  int ctype = (prec == TR_BF16 || prec == TR_FP8) ? prec : c->xdt;
  if (prec == TR_F64 && ctype == TR_F32 && !order.empty()) {
    // a large first mode product on the FP64 path: X widened to FP64 once (into
    // the second ping-pong buffer, free until the second product) for rocBLAS
    const int j = order[0];
    if (c->dims[j] > 112 || c->qr_r[j] > 112) {
      HIPCHK(c, launch_widen_f32((const float*)c->X, c->numel, c->qY1, c->stream));
      cur = c->qY1;
      ctype = TR_F64;
    }
  }
  double scale = prec == TR_FP8 ? 1.0 / (double)c->fp8_scale : 1.0;
  double* ybuf[2] = {c->qY0, c->qY1};
  int yi = 0;
  for (size_t q = 0; q < order.size(); ++q) {
    // Z, the last product of mode p's shared part, goes to its own buffer
    double* out = (paired && m == p && q + 1 == order.size()) ? c->qZ : ybuf[yi];
    rc = ttm_step(c, cur, ctype, scale, order[q], cd, out);
    if (rc) return rc;
    cur = out;
    yi ^= 1;
    ctype = TR_F64;
    scale = 1.0;
  }
  if (paired && m == p) {
    for (int j = 0; j < N; ++j) c->z_cd[j] = cd[j];
    c->z_pair = p;
    c->z_prec = prec;
    double* out = cur == c->qY0 ? c->qY1 : c->qY0;
    rc = ttm_step(c, cur, TR_F64, 1.0, p + 1, cd, out);
    if (rc) return rc;
    cur = out;
  }
  *Y = (const double*)cur;
  return TR_OK;
}

// V_n = subchain of the R-cores of the other modes, unfolded as V_n[2]
// (J' x R_m R_{m+1}, rows in the order of the Multi-TTM result); returns J'.
int build_v2(tr_als_ctx* c, int m, int64_t* Jp_out) {
  const int N = c->N;
  std::vector<int> chain;
  for (int k = 1; k < N; ++k) chain.push_back((m + k) % N);
  int64_t Jp = 1;
  for (int j : chain) Jp *= c->qr_r[j];
  int64_t Lrows = 1;
  for (int j = 0; j < m; ++j) Lrows *= c->qr_r[j];
  const int last = chain.back();
  if (!v2_direct_fits(c->R[last], c->R[m], c->R[m + 1])) {   // full table, then reordered
    int rc = build_table_ex(c, chain, c->R[m + 1], c->qT, c->qR, c->qr_r, c->qY0, c->qY1);
    if (rc) return rc;
    HIPCHK(c, launch_table_to_v2(c->qT, Jp, Lrows, c->R[m], c->R[m + 1], c->qV2, c->stream));
    *Jp_out = Jp;
    return TR_OK;
  }
  // the subchain without its last core as a table, then the last step
  // written straight in the V_n[2] layout
  chain.pop_back();
  int rc = build_table_ex(c, chain, c->R[m + 1], c->qT, c->qR, c->qr_r, c->qY0, c->qY1);
  if (rc) return rc;
  HIPCHK(c, launch_v2_direct(c->qT, Jp / c->qr_r[last], c->qR[last], c->qr_r[last], c->R[last], c->R[m], c->R[m + 1],
                             Lrows, c->qV2, c->stream));
  *Jp_out = Jp;
  return TR_OK;
}

// One QR-variant mode update (Alg. 3): V_n = subchain of the R-cores; QR of
// V_n[2] = Q_0 R_[2] by shifted Cholesky-QR (three passes); Y = X x_{j!=n} Q_j^T
// (most-compressing mode first); W_n = Y_[n] Q_0; G_n(2) R_[2]^T = W_n by
// substitution; commit; re-factor core n and refresh its R-core Gram.  The
// first pass's Gram V_n[2]^T V_n[2] is the ring product of the R-cores' Grams
// (Prop. 3.1 applied to the R-cores), as in Alg. 4: only its Cholesky factor,
// taken with the shift, enters, as a preconditioner; the second and third
// passes form their Grams from the rows.
// The same update for n = R_n R_{n+1} > 128, its large products on rocBLAS:
// the Grams split over chunks of rows, the shifted Cholesky-QR passes
// A <- A L^{-T} as in-place triangular solves with the blocked Cholesky factor
// (the third applied to W_n instead of V_n[2]), W_n = Y_[n] Q_0, and
// G_n(2) = W_n R^{-T}.
int update_mode_qr_large(tr_als_ctx* c, int m, int prec, bool in_sweep, int64_t Jp) {
  hipStream_t s = c->stream;
  const int Ra = c->R[m], Rb = c->R[m + 1], n = Ra * Rb;
  const double one = 1.0;
  int rc = blas_on(c, s);
  if (rc) return rc;
  double* A = c->qV2;   // V_n[2], orthogonalised in place (two passes; Q_0 = A L_3^{-T})
  for (int it = 0; it < 3; ++it) {
    // first pass: V_n[2]^T V_n[2] from the ring of the R-cores' Grams
    rc = it == 0 ? compute_coef(c, m, c->qG, s) : blas_long_product(c, true, A, Jp, A, Jp, Jp, n, n, c->qG, s);
    if (rc) return rc;
    if (it == 0) HIPCHK(c, launch_shift_and_add(c->qG, n, Jp, c->qshift, s));
    rc = chol_lower_blocked(c, c->qG, n, c->qL[it], c->qLT, s);
    if (rc) return rc;
    if (it < 2)
      BLASCHK(c, rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                               rocblas_diagonal_non_unit, (int)Jp, n, &one, c->qL[it], n, A, (int)Jp));
  }
  {
    MatView L1{c->qL[0], n, 0, 0, 0}, L2{c->qL[1], n, 0, 0, 0}, L3{c->qL[2], n, 0, 0, 0}, Lp{c->qLp, n, 0, 0, 0};
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, L1, L2, 0.0, nullptr, 0, c->qLp, n, s));
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, Lp, L3, 0.0, nullptr, 0, c->qLt, n, s));
  }
  int64_t cd[TR_MAXN];
  const double* Y = nullptr;
  rc = multi_ttm_y(c, m, prec, in_sweep, &Y, cd);
  if (rc) return rc;
  rc = blas_on(c, s);
  if (rc) return rc;
  // W_n = Y_[n] Q_0 = (Y_[n] A) L_3^{-T}
  rc = blas_mode_product(c, Y, cd, m, A, Jp, n, c->qW, Y == c->qY0 ? c->qY1 : c->qY0, s);
  if (rc) return rc;
  const int64_t I = c->dims[m];
  BLASCHK(c, rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                           rocblas_diagonal_non_unit, (int)I, n, &one, c->qL[2], n, c->qW, (int)I));
  // G_n(2) R_[2]^T = W_n with R_[2]^T = L_1 L_2 L_3 (lower): G L = W
  HIPCHK(c, hipMemcpyAsync(c->Gn, c->qW, (size_t)I * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  BLASCHK(c, rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                           rocblas_diagonal_non_unit, (int)I, n, &one, c->qLt, n, c->Gn, (int)I));
  HIPCHK(c, launch_commit_core(c->Gn, I, Ra, Rb, c->cores[m], c->status, s));
  rc = qr_core(c, m);
  if (rc) return rc;
  HIPCHK(c, launch_gram(c->qR[m], Ra, c->qr_r[m], Rb, c->gram[m], s));
  return TR_OK;
}

int update_mode_qr(tr_als_ctx* c, int m, int prec, bool in_sweep) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const int Ra = c->R[m], Rb = c->R[m + 1], n = Ra * Rb;
  // V_n[2] (J' x n), rows in the order of the Multi-TTM result below
  int64_t Jp = 1;
  int rc = build_v2(c, m, &Jp);
  if (rc) return rc;
  if (n > 128) return update_mode_qr_large(c, m, prec, in_sweep, Jp);
  // shifted Cholesky-QR: passes A <- A L^{-T}, R^T = L1 L2 L3; the first two
  // are applied to V_n[2], the third to W_n
  double* A = c->qV2;
  double* bufs[2] = {c->qQa, c->qQb};
  for (int it = 0; it < 3; ++it) {
    if (it == 0) {   // V_n[2]^T V_n[2] from the ring of the R-cores' Grams
      rc = compute_coef(c, m, c->qG, s);
      if (rc) return rc;
    } else {
      HIPCHK(c, launch_tall_atb(A, Jp, A, Jp, Jp, n, n, 0, 1, 1, 1, c->qpart, c->qpart_elems, c->qG, s));
    }
    if (it == 0) HIPCHK(c, launch_shift_and_add(c->qG, n, Jp, c->qshift, s));
    HIPCHK(c, launch_chol_lds(c->qG, n, c->qL[it], c->qLT, c->rdiag, c->status, s));
    if (it == 2) break;   // Q_0 = A L_3^{-T} is applied to W_n instead
    HIPCHK(c, launch_trsm_rhs(c->qL[it], c->rdiag, n, nullptr, n, c->qRi, 0, c->status, s, 1));
    if (n <= 112) {
      HIPCHK(c, launch_tall_gemm(A, Jp, Jp, n, c->qRi, n, n, bufs[it & 1], Jp, s, true));
    } else {
      MatView Av{A, Jp, 0, 0, 0}, Ri{c->qRi, n, 0, 0, 0};
      HIPCHK(c, launch_gemm64(Jp, n, n, 1.0, Av, Ri, 0.0, nullptr, 0, bufs[it & 1], Jp, s));
    }
    A = bufs[it & 1];
  }
  {
    MatView L1{c->qL[0], n, 0, 0, 0}, L2{c->qL[1], n, 0, 0, 0}, L3{c->qL[2], n, 0, 0, 0}, Lp{c->qLp, n, 0, 0, 0};
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, L1, L2, 0.0, nullptr, 0, c->qLp, n, s));
    HIPCHK(c, launch_gemm64(n, n, n, 1.0, Lp, L3, 0.0, nullptr, 0, c->qLt, n, s));
  }
  int64_t cd[TR_MAXN];
  const double* Y = nullptr;
  rc = multi_ttm_y(c, m, prec, in_sweep, &Y, cd);
  if (rc) return rc;
  // W_n = Y_[n] Q_0 = (Y_[n] A) L_3^{-T} (I_n x n), Y_[n] A staged in M
  HIPCHK(c, launch_tall_atb(Y, 0, A, Jp, Jp, (int)c->dims[m], n, 1, prod(cd, 0, m), c->dims[m],
                            prod(cd, m + 1, N), c->qpart, c->qpart_elems, c->M, s));
  HIPCHK(c, launch_trsm_rhs(c->qL[2], c->rdiag, n, c->M, c->dims[m], c->qW, 0, c->status, s, 1));
  // G_n(2) = W_n R^{-T}: backward substitution with L = R^T
  HIPCHK(c, launch_trsm_rhs(c->qLt, nullptr, n, c->qW, c->dims[m], c->Gn, 0, c->status, s, 2));
  HIPCHK(c, launch_commit_core(c->Gn, c->dims[m], Ra, Rb, c->cores[m], c->status, s));
  rc = qr_core(c, m);
  if (rc) return rc;
  HIPCHK(c, launch_gram(c->qR[m], Ra, c->qr_r[m], Rb, c->gram[m], s));
  return TR_OK;
}

// One QRNE mode update (Alg. 4): S_n from the ring of the R-cores' Grams and
// its inverse; V_n[2] from the R-cores; Y = X x_{j!=n} Q_j^T; M_n = Y_[n] V_n[2];
// G_n(2) = M_n S_n^{-1} with iterative refinement; commit; re-factor core n
// and refresh its R-core Gram.  The Grams of the R-cores equal those of the
// cores (Q_j has orthonormal columns); Alg. 4 forms them from the R-cores.
int update_mode_qrne(tr_als_ctx* c, int m, int prec, int refine, bool in_sweep) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const int Ra = c->R[m], Rb = c->R[m + 1], n = Ra * Rb;
  int rc = compute_coef(c, m, c->S, s);
  if (rc) return rc;
  if (c->solve == TR_SOLVE_PINV) {
    HIPCHK(c, launch_pinv(c->S, n, pinv_rcond(c, n), c->Sinv, c->pinvw, c->status, s));
  } else if (spd_inverse_fits(n)) {
    HIPCHK(c, launch_spd_inverse(c->S, n, c->Sinv, c->status, s));
  } else {
    rc = spd_inverse_blocked(c, c->S, n, c->Sinv, c->blkw, s);
    if (rc) return rc;
  }
  int64_t Jp = 1;
  rc = build_v2(c, m, &Jp);
  if (rc) return rc;
  int64_t cd[TR_MAXN];
  const double* Y = nullptr;
  rc = multi_ttm_y(c, m, prec, in_sweep, &Y, cd);
  if (rc) return rc;
  // M_n = Y_[n] V_n[2] (I_n x n)
  if (n > 128) {
    rc = blas_on(c, s);
    if (rc) return rc;
    rc = blas_mode_product(c, Y, cd, m, c->qV2, Jp, n, c->M, Y == c->qY0 ? c->qY1 : c->qY0, s);
    if (rc) return rc;
  } else {
    HIPCHK(c, launch_tall_atb(Y, 0, c->qV2, Jp, Jp, (int)c->dims[m], n, 1, prod(cd, 0, m), c->dims[m],
                              prod(cd, m + 1, N), c->qpart, c->qpart_elems, c->M, s));
  }
  HIPCHK(c, launch_ne_apply(c->M, c->dims[m], n, c->S, c->Sinv, refine, c->Gn, c->status, s));
  HIPCHK(c, launch_commit_core(c->Gn, c->dims[m], Ra, Rb, c->cores[m], c->status, s));
  rc = qr_core(c, m);
  if (rc) return rc;
  HIPCHK(c, launch_gram(c->qR[m], Ra, c->qr_r[m], Rb, c->gram[m], s));
  return TR_OK;
}

int read_status(tr_als_ctx* c) {
  int st = 0;
  HIPCHK(c, hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->prof) {
    for (auto& e : c->evs) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) { c->prof_ms += ms; c->prof_launches++; }
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    c->evs.clear();
  }
  if (st == 0) return TR_OK;
  // the context stays usable: clear the latched word for the next call
  HIPCHK(c, hipMemsetAsync(c->status, 0, sizeof(int), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (st & ST_SINGULAR) return fail(c, TR_ESINGULAR, "coefficient matrix not positive definite (or zero pivot)");
  return fail(c, TR_ENONFINITE, "non-finite value in M_n or in an updated core");
}

int store_cores(tr_als_ctx* c) {
  for (int k = 0; k < c->N; ++k) {
    const size_t bytes = (size_t)c->R[k] * c->dims[k] * c->R[k + 1] * sizeof(double);
    HIPCHK(c, hipMemcpyAsync(c->user_cores[k], c->cores[k], bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  return TR_OK;
}

int valid_ctx(const tr_als_ctx* c) { return c != nullptr && c->N >= 2; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* tr_als_strerror(int status) {
  switch (status) {
    case TR_OK: return "ok";
    case TR_EINVAL: return "invalid argument";
    case TR_ENOMEM: return "out of device memory";
    case TR_EHIP: return "HIP runtime error";
    case TR_ESINGULAR: return "singular coefficient matrix";
    case TR_ENONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* tr_als_last_error(const tr_als_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int tr_als_destroy(tr_als_ctx* ctx) {
  if (!ctx) return TR_OK;
  if (ctx->measure) {
    delete ctx;
    return TR_OK;
  }
  (void)hipStreamSynchronize(ctx->stream);   // the caller's stream, possibly the default one
  for (auto& e : ctx->evs) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& row : ctx->graphs)
    for (auto& g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (ctx->stream2) {
    (void)hipStreamSynchronize(ctx->stream2);
    if (ctx->own_stream2) (void)hipStreamDestroy(ctx->stream2);
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->canary) check_guards(ctx);
  if (ctx->blas) (void)rocblas_destroy_handle(ctx->blas);
  for (void* p : ctx->allocs) (void)hipFree(p);
  delete ctx;
  return TR_OK;
}

int tr_als_init(tr_als_ctx** out, int N, const int64_t* dims, const int64_t* ranks, const void* X, int x_dtype,
                double* const* cores, int variant, void* hip_stream) {
  return trx_init(out, N, dims, ranks, X, x_dtype, cores, variant, (hipStream_t)hip_stream, TrxOpts());
}

}  // extern "C"

int trx_init(tr_als_ctx** out, int N, const int64_t* dims, const int64_t* ranks, const void* X, int x_dtype,
             double* const* cores, int variant, hipStream_t hip_stream, const TrxOpts& o) {
  if (!out) return TR_EINVAL;
  *out = nullptr;
  if (o.measure) {
    if (!o.measured) return TR_EINVAL;
    *o.measured = 0;
  }
  if (N < 2 || N > TR_MAXN || !dims || !ranks || (!o.measure && (!X || !cores))) return TR_EINVAL;
  if (x_dtype != TR_F64 && x_dtype != TR_F32) return TR_EINVAL;
  if (variant != TR_NE && variant != TR_QR && variant != TR_QRNE) return TR_EINVAL;
  int64_t numel = 1;
  for (int k = 0; k < N; ++k) {
    if (dims[k] < 1 || ranks[k] < 1 || ranks[k] > TR_MAXR) return TR_EINVAL;
    if (numel > (int64_t(1) << 62) / dims[k]) return TR_EINVAL;
    numel *= dims[k];
    if (!o.measure && !cores[k]) return TR_EINVAL;
  }
  tr_als_ctx* c = new tr_als_ctx();
  c->measure = o.measure;
  c->region = o.region;
  static const bool env_canary = getenv("TR_ALS_CANARY") && getenv("TR_ALS_CANARY")[0] == '1';
  c->canary = env_canary;
  c->region_cap = o.region_bytes;
  c->N = N;
  for (int k = 0; k < N; ++k) { c->dims[k] = dims[k]; c->R[k] = (int)ranks[k]; }
  c->R[N] = c->R[0];
  c->variant = variant;
  c->xdt = x_dtype;
  c->X = X;
  c->numel = numel;
  c->stream = hip_stream;
  if (!o.measure) c->user_cores.assign(cores, cores + N);
  if (const char* ev = getenv("TR_ALS_NO_GRAPH")) c->graphs_ok = (ev[0] == '0');
  if (o.graphs >= 0) c->graphs_ok = o.graphs == 1;
  for (int m = 0; m < N; ++m) c->plan[m] = make_plan(c, m);
  // within a sweep, mode m can reuse mode m-1's group table when the groups
  // match and the core updated by mode m-1 is not part of it
  for (int m = 1; m < N; ++m) {
    const Plan& a = c->plan[m - 1];
    Plan& b = c->plan[m];
    b.reuse_prev = a.regime == 1 && b.regime == 1 && a.gcores == b.gcores &&
                   std::find(b.gcores.begin(), b.gcores.end(), m - 1) == b.gcores.end();
    // X and the table being the same, so is the stage-1 result: mode m-1
    // leaves it in Y0 when its absorptions take at most two steps (the first
    // writes Y1 or M, the second M)
    b.reuse_y = b.reuse_prev && !a.steps.empty() && a.steps.size() <= 2 && !b.steps.empty();
  }

  // workspace sizes
  int64_t maxI = 0, maxRR = 0, maxF = 0, maxT = 0, maxW = 0;
  for (int k = 0; k < N; ++k) {
    maxI = std::max<int64_t>(maxI, dims[k]);
    maxRR = std::max<int64_t>(maxRR, (int64_t)c->R[k] * c->R[k + 1]);
    maxW = std::max<int64_t>(maxW, (int64_t)c->R[k] * c->R[k] * c->R[k + 1] * c->R[k + 1]);
  }
  // ring intermediates of mode m: R_{m+1}^2 x R_{k+1}^2 after the factor K_k
  for (int m = 0; m < N; ++m) {
    const int64_t a = (int64_t)c->R[(m + 1) % N] * c->R[(m + 1) % N];
    for (int q = 2; q < N; ++q) {
      const int64_t r = c->R[(m + q + 1) % N];
      maxW = std::max<int64_t>(maxW, a * r * r);
    }
  }
  int64_t maxY = 16;
  for (int m = 0; m < N; ++m) {
    const Plan& p = c->plan[m];
    maxF = std::max(maxF, std::max(table_elems(c, p.f1c, p.Rmid), table_elems(c, p.f2c, p.Rmid)));
    maxT = std::max(maxT, std::max(table_build_max(c, p.f1c), table_build_max(c, p.f2c)));
    if (p.regime == 1) {
      maxF = std::max(maxF, table_elems(c, p.gcores, 1));
      maxT = std::max(maxT, table_build_max(c, p.gcores));
      maxY = std::max(maxY, p.gM * p.gC);
    }
  }
  size_t pbytes = 0;
  int rc = TR_OK;
  auto A = [&](void** p, size_t b) { if (rc == TR_OK) rc = alloc(c, p, b); };
  for (int k = 0; k < N; ++k) {
    A((void**)&c->cores[k], (size_t)c->R[k] * dims[k] * c->R[k + 1] * 8);
    A((void**)&c->gram[k], (size_t)c->R[k] * c->R[k + 1] * c->R[k] * c->R[k + 1] * 8);
  }
  A((void**)&c->F1, (size_t)maxF * 8);
  A((void**)&c->F2, (size_t)maxF * 8);
  A((void**)&c->T0, (size_t)maxT * 8);
  A((void**)&c->T1, (size_t)maxT * 8);
  A((void**)&c->M, (size_t)maxI * maxRR * 8);
  A((void**)&c->Gn, (size_t)maxI * maxRR * 8);
  A((void**)&c->G0u, (size_t)maxI * maxRR * 8);
  A((void**)&c->S, (size_t)maxRR * maxRR * 8);
  A((void**)&c->Lf, (size_t)maxRR * maxRR * 8);
  A((void**)&c->LTf, (size_t)maxRR * maxRR * 8);
  A((void**)&c->cholw, (size_t)maxRR * maxRR * 8);
  A((void**)&c->LinvT, (size_t)maxRR * maxRR * 8);
  A((void**)&c->Sinv, (size_t)maxRR * maxRR * 8);
  A((void**)&c->pinvw, (size_t)2 * maxRR * maxRR * 8);
  A((void**)&c->blkw, (size_t)spd_inverse_blocked_ws((int)maxRR) * 8);
  A((void**)&c->rdiag, 256 * 8);
  A((void**)&c->Tsol, (size_t)maxI * maxRR * 8);
  A((void**)&c->W0, (size_t)maxW * 8);
  A((void**)&c->Y0, (size_t)maxY * 8);
  A((void**)&c->Y1, (size_t)maxY * 8);
  A((void**)&c->W1, (size_t)maxW * 8);
  if (N >= 4) {
    A((void**)&c->Wpre[0], (size_t)maxW * 8);
    A((void**)&c->Wpre[1], (size_t)maxW * 8);
  }
  c->w_cap = maxW;
  A((void**)&c->dpart, (size_t)c->nred * 8);
  A((void**)&c->fpart, (size_t)c->nred * 4);
  A((void**)&c->dscal, 8 * 8);
  A((void**)&c->fscal, 8 * 4);
  A((void**)&c->status, 16);
  if (rc) { std::string e = c->err; tr_als_destroy(c); (void)e; return rc; }
  size_t btb = 16;
  for (int m = 0; m < N; ++m)
    for (int prec = TR_F64; prec <= TR_FP8; ++prec) {
      if (c->plan[m].regime == 1) {
        const int es = prec == TR_BF16 ? 2 : prec == TR_FP8 ? 1 : (x_dtype == TR_F64 ? 8 : 4);
        for (int mt : {64, 128}) {
          XgArgs g = xg_config(c, m, prec, X, es, false, mt);
          pbytes = std::max(pbytes, xg_partial_bytes(g, prec));
          btb = std::max(btb, xg_bt_bytes(g, prec));
        }
      } else {
        XsCfg x = xs_config(c, m, prec);
        pbytes = std::max(pbytes, partial_bytes_needed(x, prec));
        if (c->plan[m].slab && prec != TR_FP8) {
          const XslabArgs a = xslab_config(c, m, X);
          pbytes = std::max(pbytes, xslab_partial_bytes(a, prec));
          btb = std::max(btb, xslab_bt_bytes(a, prec));
        }
      }
    }
  A(&c->partial, pbytes);
  c->partial_bytes = pbytes;
  A(&c->Bt, btb);
  c->bt_bytes = btb;
  if (variant == TR_QR || variant == TR_QRNE) {
    int64_t maxJ = 1, maxTT = 1, maxHn = 1, nq = 128;
    for (int k = 0; k < N; ++k) c->qr_r[k] = std::min<int64_t>(dims[k], (int64_t)c->R[k] * c->R[k + 1]);
    for (int m = 0; m < N; ++m) {
      int64_t Jp = 1, tb = 1;
      for (int k = 1; k < N; ++k) {
        const int j = (m + k) % N;
        Jp *= c->qr_r[j];
        tb = std::max(tb, Jp * c->R[(m + 1) % N] * c->R[j + 1]);
      }
      const int64_t n = (int64_t)c->R[m] * c->R[m + 1];
      maxJ = std::max(maxJ, Jp * n);
      maxTT = std::max(maxTT, tb);
      maxHn = std::max(maxHn, (int64_t)dims[m] * n);
      nq = std::max(nq, n);
    }
    maxTT = std::max(maxTT, maxJ);
    for (int k = 0; k < N; ++k) {
      A((void**)&c->qQ[k], (size_t)dims[k] * c->qr_r[k] * 8);
      A((void**)&c->qR[k], (size_t)c->R[k] * c->qr_r[k] * c->R[k + 1] * 8);
    }
    A((void**)&c->qA, (size_t)maxHn * 8);
    A((void**)&c->qV, (size_t)maxHn * 8);
    A((void**)&c->qtau, 1024 * 8);
    A((void**)&c->qRt, (size_t)maxHn * 8);
    A((void**)&c->qT, (size_t)maxTT * 8);
    A((void**)&c->qV2, (size_t)maxJ * 8);
    A((void**)&c->qQa, (size_t)maxJ * 8);
    A((void**)&c->qQb, (size_t)maxJ * 8);
    A((void**)&c->qY0, (size_t)std::max(numel, maxTT) * 8);
    A((void**)&c->qY1, (size_t)std::max(numel, maxTT) * 8);
    if (N >= 3) A((void**)&c->qZ, (size_t)numel * 8);
    A((void**)&c->qW, (size_t)maxI * nq * 8);
    for (int it = 0; it < 3; ++it) A((void**)&c->qL[it], (size_t)nq * nq * 8);
    A((void**)&c->qG, (size_t)nq * nq * 8);
    A((void**)&c->qLT, (size_t)std::max<int64_t>(nq * nq, 3 * 112 * 112) * 8);
    A((void**)&c->qRi, (size_t)nq * nq * 8);
    A((void**)&c->qLp, (size_t)nq * nq * 8);
    A((void**)&c->qLt, (size_t)nq * nq * 8);
    A((void**)&c->qshift, 64);
    c->qpart_elems = (int64_t)512 * 128 * 128;
    A((void**)&c->qpart, (size_t)c->qpart_elems * 8);
    if (rc) { tr_als_destroy(c); return rc; }
  }
  // One transposed low-precision shadow serves the two-stage modes of the NE
  // variant that contract the slowest modes at the first such split
  // (TR_ALS_NO_XT=1: none, those modes read the plain shadow).
  static const bool no_xt = getenv("TR_ALS_NO_XT") && getenv("TR_ALS_NO_XT")[0] == '1';
  if (variant == TR_NE && !no_xt)
    for (int m = 0; m < N; ++m)
      if (c->plan[m].regime == 1 && c->plan[m].nn) {
        c->t_gK = c->plan[m].gK;
        break;
      }
  if (o.shadow_mask & (1u << TR_BF16)) {
    A(&c->xbf16, (size_t)numel * 2);
    if (c->t_gK) A(&c->xbf16t, (size_t)numel * 2);
  }
  if (o.shadow_mask & (1u << TR_FP8)) {
    A(&c->xfp8, (size_t)numel);
    if (c->t_gK) A(&c->xfp8t, (size_t)numel);
  }
  if (rc) { tr_als_destroy(c); return rc; }
  if (c->measure) {
    *o.measured = c->region_off;
    tr_als_destroy(c);
    return TR_OK;
  }

  hipStream_t s = c->stream;
  auto hipfail = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return false;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return true;
  };
  fill_guards(c, s);
  if (hipfail(hipMemsetAsync(c->status, 0, 16, s), "memset") ||
      (o.stream2 ? ((c->stream2 = o.stream2), (c->own_stream2 = false)) :
                   hipfail(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking), "stream")) ||
      hipfail(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "event") ||
      hipfail(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "event")) {
    tr_als_destroy(c);
    return TR_EHIP;
  }
  for (int k = 0; k < N; ++k) {
    const size_t bytes = (size_t)c->R[k] * dims[k] * c->R[k + 1] * 8;
    if (hipfail(hipMemcpyAsync(c->cores[k], cores[k], bytes, hipMemcpyDeviceToDevice, s), "copy cores") ||
        hipfail(launch_gram(c->cores[k], c->R[k], dims[k], c->R[k + 1], c->gram[k], s), "gram")) {
      tr_als_destroy(c);
      return TR_EHIP;
    }
  }
  if (variant == TR_QR || variant == TR_QRNE) {
    for (int k = 0; k < N && rc == TR_OK; ++k) rc = qr_core(c, k);
    if (rc) { tr_als_destroy(c); return rc; }
  }
  if (variant == TR_QR || variant == TR_QRNE)   // kept as the Grams of the R-cores
    for (int k = 0; k < N; ++k)
      if (hipfail(launch_gram(c->qR[k], c->R[k], c->qr_r[k], c->R[k + 1], c->gram[k], s), "gram")) {
        tr_als_destroy(c);
        return TR_EHIP;
      }
  if (hipfail(launch_sumsq(X, x_dtype, numel, c->dpart, c->nred, c->dscal, s), "sumsq")) {
    tr_als_destroy(c);
    return TR_EHIP;
  }
  // asynchronous creation leaves ||X||^2 on the device (dscal[0])
  if (!o.no_sync && (hipfail(hipMemcpyAsync(&c->xnorm2, c->dscal, 8, hipMemcpyDeviceToHost, s), "copy norm") ||
                     hipfail(hipStreamSynchronize(s), "sync"))) {
    tr_als_destroy(c);
    return TR_EHIP;
  }
  *out = c;
  return TR_OK;
}

size_t trx_footprint(int N, const int64_t* dims, const int64_t* ranks, int x_dtype, int variant,
                     unsigned shadow_mask) {
  TrxOpts o;
  size_t bytes = 0;
  o.measure = true;
  o.measured = &bytes;
  o.shadow_mask = shadow_mask;
  tr_als_ctx* c = nullptr;
  if (trx_init(&c, N, dims, ranks, nullptr, x_dtype, nullptr, variant, nullptr, o) != TR_OK) return 0;
  return bytes;
}

// ---------------------------------------------------------------------------
// Planted-tensor generator: true cores (Philox normals), the split of mode 1's
// subchain into two partial-subchain tables (as for the fit), X_true tiles,
// relative noise; optionally N(0,1) initial cores from the same key.
// ---------------------------------------------------------------------------
namespace {

struct GenLayout {
  Plan p;
  size_t cores[TR_MAXN] = {0};
  size_t F1 = 0, F2 = 0, T0 = 0, T1 = 0, G0 = 0, part = 0, scal = 0, total = 0;
  int nblk = 1024;
};

bool gen_shape(tr_als_ctx& g, int N, const int64_t* dims, const int64_t* ranks) {
  if (N < 2 || N > TR_MAXN || !dims || !ranks) return false;
  g.N = N;
  g.numel = 1;
  for (int k = 0; k < N; ++k) {
    if (dims[k] < 1 || ranks[k] < 1 || ranks[k] > TR_MAXR) return false;
    if (g.numel > (int64_t(1) << 62) / dims[k]) return false;
    g.dims[k] = dims[k];
    g.R[k] = (int)ranks[k];
    g.numel *= dims[k];
  }
  g.R[N] = g.R[0];
  return true;
}

GenLayout gen_layout(tr_als_ctx& g, bool need_true) {
  GenLayout L;
  L.p = make_plan(&g, 0);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += trx_round(bytes ? bytes : 16); return o; };
  for (int k = 0; k < g.N; ++k)
    L.cores[k] = need_true ? take((size_t)g.R[k] * g.dims[k] * g.R[k + 1] * 8) : 0;
  L.F1 = take((size_t)table_elems(&g, L.p.f1c, L.p.Rmid) * 8);
  L.F2 = take((size_t)table_elems(&g, L.p.f2c, L.p.Rmid) * 8);
  const int64_t tb = std::max<int64_t>(1, std::max(table_build_max(&g, L.p.f1c), table_build_max(&g, L.p.f2c)));
  L.T0 = take((size_t)tb * 8);
  L.T1 = take((size_t)tb * 8);
  L.G0 = take((size_t)L.p.I * L.p.Ra * L.p.Rb * 8);
  L.part = take((size_t)2 * L.nblk * 8);
  L.scal = take(8 * 8);
  L.total = off;
  return L;
}

}  // namespace

size_t trx_gen_workspace(int N, const int64_t* dims, const int64_t* ranks, bool need_true_cores) {
  tr_als_ctx g;
  if (!gen_shape(g, N, dims, ranks)) return 0;
  return gen_layout(g, need_true_cores).total;
}

int trx_gen(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X, int x_dtype,
            double* const* true_cores, double* const* init_cores, char* ws, size_t ws_bytes, hipStream_t s,
            std::string* err) {
  tr_als_ctx g;
  auto bad = [&](int code, const char* msg) { if (err) *err = msg; return code; };
  if (!gen_shape(g, N, dims, ranks) || !X || !ws || (x_dtype != TR_F64 && x_dtype != TR_F32) || !(eta >= 0.0))
    return bad(TR_EINVAL, "invalid generator arguments");
  const GenLayout L = gen_layout(g, true_cores == nullptr);
  if (ws_bytes < L.total) return bad(TR_EINVAL, "generator workspace too small");
  g.stream = s;
  for (int k = 0; k < N; ++k) {
    g.cores[k] = true_cores ? true_cores[k] : (double*)(ws + L.cores[k]);
    const int64_t n = (int64_t)g.R[k] * g.dims[k] * g.R[k + 1];
    if (launch_philox_normal(g.cores[k], n, seed, GEN_SID_TRUE + k, s) != hipSuccess)
      return bad(TR_EHIP, "generator launch failed");
    if (init_cores && launch_philox_normal(init_cores[k], n, seed, GEN_SID_INIT + k, s) != hipSuccess)
      return bad(TR_EHIP, "generator launch failed");
  }
  double* F1 = (double*)(ws + L.F1);
  double* F2 = (double*)(ws + L.F2);
  double* G0 = (double*)(ws + L.G0);
  const Plan& p = L.p;
  int rc = build_table_ex(&g, p.f1c, p.Rmid, F1, g.cores, g.dims, (double*)(ws + L.T0), (double*)(ws + L.T1));
  if (rc == TR_OK)
    rc = build_table_ex(&g, p.f2c, p.Rmid, F2, g.cores, g.dims, (double*)(ws + L.T0), (double*)(ws + L.T1));
  if (rc) return bad(rc, g.err.c_str());
  if (launch_core_unfold(g.cores[0], p.Ra, p.I, p.Rb, G0, s) != hipSuccess ||
      launch_gen_planted(X, x_dtype, p.I, p.K, G0, F1, F2, p.d1, p.m1, p.d2, p.m2, p.Rb, p.Rmid, p.Ra, seed, eta,
                         (double*)(ws + L.part), L.nblk, (double*)(ws + L.scal), s) != hipSuccess)
    return bad(TR_EHIP, "generator launch failed");
  return TR_OK;
}

extern "C" {

int tr_gen_planted(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X,
                   int x_dtype, double* const* true_cores, double* const* init_cores, void* hip_stream) {
  if (N < 2 || N > TR_MAXN || !dims || !ranks || !X) return TR_EINVAL;
  const size_t ws = trx_gen_workspace(N, dims, ranks, true_cores == nullptr);
  if (ws == 0) return TR_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  void* buf = nullptr;
  if (hipMalloc(&buf, ws) != hipSuccess) {
    (void)hipGetLastError();
    return TR_ENOMEM;
  }
  int rc = trx_gen(N, dims, ranks, seed, eta, X, x_dtype, true_cores, init_cores, (char*)buf, ws, s, nullptr);
  const hipError_t e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (rc == TR_OK && e != hipSuccess) rc = TR_EHIP;
  return rc;
}

// <A, B> of two tensors in TR format with the same dims (Sec. 3.4, read as
// the trace of the product of the transfer matrices T_1 ... T_N): per core
// the cross Gram A_k(2)^T B_k(2) on FP64 MFMA, reindexed into T_k, the ring
// product, its trace.
static int tr_inner_impl(int N, const int64_t* dims, const int64_t* ranksA, double* const* coresA,
                         const int64_t* ranksB, double* const* coresB, double* out, hipStream_t s) {
  if (N < 2 || N > TR_MAXN || !dims || !ranksA || !ranksB || !coresA || !coresB || !out) return TR_EINVAL;
  int64_t maxU = 1, maxE = 1, maxP = 1;
  int RA[TR_MAXN + 1], RB[TR_MAXN + 1];
  for (int k = 0; k < N; ++k) {
    if (dims[k] < 1 || ranksA[k] < 1 || ranksA[k] > TR_MAXR || ranksB[k] < 1 || ranksB[k] > TR_MAXR ||
        !coresA[k] || !coresB[k])
      return TR_EINVAL;
    RA[k] = (int)ranksA[k];
    RB[k] = (int)ranksB[k];
  }
  RA[N] = RA[0];
  RB[N] = RB[0];
  for (int k = 0; k < N; ++k) {
    maxU = std::max<int64_t>(maxU, dims[k] * std::max(RA[k] * RA[k + 1], RB[k] * RB[k + 1]));
    maxE = std::max<int64_t>(maxE, (int64_t)RA[k] * RA[k + 1] * RB[k] * RB[k + 1]);
    maxP = std::max<int64_t>(maxP, (int64_t)RA[0] * RB[0] * RA[k + 1] * RB[k + 1]);
  }
  const size_t bytes = (size_t)(2 * maxU + 2 * maxE + 2 * maxP + 8) * sizeof(double);
  char* ws = nullptr;
  if (hipMalloc((void**)&ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return TR_ENOMEM;
  }
  double* UA = (double*)ws;
  double* UB = UA + maxU;
  double* E = UB + maxU;
  double* T = E + maxE;
  double* P[2] = {T + maxE, T + maxE + maxP};
  double* res = P[1] + maxP;
  int rc = TR_OK;
  int cur = 0;
  const int64_t rows = (int64_t)RA[0] * RB[0];
  for (int k = 0; k < N && rc == TR_OK; ++k) {
    const int64_t I = dims[k];
    const int na = RA[k] * RA[k + 1], nb = RB[k] * RB[k + 1];
    const int64_t cols = (int64_t)RA[k + 1] * RB[k + 1];
    MatView At{UA, I, 2, 0, 0}, Bv{UB, I, 0, 0, 0};
    double* Tk = k == 0 ? P[0] : T;
    if (launch_core_unfold(coresA[k], RA[k], I, RA[k + 1], UA, s) != hipSuccess ||
        launch_core_unfold(coresB[k], RB[k], I, RB[k + 1], UB, s) != hipSuccess ||
        launch_gemm64(na, nb, I, 1.0, At, Bv, 0.0, nullptr, 0, E, na, s) != hipSuccess ||
        launch_transfer_from_cross_gram(E, RA[k], RA[k + 1], RB[k], RB[k + 1], Tk, s) != hipSuccess) {
      rc = TR_EHIP;
      break;
    }
    if (k > 0) {
      const int64_t inner = (int64_t)RA[k] * RB[k];
      MatView Pv{P[cur], rows, 0, 0, 0}, Tv{T, inner, 0, 0, 0};
      if (launch_gemm64(rows, cols, inner, 1.0, Pv, Tv, 0.0, nullptr, 0, P[cur ^ 1], rows, s) != hipSuccess) {
        rc = TR_EHIP;
        break;
      }
      cur ^= 1;
    }
  }
  double v = 0.0;
  if (rc == TR_OK && (launch_trace(P[cur], rows, res, s) != hipSuccess ||
                      hipMemcpyAsync(&v, res, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess))
    rc = TR_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess && rc == TR_OK) rc = TR_EHIP;
  (void)hipGetLastError();
  (void)hipFree(ws);
  if (rc == TR_OK) *out = v;
  return rc;
}

int tr_inner(int N, const int64_t* dims, const int64_t* ranksA, double* const* coresA, const int64_t* ranksB,
             double* const* coresB, double* inner, void* hip_stream) {
  return tr_inner_impl(N, dims, ranksA, coresA, ranksB, coresB, inner, (hipStream_t)hip_stream);
}

int tr_norm(int N, const int64_t* dims, const int64_t* ranks, double* const* cores, double* norm,
            void* hip_stream) {
  if (!norm) return TR_EINVAL;
  double v = 0.0;
  const int rc = tr_inner_impl(N, dims, ranks, cores, ranks, cores, &v, (hipStream_t)hip_stream);
  if (rc == TR_OK) *norm = std::sqrt(std::max(0.0, v));
  return rc;
}

// Allocation-free variant of the generator: its workspace lives in `scratch`,
// a device array of TR_GEN_SCRATCH_MAX bytes that every GPU the library runs
// on holds for the life of the process.  Host code never uses the array's
// name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept in scratch_dev.
static __device__ __align__(256) char scratch[TR_GEN_SCRATCH_MAX];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_dev[SCRATCH_DEVICES] = {nullptr};

int scratch_address(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return TR_EHIP;
  }
  if (dev < 0 || dev >= SCRATCH_DEVICES) return TR_EINVAL;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return TR_EHIP;
    }
    scratch_dev[dev] = static_cast<char*>(p);
  }
  *out = scratch_dev[dev];
  return TR_OK;
}
}  // namespace

int tr_gen_planted_noalloc(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X,
                           int x_dtype, double* const* true_cores, double* const* init_cores, void* hip_stream) {
  if (N < 2 || N > TR_MAXN || !dims || !ranks || !X) return TR_EINVAL;
  const size_t ws = trx_gen_workspace(N, dims, ranks, true_cores == nullptr);
  if (ws == 0) return TR_EINVAL;
  if (ws > TR_GEN_SCRATCH_MAX) return TR_ENOMEM;
  char* buf = nullptr;
  const int rc = scratch_address(&buf);
  if (rc) return rc;
  // every byte of the workspace the kernels read is written by them first
  // (cores, tables, per-block partial sums), so nothing needs clearing
  return trx_gen(N, dims, ranks, seed, eta, X, x_dtype, true_cores, init_cores, buf, ws,
                 (hipStream_t)hip_stream, nullptr);
}

}  // extern "C"

extern "C" {

static int update_mode(tr_als_ctx* c, int m, int prec, int refine, bool in_sweep) {
  // a rank-deficient V_n[2] breaks the Cholesky-QR before R_[2] exists: with
  // the pseudo-inverse solve the QR variant takes Alg. 4's route (the same
  // half-size problem, min ||Y_[n] - G V_n[2]^T||, through V_n[2]^T V_n[2])
  if (c->variant == TR_QR && c->solve != TR_SOLVE_PINV) return update_mode_qr(c, m, prec, in_sweep);
  if (c->variant == TR_QR || c->variant == TR_QRNE) return update_mode_qrne(c, m, prec, refine, in_sweep);
  return update_mode_ne(c, m, prec, refine, in_sweep);
}

// One sweep of mode updates captured into a HIP graph and replayed: the sweep
// issues ~20 small kernels per mode whose launch cost would otherwise show.
// Profiled runs launch eagerly.
static hipGraphExec_t sweep_graph(tr_als_ctx* c, int prec, int refine) {
  if (!c->graphs_ok || c->prof || c->variant != TR_NE) return nullptr;
  if (c->graphs[prec][refine]) return c->graphs[prec][refine];
  if (ensure_shadow(c, prec) != TR_OK) return nullptr;
  // The caller's stream may be the legacy default stream, which cannot be
  // captured: capture on a private stream instead (capturing runs nothing)
  // and launch the graph onto the caller's stream.
  hipError_t e = hipSuccess;
  if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->graphs_ok = false;
    c->graph_note = std::string("begin capture: ") + hipGetErrorString(e);
    return nullptr;
  }
  hipGraph_t g = nullptr;
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  int rc = TR_OK;
  for (int m = 0; m < c->N && rc == TR_OK; ++m) rc = update_mode(c, m, prec, refine, true);
  const std::string mode_err = c->err;
  c->stream = user;
  e = hipStreamEndCapture(c->cap_stream, &g);
  hipGraphExec_t ex = nullptr;
  if (rc == TR_OK && e == hipSuccess && g) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (rc != TR_OK || e != hipSuccess || !ex) {
    (void)hipGetLastError();
    c->graphs_ok = false;
    c->graph_note = rc != TR_OK ? "mode update under capture: " + mode_err
                                : std::string("end capture / instantiate: ") + hipGetErrorString(e);
    c->err.clear();
    return nullptr;
  }
  c->graphs[prec][refine] = ex;
  return ex;
}

static int enqueue_sweeps(tr_als_ctx* c, int nsweeps, int prec, int refine) {
  hipGraphExec_t ex = nsweeps > 0 ? sweep_graph(c, prec, refine) : nullptr;
  for (int sw = 0; sw < nsweeps; ++sw) {
    if (ex) {
      HIPCHK(c, hipGraphLaunch(ex, c->stream));
      continue;
    }
    for (int m = 0; m < c->N; ++m) {
      int rc = update_mode(c, m, prec, refine, true);
      if (rc) return rc;
    }
  }
  return TR_OK;
}

static int enqueue_fit(tr_als_ctx* c) {
  hipStream_t s = c->stream;
  const Plan& p = c->plan[0];
  int rc = build_table(c, p.f1c, p.Rmid, c->F1);
  if (rc) return rc;
  rc = build_table(c, p.f2c, p.Rmid, c->F2);
  if (rc) return rc;
  HIPCHK(c, launch_core_unfold(c->cores[0], p.Ra, p.I, p.Rb, c->G0u, s));
  HIPCHK(c, launch_fit(c->X, c->xdt, p.I, p.K, c->G0u, c->F1, c->F2, p.d1, p.m1, p.d2, p.m2, p.Rb, p.Rmid, p.Ra,
                       c->dpart, c->nred, c->dscal + 1, s));
  return TR_OK;
}

int tr_als_sweep(tr_als_ctx* c, int nsweeps, int prec, int refine) {
  if (!valid_ctx(c)) return TR_EINVAL;
  if (nsweeps < 0 || prec < TR_F64 || prec > TR_FP8 || refine < 0 || refine > 4)
    return fail(c, TR_EINVAL, "bad sweep arguments");
  c->err.clear();
  int rc = enqueue_sweeps(c, nsweeps, prec, refine);
  if (rc) return rc;
  rc = read_status(c);
  // cores written back in either case: on error they hold the last good update
  int rc2 = store_cores(c);
  if (rc2) return rc2;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return rc;
}

// The Sec. 4 error identities from the last mode's intermediates, after a
// sweep: dscal[4] = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2 (dscal[5], dscal[6] the
// two terms).
static int enqueue_cheap_fit(tr_als_ctx* c) {
  const int m = c->N - 1;
  const int n = c->R[m] * c->R[m + 1];
  if (2 * cheap_fit_blocks(c->dims[m]) > c->nred) return fail(c, TR_EINVAL, "internal: partial buffer too small");
  const bool qr = c->variant == TR_QR && c->solve != TR_SOLVE_PINV;
  HIPCHK(c, launch_cheap_fit(qr ? c->qW : c->M, c->Gn, qr ? c->qLt : c->S, qr ? 1 : 0, c->dims[m], n, c->dscal,
                             c->dpart, c->dscal + 4, c->stream));
  return TR_OK;
}

int tr_als_run(tr_als_ctx* c, int max_sweeps, int prec, int refine, double tol, int* sweeps_done,
               double* rel_err) {
  if (!valid_ctx(c)) return TR_EINVAL;
  if (max_sweeps < 1 || prec < TR_F64 || prec > TR_FP8 || refine < 0 || refine > 4 || !(tol >= 0.0) ||
      !sweeps_done || !rel_err)
    return fail(c, TR_EINVAL, "bad arguments");
  c->err.clear();
  *sweeps_done = 0;
  double prev = -1.0;
  int rc = TR_OK;
  for (int k = 1; k <= max_sweeps; ++k) {
    rc = enqueue_sweeps(c, 1, prec, refine);
    if (rc == TR_OK) rc = enqueue_cheap_fit(c);
    if (rc) break;
    double r2 = 0.0;
    HIPCHK(c, hipMemcpyAsync(&r2, c->dscal + 4, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    rc = read_status(c);   // synchronises: r2 is valid after it
    if (rc) break;
    *sweeps_done = k;
    const double f = c->xnorm2 > 0 ? std::sqrt(std::max(0.0, r2)) / std::sqrt(c->xnorm2) : 0.0;
    *rel_err = f;
    if (prev >= 0.0 && std::fabs(prev - f) <= tol) break;
    prev = f;
  }
  const int rc2 = store_cores(c);
  if (rc2) return rc2;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return rc;
}

int tr_als_set_solve(tr_als_ctx* c, int solve, double rcond) {
  if (!valid_ctx(c)) return TR_EINVAL;
  if ((solve != TR_SOLVE_FACTOR && solve != TR_SOLVE_PINV) || !(rcond >= 0.0) || rcond >= 1.0)
    return fail(c, TR_EINVAL, "bad solve arguments");
  for (int m = 0; m < c->N; ++m)
    if (solve == TR_SOLVE_PINV && !pinv_fits(c->R[m] * c->R[m + 1]))
      return fail(c, TR_EINVAL, "R_n R_{n+1} too large for the pseudo-inverse");
  c->solve = solve;
  c->rcond = rcond;
  // captured sweeps embed the solve: drop them
  for (auto& row : c->graphs)
    for (auto& g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TR_OK;
}

int tr_als_update_mode(tr_als_ctx* c, int n, int prec, int refine) {
  if (!valid_ctx(c) || n < 1 || n > c->N || prec < TR_F64 || prec > TR_FP8 || refine < 0 || refine > 4)
    return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  int rc = update_mode(c, n - 1, prec, refine, false);
  if (rc) return rc;
  return read_status(c);
}

int tr_als_store_cores(tr_als_ctx* c) {
  if (!valid_ctx(c)) return TR_EINVAL;
  int rc = store_cores(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TR_OK;
}

int tr_als_mttsp(tr_als_ctx* c, int n, int prec, double* Mout) {
  if (!valid_ctx(c) || n < 1 || n > c->N || prec < TR_F64 || prec > TR_FP8 || !Mout)
    return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  int rc = compute_mttsp(c, n - 1, prec, Mout);
  if (rc) return rc;
  return read_status(c);
}

int tr_als_coef(tr_als_ctx* c, int n, double* Sout) {
  if (!valid_ctx(c) || n < 1 || n > c->N || !Sout) return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  int rc = compute_coef(c, n - 1, Sout, c->stream);
  if (rc) return rc;
  return read_status(c);
}

int tr_als_gram(tr_als_ctx* c, int k, double* Eout) {
  if (!valid_ctx(c) || k < 1 || k > c->N || !Eout) return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  const int m = k - 1;
  const size_t n = (size_t)c->R[m] * c->R[m + 1];
  HIPCHK(c, hipMemcpyAsync(Eout, c->gram[m], n * n * 8, hipMemcpyDeviceToDevice, c->stream));
  return read_status(c);
}

int tr_als_mode_regime(const tr_als_ctx* c, int n) {
  if (!c || c->N < 2 || n < 1 || n > c->N) return TR_EINVAL;
  return c->plan[n - 1].slab ? 3 : c->plan[n - 1].regime;
}

int tr_als_xnorm2(const tr_als_ctx* c, double* out) {
  if (!c || !out) return TR_EINVAL;
  *out = c->xnorm2;
  return TR_OK;
}

int tr_als_fit(tr_als_ctx* c, double* rel_err) {
  if (!valid_ctx(c) || !rel_err) return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  hipStream_t s = c->stream;
  int rc = enqueue_fit(c);
  if (rc) return rc;
  double ss = 0.0;
  HIPCHK(c, hipMemcpyAsync(&ss, c->dscal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  *rel_err = c->xnorm2 > 0 ? std::sqrt(std::max(0.0, ss)) / std::sqrt(c->xnorm2) : 0.0;
  return read_status(c);
}

}  // extern "C"

int trx_run_async(tr_als_ctx* c, int nmixed, int prec_mixed, int nfin, int prec_fin, int refine, int* status_host,
                  double* scal_host) {
  if (!valid_ctx(c)) return TR_EINVAL;
  int rc = enqueue_sweeps(c, nmixed, prec_mixed, refine);
  if (rc == TR_OK) rc = enqueue_sweeps(c, nfin, prec_fin, refine);
  if (rc == TR_OK) rc = store_cores(c);
  if (rc == TR_OK) rc = enqueue_fit(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(status_host, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(scal_host, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return TR_OK;
}

const char* trx_status_text(int st) {
  if (st & ST_SINGULAR) return "coefficient matrix not positive definite (or zero pivot)";
  if (st & ST_NONFINITE) return "non-finite value in M_n or in an updated core";
  return "";
}

extern "C" {

int tr_als_debug_overruns(void) { return g_overruns.load(); }

int tr_als_debug_graphs(const tr_als_ctx* c, char* note, int note_len) {
  if (!valid_ctx(c)) return TR_EINVAL;
  if (note && note_len > 0) {
    const size_t k = std::min((size_t)(note_len - 1), c->graph_note.size());
    std::memcpy(note, c->graph_note.data(), k);
    note[k] = 0;
  }
  int count = 0;
  for (const auto& row : c->graphs)
    for (hipGraphExec_t ex : row) count += ex != nullptr;
  return count;
}

int tr_als_debug_shadow(tr_als_ctx* c, int prec, int transposed, void* out, float* scale, int64_t* split_k) {
  if (!valid_ctx(c) || !out || !scale || (prec != TR_BF16 && prec != TR_FP8))
    return c ? fail(c, TR_EINVAL, "bad arguments") : TR_EINVAL;
  int rc = ensure_shadow(c, prec);
  if (rc) return rc;
  const void* src = prec == TR_BF16 ? (transposed ? c->xbf16t : c->xbf16) : (transposed ? c->xfp8t : c->xfp8);
  if (!src) return fail(c, TR_EINVAL, "the context keeps no such shadow");
  HIPCHK(c, hipMemcpyAsync(out, src, (size_t)c->numel * (prec == TR_BF16 ? 2 : 1), hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *scale = prec == TR_FP8 ? c->fp8_scale : 1.0f;
  if (split_k) *split_k = transposed ? c->t_gK : 0;
  return TR_OK;
}

int tr_als_profile_enable(tr_als_ctx* c, int enable) {
  if (!valid_ctx(c)) return TR_EINVAL;
  c->prof = enable != 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  return TR_OK;
}

int tr_als_profile_read(tr_als_ctx* c, double* ms, int64_t* launches, double* bytes_per_launch) {
  if (!valid_ctx(c) || !ms || !launches || !bytes_per_launch) return TR_EINVAL;
  *ms = c->prof_ms;
  *launches = c->prof_launches;
  *bytes_per_launch = c->prof_bytes;
  return TR_OK;
}

}  // extern "C"
