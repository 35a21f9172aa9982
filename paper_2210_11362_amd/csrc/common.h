// Shared declarations of the gfx950 TR-ALS library (device helpers, launch
// wrappers, status flags).  Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TR_MAXN 8
#define TR_MAXR 24

// Bits latched into the device status word.
enum { ST_SINGULAR = 1, ST_NONFINITE = 2 };

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One byte of OCP FP8 E4M3.
struct fp8e4m3 { uint8_t v; };

// Arguments of the X-streaming contraction (the MTTSP).  The data tensor is
// seen as a matrix A[i, k] (i = mode-n index, k = the other indices) and the
// subchain row for k is formed as F1[f1(k)] * F2[f2(k)].
struct XsArgs {
  const void* X;
  int64_t I;          // rows (I_n)
  int64_t K;          // contraction length (prod_{j != n} I_j)
  int64_t L;          // extent of the fast group (layout 1)
  int layout;         // 0: A[i,k] at i + I*k;  1: at (k%L) + L*i + L*I*(k/L)
  const double* F1;   // K1 entries, each Rb x Rmid, column-major (b fastest)
  const double* F2;   // K2 entries, each Rmid x Ra, column-major (m fastest)
  int64_t d1, m1, d2, m2;   // f1(k) = (k/d1) % m1, f2(k) = (k/d2) % m2
  int Rb, Rmid, Ra;   // R_{n+1}, bond, R_n
  int MT, NT;         // output tile rows / columns (multiples of 16)
  int NTb;            // b-values per column tile (NT >= Ra*NTb)
  int n_mt, n_nt;     // number of tiles along rows / columns
  int64_t k_per_split;
  int nsplit;
  int wgm, wgn;       // 2-D arrangement of the 4 waves over the tile
  const double* tmax; // FP8: device max|F1|, max|F2| (the table scale is derived from them in the kernel)
  void* partial;      // [nsplit][n_mt*n_nt][MT][NT] FP32 (FP64 for the FP64 path)
};

// Arguments of the two-stage MTTSP's stage 1: Y[r, c] = sum_k A[r, k] B[k, c]
// with A = X as a matrix (nn: A[r,k] = X[r + M*k]; else A[r,k] = X[k + K*r])
// and B stored transposed (Bt[c*ldb + k], zero-padded to n_nt*NT rows).
struct XgArgs {
  const void* X;
  int64_t M, K;
  int C;              // columns of Y (bond pairs)
  int nn;             // 1: group = slowest modes; 0: group = fastest modes
  int vec_ok;         // contiguous runs of A (rows, or columns when nn) start 16-byte aligned
  int MT, NT, n_mt, n_nt;
  const void* Bt;
  int64_t ldb;
  int64_t k_per_split;
  int nsplit;
  int xcd_map;        // 1: 1-D grid, workgroups on one XCD share k-splits (nsplit % 8 == 0)
  const double* tmax; // FP8: device max|T| of the operand table (its scale is derived from it)
  void* partial;      // [nsplit][n_mt*n_nt][MT][NT] FP32 (FP64 for the FP64 path)
};

// FP8 operand tables are stored as two E4M3 parts at one power-of-two scale s
// (hi = fp8(T s), lo = fp8(T s - hi)), both contracted into the same FP32
// accumulator: 3 fraction bits per part, about 7 together.  s = 2^floor(log2(448 / bound))
// for a bound on |T| (1 when the bound is 0); the same expression on both
// sides of the contraction.
__device__ __forceinline__ double fp8_table_scale(double bound) {
  if (!(bound > 0.0)) return 1.0;
  int e = 0;
  (void)frexp(448.0 / bound, &e);   // 448 / bound = m 2^e, m in [0.5, 1)
  return ldexp(1.0, e - 1);
}

// Arguments of the slab contraction of an order-3 tensor (k_slab.hip): rows i
// of the output mode, the contracted mode k (against a table of its core) and
// the slab mode l (its core absorbed per slab).
struct XslabArgs {
  const void* X;
  int64_t In, Ik, Il;     // extents of the output, contracted and slab modes
  int64_t sn, sk, sl;     // their strides in X (elements); sn == 1 or sk == 1
  int caseB;              // 0: table G_c1[b, k, m], absorb G_c2[m, l, a]; 1: table G_c2[m, k, a], absorb G_c1[b, l, m]
  const double* Gl;       // the absorbed core (FP64)
  int Rm, Ro, Rg, Rn;     // middle rank, other rank of the absorbed core, range of the group index, R_n
  int NG, TWg, OWg;       // group size, table columns per group (multiple of 16), outputs per group
  int n_mt, n_g;
  int64_t ldb;            // k-stride of the table (Ik rounded up to the k tile)
  const void* Bt;         // table, transposed, operand type: [g TWg + m + Rm u][k]
  int64_t l_per_split;
  int nsplit;
  void* partial;          // [nsplit][n_mt n_g][128][OWg] FP32 (FP64 on the FP64 path)
};
int xslab_kt(int prec);
size_t xslab_lds_bytes(const XslabArgs& a, int prec);
int xslab_group(int Rm, int Ro);
int xslab_rows();
hipError_t launch_xslab_table(const XslabArgs& a, const double* Gk, int prec, void* Bt, hipStream_t s);
hipError_t launch_xslab(const XslabArgs& a, int prec, int xdt, size_t lds, hipStream_t s);
hipError_t launch_xslab_reduce(const XslabArgs& a, int prec, double out_scale, double* M, int* status,
                               hipStream_t s);

// Host-side launchers (defined in the .hip files).
int xgemm_kt(int prec);
hipError_t launch_xgemm(const XgArgs& g, int prec, int xdt, hipStream_t s);
hipError_t launch_xg_reduce(const XgArgs& g, int prec, double out_scale, double* Y, int* status, hipStream_t s);
// Operand table (transposed, zero-padded, in the operand type; not FP8) of a
// group of one or two cores, formed directly from the cores.
hipError_t launch_group_bt(const double* G0, int Rl, int64_t I0, int Rm, const double* G1, int64_t I1, int two,
                           int64_t K, int C, int Crows, int64_t ldb, int prec, void* Bt, hipStream_t s);
hipError_t launch_table_to_bt(const double* T, int64_t K, int C, int Crows, int64_t ldb, int prec, double scale,
                              void* Bt, hipStream_t s,
                              const double* tmax = nullptr);
hipError_t launch_absorb(const double* Y, int64_t lo, int64_t I, int64_t hi, int Ru, int Rc, const double* core,
                         int Rl, int Rr, int side, int final_out, double* out, double* part, size_t part_bytes,
                         hipStream_t s);
hipError_t launch_bond_to_M(const double* Y, int64_t In, int Ru, int Rc, double* M, hipStream_t s);
hipError_t launch_xstream(const XsArgs& a, int prec, int xdt, int kt, int wlay, size_t lds, hipStream_t s);
size_t xstream_lds_bytes(const XsArgs& a, int prec, int kt);
hipError_t launch_xs_reduce(const XsArgs& a, int prec, double out_scale, double* M, int* status, hipStream_t s);

hipError_t launch_core_to_table(const double* core, int Rl, int64_t I, int Rr, double* out, hipStream_t s);
hipError_t launch_chain_step(const double* T, int64_t J, int Rl, int Rm, const double* core, int64_t I, int Rr,
                             double* out, hipStream_t s);
hipError_t launch_identity_table(int R, double* out, hipStream_t s);
hipError_t launch_core_unfold(const double* core, int Ra, int64_t I, int Rb, double* out, hipStream_t s);
hipError_t launch_gram(const double* core, int Rl, int64_t I, int Rr, double* E, hipStream_t s);

// Generic FP64 operand view for the small GEMMs: plain column-major matrix
// (kind 0), its transpose (kind 2), or a Gram E (RlRr x RlRr) read in Kronecker
// order (kind 1):
//   K[(b + Rl*b'), (c + Rr*c')] = E[(b + Rl*c) + RlRr*(b' + Rl*c')].
struct MatView { const double* p; int64_t ld; int kind; int Rl, Rr; };
hipError_t launch_gemm64(int64_t M, int64_t N, int64_t K, double alpha, MatView A, MatView B, double beta,
                         const double* Cin, int64_t ldcin, double* C, int64_t ldc, hipStream_t s,
                         int* finite_status = nullptr);
hipError_t launch_realign_S(MatView W, int Ra, int Rb, double* S, hipStream_t s);
// The last ring GEMM W = A B (Rb^2 x Ra^2, inner K) stored straight into S_n<2>
// with launch_realign_S's map.
hipError_t launch_gemm64_realign(int64_t K, MatView A, MatView B, int Ra, int Rb, double* S, hipStream_t s);
// One FP64 product C = alpha A B + beta Cin (M x N, inner K); Ra > 0 stores it
// realigned as S_n<2> (Ra = R_n, Rb = R_{n+1}, M = Rb^2, N = Ra^2).
struct Gemm64Desc {
  int64_t M, N, K;
  double alpha;
  MatView A, B;
  double beta;
  const double* Cin;
  int64_t ldcin;
  double* C;
  int64_t ldc;
  int Ra, Rb;
};
inline int64_t gemm64_blocks(const Gemm64Desc& g) { return ((g.M + 15) / 16) * ((g.N + 15) / 16); }
Gemm64Desc gemm64_realign_desc(int64_t K, MatView A, MatView B, int Ra, int Rb, double* S);
// Two independent products in one launch.
hipError_t launch_gemm64_pair(const Gemm64Desc& g0, const Gemm64Desc& g1, hipStream_t s);
hipError_t launch_chol(const double* S, int n, double* L, double* LT, double* work, int* status, hipStream_t s);
bool solve_in_lds(int n);
// S^{-1} of an SPD matrix with n <= 128 by the symmetric sweep operator (one
// workgroup, registers); a non-positive pivot latches ST_SINGULAR.
bool spd_inverse_fits(int n);
// Raises kernel k's dynamic-LDS limit when it needs more than the default 64 KB.
inline hipError_t allow_lds(const void* k, size_t lds) {
  return lds > 64 * 1024 ? hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) : hipSuccess;
}
#define LDSCHK(k, lds)                                   \
  do {                                                   \
    const hipError_t lds_e_ = allow_lds((k), (lds));     \
    if (lds_e_ != hipSuccess) return lds_e_;             \
  } while (0)
// dst[r + ld_dst c] = src[r + ld_src c] for a rows x cols block (trans = 1:
// src[c + ld_src r]; src == nullptr: zeros; add: dst += the value)
hipError_t launch_copy_block(const double* src, int64_t ld_src, int rows, int cols, double* dst, int64_t ld_dst,
                             hipStream_t s, int trans = 0, bool add = false);
hipError_t launch_spd_inverse(const double* S, int n, double* Sinv, int* status, hipStream_t s);
hipError_t launch_chol_lds(const double* S, int n, double* L, double* LT, double* rdiag, int* status, hipStream_t s);
hipError_t launch_trsm_rhs(const double* L, const double* rdiag, int n, const double* Rhs, int64_t I, double* G,
                           int accumulate, const int* status, hipStream_t s, int mode = 0);
// QR variant
hipError_t launch_householder_qr(double* A, int64_t m, int n, double* V, double* tau, double* Q, double* R,
                                 hipStream_t s);
// Whether launch_householder_qr factors an m x n matrix in one workgroup's
// registers (m <= 256, n <= 128, the reflectors within 128 KB of LDS).
bool householder_in_registers(int64_t m, int n);
// out[e] = (double)x[e], e < n.
hipError_t launch_widen_f32(const float* x, int64_t n, double* out, hipStream_t s);
// C[e] = sum over the nchunk partials part[c * n + e] (fixed summation order).
// C[e] = sum over the nchunk partials part[c * n + e] (fixed summation order).
hipError_t launch_sum_chunks(const double* part, int nchunk, int64_t n, double* C, hipStream_t s);
// out[i + I*(l + L*t)] = in[l + L*(i + I*t)] (each L x I slice transposed).
hipError_t launch_slice_transpose(const double* in, int64_t L, int64_t I, int64_t T, double* out, hipStream_t s);
hipError_t launch_sum_chunks(const double* part, int nchunk, int64_t n, double* C, hipStream_t s);
hipError_t launch_tall_atb(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t K, int P, int Q,
                           int mode, int64_t L, int64_t Ip, int64_t T, double* part, int64_t part_elems, double* C,
                           hipStream_t s);
hipError_t launch_ttm(const void* in, int in_type, int64_t L, int64_t I, int64_t T, const double* Q, int R,
                      double scale, double* out, hipStream_t s);
hipError_t launch_transpose(const double* A, int64_t rows, int64_t cols, double* At, hipStream_t s);
// C = A B for a tall column-major A (M x K) and a small B (K x N), K, N <= 112;
// b_upper: B is upper triangular (its zero blocks below the diagonal are skipped).
hipError_t launch_tall_gemm(const double* A, int64_t lda, int64_t M, int K, const double* B, int ldb, int N,
                            double* C, int64_t ldc, hipStream_t s, bool b_upper = false);
hipError_t launch_table_to_v2(const double* T, int64_t J, int64_t L, int Ra, int Rb, double* V2, hipStream_t s);
// V2[k' + J*(a + Ra*b)] = sum_m Tp[j][b + Rb*m] core[m + Rm*(i + I*a)] with
// j + Jp*i the subchain row of Multi-TTM row k' (J = Jp*I, L rows before n).
hipError_t launch_v2_direct(const double* Tp, int64_t Jp, const double* core, int64_t I, int Rm, int Ra, int Rb,
                            int64_t L, double* V2, hipStream_t s);
inline bool v2_direct_fits(int Rm, int Ra, int Rb) { return ((Rb * Rm + Rm * Ra) | 1) * 8 <= 64 * 1024; }
hipError_t launch_shift_and_add(double* G, int n, int64_t m, double* sbuf, hipStream_t s);
hipError_t launch_core_fold(const double* G2, int64_t I, int Ra, int Rb, double* core, hipStream_t s);
hipError_t launch_chol_inv(const double* S, int n, double* L, double* LT, double* LinvT, double* work, int* status,
                           hipStream_t s);
hipError_t launch_chol_solve(const double* L, const double* LT, int n, const double* Rhs, int64_t I,
                             double* G, int accumulate, const int* status, hipStream_t s);
// Normal-equation apply: G = M S^{-1} plus `refine` refinement steps
// (R = M - G S, G += R S^{-1}), 8 rows of M per workgroup; a non-finite G
// latches ST_NONFINITE.  Skipped when the status word is set.
hipError_t launch_ne_apply(const double* M, int64_t I, int n, const double* S, const double* Sinv, int refine,
                           double* G, int* status, hipStream_t s);
// Commit G into the core layout (status word clear) and write the core's Gram.
hipError_t launch_commit_gram(const double* G, int64_t I, int Ra, int Rb, double* core, double* E, int* status,
                              hipStream_t s);
hipError_t launch_commit_core(const double* G, int64_t I, int Ra, int Rb, double* core, int* status, hipStream_t s,
                              bool checked = false);
hipError_t launch_sumsq(const void* X, int xdt, int64_t n, double* partials, int nblk, double* out, hipStream_t s);
hipError_t launch_absmax(const void* X, int xdt, int64_t n, float* partials, int nblk, float* out, hipStream_t s);
hipError_t launch_to_bf16(const void* X, int xdt, int64_t n, void* out, hipStream_t s);
// Transposed low-precision shadow (BF16, or FP8 with the scale of absmax) of
// X seen as an M x K matrix: out[k + K*r] = X[r + M*k].
hipError_t launch_to_lowp_t(const void* X, int xdt, int64_t M, int64_t K, const float* absmax, int prec, void* out,
                            hipStream_t s);
hipError_t launch_to_fp8(const void* X, int xdt, int64_t n, const float* absmax, float* scale_out, void* out,
                         hipStream_t s);
hipError_t launch_fit(const void* X, int xdt, int64_t I, int64_t K, const double* G0, const double* F1,
                      const double* F2, int64_t d1, int64_t m1, int64_t d2, int64_t m2, int Rb, int Rmid, int Ra,
                      double* partials, int nblk, double* out, hipStream_t s);
hipError_t launch_table_absmax(const double* T, int64_t n, double* out, hipStream_t s);
// pseudo-inverse of a square FP64 matrix by the one-sided Jacobi SVD (one
// workgroup); singular values <= rcond * max count as zero; work: 2 n^2 doubles
bool pinv_fits(int n);
hipError_t launch_pinv(const double* A, int n, double rcond, double* Apinv, double* work, int* status,
                       hipStream_t s);
// cheap in-loop error (Sec. 4): rows of A (M_N or W_N) and G = G_N(2) (I x n);
// mode 0: B = S_N (n x n), mode 1: B = R_[2]^T (lower); out[0] = ||X||^2 - 2a + b,
// out[1] = a = <X, Xhat>, out[2] = b = ||Xhat||^2.  partials: 2 * cheap_fit_blocks(I)
int cheap_fit_blocks(int64_t I);
hipError_t launch_cheap_fit(const double* A, const double* G, const double* B, int mode, int64_t I, int n,
                            const double* xnorm2, double* partials, double* out, hipStream_t s);
// TR inner product (Sec. 3.4): cross Gram E (RaRb x SaSb) -> transfer matrix
// T ((Ra Sa) x (Rb Sb)), and the trace of a square n x n matrix
hipError_t launch_transfer_from_cross_gram(const double* E, int Ra, int Rb, int Sa, int Sb, double* T,
                                           hipStream_t s);
hipError_t launch_trace(const double* P, int64_t n, double* out, hipStream_t s);
// planted-tensor generator (serving)
hipError_t launch_philox_normal(double* out, int64_t n, uint64_t seed, uint32_t sid, hipStream_t s);
hipError_t launch_gen_planted(void* X, int xdt, int64_t I, int64_t K, const double* G0, const double* F1,
                              const double* F2, int64_t d1, int64_t m1, int64_t d2, int64_t m2, int Rb, int Rmid,
                              int Ra, uint64_t seed, double eta, double* partials, int nblk, double* scal,
                              hipStream_t s);
// Philox stream ids of the generator's normal numbers
enum { GEN_SID_NOISE = 0, GEN_SID_TRUE = 0x100, GEN_SID_INIT = 0x200 };
