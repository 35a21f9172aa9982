// FP64 normal-equation solve G S = M with S = L L^T (Alg. 2's solve step):
// a blocked Cholesky in one workgroup (matrix in LDS) and a blocked
// forward/backward substitution that runs 16 right-hand sides per workgroup
// with L staged in LDS.  A non-positive or non-finite pivot latches
// ST_SINGULAR; later steps see the status word and leave their outputs alone.
#include "common.h"
#include "../../include/tr_als.h"

namespace {

#ifndef TR_SOLVE_NB
#define TR_SOLVE_NB 8
#endif
constexpr int NB = TR_SOLVE_NB;   // block size of the blocked algorithms
constexpr int NRHS = 16;    // right-hand sides per workgroup

// Value of v held by lane src (uniform src), as a wave-wide broadcast.
__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Right-looking blocked Cholesky.  The matrix is padded in LDS to np (a
// multiple of 16) with an identity block, so every block has 16 columns and
// the inner loops have fixed trip counts: blockdiag(S, I) = blockdiag(L, I) L^T.
__global__ __launch_bounds__(256) void chol_lds_kernel(const double* S, int n, double* L, double* LT, int* status,
                                                       double* rdg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);
  __shared__ int bad;
  __shared__ double rdiag[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = (n + NB - 1) / NB * NB;
  if (tid == 0) bad = (*status != 0);
  for (int e = tid; e < np * np; e += 256) {
    const int i = e % np, j = e / np;
    A[e] = (i < n && j < n) ? S[i + n * j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (bad) return;
  for (int J = 0; J < np; J += NB) {
    if (wave == 0) {
      // diagonal block: lane i < 16 holds row J+i in registers; pivots and
      // column entries are broadcast with readlane (no LDS round trips)
      double a[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) a[j] = (lane < NB && j <= lane) ? A[(J + lane) + np * (J + j)] : 0.0;
      bool okall = true;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const double d = bcast(a[k], k);
        const bool ok = (d > 0.0) && isfinite(d);
        okall = okall && ok;
        const double piv = ok ? sqrt(d) : 1.0;
        const double rp = 1.0 / piv;
        if (lane == k) { a[k] = piv; rdiag[J + k] = rp; }
        if (lane > k) a[k] *= rp;
#pragma unroll
        for (int j = k + 1; j < NB; ++j) {
          const double ljk = bcast(a[k], j);
          if (lane >= j) a[j] -= a[k] * ljk;
        }
      }
      if (!okall && lane == 0) bad = 1;
      if (lane < NB) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j <= lane) A[(J + lane) + np * (J + j)] = a[j];
      }
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) atomicOr(status, ST_SINGULAR);
      return;
    }
    // panel: rows below the block, X L_JJ^T = A_panel
    const int m = np - J - NB;
    if (tid < m) {
      const int i = J + NB + tid;
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = A[i + np * (J + c)];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double v = x[c];
#pragma unroll
        for (int t = 0; t < c; ++t) v -= x[t] * A[(J + c) + np * (J + t)];
        x[c] = v * rdiag[J + c];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) A[i + np * (J + c)] = x[c];
    }
    __syncthreads();
    // trailing update of the lower triangle in 4x4 register tiles
    const int mt = m / 4;
    const int ntiles = mt * (mt + 1) / 2;
    for (int t = tid; t < ntiles; t += 256) {
      int ti = 0, acc0 = 0;
      while (acc0 + ti + 1 <= t) { acc0 += ti + 1; ++ti; }
      const int tj = t - acc0;   // 0..ti
      const int i0 = J + NB + 4 * ti, j0 = J + NB + 4 * tj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double pi[4], pj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          pi[a] = A[(i0 + a) + np * (J + c)];
          pj[a] = A[(j0 + a) + np * (J + c)];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += pi[a] * pj[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (j0 + b <= i0 + a) A[(i0 + a) + np * (j0 + b)] -= acc[a][b];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += 256) {
    const int i = e % n, j = e / n;
    const double v = (i >= j) ? A[i + np * j] : 0.0;
    L[e] = v;
    LT[j + n * i] = v;
  }
  for (int e = tid; e < np; e += 256) rdg[e] = rdiag[e];
}

// G[r, :] (+)= solution g of g S = rhs[r, :] for 16 rows r per workgroup
// (Rhs == nullptr stands for the n x n identity, giving G = S^{-1}):
// forward L z^T = rhs^T, then backward L^T g^T = z^T, both blocked by 16 on
// an identity-padded copy of L (fixed trip counts in every inner loop).
__global__ __launch_bounds__(256) void trsm_rhs_kernel(const double* Lg, const double* rdg, int n, const double* Rhs,
                                                       int64_t I, double* G, int accumulate, const int* status,
                                                       int mode) {
  // mode 0: g S = rhs with S = L L^T; 1: g L^T = rhs (forward only);
  // 2: g L = rhs (backward only).  rdg == nullptr: reciprocals taken from L.
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double rd[256];
  if (*status != 0) return;
  const int np = (n + NB - 1) / NB * NB;
  for (int e = threadIdx.x; e < np; e += 256) rd[e] = rdg ? rdg[e] : (e < n ? 1.0 / Lg[e + (int64_t)n * e] : 1.0);
  double* Ls = reinterpret_cast<double*>(smem_raw);   // np x np column-major
  double* B = Ls + (size_t)np * np;                   // NRHS x np, row r at B[r + NRHS*j]
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * NRHS;
  for (int e = tid; e < np * np; e += 256) {
    const int i = e % np, j = e / np;
    Ls[e] = (i < n && j < n) ? Lg[i + n * j] : (i == j ? 1.0 : 0.0);
  }
  for (int e = tid; e < NRHS * np; e += 256) {
    const int r = e % NRHS, j = e / NRHS;
    double v = 0.0;
    if (r0 + r < I && j < n) v = Rhs ? Rhs[(r0 + r) + I * j] : (r0 + r == j ? 1.0 : 0.0);
    B[e] = v;
  }
  __syncthreads();
  // forward: z_j = (b_j - sum_{t<j} L[j,t] z_t) / L[j,j]
  for (int J = 0; J < np && mode != 2; J += NB) {
    if (tid < NRHS) {
      const int r = tid;
      double z[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) z[c] = B[r + NRHS * (J + c)];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double v = z[c];
#pragma unroll
        for (int t = 0; t < c; ++t) v -= Ls[(J + c) + np * (J + t)] * z[t];
        z[c] = v * rd[J + c];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) B[r + NRHS * (J + c)] = z[c];
    }
    __syncthreads();
    for (int e = tid; e < NRHS * (np - J - NB); e += 256) {
      const int r = e % NRHS, j = J + NB + e / NRHS;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) v += Ls[j + np * (J + c)] * B[r + NRHS * (J + c)];
      B[r + NRHS * j] -= v;
    }
    __syncthreads();
  }
  // backward: g_j = (z_j - sum_{t>j} L[t,j] g_t) / L[j,j]
  for (int J = np - NB; J >= 0 && mode != 1; J -= NB) {
    if (tid < NRHS) {
      const int r = tid;
      double g[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) g[c] = B[r + NRHS * (J + c)];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        const int c = NB - 1 - cc;
        double v = g[c];
#pragma unroll
        for (int t = c + 1; t < NB; ++t) v -= Ls[(J + t) + np * (J + c)] * g[t];
        g[c] = v * rd[J + c];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) B[r + NRHS * (J + c)] = g[c];
    }
    __syncthreads();
    for (int e = tid; e < NRHS * J; e += 256) {
      const int r = e % NRHS, j = e / NRHS;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) v += Ls[(J + c) + np * j] * B[r + NRHS * (J + c)];
      B[r + NRHS * j] -= v;
    }
    __syncthreads();
  }
  for (int e = tid; e < NRHS * n; e += 256) {
    const int r = e % NRHS, j = e / NRHS;
    if (r0 + r < I) {
      if (accumulate) G[(r0 + r) + I * j] += B[e];
      else G[(r0 + r) + I * j] = B[e];
    }
  }
}

// Reciprocal of a positive FP64 pivot: hardware estimate plus two Newton steps
// (within an ulp or two of 1/d; the solve that uses the inverse is refined).
__device__ __forceinline__ double pivot_recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// S^{-1} of a symmetric positive definite S (n <= 16 * NBT) by the symmetric
// sweep operator: sweeping pivot k of A sets
//   A_ij -= A_ik A_kj / A_kk  (i, j != k),  A_ik = A_ki = A_ik / A_kk,  A_kk = -1 / A_kk,
// and sweeping every pivot of S leaves -S^{-1}.  For SPD S every pivot is a
// Schur-complement diagonal, hence positive; a pivot that is not (S not
// positive definite in working precision) latches ST_SINGULAR.
//
// One workgroup of 16 x 16 threads holds the matrix in registers: thread
// (ti, tj) owns A(16r + ti, 16c + tj) for the lower block triangle c <= r
// (the upper halves of the diagonal blocks are scratch, never read).  Per
// pivot the current column k is exchanged through a double-buffered LDS
// vector, so each pivot costs one barrier.
template <int NBT>
__global__ __launch_bounds__(256) void spd_sweep_inv_kernel(const double* __restrict__ S, int n,
                                                            double* __restrict__ Sinv, int* status) {
  __shared__ double col[2][16 * NBT];
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  if (*status != 0) return;
  double a[NBT][NBT];
#pragma unroll
  for (int r = 0; r < NBT; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      const int i = 16 * r + ti, j = 16 * c + tj;
      a[r][c] = (i < n && j < n) ? S[i + (int64_t)n * j] : (i == j ? 1.0 : 0.0);
    }
  // column 0 (canonical entries (i, 0), i >= 0, owned by tj == 0)
  if (tj == 0) {
#pragma unroll
    for (int r = 0; r < NBT; ++r) col[0][16 * r + ti] = a[r][0];
  }
  int buf = 0;
#pragma unroll
  for (int rk = 0; rk < NBT; ++rk) {
    const int tend = min(16, n - 16 * rk);
    for (int tk = 0; tk < tend; ++tk) {
      const int k = 16 * rk + tk;
      __syncthreads();
      const double* cb = col[buf];
      const double d = cb[k];
      if (!(d > 0.0) || !isfinite(d)) {   // same value in every thread: uniform exit
        if (tid == 0) atomicOr(status, ST_SINGULAR);
        return;
      }
      const double p = pivot_recip(d);
      double x[NBT], v[NBT];
#pragma unroll
      for (int r = 0; r < NBT; ++r) {
        x[r] = cb[16 * r + ti];
        v[r] = cb[16 * r + tj] * p;
      }
#pragma unroll
      for (int r = 0; r < NBT; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) a[r][c] = fma(-x[r], v[c], a[r][c]);
      // column k, rows i >= k: A_ik / A_kk, and -1 / A_kk on the diagonal
      if (tj == tk) {
#pragma unroll
        for (int r = rk; r < NBT; ++r) a[r][rk] = (16 * r + ti == k) ? -p : x[r] * p;
      }
      // row k, columns j < k: A_jk / A_kk
      if (ti == tk) {
#pragma unroll
        for (int c = 0; c <= rk; ++c)
          if (16 * c + tj < k) a[rk][c] = v[c];
      }
      // publish column k + 1 into the other buffer: entries (i, k+1) with
      // i >= k+1 from its column owners, (k+1, j) with j < k+1 from its row owners
      const int k1 = k + 1;
      double* cn = col[buf ^ 1];
      if (k1 < n) {
        if (tk + 1 < 16) {
          const int t1 = tk + 1;
          if (tj == t1) {
#pragma unroll
            for (int r = rk; r < NBT; ++r)
              if (16 * r + ti >= k1) cn[16 * r + ti] = a[r][rk];
          }
          if (ti == t1) {
#pragma unroll
            for (int c = 0; c <= rk; ++c)
              if (16 * c + tj < k1) cn[16 * c + tj] = a[rk][c];
          }
        } else if (rk + 1 < NBT) {
          if (tj == 0) {
#pragma unroll
            for (int r = rk + 1; r < NBT; ++r) cn[16 * r + ti] = a[r][rk + 1];
          }
          if (ti == 0) {
#pragma unroll
            for (int c = 0; c <= rk; ++c) cn[16 * c + tj] = a[rk + 1][c];
          }
        }
      }
      buf ^= 1;
    }
  }
  // -A = S^{-1}: write both triangles from the canonical entries
#pragma unroll
  for (int r = 0; r < NBT; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      const int i = 16 * r + ti, j = 16 * c + tj;
      if (i < n && j <= i) {
        const double v = -a[r][c];
        Sinv[i + (int64_t)n * j] = v;
        Sinv[j + (int64_t)n * i] = v;
      }
    }
}

}  // namespace

// LDS-resident versions for n <= 128; larger systems use the global-memory
// Cholesky and the one-wave-per-row solve.
bool solve_in_lds(int n) { return n <= 128; }

hipError_t launch_chol_lds(const double* S, int n, double* L, double* LT, double* rdiag, int* status, hipStream_t s) {
  const int np = (n + NB - 1) / NB * NB;
  const size_t lds = (size_t)np * np * sizeof(double);
  if (lds > 64 * 1024) hipFuncSetAttribute((const void*)chol_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(chol_lds_kernel, dim3(1), dim3(256), lds, s, S, n, L, LT, status, rdiag);
  return hipGetLastError();
}

hipError_t launch_trsm_rhs(const double* L, const double* rdiag, int n, const double* Rhs, int64_t I, double* G,
                           int accumulate, const int* status, hipStream_t s, int mode) {
  const int np = (n + NB - 1) / NB * NB;
  const size_t lds = ((size_t)np * np + (size_t)NRHS * np) * sizeof(double);
  if (lds > 64 * 1024) hipFuncSetAttribute((const void*)trsm_rhs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(trsm_rhs_kernel, dim3((unsigned)((I + NRHS - 1) / NRHS)), dim3(256), lds, s, L, rdiag, n, Rhs,
                     I, G, accumulate, status, mode);
  return hipGetLastError();
}

bool spd_inverse_fits(int n) { return n >= 1 && n <= 128; }

hipError_t launch_spd_inverse(const double* S, int n, double* Sinv, int* status, hipStream_t s) {
  const int nbt = (n + 15) / 16;
  switch (nbt) {
#define SPD_INV_CASE(B) \
  case B: hipLaunchKernelGGL(spd_sweep_inv_kernel<B>, dim3(1), dim3(256), 0, s, S, n, Sinv, status); break;
    SPD_INV_CASE(1) SPD_INV_CASE(2) SPD_INV_CASE(3) SPD_INV_CASE(4)
    SPD_INV_CASE(5) SPD_INV_CASE(6) SPD_INV_CASE(7) SPD_INV_CASE(8)
#undef SPD_INV_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
