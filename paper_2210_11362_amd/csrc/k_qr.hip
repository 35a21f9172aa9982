// Kernels of the QR-stabilised update (Alg. 3), all FP64 except the first TTM,
// which reads X in the contraction precision:
//   - Householder QR of a core's mode-2 unfolding (Definition of the mode-n QR):
//     explicit Q (I x r) and R (r x RR), r = min(I, RR);
//   - tall products C = A^T B over millions of rows (Gram of V_n[2] for the
//     shifted Cholesky-QR, and W_n = Y_[n] Q_0) on FP64 MFMA with ordered split-K;
//   - mode products (TTM, Sec. 2) for the Multi-TTM Y = X x_{j != n} Q_j^T.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

__device__ __forceinline__ void mma64(f64x4& c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename Tin>
__device__ __forceinline__ double ttm_in(const Tin* p) { return (double)*p; }
template <>
__device__ __forceinline__ double ttm_in<uint8_t>(const uint8_t* p) {
  return (double)__builtin_amdgcn_cvt_f32_fp8((int)*p, 0);
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Householder QR of A (m x n, column-major, overwritten).  One workgroup of
// 1024 threads; columns are processed in order, each trailing column updated
// by one wave.  Writes Q (m x r) and R (r x n), r = min(m, n).  V (m x r)
// keeps the reflectors, tau (r) their scales.
__global__ __launch_bounds__(1024) void householder_qr_kernel(double* A, int64_t m, int n, double* V, double* tau,
                                                              double* Q, double* R) {
  __shared__ double red[1024];
  __shared__ double sh_alpha, sh_beta;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = (int)min<int64_t>(m, n);
  for (int k = 0; k < r; ++k) {
    // norm of A[k:m, k]
    double s = 0.0;
    for (int64_t i = k + tid; i < m; i += 1024) s += A[i + m * k] * A[i + m * k];
    const double nrm2 = block_sum(s, red);
    if (tid == 0) {
      const double x0 = A[k + m * k];
      const double nrm = sqrt(nrm2);
      const double alpha = (x0 >= 0.0) ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
      sh_alpha = alpha;
      sh_beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
      A[k + m * k] = v0;   // the reflector lives in A[k:m, k] for the moment
    }
    __syncthreads();
    const double beta = sh_beta;
    for (int64_t i = k + tid; i < m; i += 1024) V[i + m * k] = A[i + m * k];
    for (int64_t i = tid; i < k; i += 1024) V[i + m * k] = 0.0;
    if (tid == 0) tau[k] = beta;
    __syncthreads();
    // apply H = I - beta v v^T to the trailing columns, one wave per column
    for (int j = k + 1 + wave; j < n; j += 16) {
      double d = 0.0;
      for (int64_t i = k + lane; i < m; i += 64) d += V[i + m * k] * A[i + m * j];
      for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
      const double f = beta * d;
      for (int64_t i = k + lane; i < m; i += 64) A[i + m * j] -= f * V[i + m * k];
    }
    __syncthreads();
    if (tid == 0) A[k + m * k] = sh_alpha;
    for (int64_t i = k + 1 + tid; i < m; i += 1024) A[i + m * k] = 0.0;
    __syncthreads();
  }
  // R = upper part of the first r rows
  for (int64_t e = tid; e < (int64_t)r * n; e += 1024) {
    const int i = (int)(e % r), j = (int)(e / r);
    R[e] = (i <= j) ? A[i + m * j] : 0.0;
  }
  // Q = H_0 H_1 ... H_{r-1} [I_r; 0]: apply the reflectors from the last
  for (int64_t e = tid; e < m * r; e += 1024) {
    const int64_t i = e % m, j = e / m;
    Q[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = r - 1; k >= 0; --k) {
    const double beta = tau[k];
    for (int j = wave; j < r; j += 16) {
      double d = 0.0;
      for (int64_t i = k + lane; i < m; i += 64) d += V[i + m * k] * Q[i + m * j];
      for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
      const double f = beta * d;
      for (int64_t i = k + lane; i < m; i += 64) Q[i + m * j] -= f * V[i + m * k];
    }
    __syncthreads();
  }
}

// A double moved across lanes by one DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Sum over the 64 lanes of a wave (all lanes active): pairwise within each row
// of 16 lanes by DPP (swap neighbours, swap pairs, mirror the half rows, mirror
// the rows; every lane of a row then holds the same bits), then the four row
// sums read out and added in a fixed order, so every lane gets the same bits.
__device__ __forceinline__ double wave_sum64(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The same factorization for small unfoldings (m <= 64*RT, n <= 16*CW, the
// reflectors fitting in LDS).  Wave w keeps columns j = w + 16c in registers,
// rows across lanes (i = lane + 64t).  Step k: the wave owning column k forms
// the reflector from its registers and stores it in LDS; after one barrier
// every wave applies it to its own trailing columns.  Q = H_0 ... H_{r-1}[I_r; 0]
// then needs no barrier: each wave applies the reflectors to its own columns of
// Q, skipping H_k for k > j, which leaves e_j unchanged (v_k is zero above row k).
template <int RT, int CW>
__global__ __launch_bounds__(1024) void householder_qr_reg_kernel(const double* A, int m, int n, double* Q,
                                                                  double* R) {
  extern __shared__ double vs[];   // reflector k at vs[k*m + i], zero for i < k
  __shared__ double tau_s[16 * CW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = min(m, n);
  double a[CW][RT];
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t, j = wave + 16 * c;
      a[c][t] = (i < m && j < n) ? A[i + (int64_t)m * j] : 0.0;
    }
  for (int k = 0; k < r; ++k) {
    if (wave == (k & 15)) {
      const int kc = k >> 4;
      double col[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) col[t] = 0.0;
#pragma unroll
      for (int c = 0; c < CW; ++c)
        if (c == kc) {
#pragma unroll
          for (int t = 0; t < RT; ++t) col[t] = a[c][t];
        }
      double s = 0.0, x0p = 0.0;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = lane + 64 * t;
        if (i >= k && i < m) s += col[t] * col[t];
        if (i == k) x0p = col[t];
      }
      const double nrm2 = wave_sum64(s);
      const double x0 = readlane_f64(x0p, k & 63);
      const double nrm = sqrt(nrm2);
      const double alpha = (x0 >= 0.0) ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vtv = nrm2 - x0 * x0 + v0 * v0;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = lane + 64 * t;
        if (i < m) vs[(int64_t)k * m + i] = (i < k) ? 0.0 : (i == k ? v0 : col[t]);
      }
      if (lane == 0) tau_s[k] = vtv > 0.0 ? 2.0 / vtv : 0.0;
      // column k is final: R's entries above the diagonal, alpha on it, zeros below
#pragma unroll
      for (int c = 0; c < CW; ++c)
        if (c == kc) {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const int i = lane + 64 * t;
            if (i == k) a[c][t] = alpha;
            else if (i > k) a[c][t] = 0.0;
          }
        }
    }
    __syncthreads();
    const double beta = tau_s[k];
    double v[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      v[t] = (i < m) ? vs[(int64_t)k * m + i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int j = wave + 16 * c;
      if (j > k && j < n) {
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < RT; ++t) d += v[t] * a[c][t];
        const double f = beta * wave_sum64(d);
#pragma unroll
        for (int t = 0; t < RT; ++t) a[c][t] -= f * v[t];
      }
    }
  }
  // R (r x n): the upper part of the first r rows
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t, j = wave + 16 * c;
      if (i < r && j < n) R[i + (int64_t)r * j] = (i <= j) ? a[c][t] : 0.0;
    }
  // Q (m x r); the last step's barrier made every reflector visible
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int t = 0; t < RT; ++t) a[c][t] = (lane + 64 * t == wave + 16 * c) ? 1.0 : 0.0;
  const int jmax = min(r - 1, wave + 16 * (CW - 1));
  for (int k = jmax; k >= 0; --k) {
    const double beta = tau_s[k];
    double v[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t;
      v[t] = (i < m) ? vs[(int64_t)k * m + i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int j = wave + 16 * c;
      if (j >= k && j < r) {
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < RT; ++t) d += v[t] * a[c][t];
        const double f = beta * wave_sum64(d);
#pragma unroll
        for (int t = 0; t < RT; ++t) a[c][t] -= f * v[t];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CW; ++c)
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int i = lane + 64 * t, j = wave + 16 * c;
      if (i < m && j < r) Q[i + (int64_t)m * j] = a[c][t];
    }
}

// C_part[chunk] = A^T B over rows [chunk*kc, ...): A is K x P, B is K x Q,
// both column-major (lda, ldb).  Mode 1 reads A through the Multi-TTM layout:
// A(k, p) = Y[l + L*(p + Ip*t)] with the row index k = l + L*t, the order in
// which Y is stored (B's rows come in the same order).
struct TallArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int64_t K; int P, Q;
  int64_t kc;            // rows per chunk
  int mode;              // 0 plain, 1 Multi-TTM layout
  int64_t L, Ip, T;      // mode 1 layout
  double* part;          // [nchunk][P][Q] (column-major P x Q per chunk)
};

__global__ __launch_bounds__(256) void tall_atb_kernel(TallArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbp = (g.P + 15) / 16, nbq = (g.Q + 15) / 16;
  const int64_t k0 = (int64_t)blockIdx.x * g.kc;
  const int64_t k1 = min(g.K, k0 + g.kc);
  double* out = g.part + (size_t)blockIdx.x * g.P * g.Q;
  for (int blk = wave; blk < nbp * nbq; blk += 4) {
    const int bp = blk % nbp, bq = blk / nbp;
    const int p = bp * 16 + (lane & 15), q = bq * 16 + (lane & 15);
    f64x4 acc = {0, 0, 0, 0};
    for (int64_t kb = k0; kb < k1; kb += 4) {
      const int64_t k = kb + (lane >> 4);
      double av = 0.0, bv = 0.0;
      if (k < k1) {
        if (p < g.P) {
          if (g.mode == 0) av = g.A[k + g.lda * p];
          else {
            const int64_t l = k % g.L, t = k / g.L;
            av = g.A[l + g.L * (p + g.Ip * t)];
          }
        }
        if (q < g.Q) bv = g.B[k + g.ldb * q];
      }
      mma64(acc, av, bv);
    }
    for (int v = 0; v < 4; ++v) {
      const int row = bp * 16 + (lane >> 4) + 4 * v, col = bq * 16 + (lane & 15);
      if (row < g.P && col < g.Q) out[row + (int64_t)g.P * col] = acc[v];
    }
  }
}

// The same product, register-blocked: a wave owns 16-row blocks of C and
// keeps all NBQ of its 16-column tiles in accumulators, so each A fragment
// is loaded once per k-step; four k-steps of (clamped) operand loads are in
// flight together.  Per tile the sum over k runs in increasing k, as in
// tall_atb_kernel.
template <int NBQ>
__global__ __launch_bounds__(256) void tall_atb_rb_kernel(TallArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbp = (g.P + 15) / 16;
  const int64_t k0 = (int64_t)blockIdx.x * g.kc;
  const int64_t k1 = min(g.K, k0 + g.kc);
  double* out = g.part + (size_t)blockIdx.x * g.P * g.Q;
  constexpr int KU = 4;
  for (int bp = wave; bp < nbp; bp += 4) {
    const int p = bp * 16 + (lane & 15), pc = min(p, g.P - 1);
    f64x4 acc[NBQ];
#pragma unroll
    for (int bq = 0; bq < NBQ; ++bq) acc[bq] = f64x4{0, 0, 0, 0};
    for (int64_t kb = k0; kb < k1; kb += 4 * KU) {
      double av[KU], bv[KU][NBQ];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t k = kb + 4 * u + (lane >> 4);
        const bool kin = k < k1;
        const int64_t kc = kin ? k : k0;
        double a;
        if (g.mode == 0) {
          a = g.A[kc + g.lda * pc];
        } else {
          const int64_t l = kc % g.L, t = kc / g.L;
          a = g.A[l + g.L * (pc + g.Ip * t)];
        }
        av[u] = (kin && p < g.P) ? a : 0.0;
#pragma unroll
        for (int bq = 0; bq < NBQ; ++bq) {
          const int q = bq * 16 + (lane & 15);
          const double b = g.B[kc + g.ldb * min(q, g.Q - 1)];
          bv[u][bq] = (kin && q < g.Q) ? b : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int bq = 0; bq < NBQ; ++bq) mma64(acc[bq], av[u], bv[u][bq]);
    }
#pragma unroll
    for (int bq = 0; bq < NBQ; ++bq)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = bp * 16 + (lane >> 4) + 4 * v, col = bq * 16 + (lane & 15);
        if (row < g.P && col < g.Q) out[row + (int64_t)g.P * col] = acc[bq][v];
      }
  }
}

// The same product with the operands staged through LDS: each k-slab of
// GKS rows is read with lanes along k (coalesced for column-major operands),
// stored as [column][k] and consumed by the four waves, which split the
// 16x16 output tiles between them.  Element (k, p) of A sits at
// base(k) + sp * p: base(k) = k, sp = lda in the plain layout, and
// base(k) = l + L*Ip*t, sp = L in the Multi-TTM layout (l = k mod L,
// t = k div L).  With A == B (a Gram matrix) only the tiles on or above the
// diagonal are formed and each is written to both halves, so the result is
// exactly symmetric.  Within a slab, MFMA step (j, e) takes from lane group
// kq the row k = 8j + 2kq + e for both operands.
constexpr int GKS = 32, GST = GKS + 2, GLD = 256 / GKS;

// NB: 16-row blocks held per operand (rows past P or Q are zero); GRAM: A is
// B.  Waves whose tile count is below TMAX repeat tile 0 and drop the result.
template <int NB, bool GRAM>
__global__ __launch_bounds__(256) void tall_atb_lds_kernel(TallArgs g) {
  constexpr int NT = GRAM ? NB * (NB + 1) / 2 : NB * NB, TMAX = (NT + 3) / 4, NR = NB * 16 / GLD;
  extern __shared__ __align__(16) double gsm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kk = tid % GKS, pg = tid / GKS;
  const int nbp = (g.P + 15) / 16, nbq = (g.Q + 15) / 16;
  double* As = gsm;
  double* Bs = GRAM ? gsm : gsm + NB * 16 * GST;
  const int64_t k0 = (int64_t)blockIdx.x * g.kc;
  const int64_t k1 = min(g.K, k0 + g.kc);
  const int64_t sp = g.mode == 0 ? g.lda : g.L;
  const int ntile = GRAM ? nbp * (nbp + 1) / 2 : nbp * nbq;
  int offa[TMAX], offb[TMAX], tbp[TMAX], tbq[TMAX];
  int nt = 0;
#pragma unroll
  for (int s = 0; s < TMAX; ++s) {
    const int i = wave + 4 * s;
    int bp = 0, bq = 0;
    if (i < ntile) {
      ++nt;
      if (GRAM) {
        int r = i;
        while (r > bq) { r -= bq + 1; ++bq; }
        bp = r;
      } else {
        bp = i % nbp; bq = i / nbp;
      }
    }
    tbp[s] = bp; tbq[s] = bq;
    offa[s] = (bp * 16 + (lane & 15)) * GST + 2 * (lane >> 4);
    offb[s] = (bq * 16 + (lane & 15)) * GST + 2 * (lane >> 4);
  }
  f64x4 acc[TMAX];
#pragma unroll
  for (int s = 0; s < TMAX; ++s) acc[s] = f64x4{0, 0, 0, 0};
  double ra[NR], rb[NR];
  auto load = [&](int64_t ks) {
    const int64_t k = ks + kk;
    const bool kin = k < k1;
    const int64_t kc = kin ? k : k0;
    int64_t base = kc;
    if (g.mode != 0) { const int64_t l = kc % g.L, t = kc / g.L; base = l + g.L * g.Ip * t; }
    const double* pa = g.A + base;
    const double* pb = g.B + kc;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int p = pg + GLD * i;
      const double va = pa[sp * min(p, g.P - 1)];
      ra[i] = (kin && p < g.P) ? va : 0.0;
      if (!GRAM) {
        const double vb = pb[g.ldb * min(p, g.Q - 1)];
        rb[i] = (kin && p < g.Q) ? vb : 0.0;
      }
    }
  };
  if (k0 < k1) load(k0);
  for (int64_t ks = k0; ks < k1; ks += GKS) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int p = pg + GLD * i;
      As[p * GST + kk] = ra[i];
      if (!GRAM) Bs[p * GST + kk] = rb[i];
    }
    __syncthreads();
    if (ks + GKS < k1) load(ks + GKS);
#pragma unroll
    for (int j = 0; j < GKS / 8; ++j) {
      double2 a[TMAX], b[TMAX];
#pragma unroll
      for (int s = 0; s < TMAX; ++s) {
        a[s] = *reinterpret_cast<const double2*>(As + offa[s] + 8 * j);
        b[s] = *reinterpret_cast<const double2*>(Bs + offb[s] + 8 * j);
      }
#pragma unroll
      for (int s = 0; s < TMAX; ++s) mma64(acc[s], a[s].x, b[s].x);
#pragma unroll
      for (int s = 0; s < TMAX; ++s) mma64(acc[s], a[s].y, b[s].y);
    }
  }
  double* out = g.part + (size_t)blockIdx.x * g.P * g.Q;
#pragma unroll
  for (int s = 0; s < TMAX; ++s)
    if (s < nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tbp[s] * 16 + (lane >> 4) + 4 * v, col = tbq[s] * 16 + (lane & 15);
        if (row < g.P && col < g.Q) {
          out[row + (int64_t)g.P * col] = acc[s][v];
          if (GRAM && tbp[s] != tbq[s]) out[col + (int64_t)g.P * row] = acc[s][v];
        }
      }
}

// Gram C = A^T A of a tall column-major A (K x P, P <= 112) with no LDS
// staging.  The MFMA fragment of a 16-column block (lane: column lane&15, rows
// 4*(lane>>4) .. +3 of a 16-row group) is the same for both operands, so each
// wave loads every block once per 16 rows and accumulates all NB(NB+1)/2 tiles
// of the block upper triangle, loading the next group while the MFMAs run.
// Waves take interleaved 16-row groups of the workgroup's chunk; their sums are
// added in LDS in wave order, so the result does not depend on timing.
// 16-row groups a wave holds (GF_G * 64 rows per step of the workgroup): two
// measured slower (366 against 316 us for 10^6 x 100)
constexpr int GF_G = 1;
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void gram_frag_kernel(
    const double* A, int64_t lda, int64_t K, int P, int64_t kc, double* part) {
  constexpr int NT = NB * (NB + 1) / 2, RS = 64 * GF_G;
  extern __shared__ __align__(16) double gred[];   // NT * 256 doubles
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, kq = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * kc;
  const int64_t k1 = min(K, k0 + kc);
  const double* pc[NB];
  bool cin[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = b * 16 + cl;
    cin[b] = c < P;
    pc[b] = A + lda * (int64_t)min(c, P - 1);
  }
  f64x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f64x4{0, 0, 0, 0};
  double2 f[GF_G][NB][2];
  // half h of the fragments of group s, the 16 rows at g + 16 s: rows
  // g + 16 s + 4kq + 2h, +1
  auto load = [&](int64_t g, int s, int h) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t k = g + 16 * s + 4 * kq + 2 * h;
      if (cin[b] && k + 1 < k1) {
        f[s][b][h] = *reinterpret_cast<const double2*>(pc[b] + k);
      } else {
        f[s][b][h].x = (cin[b] && k < k1) ? pc[b][k] : 0.0;
        f[s][b][h].y = 0.0;
      }
    }
  };
  auto mfma = [&](int s, int h) {
    int t = 0;
#pragma unroll
    for (int bq = 0; bq < NB; ++bq)
#pragma unroll
      for (int bp = 0; bp <= bq; ++bp, ++t) mma64(acc[t], f[s][bp][h].x, f[s][bq][h].x);
    t = 0;
#pragma unroll
    for (int bq = 0; bq < NB; ++bq)
#pragma unroll
      for (int bp = 0; bp <= bq; ++bp, ++t) mma64(acc[t], f[s][bp][h].y, f[s][bq][h].y);
  };
  // a wave takes GF_G consecutive 16-row groups of each RS-row step; each
  // half is reloaded for the next step as soon as its MFMAs are issued, so a
  // load has the other halves' MFMAs to arrive
  int64_t g = k0 + 16 * GF_G * wave;
  if (g < k1) {
#pragma unroll
    for (int s = 0; s < GF_G; ++s) {
      load(g, s, 0);
      load(g, s, 1);
    }
  }
  // (past the chunk end the loads return zeros, so they need no branch)
  for (; g < k1; g += RS) {
#pragma unroll
    for (int s = 0; s < GF_G; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        mfma(s, h);
        load(g + RS, s, h);
      }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* p = gred + (t * 64 + lane) * 4 + v;
          *p = (w == 0) ? acc[t][v] : *p + acc[t][v];
        }
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * P * P;
  for (int e = threadIdx.x; e < NT * 64; e += 256) {
    const int t = e >> 6, l = e & 63;
    int bq = 0, r = t;
    while (r > bq) { r -= bq + 1; ++bq; }
    const int bp = r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = bp * 16 + (l >> 4) + 4 * v, col = bq * 16 + (l & 15);
      if (row < P && col < P) {
        const double x = gred[e * 4 + v];
        out[row + (int64_t)P * col] = x;
        if (bp != bq) out[col + (int64_t)P * row] = x;
      }
    }
  }
}

// C (P x Q) = A^T B for two different tall operands (K rows, P, Q <= 16*NB)
// with the MFMA fragments loaded straight into registers, as in the Gram
// kernel above.  Element (k, p) of A sits at A[k*ks + p*ps] (used for the
// row-major layout of a first-mode unfolding; k-contiguous operands take the
// LDS-staged kernel below); B is column-major (ld ldb).  The NB x NB output
// tiles, in column-major tile order, are dealt to the four waves in runs of
// ceil(NB^2/4), so a wave's accumulators fit its registers; every wave runs
// over the whole chunk (the repeated fragment loads hit the caches) and
// stores its own tiles.  In the group of 16 rows starting at row g, lane
// (c, kq) holds rows g + 4kq + j, j = 0..3, of both operands.
// (AtbArgs' L and LIp describe A in the Multi-TTM layout for the LDS-staged
// kernel: element (k, p) at A[l + LIp*t + L*p], k = l + L*t.)
struct AtbArgs {
  const double* A; int64_t ks, ps, L, LIp;
  const double* B; int64_t ldb;
  int64_t K, kc; int P, Q;
  double* part;
};

template <int NB, int W, int G, bool BV>
__device__ __forceinline__ void atb_frag_wave(const AtbArgs& g) {
  constexpr int NT = NB * NB, TW = (NT + 3) / 4, T0 = W * TW < NT ? W * TW : NT;
  constexpr int T1 = T0 + TW < NT ? T0 + TW : NT;
  constexpr int NTW = T1 > T0 ? T1 - T0 : 1, BQ0 = T0 / NB, NQ = T1 > T0 ? (T1 - 1) / NB - BQ0 + 1 : 1;
  constexpr int RS = 16 * G;   // rows per loop step
  if (T1 <= T0) return;
  const int lane = threadIdx.x & 63, cl = lane & 15, kq = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * g.kc;
  const int64_t k1 = min(g.K, k0 + g.kc);
  // Columns past P or Q read column P-1 or Q-1: those rows and columns of the
  // tiles are never stored, and the MFMA keeps them apart from the rest.
  // Rows past the chunk read a row inside it with B's value zeroed, so every
  // load is unconditional (no branch around it).
  const double* acol[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acol[b] = g.A + (int64_t)min(16 * b + cl, g.P - 1) * g.ps;
  const double* bcol[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) bcol[u] = g.B + g.ldb * min(16 * (BQ0 + u) + cl, g.Q - 1);
  f64x4 acc[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) acc[t] = f64x4{0, 0, 0, 0};
  // G 16-row groups in registers (rows j = 4s + jj: group s, row jj of the
  // lane), reloaded a quarter (two rows) at a time as each quarter's MFMAs
  // are issued, so a load has 2G - 1 quarters of MFMAs to arrive.  One group
  // measured fastest (100 x 100 result, 10^6 rows: 630-870 us against
  // 950-1350 us for two and 720-1130 us for three).
  double fa[NB][4 * G], fb[NQ][4 * G];
  // per group s: the element offset of the lane's first row, advanced with
  // the rows
  int64_t rg[G];
#pragma unroll
  for (int sg = 0; sg < G; ++sg) rg[sg] = (k0 + 16 * sg + 4 * kq) * g.ks;
  auto load = [&](int64_t gg, int q) {
    const int sg = q >> 1, h = q & 1;
    const int64_t rb = gg + 16 * sg + 4 * kq;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int jj = 2 * h + e;
      const int64_t r = rb + jj;
      const int64_t ro = r < k1 ? rg[sg] + jj * g.ks : 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) fa[b][4 * sg + jj] = acol[b][ro];
    }
    if (BV) {   // ldb and the chunk ends even: rows rb + 2h, +1 are in or out together
      const int64_t r = rb + 2 * h;
      const double m = r < k1 ? 1.0 : 0.0;
      const int64_t rc = r < k1 ? r : k0;
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const double2 v = *reinterpret_cast<const double2*>(bcol[u] + rc);
        fb[u][4 * sg + 2 * h] = m * v.x;
        fb[u][4 * sg + 2 * h + 1] = m * v.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t r = rb + 2 * h + e;
        const double m = r < k1 ? 1.0 : 0.0;
        const int64_t rc = r < k1 ? r : k0;
#pragma unroll
        for (int u = 0; u < NQ; ++u) fb[u][4 * sg + 2 * h + e] = m * bcol[u][rc];
      }
    }
  };
  auto mfma = [&](int q) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int t = T0; t < T1; ++t) mma64(acc[t - T0], fa[t % NB][2 * q + e], fb[t / NB - BQ0][2 * q + e]);
  };
  int64_t gg = k0;
#pragma unroll
  for (int q = 0; q < 2 * G; ++q) load(gg, q);
  // past the chunk end the loads are redirected as above, so the loop has no
  // branches around them
  for (; gg < k1; gg += RS) {
#pragma unroll
    for (int sg = 0; sg < G; ++sg) rg[sg] += RS * g.ks;
#pragma unroll
    for (int q = 0; q < 2 * G; ++q) {
      mfma(q);
      load(gg + RS, q);
    }
  }
  double* out = g.part + (size_t)blockIdx.x * g.P * g.Q;
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const int bp = t % NB, bq = t / NB;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = bp * 16 + (lane >> 4) + 4 * v, col = bq * 16 + cl;
      if (row < g.P && col < g.Q) out[row + (int64_t)g.P * col] = acc[t - T0][v];
    }
  }
}

// Row groups held per wave and workgroups (row chunks) per launch of
// atb_frag_kernel.
constexpr int ATB_G = 1, ATB_CHUNKS = 512;

template <int NB, bool BV>
__global__ __launch_bounds__(256) void atb_frag_kernel(AtbArgs g) {
  switch (threadIdx.x >> 6) {
    case 0: atb_frag_wave<NB, 0, ATB_G, BV>(g); break;
    case 1: atb_frag_wave<NB, 1, ATB_G, BV>(g); break;
    case 2: atb_frag_wave<NB, 2, ATB_G, BV>(g); break;
    default: atb_frag_wave<NB, 3, ATB_G, BV>(g); break;
  }
}

// The same product with both operands staged through LDS: a workgroup copies
// each 16-row step of A and B (coalesced, every element read once) into LDS
// as [column][row] (row pitch AL_KP, conflict-free 16-byte fragment reads),
// double-buffered with one barrier per step, and each wave forms its run of
// output tiles from the LDS fragments, as above.  Lane (c, kq) takes rows
// 4kq + j, j = 0..3, of the step.
constexpr int AL_ROWS = 16, AL_KP = AL_ROWS + 2;
template <int NB, int W>
__device__ __forceinline__ void atb_lds_mma(const double* As, const double* Bs, f64x4* acc) {
  constexpr int NT = NB * NB, TW = (NT + 3) / 4, T0 = W * TW < NT ? W * TW : NT;
  constexpr int T1 = T0 + TW < NT ? T0 + TW : NT;
  constexpr int BQ0 = T0 / NB, NQ = T1 > T0 ? (T1 - 1) / NB - BQ0 + 1 : 1;
  if (T1 <= T0) return;
  const int lane = threadIdx.x & 63, cl = lane & 15, kq = lane >> 4;
  double fa[NB][4], fb[NQ][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const double* q = As + (16 * b + cl) * AL_KP + 4 * kq;
    const double2 x = *reinterpret_cast<const double2*>(q), y = *reinterpret_cast<const double2*>(q + 2);
    fa[b][0] = x.x; fa[b][1] = x.y; fa[b][2] = y.x; fa[b][3] = y.y;
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const double* q = Bs + (16 * (BQ0 + u) + cl) * AL_KP + 4 * kq;
    const double2 x = *reinterpret_cast<const double2*>(q), y = *reinterpret_cast<const double2*>(q + 2);
    fb[u][0] = x.x; fb[u][1] = x.y; fb[u][2] = y.x; fb[u][3] = y.y;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int t = T0; t < T1; ++t) mma64(acc[t - T0], fa[t % NB][j], fb[t / NB - BQ0][j]);
}

template <int NB, int W>
__device__ __forceinline__ void atb_lds_store(const AtbArgs& g, const f64x4* acc) {
  constexpr int NT = NB * NB, TW = (NT + 3) / 4, T0 = W * TW < NT ? W * TW : NT;
  constexpr int T1 = T0 + TW < NT ? T0 + TW : NT;
  const int lane = threadIdx.x & 63;
  double* out = g.part + (size_t)blockIdx.x * g.P * g.Q;
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const int bp = t % NB, bq = t / NB;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = bp * 16 + (lane >> 4) + 4 * v, col = bq * 16 + (lane & 15);
      if (row < g.P && col < g.Q) out[row + (int64_t)g.P * col] = acc[t - T0][v];
    }
  }
}

// LAY: A in the Multi-TTM layout (else column-major: k contiguous).
template <int NB, bool LAY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void atb_lds_kernel(AtbArgs g) {
  constexpr int NP = 16 * NB, OPS = NP * AL_KP, TW = (NB * NB + 3) / 4;
  extern __shared__ __align__(16) double als[];   // 2 buffers x (A, B) x NP x AL_KP
  const int tid = threadIdx.x, wave = tid >> 6;
  const int kk = tid % AL_ROWS, pp = tid / AL_ROWS;   // this thread's row of a step, first column
  const int64_t k0 = (int64_t)blockIdx.x * g.kc;
  const int64_t k1 = min(g.K, k0 + g.kc);
  const int nsteps = (int)((k1 - k0 + AL_ROWS - 1) / AL_ROWS);
  // position of the thread's row in A's layout, advanced AL_ROWS rows a step
  // (L below 2^31 here)
  uint32_t lr = 0;
  int64_t ro = 0;
  {
    const int64_t r0 = k0 + kk;
    if (LAY) { lr = (uint32_t)(r0 % g.L); ro = lr + g.LIp * (r0 / g.L); }
    else ro = r0 * g.ks;
  }
  const int64_t ps = LAY ? g.L : g.ps;
  double ra[NB], rb[NB];
  auto load = [&](int st) {
    const int64_t r = k0 + (int64_t)st * AL_ROWS + kk;
    const bool rin = r < k1;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int p = pp + 16 * i;
      ra[i] = (rin && p < g.P) ? g.A[ro + ps * p] : 0.0;
      rb[i] = (rin && p < g.Q) ? g.B[r + g.ldb * p] : 0.0;
    }
  };
  auto advance = [&]() {
    if (LAY) {
      const uint32_t L32 = (uint32_t)g.L, w = (lr + (uint32_t)AL_ROWS) / L32;
      lr = lr + (uint32_t)AL_ROWS - w * L32;
      ro += AL_ROWS + (int64_t)w * (g.LIp - g.L);
    } else {
      ro += AL_ROWS * g.ks;
    }
  };
  auto stash = [&](int buf) {
    double* As = als + buf * 2 * OPS;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      As[(pp + 16 * i) * AL_KP + kk] = ra[i];
      As[OPS + (pp + 16 * i) * AL_KP + kk] = rb[i];
    }
  };
  f64x4 acc[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t) acc[t] = f64x4{0, 0, 0, 0};
  if (nsteps > 0) {
    load(0);
    stash(0);
  }
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const bool more = st + 1 < nsteps;
    if (more) {
      advance();
      load(st + 1);
    }
    const double* As = als + (st & 1) * 2 * OPS;
    switch (wave) {
      case 0: atb_lds_mma<NB, 0>(As, As + OPS, acc); break;
      case 1: atb_lds_mma<NB, 1>(As, As + OPS, acc); break;
      case 2: atb_lds_mma<NB, 2>(As, As + OPS, acc); break;
      default: atb_lds_mma<NB, 3>(As, As + OPS, acc); break;
    }
    if (more) stash((st + 1) & 1);
    __syncthreads();
  }
  switch (wave) {
    case 0: atb_lds_store<NB, 0>(g, acc); break;
    case 1: atb_lds_store<NB, 1>(g, acc); break;
    case 2: atb_lds_store<NB, 2>(g, acc); break;
    default: atb_lds_store<NB, 3>(g, acc); break;
  }
}

// C = sum over chunks; a block takes 64 outputs, its four waves each sum a
// contiguous quarter of the chunks, and the quarters are added in order.
__global__ __launch_bounds__(256) void sum_chunks_kernel(const double* part, int nchunk, int64_t n, double* C) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const int64_t ec = e < n ? e : n - 1;
  const int per = (nchunk + 3) / 4, c0 = wave * per, c1 = min(nchunk, c0 + per);
  double s = 0.0;
#pragma unroll 8
  for (int c = c0; c < c1; ++c) s += part[(size_t)c * n + ec];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && e < n) C[e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Mode product: out(l, r, t) = scale * sum_i in(l + L*(i + I*t)) Q(i + I*r).
template <typename Tin>
__global__ void ttm_kernel(const Tin* in, int64_t L, int64_t I, int64_t T, const double* Q, int R, double scale,
                           double* out) {
  const int64_t n = L * R * T;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e % L;
    const int64_t r = (e / L) % R;
    const int64_t t = e / (L * R);
    const Tin* x = in + l + L * I * t;
    const double* q = Q + I * r;
    double s = 0.0;
    for (int64_t i = 0; i < I; ++i) s += (double)x[L * i] * q[i];
    out[e] = s * scale;
  }
}

__global__ void ttm_fp8_kernel(const uint8_t* in, int64_t L, int64_t I, int64_t T, const double* Q, int R,
                               double scale, double* out) {
  const int64_t n = L * R * T;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e % L;
    const int64_t r = (e / L) % R;
    const int64_t t = e / (L * R);
    const uint8_t* x = in + l + L * I * t;
    const double* q = Q + I * r;
    double s = 0.0;
    for (int64_t i = 0; i < I; ++i) {
      const float v = __builtin_amdgcn_cvt_f32_fp8((int)x[L * i], 0);
      s += (double)v * q[i];
    }
    out[e] = s * scale;
  }
}

// The same mode product, register-blocked: a workgroup takes TRB consecutive
// r (their columns of Q staged in LDS) and a thread one (l, t) pair, so each
// input element is read once per TRB outputs instead of once per output.
// Summation over i in increasing order, as in ttm_kernel.
constexpr int TRB = 16;
template <typename Tin>
__global__ __launch_bounds__(256) void ttm_rb_kernel(const Tin* in, int64_t L, int64_t I, int64_t T, const double* Q,
                                                     int R, double scale, double* out) {
  extern __shared__ double qs[];   // [I][TRB]: Q(i, r0 + rr)
  const int tid = threadIdx.x, r0 = blockIdx.y * TRB;
  for (int64_t e = tid; e < I * TRB; e += 256) {
    const int64_t i = e % I;
    const int rr = (int)(e / I);
    qs[i * TRB + rr] = r0 + rr < R ? Q[i + I * (r0 + rr)] : 0.0;
  }
  __syncthreads();
  const int64_t LT = L * T;
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < LT; e += (int64_t)gridDim.x * 256) {
    const int64_t l = e % L, t = e / L;
    const Tin* x = in + l + L * I * t;
    double acc[TRB];
#pragma unroll
    for (int rr = 0; rr < TRB; ++rr) acc[rr] = 0.0;
    for (int64_t i = 0; i < I; ++i) {
      const double xv = ttm_in(x + L * i);
      const double* q = qs + i * TRB;
#pragma unroll
      for (int rr = 0; rr < TRB; ++rr) acc[rr] = fma(xv, q[rr], acc[rr]);
    }
#pragma unroll
    for (int rr = 0; rr < TRB; ++rr)
      if (r0 + rr < R) out[l + L * (r0 + rr) + L * (int64_t)R * t] = acc[rr] * scale;
  }
}

// out[i + I*(l + L*t)] = in[l + L*(i + I*t)]: every slice t (an L x I matrix)
// transposed, through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void slice_transpose_kernel(const double* in, int64_t L, int64_t I, int64_t T,
                                                              double* out) {
  __shared__ double tile[32][33];
  const int64_t nl = (L + 31) / 32;
  const int64_t l0 = (blockIdx.x % nl) * 32, i0 = (blockIdx.x / nl) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int64_t t = blockIdx.y; t < T; t += gridDim.y) {
    const double* src = in + L * I * t;
    double* dst = out + L * I * t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t l = l0 + tx, i = i0 + ty + 8 * k;
      if (l < L && i < I) tile[ty + 8 * k][tx] = src[l + L * i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = i0 + tx, l = l0 + ty + 8 * k;
      if (l < L && i < I) dst[i + I * l] = tile[tx][ty + 8 * k];
    }
    __syncthreads();
  }
}

__global__ void transpose_kernel(const double* A, int64_t rows, int64_t cols, double* At) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  At[j + cols * i] = A[e];
}

// V2[k' + J*(a + Ra*b)] = T[k*C + b + Rb*a]: the bond order of the subchain
// table turned into the column order a + R_n*b of G_n(2), and the rows
// reordered from the chain's cyclic index k = t + (J/L)*l (t over the modes
// after n, l over those before it) to k' = l + L*t, the order in which the
// Multi-TTM result stores them.  A row permutation leaves the Gram matrix,
// the triangular factor and W_n = Y_[n]^T Q_0 unchanged.
__device__ __forceinline__ int64_t v2_src_row(int64_t kp, int64_t J, int64_t L) {
  return kp / L + (J / L) * (kp % L);
}
__global__ void table_to_v2_kernel(const double* T, int64_t J, int64_t L, int Ra, int Rb, double* V2) {
  const int64_t C = (int64_t)Ra * Rb;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * C) return;
  const int64_t kp = e % J, col = e / J;
  const int64_t a = col % Ra, b = col / Ra;
  V2[e] = T[v2_src_row(kp, J, L) * C + b + Rb * a];
}

// The same reordering through LDS: a block gathers V2T_ROWS table rows (each
// read whole and contiguous) and writes each output column as one run.
constexpr int V2T_ROWS = 32;
__global__ __launch_bounds__(256) void table_to_v2_tiled_kernel(const double* T, int64_t J, int64_t L, int Ra,
                                                                 int Rb, double* V2) {
  extern __shared__ __align__(16) double vsm[];
  const int C = Ra * Rb, pitch = C + 1;
  const int64_t k0 = (int64_t)blockIdx.x * V2T_ROWS;
  const int nk = (int)min<int64_t>(V2T_ROWS, J - k0);
  for (int e = threadIdx.x; e < nk * C; e += 256) {
    const int kl = e / C, c = e % C;
    vsm[kl * pitch + c] = T[v2_src_row(k0 + kl, J, L) * C + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < V2T_ROWS * C; e += 256) {
    const int kl = e % V2T_ROWS, col = e / V2T_ROWS;
    const int a = col % Ra, b = col / Ra;
    if (kl < nk) V2[k0 + kl + J * col] = vsm[kl * pitch + b + Rb * a];
  }
}

// The last step of the subchain written straight in the V_n[2] layout: row
// k' of V2 (Multi-TTM order) is table row src = v2_src_row(k') = j + Jp*i of
// the full subchain, whose entry is Tp[j] (Rb x Rm, the subchain without its
// last core) times the slice i of the last core (Rm x Ra):
//   V2[k' + J*(a + Ra*b)] = sum_m Tp[j][b + Rb*m] * core[m + Rm*(i + I*a)],
// summed over m in increasing order (the chain step's order, so the values
// are those of the two-pass build).  A block stages its rows' operands in
// LDS, then each thread forms outputs of one row, a column at a time, so
// consecutive lanes write consecutive rows of a column.
__global__ __launch_bounds__(256) void v2_direct_kernel(const double* Tp, int64_t Jp, const double* core, int64_t I,
                                                        int Rm, int Ra, int Rb, int64_t L, int rows, double* V2) {
  extern __shared__ __align__(16) double vds[];
  const int tc = Rb * Rm, gc = Rm * Ra, pitch = (tc + gc) | 1;   // odd pitch: rows spread over the banks
  const int64_t J = Jp * I, C = (int64_t)Ra * Rb;
  const int64_t k0 = (int64_t)blockIdx.x * rows;
  const int nk = (int)min<int64_t>(rows, J - k0);
  for (int kl = threadIdx.x / 64; kl < nk; kl += 4) {   // one wave per row
    const int64_t src = v2_src_row(k0 + kl, J, L), j = src % Jp, i = src / Jp;
    double* d = vds + (int64_t)kl * pitch;
    const double* tp = Tp + j * tc;
    for (int e = threadIdx.x & 63; e < tc; e += 64) d[e] = tp[e];
    for (int e = threadIdx.x & 63; e < gc; e += 64) {
      const int m = e % Rm, a = e / Rm;
      d[tc + e] = core[m + Rm * (i + I * a)];
    }
  }
  __syncthreads();
  const int kl = threadIdx.x % rows, nq = 256 / rows;
  if (kl >= nk) return;
  const double* t = vds + (int64_t)kl * pitch;
  const double* gsl = t + tc;
  for (int64_t col = threadIdx.x / rows; col < C; col += nq) {
    const int a = (int)(col % Ra), b = (int)(col / Ra);
    double acc = 0.0;
    for (int m = 0; m < Rm; ++m) acc += t[b + Rb * m] * gsl[m + Rm * a];
    V2[k0 + kl + J * col] = acc;
  }
}

// Batched C_b = scale * A_b B for tall A_b (M x K) and a small B (K x N, ld
// ldb), K, N <= 16*NB.  Element (m, k) of A_b sits at A[b*sa + m*rs + k*ks]
// and (m, n) of C_b at C[b*sc + m*crs + n*cns]: a column-major matrix, one
// t-slice of a mode product, or the row-major first-mode product.  B is
// staged once per workgroup in LDS as [n][k]; each wave then takes 16-row
// tiles of the batches' rows laid end to end (a tile may span two batches)
// with no further barrier: the tile's A fragments come straight from memory
// into registers, the next tile's while the current one's MFMAs run, and the
// wave forms all the column tiles of C for its rows.  With column-major C
// the MFMA forms C^T = B^T A^T, so a store covers 16 consecutive rows; with
// row-major C (ROWOUT) it forms C = A B, so a store covers 16 consecutive
// columns.  Step (j, e) takes from lane group kq the inner index
// k = 8j + 2kq + e; k past K reads A at k = K-1 against zero rows of B.
// UPPER: B is upper triangular (B[k, n] = 0 for k > n, as L^{-T} in the
// Cholesky-QR passes), so step j skips the column tiles whose columns all lie
// below k = 8j (tile ct needs 8j <= 16ct + 15, i.e. ct >= j/2): about 60 % of
// the MFMAs at K = N = 100, with the same sums (the skipped terms are
// products with exact zeros).
struct TGArgs {
  const void* A; int64_t rs, ks, sa, M; int K;
  const double* B; int ldb, N;
  double* C; int64_t crs, cns, sc, nbatch;
  double scale;
};
constexpr int TG_WAVES = 4;
template <int NB, bool TRIM, bool ROWOUT, bool UPPER, typename Tin>
__global__ __launch_bounds__(64 * TG_WAVES) void tall_gemm_kernel(TGArgs g) {
  // k steps of 8: all 16*NB values of k, or (TRIM, K <= 16*NB - 8) one fewer
  constexpr int NP = 16 * NB, BST = NP + 2, KJ = 2 * NB - (TRIM ? 1 : 0);
  extern __shared__ __align__(16) double tsm[];   // B as [n][k], NP x BST
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cl = lane & 15, kq = lane >> 4;
  const int K = g.K, N = g.N;
  for (int e = tid; e < NP * NP; e += 64 * TG_WAVES) {
    const int n = e / NP, k = e % NP;
    tsm[n * BST + k] = (n < N && k < K) ? g.B[k + (int64_t)g.ldb * n] : 0.0;
  }
  __syncthreads();
  const Tin* A = static_cast<const Tin*>(g.A);
  const int64_t rows = g.M * g.nbatch, ntile = (rows + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * TG_WAVES;
  double2 cur[KJ], nxt[KJ];
  // A fragments of the tile's rows (row tile*16 + cl of the lane; rows past
  // the end read the last row and are not stored)
  auto load = [&](int64_t tile, double2* f) {
    const int64_t r = min(tile * 16 + cl, rows - 1);
    const int64_t b = r / g.M, m = r - b * g.M;
    const Tin* ab = A + b * g.sa + m * g.rs;
#pragma unroll
    for (int j = 0; j < KJ; ++j) {
      const int k = 8 * j + 2 * kq;
      f[j].x = ttm_in(ab + g.ks * min(k, K - 1));
      f[j].y = ttm_in(ab + g.ks * min(k + 1, K - 1));
    }
  };
  int64_t tile = (int64_t)blockIdx.x * TG_WAVES + wave;
  if (tile < ntile) load(tile, cur);
  for (; tile < ntile; tile += wstride) {
    const int64_t tn = tile + wstride;
    load(tn < ntile ? tn : tile, nxt);
    f64x4 acc[NB];
#pragma unroll
    for (int ct = 0; ct < NB; ++ct) acc[ct] = f64x4{0, 0, 0, 0};
    // KJ steps of k and all 16*NB values of n (padding is zero in B): fixed trip
    // counts keep the fragments in fixed registers.  The B fragments of step
    // j + 1 are read from LDS while step j's MFMAs run.
    double2 bv[2][NB];
#pragma unroll
    for (int ct = 0; ct < NB; ++ct)
      bv[0][ct] = *reinterpret_cast<const double2*>(tsm + (16 * ct + cl) * BST + 2 * kq);
#pragma unroll
    for (int j = 0; j < KJ; ++j) {
      if (j + 1 < KJ) {
#pragma unroll
        for (int ct = UPPER ? (j + 1) / 2 : 0; ct < NB; ++ct)
          bv[(j + 1) & 1][ct] =
              *reinterpret_cast<const double2*>(tsm + (16 * ct + cl) * BST + 8 * (j + 1) + 2 * kq);
      }
#pragma unroll
      for (int ct = UPPER ? j / 2 : 0; ct < NB; ++ct) {
        const double2 b = bv[j & 1][ct];
        if (ROWOUT) {
          mma64(acc[ct], cur[j].x, b.x);
          mma64(acc[ct], cur[j].y, b.y);
        } else {
          mma64(acc[ct], b.x, cur[j].x);
          mma64(acc[ct], b.y, cur[j].y);
        }
      }
      // keep later steps' LDS reads from being hoisted over these MFMAs (all
      // of them at once would not fit the registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ROWOUT) {   // lane: rows tile*16 + kq + 4v, column 16ct + cl
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = tile * 16 + kq + 4 * v;
        if (r < rows) {
          const int64_t b = r / g.M, m = r - b * g.M;
          double* cb = g.C + b * g.sc + m * g.crs;
#pragma unroll
          for (int ct = 0; ct < NB; ++ct) {
            const int n = 16 * ct + cl;
            if (n < N) cb[(int64_t)n * g.cns] = g.scale * acc[ct][v];
          }
        }
      }
    } else {        // lane: row tile*16 + cl, columns 16ct + kq + 4v
      const int64_t r = tile * 16 + cl;
      if (r < rows) {
        const int64_t b = r / g.M, m = r - b * g.M;
        double* cb = g.C + b * g.sc + m * g.crs;
#pragma unroll
        for (int ct = 0; ct < NB; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = 16 * ct + kq + 4 * v;
            if (n < N) cb[(int64_t)n * g.cns] = g.scale * acc[ct][v];
          }
      }
    }
#pragma unroll
    for (int j = 0; j < KJ; ++j) cur[j] = nxt[j];
  }
}

template <typename Tin>
hipError_t launch_tg(const TGArgs& g, hipStream_t s, bool upper = false) {
  const int nb = max((g.K + 15) / 16, (g.N + 15) / 16);
  const bool rowout = g.cns == 1 && g.crs != 1;
  if (g.M <= 0 || g.K <= 0 || g.N <= 0 || g.nbatch <= 0 || nb > 7) return hipErrorInvalidValue;
  if (upper && (rowout || !std::is_same<Tin, double>::value)) return hipErrorInvalidValue;
  const size_t lds = (size_t)16 * nb * (16 * nb + 2) * sizeof(double);
  const int64_t ntile = (g.M * g.nbatch + 15) / 16;
  const dim3 grid((unsigned)std::min<int64_t>((ntile + TG_WAVES - 1) / TG_WAVES, 256));
  const void* k = nullptr;
  const bool trim = g.K <= 16 * nb - 8;
  if (upper) {   // column-major output, FP64 input
    switch (nb * 2 + (trim ? 1 : 0)) {
#define TG_UCASE(NBV) \
  case 2 * NBV: k = (const void*)tall_gemm_kernel<NBV, false, false, true, double>; break; \
  case 2 * NBV + 1: k = (const void*)tall_gemm_kernel<NBV, true, false, true, double>; break;
      TG_UCASE(1) TG_UCASE(2) TG_UCASE(3) TG_UCASE(4) TG_UCASE(5) TG_UCASE(6) TG_UCASE(7)
#undef TG_UCASE
    }
  } else {
    switch (nb * 4 + (trim ? 2 : 0) + (rowout ? 1 : 0)) {
#define TG_CASE(NBV) \
  case 4 * NBV: k = (const void*)tall_gemm_kernel<NBV, false, false, false, Tin>; break; \
  case 4 * NBV + 1: k = (const void*)tall_gemm_kernel<NBV, false, true, false, Tin>; break; \
  case 4 * NBV + 2: k = (const void*)tall_gemm_kernel<NBV, true, false, false, Tin>; break; \
  case 4 * NBV + 3: k = (const void*)tall_gemm_kernel<NBV, true, true, false, Tin>; break;
      TG_CASE(1) TG_CASE(2) TG_CASE(3) TG_CASE(4) TG_CASE(5) TG_CASE(6) TG_CASE(7)
#undef TG_CASE
    }
  }
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  TGArgs a = g;
  void* args[] = {(void*)&a};
  return hipLaunchKernel(k, grid, dim3(64 * TG_WAVES), args, lds, s);
}

// core[a + Ra*(i + I*b)] = G2[i + I*(a + Ra*b)]  (inverse of the mode-2 unfolding)
__global__ void core_fold_kernel(const double* G2, int64_t I, int Ra, int Rb, double* core) {
  const int64_t n = I * Ra * Rb;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int a = (int)(e % Ra);
  const int64_t i = (e / Ra) % I;
  const int b = (int)(e / ((int64_t)Ra * I));
  core[e] = G2[i + I * (a + (int64_t)Ra * b)];
}

// A + s*I in place on the diagonal.
__global__ void add_diag_kernel(double* A, int n, const double* s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i + (int64_t)n * i] += *s;
}

// shift for the shifted Cholesky QR: s = 11 (m n + n (n + 1)) u ||A||_F^2, with
// ||A||_F^2 = trace(A^T A).
__global__ void shift_kernel(const double* G, int n, int64_t m, double* s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += G[i + (int64_t)n * i];
    const double u = 1.1102230246251565e-16;
    *s = 11.0 * ((double)m * n + (double)n * (n + 1)) * u * tr;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

bool householder_in_registers(int64_t m, int n) {
  return m <= 256 && n <= 128 && (size_t)(m * std::min<int64_t>(m, n)) * sizeof(double) <= 128 * 1024;
}

hipError_t launch_householder_qr(double* A, int64_t m, int n, double* V, double* tau, double* Q, double* R,
                                 hipStream_t s) {
  const int64_t r = std::min<int64_t>(m, n);
  const size_t lds = (size_t)(m * r) * sizeof(double);
  if (householder_in_registers(m, n)) {   // registers + reflectors in LDS
    const void* k = m <= 64    ? (const void*)householder_qr_reg_kernel<1, 8>
                    : m <= 128 ? (const void*)householder_qr_reg_kernel<2, 8>
                               : (const void*)householder_qr_reg_kernel<4, 8>;
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    const double* Ac = A;
    const int mi = (int)m;
    void* args[] = {(void*)&Ac, (void*)&mi, (void*)&n, (void*)&Q, (void*)&R};
    return hipLaunchKernel(k, dim3(1), dim3(1024), args, lds, s);
  }
  hipLaunchKernelGGL(householder_qr_kernel, dim3(1), dim3(1024), 0, s, A, m, n, V, tau, Q, R);
  return hipGetLastError();
}

// C (P x Q) = A^T B over K rows, ordered split-K; part must hold nchunk*P*Q.
hipError_t launch_tall_atb(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t K, int P, int Q,
                           int mode, int64_t L, int64_t Ip, int64_t T, double* part, int64_t part_elems, double* C,
                           hipStream_t s) {
  TallArgs g;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.K = K; g.P = P; g.Q = Q; g.mode = mode;
  g.L = L; g.Ip = Ip; g.T = T; g.part = part;
  int64_t nchunk = std::min<int64_t>(512, std::max<int64_t>(1, part_elems / ((int64_t)P * Q)));
  nchunk = std::min<int64_t>(nchunk, cdiv(K, 64));
  const bool gram = mode == 0 && A == B && lda == ldb && P == Q;
  const int nb = std::max((P + 15) / 16, (Q + 15) / 16);
  if (gram && nb <= 7 && lda % 2 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0) {   // fragments in registers
    nchunk = std::min<int64_t>(nchunk, 256);
    const int64_t kc = cdiv(cdiv(K, nchunk), 64 * GF_G) * (64 * GF_G);
    nchunk = cdiv(K, kc);
    const size_t lds = (size_t)(nb * (nb + 1) / 2) * 256 * sizeof(double);
    const dim3 grid((unsigned)nchunk);
    switch (nb) {
#define GRAM_FRAG(B) \
  case B: hipLaunchKernelGGL(gram_frag_kernel<B>, grid, dim3(256), lds, s, A, lda, K, P, kc, part); break;
      GRAM_FRAG(1) GRAM_FRAG(2) GRAM_FRAG(3) GRAM_FRAG(4) GRAM_FRAG(5) GRAM_FRAG(6) GRAM_FRAG(7)
#undef GRAM_FRAG
      default: return hipErrorInvalidValue;
    }
    const int64_t n = (int64_t)P * Q;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(cdiv(n, 64)), dim3(256), 0, s, (const double*)part, (int)nchunk, n, C);
    return hipGetLastError();
  }
  // two operands: A strided (plain, a first-mode or last-mode unfolding) or
  // in the Multi-TTM layout
  AtbArgs fa{A, 1, lda, 1, 0, B, ldb, K, 0, P, Q, part};
  bool frag = !gram && nb <= 7 && P > 0 && Q > 0;
  if (mode == 1) {
    if (L == 1) { fa.ks = Ip; fa.ps = 1; }
    else if (T == 1) { fa.ks = 1; fa.ps = L; }
    else if (L < ((int64_t)1 << 31)) { fa.L = L; fa.LIp = L * Ip; fa.ps = L; }
    else frag = false;
  }
  if (frag) {
    nchunk = std::min<int64_t>(nchunk, ATB_CHUNKS);
    fa.kc = cdiv(cdiv(K, nchunk), 16 * ATB_G) * (16 * ATB_G);
    nchunk = cdiv(K, fa.kc);
    const size_t lds = 0;
    const bool bv = ldb % 2 == 0 && K % 2 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
    const dim3 grid((unsigned)nchunk);
    // A with k contiguous (column-major or the Multi-TTM layout): staged
    // through LDS, two workgroups a CU; a row-major A: fragments straight
    // from memory (at 10^6 x 100: L = 10^4 509 against 850 us, L = 100 586
    // against 690, column-major 481 against 870; row-major 640 against 700)
    const bool use_lds = fa.L > 1 || fa.ks == 1;
    if (use_lds) {
      const size_t ldsb = (size_t)4 * 16 * nb * AL_KP * sizeof(double);
      switch (nb * 2 + (fa.L > 1 ? 1 : 0)) {
#define ATB_LDS_CASE(NBV) \
  case 2 * NBV: hipLaunchKernelGGL((atb_lds_kernel<NBV, false>), grid, dim3(256), ldsb, s, fa); break; \
  case 2 * NBV + 1: hipLaunchKernelGGL((atb_lds_kernel<NBV, true>), grid, dim3(256), ldsb, s, fa); break;
        ATB_LDS_CASE(1) ATB_LDS_CASE(2) ATB_LDS_CASE(3) ATB_LDS_CASE(4) ATB_LDS_CASE(5) ATB_LDS_CASE(6) ATB_LDS_CASE(7)
#undef ATB_LDS_CASE
        default: return hipErrorInvalidValue;
      }
      const int64_t n = (int64_t)P * Q;
      hipLaunchKernelGGL(sum_chunks_kernel, dim3(cdiv(n, 64)), dim3(256), 0, s, (const double*)part, (int)nchunk, n,
                         C);
      return hipGetLastError();
    }
    switch (nb * 2 + (bv ? 1 : 0)) {
#define ATB_FRAG(NBV) \
  case 2 * NBV: hipLaunchKernelGGL((atb_frag_kernel<NBV, false>), grid, dim3(256), lds, s, fa); break; \
  case 2 * NBV + 1: hipLaunchKernelGGL((atb_frag_kernel<NBV, true>), grid, dim3(256), lds, s, fa); break;
      ATB_FRAG(1) ATB_FRAG(2) ATB_FRAG(3) ATB_FRAG(4) ATB_FRAG(5) ATB_FRAG(6) ATB_FRAG(7)
#undef ATB_FRAG
      default: return hipErrorInvalidValue;
    }
    const int64_t n = (int64_t)P * Q;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(cdiv(n, 64)), dim3(256), 0, s, (const double*)part, (int)nchunk, n, C);
    return hipGetLastError();
  }
  const size_t lds = (size_t)(gram ? 1 : 2) * nb * 16 * GST * sizeof(double);
  if (nb <= 8 && lds <= 64 * 1024) {   // LDS-staged slabs
    g.kc = cdiv(cdiv(K, nchunk), GKS) * GKS;
    nchunk = cdiv(K, g.kc);
    const dim3 grid((unsigned)nchunk);
    switch (nb * 2 + (gram ? 1 : 0)) {
#define TALL_LDS(B) \
  case 2 * B: hipLaunchKernelGGL((tall_atb_lds_kernel<B, false>), grid, dim3(256), lds, s, g); break; \
  case 2 * B + 1: hipLaunchKernelGGL((tall_atb_lds_kernel<B, true>), grid, dim3(256), lds, s, g); break;
      TALL_LDS(1) TALL_LDS(2) TALL_LDS(3) TALL_LDS(4) TALL_LDS(5) TALL_LDS(6) TALL_LDS(7)
      case 17: hipLaunchKernelGGL((tall_atb_lds_kernel<8, true>), grid, dim3(256), lds, s, g); break;
#undef TALL_LDS
      default: return hipErrorInvalidValue;
    }
    const int64_t n = (int64_t)P * Q;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(cdiv(n, 64)), dim3(256), 0, s, (const double*)part, (int)nchunk, n, C);
    return hipGetLastError();
  }
  g.kc = cdiv(cdiv(K, nchunk), 4) * 4;
  nchunk = cdiv(K, g.kc);
  switch ((Q + 15) / 16) {   // register-blocked for Q <= 128
#define TALL_CASE(B) \
  case B: hipLaunchKernelGGL(tall_atb_rb_kernel<B>, dim3((unsigned)nchunk), dim3(256), 0, s, g); break;
    TALL_CASE(1) TALL_CASE(2) TALL_CASE(3) TALL_CASE(4) TALL_CASE(5) TALL_CASE(6) TALL_CASE(7) TALL_CASE(8)
#undef TALL_CASE
    default: hipLaunchKernelGGL(tall_atb_kernel, dim3((unsigned)nchunk), dim3(256), 0, s, g); break;
  }
  const int64_t n = (int64_t)P * Q;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(cdiv(n, 64)), dim3(256), 0, s, (const double*)part, (int)nchunk, n, C);
  return hipGetLastError();
}

hipError_t launch_ttm(const void* in, int in_type, int64_t L, int64_t I, int64_t T, const double* Q, int R,
                      double scale, double* out, hipStream_t s) {
  if (I <= 112 && R <= 112 && (L == 1 || L >= 16)) {   // MFMA tiles
    TGArgs g;
    if (L == 1) g = TGArgs{in, I, 1, 0, T, (int)I, Q, (int)I, R, out, R, 1, 0, 1, scale};
    else g = TGArgs{in, 1, L, L * I, L, (int)I, Q, (int)I, R, out, 1, L, L * R, T, scale};
    switch (in_type) {
      case TR_F64: return launch_tg<double>(g, s);
      case TR_F32: return launch_tg<float>(g, s);
      case TR_BF16: return launch_tg<__bf16>(g, s);
      default: return launch_tg<uint8_t>(g, s);
    }
  }
  const size_t lds = (size_t)I * TRB * sizeof(double);
  if (lds <= 64 * 1024) {
    const dim3 grid((unsigned)std::min<int64_t>(cdiv(L * T, 256), 16384), (unsigned)cdiv(R, TRB));
    switch (in_type) {
      case TR_F64: hipLaunchKernelGGL(ttm_rb_kernel<double>, grid, dim3(256), lds, s, (const double*)in, L, I, T, Q, R, scale, out); break;
      case TR_F32: hipLaunchKernelGGL(ttm_rb_kernel<float>, grid, dim3(256), lds, s, (const float*)in, L, I, T, Q, R, scale, out); break;
      case TR_BF16: hipLaunchKernelGGL(ttm_rb_kernel<__bf16>, grid, dim3(256), lds, s, (const __bf16*)in, L, I, T, Q, R, scale, out); break;
      default: hipLaunchKernelGGL(ttm_rb_kernel<uint8_t>, grid, dim3(256), lds, s, (const uint8_t*)in, L, I, T, Q, R, scale, out); break;
    }
    return hipGetLastError();
  }
  const int64_t n = L * R * T;
  const int64_t grid = std::min<int64_t>(cdiv(n, 256), 65536);
  switch (in_type) {
    case TR_F64: hipLaunchKernelGGL(ttm_kernel<double>, dim3(grid), dim3(256), 0, s, (const double*)in, L, I, T, Q, R, scale, out); break;
    case TR_F32: hipLaunchKernelGGL(ttm_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)in, L, I, T, Q, R, scale, out); break;
    case TR_BF16: hipLaunchKernelGGL(ttm_kernel<__bf16>, dim3(grid), dim3(256), 0, s, (const __bf16*)in, L, I, T, Q, R, scale, out); break;
    default: hipLaunchKernelGGL(ttm_fp8_kernel, dim3(grid), dim3(256), 0, s, (const uint8_t*)in, L, I, T, Q, R, scale, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_sum_chunks(const double* part, int nchunk, int64_t n, double* C, hipStream_t s) {
  if (nchunk < 1 || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)cdiv(n, 64)), dim3(256), 0, s, part, nchunk, n, C);
  return hipGetLastError();
}

hipError_t launch_slice_transpose(const double* in, int64_t L, int64_t I, int64_t T, double* out, hipStream_t s) {
  const int64_t tiles = cdiv(L, 32) * cdiv(I, 32);
  if (L < 1 || I < 1 || T < 1 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(slice_transpose_kernel, dim3((unsigned)tiles, (unsigned)std::min<int64_t>(T, 65535)), dim3(256), 0,
                     s, in, L, I, T, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* A, int64_t rows, int64_t cols, double* At, hipStream_t s) {
  hipLaunchKernelGGL(transpose_kernel, dim3(cdiv(rows * cols, 256)), dim3(256), 0, s, A, rows, cols, At);
  return hipGetLastError();
}

hipError_t launch_table_to_v2(const double* T, int64_t J, int64_t L, int Ra, int Rb, double* V2, hipStream_t s) {
  if (L <= 0 || J % L != 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)V2T_ROWS * (Ra * Rb + 1) * sizeof(double);
  if (lds <= 64 * 1024) {
    hipLaunchKernelGGL(table_to_v2_tiled_kernel, dim3((unsigned)cdiv(J, V2T_ROWS)), dim3(256), lds, s, T, J, L, Ra, Rb,
                       V2);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(table_to_v2_kernel, dim3(cdiv(J * Ra * Rb, 256)), dim3(256), 0, s, T, J, L, Ra, Rb, V2);
  return hipGetLastError();
}

hipError_t launch_v2_direct(const double* Tp, int64_t Jp, const double* core, int64_t I, int Rm, int Ra, int Rb,
                            int64_t L, double* V2, hipStream_t s) {
  const int64_t J = Jp * I;
  if (Jp <= 0 || I <= 0 || Rm <= 0 || Ra <= 0 || Rb <= 0 || L <= 0 || J % L != 0) return hipErrorInvalidValue;
  if (!v2_direct_fits(Rm, Ra, Rb)) return hipErrorInvalidValue;
  const size_t row_bytes = (size_t)((Rb * Rm + Rm * Ra) | 1) * sizeof(double);
  // 16 rows a block: six blocks a CU keep more rows' loads in flight than
  // three of 32 rows (10^6 x 100: 460-560 us against 570-700 us; 8 rows
  // 490-580 us, 64 rows 1440-1680 us)
  int rows = 16;
  while (rows > 1 && rows * row_bytes > 60 * 1024) rows /= 2;
  hipLaunchKernelGGL(v2_direct_kernel, dim3((unsigned)cdiv(J, rows)), dim3(256), rows * row_bytes, s, Tp, Jp, core, I,
                     Rm, Ra, Rb, L, rows, V2);
  return hipGetLastError();
}

hipError_t launch_core_fold(const double* G2, int64_t I, int Ra, int Rb, double* core, hipStream_t s) {
  hipLaunchKernelGGL(core_fold_kernel, dim3(cdiv(I * Ra * Rb, 256)), dim3(256), 0, s, G2, I, Ra, Rb, core);
  return hipGetLastError();
}

hipError_t launch_shift_and_add(double* G, int n, int64_t m, double* sbuf, hipStream_t s) {
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(64), 0, s, (const double*)G, n, m, sbuf);
  hipLaunchKernelGGL(add_diag_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, G, n, (const double*)sbuf);
  return hipGetLastError();
}

hipError_t launch_tall_gemm(const double* A, int64_t lda, int64_t M, int K, const double* B, int ldb, int N,
                            double* C, int64_t ldc, hipStream_t s, bool b_upper) {
  TGArgs g{A, 1, lda, 0, M, K, B, ldb, N, C, 1, ldc, 0, 1, 1.0};
  return launch_tg<double>(g, s, b_upper);
}
