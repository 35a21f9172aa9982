// Two by-products of the ALS intermediates (Sec. 3.4 and Sec. 4):
//  * the cheap in-loop error: after the update of mode N,
//      ||X - Xhat||^2 = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2,
//    with <X, Xhat> = <M_N, G_N(2)> and ||Xhat||^2 = <S_N<2>, G_N(2)^T G_N(2)>
//    (normal-equation variants; QRNE's M_N = Y_[N] V_N[2] and S_N from the
//    R-core Grams give the same two numbers), or, for the QR variant,
//    <X, Xhat> = <W_N, G_N(2) R_[2]^T> and ||Xhat||^2 = ||G_N(2) R_[2]^T||^2;
//  * the inner product of two tensors in TR format: with the transfer matrices
//    T_k[(a,a'),(b,b')] = sum_i A_k(a,i,b) B_k(a',i,b'), <A, B> is the trace of
//    T_1 T_2 ... T_N (the pair-space trace of the Gram-tensor chain).
// Everything in FP64; every reduction in a fixed order (deterministic).
#include <algorithm>

#include "common.h"

namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int CF_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = CF_THREADS / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Rows i = blockIdx.x, blockIdx.x + gridDim.x, ... of the I x n matrices A
// (M_N or W_N) and G (G_N(2)), column-major.  mode 0: z = g S (S symmetric
// n x n), a += <A_i, g>, b += <g, z>.  mode 1: z = g L with L = R_[2]^T lower
// triangular, a += <A_i, z>, b += <z, z>.  partials[2 blk] = a, [2 blk + 1] = b.
__global__ __launch_bounds__(CF_THREADS) void cheap_fit_kernel(const double* A, const double* G, const double* B,
                                                                int mode, int64_t I, int n, double* partials) {
  extern __shared__ double g[];   // one row of G
  __shared__ double red[CF_THREADS];
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x; i < I; i += gridDim.x) {
    for (int j = threadIdx.x; j < n; j += CF_THREADS) g[j] = G[i + I * j];
    __syncthreads();
    double pa = 0.0, pb = 0.0;
    for (int j = threadIdx.x; j < n; j += CF_THREADS) {
      const double* col = B + (int64_t)n * j;
      double z = 0.0;
      if (mode == 0) {
        for (int k = 0; k < n; ++k) z = fma(g[k], col[k], z);
        pa = fma(A[i + I * j], g[j], pa);
        pb = fma(g[j], z, pb);
      } else {
        for (int k = j; k < n; ++k) z = fma(g[k], col[k], z);
        pa = fma(A[i + I * j], z, pa);
        pb = fma(z, z, pb);
      }
    }
    a += block_sum(pa, red);
    b += block_sum(pb, red);
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}

// out[0] = ||X||^2 - 2 a + b from the block partials (in block order), out[1] = a, out[2] = b
__global__ void cheap_fit_finish_kernel(const double* partials, int nblk, const double* xnorm2, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
      a += partials[2 * k];
      b += partials[2 * k + 1];
    }
    out[0] = *xnorm2 - 2.0 * a + b;
    out[1] = a;
    out[2] = b;
  }
}

// E (RaRb x SaSb, rows a + Ra b, columns a' + Sa b') -> T ((Ra Sa) x (Rb Sb),
// rows a + Ra a', columns b + Rb b').
__global__ void transfer_from_cross_gram_kernel(const double* E, int Ra, int Rb, int Sa, int Sb, double* T) {
  const int64_t n = (int64_t)Ra * Rb * Sa * Sb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rows = (int64_t)Ra * Sa;
    const int64_t r = e % rows, c = e / rows;
    const int a = (int)(r % Ra), ap = (int)(r / Ra);
    const int bb = (int)(c % Rb), bp = (int)(c / Rb);
    T[e] = E[(a + (int64_t)Ra * bb) + (int64_t)Ra * Rb * (ap + (int64_t)Sa * bp)];
  }
}

__global__ void trace_kernel(const double* P, int64_t n, double* out) {
  __shared__ double red[CF_THREADS];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += CF_THREADS) s += P[i + n * i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

}  // namespace

int cheap_fit_blocks(int64_t I) { return (int)std::min<int64_t>(std::max<int64_t>(I, 1), 512); }

hipError_t launch_cheap_fit(const double* A, const double* G, const double* B, int mode, int64_t I, int n,
                            const double* xnorm2, double* partials, double* out, hipStream_t s) {
  const int nblk = cheap_fit_blocks(I);
  const size_t lds = (size_t)n * sizeof(double);
  hipLaunchKernelGGL(cheap_fit_kernel, dim3(nblk), dim3(CF_THREADS), lds, s, A, G, B, mode, I, n, partials);
  hipLaunchKernelGGL(cheap_fit_finish_kernel, dim3(1), dim3(64), 0, s, (const double*)partials, nblk, xnorm2, out);
  return hipGetLastError();
}

hipError_t launch_transfer_from_cross_gram(const double* E, int Ra, int Rb, int Sa, int Sb, double* T,
                                           hipStream_t s) {
  const int64_t n = (int64_t)Ra * Rb * Sa * Sb;
  hipLaunchKernelGGL(transfer_from_cross_gram_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)),
                     dim3(256), 0, s, E, Ra, Rb, Sa, Sb, T);
  return hipGetLastError();
}

hipError_t launch_trace(const double* P, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(CF_THREADS), 0, s, P, n, out);
  return hipGetLastError();
}
