// Pseudo-inverse of a small square FP64 matrix by the one-sided Jacobi SVD
// (Hestenes): the rank-deficient-safe solve of the mode update (the remark
// after Alg. 3: solve through an SVD when the coefficient matrix is rank
// deficient).  For the normal equations A = S_n (symmetric positive
// semidefinite); singular values at or below rcond * sigma_max count as zero,
// so G = M A^+ is the minimum-norm least-squares update.
//
// One workgroup.  U (a copy of A, rotated) and V (accumulated rotations) live
// in a global work buffer (2 n^2 doubles, L2-resident at these sizes).  Every
// round of the round-robin ordering rotates n/2 disjoint column pairs, one
// pair per wave at a time; a barrier separates rounds.  Sweeps repeat until a
// whole sweep rotates nothing (or 40 sweeps).  The order of every reduction is
// fixed: the result is deterministic.
#include <algorithm>

#include "common.h"

namespace {

constexpr int PJ_THREADS = 1024;
constexpr int PJ_WAVES = PJ_THREADS / 64;
constexpr int PJ_MAX_SWEEPS = 40;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// player k of round r of the round-robin schedule over m (even) players:
// player m-1 stays, the others rotate
__device__ __forceinline__ int rr_player(int k, int r, int m) {
  if (k == m - 1) return m - 1;
  return (k + r) % (m - 1);
}

__global__ __launch_bounds__(PJ_THREADS) void pinv_jacobi_kernel(const double* A, int n, double rcond, double* Apinv,
                                                                 double* work, int* status) {
  double* U = work;                 // n x n, column-major
  double* V = work + (size_t)n * n;
  __shared__ int rotated;
  __shared__ double sigma[1024];
  __shared__ double smax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t e = tid; e < (int64_t)n * n; e += PJ_THREADS) {
    U[e] = A[e];
    V[e] = (e % n) == (e / n) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m = n + (n & 1);        // players; an odd n gets a dummy column n
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < PJ_MAX_SWEEPS; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int pr = wave; pr < m / 2; pr += PJ_WAVES) {
        int p = rr_player(pr, r, m), q = rr_player(m - 1 - pr, r, m);
        if (p > q) { const int t = p; p = q; q = t; }
        if (q >= n) continue;       // the dummy column
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double up = U[i + (int64_t)n * p], uq = U[i + (int64_t)n * q];
          a = fma(up, up, a);
          b = fma(uq, uq, b);
          g = fma(up, uq, g);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        g = wave_sum(g);
        if (fabs(g) <= eps * sqrt(a * b) || g == 0.0) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < n; i += 64) {
          const double up = U[i + (int64_t)n * p], uq = U[i + (int64_t)n * q];
          U[i + (int64_t)n * p] = c * up - s * uq;
          U[i + (int64_t)n * q] = s * up + c * uq;
          const double vp = V[i + (int64_t)n * p], vq = V[i + (int64_t)n * q];
          V[i + (int64_t)n * p] = c * vp - s * vq;
          V[i + (int64_t)n * q] = s * vp + c * vq;
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // sigma_j = |U_j|; the columns of U / sigma are the left singular vectors
  for (int j = wave; j < n; j += PJ_WAVES) {
    double s2 = 0.0;
    for (int i = lane; i < n; i += 64) s2 = fma(U[i + (int64_t)n * j], U[i + (int64_t)n * j], s2);
    s2 = wave_sum(s2);
    if (lane == 0) sigma[j] = sqrt(s2);
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    bool finite = true;
    for (int j = 0; j < n; ++j) {
      mx = fmax(mx, sigma[j]);
      finite = finite && isfinite(sigma[j]);
    }
    smax = mx;
    if (!finite) atomicOr(status, ST_NONFINITE);
  }
  __syncthreads();
  const double thr = rcond * smax;
  // A^+ = sum_j v_j (1 / sigma_j^2) (U_j)^T, with U_j = sigma_j u_j unnormalised
  for (int64_t e = tid; e < (int64_t)n * n; e += PJ_THREADS) {
    const int i = (int)(e % n), k = (int)(e / n);
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      const double sj = sigma[j];
      if (sj > thr && sj > 0.0) acc = fma(V[i + (int64_t)n * j] / (sj * sj), U[k + (int64_t)n * j], acc);
    }
    Apinv[e] = acc;
  }
}

}  // namespace

bool pinv_fits(int n) { return n >= 1 && n <= 1024; }

hipError_t launch_pinv(const double* A, int n, double rcond, double* Apinv, double* work, int* status,
                       hipStream_t s) {
  hipLaunchKernelGGL(pinv_jacobi_kernel, dim3(1), dim3(PJ_THREADS), 0, s, A, n, rcond, Apinv, work, status);
  return hipGetLastError();
}
