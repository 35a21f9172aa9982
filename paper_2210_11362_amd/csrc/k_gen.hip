// Device generation of planted TR tensors for the serving loop: standard
// normals from the counter-based Philox4x32-10 generator (Salmon, Moraes,
// Dror, Shaw, SC'11) with the Box-Muller transform, the tensor X_true = TR(G)
// reconstructed tile by tile as X_[1] = G_1(2) (G^{!=1}_[2])^T on FP64 MFMA,
// and relative noise X = X_true + eta (|X_true| / |N|) N (the paper's synthetic
// data recipe, Sec. 4).
#include <algorithm>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

__device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

// Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the two
// round constants, swaps the halves around and xors in the key, which is
// bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = mulhi32(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = mulhi32(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// Normal number e of stream `sid` under key `seed`.  Normals come in pairs:
// pair p = e/2 is drawn from the counter (p mod 2^32, p / 2^32, sid, 0); two
// 53-bit uniforms u, v in (0,1) from words (0,1) and (2,3); element 2p is
// sqrt(-2 ln u) cos(2 pi v), element 2p+1 the same with sin.
__device__ __forceinline__ double philox_normal(uint64_t e, uint64_t seed, uint32_t sid) {
  const uint64_t p = e >> 1;
  uint32_t c[4] = {(uint32_t)p, (uint32_t)(p >> 32), sid, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((((uint64_t)c[3]) << 32) | c[2]) >> 11;
  const double u = ((double)a + 0.5) * 0x1p-53;
  const double v = ((double)b + 0.5) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u));
  const double t = 6.283185307179586 * v;
  return (e & 1) ? r * sin(t) : r * cos(t);
}

__global__ __launch_bounds__(256) void philox_normal_kernel(double* out, int64_t n, uint64_t seed, uint32_t sid) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    out[e] = philox_normal((uint64_t)e, seed, sid);
}

__device__ __forceinline__ void mma64(f64x4& acc, double a, double b) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T cast_out(double x) { return (T)x; }

// Pass 1: X_true tiles.  Per tile of KT columns k (modes 2..N), the subchain
// rows B[k, (a,b)] = F1[f1(k)] F2[f2(k)] go to LDS; then 16x16 output blocks
// X[i, k] = sum_c G0[i, c] B[k, c] come from the FP64 MFMA with the k block as
// the row operand, so that the 16 lanes of a row group hold 16 consecutive i
// (contiguous in X).  Each block also sums |X_true|^2 and, with noise, the
// squares of the noise numbers of its elements.
template <typename T>
__global__ __launch_bounds__(256) void gen_pass1_kernel(T* X, int64_t I, int64_t K, const double* G0, const double* F1,
                                                       const double* F2, int64_t d1, int64_t m1, int64_t d2,
                                                       int64_t m2, int Rb, int Rmid, int Ra, int KT, uint64_t seed,
                                                       int with_noise, double* part_t, double* part_n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int RR = Ra * Rb;
  const int RR4 = (RR + 3) & ~3;
  double* Bs = reinterpret_cast<double*>(smem_raw);  // [KT][RR4 + 1]
  const int BST = RR4 + 1;
  __shared__ double red_t[256], red_n[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ntile = (K + KT - 1) / KT;
  const int nbr = (int)((I + 15) / 16);
  double st = 0.0, sn = 0.0;
  for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int64_t k0 = t * KT;
    const int kvalid = (int)min((int64_t)KT, K - k0);
    __syncthreads();
    for (int e = tid; e < KT * BST; e += 256) {
      const int kk = e / BST, c = e % BST;
      double s = 0.0;
      if (kk < kvalid && c < RR) {
        const int64_t k = k0 + kk;
        const double* f1 = F1 + ((k / d1) % m1) * (int64_t)(Rb * Rmid);
        const double* f2 = F2 + ((k / d2) % m2) * (int64_t)(Rmid * Ra);
        const int aa = c % Ra, b = c / Ra;
        for (int m = 0; m < Rmid; ++m) s += f1[b + Rb * m] * f2[m + Rmid * aa];
      }
      Bs[e] = s;
    }
    __syncthreads();
    const int ncb = KT / 16;
    for (int ob = wave; ob < nbr * ncb; ob += 4) {
      const int br = ob / ncb, bc = ob % ncb;
      const int64_t i = (int64_t)br * 16 + (lane & 15);
      const int kka = bc * 16 + (lane & 15);
      f64x4 acc = {0, 0, 0, 0};
      for (int c0 = 0; c0 < RR4; c0 += 4) {
        const int c = c0 + (lane >> 4);
        const double av = Bs[kka * BST + c];
        const double bv = (i < I && c < RR) ? G0[i + I * c] : 0.0;
        mma64(acc, av, bv);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int kk = bc * 16 + (lane >> 4) + 4 * v;
        if (i < I && kk < kvalid) {
          const double x = acc[v];
          const int64_t e = i + I * (k0 + kk);
          X[e] = cast_out<T>(x);
          st += x * x;
          if (with_noise) {
            const double z = philox_normal((uint64_t)e, seed, 0u);
            sn += z * z;
          }
        }
      }
    }
  }
  red_t[tid] = st;
  red_n[tid] = sn;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) { red_t[tid] += red_t[tid + w]; red_n[tid] += red_n[tid + w]; }
    __syncthreads();
  }
  if (tid == 0) { part_t[blockIdx.x] = red_t[0]; part_n[blockIdx.x] = red_n[0]; }
}

// Ordered sums of the block partials and the noise scale eta |X_true| / |N|.
__global__ void gen_finish_kernel(const double* part_t, const double* part_n, int n, double eta, double* scal) {
  if (threadIdx.x != 0) return;
  double st = 0.0, sn = 0.0;
  for (int b = 0; b < n; ++b) { st += part_t[b]; sn += part_n[b]; }
  scal[0] = st;
  scal[1] = sn;
  scal[2] = sn > 0.0 ? eta * sqrt(st) / sqrt(sn) : 0.0;
}

// Pass 2: X = X + scale N, element by element in X's type.
template <typename T>
__global__ __launch_bounds__(256) void gen_pass2_kernel(T* X, int64_t n, uint64_t seed, const double* scal) {
  const double sc = scal[2];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    X[e] = cast_out<T>((double)X[e] + sc * philox_normal((uint64_t)e, seed, 0u));
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_philox_normal(double* out, int64_t n, uint64_t seed, uint32_t sid, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = std::min<int64_t>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(philox_normal_kernel, dim3((unsigned)grid), dim3(256), 0, s, out, n, seed, sid);
  return hipGetLastError();
}

hipError_t launch_gen_planted(void* X, int xdt, int64_t I, int64_t K, const double* G0, const double* F1,
                              const double* F2, int64_t d1, int64_t m1, int64_t d2, int64_t m2, int Rb, int Rmid,
                              int Ra, uint64_t seed, double eta, double* partials, int nblk, double* scal,
                              hipStream_t s) {
  const int RR4 = (Ra * Rb + 3) & ~3;
  const int kt = RR4 > 448 ? 16 : 32;
  const size_t lds = (size_t)kt * (RR4 + 1) * sizeof(double);
  const int noise = eta != 0.0 ? 1 : 0;
  double* pt = partials;
  double* pn = partials + nblk;
  LDSCHK((const void*)gen_pass1_kernel<double>, lds);
  LDSCHK((const void*)gen_pass1_kernel<float>, lds);
  const int64_t n = I * K;
  const int64_t grid2 = std::min<int64_t>(cdiv(n, 256), 16384);
  if (xdt == TR_F64) {
    hipLaunchKernelGGL(gen_pass1_kernel<double>, dim3(nblk), dim3(256), lds, s, (double*)X, I, K, G0, F1, F2, d1, m1,
                       d2, m2, Rb, Rmid, Ra, kt, seed, noise, pt, pn);
    hipLaunchKernelGGL(gen_finish_kernel, dim3(1), dim3(64), 0, s, pt, pn, nblk, eta, scal);
    if (noise)
      hipLaunchKernelGGL(gen_pass2_kernel<double>, dim3((unsigned)grid2), dim3(256), 0, s, (double*)X, n, seed,
                         (const double*)scal);
  } else {
    hipLaunchKernelGGL(gen_pass1_kernel<float>, dim3(nblk), dim3(256), lds, s, (float*)X, I, K, G0, F1, F2, d1, m1,
                       d2, m2, Rb, Rmid, Ra, kt, seed, noise, pt, pn);
    hipLaunchKernelGGL(gen_finish_kernel, dim3(1), dim3(64), 0, s, pt, pn, nblk, eta, scal);
    if (noise)
      hipLaunchKernelGGL(gen_pass2_kernel<float>, dim3((unsigned)grid2), dim3(256), 0, s, (float*)X, n, seed,
                         (const double*)scal);
  }
  return hipGetLastError();
}
