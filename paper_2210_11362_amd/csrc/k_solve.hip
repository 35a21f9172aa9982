// FP64 normal-equation solve G S = M with S = L L^T (Alg. 2's solve step):
// a blocked Cholesky in one workgroup (matrix in LDS) and a blocked
// forward/backward substitution that runs 16 right-hand sides per workgroup
// with L staged in LDS.  A non-positive or non-finite pivot latches
// ST_SINGULAR; later steps see the status word and leave their outputs alone.
#include <type_traits>
#include <utility>

#include <algorithm>

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

// Right-looking blocked Cholesky.  The matrix is padded in LDS to np (a
// multiple of NB) with an identity block, so every block has NB columns and
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

// Lane exchanges of a double within a wave64.
template <int P> __device__ __forceinline__ double row_bcast(double x) {   // lane (l & ~15) | P
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, 0x150 + P, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0x150 + P, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_get(double x, int src) {             // lane src (any)
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)u);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_uniform(double x, int src) {         // lane src, as a scalar
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_readlane((int)u, src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ f64x4 mma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

constexpr int PST = 17;   // panel row stride in doubles (odd: spreads rows over the LDS banks)

// S^{-1} of a symmetric positive definite S (n <= 16 * NBT) by the symmetric
// sweep operator.  Sweeping pivot k of A sets
//   A_ij -= A_ik A_kj / A_kk  (i, j != k),  A_ik = A_ik / A_kk,  A_kj = A_kj / A_kk,  A_kk = -1 / A_kk,
// and sweeping every pivot of S leaves -S^{-1}.  Sweeping the 16 pivots of a
// diagonal block D = A_kk at once is the block form
//   A_ij -= A_ik D^{-1} A_kj,  A_ik = A_ik D^{-1},  A_kj = D^{-1} A_kj,  A_kk = -D^{-1},
// which is what this kernel does, block by block.  For SPD S every scalar
// pivot met inside D is a Schur-complement diagonal, hence positive; one that
// is not (S not positive definite in working precision) latches ST_SINGULAR.
//
// One workgroup of NW waves.  The lower block triangle lives in registers
// as 16x16 FP64 MFMA accumulator tiles (lane l, element v holds row
// (l >> 4) + 4v, column l & 15); with four waves wave W owns block rows W and
// NBT-1-W, with eight waves block row W alone (used for eight block rows,
// where the four-wave form spills heavily; at seven it spills a little and
// still measures faster: 27 us against 33 us at n = 100), fixed at compile
// time so that each wave's update is straight-line MFMA code.  Per
// block step the owners publish block column k to LDS (one barrier); every
// wave then sweeps D in its own registers (pivot column by DPP row broadcast,
// pivot row by bpermute, no barrier) and applies the block update to its
// tiles.  D^{-1} is symmetric, so the same registers serve as its A-operand
// and B-operand fragments, and (-D^{-1}) A_kr computed in the accumulator
// layout is already the A-operand of -A_rk D^{-1}.
template <int NBT, int NW, int W>
__device__ __forceinline__ void spd_block_inv_wave(const double* __restrict__ S, int n, double* __restrict__ Sinv,
                                                   int* status, double* panel, int lane) {
  constexpr int NP = 16 * NBT;
  constexpr int ROW[2] = {W, NW == 4 ? NBT - 1 - W : NBT};
  constexpr bool HAS[2] = {W < NBT, NW == 4 && NBT - 1 - W > W};
  constexpr int MAXR = HAS[1] ? ROW[1] : HAS[0] ? ROW[0] : -1;   // highest block row owned
  const int g = lane >> 4, c16 = lane & 15;
  f64x4 t[2][NBT];
  static_for<0, 2>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    if constexpr (HAS[s]) {
#pragma unroll
      for (int c = 0; c <= ROW[s]; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ROW[s] + g + 4 * v, j = 16 * c + c16;   // padded to the identity
          const double x = S[min(i, n - 1) + (int64_t)n * min(j, n - 1)];
          t[s][c][v] = (i < n && j < n) ? x : (i == j ? 1.0 : 0.0);
        }
    }
  });
  // block column k of the current matrix: P[i][q] = A(i, 16k + q), from the
  // tiles (r, k), r >= k, and (by symmetry) the tiles (k, c), c < k
  auto publish = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double* P = panel + (k & 1) * NP * PST;
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value, r = ROW[s];
      if constexpr (HAS[s] && r >= k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(16 * r + g + 4 * v) * PST + c16] = t[s][k][v];
      }
      if constexpr (HAS[s] && r == k) {
#pragma unroll
        for (int c = 0; c < k; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) P[(16 * c + c16) * PST + g + 4 * v] = t[s][c][v];
      }
    });
  };
  bool stop = false;
  auto step = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (stop) return;
    __syncthreads();
    const double* P = panel + (k & 1) * NP * PST;
    // D (lower triangle mirrored) in the accumulator layout, swept in place to -D^{-1}
    double a[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = g + 4 * v;
      const double lo = P[(16 * k + row) * PST + c16], up = P[(16 * k + c16) * PST + row];
      a[v] = row >= c16 ? lo : up;
    }
    bool bad = false;
    static_for<0, 16>([&](auto pc) {
      constexpr int p = decltype(pc)::value, pv = p >> 2, pg = p & 3;
      const double app = lane_uniform(a[pv], (pg << 4) | p);
      bad |= !(app > 0.0) || !isfinite(app);
      const double rp = pivot_recip(app);
      double colv[4];   // A(g + 4v, p): lane p of this lane's 16-lane row
#pragma unroll
      for (int v = 0; v < 4; ++v) colv[v] = row_bcast<p>(a[v]);
      const double rowv = lane_get(a[pv], (pg << 4) | c16);   // A(p, c16)
      // column p: A(i, p) / A_pp; row p: A(p, j) / A_pp; diagonal: -1 / A_pp
      const bool colp = c16 == p;
      const double tsel = colp ? -rp : rowv * rp;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double nv = fma(-colv[v], tsel, colp ? 0.0 : a[v]);
        if (g + 4 * v == p) nv = tsel;
        a[v] = nv;
      }
      __builtin_amdgcn_sched_barrier(0);   // one pivot at a time: keeps the live ranges short
    });
    // the same pivots in every wave: uniform exit
    if (__builtin_amdgcn_readfirstlane((int)bad)) {
      if (W == 0 && lane == 0) atomicOr(status, ST_SINGULAR);
      stop = true;
      return;
    }
    __builtin_amdgcn_sched_barrier(0);
    // B-operand fragments of block column k: A_kc(4q + g, c16) = A(16c + c16, 16k + 4q + g)
    auto frag = [&](int c, double* f) {
#pragma unroll
      for (int q = 0; q < 4; ++q) f[q] = P[(16 * c + c16) * PST + 4 * q + g];
    };
    // per owned row r: its fragments and (-D^{-1}) A_kr, whose element q is the
    // A-operand fragment q of -A_rk D^{-1}
    double pr[2][4];
    f64x4 nw[2];
    static_for<0, 2>([&](auto sc) {
      constexpr int s = decltype(sc)::value, r = ROW[s];
      if constexpr (HAS[s]) {
        frag(r, pr[s]);
        nw[s] = f64x4{0, 0, 0, 0};
        if constexpr (r != k) {
#pragma unroll
          for (int q = 0; q < 4; ++q) nw[s] = mma64(a[q], pr[s][q], nw[s]);
        }
      }
    });
    // column by column, both owned rows
    static_for<0, MAXR + 1>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      double pc[4];
      frag(c, pc);
      static_for<0, 2>([&](auto sc) {
        constexpr int s = decltype(sc)::value, r = ROW[s];
        if constexpr (HAS[s] && c <= r) {
          if constexpr (r == k && c == k) {
#pragma unroll
            for (int v = 0; v < 4; ++v) t[s][c][v] = a[v];
          } else if constexpr (r == k) {            // A_kc <- D^{-1} A_kc
            f64x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) acc = mma64(a[q], pc[q], acc);
            t[s][c] = -acc;
          } else if constexpr (c == k) {            // A_rk <- A_rk D^{-1}
            f64x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) acc = mma64(pr[s][q], a[q], acc);
            t[s][c] = -acc;
          } else {                                  // A_rc <- A_rc - A_rk D^{-1} A_kc
#pragma unroll
            for (int q = 0; q < 4; ++q) t[s][c] = mma64(nw[s][q], pc[q], t[s][c]);
          }
        }
      });
    });
    if constexpr (k + 1 < NBT) publish(std::integral_constant<int, k + 1>{});
  };
  publish(std::integral_constant<int, 0>{});
  static_for<0, NBT>(step);
  if (stop) return;
  // -A = S^{-1}: write both triangles from the lower entries
  static_for<0, 2>([&](auto sc) {
    constexpr int s = decltype(sc)::value, r = ROW[s];
    if constexpr (HAS[s]) {
#pragma unroll
      for (int c = 0; c <= r; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * r + g + 4 * v, j = 16 * c + c16;
          if (i < n && j <= i) {
            const double val = -t[s][c][v];
            Sinv[i + (int64_t)n * j] = val;
            Sinv[j + (int64_t)n * i] = val;
          }
        }
    }
  });
}

template <int NBT, int NW>
__global__ __launch_bounds__(NW * 64) void spd_block_inv_kernel(const double* __restrict__ S, int n,
                                                                double* __restrict__ Sinv, int* status) {
  __shared__ double panel[2 * 16 * NBT * PST];
  if (*status != 0) return;
  const int lane = threadIdx.x & 63;
  switch (__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) {   // wave index, uniform per wave
    case 0: spd_block_inv_wave<NBT, NW, 0>(S, n, Sinv, status, panel, lane); break;
    case 1: spd_block_inv_wave<NBT, NW, 1>(S, n, Sinv, status, panel, lane); break;
    case 2: spd_block_inv_wave<NBT, NW, 2>(S, n, Sinv, status, panel, lane); break;
    case 3: spd_block_inv_wave<NBT, NW, 3>(S, n, Sinv, status, panel, lane); break;
    case 4: if constexpr (NW == 8) spd_block_inv_wave<NBT, NW, 4>(S, n, Sinv, status, panel, lane); break;
    case 5: if constexpr (NW == 8) spd_block_inv_wave<NBT, NW, 5>(S, n, Sinv, status, panel, lane); break;
    case 6: if constexpr (NW == 8) spd_block_inv_wave<NBT, NW, 6>(S, n, Sinv, status, panel, lane); break;
    default: if constexpr (NW == 8) spd_block_inv_wave<NBT, NW, 7>(S, n, Sinv, status, panel, lane); break;
  }
}

}  // namespace

// LDS-resident versions for n <= 128; larger systems use the global-memory
// Cholesky and the one-wave-per-row solve.
bool solve_in_lds(int n) { return n <= 128; }

hipError_t launch_chol_lds(const double* S, int n, double* L, double* LT, double* rdiag, int* status, hipStream_t s) {
  const int np = (n + NB - 1) / NB * NB;
  const size_t lds = (size_t)np * np * sizeof(double);
  if (lds > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute((const void*)chol_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(chol_lds_kernel, dim3(1), dim3(256), lds, s, S, n, L, LT, status, rdiag);
  return hipGetLastError();
}

hipError_t launch_trsm_rhs(const double* L, const double* rdiag, int n, const double* Rhs, int64_t I, double* G,
                           int accumulate, const int* status, hipStream_t s, int mode) {
  const int np = (n + NB - 1) / NB * NB;
  const size_t lds = ((size_t)np * np + (size_t)NRHS * np) * sizeof(double);
  if (lds > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute((const void*)trsm_rhs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(trsm_rhs_kernel, dim3((unsigned)((I + NRHS - 1) / NRHS)), dim3(256), lds, s, L, rdiag, n, Rhs,
                     I, G, accumulate, status, mode);
  return hipGetLastError();
}

namespace {
// dst[r + ldd c] = src[r + lds c] (trans: src[c + lds r]; src == nullptr: 0;
// add: dst += the value)
__global__ void copy_block_kernel(const double* src, int64_t lds_, int rows, int cols, double* dst, int64_t ldd,
                                  int trans, int add) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % rows, c = e / rows;
    const double v = src ? (trans ? src[c + lds_ * r] : src[r + lds_ * c]) : 0.0;
    dst[r + ldd * c] = add ? dst[r + ldd * c] + v : v;
  }
}
}  // namespace

hipError_t launch_copy_block(const double* src, int64_t ld_src, int rows, int cols, double* dst, int64_t ld_dst,
                             hipStream_t s, int trans, bool add) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s,
                     src, ld_src, rows, cols, dst, ld_dst, trans, add ? 1 : 0);
  return hipGetLastError();
}

// n <= 128 (eight 16-wide pivot blocks); larger matrices go through the
// blocked inverse built on the LDS Cholesky
bool spd_inverse_fits(int n) { return n >= 1 && n <= 128; }

hipError_t launch_spd_inverse(const double* S, int n, double* Sinv, int* status, hipStream_t s) {
  const int nbt = (n + 15) / 16;
  switch (nbt) {
#define SPD_INV_CASE(B, NW) \
  case B: hipLaunchKernelGGL((spd_block_inv_kernel<B, NW>), dim3(1), dim3(NW * 64), 0, s, S, n, Sinv, status); break;
    SPD_INV_CASE(1, 4) SPD_INV_CASE(2, 4) SPD_INV_CASE(3, 4) SPD_INV_CASE(4, 4)
    SPD_INV_CASE(5, 4) SPD_INV_CASE(6, 4) SPD_INV_CASE(7, 4) SPD_INV_CASE(8, 8)
#undef SPD_INV_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
