// X-streaming contraction (the MTTSP of Alg. 2): M_n = X_[n] G^{!=n}_[2].
//
// X is read once, coalesced, into LDS tiles A[i, k] (i = mode-n index, k = the
// other indices in memory order).  For every k of a tile the subchain row
// G^{!=n}(k) = F1[f1(k)] F2[f2(k)] (an R_{n+1} x R_n matrix, Sec. 2 subchain
// definition) is formed in LDS from two small tables of partial subchains, and
// the tile product A * B is accumulated on MFMA.  Work is split over k
// (split-K); every workgroup writes its partial tile and a second kernel sums
// the partials in a fixed order in FP64, so the result is deterministic.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

template <int P> struct PT;
template <> struct PT<TR_F64>  { using op_t = double;  using gen_t = double; using acc_t = f64x4; static constexpr int KS = 4;  };
template <> struct PT<TR_F32>  { using op_t = float;   using gen_t = float;  using acc_t = f32x4; static constexpr int KS = 4;  };
template <> struct PT<TR_BF16> { using op_t = __bf16;  using gen_t = float;  using acc_t = f32x4; static constexpr int KS = 32; };
template <> struct PT<TR_FP8>  { using op_t = uint8_t; using gen_t = float;  using acc_t = f32x4; static constexpr int KS = 32; };

// Row padding (in elements) of the LDS tiles: keeps 16-byte alignment for the
// packed fragments and spreads the 16 rows of a fragment over the banks.
template <int P> struct Pad { static constexpr int v = 4; };
template <> struct Pad<TR_F64> { static constexpr int v = 2; };
template <> struct Pad<TR_BF16> { static constexpr int v = 8; };
template <> struct Pad<TR_FP8> { static constexpr int v = 16; };

__device__ __forceinline__ void mma(f32x4& c, float a, float b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ void mma(f64x4& c, double a, double b) { c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ __forceinline__ void mma(f32x4& c, bf16x8 a, bf16x8 b) { c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ void mma(f32x4& c, long a, long b) { c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }

template <int P> struct Frag;
template <> struct Frag<TR_F64> {
  using t = double;
  static __device__ __forceinline__ t ld(const double* p, int row, int st, int kb, int lane) { return p[row * st + kb + (lane >> 4)]; }
};
template <> struct Frag<TR_F32> {
  using t = float;
  static __device__ __forceinline__ t ld(const float* p, int row, int st, int kb, int lane) { return p[row * st + kb + (lane >> 4)]; }
};
template <> struct Frag<TR_BF16> {
  using t = bf16x8;
  static __device__ __forceinline__ t ld(const __bf16* p, int row, int st, int kb, int lane) {
    return *reinterpret_cast<const bf16x8*>(p + row * st + kb + 8 * (lane >> 4));
  }
};
template <> struct Frag<TR_FP8> {
  using t = long;
  static __device__ __forceinline__ t ld(const uint8_t* p, int row, int st, int kb, int lane) {
    return *reinterpret_cast<const long*>(p + row * st + kb + 8 * (lane >> 4));
  }
};

// Conversion of a generated subchain value to the operand type.
template <int P> __device__ __forceinline__ typename PT<P>::op_t to_op(typename PT<P>::gen_t v);
template <> __device__ __forceinline__ double to_op<TR_F64>(double v) { return v; }
template <> __device__ __forceinline__ float to_op<TR_F32>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 to_op<TR_BF16>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ uint8_t to_op<TR_FP8>(float v) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
}

// Conversion of a stored X element to the operand type.  BF16/FP8 read the
// shadow copy, whose bits are already in operand format.
template <int P, typename Tin> __device__ __forceinline__ typename PT<P>::op_t x_to_op(Tin v);
template <> __device__ __forceinline__ double x_to_op<TR_F64, double>(double v) { return v; }
template <> __device__ __forceinline__ double x_to_op<TR_F64, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ float x_to_op<TR_F32, float>(float v) { return v; }
template <> __device__ __forceinline__ float x_to_op<TR_F32, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ __bf16 x_to_op<TR_BF16, __bf16>(__bf16 v) { return v; }
template <> __device__ __forceinline__ uint8_t x_to_op<TR_FP8, uint8_t>(uint8_t v) { return v; }

// Row / column of accumulator element v held by lane (16x16 MFMA result).
template <int P> __device__ __forceinline__ int acc_row(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<TR_F64>(int lane, int v) { return (lane >> 4) + 4 * v; }

constexpr int NTHR = 256;

template <int P, typename Tin, int KT, int WM, int WN>
__global__ __launch_bounds__(NTHR) void xstream_kernel(XsArgs a) {
  using op_t = typename PT<P>::op_t;
  using gen_t = typename PT<P>::gen_t;
  using acc_t = typename PT<P>::acc_t;
  constexpr int KS = PT<P>::KS;
  constexpr int ST = KT + Pad<P>::v;
  extern __shared__ __align__(16) unsigned char smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int otile = blockIdx.x;
  const int split = blockIdx.y;
  const int mt = otile / a.n_nt, nt = otile % a.n_nt;
  const int MT = a.MT, NT = a.NT;
  const int64_t i0 = (int64_t)mt * MT;
  const int b0 = nt * a.NTb;
  const int bcount = min(a.NTb, a.Rb - b0);
  // F1 rows are staged only for this workgroup's b-range (NTb values)
  const int Bw4 = (a.NTb + 3) & ~3, Ra4 = (a.Ra + 3) & ~3;
  const int row1 = a.Rmid * Bw4, row2 = a.Rmid * Ra4;
  const int s1max = (a.d1 == 1) ? KT : min((int64_t)KT, (KT + a.d1 - 1) / a.d1 + 1);

  // FP8: the generated subchain rows are stored as hi and lo E4M3 parts
  // (NT rows each), both contracted into the same accumulators
  constexpr int NPART = P == TR_FP8 ? 2 : 1;
  op_t* Xs = reinterpret_cast<op_t*>(smem);
  op_t* Bs = Xs + MT * ST;
  gen_t* F1s = reinterpret_cast<gen_t*>(smem + (((size_t)(MT + NPART * NT) * ST * sizeof(op_t) + 15) & ~(size_t)15));
  gen_t* F2s = F1s + (size_t)s1max * row1;

  const Tin* X = reinterpret_cast<const Tin*>(a.X);
  // FP8 scale of the generated rows from the device bound max|F1| max|F2| Rmid
  const gen_t bscale = P == TR_FP8 ? (gen_t)fp8_table_scale(a.tmax[0] * a.tmax[1] * a.Rmid) : (gen_t)1;

  // columns of the B tile that are never written by the generator stay zero
  for (int e = tid; e < NPART * NT * ST; e += NTHR) Bs[e] = to_op<P>((gen_t)0);

  // wave -> block sub-grid
  const int MB = MT / 16, NB = NT / 16;
  const int wm = wave % a.wgm, wn = wave / a.wgm;
  const int pbm = (MB + a.wgm - 1) / a.wgm, pbn = (NB + a.wgn - 1) / a.wgn;
  const int br0 = wm * pbm, bc0 = wn * pbn;
  const int nbr = max(0, min(pbm, MB - br0)), nbc = max(0, min(pbn, NB - bc0));

  acc_t acc[WM][WN];
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int c = 0; c < WN; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[r][c][v] = 0;

  const int64_t kbeg = (int64_t)split * a.k_per_split;
  const int64_t kend = min(a.K, kbeg + a.k_per_split);
  const int kk_t = tid % KT;             // this thread's column of the tile (loader layout 1, generator)
  const int rstep = NTHR / KT;

  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    const int kvalid = (int)min((int64_t)KT, kend - k0);
    __syncthreads();

    // ---- X tile -> Xs[i][kk]: every load of the tile in flight before the
    // LDS stores (one round trip to memory per tile, not one per element) ----
    constexpr int XE = (128 * KT) / NTHR;   // MT <= 128
    if (a.layout == 0) {
      // A[i, k] at i + I*k: consecutive threads walk i (contiguous in memory)
      op_t xv[XE];
#pragma unroll
      for (int q = 0; q < XE; ++q) {
        const int e = tid + q * NTHR;
        const int ii = e % MT, kk = e / MT;
        const int64_t i = i0 + ii;
        xv[q] = (e < MT * KT && i < a.I && kk < kvalid) ? x_to_op<P, Tin>(X[i + a.I * (k0 + kk)])
                                                         : to_op<P>((gen_t)0);
      }
#pragma unroll
      for (int q = 0; q < XE; ++q) {
        const int e = tid + q * NTHR;
        if (e < MT * KT) Xs[(e % MT) * ST + e / MT] = xv[q];
      }
    } else {
      // A[i, k] at (k % L) + L*i + L*I*(k / L): consecutive threads walk k
      const int64_t k = k0 + kk_t;
      const bool kok = kk_t < kvalid;
      const int64_t koff = kok ? (k % a.L) + a.L * a.I * (k / a.L) : 0;
      const int ii0 = tid / KT;
      op_t xv[XE];
#pragma unroll
      for (int q = 0; q < XE; ++q) {
        const int ii = ii0 + q * rstep;
        const int64_t i = i0 + ii;
        xv[q] = (ii < MT && kok && i < a.I) ? x_to_op<P, Tin>(X[koff + a.L * i]) : to_op<P>((gen_t)0);
      }
#pragma unroll
      for (int q = 0; q < XE; ++q) {
        const int ii = ii0 + q * rstep;
        if (ii < MT) Xs[ii * ST + kk_t] = xv[q];
      }
    }

    // ---- stage the partial-subchain rows this tile needs, eight loads per
    // thread in flight at a time ----
    const int64_t s1f = k0 / a.d1, s2f = k0 / a.d2;
    const int ns1 = (int)((k0 + kvalid - 1) / a.d1 - s1f + 1);
    const int ns2 = (int)((k0 + kvalid - 1) / a.d2 - s2f + 1);
    {
      const int tot = ns1 * row1;
      for (int base = tid; base < tot; base += 8 * NTHR) {
        gen_t t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = base + j * NTHR;
          const int sidx = e / row1, el = e % row1;
          const int m = el / Bw4, bl = el % Bw4;
          t[j] = (e < tot && bl < bcount)
                     ? (gen_t)a.F1[((s1f + sidx) % a.m1) * (int64_t)(a.Rb * a.Rmid) + (b0 + bl) + a.Rb * m]
                     : (gen_t)0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = base + j * NTHR;
          if (e < tot) F1s[e] = t[j];
        }
      }
    }
    {
      const int tot = ns2 * row2;
      for (int base = tid; base < tot; base += 8 * NTHR) {
        gen_t t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = base + j * NTHR;
          const int sidx = e / row2, el = e % row2;
          const int m = el / Ra4, aa = el % Ra4;
          t[j] = (e < tot && aa < a.Ra)
                     ? (gen_t)a.F2[((s2f + sidx) % a.m2) * (int64_t)(a.Rmid * a.Ra) + m + a.Rmid * aa]
                     : (gen_t)0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = base + j * NTHR;
          if (e < tot) F2s[e] = t[j];
        }
      }
    }
    __syncthreads();

    // ---- subchain rows -> Bs[c][kk], c = a + Ra*b (local b) ----
    {
      const bool kok = kk_t < kvalid;
      const int s1 = kok ? (int)((k0 + kk_t) / a.d1 - s1f) : 0;
      const int s2 = kok ? (int)((k0 + kk_t) / a.d2 - s2f) : 0;
      const gen_t* f1 = F1s + s1 * row1;
      const gen_t* f2 = F2s + s2 * row2;
      const int nab = Ra4 >> 2, nbb = (bcount + 3) >> 2;
      for (int q = tid / KT; q < nab * nbb; q += rstep) {
        const int ab = q % nab, bb = q / nab;
        gen_t g[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) g[x][y] = 0;
        if (kok) {
          for (int m = 0; m < a.Rmid; ++m) {
            gen_t fa[4], fb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) fa[x] = f2[m * Ra4 + 4 * ab + x];
#pragma unroll
            for (int y = 0; y < 4; ++y) fb[y] = f1[m * Bw4 + 4 * bb + y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) g[x][y] += fa[x] * fb[y];
          }
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            const int aa = 4 * ab + x, bl = 4 * bb + y;
            if (aa < a.Ra && bl < bcount) {
              const gen_t v = g[x][y] * bscale;
              const op_t hi = to_op<P>(v);
              Bs[(aa + a.Ra * bl) * ST + kk_t] = hi;
              if constexpr (P == TR_FP8)
                Bs[(NT + aa + a.Ra * bl) * ST + kk_t] = to_op<P>(v - __builtin_amdgcn_cvt_f32_fp8((int)hi, 0));
            }
          }
      }
    }
    __syncthreads();

    // ---- MFMA: acc += Xs * Bs^T ----
    using frag_t = typename Frag<P>::t;
#pragma unroll 2
    for (int kb = 0; kb < KT; kb += KS) {
#pragma unroll
      for (int part = 0; part < NPART; ++part) {
        frag_t bf[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c)
          if (c < nbc) bf[c] = Frag<P>::ld(Bs + part * NT * ST, (bc0 + c) * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
        for (int r = 0; r < WM; ++r) {
          if (r < nbr) {
            const frag_t af = Frag<P>::ld(Xs, (br0 + r) * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
            for (int c = 0; c < WN; ++c)
              if (c < nbc) mma(acc[r][c], af, bf[c]);
          }
        }
      }
    }
  }

  // ---- partial tile out ----
  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  part_t* out = reinterpret_cast<part_t*>(a.partial) +
                ((size_t)split * (a.n_mt * a.n_nt) + otile) * (size_t)MT * NT;
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int c = 0; c < WN; ++c)
      if (r < nbr && c < nbc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (br0 + r) * 16 + acc_row<P>(lane, v);
          const int col = (bc0 + c) * 16 + (lane & 15);
          out[(size_t)row * NT + col] = (part_t)acc[r][c][v];
        }
      }
  // blocks of the tile owned by no wave do not exist (the wave grid covers it)
}

template <int P>
__global__ void xs_reduce_kernel(XsArgs a, double out_scale, double* M, int* status) {
  // one thread per element of the padded partial tiles, column fastest, so the
  // split-K partials are read coalesced
  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  const int64_t tsz = (int64_t)a.MT * a.NT;
  const int64_t ntiles = (int64_t)a.n_mt * a.n_nt;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * tsz) return;
  const int otile = (int)(idx / tsz);
  const int ii = (int)((idx % tsz) / a.NT), col = (int)(idx % a.NT);
  const int mt = otile / a.n_nt, nt = otile % a.n_nt;
  const int64_t i = (int64_t)mt * a.MT + ii;
  const int aa = col % a.Ra, bl = col / a.Ra;
  const int b = nt * a.NTb + bl;
  if (i >= a.I || bl >= a.NTb || b >= a.Rb) return;
  const part_t* p = reinterpret_cast<const part_t*>(a.partial) + idx;
  const size_t sstride = (size_t)(ntiles * tsz);
  double s = 0.0;
  for (int sp = 0; sp < a.nsplit; ++sp) s += (double)p[sp * sstride];
  if (a.tmax) out_scale /= fp8_table_scale(a.tmax[0] * a.tmax[1] * a.Rmid);   // FP8
  s *= out_scale;
  if (!isfinite(s)) atomicOr(status, ST_NONFINITE);
  M[i + a.I * (int64_t)(aa + a.Ra * b)] = s;
}

template <int P, typename Tin, int KT>
hipError_t launch_t(const XsArgs& a, int wlay, size_t lds, hipStream_t s) {
  dim3 grid(a.n_mt * a.n_nt, a.nsplit);
  if (wlay == 0) {
    auto k = xstream_kernel<P, Tin, KT, 4, 4>;
    LDSCHK((const void*)k, lds);
    hipLaunchKernelGGL(k, grid, dim3(NTHR), lds, s, a);
  } else if (wlay == 1) {
    auto k = xstream_kernel<P, Tin, KT, 8, 2>;
    LDSCHK((const void*)k, lds);
    hipLaunchKernelGGL(k, grid, dim3(NTHR), lds, s, a);
  } else {
    auto k = xstream_kernel<P, Tin, KT, 2, 8>;
    LDSCHK((const void*)k, lds);
    hipLaunchKernelGGL(k, grid, dim3(NTHR), lds, s, a);
  }
  return hipGetLastError();
}

template <int P> size_t op_size() { return sizeof(typename PT<P>::op_t); }
template <int P> size_t gen_size() { return sizeof(typename PT<P>::gen_t); }

}  // namespace

size_t xstream_lds_bytes(const XsArgs& a, int prec, int kt) {
  size_t ops, gens;
  int pad;
  switch (prec) {
    case TR_F64: ops = op_size<TR_F64>(); gens = gen_size<TR_F64>(); pad = Pad<TR_F64>::v; break;
    case TR_F32: ops = op_size<TR_F32>(); gens = gen_size<TR_F32>(); pad = Pad<TR_F32>::v; break;
    case TR_BF16: ops = op_size<TR_BF16>(); gens = gen_size<TR_BF16>(); pad = Pad<TR_BF16>::v; break;
    default: ops = op_size<TR_FP8>(); gens = gen_size<TR_FP8>(); pad = Pad<TR_FP8>::v; break;
  }
  const size_t st = kt + pad;
  size_t bytes = (((size_t)(a.MT + (prec == TR_FP8 ? 2 : 1) * a.NT) * st * ops) + 15) & ~(size_t)15;
  const int Bw4 = (a.NTb + 3) & ~3, Ra4 = (a.Ra + 3) & ~3;
  auto smax = [&](int64_t d) -> int64_t { return d == 1 ? kt : std::min<int64_t>(kt, (kt + d - 1) / d + 1); };
  bytes += (size_t)(smax(a.d1) * a.Rmid * Bw4 + smax(a.d2) * a.Rmid * Ra4) * gens;
  return bytes;
}

hipError_t launch_xstream(const XsArgs& a, int prec, int xdt, int kt, int wlay, size_t lds, hipStream_t s) {
  if (prec == TR_F64) {
    if (xdt == TR_F64) return kt == 32 ? launch_t<TR_F64, double, 32>(a, wlay, lds, s) : launch_t<TR_F64, double, 16>(a, wlay, lds, s);
    return kt == 32 ? launch_t<TR_F64, float, 32>(a, wlay, lds, s) : launch_t<TR_F64, float, 16>(a, wlay, lds, s);
  }
  if (prec == TR_F32) {
    if (xdt == TR_F64) return kt == 64 ? launch_t<TR_F32, double, 64>(a, wlay, lds, s) : launch_t<TR_F32, double, 32>(a, wlay, lds, s);
    return kt == 64 ? launch_t<TR_F32, float, 64>(a, wlay, lds, s) : launch_t<TR_F32, float, 32>(a, wlay, lds, s);
  }
  if (prec == TR_BF16) return kt == 64 ? launch_t<TR_BF16, __bf16, 64>(a, wlay, lds, s) : launch_t<TR_BF16, __bf16, 32>(a, wlay, lds, s);
  return kt == 64 ? launch_t<TR_FP8, uint8_t, 64>(a, wlay, lds, s) : launch_t<TR_FP8, uint8_t, 32>(a, wlay, lds, s);
}

hipError_t launch_xs_reduce(const XsArgs& a, int prec, double out_scale, double* M, int* status, hipStream_t s) {
  const int64_t n = (int64_t)a.n_mt * a.n_nt * a.MT * a.NT;
  const int blk = 256;
  const int64_t grid = (n + blk - 1) / blk;
  if (prec == TR_F64) hipLaunchKernelGGL(xs_reduce_kernel<TR_F64>, dim3(grid), dim3(blk), 0, s, a, out_scale, M, status);
  else hipLaunchKernelGGL(xs_reduce_kernel<TR_F32>, dim3(grid), dim3(blk), 0, s, a, out_scale, M, status);
  return hipGetLastError();
}
