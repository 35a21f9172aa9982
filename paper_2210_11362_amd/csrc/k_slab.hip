// X contraction of an order-3 tensor with large ranks, slab by slab.
//
// For mode n the subchain row is G^{!=n}(i_c1, i_c2) = G_c1(i_c1) G_c2(i_c2)
// (c1 = n+1, c2 = n+2 cyclically; Sec. 2 subchain).  One of the other two
// modes, kappa, is contracted on MFMA against a fixed table of its core; the
// other, lambda, is walked slab by slab and its core absorbed right after:
//   case A (kappa = c1, lambda = c2):
//     T_l(i, (m, b)) = sum_k X(i, k, l) G_c1[b, k, m]
//     M(i, a + R_n b) += sum_m T_l(i, (m, b)) G_c2[m, l, a]
//   case B (kappa = c2, lambda = c1):
//     T_l(i, (m, a)) = sum_k X(i, k, l) G_c2[m, k, a]
//     M(i, a + R_n b) += sum_m G_c1[b, l, m] T_l(i, (m, a))
// so no subchain row is ever generated per k (the fused kernel's cost at
// large R), and X is read once per column group.  A workgroup owns a tile of
// rows i, one group of NG values of b (case A) or a (case B), and a range of
// slabs; T lives in MFMA accumulators over the slab's k loop, is spilled to
// LDS and absorbed into registers (FP64 on the FP64 path, else FP32); partial
// results per slab range are
// summed in a fixed order in FP64 by xslab_reduce_kernel.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int P> struct ST_;
template <> struct ST_<TR_F64>  { using op_t = double; using acc_t = f64x4; using t_t = double; static constexpr int KS = 4;  static constexpr int PAD = 2; };
template <> struct ST_<TR_F32>  { using op_t = float;  using acc_t = f32x4; using t_t = float;  static constexpr int KS = 4;  static constexpr int PAD = 4; };
template <> struct ST_<TR_BF16> { using op_t = __bf16; using acc_t = f32x4; using t_t = float;  static constexpr int KS = 32; static constexpr int PAD = 8; };

__device__ __forceinline__ void mma(f32x4& c, float a, float b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ void mma(f64x4& c, double a, double b) { c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ __forceinline__ void mma(f32x4& c, bf16x8 a, bf16x8 b) { c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

template <int P> struct Fr;
template <> struct Fr<TR_F64> {
  using t = double;
  static __device__ __forceinline__ t ld(const double* p, int row, int st, int kb, int lane) { return p[row * st + kb + (lane >> 4)]; }
};
template <> struct Fr<TR_F32> {
  using t = float;
  static __device__ __forceinline__ t ld(const float* p, int row, int st, int kb, int lane) { return p[row * st + kb + (lane >> 4)]; }
};
template <> struct Fr<TR_BF16> {
  using t = bf16x8;
  static __device__ __forceinline__ t ld(const __bf16* p, int row, int st, int kb, int lane) {
    return *reinterpret_cast<const bf16x8*>(p + row * st + kb + 8 * (lane >> 4));
  }
};

template <int P> __device__ __forceinline__ int acc_row(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<TR_F64>(int lane, int v) { return (lane >> 4) + 4 * v; }

template <int P, typename Tin> __device__ __forceinline__ typename ST_<P>::op_t cvt(Tin v);
template <> __device__ __forceinline__ double cvt<TR_F64, double>(double v) { return v; }
template <> __device__ __forceinline__ double cvt<TR_F64, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ float cvt<TR_F32, float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt<TR_F32, double>(double v) { return (float)v; }

constexpr int NTHR = 256;
constexpr int MTX = 128;     // rows per tile
constexpr int TWX = 128;     // T columns per group (NG * Rm <= TWX)
constexpr int UPT = 2;       // group values per thread in the absorption (two threads per row: NG <= 4)
constexpr int XPT = 32;      // largest other rank of the absorbed core
constexpr int RMX = 32;      // largest middle rank

template <int P, typename Tin, int KT>
__global__ __launch_bounds__(NTHR) void xslab_kernel(XslabArgs a) {
  using op_t = typename ST_<P>::op_t;
  using acc_t = typename ST_<P>::acc_t;
  using t_t = typename ST_<P>::t_t;
  constexpr int KS = ST_<P>::KS;
  constexpr int ST = KT + ST_<P>::PAD;
  constexpr int WM = MTX / 16 / (NTHR / 64), WN = 8;   // 4 waves stacked over the rows, each 2 x 8 blocks of 16 x 16
  extern __shared__ __align__(16) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x, split = blockIdx.y;
  const int mt = tile / a.n_g, g = tile % a.n_g;
  const int64_t i0 = (int64_t)mt * MTX;
  const int ng = min(a.NG, a.Rg - g * a.NG);       // values of the group index in this group
  const int TW = ng * a.Rm;                        // T columns used
  const int TWp = (TW + 15) & ~15;
  const int NBc = TWp / 16;

  // BF16: the table is held as hi + lo BF16 parts (two products), so that
  // only X is rounded to BF16; FP32 / FP64 tables are one part
  constexpr int NPART = P == TR_BF16 ? 2 : 1;
  // LDS: the X and table tiles of the k loop, and (after it, in the same
  // bytes) the spilled T of the slab; then the slab of the absorbed core
  op_t* Xs = reinterpret_cast<op_t*>(smem);                // MTX x ST
  op_t* Bs = Xs + MTX * ST;                                // NPART x TWX x ST
  t_t* Ts = reinterpret_cast<t_t*>(smem);                  // MTX x TSW, aliases Xs / Bs
  const int TSW = a.TWg + 1;                               // padded row of Ts (odd: conflict-free rows)
  const size_t xb_bytes = ((size_t)(MTX + NPART * TWX) * ST * sizeof(op_t) + 15) & ~(size_t)15;
  const size_t ts_bytes = ((size_t)MTX * TSW * sizeof(t_t) + 15) & ~(size_t)15;
  t_t* Gls = reinterpret_cast<t_t*>(smem + (xb_bytes > ts_bytes ? xb_bytes : ts_bytes));   // Rm x Ro

  const Tin* X = reinterpret_cast<const Tin*>(a.X);
  const op_t* Bt = reinterpret_cast<const op_t*>(a.Bt);   // [col][k], ldb = a.ldb

  // absorbed outputs of this thread: row i = tid % 128, group values
  // u = u_lo .. u_lo + UPT - 1 (the threads of a row split the group)
  const int my_i = tid & (MTX - 1);
  const int u_lo = (tid / MTX) * UPT;
  t_t macc[UPT][XPT];      // FP64 on the FP64 path, else FP32
#pragma unroll
  for (int uu = 0; uu < UPT; ++uu)
#pragma unroll
    for (int x = 0; x < XPT; ++x) macc[uu][x] = 0;

  const int64_t l_beg = (int64_t)split * a.l_per_split;
  const int64_t l_end = min(a.Il, l_beg + a.l_per_split);
  // operand chunks in registers; BF16 fetches them one k step ahead (and the
  // next slab's first chunk during the last step of a slab) so that their
  // global loads overlap the MFMAs of the current chunk
  // BF16: 16-byte loads of 8 consecutive elements (rows i when they are
  // contiguous, else k) and of the table; other types element by element
  constexpr int VW = P == TR_BF16 ? 8 : 1;
  constexpr int XE = MTX * KT / NTHR / VW;
  constexpr int BE = TWX * KT / NTHR / VW;
  using vec_t = typename std::conditional<P == TR_BF16, u32x4, op_t>::type;
  vec_t xv[XE];
  vec_t bv[NPART][BE];
  const bool rows_c = a.sn == 1;   // rows contiguous in X (else k contiguous)
  auto load_chunk = [&](int64_t l, int64_t k0) {
    const Tin* Xl = X + a.sl * l;
    const int kvalid = (int)min((int64_t)KT, a.Ik - k0);
    if constexpr (P == TR_BF16) {
      // whole vectors are in or out: In and Ik are multiples of 8 and the
      // strides keep 16-byte alignment (checked by the host)
      if (rows_c) {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          const int iv = e % (MTX / VW), kk = e / (MTX / VW);
          const int64_t i = i0 + VW * iv;
          xv[q] = (i < a.In && kk < kvalid) ? *reinterpret_cast<const u32x4*>(Xl + i + a.sk * (k0 + kk))
                                           : u32x4{0, 0, 0, 0};
        }
      } else {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          const int kv = e % (KT / VW), ii = e / (KT / VW);
          const int64_t i = i0 + ii;
          xv[q] = (i < a.In && VW * kv < kvalid) ? *reinterpret_cast<const u32x4*>(Xl + a.sn * i + k0 + VW * kv)
                                                : u32x4{0, 0, 0, 0};
        }
      }
#pragma unroll
      for (int part = 0; part < NPART; ++part) {
        const op_t* Bp = Bt + (size_t)part * a.n_g * a.TWg * a.ldb;
#pragma unroll
        for (int q = 0; q < BE; ++q) {
          const int e = tid + q * NTHR;
          const int kv = e % (KT / VW), cl = e / (KT / VW);
          bv[part][q] = (cl < TWp) ? *reinterpret_cast<const u32x4*>(Bp + (int64_t)(g * a.TWg + cl) * a.ldb + k0 + VW * kv)
                                   : u32x4{0, 0, 0, 0};
        }
      }
    } else {
      if (rows_c) {              // threads walk i
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          const int ii = e % MTX, kk = e / MTX;
          const int64_t i = i0 + ii;
          xv[q] = (i < a.In && kk < kvalid) ? cvt<P, Tin>(Xl[i + a.sk * (k0 + kk)]) : (op_t)0;
        }
      } else {                   // threads walk k
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          const int kk = e % KT, ii = e / KT;
          const int64_t i = i0 + ii;
          xv[q] = (i < a.In && kk < kvalid) ? cvt<P, Tin>(Xl[a.sn * i + (k0 + kk)]) : (op_t)0;
        }
      }
#pragma unroll
      for (int part = 0; part < NPART; ++part) {   // table chunk (zero-padded beyond ldb)
        const op_t* Bp = Bt + (size_t)part * a.n_g * a.TWg * a.ldb;
#pragma unroll
        for (int q = 0; q < BE; ++q) {
          const int e = tid + q * NTHR;
          const int kk = e % KT, cl = e / KT;
          bv[part][q] = (cl < TWp) ? Bp[(int64_t)(g * a.TWg + cl) * a.ldb + k0 + kk] : (op_t)0;
        }
      }
    }
  };
  auto store_chunk = [&]() {
    if constexpr (P == TR_BF16) {
      if (rows_c) {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          const int iv = e % (MTX / VW), kk = e / (MTX / VW);
          const __bf16* v = reinterpret_cast<const __bf16*>(&xv[q]);
#pragma unroll
          for (int j = 0; j < VW; ++j) Xs[(VW * iv + j) * ST + kk] = v[j];
        }
      } else {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          *reinterpret_cast<u32x4*>(Xs + (e / (KT / VW)) * ST + VW * (e % (KT / VW))) = xv[q];
        }
      }
#pragma unroll
      for (int part = 0; part < NPART; ++part)
#pragma unroll
        for (int q = 0; q < BE; ++q) {
          const int e = tid + q * NTHR;
          *reinterpret_cast<u32x4*>(Bs + part * TWX * ST + (e / (KT / VW)) * ST + VW * (e % (KT / VW))) = bv[part][q];
        }
    } else {
      if (rows_c) {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          Xs[(e % MTX) * ST + e / MTX] = xv[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < XE; ++q) {
          const int e = tid + q * NTHR;
          Xs[(e / KT) * ST + e % KT] = xv[q];
        }
      }
#pragma unroll
      for (int part = 0; part < NPART; ++part)
#pragma unroll
        for (int q = 0; q < BE; ++q) {
          const int e = tid + q * NTHR;
          Bs[part * TWX * ST + (e / KT) * ST + e % KT] = bv[part][q];
        }
    }
  };
  // BF16 fetches one chunk ahead; the wider types (no register room for a
  // second chunk) fetch each chunk right before storing it
  constexpr bool PREF = P == TR_BF16;
  if (PREF && l_beg < l_end) load_chunk(l_beg, 0);
  for (int64_t l = l_beg; l < l_end; ++l) {
    acc_t acc[WM][WN];
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int c = 0; c < WN; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[r][c][v] = 0;
    for (int64_t k0 = 0; k0 < a.Ik; k0 += KT) {
      __syncthreads();             // the tiles (or, at k0 = 0, the previous slab's T) are free
      if constexpr (!PREF) load_chunk(l, k0);
      store_chunk();
      __syncthreads();
      if constexpr (PREF) {
        if (k0 + KT < a.Ik) load_chunk(l, k0 + KT);
        else if (l + 1 < l_end) load_chunk(l + 1, 0);
      }
      using frag_t = typename Fr<P>::t;
#pragma unroll
      for (int part = 0; part < NPART; ++part)
#pragma unroll
        for (int kb = 0; kb < KT; kb += KS) {
          frag_t bf[WN];
#pragma unroll
          for (int c = 0; c < WN; ++c)
            if (c < NBc) bf[c] = Fr<P>::ld(Bs + part * TWX * ST, c * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
          for (int r = 0; r < WM; ++r) {
            const frag_t af = Fr<P>::ld(Xs, (wave * WM + r) * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
            for (int c = 0; c < WN; ++c)
              if (c < NBc) mma(acc[r][c], af, bf[c]);
          }
        }
    }
    // T -> LDS, slab of the absorbed core -> LDS
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int c = 0; c < WN; ++c)
        if (c < NBc) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = (wave * WM + r) * 16 + acc_row<P>(lane, v);
            const int col = c * 16 + (lane & 15);
            Ts[row * TSW + col] = (t_t)acc[r][c][v];
          }
        }
    // Gls[m * Ro + x]: case A G_c2[m, l, x=a] at m + Rm (l + Il a); case B G_c1[x=b, l, m] at b + Rb (l + Il m)
    for (int e = tid; e < a.Rm * a.Ro; e += NTHR) {
      const int m = e / a.Ro, x = e % a.Ro;
      const int64_t src = a.caseB ? (x + (int64_t)a.Ro * (l + a.Il * m)) : (m + (int64_t)a.Rm * (l + a.Il * x));
      Gls[e] = (t_t)a.Gl[src];
    }
    __syncthreads();
    // absorb: outputs (u, x) of this thread's row, x in [0, Ro), one middle
    // index m at a time (in increasing m), straight into the accumulators
    if (i0 + my_i < a.In) {
      const t_t* trow = Ts + my_i * TSW;
#pragma unroll
      for (int uu = 0; uu < UPT; ++uu) {
        const int u = u_lo + uu;
        if (u < ng) {
          for (int m = 0; m < a.Rm; ++m) {
            const t_t tv = trow[m + a.Rm * u];
            const t_t* gm = Gls + m * a.Ro;
#pragma unroll
            for (int x = 0; x < XPT; ++x)
              if (x < a.Ro) macc[uu][x] += tv * gm[x];
          }
        }
      }
    }
  }
  // partial [split][tile][row][u * Ro + x] (FP32, or FP64 on the FP64 path)
  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  part_t* out = reinterpret_cast<part_t*>(a.partial) +
                ((size_t)split * (a.n_mt * a.n_g) + tile) * (size_t)MTX * a.OWg;
  if (i0 + my_i < a.In) {
#pragma unroll
    for (int uu = 0; uu < UPT; ++uu)
#pragma unroll
      for (int x = 0; x < XPT; ++x)
        if (u_lo + uu < ng && x < a.Ro) out[(size_t)my_i * a.OWg + (u_lo + uu) * a.Ro + x] = (part_t)macc[uu][x];
  }
}

// Sum of the split partials in split order (FP64), scaled, into M(i, a + R_n b).
template <int P>
__global__ void xslab_reduce_kernel(XslabArgs a, double out_scale, double* M, int* status) {
  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  const int64_t tsz = (int64_t)MTX * a.OWg;
  const int64_t ntiles = (int64_t)a.n_mt * a.n_g;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * tsz) return;
  const int tile = (int)(idx / tsz);
  const int row = (int)((idx % tsz) / a.OWg), o = (int)(idx % a.OWg);
  const int mt = tile / a.n_g, g = tile % a.n_g;
  const int64_t i = (int64_t)mt * MTX + row;
  const int u = o / a.Ro, x = o % a.Ro;
  const int gu = g * a.NG + u;
  if (i >= a.In || u >= a.NG || gu >= a.Rg) return;
  const part_t* p = reinterpret_cast<const part_t*>(a.partial) + idx;
  const size_t sstride = (size_t)(ntiles * tsz);
  double s = 0.0;
  for (int sp = 0; sp < a.nsplit; ++sp) s += (double)p[sp * sstride];
  s *= out_scale;
  if (!isfinite(s)) atomicOr(status, ST_NONFINITE);
  // case A: u = b (group index), x = a; case B: u = a, x = b
  const int aa = a.caseB ? gu : x, bb = a.caseB ? x : gu;
  M[i + a.In * (int64_t)(aa + a.Rn * bb)] = s;
}

// Operand table, transposed, in the operand type: column c = g TWg + m + Rm u
// of group g holds, over k, case A G_k[b = g NG + u, k, m] (left rank Rg, right
// rank Rm); case B G_k[m, k, a = g NG + u] (left rank Rm, right rank Rg);
// columns beyond the group's values and k beyond Ik are zero.
// BF16 tables hold two parts: hi = bf16(v) and, n entries later, lo = bf16(v - hi).
template <typename T>
__global__ void xslab_table_kernel(XslabArgs a, const double* Gk, T* Bt) {
  const int64_t n = (int64_t)a.n_g * a.TWg * a.ldb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % a.ldb;
    const int c = (int)(e / a.ldb);
    const int g = c / a.TWg, cl = c % a.TWg;
    const int m = cl % a.Rm, u = cl / a.Rm;
    const int gu = g * a.NG + u;
    double v = 0.0;
    if (k < a.Ik && u < a.NG && gu < a.Rg && cl < a.NG * a.Rm)
      v = a.caseB ? Gk[m + (int64_t)a.Rm * (k + a.Ik * gu)] : Gk[gu + (int64_t)a.Rg * (k + a.Ik * m)];
    if constexpr (std::is_same<T, __bf16>::value) {
      const __bf16 hi = (__bf16)(float)v;
      Bt[e] = hi;
      Bt[e + n] = (__bf16)(float)(v - (double)(float)hi);
    } else {
      Bt[e] = (T)v;
    }
  }
}

template <int P, typename Tin>
hipError_t launch_kt(const XslabArgs& a, size_t lds, hipStream_t s) {
  constexpr int KT = P == TR_BF16 ? 64 : (P == TR_F32 ? 32 : 16);
  auto k = xslab_kernel<P, Tin, KT>;
  LDSCHK((const void*)k, lds);
  hipLaunchKernelGGL(k, dim3(a.n_mt * a.n_g, a.nsplit), dim3(NTHR), lds, s, a);
  return hipGetLastError();
}

}  // namespace

int xslab_kt(int prec) { return prec == TR_BF16 ? 64 : (prec == TR_F32 ? 32 : 16); }

size_t xslab_lds_bytes(const XslabArgs& a, int prec) {
  const int kt = xslab_kt(prec);
  const size_t ops = prec == TR_F64 ? 8 : prec == TR_F32 ? 4 : 2;
  const size_t ts = prec == TR_F64 ? 8 : 4;
  const int pad = prec == TR_F64 ? 2 : prec == TR_F32 ? 4 : 8;
  const int nparts = prec == TR_BF16 ? 2 : 1;
  size_t b = ((size_t)(MTX + nparts * TWX) * (kt + pad) * ops + 15) & ~(size_t)15;
  const size_t tsb = ((size_t)MTX * (a.TWg + 1) * ts + 15) & ~(size_t)15;   // T aliases the tiles
  return std::max(b, tsb) + (size_t)a.Rm * a.Ro * ts;
}

// Group size of the slab kernel for a middle rank Rm and the absorbed core's
// other rank Ro, or 0 when it does not apply.
int xslab_group(int Rm, int Ro) {
  if (Rm < 1 || Rm > RMX || Ro < 1 || Ro > XPT) return 0;
  return std::min(NTHR / MTX * UPT, TWX / Rm);
}
int xslab_rows() { return MTX; }

hipError_t launch_xslab_table(const XslabArgs& a, const double* Gk, int prec, void* Bt, hipStream_t s) {
  const int64_t n = (int64_t)a.n_g * a.TWg * a.ldb;
  const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 8192));
  switch (prec) {
    case TR_F64: hipLaunchKernelGGL(xslab_table_kernel<double>, grid, dim3(256), 0, s, a, Gk, (double*)Bt); break;
    case TR_F32: hipLaunchKernelGGL(xslab_table_kernel<float>, grid, dim3(256), 0, s, a, Gk, (float*)Bt); break;
    case TR_BF16: hipLaunchKernelGGL(xslab_table_kernel<__bf16>, grid, dim3(256), 0, s, a, Gk, (__bf16*)Bt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_xslab(const XslabArgs& a, int prec, int xdt, size_t lds, hipStream_t s) {
  if (prec == TR_F64) return xdt == TR_F64 ? launch_kt<TR_F64, double>(a, lds, s) : launch_kt<TR_F64, float>(a, lds, s);
  if (prec == TR_F32) return xdt == TR_F64 ? launch_kt<TR_F32, double>(a, lds, s) : launch_kt<TR_F32, float>(a, lds, s);
  if (prec == TR_BF16) return launch_kt<TR_BF16, __bf16>(a, lds, s);
  return hipErrorInvalidValue;
}

hipError_t launch_xslab_reduce(const XslabArgs& a, int prec, double out_scale, double* M, int* status,
                               hipStream_t s) {
  const int64_t n = (int64_t)a.n_mt * a.n_g * MTX * a.OWg;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (prec == TR_F64) hipLaunchKernelGGL(xslab_reduce_kernel<TR_F64>, grid, dim3(256), 0, s, a, out_scale, M, status);
  else hipLaunchKernelGGL(xslab_reduce_kernel<TR_F32>, grid, dim3(256), 0, s, a, out_scale, M, status);
  return hipGetLastError();
}
