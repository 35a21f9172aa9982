// Two-stage MTTSP (the compressible case of Alg. 2's MTTSP step).
//
// Stage 1 contracts X over one memory-contiguous group of modes g with the
// partial subchain of those modes (a table B, Sec. 2 subchain product):
//   Y[r, c] = sum_k A[r, k] B[k, c],  A = X seen as a matrix whose columns
//   (NN: A[r,k] = X[r + M*k], group = slowest modes) or rows (TN: A[r,k] =
//   X[k + K*r], group = fastest modes) run over the group.
// It is a tall-skinny GEMM on MFMA that reads X exactly once and writes
// split-K partial tiles; their ordered reduction, the operand tables and
// stage 2 (absorbing the remaining modes) live in k_stage2.hip.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int P> struct PT;
template <> struct PT<TR_F64>  { using op_t = double;  using acc_t = f64x4; static constexpr int KS = 4;  };
template <> struct PT<TR_F32>  { using op_t = float;   using acc_t = f32x4; static constexpr int KS = 4;  };
template <> struct PT<TR_BF16> { using op_t = __bf16;  using acc_t = f32x4; static constexpr int KS = 32; };
template <> struct PT<TR_FP8>  { using op_t = uint8_t; using acc_t = f32x4; static constexpr int KS = 32; };

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

template <int P, typename Tin> __device__ __forceinline__ typename PT<P>::op_t x_to_op(Tin v);
template <> __device__ __forceinline__ double x_to_op<TR_F64, double>(double v) { return v; }
template <> __device__ __forceinline__ double x_to_op<TR_F64, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ float x_to_op<TR_F32, float>(float v) { return v; }
template <> __device__ __forceinline__ float x_to_op<TR_F32, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ __bf16 x_to_op<TR_BF16, __bf16>(__bf16 v) { return v; }
template <> __device__ __forceinline__ uint8_t x_to_op<TR_FP8, uint8_t>(uint8_t v) { return v; }

template <int P> __device__ __forceinline__ int acc_row(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<TR_F64>(int lane, int v) { return (lane >> 4) + 4 * v; }

constexpr int NTHR = 256;

// Elements per 16-byte vector of the operand type.
template <int P> struct Vec { static constexpr int n = 16 / sizeof(typename PT<P>::op_t); };

template <int P, typename Tin, bool NN, bool VEC, int MT, int KT, int NBMAX>
__global__ __launch_bounds__(NTHR) void xgemm_kernel(XgArgs g) {
  using op_t = typename PT<P>::op_t;
  using acc_t = typename PT<P>::acc_t;
  using frag_t = typename Frag<P>::t;
  constexpr int KS = PT<P>::KS;
  constexpr int ST = KT + Pad<P>::v;
  constexpr int V = Vec<P>::n;
  constexpr int AV = MT * KT / V / NTHR;
  constexpr int KV = KT / V;                  // packed vectors along a tile row
  constexpr int MBW = MT / 64;                // row blocks per wave (waves stacked along rows)
  constexpr int NPART = P == TR_FP8 ? 2 : 1;  // FP8 tables: hi and lo parts, NT rows each
  extern __shared__ __align__(16) unsigned char smem[];
  op_t* As = reinterpret_cast<op_t*>(smem);
  op_t* Bs = As + MT * ST;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Tile and k-split of this workgroup.  Workgroups are dispatched round-robin
  // over the 8 XCDs by linear id; with xcd_map the ones that land on one XCD
  // take the same k-splits, so each slice of the operand table is fetched
  // into one L2 and reused there by every row tile.
  const int ntiles = g.n_mt * g.n_nt;
  int tile, split;
  if (g.xcd_map) {
    const int L = blockIdx.x, xcd = L & 7, j = L >> 3, s8 = g.nsplit >> 3;
    split = xcd * s8 + j % s8;
    tile = j / s8;
  } else {
    tile = blockIdx.x;
    split = blockIdx.y;
  }
  const int mt = tile % g.n_mt, nt = tile / g.n_mt;
  const int64_t r0 = (int64_t)mt * MT;
  const int NT = g.NT, NB = NT / 16;
  const Tin* X = reinterpret_cast<const Tin*>(g.X);
  const op_t* Bt = reinterpret_cast<const op_t*>(g.Bt) + (size_t)nt * NT * g.ldb;
  const size_t bpart = (size_t)g.n_nt * NT * g.ldb;   // elements from one table part to the next

  const int64_t kbeg = (int64_t)split * g.k_per_split;
  const int64_t kend = min(g.K, kbeg + g.k_per_split);

  acc_t acc[MBW][NBMAX];
#pragma unroll
  for (int r = 0; r < MBW; ++r)
#pragma unroll
    for (int c = 0; c < NBMAX; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[r][c][v] = 0;

  // per-thread coordinates of its packed A vectors: (row, kvec)
  op_t areg[VEC ? 1 : AV][V];
  // VEC (fastest-modes group, A[r,k] = X[k + K*r]): one 16-byte load per
  // packed vector.
  u32x4 vreg[VEC ? AV : 1];
  auto load_a = [&](int64_t k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHR, kv = e % KV, row = e / KV;
        const int64_t r = r0 + row, kb = k0 + kv * V;
        vreg[q] = (r < g.M && kb < kend) ? *reinterpret_cast<const u32x4*>(X + kb + g.K * r) : u32x4{0, 0, 0, 0};
      }
    } else {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHR;
        int row, kv;
        if (NN) { row = e % MT; kv = e / MT; }   // consecutive threads walk rows (contiguous in X)
        else { kv = e % KV; row = e / KV; }      // consecutive threads walk k (contiguous in X)
        const int64_t r = r0 + row;
        const int64_t kb = k0 + kv * V;
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const int64_t k = kb + j;
          op_t v = x_to_op<P, Tin>((Tin)0);
          if (r < g.M && k < kend) v = x_to_op<P, Tin>(NN ? X[r + g.M * k] : X[k + g.K * r]);
          areg[q][j] = v;
        }
      }
    }
  };
  auto store_a = [&]() {
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHR, kv = e % KV, row = e / KV;
        *reinterpret_cast<u32x4*>(As + row * ST + kv * V) = vreg[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < AV; ++q) {
        const int e = tid + q * NTHR;
        int row, kv;
        if (NN) { row = e % MT; kv = e / MT; }
        else { kv = e % KV; row = e / KV; }
        op_t* dst = As + row * ST + kv * V;
#pragma unroll
        for (int j = 0; j < V; ++j) dst[j] = areg[q][j];
      }
    }
  };
  // B tile: NT rows of KT contiguous elements, zero-padded in the table
  // itself.  For 8/16-bit operands it is fetched into registers one tile
  // ahead of its LDS store; wider operands copy it when it is needed.
  // LDS row q of the B tile: row q % NT of table part q / NT
  constexpr int BQ = (NPART * NBMAX * 16 * KV + NTHR - 1) / NTHR;
  constexpr bool BPF = BQ <= 4;
  u32x4 breg[BPF ? BQ : 1];
  auto b_src = [&](int q, int64_t k) { return Bt + (size_t)(q / NT) * bpart + (size_t)(q % NT) * g.ldb + k; };
  auto load_b = [&](int64_t k0) {
    if constexpr (BPF) {
#pragma unroll
      for (int q = 0; q < BQ; ++q) {
        const int e = tid + q * NTHR;
        if (e < NPART * NT * KV) {
          const int row = e / KV, kv = e % KV;
          breg[q] = *reinterpret_cast<const u32x4*>(b_src(row, k0 + kv * V));
        }
      }
    }
  };
  auto store_b = [&](int64_t k0) {
    if constexpr (BPF) {
#pragma unroll
      for (int q = 0; q < BQ; ++q) {
        const int e = tid + q * NTHR;
        if (e < NPART * NT * KV) {
          const int row = e / KV, kv = e % KV;
          *reinterpret_cast<u32x4*>(Bs + row * ST + kv * V) = breg[q];
        }
      }
    } else {
      for (int e = tid; e < NPART * NT * KV; e += NTHR) {
        const int row = e / KV, kv = e % KV;
        *reinterpret_cast<u32x4*>(Bs + row * ST + kv * V) = *reinterpret_cast<const u32x4*>(b_src(row, k0 + kv * V));
      }
    }
  };

  if (kbeg < kend) {
    load_a(kbeg);
    load_b(kbeg);
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    __syncthreads();
    store_a();
    store_b(k0);
    __syncthreads();
    if (k0 + KT < kend) {                    // next tile's global loads overlap the MFMAs below
      load_a(k0 + KT);
      load_b(k0 + KT);
    }
#pragma unroll
    for (int kb = 0; kb < KT; kb += KS) {
      frag_t af[MBW];
#pragma unroll
      for (int r = 0; r < MBW; ++r) af[r] = Frag<P>::ld(As, (wave * MBW + r) * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
      for (int c = 0; c < NBMAX; ++c) {
        if (c < NB) {
#pragma unroll
          for (int part = 0; part < NPART; ++part) {
            const frag_t bf = Frag<P>::ld(Bs + part * NT * ST, c * 16 + (lane & 15), ST, kb, lane);
#pragma unroll
            for (int r = 0; r < MBW; ++r) mma(acc[r][c], af[r], bf);
          }
        }
      }
    }
  }

  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  part_t* out = reinterpret_cast<part_t*>(g.partial) + ((size_t)split * ntiles + tile) * (size_t)MT * NT;
#pragma unroll
  for (int r = 0; r < MBW; ++r)
#pragma unroll
    for (int c = 0; c < NBMAX; ++c)
      if (c < NB) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (wave * MBW + r) * 16 + acc_row<P>(lane, v);
          out[(size_t)row * NT + c * 16 + (lane & 15)] = (part_t)acc[r][c][v];
        }
      }
}



template <int P, typename Tin, bool NN, bool VEC, int MT, int KT>
hipError_t launch_g(const XgArgs& g, hipStream_t s) {
  using op_t = typename PT<P>::op_t;
  const size_t lds = (size_t)(MT + (P == TR_FP8 ? 2 : 1) * g.NT) * (KT + Pad<P>::v) * sizeof(op_t);
  const dim3 grid = g.xcd_map ? dim3((unsigned)(g.n_mt * g.n_nt * g.nsplit)) : dim3(g.n_mt * g.n_nt, g.nsplit);
  auto k = xgemm_kernel<P, Tin, NN, VEC, MT, KT, 8>;
  LDSCHK((const void*)k, lds);
  hipLaunchKernelGGL(k, grid, dim3(NTHR), lds, s, g);
  return hipGetLastError();
}

// Vector loads of A: rows of the fastest-modes group when the operand type is
// the stored type and the rows start 16-byte aligned (vec_ok).
template <int P, typename Tin, bool NN, int MT, int KT>
hipError_t launch_v(const XgArgs& g, hipStream_t s) {
  constexpr bool can_vec = !NN && sizeof(Tin) == sizeof(typename PT<P>::op_t);
  if (can_vec && g.vec_ok) return launch_g<P, Tin, NN, can_vec, MT, KT>(g, s);
  return launch_g<P, Tin, NN, false, MT, KT>(g, s);
}

template <int P, typename Tin>
hipError_t launch_p(const XgArgs& g, hipStream_t s) {
  constexpr int KT = (P == TR_F64) ? 32 : 64;
  if (g.MT == 64) return g.nn ? launch_v<P, Tin, true, 64, KT>(g, s) : launch_v<P, Tin, false, 64, KT>(g, s);
  return g.nn ? launch_v<P, Tin, true, 128, KT>(g, s) : launch_v<P, Tin, false, 128, KT>(g, s);
}

}  // namespace
int xgemm_kt(int prec) { return prec == TR_F64 ? 32 : 64; }

hipError_t launch_xgemm(const XgArgs& g, int prec, int xdt, hipStream_t s) {
  if (prec == TR_F64) return xdt == TR_F64 ? launch_p<TR_F64, double>(g, s) : launch_p<TR_F64, float>(g, s);
  if (prec == TR_F32) return xdt == TR_F64 ? launch_p<TR_F32, double>(g, s) : launch_p<TR_F32, float>(g, s);
  if (prec == TR_BF16) return launch_p<TR_BF16, __bf16>(g, s);
  return launch_p<TR_FP8, uint8_t>(g, s);
}
