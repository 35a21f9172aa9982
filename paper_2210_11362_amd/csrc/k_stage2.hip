// Stage 2 of the two-stage MTTSP (Alg. 2's MTTSP step): operand tables for
// the stage-1 GEMM (Sec. 2 subchain product), the ordered split-K reduction
// of its partial tiles into the FP64 intermediate, and the absorptions of the
// remaining modes into M_n.  All FP64, deterministic reduction orders.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "../../include/tr_als.h"

namespace {

// Y[r + M*c] = out_scale * sum over splits of the partial tiles (fixed
// order).  A workgroup takes a block of 64 rows x 16 columns of one tile:
// partial rows are read as 16-column runs (row-major tiles), summed,
// transposed through LDS and written as 64-row runs of the column-major Y.
// Each thread has four elements.
template <int P>
__global__ __launch_bounds__(256) void xg_reduce_kernel(XgArgs g, int MT, double out_scale, double* Y, int* status) {
  using part_t = typename std::conditional<P == TR_F64, double, float>::type;
  if (g.tmax) out_scale /= fp8_table_scale(*g.tmax);   // FP8: undo the table's scale
  __shared__ double tl[16][65];
  const int NT = g.NT;
  const int64_t tsz = (int64_t)MT * NT;
  const int64_t ntile = (int64_t)g.n_mt * g.n_nt;
  const int rbs = MT / 64, cbs = NT / 16;
  const int64_t tile = blockIdx.x / (rbs * cbs);
  const int rem = (int)(blockIdx.x % (rbs * cbs));
  const int rb = (rem % rbs) * 64, cb = (rem / rbs) * 16;
  const int mt = (int)(tile % g.n_mt), nt = (int)(tile / g.n_mt);
  const part_t* base = reinterpret_cast<const part_t*>(g.partial) + tile * tsz + (int64_t)rb * NT + cb;
  const size_t ss = (size_t)(ntile * tsz);
  // up to SB splits of all four elements in flight at once (clamped indices:
  // the surplus loads repeat the last split and are not summed), summed in
  // split order
  constexpr int SB = 12;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sp0 = 0; sp0 < g.nsplit; sp0 += SB) {
    part_t v[4][SB];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q, row = e >> 4, col = e & 15;
      const part_t* p = base + (int64_t)row * NT + col;
#pragma unroll
      for (int u = 0; u < SB; ++u) v[q][u] = p[(size_t)min(sp0 + u, g.nsplit - 1) * ss];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < SB; ++u) acc[q] += sp0 + u < g.nsplit ? (double)v[q][u] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q, row = e >> 4, col = e & 15;
    tl[col][row] = acc[q] * out_scale;
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q, col = e >> 6, row = e & 63;
    const int64_t r = (int64_t)mt * MT + rb + row, c = (int64_t)nt * NT + cb + col;
    if (r < g.M && c < g.C) {
      const double v = tl[col][row];
      bad = bad || !isfinite(v);
      Y[r + g.M * c] = v;
    }
  }
  if (bad) atomicOr(status, ST_NONFINITE);
}

// FP8: Bt holds the hi part in rows [0, Crows) and the lo part in rows
// [Crows, 2 Crows), at the scale derived from the device max |T|.
__global__ void table_to_bt_fp8_kernel(const double* T, int64_t K, int C, int Crows, int64_t ldb, const double* tmax,
                                       uint8_t* Bt) {
  const int64_t c = blockIdx.y;
  const double sc = fp8_table_scale(*tmax);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ldb; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = c * ldb + k;
    const double v = (c < C && k < K) ? T[k * C + c] * sc : 0.0;
    const uint8_t hi = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32((float)v, 0.0f, 0, false) & 0xff);
    const double r = v - (double)__builtin_amdgcn_cvt_f32_fp8((int)hi, 0);
    Bt[e] = hi;
    Bt[e + (int64_t)Crows * ldb] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32((float)r, 0.0f, 0, false) & 0xff);
  }
}

// Bt[c * ldb + k] = op(T[k * C + c] * scale), zero for k >= K or c >= C (padding).
template <typename O>
__global__ void table_to_bt_kernel(const double* T, int64_t K, int C, int Crows, int64_t ldb, double scale, O* Bt) {
  const int64_t c = blockIdx.y;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ldb; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = c * ldb + k;
    const double v = (c < C && k < K) ? T[k * C + c] * scale : 0.0;
    if constexpr (std::is_same<O, uint8_t>::value)
      Bt[e] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32((float)v, 0.0f, 0, false) & 0xff);
    else if constexpr (std::is_same<O, __bf16>::value)
      Bt[e] = (__bf16)(float)v;
    else
      Bt[e] = (O)v;
  }
}

// Operand table of a group of one or two cores straight from the cores (no
// FP64 table in between): entry k = j + I0*i of the partial subchain
// G0(:, j, :) G1(:, i, :) (one core: G0(:, k, :)), column r + Rl*c, written
// transposed and zero-padded like table_to_bt_kernel.  A workgroup forms the
// Rl x 64 entries (r, k) of one c and 64 consecutive k, summing over the
// inner bond in increasing order in FP64, with r fastest across lanes so that
// the reads of G0 (r fastest in memory) are contiguous; the tile goes through
// LDS and is stored with k fastest.  blockIdx.y = c; the last y row writes the
// padding rows C..Crows-1.
constexpr int GBT_K = 64;
template <typename O>
__global__ __launch_bounds__(256) void group_bt_kernel(const double* G0, int Rl, int64_t I0, int Rm,
                                                       const double* G1, int64_t I1, int two, int64_t K, int C,
                                                       int Crows, int64_t ldb, O* Bt) {
  extern __shared__ double tile[];   // [Rl][GBT_K + 1]
  const int c = blockIdx.y, Rc = C / Rl, tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * GBT_K;
  auto put = [&](int col, int64_t k, double v) {
    if constexpr (std::is_same<O, __bf16>::value) Bt[col * ldb + k] = (__bf16)(float)v;
    else Bt[col * ldb + k] = (O)v;
  };
  if (c == Rc) {   // padding rows
    for (int e = tid; e < (Crows - C) * GBT_K; e += 256) {
      const int col = C + e / GBT_K, kk = e % GBT_K;
      if (k0 + kk < ldb) put(col, k0 + kk, 0.0);
    }
    return;
  }
  for (int e = tid; e < Rl * GBT_K; e += 256) {
    const int r = e % Rl, kk = e / Rl;
    const int64_t k = k0 + kk;
    double acc = 0.0;
    if (k < K) {
      if (two) {
        const int64_t j = k % I0, i = k / I0;
        const double* g0 = G0 + r + (int64_t)Rl * j;
        const double* g1 = G1 + (int64_t)Rm * (i + I1 * c);
        const int64_t st = (int64_t)Rl * I0;
#pragma unroll 10
        for (int m = 0; m < Rm; ++m) acc = fma(g0[st * m], g1[m], acc);
      } else {
        acc = G0[r + (int64_t)Rl * (k + I0 * c)];
      }
    }
    tile[r * (GBT_K + 1) + kk] = acc;
  }
  __syncthreads();
  for (int e = tid; e < Rl * GBT_K; e += 256) {
    const int r = e / GBT_K, kk = e % GBT_K;
    if (k0 + kk < ldb) put(r + Rl * c, k0 + kk, tile[r * (GBT_K + 1) + kk]);
  }
}

// Stage 2: absorb one mode of the intermediate.  Y is [lo][I][hi][bond] with
// bond = u + Ru*c.  side 0 contracts u with the core's right index (new u =
// core's left index); side 1 contracts c with the core's left index (new c =
// core's right index).  Out is [lo][hi][bond'].  When final != 0 the one mode
// left (lo*hi = I_n) is written as M[i + I_n*(c + Rc*u)]: the column order
// a + R_n*b of G_n(2) with a = c, b = u.
//
// Lanes run over l when lo is wide (coalesced reads of Y); otherwise one
// workgroup reduces one output over (i, x).  Either way the reduction order is
// fixed, so the result is deterministic.
struct AbsorbArgs {
  const double* Y; int64_t lo, I, hi; int Ru, Rc; const double* core; int Rl, Rr, side, final_out; double* out;
};

__device__ __forceinline__ double absorb_term2(const AbsorbArgs& a, int64_t l, int64_t h, int u2, int c2, int64_t i,
                                              int x) {
  const int64_t sI = a.lo, sH = a.lo * a.I, sB = a.lo * a.I * a.hi;
  if (a.side == 0)
    return a.core[u2 + (int64_t)a.Rl * (i + a.I * x)] * a.Y[l + sI * i + sH * h + sB * (x + (int64_t)a.Ru * c2)];
  return a.Y[l + sI * i + sH * h + sB * (u2 + (int64_t)a.Ru * x)] * a.core[x + (int64_t)a.Rc * (i + a.I * c2)];
}

__device__ __forceinline__ void absorb_store(const AbsorbArgs& a, int64_t l, int64_t h, int u2, int c2, double v) {
  const int Ru2 = a.side == 0 ? a.Rl : a.Ru;
  const int Rc2 = a.side == 0 ? a.Rc : a.Rr;
  if (a.final_out) a.out[(l + a.lo * h) + a.lo * a.hi * (c2 + (int64_t)Rc2 * u2)] = v;
  else a.out[l + a.lo * (h + a.hi * (u2 + (int64_t)Ru2 * c2))] = v;
}

// lanes over 64 consecutive l; 16 waves split the i range, each keeping 4 rows
// of loads in flight; grid (l-blocks, hi, bond')
__global__ __launch_bounds__(1024) void absorb_lanes_kernel(AbsorbArgs a) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t l = (int64_t)blockIdx.x * 64 + lane;
  const int64_t h = blockIdx.y;
  const int Ru2 = a.side == 0 ? a.Rl : a.Ru;
  const int bnd = blockIdx.z;
  const int u2 = bnd % Ru2, c2 = bnd / Ru2;
  const int R = a.side == 0 ? a.Ru : a.Rc;
  const int64_t i0 = a.I * wave / 16, i1 = a.I * (wave + 1) / 16;
  double s = 0.0;
  if (l < a.lo) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int x = 0; x < R; ++x) {
      int64_t i = i0;
      for (; i + 4 <= i1; i += 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s4[q] += absorb_term2(a, l, h, u2, c2, i + q, x);
      }
      for (; i < i1; ++i) s4[0] += absorb_term2(a, l, h, u2, c2, i, x);
    }
    s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && l < a.lo) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += red[w][lane];
    absorb_store(a, l, h, u2, c2, t);
  }
}

// one workgroup per output; 256 threads split the (i, x) range
__global__ __launch_bounds__(256) void absorb_block_kernel(AbsorbArgs a) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int Ru2 = a.side == 0 ? a.Rl : a.Ru;
  const int64_t e = blockIdx.x;
  const int64_t l = e % a.lo, h = (e / a.lo) % a.hi;
  const int bnd = (int)(e / (a.lo * a.hi));
  const int u2 = bnd % Ru2, c2 = bnd / Ru2;
  const int R = a.side == 0 ? a.Ru : a.Rc;
  const int64_t T = a.I * R;
  double s = 0.0;
  for (int64_t t = tid; t < T; t += 256) s += absorb_term2(a, l, h, u2, c2, t / R, (int)(t % R));
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) absorb_store(a, l, h, u2, c2, red[0]);
}

// Narrow fast extents (lo < 32) as a tall-skinny product: output row
// (l, h, p) x column f, summed over k = (i, x) with i fastest.  A lane owns
// one row and all Rf columns; the waves of a workgroup and S workgroups split
// the k range; core values are wave-uniform (scalar loads).  Partial sums are
// combined in a fixed order (waves in LDS, workgroups by absorb_sum_kernel).
__device__ __forceinline__ int64_t absorb_index(const AbsorbArgs& a, int64_t l, int64_t h, int u2, int c2) {
  const int Ru2 = a.side == 0 ? a.Rl : a.Ru;
  const int Rc2 = a.side == 0 ? a.Rc : a.Rr;
  if (a.final_out) return (l + a.lo * h) + a.lo * a.hi * (c2 + (int64_t)Rc2 * u2);
  return l + a.lo * (h + a.hi * (u2 + (int64_t)Ru2 * c2));
}

template <int B, bool SIDE0>
__global__ __launch_bounds__(256) void absorb_narrow_kernel(AbsorbArgs a, double* part, int64_t out_elems) {
  __shared__ double red[4][B][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Rx = SIDE0 ? a.Ru : a.Rc, Rf = SIDE0 ? a.Rl : a.Rr, Rp = SIDE0 ? a.Rc : a.Ru;
  const int64_t LH = a.lo * a.hi, rows = LH * Rp;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const bool live = r < rows;
  const int64_t rc = live ? r : 0;
  const int64_t lh = rc % LH, l = lh % a.lo, h = lh / a.lo;
  const int p = (int)(rc / LH);
  const int64_t sB = a.lo * a.I * a.hi;
  const double* yrow = a.Y + l + a.lo * a.I * h + sB * (SIDE0 ? (int64_t)a.Ru * p : (int64_t)p);
  const int64_t sx = SIDE0 ? sB : sB * a.Ru;   // Y stride of x
  // k range of this workgroup, then of this wave
  const int64_t K = a.I * Rx, S = gridDim.y;
  const int64_t kb = K * blockIdx.y / S, ke = K * (blockIdx.y + 1) / S;
  const int64_t k0 = kb + (ke - kb) * wave / 4, k1 = kb + (ke - kb) * (wave + 1) / 4;
  double acc[B];
#pragma unroll
  for (int f = 0; f < B; ++f) acc[f] = 0.0;
  int64_t i = k0 % a.I;
  int x = (int)(k0 / a.I);
  const int64_t cf = SIDE0 ? 1 : (int64_t)a.Rc * a.I;   // core stride of f
  for (int64_t k = k0; k < k1; k += 4) {   // four values of k per step: their loads in flight together
    double y[4];
    int64_t ii[4];
    int xx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = live && k + u < k1;
      ii[u] = i;
      xx[u] = x;
      const double v = yrow[ok ? a.lo * i + sx * x : 0];
      y[u] = ok ? v : 0.0;
      if (++i == a.I) { i = 0; ++x; }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int xu = k + u < k1 ? xx[u] : 0;   // clamped: the term is zero anyway
      const int64_t iu = k + u < k1 ? ii[u] : 0;
      const double* c = SIDE0 ? a.core + (int64_t)a.Rl * (iu + a.I * xu) : a.core + xu + (int64_t)a.Rc * iu;
#pragma unroll
      for (int f = 0; f < B; ++f) acc[f] = fma(y[u], c[cf * (f < Rf ? f : 0)], acc[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < B; ++f) red[wave][f][lane] = acc[f];
  __syncthreads();
  if (wave == 0 && live) {
    for (int f = 0; f < Rf; ++f) {
      const double v = (red[0][f][lane] + red[1][f][lane]) + (red[2][f][lane] + red[3][f][lane]);
      const int64_t e = absorb_index(a, l, h, SIDE0 ? f : p, SIDE0 ? p : f);
      if (S == 1) a.out[e] = v;
      else part[blockIdx.y * out_elems + e] = v;
    }
  }
}

// Single-read absorption.  With x the contracted bond index, p the passive
// one and f the free index of the core (side 0: x = u, p = c, f = the core's
// left index; side 1: x = c, p = u, f = the core's right index), output
// (l, h, p, f) is the sum over (i, x) of Y[l, i, h, bond(x, p)] core(f, i, x).
// A lane keeps all f of its output group in registers, so every Y element is
// loaded once, and issues the Rx loads of one i together (memory-level
// parallelism); core values come from LDS as wave-uniform broadcasts.
// Lanes run on l (lo >= 32: narrow fast extents use the one-output-per-
// workgroup kernel above); 8 waves and S workgroups split i, and the partial
// sums are added in a fixed order.
struct Absorb2 {
  const double* Y; int64_t lo, I, hi; int Ru, Rc, Rl, Rr, final_out; const double* core; double* out;
  double* part; int S; int64_t out_elems;
};

template <bool SIDE0>
__device__ __forceinline__ int64_t absorb2_out(const Absorb2& a, int64_t l, int64_t h, int p, int f) {
  const int u2 = SIDE0 ? f : p, c2 = SIDE0 ? p : f;
  const int Ru2 = SIDE0 ? a.Rl : a.Ru, Rc2 = SIDE0 ? a.Rc : a.Rr;
  if (a.final_out) return (l + a.lo * h) + a.lo * a.hi * (c2 + (int64_t)Rc2 * u2);
  return l + a.lo * (h + a.hi * (u2 + (int64_t)Ru2 * c2));
}

// core(f, i, x) -> cs[((i - i0) * Rx + x) * Rf + f] for i in [i0, i1)
template <bool SIDE0>
__device__ __forceinline__ void absorb2_stage_core(const Absorb2& a, int64_t i0, int64_t i1, double* cs) {
  const int Rx = SIDE0 ? a.Ru : a.Rc, Rf = SIDE0 ? a.Rl : a.Rr;
  const int n = (int)((i1 - i0) * Rx * Rf);   // a slice of one core: 32-bit offsets
  const int bd = blockDim.x;
  for (int e0 = 0; e0 < n; e0 += 4 * bd) {    // four loads in flight per thread (clamped index)
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + (int)threadIdx.x + u * bd, ec = e < n ? e : 0;
      const int f = ec % Rf, q = ec / Rf, x = q % Rx;
      const int64_t i = i0 + q / Rx;
      v[u] = SIDE0 ? a.core[f + (int64_t)a.Rl * (i + a.I * x)] : a.core[x + (int64_t)a.Rc * (i + a.I * f)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + (int)threadIdx.x + u * bd < n) cs[e0 + threadIdx.x + u * bd] = v[u];
  }
}

constexpr int AW_WAVES = 8;

// EXACT: Rx == Rf == B, so every rank loop has a fixed trip count.
template <int B, bool SIDE0, bool EXACT>
__global__ __launch_bounds__(64 * AW_WAVES) void absorb_wide_kernel(Absorb2 a, int64_t chunk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* cs = reinterpret_cast<double*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t l = (int64_t)blockIdx.x * 64 + lane;
  const int Rx = EXACT ? B : (SIDE0 ? a.Ru : a.Rc), Rf = EXACT ? B : (SIDE0 ? a.Rl : a.Rr);
  const int64_t h = blockIdx.y % a.hi;
  const int p = (int)(blockIdx.y / a.hi);
  const int sp = blockIdx.z;
  const int64_t ib = (int64_t)sp * chunk, ie = min(a.I, ib + chunk);
  absorb2_stage_core<SIDE0>(a, ib, ie, cs);
  __syncthreads();
  const int64_t i0 = ib + (ie - ib) * wave / AW_WAVES, i1 = ib + (ie - ib) * (wave + 1) / AW_WAVES;
  double acc[B];
#pragma unroll
  for (int f = 0; f < B; ++f) acc[f] = 0.0;
  const int64_t sx = SIDE0 ? a.lo * a.I * a.hi : a.lo * a.I * a.hi * a.Ru;   // Y stride of x
  const int64_t y0 = l + a.lo * a.I * h + a.lo * a.I * a.hi * (SIDE0 ? (int64_t)a.Ru * p : (int64_t)p);
  if (l < a.lo) {
    for (int64_t i = i0; i < i1; ++i) {
      double y[B];
#pragma unroll
      for (int x = 0; x < B; ++x) {   // unconditional loads (clamped index): all in flight together
        const double v = a.Y[y0 + a.lo * i + sx * (EXACT || x < Rx ? x : 0)];
        y[x] = EXACT || x < Rx ? v : 0.0;
      }
      const double* c = cs + (i - ib) * Rx * Rf;
#pragma unroll
      for (int x = 0; x < B; ++x) {
        if (EXACT || x < Rx) {
#pragma unroll
          for (int f = 0; f < B; ++f)
            if (EXACT || f < Rf) acc[f] += y[x] * c[x * Rf + f];
        }
      }
    }
  }
  __syncthreads();   // the core slice is dead: its LDS holds the wave partials now
  double* red = cs;  // [AW_WAVES][B][64]
#pragma unroll
  for (int f = 0; f < B; ++f) red[(wave * B + f) * 64 + lane] = acc[f];
  __syncthreads();
  if (wave == 0 && l < a.lo) {
    for (int f = 0; f < Rf; ++f) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < AW_WAVES; ++w) v += red[(w * B + f) * 64 + lane];
      const int64_t e = absorb2_out<SIDE0>(a, l, h, p, f);
      if (a.S == 1) a.out[e] = v;
      else a.part[(int64_t)sp * a.out_elems + e] = v;
    }
  }
}

// out[e] = sum over splits s (in order) of part[s][e]
__global__ void absorb_sum_kernel(const double* part, int S, int64_t n, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += part[(int64_t)s * n + e];
  out[e] = v;
}

// M[i + In*(c + Rc*u)] = Y[i + In*(u + Ru*c)] : final reordering when no mode is
// left to absorb.
__global__ void bond_to_M_kernel(const double* Y, int64_t In, int Ru, int Rc, double* M) {
  const int64_t n = In * Ru * Rc;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t i = e % In;
  const int b = (int)(e / In);
  const int u = b % Ru, c = b / Ru;
  M[i + In * (c + (int64_t)Rc * u)] = Y[e];
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_xg_reduce(const XgArgs& g, int prec, double out_scale, double* Y, int* status, hipStream_t s) {
  const int64_t blocks = (int64_t)g.n_mt * g.n_nt * (g.MT / 64) * (g.NT / 16);
  if (prec == TR_F64)
    hipLaunchKernelGGL(xg_reduce_kernel<TR_F64>, dim3((unsigned)blocks), dim3(256), 0, s, g, g.MT, out_scale, Y, status);
  else
    hipLaunchKernelGGL(xg_reduce_kernel<TR_F32>, dim3((unsigned)blocks), dim3(256), 0, s, g, g.MT, out_scale, Y, status);
  return hipGetLastError();
}

hipError_t launch_table_to_bt(const double* T, int64_t K, int C, int Crows, int64_t ldb, int prec, double scale,
                              void* Bt, hipStream_t s, const double* tmax) {
  const dim3 grid((unsigned)std::min<int64_t>(cdiv(ldb, 256), 64), (unsigned)Crows);
  if (prec == TR_FP8) {
    if (!tmax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(table_to_bt_fp8_kernel, grid, dim3(256), 0, s, T, K, C, Crows, ldb, tmax, (uint8_t*)Bt);
    return hipGetLastError();
  }
  switch (prec) {
    case TR_F64: hipLaunchKernelGGL(table_to_bt_kernel<double>, dim3(grid), dim3(256), 0, s, T, K, C, Crows, ldb, scale, (double*)Bt); break;
    case TR_F32: hipLaunchKernelGGL(table_to_bt_kernel<float>, dim3(grid), dim3(256), 0, s, T, K, C, Crows, ldb, scale, (float*)Bt); break;
    case TR_BF16: hipLaunchKernelGGL(table_to_bt_kernel<__bf16>, dim3(grid), dim3(256), 0, s, T, K, C, Crows, ldb, scale, (__bf16*)Bt); break;
    default: hipLaunchKernelGGL(table_to_bt_kernel<uint8_t>, dim3(grid), dim3(256), 0, s, T, K, C, Crows, ldb, scale, (uint8_t*)Bt); break;
  }
  return hipGetLastError();
}

hipError_t launch_group_bt(const double* G0, int Rl, int64_t I0, int Rm, const double* G1, int64_t I1, int two,
                           int64_t K, int C, int Crows, int64_t ldb, int prec, void* Bt, hipStream_t s) {
  if (Rl > 24) return hipErrorInvalidValue;
  const dim3 grid((unsigned)cdiv(ldb, GBT_K), (unsigned)(C / Rl + 1));
  const size_t lds = (size_t)Rl * (GBT_K + 1) * sizeof(double);
  switch (prec) {
    case TR_F64:
      hipLaunchKernelGGL(group_bt_kernel<double>, grid, dim3(256), lds, s, G0, Rl, I0, Rm, G1, I1, two, K, C, Crows, ldb,
                         (double*)Bt);
      break;
    case TR_F32:
      hipLaunchKernelGGL(group_bt_kernel<float>, grid, dim3(256), lds, s, G0, Rl, I0, Rm, G1, I1, two, K, C, Crows, ldb,
                         (float*)Bt);
      break;
    case TR_BF16:
      hipLaunchKernelGGL(group_bt_kernel<__bf16>, grid, dim3(256), lds, s, G0, Rl, I0, Rm, G1, I1, two, K, C, Crows,
                         ldb, (__bf16*)Bt);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

constexpr size_t ABSORB_LDS_MAX = 96 * 1024;

template <int B, bool SIDE0, bool EXACT>
hipError_t launch_absorb2(const Absorb2& a, hipStream_t s) {
  const int Rx = SIDE0 ? a.Ru : a.Rc, Rf = SIDE0 ? a.Rl : a.Rr, Rp = SIDE0 ? a.Rc : a.Ru;
  const size_t row = (size_t)Rx * Rf * sizeof(double);   // core bytes per value of i
  if (a.lo >= 32) {
    const int64_t chunk = cdiv(a.I, a.S);
    const size_t lds = std::max((size_t)chunk * row, (size_t)AW_WAVES * B * 64 * sizeof(double));
    LDSCHK(((const void*)absorb_wide_kernel<B, SIDE0, EXACT>), lds);
    dim3 grid((unsigned)cdiv(a.lo, 64), (unsigned)(a.hi * Rp), (unsigned)cdiv(a.I, chunk));
    hipLaunchKernelGGL((absorb_wide_kernel<B, SIDE0, EXACT>), grid, dim3(64 * AW_WAVES), lds, s, a, chunk);
    if (a.S > 1)
      hipLaunchKernelGGL(absorb_sum_kernel, dim3((unsigned)cdiv(a.out_elems, 256)), dim3(256), 0, s, a.part, a.S,
                         a.out_elems, a.out);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_absorb(const double* Y, int64_t lo, int64_t I, int64_t hi, int Ru, int Rc, const double* core,
                         int Rl, int Rr, int side, int final_out, double* out, double* part, size_t part_bytes,
                         hipStream_t s) {
  const int Ru2 = side == 0 ? Rl : Ru, Rc2 = side == 0 ? Rc : Rr;
  const int Rx = side == 0 ? Ru : Rc, Rf = side == 0 ? Rl : Rr, Rp = side == 0 ? Rc : Ru;
  const int64_t out_elems = lo * hi * Ru2 * Rc2;
  const size_t row = (size_t)Rx * Rf * sizeof(double);
  const int Bn = std::max(Rx, Rf);
  if (lo >= 32 && Bn <= 24 && row * AW_WAVES <= ABSORB_LDS_MAX) {
    Absorb2 a{Y, lo, I, hi, Ru, Rc, Rl, Rr, final_out, core, out, part, 1, out_elems};
    // split i over workgroups until there are ~1024 of them, at least 2 values
    // of i per wave, within the LDS budget for the core slice and the
    // partial-sum buffer
    const int64_t groups = cdiv(lo, 64) * hi * Rp;
    int64_t S = std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, groups), I / (2 * AW_WAVES)));
    while (S > 1 && ((size_t)S * out_elems * sizeof(double) > part_bytes)) --S;
    while ((size_t)cdiv(I, S) * row > ABSORB_LDS_MAX) ++S;
    a.S = (int)cdiv(I, cdiv(I, S));
    if (a.S > 1 && (size_t)a.S * out_elems * sizeof(double) > part_bytes) a.S = 0;   // no room: other kernels
    if (a.S > 0) {
      if (Rx == Rf) {   // equal ranks: fixed trip counts for the common ones
        switch (Rx) {
#define AW_EXACT(R) \
  case R: return side == 0 ? launch_absorb2<R, true, true>(a, s) : launch_absorb2<R, false, true>(a, s);
          AW_EXACT(4) AW_EXACT(8) AW_EXACT(10) AW_EXACT(12) AW_EXACT(16) AW_EXACT(20)
#undef AW_EXACT
          default: break;
        }
      }
      if (side == 0) {
        if (Bn <= 8) return launch_absorb2<8, true, false>(a, s);
        if (Bn <= 16) return launch_absorb2<16, true, false>(a, s);
        return launch_absorb2<24, true, false>(a, s);
      }
      if (Bn <= 8) return launch_absorb2<8, false, false>(a, s);
      if (Bn <= 16) return launch_absorb2<16, false, false>(a, s);
      return launch_absorb2<24, false, false>(a, s);
    }
  }
  AbsorbArgs a{Y, lo, I, hi, Ru, Rc, core, Rl, Rr, side, final_out, out};
  if (lo >= 32) {
    dim3 grid((unsigned)cdiv(lo, 64), (unsigned)hi, (unsigned)(Ru2 * Rc2));
    hipLaunchKernelGGL(absorb_lanes_kernel, grid, dim3(1024), 0, s, a);
  } else if (Rf <= 24 && cdiv(lo * hi * Rp, 64) <= 0x7fffffff) {
    const int64_t rb = cdiv(lo * hi * Rp, 64);
    // k splits until ~512 workgroups, at least 64 values of k per split, within the partial buffer
    int64_t S = std::max<int64_t>(1, std::min<int64_t>(cdiv(512, rb), (I * Rx) / 64));
    S = std::min<int64_t>(S, 65535);
    while (S > 1 && (size_t)S * out_elems * sizeof(double) > part_bytes) --S;
    const dim3 grid((unsigned)rb, (unsigned)S);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, a, part, out_elems); };
    if (side == 0) {
      if (Rf <= 8) go(absorb_narrow_kernel<8, true>);
      else if (Rf <= 16) go(absorb_narrow_kernel<16, true>);
      else go(absorb_narrow_kernel<24, true>);
    } else {
      if (Rf <= 8) go(absorb_narrow_kernel<8, false>);
      else if (Rf <= 16) go(absorb_narrow_kernel<16, false>);
      else go(absorb_narrow_kernel<24, false>);
    }
    if (S > 1)
      hipLaunchKernelGGL(absorb_sum_kernel, dim3((unsigned)cdiv(out_elems, 256)), dim3(256), 0, s, part, (int)S,
                         out_elems, out);
  } else {
    hipLaunchKernelGGL(absorb_block_kernel, dim3((unsigned)(lo * hi * Ru2 * Rc2)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_bond_to_M(const double* Y, int64_t In, int Ru, int Rc, double* M, hipStream_t s) {
  const int64_t n = In * Ru * Rc;
  hipLaunchKernelGGL(bond_to_M_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, Y, In, Ru, Rc, M);
  return hipGetLastError();
}
