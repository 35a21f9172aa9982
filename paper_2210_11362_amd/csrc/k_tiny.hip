// Batched lane of the serving loop: one persistent workgroup runs a whole
// small TR-ALS job (every sweep of Alg. 2 with the normal-equation solve, then
// the fit), and one launch carries many jobs, so a job costs no kernel
// launches of its own.  Per mode update m, inside the workgroup:
//   1. partial-subchain tables of the modes after m (TA, entries t) and before
//      m (TB, entries l), FP64;
//   2. M_m[i, a + R_m b] = sum_{l,t} X(l, i, t) sum_c TA[t][b, c] TB[l][c, a]
//      in tiles of 32 (l, t) pairs: subchain rows and X rounded to the
//      contraction type, FP32 accumulation (FP64 for the FP64 path);
//   3. W = K_{m+1} ... K_{m-1} from the Kronecker-form Grams (Prop. 3.1),
//      S_m realigned from W, Cholesky in LDS;
//   4. G = M S^{-1} by substitution, refinement G += (M - G S) S^{-1};
//   5. non-finite / breakdown checks latch the job's status word; otherwise
//      core m and its Gram are replaced.
// Limits (checked by the host): order 2..4, R_k <= 8, I_k <= 128,
// prod(I_k) <= 2^18; contraction types FP64, FP32, BF16.
#include <algorithm>

#include "common.h"
#include "tiny.h"
#include "../../include/tr_als.h"

namespace {

constexpr int TT = 256;      // threads per job
constexpr int KP = 32;       // (l, t) pairs per contraction tile
constexpr int RRMAX = 64;
constexpr int IMAX = 128;
constexpr int QMAX = IMAX * RRMAX / TT;   // M entries per thread

struct Shape {
  int N;
  int64_t dims[4];
  int R[5];
};

__device__ __forceinline__ float to_bf16f(float v) { return (float)(__bf16)v; }

// table of the chain of cores cl[0..cnt) (first index fastest over the chain's
// mode indices): out[e * Rl * Rr + r + Rl * c] = (G_{cl0}(i0) ... )[r, c]
__device__ void tiny_chain(const Shape& s, double* const* cores, const int* cl, int cnt, double* out, double* tmp,
                           int64_t* entries) {
  const int tid = threadIdx.x;
  if (cnt == 0) {
    *entries = 1;
    return;
  }
  const int Rl = s.R[cl[0]];
  int64_t J = s.dims[cl[0]];
  double* cur = (cnt == 1) ? out : ((cnt % 2 == 0) ? tmp : out);
  {
    const int k = cl[0], Rr = s.R[k + 1];
    const int64_t n = (int64_t)Rl * J * Rr;
    for (int64_t e = tid; e < n; e += TT) {
      const int r = (int)(e % Rl);
      const int64_t i = (e / Rl) % J;
      const int c = (int)(e / ((int64_t)Rl * J));
      cur[i * Rl * Rr + r + (int64_t)Rl * c] = cores[k][e];
    }
  }
  __syncthreads();
  for (int q = 1; q < cnt; ++q) {
    const int k = cl[q], Rm = s.R[k], Rr = s.R[k + 1];
    const int64_t I = s.dims[k];
    double* nxt = (cur == out) ? tmp : out;
    const int64_t n = J * I * Rl * Rr;
    for (int64_t e = tid; e < n; e += TT) {
      const int64_t ent = e / ((int64_t)Rl * Rr);
      const int rc = (int)(e % ((int64_t)Rl * Rr));
      const int r = rc % Rl, c = rc / Rl;
      const int64_t j = ent % J, i = ent / J;
      const double* t = cur + j * (int64_t)Rl * Rm;
      const double* g = cores[k] + i * Rm + (int64_t)Rm * I * c;
      double acc = 0.0;
      for (int m = 0; m < Rm; ++m) acc += t[r + (int64_t)Rl * m] * g[m];
      nxt[e] = acc;
    }
    J *= I;
    cur = nxt;
    __syncthreads();
  }
  *entries = J;
}

// Gram of core k: E[p, q] = sum_i G(2)[i, p] G(2)[i, q], p = a + Rl b
__device__ void tiny_gram(const Shape& s, const double* core, int k, double* E) {
  const int Rl = s.R[k], Rr = s.R[k + 1], n = Rl * Rr;
  const int64_t I = s.dims[k];
  for (int e = threadIdx.x; e < n * n; e += TT) {
    const int p = e % n, q = e / n;
    const int64_t op = (p % Rl) + (int64_t)Rl * I * (p / Rl), oq = (q % Rl) + (int64_t)Rl * I * (q / Rl);
    double acc = 0.0;
    for (int64_t i = 0; i < I; ++i) acc += core[op + Rl * i] * core[oq + Rl * i];
    E[e] = acc;
  }
}

template <int P>
struct TinyOp { using t = float; };
template <>
struct TinyOp<TR_F64> { using t = double; };

template <int P>
__device__ __forceinline__ typename TinyOp<P>::t tiny_round(double v) {
  if constexpr (P == TR_F64) return v;
  else if constexpr (P == TR_BF16) return to_bf16f((float)v);
  else return (float)v;
}

// M_m into Mout (I x RR, column-major), contraction type P
template <int P, typename TX>
__device__ void tiny_mttsp(const Shape& s, const TX* X, int m, const double* TA, const double* TB, int64_t T,
                           int64_t L, double* Mout, unsigned char* lds) {
  using op = typename TinyOp<P>::t;
  const int tid = threadIdx.x;
  const int64_t I = s.dims[m];
  const int Ra = s.R[m], Rb = s.R[m + 1], R0 = s.R[0];
  const int RR = Ra * Rb;
  op* Zs = reinterpret_cast<op*>(lds);        // [KP][RR]
  op* Xs = Zs + KP * RRMAX;                   // [KP][I]
  const int64_t K = L * T;
  const int nout = (int)I * RR;
  op acc[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) acc[q] = 0;
  for (int64_t k0 = 0; k0 < K; k0 += KP) {
    const int kv = (int)min((int64_t)KP, K - k0);
    __syncthreads();
    for (int e = tid; e < KP * RR; e += TT) {
      const int kk = e / RR, c = e % RR;
      double z = 0.0;
      if (kk < kv) {
        const int64_t k = k0 + kk, l = k % L, t = k / L;
        const int a = c % Ra, b = c / Ra;
        const double* ta = TA + t * (int64_t)Rb * R0;
        const double* tb = TB + l * (int64_t)R0 * Ra;
        for (int cc = 0; cc < R0; ++cc) z += ta[b + Rb * cc] * tb[cc + R0 * a];
      }
      Zs[e] = tiny_round<P>(z);
    }
    for (int e = tid; e < KP * (int)I; e += TT) {
      const int kk = e / (int)I, i = e % (int)I;
      double x = 0.0;
      if (kk < kv) {
        const int64_t k = k0 + kk, l = k % L, t = k / L;
        x = (double)X[l + L * i + L * I * t];
      }
      Xs[kk * I + i] = tiny_round<P>(x);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int o = tid + TT * q;
      if (o < nout) {
        const int i = o % (int)I, c = o / (int)I;
        op a2 = acc[q];
        for (int kk = 0; kk < KP; ++kk) a2 += Xs[kk * I + i] * Zs[kk * RR + c];
        acc[q] = a2;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int o = tid + TT * q;
    if (o < nout) Mout[o] = (double)acc[q];
  }
  __syncthreads();
}

}  // namespace

namespace {

struct TinyWs {
  int64_t gram[4], ta, tb, tmp, M, G, Res, W0, W1, total;
};

__host__ __device__ inline TinyWs tiny_ws_layout(int N, const int64_t* dims, const int* R) {
  TinyWs w{};
  int64_t off = 0;
  for (int k = 0; k < N; ++k) {
    w.gram[k] = off;
    off += (int64_t)R[k] * R[k + 1] * R[k] * R[k + 1];
  }
  // chain tables pair non-adjacent ranks (R_{m+1} with R_1, R_1 with R_m) and
  // the ring products are R_{m+1}^2 x R_j^2, so they are sized by maxR^2
  int64_t numel = 1, maxI = 1, maxRR = 1, maxR2 = 1, tab = 1;
  for (int k = 0; k < N; ++k) {
    numel *= dims[k];
    maxI = dims[k] > maxI ? dims[k] : maxI;
    maxRR = (int64_t)R[k] * R[k + 1] > maxRR ? (int64_t)R[k] * R[k + 1] : maxRR;
    maxR2 = (int64_t)R[k] * R[k] > maxR2 ? (int64_t)R[k] * R[k] : maxR2;
  }
  for (int k = 0; k < N; ++k) {
    const int64_t rest = numel / dims[k];
    tab = rest * maxR2 > tab ? rest * maxR2 : tab;
  }
  w.ta = off; off += tab;
  w.tb = off; off += tab;
  w.tmp = off; off += tab;
  w.M = off; off += maxI * maxRR;
  w.G = off; off += maxI * maxRR;
  w.Res = off; off += maxI * maxRR;
  w.W0 = off; off += maxR2 * maxR2;
  w.W1 = off; off += maxR2 * maxR2;
  w.total = off;
  return w;
}

// One mode update of job J (normal equations with refinement).
template <typename TX>
__device__ void tiny_update(const TinyJob& J, const Shape& s, const TinyWs& w, int m, int prec, int* bad,
                            unsigned char* lds) {
  const int tid = threadIdx.x;
  const int N = s.N;
  double* ws = J.ws;
  const int Ra = s.R[m], Rb = s.R[m + 1], n = Ra * Rb;
  const int64_t I = s.dims[m];
  // 1. tables: after = m+1..N-1, before = 0..m-1
  int after[4], before[4], na = 0, nb = 0;
  for (int k = m + 1; k < N; ++k) after[na++] = k;
  for (int k = 0; k < m; ++k) before[nb++] = k;
  double* TA = ws + w.ta;
  double* TB = ws + w.tb;
  if (na == 0 || nb == 0) {
    // identity R_0 x R_0 table stands in for an empty chain
    double* id = (na == 0) ? TA : TB;
    for (int e = tid; e < s.R[0] * s.R[0]; e += TT) id[e] = (e % s.R[0] == e / s.R[0]) ? 1.0 : 0.0;
  }
  __syncthreads();
  int64_t T = 1, L = 1;     // the same in every thread
  if (na) tiny_chain(s, J.cores, after, na, TA, ws + w.tmp, &T);
  if (nb) tiny_chain(s, J.cores, before, nb, TB, ws + w.tmp, &L);
  __syncthreads();
  // 2. M
  const TX* X = reinterpret_cast<const TX*>(J.X);
  double* M = ws + w.M;
  if (prec == TR_F64) tiny_mttsp<TR_F64>(s, X, m, TA, TB, T, L, M, lds);
  else if (prec == TR_BF16) tiny_mttsp<TR_BF16>(s, X, m, TA, TB, T, L, M, lds);
  else tiny_mttsp<TR_F32>(s, X, m, TA, TB, T, L, M, lds);
  // 3. W = K_{m+1} ... K_{m-1} (Kronecker-form Grams), S realigned, Cholesky
  double* Wc = ws + w.W0;
  double* Wn = ws + w.W1;
  const int k1 = (m + 1) % N;
  int rows = s.R[k1] * s.R[k1];
  {
    const int Rl = s.R[k1], Rr = s.R[k1 + 1], c2 = Rr * Rr;
    const double* E = ws + w.gram[k1];
    for (int e = tid; e < rows * c2; e += TT) {
      const int r = e % rows, c = e / rows;
      const int b = r % Rl, bp = r / Rl, cc = c % Rr, cp = c / Rr;
      Wc[e] = E[(b + Rl * cc) + (int64_t)(Rl * Rr) * (bp + Rl * cp)];
    }
  }
  __syncthreads();
  for (int q = 2; q < N; ++q) {
    const int k = (m + q) % N;
    const int Rl = s.R[k], Rr = s.R[k + 1], inner = Rl * Rl, cols = Rr * Rr;
    const double* E = ws + w.gram[k];
    for (int e = tid; e < rows * cols; e += TT) {
      const int r = e % rows, c = e / rows;
      const int cc = c % Rr, cp = c / Rr;
      double acc = 0.0;
      for (int j = 0; j < inner; ++j) {
        const int b = j % Rl, bp = j / Rl;
        acc += Wc[r + (int64_t)rows * j] * E[(b + Rl * cc) + (int64_t)(Rl * Rr) * (bp + Rl * cp)];
      }
      Wn[e] = acc;
    }
    __syncthreads();
    double* t = Wc; Wc = Wn; Wn = t;
  }
  // S[(a + Ra b), (a' + Ra b')] = W[(b + Rb b'), (a + Ra a')]; W is Rb^2 x Ra^2
  double* S = reinterpret_cast<double*>(lds);             // n x n in LDS
  for (int e = tid; e < n * n; e += TT) {
    const int p = e % n, q = e / n;
    const int a = p % Ra, b = p / Ra, ap = q % Ra, bp = q / Ra;
    S[e] = Wc[(b + Rb * bp) + (int64_t)(Rb * Rb) * (a + Ra * ap)];
  }
  __syncthreads();
  double* Sg = ws + w.W1 == Wc ? ws + w.W0 : ws + w.W1;   // free global copy of S for the residual
  for (int e = tid; e < n * n; e += TT) Sg[e] = S[e];
  __shared__ int chol_ok;
  if (tid == 0) chol_ok = 1;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = S[k + n * k];
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) chol_ok = 0;
      break;
    }
    const double lkk = sqrt(d), r = 1.0 / lkk;
    __syncthreads();
    if (tid == 0) S[k + n * k] = lkk;
    for (int i = k + 1 + tid; i < n; i += TT) S[i + n * k] *= r;
    __syncthreads();
    const int mm = n - k - 1;
    for (int e = tid; e < mm * mm; e += TT) {
      const int ii = e % mm, jj = e / mm;
      if (ii >= jj) S[(k + 1 + ii) + n * (k + 1 + jj)] -= S[(k + 1 + ii) + n * k] * S[(k + 1 + jj) + n * k];
    }
    __syncthreads();
  }
  __syncthreads();
  if (!chol_ok) {
    if (tid == 0) *bad |= ST_SINGULAR;
    __syncthreads();
    return;
  }
  // 4. G rows: L L^T g = rhs, one thread per row, substitution in place in
  //    the row's buffer (G for the first solve, Res for each correction)
  double* G = ws + w.G;
  double* Res = ws + w.Res;
  for (int pass = 0; pass <= J.refine; ++pass) {
    double* y = pass == 0 ? G : Res;
    for (int64_t i = tid; i < I; i += TT) {
      if (pass == 0)
        for (int p = 0; p < n; ++p) y[i + I * p] = M[i + I * p];
      for (int p = 0; p < n; ++p) {
        double v = y[i + I * p];
        for (int q = 0; q < p; ++q) v -= S[p + n * q] * y[i + I * q];
        y[i + I * p] = v / S[p + n * p];
      }
      for (int p = n - 1; p >= 0; --p) {
        double v = y[i + I * p];
        for (int q = p + 1; q < n; ++q) v -= S[q + n * p] * y[i + I * q];
        y[i + I * p] = v / S[p + n * p];
      }
      if (pass > 0)
        for (int p = 0; p < n; ++p) G[i + I * p] += y[i + I * p];
    }
    __syncthreads();
    if (pass < J.refine) {
      // Res = M - G S
      for (int64_t e = tid; e < I * n; e += TT) {
        const int64_t i = e % I;
        const int q = (int)(e / I);
        double v = M[e];
        for (int p = 0; p < n; ++p) v -= G[i + I * p] * Sg[p + n * q];
        Res[e] = v;
      }
      __syncthreads();
    }
  }
  // 5. checks and commit
  __shared__ int finite_all;
  if (tid == 0) finite_all = 1;
  __syncthreads();
  for (int64_t e = tid; e < I * n; e += TT)
    if (!isfinite(G[e]) || !isfinite(M[e])) finite_all = 0;
  __syncthreads();
  if (!finite_all) {
    if (tid == 0) *bad |= ST_NONFINITE;
    __syncthreads();
    return;
  }
  double* core = J.cores[m];
  for (int64_t e = tid; e < I * n; e += TT) {
    const int a = (int)(e % Ra);
    const int64_t i = (e / Ra) % I;
    const int b = (int)(e / ((int64_t)Ra * I));
    core[e] = G[i + I * (a + (int64_t)Ra * b)];
  }
  __syncthreads();
  tiny_gram(s, core, m, ws + w.gram[m]);
  __syncthreads();
}

template <typename TX>
__device__ void tiny_job(const TinyJob& J, unsigned char* lds) {
  const int tid = threadIdx.x;
  Shape s;
  s.N = J.N;
  for (int k = 0; k < 4; ++k) s.dims[k] = J.dims[k];
  for (int k = 0; k < 5; ++k) s.R[k] = J.R[k];
  const TinyWs w = tiny_ws_layout(s.N, s.dims, s.R);
  const TX* X = reinterpret_cast<const TX*>(J.X);
  int64_t numel = 1;
  for (int k = 0; k < s.N; ++k) numel *= s.dims[k];
  __shared__ double red[TT];
  __shared__ int bad;
  // ||X||^2
  double acc = 0.0;
  for (int64_t e = tid; e < numel; e += TT) acc += (double)X[e] * (double)X[e];
  red[tid] = acc;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int h = TT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double xnorm2 = red[0];
  __syncthreads();
  for (int k = 0; k < s.N; ++k) tiny_gram(s, J.cores[k], k, J.ws + w.gram[k]);
  __syncthreads();
  const int nsw = J.nmixed + J.nfin;
  for (int sw = 0; sw < nsw; ++sw) {
    const int prec = sw < J.nmixed ? J.pmixed : J.pfin;
    for (int m = 0; m < s.N; ++m) tiny_update<TX>(J, s, w, m, prec, &bad, lds);
  }
  // fit: Xhat_[1] = G_1(2) (G^{!=1}_[2])^T, residual accumulated in FP64
  {
    const int m = 0, Ra = s.R[0], Rb = s.R[1], n = Ra * Rb;
    int after[4], na = 0;
    for (int k = 1; k < s.N; ++k) after[na++] = k;
    double* TA = J.ws + w.ta;
    int64_t T;
    tiny_chain(s, J.cores, after, na, TA, J.ws + w.tmp, &T);
    __syncthreads();
    const int64_t I = s.dims[m];
    const double* core = J.cores[0];
    double r2 = 0.0;
    for (int64_t e = tid; e < numel; e += TT) {
      const int64_t i = e % I, t = e / I;
      const double* ta = TA + t * (int64_t)Rb * Ra;
      double xh = 0.0;
      for (int c = 0; c < n; ++c) {
        const int a = c % Ra, b = c / Ra;
        xh += core[a + (int64_t)Ra * (i + I * b)] * ta[b + Rb * a];
      }
      const double d = (double)X[e] - xh;
      r2 += d * d;
    }
    red[tid] = r2;
    __syncthreads();
    for (int h = TT / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) {
      J.scal[0] = xnorm2;
      J.scal[1] = red[0];
      *J.status = bad;
    }
  }
}

__global__ __launch_bounds__(TT) void tiny_als_kernel(const TinyJob* jobs) {
  __shared__ __align__(16) unsigned char lds[(KP * RRMAX + KP * IMAX) * sizeof(double)];
  const TinyJob& J = jobs[blockIdx.x];
  if (J.xdt == TR_F64) tiny_job<double>(J, lds);
  else tiny_job<float>(J, lds);
}

}  // namespace

size_t tiny_ws_bytes(int N, const int64_t* dims, const int64_t* ranks) {
  int R[5];
  for (int k = 0; k < N; ++k) R[k] = (int)ranks[k];
  R[N] = R[0];
  return (size_t)tiny_ws_layout(N, dims, R).total * sizeof(double) + 64;
}

bool tiny_eligible(int N, const int64_t* dims, const int64_t* ranks) {
  if (N < 2 || N > 4) return false;
  int64_t numel = 1;
  for (int k = 0; k < N; ++k) {
    // R_k <= 8 keeps every Kronecker-form Gram within 64 x 64
    if (dims[k] > IMAX || ranks[k] > 8) return false;
    numel *= dims[k];
  }
  return numel <= (int64_t(1) << 18);
}

void tiny_fill(TinyJob* j, int N, const int64_t* dims, const int64_t* ranks, const void* X, int xdt,
               double* const* cores, double* ws, int nmixed, int pmixed, int nfin, int pfin, int refine) {
  *j = TinyJob{};
  j->N = N;
  for (int k = 0; k < N; ++k) { j->dims[k] = dims[k]; j->R[k] = (int)ranks[k]; j->cores[k] = cores[k]; }
  j->R[N] = j->R[0];
  j->X = X;
  j->xdt = xdt;
  j->ws = ws;
  j->nmixed = nmixed; j->pmixed = pmixed; j->nfin = nfin; j->pfin = pfin; j->refine = refine;
  // status word and norms after the FP64 scratch
  const size_t w = tiny_ws_layout(N, dims, j->R).total;
  j->status = reinterpret_cast<int*>(ws + w);
  j->scal = ws + w + 2;
}

hipError_t launch_tiny_als(const TinyJob* d_jobs, int njobs, hipStream_t s) {
  if (njobs < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tiny_als_kernel, dim3((unsigned)njobs), dim3(TT), 0, s, d_jobs);
  return hipGetLastError();
}

size_t tiny_job_desc_bytes() { return sizeof(TinyJob); }
