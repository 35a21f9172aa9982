// Internal interfaces between the TR-ALS context (tr_als.hip), the planted-
// tensor generator and the serving runtime (tr_srv.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/tr_als.h"

// Byte alignment of every buffer carved from a caller-supplied region.
constexpr size_t TRX_ALIGN = 256;
inline size_t trx_round(size_t b) { return (b + TRX_ALIGN - 1) / TRX_ALIGN * TRX_ALIGN; }

// How a context gets its device memory and streams.
struct TrxOpts {
  char* region = nullptr;        // carve all workspace from here (no hipMalloc / hipFree)
  size_t region_bytes = 0;
  bool measure = false;          // only size the workspace: *measured = bytes, no device work
  size_t* measured = nullptr;
  hipStream_t stream2 = nullptr; // borrowed stream for the coefficient branch (else one is created)
  unsigned shadow_mask = 0;      // bit p set: the X shadow of precision p is reserved at init
  int graphs = -1;               // -1: environment default, 0: never capture sweeps, 1: capture
  bool no_sync = false;          // leave ||X||^2 on the device; creation never waits on the stream
};

int trx_init(tr_als_ctx** out, int N, const int64_t* dims, const int64_t* ranks, const void* X, int x_dtype,
             double* const* cores, int variant, hipStream_t stream, const TrxOpts& o);

// Workspace bytes of a context (all buffers, shadows of the precisions in
// shadow_mask), or 0 when the arguments are invalid.
size_t trx_footprint(int N, const int64_t* dims, const int64_t* ranks, int x_dtype, int variant,
                     unsigned shadow_mask);

// Planted-tensor generator (TR of N(0,1) cores plus relative Gaussian noise,
// all normals from Philox4x32-10): workspace bytes and the generator itself.
size_t trx_gen_workspace(int N, const int64_t* dims, const int64_t* ranks, bool need_true_cores);
int trx_gen(int N, const int64_t* dims, const int64_t* ranks, uint64_t seed, double eta, void* X, int x_dtype,
            double* const* true_cores, double* const* init_cores, char* ws, size_t ws_bytes, hipStream_t s,
            std::string* err);

// Asynchronous job body for the serving executor: nmixed sweeps in prec_mixed,
// nfin in prec_fin, cores written back, fit, then the latched status word and
// (||X||^2, fit residual^2) copied to the given pinned host memory, all
// enqueued on the context's stream without waiting (FP8 still reads its scale
// back).  A solve failure latches the status word; later updates then leave
// the cores unchanged.
int trx_run_async(tr_als_ctx* c, int nmixed, int prec_mixed, int nfin, int prec_fin, int refine, int* status_host,
                  double* scal_host);
const char* trx_status_text(int status_word);
