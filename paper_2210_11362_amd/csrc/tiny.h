// Batched lane of the serving loop: descriptor of one small job run entirely
// by one workgroup of a batch launch, and its host helpers (k_tiny.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct TinyJob {
  int N;
  int64_t dims[4];
  int R[5];
  const void* X;
  int xdt;
  double* cores[4];      // initial cores in, final cores out (device)
  double* ws;            // FP64 scratch of tiny_ws_bytes bytes
  int nmixed, pmixed, nfin, pfin, refine;
  int* status;           // inside ws: latched status word
  double* scal;          // inside ws: ||X||^2, residual^2
};

// Whether a job fits the batched lane (order 2..4, R_k <= 8, I_k <= 128,
// prod(I_k) <= 2^18); contraction type and variant are checked by the caller.
bool tiny_eligible(int N, const int64_t* dims, const int64_t* ranks);
size_t tiny_ws_bytes(int N, const int64_t* dims, const int64_t* ranks);
void tiny_fill(TinyJob* j, int N, const int64_t* dims, const int64_t* ranks, const void* X, int xdt,
               double* const* cores, double* ws, int nmixed, int pmixed, int nfin, int pfin, int refine);
hipError_t launch_tiny_als(const TinyJob* d_jobs, int njobs, hipStream_t s);
