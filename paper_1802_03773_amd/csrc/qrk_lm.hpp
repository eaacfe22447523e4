// Launchers of the Levenberg-Marquardt iteration kernels (lm.hip), internal to libqrkit.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrk_batch.hpp"

namespace qrk {

// Block-angular model evaluation and its per-problem reduction.  jac = true at x: J(x) into
// A and B (the handle's B layout), b = -f, d and J^T f (block and dense columns), F = |f|^2/2
// into Fout.  jac = false at x + p: F_new into Fout only.  part [nwg][2][kMaxDense] and
// fpart [nwg] are scratch.
template <typename T>
hipError_t launch_lmba_eval(const BatchView& bv, bool jac, const T* A0, const T* B0, const T* y, double c,
                            const double* x, const double* p, T* A, T* B, T* b, double* d, double* gJ,
                            double* part, double* fpart, double* Fout, hipStream_t st);

// Banded model evaluation for P problems of M rows / N unknowns / w values per row.  jac =
// true at x: J(x) into vals, b = -f, f (float64), d and J^T f, F into Fout; jac = false at
// x + p: F_new into Fout.  fpart holds P * ceil(M / 256) doubles.
template <typename T>
hipError_t launch_lmbd_eval(int P, int64_t M, int64_t N, int w, bool jac, const int32_t* row_start, const int32_t* fr,
                            const T* vals0, const T* y, double c, const double* x, const double* p, T* vals, T* b,
                            double* f, double* d, double* gJ, double* fpart, double* Fout, hipStream_t st);

// stage 0: pred = p^T (lam D^2 p - J^T f) / 2 per problem.  stage 1: gain ratio, damping
// update, accept flags, log row of this iteration, iteration counter, x += p where accepted.
// workgroups per problem of the predicted-decrease sum (its partials buffer holds P of them)
int lm_pred_blocks(int64_t maxN);
hipError_t launch_lm_control(int P, int64_t maxN, const int64_t* noff, const double* p, const double* d,
                             const double* gJ, double* lam, double* nu, const double* F, const double* Fnew,
                             double* pred, double* predpart, int* acc, int* iter, double* log, int max_log, double* x,
                             hipStream_t st, int stage);

// nu = 2 for every problem, iteration counter = 0.
hipError_t launch_lm_init(int P, double* nu, int* iter, hipStream_t st);

}  // namespace qrk
