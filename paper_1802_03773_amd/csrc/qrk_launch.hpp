// Host-side launchers of the qrkit kernels (internal to libqrkit.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrk {

// Per-block Householder QR of [A_i; sqrt(lam) D_i] with Q_i^T applied to [B_i | b_i; 0 | 0].
// Writes R_i (Rblk), coupling rows S_i | c_i (Sc, ld nB+1) and the m_i reduced rows of
// every block to Red (row r0+k of Red is reduced row k of the block starting at r0).
// max_rows = max_i m_i + n must be <= 64.
template <typename T>
hipError_t launch_blockqr(int64_t K, int n, int nB, int max_rows, const int64_t* row_off,
                          const T* A, const T* B, int64_t ldb, const T* b, const double* d,
                          double sqrt_lam, T* Rblk, T* Sc, T* Red, int64_t ldr, int grid,
                          hipStream_t st);

// Stream rows [g*rows_per_wg, (g+1)*rows_per_wg) of X (nrows x L, row stride ldx) into
// an L x L upper-triangular R per workgroup g (Householder merges); workgroup 0 starts
// from diag(sqrt_lam * dB) (dB may be null).  Rout is [grid][L][L].
template <typename T>
hipError_t launch_tsqr_stream(const T* X, int64_t ldx, int64_t nrows, int L, int64_t rows_per_wg,
                              int grid, const double* dB, double sqrt_lam, T* Rout, hipStream_t st);

// Float32 tall-skinny QR on the matrix cores: nleaves waves each stream a contiguous
// share of the nrows x L rows of X (row stride ldx) into a triangle, then merge pairwise in
// the same launch; the root goes to Rout (L x L row-major).  Leaf 0 starts from
// diag(sqrt_lam * dB) when dB is not null.  slots holds 2*nleaves triangles of
// tsqr_mfma_slot_floats(L) floats; counters holds 2*nleaves+2 ints (cleared here).
int tsqr_mfma_slot_floats(int L);
hipError_t launch_tsqr_mfma(const float* X, int64_t ldx, int64_t nrows, int L, int nleaves,
                            const double* dB, double sqrt_lam, float* slots, int* counters,
                            float* Rout, hipStream_t st);

// R_B p_B = c_B (RB is L x L with c_B in column L-1); writes p[off .. off+nB) as double.
template <typename T>
hipError_t launch_backsub_dense(const T* RB, int L, double* p, int64_t off, int* status,
                                hipStream_t st);

// p_i = R_i^{-1} (c_i - S_i p_B) for every block; p_B read from p[K*n ..].
template <typename T>
hipError_t launch_backsub_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, double* p,
                                 int* status, int grid, hipStream_t st);

// Refinement, pass 1: per pack of whole blocks (pack_blk[k] .. pack_blk[k+1], at most 64
// rows): r = b - J p, g_i = A_i^T r - lam d_i^2 p_i, y_i = R_i^{-T} g_i, and per-workgroup
// partial sums of B^T r - S_i^T y_i (part[wg][nB]).
template <typename T>
hipError_t launch_refine_residual(int64_t npacks, const int64_t* pack_blk, int64_t K, int n, int nB,
                                  const int64_t* row_off, const T* A, const T* B, int64_t ldb, const T* b,
                                  const double* d, double lam, const T* Rblk, const T* Sc,
                                  const double* p, double* y, double* part, int grid, hipStream_t st);

// Refinement, pass 2: g_B = sum(part) - lam d_B^2 p_B; y_B = R_B^{-T} g_B; dB = R_B^{-1} y_B;
// p_B += dB; dB stored to delta_B.
template <typename T>
hipError_t launch_refine_dense(int nparts, int nB, const double* part, const T* RB, const double* dvec,
                               double lam, double* p, int64_t off, double* delta_B, hipStream_t st);

// Refinement, pass 3: delta_i = R_i^{-1}(y_i - S_i delta_B); p_i += delta_i.
template <typename T>
hipError_t launch_refine_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* y,
                                const double* delta_B, double* p, int grid, hipStream_t st);

// Adjoint pieces.  u = (R^T R)^{-1} g through the structured R:
//   launch_adjoint_fwd_blocks: y_i = R_i^{-T} g_i (-> y), per-workgroup partials of -S_i^T y_i;
//   launch_adjoint_dense:      u_B = R_B^{-1} R_B^{-T} (g_B + sum of partials);
//   launch_adjoint_blocks:     u_i = R_i^{-1} (y_i - S_i u_B).
template <typename T>
hipError_t launch_adjoint_fwd_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* g,
                                     double* y, double* part, int grid, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_dense(int nparts, int nB, const double* part, const T* RB, const double* gB,
                                double* uB, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* y,
                                 const double* uB, double* u, int grid, hipStream_t st);
// Gradients on the structural nonzeros, per pack of whole blocks (one row per lane):
//   r = b - J p, Ju = J u;  dA = r u_i^T - Ju p_i^T;  dB = r u_B^T - Ju p_B^T;  db = Ju.
template <typename T>
hipError_t launch_adjoint_rows(int64_t npacks, const int64_t* pack_blk, int64_t K, int n, int nB,
                               const int64_t* row_off, const T* A, const T* B, int64_t ldb, const T* b,
                               const double* p, const double* u, T* dA, T* dB, T* db, int grid,
                               hipStream_t st);
// dd_j = -2 lam u_j d_j p_j and dlam = -sum_j u_j d_j^2 p_j over P problems of N unknowns
// (deterministic two-level sum; part holds at least 1024 doubles).
hipError_t launch_adjoint_vec(int P, int64_t N, const double* u, const double* d, const double* p,
                              double lam, double* dd, double* dlam, double* part, hipStream_t st);

}  // namespace qrk
