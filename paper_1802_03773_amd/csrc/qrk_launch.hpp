// Host-side launchers of the qrkit kernels (internal to libqrkit.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrk_batch.hpp"

namespace qrk {

// Per-block Householder QR of [A_i; sqrt(lam_p) D_i] with Q_i^T applied to [B_i | b_i; 0 | 0]
// for the blocks blk_list[begin .. begin + count) (or begin .. begin + count when blk_list is
// null), all of class cls (the grouping of block_classes.hpp).  Writes R_i (Rblk, global
// block order), the coupling rows S_i | c_i (Sc, the problem's slice, row stride L_p) and the
// m_i reduced rows of every block into the problem's slice of Red (row stride ldr_p).
// pro: the clearing and lambda store of the factor call's first launch (an empty prologue for
// the others).  cam non-null: the coupled columns are cameras of ldb columns (nB = ncam *
// ldb), B holds each row's ldb values and cam[row] (indexed like the rows of A) its camera.
template <typename T>
hipError_t launch_blockqr(const int32_t* blk_list, int64_t begin, int64_t count, int cls, int n, int probs_count,
                          const ProbDesc* probs, const int32_t* blk_prob, const int64_t* row_off, const T* A,
                          const T* B, const int32_t* cam, const T* b, const double* d, const double* lam, T* Rblk,
                          T* Sc, T* Red, const BqrPrologue& pro, const QKeep& qk, hipStream_t st);

// Per-block QR with compile-time block width N, for blocks with m_i >= N (rows: 16, 32 or
// 64 register rows, m_i + N <= rows; slots: 1 or 2, nB + 1 <= 64 slots).
template <typename T, int N>
hipError_t launch_blockqr_n(const int32_t* blk_list, int64_t begin, int64_t count, int rows, int slots,
                            const ProbDesc* probs, const int32_t* blk_prob, const int64_t* row_off, const T* A,
                            const T* B, const int32_t* cam, const T* b, const double* d, const double* lam, T* Rblk,
                            T* Sc, T* Red, const BqrPrologue& pro, const QKeep& qk, hipStream_t st);

// One workgroup of the float64 tall-skinny QR: stream rows [r0, r1) of its input (row
// stride ldx, L columns) into an L x L upper-triangular R (Householder merges) written
// row-major at out_off.  Input buffer: in_buf 0 the reduced rows (x_off from Red), 1 or 2 a
// partial-triangle buffer; output: out_buf 0 the problem's R_B | c_B (in RB), 1 or 2 a
// partial buffer.  seed >= 0: the leaf starts from diag(sqrt(lam_q) d_B) of problem q = seed.
struct TsqrWg {
  int64_t x_off, r0, r1, out_off;
  int32_t ldx, L, seed;
  int8_t in_buf, out_buf;
};
// One launch per level (count workgroups from wg): the leaves of every problem, then the
// fanin-way merges of each problem's triangles, level by level; Lmax: the widest problem.
template <typename T>
hipError_t launch_tsqr_stream(const TsqrWg* wg, int count, int Lmax, const ProbDesc* probs, int n, const T* Red,
                              const double* d, const double* lam, T* part0, T* part1, T* RB, hipStream_t st);

// Float32 tall-skinny QR on the matrix cores for a batch: the global leaves
// [cls_begin[c], cls_begin[c] + cls_count[c]) are the leaves of the problems with c
// 16-column blocks (leaf_prob / leaf_idx: problem and index within it); one launch per c.
// Each problem's leaves merge pairwise in the same launch (its slots from slot0, counters
// from ctr0; nctr counters in all, cleared here) and its root goes to RB + rboff.
// bf16x3: the trailing updates' two large products are formed as three bf16 products each
// (hi hi' + hi lo' + lo hi', fp32 accumulation).
int tsqr_mfma_slot_floats(int L);
// p[0 .. n) = 0 (a kernel, so it may be captured into a graph).
hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t st);

// Pipelined merge tree of a single problem whose leaves stored their triangles (tree_sep):
// nnodes inner nodes in level order (node_l / node_r child references, r < 0 leaf -1 - r),
// flags[nnodes * ncb] cleared beforehand; ncb <= kTreeMaxNCB.  The root writes R_B | c_B.
constexpr int kTreeMaxNCB = 8;
hipError_t launch_tsqr_tree(int ncb, const ProbDesc* probs, const int32_t* node_l, const int32_t* node_r,
                            int nnodes, float* slots, int* flags, float* RB, int* status, const QStore& qs,
                            hipStream_t st);
// Leaves of classes 8 and 7 by their launches; the leaves from queue_begin on (classes
// kQueueNCB .. 1, listed widest first) by one persistent launch of at most `cus` workgroups
// that takes them from the device counter *qhead (cleared with the counters) when use_queue is
// set and more than one of those classes is present, else by a launch per class.
hipError_t launch_tsqr_mfma(bool bf16x3, const int* cls_begin, const int* cls_count, int queue_begin, bool use_queue,
                            int cus,
                            const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs, int n,
                            const float* Red, const double* d, const double* lam, float* slots, int* counters,
                            int64_t nctr, int* qhead, float* RB, const QStore& qs, hipStream_t st);

// R_B p_B = c_B for every problem (RB_p is L x L with c_B in column L-1, or c_B from cext,
// laid out like p, when that is given); writes p_B.
template <typename T>
hipError_t launch_backsub_dense(const BatchView& bv, const T* RB, double* p, int* status, hipStream_t st,
                                const double* cext = nullptr);

// p_i = R_i^{-1} (c_i - S_i p_B) for every block (c_i from S|c, or from cext laid out like p);
// p_B read from p.
template <typename T>
hipError_t launch_backsub_blocks(const BatchView& bv, const T* Rblk, const T* Sc, double* p, int* status,
                                 hipStream_t st, const double* cext = nullptr);

// Vertical concatenation (vcat.hip): the stage problem's rows [R1_i; R2_i], [S1_i; S2_i] (row
// stride L), [c1_i; c2_i] and the two dense triangles (at row red_row of Red, stride ldr).
template <typename T>
hipError_t launch_vcat_gather(int64_t K, int n, int L, const T* R1, const T* R2, const T* Sc1, const T* Sc2,
                              const T* RB1, const T* RB2, T* A, T* B, T* b, T* Red, int64_t red_row, int64_t ldr,
                              hipStream_t st);
// y += ypart; part0[j] += sum_w part[w][j] - lam_part d_B,part[j]^2 p_B[j] (j < nB).
hipError_t launch_vcat_merge(int64_t ny, double* y, const double* ypart, double* part0, const double* part, int nwg,
                             int nB, const double* lam_part, const double* dB_part, const double* pB,
                             hipStream_t st);

// Q^T b with the stored Q of a float32 block-angular factor (stored_q.hip): b [M] float, the
// first N entries (laid out like p) to c; xr [M], uslots and counters[0 .. nctr) are work
// space (the counters are cleared here).
hipError_t launch_apply_qt(const BatchView& bv, const int* cls_begin, const int* cls_count,
                           const int32_t* leaf_prob, const int32_t* leaf_idx, const float* b, const QKeep& qk,
                           const QStore& qs, float* xr, float* uslots, int* counters, int64_t nctr, double* c,
                           hipStream_t st);

// Refinement, pass 1: per pack of whole blocks (at most 64 rows): r = b - J p,
// g_i = A_i^T r - lam d_i^2 p_i, y_i = R_i^{-T} g_i, and per-workgroup partial sums of
// B^T r - S_i^T y_i (part[wg][kMaxDense]).  cam non-null: camera columns, as for
// launch_blockqr.
template <typename T>
hipError_t launch_refine_residual(const BatchView& bv, const T* A, const T* B, const int32_t* cam, const T* b,
                                  const double* d, const T* Rblk, const T* Sc, const double* p, double* y,
                                  double* part, hipStream_t st);

// Refinement, pass 2: g_B = sum(part) - lam d_B^2 p_B; y_B = R_B^{-T} g_B; dB = R_B^{-1} y_B;
// p_B += dB; dB stored to delta_B[p * kMaxDense ..].
template <typename T>
hipError_t launch_refine_dense(const BatchView& bv, const double* part, const T* RB, const double* dvec,
                               double* p, double* delta_B, hipStream_t st);

// Refinement, pass 3: delta_i = R_i^{-1}(y_i - S_i delta_B); p_i += delta_i.
template <typename T>
hipError_t launch_refine_blocks(const BatchView& bv, const T* Rblk, const T* Sc, const double* y,
                                const double* delta_B, double* p, hipStream_t st);

// Adjoint pieces (a single problem).  u = (R^T R)^{-1} g through the structured R:
//   launch_adjoint_fwd_blocks: y_i = R_i^{-T} g_i (-> y), per-workgroup partials of -S_i^T y_i
//                              (grid workgroups, row stride kMaxDense);
//   launch_adjoint_dense:      u_B = R_B^{-1} R_B^{-T} (g_B + sum of partials);
//   launch_adjoint_blocks:     u_i = R_i^{-1} (y_i - S_i u_B).
template <typename T>
hipError_t launch_adjoint_fwd_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* g,
                                     double* y, double* part, int grid, hipStream_t st);
template <typename T>
hipError_t launch_adjoint_dense(const BatchView& bv, const double* part, const T* RB, const double* g, double* u,
                                hipStream_t st);
template <typename T>
hipError_t launch_adjoint_blocks(const BatchView& bv, const T* Rblk, const T* Sc, const double* y, double* u,
                                 hipStream_t st);
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
