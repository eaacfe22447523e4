// Handle layout shared by the host-side translation units of libqrkit.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "qrk_batch.hpp"
#include "qrk_launch.hpp"
#include "qrkit.h"

namespace qrk {

enum HandleKind { KIND_BLOCKANGULAR = 0, KIND_BANDED = 1 };

hipError_t launch_fill_int(int* ptr, int value, hipStream_t st);
hipError_t launch_fill_double(double* p, int64_t n, double value, hipStream_t st);
// out[2q], out[2q+1] = sum over problem q's unknowns [noff[q], noff[q+1]) of (p - pold)^2 and p^2
hipError_t launch_rel_change(int P, const int64_t* noff, const double* p, const double* pold, double* out,
                             hipStream_t st);
template <typename T>
hipError_t launch_to_type(const double* src, T* dst, int64_t n, hipStream_t st);
// blocks of their own widths: A and d into the handle's n columns per block, p back out
template <typename T>
hipError_t launch_ragged_in(int64_t K, int n, int nB, const int64_t* row_off, const int32_t* ncol,
                            const int64_t* aoff, const int64_t* poff, const T* Au, const double* du, T* Ap,
                            double* dp, hipStream_t st);
hipError_t launch_ragged_out(int64_t K, int n, int nB, const int32_t* ncol, const int64_t* poff, const double* pp,
                             double* pu, hipStream_t st);
template <typename T>
hipError_t launch_colnorms(int64_t K, int n, int nB, int64_t M, const int64_t* row_off, const T* A,
                           const T* B, int64_t ldb, const int32_t* cam, double* d, double* part, int nparts,
                           hipStream_t st);

}  // namespace qrk

struct qrk_handle_s {
  qrk::HandleKind kind = qrk::KIND_BLOCKANGULAR;
  qrk_dtype dtype = QRK_F32;
  qrk_mode mode = QRK_PLAIN;

  // shape (block-angular: totals over the batch; nB, ldb and ldr are those of problem 0)
  int64_t K = 0;       // blocks
  int n = 0;           // columns per block
  int nB = 0;          // dense columns
  int64_t M = 0;       // rows of J
  int64_t N = 0;       // columns of J
  int64_t ldb = 0;
  int max_rows = 0;    // max_i m_i + n
  int w = 0;           // banded: values per row
  int band_method = 0; // banded: 0 Givens, 1 block-banded compact WY (fp32), 2 (BF16x3)
  int P = 1;           // problems stacked in the handle

  // block-angular batch layout (a single problem is the batch of one)
  std::vector<qrk::ProbDesc> probs_h;
  qrk::ProbDesc* probs_d = nullptr;
  int32_t* blk_prob = nullptr;   // [K]
  int32_t* blk_list = nullptr;   // [blk_list_n] blocks grouped by per-block QR class
  int64_t blk_list_n = 0;        // 0: one class, covering blocks 0 .. K-1 in order
  int64_t bq_begin[8] = {0};     // per-block QR class (block_classes.hpp): range in blk_list
  int64_t bq_count[8] = {0};
  int32_t* wg_prob = nullptr;    // [nwg]
  int32_t* leaf_prob = nullptr;  // [leaf_cap]
  int32_t* leaf_idx = nullptr;   // [leaf_cap]
  int64_t leaf_cap = 0;
  int64_t slot_cap = 0;          // floats
  int64_t ctr_cap = 0;           // ints
  int64_t nctr = 1;              // counters in use
  int32_t* node_l = nullptr;     // pipelined merge tree of a single problem (tree_sep):
  int32_t* node_r = nullptr;     //   child references of the inner nodes, level order
  int64_t node_cap = 0;
  int nnodes = 0;                //   0: the merges run inside the leaf launch
  int cls_begin[9] = {0};        // float32 leaves grouped by 16-column-block count, widest first
  int queue_begin = 0;           // first leaf of the persistent launch (classes 6 .. 1)
  int64_t qhead_off = 0;         // its queue head among the counters
  int cus = 256;                 // compute units of the device
  char arch[32] = {0};           // its architecture name (autotuner cache key)
  // autotuner knobs (tune_cache.hpp): leaf queue on or off, refinement workgroups scale; nwg_cap
  // is the refinement workgroup capacity reserved at create (the count at the largest scale)
  int leaf_queue = 1;
  double refine_scale = 1.0;
  int nwg_cap = 1;
  int widths = 1;                // float32 leaf classes of at most kQueueNCB column blocks present
  int cls_count[9] = {0};
  int nwg = 1;                   // refinement workgroups over the batch
  int max_L = 1;
  double leaf_scale = 1.0;       // multiplies the default rows per leaf (autotuner)
  double* lam_d = nullptr;       // owned damping of a single-problem factor call
  const double* lam_ptr = nullptr;  // damping the kernels read ([P], device)

  // launch shape; shape_gen counts the changes of the dense-part leaf layout (device tables and
  // workspace pointers), so that a graph captured before a change is re-captured
  uint64_t shape_gen = 0;
  int grid_blocks = 1;
  int refine_grid = 1;
  int leaves = 1;
  int fanin = 8;
  int64_t ldr = 0;

  // owned device workspace
  std::vector<void*> allocs;
  int64_t ws_bytes = 0;
  int64_t* row_off_d = nullptr;
  int64_t* pack_blk = nullptr;  // packs of whole blocks with at most 64 rows: [npacks+1]
  int64_t npacks = 0;
  void* Rblk = nullptr;   // [K][n][n]
  void* Sc = nullptr;     // [K][n][nB+1]
  void* Red = nullptr;    // [M][ldr]
  void* RB = nullptr;     // [nB+1][nB+1]
  void* part0 = nullptr;  // TSQR partial triangles (float64 path): even levels
  void* part1 = nullptr;  // odd levels
  int64_t part_cap0 = 0, part_cap1 = 0;  // elements
  // float64 dense part: every level's workgroups (all problems), level by level
  qrk::TsqrWg* tsqr_wg = nullptr;
  int64_t tsqr_wg_cap = 0;
  std::vector<int> tsqr_lvl_begin, tsqr_lvl_count;
  float* slots = nullptr; // TSQR tree slots (float32 matrix-core path)
  int* counters = nullptr;
  int max_leaves = 1;
  double* ybuf = nullptr;     // refinement: y_i per block
  double* refpart = nullptr;  // refinement: per-workgroup partial sums
  double* deltaB = nullptr;   // refinement: dense-part correction
  double* ubuf = nullptr;     // adjoint: u = (R^T R)^{-1} g
  double* Jubuf = nullptr;    // adjoint: J u
  int* status = nullptr;
  void* bandR = nullptr;      // banded: [P][N][w]
  void* bandc = nullptr;      // banded: [P][N]
  double* bandinv = nullptr;  // banded: reciprocal pivots 1 / R[j][j], [P][N]
  int32_t* bandfr = nullptr;  // banded: first row with start >= c, [P][N+1]
  void* bandR16 = nullptr;    // banded: sweep copy of the band, [P][N][16] (null if not kept)
  // two-stage damping (qrk_factor_lambda): the factor of J alone kept aside, c of that factor
  // as a contiguous vector, and the handle of the second-stage problem
  bool lam_base_saved = false;
  void* Rblk0 = nullptr;
  void* Sc0 = nullptr;
  void* RB0 = nullptr;
  void* c0 = nullptr;
  qrk_handle_s* lam_stage = nullptr;
  double* rbuf = nullptr;     // banded: residual / J u, [P][M] each
  double* jubuf = nullptr;
  double* gbuf = nullptr;     // banded: [P][N]
  double* vecpart = nullptr;  // adjoint vector-term partials
  int64_t* tol_noff = nullptr;   // qrk_solve_tol: unknown offsets [P+1] and norms [2P] (first call)
  double* tol_norms = nullptr;
  // stored Q (qrk_set_keep_q; float32 block-angular handles): the per-block reflectors (qk), the
  // compact-WY panels of the dense-part tiles and merge nodes (offsets in the ProbDescs), and
  // the application's work space: the reduced right-hand side [M] and the merge vectors
  bool keep_q = false;
  bool q_valid = false;          // the last factor call stored Q
  qrk::QKeep qk;
  std::vector<qrk::QOff> qoff_h;  // [P]
  qrk::QOff* qoff_d = nullptr;
  float* q_tiles = nullptr;
  float* q_nodes = nullptr;
  float* q_xr = nullptr;
  float* q_u = nullptr;
  int64_t q_tiles_cap = 0, q_nodes_cap = 0, q_u_cap = 0;  // floats
  int64_t q_tiles_n = 0, q_nodes_n = 0, q_u_n = 0;        // floats the current layout needs
  double* q_c = nullptr;         // Q^T b of qrk_solve_qt, laid out like p [N]
  // vertical concatenation (qrk_factor_vcat): the handles whose rows were added to this factor
  // (borrowed until the next factor call), the stage problem that merges two factors and its
  // inputs (the interleaved rows of R1, R2)
  // blocks of their own widths (qrk_create_blockangular_ncol): the handle runs them at n
  // columns; A, d and p of the caller's layout are moved in and out around factor and solve
  bool ragged = false;
  int64_t rg_N = 0;            // unknowns of the caller's layout: sum of ncol_i, plus nB
  int32_t* rg_ncol = nullptr;  // [K]
  int64_t* rg_aoff = nullptr;  // [K + 1] first value of block i in the caller's A
  int64_t* rg_poff = nullptr;  // [K + 1] first unknown of block i in the caller's d and p
  void* rg_A = nullptr;        // [M x n]
  double* rg_d = nullptr;      // [N]
  double* rg_p = nullptr;      // [N]
  // camera columns (qrk_create_blockangular_cam): nB = ncam * cw, B holds cw values per row
  // (row stride ldb = cw) and cam the camera of every row (the caller's device array)
  bool camb = false;
  int32_t ncam = 0, cw = 0;
  const int32_t* cam = nullptr;
  std::vector<qrk_handle_s*> vparts;
  qrk_handle_s* vcat_stage = nullptr;
  void* vA = nullptr;
  void* vB = nullptr;
  void* vb = nullptr;

  // phase timing: event pairs in a ring, summed on read
  struct ProfRec {
    int phase;
    hipEvent_t start, stop;
  };
  std::vector<ProfRec> prof_pool;  // created at enable time
  int prof_used = 0;
  bool prof_on = false;
  double prof_ms[QRK_NPHASES] = {0};
  int prof_cnt[QRK_NPHASES] = {0};

  // borrowed inputs of the last factor call
  const void* A = nullptr;
  const void* B = nullptr;
  const void* b = nullptr;
  const double* d = nullptr;
  const int32_t* row_start = nullptr;
  double lam = 0.0;
  bool factored = false;
};

qrk_status banded_adjoint(qrk_handle h, const double* p, const double* g, void* dvals, void* db,
                          double* dlam, double* dd, hipStream_t st);
qrk_status blockangular_adjoint(qrk_handle h, const double* p, const double* g, void* dA, void* dB,
                                void* db, double* dlam, double* dd, hipStream_t st);

// Block-angular factor / solve on the handle's current (borrowed) inputs and damping, and
// the batch view the kernels take; shared with the LM driver.
qrk_status blockangular_factor(qrk_handle h, hipStream_t st);
qrk_status blockangular_solve(qrk_handle h, double* p, int sweeps, hipStream_t st);
qrk::BatchView blockangular_view(qrk_handle h);
// Banded factor / solve on the handle's current inputs and damping ([P] at h->lam_ptr).
qrk_status banded_factor(qrk_handle h, hipStream_t st);
qrk_status banded_solve(qrk_handle h, double* p, int sweeps, hipStream_t st);
qrk_status banded_refine(qrk_handle h, double* p, int sweeps, const void* b, hipStream_t st);
// `sweeps` refinement sweeps of a block-angular handle for the right-hand side b (the handle's type)
qrk_status blockangular_refine(qrk_handle h, double* p, int sweeps, const void* b, hipStream_t st);

// Stored Q: allocate the storage the current leaf layout needs (set_keep_q and every layout
// change while it is on).
qrk_status ensure_q_storage(qrk_handle h);

// Workspace allocation shared by the create functions (records the allocation in h).
qrk_status handle_alloc(qrk_handle h, void** out, size_t bytes);
void handle_free(qrk_handle h);

// Phase timing helpers: prof_begin returns the record index (or -1 when off or full).
int prof_begin(qrk_handle h, int phase, hipStream_t st);
void prof_end(qrk_handle h, int rec, hipStream_t st);
