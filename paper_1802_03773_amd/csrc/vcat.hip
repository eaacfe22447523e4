// Vertical concatenation of two factored block-angular problems over the same columns (QRkit
// Section 4.5, Eq. vcatDecomp): [A1; A2] = blkdiag(Q1, Q2) [R1; R2], and the row permutation that
// interleaves R1 and R2 block by block makes P [R1; R2] block-angular again.  These kernels build
// that permuted matrix as the input of one more structured QR (the factor call's own kernels), and
// merge the second part's terms into a refinement sweep of the stacked problem.
#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_launch.hpp"

namespace qrk {

// Block i of the stage problem: rows [R1_i; R2_i] (A, 2n x n), [S1_i; S2_i] (B, 2n x L with row
// stride L, of which the first nB columns are read) and [c1_i; c2_i] (b, 2n).  The dense part's
// extra rows: R1_B | c1_B then R2_B | c2_B (each L x L, row-major, the residual entry included),
// written at row `red_row` of the stage's reduced rows (stride ldr).  One thread per element.
template <typename T>
__global__ void __launch_bounds__(256)
k_vcat_gather(int64_t K, int n, int L, const T* __restrict__ R1, const T* __restrict__ R2, const T* __restrict__ Sc1,
              const T* __restrict__ Sc2, const T* __restrict__ RB1, const T* __restrict__ RB2, T* __restrict__ A,
              T* __restrict__ B, T* __restrict__ b, T* __restrict__ Red, int64_t red_row, int64_t ldr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nA = K * 2 * n * n, nS = K * 2 * n * L, nR = 2 * (int64_t)L * L;
  if (t < nA) {
    const int64_t i = t / (2 * n * n), e = t % (2 * n * n);  // block, element of [R1_i; R2_i]
    const int64_t part = e / (n * n), f = e % (n * n);
    A[t] = (part == 0 ? R1 : R2)[i * n * n + f];
  } else if (t < nA + nS) {
    const int64_t u = t - nA;
    const int64_t i = u / (2 * n * L), e = u % (2 * n * L);
    const int64_t part = e / (n * L), f = e % (n * L);  // row f / L of S_part_i | c_part_i
    const T v = (part == 0 ? Sc1 : Sc2)[i * n * L + f];
    B[u] = v;
    if (f % L == L - 1) b[i * 2 * n + part * n + f / L] = v;  // the c column
  } else if (t < nA + nS + nR) {
    const int64_t u = t - nA - nS;
    const int64_t part = u / ((int64_t)L * L), f = u % ((int64_t)L * L);
    Red[(red_row + part * L + f / L) * ldr + f % L] = (part == 0 ? RB1 : RB2)[f];
  }
}

template <typename T>
hipError_t launch_vcat_gather(int64_t K, int n, int L, const T* R1, const T* R2, const T* Sc1, const T* Sc2,
                              const T* RB1, const T* RB2, T* A, T* B, T* b, T* Red, int64_t red_row, int64_t ldr,
                              hipStream_t st) {
  const int64_t total = K * 2 * n * n + K * 2 * n * L + 2 * (int64_t)L * L;
  if (total < 1) return hipSuccess;
  hipLaunchKernelGGL((k_vcat_gather<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, K, n, L, R1, R2,
                     Sc1, Sc2, RB1, RB2, A, B, b, Red, red_row, ldr);
  return hipGetLastError();
}

// A refinement sweep of the stacked problem from its parts' pass 1 (each part's J and b with the
// stacked factor's R): y += y_part (the blocks' R_i^{-T} g_i is linear in g_i), and the part's
// workgroup partials of the dense part's right-hand side, summed in workgroup order, minus its
// own dense damping term lam_part d_part,B^2 p_B, added to the first partial row of the stacked
// problem (single problems: partial rows of kMaxDense doubles).
__global__ void __launch_bounds__(256)
k_vcat_merge(int64_t ny, double* __restrict__ y, const double* __restrict__ ypart, double* __restrict__ part0,
             const double* __restrict__ part, int nwg, int nB, const double* __restrict__ lam_part,
             const double* __restrict__ dB_part, const double* __restrict__ pB) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ny) y[t] += ypart[t];
  if (blockIdx.x == 0 && (int)threadIdx.x < nB) {
    const int j = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += part[(int64_t)w * kMaxDense + j];
    const double lam = *lam_part;
    part0[j] += s - lam * dB_part[j] * dB_part[j] * pB[j];
  }
}

hipError_t launch_vcat_merge(int64_t ny, double* y, const double* ypart, double* part0, const double* part, int nwg,
                             int nB, const double* lam_part, const double* dB_part, const double* pB,
                             hipStream_t st) {
  if (nB > kMaxDense - 1) return hipErrorInvalidValue;
  const int64_t grid = std::max<int64_t>(1, (ny + 255) / 256);
  hipLaunchKernelGGL(k_vcat_merge, dim3((unsigned)grid), dim3(256), 0, st, ny, y, ypart, part0, part, nwg, nB,
                     lam_part, dB_part, pB);
  return hipGetLastError();
}

#define QRK_INST(T)                                                                                        \
  template hipError_t launch_vcat_gather<T>(int64_t, int, int, const T*, const T*, const T*, const T*,      \
                                            const T*, const T*, T*, T*, T*, T*, int64_t, int64_t, hipStream_t);
QRK_INST(float)
QRK_INST(double)
#undef QRK_INST

}  // namespace qrk
