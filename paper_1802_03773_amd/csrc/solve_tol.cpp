// qrk_solve_tol: the back-substitution through the stored R, then float64-residual refinement
// sweeps until the correction of every problem is small relative to its solution, or a sweep
// limit is reached (the early stop of the LM step solve's boundary).  The change norms are
// summed on the device; the host reads them after each sweep to decide whether to go on.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "qrk_device.hpp"
#include "qrk_host.hpp"
#include "qrkit.h"

using namespace qrk;

namespace {

// Offsets of every problem's unknowns in p, and room for the norms (the first call only).
qrk_status tol_buffers(qrk_handle h) {
  if (h->tol_noff) return QRK_OK;
  const int P = h->P;
  std::vector<int64_t> off((size_t)P + 1, 0);
  for (int q = 0; q < P; ++q)
    off[(size_t)q + 1] = off[(size_t)q] + (h->kind == KIND_BLOCKANGULAR
                                               ? h->probs_h[(size_t)q].K * h->n + h->probs_h[(size_t)q].nB
                                               : h->N);
  qrk_status s;
  void* a = nullptr;
  void* b = nullptr;
  if ((s = handle_alloc(h, &a, sizeof(int64_t) * off.size())) != QRK_OK ||
      (s = handle_alloc(h, &b, sizeof(double) * 2 * (size_t)P)) != QRK_OK)
    return s;
  if (hipMemcpy(a, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice) != hipSuccess) return QRK_EHIP;
  h->tol_noff = static_cast<int64_t*>(a);
  h->tol_norms = static_cast<double*>(b);
  return QRK_OK;
}

qrk_status solve_tol(qrk_handle h, double* p, int32_t max_sweeps, double rel_tol, int32_t* sweeps_host,
                     hipStream_t st) {
  qrk_status s = tol_buffers(h);
  if (s != QRK_OK) return s;
  if ((s = h->kind == KIND_BLOCKANGULAR ? blockangular_solve(h, p, 0, st) : banded_solve(h, p, 0, st)) != QRK_OK)
    return s;
  const int P = h->P;
  const int64_t np = h->kind == KIND_BLOCKANGULAR ? h->N : (int64_t)P * h->N;
  std::vector<double> norms(2 * (size_t)P);
  std::vector<int> open((size_t)P, 1);  // problems still above the tolerance
  bool converged = max_sweeps == 0;
  int done = 0;
  while (done < max_sweeps) {
    // pold in the adjoint's scratch vector, one sweep, then the change norms
    if (hipMemcpyAsync(h->ubuf, p, sizeof(double) * (size_t)np, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return QRK_EHIP;
    s = h->kind == KIND_BLOCKANGULAR ? blockangular_refine(h, p, 1, h->b, st) : banded_refine(h, p, 1, h->b, st);
    if (s != QRK_OK) return s;
    if (launch_rel_change(P, h->tol_noff, p, h->ubuf, h->tol_norms, st) != hipSuccess ||
        hipMemcpyAsync(norms.data(), h->tol_norms, sizeof(double) * norms.size(), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QRK_EHIP;
    ++done;
    converged = true;
    for (int q = 0; q < P; ++q) {
      open[(size_t)q] = !(std::sqrt(norms[2 * (size_t)q]) <= rel_tol * std::sqrt(norms[2 * (size_t)q + 1]));
      if (open[(size_t)q]) converged = false;
    }
    if (converged) break;
  }
  if (sweeps_host) *sweeps_host = done;
  if (converged) return QRK_OK;
  // mark the problems that used every sweep above the tolerance (read by qrk_status_get)
  const int nw = h->kind == KIND_BLOCKANGULAR ? P : 1;
  std::vector<int> words((size_t)nw, 0);
  if (hipMemcpyAsync(words.data(), h->status, sizeof(int) * (size_t)nw, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QRK_EHIP;
  for (int q = 0; q < P; ++q)
    if (open[(size_t)q]) words[(size_t)(nw == 1 ? 0 : q)] |= ST_NOTCONVERGED;
  if (hipMemcpyAsync(h->status, words.data(), sizeof(int) * (size_t)nw, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QRK_EHIP;
  return QRK_ENOTCONVERGED;
}

}  // namespace

extern "C" {

qrk_status qrk_solve_tol(qrk_handle h, double* p, int32_t max_sweeps, double rel_tol, int32_t* sweeps_host,
                         void* stream) {
  if (!h || !p || !h->factored || max_sweeps < 0 || max_sweeps > 8 || !(rel_tol >= 0.0) || !std::isfinite(rel_tol))
    return QRK_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!h->ragged) return solve_tol(h, p, max_sweeps, rel_tol, sweeps_host, st);
  // blocks of their own widths: the sweeps run on the handle's layout, p is written back after
  const qrk_status s = solve_tol(h, h->rg_p, max_sweeps, rel_tol, sweeps_host, st);
  if (s != QRK_OK && s != QRK_ENOTCONVERGED) return s;
  return launch_ragged_out(h->K, h->n, h->nB, h->rg_ncol, h->rg_poff, h->rg_p, p, st) == hipSuccess ? s : QRK_EHIP;
}

}  // extern "C"
