// Per-block QR for blocks of width 1 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 1)
QRK_BQRN_INST(double, 1)
}  // namespace qrk
