// Per-block QR for blocks of width 3 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 3)
QRK_BQRN_INST(double, 3)
}  // namespace qrk
