// Per-block QR for blocks of width 8 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 8)
QRK_BQRN_INST(double, 8)
}  // namespace qrk
