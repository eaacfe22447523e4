// Per-block QR for blocks of width 2 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 2)
QRK_BQRN_INST(double, 2)
}  // namespace qrk
