// Per-block QR for blocks of width 5 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 5)
QRK_BQRN_INST(double, 5)
}  // namespace qrk
