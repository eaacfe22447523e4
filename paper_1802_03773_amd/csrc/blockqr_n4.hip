// Per-block QR for blocks of width 4 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 4)
QRK_BQRN_INST(double, 4)
}  // namespace qrk
