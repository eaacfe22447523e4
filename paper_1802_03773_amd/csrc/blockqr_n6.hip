// Per-block QR for blocks of width 6 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 6)
QRK_BQRN_INST(double, 6)
}  // namespace qrk
