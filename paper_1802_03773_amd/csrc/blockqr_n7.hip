// Per-block QR for blocks of width 7 (float and double).
#include "blockqr_n_kernel.hpp"

namespace qrk {
QRK_BQRN_INST(float, 7)
QRK_BQRN_INST(double, 7)
}  // namespace qrk
