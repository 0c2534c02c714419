// Kernel instantiations: the exchange ablation (every neighbour exchange
// through LDS), FP32 level kernels.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdLdsTable kFwdLds = make_fwd_lds_table();
InvLdsTable kInvLds = make_inv_lds_table();
}  // namespace dwt2
