// Kernel instantiations for bf16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdBF16 = make_fwd_table<bf16_t>();
InvTable kInvBF16 = make_inv_table<bf16_t>();
}  // namespace dwt2
