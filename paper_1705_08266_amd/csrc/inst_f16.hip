// Kernel instantiations for f16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdF16 = make_fwd_table<__half>();
InvTable kInvF16 = make_inv_table<__half>();
}  // namespace dwt2
