// Kernel instantiations for f32 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdF32 = make_fwd_table<float>();
InvTable kInvF32 = make_inv_table<float>();
}  // namespace dwt2
