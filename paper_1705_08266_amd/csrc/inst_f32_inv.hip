// Kernel instantiations: inv levels with f32 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTable kInvF32 = make_inv_table<float>();
InvBatchTable kInvBatchF32 = make_inv_batch_table<float>();
InvTailTable kInvTailF32 = make_inv_tail_table<float>();
}  // namespace dwt2
