// Kernel instantiations: fused finest levels (head), inv, f32 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvHeadTable kInvHeadF32 = make_inv_head_table<float>();
InvHeadBatchTable kInvHeadBatchF32 = make_inv_head_batch_table<float>();
}  // namespace dwt2
