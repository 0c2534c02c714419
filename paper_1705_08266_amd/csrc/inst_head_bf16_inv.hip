// Kernel instantiations: fused finest levels (head), inv, bf16 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvHeadTable kInvHeadBF16 = make_inv_head_table<bf16_t>();
InvHeadBatchTable kInvHeadBatchBF16 = make_inv_head_batch_table<bf16_t>();
}  // namespace dwt2
