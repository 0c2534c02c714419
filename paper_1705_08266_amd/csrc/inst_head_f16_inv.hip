// Kernel instantiations: fused finest levels (head), inv, f16 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvHeadTable kInvHeadF16 = make_inv_head_table<__half>();
InvHeadBatchTable kInvHeadBatchF16 = make_inv_head_batch_table<__half>();
}  // namespace dwt2
