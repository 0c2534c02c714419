// Kernel instantiations: inv levels with bf16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTable kInvBF16 = make_inv_table<bf16_t>();
InvBatchTable kInvBatchBF16 = make_inv_batch_table<bf16_t>();
InvTailTable kInvTailBF16 = make_inv_tail_table<bf16_t>();
}  // namespace dwt2
