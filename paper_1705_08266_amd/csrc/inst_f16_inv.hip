// Kernel instantiations: inv levels with f16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTable kInvF16 = make_inv_table<__half>();
InvBatchTable kInvBatchF16 = make_inv_batch_table<__half>();
InvTailTable kInvTailF16 = make_inv_tail_table<__half>();
}  // namespace dwt2
