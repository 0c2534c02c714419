// Kernel instantiations: fwd levels with f16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdF16 = make_fwd_table<__half>();
FwdBatchTable kFwdBatchF16 = make_fwd_batch_table<__half>();
FwdTailTable kFwdTailF16 = make_fwd_tail_table<__half>();
}  // namespace dwt2
