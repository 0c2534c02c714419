// Kernel instantiations: fwd levels with bf16 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdBF16 = make_fwd_table<bf16_t>();
FwdBatchTable kFwdBatchBF16 = make_fwd_batch_table<bf16_t>();
FwdTailTable kFwdTailBF16 = make_fwd_tail_table<bf16_t>();
}  // namespace dwt2
