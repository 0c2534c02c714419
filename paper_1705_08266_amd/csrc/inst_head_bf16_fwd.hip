// Kernel instantiations: fused finest levels (head), fwd, bf16 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdHeadTable kFwdHeadBF16 = make_fwd_head_table<bf16_t>();
FwdHeadBatchTable kFwdHeadBatchBF16 = make_fwd_head_batch_table<bf16_t>();
}  // namespace dwt2
