// Kernel instantiations: fused finest levels (head), fwd, f16 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdHeadTable kFwdHeadF16 = make_fwd_head_table<__half>();
FwdHeadBatchTable kFwdHeadBatchF16 = make_fwd_head_batch_table<__half>();
}  // namespace dwt2
