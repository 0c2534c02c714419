// Kernel instantiations: fused finest levels (head), fwd, f32 storage of
// user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdHeadTable kFwdHeadF32 = make_fwd_head_table<float>();
FwdHeadBatchTable kFwdHeadBatchF32 = make_fwd_head_batch_table<float>();
}  // namespace dwt2
