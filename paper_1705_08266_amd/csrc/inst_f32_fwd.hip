// Kernel instantiations: fwd levels with f32 storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTable kFwdF32 = make_fwd_table<float>();
FwdBatchTable kFwdBatchF32 = make_fwd_batch_table<float>();
FwdTailTable kFwdTailF32 = make_fwd_tail_table<float>();
}  // namespace dwt2
