// Kernel instantiations: planned-batch (device table) fwd launches with bf16
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTableTable kFwdPlanBF16 = make_fwd_table_table<bf16_t>();
FwdHeadPlanTable kFwdHeadPlanBF16 = make_fwd_head_plan_table<bf16_t>();
}  // namespace dwt2
