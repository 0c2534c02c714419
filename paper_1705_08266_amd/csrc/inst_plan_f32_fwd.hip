// Kernel instantiations: planned-batch (device table) fwd launches with f32
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTableTable kFwdPlanF32 = make_fwd_table_table<float>();
FwdHeadPlanTable kFwdHeadPlanF32 = make_fwd_head_plan_table<float>();
}  // namespace dwt2
