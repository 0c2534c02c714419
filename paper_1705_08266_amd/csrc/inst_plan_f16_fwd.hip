// Kernel instantiations: planned-batch (device table) fwd launches with f16
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
FwdTableTable kFwdPlanF16 = make_fwd_table_table<__half>();
FwdHeadPlanTable kFwdHeadPlanF16 = make_fwd_head_plan_table<__half>();
}  // namespace dwt2
