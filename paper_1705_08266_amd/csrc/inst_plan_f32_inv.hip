// Kernel instantiations: planned-batch (device table) inv launches with f32
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTableTable kInvPlanF32 = make_inv_table_table<float>();
InvHeadPlanTable kInvHeadPlanF32 = make_inv_head_plan_table<float>();
}  // namespace dwt2
