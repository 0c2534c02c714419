// Kernel instantiations: planned-batch (device table) inv launches with bf16
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTableTable kInvPlanBF16 = make_inv_table_table<bf16_t>();
InvHeadPlanTable kInvHeadPlanBF16 = make_inv_head_plan_table<bf16_t>();
}  // namespace dwt2
