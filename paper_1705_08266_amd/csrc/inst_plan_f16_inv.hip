// Kernel instantiations: planned-batch (device table) inv launches with f16
// storage of user-visible buffers.
#include "dwt2_table.hpp"

namespace dwt2 {
InvTableTable kInvPlanF16 = make_inv_table_table<__half>();
InvHeadPlanTable kInvHeadPlanF16 = make_inv_head_plan_table<__half>();
}  // namespace dwt2
