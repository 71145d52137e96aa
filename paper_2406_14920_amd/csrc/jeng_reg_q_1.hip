// jeng_reg_q_1.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_1.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_1(int lx, int ly)
{
    if (lx == 4 && ly == 4) return &queue_launch<JArgs, jeng_reg_q<4, 4>, 64>;
    if (lx == 5 && ly == 2) return &queue_launch<JArgs, jeng_reg_q<5, 2>, 64>;
    if (lx == 4 && ly == 2) return &queue_launch<JArgs, jeng_reg_q<4, 2>, 64>;
    if (lx == 2 && ly == 6) return &queue_launch<JArgs, jeng_reg_q<2, 6>, 64>;
    if (lx == 5 && ly == 5) return &queue_launch<JArgs, jeng_reg_q<5, 5>, 64>;
    return nullptr;
}

}  // namespace md
