// jeng_reg_q_0.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_0.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_0(int lx, int ly)
{
    if (lx == 3 && ly == 5) return &queue_launch<JArgs, jeng_reg_q<3, 5>, 64>;
    if (lx == 4 && ly == 3) return &queue_launch<JArgs, jeng_reg_q<4, 3>, 64>;
    if (lx == 3 && ly == 3) return &queue_launch<JArgs, jeng_reg_q<3, 3>, 64>;
    if (lx == 1 && ly == 6) return &queue_launch<JArgs, jeng_reg_q<1, 6>, 64>;
    if (lx == 5 && ly == 6) return &queue_launch<JArgs, jeng_reg_q<5, 6>, 64>;
    return nullptr;
}

}  // namespace md
