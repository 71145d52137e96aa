// jeng_reg_q_0.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_0.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_0(int lx, int ly, bool fp32)
{
    if (lx == 3 && ly == 5)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<3, 5, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<3, 5, double>, 64>;
    if (lx == 4 && ly == 3)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<4, 3, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<4, 3, double>, 64>;
    if (lx == 3 && ly == 3)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<3, 3, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<3, 3, double>, 64>;
    if (lx == 1 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<1, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<1, 6, double>, 64>;
    if (lx == 5 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 6, double>, 64>;
    return nullptr;
}

}  // namespace md
