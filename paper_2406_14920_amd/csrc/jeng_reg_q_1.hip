// jeng_reg_q_1.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_1.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_1(int lx, int ly, bool fp32)
{
    if (lx == 4 && ly == 4)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<4, 4, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<4, 4, double>, 64>;
    if (lx == 5 && ly == 2)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 2, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 2, double>, 64>;
    if (lx == 4 && ly == 2)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<4, 2, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<4, 2, double>, 64>;
    if (lx == 2 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<2, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<2, 6, double>, 64>;
    if (lx == 5 && ly == 5)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 5, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 5, double>, 64>;
    return nullptr;
}

}  // namespace md
