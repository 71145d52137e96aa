// jeng_reg_q_3.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_3.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_3(int lx, int ly, bool fp32)
{
    if (lx == 2 && ly == 5)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<2, 5, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<2, 5, double>, 64>;
    if (lx == 3 && ly == 4)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<3, 4, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<3, 4, double>, 64>;
    if (lx == 1 && ly == 5)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<1, 5, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<1, 5, double>, 64>;
    if (lx == 5 && ly == 1)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 1, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 1, double>, 64>;
    if (lx == 4 && ly == 5)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<4, 5, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<4, 5, double>, 64>;
    if (lx == 4 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<4, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<4, 6, double>, 64>;
    return nullptr;
}

}  // namespace md
