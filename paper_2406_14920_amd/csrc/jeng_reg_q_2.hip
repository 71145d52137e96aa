// jeng_reg_q_2.hip -- queue forms (batch launches) of the register J-engine
// classes of jeng_reg_2.hip.
#include "jeng_reg.hpp"

namespace md {

QueueLaunchFn jeng_reg_queue_fn_2(int lx, int ly, bool fp32)
{
    if (lx == 5 && ly == 3)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 3, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 3, double>, 64>;
    if (lx == 0 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<0, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<0, 6, double>, 64>;
    if (lx == 2 && ly == 4)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<2, 4, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<2, 4, double>, 64>;
    if (lx == 6 && ly == 0)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<6, 0, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<6, 0, double>, 64>;
    if (lx == 3 && ly == 6)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<3, 6, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<3, 6, double>, 64>;
    if (lx == 5 && ly == 4)
        return fp32 ? &queue_launch<JArgs, jeng_reg_q<5, 4, float>, 64>
                    : &queue_launch<JArgs, jeng_reg_q<5, 4, double>, 64>;
    return nullptr;
}

}  // namespace md
