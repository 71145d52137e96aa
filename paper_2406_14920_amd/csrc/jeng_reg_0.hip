// jeng_reg_0.hip -- one share of the register J-engine instantiations.
#include "jeng_reg.hpp"

namespace md {

bool launch_jeng_reg_0(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st)
{
    if (lx == 3 && ly == 5) { jeng_reg_launch_t<3, 5>(a, fp32, st); return true; }
    if (lx == 4 && ly == 3) { jeng_reg_launch_t<4, 3>(a, fp32, st); return true; }
    if (lx == 3 && ly == 3) { jeng_reg_launch_t<3, 3>(a, fp32, st); return true; }
    if (lx == 1 && ly == 6) { jeng_reg_launch_t<1, 6>(a, fp32, st); return true; }
    if (lx == 5 && ly == 6) { jeng_reg_launch_t<5, 6>(a, fp32, st); return true; }
    return false;
}

}  // namespace md
