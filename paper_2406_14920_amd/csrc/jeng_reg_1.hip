// jeng_reg_1.hip -- one share of the register J-engine instantiations.
#include "jeng_reg.hpp"

namespace md {

bool launch_jeng_reg_1(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st)
{
    if (lx == 4 && ly == 4) { jeng_reg_launch_t<4, 4>(a, fp32, st); return true; }
    if (lx == 5 && ly == 2) { jeng_reg_launch_t<5, 2>(a, fp32, st); return true; }
    if (lx == 4 && ly == 2) { jeng_reg_launch_t<4, 2>(a, fp32, st); return true; }
    if (lx == 2 && ly == 6) { jeng_reg_launch_t<2, 6>(a, fp32, st); return true; }
    if (lx == 5 && ly == 5) { jeng_reg_launch_t<5, 5>(a, fp32, st); return true; }
    return false;
}

}  // namespace md
