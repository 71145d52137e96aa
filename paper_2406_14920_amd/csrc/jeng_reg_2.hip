// jeng_reg_2.hip -- one share of the register J-engine instantiations.
#include "jeng_reg.hpp"

namespace md {

bool launch_jeng_reg_2(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st)
{
    if (lx == 5 && ly == 3) { jeng_reg_launch_t<5, 3>(a, fp32, st); return true; }
    if (lx == 0 && ly == 6) { jeng_reg_launch_t<0, 6>(a, fp32, st); return true; }
    if (lx == 2 && ly == 4) { jeng_reg_launch_t<2, 4>(a, fp32, st); return true; }
    if (lx == 6 && ly == 0) { jeng_reg_launch_t<6, 0>(a, fp32, st); return true; }
    if (lx == 3 && ly == 6) { jeng_reg_launch_t<3, 6>(a, fp32, st); return true; }
    if (lx == 5 && ly == 4) { jeng_reg_launch_t<5, 4>(a, fp32, st); return true; }
    return false;
}

}  // namespace md
