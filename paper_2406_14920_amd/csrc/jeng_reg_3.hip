// jeng_reg_3.hip -- one share of the register J-engine instantiations.
#include "jeng_reg.hpp"

namespace md {

bool launch_jeng_reg_3(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st)
{
    if (lx == 2 && ly == 5) { jeng_reg_launch_t<2, 5>(a, fp32, st); return true; }
    if (lx == 3 && ly == 4) { jeng_reg_launch_t<3, 4>(a, fp32, st); return true; }
    if (lx == 1 && ly == 5) { jeng_reg_launch_t<1, 5>(a, fp32, st); return true; }
    if (lx == 5 && ly == 1) { jeng_reg_launch_t<5, 1>(a, fp32, st); return true; }
    if (lx == 4 && ly == 5) { jeng_reg_launch_t<4, 5>(a, fp32, st); return true; }
    if (lx == 4 && ly == 6) { jeng_reg_launch_t<4, 6>(a, fp32, st); return true; }
    return false;
}

}  // namespace md
