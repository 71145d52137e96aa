// k_wave_2.hip -- one share of the wave-cooperative exchange instantiations
// (the classes are spread over several files so that they compile in parallel).
#include "class_lists.hpp"
#include "k_wave.hpp"

namespace md {

bool launch_k_wave_2(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st)
{
#define MD_CASE(A_, B_, C_, D_)                                       \
    if (la == A_ && lb == B_ && lc == C_ && ld == D_) {               \
        launch_k_wave_t<A_, B_, C_, D_>(a, fp32, st);                       \
        return true;                                                  \
    }
    MD_K_WAVE_PART2(MD_CASE)
#undef MD_CASE
    return false;
}

}  // namespace md
