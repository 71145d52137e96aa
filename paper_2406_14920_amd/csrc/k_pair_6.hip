// k_pair_6.hip -- instantiations of the bra-shared exchange kernel.
#include "class_lists.hpp"
#include "k_pair.hpp"

namespace md {

bool launch_k_pair_6(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st)
{
#define MD_CASE(A_, B_, C_, D_)                                   \
    if (la == A_ && lb == B_ && lc == C_ && ld == D_) {           \
        launch_k_pair_t<A_, B_, C_, D_>(a, nchunks, fp32, st);          \
        return true;                                              \
    }
    MD_K_PAIR_PART6(MD_CASE)
#undef MD_CASE
    return false;
}

}  // namespace md
