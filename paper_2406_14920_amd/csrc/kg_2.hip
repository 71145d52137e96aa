// kg_2.hip -- one share of the exchange-gradient instantiations.
#include "class_lists.hpp"
#include "grad.hpp"

namespace md {

bool launch_kg_2(int la, int lb, int lc, int ld, const KGArgs &g, int blocks, hipStream_t st)
{
#define MD_CASE(A_, B_, C_, D_)                                   \
    if (la == A_ && lb == B_ && lc == C_ && ld == D_) {           \
        launch_kg_any<A_, B_, C_, D_>(g, blocks, st);               \
        return true;                                              \
    }
    MD_KG_PART2(MD_CASE)
#undef MD_CASE
    return false;
}

}  // namespace md
