// grid.hpp -- constant shared by the grid kernels and their host set-up.
#pragma once

namespace md {

// the grid kernels drop a primitive pair at a point where p |r - P|^2 exceeds
// this (exp(-100) ~ 4e-44; the paper's cut-off value)
constexpr double kGridCut = 100.0;

}  // namespace md
