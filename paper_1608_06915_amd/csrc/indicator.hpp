// indicator.hpp -- launcher of the per-brick under-resolution indicator (indicator.hip).
#pragma once
#include "elbm_dev.hpp"

namespace elbm {

// Largest |gamma - 2| over each brick's fluid nodes of `level`, stored at the brick's
// place in the dense brick grid `grid` (x fastest); -1 where a brick has no fluid node
// or no brick exists.  `lev_dev` must hold a per-node gamma buffer for the level.
int launch_gamma_indicator(int D, const LevelStatic *lev_dev, int level, int nbricks, const int32_t *borg, Dims box,
                           Dims grid, float *out, void *stream);

}  // namespace elbm
