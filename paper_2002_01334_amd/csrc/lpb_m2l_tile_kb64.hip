// Per-offset tiled M2L with fixed KB, FP64.
#include "lpb_m2l_tile_kb.h"

namespace lpb {

template bool launch_m2l_tile_kb<double>(const EvalArgs<double>&, bool, hipStream_t);

}  // namespace lpb
