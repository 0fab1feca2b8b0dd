// Per-offset tiled M2L with fixed KB, FP32.
#include "lpb_m2l_tile_kb.h"

namespace lpb {

template bool launch_m2l_tile_kb<float>(const EvalArgs<float>&, bool, hipStream_t);

}  // namespace lpb
