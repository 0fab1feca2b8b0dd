// Orbit-form tiled M2L instantiated for p = 14, 15.
#include "lpb_m2l_orbit.h"

namespace lpb {

template void launch_m2l_orbit_p<14>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<15>(const EvalArgs<float>&, hipStream_t);

}  // namespace lpb
