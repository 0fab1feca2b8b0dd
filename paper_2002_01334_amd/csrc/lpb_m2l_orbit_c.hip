// Orbit-form tiled M2L instantiated for p = 12, 13.
#include "lpb_m2l_orbit.h"

namespace lpb {

template void launch_m2l_orbit_p<12>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<13>(const EvalArgs<float>&, hipStream_t);

}  // namespace lpb
