// Orbit-form tiled M2L instantiated for p = 10, 11.
#include "lpb_m2l_orbit.h"

namespace lpb {

template void launch_m2l_orbit_p<10>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<11>(const EvalArgs<float>&, hipStream_t);

}  // namespace lpb
