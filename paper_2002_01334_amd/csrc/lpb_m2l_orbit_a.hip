// Orbit-form tiled M2L instantiated for p = 5, 6, 7, 8, 9.
#include "lpb_m2l_orbit.h"

namespace lpb {

template void launch_m2l_orbit_p<5>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<6>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<7>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<8>(const EvalArgs<float>&, hipStream_t);
template void launch_m2l_orbit_p<9>(const EvalArgs<float>&, hipStream_t);

}  // namespace lpb
