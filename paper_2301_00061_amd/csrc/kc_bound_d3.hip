// Bound kernels instantiated for d = 3 attributes.
#include "kc_bound_impl.h"
#define DV_ 3
KC_BOUND_DISPATCH(launch_d3, launch_obj64_d3)
