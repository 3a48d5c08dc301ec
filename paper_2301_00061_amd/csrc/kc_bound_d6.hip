// Bound kernels instantiated for d = 6 attributes.
#include "kc_bound_impl.h"
#define DV_ 6
KC_BOUND_DISPATCH(launch_d6, launch_obj64_d6)
