// Bound kernels instantiated for d = 4 attributes.
#include "kc_bound_impl.h"
#define DV_ 4
KC_BOUND_DISPATCH(launch_d4, launch_obj64_d4)
