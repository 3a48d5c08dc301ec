// Bound kernels instantiated for d = 1 attributes.
#include "kc_bound_impl.h"
#define DV_ 1
KC_BOUND_DISPATCH(launch_d1, launch_obj64_d1)
