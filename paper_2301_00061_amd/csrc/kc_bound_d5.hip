// Bound kernels instantiated for d = 5 attributes.
#include "kc_bound_impl.h"
#define DV_ 5
KC_BOUND_DISPATCH(launch_d5, launch_obj64_d5)
