// Bound kernels instantiated for d = 8 attributes.
#include "kc_bound_impl.h"
#define DV_ 8
KC_BOUND_DISPATCH(launch_d8, launch_obj64_d8)
