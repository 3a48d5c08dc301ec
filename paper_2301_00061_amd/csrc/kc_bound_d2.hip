// Bound kernels instantiated for d = 2 attributes.
#include "kc_bound_impl.h"
#define DV_ 2
KC_BOUND_DISPATCH(launch_d2, launch_obj64_d2)
