// Bound kernels instantiated for d = 7 attributes.
#include "kc_bound_impl.h"
#define DV_ 7
KC_BOUND_DISPATCH(launch_d7, launch_obj64_d7)
