// Bound kernels instantiated for any attribute count d <= 16 (generic).
#include "kc_bound_impl.h"
#define DV_ 0
KC_BOUND_DISPATCH(launch_d0, launch_obj64_d0)
