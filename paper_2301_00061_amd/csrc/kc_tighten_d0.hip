// Tightening kernel variants for any attribute count up to 16.
#define DV_ 0
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH_GENERIC(launch_tighten_d0)
