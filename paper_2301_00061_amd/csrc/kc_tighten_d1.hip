// Tightening kernel variants for 1 attribute.
#define DV_ 1
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d1)
