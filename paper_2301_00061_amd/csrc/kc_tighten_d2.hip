// Tightening kernel variants for 2 attributes.
#define DV_ 2
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d2)
