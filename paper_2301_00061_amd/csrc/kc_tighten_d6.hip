// Tightening kernel variants for 6 attributes.
#define DV_ 6
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d6)
