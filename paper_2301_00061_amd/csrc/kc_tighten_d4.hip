// Tightening kernel variants for 4 attributes.
#define DV_ 4
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d4)
