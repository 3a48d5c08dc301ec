// Tightening kernel variants for 3 attributes.
#define DV_ 3
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d3)
