// Tightening kernel variants for 5 attributes.
#define DV_ 5
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d5)
