// Tightening kernel variants for 8 attributes.
#define DV_ 8
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d8)
