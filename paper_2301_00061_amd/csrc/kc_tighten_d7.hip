// Tightening kernel variants for 7 attributes.
#define DV_ 7
#include "kc_tighten_impl.h"
KC_TIGHTEN_DISPATCH(launch_tighten_d7)
