// Significance and characteristic profile (Eq. 1, Eq. 2) on the device.
#include "common.h"
