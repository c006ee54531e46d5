// MoCHy-A+ (Algorithm 5) on the device: filled in by the sampling kernels.
#include "common.h"
