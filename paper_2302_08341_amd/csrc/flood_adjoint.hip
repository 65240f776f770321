// Discrete adjoint kernels of libflood (placeholder translation unit).
#include "flood_internal.h"
