// Adjoint of the forward propagation (placeholder translation unit; the
// adjoint kernels are added here).
#include "rheed_internal.h"
