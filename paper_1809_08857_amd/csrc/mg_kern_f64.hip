// Stencil kernels instantiated for double storage.
#include "mg_launch.cuh"
MG_DEFINE_TYPE_ENTRIES(double, f64)
