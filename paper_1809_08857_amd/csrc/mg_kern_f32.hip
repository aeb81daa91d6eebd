// Stencil kernels instantiated for float storage.
#include "mg_launch.cuh"
MG_DEFINE_TYPE_ENTRIES(float, f32)
