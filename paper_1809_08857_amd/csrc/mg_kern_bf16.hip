// Stencil kernels instantiated for bf16 storage.
#include "mg_launch.cuh"
MG_DEFINE_TYPE_ENTRIES(mg::bf16, bf16)
