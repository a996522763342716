// forward kernels, float
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 1
#include "sph_instances.inl"
