// backward and double-backward kernels, float
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 2
#include "sph_instances.inl"
