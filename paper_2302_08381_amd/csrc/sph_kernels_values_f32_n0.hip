// values-only forward kernels, float, scaled harmonics
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 1
#define SPH_NORM 0
#include "sph_instances.inl"
