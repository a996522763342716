// values-only forward kernels, float, normalised harmonics
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 1
#define SPH_NORM 1
#include "sph_instances.inl"
