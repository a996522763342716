// values-only forward kernels, double, normalised harmonics
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 1
#define SPH_NORM 1
#include "sph_instances.inl"
