// values-only forward kernels, double, scaled harmonics
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 1
#define SPH_NORM 0
#include "sph_instances.inl"
