// forward kernels, double
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 1
#include "sph_instances.inl"
