// backward and double-backward kernels, double
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 2
#include "sph_instances.inl"
