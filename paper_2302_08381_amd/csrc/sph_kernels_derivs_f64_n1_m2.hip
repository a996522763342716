// forward kernels with derivatives (Y and fused backward), double, normalised harmonics
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 3
#define SPH_NORM 1
#define SPH_MODE 2
#include "sph_instances.inl"
