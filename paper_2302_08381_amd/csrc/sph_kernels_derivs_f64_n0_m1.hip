// forward kernels with derivatives (Y, dY and fused backward), double, scaled harmonics
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 3
#define SPH_NORM 0
#define SPH_MODE 1
#include "sph_instances.inl"
