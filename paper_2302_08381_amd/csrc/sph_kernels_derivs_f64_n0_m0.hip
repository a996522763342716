// forward kernels with derivatives (Y and dY), double, scaled harmonics
#define SPH_T double
#define SPH_SUFFIX f64
#define SPH_FAMILY 3
#define SPH_NORM 0
#define SPH_MODE 0
#include "sph_instances.inl"
