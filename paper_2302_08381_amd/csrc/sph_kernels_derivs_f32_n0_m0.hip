// forward kernels with derivatives (Y and dY), float, scaled harmonics
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 3
#define SPH_NORM 0
#define SPH_MODE 0
#include "sph_instances.inl"
