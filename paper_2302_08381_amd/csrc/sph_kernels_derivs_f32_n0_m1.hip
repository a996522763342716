// forward kernels with derivatives (Y, dY and fused backward), float, scaled harmonics
#define SPH_T float
#define SPH_SUFFIX f32
#define SPH_FAMILY 3
#define SPH_NORM 0
#define SPH_MODE 1
#include "sph_instances.inl"
