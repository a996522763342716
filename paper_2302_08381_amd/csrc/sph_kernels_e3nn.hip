// e3nn's conventions (Sec. III.B: the method's library offers wrappers that
// follow them).  e3nn's real harmonics take y as the polar axis: they are
// the standard ones (Eq. real-sh-cartesian) evaluated at the cyclically
// permuted point (z, x, y), whose degree-1 values are then proportional to
// (x, y, z) in that order, times a per-degree normalisation factor.  The
// forward itself runs unchanged on the permuted points; these two kernels
// prepare them and convert the outputs in place.
#include "sph_device.hpp"
#include "sph_launch.hpp"

namespace sph {
namespace {

constexpr int kConvThreads = 256;

// out[i] = (z_i, x_i, y_i).  Each thread reads its own point before writing
// it, so out may equal xyz.
template <typename T>
__global__ __launch_bounds__(kConvThreads) void k_e3nn_coordinates(const T* xyz, int64_t n, T* out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kConvThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kConvThreads + threadIdx.x; i < n; i += stride) {
    const T x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    out[3 * i] = z;
    out[3 * i + 1] = x;
    out[3 * i + 2] = y;
  }
}

// Per column k of degree l, one thread: Y[p][k] *= c_l and, for the
// derivatives taken at (x', y', z') = (z, x, y), the rows go back to the
// caller's axes: d/dx = d/dy', d/dy = d/dz', d/dz = d/dx'.
//   normalization 0 (integral): c_l = 1, the library's own (unit L2 norm on
//   the sphere); 1 (component): c_l = sqrt(4 pi), so sum_m Y_lm^2 = 2l+1 on
//   the unit sphere; 2 (norm): c_l = sqrt(4 pi / (2l+1)), so the sum is 1.
template <typename T>
__global__ __launch_bounds__(kConvThreads) void k_e3nn_convert(int64_t n, int K, int normalization, T* Y, T* dY) {
  const int64_t total = n * K;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kConvThreads;
  constexpr double kFourPi = 12.566370614359172953850573533118;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kConvThreads + threadIdx.x; t < total; t += stride) {
    const int64_t p = t / K;
    const int k = static_cast<int>(t - p * K);
    int l = static_cast<int>(sqrt(static_cast<double>(k)));
    l += (l + 1) * (l + 1) <= k ? 1 : 0;
    l -= l * l > k ? 1 : 0;
    T c = T(1);
    if (normalization == 1) c = static_cast<T>(sqrt(kFourPi));
    if (normalization == 2) c = static_cast<T>(sqrt(kFourPi / (2 * l + 1)));
    Y[t] *= c;
    if (dY != nullptr) {
      T* d = dY + p * 3 * K + k;
      const T d0 = d[0], d1 = d[K], d2 = d[2 * K];
      d[0] = c * d1;
      d[K] = c * d2;
      d[2 * K] = c * d0;
    }
  }
}

unsigned conv_grid(int64_t work) {
  const int64_t blocks = (work + kConvThreads - 1) / kConvThreads;
  return static_cast<unsigned>(blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks));
}

}  // namespace

hipError_t e3nn_coordinates_launch(int dtype64, const void* xyz, int64_t n, void* out, hipStream_t s) {
  if (dtype64)
    hipLaunchKernelGGL(k_e3nn_coordinates<double>, dim3(conv_grid(n)), dim3(kConvThreads), 0, s,
                       static_cast<const double*>(xyz), n, static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_e3nn_coordinates<float>, dim3(conv_grid(n)), dim3(kConvThreads), 0, s,
                       static_cast<const float*>(xyz), n, static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t e3nn_convert_launch(int dtype64, int64_t n, int L, int normalization, void* Y, void* dY,
                               hipStream_t s) {
  const int K = (L + 1) * (L + 1);
  if (dtype64)
    hipLaunchKernelGGL(k_e3nn_convert<double>, dim3(conv_grid(n * K)), dim3(kConvThreads), 0, s, n, K,
                       normalization, static_cast<double*>(Y), static_cast<double*>(dY));
  else
    hipLaunchKernelGGL(k_e3nn_convert<float>, dim3(conv_grid(n * K)), dim3(kConvThreads), 0, s, n, K,
                       normalization, static_cast<float*>(Y), static_cast<float*>(dY));
  return hipGetLastError();
}

}  // namespace sph
