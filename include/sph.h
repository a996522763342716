/*
 * sph.h -- C ABI of libsph: real spherical harmonics and their Cartesian
 * derivatives for batches of points on AMD Instinct MI355X (gfx950).
 *
 * The method is the Cartesian formulation of "Fast evaluation of spherical
 * harmonics with sphericart" (arXiv:2302.08381): scaled (solid) harmonics
 * r^l Y_l^m = F_l^{|m|} Q_l^{|m|}(z,r) {s_|m|, 1/sqrt2, c_m}
 * (Eq. real-sh-cartesian) built from the polynomials Q_l^m, s_m, c_m of
 * Eq. define-q by the recursions of Eqs. iter-q-alt and iter-sc, with the
 * prefactors F_l^m (Eq. Flm, App. C) folded into Q, and the derivatives of
 * Eq. iter-deri.  The normalised harmonics are the scaled ones evaluated at
 * x/r with the chain rule applied to the derivatives (Sec. III).
 *
 * Conventions shared by every entry point
 * --------------------------------------
 * - Layout: contiguous row-major arrays.  For l_max = L there are
 *   K = (L+1)^2 harmonics per point; column k = l*l + l + m with m running
 *   from -l to l.  xyz is [n,3]; Y is [n,K]; dY is [n,3,K] (for each point,
 *   the x, y and z derivative blocks of K values each).
 * - Memory: every data pointer is a DEVICE pointer owned by the caller.
 *   The library never allocates, frees or retains caller memory.  Outputs
 *   must not overlap inputs.  16-byte aligned base pointers take the
 *   vectorised store path; other alignments are accepted and slower.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  All work is enqueued asynchronously on it; nothing
 *   synchronises the host except where stated.
 * - Errors: arguments are validated on the host before anything is
 *   enqueued.  On an error the call returns a non-zero sph_status_t, writes
 *   nothing, and sph_last_error() holds a message (per host thread).
 *   n = 0 (or n_env = 0) is valid and enqueues nothing (except a requested
 *   status word, below).  A failed kernel launch returns SPH_ERR_DEVICE.
 * - One exception: CSR offsets.  The offsets of the CSR entry points
 *   (sph_batched_compute, sph_radial_expansion and its backward) live in
 *   device memory, so the host does not read them: doing so would need a
 *   device-to-host copy and a synchronisation on every call, which rules
 *   out asynchronous launches and graph capture.  The kernel checks them
 *   instead (offsets[0] == 0, non-decreasing, offsets[n_env] == n_points)
 *   and writes SPH_OK or SPH_ERR_OFFSETS to the caller's optional status
 *   word.  The call itself returns SPH_OK once the launch is enqueued; what
 *   the outputs hold when the offsets are inconsistent is stated per entry
 *   point.  A caller that passes no status word gets no report.
 * - Numerics: NaN/Inf inputs propagate to the outputs; they are not errors.
 *   At r = 0 the scaled harmonics take their polynomial values; the
 *   normalised ones return Y_0^0 = 1/(2 sqrt(pi)) and 0 for every other
 *   value and derivative.  float32 kernels work in float32 throughout;
 *   float64 kernels in float64.
 * - Range: 0 <= l_max <= sph_max_lmax() (32).
 */
#ifndef SPH_H_
#define SPH_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPH_F32 = 0, /* float  */
  SPH_F64 = 1  /* double */
} sph_dtype_t;

typedef enum {
  SPH_OK = 0,
  SPH_ERR_NULL = 1,    /* a required pointer is NULL while n > 0            */
  SPH_ERR_INVALID = 2, /* n < 0, normalize not 0/1, bad dtype, bad option   */
  SPH_ERR_LMAX = 3,    /* l_max < 0 or l_max > sph_max_lmax()               */
  SPH_ERR_OFFSETS = 4, /* CSR offsets inconsistent (batched entry point)    */
  SPH_ERR_DEVICE = 5   /* the HIP runtime reported an error                 */
} sph_status_t;

/* (l_max+1)^2, the number of harmonics per point; -1 if l_max < 0. */
int32_t sph_num_components(int32_t l_max);

/* Largest supported l_max (32). */
int32_t sph_max_lmax(void);

/* Static description of a status code.  Never NULL. */
const char* sph_status_string(int32_t status);

/* Detail of the last error on the calling host thread ("" if none). */
const char* sph_last_error(void);

/* Library version string, e.g. "1.0.0 gfx950". */
const char* sph_version(void);

/*
 * sph_compute -- Y[n,K] for n points.
 * Sec. II (Eqs. real-sh-cartesian, define-q, iter-q-alt, iter-sc) and
 * Sec. III (normalised variant).
 *   xyz        in  [n,3]  point coordinates
 *   n          number of points (>= 0)
 *   l_max      0..sph_max_lmax()
 *   normalize  0: scaled harmonics r^l Y_l^m; 1: normalised Y_l^m
 *   dtype      element type of xyz and Y
 *   Y          out [n,K]
 */
int32_t sph_compute(const void* xyz, int64_t n, int32_t l_max, int32_t normalize,
                    int32_t dtype, void* Y, void* stream);

/*
 * sph_compute_with_gradients -- Y[n,K] and dY[n,3,K] = dY/dxyz in one pass.
 * Derivatives from Eq. iter-deri (Sec. II) with the product rule; for
 * normalize = 1 the chain rule through x/r (Sec. III).
 *   dY         out [n,3,K]; dY[i,a,k] = d Y[i,k] / d xyz[i,a]
 * Other arguments as sph_compute.
 */
int32_t sph_compute_with_gradients(const void* xyz, int64_t n, int32_t l_max,
                                   int32_t normalize, int32_t dtype, void* Y,
                                   void* dY, void* stream);

/*
 * sph_backward -- grad_xyz[i,a] = sum_k grad_Y[i,k] * dY[i,a,k].
 * The vector-Jacobian product of the forward, reusing the derivatives it
 * stored (the custom backward of Sec. III).
 *   dY         in  [n,3,K] as written by sph_compute_with_gradients
 *   grad_Y     in  [n,K]   upstream gradient dL/dY
 *   grad_xyz   out [n,3]
 */
int32_t sph_backward(const void* dY, const void* grad_Y, int64_t n, int32_t l_max,
                     int32_t dtype, void* grad_xyz, void* stream);

/*
 * sph_double_backward -- the derivatives of L' = sum_{i,a} v[i,a] grad_xyz[i,a]
 * where grad_xyz is the output of sph_backward:
 *   grad_grad_Y[i,k] = sum_a v[i,a] dY[i,a,k]
 *   grad_xyz2[i,b]   = sum_k grad_Y[i,k] sum_a v[i,a] d2Y[i,k]/dxyz_a dxyz_b
 * Second derivatives come from applying Eq. iter-deri twice (Sec. II:
 * derivatives of any order); they are formed in registers from xyz and
 * never stored.
 *   xyz            in  [n,3]
 *   grad_Y         in  [n,K]
 *   v              in  [n,3]  (upstream gradient of grad_xyz)
 *   grad_grad_Y    out [n,K]  (may be NULL: not computed)
 *   grad_xyz2      out [n,3]  (may be NULL: not computed)
 */
int32_t sph_double_backward(const void* xyz, const void* grad_Y, const void* v,
                            int64_t n, int32_t l_max, int32_t normalize,
                            int32_t dtype, void* grad_grad_Y, void* grad_xyz2,
                            void* stream);

/*
 * sph_compute_with_hessians -- Y[n,K], dY[n,3,K] and the second derivatives
 * d2Y[n,3,3,K], d2Y[i,a,b,k] = d^2 Y[i,k] / (d xyz[i,a] d xyz[i,b]) (the full
 * symmetric 3x3 block of every column).  Sec. II: the Cartesian recursion
 * gives derivatives of any order; here Eq. iter-deri is applied twice, with
 * the product rule and, for normalize = 1, the chain rule through x/r
 * (Sec. III).  At r = 0 the normalised second derivatives are 0.
 *   Y          out [n,K]       (required)
 *   dY         out [n,3,K]     (may be NULL: not stored)
 *   d2Y        out [n,3,3,K]   (required)
 * Other arguments as sph_compute.  Two launches on `stream`: the forward of
 * sph_compute_with_gradients, then the second-derivative kernel.
 */
int32_t sph_compute_with_hessians(const void* xyz, int64_t n, int32_t l_max,
                                  int32_t normalize, int32_t dtype, void* Y,
                                  void* dY, void* d2Y, void* stream);

/*
 * e3nn's conventions (Sec. III.B: the method's library provides wrappers
 * that follow them).  e3nn's real harmonics take y as the polar axis: they
 * are this library's harmonics evaluated at the cyclically permuted point
 * (z, x, y) (so that degree 1 is proportional to (x, y, z), in that order),
 * times a per-degree normalisation factor, with the derivatives taken along
 * the caller's axes.  A call of e3nn's convention is
 *   sph_e3nn_coordinates(xyz -> xyz_p), sph_compute_with_gradients(xyz_p ->
 *   Y, dY), sph_e3nn_convert(Y, dY),
 * all on one stream; the backward of the result is sph_backward with the
 * converted dY.
 *
 * sph_e3nn_coordinates -- xyz_p[i] = (xyz[i,2], xyz[i,0], xyz[i,1]).
 *   xyz        in  [n,3]
 *   xyz_p      out [n,3]; may be xyz itself (each point is read before it is
 *              written), must not overlap it otherwise
 * Errors: SPH_ERR_NULL for a NULL buffer with n > 0; SPH_ERR_INVALID for
 * n < 0, a bad dtype or a partial overlap.
 */
int32_t sph_e3nn_coordinates(const void* xyz, int64_t n, int32_t dtype,
                             void* xyz_p, void* stream);

/*
 * sph_e3nn_convert -- in place, turns Y[n,K] (and dY[n,3,K]) computed at
 * sph_e3nn_coordinates' points into e3nn's convention:
 *   Y[i,k] *= c_l,  (dY[i,0,k], dY[i,1,k], dY[i,2,k]) <-
 *                   c_l (dY[i,1,k], dY[i,2,k], dY[i,0,k])   (k of degree l)
 * (the derivatives along the permuted axes (z, x, y) become derivatives
 * along (x, y, z)).
 *   normalization  0 "integral": c_l = 1 (this library's, unit L2 norm on
 *                  the sphere); 1 "component": c_l = sqrt(4 pi), so that
 *                  sum_m Y_lm^2 = 2l+1 on the unit sphere; 2 "norm":
 *                  c_l = sqrt(4 pi / (2l+1)), so that the sum is 1
 *   Y              in/out [n,K] (required)
 *   dY             in/out [n,3,K] (may be NULL)
 * Errors: SPH_ERR_NULL for a NULL Y with n > 0; SPH_ERR_LMAX; SPH_ERR_INVALID
 * for n < 0, a bad dtype or normalization, or overlapping Y and dY.
 */
int32_t sph_e3nn_convert(int64_t n, int32_t l_max, int32_t normalization,
                         int32_t dtype, void* Y, void* dY, void* stream);

/*
 * sph_batched_compute -- many neighbour lists in one persistent launch.
 * The points of n_env environments are concatenated (CSR): environment e
 * owns rows offsets[e] .. offsets[e+1]-1 of xyz (Sec. III: the harmonics of
 * the neighbours of each selected atom).  Every output follows the
 * concatenated row order.  The launch is a persistent kernel replayed from a
 * cached hipGraph: one graph per (dtype, l_max, normalize, outputs)
 * combination and kernel, whose grid and arguments each call sets, so calls
 * with a changing n_points reuse it.  On the first call for a combination
 * with at least 16384 points, outside a stream capture, the library times
 * its candidate launches on the caller's own buffers and keeps the fastest;
 * the timing synchronises the host once.  Smaller or captured calls use the
 * defaults and leave the combination to be tuned by a later call.  The
 * candidates are every kernel variant (the unrolled compile-time kernel on
 * its default tile, the same on a 16-point tile, the
 * run-time-degree kernel, the 16-point tile with its degrees split between
 * two waves, and for l_max <= 3 the kernel with one lane per point) crossed
 * with every persistent-grid size.
 *   xyz        in  [n_points,3]
 *   offsets    in  int64 [n_env+1], DEVICE memory
 *   n_env      number of environments (>= 0)
 *   n_points   total number of points; must equal offsets[n_env]
 *   Y          out [n_points,K]
 *   dY         out [n_points,3,K]  (may be NULL: derivatives not stored)
 *   grad_Y     in  [n_points,K]    (may be NULL: no backward)
 *   grad_xyz   out [n_points,3]    (required iff grad_Y is given) --
 *              the backward of sph_backward, fused into the same pass
 *   status     out int32 [1], DEVICE memory (may be NULL).  The kernel
 *              checks offsets[0] == 0, non-decreasing offsets and
 *              offsets[n_env] == n_points, and writes SPH_OK or
 *              SPH_ERR_OFFSETS there.  The outputs do not depend on the
 *              offsets, so they are complete either way.
 */
int32_t sph_batched_compute(const void* xyz, const int64_t* offsets, int64_t n_env,
                            int64_t n_points, int32_t l_max, int32_t normalize,
                            int32_t dtype, void* Y, void* dY, const void* grad_Y,
                            void* grad_xyz, int32_t* status, void* stream);

/*
 * sph_radial_expansion -- the expansion of each environment in radial
 * functions times harmonics (Sec. I, Eq. expansion):
 *   c[e, n, l^2+l+m] = sum over offsets[e] <= j < offsets[e+1] of
 *                      R[j, l, n] * Y_l^m(xyz[j])
 * with Y the normalised harmonics of the direction (normalize = 1) or the
 * solid harmonics r^l Y (normalize = 0).  The radial values R are the
 * caller's: the paper leaves the radial basis open.  The harmonics are
 * contracted on chip and never written to memory.
 *   xyz        in  [n_points,3]
 *   offsets    in  int64 [n_env+1], DEVICE memory (CSR, as in
 *              sph_batched_compute)
 *   n_env      number of environments (>= 0)
 *   n_points   total number of points; must equal offsets[n_env]
 *   R          in  [n_points, l_max+1, n_max]: R[j,l,n] = R_nl(r_j)
 *   n_max      radial channels, 1 .. 64
 *   c          out [n_env, n_max, (l_max+1)^2]; empty environments get 0
 *   status     out int32 [1], DEVICE memory (may be NULL): SPH_OK or
 *              SPH_ERR_OFFSETS, checked as in sph_batched_compute.  With
 *              inconsistent offsets each environment's range is clamped to
 *              [0, n_points] (no access outside the buffers) and c is
 *              undefined.
 * SPH_ERR_INVALID if l_max and n_max need more than one block's 160 KiB of
 * LDS for an 8-point chunk (never for n_max <= 8, or l_max <= 16 with
 * n_max <= 32).
 */
int32_t sph_radial_expansion(const void* xyz, const int64_t* offsets, int64_t n_env,
                             int64_t n_points, const void* R, int32_t n_max,
                             int32_t l_max, int32_t normalize, int32_t dtype,
                             void* c, int32_t* status, void* stream);

/*
 * sph_radial_expansion_backward -- the backward of sph_radial_expansion for
 * an upstream gradient grad_c = dL/dc (chain rule through Eq. expansion and
 * the Cartesian derivatives of Eq. iter-deri):
 *   grad_R[j, l, n] = sum_m grad_c[e, n, l^2+l+m] * Y_l^m(xyz[j])
 *   grad_xyz[j, a]  = sum_{n,k} grad_c[e, n, k] * R[j, l(k), n]
 *                     * dY_k/dx_a(xyz[j])
 * for the environment e holding point j.  Neither Y nor dY is stored.
 *   xyz, offsets, n_env, n_points, R, l_max, normalize, dtype, status:
 *              as in sph_radial_expansion
 *   n_max      radial channels, 1 .. 16
 *   grad_c     in  [n_env, n_max, (l_max+1)^2]
 *   grad_xyz   out [n_points, 3]              (may be NULL)
 *   grad_R     out [n_points, l_max+1, n_max] (may be NULL)
 * Rows of points outside every environment's range (possible only with
 * inconsistent offsets) are not written.
 */
int32_t sph_radial_expansion_backward(const void* xyz, const int64_t* offsets, int64_t n_env,
                                      int64_t n_points, const void* R, int32_t n_max,
                                      int32_t l_max, int32_t normalize, int32_t dtype,
                                      const void* grad_c, void* grad_xyz, void* grad_R,
                                      int32_t* status, void* stream);

/*
 * sph_batched_set_options -- batched-path controls (process-wide).
 *   use_graph  1: replay cached hipGraphs (default); 0: plain launches
 *   autotune   1: time the candidate launches on first use (default);
 *              0: use the built-in defaults
 */
int32_t sph_batched_set_options(int32_t use_graph, int32_t autotune);

/*
 * sph_batched_get_config -- the launch chosen for a combination, as
 * "kernel=<v> blocks_per_cu=<b> tile_points=<t>" in buf (NUL-terminated, at
 * most len bytes).  v is default, tile16, runtime_degree or degree_split;
 * blocks_per_cu = 0 means one tile per block.  Returns SPH_ERR_INVALID if
 * nothing was chosen yet.
 */
int32_t sph_batched_get_config(int32_t l_max, int32_t normalize, int32_t dtype,
                               int32_t store_dY, int32_t with_backward,
                               char* buf, int32_t len);

/*
 * sph_batched_set_config -- fixes the launch of a combination instead of
 * timing the candidates (for callers that need a known launch, e.g. before
 * capturing a graph, and for testing every variant).
 *   variant        0 default, 1 tile16, 2 runtime_degree, 3 degree_split,
 *                  4 one_lane (as in sph_batched_get_config)
 *   blocks_per_cu  0 .. 64 (0: one tile per block)
 * Returns SPH_ERR_INVALID for an unknown combination, a variant that does
 * not exist for it, or an out of range blocks_per_cu; SPH_ERR_LMAX for l_max
 * out of range.  With dY or the backward: tile16 exists wherever the
 * default is unrolled (float l_max <= 12, double l_max <= 8),
 * runtime_degree for every l_max, degree_split for float 9 <= l_max <= 12,
 * double 4 <= l_max <= 8 and, without the backward, every larger l_max;
 * one_lane for l_max <= 3; a variant may name the default kernel.  Values
 * only: runtime_degree where the default is unrolled.
 */
int32_t sph_batched_set_config(int32_t l_max, int32_t normalize, int32_t dtype,
                               int32_t store_dY, int32_t with_backward,
                               int32_t variant, int32_t blocks_per_cu);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H_ */
