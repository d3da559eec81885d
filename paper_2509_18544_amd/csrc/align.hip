// Alignment of the template to the science frame (include/sfft_align.h):
// polynomial pixel map, normalised 6-tap Lanczos-3 resampling of the image
// and its mask, and the PSF stamp resampled by the map's Jacobian.
//
// The image resampling is a gather: every output pixel reads 36 template
// pixels (the neighbouring outputs read nearly the same ones, so the reuse is
// served by L1/L2) and 36 mask bytes, and writes one value and one mask byte.
// Blocks cover 64 x 4 output tiles (one wave per row of 64 pixels: the
// template rows a wave touches are contiguous), and consecutive tiles go to
// one XCD so that neighbouring tiles share its L2.
// The arithmetic is FP64 and bound by the FP64 units rather than by memory,
// so the Lanczos weights take one sincos(pi f / 3) per axis and no division
// (lanczos6); an integer offset (f = 0) gives the weights (0, 0, 1, 0, 0, 0)
// exactly and the copy is exact.  Images of T = double or float.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/sfft.h"
#include "../../include/sfft_align.h"
#include "common.hpp"

namespace {

constexpr int AX = 64, AY = 4;   // output tile (pixels): 4 waves, one row of 64 each
constexpr int PSF_MAXS = 31;
constexpr int PSF_THREADS = 1024;
constexpr int IMG_MAX = 65536;

__device__ __forceinline__ void map_eval(const sfft_pixel_map& M, double x, double y, double* xt, double* yt) {
  const double u = x - M.x_ref, v = y - M.y_ref;
  double m[10];
  m[0] = 1.0;
  m[1] = u;
  m[2] = v;
  m[3] = u * u;
  m[4] = u * v;
  m[5] = v * v;
  m[6] = m[3] * u;
  m[7] = m[3] * v;
  m[8] = u * m[5];
  m[9] = m[5] * v;
  const int nm = (M.deg + 1) * (M.deg + 2) / 2;
  double a = 0.0, b = 0.0;
  for (int j = 0; j < nm; ++j) {
    a += M.cx[j] * m[j];
    b += M.cy[j] * m[j];
  }
  *xt = a;
  *yt = b;
}

// Jacobian [[dx_t/dx, dx_t/dy], [dy_t/dx, dy_t/dy]] of the map at (x, y)
__device__ __forceinline__ void map_jacobian(const sfft_pixel_map& M, double x, double y, double J[4]) {
  const double u = x - M.x_ref, v = y - M.y_ref;
  // d/du and d/dv of the monomials 1; u, v; u^2, uv, v^2; u^3, u^2 v, u v^2, v^3
  const double du[10] = {0.0, 1.0, 0.0, 2.0 * u, v, 0.0, 3.0 * u * u, 2.0 * u * v, v * v, 0.0};
  const double dv[10] = {0.0, 0.0, 1.0, 0.0, u, 2.0 * v, 0.0, u * u, 2.0 * u * v, 3.0 * v * v};
  const int nm = (M.deg + 1) * (M.deg + 2) / 2;
  J[0] = J[1] = J[2] = J[3] = 0.0;
  for (int j = 0; j < nm; ++j) {
    J[0] += M.cx[j] * du[j];
    J[1] += M.cx[j] * dv[j];
    J[2] += M.cy[j] * du[j];
    J[3] += M.cy[j] * dv[j];
  }
}

// Lanczos-3 weights of the taps k = -2..3 at offsets t = f - k (0 <= f < 1),
// L(t) = 3 sin(pi t) sin(pi t / 3) / (pi^2 t^2), L(0) = 1, up to one common
// factor (the caller normalises by their sum, which it gets back): with
//   sin(pi (f - k))     = (-1)^k sin(pi f),  sin(pi f) = s (3 - 4 s^2), s = sin(pi f / 3),
//   sin(pi (f - k) / 3) = s cos(pi k / 3) - c sin(pi k / 3),  c = cos(pi f / 3),
// and 1 / t_k^2 = (prod_{j != k} t_j^2) / prod_j t_j^2, the weights need one
// sincos and no division.  f = 0 gives (0, 0, 1, 0, 0, 0) exactly.
__device__ __forceinline__ double lanczos6(double f, double w[6]) {
  constexpr double H = 0.86602540378443864676;               // sin(pi / 3)
  constexpr double C3[6] = {-0.5, 0.5, 1.0, 0.5, -0.5, -1.0};  // cos(pi k / 3)
  constexpr double S3[6] = {-H, -H, 0.0, H, H, 0.0};           // sin(pi k / 3)
  if (f == 0.0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) w[k] = (k == 2) ? 1.0 : 0.0;
    return 1.0;
  }
  double s3, c3;
  sincospi(f * (1.0 / 3.0), &s3, &c3);
  const double sp = s3 * (3.0 - 4.0 * s3 * s3);
  double t2[6], pre[6], suf[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double t = f - (double)(k - 2);
    t2[k] = t * t;
  }
  pre[0] = 1.0;
#pragma unroll
  for (int k = 1; k < 6; ++k) pre[k] = pre[k - 1] * t2[k - 1];
  suf[5] = 1.0;
#pragma unroll
  for (int k = 4; k >= 0; --k) suf[k] = suf[k + 1] * t2[k + 1];
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double sk = (k & 1) ? -sp : sp;                     // (-1)^k sin(pi f)
    w[k] = sk * (s3 * C3[k] - c3 * S3[k]) * (pre[k] * suf[k]);
    sum += w[k];
  }
  return sum;
}

template <typename T>
__global__ __launch_bounds__(AX * AY) void align_image_kernel(sfft_pixel_map M, const T* __restrict__ src,
                                                              const uint8_t* __restrict__ smask, int nyt, int nxt,
                                                              int64_t ldt, T* __restrict__ out,
                                                              uint8_t* __restrict__ omask, int ny, int nx, int64_t ld,
                                                              int tiles_x, int ntiles) {
  const int tile = sfft::xcd_remap(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int x = tx * AX + (threadIdx.x & (AX - 1)), y = ty * AY + (threadIdx.x / AX);
  if (x >= nx || y >= ny) return;
  double xt, yt;
  map_eval(M, (double)x, (double)y, &xt, &yt);
  const int64_t o = (int64_t)y * ld + x;
  // all 36 taps inside: 2 <= floor(x_t) <= nx_t - 4 (a NaN coordinate fails too)
  if (!(xt >= 2.0 && xt < (double)(nxt - 3) && yt >= 2.0 && yt < (double)(nyt - 3))) {
    out[o] = (T)0;
    omask[o] = 1;
    return;
  }
  const int i0 = (int)floor(xt), j0 = (int)floor(yt);
  double wx[6], wy[6];
  const double sx = lanczos6(xt - (double)i0, wx);
  const double sy = lanczos6(yt - (double)j0, wy);
  const T* __restrict__ r = src + (int64_t)(j0 - 2) * ldt + (i0 - 2);
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) a += wx[i] * (double)r[(int64_t)j * ldt + i];
    acc += wy[j] * a;
  }
  int mk = 0;
  if (smask != nullptr) {
    const uint8_t* __restrict__ q = smask + (int64_t)(j0 - 2) * ldt + (i0 - 2);
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int i = 0; i < 6; ++i) mk |= q[(int64_t)j * ldt + i];
  }
  out[o] = (T)(acc / (sx * sy));
  omask[o] = mk != 0 ? 1 : 0;
}

// One block: every output tap samples the template stamp at J (u, v) (taps
// outside the stamp count as 0), then the stamp is scaled to the template
// stamp's sum.
__global__ __launch_bounds__(PSF_THREADS) void align_psf_kernel(sfft_pixel_map M, double x0, double y0,
                                                                const double* __restrict__ psf_t, int st,
                                                                double* __restrict__ psf, int s) {
  __shared__ double red[2][PSF_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double J[4];
  map_jacobian(M, x0, y0, J);
  const int L = 2 * s + 1, Lt = 2 * st + 1;
  double part = 0.0, tin = 0.0;
  for (int e = tid; e < Lt * Lt; e += PSF_THREADS) tin += psf_t[e];
  for (int e = tid; e < L * L; e += PSF_THREADS) {
    const double u = (double)(e % L - s), v = (double)(e / L - s);
    const double xt = (double)st + J[0] * u + J[1] * v;
    const double yt = (double)st + J[2] * u + J[3] * v;
    const double fi = floor(xt), fj = floor(yt);
    double wx[6], wy[6];
    const double sx = lanczos6(xt - fi, wx);
    const double sy = lanczos6(yt - fj, wy);
    double num = 0.0;
    for (int j = 0; j < 6; ++j) {
      const double jj = fj + (double)(j - 2);
      if (jj < 0.0 || jj > (double)(Lt - 1)) continue;
      double a = 0.0;
      for (int i = 0; i < 6; ++i) {
        const double ii = fi + (double)(i - 2);
        if (ii < 0.0 || ii > (double)(Lt - 1)) continue;
        a += wx[i] * psf_t[(int)jj * Lt + (int)ii];
      }
      num += wy[j] * a;
    }
    const double val = num / (sx * sy);
    psf[e] = val;
    part += val;
  }
  for (int off = 32; off > 0; off >>= 1) {
    part += __shfl_down(part, off, 64);
    tin += __shfl_down(tin, off, 64);
  }
  if (lane == 0) {
    red[0][wave] = part;
    red[1][wave] = tin;
  }
  __syncthreads();
  double tot = 0.0, sum_t = 0.0;
  for (int k = 0; k < PSF_THREADS / 64; ++k) {
    tot += red[0][k];
    sum_t += red[1][k];
  }
  if (tot == 0.0) return;
  const double scale = sum_t / tot;
  for (int e = tid; e < L * L; e += PSF_THREADS) psf[e] *= scale;
}

int check_map(const sfft_pixel_map* m) {
  if (m == nullptr || m->deg < 0 || m->deg > 3) return SFFT_EINVAL;
  return SFFT_OK;
}

}  // namespace

extern "C" {

int sfft_align_image(const sfft_pixel_map* map, int32_t mode, void* hip_stream, const void* tmpl,
                     const uint8_t* tmpl_mask, int32_t ny_t, int32_t nx_t, int64_t ld_t, void* out,
                     uint8_t* out_mask, int32_t ny, int32_t nx, int64_t ld) {
  if (check_map(map) != SFFT_OK || tmpl == nullptr || out == nullptr || out_mask == nullptr) return SFFT_EINVAL;
  if (mode != SFFT_MODE_F64 && mode != SFFT_MODE_F32C) return SFFT_EINVAL;
  if (ny_t < 1 || nx_t < 1 || ny < 1 || nx < 1 || ny_t > IMG_MAX || nx_t > IMG_MAX || ny > IMG_MAX || nx > IMG_MAX)
    return SFFT_EINVAL;
  if (ld_t < nx_t || ld < nx) return SFFT_EINVAL;
  const size_t es = mode == SFFT_MODE_F64 ? sizeof(double) : sizeof(float);
  {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(tmpl), a1 = a0 + ((size_t)(ny_t - 1) * ld_t + nx_t) * es;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + ((size_t)(ny - 1) * ld + nx) * es;
    if (a0 < b1 && b0 < a1) return SFFT_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const int tiles_x = (nx + AX - 1) / AX, tiles_y = (ny + AY - 1) / AY;
  const int ntiles = tiles_x * tiles_y;
  const int grid = ((ntiles + 7) / 8) * 8;   // whole XCD rounds for the remap
  if (mode == SFFT_MODE_F64)
    align_image_kernel<double><<<grid, AX * AY, 0, s>>>(*map, static_cast<const double*>(tmpl), tmpl_mask, ny_t, nx_t,
                                                        ld_t, static_cast<double*>(out), out_mask, ny, nx, ld, tiles_x,
                                                        ntiles);
  else
    align_image_kernel<float><<<grid, AX * AY, 0, s>>>(*map, static_cast<const float*>(tmpl), tmpl_mask, ny_t, nx_t,
                                                       ld_t, static_cast<float*>(out), out_mask, ny, nx, ld, tiles_x,
                                                       ntiles);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EHIP;
}

int sfft_align_psf(const sfft_pixel_map* map, double x0, double y0, void* hip_stream, const double* psf_t,
                   int32_t s_t, double* psf_out, int32_t s) {
  if (check_map(map) != SFFT_OK || psf_t == nullptr || psf_out == nullptr) return SFFT_EINVAL;
  if (s_t < 0 || s_t > PSF_MAXS || s < 0 || s > PSF_MAXS) return SFFT_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  align_psf_kernel<<<1, PSF_THREADS, 0, st>>>(*map, x0, y0, psf_t, s_t, psf_out, s);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EHIP;
}

}  // extern "C"
