// GPU renderer of the warm-start training frames (include/sfft_render.h).
//
// The learned warm start is trained on solves of frames shaped like Roman
// detector images (4088 x 4088, ~40 000 Moffat stars whose width varies over
// the focal plane, sky, read noise, a quadratic background, bright-star
// masks).  Rendering 20 000 such pairs on the host would take over ten
// core-hours, so the frames are drawn here from a catalogue drawn on the host
// (positions, fluxes, widths: all the random numbers except the pixel noise).
// The pixel noise comes from Philox4x32-10 (Salmon et al., SC 2011) keyed by
// the frame's noise seed, with the pixel index as the counter, so that every
// pixel's noise is a pure function of (seed, stream, pixel) and a host
// implementation of the same generator reproduces the frame.
//
// Per image: model(y, x) = sum over stars with |x - cx|, |y - cy| <= H of
// flux (1 + r^2/alpha^2)^-beta / norm, cx = floor(x_star + 1/2), r the
// distance from the star to the pixel centre, norm the profile's sum over the
// star's (2H+1)^2 stamp; the science image adds the background
// 5 (b0 + b1 xh + b2 yh + (b3 xh^2 + b4 xh yh + b5 yh^2)/2); the noise is the
// normal limit of Poisson(lam), lam = model + sky (sky = 1000 e-, so lam is
// large): value = lam + sqrt(lam) z1 + 8 z2 - sky.  The mask marks the disks
// of radius mask_r around the stars that have one.  FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/sfft.h"
#include "../../include/sfft_render.h"

namespace {

constexpr int RT = 32;            // output tile side (pixels), also the catalogue's tile side
constexpr int RHALF = 12;         // star stamps are (2 RHALF + 1)^2
constexpr int RTHREADS = 256;
constexpr int RMAXS = 1024;       // stars staged per block (a 3 x 3 neighbourhood of tiles)
constexpr double SKY = 1000.0, READ = 8.0;

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += W0;
    k1 += W1;
  }
}

// two standard normals for pixel `idx` of noise stream `stream` (Box-Muller of two
// 53-bit uniforms built from the four output words)
__device__ __forceinline__ void philox_normals(uint64_t idx, uint32_t stream, uint64_t seed, double* z1, double* z2) {
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0u};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = ((double)((((uint64_t)(c[0] >> 11)) << 32) | c[1]) + 0.5) * 0x1p-53;
  const double u2 = ((double)((((uint64_t)(c[2] >> 11)) << 32) | c[3]) + 0.5) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  double s, co;
  sincospi(2.0 * u2, &s, &co);
  *z1 = r * co;
  *z2 = r * s;
}

__device__ __forceinline__ double moffat_alpha(double fwhm, double beta) {
  return fwhm / (2.0 * sqrt(exp2(1.0 / beta) - 1.0));
}

// Profile sums over each star's stamp, one wave per star: norm[2i] template, norm[2i+1] science.
__global__ __launch_bounds__(256) void star_norm_kernel(sfft_ws_frame F, double* __restrict__ norm) {
  const int star = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (star >= F.nstar) return;
  const double x = F.xs[star], y = F.ys[star];
  const double cx = floor(x + 0.5), cy = floor(y + 0.5);
  const double at = moffat_alpha(F.fw_t[star], F.beta), as = moffat_alpha(F.fw_s[star], F.beta);
  const double it2 = 1.0 / (at * at), is2 = 1.0 / (as * as);
  constexpr int L = 2 * RHALF + 1;
  double st = 0.0, ss = 0.0;
  for (int e = lane; e < L * L; e += 64) {
    const double dx = cx + (double)(e % L - RHALF) - x, dy = cy + (double)(e / L - RHALF) - y;
    const double r2 = dx * dx + dy * dy;
    st += pow(1.0 + r2 * it2, -F.beta);
    ss += pow(1.0 + r2 * is2, -F.beta);
  }
  for (int off = 32; off > 0; off >>= 1) {
    st += __shfl_down(st, off, 64);
    ss += __shfl_down(ss, off, 64);
  }
  if (lane == 0) {
    norm[2 * star] = st;
    norm[2 * star + 1] = ss;
  }
}

// One block per RT x RT output tile: the stars of the 3 x 3 neighbourhood of
// catalogue tiles are staged in LDS (in tile order, then catalogue order),
// then every pixel sums the stars whose stamp covers it, in that order.
__global__ __launch_bounds__(RTHREADS) void render_kernel(sfft_ws_frame F, const double* __restrict__ norm,
                                                          double* __restrict__ sci, double* __restrict__ tmpl,
                                                          uint8_t* __restrict__ mask, int64_t ld, int* overflow) {
  __shared__ double sx[RMAXS], sy[RMAXS], ft[RMAXS], fs[RMAXS], it2[RMAXS], is2[RMAXS], mr2[RMAXS];
  __shared__ int base[10];
  const int nt = (F.n + RT - 1) / RT;
  const int tx = blockIdx.x % nt, ty = blockIdx.x / nt;
  const int tid = threadIdx.x;
  // the neighbourhood's tiles in row-major order and their star ranges
  if (tid == 0) {
    int acc = 0;
    for (int k = 0; k < 9; ++k) {
      const int gx = tx + k % 3 - 1, gy = ty + k / 3 - 1;
      base[k] = acc;
      if (gx >= 0 && gx < nt && gy >= 0 && gy < nt) {
        const int t = gy * nt + gx;
        acc += F.tile_start[t + 1] - F.tile_start[t];
      }
    }
    base[9] = acc;
    if (acc > RMAXS) atomicOr(overflow, 1);
  }
  __syncthreads();
  const int ns = min(base[9], RMAXS);
  for (int e = tid; e < ns; e += RTHREADS) {
    int k = 0;
    while (k < 8 && e >= base[k + 1]) ++k;
    const int gx = tx + k % 3 - 1, gy = ty + k / 3 - 1;
    const int i = F.tile_start[gy * nt + gx] + (e - base[k]);
    sx[e] = F.xs[i];
    sy[e] = F.ys[i];
    ft[e] = F.flux[i] / norm[2 * i];
    fs[e] = F.flux[i] / norm[2 * i + 1];
    const double at = moffat_alpha(F.fw_t[i], F.beta), as = moffat_alpha(F.fw_s[i], F.beta);
    it2[e] = 1.0 / (at * at);
    is2[e] = 1.0 / (as * as);
    mr2[e] = F.mask_r[i] > 0.0 ? F.mask_r[i] * F.mask_r[i] : -1.0;
  }
  __syncthreads();
  const double sxh = 2.0 / (double)(F.n - 1);
  for (int p = tid; p < RT * RT; p += RTHREADS) {
    const int x = tx * RT + (p % RT), y = ty * RT + (p / RT);
    if (x >= F.n || y >= F.n) continue;
    double mt = 0.0, ms = 0.0;
    bool masked = false;
    for (int e = 0; e < ns; ++e) {
      const double cx = floor(sx[e] + 0.5), cy = floor(sy[e] + 0.5);
      const double dx = (double)x - sx[e], dy = (double)y - sy[e];
      const double r2 = dx * dx + dy * dy;
      masked |= r2 <= mr2[e];
      if (fabs((double)x - cx) > RHALF || fabs((double)y - cy) > RHALF) continue;
      mt += ft[e] * pow(1.0 + r2 * it2[e], -F.beta);
      ms += fs[e] * pow(1.0 + r2 * is2[e], -F.beta);
    }
    const double xh = (double)x * sxh - 1.0, yh = (double)y * sxh - 1.0;
    ms += 5.0 * (F.bc[0] + F.bc[1] * xh + F.bc[2] * yh +
                 0.5 * (F.bc[3] * xh * xh + F.bc[4] * xh * yh + F.bc[5] * yh * yh));
    const uint64_t idx = (uint64_t)y * (uint64_t)F.n + (uint64_t)x;
    double z1, z2;
    const int64_t o = (int64_t)y * ld + x;
    philox_normals(idx, 0u, F.noise_seed, &z1, &z2);
    double lam = fmax(ms, 0.0) + SKY;
    sci[o] = lam + sqrt(lam) * z1 + READ * z2 - SKY;
    philox_normals(idx, 1u, F.noise_seed, &z1, &z2);
    lam = fmax(mt, 0.0) + SKY;
    tmpl[o] = lam + sqrt(lam) * z1 + READ * z2 - SKY;
    mask[o] = masked ? 1 : 0;
  }
}

}  // namespace

extern "C" {

int sfft_render_ws_frame(const sfft_ws_frame* f, void* hip_stream, double* sci, double* tmpl, uint8_t* mask,
                         int64_t ld, double* norm_scratch, int32_t* overflow) {
  if (f == nullptr || sci == nullptr || tmpl == nullptr || mask == nullptr || norm_scratch == nullptr ||
      overflow == nullptr)
    return SFFT_EINVAL;
  if (f->n < 2 || f->n > 8192 || ld < f->n || f->nstar < 0 || !(f->beta > 1.0)) return SFFT_EINVAL;
  if (f->nstar > 0 && (f->xs == nullptr || f->ys == nullptr || f->flux == nullptr || f->fw_s == nullptr ||
                       f->fw_t == nullptr || f->mask_r == nullptr))
    return SFFT_EINVAL;
  if (f->tile_start == nullptr) return SFFT_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (f->nstar > 0) {
    star_norm_kernel<<<(f->nstar + 3) / 4, 256, 0, s>>>(*f, norm_scratch);
    if (hipGetLastError() != hipSuccess) return SFFT_EHIP;
  }
  const int nt = (f->n + RT - 1) / RT;
  render_kernel<<<nt * nt, RTHREADS, 0, s>>>(*f, norm_scratch, sci, tmpl, mask, ld, overflow);
  if (hipGetLastError() != hipSuccess) return SFFT_EHIP;
  return SFFT_OK;
}

}  // extern "C"
