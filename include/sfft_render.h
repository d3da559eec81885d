/*
 * sfft_render.h -- C ABI of the GPU renderer of the warm-start training frames.
 *
 * The learned warm start of the subtraction (include/sfft_mlp.h) is trained
 * on the method's own solves of frames shaped like the paper's Roman detector
 * images ("GPU acceleration and performance": 4088 x 4088 frames; "Statement
 * of need": a PSF that varies across the focal plane).  Twenty thousand such
 * pairs cannot be rendered on the host in useful time, so the pixels are
 * drawn here from a catalogue the caller draws: the GPU evaluates every star
 * and draws the pixel noise from Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, SC 2011) with the frame's seed as key and (pixel index, stream) as
 * counter, so the frame is a pure function of the catalogue.
 */
#ifndef SFFT_RENDER_H_
#define SFFT_RENDER_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One frame's catalogue.  Stars are sorted by catalogue tile: tile
 * (tx, ty) = (clamp(floor(x / 32)), clamp(floor(y / 32))) to [0, nt), nt =
 * ceil(n / 32), row-major; tile_start[t] .. tile_start[t + 1] are its stars
 * (nt^2 + 1 entries).  Pointers are DEVICE arrays of nstar entries. */
typedef struct {
  int32_t n;                  /* frame side (pixels) */
  int32_t nstar;
  double beta;                /* Moffat exponent (> 1) */
  double bc[6];               /* science background 5 (b0 + b1 xh + b2 yh + (b3 xh^2 + b4 xh yh + b5 yh^2)/2) */
  uint64_t noise_seed;        /* Philox key */
  const double* xs;           /* star positions (pixel coordinates, may lie up to a few pixels outside) */
  const double* ys;
  const double* flux;         /* e- */
  const double* fw_s;         /* FWHM of the star in the science / template image (pixels) */
  const double* fw_t;
  const double* mask_r;       /* radius of the star's masked disk, <= 0 = none (radii < 20) */
  const int32_t* tile_start;
} sfft_ws_frame;

/* Render one frame on `hip_stream`: science and template images (device
 * double, pitch ld) and the mask (device uint8, pitch ld, 1 = excluded).
 *   model = sum over stars whose 25 x 25 stamp covers the pixel of
 *           flux (1 + r^2/alpha^2)^-beta / (the profile's sum over the stamp),
 *           alpha = FWHM / (2 sqrt(2^(1/beta) - 1)); the science model adds the
 *           background; each image: lam + sqrt(lam) z1 + 8 z2 - 1000 with
 *           lam = model + 1000 e- (the normal limit of Poisson(lam)) and
 *           (z1, z2) the Box-Muller normals of Philox4x32-10 words for counter
 *           (pixel index low, high, stream, 0), stream 0 science, 1 template.
 * norm_scratch: device double[2 nstar]; overflow: device int32, set nonzero if
 * a 96 x 96 neighbourhood held more than 1024 stars (those are then dropped).
 * FP64.  SFFT_EINVAL for NULL pointers, n outside [2, 8192], ld < n or
 * beta <= 1. */
int sfft_render_ws_frame(const sfft_ws_frame* f, void* hip_stream, double* sci, double* tmpl, uint8_t* mask,
                         int64_t ld, double* norm_scratch, int32_t* overflow);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_RENDER_H_ */
