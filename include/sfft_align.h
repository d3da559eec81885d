/*
 * sfft_align.h -- C ABI of the alignment of the template to the science frame.
 *
 * Pipeline step 4 of the phrosty paper ("Pipeline steps") aligns the
 * reference image, its PSF and its detection mask to the science image before
 * cross-convolution (step 5) and subtraction (step 6); the paper singles out
 * alignment and resampling as the code its authors worked hardest to speed up
 * ("GPU acceleration and performance") but prints neither the coordinate
 * model nor the interpolation.  This library fixes them as follows.
 *
 * Geometry: a polynomial map from science to template pixel coordinates
 * (x fastest, pixel centres at integers), u = x - x_ref, v = y - y_ref,
 *   x_t = sum_j cx[j] u^p_j v^q_j,   y_t = sum_j cy[j] u^p_j v^q_j,
 * monomials graded by d = p + q then q ascending (1; u, v; u^2, u v, v^2;
 * u^3, u^2 v, u v^2, v^3), degree 0..3 -- an affine first-order WCS, or one
 * with a SIP-style distortion.
 *
 * Interpolation: Lanczos-3, L(t) = sinc(t) sinc(t/3) on |t| < 3 (sinc(t) =
 * sin(pi t)/(pi t), L(0) = 1), over the 6 x 6 taps i = floor(x_t)-2 ..
 * floor(x_t)+3 (likewise j), with the weights normalised to unit sum in each
 * direction (constants are kept exactly; integer offsets copy exactly).
 *
 * Conventions: device pointers owned by the caller, row-major with pitch
 * ld (elements); work is enqueued on `hip_stream` (NULL = default stream);
 * arguments are checked before anything is enqueued (SFFT_EINVAL); inputs are
 * never modified.  Arithmetic is FP64 in both modes.
 */
#ifndef SFFT_ALIGN_H_
#define SFFT_ALIGN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t deg;            /* polynomial degree of the map, 0..3 */
  double x_ref, y_ref;    /* u = x - x_ref, v = y - y_ref (science pixels) */
  double cx[10], cy[10];  /* coefficients of the (deg+1)(deg+2)/2 monomials; the rest ignored */
} sfft_pixel_map;

/* Resample the template image (and mask) onto the science grid.
 *   tmpl: ny_t x nx_t, pitch ld_t, double (SFFT_MODE_F64) or float
 *         (SFFT_MODE_F32C); tmpl_mask: uint8 of the same pitch, nonzero =
 *         masked, or NULL (no mask);
 *   out: ny x nx, pitch ld, same type as tmpl; out_mask: uint8, pitch ld.
 * An output pixel whose 36 taps all lie in the template is the normalised
 * Lanczos-3 sum; out_mask is 1 if any of its 36 tap pixels is masked, else
 * 0.  A pixel with a tap outside the template (or a non-finite coordinate)
 * gets out = 0 and out_mask = 1.  SFFT_EINVAL: NULL image pointers, deg
 * outside 0..3, sizes < 1 or > 65536, ld_t < nx_t, ld < nx, an unknown mode,
 * or out overlapping tmpl. */
int sfft_align_image(const sfft_pixel_map* map, int32_t mode, void* hip_stream, const void* tmpl,
                     const uint8_t* tmpl_mask, int32_t ny_t, int32_t nx_t, int64_t ld_t, void* out,
                     uint8_t* out_mask, int32_t ny, int32_t nx, int64_t ld);

/* Align the template PSF stamp (side 2 s_t + 1, centre tap at index s_t,
 * zero outside the stamp; device double) to the science frame at the science
 * point (x0, y0): out (side 2 s + 1, device double) samples it by Lanczos-3 at
 * the template offsets J (u, v), J the map's Jacobian at (x0, y0), scaled so
 * that its sum equals the template stamp's.  One block.  SFFT_EINVAL: NULL
 * pointers, deg outside 0..3, s_t or s outside 0..31. */
int sfft_align_psf(const sfft_pixel_map* map, double x0, double y0, void* hip_stream, const double* psf_t,
                   int32_t s_t, double* psf_out, int32_t s);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_ALIGN_H_ */
