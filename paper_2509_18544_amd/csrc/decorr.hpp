// Decorrelation kernel of the difference image (pipeline step 7 of the
// paper's "Pipeline steps": fit the decorrelation kernel and apply it to the
// difference image, the science PSF and the cross-convolved science image).
//
// The paper gives no formula; the kernel computed here is the one that
// whitens the difference image's noise when the science and template images
// carry independent white noise (standard deviations sigma_s, sigma_r) and
// were cross-convolved (S' = P_R * S, R' = P_S * R) before the subtraction
// D = S' - K * R' - background:
//   N(f)   = sigma_s^2 |P_R^(f)|^2 + sigma_r^2 |K_c^(f)|^2 |P_S^(f)|^2,
//   Psi^(f) = sqrt((sigma_s^2 + sigma_r^2) / N(f)),
// with K_c the matching kernel at the frame centre (xh = yh = 0),
//   K_c(u) = sum_a k_{a,u} (-u_x sx)^p_a (-u_y sy)^q_a,
// and every spectrum the DFT on a DEC_ND x DEC_ND grid of the stamp placed
// with its centre tap at index (0, 0).  Psi^ is real and even (N is even), so
// the kernel is psi(u) = (1 / DEC_ND^2) sum_f Psi^(f) cos(2 pi f.u / DEC_ND),
// evaluated at the (2t+1)^2 central taps.  FP64 throughout; one block.
#pragma once

#include "common.hpp"

namespace sfft {

constexpr int DEC_ND = 64;            // DFT grid side
constexpr int DEC_THREADS = 1024;
constexpr int DEC_MAXS = 15;          // stamps up to 31 x 31
constexpr int DEC_MAXL = 2 * DEC_MAXS + 1;

struct DecParams {
  int w, nk;            // matching kernel half-width and number of monomials
  int s, t;             // PSF stamp and output half-widths
  double sx, sy;        // 2/(nx-1), 2/(ny-1)
  double var_s, var_r;  // sigma_s^2, sigma_r^2
  int8_t kpx[15], kqy[15];
};

__global__ __launch_bounds__(DEC_THREADS) void decorr_kernel(DecParams Q, const double* __restrict__ theta,
                                                             const double* __restrict__ psf_sci,
                                                             const double* __restrict__ psf_tmpl,
                                                             const cplx<double>* __restrict__ tw,
                                                             double* __restrict__ psi) {
  __shared__ double kc[DEC_MAXL * DEC_MAXL];
  __shared__ double ps[DEC_MAXL * DEC_MAXL];
  __shared__ double pr[DEC_MAXL * DEC_MAXL];
  __shared__ cplx<double> e64[DEC_ND];            // e^{-2 pi i m / DEC_ND}
  __shared__ double spec[DEC_ND * DEC_ND];        // Psi^ on the grid
  const int tid = threadIdx.x;
  const int L = 2 * Q.w + 1, L2 = L * L;
  const int LS = 2 * Q.s + 1, LS2 = LS * LS;
  // the matching kernel at the frame centre, the stamps and the grid twiddles
  for (int e = tid; e < L2; e += DEC_THREADS) {
    const int ux = e % L - Q.w, uy = e / L - Q.w;
    double v = 0.0;
    for (int a = 0; a < Q.nk; ++a) v += theta[a * L2 + e] * ipow(-ux * Q.sx, Q.kpx[a]) * ipow(-uy * Q.sy, Q.kqy[a]);
    kc[e] = v;
  }
  for (int e = tid; e < LS2; e += DEC_THREADS) {
    ps[e] = psf_sci[e];
    pr[e] = psf_tmpl[e];
  }
  if (tid < DEC_ND) e64[tid] = tw[tid * (TW_N / DEC_ND)];
  __syncthreads();
  // spectra and Psi^ at the grid frequencies (fy, fx), four per thread
  for (int f = tid; f < DEC_ND * DEC_ND; f += DEC_THREADS) {
    const int fy = f / DEC_ND, fx = f % DEC_ND;
    cplx<double> a = mk(0.0, 0.0), b = mk(0.0, 0.0), k = mk(0.0, 0.0);
    for (int e = 0; e < LS2; ++e) {
      const int ux = e % LS - Q.s, uy = e / LS - Q.s;
      const cplx<double> t = e64[(fy * uy + fx * ux) & (DEC_ND - 1)];
      a = a + scale(t, pr[e]);
      b = b + scale(t, ps[e]);
    }
    for (int e = 0; e < L2; ++e) {
      const int ux = e % L - Q.w, uy = e / L - Q.w;
      k = k + scale(e64[(fy * uy + fx * ux) & (DEC_ND - 1)], kc[e]);
    }
    const double na = a.x * a.x + a.y * a.y, nb = b.x * b.x + b.y * b.y, nk = k.x * k.x + k.y * k.y;
    spec[f] = sqrt((Q.var_s + Q.var_r) / (Q.var_s * na + Q.var_r * nk * nb));
  }
  __syncthreads();
  // psi(u) = (1/ND^2) sum_f Psi^(f) cos(2 pi (fy uy + fx ux) / ND) at |u| <= t
  const int LT = 2 * Q.t + 1;
  for (int e = tid; e < LT * LT; e += DEC_THREADS) {
    const int ux = e % LT - Q.t, uy = e / LT - Q.t;
    double acc = 0.0;
    for (int f = 0; f < DEC_ND * DEC_ND; ++f) {
      const int fy = f / DEC_ND, fx = f % DEC_ND;
      acc += spec[f] * e64[(fy * uy + fx * ux) & (DEC_ND - 1)].x;
    }
    psi[e] = acc / (double)(DEC_ND * DEC_ND);
  }
}

}  // namespace sfft
