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
// evaluated at the (2t+1)^2 central taps.  FP64 throughout; two launches
// (frequencies, then taps), each spread over the whole device.
#pragma once

#include "common.hpp"

namespace sfft {

constexpr int DEC_ND = 64;            // DFT grid side
constexpr int DEC_MAXS = 15;          // stamps up to 31 x 31
constexpr int DEC_MAXL = 2 * DEC_MAXS + 1;

struct DecParams {
  int w, nk;            // matching kernel half-width and number of monomials
  int s, t;             // PSF stamp and output half-widths
  double sx, sy;        // 2/(nx-1), 2/(ny-1)
  double var_s, var_r;  // sigma_s^2, sigma_r^2
  int8_t kpx[15], kqy[15];
};

// Pass 1, frequencies: block b takes DEC_FPB grid frequencies, DEC_TPF
// lanes per frequency (each sums a stride of the stamp taps, then a shuffle
// reduction); every block forms K_c and stages the stamps in LDS.
constexpr int DEC_SPEC_THREADS = 256;
constexpr int DEC_TPF = 16;                                   // lanes per frequency
constexpr int DEC_FPB = DEC_SPEC_THREADS / DEC_TPF;           // frequencies per block
constexpr int DEC_SPEC_BLOCKS = DEC_ND * DEC_ND / DEC_FPB;
constexpr int DEC_INV_THREADS = 256;

__global__ __launch_bounds__(DEC_SPEC_THREADS) void decorr_spec_kernel(DecParams Q, const double* __restrict__ theta,
                                                                       const double* __restrict__ psf_sci,
                                                                       const double* __restrict__ psf_tmpl,
                                                                       const cplx<double>* __restrict__ tw,
                                                                       double* __restrict__ spec) {
  __shared__ double kc[DEC_MAXL * DEC_MAXL];
  __shared__ double ps[DEC_MAXL * DEC_MAXL];
  __shared__ double pr[DEC_MAXL * DEC_MAXL];
  __shared__ cplx<double> e64[DEC_ND];            // e^{-2 pi i m / DEC_ND}
  const int tid = threadIdx.x;
  const int L = 2 * Q.w + 1, L2 = L * L;
  const int LS = 2 * Q.s + 1, LS2 = LS * LS;
  // the matching kernel at the frame centre, the stamps and the grid twiddles
  for (int e = tid; e < L2; e += DEC_SPEC_THREADS) {
    const int ux = e % L - Q.w, uy = e / L - Q.w;
    double v = 0.0;
    for (int a = 0; a < Q.nk; ++a) v += theta[a * L2 + e] * ipow(-ux * Q.sx, Q.kpx[a]) * ipow(-uy * Q.sy, Q.kqy[a]);
    kc[e] = v;
  }
  for (int e = tid; e < LS2; e += DEC_SPEC_THREADS) {
    ps[e] = psf_sci[e];
    pr[e] = psf_tmpl[e];
  }
  if (tid < DEC_ND) e64[tid] = tw[tid * (TW_N / DEC_ND)];
  __syncthreads();
  const int f = blockIdx.x * DEC_FPB + tid / DEC_TPF, sub = tid % DEC_TPF;
  const int fy = f / DEC_ND, fx = f % DEC_ND;
  cplx<double> a = mk(0.0, 0.0), b = mk(0.0, 0.0), k = mk(0.0, 0.0);
  for (int e = sub; e < LS2; e += DEC_TPF) {
    const int ux = e % LS - Q.s, uy = e / LS - Q.s;
    const cplx<double> t = e64[(fy * uy + fx * ux) & (DEC_ND - 1)];
    a = a + scale(t, pr[e]);
    b = b + scale(t, ps[e]);
  }
  for (int e = sub; e < L2; e += DEC_TPF) {
    const int ux = e % L - Q.w, uy = e / L - Q.w;
    k = k + scale(e64[(fy * uy + fx * ux) & (DEC_ND - 1)], kc[e]);
  }
  for (int off = DEC_TPF / 2; off > 0; off >>= 1) {
    a.x += __shfl_down(a.x, off, DEC_TPF);
    a.y += __shfl_down(a.y, off, DEC_TPF);
    b.x += __shfl_down(b.x, off, DEC_TPF);
    b.y += __shfl_down(b.y, off, DEC_TPF);
    k.x += __shfl_down(k.x, off, DEC_TPF);
    k.y += __shfl_down(k.y, off, DEC_TPF);
  }
  if (sub == 0) {
    const double na = a.x * a.x + a.y * a.y, nb = b.x * b.x + b.y * b.y, nk = k.x * k.x + k.y * k.y;
    spec[f] = sqrt((Q.var_s + Q.var_r) / (Q.var_s * na + Q.var_r * nk * nb));
  }
}

// Pass 2, taps: block e forms psi(u) = (1/ND^2) sum_f Psi^(f) cos(2 pi (fy uy + fx ux) / ND)
// for one of the (2t+1)^2 central taps.
__global__ __launch_bounds__(DEC_INV_THREADS) void decorr_inv_kernel(DecParams Q, const double* __restrict__ spec,
                                                                     const cplx<double>* __restrict__ tw,
                                                                     double* __restrict__ psi) {
  __shared__ double cs[DEC_ND];                  // cos(2 pi m / DEC_ND)
  __shared__ double part[DEC_INV_THREADS / 64];
  const int tid = threadIdx.x;
  if (tid < DEC_ND) cs[tid] = tw[tid * (TW_N / DEC_ND)].x;
  __syncthreads();
  const int LT = 2 * Q.t + 1;
  const int e = blockIdx.x;
  const int ux = e % LT - Q.t, uy = e / LT - Q.t;
  double acc = 0.0;
  for (int f = tid; f < DEC_ND * DEC_ND; f += DEC_INV_THREADS) {
    const int fy = f / DEC_ND, fx = f % DEC_ND;
    acc += spec[f] * cs[(fy * uy + fx * ux) & (DEC_ND - 1)];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((tid & 63) == 0) part[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < DEC_INV_THREADS / 64; ++q) t += part[q];
    psi[e] = t / (double)(DEC_ND * DEC_ND);
  }
}

}  // namespace sfft
