// Difference image D = S - sum_{a,u} k_{a,u} T_u(m_a R) - sum_b c_b m_b.
//
// The polynomial weight acts on template pixels before the shift.  Writing
// m_a at the source pixel z - u as a polynomial in the output pixel z,
//   xh(x - u_x) = xh(x) - 2 u_x/(nx-1),   yh(y - u_y) = yh(y) - 2 u_y/(ny-1),
//   m_(p,q)(z - u) = sum_{i<=p, j<=q} C(p,i) C(q,j) (-dx)^(p-i) (-dy)^(q-j) m_(i,j)(z),
// gives model(z) = sum_a' m_a'(z) sum_u k'_{a',u} R(z - u) with
// k'_{a',u} = sum_a k_{a,u} e_{a,a'}(u): nK plain convolutions of the same
// unmasked template, combined with the output-side monomials.  Pixels outside
// the frame contribute zero (linear convolution, no wrap-around).
//
// kprime_kernel : k' from theta (FP64).
// subtract_kernel: LDS-tiled direct convolution (16 x 64 output tile per block,
//                  4 pixels x nK accumulators per thread, FP64 accumulation).
#pragma once

#include "common.hpp"

namespace sfft {

struct SubParams {
  int ny, nx, w, nk, nb;
  int64_t ld;
  int8_t kpx[15], kqy[15];
  int8_t bpx[15], bqy[15];
};

__device__ __forceinline__ double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return r;
}

__global__ void kprime_kernel(SubParams P, const double* __restrict__ theta, double* __restrict__ kp) {
  const int L = 2 * P.w + 1;
  const int L2 = L * L;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= L2) return;
  const int uy = u / L - P.w, ux = u % L - P.w;
  const double dx = 2.0 * (double)ux / (double)(P.nx - 1);
  const double dy = 2.0 * (double)uy / (double)(P.ny - 1);
  for (int ap = 0; ap < P.nk; ++ap) {
    const int i = P.kpx[ap], j = P.kqy[ap];
    double s = 0.0;
    for (int a = 0; a < P.nk; ++a) {
      const int p = P.kpx[a], q = P.kqy[a];
      if (i > p || j > q) continue;
      double e = binom(p, i) * binom(q, j);
      for (int t = 0; t < p - i; ++t) e *= -dx;
      for (int t = 0; t < q - j; ++t) e *= -dy;
      s += theta[a * L2 + u] * e;
    }
    kp[ap * L2 + u] = s;
  }
}

constexpr int SUB_TY = 16;
constexpr int SUB_TX = 64;

// Dynamic LDS: tile (SUB_TY + 2w) x (SUB_TX + 2w) doubles, then nK * L^2 doubles of k'.
template <typename T, int NK>
__global__ __launch_bounds__(256) void subtract_kernel(SubParams P, const T* __restrict__ sci,
                                                       const T* __restrict__ tmpl, const double* __restrict__ kp,
                                                       const double* __restrict__ theta, T* __restrict__ diff) {
  extern __shared__ double sm[];
  const int w = P.w;
  const int L = 2 * w + 1;
  const int L2 = L * L;
  const int TW = SUB_TX + 2 * w;
  const int TH = SUB_TY + 2 * w;
  double* tile = sm;
  double* kps = sm + TW * TH;
  const int y0 = blockIdx.y * SUB_TY;
  const int x0 = blockIdx.x * SUB_TX;
  const int tid = threadIdx.x;
  for (int e = tid; e < TW * TH; e += 256) {
    const int r = e / TW, c = e % TW;
    const int y = y0 - w + r, x = x0 - w + c;
    tile[e] = (y >= 0 && y < P.ny && x >= 0 && x < P.nx) ? (double)tmpl[(int64_t)y * P.ld + x] : 0.0;
  }
  for (int e = tid; e < NK * L2; e += 256) kps[e] = kp[e];
  __syncthreads();
  const int ty = tid >> 4;          // 0..15
  const int tx = (tid & 15) * 4;    // 0..60
  double acc[NK][4];
#pragma unroll
  for (int a = 0; a < NK; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[a][i] = 0.0;
  for (int uy = -w; uy <= w; ++uy) {
    const double* trow = tile + (ty - uy + w) * TW + tx + w;
    const double* krow = kps + (uy + w) * L + w;
    for (int ux = -w; ux <= w; ++ux) {
      double rv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) rv[i] = trow[i - ux];
#pragma unroll
      for (int a = 0; a < NK; ++a) {
        const double k = krow[a * L2 + ux];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[a][i] += k * rv[i];
      }
    }
  }
  const int y = y0 + ty;
  if (y >= P.ny) return;
  const double yh = 2.0 * (double)y / (double)(P.ny - 1) - 1.0;
  const int nkk = NK * L2;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int x = x0 + tx + i;
    if (x >= P.nx) continue;
    const double xh = 2.0 * (double)x / (double)(P.nx - 1) - 1.0;
    double model = 0.0;
#pragma unroll
    for (int a = 0; a < NK; ++a) {
      double m = 1.0;
      for (int t = 0; t < P.kpx[a]; ++t) m *= xh;
      for (int t = 0; t < P.kqy[a]; ++t) m *= yh;
      model += m * acc[a][i];
    }
    for (int b = 0; b < P.nb; ++b) {
      double m = 1.0;
      for (int t = 0; t < P.bpx[b]; ++t) m *= xh;
      for (int t = 0; t < P.bqy[b]; ++t) m *= yh;
      model += theta[nkk + b] * m;
    }
    const int64_t o = (int64_t)y * P.ld + x;
    diff[o] = (T)((double)sci[o] - model);
  }
}

}  // namespace sfft
