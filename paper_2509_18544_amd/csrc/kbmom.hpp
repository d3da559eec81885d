// The template-background block of the normal matrix without correlations.
//
//   Omega[(a,u), b] = sum_z A_a(z - u) G(z) m_b(z),   A_a = m_a G_R R.
//
// Split G = 1 - (1 - G):
//   * the whole-frame part, with z' = z - u (A_a vanishes within w of the
//     edge, so z' + u stays in the frame) and the binomial expansion of
//     m_b(z' + u) = (xh' + u_x sx)^p_b (yh' + u_y sy)^q_b, is
//       sum_{i<=p_b, j<=q_b} C(p_b,i) C(q_b,j) (u_x sx)^(p_b-i) (u_y sy)^(q_b-j) mu(p_a+i, q_a+j),
//     mu(p, q) = sum_z G_R R xh^p yh^q: FP64 moments of the template over
//     the frame (moments_kernel / moments_reduce_kernel);
//   * the excluded part, sum over the excluded pixels z of A_a(z - u) m_b(z),
//     with m_a(z - u) expanded around z the same way, is
//       sum_{p'<=p_a, q'<=q_a} C(p_a,p') C(q_a,q') (-u_x sx)^(p_a-p') (-u_y sy)^(q_a-q') T(p'+p_b, q'+q_b)(u),
//     T(p, q)(u) = sum_{z excluded} (G_R R)(z - u) xh(z)^p yh(z)^q: one sum
//     per lag u and monomial of degree <= DK + DB over the excluded pixels.
// The transform route thus needs no background planes: their forward
// transforms and their nK nB correlation windows are replaced by these sums,
// whose cost follows the number of excluded pixels.
//
// Kernels (per pair, after the excluded-pixel list of outmask.hpp):
//   kb_pad     : the zero border of G_R R on the frame padded by w (the row
//                pass writes the frame itself, in the input type), so that
//                (G_R R)(z - u) is one load;
//   kb_mask    : T(c)(u) partial sums, one block per (chunk of the excluded
//                pixels, up to 512 lags); the chunks are fixed, so the grid
//                does not depend on the data;
//   kb_reduce  : T = sum of the chunks' partial sums, chunks in order;
//   kb_combine : the two parts above into kbd[(a,u) nB + b] (FP64), which the
//                gather copies into both triangles of Omega.
#pragma once

#include "assemble.hpp"
#include "outmask.hpp"

namespace sfft {

constexpr int KB_CHUNKS = 128;   // excluded-pixel chunks per pair (fixed grid)
constexpr int KB_SUB = 64;       // excluded pixels staged in LDS per step
constexpr int KB_MAX_THREADS = 512;   // threads per block (at most)
constexpr int KB_LPT = 2;              // lags per thread (each staged monomial read feeds both)

struct KbParams {
  int ny, nx, w, L, nk, nb, nkk, nmu;
  int pitch;                      // padded-frame row of the excluded-pixel list (nx + 2w)
  int64_t ld;
  double sx, sy;
  int8_t kpx[MAX_NB], kqy[MAX_NB];
  int8_t bpx[MAX_NB], bqy[MAX_NB];
};

__device__ __forceinline__ double kb_binom(int n, int k) {
  constexpr double tab[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  return tab[n][k];
}

// The border of the padded frame of G_R R (the row pass writes the frame
// itself): rows [0, w) and [ny + w, ny + 2w), and columns [0, w) and
// [nx + w, nx + 2w) of the rows between.
template <typename T>
__global__ __launch_bounds__(256) void kb_pad_kernel(KbParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  T* __restrict__ grp = ws_at<T>(PS, pr, O.kbgrp);
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nrow = (int64_t)2 * P.w * P.pitch;   // whole border rows
  if (e < nrow) {
    const int r = (int)(e / P.pitch), c = (int)(e - (int64_t)r * P.pitch);
    const int py = r < P.w ? r : P.ny + r;
    grp[(int64_t)py * P.pitch + c] = (T)0;
    return;
  }
  const int64_t f = e - nrow;
  if (f >= (int64_t)2 * P.w * P.ny) return;
  const int y = (int)(f / (2 * P.w)), c = (int)(f - (int64_t)y * 2 * P.w);
  const int px = c < P.w ? c : P.nx + c;
  grp[(int64_t)(y + P.w) * P.pitch + px] = (T)0;
}

// part[chunk][c][u] = sum over the chunk's excluded pixels z of (G_R R)(z - u) m_c(z),
// m_c the monomials of degree <= DSUM = DK + DB (graded order).  A thread
// owns KB_LPT lags u (blockDim apart); the pixels of a step and their
// monomials are staged in LDS (the monomials padded to an even count, read as
// pairs), and each monomial read serves all the thread's lags.
template <typename T, int DSUM>
__global__ __launch_bounds__(KB_MAX_THREADS) void kb_mask_kernel(KbParams P, PairSet PS, WsOff O, OmaskOff M) {
  constexpr int NMU = (DSUM + 1) * (DSUM + 2) / 2;
  constexpr int NMP = (NMU + 1) & ~1;
  const int pr = blockIdx.z;
  const T* __restrict__ grp = ws_at<const T>(PS, pr, O.kbgrp);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  const int* __restrict__ list = ws_at<const int>(PS, pr, M.list);
  double* __restrict__ part = ws_at<double>(PS, pr, O.kbpart);
  const int count = mask == nullptr ? 0 : ws_at<const int>(PS, pr, M.offs)[P.ny];
  __shared__ int spo[KB_SUB];
  __shared__ __align__(16) double smo[KB_SUB][NMP];
  const int tid = threadIdx.x;
  const int L2 = P.L * P.L;
  int ui[KB_LPT], uoff[KB_LPT];   // (z - u) = pix(z) - uoff in the padded frame
#pragma unroll
  for (int l = 0; l < KB_LPT; ++l) {
    ui[l] = (blockIdx.y * KB_LPT + l) * blockDim.x + tid;
    const int uu = min(ui[l], L2 - 1);
    uoff[l] = (uu / P.L - P.w) * P.pitch + (uu % P.L - P.w);
  }
  const int per = (count + KB_CHUNKS - 1) / KB_CHUNKS;
  const int k0 = min(count, (int)blockIdx.x * per), k1 = min(count, k0 + per);
  double acc[KB_LPT][NMU];
#pragma unroll
  for (int l = 0; l < KB_LPT; ++l)
#pragma unroll
    for (int c = 0; c < NMU; ++c) acc[l][c] = 0.0;
  for (int kb = k0; kb < k1; kb += KB_SUB) {
    __syncthreads();   // the previous step's pixels have been read
    if (tid < KB_SUB) {
      const int k = kb + tid;
      const int p = k < k1 ? list[k] : list[k0];   // padded-frame offset of the pixel
      const int y = p / P.pitch - P.w;
      const int x = p - (y + P.w) * P.pitch - P.w;
      spo[tid] = p;
      const double xh = (double)x * P.sx - 1.0, yh = (double)y * P.sy - 1.0;
#pragma unroll
      for (int c = 0; c < NMP; ++c) {
        int pc, qc;
        mono_of(c, &pc, &qc);
        smo[tid][c] = c < NMU ? ipow(xh, pc) * ipow(yh, qc) : 0.0;
      }
    }
    __syncthreads();
    // pixels in groups of four: the four loads are issued before their
    // products (the pixels are still summed one after another, in order)
    const int nsub = min(KB_SUB, k1 - kb);
    int j = 0;
    for (; j + 4 <= nsub; j += 4) {
      double v[4][KB_LPT];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int l = 0; l < KB_LPT; ++l) v[t][l] = (double)grp[spo[j + t] - uoff[l]];   // zero on the w-strip, excluded, outside
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < NMU; ++c) {
          const double m = smo[j + t][c];
#pragma unroll
          for (int l = 0; l < KB_LPT; ++l) acc[l][c] = fma(v[t][l], m, acc[l][c]);
        }
    }
    for (; j < nsub; ++j) {
      double v[KB_LPT];
#pragma unroll
      for (int l = 0; l < KB_LPT; ++l) v[l] = (double)grp[spo[j] - uoff[l]];
#pragma unroll
      for (int c = 0; c < NMU; ++c) {
        const double m = smo[j][c];
#pragma unroll
        for (int l = 0; l < KB_LPT; ++l) acc[l][c] = fma(v[l], m, acc[l][c]);
      }
    }
  }
#pragma unroll
  for (int l = 0; l < KB_LPT; ++l)
    if (ui[l] < L2)
#pragma unroll
      for (int c = 0; c < NMU; ++c) part[((int64_t)blockIdx.x * NMU + c) * L2 + ui[l]] = acc[l][c];
}

// T[c][u] = sum over the chunks of part[chunk][c][u], chunks in order
__global__ void kb_reduce_kernel(KbParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ part = ws_at<const double>(PS, pr, O.kbpart);
  double* __restrict__ Tm = ws_at<double>(PS, pr, O.kbT);
  const int L2 = P.L * P.L;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nmu * L2) return;
  double v = 0.0;
  for (int ch = 0; ch < KB_CHUNKS; ++ch) v += part[(int64_t)ch * P.nmu * L2 + i];
  Tm[i] = v;
}

// kbd[(a,u) nB + b] = whole-frame part - excluded part (see the top of the file)
__global__ void kb_combine_kernel(KbParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ amom = ws_at<const double>(PS, pr, O.amom);
  const double* __restrict__ Tm = ws_at<const double>(PS, pr, O.kbT);
  double* __restrict__ kbd = ws_at<double>(PS, pr, O.kbd);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.nkk * P.nb) return;
  const int i = e / P.nb, b = e - i * P.nb;
  const int L2 = P.L * P.L;
  const int a = i / L2, u = i - a * L2;
  const int uy = u / P.L - P.w, ux = u % P.L - P.w;
  const double dx = (double)ux * P.sx, dy = (double)uy * P.sy;
  const int pa = P.kpx[a], qa = P.kqy[a], pb = P.bpx[b], qb = P.bqy[b];
  double whole = 0.0;
  for (int ii = 0; ii <= pb; ++ii)
    for (int jj = 0; jj <= qb; ++jj)
      whole += kb_binom(pb, ii) * kb_binom(qb, jj) * ipow(dx, pb - ii) * ipow(dy, qb - jj) *
               amom[mono_index(pa + ii, qa + jj)];
  double excl = 0.0;
  for (int pp = 0; pp <= pa; ++pp)
    for (int qq = 0; qq <= qa; ++qq)
      excl += kb_binom(pa, pp) * kb_binom(qa, qq) * ipow(-dx, pa - pp) * ipow(-dy, qa - qq) *
              Tm[(int64_t)mono_index(pp + pb, qq + qb) * L2 + u];
  kbd[e] = whole - excl;
}

}  // namespace sfft
