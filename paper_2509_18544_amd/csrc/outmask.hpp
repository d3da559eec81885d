// Output-masked fit: the least squares restricted to the good output pixels.
//
// The default fit zero-fills excluded pixels, so that every normal-matrix
// entry is a correlation.  Restricting the sum to the good output pixels
// instead gives Omega = Phi^T diag(G) Phi = Omega_zf - Phi_M^T Phi_M, with
// Phi_M the design-matrix rows at the excluded pixels z.  Those rows vanish
// in the background columns (G m_b = 0 at z) and in the target (S_m = G S =
// 0 at z), so the correction touches the kernel block alone and beta is
// unchanged:
//   Omega[(a,u),(b,v)] -= sum_{z excluded} A_a(z - u) A_b(z - v).
// That is a symmetric rank-|M| update of an (L^2 nK)^2 block: a dense
// contraction over the excluded pixels, run on the FP64 matrix cores.
//
// Data flow (one pair, after the zero-filled Omega is assembled):
//   om_planes : A_a = m_a G_R R in FP64 on frames padded by w zeros on every
//               side, so that A_a(z - u) is one load without bounds checks;
//   (counts)  : excluded pixels per image row, from the build's moments pass
//               (nx minus the row's sum of G);
//   om_scan   : row offsets (exclusive prefix), total at offs[ny];
//   om_list   : padded-frame offsets of the excluded pixels, row-major order;
//   om_syrk   : one block per 64 x 64 tile of the lower triangle of the
//               kernel block: chunks of 64 excluded pixels are gathered into
//               LDS (row (a,u) of pixel z: A_a(z - u)) and multiplied on
//               v_mfma_f64_16x16x4f64; the tile and its transpose are then
//               subtracted from Omega.  The pixel sum runs in a fixed order,
//               so results are reproducible bit for bit.
#pragma once

#include "cholesky.hpp"
#include "common.hpp"

namespace sfft {

constexpr int OM_KC = 64;   // excluded pixels per chunk of the contraction

struct OmaskParams {
  int ny, nx, w, nk, L, nkk, n;   // n: row pitch of Omega
  int pitch;                      // nx + 2w: row of a padded plane
  int64_t plane;                  // (ny + 2w) * pitch
  int64_t ld;                     // input row pitch (elements)
  double sx, sy;                  // 2/(nx-1), 2/(ny-1)
  int8_t px[MAX_NB], qy[MAX_NB];  // kernel monomials m_a = xh^px yh^qy
  int ntile;                      // ceil(nkk / 64)
};

// Workspace offsets of the output-mask buffers (the same for every pair of a group).
struct OmaskOff {
  size_t planes, cnt, offs, list, omega;
};

template <typename T>
__global__ __launch_bounds__(256) void om_planes_kernel(OmaskParams P, PairSet PS, OmaskOff O) {
  const int pr = blockIdx.z;
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  double* __restrict__ Ap = ws_at<double>(PS, pr, O.planes) + (int64_t)blockIdx.y * P.plane;
  const int a = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= P.plane) return;
  const int py = (int)(e / P.pitch), px = (int)(e - (int64_t)py * P.pitch);
  const int y = py - P.w, x = px - P.w;
  // the template side of the fit: m_a G_R R (zero on the w-strip, at excluded pixels and outside)
  const bool in = y >= P.w && y < P.ny - P.w && x >= P.w && x < P.nx - P.w;
  double v = 0.0;
  if (in && (mask == nullptr || mask[(int64_t)y * P.ld + x] == 0)) {
    const double xh = (double)x * P.sx - 1.0, yh = (double)y * P.sy - 1.0;
    v = ipow(xh, P.px[a]) * ipow(yh, P.qy[a]) * (double)tmpl[(int64_t)y * P.ld + x];
  }
  Ap[e] = v;
}

// exclusive prefix of the row counts: offs[y], and the total at offs[ny]
__global__ __launch_bounds__(1024) void om_scan_kernel(OmaskParams P, PairSet PS, OmaskOff O) {
  const int pr = blockIdx.z;
  const int* __restrict__ cnt = ws_at<const int>(PS, pr, O.cnt);
  int* __restrict__ offs = ws_at<int>(PS, pr, O.offs);
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int per = (P.ny + 1023) / 1024;
  const int y0 = min(tid * per, P.ny), y1 = min(y0 + per, P.ny);
  int s = 0;
  for (int y = y0; y < y1; ++y) s += cnt[y];
  part[tid] = s;
  __syncthreads();
  // inclusive scan of the 1024 partial sums (Hillis-Steele)
  for (int d = 1; d < 1024; d <<= 1) {
    const int v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = tid > 0 ? part[tid - 1] : 0;
  for (int y = y0; y < y1; ++y) {
    offs[y] = run;
    run += cnt[y];
  }
  if (tid == 1023) offs[P.ny] = part[1023];
}

// padded-frame offsets (y + w) * pitch + (x + w) of the excluded pixels of row y, x ascending.
// A thread takes OM_LPT consecutive pixels of a chunk of 256 OM_LPT (one
// chunk per row up to 4096 columns): its mask bytes are loaded together, its
// excluded pixels counted, and a prefix of the counts over the block (lanes by
// shuffles, then the four waves) places them.
constexpr int OM_LPT = 16;
__global__ __launch_bounds__(256) void om_list_kernel(OmaskParams P, PairSet PS, OmaskOff O) {
  const int pr = blockIdx.z;
  const uint8_t* __restrict__ mask = PS.mask[pr];
  if (mask == nullptr) return;
  const int* __restrict__ offs = ws_at<const int>(PS, pr, O.offs);
  int* __restrict__ list = ws_at<int>(PS, pr, O.list);
  __shared__ int wsum[4];
  const int y = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint8_t* __restrict__ row = mask + (int64_t)y * P.ld;
  int base = offs[y];
  for (int x0 = 0; x0 < P.nx; x0 += 256 * OM_LPT) {
    const int xs = x0 + tid * OM_LPT;
    uint8_t v[OM_LPT];
#pragma unroll
    for (int i = 0; i < OM_LPT; ++i) v[i] = row[min(xs + i, P.nx - 1)];   // clamped, then selected
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < OM_LPT; ++i) bits |= (xs + i < P.nx && v[i] != 0) ? (1u << i) : 0u;
    const int cnt = __popc(bits);
    int inc = cnt;   // inclusive prefix over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(inc, d);
      if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    int at = base + before + inc - cnt;
    const int o = (y + P.w) * P.pitch + xs + P.w;
    while (bits != 0) {
      const int i = __ffs(bits) - 1;
      bits &= bits - 1;
      list[at++] = o + i;
    }
    base += tot;
    __syncthreads();   // wsum is rewritten by the next chunk
  }
}

// Omega_KK -= Phi_M^T Phi_M, one 64 x 64 tile of the lower triangle per block.
__global__ __launch_bounds__(256) void om_syrk_kernel(OmaskParams P, PairSet PS, OmaskOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ Ap = ws_at<const double>(PS, pr, O.planes);
  const int* __restrict__ list = ws_at<const int>(PS, pr, O.list);
  const int count = ws_at<const int>(PS, pr, O.offs)[P.ny];
  double* __restrict__ omega = ws_at<double>(PS, pr, O.omega);
  if (count == 0) return;
  __shared__ double A[NB][NB + 1], B[NB][NB + 1];
  __shared__ int pix[2][OM_KC];
  // tile (ti, tj), ti >= tj, from the block index t = ti (ti + 1) / 2 + tj
  const int t = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int tid = threadIdx.x, r = tid & 63, kq = tid >> 6;
  const int L2 = P.L * P.L;
  // the gather offset of row (a, u): A_a(z - u) = Ap[a * plane - u_y * pitch - u_x + pix(z)]
  auto row_off = [&](int i, bool* ok) -> int64_t {
    *ok = i < P.nkk;
    const int ii = min(i, P.nkk - 1);
    const int a = ii / L2, rem = ii - a * L2;
    const int uy = rem / P.L - P.w, ux = rem % P.L - P.w;
    return (int64_t)a * P.plane - (int64_t)uy * P.pitch - ux;
  };
  bool okA, okB;
  const int64_t offA = row_off(ti * NB + r, &okA);
  const int64_t offB = row_off(tj * NB + r, &okB);
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
  // Chunk c's gathers are issued while the matrix cores work on chunk c - 1
  // (registers va, vb), and the pixel list is staged two chunks ahead in a
  // double buffer, so the scattered loads overlap the products.
  const int nch = (count + OM_KC - 1) / OM_KC;
  double va[OM_KC / 4], vb[OM_KC / 4];
  auto stage_pix = [&](int c, int* dst) {
    if (tid < OM_KC) {
      const int k = c * OM_KC + tid;
      dst[tid] = k < count ? list[k] : -1;
    }
  };
  auto gather = [&](const int* px) {
    // every load is issued before any is used (clamped to pixel 0 of the chunk)
#pragma unroll
    for (int m = 0; m < OM_KC / 4; ++m) {
      const int p = px[kq + 4 * m];
      const int64_t q = p >= 0 ? p : px[0];
      va[m] = Ap[offA + q];
      vb[m] = Ap[offB + q];
    }
  };
  stage_pix(0, pix[0]);
  if (nch > 1) stage_pix(1, pix[1]);
  __syncthreads();
  gather(pix[0]);
  for (int c = 0; c < nch; ++c) {
    const int* px = pix[c & 1];
    __syncthreads();   // the previous chunk's tiles have been read; pix[(c + 1) & 1] is staged
#pragma unroll
    for (int m = 0; m < OM_KC / 4; ++m) {
      const int k = kq + 4 * m;
      const bool live = px[k] >= 0;
      A[r][k] = (live && okA) ? va[m] : 0.0;
      B[r][k] = (live && okB) ? vb[m] : 0.0;
    }
    __syncthreads();
    // chunk c + 2's list entry is loaded before the gathers and stored after
    // the products, so that waiting for it does not wait for them
    const bool stage = tid < OM_KC && c + 2 < nch;
    int pnext = -1;
    if (stage) {
      const int k = (c + 2) * OM_KC + tid;
      pnext = k < count ? list[k] : -1;
    }
    if (c + 1 < nch) gather(pix[(c + 1) & 1]);
#pragma unroll 4
    for (int m0 = 0; m0 < OM_KC; m0 += 4) {
      const int kk = m0 + lk;
      const double a0 = A[wm + lr][kk], a1 = A[wm + 16 + lr][kk];
      const double b0 = B[wn + lr][kk], b1 = B[wn + 16 + lr][kk];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (stage) pix[c & 1][tid] = pnext;   // chunk c's list is no longer read
  }
  // Omega[i][j] -= acc and, off the diagonal tiles, Omega[j][i] likewise
  // (a diagonal tile holds both triangles itself): every entry once
  const int i0 = ti * NB, j0 = tj * NB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int i = i0 + wm + 16 * a + lk + 4 * rr, j = j0 + wn + 16 * c + lr;
        if (i < P.nkk && j < P.nkk) {
          omega[(int64_t)i * P.n + j] -= acc[a][c][rr];
          if (ti != tj) omega[(int64_t)j * P.n + i] -= acc[a][c][rr];
        }
      }
}

}  // namespace sfft
