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
//                  4 pixels x nK accumulators per thread, FP64 accumulation);
//                  used for the border columns that the spectral route below
//                  cannot produce exactly.
#pragma once

#include "common.hpp"

namespace sfft {

struct SubParams {
  int ny, nx, w, nk, nb;
  int xbeg, xend;        // the direct kernel writes columns [xbeg, xend) only
  int xbeg2, xend2;      // narrow-band kernel: a second band (empty when xend2 <= xbeg2)
  int64_t ld;
  int8_t kpx[15], kqy[15];
  int8_t bpx[15], bqy[15];
};

__device__ __forceinline__ double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return r;
}

// one thread per (a', u): the nK x L^2 outputs in parallel
__global__ void kprime_kernel(SubParams P, const double* __restrict__ theta, double* __restrict__ kp) {
  const int L = 2 * P.w + 1;
  const int L2 = L * L;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= P.nk * L2) return;
  const int ap = id / L2;
  const int u = id - ap * L2;
  const int uy = u / L - P.w, ux = u % L - P.w;
  const double dx = 2.0 * (double)ux / (double)(P.nx - 1);
  const double dy = 2.0 * (double)uy / (double)(P.ny - 1);
  {
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

// Direct D on the narrow column bands [P.xbeg, P.xend) and [P.xbeg2, P.xend2):
// one wave per pixel, the lanes split the nK L^2 kernel taps (k' in LDS) and
// sum by shuffles.  The template loads of a lane are unconditional (clamped
// into the frame, then selected) so that several are in flight.  Same
// arithmetic as subtract_kernel below, summed in a different order.
constexpr int BAND_WAVES = 8;
__global__ __launch_bounds__(64 * BAND_WAVES) void subtract_band_kernel(SubParams P, const void* __restrict__ sci_v,
                                                                        const void* __restrict__ tmpl_v, int is_f64,
                                                                        const double* __restrict__ kp,
                                                                        const double* __restrict__ theta,
                                                                        void* __restrict__ diff_v) {
  extern __shared__ double kps[];
  const int w = P.w;
  const int L = 2 * w + 1;
  const int L2 = L * L;
  const int nkk = P.nk * L2;
  const int bw0 = P.xend - P.xbeg;
  const int bw1 = max(0, P.xend2 - P.xbeg2);
  for (int e = threadIdx.x; e < nkk; e += 64 * BAND_WAVES) kps[e] = kp[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  int64_t id = (int64_t)blockIdx.x * BAND_WAVES + (threadIdx.x >> 6);
  int y, x;
  if (id < (int64_t)bw0 * P.ny) {
    y = (int)(id / bw0);
    x = P.xbeg + (int)(id - (int64_t)y * bw0);
  } else {
    id -= (int64_t)bw0 * P.ny;
    if (id >= (int64_t)bw1 * P.ny) return;
    y = (int)(id / bw1);
    x = P.xbeg2 + (int)(id - (int64_t)y * bw1);
  }
  const double yh = 2.0 * (double)y / (double)(P.ny - 1) - 1.0;
  const double xh = 2.0 * (double)x / (double)(P.nx - 1) - 1.0;
  double acc = 0.0;
#pragma unroll 4
  for (int t = lane; t < nkk; t += 64) {
    const int a = t / L2;
    const int r = t - a * L2;
    const int uy = r / L - w;
    const int ux = r - (uy + w) * L - w;
    const int sy = y - uy, sx = x - ux;
    const bool in = sy >= 0 && sy < P.ny && sx >= 0 && sx < P.nx;
    const int64_t o = (int64_t)min(max(sy, 0), P.ny - 1) * P.ld + min(max(sx, 0), P.nx - 1);
    const double tv = is_f64 ? reinterpret_cast<const double*>(tmpl_v)[o]
                             : (double)reinterpret_cast<const float*>(tmpl_v)[o];
    double m = 1.0;
    for (int q = 0; q < P.kpx[a]; ++q) m *= xh;
    for (int q = 0; q < P.kqy[a]; ++q) m *= yh;
    acc += in ? kps[t] * m * tv : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane != 0) return;
  double model = acc;
  for (int b = 0; b < P.nb; ++b) {
    double m = 1.0;
    for (int q = 0; q < P.bpx[b]; ++q) m *= xh;
    for (int q = 0; q < P.bqy[b]; ++q) m *= yh;
    model += theta[nkk + b] * m;
  }
  const int64_t o = (int64_t)y * P.ld + x;
  if (is_f64) {
    reinterpret_cast<double*>(diff_v)[o] = reinterpret_cast<const double*>(sci_v)[o] - model;
  } else {
    reinterpret_cast<float*>(diff_v)[o] = (float)((double)reinterpret_cast<const float*>(sci_v)[o] - model);
  }
}

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
  const int x0 = P.xbeg + blockIdx.x * SUB_TX;
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
    if (x >= P.xend) continue;
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

// ---------------------------------------------------------------------------
// Spectral route for the interior (x-direction by FFT, y-direction direct)
// ---------------------------------------------------------------------------
// With m_a = xh^p yh^q, the kernel term is
//   sum_{u_y} yh(y-u_y)^q [ sum_{u_x} k_a(u_y,u_x) (xh^p R)(y-u_y, x-u_x) ].
// Along x the bracket is a convolution: with U_p(y, kx) the R2C transform of
// the row xh^p R and K_a(u_y, kx) = sum_{u_x} k_a(u_y, u_x) e^{-2 pi i kx u_x/Px},
//   M(y, kx) = sum_a sum_{u_y} K_a(u_y, kx) yh(y-u_y)^q U_p(y-u_y, kx)   (0 <= y-u_y < ny)
// is the row transform of the model; a C2R transform per row gives the model,
// exact wherever the circular x-convolution does not wrap into the frame
// (x >= w - (Px - nx) and x < Px - w); the remaining border columns are
// recomputed by the direct kernel above.  All of it in FP64.
struct SpecParams {
  int ny, nx, w, nk, nb;
  int lgPx, H;           // Px = 2^lgPx, H = Px / 2; spectra rows hold H + 1 values
  int64_t ld;
  int rows_per_block;
  int nrowblk;
  double sx, sy;
  int8_t kpx[15], kqy[15];
  int8_t bpx[15], bqy[15];
};

constexpr int SUB_MAXP = 5;   // x powers of the background polynomial (degree <= 4)

// rows per block of the subtraction's row transforms (a power of two)
__host__ __device__ constexpr int sub_row_rows(int nmax, int lgh) { return (nmax >> lgh) < 64 ? (nmax >> lgh) : 64; }

// R2C of the rows xh^p R (p = 0..DK) -> Uq[p][y][0..H]
template <typename T, int THREADS, int NMAX, int LGH>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 4 : 2) void sub_rowfwd_kernel(SpecParams P, const T* __restrict__ tmpl,
                                                             cplx<double>* __restrict__ Uq,
                                                             const cplx<double>* __restrict__ tw, int npow) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  constexpr int RB = sub_row_rows(NMAX, LGH);
  constexpr int H = 1 << LGH;             // H = Px / 2
  constexpr int NPT = (RB * H) / THREADS;
  static_assert(NPT * THREADS == RB * H, "whole pairs per thread");
  const int y0 = blockIdx.x * RB;
  const int tid = threadIdx.x;
  constexpr int twsx = TW_LOG - (LGH + 1);
  const LdsRows<double, LGH> lds{buf};
  // the thread's pairs of R, read once (clamped into the frame, unconditional)
  T r0[NPT], r1[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int e = tid + i * THREADS;
    const int y = min(y0 + (e >> LGH), P.ny - 1);
    const int x0 = 2 * (e & (H - 1));
    const T* row = tmpl + (int64_t)y * P.ld;
    r0[i] = row[min(x0, P.nx - 1)];
    r1[i] = row[min(x0 + 1, P.nx - 1)];
  }
  for (int p = 0; p < npow; ++p) {
    __syncthreads();
    // the lane index passes through an empty asm so that the per-pair
    // coordinates are recomputed per power instead of held in registers
    int lane = tid;
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = lane + i * THREADS;
      const int y = y0 + (e >> LGH);
      const int x0 = 2 * (e & (H - 1)), x1 = x0 + 1;
      const double xh0 = (double)x0 * P.sx - 1.0, xh1 = (double)x1 * P.sx - 1.0;
      double p0 = 1.0, p1 = 1.0;
      for (int q = 0; q < p; ++q) {
        p0 *= xh0;
        p1 *= xh1;
      }
      const bool in = y < P.ny;
      const double v0 = (in && x0 < P.nx) ? p0 * (double)r0[i] : 0.0;
      const double v1 = (in && x1 < P.nx) ? p1 * (double)r1[i] : 0.0;
      buf[lds_pad(e)] = mk(v0, v1);
    }
    __syncthreads();
    fft_run<double, NMAX, THREADS, false, true, true, LGH, 4>(buf, RB, tw, lds, lds);
    __syncthreads();
#pragma unroll 3
    for (int e = tid; e < RB * (H + 1); e += THREADS) {
      const int r = e / (H + 1);
      const int k = e - r * (H + 1);
      const int y = y0 + r;
      if (y >= P.ny) continue;
      const cplx<double> z0 = buf[lds_pad(r * H)];
      cplx<double> out;
      if (k == 0) {
        out = mk(z0.x + z0.y, 0.0);
      } else if (k == H) {
        out = mk(z0.x - z0.y, 0.0);
      } else {
        const cplx<double> zk = buf[lds_pad(r * H + k)];
        const cplx<double> zm = conjg(buf[lds_pad(r * H + H - k)]);
        const cplx<double> e2 = zk + zm;
        const cplx<double> o2 = rot90<double, false>(zk - zm);
        out = scale(e2 + twid<double, false>(tw, k << twsx) * o2, 0.5);
      }
      Uq[((int64_t)p * P.ny + y) * (H + 1) + k] = out;
    }
  }
}

// K[a][u_y][kx] = sum_{u_x} k_{a,u} e^{-2 pi i kx u_x / Px}
__global__ void sub_kspec_kernel(SpecParams P, const double* __restrict__ theta, cplx<double>* __restrict__ K,
                                 const cplx<double>* __restrict__ tw) {
  const int L = 2 * P.w + 1;
  const int H = P.H;
  const int row = blockIdx.y;            // a * L + (u_y + w)
  const int kx = blockIdx.x * blockDim.x + threadIdx.x;
  if (kx > H) return;
  const int a = row / L;
  const int uyi = row - a * L;
  const int twsx = TW_LOG - P.lgPx;
  const int Px = 2 * H;
  cplx<double> acc = mk(0.0, 0.0);
#pragma unroll 4
  for (int uxi = 0; uxi < L; ++uxi) {
    const int ux = uxi - P.w;
    const double k = theta[a * L * L + uyi * L + uxi];
    const int m = (int)(((int64_t)kx * (ux + Px)) & (Px - 1));
    acc = acc + scale(twid<double, false>(tw, m << twsx), k);
  }
  K[(int64_t)row * (H + 1) + kx] = acc;
}

// Filters with the y-weight moved to the output row.  With yh(y - u_y) =
// yh(y) - u_y sy and the binomial expansion of its q-th power,
//   sum_a K_a(u_y) yh(y - u_y)^q_a U_{p_a}(y - u_y)
//     = sum_{p,e} yh(y)^e sum_{u_y} G_{p,e}(u_y) U_p(y - u_y),
//   G_{p,e}(u_y) = sum_{q >= e} C(q, e) (-u_y sy)^(q-e) K_{(p,q)}(u_y).
// The pairs (p, e) are the monomials themselves; G[(p,e)] takes the place of
// K[(p,q)] in the same layout, one thread per (u_y, kx).
__global__ void sub_gspec_kernel(SpecParams P, const cplx<double>* __restrict__ K, cplx<double>* __restrict__ G) {
  const int L = 2 * P.w + 1;
  const int H = P.H;
  const int uyi = blockIdx.y;
  const int kx = blockIdx.x * blockDim.x + threadIdx.x;
  if (kx > H) return;
  const double d = -(double)(uyi - P.w) * P.sy;   // -u_y sy
  for (int g = 0; g < P.nk; ++g) {
    const int p = P.kpx[g], e = P.kqy[g];
    cplx<double> acc = mk(0.0, 0.0);
    for (int a = 0; a < P.nk; ++a) {
      if (P.kpx[a] != p || P.kqy[a] < e) continue;
      const int q = P.kqy[a];
      const double c = binom(q, e) * ipow(d, q - e);
      acc = acc + scale(K[((int64_t)a * L + uyi) * (H + 1) + kx], c);
    }
    G[((int64_t)g * L + uyi) * (H + 1) + kx] = acc;
  }
}

// M(y, kx) = sum_a sum_{u_y} K[a][u_y][kx] yh(y - u_y)^q_a U_{p_a}(y - u_y, kx)
//          = sum_{p,e} yh(y)^e sum_{u_y} G[(p,e)][u_y][kx] U_p(y - u_y, kx)   (sub_gspec_kernel).
// Block: 64 kx columns (the lanes) x SUBC_WAVES waves of SUBC_TY output rows.
// For each x power p the block stages the source rows of U_p it needs in LDS
// once (HBM traffic ~ (1 + 2W / SUBC_RB) x the source).  For each filter of
// that power a thread takes the taps in groups of SUBC_GT (the next group's
// loads in flight meanwhile); within a group it sweeps the TY + GT - 1 source
// rows the group reaches, reading each from LDS once and adding it to every
// output row it feeds, so a source row is read (TY + GT - 1) / (GT TY) times per
// output and tap instead of once.  The last group is padded with zero taps
// (the window carries GT - 1 extra rows above for their reads).  The output
// rows are finally weighted by yh(y)^e.
constexpr int SUBC_TY = 6;                        // output rows per wave
constexpr int SUBC_WAVES = 8;
constexpr int SUBC_RB = SUBC_TY * SUBC_WAVES;     // output rows per block
constexpr int SUBC_GT = 4;                        // filter taps per group
constexpr int SUBC_PADR = SUBC_GT - 1;            // window rows above for the padded taps

__host__ __device__ constexpr size_t sub_conv_lds_bytes(int w) {
  return (size_t)(SUBC_RB + 2 * w + SUBC_PADR) * 64 * sizeof(cplx<double>);
}

template <int W>
__global__ __launch_bounds__(64 * SUBC_WAVES) void sub_conv_kernel(SpecParams P, const cplx<double>* __restrict__ Uq,
                                                                   const cplx<double>* __restrict__ G,
                                                                   cplx<double>* __restrict__ Mh) {
  constexpr int L = 2 * W + 1;
  constexpr int GT = SUBC_GT;
  constexpr int NG = (L + GT - 1) / GT;           // tap groups (the last one padded)
  constexpr int WINB = SUBC_RB + 2 * W + SUBC_PADR;   // window rows: source rows yb - W - PADR ..
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<double>* win = reinterpret_cast<cplx<double>*>(smem_raw);   // [WINB][64]
  const int H = P.H;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // blocks (column group bx, row band by) in y-major order through xcd_remap:
  // bands that share halo rows run on one XCD at about the same time
  const int nby = (P.ny + SUBC_RB - 1) / SUBC_RB;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = bid / nby, by = bid - bx * nby;
  if (bx * 64 > P.H) return;
  const int kx0 = bx * 64;
  const int kx = kx0 + lane;
  const int yb = by * SUBC_RB;                    // first output row of the block
  const int y0 = yb + wave * SUBC_TY;             // first output row of the wave
  cplx<double> acc[SUBC_TY];
#pragma unroll
  for (int t = 0; t < SUBC_TY; ++t) acc[t] = mk(0.0, 0.0);
  int pmax = 0;
  for (int a = 0; a < P.nk; ++a) pmax = max(pmax, (int)P.kpx[a]);
  for (int p = 0; p <= pmax; ++p) {
    const cplx<double>* Up = Uq + (int64_t)p * P.ny * (H + 1);
    __syncthreads();   // the previous power's rows have been read
    for (int e = tid; e < WINB * 64; e += 64 * SUBC_WAVES) {
      const int r = e >> 6, c = e & 63;
      const int ys = yb - W - SUBC_PADR + r;
      cplx<double> u = mk(0.0, 0.0);
      if (ys >= 0 && ys < P.ny && kx0 + c <= H) u = Up[(int64_t)ys * (H + 1) + kx0 + c];
      win[e] = u;
    }
    __syncthreads();
    if (kx > H) continue;
    for (int g = 0; g < P.nk; ++g) {
      if (P.kpx[g] != p) continue;
      const int ex = P.kqy[g];
      const cplx<double>* Ga = G + (int64_t)g * L * (H + 1) + kx;
      // output row y0 + t with tap u reads source row y0 + t + W - u, i.e.
      // window offset d = t - u from wl
      const cplx<double>* wl = win + (wave * SUBC_TY + 2 * W + SUBC_PADR) * 64 + lane;
      cplx<double> part[SUBC_TY];
#pragma unroll
      for (int t = 0; t < SUBC_TY; ++t) part[t] = mk(0.0, 0.0);
      cplx<double> kn[GT];   // taps of the next group (zero past the filter)
#pragma unroll
      for (int i = 0; i < GT; ++i) {
        const cplx<double> t = Ga[(int64_t)min(i, L - 1) * (H + 1)];
        kn[i] = i < L ? t : mk(0.0, 0.0);
      }
#pragma unroll 1
      for (int gi = 0; gi < NG; ++gi) {
        const int u0 = gi * GT;
        cplx<double> kv[GT];
#pragma unroll
        for (int i = 0; i < GT; ++i) {
          kv[i] = kn[i];
          const int u = u0 + GT + i;
          const cplx<double> t = Ga[(int64_t)min(u, L - 1) * (H + 1)];
          kn[i] = u < L ? t : mk(0.0, 0.0);
        }
        // source offsets d = t - u for this group run over [-(u0 + GT - 1), TY - 1 - u0]
        const cplx<double>* src = wl - (u0 + GT - 1) * 64;
#pragma unroll
        for (int dr = 0; dr < SUBC_TY + GT - 1; ++dr) {
          const cplx<double> v = src[dr * 64];
#pragma unroll
          for (int i = 0; i < GT; ++i) {
            const int t = dr - (GT - 1) + i;   // output row fed by tap u0 + i
            if (t >= 0 && t < SUBC_TY) part[t] = cmac(part[t], kv[i], v);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < SUBC_TY; ++t) {
        const double wy = ex > 0 ? ipow((double)(y0 + t) * P.sy - 1.0, ex) : 1.0;
        acc[t] = acc[t] + scale(part[t], wy);
      }
    }
  }
  if (kx > H) return;
#pragma unroll
  for (int t = 0; t < SUBC_TY; ++t) {
    const int y = y0 + t;
    if (y < P.ny) Mh[(int64_t)y * (H + 1) + kx] = acc[t];
  }
}

// C2R of M(y, .) and D = S - model - background on the columns [xlo, xhi).
// E(k) = (X(k) + conj X(H-k))/2, O(k) = (X(k) - conj X(H-k)) e^{2 pi i k/Px}/2,
// z = IDFT_H(E + i O)/H, model(2j) = Re z(j), model(2j+1) = Im z(j).
template <typename T, int THREADS, int NMAX, int LGH>
__global__ __launch_bounds__(THREADS) void sub_rowinv_kernel(SpecParams P, const cplx<double>* __restrict__ Mh,
                                                             const T* __restrict__ sci,
                                                             const double* __restrict__ theta, T* __restrict__ diff,
                                                             const cplx<double>* __restrict__ tw, int xlo, int xhi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  constexpr int RB = sub_row_rows(NMAX, LGH);
  constexpr int H = 1 << LGH;             // H = Px / 2
  constexpr int NPT = (RB * H) / THREADS;
  static_assert(NPT * THREADS == RB * H, "whole values per thread");
  const int y0 = blockIdx.x * RB;
  const int tid = threadIdx.x;
  constexpr int twsx = TW_LOG - (LGH + 1);
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int e = tid + i * THREADS;
    const int r = e >> LGH;
    const int k = e & (H - 1);
    const int y = y0 + r;
    // rows past ny read row ny - 1 and are dropped: every load is unconditional
    const cplx<double>* row = Mh + (int64_t)min(y, P.ny - 1) * (H + 1);
    const cplx<double> xk = row[k];
    const cplx<double> xm = conjg(row[H - k]);
    const cplx<double> e2 = xk + xm;                                       // 2 E
    const cplx<double> o2 = twid<double, true>(tw, k << twsx) * (xk - xm);  // 2 O
    const cplx<double> z = scale(e2 + rot90<double, true>(o2), 0.5);       // E + i O
    buf[lds_pad(e)] = y < P.ny ? z : mk(0.0, 0.0);
  }
  __syncthreads();
  const LdsRows<double, LGH> lds{buf};
  // background along each of the block's rows as a polynomial in xh:
  // bg(x, y) = sum_p c_p(y) xh^p with c_p(y) = sum over terms b with x power p
  // of theta_b yh^(q_b), evaluated by Horner's rule per pixel
  __shared__ double bcoef[RB][SUB_MAXP];
  const int L2 = (2 * P.w + 1) * (2 * P.w + 1);
  const int nkk = P.nk * L2;
  if (tid < RB * SUB_MAXP) {
    const int r = tid / SUB_MAXP, pw = tid - r * SUB_MAXP;
    const double yh = (double)(y0 + r) * P.sy - 1.0;
    double c = 0.0;
    for (int b = 0; b < P.nb; ++b)
      if (P.bpx[b] == pw) c += theta[nkk + b] * ipow(yh, P.bqy[b]);
    bcoef[r][pw] = c;
  }
  int pdeg = 0;
  for (int b = 0; b < P.nb; ++b) pdeg = max(pdeg, (int)P.bpx[b]);
  fft_run<double, NMAX, THREADS, true, true, true, LGH, 4>(buf, RB, tw, lds, lds);
  __syncthreads();
  const double invH = 1.0 / (double)H;
  // pixels x = xlo + tid + i THREADS of every row; the science values of the
  // thread are all loaded (clamped into the frame) before any is used
  constexpr int XPT = (2 * H + THREADS - 1) / THREADS;
  T sv[RB][XPT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int y = min(y0 + r, P.ny - 1);
      const int x = min(xlo + tid + i * THREADS, xhi - 1);
      sv[r][i] = sci[(int64_t)y * P.ld + x];
    }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int y = y0 + r;
    if (y >= P.ny) continue;
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int x = xlo + tid + i * THREADS;
      if (x >= xhi) continue;
      const cplx<double> z = buf[lds_pad(r * H + (x >> 1))];
      const double model = ((x & 1) ? z.y : z.x) * invH;
      const double xh = (double)x * P.sx - 1.0;
      double bg = bcoef[r][pdeg];
      for (int pw = pdeg - 1; pw >= 0; --pw) bg = bg * xh + bcoef[r][pw];
      diff[(int64_t)y * P.ld + x] = (T)((double)sv[r][i] - model - bg);
    }
  }
}

}  // namespace sfft
