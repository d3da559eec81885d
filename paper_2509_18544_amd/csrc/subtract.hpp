// Difference image D = S - sum_{a,u} k_{a,u} T_u(m_a R) - sum_b c_b m_b.
//
// The polynomial weight acts on template pixels before the shift.  Writing
// m_a at the source pixel z - u as a polynomial in the output pixel z,
//   xh(x - u_x) = xh(x) - 2 u_x/(nx-1),   yh(y - u_y) = yh(y) - 2 u_y/(ny-1),
//   m_(p,q)(z - u) = sum_{i<=p, j<=q} C(p,i) C(q,j) (-dx)^(p-i) (-dy)^(q-j) m_(i,j)(z),
// gives model(z) = sum_a' m_a'(z) sum_u k'_{a',u} R(z - u) with
// k'_{a',u} = sum_a k_{a,u} e_{a,a'}(u): nK plain convolutions of the same
// unmasked template, combined with the output-side monomials.  Pixels outside
// the frame contribute zero (linear convolution, no wrap-around).  The border
// columns that the spectral route below cannot produce exactly are summed
// this way, directly, with k' (band_model).
#pragma once

#include "common.hpp"

namespace sfft {

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
// (x >= w - (Px - nx) and x < Px - w).  The remaining border columns (at most
// w on each side) are summed directly in the inverse row pass.  All of it in
// FP64, and the spectra U_p and M are stored as complex128 in both modes:
// complex64 storage moves the FP32 rounding of every spectral value into
// every pixel of the model (about 1e-6 of |D| over the frame at 4096^2, with
// single faint pixels above 1e-5 of their local scale).
struct SpecParams {
  int ny, nx, w, nk, nb;
  int lgPx, H;           // Px = 2^lgPx, H = Px / 2; spectra rows hold H + 1 values
  int64_t ld;
  int rows_per_block;
  int nrowblk;
  double sx, sy;
  int8_t kpx[15], kqy[15];
  int8_t bpx[15], bqy[15];
  int xp32;              // x-power spectra p >= 1 stored as complex64 (FP32C); p = 0 always complex128
};

// Byte offset of the x-power row spectra of power p in the subtraction's
// buffer: power 0 as complex128, then powers 1.. as complex64 (xp32) or
// complex128.  The powers p >= 1 enter the model multiplied by the spatial
// variation of the kernel, so their FP32 rounding stays well below that of
// the FP32 images (power 0 is kept in FP64: its rounding would be spread by
// the inverse transform over every pixel of the row at the full model scale).
__host__ __device__ inline size_t sub_xpow_off(int p, int ny, int H, int xp32) {
  if (p == 0) return 0;
  const size_t row = (size_t)ny * (H + 1);
  return ((row * sizeof(cplx<double>) + 255) & ~(size_t)255) +
         (size_t)(p - 1) * row * (xp32 ? sizeof(cplx<float>) : sizeof(cplx<double>));
}

constexpr int SUB_MAXP = 5;   // x powers of the background polynomial (degree <= 4)

// rows per block of the subtraction's row transforms (a power of two)
__host__ __device__ constexpr int sub_row_rows(int nmax, int lgh) { return (nmax >> lgh) < 64 ? (nmax >> lgh) : 64; }

// R2C of the rows xh^p R (p = 0..DK) -> Uq[p][y][0..H] (layout: sub_xpow_off)
template <typename T, int THREADS, int NMAX, int LGH>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 4 : 2) void sub_rowfwd_kernel(SpecParams P, PairSet PS, WsOff O,
                                                                                     int npow) {
  const int pr = blockIdx.z;
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  unsigned char* __restrict__ Ub = ws_at<unsigned char>(PS, pr, O.Uq);
  const cplx<double>* __restrict__ tw = ws_at<const cplx<double>>(PS, pr, O.tw64);
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
    const bool f32 = P.xp32 && p > 0;
    cplx<double>* __restrict__ Uq = reinterpret_cast<cplx<double>*>(Ub + sub_xpow_off(p, P.ny, H, P.xp32));
    cplx<float>* __restrict__ Uqf = reinterpret_cast<cplx<float>*>(Uq);
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
      const int64_t o = (int64_t)y * (H + 1) + k;
      if (f32)
        Uqf[o] = mk((float)out.x, (float)out.y);
      else
        Uq[o] = out;
    }
  }
}

// Binomial coefficients C(n, k) for n <= 4 (polynomial degrees are at most 4).
__device__ __forceinline__ double binom4(int n, int k) {
  constexpr double tab[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  return tab[n][k];
}

// Filters of the y-convolution and the output-side kernel k', in one launch.
//
// The y-weight moves to the output row: with yh(y - u_y) = yh(y) - u_y sy
// and the binomial expansion of its q-th power,
//   sum_a K_a(u_y) yh(y - u_y)^q_a U_{p_a}(y - u_y)
//     = sum_{p,e} yh(y)^e sum_{u_y} G_{p,e}(u_y) U_p(y - u_y),
//   G_{p,e}(u_y, kx) = sum_{u_x} e^{-2 pi i kx u_x / Px} gamma_{p,e}(u_y, u_x),
//   gamma_{p,e}(u_y, u_x) = sum_{q >= e} C(q, e) (-u_y sy)^(q-e) k_{(p,q),u}.
// The pairs (p, e) are the monomials themselves, so G[g] (g = (p, e)) has
// the layout of the coefficients: G[(g L + u_y + w)(H + 1) + kx].
// Blocks [0, ngb): a block takes one u_y and 256 kx; it forms gamma of its
// u_y in LDS, then each thread sums every G_g of its kx.
// Blocks [ngb, ..): one thread per (a', u) forming k'_{a',u} =
//   sum_a k_{a,u} C(p_a, p') C(q_a, q') (-u_x sx)^(p_a - p') (-u_y sy)^(q_a - q')
// for the border columns.
constexpr int PREP_THREADS = 256;
__global__ __launch_bounds__(PREP_THREADS) void sub_prep_kernel(SpecParams P, PairSet PS, WsOff O, int ngb) {
  const int pr = blockIdx.z;
  const double* __restrict__ theta = PS.coeffs[pr];
  cplx<double>* __restrict__ G = ws_at<cplx<double>>(PS, pr, O.G);
  double* __restrict__ kp = ws_at<double>(PS, pr, O.kp);
  const cplx<double>* __restrict__ tw = ws_at<const cplx<double>>(PS, pr, O.tw64);
  constexpr int LMAX = 2 * 15 + 1;
  __shared__ double gam[15][LMAX];
  const int L = 2 * P.w + 1;
  const int L2 = L * L;
  const int H = P.H;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= ngb) {
    const int id = ((int)blockIdx.x - ngb) * PREP_THREADS + tid;
    if (id >= P.nk * L2) return;
    const int ap = id / L2;
    const int u = id - ap * L2;
    const int uy = u / L - P.w, ux = u % L - P.w;
    const double dx = (double)ux * P.sx, dy = (double)uy * P.sy;
    const int i = P.kpx[ap], j = P.kqy[ap];
    double acc = 0.0;
    for (int a = 0; a < P.nk; ++a) {
      const int pa = P.kpx[a], qa = P.kqy[a];
      if (i > pa || j > qa) continue;
      acc += theta[a * L2 + u] * binom4(pa, i) * binom4(qa, j) * ipow(-dx, pa - i) * ipow(-dy, qa - j);
    }
    kp[ap * L2 + u] = acc;
    return;
  }
  const int nkb = (H + 1 + PREP_THREADS - 1) / PREP_THREADS;   // blocks per u_y row
  const int uyi = (int)blockIdx.x / nkb;
  const double d = -(double)(uyi - P.w) * P.sy;                // -u_y sy
  for (int e = tid; e < P.nk * L; e += PREP_THREADS) {
    const int g = e / L, uxi = e - g * L;
    const int pg = P.kpx[g], eg = P.kqy[g];
    double v = 0.0;
    for (int a = 0; a < P.nk; ++a) {
      if (P.kpx[a] != pg || P.kqy[a] < eg) continue;
      const int q = P.kqy[a];
      v += binom4(q, eg) * ipow(d, q - eg) * theta[a * L2 + uyi * L + uxi];
    }
    gam[g][uxi] = v;
  }
  __syncthreads();
  const int kx = ((int)blockIdx.x - uyi * nkb) * PREP_THREADS + tid;
  if (kx > H) return;
  const int twsx = TW_LOG - P.lgPx;
  const int Px = 2 * H;
  cplx<double> acc[15];
#pragma unroll
  for (int g = 0; g < 15; ++g) acc[g] = mk(0.0, 0.0);
  for (int uxi = 0; uxi < L; ++uxi) {
    const int m = (int)(((int64_t)kx * (uxi - P.w + Px)) & (Px - 1));
    const cplx<double> t = twid<double, false>(tw, m << twsx);
#pragma unroll
    for (int g = 0; g < 15; ++g)
      if (g < P.nk) acc[g] = acc[g] + scale(t, gam[g][uxi]);
  }
#pragma unroll
  for (int g = 0; g < 15; ++g)
    if (g < P.nk) G[((int64_t)g * L + uyi) * (H + 1) + kx] = acc[g];
}

constexpr int SUBC_TY = 6;                        // output rows per wave
constexpr int SUBC_WAVES = 8;
constexpr int SUBC_RB = SUBC_TY * SUBC_WAVES;     // output rows per block
constexpr int SUBC_GT = 4;                        // filter taps per group
constexpr int SUBC_PADR = SUBC_GT - 1;            // window rows above for the padded taps

__host__ __device__ constexpr size_t sub_conv_lds_bytes(int w) {
  return (size_t)(SUBC_RB + 2 * w + SUBC_PADR) * 64 * sizeof(cplx<double>);
}

template <int W>
__global__ __launch_bounds__(64 * SUBC_WAVES) void sub_conv_kernel(SpecParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  // the template's x-power row spectra: this pair's, or those of the pair whose template it shares
  const unsigned char* __restrict__ Ub = PS.tws[pr] + O.Uq;
  const cplx<double>* __restrict__ G = ws_at<const cplx<double>>(PS, pr, O.G);
  cplx<double>* __restrict__ Mh = ws_at<cplx<double>>(PS, pr, O.Mh);
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
    const bool f32 = P.xp32 && p > 0;
    const cplx<double>* Up = reinterpret_cast<const cplx<double>*>(Ub + sub_xpow_off(p, P.ny, H, P.xp32));
    const cplx<float>* Upf = reinterpret_cast<const cplx<float>*>(Up);
    __syncthreads();   // the previous power's rows have been read
    for (int e = tid; e < WINB * 64; e += 64 * SUBC_WAVES) {
      const int r = e >> 6, c = e & 63;
      const int ys = yb - W - SUBC_PADR + r;
      cplx<double> u = mk(0.0, 0.0);
      if (ys >= 0 && ys < P.ny && kx0 + c <= H) {
        const int64_t o = (int64_t)ys * (H + 1) + kx0 + c;
        if (f32) {
          const cplx<float> v = Upf[o];
          u = mk((double)v.x, (double)v.y);
        } else {
          u = Up[o];
        }
      }
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

// Direct model value at one border pixel (y, x), computed by one wave: the
// lanes split the L^2 offsets u, load the template value R(y - u_y, x - u_x)
// once per offset and sum sum_a k'_{a',u} m_a'(y, x) over the nK output-side
// monomials (evaluated once per pixel), then reduce by shuffles (lane 0 holds
// the total).  The template loads of a lane are unconditional (clamped into
// the frame, then selected) so that several are in flight.
template <typename T>
__device__ __forceinline__ double band_model(const SpecParams& P, int y, int x, const T* __restrict__ tmpl,
                                             const double* __restrict__ kp, int lane) {
  const int w = P.w;
  const int L = 2 * w + 1;
  const int L2 = L * L;
  const double yh = (double)y * P.sy - 1.0;
  const double xh = (double)x * P.sx - 1.0;
  double m[15];
#pragma unroll
  for (int a = 0; a < 15; ++a) m[a] = a < P.nk ? ipow(xh, P.kpx[a]) * ipow(yh, P.kqy[a]) : 0.0;
  double acc = 0.0;
#pragma unroll 4
  for (int r = lane; r < L2; r += 64) {
    const int uy = r / L - w;
    const int ux = r - (uy + w) * L - w;
    const int sy = y - uy, sx = x - ux;
    const bool in = sy >= 0 && sy < P.ny && sx >= 0 && sx < P.nx;
    const int64_t o = (int64_t)min(max(sy, 0), P.ny - 1) * P.ld + min(max(sx, 0), P.nx - 1);
    const double tv = (double)tmpl[o];
    double k = 0.0;
#pragma unroll
    for (int a = 0; a < 15; ++a)
      if (a < P.nk) k = fma(kp[a * L2 + r], m[a], k);
    acc += in ? k * tv : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  return acc;
}

// C2R of M(y, .) and D = S - model - background (apply_only: the model K * R
// itself, with no science image or background) on the columns [xlo, xhi)
// (blocks nbandblk.. , RB rows each); the border columns [0, xlo) and
// [xhi, nx) by direct sums (band_model) in blocks 0 .. nbandblk - 1, one wave
// per pixel.
// E(k) = (X(k) + conj X(H-k))/2, O(k) = (X(k) - conj X(H-k)) e^{2 pi i k/Px}/2,
// z = IDFT_H(E + i O)/H, model(2j) = Re z(j), model(2j+1) = Im z(j).
template <typename T, int THREADS, int NMAX, int LGH>
__global__ __launch_bounds__(THREADS) void sub_rowinv_kernel(SpecParams P, PairSet PS, WsOff O, int xlo, int xhi,
                                                             int nbandblk, int apply_only) {
  const int pr = blockIdx.z;
  const cplx<double>* __restrict__ Mh = ws_at<const cplx<double>>(PS, pr, O.Mh);
  const T* __restrict__ sci = static_cast<const T*>(PS.sci[pr]);
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const double* __restrict__ theta = PS.coeffs[pr];
  const double* __restrict__ kp = ws_at<const double>(PS, pr, O.kp);
  T* __restrict__ diff = static_cast<T*>(PS.diff[pr]);
  const cplx<double>* __restrict__ tw = ws_at<const cplx<double>>(PS, pr, O.tw64);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  constexpr int RB = sub_row_rows(NMAX, LGH);
  constexpr int H = 1 << LGH;             // H = Px / 2
  constexpr int NPT = (RB * H) / THREADS;
  static_assert(NPT * THREADS == RB * H, "whole values per thread");
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nbandblk) {
    // border columns [0, xlo) and [xhi, nx): one wave per pixel, direct sums.
    // These blocks come first in the grid so that their load latencies
    // overlap the transform blocks that follow.
    const int nleft = xlo, nband = xlo + (P.nx - xhi);
    const int lane = tid & 63;
    const int64_t pix = (int64_t)blockIdx.x * (THREADS / 64) + (tid >> 6);
    if (pix >= (int64_t)nband * P.ny) return;
    const int y = (int)(pix / nband);
    const int c = (int)(pix - (int64_t)y * nband);
    const int x = c < nleft ? c : xhi + (c - nleft);
    const double model = band_model<T>(P, y, x, tmpl, kp, lane);
    if (lane == 0 && apply_only) {
      diff[(int64_t)y * P.ld + x] = (T)model;
    } else if (lane == 0) {
      const int L2 = (2 * P.w + 1) * (2 * P.w + 1);
      const double xh = (double)x * P.sx - 1.0, yh = (double)y * P.sy - 1.0;
      double bg = 0.0;
      for (int b = 0; b < P.nb; ++b) bg += theta[P.nk * L2 + b] * ipow(xh, P.bpx[b]) * ipow(yh, P.bqy[b]);
      const int64_t o = (int64_t)y * P.ld + x;
      diff[o] = (T)((double)sci[o] - model - bg);
    }
    return;
  }
  const int y0 = ((int)blockIdx.x - nbandblk) * RB;
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
    for (int b = 0; b < (apply_only ? 0 : P.nb); ++b)
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
      sv[r][i] = apply_only ? (T)0 : sci[(int64_t)y * P.ld + x];   // no science image when applying K
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
      diff[(int64_t)y * P.ld + x] = apply_only ? (T)model : (T)((double)sv[r][i] - model - bg);
    }
  }
}

}  // namespace sfft
