// Assembly of the normal equations Omega theta = beta from FFT cross-correlations.
//
// The entries are lag windows of cross-correlations of the polynomial-weighted
// planes (see sfft.h for the fit):
//   Omega[(a,u),(b,v)] = C_ab(u - v),  C_ab(d) = sum_z A_a(z) A_b(z + d),  |d| <= 2w
//   Omega[(a,u), b]    = sum_z A_a(z) (G m_b)(z + u),                    |u| <= w
//   beta[(a,u)]        = sum_z A_a(z) S_m(z + u)
//   Omega[b, b'] = sum G m_b m_b',  beta[b] = sum G m_b S      (FP64 moments)
// Because A_a is zero within w pixels of the frame edge, circular transforms of
// any period P >= N give these linear correlations exactly, so the transform
// size is the next power of two >= N on each axis (P = 4096 for 4088).
//
// Data flow (one pair):
//   row_fwd   : each plane row (generated on the fly from S, R, mask) -> R2C
//               along x; written transposed, U[p][kx][y] (kx = 0 packs the
//               real DC and Nyquist values as re/im).
//   col_fwd   : FFT along y of every column, in place; column 0 is unpacked
//               into the DC column 0 and the Nyquist column H.  Output order
//               is residue-major: slot k1*P2 + k2 holds X(ky = k1 + P1 k2).
//   corr      : per column kx, every needed product conj(X_a) X_b and its
//               inverse transform along y evaluated only on the lag rows
//               |j| <= hw, via F_k1(r) = sum_k2 Z(k1 + P1 k2) e^{2 pi i k2 r/P2}
//               and V(j) = sum_k1 e^{2 pi i k1 j/Py} F_k1(j mod P2).  Spectra are
//               stored in the mode's type; products, the inner transform and
//               the sum over k1 are FP64 in both modes.
//   row_win   : inverse along x of the lag rows, only on the lag columns, in
//               FP64, using the Hermitian symmetry of real correlations.
//   moments   : FP64 per-row sums for the background block; non-finite scan.
//   gather    : scatter the windows and moments into dense Omega and beta.
#pragma once

#include "common.hpp"

namespace sfft {

constexpr int P2 = 16;        // inner (register) transform length of the pruned inverse
constexpr int LG_P2 = 4;
constexpr int JMAX = 19;      // lag rows handled per correlation work item
constexpr int MAX_DEG = 4;    // polynomial degree limit for DK and DB
constexpr int MAX_NB = (MAX_DEG + 1) * (MAX_DEG + 2) / 2;   // 15 monomials
constexpr int MAX_PLANES = 2 * MAX_NB + 1;
constexpr int MAX_ITEMS = 512;

struct PolyTab {
  int8_t px[MAX_NB];
  int8_t qy[MAX_NB];
};

// One correlation work item: lag rows [jlo, jlo + nj) of pair (left, right).
struct CorrItem {
  int16_t left, right;   // plane indices
  int16_t jlo, nj;       // first lag row (signed) and count (<= JMAX)
  int32_t vrow;          // row in V where lag row jlo goes
};

struct AsmParams {
  int ny, nx, w, nk, nb, nplanes;
  int lgPy, lgPx;        // transform sizes Py = 2^lgPy, Px = 2^lgPx
  int H;                 // Px / 2
  int64_t ld;            // input row pitch (elements)
  int rows_per_block;    // row_fwd rows per block
  int nrowblk;           // number of row blocks
  int nitems;            // correlation items
  int vrows;             // rows of V (sum over pairs of window heights)
  PolyTab kpoly, bpoly;
  int nmom;              // per-row moments: (2DB+1) G-moments + (DB+1) S-moments
  int db;
};

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int i = 0; i < p; ++i) r *= x;
  return r;
}

// value of plane p at (y, x): A_a = m_a G_R R, G m_b, or G S
template <typename T>
__device__ __forceinline__ T plane_value(const AsmParams& P, int p, int y, int x, const T* __restrict__ sci,
                                         const T* __restrict__ tmpl, const uint8_t* __restrict__ mask) {
  if (x >= P.nx) return (T)0;
  const int64_t o = (int64_t)y * P.ld + x;
  const bool good = (mask == nullptr) || (mask[o] == 0);
  if (!good) return (T)0;
  const double xh = 2.0 * (double)x / (double)(P.nx - 1) - 1.0;
  const double yh = 2.0 * (double)y / (double)(P.ny - 1) - 1.0;
  if (p < P.nk) {
    const int w = P.w;
    if (y < w || y >= P.ny - w || x < w || x >= P.nx - w) return (T)0;
    const double m = ipow(xh, P.kpoly.px[p]) * ipow(yh, P.kpoly.qy[p]);
    return (T)(m * (double)tmpl[o]);
  }
  if (p < P.nk + P.nb) {
    const int b = p - P.nk;
    return (T)(ipow(xh, P.bpoly.px[b]) * ipow(yh, P.bpoly.qy[b]));
  }
  return sci[o];
}

// XCD-aware block order: consecutive row blocks land on the same XCD (blocks
// are dispatched round-robin over the 8 XCDs), so the transposed 64-byte
// segments that neighbouring row blocks write into one line meet in one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int per = (nblk + 7) >> 3;
  const int xcd = bid & 7;
  const int slot = bid >> 3;
  const int r = xcd * per + slot;
  return r;
}

// ---------------------------------------------------------------------------
// row_fwd: R2C along x of every plane row; transposed write into U
// ---------------------------------------------------------------------------
// LDS: rows_per_block * H complex values.  Each row is packed as
// z(j) = x(2j) + i x(2j+1), transformed with an H-point FFT and split:
//   X(k) = E(k) + e^{-2 pi i k/Px} O(k),  E = (Z(k) + conj Z(H-k))/2,
//   O = (Z(k) - conj Z(H-k))/(2i);   slot 0 holds (X(0), X(H)).
template <typename T, int THREADS, int NMAX>
__global__ __launch_bounds__(THREADS) void row_fwd_kernel(AsmParams P, const T* __restrict__ sci,
                                                          const T* __restrict__ tmpl,
                                                          const uint8_t* __restrict__ mask, cplx<T>* __restrict__ U,
                                                          const cplx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int rb = xcd_remap(blockIdx.x, gridDim.x);
  if (rb >= P.nrowblk) return;
  const int RB = P.rows_per_block;
  const int y0 = rb * RB;
  const int H = P.H;
  const int lgH = P.lgPx - 1;
  const int Py = 1 << P.lgPy;
  const int64_t pstride = (int64_t)(H + 1) * Py;
  const int tid = threadIdx.x;
  const int twsx = TW_LOG - P.lgPx;
  for (int p = 0; p < P.nplanes; ++p) {
    for (int e = tid; e < RB * H; e += THREADS) {
      const int r = e >> lgH;
      const int j = e & (H - 1);
      const int y = y0 + r;
      cplx<T> z = mk((T)0, (T)0);
      if (y < P.ny) {
        z.x = plane_value<T>(P, p, y, 2 * j, sci, tmpl, mask);
        z.y = plane_value<T>(P, p, y, 2 * j + 1, sci, tmpl, mask);
      }
      buf[e] = z;
    }
    __syncthreads();
    fft_lds<T, NMAX, THREADS, false>(buf, lgH, RB, H, tw);
    // split and write: e -> (kx, r) with r fastest so that a column segment is contiguous
    cplx<T>* Up = U + (int64_t)p * pstride;
    for (int e = tid; e < RB * H; e += THREADS) {
      const int r = e % RB;
      const int k = e / RB;
      const int y = y0 + r;
      if (y >= P.ny) continue;
      const cplx<T>* row = buf + r * H;
      const cplx<T> zk = row[k];
      const cplx<T> zm = conjg(row[(H - k) & (H - 1)]);
      cplx<T> out;
      if (k == 0) {
        // E(0) = Re Z0, O(0) = Im Z0; X(0) = E + O, X(H) = E - O
        out = mk(zk.x + zk.y, zk.x - zk.y);
      } else {
        const cplx<T> e2 = zk + zm;                 // 2 E
        const cplx<T> o2 = rot90<T, false>(zk - zm);  // 2 O = -i (Z - conj Z(H-k))
        const cplx<T> t = twid<T, false>(tw, k << twsx);
        out = scale(e2 + t * o2, (T)0.5);
      }
      Up[(int64_t)k * Py + y] = out;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// col_fwd: FFT along y of every column (in place), residue-major output
// ---------------------------------------------------------------------------
// Block = `cpb` consecutive columns of one plane.  Column 0 holds the packed
// (DC, Nyquist) real-column pair z = x0 + i xN; after the transform
// X0(ky) = (Z(ky) + conj Z(-ky))/2 and XN(ky) = (Z(ky) - conj Z(-ky))/(2i),
// written to columns 0 and H.
template <typename T, int THREADS, int NMAX>
__global__ __launch_bounds__(THREADS) void col_fwd_kernel(AsmParams P, cplx<T>* __restrict__ U,
                                                          const cplx<T>* __restrict__ tw, int cpb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int p = blockIdx.y;
  const int kx0 = blockIdx.x * cpb;
  const int Py = 1 << P.lgPy;
  const int lgPy = P.lgPy;
  const int H = P.H;
  const int tid = threadIdx.x;
  cplx<T>* Up = U + (int64_t)p * (H + 1) * Py;
  const int ncol = min(cpb, H - kx0);
  for (int e = tid; e < ncol * Py; e += THREADS) {
    const int c = e >> lgPy;
    const int y = e & (Py - 1);
    buf[e] = (y < P.ny) ? Up[(int64_t)(kx0 + c) * Py + y] : mk((T)0, (T)0);
  }
  __syncthreads();
  fft_lds<T, NMAX, THREADS, false>(buf, lgPy, ncol, Py, tw);
  const int lgP1 = lgPy - LG_P2;
  for (int e = tid; e < ncol * Py; e += THREADS) {
    const int c = e >> lgPy;
    const int s = e & (Py - 1);           // output slot = k1 * P2 + k2
    const int k1 = s >> LG_P2;
    const int k2 = s & (P2 - 1);
    const int ky = k1 + (k2 << lgP1);
    const cplx<T>* col = buf + (c << lgPy);
    if (kx0 + c == 0) {
      const cplx<T> z = col[ky];
      const cplx<T> zm = conjg(col[(Py - ky) & (Py - 1)]);
      Up[s] = scale(z + zm, (T)0.5);
      Up[(int64_t)H * Py + s] = scale(rot90<T, false>(z - zm), (T)0.5);
    } else {
      Up[(int64_t)(kx0 + c) * Py + s] = col[ky];
    }
  }
}

// ---------------------------------------------------------------------------
// corr: spectral products and pruned inverse along y on the lag rows
// ---------------------------------------------------------------------------
// One block per column kx in [0, H].  Residues k1 are processed in chunks of
// C1; for each chunk all planes' slots [k1*P2, (k1+1)*P2) are staged in LDS.
// Item i (pair, lag rows) is handled by `lanes` threads that split the
// residues; at the end the lanes are summed in LDS and written to V.
// For lag row j = jlo + t: V(j) = sum_k1 e^{2 pi i k1 j/Py} F_k1(j mod P2).  The
// residue rotation j mod P2 = (jlo + t) mod P2 is folded into the inner DFT by
// pre-multiplying Z(k2) by e^{2 pi i k2 s/P2}, s = jlo mod P2, so that output t
// of the DFT is F_k1((jlo + t) mod P2).
template <typename T, int THREADS>
__global__ __launch_bounds__(THREADS) void corr_kernel(AsmParams P, const cplx<T>* __restrict__ U,
                                                       const CorrItem* __restrict__ items,
                                                       cplx<double>* __restrict__ V,
                                                       const cplx<T>* __restrict__ tw,
                                                       const cplx<double>* __restrict__ twd, int C1) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* stage = reinterpret_cast<cplx<T>*>(smem_raw);
  const int kx = blockIdx.x;
  const int H = P.H;
  const int Py = 1 << P.lgPy;
  const int lgPy = P.lgPy;
  const int P1 = Py >> LG_P2;
  const int tid = threadIdx.x;
  const int nitems = P.nitems;
  const int lanes = max(1, THREADS / nitems);
  const int64_t pstride = (int64_t)(H + 1) * Py;

  for (int base = 0; base < nitems * lanes; base += THREADS) {
    const int gt = base + tid;
    const int item_id = gt / lanes;
    const int lane = gt % lanes;
    const bool active = item_id < nitems;
    CorrItem it;
    it.left = 0;
    it.right = 0;
    it.jlo = 0;
    it.nj = 0;
    it.vrow = 0;
    if (active) it = items[item_id];
    // pre-rotation by s = jlo mod P2 (FP64: the correlation arithmetic is FP64 in both modes)
    const int s = ((int)it.jlo % P2 + P2) % P2;
    cplx<double> rot[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) rot[k2] = twid<double, true>(twd, (k2 * s) << (TW_LOG - LG_P2));
    cplx<double> acc[JMAX];
#pragma unroll
    for (int t = 0; t < JMAX; ++t) acc[t] = mk(0.0, 0.0);

    for (int k1c = 0; k1c < P1; k1c += C1) {
      const int nc = min(C1, P1 - k1c);
      __syncthreads();
      // stage slots [k1c*P2, (k1c+nc)*P2) of every plane
      const int per_plane = nc * P2;
      for (int e = tid; e < P.nplanes * per_plane; e += THREADS) {
        const int pl = e / per_plane;
        const int o = e - pl * per_plane;
        stage[e] = U[pl * pstride + (int64_t)kx * Py + (int64_t)k1c * P2 + o];
      }
      __syncthreads();
      if (!active) continue;
      for (int c = lane; c < nc; c += lanes) {
        const int k1 = k1c + c;
        const cplx<T>* xa = stage + it.left * per_plane + c * P2;
        const cplx<T>* xb = stage + it.right * per_plane + c * P2;
        cplx<double> z[P2];
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) {
          const cplx<double> a = mk((double)xa[k2].x, (double)xa[k2].y);
          const cplx<double> b = mk((double)xb[k2].x, (double)xb[k2].y);
          z[k2] = cmulc(a, b) * rot[k2];
        }
        dft16<double, true>(z);
        // outer twiddle e^{2 pi i k1 j / Py} for j = jlo + t, by recurrence in FP64
        const int m0 = ((k1 * (int)it.jlo) % Py + Py) % Py;
        cplx<double> tj = conjg(twd[m0 << (TW_LOG - lgPy)]);
        const cplx<double> step = conjg(twd[k1 << (TW_LOG - lgPy)]);
#pragma unroll
        for (int t = 0; t < JMAX; ++t) {
          if (t < it.nj) {
            acc[t] = acc[t] + tj * z[t & (P2 - 1)];
            tj = tj * step;
          }
        }
      }
    }
    // reduce the lanes of each item through LDS (reuse the staging area)
    __syncthreads();
    cplx<double>* red = reinterpret_cast<cplx<double>*>(smem_raw);
    if (active) {
#pragma unroll
      for (int t = 0; t < JMAX; ++t) red[tid * JMAX + t] = acc[t];
    }
    __syncthreads();
    if (active && lane == 0) {
      for (int t = 0; t < it.nj; ++t) {
        cplx<double> sum = mk(0.0, 0.0);
        for (int l = 0; l < lanes; ++l) sum = sum + red[(tid + l) * JMAX + t];
        V[(int64_t)kx * P.vrows + it.vrow + t] = sum;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// row_win: inverse along x restricted to the lag columns, FP64
// ---------------------------------------------------------------------------
// C(j, i) = 1/(Py Px) [ V(j,0) + (-1)^i V(j,H) + 2 Re sum_{kx=1}^{H-1} V(j,kx) e^{2 pi i kx i / Px} ]
// One block per V row; the window half-width of the row's pair is hw.
struct WinRow {
  int32_t vrow;     // row of V
  int32_t out;      // offset of the first window value of this row in `win`
  int32_t hw;       // half-width of the lag columns
};

template <int THREADS, int IMAX>
__global__ __launch_bounds__(THREADS) void row_win_kernel(AsmParams P, const cplx<double>* __restrict__ V,
                                                          const WinRow* __restrict__ rows, double* __restrict__ win,
                                                          const cplx<double>* __restrict__ twd) {
  static_assert(THREADS == 64, "one wave per window row");
  const WinRow R = rows[blockIdx.x];
  const int H = P.H;
  const int lgPx = P.lgPx;
  const int tid = threadIdx.x;
  const int ni = 2 * R.hw + 1;
  double acc[IMAX];
#pragma unroll
  for (int i = 0; i < IMAX; ++i) acc[i] = 0.0;
  for (int kx = tid; kx <= H; kx += THREADS) {
    const cplx<double> v = V[(int64_t)kx * P.vrows + R.vrow];
    if (kx == 0 || kx == H) {
      // real values with weight 1; the Nyquist column alternates in sign, (-1)^(i - hw)
      const bool nyq = (kx == H);
      double sg = (nyq && (R.hw & 1)) ? -1.0 : 1.0;
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        if (i < ni) {
          acc[i] += sg * v.x;
          if (nyq) sg = -sg;
        }
      }
    } else {
      // 2 Re(v e^{2 pi i kx (i - hw)/Px}) by FP64 recurrence
      const int m0 = (int)(((int64_t)kx * (int64_t)(2 * H - R.hw)) & (int64_t)(2 * H - 1));
      cplx<double> t = conjg(twd[m0 << (TW_LOG - lgPx)]);
      const cplx<double> st = conjg(twd[kx << (TW_LOG - lgPx)]);
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        if (i < ni) {
          acc[i] += 2.0 * (v.x * t.x - v.y * t.y);
          t = t * st;
        }
      }
    }
  }
  const double norm = 1.0 / ((double)(1 << P.lgPy) * (double)(2 * H));
#pragma unroll
  for (int i = 0; i < IMAX; ++i) {
    if (i < ni) {
      double v = acc[i];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (tid == 0) win[R.out + i] = v * norm;
    }
  }
}

// ---------------------------------------------------------------------------
// moments: per-row FP64 sums for the background block, and the non-finite scan
// ---------------------------------------------------------------------------
// mom[y][p]          = sum_x G xh^p,      p in [0, 2DB]
// mom[y][2DB+1+p]    = sum_x G S xh^p,    p in [0, DB]
template <typename T, int THREADS>
__global__ __launch_bounds__(THREADS) void moments_kernel(AsmParams P, const T* __restrict__ sci,
                                                          const T* __restrict__ tmpl,
                                                          const uint8_t* __restrict__ mask,
                                                          double* __restrict__ mom, int* __restrict__ nonfinite) {
  constexpr int NG_MAX = 2 * MAX_DEG + 1;
  constexpr int NS_MAX = MAX_DEG + 1;
  __shared__ double red[THREADS];
  const int y = blockIdx.x;
  const int tid = threadIdx.x;
  const int nG = 2 * P.db + 1;
  const int nS = P.db + 1;
  double ag[NG_MAX], as[NS_MAX];
#pragma unroll
  for (int i = 0; i < NG_MAX; ++i) ag[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NS_MAX; ++i) as[i] = 0.0;
  bool bad = false;
  for (int x = tid; x < P.nx; x += THREADS) {
    const int64_t o = (int64_t)y * P.ld + x;
    const double s = (double)sci[o];
    const double r = (double)tmpl[o];
    bad |= !isfinite(s) || !isfinite(r);
    const bool good = (mask == nullptr) || (mask[o] == 0);
    if (!good) continue;
    const double xh = 2.0 * (double)x / (double)(P.nx - 1) - 1.0;
    double pw = 1.0;
#pragma unroll
    for (int p = 0; p < NG_MAX; ++p) {
      if (p < nG) ag[p] += pw;
      if (p < NS_MAX && p < nS) as[p] += pw * s;
      pw *= xh;
    }
  }
  if (bad) atomicOr(nonfinite, 1);
#pragma unroll
  for (int i = 0; i < NG_MAX + NS_MAX; ++i) {
    const bool use = (i < NG_MAX) ? (i < nG) : (i - NG_MAX < nS);
    if (use) {
      red[tid] = (i < NG_MAX) ? ag[i < NG_MAX ? i : 0] : as[i >= NG_MAX ? i - NG_MAX : 0];
      __syncthreads();
      for (int s2 = THREADS / 2; s2 > 0; s2 >>= 1) {
        if (tid < s2) red[tid] += red[tid + s2];
        __syncthreads();
      }
      if (tid == 0) mom[(int64_t)y * P.nmom + ((i < NG_MAX) ? i : nG + (i - NG_MAX))] = red[0];
      __syncthreads();
    }
  }
}

// One block: Omega_BB and beta_B from the per-row moments (fixed summation order).
template <int THREADS>
__global__ __launch_bounds__(THREADS) void moments_reduce_kernel(AsmParams P, const double* __restrict__ mom,
                                                                 double* __restrict__ obb, double* __restrict__ bb) {
  __shared__ double red[THREADS];
  const int tid = threadIdx.x;
  const int nb = P.nb;
  const int nG = 2 * P.db + 1;
  for (int q = 0; q < nb * nb + nb; ++q) {
    double acc = 0.0;
    for (int y = tid; y < P.ny; y += THREADS) {
      const double yh = 2.0 * (double)y / (double)(P.ny - 1) - 1.0;
      if (q < nb * nb) {
        const int b = q / nb, c = q % nb;
        const int p = P.bpoly.px[b] + P.bpoly.px[c];
        const int e = P.bpoly.qy[b] + P.bpoly.qy[c];
        acc += ipow(yh, e) * mom[(int64_t)y * P.nmom + p];
      } else {
        const int b = q - nb * nb;
        acc += ipow(yh, P.bpoly.qy[b]) * mom[(int64_t)y * P.nmom + nG + P.bpoly.px[b]];
      }
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = THREADS / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      if (q < nb * nb) obb[q] = red[0];
      else bb[q - nb * nb] = red[0];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// gather: dense Omega (both triangles) and beta
// ---------------------------------------------------------------------------
struct GatherParams {
  int n, nkk, L, w, nk, nb;
  int kk_off[MAX_NB * MAX_NB];  // window offset of C_ab for a <= b (index a*nk + b)
  int kb_off[MAX_NB * MAX_NB];  // window offset of corr(A_a, G m_b) (index a*nb + b)
  int ks_off[MAX_NB];           // window offset of corr(A_a, S_m)
};

__global__ void gather_kernel(GatherParams G, const double* __restrict__ win, const double* __restrict__ obb,
                              const double* __restrict__ bb, double* __restrict__ omega,
                              double* __restrict__ beta) {
  const int r = blockIdx.y;
  const int L = G.L, w = G.w;
  const int L2 = L * L;
  const int WK = 4 * w + 1;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < G.n; c += gridDim.x * blockDim.x) {
    double v;
    if (r < G.nkk && c < G.nkk) {
      const int a = r / L2, ur = r - a * L2;
      const int b = c / L2, vc = c - b * L2;
      const int uy = ur / L - w, ux = ur % L - w;
      const int vy = vc / L - w, vx = vc % L - w;
      if (a <= b) {
        v = win[G.kk_off[a * G.nk + b] + (uy - vy + 2 * w) * WK + (ux - vx + 2 * w)];
      } else {
        v = win[G.kk_off[b * G.nk + a] + (vy - uy + 2 * w) * WK + (vx - ux + 2 * w)];
      }
    } else if (r < G.nkk) {
      const int a = r / L2, ur = r - a * L2;
      const int b = c - G.nkk;
      v = win[G.kb_off[a * G.nb + b] + ur];
    } else if (c < G.nkk) {
      const int a = c / L2, uc = c - a * L2;
      const int b = r - G.nkk;
      v = win[G.kb_off[a * G.nb + b] + uc];
    } else {
      v = obb[(r - G.nkk) * G.nb + (c - G.nkk)];
    }
    omega[(int64_t)r * G.n + c] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (r < G.nkk) {
      const int a = r / L2, ur = r - a * L2;
      beta[r] = win[G.ks_off[a] + ur];
    } else {
      beta[r] = bb[r - G.nkk];
    }
  }
}

}  // namespace sfft
