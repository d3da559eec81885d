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
// lag rows per correlation work item: JROWS_WIDE when the template-template
// windows (4w + 1 rows) are wider than JROWS_NARROW, so that one item covers
// a whole window up to w = 9 and every item shares the rotation of -2w;
// JROWS_NARROW otherwise (fewer accumulators left idle)
constexpr int JROWS_NARROW = 19;
constexpr int JROWS_WIDE = 37;
constexpr int JMAX = JROWS_WIDE;   // the largest
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
  int16_t jlo, nj;       // first lag row (signed) and count (<= the plan's rows per item)
  int32_t vrow;          // row in V where lag row jlo goes
  int16_t jidx;          // index of jlo in the list of distinct first lag rows
  int16_t skip;          // the first `skip` lag rows are accumulated but not kept
};

constexpr int MAX_JLO = 8;  // distinct first lag rows among the items

constexpr int MAX_BASE = 2 * MAX_DEG + 3;   // x-weighted base rows: DK+1 + DB+1 + 1

struct AsmParams {
  int ny, nx, w, nk, nb, nplanes;
  int nbase, nbk, nbb;   // base rows: xh^p G_R R (p <= DK), xh^p G (p <= DB), G S
  double sx, sy;         // 2/(nx-1), 2/(ny-1): xh = x sx - 1, yh = y sy - 1
  int8_t base_first[MAX_BASE];   // outputs of base b: out_plane/out_q[base_first[b] .. + base_count[b])
  int8_t base_count[MAX_BASE];
  int8_t out_plane[MAX_PLANES];
  int8_t out_q[MAX_PLANES];
  int lgPy, lgPx;        // transform sizes Py = 2^lgPy, Px = 2^lgPx
  int H;                 // Px / 2
  int64_t ld;            // input row pitch (elements)
  int rows_per_block;    // row_fwd rows per block
  int nrowblk;           // number of row blocks
  int nitems;            // correlation items
  int vrows;             // rows of V (sum over pairs of window heights)
  PolyTab kpoly, bpoly;
  int nmom;              // per-row moments: (2DB+1) G-moments + (DB+1) S-moments + (DK+DB+1) G_R R moments
  int db;
  int na;                // DK + DB + 1: x powers of the G_R R moments
  int nmu;               // monomials of degree <= DK + DB
  int corr_lanes;        // threads per correlation item (divides into 64)
  int njlo;              // distinct first lag rows and their values
  int16_t jlo_list[MAX_JLO];
  int dir_tpr;           // direct route: threads per image row (power of two)
  // Which planes a build transforms and stages.  A full build transforms
  // every base row and stages all nplanes planes from its own workspace.  A
  // build of the right-hand side only (a pair that shares its template and
  // mask with another pair) transforms the science base alone and stages
  // nstaged = nK + 1 planes: the nK template planes from the sharing pair's
  // workspace (PS.tws), then its own science plane (plane nK + nB).
  int base_lo;           // first base row transformed (0, or nbase - 1)
  int nstaged;           // planes staged by the correlation kernel
  int nshared;           // of those, how many are read from PS.tws (the rest from PS.ws)
  int plane_skip;        // own-workspace plane of staged plane s >= nshared: s + plane_skip
};

// ---------------------------------------------------------------------------
// row_fwd: R2C along x of the x-weighted base rows; column-pair tiled write
// ---------------------------------------------------------------------------
// Every plane factors as (x part) * (y part): A_(p,q) = yh^q * [xh^p G_R R],
// G m_(p,q) = yh^q * [xh^p G], S_m = [G S].  Along a row yh is constant, so
// only the DK+DB+3 bracketed base rows are transformed here; the yh^q weight
// is applied by the column pass before its transform along y.
//
// Base row b at row y is packed as z(j) = x(2j) + i x(2j+1), transformed with
// an H-point FFT and split:
//   X(k) = E(k) + e^{-2 pi i k/Px} O(k),  E = (Z(k) + conj Z(H-k))/2,
//   O = (Z(k) - conj Z(H-k))/(2i);   slot 0 holds (X(0), X(H)).
// Output layout Ub[b][kx/2][y][kx%2]: the rows of one block and one column
// pair form one contiguous segment of 2 * rows * 8 bytes (FP32).
//
// Bases: b < nbk: xh^b G_R R (R zero outside the interior [w, n-w) of both
// axes), b < nbk + nbb: xh^(b-nbk) G, last: G S, with G = 0 at masked pixels
// and outside the frame.  A thread packs the same NPT pairs for every base, so
// it reads the mask once and keeps the G and G_R flags of its pairs as bits;
// every input load is unconditional (clamped into the frame, then selected),
// so a thread's loads for one base are all in flight together.
constexpr int ROW_RPAD = 16;   // LDS row padding of the row pass (rows 128 B apart in bank space)
__host__ __device__ constexpr int row_pass_rows(int nmax, int lgh) { return (nmax >> lgh) < 64 ? (nmax >> lgh) : 64; }
__host__ __device__ constexpr int row_pass_lds(int nmax, int lgh) {
  return lds_rows_size(row_pass_rows(nmax, lgh), lgh, ROW_RPAD);
}

template <typename T, int THREADS, int NMAX, int LGH>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 4 : 2) void row_fwd_kernel(AsmParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const T* __restrict__ sci = static_cast<const T*>(PS.sci[pr]);
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  cplx<T>* __restrict__ U = ws_at<cplx<T>>(PS, pr, O.Ub);
  const cplx<T>* __restrict__ tw = ws_at<const cplx<T>>(PS, pr, sizeof(T) == 4 ? O.tw32 : O.tw64);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int H = 1 << LGH;            // H = Px / 2
  constexpr int RB = row_pass_rows(NMAX, LGH);
  constexpr int NPT = (RB * H) / THREADS;
  static_assert(NPT * THREADS == RB * H && NPT >= 2 && NPT <= 16 && NPT % 2 == 0,
                "whole pairs per thread (an even number: two outputs per store), flags in 32 bits");
  const int rb = xcd_remap(blockIdx.x, gridDim.x);
  if (rb >= P.nrowblk) return;
  const int y0 = rb * RB;
  const int Py = 1 << P.lgPy;
  const int64_t pstride = (int64_t)H * Py;   // elements per base plane
  const int tid = threadIdx.x;
  constexpr int twsx = TW_LOG - (LGH + 1);
  const LdsRows<T, LGH, ROW_RPAD> lds{buf};
  const int nx = P.nx, ny = P.ny, w = P.w;
  // input offset of pixel (y, x), clamped into the frame so that every load is valid
  auto offs = [&](int y, int x) -> int64_t { return (int64_t)min(y, ny - 1) * P.ld + min(x, nx - 1); };
  uint32_t good = 0;    // bit 2i (+1): G of pixel 2j (2j+1) of pair i
  uint32_t gint = 0;    // the same, and inside the interior (G_R)
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int e = tid + i * THREADS;
    const int y = y0 + (e >> LGH);
    const int x0 = 2 * (e & (H - 1));
    const bool in0 = y < ny && x0 < nx, in1 = y < ny && x0 + 1 < nx;
    const bool g0 = in0 && (mask == nullptr || mask[offs(y, x0)] == 0);
    const bool g1 = in1 && (mask == nullptr || mask[offs(y, x0 + 1)] == 0);
    const bool iy = y >= w && y < ny - w;
    const bool i0 = g0 && iy && x0 >= w && x0 < nx - w;
    const bool i1 = g1 && iy && x0 + 1 >= w && x0 + 1 < nx - w;
    good |= ((uint32_t)g0 << (2 * i)) | ((uint32_t)g1 << (2 * i + 1));
    gint |= ((uint32_t)i0 << (2 * i)) | ((uint32_t)i1 << (2 * i + 1));
  }
  // FP64: the thread's template pairs, read once for all the x-power bases
  // (in FP32 the 32 registers they take would spill at four waves per SIMD,
  // so each base reads them again)
  constexpr bool CACHE_T = sizeof(T) == sizeof(double);
  T tv[CACHE_T ? NPT : 1][2];
  if constexpr (CACHE_T) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = tid + i * THREADS;
      const int y = y0 + (e >> LGH);
      const int x0 = 2 * (e & (H - 1));
      tv[i][0] = tmpl[offs(y, x0)];
      tv[i][1] = tmpl[offs(y, x0 + 1)];
    }
  }
  for (int b = P.base_lo; b < P.nbase; ++b) {
    __syncthreads();   // the previous base's split has read the buffer
    // packed base rows z(j) = x(2j) + i x(2j+1)
    const int kind = b < P.nbk ? 0 : (b < P.nbk + P.nbb ? 1 : 2);
    const int pw = kind == 0 ? b : b - P.nbk;
    // the lane index passes through an empty asm so that the per-pair
    // coordinates are recomputed per base instead of held in registers
    int lane = tid;
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = lane + i * THREADS;
      const int r = e >> LGH;
      const int j = e & (H - 1);
      const int x0 = 2 * j;
      const uint32_t flags = kind == 0 ? gint : good;
      const bool g0 = (flags >> (2 * i)) & 1u, g1 = (flags >> (2 * i + 1)) & 1u;
      cplx<T> z;
      if (kind == 2) {
        const int y = y0 + r;
        const T s0 = sci[offs(y, x0)], s1 = sci[offs(y, x0 + 1)];
        z = mk(g0 ? s0 : (T)0, g1 ? s1 : (T)0);
      } else {
        const double xh0 = (double)x0 * P.sx - 1.0;
        const double xh1 = (double)(x0 + 1) * P.sx - 1.0;
        double p0 = 1.0, p1 = 1.0;
        for (int q = 0; q < pw; ++q) {
          p0 *= xh0;
          p1 *= xh1;
        }
        if (kind == 0) {
          const int y = y0 + r;
          T t0, t1;
          if constexpr (CACHE_T) {
            t0 = tv[i][0];
            t1 = tv[i][1];
          } else {
            t0 = tmpl[offs(y, x0)];
            t1 = tmpl[offs(y, x0 + 1)];
          }
          z = mk(g0 ? (T)(p0 * (double)t0) : (T)0, g1 ? (T)(p1 * (double)t1) : (T)0);
          if (b == 0 && y < ny) {
            // G_R R itself into the frame padded by w (the template-background
            // block's excluded-pixel sums read it; kb_pad_kernel clears the border)
            T* g = ws_at<T>(PS, pr, O.kbgrp) + (int64_t)(y + w) * (nx + 2 * w) + w;
            if (x0 < nx) g[x0] = z.x;
            if (x0 + 1 < nx) g[x0 + 1] = z.y;
          }
        } else
          z = mk(g0 ? (T)p0 : (T)0, g1 ? (T)p1 : (T)0);
      }
      buf[lds.at(r, j)] = z;
    }
    __syncthreads();
    fft_run<T, NMAX, THREADS, false, true, true, LGH, 4, decltype(lds), decltype(lds), ROW_RPAD>(buf, RB, tw, lds,
                                                                                                 lds);
    __syncthreads();
    // split and write: a thread forms both values of one (column pair, row)
    // and stores them together; consecutive threads take consecutive rows of
    // one column pair, whose RB rows form one contiguous segment
    cplx<T>* Ub = U + (int64_t)b * pstride;
    auto split = [&](int r, int k) -> cplx<T> {
      const cplx<T> zk = buf[lds.at(r, k)];
      const cplx<T> zm = conjg(buf[lds.at(r, (H - k) & (H - 1))]);
      if (k == 0) return mk(zk.x + zk.y, zk.x - zk.y);   // E(0) = Re Z0, O(0) = Im Z0: (X(0), X(H))
      const cplx<T> e2 = zk + zm;                        // 2 E
      const cplx<T> o2 = rot90<T, false>(zk - zm);       // 2 O = -i (Z - conj Z(H-k))
      const cplx<T> t = twid<T, false>(tw, k << twsx);
      return scale(e2 + t * o2, (T)0.5);
    };
#pragma unroll 4
    for (int i = 0; i < NPT / 2; ++i) {
      const int e = tid + i * THREADS;
      const int c = e / RB;
      const int r = e - c * RB;
      const int y = y0 + r;
      if (y >= ny) continue;
      const cplx<T> o0 = split(r, 2 * c), o1 = split(r, 2 * c + 1);
      cplx<T>* dst = Ub + ((int64_t)c * Py + y) * 2;
      if constexpr (sizeof(T) == sizeof(float)) {
        *reinterpret_cast<float4*>(dst) = make_float4(o0.x, o0.y, o1.x, o1.y);
      } else {
        dst[0] = o0;
        dst[1] = o1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// col_fwd: y-weight, FFT along y, residue-major write of every output plane
// ---------------------------------------------------------------------------
// Block = (column pair c, base b).  The pair block of Ub[b] (two columns,
// rows past ny zero) is read from HBM once, into the registers of the first
// transform pass: thread j < 2 Py / R0 holds the R0 inputs y = jj + r Py/R0
// of butterfly jj of column kb (j = kb Py/R0 + jj).  For each output plane o
// built from base b (weight yh^q) the first pass weights those registers,
// applies its radix-R0 DFT (no twiddles: Ns = 1) and writes LDS; the later
// passes run in LDS, the last one (radix 16, so its output index is
// ky = k1 + P1 k2 with k1 < P1 = Py/16) placing X(ky) at slot k1*P2 + k2; the
// two columns then leave as one contiguous block of X[o][kx][slot].
//   Pair 0 holds the packed real column pair z = x0 + i xH (DC and Nyquist
// columns) in its column 0: X0(ky) = (Z(ky) + conj Z(-ky))/2 and
// XH(ky) = (Z(ky) - conj Z(-ky))/(2i) go to columns 0 and H; its column 1 is
// written as usual.
template <typename T, int THREADS, int NMAX, int LGPY, int LGM>
__global__ __launch_bounds__(THREADS, sizeof(T) == 4 ? 4 : 2) void col_fwd_kernel(AsmParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const cplx<T>* __restrict__ Ub = ws_at<const cplx<T>>(PS, pr, O.Ub);
  cplx<T>* __restrict__ X = ws_at<cplx<T>>(PS, pr, O.U);
  const cplx<T>* __restrict__ tw = ws_at<const cplx<T>>(PS, pr, sizeof(T) == 4 ? O.tw32 : O.tw64);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int npairs = P.H / 2;           // pairs 0 .. H/2-1
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  if (id >= npairs * (P.nbase - P.base_lo)) return;
  const int b = P.base_lo + id / npairs;
  const int c = id - (b - P.base_lo) * npairs;
  constexpr int lgPy = LGPY;
  constexpr int Py = 1 << LGPY;
  const int H = P.H;
  const cplx<T>* blk = Ub + (int64_t)b * H * Py + (int64_t)c * Py * 2;
  constexpr int lgP1 = lgPy - LG_P2;
  constexpr int P1 = 1 << lgP1;
  const int tid = threadIdx.x;
  // first pass: radix R0 = 2^LGR0 over M0 = Py/R0 butterflies per column,
  // one butterfly per thread
  static_assert(THREADS >= 512 && NMAX >= 2 * Py, "two columns per block");
  constexpr int LGR0 = fft_first_lgr(LGPY, LGM);
  constexpr int R0 = 1 << LGR0;
  constexpr int lgM0 = lgPy - LGR0;
  static_assert((2 << lgM0) <= THREADS, "one first-pass butterfly per thread");
  const bool act = tid < (2 << lgM0);
  const int kb = tid >> lgM0;
  const int jj = tid & ((1 << lgM0) - 1);
  // rows past ny are never written by the row pass: read a valid row and
  // select zero, so that every load is unconditional
  const int jb = act ? jj : 0;
  cplx<T> raw[R0];
#pragma unroll
  for (int r = 0; r < R0; ++r) {
    const int y = jb + (r << lgM0);
    const cplx<T> t = blk[2 * min(y, P.ny - 1) + (kb & 1)];
    raw[r] = (act && y < P.ny) ? t : mk((T)0, (T)0);
  }
  // The last pass (radix 16 = P2, span Ns = P1) hands over ky = i0 + c with
  // i0 < P1 and c = r P1, r < 16, and puts X(ky) at slot k1*P2 + k2 =
  // i0*P2 + r of the LDS buffer (k1 = ky mod P1, k2 = ky / P1).
  static_assert(LGM == LG_P2, "the last column pass must have radix P2");
  auto store_res = [&](int kbo, int i0, int c, cplx<T> v) {
    buf[lds_pad(kbo * Py + (i0 << LG_P2)) + (c >> lgP1)] = v;
  };
  for (int oi = 0; oi < P.base_count[b]; ++oi) {
    const int o = P.out_plane[P.base_first[b] + oi];
    const int q = P.out_q[P.base_first[b] + oi];
    __syncthreads();   // the previous output's copy-out has read the buffer
    if (act) {
      cplx<T> v[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int y = jj + (r << lgM0);
        const T yh = (T)((double)y * P.sy - 1.0);
        T w = (T)1;
        for (int i = 0; i < q; ++i) w *= yh;
        v[r] = scale(raw[r], w);
      }
      dftR<T, R0, false>(v);
#pragma unroll
      for (int r = 0; r < R0; ++r) buf[lds_pad(kb * Py + (jj << LGR0) + r)] = v[r];
    }
    __syncthreads();
    fft_tail<T, NMAX, THREADS, false, true, LGPY, LGR0, LGM, decltype(store_res)>(buf, 2, tw, store_res);
    __syncthreads();
    cplx<T>* Xo = X + (int64_t)o * (H + 1) * Py;
    if (c > 0) {
      // columns 2c, 2c+1 are contiguous: one coalesced block
      cplx<T>* Xc = Xo + (int64_t)(2 * c) * Py;
      for (int e = tid; e < 2 * Py; e += THREADS) Xc[e] = buf[lds_pad(e)];
    } else {
      for (int e = tid; e < 2 * Py; e += THREADS) {
        if (e >= Py) {
          Xo[e] = buf[lds_pad(e)];
          continue;
        }
        // slot e holds ky = k1 + P1 k2 with k1 = e / P2, k2 = e mod P2; -ky sits at slot(-ky)
        const int ky = (e >> LG_P2) + ((e & (P2 - 1)) << lgP1);
        const int km = (Py - ky) & (Py - 1);
        const cplx<T> z = buf[lds_pad(e)];
        const cplx<T> zm = conjg(buf[lds_pad(((km & (P1 - 1)) << LG_P2) + (km >> lgP1))]);
        Xo[e] = scale(z + zm, (T)0.5);
        Xo[(int64_t)H * Py + e] = scale(rot90<T, false>(z - zm), (T)0.5);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// corr: spectral products and pruned inverse along y on the lag rows
// ---------------------------------------------------------------------------
// One block per column kx in [0, H), with the Nyquist column H packed into
// block 0: the columns kx = 0 and kx = H of a real image's 2-D transform are
// conjugate-symmetric in ky, so their lag correlations V_0(j) and V_H(j) are
// real and block 0 forms the single inverse of Z_0 + i Z_H, whose real and
// imaginary parts are V_0 and V_H (row_win_kernel reads them so).  That makes
// the grid H uniform blocks instead of H + 1, with no lone block in a last
// round.  Block 0 stages both columns with half the residue chunk.
// Residues k1 are processed in chunks of C1 (block 0: C1dc); for each chunk
// every staged plane's P2 values X(k1 + P1 k2) are staged in LDS in FP64.  With Z(k2) = conj(X_left(k2)) X_right(k2) and the inner inverse
// DFT F(r) = sum_k2 Z(k2) e^{2 pi i k2 r/P2}, lag row j = jlo + t accumulates
//   V(j) += e^{2 pi i k1 j/Py} F((jlo + t) mod P2).
// The rotation s = jlo mod P2 is a compile-time case of a switch (items are
// sorted by s, so a wave normally takes one case) to keep every register
// index static.  Item i (pair, lag rows) is handled by `lanes` consecutive
// threads that split the residues; at the end the lanes are summed in LDS.
// Products, the inner transform and the accumulation are FP64 in both modes.
// Staged spectra: residue c of plane pl at stage[pl * corr_plane_stride(C1) + c * CORR_RS].
// The padded strides spread the 16-byte reads of a wave, whose lanes take
// different residues and planes, over the LDS banks: 17 complex values per
// residue put the residues c of one plane on consecutive 16-byte slots (mod
// 16), and a plane stride of 9 mod 16 slots keeps the 9 residues that the
// lanes of one item read from overlapping those of the next item's plane
// (neighbouring items mostly read neighbouring planes).
constexpr int CORR_RS = P2 + 1;
constexpr int CORR_LB = 8;   // staging loads in flight per thread
constexpr int CORR_RED_ROWS = 10;   // lag rows per part of the lanes' reduction
__host__ __device__ constexpr int corr_plane_stride(int c1) {
  return ((c1 * CORR_RS + 12) & ~15) + 9;
}
// elements of the staged spectra of nst planes (element size esize), rounded
// up to a whole 16 bytes: the chunk's FP64 outer twiddles follow them
__host__ __device__ constexpr int corr_stage_elems(int nst, int per_plane, int esize) {
  return esize == 16 ? nst * per_plane : ((nst * per_plane + 1) & ~1);
}
// complex elements reserved at the start of the correlation kernel's LDS for
// the per-chunk twiddle steps (njlo x jm), rounded up to 256 bytes
__host__ __device__ constexpr int corr_step_elems(int njlo, int jm) { return (njlo * jm + 15) & ~15; }

template <int S, int JM>
__device__ __forceinline__ void corr_accumulate(cplx<double>* acc, const cplx<double>* f,
                                                const cplx<double>* __restrict__ tw) {
  // all JM rows are accumulated (rows past the item's count are never written out);
  // four FMAs per complex multiply-add
#pragma unroll
  for (int t = 0; t < JM; ++t) acc[t] = cmac(acc[t], tw[t], f[(S + t) & (P2 - 1)]);
}

template <typename T, int THREADS, int JM>
__global__ __launch_bounds__(THREADS, 2) void corr_kernel(AsmParams P, PairSet PS, WsOff O, int C1, int C1dc) {
  const int pr = blockIdx.z;
  const cplx<T>* __restrict__ U = ws_at<const cplx<T>>(PS, pr, O.U);
  const cplx<T>* __restrict__ Ut = reinterpret_cast<const cplx<T>*>(PS.tws[pr] + O.U);   // template-side planes
  const CorrItem* __restrict__ items = ws_at<const CorrItem>(PS, pr, O.items);
  cplx<double>* __restrict__ V = ws_at<cplx<double>>(PS, pr, O.V);
  const cplx<double>* __restrict__ twd = ws_at<const cplx<double>>(PS, pr, O.tw64);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // LDS: [twstep: njlo x JM] [stage: spectra, then the chunk's outer twiddles].
  // The lane reduction at the end of a pass of items overlays the stage only,
  // so the steps survive into the next pass.
  cplx<double>* twstep = reinterpret_cast<cplx<double>*>(smem_raw);   // [njlo][JM]
  // the spectra are staged in their input precision (converted to FP64 as
  // they are read): in FP32C that halves the stage, so a chunk holds more
  // residues
  cplx<T>* stage = reinterpret_cast<cplx<T>*>(twstep + corr_step_elems(P.njlo, JM));
  const int kx = blockIdx.x;
  const bool pk = kx == 0;                     // the DC and Nyquist columns, packed
  const int H = P.H;
  const int Py = 1 << P.lgPy;
  const int lgPy = P.lgPy;
  const int P1 = Py >> LG_P2;
  const int tid = threadIdx.x;
  const int nitems = P.nitems;           // item slots, padded so rotation groups start on a wave
  const int lanes = P.corr_lanes;        // threads per item; items never straddle a wave
  const int ipw = 64 / lanes;            // items per wave
  const int nwaves = (nitems + ipw - 1) / ipw;
  const int64_t pstride = (int64_t)(H + 1) * Py;
  const int C = pk ? C1dc : C1;                // residues per chunk of this block
  const int nst = pk ? 2 * P.nstaged : P.nstaged;   // staged planes (block 0: column 0, then column H)
  const int per_plane = corr_plane_stride(C);
  // outer twiddles e^{2 pi i k1 (jlo + t)/Py} of the chunk, per distinct jlo, after the spectra
  cplx<double>* twc = reinterpret_cast<cplx<double>*>(stage + corr_stage_elems(nst, per_plane, (int)sizeof(cplx<T>)));   // [njlo][C][JM]
  // e^{2 pi i C j / Py}: advancing k1 by one chunk multiplies each outer twiddle by it
  for (int e = tid; e < P.njlo * JM; e += THREADS) {
    const int ji = e / JM, t = e - ji * JM;
    const int m = (C * ((int)P.jlo_list[ji] + t)) & (Py - 1);
    twstep[e] = conjg(twd[m << (TW_LOG - lgPy)]);
  }

  for (int wbase = 0; wbase < nwaves; wbase += THREADS / 64) {
    const int wv = wbase + (tid >> 6);
    const int wl = tid & 63;
    const int item_id = wv * ipw + wl / lanes;
    const int lane = wl % lanes;
    const bool active = (wl < ipw * lanes) && (item_id < nitems) && items[min(item_id, nitems - 1)].nj > 0;
    CorrItem it;
    it.left = 0;
    it.right = 0;
    it.jlo = 0;
    it.nj = 0;
    it.vrow = 0;
    if (active) it = items[item_id];
    const int srot = ((int)it.jlo % P2 + P2) % P2;
    cplx<double> acc[JM];
#pragma unroll
    for (int t = 0; t < JM; ++t) acc[t] = mk(0.0, 0.0);

    for (int k1c = 0; k1c < P1; k1c += C) {
      const int nc = min(C, P1 - k1c);
      __syncthreads();
      // spectra: two neighbouring values per load (16 bytes in FP32).  The
      // loads of a batch of CORR_LB per thread are all issued before any is
      // converted and stored, so their latencies overlap.
      const int npr = nc * (P2 / 2);
      const int ntot = nst * npr;
      // plane of element e: floor(e / npr) as the truncation of (e + 1/2) / npr
      // in FP32.  That quotient is at least 1/(2 npr) >= 2^-12 away from an
      // integer (npr <= 8 P1 <= 2048), and FP32 moves it by less than
      // 62 planes x 2^-23 (e < 2^23 is exact in FP32), so the truncation is
      // exact; it replaces two integer divisions per element.
      const float inv_npr = 1.0f / (float)npr;
      auto plane_of = [&](int e) { return (int)(((float)e + 0.5f) * inv_npr); };
      for (int e0 = tid; e0 < ntot; e0 += CORR_LB * THREADS) {
        cplx<T> q[CORR_LB][2];
#pragma unroll
        for (int b = 0; b < CORR_LB; ++b) {
          const int e = min(e0 + b * THREADS, ntot - 1);   // a valid element; the copy is dropped below
          const int pl = plane_of(e);
          const int o = 2 * (e - pl * npr);
          const bool hi = pl >= P.nstaged;                 // block 0: the Nyquist column's planes
          const int col = hi ? H : kx;
          const int sp = pl - (hi ? P.nstaged : 0);        // staged plane -> workspace and plane
          const bool sh = sp < P.nshared;
          // element offsets fit in 32 bits: at most 31 planes of 2049 x 4096
          const cplx<T>* src = (sh ? Ut : U) + (uint32_t)((sh ? sp : sp + P.plane_skip) * (int)pstride +
                                                          col * Py + k1c * P2 + o);
          if constexpr (sizeof(T) == sizeof(float)) {
            const float4 f = *reinterpret_cast<const float4*>(src);
            q[b][0] = mk(f.x, f.y);
            q[b][1] = mk(f.z, f.w);
          } else {
            q[b][0] = src[0];
            q[b][1] = src[1];
          }
        }
#pragma unroll
        for (int b = 0; b < CORR_LB; ++b) {
          const int e = e0 + b * THREADS;
          if (e < ntot) {
            const int pl = plane_of(e);
            const int o = 2 * (e - pl * npr);
            cplx<T>* dst = stage + pl * per_plane + (o >> LG_P2) * CORR_RS + (o & (P2 - 1));
            dst[0] = q[b][0];
            dst[1] = q[b][1];
          }
        }
      }
      // outer twiddles: from the table for the first chunk (Py is a power of two,
      // so the index is the product masked to [0, Py)), then by the FP64 step
      for (int ji = 0; ji < P.njlo; ++ji) {
        const int jlo = P.jlo_list[ji];
        int r0 = tid;
        asm volatile("" : "+v"(r0));
        for (int r = r0; r < C * JM; r += THREADS) {
          const int t = r % JM;
          cplx<double>& w = twc[ji * C * JM + r];
          if (k1c == 0) {
            const int c = r / JM;
            const int m = (c * (jlo + t)) & (Py - 1);
            w = conjg(twd[m << (TW_LOG - lgPy)]);
          } else {
            w = w * twstep[ji * JM + t];
          }
        }
      }
      __syncthreads();
      if (!active) continue;
      // the item lane is formed again per chunk (from an opaque thread index)
      // instead of being held across the staging
      int tl = tid;
      asm volatile("" : "+v"(tl));
      for (int c = (tl & 63) % lanes; c < nc; c += lanes) {
        const int k1 = k1c + c;
        const cplx<T>* xa = stage + it.left * per_plane + c * CORR_RS;
        const cplx<T>* xb = stage + it.right * per_plane + c * CORR_RS;
        auto d64 = [](cplx<T> v) { return mk((double)v.x, (double)v.y); };
        cplx<double> z[P2];
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) z[k2] = cmulc(d64(xa[k2]), d64(xb[k2]));
        if (pk) {
          // + i Z_H: the Nyquist column's product on the imaginary axis
          const cplx<T>* ya = xa + P.nstaged * per_plane;
          const cplx<T>* yb = xb + P.nstaged * per_plane;
#pragma unroll
          for (int k2 = 0; k2 < P2; ++k2) z[k2] = z[k2] + rot90<double, true>(cmulc(d64(ya[k2]), d64(yb[k2])));
        }
        dft16<double, true>(z);
        const cplx<double>* twt = twc + ((int)it.jidx * C + c) * JM;
        (void)k1;
        switch (srot) {
#define CORR_CASE(SV) \
  case SV:            \
    corr_accumulate<SV, JM>(acc, z, twt); \
    break;
          CORR_CASE(0) CORR_CASE(1) CORR_CASE(2) CORR_CASE(3) CORR_CASE(4) CORR_CASE(5) CORR_CASE(6) CORR_CASE(7)
          CORR_CASE(8) CORR_CASE(9) CORR_CASE(10) CORR_CASE(11) CORR_CASE(12) CORR_CASE(13) CORR_CASE(14)
          CORR_CASE(15)
#undef CORR_CASE
        }
      }
    }
    // sum the lanes of each item through LDS, CORR_RED_ROWS lag rows at a time
    // (over the staged spectra, which are dead until the next pass restages them)
    cplx<double>* red = reinterpret_cast<cplx<double>*>(stage);
    constexpr int HALF = CORR_RED_ROWS;
#pragma unroll
    for (int h = 0; h < (JM + HALF - 1) / HALF; ++h) {
      // the thread index and the item go through an empty asm, so that their
      // addresses and fields are formed here rather than hoisted to the
      // kernel's start and held (spilled) across the residue loop
      int tr = tid;
      asm volatile("" : "+v"(tr));
      const int ir = min((wbase + (tr >> 6)) * ipw + (tr & 63) / lanes, nitems - 1);   // item_id
      cplx<double>* mine = red + tr * HALF;
      __syncthreads();
      if (active) {
#pragma unroll
        for (int t = 0; t < HALF; ++t) {
          const int tt = h * HALF + t;
          if (tt < JM) mine[t] = acc[tt];
        }
      }
      __syncthreads();
      if (active && lane == 0) {
        const CorrItem iv = items[ir];
        for (int t = 0; t < HALF; ++t) {
          const int tt = h * HALF + t;
          if (tt >= iv.nj) break;
          if (tt < iv.skip) continue;
          cplx<double> sum = mk(0.0, 0.0);
          for (int l = 0; l < lanes; ++l) sum = sum + mine[l * HALF + t];
          V[(int64_t)kx * P.vrows + iv.vrow + tt] = sum;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// direct route: lag windows as plain sums over the frame (no transforms)
// ---------------------------------------------------------------------------
// win[out + (dx + hw)] = sum_y,x X_l(y, x) X_r(y + dy, x + dx) for one window
// row (pair, dy), dx in [-hw, hw]; X_r is zero outside the frame.  Planes:
// 0..nK-1 the template planes m_a G_R R, nK..nK+nB-1 the background planes
// G m_b, nK+nB the masked science image G S, all evaluated on the fly in
// FP64.  One block per (window row, band of DIR_BAND image rows); partial
// sums per band, summed over the bands in a fixed order by dir_reduce_kernel.
struct DirectRow {
  int16_t left, right;   // planes
  int16_t hw, dy;        // lag half-width along x, lag along y
  int32_t out;           // offset of the window row in `win`
};
constexpr int DIR_XB = 4;       // consecutive x per thread (register reuse of the right row)
constexpr int DIR_HWMAX = 18;   // lag half-widths up to 2w with w <= 9
constexpr int DIR_BAND = 64;    // image rows per block
constexpr int DIR_MAX_NX = 1024;
constexpr int DIR_MIN_TPR = 4;

template <typename T>
__device__ __forceinline__ double plane_value(const AsmParams& P, int pl, int y, int x, const T* __restrict__ sci,
                                              const T* __restrict__ tmpl, const uint8_t* __restrict__ mask) {
  if (y < 0 || y >= P.ny || x < 0 || x >= P.nx) return 0.0;
  const int64_t o = (int64_t)y * P.ld + x;
  if (mask != nullptr && mask[o] != 0) return 0.0;
  if (pl < P.nk) {
    const int w = P.w;
    if (y < w || y >= P.ny - w || x < w || x >= P.nx - w) return 0.0;
    const double xh = (double)x * P.sx - 1.0, yh = (double)y * P.sy - 1.0;
    return ipow(xh, P.kpoly.px[pl]) * ipow(yh, P.kpoly.qy[pl]) * (double)tmpl[o];
  }
  if (pl < P.nk + P.nb) {
    const int b = pl - P.nk;
    const double xh = (double)x * P.sx - 1.0, yh = (double)y * P.sy - 1.0;
    return ipow(xh, P.bpoly.px[b]) * ipow(yh, P.bpoly.qy[b]);
  }
  return (double)sci[o];
}

template <typename T, int THREADS>
__global__ __launch_bounds__(THREADS) void direct_win_kernel(AsmParams P, PairSet PS, WsOff O, int nwin) {
  const int pr = blockIdx.z;
  const T* __restrict__ sci = static_cast<const T*>(PS.sci[pr]);
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  const DirectRow* __restrict__ rows = ws_at<const DirectRow>(PS, pr, O.drows);
  double* __restrict__ part = ws_at<double>(PS, pr, O.U);   // per-band partial sums
  constexpr int NACC = 2 * DIR_HWMAX + 1;
  constexpr int MAXRPP = THREADS / DIR_MIN_TPR;
  // rpp staged rows of tpr * DIR_XB + 2 hw values: at most THREADS * DIR_XB + MAXRPP * 2 DIR_HWMAX
  __shared__ double rbuf[THREADS * DIR_XB + MAXRPP * 2 * DIR_HWMAX];
  __shared__ double red[THREADS / 64][NACC];
  const DirectRow R = rows[blockIdx.x];
  const int hw = R.hw;
  const int tpr = P.dir_tpr;
  const int rpp = THREADS / tpr;
  const int rstride = tpr * DIR_XB + 2 * hw;
  const int tid = threadIdx.x;
  const int sub = tid / tpr, tx = tid - sub * tpr;
  const int y_begin = blockIdx.y * DIR_BAND;
  const int y_end = min(P.ny, y_begin + DIR_BAND);
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = 0.0;

  for (int yb = y_begin; yb < y_end; yb += rpp) {
    const int y = yb + sub;
    __syncthreads();   // the previous rows have been read
    double* rr = rbuf + sub * rstride;
    for (int e = tx; e < rstride; e += tpr)
      rr[e] = (y < y_end) ? plane_value<T>(P, R.right, y + R.dy, e - hw, sci, tmpl, mask) : 0.0;
    __syncthreads();
    if (y >= y_end) continue;
    const int x0 = tx * DIR_XB;
    double xl[DIR_XB];
#pragma unroll
    for (int k = 0; k < DIR_XB; ++k) xl[k] = plane_value<T>(P, R.left, y, x0 + k, sci, tmpl, mask);
    // rr[x0 + j] = X_r(y + dy, x0 + j - hw); x = x0 + k pairs with lag dx = j - k - hw
    const double* rx = rr + x0;
#pragma unroll
    for (int j = 0; j < NACC + DIR_XB - 1; ++j) {
      if (j < 2 * hw + DIR_XB) {
        const double v = rx[j];
#pragma unroll
        for (int k = 0; k < DIR_XB; ++k) {
          const int d = j - k;
          if (d >= 0 && d < NACC) {
            if (d <= 2 * hw) acc[d] += xl[k] * v;
          }
        }
      }
    }
  }
  // block sum of every lag: waves by shuffles, then the waves in order
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int d = 0; d < NACC; ++d) {
    if (d <= 2 * hw) {
      double v = acc[d];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[wave][d] = v;
    }
  }
  __syncthreads();
  if (tid <= 2 * hw) {
    double v = 0.0;
    for (int wv = 0; wv < THREADS / 64; ++wv) v += red[wv][tid];
    part[(int64_t)blockIdx.y * nwin + R.out + tid] = v;
  }
}

// win[i] = sum over bands of part[band][i], bands in order
__global__ void dir_reduce_kernel(PairSet PS, WsOff O, int nband, int nwin) {
  const int pr = blockIdx.z;
  const double* __restrict__ part = ws_at<const double>(PS, pr, O.U);
  double* __restrict__ win = ws_at<double>(PS, pr, O.win);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nwin) return;
  double v = 0.0;
  for (int b = 0; b < nband; ++b) v += part[(int64_t)b * nwin + i];
  win[i] = v;
}

// ---------------------------------------------------------------------------
// MFMA route: lag windows as FP64 matrix-core products (no transforms)
// ---------------------------------------------------------------------------
// For a source row y' of the right plane X_r and the 16 lags dy of a tile,
//   C(dy, dx) += sum_x X_l(y' - dy, x) X_r(y', x + dx)
// is the product of the 16 x K matrix A[dy][x] = X_l(y' - dy, x) (rows of the
// left plane) and the K x 16 Hankel matrix B[x][dx] = X_r(y', x + dx), run on
// v_mfma_f64_16x16x4f64 with K = 4 pixels per instruction and every dx tile
// of the window sharing the A operand.  Summing over y' and x gives the lag
// window itself (z = (y' - dy, x) runs over the frame).
// A block owns one (pair, dy tile), one chunk of MFMA_XC columns x and one
// band of source rows y'.  It sweeps the band row by row: the 16 left-plane
// rows of the tile sit in an LDS ring (one new row enters per step, the row
// of the largest y), the right-plane row with its +-hw margin beside it, and
// the next step's values are loaded into registers while the matrix cores
// run.  The four waves split the chunk's columns, each accumulating every dx
// tile; at the end the waves' tiles are summed through LDS and the block
// writes one partial window per (chunk, band), summed over chunks and bands
// in a fixed order by dir_reduce_kernel.  Operand layout of the MFMA: lane l
// gives A[l%16][l/16] and B[l/16][l%16]; register r of lane l holds
// D[l/16 + 4r][l%16].
struct MfmaTile {
  int16_t left, right;   // planes
  int16_t hw, dy0;       // lag half-width; the tile's lags are dy0 .. dy0 + 15
  int32_t out;           // offset of the pair's window ((2hw+1) x (2hw+1), dy-major) in `win`
};
constexpr int MFMA_XC = 256;                    // columns per block, 64 per wave
constexpr int MFMA_MAXT = 4;                    // dx tiles: 2 hw + 1 <= 64
constexpr int MFMA_RS = MFMA_XC + 4;            // ring row stride (doubles): spreads the 16 rows over the banks
constexpr int MFMA_XR = MFMA_XC + 2 * 32;       // right-plane row with its margin (hw <= 31)
constexpr int MFMA_THREADS = 256;
typedef double mf64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(MFMA_THREADS) void mfma_win_kernel(AsmParams P, PairSet PS, WsOff O, int nwin,
                                                                int nxc, int band) {
  const int pr = blockIdx.z;
  const T* __restrict__ sci = static_cast<const T*>(PS.sci[pr]);
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  const MfmaTile Tl = ws_at<const MfmaTile>(PS, pr, O.mtiles)[blockIdx.x];
  double* __restrict__ part = ws_at<double>(PS, pr, O.U);   // [chunk, band] partial windows
  __shared__ double ring[16 * MFMA_RS];
  __shared__ double xr[MFMA_XR];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int xc = (int)blockIdx.y % nxc, yb = (int)blockIdx.y / nxc;
  const int x0 = xc * MFMA_XC;
  const int ylo = yb * band, yhi = min(P.ny, ylo + band);
  const int hw = Tl.hw, dy0 = Tl.dy0;
  const int ndx = (2 * hw + 1 + 15) / 16;
  const int nxr = MFMA_XC + 2 * hw;               // right-plane values per step
  // prologue: the 15 older rows of the first step's tile (rows ylo - dy0 - 15 .. ylo - dy0 - 1)
  for (int e = tid; e < 15 * MFMA_XC; e += MFMA_THREADS) {
    const int m = e / MFMA_XC + 1, j = e - (m - 1) * MFMA_XC;
    const int row = ylo - dy0 - m;
    ring[(row & 15) * MFMA_RS + j] = plane_value<T>(P, Tl.left, row, x0 + j, sci, tmpl, mask);
  }
  // the values entering at step y: ring row y - dy0 and the right-plane row y
  double av = 0.0, xv0 = 0.0, xv1 = 0.0;
  auto fetch = [&](int y) {
    av = plane_value<T>(P, Tl.left, y - dy0, x0 + tid, sci, tmpl, mask);
    xv0 = plane_value<T>(P, Tl.right, y, x0 - hw + tid, sci, tmpl, mask);
    xv1 = tid + MFMA_THREADS < nxr ? plane_value<T>(P, Tl.right, y, x0 - hw + tid + MFMA_THREADS, sci, tmpl, mask)
                                   : 0.0;
  };
  auto store = [&](int y) {
    ring[((y - dy0) & 15) * MFMA_RS + tid] = av;
    xr[tid] = xv0;
    if (tid + MFMA_THREADS < nxr) xr[tid + MFMA_THREADS] = xv1;
  };
  for (int e = tid; e < MFMA_XR; e += MFMA_THREADS) xr[e] = 0.0;   // the margin past nxr stays zero
  __syncthreads();
  if (ylo < yhi) {
    fetch(ylo);
    store(ylo);
  }
  mf64x4 acc[MFMA_MAXT];
#pragma unroll
  for (int t = 0; t < MFMA_MAXT; ++t) acc[t] = mf64x4{0.0, 0.0, 0.0, 0.0};
  const int xw = wave * (MFMA_XC / 4);            // this wave's first column in the chunk
  for (int y = ylo; y < yhi; ++y) {
    __syncthreads();
    if (y + 1 < yhi) fetch(y + 1);                // in flight while the matrix cores run
    const double* arow = ring + ((y - dy0 - lr) & 15) * MFMA_RS + xw + lk;
    const double* brow = xr + xw + lk + lr;
#pragma unroll 4
    for (int ks = 0; ks < MFMA_XC / 16; ++ks) {
      const double a = arow[4 * ks];
#pragma unroll
      for (int t = 0; t < MFMA_MAXT; ++t)
        if (t < ndx) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, brow[4 * ks + 16 * t], acc[t], 0, 0, 0);
    }
    __syncthreads();
    if (y + 1 < yhi) store(y + 1);
  }
  // sum the four waves' tiles through LDS (over the ring), then write the partial window
  __syncthreads();
  double* red = ring;   // [wave][t][16 x 16]
#pragma unroll
  for (int t = 0; t < MFMA_MAXT; ++t)
    if (t < ndx)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * MFMA_MAXT + t) * 256 + (lk + 4 * r) * 16 + lr] = acc[t][r];
  __syncthreads();
  const int h = 2 * hw + 1;
  double* dst = part + (int64_t)blockIdx.y * nwin + Tl.out;
  for (int t = 0; t < ndx; ++t) {
    const int m = tid >> 4, n = tid & 15;
    const int dy = dy0 + m, dx = -hw + 16 * t + n;
    const double v = (red[(0 * MFMA_MAXT + t) * 256 + tid] + red[(1 * MFMA_MAXT + t) * 256 + tid]) +
                     (red[(2 * MFMA_MAXT + t) * 256 + tid] + red[(3 * MFMA_MAXT + t) * 256 + tid]);
    if (dy <= hw && dx <= hw) dst[(dy + hw) * h + (dx + hw)] = v;
  }
}

// ---------------------------------------------------------------------------
// row_win: inverse along x restricted to the lag columns, FP64
// ---------------------------------------------------------------------------
// C(j, i) = 1/(Py Px) [ V(j,0) + (-1)^i V(j,H) + 2 Re sum_{kx=1}^{H-1} V(j,kx) e^{2 pi i kx i / Px} ]
// One wave per V row (nrows rows); the window half-width of the row's pair is hw.
struct WinRow {
  int32_t vrow;     // row of V
  int32_t out;      // offset of the first window value of this row in `win`
  int32_t hw;       // half-width of the lag columns
};

template <int THREADS, int IMAX>
__global__ __launch_bounds__(THREADS) void row_win_kernel(AsmParams P, PairSet PS, WsOff O, int nrows) {
  const int pr = blockIdx.z;
  const cplx<double>* __restrict__ V = ws_at<const cplx<double>>(PS, pr, O.V);
  const WinRow* __restrict__ rows = ws_at<const WinRow>(PS, pr, O.wrows);
  double* __restrict__ win = ws_at<double>(PS, pr, O.win);
  const cplx<double>* __restrict__ twd = ws_at<const cplx<double>>(PS, pr, O.tw64);
  static_assert(THREADS == 64, "one wave per window row");
  constexpr int HMAX = (IMAX - 1) / 2;   // largest half-width
  // V is stored [kx][vrow]: neighbouring rows share every cache line they
  // read, so they run on one XCD at about the same time (xcd_remap)
  const int rid = xcd_remap(blockIdx.x, gridDim.x);
  if (rid >= nrows) return;
  const WinRow R = rows[rid];
  const int H = P.H;
  const int lgPx = P.lgPx;
  const int tid = threadIdx.x;
  const int hw = R.hw;
  // With m = i - hw in [-hw, hw] and theta = 2 pi kx / Px:
  //   sum_kx w_kx Re(V e^{i theta m}) = Cc(|m|) - sgn(m) Cs(|m|),
  //   Cc(m) = sum w_kx Re V cos(theta m),  Cs(m) = sum w_kx Im V sin(theta m),
  // (w = 1 at kx = 0 and H, 2 between), so only m = 0 .. hw are accumulated.
  double cc[HMAX + 1], cs[HMAX + 1];
#pragma unroll
  for (int m = 0; m <= HMAX; ++m) cc[m] = cs[m] = 0.0;
  for (int kx = tid; kx < H; kx += THREADS) {
    const cplx<double> v = V[(int64_t)kx * P.vrows + R.vrow];
    if (kx == 0) {
      // the packed DC (real part) and Nyquist (imaginary part) columns: real
      // values with weight 1; at the Nyquist column cos(pi m) = (-1)^m
      double sg = 1.0;
#pragma unroll
      for (int m = 0; m <= HMAX; ++m) {
        if (m <= hw) {
          cc[m] += v.x + sg * v.y;
          sg = -sg;
        }
      }
    } else {
      // e^{i theta m} by FP64 recurrence from m = 0
      const cplx<double> st = conjg(twd[kx << (TW_LOG - lgPx)]);
      const double vr = 2.0 * v.x, vi = 2.0 * v.y;
      cplx<double> t = mk(1.0, 0.0);
#pragma unroll
      for (int m = 0; m <= HMAX; ++m) {
        if (m <= hw) {
          cc[m] += vr * t.x;
          cs[m] += vi * t.y;
          t = t * st;
        }
      }
    }
  }
  const double norm = 1.0 / ((double)(1 << P.lgPy) * (double)(2 * H));
#pragma unroll
  for (int m = 0; m <= HMAX; ++m) {
    if (m <= hw) {
      double c = cc[m], d = cs[m];
      for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        d += __shfl_down(d, off, 64);
      }
      if (tid == 0) {
        win[R.out + hw + m] = (c - d) * norm;
        if (m > 0) win[R.out + hw - m] = (c + d) * norm;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// moments: per-row FP64 sums for the background block, and the non-finite scan
// ---------------------------------------------------------------------------
// mom[y][p]          = sum_x G xh^p,      p in [0, 2DB]
// mom[y][2DB+1+p]    = sum_x G S xh^p,    p in [0, DB]
// mom[y][3DB+2+p]    = sum_x G_R R xh^p,  p in [0, DK+DB]   (G_R R: the template side, w-strip excluded)
// Per-row moments, the polynomial degrees DB (background) and DK (kernel)
// fixed at compile time so that only the powers in use are summed:
// G xh^p (p <= 2 DB), G S xh^p (p <= DB), G_R R xh^p (p <= DK + DB); the
// row's count of excluded pixels; a flag for non-finite inputs.
template <typename T, int THREADS, int DB, int DK>
__global__ __launch_bounds__(THREADS) void moments_kernel(AsmParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const T* __restrict__ sci = static_cast<const T*>(PS.sci[pr]);
  const T* __restrict__ tmpl = static_cast<const T*>(PS.tmpl[pr]);
  const uint8_t* __restrict__ mask = PS.mask[pr];
  double* __restrict__ mom = ws_at<double>(PS, pr, O.mom);
  int* __restrict__ nonfinite = ws_at<int>(PS, pr, O.flags) + 1;
  constexpr int NG = 2 * DB + 1;
  constexpr int NS = DB + 1;
  constexpr int NA = DK + DB + 1;
  constexpr int NM = NG + NS + NA;       // the row's moments, in this order (the layout of mom)
  constexpr int NP = NG > NA ? NG : NA;  // powers of xh in use
  constexpr int NW = THREADS / 64;
  __shared__ double red[NW][NM];
  const int y = blockIdx.x;
  const int tid = threadIdx.x;
  const bool inty = y >= P.w && y < P.ny - P.w;
  double acc[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) acc[i] = 0.0;
  bool bad = false;
  const T* srow = sci + (int64_t)y * P.ld;
  const T* rrow = tmpl + (int64_t)y * P.ld;
  const uint8_t* mrow = mask ? mask + (int64_t)y * P.ld : nullptr;
#pragma unroll 4
  for (int x = tid; x < P.nx; x += THREADS) {
    const T sv = srow[x];
    const T rv = rrow[x];
    const bool good = (mrow == nullptr) || (mrow[x] == 0);
    bad |= !isfinite(sv) || !isfinite(rv);
    const double g = good ? 1.0 : 0.0;
    const double s = good ? (double)sv : 0.0;
    const double r = (good && inty && x >= P.w && x < P.nx - P.w) ? (double)rv : 0.0;
    const double xh = (double)x * P.sx - 1.0;
    double pw = 1.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p < NG) acc[p] += g * pw;
      if (p < NS) acc[NG + p] += s * pw;
      if (p < NA) acc[NG + NS + p] += r * pw;
      pw *= xh;
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][i] = v;
  }
  __syncthreads();
  if (tid < NM) {
    double v = 0.0;
    for (int k = 0; k < NW; ++k) v += red[k][tid];
    mom[(int64_t)y * P.nmom + tid] = v;
    // sum_x G is the row's count of good pixels: the rest are excluded
    if (tid == 0) ws_at<int>(PS, pr, O.omcnt)[y] = P.nx - (int)(v + 0.5);
  }
}

// (p, q) of monomial c in the graded order (degree d = p + q, then q ascending)
__host__ __device__ inline void mono_of(int c, int* p, int* q) {
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= c) ++d;
  *q = c - d * (d + 1) / 2;
  *p = d - *q;
}
__host__ __device__ constexpr int mono_index(int p, int q) { return (p + q) * (p + q + 1) / 2 + q; }

// Omega_BB, beta_B and the template moments mu(p, q) = sum G_R R xh^p yh^q
// (p + q <= DK + DB) from the per-row moments: one block per output, fixed
// summation order (deterministic).
template <int THREADS>
__global__ __launch_bounds__(THREADS) void moments_reduce_kernel(AsmParams P, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ mom = ws_at<const double>(PS, pr, O.mom);
  double* __restrict__ obb = ws_at<double>(PS, pr, O.obb);
  double* __restrict__ bb = ws_at<double>(PS, pr, O.bb);
  double* __restrict__ amom = ws_at<double>(PS, pr, O.amom);
  __shared__ double red[THREADS / 64];
  const int tid = threadIdx.x;
  const int nb = P.nb;
  const int nG = 2 * P.db + 1;
  const int q = blockIdx.x;
  double acc = 0.0;
  int col, e;
  if (q < nb * nb) {
    const int b = q / nb, c = q % nb;
    col = P.bpoly.px[b] + P.bpoly.px[c];
    e = P.bpoly.qy[b] + P.bpoly.qy[c];
  } else if (q < nb * nb + nb) {
    const int b = q - nb * nb;
    col = nG + P.bpoly.px[b];
    e = P.bpoly.qy[b];
  } else {
    int pc, qc;
    mono_of(q - nb * nb - nb, &pc, &qc);
    col = nG + (P.db + 1) + pc;
    e = qc;
  }
#pragma unroll 4
  for (int y = tid; y < P.ny; y += THREADS) {
    const double yh = (double)y * P.sy - 1.0;
    acc += ipow(yh, e) * mom[(int64_t)y * P.nmom + col];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int k = 0; k < THREADS / 64; ++k) v += red[k];
    if (q < nb * nb) obb[q] = v;
    else if (q < nb * nb + nb) bb[q - nb * nb] = v;
    else amom[q - nb * nb - nb] = v;
  }
}

// ---------------------------------------------------------------------------
// gather: dense Omega (both triangles) and beta
// ---------------------------------------------------------------------------
struct GatherParams {
  int n, nkk, L, w, nk, nb;
  int kb_dense;                 // Omega_KB from kbd[(a,u) nB + b] (transform route) instead of windows
  int kk_off[MAX_NB * MAX_NB];  // window offset of C_ab for a <= b (index a*nk + b)
  int kb_off[MAX_NB * MAX_NB];  // window offset of corr(A_a, G m_b) (index a*nb + b)
  int ks_off[MAX_NB];           // window offset of corr(A_a, S_m)
};

__global__ void gather_kernel(GatherParams G, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ win = ws_at<const double>(PS, pr, O.win);
  const double* __restrict__ obb = ws_at<const double>(PS, pr, O.obb);
  const double* __restrict__ bb = ws_at<const double>(PS, pr, O.bb);
  double* __restrict__ omega = ws_at<double>(PS, pr, O.omega);
  double* __restrict__ beta = ws_at<double>(PS, pr, O.beta);
  const double* __restrict__ kbd = ws_at<const double>(PS, pr, O.kbd);
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
      v = G.kb_dense ? kbd[(int64_t)r * G.nb + b] : win[G.kb_off[a * G.nb + b] + ur];
    } else if (c < G.nkk) {
      const int a = c / L2, uc = c - a * L2;
      const int b = r - G.nkk;
      v = G.kb_dense ? kbd[(int64_t)c * G.nb + b] : win[G.kb_off[a * G.nb + b] + uc];
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

// beta alone (a build of the right-hand side only: Omega is the sharing pair's)
__global__ void gather_beta_kernel(GatherParams G, PairSet PS, WsOff O) {
  const int pr = blockIdx.z;
  const double* __restrict__ win = ws_at<const double>(PS, pr, O.win);
  const double* __restrict__ bb = ws_at<const double>(PS, pr, O.bb);
  double* __restrict__ beta = ws_at<double>(PS, pr, O.beta);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= G.n) return;
  const int L2 = G.L * G.L;
  if (r < G.nkk) {
    const int a = r / L2, ur = r - a * L2;
    beta[r] = win[G.ks_off[a] + ur];
  } else {
    beta[r] = bb[r - G.nkk];
  }
}

// The non-finite flag of every pair of the group, cleared before a build.
__global__ void clear_nonfinite_kernel(PairSet PS, WsOff O) {
  if (threadIdx.x == 0) ws_at<int>(PS, blockIdx.z, O.flags)[1] = 0;
}

}  // namespace sfft
