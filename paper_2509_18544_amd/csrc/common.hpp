// Device-side building blocks shared by the SFFT kernels (gfx950, wave64).
//
//  * cplx<T>     -- complex value of float or double with the few operations
//                   the transforms need.
//  * dft2/4/8/16 -- in-register DFTs of size 2..16 (forward: exp(-2 pi i jk/R),
//                   inverse: exp(+2 pi i jk/R), unnormalised).
//  * fft_pass / fft_run / fft_rest -- radix-R passes of a self-sorting
//                   (Stockham) FFT on a batch of power-of-two transforms, with
//                   the first and last pass reading and writing through
//                   accessors and the passes in between in place in LDS.
//
// Twiddle factors come from a table tw[m] = exp(-2 pi i m / TW_N) computed in
// FP64 on the host and rounded once to T; the inverse direction conjugates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfft {

constexpr int TW_LOG = 12;            // twiddle table length 4096 = largest FFT size
constexpr int TW_N = 1 << TW_LOG;
constexpr int MAX_LOG_P = 12;         // frames up to 4096 pixels per side
constexpr int MIN_LOG_P = 6;          // FFT sizes are at least 64

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cplx<T> conjg(cplx<T> a) { return mk(a.x, -a.y); }
// conj(a) * b
// acc + a * b as four fused multiply-adds (the plain expression rounds the
// product before the sum and costs two more instructions)
template <typename T>
__device__ __forceinline__ cplx<T> cmac(cplx<T> acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}

template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// multiply by -i (forward quarter turn) or +i (inverse quarter turn)
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}
// Twiddle exp(-+2 pi i m / TW_N) from the forward table.  FP64 transforms read
// the whole table; FP32 transforms read only its first half tw[0 .. TW_N/2)
// (16 KB, friendlier to L1) and use exp(-2 pi i (m + TW_N/2) / TW_N) = -tw[m],
// an exact sign flip.
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> twid(const cplx<T>* __restrict__ tw, int m) {
  if constexpr (sizeof(T) == sizeof(double)) {
    const cplx<T> t = tw[(uint32_t)m & (uint32_t)(TW_N - 1)];
    return INV ? conjg(t) : t;
  } else {
    const cplx<float> t = tw[(uint32_t)m & (uint32_t)(TW_N / 2 - 1)];
    const uint32_t flip = ((uint32_t)m & (uint32_t)(TW_N / 2)) << (31 - (TW_LOG - 1));
    const uint32_t xr = __float_as_uint(t.x) ^ flip;
    const uint32_t yr = __float_as_uint(t.y) ^ flip ^ (INV ? 0x80000000u : 0u);
    return cplx<T>{__uint_as_float(xr), __uint_as_float(yr)};
  }
}

// ---------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2, cplx<T>& a3) {
  cplx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot90<T, INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>* v) { dft4<T, INV>(v[0], v[1], v[2], v[3]); }

// multiply by exp(-+2 pi i k / 8) for k = 1, 2, 3
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> w8_1(cplx<T> a) {
  const T r = (T)0.70710678118654752440;
  // forward: (1 - i)/sqrt2 ; inverse: (1 + i)/sqrt2
  return INV ? mk(r * (a.x - a.y), r * (a.x + a.y)) : mk(r * (a.x + a.y), r * (a.y - a.x));
}
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> w8_3(cplx<T> a) {
  const T r = (T)0.70710678118654752440;
  // forward: (-1 - i)/sqrt2 ; inverse: (-1 + i)/sqrt2
  return INV ? mk(-r * (a.x + a.y), r * (a.x - a.y)) : mk(r * (a.y - a.x), -r * (a.x + a.y));
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  o1 = w8_1<T, INV>(o1);
  o2 = rot90<T, INV>(o2);
  o3 = w8_3<T, INV>(o3);
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + o1;
  v[5] = e1 - o1;
  v[2] = e2 + o2;
  v[6] = e2 - o2;
  v[3] = e3 + o3;
  v[7] = e3 - o3;
}

// 16-point DFT as 4 x 4: DFT4 over stride-4 subsequences, twiddle w16^(m k1), DFT4 over m.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T>* v) {
  const T c1 = (T)0.92387953251128675613;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977173;  // sin(pi/8)
  const T r = (T)0.70710678118654752440;
  cplx<T> d[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    d[m][0] = v[m];
    d[m][1] = v[m + 4];
    d[m][2] = v[m + 8];
    d[m][3] = v[m + 12];
    dft4<T, INV>(d[m][0], d[m][1], d[m][2], d[m][3]);
  }
  // twiddles w16^(m*k1), w16 = exp(-+ 2 pi i / 16)
  const T sg = INV ? (T)1 : (T)-1;
  // m = 1: k1 = 1, 2, 3 -> w^1, w^2, w^3
  d[1][1] = d[1][1] * mk(c1, sg * s1);
  d[1][2] = d[1][2] * mk(r, sg * r);
  d[1][3] = d[1][3] * mk(s1, sg * c1);
  // m = 2: w^2, w^4, w^6
  d[2][1] = d[2][1] * mk(r, sg * r);
  d[2][2] = rot90<T, INV>(d[2][2]);
  d[2][3] = d[2][3] * mk(-r, sg * r);
  // m = 3: w^3, w^6, w^9
  d[3][1] = d[3][1] * mk(s1, sg * c1);
  d[3][2] = d[3][2] * mk(-r, sg * r);
  d[3][3] = d[3][3] * mk(-c1, -sg * s1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cplx<T> a0 = d[0][k1], a1 = d[1][k1], a2 = d[2][k1], a3 = d[3][k1];
    dft4<T, INV>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}
// ---------------------------------------------------------------------------
// Stockham passes with compile-time sizes
// ---------------------------------------------------------------------------
// LDS buffers used by these passes are padded by one element every 16
// (lds_pad) so that the strided Stockham stores do not pile onto one bank.
// Transform b of a batch starts at element b * N of the unpadded index space.
// Every size (N = 2^LGN, the radix, the span Ns already transformed) is a
// template parameter, so that the index arithmetic folds into constants and
// the LDS offsets into the instructions' immediate fields.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_padded_size(int n) { return n + (n >> 4) + 1; }

// radix of the first pass when the later ones have radix 2^LGM
__host__ __device__ constexpr int fft_first_lgr(int lgn, int lgm) { return (lgn % lgm) ? (lgn % lgm) : lgm; }

// Offset of padded element i0 + c from padded element i0, where the
// accessors below guarantee that adding c moves i0 across whole 16-element
// groups only: lds_pad(x + c) = lds_pad(x) + c + (c >> 4).
__host__ __device__ constexpr int pad_off(int c) { return c + (c >> 4); }

// One radix-R pass over `batch` transforms of length 2^LGN.  Butterfly j
// (0 <= j < N/R) takes inputs x[j + r N/R] = load(b, j, r N/R), twiddles input r
// by w_{Ns R}^{r k} (Ns = 2^LGNS, k = j mod Ns), applies the R-point DFT and
// hands output r to store(b, (j - k) R + k, r Ns, value).  Accessors get the
// element index split as i0 + c with c a compile-time constant after
// unrolling; in-LDS accessors place it at lds_pad(b N + i0) + pad_off(c).
// That is exact here: for the loads i0 = j < M = N/R and c = r M; for the
// stores i0 = (j - k) R + k and c = r Ns; N, M, Ns, R are powers of two with
// N >= 16, so c either is a multiple of 16 or stays inside the 16-group of i0.
//   IN_PLACE = false: each butterfly is loaded, computed and stored in turn
//                     (source and destination are different buffers).
//   IN_PLACE = true : every thread first loads all its butterflies (at most
//                     ITEMS), then a barrier, then the stores.
// No barrier after the stores.
template <typename T, int R, int LGNS, bool INV>
__device__ __forceinline__ void fft_butterfly(cplx<T>* v, int k, const cplx<T>* __restrict__ tw) {
  constexpr int lgR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  constexpr int tws = TW_LOG - (LGNS + lgR);
  if constexpr (LGNS > 0) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = v[r] * twid<T, INV>(tw, (r * k) << tws);
  }
  dftR<T, R, INV>(v);
}

template <typename T, int R, int LGN, int LGNS, int ITEMS, int THREADS, bool INV, bool IN_PLACE, class Load,
          class Store>
__device__ __forceinline__ void fft_pass(int batch, const cplx<T>* __restrict__ tw, Load load, Store store) {
  constexpr int lgR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  constexpr int lgM = LGN - lgR;
  constexpr int M = 1 << lgM;
  constexpr int Ns = 1 << LGNS;
  static_assert(LGNS + lgR <= LGN && LGN >= 4, "pass exceeds the transform length");
  const int all = M * batch;
  // the lane index passes through an empty asm so that this pass's index and
  // address arithmetic is redone here instead of being hoisted out of the
  // caller's loops into registers held across them
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  if constexpr (!IN_PLACE) {
    for (int j = tid; j < all; j += THREADS) {
      const int b = j >> lgM;
      const int jj = j & (M - 1);
      const int k = jj & (Ns - 1);
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = load(b, jj, r * M);
      fft_butterfly<T, R, LGNS, INV>(v, k, tw);
      const int base = ((jj - k) << lgR) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) store(b, base, r * Ns, v[r]);
    }
  } else {
    cplx<T> v[ITEMS][R];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int j = tid + it * THREADS;
      if (j < all) {
        const int b = j >> lgM;
        const int jj = j & (M - 1);
        const int k = jj & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = load(b, jj, r * M);
        fft_butterfly<T, R, LGNS, INV>(v[it], k, tw);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int j = tid + it * THREADS;
      if (j < all) {
        const int b = j >> lgM;
        const int jj = j & (M - 1);
        const int k = jj & (Ns - 1);
        const int base = ((jj - k) << lgR) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) store(b, base, r * Ns, v[it][r]);
      }
    }
  }
}

// In-LDS accessors of the padded buffer holding `batch` rows of 2^LGN values;
// row b starts RPAD extra elements further on (rows that are a multiple of
// 256 bytes apart would otherwise share their LDS banks).
template <typename T, int LGN, int RPAD = 0>
struct LdsRows {
  cplx<T>* buf;
  __device__ __forceinline__ static int at(int b, int i) { return lds_pad((b << LGN) + i) + b * RPAD; }
  __device__ __forceinline__ cplx<T> operator()(int b, int i0, int c) const { return buf[at(b, i0) + pad_off(c)]; }
  __device__ __forceinline__ void operator()(int b, int i0, int c, cplx<T> v) const { buf[at(b, i0) + pad_off(c)] = v; }
};
// elements of such a buffer
__host__ __device__ constexpr int lds_rows_size(int batch, int lgn, int rpad) {
  return lds_padded_size(batch << lgn) + batch * rpad;
}

// Passes from span 2^LGNS to the end of a transform of length 2^LGN held in
// the padded LDS buffer `buf` (the earlier passes have been written there and
// followed by a barrier).  All have radix 2^LGM; the passes in between run in
// place, the last one writes through `storeN` (in place when LAST_IN_LDS says
// that storeN writes `buf`).  No barrier after the final stores.
template <typename T, int NMAX, int THREADS, bool INV, bool LAST_IN_LDS, int LGN, int LGNS, int LGM, class StoreN,
          int RPAD = 0>
__device__ __forceinline__ void fft_tail(cplx<T>* buf, int batch, const cplx<T>* __restrict__ tw, StoreN storeN) {
  static_assert(LGM == 3 || LGM == 4, "later radix 8 or 16");
  static_assert((LGN - LGNS) % LGM == 0 && LGNS < LGN, "later passes must tile the remaining bits");
  constexpr int RM = 1 << LGM;
  constexpr int IM = (NMAX / RM + THREADS - 1) / THREADS;
  const LdsRows<T, LGN, RPAD> lds{buf};
  if constexpr (LGNS + LGM < LGN) {
    fft_pass<T, RM, LGN, LGNS, IM, THREADS, INV, true>(batch, tw, lds, lds);
    __syncthreads();
    fft_tail<T, NMAX, THREADS, INV, LAST_IN_LDS, LGN, LGNS + LGM, LGM, StoreN, RPAD>(buf, batch, tw, storeN);
  } else {
    fft_pass<T, RM, LGN, LGNS, IM, THREADS, INV, LAST_IN_LDS>(batch, tw, lds, storeN);
  }
}

// Complete transform of `batch` rows of length 2^LGN: the first pass (radix
// 2^fft_first_lgr(LGN, LGM)) reads through `load0`, the last pass writes
// through `storeN`, the passes in between run in place in `buf`.
// FIRST_IN_LDS says that load0 reads `buf` and LAST_IN_LDS that storeN writes
// it (those passes then run in place).  NMAX bounds N * batch, THREADS is the
// block size, RPAD the row padding of `buf` (LdsRows).  Barriers separate the
// passes; there is none after the final stores.
template <typename T, int NMAX, int THREADS, bool INV, bool FIRST_IN_LDS, bool LAST_IN_LDS, int LGN, int LGM,
          class Load0, class StoreN, int RPAD = 0>
__device__ __forceinline__ void fft_run(cplx<T>* buf, int batch, const cplx<T>* __restrict__ tw, Load0 load0,
                                        StoreN storeN) {
  constexpr int LGR0 = fft_first_lgr(LGN, LGM);
  constexpr int R0 = 1 << LGR0;
  constexpr int I0 = (NMAX / R0 + THREADS - 1) / THREADS;
  if constexpr (LGR0 == LGN) {
    fft_pass<T, R0, LGN, 0, I0, THREADS, INV, FIRST_IN_LDS || LAST_IN_LDS>(batch, tw, load0, storeN);
  } else {
    const LdsRows<T, LGN, RPAD> lds{buf};
    fft_pass<T, R0, LGN, 0, I0, THREADS, INV, FIRST_IN_LDS>(batch, tw, load0, lds);
    __syncthreads();
    fft_tail<T, NMAX, THREADS, INV, LAST_IN_LDS, LGN, LGR0, LGM, StoreN, RPAD>(buf, batch, tw, storeN);
  }
}

// XCD-aware block order: blocks are dispatched round-robin over the 8 XCDs,
// each with its own L2, so block bid is given work item xcd_remap(bid): each
// XCD then takes one contiguous eighth of the items (neighbouring items that
// share input lines, or write into one line, meet in one L2).  nblk must be a
// multiple of 8; the map is a permutation of [0, nblk).
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int per = nblk >> 3;
  return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// ---------------------------------------------------------------------------
// batched launches
// ---------------------------------------------------------------------------
// A launch serves a group of up to MAX_GROUP pairs that share a descriptor and
// a row pitch, so that every size, table and workspace offset is the same for
// all of them: pair blockIdx.z reads its own images and workspace through a
// PairSet passed by value (a captured graph holds the pointers themselves).
constexpr int MAX_GROUP = 32;
struct PairSet {
  const void* sci[MAX_GROUP];
  const void* tmpl[MAX_GROUP];
  const uint8_t* mask[MAX_GROUP];   // entries may be null (no mask)
  unsigned char* ws[MAX_GROUP];     // the pair's workspace
  // workspace holding the pair's template-side data (template spectra and
  // row spectra, normal matrix, factor, solve outcome): ws itself, or the
  // workspace of the pair whose template and mask this pair shares
  unsigned char* tws[MAX_GROUP];
  double* coeffs[MAX_GROUP];        // theta: read by the subtraction, written by the solve's copy-out
  void* diff[MAX_GROUP];
  int32_t* info[MAX_GROUP];         // per-pair solve outcome (entries may be null)
};
// Byte offsets of the workspace buffers (the same for every pair of a group).
struct WsOff {
  size_t Ub, U, V, win, mom, obb, bb, omega, beta, kp, flags, tw32, tw64, items, wrows, drows, mtiles, theta;
  size_t Uq, Mh, G;   // the subtraction's buffers (inside the U region)
  size_t amom, kbpart, kbT, kbd, kbgrp;   // template moments and the template-background block
  size_t omcnt;                            // excluded pixels per image row
};
template <typename X>
__device__ __forceinline__ X* ws_at(const PairSet& S, int pr, size_t off) {
  return reinterpret_cast<X*>(S.ws[pr] + off);
}

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int i = 0; i < p; ++i) r *= x;
  return r;
}

}  // namespace sfft
