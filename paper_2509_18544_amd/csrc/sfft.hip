// Host runtime and C ABI of the SFFT subtraction library (see include/sfft.h).
//
// A plan owns (or borrows) one workspace carved into the buffers below and a
// HIP stream on which every call enqueues its kernels; no call synchronises
// except sfft_status().
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <algorithm>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/sfft.h"
#include "assemble.hpp"
#include "cholesky.hpp"
#include "common.hpp"
#include "decorr.hpp"
#include "subtract.hpp"
#include "outmask.hpp"
#include "kbmom.hpp"

using namespace sfft;

namespace {

constexpr int ASM_THREADS = 256;
constexpr int FFT_THREADS = 512;     // row and column transform blocks
constexpr int SUB_NMAX = 4096;       // complex FP64 elements per subtraction row-transform block (64 KB)
constexpr int ROW_NMAX_F32 = 8192;    // complex elements in the row-pass LDS buffer (64 KB)
constexpr int ROW_NMAX_F64 = 4096;    // 64 KB
constexpr int COL_NMAX = 8192;        // complex elements per column-pass block (two columns)
constexpr int COL_LGM = 4;            // later passes of the column transform: radix 16 (radix 8 measured slower)
constexpr int WIN_THREADS = 64;
constexpr int WIN_IMAX = 64;
constexpr int MAX_N = 8192;           // unknowns (the triangular solves keep x in LDS)
constexpr int MAX_W = 15;
constexpr double DIR_AUTO_FMA = 1.0e9;   // direct lag sums below this many multiply-adds (small frames)
constexpr int MFMA_TARGET_BLOCKS = 2048;  // the MFMA route splits the rows into bands up to about this many blocks
constexpr int MAX_MTILES = MFMA_MAXT * MAX_ITEMS;   // (pair, dy tile) units of the MFMA route

// how the lag windows are computed
enum Route { ROUTE_FFT = 0, ROUTE_DIRECT = 1, ROUTE_MFMA = 2 };

// A vector of fixed capacity held inline: filling it never allocates, so a
// plan can be derived into static storage (the no-allocation entry point).
template <typename T, int CAP>
struct FixedVec {
  T v[CAP];
  int n = 0;
  void clear() { n = 0; }
  bool push_back(const T& x) {
    if (n >= CAP) return false;
    v[n++] = x;
    return true;
  }
  int size() const { return n; }
  T* data() { return v; }
  const T* data() const { return v; }
  T& operator[](int i) { return v[i]; }
  const T& operator[](int i) const { return v[i]; }
  T& back() { return v[n - 1]; }
  T* begin() { return v; }
  T* end() { return v + n; }
  const T* begin() const { return v; }
  const T* end() const { return v + n; }
};

// lag rows of all windows: every item covers at most JMAX of them
constexpr int MAX_VROWS = JMAX * MAX_ITEMS;

struct Layout {
  size_t Ub, U, V, win, mom, obb, bb, omega, beta, F, Linv, theta, y, r, d, w, kp, flags, tw32, tw64, items, wrows, drows,
      mtiles, ratio, job, rjob, om_planes, om_cnt, om_offs, om_list, amom, kbpart, kbT, kbd, kbgrp;
  size_t total;
};

struct Derived {
  int ny, nx, w, dk, db, mode, refine;
  int L, nk, nb, nkk, n;
  int lgPy, lgPx, Py, Px, H;
  int nplanes;
  int nmu;   // monomials of degree <= DK + DB (moments of G_R R, excluded-pixel sums)
  int nbase, nbk, nbb;
  // right-hand side only: the template and mask are another pair's, whose
  // template spectra, normal matrix and factor this plan uses (its own build
  // transforms the science base and forms beta alone)
  bool rhs_only;
  int base_lo, nstaged, nshared, plane_skip;
  bool omask;   // output-masked fit: the excluded pixels' rows are taken out of Omega
  int8_t base_first[MAX_BASE], base_count[MAX_BASE], out_plane[MAX_PLANES], out_q[MAX_PLANES];
  int rows_per_block, nrowblk;
  int nmom;
  int nitems, vrows, nwin, nblk;
  int corr_lanes;
  int jrows;   // lag rows per correlation item (JROWS_NARROW or JROWS_WIDE)
  int njlo;
  int16_t jlo_list[MAX_JLO];
  size_t csize;   // sizeof complex element of the transforms
  FixedVec<CorrItem, MAX_ITEMS> items;
  FixedVec<WinRow, MAX_VROWS> wrows;
  int route;                      // Route: transforms, direct sums or matrix-core products
  int nratio;                     // constant photometric ratio: nK - 1 constraints, else 0
  FixedVec<DirectRow, MAX_VROWS> drows;
  FixedVec<MfmaTile, MAX_MTILES> mtiles;
  int mfma_nxc, mfma_band, mfma_nband;   // MFMA route: column chunks, rows per band, bands
  int dir_tpr, dir_nband;
  GatherParams gp;
  PolyTab kpoly, bpoly;
};

int ilog2_ceil(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

void monomial_table(int deg, PolyTab* t) {
  int j = 0;
  std::memset(t, 0, sizeof(*t));
  for (int d = 0; d <= deg; ++d)
    for (int q = 0; q <= d; ++q) {
      t->px[j] = (int8_t)(d - q);
      t->qy[j] = (int8_t)q;
      ++j;
    }
}

int validate(const sfft_desc* d) {
  if (d == nullptr) return SFFT_EINVAL;
  if (d->w < 0 || d->w > MAX_W) return SFFT_EINVAL;
  if (d->dk < 0 || d->dk > MAX_DEG || d->db < 0 || d->db > MAX_DEG) return SFFT_EINVAL;
  if (d->ny < 4 * d->w + 2 || d->nx < 4 * d->w + 2) return SFFT_EINVAL;
  if (d->ny < 2 || d->nx < 2) return SFFT_EINVAL;
  if (d->ny > (1 << MAX_LOG_P) || d->nx > (1 << MAX_LOG_P)) return SFFT_EINVAL;
  if (d->mode != SFFT_MODE_F64 && d->mode != SFFT_MODE_F32C) return SFFT_EINVAL;
  if (d->refine_steps < -1 || d->refine_steps > 10) return SFFT_EINVAL;
  if ((d->flags & ~(3 | SFFT_FLAG_CONST_RATIO | SFFT_FLAG_OUTPUT_MASK)) != 0) return SFFT_EINVAL;
  if ((d->flags & 3) == SFFT_FLAG_ASSEMBLY_DIRECT && (d->nx > DIR_MAX_NX || 2 * d->w > DIR_HWMAX)) return SFFT_EINVAL;
  const int L = 2 * d->w + 1;
  const int nk = (d->dk + 1) * (d->dk + 2) / 2, nb = (d->db + 1) * (d->db + 2) / 2;
  const int64_t n = (int64_t)L * L * nk + nb;
  if (n > MAX_N) return SFFT_EINVAL;
  return SFFT_OK;
}

// Everything about a plan that depends only on the descriptor (and, for a
// plan of the right-hand side only, on that role).
int derive(const sfft_desc* d, Derived* D, bool rhs_only = false) {
  int st = validate(d);
  if (st != SFFT_OK) return st;
  D->ny = d->ny;
  D->nx = d->nx;
  D->w = d->w;
  D->dk = d->dk;
  D->db = d->db;
  D->mode = d->mode;
  D->refine = d->refine_steps < 0 ? 1 : d->refine_steps;
  D->L = 2 * d->w + 1;
  D->nk = (d->dk + 1) * (d->dk + 2) / 2;
  D->nb = (d->db + 1) * (d->db + 2) / 2;
  D->nratio = (d->flags & SFFT_FLAG_CONST_RATIO) ? D->nk - 1 : 0;
  D->nkk = D->L * D->L * D->nk;
  D->n = D->nkk + D->nb;
  D->lgPy = std::max(MIN_LOG_P, ilog2_ceil(d->ny));
  D->lgPx = std::max(MIN_LOG_P, ilog2_ceil(d->nx));
  D->Py = 1 << D->lgPy;
  D->Px = 1 << D->lgPx;
  D->H = D->Px / 2;
  // planes of the transform route: the nK template planes A_a and the
  // masked science image S_m (plane nK).  The template-background block
  // Omega_KB comes from FP64 moments and the excluded pixels instead of
  // correlations with the background planes G m_b (kb_* kernels).
  D->nplanes = D->nk + 1;
  D->nmu = (d->dk + d->db + 1) * (d->dk + d->db + 2) / 2;
  D->rhs_only = rhs_only;
  D->omask = (d->flags & SFFT_FLAG_OUTPUT_MASK) != 0;
  // base rows and the output planes built from each (plane index, y-power)
  D->nbk = d->dk + 1;
  D->nbb = 0;   // no background bases (Omega_KB from moments)
  D->nbase = D->nbk + D->nbb + 1;
  // planes of a full build: every base, all planes staged from the own
  // workspace; right-hand side only: the science base, and the nK template
  // planes (shared) followed by the own science plane nK
  D->base_lo = rhs_only ? D->nbase - 1 : 0;
  D->nstaged = D->nplanes;
  D->nshared = rhs_only ? D->nk : D->nplanes;
  D->plane_skip = 0;
  {
    int cursor = 0;
    for (int b = 0; b < D->nbase; ++b) {
      D->base_first[b] = (int8_t)cursor;
      int cnt = 0;
      if (b < D->nbk) {
        for (int j = 0, dd = 0; dd <= d->dk; ++dd)
          for (int q = 0; q <= dd; ++q, ++j)
            if (dd - q == b) {
              D->out_plane[cursor] = (int8_t)j;
              D->out_q[cursor] = (int8_t)q;
              ++cursor;
              ++cnt;
            }
      } else if (b < D->nbk + D->nbb) {
        const int pb = b - D->nbk;
        for (int j = 0, dd = 0; dd <= d->db; ++dd)
          for (int q = 0; q <= dd; ++q, ++j)
            if (dd - q == pb) {
              D->out_plane[cursor] = (int8_t)(D->nk + j);
              D->out_q[cursor] = (int8_t)q;
              ++cursor;
              ++cnt;
            }
      } else {
        D->out_plane[cursor] = (int8_t)D->nk;
        D->out_q[cursor] = 0;
        ++cursor;
        cnt = 1;
      }
      D->base_count[b] = (int8_t)cnt;
    }
  }
  D->csize = d->mode == SFFT_MODE_F64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  const int rowmax = d->mode == SFFT_MODE_F64 ? ROW_NMAX_F64 : ROW_NMAX_F32;
  D->rows_per_block = row_pass_rows(rowmax, D->lgPx - 1);   // fixed per transform size (the kernel's own constant)
  D->nrowblk = (d->ny + D->rows_per_block - 1) / D->rows_per_block;
  // per-row moments: (2DB+1) of G, (DB+1) of G S, (DK+DB+1) of G_R R
  D->nmom = (2 * d->db + 1) + (d->db + 1) + (d->dk + d->db + 1);
  D->nblk = (D->n + NB - 1) / NB;
  monomial_table(d->dk, &D->kpoly);
  monomial_table(d->db, &D->bpoly);

  // correlation pairs -> items (lag rows in chunks of jrows), window rows, gather offsets
  // the widest windows: the template-template ones (|d| <= 2w), or in a
  // right-hand-side-only plan the template-science ones (|d| <= w)
  const int wmax = rhs_only ? d->w : 2 * d->w;
  D->jrows = 2 * wmax + 1 > JROWS_NARROW ? JROWS_WIDE : JROWS_NARROW;
  D->items.clear();
  D->wrows.clear();
  D->drows.clear();
  D->mtiles.clear();
  int vrow = 0, wo = 0;
  bool fits = true;   // every table stayed within its capacity
  // planes are numbered 0..nplanes-1; the correlation items name staged planes
  // (the transform route stages the template planes and the science plane, nK)
  auto staged = [&](int plane) { return plane == D->nk + D->nb ? D->nk : plane; };
  // a window of lags |d| <= hw of planes (left, right): correlation items and
  // window rows of the transform route (when fft), rows and tiles of the
  // direct and matrix-core routes (always)
  auto add_pair = [&](int left, int right, int hw, bool fft) {
    const int h = 2 * hw + 1;
    // items start on the grid -wmax + k jrows of the widest windows (|d| <= wmax),
    // so that every item has one of their rotations jlo mod P2: an item of a
    // narrower window accumulates its jrows rows from such a start and keeps
    // the rows [skip, nj) that fall inside it
    for (int j = -wmax; fft && j <= hw; j += D->jrows) {
      const int lo = std::max(j, -hw), hi = std::min(j + D->jrows - 1, hw);
      if (lo > hi) continue;
      CorrItem it;
      it.left = (int16_t)staged(left);
      it.right = (int16_t)staged(right);
      it.jlo = (int16_t)j;
      it.nj = (int16_t)(hi - j + 1);
      it.vrow = vrow + (j + hw);   // V row of lag row j (rows below skip are never written)
      it.jidx = 0;
      it.skip = (int16_t)(lo - j);
      fits &= D->items.push_back(it);
    }
    for (int j = 0; j < h; ++j) {
      if (fft) {
        WinRow r;
        r.vrow = vrow + j;
        r.out = wo + j * h;
        r.hw = hw;
        fits &= D->wrows.push_back(r);
      }
      DirectRow q;
      q.left = (int16_t)left;
      q.right = (int16_t)right;
      q.hw = (int16_t)hw;
      q.dy = (int16_t)(j - hw);
      q.out = wo + j * h;
      fits &= D->drows.push_back(q);
    }
    for (int dy0 = -hw; dy0 <= hw; dy0 += 16) {
      MfmaTile t;
      t.left = (int16_t)left;
      t.right = (int16_t)right;
      t.hw = (int16_t)hw;
      t.dy0 = (int16_t)dy0;
      t.out = wo;
      fits &= D->mtiles.push_back(t);
    }
    const int off = wo;
    if (fft) vrow += h;
    wo += h * h;
    return off;
  };
  const int w = d->w;
  if (!rhs_only) {
    for (int a = 0; a < D->nk; ++a)
      for (int b = a; b < D->nk; ++b) D->gp.kk_off[a * D->nk + b] = add_pair(a, b, 2 * w, true);
    // the template-background windows: direct and matrix-core routes only
    for (int a = 0; a < D->nk; ++a)
      for (int b = 0; b < D->nb; ++b) D->gp.kb_off[a * D->nb + b] = add_pair(a, D->nk + b, w, false);
  }
  for (int a = 0; a < D->nk; ++a) D->gp.ks_off[a] = add_pair(a, D->nk + D->nb, w, true);
  if (!fits) return SFFT_EINVAL;   // more correlation items than the kernels take
  // items sorted by their residue rotation (jlo mod P2) so that a wave of the
  // correlation kernel normally takes a single case of its rotation switch
  // (a stable insertion sort: no allocation, at most MAX_ITEMS items)
  {
    auto rot_of = [](const CorrItem& x) { return ((x.jlo % P2) + P2) % P2; };
    for (int i = 1; i < D->items.size(); ++i) {
      const CorrItem x = D->items[i];
      int j = i - 1;
      while (j >= 0 && rot_of(D->items[j]) > rot_of(x)) {
        D->items[j + 1] = D->items[j];
        --j;
      }
      D->items[j + 1] = x;
    }
  }
  // threads per item: the largest count (<= 64) that keeps all real items in
  // one pass of the block; each rotation group is padded with empty items
  // (nj = 0) to a whole number of waves so that a wave takes one switch case.
  {
    const int real = (int)D->items.size();
    int lanes = 1;
    for (int l = 64; l >= 1; --l) {
      const int ipw = 64 / l;
      // waves needed with group padding
      int waves = 0;
      int i = 0;
      while (i < D->items.size()) {
        const int rot = ((D->items[i].jlo % P2) + P2) % P2;
        int cnt = 0;
        while (i < D->items.size() && ((D->items[i].jlo % P2) + P2) % P2 == rot) {
          ++cnt;
          ++i;
        }
        waves += (cnt + ipw - 1) / ipw;
      }
      if (waves * 64 <= 256 * 4) {   // at most four passes of a 256-thread block
        if (waves <= 4) {
          lanes = l;
          break;
        }
      }
      (void)real;
    }
    D->corr_lanes = lanes;
    const int ipw = 64 / lanes;
    FixedVec<CorrItem, MAX_ITEMS> padded;
    int i = 0;
    while (i < D->items.size()) {
      const int rot = ((D->items[i].jlo % P2) + P2) % P2;
      int cnt = 0;
      while (i < D->items.size() && ((D->items[i].jlo % P2) + P2) % P2 == rot) {
        fits &= padded.push_back(D->items[i]);
        ++cnt;
        ++i;
      }
      while (cnt % ipw != 0) {
        CorrItem e = padded.back();
        e.nj = 0;
        fits &= padded.push_back(e);
        ++cnt;
      }
    }
    if (!fits) return SFFT_EINVAL;
    D->items = padded;
    // every wave of the correlation kernel takes ipw consecutive items: they
    // must share one rotation (the kernel reads it from the wave's first item)
    for (int i = 0; i < D->items.size(); ++i)
      if (((D->items[i].jlo % P2) + P2) % P2 != ((D->items[(i / ipw) * ipw].jlo % P2) + P2) % P2) return SFFT_EINVAL;
  }
  D->nitems = (int)D->items.size();
  // distinct first lag rows (the correlation kernel tabulates their twiddles per chunk)
  D->njlo = 0;
  for (CorrItem& it : D->items) {
    int ji = -1;
    for (int i = 0; i < D->njlo; ++i)
      if (D->jlo_list[i] == it.jlo) ji = i;
    if (ji < 0) {
      if (D->njlo >= MAX_JLO) return SFFT_EINVAL;
      D->jlo_list[D->njlo] = it.jlo;
      ji = D->njlo++;
    }
    it.jidx = (int16_t)ji;
  }
  D->vrows = vrow;
  D->nwin = wo;
  // assembly route: forced by the descriptor, else direct sums when their
  // multiply-adds stay below DIR_AUTO_FMA (small frames)
  {
    double fma = 0.0;
    for (const DirectRow& q : D->drows) fma += (2.0 * q.hw + 1.0) * (double)d->ny * (double)d->nx;
    const bool ok = d->nx <= DIR_MAX_NX && 2 * d->w <= DIR_HWMAX;
    const int rf = d->flags & 3;
    const bool direct = rf == SFFT_FLAG_ASSEMBLY_DIRECT || (rf == SFFT_FLAG_ASSEMBLY_AUTO && ok && fma <= DIR_AUTO_FMA);
    D->route = rf == SFFT_FLAG_ASSEMBLY_MFMA ? ROUTE_MFMA : (direct ? ROUTE_DIRECT : ROUTE_FFT);
    // MFMA route: column chunks, then row bands until the grid has about
    // MFMA_TARGET_BLOCKS blocks (bands of at least 16 rows)
    D->mfma_nxc = (d->nx + MFMA_XC - 1) / MFMA_XC;
    const int base = std::max(1, D->mtiles.size() * D->mfma_nxc);
    const int nb_max = std::max(1, d->ny / 16);
    const int nband = std::min(nb_max, std::max(1, (MFMA_TARGET_BLOCKS + base - 1) / base));
    D->mfma_band = (d->ny + nband - 1) / nband;
    D->mfma_nband = (d->ny + D->mfma_band - 1) / D->mfma_band;
    int tpr = DIR_MIN_TPR;
    while (tpr * DIR_XB < d->nx) tpr *= 2;
    D->dir_tpr = tpr;
    D->dir_nband = (d->ny + DIR_BAND - 1) / DIR_BAND;
  }
  if (D->nitems > MAX_ITEMS) return SFFT_EINVAL;
  D->gp.n = D->n;
  D->gp.nkk = D->nkk;
  D->gp.L = D->L;
  D->gp.w = w;
  D->gp.nk = D->nk;
  D->gp.nb = D->nb;
  return SFFT_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// radix (log2) of the first pass of a 2^lgN-point transform: the remainder of
// lgN mod 4, or 4 (the later passes are all radix 16)
// first pass radix of a plan whose later passes have radix 2^lgm

Layout layout_of(const Derived& D) {
  Layout Lo;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  Lo.Ub = take((size_t)D.nbase * D.H * D.Py * D.csize);
  {
    // the subtraction's spectra reuse the assembly's spectra region (not live at the same time)
    const size_t asm_bytes = (size_t)D.nplanes * (D.H + 1) * D.Py * D.csize;
    // x-power spectra, model spectrum and filters G (FP64)
    const size_t sub_bytes = align256(sub_xpow_off(D.dk + 1, D.ny, D.H, 0)) +
                             align256((size_t)D.ny * (D.H + 1) * sizeof(cplx<double>)) +
                             align256((size_t)D.nk * D.L * (D.H + 1) * sizeof(cplx<double>));
    // direct and MFMA route partial sums (per band, per chunk and band)
    const size_t dir_bytes = (size_t)D.dir_nband * D.nwin * sizeof(double);
    const size_t mfma_bytes = (size_t)D.mfma_nxc * D.mfma_nband * D.nwin * sizeof(double);
    // (also the decorrelation kernel's grid spectrum)
    const size_t dec_bytes = (size_t)DEC_ND * DEC_ND * sizeof(double);
    Lo.U = take(std::max(std::max(std::max(asm_bytes, sub_bytes), std::max(dir_bytes, mfma_bytes)), dec_bytes));
  }
  Lo.V = take((size_t)(D.H + 1) * D.vrows * sizeof(cplx<double>));
  Lo.win = take((size_t)D.nwin * sizeof(double));
  Lo.mom = take((size_t)D.ny * D.nmom * sizeof(double));
  Lo.obb = take((size_t)D.nb * D.nb * sizeof(double));
  Lo.bb = take((size_t)D.nb * sizeof(double));
  Lo.omega = take((size_t)D.n * D.n * sizeof(double));
  Lo.beta = take((size_t)D.n * sizeof(double));
  Lo.F = take((size_t)D.n * D.n * sizeof(double));
  Lo.Linv = take((size_t)D.nblk * NB * NB * sizeof(double));
  Lo.theta = take((size_t)D.n * sizeof(double));
  Lo.y = take((size_t)D.n * sizeof(double));
  Lo.r = take((size_t)D.n * sizeof(double));
  Lo.d = take((size_t)D.n * sizeof(double));
  Lo.w = take((size_t)D.n * sizeof(double));
  Lo.kp = take((size_t)D.nk * D.L * D.L * sizeof(double));
  Lo.flags = take(2 * sizeof(int));
  Lo.tw32 = take((size_t)TW_N * sizeof(cplx<float>));
  Lo.tw64 = take((size_t)TW_N * sizeof(cplx<double>));
  Lo.items = take((size_t)D.nitems * sizeof(CorrItem));
  Lo.wrows = take((size_t)D.wrows.size() * sizeof(WinRow));
  Lo.drows = take((size_t)D.drows.size() * sizeof(DirectRow));
  Lo.mtiles = take((size_t)D.mtiles.size() * sizeof(MfmaTile));
  // constant photometric ratio: C^T, Z and the substitution vectors of each constraint column
  Lo.ratio = take((size_t)6 * D.nratio * D.n * sizeof(double));
  Lo.job = take((size_t)(1 + D.nratio) * sizeof(SolveJob));
  Lo.rjob = take(sizeof(RatioJob));
  // output-masked fit: padded FP64 template planes, row counts and offsets, the excluded pixels
  {
    const size_t plane = (size_t)(D.ny + 2 * D.w) * (D.nx + 2 * D.w);
    Lo.om_planes = take(D.omask ? (size_t)D.nk * plane * sizeof(double) : 0);
    // the excluded-pixel list also serves the template-background block
    Lo.om_cnt = take((size_t)D.ny * sizeof(int));
    Lo.om_offs = take((size_t)(D.ny + 1) * sizeof(int));
    Lo.om_list = take((size_t)D.ny * D.nx * sizeof(int));
  }
  // template-background block: moments, excluded-pixel partial sums and sums, the block
  Lo.amom = take((size_t)D.nmu * sizeof(double));
  Lo.kbpart = take((size_t)KB_CHUNKS * D.nmu * D.L * D.L * sizeof(double));
  Lo.kbT = take((size_t)D.nmu * D.L * D.L * sizeof(double));
  Lo.kbd = take((size_t)D.nkk * D.nb * sizeof(double));
  Lo.kbgrp = take((size_t)(D.ny + 2 * D.w) * (D.nx + 2 * D.w) * (D.mode == SFFT_MODE_F64 ? 8 : 4));
  Lo.total = off;
  return Lo;
}

// exp(-2 pi i m / TW_N) in FP64, from long-double sin/cos on the first octant
// and exact symmetries elsewhere.
void twiddle_tables(cplx<double>* t64, cplx<float>* t32) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int m = 0; m < TW_N; ++m) {
    // angle = 2 pi m / N; reduce to [0, pi/4] by octant symmetry
    const int oct = m / (TW_N / 8);
    const int r = m % (TW_N / 8);
    long double c, s;
    auto cs = [&](int k, long double* co, long double* si) {
      const long double a = 2.0L * pi * (long double)k / (long double)TW_N;
      *co = cosl(a);
      *si = sinl(a);
    };
    long double c0, s0, c1, s1;
    cs(r, &c0, &s0);                       // angle r
    cs(TW_N / 8 - r, &c1, &s1);            // angle pi/4 - r (complement inside the octant)
    switch (oct) {
      case 0: c = c0; s = s0; break;                       // theta
      case 1: c = s1; s = c1; break;                       // pi/2 - (pi/4 - r') = pi/4 + r
      case 2: c = -s0; s = c0; break;                      // pi/2 + r
      case 3: c = -c1; s = s1; break;                      // pi - (pi/4 - r)
      case 4: c = -c0; s = -s0; break;                     // pi + r
      case 5: c = -s1; s = -c1; break;                     // 3pi/2 - (pi/4 - r)
      case 6: c = s0; s = -c0; break;                      // 3pi/2 + r
      default: c = c1; s = -s1; break;                     // 2pi - (pi/4 - r)
    }
    t64[m].x = (double)c;
    t64[m].y = -(double)s;   // forward sign
    t32[m].x = (float)t64[m].x;
    t32[m].y = (float)t64[m].y;
  }
}

}  // namespace

// roctx range over a scope (host-side enqueue of an ABI call or a stage), so
// that a marker trace shows which kernels each call and stage launched.
struct RoctxScope {
  explicit RoctxScope(const char* name) { roctxRangePushA(name); }
  ~RoctxScope() { roctxRangePop(); }
  RoctxScope(const RoctxScope&) = delete;
  RoctxScope& operator=(const RoctxScope&) = delete;
};

namespace {
const char* const kStageNames[SFFT_NUM_STAGES] = {"moments", "row_fwd", "col_fwd", "corr", "row_win",
                                                  "gather", "factor", "solve", "subtract", "outmask"};
}

// Optional per-stage device timing with events recorded on the plan's stream.
struct StageTimer {
  bool on = false;
  bool silent = false;   // no roctx ranges either (the no-allocation path calls nothing that may allocate)
  unsigned mask = 0;   // stages timed while on (bit s = stage s)
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[SFFT_NUM_STAGES];
  double ms[SFFT_NUM_STAGES] = {};
  int64_t cnt[SFFT_NUM_STAGES] = {};
  hipEvent_t open_ev = nullptr;
  int open_stage = -1;
  bool ranged = false;   // a roctx range is open for the current stage

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // keep at least n events ready so that timing does not create any while enabled
  void reserve(size_t n) {
    while (pool.size() < n) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return;
      pool.push_back(e);
    }
  }
  void begin(int st, hipStream_t s) {
    if (silent) return;
    if (ranged) roctxRangePop();   // a stage left by an error return
    roctxRangePushA(kStageNames[st]);
    ranged = true;
    if (!on || ((mask >> st) & 1u) == 0) return;
    open_ev = take();
    open_stage = st;
    if (open_ev) (void)hipEventRecord(open_ev, s);
  }
  void end(hipStream_t s) {
    if (silent) return;
    if (ranged) {
      roctxRangePop();
      ranged = false;
    }
    if (!on || open_stage < 0) return;
    hipEvent_t e = take();
    if (open_ev && e) {
      (void)hipEventRecord(e, s);
      pending[open_stage].push_back({open_ev, e});
    }
    open_stage = -1;
    open_ev = nullptr;
  }
  void fold() {
    for (int st = 0; st < SFFT_NUM_STAGES; ++st) {
      for (auto& pr : pending[st]) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
          ms[st] += t;
          cnt[st] += 1;
        }
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[st].clear();
    }
  }
  void release() {
    for (int st = 0; st < SFFT_NUM_STAGES; ++st) {
      for (auto& pr : pending[st]) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
      pending[st].clear();
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

struct sfft_plan_s {
  sfft_desc desc;
  StageTimer timer;
  // a batch handle owns one single-pair plan per pair (all on the batch's
  // stream) and a device table of their solve jobs
  bool is_batch = false;
  std::vector<sfft_plan_s*> members;
  // a batch member that shares its template and mask: the member that owns
  // them (its template spectra, normal matrix, factor and row spectra)
  sfft_plan_s* tplan = nullptr;
  std::vector<int> tmpl_of;         // batch: per pair, the pair whose template and mask it uses
  SolveJob* jobs_dev = nullptr;     // [jobs owning a factor | jobs sharing one | constraint-column jobs]
  RatioJob* rjobs_dev = nullptr;    // projection jobs (pairs with a constant photometric ratio)
  std::vector<SolveJob> jobs_host;
  RatioJob rjob_host;
  int nfac = 0, nsub = 0, nratio = 0;
  int max_n = 0, max_nblk = 0;
  // graph of one captured batch run (sfft_batch_capture / sfft_batch_launch)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int corr_c1 = 0;   // residue chunk of the correlation kernel, 0 = default (sfft_autotune sets it)
  Derived D;
  Layout Lo;
  hipStream_t stream;
  unsigned char* ws;
  bool owns_ws;
  bool built;
  std::vector<cplx<double>> tw64h;
  std::vector<cplx<float>> tw32h;
  template <typename X>
  X* at(size_t off) const {
    return reinterpret_cast<X*>(ws + off);
  }
};

#define HIP_TRY(expr)                       \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return SFFT_EHIP; \
  } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

namespace {

AsmParams asm_params(const sfft_plan_s* p, int64_t ld) {
  const Derived& D = p->D;
  AsmParams A;
  std::memset(&A, 0, sizeof(A));
  A.ny = D.ny;
  A.nx = D.nx;
  A.w = D.w;
  A.nk = D.nk;
  A.nb = D.nb;
  A.nplanes = D.nplanes;
  A.lgPy = D.lgPy;
  A.lgPx = D.lgPx;
  A.H = D.H;
  A.ld = ld;
  A.rows_per_block = D.rows_per_block;
  A.nrowblk = D.nrowblk;
  A.nitems = D.nitems;
  A.corr_lanes = D.corr_lanes;
  A.njlo = D.njlo;
  A.dir_tpr = D.dir_tpr;
  A.base_lo = D.base_lo;
  A.nstaged = D.nstaged;
  A.nshared = D.nshared;
  A.plane_skip = D.plane_skip;
  for (int i = 0; i < MAX_JLO; ++i) A.jlo_list[i] = i < D.njlo ? D.jlo_list[i] : 0;
  A.vrows = D.vrows;
  A.kpoly = D.kpoly;
  A.bpoly = D.bpoly;
  A.nmom = D.nmom;
  A.db = D.db;
  A.na = D.dk + D.db + 1;
  A.nmu = D.nmu;
  A.nbase = D.nbase;
  A.nbk = D.nbk;
  A.nbb = D.nbb;
  A.sx = 2.0 / (double)(D.nx - 1);
  A.sy = 2.0 / (double)(D.ny - 1);
  for (int b = 0; b < MAX_BASE; ++b) {
    A.base_first[b] = D.base_first[b];
    A.base_count[b] = b < D.nbase ? D.base_count[b] : 0;
  }
  for (int i = 0; i < MAX_PLANES; ++i) {
    A.out_plane[i] = D.out_plane[i];
    A.out_q[i] = D.out_q[i];
  }
  return A;
}

// Byte offsets of the workspace buffers handed to the kernels.
WsOff ws_offsets(const Derived& D, const Layout& Lo) {
  WsOff O;
  O.Ub = Lo.Ub;
  O.U = Lo.U;
  O.V = Lo.V;
  O.win = Lo.win;
  O.mom = Lo.mom;
  O.obb = Lo.obb;
  O.bb = Lo.bb;
  O.omega = Lo.omega;
  O.beta = Lo.beta;
  O.kp = Lo.kp;
  O.flags = Lo.flags;
  O.tw32 = Lo.tw32;
  O.tw64 = Lo.tw64;
  O.items = Lo.items;
  O.wrows = Lo.wrows;
  O.drows = Lo.drows;
  O.mtiles = Lo.mtiles;
  O.theta = Lo.theta;
  O.amom = Lo.amom;
  O.kbpart = Lo.kbpart;
  O.kbT = Lo.kbT;
  O.kbd = Lo.kbd;
  O.kbgrp = Lo.kbgrp;
  O.omcnt = Lo.om_cnt;
  // the subtraction's x-power spectra, model spectrum and filters reuse the U region
  O.Uq = Lo.U;
  // (the x-power spectra end at most at sub_xpow_off(dk + 1, .., xp32 = 0))
  O.Mh = O.Uq + align256(sub_xpow_off(D.dk + 1, D.ny, D.H, 0));
  O.G = O.Mh + align256((size_t)D.ny * (D.H + 1) * sizeof(cplx<double>));
  return O;
}

KbParams kb_params(const sfft_plan_s* p, int64_t ld) {
  const Derived& D = p->D;
  KbParams K;
  std::memset(&K, 0, sizeof(K));
  K.ny = D.ny;
  K.nx = D.nx;
  K.w = D.w;
  K.L = D.L;
  K.nk = D.nk;
  K.nb = D.nb;
  K.nkk = D.nkk;
  K.nmu = D.nmu;
  K.pitch = D.nx + 2 * D.w;
  K.ld = ld;
  K.sx = 2.0 / (double)(D.nx - 1);
  K.sy = 2.0 / (double)(D.ny - 1);
  for (int i = 0; i < D.nk; ++i) {
    K.kpx[i] = D.kpoly.px[i];
    K.kqy[i] = D.kpoly.qy[i];
  }
  for (int i = 0; i < D.nb; ++i) {
    K.bpx[i] = D.bpoly.px[i];
    K.bqy[i] = D.bpoly.qy[i];
  }
  return K;
}

OmaskParams om_params(const sfft_plan_s* p, int64_t ld) {
  const Derived& D = p->D;
  OmaskParams P;
  std::memset(&P, 0, sizeof(P));
  P.ny = D.ny;
  P.nx = D.nx;
  P.w = D.w;
  P.nk = D.nk;
  P.L = D.L;
  P.nkk = D.nkk;
  P.n = D.n;
  P.pitch = D.nx + 2 * D.w;
  P.plane = (int64_t)(D.ny + 2 * D.w) * P.pitch;
  P.ld = ld;
  P.sx = 2.0 / (double)(D.nx - 1);
  P.sy = 2.0 / (double)(D.ny - 1);
  for (int i = 0; i < D.nk; ++i) {
    P.px[i] = D.kpoly.px[i];
    P.qy[i] = D.kpoly.qy[i];
  }
  P.ntile = (D.nkk + NB - 1) / NB;
  return P;
}

OmaskOff om_off(const sfft_plan_s* p) {
  OmaskOff O;
  O.planes = p->Lo.om_planes;
  O.cnt = p->Lo.om_cnt;
  O.offs = p->Lo.om_offs;
  O.list = p->Lo.om_list;
  O.omega = p->Lo.omega;
  return O;
}

// The excluded pixels of the np pairs of PS, listed in row-major order (the
// row counts come from the moments pass of the build: their prefix, then the
// list).
int om_list_impl(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld) {
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  const OmaskParams P = om_params(p, ld);
  const OmaskOff O = om_off(p);
  om_scan_kernel<<<dim3(1, 1, np), 1024, 0, s>>>(P, PS, O);
  LAUNCH_CHECK();
  om_list_kernel<<<dim3(D.ny, 1, np), 256, 0, s>>>(P, PS, O);
  LAUNCH_CHECK();
  return SFFT_OK;
}

// The buffers of one pair on its plan's workspace, as a group of one.
PairSet pair_set_one(const sfft_plan_s* p, const void* sci, const void* tmpl, const uint8_t* mask,
                     const double* coeffs, void* diff, int32_t* info);

// Residue chunk of the correlation kernel: the spectra of C1 residues of every
// plane (FP64, padded) and their outer twiddles are staged in LDS per chunk;
// block 0, which carries the DC and Nyquist columns, stages both with the
// chunk corr_dc_chunk(C1).  Layout: the twiddle steps, then the largest of
// the two stages (spectra and the chunk's outer twiddles) and the
// lane-reduction buffer that overlays them.
int corr_dc_chunk(int C1) { return std::max(1, C1 / 2); }
size_t corr_lds_bytes(const Derived& D, int C1) {
  const size_t steps = (size_t)corr_step_elems(D.njlo, D.jrows) * sizeof(cplx<double>);
  const int cd = corr_dc_chunk(C1);
  const size_t stage = (size_t)corr_stage_elems(D.nstaged, corr_plane_stride(C1), (int)D.csize) * D.csize +
                       (size_t)D.njlo * C1 * D.jrows * sizeof(cplx<double>);
  const size_t stage_dc =
      (size_t)corr_stage_elems(2 * D.nstaged, corr_plane_stride(cd), (int)D.csize) * D.csize +
      (size_t)D.njlo * cd * D.jrows * sizeof(cplx<double>);
  const size_t red = (size_t)ASM_THREADS * CORR_RED_ROWS * sizeof(cplx<double>);
  return steps + std::max(std::max(stage, stage_dc), red);
}

// Default chunk: the largest multiple of the item lanes whose LDS fits 80 KB
// (two blocks per CU); sfft_autotune may pick another.
int corr_default_c1(const Derived& D) {
  const int P1 = D.Py / P2;
  const int lanes = D.corr_lanes;
  constexpr size_t budget = 80 * 1024;
  int C1 = P1;
  while (C1 > 1 && corr_lds_bytes(D, C1) > budget) --C1;
  if (C1 >= lanes) C1 = (C1 / lanes) * lanes;   // whole rounds of the item lanes
  return std::max(C1, 1);
}

template <typename T>
int launch_corr(sfft_plan_s* p, const AsmParams& A, const PairSet& PS, int np, int C1, bool timed) {
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  const size_t lds = corr_lds_bytes(D, C1);
  auto kfn = D.jrows == JROWS_WIDE ? corr_kernel<T, ASM_THREADS, JROWS_WIDE> : corr_kernel<T, ASM_THREADS, JROWS_NARROW>;
  HIP_TRY(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (timed) p->timer.begin(SFFT_STAGE_CORR, s);
  kfn<<<dim3(D.H, 1, np), ASM_THREADS, lds, s>>>(A, PS, ws_offsets(D, p->Lo), C1, corr_dc_chunk(C1));
  LAUNCH_CHECK();
  if (timed) p->timer.end(s);
  return SFFT_OK;
}

// moments reduction and the Omega/beta gather (both assembly routes)
int gather_impl(sfft_plan_s* p, const AsmParams& A, const PairSet& PS, int np) {
  const Derived& D = p->D;
  const WsOff O = ws_offsets(D, p->Lo);
  hipStream_t s = p->stream;
  p->timer.begin(SFFT_STAGE_GATHER, s);
  moments_reduce_kernel<ASM_THREADS><<<dim3(D.nb * D.nb + D.nb + D.nmu, 1, np), ASM_THREADS, 0, s>>>(A, PS, O);
  LAUNCH_CHECK();
  GatherParams G = D.gp;
  G.kb_dense = D.route == ROUTE_FFT ? 1 : 0;
  if (D.rhs_only) {
    gather_beta_kernel<<<dim3((D.n + 255) / 256, 1, np), 256, 0, s>>>(G, PS, O);
  } else {
    if (G.kb_dense) {
      const KbParams K = kb_params(p, A.ld);
      kb_combine_kernel<<<dim3((D.nkk * D.nb + 255) / 256, 1, np), 256, 0, s>>>(K, PS, O);
      LAUNCH_CHECK();
    }
    gather_kernel<<<dim3((D.n + 255) / 256, D.n, np), 256, 0, s>>>(G, PS, O);
  }
  LAUNCH_CHECK();
  p->timer.end(s);
  return SFFT_OK;
}

// Output-masked fit: the excluded pixels' rows taken out of the assembled
// (zero-filled) Omega of the np pairs of PS.
template <typename T>
int omask_impl(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld) {
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  const OmaskParams P = om_params(p, ld);
  const OmaskOff O = om_off(p);
  p->timer.begin(SFFT_STAGE_OUTMASK, s);
  om_planes_kernel<T><<<dim3((unsigned)((P.plane + 255) / 256), D.nk, np), 256, 0, s>>>(P, PS, O);
  LAUNCH_CHECK();
  // the transform route has listed the excluded pixels already (template-background block)
  if (D.route != ROUTE_FFT) {
    const int st = om_list_impl(p, PS, np, ld);
    if (st != SFFT_OK) return st;
  }
  om_syrk_kernel<<<dim3(P.ntile * (P.ntile + 1) / 2, 1, np), 256, 0, s>>>(P, PS, O);
  LAUNCH_CHECK();
  p->timer.end(s);
  return SFFT_OK;
}

// The template-background block of the transform route: excluded-pixel list,
// the excluded-pixel sums T(c)(u), reduced over the chunks (kb_combine then
// forms the block in the gather, after the template moments).
template <typename T>
int kb_impl(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld) {
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  int st = om_list_impl(p, PS, np, ld);
  if (st != SFFT_OK) return st;
  const KbParams K = kb_params(p, ld);
  const WsOff O = ws_offsets(D, p->Lo);
  const int L2 = D.L * D.L;
  {
    const int64_t nb_px = (int64_t)2 * D.w * (D.nx + 2 * D.w) + (int64_t)2 * D.w * D.ny;
    if (nb_px > 0) {
      kb_pad_kernel<T><<<dim3((unsigned)((nb_px + 255) / 256), 1, np), 256, 0, s>>>(K, PS, O);
      LAUNCH_CHECK();
    }
  }
  // KB_LPT lags per thread, in blocks of whole waves of at most 512 threads
  const int nth = std::min(KB_MAX_THREADS, ((L2 + KB_LPT * 64 - 1) / (KB_LPT * 64)) * 64);
  const dim3 g(KB_CHUNKS, (L2 + KB_LPT * nth - 1) / (KB_LPT * nth), np);
  switch (D.dk + D.db) {
#define KB_CASE(DS)                                                                  \
  case DS:                                                                           \
    kb_mask_kernel<T, DS><<<g, nth, 0, s>>>(K, PS, O, om_off(p));                    \
    break;
    KB_CASE(0) KB_CASE(1) KB_CASE(2) KB_CASE(3) KB_CASE(4) KB_CASE(5) KB_CASE(6) KB_CASE(7) KB_CASE(8)
#undef KB_CASE
    default:
      return SFFT_EINVAL;
  }
  LAUNCH_CHECK();
  kb_reduce_kernel<<<dim3((D.nmu * L2 + 255) / 256, 1, np), 256, 0, s>>>(K, PS, O);
  LAUNCH_CHECK();
  return SFFT_OK;
}

// Assembly of Omega and beta for the np pairs of PS, which share the plan
// p's descriptor and row pitch (p is one of them: its sizes, tables and
// workspace offsets are every pair's).
template <typename T>
int build_core(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld);

template <typename T>
int build_impl(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld) {
  int st = build_core<T>(p, PS, np, ld);
  // a pair that shares its template uses its owner's (corrected) Omega, and
  // its beta needs no correction (the target is zero at excluded pixels)
  if (st == SFFT_OK && p->D.omask && !p->D.rhs_only) st = omask_impl<T>(p, PS, np, ld);
  return st;
}

template <typename T>
int build_core(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld) {
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  const AsmParams A = asm_params(p, ld);
  const WsOff O = ws_offsets(D, p->Lo);

  clear_nonfinite_kernel<<<dim3(1, 1, np), 64, 0, s>>>(PS, O);
  LAUNCH_CHECK();
  p->timer.begin(SFFT_STAGE_MOMENTS, s);
  switch (D.db * (MAX_DEG + 1) + D.dk) {
#define MOM_CASE(DBV, DKV)                                                                        \
  case DBV * (MAX_DEG + 1) + DKV:                                                                 \
    moments_kernel<T, ASM_THREADS, DBV, DKV><<<dim3(D.ny, 1, np), ASM_THREADS, 0, s>>>(A, PS, O); \
    break;
#define MOM_ROW(DBV) MOM_CASE(DBV, 0) MOM_CASE(DBV, 1) MOM_CASE(DBV, 2) MOM_CASE(DBV, 3) MOM_CASE(DBV, 4)
    MOM_ROW(0) MOM_ROW(1) MOM_ROW(2) MOM_ROW(3) MOM_ROW(4)
#undef MOM_ROW
#undef MOM_CASE
    default:
      return SFFT_EINVAL;
  }
  LAUNCH_CHECK();
  p->timer.end(s);

  constexpr int RN = std::is_same<T, float>::value ? ROW_NMAX_F32 : ROW_NMAX_F64;
  if (D.route == ROUTE_MFMA) {
    // lag windows as FP64 matrix-core products, partial per (column chunk, row band)
    const int nparts = D.mfma_nxc * D.mfma_nband;
    p->timer.begin(SFFT_STAGE_CORR, s);
    mfma_win_kernel<T><<<dim3((unsigned)D.mtiles.size(), (unsigned)nparts, np), MFMA_THREADS, 0, s>>>(
        A, PS, O, D.nwin, D.mfma_nxc, D.mfma_band);
    LAUNCH_CHECK();
    p->timer.end(s);
    p->timer.begin(SFFT_STAGE_ROW_WIN, s);
    dir_reduce_kernel<<<dim3((D.nwin + 255) / 256, 1, np), 256, 0, s>>>(PS, O, nparts, D.nwin);
    LAUNCH_CHECK();
    p->timer.end(s);
    return gather_impl(p, A, PS, np);
  }
  if (D.route == ROUTE_DIRECT) {
    p->timer.begin(SFFT_STAGE_CORR, s);
    direct_win_kernel<T, ASM_THREADS><<<dim3((unsigned)D.drows.size(), (unsigned)D.dir_nband, np), ASM_THREADS, 0, s>>>(
        A, PS, O, D.nwin);
    LAUNCH_CHECK();
    p->timer.end(s);
    p->timer.begin(SFFT_STAGE_ROW_WIN, s);
    dir_reduce_kernel<<<dim3((D.nwin + 255) / 256, 1, np), 256, 0, s>>>(PS, O, D.dir_nband, D.nwin);
    LAUNCH_CHECK();
    p->timer.end(s);
    return gather_impl(p, A, PS, np);
  }
  {
    const size_t lds = (size_t)row_pass_lds(RN, D.lgPx - 1) * sizeof(cplx<T>);
    const int grid = ((D.nrowblk + 7) / 8) * 8;   // whole XCD rounds for the remap
    p->timer.begin(SFFT_STAGE_ROW_FWD, s);
    switch (D.lgPx - 1) {
#define ROW_CASE(LG)                                                                                       \
  case LG: {                                                                                               \
    auto kfn = row_fwd_kernel<T, FFT_THREADS, RN, LG>;                                                     \
    HIP_TRY(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    kfn<<<dim3(grid, 1, np), FFT_THREADS, lds, s>>>(A, PS, O);                                             \
    break;                                                                                                 \
  }
      ROW_CASE(5) ROW_CASE(6) ROW_CASE(7) ROW_CASE(8) ROW_CASE(9) ROW_CASE(10) ROW_CASE(11)
      default:
        return SFFT_EINVAL;
#undef ROW_CASE
    }
    LAUNCH_CHECK();
    p->timer.end(s);
  }
  {
    const size_t lds = (size_t)lds_padded_size(2 * D.Py) * sizeof(cplx<T>);
    const int nblk = (D.H / 2) * (D.nbase - D.base_lo);
    const int grid = ((nblk + 7) / 8) * 8;
    p->timer.begin(SFFT_STAGE_COL_FWD, s);
    switch (D.lgPy) {
#define COL_CASE(LG)                                                                                        \
  case LG: {                                                                                                \
    auto kfn = col_fwd_kernel<T, FFT_THREADS, COL_NMAX, LG, COL_LGM>;                                       \
    HIP_TRY(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));  \
    kfn<<<dim3(grid, 1, np), FFT_THREADS, lds, s>>>(A, PS, O);                                              \
    break;                                                                                                  \
  }
      COL_CASE(6) COL_CASE(7) COL_CASE(8) COL_CASE(9) COL_CASE(10) COL_CASE(11) COL_CASE(12)
      default:
        return SFFT_EINVAL;
#undef COL_CASE
    }
    LAUNCH_CHECK();
    p->timer.end(s);
  }
  {
    const int st = launch_corr<T>(p, A, PS, np, p->corr_c1 > 0 ? p->corr_c1 : corr_default_c1(D), true);
    if (st != SFFT_OK) return st;
  }
  p->timer.begin(SFFT_STAGE_ROW_WIN, s);
  {
    const int nrows = (int)D.wrows.size();
    row_win_kernel<WIN_THREADS, WIN_IMAX><<<dim3(((nrows + 7) / 8) * 8, 1, np), WIN_THREADS, 0, s>>>(A, PS, O, nrows);
  }
  LAUNCH_CHECK();
  p->timer.end(s);
  if (!D.rhs_only) {
    p->timer.begin(SFFT_STAGE_GATHER, s);
    const int st = kb_impl<T>(p, PS, np, ld);
    p->timer.end(s);
    if (st != SFFT_OK) return st;
  }
  return gather_impl(p, A, PS, np);
}

// The solve of a set of pairs: the first nfac jobs own a factor each; all
// nsub jobs (those, then one per constraint column of the pairs with a
// constant photometric ratio) are substituted and refined against them; the
// nratio projection jobs then combine each such pair's columns.
struct SolveTable {
  const SolveJob* jobs;
  int nfac, nsub;
  const RatioJob* rjobs;
  int nratio;
};

// FP64 Cholesky, triangular solves and refinement for a table of jobs: one
// launch per block step serves every pair of the table.
int solve_jobs(hipStream_t s, const SolveTable& T, int max_n, int max_nblk, int refine, StageTimer* tm) {
  const SolveJob* jobs = T.jobs;
  const int njobs = T.nfac;
  tm->begin(SFFT_STAGE_FACTOR, s);
  reset_info_kernel<<<(njobs + 63) / 64, 64, 0, s>>>(jobs, njobs);
  LAUNCH_CHECK();
  {
    dim3 g((max_n + 3) / 4, njobs);   // one wave per row
    copy_omega_kernel<<<g, 256, 0, s>>>(jobs);
    LAUNCH_CHECK();
  }
  // diagonal block 0; each next diagonal block is factored inside the
  // trailing update that completes it.  Block steps go in pairs: panel k,
  // the update of block column k + 1 alone (and its factor), panel k + 1,
  // then one rank-128 update of the rest with both panels (the trailing
  // matrix is read and written once per two steps); a last odd step alone.
  potrf_diag_kernel<<<njobs, 256, 0, s>>>(jobs, 0);
  LAUNCH_CHECK();
  auto syrk = [&](int k, int npanel, int colonly) -> int {
    const int T = max_nblk - k - npanel;
    const int ntile = colonly ? T : T * (T + 1) / 2;
    const int grid = njobs + ((njobs * (ntile - 1) + 7) / 8) * 8;   // diagonal blocks, then whole XCD rounds
    syrk_kernel<<<grid, 256, 0, s>>>(jobs, k, njobs, ntile, 1, npanel, colonly);
    LAUNCH_CHECK();
    return SFFT_OK;
  };
  for (int k = 0; k + 1 < max_nblk;) {
    trsm_kernel<<<dim3(max_nblk - k - 1, njobs), 256, 0, s>>>(jobs, k);
    LAUNCH_CHECK();
    if (k + 2 < max_nblk) {
      int st = syrk(k, 1, 1);
      if (st != SFFT_OK) return st;
      trsm_kernel<<<dim3(max_nblk - k - 2, njobs), 256, 0, s>>>(jobs, k + 1);
      LAUNCH_CHECK();
      st = syrk(k, 2, 0);
      if (st != SFFT_OK) return st;
      k += 2;
    } else {
      const int st = syrk(k, 1, 0);
      if (st != SFFT_OK) return st;
      k += 1;
    }
  }
  tm->end(s);
  tm->begin(SFFT_STAGE_SOLVE, s);
  const int nsub = T.nsub;
  if (T.nratio > 0) {
    ratio_rhs_kernel<<<dim3((max_n + 255) / 256, T.nratio), 256, 0, s>>>(T.rjobs);
    LAUNCH_CHECK();
  }
  // blocked right-looking substitutions: one launch per block step, one
  // block per row block still to be updated
  auto solve_lower = [&](int which) -> int {
    for (int k = 0; k < max_nblk; ++k) {
      trsv_lower_step_kernel<<<dim3(max_nblk - k, nsub), 256, 0, s>>>(jobs, k, which);
      LAUNCH_CHECK();
    }
    return SFFT_OK;
  };
  auto solve_upper = [&](int which) -> int {
    for (int k = max_nblk - 1; k >= 0; --k) {
      trsv_upper_step_kernel<<<dim3(k + 1, nsub), 256, 0, s>>>(jobs, k, which);
      LAUNCH_CHECK();
    }
    return SFFT_OK;
  };
  int st = solve_lower(0);
  if (st == SFFT_OK) st = solve_upper(0);
  if (st != SFFT_OK) return st;
  for (int it = 0; it < refine; ++it) {
    residual_jobs_kernel<<<dim3((max_n + 3) / 4, nsub), 256, 0, s>>>(jobs);
    LAUNCH_CHECK();
    st = solve_lower(1);
    if (st == SFFT_OK) st = solve_upper(1);
    if (st != SFFT_OK) return st;
    axpy_jobs_kernel<<<dim3((max_n + 255) / 256, nsub), 256, 0, s>>>(jobs);
    LAUNCH_CHECK();
  }
  if (T.nratio > 0) {
    ratio_project_kernel<<<T.nratio, 256, 0, s>>>(T.rjobs);
    LAUNCH_CHECK();
  }
  tm->end(s);
  return SFFT_OK;
}

// A plan's solve job; a plan that shares its template takes the normal
// matrix, the factor and the outcome of the plan that owns the template.
SolveJob job_of(sfft_plan_s* p) {
  const Layout& Lo = p->Lo;
  const sfft_plan_s* t = p->tplan != nullptr ? p->tplan : p;
  SolveJob J;
  J.F = t->at<double>(t->Lo.F);
  J.Linv = t->at<double>(t->Lo.Linv);
  J.omega = t->at<double>(t->Lo.omega);
  J.beta = p->at<double>(Lo.beta);
  J.theta = p->at<double>(Lo.theta);
  J.y = p->at<double>(Lo.y);
  J.r = p->at<double>(Lo.r);
  J.d = p->at<double>(Lo.d);
  J.w = p->at<double>(Lo.w);
  J.info = t->at<int>(t->Lo.flags);
  J.n = p->D.n;
  J.nblk = p->D.nblk;
  return J;
}

// A plan's constraint-column jobs (constant photometric ratio, D.nratio of
// them, sharing its factor) and its projection job.  The ratio region holds
// six arrays of nratio x n: C^T, Z, and the y, r, d, w vectors of the jobs.
void ratio_jobs_of(sfft_plan_s* p, std::vector<SolveJob>* cj, RatioJob* rj) {
  const Derived& D = p->D;
  const int nc = D.nratio, n = D.n;
  double* base = p->at<double>(p->Lo.ratio);
  auto arr = [&](int k) { return base + (size_t)k * nc * n; };
  const SolveJob J0 = job_of(p);
  for (int c = 0; c < nc; ++c) {
    SolveJob J = J0;
    J.beta = arr(0) + (size_t)c * n;
    J.theta = arr(1) + (size_t)c * n;
    J.y = arr(2) + (size_t)c * n;
    J.r = arr(3) + (size_t)c * n;
    J.d = arr(4) + (size_t)c * n;
    J.w = arr(5) + (size_t)c * n;
    cj->push_back(J);
  }
  rj->theta = J0.theta;
  rj->Z = arr(1);
  rj->E = arr(0);
  rj->info = J0.info;
  rj->n = n;
  rj->L2 = D.L * D.L;
  rj->nc = nc;
}

// A single plan's solve tables in its workspace: [its job, constraint jobs] and
// the projection job.  Uploaded on `s` from `host` (kept alive by the caller
// until the stream has run the copies).
int upload_solve_tables(sfft_plan_s* p, hipStream_t s, std::vector<SolveJob>* host, RatioJob* rj) {
  host->assign(1, job_of(p));
  ratio_jobs_of(p, host, rj);
  HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.job), host->data(), host->size() * sizeof(SolveJob),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.rjob), rj, sizeof(RatioJob), hipMemcpyHostToDevice, s));
  return SFFT_OK;
}

SolveTable plan_table(sfft_plan_s* p) {
  SolveTable T;
  T.jobs = p->at<SolveJob>(p->Lo.job);
  T.nfac = 1;
  T.nsub = 1 + p->D.nratio;
  T.rjobs = p->at<RatioJob>(p->Lo.rjob);
  T.nratio = p->D.nratio > 0 ? 1 : 0;
  return T;
}

// Convolve-and-subtract for the np pairs of PS (same descriptor and row pitch
// as the plan p): D = S - model - background with theta from PS.coeffs; with
// apply_only, the model K * R alone (PS.tmpl = the image, PS.coeffs = the
// kernel coefficients, no science image).
// With shared_rows, the pairs' template row spectra are those of the pairs
// whose templates they share (PS.tws), already formed: the row pass is skipped.
template <typename T>
int subtract_impl(sfft_plan_s* p, const PairSet& PS, int np, int64_t ld, bool apply_only = false,
                  bool shared_rows = false) {
  const Derived& D = p->D;
  const WsOff O = ws_offsets(D, p->Lo);
  hipStream_t s = p->stream;
  p->timer.begin(SFFT_STAGE_SUBTRACT, s);
  // columns the circular x-convolution cannot produce exactly: [0, xl) and
  // [xr, nx), at most w on each side (xr - xl >= nx - 2w > 0 for every valid plan)
  const int xl = std::max(0, std::min(D.nx, D.w - (D.Px - D.nx)));
  const int xr = std::max(xl, std::min(D.nx, D.Px - D.w));
  SpecParams S;
  std::memset(&S, 0, sizeof(S));
  S.ny = D.ny;
  S.nx = D.nx;
  S.w = D.w;
  S.nk = D.nk;
  S.nb = D.nb;
  S.lgPx = D.lgPx;
  S.H = D.H;
  S.ld = ld;
  S.rows_per_block = sub_row_rows(SUB_NMAX, D.lgPx - 1);   // the kernels' own constant
  S.nrowblk = (D.ny + S.rows_per_block - 1) / S.rows_per_block;
  S.sx = 2.0 / (double)(D.nx - 1);
  S.sy = 2.0 / (double)(D.ny - 1);
  S.xp32 = sizeof(T) == sizeof(float);   // FP32C: x-power spectra p >= 1 as complex64
  for (int i = 0; i < D.nk; ++i) {
    S.kpx[i] = D.kpoly.px[i];
    S.kqy[i] = D.kpoly.qy[i];
  }
  for (int i = 0; i < D.nb; ++i) {
    S.bpx[i] = D.bpoly.px[i];
    S.bqy[i] = D.bpoly.qy[i];
  }
  {
    // filters G and the border kernel k' in one launch
    const int L2 = D.L * D.L;
    const int ngb = ((D.H + 1 + PREP_THREADS - 1) / PREP_THREADS) * D.L;
    const int nkb = (D.nk * L2 + PREP_THREADS - 1) / PREP_THREADS;
    sub_prep_kernel<<<dim3(ngb + nkb, 1, np), PREP_THREADS, 0, s>>>(S, PS, O, ngb);
    LAUNCH_CHECK();
  }
  const size_t lds = (size_t)lds_padded_size(S.rows_per_block * D.H) * sizeof(cplx<double>);
  switch (shared_rows ? -1 : D.lgPx - 1) {
    case -1:
      break;
#define SUBF_CASE(LG)                                                                                       \
  case LG: {                                                                                                \
    auto kf = sub_rowfwd_kernel<T, FFT_THREADS, SUB_NMAX, LG>;                                              \
    HIP_TRY(hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));   \
    kf<<<dim3(S.nrowblk, 1, np), FFT_THREADS, lds, s>>>(S, PS, O, D.dk + 1);                                \
    break;                                                                                                  \
  }
    SUBF_CASE(5) SUBF_CASE(6) SUBF_CASE(7) SUBF_CASE(8) SUBF_CASE(9) SUBF_CASE(10) SUBF_CASE(11)
    default:
      return SFFT_EINVAL;
#undef SUBF_CASE
  }
  LAUNCH_CHECK();
  {
    const int nconv = ((D.H + 1 + 63) / 64) * ((D.ny + SUBC_RB - 1) / SUBC_RB);
    const int g = ((nconv + 7) / 8) * 8;   // whole XCD rounds for the remap
    const size_t lds_c = sub_conv_lds_bytes(D.w);
    switch (D.w) {
#define CONV_CASE(WV)                                                                                          \
  case WV: {                                                                                                   \
    auto kc = sub_conv_kernel<WV>;                                                                             \
    HIP_TRY(hipFuncSetAttribute((const void*)kc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_c));   \
    kc<<<dim3(g, 1, np), 64 * SUBC_WAVES, lds_c, s>>>(S, PS, O);                                               \
    break;                                                                                                     \
  }
      CONV_CASE(0) CONV_CASE(1) CONV_CASE(2) CONV_CASE(3) CONV_CASE(4) CONV_CASE(5) CONV_CASE(6) CONV_CASE(7)
      CONV_CASE(8) CONV_CASE(9) CONV_CASE(10) CONV_CASE(11) CONV_CASE(12) CONV_CASE(13) CONV_CASE(14) CONV_CASE(15)
#undef CONV_CASE
      default:
        return SFFT_EINVAL;
    }
    LAUNCH_CHECK();
  }
  // border pixels, one wave each, in the leading blocks of the inverse pass
  const int64_t nbandpx = (int64_t)(xl + (D.nx - xr)) * D.ny;
  const int nbandblk = (int)((nbandpx + FFT_THREADS / 64 - 1) / (FFT_THREADS / 64));
  switch (D.lgPx - 1) {
#define SUBI_CASE(LG)                                                                                       \
  case LG: {                                                                                                \
    auto ki = sub_rowinv_kernel<T, FFT_THREADS, SUB_NMAX, LG>;                                              \
    HIP_TRY(hipFuncSetAttribute((const void*)ki, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));   \
    ki<<<dim3(nbandblk + S.nrowblk, 1, np), FFT_THREADS, lds, s>>>(S, PS, O, xl, xr, nbandblk,              \
                                                                   apply_only ? 1 : 0);                     \
    break;                                                                                                  \
  }
    SUBI_CASE(5) SUBI_CASE(6) SUBI_CASE(7) SUBI_CASE(8) SUBI_CASE(9) SUBI_CASE(10) SUBI_CASE(11)
    default:
      return SFFT_EINVAL;
#undef SUBI_CASE
  }
  LAUNCH_CHECK();
  p->timer.end(s);
  return SFFT_OK;
}

PairSet pair_set_one(const sfft_plan_s* p, const void* sci, const void* tmpl, const uint8_t* mask,
                     const double* coeffs, void* diff, int32_t* info) {
  PairSet S;
  std::memset(&S, 0, sizeof(S));
  S.sci[0] = sci;
  S.tmpl[0] = tmpl;
  S.mask[0] = mask;
  S.ws[0] = p->ws;
  S.tws[0] = p->ws;
  S.coeffs[0] = const_cast<double*>(coeffs);
  S.diff[0] = diff;
  S.info[0] = info;
  return S;
}

}  // namespace

extern "C" {

int sfft_num_coeffs(const sfft_desc* d, int64_t* n) {
  if (n == nullptr) return SFFT_EINVAL;
  const int st = validate(d);
  if (st != SFFT_OK) return st;
  const int64_t L = 2 * d->w + 1;
  *n = L * L * ((d->dk + 1) * (d->dk + 2) / 2) + (d->db + 1) * (d->db + 2) / 2;
  return SFFT_OK;
}

int sfft_workspace_bytes(const sfft_desc* d, size_t* bytes) {
  if (bytes == nullptr) return SFFT_EINVAL;
  Derived* D = new (std::nothrow) Derived();   // its tables are held inline: too large for the stack
  if (D == nullptr) return SFFT_ENOMEM;
  const int st = derive(d, D);
  if (st == SFFT_OK) *bytes = layout_of(*D).total;
  delete D;
  return st;
}

// A plan of one pair; with rhs_only, a batch member that forms only its
// right-hand side (its template and mask are another member's).
static int plan_create(const sfft_desc* d, void* hip_stream, void* workspace, size_t workspace_bytes, bool rhs_only,
                       sfft_handle* out) {
  if (out == nullptr) return SFFT_EINVAL;
  *out = nullptr;
  sfft_plan_s* p = new (std::nothrow) sfft_plan_s();
  if (p == nullptr) return SFFT_ENOMEM;
  int st = derive(d, &p->D, rhs_only);
  if (st != SFFT_OK) {
    delete p;
    return st;
  }
  p->desc = *d;
  p->Lo = layout_of(p->D);
  if (rhs_only) {
    // the layout of a full plan of the same descriptor (its tables are the
    // larger ones), so that every buffer a sharing pair reads from its
    // owner's workspace sits at the offset of its own
    Derived* Df = new (std::nothrow) Derived();   // tables held inline: too large for the stack
    if (Df == nullptr) {
      delete p;
      return SFFT_ENOMEM;
    }
    st = derive(d, Df, false);
    if (st == SFFT_OK) p->Lo = layout_of(*Df);
    delete Df;
    if (st != SFFT_OK) {
      delete p;
      return st;
    }
  }
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  p->built = false;
  if (workspace != nullptr) {
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {   // the carve-up keeps 256-byte alignment
      delete p;
      return SFFT_EINVAL;
    }
    if (workspace_bytes < p->Lo.total) {
      delete p;
      return SFFT_ENOMEM;
    }
    p->ws = reinterpret_cast<unsigned char*>(workspace);
    p->owns_ws = false;
  } else {
    void* m = nullptr;
    if (hipMalloc(&m, p->Lo.total) != hipSuccess) {
      (void)hipGetLastError();
      delete p;
      return SFFT_ENOMEM;
    }
    p->ws = reinterpret_cast<unsigned char*>(m);
    p->owns_ws = true;
  }
  p->tw64h.resize(TW_N);
  p->tw32h.resize(TW_N);
  twiddle_tables(p->tw64h.data(), p->tw32h.data());
  hipStream_t s = p->stream;
  bool ok = true;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.tw64), p->tw64h.data(), TW_N * sizeof(cplx<double>), hipMemcpyHostToDevice,
                       s) == hipSuccess;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.tw32), p->tw32h.data(), TW_N * sizeof(cplx<float>), hipMemcpyHostToDevice,
                       s) == hipSuccess;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.items), p->D.items.data(), p->D.items.size() * sizeof(CorrItem),
                       hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.wrows), p->D.wrows.data(), p->D.wrows.size() * sizeof(WinRow),
                       hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.drows), p->D.drows.data(), p->D.drows.size() * sizeof(DirectRow),
                       hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(p->at<void>(p->Lo.mtiles), p->D.mtiles.data(), p->D.mtiles.size() * sizeof(MfmaTile),
                       hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= upload_solve_tables(p, s, &p->jobs_host, &p->rjob_host) == SFFT_OK;
  // host staging vectors of pageable memory: make sure the copies are done before returning
  ok &= hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    if (p->owns_ws) (void)hipFree(p->ws);
    delete p;
    return SFFT_EHIP;
  }
  *out = p;
  return SFFT_OK;
}

int sfft_plan(const sfft_desc* d, void* hip_stream, void* workspace, size_t workspace_bytes, sfft_handle* out) {
  RoctxScope range_("sfft_plan");
  return plan_create(d, hip_stream, workspace, workspace_bytes, false, out);
}

int sfft_build_system(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld) {
  RoctxScope range_("sfft_build_system");
  if (p == nullptr || p->is_batch || sci == nullptr || tmpl == nullptr || ld < p->D.nx) return SFFT_EINVAL;
  const PairSet PS = pair_set_one(p, sci, tmpl, mask, nullptr, nullptr, nullptr);
  const int st = p->D.mode == SFFT_MODE_F64 ? build_impl<double>(p, PS, 1, ld) : build_impl<float>(p, PS, 1, ld);
  if (st == SFFT_OK) p->built = true;
  return st;
}

int sfft_get_system(sfft_handle p, double* omega, double* rhs) {
  if (p == nullptr || p->is_batch) return SFFT_EINVAL;
  if (!p->built) return SFFT_ESTATE;
  const size_t n = (size_t)p->D.n;
  if (omega != nullptr)
    HIP_TRY(hipMemcpyAsync(omega, p->at<double>(p->Lo.omega), n * n * sizeof(double), hipMemcpyDeviceToDevice,
                           p->stream));
  if (rhs != nullptr)
    HIP_TRY(hipMemcpyAsync(rhs, p->at<double>(p->Lo.beta), n * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  return SFFT_OK;
}

int sfft_solve(sfft_handle p, double* coeffs, int32_t* info) {
  RoctxScope range_("sfft_solve");
  if (p == nullptr || coeffs == nullptr || p->is_batch) return SFFT_EINVAL;
  if (!p->built) return SFFT_ESTATE;
  const Derived& D = p->D;
  const Layout& Lo = p->Lo;
  hipStream_t s = p->stream;
  int st = solve_jobs(s, plan_table(p), D.n, D.nblk, D.refine, &p->timer);
  if (st != SFFT_OK) return st;
  copy_out_kernel<<<(D.n + 255) / 256, 256, 0, s>>>(p->at<double>(Lo.theta), coeffs, D.n, p->at<int>(Lo.flags), info);
  LAUNCH_CHECK();
  return SFFT_OK;
}

int sfft_residual(sfft_handle p, const double* coeffs, double* rho) {
  RoctxScope range_("sfft_residual");
  if (p == nullptr || p->is_batch || coeffs == nullptr || rho == nullptr) return SFFT_EINVAL;
  if (!p->built) return SFFT_ESTATE;
  const Derived& D = p->D;
  const Layout& Lo = p->Lo;
  hipStream_t s = p->stream;
  residual_kernel<<<(D.n + 3) / 4, 256, 0, s>>>(p->at<double>(Lo.omega), D.n, p->at<double>(Lo.beta), coeffs,
                                                p->at<double>(Lo.r));
  LAUNCH_CHECK();
  norm_ratio_kernel<<<1, 256, 0, s>>>(p->at<double>(Lo.r), p->at<double>(Lo.beta), D.n, rho);
  LAUNCH_CHECK();
  return SFFT_OK;
}

int sfft_fit_background(sfft_handle p, double* coeffs) {
  RoctxScope range_("sfft_fit_background");
  if (p == nullptr || p->is_batch || coeffs == nullptr) return SFFT_EINVAL;
  if (!p->built) return SFFT_ESTATE;
  const Derived& D = p->D;
  if (D.nb > FITBG_MAX_NB) return SFFT_EINVAL;
  fit_background_kernel<<<1, 256, 0, p->stream>>>(p->at<double>(p->Lo.omega), D.n, D.nkk, p->at<double>(p->Lo.beta),
                                                  coeffs);
  LAUNCH_CHECK();
  return SFFT_OK;
}

int sfft_subtract(sfft_handle p, const void* sci, const void* tmpl, const double* coeffs, void* diff, int64_t ld) {
  RoctxScope range_("sfft_subtract");
  if (p == nullptr || p->is_batch || sci == nullptr || tmpl == nullptr || coeffs == nullptr || diff == nullptr || ld < p->D.nx)
    return SFFT_EINVAL;
  const PairSet PS = pair_set_one(p, sci, tmpl, nullptr, coeffs, diff, nullptr);
  return p->D.mode == SFFT_MODE_F64 ? subtract_impl<double>(p, PS, 1, ld) : subtract_impl<float>(p, PS, 1, ld);
}

int sfft_apply_kernel(sfft_handle p, const void* img, const double* kcoef, void* out, int64_t ld) {
  RoctxScope range_("sfft_apply_kernel");
  if (p == nullptr || p->is_batch || img == nullptr || kcoef == nullptr || out == nullptr || ld < p->D.nx ||
      img == out)
    return SFFT_EINVAL;
  const PairSet PS = pair_set_one(p, nullptr, img, nullptr, kcoef, out, nullptr);
  return p->D.mode == SFFT_MODE_F64 ? subtract_impl<double>(p, PS, 1, ld, true)
                                    : subtract_impl<float>(p, PS, 1, ld, true);
}

int sfft_decorrelation_kernel(sfft_handle p, const double* coeffs, const double* psf_sci, const double* psf_tmpl,
                              int32_t s, double sigma_sci, double sigma_tmpl, int32_t t, double* psi) {
  RoctxScope range_("sfft_decorrelation_kernel");
  if (p == nullptr || p->is_batch || coeffs == nullptr || psf_sci == nullptr || psf_tmpl == nullptr || psi == nullptr)
    return SFFT_EINVAL;
  if (s < 0 || s > DEC_MAXS || t < 0 || t > DEC_MAXS) return SFFT_EINVAL;
  if (!(sigma_sci > 0.0) || !(sigma_tmpl > 0.0) || !std::isfinite(sigma_sci) || !std::isfinite(sigma_tmpl))
    return SFFT_EINVAL;
  const Derived& D = p->D;
  DecParams Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.w = D.w;
  Q.nk = D.nk;
  Q.s = s;
  Q.t = t;
  Q.sx = 2.0 / (double)(D.nx - 1);
  Q.sy = 2.0 / (double)(D.ny - 1);
  Q.var_s = sigma_sci * sigma_sci;
  Q.var_r = sigma_tmpl * sigma_tmpl;
  for (int i = 0; i < D.nk; ++i) {
    Q.kpx[i] = D.kpoly.px[i];
    Q.kqy[i] = D.kpoly.qy[i];
  }
  // the grid spectrum Psi^ goes to the head of the spectra region (free between calls)
  double* spec = p->at<double>(p->Lo.U);
  decorr_spec_kernel<<<DEC_SPEC_BLOCKS, DEC_SPEC_THREADS, 0, p->stream>>>(
      Q, coeffs, psf_sci, psf_tmpl, p->at<cplx<double>>(p->Lo.tw64), spec);
  LAUNCH_CHECK();
  decorr_inv_kernel<<<(2 * t + 1) * (2 * t + 1), DEC_INV_THREADS, 0, p->stream>>>(
      Q, spec, p->at<cplx<double>>(p->Lo.tw64), psi);
  LAUNCH_CHECK();
  return SFFT_OK;
}

int sfft_status(sfft_handle p, int32_t* info_out, int32_t* nonfinite_out) {
  if (p == nullptr) return SFFT_EINVAL;
  HIP_TRY(hipStreamSynchronize(p->stream));
  int flags[2] = {0, 0};
  if (p->is_batch) {
    // worst outcome over the pairs: the first non-zero info, any non-finite flag
    for (sfft_plan_s* m : p->members) {
      int f[2] = {0, 0};
      HIP_TRY(hipMemcpy(f, m->at<int>(m->Lo.flags), sizeof(f), hipMemcpyDeviceToHost));
      if (m->tplan != nullptr)   // the factor's outcome is recorded by the template's owner
        HIP_TRY(hipMemcpy(f, m->tplan->at<int>(m->tplan->Lo.flags), sizeof(int), hipMemcpyDeviceToHost));
      if (flags[0] == 0) flags[0] = f[0];
      flags[1] |= f[1];
    }
  } else {
    HIP_TRY(hipMemcpy(flags, p->at<int>(p->Lo.flags), sizeof(flags), hipMemcpyDeviceToHost));
  }
  if (info_out) *info_out = flags[0];
  if (nonfinite_out) *nonfinite_out = flags[1];
  if (flags[1] != 0) return SFFT_ENONFINITE;
  if (flags[0] != 0) return SFFT_ENOTSPD;
  return SFFT_OK;
}

int sfft_timing_enable(sfft_handle p, int stage_mask) {
  if (p == nullptr || (stage_mask & ~SFFT_TIMING_ALL) != 0) return SFFT_EINVAL;
  const unsigned m = (unsigned)stage_mask;
  int timed = 0;
  for (int st = 0; st < SFFT_NUM_STAGES; ++st) timed += (m >> st) & 1u;
  auto setup = [&](StageTimer& t) {
    t.on = m != 0;
    t.mask = m;
    if (m != 0) t.reserve((size_t)timed * 2 * SFFT_TIMING_RESERVE);
  };
  setup(p->timer);
  for (sfft_plan_s* q : p->members) setup(q->timer);
  return SFFT_OK;
}

int sfft_timing_read(sfft_handle p, double* ms, int64_t* count) {
  if (p == nullptr) return SFFT_EINVAL;
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->timer.fold();
  for (sfft_plan_s* m : p->members) {
    m->timer.fold();
    for (int st = 0; st < SFFT_NUM_STAGES; ++st) {
      p->timer.ms[st] += m->timer.ms[st];
      p->timer.cnt[st] += m->timer.cnt[st];
      m->timer.ms[st] = 0.0;
      m->timer.cnt[st] = 0;
    }
  }
  for (int st = 0; st < SFFT_NUM_STAGES; ++st) {
    if (ms) ms[st] = p->timer.ms[st];
    if (count) count[st] = p->timer.cnt[st];
    p->timer.ms[st] = 0.0;
    p->timer.cnt[st] = 0;
  }
  return SFFT_OK;
}

void sfft_destroy(sfft_handle p) {
  if (p == nullptr) return;
  (void)hipStreamSynchronize(p->stream);
  p->timer.release();
  if (p->gexec != nullptr) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph != nullptr) (void)hipGraphDestroy(p->graph);
  for (sfft_plan_s* m : p->members) sfft_destroy(m);
  p->members.clear();
  if (p->jobs_dev != nullptr) (void)hipFree(p->jobs_dev);
  if (p->owns_ws && p->ws != nullptr) {
    (void)hipStreamSynchronize(p->stream);
    (void)hipFree(p->ws);
  }
  delete p;
}

int sfft_batch_workspace_bytes(const sfft_desc* descs, int32_t npairs, size_t* bytes) {
  if (descs == nullptr || bytes == nullptr || npairs <= 0) return SFFT_EINVAL;
  size_t tot = 0, njobs = 0, nratio = 0;
  for (int i = 0; i < npairs; ++i) {
    size_t b = 0;
    const int st = sfft_workspace_bytes(&descs[i], &b);
    if (st != SFFT_OK) return st;
    tot += b;
    const int nk = (descs[i].dk + 1) * (descs[i].dk + 2) / 2;
    const int nc = (descs[i].flags & SFFT_FLAG_CONST_RATIO) ? nk - 1 : 0;
    njobs += 1 + nc;
    nratio += nc > 0 ? 1 : 0;
  }
  // the job tables: every pair's jobs, then the projection jobs
  *bytes = tot + align256(njobs * sizeof(SolveJob)) + std::max<size_t>(1, nratio) * sizeof(RatioJob);
  return SFFT_OK;
}

// A batch plan; tmpl_of (may be null) names for each pair the pair whose
// template and mask it uses (itself, or an earlier pair that uses its own).
static int batch_create(const sfft_desc* descs, const int32_t* tmpl_of, int32_t npairs, void* hip_stream,
                        sfft_handle* out) {
  if (out == nullptr || descs == nullptr || npairs <= 0) return SFFT_EINVAL;
  *out = nullptr;
  for (int i = 0; i < npairs; ++i) {
    const int st = validate(&descs[i]);
    if (st != SFFT_OK) return st;
    // the batched solve runs one refinement schedule for every pair
    const int r0 = descs[0].refine_steps < 0 ? 1 : descs[0].refine_steps;
    const int ri = descs[i].refine_steps < 0 ? 1 : descs[i].refine_steps;
    if (ri != r0) return SFFT_EINVAL;
    if (tmpl_of != nullptr) {
      const int o = tmpl_of[i];
      if (o < 0 || o > i || tmpl_of[o] != o) return SFFT_EINVAL;
      if (o != i && std::memcmp(&descs[o], &descs[i], sizeof(sfft_desc)) != 0) return SFFT_EINVAL;
    }
  }
  sfft_plan_s* b = new (std::nothrow) sfft_plan_s();
  if (b == nullptr) return SFFT_ENOMEM;
  b->is_batch = true;
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->ws = nullptr;
  b->owns_ws = false;
  b->built = false;
  for (int i = 0; i < npairs; ++i) {
    const int o = tmpl_of != nullptr ? tmpl_of[i] : i;
    sfft_handle m = nullptr;
    const int st = plan_create(&descs[i], hip_stream, nullptr, 0, o != i, &m);
    if (st != SFFT_OK) {
      sfft_destroy(b);
      return st;
    }
    if (o != i) m->tplan = b->members[o];
    b->members.push_back(m);
    b->tmpl_of.push_back(o);
    b->max_n = std::max(b->max_n, m->D.n);
    b->max_nblk = std::max(b->max_nblk, m->D.nblk);
  }
  // jobs: the pairs that own a factor (their own template), then the pairs
  // that use another pair's factor, then the constraint-column jobs; one
  // projection job per pair with a constant photometric ratio
  for (sfft_plan_s* m : b->members)
    if (m->tplan == nullptr) b->jobs_host.push_back(job_of(m));
  b->nfac = (int)b->jobs_host.size();
  for (sfft_plan_s* m : b->members)
    if (m->tplan != nullptr) b->jobs_host.push_back(job_of(m));
  std::vector<RatioJob> rjobs;
  for (sfft_plan_s* m : b->members) {
    if (m->D.nratio == 0) continue;
    RatioJob rj;
    ratio_jobs_of(m, &b->jobs_host, &rj);
    rjobs.push_back(rj);
  }
  b->nsub = (int)b->jobs_host.size();
  b->nratio = (int)rjobs.size();
  const size_t job_bytes = align256(b->jobs_host.size() * sizeof(SolveJob));
  void* jd = nullptr;
  if (hipMalloc(&jd, job_bytes + std::max<size_t>(1, rjobs.size()) * sizeof(RatioJob)) != hipSuccess) {
    (void)hipGetLastError();
    sfft_destroy(b);
    return SFFT_ENOMEM;
  }
  b->jobs_dev = reinterpret_cast<SolveJob*>(jd);
  b->rjobs_dev = reinterpret_cast<RatioJob*>(static_cast<unsigned char*>(jd) + job_bytes);
  if (hipMemcpy(b->jobs_dev, b->jobs_host.data(), b->jobs_host.size() * sizeof(SolveJob), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (!rjobs.empty() &&
       hipMemcpy(b->rjobs_dev, rjobs.data(), rjobs.size() * sizeof(RatioJob), hipMemcpyHostToDevice) != hipSuccess)) {
    sfft_destroy(b);
    return SFFT_EHIP;
  }
  *out = b;
  return SFFT_OK;
}

int sfft_batch_plan(const sfft_desc* descs, int32_t npairs, void* hip_stream, sfft_handle* out) {
  RoctxScope range_("sfft_batch_plan");
  return batch_create(descs, nullptr, npairs, hip_stream, out);
}

int sfft_batch_plan_shared(const sfft_desc* descs, const int32_t* tmpl_of, int32_t npairs, void* hip_stream,
                           sfft_handle* out) {
  RoctxScope range_("sfft_batch_plan_shared");
  if (tmpl_of == nullptr) return SFFT_EINVAL;
  return batch_create(descs, tmpl_of, npairs, hip_stream, out);
}

int sfft_batch_run(sfft_handle b, const void* const* sci, const void* const* tmpl, const uint8_t* const* mask,
                   const int64_t* ld, double* const* coeffs, void* const* diff, int32_t* info) {
  RoctxScope range_("sfft_batch_run");
  if (b == nullptr || !b->is_batch || sci == nullptr || tmpl == nullptr || ld == nullptr || coeffs == nullptr ||
      diff == nullptr)
    return SFFT_EINVAL;
  const int np = (int)b->members.size();
  for (int i = 0; i < np; ++i)
    if (sci[i] == nullptr || tmpl[i] == nullptr || coeffs[i] == nullptr || diff[i] == nullptr ||
        ld[i] < b->members[i]->D.nx)
      return SFFT_EINVAL;
  // a pair that shares a template must be given that pair's template, mask
  // and row pitch; it assembles with the same route
  for (int i = 0; i < np; ++i) {
    const int o = b->tmpl_of[i];
    if (o == i) continue;
    const uint8_t* mi = mask ? mask[i] : nullptr;
    const uint8_t* mo = mask ? mask[o] : nullptr;
    if (tmpl[i] != tmpl[o] || mi != mo || ld[i] != ld[o]) return SFFT_EINVAL;
    b->members[i]->D.route = b->members[o]->D.route;
  }
  hipStream_t s = b->stream;
  // groups of pairs with the same descriptor, row pitch and correlation
  // chunk, at most MAX_GROUP each: every launch of a group serves all of its
  // pairs (pair = blockIdx.z), so small cutouts fill the device together and
  // large ones share one launch tail
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < np; ++i) {
    const sfft_plan_s* mi = b->members[i];
    bool placed = false;
    for (auto& g : groups) {
      const sfft_plan_s* mj = b->members[g[0]];
      if ((int)g.size() < MAX_GROUP && ld[g[0]] == ld[i] && mj->corr_c1 == mi->corr_c1 &&
          mj->D.rhs_only == mi->D.rhs_only && mj->D.route == mi->D.route &&
          std::memcmp(&mj->desc, &mi->desc, sizeof(sfft_desc)) == 0) {
        g.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) groups.push_back(std::vector<int>(1, i));
  }
  auto set_of = [&](const std::vector<int>& g) {
    PairSet S;
    std::memset(&S, 0, sizeof(S));
    for (size_t k = 0; k < g.size(); ++k) {
      const int i = g[k];
      S.sci[k] = sci[i];
      S.tmpl[k] = tmpl[i];
      S.mask[k] = mask ? mask[i] : nullptr;
      S.ws[k] = b->members[i]->ws;
      S.tws[k] = b->members[b->tmpl_of[i]]->ws;
      S.coeffs[k] = coeffs[i];
      S.diff[k] = diff[i];
      S.info[k] = info ? info + i : nullptr;
    }
    return S;
  };
  // assembly, one group at a time: the groups that own their templates
  // first (the others read their template spectra)
  for (int pass = 0; pass < 2; ++pass)
    for (const auto& g : groups) {
      sfft_plan_s* lead = b->members[g[0]];
      if (lead->D.rhs_only != (pass == 1)) continue;
      const PairSet PS = set_of(g);
      const int n = (int)g.size();
      const int st = lead->D.mode == SFFT_MODE_F64 ? build_impl<double>(lead, PS, n, ld[g[0]])
                                                   : build_impl<float>(lead, PS, n, ld[g[0]]);
      if (st != SFFT_OK) return st;
      for (int i : g) b->members[i]->built = true;
    }
  // one batched factorisation (one per template) and solve for all pairs
  SolveTable T;
  T.jobs = b->jobs_dev;
  T.nfac = b->nfac;
  T.nsub = b->nsub;
  T.rjobs = b->rjobs_dev;
  T.nratio = b->nratio;
  int st = solve_jobs(s, T, b->max_n, b->max_nblk, b->members[0]->D.refine, &b->timer);
  if (st != SFFT_OK) return st;
  for (const auto& g : groups) {
    const sfft_plan_s* lead = b->members[g[0]];
    copy_out_group_kernel<<<dim3((lead->D.n + 255) / 256, 1, (int)g.size()), 256, 0, s>>>(
        set_of(g), ws_offsets(lead->D, lead->Lo), lead->D.n);
    LAUNCH_CHECK();
  }
  // convolve-and-subtract, one group at a time: the template owners first
  // (their row spectra of the template serve the pairs that share it)
  for (int pass = 0; pass < 2; ++pass)
    for (const auto& g : groups) {
      sfft_plan_s* lead = b->members[g[0]];
      const bool shared = lead->D.rhs_only;
      if (shared != (pass == 1)) continue;
      const PairSet PS = set_of(g);
      const int n = (int)g.size();
      st = lead->D.mode == SFFT_MODE_F64 ? subtract_impl<double>(lead, PS, n, ld[g[0]], false, shared)
                                         : subtract_impl<float>(lead, PS, n, ld[g[0]], false, shared);
      if (st != SFFT_OK) return st;
    }
  return SFFT_OK;
}

int sfft_autotune(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld, int32_t* c1_out,
                  float* ms_out, int32_t cap, int32_t* count_out) {
  RoctxScope range_("sfft_autotune");
  if (p == nullptr || sci == nullptr || tmpl == nullptr || cap < 0) return SFFT_EINVAL;
  if (cap > 0 && (c1_out == nullptr || ms_out == nullptr)) return SFFT_EINVAL;
  if (p->is_batch && p->members.empty()) return SFFT_EINVAL;
  sfft_plan_s* t = p->is_batch ? p->members[0] : p;
  if (ld < t->D.nx) return SFFT_EINVAL;
  if (count_out) *count_out = 0;
  if (t->D.route != ROUTE_FFT) return SFFT_OK;   // only the transform route has a correlation chunk
  int st = sfft_build_system(t, sci, tmpl, mask, ld);
  if (st != SFFT_OK) return st;
  const Derived& D = t->D;
  const int P1 = D.Py / P2;
  std::vector<int> cand;
  for (int c = D.corr_lanes; c <= P1; c += D.corr_lanes)
    if (corr_lds_bytes(D, c) <= 160 * 1024) cand.push_back(c);
  if (cand.empty()) return SFFT_OK;
  while (cand.size() > 12) {   // keep every other candidate, always the smallest and largest
    std::vector<int> k;
    for (size_t i = 0; i < cand.size(); i += 2) k.push_back(cand[i]);
    if (k.back() != cand.back()) k.push_back(cand.back());
    cand.swap(k);
  }
  const AsmParams A = asm_params(t, ld);
  const PairSet PS = pair_set_one(t, sci, tmpl, mask, nullptr, nullptr, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SFFT_EHIP;
  }
  int best = 0;
  float best_ms = 0.0f;
  int n = 0;
  st = SFFT_OK;
  for (int c : cand) {
    constexpr int REPS = 3;
    for (int r = 0; r <= REPS && st == SFFT_OK; ++r) {
      if (r == 1) st = hipEventRecord(e0, t->stream) == hipSuccess ? SFFT_OK : SFFT_EHIP;
      if (st == SFFT_OK)
        st = D.mode == SFFT_MODE_F64 ? launch_corr<double>(t, A, PS, 1, c, false)
                                     : launch_corr<float>(t, A, PS, 1, c, false);
    }
    if (st == SFFT_OK) st = hipEventRecord(e1, t->stream) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    if (st == SFFT_OK) st = hipEventSynchronize(e1) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    float ms = 0.0f;
    if (st == SFFT_OK) st = hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    if (st != SFFT_OK) break;
    ms /= (float)REPS;
    if (n < cap) {
      c1_out[n] = c;
      ms_out[n] = ms;
    }
    ++n;
    if (best == 0 || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SFFT_OK) return st;
  t->corr_c1 = best;
  if (p->is_batch)
    for (sfft_plan_s* m : p->members)
      if (std::memcmp(&m->desc, &t->desc, sizeof(sfft_desc)) == 0) m->corr_c1 = best;
  if (count_out) *count_out = std::min(n, (int)cap);
  return SFFT_OK;
}

int sfft_autotune_route(sfft_handle p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld,
                        float* ms_out, int32_t* route_out) {
  RoctxScope range_("sfft_autotune_route");
  if (p == nullptr || sci == nullptr || tmpl == nullptr) return SFFT_EINVAL;
  if (p->is_batch && p->members.empty()) return SFFT_EINVAL;
  sfft_plan_s* t = p->is_batch ? p->members[0] : p;
  if (ld < t->D.nx) return SFFT_EINVAL;
  const Derived& D = t->D;
  const int r0 = D.route;
  const bool direct_ok = D.nx <= DIR_MAX_NX && 2 * D.w <= DIR_HWMAX;
  const bool tunable = (t->desc.flags & 3) == SFFT_FLAG_ASSEMBLY_AUTO;
  const PairSet PS = pair_set_one(t, sci, tmpl, mask, nullptr, nullptr, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SFFT_EHIP;
  }
  float ms[3] = {-1.0f, -1.0f, -1.0f};
  int st = SFFT_OK;
  int best = r0;
  for (int r = ROUTE_FFT; r <= ROUTE_MFMA && st == SFFT_OK; ++r) {
    if (r == ROUTE_DIRECT && !direct_ok) continue;
    t->D.route = r;
    constexpr int REPS = 3;
    for (int k = 0; k <= REPS && st == SFFT_OK; ++k) {   // one warm-up build, then REPS timed
      if (k == 1) st = hipEventRecord(e0, t->stream) == hipSuccess ? SFFT_OK : SFFT_EHIP;
      if (st == SFFT_OK)
        st = D.mode == SFFT_MODE_F64 ? build_impl<double>(t, PS, 1, ld) : build_impl<float>(t, PS, 1, ld);
    }
    if (st == SFFT_OK) st = hipEventRecord(e1, t->stream) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    if (st == SFFT_OK) st = hipEventSynchronize(e1) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    float v = 0.0f;
    if (st == SFFT_OK) st = hipEventElapsedTime(&v, e0, e1) == hipSuccess ? SFFT_OK : SFFT_EHIP;
    if (st != SFFT_OK) break;
    ms[r] = v / (float)REPS;
    if (tunable && (r == ROUTE_FFT || ms[r] < ms[best])) best = r;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  t->D.route = st == SFFT_OK ? best : r0;
  if (st == SFFT_OK && p->is_batch)
    for (sfft_plan_s* m : p->members)
      if (std::memcmp(&m->desc, &t->desc, sizeof(sfft_desc)) == 0) m->D.route = best;
  if (ms_out)
    for (int r = 0; r < 3; ++r) ms_out[r] = ms[r];
  if (route_out) *route_out = t->D.route + 1;   // the descriptor's flag value of the route
  return st;
}

int sfft_batch_capture(sfft_handle b, const void* const* sci, const void* const* tmpl, const uint8_t* const* mask,
                       const int64_t* ld, double* const* coeffs, void* const* diff, int32_t* info) {
  RoctxScope range_("sfft_batch_capture");
  if (b == nullptr || !b->is_batch || b->stream == nullptr) return SFFT_EINVAL;
  if (b->gexec != nullptr) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph != nullptr) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  // event timing would put event records into the graph: off while capturing
  std::vector<bool> timing;
  timing.push_back(b->timer.on);
  b->timer.on = false;
  for (sfft_plan_s* m : b->members) {
    timing.push_back(m->timer.on);
    m->timer.on = false;
  }
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const int st = sfft_batch_run(b, sci, tmpl, mask, ld, coeffs, diff, info);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  b->timer.on = timing[0];
  for (size_t i = 0; i < b->members.size(); ++i) b->members[i]->timer.on = timing[i + 1];
  if (st != SFFT_OK || e != hipSuccess || g == nullptr) {
    if (g != nullptr) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return st != SFFT_OK ? st : SFFT_EHIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return SFFT_EHIP;
  }
  b->graph = g;
  b->gexec = x;
  return SFFT_OK;
}

int sfft_batch_launch(sfft_handle b) {
  RoctxScope range_("sfft_batch_launch");
  if (b == nullptr || !b->is_batch) return SFFT_EINVAL;
  if (b->gexec == nullptr) return SFFT_ESTATE;
  HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
  return SFFT_OK;
}

// ---------------------------------------------------------------------------
// The no-allocation entry point
// ---------------------------------------------------------------------------
}  // extern "C"

// Device memory of sfft_subtract_pair_noalloc: one copy per GPU, set aside when
// the library's code object is loaded on that GPU and held until the process
// ends.  In host code this name is only a stand-in for the symbol: the address
// of a GPU's copy comes from hipGetSymbolAddress at set-up and is the only one
// ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[SFFT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 16;
// the twiddle tables sit at the end of the scratch (uploaded once per GPU);
// a plan's workspace takes the bytes before them
constexpr size_t SCR_TW32 = SFFT_NOALLOC_SCRATCH_BYTES - (size_t)TW_N * sizeof(cplx<float>);
constexpr size_t SCR_TW64 = SCR_TW32 - (size_t)TW_N * sizeof(cplx<double>);
static_assert(SCR_TW64 % 256 == 0, "256-byte aligned carve-up");

struct NoAllocDevice {
  std::mutex mu;
  bool ready = false;               // set-up done on this GPU
  unsigned char* ptr = nullptr;     // this GPU's address of `scratch`
  bool have_desc = false;           // the scratch holds the tables of `desc`
  sfft_desc desc;
  sfft_plan_s plan;                 // host state of the single-pair plan (tables held inline)
};
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];
std::mutex g_tw_mu;
bool g_tw_ready = false;
cplx<double> g_tw64[TW_N];
cplx<float> g_tw32[TW_N];

template <typename T>
int noalloc_run(sfft_plan_s* p, const void* sci, const void* tmpl, const uint8_t* mask, int64_t ld, double* coeffs,
                void* diff, int32_t* info) {
  const PairSet PS = pair_set_one(p, sci, tmpl, mask, coeffs, diff, info);
  int st = build_impl<T>(p, PS, 1, ld);
  if (st != SFFT_OK) return st;
  const Derived& D = p->D;
  hipStream_t s = p->stream;
  st = solve_jobs(s, plan_table(p), D.n, D.nblk, D.refine, &p->timer);
  if (st != SFFT_OK) return st;
  copy_out_group_kernel<<<dim3((D.n + 255) / 256, 1, 1), 256, 0, s>>>(PS, ws_offsets(D, p->Lo), D.n);
  LAUNCH_CHECK();
  return subtract_impl<T>(p, PS, 1, ld);
}

}  // namespace

extern "C" {

int sfft_subtract_pair_noalloc(const sfft_desc* d, void* hip_stream, const void* sci, const void* tmpl,
                               const uint8_t* mask, int64_t ld, double* coeffs, void* diff, int32_t* info) {
  if (d == nullptr || sci == nullptr || tmpl == nullptr || coeffs == nullptr || diff == nullptr) return SFFT_EINVAL;
  int st = validate(d);
  if (st != SFFT_OK) return st;
  if (ld < d->nx) return SFFT_EINVAL;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SFFT_EINVAL;
  NoAllocDevice& g = g_noalloc[dev];
  std::lock_guard<std::mutex> lock(g.mu);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  sfft_plan_s* p = &g.plan;
  if (!g.ready) {
    // set-up, once per GPU with that GPU current: its address of the array,
    // and the FP64/FP32 twiddle tables at the end of it
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr) return SFFT_EHIP;
    {
      std::lock_guard<std::mutex> tl(g_tw_mu);
      if (!g_tw_ready) {
        twiddle_tables(g_tw64, g_tw32);
        g_tw_ready = true;
      }
    }
    unsigned char* base = static_cast<unsigned char*>(ptr);
    HIP_TRY(hipMemcpyAsync(base + SCR_TW64, g_tw64, sizeof(g_tw64), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(base + SCR_TW32, g_tw32, sizeof(g_tw32), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    g.ptr = base;
    p->timer.silent = true;
    g.ready = true;
  }
  if (!g.have_desc || std::memcmp(&g.desc, d, sizeof(sfft_desc)) != 0) {
    // a new descriptor: derive the plan into the static host state, check the
    // size, upload its tables (the previous call's kernels on this stream
    // read the old ones first)
    g.have_desc = false;
    st = derive(d, &p->D);
    if (st != SFFT_OK) return st;
    p->Lo = layout_of(p->D);
    if (p->Lo.total > SCR_TW64) return SFFT_ETOOBIG;
    p->Lo.tw64 = SCR_TW64;
    p->Lo.tw32 = SCR_TW32;
    p->desc = *d;
    p->ws = g.ptr;
    p->owns_ws = false;
    p->stream = s;
    const Derived& D = p->D;
    HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.items), D.items.data(), (size_t)D.items.size() * sizeof(CorrItem),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.wrows), D.wrows.data(), (size_t)D.wrows.size() * sizeof(WinRow),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.drows), D.drows.data(), (size_t)D.drows.size() * sizeof(DirectRow),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->at<void>(p->Lo.mtiles), D.mtiles.data(), (size_t)D.mtiles.size() * sizeof(MfmaTile),
                           hipMemcpyHostToDevice, s));
    std::vector<SolveJob> jobs;
    RatioJob rj;
    st = upload_solve_tables(p, s, &jobs, &rj);
    if (st != SFFT_OK) return st;
    // the host tables (and `jobs`, `rj`) may change once the copies have been made
    HIP_TRY(hipStreamSynchronize(s));
    g.desc = *d;
    g.have_desc = true;
  }
  p->stream = s;
  p->built = true;
  return p->D.mode == SFFT_MODE_F64 ? noalloc_run<double>(p, sci, tmpl, mask, ld, coeffs, diff, info)
                                    : noalloc_run<float>(p, sci, tmpl, mask, ld, coeffs, diff, info);
}

const char* sfft_strerror(int status) {
  switch (status) {
    case SFFT_OK: return "success";
    case SFFT_EINVAL: return "invalid argument or descriptor";
    case SFFT_ENOMEM: return "out of device memory or workspace too small";
    case SFFT_EHIP: return "HIP runtime error";
    case SFFT_ENOTSPD: return "normal matrix is not positive definite";
    case SFFT_ESTATE: return "call out of order (build the system first)";
    case SFFT_ENONFINITE: return "non-finite value in the science or template image";
    case SFFT_ETOOBIG:
      return "the pair needs more device memory than the no-allocation entry point's static scratch holds";
    default: return "unknown status";
  }
}

}  // extern "C"
