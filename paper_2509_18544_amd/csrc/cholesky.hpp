// FP64 solve of the normal equations: blocked right-looking Cholesky
// Omega = L L^T, triangular solves, iterative refinement, residual norm.
//
// The factor F is a row-major n x n copy of Omega; only its lower triangle is
// read or written meaningfully.  Block size NB = 64.  Step k of the
// factorisation is three launches:
//   potrf_diag : factor the diagonal block in LDS and store its inverse
//                (Linv[k], 64 x 64) for the panel solve and the substitutions;
//   trsm       : L_ik = A_ik L_kk^{-T} for every row block i below;
//   syrk       : A_ij -= L_ik L_jk^T for every lower tile (i >= j) of the rest.
// A non-positive (or non-finite) pivot sets *info = global column + 1 and all
// later kernels return immediately (LAPACK potrf convention).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace sfft {

constexpr int NB = 64;
typedef double f64x4 __attribute__((ext_vector_type(4)));

// One pair's solve: every kernel below takes a device table of jobs and
// finds its pair from the block index, so that one launch serves a batch.
struct SolveJob {
  double* F;            // n x n factor (row-major, lower triangle used)
  double* Linv;         // nblk blocks of NB x NB: inverses of the diagonal blocks
  const double* omega;  // assembled normal matrix (kept for the residual)
  const double* beta;
  double* theta;
  double* y;
  double* r;
  double* d;
  double* w;            // right-hand side being updated by the substitutions
  int* info;
  int n, nblk;
};

// acc = A B^T (64 x 64 tiles in LDS, K = NB) for this wave's 32 x 32 quarter
// (rows wm.., columns wn..), on the FP64 matrix cores as 2 x 2 MFMA 16x16x4
// tiles.  Operand layout of the 16x16x4 f64 MFMA: lane l gives A[row l%16][k
// l/16] and B^T[k l/16][col l%16]; result register r of lane l is
// D[l/16 + 4 r][l%16] (lr = l%16, lk = l/16 below; checked on the device).
__device__ __forceinline__ void tile_abt(const double (*A)[NB + 1], const double (*B)[NB + 1], int wm, int wn,
                                         int lr, int lk, f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int m0 = 0; m0 < NB; m0 += 4) {
    const int kk = m0 + lk;
    const double a0 = A[wm + lr][kk], a1 = A[wm + 16 + lr][kk];
    const double b0 = B[wn + lr][kk], b1 = B[wn + 16 + lr][kk];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// Cross-lane read of a double held by lane l (two 32-bit reads into scalar registers).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Factor a 64 x 64 diagonal block with a block of 256 threads (4 waves).
//  T: the block in LDS (lower triangle read; rows and columns >= nb are
//  replaced by the identity, whose factor and inverse are the identity, so
//  every loop runs over the full 64 with static bounds); cb0, cb1, dv: 64
//  doubles of LDS each; sflag: 2 ints of LDS.  On success L goes to F (rows
//  and columns < nb, lower triangle, global offset k0, row pitch n) and
//  L^{-1} to Linv (64 x 64 row-major, zero outside nb); returns 0.  A
//  non-positive or non-finite pivot at column j returns j + 1 and stores
//  nothing (the factorisation loop still runs to its end on meaningless
//  values, so that every wave takes every barrier).  Every thread of the
//  block must call it; the return value is the same on every thread.
//  Factorisation: wave q owns columns 16q..16q+15 of every row (lane = row).
//  At column j the owning wave reads the pivot from lane j across lanes,
//  scales its column and publishes it (and the outcome) in LDS; after one
//  barrier every wave applies the rank-1 update to its columns > j.  The
//  column buffer and the outcome alternate between two slots, so one barrier
//  per column suffices: a slot is rewritten two columns later, after every
//  wave has passed the barrier that follows its last read.
//  Inverse X = L^{-1} on wave 0 alone (the columns are independent, so no
//  barrier): lane c holds column c in registers; step j finishes X[j][c]
//  (times 1 / L[j][j], computed beforehand) and applies
//  X[i][c] -= L[i][j] X[j][c] to the rows i > j, L[i][j] read from the tile
//  as a broadcast.  Spreading it over the four waves took a barrier per row
//  and was slower.
__device__ __forceinline__ int potrf_block64(double (*T)[NB + 1], double* cb0, double* cb1, double* dv, int* sflag,
                                             int nb, double* __restrict__ F, int n, int k0,
                                             double* __restrict__ Linv) {
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  const int c0 = q * 16;
  double a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = c0 + m;
    a[m] = (lane < nb && c < nb) ? (c <= lane ? T[lane][c] : 0.0) : (lane == c ? 1.0 : 0.0);
  }
  int fail = 0;   // the first bad pivot (the same on every thread); the loop runs on regardless
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double* __restrict__ col = (j & 1) ? cb1 : cb0;
    if (q == (j >> 4)) {
      const double v = a[j & 15];
      const double d = readlane_f64(v, j);
      const bool bad = !(d > 0.0) || !isfinite(d);
      if (lane == 0) sflag[j & 1] = bad ? j + 1 : 0;
      const double sd = sqrt(d);
      const double l = lane > j ? v * (1.0 / sd) : (lane == j ? sd : 0.0);
      a[j & 15] = l;
      col[lane] = l;
    }
    __syncthreads();
    if (fail == 0) fail = sflag[j & 1];
    if (c0 + 15 > j) {
      const double lij = col[lane];
#pragma unroll
      for (int m = 0; m < 16; ++m)
        if (c0 + m > j) a[m] -= lij * col[c0 + m];
    }
  }
  if (fail != 0) return fail;
  // L into the tile (the upper part holds values that are never read)
#pragma unroll
  for (int m = 0; m < 16; ++m) T[lane][c0 + m] = a[m];
  __syncthreads();
  if (q == 0) dv[lane] = 1.0 / T[lane][lane];
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    if (r < nb && c <= r) F[(int64_t)(k0 + r) * n + k0 + c] = T[r][c];
  }
  __syncthreads();
  // the inverse on one wave: its columns are independent, so lane c forms
  // column c by right-looking substitution with no barrier (L read from the
  // tile as a broadcast); the other waves are done
  if (q != 0) return 0;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = (i == lane) ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    x[j] *= dv[j];
#pragma unroll
    for (int i = j + 1; i < NB; ++i) x[i] -= T[i][j] * x[j];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) Linv[i * NB + lane] = (i < nb && lane < nb) ? x[i] : 0.0;
  return 0;
}

// Diagonal block k of every job (one block of 256 per job): the first block
// of each factorisation; the later ones are factored inside syrk_kernel.
__global__ __launch_bounds__(256) void potrf_diag_kernel(const SolveJob* __restrict__ jobs, int k) {
  __shared__ double T[NB][NB + 1];
  __shared__ double cb[3][NB];
  __shared__ int sflag[2];
  const SolveJob J = jobs[blockIdx.x];
  if (k >= J.nblk || *J.info != 0) return;
  const int n = J.n;
  const int k0 = k * NB;
  const int nb = min(NB, n - k0);
  const int tid = threadIdx.x;
  {
    // every load of the thread is issued (clamped into the block) before any is stored
    constexpr int PER = NB * NB / 256;
    double v[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * 256, r = e >> 6, c = e & 63;
      v[t] = J.F[(int64_t)(k0 + min(r, nb - 1)) * n + k0 + min(c, nb - 1)];
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * 256, r = e >> 6, c = e & 63;
      T[r][c] = v[t];
    }
  }
  __syncthreads();
  const int f = potrf_block64(T, cb[0], cb[1], cb[2], sflag, nb, J.F, n, k0, J.Linv + (size_t)k * NB * NB);
  if (f != 0 && tid == 0) *J.info = k0 + f;
}

// Row block bi (after block k): L = A Linv^T, 64 x 64 x 64 in LDS.
__global__ __launch_bounds__(256) void trsm_kernel(const SolveJob* __restrict__ jobs, int k) {
  __shared__ double A[NB][NB + 1];
  __shared__ double B[NB][NB + 1];
  const SolveJob J = jobs[blockIdx.y];
  if (k >= J.nblk - 1 || *J.info != 0) return;
  double* __restrict__ F = J.F;
  const int n = J.n;
  const int k0 = k * NB;
  const double* __restrict__ Linv = J.Linv + (size_t)k * NB * NB;
  const int tid = threadIdx.x;
  const int nb = min(NB, n - k0);
  const int r0 = k0 + NB + blockIdx.x * NB;
  const int nr = min(NB, n - r0);
  if (nr <= 0) return;
  {
    // every load of the thread is issued (clamped into the block) before any is stored
    constexpr int PER = NB * NB / 256;
    double av[PER], bv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * 256;
      const int i = e / NB, j = e % NB;
      av[q] = F[(int64_t)(r0 + min(i, nr - 1)) * n + k0 + min(j, nb - 1)];
      bv[q] = Linv[e];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * 256;
      const int i = e / NB, j = e % NB;
      A[i][j] = (i < nr && j < nb) ? av[q] : 0.0;
      B[i][j] = bv[q];
    }
  }
  __syncthreads();
  // L = A Linv^T on the matrix cores (see tile_abt)
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
  tile_abt(A, B, wm, wn, lr, lk, acc);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wm + 16 * a + lk + 4 * r, j = wn + 16 * c + lr;
        if (i < nr && j < nb) F[(int64_t)(r0 + i) * n + k0 + j] = acc[a][c][r];
      }
}

// Lower tiles (I >= J) of the trailing matrix after the npanel panels of
// block columns k .. k + npanel - 1 (rows from t0 = (k + npanel) NB):
// A_IJ -= sum over the panels of L_I L_J^T.  Two panels (a rank-128 update)
// read and write the trailing matrix once for two block steps.  With colonly,
// only the tiles (I, 0) of the first block column (one panel): the column a
// two-panel step needs updated and factored before its second panel solve.
// With fuse_diag, the first njobs blocks take tile (0, 0) of each job -- the
// next diagonal block -- and factor it as soon as it is updated (look-ahead:
// the next factorisation step runs while the rest of the update does); the
// other blocks take the remaining tiles, ntile - 1 per job.  Without it, one
// block per (job, tile).  Both through xcd_remap: an XCD takes a contiguous
// run of tiles, so tiles of one row I (sharing the panel L_I) and of
// neighbouring rows find the panels in its L2.
__global__ __launch_bounds__(256, 2) void syrk_kernel(const SolveJob* __restrict__ jobs, int k, int njobs, int ntile,
                                                   int fuse_diag, int npanel, int colonly) {
  __shared__ double A[NB][NB + 1];
  __shared__ double B[NB][NB + 1];
  __shared__ int sflag[2];
  int jb, b;
  if (fuse_diag) {
    if ((int)blockIdx.x < njobs) {
      jb = blockIdx.x;
      b = 0;
    } else {
      const int per = ntile - 1;
      const int id = xcd_remap(blockIdx.x - njobs, gridDim.x - njobs);
      if (per <= 0 || id >= njobs * per) return;
      jb = id / per;
      b = 1 + (id - jb * per);
    }
  } else {
    const int id = xcd_remap(blockIdx.x, gridDim.x);
    if (id >= njobs * ntile) return;
    jb = id / ntile;
    b = id - jb * ntile;
  }
  const SolveJob job = jobs[jb];
  if (k + npanel >= job.nblk || *job.info != 0) return;   // no trailing matrix for this job
  double* __restrict__ F = job.F;
  const int n = job.n;
  const int k0 = k * NB;
  const int T = job.nblk - k - npanel;   // trailing block rows
  if (colonly ? b >= T : b >= T * (T + 1) / 2) return;
  const int tid = threadIdx.x;
  const int t0 = k0 + npanel * NB;  // first trailing row
  // triangular tile enumeration: b = I (I+1)/2 + J (colonly: I = b, J = 0)
  int I = b, J = 0;
  if (!colonly) {
    I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    J = b - I * (I + 1) / 2;
  }
  const int ri = t0 + I * NB, rj = t0 + J * NB;
  const int ni = min(NB, n - ri), nj = min(NB, n - rj);
  if (ni <= 0 || nj <= 0) return;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
  for (int pa = 0; pa < npanel; ++pa) {
    const int c0 = k0 + pa * NB;   // the panel's columns (a full block: the trailing matrix lies beyond it)
    const int nb = min(NB, n - c0);
    if (pa > 0) __syncthreads();   // the previous panel's tiles have been read
    {
      // every load of the thread is issued (clamped into the panels) before any is stored
      constexpr int PER = NB * NB / 256;
      double av[PER], bv[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * 256;
        const int i = e / NB, m = min(e % NB, nb - 1);
        av[q] = F[(int64_t)(ri + min(i, ni - 1)) * n + c0 + m];
        bv[q] = F[(int64_t)(rj + min(i, nj - 1)) * n + c0 + m];
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * 256;
        const int i = e / NB, m = e % NB;
        A[i][m] = (i < ni && m < nb) ? av[q] : 0.0;
        B[i][m] = (i < nj && m < nb) ? bv[q] : 0.0;
      }
    }
    __syncthreads();
    if (pa == 0) {
      tile_abt(A, B, wm, wn, lr, lk, acc);
    } else {
      f64x4 acc2[2][2];
      tile_abt(A, B, wm, wn, lr, lk, acc2);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = acc[a][c] + acc2[a][c];
    }
  }
  // read-modify-write of the tile: the reads are unconditional (clamped) so
  // that they are all in flight together; only the stores are predicated
  double fv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = min(wm + 16 * a + lk + 4 * r, ni - 1), j = min(wn + 16 * c + lr, nj - 1);
        fv[a][c][r] = F[(int64_t)(ri + i) * n + rj + j];
      }
  if (!(fuse_diag && b == 0)) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wm + 16 * a + lk + 4 * r, j = wn + 16 * c + lr;
          if (i < ni && j < nj && (I != J || j <= i)) F[(int64_t)(ri + i) * n + rj + j] = fv[a][c][r] - acc[a][c][r];
        }
    return;
  }
  // the next diagonal block: updated tile into LDS, then factored here
  __syncthreads();   // every wave is done reading A and B
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) A[wm + 16 * a + lk + 4 * r][wn + 16 * c + lr] = fv[a][c][r] - acc[a][c][r];
  __syncthreads();
  const int f = potrf_block64(A, B[0], B[1], B[2], sflag, ni, F, n, ri, job.Linv + (size_t)(k + npanel) * NB * NB);
  if (f != 0 && tid == 0) *job.info = ri + f;
}

// Blocked right-looking substitutions, one launch per block step k; block
// (ib, job) of the launch owns one row block, the block of lanes l = 0..63 x
// quarters q = 0..3 (the waves) of a 64 x 64 tile.
//  Forward L y = b (which = 0: b = beta, 1: b = r), blocks i = k + ib:
//    every block forms y_k = Linv_k w_k (w_k = b_k at k = 0); block i = k
//    stores it, blocks i > k update w_i = (k == 0 ? b_i : w_i) - L_ik y_k.
//  Back L^T x = y (which = 0: x = theta, 1: x = d), blocks j = ib <= k:
//    every block forms x_k = Linv_k^T w_k (w_k = y_k at k = nblk - 1);
//    block j = k stores it, blocks j < k update
//    w_j = (k == nblk - 1 ? y_j : w_j) - L_kj^T x_k.
// Row blocks of a launch only read w_k, which no block of it writes.
// 64-element sums over the four quarters: partial of quarter q, lane l in part[q][l].
__device__ __forceinline__ double trsv_quarter_sum(double (*part)[NB + 1], int lane) {
  return (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

__global__ __launch_bounds__(256) void trsv_lower_step_kernel(const SolveJob* __restrict__ jobs, int k, int which) {
  __shared__ double part[4][NB + 1];
  __shared__ double yk[NB];
  const SolveJob J = jobs[blockIdx.y];
  if (k >= J.nblk || *J.info != 0) return;
  const int i = k + (int)blockIdx.x;
  if (i >= J.nblk) return;
  const int n = J.n;
  const int k0 = k * NB, nb = min(NB, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  const double* __restrict__ b = which == 0 ? J.beta : J.r;
  const double* __restrict__ wk = k == 0 ? b : J.w;
  // y_k = Linv_k w_k (Linv_k is zero past row / column nb)
  const double* __restrict__ Li = J.Linv + (size_t)k * NB * NB;
  {
    double lv[16], bv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int c = q * 16 + m;
      lv[m] = Li[lane * NB + c];
      bv[m] = wk[k0 + min(c, nb - 1)];
    }
    double a = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) a += lv[m] * bv[m];
    part[q][lane] = a;
  }
  __syncthreads();
  if (q == 0) yk[lane] = trsv_quarter_sum(part, lane);
  __syncthreads();
  if (i == k) {
    if (tid < nb) J.y[k0 + tid] = yk[tid];
    return;
  }
  // w_i -= L_ik y_k: row i0 + lane, columns of quarter q
  const int i0 = i * NB, ni = min(NB, n - i0);
  const double* __restrict__ row = J.F + (int64_t)(i0 + min(lane, ni - 1)) * n + k0;
  {
    double fv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) fv[m] = row[min(q * 16 + m, nb - 1)];
    double a = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) a += fv[m] * yk[q * 16 + m];
    __syncthreads();
    part[q][lane] = a;
  }
  __syncthreads();
  if (q == 0 && lane < ni) {
    const double* __restrict__ wi = k == 0 ? b : J.w;
    J.w[i0 + lane] = wi[i0 + lane] - trsv_quarter_sum(part, lane);
  }
}

__global__ __launch_bounds__(256) void trsv_upper_step_kernel(const SolveJob* __restrict__ jobs, int k, int which) {
  __shared__ double part[4][NB + 1];
  __shared__ double xk[NB];
  const SolveJob J = jobs[blockIdx.y];
  if (k >= J.nblk || *J.info != 0) return;
  const int j = (int)blockIdx.x;
  if (j > k) return;
  const int n = J.n;
  const int k0 = k * NB, nb = min(NB, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  const bool first = (k == J.nblk - 1);
  const double* __restrict__ wk = first ? J.y : J.w;
  // x_k = Linv_k^T w_k: x[c] = sum_m Linv_k[m][c] w_k[m], c = lane
  const double* __restrict__ Li = J.Linv + (size_t)k * NB * NB;
  {
    double lv[16], bv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int r = q * 16 + m;
      lv[m] = Li[r * NB + lane];
      bv[m] = wk[k0 + min(r, nb - 1)];
    }
    double a = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) a += lv[m] * bv[m];
    part[q][lane] = a;
  }
  __syncthreads();
  if (q == 0) xk[lane] = trsv_quarter_sum(part, lane);
  __syncthreads();
  double* __restrict__ x = which == 0 ? J.theta : J.d;
  if (j == k) {
    if (tid < nb) x[k0 + tid] = xk[tid];
    return;
  }
  // w_j -= L_kj^T x_k: column j0 + lane, rows k0 + (quarter q)
  const int j0 = j * NB;   // j < k, so the block is full
  {
    double fv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) fv[m] = J.F[(int64_t)(k0 + min(q * 16 + m, nb - 1)) * n + j0 + lane];
    double a = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) a += (q * 16 + m < nb) ? fv[m] * xk[q * 16 + m] : 0.0;
    __syncthreads();
    part[q][lane] = a;
  }
  __syncthreads();
  if (q == 0) {
    const double* __restrict__ wj = first ? J.y : J.w;
    J.w[j0 + lane] = wj[j0 + lane] - trsv_quarter_sum(part, lane);
  }
}

__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ A, int n,
                                                       const double* __restrict__ b, const double* __restrict__ x,
                                                       double* __restrict__ r) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= n) return;
  const double* a = A + (int64_t)row * n;
  double acc = 0.0;
#pragma unroll 8
  for (int c = lane; c < n; c += 64) acc += a[c] * x[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) r[row] = b[row] - acc;
}

// F <- Omega for every job (grid: chunks x jobs)
// F = Omega on and below the diagonal (no kernel reads F above it: the
// diagonal factor loads only its lower part, the panel and trailing loads are
// strictly below, and the upper part of a diagonal trailing tile is read but
// never stored).  One wave per row, 16-byte copies where the row is aligned.
__global__ __launch_bounds__(256) void copy_omega_kernel(const SolveJob* __restrict__ jobs) {
  const SolveJob J = jobs[blockIdx.y];
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= J.n) return;
  const int lane = threadIdx.x & 63;
  const double* __restrict__ src = J.omega + (int64_t)i * J.n;
  double* __restrict__ dst = J.F + (int64_t)i * J.n;
  if ((J.n & 1) == 0) {
    // pairs (c, c+1) with c even <= i; c + 1 <= n - 1 as n is even
#pragma unroll 4
    for (int c = 2 * lane; c <= i; c += 128)
      *reinterpret_cast<double2*>(dst + c) = *reinterpret_cast<const double2*>(src + c);
  } else {
#pragma unroll 4
    for (int c = lane; c <= i; c += 64) dst[c] = src[c];
  }
}

// r = beta - Omega theta for every job (one wave per row)
__global__ __launch_bounds__(256) void residual_jobs_kernel(const SolveJob* __restrict__ jobs) {
  const SolveJob J = jobs[blockIdx.y];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= J.n || *J.info != 0) return;
  const double* a = J.omega + (int64_t)row * J.n;
  double acc = 0.0;
  // unrolled so that a lane keeps several row loads in flight
#pragma unroll 8
  for (int c = lane; c < J.n; c += 64) acc += a[c] * J.theta[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) J.r[row] = J.beta[row] - acc;
}

// theta += d for every job whose factorisation succeeded
__global__ __launch_bounds__(256) void axpy_jobs_kernel(const SolveJob* __restrict__ jobs) {
  const SolveJob J = jobs[blockIdx.y];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < J.n && *J.info == 0) J.theta[i] += J.d[i];
}

// info reset for every job
__global__ void reset_info_kernel(const SolveJob* __restrict__ jobs, int njobs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < njobs) *jobs[i].info = 0;
}

// x += d (only if the factorisation succeeded)
__global__ void axpy_kernel(double* __restrict__ x, const double* __restrict__ d, int n,
                            const int* __restrict__ info) {
  if (*info != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

__global__ void copy_out_kernel(const double* __restrict__ src, double* __restrict__ dst, int n,
                                const int* __restrict__ info, int* __restrict__ info_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int inf = *info;
  if (i == 0 && info_out != nullptr) *info_out = inf;
  if (inf != 0) return;
  if (i < n) dst[i] = src[i];
}

// theta -> the caller's coefficients and the solve outcome -> info, for every
// pair of a group (pair blockIdx.z); coefficients untouched if info != 0
__global__ void copy_out_group_kernel(PairSet PS, WsOff O, int n) {
  const int pr = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int inf = reinterpret_cast<const int*>(PS.tws[pr] + O.flags)[0];   // the outcome of the factor used
  if (i == 0 && PS.info[pr] != nullptr) *PS.info[pr] = inf;
  if (inf != 0) return;
  if (i < n) PS.coeffs[pr][i] = ws_at<const double>(PS, pr, O.theta)[i];
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// rho = ||r|| / ||b|| (single block)
__global__ __launch_bounds__(256) void norm_ratio_kernel(const double* __restrict__ r,
                                                         const double* __restrict__ b, int n,
                                                         double* __restrict__ rho) {
  __shared__ double s1[256], s2[256];
  const int tid = threadIdx.x;
  double a = 0.0, c = 0.0;
  for (int i = tid; i < n; i += 256) {
    a += r[i] * r[i];
    c += b[i] * b[i];
  }
  s1[tid] = a;
  s2[tid] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      s1[tid] += s1[tid + s];
      s2[tid] += s2[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) *rho = (s2[0] > 0.0) ? sqrt(s1[0] / s2[0]) : sqrt(s1[0]);
}

// Background for a fixed kernel: x[nkk..n) <- solution of
// Omega_BB c = beta_B - Omega_BK k with k = x[0..nkk) (one block of 256;
// nb = n - nkk <= 15).  The nb x nb system is factored by one thread
// (Cholesky, FP64); a non-positive pivot leaves NaN in the background.
constexpr int FITBG_MAX_NB = 15;
__global__ __launch_bounds__(256) void fit_background_kernel(const double* __restrict__ A, int n, int nkk,
                                                             const double* __restrict__ b, double* __restrict__ x) {
  __shared__ double rhs[FITBG_MAX_NB];
  __shared__ double M[FITBG_MAX_NB * FITBG_MAX_NB];
  const int nb = n - nkk;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  for (int r = wave; r < nb; r += 4) {
    const double* a = A + (int64_t)(nkk + r) * n;
    double acc = 0.0;
    for (int c = lane; c < nkk; c += 64) acc += a[c] * x[c];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) rhs[r] = b[nkk + r] - acc;
  }
  for (int i = threadIdx.x; i < nb * nb; i += 256) M[i] = A[(int64_t)(nkk + i / nb) * n + nkk + i % nb];
  __syncthreads();
  if (threadIdx.x != 0) return;
  bool ok = true;
  for (int j = 0; j < nb && ok; ++j) {
    double d = M[j * nb + j];
    for (int k = 0; k < j; ++k) d -= M[j * nb + k] * M[j * nb + k];
    if (!(d > 0.0)) {
      ok = false;
      break;
    }
    d = sqrt(d);
    M[j * nb + j] = d;
    for (int i = j + 1; i < nb; ++i) {
      double s = M[i * nb + j];
      for (int k = 0; k < j; ++k) s -= M[i * nb + k] * M[j * nb + k];
      M[i * nb + j] = s / d;
    }
  }
  if (!ok) {
    for (int i = 0; i < nb; ++i) x[nkk + i] = __builtin_nan("");
    return;
  }
  for (int i = 0; i < nb; ++i) {            // L y = rhs
    double s = rhs[i];
    for (int k = 0; k < i; ++k) s -= M[i * nb + k] * rhs[k];
    rhs[i] = s / M[i * nb + i];
  }
  for (int i = nb - 1; i >= 0; --i) {       // L^T c = y
    double s = rhs[i];
    for (int k = i + 1; k < nb; ++k) s -= M[k * nb + i] * rhs[k];
    rhs[i] = s / M[i * nb + i];
  }
  for (int i = 0; i < nb; ++i) x[nkk + i] = rhs[i];
}


// Constant photometric ratio.  The kernel's flux ratio at a point source at z
// is sum_a m_a(z) s_a with s_a = sum_u k_{a,u}; it is the same everywhere
// exactly when s_a = 0 for every non-constant monomial a >= 1.  With those
// nc = nK - 1 constraints C theta = 0 the least-squares minimum is
//   theta = theta0 - Z lambda,  Z = Omega^{-1} C^T,  (C Z) lambda = C theta0,
// theta0 = Omega^{-1} beta the free solution.  The columns of Z are solved
// by substitution jobs that share the factor (right-hand sides: the columns
// of C^T, the indicators of the kernel blocks a = 1..nc).
constexpr int RATIO_MAXC = 14;   // nK - 1 for DK <= 4
struct RatioJob {
  double* theta;   // theta0 in, the constrained solution out
  double* Z;       // nc columns of n (theta of the constraint jobs)
  double* E;       // nc columns of n: C^T (beta of the constraint jobs)
  const int* info;
  int n, L2, nc;
};

// E[c][i] = [i lies in kernel block c + 1]; grid (ceil(n / 256), jobs)
__global__ void ratio_rhs_kernel(const RatioJob* __restrict__ jobs) {
  const RatioJob J = jobs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= J.n) return;
  const int a = i / J.L2;   // >= nK (never c + 1) on the background coefficients
  for (int c = 0; c < J.nc; ++c) J.E[(int64_t)c * J.n + i] = (a == c + 1) ? 1.0 : 0.0;
}

// One block of 256 per job: M = C Z and C theta0 as block sums (a wave per
// entry), the nc x nc SPD system by Cholesky on one thread (FP64; a
// non-positive pivot leaves NaN in theta), then theta -= Z lambda.
__global__ __launch_bounds__(256) void ratio_project_kernel(const RatioJob* __restrict__ jobs) {
  __shared__ double M[RATIO_MAXC][RATIO_MAXC + 1];   // [C Z | C theta0]
  __shared__ double lam[RATIO_MAXC];
  __shared__ int ok;
  const RatioJob J = jobs[blockIdx.x];
  if (*J.info != 0) return;
  const int nc = J.nc, n = J.n, L2 = J.L2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < nc * (nc + 1); q += 4) {
    const int a = q / (nc + 1), b = q - a * (nc + 1);
    const double* __restrict__ v = (b < nc ? J.Z + (int64_t)b * n : J.theta) + (int64_t)(a + 1) * L2;
    double acc = 0.0;
    for (int u = lane; u < L2; u += 64) acc += v[u];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) M[a][b] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    for (int j = 0; j < nc && ok; ++j) {      // M = G G^T in the lower triangle
      double d = M[j][j];
      for (int k = 0; k < j; ++k) d -= M[j][k] * M[j][k];
      if (!(d > 0.0)) {
        ok = 0;
        break;
      }
      d = sqrt(d);
      M[j][j] = d;
      for (int i = j + 1; i < nc; ++i) {
        double t = M[i][j];
        for (int k = 0; k < j; ++k) t -= M[i][k] * M[j][k];
        M[i][j] = t / d;
      }
    }
    if (ok) {
      for (int i = 0; i < nc; ++i) {            // G y = C theta0
        double t = M[i][nc];
        for (int k = 0; k < i; ++k) t -= M[i][k] * lam[k];
        lam[i] = t / M[i][i];
      }
      for (int i = nc - 1; i >= 0; --i) {       // G^T lambda = y
        double t = lam[i];
        for (int k = i + 1; k < nc; ++k) t -= M[k][i] * lam[k];
        lam[i] = t / M[i][i];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    double t = J.theta[i];
    if (ok) {
      for (int c = 0; c < nc; ++c) t -= J.Z[(int64_t)c * n + i] * lam[c];
    } else {
      t = __builtin_nan("");
    }
    J.theta[i] = t;
  }
}

}  // namespace sfft
