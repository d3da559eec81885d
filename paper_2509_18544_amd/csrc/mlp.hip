// Warm-start network of the SFFT library: FP32 training and BF16 inference of
// a fully connected ReLU network on the gfx950 matrix cores (see
// include/sfft_mlp.h).
//
// Every product is one tiled GEMM kernel, C = op(A) op(B) with a fused
// epilogue (bias, ReLU, ReLU-derivative mask, FP64 de-standardisation).
// Tiles of 64 x 64 outputs per 256-thread block (four waves, one 32 x 32
// MFMA accumulator each), K staged through LDS in steps of 32 with both
// operands stored K-contiguous, which is the order the MFMA operands take.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/sfft.h"
#include "../../include/sfft_mlp.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int MAX_LAYERS = 8;
constexpr int MAX_DIM = 8192;
constexpr int TM = 64, TN = 64, TK = 32;
constexpr int GEMM_THREADS = 256;

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_RELU_MASK = 3, EPI_BIAS_AFFINE_F64 = 4 };

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN).
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <bool BF16>
struct Lds;
template <>
struct Lds<false> {
  using T = float;
  static constexpr int LD = TK + 1;   // odd stride: conflict-free column reads
};
template <>
struct Lds<true> {
  using T = uint16_t;
  static constexpr int LD = TK + 8;   // 80-byte rows keep 16-byte alignment for 8-wide operand reads
};

template <bool BF16>
__device__ inline typename Lds<BF16>::T cvt(float v) {
  if constexpr (BF16) return to_bf16(v);
  else return v;
}
template <bool BF16>
__device__ inline typename Lds<BF16>::T cvt(uint16_t v) {
  static_assert(BF16, "BF16 weights feed the BF16 kernel only");
  return v;
}

struct GemmArgs {
  const float* A;
  const void* B;
  void* C;
  const float* bias;
  const float* aux;
  const double* scale;
  const double* shift;
  int lda, ldb, ldc, ldaux;
  int M, N, K;
};

// C[m][n] = sum_k A(m,k) B(k,n), A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Tb is float, or uint16_t holding
// BF16 bits (BF16 kernel only).
template <typename Tb, bool BF16, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_kernel(GemmArgs g) {
  using T = typename Lds<BF16>::T;
  constexpr int LD = Lds<BF16>::LD;
  __shared__ __attribute__((aligned(16))) T As[TM * LD];
  __shared__ __attribute__((aligned(16))) T Bs[TN * LD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const Tb* Bg = static_cast<const Tb*>(g.B);

  constexpr int PER = TM * TK / GEMM_THREADS;   // 8 elements of each tile per thread
  f32x16 acc;
  for (int j = 0; j < 16; ++j) acc[j] = 0.0f;

  for (int k0 = 0; k0 < g.K; k0 += TK) {
    T ra[PER], rb[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * GEMM_THREADS;
      int m, k;
      if (TA) { k = idx / TM; m = idx % TM; }
      else { m = idx / TK; k = idx % TK; }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.0f;
      if (gm < g.M && gk < g.K) v = TA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk];
      ra[e] = cvt<BF16>(v);
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * GEMM_THREADS;
      int n, k;
      if (TB) { n = idx / TK; k = idx % TK; }
      else { k = idx / TN; n = idx % TN; }
      const int gn = n0 + n, gk = k0 + k;
      Tb v = Tb(0);
      if (gn < g.N && gk < g.K) v = TB ? Bg[(size_t)gn * g.ldb + gk] : Bg[(size_t)gk * g.ldb + gn];
      rb[e] = cvt<BF16>(v);
    }
    __syncthreads();   // the previous step's operand reads are done
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * GEMM_THREADS;
      int m, k;
      if (TA) { k = idx / TM; m = idx % TM; }
      else { m = idx / TK; k = idx % TK; }
      As[m * LD + k] = ra[e];
      int n, kb;
      if (TB) { n = idx / TK; kb = idx % TK; }
      else { kb = idx / TN; n = idx % TN; }
      Bs[n * LD + kb] = rb[e];
    }
    __syncthreads();
    const int ra_row = (wm * 32 + (lane & 31)) * LD;
    const int rb_row = (wn * 32 + (lane & 31)) * LD;
    if constexpr (BF16) {
      // 32x32x16: lane supplies 8 consecutive k at k = 8*(lane/32)
#pragma unroll
      for (int ks = 0; ks < TK; ks += 16) {
        const int kc = ks + 8 * (lane >> 5);
        const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&As[ra_row + kc]));
        const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&Bs[rb_row + kc]));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      // 32x32x2: lane supplies k = lane/32
#pragma unroll
      for (int ks = 0; ks < TK; ks += 2) {
        const int kc = ks + (lane >> 5);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[ra_row + kc], Bs[rb_row + kc], acc, 0, 0, 0);
      }
    }
  }

  // accumulator j of lane l holds C[8*(j/4) + 4*(l/32) + j%4][l%32] of the wave's 32x32 tile
  const int n = n0 + wn * 32 + (lane & 31);
  if (n >= g.N) return;
  float bn = 0.0f;
  if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU || EPI == EPI_BIAS_AFFINE_F64) bn = g.bias[n];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int m = m0 + wm * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    if (m >= g.M) continue;
    float v = acc[j];
    if (EPI == EPI_BIAS) v += bn;
    if (EPI == EPI_BIAS_RELU) v = fmaxf(v + bn, 0.0f);
    if (EPI == EPI_RELU_MASK) v = g.aux[(size_t)m * g.ldaux + n] > 0.0f ? v : 0.0f;
    if (EPI == EPI_BIAS_AFFINE_F64) {
      const double s = g.scale ? g.scale[n] : 1.0;
      const double t = g.shift ? g.shift[n] : 0.0;
      static_cast<double*>(g.C)[(size_t)m * g.ldc + n] = (double)(v + bn) * s + t;
    } else {
      static_cast<float*>(g.C)[(size_t)m * g.ldc + n] = v;
    }
  }
}

// out[n] = sum_m g[m*ld + n] (FP64 sum in fixed order), one thread per column.
__global__ void colsum_kernel(const float* g, int ld, int M, int N, float* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += g[(size_t)m * ld + n];
  out[n] = (float)s;
}

constexpr int MSE_THREADS = 1024;

__global__ __launch_bounds__(MSE_THREADS) void mse_kernel(const float* y, const float* t, int64_t count, float* dy,
                                                          double* loss) {
  __shared__ double part[MSE_THREADS];
  const float sc = (float)(2.0 / (double)count);
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += MSE_THREADS) {
    const float d = y[i] - t[i];
    dy[i] = sc * d;
    s += (double)d * (double)d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = MSE_THREADS / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (double)count;
}

__global__ void adam_kernel(float* p, const float* g, float* m1, float* m2, int64_t count, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a * c1) / (sqrtf(b * c2) + eps);
}

__global__ void to_bf16_kernel(const float* src, uint16_t* dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = to_bf16(src[i]);
}

__global__ void copy_f32_kernel(const float* src, float* dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

template <typename Tb, bool BF16, bool TA, bool TB, int EPI>
int launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return SFFT_OK;
  dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM);
  gemm_kernel<Tb, BF16, TA, TB, EPI><<<grid, GEMM_THREADS, 0, s>>>(g);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EHIP;
}

GemmArgs gemm_args(const float* A, int lda, const void* B, int ldb, void* C, int ldc, int M, int N, int K) {
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

}  // namespace

struct sfft_mlp_s {
  int nl = 0;
  int dims[MAX_LAYERS + 1] = {};
  int64_t woff[MAX_LAYERS + 1] = {};   // offset of W_l in the flat parameter vector (1-based l)
  int64_t boff[MAX_LAYERS + 1] = {};
  int64_t nparams = 0;
  int max_batch = 0;
  int maxdim = 0;
  hipStream_t stream = nullptr;
  float* acts = nullptr;           // h_1 .. h_{nl-1}, each [max_batch][dims[l]]
  int64_t aoff[MAX_LAYERS + 1] = {};
  float* g0 = nullptr;             // gradient ping-pong, [max_batch][maxdim]
  float* g1 = nullptr;
  uint16_t* wbf = nullptr;         // BF16 copy of the parameter vector
  float* pf = nullptr;             // FP32 copy (biases of the inference path)
  int fwd_batch = -1;              // batch of the last training forward, -1 = none
  bool have_bf16 = false;
  void* mem = nullptr;

  float* act(int l) const { return acts + aoff[l]; }
};

namespace {

int check_batch(const sfft_mlp_s* m, int32_t batch) {
  return (batch >= 1 && batch <= m->max_batch) ? SFFT_OK : SFFT_EINVAL;
}

int blocks_of(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

extern "C" {

int sfft_mlp_create(const int32_t* dims, int32_t nlayers, int32_t max_batch, void* hip_stream, sfft_mlp* out) {
  if (out == nullptr) return SFFT_EINVAL;
  *out = nullptr;
  if (dims == nullptr || nlayers < 1 || nlayers > MAX_LAYERS || max_batch < 1 || max_batch > (1 << 20))
    return SFFT_EINVAL;
  for (int i = 0; i <= nlayers; ++i)
    if (dims[i] < 1 || dims[i] > MAX_DIM) return SFFT_EINVAL;
  sfft_mlp_s* m = new (std::nothrow) sfft_mlp_s();
  if (m == nullptr) return SFFT_ENOMEM;
  m->nl = nlayers;
  m->max_batch = max_batch;
  m->stream = reinterpret_cast<hipStream_t>(hip_stream);
  int64_t off = 0, aoff = 0;
  for (int i = 0; i <= nlayers; ++i) {
    m->dims[i] = dims[i];
    m->maxdim = dims[i] > m->maxdim ? dims[i] : m->maxdim;
  }
  for (int l = 1; l <= nlayers; ++l) {
    m->woff[l] = off;
    off += (int64_t)dims[l - 1] * dims[l];
    m->boff[l] = off;
    off += dims[l];
    m->aoff[l] = aoff;
    if (l < nlayers) aoff += (int64_t)max_batch * dims[l];
  }
  m->nparams = off;
  const size_t a_bytes = (size_t)(aoff > 0 ? aoff : 1) * sizeof(float);
  const size_t g_bytes = (size_t)max_batch * m->maxdim * sizeof(float);
  const size_t w_bytes = ((size_t)off * sizeof(uint16_t) + 255) & ~(size_t)255;
  const size_t p_bytes = (size_t)off * sizeof(float);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t total = up(a_bytes) + 2 * up(g_bytes) + w_bytes + up(p_bytes);
  if (hipMalloc(&m->mem, total) != hipSuccess) {
    (void)hipGetLastError();
    delete m;
    return SFFT_ENOMEM;
  }
  unsigned char* base = static_cast<unsigned char*>(m->mem);
  m->acts = reinterpret_cast<float*>(base);
  base += up(a_bytes);
  m->g0 = reinterpret_cast<float*>(base);
  base += up(g_bytes);
  m->g1 = reinterpret_cast<float*>(base);
  base += up(g_bytes);
  m->wbf = reinterpret_cast<uint16_t*>(base);
  base += w_bytes;
  m->pf = reinterpret_cast<float*>(base);
  *out = m;
  return SFFT_OK;
}

int sfft_mlp_param_count(sfft_mlp m, int64_t* count) {
  if (m == nullptr || count == nullptr) return SFFT_EINVAL;
  *count = m->nparams;
  return SFFT_OK;
}

int sfft_mlp_forward(sfft_mlp m, const float* params, const float* x, int32_t batch, float* y) {
  if (m == nullptr || params == nullptr || x == nullptr || y == nullptr) return SFFT_EINVAL;
  if (check_batch(m, batch) != SFFT_OK) return SFFT_EINVAL;
  m->fwd_batch = -1;
  for (int l = 1; l <= m->nl; ++l) {
    const bool last = l == m->nl;
    const float* A = l == 1 ? x : m->act(l - 1);
    GemmArgs g = gemm_args(A, m->dims[l - 1], params + m->woff[l], m->dims[l], last ? (void*)y : (void*)m->act(l),
                           m->dims[l], batch, m->dims[l], m->dims[l - 1]);
    g.bias = params + m->boff[l];
    const int st = last ? launch_gemm<float, false, false, false, EPI_BIAS>(g, m->stream)
                        : launch_gemm<float, false, false, false, EPI_BIAS_RELU>(g, m->stream);
    if (st != SFFT_OK) return st;
  }
  m->fwd_batch = batch;
  return SFFT_OK;
}

int sfft_mlp_backward(sfft_mlp m, const float* params, const float* x, const float* dy, int32_t batch, float* grad) {
  if (m == nullptr || params == nullptr || x == nullptr || dy == nullptr || grad == nullptr) return SFFT_EINVAL;
  if (check_batch(m, batch) != SFFT_OK) return SFFT_EINVAL;
  if (m->fwd_batch != batch) return SFFT_ESTATE;
  const float* g = dy;
  float* bufs[2] = {m->g0, m->g1};
  int which = 0;
  for (int l = m->nl; l >= 1; --l) {
    const int din = m->dims[l - 1], dout = m->dims[l];
    const float* H = l == 1 ? x : m->act(l - 1);
    // dW_l = H_{l-1}^T g: [din x dout], contraction over the batch
    GemmArgs gw = gemm_args(H, din, g, dout, grad + m->woff[l], dout, din, dout, batch);
    int st = launch_gemm<float, false, true, false, EPI_STORE>(gw, m->stream);
    if (st != SFFT_OK) return st;
    colsum_kernel<<<blocks_of(dout, 256), 256, 0, m->stream>>>(g, dout, batch, dout, grad + m->boff[l]);
    if (hipGetLastError() != hipSuccess) return SFFT_EHIP;
    if (l > 1) {
      // g_{l-1} = (g W_l^T) * [h_{l-1} > 0]
      float* gn = bufs[which];
      which ^= 1;
      GemmArgs gd = gemm_args(g, dout, params + m->woff[l], dout, gn, din, batch, din, dout);
      gd.aux = m->act(l - 1);
      gd.ldaux = din;
      st = launch_gemm<float, false, false, true, EPI_RELU_MASK>(gd, m->stream);
      if (st != SFFT_OK) return st;
      g = gn;
    }
  }
  return SFFT_OK;
}

int sfft_mlp_mse(sfft_mlp m, const float* y, const float* t, int32_t batch, float* dy, double* loss) {
  if (m == nullptr || y == nullptr || t == nullptr || dy == nullptr || loss == nullptr) return SFFT_EINVAL;
  if (check_batch(m, batch) != SFFT_OK) return SFFT_EINVAL;
  const int64_t count = (int64_t)batch * m->dims[m->nl];
  mse_kernel<<<1, MSE_THREADS, 0, m->stream>>>(y, t, count, dy, loss);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EHIP;
}

int sfft_mlp_adam_step(sfft_mlp m, float* params, const float* grad, float* m1, float* m2, int32_t step, float lr,
                       float b1, float b2, float eps) {
  if (m == nullptr || params == nullptr || grad == nullptr || m1 == nullptr || m2 == nullptr || step < 1)
    return SFFT_EINVAL;
  if (!(b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f && eps > 0.0f && lr >= 0.0f)) return SFFT_EINVAL;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)step)));
  adam_kernel<<<blocks_of(m->nparams, 256), 256, 0, m->stream>>>(params, grad, m1, m2, m->nparams, lr, b1, b2, eps,
                                                                  c1, c2);
  return hipGetLastError() == hipSuccess ? SFFT_OK : SFFT_EHIP;
}

int sfft_mlp_set_weights_bf16(sfft_mlp m, const float* params) {
  if (m == nullptr || params == nullptr) return SFFT_EINVAL;
  to_bf16_kernel<<<blocks_of(m->nparams, 256), 256, 0, m->stream>>>(params, m->wbf, m->nparams);
  if (hipGetLastError() != hipSuccess) return SFFT_EHIP;
  copy_f32_kernel<<<blocks_of(m->nparams, 256), 256, 0, m->stream>>>(params, m->pf, m->nparams);
  if (hipGetLastError() != hipSuccess) return SFFT_EHIP;
  m->have_bf16 = true;
  return SFFT_OK;
}

int sfft_mlp_infer(sfft_mlp m, const float* x, int32_t batch, const double* scale, const double* shift, double* theta,
                   int64_t ld_theta) {
  if (m == nullptr || x == nullptr || theta == nullptr) return SFFT_EINVAL;
  if (check_batch(m, batch) != SFFT_OK || ld_theta < m->dims[m->nl] || ld_theta > (int64_t)1 << 30) return SFFT_EINVAL;
  if ((scale == nullptr) != (shift == nullptr)) return SFFT_EINVAL;
  if (!m->have_bf16) return SFFT_ESTATE;
  // the training forward's activations are overwritten
  m->fwd_batch = -1;
  for (int l = 1; l <= m->nl; ++l) {
    const bool last = l == m->nl;
    const float* A = l == 1 ? x : m->act(l - 1);
    GemmArgs g = gemm_args(A, m->dims[l - 1], m->wbf + m->woff[l], m->dims[l],
                           last ? (void*)theta : (void*)m->act(l), last ? (int)ld_theta : m->dims[l], batch,
                           m->dims[l], m->dims[l - 1]);
    g.bias = m->pf + m->boff[l];
    g.scale = scale;
    g.shift = shift;
    const int st = last ? launch_gemm<uint16_t, true, false, false, EPI_BIAS_AFFINE_F64>(g, m->stream)
                        : launch_gemm<uint16_t, true, false, false, EPI_BIAS_RELU>(g, m->stream);
    if (st != SFFT_OK) return st;
  }
  return SFFT_OK;
}

void sfft_mlp_destroy(sfft_mlp m) {
  if (m == nullptr) return;
  if (m->mem) (void)hipFree(m->mem);
  delete m;
}

}  // extern "C"
