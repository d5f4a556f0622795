// Warm-start network: GELU MLP with BF16 GEMM operands on the gfx950 matrix
// cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation, FP32 master weights and
// Adam.  Forward, backward and optimizer kernels are all here.
//
// GEMM: C[M x N] = A[M x K] B[K x N] with A and B read through (row, column)
// strides, so the forward product (A W'), the input gradient (dZ W) and the
// weight gradient (dZ' A) share one kernel.  A 256-thread workgroup computes a
// 64 x 64 tile; each wave a 32 x 32 sub-tile as 2 x 2 MFMA 16x16 blocks; K is
// staged through LDS in chunks of 64 with 16-byte loads along whichever index
// of an operand is contiguous (A as rows x k, B as columns x k, so both
// fragments are 8 consecutive bf16 per lane).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace nrto {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                          // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int GT_M = 64, GT_N = 64, GT_K = 64, GT_PAD = 8;

// Stage a GT_ROWS x GT_K tile of an operand X (X[r][k] = X[r * sr + k * sk],
// r < R, k < K) into LDS as tile[r][k] (k contiguous).  Vector loads of 8
// bf16 along k when k is the contiguous index, along r when r is; otherwise
// (or at a ragged edge) one element at a time.
template <int ROWS>
__device__ __forceinline__ void stage_tile(uint16_t (*tile)[GT_K + GT_PAD], const uint16_t* __restrict__ X, int64_t sr,
                                           int64_t sk, int r0, int k0, int R, int K, int tid) {
  const bool kvec = (sk == 1) && (sr % 8 == 0) && ((((uintptr_t)X) & 15) == 0);
  const bool rvec = !kvec && (sr == 1) && (sk % 8 == 0) && ((((uintptr_t)X) & 15) == 0);
  if (kvec) {
    for (int v = tid; v < ROWS * GT_K / 8; v += 256) {
      const int r = v / (GT_K / 8), c = (v - r * (GT_K / 8)) * 8;
      const int gr = r0 + r, gk = k0 + c;
      u16x8 val;
      if (gr < R && gk + 8 <= K) {
        val = *(const u16x8*)(X + (int64_t)gr * sr + gk);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) val[j] = (gr < R && gk + j < K) ? X[(int64_t)gr * sr + gk + j] : (uint16_t)0;
      }
      *(u16x8*)&tile[r][c] = val;
    }
  } else if (rvec) {
    for (int v = tid; v < ROWS * GT_K / 8; v += 256) {
      const int c = v / (ROWS / 8), r = (v - c * (ROWS / 8)) * 8;
      const int gr = r0 + r, gk = k0 + c;
      u16x8 val;
      if (gk < K && gr + 8 <= R) {
        val = *(const u16x8*)(X + gr + (int64_t)gk * sk);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) val[j] = (gk < K && gr + j < R) ? X[gr + j + (int64_t)gk * sk] : (uint16_t)0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) tile[r + j][c] = val[j];
    }
  } else {
    for (int idx = tid; idx < ROWS * GT_K; idx += 256) {
      const int r = idx / GT_K, c = idx - r * GT_K;
      const int gr = r0 + r, gk = k0 + c;
      tile[r][c] = (gr < R && gk < K) ? X[(int64_t)gr * sr + (int64_t)gk * sk] : (uint16_t)0;
    }
  }
}

// GEMM C = A B on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): a
// 256-work-item workgroup computes a 64 x 64 tile, each wave a 32 x 32
// sub-tile as 2 x 2 blocks of 16 x 16; K is staged through LDS 64 at a time.
// A lane feeds 8 consecutive k of one row of A and of one column of B (the same
// k for both operands, so the product does not depend on how the instruction
// assigns k to lanes); the 16 x 16 result block leaves lane l with rows
// 4 (l / 16) + r, r < 4, of column l % 16.
template <int EPI>
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(const uint16_t* __restrict__ A, int64_t sam, int64_t sak, const uint16_t* __restrict__ B,
                 int64_t sbk, int64_t sbn, int M, int N, int K, float* __restrict__ C, int64_t ldc,
                 const float* __restrict__ bias, uint16_t* __restrict__ Cb) {
  __shared__ __align__(16) uint16_t As[GT_M][GT_K + GT_PAD];
  __shared__ __align__(16) uint16_t Bs[GT_N][GT_K + GT_PAD];
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GT_K) {
    stage_tile<GT_M>(As, A, sam, sak, m0, k0, M, K, tid);
    stage_tile<GT_N>(Bs, B, sbn, sbk, n0, k0, N, K, tid);   // B staged as [n][k]
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GT_K; kk += 32) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)&As[wm * 32 + i * 16 + (lane & 15)][kk + 8 * (lane >> 4)]);
        b[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)&Bs[wn * 32 + i * 16 + (lane & 15)][kk + 8 * (lane >> 4)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          float v = acc[i][j][r];
          if (EPI != EPI_STORE) v += bias[gn];
          C[gm * ldc + gn] = v;
          if (EPI == EPI_BIAS_GELU) Cb[gm * ldc + gn] = f2bf(gelu_f(v));
        }
      }
}

__global__ void normalize_in_kernel(const float* X, const float* mean, const float* stdv, int B, int D, uint16_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * D) return;
  const int d = (int)(i % D);
  out[i] = f2bf((X[i] - mean[d]) / stdv[d]);
}

__global__ void denorm_out_kernel(const float* Yn, const float* mean, const float* stdv, int B, int D, float* Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * D) return;
  const int d = (int)(i % D);
  Y[i] = Yn[i] * stdv[d] + mean[d];
}

// dY = 2 (Y - (T - mean) / std) / (B D); loss += sum (Y - Tn)^2 / (B D); bf16 copy for the GEMMs.
__global__ void mse_grad_kernel(const float* Y, const float* T, const float* mean, const float* stdv, int B, int D,
                                float* dY, uint16_t* dYb, float* loss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float c = 0.f;
  if (i < (int64_t)B * D) {
    const int d = (int)(i % D);
    const float diff = Y[i] - (T[i] - mean[d]) / stdv[d];
    const float inv = 1.0f / ((float)B * (float)D);
    dY[i] = 2.0f * diff * inv;
    dYb[i] = f2bf(dY[i]);
    c = diff * diff * inv;
  }
  c = wave_sum(c);
  if (lane_id() == 0) atomicAdd(loss, c);
}

// dZ = dA * gelu'(Z) (fp32 and bf16 copies)
__global__ void gelu_back_kernel(const float* dA, const float* Z, int64_t n, float* dZ, uint16_t* dZb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = dA[i] * gelu_grad_f(Z[i]);
  dZ[i] = g;
  dZb[i] = f2bf(g);
}

// db[n] = sum_m dZ[m][n]
__global__ void colsum_kernel(const float* dZ, int B, int N, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < B; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* pb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void to_bf16_kernel(const float* x, int64_t n, uint16_t* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

}  // namespace nrto

using namespace nrto;

struct nrto_ws_s {
  hipStream_t stream = nullptr;
  std::vector<int> w;       // widths
  int L = 0, max_batch = 0;
  std::vector<float*> W, b, gW, gb, mW, vW, mb, vb;
  std::vector<uint16_t*> Wb;
  std::vector<float*> Z;    // pre-activations per layer (max_batch x w[l+1])
  std::vector<uint16_t*> Ab;  // bf16 activations per layer input (max_batch x w[l])
  float *dA = nullptr, *dZ = nullptr, *loss = nullptr, *Yout = nullptr;
  uint16_t* dZb = nullptr;
  float *xmean = nullptr, *xstd = nullptr, *ymean = nullptr, *ystd = nullptr;
  int t = 0;
  std::vector<void*> allocs;
  std::string err;
};

static nrto_status ws_err(nrto_ws ws, nrto_status s, const std::string& m) {
  if (ws) ws->err = m;
  return set_global_error(s, m);
}

template <typename T>
static bool ws_alloc(nrto_ws ws, T** p, int64_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
  (void)hipMemsetAsync(q, 0, (size_t)std::max<int64_t>(n, 1) * sizeof(T), ws->stream);
  ws->allocs.push_back(q);
  *p = (T*)q;
  return true;
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

static hipError_t gemm(nrto_ws ws, int epi, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                       int64_t sbn, int M, int N, int K, float* C, int64_t ldc, const float* bias, uint16_t* Cb) {
  dim3 grid((N + GT_N - 1) / GT_N, (M + GT_M - 1) / GT_M), block(256);
  if (epi == EPI_STORE)
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI_STORE>, grid, block, 0, ws->stream, A, sam, sak, B, sbk, sbn, M, N, K, C, ldc, bias, Cb);
  else if (epi == EPI_BIAS_GELU)
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI_BIAS_GELU>, grid, block, 0, ws->stream, A, sam, sak, B, sbk, sbn, M, N, K, C, ldc, bias, Cb);
  else
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI_BIAS>, grid, block, 0, ws->stream, A, sam, sak, B, sbk, sbn, M, N, K, C, ldc, bias, Cb);
  return hipGetLastError();
}

extern "C" nrto_status nrto_ws_create(const int32_t* widths, int32_t n_widths, int32_t max_batch, uint64_t seed,
                                      void* stream, nrto_ws* out) {
  if (!out || !widths || n_widths < 2 || max_batch < 1) return set_global_error(NRTO_ERR_ARG, "bad arguments");
  for (int i = 0; i < n_widths; ++i)
    if (widths[i] < 1 || widths[i] > 65536) return set_global_error(NRTO_ERR_ARG, "bad width");
  nrto_ws ws = new (std::nothrow) nrto_ws_s();
  if (!ws) return set_global_error(NRTO_ERR_ALLOC, "out of host memory");
  ws->stream = (hipStream_t)stream;
  ws->w.assign(widths, widths + n_widths);
  ws->L = n_widths - 1;
  ws->max_batch = max_batch;
  const int L = ws->L;
  ws->W.resize(L); ws->b.resize(L); ws->gW.resize(L); ws->gb.resize(L);
  ws->mW.resize(L); ws->vW.resize(L); ws->mb.resize(L); ws->vb.resize(L);
  ws->Wb.resize(L); ws->Z.resize(L); ws->Ab.resize(L + 1);
  int maxw = 0;
  for (int x : ws->w) maxw = std::max(maxw, x);
  bool ok = true;
  for (int l = 0; l < L && ok; ++l) {
    const int64_t nw = (int64_t)ws->w[l] * ws->w[l + 1], nb = ws->w[l + 1];
    ok = ws_alloc(ws, &ws->W[l], nw) && ws_alloc(ws, &ws->b[l], nb) && ws_alloc(ws, &ws->gW[l], nw) &&
         ws_alloc(ws, &ws->gb[l], nb) && ws_alloc(ws, &ws->mW[l], nw) && ws_alloc(ws, &ws->vW[l], nw) &&
         ws_alloc(ws, &ws->mb[l], nb) && ws_alloc(ws, &ws->vb[l], nb) && ws_alloc(ws, &ws->Wb[l], nw) &&
         ws_alloc(ws, &ws->Z[l], (int64_t)max_batch * ws->w[l + 1]);
  }
  for (int l = 0; l <= L && ok; ++l) ok = ws_alloc(ws, &ws->Ab[l], (int64_t)max_batch * ws->w[l]);
  ok = ok && ws_alloc(ws, &ws->dA, (int64_t)max_batch * maxw) && ws_alloc(ws, &ws->dZ, (int64_t)max_batch * maxw) &&
       ws_alloc(ws, &ws->dZb, (int64_t)max_batch * maxw) && ws_alloc(ws, &ws->loss, 1) &&
       ws_alloc(ws, &ws->Yout, (int64_t)max_batch * ws->w[L]) && ws_alloc(ws, &ws->xmean, ws->w[0]) &&
       ws_alloc(ws, &ws->xstd, ws->w[0]) && ws_alloc(ws, &ws->ymean, ws->w[L]) && ws_alloc(ws, &ws->ystd, ws->w[L]);
  if (!ok) {
    nrto_ws_destroy(ws);
    return set_global_error(NRTO_ERR_ALLOC, "hipMalloc failed");
  }
  // initial weights: uniform +-sqrt(6/(fan_in+fan_out)) from SplitMix64; biases 0; unit normalisation
  for (int l = 0; l < L; ++l) {
    const int fi = ws->w[l], fo = ws->w[l + 1];
    std::vector<float> h((size_t)fi * fo);
    const double a = std::sqrt(6.0 / (fi + fo));
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + (uint64_t)(l + 1) * 0xD1B54A32D192ED03ull;
    for (size_t i = 0; i < h.size(); ++i) {
      st += 0x9E3779B97F4A7C15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
      h[i] = (float)((2.0 * u - 1.0) * a);
    }
    (void)hipMemcpyAsync(ws->W[l], h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, ws->stream);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk((int64_t)h.size())), dim3(256), 0, ws->stream, ws->W[l], (int64_t)h.size(), ws->Wb[l]);
  }
  std::vector<float> ones(maxw, 1.0f);
  (void)hipMemcpyAsync(ws->xstd, ones.data(), sizeof(float) * ws->w[0], hipMemcpyHostToDevice, ws->stream);
  (void)hipMemcpyAsync(ws->ystd, ones.data(), sizeof(float) * ws->w[L], hipMemcpyHostToDevice, ws->stream);
  if (hipStreamSynchronize(ws->stream) != hipSuccess) {
    nrto_ws_destroy(ws);
    return set_global_error(NRTO_ERR_HIP, "initialisation failed");
  }
  *out = ws;
  return NRTO_OK;
}

extern "C" void nrto_ws_destroy(nrto_ws ws) {
  if (!ws) return;
  (void)hipStreamSynchronize(ws->stream);
  for (void* p : ws->allocs) (void)hipFree(p);
  delete ws;
}

extern "C" nrto_status nrto_ws_set_norm(nrto_ws ws, const float* xmean, const float* xstd, const float* ymean,
                                        const float* ystd) {
  if (!ws) return set_global_error(NRTO_ERR_ARG, "null handle");
  const int D0 = ws->w[0], DL = ws->w[ws->L];
  hipStream_t s = ws->stream;
  if (xmean) (void)hipMemcpyAsync(ws->xmean, xmean, sizeof(float) * D0, hipMemcpyHostToDevice, s);
  if (xstd) (void)hipMemcpyAsync(ws->xstd, xstd, sizeof(float) * D0, hipMemcpyHostToDevice, s);
  if (ymean) (void)hipMemcpyAsync(ws->ymean, ymean, sizeof(float) * DL, hipMemcpyHostToDevice, s);
  if (ystd) (void)hipMemcpyAsync(ws->ystd, ystd, sizeof(float) * DL, hipMemcpyHostToDevice, s);
  if (hipStreamSynchronize(s) != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, "copy failed");
  return NRTO_OK;
}

// Forward pass over batch rows of X (device, fp32, batch x w0); leaves the
// normalised output in Z[L-1].
static nrto_status ws_forward(nrto_ws ws, const float* X, int batch) {
  const int L = ws->L;
  hipStream_t s = ws->stream;
  hipLaunchKernelGGL(normalize_in_kernel, dim3(nblk((int64_t)batch * ws->w[0])), dim3(256), 0, s, X, ws->xmean,
                     ws->xstd, batch, ws->w[0], ws->Ab[0]);
  for (int l = 0; l < L; ++l) {
    const int fi = ws->w[l], fo = ws->w[l + 1];
    hipError_t e = gemm(ws, l < L - 1 ? EPI_BIAS_GELU : EPI_BIAS, ws->Ab[l], fi, 1, ws->Wb[l], 1, fi, batch, fo, fi,
                        ws->Z[l], fo, ws->b[l], ws->Ab[l + 1]);
    if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
  }
  return NRTO_OK;
}

extern "C" nrto_status nrto_ws_infer(nrto_ws ws, const float* X, int32_t batch, float* Y) {
  if (!ws || !X || !Y) return set_global_error(NRTO_ERR_ARG, "null argument");
  if (batch < 1 || batch > ws->max_batch) return ws_err(ws, NRTO_ERR_ARG, "batch out of range");
  nrto_status st = ws_forward(ws, X, batch);
  if (st != NRTO_OK) return st;
  const int DL = ws->w[ws->L];
  hipLaunchKernelGGL(denorm_out_kernel, dim3(nblk((int64_t)batch * DL)), dim3(256), 0, ws->stream, ws->Z[ws->L - 1],
                     ws->ymean, ws->ystd, batch, DL, Y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
  return NRTO_OK;
}

// Gradients of the loss into gW, gb; loss into ws->loss.
static nrto_status ws_backward(nrto_ws ws, const float* X, const float* Tgt, int batch) {
  nrto_status st = ws_forward(ws, X, batch);
  if (st != NRTO_OK) return st;
  const int L = ws->L;
  hipStream_t s = ws->stream;
  const int DL = ws->w[L];
  (void)hipMemsetAsync(ws->loss, 0, sizeof(float), s);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nblk((int64_t)batch * DL)), dim3(256), 0, s, ws->Z[L - 1], Tgt, ws->ymean,
                     ws->ystd, batch, DL, ws->dZ, ws->dZb, ws->loss);
  for (int l = L - 1; l >= 0; --l) {
    const int fi = ws->w[l], fo = ws->w[l + 1];
    // dW = dZ' A_l  (fo x fi), db = colsum dZ
    hipError_t e = gemm(ws, EPI_STORE, ws->dZb, 1, fo, ws->Ab[l], fi, 1, fo, fi, batch, ws->gW[l], fi, nullptr, nullptr);
    if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
    hipLaunchKernelGGL(colsum_kernel, dim3(nblk(fo)), dim3(256), 0, s, ws->dZ, batch, fo, ws->gb[l]);
    if (l > 0) {
      // dA = dZ W (batch x fi), then dZ_{l-1} = dA * gelu'(Z_{l-1})
      e = gemm(ws, EPI_STORE, ws->dZb, fo, 1, ws->Wb[l], fi, 1, batch, fi, fo, ws->dA, fi, nullptr, nullptr);
      if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
      hipLaunchKernelGGL(gelu_back_kernel, dim3(nblk((int64_t)batch * fi)), dim3(256), 0, s, ws->dA, ws->Z[l - 1],
                         (int64_t)batch * fi, ws->dZ, ws->dZb);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
  return NRTO_OK;
}

extern "C" nrto_status nrto_ws_train_step(nrto_ws ws, const float* X, const float* Tgt, int32_t batch, float lr,
                                          float* loss_host) {
  if (!ws || !X || !Tgt) return set_global_error(NRTO_ERR_ARG, "null argument");
  if (batch < 1 || batch > ws->max_batch) return ws_err(ws, NRTO_ERR_ARG, "batch out of range");
  nrto_status st = ws_backward(ws, X, Tgt, batch);
  if (st != NRTO_OK) return st;
  ws->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  // bias corrections 1 - beta^t in double: in float, 1 - 0.999^2 loses five digits to cancellation
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)ws->t));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)ws->t));
  for (int l = 0; l < ws->L; ++l) {
    const int64_t nw = (int64_t)ws->w[l] * ws->w[l + 1], nb = ws->w[l + 1];
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(nw)), dim3(256), 0, ws->stream, ws->W[l], ws->gW[l], ws->mW[l], ws->vW[l],
                       nw, lr, b1, b2, eps, c1, c2, ws->Wb[l]);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(nb)), dim3(256), 0, ws->stream, ws->b[l], ws->gb[l], ws->mb[l], ws->vb[l],
                       nb, lr, b1, b2, eps, c1, c2, (uint16_t*)nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
  if (loss_host) {
    e = hipMemcpyAsync(loss_host, ws->loss, sizeof(float), hipMemcpyDeviceToHost, ws->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ws->stream);
    if (e != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, hipGetErrorString(e));
  }
  return NRTO_OK;
}

extern "C" nrto_status nrto_ws_gradients(nrto_ws ws, const float* X, const float* Tgt, int32_t batch, float* grads,
                                         float* loss_host) {
  if (!ws || !X || !Tgt || !grads) return set_global_error(NRTO_ERR_ARG, "null argument");
  if (batch < 1 || batch > ws->max_batch) return ws_err(ws, NRTO_ERR_ARG, "batch out of range");
  nrto_status st = ws_backward(ws, X, Tgt, batch);
  if (st != NRTO_OK) return st;
  size_t off = 0;
  for (int l = 0; l < ws->L; ++l) {
    const size_t nw = (size_t)ws->w[l] * ws->w[l + 1], nb = ws->w[l + 1];
    (void)hipMemcpyAsync(grads + off, ws->gW[l], nw * sizeof(float), hipMemcpyDeviceToHost, ws->stream);
    off += nw;
    (void)hipMemcpyAsync(grads + off, ws->gb[l], nb * sizeof(float), hipMemcpyDeviceToHost, ws->stream);
    off += nb;
  }
  if (loss_host) (void)hipMemcpyAsync(loss_host, ws->loss, sizeof(float), hipMemcpyDeviceToHost, ws->stream);
  if (hipStreamSynchronize(ws->stream) != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, "copy failed");
  return NRTO_OK;
}

extern "C" nrto_status nrto_ws_params(nrto_ws ws, float* get, const float* set) {
  if (!ws) return set_global_error(NRTO_ERR_ARG, "null handle");
  size_t off = 0;
  for (int l = 0; l < ws->L; ++l) {
    const size_t nw = (size_t)ws->w[l] * ws->w[l + 1], nb = ws->w[l + 1];
    if (get) {
      (void)hipMemcpyAsync(get + off, ws->W[l], nw * sizeof(float), hipMemcpyDeviceToHost, ws->stream);
      (void)hipMemcpyAsync(get + off + nw, ws->b[l], nb * sizeof(float), hipMemcpyDeviceToHost, ws->stream);
    }
    if (set) {
      (void)hipMemcpyAsync(ws->W[l], set + off, nw * sizeof(float), hipMemcpyHostToDevice, ws->stream);
      (void)hipMemcpyAsync(ws->b[l], set + off + nw, nb * sizeof(float), hipMemcpyHostToDevice, ws->stream);
      hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk((int64_t)nw)), dim3(256), 0, ws->stream, ws->W[l], (int64_t)nw, ws->Wb[l]);
    }
    off += nw + nb;
  }
  if (hipStreamSynchronize(ws->stream) != hipSuccess) return ws_err(ws, NRTO_ERR_HIP, "copy failed");
  return NRTO_OK;
}

extern "C" nrto_status nrto_ws_gemm_bf16(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                                         int64_t sbn, int32_t M, int32_t N, int32_t K, float* C, void* stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return set_global_error(NRTO_ERR_ARG, "bad arguments");
  dim3 grid((N + GT_N - 1) / GT_N, (M + GT_M - 1) / GT_M), block(256);
  hipLaunchKernelGGL(gemm_bf16_kernel<EPI_STORE>, grid, block, 0, (hipStream_t)stream, A, sam, sak, B, sbk, sbn, M, N, K,
                     C, (int64_t)N, (const float*)nullptr, (uint16_t*)nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_global_error(NRTO_ERR_HIP, hipGetErrorString(e));
  return NRTO_OK;
}
