// Training and evaluation kernels of the learned step-size controller's
// network: x (16 features) -> tanh(W1 x + b1) (64) -> tanh(W2 h1 + b2) (64)
// -> w3 . h2 + b3.  Weights, inputs and first-layer activations are bf16,
// accumulation fp32; the dense products run on the matrix cores
// (v_mfma_f32_16x16x16_bf16).  One workgroup of 4 wavefronts takes a tile of
// 64 samples; wavefront w owns samples 16w .. 16w+15 in the forward pass and
// output rows 16w .. 16w+15 of the weight-gradient products.
//
// MFMA 16x16x16 operand layout (lane l, j = 0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + j     B[k][n]: n = l % 16, k = 4 (l / 16) + j
//   D[i][n]: n = l % 16, i = 4 (l / 16) + j
//
// Loss: weighted mean squared error sum_b w_b (y_b - t_b)^2 / sum_b w_b; the
// gradient is accumulated over workgroups with fp32 atomics.  Adam keeps fp32
// master weights and refreshes their bf16 copy.  Sample b of a minibatch is
// row idx[b] of the data set (row b without an index array), so a shuffled
// minibatch is gathered by the kernels as they load it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/hode.h"
#include "hode_dev.h"

namespace hode {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NI = MLP_IN, NHID = MLP_H;
constexpr int O_W1 = 0, O_B1 = O_W1 + NHID * NI, O_W2 = O_B1 + NHID, O_B2 = O_W2 + NHID * NHID,
              O_W3 = O_B2 + NHID, O_B3 = O_W3 + NHID;

__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ inline float bf(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ inline bf16x4 ld4(const uint16_t* p) {
  bf16x4 r;
  r[0] = (short)p[0];
  r[1] = (short)p[1];
  r[2] = (short)p[2];
  r[3] = (short)p[3];
  return r;
}

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 63 KB: within the 64 KB one workgroup may allocate.
struct Smem {
  uint16_t Xq[64][NI], XqT[NI][64];
  uint16_t W1[NHID][NI];
  uint16_t W2[NHID][NHID], W2T[NHID][NHID];
  uint16_t H1q[64][NHID], H1qT[NHID][64];
  uint16_t dH2[64][NHID], dH2T[NHID][64], dH1T[NHID][64];
  float b1[NHID], b2[NHID], w3[NHID], b3;
  float y[64], dy[64], wt[64], tg[64];
};

// Data-set row of minibatch sample b.
__device__ inline int64_t row_of(const int64_t* __restrict__ idx, int64_t b) { return idx ? idx[b] : b; }

// Forward pass of one 64-sample tile; leaves h2 of this wave's rows in
// `h2` (D layout, 4 column tiles) and y in s.y.  Rows >= B read zeros.
__device__ void forward_tile(Smem& s, const uint16_t* __restrict__ Wb, const float* __restrict__ X,
                             const int64_t* __restrict__ idx, int64_t b0, int64_t B, f32x4 (&h2)[4]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int e = t; e < 64 * NI; e += 256) {
    const int r = e / NI, k = e % NI;
    const float x = (b0 + r < B) ? X[row_of(idx, b0 + r) * NI + k] : 0.f;
    const uint16_t q = to_bf16(x);
    s.Xq[r][k] = q;
    s.XqT[k][r] = q;
  }
  for (int e = t; e < NHID * NI; e += 256) s.W1[e / NI][e % NI] = Wb[O_W1 + e];
  for (int e = t; e < NHID * NHID; e += 256) {
    const uint16_t q = Wb[O_W2 + e];
    s.W2[e / NHID][e % NHID] = q;
    s.W2T[e % NHID][e / NHID] = q;
  }
  if (t < NHID) {
    s.b1[t] = bf(Wb[O_B1 + t]);
    s.b2[t] = bf(Wb[O_B2 + t]);
    s.w3[t] = bf(Wb[O_W3 + t]);
  }
  if (t == 0) s.b3 = bf(Wb[O_B3]);
  __syncthreads();
  const int li = lane & 15, lk = 4 * (lane >> 4);
  // layer 1: A1 = Xq W1^T (K = 16)
  for (int ct = 0; ct < 4; ++ct) {
    f32x4 acc = {0, 0, 0, 0};
    acc = mfma(ld4(&s.Xq[16 * w + li][lk]), ld4(&s.W1[16 * ct + li][lk]), acc);
    const int n = 16 * ct + li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * w + lk + j;
      const float h = tanhf(acc[j] + s.b1[n]);
      const uint16_t q = to_bf16(h);
      s.H1q[r][n] = q;
      s.H1qT[n][r] = q;
    }
  }
  __syncthreads();
  // layer 2: A2 = H1q W2^T (K = 64), y = h2 . w3 + b3
  float part[4] = {0, 0, 0, 0};
  for (int ct = 0; ct < 4; ++ct) {
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc = mfma(ld4(&s.H1q[16 * w + li][16 * kt + lk]), ld4(&s.W2[16 * ct + li][16 * kt + lk]), acc);
    const int n = 16 * ct + li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float h = tanhf(acc[j] + s.b2[n]);
      h2[ct][j] = h;
      part[j] += h * s.w3[n];
    }
  }
  // sum over the 16 lanes of a row group (the columns of each tile)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = part[j];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    if (li == 0) s.y[16 * w + lk + j] = v + s.b3;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void mlp_forward_k(const uint16_t* __restrict__ Wb, const float* __restrict__ X,
                                                     float* __restrict__ Y, int64_t B) {
  __shared__ Smem s;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  f32x4 h2[4];
  forward_tile(s, Wb, X, nullptr, b0, B, h2);
  const int t = threadIdx.x;
  if (t < 64 && b0 + t < B) Y[b0 + t] = s.y[t];
}

__global__ __launch_bounds__(256) void mlp_wsum_k(const float* __restrict__ Wt, const int64_t* __restrict__ idx,
                                                  int64_t B, double* __restrict__ acc) {
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < B; i += (int64_t)gridDim.x * 256)
    v += Wt[row_of(idx, i)];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, v);
}

// acc[0] = sum of weights (input), acc[1] += loss
__global__ __launch_bounds__(256) void mlp_grad_k(const uint16_t* __restrict__ Wb, const float* __restrict__ X,
                                                  const float* __restrict__ T, const float* __restrict__ Wt,
                                                  const int64_t* __restrict__ idx, int64_t B,
                                                  float* __restrict__ grad, double* __restrict__ acc) {
  __shared__ Smem s;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = 4 * (lane >> 4);
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  f32x4 h2[4];
  forward_tile(s, Wb, X, idx, b0, B, h2);
  const double inv_sw = 1.0 / acc[0];
  if (t < 64) {
    const bool in = b0 + t < B;
    const int64_t row = in ? row_of(idx, b0 + t) : 0;
    const float wt = in ? Wt[row] : 0.f, tg = in ? T[row] : 0.f;
    const float d = s.y[t] - tg;
    s.dy[t] = (float)(2.0 * wt * d * inv_sw);
    double l = (double)wt * d * d * inv_sw;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (t == 0) atomicAdd(&acc[1], l);
  }
  __syncthreads();
  // dH2 = dy w3 (1 - h2^2); dw3 = sum_b dy h2; db2 = sum_b dH2; db3 = sum dy
  for (int ct = 0; ct < 4; ++ct) {
    const int n = 16 * ct + li;
    float sw3 = 0, sb2 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * w + lk + j;
      const float h = h2[ct][j];
      const float g = s.dy[r] * s.w3[n] * (1.f - h * h);
      sw3 += s.dy[r] * h;
      sb2 += g;
      const uint16_t q = to_bf16(g);
      s.dH2[r][n] = q;
      s.dH2T[n][r] = q;
    }
    // reduce over the 4 row groups of the wave (lanes n, n+16, n+32, n+48)
    sw3 += __shfl_xor(sw3, 16, 64);
    sw3 += __shfl_xor(sw3, 32, 64);
    sb2 += __shfl_xor(sb2, 16, 64);
    sb2 += __shfl_xor(sb2, 32, 64);
    if (lane < 16) {
      atomicAdd(&grad[O_W3 + n], sw3);
      atomicAdd(&grad[O_B2 + n], sb2);
    }
  }
  if (t < 64) {
    float v = s.dy[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (t == 0) atomicAdd(&grad[O_B3], v);
  }
  __syncthreads();
  // dW2[j][i] = sum_b dH2[b][j] H1q[b][i]: rows j of tile w, K = batch
  for (int it = 0; it < 4; ++it) {
    f32x4 acc4 = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc4 = mfma(ld4(&s.dH2T[16 * w + li][16 * kt + lk]), ld4(&s.H1qT[16 * it + li][16 * kt + lk]), acc4);
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&grad[O_W2 + (16 * w + lk + j) * NHID + 16 * it + li], acc4[j]);
  }
  // dH1[b][i] = (sum_j dH2[b][j] W2[j][i]) (1 - h1^2): rows b of tile w, K = j
  for (int it = 0; it < 4; ++it) {
    f32x4 acc4 = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc4 = mfma(ld4(&s.dH2[16 * w + li][16 * kt + lk]), ld4(&s.W2T[16 * it + li][16 * kt + lk]), acc4);
    const int n = 16 * it + li;
    float sb1 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 16 * w + lk + j;
      const float h = bf(s.H1q[r][n]);  // the layer's bf16 activation
      const float g = acc4[j] * (1.f - h * h);
      sb1 += g;
      s.dH1T[n][r] = to_bf16(g);
    }
    sb1 += __shfl_xor(sb1, 16, 64);
    sb1 += __shfl_xor(sb1, 32, 64);
    if (lane < 16) atomicAdd(&grad[O_B1 + n], sb1);
  }
  __syncthreads();
  // dW1[i][k] = sum_b dH1[b][i] Xq[b][k]: rows i of tile w, K = batch
  {
    f32x4 acc4 = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc4 = mfma(ld4(&s.dH1T[16 * w + li][16 * kt + lk]), ld4(&s.XqT[li][16 * kt + lk]), acc4);
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&grad[O_W1 + (16 * w + lk + j) * NI + li], acc4[j]);
  }
}

__global__ __launch_bounds__(256) void fill_k(float* __restrict__ p, int64_t n, double* __restrict__ d, int nd) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
  if (i < nd) d[i] = 0.0;
}

__global__ __launch_bounds__(256) void adam_k(float* __restrict__ Wm, uint16_t* __restrict__ Wb,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = Wm[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  Wm[i] = w;
  Wb[i] = to_bf16(w);
}

__global__ __launch_bounds__(256) void quantize_k(const float* __restrict__ Wm, uint16_t* __restrict__ Wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < MLP_NPARAM) Wb[i] = to_bf16(Wm[i]);
}

// Scratch of the allocation-free training step: the two loss sums (offset
// 0) and the gradient of the 5313 parameters (offset 256), one copy per GPU,
// held until the process ends.  Host code never passes this array's name to
// a kernel: it stands for the device copy only in device code, so the host
// resolves each GPU's address once (noalloc_scratch) and passes that.
constexpr size_t kScratchAccOff = 0, kScratchGradOff = 256;
constexpr size_t kScratchBytes = (kScratchGradOff + sizeof(float) * MLP_NPARAM + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the GPU that runs `stream` (the current
// device for the null stream), resolved on the first call per device with
// that device current and cached.
int noalloc_scratch(hipStream_t stream, unsigned char** out) {
  int dev = -1;
  if (stream) {
    hipDevice_t d;
    if (hipStreamGetDevice(stream, &d) != hipSuccess) return HODE_EHIP;
    dev = (int)d;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return HODE_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return HODE_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return HODE_EHIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return HODE_EHIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return HODE_EHIP;
    if (e != hipSuccess || !p) return HODE_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return HODE_OK;
}

}  // namespace
}  // namespace hode

using namespace hode;

extern "C" {

int hode_mlp_forward(const uint16_t* Wb, const float* X, float* Y, int64_t B, void* stream) {
  if (!Wb || !X || !Y || B < 0) return HODE_EINVAL;
  if (B == 0) return HODE_OK;
  hipStream_t s = (hipStream_t)stream;
  mlp_forward_k<<<(unsigned)((B + 63) / 64), 256, 0, s>>>(Wb, X, Y, B);
  if (hipGetLastError() != hipSuccess) return HODE_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? HODE_OK : HODE_EHIP;
}

int hode_mlp_quantize(const float* Wm, uint16_t* Wb, void* stream) {
  if (!Wm || !Wb) return HODE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  quantize_k<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(Wm, Wb);
  if (hipGetLastError() != hipSuccess) return HODE_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? HODE_OK : HODE_EHIP;
}

int hode_mlp_loss_grad(const uint16_t* Wb, const float* X, const float* T, const float* Wt, const int64_t* idx,
                       int64_t B, float* grad, double* acc, double* loss_out, void* stream) {
  if (!Wb || !X || !T || !Wt || !grad || !acc || B < 1) return HODE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  fill_k<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(grad, MLP_NPARAM, acc, 2);
  int gw = (int)std::min<int64_t>((B + 255) / 256, 1024);
  mlp_wsum_k<<<gw, 256, 0, s>>>(Wt, idx, B, acc);
  mlp_grad_k<<<(unsigned)((B + 63) / 64), 256, 0, s>>>(Wb, X, T, Wt, idx, B, grad, acc);
  if (hipGetLastError() != hipSuccess) return HODE_EHIP;
  if (loss_out) {
    double h[2];
    if (hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return HODE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return HODE_EHIP;
    *loss_out = h[1];
  }
  return HODE_OK;
}

int hode_mlp_train_step(const float* X, const float* T, const float* Wt, const int64_t* idx, int64_t B, float* Wm,
                        uint16_t* Wb, float* m, float* v, float* grad, double* acc, int64_t step, float lr,
                        double* loss_out, void* stream) {
  if (!Wm || !m || !v || step < 1 || !(lr > 0)) return HODE_EINVAL;
  int rc = hode_mlp_loss_grad(Wb, X, T, Wt, idx, B, grad, acc, nullptr, stream);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
  adam_k<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(Wm, Wb, grad, m, v, lr, c1, c2);
  if (hipGetLastError() != hipSuccess) return HODE_EHIP;
  if (loss_out) {
    double h[2];
    if (hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return HODE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return HODE_EHIP;
    *loss_out = h[1];
  }
  return HODE_OK;
}

int hode_mlp_train_step_noalloc(const float* X, const float* T, const float* Wt, const int64_t* idx, int64_t B,
                                float* Wm, uint16_t* Wb, float* m, float* v, int64_t step, float lr,
                                double* loss_out, void* stream) {
  if (!X || !T || !Wt || !Wb || !Wm || !m || !v || step < 1 || !(lr > 0)) return HODE_EINVAL;
  if (B < 1 || B > HODE_MLP_NOALLOC_MAX_B) return HODE_EINVAL;  // outside 1 .. 2^31 - 1 samples
  unsigned char* base = nullptr;
  const int rc = noalloc_scratch((hipStream_t)stream, &base);
  if (rc) return rc;
  // the same kernels as hode_mlp_train_step, with the gradient and the loss
  // sums in this GPU's scratch (cleared by the first kernel of every call)
  return hode_mlp_train_step(X, T, Wt, idx, B, Wm, Wb, m, v, (float*)(base + kScratchGradOff),
                             (double*)(base + kScratchAccOff), step, lr, loss_out, stream);
}

}  // extern "C"
