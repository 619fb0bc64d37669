// Learned pair-insertion proposal: a 3-layer perceptron (352 -> 128 -> 128 -> 128)
// that maps features of a configuration and a flavor to two 64-bin categorical
// densities, one for the creator time tau_s and one for the pair length l.  BF16
// weights and activations on the matrix cores (v_mfma_f32_32x32x16_bf16, FP32
// accumulation), FP32 master weights, softmax / cross-entropy, backward and Adam
// all on the device.  The proposal density of a pair is
//   q(tau_s, l) = (1 - eps) p_tau(bin tau_s) (64 / beta) p_l(bin l) (64 / beta) + eps / beta^2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "hyb_internal.h"
#include "mlp_kernels.h"

namespace hyb {

#define MLP_HIP_TRY(expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// ---- matrix-core GEMM ---------------------------------------------------------

// C[i][j] = sum_k A(i, k) B(k, j) (+ bias[j]), A(i, k) = A[i * sai + k * sak],
// B(k, j) = B[k * sbk + j * sbj], BF16 operands, FP32 accumulation.  One wavefront
// per 32 x 32 tile of C; operands are gathered element by element (any strides),
// out-of-range rows / columns / depth read as zero.
// Epilogue: relu != 0 clamps at zero; mask (FP32, same layout as C) zeroes C where
// mask <= 0 (the ReLU derivative); Cb receives a BF16 copy.
__global__ __launch_bounds__(64) void k_gemm_bf16(int M, int N, int K, const __bf16* __restrict__ A, int64_t sai,
                                                  int64_t sak, const __bf16* __restrict__ B, int64_t sbk,
                                                  int64_t sbj, float* __restrict__ C, int64_t ldc,
                                                  const float* __restrict__ bias, int relu,
                                                  const float* __restrict__ mask, __bf16* __restrict__ Cb,
                                                  int64_t ldcb) {
  const int l = threadIdx.x;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int ia = i0 + (l & 31), jb = j0 + (l & 31), kh = 8 * (l >> 5);
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kh + e;
      a[e] = (ia < M && k < K) ? A[ia * sai + k * sak] : __bf16(0.0f);
      b[e] = (jb < N && k < K) ? B[k * sbk + jb * sbj] : __bf16(0.0f);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + (v >> 2) * 8 + (l >> 5) * 4 + (v & 3);
    const int j = j0 + (l & 31);
    if (i < M && j < N) {
      float x = acc[v];
      if (bias) x += bias[j];
      if (relu && x < 0.0f) x = 0.0f;
      if (mask && !(mask[i * ldc + j] > 0.0f)) x = 0.0f;
      C[i * ldc + j] = x;
      if (Cb) Cb[i * ldcb + j] = __bf16(x);
    }
  }
}

// ---- loss and its gradient -----------------------------------------------------

// Per sample: two softmaxes over 64 logits; loss = -log p_tau[t0] - log p_l[t1];
// dZ = (softmax - onehot) / B (FP32 and BF16 copies).  One wavefront per sample.
__global__ __launch_bounds__(64) void k_softmax_ce(int Bn, const float* __restrict__ Z, const int32_t* __restrict__ tgt,
                                                   float* __restrict__ dZ, __bf16* __restrict__ dZb,
                                                   float* __restrict__ loss) {
  const int m = blockIdx.x, l = threadIdx.x;
  if (m >= Bn) return;
  float tot = 0.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float z = Z[m * MLP_OUT + h * MLP_BINS + l];
    float mx = z;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    const float e = expf(z - mx);
    float s = e;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float p = e / s;
    const int t = tgt[2 * m + h];
    const float g = (p - (l == t ? 1.0f : 0.0f)) / float(Bn);
    dZ[m * MLP_OUT + h * MLP_BINS + l] = g;
    dZb[m * MLP_OUT + h * MLP_BINS + l] = __bf16(g);
    if (l == t) tot += -(z - mx - logf(s));
  }
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if (l == 0) loss[m] = tot;
}

// db[j] = sum_m dZ[m][j], added in row order.  The rows are loaded in batches of
// 32 before they are added, so 32 loads are in flight instead of one.
__global__ void k_colsum(int Bn, int N, const float* __restrict__ dZ, float* __restrict__ db) {
  constexpr int U = 32;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  int m = 0;
  for (; m + U <= Bn; m += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = dZ[size_t(m + u) * N + j];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; m < Bn; ++m) s += dZ[size_t(m) * N + j];
  db[j] = s;
}

// Adam on FP32 master weights; refreshes the BF16 copy.
__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, __bf16* __restrict__ wb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float upd = lr * (a / c1) / (sqrtf(b / c2) + eps);
  w[i] -= upd;
  if (wb) wb[i] = __bf16(w[i]);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, __bf16* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = __bf16(x[i]);
}

// ---- host helpers --------------------------------------------------------------

static int gemm(int M, int N, int K, const __bf16* A, int64_t sai, int64_t sak, const __bf16* B, int64_t sbk,
                int64_t sbj, float* C, int64_t ldc, const float* bias, int relu, const float* mask, __bf16* Cb,
                int64_t ldcb, hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  dim3 grid((M + 31) / 32, (N + 31) / 32);
  k_gemm_bf16<<<grid, 64, 0, s>>>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, relu, mask, Cb, ldcb);
  MLP_HIP_TRY(hipGetLastError());
  return 0;
}

int mlp_forward(hyb_mlp* p, int Bn, const __bf16* X, MlpActs& a, hipStream_t s) {
  int rc;
  if ((rc = gemm(Bn, MLP_H, MLP_IN, X, MLP_IN, 1, p->wb[0], 1, MLP_IN, a.z1, MLP_H, p->bias[0], 1, nullptr, a.h1,
                 MLP_H, s)))
    return rc;
  if ((rc = gemm(Bn, MLP_H, MLP_H, a.h1, MLP_H, 1, p->wb[1], 1, MLP_H, a.z2, MLP_H, p->bias[1], 1, nullptr, a.h2,
                 MLP_H, s)))
    return rc;
  return gemm(Bn, MLP_OUT, MLP_H, a.h2, MLP_H, 1, p->wb[2], 1, MLP_H, a.z3, MLP_OUT, p->bias[2], 0, nullptr, nullptr,
              0, s);
}

int mlp_ensure(hyb_mlp* p, int Bn);
static int grow(hyb_mlp* p, int Bn) { return mlp_ensure(p, Bn); }

int mlp_ensure(hyb_mlp* p, int Bn) {
  if (Bn <= p->cap) return 0;
  // every new buffer is allocated before any old one is released: on failure the
  // network keeps its old buffers and capacity, and nothing allocated here leaks
  std::vector<void*> fresh;
  bool ok = true;
  auto alloc = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (!ok || hipMalloc(&q, bytes) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    fresh.push_back(q);
    return q;
  };
  const size_t B = size_t(Bn);
  MlpActs a{};
  a.z1 = static_cast<float*>(alloc(B * MLP_H * 4));
  a.z2 = static_cast<float*>(alloc(B * MLP_H * 4));
  a.z3 = static_cast<float*>(alloc(B * MLP_OUT * 4));
  a.h1 = static_cast<__bf16*>(alloc(B * MLP_H * 2));
  a.h2 = static_cast<__bf16*>(alloc(B * MLP_H * 2));
  float* dz3 = static_cast<float*>(alloc(B * MLP_OUT * 4));
  float* dz2 = static_cast<float*>(alloc(B * MLP_H * 4));
  float* dz1 = static_cast<float*>(alloc(B * MLP_H * 4));
  __bf16* dz3b = static_cast<__bf16*>(alloc(B * MLP_OUT * 2));
  __bf16* dz2b = static_cast<__bf16*>(alloc(B * MLP_H * 2));
  __bf16* dz1b = static_cast<__bf16*>(alloc(B * MLP_H * 2));
  float* loss = static_cast<float*>(alloc(B * 4));
  if (!ok) {
    for (void* q : fresh) (void)hipFree(q);
    return set_error(HYB_E_OOM, "MLP activations for batch %d", Bn);
  }
  // work already queued on the old buffers must finish before they are released
  MLP_HIP_TRY(hipDeviceSynchronize());
  for (void* q : p->act_allocs) (void)hipFree(q);
  p->act_allocs = fresh;
  p->acts = a;
  p->dz3 = dz3;
  p->dz2 = dz2;
  p->dz1 = dz1;
  p->dz3b = dz3b;
  p->dz2b = dz2b;
  p->dz1b = dz1b;
  p->loss = loss;
  p->cap = Bn;
  return 0;
}

// Gradients of the mean loss over the batch into p->grad (FP32, same layout as the
// weights); *loss_out = mean loss (host, synchronises) when non-null.
static int mlp_backward(hyb_mlp* p, int Bn, const __bf16* X, const int32_t* tgt, float* loss_out, hipStream_t s) {
  int rc = grow(p, Bn);
  if (rc) return rc;
  MlpActs& a = p->acts;
  if ((rc = mlp_forward(p, Bn, X, a, s))) return rc;
  k_softmax_ce<<<Bn, 64, 0, s>>>(Bn, a.z3, tgt, p->dz3, p->dz3b, p->loss);
  // layer 3: dWT3[n][k] = sum_m dZ3[m][n] H2[m][k]; db3; dZ2 = (dZ3 W3^T) masked by Z2 > 0
  if ((rc = gemm(MLP_OUT, MLP_H, Bn, p->dz3b, 1, MLP_OUT, a.h2, MLP_H, 1, p->grad[2], MLP_H, nullptr, 0, nullptr,
                 nullptr, 0, s)))
    return rc;
  k_colsum<<<MLP_OUT / 64, 64, 0, s>>>(Bn, MLP_OUT, p->dz3, p->gbias[2]);
  if ((rc = gemm(Bn, MLP_H, MLP_OUT, p->dz3b, MLP_OUT, 1, p->wb[2], MLP_H, 1, p->dz2, MLP_H, nullptr, 0, a.z2,
                 p->dz2b, MLP_H, s)))
    return rc;
  // layer 2
  if ((rc = gemm(MLP_H, MLP_H, Bn, p->dz2b, 1, MLP_H, a.h1, MLP_H, 1, p->grad[1], MLP_H, nullptr, 0, nullptr, nullptr,
                 0, s)))
    return rc;
  k_colsum<<<MLP_H / 64, 64, 0, s>>>(Bn, MLP_H, p->dz2, p->gbias[1]);
  if ((rc = gemm(Bn, MLP_H, MLP_H, p->dz2b, MLP_H, 1, p->wb[1], MLP_H, 1, p->dz1, MLP_H, nullptr, 0, a.z1, p->dz1b,
                 MLP_H, s)))
    return rc;
  // layer 1
  if ((rc = gemm(MLP_H, MLP_IN, Bn, p->dz1b, 1, MLP_H, X, MLP_IN, 1, p->grad[0], MLP_IN, nullptr, 0, nullptr, nullptr,
                 0, s)))
    return rc;
  k_colsum<<<MLP_H / 64, 64, 0, s>>>(Bn, MLP_H, p->dz1, p->gbias[0]);
  MLP_HIP_TRY(hipGetLastError());
  if (loss_out) {
    std::vector<float> l(Bn);
    MLP_HIP_TRY(hipMemcpyAsync(l.data(), p->loss, sizeof(float) * Bn, hipMemcpyDeviceToHost, s));
    MLP_HIP_TRY(hipStreamSynchronize(s));
    double t = 0.0;
    for (float x : l) t += x;
    *loss_out = float(t / Bn);
  }
  return 0;
}

}  // namespace hyb

using namespace hyb;

namespace {
const int kWSize[3] = {MLP_H * MLP_IN, MLP_H * MLP_H, MLP_OUT * MLP_H};  // WT[n][k]
const int kBSize[3] = {MLP_H, MLP_H, MLP_OUT};

// splitmix64 (Steele, Lea, Flood 2014) for the initial weights
uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

extern "C" {

int hyb_mlp_destroy(hyb_mlp* p) {
  if (!p) return HYB_OK;
  for (void* q : p->allocs) (void)hipFree(q);
  for (void* q : p->act_allocs) (void)hipFree(q);
  delete p;
  return HYB_OK;
}

int hyb_mlp_create(uint64_t seed, hyb_mlp** out) {
  if (!out) return set_error(HYB_E_ARG, "NULL argument");
  *out = nullptr;
  hyb_mlp* p = new hyb_mlp();
  auto alloc = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
    p->allocs.push_back(q);
    (void)hipMemset(q, 0, bytes);
    return q;
  };
  for (int L = 0; L < 3; ++L) {
    p->w[L] = static_cast<float*>(alloc(size_t(kWSize[L]) * 4));
    p->wb[L] = static_cast<__bf16*>(alloc(size_t(kWSize[L]) * 2));
    p->grad[L] = static_cast<float*>(alloc(size_t(kWSize[L]) * 4));
    p->m1[L] = static_cast<float*>(alloc(size_t(kWSize[L]) * 4));
    p->m2[L] = static_cast<float*>(alloc(size_t(kWSize[L]) * 4));
    p->bias[L] = static_cast<float*>(alloc(size_t(kBSize[L]) * 4));
    p->gbias[L] = static_cast<float*>(alloc(size_t(kBSize[L]) * 4));
    p->bm1[L] = static_cast<float*>(alloc(size_t(kBSize[L]) * 4));
    p->bm2[L] = static_cast<float*>(alloc(size_t(kBSize[L]) * 4));
  }
  for (void* q : p->allocs)
    if (!q) {
      hyb_mlp_destroy(p);
      return set_error(HYB_E_OOM, "MLP weights");
    }
  // He-uniform initial weights from a counter-free splitmix stream; zero biases
  uint64_t st = seed;
  const int fan_in[3] = {MLP_IN, MLP_H, MLP_H};
  for (int L = 0; L < 3; ++L) {
    std::vector<float> h(kWSize[L]);
    const double lim = std::sqrt(6.0 / fan_in[L]) * (L == 2 ? 0.1 : 1.0);
    for (auto& x : h) x = float(lim * (2.0 * (double(splitmix(st) >> 11) / 9007199254740992.0) - 1.0));
    if (hipMemcpy(p->w[L], h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      hyb_mlp_destroy(p);
      return set_error(HYB_E_HIP, "MLP weight upload");
    }
    k_to_bf16<<<(kWSize[L] + 255) / 256, 256>>>(kWSize[L], p->w[L], p->wb[L]);
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    hyb_mlp_destroy(p);
    return set_error(HYB_E_HIP, "MLP initialisation");
  }
  *out = p;
  return HYB_OK;
}

int hyb_mlp_get_weights(const hyb_mlp* p, float* w, float* b) {
  if (!p) return set_error(HYB_E_ARG, "NULL argument");
  size_t ow = 0, ob = 0;
  for (int L = 0; L < 3; ++L) {
    if (w) MLP_HIP_TRY(hipMemcpy(w + ow, p->w[L], size_t(kWSize[L]) * 4, hipMemcpyDeviceToHost));
    if (b) MLP_HIP_TRY(hipMemcpy(b + ob, p->bias[L], size_t(kBSize[L]) * 4, hipMemcpyDeviceToHost));
    ow += kWSize[L];
    ob += kBSize[L];
  }
  return HYB_OK;
}

int hyb_mlp_set_weights(hyb_mlp* p, const float* w, const float* b) {
  if (!p || !w || !b) return set_error(HYB_E_ARG, "NULL argument");
  size_t ow = 0, ob = 0;
  for (int L = 0; L < 3; ++L) {
    MLP_HIP_TRY(hipMemcpy(p->w[L], w + ow, size_t(kWSize[L]) * 4, hipMemcpyHostToDevice));
    MLP_HIP_TRY(hipMemcpy(p->bias[L], b + ob, size_t(kBSize[L]) * 4, hipMemcpyHostToDevice));
    k_to_bf16<<<(kWSize[L] + 255) / 256, 256>>>(kWSize[L], p->w[L], p->wb[L]);
    // Adam starts over: first and second moments back to zero with the step count
    MLP_HIP_TRY(hipMemset(p->m1[L], 0, size_t(kWSize[L]) * 4));
    MLP_HIP_TRY(hipMemset(p->m2[L], 0, size_t(kWSize[L]) * 4));
    MLP_HIP_TRY(hipMemset(p->bm1[L], 0, size_t(kBSize[L]) * 4));
    MLP_HIP_TRY(hipMemset(p->bm2[L], 0, size_t(kBSize[L]) * 4));
    ow += kWSize[L];
    ob += kBSize[L];
  }
  MLP_HIP_TRY(hipDeviceSynchronize());
  p->t = 0;
  return HYB_OK;
}

int hyb_mlp_forward(hyb_mlp* p, int32_t n, const void* X, float* logits, void* stream) {
  if (!p || !X || !logits) return set_error(HYB_E_ARG, "NULL argument");
  if (n <= 0) return n == 0 ? HYB_OK : set_error(HYB_E_ARG, "negative batch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = grow(p, n);
  if (rc) return rc;
  MlpActs a = p->acts;
  a.z3 = logits;
  return mlp_forward(p, n, static_cast<const __bf16*>(X), a, s);
}

int hyb_mlp_gradients(hyb_mlp* p, int32_t n, const void* X, const int32_t* targets, float* w_grad, float* b_grad,
                      float* loss, void* stream) {
  if (!p || !X || !targets) return set_error(HYB_E_ARG, "NULL argument");
  if (n <= 0) return set_error(HYB_E_ARG, "batch must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = mlp_backward(p, n, static_cast<const __bf16*>(X), targets, loss, s);
  if (rc) return rc;
  size_t ow = 0, ob = 0;
  for (int L = 0; L < 3; ++L) {
    if (w_grad)
      MLP_HIP_TRY(hipMemcpyAsync(w_grad + ow, p->grad[L], size_t(kWSize[L]) * 4, hipMemcpyDeviceToHost, s));
    if (b_grad)
      MLP_HIP_TRY(hipMemcpyAsync(b_grad + ob, p->gbias[L], size_t(kBSize[L]) * 4, hipMemcpyDeviceToHost, s));
    ow += kWSize[L];
    ob += kBSize[L];
  }
  MLP_HIP_TRY(hipStreamSynchronize(s));
  return HYB_OK;
}

int hyb_mlp_train_step(hyb_mlp* p, int32_t n, const void* X, const int32_t* targets, float lr, float* loss,
                       void* stream) {
  if (!p || !X || !targets) return set_error(HYB_E_ARG, "NULL argument");
  if (n <= 0 || !(lr > 0.0f)) return set_error(HYB_E_ARG, "batch and learning rate must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = mlp_backward(p, n, static_cast<const __bf16*>(X), targets, loss, s);
  if (rc) return rc;
  p->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - std::pow(b1, float(p->t)), c2 = 1.0f - std::pow(b2, float(p->t));
  for (int L = 0; L < 3; ++L) {
    k_adam<<<(kWSize[L] + 255) / 256, 256, 0, s>>>(kWSize[L], p->w[L], p->grad[L], p->m1[L], p->m2[L], p->wb[L], lr,
                                                   b1, b2, eps, c1, c2);
    k_adam<<<1, 128, 0, s>>>(kBSize[L], p->bias[L], p->gbias[L], p->bm1[L], p->bm2[L], nullptr, lr, b1, b2, eps, c1,
                             c2);
  }
  MLP_HIP_TRY(hipGetLastError());
  return HYB_OK;
}

}  // extern "C"
