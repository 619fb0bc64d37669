// Shared declarations of the learned proposal: network shape, activations, the
// handle, and the feature map of a configuration (device function, one wavefront).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hyb {

constexpr int MLP_IN = 352;    // 34 F features for F <= 10, zero-padded to a multiple of 32
constexpr int MLP_H = 128;     // hidden width
constexpr int MLP_BINS = 64;   // bins of tau_s and of l on [0, beta)
constexpr int MLP_OUT = 2 * MLP_BINS;
constexpr int MLP_TBINS = 32;  // time bins of the occupation step functions

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct MlpActs {
  float* z1 = nullptr;
  float* z2 = nullptr;
  float* z3 = nullptr;
  __bf16* h1 = nullptr;
  __bf16* h2 = nullptr;
};

// Features of (configuration, flavor f) into x[0..MLP_IN): one-hot f (F entries),
// k_g / 32 for every flavor g (F entries), and for every flavor g the count of
// creators minus annihilators of g before the centre (b + 1/2) beta / 32 of each of
// 32 time bins (32 F entries); the remaining entries are zero.  The pair (ex_i,
// ex_j) of flavor ex_f (creator label ex_i, annihilator label ex_j) is left out
// when ex_f >= 0.  cre / ann / kf point at the chain's [F][kmax] lists.  All 64
// lanes take part; the values are small integers or multiples of 1/32 (exact in
// BF16).
__device__ inline void mlp_features(int F, int kmax, double beta, const int32_t* kf, const double* cre,
                                    const double* ann, int f, int ex_f, int ex_i, int ex_j, __bf16* x) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < MLP_IN; e += 64) {
    float v = 0.0f;
    if (e < F) {
      v = (e == f) ? 1.0f : 0.0f;
    } else if (e < 2 * F) {
      const int g = e - F;
      v = float(kf[g] - (g == ex_f ? 1 : 0)) * (1.0f / 32.0f);
    } else if (e < 2 * F + MLP_TBINS * F) {
      const int g = (e - 2 * F) / MLP_TBINS, b = (e - 2 * F) % MLP_TBINS;
      const double tb = (b + 0.5) * beta / MLP_TBINS;
      int cnt = 0;
      for (int q = 0; q < kf[g]; ++q) {
        if (!(g == ex_f && q == ex_i) && cre[g * kmax + q] < tb) ++cnt;
        if (!(g == ex_f && q == ex_j) && ann[g * kmax + q] < tb) --cnt;
      }
      v = float(cnt);
    }
    x[e] = __bf16(v);
  }
}

}  // namespace hyb

struct hyb_mlp {
  float* w[3] = {nullptr, nullptr, nullptr};      // FP32 master weights, output-major WT[n][k]
  __bf16* wb[3] = {nullptr, nullptr, nullptr};    // BF16 copies used by the matrix cores
  float* grad[3] = {nullptr, nullptr, nullptr};
  float* m1[3] = {nullptr, nullptr, nullptr};
  float* m2[3] = {nullptr, nullptr, nullptr};
  float* bias[3] = {nullptr, nullptr, nullptr};
  float* gbias[3] = {nullptr, nullptr, nullptr};
  float* bm1[3] = {nullptr, nullptr, nullptr};
  float* bm2[3] = {nullptr, nullptr, nullptr};
  int64_t t = 0;   // Adam step
  int cap = 0;     // batch capacity of the activation buffers
  hyb::MlpActs acts{};
  float* dz3 = nullptr;
  float* dz2 = nullptr;
  float* dz1 = nullptr;
  __bf16* dz3b = nullptr;
  __bf16* dz2b = nullptr;
  __bf16* dz1b = nullptr;
  float* loss = nullptr;
  std::vector<void*> allocs, act_allocs;
};

namespace hyb {
int mlp_forward(hyb_mlp* p, int Bn, const __bf16* X, MlpActs& a, hipStream_t s);
int mlp_ensure(hyb_mlp* p, int Bn);  // activation buffers for batches up to Bn
}  // namespace hyb
