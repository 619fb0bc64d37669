// Block SpMM over many float32 vectors: Y = (H_b - c_b) X (the Krylov step's
// H_loc|v> product, Sec. III, applied to a panel of vectors at once).
//
// Layout: panels of 16 vectors, [n_vec/16][dim][16].  A panel is one contiguous
// dim*64-byte chunk (78 KB for the 1225-dimensional 7-orbital block), so each
// panel is read from HBM exactly once with 16-byte vector loads and staged in
// LDS; the CSR gather then reads LDS only.  The next panel is prefetched into
// registers while the current one is computed (software pipelining), and the
// output panel is written once with coalesced stores.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hyb_internal.h"

namespace hyb {

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(HYB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

constexpr int SPMM_NT = 512;
constexpr int SPMM_MAXDIM = 1280;                  // 80 KB of LDS per panel
constexpr int SPMM_PF = (SPMM_MAXDIM * 4 + SPMM_NT - 1) / SPMM_NT;  // float4 prefetch slots per thread

__global__ __launch_bounds__(SPMM_NT) void k_spmm16(BlockDev B, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const double* __restrict__ diag64,
                                                    const float* __restrict__ X, float* __restrict__ Y,
                                                    int64_t n_panels) {
  __shared__ float4 sx[SPMM_MAXDIM * 4];
  const int tid = threadIdx.x;
  const int dim = B.dim;
  const int n4 = dim * 4;  // float4 per panel
  const int c = tid & 15;
  float4 pf[SPMM_PF];
  int64_t p = blockIdx.x;
  if (p < n_panels) {
    const float4* src = reinterpret_cast<const float4*>(X) + p * n4;
#pragma unroll
    for (int k = 0; k < SPMM_PF; ++k) {
      const int i = tid + k * SPMM_NT;
      if (i < n4) pf[k] = src[i];
    }
  }
  for (; p < n_panels; p += gridDim.x) {
#pragma unroll
    for (int k = 0; k < SPMM_PF; ++k) {
      const int i = tid + k * SPMM_NT;
      if (i < n4) sx[i] = pf[k];
    }
    __syncthreads();
    const int64_t pn = p + gridDim.x;
    if (pn < n_panels) {
      const float4* src = reinterpret_cast<const float4*>(X) + pn * n4;
#pragma unroll
      for (int k = 0; k < SPMM_PF; ++k) {
        const int i = tid + k * SPMM_NT;
        if (i < n4) pf[k] = src[i];
      }
    }
    const float* sxf = reinterpret_cast<const float*>(sx);
    float* dst = Y + p * int64_t(dim) * 16;
    for (int r = tid >> 4; r < dim; r += SPMM_NT / 16) {
      const int g = B.state_off + r;
      const int j0 = rowptr[g], j1 = rowptr[g + 1];
      float acc = 0.0f;
      for (int j = j0; j < j1; ++j) acc += val[j] * sxf[col[j] * 16 + c];
      dst[r * 16 + c] = static_cast<float>(diag64[g] * static_cast<double>(sxf[r * 16 + c]) + static_cast<double>(acc));
    }
    __syncthreads();
  }
}

}  // namespace hyb

using namespace hyb;

extern "C" int hyb_block_spmm(hyb_model* m, int32_t block, int64_t n_vec, const float* X, float* Y, void* stream) {
  if (!m || !X || !Y) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded");
  if (block < 0 || block >= m->n_blocks) return set_error(HYB_E_ARG, "block %d out of range", block);
  if (n_vec < 0 || n_vec % 16) return set_error(HYB_E_ARG, "n_vec must be a non-negative multiple of 16");
  const BlockDev& B = m->blocks[block];
  if (B.dim > SPMM_MAXDIM) return set_error(HYB_E_ARG, "block dimension %d exceeds %d", B.dim, SPMM_MAXDIM);
  const int64_t n_panels = n_vec / 16;
  if (n_panels == 0 || B.dim == 0) return HYB_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0, n_cu = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_spmm16), SPMM_NT, 0));
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(n_panels, int64_t(std::max(per_cu, 1)) * n_cu));
  k_spmm16<<<unsigned(grid), SPMM_NT, 0, s>>>(B, m->dev.rowptr, m->dev.col, m->dev.val32, m->dev.diag64, X, Y,
                                              n_panels);
  HIP_TRY(hipGetLastError());
  return HYB_OK;
}
