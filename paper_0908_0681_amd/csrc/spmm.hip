// Block SpMM over many float32 vectors: Y = (H_b - c_b) X (the Krylov step's
// H_loc|v> product, Sec. III, applied to a panel of vectors at once).
//
// Layout: panels of 16 vectors, [n_vec/16][dim][16].  A panel is one contiguous
// dim*64-byte chunk (78 KB for the 1225-dimensional 7-orbital block), so each
// panel is read from HBM exactly once with 16-byte vector loads and staged in
// LDS; the sparse gather then reads LDS only, and the output panel is written
// once with 16-byte stores.  Two workgroups share a CU (80 KB of LDS each), so
// one stages its panel while the other computes.
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
constexpr int SPMM_PF = (SPMM_MAXDIM * 4 + SPMM_NT - 1) / SPMM_NT;  // float4 staged per thread
constexpr int SPMM_KCH = 4;                        // ELL slots loaded together
static_assert(SPMM_PF * SPMM_NT == SPMM_MAXDIM * 4, "staging covers the LDS panel exactly");

// The matrix is read in the block's padded ELL form with the row pairs (2q, 2q + 1)
// kept together and sorted by length (slot k of ELL row i at k * dim + i, ELL row i =
// row perm[i]), so two neighbouring lanes write the two 64-byte halves of one
// 128-byte line of Y.  Each lane owns a row and all 16 vectors of the panel: a slot
// costs one column and one value load (coalesced across the wavefront's rows),
// four 16-byte LDS reads of the referenced row and 16 FMAs; the row of Y leaves
// as four 16-byte stores.
__global__ __launch_bounds__(SPMM_NT) void k_spmm16(int dim, int state_off, int kell,
                                                    const int16_t* __restrict__ ecol,
                                                    const float* __restrict__ eval,
                                                    const int16_t* __restrict__ eperm,
                                                    const int16_t* __restrict__ elen,
                                                    const double* __restrict__ diag64,
                                                    const float* __restrict__ X, float* __restrict__ Y,
                                                    int64_t n_panels) {
  __shared__ float4 sx[SPMM_MAXDIM * 4];
  const int tid = threadIdx.x;
  const int n4 = dim * 4;  // float4 per panel
  for (int64_t p = blockIdx.x; p < n_panels; p += gridDim.x) {
    // stage the panel (all loads are independent and issue back to back); the
    // second workgroup on the CU computes meanwhile
    const float4* src = reinterpret_cast<const float4*>(X) + p * n4;
    {
      // every load is issued unconditionally (index clamped into the panel) so that
      // they are all in flight together; only the in-range ones are stored
      // (the LDS panel holds exactly SPMM_PF * SPMM_NT float4, so every store is in
      // bounds; slots past the panel receive clamped copies that are never read)
      float4 t[SPMM_PF];
#pragma clang loop unroll(full)
      for (int k = 0; k < SPMM_PF; ++k) t[k] = src[min(tid + k * SPMM_NT, n4 - 1)];
#pragma clang loop unroll(full)
      for (int k = 0; k < SPMM_PF; ++k) sx[tid + k * SPMM_NT] = t[k];
    }
    __syncthreads();
    float4* dst = reinterpret_cast<float4*>(Y) + p * n4;
    // A row is four 16-byte chunks.  Lane l visits chunk (h + l) % 4 at step h and
    // keeps its accumulators in that rotated order, so that the lanes of a
    // wavefront spread over all chunk positions (and LDS bank groups) instead of
    // all reading chunk h of different rows at once.
    const int rot = tid & 3;
    for (int i = tid; i < dim; i += SPMM_NT) {
      // ELL rows are sorted by pair length, so the rows of a wavefront need about the
      // same number of slots; each lane stops at its own row's length
      const int r = eperm[i];
      const int n = elen[i];
      float acc[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
      for (int k0 = 0; k0 < n; k0 += SPMM_KCH) {
        int cc[SPMM_KCH];
        float vv[SPMM_KCH];
#pragma unroll
        for (int q = 0; q < SPMM_KCH; ++q) {
          const bool ok = k0 + q < n;
          const int k = ok ? k0 + q : n - 1;
          cc[q] = ecol[k * dim + i];
          vv[q] = ok ? eval[k * dim + i] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < SPMM_KCH; ++q) {
          const float4* xr = sx + cc[q] * 4;
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const float4 x = xr[(h + rot) & 3];
            acc[4 * h + 0] += vv[q] * x.x;
            acc[4 * h + 1] += vv[q] * x.y;
            acc[4 * h + 2] += vv[q] * x.z;
            acc[4 * h + 3] += vv[q] * x.w;
          }
        }
      }
      const double dg = diag64[state_off + r];
      const float4* xs = sx + r * 4;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float4 x = xs[(h + rot) & 3];
        float4 o;
        o.x = static_cast<float>(dg * static_cast<double>(x.x) + static_cast<double>(acc[4 * h + 0]));
        o.y = static_cast<float>(dg * static_cast<double>(x.y) + static_cast<double>(acc[4 * h + 1]));
        o.z = static_cast<float>(dg * static_cast<double>(x.z) + static_cast<double>(acc[4 * h + 2]));
        o.w = static_cast<float>(dg * static_cast<double>(x.w) + static_cast<double>(acc[4 * h + 3]));
        dst[r * 4 + ((h + rot) & 3)] = o;
      }
    }
    __syncthreads();
  }
}

}  // namespace hyb

using namespace hyb;

extern "C" int hyb_block_spmm(hyb_model* m, int32_t block, int64_t n_vec, const float* X, float* Y, void* stream) {
  if (!m || !X || !Y) return set_error(HYB_E_ARG, "NULL argument");
  if (!m->uploaded) return set_error(HYB_E_STATE, "model not uploaded");
  if (m->p.storage != HYB_CSR) return set_error(HYB_E_STATE, "the block SpMM reads the ELL copy: needs HYB_CSR storage");
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
  const int kell = m->ell_k[block];
  const int16_t* ecol = m->dev.ell_col + m->ell_off[block];
  const float* eval = m->dev.ell_val32 + m->ell_off[block];
  const int16_t* eperm = m->dev.ell_perm + B.state_off;
  const int16_t* elen = m->dev.ell_len + B.state_off;
  // kell == 0 (diagonal-only block): the slot loop is empty and no ELL entry is read
  k_spmm16<<<unsigned(grid), SPMM_NT, 0, s>>>(B.dim, B.state_off, kell, ecol, eval, eperm, elen, m->dev.diag64, X,
                                              Y, n_panels);
  HIP_TRY(hipGetLastError());
  return HYB_OK;
}
