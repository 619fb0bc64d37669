// Internal declarations shared by the host model code and the HIP kernels of libhyb.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hyb.h"

namespace hyb {

int set_error(int code, const char* fmt, ...);

// Per-block metadata as seen by the device kernels (plain POD, uploaded as an array).
struct BlockDev {
  int32_t dim;        // number of states in the block
  int32_t state_off;  // offset of the block's states in the packed state / row arrays
  int32_t n_up, n_dn;
  double shift;       // c_b: lowest eigenvalue of the block; kernels apply H_b - c_b
  int32_t up_states;  // C(n_orb, n_up): index of state (up, dn) = rank_half[dn] * up_states + rank_half[up]
  float width;        // spectral width of the block (exact with the host spectrum, else a
                      // Gershgorin bound): weights a path's expected cost in the queue order
};

struct DeviceModel {
  // basis
  uint32_t* states = nullptr;   // [n_states] packed by block, ascending inside a block
  int32_t* rank = nullptr;      // [n_states] state integer -> index inside its block
  int16_t* rank_half = nullptr; // [2^n_orb] one spin's occupation pattern -> its rank among the
                                // patterns of the same popcount (ascending integers)
  BlockDev* blocks = nullptr;   // [n_blocks]
  // off-diagonal CSR over the packed rows (column = index inside the same block)
  int32_t* rowptr = nullptr;    // [n_states + 1]
  int32_t* col = nullptr;       // [nnz]
  double* val64 = nullptr;      // [nnz]
  float* val32 = nullptr;       // [nnz]
  double* diag64 = nullptr;     // [n_states] h_ii - c_b
  // padded ELL copy of the off-diagonal part, per block [ell_k[b]][dim_b] (column-major
  // by slot), in-block column as int16 and value as float32; short rows are padded
  // with their own index and 0
  int16_t* ell_col = nullptr;
  float* ell_val32 = nullptr;
  int16_t* ell_perm = nullptr;  // [dim_b] per block: row pairs by descending length (ELL row i is row perm[i])
  int16_t* ell_len = nullptr;   // [dim_b] per block: length of ELL row i
  // the same rows in natural order for the trace kernels, every block padded to the
  // model-wide slot count tell_k: slot k of row r of block b at
  // state_off_b * tell_k + k * dim_b + r
  int16_t* tell_col = nullptr;
  double* tell_val64 = nullptr;
  float* tell_val32 = nullptr;
  // retained set
  int32_t* ret_block = nullptr; // [n_ret]
  double* ret_energy = nullptr; // [n_ret]
  int64_t* ret_off = nullptr;   // [n_ret] offset into ret_vec
  double* ret_vec64 = nullptr;
  float* ret_vec32 = nullptr;
  // per-batch workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int device = -1;
};

}  // namespace hyb

struct hyb_model {
  hyb_model_params p{};
  std::vector<double> eps;
  int n_orb = 0, F = 0, n_blocks = 0, max_dim = 0;
  int64_t n_states = 0;
  // basis
  std::vector<uint32_t> states;      // packed by block
  std::vector<int32_t> rank;         // state -> index inside block
  std::vector<int16_t> rank_half;    // one spin's pattern -> rank among same-popcount patterns
  std::vector<int32_t> block_of;     // state -> block
  std::vector<hyb::BlockDev> blocks;
  // H_loc: diagonal + off-diagonal CSR (packed rows)
  std::vector<double> diag;          // h_ii
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  // spectrum
  std::vector<std::vector<double>> evals;   // per block, ascending
  double E0 = 0.0;
  // retained set
  std::vector<int32_t> ret_block;
  std::vector<int32_t> ret_index;    // eigen-index of each retained state inside its block
  std::vector<double> ret_energy;
  std::vector<int64_t> ret_off;
  std::vector<double> ret_vec;
  // ELL layout of each block (built at upload): slots per row and offset of the block
  std::vector<int32_t> ell_k;
  int32_t tell_k = 0;            // largest number of off-diagonal entries in a row
  std::vector<int64_t> ell_off;
  // device side
  bool uploaded = false;
  uint64_t dev_gen = 0;     // bumped by every upload: device pointers captured earlier are stale
  hyb::DeviceModel dev;
  int variant = -1;         // trace kernel variant (-1 = automatic)
  int chunk = 1;            // operators per path-step launch (1 = one launch per step kind)
  bool timing = false;
  float last_ms[7] = {0, 0, 0, 0, 0, 0, 0};
  void* events[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<void*> step_events;  // pairs around each step launch when timing
  void* mat = nullptr;      // matrix formulation (matrix.hip), built by hyb_matrix_build
};

namespace hyb {
// eigen.cpp
// Dense symmetric eigensolver: eigenvalues (ascending) of the n x n row-major matrix a;
// if n_vec > 0, also the eigenvectors of the n_vec lowest eigenvalues (columns of
// vec, row-major n x n_vec).  Returns 0 or a negative error code.
int sym_eig(int n, const double* a, double* evals, int n_vec, double* vec);
void free_device(hyb_model* m);
void matrix_release(hyb_model* m);  // matrix.hip: frees the matrix formulation's device data
// 0 when E0 and the retained set exist (always with HYB_SPECTRUM_HOST; after
// hyb_init_lanczos with HYB_SPECTRUM_DEVICE), else a state error.
inline int require_spectrum(const hyb_model* m) {
  return m->ret_block.empty() ? set_error(HYB_E_STATE, "no retained set yet: a model created with "
                                          "HYB_SPECTRUM_DEVICE needs hyb_init_lanczos first")
                              : 0;
}
}  // namespace hyb
