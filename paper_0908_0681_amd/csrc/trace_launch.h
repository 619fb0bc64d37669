// Device-resident trace launch used by the Monte Carlo layer: operator arrays,
// per-configuration ranges and outputs already live on the device, and the grids
// are sized for every (configuration, retained state) pair so that no host
// synchronisation is needed between launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct hyb_model;

namespace hyb {

// Bytes of workspace trace_resident needs for n_configs configurations.
size_t trace_ws_bytes(const hyb_model* m, int n_configs);

// Tr_R of configuration c = ops [begin[c], ends[c]) of (tau, flavor, dagger), for
// c < n_configs, into out_log[c] / out_sign[c].  max_ops bounds every range's
// length.  Validation and propagation error bits are ORed into *err_accum on the
// device.  Enqueued on stream s; returns 0 or a negative status (launch errors).
int trace_resident(hyb_model* m, int n_configs, const int64_t* begin, const int64_t* ends, const double* tau,
                   const int16_t* flavor, const int8_t* dagger, int max_ops, double beta, void* ws,
                   double* out_log, int8_t* out_sign, int32_t* err_accum, hipStream_t s);

// The kernel variant trace_resident launches for this model (it changes with
// hyb_set_trace_variant).
int trace_resident_variant(const hyb_model* m);

// Per (config, retained state) results of the last trace_resident on ws (pair id =
// config * n_retained + r): sign and log of each path's contribution t_r, and the
// block the path occupies at beta/2 (-1 for a path that leaves the physical range).
struct ResidentPairs {
  const int8_t* sign;
  const double* log;
  const int32_t* midblk;
};
ResidentPairs trace_resident_pairs(const hyb_model* m, int n_configs, void* ws);

}  // namespace hyb
