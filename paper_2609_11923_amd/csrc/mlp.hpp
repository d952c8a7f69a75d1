// mlp.hpp -- interface between the warm-start kernels (mlp.hip) and the solver runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/cfr.h"

namespace cfrx {

// Inputs of the feature kernel; one row per canonical information set (games in order).
struct FeatureArgs {
    const int32_t *canon_off;  // [I + 1] canonical slot offsets (global over the batch)
    const int8_t *player;      // [I] acting player, 1 or 2
    const int32_t *slot_map;   // [A] canonical slot -> device slot, nullptr for the identity
    const int16_t *bucket;     // [I] hand bucket 0..63, other values: none
    const int16_t *history;    // [I] public-history code 0..31, other values: none
    const float *scalars;      // [I * 8]
    int64_t I;
    uint16_t *X;               // [I][128] bf16 out
    float *mag;                // [I] out: sum of |instantaneous regret| over the first four actions
};

// R: device-order regrets after one plain iteration from zero (float or double per fp64)
hipError_t launch_features(const FeatureArgs &f, const void *R, bool fp64, hipStream_t s);
// columns 120-127 from the current strategy and the strategy sums (device order)
hipError_t launch_features_probe(const FeatureArgs &f, const void *sigma, const double *sbar, bool fp64,
                                 hipStream_t s);
hipError_t launch_warm_regrets(const int32_t *canon_off, int64_t I, const float *z, const float *mag, float scale,
                               float *R0, hipStream_t s);
cfr_status mlp_forward_internal(cfr_mlp *n, const void *x, int64_t rows, float *z, hipStream_t s);
int mlp_in_dim(const cfr_mlp *n);
int mlp_device(const cfr_mlp *n);

// the thread-local message cfr_last_error() returns
void set_last_error(const std::string &m);

}  // namespace cfrx
