// Internal constants and launchers of the learned surrogate (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "casim.h"

namespace casim {

constexpr int kMlpParams = CASIM_MLP_NPARAMS;
// offsets of W1 b1 W2 b2 W3 b3 W4 b4 in the flat parameter vector
constexpr int kOW1 = 0, kOB1 = kOW1 + 12 * 128, kOW2 = kOB1 + 128, kOB2 = kOW2 + 128 * 128;
constexpr int kOW3 = kOB2 + 128, kOB3 = kOW3 + 128 * 128, kOW4 = kOB3 + 128, kOB4 = kOW4 + 128 * 12;
static_assert(kOB4 + 12 == kMlpParams, "parameter layout");
constexpr int kMaxSplit = 64;
constexpr double kRateScale = 1e-12;          // targets are asinh(rate / kRateScale)
constexpr double kRateScaleInv = 1e12;
constexpr double kQFloor = 1e-12;             // features ln(q + kQFloor), ln(n + 1)

// splitmix64 (Steele, Lea & Flood 2014) of (seed, index) -> uniform [0, 1).
__host__ __device__ inline double hash_uniform(uint64_t seed, uint64_t i) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// float32 parameters and statistics currently held by the training context
// (nullptr when absent).
const float *mlp_params_device();
const casim_mlp_stats *mlp_stats_host();

// Inference set built by casim_surrogate_load.
struct SurrogateDev {
    const uint16_t *w;      // bfloat16 weights, transposed and padded (see casim_surrogate.hip)
    const float *bias;      // 128 + 128 + 128 + 16 biases
    const float *stats;     // casim_mlp_stats on the device
    float range_margin, maha_max;
};
bool surrogate_ready();
SurrogateDev surrogate_dev(float range_margin, float maha_max);

// Network rates of feature rows: with counters (the slot space of a
// surrogate step) the filled slots of each region, else rows [0, n).
hipError_t launch_surrogate_infer(const SurrogateDev &S, const float *feat, const uint16_t *gates, int64_t n,
                                  const unsigned long long *counters, int64_t rcap, float *rates,
                                  uint8_t *fallback, hipStream_t stream);

// Scatter slotted rates and trust-region flags back to point order.
hipError_t launch_slot_scatter(const int32_t *idx_map, int64_t ncol, int64_t nlev, int64_t ld,
                               const float *slot_rates, const uint8_t *slot_fb, float *rates_out, uint8_t *flags,
                               hipStream_t stream);

}  // namespace casim

// Thresholds of the current context (nullptr before casim_init).
const casim_thresholds *casim_current_thresholds();

// Record a HIP failure for casim_strerror; returns CASIM_EHIP.
int casim_record_hip_error(int code, const char *msg);
