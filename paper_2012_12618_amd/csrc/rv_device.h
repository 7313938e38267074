// rv_device.h -- device helpers shared by the library's kernel sources
// (rv.hip: velocity-profile estimator; rv_paper.hip: paper-literal variant).
// Not part of the C ABI.
#ifndef RV_DEVICE_H
#define RV_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kWave = 64;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;


// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// mixed into the counter words, key advanced by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        // one 32x32->64 multiply-add instruction per product
        const uint64_t p0 = (uint64_t)kPhiloxM0 * x.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * x.z;
        x = make_uint4((uint32_t)(p1 >> 32) ^ x.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ x.w ^ k1, (uint32_t)p0);
    }
    return x;
}

// Two distinct indices in [0, n) from two uniform words (multiply-shift map;
// the second index skips the first).  Requires 2 <= n < 2^31.
__device__ __forceinline__ void seed_pair(uint32_t u0, uint32_t u1, uint32_t n, uint32_t &i,
                                          uint32_t &j) {
    i = (uint32_t)(((uint64_t)u0 * n) >> 32);
    const uint32_t b = (uint32_t)(((uint64_t)u1 * (n - 1u)) >> 32);
    j = b + (b >= i ? 1u : 0u);
}

struct Span {
    int64_t lo;
    int64_t n;
    bool ok;
};

// Points [off[k] - base, off[k+1] - base) of a frame's n_points; `base` is the
// frame index of the first point when the frame is a part of a larger one.
__device__ __forceinline__ Span cluster_span(const int32_t *__restrict__ off, int64_t k,
                                             int64_t n_points, int64_t base = 0) {
    const int64_t a = off[k] - base;
    const int64_t b = off[k + 1] - base;
    Span s;
    s.ok = a >= 0 && b >= a && b <= n_points;
    s.lo = s.ok ? a : 0;
    s.n = s.ok ? b - a : 0;
    return s;
}

// Lane 0's value of v in every lane, as a wave-uniform (scalar) value.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

}  // namespace

#endif
