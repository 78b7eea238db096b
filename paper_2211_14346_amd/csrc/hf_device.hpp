// Device helpers shared by the gfx950 kernels: wave64 primitives, the
// Philox4x32-10 counter-based generator and Box-Muller normals.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Bits of lanes below the calling lane.
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// In-row lane exchanges by DPP (no LDS round trip): kCtrl is the DPP control
// word (quad_perm 0xB1 = lane ^ 1, 0x4E = lane ^ 2; 0x141 = row_half_mirror,
// lane i <-> 7 - i within eight lanes; 0x140 = row_mirror, i <-> 15 - i
// within sixteen).  Every pattern used is a permutation inside each row, so
// no lane reads outside the wavefront.
template <int kCtrl>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, kCtrl, 0xF, 0xF, false);
}

template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_i32<kCtrl>(hi), dpp_i32<kCtrl>(lo));
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds; each round multiplies
// counter words 0 and 2 by the two round constants (32x32 -> 64) and mixes
// the halves with words 1 and 3 and the round key; the key is bumped by the
// two Weyl constants between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform in (0, 1) from the top 24 bits; exact in FP32 and FP64.
template <typename T>
__device__ __forceinline__ T uniform24(uint32_t x) {
    return ((T)(x >> 8) + (T)0.5) * (T)(1.0 / 16777216.0);
}

// Box-Muller pair from two raw words: (r cos 2 pi u2, r sin 2 pi u2),
// r = sqrt(-2 ln u1).
// FP32: the hardware base-2 logarithm and the revolution-scaled sine/cosine
// units (sin(2 pi u) is one instruction on u itself).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &z0, float &z1) {
    const float u1 = uniform24<float>(a);
    const float u2 = uniform24<float>(b);
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));  // -2 ln u1
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &z0, double &z1) {
    const double u1 = uniform24<double>(a);
    const double u2 = uniform24<double>(b);
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Raw words of Philox block blk of event g, variation v.
__device__ __forceinline__ U4 philox_block(uint64_t seed, uint64_t g, uint32_t v, uint32_t blk) {
    return philox4x32_10(U4{(uint32_t)g, (uint32_t)(g >> 32), v, blk}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Gaussian draws of one Philox block: slot 4*blk + j for j = 0..3.
template <typename T>
__device__ __forceinline__ void gauss_block(uint64_t seed, uint64_t g, uint32_t v, uint32_t blk, T z[4]) {
    U4 c{(uint32_t)g, (uint32_t)(g >> 32), v, blk};
    const U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    box_muller(r.x, r.y, z[0], z[1]);
    box_muller(r.z, r.w, z[2], z[3]);
}

// Gaussian draw of a single slot (computes only the Box-Muller pair it needs).
template <typename T>
__device__ __forceinline__ T gauss_slot(uint64_t seed, uint64_t g, uint32_t v, uint32_t slot) {
    U4 c{(uint32_t)g, (uint32_t)(g >> 32), v, slot >> 2};
    const U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    T z0, z1;
    if (slot & 2u)
        box_muller(r.z, r.w, z0, z1);
    else
        box_muller(r.x, r.y, z0, z1);
    return (slot & 1u) ? z1 : z0;
}

}  // namespace hf
