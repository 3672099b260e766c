// qsgs_device.h -- device-side building blocks of libqsgs (gfx950, wave64).
//
// Philox4x32-10, the 26-direction tables, the integer form of Eq. (1), the
// XCD-aware work split and wavefront-aggregated list appends.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsgs {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // default workgroup: 4 waves
constexpr int kMaxBlock = 512;         // largest tunable workgroup of the item kernels
constexpr uint32_t kNumXcd = 8;        // workgroup b runs on XCD b % 8

// Philox counter word 3: separates the seeding stream from the two growth streams.
constexpr uint32_t kTagSeed = 1u;
constexpr uint32_t kTagGrowHi = 2u;
constexpr uint32_t kTagGrowLo = 3u;

constexpr uint64_t kOne32 = 1ull << 32;  // threshold of probability 1

// Grid values inside a growth step: 0 void, 1 solid at the step's start, 2 grown
// during this step (void at the step's start).  Between steps only 0 and 1 occur.
constexpr uint8_t kVoid = 0, kSolid = 1, kGrown = 2;

struct U4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32->64
// multiplies with the round key added by Weyl increments.  The key is wave-uniform,
// so the key schedule lives in scalar registers.
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p2 = (uint64_t)c2 * 0xCD9E8D57u;
    // three-input XOR in one instruction (LUT 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p2 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p2;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const U4& v, uint32_t i) {
  const uint32_t lo = (i & 1) ? v.y : v.x;
  const uint32_t hi = (i & 1) ? v.w : v.z;
  return (i & 2) ? hi : lo;
}

// Direction tables, 2 bits per direction d = 0..25 (d skips the centre k = 13 of
// k = (dx+1) + 3(dy+1) + 9(dz+1)).  Fields: dx+1, dy+1, dz+1 and the class.
constexpr uint64_t pack_direction_field(int field) {
  uint64_t m = 0;
  for (int d = 0; d < 26; ++d) {
    const int k = d < 13 ? d : d + 1;
    const int u[3] = {k % 3, (k / 3) % 3, k / 9};
    const int cls = (u[0] != 1) + (u[1] != 1) + (u[2] != 1) - 1;
    const int val = field < 3 ? u[field] : cls;
    m |= (uint64_t)val << (2 * d);
  }
  return m;
}
constexpr uint64_t kDirDX = pack_direction_field(0);
constexpr uint64_t kDirDY = pack_direction_field(1);
constexpr uint64_t kDirDZ = pack_direction_field(2);
constexpr uint64_t kDirClass = pack_direction_field(3);

__device__ __forceinline__ int dir_field(uint64_t table, int d) {
  return (int)((table >> (2 * d)) & 3u);
}

// Eq. (1) in integers: floor(t_ref * (20 S* - 19 cnt) / S*) capped at 2^32, for
// cnt < S* < 2^31.  The product can reach 2^68, so it is formed in two 64-bit
// pieces and divided by long division (one thread per step evaluates this).
__device__ __forceinline__ uint64_t eq1_threshold(uint64_t t_ref, uint64_t cnt, uint64_t s_star) {
  if (t_ref == 0) return 0;
  if (t_ref >= kOne32) return kOne32;  // factor >= 1 keeps probability 1
  const uint64_t num = 20ull * s_star - 19ull * cnt;      // < 2^36
  const uint64_t lo_prod = t_ref * (num & 0xFFFFFFFFull);  // < 2^64
  const uint64_t p_hi = (lo_prod >> 32) + t_ref * (num >> 32);
  const uint64_t p_lo = lo_prod & 0xFFFFFFFFull;
  const uint64_t q_hi = p_hi / s_star;
  const uint64_t r = p_hi % s_star;                        // < 2^31
  if (q_hi != 0) return kOne32;                            // quotient >= 2^32
  const uint64_t q_lo = ((r << 32) | p_lo) / s_star;       // < 2^32
  return q_lo;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-wide exclusive prefix sum of `cnt` plus one atomicAdd per wave on *counter;
// returns this lane's first slot.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t cnt, uint32_t* counter) {
  const uint32_t lane = lane_id();
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, kWave);
    if (lane >= (uint32_t)off) incl += v;
  }
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  uint32_t base = 0;
  if (lane == kWave - 1 && total != 0) base = atomicAdd(counter, total);
  base = __shfl(base, kWave - 1, kWave);
  return base + incl - cnt;
}

// Ballot variant for 0/1 counts.
__device__ __forceinline__ uint32_t wave_append_flag(bool flag, uint32_t* counter) {
  const uint64_t mask = __ballot(flag);
  if (mask == 0) return 0;  // (uniform) nothing to append
  const uint32_t lane = lane_id();
  const uint32_t total = (uint32_t)__popcll(mask);
  uint32_t base = 0;
  if (lane == 0 && total != 0) base = atomicAdd(counter, total);
  base = __shfl(base, 0, kWave);
  return base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

}  // namespace qsgs
