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
// cnt < S* < 2^31.  The product can reach 2^68: the quotient is estimated in double
// precision (a relative error of at most 2^-52, so within 2^-19 of the exact quotient
// while that is below 2^32 + 3) and its floor corrected once by the exact remainder,
// which is formed modulo 2^64 (it lies in (-S*, 2 S*), far inside the signed range).
__device__ __forceinline__ uint64_t eq1_threshold(uint64_t t_ref, uint64_t cnt, uint64_t s_star) {
  if (t_ref == 0) return 0;
  if (t_ref >= kOne32) return kOne32;  // factor >= 1 keeps probability 1
  const uint64_t num = 20ull * s_star - 19ull * cnt;  // < 2^36
  const double qd = (double)t_ref * (double)num / (double)s_star;
  if (qd >= 4294967298.0) return kOne32;  // 2^32 + 2: the quotient is at least 2^32
  uint64_t q = (uint64_t)qd;
  const int64_t rem = (int64_t)(t_ref * num - q * s_star);
  if (rem < 0)
    --q;
  else if (rem >= (int64_t)s_star)
    ++q;
  return q >= kOne32 ? kOne32 : q;
}

// floor(x / y) for x < 2^53 and y > 0: the correctly rounded double quotient lies
// within x 2^-53 / y < 1 / y of x / y, closer than the next integer whenever x / y is
// not one, so its floor is exact.
__device__ __forceinline__ uint32_t floor_div53(uint64_t x, uint64_t y) {
  return (uint32_t)((double)x / (double)y);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Cross-lane steps through DPP: an operand read from another lane of the same row of
// 16 lanes (row_shr), or the last lane of a row broadcast into later rows (row_bcast),
// a few cycles each where a shuffle through the LDS crossbar takes tens.  Lanes with
// no source read 0.  Every lane of the wavefront must be active.
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ uint32_t dpp_take(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xF, true);
}

// Inclusive prefix sum (lane i: v_0 + ... + v_i) and prefix or over the wavefront.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  v += dpp_take<0x111>(v);       // row_shr:1
  v += dpp_take<0x112>(v);       // row_shr:2
  v += dpp_take<0x114>(v);       // row_shr:4
  v += dpp_take<0x118>(v);       // row_shr:8: prefixes within each row
  v += dpp_take<0x142, 0xA>(v);  // row_bcast:15: row 0's total into row 1, row 2's into row 3
  v += dpp_take<0x143, 0xC>(v);  // row_bcast:31: the total of rows 0-1 into rows 2 and 3
  return v;
}
__device__ __forceinline__ uint32_t wave_incl_or(uint32_t v) {
  v |= dpp_take<0x111>(v);
  v |= dpp_take<0x112>(v);
  v |= dpp_take<0x114>(v);
  v |= dpp_take<0x118>(v);
  v |= dpp_take<0x142, 0xA>(v);
  v |= dpp_take<0x143, 0xC>(v);
  return v;
}

// Wave-wide exclusive prefix sum of `cnt` plus one atomicAdd per wave on *counter;
// returns this lane's first slot.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t cnt, uint32_t* counter) {
  const uint32_t lane = lane_id();
  const uint32_t incl = wave_incl_sum(cnt);
  const uint32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
  uint32_t base = 0;
  if (lane == kWave - 1 && total != 0) base = atomicAdd(counter, total);
  base = __builtin_amdgcn_readlane(base, kWave - 1);
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
