// qsgs_measure.hip -- measurement utilities (C ABI in include/qsgs.h): the occupancy one
// growth step reads, and the issue rate of plain 32-bit vector ALU instructions.
//
// Band sizes (qsgs_band_sizes), for the algorithmic byte count of a step: a step tests the
// 26 neighbours
// of every front voxel a in F_t (Sec. 2.3 step 3) and then keeps the voxels of
// F_t u New_t that still have a void neighbour (Sec. 2.3 step 4), so it reads the
// occupancy of the one-voxel band (Chebyshev distance <= 1) around F_t, then around
// F_t u New_t.  Two passes over the grid: mark F_t and F_t u New_t per cell, then count
// the cells whose closed 26-neighbourhood holds a mark of each kind.
#include "qsgs_host.h"

using namespace qsgs;
using namespace qsgs::host;

namespace {

constexpr uint32_t kBandBlock = 256;
constexpr uint32_t kBandGrid = 4096;

__device__ __forceinline__ void coords3(const Geometry& g, uint32_t v, int32_t& x, int32_t& y,
                                        int32_t& z) {
  const uint32_t q = v / (uint32_t)g.nx;
  x = (int32_t)(v - q * (uint32_t)g.nx);
  z = (int32_t)(q / (uint32_t)g.ny);
  y = (int32_t)(q - (uint32_t)z * (uint32_t)g.ny);
}

// mark[v] bit 0: v in F_t (solid before the step, with an in-domain void 26-neighbour);
// bit 1: v in F_t u New_t (New_t: void before, solid after).  Byte 0 is void, any other
// value solid.
__global__ __launch_bounds__(kBandBlock) void k_band_mark(const uint8_t* __restrict__ before,
                                                          const uint8_t* __restrict__ after,
                                                          uint8_t* __restrict__ mark,
                                                          Geometry g) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
       v += gridDim.x * blockDim.x) {
    int32_t x, y, z;
    coords3(g, v, x, y, z);
    const bool solid = before[v] != 0;
    bool front = false;
    if (solid) {
      for (int32_t dz = -1; dz <= 1 && !front; ++dz)
        for (int32_t dy = -1; dy <= 1 && !front; ++dy)
          for (int32_t dx = -1; dx <= 1; ++dx) {
            const int32_t X = x + dx, Y = y + dy, Z = z + dz;
            if (X < 0 || Y < 0 || Z < 0 || X >= g.nx || Y >= g.ny || Z >= g.nz) continue;
            if (before[(uint32_t)X + (uint32_t)g.nx * ((uint32_t)Y + (uint32_t)g.ny * (uint32_t)Z)] ==
                0) {
              front = true;
              break;
            }
          }
    }
    const bool grown = !solid && after[v] != 0;
    mark[v] = (uint8_t)((front ? 1u : 0u) | ((front || grown) ? 2u : 0u));
  }
}

// out[k] += cells whose closed in-domain 26-neighbourhood holds a cell with mark bit k.
__global__ __launch_bounds__(kBandBlock) void k_band_count(const uint8_t* __restrict__ mark,
                                                           Geometry g,
                                                           unsigned long long* __restrict__ out) {
  uint32_t c0 = 0, c1 = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
       v += gridDim.x * blockDim.x) {
    int32_t x, y, z;
    coords3(g, v, x, y, z);
    uint32_t acc = 0;
    for (int32_t dz = -1; dz <= 1; ++dz)
      for (int32_t dy = -1; dy <= 1; ++dy)
        for (int32_t dx = -1; dx <= 1; ++dx) {
          const int32_t X = x + dx, Y = y + dy, Z = z + dz;
          if (X < 0 || Y < 0 || Z < 0 || X >= g.nx || Y >= g.ny || Z >= g.nz) continue;
          acc |= mark[(uint32_t)X + (uint32_t)g.nx * ((uint32_t)Y + (uint32_t)g.ny * (uint32_t)Z)];
        }
    c0 += acc & 1u;
    c1 += (acc >> 1) & 1u;
  }
  __shared__ uint32_t s0[kBandBlock / kWave], s1[kBandBlock / kWave];
  for (int o = kWave / 2; o > 0; o >>= 1) {
    c0 += __shfl_xor(c0, o, kWave);
    c1 += __shfl_xor(c1, o, kWave);
  }
  if (threadIdx.x % kWave == 0) {
    s0[threadIdx.x / kWave] = c0;
    s1[threadIdx.x / kWave] = c1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t0 = 0, t1 = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
      t0 += s0[w];
      t1 += s1[w];
    }
    atomicAdd(&out[0], t0);
    atomicAdd(&out[1], t1);
  }
}

__global__ void k_band_zero(unsigned long long* out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0;
}

size_t band_counter_offset(uint32_t n) { return align_up((size_t)n); }

// Issue rate of plain 32-bit vector ALU instructions: eight independent chains of
// v_xor_b32 / v_add_u32 per lane (written in assembly so that every instruction stays),
// 16 instructions per iteration; one 32-bit result per thread keeps the chains live.
constexpr uint32_t kAluIters = 20000;
__global__ __launch_bounds__(256) void k_alu_rate(uint32_t* __restrict__ out, uint32_t seed) {
  uint32_t a0 = threadIdx.x ^ seed, a1 = a0 + 1u, a2 = a0 + 2u, a3 = a0 + 3u, a4 = a0 + 4u,
           a5 = a0 + 5u, a6 = a0 + 6u, a7 = a0 + 7u;
  const uint32_t b = seed * 3u + 1u;
  for (uint32_t i = 0; i < kAluIters; ++i) {
    asm volatile(
        "v_xor_b32 %0, %0, %8\n v_add_u32 %1, %1, %8\n v_xor_b32 %2, %2, %8\n"
        " v_add_u32 %3, %3, %8\n v_xor_b32 %4, %4, %8\n v_add_u32 %5, %5, %8\n"
        " v_xor_b32 %6, %6, %8\n v_add_u32 %7, %7, %8\n"
        " v_add_u32 %0, %0, %8\n v_xor_b32 %1, %1, %8\n v_add_u32 %2, %2, %8\n"
        " v_xor_b32 %3, %3, %8\n v_add_u32 %4, %4, %8\n v_xor_b32 %5, %5, %8\n"
        " v_add_u32 %6, %6, %8\n v_xor_b32 %7, %7, %8"
        : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
        : "v"(b));
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

}  // namespace

extern "C" {

size_t qsgs_band_scratch_bytes(const qsgs_dims* dims) {
  Geometry g{};
  if (check_dims(dims, &g) != QSGS_OK) return 0;
  return band_counter_offset(g.n) + 2 * sizeof(unsigned long long);
}

qsgs_status qsgs_band_sizes(const qsgs_dims* dims, const uint8_t* d_before,
                            const uint8_t* d_after, void* d_scratch, size_t scratch_bytes,
                            uint64_t* out, void* stream) {
  last_error().clear();
  Geometry g{};
  QSGS_TRY(check_dims(dims, &g));
  if (!d_before || !d_after || !d_scratch || !out)
    return fail(QSGS_ERR_INVALID, "NULL pointer argument");
  const size_t need = band_counter_offset(g.n) + 2 * sizeof(unsigned long long);
  if (scratch_bytes < need)
    return fail(QSGS_ERR_WORKSPACE, "scratch needs %zu bytes, got %zu", need, scratch_bytes);
  if (((uintptr_t)d_scratch & 7u) != 0) return fail(QSGS_ERR_INVALID, "scratch not 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* mark = (uint8_t*)d_scratch;
  unsigned long long* cnt = (unsigned long long*)(mark + band_counter_offset(g.n));
  const uint32_t blocks = std::min<uint32_t>(kBandGrid, (g.n + kBandBlock - 1) / kBandBlock);
  hipLaunchKernelGGL(k_band_zero, dim3(1), dim3(64), 0, s, cnt);
  QSGS_LAUNCHED("k_band_zero");
  hipLaunchKernelGGL(k_band_mark, dim3(blocks), dim3(kBandBlock), 0, s, d_before, d_after, mark,
                     g);
  QSGS_LAUNCHED("k_band_mark");
  hipLaunchKernelGGL(k_band_count, dim3(blocks), dim3(kBandBlock), 0, s, mark, g, cnt);
  QSGS_LAUNCHED("k_band_count");
  unsigned long long h[2] = {0, 0};
  QSGS_HIP(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  out[0] = h[0];
  out[1] = h[1];
  return QSGS_OK;
}

size_t qsgs_alu_scratch_bytes(int32_t waves_per_simd) {
  int dev = 0, cus = 0;
  if (waves_per_simd < 1 || waves_per_simd > 8 || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  return sizeof(uint32_t) * 256 * (size_t)cus * (size_t)waves_per_simd;
}

qsgs_status qsgs_alu_rate(int32_t waves_per_simd, void* d_scratch, size_t scratch_bytes,
                          double* lane_ops_per_s, void* stream) {
  last_error().clear();
  if (!d_scratch || !lane_ops_per_s) return fail(QSGS_ERR_INVALID, "NULL pointer argument");
  const size_t need = qsgs_alu_scratch_bytes(waves_per_simd);
  if (need == 0) return fail(QSGS_ERR_INVALID, "waves_per_simd must be in [1, 8]");
  if (scratch_bytes < need)
    return fail(QSGS_ERR_WORKSPACE, "scratch needs %zu bytes, got %zu", need, scratch_bytes);
  const uint32_t blocks = (uint32_t)(need / (sizeof(uint32_t) * 256));  // 4 waves each
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QSGS_HIP(hipEventCreate(&e0));
  QSGS_HIP(hipEventCreate(&e1));
  float best = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    QSGS_HIP(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_alu_rate, dim3(blocks), dim3(256), 0, s, (uint32_t*)d_scratch, 7u);
    QSGS_LAUNCHED("k_alu_rate");
    QSGS_HIP(hipEventRecord(e1, s));
    QSGS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QSGS_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0 && (best == 0.f || ms < best)) best = ms;  // the first run warms up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *lane_ops_per_s = (double)blocks * 256.0 * 16.0 * kAluIters / (best * 1e-3);
  return QSGS_OK;
}

}  // extern "C"
