// qsgs_measure.hip -- the occupancy one growth step reads, for the algorithmic byte count
// of a step (C ABI qsgs_band_sizes in include/qsgs.h).  A step tests the 26 neighbours
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

}  // extern "C"
