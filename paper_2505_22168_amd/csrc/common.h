// Shared device helpers of the GMNN HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/gmnn.h"

#define GMNN_WAVE 64

namespace gmnn {

// ---------------------------------------------------------------------------
// packed image vector: three int8 in the low 24 bits
// ---------------------------------------------------------------------------
__host__ __device__ inline int32_t pack_shift(int sx, int sy, int sz) {
  return (sx & 0xff) | ((sy & 0xff) << 8) | ((sz & 0xff) << 16);
}
__host__ __device__ inline void unpack_shift(int32_t p, int& sx, int& sy, int& sz) {
  sx = (int)(int8_t)(p & 0xff);
  sy = (int)(int8_t)((p >> 8) & 0xff);
  sz = (int)(int8_t)((p >> 16) & 0xff);
}
// canonical sort key of a pair inside a row: (j, Sx, Sy, Sz) ascending
__host__ __device__ inline uint64_t pair_key(int j, int sx, int sy, int sz) {
  return ((uint64_t)(uint32_t)j << 24) | ((uint64_t)(sx + 128) << 16) |
         ((uint64_t)(sy + 128) << 8) | (uint64_t)(sz + 128);
}

// ---------------------------------------------------------------------------
// XCD-aware block order.  The 8 XCDs of the chip (each with its own L2) take
// workgroups round-robin by block index; xcd_block maps the launch so that
// XCD x processes one contiguous run of logical blocks (nb split as evenly
// as possible), keeping the neighbour rows that nearby atoms share in one
// L2.  A bijection of [0, nb).
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// Dynamic-LDS limit of a kernel on the current device, raised to `bytes` the
// first time a launch needs it.  One process-wide table of (device, kernel)
// -> limit set (fixed size, no heap allocation), guarded by a mutex: safe
// from several host threads, and each device gets its own attribute call.
// ---------------------------------------------------------------------------
inline gmnn_status ensure_lds_limit(const void* kernel, size_t bytes) {
  struct Rec {
    int dev;
    const void* kernel;
    size_t bytes;
  };
  constexpr int kRecs = 512;
  static Rec recs[kRecs];
  static int n_recs = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMNN_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  int r = 0;
  while (r < n_recs && !(recs[r].dev == dev && recs[r].kernel == kernel)) ++r;
  if (r < n_recs && recs[r].bytes >= bytes) return GMNN_OK;
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    return GMNN_ERR_HIP;
  if (r < n_recs) recs[r].bytes = bytes;
  else if (n_recs < kRecs) recs[n_recs++] = Rec{dev, kernel, bytes};  // a full table only costs repeated calls
  return GMNN_OK;
}

// ---------------------------------------------------------------------------
// split-BF16 operands
// ---------------------------------------------------------------------------
// v - hi for the low bf16 part of v (hi = bf16(v)), with v taken as the
// rounded FP32 value: the empty asm keeps the compiler from fusing the
// product that produced v into the subtraction (an FMA there would give the
// low part of the unrounded product, and kernels that fuse differently would
// disagree in the last bits)
__device__ inline float split_low(float v, __bf16 hi) {
  asm("" : "+v"(v));
  return v - (float)hi;
}

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

// a block barrier that orders LDS accesses only: global loads in flight
// (operands prefetched for a later phase) stay in flight across it, where
// __syncthreads() would wait for them
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The value held by lane l ^ 32 (lane_xor32) or l ^ 16 (lane_xor16), in
// registers: a permlane swap of the value with itself hands every lane its
// partner's copy in one of the two outputs (no LDS round trip, unlike a
// shuffle).
__device__ inline float lane_xor32(float v) {
  const unsigned u = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __uint_as_float(lane_id() < 32 ? r[1] : r[0]);
}
__device__ inline float lane_xor16(float v) {
  const unsigned u = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __uint_as_float(((lane_id() >> 4) & 1) ? r[0] : r[1]);
}

// Sum over the 16 lanes of a row by DPP row rotations (8, 4, 2, 1), in
// registers.  Lane 0 of the row ends with the same value, bit for bit, as
// an xor butterfly over the row (at each level it adds the same two partial
// sums); other lanes hold other orderings of the row sum.
__device__ inline float row16_rot_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, false));  // row_ror:8
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, false));  // row_ror:4
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xf, 0xf, false));  // row_ror:2
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, false));  // row_ror:1
  return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, GMNN_WAVE);
  return v;
}

// inclusive prefix sum over the 64 lanes
__device__ inline int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, GMNN_WAVE);
    if (l >= o) v += t;
  }
  return v;
}

__device__ inline void raise_flag(uint32_t* status, uint32_t f) { atomicOr(status, f); }

// ---------------------------------------------------------------------------
// block-level exclusive scan of `n` int32 counts into int64 offsets (n+1
// entries, out[n] = total).  One block; every thread of the block calls it.
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ inline void block_exclusive_scan(const int32_t* __restrict__ in, int64_t* __restrict__ out,
                                            int64_t n, int64_t* total_out) {
  __shared__ int64_t sums[BLOCK];
  const int t = threadIdx.x;
  const int64_t chunk = (n + BLOCK - 1) / BLOCK;
  const int64_t b0 = t * chunk;
  const int64_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
  int64_t s = 0;
  for (int64_t k = b0; k < b1; ++k) s += in[k];
  sums[t] = s;
  __syncthreads();
  // Hillis-Steele over BLOCK partial sums
  for (int o = 1; o < BLOCK; o <<= 1) {
    int64_t v = (t >= o) ? sums[t - o] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int64_t run = (t == 0) ? 0 : sums[t - 1];
  for (int64_t k = b0; k < b1; ++k) {
    out[k] = run;
    run += in[k];
  }
  if (t == BLOCK - 1) {
    out[n] = sums[BLOCK - 1];
    if (total_out) *total_out = sums[BLOCK - 1];
  }
}

}  // namespace gmnn
