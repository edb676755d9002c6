// Pair stages of the GMNN energy/force path (gfx950, wave64).
//
//   pair_moments   Section 2.1, eq. basis_fn: per-pair geometry, equidistant
//                  Gaussians times a cosine cutoff mixed by the species-pair
//                  coefficients beta, and the moment sums
//                  Psi_{i,L,s} = c sum_j R_s(r_ij) rhat^{(x)L}, L <= 3, stored
//                  as 20 packed symmetric components per channel.
//   pair_backward  Section 3.3 (forces as gradients): given dE/dPsi (packed),
//                  the derivative of E_i w.r.t. every pair vector d_p and the
//                  per-atom virial sum_p g_p (x) d_p.
//   finish         F_k = sum_{q in row k} (g_q - g_rev(q)) (scatter-free: every
//                  force is one gather over the reverse pair index), and in
//                  extra blocks of the same grid the per-structure energies
//                  and virials (Section 2.1, eq. energy_sum) summed in FP64
//                  in a fixed order.
//
// Each atom row is processed by LPA lanes (8, 16, 32 or 64: eight, four, two or
// one atom per wave, chosen by the execution plan); the 100 moment accumulators of a lane are
// combined by a reduce-scatter (permlane swaps and DPP, no LDS, no atomics).
#include "common.h"
#include "model.h"
#include "pair_math.h"

namespace gmnn {



// ---------------------------------------------------------------------------
// also zeroes the n_counters arrival counters of the chunked reductions in
// finish (which runs later on the same stream)
template <int LPA>
__global__ void __launch_bounds__(kPairBlock) pair_moments(DevModel m, DevSystem sys, float* __restrict__ psi,
                                                           int* __restrict__ counters, int n_counters) {
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < n_counters; t += kPairBlock) counters[t] = 0;
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (LPA - 1);
  const int i = xcd_block(blockIdx.x, gridDim.x) * (kPairBlock / LPA) + threadIdx.x / LPA;
  const bool live = i < sys.n_atoms;
  float v[128];
#pragma unroll
  for (int k = 0; k < 128; ++k) v[k] = 0.0f;
  if (live) atom_moments<LPA>(m, sys, s_beta, i, q, v);
  reduce_scatter_128<LPA>(v, q);
  constexpr int OWN = 128 / LPA;
  if (live) {
#pragma unroll
    for (int e = 0; e < OWN; ++e) {
      const int idx = OWN * q + e;
      if (idx < kS * kPacked) psi[(int64_t)i * (kS * kPacked) + idx] = v[e];
    }
  }
}

// ---------------------------------------------------------------------------
// nh heads (one backward each, e.g. for the force variance): psibar
// [nh][N][100] -> gpair [nh][gstride][3]; the virial written is the mean
// over the heads
template <int LPA>
__global__ void __launch_bounds__(kPairBlock) pair_backward(DevModel m, DevSystem sys, const float* __restrict__ psibar,
                                                            float* __restrict__ gpair, float* __restrict__ virial,
                                                            int nh, int64_t gstride) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (LPA - 1);
  const int i = xcd_block(blockIdx.x, gridDim.x) * (kPairBlock / LPA) + threadIdx.x / LPA;
  const bool live = i < sys.n_atoms;
  float vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0f;
  if (live) {
    for (int hm = 0; hm < nh; ++hm) {
      float pb[kS * kPacked];
      const float* src = psibar + ((int64_t)hm * sys.n_atoms + i) * (kS * kPacked);
#pragma unroll
      for (int k = 0; k < kS * kPacked; ++k) pb[k] = src[k];
      atom_pair_backward<LPA>(m, sys, s_beta, i, q, pb, gpair + (int64_t)hm * gstride * 3, vir);
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = atom_sum<LPA>(vir[k]);
  if (live && q == 0) {
    const float inv = 1.0f / (float)nh;
#pragma unroll
    for (int k = 0; k < 9; ++k) virial[(int64_t)i * 9 + k] = vir[k] * inv;
  }
}

// ---------------------------------------------------------------------------
// blocks [0, B*nchunk): FP64 sums per structure, fixed order (first in the
// grid, so they start at once and overlap the gather);
// the last nb_gather blocks: force gather, LPA lanes per atom; with VAR, gpair
// holds one gradient set per head ([M][gstride][3]) and the kernel writes the
// mean force and the per-atom force variance (1/M) sum_m |F^m - Fbar|^2
template <int LPA, bool VAR>
__global__ void __launch_bounds__(kPairBlock) finish(int M, DevSystem sys, const float* __restrict__ gpair,
                                                     const float* __restrict__ atomic_e,
                                                     const float* __restrict__ virial, int want_stress, int nb_gather,
                                                     int64_t gstride, int nchunk, double* __restrict__ partial,
                                                     int* __restrict__ counters, float* __restrict__ forces,
                                                     float* __restrict__ force_var, double* __restrict__ energy,
                                                     double* __restrict__ energy_var, double* __restrict__ stress) {
  const int n_red = (int)gridDim.x - nb_gather;
  if ((int)blockIdx.x >= n_red) {
    const int q = threadIdx.x & (LPA - 1);
    const int i = xcd_block((int)blockIdx.x - n_red, nb_gather) * (kPairBlock / LPA) + threadIdx.x / LPA;
    const bool live = i < sys.n_atoms;
    if (!VAR) {
      float f[3] = {0.0f, 0.0f, 0.0f};
      if (live) {
        const int64_t p0 = sys.row_ptr[i], p1 = sys.row_ptr[i + 1];
        for (int64_t p = p0 + q; p < p1; p += LPA) {
          const int64_t rp = sys.rev[p];
          f[0] += gpair[3 * p] - gpair[3 * rp];
          f[1] += gpair[3 * p + 1] - gpair[3 * rp + 1];
          f[2] += gpair[3 * p + 2] - gpair[3 * rp + 2];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) f[k] = atom_sum<LPA>(f[k]);
      if (live && q == 0) {
        forces[3 * (int64_t)i] = f[0];
        forces[3 * (int64_t)i + 1] = f[1];
        forces[3 * (int64_t)i + 2] = f[2];
      }
    } else {
      float f[kMaxHeads][3];
#pragma unroll
      for (int h = 0; h < kMaxHeads; ++h) f[h][0] = f[h][1] = f[h][2] = 0.0f;
      if (live) {
        const int64_t p0 = sys.row_ptr[i], p1 = sys.row_ptr[i + 1];
        for (int64_t p = p0 + q; p < p1; p += LPA) {
          const int64_t rp = sys.rev[p];
#pragma unroll
          for (int h = 0; h < kMaxHeads; ++h) {
            if (h < M) {
              const float* g = gpair + (int64_t)h * gstride * 3;
              f[h][0] += g[3 * p] - g[3 * rp];
              f[h][1] += g[3 * p + 1] - g[3 * rp + 1];
              f[h][2] += g[3 * p + 2] - g[3 * rp + 2];
            }
          }
        }
      }
      float mean[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int h = 0; h < kMaxHeads; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          f[h][k] = atom_sum<LPA>(f[h][k]);
          if (h < M) mean[k] += f[h][k];
        }
      const float invM = 1.0f / (float)M;
#pragma unroll
      for (int k = 0; k < 3; ++k) mean[k] *= invM;
      float var = 0.0f;
#pragma unroll
      for (int h = 0; h < kMaxHeads; ++h)
        if (h < M)
#pragma unroll
          for (int k = 0; k < 3; ++k) var += (f[h][k] - mean[k]) * (f[h][k] - mean[k]);
      if (live && q == 0) {
        forces[3 * (int64_t)i] = mean[0];
        forces[3 * (int64_t)i + 1] = mean[1];
        forces[3 * (int64_t)i + 2] = mean[2];
        force_var[i] = var * invM;
      }
    }
    return;
  }
  // ---- per-structure FP64 sums: structure b = rb / nchunk, atom chunk
  // rb % nchunk; with nchunk > 1 the chunk partials go to `partial` and the
  // last chunk block of the structure (arrival counter) adds them in chunk
  // order, so the result does not depend on block scheduling
  constexpr int NW = kPairBlock / 64;
  constexpr int NV = kMaxHeads + 9;
  __shared__ double part[NW][NV];
  __shared__ double vals[NV];
  __shared__ int last;
  const int rb = blockIdx.x;
  const int b = rb / nchunk, chunk = rb % nchunk;
  const int64_t s0 = sys.atom_ptr[b], s1 = sys.atom_ptr[b + 1];
  const int64_t csz = (s1 - s0 + nchunk - 1) / nchunk;
  const int64_t a0 = s0 + chunk * csz;
  const int64_t a1 = min(s1, a0 + csz);
  // the cell (for the stress) is read now, its latency hidden by the sums
  double cell_det = 1.0;
  if (want_stress && threadIdx.x < 9) {
    const double* h = sys.cell + 9 * (int64_t)b;
    cell_det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
               h[2] * (h[3] * h[7] - h[4] * h[6]);
  }
  double accE[kMaxHeads], accV[9];
#pragma unroll
  for (int v = 0; v < kMaxHeads; ++v) accE[v] = 0.0;
#pragma unroll
  for (int v = 0; v < 9; ++v) accV[v] = 0.0;
#pragma unroll 4
  for (int64_t a = a0 + threadIdx.x; a < a1; a += kPairBlock) {
#pragma unroll
    for (int v = 0; v < kMaxHeads; ++v)
      if (v < M) accE[v] += (double)atomic_e[a * M + v];
    if (want_stress) {
#pragma unroll
      for (int v = 0; v < 9; ++v) accV[v] += (double)virial[a * 9 + v];
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < kMaxHeads ? v >= M : !want_stress) continue;  // uniform: unused heads / no stress
    double x = v < kMaxHeads ? accE[v] : accV[v - kMaxHeads];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (l == 0) part[w][v] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double x = 0.0;
    const int v = threadIdx.x;
    if (v < kMaxHeads ? v < M : want_stress != 0)
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) x += part[ww][v];
    vals[v] = x;
  }
  if (nchunk > 1) {
    __syncthreads();
    if (threadIdx.x < NV) partial[((int64_t)b * nchunk + chunk) * NV + threadIdx.x] = vals[threadIdx.x];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&counters[b], 1) == nchunk - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x < NV) {
      double x = 0.0;
      for (int c = 0; c < nchunk; ++c) x += __builtin_nontemporal_load(&partial[((int64_t)b * nchunk + c) * NV + threadIdx.x]);
      vals[threadIdx.x] = x;
    }
    if (threadIdx.x == 0) counters[b] = 0;  // ready for the next evaluation
  }
  __syncthreads();
  if (threadIdx.x < M) energy[(int64_t)b * M + threadIdx.x] = vals[threadIdx.x];
  if (want_stress && threadIdx.x < 9) stress[(int64_t)b * 9 + threadIdx.x] = vals[kMaxHeads + threadIdx.x] / fabs(cell_det);
  if (energy_var && threadIdx.x == 0) {
    double mean = 0.0;
    for (int v = 0; v < M; ++v) mean += vals[v];
    mean /= (double)M;
    double var = 0.0;
    for (int v = 0; v < M; ++v) var += (vals[v] - mean) * (vals[v] - mean);
    energy_var[b] = var / (double)M;
  }
}

template __global__ void pair_moments<8>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<16>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<32>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<64>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_backward<8>(DevModel, DevSystem, const float*, float*, float*, int, int64_t);
template __global__ void pair_backward<16>(DevModel, DevSystem, const float*, float*, float*, int, int64_t);
template __global__ void pair_backward<32>(DevModel, DevSystem, const float*, float*, float*, int, int64_t);
template __global__ void pair_backward<64>(DevModel, DevSystem, const float*, float*, float*, int, int64_t);
#define FIN(LPA, VAR)                                                                                         \
  template __global__ void finish<LPA, VAR>(int, DevSystem, const float*, const float*, const float*, int, int, \
                                            int64_t, int, double*, int*, float*, float*, double*, double*, double*);
FIN(8, false) FIN(16, false) FIN(32, false) FIN(64, false) FIN(8, true) FIN(16, true) FIN(32, true) FIN(64, true)
#undef FIN

}  // namespace gmnn
