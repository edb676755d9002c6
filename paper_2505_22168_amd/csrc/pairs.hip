// Pair stages of the GMNN energy/force path (gfx950, wave64).
//
//   pair_moments   Section 2.1, eq. basis_fn: per-pair geometry, equidistant
//                  Gaussians times a cosine cutoff mixed by the species-pair
//                  coefficients beta, and the moment sums
//                  Psi_{i,L,s} = c sum_j R_s(r_ij) rhat^{(x)L}, L <= 3, stored
//                  as 20 packed symmetric components per channel.
//   pair_backward  Section 3.3 (forces as gradients): given dE/dPsi (packed),
//                  the derivative of E_i w.r.t. every pair vector d_p and the
//                  per-atom virial sum_p g_p (x) d_p; pair_backward_heads does
//                  it for every head of a shallow ensemble at once (Section
//                  2.2, force variance).
//   finish         F_k = sum_{q in row k} (g_q - g_rev(q)) (scatter-free: every
//                  force is one gather over the reverse pair index), and in
//                  extra blocks of the same grid the per-structure energies
//                  and virials (Section 2.1, eq. energy_sum) summed in FP64
//                  in a fixed order.
//
// Each atom row is processed by LPA lanes (8, 16, 32 or 64: eight, four, two or
// one atom per wave, chosen by the execution plan); the 100 moment accumulators of a lane are
// combined by a reduce-scatter (permlane swaps and DPP, no LDS, no atomics).
// pair_moments and pair_backward take the row's pairs inside r_c only, queued
// per lane group in LDS (the list's skin pairs do not occupy lanes).
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
  __shared__ float4 s_ring[kRingBatches * kPairBlock];  // per LPA-lane group: kRingBatches LPA queued pairs
  float v[128];
#pragma unroll
  for (int k = 0; k < 128; ++k) v[k] = 0.0f;
  if (live) {
    AtomCtx c;
    load_atom(sys, i, c);
    atom_moments_compact<LPA>(m, sys, s_beta, c, q, s_ring + (threadIdx.x / LPA) * kRingBatches * LPA, v);
  }
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
// one head (the head-mean backward): psibar [N][100] -> gpair [P][3] and
// the per-atom virial
template <int LPA>
__global__ void __launch_bounds__(kPairBlock) pair_backward(DevModel m, DevSystem sys, const float* __restrict__ psibar,
                                                            float* __restrict__ gpair, float* __restrict__ virial) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (LPA - 1);
  const int i = xcd_block(blockIdx.x, gridDim.x) * (kPairBlock / LPA) + threadIdx.x / LPA;
  const bool live = i < sys.n_atoms;
  __shared__ float4 s_ring[kRingBatches * kPairBlock];  // per LPA-lane group: kRingBatches LPA queued pairs
  float vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0f;
  if (live) {
    float pb[kS * kPacked];
    const float* src = psibar + (int64_t)i * (kS * kPacked);
#pragma unroll
    for (int k = 0; k < kS * kPacked; ++k) pb[k] = src[k];
    AtomCtx c;
    load_atom(sys, i, c);
    atom_pair_backward_compact<LPA>(m, sys, s_beta, c, q, pb, s_ring + (threadIdx.x / LPA) * kRingBatches * LPA, gpair, vir);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = atom_sum<LPA>(vir[k]);
  if (live && q == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) virial[(int64_t)i * 9 + k] = vir[k];
  }
}

// ---------------------------------------------------------------------------
// One backward per head (nh > 1): 64 lanes per atom, 4 atoms per block; the
// block's dE/dPsi of every head are staged in LDS after beta, and each pair's
// geometry and radial basis serve all heads.  Dynamic LDS: beta +
// 4 * nh * 100 floats.
// head_c (may be null): per-structure head weights [B][kMaxHeads] of the
// virial (an uncertainty bias); null: the mean over heads
__global__ void __launch_bounds__(kPairBlock) pair_backward_heads(DevModel m, DevSystem sys,
                                                                  const float* __restrict__ psibar,
                                                                  float* __restrict__ gpair,
                                                                  float* __restrict__ virial, int nh,
                                                                  int64_t gstride, const float* __restrict__ head_c) {
  extern __shared__ float s_beta[];
  const int nbeta = m.n_species * m.n_species * kS * kMaxBasis;
  float* s_pb = s_beta + nbeta;  // [atom][head][100]
  const int a0 = xcd_block(blockIdx.x, gridDim.x) * kHeadsAtoms;
  stage_beta(m, s_beta);
  constexpr int NP = kS * kPacked;
  for (int t = threadIdx.x; t < kHeadsAtoms * nh * NP; t += kPairBlock) {
    const int a = t / (nh * NP), rest = t % (nh * NP);
    const int h = rest / NP, k = rest % NP;
    s_pb[t] = (a0 + a < sys.n_atoms) ? psibar[((int64_t)h * sys.n_atoms + a0 + a) * NP + k] : 0.0f;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, q = threadIdx.x & 63;
  const int i = a0 + w;
  const bool live = i < sys.n_atoms;
  float vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0f;
  const float* hw = (head_c && live) ? head_c + (int64_t)sys.atom_struct[i] * kMaxHeads : nullptr;
  if (live) atom_pair_backward_heads<64>(m, sys, s_beta, i, q, s_pb + w * nh * NP, nh, gpair, gstride, vir, hw);
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = atom_sum<64>(vir[k]);
  if (live && q == 0) {
    const float inv = head_c ? 1.0f : 1.0f / (float)nh;
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
// float4 q of x (elements 4q .. 4q+3) with the elements outside [e0, e1)
// read as zero; the float4 that ends past the array (end elements), or any
// float4 of an array that is not 16-byte aligned, is read element by element
__device__ inline float4 load4_range(const float* __restrict__ x, int64_t q, int64_t e0, int64_t e1, int64_t end,
                                     bool on, bool aligned) {
  const int64_t i = 4 * q;
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (!on || i + 4 <= e0 || i >= e1) return v;
  if (aligned && i + 4 <= end) {
    v = *(const float4*)(x + i);
  } else {
    if (i < end) v.x = x[i];
    if (i + 1 < end) v.y = x[i + 1];
    if (i + 2 < end) v.z = x[i + 2];
    if (i + 3 < end) v.w = x[i + 3];
  }
  if (i < e0 || i + 4 > e1) {
    v.x = (i >= e0 && i < e1) ? v.x : 0.0f;
    v.y = (i + 1 >= e0 && i + 1 < e1) ? v.y : 0.0f;
    v.z = (i + 2 >= e0 && i + 2 < e1) ? v.z : 0.0f;
    v.w = (i + 3 >= e0 && i + 3 < e1) ? v.w : 0.0f;
  }
  return v;
}

// Per-structure sums of atom rows [a0, a1): vals[h] = sum of the atomic
// energies of head h < M, vals[kMaxHeads + k] = sum of the virial entries k
// (want_stress), other entries 0.  All threads of the block take part.
//
// From per-atom values: the energies ([n][M]) and virials ([n][9]) are two
// flat runs of floats read as float4; thread t takes every T-th float4 from
// t on, T a multiple of the column count C, so each of its four components
// always falls in the same column, and issues its loads of both runs
// kVec at a time before adding; the 4T partials of a run then meet in a
// fixed-order tree in LDS (fan-in kFan per level).
__device__ inline void structure_sums_atoms(int M, int want_stress, int64_t a0, int64_t a1, int n_atoms,
                                            const float* __restrict__ atomic_e, const float* __restrict__ virial,
                                            double* vals) {
  constexpr int kVec = 4, kFan = 8, kLvl = 4 * kPairBlock / kFan + kMaxHeads;
  __shared__ double lvl0[2][4 * kPairBlock];
  __shared__ double lvl[2][2][kLvl];
  const int t = threadIdx.x;
  const int CE = M, CV = 9;
  const int TE = (kPairBlock / CE) * CE, TV = (kPairBlock / CV) * CV;
  const int64_t e0 = a0 * CE, e1 = a1 * CE, v0 = a0 * CV, v1 = want_stress ? a1 * CV : v0;
  const int64_t qe = e0 >> 2, qv = v0 >> 2;
  const int64_t endE = (int64_t)n_atoms * CE, endV = (int64_t)n_atoms * CV;
  const bool alE = ((uintptr_t)atomic_e & 15) == 0, alV = ((uintptr_t)virial & 15) == 0;
  double sE[4] = {0.0, 0.0, 0.0, 0.0}, sV[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; 4 * (qe + k0 * TE) < e1 || 4 * (qv + k0 * TV) < v1; k0 += kVec) {
    float4 xe[kVec], xv[kVec];
#pragma unroll
    for (int u = 0; u < kVec; ++u) {
      xe[u] = load4_range(atomic_e, qe + t + (k0 + u) * TE, e0, e1, endE, t < TE, alE);
      xv[u] = load4_range(virial, qv + t + (k0 + u) * TV, v0, v1, endV, t < TV, alV);
    }
#pragma unroll
    for (int u = 0; u < kVec; ++u) {
      sE[0] += (double)xe[u].x; sE[1] += (double)xe[u].y; sE[2] += (double)xe[u].z; sE[3] += (double)xe[u].w;
      sV[0] += (double)xv[u].x; sV[1] += (double)xv[u].y; sV[2] += (double)xv[u].z; sV[3] += (double)xv[u].w;
    }
  }
  // partial idx = 4t + c4 sums elements of column (4 q + idx) % C: the rows
  // j = idx / C of a [4T / C][C] table whose column r is (4 q + r) % C
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
    lvl0[0][4 * t + c4] = sE[c4];
    lvl0[1][4 * t + c4] = sV[c4];
  }
  int rowsE = 4 * TE / CE, rowsV = 4 * TV / CV, cur = -1;
  while (rowsE > 1 || rowsV > 1) {  // uniform
    __syncthreads();
    const double* inE = cur < 0 ? lvl0[0] : lvl[cur][0];
    const double* inV = cur < 0 ? lvl0[1] : lvl[cur][1];
    const int nx = cur < 0 ? 0 : cur ^ 1;
    const int nE = (rowsE + kFan - 1) / kFan, nV = (rowsV + kFan - 1) / kFan;
    if (t < nE * CE) {
      const int g = t / CE, r = t % CE;
      double x = 0.0;
      for (int j = g * kFan; j < min(rowsE, g * kFan + kFan); ++j) x += inE[j * CE + r];
      lvl[nx][0][g * CE + r] = x;
    }
    if (t < nV * CV) {
      const int g = t / CV, r = t % CV;
      double x = 0.0;
      for (int j = g * kFan; j < min(rowsV, g * kFan + kFan); ++j) x += inV[j * CV + r];
      lvl[nx][1][g * CV + r] = x;
    }
    rowsE = nE;
    rowsV = nV;
    cur = nx;
  }
  __syncthreads();
  if (t < kMaxHeads + 9) {
    const double* outE = cur < 0 ? lvl0[0] : lvl[cur][0];
    const double* outV = cur < 0 ? lvl0[1] : lvl[cur][1];
    double x = 0.0;
    if (t < CE) x = outE[((t - (int)((4 * qe) % CE)) % CE + CE) % CE];
    else if (t >= kMaxHeads && want_stress) x = outV[((t - kMaxHeads - (int)((4 * qv) % CV)) % CV + CV) % CV];
    vals[t] = x;
  }
}

// From the fused tile's records: tile k (atom rows [k TA, k TA + TA)) left
// in rec[k][kMaxHeads + 9] the FP64 sums of its atoms' energies and virials.
// Rows [a0, a1) = head rows before the first whole tile, the whole tiles,
// tail rows after the last; head and tail rows are read per atom.  Column c
// < C = M (+ 9 with stress) is summed by kG = kPairBlock / C thread groups,
// group g taking every kG-th head row, tile and tail row from g on (kVec
// record loads in flight), then the groups in order.
__device__ inline void structure_sums_tiled(int M, int want_stress, int64_t a0, int64_t a1, int TA,
                                            const float* __restrict__ atomic_e, const float* __restrict__ virial,
                                            const double* __restrict__ rec, double* vals) {
  constexpr int kVec = 8, NR = kMaxHeads + 9;
  __shared__ double grp[kPairBlock];
  const int t = threadIdx.x;
  const int C = M + (want_stress ? 9 : 0);
  const int G = kPairBlock / C;
  int64_t k0 = (a0 + TA - 1) / TA, k1 = a1 / TA;
  int64_t h1 = a1, t0 = a1;  // head rows [a0, h1), tiles [k0, k1), tail rows [t0, a1)
  if (k0 < k1) {
    h1 = k0 * TA;
    t0 = k1 * TA;
  } else {
    k0 = k1 = 0;
  }
  if (t < G * C) {
    const int c = t % C, g = t / C;
    const int rc = c < M ? c : kMaxHeads + (c - M);  // record column
    auto row_value = [&](int64_t a) -> double {
      return c < M ? (double)atomic_e[a * M + c] : (double)virial[a * 9 + (c - M)];
    };
    double x = 0.0;
    for (int64_t a = a0 + g; a < h1; a += G) x += row_value(a);
    for (int64_t k = k0 + g; k < k1; k += (int64_t)kVec * G) {
      double y[kVec];
#pragma unroll
      for (int u = 0; u < kVec; ++u) {
        const int64_t kk = k + (int64_t)u * G;
        y[u] = kk < k1 ? rec[kk * NR + rc] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kVec; ++u) x += y[u];
    }
    for (int64_t a = t0 + g; a < a1; a += G) x += row_value(a);
    grp[g * C + c] = x;
  }
  __syncthreads();
  if (t < kMaxHeads + 9) {
    const int c = t < kMaxHeads ? t : (want_stress ? M + (t - kMaxHeads) : C);
    double x = 0.0;
    if ((t < kMaxHeads && t < M) || (t >= kMaxHeads && want_stress))
      for (int g = 0; g < G; ++g) x += grp[g * C + c];
    vals[t] = x;
  }
}

template <int LPA, bool VAR>
__global__ void __launch_bounds__(kPairBlock) finish(int M, DevSystem sys, const float* __restrict__ gpair,
                                                     const float* __restrict__ atomic_e,
                                                     const float* __restrict__ virial, int want_stress, int nb_gather,
                                                     int64_t gstride, int nchunk, double* __restrict__ partial,
                                                     int* __restrict__ counters, float* __restrict__ forces,
                                                     float* __restrict__ force_var, double* __restrict__ energy,
                                                     double* __restrict__ energy_var,
                                                     double* __restrict__ energy_mean, double* __restrict__ stress,
                                                     const double* __restrict__ tile_part, int tile_atoms,
                                                     const float* __restrict__ head_c,
                                                     float* __restrict__ forces_heads) {
  const int n_red = (int)gridDim.x - nb_gather;
  if ((int)blockIdx.x >= n_red) {
    const int q = threadIdx.x & (LPA - 1);
    const int i = xcd_block((int)blockIdx.x - n_red, nb_gather) * (kPairBlock / LPA) + threadIdx.x / LPA;
    const bool live = i < sys.n_atoms;
    if (!VAR) {
      float f[3] = {0.0f, 0.0f, 0.0f};
      if (live) {
        const int64_t p0 = sys.row_ptr[i], p1 = sys.row_ptr[i + 1];
        int64_t p = p0 + q;
        // four of the lane's pairs per pass: every index and gradient load
        // of the pass is issued before the first sum, and the sums run in
        // the pairs' order (the same result as one pair per pass)
        constexpr int U = 4;
        for (; p + (U - 1) * LPA < p1; p += U * LPA) {
          int64_t rp[U];
#pragma unroll
          for (int u = 0; u < U; ++u) rp[u] = sys.rev[p + u * LPA];
          float d[U][3];
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) d[u][k] = gpair[3 * (p + u * LPA) + k] - gpair[3 * rp[u] + k];
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) f[k] += d[u][k];
        }
        for (; p < p1; p += LPA) {
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
        if (sys.status && !(fabsf(f[0]) + fabsf(f[1]) + fabsf(f[2]) <= 3.402823466e38f))
          raise_flag(sys.status, GMNN_FLAG_NONFINITE);
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
      // with an uncertainty bias the force weights the heads by c_h of the
      // atom's structure (sum_h c_h F^h); the variance stays that of F^h
      float fo[3] = {mean[0], mean[1], mean[2]};
      if (head_c && live) {
        const float* c = head_c + (int64_t)sys.atom_struct[i] * kMaxHeads;
        fo[0] = fo[1] = fo[2] = 0.0f;
#pragma unroll
        for (int h = 0; h < kMaxHeads; ++h)
          if (h < M)
#pragma unroll
            for (int k = 0; k < 3; ++k) fo[k] += c[h] * f[h][k];
      }
      if (live && q == 0) {
        forces[3 * (int64_t)i] = fo[0];
        forces[3 * (int64_t)i + 1] = fo[1];
        forces[3 * (int64_t)i + 2] = fo[2];
        force_var[i] = var * invM;
        if (forces_heads) {
#pragma unroll
          for (int h = 0; h < kMaxHeads; ++h)
            if (h < M)
#pragma unroll
              for (int k = 0; k < 3; ++k) forces_heads[((int64_t)h * sys.n_atoms + i) * 3 + k] = f[h][k];
        }
        if (sys.status && !(fabsf(fo[0]) + fabsf(fo[1]) + fabsf(fo[2]) + var <= 3.402823466e38f))
          raise_flag(sys.status, GMNN_FLAG_NONFINITE);
      }
    }
    return;
  }
  // ---- per-structure FP64 sums: structure b = rb / nchunk, atom chunk
  // rb % nchunk; with nchunk > 1 the chunk partials go to `partial` and the
  // last chunk block of the structure (arrival counter) adds them in chunk
  // order, so the result does not depend on block scheduling.  Every sum
  // below has a fixed order.
  constexpr int NV = kMaxHeads + 9;
  __shared__ double vals[NV];
  __shared__ int last;
  const int rb = blockIdx.x;
  const int b = rb / nchunk, chunk = rb % nchunk;
  const int64_t s0 = sys.atom_ptr[b], s1 = sys.atom_ptr[b + 1];
  const int64_t csz = (s1 - s0 + nchunk - 1) / nchunk;
  const int64_t a0 = s0 + chunk * csz;
  const int64_t a1 = max(a0, min(s1, a0 + csz));
  // the cell (for the stress) is read now, its latency hidden by the sums
  double cell_det = 1.0;
  if (want_stress && threadIdx.x < 9) {
    const double* h = sys.cell + 9 * (int64_t)b;
    cell_det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
               h[2] * (h[3] * h[7] - h[4] * h[6]);
  }
  const int t = threadIdx.x;
  if (tile_part) {
    structure_sums_tiled(M, want_stress, a0, a1, tile_atoms, atomic_e, virial, tile_part, vals);
  } else {
    structure_sums_atoms(M, want_stress, a0, a1, sys.n_atoms, atomic_e, virial, vals);
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
  if (threadIdx.x < M) {
    const double e = vals[threadIdx.x];
    energy[(int64_t)b * M + threadIdx.x] = e;
    if (sys.status && !(fabs(e) <= 1.7976931348623157e308)) raise_flag(sys.status, GMNN_FLAG_NONFINITE);
  }
  if (want_stress && threadIdx.x < 9) stress[(int64_t)b * 9 + threadIdx.x] = vals[kMaxHeads + threadIdx.x] / fabs(cell_det);
  if ((energy_var || energy_mean) && threadIdx.x == 0) {
    // head mean and population variance (1/M), heads in order
    double mean = 0.0;
    for (int v = 0; v < M; ++v) mean += vals[v];
    mean /= (double)M;
    if (energy_mean) energy_mean[b] = mean;
    if (energy_var) {
      double var = 0.0;
      for (int v = 0; v < M; ++v) var += (vals[v] - mean) * (vals[v] - mean);
      energy_var[b] = var / (double)M;
    }
  }
}

template __global__ void pair_moments<8>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<16>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<32>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_moments<64>(DevModel, DevSystem, float*, int*, int);
template __global__ void pair_backward<8>(DevModel, DevSystem, const float*, float*, float*);
template __global__ void pair_backward<16>(DevModel, DevSystem, const float*, float*, float*);
template __global__ void pair_backward<32>(DevModel, DevSystem, const float*, float*, float*);
template __global__ void pair_backward<64>(DevModel, DevSystem, const float*, float*, float*);
#define FIN(LPA, VAR)                                                                                         \
  template __global__ void finish<LPA, VAR>(int, DevSystem, const float*, const float*, const float*, int, int, \
                                            int64_t, int, double*, int*, float*, float*, double*, double*, double*, \
                                            double*, const double*, int, const float*, float*);
FIN(8, false) FIN(16, false) FIN(32, false) FIN(64, false) FIN(8, true) FIN(16, true) FIN(32, true) FIN(64, true)
#undef FIN

}  // namespace gmnn
