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
//   force_gather   F_k = sum_{q in row k} (g_q - g_rev(q)): scatter-free,
//                  every force is one gather over the reverse pair index.
//   struct_reduce  Section 2.1, eq. energy_sum: per-structure energies and
//                  virials summed in FP64 in a fixed order.
//
// Each atom row is processed by a group of 16 lanes (4 atoms per wave); the
// 100 moment accumulators of a lane are combined with a 4-step DPP
// reduce-scatter (no LDS, no atomics), after which lane q of the group owns
// components 8q .. 8q+7.
#include "common.h"
#include "model.h"

namespace gmnn {

constexpr int kLPA = 16;                 // lanes per atom
constexpr int kPairBlock = 256;          // threads per block
constexpr int kAtomsPerBlock = kPairBlock / kLPA;

// --- DPP lane exchanges inside rows of 16 lanes ----------------------------
__device__ inline float dpp_mirror(float v) {  // lane 15 - l
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xf, 0xf, false));
}
__device__ inline float dpp_half_mirror(float v) {  // lane 7 - l inside each half row
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xf, 0xf, false));
}
__device__ inline float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xf, 0xf, false));
}
__device__ inline float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}
// sum over the 16 lanes of a row (every lane gets the total)
__device__ inline float row16_sum(float v) {
  v += dpp_mirror(v);
  v += dpp_half_mirror(v);
  v += dpp_xor2(v);
  v += dpp_xor1(v);
  return v;
}

// one reduce-scatter step: keep half H of the live values, send the other
template <int H, int STEP>
__device__ inline void rs_step(float* v, int bit) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float lo = v[k], hi = v[k + H];
    const float send = bit ? lo : hi;
    const float keep = bit ? hi : lo;
    float got;
    if (STEP == 0) got = dpp_mirror(send);
    else if (STEP == 1) got = dpp_half_mirror(send);
    else if (STEP == 2) got = dpp_xor2(send);
    else got = dpp_xor1(send);
    v[k] = keep + got;
  }
}

// 128 values (100 live + 28 zero) per lane -> 8 summed values per lane,
// lane q of the 16-lane row owns indices 8q..8q+7
__device__ inline void reduce_scatter_128(float* v, int q) {
  rs_step<64, 0>(v, (q >> 3) & 1);
  rs_step<32, 1>(v, (q >> 2) & 1);
  rs_step<16, 2>(v, (q >> 1) & 1);
  rs_step<8, 3>(v, q & 1);
}

// --- radial basis ------------------------------------------------------------
struct Radial {
  float R[kS];    // c * f_c(r) * sum_k beta[s][k] g_k(r)
  float dR[kS];   // d R_s / dr
};

// Gaussians g_k = exp(-gamma (r - mu_k)^2), mu_k = r_min + k delta, by the
// recurrence g_k = g_0 a^k exp(-gamma delta^2 k^2) with a = exp(2 gamma delta tau)
template <bool DERIV>
__device__ inline void radial(const DevModel& m, const float* __restrict__ bz /*[S][8]*/, float r, Radial& out) {
  const float tau = r - m.r_min;
  const float g0 = expf(-m.gamma * tau * tau);
  const float a = expf(2.0f * m.gamma * m.delta * tau);
  const float gd2 = m.gamma * m.delta * m.delta;
  float g[kMaxBasis];
  float p = g0;
#pragma unroll
  for (int k = 0; k < kMaxBasis; ++k) {
    g[k] = (k < m.K) ? p * expf(-gd2 * (float)(k * k)) : 0.0f;
    p *= a;
  }
  float sn, cs;
  sincosf(3.14159265358979f * r / m.r_cut, &sn, &cs);
  const float fc = 0.5f * (cs + 1.0f) * m.psi_scale;
  const float dfc = -0.5f * (3.14159265358979f / m.r_cut) * sn * m.psi_scale;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    float B = 0.0f, dB = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxBasis; ++k) {
      const float bk = bz[s * kMaxBasis + k];
      B += bk * g[k];
      if (DERIV) dB += bk * (-2.0f * m.gamma * (tau - (float)k * m.delta)) * g[k];
    }
    out.R[s] = fc * B;
    if (DERIV) out.dR[s] = dfc * B + fc * dB;
  }
}

// monomials of u in packed order: 1, x y z, xx xy xz yy yz zz, xxx ... zzz
__device__ inline void monomials(float x, float y, float z, float* mo) {
  mo[0] = 1.0f;
  mo[1] = x; mo[2] = y; mo[3] = z;
  mo[4] = x * x; mo[5] = x * y; mo[6] = x * z; mo[7] = y * y; mo[8] = y * z; mo[9] = z * z;
  mo[10] = mo[4] * x; mo[11] = mo[4] * y; mo[12] = mo[4] * z; mo[13] = mo[7] * x; mo[14] = mo[5] * z;
  mo[15] = mo[9] * x; mo[16] = mo[7] * y; mo[17] = mo[7] * z; mo[18] = mo[9] * y; mo[19] = mo[9] * z;
}

// stage beta[zi][zj][s][k] into LDS as [zi][zj][s][8] (K padded to 8)
__device__ inline void stage_beta(const DevModel& m, float* s_beta) {
  const int n = m.n_species * m.n_species * kS * kMaxBasis;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int k = t % kMaxBasis;
    const int rest = t / kMaxBasis;  // (zi*nsp + zj)*S + s
    s_beta[t] = (k < m.K) ? m.beta[rest * m.K + k] : 0.0f;
  }
}

struct AtomCtx {
  float xi, yi, zi;
  float h[9];
  int zsp;
  int64_t p0, p1;
};

__device__ inline void load_atom(const DevSystem& sys, int i, AtomCtx& c) {
  c.xi = sys.pos[3 * (int64_t)i];
  c.yi = sys.pos[3 * (int64_t)i + 1];
  c.zi = sys.pos[3 * (int64_t)i + 2];
  const int b = sys.atom_struct[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) c.h[k] = (float)sys.cell[9 * (int64_t)b + k];
  c.zsp = sys.species[i];
  c.p0 = sys.row_ptr[i];
  c.p1 = sys.row_ptr[i + 1];
}

// d_p = x_j - x_i + S . h (FP32)
__device__ inline void pair_vec(const DevSystem& sys, const AtomCtx& c, int64_t p, int& j, float& dx, float& dy,
                                float& dz) {
  j = sys.nj[p];
  int sx, sy, sz;
  unpack_shift(sys.nshift[p], sx, sy, sz);
  const float fx = (float)sx, fy = (float)sy, fz = (float)sz;
  dx = (sys.pos[3 * (int64_t)j] - c.xi) + (fx * c.h[0] + fy * c.h[3] + fz * c.h[6]);
  dy = (sys.pos[3 * (int64_t)j + 1] - c.yi) + (fx * c.h[1] + fy * c.h[4] + fz * c.h[7]);
  dz = (sys.pos[3 * (int64_t)j + 2] - c.zi) + (fx * c.h[2] + fy * c.h[5] + fz * c.h[8]);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kPairBlock) pair_moments(DevModel m, DevSystem sys, float* __restrict__ psi) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (kLPA - 1);
  const int i = blockIdx.x * kAtomsPerBlock + threadIdx.x / kLPA;
  const bool live = i < sys.n_atoms;
  float v[128];
#pragma unroll
  for (int k = 0; k < 128; ++k) v[k] = 0.0f;
  if (live) {
    AtomCtx c;
    load_atom(sys, i, c);
    const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
    for (int64_t p = c.p0 + q; p < c.p1; p += kLPA) {
      int j;
      float dx, dy, dz;
      pair_vec(sys, c, p, j, dx, dy, dz);
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < m.rc2) || r2 == 0.0f) continue;
      const float r = sqrtf(r2);
      const float ir = 1.0f / r;
      Radial rad;
      radial<false>(m, bzi + sys.species[j] * kS * kMaxBasis, r, rad);
      float mo[20];
      monomials(dx * ir, dy * ir, dz * ir, mo);
#pragma unroll
      for (int s = 0; s < kS; ++s)
#pragma unroll
        for (int t = 0; t < kPacked; ++t) v[s * kPacked + t] += rad.R[s] * mo[t];
    }
  }
  reduce_scatter_128(v, q);
  if (live) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = 8 * q + e;
      if (idx < kS * kPacked) psi[(int64_t)i * (kS * kPacked) + idx] = v[e];
    }
  }
}

// ---------------------------------------------------------------------------
// dE/dd_p for every pair of the row of atom i, given psibar = dE_i/dPsi_i
// (packed components: the derivative w.r.t. each packed value as an
// independent variable).  With P_s(u) = sum_m psibar[s][m] mono_m(u):
//   g = sum_s dR_s P_s(u) u + (grad Q - (grad Q . u) u) / r,  Q = sum_s R_s P_s
__global__ void __launch_bounds__(kPairBlock) pair_backward(DevModel m, DevSystem sys, const float* __restrict__ psibar,
                                                            float* __restrict__ gpair, float* __restrict__ virial) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (kLPA - 1);
  const int i = blockIdx.x * kAtomsPerBlock + threadIdx.x / kLPA;
  const bool live = i < sys.n_atoms;
  float vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0f;
  if (live) {
    float pb[kS * kPacked];
#pragma unroll
    for (int k = 0; k < kS * kPacked; ++k) pb[k] = psibar[(int64_t)i * (kS * kPacked) + k];
    AtomCtx c;
    load_atom(sys, i, c);
    const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
    for (int64_t p = c.p0 + q; p < c.p1; p += kLPA) {
      int j;
      float dx, dy, dz;
      pair_vec(sys, c, p, j, dx, dy, dz);
      const float r2 = dx * dx + dy * dy + dz * dz;
      float gx = 0.0f, gy = 0.0f, gz = 0.0f;
      if (r2 < m.rc2 && r2 > 0.0f) {
        const float r = sqrtf(r2);
        const float ir = 1.0f / r;
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        Radial rad;
        radial<true>(m, bzi + sys.species[j] * kS * kMaxBasis, r, rad);
        float mo[20];
        monomials(ux, uy, uz, mo);
        float radial_part = 0.0f;
        float qc[kPacked];
#pragma unroll
        for (int t = 0; t < kPacked; ++t) qc[t] = 0.0f;
#pragma unroll
        for (int s = 0; s < kS; ++s) {
          float A = 0.0f;
#pragma unroll
          for (int t = 0; t < kPacked; ++t) {
            A += pb[s * kPacked + t] * mo[t];
            qc[t] += rad.R[s] * pb[s * kPacked + t];
          }
          radial_part += A * rad.dR[s];
        }
        // gradient of Q(u) = sum_t qc[t] mono_t(u) w.r.t. u
        const float x = ux, y = uy, z = uz;
        float Gx = qc[1] + 2.0f * qc[4] * x + qc[5] * y + qc[6] * z + 3.0f * qc[10] * x * x +
                   2.0f * qc[11] * x * y + 2.0f * qc[12] * x * z + qc[13] * y * y + qc[14] * y * z + qc[15] * z * z;
        float Gy = qc[2] + qc[5] * x + 2.0f * qc[7] * y + qc[8] * z + qc[11] * x * x + 2.0f * qc[13] * x * y +
                   qc[14] * x * z + 3.0f * qc[16] * y * y + 2.0f * qc[17] * y * z + qc[18] * z * z;
        float Gz = qc[3] + qc[6] * x + qc[8] * y + 2.0f * qc[9] * z + qc[12] * x * x + qc[14] * x * y +
                   2.0f * qc[15] * x * z + qc[17] * y * y + 2.0f * qc[18] * y * z + 3.0f * qc[19] * z * z;
        const float gu = Gx * x + Gy * y + Gz * z;
        gx = radial_part * x + (Gx - gu * x) * ir;
        gy = radial_part * y + (Gy - gu * y) * ir;
        gz = radial_part * z + (Gz - gu * z) * ir;
        vir[0] += gx * dx; vir[1] += gx * dy; vir[2] += gx * dz;
        vir[3] += gy * dx; vir[4] += gy * dy; vir[5] += gy * dz;
        vir[6] += gz * dx; vir[7] += gz * dy; vir[8] += gz * dz;
      }
      gpair[3 * p] = gx;
      gpair[3 * p + 1] = gy;
      gpair[3 * p + 2] = gz;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = row16_sum(vir[k]);
  if (live && q == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) virial[(int64_t)i * 9 + k] = vir[k];
  }
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kPairBlock) force_gather(DevSystem sys, const float* __restrict__ gpair,
                                                           float* __restrict__ forces) {
  const int q = threadIdx.x & (kLPA - 1);
  const int i = blockIdx.x * kAtomsPerBlock + threadIdx.x / kLPA;
  const bool live = i < sys.n_atoms;
  float f[3] = {0.0f, 0.0f, 0.0f};
  if (live) {
    const int64_t p0 = sys.row_ptr[i], p1 = sys.row_ptr[i + 1];
    for (int64_t p = p0 + q; p < p1; p += kLPA) {
      const int64_t rp = sys.rev[p];
      f[0] += gpair[3 * p] - gpair[3 * rp];
      f[1] += gpair[3 * p + 1] - gpair[3 * rp + 1];
      f[2] += gpair[3 * p + 2] - gpair[3 * rp + 2];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k] = row16_sum(f[k]);
  if (live && q == 0) {
    forces[3 * (int64_t)i] = f[0];
    forces[3 * (int64_t)i + 1] = f[1];
    forces[3 * (int64_t)i + 2] = f[2];
  }
}

// ---------------------------------------------------------------------------
// one block per structure; FP64 sums in a fixed order (deterministic)
constexpr int kReduceBlock = 256;
__global__ void __launch_bounds__(kReduceBlock) struct_reduce(int M, DevSystem sys, const float* __restrict__ atomic_e,
                                                              const float* __restrict__ virial, int want_stress,
                                                              double* __restrict__ energy, double* __restrict__ energy_var,
                                                              double* __restrict__ stress) {
  __shared__ double red[kReduceBlock];
  __shared__ double vals[kMaxHeads + 9];
  const int b = blockIdx.x;
  const int64_t a0 = sys.atom_ptr[b], a1 = sys.atom_ptr[b + 1];
  const int nv = M + (want_stress ? 9 : 0);
  for (int v = 0; v < nv; ++v) {
    double acc = 0.0;
    for (int64_t a = a0 + threadIdx.x; a < a1; a += kReduceBlock)
      acc += (v < M) ? (double)atomic_e[a * M + v] : (double)virial[a * 9 + (v - M)];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kReduceBlock / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) vals[v] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mean = 0.0;
    for (int v = 0; v < M; ++v) {
      energy[(int64_t)b * M + v] = vals[v];
      mean += vals[v];
    }
    mean /= (double)M;
    if (energy_var) {
      double var = 0.0;
      for (int v = 0; v < M; ++v) var += (vals[v] - mean) * (vals[v] - mean);
      energy_var[b] = var / (double)M;
    }
    if (want_stress) {
      const double* h = sys.cell + 9 * (int64_t)b;
      const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                         h[2] * (h[3] * h[7] - h[4] * h[6]);
      const double iv = 1.0 / fabs(det);
      for (int k = 0; k < 9; ++k) stress[(int64_t)b * 9 + k] = vals[M + k] * iv;
    }
  }
}

}  // namespace gmnn
