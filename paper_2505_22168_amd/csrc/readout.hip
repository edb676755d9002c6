// Per-tile readout of the GMNN energy/force path (gfx950, wave64, MFMA).
//
// One block of 256 threads (4 waves) owns a tile of TM atoms and runs, all in
// LDS:
//   1. expand the packed moments to full Cartesian tensors
//   2. invariants (Section 2.1, eq. contraction): the eight contraction
//      families; the 3-tensor families go through small intermediates
//      (T7 = Psi3 Psi3 over two indices, V8 = Psi3 : Psi2, M5 = Psi2 Psi2,
//      v6 = Psi2 Psi1) so each invariant is a short dot product
//   3. network (Section 2.1, eq. scale_shift): z1 = G W1 + b1, h1 = swish(z1),
//      z2 = h1 W2 + b2, h2 = swish(z2), y = h2 W3 + b3, E_i = sigma_Z y + mu_Z;
//      the two hidden products run on MFMA (16x16x32 BF16 or 16x16x4 FP32),
//      weights streamed from L2 in fragment order
//   4. backward of the head-mean energy (Section 2.2, eq. jacobian: the mean
//      force is the force of the mean energy): delta2 = swish'(z2) sigma
//      mean_m W3[:,m], delta1 = swish'(z1) (delta2 W2^T), dE/dG = delta1 W1^T
//      (two more MFMA products; swish'(z1) stays in registers because the
//      backward product hands every wave the same output fragments)
//   5. product-rule backward of the invariants to dE/dPsi, folded onto the
//      packed components
// Outputs: E_i per head and dE/dPsi (packed) for the pair backward.
#include "common.h"
#include "model.h"

namespace gmnn {

constexpr int kReadoutThreads = 256;
constexpr int PS = 201;   // atom stride (floats) of the full tensors in LDS (odd: conflict-free columns)
constexpr int IS = 225;   // atom stride of the intermediates (odd)

template <int TM, int HP, bool BF16>
struct ReadoutLds {
  static constexpr int LDA_G = BF16 ? (kFP + 8) : (kFP + 4);     // G tile row stride (elements)
  static constexpr int LDA_H = BF16 ? (HP + 8) : (HP + 4);       // h1 / delta tile row stride
  static constexpr int LDGB = kFP + 1;                           // dE/dG row stride (floats)
  static constexpr int ESZ = BF16 ? 2 : 4;
  static constexpr size_t psi = 0;
  static constexpr size_t psi_bytes = 4 * (size_t)TM * PS;
  // region A: intermediates, later delta2
  static constexpr size_t inter = psi + ((psi_bytes + 255) & ~size_t(255));
  static constexpr size_t inter_need = 4 * (size_t)TM * IS;
  static constexpr size_t d2_need = (size_t)ESZ * TM * LDA_H;
  static constexpr size_t inter_bytes = inter_need > d2_need ? inter_need : d2_need;
  // region B: G tile, later dE/dG
  static constexpr size_t g = inter + ((inter_bytes + 255) & ~size_t(255));
  static constexpr size_t g_need = (size_t)ESZ * TM * LDA_G;
  static constexpr size_t gb_need = 4 * (size_t)TM * LDGB;
  static constexpr size_t g_bytes = g_need > gb_need ? g_need : gb_need;
  // region C: h1, later delta1, later dE/dPsi (full)
  static constexpr size_t h = g + ((g_bytes + 255) & ~size_t(255));
  static constexpr size_t h_need = (size_t)ESZ * TM * LDA_H;
  static constexpr size_t pb_need = 4 * (size_t)TM * PS;
  static constexpr size_t h_bytes = h_need > pb_need ? h_need : pb_need;
  // energy partial sums [4 waves][TM][M], per-row scale
  static constexpr size_t ep = h + ((h_bytes + 255) & ~size_t(255));
  static constexpr size_t ep_bytes = 4 * 4 * (size_t)TM * kMaxHeads;
  static constexpr size_t rowsc = ep + ep_bytes;
  static constexpr size_t bytes = rowsc + 4 * 2 * (size_t)TM;
};

// --- MFMA tile products ------------------------------------------------------
template <int MB, int NBW>
__device__ inline void mma_bf16(const __bf16* __restrict__ A, int lda, const bf16x8* __restrict__ Bp, int KB, int nb0,
                                floatx4 (&acc)[MB][NBW]) {
  const int l = threadIdx.x & 63;
  const int ar = l & 15, ak = (l >> 4) * 8;
  for (int kb = 0; kb < KB; ++kb) {
    bf16x8 a[MB];
#pragma unroll
    for (int rb = 0; rb < MB; ++rb) a[rb] = *(const bf16x8*)(A + (rb * 16 + ar) * lda + kb * 32 + ak);
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      const bf16x8 b = Bp[((size_t)(nb0 + nb) * KB + kb) * 64 + l];
#pragma unroll
      for (int rb = 0; rb < MB; ++rb) acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b, acc[rb][nb], 0, 0, 0);
    }
  }
}

template <int MB, int NBW>
__device__ inline void mma_f32(const float* __restrict__ A, int lda, const float* __restrict__ Bp, int KB, int nb0,
                               floatx4 (&acc)[MB][NBW]) {
  const int l = threadIdx.x & 63;
  const int ar = l & 15, ak = l >> 4;
  for (int kb = 0; kb < KB; ++kb) {
    float a[MB];
#pragma unroll
    for (int rb = 0; rb < MB; ++rb) a[rb] = A[(rb * 16 + ar) * lda + kb * 4 + ak];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      const float b = Bp[((size_t)(nb0 + nb) * KB + kb) * 64 + l];
#pragma unroll
      for (int rb = 0; rb < MB; ++rb) acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb], b, acc[rb][nb], 0, 0, 0);
    }
  }
}

template <int MB, int NBW>
__device__ inline void zero_acc(floatx4 (&acc)[MB][NBW]) {
#pragma unroll
  for (int rb = 0; rb < MB; ++rb)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) acc[rb][nb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
}

__device__ inline float swish_parts(float z, float& dsw) {
  const float s = 1.0f / (1.0f + expf(-z));
  dsw = s * (1.0f + z * (1.0f - s));
  return z * s;
}

template <bool BF16>
__device__ inline void st_act(void* base, int idx, float v) {
  if (BF16) ((__bf16*)base)[idx] = (__bf16)v;
  else ((float*)base)[idx] = v;
}

// ---------------------------------------------------------------------------
template <int TM, int HP, bool BF16>
__global__ void __launch_bounds__(kReadoutThreads) readout(DevModel m, DevSystem sys, const float* __restrict__ psi,
                                                           float* __restrict__ atomic_e, float* __restrict__ psibar) {
  using Lds = ReadoutLds<TM, HP, BF16>;
  constexpr int MB = TM / 16;
  constexpr int NBW = HP / 64;         // 16-column blocks per wave for the hidden products
  constexpr int NBW_G = kFP / 64;      // ... for the dE/dG product (6)
  extern __shared__ __attribute__((aligned(16))) char lds[];
  float* sPsi = (float*)(lds + Lds::psi);
  float* sInter = (float*)(lds + Lds::inter);
  void* sD2 = (void*)(lds + Lds::inter);
  void* sG = (void*)(lds + Lds::g);
  float* sGb = (float*)(lds + Lds::g);
  void* sH = (void*)(lds + Lds::h);
  float* sPb = (float*)(lds + Lds::h);
  float* sEp = (float*)(lds + Lds::ep);
  float* sScale = (float*)(lds + Lds::rowsc);
  float* sShift = sScale + TM;

  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int l = tid & 63;
  const int row0 = blockIdx.x * TM;
  const int M = m.M;

  // ---- 1. load and expand the moments ------------------------------------
  for (int t = tid; t < TM * kS * kFull; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s = e / kFull, r = e % kFull;
    const int gi = row0 + a;
    float v = 0.0f;
    if (gi < sys.n_atoms) v = psi[(int64_t)gi * (kS * kPacked) + s * kPacked + c_full_to_packed[r]];
    sPsi[a * PS + e] = v;
  }
  for (int a = tid; a < TM; a += kReadoutThreads) {
    const int gi = row0 + a;
    float sc = 0.0f, sh = 0.0f;
    if (gi < sys.n_atoms) {
      const int z = sys.species[gi];
      sc = m.scale[z];
      sh = m.shift[z];
    }
    sScale[a] = sc;
    sShift[a] = sh;
  }
  __syncthreads();

#define P0(a, s) sPsi[(a) * PS + (s) * kFull]
#define P1(a, s, i) sPsi[(a) * PS + (s) * kFull + 1 + (i)]
#define P2(a, s, ij) sPsi[(a) * PS + (s) * kFull + 4 + (ij)]
#define P3(a, s, ijk) sPsi[(a) * PS + (s) * kFull + 13 + (ijk)]
  auto storeG = [&](int a, int f, float v) { st_act<BF16>(sG, a * Lds::LDA_G + f, v); };

  // ---- 2. invariants ---------------------------------------------------------
  // families 1-4 (50 features)
  for (int t = tid; t < TM * 50; t += kReadoutThreads) {
    const int a = t % TM, f = t / TM;
    float v = 0.0f;
    if (f < kFam2) {
      v = P0(a, f);
    } else if (f < kFam3) {
      const int p = f - kFam2, s1 = c_pair_s1[p], s2 = c_pair_s2[p];
#pragma unroll
      for (int i = 0; i < 3; ++i) v += P1(a, s1, i) * P1(a, s2, i);
    } else if (f < kFam4) {
      const int p = f - kFam3, s1 = c_pair_s1[p], s2 = c_pair_s2[p];
#pragma unroll
      for (int i = 0; i < 9; ++i) v += P2(a, s1, i) * P2(a, s2, i);
    } else {
      const int p = f - kFam4, s1 = c_pair_s1[p], s2 = c_pair_s2[p];
#pragma unroll
      for (int i = 0; i < 27; ++i) v += P3(a, s1, i) * P3(a, s2, i);
    }
    storeG(a, f, v);
  }
  // zero padding columns kF..kFP-1
  for (int t = tid; t < TM * (kFP - kF); t += kReadoutThreads) storeG(t % TM, kF + t / TM, 0.0f);

  // family 7: T7[p][ab] = sum_cd P3[s2]_acd P3[s3]_bcd, p = (s2 <= s3)
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, ia = (e % 9) / 3, ib = e % 3;
    const int s2 = c_pair_s1[p], s3 = c_pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int cd = 0; cd < 9; ++cd) v += P3(a, s2, ia * 9 + cd) * P3(a, s3, ib * 9 + cd);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s1 = e / 15, p = e % 15;
    float v = 0.0f;
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) v += P2(a, s1, ij) * sInter[a * IS + p * 9 + ij];
    storeG(a, kFam7 + e, v);
  }
  __syncthreads();
  // family 8: V8[s2*5+s3][i] = sum_bc P3[s2]_ibc P2[s3]_bc
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s23 = e / 3, i = e % 3;
    const int s2 = s23 / 5, s3 = s23 % 5;
    float v = 0.0f;
#pragma unroll
    for (int bc = 0; bc < 9; ++bc) v += P3(a, s2, i * 9 + bc) * P2(a, s3, bc);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 125; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s1 = e / 25, s23 = e % 25;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += P1(a, s1, i) * sInter[a * IS + s23 * 3 + i];
    storeG(a, kFam8 + e, v);
  }
  __syncthreads();
  // family 5: M5[p][ij] = (P2[s1] P2[s2])_ij, p = (s1 <= s2)
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, i = (e % 9) / 3, j = e % 3;
    const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) v += P2(a, s1, i * 3 + c) * P2(a, s2, c * 3 + j);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 35; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s1 = c_tri_s1[e], s2 = c_tri_s2[e], s3 = c_tri_s3[e];
    const int p = c_pair_index[s1][s2];
    float v = 0.0f;
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) v += sInter[a * IS + p * 9 + ij] * P2(a, s3, ij);
    storeG(a, kFam5 + e, v);
  }
  __syncthreads();
  // family 6: v6[s3*5+s1][i] = (P2[s3] P1[s1])_i
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s31 = e / 3, i = e % 3;
    const int s3 = s31 / 5, s1 = s31 % 5;
    float v = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j) v += P2(a, s3, i * 3 + j) * P1(a, s1, j);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int p = e / 5, s3 = e % 5;
    const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += sInter[a * IS + (s3 * 5 + s1) * 3 + i] * P1(a, s2, i);
    storeG(a, kFam6 + e, v);
  }
  __syncthreads();

  // ---- 3. network forward ----------------------------------------------------
  floatx4 dsw1[MB][NBW];
  {
    floatx4 acc[MB][NBW];
    zero_acc(acc);
    if (BF16) mma_bf16<MB, NBW>((const __bf16*)sG, Lds::LDA_G, m.w1_bf16, kFP / 32, w * NBW, acc);
    else mma_f32<MB, NBW>((const float*)sG, Lds::LDA_G, m.w1_f32, kFP / 4, w * NBW, acc);
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int col = (w * NBW + nb) * 16 + (l & 15);
        const float bias = m.b1[col];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (l >> 4) + j;
          float d;
          const float hv = swish_parts(acc[rb][nb][j] + bias, d);
          dsw1[rb][nb][j] = d;
          st_act<BF16>(sH, row * Lds::LDA_H + col, hv);
        }
      }
  }
  __syncthreads();
  {
    floatx4 acc[MB][NBW];
    zero_acc(acc);
    if (BF16) mma_bf16<MB, NBW>((const __bf16*)sH, Lds::LDA_H, m.w2_bf16, HP / 32, w * NBW, acc);
    else mma_f32<MB, NBW>((const float*)sH, Lds::LDA_H, m.w2_f32, HP / 4, w * NBW, acc);
    // z2 -> h2 (kept in acc), delta2 -> LDS
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int col = (w * NBW + nb) * 16 + (l & 15);
        const float bias = m.b2[col];
        const float wb = m.w3bar[col];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (l >> 4) + j;
          float d;
          const float hv = swish_parts(acc[rb][nb][j] + bias, d);
          acc[rb][nb][j] = hv;
          st_act<BF16>(sD2, row * Lds::LDA_H + col, d * sScale[row] * wb);
        }
      }
    // y_m partial sums over this wave's columns
    for (int hm = 0; hm < M; ++hm) {
      float part[MB][4];
#pragma unroll
      for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[rb][j] = 0.0f;
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int col = (w * NBW + nb) * 16 + (l & 15);
        const float w3 = m.w3[col * M + hm];
#pragma unroll
        for (int rb = 0; rb < MB; ++rb)
#pragma unroll
          for (int j = 0; j < 4; ++j) part[rb][j] += acc[rb][nb][j] * w3;
      }
#pragma unroll
      for (int rb = 0; rb < MB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v = part[rb][j];
          v += __shfl_xor(v, 8, 16);
          v += __shfl_xor(v, 4, 16);
          v += __shfl_xor(v, 2, 16);
          v += __shfl_xor(v, 1, 16);
          if ((l & 15) == 0) sEp[(w * TM + rb * 16 + 4 * (l >> 4) + j) * kMaxHeads + hm] = v;
        }
    }
  }
  __syncthreads();
  for (int t = tid; t < TM * M; t += kReadoutThreads) {
    const int a = t / M, hm = t % M;
    const int gi = row0 + a;
    if (gi < sys.n_atoms) {
      float y = m.b3[hm];
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) y += sEp[(ww * TM + a) * kMaxHeads + hm];
      atomic_e[(int64_t)gi * M + hm] = sScale[a] * y + sShift[a];
    }
  }

  // ---- 4. network backward -----------------------------------------------------
  {
    floatx4 acc[MB][NBW];
    zero_acc(acc);
    if (BF16) mma_bf16<MB, NBW>((const __bf16*)sD2, Lds::LDA_H, m.w2t_bf16, HP / 32, w * NBW, acc);
    else mma_f32<MB, NBW>((const float*)sD2, Lds::LDA_H, m.w2t_f32, HP / 4, w * NBW, acc);
    __syncthreads();  // every wave has read h1's region? (sH is not read here; delta1 overwrites h1)
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int col = (w * NBW + nb) * 16 + (l & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (l >> 4) + j;
          st_act<BF16>(sH, row * Lds::LDA_H + col, acc[rb][nb][j] * dsw1[rb][nb][j]);
        }
      }
  }
  __syncthreads();
  {
    floatx4 acc[MB][NBW_G];
    zero_acc(acc);
    if (BF16) mma_bf16<MB, NBW_G>((const __bf16*)sH, Lds::LDA_H, m.w1t_bf16, HP / 32, w * NBW_G, acc);
    else mma_f32<MB, NBW_G>((const float*)sH, Lds::LDA_H, m.w1t_f32, HP / 4, w * NBW_G, acc);
#pragma unroll
    for (int rb = 0; rb < MB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NBW_G; ++nb) {
        const int col = (w * NBW_G + nb) * 16 + (l & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (l >> 4) + j;
          sGb[row * Lds::LDGB + col] = acc[rb][nb][j];
        }
      }
  }
  __syncthreads();

  // ---- 5. backward of the invariants -> dE/dPsi ------------------------------
#define GB(a, f) sGb[(a) * Lds::LDGB + (f)]
#define PB(a, s, r) sPb[(a) * PS + (s) * kFull + (r)]
  // families 1-4
  for (int t = tid; t < TM * kS * kFull; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s = e / kFull, r = e % kFull;
    float v = 0.0f;
    if (r == 0) {
      v = GB(a, s);
    } else if (r < 4) {
      for (int s2 = 0; s2 < kS; ++s2) v += GB(a, kFam2 + c_pair_index[s][s2]) * (s == s2 ? 2.0f : 1.0f) * P1(a, s2, r - 1);
    } else if (r < 13) {
      for (int s2 = 0; s2 < kS; ++s2) v += GB(a, kFam3 + c_pair_index[s][s2]) * (s == s2 ? 2.0f : 1.0f) * P2(a, s2, r - 4);
    } else {
      for (int s2 = 0; s2 < kS; ++s2) v += GB(a, kFam4 + c_pair_index[s][s2]) * (s == s2 ? 2.0f : 1.0f) * P3(a, s2, r - 13);
    }
    sPb[a * PS + e] = v;
  }
  // family 7: recompute T7
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, ia = (e % 9) / 3, ib = e % 3;
    const int s2 = c_pair_s1[p], s3 = c_pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int cd = 0; cd < 9; ++cd) v += P3(a, s2, ia * 9 + cd) * P3(a, s3, ib * 9 + cd);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  // dPsi2[x]_ab += sum_p G7[x][p] T7[p]_ab
  for (int t = tid; t < TM * 45; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 9, ab = e % 9;
    float v = 0.0f;
    for (int p = 0; p < 15; ++p) v += GB(a, kFam7 + x * 15 + p) * sInter[a * IS + p * 9 + ab];
    PB(a, x, 4 + ab) += v;
  }
  __syncthreads();
  // Y[x][s'] = sum_s1 C7[s1][x][s'] P2[s1], C7 = G7[s1][(x,s')] (x2 if x == s')
  for (int t = tid; t < TM * 225; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int xs = e / 9, ab = e % 9;
    const int x = xs / 5, sp = xs % 5;
    const float f2 = (x == sp) ? 2.0f : 1.0f;
    const int p = c_pair_index[x][sp];
    float v = 0.0f;
#pragma unroll
    for (int s1 = 0; s1 < kS; ++s1) v += GB(a, kFam7 + s1 * 15 + p) * P2(a, s1, ab);
    sInter[a * IS + e] = f2 * v;
  }
  __syncthreads();
  // dPsi3[x]_ibc += sum_s' sum_d Y[x][s']_id P3[s']_dbc
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 27, ibc = e % 27;
    const int i = ibc / 9, bc = ibc % 9;
    float v = 0.0f;
    for (int sp = 0; sp < kS; ++sp)
#pragma unroll
      for (int d = 0; d < 3; ++d) v += sInter[a * IS + (x * 5 + sp) * 9 + i * 3 + d] * P3(a, sp, d * 9 + bc);
    PB(a, x, 13 + ibc) += v;
  }
  __syncthreads();
  // family 8: recompute V8; dPsi1[x]_i += sum_{s2,s3} G8[x][s2][s3] V8[s2 s3]_i
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s23 = e / 3, i = e % 3;
    const int s2 = s23 / 5, s3 = s23 % 5;
    float v = 0.0f;
#pragma unroll
    for (int bc = 0; bc < 9; ++bc) v += P3(a, s2, i * 9 + bc) * P2(a, s3, bc);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 15; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 3, i = e % 3;
    float v = 0.0f;
    for (int s23 = 0; s23 < 25; ++s23) v += GB(a, kFam8 + x * 25 + s23) * sInter[a * IS + s23 * 3 + i];
    PB(a, x, 1 + i) += v;
  }
  __syncthreads();
  // U8[s1 s2]_bc = sum_i P1[s1]_i P3[s2]_ibc; dPsi2[x]_bc += sum G8[s1][s2][x] U8[s1 s2]_bc
  for (int t = tid; t < TM * 225; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s12 = e / 9, bc = e % 9;
    const int s1 = s12 / 5, s2 = s12 % 5;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += P1(a, s1, i) * P3(a, s2, i * 9 + bc);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 45; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 9, bc = e % 9;
    float v = 0.0f;
    for (int s12 = 0; s12 < 25; ++s12) v += GB(a, kFam8 + s12 * 5 + x) * sInter[a * IS + s12 * 9 + bc];
    PB(a, x, 4 + bc) += v;
  }
  __syncthreads();
  // Qv[x][s3]_i = sum_s1 G8[s1][x][s3] P1[s1]_i; dPsi3[x]_ibc += sum_s3 Qv[x][s3]_i P2[s3]_bc
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int xs = e / 3, i = e % 3;
    const int x = xs / 5, s3 = xs % 5;
    float v = 0.0f;
#pragma unroll
    for (int s1 = 0; s1 < kS; ++s1) v += GB(a, kFam8 + s1 * 25 + x * 5 + s3) * P1(a, s1, i);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 27, ibc = e % 27;
    const int i = ibc / 9, bc = ibc % 9;
    float v = 0.0f;
#pragma unroll
    for (int s3 = 0; s3 < kS; ++s3) v += sInter[a * IS + (x * 5 + s3) * 3 + i] * P2(a, s3, bc);
    PB(a, x, 13 + ibc) += v;
  }
  __syncthreads();
  // family 5: recompute M5; dPsi2[x] += 3 sum_{s'<=s''} G5[x s' s''] / mult (x2 if s' != s'') M5[s' s'']
  for (int t = tid; t < TM * 135; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, i = (e % 9) / 3, j = e % 3;
    const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) v += P2(a, s1, i * 3 + c) * P2(a, s2, c * 3 + j);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 45; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int x = e / 9, ij = e % 9;
    float v = 0.0f;
    for (int p = 0; p < 15; ++p) {
      const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
      const int mult = (x == s1 && s1 == s2) ? 1 : ((x == s1 || x == s2 || s1 == s2) ? 3 : 6);
      const float c = 3.0f * (s1 != s2 ? 2.0f : 1.0f) / (float)mult;
      v += c * GB(a, kFam5 + c_tri_index[x][s1][s2]) * sInter[a * IS + p * 9 + ij];
    }
    PB(a, x, 4 + ij) += v;
  }
  __syncthreads();
  // family 6: recompute v6; dPsi1 and dPsi2
  for (int t = tid; t < TM * 75; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    const int s31 = e / 3, i = e % 3;
    const int s3 = s31 / 5, s1 = s31 % 5;
    float v = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j) v += P2(a, s3, i * 3 + j) * P1(a, s1, j);
    sInter[a * IS + e] = v;
  }
  __syncthreads();
  for (int t = tid; t < TM * 60; t += kReadoutThreads) {
    const int a = t % TM, e = t / TM;
    if (e < 15) {
      const int x = e / 3, i = e % 3;
      float v = 0.0f;
      for (int sp = 0; sp < kS; ++sp) {
        const float f2 = (x == sp) ? 2.0f : 1.0f;
        const int p = c_pair_index[x][sp];
#pragma unroll
        for (int s3 = 0; s3 < kS; ++s3) v += f2 * GB(a, kFam6 + p * 5 + s3) * sInter[a * IS + (s3 * 5 + sp) * 3 + i];
      }
      PB(a, x, 1 + i) += v;
    } else {
      const int x = (e - 15) / 9, ij = (e - 15) % 9;
      const int i = ij / 3, j = ij % 3;
      float v = 0.0f;
      for (int p = 0; p < 15; ++p) {
        const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
        v += GB(a, kFam6 + p * 5 + x) * P1(a, s1, i) * P1(a, s2, j);
      }
      PB(a, x, 4 + ij) += v;
    }
  }
  __syncthreads();
  // fold the full-tensor gradient onto the packed components
  for (int t = tid; t < TM * kS * kPacked; t += kReadoutThreads) {
    const int a = t / (kS * kPacked), e = t % (kS * kPacked);
    const int s = e / kPacked, mp = e % kPacked;
    const int gi = row0 + a;
    if (gi < sys.n_atoms) {
      float v = 0.0f;
      const int n = c_packed_mult[mp];
      for (int k = 0; k < n; ++k) v += PB(a, s, c_packed_full[mp][k]);
      psibar[(int64_t)gi * (kS * kPacked) + e] = v;
    }
  }
#undef P0
#undef P1
#undef P2
#undef P3
#undef GB
#undef PB
}

// ---------------------------------------------------------------------------
template <int TM, int HP, bool BF16>
static gmnn_status launch_readout_t(const DevModel& m, const DevSystem& sys, const float* psi, float* atomic_e,
                                    float* psibar, hipStream_t stream) {
  using Lds = ReadoutLds<TM, HP, BF16>;
  static_assert(Lds::bytes <= 160 * 1024, "readout tile does not fit in LDS");
  auto k = readout<TM, HP, BF16>;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)Lds::bytes) != hipSuccess)
      return GMNN_ERR_HIP;
    attr_set = true;
  }
  const int grid = (sys.n_atoms + TM - 1) / TM;
  if (grid == 0) return GMNN_OK;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kReadoutThreads), Lds::bytes, stream, m, sys, psi, atomic_e, psibar);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

size_t readout_lds_bytes(int tm, int hp, bool bf16) {
#define CASE(TM, HP)                                                                         \
  if (tm == TM && hp == HP) return bf16 ? ReadoutLds<TM, HP, true>::bytes : ReadoutLds<TM, HP, false>::bytes;
  CASE(16, 64) CASE(16, 128) CASE(16, 256) CASE(16, 512)
  CASE(32, 64) CASE(32, 128) CASE(32, 256) CASE(32, 512)
#undef CASE
  return 0;
}

gmnn_status launch_readout(int tm, const DevModel& m, const DevSystem& sys, bool bf16, const float* psi,
                           float* atomic_e, float* psibar, hipStream_t stream) {
  const int hp = m.HP1;
#define CASE(TM, HP)                                                                         \
  if (tm == TM && hp == HP) {                                                                \
    if (readout_lds_bytes(TM, HP, bf16) > 160 * 1024) return GMNN_ERR_UNSUPPORTED;           \
    return bf16 ? launch_readout_t<TM, HP, true>(m, sys, psi, atomic_e, psibar, stream)      \
                : launch_readout_t<TM, HP, false>(m, sys, psi, atomic_e, psibar, stream);    \
  }
  CASE(16, 64) CASE(16, 128) CASE(16, 256) CASE(16, 512)
  CASE(32, 64) CASE(32, 128) CASE(32, 256)
  if (tm == 32 && hp == 512) {
    if (!bf16) return GMNN_ERR_UNSUPPORTED;
    return launch_readout_t<32, 512, true>(m, sys, psi, atomic_e, psibar, stream);
  }
#undef CASE
  return GMNN_ERR_UNSUPPORTED;
}

}  // namespace gmnn
