// Invariants of the Cartesian moments (Section 2.1, eq. contraction) and
// their product-rule backward, for a tile of TM atoms held in LDS, executed
// by all NT threads of a block.
//
// Layouts (floats, per atom, in LDS):
//   P   full tensors, stride PS: channel s at s*40: Psi0 | Psi1[a] | Psi2[a][b] | Psi3[a][b][c]
//   I   intermediates, stride IS:
//         T7[p][ab] = sum_cd Psi3[s2]_acd Psi3[s3]_bcd, p = (s2 <= s3)     @0    (135)
//         V8[s2 s3][a] = sum_bc Psi3[s2]_abc Psi2[s3]_bc                   @135  (75)
//         M5[p][ab] = (Psi2[s1] Psi2[s2])_ab, p = (s1 <= s2)               @210  (135)
//         v6[s3 s1][a] = (Psi2[s3] Psi1[s1])_a                             @345  (75)
//         U8[s1 s2][bc] = sum_a Psi1[s1]_a Psi3[s2]_abc                    @420  (225)
//         Y[x s'][ab] = c7 sum_s1 dE/dG7[s1][(x,s')] Psi2[s1]_ab           @645  (225)
//         Qv[x s3][a] = sum_s1 dE/dG8[s1][x][s3] Psi1[s1]_a                @870  (75)
//   Pb  full-tensor gradient dE/dPsi, stride PS
// Inside every loop the task index runs atom-fastest, so the lanes of a wave
// read the same tensor entry of different atoms (odd strides: no bank
// conflicts) and take the same branch.
#pragma once

#include "common.h"
#include "tables.h"

namespace gmnn {

constexpr int PS = 201;   // atom stride of full tensors (odd)
constexpr int IS = 945;   // atom stride of the intermediates (odd)
constexpr int ISF = 421;  // ... when only the forward intermediates (T7, V8, M5, v6) are kept
constexpr int kT7 = 0, kV8 = 135, kM5 = 210, kV6 = 345, kU8 = 420, kY = 645, kQv = 870;

// LDS copies of the index tables (per-lane lookups in constant memory would
// go through the vector memory path; LDS serves them in a few cycles)
struct Tables {
  unsigned char full_to_packed[kFull];
  unsigned char packed_mult[kPacked];
  unsigned char packed_full[kPacked][6];
  unsigned char pair_s1[15], pair_s2[15];
  unsigned char pair_index[25];
  unsigned char tri_s1[35], tri_s2[35], tri_s3[35];
  unsigned char tri_index[125];
  unsigned char tri_xp[kS * 15];  // sorted-triple index of (x, s1, s2), p = (s1 <= s2)
  float c5[kS * 15];              // 3 (2 if s1 != s2) / (distinct orderings of {x, s1, s2})
};

__device__ inline void load_tables(Tables* t) {
  for (int k = threadIdx.x; k < 125; k += blockDim.x) {
    if (k < kFull) t->full_to_packed[k] = c_full_to_packed[k];
    if (k < kPacked) {
      t->packed_mult[k] = c_packed_mult[k];
      for (int e = 0; e < 6; ++e) t->packed_full[k][e] = c_packed_full[k][e];
    }
    if (k < 15) {
      t->pair_s1[k] = c_pair_s1[k];
      t->pair_s2[k] = c_pair_s2[k];
    }
    if (k < 25) t->pair_index[k] = c_pair_index[k / 5][k % 5];
    if (k < 35) {
      t->tri_s1[k] = c_tri_s1[k];
      t->tri_s2[k] = c_tri_s2[k];
      t->tri_s3[k] = c_tri_s3[k];
    }
    t->tri_index[k] = c_tri_index[k / 25][(k / 5) % 5][k % 5];
    if (k < kS * 15) {
      const int x = k / 15, p = k % 15;
      const int s1 = c_pair_s1[p], s2 = c_pair_s2[p];
      const int mult = (x == s1 && s1 == s2) ? 1 : ((x == s1 || x == s2 || s1 == s2) ? 3 : 6);
      t->tri_xp[k] = c_tri_index[x][s1][s2];
      t->c5[k] = 3.0f * (s1 != s2 ? 2.0f : 1.0f) / (float)mult;
    }
  }
}

#define GM_P0(a, s) P[(a) * PS + (s) * kFull]
#define GM_P1(a, s, i) P[(a) * PS + (s) * kFull + 1 + (i)]
#define GM_P2(a, s, ij) P[(a) * PS + (s) * kFull + 4 + (ij)]
#define GM_P3(a, s, ijk) P[(a) * PS + (s) * kFull + 13 + (ijk)]
#define GM_I(a, off) I[(a) * ISTR + (off)]

// an invariant into the network operand G: FP32, or bf16 (G[idx] = bf16(v));
// with glo > 0 also the low part G[idx + glo] = bf16(v - bf16(v)) for the
// split-BF16 first product
template <bool BF16>
__device__ inline void store_feature(void* G, int idx, float v, int glo = 0) {
  if (BF16) {
    const __bf16 h = (__bf16)v;
    ((__bf16*)G)[idx] = h;
    if (glo) ((__bf16*)G)[idx + glo] = (__bf16)split_low(v, h);
  } else {
    ((float*)G)[idx] = v;
  }
}

// pair index of (s1 <= s2) in the lexicographic pair order, as arithmetic
// (folds to a constant when both channels are compile-time constants)
__host__ __device__ constexpr int pair_idx(int s1, int s2) {
  return (s1 <= s2) ? s1 * kS - s1 * (s1 - 1) / 2 + (s2 - s1) : s2 * kS - s2 * (s2 - 1) / 2 + (s1 - s2);
}
__host__ __device__ constexpr int pair_first(int p) { return p < 5 ? 0 : p < 9 ? 1 : p < 12 ? 2 : p < 14 ? 3 : 4; }
__host__ __device__ constexpr int pair_second(int p) {
  return pair_first(p) + p - (pair_first(p) * kS - pair_first(p) * (pair_first(p) - 1) / 2);
}

// Phase A of the forward: families 1-4 and the intermediates T7, V8, M5, v6
// (all read only P).  Also zeroes the padding features.  FEATURES = false
// computes the intermediates only.  Register-blocked tasks (atom fastest):
//   pair task (a, p = (s1 <= s2)):  T7[p], M5[p]; fam4[p] = tr T7[p] and
//                                   fam3[p] = tr M5[p] (Psi2 is symmetric)
//   channel task (a, s):            V8[s, .], v6[s, .]; fam1[s]; fam2[(s, s2 >= s)]
// KS = 2 (a block with twice as many threads as tasks) runs each task's two
// independent halves on two threads: T7 + fam4 | M5 + fam3, and
// V8 | v6 + fam1 + fam2.
template <int TM, int NT, bool BF16, bool FEATURES = true, int ISTR = IS, int KS = 1>
__device__ inline void contract_forward_a(const float* __restrict__ P, float* __restrict__ I, void* G, int ldg,
                                          const Tables& tb, int glo = 0) {
  static_assert(KS == 1 || KS == 2, "one or two halves");
  const int tid = threadIdx.x;
  for (int t = tid; t < (FEATURES ? TM * (kFP - kF) : 0); t += NT)
    store_feature<BF16>(G, (t % TM) * ldg + kF + t / TM, 0.0f, glo);
  constexpr int np = TM * 15, ns = TM * kS;
  // with KS = 2 each half's tasks start on a wave boundary
  constexpr int NTASK = np + ns, NHALF = KS == 1 ? NTASK : (NTASK + 63) / 64 * 64;
  for (int tt = tid; tt < KS * NHALF; tt += NT) {
    const int half = KS == 1 ? 0 : tt / NHALF;
    const int t = KS == 1 ? tt : tt % NHALF;
    if (t >= NTASK) continue;
    const bool h0 = KS == 1 || half == 0, h1 = KS == 1 || half == 1;
    if (t < np) {
      const int a = t % TM, p = t / TM;
      const int s1 = pair_first(p), s2 = pair_second(p);
      if (h0) {
        float A3[27], B3[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
          A3[k] = GM_P3(a, s1, k);
          B3[k] = GM_P3(a, s2, k);
        }
        float tr4 = 0.0f;
#pragma unroll
        for (int ia = 0; ia < 3; ++ia)
#pragma unroll
          for (int ib = 0; ib < 3; ++ib) {
            float v = 0.0f;
#pragma unroll
            for (int cd = 0; cd < 9; ++cd) v += A3[ia * 9 + cd] * B3[ib * 9 + cd];
            GM_I(a, kT7 + p * 9 + ia * 3 + ib) = v;
            if (ia == ib) tr4 += v;
          }
        if (FEATURES) store_feature<BF16>(G, a * ldg + kFam4 + p, tr4, glo);
      }
      if (h1) {
        float A2[9], B2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          A2[k] = GM_P2(a, s1, k);
          B2[k] = GM_P2(a, s2, k);
        }
        float tr3 = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            float v = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) v += A2[i * 3 + c] * B2[c * 3 + j];
            GM_I(a, kM5 + p * 9 + i * 3 + j) = v;
            if (i == j) tr3 += v;
          }
        if (FEATURES) store_feature<BF16>(G, a * ldg + kFam3 + p, tr3, glo);
      }
    } else {
      const int u = t - np;
      const int a = u % TM, sc = u / TM;
      if (h0) {
        float A3[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) A3[k] = GM_P3(a, sc, k);
#pragma unroll
        for (int s3 = 0; s3 < kS; ++s3) {
          float B2[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) B2[k] = GM_P2(a, s3, k);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
#pragma unroll
            for (int bc = 0; bc < 9; ++bc) v += A3[i * 9 + bc] * B2[bc];
            GM_I(a, kV8 + (sc * 5 + s3) * 3 + i) = v;
          }
        }
      }
      if (h1) {
        float C2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) C2[k] = GM_P2(a, sc, k);
        float p1[kS][3];
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
          for (int j = 0; j < 3; ++j) p1[s1][j] = GM_P1(a, s1, j);
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) v += C2[i * 3 + j] * p1[s1][j];
            GM_I(a, kV6 + (sc * 5 + s1) * 3 + i) = v;
          }
        if (FEATURES) {
          store_feature<BF16>(G, a * ldg + sc, GM_P0(a, sc), glo);
#pragma unroll
          for (int s2 = 0; s2 < kS; ++s2) {
            if (s2 < sc) continue;
            float v = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              // p1[sc][i] with sc a runtime index: read it again from LDS
              v += GM_P1(a, sc, i) * p1[s2][i];
            }
            store_feature<BF16>(G, a * ldg + kFam2 + pair_idx(sc, s2), v, glo);
          }
        }
      }
    }
  }
}

// Phase B of the forward: families 5-8 from the intermediates.
//   pair task (a, p = (s1 <= s2)):  fam7[(s', p)] for every s'; fam5[(s1, s2, s3)]
//                                   for s3 >= s2; fam6[(p, s3)] for every s3
//   channel task (a, s2):           fam8[(s1, s2, s3)] for every s1, s3
template <int TM, int NT, bool BF16, int ISTR = IS>
__device__ inline void contract_forward_b(const float* __restrict__ P, const float* __restrict__ I, void* G, int ldg,
                                          const Tables& tb, int glo = 0) {
  constexpr int np = TM * 15, ns = TM * kS;
  for (int t = threadIdx.x; t < np + ns; t += NT) {
    if (t < np) {
      const int a = t % TM, p = t / TM;
      const int s1 = pair_first(p), s2 = pair_second(p);
      float t7[9], m5[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        t7[k] = GM_I(a, kT7 + p * 9 + k);
        m5[k] = GM_I(a, kM5 + p * 9 + k);
      }
#pragma unroll
      for (int sq = 0; sq < kS; ++sq) {
        float q[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k] = GM_P2(a, sq, k);
        float f7 = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) f7 += q[k] * t7[k];
        store_feature<BF16>(G, a * ldg + kFam7 + sq * 15 + p, f7, glo);
        if (sq >= s2) {
          float f5 = 0.0f;
#pragma unroll
          for (int k = 0; k < 9; ++k) f5 += m5[k] * q[k];
          store_feature<BF16>(G, a * ldg + kFam5 + tb.tri_index[s1 * 25 + s2 * 5 + sq], f5, glo);
        }
      }
      float r[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) r[i] = GM_P1(a, s2, i);
#pragma unroll
      for (int s3 = 0; s3 < kS; ++s3) {
        float f6 = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i) f6 += GM_I(a, kV6 + (s3 * 5 + s1) * 3 + i) * r[i];
        store_feature<BF16>(G, a * ldg + kFam6 + p * 5 + s3, f6, glo);
      }
    } else {
      const int u = t - np;
      const int a = u % TM, s2 = u / TM;
      float p1[kS][3];
#pragma unroll
      for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
        for (int i = 0; i < 3; ++i) p1[s1][i] = GM_P1(a, s1, i);
#pragma unroll
      for (int s3 = 0; s3 < kS; ++s3) {
        float w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) w[i] = GM_I(a, kV8 + (s2 * 5 + s3) * 3 + i);
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1) {
          float f8 = 0.0f;
#pragma unroll
          for (int i = 0; i < 3; ++i) f8 += p1[s1][i] * w[i];
          store_feature<BF16>(G, a * ldg + kFam8 + s1 * 25 + s2 * 5 + s3, f8, glo);
        }
      }
    }
  }
}

// Tangent of the invariants along a direction Pd of the moments (dual
// numbers): Gd = dG/dPsi . Pd, each family by the product rule, exactly
// (G is a polynomial of degree <= 3 in Psi).  Same task structure as the
// primal passes.  Phase A writes the tangent intermediates Id (stride IDS:
// T7, V8, M5, v6 at the primal offsets) and the tangents of families 1-4;
// phase B the tangents of families 5-8 from the primal intermediates I
// (stride IS) and Id.  Gd is FP32 with row stride ldg; the padding features
// are zeroed.
#define GM_D1(a, s, i) Pd[(a) * PS + (s) * kFull + 1 + (i)]
#define GM_D2(a, s, ij) Pd[(a) * PS + (s) * kFull + 4 + (ij)]
#define GM_D3(a, s, ijk) Pd[(a) * PS + (s) * kFull + 13 + (ijk)]
template <int TM, int NT, int IDS, int KS = 1>
__device__ inline void contract_forward_a_dual(const float* __restrict__ P, const float* __restrict__ Pd,
                                               float* __restrict__ Id, float* __restrict__ Gd, int ldg) {
  static_assert(KS == 1 || KS == 2, "one or two halves");
  const int tid = threadIdx.x;
  for (int t = tid; t < TM * (kFP - kF); t += NT) Gd[(t % TM) * ldg + kF + t / TM] = 0.0f;
  constexpr int np = TM * 15, ns = TM * kS;
  constexpr int NTASK = np + ns, NHALF = KS == 1 ? NTASK : (NTASK + 63) / 64 * 64;
  for (int tt = tid; tt < KS * NHALF; tt += NT) {
    const int half = KS == 1 ? 0 : tt / NHALF;
    const int t = KS == 1 ? tt : tt % NHALF;
    if (t >= NTASK) continue;
    const bool h0 = KS == 1 || half == 0, h1 = KS == 1 || half == 1;
    if (t < np) {
      const int a = t % TM, p = t / TM;
      const int s1 = pair_first(p), s2 = pair_second(p);
      if (h0) {
        float A3[27], B3[27], dA3[27], dB3[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
          A3[k] = GM_P3(a, s1, k);
          B3[k] = GM_P3(a, s2, k);
          dA3[k] = GM_D3(a, s1, k);
          dB3[k] = GM_D3(a, s2, k);
        }
        float tr4 = 0.0f;
#pragma unroll
        for (int ia = 0; ia < 3; ++ia)
#pragma unroll
          for (int ib = 0; ib < 3; ++ib) {
            float v = 0.0f;
#pragma unroll
            for (int cd = 0; cd < 9; ++cd) v += dA3[ia * 9 + cd] * B3[ib * 9 + cd] + A3[ia * 9 + cd] * dB3[ib * 9 + cd];
            Id[a * IDS + kT7 + p * 9 + ia * 3 + ib] = v;
            if (ia == ib) tr4 += v;
          }
        Gd[a * ldg + kFam4 + p] = tr4;
      }
      if (h1) {
        float A2[9], B2[9], dA2[9], dB2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          A2[k] = GM_P2(a, s1, k);
          B2[k] = GM_P2(a, s2, k);
          dA2[k] = GM_D2(a, s1, k);
          dB2[k] = GM_D2(a, s2, k);
        }
        float tr3 = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            float v = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) v += dA2[i * 3 + c] * B2[c * 3 + j] + A2[i * 3 + c] * dB2[c * 3 + j];
            Id[a * IDS + kM5 + p * 9 + i * 3 + j] = v;
            if (i == j) tr3 += v;
          }
        Gd[a * ldg + kFam3 + p] = tr3;
      }
    } else {
      const int u = t - np;
      const int a = u % TM, sc = u / TM;
      if (h0) {
        float A3[27], dA3[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
          A3[k] = GM_P3(a, sc, k);
          dA3[k] = GM_D3(a, sc, k);
        }
#pragma unroll
        for (int s3 = 0; s3 < kS; ++s3) {
          float B2[9], dB2[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            B2[k] = GM_P2(a, s3, k);
            dB2[k] = GM_D2(a, s3, k);
          }
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
#pragma unroll
            for (int bc = 0; bc < 9; ++bc) v += dA3[i * 9 + bc] * B2[bc] + A3[i * 9 + bc] * dB2[bc];
            Id[a * IDS + kV8 + (sc * 5 + s3) * 3 + i] = v;
          }
        }
      }
      if (h1) {
        float C2[9], dC2[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          C2[k] = GM_P2(a, sc, k);
          dC2[k] = GM_D2(a, sc, k);
        }
        float p1[kS][3], d1[kS][3];
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            p1[s1][j] = GM_P1(a, s1, j);
            d1[s1][j] = GM_D1(a, s1, j);
          }
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) v += dC2[i * 3 + j] * p1[s1][j] + C2[i * 3 + j] * d1[s1][j];
            Id[a * IDS + kV6 + (sc * 5 + s1) * 3 + i] = v;
          }
        Gd[a * ldg + sc] = Pd[a * PS + sc * kFull];
#pragma unroll
        for (int s2 = 0; s2 < kS; ++s2) {
          if (s2 < sc) continue;
          float v = 0.0f;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            // the sc entries with sc a runtime index: read them again from LDS
            v += GM_D1(a, sc, i) * p1[s2][i] + GM_P1(a, sc, i) * d1[s2][i];
          }
          Gd[a * ldg + kFam2 + pair_idx(sc, s2)] = v;
        }
      }
    }
  }
}

template <int TM, int NT, int IDS>
__device__ inline void contract_forward_b_dual(const float* __restrict__ P, const float* __restrict__ Pd,
                                               const float* __restrict__ I, const float* __restrict__ Id,
                                               float* __restrict__ Gd, int ldg, const Tables& tb) {
  constexpr int ISTR = IS;
  constexpr int np = TM * 15, ns = TM * kS;
  for (int t = threadIdx.x; t < np + ns; t += NT) {
    if (t < np) {
      const int a = t % TM, p = t / TM;
      const int s1 = pair_first(p), s2 = pair_second(p);
      float t7[9], m5[9], dt7[9], dm5[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        t7[k] = GM_I(a, kT7 + p * 9 + k);
        m5[k] = GM_I(a, kM5 + p * 9 + k);
        dt7[k] = Id[a * IDS + kT7 + p * 9 + k];
        dm5[k] = Id[a * IDS + kM5 + p * 9 + k];
      }
#pragma unroll
      for (int sq = 0; sq < kS; ++sq) {
        float q[9], dq[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          q[k] = GM_P2(a, sq, k);
          dq[k] = GM_D2(a, sq, k);
        }
        float f7 = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) f7 += dq[k] * t7[k] + q[k] * dt7[k];
        Gd[a * ldg + kFam7 + sq * 15 + p] = f7;
        if (sq >= s2) {
          float f5 = 0.0f;
#pragma unroll
          for (int k = 0; k < 9; ++k) f5 += dm5[k] * q[k] + m5[k] * dq[k];
          Gd[a * ldg + kFam5 + tb.tri_index[s1 * 25 + s2 * 5 + sq]] = f5;
        }
      }
      float r[3], dr[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        r[i] = GM_P1(a, s2, i);
        dr[i] = GM_D1(a, s2, i);
      }
#pragma unroll
      for (int s3 = 0; s3 < kS; ++s3) {
        float f6 = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          f6 += Id[a * IDS + kV6 + (s3 * 5 + s1) * 3 + i] * r[i] + GM_I(a, kV6 + (s3 * 5 + s1) * 3 + i) * dr[i];
        Gd[a * ldg + kFam6 + p * 5 + s3] = f6;
      }
    } else {
      const int u = t - np;
      const int a = u % TM, s2 = u / TM;
      float p1[kS][3], d1[kS][3];
#pragma unroll
      for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          p1[s1][i] = GM_P1(a, s1, i);
          d1[s1][i] = GM_D1(a, s1, i);
        }
#pragma unroll
      for (int s3 = 0; s3 < kS; ++s3) {
        float w[3], dw[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          w[i] = GM_I(a, kV8 + (s2 * 5 + s3) * 3 + i);
          dw[i] = Id[a * IDS + kV8 + (s2 * 5 + s3) * 3 + i];
        }
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1) {
          float f8 = 0.0f;
#pragma unroll
          for (int i = 0; i < 3; ++i) f8 += d1[s1][i] * w[i] + p1[s1][i] * dw[i];
          Gd[a * ldg + kFam8 + s1 * 25 + s2 * 5 + s3] = f8;
        }
      }
    }
  }
}
#undef GM_D1
#undef GM_D2
#undef GM_D3

#define GM_GB(a, f) Gb[(a) * ldgb + (f)]

// Phase A of the backward: intermediates U8, Y, Qv (read P and dE/dG).
//   task (a, s2, b):  U8[(s1, s2)][b, c] for every s1, c, and the five Qv
//                     entries [x = s2][s3][i] with 3 s3 + i in [5b, 5b + 5)
//   task (a, p = (x <= s')):  Y[(x, s')] and its mirror Y[(s', x)]
// KS = 2 (a block with twice as many threads as tasks) runs each task's two
// independent output groups on two threads: U8 | Qv, and the Y entries
// ab < 5 | ab >= 5.  Every output keeps its single writer and its order of
// operations, so the split changes no result.
template <int TM, int NT, int KS = 1>
__device__ inline void contract_backward_a(const float* __restrict__ P, const float* __restrict__ Gb, int ldgb,
                                           float* __restrict__ I, const Tables& tb) {
  static_assert(KS == 1 || KS == 2, "one or two halves");
  constexpr int ISTR = IS;
  constexpr int nu = TM * 15, ny = TM * 15;
  // with KS = 2 each half's tasks start on a wave boundary
  constexpr int NTASK = nu + ny, NHALF = KS == 1 ? NTASK : (NTASK + 63) / 64 * 64;
  for (int tt = threadIdx.x; tt < KS * NHALF; tt += NT) {
    const int half = KS == 1 ? 0 : tt / NHALF;
    const int t = KS == 1 ? tt : tt % NHALF;
    if (t >= NTASK) continue;
    const bool h0 = KS == 1 || half == 0, h1 = KS == 1 || half == 1;
    if (t < nu) {
      const int a = t % TM, e = t / TM;
      const int s2 = e / 3, b = e % 3;
      float p1[kS][3], p3[3][3];
#pragma unroll
      for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
        for (int i = 0; i < 3; ++i) p1[s1][i] = GM_P1(a, s1, i);
      if (h0) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) p3[i][c] = GM_P3(a, s2, i * 9 + b * 3 + c);
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            float v = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) v += p1[s1][i] * p3[i][c];
            GM_I(a, kU8 + (s1 * 5 + s2) * 9 + b * 3 + c) = v;
          }
      }
      if (h1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const int lin = 5 * b + q;
          const int s3 = lin / 3, i = lin % 3;
          float v = 0.0f;
#pragma unroll
          for (int s1 = 0; s1 < kS; ++s1) v += GM_GB(a, kFam8 + s1 * 25 + s2 * 5 + s3) * GM_P1(a, s1, i);
          GM_I(a, kQv + (s2 * 5 + s3) * 3 + i) = v;
        }
      }
    } else {
      const int u = t - nu;
      const int a = u % TM, p = u / TM;
      const int x = pair_first(p), sp = pair_second(p);
      float g[kS];
#pragma unroll
      for (int s1 = 0; s1 < kS; ++s1) g[s1] = GM_GB(a, kFam7 + s1 * 15 + p);
      const float f = (x == sp) ? 2.0f : 1.0f;
#pragma unroll
      for (int ab = 0; ab < 9; ++ab) {
        if (!(ab < 5 ? h0 : h1)) continue;
        float v = 0.0f;
#pragma unroll
        for (int s1 = 0; s1 < kS; ++s1) v += g[s1] * GM_P2(a, s1, ab);
        GM_I(a, kY + (x * 5 + sp) * 9 + ab) = f * v;
        if (x != sp) GM_I(a, kY + (sp * 5 + x) * 9 + ab) = f * v;
      }
    }
  }
}

// Phase B of the backward: every entry of the full-tensor gradient, each
// summing all of its contributions (one writer per entry).  Register-blocked
// tasks, all kinds in one pass over the threads (atom fastest):
//   Psi2 task (a, x, i):  the 3 entries (x, i, j); the Psi1 entries and the
//                         contraction intermediates are read once per task
//   Psi3 task (a, i, b):  the 15 entries (x, i, b, c), sharing the Psi2/Psi3
//                         entries of every channel across x
//   Psi01 task (a, x):    Psi0 and the 3 Psi1 entries of channel x
// KS = 2 (a block with twice as many threads as tasks) splits every task's
// sum into two halves run by two threads: the first half's partial gradient
// goes to Pb, the second's to Pb2 (every entry written in both), and
// fold_packed adds the two.  The halves: Psi2 = families 3, 5-7 of p < 11 |
// families 5-7 of p >= 11 and 8; Psi3 = channels s' < 3 | s' >= 3; Psi01 =
// families 0, 2, 6 | family 8.
template <int TM, int NT, int KS = 1>
__device__ inline void contract_backward_b(const float* __restrict__ P, const float* __restrict__ Gb, int ldgb,
                                           const float* __restrict__ I, float* __restrict__ Pb, const Tables& tb,
                                           float* __restrict__ Pb2 = nullptr) {
  constexpr int ISTR = IS;
  constexpr int n2 = TM * 15, n3 = TM * 9, n1 = TM * 5;
  // with KS = 2 each half's tasks start on a wave boundary, so a wave runs
  // one half only
  constexpr int NTASK = n2 + n3 + n1, NHALF = KS == 1 ? NTASK : (NTASK + 63) / 64 * 64;
  static_assert(KS == 1 || KS == 2, "one or two halves");
  constexpr int kPSplit = 11;
  for (int tt = threadIdx.x; tt < KS * NHALF; tt += NT) {
    const int half = KS == 1 ? 0 : tt / NHALF;
    const int t = KS == 1 ? tt : tt % NHALF;
    if (t >= NTASK) continue;
    const bool h0 = KS == 1 || half == 0, h1 = KS == 1 || half == 1;
    float* __restrict__ out = half ? Pb2 : Pb;
    if (t < n2) {
      const int a = t % TM, e = t / TM;
      const int x = e / 3, i = e % 3;
      float p1i[kS], p1[kS][3];
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        p1i[s] = GM_P1(a, s, i);
#pragma unroll
        for (int j = 0; j < 3; ++j) p1[s][j] = GM_P1(a, s, j);
      }
      float v[3] = {0.0f, 0.0f, 0.0f};
      if (h0) {
#pragma unroll
        for (int sp = 0; sp < kS; ++sp) {
          const float g = (x == sp ? 2.0f : 1.0f) * GM_GB(a, kFam3 + pair_idx(x, sp));
#pragma unroll
          for (int j = 0; j < 3; ++j) v[j] += g * GM_P2(a, sp, 3 * i + j);
        }
      }
#pragma unroll
      for (int p = 0; p < 15; ++p) {
        if (!(p < kPSplit ? h0 : h1)) continue;
        const int s1 = pair_first(p), s2 = pair_second(p);
        const float g5 = tb.c5[x * 15 + p] * GM_GB(a, kFam5 + tb.tri_xp[x * 15 + p]);
        const float g6 = GM_GB(a, kFam6 + p * 5 + x) * p1i[s1];
        const float g7 = GM_GB(a, kFam7 + x * 15 + p);
#pragma unroll
        for (int j = 0; j < 3; ++j)
          v[j] += g5 * GM_I(a, kM5 + p * 9 + 3 * i + j) + g7 * GM_I(a, kT7 + p * 9 + 3 * i + j) + g6 * p1[s2][j];
      }
      if (h1) {
#pragma unroll
        for (int s12 = 0; s12 < 25; ++s12) {
          const float g8 = GM_GB(a, kFam8 + s12 * 5 + x);
#pragma unroll
          for (int j = 0; j < 3; ++j) v[j] += g8 * GM_I(a, kU8 + s12 * 9 + 3 * i + j);
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) out[a * PS + x * kFull + 4 + 3 * i + j] = v[j];
    } else if (t < n2 + n3) {
      const int u = t - n2;
      const int a = u % TM, e = u / TM;
      const int i = e / 3, b = e % 3;
      float v[kS][3];
#pragma unroll
      for (int x = 0; x < kS; ++x) v[x][0] = v[x][1] = v[x][2] = 0.0f;
#pragma unroll
      for (int sp = 0; sp < kS; ++sp) {
        if (!(sp < 3 ? h0 : h1)) continue;
        float p3i[3], p3d[3][3], p2b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          p3i[c] = GM_P3(a, sp, i * 9 + b * 3 + c);
          p2b[c] = GM_P2(a, sp, b * 3 + c);
#pragma unroll
          for (int d = 0; d < 3; ++d) p3d[d][c] = GM_P3(a, sp, d * 9 + b * 3 + c);
        }
#pragma unroll
        for (int x = 0; x < kS; ++x) {
          const float g4 = (x == sp ? 2.0f : 1.0f) * GM_GB(a, kFam4 + pair_idx(x, sp));
          const float y0 = GM_I(a, kY + (x * 5 + sp) * 9 + i * 3);
          const float y1 = GM_I(a, kY + (x * 5 + sp) * 9 + i * 3 + 1);
          const float y2 = GM_I(a, kY + (x * 5 + sp) * 9 + i * 3 + 2);
          const float q = GM_I(a, kQv + (x * 5 + sp) * 3 + i);
#pragma unroll
          for (int c = 0; c < 3; ++c)
            v[x][c] += g4 * p3i[c] + y0 * p3d[0][c] + y1 * p3d[1][c] + y2 * p3d[2][c] + q * p2b[c];
        }
      }
#pragma unroll
      for (int x = 0; x < kS; ++x)
#pragma unroll
        for (int c = 0; c < 3; ++c) out[a * PS + x * kFull + 13 + i * 9 + b * 3 + c] = v[x][c];
    } else {
      const int u = t - n2 - n3;
      const int a = u % TM, x = u / TM;
      float v[3] = {0.0f, 0.0f, 0.0f};
      if (h0) {
#pragma unroll
        for (int sp = 0; sp < kS; ++sp) {
          const int p = pair_idx(x, sp);
          const float f2 = (x == sp) ? 2.0f : 1.0f;
          const float g2 = f2 * GM_GB(a, kFam2 + p);
#pragma unroll
          for (int k = 0; k < 3; ++k) v[k] += g2 * GM_P1(a, sp, k);
#pragma unroll
          for (int s3 = 0; s3 < kS; ++s3) {
            const float g6 = f2 * GM_GB(a, kFam6 + p * 5 + s3);
#pragma unroll
            for (int k = 0; k < 3; ++k) v[k] += g6 * GM_I(a, kV6 + (s3 * 5 + sp) * 3 + k);
          }
        }
      }
      if (h1) {
#pragma unroll
        for (int s23 = 0; s23 < 25; ++s23) {
          const float g8 = GM_GB(a, kFam8 + x * 25 + s23);
#pragma unroll
          for (int k = 0; k < 3; ++k) v[k] += g8 * GM_I(a, kV8 + s23 * 3 + k);
        }
      }
      out[a * PS + x * kFull] = h0 ? GM_GB(a, x) : 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) out[a * PS + x * kFull + 1 + k] = v[k];
    }
  }
}

// Fold the full-tensor gradient onto the packed components: out(a, k) for
// k = s*20 + t receives the sum of the full entries packed component t
// stands for, in the table's order.  With Pb2 (the second half of a split
// contract_backward_b) every entry is Pb + Pb2.  Two item orders:
//   default        one task per (atom, channel) with compile-time component
//                  indices: the 40 full entries of the channel are read once
//   WAVE_UNIFORM   each wave takes whole packed components t (its table
//                  entries are LDS broadcasts), its lanes the (atom, channel)
//                  pairs: more, shorter items, for few atoms and two halves
template <int TM, int NT, typename Out, bool WAVE_UNIFORM = false>
__device__ inline void fold_packed(const float* __restrict__ Pb, const Tables& tb, Out out,
                                   const float* __restrict__ Pb2 = nullptr) {
  if (WAVE_UNIFORM) {
    constexpr int NWV = NT / 64;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    for (int c = w; c < kPacked; c += NWV) {
      const int n = tb.packed_mult[c];
      int e[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) e[q] = tb.packed_full[c][q];
      for (int t = l; t < TM * kS; t += 64) {
        const int a = t % TM, s = t / TM;
        const float* f = Pb + a * PS + s * kFull;
        const float* f2 = Pb2 ? Pb2 + a * PS + s * kFull : nullptr;
        float x[6];
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (q < n) x[q] = f2 ? f[e[q]] + f2[e[q]] : f[e[q]];
        float v = x[0];
#pragma unroll
        for (int q = 1; q < 6; ++q)
          if (q < n) v += x[q];
        out(a, s * kPacked + c, v);
      }
    }
    return;
  }
  constexpr unsigned char mult[kPacked] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1, 1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
  constexpr unsigned char full[kPacked][6] = {
      {0}, {1}, {2}, {3}, {4}, {5, 7}, {6, 10}, {8}, {9, 11}, {12},
      {13}, {14, 16, 22}, {15, 19, 31}, {17, 23, 25}, {18, 20, 24, 28, 32, 34}, {21, 33, 37},
      {26}, {27, 29, 35}, {30, 36, 38}, {39}};
  for (int t = threadIdx.x; t < TM * kS; t += NT) {
    const int a = t % TM, s = t / TM;
    const float* f = Pb + a * PS + s * kFull;
    const float* f2 = Pb2 ? Pb2 + a * PS + s * kFull : nullptr;
    auto entry = [&](int e) { return f2 ? f[e] + f2[e] : f[e]; };
#pragma unroll
    for (int c = 0; c < kPacked; ++c) {
      float v = entry(full[c][0]);
#pragma unroll
      for (int k = 1; k < 6; ++k)
        if (k < mult[c]) v += entry(full[c][k]);
      out(a, s * kPacked + c, v);
    }
  }
}

#undef GM_GB
#undef GM_P0
#undef GM_P1
#undef GM_P2
#undef GM_P3
#undef GM_I

}  // namespace gmnn
