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
#define GM_I(a, off) I[(a) * IS + (off)]

template <bool BF16>
__device__ inline void store_feature(void* G, int idx, float v) {
  if (BF16) ((__bf16*)G)[idx] = (__bf16)v;
  else ((float*)G)[idx] = v;
}

// Phase A of the forward: families 1-4 directly, and the intermediates
// T7, V8, M5, v6 (all read only P).  Also zeroes the padding features.
// FEATURES = false computes the intermediates only.
template <int TM, int NT, bool BF16, bool FEATURES = true>
__device__ inline void contract_forward_a(const float* __restrict__ P, float* __restrict__ I, void* G, int ldg,
                                          const Tables& tb) {
  const int tid = threadIdx.x;
  for (int t = tid; t < (FEATURES ? TM * 50 : 0); t += NT) {
    const int a = t % TM, f = t / TM;
    float v = 0.0f;
    if (f < kFam2) {
      v = GM_P0(a, f);
    } else if (f < kFam3) {
      const int p = f - kFam2, s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
#pragma unroll
      for (int i = 0; i < 3; ++i) v += GM_P1(a, s1, i) * GM_P1(a, s2, i);
    } else if (f < kFam4) {
      const int p = f - kFam3, s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
#pragma unroll
      for (int i = 0; i < 9; ++i) v += GM_P2(a, s1, i) * GM_P2(a, s2, i);
    } else {
      const int p = f - kFam4, s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
#pragma unroll
      for (int i = 0; i < 27; ++i) v += GM_P3(a, s1, i) * GM_P3(a, s2, i);
    }
    store_feature<BF16>(G, a * ldg + f, v);
  }
  for (int t = tid; t < (FEATURES ? TM * (kFP - kF) : 0); t += NT)
    store_feature<BF16>(G, (t % TM) * ldg + kF + t / TM, 0.0f);
  // T7
  for (int t = tid; t < TM * 135; t += NT) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, ia = (e % 9) / 3, ib = e % 3;
    const int s2 = tb.pair_s1[p], s3 = tb.pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int cd = 0; cd < 9; ++cd) v += GM_P3(a, s2, ia * 9 + cd) * GM_P3(a, s3, ib * 9 + cd);
    GM_I(a, kT7 + e) = v;
  }
  // V8
  for (int t = tid; t < TM * 75; t += NT) {
    const int a = t % TM, e = t / TM;
    const int s23 = e / 3, i = e % 3;
    const int s2 = s23 / 5, s3 = s23 % 5;
    float v = 0.0f;
#pragma unroll
    for (int bc = 0; bc < 9; ++bc) v += GM_P3(a, s2, i * 9 + bc) * GM_P2(a, s3, bc);
    GM_I(a, kV8 + e) = v;
  }
  // M5
  for (int t = tid; t < TM * 135; t += NT) {
    const int a = t % TM, e = t / TM;
    const int p = e / 9, i = (e % 9) / 3, j = e % 3;
    const int s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) v += GM_P2(a, s1, i * 3 + c) * GM_P2(a, s2, c * 3 + j);
    GM_I(a, kM5 + e) = v;
  }
  // v6
  for (int t = tid; t < TM * 75; t += NT) {
    const int a = t % TM, e = t / TM;
    const int s31 = e / 3, i = e % 3;
    const int s3 = s31 / 5, s1 = s31 % 5;
    float v = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j) v += GM_P2(a, s3, i * 3 + j) * GM_P1(a, s1, j);
    GM_I(a, kV6 + e) = v;
  }
}

// Phase B of the forward: families 5-8 from the intermediates.
template <int TM, int NT, bool BF16>
__device__ inline void contract_forward_b(const float* __restrict__ P, const float* __restrict__ I, void* G, int ldg,
                                          const Tables& tb) {
  const int tid = threadIdx.x;
  for (int t = tid; t < TM * 35; t += NT) {  // fam5: M5[(s1,s2)] : Psi2[s3]
    const int a = t % TM, e = t / TM;
    const int p = tb.pair_index[tb.tri_s1[e] * 5 + tb.tri_s2[e]], s3 = tb.tri_s3[e];
    float v = 0.0f;
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) v += GM_I(a, kM5 + p * 9 + ij) * GM_P2(a, s3, ij);
    store_feature<BF16>(G, a * ldg + kFam5 + e, v);
  }
  for (int t = tid; t < TM * 75; t += NT) {  // fam6: v6[s3][s1] . Psi1[s2]
    const int a = t % TM, e = t / TM;
    const int p = e / 5, s3 = e % 5;
    const int s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += GM_I(a, kV6 + (s3 * 5 + s1) * 3 + i) * GM_P1(a, s2, i);
    store_feature<BF16>(G, a * ldg + kFam6 + e, v);
  }
  for (int t = tid; t < TM * 75; t += NT) {  // fam7: Psi2[s1] : T7[p]
    const int a = t % TM, e = t / TM;
    const int s1 = e / 15, p = e % 15;
    float v = 0.0f;
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) v += GM_P2(a, s1, ij) * GM_I(a, kT7 + p * 9 + ij);
    store_feature<BF16>(G, a * ldg + kFam7 + e, v);
  }
  for (int t = tid; t < TM * 125; t += NT) {  // fam8: Psi1[s1] . V8[s2 s3]
    const int a = t % TM, e = t / TM;
    const int s1 = e / 25, s23 = e % 25;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += GM_P1(a, s1, i) * GM_I(a, kV8 + s23 * 3 + i);
    store_feature<BF16>(G, a * ldg + kFam8 + e, v);
  }
}

#define GM_GB(a, f) Gb[(a) * ldgb + (f)]

// Phase A of the backward: intermediates U8, Y, Qv (read P and dE/dG).
template <int TM, int NT>
__device__ inline void contract_backward_a(const float* __restrict__ P, const float* __restrict__ Gb, int ldgb,
                                           float* __restrict__ I, const Tables& tb) {
  const int tid = threadIdx.x;
  for (int t = tid; t < TM * 225; t += NT) {  // U8
    const int a = t % TM, e = t / TM;
    const int s12 = e / 9, bc = e % 9;
    const int s1 = s12 / 5, s2 = s12 % 5;
    float v = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) v += GM_P1(a, s1, i) * GM_P3(a, s2, i * 9 + bc);
    GM_I(a, kU8 + e) = v;
  }
  for (int t = tid; t < TM * 225; t += NT) {  // Y
    const int a = t % TM, e = t / TM;
    const int xs = e / 9, ab = e % 9;
    const int x = xs / 5, sp = xs % 5;
    const int p = tb.pair_index[x * 5 + sp];
    float v = 0.0f;
#pragma unroll
    for (int s1 = 0; s1 < kS; ++s1) v += GM_GB(a, kFam7 + s1 * 15 + p) * GM_P2(a, s1, ab);
    GM_I(a, kY + e) = (x == sp ? 2.0f : 1.0f) * v;
  }
  for (int t = tid; t < TM * 75; t += NT) {  // Qv
    const int a = t % TM, e = t / TM;
    const int xs = e / 3, i = e % 3;
    const int x = xs / 5, s3 = xs % 5;
    float v = 0.0f;
#pragma unroll
    for (int s1 = 0; s1 < kS; ++s1) v += GM_GB(a, kFam8 + s1 * 25 + x * 5 + s3) * GM_P1(a, s1, i);
    GM_I(a, kQv + e) = v;
  }
}

// Phase B of the backward: every entry of the full-tensor gradient, each
// summing all of its contributions (one writer per entry).
template <int TM, int NT>
__device__ inline void contract_backward_b(const float* __restrict__ P, const float* __restrict__ Gb, int ldgb,
                                           const float* __restrict__ I, float* __restrict__ Pb, const Tables& tb) {
  const int tid = threadIdx.x;
  // Psi0 and Psi1 entries: (x, r), r in 0..3
  for (int t = tid; t < TM * 20; t += NT) {
    const int a = t % TM, e = t / TM;
    const int x = e / 4, r = e % 4;
    float v = 0.0f;
    if (r == 0) {
      v = GM_GB(a, x);
    } else {
      const int i = r - 1;
#pragma unroll
      for (int sp = 0; sp < kS; ++sp) {
        const int p = tb.pair_index[x * 5 + sp];
        const float f2 = (x == sp) ? 2.0f : 1.0f;
        v += f2 * GM_GB(a, kFam2 + p) * GM_P1(a, sp, i);
        float w6 = 0.0f;
#pragma unroll
        for (int s3 = 0; s3 < kS; ++s3) w6 += GM_GB(a, kFam6 + p * 5 + s3) * GM_I(a, kV6 + (s3 * 5 + sp) * 3 + i);
        v += f2 * w6;
      }
      float v8 = 0.0f;
#pragma unroll
      for (int s23 = 0; s23 < 25; ++s23) v8 += GM_GB(a, kFam8 + x * 25 + s23) * GM_I(a, kV8 + s23 * 3 + i);
      v += v8;
    }
    Pb[a * PS + x * kFull + r] = v;
  }
  // Psi2 entries: (x, ij)
  for (int t = tid; t < TM * 45; t += NT) {
    const int a = t % TM, e = t / TM;
    const int x = e / 9, ij = e % 9;
    const int i = ij / 3, j = ij % 3;
    float v = 0.0f;
#pragma unroll
    for (int sp = 0; sp < kS; ++sp)
      v += (x == sp ? 2.0f : 1.0f) * GM_GB(a, kFam3 + tb.pair_index[x * 5 + sp]) * GM_P2(a, sp, ij);
    float v5 = 0.0f, v6 = 0.0f, v7 = 0.0f, v8 = 0.0f;
#pragma unroll
    for (int p = 0; p < 15; ++p) {
      const int s1 = tb.pair_s1[p], s2 = tb.pair_s2[p];
      v5 += tb.c5[x * 15 + p] * GM_GB(a, kFam5 + tb.tri_xp[x * 15 + p]) * GM_I(a, kM5 + p * 9 + ij);
      v6 += GM_GB(a, kFam6 + p * 5 + x) * GM_P1(a, s1, i) * GM_P1(a, s2, j);
      v7 += GM_GB(a, kFam7 + x * 15 + p) * GM_I(a, kT7 + p * 9 + ij);
    }
#pragma unroll
    for (int s12 = 0; s12 < 25; ++s12) v8 += GM_GB(a, kFam8 + s12 * 5 + x) * GM_I(a, kU8 + s12 * 9 + ij);
    v += (v5 + v6) + (v7 + v8);
    Pb[a * PS + x * kFull + 4 + ij] = v;
  }
  // Psi3 entries: (x, i bc)
  for (int t = tid; t < TM * 135; t += NT) {
    const int a = t % TM, e = t / TM;
    const int x = e / 27, ibc = e % 27;
    const int i = ibc / 9, bc = ibc % 9;
    float v = 0.0f;
#pragma unroll
    for (int sp = 0; sp < kS; ++sp) {
      v += (x == sp ? 2.0f : 1.0f) * GM_GB(a, kFam4 + tb.pair_index[x * 5 + sp]) * GM_P3(a, sp, ibc);
#pragma unroll
      for (int d = 0; d < 3; ++d) v += GM_I(a, kY + (x * 5 + sp) * 9 + i * 3 + d) * GM_P3(a, sp, d * 9 + bc);
      v += GM_I(a, kQv + (x * 5 + sp) * 3 + i) * GM_P2(a, sp, bc);
    }
    Pb[a * PS + x * kFull + 13 + ibc] = v;
  }
}

// Fold the full-tensor gradient onto the packed components: out(a, k) for
// k = s*20 + t receives the sum of the full entries packed component t
// stands for.
template <int TM, int NT, typename Out>
__device__ inline void fold_packed(const float* __restrict__ Pb, const Tables& tb, Out out) {
  for (int t = threadIdx.x; t < TM * kS * kPacked; t += NT) {
    const int a = t / (kS * kPacked), e = t % (kS * kPacked);
    const int s = e / kPacked, mp = e % kPacked;
    float v = 0.0f;
    const int n = tb.packed_mult[mp];
    for (int k = 0; k < n; ++k) v += Pb[a * PS + s * kFull + tb.packed_full[mp][k]];
    out(a, e, v);
  }
}

#undef GM_GB
#undef GM_P0
#undef GM_P1
#undef GM_P2
#undef GM_P3
#undef GM_I

}  // namespace gmnn
