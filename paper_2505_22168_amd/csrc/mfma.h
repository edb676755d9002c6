// MFMA tile products and the network stage of a tile (gfx950).
//
// Weight layouts (filled by gmnn_model_prepare), for B = W of shape K x N:
//   BF16, 16x16x32 MFMA: fragment (nb, kb) is 64 lanes x 8 bf16, lane l holding
//     B[32 kb + 8 (l>>4) + e][16 nb + (l&15)], e = 0..7     -> one 16-byte load
//   FP32, 16x16x4 MFMA: chunk (nb, kc) is 64 lanes x 4 floats, lane l holding
//     B[16 kc + 4 (l>>4) + u][16 nb + (l&15)], u = 0..3     -> one 16-byte load
//     feeding four MFMAs (the k order inside a chunk is permuted consistently
//     for A and B, which leaves the product unchanged)
// A tiles live in LDS, row-major, rows padded so 16-byte reads stay aligned.
#pragma once

#include "common.h"
#include "model.h"
#include "tables.h"

namespace gmnn {

// Each wave owns one 16-row block rb and the 16-column blocks nb0 + i*nbs
// (i < TPW, nb < NB).  B fragments stream from L2 through a ring of register
// buffers, prefetch_depth<TPW> k-steps ahead of the MFMAs: 16 fragments
// (64 registers) in flight per wave whatever the width.  The ring of a
// product can be filled ahead of it (ring_fill), e.g. before the epilogue and
// barrier of the previous product, so its first fragments arrive during them.
template <int TPW>
constexpr int prefetch_depth() { return TPW >= 4 ? 4 : 16 / TPW > 8 ? 8 : 16 / TPW; }

template <bool BF16>
struct FragT { using type = bf16x8; };
template <>
struct FragT<false> { using type = floatx4; };  // native vector: kept in registers inside the ring

template <bool BF16, int TPW, int DEPTH = prefetch_depth<TPW>()>
struct BRing {
  static constexpr int PF = DEPTH;
  typename FragT<BF16>::type b[PF][TPW];
};

// k-steps of K: 32 per BF16 fragment, 16 per FP32 chunk (four 16x16x4 MFMAs)
template <bool BF16>
constexpr int ksteps(int K) { return BF16 ? K / 32 : K / 16; }

template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void ring_load(BRing<BF16, TPW, DEPTH>& r, int slot, const void* Bp, int KB, int kb, int nb0, int nbs,
                                 int NB) {
  using F = typename FragT<BF16>::type;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int nb = nb0 + i * nbs;
    if (nb < NB && kb < KB) r.b[slot][i] = ((const F*)Bp)[((size_t)nb * KB + kb) * 64 + l];
  }
}

// issue the first PF k-steps of the product with B = (Bbf or Bf) of K rows
template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void ring_fill(BRing<BF16, TPW, DEPTH>& r, const void* Bbf, const void* Bf, int K, int nb0, int nbs,
                                 int NB) {
  const void* Bp = BF16 ? Bbf : Bf;
#pragma unroll
  for (int s = 0; s < DEPTH; ++s) ring_load(r, s, Bp, ksteps<BF16>(K), s, nb0, nbs, NB);
}

// acc += A[rb rows] B over K, with the ring already holding k-steps 0..PF-1
template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void mma_ring(BRing<BF16, TPW, DEPTH>& r, const void* A, int lda, int rb, const void* Bbf,
                                         const void* Bf, int K, int nb0, int nbs, int NB, floatx4 (&acc)[TPW]) {
  constexpr int PF = DEPTH;
  const int l = threadIdx.x & 63;
  const void* Bp = BF16 ? Bbf : Bf;
  const int KB = ksteps<BF16>(K);
  auto step = [&](int slot, int kb) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb >= NB) continue;
      if constexpr (BF16) {
        const bf16x8 a = *(const bf16x8*)((const __bf16*)A + (rb * 16 + (l & 15)) * lda + (l >> 4) * 8 + kb * 32);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, r.b[slot][i], acc[i], 0, 0, 0);
      } else {
        const floatx4 a = *(const floatx4*)((const float*)A + (rb * 16 + (l & 15)) * lda + (l >> 4) * 4 + kb * 16);
        const floatx4 bb = r.b[slot][i];
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], bb[0], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], bb[1], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], bb[2], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], bb[3], acc[i], 0, 0, 0);
      }
    }
  };
  for (int kb = 0; kb < KB; kb += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      if (kb + s < KB) {
        step(s, kb + s);
        ring_load(r, s, Bp, KB, kb + s + PF, nb0, nbs, NB);
      }
    }
  }
}

// the same product with the ring filled on the spot (FP32 only: the training tile)
template <int TPW>
__device__ inline void mma_f32(const float* __restrict__ A, int lda, int rb, const float4* __restrict__ Bp, int KC,
                               int nb0, int nbs, int NB, floatx4 (&acc)[TPW]) {
  BRing<false, TPW> r;
  ring_fill(r, nullptr, Bp, KC * 16, nb0, nbs, NB);
  mma_ring(r, A, lda, rb, nullptr, Bp, KC * 16, nb0, nbs, NB, acc);
}

// BF16 product with the A tile kept in FP32 in LDS: the 8 values of each A
// fragment are rounded to BF16 (nearest even) as they are loaded (the
// training tile keeps its activations in FP32 for the parameter products).
// The _ring form takes the ring already holding k-steps 0..PF-1 (filled ahead
// with ring_fill), so its first fragments can arrive during earlier work.
template <int TPW, int DEPTH>
__device__ __forceinline__ void mma_bf16_a32_ring(BRing<true, TPW, DEPTH>& r, const float* __restrict__ A, int lda,
                                                  int rb, const bf16x8* __restrict__ Bp, int K, int nb0, int nbs,
                                                  int NB, floatx4 (&acc)[TPW]) {
  constexpr int PF = DEPTH;
  const int l = threadIdx.x & 63;
  const int KB = K / 32;
  const float* arow = A + (rb * 16 + (l & 15)) * lda + (l >> 4) * 8;
  auto step = [&](int slot, int kb) {
    const float4 lo = *(const float4*)(arow + kb * 32);
    const float4 hi = *(const float4*)(arow + kb * 32 + 4);
    bf16x8 a;
    a[0] = (__bf16)lo.x; a[1] = (__bf16)lo.y; a[2] = (__bf16)lo.z; a[3] = (__bf16)lo.w;
    a[4] = (__bf16)hi.x; a[5] = (__bf16)hi.y; a[6] = (__bf16)hi.z; a[7] = (__bf16)hi.w;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, r.b[slot][i], acc[i], 0, 0, 0);
    }
  };
  for (int kb = 0; kb < KB; kb += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      if (kb + s < KB) {
        step(s, kb + s);
        ring_load(r, s, Bp, KB, kb + s + PF, nb0, nbs, NB);
      }
    }
  }
}

template <int TPW>
__device__ __forceinline__ void mma_bf16_a32(const float* __restrict__ A, int lda, int rb,
                                             const bf16x8* __restrict__ Bp, int K, int nb0, int nbs, int NB,
                                             floatx4 (&acc)[TPW]) {
  BRing<true, TPW> r;
  ring_fill(r, Bp, nullptr, K, nb0, nbs, NB);
  mma_bf16_a32_ring(r, A, lda, rb, Bp, K, nb0, nbs, NB, acc);
}

// ---------------------------------------------------------------------------
// Split-BF16 products (the network's forward products in BF16 mode).  Each
// FP32 operand x is held as two bf16 parts, hi = bf16(x) and lo = bf16(x - hi)
// (x - hi is exact in FP32), and
//   acc += Ahi Bhi + Ahi Blo + Alo Bhi        (per k-step, in this order)
// keeps about 16 significant bits of every operand; the dropped Alo Blo term
// is 2^-16 relative.  Three BF16 MFMAs per k-step instead of one, FP32
// accumulation.  The A parts live in LDS (high and low parts in two arrays
// of the same layout); the B fragments stream through a ring whose slot i < TPW
// holds the high fragment of column block nb0 + i nbs and slot TPW + i its
// low fragment (same fragment layout, separate arrays).
template <bool BF16, int TPW, int DEPTH>
struct FwdRingT {
  using type = BRing<false, TPW, DEPTH>;
};
template <int TPW, int DEPTH>
struct FwdRingT<true, TPW, DEPTH> {
  using type = BRing<true, 2 * TPW, (DEPTH / 2 > 0 ? DEPTH / 2 : 1)>;
};
template <bool BF16, int TPW, int DEPTH>
using FwdRing = typename FwdRingT<BF16, TPW, DEPTH>::type;

template <int TPW, int SD>
__device__ __forceinline__ void split_ring_load(BRing<true, 2 * TPW, SD>& r, int slot, const bf16x8* Bhi,
                                                const bf16x8* Blo, int KB, int kb, int nb0, int nbs, int NB) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int nb = nb0 + i * nbs;
    if (nb < NB && kb < KB) {
      const size_t o = ((size_t)nb * KB + kb) * 64 + l;
      r.b[slot][i] = Bhi[o];
      r.b[slot][TPW + i] = Blo[o];
    }
  }
}

// first k-steps of a forward product: split fragments (BF16) or FP32 chunks
template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void fwd_ring_fill(FwdRing<BF16, TPW, DEPTH>& r, const bf16x8* Bhi, const bf16x8* Blo,
                                              const float* Bf, int K, int nb0, int nbs, int NB) {
  if constexpr (BF16) {
    constexpr int SD = DEPTH / 2 > 0 ? DEPTH / 2 : 1;
#pragma unroll
    for (int s = 0; s < SD; ++s) split_ring_load<TPW, SD>(r, s, Bhi, Blo, K / 32, s, nb0, nbs, NB);
  } else {
    ring_fill(r, nullptr, Bf, K, nb0, nbs, NB);
  }
}

// acc += A B for a forward product: split-BF16 (bf16 parts of A at A and
// Alo) or plain FP32 (A; Alo unused)
template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void fwd_mma(FwdRing<BF16, TPW, DEPTH>& r, const void* A, const void* Alo, int lda, int rb,
                                        const bf16x8* Bhi, const bf16x8* Blo, const float* Bf, int K, int nb0,
                                        int nbs, int NB, floatx4 (&acc)[TPW]) {
  if constexpr (BF16) {
    constexpr int SD = DEPTH / 2 > 0 ? DEPTH / 2 : 1;
    const int l = threadIdx.x & 63;
    const int KB = K / 32;
    const int aoff = (rb * 16 + (l & 15)) * lda + (l >> 4) * 8;
    const __bf16* ahi = (const __bf16*)A + aoff;
    const __bf16* alo_p = (const __bf16*)Alo + aoff;
    auto step = [&](int slot, int kb) {
      const bf16x8 ah = *(const bf16x8*)(ahi + kb * 32);
      const bf16x8 al = *(const bf16x8*)(alo_p + kb * 32);
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int nb = nb0 + i * nbs;
        if (nb >= NB) continue;
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, r.b[slot][i], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, r.b[slot][TPW + i], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, r.b[slot][i], acc[i], 0, 0, 0);
      }
    };
    for (int kb = 0; kb < KB; kb += SD) {
#pragma unroll
      for (int s = 0; s < SD; ++s) {
        if (kb + s < KB) {
          step(s, kb + s);
          split_ring_load<TPW, SD>(r, s, Bhi, Blo, KB, kb + s + SD, nb0, nbs, NB);
        }
      }
    }
  } else {
    mma_ring(r, A, lda, rb, nullptr, Bf, K, nb0, nbs, NB, acc);
  }
}

// store of a forward activation: FP32 (base), or its bf16 high part (base)
// and low part (lo, same layout)
template <bool BF16>
__device__ inline void st_split(void* base, void* lo, int idx, float v) {
  if constexpr (BF16) {
    const __bf16 h = (__bf16)v;
    ((__bf16*)base)[idx] = h;
    ((__bf16*)lo)[idx] = (__bf16)split_low(v, h);
  } else {
    ((float*)base)[idx] = v;
  }
}

template <int TPW>
__device__ inline void zero_acc(floatx4 (&acc)[TPW]) {
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
}

// swish(z) = z sigmoid(z) and its derivative; the sigmoid takes the hardware
// reciprocal (1 ulp) instead of a correctly rounded division, a ten-
// instruction sequence per activation in the VALU-bound network epilogues
__device__ inline float swish_parts(float z, float& dsw) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
  dsw = s * (1.0f + z * (1.0f - s));
  return z * s;
}

template <bool BF16>
__device__ inline void st_act(void* base, int idx, float v) {
  if (BF16) ((__bf16*)base)[idx] = (__bf16)v;
  else ((float*)base)[idx] = v;
}

// LDS row strides of the network tiles (elements)
template <int HP, bool BF16>
struct NetStrides {
  static constexpr int G = BF16 ? (kFP + 8) : (kFP + 4);   // invariants (A of the first product)
  static constexpr int H = BF16 ? (HP + 8) : (HP + 4);     // h1 / delta2 / delta1
  static constexpr int GB = kFP + 1;                       // dE/dG (FP32)
};

template <int TM, int HP, int NW>
struct NetShape {
  static constexpr int MB = TM / 16;                 // 16-row blocks
  static constexpr int WPR = NW / MB;                // waves per row block
  static constexpr int NBH = HP / 16;                // 16-column blocks of a hidden layer
  static constexpr int NBG = kFP / 16;               // ... of the invariants
  static constexpr int TPW = (NBH + WPR - 1) / WPR;  // column blocks per wave (hidden)
  static constexpr int TPW_G = (NBG + WPR - 1) / WPR;
};

// Network forward for the TM rows of a tile (all NW waves):
//   z1 = G W1 + b1, h1 = swish(z1); z2 = h1 W2 + b2, h2 = swish(z2);
//   y_m = h2 . W3[:,m] + b3[m], E_m = sigma y_m + mu  (written for rows < n_rows,
//   also to sEa[row][m] in LDS when sEa is not null)
// sG: invariants (read).  sH: h1 out.  swish'(z1) is returned in dsw1 (the
// backward product hands each wave exactly these output fragments again).
// MEAN: delta2 = swish'(z2) sigma mean_m W3[:,m] -> sD2 (the head-mean
// backward); otherwise swish'(z2) -> sDsw2 (FP32, row stride HP + 1) for
// per-head backwards.  sEp: [NW][16][kMaxHeads] partial sums.
// BF16 mode: both forward products are split-BF16 (fwd_mma), with the low
// parts of G at sGlo and of h1 at sHlo; fring holds the first k-steps of W1
// on entry.  sHlo may overlap sG and sD2 (the tile keeps h1's low part where
// G was and delta2 goes): barriers after each forward product's MFMAs keep
// those stores behind every wave's reads.  The backward products stay plain
// BF16: the first k-steps of W2^T are issued into `ring` before the second
// epilogue.
template <int TM, int HP, bool BF16, int NW, bool MEAN, int DEPTH>
__device__ __forceinline__ void network_forward(const DevModel& m, const void* sG, const void* sGlo, void* sH,
                                       void* sHlo, void* sD2, float* sDsw2,
                                       float* sEp, const float* sScale, const float* sShift, const int* sStruct,
                                       int row0, int n_rows,
                                       float* __restrict__ atomic_e, float* sEa,
                                       floatx4 (&dsw1)[NetShape<TM, HP, NW>::TPW],
                                       FwdRing<BF16, NetShape<TM, HP, NW>::TPW, DEPTH>& fring,
                                       BRing<BF16, NetShape<TM, HP, NW>::TPW, DEPTH>& ring) {
  using St = NetStrides<HP, BF16>;
  using Sh = NetShape<TM, HP, NW>;
  constexpr int MB = Sh::MB, WPR = Sh::WPR, NBH = Sh::NBH, TPW = Sh::TPW;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int rb = w % MB, cw = w / MB;
  const int M = m.M;
  // per-column epilogue constants of this wave, loaded ahead of the products
  float b1v[TPW], b2v[TPW], wbv[TPW], w30[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int nb = cw + i * WPR;
    const int col = (nb < NBH ? nb : 0) * 16 + (l & 15);
    b1v[i] = m.b1[col];
    b2v[i] = m.b2[col];
    wbv[i] = m.w3bar[col];
    w30[i] = m.w3[col * M];
  }
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    fwd_mma<BF16, TPW, DEPTH>(fring, sG, sGlo, St::G, rb, m.w1_bf16, m.w1lo_bf16, m.w1_f32, kFP, cw, WPR, NBH, acc);
    fwd_ring_fill<BF16, TPW, DEPTH>(fring, m.w2_bf16, m.w2lo_bf16, m.w2_f32, HP, cw, WPR, NBH);
    if (BF16) __syncthreads();  // every wave is done with G before h1's low part is stored
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBH) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (l >> 4) + j;
        float d;
        const float hv = swish_parts(acc[i][j] + b1v[i], d);
        dsw1[i][j] = d;
        st_split<BF16>(sH, sHlo, row * St::H + col, hv);
      }
    }
  }
  __syncthreads();
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    fwd_mma<BF16, TPW, DEPTH>(fring, sH, sHlo, St::H, rb, m.w2_bf16, m.w2lo_bf16, m.w2_f32, HP, cw, WPR, NBH, acc);
    // the backward's first product (W2^T) starts loading now
    ring_fill(ring, m.w2t_bf16, m.w2t_f32, HP, cw, WPR, NBH);
    if (BF16) __syncthreads();  // every wave is done with h1's low part before delta2 is stored
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBH) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (l >> 4) + j;
        float d;
        const float hv = swish_parts(acc[i][j] + b2v[i], d);
        acc[i][j] = hv;
        if (m.h2_out && row < n_rows) m.h2_out[(int64_t)(row0 + row) * HP + col] = hv;
        if (MEAN)
          st_act<BF16>(sD2, row * St::H + col,
                       d * sScale[row] * (m.head_w ? m.head_w[(int64_t)sStruct[row] * HP + col] : wbv[i]));
        else sDsw2[row * (HP + 1) + col] = d;
      }
    }
    for (int hm = 0; hm < M; ++hm) {
      float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int nb = cw + i * WPR;
        if (nb >= NBH) continue;
        const float w3 = hm == 0 ? w30[i] : m.w3[(nb * 16 + (l & 15)) * M + hm];
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] += acc[i][j] * w3;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = part[j];
        v = row16_rot_sum(v);  // lane 0 of the row: the xor-butterfly sum
        if ((l & 15) == 0) sEp[(w * 16 + 4 * (l >> 4) + j) * kMaxHeads + hm] = v;
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < TM * M; t += NW * 64) {
    const int a = t / M, hm = t % M;
    if (a < n_rows) {
      float y = m.b3[hm];
#pragma unroll
      for (int ww = 0; ww < NW; ++ww)
        if (ww % MB == a / 16) y += sEp[(ww * 16 + a % 16) * kMaxHeads + hm];
      const float e = sScale[a] * y + sShift[a];
      atomic_e[(int64_t)(row0 + a) * M + hm] = e;
      if (sEa) sEa[a * M + hm] = e;
    }
  }
}

// delta2 of head `hm`: swish'(z2) sigma W3[:,hm] -> sD2
template <int TM, int HP, bool BF16, int NW>
__device__ __forceinline__ void network_delta2_head(const DevModel& m, const float* sDsw2, const float* sScale, void* sD2,
                                           int hm) {
  using St = NetStrides<HP, BF16>;
  for (int t = threadIdx.x; t < TM * HP; t += NW * 64) {
    const int row = t / HP, col = t % HP;
    st_act<BF16>(sD2, row * St::H + col, sDsw2[row * (HP + 1) + col] * sScale[row] * m.w3[col * m.M + hm]);
  }
}

// Network backward given delta2 in sD2 and the ring holding the first k-steps
// of W2^T: delta1 = swish'(z1) (delta2 W2^T) -> sH, dE/dG = delta1 W1^T ->
// sGb (FP32).  Ends with a barrier.
template <int TM, int HP, bool BF16, int NW, int DEPTH>
__device__ __forceinline__ void network_backward(const DevModel& m, const void* sD2, void* sH, float* sGb,
                                        const floatx4 (&dsw1)[NetShape<TM, HP, NW>::TPW],
                                        BRing<BF16, NetShape<TM, HP, NW>::TPW, DEPTH>& ring) {
  using St = NetStrides<HP, BF16>;
  using Sh = NetShape<TM, HP, NW>;
  constexpr int MB = Sh::MB, WPR = Sh::WPR, NBH = Sh::NBH, NBG = Sh::NBG, TPW = Sh::TPW, TPW_G = Sh::TPW_G;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int rb = w % MB, cw = w / MB;
  BRing<BF16, TPW_G, (DEPTH < prefetch_depth<TPW_G>() ? DEPTH : prefetch_depth<TPW_G>())> ring_g;
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    mma_ring(ring, sD2, St::H, rb, m.w2t_bf16, m.w2t_f32, HP, cw, WPR, NBH, acc);
    ring_fill(ring_g, m.w1t_bf16, m.w1t_f32, HP, cw, WPR, NBG);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBH) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (l >> 4) + j;
        st_act<BF16>(sH, row * St::H + col, acc[i][j] * dsw1[i][j]);
      }
    }
  }
  __syncthreads();
  {
    floatx4 acc[TPW_G];
    zero_acc(acc);
    mma_ring(ring_g, sH, St::H, rb, m.w1t_bf16, m.w1t_f32, HP, cw, WPR, NBG, acc);
#pragma unroll
    for (int i = 0; i < TPW_G; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBG) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (l >> 4) + j;
        sGb[row * St::GB + col] = acc[i][j];
      }
    }
  }
  __syncthreads();
}

}  // namespace gmnn
