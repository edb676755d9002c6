// Streamed readout for large systems (three launches instead of the tile):
//
//   readout_features  invariants of the moments (Section 2.1, eq.
//                     contraction), 16 atoms per block -> G [N][384] in HBM
//                     (FP32, or for the BF16 network its bf16 high parts
//                     [N][384] followed by the low parts [N][384])
//   readout_network   the network, its scale/shift (eq. scale_shift) and its
//                     input gradient dE/dG, for row tiles of 32 to 64 atoms:
//                     every weight fragment fetched from L2 feeds 2 to 4 MFMA
//                     row blocks, 1/2 to 1/4 of the L2 traffic per atom of
//                     the 16-row tile
//   readout_backward  product-rule backward of the invariants, 8 atoms per
//                     block -> dE/dPsi [N][100]
//
// The arithmetic is the tile's, operation for operation (same contraction
// code, same MFMA shapes and k order, same epilogues), so both give the same
// result up to FP32 summation order.
#include "common.h"
#include "contraction.h"
#include "mfma.h"
#include "model.h"

namespace gmnn {

// invariant blocks: 6 atoms and 256 threads (about 25 KB of LDS: six
// blocks per CU, whose load and barrier waits overlap one another; the
// arithmetic of an atom's invariants does not depend on the block size)
constexpr int kRoAtoms = 6;      // atoms per invariant (features) block
constexpr int kFtThreads = 256;  // threads of an invariant block
constexpr int kRoThreads = 512;  // threads of a network block
constexpr int kRoWaves = kRoThreads / 64;

static constexpr size_t ro_al(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// shared: the tile's packed moments (one contiguous run) -> full tensors
__device__ inline void ro_load_moments(const float* __restrict__ psi, int row0, int n_rows, float* __restrict__ sPsi,
                                       const Tables& tb) {
  constexpr int NP = kS * kPacked;
  constexpr int NU = (kRoAtoms * NP + kFtThreads - 1) / kFtThreads;
  const int tid = threadIdx.x;
  float v[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = tid + u * kFtThreads;
    v[u] = t < n_rows * NP ? psi[(int64_t)row0 * NP + t] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = tid + u * kFtThreads;
    if (t < kRoAtoms * NP) {
      const int a = t / NP, e = t % NP;
      const int s = e / kPacked, c = e % kPacked;
      const int n = tb.packed_mult[c];
      for (int q = 0; q < n; ++q) sPsi[a * PS + s * kFull + tb.packed_full[c][q]] = v[u];
    }
  }
}

// ---------------------------------------------------------------------------
// 1. invariants
template <bool BF16>
struct FeatLds {
  static constexpr int ESZ = BF16 ? 2 : 4;
  static constexpr size_t tables = 0;
  static constexpr size_t psi = ro_al(sizeof(Tables));
  static constexpr size_t inter = psi + ro_al(4 * (size_t)kRoAtoms * PS);
  static constexpr size_t g = inter + ro_al(4 * (size_t)kRoAtoms * ISF);
  static constexpr size_t bytes = g + ro_al((BF16 ? 2 : 1) * (size_t)ESZ * kRoAtoms * kFP);
};

template <bool BF16>
__global__ void __launch_bounds__(kFtThreads) readout_features(DevSystem sys, const float* __restrict__ psi,
                                                               void* __restrict__ G) {
  using L = FeatLds<BF16>;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Tables& tb = *(Tables*)(lds + L::tables);
  float* sPsi = (float*)(lds + L::psi);
  float* sI = (float*)(lds + L::inter);
  char* sG = lds + L::g;
  const int row0 = xcd_block(blockIdx.x, gridDim.x) * kRoAtoms;
  const int n_rows = min(kRoAtoms, sys.n_atoms - row0);
  load_tables(&tb);
  __syncthreads();
  ro_load_moments(psi, row0, n_rows, sPsi, tb);
  __syncthreads();
  constexpr int glo = BF16 ? kRoAtoms * kFP : 0;  // low parts after the high ones
  // the first pass runs each task's two independent halves on two threads
  // when the block has threads for both (no change to any arithmetic)
  constexpr int KSF = 2 * ((kRoAtoms * 20 + 63) / 64 * 64) <= kFtThreads ? 2 : 1;
  contract_forward_a<kRoAtoms, kFtThreads, BF16, true, ISF, KSF>(sPsi, sI, sG, kFP, tb, glo);
  __syncthreads();
  contract_forward_b<kRoAtoms, kFtThreads, BF16, ISF>(sPsi, sI, sG, kFP, tb, glo);
  __syncthreads();
  // rows of G are contiguous: 16-byte copies (BF16: the high plane, then the
  // low plane N rows further)
  const int n16 = n_rows * kFP * L::ESZ / 16;
  uint4* dst = (uint4*)((char*)G + (size_t)row0 * kFP * L::ESZ);
  for (int t = threadIdx.x; t < n16; t += kFtThreads) dst[t] = ((const uint4*)sG)[t];
  if (BF16) {
    uint4* dlo = (uint4*)((char*)G + ((size_t)sys.n_atoms + row0) * kFP * L::ESZ);
    const uint4* slo = (const uint4*)(sG + (size_t)glo * L::ESZ);
    for (int t = threadIdx.x; t < n16; t += kFtThreads) dlo[t] = slo[t];
  }
}

// ---------------------------------------------------------------------------
// 2. network on row tiles of TM atoms.  Wave w owns the 16-column blocks
// w, w + 8, ... of every product, for all TM/16 row blocks; each weight
// fragment loaded from L2 feeds TM/16 MFMAs.  Every product runs transposed:
// the weight fragment is the MFMA's A operand and the activation fragment
// its B operand (the A and B fragment layouts of the 16x16x32 BF16 and
// 16x16x4 FP32 MFMAs coincide, so the packed weights and the LDS reads are
// those of the plain orientation).  A lane's accumulator then holds four
// consecutive hidden units (or features) of one atom, and every epilogue
// store is one 8-byte (BF16) or 16-byte (FP32) write instead of four
// scattered ones.  The block's barriers order LDS only (lds_barrier), so
// the weight fragments prefetched for the next product stay in flight
// through them.
constexpr int kPfPlain = 3;  // k-steps of B in flight, plain BF16 products (measured best on the 2x512 network)
constexpr int kPfSplit = 2;  // k-steps of B (high and low fragments) in flight, split products

// the first kPfPlain k-steps of a plain product's B fragments, issued ahead
// of the product (their latency then overlaps the previous phase)
template <int TPW>
__device__ inline void plain_pre(bf16x8 (&b)[kPfPlain][TPW], const bf16x8* __restrict__ Bp, int KB, int nb0, int nbs,
                                 int NB) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < kPfPlain; ++s)
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB && s < KB) b[s][i] = Bp[((size_t)nb * KB + s) * 64 + l];
    }
}

// the same for a split product (high and low parts, kPfSplit k-steps)
template <int TPW>
__device__ inline void split_pre(bf16x8 (&bh)[kPfSplit][TPW], bf16x8 (&bl)[kPfSplit][TPW],
                                 const bf16x8* __restrict__ Bhi, const bf16x8* __restrict__ Blo, int KB, int nb0,
                                 int nbs, int NB) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < kPfSplit; ++s)
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB && s < KB) {
        const size_t o = ((size_t)nb * KB + s) * 64 + l;
        bh[s][i] = Bhi[o];
        bl[s][i] = Blo[o];
      }
    }
}

// plain BF16 rows product, acc += A B, with b holding the first kPfPlain
// k-steps (plain_pre)
template <int MB, int TPW>
__device__ inline void mma_rows_bf16(const __bf16* __restrict__ A, int lda, const bf16x8* __restrict__ Bp, int KB,
                                     int nb0, int nbs, int NB, floatx4 (&acc)[MB][TPW],
                                     bf16x8 (&b)[kPfPlain][TPW]) {
  constexpr int PF = kPfPlain;
  const int l = threadIdx.x & 63;
  const __bf16* abase = A + (l & 15) * lda + (l >> 4) * 8;
  auto load = [&](bf16x8 (&dst)[TPW], int kb) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB && kb < KB) dst[i] = Bp[((size_t)nb * KB + kb) * 64 + l];
    }
  };
  auto step = [&](const bf16x8 (&bb)[TPW], int kb) {
    bf16x8 a[MB];
#pragma unroll
    for (int r = 0; r < MB; ++r) a[r] = *(const bf16x8*)(abase + r * 16 * lda + kb * 32);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB)
#pragma unroll
        for (int r = 0; r < MB; ++r) acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb[i], a[r], acc[r][i], 0, 0, 0);
    }
  };
  for (int kb = 0; kb < KB; kb += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      if (kb + s < KB) {
        step(b[s], kb + s);
        load(b[s], kb + s + PF);
      }
    }
  }
}

// split-BF16 rows product (the forward products of the BF16 network):
// acc += Ahi Bhi + Ahi Blo + Alo Bhi per k-step, in the order of fwd_mma,
// with the low part of A at A + alo elements
// (bh, bl hold the first kPfSplit k-steps: split_pre)
template <int MB, int TPW>
__device__ inline void mma_rows_split(const __bf16* __restrict__ A, int alo, int lda, const bf16x8* __restrict__ Bhi,
                                      const bf16x8* __restrict__ Blo, int KB, int nb0, int nbs, int NB,
                                      floatx4 (&acc)[MB][TPW], bf16x8 (&bh)[kPfSplit][TPW],
                                      bf16x8 (&bl)[kPfSplit][TPW]) {
  constexpr int PF = kPfSplit;
  const int l = threadIdx.x & 63;
  const __bf16* abase = A + (l & 15) * lda + (l >> 4) * 8;
  auto load = [&](bf16x8 (&dh)[TPW], bf16x8 (&dl)[TPW], int kb) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB && kb < KB) {
        const size_t o = ((size_t)nb * KB + kb) * 64 + l;
        dh[i] = Bhi[o];
        dl[i] = Blo[o];
      }
    }
  };
  auto step = [&](const bf16x8 (&h)[TPW], const bf16x8 (&lo)[TPW], int kb) {
    // one row block's A parts at a time (fewer registers live)
#pragma unroll
    for (int r = 0; r < MB; ++r) {
      const bf16x8 ah = *(const bf16x8*)(abase + r * 16 * lda + kb * 32);
      const bf16x8 al = *(const bf16x8*)(abase + alo + r * 16 * lda + kb * 32);
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int nb = nb0 + i * nbs;
        if (nb >= NB) continue;
        acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[i], ah, acc[r][i], 0, 0, 0);
        acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[i], ah, acc[r][i], 0, 0, 0);
        acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[i], al, acc[r][i], 0, 0, 0);
      }
    }
  };
  for (int kb = 0; kb < KB; kb += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      if (kb + s < KB) {
        step(bh[s], bl[s], kb + s);
        load(bh[s], bl[s], kb + s + PF);
      }
    }
  }
}

template <int MB, int TPW>
__device__ inline void mma_rows_f32(const float* __restrict__ A, int lda, const float4* __restrict__ Bp, int KC,
                                    int nb0, int nbs, int NB, floatx4 (&acc)[MB][TPW]) {
  constexpr int PF = 2;
  const int l = threadIdx.x & 63;
  const float* abase = A + (l & 15) * lda + (l >> 4) * 4;
  float4 b[PF][TPW];
  auto load = [&](float4 (&dst)[TPW], int kc) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB && kc < KC) dst[i] = Bp[((size_t)nb * KC + kc) * 64 + l];
    }
  };
  auto step = [&](const float4 (&bb)[TPW], int kc) {
    float4 a[MB];
#pragma unroll
    for (int r = 0; r < MB; ++r) a[r] = *(const float4*)(abase + r * 16 * lda + kc * 16);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = nb0 + i * nbs;
      if (nb < NB)
#pragma unroll
        for (int r = 0; r < MB; ++r) {
          acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[i].x, a[r].x, acc[r][i], 0, 0, 0);
          acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[i].y, a[r].y, acc[r][i], 0, 0, 0);
          acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[i].z, a[r].z, acc[r][i], 0, 0, 0);
          acc[r][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[i].w, a[r].w, acc[r][i], 0, 0, 0);
        }
    }
  };
#pragma unroll
  for (int s = 0; s < PF; ++s) load(b[s], s);
  for (int kc = 0; kc < KC; kc += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      if (kc + s < KC) {
        step(b[s], kc + s);
        load(b[s], kc + s + PF);
      }
    }
  }
}

template <int MB, int TPW>
__device__ inline void zero_rows(floatx4 (&acc)[MB][TPW]) {
#pragma unroll
  for (int r = 0; r < MB; ++r)
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[r][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
}

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

// four consecutive activations of one row: FP32, or BF16 (high parts at
// base, and with LO the low parts bf16(v - bf16(v)) at lo)
template <bool BF16, bool LO = false>
__device__ inline void st4(void* base, void* lo, int idx, floatx4 v) {
  if constexpr (BF16) {
    bf16x4 h, t;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h[j] = (__bf16)v[j];
      if constexpr (LO) t[j] = (__bf16)split_low(v[j], h[j]);
    }
    *(bf16x4*)((__bf16*)base + idx) = h;
    if constexpr (LO) *(bf16x4*)((__bf16*)lo + idx) = t;
  } else {
    *(floatx4*)((float*)base + idx) = v;
  }
}

// rows per network block: as many 16-row MFMA blocks as the register file
// holds with swish'(z1) kept for the backward (8 waves, 256 registers each)
template <int HP, bool BF16>
constexpr int net_rows() { return BF16 ? (HP >= 512 ? 48 : 64) : 32; }

template <int HP, bool BF16>
struct NetLds {
  using St = NetStrides<HP, BF16>;
  static constexpr int TM = net_rows<HP, BF16>();
  static constexpr int ESZ = BF16 ? 2 : 4;
  static constexpr int NS = BF16 ? 2 : 1;  // parts of a forward operand (bf16 high and low)
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
  // region B: delta2; the row scale/shift; region A: G (all parts), then h1
  // (all parts), then delta1 at its start and the per-wave energy partials
  // [NW][TM][M] right after delta1 (sized by M)
  static constexpr int GLO = TM * St::G;  // element offsets of the low parts in region A
  static constexpr int HLO = TM * St::H;
  static constexpr size_t b = 0;
  static constexpr size_t rows = b + ro_al((size_t)ESZ * TM * St::H);
  static constexpr size_t a = rows + ro_al(4 * 3 * (size_t)TM);  // scale, shift, structure of each row
  static constexpr size_t ep = a + ro_al((size_t)ESZ * TM * St::H);
  static constexpr size_t bytes(int M) {
    return mx(a + ro_al((size_t)ESZ * NS * mx((size_t)TM * St::G, (size_t)TM * St::H)),
              ep + ro_al(4 * (size_t)kRoWaves * TM * M));
  }
};

template <int HP, bool BF16>
__global__ void __launch_bounds__(kRoThreads)
    readout_network(DevModel m, DevSystem sys, const void* __restrict__ G, float* __restrict__ atomic_e,
                    float* __restrict__ dG) {
  using L = NetLds<HP, BF16>;
  using St = NetStrides<HP, BF16>;
  constexpr int TM = L::TM, MB = TM / 16, NW = kRoWaves;
  constexpr int NBH = HP / 16, NBG = kFP / 16;
  constexpr int TPW = (NBH + NW - 1) / NW, TPW_G = (NBG + NW - 1) / NW;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  char* sA = lds + L::a;
  char* sB = lds + L::b;
  float* sEp = (float*)(lds + L::ep);
  float* sScale = (float*)(lds + L::rows);
  float* sShift = sScale + TM;
  int* sStruct = (int*)(sShift + TM);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int row0 = xcd_block(blockIdx.x, gridDim.x) * TM;
  const int n_rows = min(TM, sys.n_atoms - row0);
  const int M = m.M;
  // a lane's accumulator entries j = 0..3 of a 16 x 16 block: unit (or
  // feature) uq + j of the column block, atom ar of the row block
  const int ar = l & 15, uq = 4 * (l >> 4);

  // BF16: the B fragments of each product's first k-steps are issued one
  // phase ahead (W1's with the tile's G rows, W2's before the first
  // epilogue, W2^T's and W1^T's before the second and third), so their
  // latency overlaps loads, barriers and epilogues instead of the products
  bf16x8 ph[kPfSplit][TPW], pl[kPfSplit][TPW];
  bf16x8 pb[kPfPlain][TPW], pg[kPfPlain][TPW_G];

  // G rows (each part) -> region A (row stride St::G), zero rows beyond the
  // system; every load of the tile is issued before the first store
  {
    constexpr int C16 = kFP * L::ESZ / 16;  // 16-byte chunks per row
    constexpr int NU = (L::NS * TM * C16 + kRoThreads - 1) / kRoThreads;
    const char* gbase = (const char*)G;
    uint4 v[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kRoThreads;
      const int part = t / (TM * C16), tt = t % (TM * C16);
      v[u] = uint4{0u, 0u, 0u, 0u};
      if (part < L::NS && tt < n_rows * C16)
        v[u] = ((const uint4*)(gbase + ((size_t)part * sys.n_atoms + row0) * kFP * L::ESZ))[tt];
    }
    // W1's first k-steps after the tile's rows: the LDS stores below wait
    // for the rows only
    if constexpr (BF16) split_pre<TPW>(ph, pl, m.w1_bf16, m.w1lo_bf16, kFP / 32, w, NW, NBH);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kRoThreads;
      const int part = t / (TM * C16), tt = t % (TM * C16);
      if (part < L::NS)
        *(uint4*)(sA + ((size_t)part * L::GLO + (size_t)(tt / C16) * St::G) * L::ESZ + (tt % C16) * 16) = v[u];
    }
    for (int a = tid; a < TM; a += kRoThreads) {
      float sc = 0.0f, sh = 0.0f;
      int b = 0;
      if (a < n_rows) {
        const int z = sys.species[row0 + a];
        sc = m.scale[z];
        sh = m.shift[z];
        b = sys.atom_struct[row0 + a];
      }
      sScale[a] = sc;
      sShift[a] = sh;
      sStruct[a] = b;
    }
  }
  lds_barrier();

  // z1 = G W1 + b1 (split-BF16 or FP32), h1 = swish(z1) -> region A once every
  // wave is done with G; swish'(z1) stays in registers
  floatx4 dsw1[MB][TPW];
  {
    floatx4 acc[MB][TPW];
    zero_rows(acc);
    if constexpr (BF16) {
      mma_rows_split<MB, TPW>((const __bf16*)sA, L::GLO, St::G, m.w1_bf16, m.w1lo_bf16, kFP / 32, w, NW, NBH, acc,
                              ph, pl);
      split_pre<TPW>(ph, pl, m.w2_bf16, m.w2lo_bf16, HP / 32, w, NW, NBH);
    } else {
      mma_rows_f32<MB, TPW>((const float*)sA, St::G, (const float4*)m.w1_f32, kFP / 16, w, NW, NBH, acc);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = w + i * NW;
      if (nb >= NBH) continue;
      const floatx4 bias = *(const floatx4*)(m.b1 + nb * 16 + uq);
#pragma unroll
      for (int r = 0; r < MB; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float d;
          acc[r][i][j] = swish_parts(acc[r][i][j] + bias[j], d);
          dsw1[r][i][j] = d;
        }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = w + i * NW;
      if (nb >= NBH) continue;
#pragma unroll
      for (int r = 0; r < MB; ++r)
        st4<BF16, BF16>(sA, (__bf16*)sA + L::HLO, (r * 16 + ar) * St::H + nb * 16 + uq, acc[r][i]);
    }
  }
  lds_barrier();

  // z2 = h1 W2 + b2, h2 = swish(z2); delta2 = swish'(z2) sigma wbar -> region
  // B; per-wave partial sums of h2 . W3[:,m] -> sEp (in region A, once every
  // wave is done with h1)
  {
    floatx4 acc[MB][TPW];
    zero_rows(acc);
    if constexpr (BF16) {
      mma_rows_split<MB, TPW>((const __bf16*)sA, L::HLO, St::H, m.w2_bf16, m.w2lo_bf16, HP / 32, w, NW, NBH, acc, ph,
                              pl);
      plain_pre<TPW>(pb, m.w2t_bf16, HP / 32, w, NW, NBH);
    } else {
      mma_rows_f32<MB, TPW>((const float*)sA, St::H, (const float4*)m.w2_f32, HP / 16, w, NW, NBH, acc);
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = w + i * NW;
      if (nb >= NBH) continue;
      const int col = nb * 16 + uq;
      const floatx4 bias = *(const floatx4*)(m.b2 + col);
      const floatx4 wb = *(const floatx4*)(m.w3bar + col);
#pragma unroll
      for (int r = 0; r < MB; ++r) {
        const int row = r * 16 + ar;
        floatx4 d;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float dj;
          acc[r][i][j] = swish_parts(acc[r][i][j] + bias[j], dj);
          d[j] = dj;
        }
        if (m.h2_out && row < n_rows) *(floatx4*)(m.h2_out + (int64_t)(row0 + row) * HP + col) = acc[r][i];
        const floatx4 wr = m.head_w ? *(const floatx4*)(m.head_w + (int64_t)sStruct[row] * HP + col) : wb;
        st4<BF16>(sB, nullptr, row * St::H + col, d * sScale[row] * wr);
      }
    }
    for (int hm = 0; hm < M; ++hm) {
#pragma unroll
      for (int r = 0; r < MB; ++r) {
        // per unit c = uq + j of the 16-column blocks: the sum over the
        // wave's blocks; then an xor butterfly over the 16 units (bits 3 and
        // 2 of c across the lane groups, bits 1 and 0 inside the lane), the
        // tree the tile readout's row sums take, so both readouts agree bit
        // for bit
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          const int nb = w + i * NW;
          if (nb >= NBH) continue;
          floatx4 w3;
          if (M == 1) {
            w3 = *(const floatx4*)(m.w3 + nb * 16 + uq);
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) w3[j] = m.w3[(nb * 16 + uq + j) * M + hm];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) part[j] += acc[r][i][j] * w3[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          part[j] += __shfl_xor(part[j], 32);
          part[j] += __shfl_xor(part[j], 16);
        }
        const float v = (part[0] + part[2]) + (part[1] + part[3]);
        if (l < 16) sEp[(w * TM + r * 16 + ar) * M + hm] = v;
      }
    }
  }
  lds_barrier();
  for (int t = tid; t < TM * M; t += kRoThreads) {
    const int a = t / M, hm = t % M;
    if (a < n_rows) {
      float y = m.b3[hm];
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) y += sEp[(ww * TM + a) * M + hm];
      atomic_e[(int64_t)(row0 + a) * M + hm] = sScale[a] * y + sShift[a];
    }
  }
  // forward-only pass (the energies an uncertainty bias needs first)
  if (m.fwd_only) return;

  // delta1 = swish'(z1) (delta2 W2^T) -> region A (h1 is dead)
  {
    floatx4 acc[MB][TPW];
    zero_rows(acc);
    if constexpr (BF16) {
      mma_rows_bf16<MB, TPW>((const __bf16*)sB, St::H, m.w2t_bf16, HP / 32, w, NW, NBH, acc, pb);
      plain_pre<TPW_G>(pg, m.w1t_bf16, HP / 32, w, NW, NBG);
    } else {
      mma_rows_f32<MB, TPW>((const float*)sB, St::H, (const float4*)m.w2t_f32, HP / 16, w, NW, NBH, acc);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = w + i * NW;
      if (nb >= NBH) continue;
#pragma unroll
      for (int r = 0; r < MB; ++r) st4<BF16>(sA, nullptr, (r * 16 + ar) * St::H + nb * 16 + uq, acc[r][i] * dsw1[r][i]);
    }
  }
  lds_barrier();

  // dE/dG = delta1 W1^T -> HBM [N][kFP] (FP32)
  {
    floatx4 acc[MB][TPW_G];
    zero_rows(acc);
    if constexpr (BF16) {
      mma_rows_bf16<MB, TPW_G>((const __bf16*)sA, St::H, m.w1t_bf16, HP / 32, w, NW, NBG, acc, pg);
    } else {
      mma_rows_f32<MB, TPW_G>((const float*)sA, St::H, (const float4*)m.w1t_f32, HP / 16, w, NW, NBG, acc);
    }
#pragma unroll
    for (int i = 0; i < TPW_G; ++i) {
      const int nb = w + i * NW;
      if (nb >= NBG) continue;
#pragma unroll
      for (int r = 0; r < MB; ++r) {
        const int row = r * 16 + ar;
        if (row < n_rows) *(floatx4*)(dG + (int64_t)(row0 + row) * kFP + nb * 16 + uq) = acc[r][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3. invariant backward: dE/dG and the moments -> dE/dPsi (packed).  Blocks of
// 4 atoms and 256 threads: the first forward pass runs each task's two
// independent halves on two threads; about 29 KB of LDS, so five blocks per
// CU, and each block's load and barrier waits overlap the others' arithmetic
// (the time per block is latency: few tasks per atom between barriers).
constexpr int kBkAtoms = 4;
constexpr int kBkThreads = 256;

struct BackLds {
  static constexpr int LDGB = kFP + 1;
  static constexpr size_t tables = 0;
  static constexpr size_t psi = ro_al(sizeof(Tables));
  static constexpr size_t inter = psi + ro_al(4 * (size_t)kBkAtoms * PS);
  static constexpr size_t gb = inter + ro_al(4 * (size_t)kBkAtoms * IS);
  static constexpr size_t pb = gb + ro_al(4 * (size_t)kBkAtoms * LDGB);
  static constexpr size_t bytes = pb + ro_al(4 * (size_t)kBkAtoms * PS);
};

__global__ void __launch_bounds__(kBkThreads) readout_backward(DevSystem sys, const float* __restrict__ psi,
                                                               const float* __restrict__ dG,
                                                               float* __restrict__ psibar) {
  using L = BackLds;
  constexpr int TB = kBkAtoms, NT = kBkThreads;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Tables& tb = *(Tables*)(lds + L::tables);
  float* sPsi = (float*)(lds + L::psi);
  float* sI = (float*)(lds + L::inter);
  float* sGb = (float*)(lds + L::gb);
  float* sPb = (float*)(lds + L::pb);
  const int tid = threadIdx.x;
  const int row0 = xcd_block(blockIdx.x, gridDim.x) * TB;
  const int n_rows = min(TB, sys.n_atoms - row0);
  // all loads of the tile (dE/dG rows, packed moments) issued up front
  constexpr int NG = (TB * kFP / 4 + NT - 1) / NT;  // float4 per thread
  constexpr int NP = kS * kPacked;
  constexpr int NM = (TB * NP + NT - 1) / NT;
  float4 gv[NG];
  float mv[NM];
  const float4* gsrc = (const float4*)(dG + (int64_t)row0 * kFP);
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int t = tid + u * NT;
    gv[u] = (t < TB * kFP / 4 && t * 4 / kFP < n_rows) ? gsrc[t] : float4{0.0f, 0.0f, 0.0f, 0.0f};
  }
#pragma unroll
  for (int u = 0; u < NM; ++u) {
    const int t = tid + u * NT;
    mv[u] = t < n_rows * NP ? psi[(int64_t)row0 * NP + t] : 0.0f;
  }
  load_tables(&tb);
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int t = (tid + u * NT) * 4;
    if (t >= TB * kFP) continue;
    const int a = t / kFP, f = t % kFP;
    float* d = sGb + a * L::LDGB + f;
    d[0] = gv[u].x;
    d[1] = gv[u].y;
    d[2] = gv[u].z;
    d[3] = gv[u].w;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NM; ++u) {
    const int t = tid + u * NT;
    if (t < TB * NP) {
      const int a = t / NP, e = t % NP;
      const int s = e / kPacked, c = e % kPacked;
      const int n = tb.packed_mult[c];
      for (int q = 0; q < n; ++q) sPsi[a * PS + s * kFull + tb.packed_full[c][q]] = mv[u];
    }
  }
  __syncthreads();
  constexpr int KSF = 2 * ((TB * 20 + 63) / 64 * 64) <= NT ? 2 : 1;
  // the entry pass stays unsplit: its sums then run in the tile readout's
  // order, so both readouts give bit-identical results
  constexpr int KS = 1;
  contract_forward_a<TB, NT, false, false, IS, KSF>(sPsi, sI, nullptr, 0, tb);
  __syncthreads();
  // phase A: each task's two output groups on two threads (no result changes)
  constexpr int KSA = 2 * ((TB * 30 + 63) / 64 * 64) <= NT ? 2 : 1;
  contract_backward_a<TB, NT, KSA>(sPsi, sGb, L::LDGB, sI, tb);
  __syncthreads();
  contract_backward_b<TB, NT, KS>(sPsi, sGb, L::LDGB, sI, sPb, tb);
  __syncthreads();
  auto to_psibar = [&](int a, int e, float v) {
    if (a < n_rows) psibar[(int64_t)(row0 + a) * (kS * kPacked) + e] = v;
  };
  fold_packed<TB, NT>(sPb, tb, to_psibar);
}

// ---------------------------------------------------------------------------
constexpr size_t kLdsMax = 160 * 1024;

// phases: bit 0 invariants, bit 1 network, bit 2 invariant backward
template <int HP, bool BF16>
static gmnn_status launch_stream_t(const DevModel& m, const DevSystem& sys, const float* psi, void* G, float* dG,
                                   float* atomic_e, float* psibar, hipStream_t s, hipEvent_t* ev, int phases) {
  auto mark = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], s);
  };
  using NL = NetLds<HP, BF16>;
  if (NL::bytes(m.M) > kLdsMax) return GMNN_ERR_UNSUPPORTED;
  gmnn_status st = ensure_lds_limit((const void*)readout_features<BF16>, FeatLds<BF16>::bytes);
  if (st == GMNN_OK) st = ensure_lds_limit((const void*)readout_network<HP, BF16>, NL::bytes(m.M));
  if (st == GMNN_OK) st = ensure_lds_limit((const void*)readout_backward, BackLds::bytes);
  if (st != GMNN_OK) return st;
  const int N = sys.n_atoms;
  const int g16 = (N + kRoAtoms - 1) / kRoAtoms;
  const int gn = (N + NL::TM - 1) / NL::TM;
  const int gb = (N + kBkAtoms - 1) / kBkAtoms;
  mark(0);
  if (phases & 1)
    hipLaunchKernelGGL(readout_features<BF16>, dim3(g16), dim3(kFtThreads), FeatLds<BF16>::bytes, s, sys, psi, G);
  mark(1);
  mark(2);
  if (phases & 2)
    hipLaunchKernelGGL((readout_network<HP, BF16>), dim3(gn), dim3(kRoThreads), NL::bytes(m.M), s, m, sys,
                       (const void*)G, atomic_e, dG);
  mark(3);
  mark(4);
  if (phases & 4)
    hipLaunchKernelGGL(readout_backward, dim3(gb), dim3(kBkThreads), BackLds::bytes, s, sys, psi, (const float*)dG,
                       psibar);
  mark(5);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

size_t stream_lds_bytes(int hp, bool bf16, int n_heads) {
  size_t n = 0;
#define SZ(HP) \
  if (hp == HP) n = bf16 ? NetLds<HP, true>::bytes(n_heads) : NetLds<HP, false>::bytes(n_heads);
  SZ(64) SZ(128) SZ(256) SZ(512)
#undef SZ
  if (n == 0) return ~size_t(0);
  size_t f = bf16 ? FeatLds<true>::bytes : FeatLds<false>::bytes;
  if (f > n) n = f;
  if (BackLds::bytes > n) n = BackLds::bytes;
  return n;
}

// workspace of the streamed readout: G [N][kFP] (FP32, or bf16 high and low
// planes) and dE/dG [N][kFP] FP32
size_t stream_g_bytes(int n_atoms, bool bf16) { return (size_t)n_atoms * kFP * (bf16 ? 2 * 2 : 4); }
size_t stream_dg_bytes(int n_atoms) { return (size_t)n_atoms * kFP * 4; }

// ev (may be null): 6 events recorded around the three kernels; phases:
// which of the three run (bit 0 invariants, bit 1 network, bit 2 invariant
// backward)
gmnn_status launch_stream(const DevModel& m, const DevSystem& sys, bool bf16, const float* psi, void* G, float* dG,
                          float* atomic_e, float* psibar, hipStream_t s, hipEvent_t* ev, int phases) {
  if (sys.n_atoms == 0) return GMNN_OK;
#define CASE(HP)                                                                                          \
  if (m.HP1 == HP)                                                                                        \
    return bf16 ? launch_stream_t<HP, true>(m, sys, psi, G, dG, atomic_e, psibar, s, ev, phases)          \
                : launch_stream_t<HP, false>(m, sys, psi, G, dG, atomic_e, psibar, s, ev, phases);
  CASE(64) CASE(128) CASE(256) CASE(512)
#undef CASE
  return GMNN_ERR_UNSUPPORTED;
}

}  // namespace gmnn
