// Tile kernels of the GMNN energy/force path (gfx950, wave64, MFMA).
//
// One block of 512 threads (8 waves) owns a tile of TA atoms (16, or 8 in
// the fused kernel) and keeps everything of the tile in LDS; the network
// products always run on TM = 16 rows (the MFMA block), rows past TA zero:
//   [FUSED only] pair moments of its atoms (Section 2.1, eq. basis_fn), two
//                atoms per wave with 32 lanes each (TA = 16) or one atom per
//                wave with 64 lanes (TA = 8)
//   invariants  (Section 2.1, eq. contraction): families 1-4 and the
//               intermediates T7, V8, M5, v6 in one pass, families 5-8 in a
//               second pass
//   network     (Section 2.1, eq. scale_shift) forward and the backward of
//               the head-mean energy (Section 2.2, eq. jacobian) on MFMA
//   invariants backward: intermediates U8, Y, Qv, then every entry of
//               dE/dPsi in one pass, folded onto the packed components
//   [FUSED only] pair backward of its atoms (Section 3.3): per-pair
//               gradients and the per-atom virial, on the moment stage's lanes
// The fused kernel serves small systems, where the whole step is latency
// bound and one launch per stage would dominate (8-atom tiles spread such a
// system over twice the blocks: half the pair and contraction work per
// block, the same network products); the unfused readout serves large
// systems between the high-occupancy pair kernels.
#include "common.h"
#include "contraction.h"
#include "mfma.h"
#include "model.h"
#include "pair_math.h"

namespace gmnn {

constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / 64;
constexpr int kTM = 16;
constexpr int kFusedMaxSpecies = 8;

template <int HP, bool BF16, bool FUSED, bool PERHEAD, int TA>
struct TileLds {
  using St = NetStrides<HP, BF16>;
  static constexpr int TM = kTM;
  static constexpr int LPA = kTileThreads / TA;  // fused pair stages: lanes per atom
  static constexpr int ESZ = BF16 ? 2 : 4;
  static constexpr size_t al(size_t x) { return (x + 255) & ~size_t(255); }
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t tables = 0;
  static constexpr size_t psi = al(sizeof(Tables));
  static constexpr size_t inter = psi + al(4 * (size_t)TA * PS);
  static constexpr size_t regb = inter + al(4 * (size_t)TA * IS);
  // BF16: G and h1 are held as bf16 high and low parts (split products); G's
  // two parts, later h1's low part, later delta2 and dE/dG share region b
  static constexpr size_t NSPLIT = BF16 ? 2 : 1;
  static constexpr size_t regb_bytes =
      mx(mx(NSPLIT * ESZ * TM * St::G, (size_t)ESZ * TM * St::H), 4 * (size_t)TM * St::GB);
  static constexpr size_t regc = regb + al(regb_bytes);
  static constexpr size_t regc_bytes = mx((size_t)ESZ * TM * St::H, 4 * (size_t)TM * PS);
  static constexpr size_t ep = regc + al(regc_bytes);
  static constexpr size_t rowsc = ep + al(4 * (size_t)kTileWaves * 16 * kMaxHeads);
  static constexpr size_t vir = rowsc + al(4 * 3 * (size_t)TM);  // scale, shift, structure of each row
  static constexpr size_t psibar = vir + al(4 * 9 * (size_t)TA);
  static constexpr size_t dsw2 = psibar + (FUSED ? al(4 * (size_t)TA * kS * kPacked) : 0);
  static constexpr size_t beta = dsw2 + (PERHEAD ? al(4 * (size_t)TM * (HP + 1)) : 0);
  // fused: per-atom context and first pair group of each of the LPA lanes
  static constexpr size_t pctx = beta + (FUSED ? al(4 * (size_t)kFusedMaxSpecies * kFusedMaxSpecies * kS * kMaxBasis) : 0);
  static constexpr size_t ppv = pctx + (FUSED ? al(sizeof(AtomCtx) * (size_t)TA) : 0);
  static constexpr size_t ea = ppv + (FUSED ? al(sizeof(float4) * (size_t)TA * LPA * kPairUnroll) : 0);
  static constexpr size_t bytes = ea + (FUSED ? al(4 * (size_t)TM * kMaxHeads) : 0);
};

// psibar_out: [nh][N][100] (unfused); gpair: [nh][gstride][3] (fused);
// nh = n_heads with PERHEAD (one backward per head), else 1 (head mean).
// tile_rec (fused, may be null): [tile][kMaxHeads + 9] FP64 sums over the
// tile's atoms of the energies (heads 0 .. M-1) and of the virial entries,
// each in atom order, for the per-structure sums
template <int HP, bool BF16, bool FUSED, bool PERHEAD, int TA>
__global__ void __launch_bounds__(kTileThreads)
    tile_kernel(DevModel m, DevSystem sys, const float* __restrict__ psi_in, float* __restrict__ atomic_e,
                float* __restrict__ psibar_out, float* __restrict__ gpair, float* __restrict__ virial,
                int64_t gstride, double* __restrict__ tile_rec) {
  using L = TileLds<HP, BF16, FUSED, PERHEAD, TA>;
  using Sh = NetShape<kTM, HP, kTileWaves>;
  constexpr int TM = kTM;
  constexpr int LPA = L::LPA;
  static_assert(TA == 16 || (FUSED && TA == 8), "16-atom tiles, or 8-atom fused tiles");
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Tables& tb = *(Tables*)(lds + L::tables);
  float* sPsi = (float*)(lds + L::psi);
  float* sI = (float*)(lds + L::inter);
  void* sG = (void*)(lds + L::regb);
  void* sD2 = (void*)(lds + L::regb);
  float* sGb = (float*)(lds + L::regb);
  void* sH = (void*)(lds + L::regc);
  float* sPb = (float*)(lds + L::regc);
  float* sEp = (float*)(lds + L::ep);
  float* sScale = (float*)(lds + L::rowsc);
  float* sShift = sScale + TM;
  int* sStruct = (int*)(sShift + TM);
  float* sVir = (float*)(lds + L::vir);
  float* sPsibar = (float*)(lds + L::psibar);
  float* sDsw2 = (float*)(lds + L::dsw2);
  float* s_beta = (float*)(lds + L::beta);
  AtomCtx* sCtx = (AtomCtx*)(lds + L::pctx);
  float4* sPv = (float4*)(lds + L::ppv);
  float* sEa = FUSED ? (float*)(lds + L::ea) : nullptr;

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int row0 = xcd_block(blockIdx.x, gridDim.x) * TA;
  const int n_rows = min(TA, sys.n_atoms - row0);
  const int nh = PERHEAD ? m.M : 1;

  // fused: this lane's atom context and first pair group are requested
  // before the tables and beta are staged, so their memory round trips overlap
  static_assert(TA * LPA == kTileThreads && (LPA == 32 || LPA == 64), "whole waves per atom pair");
  const int fa = LPA == 32 ? w + kTileWaves * (l >> 5) : w;  // this lane's atom
  const int fq = l & (LPA - 1);
  AtomCtx actx{};
  PairGroup g0{};
  if (FUSED && fa < n_rows) {
    load_atom(sys, row0 + fa, actx);
    fetch_pairs<LPA>(sys, actx, actx.p0 + fq, g0);
  }
  load_tables(&tb);
  for (int t = tid; t < TA * 9; t += kTileThreads) sVir[t] = 0.0f;
  if (TA < TM) {
    // network rows past the tile's atoms read zero invariants
    constexpr int ESZ = BF16 ? 2 : 4;
    constexpr int W0 = TA * NetStrides<HP, BF16>::G * ESZ / 4, W1 = TM * NetStrides<HP, BF16>::G * ESZ / 4;
    for (int t = W0 + tid; t < W1; t += kTileThreads) {
      ((uint32_t*)sG)[t] = 0u;
      if (BF16) ((uint32_t*)sG)[W1 + t] = 0u;  // low parts
    }
  }
  if (FUSED) stage_beta(m, s_beta);
  __syncthreads();

  // ---- moments -> full tensors in LDS ------------------------------------
  // fused pair stages: each wave runs two atoms at once with 32 lanes each
  // (TA = 16), or one atom with all 64 lanes (TA = 8)
  if (FUSED) {
    float v[128];
#pragma unroll
    for (int k = 0; k < 128; ++k) v[k] = 0.0f;
    if (fa < n_rows)
      atom_moments_from<LPA>(m, sys, s_beta, actx, fq, g0, v, PairCache{sCtx + fa, sPv + fa * LPA * kPairUnroll});
    reduce_scatter_128<LPA>(v, fq);
    constexpr int PER = 128 / LPA;  // values each lane owns after the reduce-scatter
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int k = PER * fq + e;
      if (k < kS * kPacked) {
        const int s = k / kPacked, t = k % kPacked;
        const int n = tb.packed_mult[t];
        for (int q = 0; q < n; ++q) sPsi[fa * PS + s * kFull + tb.packed_full[t][q]] = v[e];
      }
    }
  } else {
    // the tile's packed moments are one contiguous run: all loads issued at
    // once, coalesced, then expanded into the full tensors
    constexpr int NP = kS * kPacked;
    constexpr int NU = (TA * NP + kTileThreads - 1) / kTileThreads;
    float v[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kTileThreads;
      v[u] = t < n_rows * NP ? psi_in[(int64_t)row0 * NP + t] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kTileThreads;
      if (t < TA * NP) {
        const int a = t / NP, e = t % NP;
        const int s = e / kPacked, c = e % kPacked;
        const int n = tb.packed_mult[c];
        for (int q = 0; q < n; ++q) sPsi[a * PS + s * kFull + tb.packed_full[c][q]] = v[u];
      }
    }
  }
  __syncthreads();

  // ---- invariants ------------------------------------------------------------
  // the first weight fragments of the network start loading now
  // (one backward per head keeps more live state: a shallower ring there)
  constexpr int kDepth = PERHEAD ? 2 : prefetch_depth<Sh::TPW>();
  // BF16: split-BF16 forward products (high and low parts of G, h1, W1, W2);
  // G's low part follows its high part, h1's low part goes where G was
  constexpr int kGlo = BF16 ? TM * NetStrides<HP, BF16>::G : 0;
  void* sGlo = (void*)((__bf16*)sG + kGlo);
  void* sHlo = sG;
  FwdRing<BF16, Sh::TPW, kDepth> fring;
  BRing<BF16, Sh::TPW, kDepth> ring;
  fwd_ring_fill<BF16, Sh::TPW, kDepth>(fring, m.w1_bf16, m.w1lo_bf16, m.w1_f32, kFP, (tid >> 6) / Sh::MB, Sh::WPR,
                                       Sh::NBH);
  // 8 atoms leave threads for both halves of every task of the first pass
  constexpr int KSF = 2 * ((TA * 20 + 63) / 64 * 64) <= kTileThreads ? 2 : 1;
  contract_forward_a<TA, kTileThreads, BF16, true, IS, KSF>(sPsi, sI, sG, NetStrides<HP, BF16>::G, tb, kGlo);
  // per-atom scale / shift, by the last wave (idle in the phase above), for
  // the network epilogue
  if (tid >= kTileThreads - 64 && tid - (kTileThreads - 64) < TM) {
    const int a = tid - (kTileThreads - 64);
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
  __syncthreads();
  contract_forward_b<TA, kTileThreads, BF16>(sPsi, sI, sG, NetStrides<HP, BF16>::G, tb, kGlo);
  __syncthreads();

  // ---- network forward ---------------------------------------------------------
  floatx4 dsw1[Sh::TPW];
  network_forward<TM, HP, BF16, kTileWaves, !PERHEAD, kDepth>(m, sG, sGlo, sH, sHlo, sD2, sDsw2, sEp, sScale, sShift,
                                                              sStruct, row0, n_rows, atomic_e, sEa, dsw1, fring, ring);
  // forward-only pass (the energies an uncertainty bias needs first): the
  // readout tile stops here (uniform across the block)
  if (!FUSED && m.fwd_only) return;
  constexpr int LDGB = NetStrides<HP, BF16>::GB;
  for (int hm = 0; hm < nh; ++hm) {
    // ---- network backward (head mean, or head hm) ------------------------------
    if (PERHEAD) {
      if (hm > 0) ring_fill(ring, m.w2t_bf16, m.w2t_f32, HP, (tid >> 6) / Sh::MB, Sh::WPR, Sh::NBH);
      network_delta2_head<TM, HP, BF16, kTileWaves>(m, sDsw2, sScale, sD2, hm);
      __syncthreads();
    }
    network_backward<TM, HP, BF16, kTileWaves, kDepth>(m, sD2, sH, sGb, dsw1, ring);
    // ---- invariants backward ---------------------------------------------------
    // phase A: each task's two output groups on two threads when the tile has
    // the threads (8-atom tiles; no result changes)
    constexpr int KSA = 2 * ((TA * 30 + 63) / 64 * 64) <= kTileThreads ? 2 : 1;
    contract_backward_a<TA, kTileThreads, KSA>(sPsi, sGb, LDGB, sI, tb);
    __syncthreads();
    // an 8-atom tile has threads for both halves of every task; the second
    // half's gradient lands in the rows of sPb past the tile's atoms
    constexpr int KS = (TA * 29 * 2 <= kTileThreads) ? 2 : 1;
    static_assert(KS == 1 || 2 * TA <= TM, "both halves fit the 16-row gradient region");
    float* sPb2 = KS == 2 ? sPb + TA * PS : nullptr;
    contract_backward_b<TA, kTileThreads, KS>(sPsi, sGb, LDGB, sI, sPb, tb, sPb2);
    __syncthreads();
    if (FUSED) {
      auto to_lds = [&](int a, int e, float v) { sPsibar[a * (kS * kPacked) + e] = v; };
      fold_packed<TA, kTileThreads, decltype(to_lds), KS == 2>(sPb, tb, to_lds, sPb2);
      __syncthreads();
      // ---- pair backward -----------------------------------------------------
      float* g_head = gpair + (int64_t)hm * gstride * 3;
      {
        float vir[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) vir[k] = 0.0f;
        if (fa < n_rows) {
          float pb[kS * kPacked];
#pragma unroll
          for (int k = 0; k < kS * kPacked; ++k) pb[k] = sPsibar[fa * (kS * kPacked) + k];
          atom_pair_backward<LPA>(m, sys, s_beta, row0 + fa, fq, pb, g_head, vir,
                                  PairCache{sCtx + fa, sPv + fa * LPA * kPairUnroll});
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) vir[k] = atom_sum<LPA>(vir[k]);
        if (fq < 9) {
          float vk = vir[0];
#pragma unroll
          for (int k = 1; k < 9; ++k)
            if (fq == k) vk = vir[k];
          sVir[fa * 9 + fq] += vk;
        }
      }
      __syncthreads();
    } else {
      float* pbo = psibar_out + (int64_t)hm * sys.n_atoms * (kS * kPacked);
      fold_packed<TA, kTileThreads>(
          sPb, tb,
          [&](int a, int e, float v) {
            if (a < n_rows) pbo[(int64_t)(row0 + a) * (kS * kPacked) + e] = v;
          },
          sPb2);
      __syncthreads();
    }
  }
  if (FUSED) {
    const float inv = 1.0f / (float)nh;
    for (int t = tid; t < n_rows * 9; t += kTileThreads) virial[(int64_t)row0 * 9 + t] = sVir[t] * inv;
    if (tile_rec && tid < kMaxHeads + 9) {
      double x = 0.0;
      if (tid < m.M)
        for (int a = 0; a < n_rows; ++a) x += (double)sEa[a * m.M + tid];
      else if (tid >= kMaxHeads)
        for (int a = 0; a < n_rows; ++a) x += (double)(sVir[a * 9 + tid - kMaxHeads] * inv);
      tile_rec[(int64_t)(row0 / TA) * (kMaxHeads + 9) + tid] = x;
    }
  }
}

// ---------------------------------------------------------------------------
template <int HP, bool BF16, bool FUSED, bool PERHEAD, int TA>
static gmnn_status launch_tile_t(const DevModel& m, const DevSystem& sys, const float* psi, float* atomic_e,
                                 float* psibar, float* gpair, float* virial, int64_t gstride, double* tile_rec,
                                 hipStream_t stream) {
  using L = TileLds<HP, BF16, FUSED, PERHEAD, TA>;
  if (L::bytes > 160 * 1024) return GMNN_ERR_UNSUPPORTED;
  auto k = tile_kernel<HP, BF16, FUSED, PERHEAD, TA>;
  const gmnn_status st = ensure_lds_limit((const void*)k, L::bytes);
  if (st != GMNN_OK) return st;
  const int grid = (sys.n_atoms + TA - 1) / TA;
  if (grid == 0) return GMNN_OK;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kTileThreads), L::bytes, stream, m, sys, psi, atomic_e, psibar, gpair,
                     virial, gstride, tile_rec);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

// LDS bytes of the tile kernel (the fused one with 16-atom tiles, the larger)
size_t tile_lds_bytes(int hp, bool bf16, bool fused, bool perhead) {
#define SZ(HP) \
  if (hp == HP) { \
    if (fused && perhead) return ~size_t(0); \
    if (bf16) return fused ? TileLds<HP, true, true, false, 16>::bytes \
                           : (perhead ? TileLds<HP, true, false, true, 16>::bytes : TileLds<HP, true, false, false, 16>::bytes); \
    return fused ? TileLds<HP, false, true, false, 16>::bytes \
                 : (perhead ? TileLds<HP, false, false, true, 16>::bytes : TileLds<HP, false, false, false, 16>::bytes); \
  }
  SZ(64) SZ(128) SZ(256) SZ(512)
#undef SZ
  return ~size_t(0);
}

// the fused kernel serves the head-mean backward only: with one backward per
// head the tile would have to keep swish'(z1) for every head's product live
// across the pair stage, beyond the register file
bool tile_fused_supported(int n_species, int hp, bool bf16, bool perhead) {
  return !perhead && n_species <= kFusedMaxSpecies && tile_lds_bytes(hp, bf16, true, false) <= 160 * 1024;
}

// fused: moments + readout + pair backward in one launch (gpair, virial,
// tile records out) on tiles of tile_atoms (8 or 16) atoms; otherwise the
// readout alone (psi in, psibar out) on 16-atom tiles
gmnn_status launch_tile(bool fused, bool perhead, int tile_atoms, const DevModel& m, const DevSystem& sys, bool bf16,
                        const float* psi, float* atomic_e, float* psibar, float* gpair, float* virial,
                        int64_t gstride, double* tile_rec, hipStream_t stream) {
  if (fused && !tile_fused_supported(m.n_species, m.HP1, bf16, perhead)) return GMNN_ERR_UNSUPPORTED;
  if (fused && tile_atoms != 8 && tile_atoms != 16) return GMNN_ERR_INVALID_ARG;
#define ARGS m, sys, psi, atomic_e, psibar, gpair, virial, gstride, tile_rec, stream
#define FUSED_CASE(HP, BF) \
  return tile_atoms == 8 ? launch_tile_t<HP, BF, true, false, 8>(ARGS) : launch_tile_t<HP, BF, true, false, 16>(ARGS);
#define CASE4(HP, BF) \
  return perhead ? launch_tile_t<HP, BF, false, true, 16>(ARGS) : launch_tile_t<HP, BF, false, false, 16>(ARGS);
#define CASE(HP)                                         \
  if (m.HP1 == HP) {                                     \
    if (fused) {                                         \
      if (perhead) return GMNN_ERR_UNSUPPORTED;          \
      if (bf16) { FUSED_CASE(HP, true) }                 \
      FUSED_CASE(HP, false)                              \
    }                                                    \
    if (bf16) { CASE4(HP, true) }                        \
    CASE4(HP, false)                                     \
  }
  CASE(64) CASE(128) CASE(256) CASE(512)
#undef CASE
#undef CASE4
#undef FUSED_CASE
#undef ARGS
  return GMNN_ERR_UNSUPPORTED;
}

}  // namespace gmnn
