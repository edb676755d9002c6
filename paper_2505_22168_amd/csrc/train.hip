// Training gradients of an energy + force loss (Section 3.4: weighted loss
// terms on energies and forces; Section 3.3: forces are -dE/dx, so the force
// term needs the mixed second derivative of E).
//
// With upstream gradients ebar_b = dL/dEbar_b and lambda = dL/dF, every
// parameter gradient is the gradient of
//     Phi(theta) = sum_i a_i Ebar_i(theta) - D(theta),   a_i = ebar_{b(i)},
//     D = sum_p delta_p . dEbar/dd_p,   delta_p = lambda_j(p) - lambda_i(p),
// i.e. of the energy plus the directional derivative of the energy along
// the position perturbation lambda.  D is evaluated in forward (tangent)
// mode and Phi differentiated in reverse mode:
//   pair_tangent    Psidot_i = sum_p dPsi/dd_p . delta_p
//   train_tile      per 8 atoms: invariants G and their tangent Gdot (in
//                   dual numbers: the product rule on every contraction
//                   family, exact since G is a polynomial); the network forward in
//                   dual numbers with primal and tangent rows stacked into one
//                   16-row MFMA tile; its reverse pass; the invariant
//                   backward Psibar = J^T Gbar + (d/dPsi J Psidot)^T Gdotbar
//                   (the backward map is quadratic in Psi, so the second
//                   term is an exact central difference) and Psidotbar =
//                   J^T Gdotbar.  Writes the rows the weight products need.
//   pair_beta_grad  dPhi/dbeta per pair, reduced per (Z_i, Z_j) without
//                   atomics on the result
//   weight_grad     W1bar = [G;Gdot]^T [z1bar;z1dotbar],
//                   W2bar = [h1;h1dot]^T [z2bar;z2dotbar] as split-K MFMA
//                   products over all atoms, partials summed in a fixed order
//   reductions      bias, W3, scale and shift gradients (fixed order)
#include <algorithm>

#include "common.h"
#include "contraction.h"
#include "mfma.h"
#include "model.h"
#include "pair_math.h"

namespace gmnn {

constexpr int kTrainThreads = 512;
constexpr int kTrainWaves = kTrainThreads / 64;
constexpr int kTA = 8;  // atoms per training tile (16 MFMA rows: primal + tangent)
// phase A of the invariant backward: each task's two output groups on two
// threads when the tile has the threads (no result changes)
constexpr int kTrainKSA = 2 * ((kTA * 30 + 63) / 64 * 64) <= kTrainThreads ? 2 : 1;
// 8 atoms leave threads for both halves of every task of the invariants' first pass
constexpr int kFwdSplit = 2 * ((kTA * 20 + 63) / 64 * 64) <= kTrainThreads ? 2 : 1;

// directional derivative of every monomial at u along v
__device__ inline void dmonomials(float x, float y, float z, float vx, float vy, float vz, float* d) {
  d[0] = 0.0f;
  d[1] = vx; d[2] = vy; d[3] = vz;
  d[4] = 2.0f * x * vx; d[5] = x * vy + y * vx; d[6] = x * vz + z * vx;
  d[7] = 2.0f * y * vy; d[8] = y * vz + z * vy; d[9] = 2.0f * z * vz;
  d[10] = 3.0f * x * x * vx;
  d[11] = 2.0f * x * y * vx + x * x * vy;
  d[12] = 2.0f * x * z * vx + x * x * vz;
  d[13] = y * y * vx + 2.0f * x * y * vy;
  d[14] = y * z * vx + x * z * vy + x * y * vz;
  d[15] = z * z * vx + 2.0f * x * z * vz;
  d[16] = 3.0f * y * y * vy;
  d[17] = 2.0f * y * z * vy + y * y * vz;
  d[18] = z * z * vy + 2.0f * y * z * vz;
  d[19] = 3.0f * z * z * vz;
}

// ---------------------------------------------------------------------------
// Psidot_i = sum_p [ dR_s (u.delta) mono(u) + R_s Dmono(u)[delta_perp / r] ]
template <int LPA>
__global__ void __launch_bounds__(kPairBlock) pair_tangent(DevModel m, DevSystem sys, const float* __restrict__ lambda,
                                                           float* __restrict__ psidot) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (LPA - 1);
  const int i = xcd_block(blockIdx.x, gridDim.x) * (kPairBlock / LPA) + threadIdx.x / LPA;
  const bool live = i < sys.n_atoms;
  float v[128];
#pragma unroll
  for (int k = 0; k < 128; ++k) v[k] = 0.0f;
  if (live) {
    AtomCtx c;
    load_atom(sys, i, c);
    const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
    const float lix = lambda[3 * (int64_t)i], liy = lambda[3 * (int64_t)i + 1], liz = lambda[3 * (int64_t)i + 2];
    for (int64_t p = c.p0 + q; p < c.p1; p += LPA) {
      int j;
      float dx, dy, dz;
      pair_vec(sys, c, p, j, dx, dy, dz);
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (!(r2 < m.rc2) || r2 == 0.0f) continue;
      float r, ir;
      length_of(r2, r, ir);
      const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
      const float ex = lambda[3 * (int64_t)j] - lix, ey = lambda[3 * (int64_t)j + 1] - liy,
                  ez = lambda[3 * (int64_t)j + 2] - liz;
      const float ud = ux * ex + uy * ey + uz * ez;
      Radial rad;
      radial<true>(m, bzi + sys.species[j] * kS * kMaxBasis, r, rad);
      float mo[20], dm[20];
      monomials(ux, uy, uz, mo);
      dmonomials(ux, uy, uz, (ex - ud * ux) * ir, (ey - ud * uy) * ir, (ez - ud * uz) * ir, dm);
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        const float a = rad.dR[s] * ud;
#pragma unroll
        for (int t = 0; t < kPacked; ++t) v[s * kPacked + t] += a * mo[t] + rad.R[s] * dm[t];
      }
    }
  }
  reduce_scatter_128<LPA>(v, q);
  constexpr int OWN = 128 / LPA;
  if (live) {
#pragma unroll
    for (int e = 0; e < OWN; ++e) {
      const int idx = OWN * q + e;
      if (idx < kS * kPacked) psidot[(int64_t)i * (kS * kPacked) + idx] = v[e];
    }
  }
}

// ---------------------------------------------------------------------------
__device__ inline void swish_d2(float z, float& s, float& d1, float& d2) {
  const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-z));  // hardware reciprocal, as swish_parts
  s = z * sg;
  d1 = sg * (1.0f + z * (1.0f - sg));
  d2 = sg * (1.0f - sg) * (2.0f + z * (1.0f - 2.0f * sg));
}

// network products of the training tile: FP32 MFMA, or BF16 MFMA on the
// BF16 weight copies with the FP32 activation tile rounded on load
// one network product of the training tile (16 rows: primal + tangent) from
// a ring filled ahead with the first k-steps of its weights
template <bool BF16, int TPW, int DEPTH>
__device__ __forceinline__ void train_mma(BRing<BF16, TPW, DEPTH>& ring, const float* A, int lda, const bf16x8* Bbf,
                                          const float* Bf, int K, int nb0, int nbs, int NB, floatx4 (&acc)[TPW]) {
  if constexpr (BF16) mma_bf16_a32_ring(ring, A, lda, 0, Bbf, K, nb0, nbs, NB, acc);
  else mma_ring(ring, A, lda, 0, nullptr, Bf, K, nb0, nbs, NB, acc);
}

template <int HP>
struct TrainLds {
  static constexpr int TA = kTA;
  static constexpr int LDG = kFP + 4;   // FP32 A tiles
  static constexpr int LDH = HP + 4;
  static constexpr int LDGB = kFP + 1;
  static constexpr size_t al(size_t x) { return (x + 255) & ~size_t(255); }
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
  static constexpr size_t tables = 0;
  static constexpr size_t psi = al(sizeof(Tables));
  static constexpr size_t psid = psi + al(4 * (size_t)TA * PS);
  static constexpr size_t ptmp = psid + al(4 * (size_t)TA * PS);
  static constexpr size_t inter = ptmp + al(4 * (size_t)TA * PS);
  static constexpr size_t gt = inter + al(4 * (size_t)TA * IS);           // [16][LDG]: G rows 0-7, Gdot rows 8-15
  static constexpr size_t gtmp = gt + al(4 * (size_t)16 * LDG);           // scratch (see gtmp_bytes)
  // scratch: the tangent intermediates [8][ISF], later Gbar [16][LDGB]
  static constexpr size_t gtmp_bytes = mx(4 * (size_t)TA * ISF, 4 * (size_t)16 * LDGB);
  static constexpr size_t ht = gtmp + al(gtmp_bytes);                      // [16][LDH]: h1 / delta tiles
  static constexpr size_t pba = ht + al(4 * (size_t)16 * LDH);            // Psibar accumulator [8][PS]
  static constexpr size_t pbs = pba + al(4 * (size_t)TA * PS);            // scratch full gradient [8][PS]
  static constexpr size_t ep = pbs + al(4 * (size_t)TA * PS);             // [waves][16 rows] partial sums (2 values)
  static constexpr size_t rows = ep + al(4 * (size_t)kTrainWaves * 16 * 2);
  static constexpr size_t bytes = rows + al(4 * 4 * (size_t)TA);          // scale, a, t, y-mean sums
};

// weight-product rows: row k = 16 * tile + r, r < 8 primal atom rows, r >= 8 tangent rows
template <int HP, bool BF16>
__global__ void __launch_bounds__(kTrainThreads)
    train_tile(DevModel m, DevSystem sys, const float* __restrict__ psi, const float* __restrict__ psidot,
               const double* __restrict__ ebar, float* __restrict__ psibar, float* __restrict__ psidotbar,
               float* __restrict__ X1, float* __restrict__ Y1, float* __restrict__ X2, float* __restrict__ Y2,
               float* __restrict__ w3g, float* __restrict__ qsig) {
  using L = TrainLds<HP>;
  using Sh = NetShape<16, HP, kTrainWaves>;
  constexpr int TA = kTA;
  constexpr int TPW = Sh::TPW, TPW_G = Sh::TPW_G, NBH = Sh::NBH, NBG = Sh::NBG, WPR = Sh::WPR;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  Tables& tb = *(Tables*)(lds + L::tables);
  float* sPsi = (float*)(lds + L::psi);
  float* sPd = (float*)(lds + L::psid);
  float* sPt = (float*)(lds + L::ptmp);
  float* sI = (float*)(lds + L::inter);
  float* sGT = (float*)(lds + L::gt);
  float* sGtmp = (float*)(lds + L::gtmp);
  float* sGb = (float*)(lds + L::gtmp);
  float* sH = (float*)(lds + L::ht);
  float* sPbA = (float*)(lds + L::pba);
  float* sPbS = (float*)(lds + L::pbs);
  float* sEp = (float*)(lds + L::ep);
  float* sScale = (float*)(lds + L::rows);
  float* sA = sScale + TA;
  float* sT = sA + TA;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int row0 = xcd_block(blockIdx.x, gridDim.x) * TA;
  const int n_rows = min(TA, sys.n_atoms - row0);
  const int64_t k0 = (int64_t)blockIdx.x * 16;  // first weight-product row of this tile

  load_tables(&tb);
  for (int a = tid; a < TA; a += kTrainThreads) {
    float sc = 0.0f, aa = 0.0f;
    if (a < n_rows) {
      sc = m.scale[sys.species[row0 + a]];
      aa = (float)ebar[sys.atom_struct[row0 + a]];
    }
    sScale[a] = sc;
    sA[a] = aa;
  }
  {
    // the tile's packed moments and tangents are contiguous runs: every load
    // issued at once, then expanded into the full tensors
    constexpr int NP = kS * kPacked;
    constexpr int NU = (TA * NP + kTrainThreads - 1) / kTrainThreads;
    float v[NU], vd[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kTrainThreads;
      const bool ok = t < n_rows * NP;
      v[u] = ok ? psi[(int64_t)row0 * NP + t] : 0.0f;
      vd[u] = ok ? psidot[(int64_t)row0 * NP + t] : 0.0f;
    }
    __syncthreads();  // the tables are in LDS
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int t = tid + u * kTrainThreads;
      if (t < TA * NP) {
        const int a = t / NP, e = t % NP;
        const int s = e / kPacked, c = e % kPacked;
        const int n = tb.packed_mult[c];
        for (int q = 0; q < n; ++q) {
          sPsi[a * PS + s * kFull + tb.packed_full[c][q]] = v[u];
          sPd[a * PS + s * kFull + tb.packed_full[c][q]] = vd[u];
        }
      }
    }
  }
  __syncthreads();
  // per-atom step t = |Psi| / |Psidot| for the exact polynomial differences
  if (w < TA) {
    float n0 = 0.0f, n1 = 0.0f;
    for (int e = l; e < kS * kFull; e += 64) {
      n0 += sPsi[w * PS + e] * sPsi[w * PS + e];
      n1 += sPd[w * PS + e] * sPd[w * PS + e];
    }
    n0 = wave_sum(n0);
    n1 = wave_sum(n1);
    if (l == 0) sT[w] = (n1 > 0.0f && n0 > 0.0f) ? sqrtf(n0 / n1) : 1.0f;
  }
  __syncthreads();

  // ---- invariants G (rows 0-7) and Gdot (rows 8-15) ---------------------------
  contract_forward_a<TA, kTrainThreads, false, true, IS, kFwdSplit>(sPsi, sI, sGT, L::LDG, tb);
  __syncthreads();
  contract_forward_b<TA, kTrainThreads, false>(sPsi, sI, sGT, L::LDG, tb);
  __syncthreads();
  // Gdot = dG/dPsi . Psidot in dual numbers (exact: G is a polynomial in
  // Psi); the tangent intermediates use the scratch region
  contract_forward_a_dual<TA, kTrainThreads, ISF, kFwdSplit>(sPsi, sPd, sGtmp, sGT + 8 * L::LDG, L::LDG);
  __syncthreads();
  contract_forward_b_dual<TA, kTrainThreads, ISF>(sPsi, sPd, sI, sGtmp, sGT + 8 * L::LDG, L::LDG, tb);
  __syncthreads();
  // the first weight fragments of the network start loading now; each
  // product then fills the ring of the next one as soon as its own
  // fragments are consumed, ahead of its epilogue and barrier
  BRing<BF16, TPW> ring;
  ring_fill(ring, m.w1_bf16, m.w1_f32, kFP, w, WPR, NBH);
  // weight-product rows X1 = [G; Gdot]
  for (int t = tid; t < 16 * kFP; t += kTrainThreads) {
    const int r = t / kFP, f = t % kFP;
    X1[(k0 + r) * kFP + f] = ((r & 7) < n_rows) ? sGT[r * L::LDG + f] : 0.0f;
  }

  // ---- network forward in dual numbers ---------------------------------------------
  // the wave's output fragments: rows 4 (l>>4) + j; lanes l and l^32 hold the
  // primal (row < 8) and tangent (row + 8) value of the same column
  const bool prim = l < 32;
  const int cw = w;  // one 16-row block: waves split the columns
  floatx4 s1d[TPW], s1dd[TPW], z1dot[TPW];
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    train_mma(ring, sGT, L::LDG, m.w1_bf16, m.w1_f32, kFP, cw, WPR, NBH, acc);
    ring_fill(ring, m.w2_bf16, m.w2_f32, HP, cw, WPR, NBH);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      const int col = nb * 16 + (l & 15);
      const float bias = nb < NBH ? m.b1[col] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float zv = acc[i][j] + (prim ? bias : 0.0f);
        const float other = lane_xor32(zv);
        const float z1 = prim ? zv : other, zd = prim ? other : zv;
        float s, d1, d2;
        swish_d2(z1, s, d1, d2);
        s1d[i][j] = d1;
        s1dd[i][j] = d2;
        z1dot[i][j] = zd;
        const int row = 4 * (l >> 4) + j;
        if (nb < NBH) sH[row * L::LDH + col] = prim ? s : d1 * zd;
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < 16 * HP; t += kTrainThreads) {
    const int r = t / HP, c = t % HP;
    X2[(k0 + r) * HP + c] = ((r & 7) < n_rows) ? sH[r * L::LDH + c] : 0.0f;
  }
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    train_mma(ring, sH, L::LDH, m.w2_bf16, m.w2_f32, HP, cw, WPR, NBH, acc);
    ring_fill(ring, m.w2t_bf16, m.w2t_f32, HP, cw, WPR, NBH);
    float ypart[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // primal lanes: h2 . w3bar, tangent lanes: h2dot . w3bar
    floatx4 d2out[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      const int col = nb * 16 + (l & 15);
      const bool ok = nb < NBH;
      const float bias = ok ? m.b2[col] : 0.0f;
      const float wb = ok ? m.w3bar[col] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 4 * (l >> 4) + j;
        const int a = row & 7;
        const float zv = acc[i][j] + (prim ? bias : 0.0f);
        const float other = lane_xor32(zv);
        const float z2 = prim ? zv : other, zd = prim ? other : zv;
        float h2, d1, dd;
        swish_d2(z2, h2, d1, dd);
        const float h2d = d1 * zd;
        const float sg = sScale[a];
        const float hbar = sA[a] * sg * wb;       // dPhi/dh2
        const float hdbar = -sg * wb;             // dPhi/dh2dot
        // primal row: z2bar = hbar s' + hdbar s'' z2dot; tangent row: z2dotbar = hdbar s'
        d2out[i][j] = prim ? (hbar * d1 + hdbar * dd * zd) : (hdbar * d1);
        ypart[j] += (prim ? h2 : h2d) * wb;
        if (ok && prim && a < n_rows) w3g[(int64_t)(row0 + a) * HP + col] = (sA[a] * h2 - h2d) * sg / (float)m.M;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float v = ypart[j];
      v = row16_rot_sum(v);  // lane 0 of the row: the xor-butterfly sum
      if ((l & 15) == 0) sEp[w * 16 + 4 * (l >> 4) + j] = v;
    }
    __syncthreads();  // everyone has read h1 (sH) for the product above
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBH) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) sH[(4 * (l >> 4) + j) * L::LDH + col] = d2out[i][j];
    }
  }
  __syncthreads();
  // scale gradient per atom: a ybar_mean - ydot_mean, with y_mean = h2 . w3bar + mean b3
  if (tid < TA) {
    float yp = 0.0f, yt = 0.0f, b3m = 0.0f;
    for (int hm = 0; hm < m.M; ++hm) b3m += m.b3[hm];
    b3m /= (float)m.M;
    for (int ww = 0; ww < kTrainWaves; ++ww) {
      yp += sEp[ww * 16 + tid];
      yt += sEp[ww * 16 + 8 + tid];
    }
    if (tid < n_rows) qsig[row0 + tid] = sA[tid] * (yp + b3m) - yt;
  }
  for (int t = tid; t < 16 * HP; t += kTrainThreads) {
    const int r = t / HP, c = t % HP;
    Y2[(k0 + r) * HP + c] = ((r & 7) < n_rows) ? sH[r * L::LDH + c] : 0.0f;
  }
  // ---- network reverse ------------------------------------------------------------
  BRing<BF16, TPW_G> ring_g;
  {
    floatx4 acc[TPW];
    zero_acc(acc);
    train_mma(ring, sH, L::LDH, m.w2t_bf16, m.w2t_f32, HP, cw, WPR, NBH, acc);
    ring_fill(ring_g, m.w1t_bf16, m.w1t_f32, HP, cw, WPR, NBG);
    __syncthreads();  // all reads of [z2bar; z2dotbar] done before the tile is overwritten
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int nb = cw + i * WPR;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float hv = acc[i][j];                // primal lanes: h1bar, tangent lanes: h1dotbar
        const float other = lane_xor32(hv);
        const float hbar = prim ? hv : other, hdbar = prim ? other : hv;
        const float out = prim ? (hbar * s1d[i][j] + hdbar * s1dd[i][j] * z1dot[i][j]) : (hdbar * s1d[i][j]);
        if (nb < NBH) sH[(4 * (l >> 4) + j) * L::LDH + col] = out;
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < 16 * HP; t += kTrainThreads) {
    const int r = t / HP, c = t % HP;
    Y1[(k0 + r) * HP + c] = ((r & 7) < n_rows) ? sH[r * L::LDH + c] : 0.0f;
  }
  {
    floatx4 acc[TPW_G];
    zero_acc(acc);
    train_mma(ring_g, sH, L::LDH, m.w1t_bf16, m.w1t_f32, HP, cw, WPR, NBG, acc);
#pragma unroll
    for (int i = 0; i < TPW_G; ++i) {
      const int nb = cw + i * WPR;
      if (nb >= NBG) continue;
      const int col = nb * 16 + (l & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) sGb[(4 * (l >> 4) + j) * L::LDGB + col] = acc[i][j];  // rows 0-7 Gbar, 8-15 Gdotbar
    }
  }
  __syncthreads();

  // ---- invariant backward ---------------------------------------------------------
  const float* Gbar = sGb;
  const float* Gdbar = sGb + 8 * L::LDGB;
  // 8 atoms leave threads for both halves of every task of the invariant
  // backward; the second halves go to the G tile, free from here on
  constexpr int KS = (TA * 29 * 2 <= kTrainThreads) ? 2 : 1;
  static_assert(KS == 1 || 2 * TA * PS <= 16 * L::LDG, "both second halves fit the G tile");
  float* sPbS2 = KS == 2 ? sGT : nullptr;
  float* sPbA2 = KS == 2 ? sGT + TA * PS : nullptr;
  // Psidotbar = B(Psi; Gdotbar)
  contract_forward_a<TA, kTrainThreads, false, false, IS, kFwdSplit>(sPsi, sI, nullptr, 0, tb);  // intermediates of Psi
  __syncthreads();
  contract_backward_a<TA, kTrainThreads, kTrainKSA>(sPsi, Gdbar, L::LDGB, sI, tb);
  __syncthreads();
  contract_backward_b<TA, kTrainThreads, KS>(sPsi, Gdbar, L::LDGB, sI, sPbS, tb, sPbS2);
  __syncthreads();
  auto to_psidotbar = [&](int a, int e, float v) {
    if (a < n_rows) psidotbar[(int64_t)(row0 + a) * (kS * kPacked) + e] = v;
  };
  fold_packed<TA, kTrainThreads, decltype(to_psidotbar), KS == 2>(sPbS, tb, to_psidotbar, sPbS2);
  // Psibar = B(Psi; Gbar) + [B(Psi + t Psidot; Gdotbar) - B(Psi - t Psidot; Gdotbar)] / (2t)
  contract_backward_a<TA, kTrainThreads, kTrainKSA>(sPsi, Gbar, L::LDGB, sI, tb);
  __syncthreads();
  contract_backward_b<TA, kTrainThreads, KS>(sPsi, Gbar, L::LDGB, sI, sPbA, tb, sPbA2);
  __syncthreads();
  for (int ev = 0; ev < 2; ++ev) {
    const float sgn = ev == 0 ? 1.0f : -1.0f;
    for (int t = tid; t < TA * kS * kFull; t += kTrainThreads) {
      const int a = t % TA, e = t / TA;
      sPt[a * PS + e] = sPsi[a * PS + e] + sgn * sT[a] * sPd[a * PS + e];
    }
    __syncthreads();
    contract_forward_a<TA, kTrainThreads, false, false, IS, kFwdSplit>(sPt, sI, nullptr, 0, tb);  // intermediates of Psi +- t Psidot
    __syncthreads();
    contract_backward_a<TA, kTrainThreads, kTrainKSA>(sPt, Gdbar, L::LDGB, sI, tb);
    __syncthreads();
    contract_backward_b<TA, kTrainThreads, KS>(sPt, Gdbar, L::LDGB, sI, sPbS, tb, sPbS2);
    __syncthreads();
    for (int t = tid; t < TA * kS * kFull; t += kTrainThreads) {
      const int a = t % TA, e = t / TA;
      const float d = KS == 2 ? sPbS[a * PS + e] + sPbS2[a * PS + e] : sPbS[a * PS + e];
      sPbA[a * PS + e] += sgn * d / (2.0f * sT[a]);
    }
    __syncthreads();
  }
  auto to_psibar = [&](int a, int e, float v) {
    if (a < n_rows) psibar[(int64_t)(row0 + a) * (kS * kPacked) + e] = v;
  };
  fold_packed<TA, kTrainThreads, decltype(to_psibar), KS == 2>(sPbA, tb, to_psibar, sPbA2);
}

// ---------------------------------------------------------------------------
// dPhi/dbeta per pair:
//   c [ f_c g_k (A_s + B_s) + (f_c g_k)' (u.delta) Adot_s ]
// with A_s = Psibar_s . mono(u), Adot_s = Psidotbar_s . mono(u),
// B_s = Psidotbar_s . Dmono(u)[delta_perp / r].  The 35 values of a pair go to
// its (Z_i, Z_j) slot: for each Z_j the wave reduce-scatters the masked
// values, lane k owning slot k, and adds them to the wave's LDS copy of the
// gradient (one writer per slot); per-block copies are summed in wave order
// and written as block partials.
// Blocks of up to 16 waves (four per SIMD hide the per-atom memory round
// trips), as many as the per-wave LDS copies of the gradient allow.
constexpr int kBetaMaxThreads = 1024;
template <int BASIS>
__global__ void __launch_bounds__(kBetaMaxThreads) pair_beta_grad(DevModel m, DevSystem sys, const float* __restrict__ lambda,
                                                             const float* __restrict__ psibar,
                                                             const float* __restrict__ psidotbar,
                                                             float* __restrict__ beta_partial) {
  extern __shared__ float sm[];
  const int nsp = m.n_species;
  const int nslots = nsp * nsp * kS * kMaxBasis;
  float* s_beta = sm;
  float* s_acc = sm + nslots;  // [waves][nslots]
  const int NW = (int)blockDim.x / 64;
  stage_beta(m, s_beta);
  for (int t = threadIdx.x; t < NW * nslots; t += blockDim.x) s_acc[t] = 0.0f;
  __syncthreads();
  const int w = threadIdx.x >> 6, q = threadIdx.x & 63;
  for (int i = blockIdx.x * NW + w; i < sys.n_atoms; i += gridDim.x * NW) {
    AtomCtx c;
    load_atom(sys, i, c);
    const float* bzi = s_beta + c.zsp * nsp * kS * kMaxBasis;
    const float lix = lambda[3 * (int64_t)i], liy = lambda[3 * (int64_t)i + 1], liz = lambda[3 * (int64_t)i + 2];
    for (int64_t p0 = c.p0; p0 < c.p1; p0 += 64) {
      const int64_t p = p0 + q;
      float val[kS * kMaxBasis];
#pragma unroll
      for (int k = 0; k < kS * kMaxBasis; ++k) val[k] = 0.0f;
      int zj = -1;
      if (p < c.p1) {
        int j;
        float dx, dy, dz;
        pair_vec(sys, c, p, j, dx, dy, dz);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < m.rc2 && r2 > 0.0f) {
          zj = sys.species[j];
          float r, ir;
          length_of(r2, r, ir);
          const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
          const float ex = lambda[3 * (int64_t)j] - lix, ey = lambda[3 * (int64_t)j + 1] - liy,
                      ez = lambda[3 * (int64_t)j + 2] - liz;
          const float ud = ux * ex + uy * ey + uz * ez;
          float mo[20], dm[20];
          monomials(ux, uy, uz, mo);
          dmonomials(ux, uy, uz, (ex - ud * ux) * ir, (ey - ud * uy) * ir, (ez - ud * uz) * ir, dm);
          // basis: g_k and (f_c g_k)'
          float sn, cs;
          cutoff_cos_sin(m, r, cs, sn);

          const float fc = 0.5f * (cs + 1.0f) * m.psi_scale;
          const float dfc = -0.5f * (3.14159265358979f / m.r_cut) * sn * m.psi_scale;
          const float* pb = psibar + (int64_t)i * (kS * kPacked);
          const float* pd = psidotbar + (int64_t)i * (kS * kPacked);
          const BasisIter<BASIS> b0(m, r, cs, sn);
#pragma unroll
          for (int s = 0; s < kS; ++s) {
            float A = 0.0f, Ad = 0.0f, Bs = 0.0f;
#pragma unroll
            for (int t = 0; t < kPacked; ++t) {
              A += pb[s * kPacked + t] * mo[t];
              Ad += pd[s * kPacked + t] * mo[t];
              Bs += pd[s * kPacked + t] * dm[t];
            }
            BasisIter<BASIS> bi = b0;
#pragma unroll
            for (int k = 0; k < kMaxBasis; ++k) {
              float gk, dgk;
              bi.next(m, k, gk, dgk);
              val[s * kMaxBasis + k] = fc * gk * (A + Bs) + (dfc * gk + fc * dgk) * ud * Ad;
            }
          }
        }
      }
      for (int z = 0; z < nsp; ++z) {
        float vz[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) vz[k] = (k < kS * kMaxBasis && zj == z) ? val[k < kS * kMaxBasis ? k : 0] : 0.0f;
        // 64 values over 64 lanes: lane q ends with slot q
        rs_swap<32, 32>(vz);
        rs_swap<16, 16>(vz);
        rs_step<8, 0>(vz, (q >> 3) & 1);
        rs_step<4, 1>(vz, (q >> 2) & 1);
        rs_step<2, 2>(vz, (q >> 1) & 1);
        rs_step<1, 3>(vz, q & 1);
        if (q < kS * kMaxBasis) s_acc[w * nslots + (c.zsp * nsp + z) * kS * kMaxBasis + q] += vz[0];
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nslots; t += blockDim.x) {
    float v = 0.0f;
    for (int ww = 0; ww < NW; ++ww) v += s_acc[ww * nslots + t];
    beta_partial[(int64_t)blockIdx.x * nslots + t] = v;
  }
}

// ---------------------------------------------------------------------------
// Gradient of Phi in the positions (the loss's dL/dx, Section 3.3).  Phi
// depends on the pair vectors d_p through Psi_i (adjoint Psibar_i) and
// through Psidot_i = sum_p dPsi_i/dd_p . delta_p (adjoint Psidotbar_i), so
//   dPhi/dd_p = grad phi_{Psibar}(d_p) + D_delta grad phi_{Psidotbar}(d_p),
// phi_w(d) = sum_s R_s(|d|) sum_t w[s][t] mono_t(d/|d|) being the pair's
// moment contribution contracted with w.  The first term is the pair
// backward of the energy; the second, a Hessian-vector product, is the
// same gradient evaluated in dual numbers (value, derivative along
// delta_p), which needs R_s'' besides R_s and R_s'.  The positions' gradient
// then gathers these over the reverse index like the forces.
struct Dual {
  float v, t;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.t + b.t}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.t - b.t}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.t + a.t * b.v}; }
__device__ inline Dual operator*(float a, Dual b) { return {a * b.v, a * b.t}; }
__device__ inline Dual operator*(Dual a, float b) { return {a.v * b, a.t * b}; }
__device__ inline Dual& operator+=(Dual& a, Dual b) { a.v += b.v; a.t += b.t; return a; }

// R_s, dR_s/dr and d^2R_s/dr^2 (the basis and cutoff of radial<true>):
//   Gaussians    g_k'' = (4 gamma^2 (r - mu_k)^2 - 2 gamma) g_k
//   Bessel-like  d^2/dr^2 sinc(k x) = -(k pi / r_c)^2 sinc(k x) - 2 (cos(k x) - sinc(k x)) / r^2
//   cutoff       f_c'' = -(pi / r_c)^2 cos(pi r / r_c) / 2
template <int BASIS>
__device__ inline void radial2(const DevModel& m, const float* __restrict__ bz, float r, float (&R)[kS],
                               float (&dR)[kS], float (&d2R)[kS]) {
  float sn, cs;
  cutoff_cos_sin(m, r, cs, sn);
  const float w = 3.14159265358979f / m.r_cut;
  const float fc = 0.5f * (cs + 1.0f) * m.psi_scale;
  const float dfc = -0.5f * w * sn * m.psi_scale;
  const float d2fc = -0.5f * w * w * cs * m.psi_scale;
  float g[kMaxBasis], dg[kMaxBasis], d2g[kMaxBasis];
  if (BASIS == GMNN_BASIS_BESSEL) {
    const float ir = 1.0f / r;
    const float ix = m.rc_over_pi * ir;
    float sa = sn, ca = cs;
    float sb = 2.0f * cs * sn, cb = 2.0f * cs * cs - 1.0f;
    float sinc_a = sa * ix;
#pragma unroll
    for (int n = 0; n < kMaxBasis; ++n) {
      const float ka = (float)(n + 1) * w, kb = (float)(n + 2) * w;
      const float sinc_b = sb * ix * (1.0f / (float)(n + 2));
      g[n] = m.ck[n] * (sinc_a + sinc_b);
      dg[n] = m.ck[n] * ((ca - sinc_a) + (cb - sinc_b)) * ir;
      d2g[n] = m.ck[n] * (-(ka * ka) * sinc_a - (kb * kb) * sinc_b - 2.0f * ((ca - sinc_a) + (cb - sinc_b)) * ir * ir);
      const float sc = 2.0f * cs * sb - sa, cc = 2.0f * cs * cb - ca;
      sa = sb; ca = cb; sb = sc; cb = cc;
      sinc_a = sinc_b;
    }
  } else {
    const float tau = r - m.r_min;
    const float g0 = __expf(-m.gamma * tau * tau);
    const float a = __expf(2.0f * m.gamma * m.delta * tau);
    float p = g0;
#pragma unroll
    for (int k = 0; k < kMaxBasis; ++k) {
      const float e = tau - (float)k * m.delta;  // r - mu_k
      g[k] = p * m.ck[k];
      dg[k] = -2.0f * m.gamma * e * g[k];
      d2g[k] = (4.0f * m.gamma * m.gamma * e * e - 2.0f * m.gamma) * g[k];
      p *= a;
    }
  }
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    float B = 0.0f, dB = 0.0f, d2B = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxBasis; ++k) {
      const float bk = bz[s * kMaxBasis + k];
      B += bk * g[k];
      dB += bk * dg[k];
      d2B += bk * d2g[k];
    }
    R[s] = fc * B;
    dR[s] = dfc * B + fc * dB;
    d2R[s] = d2fc * B + 2.0f * dfc * dB + fc * d2B;
  }
}

// grad phi_w at the pair in dual numbers: pair_gradient's formula,
//   g = (sum_s dR_s P_s(u)) u + (grad Q - (grad Q . u) u) / r,
// with u, 1/r, R_s, dR_s carrying their derivatives along delta
__device__ inline void pair_gradient_dual(const float* __restrict__ w, const Dual (&R)[kS], const Dual (&dR)[kS],
                                          Dual x, Dual y, Dual z, Dual ir, Dual& gx, Dual& gy, Dual& gz) {
  Dual mo[kPacked];
  mo[0] = {1.0f, 0.0f};
  mo[1] = x; mo[2] = y; mo[3] = z;
  mo[4] = x * x; mo[5] = x * y; mo[6] = x * z; mo[7] = y * y; mo[8] = y * z; mo[9] = z * z;
  mo[10] = mo[4] * x; mo[11] = mo[4] * y; mo[12] = mo[4] * z; mo[13] = mo[7] * x; mo[14] = mo[5] * z;
  mo[15] = mo[9] * x; mo[16] = mo[7] * y; mo[17] = mo[7] * z; mo[18] = mo[9] * y; mo[19] = mo[9] * z;
  Dual radial_part = {0.0f, 0.0f};
  Dual qc[kPacked];
#pragma unroll
  for (int t = 0; t < kPacked; ++t) qc[t] = {0.0f, 0.0f};
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    Dual A = {0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < kPacked; ++t) {
      A += w[s * kPacked + t] * mo[t];
      qc[t] += R[s] * w[s * kPacked + t];
    }
    radial_part += A * dR[s];
  }
  const Dual Gx = qc[1] + 2.0f * qc[4] * x + qc[5] * y + qc[6] * z + 3.0f * qc[10] * x * x + 2.0f * qc[11] * x * y +
                  2.0f * qc[12] * x * z + qc[13] * y * y + qc[14] * y * z + qc[15] * z * z;
  const Dual Gy = qc[2] + qc[5] * x + 2.0f * qc[7] * y + qc[8] * z + qc[11] * x * x + 2.0f * qc[13] * x * y +
                  qc[14] * x * z + 3.0f * qc[16] * y * y + 2.0f * qc[17] * y * z + qc[18] * z * z;
  const Dual Gz = qc[3] + qc[6] * x + qc[8] * y + 2.0f * qc[9] * z + qc[12] * x * x + qc[14] * x * y +
                  2.0f * qc[15] * x * z + qc[17] * y * y + 2.0f * qc[18] * y * z + 3.0f * qc[19] * z * z;
  const Dual gu = Gx * x + Gy * y + Gz * z;
  gx = radial_part * x + (Gx - gu * x) * ir;
  gy = radial_part * y + (Gy - gu * y) * ir;
  gz = radial_part * z + (Gz - gu * z) * ir;
}

constexpr int kPosLanes = 64;  // lanes per atom row of the position-gradient kernels

// dPhi/dd_p for every pair (gpos [P][3]); one 64-lane group per atom
template <int BASIS>
__global__ void __launch_bounds__(kPairBlock) pair_pos_grad(DevModel m, DevSystem sys, const float* __restrict__ lambda,
                                                            const float* __restrict__ psibar,
                                                            const float* __restrict__ psidotbar,
                                                            float* __restrict__ gpos) {
  extern __shared__ float s_beta[];
  stage_beta(m, s_beta);
  __syncthreads();
  const int q = threadIdx.x & (kPosLanes - 1);
  const int i = blockIdx.x * (kPairBlock / kPosLanes) + threadIdx.x / kPosLanes;
  if (i >= sys.n_atoms) return;
  AtomCtx c;
  load_atom(sys, i, c);
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  const float* pb = psibar + (int64_t)i * (kS * kPacked);
  const float* pd = psidotbar + (int64_t)i * (kS * kPacked);
  const float lix = lambda[3 * (int64_t)i], liy = lambda[3 * (int64_t)i + 1], liz = lambda[3 * (int64_t)i + 2];
  for (int64_t p = c.p0 + q; p < c.p1; p += kPosLanes) {
    int j;
    float dx, dy, dz;
    pair_vec(sys, c, p, j, dx, dy, dz);
    const float r2 = dx * dx + dy * dy + dz * dz;
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    if (r2 < m.rc2 && r2 > 0.0f) {
      float r, ir;
      length_of(r2, r, ir);
      const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
      const float* bz = bzi + sys.species[j] * kS * kMaxBasis;
      // the energy's pair gradient with Psibar
      Radial rad;
      radial<true>(m, bz, r, rad);
      float mo[20];
      monomials(ux, uy, uz, mo);
      pair_gradient(pb, rad, mo, ux, uy, uz, ir, gx, gy, gz);
      // its derivative along delta_p with Psidotbar
      const float ex = lambda[3 * (int64_t)j] - lix, ey = lambda[3 * (int64_t)j + 1] - liy,
                  ez = lambda[3 * (int64_t)j + 2] - liz;
      const float rdot = ux * ex + uy * ey + uz * ez;  // d|d|/dt
      float R[kS], dR[kS], d2R[kS];
      radial2<BASIS>(m, bz, r, R, dR, d2R);
      Dual Rd[kS], dRd[kS];
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        Rd[s] = {R[s], dR[s] * rdot};
        dRd[s] = {dR[s], d2R[s] * rdot};
      }
      const Dual xd = {ux, (ex - ux * rdot) * ir}, yd = {uy, (ey - uy * rdot) * ir}, zd = {uz, (ez - uz * rdot) * ir};
      const Dual ird = {ir, -rdot * ir * ir};
      Dual hx, hy, hz;
      pair_gradient_dual(pd, Rd, dRd, xd, yd, zd, ird, hx, hy, hz);
      gx += hx.t;
      gy += hy.t;
      gz += hz.t;
    }
    gpos[3 * p] = gx;
    gpos[3 * p + 1] = gy;
    gpos[3 * p + 2] = gz;
  }
}

// dL/dx_i = sum over the row of (gpos[rev p] - gpos[p]) (added to dL_dpos
// with accumulate, for the per-head sum)
__global__ void __launch_bounds__(kPairBlock) pos_gather(DevSystem sys, const float* __restrict__ gpos,
                                                         float* __restrict__ dL_dpos, int accumulate) {
  const int q = threadIdx.x & (kPosLanes - 1);
  const int i = blockIdx.x * (kPairBlock / kPosLanes) + threadIdx.x / kPosLanes;
  const bool live = i < sys.n_atoms;
  float f[3] = {0.0f, 0.0f, 0.0f};
  if (live) {
    const int64_t p0 = sys.row_ptr[i], p1 = sys.row_ptr[i + 1];
    for (int64_t p = p0 + q; p < p1; p += kPosLanes) {
      const int64_t rp = sys.rev[p];
      f[0] += gpos[3 * rp] - gpos[3 * p];
      f[1] += gpos[3 * rp + 1] - gpos[3 * p + 1];
      f[2] += gpos[3 * rp + 2] - gpos[3 * p + 2];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k] = atom_sum<kPosLanes>(f[k]);
  if (live && q == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dL_dpos[3 * (int64_t)i + k] = accumulate ? dL_dpos[3 * (int64_t)i + k] + f[k] : f[k];
}

// ---------------------------------------------------------------------------
// C[M][N] = sum_k A[k][M]^T B[k][N] over the rows k of chunk blockIdx.y
// (split-K; partial[chunk][M][N]).  Each wave owns a 64 x 64 block of C as
// 4 x 4 MFMA tiles, so every value loaded feeds four (SPLIT: twelve) MFMAs.
// M and N are multiples of 64.
//   SPLIT = false: FP32 MFMA 16x16x4, four k-steps of loads issued before
//                  their MFMAs.
//   SPLIT = true:  each FP32 operand x is split into hi = bf16(x) and
//                  lo = bf16(x - hi) (nearest even), and a.b is taken as
//                  hi.hi + hi.lo + lo.hi on BF16 MFMA 16x16x32 with FP32
//                  accumulation: about 16 significant bits per product (the
//                  dropped lo.lo is below 2^-16 of |a b|) at the BF16 rate.
constexpr int kWgRows = 1024;    // rows per split-K chunk
constexpr int kWgRowsF32 = 512;  // rows per chunk of weight_grad_staged_f32 (twice the blocks)
template <bool SPLIT>
__global__ void __launch_bounds__(256) weight_grad(const float* __restrict__ A, int ldA, const float* __restrict__ B,
                                                   int ldB, int Mdim, int Ndim, int64_t K, int64_t kchunk,
                                                   float* __restrict__ partial) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tiles_n = Ndim / 64;
  const int tile = blockIdx.x * 4 + w;
  if (tile >= (Mdim / 64) * tiles_n) return;
  const int m0 = (tile / tiles_n) * 64, n0 = (tile % tiles_n) * 64;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  floatx4 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const float* ap = A + m0 + (l & 15);
  const float* bp = B + n0 + (l & 15);
  if (!SPLIT) {
    // lane l supplies A^T[m = l&15][k = l>>4] = A[k][m] and B[k = l>>4][n = l&15]
    for (int64_t k = kb; k < ke; k += 16) {
      float a[4][4], b[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t kk = k + 4 * u + (l >> 4);
        const bool ok = kk < ke;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[u][r] = ok ? ap[kk * ldA + r * 16] : 0.0f;
          b[u][r] = ok ? bp[kk * ldB + r * 16] : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][r], b[u][c], acc[r][c], 0, 0, 0);
    }
  } else {
    // lane l supplies A^T[m = l&15][k = 8 (l>>4) + e] and B[k = 8 (l>>4) + e][n = l&15], e < 8
    for (int64_t k = kb; k < ke; k += 32) {
      float a[4][8], b[4][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t kk = k + 8 * (l >> 4) + e;
        const bool ok = kk < ke;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[r][e] = ok ? ap[kk * ldA + r * 16] : 0.0f;
          b[r][e] = ok ? bp[kk * ldB + r * 16] : 0.0f;
        }
      }
      bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const __bf16 x = (__bf16)a[r][e], y = (__bf16)b[r][e];
          ah[r][e] = x;
          al[r][e] = (__bf16)(a[r][e] - (float)x);
          bh[r][e] = y;
          bl[r][e] = (__bf16)(b[r][e] - (float)y);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh[c], acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl[c], acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh[c], acc[r][c], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = m0 + r * 16 + 4 * (l >> 4) + j, col = n0 + c * 16 + (l & 15);
        partial[((int64_t)blockIdx.y * Mdim + row) * Ndim + col] = acc[r][c][j];
      }
}

// The split product of weight_grad<true> for M and N multiples of 128, with
// the operand rows staged through LDS: a block of 4 waves owns a 128 x 128
// block of C (2 x 2 waves of 64 x 64, with the fragments and the MFMA
// sequence of weight_grad<true>).  Per k-step of 32
// rows every thread loads 16 rows of one column of A and of B, splits them
// once for the whole block, and writes them to LDS as k-contiguous hi and lo
// runs; the next k-step's loads are issued before the current step's MFMAs.
constexpr int kWgBlk = 128;  // block tile edge
constexpr int kWgLdk = 40;   // LDS row stride in bf16 (32 k + 8 pad)
__global__ void __launch_bounds__(256) weight_grad_staged(const float* __restrict__ A, int ldA,
                                                          const float* __restrict__ B, int ldB, int Mdim, int Ndim,
                                                          int64_t K, int64_t kchunk, float* __restrict__ partial) {
  // [Ahi, Alo, Bhi, Blo][column][k]
  __shared__ __attribute__((aligned(16))) __bf16 sm[4][kWgBlk * kWgLdk];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int tiles_n = Ndim / kWgBlk;
  const int mb = (blockIdx.x / tiles_n) * kWgBlk, nb = (blockIdx.x % tiles_n) * kWgBlk;
  const int m0 = (w >> 1) * 64, n0 = (w & 1) * 64;  // the wave's block inside the block tile
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  floatx4 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  // staging: thread tid loads rows 16 h .. 16 h + 15 of column col of the step
  const int col = tid & (kWgBlk - 1), h = tid >> 7;
  const float* ap = A + mb + col;
  const float* bp = B + nb + col;
  float ra[16], rb[16];
  auto fetch = [&](int64_t k) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t kk = k + 16 * h + e;
      const bool ok = kk < ke;
      ra[e] = ok ? ap[kk * ldA] : 0.0f;
      rb[e] = ok ? bp[kk * ldB] : 0.0f;
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k = kb; k < ke; k += 32) {
    __syncthreads();  // the previous step's fragment reads are done
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      bf16x8 ah, al, bh, bl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = ra[8 * half + e], y = rb[8 * half + e];
        const __bf16 xh = (__bf16)x, yh = (__bf16)y;
        ah[e] = xh;
        al[e] = (__bf16)(x - (float)xh);
        bh[e] = yh;
        bl[e] = (__bf16)(y - (float)yh);
      }
      const int o = col * kWgLdk + 16 * h + 8 * half;
      *(bf16x8*)&sm[0][o] = ah;
      *(bf16x8*)&sm[1][o] = al;
      *(bf16x8*)&sm[2][o] = bh;
      *(bf16x8*)&sm[3][o] = bl;
    }
    __syncthreads();
    if (k + 32 < ke) fetch(k + 32);
    // lane l supplies A^T[m = l&15][k = 8 (l>>4) + e] and B[k = 8 (l>>4) + e][n = l&15]
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int o = (n0 + 16 * c + (l & 15)) * kWgLdk + 8 * (l >> 4);
      bh[c] = *(const bf16x8*)&sm[2][o];
      bl[c] = *(const bf16x8*)&sm[3][o];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = (m0 + 16 * r + (l & 15)) * kWgLdk + 8 * (l >> 4);
      const bf16x8 ah = *(const bf16x8*)&sm[0][o];
      const bf16x8 al = *(const bf16x8*)&sm[1][o];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[r][c], 0, 0, 0);
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[r][c], 0, 0, 0);
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[r][c], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = mb + m0 + r * 16 + 4 * (l >> 4) + j, cc = nb + n0 + c * 16 + (l & 15);
        partial[((int64_t)blockIdx.y * Mdim + row) * Ndim + cc] = acc[r][c][j];
      }
}

// The FP32 product of weight_grad<false> for M and N multiples of 128,
// staged through LDS like weight_grad_staged (128 x 128 block tile, 2 x 2
// waves of 64 x 64, k-steps of 32 rows, the next step's rows in flight
// during the MFMAs).  A column's 32 rows are stored permuted, row k at
// 8 (k % 4) + k / 4, so that the 8 values lane l supplies over the step's
// eight 16x16x4 products (rows 4 u + (l >> 4), u < 8) are contiguous.  The
// MFMA sequence per element is weight_grad<false>'s.
constexpr int kWgLdkF = 36;  // LDS row stride in floats (32 k + 4 pad)
__global__ void __launch_bounds__(256) weight_grad_staged_f32(const float* __restrict__ A, int ldA,
                                                              const float* __restrict__ B, int ldB, int Mdim,
                                                              int Ndim, int64_t K, int64_t kchunk,
                                                              float* __restrict__ partial) {
  // [A, B][column][permuted k]
  __shared__ __attribute__((aligned(16))) float sm[2][kWgBlk * kWgLdkF];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int tiles_n = Ndim / kWgBlk;
  const int mb = (blockIdx.x / tiles_n) * kWgBlk, nb = (blockIdx.x % tiles_n) * kWgBlk;
  const int m0 = (w >> 1) * 64, n0 = (w & 1) * 64;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  floatx4 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const int col = tid & (kWgBlk - 1), h = tid >> 7;
  const float* ap = A + mb + col;
  const float* bp = B + nb + col;
  float ra[16], rb[16];
  auto fetch = [&](int64_t k) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t kk = k + 16 * h + e;
      const bool ok = kk < ke;
      ra[e] = ok ? ap[kk * ldA] : 0.0f;
      rb[e] = ok ? bp[kk * ldB] : 0.0f;
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k = kb; k < ke; k += 32) {
    __syncthreads();  // the previous step's fragment reads are done
    // rows 16 h + e, e = q + 4 j (j < 4), go to 8 q + 4 h + j: one float4 per q
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = col * kWgLdkF + 8 * q + 4 * h;
      *(floatx4*)&sm[0][o] = floatx4{ra[q], ra[q + 4], ra[q + 8], ra[q + 12]};
      *(floatx4*)&sm[1][o] = floatx4{rb[q], rb[q + 4], rb[q + 8], rb[q + 12]};
    }
    __syncthreads();
    if (k + 32 < ke) fetch(k + 32);
    // lane l's values for products u < 8: rows 4 u + (l >> 4), stored at 8 (l >> 4) + u
    floatx4 bf[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int o = (n0 + 16 * c + (l & 15)) * kWgLdkF + 8 * (l >> 4);
      bf[c][0] = *(const floatx4*)&sm[1][o];
      bf[c][1] = *(const floatx4*)&sm[1][o + 4];
    }
    floatx4 af[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = (m0 + 16 * r + (l & 15)) * kWgLdkF + 8 * (l >> 4);
      af[r][0] = *(const floatx4*)&sm[0][o];
      af[r][1] = *(const floatx4*)&sm[0][o + 4];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[r][u >> 2][u & 3], bf[c][u >> 2][u & 3], acc[r][c], 0,
                                                           0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = mb + m0 + r * 16 + 4 * (l >> 4) + j, cc = nb + n0 + c * 16 + (l & 15);
        partial[((int64_t)blockIdx.y * Mdim + row) * Ndim + cc] = acc[r][c][j];
      }
}

// sum_c partial[c][i], chunks in order (eight loads in flight)
__device__ inline float sum_chunks(const float* __restrict__ partial, int nchunks, int64_t n, int64_t i) {
  float v = 0.0f;
  int c = 0;
  for (; c + 8 <= nchunks; c += 8) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = partial[(int64_t)(c + u) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; c < nchunks; ++c) v += partial[(int64_t)c * n + i];
  return v;
}

// out[i] = sum_c partial[c][i]
__global__ void sum_partials(const float* __restrict__ partial, int nchunks, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = sum_chunks(partial, nchunks, n, i);
}

// the same sums of a padded [.][ld] gradient (n = padded size), written
// unpadded into the caller's [rows][cols] array
__global__ void sum_partials_unpad(const float* __restrict__ partial, int nchunks, int64_t n, int ld, int rows,
                                   int cols, float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int r = (int)(t / cols), c = (int)(t % cols);
  dst[t] = sum_chunks(partial, nchunks, n, (int64_t)r * ld + c);
}

// column sums, stage 1: partial[chunk][c] = sum of Y[k][c] over the rows k
// of the chunk (with primal_only, the rows with (k & 15) < 8: the primal
// halves of the dual-number tiles).  Block = 64 columns x 4 row lanes; lane
// r takes rows r, r + 4, ... of the chunk; the four lane sums are added in
// lane order.  Grid (ceil(ncols / 64), chunks).
constexpr int kColChunks = 128;  // at most this many row chunks
__global__ void __launch_bounds__(256) column_partials(const float* __restrict__ Y, int ld, int64_t nrows,
                                                       int64_t rows_per_chunk, int ncols, bool primal_only,
                                                       float* __restrict__ partial) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int64_t k0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t k1 = min(nrows, k0 + rows_per_chunk);
  float v = 0.0f;
  if (c < ncols) {
    int64_t k = k0 + r;
    for (; k + 28 < k1; k += 32) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t kk = k + 4 * u;
        x[u] = (!primal_only || (kk & 15) < 8) ? Y[kk * ld + c] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; k < k1; k += 4)
      if (!primal_only || (k & 15) < 8) v += Y[k * ld + c];
  }
  red[r][cl] = v;
  __syncthreads();
  if (r == 0 && c < ncols)
    partial[(int64_t)blockIdx.y * ncols + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

// per-species sums, stage 1: block b takes atoms [b*256, b*256+256) and
// writes, in FP64, sp[b][z][0] = sum qsig_i and sp[b][z][1] = sum ebar_b(i)
// over its atoms of species z, and sp[b][nsp][0] = sum ebar_b(i) sigma_z(i)
// (fixed-shape tree sums: the result does not depend on scheduling)
constexpr int kSpeciesChunk = 256;
__global__ void __launch_bounds__(kSpeciesChunk)
    species_partials(DevModel m, DevSystem sys, const double* __restrict__ ebar, const float* __restrict__ qsig,
                     double* __restrict__ sp) {
  __shared__ double red[kSpeciesChunk / 64][kMaxSpecies + 1][2];
  const int i = blockIdx.x * kSpeciesChunk + threadIdx.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  int z = -1;
  double q = 0.0, e = 0.0;
  if (i < sys.n_atoms) {
    z = sys.species[i];
    q = (double)qsig[i];
    e = ebar[sys.atom_struct[i]];
  }
  const int nsp = m.n_species;
  for (int t = 0; t < nsp; ++t) {
    const double a = wave_sum(z == t ? q : 0.0);
    const double b = wave_sum(z == t ? e : 0.0);
    if (l == 0) {
      red[w][t][0] = a;
      red[w][t][1] = b;
    }
  }
  const double c = wave_sum(z >= 0 ? e * (double)m.scale[z] : 0.0);
  if (l == 0) red[w][nsp][0] = c;
  __syncthreads();
  if (threadIdx.x < 2 * (nsp + 1)) {
    const int t = threadIdx.x >> 1, k = threadIdx.x & 1;
    double v = 0.0;
    for (int ww = 0; ww < kSpeciesChunk / 64; ++ww) v += (t < nsp || k == 0) ? red[ww][t][k] : 0.0;
    sp[((int64_t)blockIdx.x * (kMaxSpecies + 1) + t) * 2 + k] = v;
  }
}

// stage 2: scale / shift / b3 gradients from the block partials, in block order
__global__ void species_finish(DevModel m, const double* __restrict__ sp, int nblocks, float* __restrict__ gscale,
                               float* __restrict__ gshift, float* __restrict__ gb3) {
  const int t = threadIdx.x;
  const int nsp = m.n_species;
  if (t > nsp) return;
  // block partials added in block order; the loads of 8 blocks are issued
  // before their adds so they overlap
  constexpr int kBatch = 8;
  double s1 = 0.0, s2 = 0.0;
  for (int b0 = 0; b0 < nblocks; b0 += kBatch) {
    double x[kBatch], y[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int64_t o = ((int64_t)std::min(b0 + j, nblocks - 1) * (kMaxSpecies + 1) + t) * 2;
      x[j] = sp[o];
      y[j] = sp[o + 1];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (b0 + j < nblocks) {
        s1 += x[j];
        s2 += y[j];
      }
    }
  }
  if (t < nsp) {
    gscale[t] = (float)s1;
    gshift[t] = (float)s2;
  } else {
    // dPhi/db3_m = sum_i a_i sigma_i / M (the same for every head)
    for (int hm = 0; hm < m.M; ++hm) gb3[hm] = (float)(s1 / m.M);
  }
}

// W3 gradient: every head column equals the column sum of w3g
__global__ void w3_broadcast(const float* __restrict__ w3sum, int H2, int M, float* __restrict__ gw3) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H2) return;
  for (int hm = 0; hm < M; ++hm) gw3[(int64_t)h * M + hm] = w3sum[h];
}

// beta gradient: sum of block partials in block order
__global__ void beta_unpack(const float* __restrict__ summed, int nsp, int K, float* __restrict__ gbeta) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = nsp * nsp * kS * K;
  if (t >= n) return;
  const int k = t % K, rest = t / K;
  gbeta[t] = summed[rest * kMaxBasis + k];
}

// ---------------------------------------------------------------------------
template <int HP, bool BF16>
static gmnn_status launch_train_tile_t(const DevModel& m, const DevSystem& sys, const float* psi, const float* psidot,
                                       const double* ebar, float* psibar, float* psidotbar, float* X1, float* Y1,
                                       float* X2, float* Y2, float* w3g, float* qsig, hipStream_t s) {
  using L = TrainLds<HP>;
  if (L::bytes > 160 * 1024) return GMNN_ERR_UNSUPPORTED;
  auto k = train_tile<HP, BF16>;
  const gmnn_status sa = ensure_lds_limit((const void*)k, L::bytes);
  if (sa != GMNN_OK) return sa;
  const int grid = (sys.n_atoms + kTA - 1) / kTA;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kTrainThreads), L::bytes, s, m, sys, psi, psidot, ebar, psibar, psidotbar,
                     X1, Y1, X2, Y2, w3g, qsig);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

struct TrainLayout {
  size_t psi, psidot, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, part1, part2, bpart, bsum;
  size_t cpart, w3sum, spart, bytes;
  int ccK, ccN;        // row chunks of the column sums over K rows / over N atoms
  int64_t rcK, rcN;    // rows per chunk of those sums
  int sp_blocks;       // blocks of the per-species sums
  int64_t K;           // weight-product rows
  int kchunks;          // split-K chunks the partial buffers hold (the larger count)
  int beta_blocks;
};

TrainLayout train_layout(int n_atoms, int HP, int nsp) {
  TrainLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t N = (size_t)n_atoms;
  const int64_t tiles = (n_atoms + kTA - 1) / kTA;
  L.K = tiles * 16;
  L.kchunks = (int)((L.K + kWgRowsF32 - 1) / kWgRowsF32);
  L.beta_blocks = 256;
  L.psi = take(4 * N * 100);
  L.psidot = take(4 * N * 100);
  L.psibar = take(4 * N * 100);
  L.psidotbar = take(4 * N * 100);
  L.X1 = take(4 * (size_t)L.K * kFP);
  L.Y1 = take(4 * (size_t)L.K * HP);
  L.X2 = take(4 * (size_t)L.K * HP);
  L.Y2 = take(4 * (size_t)L.K * HP);
  L.w3g = take(4 * N * HP);
  L.qsig = take(4 * N);
  L.part1 = take(4 * (size_t)L.kchunks * kFP * HP);
  L.part2 = take(4 * (size_t)L.kchunks * HP * HP);
  const size_t nslots = (size_t)nsp * nsp * kS * kMaxBasis;
  L.bpart = take(4 * (size_t)L.beta_blocks * nslots);
  L.bsum = take(4 * nslots);
  L.rcK = L.K > 0 ? (L.K + kColChunks - 1) / kColChunks : 1;
  L.rcN = N > 0 ? ((int64_t)N + kColChunks - 1) / kColChunks : 1;
  L.ccK = (int)((L.K + L.rcK - 1) / L.rcK);
  L.ccN = (int)(((int64_t)N + L.rcN - 1) / L.rcN);
  L.cpart = take(4 * (size_t)HP * (size_t)(L.ccK > L.ccN ? L.ccK : L.ccN));
  L.w3sum = take(4 * (size_t)HP);
  L.sp_blocks = (int)((N + kSpeciesChunk - 1) / kSpeciesChunk);
  L.spart = take(8 * 2 * (size_t)(kMaxSpecies + 1) * (L.sp_blocks > 0 ? L.sp_blocks : 1));
  L.bytes = off;
  return L;
}

template <int LPA>
__global__ void pair_moments(DevModel m, DevSystem sys, float* psi, int* counters, int n_counters);

bool train_supported(const DevModel& m) {
  return m.n_species <= kMaxSpecies && TrainLds<512>::bytes <= 160 * 1024 &&
         (m.HP1 == 64 || m.HP1 == 128 || m.HP1 == 256 || m.HP1 == 512);
}

size_t train_workspace_bytes(int n_atoms, int HP, int nsp) { return train_layout(n_atoms, HP, nsp).bytes; }

gmnn_status train_backward(const DevModel& m, const DevSystem& sys, bool bf16, bool lanes16, int H1, int H2,
                           const double* ebar, const float* lambda, gmnn_param_grads* g, void* ws, size_t ws_bytes,
                           float* dL_dpos, float* gpos, bool accumulate_pos, hipStream_t s) {
  const int HP = m.HP1;
  const int nsp = m.n_species;
  const TrainLayout L = train_layout(sys.n_atoms, HP, nsp);
  if (ws_bytes < L.bytes) return GMNN_ERR_WORKSPACE;
  char* W = (char*)ws;
  float* psi = (float*)(W + L.psi);
  float* psidot = (float*)(W + L.psidot);
  float* psibar = (float*)(W + L.psibar);
  float* psidotbar = (float*)(W + L.psidotbar);
  float *X1 = (float*)(W + L.X1), *Y1 = (float*)(W + L.Y1), *X2 = (float*)(W + L.X2), *Y2 = (float*)(W + L.Y2);
  float* w3g = (float*)(W + L.w3g);
  float* qsig = (float*)(W + L.qsig);
  float* part1 = (float*)(W + L.part1);
  float* part2 = (float*)(W + L.part2);
  float* bpart = (float*)(W + L.bpart);
  float* bsum = (float*)(W + L.bsum);
  const int N = sys.n_atoms;
  const int nslots = nsp * nsp * kS * kMaxBasis;
  const size_t beta_lds = sizeof(float) * (size_t)nslots;
  const int lpa = (N < 8192 && !lanes16) ? 64 : 16;
  const int nb = (N + kPairBlock / lpa - 1) / (kPairBlock / lpa);
  gmnn_status st = GMNN_OK;
  if (N > 0) {
    if (lpa == 64) {
      hipLaunchKernelGGL(pair_moments<64>, dim3(nb), dim3(kPairBlock), beta_lds, s, m, sys, psi, (int*)nullptr, 0);
      hipLaunchKernelGGL(pair_tangent<64>, dim3(nb), dim3(kPairBlock), beta_lds, s, m, sys, lambda, psidot);
    } else {
      hipLaunchKernelGGL(pair_moments<16>, dim3(nb), dim3(kPairBlock), beta_lds, s, m, sys, psi, (int*)nullptr, 0);
      hipLaunchKernelGGL(pair_tangent<16>, dim3(nb), dim3(kPairBlock), beta_lds, s, m, sys, lambda, psidot);
    }
    switch (HP) {
      case 64:
        st = bf16 ? launch_train_tile_t<64, true>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s)
                  : launch_train_tile_t<64, false>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s);
        break;
      case 128:
        st = bf16 ? launch_train_tile_t<128, true>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s)
                  : launch_train_tile_t<128, false>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s);
        break;
      case 256:
        st = bf16 ? launch_train_tile_t<256, true>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s)
                  : launch_train_tile_t<256, false>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s);
        break;
      case 512:
        st = bf16 ? launch_train_tile_t<512, true>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s)
                  : launch_train_tile_t<512, false>(m, sys, psi, psidot, ebar, psibar, psidotbar, X1, Y1, X2, Y2, w3g, qsig, s);
        break;
      default: return GMNN_ERR_UNSUPPORTED;
    }
    if (st != GMNN_OK) return st;
  }
  if (dL_dpos && N > 0) {
    // the positions' gradient from the same adjoints as the beta gradient
    const int nbp = (N + kPairBlock / kPosLanes - 1) / (kPairBlock / kPosLanes);
    auto kp = m.basis == GMNN_BASIS_BESSEL ? pair_pos_grad<GMNN_BASIS_BESSEL> : pair_pos_grad<GMNN_BASIS_GAUSSIAN>;
    const gmnn_status sp = ensure_lds_limit((const void*)kp, beta_lds);
    if (sp != GMNN_OK) return sp;
    hipLaunchKernelGGL(kp, dim3(nbp), dim3(kPairBlock), beta_lds, s, m, sys, lambda, psibar, psidotbar, gpos);
    hipLaunchKernelGGL(pos_gather, dim3(nbp), dim3(kPairBlock), 0, s, sys, gpos, dL_dpos, accumulate_pos ? 1 : 0);
  }
  // waves per block: the beta table plus one gradient copy per wave in 160 KB
  const int beta_waves = (int)std::min<size_t>(kBetaMaxThreads / 64, std::max<size_t>(1, 160 * 1024 / beta_lds - 1));
  {
    auto kb = m.basis == GMNN_BASIS_BESSEL ? pair_beta_grad<GMNN_BASIS_BESSEL> : pair_beta_grad<GMNN_BASIS_GAUSSIAN>;
    const gmnn_status sa = ensure_lds_limit((const void*)kb, beta_lds * (1 + beta_waves));
    if (sa != GMNN_OK) return sa;
    hipLaunchKernelGGL(kb, dim3(L.beta_blocks), dim3(64 * beta_waves), beta_lds * (1 + beta_waves), s, m, sys, lambda,
                       psibar, psidotbar, bpart);
  }
  // weight products, split over chunks of rows, partials summed in chunk order
  const bool staged = HP % kWgBlk == 0;
  const int64_t wg_rows = (staged && !bf16) ? kWgRowsF32 : kWgRows;
  const int kch = (int)((L.K + wg_rows - 1) / wg_rows);
  {
    const int t1 = (kFP / 64) * (HP / 64);
    const int t2 = (HP / 64) * (HP / 64);
    if (kch > 0) {
      // the BF16 path takes the split-BF16 products, the FP32 path plain FP32
      if (bf16 && staged) {
        // kFP and HP are multiples of the staged kernel's 128-wide block tile
        hipLaunchKernelGGL(weight_grad_staged, dim3((kFP / kWgBlk) * (HP / kWgBlk), kch), dim3(256), 0, s,
                           X1, kFP, Y1, HP, kFP, HP, L.K, wg_rows, part1);
        hipLaunchKernelGGL(weight_grad_staged, dim3((HP / kWgBlk) * (HP / kWgBlk), kch), dim3(256), 0, s,
                           X2, HP, Y2, HP, HP, HP, L.K, wg_rows, part2);
      } else if (staged) {
        hipLaunchKernelGGL(weight_grad_staged_f32, dim3((kFP / kWgBlk) * (HP / kWgBlk), kch), dim3(256), 0,
                           s, X1, kFP, Y1, HP, kFP, HP, L.K, wg_rows, part1);
        hipLaunchKernelGGL(weight_grad_staged_f32, dim3((HP / kWgBlk) * (HP / kWgBlk), kch), dim3(256), 0,
                           s, X2, HP, Y2, HP, HP, HP, L.K, wg_rows, part2);
      } else {
        auto wg = bf16 ? weight_grad<true> : weight_grad<false>;
        hipLaunchKernelGGL(wg, dim3((t1 + 3) / 4, kch), dim3(256), 0, s, X1, kFP, Y1, HP, kFP, HP, L.K,
                           wg_rows, part1);
        hipLaunchKernelGGL(wg, dim3((t2 + 3) / 4, kch), dim3(256), 0, s, X2, HP, Y2, HP, HP, HP, L.K,
                           wg_rows, part2);
      }
    }
    const int64_t n1 = (int64_t)kFP * HP, n2 = (int64_t)HP * HP;
    // [kFP][HP] and [HP][HP] partials summed straight into the caller's [F][H1] and [H1][H2]
    hipLaunchKernelGGL(sum_partials_unpad, dim3((kF * H1 + 255) / 256), dim3(256), 0, s, part1, kch, n1, HP,
                       kF, H1, g->W1);
    hipLaunchKernelGGL(sum_partials_unpad, dim3((H1 * H2 + 255) / 256), dim3(256), 0, s, part2, kch, n2, HP,
                       H1, H2, g->W2);
  }
  // bias, W3, scale/shift gradients: two-stage sums with chunk partials added in order
  float* cpart = (float*)(W + L.cpart);
  float* w3sum = (float*)(W + L.w3sum);
  double* spart = (double*)(W + L.spart);
  // (with no atoms there are no chunks: the sums of zero partials are zero)
  if (N > 0)
    hipLaunchKernelGGL(column_partials, dim3((H1 + 63) / 64, L.ccK), dim3(256), 0, s, Y1, HP, L.K, L.rcK, H1, true,
                       cpart);
  hipLaunchKernelGGL(sum_partials, dim3((H1 + 255) / 256), dim3(256), 0, s, cpart, L.ccK, (int64_t)H1, g->b1);
  if (N > 0)
    hipLaunchKernelGGL(column_partials, dim3((H2 + 63) / 64, L.ccK), dim3(256), 0, s, Y2, HP, L.K, L.rcK, H2, true,
                       cpart);
  hipLaunchKernelGGL(sum_partials, dim3((H2 + 255) / 256), dim3(256), 0, s, cpart, L.ccK, (int64_t)H2, g->b2);
  if (N > 0) {
    hipLaunchKernelGGL(column_partials, dim3((H2 + 63) / 64, L.ccN), dim3(256), 0, s, w3g, HP, (int64_t)N, L.rcN, H2,
                       false, cpart);
    hipLaunchKernelGGL(species_partials, dim3(L.sp_blocks), dim3(kSpeciesChunk), 0, s, m, sys, ebar, qsig, spart);
  }
  hipLaunchKernelGGL(sum_partials, dim3((H2 + 255) / 256), dim3(256), 0, s, cpart, L.ccN, (int64_t)H2, w3sum);
  hipLaunchKernelGGL(w3_broadcast, dim3((H2 + 255) / 256), dim3(256), 0, s, w3sum, H2, m.M, g->W3);
  hipLaunchKernelGGL(species_finish, dim3(1), dim3(64), 0, s, m, spart, L.sp_blocks, g->scale, g->shift, g->b3);
  hipLaunchKernelGGL(sum_partials, dim3((nslots + 255) / 256), dim3(256), 0, s, bpart, L.beta_blocks,
                     (int64_t)nslots, bsum);
  hipLaunchKernelGGL(beta_unpack, dim3((nsp * nsp * kS * m.K + 255) / 256), dim3(256), 0, s, bsum, nsp, m.K, g->beta);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

}  // namespace gmnn
