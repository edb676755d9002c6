// Device-side view of a model and the layout of its packed weight buffer.
#pragma once

#include "common.h"
#include "tables.h"

namespace gmnn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kMaxSpecies = 16;
constexpr int kMaxBasis = 8;
constexpr int kMaxHeads = 16;

// Offsets (bytes) of the packed buffer filled by gmnn_model_prepare.
//   fp32 MFMA B fragments (16x16x4):  [n/16][k/4][64] floats
//   bf16 MFMA B fragments (16x16x32): [n/16][k/32][64][8] bf16
//   W1 and W2 (the forward products) also carry a low part in the bf16
//   layout: lo = bf16(w - hi) with hi = bf16(w), so hi + lo holds w to about
//   16 significant bits (the split-BF16 forward products)
// Hidden widths are padded to HP (multiple of 64) with zero weights and
// biases, which leaves every output unchanged (swish(0) = 0).
struct PackedLayout {
  int HP1 = 0, HP2 = 0, M = 0;
  size_t w1_f32 = 0, w1t_f32 = 0, w2_f32 = 0, w2t_f32 = 0;
  size_t w1_bf16 = 0, w1t_bf16 = 0, w2_bf16 = 0, w2t_bf16 = 0;
  size_t w1lo_bf16 = 0, w2lo_bf16 = 0;
  size_t b1 = 0, b2 = 0, w3 = 0, w3bar = 0, b3 = 0;
  size_t bytes = 0;
};

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

inline PackedLayout packed_layout(int H1, int H2, int M) {
  PackedLayout L;
  L.HP1 = round_up(H1, 64);
  L.HP2 = round_up(H2, 64);
  L.M = M;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.w1_f32 = take(4 * (size_t)kFP * L.HP1);
  L.w1t_f32 = take(4 * (size_t)kFP * L.HP1);
  L.w2_f32 = take(4 * (size_t)L.HP1 * L.HP2);
  L.w2t_f32 = take(4 * (size_t)L.HP1 * L.HP2);
  L.w1_bf16 = take(2 * (size_t)kFP * L.HP1);
  L.w1t_bf16 = take(2 * (size_t)kFP * L.HP1);
  L.w2_bf16 = take(2 * (size_t)L.HP1 * L.HP2);
  L.w2t_bf16 = take(2 * (size_t)L.HP1 * L.HP2);
  L.w1lo_bf16 = take(2 * (size_t)kFP * L.HP1);
  L.w2lo_bf16 = take(2 * (size_t)L.HP1 * L.HP2);
  L.b1 = take(4 * (size_t)L.HP1);
  L.b2 = take(4 * (size_t)L.HP2);
  L.w3 = take(4 * (size_t)L.HP2 * M);
  L.w3bar = take(4 * (size_t)L.HP2);
  L.b3 = take(4 * (size_t)M);
  L.bytes = off;
  return L;
}

// Kernel-argument view of the model (plain pointers, by value).
struct DevModel {
  int n_species, K, HP1, HP2, M;
  float r_min, r_cut, rc2, gamma, delta, psi_scale;
  float half_inv_rc;    // 0.5 / r_cut: the cutoff's cosine argument in revolutions
  float rc_over_pi;     // r_cut / pi
  int basis;            // GMNN_BASIS_GAUSSIAN or GMNN_BASIS_BESSEL
  float ck[8];          // per-order basis constants for k < K (0 beyond): Gaussians
                        // exp(-gamma delta^2 k^2), Bessel-like a_k
  const float* beta;    // [nsp][nsp][S][K]
  const float* scale;   // [nsp]
  const float* shift;   // [nsp]
  const float* w1_f32;
  const float* w1t_f32;
  const float* w2_f32;
  const float* w2t_f32;
  const bf16x8* w1_bf16;
  const bf16x8* w1t_bf16;
  const bf16x8* w2_bf16;
  const bf16x8* w2t_bf16;
  const bf16x8* w1lo_bf16;  // low parts of the forward weights (split products)
  const bf16x8* w2lo_bf16;
  const float* b1;      // [HP1]
  const float* b2;      // [HP2]
  const float* w3;      // [HP2][M]
  const float* w3bar;   // [HP2] mean over heads of W3
  const float* b3;      // [M]
  // uncertainty-driven bias: per-structure output weights [B][HP2] replacing
  // the head mean of W3 in the backward (sum_m c_m W3[:, m]); null: the mean
  const float* head_w;
  int fwd_only;         // readout kernels stop after the energies (no backward)
  float* h2_out;        // [N][HP2] second hidden layer's activations, written when set
};

// System view shared by the energy kernels.
struct DevSystem {
  int n_atoms, n_structs;
  const float* pos;
  const int32_t* species;
  const double* cell;
  const int64_t* atom_ptr;
  const int32_t* atom_struct;
  const int64_t* row_ptr;
  const int32_t* nj;
  const int32_t* nshift;
  const int32_t* rev;
  uint32_t* status;  // device status word (GMNN_FLAG_*), may be null
};

}  // namespace gmnn
