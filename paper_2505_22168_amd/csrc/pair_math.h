// Per-pair device math shared by the pair kernels and the fused tile kernel:
// lane exchanges, the radial basis, monomials of the unit vector, and the
// per-atom moment accumulation / pair backward loops.
#pragma once

#include "common.h"
#include "model.h"

namespace gmnn {

constexpr int kPairBlock = 256;  // threads per block of the pair kernels
constexpr int kHeadsAtoms = kPairBlock / 64;  // atoms per block of the per-head pair backward

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

// cross-row steps: v_permlane32_swap / v_permlane16_swap exchange the kept and
// sent halves in one instruction; the sum of the two outputs is the
// reduce-scatter result in every lane (lanes with the bit clear keep the low
// half, lanes with it set the high half)
template <int H, int ROWS>
__device__ inline void rs_swap(float* v) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const unsigned a = __float_as_uint(v[k]), b = __float_as_uint(v[k + H]);
    if (ROWS == 32) {
      const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
      v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
      const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
      v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
  }
}

// 128 values (100 live + 28 zero) per lane, summed over the LPA lanes of an
// atom.  LPA = 16: lane q of the row owns indices 8q..8q+7 (v[0..7]).
// LPA = 64: lane q of the wave owns indices 2q, 2q+1 (v[0..1]).
// LPA = 32: lane q of the half wave owns indices 4q .. 4q+3 (v[0..3]).
// LPA = 8: lane q of the half row owns indices 16q .. 16q+15 (v[0..15]).
template <int LPA>
__device__ inline void reduce_scatter_128(float* v, int q) {
  if (LPA == 8) {
    rs_step<64, 1>(v, (q >> 2) & 1);
    rs_step<32, 2>(v, (q >> 1) & 1);
    rs_step<16, 3>(v, q & 1);
    return;
  }
  if (LPA == 32) {
    rs_swap<64, 16>(v);
    rs_step<32, 0>(v, (q >> 3) & 1);
    rs_step<16, 1>(v, (q >> 2) & 1);
    rs_step<8, 2>(v, (q >> 1) & 1);
    rs_step<4, 3>(v, q & 1);
    return;
  }
  if (LPA == 64) {
    rs_swap<64, 32>(v);
    rs_swap<32, 16>(v);
    rs_step<16, 0>(v, (q >> 3) & 1);
    rs_step<8, 1>(v, (q >> 2) & 1);
    rs_step<4, 2>(v, (q >> 1) & 1);
    rs_step<2, 3>(v, q & 1);
  } else {
    rs_step<64, 0>(v, (q >> 3) & 1);
    rs_step<32, 1>(v, (q >> 2) & 1);
    rs_step<16, 2>(v, (q >> 1) & 1);
    rs_step<8, 3>(v, q & 1);
  }
}

// sum over the LPA lanes of an atom (every lane gets the total)
template <int LPA>
__device__ inline float atom_sum(float v) {
  if (LPA == 8) {
    v += dpp_half_mirror(v);
    v += dpp_xor2(v);
    v += dpp_xor1(v);
    return v;
  }
  v = row16_sum(v);
  if (LPA >= 32) v += lane_xor16(v);
  if (LPA == 64) v += lane_xor32(v);
  return v;
}

// --- radial basis ------------------------------------------------------------
struct Radial {
  float R[kS];    // c * f_c(r) * sum_k beta[s][k] g_k(r)
  float dR[kS];   // d R_s / dr
};

// r and 1/r from r^2 with the hardware reciprocal square root (within 1 ulp)
__device__ inline void length_of(float r2, float& r, float& ir) {
  ir = __builtin_amdgcn_rsqf(r2);
  r = r2 * ir;
}

// cosine cutoff f_c(r) = (cos(pi r / r_c) + 1) / 2 and sin(pi r / r_c), from
// the hardware sine and cosine (argument in revolutions: r / (2 r_c); within
// about 1.3e-7 absolute on [0, 1/2])
__device__ inline void cutoff_cos_sin(const DevModel& m, float r, float& cs, float& sn) {
  const float rev = r * m.half_inv_rc;
  cs = __builtin_amdgcn_cosf(rev);
  sn = __builtin_amdgcn_sinf(rev);
}

// Basis functions g_k (k < kMaxBasis; zero for k >= K) and, with DERIV, their
// derivatives dg_k/dr, given cs, sn = cos, sin of x = pi r / r_c (the cutoff's
// argument):
//   Gaussians    g_k = exp(-gamma (r - mu_k)^2), mu_k = r_min + k delta, by
//                the recurrence g_k = g_0 a^k exp(-gamma delta^2 k^2) with
//                a = exp(2 gamma delta tau) (two exponentials per pair);
//   Bessel-like  g_n = a_n [sinc((n+1) x) + sinc((n+2) x)] with sin(kx) and
//                cos(kx) by the Chebyshev recurrence from (cs, sn): no further
//                transcendental; d/dr sinc(kx) = (cos(kx) - sinc(kx)) / r.
// m.ck holds the per-order constants (exp(-gamma delta^2 k^2), or a_n).
template <bool DERIV>
__device__ inline void basis_values(const DevModel& m, float r, float cs, float sn, float (&g)[kMaxBasis],
                                    float (&dg)[kMaxBasis]) {
  if (m.basis == GMNN_BASIS_BESSEL) {
    const float ir = 1.0f / r;
    const float ix = m.rc_over_pi * ir;  // 1 / x
    // orders k = n + 1 (a) and n + 2 (b), advanced together
    float sa = sn, ca = cs;
    float sb = 2.0f * cs * sn, cb = 2.0f * cs * cs - 1.0f;
    float sinc_a = sa * ix;
#pragma unroll
    for (int n = 0; n < kMaxBasis; ++n) {
      const float sinc_b = sb * ix * (1.0f / (float)(n + 2));
      g[n] = m.ck[n] * (sinc_a + sinc_b);
      if (DERIV) dg[n] = m.ck[n] * ((ca - sinc_a) + (cb - sinc_b)) * ir;
      const float sc = 2.0f * cs * sb - sa, cc = 2.0f * cs * cb - ca;
      sa = sb; ca = cb; sb = sc; cb = cc;
      sinc_a = sinc_b;
    }
    return;
  }
  const float tau = r - m.r_min;
  const float g0 = __expf(-m.gamma * tau * tau);
  const float a = __expf(2.0f * m.gamma * m.delta * tau);
  float p = g0;
#pragma unroll
  for (int k = 0; k < kMaxBasis; ++k) {
    g[k] = p * m.ck[k];  // ck[k] = exp(-gamma delta^2 k^2), zero for k >= K
    if (DERIV) dg[k] = -2.0f * m.gamma * (tau - (float)k * m.delta) * g[k];
    p *= a;
  }
}

// The same basis functions one order at a time (next() gives g_k, dg_k/dr
// for k = 0, 1, ...), for one basis fixed at compile time: the arithmetic of
// basis_values<true> without arrays, for kernels short of registers.
template <int BASIS>
struct BasisIter {
  float p, a, tau, ir, ix, cs2, sa, ca, sb, cb, sinc_a;
  __device__ BasisIter(const DevModel& m, float r, float cs, float sn) {
    if (BASIS == GMNN_BASIS_BESSEL) {
      ir = 1.0f / r;
      ix = m.rc_over_pi * ir;
      cs2 = 2.0f * cs;
      sa = sn; ca = cs;
      sb = 2.0f * cs * sn; cb = 2.0f * cs * cs - 1.0f;
      sinc_a = sa * ix;
    } else {
      tau = r - m.r_min;
      p = __expf(-m.gamma * tau * tau);
      a = __expf(2.0f * m.gamma * m.delta * tau);
    }
  }
  // order k (the calls go k = 0, 1, ... in turn)
  __device__ __forceinline__ void next(const DevModel& m, int k, float& g, float& dg) {
    if (BASIS == GMNN_BASIS_BESSEL) {
      const float sinc_b = sb * ix * (1.0f / (float)(k + 2));
      g = m.ck[k] * (sinc_a + sinc_b);
      dg = m.ck[k] * ((ca - sinc_a) + (cb - sinc_b)) * ir;
      const float sc = cs2 * sb - sa, cc = cs2 * cb - ca;
      sa = sb; ca = cb; sb = sc; cb = cc;
      sinc_a = sinc_b;
    } else {
      g = p * m.ck[k];
      dg = -2.0f * m.gamma * (tau - (float)k * m.delta) * g;
      p *= a;
    }
  }
};

// R_s = c f_c(r) sum_k beta[s][k] g_k(r) (and dR_s/dr with DERIV)
template <bool DERIV>
__device__ inline void radial(const DevModel& m, const float* __restrict__ bz /*[S][8]*/, float r, Radial& out) {
  float sn, cs;
  cutoff_cos_sin(m, r, cs, sn);
  float g[kMaxBasis], dg[kMaxBasis];
  basis_values<DERIV>(m, r, cs, sn, g, dg);
  const float fc = 0.5f * (cs + 1.0f) * m.psi_scale;
  const float dfc = -0.5f * (3.14159265358979f / m.r_cut) * sn * m.psi_scale;
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    float B = 0.0f, dB = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxBasis; ++k) {
      const float bk = bz[s * kMaxBasis + k];
      B += bk * g[k];
      if (DERIV) dB += bk * dg[k];
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

// d_p = x_j - x_i + S . h (FP32) of the pair with neighbour j, image code sh
__device__ inline void pair_vec_of(const AtomCtx& c, float xj, float yj, float zj, int32_t sh, float& dx, float& dy,
                                   float& dz) {
  int sx, sy, sz;
  unpack_shift(sh, sx, sy, sz);
  const float fx = (float)sx, fy = (float)sy, fz = (float)sz;
  dx = (xj - c.xi) + (fx * c.h[0] + fy * c.h[3] + fz * c.h[6]);
  dy = (yj - c.yi) + (fx * c.h[1] + fy * c.h[4] + fz * c.h[7]);
  dz = (zj - c.zi) + (fx * c.h[2] + fy * c.h[5] + fz * c.h[8]);
}

// d_p of pair p of the row
__device__ inline void pair_vec(const DevSystem& sys, const AtomCtx& c, int64_t p, int& j, float& dx, float& dy,
                                float& dz) {
  j = sys.nj[p];
  pair_vec_of(c, sys.pos[3 * (int64_t)j], sys.pos[3 * (int64_t)j + 1], sys.pos[3 * (int64_t)j + 2], sys.nshift[p], dx,
              dy, dz);
}

// The lane's pairs are taken U at a time with every load of the group issued
// before any arithmetic (neighbour index and image code, then the neighbour's
// position and species): one memory round trip per group, not per pair.
constexpr int kPairUnroll = 2;
struct PairGroup {
  float dx[kPairUnroll], dy[kPairUnroll], dz[kPairUnroll];
  int zj[kPairUnroll];
  bool ok[kPairUnroll];
};

template <int LPA>
__device__ inline void fetch_pairs(const DevSystem& sys, const AtomCtx& c, int64_t p, PairGroup& g) {
  int j[kPairUnroll];
  int32_t sh[kPairUnroll];
#pragma unroll
  for (int u = 0; u < kPairUnroll; ++u) {
    const int64_t pu = p + (int64_t)u * LPA;
    g.ok[u] = pu < c.p1;
    j[u] = g.ok[u] ? sys.nj[pu] : 0;
    sh[u] = g.ok[u] ? sys.nshift[pu] : 0;
  }
  float x[kPairUnroll], y[kPairUnroll], z[kPairUnroll];
#pragma unroll
  for (int u = 0; u < kPairUnroll; ++u) {
    x[u] = g.ok[u] ? sys.pos[3 * (int64_t)j[u]] : 0.0f;
    y[u] = g.ok[u] ? sys.pos[3 * (int64_t)j[u] + 1] : 0.0f;
    z[u] = g.ok[u] ? sys.pos[3 * (int64_t)j[u] + 2] : 0.0f;
    g.zj[u] = g.ok[u] ? sys.species[j[u]] : 0;
  }
#pragma unroll
  for (int u = 0; u < kPairUnroll; ++u) pair_vec_of(c, x[u], y[u], z[u], sh[u], g.dx[u], g.dy[u], g.dz[u]);
}

// Optional LDS cache of an atom's context and of the first pair group of each
// of its lanes, written by atom_moments and read back by atom_pair_backward
// (the fused tile runs both on the same lanes): the backward then starts
// without a global-memory round trip.  pv[q * kPairUnroll + u] = (d, zj) with
// zj = -1 for a slot past the end of the row.
struct PairCache {
  AtomCtx* ctx;  // one per atom
  float4* pv;    // [LPA][kPairUnroll] per atom
};

// ---------------------------------------------------------------------------
// moment partial sums of lane q of an atom: pairs p0+q, p0+q+LPA, ...
// v[s*20 + t] += R_s(r) mono_t(u)   (v must be zeroed by the caller).
// atom_moments_from takes the atom's context and the lane's first pair group
// already loaded (a caller can issue those loads early); atom_moments loads
// them itself.
template <int LPA>
__device__ inline void atom_moments_from(const DevModel& m, const DevSystem& sys, const float* __restrict__ s_beta,
                                         const AtomCtx& c, int q, const PairGroup& first, float (&v)[128],
                                         PairCache cache = PairCache{nullptr, nullptr}) {
  if (cache.ctx && q == 0) *cache.ctx = c;
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  for (int64_t p = c.p0 + q; p < c.p1; p += kPairUnroll * LPA) {
    PairGroup g;
    if (p == c.p0 + q) g = first;
    else fetch_pairs<LPA>(sys, c, p, g);
    if (cache.pv && p == c.p0 + q) {
#pragma unroll
      for (int u = 0; u < kPairUnroll; ++u)
        cache.pv[q * kPairUnroll + u] = make_float4(g.dx[u], g.dy[u], g.dz[u], __int_as_float(g.ok[u] ? g.zj[u] : -1));
    }
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) {
      const float dx = g.dx[u], dy = g.dy[u], dz = g.dz[u];
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (!g.ok[u]) continue;
      if (!(r2 < m.rc2) || r2 == 0.0f) {
        // a listed pair at zero distance, or with a non-finite separation (a
        // non-finite position), is left out and flagged
        if (sys.status && r2 == 0.0f) raise_flag(sys.status, GMNN_FLAG_COINCIDENT);
        if (sys.status && !(r2 <= 3.402823466e38f)) raise_flag(sys.status, GMNN_FLAG_NONFINITE);
        continue;
      }
      float r, ir;
      length_of(r2, r, ir);
      Radial rad;
      radial<false>(m, bzi + g.zj[u] * kS * kMaxBasis, r, rad);
      float mo[20];
      monomials(dx * ir, dy * ir, dz * ir, mo);
#pragma unroll
      for (int s = 0; s < kS; ++s)
#pragma unroll
        for (int t = 0; t < kPacked; ++t) v[s * kPacked + t] += rad.R[s] * mo[t];
    }
  }
}

template <int LPA>
__device__ inline void atom_moments(const DevModel& m, const DevSystem& sys, const float* __restrict__ s_beta, int i,
                                    int q, float (&v)[128], PairCache cache = PairCache{nullptr, nullptr}) {
  AtomCtx c;
  load_atom(sys, i, c);
  PairGroup g;
  fetch_pairs<LPA>(sys, c, c.p0 + q, g);
  atom_moments_from<LPA>(m, sys, s_beta, c, q, g, v, cache);
}

// dE/dd_p of one pair from dE_i/dPsi_i (pb, packed components, each an
// independent variable) and the pair's radial basis and monomials.  With
// P_s(u) = sum_t pb[s][t] mono_t(u) and Q(u) = sum_s R_s P_s(u):
//   g = (sum_s dR_s/dr P_s(u)) u + (grad Q - (grad Q . u) u) / r
// pb is indexed as pb[k]: a register array or an LDS pointer.
template <class PB>
__device__ __forceinline__ void pair_gradient(const PB& pb, const Radial& rad, const float (&mo)[20], float x, float y,
                                              float z, float ir, float& gx, float& gy, float& gz) {
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
  const float Gx = qc[1] + 2.0f * qc[4] * x + qc[5] * y + qc[6] * z + 3.0f * qc[10] * x * x +
                   2.0f * qc[11] * x * y + 2.0f * qc[12] * x * z + qc[13] * y * y + qc[14] * y * z +
                   qc[15] * z * z;
  const float Gy = qc[2] + qc[5] * x + 2.0f * qc[7] * y + qc[8] * z + qc[11] * x * x +
                   2.0f * qc[13] * x * y + qc[14] * x * z + 3.0f * qc[16] * y * y + 2.0f * qc[17] * y * z +
                   qc[18] * z * z;
  const float Gz = qc[3] + qc[6] * x + qc[8] * y + 2.0f * qc[9] * z + qc[12] * x * x + qc[14] * x * y +
                   2.0f * qc[15] * x * z + qc[17] * y * y + 2.0f * qc[18] * y * z + 3.0f * qc[19] * z * z;
  const float gu = Gx * x + Gy * y + Gz * z;
  gx = radial_part * x + (Gx - gu * x) * ir;
  gy = radial_part * y + (Gy - gu * y) * ir;
  gz = radial_part * z + (Gz - gu * z) * ir;
}

// dE/dd_p for every pair of lane q of atom i, given pb = dE_i/dPsi_i.
// Writes g_p and accumulates this lane's share of sum_p g_p (x) d_p into vir.
template <int LPA>
__device__ inline void atom_pair_backward(const DevModel& m, const DevSystem& sys, const float* __restrict__ s_beta,
                                          int i, int q, const float (&pb)[kS * kPacked], float* __restrict__ gpair,
                                          float (&vir)[9], PairCache cache = PairCache{nullptr, nullptr}) {
  AtomCtx c;
  if (cache.ctx) c = *cache.ctx;
  else load_atom(sys, i, c);
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  for (int64_t p = c.p0 + q; p < c.p1; p += kPairUnroll * LPA) {
    PairGroup g;
    if (cache.pv && p == c.p0 + q) {
#pragma unroll
      for (int u = 0; u < kPairUnroll; ++u) {
        const float4 e = cache.pv[q * kPairUnroll + u];
        g.dx[u] = e.x;
        g.dy[u] = e.y;
        g.dz[u] = e.z;
        g.zj[u] = __float_as_int(e.w);
        g.ok[u] = g.zj[u] >= 0;
      }
    } else {
      fetch_pairs<LPA>(sys, c, p, g);
    }
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) {
      if (!g.ok[u]) continue;
      const float dx = g.dx[u], dy = g.dy[u], dz = g.dz[u];
      const float r2 = dx * dx + dy * dy + dz * dz;
      float gx = 0.0f, gy = 0.0f, gz = 0.0f;
      if (r2 < m.rc2 && r2 > 0.0f) {
        float r, ir;
        length_of(r2, r, ir);
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        Radial rad;
        radial<true>(m, bzi + g.zj[u] * kS * kMaxBasis, r, rad);
        float mo[20];
        monomials(ux, uy, uz, mo);
        pair_gradient(pb, rad, mo, ux, uy, uz, ir, gx, gy, gz);
        vir[0] += gx * dx; vir[1] += gx * dy; vir[2] += gx * dz;
        vir[3] += gy * dx; vir[4] += gy * dy; vir[5] += gy * dz;
        vir[6] += gz * dx; vir[7] += gz * dy; vir[8] += gz * dz;
      }
      const int64_t pu = p + (int64_t)u * LPA;
      gpair[3 * pu] = gx;
      gpair[3 * pu + 1] = gy;
      gpair[3 * pu + 2] = gz;
    }
  }
}

// The same for nh heads at once (one backward per head): each pair's
// geometry, radial basis and monomials are computed once and serve every
// head; pbh = dE_i^h/dPsi_i for head h at pbh + h * 100 (LDS).  Head h's
// gradients go to gpair + h * gstride * 3; vir accumulates the sum over
// heads.  Per head the arithmetic is atom_pair_backward's.
// hw (may be null): per-head weights of the virial (sum_h hw[h] g^h (x) d);
// null: the plain sum over heads
template <int LPA>
__device__ inline void atom_pair_backward_heads(const DevModel& m, const DevSystem& sys,
                                                const float* __restrict__ s_beta, int i, int q,
                                                const float* __restrict__ pbh, int nh, float* __restrict__ gpair,
                                                int64_t gstride, float (&vir)[9], const float* hw = nullptr) {
  AtomCtx c;
  load_atom(sys, i, c);
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  for (int64_t p = c.p0 + q; p < c.p1; p += kPairUnroll * LPA) {
    PairGroup g;
    fetch_pairs<LPA>(sys, c, p, g);
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) {
      if (!g.ok[u]) continue;
      const float dx = g.dx[u], dy = g.dy[u], dz = g.dz[u];
      const float r2 = dx * dx + dy * dy + dz * dz;
      const int64_t pu = p + (int64_t)u * LPA;
      if (r2 < m.rc2 && r2 > 0.0f) {
        float r, ir;
        length_of(r2, r, ir);
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        Radial rad;
        radial<true>(m, bzi + g.zj[u] * kS * kMaxBasis, r, rad);
        float mo[20];
        monomials(ux, uy, uz, mo);
        for (int h = 0; h < nh; ++h) {
          float gx, gy, gz;
          pair_gradient(pbh + h * (kS * kPacked), rad, mo, ux, uy, uz, ir, gx, gy, gz);
          const float wv = hw ? hw[h] : 1.0f;
          const float vx = wv * gx, vy = wv * gy, vz = wv * gz;
          vir[0] += vx * dx; vir[1] += vx * dy; vir[2] += vx * dz;
          vir[3] += vy * dx; vir[4] += vy * dy; vir[5] += vy * dz;
          vir[6] += vz * dx; vir[7] += vz * dy; vir[8] += vz * dz;
          float* gp = gpair + (int64_t)h * gstride * 3;
          gp[3 * pu] = gx;
          gp[3 * pu + 1] = gy;
          gp[3 * pu + 2] = gz;
        }
      } else {
        for (int h = 0; h < nh; ++h) {
          float* gp = gpair + (int64_t)h * gstride * 3;
          gp[3 * pu] = 0.0f;
          gp[3 * pu + 1] = 0.0f;
          gp[3 * pu + 2] = 0.0f;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Compacted pair loops (split schedule).  A list built with a skin holds
// pairs beyond r_c (about a third of them at r_c 6 A + 1 A skin); in a
// lane-per-pair loop their lanes would idle through the whole pair
// computation.  Here each group of LPA lanes tests LPA candidates at a time
// and appends the pairs inside r_c to the group's LDS ring of kRingBatches
// LPA entries (ballot and prefix count, in candidate order).  The pair
// computation runs on queued pairs when every group of the wave still in its
// row has LPA of them (a full batch each: the wave's lanes all busy), or
// when some group's ring could not take another chunk; the remainder runs
// after the row.  The decision is wave-wide because the wave executes the
// computation whenever any of its groups does.  A ring entry is (d, tag),
// tag = zj | (p - p0) << 5.  The ring stays within one wave (the group's
// lanes), so wave-level ordering of its LDS accesses is all it needs.
constexpr int kRingTagBits = 5;  // species index bits of a ring tag (kMaxSpecies <= 32)
constexpr int kRingBatches = 4;  // ring entries per lane of a group

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the group's bits of a wave ballot, bit q = lane q of the group
template <int LPA>
__device__ inline uint64_t group_ballot(bool v) {
  const uint64_t bal = __ballot(v);
  if (LPA == 64) return bal;
  const int shift = lane_id() & (64 - LPA);
  return (bal >> shift) & ((1ull << LPA) - 1ull);
}

// Candidate chunks are fetched ahead: the pair backward keeps the neighbour
// positions and species of chunk k + 1 and the neighbour indices of chunk
// k + 2 in flight while chunk k is tested; the moments (short of registers)
// the indices of chunk k + 1 only.
struct Cand {
  float x, y, z;
  int sp;
  int32_t sh;
};
struct CandIdx {
  int j;
  int32_t sh;
};
__device__ __forceinline__ CandIdx cand_index(const DevSystem& sys, const AtomCtx& c, int64_t p) {
  CandIdx r{0, 0};
  if (p < c.p1) {
    r.j = sys.nj[p];
    r.sh = sys.nshift[p];
  }
  return r;
}
__device__ __forceinline__ Cand cand_fetch(const DevSystem& sys, const AtomCtx& c, int64_t p, CandIdx ix) {
  Cand r{0.0f, 0.0f, 0.0f, 0, ix.sh};
  if (p < c.p1) {
    r.x = sys.pos[3 * (int64_t)ix.j];
    r.y = sys.pos[3 * (int64_t)ix.j + 1];
    r.z = sys.pos[3 * (int64_t)ix.j + 2];
    r.sp = sys.species[ix.j];
  }
  return r;
}

// one candidate chunk: lane q tests pair pc + q (its neighbour fetched
// ahead); accepted pairs are appended to the ring (tail advances by their
// count); rejected ones inside the row are reported through `rejected`.
// Flags as atom_moments_from raises them.
template <int LPA>
__device__ __forceinline__ void ring_append(const DevModel& m, const DevSystem& sys, const AtomCtx& c, int q,
                                            int64_t pc, const Cand& cd, float4* __restrict__ ring, int& tail,
                                            bool& rejected) {
  const bool have = pc + q < c.p1;
  bool ok = false;
  float dx = 0.0f, dy = 0.0f, dz = 0.0f;
  if (have) {
    pair_vec_of(c, cd.x, cd.y, cd.z, cd.sh, dx, dy, dz);
    const float r2 = dx * dx + dy * dy + dz * dz;
    ok = r2 < m.rc2 && r2 > 0.0f;
    if (sys.status && r2 == 0.0f) raise_flag(sys.status, GMNN_FLAG_COINCIDENT);
    if (sys.status && !(r2 <= 3.402823466e38f)) raise_flag(sys.status, GMNN_FLAG_NONFINITE);
  }
  rejected = have && !ok;
  const uint64_t gb = group_ballot<LPA>(ok);
  const int pre = __popcll(gb & ((1ull << q) - 1ull));
  if (ok)
    ring[(tail + pre) & (kRingBatches * LPA - 1)] =
        make_float4(dx, dy, dz, __int_as_float(cd.sp | (int)(pc + q - c.p0) << kRingTagBits));
  tail += __popcll(gb);
  wave_lds_sync();
}

// one batch of queued pairs if the wave-wide rule calls for it (or always,
// with `flush`, for the remainder after the row): each group takes up to LPA
// entries, lane q the q-th
template <int LPA, class F>
__device__ __forceinline__ void ring_drain(int q, const float4* __restrict__ ring, int& head, int tail, bool flush,
                                           F&& process) {
  const int avail = tail - head;
  if (!flush) {
    const bool some_short = __ballot(avail < LPA) != 0;
    const bool some_full = __ballot(avail > (kRingBatches - 1) * LPA) != 0;
    if (some_short && !some_full) return;
  }
  const int take = avail < LPA ? avail : LPA;
  if (q < take) process(ring[(head + q) & (kRingBatches * LPA - 1)]);
  head += take;
  wave_lds_sync();
}

// moment partial sums of lane q of an atom over the pairs inside r_c (the
// accumulation of atom_moments_from, on compacted pairs)
template <int LPA>
__device__ inline void atom_moments_compact(const DevModel& m, const DevSystem& sys, const float* __restrict__ s_beta,
                                            const AtomCtx& c, int q, float4* __restrict__ ring, float (&v)[128]) {
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  auto process = [&](float4 e) {
    const float dx = e.x, dy = e.y, dz = e.z;
    const int zj = __float_as_int(e.w) & ((1 << kRingTagBits) - 1);
    const float r2 = dx * dx + dy * dy + dz * dz;
    float r, ir;
    length_of(r2, r, ir);
    Radial rad;
    radial<false>(m, bzi + zj * kS * kMaxBasis, r, rad);
    float mo[20];
    monomials(dx * ir, dy * ir, dz * ir, mo);
#pragma unroll
    for (int s = 0; s < kS; ++s)
#pragma unroll
      for (int t = 0; t < kPacked; ++t) v[s * kPacked + t] += rad.R[s] * mo[t];
  };
  // one stage of prefetch only (the neighbour indices of the next chunk): the
  // deeper pipeline of the backward costs this kernel a wave per SIMD
  int head = 0, tail = 0;
  CandIdx nxt = cand_index(sys, c, c.p0 + q);
  for (int64_t pc = c.p0; pc < c.p1; pc += LPA) {
    const Cand cd = cand_fetch(sys, c, pc + q, nxt);
    nxt = cand_index(sys, c, pc + LPA + q);
    bool rejected;
    ring_append<LPA>(m, sys, c, q, pc, cd, ring, tail, rejected);
    ring_drain<LPA>(q, ring, head, tail, false, process);
  }
  while (tail > head) ring_drain<LPA>(q, ring, head, tail, true, process);
}

// dE/dd_p for every pair of an atom's row on compacted pairs (the arithmetic
// of atom_pair_backward): pairs outside r_c get g_p = 0 at once, the others
// when their batch runs.  Accumulates lane q's share of the virial.
template <int LPA>
__device__ inline void atom_pair_backward_compact(const DevModel& m, const DevSystem& sys,
                                                  const float* __restrict__ s_beta, const AtomCtx& c, int q,
                                                  const float (&pb)[kS * kPacked], float4* __restrict__ ring,
                                                  float* __restrict__ gpair, float (&vir)[9]) {
  const float* bzi = s_beta + c.zsp * m.n_species * kS * kMaxBasis;
  auto process = [&](float4 e) {
    const float dx = e.x, dy = e.y, dz = e.z;
    const int tag = __float_as_int(e.w);
    const int zj = tag & ((1 << kRingTagBits) - 1);
    const int64_t p = c.p0 + (tag >> kRingTagBits);
    const float r2 = dx * dx + dy * dy + dz * dz;
    float r, ir;
    length_of(r2, r, ir);
    const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
    Radial rad;
    radial<true>(m, bzi + zj * kS * kMaxBasis, r, rad);
    float mo[20];
    monomials(ux, uy, uz, mo);
    float gx, gy, gz;
    pair_gradient(pb, rad, mo, ux, uy, uz, ir, gx, gy, gz);
    vir[0] += gx * dx; vir[1] += gx * dy; vir[2] += gx * dz;
    vir[3] += gy * dx; vir[4] += gy * dy; vir[5] += gy * dz;
    vir[6] += gz * dx; vir[7] += gz * dy; vir[8] += gz * dz;
    gpair[3 * p] = gx;
    gpair[3 * p + 1] = gy;
    gpair[3 * p + 2] = gz;
  };
  int head = 0, tail = 0;
  Cand cur = cand_fetch(sys, c, c.p0 + q, cand_index(sys, c, c.p0 + q));
  CandIdx nxt = cand_index(sys, c, c.p0 + LPA + q);
  for (int64_t pc = c.p0; pc < c.p1; pc += LPA) {
    const Cand cd = cur;
    cur = cand_fetch(sys, c, pc + LPA + q, nxt);
    nxt = cand_index(sys, c, pc + 2 * LPA + q);
    bool rejected;
    ring_append<LPA>(m, sys, c, q, pc, cd, ring, tail, rejected);
    if (rejected) {
      const int64_t p = pc + q;
      gpair[3 * p] = 0.0f;
      gpair[3 * p + 1] = 0.0f;
      gpair[3 * p + 2] = 0.0f;
    }
    ring_drain<LPA>(q, ring, head, tail, false, process);
  }
  while (tail > head) ring_drain<LPA>(q, ring, head, tail, true, process);
}

}  // namespace gmnn
