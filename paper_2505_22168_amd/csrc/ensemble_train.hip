// Shallow-ensemble training step (Section 2.2, eq. nll; Section 3.4):
//
//   loss_energy / loss_force   per-structure and per-component loss terms
//                   over the heads' predictions (squared error, Gaussian NLL
//                   or Gaussian CRPS of the mean against the reference, with
//                   the heads' population variance), their per-head
//                   derivatives, and block partials of the term sums
//   loss_finish     the two terms summed in block order (FP64)
//   adam_update     one Adam step over all parameter arrays, one learning
//                   rate per parameter group
//   head_view / head_accumulate
//                   per-head double backward: the head's W3 column as a
//                   one-head model, and the head's gradients added into the
//                   result in head order
//
// Derivatives of one term l(xbar, s2) with u = xbar - x_ref, s2 = variance
// + floor, s = sqrt(s2), z = |u| / s:
//   squared error  dl/dxbar = 2u,                  dl/ds2 = 0
//   NLL            dl/dxbar = u / s2,              dl/ds2 = (1/s2 - u^2/s2^2) / 2
//   CRPS           dl/dxbar = 2 Phi(u/s) - 1 = erf(u / (s sqrt 2)),
//                  dl/ds2  = (2 phi(z) - 1/sqrt(pi)) / (2 s)
// (for the CRPS the derivative of z (2 Phi(z) - 1) + 2 phi(z) in z is
// 2 Phi(z) - 1, since phi'(z) = -z phi(z)); with xbar = mean_m x^m and
// s2 = (1/M) sum_m (x^m - xbar)^2 + floor,
//   dl/dx^m = (dl/dxbar + 2 dl/ds2 (x^m - xbar)) / M.
#include <cmath>

#include "common.h"
#include "model.h"

namespace gmnn {

constexpr int kLossBlock = 256;

struct TermGrad {
  double l, dmean, dvar;
};

__device__ inline TermGrad loss_term(int kind, double u, double s2) {
  constexpr double kInvSqrtPi = 0.56418958354775628695;
  constexpr double kInvSqrt2 = 0.70710678118654752440;
  constexpr double kInvSqrt2Pi = 0.39894228040143267794;
  constexpr double kLog2Pi = 1.83787706640934548356;
  TermGrad t;
  if (kind == GMNN_LOSS_NLL) {
    t.l = 0.5 * (u * u / s2 + log(s2) + kLog2Pi);
    t.dmean = u / s2;
    t.dvar = 0.5 * (1.0 / s2 - u * u / (s2 * s2));
  } else if (kind == GMNN_LOSS_CRPS) {
    const double s = sqrt(s2);
    const double z = fabs(u) / s;
    const double phi = kInvSqrt2Pi * exp(-0.5 * z * z);
    const double e = erf(z * kInvSqrt2);  // 2 Phi(z) - 1
    t.l = s * (z * e + 2.0 * phi - kInvSqrtPi);
    t.dmean = u < 0.0 ? -e : e;
    t.dvar = (2.0 * phi - kInvSqrtPi) / (2.0 * s);
  } else {
    t.l = u * u;
    t.dmean = 2.0 * u;
    t.dvar = 0.0;
  }
  return t;
}

// fixed-order block sum: wave sums, then the waves' values in wave order
__device__ inline double block_sum(double v) {
  __shared__ double w[kLossBlock / 64];
  v = wave_sum(v);
  if (lane_id() == 0) w[threadIdx.x / 64] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kLossBlock / 64; ++k) s += w[k];
  return s;
}

// thread per structure: dL/dE_b^m and the block's sum of l_b
__global__ void __launch_bounds__(kLossBlock) loss_energy(gmnn_loss spec, int B, int M,
                                                          const int64_t* __restrict__ atom_ptr,
                                                          const double* __restrict__ energy,
                                                          const double* __restrict__ eref, double* __restrict__ dE,
                                                          double* __restrict__ part) {
  const int b = blockIdx.x * kLossBlock + threadIdx.x;
  double l = 0.0;
  // a structure without atoms has no per-atom energy: with energy_per_atom
  // it adds nothing (and gets zero gradients)
  const double na = b < B ? (double)(atom_ptr[b + 1] - atom_ptr[b]) : 0.0;
  if (b < B && spec.energy_per_atom && na == 0.0 && dE)
    for (int h = 0; h < M; ++h) dE[(int64_t)b * M + h] = 0.0;
  if (b < B && !(spec.energy_per_atom && na == 0.0)) {
    const double div = spec.energy_per_atom ? na : 1.0;
    double x[kMaxHeads];
    double mean = 0.0;
    for (int h = 0; h < M; ++h) {
      x[h] = energy[(int64_t)b * M + h] / div;
      mean += x[h];
    }
    mean /= (double)M;
    double var = 0.0;
    for (int h = 0; h < M; ++h) var += (x[h] - mean) * (x[h] - mean);
    var = var / (double)M + spec.var_floor;
    const TermGrad t = loss_term(spec.energy_kind, mean - eref[b] / div, var);
    const double w = spec.w_energy / (double)B;
    l = w * t.l;
    if (dE)
      for (int h = 0; h < M; ++h)
        dE[(int64_t)b * M + h] = w * (t.dmean + 2.0 * t.dvar * (x[h] - mean)) / ((double)M * div);
  }
  const double s = block_sum(l);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// thread per force component (i, a): dL/dF_ia^m and the block's sum of l_ia
__global__ void __launch_bounds__(kLossBlock) loss_force(gmnn_loss spec, int64_t n3, int M,
                                                         const float* __restrict__ fh, const float* __restrict__ fref,
                                                         float* __restrict__ dF, double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
  double l = 0.0;
  if (c < n3) {
    double x[kMaxHeads];
    double mean = 0.0;
    for (int h = 0; h < M; ++h) {
      x[h] = (double)fh[(int64_t)h * n3 + c];
      mean += x[h];
    }
    mean /= (double)M;
    double var = 0.0;
    for (int h = 0; h < M; ++h) var += (x[h] - mean) * (x[h] - mean);
    var = var / (double)M + spec.var_floor;
    const TermGrad t = loss_term(spec.force_kind, mean - (double)fref[c], var);
    const double w = spec.w_force / (double)n3;
    l = w * t.l;
    if (dF)
      for (int h = 0; h < M; ++h)
        dF[(int64_t)h * n3 + c] = (float)(w * (t.dmean + 2.0 * t.dvar * (x[h] - mean)) / (double)M);
  }
  const double s = block_sum(l);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one thread per term: block partials added in block order
__global__ void loss_finish(const double* __restrict__ pe, int nbe, const double* __restrict__ pf, int nbf,
                            double* __restrict__ loss) {
  if (threadIdx.x > 1) return;
  const double* p = threadIdx.x == 0 ? pe : pf;
  const int n = threadIdx.x == 0 ? nbe : nbf;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += p[k];
  loss[threadIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Adam
// ---------------------------------------------------------------------------
struct AdamSeg {
  float* p;
  const float* g;
  float* m1;
  float* m2;
  int64_t n;
  float lr;
};
struct AdamArgs {
  AdamSeg seg[9];
  // 1 - beta formed on the host in FP64: in FP32, 1 - 0.999f is 1.3e-5 off
  // in relative terms, which would bias every second-moment update
  float beta1, beta2, omb1, omb2, eps, c1, c2;  // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
};

// blockIdx.y: parameter array; grid-stride over its entries
__global__ void __launch_bounds__(256) adam_update(AdamArgs a) {
  const AdamSeg s = a.seg[blockIdx.y];
  // a frozen group (rate 0) keeps its parameters; its moments still advance,
  // as in the textbook update with a zero rate
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < s.n; k += (int64_t)gridDim.x * 256) {
    const float g = s.g[k];
    const float m1 = a.beta1 * s.m1[k] + a.omb1 * g;
    const float m2 = a.beta2 * s.m2[k] + a.omb2 * g * g;
    s.m1[k] = m1;
    s.m2[k] = m2;
    if (s.lr != 0.0f) s.p[k] -= s.lr * (m1 * a.c1) / (sqrtf(m2 * a.c2) + a.eps);
  }
}

// ---------------------------------------------------------------------------
// per-head double backward
// ---------------------------------------------------------------------------
// head h of the packed W3 [HP2][M] as a one-head vector [HP2], and column h
// of dL/dE [B][M] as the one-head upstream gradient [B]
__global__ void head_view(const float* __restrict__ w3, int HP2, int M, int h, const double* __restrict__ dE, int B,
                          float* __restrict__ w3h, double* __restrict__ dEh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < HP2) w3h[t] = w3[(int64_t)t * M + h];
  if (t < B) dEh[t] = dE[(int64_t)t * M + h];
}

struct GradSegs {
  const float* src[9];
  float* dst[9];
  int64_t n[9];
};

// head h's gradients into the result: the shared arrays (all but W3 and b3)
// copied for h = 0 and added for h > 0, so the sum runs in head order; W3's
// column h and b3[h] take the head's own gradient
__global__ void __launch_bounds__(256) head_accumulate(GradSegs g, int h, int M) {
  const int a = blockIdx.y;
  const int64_t n = g.n[a];
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const float v = g.src[a][k];
    if (a == 5)
      g.dst[a][k * M + h] = v;  // W3 [H2][M]
    else if (a == 6)
      g.dst[a][h] = v;  // b3 [M]
    else
      g.dst[a][k] = h == 0 ? v : g.dst[a][k] + v;
  }
}

gmnn_status train_backward(const DevModel& m, const DevSystem& sys, bool bf16, bool lanes16, int H1, int H2,
                           const double* ebar, const float* lambda, gmnn_param_grads* g, void* ws, size_t ws_bytes,
                           float* dL_dpos, float* gpos, bool accumulate_pos, hipStream_t s);

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// parameter counts in gmnn_param_grads order, W3 and b3 for one head
static void head_grad_sizes(const DevModel& m, int H1, int H2, int64_t n[9]) {
  n[0] = (int64_t)m.n_species * m.n_species * kS * m.K;
  n[1] = (int64_t)kF * H1;
  n[2] = H1;
  n[3] = (int64_t)H1 * H2;
  n[4] = H2;
  n[5] = H2;
  n[6] = 1;
  n[7] = m.n_species;
  n[8] = m.n_species;
}

size_t heads_backward_extra_bytes(const DevModel& m, int H1, int H2, int n_structs) {
  int64_t n[9];
  head_grad_sizes(m, H1, H2, n);
  size_t b = 0;
  for (int k = 0; k < 9; ++k) b += align256(4 * (size_t)n[k]);
  return b + align256(4 * (size_t)m.HP2) + align256(8 * (size_t)n_structs);
}

// one double backward per head (gmnn_backward with GMNN_BACKWARD_PER_HEAD):
// head h sees the model with W3[:, h], b3[h] alone, dL/dE[:, h] and
// dL/dF[h]; head_ws holds the head's gradients, its W3 column and its dL/dE
// column.  The positions' gradient (dL_dpos, optional) is summed over the
// heads in head order.
gmnn_status train_backward_heads(const DevModel& m, const DevSystem& sys, bool bf16, bool lanes16, int H1, int H2,
                                 int n_structs, const double* dE, const float* dF, gmnn_param_grads* g, void* ws,
                                 size_t train_bytes, char* head_ws, size_t head_bytes, float* dL_dpos, float* gpos,
                                 hipStream_t s) {
  if (head_bytes < heads_backward_extra_bytes(m, H1, H2, n_structs)) return GMNN_ERR_WORKSPACE;
  char* X = head_ws;
  int64_t n[9];
  head_grad_sizes(m, H1, H2, n);
  float* tmp[9];
  for (int k = 0; k < 9; ++k) {
    tmp[k] = (float*)X;
    X += align256(4 * (size_t)n[k]);
  }
  float* w3h = (float*)X;
  X += align256(4 * (size_t)m.HP2);
  double* dEh = (double*)X;
  gmnn_param_grads hg = {tmp[0], tmp[1], tmp[2], tmp[3], tmp[4], tmp[5], tmp[6], tmp[7], tmp[8]};
  GradSegs segs;
  float* dst[9] = {g->beta, g->W1, g->b1, g->W2, g->b2, g->W3, g->b3, g->scale, g->shift};
  int64_t nmax = 0;
  for (int k = 0; k < 9; ++k) {
    segs.src[k] = tmp[k];
    segs.dst[k] = dst[k];
    segs.n[k] = n[k];
    nmax = n[k] > nmax ? n[k] : nmax;
  }
  const int M = m.M;
  const int64_t n3 = 3 * (int64_t)sys.n_atoms;
  const int nv = m.HP2 > n_structs ? m.HP2 : n_structs;
  for (int h = 0; h < M; ++h) {
    hipLaunchKernelGGL(head_view, dim3((nv + 255) / 256), dim3(256), 0, s, m.w3, m.HP2, M, h, dE, n_structs, w3h,
                       dEh);
    DevModel mh = m;
    mh.M = 1;
    mh.w3 = w3h;
    mh.w3bar = w3h;
    mh.b3 = m.b3 + h;
    const gmnn_status st =
        train_backward(mh, sys, bf16, lanes16, H1, H2, dEh, dF + h * n3, &hg, ws, train_bytes, dL_dpos, gpos, h > 0, s);
    if (st != GMNN_OK) return st;
    const int nb = (int)std::min<int64_t>((nmax + 255) / 256, 512);
    hipLaunchKernelGGL(head_accumulate, dim3(nb, 9), dim3(256), 0, s, segs, h, M);
  }
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

}  // namespace gmnn

using namespace gmnn;

static int loss_blocks(int64_t n) { return (int)((n + kLossBlock - 1) / kLossBlock); }

extern "C" {

size_t gmnn_loss_workspace_bytes(const gmnn_system* sys) {
  if (!sys || sys->n_structs < 1 || sys->n_atoms < 0) return 0;
  return 8 * ((size_t)loss_blocks(sys->n_structs) + (size_t)loss_blocks(3 * (int64_t)sys->n_atoms) + 2);
}

gmnn_status gmnn_ensemble_loss(const gmnn_loss* spec, const gmnn_system* sys, int32_t n_heads, const double* energy,
                               const float* forces_heads, const double* energy_ref, const float* forces_ref,
                               double* loss, double* dL_dE, float* dL_dF, void* workspace, size_t workspace_bytes,
                               void* stream) {
  if (!spec || !sys || sys->n_structs < 1 || sys->n_atoms < 0 || !sys->atom_ptr || n_heads < 1 ||
      n_heads > kMaxHeads || !energy || !energy_ref || !loss || (sys->n_atoms > 0 && (!forces_heads || !forces_ref)))
    return GMNN_ERR_INVALID_ARG;
  for (int k : {spec->energy_kind, spec->force_kind})
    if (k != GMNN_LOSS_MSE && k != GMNN_LOSS_NLL && k != GMNN_LOSS_CRPS) return GMNN_ERR_INVALID_ARG;
  if (!(spec->var_floor >= 0.0)) return GMNN_ERR_INVALID_ARG;
  // one head has no spread: a NLL or CRPS term without a floor would divide
  // by a zero variance
  if (n_heads == 1 && spec->var_floor == 0.0)
    for (int k : {spec->w_energy != 0.0 ? spec->energy_kind : GMNN_LOSS_MSE,
                  spec->w_force != 0.0 ? spec->force_kind : GMNN_LOSS_MSE})
      if (k != GMNN_LOSS_MSE) return GMNN_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < gmnn_loss_workspace_bytes(sys)) return GMNN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int B = sys->n_structs;
  const int64_t n3 = 3 * (int64_t)sys->n_atoms;
  const int nbe = loss_blocks(B), nbf = loss_blocks(n3);
  double* pe = (double*)workspace;
  double* pf = pe + nbe;
  hipLaunchKernelGGL(loss_energy, dim3(nbe), dim3(kLossBlock), 0, s, *spec, B, n_heads, sys->atom_ptr, energy,
                     energy_ref, dL_dE, pe);
  if (nbf > 0)
    hipLaunchKernelGGL(loss_force, dim3(nbf), dim3(kLossBlock), 0, s, *spec, n3, n_heads, forces_heads, forces_ref,
                       dL_dF, pf);
  hipLaunchKernelGGL(loss_finish, dim3(1), dim3(64), 0, s, pe, nbe, pf, nbf, loss);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

gmnn_status gmnn_model_prepare(gmnn_model* m, void* stream);

gmnn_status gmnn_adam_step(gmnn_model* m, const gmnn_param_grads* grads, gmnn_param_grads* m1,
                           gmnn_param_grads* m2, const gmnn_adam* opt, void* stream) {
  if (!m || !grads || !m1 || !m2 || !opt || opt->step < 1 || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
      !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps >= 0.0) || !m->packed)
    return GMNN_ERR_INVALID_ARG;
  for (double lr : opt->lr)
    if (!(lr >= 0.0)) return GMNN_ERR_INVALID_ARG;
  if (m->n_species < 1 || m->n_species > kMaxSpecies || m->n_radial != kS || m->n_basis < 1 ||
      m->n_basis > kMaxBasis || m->hidden1 < 1 || m->hidden2 < 1 || m->n_heads < 1 || m->n_heads > kMaxHeads)
    return GMNN_ERR_INVALID_ARG;
  const int64_t nsp = m->n_species, H1 = m->hidden1, H2 = m->hidden2, M = m->n_heads;
  float* P[9] = {(float*)m->beta, (float*)m->W1, (float*)m->b1, (float*)m->W2, (float*)m->b2,
                 (float*)m->W3,   (float*)m->b3, (float*)m->scale, (float*)m->shift};
  const float* G[9] = {grads->beta, grads->W1, grads->b1, grads->W2, grads->b2,
                       grads->W3,   grads->b3, grads->scale, grads->shift};
  float* A[9] = {m1->beta, m1->W1, m1->b1, m1->W2, m1->b2, m1->W3, m1->b3, m1->scale, m1->shift};
  float* V[9] = {m2->beta, m2->W1, m2->b1, m2->W2, m2->b2, m2->W3, m2->b3, m2->scale, m2->shift};
  const int64_t n[9] = {nsp * nsp * kS * m->n_basis, (int64_t)kF * H1, H1, H1 * H2, H2, H2 * M, M, nsp, nsp};
  const int group[9] = {GMNN_GROUP_EMBEDDING, GMNN_GROUP_NN, GMNN_GROUP_NN,    GMNN_GROUP_NN,   GMNN_GROUP_NN,
                        GMNN_GROUP_NN,        GMNN_GROUP_NN, GMNN_GROUP_SCALE, GMNN_GROUP_SHIFT};
  AdamArgs a;
  int64_t nmax = 0;
  for (int k = 0; k < 9; ++k) {
    if (!P[k] || !G[k] || !A[k] || !V[k]) return GMNN_ERR_INVALID_ARG;
    a.seg[k] = {P[k], G[k], A[k], V[k], n[k], (float)opt->lr[group[k]]};
    nmax = n[k] > nmax ? n[k] : nmax;
  }
  a.beta1 = (float)opt->beta1;
  a.beta2 = (float)opt->beta2;
  a.omb1 = (float)(1.0 - opt->beta1);
  a.omb2 = (float)(1.0 - opt->beta2);
  a.eps = (float)opt->eps;
  a.c1 = (float)(1.0 / (1.0 - std::pow(opt->beta1, (double)opt->step)));
  a.c2 = (float)(1.0 / (1.0 - std::pow(opt->beta2, (double)opt->step)));
  hipStream_t s = (hipStream_t)stream;
  const int nb = (int)std::min<int64_t>((nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(adam_update, dim3(nb, 9), dim3(256), 0, s, a);
  if (hipGetLastError() != hipSuccess) return GMNN_ERR_HIP;
  return gmnn_model_prepare(m, stream);
}

double gmnn_lr_factor(const gmnn_lr_schedule* sc, int64_t step) {
  if (!sc || step < 0) return NAN;
  if (sc->kind == GMNN_LR_CONSTANT) return 1.0;
  if (sc->kind == GMNN_LR_LINEAR) {
    if (sc->total_steps < 1) return NAN;
    const double frac = (double)std::min(step, sc->total_steps) / (double)sc->total_steps;
    return 1.0 + (sc->end_factor - 1.0) * frac;
  }
  if (sc->kind == GMNN_LR_COSINE) {
    if (sc->period < 1) return NAN;
    const int64_t c = step / sc->period, r = step % sc->period;
    return std::pow(sc->decay_factor, (double)c) * 0.5 * (1.0 + std::cos(M_PI * (double)r / (double)sc->period));
  }
  return NAN;
}

}  // extern "C"
