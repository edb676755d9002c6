// C ABI entry points of the GMNN library (declared in include/gmnn.h).
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "model.h"
#include "neighbors.h"
#include "pair_math.h"

namespace gmnn {

// defined in pairs.hip / tile.hip
template <int LPA>
__global__ void pair_moments(DevModel m, DevSystem sys, float* psi, int* counters, int n_counters);
template <int LPA>
__global__ void pair_backward(DevModel m, DevSystem sys, const float* psibar, float* gpair, float* virial);
__global__ void pair_backward_heads(DevModel m, DevSystem sys, const float* psibar, float* gpair, float* virial, int nh,
                                    int64_t gstride, const float* head_c);
template <int LPA, bool VAR>
__global__ void finish(int M, DevSystem sys, const float* gpair, const float* atomic_e, const float* virial,
                       int want_stress, int nb_gather, int64_t gstride, int nchunk, double* partial, int* counters,
                       float* forces, float* force_var, double* energy, double* energy_var, double* energy_mean,
                       double* stress, const double* tile_part, int tile_atoms, const float* head_c,
                       float* forces_heads);
gmnn_status launch_tile(bool fused, bool perhead, int tile_atoms, const DevModel& m, const DevSystem& sys, bool bf16,
                        const float* psi, float* atomic_e, float* psibar, float* gpair, float* virial,
                        int64_t gstride, double* tile_rec, hipStream_t stream);
bool tile_fused_supported(int n_species, int hp, bool bf16, bool perhead);
gmnn_status launch_stream(const DevModel& m, const DevSystem& sys, bool bf16, const float* psi, void* G, float* dG,
                          float* atomic_e, float* psibar, hipStream_t s, hipEvent_t* ev, int phases);
size_t stream_lds_bytes(int hp, bool bf16, int n_heads);
size_t stream_g_bytes(int n_atoms, bool bf16);
size_t stream_dg_bytes(int n_atoms);
size_t tile_lds_bytes(int hp, bool bf16, bool fused, bool perhead);
__global__ void ll_features(DevModel m, DevSystem sys, int H2, const float* h2, double* phi);
bool train_supported(const DevModel& m);
size_t train_workspace_bytes(int n_atoms, int HP, int nsp);
size_t heads_backward_extra_bytes(const DevModel& m, int H1, int H2, int n_structs);
gmnn_status train_backward_heads(const DevModel& m, const DevSystem& sys, bool bf16, bool lanes16, int H1, int H2,
                                 int n_structs, const double* dE, const float* dF, gmnn_param_grads* g, void* ws,
                                 size_t train_bytes, char* head_ws, size_t head_bytes, float* dL_dpos, float* gpos,
                                 hipStream_t s);
gmnn_status train_backward(const DevModel& m, const DevSystem& sys, bool bf16, bool lanes16, int H1, int H2,
                           const double* ebar, const float* lambda, gmnn_param_grads* g, void* ws, size_t ws_bytes,
                           float* dL_dpos, float* gpos, bool accumulate_pos, hipStream_t s);

constexpr int kPairThreads = 256;
// below this many atoms the built-in plan takes the fused (latency) schedule,
// and no structure of a fused evaluation may be larger (one block sums each
// structure from its tiles' records); measured: the fused schedule still
// wins at 11,000 atoms, the streamed readout takes over from 16384
constexpr int kFusedMaxAtoms = 16384;
// below this many atoms the split schedule's pair kernels take 64 lanes per row
constexpr int kWideLanesMaxAtoms = 8192;
// per-structure reductions of per-atom values split into chunks of at most
// this many atoms (one block each)
constexpr int kReduceChunk = 2048;

static int64_t largest_structure(const gmnn_system* sys) {
  int64_t mx = 0;
  for (int b = 0; b < sys->n_structs; ++b) {
    const int64_t n = sys->atom_ptr_host[b + 1] - sys->atom_ptr_host[b];
    if (n > mx) mx = n;
  }
  return mx;
}

static int reduce_chunks(const gmnn_system* sys) {
  const int64_t c = (largest_structure(sys) + kReduceChunk - 1) / kReduceChunk;
  return c < 1 ? 1 : (int)c;
}

// ---------------------------------------------------------------------------
// execution plans
// ---------------------------------------------------------------------------
struct Plan {
  bool fused;   // one tile kernel for moments + readout + pair backward
  int ta;       // fused schedule: atoms per tile (8 or 16); 0 otherwise
  int lpa;      // lanes per atom row in the pair and gather kernels
  bool stream;  // split schedule: readout as three launches (64-row network tiles)
};
// the built-in fused plan halves its tiles (8 atoms) while 16-atom tiles
// would leave compute units idle
constexpr int kComputeUnits = 256;
// at and above this many atoms the built-in plan streams the readout
constexpr int kStreamMinAtoms = 16384;

// the fused tile needs few species (beta staged in its LDS), the head-mean
// backward only, and structures of at most kFusedMaxAtoms atoms (one block
// sums each structure from the tiles' records)
static bool fused_allowed(const gmnn_model* m, const gmnn_system* sys, uint32_t flags, int HP1) {
  return tile_fused_supported(m->n_species, HP1, (flags & GMNN_PREC_BF16) != 0, (flags & GMNN_WANT_FORCE_VAR) != 0) &&
         largest_structure(sys) <= kFusedMaxAtoms;
}

// fills the AUTO fields of `in` (built-in heuristic: the fused schedule for
// systems of fewer than kFusedMaxAtoms atoms, 64 lanes per atom there and for
// split systems below kWideLanesMaxAtoms, 16 beyond, 8-atom fused tiles below
// one 16-atom tile per compute unit);
// UNSUPPORTED for a plan these shapes cannot run
static gmnn_status resolve_plan(const gmnn_model* m, const gmnn_system* sys, uint32_t flags, const gmnn_plan* in,
                                Plan& out) {
  const PackedLayout L = packed_layout(m->hidden1, m->hidden2, m->n_heads);
  const int sched = in ? in->schedule : GMNN_SCHEDULE_AUTO;
  const int lpa = in ? in->lanes_per_atom : 0;
  if (sched != GMNN_SCHEDULE_AUTO && sched != GMNN_SCHEDULE_FUSED && sched != GMNN_SCHEDULE_SPLIT)
    return GMNN_ERR_INVALID_ARG;
  if (lpa != 0 && lpa != 8 && lpa != 16 && lpa != 32 && lpa != 64) return GMNN_ERR_INVALID_ARG;
  const bool small = sys->n_atoms < kFusedMaxAtoms;
  const bool can_fuse = fused_allowed(m, sys, flags, L.HP1);
  if (sched == GMNN_SCHEDULE_FUSED && !can_fuse) return GMNN_ERR_UNSUPPORTED;
  out.fused = sched == GMNN_SCHEDULE_FUSED || (sched == GMNN_SCHEDULE_AUTO && small && can_fuse);
  if (!out.fused && tile_lds_bytes(L.HP1, (flags & GMNN_PREC_BF16) != 0, false, (flags & GMNN_WANT_FORCE_VAR) != 0) >
                        160 * 1024)
    return GMNN_ERR_UNSUPPORTED;
  const int ta = in ? in->tile_atoms : 0;
  if (ta != 0 && ta != 8 && ta != 16) return GMNN_ERR_INVALID_ARG;
  if (ta != 0 && !out.fused) return GMNN_ERR_UNSUPPORTED;
  out.ta = !out.fused ? 0 : ta ? ta : ((sys->n_atoms + 15) / 16 < kComputeUnits ? 8 : 16);
  // 64 lanes per row for the fused schedule and small split evaluations, 16
  // for large ones (fuller waves over long lists)
  out.lpa = lpa ? lpa : ((out.fused || sys->n_atoms < kWideLanesMaxAtoms) ? 64 : 16);
  const int ro = in ? in->readout : GMNN_READOUT_AUTO;
  if (ro != GMNN_READOUT_AUTO && ro != GMNN_READOUT_TILE && ro != GMNN_READOUT_STREAM) return GMNN_ERR_INVALID_ARG;
  const bool can_stream = !out.fused && !(flags & GMNN_WANT_FORCE_VAR) &&
                          stream_lds_bytes(L.HP1, (flags & GMNN_PREC_BF16) != 0, m->n_heads) <= 160 * 1024;
  if (ro == GMNN_READOUT_STREAM && !can_stream) return GMNN_ERR_UNSUPPORTED;
  out.stream = ro == GMNN_READOUT_STREAM || (ro == GMNN_READOUT_AUTO && can_stream && sys->n_atoms >= kStreamMinAtoms);
  return GMNN_OK;
}

// ---------------------------------------------------------------------------
// model preparation: MFMA fragment order, padded widths
// ---------------------------------------------------------------------------
// which = 0: W1 (K = F pad 384, N = HP1); 1: W1^T (K = HP1, N = 384);
//         2: W2 (K = HP1, N = HP2);       3: W2^T (K = HP2, N = HP1)
__device__ inline float wsrc(int which, const float* W1, const float* W2, int F, int H1, int H2, int k, int n) {
  switch (which) {
    case 0: return (k < F && n < H1) ? W1[(size_t)k * H1 + n] : 0.0f;
    case 1: return (n < F && k < H1) ? W1[(size_t)n * H1 + k] : 0.0f;
    case 2: return (k < H1 && n < H2) ? W2[(size_t)k * H2 + n] : 0.0f;
    default: return (n < H1 && k < H2) ? W2[(size_t)n * H2 + k] : 0.0f;
  }
}

__global__ void pack_weights(int which, const float* __restrict__ W1, const float* __restrict__ W2, int F, int H1,
                             int H2, int Kp, int Np, float* __restrict__ out_f32, __bf16* __restrict__ out_bf16,
                             __bf16* __restrict__ out_bf16_lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Kp * Np;
  if (t >= total) return;
  // fp32 chunks: index = ((nb*KC + kc)*64 + l)*4 + u,  k = 16 kc + 4 (l>>4) + u
  {
    const int KC = Kp / 16;
    const int64_t u = t % 4, rest = t / 4;
    const int64_t l = rest % 64, rest2 = rest / 64;
    const int64_t kc = rest2 % KC, nb = rest2 / KC;
    const int k = (int)(kc * 16 + 4 * (l >> 4) + u), n = (int)(nb * 16 + (l & 15));
    out_f32[t] = wsrc(which, W1, W2, F, H1, H2, k, n);
  }
  // bf16 fragments: index = ((nb*KB + kb)*64 + l)*8 + e,  k = 32 kb + 8 (l>>4) + e
  {
    const int KB32 = Kp / 32;
    const int64_t e = t % 8, rest = t / 8;
    const int64_t l = rest % 64, rest2 = rest / 64;
    const int64_t kb = rest2 % KB32, nb = rest2 / KB32;
    const int k = (int)(kb * 32 + 8 * (l >> 4) + e), n = (int)(nb * 16 + (l & 15));
    const float w = wsrc(which, W1, W2, F, H1, H2, k, n);
    const __bf16 hi = (__bf16)w;
    out_bf16[t] = hi;
    // w - hi is exact in FP32 (hi is w's nearest bf16)
    if (out_bf16_lo) out_bf16_lo[t] = (__bf16)(w - (float)hi);
  }
}

__global__ void pack_vectors(const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ W3,
                             const float* __restrict__ b3, int H1, int H2, int HP1, int HP2, int M,
                             float* __restrict__ b1p, float* __restrict__ b2p, float* __restrict__ w3p,
                             float* __restrict__ w3bar, float* __restrict__ b3p) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < HP1) b1p[t] = t < H1 ? b1[t] : 0.0f;
  if (t < HP2) {
    b2p[t] = t < H2 ? b2[t] : 0.0f;
    float s = 0.0f;
    for (int m = 0; m < M; ++m) {
      const float v = t < H2 ? W3[(size_t)t * M + m] : 0.0f;
      w3p[(size_t)t * M + m] = v;
      s += v;
    }
    w3bar[t] = s / (float)M;
  }
  if (t < M) b3p[t] = b3[t];
}

static DevModel dev_model(const gmnn_model* m) {
  DevModel d;
  const PackedLayout L = packed_layout(m->hidden1, m->hidden2, m->n_heads);
  const char* P = (const char*)m->packed;
  d.n_species = m->n_species;
  d.K = m->n_basis;
  d.HP1 = L.HP1;
  d.HP2 = L.HP2;
  d.M = m->n_heads;
  d.r_min = m->r_min;
  d.r_cut = m->r_cut;
  d.rc2 = m->r_cut * m->r_cut;
  d.half_inv_rc = (float)(0.5 / (double)m->r_cut);
  d.gamma = m->gamma;
  d.delta = (m->r_cut - m->r_min) / (float)(m->n_basis - 1);
  d.psi_scale = m->psi_scale;
  d.rc_over_pi = (float)((double)m->r_cut / M_PI);
  d.basis = m->basis;
  for (int k = 0; k < 8; ++k) {
    double c = 0.0;
    if (k < m->n_basis) {
      if (m->basis == GMNN_BASIS_BESSEL)
        c = (k % 2 ? -1.0 : 1.0) * std::sqrt(2.0) * M_PI * std::pow((double)m->r_cut, -1.5) * (k + 1.0) * (k + 2.0) /
            std::sqrt((k + 1.0) * (k + 1.0) + (k + 2.0) * (k + 2.0));
      else
        c = std::exp(-(double)d.gamma * (double)d.delta * (double)d.delta * (double)(k * k));
    }
    d.ck[k] = (float)c;
  }
  d.beta = m->beta;
  d.scale = m->scale;
  d.shift = m->shift;
  d.w1_f32 = (const float*)(P + L.w1_f32);
  d.w1t_f32 = (const float*)(P + L.w1t_f32);
  d.w2_f32 = (const float*)(P + L.w2_f32);
  d.w2t_f32 = (const float*)(P + L.w2t_f32);
  d.w1_bf16 = (const bf16x8*)(P + L.w1_bf16);
  d.w1t_bf16 = (const bf16x8*)(P + L.w1t_bf16);
  d.w2_bf16 = (const bf16x8*)(P + L.w2_bf16);
  d.w2t_bf16 = (const bf16x8*)(P + L.w2t_bf16);
  d.w1lo_bf16 = (const bf16x8*)(P + L.w1lo_bf16);
  d.w2lo_bf16 = (const bf16x8*)(P + L.w2lo_bf16);
  d.b1 = (const float*)(P + L.b1);
  d.b2 = (const float*)(P + L.b2);
  d.w3 = (const float*)(P + L.w3);
  d.w3bar = (const float*)(P + L.w3bar);
  d.b3 = (const float*)(P + L.b3);
  d.head_w = nullptr;
  d.fwd_only = 0;
  d.h2_out = nullptr;
  return d;
}

static gmnn_status check_model(const gmnn_model* m) {
  if (!m || !m->beta || !m->W1 || !m->b1 || !m->W2 || !m->b2 || !m->W3 || !m->b3 || !m->scale || !m->shift ||
      !m->packed)
    return GMNN_ERR_INVALID_ARG;
  if (m->n_radial != kS || m->n_basis < 2 || m->n_basis > kMaxBasis || m->n_species < 1 ||
      m->n_species > kMaxSpecies || m->n_heads < 1 || m->n_heads > kMaxHeads || m->hidden1 < 1 || m->hidden2 < 1)
    return GMNN_ERR_UNSUPPORTED;
  if (m->basis != GMNN_BASIS_GAUSSIAN && m->basis != GMNN_BASIS_BESSEL) return GMNN_ERR_INVALID_ARG;
  if (!(m->r_cut > 0.0f)) return GMNN_ERR_INVALID_ARG;
  if (m->basis == GMNN_BASIS_GAUSSIAN && (!(m->r_cut > m->r_min) || !(m->gamma > 0.0f))) return GMNN_ERR_INVALID_ARG;
  const PackedLayout L = packed_layout(m->hidden1, m->hidden2, m->n_heads);
  if (L.HP1 != L.HP2 || L.HP1 > 512 || (L.HP1 != 64 && L.HP1 != 128 && L.HP1 != 256 && L.HP1 != 512))
    return GMNN_ERR_UNSUPPORTED;
  return GMNN_OK;
}

static gmnn_status check_system(const gmnn_system* s) {
  if (!s || s->n_structs < 1 || s->n_atoms < 0 || !s->atom_ptr || !s->atom_ptr_host || !s->cell || !s->cell_host ||
      !s->pbc || !s->pbc_host || (s->n_atoms > 0 && (!s->pos || !s->species)))
    return GMNN_ERR_INVALID_ARG;
  if (s->atom_ptr_host[0] != 0 || s->atom_ptr_host[s->n_structs] != s->n_atoms) return GMNN_ERR_INVALID_ARG;
  for (int b = 0; b < s->n_structs; ++b) {
    if (s->atom_ptr_host[b + 1] < s->atom_ptr_host[b]) return GMNN_ERR_INVALID_ARG;
    const double* h = s->cell_host + 9 * (size_t)b;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(h[k])) return GMNN_ERR_INVALID_ARG;
    const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                       h[2] * (h[3] * h[7] - h[4] * h[6]);
    if (!(std::fabs(det) > 1e-9)) return GMNN_ERR_INVALID_ARG;
  }
  return GMNN_OK;
}

static DevSystem dev_system(const gmnn_system* s, const gmnn_neighbors* nl) {
  DevSystem d;
  d.n_atoms = s->n_atoms;
  d.n_structs = s->n_structs;
  d.pos = s->pos;
  d.species = s->species;
  d.cell = s->cell;
  d.atom_ptr = s->atom_ptr;
  d.atom_struct = nl->atom_struct;
  d.row_ptr = nl->row_ptr;
  d.nj = nl->j;
  d.nshift = nl->shift;
  d.rev = nl->rev;
  d.status = nullptr;
  return d;
}

struct EfLayout {
  size_t psi = 0, psibar = 0, atomic_e = 0, gpair = 0, virial = 0, g = 0, dg = 0, partial = 0, counters = 0,
         tilerec = 0, head_c = 0, head_w = 0, bytes = 0;
};

static EfLayout ef_layout(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags) {
  EfLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t N = (size_t)sys->n_atoms;
  const size_t nh = (flags & GMNN_WANT_FORCE_VAR) ? (size_t)m->n_heads : 1;
  L.psi = take(4 * N * kS * kPacked);
  L.psibar = take(4 * N * kS * kPacked * nh);
  L.atomic_e = take(4 * N * (size_t)m->n_heads);
  L.gpair = take(12 * (size_t)nl->capacity * nh);
  L.virial = take(4 * 9 * N);
  L.g = take(stream_g_bytes((int)N, (flags & GMNN_PREC_BF16) != 0));
  L.dg = take(stream_dg_bytes((int)N));
  L.partial = take(8 * (size_t)(kMaxHeads + 9) * sys->n_structs * reduce_chunks(sys));
  L.counters = take(4 * (size_t)sys->n_structs);
  L.tilerec = take(8 * (size_t)(kMaxHeads + 9) * ((N + 7) / 8));  // fused: one record per tile of >= 8 atoms
  // uncertainty bias: head weights c [B][kMaxHeads] and weighted W3 vectors [B][HP2]
  L.head_c = take(4 * (size_t)kMaxHeads * sys->n_structs);
  L.head_w = take(4 * (size_t)packed_layout(m->hidden1, m->hidden2, m->n_heads).HP2 * sys->n_structs);
  L.bytes = off;
  return L;
}

// ---------------------------------------------------------------------------
// uncertainty-driven bias (Section 2.3, eq. udd): per structure b with
// energies E^m of the M heads, mean Ebar and population variance var,
//   E_b = A [exp(-var / (M N_b B^2)) - 1],
// and the force -d(Ebar + E_b)/dx = -sum_m c_m dE^m/dx with
//   c_m = 1/M + dE_b/dvar * 2 (E^m - Ebar) / M,
//   dE_b/dvar = -A / (M N_b B^2) exp(-var / (M N_b B^2)).
// ---------------------------------------------------------------------------
__global__ void udd_weights(int B, int M, const int64_t* __restrict__ atom_ptr, const double* __restrict__ energy,
                            double A, double Bw, float* __restrict__ head_c, double* __restrict__ bias_energy) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double nb = (double)(atom_ptr[b + 1] - atom_ptr[b]);
  double mean = 0.0;
  for (int h = 0; h < M; ++h) mean += energy[(int64_t)b * M + h];
  mean /= (double)M;
  double var = 0.0;
  for (int h = 0; h < M; ++h) {
    const double d = energy[(int64_t)b * M + h] - mean;
    var += d * d;
  }
  var /= (double)M;
  double eb = 0.0, deb = 0.0;
  if (nb > 0.0) {
    const double scale = 1.0 / ((double)M * nb * Bw * Bw);
    const double ex = exp(-var * scale);
    eb = A * (ex - 1.0);
    deb = -A * scale * ex;
  }
  if (bias_energy) bias_energy[b] = eb;
  for (int h = 0; h < kMaxHeads; ++h)
    head_c[(int64_t)b * kMaxHeads + h] =
        h < M ? (float)(1.0 / (double)M + deb * 2.0 * (energy[(int64_t)b * M + h] - mean) / (double)M) : 0.0f;
}

// head_w[b][col] = sum_m c_m(b) W3[col][m] (the output weights of the biased backward)
__global__ void udd_head_vectors(int B, int M, int HP, const float* __restrict__ head_c, const float* __restrict__ w3,
                                 float* __restrict__ head_w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * HP) return;
  const int64_t b = t / HP;
  const int col = (int)(t % HP);
  float v = 0.0f;
  for (int h = 0; h < M; ++h) v += head_c[b * kMaxHeads + h] * w3[(int64_t)col * M + h];
  head_w[t] = v;
}

}  // namespace gmnn

using namespace gmnn;

extern "C" {

const char* gmnn_status_string(gmnn_status s) {
  switch (s) {
    case GMNN_OK: return "ok";
    case GMNN_ERR_INVALID_ARG: return "invalid argument";
    case GMNN_ERR_CAPACITY: return "neighbour capacity too small";
    case GMNN_ERR_UNSUPPORTED: return "unsupported shape or model";
    case GMNN_ERR_HIP: return "HIP runtime error";
    case GMNN_ERR_DEVICE_FLAG: return "device status flag raised";
    case GMNN_ERR_WORKSPACE: return "workspace too small";
    case GMNN_ERR_SCRATCH_LIMIT: return "input needs more scratch than the allocation-free entry point holds";
    default: return "unknown status";
  }
}

int32_t gmnn_num_features(int32_t S) {
  if (S < 1) return 0;
  const int pairs = S * (S + 1) / 2;
  return S + 3 * pairs + S * (S + 1) * (S + 2) / 6 + 2 * pairs * S + S * S * S;
}

size_t gmnn_model_packed_bytes(const gmnn_model* m) {
  if (!m || m->hidden1 < 1 || m->hidden2 < 1 || m->n_heads < 1) return 0;
  return packed_layout(m->hidden1, m->hidden2, m->n_heads).bytes;
}

gmnn_status gmnn_model_prepare(gmnn_model* m, void* stream) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const PackedLayout L = packed_layout(m->hidden1, m->hidden2, m->n_heads);
  char* P = (char*)m->packed;
  const int F = kF, H1 = m->hidden1, H2 = m->hidden2;
  struct Job {
    int which, Kp, Np;
    size_t f, b, lo;  // lo = 0: no low part (the backward products)
  } jobs[4] = {{0, kFP, L.HP1, L.w1_f32, L.w1_bf16, L.w1lo_bf16},
               {1, L.HP1, kFP, L.w1t_f32, L.w1t_bf16, 0},
               {2, L.HP1, L.HP2, L.w2_f32, L.w2_bf16, L.w2lo_bf16},
               {3, L.HP2, L.HP1, L.w2t_f32, L.w2t_bf16, 0}};
  for (auto& j : jobs) {
    const int64_t total = (int64_t)j.Kp * j.Np;
    hipLaunchKernelGGL(pack_weights, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, j.which, m->W1, m->W2, F,
                       H1, H2, j.Kp, j.Np, (float*)(P + j.f), (__bf16*)(P + j.b),
                       j.lo ? (__bf16*)(P + j.lo) : nullptr);
  }
  const int nv = L.HP1 > L.HP2 ? L.HP1 : L.HP2;
  hipLaunchKernelGGL(pack_vectors, dim3((nv + 255) / 256), dim3(256), 0, s, m->b1, m->b2, m->W3, m->b3, H1, H2, L.HP1,
                     L.HP2, m->n_heads, (float*)(P + L.b1), (float*)(P + L.b2), (float*)(P + L.w3),
                     (float*)(P + L.w3bar), (float*)(P + L.b3));
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

}  // extern "C"

// workspace of gmnn_backward: the training workspace, the per-pair gradient
// of the positions' pass ([capacity][3]), and with GMNN_BACKWARD_PER_HEAD
// the per-head buffers
struct BwLayout {
  size_t train, gpos, heads, bytes;
};
static BwLayout bw_layout(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const PackedLayout P = packed_layout(m->hidden1, m->hidden2, m->n_heads);
  BwLayout L;
  L.train = al(train_workspace_bytes(sys->n_atoms, P.HP1, m->n_species));
  L.gpos = L.train;
  L.heads = L.gpos + al(12 * (size_t)std::max<int64_t>(nl->capacity, 0));
  L.bytes = L.heads + ((flags & GMNN_BACKWARD_PER_HEAD)
                           ? heads_backward_extra_bytes(dev_model(m), m->hidden1, m->hidden2, sys->n_structs)
                           : 0);
  return L;
}

extern "C" {

size_t gmnn_workspace_bytes(int32_t op, const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                            uint32_t flags) {
  (void)flags;
  if (!sys || check_system(sys) != GMNN_OK) return 0;
  if (op == GMNN_OP_NEIGHBORS) {
    if (!nl || !(nl->cutoff > 0.0f)) return 0;
    return nl_layout(sys, (double)nl->cutoff + 1.0e-4).bytes;
  }
  if (!m || !nl) return 0;
  if (op == GMNN_OP_ENERGY_FORCES) return ef_layout(m, sys, nl, flags).bytes;
  if (op == GMNN_OP_FEATURES) {
    const PackedLayout P = packed_layout(m->hidden1, m->hidden2, m->n_heads);
    return ef_layout(m, sys, nl, flags & GMNN_PREC_BF16).bytes + ((4 * (size_t)sys->n_atoms * P.HP2 + 255) & ~size_t(255));
  }
  if (op == GMNN_OP_BACKWARD) {
    if (check_model(m) != GMNN_OK) return 0;
    return bw_layout(m, sys, nl, flags).bytes;
  }
  return 0;
}

size_t gmnn_neighbors_workspace_bytes(const gmnn_system* sys, float cutoff, float skin) {
  if (!sys || check_system(sys) != GMNN_OK) return 0;
  return nl_layout(sys, (double)(cutoff + skin) + 1.0e-4).bytes;
}

gmnn_status gmnn_build_neighbors(const gmnn_system* sys, float cutoff, float skin, gmnn_neighbors* nl, uint32_t flags,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  gmnn_status st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!nl || !nl->row_ptr || !nl->atom_struct || !nl->n_pairs || !nl->status || nl->capacity < 0 ||
      (nl->capacity > 0 && (!nl->j || !nl->shift || !nl->rev)) || !(cutoff > 0.0f) || !(skin >= 0.0f) ||
      (!workspace && workspace_bytes > 0))
    return GMNN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  st = nl_build(sys, cutoff, skin, nl, workspace, workspace_bytes, s);
  if (st != GMNN_OK) return st;
  if (flags & GMNN_SYNC) {
    if (hipStreamSynchronize(s) != hipSuccess) return GMNN_ERR_HIP;
    uint32_t status = 0;
    int64_t np = 0;
    if (hipMemcpy(&status, nl->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GMNN_ERR_HIP;
    if (hipMemcpy(&np, nl->n_pairs, 8, hipMemcpyDeviceToHost) != hipSuccess) return GMNN_ERR_HIP;
    if (status & GMNN_FLAG_CAPACITY || np > nl->capacity) return GMNN_ERR_CAPACITY;
    if (status) return GMNN_ERR_DEVICE_FLAG;
  }
  return GMNN_OK;
}

int32_t gmnn_uses_fused_path(const gmnn_model* m, const gmnn_system* sys, uint32_t flags) {
  if (check_model(m) != GMNN_OK || check_system(sys) != GMNN_OK) return -1;
  Plan p;
  if (resolve_plan(m, sys, flags, nullptr, p) != GMNN_OK) return -1;
  return p.fused ? 1 : 0;
}

gmnn_status gmnn_resolve_plan(const gmnn_model* m, const gmnn_system* sys, uint32_t flags, const gmnn_plan* plan,
                              gmnn_plan* resolved) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  Plan p;
  st = resolve_plan(m, sys, flags, plan, p);
  if (st != GMNN_OK) return st;
  if (resolved) {
    resolved->schedule = p.fused ? GMNN_SCHEDULE_FUSED : GMNN_SCHEDULE_SPLIT;
    resolved->lanes_per_atom = p.lpa;
    resolved->readout = p.stream ? GMNN_READOUT_STREAM : GMNN_READOUT_TILE;
    resolved->tile_atoms = p.ta;
  }
  return GMNN_OK;
}

}  // extern "C"

// one evaluation; udd (may be null): the uncertainty-driven bias, which runs
// the split schedule in two passes (energies of every head first, then the
// backward with the bias's head weights)
static gmnn_status ef_run(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags,
                          const gmnn_plan* plan, gmnn_outputs* out, void* workspace, size_t workspace_bytes,
                          void* stream, void* const* stage_events, const gmnn_udd* udd) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!nl || !nl->row_ptr || !nl->atom_struct || (nl->capacity > 0 && (!nl->j || !nl->shift || !nl->rev)) || !out ||
      !out->energy || (sys->n_atoms > 0 && !out->forces) || ((flags & GMNN_WANT_STRESS) && !out->stress))
    return GMNN_ERR_INVALID_ARG;
  if ((flags & GMNN_WANT_FORCE_VAR) && !out->force_var) return GMNN_ERR_INVALID_ARG;
  if (nl->cutoff + 1e-6f < m->r_cut) return GMNN_ERR_INVALID_ARG;
  const EfLayout L = ef_layout(m, sys, nl, flags);
  if (workspace_bytes < L.bytes || !workspace) return GMNN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace;
  float* psi = (float*)(W + L.psi);
  float* psibar = (float*)(W + L.psibar);
  float* atomic_e = out->atomic_energy ? out->atomic_energy : (float*)(W + L.atomic_e);
  float* gpair = (float*)(W + L.gpair);
  float* virial = (float*)(W + L.virial);
  double* partial = (double*)(W + L.partial);
  int* counters = (int*)(W + L.counters);
  double* tilerec = (double*)(W + L.tilerec);
  const DevModel dm = dev_model(m);
  DevSystem ds = dev_system(sys, nl);
  ds.status = out->status;
  const bool bf16 = (flags & GMNN_PREC_BF16) != 0;
  const int N = sys->n_atoms;
  const size_t beta_lds = sizeof(float) * (size_t)m->n_species * m->n_species * kS * kMaxBasis;
  hipEvent_t* ev = (hipEvent_t*)stage_events;
  auto mark = [&](int k) {
    if (ev) hipEventRecord(ev[k], s);
  };
  const bool var = (flags & GMNN_WANT_FORCE_VAR) != 0;
  Plan P;
  gmnn_plan split_plan{GMNN_SCHEDULE_SPLIT, 0, GMNN_READOUT_AUTO, 0};
  if (udd) {
    // the bias needs every structure's head energies before any backward:
    // the split schedule only
    if (!(udd->B > 0.0f) || !std::isfinite(udd->A) || m->n_heads < 2) return GMNN_ERR_INVALID_ARG;
    if (plan && plan->schedule == GMNN_SCHEDULE_FUSED) return GMNN_ERR_UNSUPPORTED;
    if (plan) split_plan = *plan;
    split_plan.schedule = GMNN_SCHEDULE_SPLIT;
    plan = &split_plan;
  }
  st = resolve_plan(m, sys, flags, plan, P);
  if (st != GMNN_OK) return st;
  float* head_c = (float*)(W + L.head_c);
  float* head_w = (float*)(W + L.head_w);
  const bool fused = P.fused;
  const int lpa = P.lpa;
  // the fused schedule sums each structure in one block from the tiles'
  // records; the split one from per-atom values in chunks of kReduceChunk
  const int nchunk = fused ? 1 : reduce_chunks(sys);
  const int nb_gather = (N + kPairThreads / lpa - 1) / (kPairThreads / lpa);
  const int64_t gstride = nl->capacity;
  const int nh = var ? m->n_heads : 1;
  if (N > 0) {
    if (fused) {
      mark(0);
      st = launch_tile(true, false, P.ta, dm, ds, bf16, nullptr, atomic_e, nullptr, gpair, virial, gstride, tilerec, s);
      if (st != GMNN_OK) return st;
      for (int k = 1; k < 10; ++k) mark(k);
    } else {
      mark(0);
      const int nzc = nchunk > 1 ? sys->n_structs : 0;
#define MOMENTS(LPA) \
  hipLaunchKernelGGL(pair_moments<LPA>, dim3(nb_gather), dim3(kPairThreads), beta_lds, s, dm, ds, psi, counters, nzc)
      if (lpa == 64) MOMENTS(64);
      else if (lpa == 32) MOMENTS(32);
      else if (lpa == 16) MOMENTS(16);
      else MOMENTS(8);
#undef MOMENTS
      mark(1);
      DevModel db = dm;  // the model of the backward pass
      int phases = 7;    // streamed readout: invariants, network, invariant backward
      if (udd) {
        // pass 1: energies of every head (readout forward only), summed per
        // structure; then the head weights c_m and the weighted W3 vectors
        DevModel da = dm;
        da.fwd_only = 1;
        if (P.stream)
          st = launch_stream(da, ds, bf16, psi, W + L.g, (float*)(W + L.dg), atomic_e, psibar, s, nullptr, 3);
        else
          st = launch_tile(false, var, 16, da, ds, bf16, psi, atomic_e, psibar, nullptr, nullptr, gstride, nullptr, s);
        if (st != GMNN_OK) return st;
        const dim3 rgrid(sys->n_structs * nchunk);
#define FINISH_REDUCE(VAR)                                                                                      \
  hipLaunchKernelGGL((finish<64, VAR>), rgrid, dim3(kPairThreads), 0, s, m->n_heads, ds, gpair, atomic_e, virial,  \
                     0, 0, gstride, nchunk, partial, counters, out->forces, out->force_var, out->energy,           \
                     out->energy_var, out->energy_mean, out->stress, nullptr, 0, nullptr, nullptr)
        if (var) FINISH_REDUCE(true);
        else FINISH_REDUCE(false);
#undef FINISH_REDUCE
        hipLaunchKernelGGL(udd_weights, dim3((sys->n_structs + 63) / 64), dim3(64), 0, s, sys->n_structs, m->n_heads,
                           sys->atom_ptr, out->energy, (double)udd->A, (double)udd->B, head_c, udd->bias_energy);
        if (!var) {
          const int64_t nw = (int64_t)sys->n_structs * dm.HP2;
          hipLaunchKernelGGL(udd_head_vectors, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, sys->n_structs,
                             m->n_heads, dm.HP2, head_c, dm.w3, head_w);
          db.head_w = head_w;  // one backward with the weights c_m
        }
        phases = 6;  // pass 2 reuses the invariants
        // the pair counters of the chunked sums were used by pass 1's
        // reduction, which leaves them cleared
      }
      if (P.stream) {
        st = launch_stream(db, ds, bf16, psi, W + L.g, (float*)(W + L.dg), atomic_e, psibar, s, ev ? ev + 2 : nullptr,
                           phases);
      } else {
        mark(2);
        st = launch_tile(false, var, 16, db, ds, bf16, psi, atomic_e, psibar, nullptr, nullptr, gstride, nullptr, s);
        for (int k = 3; k < 8; ++k) mark(k);
      }
      if (st != GMNN_OK) return st;
      mark(8);
#define PAIR_BACKWARD(LPA)                                                                                 \
  hipLaunchKernelGGL(pair_backward<LPA>, dim3(nb_gather), dim3(kPairThreads), beta_lds, s, dm, ds, psibar, gpair, \
                     virial)
      if (nh > 1) {
        // one backward per head: every pair's geometry serves all heads
        const size_t lds = beta_lds + sizeof(float) * kHeadsAtoms * (size_t)nh * kS * kPacked;
        st = ensure_lds_limit((const void*)pair_backward_heads, lds);
        if (st != GMNN_OK) return st;
        hipLaunchKernelGGL(pair_backward_heads, dim3((N + kHeadsAtoms - 1) / kHeadsAtoms), dim3(kPairThreads), lds,
                           s, dm, ds, psibar, gpair, virial, nh, gstride, udd ? head_c : nullptr);
      } else if (lpa == 64) PAIR_BACKWARD(64);
      else if (lpa == 32) PAIR_BACKWARD(32);
      else if (lpa == 16) PAIR_BACKWARD(16);
      else PAIR_BACKWARD(8);
#undef PAIR_BACKWARD
      mark(9);
    }
  }
  mark(10);
  const int want_stress = (flags & GMNN_WANT_STRESS) ? 1 : 0;
  const int nbg = N > 0 ? nb_gather : 0;
  const dim3 fgrid(nbg + sys->n_structs * nchunk);
#define FINISH(LPA, VAR)                                                                                       \
  hipLaunchKernelGGL((finish<LPA, VAR>), fgrid, dim3(kPairThreads), 0, s, m->n_heads, ds, gpair, atomic_e, virial, \
                     want_stress, nbg, gstride, nchunk, partial, counters, out->forces, out->force_var, out->energy, \
                     out->energy_var, out->energy_mean, out->stress, fused ? tilerec : nullptr, fused ? P.ta : 0, \
                     (udd && var) ? head_c : nullptr, var ? out->forces_heads : nullptr)
  if (lpa == 64) {
    if (var) FINISH(64, true);
    else FINISH(64, false);
  } else if (lpa == 32) {
    if (var) FINISH(32, true);
    else FINISH(32, false);
  } else if (lpa == 16) {
    if (var) FINISH(16, true);
    else FINISH(16, false);
  } else {
    if (var) FINISH(8, true);
    else FINISH(8, false);
  }
#undef FINISH
  mark(11);
  if (hipGetLastError() != hipSuccess) return GMNN_ERR_HIP;
  if (flags & GMNN_SYNC) {
    if (hipStreamSynchronize(s) != hipSuccess) return GMNN_ERR_HIP;
    if (out->status) {
      uint32_t word = 0;
      if (hipMemcpy(&word, out->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GMNN_ERR_HIP;
      if (word) return GMNN_ERR_DEVICE_FLAG;
    }
  }
  return GMNN_OK;
}

extern "C" {

gmnn_status gmnn_energy_forces_timed(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                     uint32_t flags, const gmnn_plan* plan, gmnn_outputs* out, void* workspace,
                                     size_t workspace_bytes, void* stream, void* const* stage_events) {
  return ef_run(m, sys, nl, flags, plan, out, workspace, workspace_bytes, stream, stage_events, nullptr);
}

gmnn_status gmnn_energy_forces_udd(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                   uint32_t flags, const gmnn_plan* plan, const gmnn_udd* udd, gmnn_outputs* out,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  if (!udd) return GMNN_ERR_INVALID_ARG;
  return ef_run(m, sys, nl, flags, plan, out, workspace, workspace_bytes, stream, nullptr, udd);
}

gmnn_status gmnn_energy_forces(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags,
                               gmnn_outputs* out, void* workspace, size_t workspace_bytes, void* stream) {
  return gmnn_energy_forces_timed(m, sys, nl, flags, nullptr, out, workspace, workspace_bytes, stream, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the allocation-free entry point: its workspace is a file-scope device
// array; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in)
// ---------------------------------------------------------------------------
namespace gmnn {
static __device__ __align__(256) unsigned char scratch[GMNN_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_scratch_addr[kMaxDevices];
static std::mutex g_scratch_mu;

// device address of this device's scratch array, looked up once per device
static gmnn_status scratch_address(void** addr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMNN_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return GMNN_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GMNN_ERR_HIP;
    g_scratch_addr[dev] = p;
  }
  *addr = g_scratch_addr[dev];
  return GMNN_OK;
}
}  // namespace gmnn

extern "C" {

gmnn_status gmnn_energy_forces_noalloc(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                       uint32_t flags, gmnn_outputs* out, void* stream) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!nl) return GMNN_ERR_INVALID_ARG;
  if (ef_layout(m, sys, nl, flags).bytes > GMNN_NOALLOC_SCRATCH_BYTES) return GMNN_ERR_SCRATCH_LIMIT;
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != GMNN_OK) return st;
  return gmnn_energy_forces_timed(m, sys, nl, flags, nullptr, out, ws, GMNN_NOALLOC_SCRATCH_BYTES, stream, nullptr);
}

gmnn_status gmnn_energy_forces_plan(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                    uint32_t flags, const gmnn_plan* plan, gmnn_outputs* out, void* workspace,
                                    size_t workspace_bytes, void* stream) {
  return gmnn_energy_forces_timed(m, sys, nl, flags, plan, out, workspace, workspace_bytes, stream, nullptr);
}

gmnn_status gmnn_autotune(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags,
                          gmnn_outputs* out, void* workspace, size_t workspace_bytes, void* stream, int32_t reps,
                          gmnn_plan* best, gmnn_tune_entry* entries, int32_t max_entries, int32_t* n_entries) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!best || reps < 1 || reps > 1000 || max_entries < 0 || (max_entries > 0 && !entries))
    return GMNN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  static const int kSched[4] = {GMNN_SCHEDULE_FUSED, GMNN_SCHEDULE_FUSED, GMNN_SCHEDULE_SPLIT, GMNN_SCHEDULE_SPLIT};
  static const int kTileAtoms[4] = {16, 8, 0, 0};
  static const int kReadout[4] = {GMNN_READOUT_TILE, GMNN_READOUT_TILE, GMNN_READOUT_TILE, GMNN_READOUT_STREAM};
  static const int kLanes[4] = {8, 16, 32, 64};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GMNN_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return GMNN_ERR_HIP;
  }
  int n = 0;
  float best_us = 0.0f;
  bool have = false;
  std::vector<float> t(reps);
  for (int si = 0; si < 4 && st == GMNN_OK; ++si) {
    for (int li = 0; li < 4 && st == GMNN_OK; ++li) {
      const gmnn_plan cand = {kSched[si], kLanes[li], kReadout[si], kTileAtoms[si]};
      Plan P;
      if (resolve_plan(m, sys, flags, &cand, P) != GMNN_OK) continue;
      // warm-up (also surfaces argument errors before anything is timed)
      for (int w = 0; w < 2 && st == GMNN_OK; ++w)
        st = gmnn_energy_forces_plan(m, sys, nl, flags, &cand, out, workspace, workspace_bytes, stream);
      for (int r = 0; r < reps && st == GMNN_OK; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) st = GMNN_ERR_HIP;
        if (st == GMNN_OK) st = gmnn_energy_forces_plan(m, sys, nl, flags, &cand, out, workspace, workspace_bytes, stream);
        if (st == GMNN_OK && hipEventRecord(e1, s) != hipSuccess) st = GMNN_ERR_HIP;
        if (st == GMNN_OK && hipEventSynchronize(e1) != hipSuccess) st = GMNN_ERR_HIP;
        float ms = 0.0f;
        if (st == GMNN_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = GMNN_ERR_HIP;
        t[r] = 1000.0f * ms;
      }
      if (st != GMNN_OK) break;
      std::sort(t.begin(), t.end());
      const float med = t[reps / 2];
      if (n < max_entries) {
        entries[n].plan = cand;
        entries[n].median_us = med;
        entries[n].min_us = t[0];
      }
      ++n;
      if (!have || med < best_us) {
        have = true;
        best_us = med;
        *best = cand;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != GMNN_OK) return st;
  if (!have) return GMNN_ERR_UNSUPPORTED;
  if (n_entries) *n_entries = n;
  // leave the outputs of the chosen plan in `out`
  st = gmnn_energy_forces_plan(m, sys, nl, flags, best, out, workspace, workspace_bytes, stream);
  if (st == GMNN_OK && hipStreamSynchronize(s) != hipSuccess) st = GMNN_ERR_HIP;
  return st;
}

gmnn_status gmnn_last_layer_features(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                     uint32_t flags, double* phi, void* workspace, size_t workspace_bytes,
                                     void* stream) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!nl || !nl->row_ptr || !nl->atom_struct || (nl->capacity > 0 && (!nl->j || !nl->shift || !nl->rev)) || !phi ||
      !workspace)
    return GMNN_ERR_INVALID_ARG;
  if (nl->cutoff + 1e-6f < m->r_cut) return GMNN_ERR_INVALID_ARG;
  const uint32_t f = flags & GMNN_PREC_BF16;
  const EfLayout L = ef_layout(m, sys, nl, f);
  if (workspace_bytes < gmnn_workspace_bytes(GMNN_OP_FEATURES, m, sys, nl, f)) return GMNN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace;
  float* psi = (float*)(W + L.psi);
  float* psibar = (float*)(W + L.psibar);
  float* atomic_e = (float*)(W + L.atomic_e);
  float* h2 = (float*)(W + L.bytes);
  DevModel dm = dev_model(m);
  dm.fwd_only = 1;  // the readout forward only, recording h2
  dm.h2_out = h2;
  const DevSystem ds = dev_system(sys, nl);
  const bool bf16 = f != 0;
  Plan P;
  const gmnn_plan split{GMNN_SCHEDULE_SPLIT, 0, GMNN_READOUT_AUTO, 0};
  st = resolve_plan(m, sys, f, &split, P);
  if (st != GMNN_OK) return st;
  const int N = sys->n_atoms;
  if (N > 0) {
    const int lpa = P.lpa;
    const int nb = (N + kPairThreads / lpa - 1) / (kPairThreads / lpa);
    const size_t beta_lds = sizeof(float) * (size_t)m->n_species * m->n_species * kS * kMaxBasis;
#define MOMENTS(LPA) \
  hipLaunchKernelGGL(pair_moments<LPA>, dim3(nb), dim3(kPairThreads), beta_lds, s, dm, ds, psi, (int*)nullptr, 0)
    if (lpa == 64) MOMENTS(64);
    else if (lpa == 32) MOMENTS(32);
    else if (lpa == 16) MOMENTS(16);
    else MOMENTS(8);
#undef MOMENTS
    if (P.stream)
      st = launch_stream(dm, ds, bf16, psi, W + L.g, (float*)(W + L.dg), atomic_e, psibar, s, nullptr, 3);
    else
      st = launch_tile(false, false, 16, dm, ds, bf16, psi, atomic_e, psibar, nullptr, nullptr, nl->capacity, nullptr,
                       s);
    if (st != GMNN_OK) return st;
  }
  hipLaunchKernelGGL(ll_features, dim3(sys->n_structs), dim3(256), 0, s, dm, ds, m->hidden2, h2, phi);
  if (hipGetLastError() != hipSuccess) return GMNN_ERR_HIP;
  if ((flags & GMNN_SYNC) && hipStreamSynchronize(s) != hipSuccess) return GMNN_ERR_HIP;
  return GMNN_OK;
}

gmnn_status gmnn_backward(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, const double* dL_dE,
                          const float* dL_dF, uint32_t flags, gmnn_param_grads* grads, float* dL_dpos, void* workspace,
                          size_t workspace_bytes, void* stream) {
  gmnn_status st = check_model(m);
  if (st != GMNN_OK) return st;
  st = check_system(sys);
  if (st != GMNN_OK) return st;
  if (!nl || !nl->row_ptr || !nl->atom_struct || (nl->capacity > 0 && (!nl->j || !nl->shift || !nl->rev)) || !dL_dE ||
      (sys->n_atoms > 0 && !dL_dF) || !grads || !grads->beta || !grads->W1 || !grads->b1 || !grads->W2 ||
      !grads->b2 || !grads->W3 || !grads->b3 || !grads->scale || !grads->shift || !workspace)
    return GMNN_ERR_INVALID_ARG;
  if (nl->cutoff + 1e-6f < m->r_cut) return GMNN_ERR_INVALID_ARG;
  if (flags & GMNN_WANT_FORCE_VAR) return GMNN_ERR_UNSUPPORTED;
  const DevModel dm = dev_model(m);
  if (!train_supported(dm)) return GMNN_ERR_UNSUPPORTED;
  const BwLayout L = bw_layout(m, sys, nl, flags);
  if (workspace_bytes < L.bytes) return GMNN_ERR_WORKSPACE;
  const DevSystem ds = dev_system(sys, nl);
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace;
  float* gpos = (float*)(W + L.gpos);
  const bool bf16 = (flags & GMNN_PREC_BF16) != 0, lanes16 = (flags & GMNN_BACKWARD_LANES16) != 0;
  if (flags & GMNN_BACKWARD_PER_HEAD)
    st = train_backward_heads(dm, ds, bf16, lanes16, m->hidden1, m->hidden2, sys->n_structs, dL_dE, dL_dF, grads,
                              W, L.train, W + L.heads, L.bytes - L.heads, dL_dpos, gpos, s);
  else
    st = train_backward(dm, ds, bf16, lanes16, m->hidden1, m->hidden2, dL_dE, dL_dF, grads, W, L.train, dL_dpos,
                        gpos, false, s);
  if (st != GMNN_OK) return st;
  if ((flags & GMNN_SYNC) && hipStreamSynchronize(s) != hipSuccess) return GMNN_ERR_HIP;
  return GMNN_OK;
}

}  // extern "C"
