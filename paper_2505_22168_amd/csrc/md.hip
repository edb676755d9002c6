// Molecular dynamics on the device (Section 3.5: the whole integration loop
// stays on the GPU; the neighbour list carries a skin and is rebuilt only
// when an atom has moved more than half of it).
//
// One NVE velocity-Verlet step:
//   md_kick_drift   v += dt/2 k_u F / m;  x += dt v;  largest |x - x_ref|^2
//   list build      every kernel exits at once unless the largest
//                   displacement exceeds (skin/2)^2 (decided on the device)
//   energy/forces   the usual launches, on the skin list
//   md_kick         v += dt/2 k_u F / m; reset the displacement word
// k_u = 9.648533e-3 A fs^-2 per eV/(A amu).  Steps are captured once into a
// HIP graph and replayed; nothing in a step reads back to the host, so a
// graph of n steps is n steps without host involvement.
#include <new>

#include "common.h"
#include "neighbors.h"

namespace gmnn {

constexpr float kAccelUnit = 9.648533e-3f;  // (eV/A)/amu -> A/fs^2

__global__ void md_kick_drift(int n, float* __restrict__ pos, float* __restrict__ vel, const float* __restrict__ forces,
                              const float* __restrict__ inv_mass, float half_dt_ku, float dt,
                              const float* __restrict__ ref_pos, uint32_t* __restrict__ disp_bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float d2 = 0.0f;
  if (i < n) {
    const float a = half_dt_ku * inv_mass[i];
    float x[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float v = vel[3 * (int64_t)i + k] + a * forces[3 * (int64_t)i + k];
      vel[3 * (int64_t)i + k] = v;
      x[k] = pos[3 * (int64_t)i + k] + dt * v;
      pos[3 * (int64_t)i + k] = x[k];
      const float dx = x[k] - ref_pos[3 * (int64_t)i + k];
      d2 += dx * dx;
    }
    if (!(d2 == d2)) d2 = 3.0e38f;  // a non-finite position forces a rebuild (which flags it)
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(disp_bits, __float_as_uint(d2));  // d2 >= 0: bits order like values
}

__global__ void md_kick(int n, float* __restrict__ vel, const float* __restrict__ forces,
                        const float* __restrict__ inv_mass, float half_dt_ku, uint32_t* __restrict__ disp_bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *disp_bits = 0u;
  if (i >= n) return;
  const float a = half_dt_ku * inv_mass[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) vel[3 * (int64_t)i + k] += a * forces[3 * (int64_t)i + k];
}

__global__ void md_zero_word(uint32_t* __restrict__ w) { *w = 0u; }

struct MdGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace gmnn

using namespace gmnn;

extern "C" {

gmnn_status gmnn_energy_forces(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags,
                               gmnn_outputs* out, void* workspace, size_t workspace_bytes, void* stream);
gmnn_status gmnn_energy_forces_udd(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                   uint32_t flags, const gmnn_plan* plan, const gmnn_udd* udd, gmnn_outputs* out,
                                   void* workspace, size_t workspace_bytes, void* stream);

static size_t md_nl_bytes(const gmnn_system* sys, const gmnn_neighbors* nl) {
  return (nl_layout(sys, (double)nl->cutoff + 1.0e-4).bytes + 255) & ~size_t(255);
}

size_t gmnn_md_workspace_bytes(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, uint32_t flags) {
  if (!m || !sys || !nl || !(nl->cutoff > 0.0f)) return 0;
  const size_t ef = gmnn_workspace_bytes(GMNN_OP_ENERGY_FORCES, m, sys, nl, flags);
  if (ef == 0) return 0;
  return md_nl_bytes(sys, nl) + ef;
}

static gmnn_status md_check(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl, const gmnn_md* md,
                            uint32_t flags, size_t ws_bytes) {
  if (!m || !sys || !nl || !md || !md->inv_mass || !md->vel || !md->forces || !md->energy || !md->ref_pos ||
      !md->disp || !(md->dt > 0.0f) || !(md->skin >= 0.0f))
    return GMNN_ERR_INVALID_ARG;
  if (flags & (GMNN_WANT_STRESS | GMNN_SYNC)) return GMNN_ERR_INVALID_ARG;
  if ((flags & GMNN_WANT_FORCE_VAR) && (md->var_every < 1 || !md->force_var)) return GMNN_ERR_INVALID_ARG;
  if (md->udd && m->n_heads < 2) return GMNN_ERR_INVALID_ARG;
  if (nl->cutoff + 1e-6f < m->r_cut + md->skin) return GMNN_ERR_INVALID_ARG;
  if (ws_bytes < gmnn_md_workspace_bytes(m, sys, nl, flags)) return GMNN_ERR_WORKSPACE;
  return GMNN_OK;
}

// energies and forces at the current positions: with the bias if md->udd,
// with the per-head force variance if `var`
static gmnn_status md_forces(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                             uint32_t flags, bool var, char* ws, size_t ws_bytes, hipStream_t s) {
  const uint32_t f = (flags & ~GMNN_WANT_FORCE_VAR) | (var ? GMNN_WANT_FORCE_VAR : 0u);
  gmnn_outputs out = {md->energy, md->forces, nullptr, md->energy_var, var ? md->force_var : nullptr, nullptr,
                      nullptr, nullptr};
  if (md->udd) return gmnn_energy_forces_udd(m, sys, nl, f, nullptr, md->udd, &out, ws, ws_bytes, (void*)s);
  return gmnn_energy_forces(m, sys, nl, f, &out, ws, ws_bytes, (void*)s);
}

// one step on `stream` (no host synchronisation); k: the step's index in
// its call or graph, 1-based (the force variance runs on multiples of
// md->var_every)
static gmnn_status md_step(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                           uint32_t flags, char* ws, size_t ws_bytes, hipStream_t s, int k) {
  const int N = sys->n_atoms;
  const float half = 0.5f * md->dt * kAccelUnit;
  const int nb = (N + 255) / 256;
  const size_t nlb = md_nl_bytes(sys, nl);
  if (N > 0)
    hipLaunchKernelGGL(md_kick_drift, dim3(nb), dim3(256), 0, s, N, (float*)sys->pos, md->vel, md->forces,
                       md->inv_mass, half, md->dt, md->ref_pos, md->disp);
  const float th = 0.5f * md->skin;
  gmnn_status st = nl_build(sys, m->r_cut, md->skin, nl, ws, nlb, s, md->disp, th * th, md->ref_pos);
  if (st != GMNN_OK) return st;
  const bool var = (flags & GMNN_WANT_FORCE_VAR) && md->var_every > 0 && k % md->var_every == 0;
  st = md_forces(m, sys, nl, md, flags, var, ws + nlb, ws_bytes - nlb, s);
  if (st != GMNN_OK) return st;
  if (N > 0)
    hipLaunchKernelGGL(md_kick, dim3(nb), dim3(256), 0, s, N, md->vel, md->forces, md->inv_mass, half, md->disp);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

gmnn_status gmnn_md_init(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                         uint32_t flags, void* workspace, size_t workspace_bytes, void* stream) {
  gmnn_status st = md_check(m, sys, nl, md, flags, workspace_bytes);
  if (st != GMNN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const size_t nlb = md_nl_bytes(sys, nl);
  st = nl_build(sys, m->r_cut, md->skin, nl, ws, nlb, s, nullptr, 0.0f, md->ref_pos);
  if (st != GMNN_OK) return st;
  st = md_forces(m, sys, nl, md, flags, (flags & GMNN_WANT_FORCE_VAR) != 0, ws + nlb, workspace_bytes - nlb, s);
  if (st != GMNN_OK) return st;
  hipLaunchKernelGGL(md_zero_word, dim3(1), dim3(1), 0, s, md->disp);
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

gmnn_status gmnn_md_steps(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                          uint32_t flags, int32_t n_steps, void* workspace, size_t workspace_bytes, void* stream) {
  gmnn_status st = md_check(m, sys, nl, md, flags, workspace_bytes);
  if (st != GMNN_OK) return st;
  if (n_steps < 0) return GMNN_ERR_INVALID_ARG;
  for (int k = 0; k < n_steps; ++k) {
    st = md_step(m, sys, nl, md, flags, (char*)workspace, workspace_bytes, (hipStream_t)stream, k + 1);
    if (st != GMNN_OK) return st;
  }
  return GMNN_OK;
}

gmnn_status gmnn_md_graph_create(const gmnn_model* m, const gmnn_system* sys, gmnn_neighbors* nl, const gmnn_md* md,
                                 uint32_t flags, int32_t n_steps, void* workspace, size_t workspace_bytes,
                                 void** graph_out) {
  gmnn_status st = md_check(m, sys, nl, md, flags, workspace_bytes);
  if (st != GMNN_OK) return st;
  if (n_steps < 1 || !graph_out) return GMNN_ERR_INVALID_ARG;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return GMNN_ERR_HIP;
  MdGraph* g = new (std::nothrow) MdGraph();
  if (!g) {
    hipStreamDestroy(cs);
    return GMNN_ERR_HIP;
  }
  st = GMNN_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = GMNN_ERR_HIP;
  for (int k = 0; k < n_steps && st == GMNN_OK; ++k)
    st = md_step(m, sys, nl, md, flags, (char*)workspace, workspace_bytes, cs, k + 1);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (st == GMNN_OK && (ec != hipSuccess || !graph)) st = GMNN_ERR_HIP;
  if (st == GMNN_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) st = GMNN_ERR_HIP;
  hipStreamDestroy(cs);
  if (st != GMNN_OK) {
    if (graph) hipGraphDestroy(graph);
    delete g;
    return st;
  }
  g->graph = graph;
  *graph_out = g;
  return GMNN_OK;
}

gmnn_status gmnn_energy_forces_graph_create(const gmnn_model* m, const gmnn_system* sys, const gmnn_neighbors* nl,
                                            uint32_t flags, const gmnn_plan* plan, gmnn_outputs* out,
                                            void* workspace, size_t workspace_bytes, int32_t n_evals,
                                            void** graph_out) {
  if (n_evals < 1 || n_evals > 4096 || !graph_out || (flags & GMNN_SYNC)) return GMNN_ERR_INVALID_ARG;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return GMNN_ERR_HIP;
  // one eager evaluation first: checks the arguments and leaves every kernel
  // attribute set before the capture
  gmnn_status st = gmnn_energy_forces_plan(m, sys, nl, flags, plan, out, workspace, workspace_bytes, (void*)cs);
  if (st == GMNN_OK && hipStreamSynchronize(cs) != hipSuccess) st = GMNN_ERR_HIP;
  if (st != GMNN_OK) {
    hipStreamDestroy(cs);
    return st;
  }
  MdGraph* g = new (std::nothrow) MdGraph();
  if (!g) {
    hipStreamDestroy(cs);
    return GMNN_ERR_HIP;
  }
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = GMNN_ERR_HIP;
  for (int k = 0; k < n_evals && st == GMNN_OK; ++k)
    st = gmnn_energy_forces_plan(m, sys, nl, flags, plan, out, workspace, workspace_bytes, (void*)cs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (st == GMNN_OK && (ec != hipSuccess || !graph)) st = GMNN_ERR_HIP;
  if (st == GMNN_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) st = GMNN_ERR_HIP;
  hipStreamDestroy(cs);
  if (st != GMNN_OK) {
    if (graph) hipGraphDestroy(graph);
    delete g;
    return st;
  }
  g->graph = graph;
  *graph_out = g;
  return GMNN_OK;
}

gmnn_status gmnn_graph_launch(void* graph, void* stream) { return gmnn_md_graph_launch(graph, stream); }

void gmnn_graph_destroy(void* graph) { gmnn_md_graph_destroy(graph); }

gmnn_status gmnn_md_graph_launch(void* graph, void* stream) {
  if (!graph) return GMNN_ERR_INVALID_ARG;
  MdGraph* g = (MdGraph*)graph;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

void gmnn_md_graph_destroy(void* graph) {
  if (!graph) return;
  MdGraph* g = (MdGraph*)graph;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
