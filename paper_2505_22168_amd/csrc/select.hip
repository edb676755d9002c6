// Batch selection by last-layer gradient features (Section 2.4):
//
//   ll_features     phi(S) = gradient of the structure's head-mean energy
//                   w.r.t. one head's last-layer weights and bias (eq.
//                   lastlayer): (1/M) [sum_i sigma_Zi h2_i ; sum_i sigma_Zi],
//                   summed per structure in FP64 in atom order (the other
//                   heads' blocks of the full gradient are equal copies)
//   selection       greedy maximum-distance selection (eq. maxdist): each
//                   step picks the pool structure whose smallest distance to
//                   the training set and the structures picked so far is
//                   largest; distances in FP64, ties to the smallest index.
//                   Per step: block-wise argmax over the pool, one block
//                   for the final argmax, then the distances to the new
//                   pick update every pool entry's minimum.
#include "common.h"
#include "model.h"

namespace gmnn {

// block b: structure b; thread c < D = HP2 + 1 (column c of h2, or the
// bias entry at c = H2) -- columns H2 .. HP2 of h2 are padding and skipped
__global__ void __launch_bounds__(256) ll_features(DevModel m, DevSystem sys, int H2, const float* __restrict__ h2,
                                                   double* __restrict__ phi) {
  const int b = blockIdx.x;
  const int64_t a0 = sys.atom_ptr[b], a1 = sys.atom_ptr[b + 1];
  const double invM = 1.0 / (double)m.M;
  for (int c = threadIdx.x; c <= H2; c += blockDim.x) {
    double acc = 0.0;
    for (int64_t i = a0; i < a1; ++i) {
      const double sg = (double)m.scale[sys.species[i]];
      acc += c < H2 ? sg * (double)h2[i * m.HP2 + c] : sg;
    }
    phi[(int64_t)b * (H2 + 1) + c] = acc * invM;
  }
}

constexpr int kSelBlock = 256;

__device__ inline double dist2(const double* __restrict__ a, const double* __restrict__ b, int D) {
  double s = 0.0;
  for (int k = 0; k < D; ++k) {
    const double d = a[k] - b[k];
    s += d * d;
  }
  return s;
}

// mind[i]: smallest squared distance of pool entry i to the training set
// (or its squared norm when the training set is empty: the first pick is
// then the entry farthest from the origin)
__global__ void __launch_bounds__(kSelBlock) sel_init(const double* __restrict__ pool, int64_t n, int D,
                                                      const double* __restrict__ train, int64_t nt,
                                                      double* __restrict__ mind) {
  const int64_t i = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
  if (i >= n) return;
  const double* p = pool + i * D;
  double best;
  if (nt == 0) {
    best = 0.0;
    for (int k = 0; k < D; ++k) best += p[k] * p[k];
  } else {
    best = dist2(p, train, D);
    for (int64_t t = 1; t < nt; ++t) best = fmin(best, dist2(p, train + t * D, D));
  }
  mind[i] = best;
}

// argmax of mind over each block's slice (picked entries hold -1); ties go
// to the smaller index
__global__ void __launch_bounds__(kSelBlock) sel_argmax_blocks(const double* __restrict__ mind, int64_t n,
                                                               double* __restrict__ part_val,
                                                               int64_t* __restrict__ part_idx) {
  __shared__ double sv[kSelBlock];
  __shared__ int64_t si[kSelBlock];
  const int64_t i = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
  sv[threadIdx.x] = i < n ? mind[i] : -2.0;
  si[threadIdx.x] = i < n ? i : INT64_MAX;
  __syncthreads();
  for (int o = kSelBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + o];
      const int64_t ia = si[threadIdx.x], ib = si[threadIdx.x + o];
      if (b > a || (b == a && ib < ia)) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = ib;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_val[blockIdx.x] = sv[0];
    part_idx[blockIdx.x] = si[0];
  }
}

// one block: the step's pick from the block partials -> selected[step], *pick
__global__ void __launch_bounds__(kSelBlock) sel_pick(const double* __restrict__ part_val,
                                                      const int64_t* __restrict__ part_idx, int nparts, int step,
                                                      int32_t* __restrict__ selected, int64_t* __restrict__ pick) {
  __shared__ double sv[kSelBlock];
  __shared__ int64_t si[kSelBlock];
  double v = -3.0;
  int64_t ix = INT64_MAX;
  for (int p = threadIdx.x; p < nparts; p += kSelBlock) {
    const double a = part_val[p];
    const int64_t ia = part_idx[p];
    if (a > v || (a == v && ia < ix)) {
      v = a;
      ix = ia;
    }
  }
  sv[threadIdx.x] = v;
  si[threadIdx.x] = ix;
  __syncthreads();
  for (int o = kSelBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + o];
      const int64_t ia = si[threadIdx.x], ib = si[threadIdx.x + o];
      if (b > a || (b == a && ib < ia)) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = ib;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    selected[step] = (int32_t)si[0];
    *pick = si[0];
  }
}

// every pool entry's smallest distance now also covers the new pick; the
// pick itself leaves the pool (-1).  replace: the first pick without a
// training set (the norms that chose it are no distances to a selected entry)
__global__ void __launch_bounds__(kSelBlock) sel_update(const double* __restrict__ pool, int64_t n, int D,
                                                        const int64_t* __restrict__ pick, int replace,
                                                        double* __restrict__ mind) {
  const int64_t i = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t j = *pick;
  if (mind[i] < 0.0) return;
  if (i == j) {
    mind[i] = -1.0;
    return;
  }
  const double d = dist2(pool + i * D, pool + j * D, D);
  mind[i] = replace ? d : fmin(mind[i], d);
}

}  // namespace gmnn

using namespace gmnn;

extern "C" {

size_t gmnn_select_workspace_bytes(int64_t n_pool) {
  if (n_pool < 1) return 0;
  const int64_t nb = (n_pool + kSelBlock - 1) / kSelBlock;
  return (size_t)(8 * n_pool + 16 * nb + 64 + 255) & ~size_t(255);
}

gmnn_status gmnn_select_max_distance(const double* pool, int64_t n_pool, int32_t dim, const double* train,
                                     int64_t n_train, int32_t n_select, int32_t* selected, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  if (!pool || n_pool < 1 || dim < 1 || n_train < 0 || (n_train > 0 && !train) || n_select < 0 ||
      n_select > n_pool || (n_select > 0 && !selected) || !workspace)
    return GMNN_ERR_INVALID_ARG;
  if (workspace_bytes < gmnn_select_workspace_bytes(n_pool)) return GMNN_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nb = (n_pool + kSelBlock - 1) / kSelBlock;
  char* W = (char*)workspace;
  double* mind = (double*)W;
  double* part_val = (double*)(W + 8 * n_pool);
  int64_t* part_idx = (int64_t*)(W + 8 * n_pool + 8 * nb);
  int64_t* pick = (int64_t*)(W + 8 * n_pool + 16 * nb);
  hipLaunchKernelGGL(sel_init, dim3((unsigned)nb), dim3(kSelBlock), 0, s, pool, n_pool, dim, train, n_train, mind);
  for (int k = 0; k < n_select; ++k) {
    hipLaunchKernelGGL(sel_argmax_blocks, dim3((unsigned)nb), dim3(kSelBlock), 0, s, mind, n_pool, part_val,
                       part_idx);
    hipLaunchKernelGGL(sel_pick, dim3(1), dim3(kSelBlock), 0, s, part_val, part_idx, (int)nb, k, selected, pick);
    hipLaunchKernelGGL(sel_update, dim3((unsigned)nb), dim3(kSelBlock), 0, s, pool, n_pool, dim, pick,
                       (k == 0 && n_train == 0) ? 1 : 0, mind);
  }
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

}  // extern "C"
