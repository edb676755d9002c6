// Periodic cell-list neighbour search (gfx950).
//
// The potential sums over every neighbour j != i of atom i inside the cutoff
// (Section 2.1, eq. basis_fn); periodic cells narrower than twice the cutoff
// hold several images of one neighbour (Section 3.5), so the search enumerates
// as many cell images as the cell width requires instead of the minimum
// image.  The list is canonical (rows by i, inside a row by (j, Sx, Sy, Sz)),
// so it is bit-identical whatever order the atoms land in their cells.
//
// Kernels (one build = 8 launches, all on the caller's stream):
//   nl_setup     one block: per-structure cell grid, cell offsets, clears
//   nl_bin       thread/atom: fractional coords, image, cell, cell counts
//   scan         one block: cell counts -> cell starts
//   nl_cellfill  thread/atom: atoms into their cell slots
//   nl_rows<0>   wave/atom: count neighbours (FP64 inclusion test)
//   scan         one block: row counts -> row_ptr, n_pairs
//   nl_rows<1>   wave/atom: collect, rank-sort in LDS, write the row
//   nl_reverse   wave/atom: index of the reverse pair by binary search
#include "common.h"
#include "neighbors.h"

namespace gmnn {

// ---------------------------------------------------------------------------
// per-structure grid (device)
// ---------------------------------------------------------------------------
__device__ inline void grid_of_structure(const double* h, const uint8_t* pbc, double rbin, StructGrid& g) {
  for (int k = 0; k < 9; ++k) g.h[k] = h[k];
  // inverse of the row-vector lattice: frac_k = sum_c x_c inv[c][k]
  const double a00 = h[0], a01 = h[1], a02 = h[2];
  const double a10 = h[3], a11 = h[4], a12 = h[5];
  const double a20 = h[6], a21 = h[7], a22 = h[8];
  const double c00 = a11 * a22 - a12 * a21, c01 = a12 * a20 - a10 * a22, c02 = a10 * a21 - a11 * a20;
  const double c10 = a02 * a21 - a01 * a22, c11 = a00 * a22 - a02 * a20, c12 = a01 * a20 - a00 * a21;
  const double c20 = a01 * a12 - a02 * a11, c21 = a02 * a10 - a00 * a12, c22 = a00 * a11 - a01 * a10;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  const double id = 1.0 / det;
  // inv = adj / det with adj[c][k] = cofactor[k][c]
  g.inv[0] = c00 * id; g.inv[1] = c10 * id; g.inv[2] = c20 * id;
  g.inv[3] = c01 * id; g.inv[4] = c11 * id; g.inv[5] = c21 * id;
  g.inv[6] = c02 * id; g.inv[7] = c12 * id; g.inv[8] = c22 * id;
  const double vol = fabs(det);
  const double cr[3][3] = {{c00, c01, c02}, {c10, c11, c12}, {c20, c21, c22}};
  long long cells = 1;
  for (int k = 0; k < 3; ++k) {
    // |h_{k+1} x h_{k+2}| = |cofactor row k|; width = vol / that
    const double nrm = sqrt(cr[k][0] * cr[k][0] + cr[k][1] * cr[k][1] + cr[k][2] * cr[k][2]);
    const double width = vol / nrm;
    double fnc = floor(width / rbin);
    int nc = (fnc < 1.0) ? 1 : (fnc > (double)kMaxCellsPerAxis ? kMaxCellsPerAxis : (int)fnc);
    int m = (int)ceil(rbin * (double)nc / width);
    if (m < 1) m = 1;
    g.nc[k] = nc;
    g.m[k] = m;
    g.pbc[k] = pbc[k] ? 1 : 0;
    cells *= nc;
  }
  g.n_cells = (int)cells;
}

// disp_bits (optional): the largest squared displacement since the last
// build (float bits); the build runs only if it exceeds thresh2 (the go flag
// every later kernel of the build checks)
__global__ void __launch_bounds__(1024) nl_setup(const double* __restrict__ cell, const uint8_t* __restrict__ pbc,
                                                 int n_structs, double rbin, StructGrid* __restrict__ grids,
                                                 int64_t cell_capacity, int32_t* __restrict__ cell_count,
                                                 int32_t* __restrict__ cell_fill, int64_t* __restrict__ n_cells_total,
                                                 uint32_t* __restrict__ status, const uint32_t* __restrict__ disp_bits,
                                                 float thresh2, int* __restrict__ go) {
  __shared__ int64_t run;
  __shared__ int64_t part[1024];
  __shared__ int s_go;
  const int t = threadIdx.x;
  if (t == 0) {
    const int g = disp_bits ? (__uint_as_float(*disp_bits) > thresh2 ? 1 : 0) : 1;
    *go = g;
    s_go = g;
    run = 0;
    if (g) *status = 0u;
  }
  __syncthreads();
  if (!s_go) return;
  for (int b0 = 0; b0 < n_structs; b0 += 1024) {
    const int b = b0 + t;
    StructGrid g;
    int64_t nc = 0;
    if (b < n_structs) {
      grid_of_structure(cell + 9 * (int64_t)b, pbc + 3 * (int64_t)b, rbin, g);
      nc = g.n_cells;
    }
    part[t] = nc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int64_t v = (t >= o) ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    if (b < n_structs) {
      g.cell_offset = run + part[t] - nc;
      grids[b] = g;
    }
    __syncthreads();
    if (t == 1023) run += part[1023];
    __syncthreads();
  }
  const int64_t total = run;
  if (t == 0) {
    *n_cells_total = total;
    if (total > cell_capacity) raise_flag(status, GMNN_FLAG_CAPACITY);
  }
  const int64_t lim = total < cell_capacity ? total : cell_capacity;
  for (int64_t c = t; c < lim; c += 1024) {
    cell_count[c] = 0;
    cell_fill[c] = 0;
  }
}

__device__ inline int find_struct(const int64_t* __restrict__ atom_ptr, int n_structs, int64_t i) {
  int lo = 0, hi = n_structs - 1;  // largest b with atom_ptr[b] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (atom_ptr[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void nl_bin(const float* __restrict__ pos, const int64_t* __restrict__ atom_ptr, int n_structs,
                       int n_atoms, const StructGrid* __restrict__ grids, const int64_t* __restrict__ n_cells_total,
                       int64_t cell_capacity, int32_t* __restrict__ atom_struct, int32_t* __restrict__ atom_cell,
                       int4* __restrict__ atom_img, int32_t* __restrict__ cell_count, uint32_t* __restrict__ status,
                       const int* __restrict__ go, float* __restrict__ ref_pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  if (!*go) return;
  if (ref_pos) {
    ref_pos[3 * (int64_t)i] = pos[3 * (int64_t)i];
    ref_pos[3 * (int64_t)i + 1] = pos[3 * (int64_t)i + 1];
    ref_pos[3 * (int64_t)i + 2] = pos[3 * (int64_t)i + 2];
  }
  if (*n_cells_total > cell_capacity) return;
  const int b = find_struct(atom_ptr, n_structs, i);
  atom_struct[i] = b;
  const StructGrid& g = grids[b];
  const double x[3] = {(double)pos[3 * (int64_t)i], (double)pos[3 * (int64_t)i + 1], (double)pos[3 * (int64_t)i + 2]};
  int img[3], cc[3];
  bool bad = false;
  for (int k = 0; k < 3; ++k) {
    const double f = x[0] * g.inv[0 * 3 + k] + x[1] * g.inv[1 * 3 + k] + x[2] * g.inv[2 * 3 + k];
    if (!isfinite(f) || fabs(f) > 1.0e6) {
      bad = true;
      img[k] = 0;
      cc[k] = 0;
      continue;
    }
    double w = f;
    int n = 0;
    if (g.pbc[k]) {
      const double fl = floor(f);
      n = (int)fl;
      w = f - fl;
    }
    int c = (int)floor(w * (double)g.nc[k]);
    c = c < 0 ? 0 : (c >= g.nc[k] ? g.nc[k] - 1 : c);
    img[k] = n;
    cc[k] = c;
  }
  if (bad) raise_flag(status, GMNN_FLAG_NONFINITE);
  const int cid = g.cell_offset + (cc[0] * g.nc[1] + cc[1]) * g.nc[2] + cc[2];
  atom_cell[i] = cid;
  atom_img[i] = make_int4(img[0], img[1], img[2], (cc[0] << 20) | (cc[1] << 10) | cc[2]);
  atomicAdd(&cell_count[cid], 1);
}

__global__ void __launch_bounds__(1024) scan_i32(const int32_t* __restrict__ in, int64_t* __restrict__ out,
                                                 const int64_t* __restrict__ n_dev, int64_t n_host,
                                                 int64_t* __restrict__ total, const int* __restrict__ go,
                                                 int64_t cap) {
  if (!*go) return;
  // n_dev (if given) is clamped to n_host, the length of `in`
  int64_t n = n_host;
  if (n_dev && *n_dev < n_host) n = *n_dev;
  block_exclusive_scan<1024>(in, out, n, total);
  // cap >= 0: offsets beyond the pair capacity would send the pair kernels
  // past the list arrays, so an overflowing list is left empty (the total
  // still reports the size needed, and the capacity flag is raised later)
  if (cap >= 0) {
    __syncthreads();
    if (out[n] > cap)
      for (int64_t k = threadIdx.x; k <= n; k += 1024) out[k] = 0;
  }
}

__global__ void nl_cellfill(int n_atoms, const int32_t* __restrict__ atom_cell, const int64_t* __restrict__ cell_start,
                            const int64_t* __restrict__ n_cells_total, int64_t cell_capacity,
                            int32_t* __restrict__ cell_fill, int32_t* __restrict__ cell_atoms, const int* __restrict__ go) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_atoms) return;
  if (!*go) return;
  if (*n_cells_total > cell_capacity) return;
  const int c = atom_cell[i];
  const int slot = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + slot] = i;
}

__device__ inline int floor_div(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// FP64 inclusion test, every operation rounded once (no contraction), the
// same expression as the reference definition of the list.
__device__ inline double pair_d2(const double xi[3], const double xj[3], const double h[9], int sx, int sy, int sz) {
#pragma clang fp contract(off)
  const double fx = (double)sx, fy = (double)sy, fz = (double)sz;
  const double dx = (xj[0] - xi[0]) + ((fx * h[0] + fy * h[3]) + fz * h[6]);
  const double dy = (xj[1] - xi[1]) + ((fx * h[1] + fy * h[4]) + fz * h[7]);
  const double dz = (xj[2] - xi[2]) + ((fx * h[2] + fy * h[5]) + fz * h[8]);
  return (dx * dx + dy * dy) + dz * dz;
}

constexpr int kRowsWaves = 4;  // waves per block in nl_rows / nl_reverse

// MODE 0: count neighbours of every atom; MODE 1: collect, sort, write.
template <int MODE>
__global__ void __launch_bounds__(64 * kRowsWaves) nl_rows(
    const float* __restrict__ pos, int n_atoms, const StructGrid* __restrict__ grids,
    const int32_t* __restrict__ atom_struct, const int4* __restrict__ atom_img,
    const int64_t* __restrict__ cell_start, const int32_t* __restrict__ cell_atoms,
    const int64_t* __restrict__ n_cells_total, int64_t cell_capacity, double rc2,
    int32_t* __restrict__ row_count, const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ n_pairs,
    int64_t capacity, int32_t* __restrict__ out_j, int32_t* __restrict__ out_shift, uint32_t* __restrict__ status,
    const int* __restrict__ go) {
  __shared__ int s_excl[kRowsWaves][64];
  __shared__ int s_start[kRowsWaves][64];
  __shared__ int s_sw[kRowsWaves][64];
  __shared__ uint64_t s_keys[MODE ? kRowsWaves : 1][MODE ? GMNN_MAX_ROW : 1];
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowsWaves + w;
  if (i >= n_atoms) return;
  if (!*go) return;
  if (*n_cells_total > cell_capacity) return;
  if (MODE == 1 && *n_pairs > capacity) {
    if (i == 0 && l == 0) raise_flag(status, GMNN_FLAG_CAPACITY);
    return;
  }
  const int b = atom_struct[i];
  const StructGrid& g = grids[b];
  const int4 ii = atom_img[i];
  const int ci[3] = {(ii.w >> 20) & 1023, (ii.w >> 10) & 1023, ii.w & 1023};
  const double xi[3] = {(double)pos[3 * (int64_t)i], (double)pos[3 * (int64_t)i + 1], (double)pos[3 * (int64_t)i + 2]};
  const int w0 = 2 * g.m[0] + 1, w1 = 2 * g.m[1] + 1, w2 = 2 * g.m[2] + 1;
  const int T = w0 * w1 * w2;
  int count = 0;
  int base = 0;         // MODE 1: keys collected so far
  bool overflow = false;
  bool coincident = false;
  bool shift_range = false;
  if (MODE == 1 && row_count[i] > GMNN_MAX_ROW) {
    // flagged by the count pass; the row's slots take self pairs (zero
    // separation: every kernel skips them) so the list stays well formed
    const int64_t r0 = row_ptr[i];
    for (int e = l; e < row_count[i]; e += 64) {
      out_j[r0 + e] = i;
      out_shift[r0 + e] = 0;
    }
    return;
  }
  for (int t0 = 0; t0 < T; t0 += 64) {
    const int t = t0 + l;
    int cnt = 0, start = 0, swp = 0;
    if (t < T) {
      const int o2 = t % w2 - g.m[2];
      const int o1 = (t / w2) % w1 - g.m[1];
      const int o0 = t / (w2 * w1) - g.m[0];
      const int oo[3] = {o0, o1, o2};
      int cc[3], sw[3];
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        const int c = ci[k] + oo[k];
        if (g.pbc[k]) {
          sw[k] = floor_div(c, g.nc[k]);
          cc[k] = c - sw[k] * g.nc[k];
        } else {
          sw[k] = 0;
          cc[k] = c;
          if (c < 0 || c >= g.nc[k]) ok = false;
        }
      }
      if (ok) {
        const int cid = g.cell_offset + (cc[0] * g.nc[1] + cc[1]) * g.nc[2] + cc[2];
        start = (int)cell_start[cid];
        cnt = (int)(cell_start[cid + 1] - cell_start[cid]);
        swp = pack_shift(sw[0], sw[1], sw[2]);
      }
    }
    const int incl = wave_incl_scan(cnt);
    const int total = __shfl(incl, 63, 64);
    s_excl[w][l] = incl - cnt;
    s_start[w][l] = start;
    s_sw[w][l] = swp;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + l;
      bool acc = false;
      uint64_t key = 0;
      if (c < total) {
        // last offset slot k with excl[k] <= c
        int lo = 0, hi = 63;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_excl[w][mid] <= c) lo = mid; else hi = mid - 1;
        }
        const int j = cell_atoms[s_start[w][lo] + (c - s_excl[w][lo])];
        int swx, swy, swz;
        unpack_shift(s_sw[w][lo], swx, swy, swz);
        const int4 jj = atom_img[j];
        const int sx = swx - jj.x + ii.x, sy = swy - jj.y + ii.y, sz = swz - jj.z + ii.z;
        if (!(j == i && sx == 0 && sy == 0 && sz == 0)) {
          const double xj[3] = {(double)pos[3 * (int64_t)j], (double)pos[3 * (int64_t)j + 1],
                                (double)pos[3 * (int64_t)j + 2]};
          const double d2 = pair_d2(xi, xj, g.h, sx, sy, sz);
          if (d2 < rc2) {
            if (d2 == 0.0) {
              coincident = true;
            } else {
              acc = true;
              if (sx < -127 || sx > 127 || sy < -127 || sy > 127 || sz < -127 || sz > 127) {
                shift_range = true;
                acc = false;
              } else {
                key = pair_key(j, sx, sy, sz);
              }
            }
          }
        }
      }
      if (MODE == 0) {
        count += acc ? 1 : 0;
      } else {
        const uint64_t bal = __ballot(acc);
        const int pre = __popcll(bal & ((1ull << l) - 1ull));
        if (acc) {
          const int slot = base + pre;
          if (slot < GMNN_MAX_ROW) s_keys[w][slot] = key; else overflow = true;
        }
        base += __popcll(bal);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (coincident) raise_flag(status, GMNN_FLAG_COINCIDENT);
  if (shift_range) raise_flag(status, GMNN_FLAG_SHIFT_RANGE);
  if (MODE == 0) {
    count = wave_sum(count);
    if (l == 0) {
      // a row past the limit is truncated (and flagged): its slots are exactly
      // the ones the collect pass fills, so the list stays well formed
      row_count[i] = count < GMNN_MAX_ROW ? count : GMNN_MAX_ROW;
      if (count > GMNN_MAX_ROW) raise_flag(status, GMNN_FLAG_ROW_TOO_LONG);
    }
    return;
  }
  if (overflow) raise_flag(status, GMNN_FLAG_ROW_TOO_LONG);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int n = base < GMNN_MAX_ROW ? base : GMNN_MAX_ROW;
  const int64_t r0 = row_ptr[i];
  // rank sort (keys are unique inside a row)
  for (int e = l; e < n; e += 64) {
    const uint64_t k = s_keys[w][e];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += (s_keys[w][q] < k) ? 1 : 0;
    const int j = (int)(k >> 24);
    const int sx = (int)((k >> 16) & 0xff) - 128, sy = (int)((k >> 8) & 0xff) - 128, sz = (int)(k & 0xff) - 128;
    out_j[r0 + rank] = j;
    out_shift[r0 + rank] = pack_shift(sx, sy, sz);
  }
}

__global__ void __launch_bounds__(64 * kRowsWaves) nl_reverse(int n_atoms, const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ nj,
                                                             const int32_t* __restrict__ nshift,
                                                             const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                             int32_t* __restrict__ rev, uint32_t* __restrict__ status,
                                                             const int* __restrict__ go) {
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowsWaves + w;
  if (i >= n_atoms) return;
  if (!*go) return;
  if (*n_pairs > capacity) return;
  const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
  for (int64_t p = p0 + l; p < p1; p += 64) {
    const int j = nj[p];
    int sx, sy, sz;
    unpack_shift(nshift[p], sx, sy, sz);
    const uint64_t want = pair_key(i, -sx, -sy, -sz);
    int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1;
    int64_t found = -1;
    while (lo <= hi) {
      const int64_t mid = (lo + hi) >> 1;
      int ax, ay, az;
      unpack_shift(nshift[mid], ax, ay, az);
      const uint64_t k = pair_key(nj[mid], ax, ay, az);
      if (k == want) { found = mid; break; }
      if (k < want) lo = mid + 1; else hi = mid - 1;
    }
    if (found < 0) {
      raise_flag(status, GMNN_FLAG_ROW_TOO_LONG);
      found = p;
    }
    rev[p] = (int32_t)found;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int host_cells_bound(const double* h, const uint8_t* pbc, double rbin) {
  (void)pbc;
  const double a[3][3] = {{h[0], h[1], h[2]}, {h[3], h[4], h[5]}, {h[6], h[7], h[8]}};
  double cr[3][3];
  for (int k = 0; k < 3; ++k) {
    const double* u = a[(k + 1) % 3];
    const double* v = a[(k + 2) % 3];
    cr[k][0] = u[1] * v[2] - u[2] * v[1];
    cr[k][1] = u[2] * v[0] - u[0] * v[2];
    cr[k][2] = u[0] * v[1] - u[1] * v[0];
  }
  const double det = a[0][0] * cr[0][0] + a[0][1] * cr[0][1] + a[0][2] * cr[0][2];
  const double vol = fabs(det);
  long long cells = 1;
  for (int k = 0; k < 3; ++k) {
    const double nrm = sqrt(cr[k][0] * cr[k][0] + cr[k][1] * cr[k][1] + cr[k][2] * cr[k][2]);
    double fnc = floor(vol / nrm / rbin);
    int nc = (fnc < 1.0) ? 1 : (fnc > (double)kMaxCellsPerAxis ? kMaxCellsPerAxis : (int)fnc);
    // +1 per axis absorbs any rounding difference between host and device
    cells *= (nc + 1);
  }
  return (int)(cells > (1LL << 30) ? (1LL << 30) : cells);
}

NlLayout nl_layout(const gmnn_system* sys, double rbin) {
  NlLayout L;
  int64_t cells = 0;
  for (int b = 0; b < sys->n_structs; ++b) cells += host_cells_bound(sys->cell_host + 9 * b, sys->pbc_host + 3 * b, rbin);
  L.cell_capacity = cells;
  const int64_t N = sys->n_atoms;
  const int64_t B = sys->n_structs;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.off_grids = take(sizeof(StructGrid) * (size_t)B);
  L.off_cell_count = take(4 * (size_t)cells);
  L.off_cell_fill = take(4 * (size_t)cells);
  L.off_cell_start = take(8 * (size_t)(cells + 1));
  L.off_cells_total = take(8 * 2);
  L.off_atom_cell = take(4 * (size_t)N);
  L.off_atom_img = take(16 * (size_t)N);
  L.off_cell_atoms = take(4 * (size_t)N);
  L.off_row_count = take(4 * (size_t)N + 4);
  L.off_go = take(4);
  L.bytes = off;
  return L;
}

gmnn_status nl_build(const gmnn_system* sys, float cutoff, float skin, gmnn_neighbors* nl, void* ws,
                     size_t ws_bytes, hipStream_t stream, const uint32_t* disp_bits, float thresh2, float* ref_pos) {
  const double rl = (double)(cutoff + skin);
  const double rbin = rl + 1.0e-4;
  NlLayout L = nl_layout(sys, rbin);
  if (ws_bytes < L.bytes) return GMNN_ERR_WORKSPACE;
  char* w = (char*)ws;
  StructGrid* grids = (StructGrid*)(w + L.off_grids);
  int32_t* cell_count = (int32_t*)(w + L.off_cell_count);
  int32_t* cell_fill = (int32_t*)(w + L.off_cell_fill);
  int64_t* cell_start = (int64_t*)(w + L.off_cell_start);
  int64_t* cells_total = (int64_t*)(w + L.off_cells_total);
  int32_t* atom_cell = (int32_t*)(w + L.off_atom_cell);
  int4* atom_img = (int4*)(w + L.off_atom_img);
  int32_t* cell_atoms = (int32_t*)(w + L.off_cell_atoms);
  int32_t* row_count = (int32_t*)(w + L.off_row_count);
  int* go = (int*)(w + L.off_go);
  const int N = sys->n_atoms;
  const int B = sys->n_structs;
  const float rlf = cutoff + skin;
  const double rc2 = (double)rlf * (double)rlf;
  nl->cutoff = rlf;

  hipLaunchKernelGGL(nl_setup, dim3(1), dim3(1024), 0, stream, sys->cell, sys->pbc, B, rbin, grids,
                     L.cell_capacity, cell_count, cell_fill, cells_total, nl->status, disp_bits, thresh2, go);
  const int tb = 256;
  const int nb_atoms = (N + tb - 1) / tb;
  if (N > 0) {
    hipLaunchKernelGGL(nl_bin, dim3(nb_atoms), dim3(tb), 0, stream, sys->pos, sys->atom_ptr, B, N, grids,
                       cells_total, L.cell_capacity, nl->atom_struct, atom_cell, atom_img, cell_count, nl->status, go,
                       ref_pos);
  }
  hipLaunchKernelGGL(scan_i32, dim3(1), dim3(1024), 0, stream, cell_count, cell_start, cells_total,
                     (int64_t)L.cell_capacity, (int64_t*)nullptr, (const int*)go, (int64_t)-1);
  if (N > 0) {
    hipLaunchKernelGGL(nl_cellfill, dim3(nb_atoms), dim3(tb), 0, stream, N, atom_cell, cell_start, cells_total,
                       L.cell_capacity, cell_fill, cell_atoms, (const int*)go);
    const int nb_rows = (N + kRowsWaves - 1) / kRowsWaves;
    hipLaunchKernelGGL(nl_rows<0>, dim3(nb_rows), dim3(64 * kRowsWaves), 0, stream, sys->pos, N, grids,
                       nl->atom_struct, atom_img, cell_start, cell_atoms, cells_total, L.cell_capacity, rc2, row_count,
                       (const int64_t*)nullptr, (const int64_t*)nullptr, nl->capacity, (int32_t*)nullptr,
                       (int32_t*)nullptr, nl->status, (const int*)go);
    hipLaunchKernelGGL(scan_i32, dim3(1), dim3(1024), 0, stream, row_count, nl->row_ptr, (const int64_t*)nullptr,
                       (int64_t)N, nl->n_pairs, (const int*)go, (int64_t)nl->capacity);
    hipLaunchKernelGGL(nl_rows<1>, dim3(nb_rows), dim3(64 * kRowsWaves), 0, stream, sys->pos, N, grids,
                       nl->atom_struct, atom_img, cell_start, cell_atoms, cells_total, L.cell_capacity, rc2, row_count,
                       nl->row_ptr, nl->n_pairs, nl->capacity, nl->j, nl->shift, nl->status, (const int*)go);
    hipLaunchKernelGGL(nl_reverse, dim3(nb_rows), dim3(64 * kRowsWaves), 0, stream, N, nl->row_ptr, nl->j, nl->shift,
                       nl->n_pairs, nl->capacity, nl->rev, nl->status, (const int*)go);
  } else {
    hipLaunchKernelGGL(scan_i32, dim3(1), dim3(1024), 0, stream, row_count, nl->row_ptr, (const int64_t*)nullptr,
                       (int64_t)0, nl->n_pairs, (const int*)go, (int64_t)nl->capacity);
  }
  return hipGetLastError() == hipSuccess ? GMNN_OK : GMNN_ERR_HIP;
}

}  // namespace gmnn
