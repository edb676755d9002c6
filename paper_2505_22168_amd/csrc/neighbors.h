// Internal interface of the neighbour-list build.
#pragma once

#include "common.h"

namespace gmnn {

constexpr int kMaxCellsPerAxis = 1024;

// cell grid of one structure, computed on the device by nl_setup
struct StructGrid {
  double h[9];          // lattice vectors as rows
  double inv[9];        // inverse: frac_k = sum_c x_c inv[c*3+k]
  int nc[3];            // cells per axis
  int m[3];             // stencil half-width per axis (cells)
  int pbc[3];
  int n_cells;
  int64_t cell_offset;  // first global cell index of the structure
};

struct NlLayout {
  int64_t cell_capacity = 0;
  size_t off_grids = 0, off_cell_count = 0, off_cell_fill = 0, off_cell_start = 0, off_cells_total = 0;
  size_t off_atom_cell = 0, off_atom_img = 0, off_cell_atoms = 0, off_row_count = 0, off_go = 0;
  size_t bytes = 0;
};

NlLayout nl_layout(const gmnn_system* sys, double rbin);
// disp_bits / thresh2: build only when the largest squared displacement
// exceeds thresh2 (decided on the device; NULL = always); ref_pos (optional)
// receives the positions the list was built from
gmnn_status nl_build(const gmnn_system* sys, float cutoff, float skin, gmnn_neighbors* nl, void* ws,
                     size_t ws_bytes, hipStream_t stream, const uint32_t* disp_bits = nullptr, float thresh2 = 0.0f,
                     float* ref_pos = nullptr);

}  // namespace gmnn
