// Internal structures shared by the kernels and the host side of libbfc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfc {

// Axis-aligned box of a primitive, FP32, rounded outward from the FP64
// positions so that it contains the exact primitive.
struct Box {
  float lo[3], hi[3];
};

// Uniform grid of the broad phase.  Cell size >= (largest primitive box side
// + h) so that two primitives whose boxes are closer than h have box centres
// in the same or adjacent cells; every cell has two sub-lists (edges, then
// triangles).  Coordinates are clamped to the grid, which keeps the
// adjacency property.
struct Grid {
  double orgd[3];
  double cell, inv_cell;
  int n[3];
  int ncells;
  int nscan;  // 2 * ncells + 1 sub-list boundaries
  int coarsened;
};

// Scene data resident on the device.
struct SceneDev {
  int kind;  // 0 rod, 1 shell
  int nv, ne, nt;
  const int* edges;  // [E,2]
  const int* tris;   // [F,3]
  const double* ref; // rods [V]; shells [V,2]
  const int* comp;   // [V]
  const double* dmin;  // [C] activation of filtered pairs
  const double* thr2;  // [C,2] exact squared activation of filtered pairs (hi, lo)
  double h, eta, kappa;
  int filter;  // 0 paper, 1 none
  int mixed;   // 1: FP32 bulk arithmetic
};

// Broad-phase scratch (device pointers inside the scene workspace).
struct BroadWs {
  Box* box;          // [NP] per primitive (edges, triangles, points)
  int* cell_of;      // [NP] sub-cell id of stored primitives
  unsigned* bounds;  // [8] ordered-float min xyz, max xyz, max extent, spare
  Grid* grid;        // [1]
  int* cell_cnt;     // [2*max_cells + 1]
  int* cell_start;   // [2*max_cells + 1]
  int* sorted_id;    // [NS] stored primitives in cell order
  Box* sorted_box;   // [NS]
  int* scan_tmp;     // [scan partials]
  int max_cells;
};

// Assembly scratch.
struct AsmWs {
  unsigned long long* keys;  // [S] hash table of (row << 32 | col)
  int* slot_pos;             // [S] BSR position of each occupied slot
  int* entry_slot;           // [16 * act_cap]
  int* rowcnt;               // [V + 1]
  int* rowfill;              // [V]
  int* tmpcol;               // [16 * act_cap] unsorted columns per row
  double* epart;             // [partials] energy partial sums
  int* scan_tmp;
  long long hash_size;       // power of two
};

static const unsigned long long kEmpty = ~0ull;

}  // namespace bfc
