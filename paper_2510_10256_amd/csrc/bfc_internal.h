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

// Uniform grid of the broad phase.  Every stored primitive sits in the cell
// of its box centre (coordinates clamped to the grid); the sorted lists hold
// all cells' edges, then all cells' triangles, so that a run of cells along
// x is one contiguous range of either.  A primitive whose box is within h of
// a query box has its centre within `reach` (h + half the largest box side,
// plus slack) of the query box, so a query visits the cells of that range
// only; the cell side is free (0.7 of largest side + h here).
struct Grid {
  double orgd[3];
  double cell, inv_cell;
  double reach;
  float gapf;  // a float box gap above this is above h on every path of the exact test
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
  const double* xrest;  // [V,3] rest pose (BF_REFDIST_EUCLID_REST), else null
  int refdist;          // BF_REFDIST_PARAM or BF_REFDIST_EUCLID_REST
  const int* comp;   // [V]
  const double* dmin;  // [C] activation of filtered pairs
  const double* thr2;  // [C,2] exact squared activation of filtered pairs (hi, lo)
  double h, eta, kappa;
  // pairs under the temporary zero offset (Sec. 3.4): open-addressing table
  // of packed pair keys and their live flags (core_key null: no such pairs)
  const unsigned long long* core_key;
  const unsigned char* core_live;
  unsigned core_mask;  // slots - 1
  // culling mode (rods): element index of each edge along its polyline and
  // the polyline's edge count when it is closed (0 when open)
  const int* eidx;
  const int* eloop;
  int cull_r;
  int filter;  // 0 paper, 1 none, 2 cull
  int mixed;   // 1: projection converged to the mixed-precision tolerance
  int pq;      // threads per broad-phase query (2, 4, 8 or 16)
  unsigned* status;  // the scene's device status word (BF_S_* bits)
};

// Broad-phase scratch (device pointers inside the scene workspace).
struct BroadWs {
  Box* box;          // [NP] per primitive (edges, triangles, points)
  int* cell_of;      // [NS] sub-cell id of stored primitives
  float* part;       // [8 * BOUNDS_BLOCKS] per-block bounds
  unsigned* done;    // [1] block counter of the last-block reduction (zero between launches)
  Grid* grid;        // [1]
  int* cell_cnt;     // [2*max_cells + 1], zero between steps (edges of every cell, then triangles)
  int* cell_start;   // [2*max_cells + 1]
  int* placed_id;    // [NS] stored primitives grouped by cell (any order inside a cell)
  Box* placed_box;   // [NS]
  int* sorted_id;    // [NS] stored primitives in cell order, by id inside a cell
  Box* sorted_box;   // [NS]
  int4* sorted_vid;  // [NS] their vertex ids (edges: v0, v1, -1; triangles: t0, t1, t2)
  int* pair_cnt;     // [NQ * PQ_MAX] pairs per (query, thread of the query)
  int* pair_bsum;    // [work-groups + 1] pairs per work-group of the count pass
  int* pair_bofs;    // [work-groups + 1] their exclusive scan (the emit pass's offsets)
  long long* pair_bseg;            // [work-groups + 1] start of each group's staged pairs, -1: visit again
  unsigned long long* seg_count;   // [1] staged pairs of this step (segments are taken in any order)
  int* scan_tmp;     // [scan partials]
  int max_cells;
};

// Narrow-phase staging: active pairs compacted per tile before the final copy.
struct StageWs {
  int* si;       // [cand cap]
  int* sj;       // [cand cap]
  unsigned* sm;  // [cand cap] type | code << 8 | flags << 16
  double* sd;    // [cand cap] distance
  int* kcnt;     // [4 * G + 1] per-kind counts per tile (kind-major; kind 3: deferred)
  int* kofs;     // [4 * G + 1] their exclusive scan
  int* ccnt;     // [3 * G] per-tile N_c, N_filt, N_infeasible
  long long* dfr;  // [cand cap] deferred candidates (indices), in candidate order
  int* dfr2;       // [cand cap] deferred indices that double-double left open (k_band, any order)
  int* n2;         // [1] their number
  int* xcnt;       // [5 * XP_BLOCKS] per-range counts of the deferred results
  int* scan_tmp;
  long long cap; // staging capacity in candidates
};

// Assembly scratch.
struct AsmWs {
  int* inc_cnt;   // [V + 1] incidence entries per vertex, zero between steps
  int* inc_off;   // [V + 1] their exclusive scan
  int* inc;       // [4 * act_cap] entries 4k + s grouped by vertex
  int* colbuf;    // [16 * act_cap] stencil vertices of each entry's pair (row columns, sorted per row)
  int4* stn;      // [4 * act_cap] stencil of each incidence entry's pair, in the row's sorted entry order
  int* rowcnt;    // [V + 1] distinct columns per row
  int* mid;       // [V + 1] rows with 16 < m <= 256 entries (pass A's list, any order); mid[V] = their number
  int* big;       // [V + 1] rows with m > 256 entries (pass A's list, any order); big[V] = their number
  double* epart;  // [act_cap / 64 + 1] energy of each 64-pair tile of the evaluation
  int* scan_tmp;
};


}  // namespace bfc
