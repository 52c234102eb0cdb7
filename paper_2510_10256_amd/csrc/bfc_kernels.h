// Host-side launchers of the libbfc kernels (defined in bfc_kernels.hip).
#pragma once
#include "bfc.h"
#include "bfc_internal.h"

namespace bfc {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;
constexpr int SCAN1_MAX = 1 << 14;     // arrays up to this length are scanned by one work-group
constexpr int PQ_MAX = 16;             // threads per broad-phase query: 2, 4 (default), 8 or 16
constexpr int NW_ITEMS = 4;            // candidates per thread in the narrow phase
constexpr int LINE_BLOCKS = 8192;      // work-groups of the line-search kernels (grid-stride)
constexpr int NW_TILE = 256 * NW_ITEMS;
constexpr int NW_KINDS = 4;            // staged kinds in a narrow-phase tile: 9x9, 6x6, closed form, deferred
constexpr int NW_DEFER = 3;            // the deferred kind: decided exactly by k_exact
constexpr int XP_BLOCKS = 1024;        // work-groups of k_exact (ranges of its list) and of the deferred counts
constexpr int BAND_BLOCKS = 2048;      // work-groups of k_band (grid-stride over the deferred list)
constexpr int XP_TPB = 16;             // threads of a k_exact work-group, an LDS expansion slab each
constexpr int BOUNDS_BLOCKS = 512;     // cap on k_bounds work-groups (partials of the last-block reduction)

constexpr int SCAN_LB_TILES = 256;     // arrays of up to this many tiles take the single-pass scan
// The scan's scratch: first the single-pass scan's state (SCAN_LB_TILES 64-bit
// tile words, then a ticket and a done counter; zero when no scan runs, so
// it is cleared once when allocated), then the partials of the longer scans.
constexpr int SCAN_LB_STATE = 2 * SCAN_LB_TILES + 8;
// ints of scratch for a scan of n elements
inline long long scan_tmp_ints(long long n) { return SCAN_LB_STATE + (n + SCAN_TILE - 1) / SCAN_TILE + 1 + 16; }

// Exclusive scan; a single-pass scan that summed a missing tile total
// itself sets BF_S_SCAN_SLOW in *status (may be null).  g_scan_polls bounds
// that scan's wait for each earlier tile (loads of its published total).
extern int g_scan_polls;
void scan_excl(const int* in, int* out, const int* n_dev, int n_max, int* tmp, unsigned* status, hipStream_t st);

// Broad phase over the positions x (FP64 [V,3]) at inflation S.h.
void run_broad(const SceneDev& S, const double* x, const double* pdisp, const BroadWs& W, int* oi, int* oj,
               unsigned char* ot, long long cap, long long* count, unsigned* status, int* seg_r, unsigned* seg_t,
               long long seg_cap, hipStream_t st);
void run_accd(const SceneDev& S, const double* x, const double* pdisp, const int* ci, const int* cj,
              const unsigned char* ct, const long long* ccount, long long ccap, double s, int max_iter, double* tpair,
              int* iters, double* bred, double* t_out, hipStream_t st);
void run_core_mark(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                   const long long* ccount, long long ccap, unsigned long long* keys, unsigned char* live,
                   unsigned slots, long long cap, long long* count, unsigned* status, hipStream_t st);
void run_core_release(const SceneDev& S, const double* x, hipStream_t st);
void run_core_count(const SceneDev& S, long long* out, hipStream_t st);
void run_friction_lag(const SceneDev& S, const double* xl, const int* ai, const int* aj, const unsigned char* at,
                      const unsigned char* acode, const unsigned char* aflags, const long long* act_count,
                      long long acap, double* lam, double* w, double* n, hipStream_t st);
void run_friction_eval(const SceneDev& S, const double* x, const double* xl, const int* ai, const int* aj,
                       const unsigned char* at, const long long* act_count, long long acap, const double* lam,
                       const double* w, const double* n, double mu, double eh, int accumulate, double* E, double* G,
                       void* H, double* epart, hipStream_t st);
void run_energy(const SceneDev& S, const double* x, const double* pdisp, const double* alpha, const int* ci,
                const int* cj, const unsigned char* ct, const long long* ccount, long long ccap, double* bred,
                double* E_out, hipStream_t st);

// Narrow phase and filter (k_narrow: decisions and tile-local compaction),
// then the list: scan, k_compact, k_exact (the deferred exact decisions).
void run_narrow(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                const long long* ccount, long long ccap, const StageWs& W, hipStream_t st);
void run_compact(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                 long long ccap, const StageWs& W, int* ai, int* aj, unsigned char* at, unsigned char* acode,
                 unsigned char* aflags, double* adist, long long acap, long long* act_count, long long* counters,
                 unsigned* status, hipStream_t st);

// Per-pair barrier, gradient and projected Hessian.  The Hessian records
// (here and below) are doubles, or floats when S.mixed.
void run_eval(const SceneDev& S, const double* x, const int* ai, const int* aj, const unsigned char* at,
              const unsigned char* acode, const unsigned char* aflags, const long long* act_count, long long acap,
              double* E, double* G, void* H, double* epart, hipStream_t st);

// Assembly, structural part: needs the active list only (incidence lists,
// sorted entries, distinct columns per row).
void run_asm_structure(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                       const unsigned char* aflags, const long long* act_count, long long acap, const AsmWs& A,
                       hipStream_t st);

// Assembly, numerical part: row pointers, blocks, gradient and energy.
void run_asm_values(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                    const long long* act_count, long long acap, const double* G, const void* H, double* E_out,
                    double* g, int* row_ptr, int* col, double* val, long long bsr_cap, long long* nnzb,
                    const AsmWs& A, unsigned* status, hipStream_t st);

int run_components(const SceneDev& S, int* lab, int* flag, int* scan, int* comp, int* scan_tmp, int* d_changed,
                   hipStream_t st);

// a[0..n) = 0 for n <= 64 (a kernel: unlike a memset it may be captured)
// dst[0] = the status word, then the word is cleared (stream order).
void run_status_take(unsigned* status, unsigned* dst, hipStream_t st);
void run_zero_i64(long long* a, int n, hipStream_t st);

// Lift rest parameters to 3D points (rods (s,0,0); shells (u1,u2,0)).
void run_lift_ref(const SceneDev& S, double* xref, hipStream_t st);

// Per-component minimum of the reference distance over stencil pairs with
// 0 < dbar < h among the candidates (rods: gap; shells and the Euclidean
// reading: dbar^2 rounded).  ties [tie_cap]: the Euclidean reading's pairs
// decided exactly; flags[0] their count, flags[1] bit 0 touching primitives
// at rest, bit 1 an exact decision out of room.
void run_refmin(const SceneDev& S, const int* ci, const int* cj, const unsigned char* ct, const long long* count,
                long long cap, unsigned long long* best, long long* ties, long long tie_cap,
                unsigned long long* flags, hipStream_t st);

}  // namespace bfc
