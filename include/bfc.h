/*
 * bfc.h -- C ABI of libbfc: barrier-filtered contact evaluation for thickened
 * rods and shells on one MI355X (gfx950).
 *
 * The method (Gomez-Nogales, Chen, Martin, Garces, Kaufman, "Unlocking
 * Thickness Modeling for Codimensional Contact Simulation"):
 *   - contact stencils are point-triangle and edge-edge pairs of a rod
 *     (edge-edge only) or shell mesh (Sec. 3, first paragraphs);
 *   - in a precomputation, stencil pairs of one connected component whose
 *     reference (parametric-space) distance dbar lies in (0, h) are labelled,
 *     and d_min is the smallest such distance (Sec. 3.2);
 *   - each pair then keeps fixed barrier parameters: activation h with
 *     offset eta, or activation d_min with no offset for labelled pairs
 *     (Eq. 4; Eq. 1 when eta = 0);
 *   - the barrier is the IPC log barrier of Eq. 2 with the biphasic offset of
 *     Eq. 3, b(d, a, eta) = -(d-a)^2 ln((d-eta)/(a-eta)) for eta < d < a;
 *   - the broad phase uses the full activation h for every pair (Sec. 3.3,
 *     last paragraph);
 *   - a projected Newton solver consumes the energy, gradient and per-pair
 *     PSD-projected Hessian (App. A).
 *
 * Units are the caller's; all lengths must use one unit.
 *
 * Memory and streams.  Positions and every output buffer are device memory
 * owned by the caller (suffix _d); host arrays carry suffix _h and are copied
 * during the call that takes them.  A scene owns device memory for its copy
 * of the topology, its precomputed filter data and its scratch space; it is
 * allocated by bf_scene_create and bf_scene_reserve only, never by the four
 * per-step calls; it is stream-ordered memory (allocated on the stream given
 * to bf_scene_create, freed by bf_scene_destroy on the scene's last stream).  Every call enqueues its work on the given stream (a
 * hipStream_t passed as void*, NULL = default stream) and returns without
 * synchronising unless stated.  Calls on one scene must not overlap.
 *
 * Errors.  Argument and state errors return synchronously with a status code
 * and a thread-local message (bf_last_error).  Conditions found on the device
 * (capacity overflow, infeasible pair, an eigen-iteration at its step limit,
 * a scan that stopped waiting) set bits in the scene's device status word,
 * read by bf_status_word (which synchronises); they never abort a kernel.  On
 * overflow the device counters still hold the required size so the caller
 * can grow its buffers and call again.
 */
#ifndef BFC_H
#define BFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_scene bf_scene;

typedef enum {
  BF_OK = 0,
  BF_E_ARG = 1,      /* invalid argument (null pointer, bad size or enum) */
  BF_E_NOMEM = 2,    /* device allocation failed in create/reserve */
  BF_E_DEVICE = 3,   /* a HIP runtime call failed */
  BF_E_CAPACITY = 4, /* a caller buffer is too small (synchronous checks) */
  BF_E_STATE = 5,    /* call order violated */
  BF_E_DEGENERATE = 6 /* a degenerate rest primitive: an edge whose two vertices have the same
                         rest parameters, or a triangle of zero rest area; under
                         BF_REFDIST_EUCLID_REST also a rest pose where two primitives of one
                         component that share no vertex touch (dbar^2 <= 1e-12 h^2)
                         (bf_scene_create) */
} bf_status;

enum { BF_ROD = 0, BF_SHELL = 1 };
enum { BF_FP64 = 0, BF_MIXED = 1 };
enum { BF_FILTER_PAPER = 0, BF_FILTER_NONE = 1, BF_FILTER_CULL = 2 };
/* What the reference distance dbar of Eq. 1 and Eq. 4 measures (Sec. 3.2):
 * BF_REFDIST_PARAM (default): distance in rest-space parameters, arc length
 * for rods and 2D rest coordinates for shells (Sec. 1 and Sec. 3.4: the
 * filter analyses distances along polylines and triangulations);
 * BF_REFDIST_EUCLID_REST: the literal alternative, the Euclidean distance
 * between the two primitives at a rest pose (bf_mesh_desc.ref_pos_h).  The
 * two differ where a polyline or sheet comes back near itself at rest: a
 * rod loop's successive turns are far apart along the rod but close in
 * space, and only the Euclidean reading filters them. */
enum { BF_REFDIST_PARAM = 0, BF_REFDIST_EUCLID_REST = 1 };

/* device status word bits */
enum {
  BF_S_CAND_OVERFLOW = 1u << 0,   /* candidate list capacity exceeded */
  BF_S_ACT_OVERFLOW = 1u << 1,    /* active list capacity exceeded */
  BF_S_INFEASIBLE = 1u << 2,      /* some active pair has d <= eta (energy +inf) */
  BF_S_BSR_OVERFLOW = 1u << 3,   /* BSR block capacity exceeded */
  BF_S_CORE_OVERFLOW = 1u << 4,  /* more core pairs than bf_core_mark's capacity */
  BF_S_EIG_NOCONV = 1u << 5,     /* a pair Hessian's eigen-iteration hit its step limit
                                    (that pair's projection is not exact) */
  BF_S_SCAN_SLOW = 1u << 6,      /* a single-pass scan stopped waiting for an earlier
                                    tile's total and summed that tile itself (results
                                    exact; reported for diagnosis) */
  BF_S_EXACT_LIMIT = 1u << 7     /* an exact threshold decision needed more than the
                                    expansion length it has room for (coordinates
                                    spanning hundreds of binary orders of magnitude);
                                    the double-double decision was kept */
};

/* Pair types. */
enum { BF_PT = 0, BF_EE = 1 };

/* Per-active-pair flag bits (BF_F_CORE: under the temporary zero offset of
 * Sec. 3.4, see bf_core_mark). */
enum { BF_F_FILTERED = 1, BF_F_INFEASIBLE = 4, BF_F_CORE = 8 };

typedef struct {
  double h;        /* thickness: activation distance of unfiltered pairs (Sec. 3) */
  double eta;      /* biphasic offset of unfiltered pairs, 0 <= eta < h (Eq. 3) */
  double kappa;    /* barrier stiffness multiplying every pair energy (> 0) */
  int32_t prec;    /* BF_FP64, or BF_MIXED: the PSD projection of each pair's reduced
                      system runs in FP32 (results within 1e-5 relative instead of about
                      1e-13) and the per-pair Hessian records (bf_local) are FP32;
                      distances, decisions, energies and gradients stay FP64 in both
                      modes, which use FP32 boxes in the broad phase and exact threshold
                      decisions */
  int32_t filter;  /* BF_FILTER_PAPER (Eq. 4), BF_FILTER_NONE (offset barrier everywhere), or
                      BF_FILTER_CULL (rods only: the comparison mode of Kaldor et al. that the
                      paper discusses in Sec. 2 and App. A: pairs of edges of one polyline at
                      most cull_radius elements apart are left out of contact, every other pair
                      takes (h, eta)) */
  int32_t cull_radius; /* BF_FILTER_CULL: radius in elements (the paper uses 11, and 5); >= 1 */
  int32_t refdist;     /* BF_REFDIST_PARAM or BF_REFDIST_EUCLID_REST (above) */
} bf_params;

typedef struct {
  int32_t kind;           /* BF_ROD or BF_SHELL */
  int64_t n_verts;        /* V >= 2 */
  int64_t n_edges;        /* E >= 1; shells: every triangle edge exactly once */
  int64_t n_tris;         /* F (0 for rods) */
  const int32_t* edges_h; /* [E,2] vertex ids */
  const int32_t* tris_h;  /* [F,3] vertex ids (NULL for rods) */
  const double* ref_h;    /* rest parameters: rods [V] arc length; shells [V,2] rest 2D coords */
  const double* ref_pos_h; /* [V,3] rest pose, read under BF_REFDIST_EUCLID_REST only (else may be
                              NULL); copied at bf_scene_create */
} bf_mesh_desc;

/* Candidate or active pair list (structure of arrays, device memory).
 * Point-triangle pairs: i = vertex, j = triangle.  Edge-edge: i < j edge ids. */
typedef struct {
  int32_t* i_d;
  int32_t* j_d;
  uint8_t* type_d;   /* BF_PT / BF_EE */
  int64_t cap;       /* capacity of the three arrays */
  int64_t* count_d;  /* [1] pairs written; if > cap, the size required */
} bf_pairs;

typedef struct {
  bf_pairs p;           /* active pairs */
  uint8_t* code_d;      /* [cap] distance sub-case (which features are closest) */
  uint8_t* flags_d;     /* [cap] BF_F_* bits */
  double* dist_d;       /* [cap] distance d */
  int64_t* counters_d;  /* [4]: N_c (pairs with d < h), N_filt (filtered among them),
                           N_act (active), N_infeasible */
} bf_active;

/* Per-active-pair results, row k for active pair k.  The 12 DOFs are the
 * pair's four stencil vertices in the order (point, t0, t1, t2) or
 * (a0, a1, b0, b1), xyz each.  H holds the upper triangle of the symmetric
 * projected 12 x 12 Hessian, packed by 3 x 3 blocks (78 entries): block-row s
 * (the three rows of stencil vertex s) is block (s, s) as its upper triangle
 * (xx, xy, xz, yy, yz, zz) followed by blocks (s, t), t > s, each row-major;
 * block-rows 0, 1, 2, 3 start at 0, 33, 57 and 72.  The entries are doubles
 * in a BF_FP64 scene and floats in a BF_MIXED scene (whose projection runs in
 * FP32: storing its result in FP32 adds a rounding of 6e-8 relative per entry
 * and halves the bytes the evaluation writes and the assembly reads). */
typedef struct {
  double* E_d;  /* [cap] kappa * b (+inf for infeasible pairs) */
  double* G_d;  /* [cap,12] gradient */
  void* H_d;    /* [cap,78] projected Hessian, packed upper triangle (above): double
                   (BF_FP64) or float (BF_MIXED) */
  int64_t cap;
} bf_local;

/* Block sparse (3x3) matrix, rows = vertices, columns sorted in each row. */
typedef struct {
  int32_t* row_ptr_d;  /* [V+1] */
  int32_t* col_d;      /* [cap] */
  double* val_d;       /* [cap,9] row-major 3x3 blocks */
  int64_t cap;
  int64_t* nnzb_d;     /* [1] blocks written; if > cap, the number required */
} bf_bsr;

/* Create a scene: copies the topology and rest parameters to the device,
 * labels connected components and computes d_min per component (Sec. 3.2).
 * cand_cap / act_cap size the scene scratch used by the per-step calls
 * (narrow-phase staging, assembly incidence lists); they bound the candidate
 * and active capacities the scene accepts without bf_scene_reserve
 * (act_cap at most 2^28 pairs, BF_E_ARG beyond).  Synchronises the stream. */
bf_status bf_scene_create(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                          int64_t act_cap, void* stream, bf_scene** out);

/* Caller-owned scene memory.  bf_workspace_bytes writes to *bytes_h the
 * size of the device workspace that holds everything a scene created with
 * these arguments keeps (topology, rest data, broad-phase, narrow-phase and
 * assembly workspaces for cand_cap candidates and act_cap active pairs); it
 * touches no device.  bf_scene_create_ws creates the scene as
 * bf_scene_create does, but carves all of that from ws_d (device memory of
 * ws_bytes bytes, any alignment, owned by the caller, which must keep it
 * until bf_scene_destroy and must not touch it meanwhile); the library never
 * frees it.  Short-lived temporaries of the creation itself (component
 * labelling, the rest-space candidate list) are still allocated and freed
 * before it returns, and the optional core set (bf_core_mark) and lagged
 * friction structure (friction_lag) allocate on first use.  BF_E_CAPACITY
 * if ws_bytes is below the size bf_workspace_bytes gives.  Such a scene
 * cannot grow: bf_scene_reserve beyond its capacities returns BF_E_STATE. */
bf_status bf_workspace_bytes(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                             int64_t act_cap, int64_t* bytes_h);
bf_status bf_scene_create_ws(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                             int64_t act_cap, void* ws_d, int64_t ws_bytes, void* stream, bf_scene** out);

/* Grow the scene scratch to hold at least cand_cap candidates / act_cap
 * active pairs (allocates and synchronises the device; not for use inside
 * captured graphs). */
bf_status bf_scene_reserve(bf_scene* s, int64_t cand_cap, int64_t act_cap);

/* Frees the scene's device memory in stream order after the work last
 * enqueued for it (on the stream of its last call or batch launch); work of
 * the scene on any other stream must be complete.  Does not synchronise. */
bf_status bf_scene_destroy(bf_scene* s);

/* Precompute results: component of each vertex, number of components, and
 * per-component d_min^2 / d_min (+inf where no stencil pair is closer than
 * h).  comp_h [V], dmin2_h / dmin_h [cap_c].  Synchronises. */
bf_status bf_scene_info(bf_scene* s, int32_t* comp_h, int32_t* n_comp, double* dmin2_h,
                        double* dmin_h, int32_t cap_c);

/* Broad phase at the full activation distance h (Sec. 3.3): writes every
 * non-incident pair whose bounding boxes are closer than h (their Euclidean
 * distance, a lower bound on the primitives', below h with a relative margin
 * of 1e-9).  The list is a superset of the pairs with d < h.  x_d: [V,3]
 * FP64 positions. */
bf_status build_candidates(bf_scene* s, const double* x_d, bf_pairs* cand, void* stream);

/* Narrow phase and filter (Eq. 4): for each candidate computes the distance,
 * counts it when d < h, assigns (a, eta) = (d_min, 0) to stencil pairs with
 * 0 < dbar < h and (h, eta) otherwise, and compacts the active pairs (d < a)
 * into act.  Threshold decisions are exact for the FP64 inputs (double
 * precision with a double-double re-evaluation inside a guard band). */
bf_status filter_pairs(bf_scene* s, const double* x_d, const bf_pairs* cand, bf_active* act,
                       void* stream);

/* Barrier energy, gradient and PSD-projected Hessian of every active pair
 * (Eq. 2, Eq. 3; projection: eigenvalues clamped at zero).  While the
 * evaluation kernel runs, the scene's internal stream (forked from `stream`
 * and joined back into it before the call returns) builds the structure of
 * the assembly for this active list (incidence lists, sorted columns of
 * every row), so that assemble_grad_hess only adds values.  While `stream`
 * is being captured into a graph there is no fork: assemble_grad_hess then
 * builds the structure itself. */
bf_status eval_barrier(bf_scene* s, const double* x_d, const bf_active* act, bf_local* out,
                       void* stream);

/* Assembly: E_d[1] = sum of pair energies (+inf if any pair is infeasible),
 * g_d[V,3] = sum of pair gradients, H = sum of pair Hessian blocks over the
 * 4x4 vertex blocks of every feasible active pair's stencil.  loc must hold
 * what this scene's last eval_barrier wrote for the same active list (the
 * energy total is taken from that call's per-tile sums).  Every sum runs in a
 * fixed order: results are bitwise repeatable. */
bf_status assemble_grad_hess(bf_scene* s, const bf_active* act, const bf_local* loc, double* E_d,
                             double* g_d, bf_bsr* H, void* stream);

/* ---- line search (Sec. 3.3, last paragraph; App. A) ---------------------
 * The Newton iteration's line search needs a step that keeps every pair
 * outside its offset, and the energy alone at trial points.  The offsets
 * follow Eq. 4: eta for ordinary pairs, 0 for filtered stencil pairs.
 *
 * build_candidates_swept: the broad phase of build_candidates on the boxes
 * swept by each primitive from x to x + p (p_d: [V,3] FP64 displacements,
 * the search direction times the largest step), with the per-axis test only
 * (every pair whose swept boxes are closer than h on every axis).  The list
 * holds every pair whose d(x + tau p) < h for some tau in [0, 1], so it
 * serves the CCD below and eval_energy at any point of the segment.
 *
 * max_step_accd: for every candidate whose exact swept boxes (vertices at x
 * and x + p, FP64) are closer than h on every axis, additive CCD (Li et al.
 * 2021) with the pair's offset xi: steps of (1 - accd_s) of the gap d - xi,
 * then 0.9 of the current gap, over the bound on the relative motion after
 * removing the stencil's mean displacement; the search stops before the
 * step after which the gap falls below accd_s of its initial value, at the
 * full step 1, or after max_iter steps.  t_d[1] (device) = the smallest step
 * in [0, 1] (0 if a pair starts at or inside its offset, 1 if there is no
 * pair).  tpair_d (device, [cand->cap], may be NULL) receives each
 * candidate's step, or -1 for candidates outside the swept set; iters_d
 * (device int32 [cand->cap], may be NULL) its number of steps (0 outside the
 * set; max_iter where the cap ended the search).  accd_s in (0, 1) (0.1 is
 * usual), max_iter >= 1; BF_E_ARG otherwise.
 *
 * eval_energy: E_d[1] (device) = the filtered barrier energy (Eq. 2, Eq. 4)
 * of the candidates at positions x_d, or at x_d + alpha p_d when p_d and
 * alpha_d (device, one double, e.g. the t_d of max_step_accd) are given
 * (each coordinate x + alpha * p, product then sum); with the decisions of
 * filter_pairs; +inf if a pair is at or inside its offset.  The candidates
 * must include every pair with d < h at the evaluated point (a
 * build_candidates list there, or a swept list whose segment holds it).
 * The sum runs in a fixed order: repeatable bit for bit.
 *
 * All three enqueue on `stream` and do not synchronise; the workspace of the
 * last two is per scene (calls on one scene are stream-ordered). */
bf_status build_candidates_swept(bf_scene* s, const double* x_d, const double* p_d, bf_pairs* cand,
                                 void* stream);
bf_status max_step_accd(bf_scene* s, const double* x_d, const double* p_d, const bf_pairs* cand,
                        double accd_s, int32_t max_iter, double* t_d, double* tpair_d, int32_t* iters_d,
                        void* stream);
bf_status eval_energy(bf_scene* s, const double* x_d, const double* p_d, const double* alpha_d,
                      const bf_pairs* cand, double* E_d, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as eval_energy, with the same arguments and results (bitwise),
 * whose per-work-group partial sums live in a static device array of the
 * library (8,192 doubles, 64 KiB per device, held until the process ends)
 * instead of the scene's scratch.  It allocates nothing and takes any
 * candidate count (the energy kernel strides over the list with at most
 * 8,192 work-groups); BF_E_CAPACITY if the partials would not fit.  All
 * calls on one device share the array: calls that overlap on one device
 * race; calls one after another on a stream do not. */
bf_status eval_energy_noalloc(bf_scene* s, const double* x_d, const double* p_d, const double* alpha_d,
                              const bf_pairs* cand, double* E_d, void* stream);

/* ---- temporary zero offset (Sec. 3.4) -----------------------------------
 * Pairs that are not stencils but start closer than eta (inside the core:
 * an input intersecting within the offset) make the biphasic barrier
 * infinite.  The paper proposes a temporary filter: such pairs get offset 0
 * (activation h, the single-phase barrier) until relaxation pushes them
 * beyond eta.
 *
 * bf_core_mark: (re)builds the scene's set from the candidates at x_d: every
 * candidate with d < h and d <= eta that is not a filtered stencil (the
 * decisions of filter_pairs).  cap = the most pairs expected (the table
 * holds at least 2 cap slots; a larger set raises BF_S_CORE_OVERFLOW and
 * keeps the pairs that fit); count_d (device int64) = pairs marked.
 * Synchronises when the table has to grow.
 *
 * While a set exists, filter_pairs first releases every pair of the set that
 * is now at d > eta (for good), then gives the remaining ones (h, 0) and the
 * flag BF_F_CORE; eval_barrier, eval_energy and max_step_accd use offset 0
 * for them too.  bf_core_live: count_d = pairs not yet released.
 * bf_core_clear: drop the set.  A batch captures the set as it is when the
 * batch is created (mark before bf_batch_create). */
bf_status bf_core_mark(bf_scene* s, const double* x_d, const bf_pairs* cand, int64_t cap, int64_t* count_d,
                       void* stream);
bf_status bf_core_live(bf_scene* s, int64_t* count_d, void* stream);
bf_status bf_core_clear(bf_scene* s);

/* ---- lagged friction (App. A: IPC's contact and friction energies) --------
 * IPC's lagged friction on the active pairs.  friction_lag, at the lagged
 * positions xlag_d (the start of the time step; act from filter_pairs there):
 * per active pair k, the normal force lam[k] = kappa |b'(d)| of its barrier
 * (Eq. 2-4 with the pair's (a, eta); 0 when infeasible), the weights w[k,4]
 * of the closest points (their relative displacement is sum_q w_q dx_q for
 * the pair's stencil vertices) and the contact normal n[k,3].
 *
 * friction_eval at x_d: with dt the part of sum_q w_q (x_q - xlag_q)
 * orthogonal to n and y = |dt|, the energy mu lam f0(y) (f0(y) = y for
 * y >= eps_vh, -y^3/(3 eps_vh^2) + y^2/eps_vh + eps_vh/3 below; eps_vh = the
 * sliding threshold times the time step, > 0), its gradient [12] and its
 * Hessian [12x12] (positive semidefinite as it stands) in the layout of
 * eval_barrier.  accumulate = 0 overwrites out, 1 adds to it (after
 * eval_barrier: contact + friction); either way the energy tile sums are
 * refreshed, so assemble_grad_hess then assembles what out holds.
 * mu >= 0, eps_vh > 0; fr capacity >= act capacity. */
typedef struct {
  double* lam_d;  /* [cap] */
  double* w_d;    /* [cap,4] */
  double* n_d;    /* [cap,3] */
  int64_t cap;
} bf_friction;
bf_status friction_lag(bf_scene* s, const double* xlag_d, const bf_active* act, bf_friction* fr, void* stream);
bf_status friction_eval(bf_scene* s, const double* x_d, const double* xlag_d, const bf_active* act,
                        const bf_friction* fr, double mu, double eps_vh, int32_t accumulate, bf_local* out,
                        void* stream);
/* The friction's sums over the lagged list (same outputs and fixed order as
 * assemble_grad_hess): friction_lag also builds the assembly structure of
 * its list (incidence lists, sorted row columns) in a workspace of the
 * scene's own, so friction_assemble only adds the values that the last
 * friction_eval (accumulate = 0) wrote into loc.  act must be the list given
 * to the last friction_lag, unchanged (BF_E_STATE for any other list) and
 * within the scene's active capacity.  friction_lag synchronises the device
 * when it (re)allocates that workspace: on the first call, and when the
 * list's capacity grows; otherwise neither call synchronises. */
bf_status friction_assemble(bf_scene* s, const bf_active* act, const bf_local* loc, double* E_d, double* g_d,
                            bf_bsr* H, void* stream);

/* ---- tuning ---------------------------------------------------------------
 * Threads per broad-phase query (2, 4, 8 or 16; default 4): more threads split a
 * query's rows of grid cells finer (small scenes, few queries), fewer cost
 * less bookkeeping (large scenes).  bf_scene_tune times build_candidates with
 * each choice on the positions x_d (reps timed launches each, median) and
 * keeps the fastest; it synchronises and must not be called inside a
 * captured graph.  cand is overwritten. */
bf_status bf_scene_set_pq(bf_scene* s, int32_t pq);
bf_status bf_scene_tune(bf_scene* s, const double* x_d, bf_pairs* cand, int32_t reps, void* stream,
                        int32_t* pq_out);

/* ---- batches of independent scenes ------------------------------------------
 * A batch evaluates many scenes (independent meshes, each with its own
 * positions and buffers) with one HIP graph launch: the whole path of every
 * scene is captured once, the scenes spread over `lanes` streams inside the
 * graph (forked from and joined back to the launching stream), so the small
 * kernels of different scenes run side by side.  Scenes go to lanes by
 * decreasing primitive count, each to the least loaded lane.  lanes = 0 takes
 * 4, the hardware queues a process gets on this device.
 * Items are copied; the scenes and buffers they name must outlive the batch
 * and keep their capacities (rebuild the batch after bf_scene_reserve).
 * Results of a scene are bitwise those of its own four calls. */
typedef struct {
  bf_scene* scene;
  const double* x_d;  /* [V,3] positions, read at every step */
  bf_pairs cand;
  bf_active act;
  bf_local loc;
  double* E_d;        /* [1] */
  double* g_d;        /* [V,3] */
  bf_bsr H;
} bf_batch_item;

typedef struct bf_batch bf_batch;

/* Capture the batch (once); synchronises. */
bf_status bf_batch_create(const bf_batch_item* items, int32_t n, int32_t lanes, void* stream, bf_batch** out);
/* One step of every scene of the batch: one graph launch on `stream`. */
bf_status bf_batch_step(bf_batch* b, void* stream);
/* Lanes in use and the lane of every item (lane_of_h [n], may be NULL). */
bf_status bf_batch_info(const bf_batch* b, int32_t* lanes, int32_t* lane_of_h);
/* Waits for the batch's last launch, then frees it (the scenes stay). */
bf_status bf_batch_destroy(bf_batch* b);

/* ---- serving: requests for many registered scenes ---------------------
 * A server keeps the registered scenes' host data (copied at start) and runs
 * requests (a scene and its positions) with a worker thread of its own
 * (and a builder thread that creates the scenes made resident).
 * All its device memory is one block of budget_bytes, allocated at start.
 * A resident scene holds in it only what persists between its steps
 * (topology, rest data and filter precompute: its footprint, bf_serve_info);
 * a request on the device holds, while it runs, a block with its step's
 * workspaces (broad phase, narrow-phase staging, assembly) and buffers.
 * Admission takes requests in arrival order: one starts when a slot is free,
 * its scene is idle and its scene (if not resident) and its step fit, room
 * being made by destroying the idle resident scenes of the range that frees
 * a long enough block at the least cost (bytes to build again, then the
 * least recently used); one that
 * cannot start while a slot is free lets later ones pass in at most
 * max_bypass admission passes, after which it blocks those behind it.  At most one request per scene is on the
 * device at a time.  A request runs the whole path (build_candidates,
 * filter_pairs, eval_barrier, assemble_grad_hess) and completes when its
 * results are in host memory: energy, counters, the step's status word
 * (read and cleared) and, if g_h was given, the gradient written to g_h.  A
 * step whose buffers overflowed runs again with the scene's capacities grown
 * to the sizes it reported, up to four times while the scene and its step
 * fit the budget; an overflow left after that shows in the status bits.  A
 * request whose scene and step exceed the budget completes with
 * BF_E_CAPACITY. */
typedef struct bf_server bf_server;
typedef struct {
  int32_t n_scenes;
  const bf_mesh_desc* meshes;  /* [n_scenes] */
  const bf_params* params;     /* [n_scenes] */
  const int64_t* cand_cap;     /* [n_scenes] capacities of each scene's step */
  const int64_t* act_cap;      /* [n_scenes] */
  const int64_t* bsr_cap;      /* [n_scenes] BSR blocks */
  int64_t budget_bytes;        /* all device memory of the server: resident scenes and running steps (each
                                  scene with one step must fit) */
  int32_t slots;               /* requests on the device at once, 1..64 */
  int32_t max_bypass;          /* >= 0 */
  int32_t device;              /* HIP device of the server */
} bf_serve_config;
typedef struct {
  int32_t done;      /* 1 once the request has completed (the other fields are then set) */
  int32_t scene;
  bf_status error;   /* BF_OK, or why the request could not run (bf_last_error is per thread) */
  uint32_t status;   /* the step's status word (BF_S_* bits) */
  double E;          /* total energy (+inf if a pair is infeasible) */
  int64_t counts[5]; /* N_c, N_filt, N_act, N_infeasible, BSR blocks */
  int64_t n_bp;      /* candidates of the broad phase */
  double ms;         /* submit to completion, host clock */
  int32_t retries;   /* runs again after a capacity overflow (the scene's capacities grown to the sizes
                        its counters reported; at most four) */
} bf_serve_result;
/* Start a server (allocates the budget's device block). */
bf_status bf_serve_start(const bf_serve_config* cfg, bf_server** out);
/* Queue a request: x_h [V,3] positions of the scene's vertices (copied
 * before return); g_h [V,3] (host, may be NULL) receives the gradient and
 * must stay valid until the request completes.  *ticket_h identifies it. */
bf_status bf_serve_submit(bf_server* sv, int32_t scene, const double* x_h, double* g_h, int64_t* ticket_h);
/* State of a request (wait != 0: block until it completes).  A completed
 * request's ticket is released by the poll that reports it. */
bf_status bf_serve_poll(bf_server* sv, int64_t ticket, int32_t wait, bf_serve_result* out);
/* Resident scenes, bytes of the budget in use (resident scenes and running
 * steps), (sizes_h[n_scenes, 2], may be NULL) each scene's footprint when
 * resident and the block its step takes (at its current capacities), and
 * (events_h[4], may be NULL) the scene creations, evictions and overflow
 * re-runs since start, then the most bytes in use at once. */
bf_status bf_serve_info(bf_server* sv, int32_t* resident_h, int64_t* used_bytes_h, int64_t* sizes_h,
                        int64_t* events_h);
/* Finish every queued request, destroy the resident scenes, free all. */
bf_status bf_serve_stop(bf_server* sv);

/* Device status word (BF_S_* bits) accumulated since the last clear;
 * synchronises the stream the scene last used.  clear != 0 resets it. */
bf_status bf_status_word(bf_scene* s, uint32_t* bits_h, int32_t clear);

/* ---- per-stage timing (measurement) --------------------------------------
 * With timing on, every stage below records a pair of HIP events around its
 * kernels on the stream they run on (not while that stream is captured):
 *   BF_T_BROAD       build_candidates (grid, cells, pair count and emission)
 *   BF_T_NARROW      filter_pairs' decisions kernel (k_narrow)
 *   BF_T_COMPACT     filter_pairs' list: scan, compaction, exact decisions
 *   BF_T_EVAL        eval_barrier's evaluation kernel (k_eval)
 *   BF_T_ASM_STRUCT  the assembly's structure (eval_barrier's second stream, or
 *                    assemble_grad_hess)
 *   BF_T_ASM_VALUES  assemble_grad_hess's values
 * bf_scene_stage_ms synchronises on those events and writes the duration of
 * each stage's latest call (ms; -1 where the stage has not run since timing
 * was switched on) to ms_h[BF_T_COUNT].  Setting timing allocates events. */
/* Diagnostics of the last filter_pairs (synchronises): n_band_h, the
 * candidates with a value in FP64's relative band of 1e-9 around a threshold
 * (decided again by the exact-in-FP64 check and double-double); n_exact_h,
 * those of them that double-double left within 1e-20 of the threshold and
 * that were decided in exact arithmetic.  Either pointer may be NULL. */
bf_status bf_scene_deferred(bf_scene* s, int64_t* n_band_h, int64_t* n_exact_h);

enum { BF_T_BROAD = 0, BF_T_NARROW = 1, BF_T_COMPACT = 2, BF_T_EVAL = 3, BF_T_ASM_STRUCT = 4,
       BF_T_ASM_VALUES = 5, BF_T_COUNT = 6 };
bf_status bf_scene_set_timing(bf_scene* s, int32_t on);
bf_status bf_scene_stage_ms(bf_scene* s, float* ms_h);

/* Diagnostics: the number of loads a single-pass scan spends waiting for
 * each earlier tile's published total before it sums that tile itself
 * (BF_S_SCAN_SLOW).  Default 2^22; >= 0.  Process-wide; affects launches
 * enqueued after the call. */
bf_status bf_set_scan_poll_limit(int32_t polls);

/* Message of the last non-OK return on this thread. */
const char* bf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BFC_H */
