/*
 * vasmg.h -- C ABI of the MI355X (gfx950) V-ASMG-preconditioned CG solver for
 * P1 finite-element linear elasticity (Li, Wu, Zhang, Liu, "Vertex-based
 * auxiliary space multigrid method and its application to linear elasticity
 * equations", arXiv 2505.09064).
 *
 * The library computes the paper's solve phase: PCG (Section 2.2, Algorithm 2)
 * preconditioned by one V-cycle (Section 3, Algorithm 3 applied recursively)
 * over the vertex-based auxiliary region-tree hierarchy (Section 3.1), with
 * Gauss-Seidel smoothing (Section 2.1, Algorithm 1), bilinear/trilinear
 * restriction and prolongation (Section 3.2), Galerkin coarse operators
 * A_c = P^T A P (Section 3, equations (R), (Ac)) and a direct coarsest solve.
 * The setup (assembly of Section 2, tree, levels, Galerkin products, colouring,
 * coarsest Cholesky) runs on the host inside vasmg_setup; every step of the
 * solve runs in hand-written HIP kernels on one GPU.
 *
 * Conventions for every function:
 *  - Return value: vasmg_status, VASMG_OK (0) on success. On failure a message
 *    is available from vasmg_last_error() (thread-local, valid until the next
 *    call on the same thread).
 *  - Ownership: vasmg_setup deep-copies the mesh; the caller may free it on
 *    return. The handle owns every host and device buffer it allocates until
 *    vasmg_free. Device pointers passed to *_device functions stay owned by the
 *    caller and must stay valid until the call returns (all *_device calls are
 *    synchronous with respect to the given stream on return).
 *  - Threads: one call in flight per handle. Different handles may be used
 *    from different threads.
 *  - Layouts: user-facing vectors are FP64, vertex-major [n_vertices][dim]
 *    (DOF = vertex*dim + component). Entries of a right-hand side or initial
 *    guess at fixed DOFs are ignored; solutions are 0 there. Level vectors of the debug entry
 *    points are [n_level_vertices][dim] in the level's canonical order (fine
 *    level: free vertices in ascending mesh index; coarse levels: vertices in
 *    lexicographic (z, y, x) lattice-key order).
 */
#ifndef VASMG_H
#define VASMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vasmg_ctx* vasmg_handle;

typedef enum {
  VASMG_OK = 0,
  VASMG_EINVAL = 1,       /* invalid argument or mesh (see vasmg_last_error)        */
  VASMG_ENOMEM = 2,       /* host or device allocation failed                        */
  VASMG_EDEVICE = 3,      /* HIP runtime error, or no device / host-only handle      */
  VASMG_ENOTCONV = 4,     /* max_iters reached; x and info hold the last iterate     */
  VASMG_EBREAKDOWN = 5,   /* p^T A p <= 0 or not finite (e.g. NaN right-hand side)   */
  VASMG_EDEGENERATE = 6   /* coarsest operator not positive definite (e.g. no BCs)   */
} vasmg_status;

enum { VASMG_FP64 = 0, VASMG_FP32_PRECOND = 1 };
enum { VASMG_TREE_ALL = 0, VASMG_TREE_FREE = 1 };
enum { VASMG_PRECOND_VASMG = 0, VASMG_PRECOND_JACOBI = 1, VASMG_PRECOND_NONE = 2 };
enum { VASMG_CYCLE_V = 0, VASMG_CYCLE_W = 1, VASMG_CYCLE_ADDITIVE = 2 };
enum { VASMG_SMOOTHER_GS = 0, VASMG_SMOOTHER_JACOBI = 1 };

/* Mesh: P1 triangles (dim 2, plane strain) or tetrahedra (dim 3); Section 2. */
typedef struct {
  int32_t dim;                 /* 2 or 3                                                 */
  int64_t n_vertices;
  const double* coords;        /* [n_vertices][dim], host                                */
  int64_t n_elements;
  const int32_t* elems;        /* [n_elements][dim+1], 0-based, positively oriented      */
  const double* E;             /* [n_elements] Young's modulus, > 0                       */
  const double* nu;            /* [n_elements] Poisson ratio, in (-1, 0.5)                */
  const uint8_t* fixed;        /* [n_vertices][dim], 1 = homogeneous Dirichlet DOF.
                                  Fully fixed vertices are eliminated; a vertex with
                                  some components fixed keeps its block with an
                                  identity row and column for each fixed component and
                                  zero prolongation rows for it (a coarse component
                                  whose interpolating fine vertices all have it fixed
                                  is constrained in turn): exactly eliminating those
                                  DOFs (rollers, symmetry planes).                        */
} vasmg_mesh;

typedef struct {
  int32_t leaf_capacity;       /* max vertices per leaf region (Section 3.1.1 Step 2);
                                  0 = default (4 in 2D as in the paper, 8 in 3D)          */
  int32_t n_pre, n_post;       /* GS sweeps before/after the coarse correction (V(1,1))  */
  int32_t precision;           /* VASMG_FP64 | VASMG_FP32_PRECOND (V-cycle in FP32,
                                  PCG, SpMV, dots and coarsest solve in FP64)             */
  int32_t tree_vertices;       /* VASMG_TREE_ALL (every mesh vertex, Section 3.1.1) or
                                  VASMG_TREE_FREE (only unconstrained vertices)           */
  int64_t coarsest_max_dofs;   /* 0 = coarsen to the root region (Section 3.1.2); else
                                  the first level with <= this many DOFs is the coarsest  */
  int32_t max_iters;           /* max products A p per solve (default 10000)             */
  int32_t preconditioner;      /* VASMG_PRECOND_VASMG (default) | _JACOBI | _NONE         */
  int32_t profile;             /* 1 = per-phase device timings in vasmg_solve_info       */
  int32_t host_only;           /* 1 = build the hierarchy on the host only (no device
                                  upload; solves return VASMG_EDEVICE). Introspection.    */
  int32_t verbose;             /* 1 = print level statistics at setup                     */
  int32_t autotune;            /* 1 = time the candidate lanes-per-block-row of each
                                  level's kernels at setup and keep the fastest (results
                                  then differ from another handle's by rounding only)     */
  int32_t block_rhs;           /* 0 = solve several right-hand sides one after another;
                                  4, 8 or 16 = block width K: vasmg_solve(_device) with
                                  n_rhs > 1 runs K columns at a time as K PCG recurrences
                                  sharing every matrix read (vectors interleaved per
                                  vertex); needs the V-ASMG preconditioner, n_pre >= 1 and
                                  a coarsest level of at most 4096 / K DOFs (else EINVAL) */
  int32_t cycle;               /* VASMG_CYCLE_V (default, Algorithm 3 recursive),
                                  VASMG_CYCLE_W (two coarse visits per level, Section 3
                                  cycle modes) or VASMG_CYCLE_ADDITIVE (Section 4's
                                  B = S + P B_1 P^T: the fine-level sweeps from zero plus
                                  the prolonged V-cycle of levels 1..L of P^T r)          */
  int32_t smoother;            /* VASMG_SMOOTHER_GS (default: multicolour point GS,
                                  Algorithm 1) or VASMG_SMOOTHER_JACOBI (damped
                                  vertex-block Jacobi, Section 4's other S_h: omega =
                                  (4/3) / lambda_max(D^-1 A), estimated per level by 30
                                  power iterations at setup)                            */
  int32_t setup_device;        /* 0 = hierarchy built on the host (default); 1 = the
                                  fine assembly, the region tree, lattice keys and
                                  prolongations (Section 3.1, 3.2: the host's
                                  decisions, keys and weights bit for bit; trees deeper
                                  than 21 levels in 3D or 32 in 2D are built on the
                                  host) and the Galerkin coarse operators
                                  A_{l+1} = P_l^T A_l P_l (Section 3, equation (Ac))
                                  are formed on the current HIP device, the latter
                                  with the same columns, values equal to rounding
                                  (another order of the FP64 sums), deterministic; the
                                  level layouts are then built from the resident
                                  operators, and the host copies of the FP64 level
                                  values arrive in the background after vasmg_setup
                                  returns (vasmg_export_level and vasmg_free wait for
                                  them). With host_only = 1 every value is brought
                                  back before vasmg_setup returns and no device memory
                                  is kept (a server's setup workers); EDEVICE without a
                                  device                                                  */
  int32_t color_blocks;        /* 0 = off (default): every Gauss-Seidel cell is its own
                                  colour block; 1 = on: on 3D lattice levels whose
                                  couplings reach 3 or 4 lattice steps, cells are grouped
                                  into colour blocks of 4 steps (up to 8 cells, swept one
                                  after the other inside a block), so that 8 colours
                                  suffice instead of 27. Ignored (off) with block_rhs.
                                  Changes the sweep order, hence results (the oracle
                                  takes the same order).                                 */
  int32_t block_lanes;         /* block_rhs only: lanes per block row of the block
                                  kernels. 0 (default) = per level from its row
                                  lengths, or timed with autotune = 1; 1 = the narrow
                                  groups on every level (16 per point row, 32 per cell
                                  row); 2 = the wide groups (64). Results differ by
                                  rounding only; EINVAL outside 0..2                    */
} vasmg_options;

typedef struct {
  int32_t iterations;          /* number of products A p when ||r||/||F|| < rtol held     */
  int32_t converged;           /* 1 if the recurrence residual reached rtol               */
  double rel_res;              /* recurrence ||r_k|| / ||F||                              */
  double rel_res_true;         /* ||F - A x|| / ||F|| recomputed in FP64 at exit           */
  double t_solve_ms;           /* device time of the whole solve (hipEvent)               */
  double t_spmv_ms;            /* profile=1: accumulated fine SpMV time                   */
  double t_precond_ms;         /* profile=1: accumulated V-cycle time                     */
  double t_vector_ms;          /* profile=1: accumulated PCG vector-kernel time           */
  double bytes_model;          /* algorithmic HBM bytes of the solve (byte model)         */
  int32_t status;              /* this solve's (column's, part's) status: VASMG_OK,
                                  VASMG_ENOTCONV or VASMG_EBREAKDOWN                     */
  int32_t reserved;
} vasmg_solve_info;

/* Fill *out with the defaults for dimension dim (2 or 3). */
vasmg_status vasmg_default_options(int32_t dim, vasmg_options* out);

/* Build the hierarchy (Section 3 setup step) on the host and upload it to the
 * current HIP device. opt may be NULL (defaults). On failure *out = NULL.
 * Errors: EINVAL (bad mesh/options; duplicate vertices exceed the tree's depth
 * limit), EDEGENERATE (coarsest operator not positive definite, e.g. no fixed
 * DOFs), ENOMEM, EDEVICE. */
vasmg_status vasmg_setup(const vasmg_mesh* mesh, const vasmg_options* opt, vasmg_handle* out);

/* Solve A x = rhs for n_rhs right-hand sides with PCG (Algorithm 2) to
 * ||F - A x|| / ||F|| < rtol (Section 5 (3)). Host pointers:
 * rhs, x: [n_rhs][n_vertices][dim]; x0: same or NULL (zero initial guess);
 * info: [n_rhs] or NULL. Returns the worst status over the columns. */
vasmg_status vasmg_solve(vasmg_handle h, const double* rhs, const double* x0, double* x,
                         int32_t n_rhs, double rtol, vasmg_solve_info* info);

/* Same with device pointers (e.g. torch tensor data_ptr()), enqueued on
 * stream (a hipStream_t; NULL = default stream). Returns after the solve has
 * finished on that stream. */
vasmg_status vasmg_solve_device(vasmg_handle h, const double* d_rhs, const double* d_x0,
                                double* d_x, int32_t n_rhs, double rtol, void* stream,
                                vasmg_solve_info* info);

/* No-allocation form of vasmg_solve, for callers that cannot allocate device
 * memory while they solve (code running under HIP graph capture elsewhere in
 * the process, tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments, results and statuses as vasmg_solve (identical x and info): the
 * host arrays are staged through one fixed array of the library on each GPU,
 * 64 MiB, held from the module's load on that GPU until the process ends,
 * instead of device buffers allocated per call; the call allocates nothing
 * (the handle's buffers and PCG graphs exist from vasmg_setup / vasmg_upload).
 * Staging takes n_rhs * n_vertices * dim * 8 bytes per array (rhs, x, and x0
 * when given), each rounded up to 256 bytes; a request for more than 64 MiB
 * fails with EINVAL before anything is copied. Every call on a GPU shares that
 * GPU's array: calls on one GPU run one at a time (a second call waits for the
 * first), and the array keeps the last call's data, none of which a call reads
 * before writing it. */
vasmg_status vasmg_solve_noalloc(vasmg_handle h, const double* rhs, const double* x0, double* x,
                                 int32_t n_rhs, double rtol, vasmg_solve_info* info);

/* Upload a hierarchy built with host_only = 1 to the current HIP device (the
 * device half of vasmg_setup, which then runs any block_rhs allocation and
 * autotuning the options ask for). stream (a hipStream_t) may be NULL; if set,
 * every device allocation of the handle is stream-ordered on it
 * (hipMallocAsync, and hipFreeAsync at vasmg_free, which must then happen
 * while the stream exists): a server can then upload, solve and free on one
 * stream without synchronising the device. Errors: EINVAL (already uploaded),
 * ENOMEM, EDEVICE. On failure the handle stays unusable for solves. */
vasmg_status vasmg_upload(vasmg_handle h, void* stream);

/* Device bytes of the handle: allocated bytes once uploaded, else an upper
 * bound of what vasmg_upload will allocate (admission control). */
vasmg_status vasmg_device_bytes(vasmg_handle h, int64_t* bytes);

/* ---------------------------------------------------------------------------
 * Packed solves: several small independent problems (one load case each) run
 * as one. The packed handle's hierarchy is the block-diagonal union of the
 * parts' (level l holds every part's level l; a part with fewer levels repeats
 * its coarsest level below its depth, joined by identity prolongations, so its
 * V-cycle still ends in its exact coarse solve); its coarsest factor is the
 * parts' factors on the diagonal. One SpMV and one V-cycle per iteration serve
 * every part, so a part pays the launches once for the whole pack; each part
 * keeps its own PCG recurrence (Section 2.2, Algorithm 2: its own dot products,
 * alpha, beta and stopping test ||r|| / ||F|| < rtol) and stops when it
 * converges, as it would alone (results equal to rounding: the dot products
 * sum in another order). Only vasmg_solve_packed(_device),
 * vasmg_apply_precond_device (the union's V-cycle), the introspection calls and
 * vasmg_free apply to a packed handle (EINVAL from the other solve calls).
 * ------------------------------------------------------------------------- */

/* Packs the hierarchies of n_parts handles (host-only or uploaded; each set up
 * with the V-ASMG Gauss-Seidel V-cycle, block_rhs = 0, color_blocks = 0, and the
 * same dim, precision and n_pre / n_post; EINVAL otherwise, or when their
 * coarsest levels hold more than 4096 DOFs together) into a new host-only
 * handle; upload it with vasmg_upload. The parts stay owned by the caller and
 * unchanged; max_iters is the largest of theirs. Packed vectors are the parts'
 * user vectors one after the other: part i's [n_vertices_i][dim] block starts
 * at vertex vertex_offsets[i] (vasmg_packed_info). */
vasmg_status vasmg_pack(const vasmg_handle* parts, int32_t n_parts, vasmg_handle* out);

/* Number of parts (0: not a packed handle) and, if vertex_offsets is non-NULL,
 * the n_parts + 1 vertex offsets of the parts in packed vectors. */
vasmg_status vasmg_packed_info(vasmg_handle h, int32_t* n_parts, int64_t* vertex_offsets);

/* Solves every part from x0 = 0 with rtol. d_rhs, d_x: packed vectors (device,
 * [sum n_vertices_i][dim], FP64); info: [n_parts] host array, one report per
 * part (iterations, converged, rel_res, rel_res_true; t_solve_ms is the whole
 * packed solve's device time). Returns EBREAKDOWN if some part broke down, else
 * ENOTCONV if some part did not reach rtol within max_iters, else OK; the other
 * parts' results are valid either way. */
vasmg_status vasmg_solve_packed_device(vasmg_handle h, const double* d_rhs, double* d_x, double rtol,
                                       void* stream, vasmg_solve_info* info);

/* vasmg_solve_packed_device with host vectors (staged through device buffers). */
vasmg_status vasmg_solve_packed(vasmg_handle h, const double* rhs, double* x, double rtol,
                                vasmg_solve_info* info);

/* Release every host and device resource of h. NULL-safe. */
void vasmg_free(vasmg_handle h);

/* Message of the last failure on this thread ("" if none). */
const char* vasmg_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent solve requests (one mesh and
 * one load case each) on one GPU. A request is set up on the host by one of
 * setup_workers threads (with options.setup_device = 1 its Galerkin products on
 * the device, in transient memory outside the budget, ordered on the worker's
 * own stream), admitted first in first out as soon as one of `slots`
 * device slots is free and its device bytes (vasmg_device_bytes) fit the HBM
 * budget next to the requests already resident, then uploaded, solved and
 * freed on the slot's own stream; requests overlap on the device. Every request
 * uses the server's options (autotuning off, so a result does not depend on
 * what else is running; block_rhs ignored). Thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct vasmg_server* vasmg_server_handle;

typedef struct {
  int32_t slots;               /* concurrent device solves (streams), 1..64, default 4    */
  int32_t setup_workers;       /* host threads building hierarchies, 1..64, default 4;
                                  a setup uses the host's threads divided by the
                                  number of setups running or queued when it starts
                                  (at most setup_workers)                                */
  int64_t hbm_budget_bytes;    /* device bytes resident requests may hold together;
                                  0 = 80% of the device's free memory at creation       */
  vasmg_options options;       /* solver options of every request (leaf_capacity 0 =
                                  each request's dimension default)                      */
  int32_t pack_max_dofs;       /* 0 (default) = every request solved on its own; > 0 =
                                  a request of at most this many DOFs admitted while
                                  other such requests (same dimension and rtol) wait
                                  set up is packed with them (vasmg_pack, up to
                                  pack_max_parts, their coarsest levels within 256
                                  DOFs together): one upload and one solve for the
                                  pack, each request with its own PCG recurrence.
                                  Packed results equal the request's alone result to
                                  rounding, not bit for bit. Needs the V-ASMG
                                  Gauss-Seidel V-cycle without colour blocks.           */
  int32_t pack_max_parts;      /* largest pack, 2..256 (default 16)                       */
  int32_t pack_wait_ms;        /* batching window, 0..10000 (default 0): a slot holding a
                                  packable request waits up to this long for more while
                                  setups are still running                               */
  int32_t host_setup_max_dofs_2d; /* with options.setup_device = 1: a request of at most
                                  this many DOFs (n_vertices * dim, fixed ones included)
                                  is set up on the host all the same, where the device
                                  setup's fixed costs (launches, host round trips of the
                                  tree's rounds, allocations) exceed the host's work;
                                  >= 0, default 131072 (2D) and 16384 (3D). Both setups
                                  build the same hierarchy (the Galerkin products to
                                  rounding)                                              */
  int32_t host_setup_max_dofs_3d;
  int32_t reserved;
} vasmg_server_config;

typedef struct {
  int64_t id;
  int32_t status;              /* of the request's setup, upload or solve; ENOMEM if its
                                  device bytes exceed the whole budget                  */
  int32_t slot;                /* device slot that ran it (-1: none)                      */
  int32_t pack_size;           /* requests solved together with it in one packed solve,
                                  itself included (1: alone, 0: never admitted)          */
  int32_t setup_device;        /* 1: its hierarchy was built by the device setup          */
  int64_t device_bytes;        /* device bytes it held while resident                     */
  double t_submit_ms, t_setup_start_ms, t_setup_end_ms, t_admit_ms, t_done_ms;
                               /* server clock (ms since vasmg_server_create)             */
  vasmg_solve_info info;       /* the solve's own report                                  */
  char message[128];           /* why it failed ("" if status is OK)                      */
} vasmg_request_result;

typedef struct {
  int64_t submitted, completed, waiting_setup, waiting_admission, running;
  int64_t bytes_in_use, peak_bytes, budget_bytes;
  double t_now_ms;
} vasmg_server_counters;

/* Defaults: 4 slots, 4 setup workers, 80% of free device memory, default options. */
vasmg_status vasmg_server_default_config(vasmg_server_config* cfg);

/* Start the server's threads on the current HIP device. EDEVICE without one. */
vasmg_status vasmg_server_create(const vasmg_server_config* cfg, vasmg_server_handle* out);

/* Queue a request; mesh and rhs ([n_vertices][dim], host) are copied, so the
 * caller may free them on return. Returns its id at once. */
vasmg_status vasmg_server_submit(vasmg_server_handle s, const vasmg_mesh* mesh, const double* rhs,
                                 double rtol, int64_t* id);

/* Block until request id has finished; x ([n_vertices][dim], host) may be NULL.
 * Returns the request's status; each id can be waited for once. */
vasmg_status vasmg_server_wait(vasmg_server_handle s, int64_t id, double* x,
                               vasmg_request_result* res);

/* Counters (requests, resident bytes, peak) at this moment. */
vasmg_status vasmg_server_stats(vasmg_server_handle s, vasmg_server_counters* out);

/* Finish every queued request, stop the threads and release everything. */
void vasmg_server_destroy(vasmg_server_handle s);

/* ---------------------------------------------------------------------------
 * Introspection (hierarchy produced by the setup; host data, no device use).
 * ------------------------------------------------------------------------- */

/* Number of levels L+1 (level 0 = fine, level L = coarsest) and the DOF count
 * of the fine level (dim * free vertices). */
vasmg_status vasmg_hierarchy_info(vasmg_handle h, int32_t* n_levels, int64_t* n_dofs,
                                  int32_t* dim);

/* Per level: vertices, stored d x d blocks (structural pattern incl. diagonal),
 * colours of the Gauss-Seidel order (0 on the coarsest level), entries of
 * P_level (0 on the coarsest). */
vasmg_status vasmg_level_info(vasmg_handle h, int32_t level, int64_t* n_vertices,
                              int64_t* n_blocks, int32_t* n_colors, int64_t* p_nnz);

/* Copy level data in canonical order into caller-allocated host arrays (any
 * pointer may be NULL to skip it):
 *   keys   [n_vertices][dim] int64 lattice keys (coarse levels; fine: -1)
 *   cell   [n_vertices] int32 Gauss-Seidel cell of each vertex (cells numbered in
 *          canonical order of their lattice keys; fine level: the vertex itself;
 *          coarsest level: 0)
 *   color  [n_vertices] int32 colour of the vertex's colour block (coarsest
 *          level: 0). A sweep visits colours ascending, then the colour blocks
 *          of a colour, then the cells of a block, then the vertices of a cell
 *          in canonical order, then components (Algorithm 1 in that order).
 *   block  [n_vertices] int32 colour block of each vertex (blocks numbered in
 *          canonical order of their lattice keys; the cell where every cell is
 *          its own block; coarsest level: 0)
 *   fixed  [n_vertices] uint8 constrained components of each vertex (bit a =
 *          component a; their rows and columns of vals are those of the
 *          identity)
 *   rowptr [n_vertices+1] int64, cols [n_blocks] int32, vals [n_blocks][dim][dim] FP64
 *   p_rowptr [n_vertices+1] int64, p_cols [p_nnz] int32, p_vals [p_nnz] FP64
 *     (scalar prolongation P_level from this level's vertices to the next's).
 * On a handle set up with setup_device = 1 it first waits for the background
 * download of the level values (EDEVICE if that failed). */
vasmg_status vasmg_export_level(vasmg_handle h, int32_t level, int64_t* keys, int32_t* cell,
                                int32_t* color, int64_t* rowptr, int32_t* cols, double* vals,
                                int64_t* p_rowptr, int32_t* p_cols, double* p_vals,
                                int32_t* block, uint8_t* fixed);

/* Root box [m, M]^dim of the region tree (Section 3.1.1 Step 1) and its depth. */
vasmg_status vasmg_tree_info(vasmg_handle h, double* m, double* M, int32_t* max_depth);

/* Wall-clock milliseconds of the setup phases, in the order they ran (names
 * such as "validate+assemble", "tree", "P0", "coarse regions+P" for the host
 * tree and prolongations, "tree+P (device)" when setup_device = 1 built them
 * on the device, "galerkin" — "galerkin (+ordering)" when the device products
 * run beside the host's cells and colours —, "cells+colours", "coarsest factor", then
 * unless host_only "upload: layouts" (the level layouts and transfers),
 * "upload: autotune" (autotune = 1) and "upload: graphs" (capture and
 * instantiation of the solve's graphs); host wall time until each part
 * returned, so device work still queued counts in the next). Writes up to
 * max_out entries (name NUL-terminated, truncated to 31 characters) and the
 * number of phases to *n_out. */
typedef struct {
  char name[32];
  double ms;
} vasmg_setup_phase;
vasmg_status vasmg_setup_phases(vasmg_handle h, vasmg_setup_phase* out, int32_t max_out,
                                int32_t* n_out);

/* ---------------------------------------------------------------------------
 * Single-step device entry points (FP64 in/out, device pointers, canonical
 * level order). precision selects the level copy used: VASMG_FP64 or
 * VASMG_FP32_PRECOND (the FP32 copy exists only if the handle was set up with
 * VASMG_FP32_PRECOND). Each returns after the work finished on stream.
 * ------------------------------------------------------------------------- */

/* y = A_level x (block CSR SpMV). */
vasmg_status vasmg_spmv_device(vasmg_handle h, int32_t level, int32_t precision,
                               const double* d_x, double* d_y, void* stream);

/* x <- one GS sweep on A_level x = b (forward = colours/vertices/components
 * ascending, backward = exact reverse; Section 2.1 Algorithm 1 in colour order). */
vasmg_status vasmg_gs_sweep_device(vasmg_handle h, int32_t level, int32_t precision,
                                   int32_t backward, const double* d_b, double* d_x,
                                   void* stream);

/* b_{level+1} = P_level^T r_level (restriction, Section 3 Step 2.2). */
vasmg_status vasmg_restrict_device(vasmg_handle h, int32_t level, int32_t precision,
                                   const double* d_r, double* d_bc, void* stream);

/* x_level += P_level e_{level+1} (prolongation, Section 3 Step 2.4). */
vasmg_status vasmg_prolong_device(vasmg_handle h, int32_t level, int32_t precision,
                                  const double* d_e, double* d_x, void* stream);

/* z = B r: one V-cycle (Algorithm 3, recursive) on the fine level, using the
 * handle's precision. r, z: [n_free_vertices][dim] FP64, canonical order. */
vasmg_status vasmg_apply_precond_device(vasmg_handle h, const double* d_r, double* d_z,
                                        void* stream);

/* Test-only: caps the columns one symbolic pass of the device Galerkin product
 * covers (its LDS bitmap window; 0 = the maximum, 65,536), so that small meshes
 * reach the multi-pass path. Process-wide, read by setups that start afterwards.
 * EINVAL if cols < 0. */
vasmg_status vasmg_set_galerkin_window(int32_t cols);

/* ---------------------------------------------------------------------------
 * Measurement. One PCG iteration's device work (fine FP64 SpMV q = A p of
 * Algorithm 2, the PCG vector updates, and one V-cycle of Algorithm 3) is
 * replayed reps times outside the captured graphs with hipEvents around each
 * phase; phases are aggregated by (name, level). names: spmv_f64, pcg_vectors,
 * gs_fwd_zero, gs_fwd, residual, residual_full, restrict, coarse_solve,
 * prolong, gs_bwd. bytes is the algorithmic HBM traffic of the phase (every
 * matrix/vector array it touches read or written once per launch, the gathered
 * neighbour vector once per launch). Uses the handle's work buffers (their
 * contents are overwritten); level -1 = PCG vectors.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[32];
  int32_t level;
  int32_t launches;
  double ms;
  double bytes;
} vasmg_phase_stat;

vasmg_status vasmg_profile_iteration(vasmg_handle h, int32_t reps, void* stream,
                                     vasmg_phase_stat* out, int32_t max_out, int32_t* n_out);

#ifdef __cplusplus
}
#endif

#endif /* VASMG_H */
