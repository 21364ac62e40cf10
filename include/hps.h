/* hps.h -- C ABI of the MI355X HPS-as-multigrid Helmholtz solver.
 *
 * Problem (Sec. 2 of Lucero Lorca, "Towards a Multigrid Preconditioner
 * Interpretation of Hierarchical Poincare-Steklov Solvers"):
 *     -Lap u - kappa^2 (1 - b(x)) u = s   in (0,1)^2,
 *     d_n u + i eta u = t                 on the boundary.
 * Discretisation (Sec. 3): n x n square elements (or nx x ny, hps_desc.ny), tensor GLL grid of order N per
 * element, corner nodes removed; leaf impedance-to-impedance maps T and loads H
 * (eq. ItIOperator); skeleton system M g = RHS on the interior incoming
 * impedances (Sec. 3.2).  Solver (Sec. 4): nested-dissection merge tree whose
 * level-l Schur complements M_{l+1} = D_l - C_l A_l^-1 B_l are the merged box
 * maps; applied as the multigrid preconditioner MG(M) = F + P S^-1 R (I - M F)
 * inside flexible GMRES, with the top coarse solve either exact or a fixed
 * number of unpreconditioned GMRES iterations (Sec. 4.3).
 *
 * Conventions shared by every entry point:
 *  - Complex numbers are interleaved (re, im) doubles.
 *  - Elements e = ix + n*iy (n elements along x); element nodes (i, j) (i along
 *    x), flat index i*(N+1) + j, x_i = ix*h + (1 + xi_i) h/2 with GLL nodes xi
 *    on [-1, 1] and h = 1/n (1/max(nx, ny) on a rectangular mesh).
 *  - Canonical skeleton layout ("canonical vector"): slot (e, side, k) at flat
 *    index (e*4 + side)*(N-1) + k, sides l=0, r=1, b=2, t=3, k = 0..N-2 by
 *    increasing coordinate; length E*4*(N-1) complex.  A slot holds the
 *    incoming impedance (d_n + i eta) u of element e on that side.  Slots on
 *    the physical boundary are not unknowns: they are ignored on input and
 *    written as 0 on output.  Row s of M lives at the slot of the unknown it
 *    determines: (M g)[s] = g[s] - (T g)[Pi(s)], Pi(s) the slot across the
 *    face, so M = I - Pi T_blk (the rows of eq. faceequations).
 *  - Merge level l = 1 .. L_max = log2(n^2); level-l boxes are
 *    2^floor(l/2) x 2^floor((l-1)/2) elements; merge l pairs boxes along x for
 *    odd l and along y for even l (Fig. 1).  On an nx x ny mesh (L_max =
 *    log2(nx ny)) the merges alternate so while both directions have merges
 *    left and then run along the longer direction.
 *
 * Memory: the caller owns all device memory.  Each problem lives in ONE
 * caller-provided device workspace of hps_workspace_bytes() bytes; the library
 * allocates no device memory at all.  Array arguments are DEVICE pointers
 * unless marked [host].  All calls are asynchronous on the context's stream
 * unless marked "synchronises"; inputs may be freed once that stream has passed
 * the call.  A context is bound to one stream and is not thread-safe.
 *
 * Errors: every call returns hps_status; no exception crosses the ABI.  After a
 * failure hps_last_error(ctx) describes it.  Argument checks happen on the
 * host.  Failures found on the device are recorded in the problem's workspace
 * and reported at the next synchronising call (hps_gmres_solve, which checks
 * before its first iteration and at exit, and hps_sync): an exact zero pivot
 * in a leaf or merge factorisation as HPS_ERR_SINGULAR, its message naming the
 * problem and the element (leaf) or the merge level and pair of the first one;
 * a NaN or Inf in b_nodes or s_nodes as HPS_ERR_ARG, naming the problem and
 * element (that element's leaf map is not built).  Leaf elements close to an
 * interior Dirichlet resonance (a nearly singular interior block: its smallest
 * pivot below 0.02 of its largest) are recomputed from the complex element
 * system of Sec. 3.1 by partial-pivoting LU, so they keep full accuracy.
 */
#ifndef HPS_H
#define HPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hps_ctx hps_ctx;
typedef struct hps_problem hps_problem;

typedef enum {
  HPS_OK = 0,
  HPS_NOT_CONVERGED = 1,  /* warning: maxit reached, best iterate returned      */
  HPS_ERR_ARG = -1,       /* invalid argument (sizes, NaN/Inf, null pointers)   */
  HPS_ERR_OOM = -2,       /* workspace smaller than hps_workspace_bytes()       */
  HPS_ERR_SINGULAR = -3,  /* exact zero pivot in a leaf or merge factorisation  */
  HPS_ERR_STATE = -4,     /* call out of order (e.g. merge before build)        */
  HPS_ERR_HIP = -5        /* HIP runtime error                                  */
} hps_status;

typedef enum { HPS_FP64 = 0, HPS_MIXED = 1 } hps_precision;

/* Problem descriptor.  Defaults in brackets.
   Precision HPS_MIXED: the leaf maps are computed in FP64 (they define the outer
   operator M_1, which must stay FP64 for the outer iteration to refine toward
   the FP64 solution) and copied to FP32; merges 1..L-3 and the V-cycle on those
   levels run in complex FP32 (FP32 MFMA, FP64 vectors); merges L-2 and L-1,
   the coarse solve, Arnoldi and all residuals run in FP64. */
typedef struct {
  int32_t n;             /* elements along x (per side of a square mesh), a
                            power of two, 1 <= n <= 1024 (ny below)           */
  int32_t order;         /* GLL order N, 2 <= N <= 16                          */
  double kappa;          /* wavenumber kappa > 0 (c = kappa^2 (1 - b))         */
  double eta;            /* impedance parameter eta > 0 (the paper: eta=kappa) */
  int32_t precision;     /* hps_precision [HPS_FP64]                           */
  int32_t levels;        /* coarse level L, 1 <= L <= L_max; 0 => L_max         */
  int32_t coarse_iters;  /* k >= 1 GMRES steps on M_L; -1 => exact coarse solve
                            (requires L = L_max: direct HPS)                   */
  int32_t gamma;         /* coarse calls per level, 1..4 (0 => 1) [1]: 1 is the
                            V-cycle; gamma > 1 the gamma-cycle of Sec. 4.3, the
                            coarse correction of every level being gamma
                            stationary steps y += MG_{l+1}(r - M_{l+1} y) from
                            y = 0 (MG_{l+1} is called gamma^(l-1) times per
                            application at level l)                           */
  int32_t restart;       /* FGMRES restart length, 1..200 [60]                 */
  int32_t ny;            /* elements along y, a power of two in [1, 1024];
                            0 => n (a square mesh).  An nx x ny mesh (nx = n,
                            nx ny >= 2) takes square elements of side
                            h = 1/max(nx, ny) on (0, nx h) x (0, ny h), element
                            e = ix + nx iy; merges alternate x, y while both
                            directions have merges left, then run along the
                            longer one (L_max = log2(nx ny))                   */
} hps_desc;

/* Per-problem result of hps_gmres_solve ([host]).  Times are device times
   from HIP events on the context's stream; a group's problems share theirs. */
typedef struct {
  int32_t status;        /* HPS_OK or HPS_NOT_CONVERGED                        */
  int32_t iterations;    /* flexible GMRES iterations, counted across restarts */
  double relres_est;     /* Givens estimate of ||RHS - M g|| / ||RHS||          */
  double relres_true;    /* recomputed ||RHS - M g||_2 / ||RHS||_2 at exit      */
  double t_build_s;      /* leaf build through the latest merge level (s)      */
  double t_solve_s;      /* this call's flexible GMRES (s)                      */
} hps_info;

/* View of one level's stored operators (for inspection and testing). */
typedef struct {
  int32_t level;         /* l                                                  */
  int32_t boxes;         /* number of level-l boxes                            */
  int32_t box_nodes;     /* b = box perimeter in nodes (box map is b x b)      */
  int32_t morton;        /* 1: boxes stored in merge-tree order: box index j
                            covers the elements whose tree code shifted right
                            by l-1 equals j; bit l-1 of the code is the bit of
                            the element's x or y index that merge l consumes
                            (on a square mesh the Morton code: x bits even,
                            y bits odd)                                         */
  const void* T;         /* complex [boxes][b][b], column-major, box-local
                            boundary order [l; r; b; t]; FP64                  */
  int32_t pairs;         /* pairs merged at this level (0 at the top)          */
  int32_t shared_nodes;  /* m = length of the shared face                      */
  /* Pair j merges boxes P = 2j and Q = 2j+1.  Its shared-face unknowns are
     x = [f^Q_beta; f^P_alpha] (2m) and its kept faces y = [P.E1; Q.E2] (2e,
     each child's sides in [l; r; b; t] order without the shared side).        */
  const void* Ainv;      /* complex [pairs][2m][2m] column-major: A^-1 with
                            A = [[I, -T^P_aa], [-T^Q_bb, I]] (the shared-face
                            block of the level's skeleton system)              */
  const void* X;         /* complex [pairs][2m][2e] column-major: A^-1 B with
                            B = blkdiag(T^P_{a,E1}, T^Q_{b,E2}); columns of y on
                            physical sides are 0.  NULL at the top.           */
  int32_t fp32;          /* 1: T, Ainv and X are complex FP32 (mixed precision,
                            levels 1 .. L-3; level 1 then shows the FP32 copy
                            used by the preconditioner); 0: complex FP64      */
} hps_level_view;

/* ---- context ------------------------------------------------------------ */
/* Bind a context to a HIP stream (hipStream_t; NULL = legacy default stream). */
hps_status hps_ctx_create(void* hip_stream, hps_ctx** out);
hps_status hps_ctx_destroy(hps_ctx* ctx);
/* Last error message of this context ("" if none); valid until the next call. */
const char* hps_last_error(const hps_ctx* ctx);
/* Wait for the context's stream and report the failures recorded on the
   device by any live problem of this context (see Errors above). */
hps_status hps_sync(hps_ctx* ctx);
/* Options.  HPS_OPT_GRAPHS (default 0): replay HIP graphs captured once per
   problem (on a private capture stream) instead of launching kernels one by
   one: in hps_gmres_solve, one graph per FGMRES iteration (V-cycle, M_1
   product, CGS2, next basis vector; the iteration index is held on the device,
   so the same graph serves every iteration), and in hps_precond_apply the
   V-cycle.  Results are bitwise identical either way.  The graphs read and
   write buffers of their own (two vector copies per application), so they pay
   only where the host cannot keep ahead of the GPU, e.g. several host threads
   launching on one device at once; a single solver loop launches eagerly fast
   enough.
   HPS_OPT_TIMING (default 0): profiling aid.  Setting it (either value)
   synchronises and discards earlier records; while it is 1, every launch of a
   timed kernel is bracketed by HIP events recorded on the context's stream (the
   stream the kernel runs on; never inside a captured graph).
   Returns HPS_ERR_ARG for an unknown option. */
enum { HPS_OPT_GRAPHS = 1, HPS_OPT_TIMING = 2 };
hps_status hps_set_option(hps_ctx* ctx, int32_t option, int32_t value);
/* Timed kernels and their work unit:
   HPS_KERNEL_LEAF: the leaf kernel of hps_build_leaves, one launch per chunk of
   up to 4096 elements (of at most 32 problems of a group); unit = one element
   (its ItI map T and load H).  The interval also covers the fallback launch
   of the elements near a resonance (none in most builds). */
enum { HPS_KERNEL_LEAF = 0 };
/* [host outputs] Launches, summed device time (ms, from the events) and units
   processed by `kernel` since HPS_OPT_TIMING was last set.  Synchronises. */
hps_status hps_kernel_time(hps_ctx* ctx, int32_t kernel, int64_t* launches, double* total_ms,
                           int64_t* units);

/* ---- sizing and host-side geometry -------------------------------------- */
/* Exact device workspace (bytes) of one problem; the admission footprint. */
hps_status hps_workspace_bytes(const hps_desc* desc, size_t* bytes);
/* Admission by footprint: the most levels L (the coarse system M_L, Sec. 4.3)
   whose workspace for `count` problems of this shape fits in `budget` bytes,
   written to *levels (desc->levels is ignored).  More levels mean fewer
   outer iterations and more memory (Table 1: PMem grows and It falls with
   #levels).  HPS_ERR_OOM if not even L = 1 fits (L = L_max only, for the
   exact coarse solve); host only. */
hps_status hps_choose_levels(const hps_desc* desc, int32_t count, size_t budget, int32_t* levels);
/* [host] GLL nodes on [-1, 1] of order N: xi[N+1], increasing. */
hps_status hps_gll_nodes(int32_t order, double* xi);
/* [host] physical coordinates of all element nodes, x[E][(N+1)^2], y[...]. */
hps_status hps_node_coords(const hps_desc* desc, double* x, double* y);
/* [host] coordinates and outward unit normals of every canonical slot,
   each array [E*4*(N-1)]. */
hps_status hps_slot_coords(const hps_desc* desc, double* x, double* y,
                           double* nx, double* ny);

/* ---- problems ----------------------------------------------------------- */
/* Carve a problem out of `workspace` (device, >= hps_workspace_bytes, 256-byte
   aligned).  Copies small index tables into the workspace; synchronises. */
hps_status hps_problem_create(hps_ctx* ctx, const hps_desc* desc, void* workspace,
                              size_t bytes, hps_problem** out);
/* Frees host metadata only; the caller frees the workspace. */
hps_status hps_problem_destroy(hps_problem* p);
hps_status hps_level_view_get(const hps_problem* p, int32_t level, hps_level_view* out);

/* ---- groups: cross-problem batching ------------------------------------- */
/* A group holds `count` problems of one shape -- equal n, order, levels,
   coarse_iters, restart and precision -- whose wavenumbers kappa[i] and
   impedance parameters eta[i] may differ (desc->kappa and desc->eta are
   ignored), as do their coefficients, sources and boundary data.  The group
   lives in one caller-provided workspace; every hot-path call runs each step
   for all of its problems in the same launches (the level-l boxes of all
   problems form one batch; the Krylov iterations run in lock step with
   per-problem scalars and stopping).  A group handle is passed to the hot-path
   calls like a problem handle: their per-problem arrays (b_nodes, s_nodes, t,
   rhs, g, r, z, info) list the problems of all handles in order, so a group
   of `count` problems consumes `count` consecutive entries.
   1 <= count <= 4096.  Results equal those of the problems solved one by one
   up to rounding (summation order of split reductions). */
hps_status hps_group_workspace_bytes(const hps_desc* desc, int32_t count, size_t* bytes);
hps_status hps_group_create(hps_ctx* ctx, const hps_desc* desc, int32_t count, const double* kappa,
                            const double* eta, void* workspace, size_t bytes, hps_problem** out);
/* Number of problems behind a handle (1 for hps_problem_create). */
int32_t hps_group_size(const hps_problem* p);
/* Level view of problem `member` (0-based) of a group; hps_level_view_get is
   member 0. */
hps_status hps_member_level_view(const hps_problem* p, int32_t member, int32_t level, hps_level_view* out);

/* ---- the hot path (batch-first: `count` handles per call; per-problem arrays
   hold one entry per problem behind the handles, see groups above) ---------- */
/* Leaf ItI maps T and loads H of every element (Sec. 3.1, eq. ItIOperator).
   b_nodes[i]: real [E][(N+1)^2], the coefficient b at the element nodes.
   s_nodes[i]: complex [E][(N+1)^2] source s at the nodes, or NULL (H = 0). */
hps_status hps_build_leaves(hps_problem* const* p, int32_t count,
                            const double* const* b_nodes, const double* const* s_nodes);
/* Merge level `level` (Sec. 4.1-4.2): for 1 <= level < L, merge the level-l
   box pairs into level-(l+1) box maps, keeping W^-1 for the preconditioner.
   level == L (exact coarse mode only, L = L_max): factor the coarse system. */
hps_status hps_merge_level(hps_problem* const* p, int32_t count, int32_t level);
/* Skeleton right-hand side (Sec. 3.2): RHS[s] = (H + T_{.,phys} t)[Pi(s)].
   t[i]: complex canonical vector of incoming data; only physical slots read.
   rhs[i]: complex canonical vector (output). */
hps_status hps_set_rhs(hps_problem* const* p, int32_t count,
                       const double* const* t, double* const* rhs);
/* out = M_level g (canonical vectors; only level-`level` unknowns are read and
   written; level 1 also writes 0 at physical slots).  On the FP32 levels of
   mixed precision the FP32 box maps are applied in FP64 arithmetic. */
hps_status hps_skeleton_apply(hps_problem* const* p, int32_t count, int32_t level,
                              const double* const* g, double* const* out);
/* z = MG(M_1) r, one V-cycle (gamma = 1) or gamma-cycle with the configured
   coarse solve (Sec. 4.3).  r and z: complex canonical vectors; r is not
   modified. */
hps_status hps_precond_apply(hps_problem* const* p, int32_t count,
                             const double* const* r, double* const* z);
/* Field recovery (Sec. 3.1): with the skeleton solution g known, each
   element's incoming impedances f are known on all four sides (g on interior
   sides, the boundary data t on physical sides), and its nodal field solves
   the element system L u = [bt on the interior nodes; f on the side nodes]
   (complex LU with partial pivoting per element).  The four corner nodes
   carry no unknown (Sec. 3.1 removes them); each corner value is the mean of
   the two extrapolations, along the two sides meeting there, of the
   degree-(N-2) polynomial through the side's N-1 nodal values (a reading: the
   paper leaves corners unspecified).
   b_nodes, s_nodes (NULL: no source): as for hps_build_leaves; t, g: complex
   canonical vectors; u[i]: complex [E][(N+1)^2] output, flat node index
   i*(N+1)+j.  Requires hps_build_leaves; uses the workspace's scratch (no
   other state is changed).  Zero pivots: HPS_ERR_SINGULAR at the next
   synchronising call. */
hps_status hps_recover_field(hps_problem* const* p, int32_t count, const double* const* b_nodes,
                             const double* const* s_nodes, const double* const* t, const double* const* g,
                             double* const* u);
/* Flexible GMRES(restart) on M_1 g = rhs, right-preconditioned by MG, x0 = 0,
   until ||rhs - M_1 g|| <= tol ||rhs|| or maxit iterations (Sec. 4.3, Sec. 5).
   g: complex canonical output.  info[count] ([host]) receives per-problem
   results.  Synchronises.  Returns HPS_NOT_CONVERGED if any problem did not
   converge. */
hps_status hps_gmres_solve(hps_problem* const* p, int32_t count,
                           const double* const* rhs, double* const* g,
                           double tol, int32_t maxit, hps_info* info);

/* ---- leaf maps without device allocation --------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the leaf
   ItI maps T and loads H of `count` elements of side h (Sec. 3.1, eq.
   ItIOperator; the same kernels as hps_build_leaves), with every buffer the
   kernels need beyond the inputs and outputs -- error words, the fallback
   list, GLL tables, per-element scratch -- in one 64 MiB file-scope device
   array that each GPU the library runs on holds until the process ends.  No
   hipMalloc, hipFree or allocating library call is made.
   b_nodes: real [count][(N+1)^2] (the coefficient b at the element nodes,
   flat index i*(N+1)+j); s_nodes: complex [count][(N+1)^2] or NULL (H = 0);
   T: complex [count][4(N-1)][4(N-1)] column-major, element after element (no
   Morton placement); H: complex [count][4(N-1)].  All device pointers, on
   the context's stream; synchronises.  count is limited by the array: at most
   102 elements at N = 16, 304 at N = 12, 1372 at N = 8, 4096 for N <= 5
   (HPS_ERR_ARG beyond, its message giving the limit).  Errors as for
   hps_build_leaves (HPS_ERR_ARG for a NaN or Inf input, HPS_ERR_SINGULAR),
   naming the element.  Every call on a GPU shares that GPU's array: calls
   that overlap on one GPU (several streams or host threads) race and must be
   serialised by the caller. */
hps_status hps_leaf_maps_noalloc(hps_ctx* ctx, int32_t order, double h, double kappa, double eta,
                                 int32_t count, const double* b_nodes, const double* s_nodes,
                                 double* T, double* H);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H */
