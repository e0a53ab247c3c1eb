/*
 * mrb.h -- C ABI of the MI355X block-multiresolution solver (arXiv 1902.00088).
 *
 * The library advances an evolutionary PDE  d(phi)/dt = N(phi)  (Sec. 2, first
 * paragraph) on a graded, periodic quad/octree forest of blocks (Sec. 2.2),
 * following the multiresolution step of Sec. 2.1: refine every block by one
 * level (safety zone), synchronise ghost nodes and evolve with 4th-order central
 * finite differences and classic RK4 (Sec. 3, Sec. 4), then coarsen blocks whose
 * details fall below eps (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - Blocks.  A block at level l (1 = coarsest .. jmax) with integer coordinates
 *    c in [0, 2^l)^dim covers the level-l node indices c*(bs-1) + i, i = 0..bs-1,
 *    of a periodic unit domain with N_l = 2^l*(bs-1) unique nodes per direction
 *    (block definition, Sec. 2.2; the printed index range "0..B_s" is read as
 *    0..B_s-1).  Node data of one block is [field][k][j][i], i fastest.
 *  - Forest order.  Every array that lists blocks ("forest order") is sorted by
 *    the Morton key of (coords << (jmax - level)) with x as the least significant
 *    bit (the space-filling-curve order of Sec. 2.5).  It does not depend on
 *    pool slots.
 *  - Ownership.  The caller owns every buffer passed in: the device pool arrays
 *    given to mrb_create and all host or device arrays of later calls.  The
 *    library never frees them.  It allocates only its own descriptor, staging
 *    and scratch memory, released by mrb_destroy.
 *  - Errors.  Every call returns an mrb_status; none aborts or throws across the
 *    ABI.  On error the solver state is unchanged (capacity and topology are
 *    checked before any device write) and mrb_last_error() describes the cause.
 *    The one exception is a grid-barrier time-out of the one-launch sweep (see
 *    mrb_set_sweep), which voids the block data.
 *  - Streams.  All device work is enqueued on the HIP stream given to mrb_create.
 *    Calls that return host data (mrb_num_blocks, mrb_read_*, mrb_get_flags,
 *    mrb_mr_pass, mrb_adapt, mrb_step) synchronise that stream before returning.
 *  - A context is not thread safe; use one per host thread.
 */
#ifndef MRB_H_
#define MRB_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrb_ctx mrb_ctx;

typedef enum {
  MRB_OK = 0,
  MRB_E_ARG = -1,        /* invalid argument or unsupported configuration            */
  MRB_E_CAPACITY = -2,   /* pool (max_blocks) too small for the requested topology   */
  MRB_E_TOPOLOGY = -3,   /* forest does not tile the domain, overlaps or is not graded */
  MRB_E_STATE = -4,      /* call out of order (e.g. step before init_forest)         */
  MRB_E_DEVICE = -5,     /* a HIP runtime call failed                                */
  MRB_E_NONFINITE = -6   /* a detail norm was NaN or Inf                              */
} mrb_status;

/* physics: right-hand side N(phi) */
enum {
  MRB_ADV_CONST = 0,  /* -c.grad(phi), phys[0..2] = c                                   (Sec. 3 eq. form) */
  MRB_ADV_SWIRL = 1,  /* -u(x,y,t).grad(phi), the swirl field of Sec. 3; phys[0] = t_a (0 = steady)      */
  MRB_NS2D = 2        /* compressible Navier-Stokes, fields rho,u,v,p; phys = {gamma, mu, Pr, r_th} (Sec. 4);
                         r_th > 0 applies the shock-capturing filter after every RK4 step (Sec. 4: a
                         pressure sensor max(0, 1 - r_th/r), r = M/p^2 + 1e-16 with M the squared
                         differences of Dp = (-p_{j+1} + 2p_j - p_{j-1})/4, switching a second-order
                         filter in flux form, F = -(q_{j+1} - q_j)/4, on every field, per axis); the
                         paper's filter reference is not available, this formulation is ours */
};
enum { MRB_FP64 = 0, MRB_MIXED = 1 };          /* MIXED: FP32 stencil + FP32 slopes, FP64 state     */
enum { MRB_FORM_PLAIN = 0, MRB_FORM_FUSED = 1 };/* PLAIN: stored ghosts, per-level launches           */

typedef struct {
  int dim;             /* 2 or 3                                                            */
  int bs;              /* points per block and direction: 17 or 33 in 2D, 17 in 3D          */
  int hw;              /* ghost width of the RHS stencil: 2 (advection) or 4 (NS)            */
  int nfields;         /* 1 (advection) or 4 (NS)                                            */
  int jmax;            /* finest level, 2..12                                                */
  int max_blocks;      /* pool capacity in blocks (N_max of Sec. 2.4); max_blocks * nfields *
                          bs^dim must stay below 2^31 (32-bit offsets in the kernels)      */
  double eps;          /* detail threshold (Sec. 2.3)                                        */
  int physics;         /* MRB_ADV_CONST / MRB_ADV_SWIRL / MRB_NS2D                           */
  double phys[8];      /* see physics                                                        */
  const double *swirl_s2;   /* host, 2^jmax*(bs-1) values sin^2(pi x_i), x_i = i/N_jmax (swirl only; copied) */
  const double *swirl_s;    /* host, same length, sin(2 pi x_i)                                               */
  const double *field_scale;  /* host, nfields values or NULL: field f coarsens if max|d_f| < eps*scale[f] */
  const double *field_offset; /* host, nfields values or NULL: MIXED stages work on (y - offset[f]) in FP32 */
  int precision;       /* MRB_FP64 or MRB_MIXED                                              */
  int form;            /* MRB_FORM_PLAIN or MRB_FORM_FUSED                                    */
} mrb_config;

/* Create a solver.  u, u_new: device double arrays of max_blocks*nfields*bs^dim
 * elements; k1..k3: device arrays of the same element count, double (FP64) or
 * float (MIXED).  stream: a hipStream_t (NULL = default stream).  The arrays
 * must stay valid until mrb_destroy.  Sec. 2.4 (heavy data preallocated to N_max). */
mrb_status mrb_create(const mrb_config *cfg, double *u, double *u_new, void *k1, void *k2, void *k3,
                      void *stream, mrb_ctx **out);
mrb_status mrb_destroy(mrb_ctx *ctx);
const char *mrb_last_error(const mrb_ctx *ctx);

/* Set the forest: n blocks, host arrays level[n], coords[n*dim] (any order).
 * Rejects forests that overlap, leave holes or are not graded (Sec. 2.2, graded
 * grid: touching blocks differ by at most one level, diagonals included).
 * Block data is undefined until mrb_load_blocks. */
mrb_status mrb_init_forest(mrb_ctx *ctx, int n, const int8_t *level, const int32_t *coords);

/* Copy block data [n][nfields][bs^dim] in forest order into the pool.  data is
 * host memory (on_device = 0) or device memory (on_device = 1).  Nodes shared by
 * blocks of the same level must hold equal values (Sec. 2.5). */
mrb_status mrb_load_blocks(mrb_ctx *ctx, const double *data, int on_device);

/* Safety zone (Sec. 2.1 item 1): every block below jmax becomes its 2^dim
 * children, whose nodes take the synchronised value at the finer level
 * (prediction P of Sec. 2.3 where the finer node is new). */
mrb_status mrb_refine_all(mrb_ctx *ctx);

/* One classic RK4 step of size dt from time t on the current grid (Sec. 2.1 item
 * 2): each stage synchronises ghost nodes (same-level copy, injection from finer
 * blocks, prediction from coarser ones) and evaluates the 4th-order FD RHS. */
mrb_status mrb_rk4(mrb_ctx *ctx, double t, double dt);

/* One multiresolution analysis (Sec. 2.3): synchronise the stored state, compute
 * details D = B - P(R(B)), and set flag -1 where max|d_f| < eps*scale[f] for every
 * field (0 otherwise, and always 0 at level 1).  flags[n] (int8) and maxd[n*nfields]
 * (double, may be NULL) receive the result in forest order (host arrays). */
mrb_status mrb_mr_pass(mrb_ctx *ctx, int8_t *flags, double *maxd);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): mrb_mr_pass without any device or
 * host allocation.  Same arguments and results as mrb_mr_pass (bitwise), computed with
 * sub-tiled analysis workgroups whose per-block partial maxima and completion counters
 * live in a static device array of the library (2 MiB per GPU, held until the process
 * ends; it needs n_blocks * (8 * nfields) + 4 * n_blocks bytes, rounded up, so at most
 * about 174,000 blocks with one field or 58,000 with four: MRB_E_CAPACITY beyond).  The
 * array is cleared by a fill kernel at each call.  Every context on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads) race.
 * MRB_E_DEVICE if the array's address could not be looked up when the context was made. */
mrb_status mrb_mr_pass_noalloc(mrb_ctx *ctx, int8_t *flags, double *maxd);

/* Coarsen with the given flags (host, forest order): families of 2^dim sister
 * blocks all flagged -1 merge into their mother when the result stays graded
 * (completeness + gradedness, Sec. 2.3 last paragraph; the largest such set).
 * The mother keeps every second node (restriction R).  *n_coarsened (may be
 * NULL) receives the number of merged families.  This is also the topology-replay
 * call ("apply flags"): given flags computed elsewhere (e.g. by an FP64 run of the
 * same step), it reproduces that run's coarsening on this context's data, which is
 * how the mixed-precision form is compared on the FP64 topology. */
mrb_status mrb_coarsen(mrb_ctx *ctx, const int8_t *flags, int *n_coarsened);

/* Repeat {mrb_mr_pass; mrb_coarsen} until no family merges (Sec. 2.1 item 3).
 * *n_passes (may be NULL) receives the number of analyses. */
mrb_status mrb_adapt(mrb_ctx *ctx, int *n_passes);

/* nsteps multiresolution time steps: {refine_all; rk4(t, dt); adapt}, t advancing by dt.
 * The results are those of that sequence; the schedule differs: on forests of at
 * most 1,024 leaves, topology changes seen before replay their memoised plans, and
 * the first coarsening of each adapt is speculated from the previous step (the
 * analysis pass writes the speculated mothers; if its flags differ, the host state
 * is put back and the adapt continues from the real flags). */
mrb_status mrb_step(mrb_ctx *ctx, double t0, double dt, int nsteps);

mrb_status mrb_num_blocks(mrb_ctx *ctx, int *n);
/* Forest in forest order: level[n], coords[n*dim] (host). */
mrb_status mrb_read_forest(mrb_ctx *ctx, int8_t *level, int32_t *coords);
/* Synchronised block values [n][nfields][bs^dim] in forest order (redundant nodes
 * carry the owner's value).  out is host (on_device = 0) or device memory. */
mrb_status mrb_read_blocks(mrb_ctx *ctx, double *out, int on_device);
/* The solution on the uniform lattice of `level` (periodic, N = 2^level (bs-1) nodes
 * per direction): out[nfields][N^dim], x fastest, host (on_device = 0) or device
 * memory of nfields * N^dim doubles; level = 1..jmax.  Node m takes the synchronised
 * value V(level, m): the stored value of the finest leaf holding it on its own lattice
 * (Sec. 2.2), or, inside a coarser leaf, the prediction of Sec. 2.3 from the next
 * coarser level, applied level by level (Sec. 4 takes spectra "after refining the mesh
 * to a fixed level").  Leaves coarser than `level` are refined for the read into free
 * pool slots and the forest is put back afterwards: the solver's state is unchanged.
 * MRB_E_CAPACITY if the pool lacks the free slots for that refinement; MRB_E_ARG for a
 * level outside 1..jmax. */
mrb_status mrb_read_uniform(mrb_ctx *ctx, int level, double *out, int on_device);
/* Last analysis: flags[n], maxd[n*nfields] in forest order (host; maxd may be NULL). */
mrb_status mrb_get_flags(mrb_ctx *ctx, int8_t *flags, double *maxd);
/* Counters and timings as one JSON object (NUL-terminated, at most cap bytes).
 * Synchronises the stream when kernel timing is on. */
mrb_status mrb_stats(mrb_ctx *ctx, char *json, int cap);
/* Kernel timing: when enable != 0, every sweep-kernel launch is bracketed by HIP
 * events on the solver's stream and mrb_stats reports the accumulated device
 * time and algorithmic bytes per kernel kind; enable = 0 stops and clears. */
mrb_status mrb_timing(mrb_ctx *ctx, int enable);
/* Block tilings (the autotuner).  nsub > 0 forces nsub sub-tiles per axis (one
 * workgroup each) for the fused stage sweep, and for the overlapped-tile RK4 step
 * (mrb_set_sweep mode 3) where that tiling is compiled; nsub = 0 with reps > 0 times reps dry
 * sweeps (four stages into k1..k3/u_new, the state u is not advanced) of every
 * compiled stage tiling, in forest (Morton) order and in level-sorted order, on the
 * current forest and keeps the fastest pair, then does the
 * same for the analysis kernel (one pass; flags are recomputed) and, if the last
 * refinement plan is still the uploaded one (right after mrb_refine_all), for the
 * refinement kernel (re-run on the same parents), and the analysis of whole blocks with
 * larger workgroups where compiled; on the chosen stage tiling it also
 * times the whole sweep as four launches against one launch with grid barriers, and,
 * if every leaf is on one level and the shape has the kernel, every tiling of the
 * overlapped-tile RK4 step against the stage launches (see mrb_set_sweep).  Every
 * candidate is timed over five rounds and its fastest round
 * counts.  nsub > 0 with reps < 0 also sets -reps threads per workgroup for the stage
 * sweep, for the analysis of whole blocks and for the tile step's folded forms (first
 * analysis, refinement, second analysis, then also on nsub sub-tiles), each where that
 * form is compiled; MRB_E_ARG if none is.  nsub = 0 with reps = 0 returns to the built-in choices.  *chosen (may
 * be NULL) receives the stage tiling in use.
 * Not a step of the method: a schedule choice. */
mrb_status mrb_tune(mrb_ctx *ctx, int nsub, int reps, double dt, int *chosen);
/* Graph replay in mrb_step: the refinement, the four RK stages and the first analysis
 * of a step are captured into a HIP graph and replayed.  The kernels take the
 * topology header (block counts, buffer offsets) as a launch argument and read
 * descriptors from device memory, so a graph is captured per header and replayed
 * whenever the same header recurs (the last four are kept).  Graph-captured sweeps
 * always use four stage launches.  enable: 0 off, 1 on, 2 automatic (default: the first steps alternate
 * between graph replay and direct launches, ten each, and the faster median step wall
 * time decides).  Used only for the fused form, with kernel timing off, a non-default
 * stream and a time-independent right-hand side.  Results are identical either way.
 * MRB_E_ARG for other values. */
mrb_status mrb_set_graph(mrb_ctx *ctx, int enable);
/* How the fused form launches the four stages of an RK4 step (every block of every
 * level in each launch).  mode 0: four launches, one per stage.  mode 1: one
 * cooperative launch (one workgroup per compute unit, each taking several blocks per
 * stage), with a grid-wide barrier between stages.  The barrier waits are bounded:
 * a wait that times out ends the kernel early, the next call that synchronises the
 * stream returns MRB_E_DEVICE, and the block data is then undefined (this is the one
 * exception to "on error the state is unchanged"): every later call that needs it
 * returns MRB_E_STATE until mrb_load_blocks (or mrb_init_forest) supplies new data.
 * mode 3: where every leaf is on one level (2D, one field, halo 2: the advection
 * shapes), one launch per RK4 step over overlapped tiles: a workgroup loads u over its
 * region plus four halo widths and computes all four stages in LDS (k1 on the region
 * plus three halo widths, k2 plus two, k3 plus one, k4 on the region), repeating at
 * the halo exactly the operations the neighbours perform at their own nodes; k1..k3
 * never reach HBM.  Other forests and shapes take four launches.  Tiling: the one
 * forced or tuned by mrb_tune, else whole blocks.  In mrb_step the same launch also
 * performs the first analysis pass of the step's adapt (its halo is then three points
 * wider, so that u_new is known where the details' prediction reads it), unless the
 * autotuner found an analysis launch after it faster; and where the forest before the
 * step is on one level below jmax, the safety-zone refinement as well (the tile is
 * built from the parents: the children's values at the children's level, the parent's
 * value or its prediction, never reach HBM), unless the autotuner found the
 * refinement launch faster; and where the adapt's coarsening is speculated and merges
 * every block, its second analysis pass too (each workgroup computes the details of
 * its share of the mother's nodes on a halo six points wider; the host takes the
 * maximum over the shares), so such a step is one launch.  Where such steps repeat
 * (the forest returns to the same blocks and slots after each), mrb_step with
 * nsteps > 1 queues each step's launch before reading the previous step's flags; a
 * step whose flags miss the speculation takes the queued one back (results are the
 * same either way; mrb_stats counts queued and taken-back steps).
 * mode 2 (default): the autotuner (mrb_tune with reps > 0) times these forms on the
 * tuned tiling and keeps the fastest; four launches until then.  Results are
 * identical in every mode.  MRB_E_ARG for other values; modes 1 and 3 on the plain
 * form are accepted and ignored (it has no fused stages).
 * Not a step of the method: a schedule choice. */
mrb_status mrb_set_sweep(mrb_ctx *ctx, int mode);

/* Where mrb_step plans the topology changes of a step: the safety-zone refinement,
 * the completeness and gradedness fixed point of each coarsening (Sec. 2.3, last
 * paragraph) and the neighbour entries of every new grid.  mode 0: on the host (plans of
 * forests of at most 1,024 leaves are memoised, see mrb_step).  mode 1: on the device,
 * by plan kernels (prefix sums over the forest order, a free-slot stack and a dense index
 * of every possible block of every level), so a step reads back only a few counts per
 * analysis pass.  mode 2 (default): on the device when the refined grid would exceed
 * 1,024 leaves, on the host below.  Results are identical in every mode (same forest,
 * same slots).  The device path needs the fused form and a dense index of at most 2^26
 * blocks over all levels (otherwise the host plans), and processes blocks in forest
 * order.  Entry points other than mrb_step, mrb_num_blocks, mrb_mr_pass_noalloc and the
 * settings bring the host forest up to date first (a copy of the descriptors and the
 * free list back from the device).  MRB_E_ARG for other values.
 * Not a step of the method: a schedule choice. */
mrb_status mrb_set_topology(mrb_ctx *ctx, int mode);

/* ---------------------------------------------------------------------------
 * Learned refinement predictor.  The paper's refinement flag admits "+1 for
 * refinement" from arbitrary indicators besides the detail test (Sec. 2.3, after the
 * flag rule); here a per-block MLP predicts which blocks the safety zone (Sec. 2.1
 * item 1) needs to refine, and the exact detail threshold still decides every
 * coarsening.  2D only.  Features: per field, the 8 x 8 averages of the synchronised
 * block over bins of (bs-1)/8 nodes (last node row/column unused), x-fastest bins,
 * fields outer (nin = 64 * nfields).  Network: nin -> 64 -> 64 -> 3, GELU, FP32;
 * parameters packed W1[nin][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3]
 * (row-major).  Classes: 0 refine, 1 keep, 2 coarsen.  All arrays are host memory.
 * --------------------------------------------------------------------------- */

/* Set the model: parameters (see layout), per-field normalisation mean[nf], std[nf]
 * applied to the features (x - mean)/std; resets the Adam state. */
mrb_status mrb_mlp_init(mrb_ctx *ctx, int nin, const float *params, const float *mean, const float *std);
mrb_status mrb_mlp_get_params(mrb_ctx *ctx, float *params);
/* Raw features of the current forest: feat[n][nin], forest order. */
mrb_status mrb_mlp_features(mrb_ctx *ctx, float *feat);
/* Logits for n given feature rows: logits[n][3]. */
mrb_status mrb_mlp_forward(mrb_ctx *ctx, const float *x, int n, float *logits);
/* Gradient of the class-weighted softmax cross-entropy (weights classw[3]; the loss
 * is divided by the sum of the weights of the labels y[n]) w.r.t. the parameters:
 * grads[n_params] (may be NULL), *loss (may be NULL). */
mrb_status mrb_mlp_grad(mrb_ctx *ctx, const float *x, const int8_t *y, const float *classw, int n,
                        float *grads, float *loss);
/* One epoch over the n samples in the given order: batches of `batch`, one Adam step
 * (lr, beta 0.9/0.999, eps 1e-8) per batch; *mean_loss (may be NULL) = mean batch loss. */
mrb_status mrb_mlp_train(mrb_ctx *ctx, const float *x, const int8_t *y, const float *classw, int n, int batch,
                         float lr, float *mean_loss);
/* Prediction on the current forest: pred[n] (class), prob[n] (its softmax probability, may be NULL). */
mrb_status mrb_mlp_predict(mrb_ctx *ctx, int8_t *pred, float *prob);
/* Refine the blocks with mask[i] != 0 (forest order) and every coarser neighbour that
 * must follow to keep the grid graded; children take the synchronised finer values
 * as in mrb_refine_all.  *n_refined (may be NULL) receives the number refined. */
mrb_status mrb_refine_marked(mrb_ctx *ctx, const int8_t *mask, int *n_refined);
/* One predictor-guided MR step: refine the blocks predicted 'refine', those predicted
 * with probability < tau, and, when guard > 0, every block whose detail maximum from
 * the last analysis (Sec. 2.3) reaches guard x eps x field_scale for some field (all
 * blocks if the current grid has not been analysed); close under gradedness; RK4;
 * adapt by the exact detail threshold.  guard <= 0 leaves the choice to the
 * predictor alone. */
mrb_status mrb_step_predicted(mrb_ctx *ctx, double t, double dt, float tau, float guard, int *n_refined);
/* Training labels at a horizon (no context): block i of the grid "now" is 0 (refine)
 * if a finer block of the later grid overlaps it, 2 (coarsen) if it lies inside a
 * coarser block of the later grid, else 1 (keep). */
mrb_status mrb_horizon_labels(int dim, int n_now, const int8_t *lv_now, const int32_t *co_now, int n_later,
                              const int8_t *lv_later, const int32_t *co_later, int8_t *labels);

#ifdef __cplusplus
}
#endif
#endif /* MRB_H_ */
