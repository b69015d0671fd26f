/*
 * picbal.h -- C ABI of libpicbal.so, an MI355X (gfx950) implementation of the
 * per-box particle-in-cell step with in-situ device-side work assessment for
 * dynamic load balancing, after Rowan et al., "In-Situ Assessment of
 * Device-Side Compute Work for Dynamic Load Balancing in a GPU-Accelerated
 * PIC Code" (arXiv 2104.11385).
 *
 * What the paper defines and this library follows:
 *   - boxes (rectilinear sub-domains) and a distribution mapping that assigns
 *     each box to a rank (Sec. 2.1, Fig. 1);
 *   - per-box costs from a heuristic (weighted sum of particles and cells) or
 *     from a device clock read inside the compute-intensive kernel, summed in
 *     on-chip memory before one global atomic add (Sec. 2.2, Fig. 2a);
 *   - the load-balance efficiency E = c_avg / c_max (Eq. 1), the knapsack and
 *     Morton space-filling-curve policies, and the adopt-if-improved
 *     threshold (Sec. 2.2, Sec. 3.2, Sec. 3.3).
 * The PIC step itself (explicit Maxwell steps, Lorentz-force push, current
 * deposition, Sec. 2.1) follows Yee (1966), Boris (1970) and Esirkepov (2001)
 * with B-spline shapes of order 1, 2 or 3.
 *
 * Conventions used by every call:
 *   - Units: c = eps0 = mu0 = 1; cell size 1; time in cell/c.
 *   - Field arrays exchanged with the host are double, [nz][ny][nx] with x
 *     fastest.  Components 0..8 = Ex Ey Ez Bx By Bz Jx Jy Jz at Yee locations
 *     Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2) Bx(i,j+1/2,k+1/2)
 *     By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k); J co-located with E.
 *   - Positions exchanged with the host are double global coordinates in
 *     [0, n_d), [n][3]; momenta u = gamma v / c, [n][3].
 *   - Every pointer argument is a host pointer owned by the caller, unless
 *     stated otherwise.  The library owns pic_ctx and all device memory.
 *   - Calls that return data synchronise the context's stream first.
 *   - Status: 0 = PIC_OK, negative = error.  PIC_EINVAL leaves the context
 *     unchanged.  PIC_EDEVICE (a HIP runtime error) is sticky: the context is
 *     poisoned and only pic_finalize may follow.
 */
#ifndef PICBAL_H
#define PICBAL_H

#include <stdint.h>

#ifdef __cplusplus
#define PIC_API extern "C" __attribute__((visibility("default")))
#else
#define PIC_API __attribute__((visibility("default")))
#endif

typedef struct pic_ctx pic_ctx;

enum pic_status {
    PIC_OK = 0,
    PIC_EINVAL = -1,       /* bad sizes or arguments; context unchanged           */
    PIC_ENOMEM = -2,       /* device or host allocation failed                    */
    PIC_EDEVICE = -3,      /* HIP runtime error; sticky                           */
    PIC_ECFL = -4,         /* dt >= 1/sqrt(3): Yee scheme unstable in 3D          */
    PIC_ECAPACITY = -5,    /* more particles than the context was sized for       */
    PIC_ESTATE = -6,       /* call not valid in the current state                 */
    PIC_EUNSUPPORTED = -7  /* valid request this library does not implement       */
};

enum { PIC_FP32 = 4, PIC_FP64 = 8 };

/* Cost strategies (Sec. 2.2).  HEURISTIC: w_p * particles + w_c * cells per
 * box.  DEVICE_TIMER: wave-summed shader-clock cycles of the gather-push-
 * deposit work of each box since the last reset.  DEVICE_RTC: the same with
 * the constant-rate real-time counter.  LEARNED: the MLP's prediction of
 * DEVICE_TIMER from box features, with the heuristic as fallback. */
enum { PIC_COST_HEURISTIC = 0, PIC_COST_DEVICE_TIMER = 1, PIC_COST_DEVICE_RTC = 2, PIC_COST_LEARNED = 3 };

/* Distribution policies (Sec. 2.2). */
enum { LB_SFC = 0, LB_KNAPSACK = 1 };

/* Launch modes of the gather-push-deposit kernel.  PER_BOX: one launch per
 * (box, species), as a per-box framework issues them.  BATCHED: one launch
 * over every tile of every box.  PERSISTENT: one resident grid that pulls
 * work items (tile chunks, largest first) from a device queue. */
enum { PIC_LAUNCH_PER_BOX = 0, PIC_LAUNCH_BATCHED = 1, PIC_LAUNCH_PERSISTENT = 2 };

/* A box: half-open cell ranges [lo, hi).  The boxes must tile the domain
 * exactly (no overlap, no gap). */
typedef struct {
    int32_t lo[3], hi[3];
} pic_box;

typedef struct {
    int32_t n_cells[3];    /* domain size; periodic in every dimension;
                              n_cells[0], n_cells[1] <= 2048, n_cells[2] <= 1024 */
    double dt;             /* time step in cell/c; must satisfy dt < 1/sqrt(3)  */
    int32_t shape_order;   /* 1 (linear), 2 (quadratic) or 3 (cubic) B-splines  */
    int32_t precision;     /* PIC_FP32 or PIC_FP64 for particles and fields     */
    uint64_t seed;         /* Philox4x32-10 seed of the on-device loader        */
    double w_particle;     /* heuristic weights; the paper's 0.75 / 0.25        */
    double w_cell;
    double b_ext[3];       /* uniform initial magnetic field                    */
} pic_grid_desc;

typedef struct {
    double charge, mass;   /* normalised (electron: -1, 1)                      */
    double density;        /* macro-particle weight w = density / ppc           */
    int32_t load_mode;     /* 0: none (use pic_set_particles); 1: ppc particles
                              in every cell of [region_lo, region_hi); 2: box_ppc
                              particles in every cell of box b                  */
    int32_t ppc;
    const int32_t *box_ppc;    /* [n_boxes], load_mode 2 only; copied by pic_init */
    int32_t region_lo[3], region_hi[3];
    double u_th[3];        /* Gaussian spread of u per component                */
    double u_drift[3];     /* added to u                                        */
    int64_t capacity;      /* most particles this species may hold (for
                              pic_set_particles); 0 = the loaded count         */
} pic_species_desc;

/* Kernel tuning.  Tile edges must be one of the compiled shapes (8x8x8,
 * 8x8x4, 8x4x4, 4x4x4) and divide every box edge; halo is the number of
 * cells a particle may drift outside its tile between sorts and still use the
 * staged fields (particles beyond it take a slower global-memory path).
 * pic_init's default: 8x4x4 tiles, block 512, blocks_per_cu 2 where that
 * tile divides every box edge, two such blocks' LDS fit a CU and the
 * kernel's registers leave room for four waves per SIMD (the FP32 kernels of
 * shape orders 1 and 2); else the first of 8x4x4, 4x4x4, 8x8x4, 8x8x8 that
 * divides every box edge and whose LDS windows let three 256-thread blocks
 * share a CU (else two, else one), block 256, blocks_per_cu = the number of
 * blocks whose LDS fits on a CU (1..4); chunk 4096, sort_interval 20,
 * run_sum 1, field_overlap 1. */
typedef struct {
    int32_t tile[3];
    int32_t halo;          /* 1 */
    int32_t block;         /* threads per block: 256, 384 or 512               */
    int32_t chunk;         /* max particles per work item (PERSISTENT mode)    */
    int32_t sort_interval; /* steps between particle sorts (>= 1)              */
    int32_t blocks_per_cu; /* resident blocks per CU for PERSISTENT mode      */
    int32_t run_sum;       /* 1: particles of a tile are sorted node by node
                              and the currents of neighbouring particles that
                              keep a common reference node are summed across
                              lanes before one LDS add per run; 0: particles
                              are interleaved over nodes (one particle per
                              node and rank) and each adds its own current.
                              Results agree to rounding either way.          */
    int32_t field_overlap; /* 1: the Yee update of the z-planes that no
                              deposit of the step can reach (no current in
                              the previous step within two planes) runs on a
                              second stream beside the particle kernel, the
                              rest after it; 0: the whole update after it.
                              The arithmetic is the same either way.         */
} pic_tuning;

/* ---- lifecycle -------------------------------------------------------- */

/* Creates a context on the current HIP device: checks the grid (PIC_ECFL if
 * dt >= 1/sqrt(3); PIC_EINVAL for bad sizes or boxes that do not tile the
 * domain), allocates fields and particles in device memory, loads particles
 * with the on-device Philox loader (the recipe is documented with the Python
 * input generator), sets B = b_ext, E = J = 0, and sorts particles by tile.
 * hip_stream: a hipStream_t to run on, or NULL for a stream the library
 * creates.  species[s].box_ppc is copied.  On success *out owns the context. */
PIC_API int pic_init(const pic_grid_desc *grid, const pic_box *boxes, int32_t n_boxes,
                     const pic_species_desc *species, int32_t n_species, void *hip_stream,
                     pic_ctx **out);

/* Releases all device and host memory of the context. ctx may be NULL. */
PIC_API void pic_finalize(pic_ctx *ctx);

/* ---- the PIC step (Sec. 2.1; per-box costs Sec. 2.2) ----------------- */

/* Advances n_steps explicit steps.  Per step: gather E^n, B^n at x^n,
 * relativistic Boris push to u^{n+1/2}, move, Esirkepov current deposition
 * J^{n+1/2}, periodic wrap, then the Yee update (B half step, E full step
 * with -J, B half step).  Particles are re-sorted by tile every
 * sort_interval steps.  Device-timer costs accumulate per box.  Asynchronous
 * on the context's stream (with field_overlap, part of the field update runs
 * on a second stream of the library's, joined back into the context's stream
 * within the step).  n_steps < 0 -> PIC_EINVAL. */
PIC_API int pic_step(pic_ctx *ctx, int32_t n_steps);

/* Waits for all work queued on the context's stream. */
PIC_API int pic_sync(pic_ctx *ctx);

/* Selects the launch mode (PIC_LAUNCH_*) and whether each step is replayed
 * from a captured hipGraph (use_graph != 0). */
PIC_API int pic_set_launch_mode(pic_ctx *ctx, int32_t mode, int32_t use_graph);

/* Reads / replaces the kernel tuning.  pic_set_tuning re-sorts particles and
 * rebuilds the work queue; unsupported tiles -> PIC_EUNSUPPORTED. */
PIC_API int pic_get_tuning(pic_ctx *ctx, pic_tuning *out);
PIC_API int pic_set_tuning(pic_ctx *ctx, const pic_tuning *t);

/* Times `steps` steps for each candidate tuning of the current launch mode
 * on the context's own particles (state is saved and restored) and keeps the
 * fastest.  best and ms_per_step may be NULL. */
PIC_API int pic_autotune(pic_ctx *ctx, int32_t steps, pic_tuning *best, double *ms_per_step);

/* ---- per-box costs (Sec. 2.2) and counts ------------------------------ */

/* costs[n_boxes] (caller-owned) receives the per-box cost of `strategy`.
 * Device-timer strategies return the counters accumulated since the last
 * pic_reset_costs (or pic_init).  LEARNED predicts the next interval's
 * timer cycles from the current box features; it falls back to HEURISTIC
 * when no model is loaded, or when the prediction made at the previous
 * LEARNED call missed the most recent DEVICE_TIMER reading by more than 15%
 * relative error, sum |s pred - t| / sum t over boxes with s = sum t /
 * sum pred (a common factor does not count: mappings and E depend only on
 * cost ratios); that reading should
 * cover the whole interval the prediction was made for (read the counters
 * at its end, without a reset inside it).  Intended order per balancing
 * step: read DEVICE_TIMER, reset, then LEARNED.  *used_strategy (nullable) reports which strategy produced
 * the values. */
PIC_API int pic_box_costs(pic_ctx *ctx, int32_t strategy, double *costs, int32_t *used_strategy);

/* Zeroes the device-timer counters. */
PIC_API int pic_reset_costs(pic_ctx *ctx);

/* counts[n_boxes][n_species] (caller-owned): particles whose cell
 * floor(x) lies in each box, recounted on the device. */
PIC_API int pic_box_counts(pic_ctx *ctx, int64_t *counts);

/* ---- state access ------------------------------------------------------ */

/* Looks up n particles of species s by id (n <= 2^24, ids distinct) without
 * copying the whole species: x3[n][3] and u3[n][3] (caller-owned) receive
 * each particle's position (cell units, as pic_get_particles) and momentum,
 * found[n] 1 or 0 (then x3 and u3 hold zeros).  Allocates and frees device
 * scratch; synchronises.  PIC_EINVAL for a repeated id. */
PIC_API int pic_get_particles_by_id(pic_ctx *ctx, int32_t species, const int64_t *ids, int64_t n, double *x3,
                                    double *u3, int32_t *found);

/* The same lookup for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid allocation): no
 * hipMalloc or hipFree, and no other allocating call.  Its scratch is one
 * statically sized device array per GPU (5.5 MiB, held until the process
 * ends), whose address pic_init takes once per device.  n <= 65536, else
 * PIC_EINVAL; ids must be >= 0 and distinct (a repeated id -> PIC_EINVAL,
 * after the outputs were written).  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (other threads, other contexts) race
 * and must be serialised by the caller.  Synchronises. */
PIC_API int pic_get_particles_by_id_noalloc(pic_ctx *ctx, int32_t species, const int64_t *ids, int64_t n,
                                            double *x3, double *u3, int32_t *found);

/* Copies species s's particles to caller arrays sized by *n_inout; on return
 * *n_inout is the particle count (PIC_ECAPACITY if the arrays are too small;
 * the count is still written).  Order is unspecified; ids identify
 * particles.  Any array may be NULL. */
PIC_API int pic_get_particles(pic_ctx *ctx, int32_t species, double *x3, double *u3, double *w,
                              int64_t *id, int64_t *n_inout);

/* Replaces species s's particles with n given ones (positions must lie in
 * [0, n_d), else PIC_EINVAL).  Re-sorts.  PIC_ECAPACITY if n exceeds the
 * species' capacity (pic_species_desc.capacity, or its loaded count). */
PIC_API int pic_set_particles(pic_ctx *ctx, int32_t species, const double *x3, const double *u3,
                              const double *w, const int64_t *id, int64_t n);

/* Field component comp (0..8) to / from a caller array of n_cells doubles.
 * For J the value is that of the last completed step. */
PIC_API int pic_get_field(pic_ctx *ctx, int32_t comp, double *out);
PIC_API int pic_set_field(pic_ctx *ctx, int32_t comp, const double *in);

/* ---- load balancing (Sec. 2.2, Eq. 1): pure host functions ------------ */

/* Computes a distribution mapping of n_boxes boxes onto n_ranks ranks.
 * LB_SFC: boxes ordered along the Morton Z-curve of lo/g (g = gcd of all box
 * edge lengths; key bit 3k/3k+1/3k+2 = bit k of x/y/z), cut into n_ranks
 * contiguous runs whose largest cost sum is minimal; run r < R-1 is the
 * longest one with sum <= that minimum that leaves >= R-r-1 boxes.
 * LB_KNAPSACK: boxes by (cost desc, index asc) each go to the rank with the
 * smallest (load, index) among ranks holding fewer than ceil(1.5 n_boxes /
 * n_ranks) boxes.  rank_of_box[n_boxes] out; *efficiency (nullable) gets
 * E of the result.  PIC_EINVAL for n_ranks < 1, n_boxes < 1, or a negative
 * or NaN cost.  Deterministic: identical inputs give identical mappings. */
PIC_API int lb_distribute(const double *costs, const pic_box *boxes, int32_t n_boxes,
                          int32_t n_ranks, int32_t policy, int32_t *rank_of_box, double *efficiency);

/* E = c_avg / c_max over ranks (Eq. 1); a rank's cost is the sum of its
 * boxes' costs, boxes in ascending index; ranks with no box count as 0.
 * Returns 1 when all costs are 0, and -1 for invalid arguments. */
PIC_API double lb_efficiency(const double *costs, const int32_t *rank_of_box, int32_t n_boxes,
                             int32_t n_ranks);

/* 1 iff e_proposed >= (1 + threshold) * e_current (improvement relative to the
 * current efficiency, met or exceeded; Sec. 2.2, Sec. 3.2). */
PIC_API int lb_should_adopt(double e_current, double e_proposed, double threshold);

/* Morton key of box-grid coordinates (21 bits each). */
PIC_API uint64_t lb_morton_key(uint32_t x, uint32_t y, uint32_t z);

/* Halo traffic a mapping implies (the communication the paper expects SFC
 * to reduce, Sec. 3.3 and Sec. 6): for every face shared by two boxes on
 * different ranks (periodic domain), each of the two ranks sends
 * bytes_per_face_cell per cell of that face (e.g. guard depth x components
 * x bytes).  per_rank[n_ranks] (nullable) receives each rank's bytes,
 * *total (nullable) their sum.  PIC_EINVAL if the boxes do not tile the
 * domain or a rank is out of range. */
PIC_API int lb_comm_volume(const pic_box *boxes, int32_t n_boxes, const int32_t n_cells[3],
                           const int32_t *rank_of_box, int32_t n_ranks, double bytes_per_face_cell,
                           double *per_rank, double *total);

/* ---- learned cost model ----------------------------------------------- */

/* feat[n_boxes][16] (caller-owned) receives per-box features:
 * 0,1 ln(1+N) of species 0 and 1; 2..9 ln(1+number of cells whose particle
 * count lies in [0],[1],[2,3],[4,7],[8,15],[16,31],[32,63],[64,inf));
 * 10 ln(cells); 11 shape order; 12 1 if the box touches a domain face;
 * 13 ln(1+particles in the box's outer cell layer); 14 ln(1+max per-cell
 * count); 15 mean |u| of the box's particles (0 if none). */
PIC_API int pic_box_features(pic_ctx *ctx, float *feat);

/* Number of MLP parameters (16-64-64-1 with biases: 5313). */
PIC_API int32_t pic_mlp_nparam(void);

/* Trains the 16-64-64-1 ReLU network (bf16 matrix-core operands, fp32
 * accumulation and master weights) on the device to predict y from X
 * (X[n][16] raw features, standardised internally with their mean and std;
 * a feature that is constant over the training set gets std 0 and enters
 * as 0 whatever its value; y[n] = ln(1 + device-timer cycles), so that
 * boxes without work are represented).  The network models the residual
 * r = y - ln(1 + N), N = the box's particles from features 0 and 1 (the
 * log of the cycles per particle), standardised: it is fitted to
 * (r - mean_r) / std_r, and yhat = ln(1 + N) + mean_r + std_r * output.
 * PIC_COST_LEARNED reports max(0, exp(yhat) - 1) with the predicted
 * residual clamped to [min r, max r] of the training set.  Minimises the
 * mean squared error with Adam
 * (lr 1e-3, betas 0.9/0.999, eps 1e-8), minibatch `batch`, `epochs` passes.
 * perm[epochs][n] (nullable) gives each epoch's sample order; NULL uses a
 * seeded shuffle.  init_w[nparam] (nullable) sets the initial weights, else
 * Kaiming-uniform from seed.  loss_per_epoch[epochs] (nullable) out, the
 * mean squared error in units of y. */
PIC_API int pic_mlp_train(pic_ctx *ctx, const float *X, const float *y, int64_t n, int32_t epochs,
                          int32_t batch, const int32_t *perm, const float *init_w, uint64_t seed,
                          float *loss_per_epoch);

/* Predicts yhat[n] = ln(1 + N) + mean_r + std_r * network(standardise(X))
 * on the device (no clamp; a model set from nparam or nparam + 32 floats
 * predicts network(standardise(X))). */
PIC_API int pic_mlp_predict(pic_ctx *ctx, const float *X, int64_t n, float *yhat);

/* One forward + backward pass on a batch without updating weights:
 * *loss and grad[nparam] (gradient of the mean squared error w.r.t. the fp32
 * master weights; inputs taken as already standardised).  For gradient
 * checks. */
PIC_API int pic_mlp_loss_grad(pic_ctx *ctx, const float *X, const float *y, int64_t n,
                              float *loss, float *grad);

/* Weights in the layout W1[64][16] b1[64] W2[64][64] b2[64] W3[64] b3[1],
 * followed by the 16 feature means and 16 feature stds (0: feature ignored)
 * and then mean_r, std_r, min r, max r and the residual flag (1: the
 * network models y - ln(1 + N); 0: y itself): nparam, nparam + 32 or
 * nparam + 37 floats.  pic_mlp_set_weights with nparam floats keeps the
 * feature standardisation; with fewer than nparam + 37 it sets mean_r = 0,
 * std_r = 1, no clamp (min r > max r also means no clamp) and flag 0;
 * std_r <= 0 -> PIC_EINVAL.  pic_mlp_get_weights needs n >= nparam + 32 and
 * writes the target transform when n >= nparam + 37. */
PIC_API int pic_mlp_set_weights(pic_ctx *ctx, const float *w, int64_t n);
PIC_API int pic_mlp_get_weights(pic_ctx *ctx, float *w, int64_t n);

/* ---- measurement ------------------------------------------------------- */

/* Device-timer cost counters on (enable != 0, the default) or off.  Off, the
 * gather-push-deposit kernel reads no clock and updates no per-box counter,
 * so DEVICE_TIMER and DEVICE_RTC costs stop accumulating; this measures the
 * counters' own overhead (the paper calls the GPU-clock strategy's cost
 * negligible, Sec. 5).  Synchronises the stream when the setting changes. */
PIC_API int pic_set_cost_timer(pic_ctx *ctx, int32_t enable);

/* LDS staging of the tile windows on (enable != 0, the default) or off.
 * Off, no tile kernel runs and nothing is staged: the global-path kernel
 * pushes every particle, gathering E and B from the global field arrays and
 * adding its current to the global J with atomics (the path that particles
 * beyond the staged halo take).  Results agree to rounding; this is the unstaged reference the
 * staged kernel is measured against.  Synchronises the stream when the
 * setting changes; pic_slow_path_count then counts every particle. */
PIC_API int pic_set_staging(pic_ctx *ctx, int32_t enable);

/* With enable != 0 the library brackets each launch of the gather-push-
 * deposit kernels (tile and global-path kernel together) and of the field
 * update with HIP events on its stream.  With field_overlap set, the field
 * update so timed is the part that follows the particle kernel; the part
 * beside it runs on the library's second stream and is not timed. */
PIC_API int pic_kernel_timing(pic_ctx *ctx, int32_t enable);

/* ms[4] = total milliseconds of {gather-push-deposit, field update, sort,
 * other} since timing was enabled; launches[4] = number of launches.
 * Synchronises. */
PIC_API int pic_kernel_times(pic_ctx *ctx, double *ms, int64_t *launches);

/* Number of particles that took the global-memory path since the last call
 * (they had drifted beyond the staged halo).  Synchronises. */
PIC_API int pic_slow_path_count(pic_ctx *ctx, int64_t *count);

/* ---- errors ------------------------------------------------------------ */

PIC_API const char *pic_strerror(int code);
/* Text of the last error on ctx (or of the last failed pic_init if NULL). */
PIC_API const char *pic_last_error(pic_ctx *ctx);

#endif /* PICBAL_H */
