/*
 * abacus_nf.h -- near-field direct force of the Abacus N-body method on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (Sec. 3.1 "Force Solver Algorithm and Serial Method" of
 * Maksimova et al., AbacusSummit): a cubic periodic box of side L is cut into
 * K^3 cells.  The near field of a particle is every particle in the cells
 * within R cells of its own cell (R = 2: the 5x5x5 block), each taken at the
 * periodic image that lies in that neighbouring cell.  Its acceleration is the
 * direct O(N^2) sum over that set,
 *
 *     a_i = G*m * sum_j d_ij * g(|d_ij|),   d_ij = x_j' - x_i,
 *
 * with g the softened inverse cube: the spline law that is exactly Newtonian
 * beyond the softening length (Sec. 2.5 "Code Parameters", Sec. 5.2
 * "Accuracy") or Plummer's g = (r^2 + eps^2)^(-3/2) (Sec. 5.2).  The spline
 * interior used here is the cubic force polynomial whose value, slope and
 * curvature match 1/r^2 at r = eps: |F| eps^2 = 10u - 15u^2 + 6u^3, u = r/eps.
 *
 * Cell rule: along each axis xt = x - L*floor(x/L), c = min(floor(xt*K/L), K-1),
 * evaluated in FP64 from the FP32 input with every operation rounded on its
 * own; linear cell index (cx*K + cy)*K + cz.  Positions outside [0, L) are
 * wrapped.  Coincident particles (and the self pair) contribute zero.
 *
 * Conventions for every entry point:
 *   - Return value: ABACUS_NF_OK (0) or a negative error code below.
 *   - Argument errors are detected and returned synchronously, before any
 *     work is enqueued and before any HIP call.
 *   - Errors found on the device (non-finite input, work-list overflow) are
 *     recorded in a per-device error word and returned by abacus_nf_sync.
 *   - "Device pointer" means memory of the current HIP device (for example
 *     a torch tensor's data_ptr()).  hip_stream is a hipStream_t (NULL = the
 *     legacy default stream).  Work is enqueued on that stream in order;
 *     build_cells and forces do not block the host.
 *   - A handle must be used from one stream at a time; the library is not
 *     thread-safe for concurrent calls on the same handle.
 */
#ifndef ABACUS_NF_H
#define ABACUS_NF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABACUS_NF_OK 0
#define ABACUS_NF_EINVAL -1     /* bad argument                                   */
#define ABACUS_NF_ENOMEM -2     /* device or host allocation failed               */
#define ABACUS_NF_EDEVICE -3    /* a HIP call failed                              */
#define ABACUS_NF_ECAPACITY -4  /* a device-side list outgrew its allocation      */
#define ABACUS_NF_ENONFINITE -5 /* a position was NaN or infinite                 */
#define ABACUS_NF_ESTATE -6     /* handle used in the wrong state                 */
#define ABACUS_NF_ELIMIT -7     /* batch larger than the fixed scratch of an entry
                                   point that allocates nothing                   */

/* Softening law (Sec. 2.5, Sec. 5.2). */
typedef enum {
    ABACUS_NF_SPLINE = 0,  /* exactly 1/r^2 beyond eps; cubic force polynomial inside */
    ABACUS_NF_PLUMMER = 1  /* potential -1/sqrt(r^2 + eps^2)                          */
} abacus_nf_kind;

/* How each sink's sum of FP32 pair terms is accumulated. */
typedef enum {
    ABACUS_NF_SUM_FP32 = 0,   /* one plain FP32 running sum per sink                       */
    ABACUS_NF_SUM_COMP32 = 1, /* FP32 block sums folded with two-sum into an FP32 (hi, lo)
                                 pair; the final per-particle reduction across lanes and
                                 source parts is FP64                                       */
    ABACUS_NF_SUM_FP64 = 2    /* every FP32 pair term added into an FP64 sum (comparison)   */
} abacus_nf_sum;

/* One periodic box of a batch: particles pos[offset .. offset+n) of the
 * position array, side L = box, K cells per side.  The boxes of a batch
 * partition the position array in order: offset of box 0 is 0, each next box
 * starts where the previous ends, and the sizes add up to n_total. */
typedef struct {
    int64_t offset;
    int64_t n;
    double box;
    int32_t K;
    int32_t reserved; /* must be 0 */
} abacus_nf_box;

/* Opaque, library-owned cell structure of one batch of boxes. */
typedef struct abacus_nf_cells_s *abacus_nf_cells;

/*
 * abacus_nf_build_cells -- sort the particles into cells (Sec. 3.1: the
 * cubic lattice of CPD^3 cells per box).
 *
 *   pos      device float32 [n_total][3], x y z of each particle, any order.
 *            Read by the enqueued work only; the handle keeps its own sorted,
 *            cell-relative copy, so pos may be reused once that work is done.
 *   n_total  number of particles (0 <= n_total < 2^31).
 *   boxes    host array [n_boxes], copied during the call.
 *   n_boxes  1 <= n_boxes <= 65536.
 *   R        near-field radius in cells (1 <= R <= 3; every box needs K >= 2R+1;
 *            the sum over boxes of K^3 must be below 2^31).
 *   cells    in/out.  If *cells is NULL a new handle is allocated.  If it holds
 *            a handle from an earlier call, that handle is rebuilt in place
 *            when its allocations are large enough (no allocation, so the call
 *            may be captured in a HIP graph), and reallocated otherwise.
 *
 * Enqueues: binning, a stable sort of particles by cell (input order within a
 * cell), the cell offsets, and the cell-relative FP32 coordinates.
 * Errors: EINVAL for bad arguments; ENOMEM; EDEVICE.  Non-finite positions
 * are reported later by abacus_nf_sync as ENONFINITE.
 */
int abacus_nf_build_cells(const float *pos, int64_t n_total, const abacus_nf_box *boxes,
                          int32_t n_boxes, int32_t R, void *hip_stream, abacus_nf_cells *cells);

/*
 * abacus_nf_forces -- near-field accelerations of every particle (Sec. 3.1
 * direct sum; softening of Sec. 2.5 / Sec. 5.2).
 *
 *   cells  a handle filled by abacus_nf_build_cells on the same stream.
 *   eps    host double [n_boxes]: softening length of each box in the box's
 *          length unit (the spline radius for SPLINE, the Plummer length for
 *          PLUMMER).  Valid range: 1e-5 <= eps*K/L <= 1.
 *   kind   ABACUS_NF_SPLINE or ABACUS_NF_PLUMMER.
 *   gm     host double [n_boxes]: G times the particle mass of each box.
 *   mode   accumulation mode (abacus_nf_sum).
 *   acc    device float32 [n_total][3], written in the input order of pos.
 *          Valid after abacus_nf_sync or for later work on the same stream.
 *
 * Allocates nothing when the handle already holds the work buffers of an
 * earlier forces call of the same batch (so it may be captured in a HIP
 * graph after one eager call).
 * Errors: EINVAL, ESTATE (handle not built), ENOMEM, EDEVICE; ECAPACITY is
 * reported by abacus_nf_sync if a device work list overflows.
 */
int abacus_nf_forces(abacus_nf_cells cells, const double *eps, abacus_nf_kind kind, const double *gm,
                     abacus_nf_sum mode, float *acc, void *hip_stream);

/*
 * abacus_nf_forces_density -- the same accelerations plus the kernel density
 * estimate computed in the same near-field pass (Sec. 3.3 "Halo Finding":
 * weight 1 - r^2/b^2 for pairs closer than b).  For every particle
 *     rho_i = sum over its near field (self pair included) of max(0, 1 - r^2/b^2),
 * a dimensionless count-weighted density (multiply by m / volume as needed).
 *
 *   b      host double [n_boxes]: kernel radius of each box in its length
 *          unit (the paper uses 40% of the mean interparticle spacing).  Valid
 *          range: 1e-4 <= b*K/L <= R, so every neighbour within b is in the
 *          near field.
 *   rho    device float32 [n_total], input order.
 *   other arguments as for abacus_nf_forces; the density is summed like the
 *   force (FP32, or FP32 chunks folded into FP64 for COMP32 and FP64 modes).
 */
int abacus_nf_forces_density(abacus_nf_cells cells, const double *eps, abacus_nf_kind kind, const double *gm,
                             abacus_nf_sum mode, const double *b, float *acc, float *rho, void *hip_stream);

/*
 * abacus_nf_forces_f64 -- the same accelerations written in FP64, without the
 * final rounding to FP32 (for precision studies: the method's accuracy target
 * is a median fractional error of 1e-5, and the FP32 output alone contributes
 * up to 6e-8).  In FP32 mode the FP32 sums are converted exactly.
 *   acc    device float64 [n_total][3], input order.
 *   other arguments, errors and allocation as for abacus_nf_forces.
 */
int abacus_nf_forces_f64(abacus_nf_cells cells, const double *eps, abacus_nf_kind kind, const double *gm,
                         abacus_nf_sum mode, double *acc, void *hip_stream);

/*
 * abacus_nf_multipoles -- multipole moments of the mass in every cell (Sec. 3.1:
 * the far-field Taylor coefficients are built from the cells' multipole moments;
 * AbacusSummit uses order p = 8), computed from the handle's cell-relative
 * coordinates:
 *     M_c^(a,b,k) = m * sum_{j in c} u_j^a v_j^b w_j^k,   a + b + k <= order,
 * (u, v, w) = position relative to the centre of its cell in cell widths (the
 * complete Cartesian basis; a reading, since the paper does not print its basis).
 *
 *   order  0 <= order <= 10; components per cell (order+1)(order+2)(order+3)/6
 *          (165 for order 8), ordered by degree n = 0..order, then a = n..0,
 *          then b = n-a..0 (k = n-a-b).
 *   mass   host double [n_boxes]: particle mass m of each box.
 *   out    device float64 [n_cells][components], cells in global order (box by
 *          box, (cx*K + cy)*K + cz within a box); every cell is written.
 * Sums are FP64 in a fixed order (deterministic): the sorted particles are cut
 * into units of 1024 slots; a cell that spans several units gets the partial
 * moments of its units added in a fixed order.  The first call on a handle (or one
 * with a higher order or a larger batch) allocates the partials buffer
 * (2 x units x components doubles); later calls allocate nothing.
 */
int abacus_nf_multipoles(abacus_nf_cells cells, int32_t order, const double *mass, double *out, void *hip_stream);

/*
 * abacus_nf_taylor_forces -- add the far-field acceleration of per-cell Taylor
 * series to acc (Sec. 3.1: the far field is a Taylor expansion of the potential
 * about each cell centre, order p; its gradient at each particle is co-added to
 * the near-field force).  With (u, v, w) the position relative to the centre of
 * its cell in cell widths and Phi = sum T^(a,b,k) u^a v^b w^k over a+b+k <= order,
 *     acc_i += -(K/L) grad_(u,v,w) Phi   (evaluated in FP64, acc rounded to FP32).
 *
 *   order   0 <= order <= 10.
 *   taylor  device float64 [n_cells][components], the coefficients of every cell
 *           in the component order of abacus_nf_multipoles (cells in global order).
 *   acc     device float32 [n_total][3], input order, read and written (typically
 *           the output of abacus_nf_forces on the same stream).
 * Allocates nothing.
 */
int abacus_nf_taylor_forces(abacus_nf_cells cells, int32_t order, const double *taylor, float *acc,
                            void *hip_stream);

/*
 * Leapfrog time stepping (Sec. 2.5, time stepping: second-order kick-drift-kick
 * leapfrog with one global step per simulation; Sec. 3.1: singlestep kicks,
 * drifts and moves particles to their new cells before the next force
 * evaluation).  Positions, velocities and accelerations are device float32
 * [n_total][3] in input order.  A kick v + a dt and a drift x + v dt are
 * evaluated in FP64 from the stored FP32 values, the product rounded before the
 * sum (no fused multiply-add), and rounded once to FP32; a drifted coordinate y
 * is wrapped into [0, L) as y - L floor(y / L), and stored as 0 if its FP32
 * rounding reaches L.  dt is host double [n_boxes], one step per box (each box
 * is an independent simulation; may be negative, must be finite).
 */

/* abacus_nf_kick -- vel += acc * dt.  Needs a handle that has been built once (for the boxes). */
int abacus_nf_kick(abacus_nf_cells cells, const double *dt, const float *acc, float *vel, void *hip_stream);

/*
 * abacus_nf_drift -- pos += vel * dt, wrapped into each box.  The handle's cells
 * then describe the old positions: forces, multipoles, Taylor forces and
 * timestep return ESTATE until abacus_nf_build_cells is called again.
 */
int abacus_nf_drift(abacus_nf_cells cells, const double *dt, const float *vel, float *pos, void *hip_stream);

/*
 * abacus_nf_timestep -- the step-size criterion (Sec. 2.5, time stepping):
 *     dt_b = eta * min over the cells c of box b of sigma_c / max_{j in c} |a_j|,
 * sigma_c^2 = (1/n_c) sum_{j in c} |v_j - mean_c(v)|^2 (all three components).
 * Cells with fewer than two particles or no nonzero acceleration do not
 * constrain the step; a box without a constraining cell gets +inf.  The cells
 * must be built from the positions the velocities and accelerations belong to.
 *   vel     device float32 [n_total][3], input order.
 *   acc     device float32 [n_total][3], input order; or NULL to take max |a_j|
 *           of each cell from the last forces call on this handle since its
 *           last build (the force pass records the largest |a|^2 it writes in
 *           each cell; ESTATE if there was no such call and the batch has
 *           particles).  Accelerations
 *           changed after that call (a far-field co-add) are not seen then.
 *   eta     > 0 (AbacusSummit uses 0.25).
 *   dt_out  host double [n_boxes].
 * Sums are FP64 (velocities taken relative to the first particle of each
 * cell); |a|^2 is the FP64 sum of the squared FP32 components; the minimum is
 * exact.  Blocks on the stream (copies n_boxes doubles to the host).  The
 * first call (or one with a larger batch) allocates its partials buffer.
 */
int abacus_nf_timestep(abacus_nf_cells cells, const float *vel, const float *acc, double eta, double *dt_out,
                       void *hip_stream);

/*
 * abacus_nf_timestep_noalloc -- abacus_nf_timestep for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same criterion, kernels, arguments and
 * result, with its unit partials and per-box minima in a fixed scratch array
 * of the library (8 MiB of device memory per device it runs on, held until the
 * process ends) instead of buffers of the handle.  It calls no allocating
 * routine.  Limits: n_total <= 2^24 particles and n_boxes <= 4096; larger
 * batches return ABACUS_NF_ELIMIT before any HIP call.  Every call on a device
 * shares that device's scratch array (each call refills what it reads), so
 * calls that overlap on one device -- two streams, two host threads -- race;
 * the caller must serialise them.  Blocks on the stream like abacus_nf_timestep.
 */
int abacus_nf_timestep_noalloc(abacus_nf_cells cells, const float *vel, const float *acc, double eta,
                               double *dt_out, void *hip_stream);

/*
 * abacus_nf_kdk_step -- one leapfrog step of size dt per box, near field only:
 *     vel += acc dt/2; pos += vel dt; build the cells again (same boxes and R);
 *     acc = near-field force at the new positions; vel += acc dt/2.
 * On entry acc must hold the accelerations at the current positions (an
 * abacus_nf_forces call on this handle, or the previous step); on return it
 * holds those at the new positions, ready for the next step.  eps, kind, gm,
 * mode as for abacus_nf_forces.  Errors as for the calls it makes.
 */
int abacus_nf_kdk_step(abacus_nf_cells cells, const double *dt, const double *eps, abacus_nf_kind kind,
                       const double *gm, abacus_nf_sum mode, float *pos, float *vel, float *acc, void *hip_stream);

/*
 * abacus_nf_reorder -- the merge step (Table "tbl:timing" "Merge New Particles":
 * particles are kept cell by cell): gather the caller's per-particle arrays into
 * the sorted order of the last build, in place, so that slot s becomes input
 * index s.  The handle's permutation becomes the identity; its cells stay valid
 * for the reordered positions, so every per-particle array of the simulation
 * (positions included) must be passed, each once.  Later forces, Taylor, kick,
 * drift and timestep calls then touch those arrays nearly sequentially.
 *   vec3    host array of n_vec3 (0..64) distinct device float32 [n_total][3]
 *           pointers (positions, velocities, accelerations, ...).
 *   ids     optional device int64 [n_total] (particle identities), or NULL.
 * The first call (or one with a larger batch) allocates n_total x 12 bytes of
 * scratch; device-to-device copies move the gathered arrays back.
 */
int abacus_nf_reorder(abacus_nf_cells cells, float *const *vec3, int32_t n_vec3, int64_t *ids, void *hip_stream);

/*
 * abacus_nf_sync -- wait for the stream, then return (and clear) the first
 * error recorded on the current device since the last sync: ENONFINITE,
 * ECAPACITY, or EDEVICE if the stream itself failed.
 */
int abacus_nf_sync(void *hip_stream);

/* Release a handle and its device memory (waits for the device first).  NULL is accepted. */
int abacus_nf_free_cells(abacus_nf_cells cells);

/* Static description of an error code; never NULL. */
const char *abacus_nf_strerror(int code);

/*
 * abacus_nf_interactions -- exact number of (sink, source) pairs the forces
 * call evaluates for this handle, self pairs included: the sum over cells c
 * of n_c times the occupancy of its (2R+1)^3 neighbourhood.  Blocks on the
 * stream (copies one number to the host).
 */
int abacus_nf_interactions(abacus_nf_cells cells, void *hip_stream, int64_t *out);

/* Which internal array abacus_nf_copy_cells copies out. */
typedef enum {
    ABACUS_NF_ARRAY_PERM = 0,       /* int32 [n_total]: input index of each sorted slot          */
    ABACUS_NF_ARRAY_CELL_START = 1, /* int32 [n_cells + 1]: first slot of each cell (all boxes)   */
    ABACUS_NF_ARRAY_SPOS = 2,       /* float32 [n_total][4]: cell-relative x, y, z in cell widths,
                                       and the z cell index, per sorted slot                      */
    ABACUS_NF_ARRAY_CELL_KEY = 3,   /* int32 [n_total]: global cell index of each sorted slot     */
    ABACUS_NF_ARRAY_CELL_AMAX2 = 4  /* float64 [n_cells]: largest |a|^2 over each cell's particles
                                       as written by the last forces call since the last build
                                       (FP64 sum of the squared written components; 0 for an
                                       empty cell); ESTATE before such a call                    */
} abacus_nf_array;

/* Number of particles and of cells (all boxes) of a built handle. */
int abacus_nf_cells_size(abacus_nf_cells cells, int64_t *n_total, int64_t *n_cells);

/*
 * abacus_nf_copy_cells -- enqueue a device-to-device copy of one internal
 * array into dst (a device buffer of at least `bytes` bytes, which must
 * equal the array's size).  For inspection and tests.
 */
int abacus_nf_copy_cells(abacus_nf_cells cells, abacus_nf_array which, void *dst, int64_t bytes,
                         void *hip_stream);

/*
 * Tuning of the force kernel: the i-tile (sinks per lane), the j-tile (LDS
 * chunk of staged sources), the source unroll, the lanes that share one sink
 * in sparse cells, and the split of long source lists.  Zero fields mean
 * "library default".  The autotuner (abacus_nf_autotune) fills it.
 */
typedef struct {
    int32_t sinks_per_lane;  /* i-tile per lane: 1, 2 or 4                                  */
    int32_t chunk;           /* j-tile: sources staged per LDS chunk (multiple of 64,
                                64*unroll <= chunk <= 512)                                   */
    int32_t unroll;          /* sources in flight per lane: 1, 2 or 4                        */
    int32_t max_lanes;       /* most lanes sharing one sink (1..64)                          */
    int32_t part_sources;    /* split a tile's source list into parts of about this many
                                sources per lane (>= 1024)                                   */
    int32_t waves_per_cu;    /* persistent-kernel waves per compute unit (0 = occupancy)     */
    int32_t occupancy;       /* register budget of the kernel variant: 0 = compiler's choice,
                                6 or 8 = at least that many waves per SIMD                   */
    int32_t reserved;        /* must be 0                                                    */
    int64_t item_capacity;   /* work-list capacity override (tests); 0 = sized from the batch */
} abacus_nf_tuning;

/* Set the tuning used by later forces calls on this handle (NULL = defaults). */
int abacus_nf_set_tuning(abacus_nf_cells cells, const abacus_nf_tuning *tuning);

/* Read the tuning in effect (defaults resolved). */
int abacus_nf_get_tuning(abacus_nf_cells cells, abacus_nf_tuning *tuning);

/*
 * abacus_nf_autotune -- time candidate tunings of the force kernel on this
 * handle's data (each candidate runs `reps` times on the stream; blocking)
 * and keep the fastest.  If cache_path is not NULL the choice is looked up
 * in, and recorded to, that JSON file under a key made of the device name,
 * kind, mode and a size class of the batch.  acc receives the forces of the
 * last run.  The chosen tuning is stored in the handle and, if out is not
 * NULL, returned.  With the environment variable ABACUS_NF_AUTOTUNE_LOG=1 the
 * time of every candidate is printed to stderr.
 */
int abacus_nf_autotune(abacus_nf_cells cells, const double *eps, abacus_nf_kind kind, const double *gm,
                       abacus_nf_sum mode, float *acc, void *hip_stream, int32_t reps,
                       const char *cache_path, abacus_nf_tuning *out);

/*
 * abacus_nf_autotune_density -- the same search for the force pass with the
 * fused density estimate (abacus_nf_forces_density; b, acc and rho as there),
 * cached under its own key.
 */
int abacus_nf_autotune_density(abacus_nf_cells cells, const double *eps, abacus_nf_kind kind, const double *gm,
                               abacus_nf_sum mode, const double *b, float *acc, float *rho, void *hip_stream,
                               int32_t reps, const char *cache_path, abacus_nf_tuning *out);

/*
 * Per-stage timing with HIP events recorded on the caller's stream around the
 * stages of build_cells and forces (off by default).  abacus_nf_last_times
 * blocks until the last recorded events complete and returns milliseconds of:
 * [0] build_cells, [1] forces work list, [2] the pairwise force kernel,
 * [3] finalize.  Stages not run since timing was enabled read as -1.
 */
int abacus_nf_set_timing(abacus_nf_cells cells, int32_t enable);
int abacus_nf_last_times(abacus_nf_cells cells, float ms[4]);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int abacus_nf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ABACUS_NF_H */
