/*
 * u1ml.h -- C ABI of the u1ml library: Luscher-Weisz multilevel Monte Carlo
 * for compact U(1) lattice gauge theory in 3+1 dimensions on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Amado, Cardoso, Cardoso, Bicudo, "Study of compact U(1) flux tubes
 * in 3+1 dimensions in lattice gauge theory using GPU's" (arXiv:1208.0166):
 * Wilson action Eq. (3), Metropolis + overrelaxation updates (Sec. 2.1), the
 * two-level multilevel algorithm with frozen time-slab boundaries (Sec. 2.2),
 * the Polyakov-loop correlator <P*(0)P(r)> estimated by products of slab
 * averaged two-link operators (Eq. (8)), and the field operators
 * a^2 F_munu = sqrt(beta) Im P_munu (Eq. (5)) inserted as in Eq. (9).
 * Options (u1ml_set_estimator): the analytical multihit of Sec. 2.2 for the
 * correlator lines, the squared components of Eq. (6) as the insertion, and
 * the correlator averaged over the three axes and both orientations.
 * Ensembles of runs on the device give the connected profile of Eq. (7)
 * (u1ml_ensemble_*).
 *
 * Conventions shared by every call:
 *  - Sites (t, x, y, z), 0 <= t < T, 0 <= x, y, z < L, periodic; direction
 *    mu = 0 is time, mu = 1, 2, 3 are x, y, z.  Link angles theta in [-pi, pi).
 *  - Host link arrays are FP64 in the natural order theta[t][z][y][x][mu]
 *    (4 L^3 T doubles).  On the device links are stored per direction and
 *    parity, links[mu][parity][site/2], with time slowest, as FP64 or FP32.
 *  - Random numbers (Salmon et al., SC'11): the FP64 path draws Philox4x64-10
 *    with key (seed, 0) and counter (site, purpose<<32 | hit<<8 | mu,
 *    pass_id, 0); the FP32 path draws Philox4x32-10 with key (seed low, seed
 *    high) and counter (site, 2<<16 | hit<<8 | mu, pass_id low, pass_id high).
 *    pass_id counts Metropolis passes.  FP64 updates use only IEEE +,-,*,/
 *    plus exp, so they are a fixed function of (links, beta, eps, seed,
 *    pass_id) on any run; FP32 results do not depend on launch geometry.
 *  - Every int-returning call returns U1ML_OK (0) or a negative error code;
 *    u1ml_last_error() gives a message for the most recent failure on the
 *    calling thread.  Handles are owned by the library, are not thread safe,
 *    and distinct handles are independent (also when driven from different
 *    threads at once).  Host pointers are only read or written during the
 *    call; the library never keeps them.
 *  - Work is queued on the stream given in the options (NULL = a stream the
 *    library creates, at default priority, and destroys with the handle).
 *    Calls that return host data synchronise that stream; every copy
 *    between host and device goes through it, never through the legacy
 *    default stream.
 */
#ifndef U1ML_H
#define U1ML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define U1ML_OK 0
#define U1ML_EINVAL (-1)  /* bad argument: sizes, ranges, NULL handle */
#define U1ML_ENOMEM (-2)  /* device or host allocation failed */
#define U1ML_EDEVICE (-3) /* HIP runtime error (message kept for u1ml_last_error) */
#define U1ML_ESTATE (-4)  /* call not valid in the current state */
#define U1ML_EIO (-5)     /* checkpoint file error */

#define U1ML_COLD 0 /* all links theta = 0 */
#define U1ML_HOT 1  /* theta = pi (2u - 1), u from counter (site, 1<<32 | mu, 0, 0) */

#define U1ML_FP64 0 /* FP64 angles, deterministic elementary functions */
#define U1ML_FP32 1 /* FP32 angles, hardware transcendentals; FP64 measurements */

#define U1ML_MAX_LEVELS 3
/* Metropolis hits per link and pass: the hit index is one byte of the
 * random-number counter, so every entry point taking n_metro requires
 * 0 <= n_metro <= U1ML_MAX_HITS (EINVAL otherwise). */
#define U1ML_MAX_HITS 255
#define U1ML_MAX_FIELD_R 32

/* Field components of Eq. (5), in this order, in every field output. */
#define U1ML_EX 0 /* sqrt(beta) Im P_01 */
#define U1ML_EY 1 /* sqrt(beta) Im P_02 */
#define U1ML_EZ 2 /* sqrt(beta) Im P_03 */
#define U1ML_BX 3 /* sqrt(beta) Im P_23 */
#define U1ML_BY 4 /* sqrt(beta) Im P_31 */
#define U1ML_BZ 5 /* sqrt(beta) Im P_12 */

typedef struct u1ml_options {
    int start;        /* U1ML_COLD or U1ML_HOT (default HOT) */
    int precision;    /* U1ML_FP64 or U1ML_FP32 (default FP64) */
    double eps;       /* Metropolis proposal theta + eps * U(-1, 1), 0 <= eps <= 2 pi
                         (default 1.0) */
    void *stream;     /* hipStream_t to queue work on; NULL = a library-owned stream */
    void *dev_buf;    /* optional caller device buffer for the links, or NULL */
    size_t dev_bytes; /* its size; must be >= u1ml_link_bytes(L, T, precision) */
    int block;        /* threads per block of the update kernels; 0 = tuned default */
    int no_graphs;    /* 0 (default): repeated sweep / multilevel calls with the same
                         arguments replay a HIP graph captured on the first call
                         (multilevel runs of more than 16384 compound sweeps in
                         all are never captured); 1: always launch kernel by kernel */
} u1ml_options;

typedef struct u1ml_observables {
    double plaquette;     /* (1/6V) sum_x sum_{mu<nu} cos theta_munu(x), Eq. (3) */
    double poly_re;       /* Re of L^-3 sum_x P(x), P = prod_t U_0(x, t) */
    double poly_im;       /* Im of the same */
    double poly_abs;      /* its modulus */
    double field_mean[6]; /* lattice averages <O_c> of the Eq. (5) operators (Eq. (7) subtraction) */
    double field2_mean[6]; /* lattice averages of the squared components of Eq. (6),
                              beta (1 - Re P_munu), same component order */
} u1ml_observables;

typedef struct u1ml_lattice u1ml_lattice;
typedef struct u1ml_batch u1ml_batch;

/* Fill *opt with the defaults above. */
void u1ml_default_options(u1ml_options *opt);

/* Bytes of device memory the links of an L^3 x T lattice take (4 L^3 T words
 * of 8 (FP64) or 4 (FP32) bytes).  Pure function; 0 for invalid sizes. */
size_t u1ml_link_bytes(int L, int T, int precision);

/* Bytes of device memory a u1ml_multilevel run of one L^3 x T lattice with
 * these arguments and estimator flags allocates for its workspace (time
 * lines, level accumulators, correlator, and with n_rf > 0 the stored field
 * sums (in the link precision), weights, transforms and contraction
 * scratch), every inner sample
 * kept.  Pure function for planning; 0 for invalid arguments.  A run whose
 * field samples would not fit is replayed with one outer iteration stored
 * (u1ml_multilevel) and then needs less. */
size_t u1ml_workspace_bytes(int L, int T, int precision, int n_levels, const int *slab_sizes, const int *n_sub,
                            int n_r, int n_rf, unsigned estimator);

/* Create a lattice (Sec. 2, Sec. 2.1): L, T even, 2 <= L, T <= 256,
 * L^4 T < 2^32; beta >= 0 finite (beta = 1/g^2 of Eq. (3)).
 * Starts cold or hot per opt (NULL = defaults) and sets pass_id = 0.
 * If opt->dev_buf is given the links live there (the caller keeps ownership
 * and must keep it alive until u1ml_destroy); otherwise the library allocates.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
int u1ml_init_lattice(int L, int T, double beta, uint64_t seed, const u1ml_options *opt, u1ml_lattice **out);

/* One compound sweep (Sec. 2.1): a Metropolis pass with n_metro hits per link
 * followed by n_or overrelaxation passes; each pass visits the checkerboard
 * classes mu = 0..3 (outer), parity 0, 1 (inner).  pass_id += (n_metro > 0).
 * 0 <= n_metro <= U1ML_MAX_HITS, n_or >= 0.  Asynchronous. */
int u1ml_sweep(u1ml_lattice *lat, int n_metro, int n_or);

/* The multilevel algorithm (Sec. 2.2) for the Polyakov correlator and the
 * field insertion of Eq. (9).
 *   slab_sizes[n_levels]: time-slab thickness per level, outer to inner; each
 *     divides T and the previous one (e.g. {4, 2}).  At a level of thickness
 *     th the spatial links on time slices t = 0 (mod th) are frozen.
 *   n_sub[n_levels]: compound sweeps (n_metro, n_or) per level iteration;
 *     every iteration updates, then measures (inner level) or recurses.
 *   r_list[n_r]: separations along x, 1 <= r < L.
 *   rf_list[n_rf] (n_rf <= U1ML_MAX_FIELD_R, may be 0): separations for which the
 *     field profile is measured; each must appear in r_list.  n_rf > 0
 *     requires n_levels <= 2 and L <= 62; every inner sample's time-line sums and field
 *     slab sums are then kept in device memory (56 (T/th_inner) L^3 bytes
 *     per sample) and contracted with the final weights at the end.  A
 *     two-level run whose samples would take more than 60 % of the free
 *     device memory is run twice over the same updates instead, keeping one
 *     outer iteration's samples (see u1ml_set_debug, flag 8).
 * The chain continues from the updated links (no restore).  Results are
 * kept on the device until u1ml_measure.  Asynchronous; EINVAL on bad sizes. */
int u1ml_multilevel(u1ml_lattice *lat, int n_levels, const int *slab_sizes, const int *n_sub, int n_metro,
                    int n_or, int n_r, const int *r_list, int n_rf, const int *rf_list);

/* For callers that cannot allocate device memory during the call: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The multilevel run of u1ml_multilevel (same arguments, the
 * lattice's estimator flags, no field insertion: n_rf = 0) with its whole
 * workspace (time lines, level accumulators, descriptors, block tables) in a
 * fixed device array of U1ML_NOALLOC_BYTES compiled into the library, one
 * per GPU, held from the first lattice created on that GPU until the process
 * ends.  The call allocates no device memory, frees none, and makes no graph:
 * kernels are launched one by one on the lattice's stream.
 *   dev_correlator: caller-owned DEVICE buffer of n_r * 2 doubles; receives
 *     C_ML(r) as [n_r][2] (Re, Im), the same bits u1ml_multilevel followed
 *     by u1ml_measure gives for the same links and pass id.
 * The links and pass id advance exactly as with u1ml_multilevel; the result
 * is not kept for u1ml_measure or u1ml_ensemble_add.  Synchronises the
 * stream before returning.  EINVAL for bad arguments and for runs whose
 * workspace does not fit the array (e.g. a 24^4 two-level run {4,2} x
 * {10,20} with r = 1..12 takes 72 MB and fits; u1ml_workspace_bytes with
 * n_rf = 0 gives the size, plus a few KB of tables).  Every call on one GPU,
 * from any lattice, uses the same array: calls that overlap in time on one
 * GPU (other threads, other streams) race and give wrong results. */
#define U1ML_NOALLOC_BYTES (96u << 20)
int u1ml_multilevel_noalloc(u1ml_lattice *lat, int n_levels, const int *slab_sizes, const int *n_sub, int n_metro,
                            int n_or, int n_r, const int *r_list, double *dev_correlator);

/* Estimator options of the multilevel runs that follow (default 0).
 * U1ML_MULTIHIT (Sec. 2.2, the variance reduction the paper applies to the
 * potential): for every separation r >= 2 the temporal links of both Polyakov
 * lines are replaced by their multihit means conj(S)/|S| I_1(beta|S|)/I_0(beta|S|)
 * (S: the link's staple), in the correlator and in the slab averages that
 * multiply a field insertion made elsewhere; r = 1 (whose two lines share
 * plaquettes) and the inner slab holding a field insertion use the links
 * themselves.  Doubles the stored time lines.
 * U1ML_FIELD_SQUARED (Eq. (6)): the field insertion of Eq. (9) uses the
 * squared components a^4 F_munu^2 = beta (1 - Re P_munu) in place of the
 * Eq. (5) operators; same component order, planes and profile layout.
 * Subtract field2_mean of u1ml_observables for the connected profile of
 * Eq. (7).  EINVAL on unknown bits. */
#define U1ML_MULTIHIT 1u
#define U1ML_FIELD_SQUARED 2u
/* U1ML_SYMMETRIC: the multilevel correlator C(r) is averaged over the six
 * separations r e, e = +-x, +-y, +-z, each estimated by the same nested slab
 * averages (three times the correlator accumulators and fold work).  The -r e
 * estimate is exactly the complex conjugate of the +r e one, so the result
 * is the real part of the mean over the three axes (imaginary part 0).  The
 * field insertion stays along +x and uses the +x lines. */
#define U1ML_SYMMETRIC 4u
int u1ml_set_estimator(u1ml_lattice *lat, unsigned flags);

/* Measure the current links and return the latest multilevel results.
 *   obs (may be NULL): plain observables of the current links.
 *   correlator (may be NULL): [n_r][2] (Re, Im) of the last multilevel C(r);
 *     ESTATE if no multilevel has run.
 *   field_profile (may be NULL): [n_rf][2 planes][6 comps][L dy][L dz][2]
 *     (Re, Im) of <P*(x0) P(x0 + r e_x) O_c(x0 + d)> with
 *     d = (m, dy, dz), m = (r-1)/2 for plane 0 and r/2 for plane 1 (the two
 *     lattice planes around the mid-point of the charges); ESTATE if the last
 *     multilevel had n_rf = 0.
 * Synchronises the stream.  Caller owns the host buffers. */
int u1ml_measure(u1ml_lattice *lat, u1ml_observables *obs, double *correlator, double *field_profile);

/* Ensemble of multilevel runs and the connected profile of Eq. (7).
 * u1ml_ensemble_add adds the last multilevel run's C(r) and field profile,
 * and the lattice means <O_c> of the inserted operator set (Eq. (5), or
 * Eq. (6) with U1ML_FIELD_SQUARED) taken on the current links, to sums kept
 * on the device.  Every run of one ensemble must have the same r list, field
 * separations and operator set (EINVAL otherwise; reset to start another);
 * ESTATE if no multilevel has run.  The first add after a reset sets up the
 * sums and synchronises the stream; later adds are asynchronous.
 * u1ml_ensemble_reset empties the ensemble (host-side, no device work). */
int u1ml_ensemble_reset(u1ml_lattice *lat);
int u1ml_ensemble_add(u1ml_lattice *lat);
/* Runs added so far and the sizes the read buffers need (n_r, n_rf of the
 * ensemble's runs; 0 when empty).  Any pointer may be NULL. */
int u1ml_ensemble_info(u1ml_lattice *lat, int *n_runs, int *n_r, int *n_rf);
/* Ensemble means over the n added runs (any pointer may be NULL):
 *   correlator [n_r][2]: mean C(r);
 *   field_profile [n_rf][2][6][L][L][2]: mean <P* P O_c>, layout of u1ml_measure;
 *   connected [n_rf][2][6][L][L][2]: Eq. (7),
 *     mean <P* P O_c>(r_f, d) / mean C(r_f) - mean <O_c>, complex division
 *     (computed on the device).
 * ESTATE if the ensemble is empty, or a field output is asked of runs
 * without field.  Synchronises the stream.  Caller owns the host buffers. */
int u1ml_ensemble_read(u1ml_lattice *lat, double *correlator, double *field_profile, double *connected);

/* Plain (single configuration) correlator of the current links:
 * out[2k], out[2k+1] = L^-3 sum_x P*(x) P(x + r_k e_x).  Synchronises. */
int u1ml_plain_correlator(u1ml_lattice *lat, int n_r, const int *r_list, double *out);

/* Copy links to / from a host FP64 array theta[t][z][y][x][mu] (4 L^3 T values).
 * set_links: every value must be finite with |theta| <= 64 (EINVAL otherwise);
 * values outside [-pi, pi) are folded back by the next update of that link;
 * FP32 lattices round them.  Synchronises. */
int u1ml_get_links(u1ml_lattice *lat, double *host);
int u1ml_set_links(u1ml_lattice *lat, const double *host);

/* Metropolis pass counter used as the third Philox counter word. */
int u1ml_get_pass_id(u1ml_lattice *lat, uint64_t *pass_id);
int u1ml_set_pass_id(u1ml_lattice *lat, uint64_t pass_id);

/* Debug recording of Metropolis decisions.  flags & 1 enables a device log of
 * capacity bytes: one byte per (class pass, half-site, hit) in launch order,
 * 1 = accepted, 0 = rejected, 2 = frozen.  Passes that no longer fit are not
 * recorded.  flags = 0 disables and frees it.  Recording forces one launch
 * per class pass (no fused or captured schedule).  flags & 2 makes the field
 * insertion use the general contraction (both transforms stored, then
 * contracted by tiles) even where the fused one applies; results agree to
 * rounding.  flags & 4 folds the innermost slab averages with the per-site
 * kernel instead of the row-staged one (same bits).  flags & 8 runs every
 * two-level multilevel with field insertion in two passes (the mode taken
 * by itself when storing every inner sample would take more than 60 % of the
 * device memory available): a first
 * pass for the top-level averages, then the same updates again from the
 * restored links, contracting each outer iteration's samples as it
 * completes; same links, pass ids and correlator bits, field to rounding,
 * twice the updates. */
int u1ml_set_debug(u1ml_lattice *lat, unsigned flags, size_t capacity);
/* Copy the log out: *n_bytes = bytes recorded; copies min(cap, *n_bytes). */
int u1ml_get_accept_log(u1ml_lattice *lat, uint8_t *out, size_t cap, size_t *n_bytes);

/* Checkpoint: a text header line (format, L, T, beta, eps, seed, pass_id,
 * precision) then the FP64 links in the host order.  load requires a lattice
 * of the same L, T, precision and restores links, beta, eps, seed, pass_id.
 * EIO on file errors, EINVAL on a mismatch. */
int u1ml_save(u1ml_lattice *lat, const char *path);
int u1ml_load(u1ml_lattice *lat, const char *path);

/* Wait for all queued work of the lattice. */
int u1ml_synchronize(u1ml_lattice *lat);

/* Bytes the lattice currently holds for multilevel workspaces (the buffers
 * counted by u1ml_workspace_bytes; they grow to the largest run so far and
 * are kept for the next).  0 for NULL. */
size_t u1ml_device_bytes(const u1ml_lattice *lat);

/* Free the lattice and everything the library allocated for it. */
void u1ml_destroy(u1ml_lattice *lat);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices of different L = T and beta updated by
 * the same launches (one launch per class pass covers all of them).
 * ------------------------------------------------------------------------- */

/* n lattices, L[i] = T[i] sizes, beta[i], seed[i]; options as for one lattice
 * (dev_buf is ignored; precision and start apply to all). */
int u1ml_batch_create(int n, const int *L, const int *T, const double *beta, const uint64_t *seed,
                      const u1ml_options *opt, u1ml_batch **out);
/* One compound sweep of every lattice (th_frozen = 0). */
int u1ml_batch_sweep(u1ml_batch *b, int n_metro, int n_or);
/* The multilevel algorithm of u1ml_multilevel on every lattice of the batch
 * at once (same levels, updates and r lists; every r < L of every lattice). */
int u1ml_batch_multilevel(u1ml_batch *b, int n_levels, const int *slab_sizes, const int *n_sub, int n_metro,
                          int n_or, int n_r, const int *r_list, int n_rf, const int *rf_list);
/* One measurement cycle of every lattice: n_sweeps compound sweeps, then a
 * single-level multilevel with slab thickness th and n_sub iterations, with
 * correlators at r = 1 .. T_i/2 for lattice i.  With use_graph != 0 the
 * whole cycle is captured once into a HIP graph and replayed on later calls
 * with the same arguments.  Asynchronous. */
int u1ml_batch_cycle(u1ml_batch *b, int n_sweeps, int n_metro, int n_or, int th, int n_sub, int use_graph);
/* u1ml_set_estimator for every lattice of the batch. */
int u1ml_batch_set_estimator(u1ml_batch *b, unsigned flags);
/* Results of lattice i as in u1ml_measure: observables of its current links,
 * correlator [n_r][2] of the last cycle or batch multilevel (r = 1..T_i/2
 * after a cycle), field_profile as in u1ml_measure.  NULL pointers skip.
 * Synchronises. */
int u1ml_batch_measure(u1ml_batch *b, int i, u1ml_observables *obs, double *correlator, double *field_profile);
int u1ml_batch_get_links(u1ml_batch *b, int i, double *host);
/* u1ml_ensemble_* for a batch: one ensemble per lattice, added together. */
int u1ml_batch_ensemble_reset(u1ml_batch *b);
int u1ml_batch_ensemble_add(u1ml_batch *b);
int u1ml_batch_ensemble_info(u1ml_batch *b, int i, int *n_runs, int *n_r, int *n_rf);
int u1ml_batch_ensemble_read(u1ml_batch *b, int i, double *correlator, double *field_profile, double *connected);
int u1ml_batch_set_links(u1ml_batch *b, int i, const double *host);
/* Pass id of lattice i (the Metropolis-pass counter of its random numbers,
 * as u1ml_get/set_pass_id).  EINVAL for i outside [0, n). */
int u1ml_batch_get_pass_id(u1ml_batch *b, int i, uint64_t *pass_id);
int u1ml_batch_set_pass_id(u1ml_batch *b, int i, uint64_t pass_id);
/* Checkpoint of a batch: a header line with the number of lattices, then
 * for every lattice in order the record u1ml_save writes (header line and
 * FP64 links).  load requires a batch of as many lattices with the same L,
 * T and precision each, reads and checks every record before changing any
 * lattice, then restores links, beta, eps, seed and pass id of each, so the
 * chains continue with the random numbers they would have drawn.  EIO on
 * file errors, EINVAL on a mismatch (the batch is then unchanged). */
int u1ml_batch_save(u1ml_batch *b, const char *path);
int u1ml_batch_load(u1ml_batch *b, const char *path);
int u1ml_batch_synchronize(u1ml_batch *b);
void u1ml_batch_destroy(u1ml_batch *b);

/* Time the update kernels at each candidate block size on this lattice's
 * shape and keep the fastest for it; *best_block receives it (may be NULL).
 * Results are bitwise identical for every block size.  Leaves the links
 * unchanged (they are saved and restored).  Synchronises. */
int u1ml_autotune(u1ml_lattice *lat, int *best_block);

/* Launch shapes of the kernels of a lattice or batch.  Every value gives the
 * same results bit for bit (each output has one owner thread and a fixed
 * summation order); they only change the speed.  u1ml_*_set_tuning checks
 * the ranges (EINVAL), waits for queued work and drops captured graphs. */
typedef struct u1ml_tuning {
    int pass_block;         /* threads per block of the class-pass kernels: 64..1024, multiple of 64 */
    int pass_xcd_map;       /* 1: a class pass's blocks run in one contiguous range per XCD, so that
                               neighbouring sites share an L2; 0: the hardware's round-robin order */
    int sample_block;       /* threads per block of the per-sample kernel (time lines, field
                               operator sums): 64..1024, multiple of 64 */
    int fold_threads;       /* threads per block of the row fold of the inner averages: 64..256,
                               multiple of 64; 0 = chosen from L and the r list */
    int field_w_planes;     /* x planes per block of the field W transform: 1..64, clamped to what
                               one block's LDS holds; 0 = chosen for occupancy */
    int field_o_planes;     /* x-plane pairs per block of the field O transform; as above */
    int field_zcon_threads; /* threads per block of the field contraction: 64..256, multiple of
                               64; 0 = chosen for the fewest idle lanes */
    int fold_stage;         /* rows the row fold stages in LDS at once: 1 = those of all children
                               of a parent slab, 2 = those of one child at a time (one thread per
                               position and separation group, so at least that many threads per
                               block); 0 = 2 where 1 would take more than 16 KB per block (the
                               faster choice on the shapes measured; the autotuner leaves this
                               value as it is).  Where the mode asked for does not fit (LDS, 256
                               threads), the other is taken, else the per-site fold */
} u1ml_tuning;
int u1ml_get_tuning(u1ml_lattice *lat, u1ml_tuning *t);
int u1ml_set_tuning(u1ml_lattice *lat, const u1ml_tuning *t);
int u1ml_batch_get_tuning(u1ml_batch *b, u1ml_tuning *t);
int u1ml_batch_set_tuning(u1ml_batch *b, const u1ml_tuning *t);

/* Autotuner of a batch: times the candidate launch shapes on this batch and
 * keeps the fastest of each kernel family (one family at a time, the others
 * at their current values): the class passes' block size (64..1024) and XCD
 * block order over three compound sweeps per candidate (best of two); then,
 * if n_levels > 0, with multilevel runs of the given shape (u1ml_multilevel
 * arguments with n_metro = 1, n_or = 3), the per-sample kernel's block
 * size, the row fold's threads and, with field separations on the fast
 * contraction path, the planes per block of both field transforms and the
 * contraction's threads, each timed over its own launches only (best of two
 * runs per candidate).  The shape should keep as many samples per lattice as
 * the runs to be tuned contract at once (up to a few tens; fewer samples make
 * smaller field grids, which favour smaller blocks) while costing a small
 * n_sub.  The links and pass ids are restored; the last multilevel result is
 * discarded (ESTATE until the next run).  *best (may be NULL) receives the
 * chosen shapes.  Synchronises. */
int u1ml_batch_autotune(u1ml_batch *b, int n_levels, const int *slab_sizes, const int *n_sub, int n_r,
                        const int *r_list, int n_rf, const int *rf_list, u1ml_tuning *best);

/* Run n_sweeps compound sweeps (n_metro, n_or) like u1ml_sweep, recording a
 * HIP event pair on the lattice's stream around every class-pass kernel, and
 * return the average kernel duration in microseconds: avg_us[0] over the
 * Metropolis class passes, avg_us[1] over the overrelaxation ones (0 if none
 * ran).  The sweeps are real updates of the chain.  Synchronises. */
int u1ml_profile_sweeps(u1ml_lattice *lat, int n_sweeps, int n_metro, int n_or, double *avg_us);
/* The same for a batch (one class-pass kernel covers every lattice). */
int u1ml_batch_profile_sweeps(u1ml_batch *b, int n_sweeps, int n_metro, int n_or, double *avg_us);

/* Streaming bandwidth of the current device measured with plain grid-stride
 * kernels of 16-byte accesses (context for the roofline fractions of the
 * update kernels; not part of the method): kind 0 reads n_bytes (a buffer
 * larger than the 256 MB Infinity Cache streams HBM, a smaller one is served
 * by the cache once warm), kind 1 copies n_bytes (bytes read plus bytes
 * written counted).  One warm-up launch, then reps launches timed with HIP
 * events; *gb_per_s receives GB/s.  Allocates and frees its own buffers on a
 * stream of its own.  EINVAL unless kind is 0 or 1, n_bytes >= 1 MiB and a
 * multiple of 16, reps >= 1; ENOMEM, EDEVICE. */
int u1ml_stream_bandwidth(int kind, size_t n_bytes, int reps, double *gb_per_s);

/* Text for an error code. */
const char *u1ml_strerror(int code);
/* Message of the most recent failure on this thread ("" if none). */
const char *u1ml_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* U1ML_H */
