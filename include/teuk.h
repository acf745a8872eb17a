/*
 * libteuk -- the (2+1)D azimuthal-mode Teukolsky equation on a Kerr
 * background, advanced by the two-step Lax-Wendroff scheme on MI355X (gfx950)
 * in double, double-double or quad-double arithmetic.
 *
 * The problem is the one the paper states (Ginjupalli & Khanna, "High-Precision
 * Numerical Simulations of Rotating Black Holes Accelerated by CUDA"):
 *   - Eq. (1) (Sec. "Teukolsky Equation"): spin weight s, azimuthal number m,
 *     mass M and spin a of the hole;
 *   - Sec. "Teukolsky Code": tortoise coordinate r*, the ansatz
 *     Psi = exp(i m phi~) r^3 Phi(t, r*, theta), the momentum
 *     Pi = d_t Phi + b d_r* Phi, the first-order form Eq. (new_teu2) and its
 *     Lax-Wendroff steps Eqs. (lw1)/(lw2); Phi = Pi = 0 on both radial
 *     boundaries, and the pole condition by the parity of |m|;
 *   - Sec. "High-Order and High-Precision": tenth-order angular derivatives
 *     (second order is also offered) and the three precisions.
 *
 * Grid (readings of the paper, which states none of these):
 *   r*_i = rstar_min + i h, h = (rstar_max - rstar_min)/(n_r - 1), i = 0..n_r-1
 *     (both end nodes are the Dirichlet boundary);
 *   theta_j = (j + 1/2) pi / n_theta, j = 0..n_theta-1 (cell centres; the pole
 *     condition enters through reflected ghost rows of sign (-1)^|m|);
 *   dt = cfl * min(h, pi / n_theta).
 *
 * Host field arrays ("interchange layout") are row-major [n_theta][n_r][p]
 * doubles: theta row j, then r* node i (fastest over nodes), then the p words
 * of one real (p = 1, 2 or 4, leading word first).  A p-word real is the exact
 * sum of its words.  Inputs are renormalised on upload into non-overlapping
 * expansions (exactly for 2 words; for 4 words exactly whenever the input
 * already is one, otherwise rounded in the last word); results are
 * non-overlapping expansions.  The device layout is private to the library.
 *
 * Ownership: the library owns every handle and all device memory.  Host
 * buffers belong to the caller and are only accessed during the call.
 * Errors: every call returns TEUK_OK (0) or a negative code; the message of
 * the last failure on the calling thread is returned by teuk_last_error().
 * A failed device launch leaves the handle in a sticky TEUK_EDEVICE state.
 * Argument validation happens on the host before any device work, so it needs
 * no GPU.  Calls on one handle must not overlap; different handles are
 * independent.
 *
 * Environment (read when a handle is created; for tests):
 *   TEUK_FAULT=alloc      creation fails with TEUK_ENOMEM after validation;
 *   TEUK_FAULT=slab-abort every slab-sweep launch starts with its error word
 *                         set, so the first wait that finds its neighbour's
 *                         flag missing gives up at once (the kernel ends
 *                         early, the handle fails with TEUK_EDEVICE at its
 *                         next synchronising call);
 *   TEUK_SLAB_COOPERATIVE slab-sweep launches are cooperative launches;
 *   TEUK_NO_SCALAR_ROWS   the FP64 wide sweeps stage the radial coefficient
 *                         rows in LDS even where scalar loads could serve them
 *                         (same results, bitwise).
 */
#ifndef TEUK_H
#define TEUK_H

#ifdef __cplusplus
extern "C" {
#endif

#define TEUK_ABI_VERSION 1

typedef enum { TEUK_FP64 = 1, TEUK_DD = 2, TEUK_QD = 4 } teuk_precision; /* value = words per real */
typedef enum { TEUK_PHI_RE = 0, TEUK_PHI_IM = 1, TEUK_PI_RE = 2, TEUK_PI_IM = 3 } teuk_field;
/* r* sweep of the step kernel (see teuk_set_sweep) */
enum { TEUK_SWEEP_SEGMENT = 0, TEUK_SWEEP_WIDE = 1, TEUK_SWEEP_WIDE2 = 2, TEUK_SWEEP_SLAB = 3 };

enum {
    TEUK_OK = 0,
    TEUK_EINVAL = -1,     /* invalid argument (checked on the host) */
    TEUK_ENOMEM = -2,     /* device or host allocation failed */
    TEUK_EDEVICE = -3,    /* HIP runtime or launch failure; sticky on the handle */
    TEUK_ENOTSUP = -4,    /* valid request this build does not support */
    TEUK_ENONFINITE = -5  /* a field holds Inf or NaN (teuk_check_finite) */
};

typedef struct {
    int n_r;            /* r* nodes including both boundary nodes, >= 3 */
    int n_theta;        /* theta cells, >= 5 */
    double rstar_min;   /* units of M */
    double rstar_max;   /* > rstar_min */
    double cfl;         /* dt = cfl * min(h, pi/n_theta), > 0 */
    double mass;        /* M: 1.0, or 0.0 for the flat-space test mode (a = 0, rstar_min > 0) */
    int angular_order;  /* 10 (production, Sec. "High-Order and High-Precision") or 2 */
} teuk_grid;

typedef struct teuk teuk_t;
typedef struct teuk_batch teuk_batch_t;

/* ABI version and a short build description ("gfx950 ..."). */
int teuk_abi_version(void);
const char *teuk_build_info(void);
/* Message of the last error on this thread ("" if none). */
const char *teuk_last_error(void);

/* Validate (s, m, a/M, grid, precision) without touching a device.
 * |s| <= 2, |a/M| < 1, n_theta >= 5, n_r >= 3, rstar_min < rstar_max, cfl > 0,
 * angular_order in {2, 10}, precision in {1, 2, 4}; mass must be 1.0, or 0.0
 * with a/M = 0 and rstar_min > 0.  Returns TEUK_OK, TEUK_EINVAL, or
 * TEUK_ENOTSUP for grids this build does not take: n_theta > 256, or
 * 8 * precision * n_r * n_theta >= 2^32 (the kernels address one word plane
 * of the eight coefficient components with 32-bit offsets). */
int teuk_validate(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec);

/* Create one instance on the current HIP device: allocates its state and
 * coefficient arrays and runs the coefficient pass (tortoise inversion and
 * the Kerr factors at working precision).  Fields start at zero.
 * *out receives the handle; on failure *out is NULL. */
int teuk_create(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec,
                teuk_t **out);
int teuk_destroy(teuk_t *h);

/* Copy the four initial fields (interchange layout, n_theta*n_r*p doubles
 * each) to the device; the radial boundary nodes are then set to zero and the
 * step counter to 0.  Synchronous: the host buffers may be reused on return.
 * TEUK_ENONFINITE (nothing uploaded) if a word off the radial boundary is
 * Inf or NaN. */
int teuk_set_initial(teuk_t *h, const double *phi_re, const double *phi_im, const double *pi_re,
                     const double *pi_im);

/* Advance n >= 0 full steps (lw1 then lw2 each).  Asynchronous on the
 * handle's stream; no host round trip between steps. */
int teuk_step(teuk_t *h, long n);

/* Synchronise the handle's stream and copy one field out (interchange layout). */
int teuk_read_field(teuk_t *h, teuk_field f, double *out);

/* Time step (leading word), steps taken since set_initial, precision words. */
double teuk_dt(const teuk_t *h);
long teuk_steps_done(const teuk_t *h);
int teuk_words(const teuk_t *h);
/* Restore the step counter after a checkpoint restart (fields via
 * set_initial); an observer's next record is then due at the next multiple
 * of its cadence, and the records it holds are kept. */
int teuk_set_step_index(teuk_t *h, long n);

/* Run subsequent work on the given hipStream_t (0 = the library's own stream).
 * Waits for the work queued on the current stream first; a device error found
 * then returns TEUK_EDEVICE and leaves the handle failed (as do teuk_set_launch,
 * teuk_set_sweep, teuk_set_fuse and teuk_set_tile, which wait the same way). */
int teuk_set_stream(teuk_t *h, void *hip_stream);

/* Set *ok to 1 if every field word is finite, else 0 (returns TEUK_ENONFINITE then). */
int teuk_check_finite(teuk_t *h, int *ok);

/* Launch shape of the step kernel (tuning knobs, results are unaffected):
 * segcols = r* nodes per work item (>= 1); block = threads per workgroup,
 * at least n_theta: 64, 128 or 256 for the segment sweep, up to 512 (dd)
 * or 1024 (FP64) for the wide sweep (256 for quad-double); 0 = the default.
 * A shape that does not fit (block too large, not enough LDS) returns
 * TEUK_EINVAL and leaves the previous shape in place.  teuk_set_tile keeps
 * the block size requested before. */
int teuk_set_tile(teuk_t *h, int segcols);
int teuk_set_launch(teuk_t *h, int segcols, int block);

/* Which r* sweep the step kernel uses (results are bitwise the same):
 * TEUK_SWEEP_SEGMENT: each group of n_theta lanes walks its own segment of
 *   segcols nodes, recomputing one column of overlap on each side;
 * TEUK_SWEEP_WIDE: the groups of a block take the columns of one segment of
 *   segcols nodes in turn and pass neighbouring values through LDS, so each
 *   column is computed once;
 * TEUK_SWEEP_WIDE2: the same with each lane taking two neighbouring columns
 *   per turn (FP64 only; TEUK_ENOTSUP otherwise);
 * TEUK_SWEEP_SLAB: one persistent launch per call (at most 4096 steps each;
 *   cut where an observer record falls due): each block keeps its segment
 *   of segcols nodes in registers and LDS for all of the launch's steps and
 *   exchanges only the edge values with the neighbouring blocks through
 *   global memory and flags, so no column is computed twice and no launch
 *   falls between steps (Sec. "Teukolsky Code": the step needs one
 *   neighbour on each side in r*).  One instance, FP64 with per-point
 *   coefficients, double-double (whose stored coefficients the kernel holds
 *   in registers) or quad-double (stored coefficients loaded per stage),
 *   n_theta 64, 128 or 256, one step per launch setting (teuk_set_fuse 1);
 *   block 256, 512 or 1024 threads and a multiple of n_theta (default
 *   4 n_theta), and segcols 1, 2 or 4 (multiword: 1 or 2) times block /
 *   n_theta; the device must hold every block at once (occupancy times
 *   compute units at least the number of segments), else TEUK_ENOTSUP.
 *   Launched plainly after that check (TEUK_SLAB_COOPERATIVE: cooperatively,
 *   the runtime then guarantees that all blocks run together).  Work on other
 *   streams or processes that holds compute units can delay blocks of a plain
 *   launch; the waits are bounded, so that shows as TEUK_EDEVICE, not a hang.
 *   In particular two slab launches running at once on different streams
 *   (two handles) can each hold part of the device while waiting for blocks
 *   that cannot start: keep such handles on one stream, or launch
 *   cooperatively.  With the
 *   default block a segment length that does not fit is replaced by the
 *   shortest that does (teuk_set_launch with a block asks for exactly that
 *   shape).  No graphs are
 *   captured for it.  A wait for a neighbouring block that does not end
 *   (about a second) makes the kernel end early and the handle fail with
 *   TEUK_EDEVICE at its next synchronising call.  teuk_set_coefficients on
 *   a handle using it falls back to the default sweep.
 * -1 restores the default: wide, or segment where the wide sweep's exchange
 * slots would exceed 64 KiB of LDS (large n_theta in dd and qd).  Resets the
 * block size to the default.  teuk_get_sweep returns the sweep in use. */
int teuk_set_sweep(teuk_t *h, int sweep);
int teuk_get_sweep(const teuk_t *h);

/* Time steps per kernel launch (1, 2 or 4; results are bitwise the same).
 * With k > 1 each launch advances k steps of a segment from registers,
 * reading k extra columns on each side (so grids whose steps are bound by
 * launch and memory latency take fewer of both).  Needs the wide sweep, dd or
 * FP64 with per-point coefficients, blocks of 128..512 threads, and every
 * work item's columns (segcols + 2k, plus k padding columns where a segment
 * reaches the right boundary) within the unrolled iterations: for dd at most
 * 2 x block / n_theta (runs of one column), for FP64 at most 4 x block /
 * n_theta (runs of one) or 3 x 2 x block / n_theta (runs of two,
 * TEUK_SWEEP_WIDE2); otherwise TEUK_EINVAL and the previous setting stays.
 * teuk_step(n) runs n / k fused launches and the remainder one step per
 * launch. */
int teuk_set_fuse(teuk_t *h, int steps_per_launch);

/* Test hooks: the eight scaled coefficients at half nodes (which = 0,
 * [8][n_theta][n_r-1][p]) or nodes (which = 1, [8][n_theta][n_r][p]), or the
 * angular weights (which = 2, [2R+1][n_theta][p]).  Order of the eight:
 * s/h b, s W, s/h K_re, s/h K_im, s Ct_re, s Ct_im, s C0_re, s C0_im with
 * s = dt/2 at half nodes and s = dt at nodes.  set_ overwrites them (for
 * stepping-only checks with externally supplied coefficients, which the
 * oracle's parity tests inject).  On an FP64 handle the first set_ switches
 * the instance from per-point coefficients to stored planes (seeded from its
 * own coefficients); stored planes have no fused form, so a handle set to
 * several steps per launch falls back to one.  If the switch fails the handle
 * is unchanged; a failed upload after it leaves the handle failed. */
int teuk_get_coefficients(teuk_t *h, int which, double *out);
int teuk_set_coefficients(teuk_t *h, int which, const double *in);

/* ---- batched form: many independent instances advanced by one launch per step.
 * Instance k has its own (s, m, a/M, grid); all share one precision.  The
 * per-instance results are bitwise identical to the single-instance form. */
int teuk_batch_create(int n, const int *s, const int *m, const double *a_over_M,
                      const teuk_grid *grids, teuk_precision prec, teuk_batch_t **out);
int teuk_batch_destroy(teuk_batch_t *b);
int teuk_batch_set_initial(teuk_batch_t *b, int k, const double *phi_re, const double *phi_im,
                           const double *pi_re, const double *pi_im);
int teuk_batch_step(teuk_batch_t *b, long n);
int teuk_batch_read_field(teuk_batch_t *b, int k, teuk_field f, double *out);
int teuk_batch_set_stream(teuk_batch_t *b, void *hip_stream);
int teuk_batch_size(const teuk_batch_t *b);
double teuk_batch_dt(const teuk_batch_t *b, int k);
int teuk_batch_set_tile(teuk_batch_t *b, int segcols);
int teuk_batch_set_launch(teuk_batch_t *b, int segcols, int block);
int teuk_batch_set_sweep(teuk_batch_t *b, int sweep);
int teuk_batch_set_fuse(teuk_batch_t *b, int steps_per_launch);
/* Capture the step loop in HIP graphs of max(1, steps_per_graph / k) launches
 * (k = steps per launch; 0 = off).  One graph is kept per state buffer a
 * replay can start from, captured at its first use or by prepare_graph;
 * steps that do not fill a graph are launched directly.  Changing the launch
 * shape, the stream or the observer drops the graphs. */
int teuk_batch_use_graph(teuk_batch_t *b, int steps_per_graph);
int teuk_use_graph(teuk_t *h, int steps_per_graph);
/* Capture, instantiate and upload both graphs now, so that no later
 * teuk_step pays for it; runs no steps, returns after the upload.  No-op when
 * graphs are off. */
int teuk_prepare_graph(teuk_t *h);
int teuk_batch_prepare_graph(teuk_batch_t *b);
/* Graph replays launched since the handle was created. */
long teuk_graph_replays(const teuk_t *h);
long teuk_batch_graph_replays(const teuk_batch_t *b);

/* Host round trip (a measurement mode, Sec. "Implementation Details": the
 * first CUDA design kept the fields on the host and copied them over PCIe
 * around the step every time step).  With on != 0, after every step the
 * state of every instance is copied to pinned host memory and back before the
 * next step; results are unchanged (bitwise), graphs and fused launches are
 * not used.  on = 0 turns it off again.  TEUK_ENOMEM if the pinned buffer
 * (one instance's state) cannot be allocated. */
int teuk_set_host_round_trip(teuk_t *h, int on);
int teuk_batch_set_host_round_trip(teuk_batch_t *b, int on);

/* Observer time series (Sec. "Kerr Black Hole Tails": the field recorded at a
 * fixed location over the whole evolution, whose late-time decay is the
 * paper's result).  Records Phi (real and imaginary part, all words) at
 * n_points grid points (r* node i[p], theta row j[p]) into a device ring of
 * `capacity` records, taken after the first launch that reaches or passes the
 * next multiple of `every` steps since set_initial (with `every` a multiple
 * of the steps per launch, exactly at those multiples).  A record is
 * 1 + 2 * words * n_points doubles: the step index (as a double), then for
 * each point p the words of Re Phi and then of Im Phi.  Recording runs on the
 * handle's stream inside the step loop (also inside captured graphs) with no
 * host round trip.  set_initial clears the records.  n_points = 0 removes
 * the observer.  1 <= n_points <= 1024, every >= 1, capacity >= 1 and
 * capacity * record length <= 2^28 doubles; otherwise TEUK_EINVAL. */
int teuk_set_observer(teuk_t *h, int n_points, const int *i, const int *j, int every, long capacity);
/* Synchronise and copy out the min(held, max_records) most recent records,
 * oldest first, to out (host, that many records).  *n_out receives their
 * number, *n_total (if not NULL) the records written since set_initial
 * (those beyond `capacity` back are overwritten).  TEUK_EINVAL without an
 * observer. */
int teuk_read_observer(teuk_t *h, long max_records, double *out, long *n_out, long *n_total);

/* The coefficient pass into caller-owned device memory, allocating nothing:
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops with preallocated buffers, harnesses that forbid
 * hipMalloc).  Same arguments and validation as teuk_create, and the same
 * kernels as its coefficient pass, so the results equal teuk_get_coefficients
 * of a handle created with the same arguments, bit for bit.  Outputs (device
 * pointers, planar, theta row fastest; p = words):
 *   d_ch[(c*p + w) * (n_r-1) * n_theta + i * n_theta + j]  half nodes, c = 0..7
 *   d_cf[(c*p + w) * n_r * n_theta + i * n_theta + j]      nodes
 *   d_wt[((k+R)*p + w) * n_theta + j]                       angular weights, R = order/2
 * in the order and scaling of teuk_get_coefficients.  The intermediate tables
 * (r and Delta at nodes and half nodes, cos and sin^2 per row, for FP64 also
 * 16 radial factors per node) live in a device array of 2^20 doubles (8 MiB)
 * that each GPU the library runs on holds until the process ends; a grid
 * needing more (p (4 n_r + 2 n_theta - 2), plus 32 n_r + 2 n_theta - 16 for
 * FP64) returns TEUK_EINVAL.  Nothing in it must start at zero.  Enqueued on
 * `stream` (a hipStream_t, NULL = the null stream) on the current device,
 * asynchronously; calls that overlap on one GPU share the array and race. */
int teuk_coefficients_noalloc(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec,
                              double *d_ch, double *d_cf, double *d_wt, void *stream);

/* FP64 FMA throughput probe (the device's attainable FP64 vector rate, the
 * reference for the step kernels' FP64 operation rates): `blocks` x `threads`
 * lanes each run `chains` (1, 2, 4 or 8) independent FMA chains of `iters`
 * iterations (a multiple of 8); *tflops receives 2 * chains * iters *
 * blocks * threads / time, *ms (if not NULL) the time of the timed launch
 * (after one untimed launch), on a stream of its own.  Returns TEUK_OK,
 * TEUK_EINVAL (bad sizes; no message is set), TEUK_ENOMEM or TEUK_EDEVICE. */
int teuk_fp64_fma_probe(int chains, int blocks, int threads, long iters, double *tflops, double *ms);

/* Test hook for the multiword arithmetic itself: out[k] = op(a[k], b[k]) for
 * k < n, each operand `words` doubles (1, 2 or 4), arrays [n][words].
 * op: 0 add, 1 sub, 2 mul, 3 multiply by the double b[k][0], 4 div,
 *     5 sqrt(a), 6 exp(a), 7 log(a), 8 sin(a), 9 cos(a) (|a| <= pi/2).
 * _host runs the routines on the CPU, _device in a gfx950 kernel (host
 * arrays in both cases).  Returns TEUK_OK, TEUK_EINVAL or a device error. */
int teuk_arith_host(int words, int op, const double *a, const double *b, double *out, int n);
int teuk_arith_device(int words, int op, const double *a, const double *b, double *out, int n);

#ifdef __cplusplus
}
#endif
#endif /* TEUK_H */
