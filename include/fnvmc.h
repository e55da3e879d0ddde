/*
 * fnvmc.h -- C ABI of the MI355X (gfx950) FermiNet VMC hot path.
 *
 * The operations follow the paper "Open-Source Fermionic Neural Networks with
 * Ionic Charge Initialization" (Pranesh, Zhu, Viswanathan, Ramsundar):
 *   fn_log_psi            log|psi| of the FermiNet ansatz (FermiNet Model
 *                         section: one- and two-electron streams, envelope of
 *                         Eq. 4, Slater determinants), the quantity the
 *                         Metropolis step compares (Electron Sampler section);
 *   fn_local_energy       E = E_kin + E_el-el + E_nuc-nuc + E_nuc-el (Eq. 2)
 *                         with E_kin from Eq. 3, per walker;
 *   vmc_metropolis_step   the Electron Sampler's Gaussian proposal and
 *                         Metropolis-Hastings accept/reject on 2 log|psi|;
 *   fn_param_grad         the training gradient of Eq. 6,
 *                         2 E_p[(E_p - E_p(E_p)) d log|psi| / d theta];
 *   fn_log_psi_vjp        sum_p c_p d log|psi_p| / d theta for caller weights
 *                         c_p (the backward of log|psi| w.r.t. theta).
 *
 * Conventions (all entry points):
 *   - Pointers marked "device" are HIP device memory owned by the caller; the
 *     configuration and everything marked "host" is read during the call
 *     only.  The library keeps no pointer after it returns and allocates no
 *     memory: every temporary lives in the caller's workspace `ws`, of at
 *     least fn_workspace_bytes(cfg, B, op) bytes (256-byte aligned).
 *   - Calls enqueue work on `stream` (a hipStream_t, NULL = the default
 *     stream) and return without synchronising.  Two calls that run at the
 *     same time must not share a workspace.
 *   - Arguments are checked before anything is enqueued; a call that returns
 *     an error has enqueued nothing.  fn_last_error() then gives a message
 *     (thread-local, valid until the thread's next call).
 *   - Non-finite values are data, not errors: a walker on a node of psi gets
 *     log|psi| = -inf, sign 0 and a NaN local energy.
 *   - Walker positions x are [B][N][3] FP64, electrons ordered spin-up first.
 *     theta is the flat parameter vector (layout below) in FP64 when
 *     precision == FN_FP64 and FP32 otherwise, 16-byte aligned; gradients
 *     come back in the same type.
 *
 * Flat parameter layout (M nuclei, L layers, widths w1/w2, K determinants):
 *   for l = 0..L-1 : V_l [d_in][w1]  rows ordered h_i, g_up, g_dn, g_i_up,
 *                                    g_i_dn; then b_l [w1]
 *   for l = 0..L-2 : W2_l [d_p][w2], c2_l [w2]
 *   for spin s = up, down with n_s > 0 :
 *                    w_s [w1][K n_s] (column k n_s + i), g_s [K n_s],
 *                    pi_s [K n_s][M], Sigma_s [K n_s][M][3][3]
 *                    (FN_ENV_ISOTROPIC: sigma_s [K n_s][M] in place of Sigma_s)
 *   with d_h = 4M, d_p = 4 at layer 0, d_h = w1, d_p = w2 afterwards and
 *   d_in = 3 d_h + 2 d_p.
 */
#ifndef FNVMC_H
#define FNVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fn_status;
#define FN_OK 0
#define FN_EINVAL 1        /* invalid argument or configuration            */
#define FN_ENOMEM 2        /* workspace smaller than fn_workspace_bytes()  */
#define FN_EUNSUPPORTED 3  /* configuration outside the built limits       */
#define FN_EHIP 4          /* a HIP runtime call failed                    */

/* Arithmetic of the network.  FN_FP64: FP64 throughout.  FN_FP32: FP32
   stream layers and orbital head on the FP32 matrix cores.
   FN_BF16_MIXED: as FN_FP32 but the stream-layer matrix products take BF16
   operands on the matrix cores with FP32 accumulation.
   FN_BF16X3_MIXED: the same products with each FP32 operand split into a
   BF16 high and low part and three BF16 products accumulated in FP32.
   FN_BF16X6_MIXED: each operand split into three BF16 parts and the six
   products whose part indices sum to at most 2, accumulated in FP32 (FP32
   operand precision on the BF16 matrix cores); the orbital head uses the
   same split.
   FN_BF16W_MIXED: BF16 weights with FP32 activations.  The weight matrices
   V of the one-electron layers and the orbital head weights w are taken as
   their BF16 values (each FP32 parameter rounded to nearest even); the
   activations, tangent and Laplacian rows stay FP32 and enter the products
   split exactly into three BF16 parts, so each product is three BF16 matrix
   products whose terms are exact, accumulated in FP32.  Every call in this
   mode (values, local energies, Metropolis moves, gradients) is the network
   whose V and w are so rounded; gradients are with respect to those rounded
   entries.  Biases, the pair layers and the envelope keep FP32 parameters.
   FN_BF16W2_MIXED: as FN_BF16W_MIXED with the activations split into two
   BF16 parts (16 significant bits), two products per layer product.
   In every mode the envelope, the determinants and their derivative traces
   run in FP64. */
#define FN_FP64 0
#define FN_FP32 1
#define FN_BF16_MIXED 2
#define FN_BF16X3_MIXED 3
#define FN_BF16X6_MIXED 4
#define FN_BF16W_MIXED 5
#define FN_BF16W2_MIXED 6

/* Envelope of Eq. 4, sum_m pi_im exp(-|Sigma_im (r_j - R_m)|).
   FN_ENV_ANISOTROPIC: Sigma_im is a 3x3 matrix (9 parameters).
   FN_ENV_ISOTROPIC: the special case Sigma_im = sigma_im I, one parameter;
   the envelope is pi exp(-|sigma| |r_j - R_m|), which skips the 3x3
   products and reads one parameter per orbital and nucleus instead of nine. */
#define FN_ENV_ANISOTROPIC 0
#define FN_ENV_ISOTROPIC 1

/* Operation selector for fn_workspace_bytes. */
#define FN_OP_LOG_PSI 0
#define FN_OP_LOCAL_ENERGY 1
#define FN_OP_METROPOLIS 2
#define FN_OP_PARAM_GRAD 3

/* Built limits. */
#define FN_MAX_NUC 32
#define FN_MAX_ELEC 32
#define FN_MAX_SPIN 16
#define FN_MAX_DET 32
#define FN_MAX_LAYERS 8
#define FN_MAX_W1 1024
#define FN_MAX_W2 64

typedef struct {
    int32_t n_nuc;          /* M, 1..FN_MAX_NUC                              */
    const double *nuc_xyz;  /* host [M][3], bohr                             */
    const double *nuc_z;    /* host [M], nuclear charges                      */
    int32_t n_up, n_down;   /* electrons per spin, each 0..FN_MAX_SPIN, sum>0 */
    int32_t n_layers;       /* L one-electron layers (L-1 pair layers), >= 1  */
    int32_t w1, w2;         /* one- / two-electron stream widths              */
    int32_t n_det;          /* K determinants                                 */
    int32_t precision;      /* FN_FP64 .. FN_BF16X6_MIXED                    */
    int32_t envelope;       /* FN_ENV_ANISOTROPIC or FN_ENV_ISOTROPIC         */
} fn_config;

/* Number of scalars in the flat parameter vector; -1 if cfg is invalid. */
int64_t fn_param_count(const fn_config *cfg);

/* Bytes of device workspace that operation `op` needs for B walkers; 0 if
   cfg, B or op is invalid (fn_last_error() says why). */
size_t fn_workspace_bytes(const fn_config *cfg, int64_t B, int32_t op);

/* log|psi| (FermiNet Model section) for B walkers.
   theta: device, flat parameters.  x: device [B][N][3].
   log_abs_psi: device [B] FP64 out.  sign: device [B] int8 out (+1, -1, or 0
   on a node), may be NULL. */
fn_status fn_log_psi(const fn_config *cfg, const void *theta, const double *x, int64_t B, double *log_abs_psi,
                     int8_t *sign, void *ws, size_t ws_bytes, void *stream);

/* Local energy of Eq. 2 with the kinetic term of Eq. 3 read as
   -1/2 sum_c [(d log|psi| / dx_c)^2 + d^2 log|psi| / dx_c^2] over all 3N
   electron coordinates, evaluated by a forward-mode Laplacian.
   e_loc: device [B] FP64 out.  log_abs_psi: device [B] out or NULL.
   parts: device [B][4] out (kinetic, el-el, nuc-el, nuc-nuc) or NULL. */
fn_status fn_local_energy(const fn_config *cfg, const void *theta, const double *x, int64_t B, double *e_loc,
                          double *log_abs_psi, double *parts, void *ws, size_t ws_bytes, void *stream);

/* n_steps Metropolis-Hastings moves (Electron Sampler section): every
   electron of a walker moves by sigma z, z ~ N(0, 1); the move is kept iff
   log|psi'| is finite and log u <= 2 (log|psi'| - log|psi|), u ~ U(0, 1].
   Random numbers: Philox4x32-10 keyed by `seed`, counter (d, walker,
   low 32 bits of step0 + s, stream_id); normal deviate q of a walker takes
   call d = q/2 (Box-Muller, cos for even q, sin for odd q, u1 from words
   0-1, u2 from words 2-3), the accept uniform takes d = 0xFFFFFFFF words
   0-1; a word pair (a, b) maps to ((a << 21 | b >> 11) + 1) 2^-53.
   x: device [B][N][3] in/out.  log_abs_psi: device [B] in/out (must hold
   log|psi| of the incoming x).  n_accept: device [B] int32, incremented per
   accepted move, may be NULL. */
fn_status vmc_metropolis_step(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi, int64_t B,
                              int32_t n_steps, double sigma, uint64_t seed, uint64_t step0, uint32_t stream_id,
                              int32_t *n_accept, void *ws, size_t ws_bytes, void *stream);

/* As vmc_metropolis_step with the random numbers supplied by the caller:
   z: device [n_steps][B][3N] normal deviates, u: device [n_steps][B]
   uniforms in (0, 1]. */
fn_status vmc_metropolis_step_ext(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi, int64_t B,
                                  int32_t n_steps, double sigma, const double *z, const double *u, int32_t *n_accept,
                                  void *ws, size_t ws_bytes, void *stream);

/* vmc_metropolis_step for callers that cannot allocate memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid allocation):
   the same moves and results, with the workspace in a fixed device array of
   the library (64 MiB, one copy per GPU, held until the process ends)
   instead of a caller workspace.  No allocating call is made (the timing
   diagnostics skip this call).  FN_ENOMEM if fn_workspace_bytes(cfg, B,
   FN_OP_METROPOLIS) exceeds 64 MiB (for example LiH with 4 layers 256/32
   and 16 determinants up to about 2600 walkers).  Every call on one GPU
   shares that GPU's array: calls that overlap on one GPU (other streams,
   other threads) race and must be serialised by the caller. */
fn_status vmc_metropolis_step_noalloc(const fn_config *cfg, const void *theta, double *x, double *log_abs_psi,
                                      int64_t B, int32_t n_steps, double sigma, uint64_t seed, uint64_t step0,
                                      uint32_t stream_id, int32_t *n_accept, void *stream);

/* Grouped Metropolis moves (Electron Sampler section) for several jobs of
   one system and one parameter vector in one sequence of launches, for
   small jobs that would leave the GPU idle alone.  Job q owns the walkers
   walker0 .. walker0 + B - 1 of x, log_abs_psi and n_accept (the jobs must
   tile 0 .. B_total - 1 in order, without gaps) and draws its random numbers
   exactly as vmc_metropolis_step(seed, step0, stream_id) does for its own
   walkers 0 .. B - 1.  The kernels take the same path at every batch size
   (the small-batch split-reduction products are not used), so each job's
   results are bitwise those it gets in a group of its own, and those of
   vmc_metropolis_step with the "gemm_splitk" switch off.  jobs: host
   [n_jobs], 1 <= n_jobs <= FN_MAX_GROUP_JOBS.  Workspace:
   fn_workspace_bytes(cfg, B_total, FN_OP_METROPOLIS). */
#define FN_MAX_GROUP_JOBS 64
typedef struct {
    int64_t walker0;        /* first walker of the job in the group           */
    int64_t B;              /* walkers of the job, >= 1                      */
    uint64_t seed;
    uint64_t step0;         /* the job's step counter at this call's first move */
    uint32_t stream_id;
} fn_group_job;
fn_status vmc_metropolis_step_group(const fn_config *cfg, const void *theta, const fn_group_job *jobs, int32_t n_jobs,
                                    double *x, double *log_abs_psi, int32_t *n_accept, int64_t B_total,
                                    int32_t n_steps, double sigma, void *ws, size_t ws_bytes, void *stream);

/* Training gradient of Eq. 6 over the batch: with E the batch mean of e_loc,
   grad = sum_p (2/B)(e_loc_p - E) d log|psi_p| / d theta.
   e_loc: device [B] FP64.  grad: device [P] out (theta's type).
   stats: device [3] FP64 out (mean, variance with 1/B, standard error
   sqrt(var/B)), may be NULL.  The call takes positions and energies only:
   it recomputes the value-form stream activations (one row per electron,
   not the forward-Laplacian rows) in its own forward pass, keeps each
   layer's rows in the workspace for the backward, and the pair adjoint
   recomputes the pair activations from the positions. */
fn_status fn_param_grad(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *e_loc,
                        void *grad, double *stats, void *ws, size_t ws_bytes, void *stream);

/* Pretraining loss of Eq. 5 (FermiNet Training section) and its gradient:
   loss = (1/B) sum_p sum_{spin, k, i, j} (Phi^{k,spin}_{ij}(x_p) - T^{k,spin}_{ij,p})^2
   with Phi^{k,spin}_{ij} = orbital i of determinant k at electron j of that
   spin (envelope of Eq. 4 times the orbital head) and T the caller's target
   orbital values (Hartree-Fock in the paper; any values here).  Reading of
   the equation's N: the number of walkers B.  target_up: device
   [B][K][n_up][n_up] FP64 (row i = orbital, column j = electron; NULL if
   n_up = 0), target_dn likewise.  loss: device [1] FP64 out or NULL.
   grad: device [P] out (theta's type).  The orbital matrices come from a
   value-form forward pass; the backward is the log|psi| one below the
   determinants.  Workspace: fn_workspace_bytes(cfg, B, FN_OP_PARAM_GRAD). */
fn_status fn_pretrain_grad(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *target_up,
                           const double *target_dn, double *loss, void *grad, void *ws, size_t ws_bytes, void *stream);

/* grad = sum_p coeff_p d log|psi_p| / d theta.  coeff: device [B] FP64.
   grad: device [P] out (theta's type). */
fn_status fn_log_psi_vjp(const fn_config *cfg, const void *theta, const double *x, int64_t B, const double *coeff,
                         void *grad, void *ws, size_t ws_bytes, void *stream);

/* Batch statistics of the local energy and the weights of the Eq. 6
   gradient, in FP64: with E the batch mean of e_loc (the estimate of
   Eq. 1 over the B walkers), stats = (E, variance with 1/B, standard error
   sqrt(variance / B)) and coeff_p = 2 (e_loc_p - E) / B, so that
   fn_log_psi_vjp with these weights is the gradient of Eq. 6.
   e_loc: device [B].  stats: device [3] out or NULL.  coeff: device [B]
   out or NULL (not both NULL).  B >= 1.  No local-energy clipping; a
   non-finite e_loc makes every output non-finite. */
fn_status fn_energy_stats(const double *e_loc, int64_t B, double *stats, double *coeff, void *stream);

/* Electrons per nucleus of a molecular ion by the charge-initialisation
   policy of Algorithm 1 (Ionic Charge Initialization section), on the host.
   Starting from the neutral counts atomic_number[m] and t = ion_charge, while
   t != 0: for t < 0 the nucleus of smallest partial charge gains an
   electron, t and its partial charge grow by one; for t > 0 the nucleus of
   largest partial charge loses one, t and its partial charge shrink by one.
   Ties go to the lowest index.  partial_charge: host [n_nuc] (Mulliken
   charges of the ion, supplied by the caller); atomic_number: host [n_nuc];
   electrons: host [n_nuc] out.  FN_EINVAL if the policy would take an
   electron from a nucleus that has none, or ion_charge exceeds the neutral
   electron count; FN_EUNSUPPORTED beyond FN_MAX_ELEC electrons. */
fn_status fn_ionic_electron_counts(int32_t n_nuc, const double *partial_charge, const int32_t *atomic_number,
                                   int32_t ion_charge, int32_t *electrons);

/* Initial walkers (Electron Sampler section): electron i of every walker at
   the position of nucleus site[i] plus scale z, z ~ N(0, 1) from the
   sampler's generator (Philox4x32-10 keyed by seed, counter (d, walker,
   0xFFFFFFFF, stream_id), deviate q from call d = q/2 as in
   vmc_metropolis_step).  site: host [N] nucleus index per electron (spin-up
   electrons first).  x: device [B][N][3] out.  Only cfg's nuclei and
   electron counts are read. */
fn_status fn_init_walkers(const fn_config *cfg, const int32_t *site, double scale, uint64_t seed, uint32_t stream_id,
                          int64_t B, double *x, void *stream);

/* Message of the calling thread's last failed call ("" if none). */
const char *fn_last_error(void);

/* ------------------------------------------------------------------------
   Serving: continuous batching of VMC jobs (walker batches of atoms and ions
   of any electron count).  A job is B walkers of one system with its own
   parameters, n_steps Metropolis moves as in vmc_metropolis_step (step
   counter 0..n_steps-1, its own seed and stream_id) and then the batch
   mean, variance (1/B) and standard error of the local energy (Eq. 1, 2)
   plus the acceptance rate.
   Jobs of one system (identical configuration and nuclei, the same theta
   pointer, step size and step count) are admitted together as a gang: the
   first queued job of a gang takes later queued jobs of its system, in queue
   order, up to max_gang jobs and gang_walkers walkers in total.  A gang's
   walkers, log|psi|, counters, energies and one shared workspace sit in one
   block of the arena, and each quantum of its Metropolis steps is one
   vmc_metropolis_step_group call over all its jobs on the gang's stream.
   The server allocates no memory on the device or pinned on the host: every
   admitted gang's block lives in the caller's device arena, whose size is
   the HBM budget, and results land in the caller's pinned host buffer.
   fn_server_step() retires finished gangs (stream queries: each stream runs
   one gang at a time and must carry no other work), admits gangs in the
   arrival order of their first job while the block fits the free arena and
   a stream is free -- a job that does not fit even alone is passed by later
   jobs that do, at most 2 n_streams times, after which admission waits until
   it fits -- and enqueues the next quantum of every running gang on its
   stream, so the work of different gangs overlaps on the device.  A job's
   results do not depend on the other jobs: every call takes the kernel path
   that is the same at every batch size (no split-reduction products), and a
   job's log|psi| and energy estimate are computed over its own walkers.
   theta and x0 of a job are read until it is done and must stay valid until
   then.  Not safe against concurrent calls on the same server from several
   threads.
   ------------------------------------------------------------------------ */
typedef struct fn_server fn_server;

typedef struct {
    int32_t state;          /* 0 queued, 1 running, 2 done, 3 failed,
                               4 cancelled                                   */
    double mean, variance, std_error, acceptance;
    double submit_s, admit_s, done_s;   /* host steady clock, seconds        */
    int64_t footprint_bytes;            /* arena bytes of the job alone      */
    int32_t gang_jobs;                  /* jobs in the gang it ran in, 0 if
                                           never admitted                    */
} fn_job_result;

/* Arena bytes one job of B walkers needs alone (a gang of one); 0 if cfg or
   B is invalid.  A gang needs less than the sum of its jobs' footprints: its
   jobs share one workspace. */
size_t fn_server_job_bytes(const fn_config *cfg, int64_t B);

/* arena: device, 256-byte aligned, arena_bytes long.  streams: host array of
   n_streams hipStream_t (one running gang per stream).  quantum_steps:
   Metropolis steps enqueued per gang per fn_server_step.  max_gang: jobs per
   gang, 1..FN_MAX_GROUP_JOBS (1: every job runs alone).  gang_walkers: the
   most walkers a gang of several jobs may hold (a job larger than that runs
   alone).  host_results: pinned host memory (hipHostMalloc),
   [n_streams][max_gang][4] doubles, owned by the caller and valid until
   fn_server_destroy. */
fn_status fn_server_create(void *arena, size_t arena_bytes, void *const *streams, int32_t n_streams,
                           int32_t quantum_steps, int32_t max_gang, int64_t gang_walkers, double *host_results,
                           fn_server **out);
/* Queue a job; FN_ENOMEM if it could never fit the arena.  theta: device
   parameters (cfg's precision), x0: device [B][N][3] initial walkers. */
fn_status fn_server_submit(fn_server *srv, const fn_config *cfg, const void *theta, const double *x0, int64_t B,
                           int32_t n_steps, double sigma, uint64_t seed, uint32_t stream_id, int64_t *job);
/* One scheduler step (non-blocking). */
fn_status fn_server_step(fn_server *srv, int32_t *n_active, int32_t *n_queued);
fn_status fn_server_result(fn_server *srv, int64_t job, fn_job_result *out);
/* Cancel a job: a queued job leaves the queue; a running job stops being
   reported (state 4) while the rest of its gang runs on; once every job of a
   gang is cancelled, its enqueued work is waited for and its stream and
   arena block are freed.  Done, failed or cancelled jobs are left as they
   are. */
fn_status fn_server_cancel(fn_server *srv, int64_t job);
/* Free and total arena bytes. */
fn_status fn_server_memory(fn_server *srv, size_t *free_bytes, size_t *arena_bytes);
/* Waits for running jobs' streams, then frees the server. */
fn_status fn_server_destroy(fn_server *srv);
const char *fn_server_last_error(void);

/* Diagnostics: per-kernel timing.  While enabled, every launch of the
   library's kernels is bracketed by two HIP events recorded on the launch
   stream (creating events is the one allocation the library makes, and
   only in this mode).  fn_timing_read waits for the recorded events and
   returns, for the kernel class `name`, the summed duration in ms and the
   number of launches since the last reset; names: "stream_gemm" (per-
   electron stream-layer product), "walker_gemm" (per-walker mean-field
   product), "head_gemm", "features", "pair_stream", "spin_mean",
   "layer_epilogue", "envelope", "det", "combine", "pack", "propose",
   "accept" (counts no launches: the acceptance runs in the "combine"
   kernel of the proposal), "backward".  Not thread-safe with concurrent
   library calls.
   fn_timing_select(name) restricts the brackets to that one class (each
   pair of event records adds a few microseconds to the stream), NULL
   brackets every class again; FN_EINVAL for an unknown name. */
fn_status fn_timing_enable(int32_t on);
fn_status fn_timing_select(const char *name);
fn_status fn_timing_reset(void);
fn_status fn_timing_read(const char *name, double *total_ms, int64_t *launches);

/* Tuning switches (process-wide, set before launching work):
   "fused_layer" 0/1: one-electron layers as one fused kernel (product +
   forward-Laplacian epilogue) where the row layout allows it, instead of a
   product kernel followed by an epilogue kernel.  Both give the same
   arithmetic up to the order of the final additions.
   "layer_dma" 0/1: in the split-BF16 modes, stage the operand tiles of
   the fused layer and of the 128-column products by direct global-to-LDS
   copies into a two-stage ring (default 1) or through registers; results
   are bitwise equal.
   "gemm_splitk" 0/1: in the split-BF16 modes, products and value-form
   stream layers whose 128-row tiles would not fill the CUs (small walker
   batches in the value form) run as 32 x 32 tiles with the reduction split
   over the workgroup's four waves and summed in wave order (default 1), or
   as the tiled kernels; the two differ in summation order only.
   "gemm_wide" 0/1: products of 65..96 output columns (the orbital head of
   spins with 5 or 6 electrons) take 96-column tiles (default 1) or
   128-column tiles; results are bitwise equal.
   "pair_mfma" 0/1: FP32 pair layers, and their adjoint in the parameter
   gradient, as matrix-core products (default 1) or on the vector ALUs; the
   two differ in summation order only.  Unknown names and out-of-range
   values return FN_EINVAL.
   "layer_stack" 0/1/2: every one-electron layer of a forward-Laplacian
   pass in one kernel that keeps a workgroup's walkers in LDS (two to four
   electrons, w1 = 256): 0 never, 1 (default) in the one-pass BF16 mode,
   2 in every split-BF16 mode.  "stack_shape" 0/1/2: that kernel's
   workgroup shape (64 rows, two workgroups per CU; 64 rows with the next
   step's weights prefetched; 128 rows prefetched); bitwise the same results.
   "stack_regs" 0/1: for four electrons, two of each spin, w1 = 256, in the
   modes with one BF16 weight part (FN_BF16_MIXED, FN_BF16W_MIXED,
   FN_BF16W2_MIXED), every one-electron layer of a forward-Laplacian pass in
   one kernel that keeps the activations in registers and streams the
   weights through LDS (default 1; "layer_stack" 0 turns it off as well);
   it differs from the layer-by-layer kernels in summation order only.
   "fp32_products" 0..7 (diagnostic): in the split-BF16 modes, run the
   stream-layer (bit 0), mean-field (bit 1) and orbital-head (bit 2)
   products on the FP32 matrix cores instead.
   "pair_oc" 0/1/2/4: output columns per thread of the vector pair kernel
   (0: chosen by N and w2).  "pair_items" 0..4096: (pair, column group)
   items per workgroup of the vector kernel, pair rows per workgroup of the
   matrix-core kernel (0: default); the workgroup's LDS use caps it.
   Neither of the last two changes the arithmetic.
   "det_stage" 0/1: the determinant kernels copy a determinant's envelope
   parameters and orbital offsets into LDS before the envelope arithmetic
   where they fit (default 1) or read them from global memory; the values
   and the arithmetic are the same, so are the results, bit for bit. */
fn_status fn_tuning_set(const char *name, int64_t value);

#ifdef __cplusplus
}
#endif
#endif /* FNVMC_H */
