/*
 * ptymi: multi-mode ptychographic reconstruction on one MI355X (gfx950).
 *
 * The library reconstructs a complex object and a set of K incoherent probe
 * modes from far-field diffraction patterns recorded at overlapping scan
 * positions, with the three algorithms the ptychopy paper provides (Sec. 2.3:
 * ePIE, sequential over positions; DM, all positions batched with a stored
 * copy of the exit waves; LSQML, batched with per-position step lengths).
 * The call pattern follows the paper's step API (Sec. 3.2, Fig. 3, Listing 1):
 * initialise and load, iterate any number of times, fetch object and probe at
 * any time, then release.
 *
 * Notation (all sizes in pixels):
 *   N   probe window (square), K probe modes, J scan positions, H x W object.
 *   R_j = (y_j, x_j): top-left corner of patch j in object pixels, 0-based,
 *         real-valued; patches are read by bilinear interpolation (exact slices
 *         at integer positions) and written back by its exact adjoint.
 *   F   unitary 2-D DFT in natural order.
 *   complex64 = two little-endian float32 (re, im), interleaved.
 *
 * Conventions shared by every entry point:
 *   - Every call returns a pty_status; no C++ exception crosses this boundary.
 *     The message of the last failure is available from pty_last_error().
 *   - Arguments are validated before any device work: a null pointer or a
 *     size that does not match the plan gives PTY_E_INVALID; calls made out of
 *     order (e.g. iterating before patterns and positions are loaded) give
 *     PTY_E_STATE; a HIP failure gives PTY_E_DEVICE; a failed device
 *     allocation gives PTY_E_NOMEM and leaves the context as it was.
 *   - The caller owns every buffer it passes.  pty_load_* and pty_set_* copy
 *     the data before returning.  pty_get_* copy into the caller's buffer and
 *     synchronise.  pty_iterate only enqueues work on the context's stream;
 *     its errors surface at the next pty_get_* / pty_sync.
 *   - "on_device" = 1 means the pointer is device memory on the plan's device
 *     (e.g. a torch tensor's data_ptr()); 0 means host memory.
 *   - A context is not thread-safe; distinct contexts may run concurrently.
 */
#ifndef PTYMI_H
#define PTYMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pty_ctx pty_ctx; /* opaque; owns every device buffer it allocates */

typedef enum {
  PTY_OK = 0,
  PTY_E_INVALID = 1,     /* bad argument: null pointer, size or range */
  PTY_E_STATE = 2,       /* call out of order */
  PTY_E_NOMEM = 3,       /* device allocation failed (nothing leaked) */
  PTY_E_DEVICE = 4,      /* no usable device, or a HIP call failed */
  PTY_E_NUMERIC = 5,     /* NaN or Inf in the iteration error; state kept */
  PTY_E_UNSUPPORTED = 6  /* valid request this build does not implement */
} pty_status;

typedef enum { PTY_EPIE = 0, PTY_DM = 1, PTY_LSQML = 2 } pty_algo;

/* Plan: sizes and device.  n in {32, 64, 128, 256, 512}; 1 <= modes <= 4
 * (<= 2 at n = 512);
 * n_pos >= 1; obj_h, obj_w >= n + 1.  stream: a hipStream_t to enqueue on
 * (NULL = the library creates its own stream). */
typedef struct {
  int32_t n, modes, n_pos, obj_h, obj_w;
  int32_t device;
  void* stream;
  uint32_t flags; /* reserved, must be 0 */
} pty_plan_desc;

/* Iteration parameters; pty_default_params() fills the documented defaults.
 *   alpha, beta          ePIE object / probe step (default 1, 1).
 *   probe_update_start   first global iteration index (0-based) at which the
 *                        probe is updated; < 0 = never (Sec. 2.2, the
 *                        "after which iteration to update the probe" setting).
 *   lsqml_batch          LSQML positions per group; groups are interleaved,
 *                        group g = {j : j mod G = g}, G = ceil(J / batch)
 *                        (default 512).
 *   gamma_obj, gamma_probe  regularisers delta = gamma * max(denominator)
 *                        (DM default 1e-6; LSQML default 1e-3; a value < 0
 *                        selects the algorithm's default).
 *   beta_obj, beta_probe LSQML relaxation of the update (default 1, 1).
 *   order_seed           ePIE visiting order: 0 = identity, otherwise a
 *                        Fisher-Yates shuffle driven by SplitMix64 seeded with
 *                        order_seed + t in iteration t.
 *   chunk                patterns per Fourier-pass chunk (0 = automatic:
 *                        the value pty_autotune chose, else as many
 *                        patterns as a 96 MB scratch budget holds, rounded
 *                        down to whole waves of blocks over 256 CUs).
 *   flags                PTY_ITER_GRAPH: DM and LSQML iterations are captured
 *                        once per distinct setting into a HIP graph and
 *                        replayed (fewer launches; same kernels, same results
 *                        as eager iterations); ignored for ePIE.  Kernel
 *                        timing is suspended while graphs run.
 *                        PTY_ITER_ORTHO_MODES: after every iteration that
 *                        updated the probe (K > 1), the modes are replaced by
 *                        the orthogonal modes of their Gram matrix's
 *                        eigenbasis, in order of decreasing power, each
 *                        eigenvector phased so that its largest entry is real
 *                        positive (mixed states, Thibault & Menzel 2013); DM
 *                        exit waves are mixed alike.  The incoherent sum
 *                        sum_k |P_k|^2 and the object trajectory do not
 *                        change.  With equal mode powers the basis is not
 *                        unique.
 *                        PTY_ITER_POISSON (LSQML only, else
 *                        PTY_E_UNSUPPORTED): the exit-wave update follows
 *                        the Poisson likelihood (the other noise model of
 *                        LSQML, Odstrcil et al. 2018) instead of the modulus
 *                        projection: chi_j = F^-1[-alpha_R,j g Psi_j],
 *                        g = 1 - d / (I + 1e-6) on measured pixels (0 on
 *                        unmeasured ones), with alpha_R,j one Newton step of
 *                        pattern j's likelihood along that direction:
 *                        sum I g^2 / sum (I + d I / (I + 1e-6)) g^2, in
 *                        [0, 1].  The least-squares object and probe steps
 *                        are unchanged; E stays the amplitude error.
 *   position_start       LSQML position refinement from this global iteration
 *                        on; < 0 = never (default).  Each position moves by
 *                        the least-squares shift that explains its exit-wave
 *                        update along each axis (LSQML's position correction,
 *                        Odstrcil et al. 2018: sum Re(conj(d psi) chi) /
 *                        sum |d psi|^2 with d psi = P_k d(S_j O)/dy, /dx),
 *                        computed with the group's object and probe and
 *                        applied after the group's update, kept inside the
 *                        object.  The patch lists are rebuilt on the host
 *                        after each such iteration, so these iterations
 *                        synchronise; PTY_E_UNSUPPORTED with ePIE, DM or
 *                        PTY_ITER_GRAPH.  pty_get_positions returns them.
 *   position_max_shift   clip of each shift component per iteration, pixels
 *                        (default 0.5). */
#define PTY_ITER_GRAPH 1u
#define PTY_ITER_ORTHO_MODES 2u
#define PTY_ITER_POISSON 4u
typedef struct {
  float alpha, beta;
  int32_t probe_update_start;
  int32_t lsqml_batch;
  float gamma_obj, gamma_probe;
  float beta_obj, beta_probe;
  uint64_t order_seed;
  int32_t chunk;
  uint32_t flags; /* PTY_ITER_GRAPH | PTY_ITER_ORTHO_MODES | PTY_ITER_POISSON */
  int32_t position_start;
  float position_max_shift;
} pty_iter_params;

/* Fills *p with the defaults listed above. */
pty_status pty_default_params(pty_iter_params* p);

/* Creates a context for the plan: checks the device, allocates the object,
 * probe and pattern buffers.  *out is set only on success.
 * PTY_E_DEVICE when no device with that index is present. */
pty_status pty_create(const pty_plan_desc* plan, pty_ctx** out);

/* Loads J diffraction patterns of photon counts, J x N x N float32, row-major,
 * with the zero frequency at (N/2, N/2) (detector convention).  Each pattern
 * is normalised on load to its measured modulus sqrt(counts) in natural
 * (unshifted) order (Sec. 3.2: normalisation at initialisation).  Negative
 * counts are treated as 0. */
pty_status pty_load_patterns(pty_ctx* ctx, const float* counts, int on_device);

/* Blind start: sets the probe to a guess built from its size alone (Sec. 2.2:
 * the guess of the probe size and the number of modes).  Mode 0 is an
 * unaberrated aperture, a uniform real disk of `diameter` pixels centred on
 * the window (pixel centres within diameter / 2 of ((N-1)/2, (N-1)/2)); for
 * K > 1 the disk times x, y and x*y (centred pixel coordinates), made
 * orthogonal to the lower modes by Gram-Schmidt in that order.  Every mode
 * gets the power P / K, where P is the mean over the loaded patterns of their
 * total counts (negative counts as 0), so that with the unitary transform a
 * flat object predicts patterns of that total (Sec. 3.2's normalisation).
 * PTY_E_STATE before pty_load_patterns; PTY_E_INVALID for a diameter that is
 * not positive and finite, above 2 N, or too small to hold K independent
 * modes.  Synchronises. */
pty_status pty_guess_probe(pty_ctx* ctx, double diameter);

/* Detector mask shared by all patterns: N x N bytes in host memory, in the
 * counts' centred layout, nonzero where the pixel measured something and 0
 * where it did not (saturated or dead pixels, a beam stop: what Sec. 2.2's
 * saturated-pixel and noise-threshold preprocessing parameters exclude).  At
 * an unmeasured pixel the modulus projection keeps the model, and the pixel
 * adds nothing to the amplitude error E or to the Poisson likelihood and its
 * gradients.  May be called before or after pty_load_patterns and changed
 * between iterations; mask == NULL measures every pixel again.  Copies the
 * mask; synchronises.  A mask that leaves no pixel measured makes E 0/0
 * (PTY_E_NUMERIC at pty_get_errors). */
pty_status pty_set_mask(pty_ctx* ctx, const uint8_t* mask);

/* Loads J scan positions, J x 2 float64 (y, x), top-left corner of each patch
 * in object pixels.  Every patch must lie inside the object:
 * 0 <= y, floor(y) + N + (y non-integer) <= H, likewise for x with W. */
pty_status pty_load_positions(pty_ctx* ctx, const double* yx);

/* Sets the object, H x W complex64 (Sec. 2.2: the object guess). */
pty_status pty_set_object(pty_ctx* ctx, const void* c64, int on_device);

/* Sets the probe modes, K x N x N complex64 (Sec. 2.2: the probe guess). */
pty_status pty_set_probe(pty_ctx* ctx, const void* c64, int on_device);

/* Enqueues n_iter iterations of algorithm `algo` (Sec. 2.3) with parameters
 * `prm` (NULL = defaults).  Requires patterns, positions, object and probe.
 * The global iteration counter advances by n_iter and drives
 * probe_update_start.  DM keeps its exit waves between calls and initialises
 * them from the current object and probe when it starts after another
 * algorithm or after pty_set_object / pty_set_probe.  n_iter = 0 runs no
 * iteration; for DM and LSQML it allocates the work buffers those iterations
 * need (and synchronises), so that later calls only enqueue kernels. */
pty_status pty_iterate(pty_ctx* ctx, pty_algo algo, int32_t n_iter, const pty_iter_params* prm);

/* Copies the object (H x W complex64) / probe (K x N x N complex64) out; sync. */
pty_status pty_get_object(pty_ctx* ctx, void* out, int on_device);
pty_status pty_get_probe(pty_ctx* ctx, void* out, int on_device);

/* Copies the per-iteration amplitude error
 *   E = sum_j sum_q (sqrt(I_jq) - A_jq)^2 / sum_j sum_q A_jq^2
 * of every iteration run so far (float64, oldest first) into out[0..cap);
 * *n_written receives the number copied.  Synchronises.  Returns
 * PTY_E_NUMERIC if any of them is NaN or Inf (the values are still copied). */
pty_status pty_get_errors(pty_ctx* ctx, double* out, int32_t cap, int32_t* n_written);

/* Last LSQML step lengths (alpha_O, alpha_P) per position, J x 2 float32. */
pty_status pty_get_lsqml_steps(pty_ctx* ctx, float* out);

/* Copies the DM exit waves, J x K x N x N complex64 (host or device); sync.
 * PTY_E_STATE if DM has not run since the last change of object or probe. */
pty_status pty_get_exit_waves(pty_ctx* ctx, void* out, int on_device);

/* Current scan positions, J x 2 float64 (y, x), into host memory: the loaded
 * ones, or the refined ones after LSQML iterations with position refinement.
 * Synchronises.  PTY_E_STATE before pty_load_positions. */
pty_status pty_get_positions(pty_ctx* ctx, double* yx);

/* Device memory currently held by the context, in bytes. */
pty_status pty_mem_bytes(const pty_ctx* ctx, size_t* out);

/* Checkpoint and exact resume.  The step API lets a caller stop after any
 * iteration, fetch object and probe, and start again from supplied guesses
 * (Sec. 3.2, Listing 1; Sec. 2.2 for the guesses).  What object and probe do
 * not carry is copied here: the iteration counter (it decides
 * probe_update_start and the ePIE visiting order), the error history, the
 * NRMSE history while a truth is set, and the DM exit waves while they are
 * current.  With them a new context of the same shape continues a run
 * exactly: n iterations, save, restore, n iterations reproduce 2n.  Positions
 * refined by LSQML travel separately (pty_get_positions, then
 * pty_load_positions before the object, probe and state are restored).
 *
 * Host buffer, native byte order:
 *   64-byte header: the 8 characters "PTYSTAT1"; int32 n, modes, n_pos,
 *     obj_h, obj_w, iterations, has_exit_waves, has_nrmse; zero padding;
 *   float64 errors[iterations];
 *   float64 nrmse[iterations]                    if has_nrmse;
 *   complex64 exit waves[n_pos][modes][n][n]     if has_exit_waves,
 *     followed by the planes sum_k conj(P_k) psi_k [n_pos][n][n] that the
 *     last DM iteration left for the next object update.
 * pty_get_state: *n receives the size in bytes; out == NULL only asks for the
 * size; cap below it gives PTY_E_INVALID.  Synchronises.
 * pty_set_state: call after pty_set_object / pty_set_probe, which discard the
 * exit waves.  A wrong magic, a shape other than the context's or a size that
 * does not match the header gives PTY_E_INVALID with the context unchanged.
 * The NRMSE history is restored only when the context has a truth.
 * Synchronises. */
#define PTY_STATE_HEADER_BYTES 64
pty_status pty_get_state(pty_ctx* ctx, void* out, size_t cap, size_t* n);
pty_status pty_set_state(pty_ctx* ctx, const void* in, size_t n);


/* Kernel timing.  While enabled, every kernel launch of the context is
 * bracketed by HIP events on the context's stream and its duration is added
 * to its family's total.  Families, in this order (PTY_TIMING_FAMILIES):
 *   0 rows_fwd (gather, exit waves, forward FFT along x)
 *   1 cols     (FFT along y, modulus projection / NLL factor, inverse FFT along y)
 *   2 rows_inv (inverse FFT along x and the algorithm's epilogue)
 *   3 obj_gather (object tiles: sum_j S_j^T of per-pattern contributions)
 *   4 probe_acc  (probe sums over positions)
 *   5 probe_finish_apply
 *   6 lsq_steps  (LSQML per-position step lengths)
 *   7 epie_update
 *   8 other      (initialisation, reductions, fills)
 * pty_set_timing(ctx, 1) clears the totals and enables timing; 0 disables it.
 * pty_get_timing synchronises and copies, for the first `cap` families, the
 * summed duration in milliseconds and the number of launches. */
#define PTY_TIMING_FAMILIES 9
pty_status pty_set_timing(pty_ctx* ctx, int enable);
pty_status pty_get_timing(pty_ctx* ctx, double* ms, int64_t* launches, int32_t cap);

/* Waits for all enqueued work; reports deferred device errors. */
pty_status pty_sync(pty_ctx* ctx);

/* Releases every resource of the context (Listing 1's post call).  NULL-safe. */
void pty_destroy(pty_ctx* ctx);

/* Message of the last failure on this context (ctx == NULL: of the calling
 * thread's last failure without a context).  Never NULL. */
const char* pty_last_error(const pty_ctx* ctx);

/* Simulation mode (Listing 1's -simulate=1): expected photon counts
 * I_j = sum_k |F(P_k S_j O)|^2 of every position for the context's current
 * object, probe and positions, written centred (zero frequency at (N/2, N/2))
 * as J x N x N float32 to `out` (host or device).  If photons > 0 the context's
 * probe is first rescaled so that the mean pattern total equals `photons`.
 * Synchronises. */
pty_status pty_simulate(pty_ctx* ctx, double photons, float* out, int on_device);

/* Adjoint of the Poisson likelihood (not in the paper; a differentiable forward
 * model for gradient-based refinement).  For the loaded counts d (natural
 * order) and the scan positions R_j,
 *   L = sum_j sum_q [I_jq - d_jq log(I_jq + 1e-6)],  I_j = sum_k |F(P_k S_j O)|^2
 * (the constant log(d!) dropped).  obj (H x W) and probe (K x N x N) are
 * complex64 device pointers.  pos: J x 2 float32 (y, x) top-left corners in
 * device memory, so that positions being optimised never leave the device;
 * each coordinate is clamped into [0, H - N] (y) or [0, W - N] (x) (a NaN
 * into 0), which keeps every patch inside the object.  pos == NULL uses the
 * positions of pty_load_positions (PTY_E_STATE if none were loaded).
 * pty_nll_forward writes L to *loss (host) and synchronises; it stores no
 * exit waves.  pty_nll_backward recomputes them and writes grad_out times the
 * gradients in PyTorch's convention for complex tensors
 * (dL/dRe z + i dL/dIm z): g_obj (H x W complex64), g_probe (K x N x N
 * complex64) and g_pos (J x 2 float32, derivatives with respect to the
 * top-left corners y_j, x_j; bilinear weights differentiated at fixed floor),
 * all device pointers; any of them may be NULL.  With device positions the
 * object gradient's tile lists are built on the device.  *loss (may be NULL)
 * receives L.  Synchronises. */
pty_status pty_nll_forward(pty_ctx* ctx, const void* obj, const void* probe, const float* pos, double* loss);
pty_status pty_nll_backward(pty_ctx* ctx, const void* obj, const void* probe, const float* pos, float grad_out,
                            void* g_obj, void* g_probe, float* g_pos, double* loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * the Poisson likelihood L of pty_nll_forward over the first `count`
 * positions (1 <= count <= J) of the loaded patterns, computed with no
 * allocation of any kind.  Its work space (transform scratch, per-pattern
 * partial sums, slot list and the positions' floor/fraction form) lives in
 * one library-wide device array of PTY_NOALLOC_SCRATCH_BYTES per GPU, held
 * from the first pty_create on that GPU until the process ends.  Arguments as
 * for pty_nll_forward; `loss` is a device pointer to one double, written
 * asynchronously on the context's stream (no synchronisation, no host copy).
 * PTY_E_INVALID if count is out of range or the work space of `count`
 * positions does not fit the array (it needs count x (20 + 16 x column blocks)
 * bytes plus one pattern's K x N x N complex64 transform scratch; the
 * transforms run in as many chunks as the rest of the array requires).  Every
 * call on one GPU shares that array: calls that overlap on one GPU (from
 * different streams or threads) race and must be serialised by the caller.
 * The result equals pty_nll_forward's for the same count. */
#define PTY_NOALLOC_SCRATCH_BYTES (64u << 20)
pty_status pty_nll_forward_noalloc(pty_ctx* ctx, const void* obj, const void* probe, const float* pos,
                                   int32_t count, double* loss);

/* ------------------------------------------------------------------------
 * Evaluation against a known object (not in the paper; reconstruction
 * quality for synthetic data).
 * ---------------------------------------------------------------------- */

/* Amplitude error E (the per-iteration error of pty_get_errors; the paper
 * reports reconstruction progress but defines no metric) of the context's current object
 * and probe over all positions, without changing the state.  Synchronises. */
pty_status pty_model_error(pty_ctx* ctx, double* out);

/* Sets the true object (H x W complex64, host or device; copied) and the
 * region of interest: pixels whose illumination sum_j S_j^T sum_k |P_k|^2
 * under the current probe and positions is at least roi_frac of its maximum.
 * From then on every iteration records the invariant NRMSE
 *   min_c ||c O - O_true|| / ||O_true||   over the region (Fienup 1997)
 * on the device, read back with pty_get_nrmse (entries of iterations run
 * without a truth are undefined).  truth == NULL switches recording off.
 * Synchronises. */
pty_status pty_set_truth(pty_ctx* ctx, const void* truth, int on_device, float roi_frac);
/* NRMSE of the current object (needs a truth).  Synchronises. */
pty_status pty_nrmse(pty_ctx* ctx, double* out);
/* Copies up to cap per-iteration NRMSE values (iterations 0 .. n-1).  Synchronises. */
pty_status pty_get_nrmse(pty_ctx* ctx, double* out, int32_t cap, int32_t* n_written);

/* ------------------------------------------------------------------------
 * Learned initialiser (not in the paper): a U-Net that maps one 128 x 128
 * pattern to the amplitude and phase of the central 64 x 64 object patch,
 * trained on the device, whose patches are stitched into an object seed for
 * LSQML.
 *
 * Network: 3 x 3 convolutions (zero padding) with ReLU, 2 x 2 average
 * pooling, 2x nearest upsampling, skips concatenated after the upsampled
 * channels; channel widths 32-32-64-128-256-256-128-64-32-2 at resolutions
 * 128-64-32-16-8-8-16-32-64-64.  Parameters (float32 masters, bf16 copies used
 * by the kernels): per layer W[cout][3][3][cin] then b[cout].  Input: a
 * real-space estimate of the window's object patch from its counts d and the
 * known probe P (mode 0): est = g F^-1(A u) with A = sqrt(max(d, 0)) in
 * natural order, u = F(P) / |F(P)| (1 where F(P) = 0) and
 * g = conj(P) / (|P|^2 + 0.01 max |P|^2); its central 64 x 64 upsampled 2x
 * (nearest) to 128 x 128, channels Re, Im (so that the 64 x 64 output grid
 * lies on the target patch).  Output channel 0 amplitude, channel 1 phase of
 * the patch (the input fixes each patch's phase relative to the known probe).  Loss: mean
 * squared error; optimiser: Adam (beta 0.9, 0.999, eps 1e-8).
 * ---------------------------------------------------------------------- */
typedef struct pty_cnn pty_cnn;

/* Creates a network on `device` with buffers for batches of up to max_batch
 * patterns (about 5 MB of device memory per pattern); He-normal weights drawn
 * from `seed`, zero biases.  stream NULL: the network creates its own. */
pty_status pty_cnn_create(int32_t device, void* stream, int32_t max_batch, uint64_t seed, pty_cnn** out);
void pty_cnn_destroy(pty_cnn* net);                    /* NULL-safe */
const char* pty_cnn_last_error(const pty_cnn* net);   /* never NULL */
pty_status pty_cnn_num_params(const pty_cnn* net, int64_t* n);
/* Host copies of the float32 parameters (pty_cnn_num_params floats). */
pty_status pty_cnn_get_params(pty_cnn* net, float* out);
pty_status pty_cnn_set_params(pty_cnn* net, const float* in);
/* Forward pass: x (batch x 128 x 128 x 2 float32, device) -> y (batch x 64 x
 * 64 x 2 float32, device).  Synchronises. */
pty_status pty_cnn_forward(pty_cnn* net, const float* x, int32_t batch, float* y);
/* Loss and gradient with respect to the parameters for targets t (batch x 64
 * x 64 x 2, device); grad is a host array of pty_cnn_num_params floats.  The
 * parameters are not changed.  Synchronises. */
pty_status pty_cnn_grad(pty_cnn* net, const float* x, const float* target, int32_t batch, float* grad,
                        double* loss);
/* One Adam step with learning rate lr on the batch; *loss (may be NULL) gets
 * the loss before the step.  Synchronises. */
pty_status pty_cnn_train_step(pty_cnn* net, const float* x, const float* target, int32_t batch, float lr,
                              double* loss);
/* Network input (batch x 128 x 128 x 2, device) from `batch` windows of centred
 * counts (batch x 128 x 128, device) and the probe (1 x 128 x 128 complex64,
 * device; mode 0 is used), as described above.  Synchronises. */
pty_status pty_cnn_input(pty_cnn* net, const float* counts, int32_t batch, const void* probe, float* x);

/* Training data on the context's device and stream.
 * pty_poisson: out[i] ~ Poisson(lam[i]) (device arrays; lam < 10 by
 * inversion, larger by Hormann's transformed rejection (PTRS), both exact), a
 * counter-based stream per element keyed by seed.  pty_training_targets: for integer
 * positions and N = 128, the network targets of every window (J x 64 x 64 x 2,
 * device) from the context's object.  Both synchronise. */
pty_status pty_poisson(pty_ctx* ctx, const float* lam, float* out, size_t n, uint64_t seed);
pty_status pty_training_targets(pty_ctx* ctx, float* out);

/* Stitches J predicted patches (J x 64 x 64 x (amplitude, phase), device) into
 * an object: patch j sits at the nearest integer position of window j plus
 * (32, 32); a sequential chain in position order gives each patch a phase
 * factor e_j = z / |z|, z = sum over already stitched samples (the pixels
 * whose coordinates are multiples of 8) of S conj(c_j); the result is the
 * mean of c_j e_j over the patches covering a pixel, 1 where none does.
 * out: H x W complex64 device buffer, or NULL to replace the context's
 * object.  N must be 128.  Synchronises. */
pty_status pty_stitch(pty_ctx* ctx, const float* patches, void* out);

/* Learned seed of the context's object: the network input of every
 * stride-th loaded pattern (j = 0, stride, 2 stride, ...; 1 = all) from its
 * moduli and the context's probe, the forward pass in batches of `batch`
 * (on the context's stream), then the mean of the predicted patches over the
 * windows covering each pixel (placed as in pty_stitch, without its phase
 * chain: the patches already share the probe's phase reference), 1 where
 * none does.  With fallback != 0 the seed is kept only if its model error
 * (over the seeded windows) is not above that of the flat object O = 1 (else the flat object is used and
 * *used_fallback = 1); *e_seed and *e_flat (each may be NULL) receive the two
 * errors.  The network must live on the context's device.  Synchronises. */
pty_status pty_seed_object(pty_ctx* ctx, pty_cnn* net, int32_t batch, int32_t stride, int32_t fallback,
                           int32_t* used_fallback, double* e_seed, double* e_flat);

/* ------------------------------------------------------------------------
 * Batches of datasets and tuning (not in the paper; many reconstructions of
 * uneven size on one GPU).
 * ---------------------------------------------------------------------- */
typedef struct pty_batch pty_batch;

/* A batch over n existing contexts (not owned; they must outlive the batch
 * and should each have their own stream, so that their work overlaps on the
 * device).  *out is set only on success. */
pty_status pty_batch_create(pty_ctx* const* ctxs, int32_t n, pty_batch** out);
/* Enqueues n_iter iterations of `algo` on every context, iteration-major
 * (iteration t of every context before iteration t + 1 of any), each on its
 * context's stream; prm applies to all (PTY_ITER_GRAPH included).  On failure
 * returns the first context's status; the message names the context index. */
pty_status pty_batch_iterate(pty_batch* b, pty_algo algo, int32_t n_iter, const pty_iter_params* prm);
/* Waits for every context of the batch. */
pty_status pty_batch_sync(pty_batch* b);
void pty_batch_destroy(pty_batch* b);                  /* NULL-safe */
const char* pty_batch_last_error(const pty_batch* b); /* never NULL */

/* Chooses the Fourier-pass chunk (patterns per launch) and then the probe
 * sums' schedule (patterns summed per slice: 8, 16 or 32, each slice one
 * partial plane) for this context, algorithm and parameters by timing one
 * iteration per candidate after a warm-up iteration, then restores the
 * object, probe and iteration counter (DM restarts its exit waves from them).
 * With a non-NULL cache_path the choices are looked up in, and added to, that
 * JSON file, keyed by device architecture, N, K, J and algorithm.  *chunk (may
 * be NULL) receives the chunk; later iterations with chunk = 0 use both
 * choices.  Synchronises. */
pty_status pty_autotune(pty_ctx* ctx, pty_algo algo, const pty_iter_params* prm, const char* cache_path,
                        int32_t* chunk);
/* The choices in force: chunk and probe-sum slice size (0: the default rules). */
pty_status pty_get_tuning(pty_ctx* ctx, int32_t* chunk, int32_t* probe_slice);
/* pty_autotune for every context of a batch, in order (one cache file). */
pty_status pty_batch_autotune(pty_batch* b, pty_algo algo, const pty_iter_params* prm, const char* cache_path);

/* ------------------------------------------------------------------------
 * Strip decomposition (the paper's multi-GPU mode splits the scan into
 * sub-regions that overlap by a given size, Sec. 1 and Sec. 2.2).  DM and
 * LSQML, whose updates sum over positions, are decomposed exactly: the
 * positions are divided by row into `strips` groups of equal count, each held
 * by a context of its own (one GPU's share in a multi-GPU run) with the object
 * rows its patches touch.  Every object row has one owning strip.  Wherever
 * an iteration sums over positions, each strip sums its own and the partial
 * sums are exchanged: object numerator and denominator rows held by several
 * strips go to their owner as packed halo messages (added in strip order) and
 * come back as totals; the probe numerator and denominator of every strip
 * are packed into one message and summed over the strips (an all-reduce);
 * the maxima behind the regularisers and the amplitude error likewise.  The
 * result equals one context's iteration up to the order of the sums.  On one
 * GPU the strips run one after another on one stream.
 * ---------------------------------------------------------------------- */
typedef struct pty_domains pty_domains;

/* plan: the whole scan (n, modes, n_pos, obj_h, obj_w, device, stream;
 * flags 0); yx: its n_pos x 2 float64 top-left corners (host), as for
 * pty_load_positions; strips: 1..16, at most n_pos.  *out is set only on
 * success. */
pty_status pty_domains_create(const pty_plan_desc* plan, const double* yx, int32_t strips, pty_domains** out);
/* Counts of the whole scan (n_pos x N x N float32, centred), host or device;
 * each strip keeps its patterns'.  Synchronises. */
pty_status pty_domains_load_patterns(pty_domains* d, const float* counts, int on_device);
/* Whole object (obj_h x obj_w complex64) and probe (modes x N x N), host or
 * device; each strip keeps its rows of the object and a copy of the probe. */
pty_status pty_domains_set_object(pty_domains* d, const void* obj, int on_device);
pty_status pty_domains_set_probe(pty_domains* d, const void* probe, int on_device);
/* n_iter iterations of PTY_DM or PTY_LSQML with the parameters of
 * pty_iterate (flags 0, no position refinement; else PTY_E_UNSUPPORTED;
 * ePIE is sequential and is not decomposed).  Asynchronous. */
pty_status pty_domains_iterate(pty_domains* d, pty_algo algo, int32_t n_iter, const pty_iter_params* prm);
/* The whole object assembled from the owned rows of every strip, the probe
 * (identical in every strip), and the amplitude error of every iteration
 * over all positions, as pty_get_object / pty_get_probe / pty_get_errors. */
pty_status pty_domains_get_object(pty_domains* d, void* out, int on_device);
pty_status pty_domains_get_probe(pty_domains* d, void* out, int on_device);
pty_status pty_domains_get_errors(pty_domains* d, double* out, int32_t cap, int32_t* n_written);
/* Strip s: info[0..4] = first and one-past-last object row it holds, first
 * and one-past-last row it owns, number of positions. */
pty_status pty_domains_strip(const pty_domains* d, int32_t s, int32_t* info);
/* Bytes sent so far in halo messages (both directions) and in probe messages
 * (one per strip and all-reduce). */
pty_status pty_domains_traffic(const pty_domains* d, uint64_t* halo_bytes, uint64_t* probe_bytes);
pty_status pty_domains_sync(pty_domains* d);
void pty_domains_destroy(pty_domains* d);                  /* NULL-safe */
const char* pty_domains_last_error(const pty_domains* d); /* never NULL */

#ifdef __cplusplus
}
#endif
#endif /* PTYMI_H */
