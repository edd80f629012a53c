/*
 * ftcg.h -- C ABI of libftcg, an MI355X (gfx950) implementation of the
 * data-parallel hot path of frame theoretic convolutional gridding (FTCG),
 * McKay, Gelb, Monga, Raj, "Using Frame Theoretic Convolutional Gridding for
 * Robust Synthetic Aperture Sonar Imaging", arXiv:1706.08575.
 *
 * The path (Sec. III-A eq:ffind / eq:cgmatrix in 1D, Sec. IV eq:twodcg /
 * eq:twodcgmatrix in 2D):
 *   1. weight every non-uniform Fourier sample fhat_j by its frame-optimal
 *      quadrature weight alpha_j (the diagonal D of eq:difopt),
 *   2. spread alpha_j fhat_j onto a sigma-times oversampled uniform grid with
 *      a truncated Gaussian (the matrix Omega),
 *   3. inverse FFT the grid (the sum over psi_m = e^{2 pi i m x} / w(x)),
 *   4. divide by the window w(x) (deapodize) and crop to the n^d image.
 *
 * Conventions shared by every call:
 *   - Sample locations k are in cycles per field of view; the FOV is the
 *     centred box [-1/2, 1/2)^d; pixel p sits at x_p = (p - n/2) / n.
 *   - The image approximates I(x_p) = sum_j alpha_j fhat_j exp(+2 pi i k_j . x_p)
 *     (synthesis sign +, no 1/n normalisation).
 *   - Grid index g <-> k = (g - G/2) / sigma with G = sigma * n per axis;
 *     grid indices are taken modulo G, so samples outside the k-box
 *     [-n/2, n/2) wrap (pixel-centred evaluation is n-periodic in k).
 *   - Kernel: exp(-beta s^2) in grid units, beta = pi (sigma - 1/2) / (sigma W),
 *     2W taps per axis (the tap at distance exactly W, weight
 *     exp(-beta W^2) ~ 7e-7 at sigma = 2, W = 6, is dropped when u is integral).
 *   - Deapodization divides by Phi(x / sigma) per axis, Phi(t) =
 *     sqrt(pi / beta) exp(-pi^2 t^2 / beta), computed in float64.
 *   - Complex data are interleaved (re, im): complex128 for FTCG_F64 plans,
 *     complex64 for FTCG_F32 plans. Images are row-major; image axis a
 *     corresponds to k[:, a].
 *
 * Memory and threading:
 *   - Every pointer named *_dev is a DEVICE pointer owned by the caller; the
 *     plan owns its own device workspace and frees it in ftcg_plan_destroy.
 *   - Calls enqueue work on the plan's HIP stream and return without
 *     synchronising the host, except where a call says otherwise.
 *   - A plan is used by one host thread at a time and with one stream.
 *   - Errors are returned as status codes; no C++ exception crosses the ABI.
 *     On an error the plan is left in its previous valid state unless the
 *     status is FTCG_EHIP (then destroy the plan).
 */
#ifndef FTCG_H
#define FTCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftcg_plan_s* ftcg_plan;

/* The enumerations below have int as their underlying type in C++ as well,
 * so any int a C caller passes is a value of the type (the entry points
 * reject the ones outside the listed constants). */
#ifdef __cplusplus
#define FTCG_ENUM enum : int
#else
#define FTCG_ENUM enum
#endif

typedef FTCG_ENUM {
  FTCG_OK = 0,
  FTCG_EINVAL = 1,        /* bad argument (sizes, null pointer, non-finite k) */
  FTCG_ENOMEM = 2,        /* device allocation failed */
  FTCG_EHIP = 3,          /* a HIP runtime call failed */
  FTCG_ESTATE = 4,        /* call out of order (e.g. execute before set_points) */
  FTCG_EUNSUPPORTED = 5   /* valid request this library does not implement */
} ftcg_status;

typedef FTCG_ENUM { FTCG_F64 = 0, FTCG_F32 = 1 } ftcg_dtype;

typedef FTCG_ENUM {
  FTCG_W_PLAIN = 0,       /* frame-optimal diagonal weights, computed on the GPU in float64 */
  FTCG_W_LEARNED = 1,     /* weights predicted by the plan's MLP, audited against FTCG_W_PLAIN */
  FTCG_W_USER = 2,        /* caller supplies alpha with ftcg_set_weights */
  FTCG_W_NONE = 3,        /* alpha_j = 1 */
  FTCG_W_BAND = 4,        /* the (2r-1)-banded FTCG coefficient matrix C of eq:ftcg / eq:cr,
                             computed on the GPU in float64 (ftcg_plan_set_band) */
  FTCG_W_DENSITY = 5      /* iterative density compensation, the iterative quadrature weights
                             cited in Sec. III-A (ftcg_plan_set_density_iterations) */
} ftcg_wmode;

/* Human-readable name of a status code (static storage). */
const char* ftcg_status_string(ftcg_status s);

/* Create a plan.
 *   out           : receives the plan handle (host pointer).
 *   dim           : 1 or 2.
 *   n             : host array of dim image sizes per axis (each even, 8..8192;
 *                   in 2D both entries must be equal).
 *   half_width    : W, kernel half-width in grid cells (2..8).
 *   oversampling  : sigma; sigma * n must be an even integer and G = sigma*n
 *                   must be a power of two <= 16384 (FTCG_F32) / 8192 (FTCG_F64).
 *   dtype         : precision of values, spreading and FFT.
 *   wmode         : how the quadrature weights alpha are obtained.
 *   weight_radius : R, the infinity-norm neighbourhood (cycles/FOV) of the
 *                   frame-weight sum (eq:difopt truncated to ||k_i - k_j||_inf <= R), 0 < R <= 64.
 *   hip_stream    : hipStream_t to enqueue on (NULL = the default stream).
 * Weights follow eq:difopt; the grid and window follow eq:ffind / eq:twodcg. */
ftcg_status ftcg_plan_create(ftcg_plan* out, int dim, const int64_t* n, int half_width,
                             double oversampling, ftcg_dtype dtype, ftcg_wmode wmode,
                             double weight_radius, void* hip_stream);

/* Release the plan and its device workspace (synchronises the plan's stream).
 * Ends the lifetime of the operators Omega, D and the FFT plan of eq:cgmatrix
 * held for one raster; nothing of the method is computed. FTCG_EINVAL for a
 * NULL plan; the handle is invalid afterwards. */
ftcg_status ftcg_plan_destroy(ftcg_plan plan);

/* Set the sample locations (the raster {lambda_j}, Sec. III-A / Sec. IV eq:twoddataframe).
 *   m     : number of samples, 1 <= m < 2^31.
 *   k_dev : device float64 array, m x dim, row-major (k_dev[j*dim + a]).
 * Bins the samples by grid tile and, in FTCG_W_PLAIN / FTCG_W_LEARNED mode,
 * computes the weights. A non-finite coordinate, or one beyond 2^40 in
 * magnitude, gives FTCG_EINVAL (checked on the device; the host waits once,
 * for that check alone, while the binning passes already run). */
ftcg_status ftcg_set_points(ftcg_plan plan, int64_t m, const double* k_dev);

/* Caller-supplied quadrature weights: the diagonal D = diag(alpha) of
 * eq:cgmatrix / eq:D_alpha (2D: D_2 of eq:twodcgmatrix), used as given.
 *   alpha_dev : device float64 array of m weights in caller sample order,
 *               read (copied into the plan) before the call's work ends.
 * FTCG_W_USER plans only (else FTCG_ESTATE), after ftcg_set_points (else
 * FTCG_ESTATE); FTCG_EINVAL for NULL. Enqueues only. */
ftcg_status ftcg_set_weights(ftcg_plan plan, const double* alpha_dev);

/* Copy the quadrature weights in use, the diagonal of D (eq:D_alpha; for
 * FTCG_W_PLAIN the column-wise optimum of eq:difopt), to alpha_dev.
 *   alpha_dev          : device float64 array of m entries (caller order),
 *                        owned by the caller, written entirely.
 *   used_fallback_host : host int (may be NULL); receives 1 when a
 *                        FTCG_W_LEARNED plan fell back to the plain weights,
 *                        else 0 (then the call synchronises the stream).
 * FTCG_ESTATE before the points (and, for FTCG_W_USER, the weights) are set. */
ftcg_status ftcg_get_weights(ftcg_plan plan, double* alpha_dev, int* used_fallback_host);

/* The reconstruction A_cg(f) at the n^dim pixels: gamma = Omega D fhat
 * (weighting and spreading, eq:cgmatrix; 2D eq:twodcgmatrix), the sum over
 * psi_m = e^{2 pi i m x} / w(x) as an inverse FFT of the oversampled grid,
 * division by w (deapodization) and crop (eq:ffind, eq:twodcg).
 *   fhat_dev  : device, m complex values in caller sample order
 *               (complex128 / complex64 by dtype), read only.
 *   image_dev : device, n^dim complex values, row-major, written entirely.
 * FTCG_ESTATE before ftcg_set_points (and, for FTCG_W_USER, the weights);
 * FTCG_EINVAL for NULL pointers. Enqueues only (no host synchronisation). */
ftcg_status ftcg_execute(ftcg_plan plan, const void* fhat_dev, void* image_dev);

/* Forward (type-2) transform at the plan's raster: the adjoint of the
 * reconstruction with unit weights (Omega^T of eq:cgmatrix after the forward
 * DFT), fhat_j ~ sum_p I[p] exp(-2 pi i k_j . x_p), the analysis sum that
 * gives the data of Sec. III-A / eq:twoddataframe from an image on the pixel
 * grid. Steps: multiply by the deapodization factors, zero-pad to the
 * G^dim grid, forward FFT, interpolate with the spreading taps.
 *   image_dev : device, n^dim complex values (dtype), row-major, read only.
 *   fhat_dev  : device, m complex values (caller sample order), written
 *               entirely.
 * Uses the plan's grid and FFT workspace (an execute's grid is overwritten).
 * FTCG_ESTATE before ftcg_set_points; FTCG_EUNSUPPORTED for float64 plans
 * with tile 128 in 2D. Enqueues only. */
ftcg_status ftcg_forward(ftcg_plan plan, const void* image_dev, void* fhat_dev);

/* Dense frame approximation A_fr (Sec. III-B eq:binv, eq:afr, eq:afrm; 2D
 * Sec. IV eq:twodframe, eq:twodframeB), the accuracy reference of small
 * rasters that FTCG approximates with a banded C:
 *   zeta_n = e^{2 pi i n . x} / w(x), modes n_a in -n/2 .. n/2 - 1, w the
 *   plan's window Phi(x / sigma) per axis; Psi_{j,n} = <phi_j, zeta_n> =
 *   prod_a g(k_ja - n_a), g(t) = int_{-1/2}^{1/2} cos(2 pi t x) / w(x) dx
 *   (Gauss-Legendre, 4n + 64 nodes); beta = Psi^dagger fhat by a Householder
 *   QR in float64 (least squares when m >= n^dim, minimum norm otherwise);
 *   image[p] = sum_n beta_n e^{2 pi i n . x_p} / w(x_p).
 *   m, k_dev : the raster (device float64, m x dim); independent of set_points.
 *   fhat_dev : device complex128, m values.
 *   image_dev: device complex128, n^dim values, row-major, written entirely.
 * Float64 plans with n a power of two only; n^dim <= 4096 modes, n <= 1024,
 * min(m, n^dim) <= 4096 and m n^dim <= 2^27 (FTCG_EUNSUPPORTED otherwise).
 * FTCG_EINVAL when Psi is rank deficient (a pivot of R below 1e-14 of the
 * largest). Synchronises the stream (reads that check). */
ftcg_status ftcg_frame_approx(ftcg_plan plan, int64_t m, const double* k_dev, const void* fhat_dev,
                              void* image_dev);

/* Iterative density compensation (FTCG_W_DENSITY plans): the iterative
 * quadrature weights the paper cites in Sec. III-A, a comparator to the
 * frame weights of eq:difopt. From w = 1, each iteration spreads w with the
 * path's kernel and interpolates it back at the samples with the same taps
 * (d = Omega^T Omega w, Omega of eq:cgmatrix), then sets w <- w / d; the
 * weights are kept in float64, spread and interpolated in the plan's
 * precision. alpha = w (pi / (sigma beta))^dim, at which a uniform lattice of
 * spacing h (cycles per FOV) gets h^dim, as the frame weights do; samples
 * outside the k-box wrap onto the periodic grid and count there.
 *   ftcg_plan_set_density_iterations : iters in 1..1000 (default 20), from the
 *                        next ftcg_set_points; FTCG_ESTATE for other modes.
 * The weights are read with ftcg_get_weights; execute uses them as the
 * diagonal D. */
ftcg_status ftcg_plan_set_density_iterations(ftcg_plan plan, int iters);

/* Banded FTCG coefficient matrix (FTCG_W_BAND plans; Sec. III-C eq:ftcg,
 * eq:cr, eq:dif3; 2D Sec. IV eq:twodftcg): tau = Omega C fhat with C the
 * (2r-1)-banded matrix that minimises ||T C - I||_F column by column, T the
 * truncated Gram matrix of the data frame (the T of the diagonal weights),
 * the band J(n) = {n - r + 1, ..., n + r - 1} taken in the caller's sample
 * order (for a raster acquired pulse by pulse, neighbouring samples of a
 * pulse). Column n solves the normal equations of its least-squares problem
 * by a float64 Cholesky factorisation; r = 1 gives the diagonal weights of
 * FTCG_W_PLAIN.
 *   ftcg_plan_set_band : r in 1..16 (default 1); takes effect at the next
 *                        ftcg_set_points. FTCG_ESTATE for other weight modes.
 *   ftcg_set_points    : also computes C (one host synchronisation); returns
 *                        FTCG_EINVAL when a column's normal matrix is not
 *                        positive definite (T[:, J(n)] without full column
 *                        rank, e.g. two samples at one location within r
 *                        positions of each other).
 *   ftcg_execute       : forms c = C fhat in float64 (rounded to the plan's
 *                        precision), then spreads c with weight 1.
 *   ftcg_get_band      : copies C by columns to c_dev (device float64,
 *                        m x (2r-1), entry [n][p] = C[n - r + 1 + p, n], 0
 *                        where that row is outside 0..m-1); r_host (may be
 *                        NULL) receives r.
 * ftcg_get_weights returns FTCG_ESTATE for FTCG_W_BAND plans. */
ftcg_status ftcg_plan_set_band(ftcg_plan plan, int r);
ftcg_status ftcg_get_band(ftcg_plan plan, double* c_dev, int* r_host);

/* Steps of ftcg_execute, for per-step checks:
 *   ftcg_spread_only writes the oversampled grid H (G^dim complex, row-major,
 *   grid index g as in the conventions above) to grid_dev;
 *   ftcg_grid_to_image runs the inverse FFT, deapodization and crop on a
 *   caller grid (grid_dev is read only). */
ftcg_status ftcg_spread_only(ftcg_plan plan, const void* fhat_dev, void* grid_dev);
ftcg_status ftcg_grid_to_image(ftcg_plan plan, const void* grid_dev, void* image_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transform of ftcg_grid_to_image (inverse FFT, deapodization, crop) with no
 * plan and no allocation. Its workspace (the n x G intermediate, the twiddle
 * tables and the deapodization factors) is a static 36 MiB device array that
 * each GPU the library runs on holds until the process ends.
 *   dim, n, half_width, oversampling, dtype : as ftcg_plan_create (the grid is
 *                   G = oversampling * n per axis).
 *   grid_dev  : device, G^dim complex values (dtype), row-major, read only.
 *   image_dev : device, n^dim complex values, written entirely.
 *   hip_stream: stream to enqueue on (NULL = the default stream).
 * FTCG_EUNSUPPORTED when the workspace exceeds the array: in 2D,
 * n * G * (8 for FTCG_F32, 16 for FTCG_F64) bytes plus the tables must fit
 * 36 MiB (float32: n <= 1024 at oversampling 2; float64: n <= 1024 with
 * 32 MiB). Results equal ftcg_grid_to_image's bit for bit. Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU race.
 * Enqueues only. */
ftcg_status ftcg_grid_to_image_noalloc(int dim, int64_t n, int half_width, double oversampling,
                                       ftcg_dtype dtype, const void* grid_dev, void* image_dev,
                                       void* hip_stream);

/* Plan properties: G per axis, number of spread records after halo
 * duplication, number of tiles, tile edge. Any output pointer may be NULL. */
ftcg_status ftcg_plan_info(ftcg_plan plan, int64_t* grid_size, int64_t* n_records,
                           int64_t* n_tiles, int* tile);

/* Tile accumulation of the spreading step (Omega D fhat of eq:cgmatrix).
 *   FTCG_ACCUM_FIXED : float32 plans only (their default). Taps are scaled by a
 *                      per-tile bound, rounded to the nearest integer and
 *                      accumulated exactly as packed int32 (re, im) pairs with
 *                      one 64-bit LDS integer add per tap; results are bitwise
 *                      reproducible, error <= half of 2^-31 of the tile bound
 *                      per tap (unbiased).
 *   FTCG_ACCUM_F64   : taps accumulated with float64 LDS atomics (the default
 *                      and only mode of float64 plans); lds_copies > 1 gives
 *                      each wavefront its own partial tile, combined at the
 *                      flush with compensated (TwoSum) addition. */
typedef FTCG_ENUM { FTCG_ACCUM_FIXED = 0, FTCG_ACCUM_F64 = 1 } ftcg_accum;

/* Tuning knobs (take effect at the next ftcg_set_points; the points must be
 * set again):
 *   tile       : tile edge in grid cells (16, 32, 64, 128; 0 = automatic:
 *                32 in 2D, min(G, 1024) in 1D);
 *                FTCG_ACCUM_F64 supports tile <= 64 and
 *                lds_copies * 16 * tile * (tile + 1) <= 160 KiB.
 *   accum      : ftcg_accum (FTCG_ACCUM_FIXED needs a float32 plan).
 *   lds_copies : 1, 2 or 4 (FTCG_ACCUM_F64 only; must be 1 otherwise).
 * Returns FTCG_EUNSUPPORTED for combinations that do not fit LDS and
 * FTCG_EINVAL for values outside these sets. */
ftcg_status ftcg_plan_set_tuning(ftcg_plan plan, int tile, int accum, int lds_copies);

/* Work layout of the float32 fixed-point spread (Sec. III-A eq:cgmatrix, the
 * product Omega D fhat), taking effect at the next execute:
 *   FTCG_SPREAD_AUTO  (the default): on 2D grids with tile 32 and enough tiles
 *                     (G >= 4096 at sigma = 2), one workgroup walks a segment
 *                     of 2 tile columns by 4 or 8 tile rows and uses each
 *                     sample once per segment it reaches; otherwise one
 *                     workgroup per tile;
 *   FTCG_SPREAD_TILES : one workgroup per tile on every grid.
 * Both accumulate the same exact fixed-point taps; they differ by the float
 * rounding of the carried rows between the segment's steps and by each
 * step's quantum (under 1e-6 relative on the SAS workloads).
 * FTCG_EINVAL for other values. */
typedef enum { FTCG_SPREAD_AUTO = 0, FTCG_SPREAD_TILES = 1 } ftcg_spread_layout;
ftcg_status ftcg_plan_set_spread_layout(ftcg_plan plan, int layout);

/* Launch shape of the frame-weight sum (Sec. III-C, eq:difopt), taking effect
 * at the next weight computation:
 *   samples_per_lane : 1, 2 or 4 consecutive bin-sorted samples share each
 *                      lane's candidate reads (0 = automatic: 2 in 2D from
 *                      2^20 samples unless a sample has more than about
 *                      10^4 candidate neighbours, else 1; 4 uses the
 *                      one-sided sum);
 *   lanes_per_group  : 1, 2 or 4 lanes split every candidate range of a group
 *                      of samples and add their partial sums (2D only;
 *                      0 = automatic: 1 when a sample has more than about
 *                      10^4 candidate neighbours, else 4 below 2^21 samples
 *                      and 2 above).
 * Results agree to rounding for every shape. FTCG_EINVAL for other values. */
ftcg_status ftcg_plan_set_weight_tuning(ftcg_plan plan, int samples_per_lane, int lanes_per_group);

/* Per-step timing with HIP events on the plan's stream.
 * enable != 0 records events around every step of later calls; ftcg_plan_timing
 * synchronises the stream and returns, for each step s in
 * {0 input check + tile binning, 1 frame-weight sum kernel (alone),
 *  2 spread, 3 fft pass 1, 4 fft pass 2 + deapodize + crop, 5 neighbour binning
 *  for weights, 6 learned-weight inference, 7 learned-weight audit,
 *  8 weights from the sums (and the sums' preset), 9 banded C: band of T^2,
 *  10 banded C: normal equations, 11 banded C: c = C fhat,
 *  12 forward transform: FFT passes, 13 forward transform: interpolation,
 *  14 iterative density compensation, 15 dense frame approximation},
 * the summed milliseconds ms[s] and the number of timed intervals count[s]
 * (host arrays of FTCG_TIMING_STEPS entries; unused entries are 0), then
 * resets the sums. A step can be timed in several intervals per call (step 0:
 * the input check, then the binning after the host has read the check's
 * result; the host's wait in between is in no step). */
#define FTCG_TIMING_STEPS 16
ftcg_status ftcg_plan_enable_timing(ftcg_plan plan, int enable);
ftcg_status ftcg_plan_timing(ftcg_plan plan, double* ms, int64_t* count);

/* ------------------------------------------------------------------------
 * Learned frame weights (FTCG_W_LEARNED). Not in the paper: a small network
 * predicts the frame-optimal weight of eq:difopt from the local raster
 * geometry, and the plain float64 weights remain the fallback and the measure
 * of its error.
 *   feature of sample j : offsets k_i - k_j (float32, nearest first) of the 16
 *                         nearest other samples within ||k_i - k_j||_inf <= R,
 *                         ranked by float32 squared distance, ties by the
 *                         smaller index; missing neighbours are (R, R);
 *   base_j              : 1 / (1 + sum over the 16 of sinc^2(dx) sinc^2(dy));
 *   network             : y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3, SiLU s,
 *                         widths 32 -> 64 -> 64 -> 1; inference in half
 *                         precision weights/activations, float32 accumulation;
 *   weight              : alpha_hat_j = base_j exp(y_j);
 *   training target     : log(alpha_j / base_j), mean squared error, Adam on
 *                         float32 master weights.
 * Parameter vector (FTCG_MLP_NPARAM floats, host order): W1 [32][64]
 * row-major, b1 [64], W2 [64][64] row-major, b2 [64], W3 [64], b3 [1].
 * ------------------------------------------------------------------------ */
#define FTCG_MLP_NPARAM 6337

typedef struct ftcg_mlp_s* ftcg_mlp;

/* Create / destroy a network (parameters zero until set or loaded). */
ftcg_status ftcg_mlp_create(ftcg_mlp* out, void* hip_stream);
ftcg_status ftcg_mlp_destroy(ftcg_mlp mlp);

/* Host parameter vectors of FTCG_MLP_NPARAM floats (n must equal it).
 * Setting parameters resets the Adam state. Both calls synchronise. */
ftcg_status ftcg_mlp_set_params(ftcg_mlp mlp, const float* params_host, int64_t n);
ftcg_status ftcg_mlp_get_params(ftcg_mlp mlp, float* params_host, int64_t n);

/* Serialise parameters + Adam state (little-endian, versioned header).
 * blob_host == NULL: *bytes receives the size needed. */
ftcg_status ftcg_mlp_save(ftcg_mlp mlp, void* blob_host, size_t* bytes);
ftcg_status ftcg_mlp_load(ftcg_mlp mlp, const void* blob_host, size_t bytes);

/* Features (m x 32 float32, device) and base (m float64, device) of a 2D
 * raster k_dev (m x 2 float64, device); with target_dev != NULL also the
 * training target log(alpha / base) (m float32) from the plain weights. */
ftcg_status ftcg_mlp_features(ftcg_mlp mlp, int64_t m, const double* k_dev, double R, float* feat_dev,
                              double* base_dev, float* target_dev);

/* Network output y for n feature rows (inference kernel, half precision). */
ftcg_status ftcg_mlp_forward(ftcg_mlp mlp, int64_t n, const float* feat_dev, float* y_dev);

/* Gradient (FTCG_MLP_NPARAM floats, device) and loss (host) of the mean
 * squared error over n rows; fp16 != 0 rounds weights and activations to half
 * in the forward pass as inference does. Does not change the parameters. */
ftcg_status ftcg_mlp_loss_grad(ftcg_mlp mlp, int64_t n, const float* feat_dev, const float* target_dev,
                               int fp16, float* grad_dev, double* loss_host);

/* One Adam step (learning rate lr) on the mean squared error of n rows. */
ftcg_status ftcg_mlp_train_batch(ftcg_mlp mlp, int64_t n, const float* feat_dev, const float* target_dev,
                                 int fp16, float lr, double* loss_host);

/* Train on one raster: plain weights and features on the GPU, then Adam
 * steps over minibatches of `batch` samples (sample j in minibatch j mod
 * ceil(m / batch)). loss_host receives the mean loss over the raster. */
ftcg_status ftcg_mlp_train_raster(ftcg_mlp mlp, int64_t m, const double* k_dev, double R, int64_t batch,
                                  float lr, int fp16, double* loss_host);

/* Attach a network to a FTCG_W_LEARNED plan (the plan keeps the pointer; the
 * network must outlive it). At each ftcg_set_points the plan predicts all
 * weights, recomputes the plain weights of audit_samples evenly spaced
 * samples (caller indices floor(q m / n)), and falls back to the plain
 * weights of every sample when the relative RMS difference exceeds
 * audit_threshold (the estimated relative L2 error of the image for values
 * of equal magnitude). */
ftcg_status ftcg_plan_set_mlp(ftcg_plan plan, ftcg_mlp mlp, double audit_threshold, int64_t audit_samples);

/* Estimate of the last audit and whether the plan fell back (host outputs). */
ftcg_status ftcg_plan_learned_report(ftcg_plan plan, double* audit_estimate, int* used_fallback);

/* ------------------------------------------------------------------------
 * Batched execution: n_items independent reconstructions (pings or
 * sub-swaths) with their own sample counts and image sizes, float32,
 * kernel/oversampling/weight mode shared. Spreading of all items runs as ONE
 * persistent launch over a queue of (tile, record chunk) tasks ordered
 * heaviest first; the FFT passes run batched per grid size; ftcg_batch_execute
 * replays a captured hipGraph of the whole sequence.
 * Concatenation: item i's samples follow those of items 0..i-1 in k_dev
 * (m_i x 2 float64), fhat_dev (complex64) and alpha_dev (float64); its image
 * (n_i x n_i complex64, row-major) follows the images of items 0..i-1.
 * ------------------------------------------------------------------------ */
typedef struct ftcg_batch_s* ftcg_batch;

ftcg_status ftcg_batch_create(ftcg_batch* out, int n_items, const int64_t* n_host, int half_width,
                              double oversampling, ftcg_wmode wmode, double weight_radius, void* hip_stream);
ftcg_status ftcg_batch_destroy(ftcg_batch batch);

/* tile edge (16/32/64/128, default 32), records per task (>= 64, default
 * 4096), workgroups of the persistent launch (default 8 per CU), graph replay
 * on/off (default on). The points must be set again afterwards. */
ftcg_status ftcg_batch_set_tuning(ftcg_batch batch, int tile, int64_t chunk_records, int persistent_blocks,
                                  int use_graph);

/* FTCG_W_LEARNED batches: the network and audit of every item (see ftcg_plan_set_mlp). */
ftcg_status ftcg_batch_set_mlp(ftcg_batch batch, ftcg_mlp mlp, double audit_threshold, int64_t audit_samples);

/* m_host: n_items sample counts (host); k_dev: concatenated locations (device).
 * Synchronises the stream (task tables are built on the host). */
ftcg_status ftcg_batch_set_points(ftcg_batch batch, const int64_t* m_host, const double* k_dev);
ftcg_status ftcg_batch_set_weights(ftcg_batch batch, const double* alpha_dev);   /* FTCG_W_USER */
ftcg_status ftcg_batch_get_weights(ftcg_batch batch, double* alpha_dev);
ftcg_status ftcg_batch_execute(ftcg_batch batch, const void* fhat_dev, void* images_dev);

/* tasks of the persistent launch, tiles split over several tasks, spread
 * records and tiles over all items (host outputs, any may be NULL) */
ftcg_status ftcg_batch_info(ftcg_batch batch, int64_t* n_tasks, int64_t* n_split_tiles, int64_t* n_records,
                            int64_t* n_tiles);
ftcg_status ftcg_batch_enable_timing(ftcg_batch batch, int enable);

#ifdef __cplusplus
}
#endif

#endif /* FTCG_H */
