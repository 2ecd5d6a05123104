/*
 * libsgl -- fast spherical Gauss-Laguerre (SGL) Fourier transforms on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Prestin & Wuelker, "Fast Fourier Transforms for Spherical
 * Gauss-Laguerre Basis Functions" (arXiv:1604.05140).
 *
 *   Forward (FSGLFT, Alg. 3): samples of a function with bandlimit B on the
 *   grid of the SGL sampling theorem (Thm. 3.4) -> coefficients fhat_nlm,
 *   |m| <= l < n <= B, equal to the quadrature sum
 *       fhat_nlm = sum_{i,j,k<2B} a_i r_i^2 b~_j f(r_i,th_j,ph_k) conj(H_nlm(r_i,th_j,ph_k)).
 *   Inverse (iFSGLFT, Alg. 4): coefficients -> samples
 *       f(r_i,th_j,ph_k) = sum_{nlm} fhat_nlm H_nlm(r_i,th_j,ph_k).
 *   Both are computed in O(B^4) by separation of variables (Sect. 3.3):
 *   an FFT over the azimuth of every (r_i, th_j) ring, a Legendre projection
 *   per order m (Eq. DLT), and a radial projection per degree l (Eq. DRT).
 *
 * Grid (Thm. 3.4): r_i, a_i = nodes and weights of the 2B-point half-range
 * Gauss-Hermite rule (Thm. 3.3); th_j = (2j+1) pi / (4B), ph_k = k pi / B
 * (Thm. 3.1), j, k < 2B.  The polar weight is b~_j = (pi/B) b_j with b_j as
 * printed in Thm. 3.1: the printed b_j sum to 2 over j, and the double sum
 * over (j, k) needs the azimuthal step pi/B as well.
 *
 * Layouts (Sect. 3.4), all complex values interleaved (re, im):
 *   samples      f[psi],    psi   = 4B^2 i + 2B j + k          (8 B^3 values)
 *   coefficients fhat[omega], omega = n(n-1)(2n-1)/6 + l(l+1) + m (B(B+1)(2B+1)/6 values)
 *   a batch of functions is stored back to back (function b at b * count).
 *
 * Sample scaling.  By default samples are "scaled": s_ijk = sigma_i f(r_i,
 * th_j, ph_k) with sigma_i = sqrt(a_i) r_i.  The forward map then reads
 * fhat_nlm = sum b~_j s_ijk conj(sigma_i H_nlm), the inverse writes s.  This is
 * the paper's exp(r^2) weight compensation (Sect. 3.2, Sect. 5) carried to
 * both sides: raw samples grow like 10^B at the outer radii and leave the FP32
 * range for B > ~40, scaled samples stay below 1 in magnitude.  With
 * SGL_SAMPLES_RAW (FP64 plans only) the library takes and returns raw f.
 *
 * Precision (dtype):
 *   SGL_F64         complex128 samples/coefficients; every stage in FP64
 *                   (stages (b), (c) on FP64 MFMA).
 *   SGL_F32         complex64; FFT in FP32; stages (b), (c) on FP32 MFMA.
 *   SGL_SPLIT_BF16  complex64; FFT in FP32; stages (b), (c) as three-piece
 *                   bfloat16 splits of both operands, the six products of
 *                   order <= 2 on bf16 MFMA, accumulated in FP32.
 *   Quadrature nodes/weights and the Legendre/radial basis tables are always
 *   computed on the GPU in FP64 (three-term recurrences) and rounded once.
 *
 * Conventions.
 *   - The caller allocates and owns every sample/coefficient buffer (device
 *     memory); the plan owns its tables, workspace and streams.
 *   - Calls taking a stream are stream-ordered and asynchronous: they enqueue
 *     kernels and return; they never allocate, free or synchronize.  Plans
 *     are not thread-safe: one plan must not run two calls at once (its
 *     workspace is shared by forward and inverse).
 *   - Input buffers are never written.  Input and output must not overlap
 *     (SGL_ERR_INVALID_ARG).
 *   - Errors are returned as status codes; sgl_last_error() gives a message.
 *     Plan creation is all-or-nothing: on failure *out is NULL and nothing
 *     is leaked.
 */
#ifndef SGL_H
#define SGL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgl_plan_s* sgl_plan_t;

typedef enum {
  SGL_OK = 0,
  SGL_ERR_INVALID_ARG = 1, /* bad size, null pointer, aliasing, unknown flag   */
  SGL_ERR_UNSUPPORTED = 2, /* valid request the library does not support       */
  SGL_ERR_HIP = 3,         /* a HIP runtime call failed (see sgl_last_error)  */
  SGL_ERR_OOM = 4,         /* device allocation failed                         */
  SGL_ERR_NUMERIC = 5      /* plan-time FP64 quadrature failed a self-check    */
} sgl_status_t;

typedef enum { SGL_F64 = 0, SGL_F32 = 1, SGL_SPLIT_BF16 = 2 } sgl_dtype_t;

/* plan flags */
#define SGL_SAMPLES_RAW 1u /* raw f instead of sigma_i f (SGL_F64 only) */
#define SGL_GRAPHS 2u      /* replay each direction as a hipGraph: the first call with a
                              new (input, output) buffer pair captures and instantiates
                              it (host-side work only); later calls launch the graph.
                              Up to 8 pairs are kept (least recently used evicted). */
#define SGL_AUTOTUNE 4u    /* at plan time, time each stage launch with several
                              persistent grid sizes on scratch buffers and keep the
                              fastest (plan creation takes longer) */
#define SGL_SEMINAIVE 8u   /* seminaive Legendre step (Sect. 3.3.1, Eq. DCT, Eq.
                              dct_trick): per order m the weighted polar data go
                              through the orthonormal DCT of length 2B (an FFT of
                              length 4B per spectrum column; odd orders first take
                              a sin(theta_j) factor), then the contraction runs
                              over the cosine indices k < B with the precomputed
                              cosine-domain Legendre table (zero beyond the degree
                              l - (m mod 2)); the inverse is the transpose (the
                              contraction, then the inverse DCT).  Same results as
                              the direct sums up to rounding.  Power-of-two
                              bandlimits 8..256 only, and 8..128 in SGL_SPLIT_BF16
                              (SGL_ERR_UNSUPPORTED otherwise). */

#define SGL_MAX_B 256 /* largest supported bandlimit */

/* Create a plan for `batch` functions of bandlimit B (1 <= B <= SGL_MAX_B,
 * batch >= 1) in precision `dtype` (an sgl_dtype_t).  Builds, on the current
 * HIP device, the FP64 grid (Thm. 3.1, Thm. 3.3), the basis tables (Eq.
 * legendre_recurrence, Lemma 3.5) and the workspace; synchronizes before
 * returning.  *out receives the plan (NULL on failure). */
sgl_status_t sgl_plan(sgl_plan_t* out, int B, int batch, int dtype);

/* Like sgl_plan for nfunc functions with their own bandlimits B_list[f]
 * (host array).  Functions are packed back to back in the caller's buffers
 * at the offsets reported by sgl_offsets.  Functions of equal bandlimit share
 * tables; every stage runs as one persistent launch over a work list keyed by
 * (order, bandlimit).  flags: any of SGL_SAMPLES_RAW, SGL_GRAPHS, SGL_AUTOTUNE,
 * SGL_SEMINAIVE. */
sgl_status_t sgl_plan_ex(sgl_plan_t* out, const int* B_list, int nfunc, int dtype, unsigned flags);

/* Like sgl_plan_ex for the radially scaled basis of scale s = radial_scale > 0
 * (the radially scaled SGL functions named in Sect. 5):
 *     H^s_nlm(x) = s^(-3/2) H_nlm(x / s),
 * orthonormal for the weight exp(-|x|^2 / s^2).  Samples are taken at the radii
 * s r_i (same theta_j, phi_k); the scaled-sample convention keeps the sigma_i of
 * the unit rule (scaled samples sigma_i f(s r_i, th_j, ph_k); SGL_SAMPLES_RAW:
 * f(s r_i, th_j, ph_k)).  By the substitution x = s y the transform is the unit
 * transform with forward coefficients times s^(3/2) (inverse inputs divided by
 * it); the factor is folded into the packed radial tables at plan time, so the
 * kernels and their cost are those of s = 1.  sgl_grid returns the radii s r_i;
 * its log_a, log_sigma and sgl_table stay those of the unit rule.
 * SGL_ERR_INVALID_ARG for s <= 0 or non-finite s. */
sgl_status_t sgl_plan_scaled(sgl_plan_t* out, const int* B_list, int nfunc, int dtype, unsigned flags,
                             double radial_scale);

/* The persistent grid (blocks) of each of the SGL_NUM_SLOTS launch slots, in
 * order: forward FFT of power-of-two rings up to 256 points (and other
 * lengths outside the two Bluestein families), forward FFT of 512-point rings
 * and of Bluestein rings padded to 512, forward FFT of Bluestein rings padded
 * to <= 256, forward Legendre, forward radial, inverse radial, inverse
 * Legendre, then the three inverse FFT slots in the forward order.  A slot
 * with no work reports 0.  grids: host array of SGL_NUM_SLOTS ints. */
#define SGL_NUM_SLOTS 10
sgl_status_t sgl_launch_grids(sgl_plan_t plan, int* grids);

/* Tile of each launch slot's contraction kernel (slot order as in
 * sgl_launch_grids).  tiles: host array of 2 * SGL_NUM_SLOTS ints; receives, per
 * slot, the rows and complex columns of one work item's output tile (0, 0 for
 * the FFT slots).  The stage (b)/(c) slots of the register-staged MFMA GEMM (all
 * of stage (c), and stage (b) in SGL_F64 and SGL_F32) have two tile geometries:
 *   geometry 0: 128 rows x 64 complex columns, 8 wavefronts (the default),
 *   geometry 1:  64 rows x 32 complex columns, 4 wavefronts,
 * and the forward radial slot of SGL_SPLIT_BF16 and SGL_F32 and both Legendre
 * slots of SGL_F32 a third,
 *   geometry 2: 128 rows x 128 complex columns on a copy-fed kernel
 *               (operands by global -> LDS copies, 16 wavefronts);
 * SGL_AUTOTUNE times each (with each persistent grid) and keeps the fastest.
 * The split-form Legendre kernel has one tile, 128 rows x 128 complex columns. */
sgl_status_t sgl_launch_tiles(sgl_plan_t plan, int* tiles);

/* Select the tile geometry (0, 1 or 2, see sgl_launch_tiles) of one launch slot.
 * SGL_ERR_UNSUPPORTED for a geometry the slot does not have; SGL_ERR_INVALID_ARG
 * for a slot outside [0, SGL_NUM_SLOTS).  The slot keeps its persistent-grid
 * bound; graphs the plan captured earlier are dropped (the next call with each
 * buffer pair captures again).  Not to be called while the plan runs a call. */
sgl_status_t sgl_set_launch_tile(sgl_plan_t plan, int slot, int geometry);

/* Forward transform (Alg. 3) of every function of the plan.
 * d_samples: device, const, total_samples complex values (complex128 for
 *            SGL_F64, complex64 otherwise), psi order per function.
 * d_coeffs:  device, written, total_coeffs complex values, omega order.
 * stream:    hipStream_t (NULL = default stream). */
sgl_status_t sgl_forward(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): sgl_forward with the
 * stage intermediates (the spectrum F and the Legendre output g) placed in a
 * static device array of 64 MiB that the library holds on each GPU it runs on
 * until the process ends, instead of the plan's own workspace.  Same arguments,
 * layouts and results as sgl_forward; makes no allocation (no hipMalloc, no
 * allocating library call), launches the stage kernels eagerly (never as a graph)
 * and never synchronizes.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents: calls that may overlap on one GPU (different
 * streams or threads without ordering) race and give wrong results; calls
 * ordered on one stream are safe.  SGL_ERR_INVALID_ARG when the plan's F and g
 * together exceed 64 MiB (e.g. B = 64 with one complex128 function fits: 42 MB;
 * B = 128 does not) or when the current device is not the plan's. */
sgl_status_t sgl_forward_noalloc(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream);

/* Inverse transform (Alg. 4): d_coeffs (const) -> d_samples (written). */
sgl_status_t sgl_inverse(sgl_plan_t plan, const void* d_coeffs, void* d_samples, void* stream);

/* The naive transforms (Alg. 1 forward, Alg. 2 inverse) of every function of
 * an SGL_F64 plan, same buffers and layouts as sgl_forward / sgl_inverse:
 * every coefficient is the full quadrature sum over all (2B)^3 grid points
 * and every sample the full synthesis sum over all coefficients, in FP64, with
 * basis values from the plan's FP64 tables (O(B^6) work per function; meant
 * for B <= 64).  SGL_ERR_UNSUPPORTED for other precisions.  Stream-ordered,
 * no allocation, no synchronization; honours SGL_SAMPLES_RAW. */
sgl_status_t sgl_naive_forward(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream);
sgl_status_t sgl_naive_inverse(sgl_plan_t plan, const void* d_coeffs, void* d_samples, void* stream);

/* Cartesian midpoint-rule projection (Sect. 5: the field's practice, an
 * accuracy foil for the sampling-theorem transforms) of every function of an
 * SGL_F64 plan:
 *     fhat_nlm ~ dV sum_c f(x_c) conj(H_nlm(x_c)) exp(-|x_c|^2)
 * (weight of the SGL inner product; radially scaled plans use H^s and
 * exp(-|x|^2/s^2)).  The grid has nx cells per axis on [-h, h]^3, h =
 * half_width, cell side d = 2h/nx, dV = d^3, midpoints -h + (i + 1/2) d.
 * d_values: device, const, nfunc * nx^3 complex128, function f at f * nx^3,
 * cell (ix, iy, iz) at (ix nx + iy) nx + iz.  d_coeffs: the plan's coefficient
 * layout, written.  Basis values come from the three-term recurrences per cell
 * in FP64 (O(nx^3 B^3) work per function).  SGL_ERR_INVALID_ARG for nx outside
 * [1, 1024] or a non-positive half width; SGL_ERR_UNSUPPORTED unless SGL_F64. */
sgl_status_t sgl_midpoint_forward(sgl_plan_t plan, const void* d_values, int nx, double half_width, void* d_coeffs,
                                  void* stream);

/* Synthesis at arbitrary points: values[f * npts + p] = sum_nlm fhat_nlm H_nlm(x_p)
 * for every function f of an SGL_F64 plan (H^s for radially scaled plans).
 * d_coeffs: the plan's layout (const); d_xyz: device, const, npts x 3 doubles
 * (x, y, z), shared by all functions; d_values: device, nfunc * npts complex128,
 * written.  FP64 recurrences per point; SGL_ERR_UNSUPPORTED unless SGL_F64. */
sgl_status_t sgl_synthesize_points(sgl_plan_t plan, const void* d_coeffs, int npts, const double* d_xyz,
                                   void* d_values, void* stream);

/* Free everything the plan owns (NULL is accepted). */
sgl_status_t sgl_plan_destroy(sgl_plan_t plan);

/* Sizes and index map (Sect. 3.4).  Return -1 for out-of-range arguments. */
int64_t sgl_num_samples(int B);             /* 8 B^3 */
int64_t sgl_num_coeffs(int B);              /* B(B+1)(2B+1)/6 */
int64_t sgl_coeff_index(int n, int l, int m); /* omega(n,l,m), needs |m| <= l < n */

/* Plan totals: complex values in the sample/coefficient buffers and the number
 * of functions.  Any pointer may be NULL. */
sgl_status_t sgl_plan_info(sgl_plan_t plan, int64_t* total_samples, int64_t* total_coeffs, int* nfunc);

/* Host arrays of nfunc entries: complex-value offsets of each function in the
 * sample and coefficient buffers (either may be NULL). */
sgl_status_t sgl_offsets(sgl_plan_t plan, int64_t* sample_off, int64_t* coeff_off);

/* Copy the plan's FP64 grid for bandlimit B (which the plan must contain)
 * into host arrays (any may be NULL): r, ln a, ln sigma (length 2B) from the
 * radial rule of order 2B; theta, b~ (length 2B). */
sgl_status_t sgl_grid(sgl_plan_t plan, int B, double* r, double* log_a, double* log_sigma,
                      double* theta, double* btilde);

/* Copy one FP64 basis table for bandlimit B into a host array of B^2 (B+1)
 * doubles.  which = 0: Legendre table, for m = 0..B-1 the (B-m) x 2B block
 * Pbar_lm(cos th_j), rows l = m..B-1, block offset 2B (m B - m(m-1)/2).
 * which = 1: radial table, for l = 0..B-1 the (B-l) x 2B block
 * rho_nl(r_i) = sigma_i N_nl R_nl(r_i), rows n = l+1..B, same offsets.
 * which = 2 (SGL_SEMINAIVE plans): cosine-domain Legendre table, B^2 (B+1) / 2
 * doubles, for m = 0..B-1 the (B-m) x B block [C_2B q_lm]_k, k < B, with
 * q_lm = Pbar_lm / sin^(m mod 2) theta (Eq. DCT), rows l = m..B-1, block
 * offset B (m B - m(m-1)/2); entries beyond k = l - (m mod 2) are zero. */
sgl_status_t sgl_table(sgl_plan_t plan, int B, int which, double* host_out);

/* Per-stage kernel timing with HIP events recorded on the caller's stream.
 * While enabled every forward/inverse call records events around its stage
 * launches; sgl_stage_times accumulates them (synchronizing on the events)
 * into ms[6] (forward a, b, c, inverse c, b, a) and counts[6], then resets. */
sgl_status_t sgl_set_timing(sgl_plan_t plan, int enable);
sgl_status_t sgl_stage_times(sgl_plan_t plan, double* ms, int* counts);

/* Run the GEMM core of stages (b)/(c) once on device buffers, for tests:
 * C[M x N] = A[M x K] * X[K x N], all FP64 row-major, in precision dtype
 * (inputs rounded/split on the fly).  Synchronizes. */
sgl_status_t sgl_debug_gemm(int dtype, int M, int N, int K, const double* d_A, const double* d_X, double* d_C);

const char* sgl_status_string(sgl_status_t status);
const char* sgl_last_error(void); /* message of the last failing call on this thread */

#ifdef __cplusplus
}
#endif

#endif /* SGL_H */
