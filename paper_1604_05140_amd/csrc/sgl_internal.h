// Internal definitions shared by the libsgl translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sgl.h"

namespace sgl {

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

// Every device allocation the library makes goes through dev_malloc.  For the
// tests of all-or-nothing plan creation, the environment variable
// SGL_TEST_FAIL_ALLOC=k (read when a plan creation starts) makes the k-th
// device allocation of that creation fail as hipMalloc does when memory runs
// out (no device call is made for it); unset or 0, nothing is injected.
hipError_t dev_malloc(void** p, size_t bytes);

#define SGL_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::sgl::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return e_ == hipErrorOutOfMemory ? SGL_ERR_OOM : SGL_ERR_HIP;                \
    }                                                                              \
  } while (0)

// ---------------------------------------------------------------------------
// Global-memory views of device pointers.  A pointer read from a descriptor
// is generic to the compiler, which then emits flat memory instructions; those
// also count in the LDS wait counter, so every wait for an LDS access (each
// MFMA operand read, each barrier) would wait for all HBM loads and stores in
// flight as well, and no prefetch could overlap compute.  Accesses through
// these views compile to global instructions (vector-memory counter only).
// The cast changes no bits: global and generic addresses coincide.  The host
// pass, which only type-checks device code, sees plain pointers.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
#define SGL_G __attribute__((address_space(1)))
#else
#define SGL_G
#endif
template <typename T>
__device__ inline SGL_G T* gmem(T* p) {
  return (SGL_G T*)p;
}

// ---------------------------------------------------------------------------
// Sizes and table offsets
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t num_coeffs(int B) { return (int64_t)B * (B + 1) * (2 * B + 1) / 6; }
__host__ __device__ inline int64_t num_samples(int B) { return 8ll * B * B * B; }
__host__ __device__ inline int64_t omega(int n, int l, int m) {
  return (int64_t)n * (n - 1) * (2 * n - 1) / 6 + (int64_t)l * (l + 1) + m;
}
// Offset (in elements) of block q (order m for the Legendre table, degree l for
// the radial table) in a table of blocks (B-q) x 2B, q = 0..B-1.
__host__ __device__ inline int64_t table_block(int B, int q) {
  return 2ll * B * ((int64_t)q * B - (int64_t)q * (q - 1) / 2);
}
__host__ __device__ inline int64_t table_size(int B) { return (int64_t)B * B * (B + 1); }
// Functions per bandlimit class: the spectrum workspace (2B-1) (2B)^2 nf, the
// largest per-class buffer, stays below 2^31 complex values.
inline int class_capacity(int B) {
  const int64_t per = (int64_t)(2 * B - 1) * 4 * B * B;
  const int64_t cap = ((int64_t(1) << 31) - 1) / per;
  return (int)(cap < 1 ? 1 : (cap > (1 << 20) ? (1 << 20) : cap));
}

// ---------------------------------------------------------------------------
// Device-side description of one bandlimit class (all functions sharing B)
// ---------------------------------------------------------------------------
constexpr int kMaxRadices = 12;

struct ClassDesc {
  int B;            // bandlimit
  int nf;           // functions in the class
  int L;            // 2B, ring length
  int nrad;         // FFT radix count
  int rad[kMaxRadices];
  const int64_t* soff;  // per-function sample offsets (complex values)
  const int64_t* coff;  // per-function coefficient offsets (complex values)
  // Packed table operands in the plan precision, one per contraction:
  // 0 Legendre forward (rows l, k = j), 1 Legendre inverse (rows j, k = l),
  // 2 radial forward (rows n, k = i), 3 radial inverse (rows i, k = n).
  // Block q (order m or degree l) is row-major with the contraction length
  // padded to a multiple of the GEMM K chunk (zeros); split tables hold 3 bf16 planes of
  // Aplane elements each.
  const void* A[4];
  const int64_t* Aoff[4];  // element offset of block q
  int64_t Aplane[4];
  const double* btilde; // b~_j, 2B
  const double* sigma;  // sigma_i, 2B (raw-sample scaling)
  const void* tw;       // twiddles exp(-2 pi i q / L), q < L (double2 or float2)
  // Bluestein rings (lengths other than powers of two, 6 <= L <= 256): M is the
  // power-of-two convolution length >= 2L - 1 (0 if unused), chirp[p] =
  // exp(-i pi p^2 / L) (p < L), bhf / bhi the spectra of the forward / inverse
  // chirp kernels divided by M (M values), twM the M-point twiddles.
  int M;
  const void* chirp;
  const void* bhf;
  const void* bhi;
  const void* twM;
  void* F;              // stage (a)/(b) workspace, [(2B-1)][2B][nf*2B] complex
  void* g;              // stage (b)/(c) workspace, [l][b][m+l][2B] complex, block l at l^2 nf 2B
  // FP64 master tables (Legendre blocks by order, radial blocks by degree)
  const double* P64;
  const double* R64;
  // naive forward transform: prefix over l of (2l+1) ceil((B-l)/naive_group()), B+1 entries
  const int* naive_loff;
  // radially scaled basis: its scale s and the coefficient factors s^(3/2)
  // (forward) and s^(-3/2) (inverse) used by the naive and off-grid kernels
  // (the packed radial tables carry them for the fast path)
  double rscale, rs_fwd, rs_inv;
  const int* fid;  // plan-wide function index of each function of the class
  // Legendre contraction length on the polar side: 2B (direct sums over j) or B
  // (seminaive step: cosine-domain sums over k < B, Sect. 3.3.1)
  int kb;
  const void* dct;  // DCT constants of the seminaive step (dct_const_count(B) complex), else null
  // coefficient offsets in closed form: coff[b] = cbase + b * cstep when the
  // class's functions are stored one after another (cstep = the coefficient
  // count of B); cstep = 0 when coff must be read
  int64_t cbase, cstep;
};
// naive / midpoint forward items group this many consecutive degrees n
constexpr int kNaiveGroup = 8;

// Work items (int4): stage a {class, j, col block, 0}; stage b {class, m, row tile, col tile};
// stage c {class, l, row tile, col tile}.

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_SPLIT = 2 };

// Stage kernels (defined in sgl_fft.hip / sgl_gemm.hip)
// stage (a) work items carry the rings per block in .w; lds_bytes is the largest
// fft_lds_bytes_for over the rings of the launch
// Stage (a) runs as up to three kernels by ring-length family (mode 0: power-of-two
// rings up to 256 points and the generic path; mode 1: one-wavefront 512-point
// FFTs, i.e. 512-point rings and Bluestein length 512; mode 2: Bluestein with M <= 256)
// so that each gets only the registers its FFT size needs.  max_grid bounds the
// persistent grid (0 = the default bound).
hipError_t launch_fft_forward(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, int mode, const void* samples, int max_grid, hipStream_t s);
hipError_t launch_fft_inverse(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, int mode, void* samples, int max_grid, hipStream_t s);
void prepare_fft_kernels(const int* lds_per_mode);
size_t fft_lds_bytes_for(int prec, int rpb, int L);
// power-of-two ring lengths 16..512 take the register FFT paths (the four-step
// FFT up to 256 points, the one-wavefront kernel at 512).
__host__ __device__ inline bool fft_pow2_path(int L) { return L >= 16 && L <= 512 && (L & (L - 1)) == 0; }
// Bluestein convolution length for ring length L (0 if L takes another path)
__host__ __device__ inline int fft_bluestein_m(int L) {
  if (fft_pow2_path(L) || L < 6 || L > 256 || (L & (L - 1)) == 0) return 0;
  int M = 16;
  while (M < 2 * L - 1) M <<= 1;
  return M;
}
inline int fft_mode(int L) {
  if (L == 512) return 1;
  const int M = fft_bluestein_m(L);
  return M == 0 ? 0 : (M == 512 ? 1 : 2);
}
// Threads per stage-(a) block: 512 for the single-precision power-of-two
// family (32 rings per block at L = 256, so spectrum rows are read and written
// in 256-byte runs), 1024 for the 512-point kernels (one wavefront per ring,
// 16 rings), 256 otherwise (FP64 power-of-two, shorter Bluestein lengths).
__host__ __device__ constexpr int fft_threads(int mode, bool f64) {
  return mode == 1 ? 1024 : (mode == 0 && !f64 ? 512 : 256);
}
// Waves per SIMD the stage-(a) kernels are compiled for: two 1024-thread
// blocks of the single-precision 512-point kernel per compute unit (LDS holds
// two), i.e. at most 64 VGPRs; the others as the compiler chooses.
__host__ __device__ constexpr int fft_min_waves(int mode, bool f64) { return mode == 1 && !f64 ? 8 : 1; }
// Rings per block of the register four-step FFT of length L = R1 R2.
inline int fft_pow2_rpb(int L, int threads) {
  int r1 = 1;
  while (r1 * r1 < L) r1 <<= 1;  // R1 = sqrt(L) or sqrt(2L)
  return threads / r1;
}
// Stage (b) / (c) launches; tg selects the tile geometry of the register-staged
// GEMM (0: 128 rows x 64 complex columns, 1: 64 x 32; see gemm_tile_m), ignored
// by the split-form Legendre kernel.  The work list must have been built for
// the same geometry.
hipError_t launch_legendre(int prec, bool inverse, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork,
                           int max_grid, hipStream_t s);
hipError_t launch_radial(int prec, bool inverse, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork,
                         const void* coeffs_in, void* coeffs_out, int max_grid, hipStream_t s);
// Naive transforms (Alg. 1, Alg. 2) of every function of an FP64 plan; d_pre
// holds the per-class prefix of work items (ncls + 1 entries).
int naive_group();
hipError_t launch_naive_forward(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                const void* samples, void* coeffs, bool raw, hipStream_t s);
hipError_t launch_naive_inverse(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                const void* coeffs, void* samples, bool raw, hipStream_t s);
// Off-grid FP64 kernels of an SGL_F64 plan: Cartesian midpoint projection
// (items as the naive forward, d_pre its per-class prefix) and synthesis at
// arbitrary points (d_pre_nf: per-class prefix of function counts).
hipError_t launch_midpoint_forward(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                   const void* values, int nx, double h, void* coeffs, hipStream_t s);
hipError_t launch_synthesize_points(const ClassDesc* d_cls, const int64_t* d_pre_nf, int ncls, int64_t nitems,
                                    const void* coeffs, int npts, const double* xyz, void* values, hipStream_t s);
hipError_t launch_debug_gemm(int prec, int M, int N, int K, const double* A, const double* X, double* C,
                             hipStream_t s);
int gemm_tile_m(int tg);                           // rows per tile of geometry tg
int gemm_tile_n_complex(int tg);                   // complex columns per tile of geometry tg
// Stage (b) slots: the split form's copy-fed kernel alone (one geometry); FP32:
// the two register-staged geometries and a third, the copy-fed FP32 kernel
// (128 x 128 tiles); FP64: the two register-staged ones.
int gemm_legendre_geometries(int prec);
int gemm_tile_m_legendre(int prec, int tg);        // tile of the stage (b) work items
int gemm_tile_n_complex_legendre(int prec, int tg);
// Stage (c) slots: the two register-staged geometries, and for the forward
// contraction of the split and FP32 forms a third, the copy-fed kernel (128 x
// 128 tiles).
constexpr int kMaxTileGeo = 3;
int gemm_radial_geometries(int prec, bool inverse);
int gemm_tile_m_radial(int tg);
int gemm_tile_n_complex_radial(int tg);
int gemm_k_chunk(int prec);  // contraction chunk (table K padding) of a precision

// Plan-time FP64 kernels (sgl_tables.hip)
struct GridBuild {
  int B;
  double* r;      // 2B
  double* log_a;  // 2B
  double* log_sig;
  double* sig;
  double* theta;
  double* btilde;
  double* sig_m;  // sigma_i = sig_m * 2^sig_e (mantissa to double-double accuracy, exponent)
  double* sig_e;
};
sgl_status_t build_grid(GridBuild& g, hipStream_t s);
hipError_t build_tables(int B, const GridBuild& g, double* P64, double* R64, hipStream_t s);
hipError_t build_twiddles(int L, void* tw, bool f32, hipStream_t s);
// FP64 Bluestein tables for ring length L and convolution length M (see ClassDesc),
// written in FP64 (f32 = false) or rounded to FP32.
hipError_t build_bluestein(int L, int M, void* chirp, void* bhf, void* bhi, bool f32, hipStream_t s);
hipError_t convert_table_f32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t convert_table_split(const double* src, uint16_t* dst, int64_t n, hipStream_t s);
// Pack an FP64 natural table (Legendre for kind 0/1, radial for kind 2/3) into the
// GEMM operand layout of `kind` in precision `prec` (see ClassDesc::A), every
// value multiplied by `scale` before rounding.
// W: grid-side row length of the source table (0: 2B; B for the cosine-domain Legendre table)
hipError_t pack_table(int B, int kind, int prec, const double* T64, const int64_t* d_offs, void* dst,
                      int64_t plane, double scale, hipStream_t s, int W = 0);
// Seminaive Legendre step: the FP64 cosine-domain Legendre table (blocks m of
// (B-m) x B) and the per-class DCT constants (see k_dct_consts; the DCT kernels
// take them in FP64 for every plan precision).
hipError_t build_cos_legendre(int B, const double* P64, double* D64, hipStream_t s);
hipError_t build_dct_consts(int B, void* out, bool f32, hipStream_t s);
__host__ __device__ inline int dct_const_count(int B) { return 2 * B + B + 2 * B; }
// DCT launches of the seminaive Legendre step (sgl_dct.hip): items {class, m + B - 1,
// column tile, columns per tile}; lds_bytes from dct_lds_bytes.
hipError_t launch_dct(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork, int lds_bytes,
                      int cols, hipStream_t s);
size_t dct_lds_bytes(int prec, int B, int cols);
void prepare_dct_kernels(int lds_bytes);

}  // namespace sgl
