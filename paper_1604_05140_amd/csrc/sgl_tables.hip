// Plan-time FP64 kernels: quadrature grid (Thm. 3.1, Thm. 3.3) and basis tables
// (Eq. legendre_recurrence, Lemma 3.5), plus rounding of the tables to the
// precision of the contraction stages.
//
// Half-range Gauss-Hermite rule of order N (Thm. 3.3).  The paper computes it
// with special recurrences in high-precision arithmetic and does not give the
// procedure; here it is computed in FP64 on the GPU:
//   1. discretize the weight exp(-r^2) dr on [0, T] by composite 32-point
//      Gauss-Legendre panels (width min(0.5, 40/N), halved repeatedly towards
//      r = 0 where the zeros of p_N crowd; T = 1.6 sqrt(N) + 8);
//   2. run the Lanczos iteration on diag(x) with the square-root weights as
//      start vector: its recurrence coefficients alpha_k, beta_k (k < N) equal
//      those of the continuous weight to rounding (the start vector is carried
//      times e^300 so that no entry underflows out to r = T);
//   3. nodes r_i = zeros of p_N: Sturm-sequence bisection on the Jacobi matrix,
//      then Newton on p_N evaluated by the three-term recurrence;
//   4. weights a_i = 1 / sum_k phat_k(r_i)^2 (orthonormal phat_k), formed in
//      log space because a_i underflows FP64 for N >~ 280.
#include <math.h>

#include "sgl_internal.h"

namespace sgl {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kGL = 32;           // Gauss-Legendre points per panel
constexpr double kStartScale = 300.0;  // ln of the start-vector scale

// ---------------------------------------------------------------------------
// S^2 grid: theta_j and b~_j = (pi/B) b_j (Thm. 3.1 with the azimuthal step)
// ---------------------------------------------------------------------------
__global__ void k_polar(int B, double* theta, double* btilde) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 2 * B) return;
  const double q = (double)(2 * j + 1) / (4.0 * B);
  theta[j] = kPi * q;
  double s = 0.0;
  for (int l = 0; l < B; ++l) s += sinpi(q * (double)(2 * l + 1)) / (double)(2 * l + 1);
  btilde[j] = (kPi / B) * sinpi(q) * (2.0 / B) * s;
}

// 32-point Gauss-Legendre rule on [-1, 1] by Newton on P_32.
__global__ void k_gauss_legendre(double* x, double* w) {
  int i = threadIdx.x;
  if (i >= kGL) return;
  const int n = kGL;
  double z = cos(kPi * (i + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) < 1e-17) break;
  }
  // recompute the derivative at the converged point
  double p0 = 1.0, p1 = z;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  dp = n * (z * p1 - p0) / (z * z - 1.0);
  x[i] = z;
  w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
}

// Discretized weight: points xs and start vector vs = sqrt(w) e^{C - x^2/2}.
__global__ void k_discretize(int npanel, const double* edges, const double* glx, const double* glw, double* xs,
                             double* vs) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npanel * kGL) return;
  int p = idx / kGL, q = idx % kGL;
  double a = edges[p], b = edges[p + 1];
  double h = b - a;
  double xx = a + (glx[q] + 1.0) * 0.5 * h;
  xs[idx] = xx;
  vs[idx] = sqrt(glw[q] * 0.5 * h) * exp(kStartScale - 0.5 * xx * xx);
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  // wave reduction then cross-wave through LDS
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < NT / 64) t = red[threadIdx.x];
  if (threadIdx.x < 64) {
    for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  }
  if (threadIdx.x == 0) red[16] = t;
  __syncthreads();
  return red[16];
}

// Lanczos on diag(xs) with start vector vs (one block).  Produces the monic
// recurrence coefficients alpha_k, beta_k (k < N), beta_0 = mu_0 = sqrt(pi)/2.
constexpr int kLanczosThreads = 1024;
__global__ void __launch_bounds__(kLanczosThreads) k_lanczos(int M, int N, const double* xs, const double* vs,
                                                             double* qa, double* qb, double* alpha,
                                                             double* beta) {
  __shared__ double red[32];
  const int t = threadIdx.x;
  double ss = 0.0;
  for (int i = t; i < M; i += kLanczosThreads) ss += vs[i] * vs[i];
  double nrm = sqrt(block_sum<kLanczosThreads>(ss, red));
  for (int i = t; i < M; i += kLanczosThreads) {
    qa[i] = vs[i] / nrm;  // q_0
    qb[i] = 0.0;          // q_{-1}
  }
  if (t == 0) beta[0] = 0.88622692545275801364908374167057259;  // sqrt(pi)/2
  __syncthreads();
  double sb = 0.0;  // sqrt(beta_k)
  double* qc = qa;
  double* qp = qb;
  for (int k = 0; k < N; ++k) {
    double part = 0.0;
    for (int i = t; i < M; i += kLanczosThreads) part += xs[i] * qc[i] * qc[i];
    const double a = block_sum<kLanczosThreads>(part, red);
    double part2 = 0.0;
    for (int i = t; i < M; i += kLanczosThreads) {
      double u = (xs[i] - a) * qc[i] - sb * qp[i];
      qp[i] = u;  // overwrite q_{k-1} with the unnormalized q_{k+1}
      part2 += u * u;
    }
    const double nb = sqrt(block_sum<kLanczosThreads>(part2, red));
    for (int i = t; i < M; i += kLanczosThreads) qp[i] /= nb;
    if (t == 0) {
      alpha[k] = a;
      if (k + 1 < N) beta[k + 1] = nb * nb;
    }
    __syncthreads();
    double* tmp = qc;
    qc = qp;
    qp = tmp;
    sb = nb;
  }
}

// Number of eigenvalues of the Jacobi matrix below x (Sturm sequence via LDL^T).
__device__ int sturm_count(int N, const double* alpha, const double* beta, double x) {
  int cnt = 0;
  double d = alpha[0] - x;
  if (d == 0.0) d = -1e-300;
  if (d < 0) ++cnt;
  for (int k = 1; k < N; ++k) {
    d = (alpha[k] - x) - beta[k] / d;
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

// One thread per node: bisection + Newton, then the Christoffel weight in log form.
__global__ void k_radial_nodes(int N, const double* alpha, const double* beta, double* r, double* log_a,
                               int* status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  // Gershgorin bound
  double hi = 0.0;
  for (int k = 0; k < N; ++k) {
    double e0 = k > 0 ? sqrt(beta[k]) : 0.0;
    double e1 = k + 1 < N ? sqrt(beta[k + 1]) : 0.0;
    hi = fmax(hi, alpha[k] + e0 + e1);
  }
  double lo = 0.0;  // the weight lives on [0, inf): all zeros are positive
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(N, alpha, beta, mid) > i)
      hi = mid;
    else
      lo = mid;
  }
  // Newton on p_N / p_N' with running rescaling (the ratio is scale free).
  double x = 0.5 * (lo + hi);
  // The Sturm count is accurate to about eps * ||J|| in absolute terms, so the
  // bisection value can be that far from the zero; Newton may move it within a
  // window that is still far below the spacing of neighbouring zeros.
  double gmax = 0.0;
  for (int k = 0; k < N; ++k) gmax = fmax(gmax, fabs(alpha[k]) + 2.0 * sqrt(beta[k < N - 1 ? k + 1 : k]));
  const double win = 1e-9 * gmax + 4.0 * (hi - lo);
  const double blo = x - win, bhi = x + win;
  for (int it = 0; it < 6; ++it) {
    double p0 = 0.0, p1 = 1.0, d0 = 0.0, d1 = 0.0;
    for (int k = 0; k < N; ++k) {
      double p2 = (x - alpha[k]) * p1 - (k > 0 ? beta[k] * p0 : 0.0);
      double d2 = p1 + (x - alpha[k]) * d1 - (k > 0 ? beta[k] * d0 : 0.0);
      p0 = p1;
      p1 = p2;
      d0 = d1;
      d1 = d2;
      double m = fmax(fabs(p1), fabs(d1));
      if (m > 1e150) {
        p0 *= 1e-150; p1 *= 1e-150; d0 *= 1e-150; d1 *= 1e-150;
      }
    }
    if (d1 == 0.0) break;
    double xn = x - p1 / d1;
    if (!(xn > blo && xn < bhi)) break;  // keep the bracketed bisection value
    if (xn == x) break;
    x = xn;
  }
  r[i] = x;
  // a_i = 1 / sum_k phat_k(x)^2 with phat_0 = 1/sqrt(beta_0),
  // sqrt(beta_{k+1}) phat_{k+1} = (x - alpha_k) phat_k - sqrt(beta_k) phat_{k-1}.
  double ph0 = 0.0, ph1 = 1.0 / sqrt(beta[0]);
  double s = ph1 * ph1, lscale = 0.0;  // sum = s * e^{lscale}, phat = ph * e^{lscale/2}
  for (int k = 0; k + 1 < N; ++k) {
    double ph2 = ((x - alpha[k]) * ph1 - (k > 0 ? sqrt(beta[k]) * ph0 : 0.0)) / sqrt(beta[k + 1]);
    ph0 = ph1;
    ph1 = ph2;
    s += ph1 * ph1;
    if (s > 1e200) {
      s *= 1e-200;
      ph0 *= 1e-100;
      ph1 *= 1e-100;
      lscale += 460.51701859880913680;  // ln 1e200
    }
  }
  log_a[i] = -(log(s) + lscale);
  if (!(x > 0.0) || !isfinite(log_a[i])) atomicOr(status, 1);
}

__global__ void k_radial_derived(int N, const double* r, const double* log_a, double* log_sig, double* sig) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double ls = 0.5 * log_a[i] + log(r[i]);
  log_sig[i] = ls;
  sig[i] = exp(ls);
}

// ---------------------------------------------------------------------------
// Basis tables with an extended exponent: value = stored * e^{es}, es <= 0.
// ---------------------------------------------------------------------------
struct Ext {
  double prev, cur, es;
  __device__ void rescale() {
    // move magnitude from the stored pair into the exponent while es < 0
    double m = fabs(cur);
    if (es < 0.0 && m > 1e100) {
      double f = fmin(230.25850929940456840, -es);  // ln 1e100
      double sc = exp(-f);
      prev *= sc;
      cur *= sc;
      es += f;
    }
  }
  __device__ double value() const { return es == 0.0 ? cur : cur * exp(es); }
};

__device__ Ext ext_start(double logv, double sign) {
  Ext e;
  e.prev = 0.0;
  if (logv < -460.0) {  // store 1e-200 and keep the rest in the exponent
    e.es = logv + 460.51701859880913680;
    e.cur = sign * 1e-200;
  } else {
    e.es = 0.0;
    e.cur = sign * exp(logv);
  }
  return e;
}

// Pbar_lm(cos th_j) for l = m..B-1: normalized form of Eq. legendre_recurrence,
//   Pbar_mm = (-1)^m sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)) sin^m th,
//   Pbar_lm = a_lm (cos th Pbar_{l-1,m} - Pbar_{l-2,m} / a_{l-1,m}),
//   a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)).
__global__ void k_legendre_table(int B, const double* theta, double* P) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * 2 * B) return;
  const int m = idx / (2 * B), j = idx % (2 * B);
  const double th = theta[j];
  const double t = cos(th);
  double lp = 0.5 * log((2.0 * m + 1.0) / (4.0 * kPi));
  for (int k = 1; k <= m; ++k) lp += 0.5 * log((2.0 * k - 1.0) / (2.0 * k));
  lp += m * log(sin(th));
  Ext e = ext_start(lp, (m & 1) ? -1.0 : 1.0);
  double* blk = P + table_block(B, m);
  const int ld = 2 * B;
  blk[j] = e.value();
  double ainv_prev = 0.0;  // 1 / a_{l-1,m}
  for (int l = m + 1; l < B; ++l) {
    const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
    const double nxt = a * (t * e.cur - ainv_prev * e.prev);
    e.prev = e.cur;
    e.cur = nxt;
    e.rescale();
    blk[(int64_t)(l - m) * ld + j] = e.value();
    ainv_prev = 1.0 / a;
  }
}

// rho_nl(r_i) = sigma_i Rhat_nl(r_i) for n = l+1..B (Lemma 3.5):
//   Rhat_{l+1,l} = sqrt(2 / Gamma(l + 3/2)) r^l,  Rhat_{ll} = 0,
//   Rhat_{n+1,l} = (2n - l - 1/2 - r^2) / sqrt((n + 1/2)(n - l)) Rhat_nl
//                  - sqrt((n - 1/2)(n - l - 1) / ((n + 1/2)(n - l))) Rhat_{n-1,l}.
__global__ void k_radial_table(int B, const double* r, const double* log_sig, double* R) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * 2 * B) return;
  const int l = idx / (2 * B), i = idx % (2 * B);
  const double x = r[i], t = x * x;
  const double lv = 0.5 * log(2.0) - 0.5 * lgamma(l + 1.5) + l * log(x) + log_sig[i];
  Ext e = ext_start(lv, 1.0);
  double* blk = R + table_block(B, l);
  const int ld = 2 * B;
  blk[i] = e.value();
  for (int n = l + 1; n < B; ++n) {
    const double c1 = (2.0 * n - l - 0.5 - t) / sqrt((n + 0.5) * (double)(n - l));
    const double c2 = sqrt((n - 0.5) * (double)(n - l - 1) / ((n + 0.5) * (double)(n - l)));
    const double nxt = c1 * e.cur - c2 * e.prev;
    e.prev = e.cur;
    e.cur = nxt;
    e.rescale();
    blk[(int64_t)(n + 1 - (l + 1)) * ld + i] = e.value();
  }
}

__global__ void k_twiddles(int L, double2* tw) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L) return;
  double a = 2.0 * q / L;
  tw[q] = make_double2(cospi(a), -sinpi(a));
}
__global__ void k_twiddles_f32(int L, float2* tw) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L) return;
  double a = 2.0 * q / L;
  tw[q] = make_float2((float)cospi(a), (float)-sinpi(a));
}

// Bluestein tables: chirp c_p = exp(-i pi p^2 / L); kernel spectra
//   bhf[q] = (1/M) sum_n conj(c_|n|) exp(-2 pi i q n / M),  bhi[q] = (1/M) sum_n c_|n| exp(...),
// with the kernel index n wrapped cyclically (|n| < L, zero elsewhere).
// Angles are reduced in integers (p^2 mod 2L, qn mod M) before sincospi.
template <typename T2>
__global__ void k_bluestein(int L, int M, T2* chirp, T2* bhf, T2* bhi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < L) {
    const double a = (double)(((int64_t)q * q) % (2 * L)) / L;
    chirp[q].x = cospi(a);
    chirp[q].y = -sinpi(a);
  }
  if (q >= M) return;
  double fr = 0, fi = 0, ir = 0, ii = 0;
  for (int n = 0; n < M; ++n) {
    int t;
    if (n < L) t = n;
    else if (n > M - L) t = M - n;
    else continue;
    const double ca = (double)(((int64_t)t * t) % (2 * L)) / L;  // c_t = exp(-i pi ca)
    const double cr = cospi(ca), ci = -sinpi(ca);
    const double wa = 2.0 * (double)(((int64_t)q * n) % M) / M;  // exp(-i pi wa)
    const double wr = cospi(wa), wi = -sinpi(wa);
    // forward kernel conj(c_t), inverse kernel c_t
    fr += cr * wr + ci * wi;
    fi += cr * wi - ci * wr;
    ir += cr * wr - ci * wi;
    ii += cr * wi + ci * wr;
  }
  bhf[q].x = fr / M;
  bhf[q].y = fi / M;
  bhi[q].x = ir / M;
  bhi[q].y = ii / M;
}

__global__ void k_to_f32(const double* src, float* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_to_double(uint16_t h) { return (double)__uint_as_float(((uint32_t)h) << 16); }

// Three bf16 pieces x0 + x1 + x2 of an FP64 value (each piece rounds the remainder).
__global__ void k_to_split(const double* src, uint16_t* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = src[i];
  uint16_t h0 = bf16_rne((float)x);
  double r1 = x - bf16_to_double(h0);
  uint16_t h1 = bf16_rne((float)r1);
  double r2 = r1 - bf16_to_double(h1);
  uint16_t h2 = bf16_rne((float)r2);
  dst[i] = h0;
  dst[n + i] = h1;
  dst[2 * n + i] = h2;
}

// Packed GEMM operand from a natural FP64 table (see ClassDesc::A).
// W: the grid-side length of the table rows (2B; B for the cosine-domain
// Legendre table, whose block q starts at table_block(B, q) / 2).
__global__ void k_pack(int B, int kind, int prec, const double* T64, const int64_t* offs, void* dst,
                       int64_t plane, int kchunk, double scale, int W) {
  const int q = blockIdx.y;
  const bool fwd = kind == 0 || kind == 2;
  const int L = W;
  const int rows = fwd ? B - q : L;
  const int K = fwd ? L : B - q;
  const int pitch = (K + kchunk - 1) / kchunk * kchunk;
  const double* src = T64 + table_block(B, q) / (2 * B) * W;
  const int64_t base = offs[q];
  const int64_t n = (int64_t)rows * pitch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / pitch), k = (int)(e - (int64_t)r * pitch);
    double v = 0.0;
    if (k < K) v = scale * (fwd ? src[(int64_t)r * L + k] : src[(int64_t)k * L + r]);
    if (prec == PREC_F64) {
      reinterpret_cast<double*>(dst)[base + e] = v;
    } else if (prec == PREC_F32) {
      reinterpret_cast<float*>(dst)[base + e] = (float)v;
    } else {
      uint16_t* d = reinterpret_cast<uint16_t*>(dst);
      const uint16_t h0 = bf16_rne((float)v);
      const double r1 = v - bf16_to_double(h0);
      const uint16_t h1 = bf16_rne((float)r1);
      const double r2 = r1 - bf16_to_double(h1);
      d[base + e] = h0;
      d[plane + base + e] = h1;
      d[2 * plane + base + e] = bf16_rne((float)r2);
    }
  }
}

inline int nblk(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

sgl_status_t build_grid(GridBuild& g, hipStream_t s) {
  const int B = g.B, N = 2 * B;
  hipLaunchKernelGGL(k_polar, dim3(nblk(N, 64)), dim3(64), 0, s, B, g.theta, g.btilde);
  SGL_HIP_TRY(hipGetLastError());

  // panel edges of the discretized half-line weight
  const double h = fmin(0.5, 40.0 / N);
  const double T = 1.6 * sqrt((double)N) + 8.0;
  std::vector<double> edges{0.0};
  double w = 1e-5;
  while (edges.back() + w < h) {
    edges.push_back(edges.back() + w);
    w *= 2.0;
  }
  while (edges.back() < T) edges.push_back(edges.back() + h);
  const int npanel = (int)edges.size() - 1;
  const int M = npanel * kGL;

  double* buf = nullptr;
  const size_t nbuf = (size_t)edges.size() + 2 * kGL + 4 * (size_t)M + 2 * (size_t)N;
  SGL_HIP_TRY(dev_malloc((void**)&buf, nbuf * sizeof(double)));
  int* d_status = nullptr;
  hipError_t e = dev_malloc((void**)&d_status, sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(buf);
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return SGL_ERR_OOM;
  }
  double* d_edges = buf;
  double* glx = d_edges + edges.size();
  double* glw = glx + kGL;
  double* xs = glw + kGL;
  double* vs = xs + M;
  double* qa = vs + M;
  double* qb = qa + M;
  double* alpha = qb + M;
  double* beta = alpha + N;
  sgl_status_t st = SGL_OK;
  int h_status = 0;
  auto fail = [&](hipError_t err, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(err));
    st = SGL_ERR_HIP;
  };
  do {
    if ((e = hipMemcpyAsync(d_edges, edges.data(), edges.size() * sizeof(double), hipMemcpyHostToDevice, s)) !=
        hipSuccess) { fail(e, "copy edges"); break; }
    if ((e = hipMemsetAsync(d_status, 0, sizeof(int), s)) != hipSuccess) { fail(e, "memset"); break; }
    hipLaunchKernelGGL(k_gauss_legendre, dim3(1), dim3(64), 0, s, glx, glw);
    hipLaunchKernelGGL(k_discretize, dim3(nblk(M, 256)), dim3(256), 0, s, npanel, d_edges, glx, glw, xs, vs);
    hipLaunchKernelGGL(k_lanczos, dim3(1), dim3(kLanczosThreads), 0, s, M, N, xs, vs, qa, qb, alpha, beta);
    hipLaunchKernelGGL(k_radial_nodes, dim3(nblk(N, 64)), dim3(64), 0, s, N, alpha, beta, g.r, g.log_a,
                       d_status);
    hipLaunchKernelGGL(k_radial_derived, dim3(nblk(N, 64)), dim3(64), 0, s, N, g.r, g.log_a, g.log_sig, g.sig);
    if ((e = hipGetLastError()) != hipSuccess) { fail(e, "grid kernels"); break; }
    if ((e = hipMemcpyAsync(&h_status, d_status, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) {
      fail(e, "copy status"); break;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { fail(e, "sync"); break; }
    if (h_status != 0) {
      set_error("half-range Gauss-Hermite rule: non-positive node or non-finite weight");
      st = SGL_ERR_NUMERIC;
    }
  } while (0);
  (void)hipFree(buf);
  (void)hipFree(d_status);
  return st;
}

hipError_t build_tables(int B, const double* r, const double* log_sig, const double* theta, double* P64,
                        double* R64, hipStream_t s) {
  const int n = B * 2 * B;
  hipLaunchKernelGGL(k_legendre_table, dim3(nblk(n, 128)), dim3(128), 0, s, B, theta, P64);
  hipLaunchKernelGGL(k_radial_table, dim3(nblk(n, 128)), dim3(128), 0, s, B, r, log_sig, R64);
  return hipGetLastError();
}

hipError_t build_twiddles(int L, void* tw, bool f32, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(k_twiddles_f32, dim3(nblk(L, 128)), dim3(128), 0, s, L, (float2*)tw);
  else
    hipLaunchKernelGGL(k_twiddles, dim3(nblk(L, 128)), dim3(128), 0, s, L, (double2*)tw);
  return hipGetLastError();
}

hipError_t build_bluestein(int L, int M, void* chirp, void* bhf, void* bhi, bool f32, hipStream_t s) {
  const int n = L > M ? L : M;
  if (f32)
    hipLaunchKernelGGL(k_bluestein<float2>, dim3(nblk(n, 64)), dim3(64), 0, s, L, M, (float2*)chirp, (float2*)bhf,
                       (float2*)bhi);
  else
    hipLaunchKernelGGL(k_bluestein<double2>, dim3(nblk(n, 64)), dim3(64), 0, s, L, M, (double2*)chirp,
                       (double2*)bhf, (double2*)bhi);
  return hipGetLastError();
}

hipError_t convert_table_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t pack_table(int B, int kind, int prec, const double* T64, const int64_t* d_offs, void* dst,
                      int64_t plane, double scale, hipStream_t s, int W) {
  hipLaunchKernelGGL(k_pack, dim3(64, B), dim3(256), 0, s, B, kind, prec, T64, d_offs, dst, plane, gemm_k_chunk(prec),
                     scale, W > 0 ? W : 2 * B);
  return hipGetLastError();
}

// Cosine-domain Legendre table of the seminaive step (Sect. 3.3.1, Eq. DCT and
// Eq. dct_trick): block m (m = 0..B-1) holds rows l = m..B-1 of B values
//   D[l][k] = s_k sum_j cos(k th_j) Pbar_lm(cos th_j) / sin^par th_j,
// par = m mod 2, th_j = (2j+1) pi / 4B, s_0 = sqrt(1/2B), s_k = sqrt(2/2B),
// set to zero beyond the degree (k > l - par).  Pbar from the FP64 master table.
__global__ void k_cos_legendre(int B, const double* P64, double* D64) {
  const int m = blockIdx.y;
  const int L = 2 * B;
  const int par = m & 1;
  const double* P = P64 + table_block(B, m);
  double* D = D64 + table_block(B, m) / 2;
  const int n = (B - m) * B;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int r = e / B, k = e - r * B;
    const int l = m + r;
    double v = 0.0;
    if (k <= l - par) {
      for (int j = 0; j < L; ++j) {
        // cos(k (2j+1) pi / 2L): exact argument reduction of the rational multiple of pi
        const int q = (k * (2 * j + 1)) % (4 * L);
        double w = cospi((double)q / (double)(2 * L)) * P[(int64_t)r * L + j];
        if (par) w /= sinpi((double)(2 * j + 1) / (double)(2 * L));
        v += w;
      }
      v *= k == 0 ? sqrt(1.0 / L) : sqrt(2.0 / L);
    }
    D[e] = v;
  }
}

// Constants of the DCT kernels of a class, P2 = 4B (complex, plan precision):
// [0, P2/2) the FFT twiddles exp(-2 pi i t / P2); [P2/2, P2/2 + B) the DCT
// post-factors s_k / 2 exp(-i pi k / 4B); [P2/2 + B, P2/2 + 3B) sin th_j (real part).
template <typename T2>
__global__ void k_dct_consts(int B, T2* out) {
  const int P2 = 4 * B, L = 2 * B;
  const int n = P2 / 2 + B + L;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    double re, im;
    if (e < P2 / 2) {
      sincospi(-2.0 * e / P2, &im, &re);
    } else if (e < P2 / 2 + B) {
      const int k = e - P2 / 2;
      const double sk = (k == 0 ? sqrt(1.0 / L) : sqrt(2.0 / L)) * 0.5;
      sincospi(-(double)k / (2.0 * L), &im, &re);
      re *= sk;
      im *= sk;
    } else {
      const int j = e - P2 / 2 - B;
      re = sinpi((double)(2 * j + 1) / (double)(2 * L));
      im = 0.0;
    }
    T2 v;
    v.x = re;
    v.y = im;
    out[e] = v;
  }
}

hipError_t build_cos_legendre(int B, const double* P64, double* D64, hipStream_t s) {
  hipLaunchKernelGGL(k_cos_legendre, dim3(nblk((int64_t)B * B, 128) < 64 ? nblk((int64_t)B * B, 128) : 64, B),
                     dim3(128), 0, s, B, P64, D64);
  return hipGetLastError();
}

hipError_t build_dct_consts(int B, void* out, bool f32, hipStream_t s) {
  const int n = 2 * B + B + 2 * B;
  if (f32)
    hipLaunchKernelGGL(k_dct_consts<float2>, dim3(nblk(n, 128)), dim3(128), 0, s, B, (float2*)out);
  else
    hipLaunchKernelGGL(k_dct_consts<double2>, dim3(nblk(n, 128)), dim3(128), 0, s, B, (double2*)out);
  return hipGetLastError();
}

hipError_t convert_table_split(const double* src, uint16_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_split, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace sgl
