// Plan-time FP64 kernels: quadrature grid (Thm. 3.1, Thm. 3.3) and basis tables
// (Eq. legendre_recurrence, Lemma 3.5), plus rounding of the tables to the
// precision of the contraction stages.
//
// Half-range Gauss-Hermite rule of order N (Thm. 3.3).  The paper computes it
// with special recurrences in high-precision arithmetic and stores the values
// in double precision; it does not give the procedure.  Here it is computed on
// the GPU in double-double arithmetic (about 106 bits) and rounded once to FP64:
//   1. discretize the weight exp(-r^2) dr on [0, T] by composite 32-point
//      Gauss-Legendre panels (width min(0.5, 40/N), halved repeatedly towards
//      r = 0 where the zeros of p_N crowd; T = 1.6 sqrt(N) + 8);
//   2. run the Lanczos iteration on diag(x) with the square-root weights as
//      start vector, in double-double: its recurrence coefficients alpha_k,
//      beta_k (k < N) are those of the continuous weight up to the FP64
//      rounding of the discretization (the start vector is carried times e^300
//      so that no entry underflows out to r = T);
//   3. nodes r_i = zeros of p_N: Sturm-sequence bisection on the Jacobi matrix
//      in FP64, then Newton on p_N evaluated by the three-term recurrence in
//      double-double;
//   4. weights a_i = 1 / sum_k phat_k(r_i)^2 (orthonormal phat_k) in
//      double-double, formed in log space because a_i underflows FP64 for
//      N >~ 280.
#include <math.h>

#include "sgl_internal.h"

// No floating-point contraction in this file: the double-double arithmetic
// below relies on every sum and product being rounded separately (a multiply
// fused into a following add by the compiler breaks its error-free
// transformations), and the plan-time tables are cheap enough to build with
// separately rounded operations throughout.
#pragma clang fp contract(off)

namespace sgl {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kGL = 32;           // Gauss-Legendre points per panel
constexpr double kStartScale = 300.0;  // ln of the start-vector scale

// ---------------------------------------------------------------------------
// Double-double arithmetic: value = hi + lo with |lo| <= ulp(hi) / 2, from the
// error-free transformations of a sum (Knuth's two-sum) and of a product (FMA).
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};
__device__ inline dd ddv(double a) { return dd{a, 0.0}; }
__device__ inline dd two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd fast_two_sum(double a, double b) {  // |a| >= |b| or a == 0
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ inline dd operator+(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  const dd t = two_sum(x.lo, y.lo);
  s = fast_two_sum(s.hi, s.lo + t.hi);
  return fast_two_sum(s.hi, s.lo + t.lo);
}
__device__ inline dd operator-(dd x) { return dd{-x.hi, -x.lo}; }
__device__ inline dd operator-(dd x, dd y) { return x + (-y); }
__device__ inline dd operator*(dd x, dd y) {
  const double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, e);
  e = fma(x.lo, y.hi, e);
  return fast_two_sum(p, e);
}
__device__ inline dd operator*(dd x, double y) {
  const double p = x.hi * y;
  return fast_two_sum(p, fma(x.lo, y, fma(x.hi, y, -p)));
}
__device__ inline dd dd_div(dd x, dd y) {
  const double q1 = x.hi / y.hi;
  dd r = x - y * q1;
  const double q2 = r.hi / y.hi;
  r = r - y * q2;
  const double q3 = r.hi / y.hi;
  return fast_two_sum(q1, q2) + ddv(q3);
}
__device__ inline dd dd_sqrt(dd x) {  // x > 0: one Newton step from the FP64 root
  const double s = sqrt(x.hi);
  const dd r = x - ddv(s) * ddv(s);
  return fast_two_sum(s, r.hi / (2.0 * s));
}
__device__ inline dd dd_scale(dd x, int e) { return dd{ldexp(x.hi, e), ldexp(x.lo, e)}; }  // exact
// e^x for |x| < 700: x = k ln2 + r with |r| <= ln2 / 2, e^(r / 1024) - 1 by its
// Taylor series (nine terms reach 1e-33), squared back ten times as
// s <- 2 s + s^2 (s = e^t - 1), then scaled by 2^k.
__device__ inline dd dd_exp(dd x) {
  const dd ln2{0.6931471805599453, 2.3190468138462996e-17};
  const double k = rint(x.hi / ln2.hi);
  const dd r = dd_scale(x - ln2 * k, -10);
  dd term = r, sum = r;
  for (int n = 2; n <= 9; ++n) {
    term = dd_div(term * r, ddv((double)n));
    sum = sum + term;
  }
  for (int q = 0; q < 10; ++q) sum = dd_scale(sum, 1) + sum * sum;
  return dd_scale(sum + ddv(1.0), (int)k);
}

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

// 32-point Gauss-Legendre rule on [-1, 1] by Newton on P_32, in double-double
// (the FP64 weight formula loses up to ~5e-15 to cancellation).
__device__ inline void legendre32(dd z, dd& p, dd& dp) {
  constexpr int n = kGL;
  dd p0 = ddv(1.0), p1 = z;
  for (int k = 2; k <= n; ++k) {
    const dd p2 = dd_div(z * p1 * (2.0 * k - 1.0) - p0 * (k - 1.0), ddv((double)k));
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = dd_div((z * p1 - p0) * (double)n, z * z - ddv(1.0));
}
__global__ void k_gauss_legendre(dd* x, dd* w) {
  int i = threadIdx.x;
  if (i >= kGL) return;
  dd z = ddv(cos(kPi * (i + 0.75) / (kGL + 0.5)));
  dd p, dp;
  for (int it = 0; it < 100; ++it) {
    legendre32(z, p, dp);
    const dd dz = dd_div(p, dp);
    z = z - dz;
    if (fabs(dz.hi) < 1e-32) break;
  }
  legendre32(z, p, dp);
  x[i] = z;
  w[i] = dd_div(ddv(2.0), (ddv(1.0) - z * z) * dp * dp);
}

// Discretized weight, in double-double: points xs and start vector
// vs = sqrt(w) e^{C - x^2/2} (the relative errors of FP64 points and weights,
// ~1e-16 each, would move the recurrence coefficients by ~1e-16 and the
// smallest nodes by ~1e-16 ||J|| / r_0 relative).
__global__ void k_discretize(int npanel, const double* edges, const dd* glx, const dd* glw, dd* xs, dd* vs) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npanel * kGL) return;
  int p = idx / kGL, q = idx % kGL;
  const double a = edges[p], b = edges[p + 1];
  const dd hh = dd_scale(two_sum(b, -a), -1);  // half the panel width
  const dd x = ddv(a) + (glx[q] + ddv(1.0)) * hh;
  xs[idx] = x;
  const dd arg = ddv(kStartScale) - dd_scale(x * x, -1);
  vs[idx] = dd_sqrt(glw[q] * hh) * dd_exp(arg);
}

template <int NT>
__device__ dd block_sum_dd(dd v, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    const dd o{__shfl_down(v.hi, off, 64), __shfl_down(v.lo, off, 64)};
    v = v + o;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * wid] = v.hi;
    red[2 * wid + 1] = v.lo;
  }
  __syncthreads();
  dd t = ddv(0.0);
  if (threadIdx.x < NT / 64) t = dd{red[2 * threadIdx.x], red[2 * threadIdx.x + 1]};
  if (threadIdx.x < 64) {
    for (int off = 32; off > 0; off >>= 1) {
      const dd o{__shfl_down(t.hi, off, 64), __shfl_down(t.lo, off, 64)};
      t = t + o;
    }
  }
  if (threadIdx.x == 0) {
    red[64] = t.hi;
    red[65] = t.lo;
  }
  __syncthreads();
  return dd{red[64], red[65]};
}

// Lanczos on diag(xs) with start vector vs (one block), in double-double.
// Produces the monic recurrence coefficients alpha_k, beta_k (k < N) and
// sqrt(beta_k), each as (hi, lo) pairs; beta_0 = mu_0 = sqrt(pi)/2.  qa, qb:
// 2M doubles each (the Lanczos vectors as hi, lo pairs).
constexpr int kLanczosThreads = 1024;
__global__ void __launch_bounds__(kLanczosThreads) k_lanczos(int M, int N, const dd* xs, const dd* vs, dd* qa,
                                                             dd* qb, dd* alpha, dd* beta, dd* sbeta) {
  __shared__ double red[66];
  const int t = threadIdx.x;
  dd ss = ddv(0.0);
  for (int i = t; i < M; i += kLanczosThreads) ss = ss + vs[i] * vs[i];
  const dd inv = dd_div(ddv(1.0), dd_sqrt(block_sum_dd<kLanczosThreads>(ss, red)));
  for (int i = t; i < M; i += kLanczosThreads) {
    qa[i] = inv * vs[i];  // q_0
    qb[i] = ddv(0.0);     // q_{-1}
  }
  if (t == 0) {
    beta[0] = dd{0.886226925452758, -3.8332932499128993e-17};  // sqrt(pi) / 2 to 106 bits
    sbeta[0] = dd_sqrt(beta[0]);
  }
  __syncthreads();
  dd sb = ddv(0.0);  // sqrt(beta_k)
  dd* qc = qa;
  dd* qp = qb;
  for (int k = 0; k < N; ++k) {
    dd part = ddv(0.0);
    for (int i = t; i < M; i += kLanczosThreads) part = part + (qc[i] * qc[i]) * xs[i];
    const dd a = block_sum_dd<kLanczosThreads>(part, red);
    dd part2 = ddv(0.0);
    for (int i = t; i < M; i += kLanczosThreads) {
      const dd u = (xs[i] - a) * qc[i] - sb * qp[i];
      qp[i] = u;  // overwrite q_{k-1} with the unnormalized q_{k+1}
      part2 = part2 + u * u;
    }
    const dd nb = dd_sqrt(block_sum_dd<kLanczosThreads>(part2, red));
    const dd rn = dd_div(ddv(1.0), nb);
    for (int i = t; i < M; i += kLanczosThreads) qp[i] = qp[i] * rn;
    if (t == 0) {
      alpha[k] = a;
      if (k + 1 < N) {
        beta[k + 1] = nb * nb;
        sbeta[k + 1] = nb;
      }
    }
    __syncthreads();
    dd* tmp = qc;
    qc = qp;
    qp = tmp;
    sb = nb;
  }
}

// Number of eigenvalues of the Jacobi matrix below x (Sturm sequence via LDL^T).
__device__ int sturm_count(int N, const dd* alpha, const dd* beta, double x) {
  int cnt = 0;
  double d = alpha[0].hi - x;
  if (d == 0.0) d = -1e-300;
  if (d < 0) ++cnt;
  for (int k = 1; k < N; ++k) {
    d = (alpha[k].hi - x) - beta[k].hi / d;
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

// One thread per node: FP64 bisection, Newton in double-double, then the
// Christoffel weight in log form (double-double sums).
__global__ void k_radial_nodes(int N, const dd* alpha, const dd* beta, const dd* sbeta, double* r, double* log_a,
                               double* sig_m, double* sig_e, int* status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  // Gershgorin bound
  double hi = 0.0;
  for (int k = 0; k < N; ++k) {
    double e0 = k > 0 ? sbeta[k].hi : 0.0;
    double e1 = k + 1 < N ? sbeta[k + 1].hi : 0.0;
    hi = fmax(hi, alpha[k].hi + e0 + e1);
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
  // Newton on p_N / p_N' with running rescaling by powers of two (exact; the
  // ratio is scale free).  The Sturm count is accurate to about eps ||J|| in
  // absolute terms, so the bisection value can be that far from the zero;
  // Newton may move it within a window still far below the spacing of
  // neighbouring zeros.
  dd x = ddv(0.5 * (lo + hi));
  double gmax = 0.0;
  for (int k = 0; k < N; ++k) gmax = fmax(gmax, fabs(alpha[k].hi) + 2.0 * sbeta[k < N - 1 ? k + 1 : k].hi);
  const double win = 1e-9 * gmax + 4.0 * (hi - lo);
  const double blo = x.hi - win, bhi = x.hi + win;
  for (int it = 0; it < 12; ++it) {
    dd p0 = ddv(0.0), p1 = ddv(1.0), d0 = ddv(0.0), d1 = ddv(0.0);
    for (int k = 0; k < N; ++k) {
      const dd xa = x - alpha[k];
      dd p2 = xa * p1, d2 = p1 + xa * d1;
      if (k > 0) {
        p2 = p2 - beta[k] * p0;
        d2 = d2 - beta[k] * d0;
      }
      p0 = p1;
      p1 = p2;
      d0 = d1;
      d1 = d2;
      if (fmax(fabs(p1.hi), fabs(d1.hi)) > 0x1p500) {
        p0 = dd_scale(p0, -500); p1 = dd_scale(p1, -500); d0 = dd_scale(d0, -500); d1 = dd_scale(d1, -500);
      }
    }
    if (d1.hi == 0.0) break;
    const dd dx = dd_div(p1, d1);
    const dd xn = x - dx;
    if (!(xn.hi > blo && xn.hi < bhi)) break;  // keep the bracketed value
    x = xn;
    if (fabs(dx.hi) <= 1e-31 * fabs(x.hi)) break;
  }
  r[i] = x.hi;
  // a_i = 1 / sum_k phat_k(x)^2 with phat_0 = 1/sqrt(beta_0),
  // sqrt(beta_{k+1}) phat_{k+1} = (x - alpha_k) phat_k - sqrt(beta_k) phat_{k-1}.
  dd ph0 = ddv(0.0), ph1 = dd_div(ddv(1.0), sbeta[0]);
  dd sum = ph1 * ph1;
  int lscale = 0;  // sum = s * 2^lscale, phat = ph * 2^(lscale / 2)
  for (int k = 0; k + 1 < N; ++k) {
    dd num = (x - alpha[k]) * ph1;
    if (k > 0) num = num - sbeta[k] * ph0;
    const dd ph2 = dd_div(num, sbeta[k + 1]);
    ph0 = ph1;
    ph1 = ph2;
    sum = sum + ph1 * ph1;
    if (sum.hi > 0x1p600) {
      sum = dd_scale(sum, -600);
      ph0 = dd_scale(ph0, -300);
      ph1 = dd_scale(ph1, -300);
      lscale += 600;
    }
  }
  log_a[i] = -(log(sum.hi) + log1p(sum.lo / sum.hi) + lscale * 0.69314718055994530942);
  // sigma_i = sqrt(a_i) r_i = r_i / sqrt(sum) * 2^(-lscale/2) (lscale is even): its
  // mantissa to double-double accuracy and its power-of-two exponent
  sig_m[i] = (x * dd_div(ddv(1.0), dd_sqrt(sum))).hi;
  sig_e[i] = -0.5 * lscale;
  if (!(x.hi > 0.0) || !isfinite(log_a[i])) atomicOr(status, 1);
}

// ln sigma_i and sigma_i (0 where it underflows) from its mantissa and exponent
__global__ void k_radial_derived(int N, const double* sig_m, const double* sig_e, double* log_sig, double* sig) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  log_sig[i] = log(sig_m[i]) + sig_e[i] * 0.69314718055994530942;
  sig[i] = ldexp(sig_m[i], (int)sig_e[i]);
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

// A double-double mantissa times a power of two (start values that may leave
// the FP64 range), renormalized so that the mantissa stays near 1.
struct DdExp {
  dd m;
  int e;
  __device__ void renorm() {
    int k = 0;
    (void)frexp(m.hi, &k);
    m = dd_scale(m, -k);
    e += k;
  }
  __device__ void mul(dd f) {
    m = m * f;
    renorm();
  }
};
// Start of a recurrence from an exact-product value: stored directly when it is
// above 1e-200, else as 1e-200 e^{es} like ext_start (only the tiny values, far
// below every sum they enter, carry the log-space rounding).
__device__ Ext ext_from(DdExp v, double sign) {
  const double lv = log(fabs(v.m.hi)) + v.e * 0.69314718055994530942;
  if (lv < -460.0) return ext_start(lv, sign);
  Ext x;
  x.prev = 0.0;
  x.es = 0.0;
  x.cur = sign * ldexp(v.m.hi, v.e);
  return x;
}

// Pbar_lm(cos th_j) for l = m..B-1: normalized form of Eq. legendre_recurrence,
//   Pbar_mm = (-1)^m sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)) sin^m th,
//   Pbar_lm = a_lm (cos th Pbar_{l-1,m} - Pbar_{l-2,m} / a_{l-1,m}),
//   a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)).
__global__ void k_legendre_table(int B, const double* theta, double* P) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * 2 * B) return;
  const int m = idx / (2 * B), j = idx % (2 * B);
  // theta_j = pi q with q = (2j+1)/(4B): sine and cosine from q (theta[j] is its FP64 rounding)
  const double q = (double)(2 * j + 1) / (4.0 * B);
  const double t = cospi(q), st = sinpi(q);
  (void)theta;
  // Pbar_mm as exact products in double-double: (2m+1)/(4 pi) prod (2k-1)/(2k),
  // square-rooted, times sin^m theta
  DdExp c{dd{0.07957747154594767, -4.9196691687956215e-18} * (2.0 * m + 1.0), 0};  // (2m+1) / (4 pi)
  c.renorm();
  for (int k = 1; k <= m; ++k) c.mul(dd_div(ddv(2.0 * k - 1.0), ddv(2.0 * k)));
  if (c.e & 1) {
    c.m = dd_scale(c.m, 1);
    c.e -= 1;
  }
  DdExp v{dd_sqrt(c.m), c.e / 2};
  for (int k = 0; k < m; ++k) v.mul(ddv(st));
  Ext e = ext_from(v, (m & 1) ? -1.0 : 1.0);
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
// The start is formed as exact products in double-double (the log-space form
// rounds at the magnitude of l ln r and ln Gamma, ~1e-13 relative at B = 256):
// sigma_i from the rule, sqrt(c_l) with c_l = 2 / Gamma(l + 3/2) =
// c_{l-1} 2 / (2l + 1), c_0 = 4 / sqrt(pi), and r_i^l.
__global__ void k_radial_table(int B, const double* r, const double* sig_m, const double* sig_e, double* R) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * 2 * B) return;
  const int l = idx / (2 * B), i = idx % (2 * B);
  const double x = r[i], t = x * x;
  DdExp c{dd{2.256758334191025, 3.067091922633176e-17}, 0};  // 4 / sqrt(pi)
  c.renorm();
  for (int k = 1; k <= l; ++k) c.mul(dd_div(ddv(2.0), ddv(2.0 * k + 1.0)));
  if (c.e & 1) {
    c.m = dd_scale(c.m, 1);
    c.e -= 1;
  }
  DdExp v{dd_sqrt(c.m), c.e / 2};
  v.renorm();
  for (int k = 0; k < l; ++k) v.mul(ddv(x));
  v.mul(ddv(sig_m[i]));
  v.e += (int)sig_e[i];
  Ext e = ext_from(v, 1.0);
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
  // edges (FP64), then double-double arrays from an even offset (16-byte
  // aligned): GL nodes and weights, points xs and start vector vs, the two
  // Lanczos vectors, alpha, beta, sqrt(beta)
  const size_t off_dd = (edges.size() + 1) / 2 * 2;
  const size_t nbuf = off_dd + 2 * (2 * (size_t)kGL + 4 * (size_t)M + 3 * (size_t)N);
  SGL_HIP_TRY(dev_malloc((void**)&buf, nbuf * sizeof(double)));
  int* d_status = nullptr;
  hipError_t e = dev_malloc((void**)&d_status, sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(buf);
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return SGL_ERR_OOM;
  }
  double* d_edges = buf;
  dd* glx = reinterpret_cast<dd*>(buf + off_dd);
  dd* glw = glx + kGL;
  dd* xs = glw + kGL;
  dd* vs = xs + M;
  dd* qa = vs + M;
  dd* qb = qa + M;
  dd* alpha = qb + M;
  dd* beta = alpha + N;
  dd* sbeta = beta + N;
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
    hipLaunchKernelGGL(k_lanczos, dim3(1), dim3(kLanczosThreads), 0, s, M, N, xs, vs, qa, qb, alpha, beta, sbeta);
    hipLaunchKernelGGL(k_radial_nodes, dim3(nblk(N, 64)), dim3(64), 0, s, N, alpha, beta, sbeta, g.r, g.log_a,
                       g.sig_m, g.sig_e, d_status);
    hipLaunchKernelGGL(k_radial_derived, dim3(nblk(N, 64)), dim3(64), 0, s, N, g.sig_m, g.sig_e, g.log_sig, g.sig);
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

hipError_t build_tables(int B, const GridBuild& g, double* P64, double* R64, hipStream_t s) {
  const int n = B * 2 * B;
  hipLaunchKernelGGL(k_legendre_table, dim3(nblk(n, 128)), dim3(128), 0, s, B, g.theta, P64);
  hipLaunchKernelGGL(k_radial_table, dim3(nblk(n, 128)), dim3(128), 0, s, B, g.r, g.sig_m, g.sig_e, R64);
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
