// SGL expansions off the sampling grid, plain FP64:
//   * the Cartesian midpoint-rule projection that Sect. 5 describes as the
//     field's practice (an accuracy foil for the sampling-theorem transforms):
//       fhat_nlm ~ dV sum_c f(x_c) conj(H_nlm(x_c)) exp(-|x_c|^2)
//     over the cells of a regular grid (the weight is that of the SGL inner
//     product, Def. 1.2 and Eq. laguerre_ortho_transformed);
//   * synthesis at arbitrary points, f(x_p) = sum fhat_nlm H_nlm(x_p).
// The basis is evaluated per point by its three-term recurrences: the
// normalized Legendre recurrence (Eq. legendre_recurrence) in l and the
// generalized Laguerre recurrence (Eq. laguerre_recursion) carried in
// normalized form, u_k = N_k^(l) r^l L_k^(l+1/2)(r^2) exp(-r^2/2):
//   u_{k+1} = ((2k + l + 3/2 - r^2) u_k - sqrt(k (k + l + 1/2)) u_{k-1}) / sqrt((k+1)(k + l + 3/2)),
//   u_0 = sqrt(2 / Gamma(l + 3/2)) r^l exp(-r^2/2),  H_nlm exp(-r^2/2) = u_{n-l-1} Pbar_lm e^{i m ph}.
// Radially scaled plans evaluate the unit basis at x / s and take s^(-3/2).
#include "sgl_internal.h"

namespace sgl {
namespace {

constexpr int NT = 256;
constexpr int NG = kNaiveGroup;  // coefficients (consecutive n) per midpoint block, items as the naive forward

struct Sph {
  double r2, ct, st, ph;  // |y|^2, cos theta, sin theta, azimuth of the unit-basis point y
  double r;
};

__device__ inline Sph spherical(double x, double y, double z) {
  Sph p;
  p.r2 = x * x + y * y + z * z;
  p.r = sqrt(p.r2);
  const double rho = sqrt(x * x + y * y);
  if (p.r > 0) {
    p.ct = z / p.r;
    p.st = rho / p.r;
  } else {
    p.ct = 1.0;
    p.st = 0.0;
  }
  p.ph = atan2(y, x);
  return p;
}

// Pbar_{am, am}(cos theta) (normalized, Condon-Shortley sign), log-space start
__device__ inline double pbar_mm(int am, double st) {
  if (am == 0) return 0.28209479177387814347;  // 1 / sqrt(4 pi)
  if (st <= 0.0) return 0.0;
  double lg = 0.5 * log((2.0 * am + 1.0) / (4.0 * 3.14159265358979323846));
  for (int k = 1; k <= am; ++k) lg += 0.5 * log((2.0 * k - 1.0) / (2.0 * k));
  lg += am * log(st);
  const double v = lg < -745.0 ? 0.0 : exp(lg);
  return (am & 1) ? -v : v;
}

// Pbar_{l, am}(cos theta) by the recurrence in l
__device__ inline double pbar(int l, int am, double ct, double st) {
  double p0 = pbar_mm(am, st);
  if (l == am) return p0;
  double p1 = sqrt(2.0 * am + 3.0) * ct * p0;
  for (int q = am + 2; q <= l; ++q) {
    const double a = sqrt((4.0 * q * q - 1.0) / ((double)q * q - (double)am * am));
    const double b = sqrt(((q - 1.0) * (q - 1.0) - (double)am * am) / (4.0 * (q - 1.0) * (q - 1.0) - 1.0));
    const double p2 = a * (ct * p1 - b * p0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// u_0 of degree l at radius r (see the header comment)
__device__ inline double u_start(int l, double r, double r2) {
  if (r == 0.0) return l == 0 ? sqrt(2.0 / 0.88622692545275801365) : 0.0;  // Gamma(3/2) = sqrt(pi)/2
  const double lg = 0.5 * log(2.0) - 0.5 * lgamma(l + 1.5) + l * log(r) - 0.5 * r2;
  return lg < -745.0 ? 0.0 : exp(lg);
}

__device__ inline int class_of(const int64_t* pre, int ncls, int64_t w) {
  int c = 0;
  while (c + 1 < ncls && pre[c + 1] <= w) ++c;
  return c;
}

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  for (int q = 0; q < NT / 64; ++q) t += red[q];
  return t;
}

// Midpoint projection.  Items as the naive forward transform: (function, l, m,
// group of NG degrees n), prefix over l in ClassDesc::naive_loff.
__global__ void __launch_bounds__(NT) k_midpoint_forward(const ClassDesc* __restrict__ cls,
                                                         const int64_t* __restrict__ pre, int ncls, int64_t nitems,
                                                         const double2* __restrict__ values, int nx, double h,
                                                         double2* __restrict__ coeffs) {
  __shared__ double red[NT / 64];
  const double d = 2.0 * h / nx;
  const int ncell = nx * nx * nx;
  for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int c = class_of(pre, ncls, w);
    const ClassDesc& C = cls[c];
    const int B = C.B;
    const int per = gmem(C.naive_loff)[B];
    const int64_t rr = w - pre[c];
    const int b = (int)(rr / per);
    int q = (int)(rr - (int64_t)b * per);
    int l = 0;
    while (gmem(C.naive_loff)[l + 1] <= q) ++l;
    q -= gmem(C.naive_loff)[l];
    const int ng = (B - l + NG - 1) / NG;
    const int m = q / ng - l;
    const int n0 = l + 1 + (q - (m + l) * ng) * NG;
    const int nn = min(NG, B + 1 - n0);
    const int am = m < 0 ? -m : m;
    const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    const double inv_s = 1.0 / C.rscale;
    const double al = l + 0.5;
    const double2* f = values + (int64_t)gmem(C.fid)[b] * ncell;
    double ar[NG], ai[NG];
    for (int g = 0; g < NG; ++g) ar[g] = ai[g] = 0.0;
    for (int cell = threadIdx.x; cell < ncell; cell += NT) {
      const int ix = cell / (nx * nx), iy = (cell / nx) % nx, iz = cell % nx;
      const Sph p = spherical((-h + (ix + 0.5) * d) * inv_s, (-h + (iy + 0.5) * d) * inv_s,
                              (-h + (iz + 0.5) * d) * inv_s);
      const double2 fv = f[cell];
      // f exp(-|y|^2/2) Pbar_lm exp(-i m ph); the other exp(-|y|^2/2) is in u_k
      const double wgt = exp(-0.5 * p.r2) * sg * pbar(l, am, p.ct, p.st);
      double sn, cs;
      sincos(m * p.ph, &sn, &cs);
      const double tr = wgt * (fv.x * cs + fv.y * sn), ti = wgt * (fv.y * cs - fv.x * sn);
      // u_k for k = 0 .. n0 + nn - l - 2
      double um = 0.0, u = u_start(l, p.r, p.r2);
      const int k0 = n0 - l - 1;
      for (int k = 0; k < k0; ++k) {
        const double un = ((2.0 * k + al + 1.0 - p.r2) * u - sqrt(k * (k + al)) * um) / sqrt((k + 1.0) * (k + al + 1.0));
        um = u;
        u = un;
      }
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (g < nn) {
          ar[g] += u * tr;
          ai[g] += u * ti;
          const int k = k0 + g;
          const double un = ((2.0 * k + al + 1.0 - p.r2) * u - sqrt(k * (k + al)) * um) / sqrt((k + 1.0) * (k + al + 1.0));
          um = u;
          u = un;
        }
      }
    }
    const double scale = d * d * d * C.rs_inv;  // dV s^(-3/2)
    for (int g = 0; g < nn; ++g) {
      const double sr = block_sum(ar[g], red);
      const double si = block_sum(ai[g], red);
      if (threadIdx.x == 0) coeffs[gmem(C.coff)[b] + omega(n0 + g, l, m)] = make_double2(sr * scale, si * scale);
    }
    __syncthreads();
  }
}

// Synthesis at arbitrary points.  Item: (function, chunk of NT points); pre_nf
// is the per-class prefix of function counts.
__global__ void __launch_bounds__(NT) k_synthesize_points(const ClassDesc* __restrict__ cls,
                                                          const int64_t* __restrict__ pre_nf, int ncls, int64_t nitems,
                                                          const double2* __restrict__ coeffs, int npts,
                                                          const double* __restrict__ xyz, double2* __restrict__ out) {
  const int chunks = (npts + NT - 1) / NT;
  for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int64_t fw = w / chunks;  // function position in class order
    const int c = class_of(pre_nf, ncls, fw);
    const ClassDesc& C = cls[c];
    const int B = C.B;
    const int64_t rr = w - pre_nf[c] * chunks;
    const int b = (int)(rr / chunks);
    const int pt = (int)(rr - (int64_t)b * chunks) * NT + threadIdx.x;
    if (pt >= npts) continue;
    const double inv_s = 1.0 / C.rscale;
    const Sph p = spherical(xyz[3 * (int64_t)pt] * inv_s, xyz[3 * (int64_t)pt + 1] * inv_s,
                            xyz[3 * (int64_t)pt + 2] * inv_s);
    const double2* f = coeffs + gmem(C.coff)[b];
    double accr = 0.0, acci = 0.0;
    for (int m = 1 - B; m < B; ++m) {
      const int am = m < 0 ? -m : m;
      const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
      double sn, cs;
      sincos(m * p.ph, &sn, &cs);
      // Pbar_{l, am} for l = am, am+1, ... by the recurrence in l
      double p0 = pbar_mm(am, p.st), p1 = 0.0;
      for (int l = am; l < B; ++l) {
        double pl;
        if (l == am) {
          pl = p0;
        } else if (l == am + 1) {
          p1 = sqrt(2.0 * am + 3.0) * p.ct * p0;
          pl = p1;
        } else {
          const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)am * am));
          const double bb = sqrt(((l - 1.0) * (l - 1.0) - (double)am * am) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
          const double p2 = a * (p.ct * p1 - bb * p0);
          p0 = p1;
          p1 = p2;
          pl = p2;
        }
        // sum_n fhat_nlm u_{n-l-1}(r)
        const double al = l + 0.5;
        double um = 0.0, u = u_start(l, p.r, p.r2), sr = 0.0, si = 0.0;
        for (int n = l + 1; n <= B; ++n) {
          const double2 fv = f[omega(n, l, m)];
          sr += u * fv.x;
          si += u * fv.y;
          const int k = n - l - 1;
          const double un = ((2.0 * k + al + 1.0 - p.r2) * u - sqrt(k * (k + al)) * um) / sqrt((k + 1.0) * (k + al + 1.0));
          um = u;
          u = un;
        }
        const double ang = sg * pl;
        accr += ang * (sr * cs - si * sn);
        acci += ang * (sr * sn + si * cs);
      }
    }
    const double e = exp(0.5 * p.r2) * C.rs_inv;  // undo exp(-|y|^2/2) of u_k; s^(-3/2)
    out[(int64_t)gmem(C.fid)[b] * npts + pt] = make_double2(accr * e, acci * e);
  }
}

inline int grid_of(int64_t nitems) { return (int)(nitems < 65536 ? nitems : 65536); }

}  // namespace

hipError_t launch_midpoint_forward(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                   const void* values, int nx, double h, void* coeffs, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_midpoint_forward, dim3(grid_of(nitems)), dim3(NT), 0, s, d_cls, d_pre, ncls, nitems,
                     reinterpret_cast<const double2*>(values), nx, h, reinterpret_cast<double2*>(coeffs));
  return hipGetLastError();
}

hipError_t launch_synthesize_points(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                    const void* coeffs, int npts, const double* xyz, void* values, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_synthesize_points, dim3(grid_of(nitems)), dim3(NT), 0, s, d_cls, d_pre, ncls, nitems,
                     reinterpret_cast<const double2*>(coeffs), npts, xyz, reinterpret_cast<double2*>(values));
  return hipGetLastError();
}

}  // namespace sgl
