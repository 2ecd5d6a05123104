// The naive discrete SGL transforms (Alg. 1, Alg. 2), plain FP64, as a second
// GPU workload beside the fast path: every coefficient is the full quadrature
// sum over all (2B)^3 grid points, and every sample is the full synthesis sum
// over all B(B+1)(2B+1)/6 coefficients.  The basis factors come from the
// plan's FP64 tables (rho_nl(r_i) = sigma_i N_nl R_nl(r_i), Pbar_lm(cos th_j))
// and the FP64 azimuthal twiddles instead of per-point recurrences, so the
// cost is O(B^6) rather than O(B^7); the summation is the algorithms' own (no
// separation of variables, no FFT, no matrix cores).  With scaled samples
// s = sigma_i f the forward sum of Alg. 1 reads
//   fhat_nlm = sum_{i,j,k} b~_j s_ijk rho_nl(r_i) Pbar_lm(cos th_j) exp(-i m ph_k)
// and the synthesis of Alg. 2
//   s_ijk = sum_{n,l,m} fhat_nlm rho_nl(r_i) Pbar_lm(cos th_j) exp(+i m ph_k).
#include "sgl_internal.h"

namespace sgl {
namespace {

constexpr int NT = 256;  // threads per block
constexpr int NG = kNaiveGroup;  // coefficients (consecutive n) per forward block
constexpr int CH = 1024; // coefficients staged per inverse chunk

__device__ inline double2 cmulc(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// (m k) mod L in [0, L)
__device__ inline int phase_index(int m, int k, int L) {
  int e = (m * k) % L;
  return e < 0 ? e + L : e;
}

// class of a global item index (block-uniform; plans hold few classes)
__device__ inline int class_of(const int64_t* pre, int ncls, int64_t w) {
  int c = 0;
  while (c + 1 < ncls && pre[c + 1] <= w) ++c;
  return c;
}

// Sum a double over the block (NT threads); every thread gets the result.
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

// Alg. 1.  Item of a class: function b, degree l, order m, first degree-n
// group; loff[l] is the prefix over l of (2l+1) ceil((B-l)/NG).
__global__ void __launch_bounds__(NT) k_naive_forward(const ClassDesc* __restrict__ cls, const int64_t* __restrict__ pre,
                                                      int ncls, int64_t nitems, const double2* __restrict__ samples,
                                                      double2* __restrict__ coeffs, int raw) {
  __shared__ double red[NT / 64];
  for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int c = class_of(pre, ncls, w);
    const ClassDesc& C = cls[c];
    const int B = C.B, L = C.L;
    const int per = gmem(C.naive_loff)[B];
    const int64_t r = w - pre[c];
    const int b = (int)(r / per);
    int q = (int)(r - (int64_t)b * per);
    int l = 0;
    while (gmem(C.naive_loff)[l + 1] <= q) ++l;
    q -= gmem(C.naive_loff)[l];
    const int ng = (B - l + NG - 1) / NG;
    const int m = q / ng - l;
    const int n0 = l + 1 + (q - (m + l) * ng) * NG;
    const int nn = min(NG, B + 1 - n0);
    const int am = m < 0 ? -m : m;
    const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;  // Pbar_{l,-m} = (-1)^m Pbar_lm
    const double* P = gmem(C.P64) + table_block(B, am) + (int64_t)(l - am) * L;
    const double* R = gmem(C.R64) + table_block(B, l) + (int64_t)(n0 - l - 1) * L;
    const double2* tw = gmem(reinterpret_cast<const double2*>(C.tw));  // exp(-2 pi i q / L)
    const double2* s = samples + gmem(C.soff)[b];
    double ar[NG], ai[NG];
    for (int g = 0; g < NG; ++g) ar[g] = ai[g] = 0.0;
    const int L2 = L * L;
    const int npts = L2 * L;
    for (int p = threadIdx.x; p < npts; p += NT) {
      const int i = p / L2, jk = p - i * L2, j = jk / L, k = jk - j * L;
      double2 v = s[p];
      if (raw) {
        v.x *= gmem(C.sigma)[i];
        v.y *= gmem(C.sigma)[i];
      }
      const double wj = gmem(C.btilde)[j] * P[j] * sg;
      const double2 t = cmulc(v, tw[phase_index(m, k, L)]);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (g < nn) {
          const double rh = R[(int64_t)g * L + i] * wj;
          ar[g] += rh * t.x;
          ai[g] += rh * t.y;
        }
      }
    }
    for (int g = 0; g < nn; ++g) {
      const double sr = block_sum(ar[g], red);
      const double si = block_sum(ai[g], red);
      if (threadIdx.x == 0) coeffs[gmem(C.coff)[b] + omega(n0 + g, l, m)] = make_double2(sr * C.rs_fwd, si * C.rs_fwd);
    }
    __syncthreads();
  }
}

// n, l, m of a coefficient index omega (Sect. 3.4)
__device__ inline void decode_omega(int w, int& n, int& l, int& m) {
  n = (int)cbrt(3.0 * w) + 1;
  while (omega(n, 0, 0) > w) --n;
  while (omega(n + 1, 0, 0) <= w) ++n;
  const int r = w - (int)omega(n, 0, 0);
  l = (int)sqrt((double)r);
  while (l * l > r) --l;
  while ((l + 1) * (l + 1) <= r) ++l;
  m = r - l * (l + 1);
}

// Alg. 2.  Item of a class: function b, ring (i, j); threads take the ring's
// points k.  Coefficient chunks are staged in LDS with their radial and polar
// factors applied.
__global__ void __launch_bounds__(NT) k_naive_inverse(const ClassDesc* __restrict__ cls, const int64_t* __restrict__ pre,
                                                      int ncls, int64_t nitems, const double2* __restrict__ coeffs,
                                                      double2* __restrict__ samples, int raw) {
  __shared__ double2 Q[CH];
  __shared__ int Mq[CH];
  __shared__ double2 tws[512];
  int tw_cls = -1;
  for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int c = class_of(pre, ncls, w);
    const ClassDesc& C = cls[c];
    const int B = C.B, L = C.L;
    const int64_t r = w - pre[c];
    const int b = (int)(r / ((int64_t)L * L));
    const int ij = (int)(r - (int64_t)b * L * L);
    const int i = ij / L, j = ij - i * L;
    const int nco = (int)num_coeffs(B);
    if (c != tw_cls) {
      __syncthreads();
      const double2* tw = gmem(reinterpret_cast<const double2*>(C.tw));
      for (int q = threadIdx.x; q < L; q += NT) tws[q] = tw[q];
      tw_cls = c;
    }
    double2 acc0 = make_double2(0, 0), acc1 = make_double2(0, 0);
    const int k0 = threadIdx.x, k1 = threadIdx.x + NT;
    for (int w0 = 0; w0 < nco; w0 += CH) {
      const int cnt = min(CH, nco - w0);
      __syncthreads();
      for (int e = threadIdx.x; e < cnt; e += NT) {
        int n, l, m;
        decode_omega(w0 + e, n, l, m);
        const int am = m < 0 ? -m : m;
        const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
        const double f = sg * C.rs_inv * gmem(C.R64)[table_block(B, l) + (int64_t)(n - l - 1) * L + i] *
                         gmem(C.P64)[table_block(B, am) + (int64_t)(l - am) * L + j];
        const double2 x = coeffs[gmem(C.coff)[b] + w0 + e];
        Q[e] = make_double2(f * x.x, f * x.y);
        Mq[e] = m;
      }
      __syncthreads();
      for (int e = 0; e < cnt; ++e) {
        const double2 qv = Q[e];
        const int m = Mq[e];
        if (k0 < L) {
          const double2 t = tws[phase_index(m, k0, L)];  // conj gives exp(+i m ph_k)
          acc0.x += qv.x * t.x + qv.y * t.y;
          acc0.y += qv.y * t.x - qv.x * t.y;
        }
        if (k1 < L) {
          const double2 t = tws[phase_index(m, k1, L)];
          acc1.x += qv.x * t.x + qv.y * t.y;
          acc1.y += qv.y * t.x - qv.x * t.y;
        }
      }
    }
    double2* dst = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
    const double inv = raw ? 1.0 / gmem(C.sigma)[i] : 1.0;
    if (k0 < L) dst[k0] = make_double2(acc0.x * inv, acc0.y * inv);
    if (k1 < L) dst[k1] = make_double2(acc1.x * inv, acc1.y * inv);
  }
}

inline int grid_of(int64_t nitems) { return (int)(nitems < 65536 ? nitems : 65536); }

}  // namespace

int naive_group() { return NG; }

hipError_t launch_naive_forward(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                const void* samples, void* coeffs, bool raw, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_naive_forward, dim3(grid_of(nitems)), dim3(NT), 0, s, d_cls, d_pre, ncls, nitems,
                     reinterpret_cast<const double2*>(samples), reinterpret_cast<double2*>(coeffs), raw ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_naive_inverse(const ClassDesc* d_cls, const int64_t* d_pre, int ncls, int64_t nitems,
                                const void* coeffs, void* samples, bool raw, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_naive_inverse, dim3(grid_of(nitems)), dim3(NT), 0, s, d_cls, d_pre, ncls, nitems,
                     reinterpret_cast<const double2*>(coeffs), reinterpret_cast<double2*>(samples), raw ? 1 : 0);
  return hipGetLastError();
}

}  // namespace sgl
