// Stage (a): azimuthal DFT of every (r_i, theta_j) ring (Sect. 3.3.1, Eq.
// SFFT_rearranged inner sum; inverse: Eq. iSFFT_rearranged outer sum).
//
// Forward:  F[m][j][b,i] = w_j * sum_k s_b[i][j][k] exp(-2 pi i m k / 2B),
//           m = 1-B .. B-1 (bin +-B is not used by any coefficient),
//           w_j = b~_j (times sigma_i for raw samples).
// Inverse:  s_b[i][j][k] = sum_{m=1-B}^{B-1} F[m][j][b,i] exp(+2 pi i m k / 2B)
//           (divided by sigma_i for raw samples).
//
// One block handles RPB rings that share j and have consecutive columns
// (b, i); the rings are read (or written) contiguously, transformed by a
// mixed-radix Stockham FFT in LDS (twiddles from an FP64-built table), and the
// spectrum is written transposed to F[m][j][col], which is the operand layout
// of the Legendre stage.  Bandwidth-bound: every sample is read once and every
// spectral value written once.
#include "sgl_internal.h"

namespace sgl {
namespace {

template <typename T> struct C2;
template <> struct C2<double> { using t = double2; };
template <> struct C2<float> { using t = float2; };

template <typename T2>
__device__ inline T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T2>
__device__ inline T2 cadd(T2 a, T2 b) { T2 r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename T2>
__device__ inline T2 csub(T2 a, T2 b) { T2 r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename T2>
__device__ inline T2 conjc(T2 a) { a.y = -a.y; return a; }

// twiddle exp(sign 2 pi i q / L) from the forward table exp(-2 pi i q / L)
template <typename T2, bool INV>
__device__ inline T2 twid(const T2* tw, int q) {
  T2 w = tw[q];
  return INV ? conjc(w) : w;
}

// One Stockham stage of radix R over `nring` rings of length L held in LDS.
template <typename T2, bool INV>
__device__ void stockham_stage(const T2* in, T2* out, const T2* tw, int L, int R, int Ns, int nring) {
  const int nbf = L / R;
  const int total = nring * nbf;
  const int LR = L / R;
  for (int bf = threadIdx.x; bf < total; bf += blockDim.x) {
    const int ring = bf / nbf;
    const int j = bf - ring * nbf;
    const T2* src = in + ring * L;
    T2* dst = out + ring * L;
    const int jm = j % Ns;
    const int idxD = (j / Ns) * Ns * R + jm;
    const int tstep = jm * (L / (Ns * R));  // twiddle index step per r
    if (R == 4) {
      T2 a = src[j];
      T2 b = cmul(src[j + LR], twid<T2, INV>(tw, tstep));
      T2 c = cmul(src[j + 2 * LR], twid<T2, INV>(tw, 2 * tstep));
      T2 d = cmul(src[j + 3 * LR], twid<T2, INV>(tw, 3 * tstep));
      T2 s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = csub(b, d);
      // forward: V1 = s1 - i s3, V3 = s1 + i s3; inverse: swapped
      T2 is3;
      is3.x = -s3.y;
      is3.y = s3.x;
      dst[idxD] = cadd(s0, s2);
      dst[idxD + 2 * Ns] = csub(s0, s2);
      if (INV) {
        dst[idxD + Ns] = cadd(s1, is3);
        dst[idxD + 3 * Ns] = csub(s1, is3);
      } else {
        dst[idxD + Ns] = csub(s1, is3);
        dst[idxD + 3 * Ns] = cadd(s1, is3);
      }
    } else if (R == 2) {
      T2 a = src[j];
      T2 b = cmul(src[j + LR], twid<T2, INV>(tw, tstep));
      dst[idxD] = cadd(a, b);
      dst[idxD + Ns] = csub(a, b);
    } else {
      // general radix: direct R-point DFT of the twiddled inputs
      for (int q = 0; q < R; ++q) {
        T2 acc;
        acc.x = 0;
        acc.y = 0;
        for (int r = 0; r < R; ++r) {
          T2 v = cmul(src[j + r * LR], twid<T2, INV>(tw, (r * tstep) % L));
          acc = cadd(acc, cmul(v, twid<T2, INV>(tw, ((r * q) % R) * LR)));
        }
        dst[idxD + q * Ns] = acc;
      }
    }
  }
}

template <typename T, bool RAW>
__global__ void __launch_bounds__(256) k_fft_forward(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                                     int nwork, const void* __restrict__ samples_v) {
  using T2 = typename C2<T>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* smem = reinterpret_cast<T2*>(smem_raw);
  const T2* samples = reinterpret_cast<const T2*>(samples_v);
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    const int B = C.B, L = C.L, j = it.y;
    const int ncol = C.nf * L;
    const int rpb = it.w;
    const int col0 = it.z * rpb;
    const int nr = min(rpb, ncol - col0);
    T2* buf0 = smem;
    T2* buf1 = smem + rpb * L;
    for (int e = threadIdx.x; e < nr * L; e += blockDim.x) {
      const int r = e / L, k = e - r * L;
      const int col = col0 + r;
      const int b = col / L, i = col - b * L;
      T2 v = samples[C.soff[b] + ((int64_t)i * L + j) * L + k];
      if (RAW) {
        const T sg = (T)C.sigma[i];
        v.x *= sg;
        v.y *= sg;
      }
      buf0[r * L + k] = v;
    }
    __syncthreads();
    const T2* tw = reinterpret_cast<const T2*>(C.tw);
    T2* cur = buf0;
    T2* nxt = buf1;
    int Ns = 1;
    for (int t = 0; t < C.nrad; ++t) {
      const int R = C.rad[t];
      stockham_stage<T2, false>(cur, nxt, tw, L, R, Ns, nr);
      __syncthreads();
      T2* tmp = cur;
      cur = nxt;
      nxt = tmp;
      Ns *= R;
    }
    const T wj = (T)C.btilde[j];
    T2* F = reinterpret_cast<T2*>(C.F);
    const int nm = 2 * B - 1;
    for (int e = threadIdx.x; e < nm * nr; e += blockDim.x) {
      const int mi = e / nr, r = e - mi * nr;
      const int m = mi - (B - 1);
      const int bin = m >= 0 ? m : L + m;
      T2 v = cur[r * L + bin];
      v.x *= wj;
      v.y *= wj;
      F[((int64_t)mi * L + j) * ncol + col0 + r] = v;
    }
    __syncthreads();
  }
}

template <typename T, bool RAW>
__global__ void __launch_bounds__(256) k_fft_inverse(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                                     int nwork, void* __restrict__ samples_v) {
  using T2 = typename C2<T>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* smem = reinterpret_cast<T2*>(smem_raw);
  T2* samples = reinterpret_cast<T2*>(samples_v);
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    const int B = C.B, L = C.L, j = it.y;
    const int ncol = C.nf * L;
    const int rpb = it.w;
    const int col0 = it.z * rpb;
    const int nr = min(rpb, ncol - col0);
    T2* buf0 = smem;
    T2* buf1 = smem + rpb * L;
    const T2* F = reinterpret_cast<const T2*>(C.F);
    // bins B (not produced by any coefficient) start at zero
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      T2 z;
      z.x = 0;
      z.y = 0;
      buf0[r * L + B] = z;
    }
    const int nm = 2 * B - 1;
    for (int e = threadIdx.x; e < nm * nr; e += blockDim.x) {
      const int mi = e / nr, r = e - mi * nr;
      const int m = mi - (B - 1);
      const int bin = m >= 0 ? m : L + m;
      buf0[r * L + bin] = F[((int64_t)mi * L + j) * ncol + col0 + r];
    }
    __syncthreads();
    const T2* tw = reinterpret_cast<const T2*>(C.tw);
    T2* cur = buf0;
    T2* nxt = buf1;
    int Ns = 1;
    for (int t = 0; t < C.nrad; ++t) {
      const int R = C.rad[t];
      stockham_stage<T2, true>(cur, nxt, tw, L, R, Ns, nr);
      __syncthreads();
      T2* tmp = cur;
      cur = nxt;
      nxt = tmp;
      Ns *= R;
    }
    for (int e = threadIdx.x; e < nr * L; e += blockDim.x) {
      const int r = e / L, k = e - r * L;
      const int col = col0 + r;
      const int b = col / L, i = col - b * L;
      T2 v = cur[r * L + k];
      if (RAW) {
        const T sg = (T)(1.0 / C.sigma[i]);
        v.x *= sg;
        v.y *= sg;
      }
      samples[C.soff[b] + ((int64_t)i * L + j) * L + k] = v;
    }
    __syncthreads();
  }
}

inline int grid_for(int nwork) { return nwork < 4096 ? nwork : 4096; }

}  // namespace

// LDS bytes for rings_per_block rings of length L in the given precision
static size_t fft_lds_bytes(int prec, int rpb, int Lmax) {
  return (size_t)2 * rpb * Lmax * (prec == PREC_F64 ? sizeof(double2) : sizeof(float2));
}

hipError_t launch_fft_forward(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, const void* samples, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  dim3 grid(grid_for(nwork)), block(256);
  if (prec == PREC_F64) {
    if (raw)
      hipLaunchKernelGGL((k_fft_forward<double, true>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
    else
      hipLaunchKernelGGL((k_fft_forward<double, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
  } else {
    hipLaunchKernelGGL((k_fft_forward<float, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
  }
  return hipGetLastError();
}

hipError_t launch_fft_inverse(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, void* samples, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  dim3 grid(grid_for(nwork)), block(256);
  if (prec == PREC_F64) {
    if (raw)
      hipLaunchKernelGGL((k_fft_inverse<double, true>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
    else
      hipLaunchKernelGGL((k_fft_inverse<double, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
  } else {
    hipLaunchKernelGGL((k_fft_inverse<float, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork, samples);
  }
  return hipGetLastError();
}

size_t fft_lds_bytes_for(int prec, int rpb, int L) { return fft_lds_bytes(prec, rpb, L); }

}  // namespace sgl
