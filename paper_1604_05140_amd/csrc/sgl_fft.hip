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
#include "sgl_wave.h"

namespace sgl {
namespace {

// One Stockham stage of radix R over `nring` rings of length L held in LDS.
template <typename T2, bool INV>
__device__ void stockham_stage(const T2* in, T2* out, const SGL_G T2* tw, int L, int R, int Ns, int nring) {
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

// ---------------------------------------------------------------------------
// Power-of-two rings (L = 16 .. 256): register four-step FFT.
//   x[R2 n1 + n2], X[k1 + R1 k2]:  X = DFT_R2 over n2 of ( w_L^{n2 k1} * DFT_R1 over n1 ),
// pass 1 holds one n2 column (R1 values) per thread, pass 2 one k1 row (R2
// values); the exchange goes through LDS laid out [k1][n2][ring] so that both
// passes access it without bank conflicts, and the ring index is the fastest
// lane index in pass 2, so spectral values of RPB consecutive columns leave in
// one contiguous run per (m, j).
// ---------------------------------------------------------------------------

// Exchange pitch (complex values per [k1][n2] row of the [k1][n2][ring] layout)
// of the register four-step FFT.  In single precision it is chosen per ring
// length and direction so that both passes' 8-byte LDS accesses are free of
// bank conflicts under the measured gfx950 rules (reads: 32 consecutive lanes
// over 64 banks; writes: 16 consecutive lanes over 32 banks): the forward
// writes with the n2 index fastest and reads with the ring fastest, the inverse
// the other way round.  FP64 (16-byte values) keeps rpb + 1.
__host__ __device__ constexpr int pow2_pitch_extra(int L, bool f64, bool inv) {
  return f64 ? 1 : (inv ? (L >= 256 ? 2 : (L >= 64 ? 4 : 8)) : (L >= 256 ? 1 : (L >= 64 ? 2 : 4)));
}
// the larger of the two directions' pitches (the twiddle table follows the buffer)
__host__ __device__ constexpr int pow2_pitch_max_extra(int L, bool f64) {
  return pow2_pitch_extra(L, f64, true) > pow2_pitch_extra(L, f64, false) ? pow2_pitch_extra(L, f64, true)
                                                                         : pow2_pitch_extra(L, f64, false);
}

template <typename T, int R1, int R2, bool RAW>
__device__ inline void fwd_pow2(const ClassDesc& C, int j, int col0, int nr, int rpb,
                                const SGL_G typename C2<T>::t* __restrict__ samples, typename C2<T>::t* lds,
                                const typename C2<T>::t* tw) {
  using T2 = typename C2<T>::t;
  constexpr int L = R1 * R2, B = L / 2;
  const int t = threadIdx.x;
  const int P = rpb + pow2_pitch_extra(L, sizeof(T) == 8, false);
  if (t < rpb * R2) {
    const int r = t / R2, n2 = t % R2;
    if (r < nr) {
      const int col = col0 + r;
      const int b = col / L, i = col % L;
      const SGL_G T2* src = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
      T2 v[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) v[n1] = load_stream(&src[R2 * n1 + n2]);
      if (RAW) {
        const T sg = (T)gmem(C.sigma)[i];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) {
          v[n1].x *= sg;
          v[n1].y *= sg;
        }
      }
      dft_reg<T2, R1, false>(v);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        const T2 w = k1 == 0 ? v[k1] : cmul(v[k1], tw[(n2 * k1) % L]);
        lds[(k1 * R2 + n2) * P + r] = w;
      }
    }
  }
  __syncthreads();
  if (t < rpb * R1) {
    const int r = t % rpb, k1 = t / rpb;
    if (r < nr) {
      T2 y[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) y[n2] = lds[(k1 * R2 + n2) * P + r];
      dft_reg<T2, R2, false>(y);
      const T wj = (T)gmem(C.btilde)[j];
      const int ncol = C.nf * L;
      SGL_G T2* F = gmem(reinterpret_cast<T2*>(C.F));
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int bin = k1 + R1 * k2;
        if (bin == B) continue;
        const int mi = (bin < B ? bin : bin - L) + B - 1;
        T2 o = y[k2];
        o.x *= wj;
        o.y *= wj;
        store_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r], o);
      }
    }
  }
  __syncthreads();
}

template <typename T, int R1, int R2, bool RAW>
__device__ inline void inv_pow2(const ClassDesc& C, int j, int col0, int nr, int rpb,
                                SGL_G typename C2<T>::t* __restrict__ samples, typename C2<T>::t* lds,
                                const typename C2<T>::t* tw) {
  using T2 = typename C2<T>::t;
  constexpr int L = R1 * R2, B = L / 2;
  const int t = threadIdx.x;
  const int P = rpb + pow2_pitch_extra(L, sizeof(T) == 8, true);
  if (t < rpb * R1) {
    const int r = t % rpb, k1 = t / rpb;
    if (r < nr) {
      const int ncol = C.nf * L;
      const SGL_G T2* F = gmem(reinterpret_cast<const T2*>(C.F));
      T2 y[R2];
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int bin = k1 + R1 * k2;
        if (bin == B) {
          y[k2].x = 0;
          y[k2].y = 0;
        } else {
          const int mi = (bin < B ? bin : bin - L) + B - 1;
          y[k2] = load_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r]);
        }
      }
      dft_reg<T2, R2, true>(y);
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) {
        const T2 w = n2 == 0 ? y[n2] : cmul(y[n2], conjc(tw[(n2 * k1) % L]));
        lds[(k1 * R2 + n2) * P + r] = w;
      }
    }
  }
  __syncthreads();
  if (t < rpb * R2) {
    const int r = t / R2, n2 = t % R2;
    if (r < nr) {
      T2 v[R1];
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[k1] = lds[(k1 * R2 + n2) * P + r];
      dft_reg<T2, R1, true>(v);
      const int col = col0 + r;
      const int b = col / L, i = col % L;
      SGL_G T2* dst = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
      if (RAW) {
        const T sg = (T)(1.0 / gmem(C.sigma)[i]);
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) {
          v[n1].x *= sg;
          v[n1].y *= sg;
        }
      }
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) store_stream(&dst[R2 * n1 + n2], v[n1]);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Other ring lengths 6 <= L <= 254: Bluestein's chirp-z form on a
// power-of-two FFT of length M = 2^k >= 2L - 1 (M <= 256 here, on the register
// four-step FFT; M = 512 on the one-wavefront kernels further down):
//   X_m = c_m sum_k (x_k c_k) conj(c_{m-k}),  c_p = exp(-i pi p^2 / L),
// i.e. a cyclic convolution of length M computed as IFFT_M(FFT_M(a) * BH) with
// the kernel spectrum BH precomputed (1/M folded in).  The inverse DFT uses
// conj(c) and the conjugate kernel.  Per ring set: load and twist into LDS,
// FFT_M pass 1, exchange, pass 2 (times BH) + inverse pass A in registers,
// exchange, inverse pass B, untwist and store.  One LDS buffer of
// M x (RPB+1) complex holds the natural-order rings and both exchanges.
// ---------------------------------------------------------------------------
template <typename T, int R1, int R2, bool INV>
__device__ inline void blue_core(int rpb, int nr, typename C2<T>::t* buf, const typename C2<T>::t* twM,
                                 const typename C2<T>::t* bh, int out_r_fastest, typename C2<T>::t (&res)[R1]) {
  // buf holds rings in natural order [r][M]; on return thread (r, n2) of the
  // final pass holds z[R2 n1 + n2] in res[n1] (mapping chosen by out_r_fastest).
  using T2 = typename C2<T>::t;
  constexpr int M = R1 * R2;
  const int t = threadIdx.x;
  const int P = rpb + 1;
  T2 v[R1];
  const bool p1 = t < rpb * R2;
  const int r1 = t / R2, n21 = t % R2;
  if (p1 && r1 < nr) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) v[n1] = buf[r1 * M + R2 * n1 + n21];
  }
  __syncthreads();  // natural-order data consumed; buf becomes the exchange area
  if (p1 && r1 < nr) {
    dft_reg<T2, R1, false>(v);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      const T2 w = k1 == 0 ? v[k1] : cmul(v[k1], twM[(n21 * k1) % M]);
      buf[(k1 * R2 + n21) * P + r1] = w;
    }
  }
  __syncthreads();
  const int r2 = t % rpb, k1 = t / rpb;
  T2 y[R2];
  const bool p2 = t < rpb * R1;
  if (p2 && r2 < nr) {
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) y[n2] = buf[(k1 * R2 + n2) * P + r2];
  }
  __syncthreads();  // exchange consumed before it is rewritten
  if (p2 && r2 < nr) {
    dft_reg<T2, R2, false>(y);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[k2] = cmul(y[k2], bh[k1 + R1 * k2]);
    dft_reg<T2, R2, true>(y);
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      const T2 w = n2 == 0 ? y[n2] : cmul(y[n2], conjc(twM[(n2 * k1) % M]));
      buf[(k1 * R2 + n2) * P + r2] = w;
    }
  }
  __syncthreads();
  const int rB = out_r_fastest ? t % rpb : t / R2;
  const int n2B = out_r_fastest ? t / rpb : t % R2;
  if (t < rpb * R2 && rB < nr) {
#pragma unroll
    for (int q = 0; q < R1; ++q) res[q] = buf[(q * R2 + n2B) * P + rB];
    dft_reg<T2, R1, true>(res);
  }
}

template <typename T, int R1, int R2, bool RAW>
__device__ inline void fwd_blue(const ClassDesc& C, int j, int col0, int nr, int rpb,
                                const SGL_G typename C2<T>::t* __restrict__ samples, typename C2<T>::t* buf,
                                const typename C2<T>::t* twM, const typename C2<T>::t* chirp,
                                const typename C2<T>::t* bh) {
  using T2 = typename C2<T>::t;
  constexpr int M = R1 * R2;
  const int L = C.L, B = C.B;
  // four loads per thread in flight before any is used (indices past the ring set or the ring
  // length load a valid sample and are replaced by zero or skipped)
  const int ne = nr * M;
  for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
    T2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = min(e0 + q * (int)blockDim.x, ne - 1);
      const int r = e / M, k = e - r * M;
      const int col = col0 + r;
      const int b = col / L, i = col - b * L;
      v[q] = load_stream(&samples[gmem(C.soff)[b] + ((int64_t)i * L + j) * L + min(k, L - 1)]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + q * (int)blockDim.x;
      if (e >= ne) break;
      const int r = e / M, k = e - r * M;
      T2 w;
      w.x = 0;
      w.y = 0;
      if (k < L) {
        w = cmul(v[q], chirp[k]);
        if (RAW) {
          const T sg = (T)gmem(C.sigma)[(col0 + r) % L];
          w.x *= sg;
          w.y *= sg;
        }
      }
      buf[r * M + k] = w;
    }
  }
  __syncthreads();
  T2 z[R1];
  blue_core<T, R1, R2, false>(rpb, nr, buf, twM, bh, 1, z);
  const int t = threadIdx.x;
  const int r = t % rpb, n2 = t / rpb;
  if (t < rpb * R2 && r < nr) {
    const T wj = (T)gmem(C.btilde)[j];
    const int ncol = C.nf * L;
    SGL_G T2* F = gmem(reinterpret_cast<T2*>(C.F));
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      const int idx = R2 * n1 + n2;
      if (idx >= L || idx == B) continue;
      const int mi = (idx < B ? idx : idx - L) + B - 1;
      T2 o = cmul(z[n1], chirp[idx]);
      o.x *= wj;
      o.y *= wj;
      store_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r], o);
    }
  }
  __syncthreads();
}

template <typename T, int R1, int R2, bool RAW>
__device__ inline void inv_blue(const ClassDesc& C, int j, int col0, int nr, int rpb,
                                SGL_G typename C2<T>::t* __restrict__ samples, typename C2<T>::t* buf,
                                const typename C2<T>::t* twM, const typename C2<T>::t* chirp,
                                const typename C2<T>::t* bh) {
  using T2 = typename C2<T>::t;
  constexpr int M = R1 * R2;
  const int L = C.L, B = C.B;
  const int ncol = C.nf * L;
  const SGL_G T2* F = gmem(reinterpret_cast<const T2*>(C.F));
  // bins p < L in the ring-fastest order of F rows, twisted by conj(c_p)
  // four loads per thread in flight before any is used (bin B loads a valid row and is zeroed)
  const int ne = nr * L;
  for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
    T2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = min(e0 + q * (int)blockDim.x, ne - 1);
      const int p = e / nr, r = e - p * nr;
      const int pc = p == B ? 0 : p;
      const int mi = (pc < B ? pc : pc - L) + B - 1;
      v[q] = load_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + q * (int)blockDim.x;
      if (e >= ne) break;
      const int p = e / nr, r = e - p * nr;
      T2 w = cmul(v[q], conjc(chirp[p]));
      if (p == B) w.x = w.y = 0;
      buf[r * M + p] = w;
    }
  }
  for (int e = threadIdx.x; e < nr * (M - L); e += blockDim.x) {
    const int r = e / (M - L), p = L + e - r * (M - L);
    T2 z;
    z.x = 0;
    z.y = 0;
    buf[r * M + p] = z;
  }
  __syncthreads();
  T2 z[R1];
  blue_core<T, R1, R2, true>(rpb, nr, buf, twM, bh, 0, z);
  const int t = threadIdx.x;
  const int r = t / R2, n2 = t % R2;
  if (t < rpb * R2 && r < nr) {
    const int col = col0 + r;
    const int b = col / L, i = col - b * L;
    SGL_G T2* dst = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
    const T sg = RAW ? (T)(1.0 / gmem(C.sigma)[i]) : (T)1;
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      const int idx = R2 * n1 + n2;
      if (idx >= L) continue;
      T2 o = cmul(z[n1], conjc(chirp[idx]));
      if (RAW) {
        o.x *= sg;
        o.y *= sg;
      }
      store_stream(&dst[idx], o);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// 512-point transforms with one wavefront per ring: rings of length 512, and
// Bluestein rings whose convolution length is 512 (130 <= L <= 254).
// Lane l holds x[64 a + l] in v[a]; three radix-8 passes:
//   1: DFT_8 over a -> p, times w_512^(l p);
//   2: lane 8p + c (c = l mod 8 in pass 1) holds b = 0..7: DFT_8 over b -> q,
//      times w_64^(c q);
//   3: lane 8q + p holds c = 0..7: DFT_8 over c -> s, giving
//      X[p + 8q + 64s] = X[lane + 64s].
// Input and output share the natural lane order, so the forward transform,
// the kernel product and the inverse transform of a Bluestein convolution
// follow one another in registers.  The two exchanges go through an LDS area
// private to the wavefront, in XOR layouts that are free of bank conflicts
// for 8- and 16-byte elements, so they need ordering at wavefront scope only.
// A block is 16 wavefronts = 16 rings of consecutive columns; their areas
// also stage the spectrum rows, which are read and written in runs of 16
// columns.
// ---------------------------------------------------------------------------
constexpr int kRings512 = 16;  // rings (wavefronts) per block

// LDS tables ahead of the ring areas (small offsets, so that table reads take
// immediate offsets): w_512^(l p) at (p-1) 64 + l (p = 1..7), w_64^(c q) at
// 448 + 8 (q-1) + c, the Bluestein kernel spectrum for k = 0..256 at 504 (it is
// even in k: BH[512 - k] = BH[k]), the chirp at 761 (256 values, zero from L on).
constexpr int kTabKer = 504, kTabChirp = 761, kTab512 = 1017;  // kTabTw2 = 448 in sgl_wave.h

// Fill the block's 512-point tables for class C (block-wide; ends synchronised).
template <typename T2>
__device__ inline void load_tab512(const ClassDesc& C, const void* kernel_spectrum, T2* tab) {
  const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.M ? C.twM : C.tw));  // exp(-2 pi i q / 512)
  for (int q = threadIdx.x; q < 448; q += blockDim.x) {
    const int p = q / 64 + 1, l = q % 64;
    tab[q] = tw[(l * p) % 512];
  }
  for (int q = threadIdx.x; q < 56; q += blockDim.x) {
    const int e = q / 8 + 1, c = q % 8;
    tab[kTabTw2 + q] = tw[8 * ((c * e) % 64)];  // w_64^(c e)
  }
  if (C.M) {
    const SGL_G T2* bh = gmem(reinterpret_cast<const T2*>(kernel_spectrum));
    for (int q = threadIdx.x; q <= 256; q += blockDim.x) tab[kTabKer + q] = bh[q];
    const SGL_G T2* ch = gmem(reinterpret_cast<const T2*>(C.chirp));
    for (int q = threadIdx.x; q < 256; q += blockDim.x) {
      const T2 c = ch[min(q, C.L - 1)];
      const bool in = q < C.L;
      T2 o;
      o.x = in ? c.x : 0;
      o.y = in ? c.y : 0;
      tab[kTabChirp + q] = o;
    }
  }
  __syncthreads();
}

// Bluestein kernel product in registers: v[s] holds bin l + 64 s.
template <typename T2>
__device__ inline void kernel_product(T2 (&v)[8], const T2* tab, int l) {
  const T2* lo = tab + kTabKer + l;       // bins l + 64 s, s < 4
  const T2* hi = tab + kTabKer + 64 - l;  // bins 512 - (l + 64 s) = 64 - l + 64 (7 - s), s >= 4
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = cmul(v[s], s < 4 ? lo[64 * s] : hi[64 * (7 - s)]);
}

template <typename T, bool RAW>
__device__ inline void fwd512(const ClassDesc& C, int j, int col0, int nr, const SGL_G typename C2<T>::t* __restrict__ samples,
                              const typename C2<T>::t* tab, typename C2<T>::t* smem) {
  using T2 = typename C2<T>::t;
  constexpr int P = area_pitch<T2>();
  const int L = C.L, B = C.B;
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  T2* area = smem + wv * P;
  const T wj = (T)gmem(C.btilde)[j];
  if (wv < nr) {
    const int col = col0 + wv;
    const int b = col / L, i = col - b * L;
    const SGL_G T2* src = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
    const T sg = RAW ? (T)gmem(C.sigma)[i] : (T)1;
    T2 v[8];
    if (!C.M) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        v[a] = load_stream(&src[64 * a + l]);
        if (RAW) {
          v[a].x *= sg;
          v[a].y *= sg;
        }
      }
      fft512_wave<T2, false>(v, area, tab, l);
    } else {
      const T2* ch = tab + kTabChirp;
      // bins k >= L are zero (L <= 254: only a < 4 can hold data): loads are
      // clamped into the ring, and the chirp table is zero from L on
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int k = 64 * a + l;
        v[a] = cmul(load_stream(&src[min(k, L - 1)]), ch[k]);
        if (RAW) {
          v[a].x *= sg;
          v[a].y *= sg;
        }
      }
#pragma unroll
      for (int a = 4; a < 8; ++a) v[a].x = v[a].y = 0;
      fft512_wave<T2, false, true>(v, area, tab, l);
      kernel_product(v, tab, l);
      fft512_wave<T2, true, false, true>(v, area, tab, l);
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = cmul(v[s], ch[64 * s + l]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 64 * s + l;
      if (k < L) {
        T2 o = v[s];
        o.x *= wj;
        o.y *= wj;
        area[k] = o;
      }
    }
  }
  __syncthreads();
  // spectrum rows out: thread (row, r) = (tid / 16, tid % 16) takes rows
  // row, row + 64, ... of column r, so each row leaves as one 16-column run
  const int r = threadIdx.x & (kRings512 - 1);
  if (r < nr) {
    const int ncol = C.nf * L;
    const int nm = 2 * B - 1;
    const int64_t step = (int64_t)(blockDim.x / kRings512) * L * ncol;
    const T2* stage = smem + r * P;
    int mi = threadIdx.x / kRings512;
    SGL_G T2* dst = gmem(reinterpret_cast<T2*>(C.F)) + ((int64_t)mi * L + j) * ncol + col0 + r;
    for (; mi < nm; mi += blockDim.x / kRings512, dst += step) {
      const int m = mi - (B - 1);
      store_stream(dst, stage[m >= 0 ? m : L + m]);
    }
  }
  __syncthreads();
}

template <typename T, bool RAW>
__device__ inline void inv512(const ClassDesc& C, int j, int col0, int nr, SGL_G typename C2<T>::t* __restrict__ samples,
                              const typename C2<T>::t* tab, typename C2<T>::t* smem) {
  using T2 = typename C2<T>::t;
  constexpr int P = area_pitch<T2>();
  const int L = C.L, B = C.B;
  const SGL_G T2* F = gmem(reinterpret_cast<const T2*>(C.F));
  const int ncol = C.nf * L;
  const T2* ch = tab + kTabChirp;
  // spectrum rows -> ring areas; bin B (which no coefficient produces) and,
  // for Bluestein rings, the padding bins L..255 are zero
  const int nb = C.M ? 256 : L;
  {
    const int r = threadIdx.x & (kRings512 - 1);
    if (r < nr) {
      T2* stage = smem + r * P;
      const SGL_G T2* src = F + (int64_t)j * ncol + col0 + r;
      const int64_t row = (int64_t)L * ncol;
      // thread rows p0 + 64 s; all loads of a thread are issued before any is used (bin B and the
      // Bluestein padding bins p >= L load a valid row and are set to zero)
      // (groups of four rows: the single-precision kernel keeps to 64 registers)
      constexpr int kStep = fft_threads(1, false) / kRings512, kGroup = 4;
      const int p0 = threadIdx.x / kRings512;
      for (int g0 = 0; g0 < nb; g0 += kGroup * kStep) {
        T2 v[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
          const int p = g0 + p0 + kStep * q;
          const int pc = (p != B && p < L) ? p : 0;
          const int mi = (pc < B ? pc : pc - L) + B - 1;
          v[q] = load_stream(&src[mi * row]);
        }
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
          const int p = g0 + p0 + kStep * q;
          T2 w = v[q];
          if (C.M) w = cmul(w, conjc(ch[p]));
          if (p == B || p >= L) w.x = w.y = 0;
          stage[p] = w;
        }
      }
    }
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  T2* area = smem + wv * P;
  if (wv < nr) {
    const int col = col0 + wv;
    const int b = col / L, i = col - b * L;
    SGL_G T2* dst = samples + gmem(C.soff)[b] + ((int64_t)i * L + j) * L;
    const T sg = RAW ? (T)(1.0 / gmem(C.sigma)[i]) : (T)1;
    T2 v[8];
    if (!C.M) {
#pragma unroll
      for (int a = 0; a < 8; ++a) v[a] = area[64 * a + l];
      fft512_wave<T2, true>(v, area, tab, l);
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) v[a] = area[64 * a + l];
#pragma unroll
      for (int a = 4; a < 8; ++a) v[a].x = v[a].y = 0;
      fft512_wave<T2, false, true>(v, area, tab, l);
      kernel_product(v, tab, l);
      fft512_wave<T2, true, false, true>(v, area, tab, l);
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = cmul(v[s], conjc(ch[64 * s + l]));
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 64 * s + l;
      if (k < L) {
        T2 o = v[s];
        if (RAW) {
          o.x *= sg;
          o.y *= sg;
        }
        store_stream(&dst[k], o);
      }
    }
  }
  __syncthreads();
}

// MODE 0: power-of-two rings up to 256 points and the generic path; MODE 1:
// 512-point rings and Bluestein length 512, one wavefront per ring; MODE 2:
// Bluestein rings with M <= 256.  Each mode is its own kernel so that it gets
// only the registers its FFT size needs.
template <typename T, bool RAW, int MODE>
__global__ void __launch_bounds__(fft_threads(MODE, sizeof(T) == 8), fft_min_waves(MODE, sizeof(T) == 8)) k_fft_forward(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                                     int nwork, const void* __restrict__ samples_v) {
  using T2 = typename C2<T>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* smem = reinterpret_cast<T2*>(smem_raw);
  const SGL_G T2* samples = gmem(reinterpret_cast<const T2*>(samples_v));
  int tw_cls = -1;  // class whose twiddles sit in LDS (block-uniform)
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    const int B = C.B, L = C.L, j = it.y;
    const int ncol = C.nf * L;
    const int rpb = it.w;
    const int col0 = it.z * rpb;
    const int nr = min(rpb, ncol - col0);
    if constexpr (MODE == 1) {
      if (it.x != tw_cls) {
        load_tab512<T2>(C, C.bhf, smem);
        tw_cls = it.x;
      }
      fwd512<T, RAW>(C, j, col0, nr, samples, smem, smem + kTab512);
      continue;
    }
    if (MODE == 0 && fft_pow2_path(L)) {
      T2* twl = smem + L * (rpb + pow2_pitch_max_extra(L, sizeof(T) == 8));
      if (it.x != tw_cls) {
        const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.tw));
        for (int q = threadIdx.x; q < L; q += blockDim.x) twl[q] = tw[q];
        __syncthreads();
        tw_cls = it.x;
      }
      {
        if constexpr (MODE == 0) switch (L) {
          case 16: fwd_pow2<T, 4, 4, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 32: fwd_pow2<T, 8, 4, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 64: fwd_pow2<T, 8, 8, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 128: fwd_pow2<T, 16, 8, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          default: fwd_pow2<T, 16, 16, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
        }
      }
      continue;
    }
    if (MODE != 0 && C.M) {
      const int M = C.M;
      T2* tws = smem + M * (rpb + 1);
      T2* chs = tws + M;
      T2* bhs = chs + L;
      if (it.x != tw_cls) {
        const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.twM));
        const SGL_G T2* ch = gmem(reinterpret_cast<const T2*>(C.chirp));
        const SGL_G T2* bh = gmem(reinterpret_cast<const T2*>(C.bhf));
        for (int q = threadIdx.x; q < M; q += blockDim.x) {
          tws[q] = tw[q];
          bhs[q] = bh[q];
        }
        for (int q = threadIdx.x; q < L; q += blockDim.x) chs[q] = ch[q];
        __syncthreads();
        tw_cls = it.x;
      }
      {
        if constexpr (MODE == 2) switch (M) {
          case 16: fwd_blue<T, 4, 4, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 32: fwd_blue<T, 8, 4, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 64: fwd_blue<T, 8, 8, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 128: fwd_blue<T, 16, 8, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          default: fwd_blue<T, 16, 16, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
        }
      }
      continue;
    }
    if constexpr (MODE != 0) continue;
    T2* buf0 = smem;
    T2* buf1 = smem + rpb * L;
    for (int e = threadIdx.x; e < nr * L; e += blockDim.x) {
      const int r = e / L, k = e - r * L;
      const int col = col0 + r;
      const int b = col / L, i = col - b * L;
      T2 v = load_stream(&samples[gmem(C.soff)[b] + ((int64_t)i * L + j) * L + k]);
      if (RAW) {
        const T sg = (T)gmem(C.sigma)[i];
        v.x *= sg;
        v.y *= sg;
      }
      buf0[r * L + k] = v;
    }
    __syncthreads();
    const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.tw));
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
    const T wj = (T)gmem(C.btilde)[j];
    SGL_G T2* F = gmem(reinterpret_cast<T2*>(C.F));
    const int nm = 2 * B - 1;
    for (int e = threadIdx.x; e < nm * nr; e += blockDim.x) {
      const int mi = e / nr, r = e - mi * nr;
      const int m = mi - (B - 1);
      const int bin = m >= 0 ? m : L + m;
      T2 v = cur[r * L + bin];
      v.x *= wj;
      v.y *= wj;
      store_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r], v);
    }
    __syncthreads();
  }
}

template <typename T, bool RAW, int MODE>
__global__ void __launch_bounds__(fft_threads(MODE, sizeof(T) == 8), fft_min_waves(MODE, sizeof(T) == 8)) k_fft_inverse(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                                     int nwork, void* __restrict__ samples_v) {
  using T2 = typename C2<T>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* smem = reinterpret_cast<T2*>(smem_raw);
  SGL_G T2* samples = gmem(reinterpret_cast<T2*>(samples_v));
  int tw_cls = -1;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    const int B = C.B, L = C.L, j = it.y;
    const int ncol = C.nf * L;
    const int rpb = it.w;
    const int col0 = it.z * rpb;
    const int nr = min(rpb, ncol - col0);
    if constexpr (MODE == 1) {
      if (it.x != tw_cls) {
        load_tab512<T2>(C, C.bhi, smem);
        tw_cls = it.x;
      }
      inv512<T, RAW>(C, j, col0, nr, samples, smem, smem + kTab512);
      continue;
    }
    if (MODE == 0 && fft_pow2_path(L)) {
      T2* twl = smem + L * (rpb + pow2_pitch_max_extra(L, sizeof(T) == 8));
      if (it.x != tw_cls) {
        const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.tw));
        for (int q = threadIdx.x; q < L; q += blockDim.x) twl[q] = tw[q];
        __syncthreads();
        tw_cls = it.x;
      }
      {
        if constexpr (MODE == 0) switch (L) {
          case 16: inv_pow2<T, 4, 4, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 32: inv_pow2<T, 8, 4, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 64: inv_pow2<T, 8, 8, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          case 128: inv_pow2<T, 16, 8, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
          default: inv_pow2<T, 16, 16, RAW>(C, j, col0, nr, rpb, samples, smem, twl); break;
        }
      }
      continue;
    }
    if (MODE != 0 && C.M) {
      const int M = C.M;
      T2* tws = smem + M * (rpb + 1);
      T2* chs = tws + M;
      T2* bhs = chs + L;
      if (it.x != tw_cls) {
        const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.twM));
        const SGL_G T2* ch = gmem(reinterpret_cast<const T2*>(C.chirp));
        const SGL_G T2* bh = gmem(reinterpret_cast<const T2*>(C.bhi));
        for (int q = threadIdx.x; q < M; q += blockDim.x) {
          tws[q] = tw[q];
          bhs[q] = bh[q];
        }
        for (int q = threadIdx.x; q < L; q += blockDim.x) chs[q] = ch[q];
        __syncthreads();
        tw_cls = it.x;
      }
      {
        if constexpr (MODE == 2) switch (M) {
          case 16: inv_blue<T, 4, 4, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 32: inv_blue<T, 8, 4, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 64: inv_blue<T, 8, 8, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          case 128: inv_blue<T, 16, 8, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
          default: inv_blue<T, 16, 16, RAW>(C, j, col0, nr, rpb, samples, smem, tws, chs, bhs); break;
        }
      }
      continue;
    }
    if constexpr (MODE != 0) continue;
    T2* buf0 = smem;
    T2* buf1 = smem + rpb * L;
    const SGL_G T2* F = gmem(reinterpret_cast<const T2*>(C.F));
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
      buf0[r * L + bin] = load_stream(&F[((int64_t)mi * L + j) * ncol + col0 + r]);
    }
    __syncthreads();
    const SGL_G T2* tw = gmem(reinterpret_cast<const T2*>(C.tw));
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
        const T sg = (T)(1.0 / gmem(C.sigma)[i]);
        v.x *= sg;
        v.y *= sg;
      }
      store_stream(&samples[gmem(C.soff)[b] + ((int64_t)i * L + j) * L + k], v);
    }
    __syncthreads();
  }
}

inline int grid_for(int nwork, int max_grid) {
  const int g = max_grid > 0 ? max_grid : 4096;
  return nwork < g ? nwork : g;
}

}  // namespace

// LDS bytes for rings_per_block rings of length L in the given precision
static size_t fft_lds_bytes(int prec, int rpb, int L) {
  const size_t es = prec == PREC_F64 ? sizeof(double2) : sizeof(float2);
  if (fft_mode(L) == 1)  // ring areas + tables
    return ((size_t)kRings512 * (prec == PREC_F64 ? area_pitch<double2>() : area_pitch<float2>()) + kTab512) * es;
  if (fft_pow2_path(L))  // exchange buffer + twiddle table
    return (size_t)L * (rpb + pow2_pitch_max_extra(L, prec == PREC_F64) + 1) * es;
  if (const int M = fft_bluestein_m(L)) return ((size_t)M * (rpb + 3) + L) * es;  // buffer + tw, kernel, chirp
  return (size_t)2 * rpb * L * es;
}

template <typename K>
static void allow_lds(K kernel, int bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int MODE>
static hipError_t fft_fwd(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork, int lds,
                          const void* samples, int max_grid, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  dim3 grid(grid_for(nwork, max_grid)), block(fft_threads(MODE, prec == PREC_F64));
  if (prec == PREC_F64 && raw)
    hipLaunchKernelGGL((k_fft_forward<double, true, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  else if (prec == PREC_F64)
    hipLaunchKernelGGL((k_fft_forward<double, false, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  else
    hipLaunchKernelGGL((k_fft_forward<float, false, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  return hipGetLastError();
}

template <int MODE>
static hipError_t fft_inv(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork, int lds,
                          void* samples, int max_grid, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  dim3 grid(grid_for(nwork, max_grid)), block(fft_threads(MODE, prec == PREC_F64));
  if (prec == PREC_F64 && raw)
    hipLaunchKernelGGL((k_fft_inverse<double, true, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  else if (prec == PREC_F64)
    hipLaunchKernelGGL((k_fft_inverse<double, false, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  else
    hipLaunchKernelGGL((k_fft_inverse<float, false, MODE>), grid, block, lds, s, d_cls, d_work, nwork, samples);
  return hipGetLastError();
}

// Allow the dynamic LDS the FFT launches of a plan need (set once, at plan time).
template <int MODE>
static void allow_mode(int lds) {
  allow_lds(k_fft_forward<double, true, MODE>, lds);
  allow_lds(k_fft_forward<double, false, MODE>, lds);
  allow_lds(k_fft_forward<float, false, MODE>, lds);
  allow_lds(k_fft_inverse<double, true, MODE>, lds);
  allow_lds(k_fft_inverse<double, false, MODE>, lds);
  allow_lds(k_fft_inverse<float, false, MODE>, lds);
}
void prepare_fft_kernels(const int* lds_per_mode) {
  allow_mode<0>(lds_per_mode[0]);
  allow_mode<1>(lds_per_mode[1]);
  allow_mode<2>(lds_per_mode[2]);
}

hipError_t launch_fft_forward(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, int mode, const void* samples, int max_grid, hipStream_t s) {
  if (mode == 1) return fft_fwd<1>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
  if (mode == 2) return fft_fwd<2>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
  return fft_fwd<0>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
}

hipError_t launch_fft_inverse(int prec, bool raw, const ClassDesc* d_cls, const int4* d_work, int nwork,
                              int lds_bytes, int mode, void* samples, int max_grid, hipStream_t s) {
  if (mode == 1) return fft_inv<1>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
  if (mode == 2) return fft_inv<2>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
  return fft_inv<0>(prec, raw, d_cls, d_work, nwork, lds_bytes, samples, max_grid, s);
}

size_t fft_lds_bytes_for(int prec, int rpb, int L) { return fft_lds_bytes(prec, rpb, L); }

}  // namespace sgl
