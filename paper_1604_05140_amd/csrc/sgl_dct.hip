// Seminaive Legendre step (Sect. 3.3.1): the DCT of Eq. DCT over the polar
// index j, per order m and spectrum column, in place on the spectrum workspace
// F[(m+B-1)][j][col] between stage (a) and the cosine-domain contraction.
//
// Forward:  T_k = s_k sum_{j<2B} cos(k th_j) x_j,  x_j = F_j sin^par th_j,  k < B
//           (par = |m| mod 2; th_j = (2j+1) pi / 4B are the polar nodes).  With the
//           even extension y_j = y_{4B-1-j} = x_j and its 4B-point DFT Y,
//           sum_j cos(k th_j) x_j = exp(-i pi k / 4B) Y_k / 2.
//           T replaces rows k < B of F (the contraction reads only those).
// Inverse:  F_j = sin^par th_j sum_{k<B} s_k cos(k th_j) U_k,  U in rows k < B.
//           With a_k = s_k U_k, A_k = a_k exp(+i pi k / 4B), A_{4B-k} =
//           a_k exp(-i pi k / 4B) (0 < k < B) and all other A zero, the 4B-point
//           inverse DFT R gives sum_k a_k cos(k th_j) = (R_j + a_0) / 2.
//
// One block per (order, tile of up to 16 columns), one wavefront per column:
// the block moves the tile's rows through LDS (each row leaves and arrives as a
// run of the tile width), and each wavefront runs an in-place radix-2 FFT
// (bit-reversed input, natural-order output) of its column in LDS; at B = 128
// (4B = 512) the column runs through the three-pass radix-8 one-wavefront FFT
// instead (natural order in and out, two LDS exchanges).  The transform
// computes in FP64 for every plan precision (single-precision spectra are
// widened on load and rounded once on store): a 4B-point FFT in FP32 alone
// would add ~log2(4B) roundings to the split-bf16 form's 1e-6 budget.
#include "sgl_wave.h"

namespace sgl {
namespace {

template <typename T> struct CT;
template <> struct CT<float> { using t = float2; };
template <> struct CT<double> { using t = double2; };

template <typename T2>
__device__ inline T2 cm(T2 a, T2 b) { return cmul(a, b); }
template <typename T2>
__device__ inline T2 cconj(T2 a) { return conjc(a); }
__device__ inline void wave_sync() { wave_lds_sync(); }

// LDS of the 512-point path: the class constants, the 512-point FFT table
// (w_512^(l p), w_64^(c q)), then 16 column areas of area_pitch elements.
constexpr int kFftTab = kTabTw2 + 56;

// column pitch (elements): 16 columns read at one row fall on distinct banks
template <typename T2>
__host__ __device__ constexpr int col_pad() { return sizeof(T2) == 8 ? 2 : 1; }

template <typename T, bool INV>
__global__ void __launch_bounds__(1024) k_dct(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                              int nwork) {
  using S2 = typename CT<T>::t;  // spectrum storage
  using T2 = double2;            // arithmetic and LDS
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* tab = reinterpret_cast<T2*>(smem_raw);
  int tab_cls = -1;
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    const int B = C.B, L = 2 * B, P2 = 4 * B;
    const int nconst = dct_const_count(B);
    const int CP = P2 + col_pad<T2>();
    int lg = 0;
    while ((1 << lg) < P2) ++lg;
    const int mi = it.y, am = mi >= B - 1 ? mi - (B - 1) : (B - 1) - mi, par = am & 1;
    const int ncol = C.nf * L;
    const int cols = it.w, col0 = it.z * cols;
    const int nc = min(cols, ncol - col0);
    if (it.x != tab_cls) {
      const SGL_G T2* src = gmem(reinterpret_cast<const T2*>(C.dct));  // FP64 constants
      for (int q = threadIdx.x; q < nconst; q += blockDim.x) tab[q] = src[q];
      __syncthreads();
      tab_cls = it.x;
    }
    const T2* tw = tab;             // exp(-2 pi i t / P2), t < P2 / 2
    const T2* post = tab + P2 / 2;  // s_k / 2 exp(-i pi k / 4B), k < B
    const T2* sn = post + B;        // sin th_j (real part), j < 2B
    T2* bufs = tab + nconst;
    SGL_G S2* Fb = gmem(reinterpret_cast<S2*>(C.F)) + (int64_t)mi * L * ncol + col0;
    if (P2 == 512) {
      // --- 512-point path (B = 128): columns in areas of area_pitch elements ---
      T2* ftab = bufs;                  // w_512^(l p), w_64^(c q)
      T2* areas = ftab + kFftTab;
      constexpr int AP = area_pitch<double2>();
      for (int q = threadIdx.x; q < kFftTab; q += blockDim.x) {
        // exponent e of w_512^e from the half-circle table (w^(e+256) = -w^e)
        const int e = q < kTabTw2 ? ((q % 64) * (q / 64 + 1)) % 512 : 8 * ((((q - kTabTw2) / 8 + 1) * (q % 8)) % 64);
        T2 v = tw[e & 255];
        if (e >= 256) {
          v.x = -v.x;
          v.y = -v.y;
        }
        ftab[q] = v;
      }
      if (!INV) {
        // four loads per thread in flight before any is used
        const int ne = L * nc;
        for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
          S2 f[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = min(e0 + q * (int)blockDim.x, ne - 1);
            const int j = e / nc, r = e - j * nc;
            f[q] = load_stream(&Fb[(int64_t)j * ncol + r]);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * (int)blockDim.x;
            if (e >= ne) break;
            const int j = e / nc, r = e - j * nc;
            const double sg = par ? sn[j].x : 1.0;
            areas[r * AP + j] = make_double2(f[q].x * sg, f[q].y * sg);
          }
        }
      } else {
        for (int e = threadIdx.x; e < nc * AP; e += blockDim.x) areas[e] = make_double2(0.0, 0.0);
        __syncthreads();
        const int ne = B * nc;
        for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
          S2 f[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = min(e0 + q * (int)blockDim.x, ne - 1);
            const int k = e / nc, r = e - k * nc;
            f[q] = Fb[(int64_t)k * ncol + r];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * (int)blockDim.x;
            if (e >= ne) break;
            const int k = e / nc, r = e - k * nc;
            const T2 u = make_double2(f[q].x, f[q].y);
            const T2 p = post[k];
            T2 a = cm(u, cconj(p));
            a.x += a.x;
            a.y += a.y;
            areas[r * AP + k] = a;
            if (k > 0) {
              T2 c = cm(u, p);
              c.x += c.x;
              c.y += c.y;
              areas[r * AP + P2 - k] = c;
            }
          }
        }
      }
      __syncthreads();
      const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
      if (wv < nc) {
        T2* area = areas + wv * AP;
        T2 v[8];
        const T2 a0 = area[0];
        if (!INV) {
          // even extension: y[n] = x[n] (n < 256), y[511 - n] = x[n]
#pragma unroll
          for (int a = 0; a < 8; ++a) v[a] = a < 4 ? area[64 * a + l] : area[64 * (7 - a) + 63 - l];
          fft512_wave<T2, false>(v, area, ftab, l);
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) area[64 * s2 + l] = cm(v[s2], post[64 * s2 + l]);
        } else {
#pragma unroll
          for (int a = 0; a < 8; ++a) v[a] = area[64 * a + l];
          fft512_wave<T2, true>(v, area, ftab, l);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int j = 64 * s4 + l;
            const double f = par ? 0.5 * sn[j].x : 0.5;
            area[j] = make_double2((v[s4].x + a0.x) * f, (v[s4].y + a0.y) * f);
          }
        }
      }
      __syncthreads();
      const int nrow = INV ? L : B;
      for (int e = threadIdx.x; e < nrow * nc; e += blockDim.x) {
        const int j = e / nc, r = e - j * nc;
        const T2 v = areas[r * AP + j];
        S2 o;
        o.x = v.x;
        o.y = v.y;
        if (INV)
        store_stream(&Fb[(int64_t)j * ncol + r], o);  // read once by the inverse FFT
      else
        Fb[(int64_t)j * ncol + r] = o;
      }
      __syncthreads();
      continue;
    }
    if (!INV) {
      // rows j of the tile -> bit-reversed slots j and 4B-1-j of the even extension
      const int ne = L * nc;
      for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
        S2 f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = min(e0 + q * (int)blockDim.x, ne - 1);
          const int j = e / nc, r = e - j * nc;
          f[q] = load_stream(&Fb[(int64_t)j * ncol + r]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = e0 + q * (int)blockDim.x;
          if (e >= ne) break;
          const int j = e / nc, r = e - j * nc;
          T2 x = make_double2(f[q].x, f[q].y);
          if (par) {
            x.x *= sn[j].x;
            x.y *= sn[j].x;
          }
          T2* b = bufs + r * CP;
          b[__brev((unsigned)j) >> (32 - lg)] = x;
          b[__brev((unsigned)(P2 - 1 - j)) >> (32 - lg)] = x;
        }
      }
    } else {
      for (int e = threadIdx.x; e < nc * CP; e += blockDim.x) {
        T2 z;
        z.x = 0;
        z.y = 0;
        bufs[e] = z;
      }
      __syncthreads();
      const int ne = B * nc;
      for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
        S2 f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = min(e0 + q * (int)blockDim.x, ne - 1);
          const int k = e / nc, r = e - k * nc;
          f[q] = Fb[(int64_t)k * ncol + r];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = e0 + q * (int)blockDim.x;
          if (e >= ne) break;
          const int k = e / nc, r = e - k * nc;
          const T2 u = make_double2(f[q].x, f[q].y);
          const T2 p = post[k];
          T2* b = bufs + r * CP;
          T2 a = cm(u, cconj(p));  // a_k exp(+i pi k / 4B) / 2
          a.x += a.x;
          a.y += a.y;
          b[__brev((unsigned)k) >> (32 - lg)] = a;
          if (k > 0) {
            T2 c = cm(u, p);
            c.x += c.x;
            c.y += c.y;
            b[__brev((unsigned)(P2 - k)) >> (32 - lg)] = c;
          }
        }
      }
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wv < nc) {
      T2* b = bufs + wv * CP;
      const T2 a0 = b[0];  // inverse: A_0 = a_0 (slot 0 is its own bit reversal)
      for (int lh = 0; lh < lg; ++lh) {
        const int h = 1 << lh, stride = P2 >> (lh + 1);
        for (int t = lane; t < P2 / 2; t += 64) {
          const int pos = t & (h - 1);
          const int i0 = ((t >> lh) << (lh + 1)) + pos, i1 = i0 + h;
          const T2 wt = INV ? cconj(tw[pos * stride]) : tw[pos * stride];
          const T2 u = b[i0], v = cm(b[i1], wt);
          T2 s0, s1;
          s0.x = u.x + v.x;
          s0.y = u.y + v.y;
          s1.x = u.x - v.x;
          s1.y = u.y - v.y;
          b[i0] = s0;
          b[i1] = s1;
        }
        wave_sync();
      }
      if (!INV) {
        for (int k = lane; k < B; k += 64) b[k] = cm(b[k], post[k]);
      } else {
        for (int j = lane; j < L; j += 64) {
          T2 v = b[j];
          const double f = par ? 0.5 * sn[j].x : 0.5;
          v.x = (v.x + a0.x) * f;
          v.y = (v.y + a0.y) * f;
          b[j] = v;
        }
      }
    }
    __syncthreads();
    const int nrow = INV ? L : B;
    for (int e = threadIdx.x; e < nrow * nc; e += blockDim.x) {
      const int j = e / nc, r = e - j * nc;
      const T2 v = bufs[r * CP + j];
      S2 o;
      o.x = v.x;
      o.y = v.y;
      if (INV)
        store_stream(&Fb[(int64_t)j * ncol + r], o);  // read once by the inverse FFT
      else
        Fb[(int64_t)j * ncol + r] = o;
    }
    __syncthreads();
  }
}

template <typename K>
void allow(K kernel, int bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              bytes);
}

}  // namespace

size_t dct_lds_bytes(int, int B, int cols) {
  if (4 * B == 512)
    return ((size_t)dct_const_count(B) + kFftTab + (size_t)cols * area_pitch<double2>()) * sizeof(double2);
  return ((size_t)dct_const_count(B) + (size_t)cols * (4 * B + col_pad<double2>())) * sizeof(double2);
}

void prepare_dct_kernels(int lds_bytes) {
  allow(k_dct<float, false>, lds_bytes);
  allow(k_dct<float, true>, lds_bytes);
  allow(k_dct<double, false>, lds_bytes);
  allow(k_dct<double, true>, lds_bytes);
}

hipError_t launch_dct(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork, int lds_bytes,
                      int cols, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  const dim3 grid(nwork < 4096 ? nwork : 4096), block(64 * cols);
  if (prec == PREC_F64) {
    if (inverse)
      hipLaunchKernelGGL((k_dct<double, true>), grid, block, lds_bytes, s, d_cls, d_work, nwork);
    else
      hipLaunchKernelGGL((k_dct<double, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork);
  } else {
    if (inverse)
      hipLaunchKernelGGL((k_dct<float, true>), grid, block, lds_bytes, s, d_cls, d_work, nwork);
    else
      hipLaunchKernelGGL((k_dct<float, false>), grid, block, lds_bytes, s, d_cls, d_work, nwork);
  }
  return hipGetLastError();
}

}  // namespace sgl
