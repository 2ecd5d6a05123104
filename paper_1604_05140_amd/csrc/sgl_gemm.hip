// Stages (b) and (c): per-order contractions on MFMA.
//
// Stage (b), Legendre projection per order m (Eq. DLT with the azimuthal
// spectrum of Eq. SFFT_rearranged; inverse Eq. iSFFT_rearranged):
//   forward  g[l][m][b,i] = sum_j Pbar_lm(cos th_j) F[m][j][b,i],   l = |m|..B-1
//   inverse  F[m][j][b,i] = sum_l Pbar_lm(cos th_j) g[l][m][b,i]
// with the b~_j weight already folded into F by stage (a).  Orders m and -m
// share one launch tile list: Pbar_{l,-m} = (-1)^m Pbar_lm, so the -m columns
// run against the same table block and take the sign in the epilogue.
//
// Stage (c), radial projection per degree l (discrete R transform, Eq. DRT /
// Eq. DRT_matrix; inverse R_l^T, Sect. 3.3.2):
//   forward  fhat[b][omega(n,l,m)] = sum_i rho_nl(r_i) g[l][m][b,i],  n = l+1..B
//   inverse  g[l][m][b,i] = sum_n rho_nl(r_i) fhat[b][omega(n,l,m)]
// where rho_nl(r_i) = sigma_i N_nl R_nl(r_i) has orthonormal rows (the iDRT
// identity), so one table serves both directions.
//
// Every contraction is a real table (M x K) times complex data (K x N complex
// columns = 2N real columns).  One kernel template covers the four cases; the
// tile loaders read the operands where they live (no transposed copies) and
// the epilogues write the next stage's layout directly:
//   F  [(m+B-1)][j][b*2B+i]          (stage a <-> b)
//   g  [l][b][m+l][i], block l at l^2 * nf * 2B   (stage b <-> c)
//   fhat[b][omega]                    (stage c <-> caller)
//
// Precisions: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4), and a
// three-piece bf16 split of both operands (x = x0 + x1 + x2, each a bf16
// rounding of the remainder) whose six products of order <= 2 run on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (main product and
// corrections in separate accumulators).
#include "sgl_internal.h"

namespace sgl {
namespace {

constexpr int BM = 64;   // rows per tile
constexpr int BN = 64;   // real columns per tile (32 complex)
constexpr int BNC = BN / 2;
constexpr int BK = 32;   // contraction chunk
constexpr int NT = 256;  // threads per block (4 waves, 2 x 2 layout of 32 x 32)
constexpr int BKS = BK + 8;  // bf16 LDS row pitch (80 bytes, 16-byte aligned rows)

enum Kind { K_B_FWD = 0, K_B_INV = 1, K_C_FWD = 2, K_C_INV = 3, K_DEBUG = 4 };

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int PREC> struct DT { using t = float; };
template <> struct DT<PREC_F64> { using t = double; };

template <int PREC> struct Acc { using t = f4; };
template <> struct Acc<PREC_F64> { using t = d4; };

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// LDS footprint
template <int PREC> struct LdsSize {
  static constexpr int a = BM * (BK + 1) * (int)sizeof(typename DT<PREC>::t);
  static constexpr int x = BN * (BK + 1) * (int)sizeof(typename DT<PREC>::t);
};
template <> struct LdsSize<PREC_SPLIT> {
  static constexpr int a = 3 * BM * BKS * 2;
  static constexpr int x = 3 * BN * BKS * 2;
};

struct DebugArgs {
  int M, N, K;
  const double* A;
  const double* X;
  double* C;
};

struct Tile {
  int M, K, Ncc;   // rows, contraction length, complex columns of the group
  int row0, col0;  // first row, first complex column of the tile
  int q;           // m (stage b) or l (stage c)
  const ClassDesc* C;
};

// ---- LDS stores ------------------------------------------------------------
template <int PREC>
__device__ inline void lds_put_a(unsigned char* sm, int r, int k, const void* tab, int64_t idx, int64_t plane,
                                 bool valid) {
  if constexpr (PREC == PREC_SPLIT) {
    uint16_t* As = reinterpret_cast<uint16_t*>(sm);
    const uint16_t* t = reinterpret_cast<const uint16_t*>(tab);
    for (int p = 0; p < 3; ++p) As[(p * BM + r) * BKS + k] = valid ? t[p * plane + idx] : (uint16_t)0;
  } else {
    using T = typename DT<PREC>::t;
    T* As = reinterpret_cast<T*>(sm);
    As[r * (BK + 1) + k] = valid ? reinterpret_cast<const T*>(tab)[idx] : (T)0;
  }
}

template <int PREC>
__device__ inline void lds_put_x(unsigned char* sm, int n, int k, float vf, double vd) {
  if constexpr (PREC == PREC_SPLIT) {
    uint16_t* Xs = reinterpret_cast<uint16_t*>(sm + LdsSize<PREC>::a);
    uint16_t h0 = f2bf(vf);
    float r1 = vf - bf2f(h0);
    uint16_t h1 = f2bf(r1);
    float r2 = r1 - bf2f(h1);
    uint16_t h2 = f2bf(r2);
    Xs[(0 * BN + n) * BKS + k] = h0;
    Xs[(1 * BN + n) * BKS + k] = h1;
    Xs[(2 * BN + n) * BKS + k] = h2;
  } else if constexpr (PREC == PREC_F64) {
    double* Xs = reinterpret_cast<double*>(sm + LdsSize<PREC>::a);
    Xs[n * (BK + 1) + k] = vd;
  } else {
    float* Xs = reinterpret_cast<float*>(sm + LdsSize<PREC>::a);
    Xs[n * (BK + 1) + k] = vf;
  }
}

// ---- operand addressing ----------------------------------------------------
__device__ inline int64_t gbase(int l, int nf, int L) { return (int64_t)l * l * nf * L; }

// complex element (k, c) of the data operand; returns pointer index in complex units
template <int KIND>
__device__ inline int64_t x_index(const Tile& t, int k, int c, int& sgn) {
  const ClassDesc& C = *t.C;
  const int B = C.B, L = C.L, nf = C.nf;
  sgn = 1;
  if constexpr (KIND == K_B_FWD) {
    const int ncf = nf * L;
    const int seg = c >= ncf;
    const int cp = c - seg * ncf;
    const int mp = seg ? -t.q : t.q;
    return ((int64_t)(mp + B - 1) * L + k) * ncf + cp;
  } else if constexpr (KIND == K_B_INV) {
    const int ncf = nf * L;
    const int seg = c >= ncf;
    const int cp = c - seg * ncf;
    const int mp = seg ? -t.q : t.q;
    const int l = t.q + k;
    const int b = cp / L, i = cp - b * L;
    return gbase(l, nf, L) + ((int64_t)b * (2 * l + 1) + mp + l) * L + i;
  } else if constexpr (KIND == K_C_FWD) {
    return gbase(t.q, nf, L) + (int64_t)c * L + k;
  } else {  // K_C_INV: coefficient (n = l+1+k, l, m) of function b
    const int l = t.q;
    const int b = c / (2 * l + 1);
    const int m = c - b * (2 * l + 1) - l;
    return C.coff[b] + omega(l + 1 + k, l, m);
  }
}

// output index (complex units) and sign for element (row, c)
template <int KIND>
__device__ inline int64_t c_index(const Tile& t, int row, int c, int& sgn) {
  const ClassDesc& C = *t.C;
  const int B = C.B, L = C.L, nf = C.nf;
  sgn = 1;
  if constexpr (KIND == K_B_FWD || KIND == K_B_INV) {
    const int ncf = nf * L;
    const int seg = c >= ncf;
    const int cp = c - seg * ncf;
    const int mp = seg ? -t.q : t.q;
    if (seg && (t.q & 1)) sgn = -1;
    if constexpr (KIND == K_B_FWD) {
      const int l = t.q + row;
      const int b = cp / L, i = cp - b * L;
      return gbase(l, nf, L) + ((int64_t)b * (2 * l + 1) + mp + l) * L + i;
    } else {
      return ((int64_t)(mp + B - 1) * L + row) * ncf + cp;
    }
  } else if constexpr (KIND == K_C_FWD) {
    const int l = t.q;
    const int b = c / (2 * l + 1);
    const int m = c - b * (2 * l + 1) - l;
    return C.coff[b] + omega(l + 1 + row, l, m);
  } else {  // K_C_INV
    return gbase(t.q, nf, L) + (int64_t)c * L + row;
  }
}

// ---- the kernel ------------------------------------------------------------
template <int PREC, int KIND>
__global__ void __launch_bounds__(NT) k_gemm(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                             int nwork, const void* __restrict__ cin, void* __restrict__ cout,
                                             DebugArgs dbg) {
  using T = typename DT<PREC>::t;
  using AccT = typename Acc<PREC>::t;
  __shared__ __align__(16) unsigned char sm[LdsSize<PREC>::a + LdsSize<PREC>::x];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  int nitems = KIND == K_DEBUG ? ((dbg.M + BM - 1) / BM) * ((dbg.N + BN - 1) / BN) : nwork;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    Tile t;
    const void* tab = nullptr;
    int64_t plane = 0;
    int ld = 0;
    if constexpr (KIND == K_DEBUG) {
      const int ntn = (dbg.N + BN - 1) / BN;
      t.M = dbg.M;
      t.K = dbg.K;
      t.Ncc = (dbg.N + 1) / 2;
      t.row0 = (w / ntn) * BM;
      t.col0 = (w % ntn) * BNC;
      t.q = 0;
      t.C = nullptr;
    } else {
      const int4 it = work[w];
      const ClassDesc& C = cls[it.x];
      t.C = &C;
      t.q = it.y;
      const int B = C.B, L = C.L;
      if constexpr (KIND == K_B_FWD || KIND == K_B_INV) {
        const int rows = B - t.q;
        t.M = KIND == K_B_FWD ? rows : L;
        t.K = KIND == K_B_FWD ? L : rows;
        t.Ncc = (t.q ? 2 : 1) * C.nf * L;
        tab = C.P;
      } else {
        const int rows = B - t.q;
        t.M = KIND == K_C_FWD ? rows : L;
        t.K = KIND == K_C_FWD ? L : rows;
        t.Ncc = (2 * t.q + 1) * C.nf;
        tab = C.R;
      }
      const int64_t off = table_block(B, t.q);
      if constexpr (PREC == PREC_SPLIT) {
        tab = reinterpret_cast<const uint16_t*>(tab) + off;
        plane = table_size(B);
      } else {
        tab = reinterpret_cast<const T*>(tab) + off;
      }
      ld = L;
      t.row0 = it.z * BM;
      t.col0 = it.w * BNC;
    }

    AccT acc[2][2], acc2[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int v = 0; v < 4; ++v) {
          acc[a][b][v] = 0;
          acc2[a][b][v] = 0;
        }

    for (int k0 = 0; k0 < t.K; k0 += BK) {
      // ---- A tile -> LDS
      if constexpr (KIND == K_DEBUG) {
        for (int e = tid; e < BM * BK; e += NT) {
          const int r = e / BK, k = e - r * BK;
          const int gr = t.row0 + r, gk = k0 + k;
          const bool ok = gr < t.M && gk < t.K;
          const double v = ok ? dbg.A[(int64_t)gr * t.K + gk] : 0.0;
          if constexpr (PREC == PREC_SPLIT) {
            uint16_t* As = reinterpret_cast<uint16_t*>(sm);
            uint16_t h0 = f2bf((float)v);
            double r1 = v - (double)bf2f(h0);
            uint16_t h1 = f2bf((float)r1);
            double r2 = r1 - (double)bf2f(h1);
            As[(0 * BM + r) * BKS + k] = h0;
            As[(1 * BM + r) * BKS + k] = h1;
            As[(2 * BM + r) * BKS + k] = f2bf((float)r2);
          } else {
            reinterpret_cast<T*>(sm)[r * (BK + 1) + k] = (T)v;
          }
        }
      } else if constexpr (KIND == K_B_FWD || KIND == K_C_FWD) {
        // table block rows are contiguous in k
        for (int e = tid; e < BM * BK; e += NT) {
          const int r = e / BK, k = e - r * BK;
          const int gr = t.row0 + r, gk = k0 + k;
          lds_put_a<PREC>(sm, r, k, tab, (int64_t)gr * ld + gk, plane, gr < t.M && gk < t.K);
        }
      } else {
        // inverse: A = table block transposed, contiguous in the tile row
        for (int e = tid; e < BM * BK; e += NT) {
          const int k = e / BM, r = e - k * BM;
          const int gr = t.row0 + r, gk = k0 + k;
          lds_put_a<PREC>(sm, r, k, tab, (int64_t)gk * ld + gr, plane, gr < t.M && gk < t.K);
        }
      }
      // ---- X tile -> LDS (as [real column][k])
      if constexpr (KIND == K_DEBUG) {
        for (int e = tid; e < BN * BK; e += NT) {
          const int k = e / BN, n = e - k * BN;
          const int gk = k0 + k, gn = 2 * t.col0 + n;
          const double v = (gk < t.K && gn < dbg.N) ? dbg.X[(int64_t)gk * dbg.N + gn] : 0.0;
          lds_put_x<PREC>(sm, n, k, (float)v, v);
        }
      } else if constexpr (KIND == K_C_FWD) {
        // contiguous along k
        const T* X = reinterpret_cast<const T*>(t.C->g);
        for (int e = tid; e < BNC * BK; e += NT) {
          const int cc = e / BK, k = e - cc * BK;
          const int gk = k0 + k, c = t.col0 + cc;
          T re = 0, im = 0;
          if (gk < t.K && c < t.Ncc) {
            int sg;
            const int64_t ix = x_index<KIND>(t, gk, c, sg);
            re = X[2 * ix];
            im = X[2 * ix + 1];
          }
          lds_put_x<PREC>(sm, 2 * cc, k, (float)re, (double)re);
          lds_put_x<PREC>(sm, 2 * cc + 1, k, (float)im, (double)im);
        }
      } else {
        // contiguous along the column index
        const T* X = reinterpret_cast<const T*>(KIND == K_B_FWD ? t.C->F : (KIND == K_B_INV ? t.C->g : cin));
        for (int e = tid; e < BNC * BK; e += NT) {
          const int k = e / BNC, cc = e - k * BNC;
          const int gk = k0 + k, c = t.col0 + cc;
          T re = 0, im = 0;
          if (gk < t.K && c < t.Ncc) {
            int sg;
            const int64_t ix = x_index<KIND>(t, gk, c, sg);
            re = X[2 * ix];
            im = X[2 * ix + 1];
          }
          lds_put_x<PREC>(sm, 2 * cc, k, (float)re, (double)re);
          lds_put_x<PREC>(sm, 2 * cc + 1, k, (float)im, (double)im);
        }
      }
      __syncthreads();

      // ---- MFMA
      if constexpr (PREC == PREC_SPLIT) {
        const uint16_t* As = reinterpret_cast<const uint16_t*>(sm);
        const uint16_t* Xs = reinterpret_cast<const uint16_t*>(sm + LdsSize<PREC>::a);
        bf8 a[2][3], b[2][3];
        for (int i = 0; i < 2; ++i)
          for (int p = 0; p < 3; ++p) {
            a[i][p] = *reinterpret_cast<const bf8*>(&As[(p * BM + wr + i * 16 + lr) * BKS + 8 * lk]);
            b[i][p] = *reinterpret_cast<const bf8*>(&Xs[(p * BN + wc + i * 16 + lr) * BKS + 8 * lk]);
          }
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], acc[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], acc2[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], acc2[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], acc2[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][1], acc2[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], acc2[i][j], 0, 0, 0);
          }
      } else {
        const T* As = reinterpret_cast<const T*>(sm);
        const T* Xs = reinterpret_cast<const T*>(sm + LdsSize<PREC>::a);
        for (int kk = 0; kk < BK; kk += 4) {
          T a[2], b[2];
          for (int i = 0; i < 2; ++i) {
            a[i] = As[(wr + i * 16 + lr) * (BK + 1) + kk + lk];
            b[i] = Xs[(wc + i * 16 + lr) * (BK + 1) + kk + lk];
          }
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
              if constexpr (PREC == PREC_F64)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
              else
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
      }
      __syncthreads();
    }

    // ---- epilogue: each lane holds 4 rows of real column lane%16 of each 16x16 block:
    // rows 4*(lane/16)+v for the f32 MFMAs, rows 4*v+lane/16 for the f64 MFMA.
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const int nr = 2 * t.col0 + wc + j * 16 + lr;  // real column
        const int c = nr >> 1, part = nr & 1;
        if (c >= t.Ncc) continue;
        for (int v = 0; v < 4; ++v) {
          const int rin = PREC == PREC_F64 ? 4 * v + lk : 4 * lk + v;
          const int row = t.row0 + wr + i * 16 + rin;
          if (row >= t.M) continue;
          T val;
          if constexpr (PREC == PREC_SPLIT)
            val = acc[i][j][v] + acc2[i][j][v];
          else
            val = acc[i][j][v];
          if constexpr (KIND == K_DEBUG) {
            if (nr < dbg.N) dbg.C[(int64_t)row * dbg.N + nr] = (double)val;
          } else {
            int sg;
            const int64_t ix = c_index<KIND>(t, row, c, sg);
            T* out;
            if constexpr (KIND == K_B_FWD || KIND == K_C_INV)
              out = reinterpret_cast<T*>(t.C->g);
            else if constexpr (KIND == K_B_INV)
              out = reinterpret_cast<T*>(t.C->F);
            else
              out = reinterpret_cast<T*>(cout);
            out[2 * ix + part] = sg < 0 ? -val : val;
          }
        }
      }
  }
}

inline int grid_for(int nwork) { return nwork < 8192 ? nwork : 8192; }

template <int PREC>
hipError_t launch_kind(int kind, const ClassDesc* d_cls, const int4* d_work, int nwork, const void* cin, void* cout,
                       hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  DebugArgs dbg{0, 0, 0, nullptr, nullptr, nullptr};
  dim3 grid(grid_for(nwork)), block(NT);
  switch (kind) {
    case K_B_FWD:
      hipLaunchKernelGGL((k_gemm<PREC, K_B_FWD>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    case K_B_INV:
      hipLaunchKernelGGL((k_gemm<PREC, K_B_INV>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    case K_C_FWD:
      hipLaunchKernelGGL((k_gemm<PREC, K_C_FWD>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    default:
      hipLaunchKernelGGL((k_gemm<PREC, K_C_INV>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_any(int prec, int kind, const ClassDesc* d_cls, const int4* d_work, int nwork, const void* cin,
                      void* cout, hipStream_t s) {
  if (prec == PREC_F64) return launch_kind<PREC_F64>(kind, d_cls, d_work, nwork, cin, cout, s);
  if (prec == PREC_F32) return launch_kind<PREC_F32>(kind, d_cls, d_work, nwork, cin, cout, s);
  return launch_kind<PREC_SPLIT>(kind, d_cls, d_work, nwork, cin, cout, s);
}

}  // namespace

int gemm_tile_m() { return BM; }
int gemm_tile_n_complex() { return BNC; }

hipError_t launch_legendre(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork,
                           hipStream_t s) {
  return launch_any(prec, inverse ? K_B_INV : K_B_FWD, d_cls, d_work, nwork, nullptr, nullptr, s);
}

hipError_t launch_radial(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork,
                         const void* coeffs_in, void* coeffs_out, hipStream_t s) {
  return launch_any(prec, inverse ? K_C_INV : K_C_FWD, d_cls, d_work, nwork, coeffs_in, coeffs_out, s);
}

hipError_t launch_debug_gemm(int prec, int M, int N, int K, const double* A, const double* X, double* C,
                             hipStream_t s) {
  DebugArgs dbg{M, N, K, A, X, C};
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles == 0) return hipSuccess;
  dim3 grid(grid_for(tiles)), block(NT);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_gemm<PREC_F64, K_DEBUG>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr, dbg);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL((k_gemm<PREC_F32, K_DEBUG>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr, dbg);
  else
    hipLaunchKernelGGL((k_gemm<PREC_SPLIT, K_DEBUG>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr,
                       dbg);
  return hipGetLastError();
}

}  // namespace sgl
