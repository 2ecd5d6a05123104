// Stages (b) and (c): per-order contractions on MFMA.
//
// Stage (b), Legendre projection per order m (Eq. DLT with the azimuthal
// spectrum of Eq. SFFT_rearranged; inverse Eq. iSFFT_rearranged):
//   forward  g[l][m][b,i] = sum_j Pbar_lm(cos th_j) F[m][j][b,i],   l = |m|..B-1
//   inverse  F[m][j][b,i] = sum_l Pbar_lm(cos th_j) g[l][m][b,i]
// with the b~_j weight already folded into F by stage (a).  Orders m and -m
// share one tile list: Pbar_{l,-m} = (-1)^m Pbar_lm, so the -m columns run
// against the same table block and take the sign in the epilogue.
//
// Stage (c), radial projection per degree l (discrete R transform, Eq. DRT /
// Eq. DRT_matrix; inverse R_l^T, Sect. 3.3.2):
//   forward  fhat[b][omega(n,l,m)] = sum_i rho_nl(r_i) g[l][m][b,i],  n = l+1..B
//   inverse  g[l][m][b,i] = sum_n rho_nl(r_i) fhat[b][omega(n,l,m)]
// where rho_nl(r_i) = sigma_i N_nl R_nl(r_i) has orthonormal rows (the iDRT
// identity), so the same values serve both directions.
//
// Every contraction is a real table (M x K) times complex data (K x N complex
// columns = 2N real columns).  One kernel template covers the four cases:
//   * tile 128 x 128 real outputs, 8 waves of 64 x 32 (4 x 2 MFMA blocks of
//     16 x 16); 128 rows cover a whole Legendre block at B <= 128, so the
//     spectrum F is read from HBM once; K in chunks of 64 through LDS, with
//     two register stages: the loads of chunk c+2 are issued before the MFMAs
//     of chunk c, so each load has two MFMA phases to arrive;
//   * the table operand comes pre-packed per direction (row-major, K padded to
//     a multiple of 64 with zeros), so every table load is a 16-byte vector;
//   * data-operand loads follow the layout the previous stage wrote (16-byte
//     runs along the contiguous index), are transposed in registers so that
//     each lane holds 8 consecutive k of one column, and go to LDS as [column][k]
//     (one 16-byte LDS store per column and bf16 plane);
//   * the epilogue stages the tile through LDS and writes the next stage's
//     layout with coalesced 16-byte stores:
//       F    [(m+B-1)][j][b*2B+i]                 (stage a <-> b)
//       g    [l][b][m+l][i], block l at l^2 nf 2B  (stage b <-> c)
//       fhat [b][omega]                             (stage c <-> caller)
//
// Precisions: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4), and a
// three-piece bf16 split of both operands (x = x0 + x1 + x2, each a bf16
// rounding of the remainder) whose six products of order <= 2 run on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (main product and the five
// corrections in separate accumulators).
#include "sgl_internal.h"

namespace sgl {
namespace {

constexpr int BM = 128;      // rows per tile
constexpr int BN = 128;      // real columns per tile
constexpr int BNC = BN / 2;  // complex columns per tile
constexpr int BK = 64;       // contraction chunk
constexpr int NT = 512;      // 8 waves, 2 x 4 layout of 64 x 32
constexpr int PS = BK + 8;   // bf16 LDS pitch (80 bytes)
constexpr int PF = BK + 4;   // f32/f64 LDS pitch in elements
constexpr int EP = BN + 1;   // epilogue tile pitch (elements)

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

template <int PREC> struct Lds {
  static constexpr int a = BM * PF * (int)sizeof(typename DT<PREC>::t);
  static constexpr int x = BN * PF * (int)sizeof(typename DT<PREC>::t);
  static constexpr int ep = 64 * EP * (int)sizeof(typename DT<PREC>::t);
  static constexpr int total = (a + x) > ep ? (a + x) : ep;
};
template <> struct Lds<PREC_SPLIT> {
  static constexpr int a = 3 * BM * PS * 2;
  static constexpr int x = 3 * BN * PS * 2;
  static constexpr int ep = 64 * EP * 4;
  static constexpr int total = (a + x) > ep ? (a + x) : ep;
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
  int pitch;       // packed table row pitch
  const ClassDesc* C;
};

__device__ inline int64_t gbase(int l, int nf, int L) { return (int64_t)l * l * nf * L; }

// ---- per-thread register staging of one K chunk -----------------------------
// A: split -> 6 x uint4 (3 planes x 2 vectors); f32 -> 4 x float4; f64 -> 8 x double2.
// X: 8 consecutive k of one complex column -> 8 complex values.
template <int PREC> struct Stage {
  static constexpr int NA = PREC == PREC_SPLIT ? 6 : (PREC == PREC_F32 ? 4 : 8);
  uint4 a[NA];
  typename DT<PREC>::t xr[8], xi[8];
};

// A chunk: BM rows x BK (padded, zero filled) from a packed table block.
template <int PREC>
__device__ inline void load_a(Stage<PREC>& st, const Tile& t, const void* tab, int64_t plane, int k0, int tid) {
  if constexpr (PREC == PREC_SPLIT) {
    // 3 planes x 128 rows x 8 vectors of 8 bf16
    for (int v = 0; v < 6; ++v) {
      const int e = tid + v * NT;  // 0..3071
      const int p = e >> 10, rem = e & 1023;
      const int r = rem >> 3, kg = rem & 7;
      const int gr = t.row0 + r;
      uint4 z = make_uint4(0, 0, 0, 0);
      if (gr < t.M)
        z = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(tab) + p * plane +
                                            (int64_t)gr * t.pitch + k0 + kg * 8);
      st.a[v] = z;
    }
  } else if constexpr (PREC == PREC_F32) {
    for (int v = 0; v < 4; ++v) {
      const int e = tid + v * NT;  // 128 rows x 16 vectors of 4 floats
      const int r = e >> 4, kg = e & 15;
      const int gr = t.row0 + r;
      uint4 z = make_uint4(0, 0, 0, 0);
      if (gr < t.M)
        z = *reinterpret_cast<const uint4*>(reinterpret_cast<const float*>(tab) + (int64_t)gr * t.pitch + k0 + kg * 4);
      st.a[v] = z;
    }
  } else {
    for (int v = 0; v < 8; ++v) {
      const int e = tid + v * NT;  // 128 rows x 32 vectors of 2 doubles
      const int r = e >> 5, kg = e & 31;
      const int gr = t.row0 + r;
      uint4 z = make_uint4(0, 0, 0, 0);
      if (gr < t.M)
        z = *reinterpret_cast<const uint4*>(reinterpret_cast<const double*>(tab) + (int64_t)gr * t.pitch + k0 + kg * 2);
      st.a[v] = z;
    }
  }
}

template <int PREC>
__device__ inline void store_a(const Stage<PREC>& st, unsigned char* sm, int tid) {
  if constexpr (PREC == PREC_SPLIT) {
    uint16_t* As = reinterpret_cast<uint16_t*>(sm);
    for (int v = 0; v < 6; ++v) {
      const int e = tid + v * NT;
      const int p = e >> 10, rem = e & 1023;
      const int r = rem >> 3, kg = rem & 7;
      *reinterpret_cast<uint4*>(&As[(p * BM + r) * PS + kg * 8]) = st.a[v];
    }
  } else if constexpr (PREC == PREC_F32) {
    float* As = reinterpret_cast<float*>(sm);
    for (int v = 0; v < 4; ++v) {
      const int e = tid + v * NT;
      const int r = e >> 4, kg = e & 15;
      *reinterpret_cast<uint4*>(&As[r * PF + kg * 4]) = st.a[v];
    }
  } else {
    double* As = reinterpret_cast<double*>(sm);
    for (int v = 0; v < 8; ++v) {
      const int e = tid + v * NT;
      const int r = e >> 5, kg = e & 31;
      *reinterpret_cast<uint4*>(&As[r * PF + kg * 2]) = st.a[v];
    }
  }
}

// Per-thread decode of one data-operand column, done once per tile: the complex
// index of element (k, c) is then a cheap function of k.
struct XCol {
  int64_t base;  // index at k = 0 (linear kinds) or the constant term
  int64_t s1;    // linear coefficient
  int64_t s2;    // quadratic coefficient (stage-b inverse)
  int ok;        // column inside the group
};

template <int KIND>
__device__ inline XCol x_col(const Tile& t, int c) {
  XCol x{0, 0, 0, c < t.Ncc};
  if constexpr (KIND != K_DEBUG) {
    if (!x.ok) return x;
    const ClassDesc& C = *t.C;
    const int B = C.B, L = C.L, nf = C.nf;
    if constexpr (KIND == K_B_FWD) {
      const int ncf = nf * L;
      const int seg = c >= ncf;
      const int cp = c - seg * ncf;
      const int mp = seg ? -t.q : t.q;
      x.base = (int64_t)(mp + B - 1) * L * ncf + cp;  // + k * ncf
      x.s1 = ncf;
    } else if constexpr (KIND == K_B_INV) {
      // element (k, c) sits at g[l][b][mp+l][i], l = q + k:
      //   l^2 nf L + (2b+1) L l + (b+mp) L + i
      const int ncf = nf * L;
      const int seg = c >= ncf;
      const int cp = c - seg * ncf;
      const int mp = seg ? -t.q : t.q;
      const int b = cp / L, i = cp - b * L;
      x.s2 = (int64_t)nf * L;
      x.s1 = (int64_t)(2 * b + 1) * L;
      x.base = (int64_t)(b + mp) * L + i;
    } else if constexpr (KIND == K_C_FWD) {
      x.base = gbase(t.q, nf, L) + (int64_t)c * L;  // + k
      x.s1 = 1;
    } else {  // K_C_INV: coefficient (n = q+1+k, q, m) of function b
      const int l = t.q;
      const int b = c / (2 * l + 1);
      const int m = c - b * (2 * l + 1) - l;
      x.base = C.coff[b] + (int64_t)l * (l + 1) + m;  // + omega(n, 0, 0)
    }
  }
  return x;
}

template <int KIND>
__device__ inline int64_t x_at(const Tile& t, const XCol& x, int k) {
  if constexpr (KIND == K_B_INV) {
    const int64_t l = t.q + k;
    return x.base + l * (x.s1 + l * x.s2);
  } else if constexpr (KIND == K_C_INV) {
    const int64_t n = t.q + 1 + k;
    return x.base + n * (n - 1) * (2 * n - 1) / 6;
  } else {
    return x.base + (int64_t)k * x.s1;
  }
}

// X chunk: thread -> (complex column cc = tid & 63, k group kg = tid >> 6 of 8 rows)
template <int PREC, int KIND>
__device__ inline void load_x(Stage<PREC>& st, const Tile& t, const XCol& xc, const void* xbase,
                              const DebugArgs& dbg, int k0, int tid) {
  using T = typename DT<PREC>::t;
  const int cc = tid & 63, kg = tid >> 6;
  const int c = t.col0 + cc;
  const int kb = k0 + kg * 8;
  if constexpr (KIND == K_DEBUG) {
    for (int u = 0; u < 8; ++u) {
      const int k = kb + u;
      const int n0 = 2 * c, n1 = 2 * c + 1;
      const bool ok = k < t.K;
      st.xr[u] = (ok && n0 < dbg.N) ? (T)dbg.X[(int64_t)k * dbg.N + n0] : (T)0;
      st.xi[u] = (ok && n1 < dbg.N) ? (T)dbg.X[(int64_t)k * dbg.N + n1] : (T)0;
    }
  } else {
    const T* X = reinterpret_cast<const T*>(xbase);
    if (xc.ok) {
      if constexpr (KIND == K_C_FWD) {
        // 8 consecutive k of one column are contiguous (g rows run along i)
        const int64_t ix = x_at<KIND>(t, xc, kb);
        for (int u = 0; u < 8; ++u) {
          const bool ok = kb + u < t.K;
          st.xr[u] = ok ? X[2 * (ix + u)] : (T)0;
          st.xi[u] = ok ? X[2 * (ix + u) + 1] : (T)0;
        }
      } else {
        for (int u = 0; u < 8; ++u) {
          const int k = kb + u;
          if (k < t.K) {
            const int64_t ix = x_at<KIND>(t, xc, k);
            st.xr[u] = X[2 * ix];
            st.xi[u] = X[2 * ix + 1];
          } else {
            st.xr[u] = 0;
            st.xi[u] = 0;
          }
        }
      }
    } else {
      for (int u = 0; u < 8; ++u) {
        st.xr[u] = 0;
        st.xi[u] = 0;
      }
    }
  }
}

// Exact three-piece bf16 split of an FP32 value by truncation: x0 keeps the top
// 8 significand bits, x1 the next 8 of the (exact) remainder, and the last
// remainder has at most 8 significant bits, so x = x0 + x1 + x2 exactly.  The
// pieces are returned as FP32 bit patterns whose low halves are zero.
__device__ inline void split3(float v, uint32_t& h0, uint32_t& h1, uint32_t& h2) {
  h0 = __float_as_uint(v) & 0xFFFF0000u;
  const float r1 = v - __uint_as_float(h0);
  h1 = __float_as_uint(r1) & 0xFFFF0000u;
  h2 = __float_as_uint(r1 - __uint_as_float(h1));
}
// pack the high halves of two FP32 patterns into one dword (lo element first)
__device__ inline uint32_t pack_hi(uint32_t lo, uint32_t hi) { return __builtin_amdgcn_perm(hi, lo, 0x07060302u); }

template <int PREC>
__device__ inline void store_x(const Stage<PREC>& st, unsigned char* sm, int tid) {
  const int cc = tid & 63, kg = tid >> 6;
  if constexpr (PREC == PREC_SPLIT) {
    uint16_t* Xs = reinterpret_cast<uint16_t*>(sm + Lds<PREC>::a);
    for (int part = 0; part < 2; ++part) {
      uint32_t h[3][8];
      for (int u = 0; u < 8; ++u) split3(part ? st.xi[u] : st.xr[u], h[0][u], h[1][u], h[2][u]);
      for (int p = 0; p < 3; ++p) {
        uint4 w;
        w.x = pack_hi(h[p][0], h[p][1]);
        w.y = pack_hi(h[p][2], h[p][3]);
        w.z = pack_hi(h[p][4], h[p][5]);
        w.w = pack_hi(h[p][6], h[p][7]);
        *reinterpret_cast<uint4*>(&Xs[(p * BN + 2 * cc + part) * PS + kg * 8]) = w;
      }
    }
  } else if constexpr (PREC == PREC_F32) {
    float* Xs = reinterpret_cast<float*>(sm + Lds<PREC>::a);
    float* r0 = &Xs[(2 * cc) * PF + kg * 8];
    float* r1 = &Xs[(2 * cc + 1) * PF + kg * 8];
    *reinterpret_cast<float4*>(r0) = make_float4(st.xr[0], st.xr[1], st.xr[2], st.xr[3]);
    *reinterpret_cast<float4*>(r0 + 4) = make_float4(st.xr[4], st.xr[5], st.xr[6], st.xr[7]);
    *reinterpret_cast<float4*>(r1) = make_float4(st.xi[0], st.xi[1], st.xi[2], st.xi[3]);
    *reinterpret_cast<float4*>(r1 + 4) = make_float4(st.xi[4], st.xi[5], st.xi[6], st.xi[7]);
  } else {
    double* Xs = reinterpret_cast<double*>(sm + Lds<PREC>::a);
    double* r0 = &Xs[(2 * cc) * PF + kg * 8];
    double* r1 = &Xs[(2 * cc + 1) * PF + kg * 8];
    for (int u = 0; u < 8; u += 2) {
      *reinterpret_cast<double2*>(r0 + u) = make_double2(st.xr[u], st.xr[u + 1]);
      *reinterpret_cast<double2*>(r1 + u) = make_double2(st.xi[u], st.xi[u + 1]);
    }
  }
}

// ---- the kernel ------------------------------------------------------------
template <int PREC, int KIND>
__global__ void __launch_bounds__(NT) k_gemm(const ClassDesc* __restrict__ cls, const int4* __restrict__ work,
                                             int nwork, const void* __restrict__ cin, void* __restrict__ cout,
                                             DebugArgs dbg) {
  using T = typename DT<PREC>::t;
  using AccT = typename Acc<PREC>::t;
  __shared__ __align__(16) unsigned char sm[Lds<PREC>::total];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  const int nitems = KIND == K_DEBUG ? ((dbg.M + BM - 1) / BM) * ((dbg.N + BN - 1) / BN) : nwork;
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
    Tile t;
    const void* tab = nullptr;
    int64_t plane = 0;
    const void* xbase = nullptr;
    if constexpr (KIND == K_DEBUG) {
      const int ntn = (dbg.N + BN - 1) / BN;
      t.M = dbg.M;
      t.K = dbg.K;
      t.Ncc = (dbg.N + 1) / 2;
      t.row0 = (w / ntn) * BM;
      t.col0 = (w % ntn) * BNC;
      t.q = 0;
      t.pitch = 0;
      t.C = nullptr;
    } else {
      const int4 it = work[w];
      const ClassDesc& C = cls[it.x];
      t.C = &C;
      t.q = it.y;
      const int B = C.B, L = C.L;
      const int rows = B - t.q;
      constexpr int kind = KIND;
      if constexpr (KIND == K_B_FWD || KIND == K_B_INV)
        t.Ncc = (t.q ? 2 : 1) * C.nf * L;
      else
        t.Ncc = (2 * t.q + 1) * C.nf;
      const bool fwd = KIND == K_B_FWD || KIND == K_C_FWD;
      t.M = fwd ? rows : L;
      t.K = fwd ? L : rows;
      t.pitch = (t.K + BK - 1) / BK * BK;
      plane = C.Aplane[kind];
      tab = reinterpret_cast<const unsigned char*>(C.A[kind]) + C.Aoff[kind][t.q] * (int64_t)(PREC == PREC_SPLIT ? 2 : sizeof(T));
      t.row0 = it.z * BM;
      t.col0 = it.w * BNC;
      xbase = KIND == K_B_FWD ? C.F : (KIND == K_C_INV ? cin : C.g);
    }

    AccT acc[4][2], acc2[4][2];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 2; ++b)
        for (int v = 0; v < 4; ++v) {
          acc[a][b][v] = 0;
          if constexpr (PREC == PREC_SPLIT) acc2[a][b][v] = 0;
        }
    // wave-uniform MFMA block masks (rows / columns beyond the group)
    int nbi = 0, nbj = 0;
    {
      const int rleft = t.M - (t.row0 + wr);
      nbi = rleft <= 0 ? 0 : (rleft >= 64 ? 4 : (rleft + 15) / 16);
      const int cleft = 2 * t.Ncc - (2 * t.col0 + wc);
      nbj = cleft <= 0 ? 0 : (cleft >= 32 ? 2 : (cleft + 15) / 16);
    }

    // stage one chunk into LDS: A (table or debug matrix) and X
    auto to_lds = [&](const Stage<PREC>& st, int k0) {
      if constexpr (KIND == K_DEBUG) {
        for (int e = tid; e < BM * BK; e += NT) {
          const int r = e / BK, k = e - r * BK;
          const int gr = t.row0 + r, gk = k0 + k;
          const double v = (gr < t.M && gk < t.K) ? dbg.A[(int64_t)gr * t.K + gk] : 0.0;
          if constexpr (PREC == PREC_SPLIT) {
            uint16_t* As = reinterpret_cast<uint16_t*>(sm);
            const uint16_t h0 = f2bf((float)v);
            const double r1 = v - (double)bf2f(h0);
            const uint16_t h1 = f2bf((float)r1);
            As[(0 * BM + r) * PS + k] = h0;
            As[(1 * BM + r) * PS + k] = h1;
            As[(2 * BM + r) * PS + k] = f2bf((float)(r1 - (double)bf2f(h1)));
          } else {
            reinterpret_cast<T*>(sm)[r * PF + k] = (T)v;
          }
        }
      } else {
        store_a<PREC>(st, sm, tid);
      }
      store_x<PREC>(st, sm, tid);
    };
    const XCol xc = x_col<KIND>(t, t.col0 + (tid & 63));
    auto fetch = [&](Stage<PREC>& st, int k0) {
      if constexpr (KIND != K_DEBUG) load_a<PREC>(st, t, tab, plane, k0, tid);
      load_x<PREC, KIND>(st, t, xc, xbase, dbg, k0, tid);
    };
    // MFMAs of the chunk in LDS; k sub-steps wholly beyond K are skipped
    auto compute = [&](int k0) {
      const int kend = t.K - k0 < BK ? t.K - k0 : BK;
      if constexpr (PREC == PREC_SPLIT) {
        const uint16_t* As = reinterpret_cast<const uint16_t*>(sm);
        const uint16_t* Xs = reinterpret_cast<const uint16_t*>(sm + Lds<PREC>::a);
        for (int kk = 0; kk < BK; kk += 32) {
          if (kk >= kend) break;
          bf8 b[2][3];
          for (int j = 0; j < 2; ++j)
            if (j < nbj)
              for (int p = 0; p < 3; ++p)
                b[j][p] = *reinterpret_cast<const bf8*>(&Xs[(p * BN + wc + j * 16 + lr) * PS + kk + 8 * lk]);
          for (int i = 0; i < 4; ++i) {
            if (i >= nbi) continue;
            bf8 a[3];
            for (int p = 0; p < 3; ++p)
              a[p] = *reinterpret_cast<const bf8*>(&As[(p * BM + wr + i * 16 + lr) * PS + kk + 8 * lk]);
            for (int j = 0; j < 2; ++j) {
              if (j >= nbj) continue;
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][0], acc[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][1], acc2[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][0], acc2[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][2], acc2[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][1], acc2[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[j][0], acc2[i][j], 0, 0, 0);
            }
          }
        }
      } else {
        const T* As = reinterpret_cast<const T*>(sm);
        const T* Xs = reinterpret_cast<const T*>(sm + Lds<PREC>::a);
        for (int kk = 0; kk < BK; kk += 4) {
          if (kk >= kend) break;
          T a[4], b[2];
          for (int i = 0; i < 4; ++i) a[i] = As[(wr + i * 16 + lr) * PF + kk + lk];
          for (int j = 0; j < 2; ++j) b[j] = Xs[(wc + j * 16 + lr) * PF + kk + lk];
          for (int i = 0; i < 4; ++i) {
            if (i >= nbi) continue;
            for (int j = 0; j < 2; ++j) {
              if (j >= nbj) continue;
              if constexpr (PREC == PREC_F64)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
              else
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
          }
        }
      }
    };

    Stage<PREC> s0, s1;
    if constexpr (KIND == K_DEBUG) {
      for (int v = 0; v < Stage<PREC>::NA; ++v) s0.a[v] = s1.a[v] = make_uint4(0, 0, 0, 0);
    }
    fetch(s0, 0);
    if (BK < t.K) fetch(s1, BK);
    for (int k0 = 0; k0 < t.K; k0 += 2 * BK) {
      __syncthreads();  // the previous chunk's MFMAs are done with LDS
      to_lds(s0, k0);
      __syncthreads();
      if (k0 + 2 * BK < t.K) fetch(s0, k0 + 2 * BK);
      compute(k0);
      if (k0 + BK >= t.K) break;
      __syncthreads();
      to_lds(s1, k0 + BK);
      __syncthreads();
      if (k0 + 3 * BK < t.K) fetch(s1, k0 + 3 * BK);
      compute(k0 + BK);
    }

    // ---- epilogue through LDS, one 64-row half at a time.  Lane layout of a
    // 16 x 16 block: real column lane%16; rows 4*(lane/16)+v (f32 MFMAs) or
    // 4*v+lane/16 (f64 MFMA).
    T* E = reinterpret_cast<T*>(sm);
    for (int half = 0; half < 2; ++half) {
      if (t.row0 + half * 64 >= t.M) break;
      __syncthreads();
      if (wr == half * 64) {
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) {
              const int rin = PREC == PREC_F64 ? 4 * v + lk : 4 * lk + v;
              T val;
              if constexpr (PREC == PREC_SPLIT)
                val = acc[i][j][v] + acc2[i][j][v];
              else
                val = acc[i][j][v];
              E[(i * 16 + rin) * EP + wc + j * 16 + lr] = val;
            }
      }
      __syncthreads();
      const int rbase = t.row0 + half * 64;
      if constexpr (KIND == K_DEBUG) {
        for (int e = tid; e < 64 * BN; e += NT) {
          const int r = e / BN, n = e - r * BN;
          const int row = rbase + r, nr = 2 * t.col0 + n;
          if (row < t.M && nr < dbg.N) dbg.C[(int64_t)row * dbg.N + nr] = (double)E[r * EP + n];
        }
      } else if constexpr (KIND == K_C_INV) {
        // column-major output (g rows run along i = tile row): pairs of rows;
        // the output index of (row, c) is the stage-c forward operand index
        T* out = reinterpret_cast<T*>(t.C->g);
        const int cc = tid >> 3;            // 64 columns, 8 threads each
        const int c = t.col0 + cc;
        const XCol oc = x_col<K_C_FWD>(t, c);
        if (oc.ok) {
          for (int rp = (tid & 7) * 2; rp < 64; rp += 16) {
            const int row = rbase + rp;
            if (row >= t.M) break;
            const int64_t ix = x_at<K_C_FWD>(t, oc, row);
            const T r0 = E[rp * EP + 2 * cc], i0 = E[rp * EP + 2 * cc + 1];
            if (row + 1 < t.M) {
              const T r1 = E[(rp + 1) * EP + 2 * cc], i1 = E[(rp + 1) * EP + 2 * cc + 1];
              if constexpr (PREC == PREC_F64) {
                reinterpret_cast<double2*>(out)[ix] = make_double2(r0, i0);
                reinterpret_cast<double2*>(out)[ix + 1] = make_double2(r1, i1);
              } else {
                *reinterpret_cast<float4*>(out + 2 * ix) = make_float4(r0, i0, r1, i1);
              }
            } else {
              out[2 * ix] = r0;
              out[2 * ix + 1] = i0;
            }
          }
        }
      } else {
        // row-major outputs: each thread owns a pair of consecutive complex
        // columns (decoded once) and walks rows.  The output index of (row, c)
        // is the operand index of the opposite direction: stage-b forward
        // writes where stage-b inverse reads, and so on.
        constexpr int DUAL = KIND ^ 1;
        T* out = reinterpret_cast<T*>(KIND == K_B_FWD ? t.C->g : (KIND == K_B_INV ? t.C->F : cout));
        const int cp = (tid & 31) * 2;
        const int c = t.col0 + cp;
        const XCol o0 = x_col<DUAL>(t, c);
        const XCol o1 = x_col<DUAL>(t, c + 1);
        T s0 = 1, s1 = 1;
        if constexpr (KIND == K_B_FWD || KIND == K_B_INV) {
          const int ncf = t.C->nf * t.C->L;
          if ((t.q & 1) && c >= ncf) s0 = -1;
          if ((t.q & 1) && c + 1 >= ncf) s1 = -1;
        }
        if (o0.ok) {
          for (int r = tid >> 5; r < 64; r += NT / 32) {
            const int row = rbase + r;
            if (row >= t.M) break;
            const int64_t i0 = x_at<DUAL>(t, o0, row);
            const T re0 = s0 * E[r * EP + 2 * cp], im0 = s0 * E[r * EP + 2 * cp + 1];
            if (o1.ok) {
              const int64_t i1 = x_at<DUAL>(t, o1, row);
              const T re1 = s1 * E[r * EP + 2 * cp + 2], im1 = s1 * E[r * EP + 2 * cp + 3];
              if constexpr (PREC != PREC_F64) {
                if (i1 == i0 + 1 && ((reinterpret_cast<uintptr_t>(out + 2 * i0) & 15) == 0)) {
                  *reinterpret_cast<float4*>(out + 2 * i0) = make_float4(re0, im0, re1, im1);
                  continue;
                }
              }
              if constexpr (PREC == PREC_F64) {
                reinterpret_cast<double2*>(out)[i1] = make_double2(re1, im1);
              } else {
                out[2 * i1] = re1;
                out[2 * i1 + 1] = im1;
              }
            }
            if constexpr (PREC == PREC_F64) {
              reinterpret_cast<double2*>(out)[i0] = make_double2(re0, im0);
            } else {
              out[2 * i0] = re0;
              out[2 * i0 + 1] = im0;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

inline int grid_for(int nwork, int max_grid) {
  const int g = max_grid > 0 ? max_grid : 8192;
  return nwork < g ? nwork : g;
}

template <int PREC>
hipError_t launch_kind(int kind, const ClassDesc* d_cls, const int4* d_work, int nwork, const void* cin, void* cout,
                       int max_grid, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  DebugArgs dbg{0, 0, 0, nullptr, nullptr, nullptr};
  dim3 grid(grid_for(nwork, max_grid)), block(NT);
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
                      void* cout, int max_grid, hipStream_t s) {
  if (prec == PREC_F64) return launch_kind<PREC_F64>(kind, d_cls, d_work, nwork, cin, cout, max_grid, s);
  if (prec == PREC_F32) return launch_kind<PREC_F32>(kind, d_cls, d_work, nwork, cin, cout, max_grid, s);
  return launch_kind<PREC_SPLIT>(kind, d_cls, d_work, nwork, cin, cout, max_grid, s);
}

}  // namespace

int gemm_tile_m() { return BM; }
int gemm_tile_n_complex() { return BNC; }
int gemm_k_chunk() { return BK; }

hipError_t launch_legendre(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork,
                           int max_grid, hipStream_t s) {
  return launch_any(prec, inverse ? K_B_INV : K_B_FWD, d_cls, d_work, nwork, nullptr, nullptr, max_grid, s);
}

hipError_t launch_radial(int prec, bool inverse, const ClassDesc* d_cls, const int4* d_work, int nwork,
                         const void* coeffs_in, void* coeffs_out, int max_grid, hipStream_t s) {
  return launch_any(prec, inverse ? K_C_INV : K_C_FWD, d_cls, d_work, nwork, coeffs_in, coeffs_out, max_grid, s);
}

hipError_t launch_debug_gemm(int prec, int M, int N, int K, const double* A, const double* X, double* C,
                             hipStream_t s) {
  DebugArgs dbg{M, N, K, A, X, C};
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles == 0) return hipSuccess;
  dim3 grid(grid_for(tiles, 0)), block(NT);
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
