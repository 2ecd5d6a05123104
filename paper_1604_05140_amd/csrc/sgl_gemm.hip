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
//     spectrum F is read from HBM once; K in chunks through LDS (32 for the
//     split and FP32 forms, 64 for FP64), with register stages that issue the
//     loads of the next chunk (FP32: the next two) before the MFMAs of the
//     current one;
//   * the table operand comes pre-packed per direction (row-major, K padded to
//     a multiple of 64 with zeros), so every table load is a 16-byte vector;
//   * data-operand loads follow the layout the previous stage wrote: each
//     thread holds BK / 8 consecutive k of one column (index offsets in 32-bit
//     arithmetic from a per-column pointer), and the chunk goes to LDS as
//     [column][k] (split form: one 8-byte LDS store per column, part and bf16
//     plane); loads past the group are clamped instead of branched around;
//   * the epilogue writes the accumulators straight into the next stage's
//     layout (each store instruction covers 64-byte runs of 4 rows):
//       F    [(m+B-1)][j][b*2B+i]                 (stage a <-> b)
//       g    [l][b][m+l][i], block l at l^2 nf 2B  (stage b <-> c)
//       fhat [b][omega]                             (stage c <-> caller)
//
// Precisions: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4), and a
// three-piece bf16 split of both operands (x = x0 + x1 + x2: the packed tables
// by round-to-nearest of each remainder, the data by exact truncation, split3)
// whose six products of order <= 2 run on v_mfma_f32_16x16x32_bf16 into one
// FP32 accumulator per output, smallest products first.
//
// The split-form Legendre contractions (both directions) have a kernel of
// their own, k_legendre_split below, fed by global -> LDS copies; the forward
// radial contractions of the split and FP32 forms and the FP32 Legendre
// contractions run on the same design as a third tile geometry of their slots
// (k_radial_split, k_radial_f32, k_legendre_f32), which the plan-time
// autotuner weighs against the two of this kernel.
#include "sgl_internal.h"

namespace sgl {
namespace {

// Tile geometries of k_gemm; the plan-time autotuner picks one per launch slot.
//   TG 0: 128 rows x 64 complex columns, 512 threads, 8 waves (2 x 4) of 64 x 32
//         real outputs;
//   TG 1:  64 rows x 32 complex columns, 256 threads, 4 waves (1 x 4) of 64 x 16.
// Both stage the same number of operand elements per thread, so their register
// budgets are the same; TG 1 wastes less of its tile on the short row ranges of
// the high orders / degrees and the narrow column ranges of low degrees and
// small batches, at the price of more table re-reads per column.
template <int TG> struct Geo {
  static constexpr int BM = TG == 0 ? 128 : 64;   // rows per tile
  static constexpr int BNC = TG == 0 ? 64 : 32;   // complex columns per tile
  static constexpr int BN = 2 * BNC;              // real columns per tile
  static constexpr int NT = TG == 0 ? 512 : 256;  // threads per block
  static constexpr int WN = BN / 4;               // real columns per wave (4 waves across)
  static constexpr int NBJ = WN / 16;             // 16-column MFMA blocks per wave
};
constexpr int kNumGeo = 2;
constexpr int BM = Geo<0>::BM, BN = Geo<0>::BN, BNC = Geo<0>::BNC, NT = Geo<0>::NT;  // the default tile

enum Kind { K_B_FWD = 0, K_B_INV = 1, K_C_FWD = 2, K_C_INV = 3, K_DEBUG = 4 };

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));  // 16-byte operand vector

// Contraction chunk per precision: 32 for the bf16-split and FP32 forms (two
// blocks of 60 KB LDS fit a CU), 64 for FP64.  The packed tables pad K to it.
template <int PREC, int TG = 0> struct Cfg {
  static constexpr int BK = PREC == PREC_F64 ? 64 : 32;
  static constexpr int PS = BK;      // bf16 LDS row (elements): unpadded, 16-byte slots swizzled (swz)
  // f32/f64 LDS pitch (elements): 36 floats, 66 doubles (the FP64 operand reads,
  // 8 bytes by 32 lanes a cycle, then fall on 32 distinct bank pairs)
  static constexpr int PF = PREC == PREC_F64 ? BK + 2 : BK + 4;
  static constexpr int XN = BK / 8;  // k per thread in the data-operand staging (8 k groups)
  // 16-byte table vectors per row and per thread
  static constexpr int VR = PREC == PREC_SPLIT ? BK / 8 : (PREC == PREC_F32 ? BK / 4 : BK / 2);
  static constexpr int NA = (PREC == PREC_SPLIT ? 3 : 1) * Geo<TG>::BM * VR / Geo<TG>::NT;
  static_assert(NA * Geo<TG>::NT == (PREC == PREC_SPLIT ? 3 : 1) * Geo<TG>::BM * VR, "whole table vectors per thread");
  // register stages of the operand pipeline (loads run 1 or 2 chunks ahead):
  // one keeps the split form within 128 registers (4 waves per SIMD) and FP64
  // free of spills; FP32 has room for two
  static constexpr int NS = PREC == PREC_F32 ? 2 : 1;
  // waves per SIMD the register allocation is held to
  static constexpr int WAVES = PREC == PREC_F64 ? 2 : 4;
  // Data-operand LDS rows: real and imaginary parts in two halves, the
  // imaginary half XPAD rows after the real one ends (split: 4; FP32, FP64: 8,
  // which puts the rows an MFMA operand read takes from the two halves on
  // disjoint banks; with interleaved halves the 16-byte staging stores of 8
  // consecutive columns, 2 rows apart, fell 2-way (FP32) and 4-way (FP64) on
  // the same banks).
  static constexpr int XPAD = PREC == PREC_SPLIT ? 4 : 8;
  static constexpr int XROWS = 2 * Geo<TG>::BNC + XPAD;
};

// LDS row of real column (complex column cc, part re 0 / im 1) of the data operand
template <int PREC, int TG>
__device__ inline int xrow(int cc, int part) {
  return part * (Geo<TG>::BNC + Cfg<PREC, TG>::XPAD) + cc;
}

// Split-form LDS rows are 64 bytes (32 bf16) of four 16-byte slots; slot g of
// row r sits at position g ^ ((r >> 1) & 3), and the imaginary-part rows of
// the data operand start 4 rows after the real ones (XPAD).  Measured on
// gfx950 (bank-conflict counter, one wave issuing fixed patterns): a 16-byte
// LDS read serves 16 lanes per cycle over 64 banks, but which 16 lanes share
// a cycle is not simply consecutive; this swizzle and padding keep the MFMA
// operand reads of both operands (16 rows, one slot per lane group) and the
// 16-byte table stores free of conflicts, where the former (r >> 2) swizzle
// cost 4 extra cycles per operand read.
__device__ inline int swz(int r, int g) { return g ^ ((r >> 1) & 3); }

// Thread -> (complex column cc, k group kg of 8) of the data-operand staging.
// In the split form each 16 consecutive lanes hold the 8 k groups of two
// columns (lanes 4a..4a+3: column a & 1, k groups 4 (a >> 1) .. + 3), so their
// 8-byte LDS stores fill two whole 64-byte rows.  Measured on gfx950 with a
// one-wave probe and the bank-conflict counter: LDS writes serve 128 bytes a
// cycle (8-byte writes: 16 consecutive lanes, conflict-free when byte-address
// bits 3..6 differ between them; 16-byte writes: 8 lanes, bits 4..6), reads
// 256 bytes; 16 lanes over 16 columns (or 4 rows of 32 bytes) cost one extra
// cycle per group.  Loads of a column that runs along k come in 128-byte runs.
// (8 lanes per column, k groups in lane order, is as free of conflicts but
// took the forward radial kernel 6 more registers, one wave less per SIMD.)
template <int PREC, int TG>
__device__ inline void x_thread(int tid, int& cc, int& kg) {
  if constexpr (PREC == PREC_SPLIT) {
    cc = ((tid >> 4) << 1) | ((tid >> 2) & 1);
    kg = (tid & 3) | ((tid >> 1) & 4);
  } else {
    cc = tid & (Geo<TG>::BNC - 1);
    kg = tid / Geo<TG>::BNC;
  }
}

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

template <int PREC, int TG = 0> struct Lds {
  static constexpr int a = Geo<TG>::BM * Cfg<PREC, TG>::PF * (int)sizeof(typename DT<PREC>::t);
  static constexpr int x = Cfg<PREC, TG>::XROWS * Cfg<PREC, TG>::PF * (int)sizeof(typename DT<PREC>::t);
  static constexpr int total = a + x;
};
template <int TG> struct Lds<PREC_SPLIT, TG> {
  static constexpr int a = 3 * Geo<TG>::BM * Cfg<PREC_SPLIT, TG>::PS * 2;
  static constexpr int x = 3 * Cfg<PREC_SPLIT, TG>::XROWS * Cfg<PREC_SPLIT, TG>::PS * 2;
  static constexpr int total = a + x;
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
  const void* tab;  // packed table block (stage kinds)
  int64_t plane;    // split-plane stride of the packed table (elements)
};

// A plan constant at a wave-uniform address, read through the scalar cache (a
// generic-pointer load would be a flat load, which the compiler makes wait
// for every outstanding vector-memory operation when its result is used).
template <typename T>
__device__ inline T load_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)p;
#else
  return *p;
#endif
}

template <int PREC, int KIND, int TG>
__device__ inline Tile make_tile(const ClassDesc* cls, const int4* work, int w, const DebugArgs& dbg) {
  constexpr int BM = Geo<TG>::BM, BN = Geo<TG>::BN, BNC = Geo<TG>::BNC;
  using T = typename DT<PREC>::t;
  Tile t;
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
    t.tab = nullptr;
    t.plane = 0;
  } else {
    const int4 it = work[w];
    const ClassDesc& C = cls[it.x];
    t.C = &C;
    t.q = it.y;
    const int B = C.B, L = C.L;
    const int rows = B - t.q;
    if constexpr (KIND == K_B_FWD || KIND == K_B_INV)
      t.Ncc = (t.q ? 2 : 1) * C.nf * L;
    else
      t.Ncc = (2 * t.q + 1) * C.nf;
    constexpr bool fwd = KIND == K_B_FWD || KIND == K_C_FWD;
    // grid side: 2B, or B for the seminaive cosine-domain Legendre contraction
    const int W = (KIND == K_B_FWD || KIND == K_B_INV) ? C.kb : L;
    t.M = fwd ? rows : W;
    t.K = fwd ? W : rows;
    constexpr int BK = Cfg<PREC>::BK;
    t.pitch = (t.K + BK - 1) / BK * BK;
    t.plane = C.Aplane[KIND];
    t.tab = reinterpret_cast<const unsigned char*>(C.A[KIND]) +
            load_uniform(C.Aoff[KIND] + t.q) * (int64_t)(PREC == PREC_SPLIT ? 2 : sizeof(T));
    t.row0 = it.z * BM;
    t.col0 = it.w * BNC;
  }
  return t;
}

// ---- per-thread register staging of one K chunk -----------------------------
// A: NA 16-byte table vectors; X: XN consecutive k of one complex column.
template <int PREC, int TG> struct Stage {
  static constexpr int NA = Cfg<PREC, TG>::NA;
  u4 a[NA];
  typename DT<PREC>::t xr[Cfg<PREC, TG>::XN], xi[Cfg<PREC, TG>::XN];
};

// A chunk: BM rows x BK from a packed table block.  Rows past the block are
// clamped to its last row: they feed only output rows that are never stored.
template <int PREC, int TG>
__device__ inline void load_a(Stage<PREC, TG>& st, const Tile& t, int k0, int tid) {
  using C = Cfg<PREC, TG>;
  constexpr int BM = Geo<TG>::BM, NT = Geo<TG>::NT;
  const int rmax = t.M - 1;
  constexpr int EV = PREC == PREC_SPLIT ? 8 : (PREC == PREC_F32 ? 4 : 2);  // elements per vector
  constexpr int ES = PREC == PREC_SPLIT ? 2 : (PREC == PREC_F32 ? 4 : 8);  // element bytes
  const SGL_G unsigned char* tab = gmem(reinterpret_cast<const unsigned char*>(t.tab));
#pragma unroll
  for (int v = 0; v < C::NA; ++v) {
    const int e = tid + v * NT;  // plane, row, vector (a row's vectors in consecutive lanes)
    const int p = PREC == PREC_SPLIT ? e / (BM * C::VR) : 0;
    const int rem = e - p * (BM * C::VR);
    const int r = rem / C::VR, kg = rem - r * C::VR;
    const int gr = min(t.row0 + r, rmax);
    const int64_t off = (int64_t)gr * t.pitch + k0 + kg * EV;
    st.a[v] = *reinterpret_cast<const SGL_G u4*>(tab + ES * (PREC == PREC_SPLIT ? p * t.plane + off : off));
  }
}

template <int PREC, int TG>
__device__ inline void store_a(const Stage<PREC, TG>& st, unsigned char* sm, int tid) {
  using C = Cfg<PREC, TG>;
  constexpr int BM = Geo<TG>::BM, NT = Geo<TG>::NT;
  constexpr int EV = PREC == PREC_SPLIT ? 8 : (PREC == PREC_F32 ? 4 : 2);
  constexpr int ES = PREC == PREC_SPLIT ? 2 : (PREC == PREC_F32 ? 4 : 8);
  constexpr int P = PREC == PREC_SPLIT ? C::PS : C::PF;
#pragma unroll
  for (int v = 0; v < C::NA; ++v) {
    const int e = tid + v * NT;
    const int p = PREC == PREC_SPLIT ? e / (BM * C::VR) : 0;
    const int rem = e - p * (BM * C::VR);
    const int r = rem / C::VR, kg = rem - r * C::VR;
    const int slot = PREC == PREC_SPLIT ? swz(r, kg) : kg;
    *reinterpret_cast<u4*>(sm + ES * ((p * BM + r) * P + slot * EV)) = st.a[v];
  }
}

// One complex column of a stage operand (the data operand X of a kind, or the
// output of the opposite kind, which has the same layout): element (k, c) sits
// at p[2 * off(k)], p[2 * off(k) + 1] with a 32-bit offset off(k) (x_off) from a
// 64-bit column pointer.  Class workspaces hold fewer than 2^31 complex values.
//   K_B_FWD  F[(m+B-1)][j = k][b 2B + i]:   off = k * a,              a = nf 2B
//   K_B_INV  g[l = m + k][b][m + l][i]:     off = l (l a + b),        a = nf 2B, b = (2b+1) 2B
//   K_C_FWD  g[l][b][m + l][i = k]:         off = k
//   K_C_INV  fhat[b][omega(n = l+1+k, l, m)]: off = n (n-1) (2n-1) / 6
template <typename T>
struct XCol {
  SGL_G T* p;
  int a, b;
  T sgn;  // (-1)^m on the -m segment of stage b, else 1
};

template <int KIND, typename T>
__device__ inline XCol<T> x_col(const Tile& t, int c, T* base) {
  XCol<T> x{gmem(base), 0, 0, (T)1};
  const ClassDesc& C = *t.C;
  // class fields through the scalar cache (t.C is wave-uniform)
  const int B = load_uniform(&C.B), L = load_uniform(&C.L), nf = load_uniform(&C.nf);
  if constexpr (KIND == K_B_FWD || KIND == K_B_INV) {
    const int ncf = nf * L;
    const int seg = c >= ncf;
    const int cp = c - seg * ncf;
    const int mp = seg ? -t.q : t.q;
    if (seg && (t.q & 1)) x.sgn = (T)-1;
    if constexpr (KIND == K_B_FWD) {
      x.p = gmem(base) + 2 * ((int64_t)(mp + B - 1) * L * ncf + cp);
      x.a = ncf;
    } else {
      const int b = cp / L, i = cp - b * L;
      x.p = gmem(base) + 2 * ((int64_t)(b + mp) * L + i);
      x.a = nf * L;
      x.b = (2 * b + 1) * L;
    }
  } else if constexpr (KIND == K_C_FWD) {
    x.p = gmem(base) + 2 * ((int64_t)t.q * t.q * nf * L + (int64_t)c * L);
  } else {  // K_C_INV
    const int l = t.q;
    const int b = c / (2 * l + 1);
    const int m = c - b * (2 * l + 1) - l;
    // the function's coefficient offset: in closed form when the class's
    // functions are stored one after another (no per-lane load, which would
    // wait for every outstanding copy in the copy-fed kernels); a loaded one
    // is consumed in its own branch, so that the wait stays there and not
    // after the two paths join
    const int64_t cstep = load_uniform(&C.cstep);
    int64_t cb;
    if (cstep) {
      cb = load_uniform(&C.cbase) + b * cstep;
    } else {
      cb = gmem(load_uniform(&C.coff))[b];
      asm volatile("" ::"v"(cb));
    }
    x.p = gmem(base) + 2 * (cb + (int64_t)l * (l + 1) + m);
  }
  return x;
}

template <int KIND, typename T>
__device__ inline int x_off(const Tile& t, const XCol<T>& x, int k) {
  if constexpr (KIND == K_B_FWD) {
    return k * x.a;
  } else if constexpr (KIND == K_B_INV) {
    const int l = t.q + k;
    return l * (l * x.a + x.b);
  } else if constexpr (KIND == K_C_FWD) {
    return k;
  } else {
    const int n = t.q + 1 + k;
    return n * (n - 1) * (2 * n - 1) / 6;
  }
}

template <typename T> struct V2 { using t = float2; };
template <> struct V2<double> { using t = double2; };

// X chunk: thread -> (complex column cc, k group kg of XN rows), see x_thread.
// rows).  Columns and rows past the group are clamped to its last ones: the
// packed tables are zero past K, and extra columns are never stored.
template <int PREC, int KIND, int TG>
__device__ inline void load_x(Stage<PREC, TG>& st, const Tile& t, const XCol<typename DT<PREC>::t>& xc,
                              const DebugArgs& dbg, int k0, int tid) {
  using T = typename DT<PREC>::t;
  using T2 = typename V2<T>::t;
  constexpr int XN = Cfg<PREC, TG>::XN;
  int cc, kg;
  x_thread<PREC, TG>(tid, cc, kg);
  const int kb = k0 + kg * XN;
  if constexpr (KIND == K_DEBUG) {
    const int c = t.col0 + cc;
#pragma unroll
    for (int u = 0; u < XN; ++u) {
      const int k = kb + u;
      const int n0 = 2 * c, n1 = 2 * c + 1;
      const bool ok = k < t.K;
      st.xr[u] = (ok && n0 < dbg.N) ? (T)gmem(dbg.X)[(int64_t)k * dbg.N + n0] : (T)0;
      st.xi[u] = (ok && n1 < dbg.N) ? (T)gmem(dbg.X)[(int64_t)k * dbg.N + n1] : (T)0;
    }
  } else {
    const int kmax = t.K - 1;
    if constexpr (KIND == K_C_FWD && PREC != PREC_F64) {
      if (kb + XN <= t.K) {
        // XN consecutive k of one column are contiguous (g rows run along i)
        const SGL_G float4* src = reinterpret_cast<const SGL_G float4*>(xc.p + 2 * kb);
#pragma unroll
        for (int u = 0; u < XN / 2; ++u) {
          const float4 v = src[u];
          st.xr[2 * u] = v.x;
          st.xi[2 * u] = v.y;
          st.xr[2 * u + 1] = v.z;
          st.xi[2 * u + 1] = v.w;
        }
        return;
      }
    }
#pragma unroll
    for (int u = 0; u < XN; ++u) {
      const int k = min(kb + u, kmax);
      if constexpr (KIND == K_B_FWD) {
        // spectrum rows are read once: streaming loads keep g cached for stage (c)
        const SGL_G T* q = xc.p + 2 * x_off<KIND>(t, xc, k);
        st.xr[u] = __builtin_nontemporal_load(q);
        st.xi[u] = __builtin_nontemporal_load(q + 1);
      } else {
        const T2 v = *reinterpret_cast<const SGL_G T2*>(xc.p + 2 * x_off<KIND>(t, xc, k));
        st.xr[u] = v.x;
        st.xi[u] = v.y;
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

// X chunk to LDS as [column][k]; sgn carries the (-1)^m of the -m segment.
template <int PREC, int TG>
__device__ inline void store_x(const Stage<PREC, TG>& st, typename DT<PREC>::t sgn, unsigned char* sm, int tid) {
  using C = Cfg<PREC, TG>;
  constexpr int XN = C::XN;
  int cc, kg;
  x_thread<PREC, TG>(tid, cc, kg);
  if constexpr (PREC == PREC_SPLIT) {
    static_assert(XN == 4, "split staging holds 4 k per thread");
    uint16_t* Xs = reinterpret_cast<uint16_t*>(sm + Lds<PREC, TG>::a);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      uint32_t h[3][XN];
#pragma unroll
      for (int u = 0; u < XN; ++u) split3(sgn * (part ? st.xi[u] : st.xr[u]), h[0][u], h[1][u], h[2][u]);
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        uint2 w;
        w.x = pack_hi(h[p][0], h[p][1]);
        w.y = pack_hi(h[p][2], h[p][3]);
        const int row = xrow<PREC, TG>(cc, part);
        *reinterpret_cast<uint2*>(&Xs[(p * C::XROWS + row) * C::PS + swz(row, kg >> 1) * 8 + (kg & 1) * 4]) = w;
      }
    }
  } else if constexpr (PREC == PREC_F32) {
    static_assert(XN == 4, "f32 staging holds 4 k per thread");
    float* Xs = reinterpret_cast<float*>(sm + Lds<PREC, TG>::a);
    *reinterpret_cast<float4*>(&Xs[xrow<PREC, TG>(cc, 0) * C::PF + kg * XN]) =
        make_float4(sgn * st.xr[0], sgn * st.xr[1], sgn * st.xr[2], sgn * st.xr[3]);
    *reinterpret_cast<float4*>(&Xs[xrow<PREC, TG>(cc, 1) * C::PF + kg * XN]) =
        make_float4(sgn * st.xi[0], sgn * st.xi[1], sgn * st.xi[2], sgn * st.xi[3]);
  } else {
    double* Xs = reinterpret_cast<double*>(sm + Lds<PREC, TG>::a);
    double* r0 = &Xs[xrow<PREC, TG>(cc, 0) * C::PF + kg * XN];
    double* r1 = &Xs[xrow<PREC, TG>(cc, 1) * C::PF + kg * XN];
#pragma unroll
    for (int u = 0; u < XN; u += 2) {
      *reinterpret_cast<double2*>(r0 + u) = make_double2(sgn * st.xr[u], sgn * st.xr[u + 1]);
      *reinterpret_cast<double2*>(r1 + u) = make_double2(sgn * st.xi[u], sgn * st.xi[u + 1]);
    }
  }
}

template <int PREC, int KIND>
__device__ inline typename DT<PREC>::t* x_base(const Tile& t, const void* cin) {
  using T = typename DT<PREC>::t;
  if constexpr (KIND == K_B_FWD) return reinterpret_cast<T*>(load_uniform(&t.C->F));
  else if constexpr (KIND == K_C_INV) return const_cast<T*>(reinterpret_cast<const T*>(cin));
  else if constexpr (KIND == K_DEBUG) return nullptr;
  else return reinterpret_cast<T*>(load_uniform(&t.C->g));
}

// ---- the kernel ------------------------------------------------------------
// Persistent blocks walk the work list.  Per item: K in chunks of BK through
// LDS with NS register stages; before an item's outputs are written, the
// first chunks of the block's next item are already being loaded (split and
// FP32 forms), so the load latency of short contractions overlaps the stores.  Outputs go straight
// from the accumulators to the next stage's layout.
template <int PREC, int KIND, int TG>
__global__ void __launch_bounds__(Geo<TG>::NT) __attribute__((amdgpu_waves_per_eu(Cfg<PREC>::WAVES)))
k_gemm(const ClassDesc* __restrict__ cls, const int4* __restrict__ work, int nwork, const void* __restrict__ cin,
       void* __restrict__ cout, DebugArgs dbg) {
  using T = typename DT<PREC>::t;
  using AccT = typename Acc<PREC>::t;
  using G = Geo<TG>;
  constexpr int BM = G::BM, BN = G::BN, NT = G::NT, NBJ = G::NBJ;
  constexpr int BK = Cfg<PREC, TG>::BK, PS = Cfg<PREC, TG>::PS, PF = Cfg<PREC, TG>::PF;
  __shared__ __align__(16) unsigned char sm[Lds<PREC, TG>::total];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // wave tile: 64 rows x WN real columns (TG 0: waves 2 x 4, TG 1: 1 x 4)
  const int wr = (wave >> 2) * 64, wc = (wave & 3) * G::WN;
  const int lr = lane & 15, lk = lane >> 4;

  const int nitems = KIND == K_DEBUG ? ((dbg.M + BM - 1) / BM) * ((dbg.N + BN - 1) / BN) : nwork;
  int w = blockIdx.x;
  if (w >= nitems) return;

  auto column = [&](const Tile& tt) {
    XCol<T> x{nullptr, 0, 0, (T)1};
    if constexpr (KIND != K_DEBUG) {
      int cc, kg;
      x_thread<PREC, TG>(tid, cc, kg);
      x = x_col<KIND>(tt, min(tt.col0 + cc, tt.Ncc - 1), x_base<PREC, KIND>(tt, cin));
    }
    return x;
  };
  auto fetch = [&](Stage<PREC, TG>& st, const Tile& tt, const XCol<T>& x, int k0) {
    if constexpr (KIND != K_DEBUG) load_a<PREC, TG>(st, tt, k0, tid);
    load_x<PREC, KIND, TG>(st, tt, x, dbg, k0, tid);
  };

  Tile t = make_tile<PREC, KIND, TG>(cls, work, w, dbg);
  XCol<T> xc = column(t);
  Stage<PREC, TG> s0, s1;
  if constexpr (KIND == K_DEBUG) {
    for (int v = 0; v < Stage<PREC, TG>::NA; ++v) s0.a[v] = s1.a[v] = u4{0, 0, 0, 0};
  }
  // FP64 stages are too large to stay live across the epilogue: its items load
  // their first chunks at their start.
  constexpr bool kAhead = PREC != PREC_F64;
  constexpr int NS = Cfg<PREC>::NS;
  // the split form accumulates its six products in one FP32 accumulator per
  // output (a second one for the corrections would cost the occupancy)
  constexpr bool kCorr = false;
  if (kAhead) {
    fetch(s0, t, xc, 0);
    if (NS == 2 && BK < t.K) fetch(s1, t, xc, BK);
  }

  for (;;) {
    if (!kAhead) {
      fetch(s0, t, xc, 0);
      if (NS == 2 && BK < t.K) fetch(s1, t, xc, BK);
    }
    AccT acc[4][NBJ], acc2[4][NBJ];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NBJ; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[a][b][v] = 0;
          if constexpr (kCorr) acc2[a][b][v] = 0;
        }
    // wave-uniform MFMA block masks (rows / columns beyond the group)
    int nbi = 0, nbj = 0;
    {
      const int rleft = t.M - (t.row0 + wr);
      nbi = rleft <= 0 ? 0 : (rleft >= 64 ? 4 : (rleft + 15) / 16);
      const int cleft = 2 * t.Ncc - (2 * t.col0 + wc);
      nbj = cleft <= 0 ? 0 : (cleft >= 16 * NBJ ? NBJ : (cleft + 15) / 16);
    }

    // stage one chunk into LDS: A (table or debug matrix) and X
    auto to_lds = [&](const Stage<PREC, TG>& st, int k0) {
      if constexpr (KIND == K_DEBUG) {
        for (int e = tid; e < BM * BK; e += NT) {
          const int r = e / BK, k = e - r * BK;
          const int gr = t.row0 + r, gk = k0 + k;
          const double v = (gr < t.M && gk < t.K) ? gmem(dbg.A)[(int64_t)gr * t.K + gk] : 0.0;
          if constexpr (PREC == PREC_SPLIT) {
            uint16_t* As = reinterpret_cast<uint16_t*>(sm);
            const uint16_t h0 = f2bf((float)v);
            const double r1 = v - (double)bf2f(h0);
            const uint16_t h1 = f2bf((float)r1);
            const int ks = swz(r, k >> 3) * 8 + (k & 7);
            As[(0 * BM + r) * PS + ks] = h0;
            As[(1 * BM + r) * PS + ks] = h1;
            As[(2 * BM + r) * PS + ks] = f2bf((float)(r1 - (double)bf2f(h1)));
          } else {
            reinterpret_cast<T*>(sm)[r * PF + k] = (T)v;
          }
        }
      } else {
        store_a<PREC, TG>(st, sm, tid);
      }
      store_x<PREC, TG>(st, xc.sgn, sm, tid);
    };
    // MFMAs of the chunk in LDS; k sub-steps wholly beyond K are skipped
    auto compute = [&](int k0) {
      const int kend = t.K - k0 < BK ? t.K - k0 : BK;
      if constexpr (PREC == PREC_SPLIT) {
        const uint16_t* As = reinterpret_cast<const uint16_t*>(sm);
        const uint16_t* Xs = reinterpret_cast<const uint16_t*>(sm + Lds<PREC, TG>::a);
        static_assert(BK == 32, "one 16x16x32 MFMA step per chunk: lane slot lk covers k 8lk..8lk+7");
        if (kend > 0) {
          bf8 b[NBJ][3];
#pragma unroll
          for (int j = 0; j < NBJ; ++j)
            if (j < nbj)
#pragma unroll
              for (int p = 0; p < 3; ++p) {
                const int row = xrow<PREC, TG>((wc + j * 16 + lr) >> 1, lr & 1);
                b[j][p] =
                    *reinterpret_cast<const bf8*>(&Xs[(p * Cfg<PREC, TG>::XROWS + row) * PS + swz(row, lk) * 8]);
              }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (i >= nbi) continue;
            bf8 a[3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
              a[p] = *reinterpret_cast<const bf8*>(&As[(p * BM + wr + i * 16 + lr) * PS + swz(wr + i * 16 + lr, lk) * 8]);
#pragma unroll
            for (int j = 0; j < NBJ; ++j) {
              if (j >= nbj) continue;
              // smallest products first, the main product last
              AccT& c2 = kCorr ? acc2[i][j] : acc[i][j];
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[j][0], c2, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][1], c2, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][2], c2, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][0], c2, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][1], c2, 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][0], acc[i][j], 0, 0, 0);
            }
          }
        }
      } else {
        const T* As = reinterpret_cast<const T*>(sm);
        const T* Xs = reinterpret_cast<const T*>(sm + Lds<PREC, TG>::a);
        for (int kk = 0; kk < BK; kk += 4) {
          if (kk >= kend) break;
          T a[4], b[NBJ];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = As[(wr + i * 16 + lr) * PF + kk + lk];
#pragma unroll
          for (int j = 0; j < NBJ; ++j) b[j] = Xs[xrow<PREC, TG>((wc + j * 16 + lr) >> 1, lr & 1) * PF + kk + lk];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (i >= nbi) continue;
#pragma unroll
            for (int j = 0; j < NBJ; ++j) {
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

    if constexpr (NS == 2) {
      for (int k0 = 0; k0 < t.K; k0 += 2 * BK) {
        __syncthreads();  // the previous chunk's MFMAs are done with LDS
        to_lds(s0, k0);
        __syncthreads();
        if (k0 + 2 * BK < t.K) fetch(s0, t, xc, k0 + 2 * BK);
        compute(k0);
        if (k0 + BK >= t.K) break;
        __syncthreads();
        to_lds(s1, k0 + BK);
        __syncthreads();
        if (k0 + 3 * BK < t.K) fetch(s1, t, xc, k0 + 3 * BK);
        compute(k0 + BK);
      }
    } else {
      for (int k0 = 0; k0 < t.K; k0 += BK) {
        __syncthreads();  // the previous chunk's MFMAs are done with LDS
        to_lds(s0, k0);
        __syncthreads();
        if (k0 + BK < t.K) fetch(s0, t, xc, k0 + BK);
        compute(k0);
      }
    }

    // the block's next item: its first chunks load while this one is written
    const int wn = w + gridDim.x;
    const bool more = wn < nitems;
    Tile tn = t;
    XCol<T> xn = xc;
    if (more) {
      tn = make_tile<PREC, KIND, TG>(cls, work, wn, dbg);
      xn = column(tn);
      if (kAhead) {
        fetch(s0, tn, xn, 0);
        if (NS == 2 && BK < tn.K) fetch(s1, tn, xn, BK);
      }
    }

    // ---- epilogue: accumulators straight to the output layout.  Lane layout
    // of a 16 x 16 block: real column lane%16; rows 4*(lane/16)+v (f32 MFMAs)
    // or 4*v+lane/16 (f64 MFMA).  The output of a kind has the layout of the
    // opposite kind's operand (KIND ^ 1), except stage c inverse, whose g
    // output is column-major (rows along i).
    auto value = [&](int i, int j, int v) -> T {
      if constexpr (kCorr)
        return acc[i][j][v] + acc2[i][j][v];
      else
        return acc[i][j][v];
    };
    auto row_of = [&](int i, int v) { return t.row0 + wr + i * 16 + (PREC == PREC_F64 ? 4 * v + lk : 4 * lk + v); };
    if constexpr (KIND == K_DEBUG) {
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        const int nr = 2 * t.col0 + wc + j * 16 + lr;
        if (j >= nbj || nr >= dbg.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row_of(i, v);
            if (i < nbi && row < t.M) gmem(dbg.C)[(int64_t)row * dbg.N + nr] = (double)value(i, j, v);
          }
      }
    } else if constexpr (KIND == K_C_INV) {
      T* gout = reinterpret_cast<T*>(t.C->g);
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        const int rc = wc + j * 16 + lr;  // real column in the tile
        const int c = t.col0 + (rc >> 1);
        if (j >= nbj) continue;
        const XCol<T> oc = x_col<K_C_FWD>(t, min(c, t.Ncc - 1), gout);
        const bool okc = c < t.Ncc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i >= nbi) continue;
          if constexpr (PREC == PREC_F64) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = row_of(i, v);
              if (okc && row < t.M) oc.p[2 * row + (rc & 1)] = value(i, j, v);
            }
          } else {
            // lanes lr and lr^1 hold re / im of the same column for rows
            // r0..r0+3: swap halves so that each lane stores two complex values
            const int r0 = row_of(i, 0);
            const bool even = (rc & 1) == 0;
            const T v0 = value(i, j, 0), v1 = value(i, j, 1), v2 = value(i, j, 2), v3 = value(i, j, 3);
            const T send0 = even ? v2 : v0, send1 = even ? v3 : v1;
            const T got0 = __shfl_xor(send0, 1), got1 = __shfl_xor(send1, 1);
            const int rs = even ? r0 : r0 + 2;  // first of the two rows this lane stores
            const float4 o = even ? make_float4(v0, got0, v1, got1) : make_float4(got0, v2, got1, v3);
            if (okc) {
              if (rs + 1 < t.M) {
                *reinterpret_cast<SGL_G float4*>(oc.p + 2 * rs) = o;
              } else if (rs < t.M) {
                *reinterpret_cast<SGL_G float2*>(oc.p + 2 * rs) = make_float2(o.x, o.y);
              }
            }
          }
        }
      }
    } else {
      constexpr int DUAL = KIND ^ 1;
      T* obase = KIND == K_B_FWD ? reinterpret_cast<T*>(t.C->g)
                                 : (KIND == K_B_INV ? reinterpret_cast<T*>(t.C->F) : reinterpret_cast<T*>(cout));
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        const int rc = wc + j * 16 + lr;
        const int c = t.col0 + (rc >> 1);
        if (j >= nbj) continue;
        const XCol<T> oc = x_col<DUAL>(t, min(c, t.Ncc - 1), obase);
        SGL_G T* op = oc.p + (rc & 1);
        const bool okc = c < t.Ncc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i >= nbi) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row_of(i, v);
            if (okc && row < t.M) {
              // the spectrum rows of the inverse Legendre stage stream out (they
              // are read once, in full, by the inverse FFT)
              if constexpr (KIND == K_B_INV)
                __builtin_nontemporal_store(value(i, j, v), &op[2 * x_off<DUAL>(t, oc, row)]);
              else
                op[2 * x_off<DUAL>(t, oc, row)] = value(i, j, v);
            }
          }
        }
      }
    }
    if (!more) break;
    w = wn;
    t = tn;
    xc = xn;
  }
}

// ---- split-form Legendre and forward radial stages: operands by global -> LDS
// copies.  These contractions stream their data operand (the spectrum F and
// the intermediate g forward, g inverse).  The register-staged kernel above
// holds one chunk ahead within its register budget.  This kernel moves both
// operands with 16-byte global ->
// LDS copies (no registers, no LDS stores): the table through two LDS stages,
// the data through three, so that the data of the next two chunks are in
// flight while a chunk is used, across the boundaries of a block's items.
// All its vector-memory loads are such copies, so the waits are its own (the
// compiler makes any use of a loaded register wait for every outstanding
// copy).  The inverse writes 128 KB per item: its stores are issued by every
// lane in a fixed number, so that the next item's first wait can leave them
// outstanding (with one block per CU nothing else would hide their drain).
//   block: 1024 threads, 16 waves in a 2 x 8 layout; tile 128 rows x 128
//   complex columns; wave (wr, wc) computes rows wr..wr+63 of complex columns
//   wc..wc+15 as two 16-column MFMA blocks, real and imaginary parts;
//   table chunk (3 planes x 128 rows x 32 k, 64 bytes a row and plane, in the
//   swizzled slot order of swz): 24 copies of 1 KB (16 rows of one plane),
//   copy q by wave q % 16 (waves 0..7 also take q = 16..23);
//   Legendre data chunk (32 rows x 128 complex columns, 1 KB a row as in
//   memory): wave w copies rows 2w and 2w + 1, lane l the complex column pair
//   2l, 2l + 1; rows sit kLRow = 1040 bytes apart, so that rows 8 apart (the k
//   groups of an MFMA operand read) fall in opposite halves of the LDS banks.
//   Radial data chunk (128 complex columns x 32 k; a column of g runs along k
//   in memory): LDS row R = 128 s + c holds k = 8s..8s+7 of column c (64
//   bytes, four 16-byte slots of two k each), slot q at position
//   q ^ ((R >> 1) & 3) ^ s.  A copy fills 16 rows (16 columns of one s), four
//   lanes a 64-byte run of a column; the MFMA operand read of lane (column lr,
//   k group lk) takes the four slots of row 128 lk + c, so its 16-byte reads
//   fall on the LDS positions of the table reads (row lr, slot lk, which are
//   free of bank conflicts) up to a fixed relabelling (xor with q).
// LDS: 2 x 24 KB + 3 x 32.5 KB + one spare row = 147 KB, one block per CU
// (16 waves, as two 512-thread blocks of the kernel above).
//
// The FP32 Legendre contractions run on the same design (k_legendre_f32, a
// third tile geometry of their launch slots): the data chunk and its copies
// are the split form's; the table chunk is one FP32 plane (128 rows x 32 k,
// 128 bytes a row: 16 copies of 1 KB, copy q by wave q, eight rows of it),
// with the row's eight 16-byte slots in swizzled order (swz32); each lane
// takes k 8 lk .. 8 lk + 7 of the chunk, so that its data operand is the
// split form's eight rows of one complex column and its table fragment two
// 16-byte reads per row block, and runs eight 16 x 16 x 4 FP32 MFMA steps per
// block (the pairing of k with the MFMA's k slot is the same on both operands,
// so the sum over the chunk is complete).  LDS: 2 x 16 KB + 3 x 32.5 KB + one
// spare row = 130 KB.
constexpr int LT = 1024;
constexpr int LBNC = 128;
constexpr int kLRow = 1040;
constexpr int kLX = 32 * kLRow;  // one data stage
// one table stage, the spare row's offset and the LDS size per precision
template <int PREC> struct CopyLds {
  static constexpr int a = PREC == PREC_SPLIT ? 3 * BM * 64 : BM * 128;
  static constexpr int spare = 2 * a + 3 * kLX;
  static constexpr int total = spare + kLRow;
};

// Position of logical 16-byte slot L (k 4L .. 4L + 3) of row r of an FP32
// table stage: L ^ swz32(r).  A 16-byte LDS read serves, in each half wave,
// first the lane quads whose index (lane >> 2) & 7 has even bit parity, then
// the others (measured on gfx950), so lanes lr = 0..3, 12..15 of one k group
// share a cycle with lanes lr = 4..11 of the other k group of the half wave.
// An operand read (16 rows r0 + lr, slot 2 lk + h, r0 a multiple of 16) then
// takes 16 distinct (row parity, position) pairs per cycle, i.e. 16 distinct
// 16-byte bank groups: swz32 takes values with bit 1 clear (so lk of the
// other parity, slot 2 lk + h, lands on positions with bit 1 flipped) that
// differ within each of the sets lr >> 1 in {0, 1, 6, 7} and {2, 3, 4, 5}.
__device__ inline int swz32(int r) { return ((r >> 1) & 1) | (r & 4); }

#if defined(__HIP_DEVICE_COMPILE__)
#define SGL_L __attribute__((address_space(3)))
#else
#define SGL_L
#endif
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ inline unsigned lds_u32(const void* p) { return (unsigned)(uintptr_t)(const SGL_L void*)p; }

// One 16-byte global -> LDS copy per lane; lane l writes bytes 16 l .. 16 l + 15
// of the wave-uniform destination.  NT marks the source as read once
// (nontemporal cache policy), so that it does not evict what the next stage
// reads.
template <bool NT>
__device__ inline void copy16_to_lds(const SGL_G void* src, unsigned char* dst) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(src, (SGL_L void*)dst, 16, 0, NT ? 2 : 0);
#endif
}

// LDS accesses of this kernel are written in asm, each block waiting for its
// own LDS operations before it ends (outputs are early-clobber, so none shares
// a register with the address while reads are in flight): an LDS access that
// the compiler emits while copies are outstanding waits for all of them.
// Rows 8g + u, u = 0..7, of one complex column of a data stage (a: row 8g).
__device__ inline void lds_x8(unsigned a, f2v (&r)[8]) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile(
      "ds_read_b64 %0, %8\n\t"
      "ds_read_b64 %1, %8 offset:1040\n\t"
      "ds_read_b64 %2, %8 offset:2080\n\t"
      "ds_read_b64 %3, %8 offset:3120\n\t"
      "ds_read_b64 %4, %8 offset:4160\n\t"
      "ds_read_b64 %5, %8 offset:5200\n\t"
      "ds_read_b64 %6, %8 offset:6240\n\t"
      "ds_read_b64 %7, %8 offset:7280\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7])
      : "v"(a)
      : "memory");
#endif
}
// k 8g..8g+7 of one complex column of a radial data stage: its four 16-byte
// slots, at the LDS addresses a ^ 16 q (a: row start + 16 x the slot position
// of q = 0).
__device__ inline void lds_x4q(unsigned a, f2v (&r)[8]) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned a1 = a ^ 16u, a2 = a ^ 32u, a3 = a ^ 48u;
  f4 u0, u1, u2, u3;
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %5\n\t"
      "ds_read_b128 %2, %6\n\t"
      "ds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(u0), "=&v"(u1), "=&v"(u2), "=&v"(u3)
      : "v"(a), "v"(a1), "v"(a2), "v"(a3)
      : "memory");
  r[0] = f2v{u0[0], u0[1]}; r[1] = f2v{u0[2], u0[3]};
  r[2] = f2v{u1[0], u1[1]}; r[3] = f2v{u1[2], u1[3]};
  r[4] = f2v{u2[0], u2[1]}; r[5] = f2v{u2[2], u2[3]};
  r[6] = f2v{u3[0], u3[1]}; r[7] = f2v{u3[2], u3[3]};
#endif
}
// The three bf16 planes (8192 bytes apart) of one table fragment.
__device__ inline void lds_a3(unsigned a, u4 (&r)[3]) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile(
      "ds_read_b128 %0, %3\n\t"
      "ds_read_b128 %1, %3 offset:8192\n\t"
      "ds_read_b128 %2, %3 offset:16384\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2])
      : "v"(a)
      : "memory");
#endif
}
// The two 16-byte slots (k 8 lk .. 8 lk + 7) of one FP32 table row.
__device__ inline void lds_a2(unsigned a0, unsigned a1, f4 (&r)[2]) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile(
      "ds_read_b128 %0, %2\n\t"
      "ds_read_b128 %1, %3\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(r[0]), "=&v"(r[1])
      : "v"(a0), "v"(a1)
      : "memory");
#endif
}
// Workgroup barrier without the fence of __syncthreads (which waits for every
// outstanding vector-memory operation); also a compiler barrier for memory.
__device__ inline void bar_only() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_barrier" ::: "memory");
#endif
}
// Wait until at most N of the wave's vector-memory operations are outstanding.
// The vector-memory counter of the CDNA ISA (VM_CNT, waited on by s_waitcnt
// vmcnt) counts a wave's vector-memory loads, stores and global-to-LDS loads
// together and is decremented in the order they were issued (ISA reference,
// data dependency resolution), so "at most N outstanding" means "all but the
// last N issued have completed".
__device__ inline void wait_vm(int n) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (n == 2)
    asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
  else if (n == 18)
    asm volatile("s_waitcnt vmcnt(18)" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#endif
}

// target of the epilogue stores that fall outside the group (never read)
__device__ f2v g_spare_out[64];

// The body of the copy-fed kernels (PREC_SPLIT with KIND K_B_FWD, K_B_INV or
// K_C_FWD; PREC_F32 with K_B_FWD or K_B_INV; sm: CopyLds<PREC>::total bytes of
// LDS; coeffs: the coefficient output of K_C_FWD).
template <int PREC, int KIND>
__device__ __forceinline__ void copy_fed(unsigned char* sm, const ClassDesc* __restrict__ cls,
                                         const int4* __restrict__ work, int nwork, void* __restrict__ coeffs) {
  static_assert(KIND == K_B_FWD || KIND == K_B_INV || KIND == K_C_FWD, "Legendre kinds and the forward radial kind");
  static_assert(PREC == PREC_SPLIT || PREC == PREC_F32, "split or FP32 form");
  constexpr bool RAD = KIND == K_C_FWD;
  constexpr int BK = Cfg<PREC>::BK, PS = Cfg<PREC_SPLIT>::PS;
  static_assert(BK == 32 && PS == 32, "32-deep chunks; split form: 64-byte table rows");
  constexpr int LA = CopyLds<PREC>::a, SPARE = CopyLds<PREC>::spare;
  const int tid = threadIdx.x;
  // (the wave index is uniform; saying so keeps the row-block tests scalar)
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave >> 3) * 64, wc = (wave & 7) * 16;
  const int lr = lane & 15, lk = lane >> 4;
  // table copies per chunk of this wave (split: 24 of 1 KB, FP32: 16)
  const int nac = PREC == PREC_SPLIT && wave < 8 ? 2 : 1;
  DebugArgs nodbg{0, 0, 0, nullptr, nullptr, nullptr};

  int w = blockIdx.x;
  if (w >= nwork) return;

  // (the item index is wave-uniform; saying so keeps the work-list and class
  // reads on the scalar unit: a vector load here would make its first use
  // wait for every outstanding copy)
  auto tile = [&](int wi) {
    wi = __builtin_amdgcn_readfirstlane(wi);
    Tile tt = make_tile<PREC, KIND, 0>(cls, work, wi, nodbg);
    tt.col0 = load_uniform(&work[wi].w) * LBNC;
    return tt;
  };
  // the lane's copy source: Legendre, its complex column pair; radial, its
  // column (clamped to the group's last ones, never stored)
  auto col = [&](const Tile& tt) {
    if constexpr (RAD)
      return x_col<KIND>(tt, min(tt.col0 + (wave & 7) * 16 + (lane >> 2), tt.Ncc - 1),
                         x_base<PREC, KIND>(tt, nullptr));
    else
      return x_col<KIND>(tt, min(tt.col0 + 2 * lane, tt.Ncc - 2), x_base<PREC, KIND>(tt, nullptr));
  };
  // table chunk k0 into stage st (2: the spare row); rows past the block clamp
  // to its last row (they feed outputs that are never stored)
  auto copy_a = [&](const Tile& tt, int k0, int st) {
    const SGL_G unsigned char* tab = gmem(reinterpret_cast<const unsigned char*>(tt.tab));
    if constexpr (PREC == PREC_F32) {
      // rows 8 wave .. + 7, lane: row + lane / 8, slot position lane & 7
      const int r = 8 * wave + (lane >> 3);
      const int g = (lane & 7) ^ swz32(r);
      const int gr = min(tt.row0 + r, tt.M - 1);
      const int64_t off = (int64_t)gr * tt.pitch + k0 + g * 4;
      copy16_to_lds<false>(tab + 4 * off, sm + (st == 2 ? SPARE : st * LA + wave * 1024));
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (s >= nac) break;
        const int q = wave + 16 * s;
        const int p = q >> 3, r = 16 * (q & 7) + (lane >> 2);
        const int g = (lane & 3) ^ ((r >> 1) & 3);
        const int gr = min(tt.row0 + r, tt.M - 1);
        const int64_t off = p * tt.plane + (int64_t)gr * tt.pitch + k0 + g * 8;
        copy16_to_lds<false>(tab + 2 * off, sm + (st == 2 ? SPARE : st * LA + q * 1024));
      }
    }
  };
  // data chunk k0 into stage st (3: the spare row); rows past K clamp to the
  // last one (the table is zero there)
  auto copy_x = [&](const Tile& tt, const XCol<float>& x, int k0, int st) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if constexpr (RAD) {
        // rows 128 sg + 16 (wave & 7) .. + 15 (sg = k group), lane: row + lane / 4, slot
        // position lane & 3; K = 2B is even, so the clamped pair stays inside the column
        const int sg = (wave >> 3) + 2 * s;
        const int q = (lane & 3) ^ ((lane >> 3) & 3) ^ sg;
        const int k = min(k0 + 8 * sg + 2 * q, tt.K - 2);
        // streaming reads of g: each row tile of a degree reads it once (one tile
        // up to B = 128)
        copy16_to_lds<true>(x.p + 2 * k,
                            sm + (st == 3 ? SPARE : 2 * LA + st * kLX + (128 * sg + 16 * (wave & 7)) * 64));
      } else {
        const int k = min(k0 + 2 * wave + s, tt.K - 1);
        // the spectrum is read once: streaming copies keep g cached for stage (c);
        // g (inverse) is read by both row tiles of a column tile
        copy16_to_lds<KIND == K_B_FWD>(x.p + 2 * x_off<KIND>(tt, x, k),
                            sm + (st == 3 ? SPARE : 2 * LA + st * kLX + (2 * wave + s) * kLRow));
      }
    }
  };

  // The chunks of the block's items (w, w + G, w + 2G, ...) form one stream:
  // data copies run two chunks ahead of the chunk in use and table copies one,
  // across item boundaries, so the first chunks of the next item (of the next
  // two when the next has one chunk) are in flight while this item's last ones
  // are used.  Stream chunk g sits in data stage g % 3 and table stage g % 2;
  // past the block's last item the copies go to the spare row.
  const int G = gridDim.x;
  auto nchunks = [&](const Tile& tt) { return (tt.K + BK - 1) / BK; };
  Tile t = tile(w);
  int nc = nchunks(t);
  Tile t1 = t, t2 = t;  // the next two items (nc1, nc2 = 0: none or not needed)
  int nc1 = 0, nc2 = 0;
  if (w + G < nwork) {
    t1 = tile(w + G);
    nc1 = nchunks(t1);
    if (nc1 == 1 && w + 2 * G < nwork) {
      t2 = tile(w + 2 * G);
      nc2 = nchunks(t2);
    }
  }
  // copy sources of this item's and the next item's data columns (the next
  // item's is computed once, when it becomes the next, not at every copy)
  XCol<float> xc = col(t), xc1 = nc1 > 0 ? col(t1) : xc;
  int run = 0;  // stream index of this item's first chunk, mod 6
  bool first = true;  // no stores of an earlier item are outstanding
  // data chunk at stream position pos of this item (pos >= nc: the next items')
  auto copy_x_at = [&](int pos) {
    const int st = (run + pos) % 3;
    if (pos < nc) {
      copy_x(t, xc, pos * BK, st);
    } else if (pos - nc < nc1) {
      copy_x(t1, xc1, (pos - nc) * BK, st);
    } else if (pos - nc - nc1 < nc2) {
      copy_x(t2, col(t2), (pos - nc - nc1) * BK, st);
    } else {
      copy_x(t, xc, (nc - 1) * BK, 3);
    }
  };
  // table chunk at stream position pos <= nc of this item
  auto copy_a_at = [&](int pos) {
    if (pos < nc)
      copy_a(t, pos * BK, (run + pos) % 2);
    else if (nc1 > 0)
      copy_a(t1, 0, (run + pos) % 2);
    else
      copy_a(t, (nc - 1) * BK, 2);
  };
  copy_a_at(0);
  copy_x_at(0);
  copy_x_at(1);

  for (;;) {
    f4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f4{0, 0, 0, 0};
    int nbi = 0, nbj = 0;
    {
      const int rleft = t.M - (t.row0 + wr);
      nbi = rleft <= 0 ? 0 : (rleft >= 64 ? 4 : (rleft + 15) / 16);
      nbj = t.Ncc - (t.col0 + wc) <= 0 ? 0 : 2;
    }
    const int cc = wc + lr;  // the lane's complex column in the tile
    // (-1)^m of the -m segment: the contraction is linear, so it is applied to the outputs
    const float sg =
        (!RAD && (t.q & 1) && t.col0 + cc >= load_uniform(&t.C->nf) * load_uniform(&t.C->L)) ? -1.0f : 1.0f;

    // Chunk c: the wave waits for its copies of chunk c; one barrier then both
    // publishes every wave's copies and frees the stages of chunk c - 1, into
    // which the copies of table chunk c + 1 and data chunk c + 2 of the stream
    // go (every iteration issues the same copies).  Issue order: ... X(g),
    // A(g), X(g+1), A(g+1), X(g+2) for stream chunks g: at chunk g the two
    // copies of X(g+1) may stay outstanding, and at an item's first chunk also
    // the previous item's stores, which in the inverse every lane issues all
    // 16 of (after A(g) and X(g+1)); the forward's stores are conditional, so
    // its first chunk waits for everything.
    for (int c = 0; c < nc; ++c) {
      wait_vm(c > 0 || first ? 2 : (KIND == K_B_INV ? 18 : 0));
      bar_only();  // chunk c is in LDS; every wave is done with chunk c - 1
      copy_a_at(c + 1);
      copy_x_at(c + 2);
      if (nbj == 0 || nbi == 0) continue;
      f2v r[8];
      if constexpr (RAD) {
        const int R = 128 * lk + cc;
        lds_x4q(lds_u32(sm + 2 * LA + ((run + c) % 3) * kLX) + R * 64 + 16 * (((cc >> 1) & 3) ^ lk), r);
      } else {
        lds_x8(lds_u32(sm + 2 * LA + ((run + c) % 3) * kLX) + 8 * lk * kLRow + cc * 8, r);
      }
      const unsigned ab = lds_u32(sm + ((run + c) % 2) * LA);
      if constexpr (PREC == PREC_F32) {
        // r[u]: (re, im) of column cc at k 8 lk + u, the lane's k in MFMA step u
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i >= nbi) continue;
          const int row = wr + i * 16 + lr;
          const unsigned a0 = ab + row * 128, f = swz32(row);
          f4 av[2];
          lds_a2(a0 + 16 * ((2 * lk) ^ f), a0 + 16 * ((2 * lk + 1) ^ f), av);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float a = av[u >> 2][u & 3];
            acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, r[u][0], acc[i][0], 0, 0, 0);
            acc[i][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, r[u][1], acc[i][1], 0, 0, 0);
          }
        }
        continue;
      }
      bf8 b[2][3];
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        uint32_t h[3][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) split3(r[u][part], h[0][u], h[1][u], h[2][u]);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const u4 v = {pack_hi(h[p][0], h[p][1]), pack_hi(h[p][2], h[p][3]), pack_hi(h[p][4], h[p][5]),
                        pack_hi(h[p][6], h[p][7])};
          b[part][p] = __builtin_bit_cast(bf8, v);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i >= nbi) continue;
        const int row = wr + i * 16 + lr;
        u4 av[3];
        lds_a3(ab + (row * PS + swz(row, lk) * 8) * 2, av);
        bf8 a[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) a[p] = __builtin_bit_cast(bf8, av[p]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // smallest products first, the main product last
          f4& c2 = acc[i][j];
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[j][0], c2, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][1], c2, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][2], c2, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[j][0], c2, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][1], c2, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[j][0], c2, 0, 0, 0);
        }
      }
    }

    // The next item's first wait (vmcnt(18) in the inverse) relies on all 16
    // epilogue stores being issued after the copies of the last chunk: no
    // memory operation may move across this point.
    asm volatile("" ::: "memory");

    // epilogue: each lane holds re (block 0) and im (block 1) of complex column
    // col0 + wc + lr for rows 4 lk + v of each 16-row block: one 8-byte store
    // per value, 16 lanes covering 128 contiguous bytes of an output row.
    constexpr int DUAL = KIND ^ 1;
    float* obase = KIND == K_B_FWD ? reinterpret_cast<float*>(load_uniform(&t.C->g))
                                   : (RAD ? reinterpret_cast<float*>(coeffs)
                                          : reinterpret_cast<float*>(load_uniform(&t.C->F)));
    const int c = t.col0 + cc;
    const bool okc = nbj && c < t.Ncc;
    const XCol<float> oc = x_col<DUAL>(t, min(c, t.Ncc - 1), obase);
    if constexpr (KIND == K_B_INV) {
      // Every lane issues all 16 stores (values outside the group go to a
      // spare array: rare here, the inverse tiles have 128 rows), so that
      // their number is known at the next item's first wait.  The spectrum
      // rows stream out (read once by the iFFT).
      SGL_G f2v* spare = gmem(&g_spare_out[lane]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = t.row0 + wr + i * 16 + 4 * lk + v;
          const bool ok = okc && i < nbi && row < t.M;
          SGL_G f2v* q = ok ? reinterpret_cast<SGL_G f2v*>(oc.p + 2 * x_off<DUAL>(t, oc, min(row, t.M - 1))) : spare;
          __builtin_nontemporal_store(f2v{sg * acc[i][0][v], sg * acc[i][1][v]}, q);
        }
      }
    } else if (okc) {
      // forward: items with few rows (high orders or degrees) leave whole waves
      // idle, whose stores are skipped
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i >= nbi) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = t.row0 + wr + i * 16 + 4 * lk + v;
          if (row < t.M)
            *reinterpret_cast<SGL_G f2v*>(oc.p + 2 * x_off<DUAL>(t, oc, row)) = f2v{sg * acc[i][0][v], sg * acc[i][1][v]};
        }
      }
    }
    if (nc1 == 0) {
      wait_vm(0);  // no copy into this block's LDS outlives the block
      break;
    }
    run = (run + nc) % 6;
    first = false;
    w += G;
    t = t1;
    nc = nc1;
    xc = xc1;
    if (nc2 > 0) {
      t1 = t2;
      nc1 = nc2;
    } else {
      nc1 = 0;
      if (w + G < nwork) {
        t1 = tile(w + G);
        nc1 = nchunks(t1);
      }
    }
    if (nc1 > 0) xc1 = col(t1);
    nc2 = 0;
    if (nc1 == 1 && w + 2 * G < nwork) {
      t2 = tile(w + 2 * G);
      nc2 = nchunks(t2);
    }
  }
}

template <int KIND>
__global__ void __launch_bounds__(LT) __attribute__((amdgpu_waves_per_eu(4))) k_legendre_split(
    const ClassDesc* __restrict__ cls, const int4* __restrict__ work, int nwork) {
  __shared__ __align__(16) unsigned char sm[CopyLds<PREC_SPLIT>::total];
  copy_fed<PREC_SPLIT, KIND>(sm, cls, work, nwork, nullptr);
}

// Forward radial contraction (Eq. DRT) of the split form on the copy-fed
// design: 128 x 128 tiles, writing the coefficients.
__global__ void __launch_bounds__(LT) __attribute__((amdgpu_waves_per_eu(4))) k_radial_split(
    const ClassDesc* __restrict__ cls, const int4* __restrict__ work, int nwork, void* __restrict__ coeffs) {
  __shared__ __align__(16) unsigned char sm[CopyLds<PREC_SPLIT>::total];
  copy_fed<PREC_SPLIT, K_C_FWD>(sm, cls, work, nwork, coeffs);
}

// FP32 Legendre contractions (Eq. DLT and its inverse) on the copy-fed design:
// 128 x 128 tiles, a tile geometry of their launch slots.
template <int KIND>
__global__ void __launch_bounds__(LT) __attribute__((amdgpu_waves_per_eu(4))) k_legendre_f32(
    const ClassDesc* __restrict__ cls, const int4* __restrict__ work, int nwork) {
  __shared__ __align__(16) unsigned char sm[CopyLds<PREC_F32>::total];
  copy_fed<PREC_F32, KIND>(sm, cls, work, nwork, nullptr);
}

// FP32 forward radial contraction (Eq. DRT) on the copy-fed design: the split
// form's radial data path with the FP32 table stage and MFMA steps.
__global__ void __launch_bounds__(LT) __attribute__((amdgpu_waves_per_eu(4))) k_radial_f32(
    const ClassDesc* __restrict__ cls, const int4* __restrict__ work, int nwork, void* __restrict__ coeffs) {
  __shared__ __align__(16) unsigned char sm[CopyLds<PREC_F32>::total];
  copy_fed<PREC_F32, K_C_FWD>(sm, cls, work, nwork, coeffs);
}

inline int grid_for(int nwork, int max_grid) {
  const int g = max_grid > 0 ? max_grid : 8192;
  return nwork < g ? nwork : g;
}

template <int PREC, int TG>
hipError_t launch_gemm(int kind, const ClassDesc* d_cls, const int4* d_work, int nwork, const void* cin, void* cout,
                       dim3 grid, hipStream_t s) {
  DebugArgs dbg{0, 0, 0, nullptr, nullptr, nullptr};
  const dim3 block(Geo<TG>::NT);
  switch (kind) {
    case K_B_FWD:
      hipLaunchKernelGGL((k_gemm<PREC, K_B_FWD, TG>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    case K_B_INV:
      hipLaunchKernelGGL((k_gemm<PREC, K_B_INV, TG>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    case K_C_FWD:
      hipLaunchKernelGGL((k_gemm<PREC, K_C_FWD, TG>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
    default:
      hipLaunchKernelGGL((k_gemm<PREC, K_C_INV, TG>), grid, block, 0, s, d_cls, d_work, nwork, cin, cout, dbg);
      break;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_kind(int kind, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork, const void* cin,
                       void* cout, int max_grid, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  dim3 grid(grid_for(nwork, max_grid));
  if constexpr (PREC == PREC_F32) {
    if (tg == kNumGeo && kind == K_C_FWD) {
      hipLaunchKernelGGL(k_radial_f32, grid, dim3(LT), 0, s, d_cls, d_work, nwork, cout);
      return hipGetLastError();
    }
    if (tg == kNumGeo && kind == K_B_FWD) {
      hipLaunchKernelGGL((k_legendre_f32<K_B_FWD>), grid, dim3(LT), 0, s, d_cls, d_work, nwork);
      return hipGetLastError();
    }
    if (tg == kNumGeo && kind == K_B_INV) {
      hipLaunchKernelGGL((k_legendre_f32<K_B_INV>), grid, dim3(LT), 0, s, d_cls, d_work, nwork);
      return hipGetLastError();
    }
  }
  if constexpr (PREC == PREC_SPLIT) {
    if (kind == K_C_FWD && tg == kNumGeo) {
      hipLaunchKernelGGL(k_radial_split, grid, dim3(LT), 0, s, d_cls, d_work, nwork, cout);
      return hipGetLastError();
    }
    if (kind == K_B_FWD) {
      hipLaunchKernelGGL((k_legendre_split<K_B_FWD>), grid, dim3(LT), 0, s, d_cls, d_work, nwork);
      return hipGetLastError();
    }
    if (kind == K_B_INV) {
      hipLaunchKernelGGL((k_legendre_split<K_B_INV>), grid, dim3(LT), 0, s, d_cls, d_work, nwork);
      return hipGetLastError();
    }
  }
  return tg == 0 ? launch_gemm<PREC, 0>(kind, d_cls, d_work, nwork, cin, cout, grid, s)
                 : launch_gemm<PREC, 1>(kind, d_cls, d_work, nwork, cin, cout, grid, s);
}

hipError_t launch_any(int prec, int kind, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork,
                      const void* cin, void* cout, int max_grid, hipStream_t s) {
  if (prec == PREC_F64) return launch_kind<PREC_F64>(kind, tg, d_cls, d_work, nwork, cin, cout, max_grid, s);
  if (prec == PREC_F32) return launch_kind<PREC_F32>(kind, tg, d_cls, d_work, nwork, cin, cout, max_grid, s);
  return launch_kind<PREC_SPLIT>(kind, tg, d_cls, d_work, nwork, cin, cout, max_grid, s);
}

}  // namespace

int gemm_tile_m(int tg) { return tg == 0 ? Geo<0>::BM : Geo<1>::BM; }
int gemm_tile_n_complex(int tg) { return tg == 0 ? Geo<0>::BNC : Geo<1>::BNC; }
int gemm_legendre_geometries(int prec) { return prec == PREC_SPLIT ? 1 : (prec == PREC_F32 ? kNumGeo + 1 : kNumGeo); }
int gemm_tile_n_complex_legendre(int prec, int tg) {
  return prec == PREC_SPLIT || tg == kNumGeo ? LBNC : gemm_tile_n_complex(tg);
}
int gemm_tile_m_legendre(int prec, int tg) { return prec == PREC_SPLIT || tg == kNumGeo ? BM : gemm_tile_m(tg); }
int gemm_radial_geometries(int prec, bool inverse) { return prec != PREC_F64 && !inverse ? kNumGeo + 1 : kNumGeo; }
int gemm_tile_m_radial(int tg) { return tg == kNumGeo ? BM : gemm_tile_m(tg); }
int gemm_tile_n_complex_radial(int tg) { return tg == kNumGeo ? LBNC : gemm_tile_n_complex(tg); }
int gemm_k_chunk(int prec) {
  return prec == PREC_F64 ? Cfg<PREC_F64>::BK : (prec == PREC_F32 ? Cfg<PREC_F32>::BK : Cfg<PREC_SPLIT>::BK);
}

hipError_t launch_legendre(int prec, bool inverse, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork,
                           int max_grid, hipStream_t s) {
  return launch_any(prec, inverse ? K_B_INV : K_B_FWD, tg, d_cls, d_work, nwork, nullptr, nullptr, max_grid, s);
}

hipError_t launch_radial(int prec, bool inverse, int tg, const ClassDesc* d_cls, const int4* d_work, int nwork,
                         const void* coeffs_in, void* coeffs_out, int max_grid, hipStream_t s) {
  return launch_any(prec, inverse ? K_C_INV : K_C_FWD, tg, d_cls, d_work, nwork, coeffs_in, coeffs_out, max_grid,
                    s);
}

hipError_t launch_debug_gemm(int prec, int M, int N, int K, const double* A, const double* X, double* C,
                             hipStream_t s) {
  DebugArgs dbg{M, N, K, A, X, C};
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles == 0) return hipSuccess;
  dim3 grid(grid_for(tiles, 0)), block(NT);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_gemm<PREC_F64, K_DEBUG, 0>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr, dbg);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL((k_gemm<PREC_F32, K_DEBUG, 0>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr, dbg);
  else
    hipLaunchKernelGGL((k_gemm<PREC_SPLIT, K_DEBUG, 0>), grid, block, 0, s, nullptr, nullptr, 0, nullptr, nullptr,
                       dbg);
  return hipGetLastError();
}

}  // namespace sgl
