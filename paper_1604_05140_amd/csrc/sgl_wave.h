// Register and one-wavefront FFT building blocks shared by the stage (a)
// kernels and the DCT of the seminaive Legendre step: complex helpers, the
// in-register power-of-two DFT, and the 512-point transform with one ring per
// wavefront (exchange layouts and table layout described below).
#pragma once

#include "sgl_internal.h"

namespace sgl {

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

// Streaming store of a complex value (non-temporal: the line is not kept in
// the caches).  Used for the large outputs that the next kernel reads once in
// full (spectrum rows, samples): measured on MI355X at B = 128, batch 4, the
// caches then hold fewer dirty lines of them, and the next launches' reads
// run faster (about 7% per transform pair).
template <typename T2>
__device__ inline void store_stream(SGL_G T2* p, T2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
// Streaming load (non-temporal) of a value read once: the spectrum rows and the
// samples are larger than the caches, and streaming them keeps the smaller
// stage (b)/(c) intermediates cached between their launches.
template <typename T2>
__device__ inline T2 load_stream(const SGL_G T2* p) {
  T2 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}

// twiddle exp(sign 2 pi i q / L) from the forward table exp(-2 pi i q / L)
template <typename T2, bool INV>
__device__ inline T2 twid(const T2* tw, int q) {
  T2 w = tw[q];
  return INV ? conjc(w) : w;
}

// cos(2 pi q / 32), sin(2 pi q / 32), q < 16 (first-quadrant values and symmetry)
#define C32_0 1.0
#define C32_1 0.98078528040323044913
#define C32_2 0.92387953251128675613
#define C32_3 0.83146961230254523708
#define C32_4 0.70710678118654752440
#define C32_5 0.55557023301960222474
#define C32_6 0.38268343236508977173
#define C32_7 0.19509032201612826785
#define C32_8 0.0
__device__ constexpr double kCos32[16] = {C32_0, C32_1, C32_2, C32_3, C32_4, C32_5, C32_6, C32_7,
                                          C32_8, -C32_7, -C32_6, -C32_5, -C32_4, -C32_3, -C32_2, -C32_1};
__device__ constexpr double kSin32[16] = {C32_8, C32_7, C32_6, C32_5, C32_4, C32_3, C32_2, C32_1,
                                          C32_0, C32_1, C32_2, C32_3, C32_4, C32_5, C32_6, C32_7};

template <int R>
__host__ __device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of size R (power of two <= 32): v[k] = sum_n v[n] exp(-+2 pi i n k / R).
// HALF_IN: the inputs n >= R/2 are zero (the first butterfly stage is a copy);
// HALF_OUT: only the outputs k < R/2 are wanted (the others are left stale).
template <typename T2, int R, bool INV, bool HALF_IN = false, bool HALF_OUT = false>
__device__ inline void dft_reg(T2 (&v)[R]) {
  using Tr = decltype(v[0].x);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev<R>(i);
    if (j > i) {
      T2 t = v[i];
      v[i] = v[j];
      v[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const int q = j * (32 / len);
        T2 w;
        w.x = (Tr)kCos32[q];
        w.y = INV ? (Tr)kSin32[q] : -(Tr)kSin32[q];
        const T2 u = v[i + j];
        if (HALF_IN && len == 2) {  // the partner (bit-reversed odd slot) is zero
          v[i + j + 1] = u;
          continue;
        }
        const T2 x = v[i + j + len / 2];
        T2 t = x;
        if (q == 8) {  // times -i (forward) or +i (inverse): a swap, no arithmetic
          t.x = INV ? -x.y : x.y;
          t.y = INV ? x.x : -x.x;
        } else if (q == 4 || q == 12) {  // times (+-1 -+ i) / sqrt 2: add first, one product each
          const Tr c = (Tr)C32_4;
          const Tr sx = INV ? x.x - x.y : x.x + x.y;  // q = 4: forward (1 - i), inverse (1 + i)
          const Tr sy = INV ? x.x + x.y : x.y - x.x;
          if (q == 4) {
            t.x = c * sx;
            t.y = c * sy;
          } else {  // w^12 = w^4 (-+i)
            t.x = INV ? -(c * sy) : c * sy;
            t.y = INV ? c * sx : -(c * sx);
          }
        } else if (q != 0) {
          t = cmul(x, w);
        }
        v[i + j] = cadd(u, t);
        if (!(HALF_OUT && len == R)) v[i + j + len / 2] = csub(u, t);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 512-point transform, one wavefront per ring.
// Lane l holds x[64 a + l] in v[a]; three radix-8 passes:
//   1: DFT_8 over a -> p, times w_512^(l p);
//   2: lane 8p + c (c = l mod 8 in pass 1) holds b = 0..7: DFT_8 over b -> q,
//      times w_64^(c q);
//   3: lane 8q + p holds c = 0..7: DFT_8 over c -> s, giving
//      X[p + 8q + 64s] = X[lane + 64s].
// Input and output share the natural lane order.  The two exchanges go
// through an LDS area private to the wavefront, so they need ordering at
// wavefront scope only.  Table operand `tab`: w_512^(l p) at (p-1) 64 + l
// (p = 1..7) and w_64^(c q) at kTabTw2 + 8 (q-1) + c.
// ---------------------------------------------------------------------------
constexpr int kTabTw2 = 448;

// Orders LDS accesses of one wavefront (its LDS operations complete in issue
// order; this keeps the compiler from moving them across).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange layouts inside a ring area (elements): the first exchange puts
// (p, b, c) at 72 p + 8 b + c, the second (p, q, c) at 72 q + 8 p + (c xor p).
// Every write, and the first read, is a per-lane base plus an immediate
// offset; the second read adds one xor per element.  Both layouts are free
// of bank conflicts for single 8-byte accesses (32 lanes per cycle over 64
// banks) and for the paired ones (ds_read2 / ds_write2: 16 lanes per cycle
// and element, i.e. addresses distinct mod 16 within each quarter wave).
// The largest offset is 567; the area pitch is 568 (ring reads at one bin in
// the staging passes take a few 2- to 8-way conflicts; they are a small part).
template <typename T2>
__host__ __device__ constexpr int area_pitch() { return 568; }

template <typename T2, bool INV>
__device__ inline T2 tw_sign(T2 w) { return INV ? conjc(w) : w; }

// HALF_IN: x[64 a + l] = 0 for a >= 4; HALF_OUT: only X[l + 64 s], s < 4, wanted.
template <typename T2, bool INV, bool HALF_IN = false, bool HALF_OUT = false>
__device__ inline void fft512_wave(T2 (&v)[8], T2* ex, const T2* tab, int l) {
  const int hi = l >> 3, lo = l & 7;
  dft_reg<T2, 8, INV, HALF_IN>(v);
#pragma unroll
  for (int p = 1; p < 8; ++p) v[p] = cmul(v[p], tw_sign<T2, INV>(tab[(p - 1) * 64 + l]));
  wave_lds_sync();
  // first exchange: lane (b, c) = (hi, lo) writes p; lane (p, c) = (hi, lo) reads b
  T2* w1 = ex + l;
#pragma unroll
  for (int p = 0; p < 8; ++p) w1[72 * p] = v[p];
  wave_lds_sync();
  const T2* r1 = ex + 72 * hi + lo;
#pragma unroll
  for (int b = 0; b < 8; ++b) v[b] = r1[8 * b];
  dft_reg<T2, 8, INV>(v);
#pragma unroll
  for (int q = 1; q < 8; ++q) v[q] = cmul(v[q], tw_sign<T2, INV>(tab[kTabTw2 + 8 * (q - 1) + lo]));
  wave_lds_sync();
  // second exchange: lane (p, c) = (hi, lo) writes q; lane (q, p) = (hi, lo) reads c
  T2* w2 = ex + 8 * hi + (lo ^ hi);
#pragma unroll
  for (int q = 0; q < 8; ++q) w2[72 * q] = v[q];
  wave_lds_sync();
  // the xor addresses are formed here (an opaque copy of the lane index keeps
  // the compiler from holding eight of them live across the item loop)
  int lo2 = lo;
  asm volatile("" : "+v"(lo2));
  const T2* r2 = ex + 72 * hi + 8 * lo;
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = r2[c ^ lo2];
  dft_reg<T2, 8, INV, false, HALF_OUT>(v);
  wave_lds_sync();
}

}  // namespace sgl
