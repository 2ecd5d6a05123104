// Host side of libsgl: argument checks, plan construction (FP64 grid and
// tables on the GPU, workspace, work lists) and the stream-ordered forward /
// inverse entry points.  See include/sgl.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sgl_internal.h"

namespace sgl {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Static workspace of sgl_forward_noalloc: the stage intermediates (spectrum F
// and g) of every class of a plan, back to back, in one file-scope device array.
// Each GPU the library runs on holds its own copy, at its own address, until the
// process ends.  In host code the array's name is only a host-side stand-in:
// host code uses the address that hipGetSymbolAddress returns for the device,
// looked up once per device when a plan is created there.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up with that
// device current, once per device).
sgl_status_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the static workspace table");
    return SGL_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SGL_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SGL_OK;
}

// allocations left before the injected failure of the current plan creation (0 = none)
static thread_local long g_fail_countdown = 0;
hipError_t dev_malloc(void** p, size_t bytes) {
  if (g_fail_countdown > 0 && --g_fail_countdown == 0) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

namespace {

struct ClassHost {
  int B = 0;
  std::vector<int> funcs;
  double* grid = nullptr;  // r, log_a, log_sig, sig, theta, btilde, sig_m, sig_e (8 x 2B)
  double* P64 = nullptr;
  double* R64 = nullptr;
  void* A[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t* Aoff[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t Aplane[4] = {0, 0, 0, 0};
  void* tw = nullptr;
  void* F = nullptr;
  void* g = nullptr;
  int64_t* soff = nullptr;
  int64_t* coff = nullptr;
  int* fid = nullptr;
  int rpb = 1;
  std::vector<int> radices;
  int* naive_loff = nullptr;  // see ClassDesc
  int naive_per = 0;          // naive forward items per function
  int M = 0;  // Bluestein length (0 = not used)
  void* twM = nullptr;
  void* chirp = nullptr;
  void* bhf = nullptr;
  void* bhi = nullptr;
  double* D64 = nullptr;  // seminaive: FP64 cosine-domain Legendre table (blocks m of (B-m) x B)
  void* dct = nullptr;    // seminaive: DCT constants (see k_dct_consts)
};

std::vector<int> fft_radices(int L) {
  std::vector<int> out;
  while (L % 4 == 0) { out.push_back(4); L /= 4; }
  for (int p : {2, 3, 5, 7}) {
    while (L % p == 0) { out.push_back(p); L /= p; }
  }
  for (int q = 11; L > 1; q += 2) {
    while (L % q == 0) { out.push_back(q); L /= q; }
  }
  return out;
}

}  // namespace
}  // namespace sgl

using namespace sgl;

struct sgl_plan_s {
  int dtype = 0;
  unsigned flags = 0;
  double rscale = 1.0;  // radial scale s of the basis (1 = the unit SGL basis)
  std::vector<int> Bs;
  std::vector<int64_t> soff, coff;
  int64_t tot_s = 0, tot_c = 0;
  std::vector<ClassHost> classes;
  std::vector<void*> allocs;
  ClassDesc* d_cls = nullptr;
  // descriptors whose F and g point into the device's static workspace
  // (sgl_forward_noalloc); null when the plan's intermediates exceed it
  ClassDesc* d_cls_static = nullptr;
  size_t static_bytes = 0;  // bytes of F and g the static workspace would need
  int device = 0;           // the device the plan was created on
  int4* d_work = nullptr;
  int64_t* d_naive_pre = nullptr;  // [forward prefix][inverse prefix][function-count prefix], ncls + 1 each
  int64_t n_naive_f = 0, n_naive_i = 0;
  // stage (b)/(c) work lists per GEMM tile geometry (index tg): Legendre forward /
  // inverse, radial forward / inverse
  int off_bf[kMaxTileGeo] = {}, n_bf[kMaxTileGeo] = {}, off_bi[kMaxTileGeo] = {}, n_bi[kMaxTileGeo] = {};
  int off_cf[kMaxTileGeo] = {}, n_cf[kMaxTileGeo] = {}, off_ci[kMaxTileGeo] = {}, n_ci[kMaxTileGeo] = {};
  // seminaive Legendre step: DCT work items {class, m + B - 1, column tile, columns per tile}
  int off_dct = 0, n_dct = 0, dct_cols = 16, dct_lds = 0;
  bool seminaive() const { return (flags & SGL_SEMINAIVE) != 0; }
  // stage (a) work by FFT mode (see fft_mode): offsets, counts, LDS bytes
  int off_am[3] = {0, 0, 0}, n_am[3] = {0, 0, 0}, lds_am[3] = {0, 0, 0};
  // persistent grid bound per launch slot (0 = kernel default) and GEMM tile
  // geometry per launch slot (0 = the default tile); both set by the autotuner
  int grid[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  int tile[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // captured launch sequences, keyed by (direction, input, output)
  struct GraphEntry {
    int dir;
    const void* in;
    void* out;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<GraphEntry> graphs;
  uint64_t tick = 0;
  hipStream_t cap = nullptr;
  // timing
  bool timing = false;
  static constexpr int kRing = 64;
  std::vector<hipEvent_t> ev;  // [stage][slot][start/stop]
  int head[6] = {0, 0, 0, 0, 0, 0};
  int pending[6] = {0, 0, 0, 0, 0, 0};
  double ms[6] = {0, 0, 0, 0, 0, 0};
  int cnt[6] = {0, 0, 0, 0, 0, 0};

  ~sgl_plan_s() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (void* q : allocs) (void)hipFree(q);
  }

  sgl_status_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = dev_malloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? SGL_ERR_OOM : SGL_ERR_HIP;
    }
    allocs.push_back(*p);
    return SGL_OK;
  }
  size_t esz() const { return dtype == SGL_F64 ? 16 : 8; }
};

namespace {

#define SGL_TRY(x)                  \
  do {                              \
    sgl_status_t st_ = (x);         \
    if (st_ != SGL_OK) return st_;  \
  } while (0)

sgl_status_t build_class_data(sgl_plan_s* p, ClassHost& c, hipStream_t s);

// Build one class.  `share` (may be null) is an earlier class of the same
// bandlimit whose grid, tables and FFT constants are reused.
sgl_status_t build_class(sgl_plan_s* p, ClassHost& c, const ClassHost* share, hipStream_t s) {
  const int B = c.B, L = 2 * B;
  const int64_t ts = table_size(B);
  if (share) {
    c.grid = share->grid;
    c.P64 = share->P64;
    c.R64 = share->R64;
    for (int k = 0; k < 4; ++k) {
      c.A[k] = share->A[k];
      c.Aoff[k] = share->Aoff[k];
      c.Aplane[k] = share->Aplane[k];
    }
    c.tw = share->tw;
    c.M = share->M;
    c.twM = share->twM;
    c.chirp = share->chirp;
    c.bhf = share->bhf;
    c.bhi = share->bhi;
    c.radices = share->radices;
    c.naive_loff = share->naive_loff;
    c.naive_per = share->naive_per;
    c.D64 = share->D64;
    c.dct = share->dct;
    return build_class_data(p, c, s);
  }
  SGL_TRY(p->alloc((void**)&c.grid, 8 * (size_t)L * sizeof(double)));
  GridBuild gb{B,         c.grid,         c.grid + L,     c.grid + 2 * L, c.grid + 3 * L,
               c.grid + 4 * L, c.grid + 5 * L, c.grid + 6 * L, c.grid + 7 * L};
  SGL_TRY(build_grid(gb, s));
  SGL_TRY(p->alloc((void**)&c.P64, ts * sizeof(double)));
  SGL_TRY(p->alloc((void**)&c.R64, ts * sizeof(double)));
  SGL_HIP_TRY(build_tables(B, gb, c.P64, c.R64, s));
  const bool semi = p->seminaive();
  if (semi) {
    // seminaive step: cosine-domain Legendre table and the DCT constants
    SGL_TRY(p->alloc((void**)&c.D64, ts / 2 * sizeof(double)));
    SGL_HIP_TRY(build_cos_legendre(B, c.P64, c.D64, s));
    SGL_TRY(p->alloc(&c.dct, (size_t)dct_const_count(B) * sizeof(double2)));  // FP64 for every precision
    SGL_HIP_TRY(build_dct_consts(B, c.dct, false, s));
  }
  // packed GEMM operands, one per contraction direction
  const int prec = p->dtype == SGL_F64 ? PREC_F64 : (p->dtype == SGL_F32 ? PREC_F32 : PREC_SPLIT);
  const size_t el = prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2);
  const int KC = gemm_k_chunk(prec);
  for (int kind = 0; kind < 4; ++kind) {
    const bool fwd = kind == 0 || kind == 2;
    // grid-side length: 2B, or B for the seminaive cosine-domain Legendre operands
    const int W = (semi && kind < 2) ? B : L;
    std::vector<int64_t> offs(B);
    int64_t tot = 0;
    for (int q = 0; q < B; ++q) {
      const int rows = fwd ? B - q : W;
      const int K = fwd ? W : B - q;
      offs[q] = tot;
      tot += (int64_t)rows * ((K + KC - 1) / KC * KC);
    }
    SGL_TRY(p->alloc((void**)&c.Aoff[kind], B * sizeof(int64_t)));
    SGL_HIP_TRY(hipMemcpy(c.Aoff[kind], offs.data(), B * sizeof(int64_t), hipMemcpyHostToDevice));
    SGL_TRY(p->alloc(&c.A[kind], (size_t)tot * el * (prec == PREC_SPLIT ? 3 : 1)));
    c.Aplane[kind] = tot;
    // the radially scaled basis H^s = s^(-3/2) H(x/s) multiplies forward coefficients
    // by s^(3/2) and divides inverse inputs by it: folded into the radial operands
    const double sc = kind == 2 ? std::pow(p->rscale, 1.5) : (kind == 3 ? std::pow(p->rscale, -1.5) : 1.0);
    const double* src = kind < 2 ? (semi ? c.D64 : c.P64) : c.R64;
    SGL_HIP_TRY(pack_table(B, kind, prec, src, c.Aoff[kind], c.A[kind], tot, sc, s, W));
  }
  const bool f32 = p->dtype != SGL_F64;
  const size_t ces = f32 ? sizeof(float2) : sizeof(double2);
  SGL_TRY(p->alloc(&c.tw, (size_t)L * ces));
  SGL_HIP_TRY(build_twiddles(L, c.tw, f32, s));
  c.M = fft_bluestein_m(L);
  if (c.M) {
    SGL_TRY(p->alloc(&c.twM, (size_t)c.M * ces));
    SGL_HIP_TRY(build_twiddles(c.M, c.twM, f32, s));
    SGL_TRY(p->alloc(&c.chirp, (size_t)L * ces));
    SGL_TRY(p->alloc(&c.bhf, (size_t)c.M * ces));
    SGL_TRY(p->alloc(&c.bhi, (size_t)c.M * ces));
    SGL_HIP_TRY(build_bluestein(L, c.M, c.chirp, c.bhf, c.bhi, f32, s));
  }
  {
    const int G = naive_group();
    std::vector<int> lo(B + 1, 0);
    for (int l = 0; l < B; ++l) lo[l + 1] = lo[l] + (2 * l + 1) * ((B - l + G - 1) / G);
    c.naive_per = lo[B];
    SGL_TRY(p->alloc((void**)&c.naive_loff, (B + 1) * sizeof(int)));
    SGL_HIP_TRY(hipMemcpy(c.naive_loff, lo.data(), (B + 1) * sizeof(int), hipMemcpyHostToDevice));
  }
  c.radices = fft_radices(L);
  if ((int)c.radices.size() > kMaxRadices) {
    set_error("FFT length has too many factors");
    return SGL_ERR_UNSUPPORTED;
  }
  return build_class_data(p, c, s);
}

// Per-class workspace, function offsets and FFT blocking (not shared).
sgl_status_t build_class_data(sgl_plan_s* p, ClassHost& c, hipStream_t /*s*/) {
  const int B = c.B, L = 2 * B, nf = (int)c.funcs.size();
  const size_t es = p->esz();
  SGL_TRY(p->alloc(&c.F, (size_t)(2 * B - 1) * L * nf * L * es));
  SGL_TRY(p->alloc(&c.g, (size_t)B * B * nf * L * es));
  std::vector<int64_t> so(nf), co(nf);
  for (int q = 0; q < nf; ++q) {
    so[q] = p->soff[c.funcs[q]];
    co[q] = p->coff[c.funcs[q]];
  }
  SGL_TRY(p->alloc((void**)&c.soff, nf * sizeof(int64_t)));
  SGL_TRY(p->alloc((void**)&c.coff, nf * sizeof(int64_t)));
  SGL_HIP_TRY(hipMemcpy(c.soff, so.data(), nf * sizeof(int64_t), hipMemcpyHostToDevice));
  SGL_TRY(p->alloc((void**)&c.fid, nf * sizeof(int)));
  SGL_HIP_TRY(hipMemcpy(c.fid, c.funcs.data(), nf * sizeof(int), hipMemcpyHostToDevice));
  SGL_HIP_TRY(hipMemcpy(c.coff, co.data(), nf * sizeof(int64_t), hipMemcpyHostToDevice));
  if (fft_mode(L) == 1) {
    c.rpb = fft_threads(1, p->dtype == SGL_F64) / 64;  // one wavefront per ring
  } else if (fft_pow2_path(L)) {
    c.rpb = fft_pow2_rpb(L, fft_threads(fft_mode(L), p->dtype == SGL_F64));
  } else if (c.M) {
    c.rpb = fft_pow2_rpb(c.M, fft_threads(fft_mode(L), p->dtype == SGL_F64));
  } else {
    // rings per generic-FFT block: 64 KB of LDS for the ping-pong buffers
    const int cap = (int)(65536 / (2 * (size_t)L * es));
    c.rpb = std::max(1, std::min(64, std::min(cap, nf * L)));
  }
  return SGL_OK;
}

sgl_status_t build_work(sgl_plan_s* p, hipStream_t /*s*/) {
  std::vector<int4> wam[3], wdct;
  if (p->seminaive()) {
    // columns per DCT block: 16 unless the 4B-point FP64 column buffers of
    // B = 256 need the room of 8
    p->dct_cols = 16;
    for (auto& c : p->classes)
      if (dct_lds_bytes(p->dtype == SGL_F64 ? PREC_F64 : PREC_F32, c.B, 16) > 160 * 1024) p->dct_cols = 8;
  }
  struct Item { int cost; int4 w; };
  const int precb = p->dtype == SGL_F64 ? PREC_F64 : (p->dtype == SGL_F32 ? PREC_F32 : PREC_SPLIT);
  std::vector<Item> bf[kMaxTileGeo], bi[kMaxTileGeo], cf[kMaxTileGeo], ci[kMaxTileGeo];
  int ldsm[3] = {0, 0, 0};
  for (int ci_ = 0; ci_ < (int)p->classes.size(); ++ci_) {
    const ClassHost& c = p->classes[ci_];
    const int B = c.B, L = 2 * B, nf = (int)c.funcs.size();
    const int ncol = nf * L;
    const int ncb = (ncol + c.rpb - 1) / c.rpb;
    const int mode = fft_mode(L);
    for (int j = 0; j < L; ++j)
      for (int cb = 0; cb < ncb; ++cb) wam[mode].push_back(make_int4(ci_, j, cb, c.rpb));
    ldsm[mode] = std::max(ldsm[mode], (int)fft_lds_bytes_for(p->dtype == SGL_F64 ? PREC_F64 : PREC_F32, c.rpb, L));
    const int kb = p->seminaive() ? B : L;  // polar-side contraction length
    for (int tg = 0; tg < kMaxTileGeo; ++tg) {
      // stage (b): the split-form Legendre kernel has one tile (geometry 0)
      if (tg < gemm_legendre_geometries(precb)) {
        const int BMb = gemm_tile_m_legendre(precb, tg), BNb = gemm_tile_n_complex_legendre(precb, tg);
        for (int m = 0; m < B; ++m) {
          const int rows = B - m;
          const int ncc = (m ? 2 : 1) * nf * L;
          const int nt = (ncc + BNb - 1) / BNb;
          for (int mt = 0; mt < (rows + BMb - 1) / BMb; ++mt)
            for (int t = 0; t < nt; ++t) bf[tg].push_back({kb, make_int4(ci_, m, mt, t)});
          for (int mt = 0; mt < (kb + BMb - 1) / BMb; ++mt)
            for (int t = 0; t < nt; ++t) bi[tg].push_back({rows, make_int4(ci_, m, mt, t)});
        }
      }
      const int BM = gemm_tile_m_radial(tg), BNC = gemm_tile_n_complex_radial(tg);
      const bool fwd_c = tg < gemm_radial_geometries(precb, false), inv_c = tg < gemm_radial_geometries(precb, true);
      for (int l = 0; l < B; ++l) {
        const int rows = B - l;
        const int ncc = (2 * l + 1) * nf;
        const int nt = (ncc + BNC - 1) / BNC;
        if (fwd_c)
          for (int mt = 0; mt < (rows + BM - 1) / BM; ++mt)
            for (int t = 0; t < nt; ++t) cf[tg].push_back({L, make_int4(ci_, l, mt, t)});
        if (inv_c)
          for (int mt = 0; mt < (L + BM - 1) / BM; ++mt)
            for (int t = 0; t < nt; ++t) ci[tg].push_back({rows, make_int4(ci_, l, mt, t)});
      }
    }
    if (p->seminaive()) {
      const int nct = (ncol + p->dct_cols - 1) / p->dct_cols;
      for (int mi = 0; mi < 2 * B - 1; ++mi)
        for (int t = 0; t < nct; ++t) wdct.push_back(make_int4(ci_, mi, t, p->dct_cols));
      p->dct_lds = std::max(p->dct_lds, (int)dct_lds_bytes(p->dtype == SGL_F64 ? PREC_F64 : PREC_F32, B, p->dct_cols));
    }
  }
  // XCD-aware order.  Blocks of a launch go round-robin to the chip's 8 XCDs
  // (each with its own L2), and a persistent grid that is a multiple of 8
  // keeps list position w on XCD w % 8.  All tiles of one (class, order) read
  // the same table block, and the row tiles of one column tile the same data
  // operand, so each (class, order) group goes to one XCD (groups assigned
  // largest first to the least-loaded XCD) with its tiles adjacent in that
  // XCD's queue; the queues are interleaved, larger groups first.
  auto order = [](std::vector<Item>& v, std::vector<int4>& out) {
    constexpr int kXcd = 8;
    std::map<std::pair<int, int>, std::vector<Item>> groups;
    for (auto& it : v) groups[{it.w.x, it.w.y}].push_back(it);
    struct G { int64_t cost; std::vector<Item>* items; };
    std::vector<G> gs;
    for (auto& kv : groups) {
      int64_t c = 0;
      for (auto& it : kv.second) c += it.cost;
      std::stable_sort(kv.second.begin(), kv.second.end(),
                       [](const Item& a, const Item& b) { return a.w.w != b.w.w ? a.w.w < b.w.w : a.w.z < b.w.z; });
      gs.push_back({c, &kv.second});
    }
    std::stable_sort(gs.begin(), gs.end(), [](const G& a, const G& b) { return a.cost > b.cost; });
    std::vector<std::vector<int4>> q(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    for (auto& g : gs) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[x] += g.cost;
      for (auto& it : *g.items) q[x].push_back(it.w);
    }
    out.clear();
    std::vector<size_t> pos(kXcd, 0);
    for (size_t left = v.size(); left > 0;) {
      for (int x = 0; x < kXcd; ++x) {
        int src = x;
        if (pos[src] == q[src].size()) {  // this queue ran dry: take from the longest
          src = 0;
          for (int y = 1; y < kXcd; ++y)
            if (q[y].size() - pos[y] > q[src].size() - pos[src]) src = y;
          if (pos[src] == q[src].size()) break;
        }
        out.push_back(q[src][pos[src]++]);
        --left;
      }
    }
  };
  std::vector<int4> all;
  for (int md = 0; md < 3; ++md) {
    p->off_am[md] = (int)all.size();
    p->n_am[md] = (int)wam[md].size();
    p->lds_am[md] = ldsm[md];
    all.insert(all.end(), wam[md].begin(), wam[md].end());
  }
  auto append = [&](std::vector<Item>& v, int& off, int& n) {
    std::vector<int4> w;
    order(v, w);
    off = (int)all.size();
    n = (int)w.size();
    all.insert(all.end(), w.begin(), w.end());
  };
  for (int tg = 0; tg < kMaxTileGeo; ++tg) {
    append(bf[tg], p->off_bf[tg], p->n_bf[tg]);
    append(bi[tg], p->off_bi[tg], p->n_bi[tg]);
    append(cf[tg], p->off_cf[tg], p->n_cf[tg]);
    append(ci[tg], p->off_ci[tg], p->n_ci[tg]);
  }
  p->off_dct = (int)all.size(); p->n_dct = (int)wdct.size(); all.insert(all.end(), wdct.begin(), wdct.end());
  SGL_TRY(p->alloc((void**)&p->d_work, all.size() * sizeof(int4)));
  SGL_HIP_TRY(hipMemcpy(p->d_work, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice));

  return SGL_OK;
}

sgl_status_t make_plan(sgl_plan_s* p, hipStream_t s) {
  std::map<int, std::vector<int>> byB;
  for (int f = 0; f < (int)p->Bs.size(); ++f) byB[p->Bs[f]].push_back(f);
  // largest bandlimit first; a class holds at most class_capacity(B) functions
  // so that its workspaces stay below 2^31 complex values (the stage kernels
  // index them with 32-bit offsets)
  for (auto it = byB.rbegin(); it != byB.rend(); ++it) {
    const int cap = class_capacity(it->first);
    for (size_t f0 = 0; f0 < it->second.size(); f0 += cap) {
      ClassHost c;
      c.B = it->first;
      const size_t f1 = std::min(it->second.size(), f0 + (size_t)cap);
      c.funcs.assign(it->second.begin() + f0, it->second.begin() + f1);
      p->classes.push_back(c);
    }
  }
  for (size_t q = 0; q < p->classes.size(); ++q) {
    const ClassHost* share = (q > 0 && p->classes[q - 1].B == p->classes[q].B) ? &p->classes[q - 1] : nullptr;
    SGL_TRY(build_class(p, p->classes[q], share, s));
  }
  std::vector<ClassDesc> descs;
  for (auto& c : p->classes) {
    ClassDesc d;
    std::memset(&d, 0, sizeof(d));
    d.B = c.B;
    d.nf = (int)c.funcs.size();
    d.L = 2 * c.B;
    d.nrad = (int)c.radices.size();
    for (int q = 0; q < d.nrad; ++q) d.rad[q] = c.radices[q];
    d.soff = c.soff;
    d.coff = c.coff;
    {
      const int64_t om = (int64_t)c.B * (c.B + 1) * (2 * c.B + 1) / 6;
      bool affine = true;
      for (size_t q = 0; q < c.funcs.size(); ++q) affine = affine && p->coff[c.funcs[q]] == p->coff[c.funcs[0]] + (int64_t)q * om;
      d.cbase = p->coff[c.funcs[0]];
      d.cstep = affine ? om : 0;
    }
    for (int k = 0; k < 4; ++k) {
      d.A[k] = c.A[k];
      d.Aoff[k] = c.Aoff[k];
      d.Aplane[k] = c.Aplane[k];
    }
    d.btilde = c.grid + 5 * d.L;
    d.sigma = c.grid + 3 * d.L;
    d.tw = c.tw;
    d.M = c.M;
    d.twM = c.twM;
    d.chirp = c.chirp;
    d.bhf = c.bhf;
    d.bhi = c.bhi;
    d.F = c.F;
    d.g = c.g;
    d.P64 = c.P64;
    d.R64 = c.R64;
    d.naive_loff = c.naive_loff;
    d.rscale = p->rscale;
    d.fid = c.fid;
    d.rs_fwd = std::pow(p->rscale, 1.5);
    d.rs_inv = std::pow(p->rscale, -1.5);
    d.kb = p->seminaive() ? c.B : 2 * c.B;
    d.dct = c.dct;
    descs.push_back(d);
  }
  {
    // per-class prefix of naive work items (forward: (function, l, m, n group); inverse: (function, ring))
    std::vector<int64_t> pf(1, 0), pi(1, 0), pn(1, 0);
    for (auto& c : p->classes) {
      const int64_t nf = (int64_t)c.funcs.size(), L = 2 * c.B;
      pf.push_back(pf.back() + nf * c.naive_per);
      pi.push_back(pi.back() + nf * L * L);
      pn.push_back(pn.back() + nf);
    }
    p->n_naive_f = pf.back();
    p->n_naive_i = pi.back();
    // [forward prefix][inverse prefix][function-count prefix], ncls + 1 each
    std::vector<int64_t> all(pf);
    all.insert(all.end(), pi.begin(), pi.end());
    all.insert(all.end(), pn.begin(), pn.end());
    SGL_TRY(p->alloc((void**)&p->d_naive_pre, all.size() * sizeof(int64_t)));
    SGL_HIP_TRY(hipMemcpy(p->d_naive_pre, all.data(), all.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  SGL_TRY(p->alloc((void**)&p->d_cls, descs.size() * sizeof(ClassDesc)));
  SGL_HIP_TRY(hipMemcpy(p->d_cls, descs.data(), descs.size() * sizeof(ClassDesc), hipMemcpyHostToDevice));
  {
    // F and g of each class in the static workspace, 256-byte aligned
    SGL_HIP_TRY(hipGetDevice(&p->device));
    std::vector<size_t> offs;
    size_t tot = 0;
    for (auto& c : p->classes) {
      const size_t B = c.B, L = 2 * B, nf = c.funcs.size();
      offs.push_back(tot);
      tot += ((2 * B - 1) * L * nf * L * p->esz() + 255) / 256 * 256;
      offs.push_back(tot);
      tot += (B * B * nf * L * p->esz() + 255) / 256 * 256;
    }
    p->static_bytes = tot;
    if (tot <= kScratchBytes) {
      void* base = nullptr;
      SGL_TRY(scratch_address(p->device, &base));
      for (size_t q = 0; q < descs.size(); ++q) {
        descs[q].F = static_cast<unsigned char*>(base) + offs[2 * q];
        descs[q].g = static_cast<unsigned char*>(base) + offs[2 * q + 1];
      }
      SGL_TRY(p->alloc((void**)&p->d_cls_static, descs.size() * sizeof(ClassDesc)));
      SGL_HIP_TRY(
          hipMemcpy(p->d_cls_static, descs.data(), descs.size() * sizeof(ClassDesc), hipMemcpyHostToDevice));
    }
  }
  SGL_TRY(build_work(p, s));
  prepare_fft_kernels(p->lds_am);
  if (p->seminaive()) prepare_dct_kernels(p->dct_lds);
  if (p->flags & SGL_GRAPHS) SGL_HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  SGL_HIP_TRY(hipStreamSynchronize(s));
  return SGL_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

int prec_of(int dtype) { return dtype == SGL_F64 ? PREC_F64 : (dtype == SGL_F32 ? PREC_F32 : PREC_SPLIT); }

void time_begin(sgl_plan_s* p, int stage, hipStream_t s) {
  if (!p->timing) return;
  if (p->pending[stage] == sgl_plan_s::kRing) {
    // fold the oldest pair
    int slot = (p->head[stage] - p->pending[stage] + sgl_plan_s::kRing) % sgl_plan_s::kRing;
    hipEvent_t a = p->ev[(stage * sgl_plan_s::kRing + slot) * 2], b = p->ev[(stage * sgl_plan_s::kRing + slot) * 2 + 1];
    float ms = 0;
    if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess) {
      p->ms[stage] += ms;
      p->cnt[stage] += 1;
    }
    p->pending[stage] -= 1;
  }
  (void)hipEventRecord(p->ev[(stage * sgl_plan_s::kRing + p->head[stage]) * 2], s);
}
void time_end(sgl_plan_s* p, int stage, hipStream_t s) {
  if (!p->timing) return;
  (void)hipEventRecord(p->ev[(stage * sgl_plan_s::kRing + p->head[stage]) * 2 + 1], s);
  p->head[stage] = (p->head[stage] + 1) % sgl_plan_s::kRing;
  p->pending[stage] += 1;
}

sgl_status_t check_call(sgl_plan_t plan, const void* in, size_t nin, const void* out, size_t nout) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (!in || !out) { set_error("null data pointer"); return SGL_ERR_INVALID_ARG; }
  if (overlap(in, nin, out, nout)) { set_error("input and output overlap"); return SGL_ERR_INVALID_ARG; }
  return SGL_OK;
}

enum Slot {
  S_FFT_F0 = 0, S_FFT_F1, S_FFT_F2, S_LEG_F, S_RAD_F,
  S_RAD_I, S_LEG_I, S_FFT_I0, S_FFT_I1, S_FFT_I2, NSLOT
};
// launch order and timing stage of each direction
const int kSeq[2][5] = {{S_FFT_F0, S_FFT_F1, S_FFT_F2, S_LEG_F, S_RAD_F},
                        {S_RAD_I, S_LEG_I, S_FFT_I0, S_FFT_I1, S_FFT_I2}};
const int kStage[2][5] = {{0, 0, 0, 1, 2}, {3, 4, 5, 5, 5}};

int slot_work(const sgl_plan_s* p, int slot) {
  switch (slot) {
    case S_FFT_F0: case S_FFT_I0: return p->n_am[0];
    case S_FFT_F1: case S_FFT_I1: return p->n_am[1];
    case S_FFT_F2: case S_FFT_I2: return p->n_am[2];
    case S_LEG_F: return p->n_bf[p->tile[slot]];
    case S_LEG_I: return p->n_bi[p->tile[slot]];
    case S_RAD_F: return p->n_cf[p->tile[slot]];
    default: return p->n_ci[p->tile[slot]];
  }
}

// One stage launch.  in/out: the caller's buffers of this direction;
// cls_override: class descriptors to use instead of the plan's (null: the plan's).
hipError_t launch_slot(sgl_plan_s* p, int slot, const void* in, void* out, hipStream_t s,
                       const ClassDesc* cls_override = nullptr) {
  const int prec = prec_of(p->dtype);
  const bool raw = (p->flags & SGL_SAMPLES_RAW) != 0;
  const int g = p->grid[slot];
  const int tg = p->tile[slot];
  const ClassDesc* cls = cls_override ? cls_override : p->d_cls;
  switch (slot) {
    case S_FFT_F0: case S_FFT_F1: case S_FFT_F2: {
      const int md = slot - S_FFT_F0;
      return launch_fft_forward(prec, raw, cls, p->d_work + p->off_am[md], p->n_am[md], p->lds_am[md], md, in, g,
                                s);
    }
    case S_FFT_I0: case S_FFT_I1: case S_FFT_I2: {
      const int md = slot - S_FFT_I0;
      return launch_fft_inverse(prec, raw, cls, p->d_work + p->off_am[md], p->n_am[md], p->lds_am[md], md, out, g,
                                s);
    }
    case S_LEG_F: {
      if (p->seminaive()) {
        // seminaive step: DCT over the polar index, then the cosine-domain contraction
        hipError_t e = launch_dct(prec == PREC_F64 ? PREC_F64 : PREC_F32, false, cls, p->d_work + p->off_dct,
                                  p->n_dct, p->dct_lds, p->dct_cols, s);
        if (e != hipSuccess) return e;
      }
      return launch_legendre(prec, false, tg, cls, p->d_work + p->off_bf[tg], p->n_bf[tg], g, s);
    }
    case S_RAD_F:
      return launch_radial(prec, false, tg, cls, p->d_work + p->off_cf[tg], p->n_cf[tg], nullptr, out, g, s);
    case S_RAD_I:
      return launch_radial(prec, true, tg, cls, p->d_work + p->off_ci[tg], p->n_ci[tg], in, nullptr, g, s);
    default: {
      hipError_t e = launch_legendre(prec, true, tg, cls, p->d_work + p->off_bi[tg], p->n_bi[tg], g, s);
      if (e != hipSuccess || !p->seminaive()) return e;
      return launch_dct(prec == PREC_F64 ? PREC_F64 : PREC_F32, true, cls, p->d_work + p->off_dct, p->n_dct,
                        p->dct_lds, p->dct_cols, s);
    }
  }
}

// Stage launches of one direction, one per slot with work.  With timing on,
// events bracket each run of consecutive launches of one stage.
hipError_t launch_sequence(sgl_plan_s* p, int dir, const void* in, void* out, hipStream_t s, bool timed) {
  int open_stage = -1;
  for (int q = 0; q < 5; ++q) {
    const int slot = kSeq[dir][q];
    if (slot_work(p, slot) == 0) continue;
    const int st = kStage[dir][q];
    if (timed && st != open_stage) {
      if (open_stage >= 0) time_end(p, open_stage, s);
      time_begin(p, st, s);
      open_stage = st;
    }
    hipError_t e = launch_slot(p, slot, in, out, s);
    if (e != hipSuccess) return e;
  }
  if (timed && open_stage >= 0) time_end(p, open_stage, s);
  return hipSuccess;
}

sgl_status_t run_direction(sgl_plan_s* p, int dir, const void* in, void* out, hipStream_t s) {
  if (p->timing || !(p->flags & SGL_GRAPHS)) {
    SGL_HIP_TRY(launch_sequence(p, dir, in, out, s, p->timing));
    return SGL_OK;
  }
  for (auto& g : p->graphs) {
    if (g.dir == dir && g.in == in && g.out == out) {
      g.used = ++p->tick;
      SGL_HIP_TRY(hipGraphLaunch(g.exec, s));
      return SGL_OK;
    }
  }
  // first call with this buffer pair: capture the launch sequence on the plan's
  // own stream and keep the instantiated graph
  SGL_HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
  hipError_t le = launch_sequence(p, dir, in, out, p->cap, false);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(p->cap, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error(std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
    return SGL_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    return SGL_ERR_HIP;
  }
  if (p->graphs.size() >= 8) {
    auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                [](const sgl_plan_s::GraphEntry& a, const sgl_plan_s::GraphEntry& b) {
                                  return a.used < b.used;
                                });
    (void)hipGraphExecDestroy(lru->exec);
    p->graphs.erase(lru);
  }
  p->graphs.push_back({dir, in, out, exec, ++p->tick});
  SGL_HIP_TRY(hipGraphLaunch(exec, s));
  return SGL_OK;
}

// Tile geometries a launch slot can run with: the stage (b)/(c) slots of the
// register-staged GEMM have two (see gemm_tile_m), the forward radial slot of
// the split and FP32 forms and the FP32 Legendre slots a third (a copy-fed
// kernel), the FFT slots and the split-form Legendre kernel one.
int slot_geometries(const sgl_plan_s* p, int slot) {
  if (slot == S_RAD_F || slot == S_RAD_I) return gemm_radial_geometries(prec_of(p->dtype), slot == S_RAD_I);
  if (slot == S_LEG_F || slot == S_LEG_I) return gemm_legendre_geometries(prec_of(p->dtype));
  return 1;
}

// Plan-time autotuner: for every launch slot, time each tile geometry the slot
// has with the persistent grid bounds {1, 2, 4, 8, 16} x CUs and "one block per
// work item" on scratch buffers (three interleaved rounds of a warm-up launch
// and three timed launches, each candidate keeping its best round, so that
// clock drift during tuning does not favour the candidates timed first), then
// choose between each slot's two fastest inside whole transform pairs.
sgl_status_t autotune(sgl_plan_s* p, hipStream_t s) {
  int dev = 0, ncu = 256;
  SGL_HIP_TRY(hipGetDevice(&dev));
  SGL_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  void* tin = nullptr;
  void* tout = nullptr;
  SGL_TRY(p->alloc(&tin, (size_t)p->tot_s * p->esz()));
  SGL_TRY(p->alloc(&tout, (size_t)p->tot_c * p->esz()));
  SGL_HIP_TRY(hipMemsetAsync(tin, 0, (size_t)p->tot_s * p->esz(), s));
  SGL_HIP_TRY(hipMemsetAsync(tout, 0, (size_t)p->tot_c * p->esz(), s));
  hipEvent_t e0, e1;
  SGL_HIP_TRY(hipEventCreate(&e0));
  SGL_HIP_TRY(hipEventCreate(&e1));
  sgl_status_t st = SGL_OK;
  struct Cand { int tg, grid; };
  std::vector<std::vector<Cand>> shortlist(NSLOT);  // the two fastest candidates of each slot
  for (int slot = 0; slot < NSLOT && st == SGL_OK; ++slot) {
    const int n = slot_work(p, slot);
    if (n == 0) continue;
    const bool inv = slot >= S_RAD_I;  // inverse slots read coefficients, write samples
    const void* in = inv ? tout : tin;
    void* out = inv ? tin : tout;
    std::vector<Cand> cand;
    for (int tg = 0; tg < slot_geometries(p, slot); ++tg) {
      p->tile[slot] = tg;
      const int ntg = slot_work(p, slot);
      for (int mult : {1, 2, 4, 8, 16})
        if (mult * ncu < ntg) cand.push_back({tg, mult * ncu});
      cand.push_back({tg, ntg});
    }
    std::vector<float> tbest(cand.size(), 1e30f);
    for (int round = 0; round < 3 && st == SGL_OK; ++round) {
      for (size_t ci = 0; ci < cand.size(); ++ci) {
        p->tile[slot] = cand[ci].tg;
        p->grid[slot] = cand[ci].grid;
        hipError_t e = launch_slot(p, slot, in, out, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_slot(p, slot, in, out, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          set_error(std::string("autotune: ") + hipGetErrorString(e));
          st = SGL_ERR_HIP;
          break;
        }
        tbest[ci] = std::min(tbest[ci], ms);
      }
    }
    std::vector<size_t> order(cand.size());
    for (size_t ci = 0; ci < cand.size(); ++ci) order[ci] = ci;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return tbest[a] < tbest[b]; });
    for (size_t k = 0; k < order.size() && k < 2; ++k) shortlist[slot].push_back(cand[order[k]]);
    p->tile[slot] = cand[order[0]].tg;
    p->grid[slot] = cand[order[0]].grid;
  }
  // In context: a launch timed alone does not show what its grid and tile do
  // to the neighbouring stages (cache contents, the tail of one launch against
  // the start of the next), so the two fastest candidates of each slot are
  // timed again inside whole forward + inverse pairs (one warm-up pair, two
  // timed, two interleaved rounds), one slot at a time, and the faster kept.
  for (int slot = 0; slot < NSLOT && st == SGL_OK; ++slot) {
    if (shortlist[slot].size() < 2) continue;
    float tb[2] = {1e30f, 1e30f};
    for (int round = 0; round < 2 && st == SGL_OK; ++round)
      for (int c = 0; c < 2; ++c) {
        p->tile[slot] = shortlist[slot][c].tg;
        p->grid[slot] = shortlist[slot][c].grid;
        hipError_t e = hipSuccess;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
          if (r == 1) e = hipEventRecord(e0, s);
          if (e == hipSuccess) e = launch_sequence(p, 0, tin, tout, s, false);
          if (e == hipSuccess) e = launch_sequence(p, 1, tout, tin, s, false);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          set_error(std::string("autotune: ") + hipGetErrorString(e));
          st = SGL_ERR_HIP;
          break;
        }
        tb[c] = std::min(tb[c], ms);
      }
    const int c = tb[1] < tb[0] ? 1 : 0;
    p->tile[slot] = shortlist[slot][c].tg;
    p->grid[slot] = shortlist[slot][c].grid;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // scratch buffers are released now (plan time)
  for (void* q : {tin, tout}) {
    auto it = std::find(p->allocs.begin(), p->allocs.end(), q);
    if (it != p->allocs.end()) p->allocs.erase(it);
    (void)hipFree(q);
  }
  return st;
}

}  // namespace

extern "C" {

const char* sgl_status_string(sgl_status_t st) {
  switch (st) {
    case SGL_OK: return "SGL_OK";
    case SGL_ERR_INVALID_ARG: return "SGL_ERR_INVALID_ARG";
    case SGL_ERR_UNSUPPORTED: return "SGL_ERR_UNSUPPORTED";
    case SGL_ERR_HIP: return "SGL_ERR_HIP";
    case SGL_ERR_OOM: return "SGL_ERR_OOM";
    case SGL_ERR_NUMERIC: return "SGL_ERR_NUMERIC";
  }
  return "SGL_ERR_UNKNOWN";
}

const char* sgl_last_error(void) { return g_last_error.c_str(); }

int64_t sgl_num_samples(int B) { return (B < 1 || B > SGL_MAX_B) ? -1 : num_samples(B); }
int64_t sgl_num_coeffs(int B) { return (B < 1 || B > SGL_MAX_B) ? -1 : num_coeffs(B); }
int64_t sgl_coeff_index(int n, int l, int m) {
  if (n < 1 || l < 0 || l >= n || m < -l || m > l) return -1;
  return omega(n, l, m);
}

sgl_status_t sgl_plan_ex(sgl_plan_t* out, const int* B_list, int nfunc, int dtype, unsigned flags) {
  return sgl_plan_scaled(out, B_list, nfunc, dtype, flags, 1.0);
}

sgl_status_t sgl_plan_scaled(sgl_plan_t* out, const int* B_list, int nfunc, int dtype, unsigned flags,
                             double radial_scale) {
  if (!out) { set_error("null output pointer"); return SGL_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!(radial_scale > 0.0) || !std::isfinite(radial_scale)) {
    set_error("radial scale must be positive and finite");
    return SGL_ERR_INVALID_ARG;
  }
  if (!B_list || nfunc < 1) { set_error("need at least one function"); return SGL_ERR_INVALID_ARG; }
  if (dtype != SGL_F64 && dtype != SGL_F32 && dtype != SGL_SPLIT_BF16) {
    set_error("unknown dtype");
    return SGL_ERR_INVALID_ARG;
  }
  if (flags & ~(SGL_SAMPLES_RAW | SGL_GRAPHS | SGL_AUTOTUNE | SGL_SEMINAIVE)) {
    set_error("unknown flag");
    return SGL_ERR_INVALID_ARG;
  }
  if ((flags & SGL_SAMPLES_RAW) && dtype != SGL_F64) {
    set_error("raw samples need SGL_F64 (they leave the FP32 range for B > ~40)");
    return SGL_ERR_UNSUPPORTED;
  }
  for (int f = 0; f < nfunc; ++f) {
    if (B_list[f] < 1 || B_list[f] > SGL_MAX_B) {
      set_error("bandlimit out of range [1, " + std::to_string(SGL_MAX_B) + "]");
      return SGL_ERR_INVALID_ARG;
    }
    const int B = B_list[f];
    if ((flags & SGL_SEMINAIVE) && (B < 8 || (B & (B - 1)) != 0)) {
      set_error("the seminaive Legendre step needs power-of-two bandlimits >= 8");
      return SGL_ERR_UNSUPPORTED;
    }
    if ((flags & SGL_SEMINAIVE) && dtype == SGL_SPLIT_BF16 && B > 128) {
      // odd orders contract against P_lm / sin(theta) in the cosine domain, whose
      // entries reach ~l^1.5; with the spectrum held in FP32 the split form's error
      // at B = 256 exceeds its 1e-6 bar (2e-6 measured at n = 256, l = 255, m = 1)
      set_error("the seminaive Legendre step in split-bf16 precision needs B <= 128");
      return SGL_ERR_UNSUPPORTED;
    }
  }
  std::unique_ptr<sgl_plan_s> p(new (std::nothrow) sgl_plan_s());
  if (!p) { set_error("host allocation failed"); return SGL_ERR_OOM; }
  p->dtype = dtype;
  p->flags = flags;
  p->rscale = radial_scale;
  p->Bs.assign(B_list, B_list + nfunc);
  for (int f = 0; f < nfunc; ++f) {
    p->soff.push_back(p->tot_s);
    p->coff.push_back(p->tot_c);
    p->tot_s += num_samples(B_list[f]);
    p->tot_c += num_coeffs(B_list[f]);
  }
  hipStream_t s = nullptr;
  {
    const char* fa = std::getenv("SGL_TEST_FAIL_ALLOC");
    g_fail_countdown = fa ? std::max(0L, std::strtol(fa, nullptr, 10)) : 0;
  }
  sgl_status_t st = make_plan(p.get(), s);
  if (st == SGL_OK && (flags & SGL_AUTOTUNE)) st = autotune(p.get(), s);
  g_fail_countdown = 0;
  if (st != SGL_OK) return st;  // unique_ptr frees everything allocated so far
  *out = p.release();
  return SGL_OK;
}

sgl_status_t sgl_plan(sgl_plan_t* out, int B, int batch, int dtype) {
  if (!out) { set_error("null output pointer"); return SGL_ERR_INVALID_ARG; }
  *out = nullptr;
  if (batch < 1) { set_error("batch must be >= 1"); return SGL_ERR_INVALID_ARG; }
  if (B < 1 || B > SGL_MAX_B) {
    set_error("bandlimit out of range [1, " + std::to_string(SGL_MAX_B) + "]");
    return SGL_ERR_INVALID_ARG;
  }
  std::vector<int> Bs(batch, B);
  return sgl_plan_ex(out, Bs.data(), batch, dtype, 0u);
}

sgl_status_t sgl_plan_destroy(sgl_plan_t plan) {
  delete plan;
  return SGL_OK;
}

sgl_status_t sgl_forward(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  SGL_TRY(check_call(plan, d_samples, plan->tot_s * plan->esz(), d_coeffs, plan->tot_c * plan->esz()));
  return run_direction(plan, 0, d_samples, d_coeffs, (hipStream_t)stream);
}

sgl_status_t sgl_naive_forward(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  SGL_TRY(check_call(plan, d_samples, plan->tot_s * plan->esz(), d_coeffs, plan->tot_c * plan->esz()));
  if (plan->dtype != SGL_F64) { set_error("the naive transforms run in SGL_F64 plans only"); return SGL_ERR_UNSUPPORTED; }
  const int ncls = (int)plan->classes.size();
  SGL_HIP_TRY(launch_naive_forward(plan->d_cls, plan->d_naive_pre, ncls, plan->n_naive_f, d_samples, d_coeffs,
                                   (plan->flags & SGL_SAMPLES_RAW) != 0, (hipStream_t)stream));
  return SGL_OK;
}

sgl_status_t sgl_naive_inverse(sgl_plan_t plan, const void* d_coeffs, void* d_samples, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  SGL_TRY(check_call(plan, d_coeffs, plan->tot_c * plan->esz(), d_samples, plan->tot_s * plan->esz()));
  if (plan->dtype != SGL_F64) { set_error("the naive transforms run in SGL_F64 plans only"); return SGL_ERR_UNSUPPORTED; }
  const int ncls = (int)plan->classes.size();
  SGL_HIP_TRY(launch_naive_inverse(plan->d_cls, plan->d_naive_pre + ncls + 1, ncls, plan->n_naive_i, d_coeffs,
                                   d_samples, (plan->flags & SGL_SAMPLES_RAW) != 0, (hipStream_t)stream));
  return SGL_OK;
}

sgl_status_t sgl_midpoint_forward(sgl_plan_t plan, const void* d_values, int nx, double half_width, void* d_coeffs,
                                  void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (nx < 1 || nx > 1024) { set_error("nx must be in [1, 1024]"); return SGL_ERR_INVALID_ARG; }
  if (!(half_width > 0.0) || !std::isfinite(half_width)) {
    set_error("half_width must be positive and finite");
    return SGL_ERR_INVALID_ARG;
  }
  const size_t nval = (size_t)plan->Bs.size() * nx * nx * nx;
  SGL_TRY(check_call(plan, d_values, nval * plan->esz(), d_coeffs, plan->tot_c * plan->esz()));
  if (plan->dtype != SGL_F64) { set_error("off-grid transforms run in SGL_F64 plans only"); return SGL_ERR_UNSUPPORTED; }
  const int ncls = (int)plan->classes.size();
  SGL_HIP_TRY(launch_midpoint_forward(plan->d_cls, plan->d_naive_pre, ncls, plan->n_naive_f, d_values, nx, half_width,
                                      d_coeffs, (hipStream_t)stream));
  return SGL_OK;
}

sgl_status_t sgl_synthesize_points(sgl_plan_t plan, const void* d_coeffs, int npts, const double* d_xyz,
                                   void* d_values, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (npts < 0) { set_error("npts must be >= 0"); return SGL_ERR_INVALID_ARG; }
  if (npts == 0) return SGL_OK;
  if (!d_xyz) { set_error("null point array"); return SGL_ERR_INVALID_ARG; }
  const size_t nval = (size_t)plan->Bs.size() * npts;
  SGL_TRY(check_call(plan, d_coeffs, plan->tot_c * plan->esz(), d_values, nval * plan->esz()));
  if (overlap(d_xyz, (size_t)npts * 3 * sizeof(double), d_values, nval * plan->esz())) {
    set_error("points and output overlap");
    return SGL_ERR_INVALID_ARG;
  }
  if (plan->dtype != SGL_F64) { set_error("off-grid transforms run in SGL_F64 plans only"); return SGL_ERR_UNSUPPORTED; }
  const int ncls = (int)plan->classes.size();
  const int64_t chunks = (npts + 255) / 256;
  SGL_HIP_TRY(launch_synthesize_points(plan->d_cls, plan->d_naive_pre + 2 * (ncls + 1), ncls,
                                       chunks * (int64_t)plan->Bs.size(), d_coeffs, npts, d_xyz, d_values,
                                       (hipStream_t)stream));
  return SGL_OK;
}

sgl_status_t sgl_forward_noalloc(sgl_plan_t plan, const void* d_samples, void* d_coeffs, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  SGL_TRY(check_call(plan, d_samples, plan->tot_s * plan->esz(), d_coeffs, plan->tot_c * plan->esz()));
  if (!plan->d_cls_static) {
    set_error("the plan's stage intermediates need " + std::to_string(plan->static_bytes) +
              " bytes, more than the static workspace of " + std::to_string(kScratchBytes) + " bytes");
    return SGL_ERR_INVALID_ARG;
  }
  int dev = -1;
  SGL_HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device) {
    set_error("sgl_forward_noalloc must run on the device its plan was created on");
    return SGL_ERR_INVALID_ARG;
  }
  // the stage launches, eager (no graph), on the static workspace
  const hipStream_t s = (hipStream_t)stream;
  for (int q = 0; q < 5; ++q) {
    const int slot = kSeq[0][q];
    if (slot_work(plan, slot) == 0) continue;
    SGL_HIP_TRY(launch_slot(plan, slot, d_samples, d_coeffs, s, plan->d_cls_static));
  }
  return SGL_OK;
}

sgl_status_t sgl_inverse(sgl_plan_t plan, const void* d_coeffs, void* d_samples, void* stream) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  SGL_TRY(check_call(plan, d_coeffs, plan->tot_c * plan->esz(), d_samples, plan->tot_s * plan->esz()));
  return run_direction(plan, 1, d_coeffs, d_samples, (hipStream_t)stream);
}

sgl_status_t sgl_plan_info(sgl_plan_t plan, int64_t* total_samples, int64_t* total_coeffs, int* nfunc) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (total_samples) *total_samples = plan->tot_s;
  if (total_coeffs) *total_coeffs = plan->tot_c;
  if (nfunc) *nfunc = (int)plan->Bs.size();
  return SGL_OK;
}

sgl_status_t sgl_offsets(sgl_plan_t plan, int64_t* sample_off, int64_t* coeff_off) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (sample_off) std::copy(plan->soff.begin(), plan->soff.end(), sample_off);
  if (coeff_off) std::copy(plan->coff.begin(), plan->coff.end(), coeff_off);
  return SGL_OK;
}

static const ClassHost* find_class(sgl_plan_t plan, int B) {
  for (auto& c : plan->classes)
    if (c.B == B) return &c;
  return nullptr;
}

sgl_status_t sgl_grid(sgl_plan_t plan, int B, double* r, double* log_a, double* log_sigma, double* theta,
                      double* btilde) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  const ClassHost* c = find_class(plan, B);
  if (!c) { set_error("bandlimit not in plan"); return SGL_ERR_INVALID_ARG; }
  const int L = 2 * B;
  double* dst[6] = {r, log_a, log_sigma, nullptr, theta, btilde};
  for (int q = 0; q < 6; ++q)
    if (dst[q]) SGL_HIP_TRY(hipMemcpy(dst[q], c->grid + q * L, L * sizeof(double), hipMemcpyDeviceToHost));
  if (r && plan->rscale != 1.0)
    for (int i = 0; i < L; ++i) r[i] *= plan->rscale;  // sampling radii of the scaled basis
  return SGL_OK;
}

sgl_status_t sgl_table(sgl_plan_t plan, int B, int which, double* host_out) {
  if (!plan || !host_out || which < 0 || which > 2) { set_error("bad argument"); return SGL_ERR_INVALID_ARG; }
  const ClassHost* c = find_class(plan, B);
  if (!c) { set_error("bandlimit not in plan"); return SGL_ERR_INVALID_ARG; }
  if (which == 2 && !c->D64) { set_error("not a seminaive plan"); return SGL_ERR_INVALID_ARG; }
  const double* src = which == 0 ? c->P64 : (which == 1 ? c->R64 : c->D64);
  SGL_HIP_TRY(hipMemcpy(host_out, src, (which == 2 ? table_size(B) / 2 : table_size(B)) * sizeof(double),
                        hipMemcpyDeviceToHost));
  return SGL_OK;
}

sgl_status_t sgl_launch_grids(sgl_plan_t plan, int* grids) {
  if (!plan || !grids) { set_error("bad argument"); return SGL_ERR_INVALID_ARG; }
  for (int q = 0; q < NSLOT; ++q) grids[q] = plan->grid[q] ? plan->grid[q] : slot_work(plan, q);
  return SGL_OK;
}

sgl_status_t sgl_launch_tiles(sgl_plan_t plan, int* tiles) {
  if (!plan || !tiles) { set_error("bad argument"); return SGL_ERR_INVALID_ARG; }
  const int prec = prec_of(plan->dtype);
  for (int q = 0; q < NSLOT; ++q) {
    const int tg = plan->tile[q];
    int rows = 0, cols = 0;
    if (q == S_LEG_F || q == S_LEG_I) {
      rows = gemm_tile_m_legendre(prec, tg);
      cols = gemm_tile_n_complex_legendre(prec, tg);
    } else if (q == S_RAD_F || q == S_RAD_I) {
      rows = gemm_tile_m_radial(tg);
      cols = gemm_tile_n_complex_radial(tg);
    }
    tiles[2 * q] = rows;
    tiles[2 * q + 1] = cols;
  }
  return SGL_OK;
}

sgl_status_t sgl_set_launch_tile(sgl_plan_t plan, int slot, int geometry) {
  if (!plan || slot < 0 || slot >= NSLOT || geometry < 0) { set_error("bad argument"); return SGL_ERR_INVALID_ARG; }
  if (geometry >= slot_geometries(plan, slot)) {
    set_error("this launch slot has no such tile geometry");
    return SGL_ERR_UNSUPPORTED;
  }
  if (plan->tile[slot] != geometry) {
    plan->tile[slot] = geometry;
    // captured graphs hold the previous kernels and work lists
    for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
    plan->graphs.clear();
  }
  return SGL_OK;
}

sgl_status_t sgl_set_timing(sgl_plan_t plan, int enable) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  if (enable && plan->ev.empty()) {
    plan->ev.resize(6 * sgl_plan_s::kRing * 2);
    for (auto& e : plan->ev) SGL_HIP_TRY(hipEventCreate(&e));
  }
  plan->timing = enable != 0;
  return SGL_OK;
}

sgl_status_t sgl_stage_times(sgl_plan_t plan, double* ms, int* counts) {
  if (!plan) { set_error("null plan"); return SGL_ERR_INVALID_ARG; }
  for (int st = 0; st < 6; ++st) {
    while (plan->pending[st] > 0) {
      int slot = (plan->head[st] - plan->pending[st] + sgl_plan_s::kRing) % sgl_plan_s::kRing;
      hipEvent_t a = plan->ev[(st * sgl_plan_s::kRing + slot) * 2];
      hipEvent_t b = plan->ev[(st * sgl_plan_s::kRing + slot) * 2 + 1];
      float t = 0;
      SGL_HIP_TRY(hipEventSynchronize(b));
      SGL_HIP_TRY(hipEventElapsedTime(&t, a, b));
      plan->ms[st] += t;
      plan->cnt[st] += 1;
      plan->pending[st] -= 1;
    }
    if (ms) ms[st] = plan->ms[st];
    if (counts) counts[st] = plan->cnt[st];
    plan->ms[st] = 0;
    plan->cnt[st] = 0;
  }
  return SGL_OK;
}

sgl_status_t sgl_debug_gemm(int dtype, int M, int N, int K, const double* d_A, const double* d_X, double* d_C) {
  if (M < 0 || N < 0 || K < 0 || !d_A || !d_X || !d_C) { set_error("bad argument"); return SGL_ERR_INVALID_ARG; }
  if (dtype != SGL_F64 && dtype != SGL_F32 && dtype != SGL_SPLIT_BF16) {
    set_error("unknown dtype");
    return SGL_ERR_INVALID_ARG;
  }
  SGL_HIP_TRY(launch_debug_gemm(prec_of(dtype), M, N, K, d_A, d_X, d_C, nullptr));
  SGL_HIP_TRY(hipDeviceSynchronize());
  return SGL_OK;
}

}  // extern "C"
