// libmas: C-ABI, setup, defect-correction cycle and FGMRES on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <functional>
#include <future>
#include <mutex>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mas.h"
#include "host.hpp"
#include "kernels.hpp"

#include <hipcub/hipcub.hpp>

using namespace mas;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

namespace {

SocParams soc_params(const mas_params& p) {
  SocParams c;
  c.kind = p.soc;
  c.theta = p.theta;
  c.eps = p.soc_eps;
  return c;
}

struct MasError : std::runtime_error {
  int code;
  MasError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(call)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw MasError(e_ == hipErrorOutOfMemory ? MAS_ENOMEM : MAS_EHIP,                      \
                     std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

inline void launch_check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw MasError(MAS_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// smallest power of two >= nr (columns of a block row in the kernels over nr right-hand sides)
inline int nr_pow2(int nr) { return nr <= 1 ? 1 : 1 << (32 - __builtin_clz((unsigned)nr - 1)); }

constexpr size_t kMaxLds = 64 * 1024;  // dynamic LDS per workgroup used by the patch kernels
// operators and factor stores from this size on are read with non-temporal loads
constexpr double kStreamBytes = 64.0 * 1024 * 1024;
constexpr int kNrKT = 4;                // right-hand sides per thread in the batched patch kernel
constexpr int kWidePatch = 128;         // patches of this many DoFs or more get a 256-thread workgroup
constexpr int kFullPatch = 512;         // levels with patches this large store full velocity blocks
constexpr int kWavePb = 4;              // patches (wavefronts) per workgroup of the shared-block wave kernel
constexpr int kPanelTpb = 1024;         // threads per patch of the panel kernel (largest shared block rows)
constexpr int kPanelBytes = 32 * 1024;  // LDS of one panel of the panel kernel

// LDS of the batched patch kernel: m x C block, two MAX_NS x C blocks, the
// staged record (f values) and the patch DoF list
template <typename T>
size_t nr_lds_bytes(int64_t max_m, int C, int64_t f) {
  return (size_t)(max_m * C + 2 * MAX_NS * C + f) * sizeof(T) + (size_t)max_m * sizeof(int);
}

// Patch shapes (DoFs per velocity component x3, seeds) served by the
// thread-per-patch kernel: interior 2D Taylor-Hood / P1isoP2 patches, interior
// Scott-Vogelius element patches and the small P1isoP2/P1 patches of the
// barycentric mesh.
// Patch shapes (DoFs per velocity component, seeds) with a thread-per-patch
// bucket kernel: the interior vertex patches of 2D Taylor-Hood and P1iso
// levels and the element patches of Scott-Vogelius K0, the dominant shapes of
// those levels' patch-shape histograms (larger or 3D shapes would not fit one
// thread's registers).  A level buckets a listed shape it holds at least
// bucket_min times: with a thread per patch a bucket pays only once it fills
// the GPU (measured on 2D Taylor-Hood: 64k patches 48.9 vs 40.3 solves/s
// with / without the bucket, 16k patches 91.9 vs 101.6, 3.7k 167 vs 239).
#define MAS_FAST_SHAPES(X) X(19, 19, 0, 1) X(6, 6, 0, 3) X(10, 10, 0, 1)
static bool is_fast_shape(const int32_t* d) {
#define MAS_IS(A, B, C, D) if (d[0] == A && d[1] == B && d[2] == C && d[3] == D) return true;
  MAS_FAST_SHAPES(MAS_IS)
#undef MAS_IS
  return false;
}

// ---------------------------------------------------------------------------
// device memory owned by a handle

// Device memory of a handle.
//  OWN:    every allocation is a hipMalloc of its own, returned by release().
//  BUFFER: allocations are carved, 256-byte aligned, from a caller-owned buffer:
//          persistent ones upward from its start, temporaries (setup work
//          areas) downward from its end, given back when their scope closes.
//          A request beyond the buffer throws MAS_ENOMEM.
//  DRY:    nothing is allocated and no device work is issued; the bytes a
//          BUFFER would need (peak of both ends) are counted.  The pointers
//          handed out are never dereferenced: every device operation of the
//          upload path checks dry() first.
struct DevArena {
  enum Mode { OWN, BUFFER, DRY };
  static constexpr size_t kAlign = 256;
  Mode mode = OWN;
  std::vector<void*> ptrs;  // OWN allocations
  size_t bytes = 0;         // persistent bytes held
  char* base = nullptr;     // BUFFER start (DRY: a fake, never-dereferenced base)
  size_t cap = 0, lo = 0, hi = 0, peak = 0;
  bool dry() const { return mode == DRY; }
  static size_t round(size_t nb) { return (nb + kAlign - 1) / kAlign * kAlign; }
  void* carve(size_t nb, bool temp) {
    nb = round(std::max<size_t>(nb, 1));
    if (mode == BUFFER && lo + hi + nb > cap)
      throw MasError(MAS_ENOMEM, "workspace of " + std::to_string(cap) + " bytes is too small (at least " +
                                     std::to_string(lo + hi + nb) + " needed so far; mas_workspace_size gives the "
                                     "total)");
    void* p;
    if (temp) {
      hi += nb;
      p = base + (mode == BUFFER ? cap - hi : (size_t)1 << 40) ;
    } else {
      p = base + lo;
      lo += nb;
      bytes += nb;
    }
    peak = std::max(peak, lo + hi);
    return p;
  }
  template <typename T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    if (mode != OWN) return (T*)carve(n * sizeof(T), false);
    void* p = nullptr;
    HIPCHECK(hipMalloc(&p, n * sizeof(T)));
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    return (T*)p;
  }
  template <typename T, typename S, typename Al>
  T* upload(const std::vector<S, Al>& v, hipStream_t s) {
    T* d = alloc<T>(v.size());
    if (v.empty() || dry()) return d;
    if constexpr (std::is_same<T, S>::value) {
      HIPCHECK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    } else {
      std::vector<T> tmp(v.begin(), v.end());
      HIPCHECK(hipMemcpyAsync(d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
    return d;
  }
  // BUFFER / DRY over [buf, buf + cap) (DRY: buf is a fake base, cap unused)
  void use_buffer(void* buf, size_t c, bool count_only) {
    release();
    mode = count_only ? DRY : BUFFER;
    base = count_only ? (char*)((size_t)1 << 44) : (char*)buf;
    cap = c;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
    lo = hi = peak = 0;
    mode = OWN;
    base = nullptr;
    cap = 0;
  }
  ~DevArena() { release(); }
};

// Setup work memory that lives until the scope closes: its own hipMallocs for
// an OWN arena, the top end of the buffer otherwise.  The upload path
// synchronises its stream before a scope closes.
struct TempScope {
  DevArena& parent;
  DevArena own;  // OWN-mode allocations
  size_t hi0;
  explicit TempScope(DevArena& p) : parent(p), hi0(p.hi) {}
  template <typename T>
  T* alloc(size_t n) {
    if (parent.mode == DevArena::OWN) return own.alloc<T>(n);
    return (T*)parent.carve(std::max<size_t>(n, 1) * sizeof(T), true);
  }
  template <typename T, typename S, typename Al>
  T* upload(const std::vector<S, Al>& v, hipStream_t s) {
    if (parent.mode == DevArena::OWN) return own.upload<T>(v, s);
    T* d = alloc<T>(v.size());
    if (v.empty() || dry()) return d;
    std::vector<T> tmp(v.begin(), v.end());
    HIPCHECK(hipMemcpyAsync(d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
    return d;
  }
  bool dry() const { return parent.dry(); }
  ~TempScope() {
    if (parent.mode != DevArena::OWN) parent.hi = hi0;
  }
};

// Sparse operator on the device: CSR (TEAM lanes per row) and, when the
// padding is small, a sliced-ELL copy (64-row slices).  The product kernel is
// chosen by timing at setup.
template <typename T>
struct DCsr {
  int64_t n = 0, m = 0, nnz = 0;
  int* ptr = nullptr;
  int* ind = nullptr;
  T* val = nullptr;
  int team = 8;
  int64_t nslices = 0;
  int64_t* soff = nullptr;
  int* swidth = nullptr;
  int* sind = nullptr;
  T* sval = nullptr;
  bool use_sell = false;
  bool stream = false;  // non-temporal loads of the entries (large, read once per use in a cycle)
};

// CSR arrays only (no sliced-ELL copy): operators the factorisation reads once
template <typename T, typename Ar>
DCsr<T> upload_csr_plain(Ar& A, const Csr& C, hipStream_t s) {
  if (C.nnz() >= (int64_t)INT32_MAX) throw MasError(MAS_EINVAL, "matrix too large for 32-bit offsets");
  DCsr<T> d;
  d.n = C.nr;
  d.m = C.nc;
  d.nnz = C.nnz();
  d.ptr = A.template upload<int>(C.ptr, s);
  d.ind = A.template upload<int>(C.ind, s);
  d.val = A.template upload<T>(C.val, s);
  return d;
}

template <typename T>
DCsr<T> upload_csr(DevArena& A, const Csr& C, hipStream_t s) {
  if (C.nnz() >= (int64_t)INT32_MAX) throw MasError(MAS_EINVAL, "matrix too large for 32-bit offsets");
  DCsr<T> d;
  d.n = C.nr;
  d.m = C.nc;
  d.nnz = C.nnz();
  d.ptr = A.upload<int>(C.ptr, s);
  d.ind = A.upload<int>(C.ind, s);
  d.val = A.upload<T>(C.val, s);
  double avg = C.nr ? (double)C.nnz() / (double)C.nr : 1.0;
  int t = 1;
  while (t < 64 && 2 * t <= avg) t *= 2;
  d.team = std::max(2, t);
  // sliced ELL when it pads little
  const int64_t ns = (C.nr + 63) / 64;
  std::vector<int64_t> soff(ns + 1, 0);
  std::vector<int> sw(ns, 0);
  for (int64_t sl = 0; sl < ns; ++sl) {
    int w = 0;
    for (int64_t r = sl * 64; r < std::min<int64_t>(C.nr, sl * 64 + 64); ++r)
      w = std::max<int>(w, (int)(C.ptr[r + 1] - C.ptr[r]));
    sw[sl] = w;
    soff[sl + 1] = soff[sl] + (int64_t)w * 64;
  }
  if (ns > 0 && soff[ns] <= (int64_t)(1.3 * (double)C.nnz()) + 64) {
    // slices are independent: filled over threads, every slot written once (padding: value 0)
    std::vector<int, NoInit<int>> sind(soff[ns]);
    std::vector<T, NoInit<T>> sval(soff[ns]);
    parallel_rows(ns, [&](int64_t lo, int64_t hi) {
      for (int64_t sl = lo; sl < hi; ++sl)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t r = sl * 64 + lane;
          int c = 0;
          if (r < C.nr)
            for (int64_t e = C.ptr[r]; e < C.ptr[r + 1]; ++e, ++c) {
              sind[soff[sl] + (int64_t)c * 64 + lane] = C.ind[e];
              sval[soff[sl] + (int64_t)c * 64 + lane] = (T)C.val[e];
            }
          const int pad_col = (r < C.nr && C.ptr[r + 1] > C.ptr[r]) ? C.ind[C.ptr[r]] : 0;
          for (; c < sw[sl]; ++c) {
            sind[soff[sl] + (int64_t)c * 64 + lane] = pad_col;
            sval[soff[sl] + (int64_t)c * 64 + lane] = (T)0;
          }
        }
    });
    d.nslices = ns;
    d.soff = A.upload<int64_t>(soff, s);
    d.swidth = A.upload<int>(sw, s);
    d.sind = A.upload<int>(sind, s);
    d.sval = A.upload<T>(sval, s);
  }
  return d;
}

template <typename T, int MODE, bool NT>
void csr_launch_nt(const DCsr<T>& A, const T* x, const T* b, T* y, hipStream_t s, ChebStep<T> cs) {
  const int bs = 256;
  if (A.use_sell) {
    hipLaunchKernelGGL((k_sell<T, MODE, NT>), dim3(blocks_for(A.nslices * 64, bs)), dim3(bs), 0, s, (int)A.n,
                       A.nslices, A.soff, A.swidth, A.sind, A.sval, x, b, y, cs);
    launch_check();
    return;
  }
  const unsigned nb = blocks_for(A.n * (int64_t)A.team, bs);
  switch (A.team) {
#define CASE(TM)                                                                                            \
  case TM:                                                                                                  \
    hipLaunchKernelGGL((k_csr<T, TM, MODE, NT>), dim3(nb), dim3(bs), 0, s, (int)A.n, A.ptr, A.ind, A.val, x, b, y, \
                       cs);                                                                                 \
    break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
    default: throw MasError(MAS_EINVAL, "bad team size");
  }
  launch_check();
}

template <typename T, int MODE>
void csr_launch(const DCsr<T>& A, const T* x, const T* b, T* y, hipStream_t s, ChebStep<T> cs = {}) {
  if (A.n == 0) return;
  if constexpr (MODE <= 1) {  // products and residuals of large level operators stream their entries
    if (A.stream) {
      csr_launch_nt<T, MODE, true>(A, x, b, y, s, cs);
      return;
    }
  }
  csr_launch_nt<T, MODE, false>(A, x, b, y, s, cs);
}

// Pick the lanes-per-row of a CSR product by timing every choice once on the
// actual operand (setup-time autotuning; vectors may hold any values).
template <typename T>
void autotune_team(DCsr<T>& A, const T* x, T* y, hipStream_t s, bool on) {
  if (A.n == 0 || A.nnz < 4096 || !on) {
    A.use_sell = A.nslices > 0;
    return;
  }
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  auto time_it = [&]() {
    csr_launch<T, 0>(A, x, nullptr, y, s);  // warm
    HIPCHECK(hipEventRecord(e0, s));
    for (int rep = 0; rep < 10; ++rep) csr_launch<T, 0>(A, x, nullptr, y, s);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  const int heuristic = A.team;
  A.use_sell = false;
  float best = time_it();  // heuristic lanes per row
  int best_team = heuristic;
  for (int team : {2, 4, 8, 16, 32, 64}) {
    if (team == heuristic) continue;
    A.team = team;
    const float ms = time_it();
    if (ms < 0.95f * best) {  // change only for a clear gain
      best = ms;
      best_team = team;
    }
  }
  A.team = best_team;
  if (A.nslices > 0) {
    A.use_sell = true;
    const float ms = time_it();
    A.use_sell = ms < best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ---------------------------------------------------------------------------
// levels of the cycle

// One fixed-shape bucket handled by the thread-per-patch kernel.
struct FastBucket {
  int shape[4] = {0, 0, 0, 0};
  int64_t P = 0, Ppad = 0;
  int* dofs = nullptr;  // interleaved DoF lists, M x Ppad
  int64_t fbase = 0;    // offset of the bucket's interleaved records in fac
  int64_t ybase = 0;    // offset of the bucket's outputs in Y
};

template <typename T>
struct DPatches {
  int64_t np = 0, ndofs = 0, nfac = 0, ny = 0;
  int64_t nfac_alg = 0;  // factor entries actually read (bucket padding excluded)
  // all patches (fast buckets first), used by the factorisation
  int64_t* off = nullptr;
  int4* dims = nullptr;
  int64_t* foff = nullptr;
  int64_t* fstride = nullptr;
  int* dofs = nullptr;
  T* fac = nullptr;
  // generic patches: indices [g0, np) of the arrays above
  int64_t g0 = 0, yshift = 0;
  int max_m = 0;
  int64_t max_f = 0;
  int layout = 0;  // LAYOUT_FULL: blocks stored n x n (very large patches); LAYOUT_SHARED: one
                  // A^-1 per patch for all velocity components (identical blocks)
  std::vector<FastBucket> fast;
  // DoF -> outputs map: CSR (inv_ptr, inv_pos) or slot-major ELL (ell, width)
  int* inv_ptr = nullptr;
  int* inv_pos = nullptr;
  int* ell = nullptr;
  int ell_width = 0;
  T* w = nullptr;
  T* Y = nullptr;
  // batched path: outputs at (off[p] + slot) * nr + k, maps in that numbering
  int* ell_c = nullptr;
  int* inv_ptr_c = nullptr;
  int* inv_pos_c = nullptr;
  T* Ynr = nullptr;
  bool stream = false;  // non-temporal loads of the factor records (far larger than the caches)
  int nr_chunk = 0;  // right-hand sides per workgroup of the batched patch kernel (LDS bound)
  bool col_ok = false;   // every generic patch fits the column-streaming kernel (components <= 128 rows, packed)
  int gen_kernel = 0;    // generic patches: 0 workgroup per patch, 2 wavefront per patch streaming
                         // columns, 3 wavefront per patch on shared blocks (chosen at setup)
  int wave_tt = 0;       // row tiles of 64 of the shared-block wavefront kernel (0: not usable)
  int nco = 0;           // velocity components a shared block serves
  bool pipe_ok = false;  // the persistent pipelined workgroup kernel takes this level's patches
  bool panel_ok = false;   // the panel kernel takes this level's patches (shared packed blocks)
  bool panel_auto = false; // ... and is the level's kernel (records too large to stage in LDS)
  unsigned pipe_grid = 0;  // its workgroups (resident at once), set when first launched
  bool parts_fit[3] = {true, true, true};  // shared blocks: every generic patch's partial row sums
                                           // fit in its staged copy of A (workgroups of 64 / 128 /
                                           // 256 threads)
  int wg_tb = 256;       // threads per patch of the workgroup kernel on levels of large patches
                         // (128 or 256, timed at setup)
  bool nr_stage = true;  // the batched kernel stages factor records in LDS
};

template <typename T>
struct DDlsc {
  bool on = false;
  DCsr<T> A, B, Bt, S;
  T* minv = nullptr;
  double lamA = 0.0, lamS = 0.0;
  int64_t nv = 0, np = 0;
  T *ru = nullptr, *vs = nullptr, *tmp = nullptr, *t1 = nullptr, *t2 = nullptr;  // velocity-sized
  T *rp = nullptr, *q = nullptr, *dp = nullptr;                                 // pressure-sized
  T *cd = nullptr, *cd2 = nullptr, *cres = nullptr;                             // Chebyshev work (max size)
  // AMG stages (Section 5): a smoothed-aggregation hierarchy of S with weighted Jacobi
  struct SLev {
    int64_t n = 0;
    DCsr<T> S, P, R;          // S_k; P: S_k <- S_{k+1}, R = P^T
    T* wdinv = nullptr;       // (4/3) / rho_k / diag(S_k)
    T *x = nullptr, *b = nullptr, *res = nullptr, *d1 = nullptr, *d2 = nullptr, *corr = nullptr;
  };
  std::vector<SLev> sh;       // empty: Chebyshev stages
  double* sinv = nullptr;     // dense inverse of the (bordered) coarsest S
  int64_t sld = 0;
};

template <typename T>
struct Level {
  int64_t n = 0, nvel = 0;
  DCsr<T> K;
  DCsr<T> P, R;  // P: this level <- next level, R = P^T
  DPatches<T> pt;
  DDlsc<T> dl;
  bool relax = false;
  bool krylov = false;  // relaxation wrapped in FGMRES (Section 3.3.1)
  T *x = nullptr, *b = nullptr, *r = nullptr;
};

struct CycleBase {
  virtual ~CycleBase() = default;
  virtual void apply(const double* r, double* z, hipStream_t s) = 0;
  virtual void set_nr(int nr) = 0;
  // Every per-application scratch array of the cycle for r right-hand sides,
  // in a fixed order: f(address of the pointer field, bytes).
  virtual void scratch_arrays(int r, const std::function<void(void**, size_t)>& f) = 0;
  // per level: patches in thread-per-patch buckets, and the kernel of the others
  virtual void describe(mas_hier_info& in) const = 0;
};

// Optional event timing of the cycle's kernels, per kernel kind, with the
// algorithmic bytes each timed launch has to move.
enum TimedKind { TK_TPP = 0, TK_GENERIC = 1, TK_BATCHED = 2, TK_SELL = 3, TK_CSR = 4, TK_SPMM = 5, TK_KINDS = 6 };
struct Timing {
  struct Rec {
    hipEvent_t a, b;
    double bytes;
    int kind;
  };
  bool on = false;
  std::vector<Rec> recs;
  double ms[TK_KINDS] = {}, bytes[TK_KINDS] = {};
  int64_t launches[TK_KINDS] = {};
  void begin(hipEvent_t& e0, hipEvent_t& e1, hipStream_t s) {
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipEventRecord(e0, s));
  }
  void end(hipEvent_t e0, hipEvent_t e1, hipStream_t s, double nbytes, int kind) {
    HIPCHECK(hipEventRecord(e1, s));
    recs.push_back({e0, e1, nbytes, kind});
  }
  void reset() {
    for (int k = 0; k < TK_KINDS; ++k) ms[k] = bytes[k] = 0, launches[k] = 0;
  }
  void collect() {
    for (auto& r : recs) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.kind] += t;
      bytes[r.kind] += r.bytes;
      launches[r.kind]++;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    recs.clear();
  }
};

template <typename T>
struct Cycle : CycleBase {
  std::vector<Level<T>> lev;  // 0 = free K0, 1 = free K1, ..., back() = coarsest (dense)
  double* Cinv = nullptr;     // dense inverse of the (bordered) coarsest operator
  int64_t nc_dense = 0, ld = 0;
  int64_t* free0 = nullptr;
  int64_t* dir0 = nullptr;
  int64_t nfree0 = 0, ndir0 = 0;
  mas_params par{};
  int dim = 2;
  int nr = 1, nr_max = 1;  // right-hand sides of the current application / allocated for
  Timing* tm = nullptr;
  // relaxation wrapper workspace, shared by the levels (they relax one at a time):
  // basis V (m + 1 vectors), directions Z (m), w, FP64 partial sums, H, beta, y
  T *kv = nullptr, *kz = nullptr, *kw = nullptr;
  double *kpart = nullptr, *kh = nullptr, *kbeta = nullptr, *ky = nullptr;
  int kblk = 512;
  // Scott-Vogelius pressure transfers (Section 3.1): P0^p duplication, R0^p = M_cg^-1 (P0^p)^T M_dg
  bool sv = false;
  int64_t np0 = 0, np1 = 0;
  DCsr<T> Mdg, P0t, P0p, Mcg;
  T* mcg_dinv = nullptr;
  int mass_steps = 0;
  T *sv_t0 = nullptr, *sv_t1 = nullptr, *sv_z = nullptr, *sv_cd = nullptr, *sv_cd2 = nullptr, *sv_cres = nullptr;

  // b1 = eta R0 r0
  void restrict0(const T* r0, Level<T>& L1, hipStream_t s) {
    const int64_t nv = L1.nvel * nr;
    if (!sv) {  // Taylor-Hood: injection
      hipLaunchKernelGGL((k_scale2<T>), dim3(blocks_for(L1.n * nr, 256)), dim3(256), 0, s, L1.n * nr, nv,
                         (T)par.eta_u, (T)par.eta_p, r0, L1.b);
      launch_check();
      return;
    }
    hipLaunchKernelGGL((k_scale2<T>), dim3(blocks_for(nv, 256)), dim3(256), 0, s, nv, nv, (T)par.eta_u,
                       (T)par.eta_u, r0, L1.b);
    spmv<0>(Mdg, r0 + nv, nullptr, sv_t0, s);   // M_dg r0_p
    spmv<0>(P0t, sv_t0, nullptr, sv_t1, s);     // (P0^p)^T M_dg r0_p
    // M_cg z = t1: Jacobi-preconditioned Chebyshev with the P1 bounds lambda(D^-1 M) in [1/2, 2]
    chebyshev_iv(Mcg, sv_t1, sv_z, 0.5, 2.0, mass_steps, mcg_dinv, sv_cd, sv_cd2, sv_cres, s);
    hipLaunchKernelGGL((k_axpby<T>), dim3(blocks_for(np1 * nr, 256)), dim3(256), 0, s, np1 * nr, (T)par.eta_p,
                       sv_z, (T)0, L1.b + nv);
    launch_check();
  }

  // x0 (+)= P0 x1
  void prolong0(Level<T>& L1, Level<T>& L0, bool x_zero, hipStream_t s) {
    if (!sv) {
      hipLaunchKernelGGL((k_axpby<T>), dim3(blocks_for(L0.n * nr, 256)), dim3(256), 0, s, L0.n * nr, (T)1, L1.x,
                         x_zero ? (T)0 : (T)1, L0.x);
      launch_check();
      return;
    }
    const int64_t nv = L1.nvel * nr;
    hipLaunchKernelGGL((k_axpby<T>), dim3(blocks_for(nv, 256)), dim3(256), 0, s, nv, (T)1, L1.x,
                       x_zero ? (T)0 : (T)1, L0.x);
    launch_check();
    if (x_zero) spmv<0>(P0p, L1.x + nv, nullptr, L0.x + nv, s);
    else spmv<2>(P0p, L1.x + nv, nullptr, L0.x + nv, s);
  }

  // sparse product, timed (with its algorithmic bytes) when timing is on
  template <int MODE>
  void spmv(const DCsr<T>& A, const T* x, const T* b, T* y, hipStream_t s, ChebStep<T> cs = {}) {
    hipEvent_t e0{}, e1{};
    const bool t = tm && tm->on;
    if (t) tm->begin(e0, e1, s);
    if (nr == 1) {
      csr_launch<T, MODE>(A, x, b, y, s, cs);
    } else if (A.n > 0) {
      hipLaunchKernelGGL((k_spmm<T, MODE>), dim3(blocks_for(A.n, 256 / nr_pow2(nr))), dim3(256), 0, s, A.n, nr, nr_pow2(nr), A.ptr, A.ind,
                         A.val, x, b, y, cs);
      launch_check();
    }
    if (t) {
      const double sz = sizeof(T);
      // MODE 4 also reads the direction once more and writes the new direction and the sum
      const double vec = (A.m * sz + A.n * sz * (MODE == 0 ? 1.0 : MODE == 4 ? 5.0 : 2.0)) * nr;
      tm->end(e0, e1, s, A.nnz * (sz + 4.0) + (A.n + 1) * 4.0 + vec, nr > 1 ? TK_SPMM : A.use_sell ? TK_SELL : TK_CSR);
    }
  }

  // y ~ X^{-1} r: `deg` steps of the Chebyshev semi-iteration from y = 0 for the
  // spectrum interval [lo, hi] of D^-1 X (D^-1 = dinv, identity when null)
  // The start of the iteration (d = Dinv r / theta, res = r, y = d) is done
  // here, or, when `started`, by the product that produced r (cheb_start below).
  void chebyshev_iv(DCsr<T>& X, const T* r, T* y, double lo, double hi, int deg, const T* dinv, T* cd, T* cd2,
                    T* cres, hipStream_t s, bool started = false) {
    const int64_t n = X.n * nr;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    const unsigned nb = blocks_for(n, 256);
    if (!started) {
      hipLaunchKernelGGL((k_cheb_init<T>), dim3(nb), dim3(256), 0, s, n, r, (T)(1.0 / theta), dinv, cd, cres, y, nr);
      launch_check();
    }
    // each step is one fused product (residual update, direction, sum); the
    // directions alternate between cd and cd2
    T* dcur = cd;
    T* dnext = cd2;
    for (int k = 0; k + 1 < deg; ++k) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      spmv<4>(X, dcur, nullptr, cres, s, ChebStep<T>{(T)(rho_new * rho), (T)(2.0 * rho_new / delta), dinv, dnext, y});
      std::swap(dcur, dnext);
      rho = rho_new;
    }
  }

  // DLSC inner solves: interval [0.5^dim lam, 1.1 lam] (Table 2)
  void chebyshev(DCsr<T>& X, const T* r, T* y, double lam, int deg, DDlsc<T>& D, hipStream_t s,
                 bool started = false) {
    chebyshev_iv(X, r, y, std::pow(0.5, dim) * lam, 1.1 * lam, deg, nullptr, D.cd, D.cd2, D.cres, s, started);
  }

  // epilogue for the product that produces the right-hand side of a DLSC
  // Chebyshev solve (sign a for MODE 5): it also starts that iteration
  ChebStep<T> cheb_start(double lam, T* y, DDlsc<T>& D, T a = (T)1) const {
    const double theta = 0.5 * (std::pow(0.5, dim) * lam + 1.1 * lam);
    ChebStep<T> cs{a, (T)(1.0 / theta), nullptr, D.cd, y};
    cs.res = D.cres;
    cs.cinv = nullptr;
    return cs;
  }

  // y = one V-cycle of smoothed aggregation with weighted Jacobi for S_k y = b
  // (the DLSC AMG stages, Section 5).  Jacobi in residual form is the fused
  // Chebyshev step with a = 0 and c = 1 (the weight is folded into wdinv):
  // res -= S d, d = wdinv res, acc += d.
  void s_vcycle(DDlsc<T>& D, size_t k, const T* b, T* x, hipStream_t s) {
    auto& L = D.sh[k];
    const int64_t n = L.n * nr;
    const unsigned nb = blocks_for(n, 256);
    if (k + 1 == D.sh.size()) {
      if (nr == 1)
        hipLaunchKernelGGL((k_dense_gemv<T>), dim3(blocks_for(L.n * WAVE, 256)), dim3(256), 0, s, (int)L.n,
                           (int)D.sld, D.sinv, b, x);
      else
        hipLaunchKernelGGL((k_dense_gemm<T>), dim3(nb), dim3(256), 0, s, (int)L.n, (int)D.sld, nr, D.sinv, b, x);
      launch_check();
      return;
    }
    const int nu = par.dlsc_amg;
    const ChebStep<T> jac{(T)0, (T)1, L.wdinv, nullptr, nullptr};
    // pre-relaxation from x = 0: d = wdinv b, x = d, res = b
    hipLaunchKernelGGL((k_cheb_init<T>), dim3(nb), dim3(256), 0, s, n, b, (T)1, L.wdinv, L.d1, L.res, x, nr);
    launch_check();
    T* dc = L.d1;
    T* dn = L.d2;
    for (int j = 1; j < nu; ++j) {
      ChebStep<T> cs = jac;
      cs.dnew = dn;
      cs.acc = x;
      spmv<4>(L.S, dc, nullptr, L.res, s, cs);
      std::swap(dc, dn);
    }
    spmv<3>(L.S, dc, nullptr, L.res, s);  // res = b - S x
    auto& C = D.sh[k + 1];
    spmv<0>(L.R, L.res, nullptr, C.b, s);
    s_vcycle(D, k + 1, C.b, C.x, s);
    spmv<2>(L.P, C.x, nullptr, x, s);  // x += P x_c
    // post-relaxation: the corrections accumulate in corr, then x += corr
    ChebStep<T> st{(T)1, (T)1, nullptr, L.d1, L.corr};
    st.res = L.res;
    st.cinv = L.wdinv;
    spmv<1>(L.S, x, b, L.res, s, st);  // res = b - S x, d = wdinv res, corr = d
    dc = L.d1;
    dn = L.d2;
    for (int j = 1; j < nu; ++j) {
      ChebStep<T> cs = jac;
      cs.dnew = dn;
      cs.acc = L.corr;
      spmv<4>(L.S, dc, nullptr, L.res, s, cs);
      std::swap(dc, dn);
    }
    hipLaunchKernelGGL((k_axpby<T>), dim3(nb), dim3(256), 0, s, n, (T)1, L.corr, (T)1, x);
    launch_check();
  }

  // one DLSC sweep (Algorithm 2) on level L: x = (u, p), b = (f, g)
  void dlsc_sweep(Level<T>& L, hipStream_t s) {
    DDlsc<T>& D = L.dl;
    const int64_t nv = D.nv * nr, np = D.np * nr;
    T* u = L.x;
    T* p = L.x + nv;
    const T* f = L.b;
    const T* g = L.b + nv;
    const unsigned bv = blocks_for(nv, 256);
    // each product that produces a Chebyshev right-hand side also starts that iteration
    spmv<1>(D.A, u, f, D.ru, s);  // ru = f - A u - B^T p
    spmv<3>(D.Bt, p, nullptr, D.ru, s, cheb_start(D.lamA, D.vs, D));
    chebyshev(D.A, D.ru, D.vs, D.lamA, par.cheb_deg[0], D, s, true);  // momentum
    hipLaunchKernelGGL((k_add<T>), dim3(bv), dim3(256), 0, s, nv, u, D.vs, D.tmp);
    const bool amg = !D.sh.empty();
    if (amg) {
      spmv<1>(D.B, D.tmp, g, D.rp, s);  // rp = g - B (u + v*)
      s_vcycle(D, 0, D.rp, D.q, s);     // continuity
    } else {
      spmv<1>(D.B, D.tmp, g, D.rp, s, cheb_start(D.lamS, D.q, D));  // rp = g - B (u + v*)
      chebyshev(D.S, D.rp, D.q, D.lamS, par.cheb_deg[1], D, s, true);  // continuity
    }
    // scaled products (MODE 5: y = a m (A x)) fold the M^-1 scalings and the sign in
    spmv<5>(D.Bt, D.q, nullptr, D.t1, s, ChebStep<T>{(T)1, (T)0, D.minv, nullptr, nullptr});  // t1 = M^-1 B^T q
    spmv<5>(D.A, D.t1, nullptr, D.t2, s, ChebStep<T>{(T)1, (T)0, D.minv, nullptr, nullptr});  // t2 = M^-1 A t1
    if (amg) {
      spmv<5>(D.B, D.t2, nullptr, D.rp, s, ChebStep<T>{(T)-1, (T)0, nullptr, nullptr, nullptr});  // rp = -B t2
      s_vcycle(D, 0, D.rp, D.dp, s);  // pressure correction
    } else {
      spmv<5>(D.B, D.t2, nullptr, D.rp, s, cheb_start(D.lamS, D.dp, D, (T)-1));  // rp = -B t2
      chebyshev(D.S, D.rp, D.dp, D.lamS, par.cheb_deg[2], D, s, true);  // pressure correction
    }
    // u += v* + M^-1 B^T q, p += dp (u and p are contiguous in L.x)
    hipLaunchKernelGGL((k_dlsc_update<T>), dim3(blocks_for(nv + np, 256)), dim3(256), 0, s, nv, np, u, D.vs, D.t1,
                       D.dp);
    launch_check();
  }

  // `sweeps` relaxation sweeps on L (Vanka or DLSC); x_zero: L.x is to be taken as 0
  // One relaxation wrapped in FGMRES (Section 3.3.1): m = krylov_its iterations
  // of right-preconditioned flexible GMRES on K e = b - K x from e = 0, each
  // preconditioned by one undamped Vanka sweep; Arnoldi by modified
  // Gram-Schmidt with FP64 sums; the small least-squares problem on the device;
  // then x += Z y.  No host synchronisation (the cycle stays capturable).
  void krylov_relax(Level<T>& L, bool x_zero, hipStream_t s) {
    const int m = par.krylov_its;
    const int64_t n = L.n;
    const unsigned nb = (unsigned)std::min<int64_t>(kblk, std::max<int64_t>(1, (n + 255) / 256));
    double* part[2] = {kpart, kpart + kblk};
    const T* r0 = L.b;
    if (!x_zero) {
      spmv<1>(L.K, L.x, L.b, L.r, s);
      r0 = L.r;
    }
    // beta = ||r0||, v_0 = r0 / beta
    hipLaunchKernelGGL((k_mgs_step<T>), dim3(nb), dim3(256), 0, s, n, const_cast<T*>(r0), nullptr, nullptr, nullptr,
                       nullptr, part[0], 1);
    hipLaunchKernelGGL((k_normalize<T>), dim3(nb), dim3(256), 0, s, n, part[0], (int)nb, kbeta, r0, kv);
    launch_check();
    for (int j = 0; j < m; ++j) {
      T* vj = kv + (int64_t)j * n;
      T* zj = kz + (int64_t)j * n;
      patch_solve(L, vj, s);  // z_j = M v_j: one undamped sweep from zero
      pull(L, (T)1, zj, 0, s);
      spmv<0>(L.K, zj, nullptr, kw, s);  // w = K z_j
      for (int i = 0; i <= j + 1; ++i) {
        const T* vprev = i > 0 ? kv + (int64_t)(i - 1) * n : nullptr;
        double* hprev = i > 0 ? kh + (size_t)(i - 1) * m + j : nullptr;
        const double* pprev = i > 0 ? part[(i - 1) & 1] : nullptr;
        const T* vnext = i <= j ? kv + (int64_t)i * n : nullptr;
        hipLaunchKernelGGL((k_mgs_step<T>), dim3(nb), dim3(256), 0, s, n, kw, vprev, hprev, pprev, vnext,
                           part[i & 1], i <= j ? 0 : 1);
      }
      hipLaunchKernelGGL((k_normalize<T>), dim3(nb), dim3(256), 0, s, n, part[(j + 1) & 1], (int)nb,
                         kh + (size_t)(j + 1) * m + j, kw, kv + (int64_t)(j + 1) * n);
      launch_check();
    }
    hipLaunchKernelGGL(k_krylov_ls, dim3(1), dim3(64), 0, s, m, kh, kbeta, ky);
    if (x_zero) hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, n, L.x, (T)0);
    hipLaunchKernelGGL((k_update_x<T>), dim3(blocks_for(n, 256)), dim3(256), 0, s, n, m, kz, ky, L.x);
    launch_check();
  }

  void relax_level(Level<T>& L, int sweeps, T omega, bool x_zero, hipStream_t s) {
    if (L.krylov) {  // sweeps wrapped relaxations
      for (int k = 0; k < sweeps; ++k) krylov_relax(L, x_zero && k == 0, s);
      return;
    }
    if (L.dl.on) {
      if (x_zero) {
        hipLaunchKernelGGL((k_fill<T>), dim3(blocks_for(L.n * nr, 256)), dim3(256), 0, s, L.n * nr, L.x, (T)0);
        launch_check();
      }
      for (int k = 0; k < sweeps; ++k) dlsc_sweep(L, s);
      return;
    }
    vanka_sweeps(L, sweeps, omega, x_zero, s);
  }

  // Algorithmic bytes of one patch-solve launch over a set of patches: their
  // factor records, DoF lists and outputs, plus each distinct level-vector
  // entry they read once (at most the level size).
  double patch_bytes(const Level<T>& L, double fac_entries, double slots) const {
    const double sz = sizeof(T);
    return fac_entries * sz + slots * (4.0 + sz * nr) + std::min<double>(slots, (double)L.n) * sz * nr;
  }

  void patch_solve(Level<T>& L, const T* rin, hipStream_t s) {
    DPatches<T>& pt = L.pt;
    const bool timed = tm && tm->on;
    hipEvent_t e0{}, e1{};
    if (nr > 1) {
      if (pt.nr_chunk < 1) throw MasError(MAS_EINVAL, "patches too large for the batched kernel");
      if (timed) tm->begin(e0, e1, s);
      // fixed-shape buckets: a wavefront per patch, a lane per right-hand side
      int64_t start = 0;
      constexpr int WPB = 4;
      const bool sh = (pt.layout & LAYOUT_SHARED) != 0;
      for (const FastBucket& fb : pt.fast) {
        const dim3 gb((unsigned)((fb.P + WPB - 1) / WPB), (unsigned)((nr + WAVE - 1) / WAVE));
        const T* f = pt.fac + fb.fbase;
#define MAS_RHS(A, B, C2, D)                                                                                    \
  if (fb.shape[0] == A && fb.shape[1] == B && fb.shape[2] == C2 && fb.shape[3] == D) {                        \
    if (sh)                                                                                                    \
      hipLaunchKernelGGL((k_vanka_rhs<T, A, B, C2, D, true, WPB>), gb, dim3(WPB * WAVE), 0, s, fb.P, fb.Ppad, nr, \
                         fb.dofs, f, pt.off + start, rin, pt.Ynr);                                              \
    else                                                                                                       \
      hipLaunchKernelGGL((k_vanka_rhs<T, A, B, C2, D, false, WPB>), gb, dim3(WPB * WAVE), 0, s, fb.P, fb.Ppad,   \
                         nr, fb.dofs, f, pt.off + start, rin, pt.Ynr);                                          \
  } else
        MAS_FAST_SHAPES(MAS_RHS) { throw MasError(MAS_EINVAL, "unknown patch bucket shape"); }
#undef MAS_RHS
        start += fb.P;
      }
      // the other patches: a workgroup per patch and chunk of right-hand sides
      const int64_t ng = pt.np - pt.g0;
      if (ng > 0) {
        int C = kNrKT;
        while (C < nr && C < pt.nr_chunk) C *= 2;
        const dim3 grid((unsigned)ng, (unsigned)((nr + C - 1) / C));
        const size_t shm = nr_lds_bytes<T>(pt.max_m, C, pt.nr_stage ? pt.max_f : 0);
        const int64_t g0 = pt.g0;
        if (pt.nr_stage)
          hipLaunchKernelGGL((k_vanka_apply_nr<T, kNrKT, true>), grid, dim3(256), shm, s, ng, nr, C, pt.off + g0,
                             pt.dims + g0, pt.foff + g0, pt.fstride + g0, pt.dofs, pt.fac, rin, pt.Ynr, pt.max_m,
                             pt.max_f, pt.layout);
        else
          hipLaunchKernelGGL((k_vanka_apply_nr<T, kNrKT, false>), grid, dim3(256), shm, s, ng, nr, C, pt.off + g0,
                             pt.dims + g0, pt.foff + g0, pt.fstride + g0, pt.dofs, pt.fac, rin, pt.Ynr, pt.max_m,
                             pt.max_f, pt.layout);
      }
      launch_check();
      if (timed) tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg, (double)pt.ndofs), TK_BATCHED);
      return;
    }
    double fast_fac = 0.0, fast_slots = 0.0;
    for (const FastBucket& fb : pt.fast) {
      const unsigned nb = blocks_for(fb.P, 256);
      const int* d = fb.dofs;
      const T* f = pt.fac + fb.fbase;
      T* y = pt.Y + fb.ybase;
      const int n0 = fb.shape[0], n1 = fb.shape[1], n2 = fb.shape[2], nsd = fb.shape[3];
      const int nvb = n0 + n1 + n2;
      const double rec = (double)record_entries(n0, n1, n2, nsd, pt.layout);
      fast_fac += rec * fb.P;
      fast_slots += (double)(nvb + nsd) * fb.P;
      if (timed) tm->begin(e0, e1, s);
#define MAS_TPP_GO(A, B, C, D, NT, SH) \
  hipLaunchKernelGGL((k_vanka_tpp<T, A, B, C, D, NT, SH>), dim3(nb), dim3(256), 0, s, fb.P, fb.Ppad, d, f, rin, y)
#define MAS_TPP(A, B, C, D)                                                            \
  if (fb.shape[0] == A && fb.shape[1] == B && fb.shape[2] == C && fb.shape[3] == D) { \
    const bool sh = (pt.layout & LAYOUT_SHARED) != 0;                                   \
    if (pt.stream && sh) MAS_TPP_GO(A, B, C, D, true, true);                            \
    else if (pt.stream) MAS_TPP_GO(A, B, C, D, true, false);                            \
    else if (sh) MAS_TPP_GO(A, B, C, D, false, true);                                   \
    else MAS_TPP_GO(A, B, C, D, false, false);                                          \
  } else
      MAS_FAST_SHAPES(MAS_TPP) { throw MasError(MAS_EINVAL, "unknown patch bucket shape"); }
#undef MAS_TPP
#undef MAS_TPP_GO
      launch_check();
      if (timed) tm->end(e0, e1, s, patch_bytes(L, rec * fb.P, (double)(nvb + nsd) * fb.P), TK_TPP);
    }
    const int64_t ng = pt.np - pt.g0;
    if (ng > 0 && pt.gen_kernel == 5) {
      constexpr int PL = kPanelBytes / kPanelTpb / (int)sizeof(T);
      const size_t shm = (size_t)2 * pt.max_m * sizeof(T) + kPanelBytes;
      if (timed) tm->begin(e0, e1, s);
#define MAS_PANEL(NC, NT)                                                                                          \
  hipLaunchKernelGGL((k_vanka_panel<T, NC, NT, kPanelTpb, PL>), dim3((unsigned)ng), dim3(kPanelTpb), shm, s, ng,  \
                     pt.off + pt.g0, pt.dims + pt.g0, pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.max_m,        \
                     pt.yshift)
      if (pt.nco == 3 && pt.stream) MAS_PANEL(3, true);
      else if (pt.nco == 3) MAS_PANEL(3, false);
      else if (pt.stream) MAS_PANEL(2, true);
      else MAS_PANEL(2, false);
#undef MAS_PANEL
      launch_check();
      if (timed)
        tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg - fast_fac, (double)pt.ndofs - fast_slots), TK_GENERIC);
    } else if (ng > 0 && pt.gen_kernel == 4) {
      const bool wide = pt.max_m >= kWidePatch;
      const int tb = wide ? 256 : WAVE;
      const int sp = (pt.layout & LAYOUT_SHARED) && !pt.parts_fit[wide ? 2 : 0] ? 3 * tb : 0;
      const size_t shm = (size_t)(2 * pt.max_m + sp + pt.max_f) * sizeof(T);
      const int ul = pt.max_f <= 8 * tb ? 8 : 16;
      if (pt.pipe_grid == 0) {  // as many workgroups as stay resident
        int dev = 0, cus = 0, per = 0;
        HIPCHECK(hipGetDevice(&dev));
        HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
#define MAS_OCC(TB, NT, U) \
  HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_vanka_pipe<T, TB, NT, U>, TB, shm))
        if (tb == 256) { if (ul == 8) MAS_OCC(256, true, 8); else MAS_OCC(256, true, 16); }
        else { if (ul == 8) MAS_OCC(WAVE, true, 8); else MAS_OCC(WAVE, true, 16); }
#undef MAS_OCC
        pt.pipe_grid = (unsigned)std::max(1, cus * std::max(1, per));
      }
      const dim3 grid((unsigned)std::min<int64_t>(ng, pt.pipe_grid));
      if (timed) tm->begin(e0, e1, s);
#define MAS_PIPE(TB, NT, U)                                                                                    \
  hipLaunchKernelGGL((k_vanka_pipe<T, TB, NT, U>), grid, dim3(TB), shm, s, ng, pt.off + pt.g0, pt.dims + pt.g0, \
                     pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.max_m, pt.yshift, pt.layout, sp)
      if (tb == 256) {
        if (pt.stream) { if (ul == 8) MAS_PIPE(256, true, 8); else MAS_PIPE(256, true, 16); }
        else { if (ul == 8) MAS_PIPE(256, false, 8); else MAS_PIPE(256, false, 16); }
      } else {
        if (pt.stream) { if (ul == 8) MAS_PIPE(WAVE, true, 8); else MAS_PIPE(WAVE, true, 16); }
        else { if (ul == 8) MAS_PIPE(WAVE, false, 8); else MAS_PIPE(WAVE, false, 16); }
      }
#undef MAS_PIPE
      launch_check();
      if (timed)
        tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg - fast_fac, (double)pt.ndofs - fast_slots), TK_GENERIC);
    } else if (ng > 0 && pt.gen_kernel == 3) {
      if (timed) tm->begin(e0, e1, s);
      const dim3 grid((unsigned)((ng + kWavePb - 1) / kWavePb));
      const size_t shm = (size_t)kWavePb * 2 * pt.max_m * sizeof(T);
#define MAS_WAVE(TT, NC, NT)                                                                                          \
  hipLaunchKernelGGL((k_vanka_wave<T, TT, NC, NT, kWavePb>), grid, dim3(kWavePb * WAVE), shm, s, ng,                \
                     pt.off + pt.g0, pt.dims + pt.g0, pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.max_m, pt.yshift)
#define MAS_WAVE_NC(TT, NT)            \
  if (pt.nco == 3) MAS_WAVE(TT, 3, NT); \
  else MAS_WAVE(TT, 2, NT)
      if (pt.wave_tt == 1 && pt.stream) { MAS_WAVE_NC(1, true); }
      else if (pt.wave_tt == 1) { MAS_WAVE_NC(1, false); }
      else if (pt.stream) { MAS_WAVE_NC(2, true); }
      else { MAS_WAVE_NC(2, false); }
#undef MAS_WAVE
#undef MAS_WAVE_NC
      launch_check();
      if (timed)
        tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg - fast_fac, (double)pt.ndofs - fast_slots), TK_GENERIC);
    } else if (ng > 0 && pt.gen_kernel == 2) {
      if (timed) tm->begin(e0, e1, s);
      constexpr int WPB = 4;
      const dim3 grid((unsigned)((ng + WPB - 1) / WPB));
      if (pt.stream)
        hipLaunchKernelGGL((k_vanka_col<T, true, WPB>), grid, dim3(WPB * WAVE), 0, s, ng, pt.off + pt.g0,
                           pt.dims + pt.g0, pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.yshift);
      else
        hipLaunchKernelGGL((k_vanka_col<T, false, WPB>), grid, dim3(WPB * WAVE), 0, s, ng, pt.off + pt.g0,
                           pt.dims + pt.g0, pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.yshift);
      launch_check();
      if (timed)
        tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg - fast_fac, (double)pt.ndofs - fast_slots), TK_GENERIC);
    } else if (ng > 0) {
      // four wavefronts per patch for large patches (more loads in flight, a row per thread)
      const bool wide = pt.max_m >= kWidePatch;
      const bool sh = (pt.layout & LAYOUT_SHARED) != 0;
      // LDS: b and y (max_m each), the shared layout's partial row sums (3 TPB
      // values, unless every patch's fit in its staged copy of A), the staged record
      const int tb_stage = wide ? pt.wg_tb : WAVE;
      const int fit_k = tb_stage == 256 ? 2 : tb_stage == 128 ? 1 : 0;
      const int sp_stage = sh && !pt.parts_fit[fit_k] ? 3 * tb_stage : 0;
      const bool stage = (size_t)(2 * pt.max_m + sp_stage + pt.max_f) * sizeof(T) <= kMaxLds;
      const int tb = stage ? tb_stage : (pt.max_m >= kFullPatch ? 1024 : tb_stage);
      const int sp = stage ? sp_stage : (sh ? 3 * tb : 0);
      const size_t shm = (size_t)(2 * pt.max_m + sp + (stage ? pt.max_f : 0)) * sizeof(T);
      // loads in flight per thread while a record is staged: enough for the
      // level's longest record where that takes at most 16
      const int ul = pt.max_f <= 8 * tb ? 8 : pt.max_f <= 12 * tb ? 12 : pt.max_f <= 16 * tb ? 16
                     : pt.max_f <= 24 * tb ? 24 : 32;
      if (timed) tm->begin(e0, e1, s);
#define MAS_GENERIC(ST, TB, NT, U)                                                                                \
  hipLaunchKernelGGL((k_vanka_apply<T, ST, TB, NT, U>), dim3((unsigned)ng), dim3(TB), shm, s, ng, pt.off + pt.g0, \
                     pt.dims + pt.g0, pt.foff + pt.g0, pt.dofs, pt.fac, rin, pt.Y, pt.max_m, pt.yshift, pt.layout, sp)
#define MAS_GENERIC_UL(ST, TB, NT)                \
  if (ul == 8) MAS_GENERIC(ST, TB, NT, 8);        \
  else if (ul == 12) MAS_GENERIC(ST, TB, NT, 12); \
  else if (ul == 16) MAS_GENERIC(ST, TB, NT, 16); \
  else if (ul == 24) MAS_GENERIC(ST, TB, NT, 24); \
  else MAS_GENERIC(ST, TB, NT, 32)
      if (stage && tb == 256 && pt.stream) { MAS_GENERIC_UL(true, 256, true); }
      else if (stage && tb == 128 && pt.stream) { MAS_GENERIC_UL(true, 128, true); }
      else if (stage && pt.stream) { MAS_GENERIC_UL(true, WAVE, true); }
      else if (stage && tb == 256) { MAS_GENERIC_UL(true, 256, false); }
      else if (stage && tb == 128) { MAS_GENERIC_UL(true, 128, false); }
      else if (stage) { MAS_GENERIC_UL(true, WAVE, false); }
      else if (tb == 1024) MAS_GENERIC(false, 1024, false, 8);
      else if (tb == 256) MAS_GENERIC(false, 256, false, 8);
      else MAS_GENERIC(false, WAVE, false, 8);
#undef MAS_GENERIC
#undef MAS_GENERIC_UL
      launch_check();
      if (timed)
        tm->end(e0, e1, s, patch_bytes(L, (double)pt.nfac_alg - fast_fac, (double)pt.ndofs - fast_slots), TK_GENERIC);
    }
  }

  // Kernel for the generic (non-bucket) patches of a level: the workgroup
  // kernel or, where the level's patches fit it, the column-streaming
  // wavefront kernel, whichever is faster on this level's patches, timed at
  // setup on a zero input (3 launches each after a warm-up); without timing
  // the workgroup kernel (measured faster on the 2D and 3D Taylor-Hood levels).
  void choose_generic_kernel(Level<T>& L, bool tune, hipStream_t s) {
    DPatches<T>& pt = L.pt;
    pt.gen_kernel = 0;
    const int want = par.patch_kernel;
    if (want >= 2) {  // requested: taken where the level allows it
      if (want == 2 && pt.col_ok) pt.gen_kernel = 2;
      if (want == 3 && pt.wave_tt > 0) pt.gen_kernel = 3;
      if (want == 4 && pt.pipe_ok) pt.gen_kernel = 4;
      if (want == 5 && pt.panel_ok) pt.gen_kernel = 5;
      return;
    }
    // levels of packed shared blocks too large for LDS: the panel kernel (the
    // workgroup kernel would read such blocks uncoalesced)
    if (pt.panel_auto && want == 0) {
      pt.gen_kernel = 5;
      return;
    }
    pt.wg_tb = 256;
    if (!tune || pt.np - pt.g0 <= 0 || (pt.max_m < kWidePatch && (want == 1 || (!pt.col_ok && pt.wave_tt == 0 &&
                                                                               !pt.pipe_ok))))
      return;
    HIPCHECK(hipMemsetAsync(L.r, 0, (size_t)L.n * sizeof(T), s));
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    auto time_it = [&](int kind) {
      pt.gen_kernel = kind;
      patch_solve(L, L.r, s);
      HIPCHECK(hipEventRecord(e0, s));
      for (int rep = 0; rep < 3; ++rep) patch_solve(L, L.r, s);
      HIPCHECK(hipEventRecord(e1, s));
      HIPCHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    // candidates: 0 workgroup per patch, 2 column-streaming wavefront (packed
    // per-component blocks), 3 wavefront per patch on shared blocks, 4 the
    // persistent pipelined workgroup kernel
    // the workgroup kernel with 256 and, on levels of large patches, 128 threads per patch
    pt.wg_tb = 256;
    float t_wg = time_it(0);
    if (pt.max_m >= kWidePatch) {
      pt.wg_tb = 128;
      const float t128 = time_it(0);
      if (t128 < t_wg) t_wg = t128;
      else pt.wg_tb = 256;
    }
    float best = t_wg, t_col = -1.f, t_wave = -1.f, t_pipe = -1.f;
    int pick = 0;
    if (want != 1 && pt.col_ok && (t_col = time_it(2)) < best) best = t_col, pick = 2;
    if (want != 1 && pt.wave_tt > 0 && (t_wave = time_it(3)) < best) best = t_wave, pick = 3;
    if (want != 1 && pt.pipe_ok && (t_pipe = time_it(4)) < best) best = t_pipe, pick = 4;
    pt.gen_kernel = pick;
    if (std::getenv("MAS_TRACE_SETUP"))
      std::fprintf(stderr, "[mas setup] level of %lld rows, %lld generic patches (max %d DoFs), us per sweep: "
                   "workgroup %.1f (%d threads), column %.1f, wave %.1f, pipelined %.1f -> kernel %d\n", (long long)L.n,
                   (long long)(pt.np - pt.g0), pt.max_m, 1e3 * t_wg / 3, pt.wg_tb, t_col < 0 ? -1.0 : 1e3 * t_col / 3,
                   t_wave < 0 ? -1.0 : 1e3 * t_wave / 3, t_pipe < 0 ? -1.0 : 1e3 * t_pipe / 3, pick);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }

  void vanka_sweeps(Level<T>& L, int sweeps, T omega, bool x_zero, hipStream_t s) {
    for (int k = 0; k < sweeps; ++k) {
      const T* rin;
      if (k == 0 && x_zero) {
        rin = L.b;
      } else {
        spmv<1>(L.K, L.x, L.b, L.r, s);
        rin = L.r;
      }
      patch_solve(L, rin, s);
      pull(L, omega, L.x, (k == 0 && x_zero) ? 0 : 1, s);
    }
  }

  // x (+)= omega W sum of the patch outputs, per DoF (acc = 0: overwrite)
  void pull(Level<T>& L, T omega, T* x, int acc, hipStream_t s) {
    if (nr > 1) {
      const int nrp = nr <= 1 ? 1 : 1 << (32 - __builtin_clz((unsigned)nr - 1));  // columns per block row
      const unsigned nb = blocks_for(L.n, 256 / nrp);
      if (L.pt.ell_c)
        hipLaunchKernelGGL((k_vanka_pull_ell_nr<T>), dim3(nb), dim3(256), 0, s, (int)L.n, nr, nrp, L.pt.ell_width,
                           L.pt.ell_c, L.pt.Ynr, omega, x, acc);
      else
        hipLaunchKernelGGL((k_vanka_pull_nr<T>), dim3(nb), dim3(256), 0, s, (int)L.n, nr, nrp, L.pt.inv_ptr_c,
                           L.pt.inv_pos_c, L.pt.Ynr, L.pt.w, omega, x, acc);
    } else if (L.pt.ell) {
      hipLaunchKernelGGL((k_vanka_pull_ell<T>), dim3(blocks_for(L.n, 256)), dim3(256), 0, s, (int)L.n,
                         L.pt.ell_width, L.pt.ell, L.pt.Y, omega, x, acc);
    } else {
      hipLaunchKernelGGL((k_vanka_pull<T>), dim3(blocks_for(L.n, 256)), dim3(256), 0, s, (int)L.n, L.pt.inv_ptr,
                         L.pt.inv_pos, L.pt.Y, L.pt.w, omega, x, acc);
    }
    launch_check();
  }

  // cycle on level l >= 1 with right-hand side lev[l].b, result in lev[l].x
  void vcycle(size_t l, hipStream_t s) {
    Level<T>& L = lev[l];
    if (l + 1 == lev.size()) {
      if (nr == 1)
        hipLaunchKernelGGL((k_dense_gemv<T>), dim3(blocks_for(L.n * WAVE, 256)), dim3(256), 0, s, (int)L.n,
                           (int)ld, Cinv, L.b, L.x);
      else
        hipLaunchKernelGGL((k_dense_gemm<T>), dim3(blocks_for(L.n * nr, 256)), dim3(256), 0, s, (int)L.n, (int)ld,
                           nr, Cinv, L.b, L.x);
      launch_check();
      return;
    }
    const T om = (T)par.omega;
    bool x_zero = true;
    const int nu1 = par.relax == MAS_RELAX_VANKA_DLSC ? par.nu_dlsc : par.nu1;
    const int nu2 = par.relax == MAS_RELAX_VANKA_DLSC ? par.nu_dlsc : par.nu2;
    if (L.relax && nu1 > 0) {
      relax_level(L, nu1, om, true, s);
      x_zero = false;
    }
    Level<T>& C = lev[l + 1];
    if (x_zero) {
      spmv<0>(L.R, L.b, nullptr, C.b, s);
    } else {
      spmv<1>(L.K, L.x, L.b, L.r, s);
      spmv<0>(L.R, L.r, nullptr, C.b, s);
    }
    vcycle(l + 1, s);
    if (x_zero) {
      spmv<0>(L.P, C.x, nullptr, L.x, s);
    } else {
      spmv<2>(L.P, C.x, nullptr, L.x, s);
    }
    if (L.relax && nu2 > 0) relax_level(L, nu2, om, false, s);
  }

  void scratch_arrays(int r, const std::function<void(void**, size_t)>& f) override {
    const size_t st = sizeof(T), sd = sizeof(double);
    auto v = [&](T*& p, int64_t n) { f((void**)&p, (size_t)n * st); };
    auto vd = [&](double*& p, int64_t n) { f((void**)&p, (size_t)n * sd); };
    for (Level<T>& L : lev) {
      v(L.x, L.n * r);
      v(L.b, L.n * r);
      v(L.r, L.n * r);
      if (L.pt.np > 0) {
        v(L.pt.Y, L.pt.ny);
        if (r > 1) v(L.pt.Ynr, L.pt.ndofs * r);
      }
      if (L.dl.on) {
        DDlsc<T>& D = L.dl;
        for (T** q : {&D.ru, &D.vs, &D.tmp, &D.t1, &D.t2}) v(*q, D.nv * r);
        for (T** q : {&D.rp, &D.q, &D.dp}) v(*q, D.np * r);
        for (T** q : {&D.cd, &D.cd2, &D.cres}) v(*q, std::max(D.nv, D.np) * r);
        for (auto& Lk : D.sh)
          for (T** q : {&Lk.x, &Lk.b, &Lk.res, &Lk.d1, &Lk.d2, &Lk.corr})
            if (*q) v(*q, Lk.n * r);
      }
    }
    if (kv) {  // relaxation wrapper (one right-hand side)
      const int m = par.krylov_its;
      int64_t nmax = 0;
      for (Level<T>& L : lev)
        if (L.krylov) nmax = std::max(nmax, L.n);
      v(kv, (int64_t)(m + 1) * nmax);
      v(kz, (int64_t)m * nmax);
      v(kw, nmax);
      vd(kpart, 2 * (int64_t)kblk);
      vd(kh, (int64_t)(m + 1) * m);
      vd(kbeta, 1);
      vd(ky, m);
    }
    if (sv) {
      v(sv_t0, np0 * r);
      for (T** q : {&sv_t1, &sv_z, &sv_cd, &sv_cd2, &sv_cres}) v(*q, np1 * r);
    }
  }

  void describe(mas_hier_info& in) const override {
    for (size_t l = 0; l < lev.size() && l < 16; ++l) {
      const DPatches<T>& pt = lev[l].pt;
      int64_t nb = 0;
      for (const FastBucket& fb : pt.fast) nb += fb.P;
      in.bucket_patches[l] = nb;
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 4; ++c) in.bucket_shapes[l][4 * q + c] = q < (int)pt.fast.size() ? pt.fast[q].shape[c] : 0;
      in.patch_kernel[l] = pt.np - pt.g0 > 0 ? (pt.gen_kernel == 0 ? 1 : pt.gen_kernel) : 0;
    }
  }

  void set_nr(int k) override {
    if (k > 1 && par.krylov_its > 0)
      throw MasError(MAS_EINVAL, "the FGMRES-wrapped relaxation takes one right-hand side per call");
    nr = k;
  }

  void apply(const double* r, double* z, hipStream_t s) override {
    Level<T>& L0 = lev[0];
    Level<T>& L1 = lev[1];
    if (nr == 1)
      hipLaunchKernelGGL((k_gather<T, double>), dim3(blocks_for(nfree0, 256)), dim3(256), 0, s, nfree0, free0, r,
                         L0.b);
    else
      hipLaunchKernelGGL((k_gather_nr<T, double>), dim3(blocks_for(nfree0 * nr, 256)), dim3(256), 0, s, nfree0, nr,
                         free0, r, L0.b);
    launch_check();
    bool x_zero = true;
    if (L0.relax && par.nu1 > 0) {
      relax_level(L0, par.nu1, (T)par.omega0, true, s);
      x_zero = false;
    }
    const T* r0 = L0.b;
    if (!x_zero) {
      spmv<1>(L0.K, L0.x, L0.b, L0.r, s);
      r0 = L0.r;
    }
    restrict0(r0, L1, s);  // eta R0 r0 (eq. (3.2))
    vcycle(1, s);
    prolong0(L1, L0, x_zero, s);  // x0 += P0 x1
    if (L0.relax && par.nu2 > 0) relax_level(L0, par.nu2, (T)par.omega0, false, s);
    if (nr == 1) {
      hipLaunchKernelGGL((k_scatter<double, T>), dim3(blocks_for(nfree0, 256)), dim3(256), 0, s, nfree0, free0, L0.x,
                         z);
      if (ndir0)  // Dirichlet rows are identity rows: z_D = r_D
        hipLaunchKernelGGL(k_copy_idx, dim3(blocks_for(ndir0, 256)), dim3(256), 0, s, ndir0, dir0, r, z);
    } else {
      hipLaunchKernelGGL((k_scatter_nr<double, T>), dim3(blocks_for(nfree0 * nr, 256)), dim3(256), 0, s, nfree0, nr,
                         free0, L0.x, z);
      if (ndir0)
        hipLaunchKernelGGL(k_copy_idx_nr, dim3(blocks_for(ndir0 * nr, 256)), dim3(256), 0, s, ndir0, nr, dir0, r, z);
    }
    launch_check();
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// the handle

struct HostDlsc {
  Csr A, B, Bt, S;            // velocity block, divergence block, its transpose, B M^-1 B^T
  std::vector<double> minv;   // M_u^-1 (diagonal)
  double lamA = 0.0, lamS = 0.0;
  // AMG stages: S_0 = S, S_{k+1} = P_k^T S_k P_k, Jacobi scalings, dense (bordered) coarsest
  std::vector<Csr> Sk, Pk;
  std::vector<std::vector<double>> wdinv;
  std::vector<double> sc_dense;
  int64_t sc_ld = 0;
};

struct HostPlan {
  std::vector<Csr> Ks, Ps;                 // free level operators, P_l (level l <- l+1)
  std::vector<HostDlsc> dlsc;              // per relaxed level when the relaxation is DLSC
  std::vector<std::vector<int8_t>> fields;
  std::vector<PatchSet> patches;
  std::vector<bool> relax;
  Csr Kb;                                  // coarsest operator (bordered when singular)
  std::vector<int64_t> free0, dir0;
  Csr K0;                                  // full K0 (FGMRES operator)
  std::vector<double> pw;                  // pressure weights
  bool sv = false;
  Csr Mdg, P0t, P0p, Mcg;                  // Scott-Vogelius transfer data (free pressure numbering)
  std::vector<double> mcg_dinv;
  int mass_steps = 0;
};

struct mas_handle {
  DevArena arena;
  HostPlan plan;
  bool on_device = false;
  int32_t dim = 2, disc = MAS_TH;
  mas_params par{};
  int64_t n0 = 0, nu0 = 0;
  DCsr<double> K0full;
  std::unique_ptr<CycleBase> cyc;
  mas_hier_info info{};
  int32_t p_nullspace = 0;
  double* pw = nullptr;  // pressure weights (np0)
  double pw_sum = 0.0;
  // FGMRES work
  double *V = nullptr, *Z = nullptr, *w = nullptr, *partial = nullptr, *hdev = nullptr, *ydev = nullptr;
  double* cpart = nullptr;  // classical Gram-Schmidt dot partials ((m + 1) x blocks x right-hand sides)
  bool use_mgs = false;     // MAS_MGS: modified Gram-Schmidt instead
  double* hhost = nullptr;  // pinned
  int nblk_dot = 512;
  hipStream_t gs = nullptr;     // internal stream: solves run here (graphs cannot capture the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hipGraphExec_t> iter_graph;  // one captured FGMRES inner iteration per Krylov index
  bool use_graphs = true;
  int64_t* dir_idx = nullptr;
  int64_t ndir = 0;
  Timing tm;
};

namespace {

Csr get_csr(const mas_csr& c, const char* name) {
  if (!c.indptr || !c.indices || !c.data || c.nrows <= 0 || c.ncols <= 0)
    throw MasError(MAS_EINVAL, std::string("missing matrix ") + name);
  if (c.indptr[0] != 0) throw MasError(MAS_EINVAL, std::string(name) + ": bad indptr");
  for (int64_t i = 0; i < c.nrows; ++i)
    if (c.indptr[i + 1] < c.indptr[i]) throw MasError(MAS_EINVAL, std::string(name) + ": bad indptr");
  Csr A = csr_copy(c.nrows, c.ncols, c.indptr, c.indices, c.data);
  // row checks in parallel; the first failing row (in row order) names the error
  const int nt = setup_threads();
  std::vector<std::pair<int64_t, std::string>> bad(nt + 1, {INT64_MAX, std::string()});
  std::atomic<int> slot{0};
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    auto& mine = bad[std::min(slot.fetch_add(1), nt)];
    for (int64_t i = lo; i < hi && mine.first == INT64_MAX; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        const char* why = nullptr;
        if (A.ind[e] < 0 || A.ind[e] >= A.nc) why = ": column out of range";
        else if (e > A.ptr[i] && A.ind[e] <= A.ind[e - 1]) why = ": columns not sorted/unique";
        else if (!std::isfinite(A.val[e])) why = ": non-finite value";
        if (why) {
          mine = {i, std::string(name) + why};
          break;
        }
      }
  });
  const auto first = std::min_element(bad.begin(), bad.end(),
                                      [](const auto& a, const auto& b) { return a.first < b.first; });
  if (first->first != INT64_MAX) throw MasError(MAS_EINVAL, first->second);
  return A;
}

// Phase timings of the setup on stderr when MAS_TRACE_SETUP is set.
struct SetupTrace {
  bool on = std::getenv("MAS_TRACE_SETUP") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const std::string& what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[mas setup] %-36s %9.1f ms\n", what.c_str(),
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

// The LDS table's row capacity of the device sparse products: at most
// min(cap, 3/4 of the table) distinct columns (cap <= 0: no extra limit).
static int spgemm_table_cap(int cap) {
  const int full = kSpgSlots * 3 / 4;
  return cap > 0 ? std::min(cap, full) : full;
}

// Classical Gram-Schmidt of one Arnoldi step over the j1 basis vectors V
// (nr interleaved columns): the dots in chunks of at most kCgsChunk vectors
// (one launch per chunk, its width a template argument), their block sums,
// then the update in the same chunks; the last chunk leaves the partial norms
// of w in part_out.
static void cgs_step(int64_t n, int nr, int nrp, int j1, const double* V, double* w, double* cpart, double* hdev,
                     double* part_out, unsigned nb, hipStream_t s) {
#define MAS_CGS_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
  for (int i0 = 0; i0 < j1; i0 += kCgsChunk) {
    const int na = std::min(kCgsChunk, j1 - i0);
    switch (na) {
#define MAS_DOTS(NA) \
  case NA: hipLaunchKernelGGL((k_cgs_dots_nr<NA>), dim3(nb), dim3(256), 0, s, n, nr, nrp, i0, V, w, cpart); break;
      MAS_CGS_CASES(MAS_DOTS)
#undef MAS_DOTS
    }
  }
  hipLaunchKernelGGL(k_cgs_final_nr, dim3((unsigned)(j1 * nr)), dim3(64), 0, s, (int)nb, nr, j1, cpart, hdev);
  for (int i0 = 0; i0 < j1; i0 += kCgsChunk) {
    const int na = std::min(kCgsChunk, j1 - i0);
    const int last = i0 + na >= j1 ? 1 : 0;
    switch (na) {
#define MAS_UPD(NA)                                                                                             \
  case NA:                                                                                                      \
    hipLaunchKernelGGL((k_cgs_update_nr<NA>), dim3(nb), dim3(256), 0, s, n, nr, nrp, i0, last, V, hdev, w, \
                       part_out);                                                                               \
    break;
      MAS_CGS_CASES(MAS_UPD)
#undef MAS_UPD
    }
  }
#undef MAS_CGS_CASES
}

// ---------------------------------------------------------------------------
// Smoothed aggregation with the level operators resident on the device
// (Algorithm 1; Section 3.2 for the strength of connection).  Per level: the
// diagonal and the Gershgorin bound, the strength graph, its transfer to the
// host for the greedy aggregation, the tentative prolongator's values from the
// near-null vector (host, O(n)), the smoothed prolongator and the Galerkin
// product A_c = P^T (A P), all with the host's operations in the host's order.
// Device CSR in FP64 with 32-bit columns, rows sorted.
struct SaMat {
  int64_t nr = 0, nc = 0, nnz = 0;
  int64_t* ptr = nullptr;
  int* ind = nullptr;
  double* val = nullptr;
};

// ptr[0] = 0, ptr[i + 1] = cnt[0] + ... + cnt[i]; returns ptr[n] (a
// synchronising read).
static int64_t sa_scan(const int64_t* cnt, int64_t* ptr, int64_t n, DevArena& tmp, hipStream_t s) {
  HIPCHECK(hipMemsetAsync(ptr, 0, sizeof(int64_t), s));
  if (n > 0) {
    if (n >= (int64_t)INT32_MAX) throw MasError(MAS_EINVAL, "setup operator too large for 32-bit row counts");
    size_t b = 0;
    HIPCHECK(hipcub::DeviceScan::InclusiveSum(nullptr, b, cnt, ptr + 1, (int)n, s));
    void* t = tmp.alloc<char>(b);
    HIPCHECK(hipcub::DeviceScan::InclusiveSum(t, b, cnt, ptr + 1, (int)n, s));
  }
  int64_t last = 0;
  HIPCHECK(hipMemcpyAsync(&last, ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (last >= (int64_t)INT32_MAX) throw MasError(MAS_EINVAL, "setup operator too large for 32-bit offsets");
  return last;
}

static SaMat sa_upload(const Csr& A, DevArena& ar, hipStream_t s) {
  SaMat M;
  M.nr = A.nr;
  M.nc = A.nc;
  M.nnz = A.nnz();
  M.ptr = ar.upload<int64_t>(A.ptr, s);
  M.ind = ar.upload<int>(A.ind, s);
  M.val = ar.upload<double>(A.val, s);
  return M;
}

static Csr sa_download(const SaMat& M, hipStream_t s) {
  Csr A;
  A.nr = M.nr;
  A.nc = M.nc;
  A.ptr.resize(M.nr + 1);
  A.ind.resize(M.nnz);
  A.val.resize(M.nnz);
  HIPCHECK(hipMemcpyAsync(A.ptr.data(), M.ptr, (M.nr + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  if (M.nnz > 0) {
    HIPCHECK(hipMemcpyAsync(A.ind.data(), M.ind, M.nnz * sizeof(int), hipMemcpyDeviceToHost, s));
    if (M.val) HIPCHECK(hipMemcpyAsync(A.val.data(), M.val, M.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    else std::fill(A.val.begin(), A.val.end(), 1.0);
  }
  HIPCHECK(hipStreamSynchronize(s));
  return A;
}

// A^T with the rows of each column ascending (the host transpose's order):
// a stable radix sort of the entry numbers by column.  Pattern only when
// values is false.
static SaMat sa_transpose(const SaMat& A, bool values, DevArena& out, DevArena& tmp, hipStream_t s) {
  SaMat T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.nnz = A.nnz;
  T.ptr = out.alloc<int64_t>(T.nr + 1);
  T.ind = out.alloc<int>(A.nnz);
  T.val = values ? out.alloc<double>(A.nnz) : nullptr;
  unsigned long long* cnt = tmp.alloc<unsigned long long>(std::max<int64_t>(T.nr, 1));
  HIPCHECK(hipMemsetAsync(cnt, 0, std::max<int64_t>(T.nr, 1) * sizeof(unsigned long long), s));
  if (A.nnz > 0) {
    hipLaunchKernelGGL(k_sa_colcount, dim3(blocks_for(A.nnz, 256)), dim3(256), 0, s, A.nnz, A.ind, cnt);
    launch_check();
  }
  sa_scan((const int64_t*)cnt, T.ptr, T.nr, tmp, s);
  if (A.nnz == 0) return T;
  int* row = tmp.alloc<int>(A.nnz);
  int* seq = tmp.alloc<int>(A.nnz);
  int* perm = tmp.alloc<int>(A.nnz);
  unsigned* keys = tmp.alloc<unsigned>(A.nnz);
  hipLaunchKernelGGL(k_sa_rows, dim3(blocks_for(A.nr, 256)), dim3(256), 0, s, A.nr, A.ptr, row);
  hipLaunchKernelGGL(k_sa_iota, dim3(blocks_for(A.nnz, 256)), dim3(256), 0, s, A.nnz, seq);
  launch_check();
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < A.nc) ++bits;
  size_t b = 0;
  HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const unsigned*)A.ind, keys, seq, perm, (int)A.nnz, 0,
                                              bits, s));
  void* t = tmp.alloc<char>(b);
  HIPCHECK(hipcub::DeviceRadixSort::SortPairs(t, b, (const unsigned*)A.ind, keys, seq, perm, (int)A.nnz, 0, bits,
                                              s));
  hipLaunchKernelGGL(k_sa_gather, dim3(blocks_for(A.nnz, 256)), dim3(256), 0, s, A.nnz, perm, row, A.val, T.ind,
                     T.val);
  launch_check();
  return T;
}

// C = A B, the host product's pattern and bits: k_spgemm_row for rows whose
// distinct columns fit its LDS table, k_spgemm_dense for the others.
static SaMat sa_spgemm(const SaMat& A, const SaMat& B, int cap_limit, DevArena& out, DevArena& tmp,
                       hipStream_t s) {
  if (A.nc != B.nr) throw MasError(MAS_EINVAL, "spgemm: shape mismatch");
  SaMat C;
  C.nr = A.nr;
  C.nc = B.nc;
  const int64_t n = A.nr;
  C.ptr = out.alloc<int64_t>(n + 1);
  if (n == 0) {
    sa_scan(nullptr, C.ptr, 0, tmp, s);
    return C;
  }
  const int cap = spgemm_table_cap(cap_limit);
  int64_t* cnt = tmp.alloc<int64_t>(n);
  int* over = tmp.alloc<int>(n);
  hipLaunchKernelGGL(k_spgemm_row<0>, dim3((unsigned)n), dim3(64), 0, s, n, A.ptr, A.ind, A.val, B.ptr, B.ind,
                     B.val, cap, cnt, over, nullptr, nullptr, nullptr);
  launch_check();
  int* nover_d = tmp.alloc<int>(1);
  size_t b = 0;
  HIPCHECK(hipcub::DeviceReduce::Sum(nullptr, b, over, nover_d, (int)n, s));
  void* t = tmp.alloc<char>(b);
  HIPCHECK(hipcub::DeviceReduce::Sum(t, b, over, nover_d, (int)n, s));
  int nover = 0;
  HIPCHECK(hipMemcpyAsync(&nover, nover_d, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  // long rows: a dense slice of B.nc columns per workgroup, at most 1 GiB
  unsigned G = 0;
  double* acc = nullptr;
  int64_t* mark = nullptr;
  if (nover > 0) {
    const int64_t per = std::max<int64_t>(B.nc, 1) * (int64_t)(sizeof(double) + sizeof(int64_t));
    G = (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nover, 1024, ((int64_t)1 << 30) / per}));
    acc = tmp.alloc<double>((size_t)G * std::max<int64_t>(B.nc, 1));
    mark = tmp.alloc<int64_t>((size_t)G * std::max<int64_t>(B.nc, 1));
    HIPCHECK(hipMemsetAsync(mark, 0xff, (size_t)G * std::max<int64_t>(B.nc, 1) * sizeof(int64_t), s));
    hipLaunchKernelGGL(k_spgemm_dense<0>, dim3(G), dim3(256), 0, s, n, A.ptr, A.ind, A.val, B.ptr, B.ind, B.val,
                       B.nc, over, acc, mark, cnt, nullptr, nullptr, nullptr);
    launch_check();
  }
  C.nnz = sa_scan(cnt, C.ptr, n, tmp, s);
  C.ind = out.alloc<int>(C.nnz);
  C.val = out.alloc<double>(C.nnz);
  hipLaunchKernelGGL(k_spgemm_row<1>, dim3((unsigned)n), dim3(64), 0, s, n, A.ptr, A.ind, A.val, B.ptr, B.ind,
                     B.val, cap, cnt, over, C.ptr, C.ind, C.val);
  launch_check();
  if (nover > 0) {
    hipLaunchKernelGGL(k_spgemm_dense<1>, dim3(G), dim3(256), 0, s, n, A.ptr, A.ind, A.val, B.ptr, B.ind, B.val,
                       B.nc, over, acc, mark, cnt, C.ptr, C.ind, C.val);
    launch_check();
  }
  return C;
}

// The kept entries of A (pattern only).
static SaMat sa_select(const SaMat& A, const unsigned char* keep, DevArena& out, DevArena& tmp, hipStream_t s) {
  SaMat S;
  S.nr = S.nc = A.nr;
  S.ptr = out.alloc<int64_t>(A.nr + 1);
  int64_t* cnt = tmp.alloc<int64_t>(std::max<int64_t>(A.nr, 1));
  const unsigned g = blocks_for(std::max<int64_t>(A.nr, 1), 256);
  hipLaunchKernelGGL(k_sa_select<0>, dim3(g), dim3(256), 0, s, A.nr, A.ptr, A.ind, keep, cnt, nullptr, nullptr);
  launch_check();
  S.nnz = sa_scan(cnt, S.ptr, A.nr, tmp, s);
  S.ind = out.alloc<int>(S.nnz);
  hipLaunchKernelGGL(k_sa_select<1>, dim3(g), dim3(256), 0, s, A.nr, A.ptr, A.ind, keep, nullptr, S.ptr, S.ind);
  launch_check();
  return S;
}

// The strength graph of A with near-null vector B (the host's strength_graph).
static Csr sa_strength(const SaMat& A, const double* d, double rho, const std::vector<double>& B,
                       const SocParams& soc, DevArena& tmp, hipStream_t s) {
  const int64_t n = A.nr;
  const unsigned g = blocks_for(std::max<int64_t>(n, 1), 256);
  unsigned char* keep = tmp.alloc<unsigned char>(A.nnz);
  if (soc.kind == 1) {
    hipLaunchKernelGGL(k_sa_soc_sym, dim3(g), dim3(256), 0, s, n, A.ptr, A.ind, A.val, d, soc.theta * soc.theta,
                       keep);
    launch_check();
    return sa_download(sa_select(A, keep, tmp, tmp, s), s);
  }
  const double dt = 1.0 / rho;
  double* z = tmp.alloc<double>(A.nnz);
  const double* Bd = tmp.upload<double>(B, s);
  hipLaunchKernelGGL(k_sa_soc_evol, dim3((unsigned)n), dim3(64), 0, s, n, A.ptr, A.ind, A.val, d, Bd, dt, soc.eps,
                     z, keep);
  launch_check();
  // the union of the kept pairs and their transposes
  const SaMat S1 = sa_select(A, keep, tmp, tmp, s);
  const SaMat S1t = sa_transpose(S1, false, tmp, tmp, s);
  SaMat S;
  S.nr = S.nc = n;
  S.ptr = tmp.alloc<int64_t>(n + 1);
  int64_t* cnt = tmp.alloc<int64_t>(std::max<int64_t>(n, 1));
  hipLaunchKernelGGL(k_sa_union<0>, dim3(g), dim3(256), 0, s, n, S1.ptr, S1.ind, S1t.ptr, S1t.ind, cnt, nullptr,
                     nullptr);
  launch_check();
  S.nnz = sa_scan(cnt, S.ptr, n, tmp, s);
  S.ind = tmp.alloc<int>(S.nnz);
  hipLaunchKernelGGL(k_sa_union<1>, dim3(g), dim3(256), 0, s, n, S1.ptr, S1.ind, S1t.ptr, S1t.ind, nullptr, S.ptr,
                     S.ind);
  launch_check();
  return sa_download(S, s);
}

// sa_field (Algorithm 1 on one scalar field) with the level operators on the
// device: the same prolongators and near-null vectors, bit for bit.
void device_sa_field(const Csr& A0, const SocParams& soc, int max_coarse, int max_levels, int cap,
                     std::vector<Csr>& Ps, std::vector<std::vector<double>>& Bs, hipStream_t s) {
  Ps.clear();
  Bs.clear();
  std::vector<double> B(A0.nr, 1.0);
  Bs.push_back(B);
  auto cur = std::make_unique<DevArena>();
  SaMat A = sa_upload(A0, *cur, s);
  while (A.nr > max_coarse && (int)Ps.size() + 1 < max_levels) {
    DevArena lv;  // this level's work memory
    const int64_t n = A.nr;
    const unsigned g = blocks_for(n, 256);
    double* d = lv.alloc<double>(n);
    double* ratio = lv.alloc<double>(n);
    hipLaunchKernelGGL(k_sa_diag, dim3(g), dim3(256), 0, s, n, A.ptr, A.ind, A.val, d, ratio);
    launch_check();
    const unsigned nb = std::min(1024u, g);
    double* part = lv.alloc<double>(nb);
    hipLaunchKernelGGL(k_sa_max, dim3(nb), dim3(256), 0, s, n, ratio, part);
    launch_check();
    std::vector<double> hp(nb);
    HIPCHECK(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double rho = 0.0;
    for (double v : hp) rho = std::max(rho, v);
    int32_t nc = 0;
    const std::vector<int32_t> agg = aggregate(sa_strength(A, d, rho, B, soc, lv, s), &nc);
    if (nc >= A.nr) break;
    // tentative interpolation from the near-null vector (host, one value per row)
    std::vector<double> nrm2(nc, 0.0);
    for (int64_t i = 0; i < n; ++i) nrm2[agg[i]] += B[i] * B[i];
    std::vector<double> Bc(nc);
    for (int32_t J = 0; J < nc; ++J) Bc[J] = std::sqrt(nrm2[J]);
    std::vector<double> tv(n);
    for (int64_t i = 0; i < n; ++i) tv[i] = B[i] / Bc[agg[i]];
    SaMat T;
    T.nr = T.nnz = n;
    T.nc = nc;
    T.ptr = lv.alloc<int64_t>(n + 1);
    hipLaunchKernelGGL(k_sa_iota64, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n + 1, T.ptr);
    launch_check();
    T.ind = lv.upload<int>(agg, s);
    T.val = lv.upload<double>(tv, s);
    // P = (I - omega D^-1 A) T, omega = (4/3) / rho
    const double omega = (4.0 / 3.0) / rho;
    SaMat DA = A;
    DA.val = lv.alloc<double>(A.nnz);
    hipLaunchKernelGGL(k_sa_scale, dim3(g), dim3(256), 0, s, n, A.ptr, A.val, d, DA.val);
    launch_check();
    SaMat P = sa_spgemm(DA, T, cap, lv, lv, s);
    hipLaunchKernelGGL(k_sa_smooth, dim3(g), dim3(256), 0, s, n, P.ptr, P.ind, P.val, T.ind, T.val, omega);
    launch_check();
    // A_c = P^T (A P), kept on the device for the next level
    auto next = std::make_unique<DevArena>();
    const SaMat AP = sa_spgemm(A, P, cap, lv, lv, s);
    const SaMat Pt = sa_transpose(P, true, lv, lv, s);
    const SaMat Ac = sa_spgemm(Pt, AP, cap, *next, lv, s);
    Ps.push_back(sa_download(P, s));  // synchronises the stream
    A = Ac;
    cur = std::move(next);
    B = Bc;
    Bs.push_back(B);
  }
  HIPCHECK(hipStreamSynchronize(s));
}

// device_sa_field for several fields: with setup threads, each field on a
// host thread and a stream of its own (the host's aggregation of one field
// overlaps the device work of the others); otherwise one after another on s.
// Each field's hierarchy is the same either way.
void device_sa_fields(const std::vector<Csr>& A, const SocParams& soc, int max_coarse, int max_levels, int cap,
                      std::vector<std::vector<Csr>>& Ps, std::vector<std::vector<std::vector<double>>>& Bs,
                      hipStream_t s) {
  const size_t nf = A.size();
  Ps.assign(nf, {});
  Bs.assign(nf, {});
  if (setup_threads() <= 1 || nf <= 1) {
    for (size_t f = 0; f < nf; ++f) device_sa_field(A[f], soc, max_coarse, max_levels, cap, Ps[f], Bs[f], s);
    return;
  }
  HIPCHECK(hipStreamSynchronize(s));
  int device = 0;
  HIPCHECK(hipGetDevice(&device));
  std::vector<std::future<void>> jobs;
  for (size_t f = 0; f < nf; ++f)
    jobs.push_back(std::async(std::launch::async, [&, f] {
      HIPCHECK(hipSetDevice(device));
      hipStream_t st = nullptr;
      HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      try {
        device_sa_field(A[f], soc, max_coarse, max_levels, cap, Ps[f], Bs[f], st);
      } catch (...) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        throw;
      }
      HIPCHECK(hipStreamDestroy(st));
    }));
  for (auto& j : jobs) j.wait();
  for (auto& j : jobs) j.get();  // rethrows the first field's error, if any
}

// The Galerkin products of the level operators (Algorithm 1),
// K_{l+1} = P_l^T (K_l P_l), on the device: each K_l stays there for the next
// product, and the host receives every K_{l+1} (the patch extraction and the
// level uploads read it).  The kernels of the per-field products, so the
// host's bits.
struct DeviceGalerkin {
  hipStream_t s = nullptr;
  int cap = 0;
  std::unique_ptr<DevArena> ar;  // holds K
  SaMat K;
  Csr next(const Csr& P, const Csr& Kh) {
    if (!ar) {
      ar = std::make_unique<DevArena>();
      K = sa_upload(Kh, *ar, s);
    }
    DevArena lv;  // this product's work memory
    const SaMat Pd = sa_upload(P, lv, s);
    const SaMat AP = sa_spgemm(K, Pd, cap, lv, lv, s);
    const SaMat Pt = sa_transpose(Pd, true, lv, lv, s);
    auto nar = std::make_unique<DevArena>();
    const SaMat Kc = sa_spgemm(Pt, AP, cap, *nar, lv, s);
    Csr out = sa_download(Kc, s);  // synchronises the stream
    K = Kc;
    ar = std::move(nar);
    return out;
  }
};

// dense inverse of an n x n FP64 matrix on the device (Gauss-Jordan, partial pivoting)
void dense_inverse(DevArena& ar, double* A, int n, hipStream_t s) {
  TempScope tmp(ar);
  double* rowk = tmp.alloc<double>(n);
  double* colk = tmp.alloc<double>(n);
  int* perm = tmp.alloc<int>(n);
  int* flag = tmp.alloc<int>(1);
  if (ar.dry()) return;
  HIPCHECK(hipMemsetAsync(flag, 0, sizeof(int), s));
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, n, k, A, perm, flag);
    hipLaunchKernelGGL(k_gj_save, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, k, A, rowk, colk);
    hipLaunchKernelGGL(k_gj_step, dim3(blocks_for((int64_t)n * n, 256)), dim3(256), 0, s, n, k, A, rowk, colk);
  }
  for (int k = n - 1; k >= 0; --k)
    hipLaunchKernelGGL(k_gj_colswap, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, k, perm, A);
  launch_check();
  int hflag = 0;
  HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hflag) throw MasError(MAS_ESINGULAR_PATCH, "coarsest-level operator is singular");
}

// Patch shapes of a level that get thread-per-patch buckets: listed fast
// shapes held at least bucket_min times.
static bool has_buckets(const PatchSet& ps, const mas_params& par) {
  std::map<std::array<int, 4>, int64_t> cnt;
  for (int64_t p = 0; p < ps.np(); ++p) {
    const int32_t* q = &ps.dims[4 * p];
    if (is_fast_shape(q)) cnt[{q[0], q[1], q[2], q[3]}]++;
  }
  for (auto& kv : cnt)
    if (kv.second >= std::max<int64_t>(1, par.bucket_min)) return true;
  return false;
}

// Record layout of a level's patch factors.  Identical component blocks
// (found by the host analysis) are stored once.  Levels of very large patches
// without buckets keep full blocks: twice the values of the packed triangle,
// but every row sweep of the patch kernels reads them with consecutive
// addresses across threads.
static int patch_layout(const PatchSet& ps, bool buckets, const mas_params& par) {
  int layout = ps.shared ? LAYOUT_SHARED : 0;
  if (!buckets && ps.max_m >= std::max(1, par.full_patch_min)) layout |= LAYOUT_FULL;
  return layout;
}

template <typename T>
void build_patches(DevArena& ar, Level<T>& L, const PatchSet& ps, const DCsr<double>& K64, int level, int nr_max,
                   const mas_params& par, hipStream_t s) {
  DPatches<T>& d = L.pt;
  const int64_t np = ps.np();
  d.np = np;
  d.ndofs = (int64_t)ps.dofs.size();
  d.max_m = ps.max_m;
  d.max_f = ps.max_f;
  for (int64_t p = 0; p < np; ++p)
    if (ps.dims[4 * p + 3] > MAX_NS || ps.dims[4 * p + 3] < 1) throw MasError(MAS_EINVAL, "patch seed count out of range");
  // ---- order: fast buckets (one per shape, at least 64 patches) first, then the rest
  std::vector<std::vector<int64_t>> groups;
  std::vector<std::array<int, 4>> gshape;
  std::vector<int64_t> generic;
  {
    std::vector<int64_t> cnt_idx;
    std::map<std::array<int, 4>, std::vector<int64_t>> by;
    for (int64_t p = 0; p < np; ++p) {
      const int32_t* q = &ps.dims[4 * p];
      if (is_fast_shape(q)) by[{q[0], q[1], q[2], q[3]}].push_back(p);
      else generic.push_back(p);
    }
    const int64_t min_bucket = std::max<int64_t>(1, par.bucket_min);
    for (auto& kv : by) {
      if ((int64_t)kv.second.size() >= min_bucket) {
        gshape.push_back(kv.first);
        groups.push_back(kv.second);
      } else {
        generic.insert(generic.end(), kv.second.begin(), kv.second.end());
      }
    }
    std::sort(generic.begin(), generic.end());
  }
  const int layout = patch_layout(ps, !groups.empty(), par);
  d.layout = layout;
  std::vector<int64_t> order;
  for (auto& g : groups) order.insert(order.end(), g.begin(), g.end());
  const int64_t g0 = (int64_t)order.size();
  order.insert(order.end(), generic.begin(), generic.end());
  // ---- arrays in the new order
  std::vector<int64_t> off(np + 1, 0), foff(np), fstr(np);
  std::vector<int32_t> dims(4 * np), dofs;
  dofs.reserve(ps.dofs.size());
  std::vector<int64_t> ypos;  // output position of every (patch, slot), in the order of dofs
  ypos.reserve(ps.dofs.size());
  int64_t fcur = 0, ycur = 0;
  d.fast.clear();
  int64_t pnew = 0;
  for (size_t b = 0; b < groups.size(); ++b) {
    FastBucket fb;
    for (int c = 0; c < 4; ++c) fb.shape[c] = gshape[b][c];
    fb.P = (int64_t)groups[b].size();
    fb.Ppad = (fb.P + 63) / 64 * 64;
    const int M = fb.shape[0] + fb.shape[1] + fb.shape[2] + fb.shape[3];
    const int64_t F = record_entries(fb.shape[0], fb.shape[1], fb.shape[2], fb.shape[3], layout);
    fb.fbase = fcur;
    fb.ybase = ycur;
    // interleaved across the bucket: element q of patch i at q * Ppad + i
    std::vector<int32_t> il((size_t)M * fb.Ppad, 0);
    for (int64_t i = 0; i < fb.P; ++i, ++pnew) {
      const int64_t p = groups[b][i];
      for (int c = 0; c < 4; ++c) dims[4 * pnew + c] = ps.dims[4 * p + c];
      foff[pnew] = fcur + i;
      fstr[pnew] = fb.Ppad;
      for (int k = 0; k < M; ++k) {
        const int32_t j = ps.dofs[ps.off[p] + k];
        dofs.push_back(j);
        ypos.push_back(ycur + (int64_t)k * fb.Ppad + i);
        il[(size_t)k * fb.Ppad + i] = j;
      }
      off[pnew + 1] = (int64_t)dofs.size();
    }
    fb.dofs = ar.upload<int>(il, s);
    fcur += F * fb.Ppad;
    ycur += (int64_t)M * fb.Ppad;
    d.fast.push_back(fb);
  }
  d.g0 = g0;
  d.yshift = (int64_t)dofs.size() - ycur;  // generic outputs follow the fast buckets in Y
  for (int64_t p : generic) {
    for (int c = 0; c < 4; ++c) dims[4 * pnew + c] = ps.dims[4 * p + c];
    foff[pnew] = fcur;
    fstr[pnew] = 1;
    const int32_t* q = &ps.dims[4 * p];
    fcur += record_entries(q[0], q[1], q[2], q[3], layout);
    for (int64_t k = ps.off[p]; k < ps.off[p + 1]; ++k) {
      ypos.push_back(ycur);
      ++ycur;
      dofs.push_back(ps.dofs[k]);
    }
    off[pnew + 1] = (int64_t)dofs.size();
    ++pnew;
  }
  d.nfac = fcur;
  // stored values without the buckets' padding, and the longest record
  d.nfac_alg = 0;
  d.max_f = 0;
  for (int64_t p = 0; p < np; ++p) {
    const int32_t* q = &ps.dims[4 * p];
    const int64_t rec = record_entries(q[0], q[1], q[2], q[3], layout);
    d.nfac_alg += rec;
    d.max_f = std::max(d.max_f, rec);
  }
  // the column-streaming kernel takes packed, per-component blocks of at most 2 x 64 rows
  d.col_ok = layout == 0 && !generic.empty();
  for (int64_t p : generic)
    for (int c = 0; c < 3; ++c) d.col_ok = d.col_ok && ps.dims[4 * p + c] <= 2 * WAVE;
  // shared blocks, workgroup kernel: where the partial row sums of a patch's
  // thread groups (G = TPB / n groups) fit in the LDS copy of its block
  d.parts_fit[0] = d.parts_fit[1] = d.parts_fit[2] = true;
  if (layout & LAYOUT_SHARED)
    for (int64_t p : generic) {
      const int32_t* q = &ps.dims[4 * p];
      const int64_t nvp = q[0] + q[1] + q[2];
      const int tbs[3] = {WAVE, 128, 256};
      for (int k = 0; k < 3; ++k) {
        const int64_t G = q[0] >= tbs[k] ? 1 : tbs[k] / q[0];
        if ((G - 1) * nvp > blk_size(q[0], layout & LAYOUT_FULL)) d.parts_fit[k] = false;
      }
    }
  // the persistent pipelined kernel: staged records of at most 16 values per
  // thread, at most 4 DoFs per thread
  {
    const int tbp = ps.max_m >= kWidePatch ? 256 : WAVE;
    const int spp = (layout & LAYOUT_SHARED) && !d.parts_fit[tbp == 256 ? 2 : 0] ? 3 * tbp : 0;
    d.pipe_ok = !generic.empty() && d.max_f <= 16 * tbp && ps.max_m <= 4 * tbp &&
                (size_t)(2 * ps.max_m + spp + d.max_f) * sizeof(T) <= kMaxLds;
  }
  // the panel kernel: packed shared blocks of at most kPanelTpb rows, records too large to stage
  {
    int maxn = 0;
    for (int64_t p : generic) maxn = std::max(maxn, (int)ps.dims[4 * p]);
    const int tbs = ps.max_m >= kWidePatch ? 256 : WAVE;
    const bool stageable = (size_t)(2 * ps.max_m + 3 * tbs + d.max_f) * sizeof(T) <= kMaxLds;
    d.panel_ok = layout == LAYOUT_SHARED && !generic.empty() && maxn <= kPanelTpb &&
                 (ps.dim == 2 || ps.dim == 3) && (size_t)2 * ps.max_m * sizeof(T) + kPanelBytes <= kMaxLds;
    d.panel_auto = d.panel_ok && !stageable;
  }
  // the shared-block wavefront kernel: packed shared blocks of at most 2 x 64 rows
  d.wave_tt = 0;
  if (layout == LAYOUT_SHARED && !generic.empty()) {
    int maxn = 0;
    for (int64_t p : generic) maxn = std::max(maxn, (int)ps.dims[4 * p]);
    const int tt = (maxn + WAVE - 1) / WAVE;
    if (tt <= 2 && (ps.dim == 2 || ps.dim == 3) && (size_t)kWavePb * 2 * ps.max_m * sizeof(T) <= kMaxLds)
      d.wave_tt = tt;
  }
  if (layout & LAYOUT_SHARED) d.nco = ps.dim;

  d.stream = (double)d.nfac * sizeof(T) >= kStreamBytes;

  d.ny = ycur;
  // ---- DoF -> output positions, in patch order (deterministic sums)
  const int64_t n = L.n;
  std::vector<int32_t> cnt(n, 0);
  for (int32_t j : dofs) cnt[j]++;
  std::vector<int32_t> iptr(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) iptr[j + 1] = iptr[j] + cnt[j];
  std::vector<int32_t> ipos(dofs.size());
  std::vector<int32_t> fillp(iptr.begin(), iptr.end() - 1);
  for (size_t k = 0; k < dofs.size(); ++k) ipos[fillp[dofs[k]]++] = (int32_t)ypos[k];
  int width = 0;
  for (int64_t j = 0; j < n; ++j) width = std::max(width, cnt[j]);
  const double avg = n ? (double)dofs.size() / (double)n : 1.0;
  if (width <= 16 && width <= 2.5 * avg + 1) {
    std::vector<int32_t> ell((size_t)width * n, -1);
    for (int64_t j = 0; j < n; ++j)
      for (int32_t q = iptr[j]; q < iptr[j + 1]; ++q) ell[(size_t)(q - iptr[j]) * n + j] = ipos[q];
    d.ell = ar.upload<int>(ell, s);
    d.ell_width = width;
  } else {
    d.inv_ptr = ar.upload<int>(iptr, s);
    d.inv_pos = ar.upload<int>(ipos, s);
    std::vector<double> w(n, 0.0);
    for (int64_t j = 0; j < n; ++j)
      if (cnt[j] > 0) w[j] = 1.0 / (double)cnt[j];
    d.w = ar.upload<T>(w, s);
  }
  if (nr_max > 1) {
    // batched path: outputs at (off[p] + slot) * nr + k
    std::vector<int32_t> cpos(dofs.size());
    std::vector<int32_t> fillc(iptr.begin(), iptr.end() - 1);
    for (size_t q = 0; q < dofs.size(); ++q) cpos[fillc[dofs[q]]++] = (int32_t)q;
    if (d.ell) {
      std::vector<int32_t> ellc((size_t)width * n, -1);
      for (int64_t j = 0; j < n; ++j)
        for (int32_t q = iptr[j]; q < iptr[j + 1]; ++q) ellc[(size_t)(q - iptr[j]) * n + j] = cpos[q];
      d.ell_c = ar.upload<int>(ellc, s);
    } else {
      d.inv_ptr_c = d.inv_ptr;
      d.inv_pos_c = ar.upload<int>(cpos, s);
    }
    d.Ynr = ar.alloc<T>((size_t)d.ndofs * nr_max);
    // right-hand sides per workgroup (a power of two from kNrKT to 64) of the
    // batched kernel: its m x C block must fit in LDS.  The factor record is
    // staged too when that still leaves room for min(16, nr_max) of them.
    auto max_c = [&](int64_t f) {
      int c = 0;
      for (int t = kNrKT; t <= 64; t *= 2)
        if (nr_lds_bytes<T>(d.max_m, t, f) <= kMaxLds) c = t;
      return c;
    };
    const int want = std::min(16, std::max(kNrKT, nr_max));
    const int c_stage = max_c(d.max_f), c_plain = max_c(0);
    d.nr_stage = c_stage >= want;
    d.nr_chunk = d.nr_stage ? c_stage : c_plain;
  }
  d.off = ar.upload<int64_t>(off, s);
  {
    int4* dd = ar.alloc<int4>(np);
    if (!ar.dry()) {
      HIPCHECK(hipMemcpyAsync(dd, dims.data(), dims.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
    d.dims = dd;
  }
  d.foff = ar.upload<int64_t>(foff, s);
  d.fstride = ar.upload<int64_t>(fstr, s);
  d.dofs = ar.upload<int>(dofs, s);
  d.Y = ar.alloc<T>(d.ny);
  d.fac = ar.alloc<T>(d.nfac);
  // ---- FP64 factorisation on the GPU
  int max_nc = 0, max_nv = 0;
  for (int64_t p = 0; p < np; ++p) {
    const int32_t* q = &ps.dims[4 * p];
    max_nc = std::max({max_nc, q[0], q[1], q[2]});
    max_nv = std::max(max_nv, q[0] + q[1] + q[2]);
  }
  const int64_t stride = (int64_t)max_nc * max_nc + 2 * (int64_t)max_nv * MAX_NS;
  const size_t lds_bytes = (size_t)stride * sizeof(double);
  TempScope work(ar);  // factorisation work areas, released at the end of this level
  int64_t* bad = work.alloc<int64_t>(1);
  int64_t init = INT64_MAX;
  const bool use_lds = lds_bytes <= kMaxLds;
  const unsigned grid = use_lds ? (unsigned)std::min<int64_t>(np, 65536) : (unsigned)std::min<int64_t>(np, 1024);
  double* gwork = use_lds ? nullptr : work.alloc<double>((size_t)stride * grid);
  if (ar.dry()) return;
  HIPCHECK(hipMemcpyAsync(bad, &init, sizeof(int64_t), hipMemcpyHostToDevice, s));
  // 4 (blocks in LDS) or 16 (blocks in global memory) wavefronts per patch: the
  // row updates of a Gauss-Jordan step are split between them
  if (use_lds)
    hipLaunchKernelGGL((k_vanka_factor<T, 256>), dim3(grid), dim3(256), lds_bytes, s, np, d.off, d.dims, d.foff,
                       d.fstride, d.dofs, K64.ptr, K64.ind, K64.val, d.fac, gwork, stride, 1, max_nv, 1e-14, bad,
                       d.layout);
  else {
    // blocks in global memory: blocked Gauss-Jordan with LDS panels when they fit
    const size_t panel = (size_t)(kGjBlock * kGjBlock + 2 * kGjBlock * max_nc) * sizeof(double);
    int dev = 0, max_lds = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const bool blocked = panel <= (size_t)max_lds && par.factor_blocked != 0;
    hipLaunchKernelGGL((k_vanka_factor<T, 1024>), dim3(grid), dim3(1024), blocked ? panel : 0, s, np, d.off, d.dims,
                       d.foff, d.fstride, d.dofs, K64.ptr, K64.ind, K64.val, d.fac, gwork, stride, blocked ? 2 : 0,
                       max_nv, 1e-14, bad, d.layout);
  }
  launch_check();
  int64_t hbad = 0;
  HIPCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hbad != INT64_MAX) {
    const int64_t orig = order[hbad];
    throw MasError(MAS_ESINGULAR_PATCH,
                   "singular patch block on level " + std::to_string(level) + ", patch " + std::to_string(orig));
  }
}

template <typename T>
std::unique_ptr<Cycle<T>> build_cycle(mas_handle* h, const std::vector<Csr>& Ks, const std::vector<Csr>& Ps,
                                      const std::vector<std::vector<int8_t>>& fields,
                                      const std::vector<PatchSet>& patches, const std::vector<HostDlsc>& dlsc,
                                      const std::vector<bool>& relax,
                                      const Csr& Kc_bordered, const std::vector<int64_t>& free0,
                                      const std::vector<int64_t>& dir0, hipStream_t s) {
  DevArena& ar = h->arena;
  SetupTrace tr;
  const bool tune = h->par.autotune != 0 && !ar.dry();
  auto cyc = std::make_unique<Cycle<T>>();
  cyc->par = h->par;
  cyc->dim = h->dim;
  cyc->nr_max = std::max(1, h->par.nrhs_max);
  cyc->tm = &h->tm;
  const size_t nl = Ks.size();
  cyc->lev.resize(nl);
  for (size_t l = 0; l < nl; ++l) {
    Level<T>& L = cyc->lev[l];
    L.n = Ks[l].nr;
    L.nvel = 0;
    for (int8_t f : fields[l]) L.nvel += (f < h->dim);
    L.relax = relax[l];
    L.x = ar.alloc<T>((size_t)L.n * cyc->nr_max);
    L.b = ar.alloc<T>((size_t)L.n * cyc->nr_max);
    L.r = ar.alloc<T>((size_t)L.n * cyc->nr_max);
    if (l + 1 < nl) {
      L.K = upload_csr<T>(ar, Ks[l], s);
      // the residual product of a Vanka level reads K once per relaxation
      L.K.stream = L.relax && dlsc[l].A.nr == 0 && (double)L.K.nnz * (sizeof(T) + 4) >= kStreamBytes;
      if (l >= 1) {
        L.P = upload_csr<T>(ar, Ps[l], s);
        L.R = upload_csr<T>(ar, transpose(Ps[l]), s);
      }
      if (tr.on && !ar.dry()) HIPCHECK(hipStreamSynchronize(s));
      tr.mark("device: level " + std::to_string(l) + " operators");
      if (L.relax && !patches[l].off.empty()) {
        if constexpr (std::is_same<T, double>::value) {
          build_patches<T>(ar, L, patches[l], L.K, (int)l, cyc->nr_max, h->par, s);
        } else {  // the FP64 operator lives only while the patches are factorised
          TempScope tmp(ar);
          const DCsr<double> K64 = upload_csr_plain<double>(tmp, Ks[l], s);
          build_patches<T>(ar, L, patches[l], K64, (int)l, cyc->nr_max, h->par, s);
        }
        tr.mark("device: level " + std::to_string(l) + " patches");
      }
      if (L.relax && dlsc[l].A.nr > 0) {
        const HostDlsc& H = dlsc[l];
        DDlsc<T>& D = L.dl;
        D.on = true;
        D.nv = H.A.nr;
        D.np = H.B.nr;
        D.A = upload_csr<T>(ar, H.A, s);
        D.B = upload_csr<T>(ar, H.B, s);
        D.Bt = upload_csr<T>(ar, H.Bt, s);
        D.S = upload_csr<T>(ar, H.S, s);
        D.minv = ar.upload<T>(H.minv, s);
        D.lamA = H.lamA;
        D.lamS = H.lamS;
        const int64_t R = cyc->nr_max;
        for (T** v : {&D.ru, &D.vs, &D.tmp, &D.t1, &D.t2}) *v = ar.alloc<T>(D.nv * R);
        for (T** v : {&D.rp, &D.q, &D.dp}) *v = ar.alloc<T>(D.np * R);
        D.cd = ar.alloc<T>(std::max(D.nv, D.np) * R);
        D.cd2 = ar.alloc<T>(std::max(D.nv, D.np) * R);
        D.cres = ar.alloc<T>(std::max(D.nv, D.np) * R);
        if (!H.Sk.empty()) {
          D.sh.resize(H.Sk.size());
          for (size_t k = 0; k < H.Sk.size(); ++k) {
            auto& Lk = D.sh[k];
            Lk.n = H.Sk[k].nr;
            Lk.x = ar.alloc<T>(Lk.n * R);
            Lk.b = ar.alloc<T>(Lk.n * R);
            if (k + 1 == H.Sk.size()) break;
            Lk.S = upload_csr<T>(ar, H.Sk[k], s);
            Lk.P = upload_csr<T>(ar, H.Pk[k], s);
            Lk.R = upload_csr<T>(ar, transpose(H.Pk[k]), s);
            Lk.wdinv = ar.upload<T>(H.wdinv[k], s);
            for (T** v : {&Lk.res, &Lk.d1, &Lk.d2, &Lk.corr}) *v = ar.alloc<T>(Lk.n * R);
          }
          D.sinv = ar.upload<double>(H.sc_dense, s);
          dense_inverse(ar, D.sinv, (int)H.sc_ld, s);
          D.sld = H.sc_ld;
        }
      }
    }
  }
  if (tr.on && !ar.dry()) HIPCHECK(hipStreamSynchronize(s));
  tr.mark("device: levels, factorisation");
  // relaxation wrapper (Section 3.3.1): every Vanka level except the Scott-Vogelius K0
  if (h->par.krylov_its > 0) {
    const int m = h->par.krylov_its;
    int64_t nmax = 0;
    for (size_t l = 0; l + 1 < nl; ++l) {
      Level<T>& L = cyc->lev[l];
      L.krylov = L.relax && !L.dl.on && L.pt.np > 0 && !(h->disc == MAS_SV && l == 0);
      if (L.krylov) nmax = std::max(nmax, L.n);
    }
    if (nmax > 0) {
      cyc->kv = ar.alloc<T>((size_t)(m + 1) * nmax);
      cyc->kz = ar.alloc<T>((size_t)m * nmax);
      cyc->kw = ar.alloc<T>((size_t)nmax);
      cyc->kpart = ar.alloc<double>((size_t)2 * cyc->kblk);
      cyc->kh = ar.alloc<double>((size_t)(m + 1) * m);
      cyc->kbeta = ar.alloc<double>(1);
      cyc->ky = ar.alloc<double>((size_t)m);
    }
  }
  // lanes per row of every sparse product, timed on the operands
  for (size_t l = 0; l + 1 < nl; ++l) {
    Level<T>& L = cyc->lev[l];
    autotune_team<T>(L.K, L.x, L.r, s, tune);
    if (L.relax && L.pt.np > 0) cyc->choose_generic_kernel(L, tune, s);
    if (L.dl.on) {
      autotune_team<T>(L.dl.A, L.dl.ru, L.dl.vs, s, tune);
      autotune_team<T>(L.dl.S, L.dl.rp, L.dl.q, s, tune);
      autotune_team<T>(L.dl.B, L.dl.ru, L.dl.rp, s, tune);
      autotune_team<T>(L.dl.Bt, L.dl.rp, L.dl.ru, s, tune);
      for (size_t k = 0; k + 1 < L.dl.sh.size(); ++k) {
        auto& Sl = L.dl.sh[k];
        autotune_team<T>(Sl.S, Sl.x, Sl.res, s, tune);
        autotune_team<T>(Sl.R, Sl.res, L.dl.sh[k + 1].b, s, tune);
        autotune_team<T>(Sl.P, L.dl.sh[k + 1].x, Sl.x, s, tune);
      }
    }
    if (l >= 1) {
      Level<T>& C = cyc->lev[l + 1];
      autotune_team<T>(L.R, L.r, C.b, s, tune);
      autotune_team<T>(L.P, C.x, L.x, s, tune);
    }
  }
  if (tr.on && !ar.dry()) HIPCHECK(hipStreamSynchronize(s));
  tr.mark("device: product autotune");
  // coarsest: dense inverse of the bordered operator
  const int64_t nb = Kc_bordered.nr;
  std::vector<double> dense((size_t)nb * nb, 0.0);
  for (int64_t i = 0; i < nb; ++i)
    for (int64_t e = Kc_bordered.ptr[i]; e < Kc_bordered.ptr[i + 1]; ++e) dense[i * nb + Kc_bordered.ind[e]] = Kc_bordered.val[e];
  cyc->Cinv = ar.upload<double>(dense, s);
  dense_inverse(ar, cyc->Cinv, (int)nb, s);
  tr.mark("device: coarsest inverse");
  cyc->ld = nb;
  cyc->nc_dense = nb;
  cyc->free0 = ar.upload<int64_t>(free0, s);
  cyc->dir0 = ar.upload<int64_t>(dir0, s);
  cyc->nfree0 = (int64_t)free0.size();
  cyc->ndir0 = (int64_t)dir0.size();
  const HostPlan& pl = h->plan;
  if (pl.sv) {
    cyc->sv = true;
    cyc->np0 = pl.Mdg.nr;
    cyc->np1 = pl.Mcg.nr;
    cyc->Mdg = upload_csr<T>(ar, pl.Mdg, s);
    cyc->P0t = upload_csr<T>(ar, pl.P0t, s);
    cyc->P0p = upload_csr<T>(ar, pl.P0p, s);
    cyc->Mcg = upload_csr<T>(ar, pl.Mcg, s);
    cyc->mcg_dinv = ar.upload<T>(pl.mcg_dinv, s);
    cyc->mass_steps = pl.mass_steps;
    const int64_t R = cyc->nr_max;
    cyc->sv_t0 = ar.alloc<T>(cyc->np0 * R);
    cyc->sv_t1 = ar.alloc<T>(cyc->np1 * R);
    cyc->sv_z = ar.alloc<T>(cyc->np1 * R);
    cyc->sv_cd = ar.alloc<T>(cyc->np1 * R);
    cyc->sv_cd2 = ar.alloc<T>(cyc->np1 * R);
    cyc->sv_cres = ar.alloc<T>(cyc->np1 * R);
    for (DCsr<T>* A : {&cyc->Mdg, &cyc->P0t, &cyc->P0p, &cyc->Mcg}) A->use_sell = false;
  }
  return cyc;
}

// The smoothed-aggregation hierarchy of S for the DLSC AMG stages (Section 5):
// Algorithm 1's scalar SA on S, Galerkin products, Jacobi weight (4/3) / rho
// with rho = max_i sum_j |s_ij| / s_ii per level, and the coarsest operator as
// a dense matrix, bordered with its near-null vector when S is singular.
void s_hierarchy(HostDlsc& D, const mas_params& par, bool singular) {
  std::vector<std::vector<double>> Bs;
  sa_field(D.S, soc_params(par), par.max_coarse, par.max_levels, D.Pk, Bs);
  D.Sk.assign(1, D.S);
  for (const Csr& P : D.Pk) D.Sk.push_back(galerkin(P, D.Sk.back()));
  D.wdinv.clear();
  for (size_t k = 0; k + 1 < D.Sk.size(); ++k) {
    const Csr& A = D.Sk[k];
    std::vector<double> d(A.nr, 0.0), w(A.nr);
    double rho = 0.0;
    for (int64_t i = 0; i < A.nr; ++i) {
      double sum = 0.0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        sum += std::fabs(A.val[e]);
        if (A.ind[e] == i) d[i] = A.val[e];
      }
      if (!(d[i] > 0.0)) throw MasError(MAS_EINVAL, "B M^-1 B^T has a non-positive diagonal entry");
      rho = std::max(rho, sum / d[i]);
    }
    for (int64_t i = 0; i < A.nr; ++i) w[i] = (4.0 / 3.0) / rho / d[i];
    D.wdinv.push_back(std::move(w));
  }
  const Csr& C = D.Sk.back();
  const int64_t m = C.nr, ld = singular ? m + 1 : m;
  check_dense_coarse(ld, par.max_coarse, "B M^-1 B^T of the DLSC AMG stages");
  D.sc_ld = ld;
  D.sc_dense.assign((size_t)ld * ld, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t e = C.ptr[i]; e < C.ptr[i + 1]; ++e) D.sc_dense[i * ld + C.ind[e]] = C.val[e];
  if (singular) {
    const std::vector<double>& nv = Bs.back();
    double nn = 0.0;
    for (double v : nv) nn += v * v;
    nn = std::sqrt(nn);
    for (int64_t i = 0; i < m; ++i) {
      D.sc_dense[i * ld + m] = nv[i] / nn;
      D.sc_dense[m * ld + i] = nv[i] / nn;
    }
  }
}

// dev: a device may be used (mas_setup; stream s).  With device_sa the
// per-field smoothed aggregation, and with device_galerkin the Galerkin
// products of the level operators, then run on it, with the same results as
// the host's, bit for bit; mas_analyze runs both on the host.
void analyze_impl(mas_handle* h, const mas_problem* pr, bool dev = false, hipStream_t s = nullptr) {
  SetupTrace tr;
  const bool dev_sa = dev && h->par.device_sa != 0;
  dev = dev && h->par.device_galerkin != 0;
  const int d = pr->dim;
  if (d != 2 && d != 3) throw MasError(MAS_EINVAL, "dim must be 2 or 3");
  if (pr->disc != MAS_TH && pr->disc != MAS_SV) throw MasError(MAS_EINVAL, "unknown discretisation");
  if (pr->disc == MAS_SV && d != 2) throw MasError(MAS_EINVAL, "Scott-Vogelius is supported in 2D");
  h->dim = d;
  h->disc = pr->disc;
  const mas_params& par = h->par;
  if (par.relax != MAS_RELAX_VANKA && par.relax != MAS_RELAX_DLSC && par.relax != MAS_RELAX_VANKA_DLSC)
    throw MasError(MAS_EINVAL, "unknown relaxation");
  for (int q = 0; q < 3; ++q)
    if (par.relax != MAS_RELAX_VANKA && par.cheb_deg[q] < 1) throw MasError(MAS_EINVAL, "Chebyshev degrees must be >= 1");
  if (par.relax == MAS_RELAX_VANKA_DLSC && (par.nu_dlsc < 0 || par.nu_dlsc > 16))
    throw MasError(MAS_EINVAL, "nu_dlsc must be in [0, 16]");
  if (par.dlsc_amg < 0 || par.dlsc_amg > 8) throw MasError(MAS_EINVAL, "dlsc_amg must be in [0, 8]");
  if (par.schedule < MAS_DC_ALL || par.schedule > MAS_HO_AMG) throw MasError(MAS_EINVAL, "unknown schedule");
  // HO-AMG (the remark after Algorithm 1): the hierarchy is built from K0 itself
  const bool ho = par.schedule == MAS_HO_AMG;
  if (ho && pr->disc != MAS_TH) throw MasError(MAS_EINVAL, "HO-AMG is supported for Taylor-Hood only");
  if (ho) {  // no defect-correction level: b1 = r0 exactly
    h->par.eta_u = 1.0;
    h->par.eta_p = 1.0;
  }
  Csr K0 = get_csr(pr->K0, "K0");
  Csr K1 = ho ? K0 : get_csr(pr->K1, "K1");
  const int8_t* field1 = ho ? pr->field0 : pr->field1;
  const uint8_t* dir1 = ho ? pr->dir0 : pr->dir1;
  Csr Ap = get_csr(pr->Ap, "Ap");
  const int64_t n0 = K0.nr, n1 = K1.nr;
  if (K0.nc != n0 || K1.nc != n1 || Ap.nr != Ap.nc) throw MasError(MAS_EINVAL, "operators must be square");
  if (!pr->field0 || !field1 || !pr->dir0 || !dir1) throw MasError(MAS_EINVAL, "missing field or Dirichlet map");
  h->n0 = n0;
  if (par.restart < 1 || par.restart > 200) throw MasError(MAS_EINVAL, "restart must be in [1, 200]");
  if (par.nrhs_max < 1 || par.nrhs_max > 64) throw MasError(MAS_EINVAL, "nrhs_max must be in [1, 64]");
  if (par.krylov_its < 0 || par.krylov_its > 8) throw MasError(MAS_EINVAL, "krylov_its must be in [0, 8]");
  if (par.max_coarse < 1 || par.max_levels < 1) throw MasError(MAS_EINVAL, "bad coarsening limits");
  if (par.soc != MAS_SOC_EVOLUTION && par.soc != MAS_SOC_SYMMETRIC) throw MasError(MAS_EINVAL, "unknown soc");
  if (!(par.soc_eps > 0.0) || !std::isfinite(par.soc_eps)) throw MasError(MAS_EINVAL, "soc_eps must be positive");
  if (par.gram_schmidt != MAS_GS_CLASSICAL && par.gram_schmidt != MAS_GS_MODIFIED)
    throw MasError(MAS_EINVAL, "unknown gram_schmidt");
  if (par.full_patch_min < 1 || par.bucket_min < 1) throw MasError(MAS_EINVAL, "full_patch_min and bucket_min must be >= 1");
  if (par.patch_kernel < 0 || par.patch_kernel > 5) throw MasError(MAS_EINVAL, "patch_kernel must be 0..5");
  if (par.device_sa != 0 && par.device_sa != 1) throw MasError(MAS_EINVAL, "device_sa must be 0 or 1");
  if (par.spgemm_cap < 0) throw MasError(MAS_EINVAL, "spgemm_cap must be >= 0");
  std::vector<int64_t> free0, dir0, free1;
  std::vector<int8_t> f0, f1;
  int64_t nu0 = 0, np0 = 0;
  for (int64_t i = 0; i < n0; ++i) {
    if (pr->field0[i] < 0 || pr->field0[i] > d) throw MasError(MAS_EINVAL, "field0 out of range");
    if (i > 0 && pr->field0[i] < pr->field0[i - 1]) throw MasError(MAS_EINVAL, "K0 unknowns must be field-blocked");
    if (pr->field0[i] < d) ++nu0; else ++np0;
    if (pr->dir0[i]) {
      if (pr->field0[i] == d) throw MasError(MAS_EINVAL, "Dirichlet pressure rows are not supported");
      dir0.push_back(i);
    } else {
      free0.push_back(i);
      f0.push_back(pr->field0[i]);
    }
  }
  for (int64_t i = 0; i < n1; ++i) {
    if (field1[i] < 0 || field1[i] > d) throw MasError(MAS_EINVAL, "field1 out of range");
    if (i > 0 && field1[i] < field1[i - 1]) throw MasError(MAS_EINVAL, "K1 unknowns must be field-blocked");
    if (!dir1[i]) {
      free1.push_back(i);
      f1.push_back(field1[i]);
    }
  }
  h->nu0 = nu0;
  Csr K0f = submatrix(K0, free0, free0);
  Csr K1f = submatrix(K1, free1, free1);
  tr.mark("validation, free blocks");
  // the two velocity spaces share their nodes (Section 3.1)
  int64_t nv0 = 0, nv1 = 0;
  for (auto f : f0) nv0 += (f < d);
  for (auto f : f1) nv1 += (f < d);
  if (nv0 != nv1) throw MasError(MAS_EINVAL, "K0 and K1 must share their free velocity DoFs");
  if (pr->disc == MAS_TH && (int64_t)free0.size() != (int64_t)free1.size())
    throw MasError(MAS_EINVAL, "K0 and K1 free DoFs must coincide for Taylor-Hood");
  // ---- Algorithm 1: per-field smoothed aggregation on K1's velocity blocks and A_p
  std::vector<std::vector<int64_t>> blocks(d + 1);
  for (int64_t i = 0; i < (int64_t)f1.size(); ++i) blocks[f1[i]].push_back(i);
  if ((int64_t)blocks[d].size() != Ap.nr) throw MasError(MAS_EINVAL, "Ap size does not match K1's pressure block");
  std::vector<std::vector<Csr>> fP;
  std::vector<std::vector<std::vector<double>>> fB;
  if (pr->n_prebuilt > 0) {
    // a hierarchy built elsewhere: the per-field interpolations replace the
    // smoothed aggregation; only the coarsest pressure near-null vector is read
    if (!pr->prebuilt_P) throw MasError(MAS_EINVAL, "n_prebuilt > 0 needs prebuilt_P");
    const int L = pr->n_prebuilt;
    if (L + 1 > 16) throw MasError(MAS_EINVAL, "too many prebuilt levels");
    fP.assign(d + 1, {});
    fB.assign(d + 1, {});
    for (int f = 0; f <= d; ++f) {
      for (int l = 0; l < L; ++l) {
        Csr P = get_csr(pr->prebuilt_P[(size_t)l * (d + 1) + f], "prebuilt_P");
        const int64_t rows = l == 0 ? (int64_t)blocks[f].size() : fP[f][l - 1].nc;
        if (P.nr != rows || P.nc < 1 || P.nc > P.nr)
          throw MasError(MAS_EINVAL, "prebuilt_P[" + std::to_string(l * (d + 1) + f) + "] is " +
                                         std::to_string(P.nr) + " x " + std::to_string(P.nc) + "; it needs " +
                                         std::to_string(rows) + " rows (the field's DoFs of the finer level) and "
                                         "at most as many columns");
        fP[f].push_back(std::move(P));
      }
      fB[f].resize(L + 1);
    }
    if (pr->p_nullspace) {
      if (!pr->prebuilt_null_p) throw MasError(MAS_EINVAL, "prebuilt_null_p is required with p_nullspace");
      const int64_t nc = fP[d][L - 1].nc;
      fB[d][L].assign(pr->prebuilt_null_p, pr->prebuilt_null_p + nc);
      for (double v : fB[d][L])
        if (!std::isfinite(v)) throw MasError(MAS_EINVAL, "prebuilt_null_p has a non-finite entry");
    }
  } else {
    std::vector<Csr> Af;
    for (int f = 0; f <= d; ++f) Af.push_back((f < d) ? submatrix(K1f, blocks[f], blocks[f]) : Ap);
    if (dev_sa) {
      device_sa_fields(Af, soc_params(par), par.max_coarse, par.max_levels, par.spgemm_cap, fP, fB, s);
    } else {
      sa_fields(Af, soc_params(par), par.max_coarse, par.max_levels, fP, fB);
    }
  }
  size_t lmax = SIZE_MAX;
  for (int f = 0; f <= d; ++f) lmax = std::min(lmax, fP[f].size() + 1);
  tr.mark(dev_sa ? "smoothed aggregation (device)" : "smoothed aggregation");
  {
    // the coarsest level is the one after lmax - 1 coarsenings of every field
    // (a field that coarsened further is cut there), inverted densely with
    // its border
    int64_t nL = pr->p_nullspace ? 1 : 0;
    for (int f = 0; f <= d; ++f) nL += lmax >= 2 ? fP[f][lmax - 2].nc : (int64_t)blocks[f].size();
    check_dense_coarse(nL, par.max_coarse, "coarsest saddle operator");
  }
  // levels: 0 = K0f, 1 = K1f, 2.. = Galerkin
  std::vector<Csr> Ks;
  Ks.push_back(std::move(K0f));
  Ks.push_back(std::move(K1f));
  std::vector<Csr> Ps{Csr(), Csr()};
  std::vector<std::vector<int8_t>> fields{f0, f1};
  DeviceGalerkin dg;
  dg.s = s;
  dg.cap = par.spgemm_cap;
  for (size_t l = 0; l + 1 < lmax; ++l) {
    std::vector<const Csr*> bl;
    for (int f = 0; f <= d; ++f) bl.push_back(&fP[f][l]);
    Csr P = block_diag(bl);
    Csr Kc = dev ? dg.next(P, Ks.back()) : galerkin(P, Ks.back());
    std::vector<int8_t> fc;
    for (int f = 0; f <= d; ++f) fc.insert(fc.end(), (size_t)fP[f][l].nc, (int8_t)f);
    Ps.back() = P;  // P of the finer level
    Ks.push_back(std::move(Kc));
    Ps.push_back(Csr());
    fields.push_back(std::move(fc));
  }
  const size_t nl = Ks.size();  // includes the coarsest
  tr.mark(dev ? "Galerkin products (device)" : "Galerkin products");
  if (nl > 16) throw MasError(MAS_EINVAL, "too many levels");
  // relaxation schedule (Section 4): index 0 = K0, 1 = K1, ...
  std::vector<bool> relax(nl, true);
  relax[nl - 1] = false;
  if (par.schedule == MAS_DC_SKIP1 && nl > 2) relax[1] = false;
  if (par.schedule == MAS_DC_SKIP0 || ho) relax[0] = false;
  if (par.schedule == MAS_DC_SKIP1 && nl == 2) relax[1] = false;
  std::vector<PatchSet> patches(nl);
  std::vector<HostDlsc> dl(nl);
  for (size_t l = 0; l + 1 < nl; ++l) {
    if (!relax[l]) continue;
    if (par.relax == MAS_RELAX_VANKA || (par.relax == MAS_RELAX_VANKA_DLSC && l == 0)) {
      if (l == 0 && pr->disc == MAS_SV) {
        // three pressure seeds per element (Section 3.3.1)
        if (!pr->elem_p0 || pr->n_elem <= 0) throw MasError(MAS_EINVAL, "elem_p0 is required for Scott-Vogelius");
        std::vector<int64_t> pos(n0, -1);
        for (size_t q = 0; q < free0.size(); ++q) pos[free0[q]] = (int64_t)q;
        std::vector<int32_t> seeds((size_t)pr->n_elem * 3);
        for (int64_t e = 0; e < pr->n_elem * 3; ++e) {
          const int64_t g = pr->elem_p0[e];
          if (g < 0 || g >= n0 || pr->field0[g] != d) throw MasError(MAS_EINVAL, "elem_p0 must name pressure rows");
          seeds[e] = (int32_t)pos[g];
        }
        patches[l] = patches_element_seeds(Ks[l], fields[l], d, seeds, 3);
      } else {
        patches[l] = patches_single_seed(Ks[l], fields[l], d);
      }
      patches[l].shared = h->par.share_blocks != 0 && identical_component_blocks(Ks[l], fields[l], d, patches[l]);
      continue;
    }
    // DLSC (Algorithm 2): blocks of K_l, M_u = diag(P2 mass) on K0, I on the iso levels
    std::vector<int64_t> iv, ip;
    for (int64_t i = 0; i < Ks[l].nr; ++i) (fields[l][i] < d ? iv : ip).push_back(i);
    HostDlsc& D = dl[l];
    D.A = submatrix(Ks[l], iv, iv);
    D.B = submatrix(Ks[l], ip, iv);
    D.Bt = transpose(D.B);
    D.minv.assign(iv.size(), 1.0);
    if ((l == 0 || (ho && l == 1)) && pr->mu_diag0) {  // the level whose operator is K0
      int64_t q = 0;
      for (int64_t i = 0; i < n0; ++i) {
        if (pr->field0[i] >= d || pr->dir0[i]) continue;
        const double m = pr->mu_diag0[i];
        if (!(m > 0.0) || !std::isfinite(m)) throw MasError(MAS_EINVAL, "mu_diag0 must be positive");
        D.minv[q++] = 1.0 / m;
      }
    }
    Csr BM = D.B;
    for (int64_t i = 0; i < BM.nr; ++i)
      for (int64_t e = BM.ptr[i]; e < BM.ptr[i + 1]; ++e) BM.val[e] *= D.minv[BM.ind[e]];
    D.S = spgemm(BM, D.Bt);
    D.lamA = lanczos_max(D.A, par.seed + 2 * l, 20);
    D.lamS = lanczos_max(D.S, par.seed + 2 * l + 1, 20);
    if (par.dlsc_amg > 0) s_hierarchy(D, par, pr->p_nullspace != 0);
  }
  tr.mark("patches / DLSC operators");
  // coarsest operator, bordered with the coarse pressure null vector
  const Csr& KL = Ks.back();
  Csr Kb = KL;
  h->p_nullspace = pr->p_nullspace;
  if (pr->p_nullspace) {
    const std::vector<double>& Bp = fB[d][lmax - 1];
    std::vector<double> nvec(KL.nr, 0.0);
    int64_t q = 0;
    double nn = 0.0;
    for (int64_t i = 0; i < KL.nr; ++i)
      if (fields.back()[i] == d) {
        nvec[i] = Bp[q++];
        nn += nvec[i] * nvec[i];
      }
    nn = std::sqrt(nn);
    Kb.nr = Kb.nc = KL.nr + 1;
    Kb.ptr.clear();
    Kb.ind.clear();
    Kb.val.clear();
    Kb.ptr.push_back(0);
    for (int64_t i = 0; i < KL.nr; ++i) {
      for (int64_t e = KL.ptr[i]; e < KL.ptr[i + 1]; ++e) {
        Kb.ind.push_back(KL.ind[e]);
        Kb.val.push_back(KL.val[e]);
      }
      if (nvec[i] != 0.0) {
        Kb.ind.push_back((int32_t)KL.nr);
        Kb.val.push_back(nvec[i] / nn);
      }
      Kb.ptr.push_back((int64_t)Kb.ind.size());
    }
    for (int64_t i = 0; i < KL.nr; ++i)
      if (nvec[i] != 0.0) {
        Kb.ind.push_back((int32_t)i);
        Kb.val.push_back(nvec[i] / nn);
      }
    Kb.ptr.push_back((int64_t)Kb.ind.size());
  }
  HostPlan& pl = h->plan;
  pl.sv = pr->disc == MAS_SV;
  if (pl.sv) {
    const int64_t np1 = (int64_t)blocks[d].size();
    Csr Pp = get_csr(pr->Pp0, "Pp0"), Md = get_csr(pr->Mdg, "Mdg"), Mc = get_csr(pr->Mcg, "Mcg");
    if (Pp.nr != np0 || Pp.nc != np1 || Md.nr != np0 || Md.nc != np0 || Mc.nr != np1 || Mc.nc != np1)
      throw MasError(MAS_EINVAL, "Scott-Vogelius transfer operators have wrong shapes");
    pl.P0p = Pp;
    pl.P0t = transpose(Pp);
    pl.Mdg = Md;
    pl.Mcg = Mc;
    pl.mcg_dinv.assign(np1, 0.0);
    for (int64_t i = 0; i < np1; ++i)
      for (int64_t e = Mc.ptr[i]; e < Mc.ptr[i + 1]; ++e)
        if (Mc.ind[e] == i) pl.mcg_dinv[i] = 1.0 / Mc.val[e];
    // Chebyshev steps for the mass solve: error <= 2 (1/3)^k for the P1 interval [1/2, 2]
    const double tol = std::max(par.mass_rtol, 1e-16);
    pl.mass_steps = (int)std::ceil(std::log(2.0 / tol) / std::log(3.0));
  }
  pl.pw.clear();
  if (pr->p_weight0) {
    pl.pw.assign(pr->p_weight0, pr->p_weight0 + np0);
    h->pw_sum = 0.0;
    for (double v : pl.pw) h->pw_sum += v;
  }
  // info
  mas_hier_info& in = h->info;
  in.n_levels = (int32_t)nl;
  for (size_t l = 0; l < nl; ++l) {
    in.n[l] = Ks[l].nr;
    in.nnz[l] = Ks[l].nnz();
    int64_t nv = 0;
    for (auto f : fields[l]) nv += (f < d);
    in.n_vel[l] = nv;
    if (relax[l] && !patches[l].off.empty()) {
      in.n_patches[l] = patches[l].np();
      in.patch_dofs[l] = (int64_t)patches[l].dofs.size();
      const PatchSet& ps = patches[l];
      const int layout = patch_layout(ps, has_buckets(ps, h->par), h->par);
      int64_t fe = 0;
      for (int64_t p = 0; p < ps.np(); ++p) {
        const int32_t* q = &ps.dims[4 * p];
        fe += record_entries(q[0], q[1], q[2], q[3], layout);
      }
      in.factor_entries[l] = fe;
      in.patch_layout[l] = layout;
    }
    in.p_nnz[l] = (l >= 2) ? Ps[l - 1].nnz() : 0;
  }
  in.coarse_n = Kb.nr;
  pl.Ks = std::move(Ks);
  pl.Ps = std::move(Ps);
  pl.fields = std::move(fields);
  pl.patches = std::move(patches);
  pl.dlsc = std::move(dl);
  pl.relax = std::move(relax);
  pl.Kb = std::move(Kb);
  pl.free0 = std::move(free0);
  pl.dir0 = std::move(dir0);
  pl.K0 = std::move(K0);
}

void upload_impl(mas_handle* h, hipStream_t s) {
  HostPlan& pl = h->plan;
  const mas_params& par = h->par;
  const bool dry = h->arena.dry();
  const bool tune = par.autotune != 0 && !dry;
  const int64_t n0 = h->n0;
  h->K0full = upload_csr<double>(h->arena, pl.K0, s);
  h->K0full.stream = (double)h->K0full.nnz * 12.0 >= kStreamBytes;  // one FGMRES product per iteration
  {
    TempScope tmp(h->arena);
    double* tx = tmp.alloc<double>(n0);
    double* ty = tmp.alloc<double>(n0);
    if (!dry) HIPCHECK(hipMemsetAsync(tx, 0, n0 * sizeof(double), s));
    autotune_team<double>(h->K0full, tx, ty, s, tune);
    if (!dry) HIPCHECK(hipStreamSynchronize(s));
  }
  if (par.precision == MAS_FP32)
    h->cyc = build_cycle<float>(h, pl.Ks, pl.Ps, pl.fields, pl.patches, pl.dlsc, pl.relax, pl.Kb, pl.free0, pl.dir0,
                                s);
  else
    h->cyc = build_cycle<double>(h, pl.Ks, pl.Ps, pl.fields, pl.patches, pl.dlsc, pl.relax, pl.Kb, pl.free0, pl.dir0,
                                 s);
  h->cyc->describe(h->info);
  h->dir_idx = h->arena.upload<int64_t>(pl.dir0, s);
  h->ndir = (int64_t)pl.dir0.size();
  if (!pl.pw.empty()) h->pw = h->arena.upload<double>(pl.pw, s);
  const int m = std::max(1, par.restart);
  const int64_t R = std::max(1, par.nrhs_max);
  h->V = h->arena.alloc<double>((size_t)(m + 1) * n0 * R);
  h->Z = h->arena.alloc<double>((size_t)m * n0 * R);
  h->w = h->arena.alloc<double>((size_t)n0 * R);
  h->partial = h->arena.alloc<double>((size_t)2 * h->nblk_dot * R);
  h->cpart = h->arena.alloc<double>((size_t)(m + 1) * h->nblk_dot * R);
  h->use_mgs = par.gram_schmidt == MAS_GS_MODIFIED;
  h->hdev = h->arena.alloc<double>((size_t)(m + 2) * R);
  h->ydev = h->arena.alloc<double>((size_t)(m + 1) * R);
  if (dry) return;  // workspace query: sizes only, the handle stays analysed-only
  HIPCHECK(hipHostMalloc((void**)&h->hhost, (size_t)(m + 2) * R * sizeof(double), hipHostMallocDefault));
  HIPCHECK(hipStreamCreateWithFlags(&h->gs, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
  h->iter_graph.assign(m, nullptr);
  h->use_graphs = par.graphs != 0;
  HIPCHECK(hipStreamSynchronize(s));
  h->on_device = true;  // the host plan stays: mas_release / mas_upload rebuild from it
}

// Frees every device resource of the handle; the host analysis stays.
void release_device(mas_handle* h) {
  // work of the caller's streams may still read the handle's arrays (a caller
  // workspace too); a DRY arena never reached the device
  if (h->on_device || h->gs || h->hhost || !h->arena.ptrs.empty() || h->arena.mode == DevArena::BUFFER)
    (void)hipDeviceSynchronize();
  for (hipGraphExec_t& g : h->iter_graph)
    if (g) (void)hipGraphExecDestroy(g);
  h->iter_graph.clear();
  h->cyc.reset();
  h->arena.release();
  if (h->gs) (void)hipStreamDestroy(h->gs);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  if (h->hhost) (void)hipHostFree(h->hhost);
  h->gs = nullptr;
  h->ev_in = h->ev_out = nullptr;
  h->hhost = nullptr;
  h->V = h->Z = h->w = h->partial = h->hdev = h->ydev = h->cpart = nullptr;
  h->pw = nullptr;
  h->dir_idx = nullptr;
  h->K0full = DCsr<double>{};
  for (int l = 0; l < 16; ++l) {
    h->info.bucket_patches[l] = 0;
    h->info.patch_kernel[l] = 0;
    for (int q = 0; q < 16; ++q) h->info.bucket_shapes[l][q] = 0;
  }
  h->on_device = false;
}

// ---------------------------------------------------------------------------
// FGMRES (FP64)

// *out = x . y (or ||x|| when take_sqrt and x == y), reduced on the device
void dev_dot(mas_handle* h, const double* x, const double* y, int64_t n, hipStream_t s, double* out_dev,
             bool take_sqrt) {
  hipLaunchKernelGGL(k_mgs_step<double>, dim3(h->nblk_dot), dim3(256), 0, s, n, const_cast<double*>(x), nullptr, nullptr,
                     nullptr, take_sqrt ? nullptr : y, h->partial, take_sqrt ? 1 : 0);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, h->nblk_dot, h->partial, out_dev, take_sqrt ? 1 : 0);
  launch_check();
}

// FGMRES inner iteration j: z_j = B v_j, w = K0 z_j, modified Gram-Schmidt
// against v_0..v_j (one kernel per step), v_{j+1} = w / ||w||, H column ->
// pinned host memory.
void inner_iteration(mas_handle* h, int j, hipStream_t s) {
  const int64_t n = h->n0;
  double* vj = h->V + (int64_t)j * n;
  double* zj = h->Z + (int64_t)j * n;
  h->cyc->apply(vj, zj, s);
  double* w = h->w;
  csr_launch<double, 0>(h->K0full, zj, nullptr, w, s);
  double* part[2] = {h->partial, h->partial + h->nblk_dot};
  int pn = 0;  // the partial buffer the normalisation reads
  if (h->use_mgs) {  // modified Gram-Schmidt, one kernel per basis vector
    for (int i = 0; i <= j + 1; ++i) {
      const double* vprev = i > 0 ? h->V + (int64_t)(i - 1) * n : nullptr;
      double* hprev = i > 0 ? h->hdev + (i - 1) : nullptr;
      const double* pprev = i > 0 ? part[(i - 1) & 1] : nullptr;
      const double* vnext = i <= j ? h->V + (int64_t)i * n : nullptr;
      hipLaunchKernelGGL(k_mgs_step<double>, dim3(h->nblk_dot), dim3(256), 0, s, n, w, vprev, hprev, pprev, vnext,
                         part[i & 1], i <= j ? 0 : 1);
    }
    pn = (j + 1) & 1;
  } else {  // classical Gram-Schmidt: every dot in one sweep, then one update
    cgs_step(n, 1, 1, j + 1, h->V, w, h->cpart, h->hdev, part[0], (unsigned)h->nblk_dot, s);
  }
  hipLaunchKernelGGL(k_normalize<double>, dim3(h->nblk_dot), dim3(256), 0, s, n, part[pn], h->nblk_dot,
                     h->hdev + j + 1, w, h->V + (int64_t)(j + 1) * n);
  launch_check();
  HIPCHECK(hipMemcpyAsync(h->hhost, h->hdev, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
}

void run_inner_iteration(mas_handle* h, int j, hipStream_t s) {
  if (!h->use_graphs || h->tm.on) {
    inner_iteration(h, j, s);
    return;
  }
  if (!h->iter_graph[j]) {
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      inner_iteration(h, j, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHECK(hipStreamEndCapture(s, &g));
    hipGraphExec_t ex = nullptr;
    HIPCHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    h->iter_graph[j] = ex;
  }
  HIPCHECK(hipGraphLaunch(h->iter_graph[j], s));
}

double host_scalar(mas_handle* h, const double* dev, hipStream_t s) {
  HIPCHECK(hipMemcpyAsync(h->hhost, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return h->hhost[0];
}

int fgmres(mas_handle* h, const double* b, double* x, double rtol, int max_it, mas_solve_info* info,
           hipStream_t s) {
  const int64_t n = h->n0;
  const int m = std::max(1, h->par.restart);
  double* r = h->w;  // the residual lives in w between cycles
  dev_dot(h, b, b, n, s, h->hdev, true);
  const double bnorm = host_scalar(h, h->hdev, s);
  hipLaunchKernelGGL((k_fill<double>), dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, 0.0);
  launch_check();
  std::vector<double> hist;
  if (!(bnorm > 0.0)) {
    HIPCHECK(hipStreamSynchronize(s));
    if (info) *info = mas_solve_info{0, 1, 0.0, NAN};
    return std::isfinite(bnorm) ? MAS_OK : MAS_ENAN;
  }
  const double target = rtol * bnorm;
  double beta = bnorm;
  hist.push_back(beta);
  int it = 0;
  bool converged = false;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  HIPCHECK(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  while (true) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    hipLaunchKernelGGL(k_scale_inv, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, beta, r, h->V);
    launch_check();
    int k = 0;
    for (int j = 0; j < m; ++j) {
      run_inner_iteration(h, j, s);
      HIPCHECK(hipStreamSynchronize(s));
      for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = h->hhost[i];
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
      cs[j] = H[(size_t)j * m + j] / den;
      sn[j] = H[(size_t)(j + 1) * m + j] / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      k = j + 1;
      const double est = std::fabs(g[j + 1]);
      hist.push_back(est);
      if (!std::isfinite(est)) {
        if (info) *info = mas_solve_info{it, 0, NAN, NAN};
        return MAS_ENAN;
      }
      if (est <= target || it >= max_it) break;
    }
    // y = H^-1 g (upper triangular), x += Z y, true residual
    std::vector<double> y(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= H[(size_t)i * m + q] * y[q];
      y[i] = t / H[(size_t)i * m + i];
    }
    std::memcpy(h->hhost, y.data(), k * sizeof(double));
    HIPCHECK(hipMemcpyAsync(h->ydev, h->hhost, k * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_update_x<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, k, h->Z, h->ydev, x);
    launch_check();
    csr_launch<double, 1>(h->K0full, x, b, r, s);
    dev_dot(h, r, r, n, s, h->hdev, true);
    beta = host_scalar(h, h->hdev, s);
    if (!std::isfinite(beta)) {
      if (info) *info = mas_solve_info{it, 0, NAN, NAN};
      return MAS_ENAN;
    }
    if (beta <= target) {
      converged = true;
      break;
    }
    if (it >= max_it) break;
  }
  // zero-mean pressure
  if (h->p_nullspace && h->pw) {
    const int64_t np0 = n - h->nu0;
    dev_dot(h, x + h->nu0, h->pw, np0, s, h->hdev, false);
    const double mean = host_scalar(h, h->hdev, s) / h->pw_sum;
    hipLaunchKernelGGL((k_fill<double>), dim3(blocks_for(np0, 256)), dim3(256), 0, s, np0, h->w, -mean);
    hipLaunchKernelGGL((k_axpby<double>), dim3(blocks_for(np0, 256)), dim3(256), 0, s, np0, 1.0, h->w, 1.0,
                       x + h->nu0);
    launch_check();
    HIPCHECK(hipStreamSynchronize(s));
  }
  if (info) {
    info->iters = it;
    info->converged = converged ? 1 : 0;
    info->relres = beta / bnorm;
    info->conv_factor = hist.size() >= 11 ? std::pow(hist.back() / hist[hist.size() - 11], 0.1) : NAN;
  }
  return converged ? MAS_OK : MAS_NOT_CONVERGED;
}

// FGMRES for nr right-hand sides at once: independent Krylov spaces per column,
// advanced in lockstep so every cycle application is batched.  Each column has
// its own Givens rotations and tolerance; a column stops rotating once its
// estimate reaches its tolerance, and its iterate uses its own Krylov size.
// Restarted FGMRES for nr columns (Section 4).  fresh == nullptr: every column
// starts from x = 0 and runs to convergence or max_it.  Otherwise column k
// starts from x = 0 when fresh[k], else continues from the x it holds, and the
// call ends after max_cycles restart cycles (a scheduling step of continuous
// batching); info[k].iters then counts the iterations run in this call.
int fgmres_nr(mas_handle* h, const double* b, double* x, int nr, const double* rtol, int max_it,
              mas_solve_info* info, hipStream_t s, const int32_t* fresh = nullptr, int max_cycles = INT_MAX) {
  const int64_t n = h->n0;
  const int m = std::max(1, h->par.restart);
  int nrp = 1;
  while (nrp < nr) nrp *= 2;
  const unsigned nb = (unsigned)h->nblk_dot;
  double* r = h->w;
  auto col_norms = [&](const double* v, std::vector<double>& out) {
    hipLaunchKernelGGL(k_mgs_step_nr, dim3(nb), dim3(256), 0, s, n, nr, nrp, const_cast<double*>(v), nullptr, nullptr,
                       nullptr, nullptr, h->partial, 1);
    hipLaunchKernelGGL(k_reduce_final_nr, dim3(1), dim3(64), 0, s, (int)nb, nr, h->partial, h->hdev, 1);
    launch_check();
    HIPCHECK(hipMemcpyAsync(h->hhost, h->hdev, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    out.assign(h->hhost, h->hhost + nr);
  };
  std::vector<double> bnorm, beta;
  col_norms(b, bnorm);
  if (!fresh) {
    hipLaunchKernelGGL((k_fill<double>), dim3(blocks_for(n * nr, 256)), dim3(256), 0, s, n * nr, x, 0.0);
    HIPCHECK(hipMemcpyAsync(r, b, n * nr * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    // fresh columns start from zero, the others from their x: r = b - K0 x
    for (int k = 0; k < nr; ++k) h->hhost[k] = fresh[k] ? 0.0 : 1.0;
    HIPCHECK(hipMemcpyAsync(h->hdev, h->hhost, nr * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scale_cols_inplace, dim3(blocks_for(n * nr, 256)), dim3(256), 0, s, n, nr, h->hdev, x);
    hipLaunchKernelGGL((k_spmm<double, 1>), dim3(blocks_for(n, 256 / nr_pow2(nr))), dim3(256), 0, s, n, nr, nr_pow2(nr), h->K0full.ptr,
                       h->K0full.ind, h->K0full.val, x, b, r, ChebStep<double>{});
    launch_check();
  }
  std::vector<double> target(nr);
  std::vector<int> done(nr, 0), iters(nr, 0), used(nr, 0);
  std::vector<std::vector<double>> hist(nr);
  for (int k = 0; k < nr; ++k) {
    if (!std::isfinite(bnorm[k])) {
      if (info) for (int q = 0; q < nr; ++q) info[q] = mas_solve_info{0, 0, NAN, NAN};
      return MAS_ENAN;
    }
    target[k] = rtol[k] * bnorm[k];
    done[k] = bnorm[k] == 0.0;
    hist[k].push_back(bnorm[k]);
  }
  beta = bnorm;
  if (fresh) {
    std::vector<double> r0;
    col_norms(r, r0);
    for (int k = 0; k < nr; ++k) {
      if (!std::isfinite(r0[k])) {
        if (info) for (int q = 0; q < nr; ++q) info[q] = mas_solve_info{0, 0, NAN, NAN};
        return MAS_ENAN;
      }
      beta[k] = r0[k];
      done[k] = done[k] || r0[k] <= target[k];
      hist[k].assign(1, r0[k]);
    }
  }
  const std::vector<int> done_at_start = done;
  int it = 0, cycles = 0;
  std::vector<double> H((size_t)nr * (m + 1) * m), cs((size_t)nr * m), sn((size_t)nr * m), g((size_t)nr * (m + 1));
  std::vector<int> kcol(nr);
  h->cyc->set_nr(nr);
  while (true) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    std::vector<int> active(nr);
    for (int k = 0; k < nr; ++k) {
      g[(size_t)k * (m + 1)] = beta[k];
      active[k] = !done[k];
      kcol[k] = 0;
    }
    std::memcpy(h->hhost, beta.data(), nr * sizeof(double));
    HIPCHECK(hipMemcpyAsync(h->hdev, h->hhost, nr * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scale_cols, dim3(blocks_for(n * nr, 256)), dim3(256), 0, s, n, nr, h->hdev, r, h->V);
    launch_check();
    int kk = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = h->V + (int64_t)j * n * nr;
      double* zj = h->Z + (int64_t)j * n * nr;
      h->cyc->apply(vj, zj, s);
      double* w = h->w;
      hipLaunchKernelGGL((k_spmm<double, 0>), dim3(blocks_for(n, 256 / nr_pow2(nr))), dim3(256), 0, s, n, nr, nr_pow2(nr), h->K0full.ptr,
                         h->K0full.ind, h->K0full.val, zj, nullptr, w, ChebStep<double>{});
      double* part[2] = {h->partial, h->partial + (size_t)nb * nr};
      int pn = 0;
      if (h->use_mgs) {
        for (int i = 0; i <= j + 1; ++i) {
          const double* vprev = i > 0 ? h->V + (int64_t)(i - 1) * n * nr : nullptr;
          double* hprev = i > 0 ? h->hdev + (size_t)(i - 1) * nr : nullptr;
          const double* pprev = i > 0 ? part[(i - 1) & 1] : nullptr;
          const double* vnext = i <= j ? h->V + (int64_t)i * n * nr : nullptr;
          hipLaunchKernelGGL(k_mgs_step_nr, dim3(nb), dim3(256), 0, s, n, nr, nrp, w, vprev, hprev, pprev, vnext,
                             part[i & 1], i <= j ? 0 : 1);
        }
        pn = (j + 1) & 1;
      } else {
        cgs_step(n, nr, nrp, j + 1, h->V, w, h->cpart, h->hdev, part[0], (unsigned)nb, s);
      }
      hipLaunchKernelGGL(k_normalize_nr, dim3(nb), dim3(256), 0, s, n, nr, part[pn], (int)nb,
                         h->hdev + (size_t)(j + 1) * nr, w, h->V + (int64_t)(j + 1) * n * nr);
      launch_check();
      HIPCHECK(hipMemcpyAsync(h->hhost, h->hdev, (size_t)(j + 2) * nr * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      ++it;
      kk = j + 1;
      bool any = false;
      if (std::getenv("MAS_DEBUG_FGMRES")) {
        std::fprintf(stderr, "[fgmres_nr] it %d j %d h:", it, j);
        for (int k = 0; k < nr; ++k) std::fprintf(stderr, " %.3e/%.3e", h->hhost[(size_t)j * nr + k], h->hhost[(size_t)(j + 1) * nr + k]);
        std::fprintf(stderr, "\n");
      }
      for (int k = 0; k < nr; ++k) {
        if (!active[k]) continue;
        double* Hk = &H[(size_t)k * (m + 1) * m];
        double* ck = &cs[(size_t)k * m];
        double* sk = &sn[(size_t)k * m];
        double* gk = &g[(size_t)k * (m + 1)];
        for (int i = 0; i <= j + 1; ++i) Hk[(size_t)i * m + j] = h->hhost[(size_t)i * nr + k];
        for (int i = 0; i < j; ++i) {
          double t = ck[i] * Hk[(size_t)i * m + j] + sk[i] * Hk[(size_t)(i + 1) * m + j];
          Hk[(size_t)(i + 1) * m + j] = -sk[i] * Hk[(size_t)i * m + j] + ck[i] * Hk[(size_t)(i + 1) * m + j];
          Hk[(size_t)i * m + j] = t;
        }
        const double den = std::hypot(Hk[(size_t)j * m + j], Hk[(size_t)(j + 1) * m + j]);
        kcol[k] = j + 1;
        if (den == 0.0) {  // breakdown: the column is solved in this space
          active[k] = 0;
          continue;
        }
        ck[j] = Hk[(size_t)j * m + j] / den;
        sk[j] = Hk[(size_t)(j + 1) * m + j] / den;
        Hk[(size_t)j * m + j] = den;
        Hk[(size_t)(j + 1) * m + j] = 0.0;
        gk[j + 1] = -sk[j] * gk[j];
        gk[j] = ck[j] * gk[j];
        const double est = std::fabs(gk[j + 1]);
        hist[k].push_back(est);
        if (!std::isfinite(est)) {
          if (info) for (int q = 0; q < nr; ++q) info[q] = mas_solve_info{it, 0, NAN, NAN};
          h->cyc->set_nr(1);
          return MAS_ENAN;
        }
        if (est <= target[k]) active[k] = 0;
        else any = true;
      }
      if (!any || it >= max_it) break;
    }
    // per-column least-squares solutions, x += Z y
    std::vector<double> y((size_t)kk * nr, 0.0);
    for (int k = 0; k < nr; ++k) {
      const double* Hk = &H[(size_t)k * (m + 1) * m];
      const double* gk = &g[(size_t)k * (m + 1)];
      const int kc = kcol[k];
      for (int i = kc - 1; i >= 0; --i) {
        if (Hk[(size_t)i * m + i] == 0.0) continue;
        double t = gk[i];
        for (int q = i + 1; q < kc; ++q) t -= Hk[(size_t)i * m + q] * y[(size_t)q * nr + k];
        y[(size_t)i * nr + k] = t / Hk[(size_t)i * m + i];
      }
    }
    std::memcpy(h->hhost, y.data(), y.size() * sizeof(double));
    HIPCHECK(hipMemcpyAsync(h->ydev, h->hhost, y.size() * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_update_x_nr, dim3(blocks_for(n * nr, 256)), dim3(256), 0, s, n, nr, kk, h->Z, h->ydev, x);
    hipLaunchKernelGGL((k_spmm<double, 1>), dim3(blocks_for(n, 256 / nr_pow2(nr))), dim3(256), 0, s, n, nr, nr_pow2(nr), h->K0full.ptr,
                       h->K0full.ind, h->K0full.val, x, b, r, ChebStep<double>{});
    launch_check();
    col_norms(r, beta);
    bool all = true;
    ++cycles;
    for (int k = 0; k < nr; ++k) {
      if (!std::isfinite(beta[k])) {
        if (info) for (int q = 0; q < nr; ++q) info[q] = mas_solve_info{it, 0, NAN, NAN};
        h->cyc->set_nr(1);
        return MAS_ENAN;
      }
      // iterations this column used: a column idle for the rest of a cycle (its
      // estimate met the tolerance) does not count them
      if (!done[k]) used[k] += kcol[k];
      if (!done[k] && beta[k] <= target[k]) {
        done[k] = 1;
        iters[k] = used[k];
      }
      all = all && done[k];
    }
    if (all || it >= max_it || cycles >= max_cycles) break;
  }
  for (int k = 0; k < nr; ++k)
    if (!done[k]) iters[k] = used[k];
  // zero-mean pressure per column (a scheduling step: the columns that converged in it)
  if (h->p_nullspace && h->pw) {
    const int64_t np0 = n - h->nu0;
    hipLaunchKernelGGL(k_wdot_nr, dim3(nb), dim3(256), 0, s, np0, nr, nrp, h->pw, x + h->nu0 * nr, h->partial);
    hipLaunchKernelGGL(k_reduce_final_nr, dim3(1), dim3(64), 0, s, (int)nb, nr, h->partial, h->hdev, 0);
    launch_check();
    HIPCHECK(hipMemcpyAsync(h->hhost, h->hdev, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int k = 0; k < nr; ++k)
      h->hhost[k] = (fresh && (!done[k] || done_at_start[k])) ? 0.0 : -h->hhost[k] / h->pw_sum;
    HIPCHECK(hipMemcpyAsync(h->hdev, h->hhost, nr * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_add_cols, dim3(blocks_for(np0 * nr, 256)), dim3(256), 0, s, np0, nr, h->hdev,
                       x + h->nu0 * nr);
    launch_check();
    HIPCHECK(hipStreamSynchronize(s));
  }
  h->cyc->set_nr(1);
  bool all = true;
  for (int k = 0; k < nr; ++k) {
    all = all && done[k];
    if (info) {
      info[k].iters = iters[k];
      info[k].converged = done[k];
      info[k].relres = bnorm[k] > 0 ? beta[k] / bnorm[k] : 0.0;
      const auto& hh = hist[k];
      info[k].conv_factor = hh.size() >= 11 ? std::pow(hh.back() / hh[hh.size() - 11], 0.1) : NAN;
    }
  }
  return all ? MAS_OK : MAS_NOT_CONVERGED;
}

int fail(const MasError& e) {
  g_last_error = e.what();
  return e.code;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI

extern "C" {

void mas_default_params(int32_t dim, int32_t disc, int32_t relax, mas_params* out) {
  if (!out) return;
  mas_params p{};
  p.relax = relax;
  p.schedule = MAS_DC_ALL;
  p.nu1 = p.nu2 = (relax == MAS_RELAX_DLSC) ? 2 : 1;
  p.omega0 = 0.5;
  p.omega = 0.5;
  p.eta_u = 1.0;
  p.eta_p = 1.0;
  if (disc == MAS_SV && relax == MAS_RELAX_VANKA_DLSC) {  // Table 4, structured meshes, Vanka-DLSC
    p.omega0 = 0.87;
    p.eta_p = 2.96;
  } else if (disc == MAS_SV) {  // Table 4, structured meshes, Vanka on all levels
    p.omega0 = 0.78;
    p.eta_p = 2.68;
  }
  if (dim == 3) {
    p.cheb_deg[0] = 4; p.cheb_deg[1] = 4; p.cheb_deg[2] = 16;
  } else {
    p.cheb_deg[0] = 3; p.cheb_deg[1] = 3; p.cheb_deg[2] = 6;
  }
  p.precision = MAS_FP64;
  p.restart = 20;
  p.max_coarse = 300;
  p.max_levels = 10;
  p.theta = 0.02;
  p.seed = 0x5EED;
  p.mass_rtol = 1e-14;
  p.nrhs_max = 1;
  p.krylov_its = 0;
  p.nu_dlsc = 2;
  p.dlsc_amg = 0;
  // evolution strength (Section 3.2) for Taylor-Hood; Scott-Vogelius keeps the
  // symmetric measure: on Alfeld meshes the evolution measure coarsens the K1
  // pressure at about half the velocity rate, and stationary omega = 0.5 Vanka
  // then diverges on the coarse saddle levels
  p.soc = disc == MAS_SV ? MAS_SOC_SYMMETRIC : MAS_SOC_EVOLUTION;
  p.soc_eps = 4.0;
  p.gram_schmidt = MAS_GS_CLASSICAL;
  p.autotune = 1;
  p.graphs = 1;
  p.full_patch_min = kFullPatch;
  p.bucket_min = 32768;
  p.factor_blocked = 1;
  p.device_galerkin = 1;
  p.share_blocks = 1;
  p.patch_kernel = 0;
  p.device_sa = 1;
  p.spgemm_cap = 0;
  *out = p;
}

int mas_setup(const mas_problem* prob, const mas_params* par, void* stream, mas_handle** out) {
  if (!prob || !par || !out) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  *out = nullptr;
  auto h = std::make_unique<mas_handle>();
  h->par = *par;
  try {
    analyze_impl(h.get(), prob, true, (hipStream_t)stream);
    upload_impl(h.get(), (hipStream_t)stream);
  } catch (const MasError& e) {
    release_device(h.get());
    return fail(e);
  } catch (const std::bad_alloc&) {
    release_device(h.get());
    g_last_error = "host allocation failed";
    return MAS_ENOMEM;
  } catch (const std::exception& e) {
    release_device(h.get());
    g_last_error = e.what();
    return MAS_EINVAL;
  }
  *out = h.release();
  return MAS_OK;
}

int mas_analyze(const mas_problem* prob, const mas_params* par, mas_handle** out) {
  if (!prob || !par || !out) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  *out = nullptr;
  auto h = std::make_unique<mas_handle>();
  h->par = *par;
  try {
    analyze_impl(h.get(), prob);
  } catch (const MasError& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MAS_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MAS_EINVAL;
  }
  *out = h.release();
  return MAS_OK;
}

int mas_apply(mas_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  if (!h || !r || !z) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  if (!h->on_device) {
    g_last_error = "handle was analysed only; call mas_setup";
    return MAS_EINVAL;
  }
  if (nrhs < 1 || nrhs > std::max(1, h->par.nrhs_max)) {
    g_last_error = "nrhs must be in [1, nrhs_max]";
    return MAS_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    h->cyc->set_nr(nrhs);
    h->cyc->apply(r, z, s);
    h->cyc->set_nr(1);
    if (h->tm.on) {  // the timed launches of this application, for mas_get_timing
      HIPCHECK(hipStreamSynchronize(s));
      h->tm.collect();
    }
  } catch (const MasError& e) {
    h->cyc->set_nr(1);
    return fail(e);
  }
  return MAS_OK;
}

static int solve_impl(mas_handle* h, const double* b, double* x, int32_t nrhs, const double* rtol, int32_t max_it,
                      mas_solve_info* info, void* stream) {
  if (!h || !b || !x || !rtol || max_it < 1) {
    g_last_error = "bad argument";
    return MAS_EINVAL;
  }
  if (!h->on_device) {
    g_last_error = "handle was analysed only; call mas_setup";
    return MAS_EINVAL;
  }
  if (nrhs < 1 || nrhs > std::max(1, h->par.nrhs_max)) {
    g_last_error = "nrhs must be in [1, nrhs_max]";
    return MAS_EINVAL;
  }
  for (int k = 0; k < nrhs; ++k)
    if (!(rtol[k] >= 0.0)) {
      g_last_error = "bad argument";
      return MAS_EINVAL;
    }
  try {
    hipStream_t us = (hipStream_t)stream;
    hipStream_t s = h->gs;
    HIPCHECK(hipEventRecord(h->ev_in, us));
    HIPCHECK(hipStreamWaitEvent(s, h->ev_in, 0));
    int rc = nrhs == 1 ? fgmres(h, b, x, rtol[0], max_it, info, s) : fgmres_nr(h, b, x, nrhs, rtol, max_it, info, s);
    HIPCHECK(hipEventRecord(h->ev_out, s));
    HIPCHECK(hipStreamWaitEvent(us, h->ev_out, 0));
    if (h->tm.on) {
      HIPCHECK(hipStreamSynchronize(s));
      h->tm.collect();
    }
    if (rc == MAS_ENAN) g_last_error = "residual is not finite";
    return rc;
  } catch (const MasError& e) {
    return fail(e);
  }
}

int mas_solve(mas_handle* h, const double* b, double* x, int32_t nrhs, double rtol, int32_t max_it,
              mas_solve_info* info, void* stream) {
  if (nrhs < 1 || nrhs > 64) {
    g_last_error = "nrhs must be in [1, nrhs_max]";
    return MAS_EINVAL;
  }
  double tols[64];
  for (int k = 0; k < nrhs; ++k) tols[k] = rtol;
  return solve_impl(h, b, x, nrhs, tols, max_it, info, stream);
}

int mas_solve_rtols(mas_handle* h, const double* b, double* x, int32_t nrhs, const double* rtol, int32_t max_it,
                    mas_solve_info* info, void* stream) {
  return solve_impl(h, b, x, nrhs, rtol, max_it, info, stream);
}

int mas_solve_step(mas_handle* h, const double* b, double* x, int32_t nrhs, const double* rtol, const int32_t* fresh,
                   int32_t cycles, mas_solve_info* info, void* stream) {
  if (!h || !b || !x || !rtol || !fresh || cycles < 1) {
    g_last_error = "bad argument";
    return MAS_EINVAL;
  }
  if (!h->on_device) {
    g_last_error = "handle was analysed only; call mas_setup";
    return MAS_EINVAL;
  }
  if (nrhs < 1 || nrhs > std::max(1, h->par.nrhs_max)) {
    g_last_error = "nrhs must be in [1, nrhs_max]";
    return MAS_EINVAL;
  }
  for (int k = 0; k < nrhs; ++k)
    if (!(rtol[k] >= 0.0)) {
      g_last_error = "bad argument";
      return MAS_EINVAL;
    }
  if (h->par.krylov_its > 0 && nrhs > 1) {
    g_last_error = "the FGMRES-wrapped relaxation takes one right-hand side per call";
    return MAS_EINVAL;
  }
  try {
    hipStream_t us = (hipStream_t)stream;
    hipStream_t s = h->gs;
    HIPCHECK(hipEventRecord(h->ev_in, us));
    HIPCHECK(hipStreamWaitEvent(s, h->ev_in, 0));
    const int max_it = cycles * std::max(1, h->par.restart);
    int rc = fgmres_nr(h, b, x, nrhs, rtol, max_it, info, s, fresh, cycles);
    HIPCHECK(hipEventRecord(h->ev_out, s));
    HIPCHECK(hipStreamWaitEvent(us, h->ev_out, 0));
    if (rc == MAS_ENAN) g_last_error = "residual is not finite";
    return rc;
  } catch (const MasError& e) {
    h->cyc->set_nr(1);
    return fail(e);
  }
}

int mas_get_info(const mas_handle* h, mas_hier_info* out) {
  if (!h || !out) return MAS_EINVAL;
  *out = h->info;
  out->device_bytes = (int64_t)h->arena.bytes;
  return MAS_OK;
}

int mas_scale_rows(mas_handle* h, double* x, int32_t nrhs, const double* s_u, const double* s_p,
                   int32_t dirichlet_inverse, void* stream) {
  if (!h || !x || !s_u || !s_p || nrhs < 1 || nrhs > 64) {
    g_last_error = "bad argument";
    return MAS_EINVAL;
  }
  if (!h->on_device) {
    g_last_error = "handle was analysed only; call mas_setup";
    return MAS_EINVAL;
  }
  try {
    hipStream_t s = (hipStream_t)stream;
    double* d = h->ydev;  // 2 * nrhs factors staged through pinned memory
    if ((size_t)(h->par.restart + 1) * std::max(1, h->par.nrhs_max) < (size_t)2 * nrhs)
      throw MasError(MAS_EINVAL, "nrhs too large for this handle");
    HIPCHECK(hipStreamSynchronize(s));
    std::memcpy(h->hhost, s_u, nrhs * sizeof(double));
    std::memcpy(h->hhost + nrhs, s_p, nrhs * sizeof(double));
    HIPCHECK(hipMemcpyAsync(d, h->hhost, 2 * nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scale_rows_nr, dim3(blocks_for(h->n0 * nrhs, 256)), dim3(256), 0, s, h->n0, nrhs, h->nu0, d,
                       d + nrhs, x);
    launch_check();
    if (dirichlet_inverse && h->ndir) {
      // identity rows: net factor 1 / s_u
      HIPCHECK(hipStreamSynchronize(s));
      for (int k = 0; k < nrhs; ++k) h->hhost[k] = 1.0 / (s_u[k] * s_u[k]);
      HIPCHECK(hipMemcpyAsync(d, h->hhost, nrhs * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_scale_idx_nr, dim3(blocks_for(h->ndir * nrhs, 256)), dim3(256), 0, s, h->ndir, nrhs,
                         h->dir_idx, d, x);
      launch_check();
    }
    HIPCHECK(hipStreamSynchronize(s));
  } catch (const MasError& e) {
    return fail(e);
  }
  return MAS_OK;
}

int mas_export_level(const mas_handle* h, int32_t level, int64_t* nrows, int64_t* nnz, int64_t* indptr,
                     int32_t* indices, double* data) {
  if (!h || level < 0 || level >= (int32_t)h->plan.Ks.size()) {
    g_last_error = "bad level";
    return MAS_EINVAL;
  }
  const Csr& A = h->plan.Ks[level];
  if (nrows) *nrows = A.nr;
  if (nnz) *nnz = A.nnz();
  if (indptr) std::memcpy(indptr, A.ptr.data(), (A.nr + 1) * sizeof(int64_t));
  if (indices) std::memcpy(indices, A.ind.data(), A.nnz() * sizeof(int32_t));
  if (data) std::memcpy(data, A.val.data(), A.nnz() * sizeof(double));
  return MAS_OK;
}

int mas_set_timing(mas_handle* h, int32_t enable) {
  if (!h) return MAS_EINVAL;
  h->tm.on = enable != 0;
  h->tm.reset();
  return MAS_OK;
}

int mas_get_timing(const mas_handle* h, double* out, int32_t n) {
  if (!h || !out) return MAS_EINVAL;
  for (int k = 0; k < TK_KINDS; ++k) {
    const double v[3] = {h->tm.ms[k], (double)h->tm.launches[k], h->tm.bytes[k]};
    for (int q = 0; q < 3; ++q)
      if (3 * k + q < n) out[3 * k + q] = v[q];
  }
  return MAS_OK;
}

int mas_release(mas_handle* h) {
  if (!h) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  release_device(h);
  return MAS_OK;
}

int mas_upload(mas_handle* h, void* stream) {
  if (!h) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  if (h->on_device) return MAS_OK;
  try {
    upload_impl(h, (hipStream_t)stream);
  } catch (const MasError& e) {
    release_device(h);
    return fail(e);
  } catch (const std::bad_alloc&) {
    release_device(h);
    g_last_error = "host allocation failed";
    return MAS_ENOMEM;
  } catch (const std::exception& e) {
    release_device(h);
    g_last_error = e.what();
    return MAS_EINVAL;
  }
  return MAS_OK;
}

// ---------------------------------------------------------------------------
// mas_apply_static: the cycle's per-application scratch in a file-scope device
// array.  Every device the library runs on holds its own copy of the array
// until the process ends; host code takes its address on that device from
// hipGetSymbolAddress (the array's name is only a host-side stand-in).

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// address of `scratch` on the current device (looked up once per device)
void* device_scratch() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw MasError(MAS_EINVAL, "device ordinal out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw MasError(MAS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

int mas_apply_static(mas_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  if (!h || !r || !z) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  if (!h->on_device) {
    g_last_error = "handle was analysed only; call mas_setup";
    return MAS_EINVAL;
  }
  if (nrhs < 1 || nrhs > std::max(1, h->par.nrhs_max)) {
    g_last_error = "nrhs must be in [1, nrhs_max]";
    return MAS_EINVAL;
  }
  // bytes this call's scratch takes, each array rounded to 256 bytes
  size_t need = 0;
  h->cyc->scratch_arrays(nrhs, [&](void**, size_t b) { need += DevArena::round(std::max<size_t>(b, 1)); });
  if (need > kStaticScratchBytes) {
    g_last_error = "mas_apply_static: this handle's cycle scratch for " + std::to_string(nrhs) +
                   " right-hand side(s) is " + std::to_string(need) + " bytes, above the static scratch of " +
                   std::to_string(kStaticScratchBytes) + " bytes (use mas_apply)";
    return MAS_EINVAL;
  }
  std::vector<void*> saved;
  bool moved = false;
  const bool timing = h->tm.on;
  try {
    char* base = (char*)device_scratch();
    size_t off = 0;
    h->cyc->scratch_arrays(nrhs, [&](void** p, size_t b) {
      saved.push_back(*p);
      *p = base + off;
      off += DevArena::round(std::max<size_t>(b, 1));
    });
    moved = true;
    h->tm.on = false;  // no event timing here: it would create events during the call
    hipStream_t s = (hipStream_t)stream;
    h->cyc->set_nr(nrhs);
    h->cyc->apply(r, z, s);
    h->cyc->set_nr(1);
  } catch (const MasError& e) {
    h->cyc->set_nr(1);
    h->tm.on = timing;
    if (moved) {
      size_t k = 0;
      h->cyc->scratch_arrays(nrhs, [&](void** p, size_t) { *p = saved[k++]; });
    }
    return fail(e);
  }
  h->tm.on = timing;
  size_t k = 0;
  h->cyc->scratch_arrays(nrhs, [&](void** p, size_t) { *p = saved[k++]; });
  return MAS_OK;
}

int mas_workspace_size(mas_handle* h, size_t* bytes) {
  if (!h || !bytes) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  if (h->on_device) {
    g_last_error = "the handle is on the device: query the workspace size before mas_upload_ws";
    return MAS_EINVAL;
  }
  int rc = MAS_OK;
  try {
    h->arena.use_buffer(nullptr, 0, true);
    upload_impl(h, nullptr);  // sizes only: nothing is allocated or launched
    *bytes = h->arena.peak;
  } catch (const MasError& e) {
    rc = fail(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    rc = MAS_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    rc = MAS_EINVAL;
  }
  release_device(h);  // drops the counted (never dereferenced) pointers
  return rc;
}

int mas_upload_ws(mas_handle* h, void* dev_ws, size_t ws_bytes, void* stream) {
  if (!h || !dev_ws) {
    g_last_error = "null argument";
    return MAS_EINVAL;
  }
  if (h->on_device) {
    g_last_error = "the handle is already on the device";
    return MAS_EINVAL;
  }
  if ((uintptr_t)dev_ws % DevArena::kAlign != 0) {
    g_last_error = "dev_ws must be 256-byte aligned";
    return MAS_EINVAL;
  }
  try {
    h->arena.use_buffer(dev_ws, ws_bytes, false);
    upload_impl(h, (hipStream_t)stream);
  } catch (const MasError& e) {
    release_device(h);
    return fail(e);
  } catch (const std::bad_alloc&) {
    release_device(h);
    g_last_error = "host allocation failed";
    return MAS_ENOMEM;
  } catch (const std::exception& e) {
    release_device(h);
    g_last_error = e.what();
    return MAS_EINVAL;
  }
  return MAS_OK;
}

int mas_destroy(mas_handle* h) {
  if (!h) return MAS_OK;
  release_device(h);
  delete h;
  return MAS_OK;
}

const char* mas_error_string(int status) {
  switch (status) {
    case MAS_OK: return "ok";
    case MAS_NOT_CONVERGED: return "not converged";
    case MAS_EINVAL: return "invalid argument";
    case MAS_ESINGULAR_PATCH: return "singular patch or coarse operator";
    case MAS_ENOMEM: return "out of memory";
    case MAS_EHIP: return "HIP runtime error";
    case MAS_ENAN: return "non-finite residual";
    default: return "unknown status";
  }
}

const char* mas_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
