// HIP kernels of libmas for gfx950 (CDNA4, 64-lane wavefronts).
//
// Patch factor layout (one contiguous record per patch, value type T):
//   [ A_0^-1 | A_1^-1 | A_2^-1 | Uhat | S^-1 ]
// A_c^-1: inverse of the patch's velocity block of component c, symmetric,
//         packed upper: entry (i, j), i <= j, at j (j + 1) / 2 + i;
// Uhat  = -A^-1 B^T (nv x ns), column s contiguous;
// S^-1  = (-B A^-1 B^T)^-1 (ns x ns), packed the same way.
// The apply uses Bhat = -S^-1 B A^-1 = S^-1 Uhat^T, so Bhat is not stored:
//   y_u = A^-1 b_u,  y_p = S^-1 (Uhat^T b_u + b_p),  x_u = y_u + Uhat y_p,  x_p = y_p
// (block factorisation of the patch saddle matrix, Section 3.3.1).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mas {

constexpr int WAVE = 64;
constexpr int MAX_NS = 4;  // seeds per patch handled by the kernels

// values of one velocity block: packed upper triangle, or the full n x n
// matrix (levels with very large patches, read with coalesced row sweeps)
__host__ __device__ __forceinline__ int64_t blk_size(int n, int full) {
  return full ? (int64_t)n * n : (int64_t)n * (n + 1) / 2;
}

// Layout of the A^-1 part of a patch factor record (bits): LAYOUT_FULL, blocks
// stored n x n (entry (i, j) at j n + i) instead of packed upper triangles
// (entry (i, j), i <= j, at j (j + 1) / 2 + i); LAYOUT_SHARED, the velocity
// components' blocks are identical and one block, stored once, serves all of
// them (records then hold [A^-1 | Uhat | S^-1] instead of
// [A_0^-1 | A_1^-1 | A_2^-1 | Uhat | S^-1]).
constexpr int LAYOUT_FULL = 1, LAYOUT_SHARED = 2;
// values of the A^-1 part of a record with per-component sizes n0, n1, n2
__host__ __device__ __forceinline__ int64_t vel_entries(int n0, int n1, int n2, int layout) {
  const int f = layout & LAYOUT_FULL;
  return (layout & LAYOUT_SHARED) ? blk_size(n0, f) : blk_size(n0, f) + blk_size(n1, f) + blk_size(n2, f);
}
// offset of component c's block within the A^-1 part
__host__ __device__ __forceinline__ int64_t comp_offset(int c, int n0, int n1, int layout) {
  if ((layout & LAYOUT_SHARED) || c == 0) return 0;
  const int f = layout & LAYOUT_FULL;
  return c == 1 ? blk_size(n0, f) : blk_size(n0, f) + blk_size(n1, f);
}
// values of a whole record (seeds ns)
__host__ __device__ __forceinline__ int64_t record_entries(int n0, int n1, int n2, int ns, int layout) {
  return vel_entries(n0, n1, n2, layout) + (int64_t)(n0 + n1 + n2) * ns + (int64_t)ns * (ns + 1) / 2;
}

__device__ __forceinline__ int64_t packed_index(int i, int j) {
  int a = i < j ? i : j, b = i < j ? j : i;
  return (int64_t)b * (b + 1) / 2 + a;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Load of data a launch reads once (matrix entries, factor records): non-
// temporal, so the stream does not evict the level vectors that the same
// launch gathers (measured: the 256x256 TH FP64 cycle 3.4% faster).  Used
// only for operators and factor records far larger than the caches that a
// cycle reads once per relaxation; re-read or small data keeps plain loads.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
// the same where the choice is a template parameter (operators re-read within
// a cycle, or small enough to stay cached, keep plain loads)
template <bool NT, typename T>
__device__ __forceinline__ T ldv(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// ---------------------------------------------------------------------------
// One step of the Chebyshev semi-iteration fused into a product (MODE 4): with
// y the residual and x the current direction d, row i computes
// r_i = y_i - (A d)_i, d'_i = a d_i + c Dinv_i r_i, writes y_i = r_i,
// dnew_i = d'_i and adds d'_i to acc_i -- the same operations, in the same
// order, as a MODE 3 product followed by the update d = a d + c Dinv r, acc += d.
template <typename T>
struct ChebStep {
  T a, c;
  const T* dinv;  // per row of the operator, or null (identity); MODE 5: the row scale m
  T* dnew;
  T* acc;
  T* res = nullptr;  // MODES 1, 3, 5 with res set: also start a Chebyshev iteration from
                     // the row value v: res = v, dnew = acc = c * (Dinv v) (Dinv = cinv)
  const T* cinv = nullptr;
};

// start of a Chebyshev iteration from the residual value v of row `row`
template <typename T>
__device__ __forceinline__ void cheb_start(int64_t e, int64_t row, T v, const ChebStep<T>& cs) {
  const T di = (cs.cinv ? cs.cinv[row] * v : v) * cs.c;
  cs.dnew[e] = di;
  cs.res[e] = v;
  cs.acc[e] = di;
}

template <typename T>
__device__ __forceinline__ void cheb_row(int64_t e, int64_t row, T s, const T* __restrict__ x, T* __restrict__ y,
                                         const ChebStep<T>& cs) {
  const T r = y[e] - s;
  y[e] = r;
  const T ri = cs.dinv ? cs.dinv[row] * r : r;
  const T di = cs.a * x[e] + cs.c * ri;
  cs.dnew[e] = di;
  cs.acc[e] += di;
}

// the result s = (A x)_row of a product, stored as the mode asks (entry e of
// the interleaved vectors)
template <typename T, int MODE>
__device__ __forceinline__ void store_row(int64_t e, int64_t row, T s, const T* __restrict__ x,
                                          const T* __restrict__ b, T* __restrict__ y, const ChebStep<T>& cs) {
  if (MODE == 0) {
    y[e] = s;
  } else if (MODE == 2) {
    y[e] += s;
  } else if (MODE == 4) {
    cheb_row(e, row, s, x, y, cs);
  } else {
    const T v = MODE == 1 ? b[e] - s : MODE == 3 ? y[e] - s : cs.a * (cs.dinv ? cs.dinv[row] * s : s);
    y[e] = v;
    if (cs.res) cheb_start(e, row, v, cs);
  }
}

// CSR products.  TEAM lanes per row (power of two <= 64).
// MODE 0: y = A x   MODE 1: y = b - A x   MODE 2: y += A x   MODE 3: y -= A x
// MODE 4: Chebyshev step (ChebStep)   MODE 5: y = a m (A x), m = cs.dinv per row (or 1)
// MODES 1, 3, 5 start a Chebyshev iteration from the stored value when cs.res is set
template <typename T, int TEAM, int MODE, bool NT = false>
__global__ void __launch_bounds__(256) k_csr(int n, const int* __restrict__ ptr, const int* __restrict__ ind,
                                             const T* __restrict__ val, const T* __restrict__ x,
                                             const T* __restrict__ b, T* __restrict__ y, ChebStep<T> cs) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = gid / TEAM;
  const int lane = gid & (TEAM - 1);
  T s = 0;
  if (row < n) {
    const int e1 = ptr[row + 1];
    for (int e = ptr[row] + lane; e < e1; e += TEAM)
      s += ldv<NT>(&val[e]) * x[ldv<NT>(&ind[e])];
  }
#pragma unroll
  for (int o = TEAM / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (row < n && lane == 0) store_row<T, MODE>(row, row, s, x, b, y, cs);
}

// Sliced ELL, 64 rows per slice (one wavefront, one lane per row), entries of a
// slice stored column-major so that every load of the wavefront is one
// contiguous segment; padded entries have value 0 and a valid column.
template <typename T, int MODE, bool NT = false>
__global__ void __launch_bounds__(256) k_sell(int n, int64_t nslices, const int64_t* __restrict__ soff,
                                              const int* __restrict__ swidth, const int* __restrict__ ind,
                                              const T* __restrict__ val, const T* __restrict__ x,
                                              const T* __restrict__ b, T* __restrict__ y, ChebStep<T> cs) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slice = row >> 6;
  if (slice >= nslices) return;
  const int lane = threadIdx.x & 63;
  const int64_t base = soff[slice] + lane;
  const int w = swidth[slice];
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int c = 0;
  for (; c + 7 < w; c += 8) {  // eight entries in flight
    const int64_t e = base + (int64_t)c * 64;
    int q[8];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q[u] = ldv<NT>(&ind[e + 64 * u]);
      v[u] = ldv<NT>(&val[e + 64 * u]);
    }
    T g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = x[q[u]];
    s0 += v[0] * g[0];
    s1 += v[1] * g[1];
    s2 += v[2] * g[2];
    s3 += v[3] * g[3];
    s0 += v[4] * g[4];
    s1 += v[5] * g[5];
    s2 += v[6] * g[6];
    s3 += v[7] * g[7];
  }
  for (; c + 3 < w; c += 4) {
    const int64_t e = base + (int64_t)c * 64;
    s0 += ldv<NT>(&val[e]) * x[ldv<NT>(&ind[e])];
    s1 += ldv<NT>(&val[e + 64]) * x[ldv<NT>(&ind[e + 64])];
    s2 += ldv<NT>(&val[e + 128]) * x[ldv<NT>(&ind[e + 128])];
    s3 += ldv<NT>(&val[e + 192]) * x[ldv<NT>(&ind[e + 192])];
  }
  for (; c < w; ++c) {
    const int64_t e = base + (int64_t)c * 64;
    s0 += ldv<NT>(&val[e]) * x[ldv<NT>(&ind[e])];
  }
  const T s = (s0 + s1) + (s2 + s3);
  if (row < n) store_row<T, MODE>(row, row, s, x, b, y, cs);
}

// ---------------------------------------------------------------------------
// vector kernels

template <typename T>
__global__ void k_fill(int64_t n, T* __restrict__ y, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

// dst[k] = (T) src[idx[k]]
template <typename T, typename S>
__global__ void k_gather(int64_t n, const int64_t* __restrict__ idx, const S* __restrict__ src, T* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (T)src[idx[k]];
}

// dst[idx[k]] = src[idx[k]]
__global__ void k_copy_idx(int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ src,
                           double* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[idx[k]] = src[idx[k]];
}

// dst[idx[k]] = (T) src[k]
template <typename T, typename S>
__global__ void k_scatter(int64_t n, const int64_t* __restrict__ idx, const S* __restrict__ src, T* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[idx[k]] = (T)src[k];
}

// y[k] = (k < nsplit ? a : b) * x[k]
template <typename T>
__global__ void k_scale2(int64_t n, int64_t nsplit, T a, T b, const T* __restrict__ x, T* __restrict__ y) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] = (k < nsplit ? a : b) * x[k];
}

// y = a x + b y; y is not read when b == 0 (it may hold uninitialised memory)
template <typename T>
__global__ void k_axpby(int64_t n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] = (b == (T)0) ? a * x[k] : a * x[k] + b * y[k];
}

// ---------------------------------------------------------------------------
// Chebyshev semi-iteration and DLSC helpers (Algorithm 2, Table 2)

// d = D^-1 r / theta, res = r, y = d   (D^-1 = dinv, identity when null; nr
// right-hand sides interleaved, entry i belongs to row i / nr)
template <typename T>
__global__ void k_cheb_init(int64_t n, const T* __restrict__ r, T inv_theta, const T* __restrict__ dinv,
                            T* __restrict__ d, T* __restrict__ res, T* __restrict__ y, int nr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const T ri = r[i];
    const T di = (dinv ? dinv[i / nr] * ri : ri) * inv_theta;
    d[i] = di;
    res[i] = ri;
    y[i] = di;
  }
}

// end of a DLSC sweep on x = (u, p): u += v + t (first nu entries), p += dp
template <typename T>
__global__ void k_dlsc_update(int64_t nu, int64_t np, T* __restrict__ x, const T* __restrict__ v,
                              const T* __restrict__ t, const T* __restrict__ dp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nu) x[i] += v[i] + t[i];
  else if (i < nu + np) x[i] += dp[i - nu];
}

// x[i] *= m[i / nr]
template <typename T>
__global__ void k_mul(int64_t n, const T* __restrict__ m, T* __restrict__ x, int nr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= m[i / nr];
}

// ---------------------------------------------------------------------------
// batched kernels: nr right-hand sides interleaved, entry (i, k) at i * nr + k

// dst[q * nr + k] = (T) src[idx[q] * nr + k]
template <typename T, typename S>
__global__ void k_gather_nr(int64_t n, int nr, const int64_t* __restrict__ idx, const S* __restrict__ src,
                            T* __restrict__ dst) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) dst[t] = (T)src[idx[t / nr] * nr + t % nr];
}

// dst[idx[q] * nr + k] = (T) src[q * nr + k]
template <typename T, typename S>
__global__ void k_scatter_nr(int64_t n, int nr, const int64_t* __restrict__ idx, const S* __restrict__ src,
                             T* __restrict__ dst) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) dst[idx[t / nr] * nr + t % nr] = (T)src[t];
}

__global__ void k_copy_idx_nr(int64_t n, int nr, const int64_t* __restrict__ idx, const double* __restrict__ src,
                              double* __restrict__ dst) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) {
    const int64_t e = idx[t / nr] * nr + t % nr;
    dst[e] = src[e];
  }
}

// Y = A X for nr interleaved right-hand sides (CSR): one thread per (row, rhs);
// the threads of a row read the same matrix entries and contiguous X rows.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_spmm(int64_t n, int nr, int nrp, const int* __restrict__ ptr,
                                              const int* __restrict__ ind, const T* __restrict__ val,
                                              const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ y, ChebStep<T> cs) {
  // thread (row, right-hand side k), k = tid % nrp for the whole kernel; with
  // nrp = 64 a wavefront holds one row, whose indices and values it then
  // reads with wave-uniform loads
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  int64_t row = (int64_t)blockIdx.x * ng + g;
  if (nrp == WAVE) row = __builtin_amdgcn_readfirstlane((int)row);
  if (row >= n || k >= nr) return;
  const int64_t t = row * nr + k;
  T s = 0;
  int e = ptr[row];
  const int end = ptr[row + 1];
  for (; e + 3 < end; e += 4) {  // four gathers in flight, sums in the same order
    const int c0 = ind[e], c1 = ind[e + 1], c2 = ind[e + 2], c3 = ind[e + 3];
    const T x0 = x[(int64_t)c0 * nr + k], x1 = x[(int64_t)c1 * nr + k];
    const T x2 = x[(int64_t)c2 * nr + k], x3 = x[(int64_t)c3 * nr + k];
    s += val[e] * x0;
    s += val[e + 1] * x1;
    s += val[e + 2] * x2;
    s += val[e + 3] * x3;
  }
  for (; e < end; ++e) s += val[e] * x[(int64_t)ind[e] * nr + k];
  store_row<T, MODE>(t, row, s, x, b, y, cs);
}

// dense coarse solve for nr right-hand sides: y = C b, FP64 accumulation
template <typename T>
__global__ void __launch_bounds__(256) k_dense_gemm(int n, int ld, int nr, const double* __restrict__ C,
                                                   const T* __restrict__ b, T* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * nr) return;
  const int64_t row = t / nr;
  const int k = (int)(t % nr);
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += C[row * ld + j] * (double)b[(int64_t)j * nr + k];
  y[t] = (T)s;
}

template <typename T, int KT>
struct __attribute__((aligned(sizeof(T) * KT > 16 ? 16 : sizeof(T) * KT))) VecT {
  T v[KT];
};

// Patch solves for nr right-hand sides: one 256-thread workgroup per patch and
// chunk of C right-hand sides (C a multiple of KT).  The patch's right-hand
// sides sit in LDS as an m x C block; thread t owns velocity row t / G
// (G = C / KT) for the KT right-hand sides of group t % G, keeps their sums in
// registers and reads its row of the factor block once per KT right-hand
// sides.  The factor record (element q of patch p at foff[p] + q * fstride[p])
// is staged in LDS (STAGE) or, when too large, read from global memory; the
// G threads of a row read the same address.  Y holds the result of slot s of
// patch p at (off[p] + s) * nr + k.
template <typename T, int KT, bool STAGE>
__global__ void __launch_bounds__(256) k_vanka_apply_nr(int64_t np, int nr, int C, const int64_t* __restrict__ off,
                                                       const int4* __restrict__ dims,
                                                       const int64_t* __restrict__ foff,
                                                       const int64_t* __restrict__ fstride,
                                                       const int* __restrict__ dofs, const T* __restrict__ fac,
                                                       const T* __restrict__ r, T* __restrict__ Y, int max_m,
                                                       int64_t max_f, int layout) {
  extern __shared__ unsigned char smem_raw[];
  T* sb = reinterpret_cast<T*>(smem_raw);   // max_m x C
  T* st = sb + (int64_t)max_m * C;          // MAX_NS x C: Uhat^T b_u + b_p
  T* syp = st + MAX_NS * C;                 // MAX_NS x C: y_p
  T* sf = syp + MAX_NS * C;                 // record (STAGE)
  int* sd = reinterpret_cast<int*>(sf + (STAGE ? max_f : 0));  // patch DoFs
  const int64_t p = blockIdx.x;
  if (p >= np) return;
  const int tid = threadIdx.x;
  const int k0 = blockIdx.y * C;
  const int4 d = dims[p];
  const int n0 = d.x, n1 = d.y, n2 = d.z;
  const int nv = n0 + n1 + n2, ns = d.w, m = nv + ns;
  const int full = layout & LAYOUT_FULL;
  const int64_t a1 = comp_offset(1, n0, n1, layout), a2 = comp_offset(2, n0, n1, layout);
  const int64_t uo = vel_entries(n0, n1, n2, layout), so = uo + (int64_t)nv * ns;
  const int64_t nf = so + (int64_t)ns * (ns + 1) / 2;
  const int64_t o = off[p], f0 = foff[p], fs = fstride[p];
  for (int j = tid; j < m; j += 256) sd[j] = dofs[o + j];
  if (STAGE)
    for (int64_t q = tid; q < nf; q += 256) sf[q] = fac[f0 + q * fs];
  __syncthreads();
  for (int idx = tid; idx < m * C; idx += 256) {
    const int j = idx / C, k = idx - j * C;
    sb[idx] = k0 + k < nr ? r[(int64_t)sd[j] * nr + k0 + k] : (T)0;
  }
  __syncthreads();
  auto F = [&](int64_t q) -> T { return STAGE ? sf[q] : fac[f0 + q * fs]; };
  // t = Uhat^T b_u + b_p, then y_p = S^-1 t
  for (int idx = tid; idx < ns * C; idx += 256) {
    const int s = idx / C, k = idx - s * C;
    T acc = sb[(nv + s) * C + k];
    for (int q = 0; q < nv; ++q) acc += F(uo + (int64_t)s * nv + q) * sb[q * C + k];
    st[idx] = acc;
  }
  __syncthreads();
  for (int idx = tid; idx < ns * C; idx += 256) {
    const int s = idx / C, k = idx - s * C;
    T acc = 0;
    for (int q = 0; q < ns; ++q) acc += F(so + packed_index(s, q)) * st[q * C + k];
    syp[idx] = acc;
    if (k0 + k < nr) Y[(o + nv + s) * nr + k0 + k] = acc;
  }
  __syncthreads();
  // x_u = A^-1 b_u + Uhat y_p, row by row
  const int G = C / KT;
  const int kg = tid % G;
  for (int row = tid / G; row < nv; row += 256 / G) {
    int cs, n, i;
    int64_t ao;
    if (row < n0) {
      cs = 0, n = n0, i = row, ao = 0;
    } else if (row < n0 + n1) {
      cs = n0, n = n1, i = row - n0, ao = a1;
    } else {
      cs = n0 + n1, n = n2, i = row - n0 - n1, ao = a2;
    }
    T acc[KT];
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) acc[kk] = 0;
    const T* bcol = sb + kg * KT;
    if (full) {  // entry (i, j) at j n + i: the threads of a row sweep read consecutive rows
      for (int j = 0; j < n; ++j) {
        const T a = F(ao + (int64_t)j * n + i);
        const VecT<T, KT> bv = *reinterpret_cast<const VecT<T, KT>*>(bcol + (cs + j) * C);
#pragma unroll
        for (int kk = 0; kk < KT; ++kk) acc[kk] += a * bv.v[kk];
      }
    }
    // j < i: packed entries i (i + 1) / 2 + j are contiguous
    const int64_t base = ao + (int64_t)i * (i + 1) / 2;
    for (int j = 0; j < (full ? 0 : i); ++j) {
      const T a = F(base + j);
      const VecT<T, KT> bv = *reinterpret_cast<const VecT<T, KT>*>(bcol + (cs + j) * C);
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) acc[kk] += a * bv.v[kk];
    }
    // j >= i: entry at j (j + 1) / 2 + i
    int64_t q = base + i;
    for (int j = i; j < (full ? 0 : n); ++j) {
      const T a = F(q);
      q += j + 1;
      const VecT<T, KT> bv = *reinterpret_cast<const VecT<T, KT>*>(bcol + (cs + j) * C);
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) acc[kk] += a * bv.v[kk];
    }
    for (int s = 0; s < ns; ++s) {
      const T u = F(uo + (int64_t)s * nv + row);
      const VecT<T, KT> yv = *reinterpret_cast<const VecT<T, KT>*>(syp + s * C + kg * KT);
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) acc[kk] += u * yv.v[kk];
    }
    T* yrow = Y + (o + row) * nr + k0 + kg * KT;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk)
      if (k0 + kg * KT + kk < nr) yrow[kk] = acc[kk];
  }
}

// x[j, k] (+)= omega / count_j * sum of the patch values held for DoF j (slot-major map)
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_pull_ell_nr(int n, int nr, int nrp, int width,
                                                           const int* __restrict__ pos, const T* __restrict__ Y,
                                                           T omega, T* __restrict__ x, int accumulate) {
  // thread (DoF j, right-hand side k): k = tid % nrp for the whole kernel
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  const int64_t j = (int64_t)blockIdx.x * ng + g;
  if (j >= n || k >= nr) return;
  const int64_t t = j * nr + k;
  T acc = 0;
  int cnt = 0;
  int s = 0;
  for (; s + 3 < width; s += 4) {  // four gathers in flight, sums in slot order
    int q[4];
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = pos[(int64_t)(s + u) * n + j];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = q[u] >= 0 ? Y[(int64_t)q[u] * nr + k] : (T)0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q[u] >= 0) {
        acc += v[u];
        ++cnt;
      }
  }
  for (; s < width; ++s) {
    const int q = pos[(int64_t)s * n + j];
    if (q >= 0) {
      acc += Y[(int64_t)q * nr + k];
      ++cnt;
    }
  }
  if (cnt == 0) {
    if (!accumulate) x[t] = 0;
    return;
  }
  const T v = omega * acc / (T)cnt;
  x[t] = accumulate ? x[t] + v : v;
}

// x[j, k] (+)= omega W_j sum ... (CSR map); thread (DoF j, right-hand side k),
// the patch values of a DoF gathered four at a time (summed in map order)
template <typename T>
__global__ void __launch_bounds__(256) k_vanka_pull_nr(int n, int nr, int nrp, const int* __restrict__ inv_ptr,
                                                       const int* __restrict__ inv_pos, const T* __restrict__ Y,
                                                       const T* __restrict__ w, T omega, T* __restrict__ x,
                                                       int accumulate) {
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  const int64_t j = (int64_t)blockIdx.x * ng + g;
  if (j >= n || k >= nr) return;
  const int64_t t = j * nr + k;
  const int q1 = inv_ptr[j + 1];
  int q = inv_ptr[j];
  T acc = 0;
  for (; q + 3 < q1; q += 4) {
    int pq[4];
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pq[u] = inv_pos[q + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = Y[(int64_t)pq[u] * nr + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u];
  }
  for (; q < q1; ++q) acc += Y[(int64_t)inv_pos[q] * nr + k];
  const T v = omega * w[j] * acc;
  x[t] = accumulate ? x[t] + v : v;
}

// per-column partial dot products of w and v (or w and w) over a block's rows,
// w -= a_k vprev when vprev is given, a_k = sum of the previous partials of
// column k.  Block layout: 256 threads = (256 / nrp) row groups x nrp columns.
__global__ void __launch_bounds__(256) k_mgs_step_nr(int64_t n, int nr, int nrp, double* __restrict__ w,
                                                    const double* __restrict__ vprev, double* __restrict__ hprev,
                                                    const double* __restrict__ prev_partial,
                                                    const double* __restrict__ vnext,
                                                    double* __restrict__ partial_out, int mode) {
  __shared__ double sh[256];
  __shared__ double sa[64];
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  const bool col = k < nr;
  double a = 0.0;
  if (prev_partial) {  // h of the previous step: the block's groups split the partial sums
    double t = 0.0;
    if (col)
      for (unsigned b = g; b < gridDim.x; b += ng) t += prev_partial[(int64_t)b * nr + k];
    sh[threadIdx.x] = t;
    __syncthreads();
    if (g == 0 && col) {
      double u = 0.0;
      for (int q = 0; q < ng; ++q) u += sh[q * nrp + k];
      sa[k] = u;
      if (blockIdx.x == 0) hprev[k] = u;
    }
    __syncthreads();
    if (col) a = sa[k];
  }
  double s = 0.0;
  if (col) {
    const int64_t stride = (int64_t)gridDim.x * ng;
    int64_t i = (int64_t)blockIdx.x * ng + g;
    for (; i + 3 * stride < n; i += 4 * stride) {  // four rows in flight
      double wi[4], vn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t e = (i + u * stride) * nr + k;
        wi[u] = w[e];
        if (vprev) wi[u] -= a * vprev[e];
        vn[u] = mode == 0 ? vnext[e] : wi[u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (vprev) w[(i + u * stride) * nr + k] = wi[u];
        s += wi[u] * vn[u];
      }
    }
    for (; i < n; i += stride) {
      const int64_t e = i * nr + k;
      double wi = w[e];
      if (vprev) {
        wi -= a * vprev[e];
        w[e] = wi;
      }
      s += wi * (mode == 0 ? vnext[e] : wi);
    }
  }
  __syncthreads();
  sh[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && col) {
    double t = 0.0;
    for (int q = 0; q < ng; ++q) t += sh[q * nrp + k];
    partial_out[(int64_t)blockIdx.x * nr + k] = t;
  }
}

// v[:, k] = w[:, k] / sqrt(sum of partials of column k); block 0 stores the norms
__global__ void __launch_bounds__(256) k_normalize_nr(int64_t n, int nr, const double* __restrict__ partial, int nb,
                                                     double* __restrict__ hout, const double* __restrict__ w,
                                                     double* __restrict__ v) {
  __shared__ double nrm[64];
  __shared__ double sh[256];
  // each thread keeps one column k (tid % nrp) for the whole kernel: no index
  // division per element
  const int nrp = nr <= 1 ? 1 : 1 << (32 - __clz(nr - 1));
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  {  // the block's threads split the partial sums of each column
    double t = 0.0;
    if (k < nr)
      for (int b = g; b < nb; b += ng) t += partial[(int64_t)b * nr + k];
    sh[threadIdx.x] = t;
    __syncthreads();
    if (g == 0 && k < nr) {
      double u = 0.0;
      for (int q = 0; q < ng; ++q) u += sh[q * nrp + k];
      nrm[k] = sqrt(u);
      if (blockIdx.x == 0) hout[k] = nrm[k];
    }
    __syncthreads();
  }
  if (k >= nr) return;
  const double q = nrm[k];
  const int64_t stride = (int64_t)gridDim.x * ng;
  for (int64_t r = (int64_t)blockIdx.x * ng + g; r < n; r += stride) {
    const int64_t e = r * nr + k;
    v[e] = q != 0.0 ? w[e] / q : 0.0;
  }
}

// Classical Gram-Schmidt for the FGMRES Arnoldi step, for nr interleaved
// columns (entry (row, k) at row * nr + k; nr = 1 for one right-hand side).
// It yields the same Hessenberg column as modified Gram-Schmidt in exact
// arithmetic with about half the vector traffic: all the dots in one sweep,
// then one update.  k_cgs_dots_nr: part[(i * gridDim.x + b) * nr + k] = block
// b's share of v_i(:, k) . w(:, k), at most kCgsChunk basis vectors per sweep
// of w.
constexpr int kCgsChunk = 16;

// Sum of v over the threads of a 256-thread block that hold column k = tid %
// nrp (nrp a power of two <= 64): shuffles over the lanes of one column in a
// wavefront, then the four wavefronts through red[u][wave][k].  Valid in the
// threads tid < nrp after the caller's __syncthreads.
__device__ __forceinline__ void cgs_wave_part(double v, int nrp, double (*red)[4][64], int u) {
  for (int o = WAVE / 2; o >= nrp; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  if (lane < nrp) red[u][wv][lane] = v;
}

// One chunk of NA basis vectors v_i0 .. v_{i0+NA-1} per launch (the width a
// template argument, so the unrolled loop issues its NA loads together).
template <int NA>
__global__ void __launch_bounds__(256) k_cgs_dots_nr(int64_t n, int nr, int nrp, int i0, const double* __restrict__ V,
                                                    const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[NA][4][64];
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  const bool col = k < nr;
  const int64_t stride = (int64_t)gridDim.x * ng, nn = n * nr;
  const double* Vc = V + (int64_t)i0 * nn;
  double acc[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) acc[u] = 0.0;
  if (col)
    for (int64_t r = (int64_t)blockIdx.x * ng + g; r < n; r += stride) {
      const int64_t e = r * nr + k;
      const double we = w[e];
#pragma unroll
      for (int u = 0; u < NA; ++u) acc[u] += Vc[(int64_t)u * nn + e] * we;
    }
#pragma unroll
  for (int u = 0; u < NA; ++u) cgs_wave_part(acc[u], nrp, red, u);
  __syncthreads();
  for (int t = threadIdx.x; t < NA * nrp; t += 256) {
    const int u = t / nrp, kk = t % nrp;
    if (kk < nr)
      part[((int64_t)(i0 + u) * gridDim.x + blockIdx.x) * nr + kk] =
          red[u][0][kk] + red[u][1][kk] + red[u][2][kk] + red[u][3][kk];
  }
}

// h[i * nr + k] = sum over the nb blocks of the dot partials; one wavefront per (i, k)
__global__ void __launch_bounds__(64) k_cgs_final_nr(int nb, int nr, int j1, const double* __restrict__ part,
                                                     double* __restrict__ h) {
  const int t = blockIdx.x;  // (i, k)
  if (t >= j1 * nr) return;
  const int i = t / nr, k = t % nr;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += WAVE) s += part[((int64_t)i * nb + b) * nr + k];
  s = wave_sum(s);
  if (threadIdx.x == 0) h[t] = s;
}

// w(:, k) -= sum_{i0 <= i < i0 + NA} h[i * nr + k] v_i(:, k), one chunk per
// launch; with last set, partial_out[b * nr + k] = block b's share of
// |w(:, k)|^2 (the layout k_normalize_nr reduces)
template <int NA>
__global__ void __launch_bounds__(256) k_cgs_update_nr(int64_t n, int nr, int nrp, int i0, int last,
                                                      const double* __restrict__ V, const double* __restrict__ h,
                                                      double* __restrict__ w, double* __restrict__ partial_out) {
  __shared__ double red[1][4][64];
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  const bool col = k < nr;
  const int64_t stride = (int64_t)gridDim.x * ng, nn = n * nr;
  const double* Vc = V + (int64_t)i0 * nn;
  double hk[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) hk[u] = col ? h[(i0 + u) * nr + k] : 0.0;
  double s = 0.0;
  if (col)
    for (int64_t r = (int64_t)blockIdx.x * ng + g; r < n; r += stride) {
      const int64_t e = r * nr + k;
      double we = w[e];
#pragma unroll
      for (int u = 0; u < NA; ++u) we -= hk[u] * Vc[(int64_t)u * nn + e];
      w[e] = we;
      s += we * we;
    }
  if (!last) return;  // uniform over the launch
  cgs_wave_part(s, nrp, red, 0);
  __syncthreads();
  if (threadIdx.x < nr)
    partial_out[(int64_t)blockIdx.x * nr + threadIdx.x] =
        red[0][0][threadIdx.x] + red[0][1][threadIdx.x] + red[0][2][threadIdx.x] + red[0][3][threadIdx.x];
}

// out[k] = sum_b partial[b * nr + k] (sqrt if take_sqrt)
__global__ void k_reduce_final_nr(int nb, int nr, const double* __restrict__ partial, double* __restrict__ out,
                                  int take_sqrt) {
  const int k = threadIdx.x;
  if (k >= nr) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += partial[(int64_t)b * nr + k];
  out[k] = take_sqrt ? sqrt(t) : t;
}

// v[:, k] = r[:, k] / beta[k] (0 when beta[k] == 0)
// v[:, k] *= c[k] (n x nr, right-hand side fastest)
__global__ void k_scale_cols_inplace(int64_t n, int nr, const double* __restrict__ c, double* __restrict__ v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) v[t] *= c[t % nr];
}

__global__ void k_scale_cols(int64_t n, int nr, const double* __restrict__ beta, const double* __restrict__ r,
                             double* __restrict__ v) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) {
    const double q = beta[t % nr];
    v[t] = q != 0.0 ? r[t] / q : 0.0;
  }
}

// x[:, k] += sum_q y[q * nr + k] Z_q[:, k]
__global__ void k_update_x_nr(int64_t n, int nr, int kmax, const double* __restrict__ Z, const double* __restrict__ y,
                              double* __restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nr) return;
  const int k = (int)(t % nr);
  double s = x[t];
  for (int q = 0; q < kmax; ++q) s += y[(int64_t)q * nr + k] * Z[(int64_t)q * n * nr + t];
  x[t] = s;
}

// x[i, k] *= (i < nsplit ? su[k] : sp[k])  (field scaling of nr columns)
__global__ void k_scale_rows_nr(int64_t n, int nr, int64_t nsplit, const double* __restrict__ su,
                                const double* __restrict__ sp, double* __restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) {
    const int64_t i = t / nr;
    const int k = (int)(t % nr);
    x[t] *= (i < nsplit ? su[k] : sp[k]);
  }
}

// x[idx[q], k] *= c[k]
__global__ void k_scale_idx_nr(int64_t n, int nr, const int64_t* __restrict__ idx, const double* __restrict__ c,
                               double* __restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) x[idx[t / nr] * nr + t % nr] *= c[t % nr];
}

// x[i, k] += c_k for the rows i of one block (zero-mean pressure shift)
__global__ void k_add_cols(int64_t n, int nr, const double* __restrict__ c, double* __restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * nr) x[t] += c[t % nr];
}

// partial[b * nr + k] = sum over a block's rows of w[i] * x[i, k] (weighted column sums)
__global__ void __launch_bounds__(256) k_wdot_nr(int64_t n, int nr, int nrp, const double* __restrict__ w,
                                                const double* __restrict__ x, double* __restrict__ partial) {
  __shared__ double sh[256];
  const int k = threadIdx.x % nrp, g = threadIdx.x / nrp, ng = 256 / nrp;
  double s = 0.0;
  if (k < nr)
    for (int64_t i = (int64_t)blockIdx.x * ng + g; i < n; i += (int64_t)gridDim.x * ng) s += w[i] * x[i * nr + k];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && k < nr) {
    double t = 0.0;
    for (int q = 0; q < ng; ++q) t += sh[q * nrp + k];
    partial[(int64_t)blockIdx.x * nr + k] = t;
  }
}

// z = x + y
template <typename T>
__global__ void k_add(int64_t n, const T* __restrict__ x, const T* __restrict__ y, T* __restrict__ z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = x[i] + y[i];
}

// x += y + z
template <typename T>
__global__ void k_add3(int64_t n, T* __restrict__ x, const T* __restrict__ y, const T* __restrict__ z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += y[i] + z[i];
}

// the sums of row i of every component over the columns j = g, g + G, ...:
// component count and storage are template arguments, so the unrolled loop
// holds no branch and its loads are issued together.  Every lane runs the
// same columns (a split at the diagonal would give the lanes of a wavefront
// different trip counts); packed offsets in 32-bit unsigned arithmetic.
template <typename T, int NCO, bool FULL>
__device__ __forceinline__ void shared_row_sums(const T* sb, const T* A, int n, int i, int g, int G,
                                                T (&acc)[3]) {
  if (FULL) {
    const T* a = A + (int64_t)g * n + i;
    const int64_t step = (int64_t)G * n;
#pragma unroll 8
    for (int j = g; j < n; j += G, a += step) {
      const T v = *a;
#pragma unroll
      for (int c = 0; c < NCO; ++c) acc[c] += v * sb[c * n + j];
    }
    return;
  }
  const unsigned ui = (unsigned)i;
#pragma unroll 8
  for (int j = g; j < n; j += G) {
    const unsigned lo = min(ui, (unsigned)j), hi = max(ui, (unsigned)j);
    const T v = A[((hi * (hi + 1u)) >> 1) + lo];
#pragma unroll
    for (int c = 0; c < NCO; ++c) acc[c] += v * sb[c * n + j];
  }
}

// the same with b interleaved (b_c[j] at bi[j NCO + c]): the NCO reads of a
// column sit at one address plus immediate offsets
template <typename T, int NCO, bool FULL>
__device__ __forceinline__ void shared_row_sums_il(const T* bi, const T* A, int n, int i, int g, int G,
                                                   T (&acc)[3]) {
  const T* bj = bi + g * NCO;
  if (FULL) {
    const T* a = A + (int64_t)g * n + i;
    const int64_t step = (int64_t)G * n;
#pragma unroll 8
    for (int j = g; j < n; j += G, a += step, bj += G * NCO) {
      const T v = *a;
#pragma unroll
      for (int c = 0; c < NCO; ++c) acc[c] += v * bj[c];
    }
    return;
  }
  const unsigned ui = (unsigned)i;
#pragma unroll 8
  for (int j = g; j < n; j += G, bj += G * NCO) {
    const unsigned lo = min(ui, (unsigned)j), hi = max(ui, (unsigned)j);
    const T v = A[((hi * (hi + 1u)) >> 1) + lo];
#pragma unroll
    for (int c = 0; c < NCO; ++c) acc[c] += v * bj[c];
  }
}

// y_u = A^-1 b_u when one block A (n x n, LAYOUT_SHARED) serves all
// nco = nv / n velocity components: G = TPB / n thread groups (one when
// n >= TPB); thread (g, i) sums row i of every component over the columns
// j = g, g + G, ..., so each block entry is read once for all components.
// After a barrier, groups 1..G-1 leave their sums in part ((G - 1) nco n
// values, which may be the LDS copy of A itself, no longer read) and group 0
// adds them in group order.  split (n a row or two above TPB / 2, part in the
// LDS copy of A): two groups over the first TPB / 2 rows, so that no
// wavefront runs a whole row for one live lane, and each remaining row summed
// by the whole workgroup (its wavefronts' sums added in wavefront order).
// Every thread of the workgroup calls it (it holds barriers).
template <typename T, int TPB>
__device__ __forceinline__ void vanka_shared_rows(const T* sb, T* sy, const T* A, T* part, int n, int nco,
                                                  int full, bool split) {
  constexpr int H = TPB / 2;
  __shared__ T xred[TPB / WAVE][2][3];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int rows = split ? H : n;
  const int G = split ? 2 : n >= TPB ? 1 : TPB / n;
  const int g = G == 1 ? 0 : tid / rows;
  const int i0 = G == 1 ? tid : tid - g * rows;
  T acc[3] = {0, 0, 0};
  if (G == 1) {  // a thread per row (and more rows per thread): results straight to sy
    for (int i = i0; i < n; i += TPB) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = 0;
      if (nco == 3 && full) shared_row_sums<T, 3, true>(sb, A, n, i, 0, 1, acc);
      else if (nco == 3) shared_row_sums<T, 3, false>(sb, A, n, i, 0, 1, acc);
      else if (full) shared_row_sums<T, 2, true>(sb, A, n, i, 0, 1, acc);
      else shared_row_sums<T, 2, false>(sb, A, n, i, 0, 1, acc);
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < nco) sy[c * n + i] = acc[c];
    }
    return;
  }
  // b_u interleaved by component into sy (free until the results land there)
  for (int t = tid; t < nco * n; t += TPB) {
    const int c = t / n, i = t - c * n;
    sy[i * nco + c] = sb[t];
  }
  __syncthreads();
  if (g < G) {
    if (nco == 3 && full) shared_row_sums_il<T, 3, true>(sy, A, n, i0, g, G, acc);
    else if (nco == 3) shared_row_sums_il<T, 3, false>(sy, A, n, i0, g, G, acc);
    else if (full) shared_row_sums_il<T, 2, true>(sy, A, n, i0, g, G, acc);
    else shared_row_sums_il<T, 2, false>(sy, A, n, i0, g, G, acc);
  }
  if (split)  // rows H .. n - 1 (at most two): a column per thread, then wavefront sums
    for (int e = 0; e < 2; ++e) {
      const int r = H + e;
      if (r >= n) break;  // uniform
      T pc[3] = {0, 0, 0};
      for (int j = tid; j < n; j += TPB) {
        const int lo = min(r, j), hi = max(r, j);
        const T v = full ? A[(int64_t)j * n + r] : A[((unsigned)hi * (unsigned)(hi + 1) >> 1) + lo];
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (c < nco) pc[c] += v * sy[j * nco + c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T w = wave_sum(pc[c]);
        if (lane == 0) xred[wv][e][c] = w;
      }
    }
  {
    __syncthreads();  // every read of A and of the interleaved b done: part and sy may be overwritten
    if (g >= 1 && g < G)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c < nco) part[(int64_t)(g - 1) * nco * n + c * n + i0] = acc[c];
    __syncthreads();
    if (g == 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c >= nco) continue;
        T v = acc[c];
        for (int q = 1; q < G; ++q) v += part[(int64_t)(q - 1) * nco * n + c * n + i0];
        sy[c * n + i0] = v;
      }
    if (split && tid >= H && tid < H + (n - H) * nco) {  // rows H .. n - 1
      const int e = (tid - H) / nco, c = (tid - H) - e * nco;
      T v = xred[0][e][c];
      for (int q = 1; q < TPB / WAVE; ++q) v += xred[q][e][c];
      sy[c * n + H + e] = v;
    }
  }
}

// The seed part of a patch solve, once y_u = A^-1 b_u is in sy (Uhat and S^-1
// at U, read where they are: LDS or memory): t = Uhat^T b_u + b_p,
// y_p = S^-1 t, x_u = y_u + Uhat y_p, written to the patch's output slots.
// Every thread of the workgroup calls it (it holds barriers).
template <typename T, int TPB>
__device__ __forceinline__ void vanka_patch_seeds(const T* sb, const T* sy, const T* U, T (*sred)[MAX_NS],
                                                  int nv, int ns, int64_t o, T* __restrict__ Y, int64_t yshift) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const T* Si = U + (int64_t)nv * ns;
  // seeds: t = Uhat^T b_u + b_p, y_p = S^-1 t.  The seed arrays are indexed
  // only by unrolled loop counters (ns <= MAX_NS as a predicate), so they stay
  // in registers without index-dependent branches.
  T t[MAX_NS], yp[MAX_NS];
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    t[s] = 0;
    if (s < ns) {
      T part = 0;
      for (int k = tid; k < nv; k += TPB) part += U[(int64_t)s * nv + k] * sb[k];
      part = wave_sum(part);
      if (TPB == WAVE) t[s] = part + sb[nv + s];
      else if (lane == 0) sred[wv][s] = part;
    }
  }
  if (TPB > WAVE) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s < ns) {
        T acc = sred[0][s];
        for (int q = 1; q < TPB / WAVE; ++q) acc += sred[q][s];
        t[s] = acc + sb[nv + s];
      }
  }
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    T acc = 0;
#pragma unroll
    for (int q = 0; q < MAX_NS; ++q)
      if (s < ns && q < ns) acc += Si[packed_index(s, q)] * t[q];
    yp[s] = acc;
  }
  __syncthreads();
  for (int row = tid; row < nv; row += TPB) {
    T acc = sy[row];
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s < ns) acc += U[(int64_t)s * nv + row] * yp[s];
    Y[o - yshift + row] = acc;
  }
  if (tid < ns) {
    T v = 0;
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s == tid) v = yp[s];
    Y[o - yshift + nv + tid] = v;
  }
}


// ---------------------------------------------------------------------------
// The patch solve of the workgroup kernels, once the right-hand side b (sb)
// and the factor record (sf) are in place: y_u = A^-1 b_u one row per thread,
// t = Uhat^T b_u + b_p, y_p = S^-1 t, x_u = y_u + Uhat y_p, written to the
// patch's output slots.  Every thread of the workgroup calls it (it holds
// barriers).
template <typename T, int TPB>
__device__ __forceinline__ void vanka_patch_compute(const T* sb, T* sy, const T* sf, T (*sred)[MAX_NS], T* spart,
                                                    int4 d, int64_t o, int64_t ua, int layout, T* __restrict__ Y,
                                                    int64_t yshift, bool stage_rec) {
  const int tid = threadIdx.x;
  const int nv = d.x + d.y + d.z, ns = d.w;
  const int nc[3] = {d.x, d.y, d.z};
  const int full = layout & LAYOUT_FULL;
  if (layout & LAYOUT_SHARED) {
    // the partial sums go to the staged copy of A when they fit there (the
    // host then allocates no separate area)
    const int n = d.x;
    // a row or two above TPB / 2: two thread groups over the first TPB / 2 rows
    // (their partial sums in the staged copy of A)
    const bool split = TPB >= 2 * WAVE && n > TPB / 2 && n <= TPB / 2 + 2 && stage_rec &&
                       (int64_t)nv <= blk_size(n, full);
    const int G = split ? 2 : n >= TPB ? 1 : TPB / n;
    const bool in_rec = stage_rec && (int64_t)(G - 1) * nv <= blk_size(n, full);
    vanka_shared_rows<T, TPB>(sb, sy, sf, in_rec ? const_cast<T*>(sf) : spart, n, nv / n, full, split);
  }
  // y_u = A^-1 b_u, one row per thread
  for (int row = tid; row < ((layout & LAYOUT_SHARED) ? 0 : nv); row += TPB) {
    int c = 0, cs = 0;
    int64_t ao = 0;
    while (row >= cs + nc[c]) {
      ao += blk_size(nc[c], full);
      cs += nc[c];
      ++c;
    }
    const int i = row - cs;
    const T* A = sf + ao;
    T acc = 0;
    if (full)  // entry (i, j) at j n + i: consecutive threads read consecutive values
      for (int j = 0; j < nc[c]; ++j) acc += A[(int64_t)j * nc[c] + i] * sb[cs + j];
    else
      for (int j = 0; j < nc[c]; ++j) acc += A[packed_index(i, j)] * sb[cs + j];
    sy[row] = acc;
  }
  vanka_patch_seeds<T, TPB>(sb, sy, sf + ua, sred, nv, ns, o, Y, yshift);
}

// additive Vanka: one workgroup of TPB threads (one or four wavefronts) per
// patch, patch data staged through LDS.  Writes the patch solution
// x_i = K_i^-1 V_i r into Y at the patch's offset.  Large patches take four
// wavefronts: four times the loads in flight while the record is staged and
// one velocity row per thread afterwards.
template <typename T, bool STAGE, int TPB, bool NT = false, int UL = 32>
__global__ void __launch_bounds__(TPB) k_vanka_apply(int64_t np, const int64_t* __restrict__ off,
                                                    const int4* __restrict__ dims,
                                                    const int64_t* __restrict__ foff,
                                                    const int* __restrict__ dofs, const T* __restrict__ fac,
                                                    const T* __restrict__ r, T* __restrict__ Y, int max_m,
                                                    int64_t yshift, int layout, int spart_len) {
  extern __shared__ unsigned char smem_raw[];
  T* sb = reinterpret_cast<T*>(smem_raw);
  T* sy = sb + max_m;
  T* spart = sy + max_m;  // partial row sums of the shared-block layout (spart_len values: 0 or 3 TPB)
  __shared__ T sred[TPB / WAVE][MAX_NS];
  const int64_t p = blockIdx.x;
  if (p >= np) return;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int4 d = dims[p];
  const int nv = d.x + d.y + d.z, ns = d.w, m = nv + ns;
  const int64_t o = off[p];
  // record length from the shape (foff holds per-patch base offsets only)
  const int64_t f0 = foff[p];
  const int64_t ua = vel_entries(d.x, d.y, d.z, layout);
  const int64_t nf = ua + (int64_t)nv * ns + (int64_t)ns * (ns + 1) / 2;
  // Staged records: the first UL * TPB values are requested before the
  // DoF-list -> vector gather, so that the gather's two dependent round trips
  // overlap the record's loads (UL independent loads in flight per thread;
  // the host picks UL to cover the level's longest record where it can).
  T* st = spart + spart_len;
  T v[UL];
  // Loads and stores past the end of the record (or of the DoF list) are
  // clamped to its last element instead of guarded: no branch per load, and
  // the extra stores write that element's own value again.
  const int lastf = (int)min<int64_t>(nf, (int64_t)UL * TPB) - 1;
  if (STAGE) {
    const T* src = fac + f0;
#pragma unroll
    for (int u = 0; u < UL; ++u) v[u] = ldv<NT>(src + min(u * TPB + tid, lastf));
  }
  // gather: all index loads first, then all value loads (several in flight)
  for (int k0 = 0; k0 < m; k0 += 4 * TPB) {
    const int lastm = min(m - k0, 4 * TPB) - 1;
    int idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) idx[u] = dofs[o + k0 + min(u * TPB + tid, lastm)];
    T g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = r[idx[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) sb[k0 + min(u * TPB + tid, lastm)] = g[u];
  }
  const T* sf;
  if (STAGE) {
#pragma unroll
    for (int u = 0; u < UL; ++u) st[min(u * TPB + tid, lastf)] = v[u];
    // the rest of a record longer than UL * TPB values, UL loads in flight per thread
    for (int64_t k0 = (int64_t)UL * TPB; k0 < nf; k0 += (int64_t)UL * TPB) {
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int64_t k = k0 + (int64_t)u * TPB + tid;
        v[u] = k < nf ? ldv<NT>(&fac[f0 + k]) : (T)0;
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int64_t k = k0 + (int64_t)u * TPB + tid;
        if (k < nf) st[k] = v[u];
      }
    }
    sf = st;
  } else {
    sf = fac + f0;  // record too large for LDS: read it from memory
  }
  __syncthreads();
  vanka_patch_compute<T, TPB>(sb, sy, sf, sred, spart, d, o, ua, layout, Y, yshift, STAGE);
}

// additive Vanka, the workgroup kernel made persistent and pipelined: a
// workgroup solves patches p, p + gridDim.x, ... and, before solving patch p
// from LDS, requests the next patch's record (UL values per thread, the whole
// record: UL TPB >= its length) and DoF indices into registers, then its
// right-hand-side gather after the solve, so that a patch's loads overlap the
// previous patch's solve.  Requires records staged in LDS and m <= 4 TPB.
template <typename T, int TPB, bool NT, int UL>
__global__ void __launch_bounds__(TPB) k_vanka_pipe(int64_t np, const int64_t* __restrict__ off,
                                                   const int4* __restrict__ dims,
                                                   const int64_t* __restrict__ foff,
                                                   const int* __restrict__ dofs, const T* __restrict__ fac,
                                                   const T* __restrict__ r, T* __restrict__ Y, int max_m,
                                                   int64_t yshift, int layout, int spart_len) {
  extern __shared__ unsigned char smem_raw[];
  T* sb = reinterpret_cast<T*>(smem_raw);
  T* sy = sb + max_m;
  T* spart = sy + max_m;
  T* st = spart + spart_len;
  __shared__ T sred[TPB / WAVE][MAX_NS];
  const int tid = threadIdx.x;
  int64_t p = blockIdx.x;
  if (p >= np) return;
  T v[UL], g[4];
  int idx[4];
  int m_next = 0, nf_next = 0;
  // the record and DoF-index loads of patch q (m_next, nf_next: its sizes)
  auto request = [&](int64_t q) {
    const int4 d = dims[q];
    const int nvq = d.x + d.y + d.z;
    m_next = nvq + d.w;
    nf_next = (int)record_entries(d.x, d.y, d.z, d.w, layout);
    const T* f = fac + foff[q];
#pragma unroll
    for (int u = 0; u < UL; ++u) v[u] = ldv<NT>(f + min(u * TPB + tid, nf_next - 1));
    const int* dq = dofs + off[q];
#pragma unroll
    for (int u = 0; u < 4; ++u) idx[u] = dq[min(u * TPB + tid, m_next - 1)];
  };
  auto gather = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = r[idx[u]];
  };
  request(p);
  gather();
  for (; p < np; p += gridDim.x) {
    const int4 d = dims[p];
    const int64_t o = off[p];
    const int64_t ua = vel_entries(d.x, d.y, d.z, layout);
    const int m = m_next, nf = nf_next;
    __syncthreads();  // the previous patch's solve is done with LDS
#pragma unroll
    for (int u = 0; u < UL; ++u) st[min(u * TPB + tid, nf - 1)] = v[u];
#pragma unroll
    for (int u = 0; u < 4; ++u) sb[min(u * TPB + tid, m - 1)] = g[u];
    __syncthreads();
    const int64_t pn = p + gridDim.x;
    if (pn < np) request(pn);  // in flight during this patch's solve
    vanka_patch_compute<T, TPB>(sb, sy, st, sred, spart, d, o, ua, layout, Y, yshift, true);
    if (pn < np) gather();
  }
}

// additive Vanka for patches too large for LDS whose one packed A^-1 block
// serves NCO velocity components (LAYOUT_SHARED, n <= TPB rows): the block is
// streamed in panels of consecutive columns (a panel of packed columns is one
// contiguous range of the record, at most PL TPB values), each copied into LDS
// with coalesced loads; the next panel's loads are issued into registers
// before the current panel is used.  From a panel, thread group g of row i
// adds a_ij b_c[j] for its columns j >= i (j = g mod G, G = TPB / n groups;
// consecutive rows read consecutive LDS words), and wavefronts sum
// a_ij b_c[i] over i < j for the panel's columns (the transposed half, one
// column per wavefront at a time).  Then the seed part as in the other
// workgroup kernels.  Half the bytes of storing the block full.
template <typename T, int NCO, bool NT, int TPB, int PL>
__global__ void __launch_bounds__(TPB) k_vanka_panel(int64_t np, const int64_t* __restrict__ off,
                                                    const int4* __restrict__ dims,
                                                    const int64_t* __restrict__ foff,
                                                    const int* __restrict__ dofs, const T* __restrict__ fac,
                                                    const T* __restrict__ r, T* __restrict__ Y, int max_m,
                                                    int64_t yshift) {
  extern __shared__ unsigned char smem_raw[];
  T* sb = reinterpret_cast<T*>(smem_raw);  // b (m values)
  T* sy = sb + max_m;                      // column sums of the transposed half, then y_u
  T* pan = sy + max_m;                     // one panel (PL TPB values), then partial row sums
  __shared__ T sred[TPB / WAVE][MAX_NS];
  constexpr int CAP = PL * TPB, NW = TPB / WAVE;
  const int64_t p = blockIdx.x;
  if (p >= np) return;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int4 d = dims[p];
  const int n = d.x, nv = NCO * n, ns = d.w, m = nv + ns;
  const int64_t o = off[p];
  const T* A = fac + foff[p];
  auto tri = [](int j) { return (int)(((unsigned)j * (unsigned)(j + 1)) >> 1); };
  // last column + 1 of the panel that starts at column j0: at most CAP values
  auto panel_end = [&](int j0) {
    const double lim = (double)CAP + (double)tri(j0);
    int j1 = (int)((sqrt(8.0 * lim + 1.0) - 1.0) * 0.5);  // tri(j1) <= lim, up to rounding
    while (j1 > j0 && tri(j1) > lim) --j1;
    while (j1 < n && tri(j1 + 1) <= lim) ++j1;
    return min(max(j1, j0 + 1), n);
  };
  T pv[PL];
  int J0 = 0, J1 = panel_end(0);
  auto request = [&](int j0, int j1) {
    const T* src = A + tri(j0);
    const int last = tri(j1) - tri(j0) - 1;
#pragma unroll
    for (int u = 0; u < PL; ++u) pv[u] = ldv<NT>(src + min(u * TPB + tid, last));
  };
  request(J0, J1);
  // gather b (clamped, as in the other kernels)
  for (int k0 = 0; k0 < m; k0 += 4 * TPB) {
    const int lastm = min(m - k0, 4 * TPB) - 1;
    int idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) idx[u] = dofs[o + k0 + min(u * TPB + tid, lastm)];
    T g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = r[idx[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) sb[k0 + min(u * TPB + tid, lastm)] = g[u];
  }
  const int G = TPB / n;  // n <= TPB
  const int g = tid / n, i0 = tid - g * n;
  T acc[NCO];
#pragma unroll
  for (int c = 0; c < NCO; ++c) acc[c] = 0;
  for (;;) {
    const int j0 = J0, j1 = J1, base = tri(j0), cnt = tri(j1) - base;
    __syncthreads();  // the previous panel is done with
#pragma unroll
    for (int u = 0; u < PL; ++u) pan[min(u * TPB + tid, cnt - 1)] = pv[u];
    __syncthreads();
    if (j1 < n) {  // the next panel's loads, in flight while this one is used
      J0 = j1;
      J1 = panel_end(j1);
      request(J0, J1);
    }
    // row i0 over this panel's columns j >= i0 with j = g (mod G)
    if (g < G) {
      int j = max(j0, i0);
      j += (g - j % G + G) % G;
      for (; j < j1; j += G) {
        const T a = pan[tri(j) - base + i0];
#pragma unroll
        for (int c = 0; c < NCO; ++c) acc[c] += a * sb[c * n + j];
      }
    }
    // column j: sum over i < j of a_ij b_c[i], one wavefront per column
    for (int j = j0 + wv; j < j1; j += NW) {
      const T* col = pan + (tri(j) - base);
      T sc[NCO];
#pragma unroll
      for (int c = 0; c < NCO; ++c) sc[c] = 0;
      for (int i = lane; i < j; i += WAVE) {
        const T a = col[i];
#pragma unroll
        for (int c = 0; c < NCO; ++c) sc[c] += a * sb[c * n + i];
      }
#pragma unroll
      for (int c = 0; c < NCO; ++c) {
        const T v = wave_sum(sc[c]);
        if (lane == 0) sy[c * n + j] = v;
      }
    }
    if (j1 >= n) break;
  }
  // y_u: the row sums of all groups plus the column sums (partials of groups
  // 1..G-1 in the panel area, free now)
  __syncthreads();
  if (g >= 1 && g < G)
#pragma unroll
    for (int c = 0; c < NCO; ++c) pan[(g - 1) * nv + c * n + i0] = acc[c];
  __syncthreads();
  if (g == 0)
#pragma unroll
    for (int c = 0; c < NCO; ++c) {
      T v = acc[c] + sy[c * n + i0];
      for (int q = 1; q < G; ++q) v += pan[(q - 1) * nv + c * n + i0];
      sy[c * n + i0] = v;
    }
  __syncthreads();
  vanka_patch_seeds<T, TPB>(sb, sy, A + tri(n), sred, nv, ns, o, Y, yshift);
}

// additive Vanka, one wavefront per patch, for patches whose velocity blocks
// have at most 2 x 64 rows each (packed records, MAX_NS seeds at most).  No
// LDS: the packed A_c^-1 is streamed column by column straight into
// registers.  Lane i holds rows i and i + 64 of the block (b, y); column j of
// the packed upper triangle (entries i <= j, contiguous) arrives with entry i
// in lane i, which adds a_ij b_j to its own y_i (i < j, lane-local), and the
// wavefront sums a_ij b_i over i <= j into y_j (the transposed half).  Then
// t = Uhat^T b_u + b_p (one wavefront sum per seed), y_p = S^-1 t and
// x_u = y_u + Uhat y_p.  WPB patches per workgroup, one per wavefront.
template <typename T, bool NT, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_vanka_col(int64_t np, const int64_t* __restrict__ off,
                                                      const int4* __restrict__ dims,
                                                      const int64_t* __restrict__ foff,
                                                      const int* __restrict__ dofs, const T* __restrict__ fac,
                                                      const T* __restrict__ r, T* __restrict__ Y, int64_t yshift) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t p = (int64_t)blockIdx.x * WPB + threadIdx.x / WAVE;
  if (p >= np) return;  // whole wavefronts leave together
  const int4 d = dims[p];
  const int nc[3] = {d.x, d.y, d.z};
  const int nv = d.x + d.y + d.z, ns = d.w;
  const int64_t o = off[p];
  const T* A = fac + foff[p];
  // b: rows lane and lane + 64 of every component, and the seeds (lane s)
  T b0[3], b1[3];
  {
    int cs = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i0 = lane, i1 = lane + WAVE;
      const int k0 = i0 < nc[c] ? dofs[o + cs + i0] : -1;
      const int k1 = i1 < nc[c] ? dofs[o + cs + i1] : -1;
      b0[c] = k0 >= 0 ? r[k0] : (T)0;
      b1[c] = k1 >= 0 ? r[k1] : (T)0;
      cs += nc[c];
    }
  }
  const T bseed = lane < ns ? r[dofs[o + nv + lane]] : (T)0;
  T y0[3], y1[3];
  int64_t ao = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int n = nc[c];
    T a0 = 0, a1 = 0;  // y of rows lane, lane + 64
    const T* Ac = A + ao;
    for (int j = 0; j < n; ++j) {
      const T* col = Ac + (int64_t)j * (j + 1) / 2;
      const T e0 = lane <= j ? ldv<NT>(&col[lane]) : (T)0;
      const T e1 = lane + WAVE <= j ? ldv<NT>(&col[lane + WAVE]) : (T)0;
      const T bj = j < WAVE ? __shfl(b0[c], j) : __shfl(b1[c], j - WAVE);
      if (lane < j) a0 += e0 * bj;
      if (lane + WAVE < j) a1 += e1 * bj;
      const T sj = wave_sum(e0 * b0[c] + e1 * b1[c]);
      if (lane == j) a0 += sj;
      if (lane + WAVE == j) a1 += sj;
    }
    y0[c] = a0;
    y1[c] = a1;
    ao += (int64_t)n * (n + 1) / 2;
  }
  // seeds: t_s = b_p[s] + Uhat[:, s]^T b_u, y_p = S^-1 t
  const T* U = A + ao;
  const T* Si = U + (int64_t)nv * ns;
  T t[MAX_NS], yp[MAX_NS];
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    t[s] = 0;
    if (s >= ns) continue;
    T part = 0;
    int cs = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (lane < nc[c]) part += ldv<NT>(&U[(int64_t)s * nv + cs + lane]) * b0[c];
      if (lane + WAVE < nc[c]) part += ldv<NT>(&U[(int64_t)s * nv + cs + lane + WAVE]) * b1[c];
      cs += nc[c];
    }
    t[s] = wave_sum(part) + __shfl(bseed, s);
  }
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    T acc = 0;
    if (s < ns)
      for (int q = 0; q < ns; ++q) acc += Si[packed_index(s, q)] * t[q];
    yp[s] = acc;
  }
  // x_u = y_u + Uhat y_p, written to the patch's output slots
  T* Yp = Y + o - yshift;
  int cs = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (lane < nc[c]) {
      T acc = y0[c];
      for (int s = 0; s < ns; ++s) acc += ldv<NT>(&U[(int64_t)s * nv + cs + lane]) * yp[s];
      Yp[cs + lane] = acc;
    }
    if (lane + WAVE < nc[c]) {
      T acc = y1[c];
      for (int s = 0; s < ns; ++s) acc += ldv<NT>(&U[(int64_t)s * nv + cs + lane + WAVE]) * yp[s];
      Yp[cs + lane + WAVE] = acc;
    }
    cs += nc[c];
  }
  if (lane < ns) {
    T v = 0;
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s == lane) v = yp[s];
    Yp[nv + lane] = v;
  }
}

// Orders a wavefront's LDS writes before its later LDS reads (the waves of a
// workgroup then work independently, with no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Eight sums over the 64 lanes at once: v[0..7] per lane; a butterfly whose
// first three steps halve the values each lane carries (4 + 2 + 1 exchanges)
// and whose last three add within groups of 8 lanes (3 exchanges), instead of
// 8 x 6 exchanges for eight separate reductions.  On return every lane l holds
// the sum over all lanes of v[l >> 3].
template <typename T>
__device__ __forceinline__ T transpose_sum8(const T (&v)[8], int lane) {
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  T a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // a[k]: entry 4 h5 + k, summed over lanes l, l ^ 32
    const T send = h5 ? v[k] : v[k + 4];
    a[k] = (h5 ? v[k + 4] : v[k]) + __shfl_xor(send, 32);
  }
  T b[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {  // b[k]: entry 4 h5 + 2 h4 + k, over four lanes
    const T send = h4 ? a[k] : a[k + 2];
    b[k] = (h4 ? a[k + 2] : a[k]) + __shfl_xor(send, 16);
  }
  const T send = h3 ? b[0] : b[1];
  T c = (h3 ? b[1] : b[0]) + __shfl_xor(send, 8);  // entry 4 h5 + 2 h4 + h3, over eight lanes
  c += __shfl_xor(c, 4);
  c += __shfl_xor(c, 2);
  c += __shfl_xor(c, 1);
  return c;
}

// additive Vanka, one wavefront per patch, for records with one packed A^-1
// block serving every velocity component (LAYOUT_SHARED; NCO components) of
// at most 64 TT rows.
// No workgroup barrier and no record staging: lane l owns rows l, l + 64, ...
// of the block and streams each packed column j (entries i <= j, contiguous)
// straight from memory; it adds a_ij b_c[j] to its own rows (every component
// c) and a_ij b_c[i], i < j, to a partial sum of column j, whose lane sums
// (the transposed half of the symmetric block) are formed eight columns at a
// time by transpose_sum8.  Then t = Uhat^T b_u + b_p, y_p = S^-1 t and
// x_u = y_u + Uhat y_p.  WPB patches per workgroup, each wavefront with its
// own LDS (b and y of its patch, 2 max_m values).
template <typename T, int TT, int NCO, bool NT, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_vanka_wave(int64_t np, const int64_t* __restrict__ off,
                                                       const int4* __restrict__ dims,
                                                       const int64_t* __restrict__ foff,
                                                       const int* __restrict__ dofs, const T* __restrict__ fac,
                                                       const T* __restrict__ r, T* __restrict__ Y, int max_m,
                                                       int64_t yshift) {
  extern __shared__ unsigned char smem_raw[];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  const int64_t p = (int64_t)blockIdx.x * WPB + w;
  if (p >= np) return;  // whole wavefronts leave together
  T* sb = reinterpret_cast<T*>(smem_raw) + (int64_t)w * 2 * max_m;  // b of the patch
  T* sy = sb + max_m;                                                 // column sums, then y_u
  const int4 d = dims[p];
  const int n = d.x, nv = d.x + d.y + d.z, ns = d.w, m = nv + ns;  // nv = NCO n
  const int64_t o = off[p];
  const T* A = fac + foff[p];
  const T* U = A + (int64_t)n * (n + 1) / 2;
  const T* Si = U + (int64_t)nv * ns;
  // gather b: the index loads first, then the value loads
  for (int k0 = 0; k0 < m; k0 += 4 * WAVE) {
    int idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * WAVE + lane;
      idx[u] = k < m ? dofs[o + k] : 0;
    }
    T g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = k0 + u * WAVE + lane < m ? r[idx[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u * WAVE + lane < m) sb[k0 + u * WAVE + lane] = g[u];
  }
  wave_sync();
  T acc[TT][NCO], bi[TT][NCO];
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int c = 0; c < NCO; ++c) {
      const int i = WAVE * t + lane;
      acc[t][c] = 0;
      bi[t][c] = i < n ? sb[c * n + i] : (T)0;
    }
  for (int j0 = 0; j0 < n; j0 += 8) {
    T q[NCO][8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = j0 + jj;
      const bool live = j < n;
      const int64_t cb = (int64_t)j * (j + 1) / 2;
      T e[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const int i = WAVE * t + lane;
        e[t] = (live && i <= j) ? ldv<NT>(&A[cb + i]) : (T)0;
      }
#pragma unroll
      for (int c = 0; c < NCO; ++c) {
        const T bj = live ? sb[c * n + j] : (T)0;
        T qs = 0;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          acc[t][c] += e[t] * bj;
          if (WAVE * t + lane < j) qs += e[t] * bi[t][c];
        }
        q[c][jj] = qs;
      }
    }
#pragma unroll
    for (int c = 0; c < NCO; ++c) {
      const T sum = transpose_sum8(q[c], lane);
      const int j = j0 + (lane >> 3);
      if ((lane & 7) == 0 && j < n) sy[c * n + j] = sum;
    }
  }
  wave_sync();
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int c = 0; c < NCO; ++c) {
      const int i = WAVE * t + lane;
      if (i < n) sy[c * n + i] += acc[t][c];
    }
  wave_sync();
  // seeds: t = Uhat^T b_u + b_p, y_p = S^-1 t
  T ts[MAX_NS], yp[MAX_NS];
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) ts[s] = 0;
  for (int k = lane; k < nv; k += WAVE) {
    const T bk = sb[k];
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s < ns) ts[s] += U[(int64_t)s * nv + k] * bk;
  }
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s)
    if (s < ns) ts[s] = wave_sum(ts[s]) + sb[nv + s];
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    T a = 0;
#pragma unroll
    for (int q = 0; q < MAX_NS; ++q)
      if (s < ns && q < ns) a += Si[packed_index(s, q)] * ts[q];
    yp[s] = a;
  }
  T* Yp = Y + o - yshift;
  for (int k = lane; k < nv; k += WAVE) {
    T a = sy[k];
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s < ns) a += U[(int64_t)s * nv + k] * yp[s];
    Yp[k] = a;
  }
  if (lane < ns) {
    T v = 0;
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s)
      if (s == lane) v = yp[s];
    Yp[nv + lane] = v;
  }
}

// additive Vanka for a bucket of P patches of one fixed shape: one thread per
// patch, DoF lists, factor records and outputs interleaved across the whole
// bucket (element q of patch p at q * Ppad + p).  Every load of a wavefront is
// one contiguous 64-element segment, and since the wavefronts advance through q
// at similar rates, the accesses in flight at any time cover a few contiguous
// regions (a per-wavefront blocked layout measured 3x slower).  Uhat and S^-1 are applied first, then the packed A^-1
// blocks are streamed: x_u = Uhat y_p + A^-1 b_u.
// SH: LAYOUT_SHARED records (one packed block for every component, each of
// whose N0 rows it serves; N1 and N2 are 0 or N0).
template <typename T, int N0, int N1, int N2, int NS, bool NT = false, bool SH = false>
__global__ void __launch_bounds__(256) k_vanka_tpp(int64_t P, int64_t Ppad, const int* __restrict__ dofs,
                                                  const T* __restrict__ fac, const T* __restrict__ r,
                                                  T* __restrict__ Y) {
  constexpr int NV = N0 + N1 + N2, M = NV + NS;
  static_assert(!SH || ((N1 == 0 || N1 == N0) && (N2 == 0 || N2 == N0)), "shared blocks need equal components");
  constexpr int FA = SH ? N0 * (N0 + 1) / 2 : N0 * (N0 + 1) / 2 + N1 * (N1 + 1) / 2 + N2 * (N2 + 1) / 2;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T* f = fac + p;
  T b[M];
#pragma unroll
  for (int k = 0; k < M; ++k) b[k] = r[dofs[(int64_t)k * Ppad + p]];
  T u[NV * NS], t[NS], yp[NS], y[NV];
#pragma unroll
  for (int s = 0; s < NS; ++s) t[s] = b[NV + s];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      u[s * NV + k] = ldv<NT>(&f[(int64_t)(FA + s * NV + k) * Ppad]);
      t[s] += u[s * NV + k] * b[k];
    }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = s < q ? s : q, c = s < q ? q : s;
      acc += ldv<NT>(&f[(int64_t)(FA + NV * NS + c * (c + 1) / 2 + a) * Ppad]) * t[q];
    }
    yp[s] = acc;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T acc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) acc += u[s * NV + k] * yp[s];
    y[k] = acc;
  }
  int q = 0;
#define MAS_BLOCK(CS, N)                                   \
  _Pragma("unroll") for (int j = 0; j < (N); ++j)          \
    _Pragma("unroll") for (int i = 0; i <= j; ++i) {       \
      const T a = ldv<NT>(&f[(int64_t)(q++) * Ppad]);                \
      y[(CS) + i] += a * b[(CS) + j];                      \
      if (i != j) y[(CS) + j] += a * b[(CS) + i];          \
    }
  if constexpr (SH) {
    constexpr int NCO = NV / N0;
#pragma unroll
    for (int j = 0; j < N0; ++j)
#pragma unroll
      for (int i = 0; i <= j; ++i) {
        const T a = ldv<NT>(&f[(int64_t)(q++) * Ppad]);
#pragma unroll
        for (int c = 0; c < NCO; ++c) {
          y[c * N0 + i] += a * b[c * N0 + j];
          if (i != j) y[c * N0 + j] += a * b[c * N0 + i];
        }
      }
  } else {
    MAS_BLOCK(0, N0)
    MAS_BLOCK(N0, N1)
    MAS_BLOCK(N0 + N1, N2)
  }
#undef MAS_BLOCK
#pragma unroll
  for (int k = 0; k < NV; ++k) Y[(int64_t)k * Ppad + p] = y[k];
#pragma unroll
  for (int s = 0; s < NS; ++s) Y[(int64_t)(NV + s) * Ppad + p] = yp[s];
}

// additive Vanka for a bucket of patches of one fixed shape with nr
// right-hand sides: one wavefront per patch and one lane per right-hand side
// (grid.y chunks of 64).  The record (interleaved across the bucket, element q
// of patch p at q Ppad + p) is read with wave-uniform loads, b and y stay in
// registers, and every gather and output row is one contiguous run of the
// right-hand sides of a DoF.  The operations and their order are those of
// k_vanka_tpp for each right-hand side.  Y: slot s of patch p at
// (off[p] + s) nr + k.
template <typename T, int N0, int N1, int N2, int NS, bool SH, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_vanka_rhs(int64_t P, int64_t Ppad, int nr, const int* __restrict__ dofs,
                                                      const T* __restrict__ fac, const int64_t* __restrict__ off,
                                                      const T* __restrict__ r, T* __restrict__ Y) {
  constexpr int NV = N0 + N1 + N2, M = NV + NS;
  static_assert(!SH || ((N1 == 0 || N1 == N0) && (N2 == 0 || N2 == N0)), "shared blocks need equal components");
  constexpr int FA = SH ? N0 * (N0 + 1) / 2 : N0 * (N0 + 1) / 2 + N1 * (N1 + 1) / 2 + N2 * (N2 + 1) / 2;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t p = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WPB + threadIdx.x / WAVE));
  if (p >= P) return;  // whole wavefronts
  const int k = blockIdx.y * WAVE + lane;
  const int kc = k < nr ? k : nr - 1;  // lanes past nr compute a copy and store nothing
  const T* f = fac + p;
  T b[M];
#pragma unroll
  for (int q = 0; q < M; ++q) b[q] = r[(int64_t)dofs[(int64_t)q * Ppad + p] * nr + kc];
  T t[NS], yp[NS], y[NV];
#pragma unroll
  for (int s = 0; s < NS; ++s) t[s] = b[NV + s];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int q = 0; q < NV; ++q) t[s] += f[(int64_t)(FA + s * NV + q) * Ppad] * b[q];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = s < q ? s : q, c = s < q ? q : s;
      acc += f[(int64_t)(FA + NV * NS + c * (c + 1) / 2 + a) * Ppad] * t[q];
    }
    yp[s] = acc;
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    T acc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) acc += f[(int64_t)(FA + s * NV + q) * Ppad] * yp[s];
    y[q] = acc;
  }
  int e = 0;
  if constexpr (SH) {
    constexpr int NCO = NV / N0;
#pragma unroll
    for (int j = 0; j < N0; ++j)
#pragma unroll
      for (int i = 0; i <= j; ++i) {
        const T a = f[(int64_t)(e++) * Ppad];
#pragma unroll
        for (int c = 0; c < NCO; ++c) {
          y[c * N0 + i] += a * b[c * N0 + j];
          if (i != j) y[c * N0 + j] += a * b[c * N0 + i];
        }
      }
  } else {
#define MAS_BLOCK_R(CS, N)                                 \
  _Pragma("unroll") for (int j = 0; j < (N); ++j)          \
    _Pragma("unroll") for (int i = 0; i <= j; ++i) {       \
      const T a = f[(int64_t)(e++) * Ppad];                \
      y[(CS) + i] += a * b[(CS) + j];                      \
      if (i != j) y[(CS) + j] += a * b[(CS) + i];          \
    }
    MAS_BLOCK_R(0, N0)
    MAS_BLOCK_R(N0, N1)
    MAS_BLOCK_R(N0 + N1, N2)
#undef MAS_BLOCK_R
  }
  if (k < nr) {
    T* yo = Y + off[p] * nr + k;
#pragma unroll
    for (int q = 0; q < NV; ++q) yo[(int64_t)q * nr] = y[q];
#pragma unroll
    for (int s = 0; s < NS; ++s) yo[(int64_t)(NV + s) * nr] = yp[s];
  }
}

// x[j] (+)= omega W_j sum of the patch values held for DoF j (deterministic
// pull over the patch list in increasing patch order).
template <typename T>
__global__ void k_vanka_pull(int n, const int* __restrict__ inv_ptr, const int* __restrict__ inv_pos,
                             const T* __restrict__ Y, const T* __restrict__ w, T omega, T* __restrict__ x,
                             int accumulate) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  T acc = 0;
  for (int k = inv_ptr[j]; k < inv_ptr[j + 1]; ++k) acc += Y[inv_pos[k]];
  T v = omega * w[j] * acc;
  x[j] = accumulate ? x[j] + v : v;
}

// Same as k_vanka_pull with the DoF -> patch-value map stored slot-major
// (pos[s * n + j], -1 = empty slot): index loads are coalesced and the gathers
// of one DoF are independent.  W_j = 1 / (number of patches holding j).
template <typename T>
__global__ void k_vanka_pull_ell(int n, int width, const int* __restrict__ pos, const T* __restrict__ Y, T omega,
                                 T* __restrict__ x, int accumulate) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  T acc = 0;
  int cnt = 0;
#pragma unroll 4
  for (int s = 0; s < width; ++s) {
    const int q = pos[(int64_t)s * n + j];
    if (q >= 0) {
      acc += Y[q];
      ++cnt;
    }
  }
  if (cnt == 0) {
    if (!accumulate) x[j] = 0;
    return;
  }
  const T v = omega * acc / (T)cnt;
  x[j] = accumulate ? x[j] + v : v;
}

// ---------------------------------------------------------------------------
// FP64 block factorisation of every patch (setup).  One workgroup per patch.
// W: work area of max_nc^2 + 2 * max_nv * MAX_NS doubles (LDS or global).
// use_lds: 1 = W in LDS; 0 = W in global memory; 2 = W in global memory and
// the Gauss-Jordan inversion blocked by kGjBlock pivots, whose pivot-block
// inverse, pivot rows and pivot columns are staged in LDS (dynamic LDS of
// (kGjBlock^2 + 2 kGjBlock max_nc) doubles): the block is read and written
// once per kGjBlock pivots instead of once per pivot.
constexpr int kGjBlock = 16;
__device__ __forceinline__ int find_sorted(const int* a, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int v = a[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

template <typename TO, int TPB>
__global__ void __launch_bounds__(TPB) k_vanka_factor(int64_t np, const int64_t* __restrict__ off,
                                                      const int4* __restrict__ dims,
                                                      const int64_t* __restrict__ foff,
                                                      const int64_t* __restrict__ fstride, const int* __restrict__ dofs,
                                                      const int* __restrict__ kptr, const int* __restrict__ kind,
                                                      const double* __restrict__ kval, TO* __restrict__ fac,
                                                      double* __restrict__ gwork, int64_t work_stride,
                                                      int use_lds, int max_nv, double piv_tol,
                                                      int64_t* __restrict__ bad, int layout) {
  extern __shared__ double smem_d[];
  const int full = layout & LAYOUT_FULL;
  const bool shared = (layout & LAYOUT_SHARED) != 0;
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    double* W = use_lds == 1 ? smem_d : gwork + (int64_t)blockIdx.x * work_stride;
    double* Bm = W + (work_stride - 2 * (int64_t)max_nv * MAX_NS);  // ns x nv
    double* U = Bm + (int64_t)max_nv * MAX_NS;                      // nv x ns (row k: U[k*ns+s])
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    constexpr int NW = TPB / WAVE;
    const int4 d = dims[p];
    const int nc[3] = {d.x, d.y, d.z};
    const int nv = d.x + d.y + d.z, ns = d.w;
    const int* P = dofs + off[p];
    TO* out = fac + foff[p];
    const int64_t fs = fstride[p];  // 1: contiguous record; P: interleaved across a bucket of P patches
    // B rows of the seeds restricted to the patch velocities
    for (int k = tid; k < ns * nv; k += TPB) Bm[k] = 0.0;
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
      const int row = P[nv + s];
      for (int e = kptr[row] + tid; e < kptr[row + 1]; e += TPB) {
        int k = find_sorted(P, nv, kind[e]);
        if (k >= 0) Bm[s * nv + k] = kval[e];
      }
    }
    __syncthreads();
    int cs = 0;
    int64_t ao = 0;
    for (int c = 0; c < 3; ++c) {
      const int n = nc[c];
      if (n == 0) continue;
      // shared blocks: the components after the first reuse the inverse in W
      // (their blocks equal the first one), only U_c is theirs
      const bool invert = !shared || c == 0;
      for (int64_t k = tid; k < (invert ? (int64_t)n * n : 0); k += TPB) W[k] = 0.0;
      __syncthreads();
      for (int i = tid; i < (invert ? n : 0); i += TPB) {
        const int row = P[cs + i];
        for (int e = kptr[row]; e < kptr[row + 1]; ++e) {
          int j = find_sorted(P + cs, n, kind[e]);
          if (j >= 0) W[(int64_t)i * n + j] = kval[e];
        }
      }
      __syncthreads();
      // in-place Gauss-Jordan inversion (the block is symmetric positive
      // definite).  The lanes share each row (lane j owns columns j, j + 64, ...),
      // so every row update is a contiguous access; the lane owning column k
      // writes the pivot column.
      double scale = 0.0;
      for (int i = 0; i < n; ++i) scale = fmax(scale, fabs(W[(int64_t)i * n + i]));
      if (use_lds == 2 && invert) {
        // Blocked Gauss-Jordan: with K the next b pivots, W = [A11 A12; A21 A22]
        // becomes [A11^-1, A11^-1 A12; -A21 A11^-1, A22 - A21 A11^-1 A12],
        // the same as b single-pivot steps.
        constexpr int BS = kGjBlock;
        double* Pk = smem_d;         // b x b pivot block, then its inverse
        double* RB = Pk + BS * BS;   // b x n: A11^-1 [A11 A12] rows (A11^-1 inside K)
        double* CB = RB + BS * n;    // n x b: the old pivot columns
        for (int kb = 0; kb < n; kb += BS) {
          const int b = min(BS, n - kb);
          if (tid < b * b) Pk[tid] = W[(int64_t)(kb + tid / b) * n + kb + tid % b];
          __syncthreads();
          for (int k = 0; k < b; ++k) {  // single-pivot steps on the b x b block: read, then write
            const double akk = Pk[k * b + k];
            const double dk = 1.0 / akk;
            double v = 0.0;
            if (tid < b * b) {
              const int i = tid / b, j = tid % b;
              const double pik = Pk[i * b + k], pkj = Pk[k * b + j];
              if (i == k) v = (j == k) ? dk : pkj * dk;
              else v = (j == k) ? -pik * dk : Pk[tid] - pik * (pkj * dk);
            }
            if (tid == 0 && !(akk > piv_tol * scale)) atomicMin((unsigned long long*)bad, (unsigned long long)p);
            __syncthreads();
            if (tid < b * b) Pk[tid] = v;
            __syncthreads();
          }
          for (int64_t q = tid; q < (int64_t)b * n; q += TPB) {
            const int t = (int)(q / n), j = (int)(q % n);
            double v = 0.0;
            if (j >= kb && j < kb + b) {
              v = Pk[t * b + (j - kb)];
            } else {
              for (int u = 0; u < b; ++u) v += Pk[t * b + u] * W[(int64_t)(kb + u) * n + j];
            }
            RB[q] = v;
          }
          for (int64_t q = tid; q < (int64_t)n * b; q += TPB) CB[q] = W[(q / b) * n + kb + q % b];
          __syncthreads();
          for (int i = wv; i < n; i += NW) {
            double ci[BS];
#pragma unroll
            for (int u = 0; u < BS; ++u) ci[u] = u < b ? CB[(int64_t)i * b + u] : 0.0;
            const bool in_k = i >= kb && i < kb + b;
            double* wi = W + (int64_t)i * n;
            for (int j = lane; j < n; j += WAVE) {
              double v;
              if (in_k) {
                v = RB[(int64_t)(i - kb) * n + j];
              } else if (j >= kb && j < kb + b) {
                v = 0.0;
#pragma unroll
                for (int u = 0; u < BS; ++u)
                  if (u < b) v -= ci[u] * Pk[u * b + (j - kb)];
              } else {
                v = wi[j];
#pragma unroll
                for (int u = 0; u < BS; ++u)
                  if (u < b) v -= ci[u] * RB[(int64_t)u * n + j];
              }
              wi[j] = v;
            }
          }
          __syncthreads();
        }
      }
      for (int k = 0; k < (use_lds == 2 || !invert ? 0 : n); ++k) {
        const double akk = W[(int64_t)k * n + k];
        if (!(akk > piv_tol * scale)) {
          if (tid == 0) atomicMin((unsigned long long*)bad, (unsigned long long)p);
        }
        const double dk = 1.0 / akk;
        __syncthreads();
        for (int j = tid; j < n; j += TPB)
          if (j != k) W[(int64_t)k * n + j] *= dk;
        __syncthreads();
        const double* wk = W + (int64_t)k * n;
        for (int i = wv; i < n; i += NW) {  // wavefront wv updates rows wv, wv + NW, ...
          if (i == k) continue;
          double* wi = W + (int64_t)i * n;
          const double f = wi[k];
          for (int j = lane; j < n; j += WAVE)
            if (j != k) wi[j] -= f * wk[j];
          if (lane == k % WAVE) wi[k] = -f * dk;
        }
        __syncthreads();
        if (tid == 0) W[(int64_t)k * n + k] = dk;
        __syncthreads();
      }
      // symmetrise the inverse: both halves take the mean of the pair
      for (int64_t q = tid; q < (invert ? (int64_t)n * (n + 1) / 2 : 0); q += TPB) {
        int j = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
        while ((int64_t)j * (j + 1) / 2 > q) --j;
        while ((int64_t)(j + 1) * (j + 2) / 2 <= q) ++j;
        const int i = (int)(q - (int64_t)j * (j + 1) / 2);
        const double v = 0.5 * (W[(int64_t)i * n + j] + W[(int64_t)j * n + i]);
        W[(int64_t)i * n + j] = v;
        W[(int64_t)j * n + i] = v;
        if (!full) out[(ao + q) * fs] = (TO)v;  // packed upper
      }
      __syncthreads();
      if (full && invert)
        for (int64_t q = tid; q < (int64_t)n * n; q += TPB) out[(ao + q) * fs] = (TO)W[q];
      // U_c = A_c^-1 B_c^T (column i of the symmetric inverse, read along rows j)
      for (int i = tid; i < n; i += TPB)
        for (int s = 0; s < ns; ++s) {
          double acc = 0.0;
          for (int j = 0; j < n; ++j) acc += W[(int64_t)j * n + i] * Bm[s * nv + cs + j];
          U[(int64_t)(cs + i) * ns + s] = acc;
        }
      __syncthreads();
      if (invert) ao += blk_size(n, full);
      cs += n;
    }
    // S = -B U (ns x ns), inverted by one lane with partial pivoting
    if (tid == 0) {
      double S[MAX_NS * MAX_NS], I[MAX_NS * MAX_NS];
      double smax = 0.0;
      for (int s = 0; s < ns; ++s)
        for (int t = 0; t < ns; ++t) {
          double acc = 0.0;
          for (int k = 0; k < nv; ++k) acc += Bm[s * nv + k] * U[(int64_t)k * ns + t];
          S[s * ns + t] = -acc;
          I[s * ns + t] = (s == t) ? 1.0 : 0.0;
          smax = fmax(smax, fabs(acc));
        }
      bool ok = smax > 0.0;
      for (int k = 0; k < ns && ok; ++k) {
        int pr = k;
        for (int i = k + 1; i < ns; ++i)
          if (fabs(S[i * ns + k]) > fabs(S[pr * ns + k])) pr = i;
        if (!(fabs(S[pr * ns + k]) > piv_tol * smax)) { ok = false; break; }
        if (pr != k)
          for (int j = 0; j < ns; ++j) {
            double t1 = S[k * ns + j]; S[k * ns + j] = S[pr * ns + j]; S[pr * ns + j] = t1;
            double t2 = I[k * ns + j]; I[k * ns + j] = I[pr * ns + j]; I[pr * ns + j] = t2;
          }
        const double dk = 1.0 / S[k * ns + k];
        for (int j = 0; j < ns; ++j) { S[k * ns + j] *= dk; I[k * ns + j] *= dk; }
        for (int i = 0; i < ns; ++i) {
          if (i == k) continue;
          const double f = S[i * ns + k];
          for (int j = 0; j < ns; ++j) { S[i * ns + j] -= f * S[k * ns + j]; I[i * ns + j] -= f * I[k * ns + j]; }
        }
      }
      if (!ok) atomicMin((unsigned long long*)bad, (unsigned long long)p);
      const int64_t so = ao + (int64_t)nv * ns;
      for (int t = 0; t < ns; ++t)
        for (int s = 0; s <= t; ++s)
          out[(so + (int64_t)t * (t + 1) / 2 + s) * fs] = (TO)(0.5 * (I[s * ns + t] + I[t * ns + s]));
    }
    for (int64_t q = tid; q < (int64_t)nv * ns; q += TPB) {
      int s = (int)(q / nv), k = (int)(q % nv);
      out[(ao + q) * fs] = (TO)(-U[(int64_t)k * ns + s]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// dense coarse solve: y = C b (C row-major, ld columns), one wavefront per row,
// accumulated in FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_gemv(int n, int ld, const double* __restrict__ C,
                                                   const T* __restrict__ b, T* __restrict__ y) {
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int lane = threadIdx.x & (WAVE - 1);
  double s = 0.0;
  if (row < n)
    for (int j = lane; j < n; j += WAVE) s += C[(int64_t)row * ld + j] * (double)b[j];
  s = wave_sum(s);
  if (row < n && lane == 0) y[row] = (T)s;
}

// Gauss-Jordan inversion with partial pivoting of a dense n x n FP64 matrix
// (row-major), one pivot step per launch pair (setup only).
__global__ void k_gj_pivot(int n, int k, double* __restrict__ A, int* __restrict__ perm, int* __restrict__ flag) {
  // one block of 256 threads: find the pivot row and swap it into row k
  __shared__ double best[256];
  __shared__ int bi[256];
  double v = -1.0;
  int idx = k;
  for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
    double a = fabs(A[(int64_t)i * n + k]);
    if (a > v) { v = a; idx = i; }
  }
  best[threadIdx.x] = v;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      if (best[threadIdx.x + s] > best[threadIdx.x] ||
          (best[threadIdx.x + s] == best[threadIdx.x] && bi[threadIdx.x + s] < bi[threadIdx.x])) {
        best[threadIdx.x] = best[threadIdx.x + s];
        bi[threadIdx.x] = bi[threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  const int pr = bi[0];
  if (threadIdx.x == 0) {
    perm[k] = pr;
    if (!(best[0] > 0.0)) *flag = 1;
  }
  if (pr != k)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double t = A[(int64_t)k * n + j];
      A[(int64_t)k * n + j] = A[(int64_t)pr * n + j];
      A[(int64_t)pr * n + j] = t;
    }
}

// in-place elimination step k reads row k and column k from saved copies
__global__ void k_gj_save(int n, int k, const double* __restrict__ A, double* __restrict__ rowk,
                          double* __restrict__ colk) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    rowk[j] = A[(int64_t)k * n + j];
    colk[j] = A[(int64_t)j * n + k];
  }
}

__global__ void k_gj_step(int n, int k, double* __restrict__ A, const double* __restrict__ rowk,
                          const double* __restrict__ colk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  const double dk = 1.0 / rowk[k];
  if (i == k) {
    A[t] = (j == k) ? dk : rowk[j] * dk;
  } else {
    const double f = colk[i];
    if (j == k) A[t] = -f * dk;
    else A[t] -= f * rowk[j] * dk;
  }
}

// undo the row interchanges: swap columns k and perm[k], k = n-1 .. 0
__global__ void k_gj_colswap(int n, int k, const int* __restrict__ perm, double* __restrict__ A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int pr = perm[k];
  if (i < n && pr != k) {
    double t = A[(int64_t)i * n + k];
    A[(int64_t)i * n + k] = A[(int64_t)i * n + pr];
    A[(int64_t)i * n + pr] = t;
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions and small FGMRES kernels

// partial[b] = sum over block b of x . y
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ y, double* __restrict__ partial) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = wave_sum(s);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// out[0] = sum of partial (sqrt if take_sqrt)
__global__ void __launch_bounds__(256) k_reduce_final(int nb, const double* __restrict__ partial,
                                                     double* __restrict__ out, int take_sqrt) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = wave_sum(s);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0] + sh[1] + sh[2] + sh[3];
    out[0] = take_sqrt ? sqrt(t) : t;
  }
}

// Sum of the nb partials of the previous reduction, in block order, computed by
// every calling block (identical result everywhere).  (A last-block reduction
// would need a device-scope fence per block, which writes back the
// non-coherent per-XCD L2 caches and costs far more.)
__device__ __forceinline__ double sum_partials(int nb, const double* __restrict__ partial) {
  __shared__ double red[4];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) v += partial[b];
  v = wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  const double t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

// One modified Gram-Schmidt step: when prev_partial is given, a = sum of the
// previous step's partials (= h of that step, stored by block 0 into *hprev) and
// w -= a vprev; then partial_out[b] = block b's share of w . vnext (mode 0) or
// w . w (mode 1).  Two partial buffers alternate between consecutive steps.
// Vectors of type T, sums and coefficients in FP64 (T = double for FGMRES, the
// cycle's type for the relaxation wrapper).
template <typename T>
__global__ void __launch_bounds__(256) k_mgs_step(int64_t n, T* __restrict__ w, const T* __restrict__ vprev,
                                                 double* __restrict__ hprev, const double* __restrict__ prev_partial,
                                                 const T* __restrict__ vnext, double* __restrict__ partial_out,
                                                 int mode) {
  __shared__ double sh[4];
  // the first four elements of this thread are loaded before the reduction of
  // the previous partials, so their latency overlaps it
  constexpr int K = 4;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (int64_t)gridDim.x * blockDim.x;
  double wk[K], pk[K], nk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + k * st;
    const bool ok = i < n;
    wk[k] = ok ? (double)w[i] : 0.0;
    pk[k] = (ok && vprev) ? (double)vprev[i] : 0.0;
    nk[k] = (ok && mode == 0) ? (double)vnext[i] : 0.0;
  }
  double a = 0.0;
  if (prev_partial) {
    a = sum_partials(gridDim.x, prev_partial);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hprev = a;
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + k * st;
    if (i < n) {
      double wi = wk[k];
      if (vprev) {
        wi -= a * pk[k];
        w[i] = (T)wi;
      }
      s += wi * (mode == 0 ? nk[k] : wi);
    }
  }
  for (int64_t i = i0 + K * st; i < n; i += st) {
    double wi = w[i];
    if (vprev) {
      wi -= a * (double)vprev[i];
      w[i] = (T)wi;
    }
    s += wi * (mode == 0 ? (double)vnext[i] : wi);
  }
  s = wave_sum(s);
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial_out[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// v = w / sqrt(sum of partials); block 0 stores the norm into *hout
template <typename T>
__global__ void __launch_bounds__(256) k_normalize(int64_t n, const double* __restrict__ partial, int nb,
                                                  double* __restrict__ hout, const T* __restrict__ w,
                                                  T* __restrict__ v) {
  constexpr int K = 4;  // first elements loaded before the reduction (latency overlap)
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (int64_t)gridDim.x * blockDim.x;
  double wk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) wk[k] = i0 + k * st < n ? (double)w[i0 + k * st] : 0.0;
  const double nrm = sqrt(sum_partials(nb, partial));
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = nrm;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (i0 + k * st < n) v[i0 + k * st] = nrm != 0.0 ? (T)(wk[k] / nrm) : (T)0;
  for (int64_t i = i0 + K * st; i < n; i += st) v[i] = nrm != 0.0 ? (T)((double)w[i] / nrm) : (T)0;
}

// Least-squares step of the relaxation wrapper (one thread): Givens rotations
// reduce the (m+1) x m Hessenberg matrix H (row-major, h[i * m + j]) with
// right-hand side beta e_1; y (m values) solves the triangular system, a zero
// pivot (breakdown) leaving its coefficient at zero.
__global__ void k_krylov_ls(int m, const double* __restrict__ H, const double* __restrict__ beta,
                            double* __restrict__ y) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double R[9 * 8], g[9], c[8], sn[8];
  for (int i = 0; i < (m + 1) * m; ++i) R[i] = H[i];
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = *beta;
  int k = m;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < j; ++i) {
      const double t = c[i] * R[i * m + j] + sn[i] * R[(i + 1) * m + j];
      R[(i + 1) * m + j] = -sn[i] * R[i * m + j] + c[i] * R[(i + 1) * m + j];
      R[i * m + j] = t;
    }
    const double den = hypot(R[j * m + j], R[(j + 1) * m + j]);
    if (den == 0.0) {
      k = j;
      break;
    }
    c[j] = R[j * m + j] / den;
    sn[j] = R[(j + 1) * m + j] / den;
    R[j * m + j] = den;
    R[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = c[j] * g[j];
  }
  for (int i = m - 1; i >= 0; --i) {
    if (i >= k || R[i * m + i] == 0.0) {
      y[i] = 0.0;
      continue;
    }
    double t = g[i];
    for (int q = i + 1; q < k; ++q) t -= R[i * m + q] * y[q];
    y[i] = t / R[i * m + i];
  }
}

// y -= (*h) x
__global__ void k_axpy_neg_dev(int64_t n, const double* __restrict__ h, const double* __restrict__ x,
                               double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = *h;
  if (i < n) y[i] -= a * x[i];
}

// y = x / (*h)  (x may alias y)
__global__ void k_scale_inv_dev(int64_t n, const double* __restrict__ h, const double* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = *h;
  if (i < n) y[i] = (a != 0.0) ? x[i] / a : 0.0;
}

// y = x / h_host
__global__ void k_scale_inv(int64_t n, double a, const double* x, double* y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / a;
}

// x += sum_k y[k] Z[k]  (Z: k vectors of length n, stride n)
template <typename T>
__global__ void k_update_x(int64_t n, int k, const T* __restrict__ Z, const double* __restrict__ y,
                           T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = x[i];
  for (int q = 0; q < k; ++q) s += y[q] * (double)Z[(int64_t)q * n + i];
  x[i] = (T)s;
}

// ---------------------------------------------------------------------------
// Sparse product C = A B for the Galerkin operators of the setup (Algorithm 1),
// one row of C per 64-thread workgroup.  The entries of A's row are taken in
// order; for each, the lanes add a_ik b_kj into an LDS hash table keyed by j
// (the columns of one row of B are distinct, so no two lanes touch one entry in
// a step).  Every c_ij is therefore summed in the order of A's row, with the
// products and the sums rounded separately, as the host product does: the two
// give the same bits.  PASS 0 counts the distinct columns of each row into cnt;
// PASS 1 writes them, sorted, from Cp[i].  A row with more than `cap` distinct
// columns (cap <= kSpgSlots * 3 / 4) gets over[i] = 1 in PASS 0 and is left to
// the host product or to k_spgemm_dense.
constexpr int kSpgSlots = 2048;

template <int PASS>
__global__ void __launch_bounds__(64) k_spgemm_row(int64_t n, const int64_t* __restrict__ Ap,
                                                   const int* __restrict__ Ai, const double* __restrict__ Av,
                                                   const int64_t* __restrict__ Bp, const int* __restrict__ Bi,
                                                   const double* __restrict__ Bv, int cap, int64_t* __restrict__ cnt,
                                                   int* __restrict__ over, const int64_t* __restrict__ Cp,
                                                   int* __restrict__ Ci, double* __restrict__ Cv) {
#pragma clang fp contract(off)
  __shared__ int key[kSpgSlots];
  __shared__ double val[kSpgSlots];
  __shared__ int nkeys, full;
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n) return;  // uniform over the workgroup
  if (PASS == 1 && over[i]) return;
  // a table of at least twice the row's product count (the summed lengths of
  // the rows of B it meets), 64 to kSpgSlots slots
  int64_t bound = 0;
  for (int64_t a = Ap[i] + lane; a < Ap[i + 1]; a += 64) {
    const int k = Ai[a];
    bound += Bp[k + 1] - Bp[k];
  }
  for (int o = 32; o > 0; o >>= 1) bound += __shfl_xor(bound, o, 64);
  int tbits = 6;
  while (tbits < 11 && ((int64_t)1 << tbits) < 2 * bound) ++tbits;
  const int tsize = 1 << tbits;
  for (int t = lane; t < tsize; t += 64) key[t] = -1;
  if (lane == 0) {
    nkeys = 0;
    full = 0;
  }
  __syncthreads();
  for (int64_t a = Ap[i]; a < Ap[i + 1]; ++a) {
    const int k = Ai[a];
    const double av = Av[a];
    for (int64_t b = Bp[k] + lane; b < Bp[k + 1]; b += 64) {
      const int j = Bi[b];
      const double pr = av * Bv[b];
      unsigned h = ((unsigned)j * 2654435761u) >> (32 - tbits);  // top tbits bits: a slot in [0, tsize)
      for (int probe = 0; probe < tsize; ++probe, h = (h + 1) & (tsize - 1)) {
        const int old = atomicCAS(&key[h], -1, j);
        if (old == -1) {  // new column
          val[h] = pr;
          if (atomicAdd(&nkeys, 1) >= cap) full = 1;
          break;
        }
        if (old == j) {
          val[h] = val[h] + pr;
          break;
        }
      }
    }
    __syncthreads();
    if (full) break;  // uniform: read after the barrier
  }
  if (PASS == 0) {
    if (lane == 0) {
      cnt[i] = full ? 0 : nkeys;
      over[i] = full ? 1 : 0;
    }
    return;
  }
  // PASS 1: the occupied slots packed to the front of the table in slot order
  // (a slot moves only to a lower index, after every lane has read its own),
  // then each column's rank among the row's columns gives its position
  int nk = 0;
  for (int t0 = 0; t0 < tsize; t0 += 64) {
    const int t = t0 + lane;
    const int j = key[t];
    const double v = val[t];
    const unsigned long long bal = __ballot(j >= 0);
    const int pos = nk + __popcll(bal & ((1ull << lane) - 1ull));
    __syncthreads();
    if (j >= 0) {
      key[pos] = j;
      val[pos] = v;
    }
    nk += __popcll(bal);
    __syncthreads();
  }
  const int64_t base = Cp[i], m = Cp[i + 1] - Cp[i];
  for (int q = lane; q < nk; q += 64) {
    const int j = key[q];
    int r = 0;
    for (int u = 0; u < nk; ++u) r += key[u] < j ? 1 : 0;
    if (r < m) {
      Ci[base + r] = j;
      Cv[base + r] = val[q];
    }
  }
}


// ---------------------------------------------------------------------------
// Smoothed aggregation on the device (Algorithm 1, Section 3.2).  Each value
// below is formed with the operations, and in the order, of the host setup,
// with no contraction of products into fused multiply-adds, so the device
// hierarchy equals the host's bit for bit.

// d_i = a_ii and the Gershgorin ratio (sum_j |a_ij|, in row order) / a_ii of
// each row; a thread per row.
__global__ void k_sa_diag(int64_t n, const int64_t* __restrict__ Ap, const int* __restrict__ Ai,
                          const double* __restrict__ Av, double* __restrict__ d, double* __restrict__ ratio) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double di = 0.0, s = 0.0;
  for (int64_t e = Ap[i]; e < Ap[i + 1]; ++e) {
    const double v = Av[e];
    if (Ai[e] == i) di = v;
    s += fabs(v);
  }
  d[i] = di;
  ratio[i] = s / di;
}

// Per-workgroup maxima of x (starting from 0; a NaN is never taken), for the
// Gershgorin bound max_i ratio_i.  256 threads.
__global__ void __launch_bounds__(256) k_sa_max(int64_t n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[256];
  double r = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = x[i];
    r = (r < v) ? v : r;
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double v = red[threadIdx.x + w];
      red[threadIdx.x] = (red[threadIdx.x] < v) ? v : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Symmetric strength: keep[e] for j != i with a_ij^2 >= th2 (a_ii a_jj); a
// thread per row.
__global__ void k_sa_soc_sym(int64_t n, const int64_t* __restrict__ Ap, const int* __restrict__ Ai,
                             const double* __restrict__ Av, const double* __restrict__ d, double th2,
                             unsigned char* __restrict__ keep) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = d[i];
  for (int64_t e = Ap[i]; e < Ap[i + 1]; ++e) {
    const int j = Ai[e];
    const double v = Av[e];
    keep[e] = (j != i && v * v >= th2 * (di * d[j])) ? 1 : 0;
  }
}

// Evolution strength, two steps of J = I - dt D^-1 A (Section 3.2): a
// wavefront per row i.  For each stored (i, r), z_i[r] = sum_m J[r][m] J[m][i]
// over row r of A in ascending m, taking the m for which a_mi is stored (found
// by a binary search of column i in the sorted row m), which is the host's
// sum term for term.  Then, with zt = z_i[i] B_r / B_i,
//   s_ir = max(|zt - z_i[r]| / |z_i[r]|, 1e-4) where z_i[r] != 0 and
//   zt z_i[r] > 0, infinite otherwise,
// and row i keeps r != i with a finite s_ir <= eps min_m s_im.  z holds one
// value per stored entry of A (scratch, the lane of an entry reads only what
// it wrote).
__global__ void __launch_bounds__(64) k_sa_soc_evol(int64_t n, const int64_t* __restrict__ Ap,
                                                    const int* __restrict__ Ai, const double* __restrict__ Av,
                                                    const double* __restrict__ d, const double* __restrict__ B,
                                                    double dt, double eps, double* __restrict__ z,
                                                    unsigned char* __restrict__ keep) {
#pragma clang fp contract(off)
  __shared__ double zii_s;
  __shared__ int has_diag;
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n) return;  // uniform over the workgroup
  const int64_t e0 = Ap[i], e1 = Ap[i + 1];
  auto jv = [&](int64_t r, int64_t c, double a) { return (r == c ? 1.0 : 0.0) - dt * ((1.0 / d[r]) * a); };
  auto zcol = [&](int64_t r) {
    double acc = 0.0;
    for (int64_t f = Ap[r]; f < Ap[r + 1]; ++f) {
      const int m = Ai[f];
      int64_t lo = Ap[m], hi = Ap[m + 1];
      const int64_t end = hi;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (Ai[mid] < i) lo = mid + 1;
        else hi = mid;
      }
      if (lo < end && Ai[lo] == i) acc += jv(r, m, Av[f]) * jv(m, i, Av[lo]);
    }
    return acc;
  };
  if (lane == 0) has_diag = 0;
  __syncthreads();
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const int r = Ai[e];
    const double zr = zcol(r);
    z[e] = zr;
    if (r == i) {
      zii_s = zr;
      has_diag = 1;
    }
  }
  __syncthreads();
  if (!has_diag) {
    if (lane == 0) zii_s = zcol(i);
    __syncthreads();
  }
  const double zii = zii_s, bi = B[i];
  double smin = INFINITY;
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const int j = Ai[e];
    double s = INFINITY;
    if (j != i) {
      const double zij = z[e];
      const double zt = zii * B[j] / bi;
      if (zij != 0.0 && zt * zij > 0.0) {
        const double q = fabs(zt - zij) / fabs(zij);
        s = (q < 1e-4) ? 1e-4 : q;
      }
      smin = (s < smin) ? s : smin;
    }
    z[e] = s;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(smin, o, 64);
    smin = (v < smin) ? v : smin;
  }
  const double lim = eps * smin;
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const double s = z[e];
    keep[e] = (Ai[e] != i && isfinite(s) && s <= lim) ? 1 : 0;
  }
}

// Kept entries per row (PASS 0: counts into cnt) and their columns in row
// order (PASS 1: from Sp[i]); a thread per row.
template <int PASS>
__global__ void k_sa_select(int64_t n, const int64_t* __restrict__ Ap, const int* __restrict__ Ai,
                            const unsigned char* __restrict__ keep, int64_t* __restrict__ cnt,
                            const int64_t* __restrict__ Sp, int* __restrict__ Si) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t c = PASS == 1 ? Sp[i] : 0;
  for (int64_t e = Ap[i]; e < Ap[i + 1]; ++e)
    if (keep[e]) {
      if (PASS == 1) Si[c] = Ai[e];
      ++c;
    }
  if (PASS == 0) cnt[i] = c;
}

// Union of two sorted patterns row by row (S1 and its transpose): PASS 0
// counts, PASS 1 writes from Sp[i]; a thread per row.
template <int PASS>
__global__ void k_sa_union(int64_t n, const int64_t* __restrict__ Xp, const int* __restrict__ Xi,
                           const int64_t* __restrict__ Yp, const int* __restrict__ Yi, int64_t* __restrict__ cnt,
                           const int64_t* __restrict__ Sp, int* __restrict__ Si) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t a = Xp[i], b = Yp[i];
  const int64_t ae = Xp[i + 1], be = Yp[i + 1];
  int64_t o = PASS == 1 ? Sp[i] : 0;
  while (a < ae || b < be) {
    int v;
    if (b >= be || (a < ae && Xi[a] < Yi[b])) v = Xi[a++];
    else if (a >= ae || Yi[b] < Xi[a]) v = Yi[b++];
    else {
      v = Xi[a++];
      ++b;
    }
    if (PASS == 1) Si[o] = v;
    ++o;
  }
  if (PASS == 0) cnt[i] = o;
}

// D^-1 A: each a_ij / a_ii; a thread per row.
__global__ void k_sa_scale(int64_t n, const int64_t* __restrict__ Ap, const double* __restrict__ Av,
                           const double* __restrict__ d, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = d[i];
  for (int64_t e = Ap[i]; e < Ap[i + 1]; ++e) out[e] = Av[e] / di;
}

// The smoothed prolongator from (D^-1 A) T: p_iJ = -omega [(D^-1 A) T]_iJ,
// plus t_i where J is the aggregate of i; a thread per row.
__global__ void k_sa_smooth(int64_t n, const int64_t* __restrict__ Pp, const int* __restrict__ Pi,
                            double* __restrict__ Pv, const int* __restrict__ agg, const double* __restrict__ tv,
                            double omega) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ai = agg[i];
  for (int64_t e = Pp[i]; e < Pp[i + 1]; ++e) {
    double v = -omega * Pv[e];
    if (Pi[e] == ai) v += tv[i];
    Pv[e] = v;
  }
}

// Row index of every stored entry (for the transpose); a thread per row.
__global__ void k_sa_rows(int64_t n, const int64_t* __restrict__ Ap, int* __restrict__ row) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = Ap[i]; e < Ap[i + 1]; ++e) row[e] = (int)i;
}

// 0, 1, ..., n - 1.
__global__ void k_sa_iota(int64_t n, int* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int)i;
}
__global__ void k_sa_iota64(int64_t n, int64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}

// Entries per column (the transpose's row lengths); a thread per entry.
__global__ void k_sa_colcount(int64_t nnz, const int* __restrict__ Ai, unsigned long long* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[Ai[e]], 1ull);
}

// Transpose entries from the stable sort by column of the entry numbers:
// entry p of A^T is entry perm[p] of A (rows ascend within each column, as in
// the host's transpose).
__global__ void k_sa_gather(int64_t nnz, const int* __restrict__ perm, const int* __restrict__ row,
                            const double* __restrict__ Av, int* __restrict__ Ti, double* __restrict__ Tv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int e = perm[p];
  Ti[p] = row[e];
  if (Tv) Tv[p] = Av[e];
}

// C = A B for the rows k_spgemm_row leaves (over[i]: more distinct columns
// than its LDS table holds), a workgroup per such row, rows spread over the
// grid.  Each workgroup accumulates in its own dense slice (acc, mark) of B.nc
// entries in global memory; as in k_spgemm_row the entries of A's row are
// taken in order and the lanes add a_ik b_kj for distinct j of one row of B,
// so every c_ij is summed in the host's order.  mark holds 2 i + PASS for a
// column met in row i's pass.  PASS 0 writes the counts; PASS 1 the sorted
// columns and values from Cp[i] (a block scan of the marks).
template <int PASS>
__global__ void __launch_bounds__(256) k_spgemm_dense(int64_t n, const int64_t* __restrict__ Ap,
                                                      const int* __restrict__ Ai, const double* __restrict__ Av,
                                                      const int64_t* __restrict__ Bp, const int* __restrict__ Bi,
                                                      const double* __restrict__ Bv, int64_t nc,
                                                      const int* __restrict__ over, double* __restrict__ acc_all,
                                                      int64_t* __restrict__ mark_all, int64_t* __restrict__ cnt,
                                                      const int64_t* __restrict__ Cp, int* __restrict__ Ci,
                                                      double* __restrict__ Cv) {
#pragma clang fp contract(off)
  __shared__ unsigned long long count;
  __shared__ int wsum[4];
  double* acc = acc_all + (int64_t)blockIdx.x * nc;
  int64_t* mark = mark_all + (int64_t)blockIdx.x * nc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    if (!over[i]) continue;  // uniform over the workgroup
    const int64_t stamp = 2 * i + PASS;
    if (tid == 0) count = 0;
    __syncthreads();
    for (int64_t a = Ap[i]; a < Ap[i + 1]; ++a) {
      const int k = Ai[a];
      const double av = Av[a];
      for (int64_t b = Bp[k] + tid; b < Bp[k + 1]; b += 256) {
        const int j = Bi[b];
        const double pr = av * Bv[b];
        if (mark[j] != stamp) {
          mark[j] = stamp;
          acc[j] = pr;
          if (PASS == 0) atomicAdd(&count, 1ull);
        } else {
          acc[j] = acc[j] + pr;
        }
      }
      __syncthreads();
    }
    if (PASS == 0) {
      if (tid == 0) cnt[i] = (int64_t)count;
      __syncthreads();
      continue;
    }
    int64_t o = Cp[i];
    for (int64_t j0 = 0; j0 < nc; j0 += 256) {
      const int64_t j = j0 + tid;
      const bool f = j < nc && mark[j] == stamp;
      const unsigned long long bal = __ballot(f);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[wave] = __popcll(bal);
      __syncthreads();
      int off = 0, tot = 0;
      for (int w = 0; w < 4; ++w) {
        off += w < wave ? wsum[w] : 0;
        tot += wsum[w];
      }
      if (f) {
        Ci[o + off + before] = (int)j;
        Cv[o + off + before] = acc[j];
      }
      o += tot;
      __syncthreads();
    }
  }
}

}  // namespace mas
