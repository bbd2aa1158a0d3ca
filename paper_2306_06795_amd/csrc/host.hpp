// Host-side setup of libmas: sparse matrices, per-field smoothed aggregation
// (Algorithm 1), algebraic Vanka patches (Section 3.3.1), Lanczos estimates
// for the Chebyshev intervals (Table 2).  Plain C++17, no HIP.
#pragma once
#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

namespace mas {

// Allocator whose value-less construct leaves the element uninitialised: large
// products are sized first and filled by several threads, which then also do
// the first touch of their pages.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) {}
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    if constexpr (sizeof...(A) == 0)
      ::new ((void*)p) U;
    else
      ::new ((void*)p) U(std::forward<A>(a)...);
  }
};

struct Csr {
  int64_t nr = 0, nc = 0;
  std::vector<int64_t> ptr;  // nr + 1
  std::vector<int32_t, NoInit<int32_t>> ind;  // sorted within each row
  std::vector<double, NoInit<double>> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr[nr]; }
};

struct Error {
  int code;
  std::string msg;
};

Csr csr_copy(int64_t nr, int64_t nc, const int64_t* ptr, const int32_t* ind, const double* val);
// rows/cols: kept indices (ascending); structure of A restricted to them, explicit zeros kept
Csr submatrix(const Csr& A, const std::vector<int64_t>& rows, const std::vector<int64_t>& cols);
Csr transpose(const Csr& A);
// threads of the host setup: hardware threads, or MAS_SETUP_THREADS, at most 16
int setup_threads();
// f(lo, hi) over [0, n) in contiguous ascending chunks, one per thread
void parallel_rows(int64_t n, const std::function<void(int64_t, int64_t)>& f);
// C = A B with the structural pattern of the product (no entry dropped)
Csr spgemm(const Csr& A, const Csr& B);
Csr galerkin(const Csr& P, const Csr& A);  // P^T A P
Csr block_diag(const std::vector<const Csr*>& blocks);
void spmv(const Csr& A, const double* x, double* y);

// ---- smoothed aggregation for one scalar field
// Strength of connection: kind 0 = evolution measure (Section 3.2) with filter
// eps, kind 1 = symmetric a_ij^2 >= theta^2 a_ii a_jj.
struct SocParams {
  int kind = 0;
  double theta = 0.02;
  double eps = 4.0;
};
// strong off-diagonal pairs of A (symmetric pattern, values 1); B: near-null vector
Csr strength_graph(const Csr& A, const std::vector<double>& B, const SocParams& soc);
// standard three-pass aggregation of a strength graph, nodes in index order
std::vector<int32_t> aggregate(const Csr& S, int32_t* n_agg);
void sa_field(const Csr& A, const SocParams& soc, int max_coarse, int max_levels,
              std::vector<Csr>& Ps, std::vector<std::vector<double>>& Bs);
// sa_field for several fields at once, one thread per field.
void sa_fields(const std::vector<Csr>& A, const SocParams& soc, int max_coarse, int max_levels,
               std::vector<std::vector<Csr>>& Ps, std::vector<std::vector<std::vector<double>>>& Bs);
// Largest matrix the dense coarsest solve takes (rows, border included) unless
// max_coarse is larger: a coarsening that stalls above it is refused
// (std::runtime_error naming `what`) instead of inverting a matrix of that size.
constexpr int64_t kMaxDenseCoarse = 8192;
void check_dense_coarse(int64_t n, int max_coarse, const char* what);

// ---- Vanka patches of one level (velocity rows sorted, then the seeds)
struct PatchSet {
  int32_t dim = 2;
  std::vector<int64_t> off;   // np + 1 offsets into dofs
  std::vector<int32_t> dofs;  // level DoF ids
  std::vector<int32_t> dims;  // np x 4: DoFs per velocity component (3 slots) and seeds
  std::vector<int64_t> foff;  // np + 1 offsets into the packed factor store
  std::vector<int32_t> inv_ptr, inv_pos;  // DoF -> positions in dofs (ascending)
  std::vector<double> w;      // partition of unity per DoF
  int64_t np() const { return (int64_t)off.size() - 1; }
  int32_t max_m = 0;
  int64_t max_f = 0;
  bool shared = false;  // every patch's velocity blocks are identical across components
};
PatchSet patches_single_seed(const Csr& K, const std::vector<int8_t>& field, int dim);
// True when, in every patch, the velocity block of each component equals the
// component-0 block value for value (bitwise): the level's component blocks
// of K are identical under the order-preserving map between the components'
// DoFs (the vector Laplacian with the same boundary conditions on every
// component, Section 2), and every patch holds, for each component, the
// images of its component-0 DoFs.  The patch factors then hold one A^-1 for
// all components (the block-diagonal structure of Section 3.3.1, with the
// blocks' equality used as well).
bool identical_component_blocks(const Csr& K, const std::vector<int8_t>& field, int dim, const PatchSet& ps);
PatchSet patches_element_seeds(const Csr& K, const std::vector<int8_t>& field, int dim,
                               const std::vector<int32_t>& seeds, int ns);

// ---- misc
double lanczos_max(const Csr& A, uint64_t seed, int steps);
double lanczos_max_op(int64_t n, const std::function<void(const double*, double*)>& op, uint64_t seed,
                      int steps);
uint64_t splitmix64(uint64_t seed, uint64_t counter);

}  // namespace mas
