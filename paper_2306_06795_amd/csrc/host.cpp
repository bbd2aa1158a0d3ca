// Host-side setup pieces of libmas (see host.hpp).
#include "host.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <future>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>

namespace mas {

int setup_threads() {
  static const int n = [] {
    int t = (int)std::thread::hardware_concurrency();
    if (const char* e = std::getenv("MAS_SETUP_THREADS")) t = std::atoi(e);
    return std::max(1, std::min(t, 16));
  }();
  return n;
}

// f(lo, hi) over [0, n) in contiguous chunks, one per thread
void parallel_rows(int64_t n, const std::function<void(int64_t, int64_t)>& f) {
  const int64_t nt = std::min<int64_t>(setup_threads(), std::max<int64_t>(1, n / 4096));
  if (nt <= 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt);
  for (auto& x : th) x.join();
}

Csr csr_copy(int64_t nr, int64_t nc, const int64_t* ptr, const int32_t* ind, const double* val) {
  Csr A;
  A.nr = nr;
  A.nc = nc;
  A.ptr.assign(ptr, ptr + nr + 1);
  const int64_t nnz = A.ptr[nr];
  A.ind.resize(nnz);
  A.val.resize(nnz);
  parallel_rows(nnz, [&](int64_t lo, int64_t hi) {
    std::copy(ind + lo, ind + hi, A.ind.begin() + lo);
    std::copy(val + lo, val + hi, A.val.begin() + lo);
  });
  return A;
}

Csr submatrix(const Csr& A, const std::vector<int64_t>& rows, const std::vector<int64_t>& cols) {
  std::vector<int64_t> cmap(A.nc, -1);
  for (size_t k = 0; k < cols.size(); ++k) cmap[cols[k]] = (int64_t)k;
  Csr B;
  B.nr = (int64_t)rows.size();
  B.nc = (int64_t)cols.size();
  B.ptr.assign(B.nr + 1, 0);
  parallel_rows(B.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      const int64_t i = rows[r];
      int64_t c = 0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (cmap[A.ind[e]] >= 0) ++c;
      B.ptr[r + 1] = c;
    }
  });
  for (int64_t r = 0; r < B.nr; ++r) B.ptr[r + 1] += B.ptr[r];
  B.ind.resize(B.ptr[B.nr]);
  B.val.resize(B.ptr[B.nr]);
  parallel_rows(B.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      int64_t i = rows[r], o = B.ptr[r];
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        const int64_t j = cmap[A.ind[e]];
        if (j >= 0) {  // cols ascending -> mapped indices stay sorted
          B.ind[o] = (int32_t)j;
          B.val[o] = A.val[e];
          ++o;
        }
      }
    }
  });
  return B;
}

Csr transpose(const Csr& A) {
  Csr T;
  T.nr = A.nc;
  T.nc = A.nr;
  T.ptr.assign(T.nr + 1, 0);
  for (int64_t e = 0; e < A.nnz(); ++e) T.ptr[A.ind[e] + 1]++;
  for (int64_t i = 0; i < T.nr; ++i) T.ptr[i + 1] += T.ptr[i];
  T.ind.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nr; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      int64_t o = pos[A.ind[e]]++;
      T.ind[o] = (int32_t)i;
      T.val[o] = A.val[e];
    }
  return T;
}

// Rows are independent and each entry is summed in the order of A's row, so the
// result does not depend on the number of threads.
Csr spgemm(const Csr& A, const Csr& B) {
  if (A.nc != B.nr) throw std::runtime_error("spgemm: shape mismatch");
  Csr C;
  C.nr = A.nr;
  C.nc = B.nc;
  C.ptr.assign(C.nr + 1, 0);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    std::vector<int64_t> mark(B.nc, -1);
    for (int64_t i = lo; i < hi; ++i) {
      int64_t c = 0;
      for (int64_t a = A.ptr[i]; a < A.ptr[i + 1]; ++a) {
        const int64_t k = A.ind[a];
        for (int64_t b = B.ptr[k]; b < B.ptr[k + 1]; ++b) {
          const int64_t j = B.ind[b];
          if (mark[j] != i) {
            mark[j] = i;
            ++c;
          }
        }
      }
      C.ptr[i + 1] = c;
    }
  });
  for (int64_t i = 0; i < C.nr; ++i) C.ptr[i + 1] += C.ptr[i];
  C.ind.resize(C.ptr[C.nr]);
  C.val.resize(C.ptr[C.nr]);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    std::vector<int64_t> mark(B.nc, -1);
    std::vector<double> acc(B.nc, 0.0);
    std::vector<int32_t> cols;
    for (int64_t i = lo; i < hi; ++i) {
      cols.clear();
      for (int64_t a = A.ptr[i]; a < A.ptr[i + 1]; ++a) {
        const int64_t k = A.ind[a];
        const double av = A.val[a];
        for (int64_t b = B.ptr[k]; b < B.ptr[k + 1]; ++b) {
          const int64_t j = B.ind[b];
          if (mark[j] != i) {
            mark[j] = i;
            cols.push_back((int32_t)j);
            acc[j] = av * B.val[b];
          } else {
            acc[j] += av * B.val[b];
          }
        }
      }
      std::sort(cols.begin(), cols.end());
      int64_t o = C.ptr[i];
      for (int32_t j : cols) {
        C.ind[o] = j;
        C.val[o] = acc[j];
        ++o;
      }
    }
  });
  return C;
}

Csr galerkin(const Csr& P, const Csr& A) { return spgemm(transpose(P), spgemm(A, P)); }

Csr block_diag(const std::vector<const Csr*>& blocks) {
  Csr C;
  for (auto* b : blocks) {
    C.nr += b->nr;
    C.nc += b->nc;
  }
  C.ptr.assign(1, 0);
  int64_t roff = 0, coff = 0;
  (void)roff;
  for (auto* b : blocks) {
    for (int64_t i = 0; i < b->nr; ++i) {
      for (int64_t e = b->ptr[i]; e < b->ptr[i + 1]; ++e) {
        C.ind.push_back((int32_t)(b->ind[e] + coff));
        C.val.push_back(b->val[e]);
      }
      C.ptr.push_back((int64_t)C.ind.size());
    }
    coff += b->nc;
  }
  return C;
}

void spmv(const Csr& A, const double* x, double* y) {
  for (int64_t i = 0; i < A.nr; ++i) {
    double s = 0.0;
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) s += A.val[e] * x[A.ind[e]];
    y[i] = s;
  }
}

// ---------------------------------------------------------------------------
// smoothed aggregation, one scalar field

static std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d(A.nr, 0.0);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (A.ind[e] == i) d[i] = A.val[e];
  });
  return d;
}

// Gershgorin bound max_i sum_j |a_ij| / a_ii of rho(D^-1 A), each row summed in
// row order (the same bound sets the evolution time step and the smoothing
// weight; it does not depend on the thread count).
static double gershgorin_rho(const Csr& A, const std::vector<double>& d) {
  std::vector<double> ratio(A.nr);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      double s = 0.0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) s += std::fabs(A.val[e]);
      ratio[i] = s / d[i];
    }
  });
  double rho = 0.0;
  for (int64_t i = 0; i < A.nr; ++i) rho = std::max(rho, ratio[i]);
  return rho;
}

// Strong-pattern builder: keep(i, e) decides entry e of row i; rows are counted,
// then filled, in parallel.
template <class Keep>
static Csr select_entries(const Csr& A, Keep keep) {
  Csr S;
  S.nr = S.nc = A.nr;
  S.ptr.assign(A.nr + 1, 0);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t c = 0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) c += keep(i, e) ? 1 : 0;
      S.ptr[i + 1] = c;
    }
  });
  for (int64_t i = 0; i < A.nr; ++i) S.ptr[i + 1] += S.ptr[i];
  S.ind.resize(S.ptr[A.nr]);
  parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t o = S.ptr[i];
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (keep(i, e)) S.ind[o++] = A.ind[e];
    }
  });
  S.val.assign(S.ind.size(), 1.0);
  return S;
}

// Classical symmetric strength: j != i with a_ij^2 >= theta^2 (a_ii a_jj).
static Csr strength_symmetric(const Csr& A, double theta) {
  std::vector<double> d = diagonal(A);
  const double th2 = theta * theta;
  return select_entries(A, [&](int64_t i, int64_t e) {
    const int64_t j = A.ind[e];
    const double v = A.val[e];
    return j != i && v * v >= th2 * (d[i] * d[j]);
  });
}

// Evolution strength (Section 3.2; Olson, Schroder, Tuminaro, NLAA 2010), two
// relaxation steps.  With J = I - dt D^-1 A (dt = 1 / Gershgorin bound), the
// evolved delta of point i is z_i = J J e_i, so for a stored neighbour j
//   z_i[j] = sum_m J[j][m] J[m][i]      (m over row j of A, ascending),
// read from row j of A and column i of A (row i of A^T, held as a dense
// column of J per row i in a thread-private scratch).  The near-null vector
// B gives the constrained approximation zt_j = z_i[i] B_j / B_i, and
//   s_ij = max(|zt_j - z_i[j]| / |z_i[j]|, 1e-4),
// infinite when z_i[j] = 0 or zt_j z_i[j] <= 0.  Row i keeps j when
// s_ij <= eps * min_m s_im (finite), and the graph is the union of the kept
// pairs and their transposes.
static Csr strength_evolution(const Csr& A, const std::vector<double>& B, double eps) {
  const int64_t n = A.nr;
  std::vector<double> d = diagonal(A);
  const double dt = 1.0 / gershgorin_rho(A, d);
  const Csr At = transpose(A);
  // J[r][c] for stored (r, c) of A: delta_rc - dt * ((1 / d_r) a_rc)
  auto jv = [&](int64_t r, int64_t c, double a) { return (r == c ? 1.0 : 0.0) - dt * ((1.0 / d[r]) * a); };
  std::vector<double> s(A.nnz());
  std::vector<char> keep(A.nnz(), 0);
  parallel_rows(n, [&](int64_t lo, int64_t hi) {
    std::vector<double> colJ(n, 0.0);
    std::vector<int64_t> mark(n, -1);
    for (int64_t i = lo; i < hi; ++i) {
      // column i of J: J[m][i] for m with a_mi stored
      for (int64_t e = At.ptr[i]; e < At.ptr[i + 1]; ++e) {
        const int64_t m = At.ind[e];
        colJ[m] = jv(m, i, At.val[e]);
        mark[m] = i;
      }
      auto zcol = [&](int64_t r) {  // z_i[r] = sum_m J[r][m] J[m][i]
        double z = 0.0;
        for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) {
          const int64_t m = A.ind[e];
          if (mark[m] == i) z += jv(r, m, A.val[e]) * colJ[m];
        }
        return z;
      };
      const double zii = zcol(i);
      double smin = INFINITY;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        const int64_t j = A.ind[e];
        s[e] = INFINITY;
        if (j == i) continue;
        const double zij = zcol(j);
        const double zt = zii * B[j] / B[i];
        if (zij != 0.0 && zt * zij > 0.0) s[e] = std::max(std::fabs(zt - zij) / std::fabs(zij), 1e-4);
        smin = std::min(smin, s[e]);
      }
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        keep[e] = A.ind[e] != i && std::isfinite(s[e]) && s[e] <= eps * smin;
    }
  });
  Csr S1 = select_entries(A, [&](int64_t, int64_t e) { return keep[e] != 0; });
  const Csr S1t = transpose(S1);
  // union of S1 and its transpose, rows sorted
  Csr S;
  S.nr = S.nc = n;
  S.ptr.assign(n + 1, 0);
  auto merge = [&](int64_t i, int32_t* out) {
    int64_t a = S1.ptr[i], ae = S1.ptr[i + 1], b = S1t.ptr[i], be = S1t.ptr[i + 1], c = 0;
    while (a < ae || b < be) {
      int32_t v;
      if (b >= be || (a < ae && S1.ind[a] < S1t.ind[b])) v = S1.ind[a++];
      else if (a >= ae || S1t.ind[b] < S1.ind[a]) v = S1t.ind[b++];
      else { v = S1.ind[a++]; ++b; }
      if (out) out[c] = v;
      ++c;
    }
    return c;
  };
  parallel_rows(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) S.ptr[i + 1] = merge(i, nullptr);
  });
  for (int64_t i = 0; i < n; ++i) S.ptr[i + 1] += S.ptr[i];
  S.ind.resize(S.ptr[n]);
  parallel_rows(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) merge(i, &S.ind[S.ptr[i]]);
  });
  S.val.assign(S.ind.size(), 1.0);
  return S;
}

Csr strength_graph(const Csr& A, const std::vector<double>& B, const SocParams& soc) {
  if (soc.kind == 1) return strength_symmetric(A, soc.theta);
  return strength_evolution(A, B, soc.eps);
}

std::vector<int32_t> aggregate(const Csr& S, int32_t* n_agg) {
  const int64_t n = S.nr;
  std::vector<int32_t> agg(n, -1);
  std::vector<char> first(n, 0);
  int32_t na = 0;
  // pass 1: seed where every strong neighbour is still free
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
      if (agg[S.ind[e]] >= 0) {
        free_nb = false;
        break;
      }
    if (!free_nb) continue;
    agg[i] = na;
    first[i] = 1;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e) {
      agg[S.ind[e]] = na;
      first[S.ind[e]] = 1;
    }
    ++na;
  }
  // pass 2: join the aggregate of the lowest-numbered strong neighbour from pass 1
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
      if (first[S.ind[e]]) {
        agg[i] = agg[S.ind[e]];
        break;
      }
  }
  // pass 3: new aggregates from what is left
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
      if (agg[S.ind[e]] < 0) agg[S.ind[e]] = na;
    ++na;
  }
  *n_agg = na;
  return agg;
}

void sa_field(const Csr& A0, const SocParams& soc, int max_coarse, int max_levels, std::vector<Csr>& Ps,
              std::vector<std::vector<double>>& Bs) {
  Ps.clear();
  Bs.clear();
  std::vector<double> B(A0.nr, 1.0);
  Bs.push_back(B);
  Csr A = A0;
  while (A.nr > max_coarse && (int)Ps.size() + 1 < max_levels) {
    int32_t nc = 0;
    std::vector<int32_t> agg = aggregate(strength_graph(A, B, soc), &nc);
    if (nc >= A.nr) break;
    // tentative interpolation from the near-null vector
    std::vector<double> nrm2(nc, 0.0);
    for (int64_t i = 0; i < A.nr; ++i) nrm2[agg[i]] += B[i] * B[i];
    std::vector<double> Bc(nc);
    for (int32_t J = 0; J < nc; ++J) Bc[J] = std::sqrt(nrm2[J]);
    Csr T;
    T.nr = A.nr;
    T.nc = nc;
    T.ptr.resize(A.nr + 1);
    T.ind.resize(A.nr);
    T.val.resize(A.nr);
    for (int64_t i = 0; i < A.nr; ++i) {
      T.ptr[i] = i;
      T.ind[i] = agg[i];
      T.val[i] = B[i] / Bc[agg[i]];
    }
    T.ptr[A.nr] = A.nr;
    // P = (I - omega D^-1 A) T, omega = (4/3) / max_i sum_j |a_ij| / a_ii
    std::vector<double> d = diagonal(A);
    const double omega = (4.0 / 3.0) / gershgorin_rho(A, d);
    Csr DA = A;
    parallel_rows(A.nr, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i)
        for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) DA.val[e] = A.val[e] / d[i];
    });
    Csr P = spgemm(DA, T);
    parallel_rows(P.nr, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i)
        for (int64_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) {
          double v = -omega * P.val[e];
          if (P.ind[e] == agg[i]) v += T.val[i];
          P.val[e] = v;
        }
    });
    A = galerkin(P, A);
    Ps.push_back(std::move(P));
    B = Bc;
    Bs.push_back(B);
  }
}

void check_dense_coarse(int64_t n, int max_coarse, const char* what) {
  const int64_t lim = std::max<int64_t>(max_coarse, kMaxDenseCoarse);
  if (n > lim)
    throw std::runtime_error(std::string(what) + ": smoothed aggregation stopped at " + std::to_string(n) +
                             " unknowns, more than the dense coarsest solve takes (" + std::to_string(lim) +
                             "): raise max_levels or max_coarse, or use the evolution strength measure");
}

// One hierarchy per field, the fields on threads of their own (each field's
// hierarchy is the same as when built alone).
void sa_fields(const std::vector<Csr>& A, const SocParams& soc, int max_coarse, int max_levels,
               std::vector<std::vector<Csr>>& Ps, std::vector<std::vector<std::vector<double>>>& Bs) {
  const size_t nf = A.size();
  Ps.assign(nf, {});
  Bs.assign(nf, {});
  if (setup_threads() <= 1 || nf <= 1) {
    for (size_t f = 0; f < nf; ++f) sa_field(A[f], soc, max_coarse, max_levels, Ps[f], Bs[f]);
    return;
  }
  std::vector<std::future<void>> jobs;
  for (size_t f = 0; f < nf; ++f)
    jobs.push_back(std::async(std::launch::async, [&, f] { sa_field(A[f], soc, max_coarse, max_levels, Ps[f], Bs[f]); }));
  for (auto& j : jobs) j.wait();
  for (auto& j : jobs) j.get();  // rethrows the first field's error, if any
}

// ---------------------------------------------------------------------------
// Vanka patches

static void finish_patches(PatchSet& ps, int64_t n) {
  const int64_t np = ps.np();
  ps.inv_ptr.assign(n + 1, 0);
  for (int32_t j : ps.dofs) ps.inv_ptr[j + 1]++;
  for (int64_t j = 0; j < n; ++j) ps.inv_ptr[j + 1] += ps.inv_ptr[j];
  ps.inv_pos.resize(ps.dofs.size());
  std::vector<int32_t> fill(ps.inv_ptr.begin(), ps.inv_ptr.end() - 1);
  for (size_t k = 0; k < ps.dofs.size(); ++k) ps.inv_pos[fill[ps.dofs[k]]++] = (int32_t)k;
  ps.w.assign(n, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    int32_t c = ps.inv_ptr[j + 1] - ps.inv_ptr[j];
    if (c > 0) ps.w[j] = 1.0 / (double)c;
  }
  ps.foff.assign(np + 1, 0);
  ps.max_m = 0;
  ps.max_f = 0;
  for (int64_t p = 0; p < np; ++p) {
    const int32_t* d = &ps.dims[4 * p];
    int64_t nv = d[0] + d[1] + d[2], ns = d[3];
    int64_t f = 0;
    for (int c = 0; c < 3; ++c) f += (int64_t)d[c] * (d[c] + 1) / 2;
    f += nv * ns + ns * (ns + 1) / 2;
    ps.foff[p + 1] = ps.foff[p] + f;
    ps.max_m = std::max<int32_t>(ps.max_m, (int32_t)(nv + ns));
    ps.max_f = std::max(ps.max_f, f);
  }
}

static void push_patch(PatchSet& ps, const std::vector<int32_t>& vel, const std::vector<int8_t>& field,
                       const int32_t* seeds, int ns) {
  int32_t cnt[3] = {0, 0, 0};
  for (int32_t j : vel) {
    cnt[field[j]]++;
    ps.dofs.push_back(j);
  }
  for (int s = 0; s < ns; ++s) ps.dofs.push_back(seeds[s]);
  ps.dims.push_back(cnt[0]);
  ps.dims.push_back(cnt[1]);
  ps.dims.push_back(cnt[2]);
  ps.dims.push_back(ns);
  ps.off.push_back((int64_t)ps.dofs.size());
}

PatchSet patches_single_seed(const Csr& K, const std::vector<int8_t>& field, int dim) {
  PatchSet ps;
  ps.dim = dim;
  ps.off.push_back(0);
  std::vector<int32_t> vel;
  for (int64_t i = 0; i < K.nr; ++i) {
    if (field[i] != dim) continue;
    vel.clear();
    for (int64_t e = K.ptr[i]; e < K.ptr[i + 1]; ++e)
      if (field[K.ind[e]] < dim) vel.push_back(K.ind[e]);  // already ascending
    int32_t seed = (int32_t)i;
    push_patch(ps, vel, field, &seed, 1);
  }
  finish_patches(ps, K.nr);
  return ps;
}

PatchSet patches_element_seeds(const Csr& K, const std::vector<int8_t>& field, int dim,
                               const std::vector<int32_t>& seeds, int ns) {
  PatchSet ps;
  ps.dim = dim;
  ps.off.push_back(0);
  std::vector<int32_t> vel;
  const int64_t ne = (int64_t)seeds.size() / ns;
  for (int64_t e = 0; e < ne; ++e) {
    vel.clear();
    for (int s = 0; s < ns; ++s) {
      int64_t i = seeds[e * ns + s];
      for (int64_t k = K.ptr[i]; k < K.ptr[i + 1]; ++k)
        if (field[K.ind[k]] < dim) vel.push_back(K.ind[k]);
    }
    std::sort(vel.begin(), vel.end());
    vel.erase(std::unique(vel.begin(), vel.end()), vel.end());
    push_patch(ps, vel, field, &seeds[e * ns], ns);
  }
  finish_patches(ps, K.nr);
  return ps;
}

bool identical_component_blocks(const Csr& K, const std::vector<int8_t>& field, int dim, const PatchSet& ps) {
  if (dim < 2 || ps.np() == 0) return false;
  std::vector<std::vector<int32_t>> idx(dim);  // DoFs of each component, ascending
  for (int64_t i = 0; i < K.nr; ++i)
    if (field[i] < dim) idx[field[i]].push_back((int32_t)i);
  const size_t m = idx[0].size();
  for (int c = 1; c < dim; ++c)
    if (idx[c].size() != m) return false;
  std::vector<int32_t> rank(K.nr, -1);  // position of a velocity DoF within its component
  for (int c = 0; c < dim; ++c)
    for (size_t k = 0; k < m; ++k) rank[idx[c][k]] = (int32_t)k;
  // row k of the component-c block against row k of the component-0 block:
  // the same columns (by rank; rows are sorted, ranks keep the order) and the
  // same bits
  std::atomic<bool> same{true};
  parallel_rows((int64_t)m, [&](int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, double>> a, b;
    auto row = [&](int c, int64_t k, std::vector<std::pair<int32_t, double>>& out) {
      out.clear();
      const int32_t r = idx[c][k];
      for (int64_t e = K.ptr[r]; e < K.ptr[r + 1]; ++e)
        if (field[K.ind[e]] == c) out.emplace_back(rank[K.ind[e]], K.val[e]);
    };
    for (int64_t k = lo; k < hi && same.load(std::memory_order_relaxed); ++k) {
      row(0, k, a);
      for (int c = 1; c < dim; ++c) {
        row(c, k, b);
        bool eq = a.size() == b.size();
        for (size_t q = 0; eq && q < a.size(); ++q)
          eq = a[q].first == b[q].first && std::memcmp(&a[q].second, &b[q].second, sizeof(double)) == 0;
        if (!eq) {
          same.store(false, std::memory_order_relaxed);
          break;
        }
      }
    }
  });
  if (!same.load()) return false;
  // every patch: equal component counts, component c's DoFs at [c n, (c + 1) n)
  // of its velocity list, each the image of the component-0 DoF at the same place
  for (int64_t p = 0; p < ps.np(); ++p) {
    const int32_t* q = &ps.dims[4 * p];
    const int32_t n = q[0];
    if (n == 0) return false;
    for (int c = 0; c < 3; ++c)
      if (q[c] != (c < dim ? n : 0)) return false;
    const int32_t* D = &ps.dofs[ps.off[p]];
    for (int c = 0; c < dim; ++c)
      for (int32_t i = 0; i < n; ++i) {
        const int32_t j = D[c * n + i];
        if (field[j] != c || (c > 0 && j != idx[c][rank[D[i]]])) return false;
      }
  }
  return true;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014) and Lanczos

uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence bisection
static double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // number of eigenvalues < x
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
      double qq = q == 0.0 ? 1e-300 : q;
      q = a[i] - x - b[i - 1] * b[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= n) hi = mid; else lo = mid;
  }
  return hi;
}

double lanczos_max_op(int64_t n, const std::function<void(const double*, double*)>& op, uint64_t seed,
                      int steps) {
  std::vector<std::vector<double>> V;
  std::vector<double> v(n), w(n);
  double nrm = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t z = splitmix64(seed, (uint64_t)i);
    v[i] = (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    nrm += v[i] * v[i];
  }
  nrm = std::sqrt(nrm);
  for (auto& x : v) x /= nrm;
  V.push_back(v);
  std::vector<double> alpha, beta;
  const int k = (int)std::min<int64_t>(steps, n);
  for (int j = 0; j < k; ++j) {
    op(V[j].data(), w.data());
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += V[j][i] * w[i];
    alpha.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (auto& u : V) {
        double c = 0.0;
        for (int64_t i = 0; i < n; ++i) c += u[i] * w[i];
        for (int64_t i = 0; i < n; ++i) w[i] -= c * u[i];
      }
    double bn = 0.0;
    for (int64_t i = 0; i < n; ++i) bn += w[i] * w[i];
    bn = std::sqrt(bn);
    if (j == k - 1 || bn == 0.0) break;
    beta.push_back(bn);
    for (int64_t i = 0; i < n; ++i) v[i] = w[i] / bn;
    V.push_back(v);
  }
  beta.resize(alpha.size() > 0 ? alpha.size() - 1 : 0);
  return tridiag_max_eig(alpha, beta);
}

double lanczos_max(const Csr& A, uint64_t seed, int steps) {
  return lanczos_max_op(A.nr, [&](const double* x, double* y) { spmv(A, x, y); }, seed, steps);
}

}  // namespace mas
