/*
 * mas.h -- C-ABI of libmas: the solve phase of the monolithic defect-correction
 * AMG preconditioner for Stokes saddle systems (Voronin, MacLachlan, Olson,
 * Tuminaro, "Monolithic Algebraic Multigrid Preconditioners for the Stokes
 * Equations", arXiv 2306.06795), on one AMD MI355X (gfx950).
 *
 * The caller hands over the assembled operators the paper's method starts
 * from (Section 3.1): the high-order saddle matrix K0 (Taylor-Hood P2/P1 or
 * Scott-Vogelius P2/P1disc), the low-order P1isoP2/P1 matrix K1 and the
 * pressure stiffness matrix A_p (the auxiliary operator of Algorithm 1), with
 * the DoF-to-field map.  mas_setup builds the hierarchy and relaxation data,
 * mas_apply applies one defect-correction cycle (eq. (3.1)), mas_solve runs
 * restarted right-preconditioned FGMRES(restart) with that preconditioner
 * (Section 4).
 *
 * Conventions
 *  - Unknowns are field-blocked: [u_0; ...; u_{dim-1}; p].  field[i] is the
 *    velocity component 0..dim-1 of row i, or dim for a pressure row.
 *  - K0 and K1 are symmetric, full size, with Dirichlet velocity rows stored
 *    as identity rows and their columns removed (Dirichlet data lifted into
 *    the right-hand side by the caller).  Column indices sorted in each row.
 *  - Host arrays passed to mas_setup are borrowed for the duration of the
 *    call only.  Device arrays passed to mas_apply / mas_solve are owned by
 *    the caller.  All device work is enqueued on the stream given (a
 *    hipStream_t passed as void*; NULL = the default stream).
 *  - Every function returns a status code (MAS_OK = 0, a warning > 0, an
 *    error < 0); mas_last_error() gives a thread-local message for the last
 *    failing call.  No C++ exception crosses this interface.
 *  - A handle may be used from one host thread and one stream at a time.
 */
#ifndef MAS_H
#define MAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mas_handle mas_handle;

enum mas_status {
  MAS_OK = 0,
  MAS_NOT_CONVERGED = 1,   /* warning: max_it reached, x holds the last iterate */
  MAS_EINVAL = -1,         /* bad argument, shape or field-map mismatch, non-finite value */
  MAS_ESINGULAR_PATCH = -2,/* a patch block or Schur complement is singular (message names it) */
  MAS_ENOMEM = -3,         /* device or host allocation failed */
  MAS_EHIP = -4,           /* a HIP runtime call failed */
  MAS_ENAN = -5            /* the residual became NaN or Inf */
};

enum mas_disc { MAS_TH = 0, MAS_SV = 1 };                 /* Section 2.1 */
/* Sections 3.3.1, 3.3.2; MAS_RELAX_VANKA_DLSC is the hybrid of the Scott-Vogelius
 * parameter study (Section 4, Table 4): Vanka on K0 (nu1/nu2 sweeps, omega0) and
 * nu_dlsc DLSC sweeps on every relaxed level of the K1 hierarchy. */
enum mas_relax { MAS_RELAX_VANKA = 0, MAS_RELAX_DLSC = 1, MAS_RELAX_VANKA_DLSC = 2 };
/* Section 4.  MAS_HO_AMG: Algorithm 1 applied to K0 itself (the remark after
 * Algorithm 1, compared in Section 4): the hierarchy starts at K0, there is no
 * defect-correction level, eta_u/eta_p and omega0 are not used (omega on every
 * level), and K1/field1/dir1 of mas_problem are not read (Ap is).  Taylor-Hood
 * only: mas_setup/mas_analyze return MAS_EINVAL for Scott-Vogelius. */
enum mas_schedule { MAS_DC_ALL = 0, MAS_DC_SKIP1 = 1, MAS_DC_SKIP0 = 2, MAS_HO_AMG = 3 };
enum mas_precision { MAS_FP64 = 0, MAS_FP32 = 1 };        /* number type of the cycle */
/* Strength of connection of Algorithm 1.  MAS_SOC_EVOLUTION: the evolution
 * measure Section 3.2 uses (Olson, Schroder, Tuminaro, NLAA 2010): two Jacobi
 * steps z_i = (I - dt D^-1 A)^2 e_i, dt = 1 / max_i sum_j |a_ij| / a_ii; for a
 * stored neighbour j, s_ij = |zt_j - z_i[j]| / |z_i[j]| with zt = z_i[i] B / B_i
 * (B the level's near-null vector), infinite when z_i[j] = 0 or zt_j z_i[j] <= 0,
 * floored at 1e-4; j is strong for i when s_ij <= soc_eps min_k s_ik; the graph
 * is symmetrised (union).  MAS_SOC_SYMMETRIC: a_ij^2 >= theta^2 a_ii a_jj, the
 * classical measure Section 3.2 reports needed tuning. */
enum mas_soc { MAS_SOC_EVOLUTION = 0, MAS_SOC_SYMMETRIC = 1 };
/* Orthogonalisation of the FGMRES Arnoldi step (Section 4): classical
 * Gram-Schmidt in one pass (every dot product of the step in one sweep over
 * the basis), or modified Gram-Schmidt (one basis vector at a time). */
enum mas_gram_schmidt { MAS_GS_CLASSICAL = 0, MAS_GS_MODIFIED = 1 };

/* CSR matrix in host memory: row pointers int64 (nrows+1), column indices
 * int32 (sorted within each row), values FP64.  Explicitly stored zeros are
 * part of the structure (patches are read from structure, Section 3.3.1). */
typedef struct {
  int64_t nrows, ncols;
  const int64_t* indptr;
  const int32_t* indices;
  const double* data;
} mas_csr;

typedef struct {
  int32_t dim;            /* 2 or 3 */
  int32_t disc;           /* mas_disc */
  mas_csr K0;             /* high-order saddle operator, n0 x n0 */
  mas_csr K1;             /* P1isoP2/P1 saddle operator, n1 x n1 (same velocity DoFs as K0) */
  mas_csr Ap;             /* pressure stiffness of K1's pressure space, np1 x np1 */
  const int8_t* field0;   /* n0 */
  const int8_t* field1;   /* n1 */
  const uint8_t* dir0;    /* n0, 1 = Dirichlet row */
  const uint8_t* dir1;    /* n1 */
  int32_t p_nullspace;    /* 1: velocity prescribed on the whole boundary, the
                             pressure is determined up to a constant (Section 2) */
  const double* p_weight0;/* np0 = #pressure rows of K0: int psi_i (zero-mean
                             pressure after mas_solve); may be NULL */
  const double* mu_diag0; /* nu0 = #velocity rows of K0: diagonal velocity mass
                             for DLSC on K0 (Section 3.3.2); NULL = identity */
  /* Scott-Vogelius only (Section 3.1): */
  int64_t n_elem;         /* number of elements */
  const int64_t* elem_p0; /* n_elem x 3: K0 row ids of each element's pressures */
  mas_csr Pp0;            /* np0 x np1 duplication P1 -> P1disc */
  mas_csr Mdg;            /* np0 x np0 P1disc mass */
  mas_csr Mcg;            /* np1 x np1 P1 mass */
  /* Optional prebuilt hierarchy (Algorithm 1 skipped; for parity runs that
   * must use a hierarchy built elsewhere).  n_prebuilt = 0: smoothed
   * aggregation builds the hierarchy.  n_prebuilt = L > 0: L coarsening steps,
   * prebuilt_P[l * (dim + 1) + f] (host CSR) interpolates field f (0..dim-1:
   * velocity components, dim: pressure) from hierarchy level l + 1 to level l,
   * level 0 being K1 on its free DoFs (K0 for MAS_HO_AMG); its rows are the
   * field's DoFs of the finer level in increasing order, its columns the
   * field's DoFs of the coarser level.  The coarse operators are the Galerkin
   * products of eq. (3.4).  prebuilt_null_p (required when p_nullspace is set):
   * the pressure near-null vector on the coarsest level (columns of the last
   * pressure interpolation), used to border the coarsest solve.  Borrowed for
   * the call like every host array.  The smoothed-aggregation hierarchies of
   * the DLSC AMG stages (dlsc_amg > 0) are still built by the library. */
  int32_t n_prebuilt;
  const mas_csr* prebuilt_P;
  const double* prebuilt_null_p;
} mas_problem;

typedef struct {
  int32_t relax;          /* mas_relax on levels >= 0 */
  int32_t schedule;       /* mas_schedule */
  int32_t nu1, nu2;       /* pre/post relaxation sweeps per level (wrapped relaxations when
                             krylov_its > 0) */
  double omega0, omega;   /* Vanka damping on K0 and on the K1 hierarchy */
  double eta_u, eta_p;    /* residual weights of eq. (3.2) */
  int32_t cheb_deg[3];    /* DLSC Chebyshev degrees (momentum, continuity, pressure; Table 2) */
  int32_t precision;      /* mas_precision of the cycle (FGMRES is always FP64) */
  int32_t restart;        /* FGMRES restart length (20 in Section 4) */
  int32_t max_coarse;     /* per-field coarsest size of smoothed aggregation */
  int32_t max_levels;     /* per-field maximum number of levels */
  double theta;           /* threshold of MAS_SOC_SYMMETRIC: a_ij^2 >= theta^2 a_ii a_jj */
  uint64_t seed;          /* SplitMix64 seed of the Lanczos start vectors */
  double mass_rtol;       /* relative tolerance of the SV pressure-mass solve */
  int32_t nrhs_max;       /* most right-hand sides one mas_apply / mas_solve may carry (1..64) */
  int32_t krylov_its;     /* 0: damped stationary Vanka sweeps (omega0, omega); k = 1..8: each
                             wrapped relaxation is k iterations of FGMRES preconditioned by one
                             undamped Vanka sweep (Section 3.3.1), on every Vanka level except
                             K0 of Scott-Vogelius (stationary there); one right-hand side per call */
  int32_t nu_dlsc;        /* MAS_RELAX_VANKA_DLSC: DLSC sweeps pre and post on the K1 hierarchy
                             (2, the DLSC sweep count of Section 4); unused otherwise */
  int32_t dlsc_amg;       /* 0: DLSC continuity and pressure-correction stages by Chebyshev (Table 2);
                             k = 1..8: each by one smoothed-aggregation V-cycle on B M^-1 B^T with k
                             weighted-Jacobi sweeps (weight 4/3 over the largest absolute row sum of
                             D^-1 S) before and after the coarse correction (Section 5) */
  int32_t soc;            /* mas_soc (default: MAS_SOC_EVOLUTION for Taylor-Hood, MAS_SOC_SYMMETRIC
                             for Scott-Vogelius, whose Alfeld-mesh pressure the evolution measure
                             coarsens at about half the velocity rate) */
  double soc_eps;         /* evolution filter epsilon (4) */
  int32_t gram_schmidt;   /* mas_gram_schmidt of mas_solve (MAS_GS_CLASSICAL) */
  int32_t autotune;       /* 1: each sparse product's kernel (sliced-ELL or CSR, lanes per row) is
                             chosen by timing at setup, so the summation order of a row may differ
                             between setups; 0: a fixed rule of the operator's shape (the same
                             choice, bit for bit the same results, in every setup) */
  int32_t graphs;         /* 1: each FGMRES iteration replays a captured hipGraph; 0: eager launches
                             (same results) */
  int32_t full_patch_min; /* patch size from which a level without fixed-shape buckets stores its
                             A_c^-1 blocks full instead of packed (512) */
  int32_t bucket_min;     /* fewest patches of one fixed shape that get a thread-per-patch bucket
                             (32768: a bucket pays only once its threads fill the GPU); smaller
                             groups take the generic patch kernels */
  int32_t factor_blocked; /* 1: blocked Gauss-Jordan for patch blocks whose panel fits in LDS;
                             0: single-pivot Gauss-Jordan everywhere */
  int32_t device_galerkin;/* 1 (default): in mas_setup the Galerkin products of the level
                             operators (Algorithm 1) run on the device, each operator kept there
                             for the next product (same values as the host's, bit for bit); 0: on
                             the host */
  int32_t share_blocks;   /* 1: a level whose patches have identical velocity blocks in every
                             component (the vector Laplacian with the same boundary conditions on
                             each component, Section 2; checked bit for bit by the analysis)
                             stores one A^-1 per patch for all components; 0: one per component */
  int32_t patch_kernel;   /* kernel of the patches outside the thread-per-patch buckets: 0 the
                             fastest on each level, timed at upload (autotune = 1; the workgroup
                             kernel with autotune = 0); 1 workgroup per patch; 2 wavefront per
                             patch streaming the packed columns of per-component blocks; 3
                             wavefront per patch on shared blocks; 4 persistent workgroups, each
                             loading its next patch while it solves the current one; 5 panels of
                             a packed shared block streamed through LDS (the kernel of levels
                             whose packed shared records are too large for LDS, taken there also
                             by 0).  A
                             level the requested kernel does not take (2: shared or full blocks,
                             or components above 128 rows; 3: blocks not shared, full, or above
                             128 rows; 4: records that do not fit in LDS or exceed 16 values per
                             thread; 5: blocks not shared or above 1024 rows) uses 1 */
  int32_t device_sa;      /* 1: Algorithm 1's per-field smoothed aggregation runs on the device
                             with each level operator resident there: the Gershgorin bound, the
                             strength of connection (Section 3.2), the smoothed prolongator and the
                             field's Galerkin product; the strength graph goes to the host, whose
                             greedy aggregation (sequential by definition) returns the aggregates
                             and the tentative prolongator's values; the finished prolongators come
                             back as the hierarchy's output.  The same hierarchy as the host's, bit
                             for bit.  Default 1; mas_analyze, which has no device, and 0: on the host */
  int32_t spgemm_cap;     /* 0: the device sparse products of the setup keep up to 1536 distinct
                             columns of a row in LDS and take longer rows through a global-memory
                             kernel; k > 0: at most min(k, 1536) in LDS (a test of the long-row
                             path) */
} mas_params;

typedef struct {
  int32_t iters;          /* FGMRES iterations (preconditioner applications) */
  int32_t converged;
  double relres;          /* true ||b - K0 x|| / ||b|| at exit */
  double conv_factor;     /* geometric mean of the last 10 residual reductions (Section 4) */
} mas_solve_info;

typedef struct {
  int32_t n_levels;       /* 1 (K0) + hierarchy levels K1..K_L */
  int64_t n[16];          /* free rows per level (0 = K0) */
  int64_t nnz[16];        /* stored entries per level operator */
  int64_t n_vel[16];      /* velocity rows per level */
  int64_t n_patches[16];  /* Vanka patches per relaxed level (0 if none) */
  int64_t patch_dofs[16]; /* sum of patch sizes per level */
  int64_t factor_entries[16]; /* stored factor values per level (layout: patch_layout) */
  int64_t p_nnz[16];      /* entries of P_l (level l -> l-1), 0 for l <= 1 */
  int64_t coarse_n;       /* rows of the dense coarsest solve (incl. border) */
  int64_t device_bytes;   /* device memory held by the handle (0 after mas_analyze) */
  int64_t bucket_patches[16]; /* patches per level solved by the thread-per-patch bucket kernels */
  int32_t patch_kernel[16];   /* kernel of the other patches of a level, chosen at upload by
                                 timing: 0 none, 1 workgroup per patch, 2 wavefront per patch
                                 streaming the packed columns of per-component blocks, 3
                                 wavefront per patch streaming the columns of a shared block,
                                 4 persistent pipelined workgroups, 5 panels of a shared block
                                 streamed through LDS */
  int32_t bucket_shapes[16][16]; /* per level, up to 4 bucketed shapes (velocity DoFs per
                                    component x3, seeds), zero-padded, in launch order */
  int32_t patch_layout[16];   /* per level, bits of the factor records' A^-1 part: 1 = blocks
                                 stored full (n x n) instead of packed upper triangles (levels
                                 of patches of full_patch_min DoFs or more, no buckets);
                                 2 = one block for every velocity component (share_blocks) */
} mas_hier_info;

/* Default parameters: Section 4 / Tables 2 and 4 where the paper fixes them. */
void mas_default_params(int32_t dim, int32_t disc, int32_t relax, mas_params* out);

/* Build the hierarchy (Algorithm 1 on K1 and A_p, per-field smoothed
 * aggregation), the Vanka patches of every relaxed level with their block
 * factorisation computed on the GPU in FP64 (eqs. (3.6)-(3.8)), or the DLSC
 * operators, and the dense coarsest-level inverse.
 * Errors: MAS_EINVAL (also when the coarsest level, every field cut at the
 * common depth of Algorithm 1 and the border included, exceeds
 * max(max_coarse, 8192) rows, which the dense coarsest solve would not take),
 * MAS_ESINGULAR_PATCH, MAS_ENOMEM, MAS_EHIP. */
int mas_setup(const mas_problem* prob, const mas_params* par, void* stream, mas_handle** out);

/* Host-only analysis: the hierarchy (Algorithm 1) and the patches, without
 * touching the GPU.  Until mas_upload the handle supports mas_get_info,
 * mas_export_level and mas_destroy only (no device is needed).  Errors as
 * mas_setup. */
int mas_analyze(const mas_problem* prob, const mas_params* par, mas_handle** out);

/* Move an analysed (or released) handle onto the current device: the device
 * half of mas_setup (operator upload, patch factorisation, coarse inverse,
 * solver workspace).  No-op for a handle already on the device.  On error the
 * handle is left analysed-only.  Errors: MAS_ENOMEM, MAS_ESINGULAR_PATCH,
 * MAS_EHIP. */
int mas_upload(mas_handle* h, void* stream);

/* Device bytes mas_upload_ws needs for an analysed (not uploaded) handle: its
 * operators, factors, level vectors and FGMRES basis plus the peak of the
 * setup's temporary work areas, each piece rounded to 256 bytes.  Computed
 * on the host from the analysis (no device is touched; the handle stays
 * analysed-only).  Errors: MAS_EINVAL for NULL arguments or a handle already
 * on the device. */
int mas_workspace_size(mas_handle* h, size_t* bytes);

/* mas_upload into caller-owned device memory: every device array of the
 * handle (and the setup's temporaries) is carved from dev_ws, which must be
 * 256-byte aligned, at least mas_workspace_size bytes, and stay allocated and
 * untouched by the caller until mas_release or mas_destroy returns.  The
 * library allocates only its pinned host staging (a few KB), one internal
 * stream and two events.  Errors: MAS_EINVAL (NULL or misaligned dev_ws, or a
 * handle already on the device), MAS_ENOMEM (ws_bytes too small; the message
 * names the bytes needed so far), MAS_ESINGULAR_PATCH, MAS_EHIP. */
int mas_upload_ws(mas_handle* h, void* dev_ws, size_t ws_bytes, void* stream);

/* Free every device resource of the handle (waits for the device first),
 * keeping the host analysis so that mas_upload can restore it without
 * repeating Algorithm 1.  mas_get_info then reports device_bytes = 0.
 * Errors: MAS_EINVAL for a NULL handle; releasing a released handle is a
 * no-op. */
int mas_release(mas_handle* h);

/* z = B r: one defect-correction cycle (eq. (3.1)) applied to nrhs right-hand
 * sides.  r, z: device FP64, n0 x nrhs row-major (right-hand side fastest),
 * owned by the caller and not retained; r is only read, and z must not
 * overlap it.  Dirichlet rows are returned unchanged (z_D = r_D).
 * Asynchronous on `stream` (NULL: the default stream).  Errors: MAS_EINVAL for
 * NULL arguments, an analysed-only handle or nrhs outside [1, nrhs_max];
 * MAS_EHIP when a launch fails (the contents of z are then undefined). */
int mas_apply(mas_handle* h, const double* r, double* z, int32_t nrhs, void* stream);

/* mas_apply for callers that cannot allocate device memory during the call or
 * must not hold per-handle cycle buffers (code under stream capture, tight
 * serving loops, allocation-free harnesses): the same cycle, the same
 * arguments and the same result as mas_apply, bit for bit, but the cycle's
 * per-application scratch (level vectors, patch outputs, DLSC, relaxation-
 * wrapper and Scott-Vogelius work vectors) lives in a file-scope device array
 * of 64 MiB, one per device, held until the process ends.  The call makes no
 * device or host allocation and no event-timing (mas_set_timing is ignored
 * during it).  Every call on one device shares that device's array and leaves
 * its contents behind (each cycle writes what it reads first): calls that
 * overlap on one device race, so callers serialise them.  Errors as mas_apply,
 * and MAS_EINVAL when the scratch this handle needs for nrhs right-hand sides
 * exceeds 64 MiB (the message names the bytes). */
int mas_apply_static(mas_handle* h, const double* r, double* z, int32_t nrhs, void* stream);

/* FGMRES for K0 x = b from x0 = 0 (Section 4).  b, x: device FP64 n0 x nrhs.
 * Stops when ||b - K0 x|| <= rtol ||b|| (true residual) or after max_it
 * iterations.  With p_nullspace and p_weight0 the returned pressure has zero
 * mean.  info (host, nrhs entries) may be NULL.  Returns MAS_OK,
 * MAS_NOT_CONVERGED or an error.  Synchronises the stream. */
int mas_solve(mas_handle* h, const double* b, double* x, int32_t nrhs, double rtol,
              int32_t max_it, mas_solve_info* info, void* stream);

/* mas_solve with one tolerance per right-hand side (rtol: host array of nrhs,
 * each >= 0).  Column k stops updating once ||b_k - K0 x_k|| <= rtol[k] ||b_k||,
 * so a column's result does not depend on the tolerances of the columns
 * solved beside it.  Errors as mas_solve (MAS_EINVAL for a negative or NaN
 * tolerance). */
int mas_solve_rtols(mas_handle* h, const double* b, double* x, int32_t nrhs, const double* rtol,
                    int32_t max_it, mas_solve_info* info, void* stream);

/* One scheduling step of continuous batching over nrhs right-hand-side slots
 * (a serving layer admits and retires requests between steps).  b, x: device
 * FP64 n0 x nrhs as in mas_solve; rtol, fresh: host arrays of nrhs.  Column k
 * starts from x_k = 0 when fresh[k] != 0 (a request just admitted to slot k),
 * else continues from the x_k it holds; every column not yet at
 * ||b_k - K0 x_k|| <= rtol[k] ||b_k|| then runs at most `cycles` restart cycles
 * of FGMRES(restart) (Section 4), so the iterates of a column are those
 * mas_solve computes for it alone, up to rounding, whatever the other slots
 * do.  A column with b_k = 0 is an idle slot (fresh: x_k = 0).  info (host,
 * nrhs, required): iterations run in this call, converged flag, true relative
 * residual at the end of the call.  Columns that converge in this call get the
 * zero-mean pressure of mas_solve; the others are left as iterates.  Returns
 * MAS_OK when every column has converged, MAS_NOT_CONVERGED otherwise (the
 * caller steps again), or an error (MAS_EINVAL for NULL arguments, cycles < 1,
 * a negative tolerance, nrhs outside [1, nrhs_max] or several right-hand
 * sides with the FGMRES-wrapped relaxation; MAS_ENAN).  Synchronises the
 * stream. */
int mas_solve_step(mas_handle* h, const double* b, double* x, int32_t nrhs, const double* rtol,
                   const int32_t* fresh, int32_t cycles, mas_solve_info* info, void* stream);

/* Sizes of the built hierarchy (host structure owned by the caller), and the
 * device bytes the handle holds.  Errors: MAS_EINVAL for NULL arguments. */
int mas_get_info(const mas_handle* h, mas_hier_info* out);

/* x (device FP64, n0 x nrhs row-major): velocity rows of column k times s_u[k],
 * pressure rows times s_p[k] (s_u, s_p: host arrays of nrhs); with
 * dirichlet_inverse, Dirichlet rows get 1 / s_u[k] instead.  With
 * S = diag(sqrt(nu) I, I / sqrt(nu)) the free-free block of the operator with
 * viscosity nu is S K S (K the nu = 1 operator, Dirichlet rows identity in
 * both), so several viscosities can share one hierarchy: c = S^-1 b on free
 * rows and S b on Dirichlet rows (dirichlet_inverse = 1), solve K y = c, then
 * x = S^-1 y (dirichlet_inverse = 0).  Synchronises the stream. */
int mas_scale_rows(mas_handle* h, double* x, int32_t nrhs, const double* s_u, const double* s_p,
                   int32_t dirichlet_inverse, void* stream);

/* Copy level l's operator (0 = free K0, 1 = free K1, ...) to host CSR arrays
 * the caller owns and sizes: indptr nrows + 1, indices and data nnz.  Any of
 * the five output pointers may be NULL and is then skipped (first call with
 * the arrays NULL to get the sizes).  Works on analysed-only handles.
 * Errors: MAS_EINVAL for a NULL handle or a level outside [0, n_levels). */
int mas_export_level(const mas_handle* h, int32_t level, int64_t* nrows, int64_t* nnz,
                     int64_t* indptr, int32_t* indices, double* data);

/* Event timing of the cycle's kernel launches during mas_solve / mas_apply
 * (for measurement; while on, graph replay is off and both calls synchronise
 * their stream before returning).  mas_get_timing fills
 * up to n (at most 18) values, three per kernel kind k: out[3k] summed time
 * (ms), out[3k+1] launches, out[3k+2] their summed algorithmic bytes.  Kinds:
 * 0 thread-per-patch bucket kernel, 1 wavefront-per-patch kernel, 2 batched
 * (several right-hand sides) patch kernel, 3 sliced-ELL product, 4 CSR
 * product, 5 batched CSR product.  Patch-kernel
 * bytes: factor records, DoF lists, patch outputs, and each distinct level
 * vector entry read once; sparse products: values, column and row indices,
 * vectors. */
int mas_set_timing(mas_handle* h, int32_t enable);  /* resets the sums; MAS_EINVAL: NULL */
int mas_get_timing(const mas_handle* h, double* out, int32_t n);  /* MAS_EINVAL: NULL */

/* Free the handle, its device memory and its host analysis (waits for the
 * device first).  NULL is accepted and ignored. */
int mas_destroy(mas_handle* h);
const char* mas_error_string(int status);
const char* mas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MAS_H */
