/*
 * afsbem -- per-frequency Laplace-domain elastodynamic boundary-element solve
 * on AMD Instinct MI355X (gfx950), and the frequency-domain drivers on top.
 *
 * The operation (Xiao, Rong, Ye, Zhang, "An efficient adaptive frequency
 * sampling scheme for large-scale transient boundary element analysis",
 * Section 2.1, Eq. 1 and Eq. 2): for a complex frequency s, the boundary
 * integral equation
 *     c_ij u_j(x) + PV int_G T_ij(x,y;s) u_j(y) dG = int_G U_ij(x,y;s) t_j(y) dG
 * is discretised on a closed surface of flat triangles with constant u and t
 * per element, collocated at element centroids (c = 1/2 I there), giving the
 * N x N complex system A(s) a(s) = b(s), N = 3 * n_tri.  Per element either the
 * traction is prescribed (kind 0: the displacement is unknown) or the
 * displacement is prescribed (kind 1: the traction is unknown).
 * The system is solved by GMRES (Section 2.1) with a right block-diagonal
 * (block-Jacobi) preconditioner (Section 4).
 *
 * Conventions
 *  - Status codes: 0 success, < 0 error (AFSBEM_E*).  On error, outputs are left
 *    untouched and afsbem_last_error() returns a thread-local message.
 *  - Complex numbers are interleaved (re, im) doubles unless stated otherwise.
 *  - Element vectors are [n_tri][3] (x, y, z components), frequency-major for
 *    several frequencies: [n_s][n_tri][3].
 *  - Matrices on the device are column-major with leading dimension
 *    lda = N rounded up to a multiple of 64: entry (row, col) at col*lda + row.
 *  - Handles are opaque and owned by the library; free them with *_destroy.
 *    Host arrays passed in are copied; the library never frees caller memory.
 *  - *_device entry points take device pointers allocated by the caller (for
 *    instance PyTorch tensors) and a hipStream_t passed as void*; work is
 *    enqueued on that stream and results are valid once it has completed.
 *  - One problem handle must not be used from two threads at once.
 */
#ifndef AFSBEM_H
#define AFSBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    AFSBEM_OK = 0,
    AFSBEM_EINVAL = -1,     /* invalid argument (size, index, null pointer, degenerate triangle) */
    AFSBEM_ENOMEM = -2,     /* device or host allocation failed */
    AFSBEM_EDEVICE = -3,    /* HIP runtime error */
    AFSBEM_ENOCONV = -4,    /* outputs written, but the final FP64 residual exceeds the tolerance */
    AFSBEM_EBREAKDOWN = -5, /* Krylov breakdown that restarting did not cure */
    AFSBEM_ENAN = -6        /* NaN or Inf met in the residual */
};

typedef struct afsbem_mesh afsbem_mesh;
typedef struct afsbem_problem afsbem_problem;

/* Thread-local text of the last error; never NULL. */
const char *afsbem_last_error(void);
int afsbem_version(int *major, int *minor);

/* ------------------------------------------------------------------ mesh ---
 * xyz: [n_vert][3] doubles; tri: [n_tri][3] vertex indices.  The triangle
 * normal (v1-v0)x(v2-v0) must point out of the elastic domain (into cavities,
 * outward on the faces of a bounded body).  Rejects indices out of range and
 * zero-area triangles (AFSBEM_EINVAL).  Arrays are copied. */
int afsbem_mesh_create(const double *xyz, int64_t n_vert, const int32_t *tri, int64_t n_tri,
                       afsbem_mesh **out);
int afsbem_mesh_destroy(afsbem_mesh *mesh);

/* Six-node (curved quadratic) triangles, the paper's own discretisation
 * (Section 2.1): tri6 [n_tri][6] holds the corners v0 v1 v2, then the
 * mid-edge nodes of edges 01, 12, 20; the element map is the quadratic
 * interpolant of the six nodes and its normal (x_xi x x_eta) must point out of
 * the elastic domain.  A problem built on such a mesh is discretised by the
 * locally-corrected Nystrom method: the unknowns sit at the six points of the
 * 6-point Gauss rule of every element (point 6 e + q is rule point q of
 * element e, q = 0..2 the orbit (a, a, 1-2a), q = 3..5 the orbit (b, b, 1-2b),
 * the odd barycentric coordinate at position q % 3), so n_k = 6 n_tri points
 * with three unknowns each.  Far elements use the rule itself; near elements
 * locally corrected weights (recursive subdivision of the parameter triangle,
 * same far_ratio/max_subdiv test as the flat elements, applied to each piece's
 * image); the element holding the target point polar coordinates about it in
 * the parameter plane (self_n_theta x self_n_rho per half of each of the three
 * sub-triangles) with the strongly singular part as a principal value.  Every
 * per-point array of the problem (boundary values, solutions, bc_kind expanded
 * per element) then has n_k entries.  Matrix-free application is not
 * available for these problems.  Rejects indices out of range
 * (AFSBEM_EINVAL); arrays are copied. */
int afsbem_mesh_create_quadratic(const double *xyz, int64_t n_vert, const int32_t *tri6, int64_t n_tri,
                                 afsbem_mesh **out);

/* -------------------------------------------------------------- problem ---
 * Isotropic material (Section 2.1): shear modulus mu, Poisson ratio nu in
 * (-1, 0.5), density rho; c_s = sqrt(mu/rho), c_p = sqrt((lambda+2mu)/rho). */
typedef struct {
    double mu, nu, rho;
} afsbem_material;

/* Quadrature policy (the paper's Section 2.1 names regular Gauss rules,
 * recursive subdivision for nearly singular integrals and a dedicated scheme
 * for singular ones; this library uses):
 *   far_ratio   -- the 7-point degree-5 rule when |x - c_n| >= far_ratio * h_n
 *                  (h_n = longest edge), else 4-way midpoint subdivision with
 *                  the same test on every sub-triangle (default 2.0)
 *   max_subdiv  -- subdivision depth limit (default 8)
 *   self_n_theta, self_n_rho -- Gauss-Legendre orders of the polar rule on each
 *                  of the three sub-triangles of the self element (16, 16). */
typedef struct {
    double far_ratio;
    int32_t max_subdiv;
    int32_t self_n_theta, self_n_rho;
} afsbem_quad_policy;

/* bc_kind: [n_tri] (per element of the mesh), 0 = traction prescribed, 1 = displacement prescribed.
 * policy may be NULL (defaults).  Builds the s-independent quadrature plan
 * (element geometry, near-pair subdivision leaves, self-element polar tables
 * and static principal values) and uploads it to the current HIP device. */
int afsbem_problem_create(const afsbem_mesh *mesh, const afsbem_material *mat, const int8_t *bc_kind,
                          const afsbem_quad_policy *policy, afsbem_problem **out);
int afsbem_problem_destroy(afsbem_problem *p);

/* Sizes of the plan: n_tri (collocation points: elements of a flat mesh, six
 * per element of a six-node mesh; the system has 3 n_tri unknowns), number of
 * near pairs, number of subdivision leaves, number of self quadrature nodes per
 * collocation point.  Any pointer may be NULL. */
int afsbem_problem_info(const afsbem_problem *p, int64_t *n_tri, int64_t *n_near_pairs,
                        int64_t *n_leaves, int64_t *self_nodes_per_element);

/* Host copy of the collocation points (one per flat element, six per six-node
 * element): out8 [n][8] = point (3), unit normal (3), weight (the element area
 * for flat elements, w_q J_q for the Nystrom points), boundary kind.  n is the
 * n_tri of afsbem_problem_info. */
int afsbem_problem_points(const afsbem_problem *p, double *out8);

/* ------------------------------------------------ step-level entry points ---
 * Matrix storage formats on the device (N = 3 n_tri, column-major):
 *   AFSBEM_FMT_C128  -- one plane of complex<double>, N*N*16 bytes;
 *   AFSBEM_FMT_SPLIT -- two planes of complex<float>: hi = fp32(A), lo =
 *                       fp32(A - hi); hi+lo carries A to ~2^-48 relative.
 *                       N*N*8 bytes each. */
enum { AFSBEM_FMT_C128 = 0, AFSBEM_FMT_SPLIT = 1 };

/* Assembles A(s) and b(s) of Eq. 2 at one s on the device.
 * d_bc_val: [n_tri][3] complex<double>, the prescribed traction or displacement
 * at this s.  d_A (and d_A_lo for SPLIT) must hold N*lda entries; d_b N complex
 * doubles.  d_precond (nullable): [n_tri][3][3] complex<double> receives the
 * inverses of the 3x3 diagonal blocks (row-major per block). */
int afsbem_assemble_device(afsbem_problem *p, double s_re, double s_im, const void *d_bc_val,
                           int format, void *d_A, void *d_A_lo, void *d_b, void *d_precond,
                           void *hip_stream);

/* y = A x on the device.  precision 0: FP64 product (C128, or hi+lo of SPLIT);
 * precision 1: FP32 product of the hi plane with FP32 accumulation (SPLIT only).
 * x and y are N complex doubles. */
int afsbem_matvec_device(afsbem_problem *p, int format, int precision, const void *d_A,
                         const void *d_A_lo, const void *d_x, void *d_y, void *hip_stream);

/* afsbem_matvec_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, layouts and result up to the order of the FP64
 * partial sums.  The partial sums of the column split go to a fixed array of
 * 16 MiB per device inside the library, held until the process ends; no
 * hipMalloc, hipFree or allocating library routine is called.  N = 3 n_tri
 * above 1,048,576 is rejected (AFSBEM_EINVAL).  Every call on a device shares
 * that device's array: calls that overlap on one device (several streams or
 * threads) race and must be serialised by the caller. */
int afsbem_matvec_device_noalloc(afsbem_problem *p, int format, int precision, const void *d_A,
                                 const void *d_A_lo, const void *d_x, void *d_y, void *hip_stream);

/* Matrix-free product at one s (Eq. 2 without a stored matrix): the far-field
 * rule is evaluated on the fly for every pair m != n (precision 0: FP64;
 * 1: FP32 evaluation with FP64 sums over sources) and the near-pair
 * corrections and self blocks (FP64, formed here) are added.  d_x, d_y
 * (nullable together): N complex doubles, y = A(s) x.  d_b (nullable): N
 * complex doubles, b(s) from d_bc_val ([n_tri][3] complex, nullable when no b
 * is asked for).  Temporary device memory O(N + near pairs) is taken from the
 * stream-ordered allocator. */
int afsbem_matvec_free_device(afsbem_problem *p, double s_re, double s_im, int precision,
                              const void *d_bc_val, const void *d_x, void *d_y, void *d_b,
                              void *hip_stream);

/* Autotuning of launch parameters (on by default): the first product of a
 * given size and format on a device measures the candidate column splits of
 * the dense GEMV (1/4x to 4x of the default) on the live operands with HIP
 * events and keeps the fastest for the rest of the process.  enabled = 0
 * uses the defaults for sizes not yet tuned. */
/* Hierarchical form of the matrix-free operator at s (the inner operator of
 * matrix_free = 2; Section 2.1 names an accelerated product, this is the
 * low-rank one described at afsbem_solve_opts.matrix_free): builds the
 * frequency's near/self blocks, dense blocks and cross-approximation factors,
 * then y = A_H(s) x for d_x, d_y (N complex doubles, device).  max_rank,
 * n_lowrank, n_dense (nullable): the largest rank found, the numbers of
 * low-rank and dense blocks.  Returns AFSBEM_ENOCONV (y still written, from
 * the factors as found) when a block did not reach eps within 128 terms.
 * Flat-element problems only. */
/* Host-side view of the quadrature plan a problem on this mesh would use
 * (nothing is uploaded; no device needed): out4 = collocation points (the
 * n_tri of afsbem_problem_info), near pairs, subdivision leaves, preconditioner
 * clusters.  Flat or six-node meshes; policy nullable (defaults). */
int afsbem_plan_info(const afsbem_mesh *mesh, const int8_t *bc_kind, const afsbem_quad_policy *policy,
                     int64_t *out4);

/* Host-side view of the hierarchical operator's block partition for a flat
 * mesh (nothing is uploaded; no device needed): out8 = element count n, dense
 * blocks, low-rank blocks, element pairs covered by all blocks (n^2 for a
 * partition), near pairs falling in low-rank blocks (0), the largest low-rank
 * block side (elements), elements covered by the leaves (n), entries of the
 * per-leaf block lists.  policy nullable (defaults). */
int afsbem_hmat_partition_info(const afsbem_mesh *mesh, const int8_t *bc_kind, const afsbem_quad_policy *policy,
                                double eta, int64_t *out8);

int afsbem_hmat_matvec_device(afsbem_problem *p, double s_re, double s_im, double eps, double eta, const void *d_x,
                              void *d_y, int32_t *max_rank, int64_t *n_lowrank, int64_t *n_dense,
                              void *hip_stream);

int afsbem_autotune_set(int enabled);
/* Text table of the tuned choices and the measured times; len receives the
 * full length, buf (nullable, cap bytes) a NUL-terminated copy. */
int afsbem_autotune_report(char *buf, int64_t cap, int64_t *len);

/* Preconditioner clusters of the plan: n_clusters, ptr_out [n_clusters+1]
 * offsets into elem_out [n_tri] (element indices grouped by cluster); the
 * arrays are nullable (query the count first). */
int afsbem_problem_clusters(const afsbem_problem *p, int64_t *n_clusters, int64_t *ptr_out, int32_t *elem_out);

/* z = M^-1 v with M the block diagonal of A over the clusters (FP32
 * inverses built from d_A on the device, FP64 application). */
int afsbem_precond_apply_device(afsbem_problem *p, int format, const void *d_A, const void *d_A_lo,
                                const void *d_v, void *d_z, void *hip_stream);

/* ---------------------------------------------------------------- solve --- */
enum { AFSBEM_PREC_FP64 = 0, AFSBEM_PREC_MIXED = 1 };
/* Initial guesses.  PREV: the previous frequency's solution (for the first
 * frequency of a call: d_x0 when given, one [N] vector); USER: d_x0;
 * LEARNED: the warm-start network of the problem (trained on the solutions of
 * all frequencies it has solved so far, across calls) combined with the
 * previous solution; the network is skipped for 8 frequencies after three
 * gains below 1.3 over the previous solution alone, and retired for the
 * problem (no queries, no training: PREV behaviour) after three such closures
 * with no better gain in between.  EXTRAP: the linear extrapolation in s of
 * s*a from the two preceding frequencies of the call (needs d_a_out; PREV for
 * the second frequency, d_x0 for the first).  Every guess x0 is rescaled (or the pair combined) to
 * minimise ||b - A x0|| before the Krylov solve. */
/* Failure handling of afsbem_solve_device / afsbem_solve (stats.fallback):
 * a starting guess whose residual is not finite or not below ||b|| is
 * replaced by the zero start (fallback 1); mixed refinement whose outer FP64
 * residual is not finite, or fails twice in a row to drop below 0.9 of its
 * previous value, continues as FP64 GMRES from the best iterate (fallback 2).
 * The fault_inject bits force these conditions from the host (the kernels
 * run as usual): NAN_START replaces the starting guess by NaNs, STALL_INNER
 * discards every inner correction. */
enum { AFSBEM_FAULT_NAN_START = 1, AFSBEM_FAULT_STALL_INNER = 2 };
enum { AFSBEM_WARM_NONE = 0, AFSBEM_WARM_PREV = 1, AFSBEM_WARM_USER = 2, AFSBEM_WARM_LEARNED = 3,
       AFSBEM_WARM_MODEL = 4 /* afsbem_afs_run_problem only, see there */, AFSBEM_WARM_EXTRAP = 5,
       /* zero start; the caller's vector of each frequency (d_x0) augments the search space of the
          first GMRES cycle, as the network's prediction does with learn_aug = 1 */
       AFSBEM_WARM_USER_AUG = 6 };

typedef struct {
    double tol;          /* target FP64 true relative residual ||b - A x|| / ||b|| (1e-6) */
    int32_t restart;     /* GMRES restart length m (50; afsbem_solve_device and afsbem_solve take up
                            to 4000, the batched solve 500); the basis holds (m + 1) N complex
                            doubles of device memory */
    int32_t max_iter;    /* cap on matrix-vector products per frequency (1000) */
    int32_t precision;   /* AFSBEM_PREC_FP64 or AFSBEM_PREC_MIXED */
    int32_t warm_start;  /* AFSBEM_WARM_* */
    double inner_tol;    /* mixed: relative reduction asked of each FP32 inner solve; the target
                            is max(inner_tol * ||r||, tol * ||b|| / 2) (default 0: aim at tol) */
    int32_t batch;       /* afsbem_solve_device: 1 = one frequency at a time on the caller's
                            stream; 2 = two in flight, the assembly of frequency k+1 on one
                            library stream starting when frequency k's first inner solve (mixed
                            path, on another stream) is within 50x of its target, or with its
                            first FP64 residual; otherwise (default 0) two in flight, the
                            assembly of frequency k+1 overlapping the whole Krylov phase of
                            frequency k.  afsbem_solve_batched_device: >= 1 caps the systems of
                            a wave (default 0: memory-bound, at most 64) */
    uint32_t fault_inject; /* test hooks (AFSBEM_FAULT_* bits), 0 in production */
    int32_t profile;     /* 1: time every matrix-vector kernel with HIP events (stats.gemv_*) */
    int32_t learn_steps; /* AFSBEM_WARM_LEARNED: Adam steps after each solved frequency (0: 24) */
    int32_t precond;     /* block-diagonal preconditioner: 0 = one 3x3 block per collocation point;
                            1 = blocks over spatial clusters of up to 49 elements (recursive
                            coordinate bisection), inverted in FP32 on the device (with
                            matrix_free: the blocks are evaluated, far rule + near/self blocks) */
    int32_t matrix_free; /* 1: no stored matrix; every product evaluates the far-field rule on the
                            fly (FP64, or FP32 for the inner products of the mixed path) and adds
                            the near/self blocks formed once per frequency in FP64; memory
                            O(N + near pairs) instead of O(N^2).
                            2: as 1, but the inner products of the mixed path use a hierarchical
                            form of the same operator built once per frequency (a fast far field
                            in place of the accelerated product the paper takes, Section 2.1):
                            admissible cluster pairs as low-rank factors from adaptive cross
                            approximation to hmat_eps, the rest as dense blocks; the FP64 outer
                            residual stays the on-the-fly operator.  Needs precision = MIXED;
                            an admissible block that does not reach hmat_eps within 128 terms
                            leaves that frequency on the on-the-fly inner operator. */
    int32_t no_graph;    /* batched solve: 1 = launch every kernel directly instead of replaying
                            the captured graphs of four Arnoldi steps (default 0) */
    double hmat_eps;     /* matrix_free = 2: relative accuracy of each low-rank block (0: 1e-5) */
    double hmat_eta;     /* matrix_free = 2: admissibility, separation >= hmat_eta x the larger
                            cluster radius (0: 1.0) */
    int32_t learn_aug;   /* AFSBEM_WARM_LEARNED: role of the network's prediction.  0: it enters
                            the starting iterate (residual-minimising combination with the
                            previous solution); 1: it augments the search space of the first
                            GMRES cycle instead (its image is projected out of the Arnoldi
                            vectors and its coefficient found by the same least-squares problem;
                            the start is the previous solution; a vector whose projection
                            lowers the residual by less than 5 % is declined after its product);
                            2: both */
    int32_t no_recycle;  /* mixed path: 0 (default) = the correction of every refinement step after
                            the first is sought in the first inner solve's Krylov subspace (same
                            FP32 operator) augmented by new Arnoldi vectors of the part of the
                            residual outside it; 1 = each inner solve builds a fresh Krylov space */
} afsbem_solve_opts;

typedef struct {
    int32_t iters;        /* matrix-vector products in the Krylov solver */
    int32_t refine_steps; /* FP64 residual evaluations (mixed) */
    int32_t fallback;     /* 0 none; 1 warm start rejected; 2 mixed fell back to FP64 */
    int32_t status;       /* per-frequency status code */
    double rel_res_fp64;  /* final ||b - A x|| / ||b|| with the FP64 operator */
    double t_assemble_ms, t_solve_ms;
    double bytes;         /* algorithmic matrix bytes streamed */
    /* with opts.profile: device time of the GEMV kernels (partial-sum pass
     * excluded) of the Krylov operator (FP32 hi plane in the mixed path, FP64 in
     * the plain path) and of the FP64 residual operator of the mixed path */
    double gemv_ms, gemv64_ms;
    int32_t gemv_count, gemv64_count;
    double rel_res_start; /* ||b - A x0|| / ||b|| of the starting iterate (1 from zero) */
    int32_t used_net;     /* 1 if the warm-start network's prediction entered x0 */
    int32_t pad_;
    double t_far_ms;      /* with opts.profile: device time of the far-field kernel of the
                             assembly (stored operators), else 0 */
} afsbem_solve_stats;

/* Fills opts with the defaults listed above. */
int afsbem_solve_opts_default(afsbem_solve_opts *opts);

/* Solves A(s_k) a_k = b_k for n_s frequencies s (host array, 2*n_s doubles).
 * d_bc_val: [n_s][n_tri][3] complex<double> prescribed values at each s.
 * d_x0: nullable [n_s][N] complex<double> initial guesses (used with
 *       AFSBEM_WARM_USER; with PREV or LEARNED its first N entries stand for
 *       the solution preceding the first frequency).  With PREV or LEARNED the
 *       start of frequency k > 0 is the solution of the nearest frequency
 *       (in |s - s_k|) among those before it in the call: the previous one
 *       for an ordered list; EXTRAP uses the two previous ones.
 * Outputs (each nullable): d_a_out [n_s][N] solution vector, d_u_out and
 * d_t_out [n_s][n_tri][3] displacement and traction per element.
 * stats: nullable host array of n_s entries.
 * Returns AFSBEM_ENOCONV if any frequency missed the tolerance (outputs are
 * still written with the best iterate). */
int afsbem_solve_device(afsbem_problem *p, int32_t n_s, const double *s, const void *d_bc_val,
                        const void *d_x0, void *d_a_out, void *d_u_out, void *d_t_out,
                        const afsbem_solve_opts *opts, afsbem_solve_stats *stats, void *hip_stream);

/* Host-pointer variant of afsbem_solve_device: s, bc_val [n_s][n_tri][3],
 * x0 (nullable), a_out [n_s][N], u_out and t_out [n_s][n_tri][3] (each
 * nullable) are host arrays owned by the caller; the library copies them to
 * and from device buffers of its own (freed before return) and works on the
 * null stream.  Same options, statistics and return codes. */
int afsbem_solve(afsbem_problem *p, int32_t n_s, const double *s, const double *bc_val, const double *x0,
                 double *a_out, double *u_out, double *t_out, const afsbem_solve_opts *opts,
                 afsbem_solve_stats *stats);

/* Batched solve of many independent systems: every frequency of every problem
 * in the call (several meshes of uneven size allowed, all on the current
 * device).  The per-frequency operation is the one of afsbem_solve_device
 * (collocation system of Sec. 2 at each Laplace parameter); here the systems
 * advance in lockstep, one kernel launch per Krylov step serving all of them,
 * which keeps the device full when single systems are small.
 *   probs[p], n_s[p]: problem handles and their frequency counts.
 *   s: host array, 2 * sum(n_s) doubles, the frequencies of problem 0, then
 *      of problem 1, ...
 *   d_bc_val[p]: [n_s[p]][n_tri_p][3] complex<double> device array.
 *   d_a_out[p], d_u_out[p], d_t_out[p]: nullable device outputs, layouts as
 *      in afsbem_solve_device; the pointer arrays themselves may be null.
 *   stats: nullable host array of sum(n_s) entries, same order as s.
 * Options: tol, restart, max_iter, precision (FP64, or MIXED: FP32 hi-plane
 * inner cycles with FP64 residuals), precond (0 or 1 as in
 * afsbem_solve_device), no_graph.  Systems are solved in waves that fit a
 * slot of min(30 % of free device memory, 16 GiB) (at least one system, at
 * most 64, or opts.batch if >= 1); two slots alternate so that the next wave
 * is assembled while the current one is solved.  The device memory and
 * streams are kept by probs[0] for later calls (freed with it).  Warm starts
 * and the matrix-free operator are not available here (AFSBEM_EINVAL).  Work
 * is ordered after hip_stream's prior work and the call returns after the
 * outputs are written.  Returns AFSBEM_ENOCONV if any system missed the
 * tolerance. */
int afsbem_solve_batched_device(int32_t n_prob, afsbem_problem *const *probs, const int32_t *n_s,
                                const double *s, const void *const *d_bc_val, void *const *d_a_out,
                                void *const *d_u_out, void *const *d_t_out, const afsbem_solve_opts *opts,
                                afsbem_solve_stats *stats, void *hip_stream);


/* ======================================================= learned warm start
 * A multilayer perceptron (not part of the paper) that maps per-element
 * features at a frequency to the element's solution components; it is
 * trained on solutions of earlier frequencies and supplies initial guesses.
 *   Z1 = X W1 + b1, H1 = silu(Z1), Z2 = H1 W2 + b2, H2 = silu(Z2), Y = H2 W3 + b3
 * Flat FP32 parameters: W1 [d_in][hidden] row-major, b1 [hidden],
 * W2 [hidden][hidden], b2 [hidden], W3 [hidden][d_out], b3 [d_out].
 * X [n][d_in], Y and T [n][d_out] row-major FP32 device arrays.
 * mode 1: bfloat16 matrix-core products with FP32 accumulation (production);
 * mode 0: FP32 fused multiply-adds (reference arithmetic). */
int afsbem_mlp_n_params(int32_t d_in, int32_t hidden, int32_t d_out, int64_t *n);
int afsbem_mlp_forward(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, const float *d_params,
                       const float *d_X, float *d_Y, int mode, void *hip_stream);
/* d_grad [n_params] receives the gradient of mean((Y - T)^2); d_loss
 * (nullable) one float, the loss. */
int afsbem_mlp_loss_grad(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, const float *d_params,
                         const float *d_X, const float *d_T, float *d_grad, float *d_loss, int mode,
                         void *hip_stream);
/* One Adam step (step counter t >= 1) in place on d_params with moments d_m, d_v. */
int afsbem_mlp_adam(int64_t n_params, float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t t,
                    float lr, float beta1, float beta2, float eps, void *hip_stream);
/* One training step on the matrix cores (mode 1 arithmetic): loss and
 * gradient of mean((Y - T)^2) over the n rows of d_X / d_T, then the Adam step
 * t (>= 1) in place on d_params with moments d_m, d_v; the gradient planes of
 * the batch split are added and applied in one pass (the full gradient is not
 * stored).  d_loss (nullable): one float, the loss before the step.  Work
 * memory comes from the stream-ordered allocator. */
int afsbem_mlp_train_step(int32_t d_in, int32_t hidden, int32_t d_out, int32_t n, float *d_params,
                          const float *d_X, const float *d_T, float *d_m, float *d_v, int32_t t, float lr,
                          float beta1, float beta2, float eps, float *d_loss, void *hip_stream);

/* ===================================================================== drivers
 * Host-side frequency-domain drivers on top of the solve.  Complex arrays are
 * interleaved (re, im) doubles; all arrays are caller-owned host memory. */

/* Fourier-series method (Section 2.2, Eq. 3-4): s_k = eta + i 2 pi k / P,
 * k = 0..Ns/2 (Ns even); s_out holds Ns/2 + 1 complex values. */
int afsbem_fsm_grid(double P, double eta, int32_t Ns, double *s_out);

/* Inverse Laplace transform by the trapezoidal rule on the Bromwich line
 * evaluated with an FFT:  h(t_n) = (e^{eta t_n} / P) Re sum_{k=0}^{Ns-1} W_k H_k
 * e^{2 pi i k n / Ns},  t_n = n P / Ns, with H_{Ns-k} = conj(H_k) and the
 * Nyquist term at half weight (trapezoid end points).  H: [n_sig][Ns/2+1]
 * complex samples at afsbem_fsm_grid; window 0 = none, 1 = Hann
 * W_k = (1 + cos(2 pi k / Ns)) / 2.  h_out: [n_sig][Ns] real.  The factor
 * 1/P that Eq. 4 omits is included. */
int afsbem_fsm_invert(double P, double eta, int32_t Ns, int window, int64_t n_sig, const double *H,
                      double *h_out);

/* Vector fitting with common poles (Section 2.3, Eq. 5): f_k(s) = sum_m r_km /
 * (s - a_m), strictly proper, real-coefficient structure (conjugate pairs).
 * s: [J] complex samples, F: [K][J] complex data, M poles.  init_poles
 * (nullable, [M] complex): default pairs -b/100 +- i b, b equally spaced in
 * (0, omega_max] (omega_max <= 0: the largest Im s), plus one real pole for odd M.
 * n_iter pole-identification passes (stops early when the poles settle);
 * unstable poles are kept.  Outputs: poles_out [M], residues_out [K][M]
 * complex, rms_out (nullable) the root-mean-square misfit on the samples. */
int afsbem_vf_fit(int32_t J, const double *s, int32_t K, const double *F, int32_t M,
                  const double *init_poles, int32_t n_iter, double omega_max, double *poles_out,
                  double *residues_out, double *rms_out);
/* Residue identification for n_fun functions with fixed poles (conjugate
 * pairs must be complete); residues_out [n_fun][M] in the given pole order. */
int afsbem_vf_residues(int32_t J, const double *s, int64_t n_fun, const double *F, int32_t M,
                       const double *poles, double *residues_out);
/* f_out [n_fun][n_s] complex: the model at the points s. */
int afsbem_vf_eval(int32_t M, const double *poles, int64_t n_fun, const double *residues, int32_t n_s,
                   const double *s, double *f_out);
/* f_out [n_fun][n_t] real: the time response sum_m r_km e^{a_m t} (the exact
 * inverse transform of the model; Eq. 6 prints the exponent's sign the other
 * way, which would contradict Eq. 5). */
int afsbem_vf_eval_time(int32_t M, const double *poles, int64_t n_fun, const double *residues, int32_t n_t,
                        const double *t, double *f_out);

/* Adaptive frequency sampling (Section 3, Eq. 7-14, the Algorithm of 3.4).
 * T: period, eta: abscissa, Ns: FSM resolution (Omega = pi Ns / T), J0 initial
 * Chebyshev-type frequencies w_j = Omega [1 - cos(j pi / (2 (J0-1)))] (the
 * printed formula lacks the pi), fitting orders floor(J/alpha_H), floor(J/alpha_L),
 * thresholds E1_bar, E2_bar, Jc validation steps, max_Nc cap (0 = Ns/2 + 1),
 * grid_pts points of the uniform grid on which maxima over [0, Omega] are
 * taken, n_iter pole-identification passes per fit.  q (default 1, the
 * paper's rule) new frequencies per analysis step, requested from the response
 * in one call (one batched solve): the largest discrepancy as in Section 3.2,
 * then the next largest local maxima of the same discrepancy at least dw/4
 * from every sample and every earlier pick (fewer when none is left); the Jc
 * validation steps add one frequency each, as in the paper. */
typedef struct {
    double T, eta;
    int32_t Ns, J0;
    double alpha_H, alpha_L, E1_bar, E2_bar;
    int32_t Jc, max_Nc, grid_pts, n_iter;
    int32_t q;
} afsbem_afs_params;

typedef struct afsbem_afs_result afsbem_afs_result;

/* Response callback: fills f_out [n_s][Kt] complex with the responses at the
 * n_s complex frequencies s; columns 0..K-1 are the observation response
 * functions used for pole identification, K..Kt-1 further test functions.
 * Returns 0 on success. */
typedef int (*afsbem_response_fn)(int32_t n_s, const double *s, int32_t Kt, double *f_out, void *user);

/* All-DOF time synthesis: the time responses (Eq. 6) of every unknown from
 * its samples, with the common poles of a vector-fitting model.  For each n
 * the residues with these poles are identified by least squares from the
 * samples X[j][n] at s_j (as in Section 2.3, real-coefficient basis), and
 * h[n][k] = sum_m r_nm e^{a_m t_k} (real part).  Computed as one FP64
 * matrix-core contraction over 2 J terms per output.
 * poles [M], s [J] (complex, host); d_X [J][N] complex<double> (device);
 * t [Nt] (host); d_h [N][Nt] double (device, written); d_X 16-byte and d_h
 * 8-byte aligned.  Needs the number of real basis functions (M, counting a
 * conjugate pair as two) <= 2 J.  Synchronises the stream; AFSBEM_EINVAL on
 * bad sizes, null pointers, alignment or too many poles. */
int afsbem_time_synthesis_device(int32_t M, const double *poles, int32_t J, const double *s, int64_t N,
                                 const void *d_X, int32_t Nt, const double *t, void *d_h, void *hip_stream);

/* The same per-unknown models (residues identified from the samples X[j][n]
 * at s_j with the common poles, Section 2.3) evaluated at n_z complex
 * frequencies z (Eq. 5): H[n][k] = sum_m r_nm / (z_k - a_m).  The same FP64
 * matrix-core contraction, with the basis functions' values at z_k in place of
 * their time responses.  poles [M], s [J], z [n_z] (complex, host); d_X [J][N]
 * complex<double> (device, 16-byte aligned); d_H [N][n_z] complex<double>
 * (device, written); n_z <= 2^24.  Synchronises the stream; AFSBEM_EINVAL on
 * bad sizes, null pointers, alignment or too many poles.  With z = the FSM grid this
 * feeds afsbem_fsm_invert_device (the model's Fourier-series inversion for
 * every unknown). */
int afsbem_model_sample_device(int32_t M, const double *poles, int32_t J, const double *s, int64_t N,
                               const void *d_X, int32_t n_z, const double *z, void *d_H, void *hip_stream);

/* Fourier-series inversion (Section 2.2, Eq. 4 with its 1/P factor) of n_sig
 * signals at once on the GPU; the definition of afsbem_fsm_invert (trapezoid
 * end points at +-Omega with half weight, optional Hann window), computed by a
 * batched FFT.  d_H [n_sig][Ns/2+1] complex<double> (device, 16-byte aligned):
 * the samples at s_k = eta + 2 pi i k / P; d_h [n_sig][Ns] double (device,
 * written): h(t_n), t_n = n P / Ns.  Ns a power of two in [2, 4096].
 * Synchronises the stream; AFSBEM_EINVAL on bad sizes, null pointers or
 * alignment. */
int afsbem_fsm_invert_device(double P, double eta, int32_t Ns, int window, int64_t n_sig, const void *d_H,
                             void *d_h, void *hip_stream);

/* Defaults: alpha_H 2.0, alpha_L 2.3, E1_bar 1e-4, E2_bar 2e-3, Jc 3, J0 16
 * (Section 3.4), grid_pts 2048, n_iter 10, max_Nc 0; T, eta, Ns placeholders. */
int afsbem_afs_params_default(afsbem_afs_params *p);
/* Runs AFS with any response (a mock, or afsbem_afs_run_problem's BEM solve). */
int afsbem_afs_run(const afsbem_afs_params *p, int32_t K, int32_t Kt, afsbem_response_fn fn, void *user,
                   afsbem_afs_result **out);
/* AFS driving the GPU solve of a problem: at each requested s the boundary
 * values are bc_shape * load(s) (load_kind 0: Heaviside, load = 1/s; 1:
 * constant 1), bc_shape [n_tri][3] real; the Kt responses are the solution-vector
 * entries dof_idx[0..Kt-1] (the first K are the observation functions).  The
 * initial frequencies are solved in one call (assembly overlapped with the
 * Krylov phases).  Initial guess of each new frequency by opts->warm_start:
 * NONE zero; PREV, USER the solution at the nearest sampled frequency;
 * LEARNED the warm-start network's prediction (trained after every solve of
 * the run) combined with that nearest solution; MODEL the prediction of the current order-M_H vector-fitting
 * model (Section 3) for every unknown -- the residues of each unknown with the
 * model's poles, identified from all solved samples by least squares as in
 * Section 2.3, evaluated at the new s -- (nearest sample while there is no
 * model with fewer poles than samples).  Every guess is rescaled to minimise
 * the residual.  opts may be NULL (zero start). */
int afsbem_afs_run_problem(afsbem_problem *p, const afsbem_afs_params *params, const double *bc_shape,
                           int load_kind, const int64_t *dof_idx, int32_t K, int32_t Kt,
                           const afsbem_solve_opts *opts, afsbem_afs_result **out);
int afsbem_afs_result_info(const afsbem_afs_result *r, int32_t *Nc, int32_t *M, int32_t *n_steps,
                           int32_t *converged);
/* afsbem_afs_run_problem: total Krylov products of all its solves (0 for afsbem_afs_run). */
int afsbem_afs_result_work(const afsbem_afs_result *r, int64_t *matvecs);
/* How the run ended (each pointer nullable).  capped: 1 if the sample cap
 * max_Nc ended it, also when it cut the Jc validation steps of Eq. 14 short
 * (converged is then 0: convergence needs all Jc steps to pass).
 * unconverged_solves (afsbem_afs_run_problem): samples whose solve missed
 * opts.tol; their best iterate was still sampled, and converged is 0 when any
 * did.  worst_rel_res: the largest FP64 true relative residual of those solves
 * (0 for afsbem_afs_run). */
int afsbem_afs_result_status(const afsbem_afs_result *r, int32_t *capped, int32_t *unconverged_solves,
                             double *worst_rel_res);
/* Copies (each pointer nullable): s_out [Nc] complex samples in the order
 * taken, F_out [Nc][Kt] complex responses, poles_out [M] and residues_out
 * [Kt][M] of the final order-M_H model, E1_out and E2_out [n_steps]. */
int afsbem_afs_result_get(const afsbem_afs_result *r, double *s_out, double *F_out, double *poles_out,
                          double *residues_out, double *E1_out, double *E2_out);
int afsbem_afs_result_destroy(afsbem_afs_result *r);

#ifdef __cplusplus
}
#endif
#endif /* AFSBEM_H */
