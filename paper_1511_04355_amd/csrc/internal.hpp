// Internal declarations of the afsbem library (not part of the public ABI).
#pragma once

#include <complex>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/afsbem.h"

namespace afsbem {

// ------------------------------------------------------------------ errors --
void set_error(const std::string &msg);

struct Error {
    int code;
    std::string msg;
};

#define AFS_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::afsbem::Error{AFSBEM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define AFS_REQUIRE(cond, code, msg)                                                            \
    do {                                                                                       \
        if (!(cond))                                                                           \
            throw ::afsbem::Error{(code), (msg)};                                              \
    } while (0)

// -------------------------------------------------------------- materials --
struct MaterialDerived {
    double mu, nu, rho, lam;
    double cs, cp, beta;       // beta = cs / cp
    double lam_over_mu;
};
MaterialDerived derive_material(const afsbem_material &m);

// ------------------------------------------------------------------ plan --
// Per-element source record read with wave-uniform (scalar) loads by the far
// field kernel: 7 quadrature nodes (x, y, z, weight*area), unit normal, kind.
constexpr int kFarNodes = 7;
constexpr int kClusterElems = 49;                  // elements per preconditioner cluster (at most)
constexpr int kClusterDim = 3 * kClusterElems;      // unknowns per cluster block (at most)
constexpr int kLeafElems = 32;                     // elements per leaf of the hierarchical operator (at most)
constexpr int kSrcStride = 32;  // doubles per element record

struct HostPlan {
    int64_t n_tri = 0;
    // element geometry
    std::vector<double> vtx;       // [n][9] vertex coordinates p0, p1, p2
    std::vector<double> cen;       // [n][3] centroid (collocation point)
    std::vector<double> nrm;       // [n][3]
    std::vector<double> area;      // [n]
    std::vector<double> hmax;      // [n] longest edge
    std::vector<double> src;       // [n][kSrcStride]
    std::vector<int8_t> kind;      // [n]
    // near pairs, CSR by collocation row element
    std::vector<int64_t> near_ptr; // [n+1]
    std::vector<int32_t> near_col; // [nnz] source element
    std::vector<int32_t> near_row; // [nnz] collocation element
    std::vector<int64_t> leaf_ptr; // [nnz+1]
    std::vector<double> leaves;    // [n_leaves][10]: p0(3), e1(3), e2(3), area
    std::vector<int32_t> near_order; // [nnz] pairs by decreasing leaf count (work order of the near kernel)
    // self element polar tables
    int n_theta = 16, n_rho = 16;
    std::vector<double> self_ang;  // [n][3*n_theta][5]: e(3), R, w_theta
    std::vector<double> self_cpv;  // [n][9] principal value of the static 1/r^2 part (real)
    std::vector<double> gl_rho;    // [n_rho][2]: node in [0,1], weight on [0,1]
    std::vector<double> coef;      // [16][4]: a_n, b_n, (n-1) a_n, (n-1) b_n
    // preconditioner clusters (recursive coordinate bisection of the centroids)
    std::vector<int64_t> clus_ptr; // [n_clusters+1]
    std::vector<int32_t> clus_elem;// [n] elements grouped by cluster
    // Nystrom discretisation of six-node elements (disc = 1).  Every field
    // above then describes the n_tri = 6 n_el unknown-carrying points (node
    // 6 e + q at rule point q of element e): cen/nrm the points and normals,
    // src one record per point (y, w J, normal, kind), the near CSR pairs
    // (target point, source element) with leaves = parameter-plane triangles.
    int disc = 0;
    int64_t n_el = 0;
    std::vector<double> nys_geom;  // [n_el][18] the six nodes of each element
    std::vector<double> nys_leaves;// [n_leaves][6] (xi, eta) of three corners
    std::vector<double> nys_self;  // [6][6 * n_theta][4] cos, sin, w_theta, R per angle
    double nys_pt[12];             // rule points (xi, eta)
    double nys_lag[36];            // Lagrange basis: L_b = sum_k lag[6b+k] m_k(xi, eta)
};

// six-node elements: xyz [nv][3], tri6 [n_el][6] (corners, then mid-edge
// nodes of edges 01, 12, 20), kind per element
void build_plan_nystrom(const double *xyz, int64_t nv, const int32_t *tri6, int64_t n_el, const int8_t *kind,
                        const afsbem_quad_policy &pol, const MaterialDerived &mat, HostPlan &out);
void plan_clusters(HostPlan &P);
void plan_series(const MaterialDerived &mat, HostPlan &P);

void build_plan(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, const int8_t *kind,
                const afsbem_quad_policy &pol, const MaterialDerived &mat, HostPlan &out);

// Gauss-Legendre rule on [-1, 1] (Newton iteration on Legendre polynomials).
void gauss_legendre(int n, double *x, double *w);

struct DevicePlan {
    int64_t n_tri = 0, nnz = 0, n_leaves = 0;
    int n_theta = 16, n_rho = 16;
    double *colx = nullptr, *coly = nullptr, *colz = nullptr; // collocation points SoA
    double *src = nullptr;
    int8_t *kind = nullptr;
    int64_t *near_ptr = nullptr;
    int32_t *near_col = nullptr, *near_row = nullptr, *near_order = nullptr;
    int64_t *leaf_ptr = nullptr;
    double *leaves = nullptr;
    double *self_ang = nullptr, *self_cpv = nullptr, *gl_rho = nullptr;
    double *nrm = nullptr;         // [n][3]
    double *coef = nullptr;        // [16][4] series coefficients of the radial functions
    double *col64 = nullptr;       // [n][4] collocation points (x, y, z, 0)
    float *col32 = nullptr, *src32 = nullptr, *coef32 = nullptr;  // FP32 copies for on-the-fly evaluation
    int64_t n_clusters = 0;
    int64_t *clus_ptr = nullptr;
    int32_t *clus_elem = nullptr;
    int disc = 0;                  // 1: Nystrom points of six-node elements
    int64_t n_el = 0;
    double *nys_geom = nullptr, *nys_leaves = nullptr, *nys_self = nullptr;
    double *nys_tab = nullptr;     // [48]: rule points (12), then the Lagrange basis (36)
};

// -------------------------------------------------------------- problem --
struct Workspace;
struct LearnState;
struct BatchArena;
struct HmatPlan;

struct Problem {
    MaterialDerived mat;
    afsbem_quad_policy pol;
    HostPlan host;
    DevicePlan dev;
    int device = 0;
    Workspace *ws = nullptr, *ws2 = nullptr;      // second workspace: two frequencies in flight
    hipStream_t st_asm = nullptr, st_sol = nullptr;  // library streams (default priority)
    LearnState *learn = nullptr;                     // warm-start network (created on first use)
    BatchArena *barena = nullptr;                    // batched-solve memory (created on first use)
    HmatPlan *hmat = nullptr;                        // hierarchical far field (created on first use)
    double hm_need = 0.0;                            // factor entries the largest build so far took
};

// ----------------------------------------------------- kernel launchers --
struct KernelParams {
    double s_re, s_im;
    double inv_cs;        // 1 / c_s
    double beta;          // c_s / c_p
    double c_u;           // 1 / (4 pi mu)
    double lam_over_mu;
    double inv_ks2;       // c_s^2 / |s|^2: 1/|x|^2 = inv_ks2 / r^2 (0 at s = 0)
};
KernelParams kernel_params(const MaterialDerived &m, double s_re, double s_im);

// Assembly scratch sizes for a problem: b partial sums of the far field
// ([n_chunks][N] complex), per-self b ([n][3]), per-near-pair b corrections.
int far_source_chunks(int64_t n_tri);
size_t assembly_scratch_bytes(const Problem &p);

// Launch the whole assembly: far field, near pairs, self elements, b and the
// block-Jacobi inverses.  format: AFSBEM_FMT_*.
void launch_assembly(const Problem &p, const KernelParams &kp, const double *bc_val, int format,
                     void *A, void *A_lo, double *b, double *precond, void *scratch,
                     hipStream_t st, hipEvent_t far_begin = nullptr, hipEvent_t far_end = nullptr);

// Nystrom assembly (disc = 1): near-pair and self-element kernels; the far
// field runs through the collocation far kernel with one node per source.
void launch_nystrom_near_self(const Problem &p, const KernelParams &kp, const double *bc_val, int format, void *A,
                              void *A_lo, double *bself, double *corr, double *precond, hipStream_t st);

// Matrix-free operator (no stored dense matrix).  Per frequency: the near-pair
// correction blocks (exact minus the far rule) [nnz][9] and the self blocks
// [nt][9] (complex, row-major 3x3), b's near/self parts in scratch, and the
// block-Jacobi inverses; per application the far rule is evaluated on the fly.
constexpr int kFmtBlocks = 2;
void launch_block_setup(const Problem &p, const KernelParams &kp, const double *bc_val, double *nearblk,
                        double *selfblk, double *precond, void *scratch, hipStream_t st);
// b = sum of S far partials [S][N] (bpart) + the near/self parts held in scratch
void launch_finalize_b(const Problem &p, int S, const double *bpart, const void *scratch, double *b,
                       hipStream_t st);
// source chunks of the on-the-fly far field and its partial-sum scratch
int mf_chunks(int64_t n_tri);
// y = A x (comp = 0) or the right-hand-side operator applied to the boundary
// values (comp = 1, y = b's far part; use launch_finalize_b for b).
// precision 0: FP64 evaluation, 1: FP32 evaluation (FP64 sums over sources).
void mf_apply(const Problem &p, const KernelParams &kp, int precision, int comp, const double *nearblk,
              const double *selfblk, const double *x, double *y, double *partial, hipStream_t st);

// y = A x.  precision 0: FP64, 1: FP32 hi plane.  partial: scratch of
// gemv_chunks(N) * N complex doubles.
int gemv_chunks(int64_t N);
void launch_gemv(int64_t N, int format, int precision, const void *A, const void *A_lo,
                 const double *x, double *y, double *partial, hipStream_t st,
                 hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
// The same product with its partial sums in a fixed per-device array of the
// library (no allocation; default column split, reduced to fit); N above
// gemv_noalloc_max_n() is rejected.
int64_t gemv_noalloc_max_n();
void launch_gemv_noalloc(int64_t N, int format, int precision, const void *A, const void *A_lo,
                         const double *x, double *y, hipStream_t st);

// starting guesses of a multi-frequency call (solver.cpp)
bool extrap_coeffs(std::complex<double> s0, std::complex<double> s1, std::complex<double> s2,
                   std::complex<double> &c1, std::complex<double> &c2);
const double *start_guess(const afsbem_solve_opts &o, int32_t k, int64_t N, const double *s, const double *x0_user,
                          const double *a_out, double *xbuf, hipStream_t st);

// ------------------------------------------------------ vector kernels --
// All vectors are complex<double> interleaved, length N (complex entries).
void vec_precond(int64_t n_tri, const double *Dinv, const double *v, double *z, hipStream_t st);
void vec_sub(int64_t N, const double *a, const double *b, double *out, hipStream_t st);   // out = a - b
// out = alpha x + beta y (complex scalars passed by value; out may alias)
void vec_axpby(int64_t N, double ar, double ai, const double *x, double br, double bi, const double *y, double *out,
               hipStream_t st);
// Multi-dot: out[i] = sum_r conj(V_i[r]) w[r], i < nv (two launches per
// kMdotMaxVectors vectors); V rows strided by ldv.  partial: mdot_scratch_bytes(N, nv_max) bytes
// (a reserved head of kMdotCounterBytes, then the per-block partial sums).
constexpr int kMdotMaxVectors = 512;
constexpr int kMdotMaxBlocks = 1024;
constexpr int kMdotCounterBytes = kMdotMaxVectors * 4;
size_t mdot_scratch_bytes(int64_t N, int nv_max);
void vec_mdot(int64_t N, int nv, const double *V, int64_t ldv, const double *w, double *partial,
              double *out, hipStream_t st);
// w -= sum_i h[i] V_i
void vec_mupdate(int64_t N, int nv, const double *V, int64_t ldv, const double *h, double *w,
                 hipStream_t st);
// out = x / norm (norm read from device scalar nrm2 = ||x||^2)
void vec_normalize(int64_t N, const double *nrm2, const double *x, double *out, hipStream_t st);
// out += a x + b conj(x)  (complex a, b)
void vec_axpy_conj(int64_t N, double ar, double ai, double br, double bi, const double *x, double *out,
                   hipStream_t st);
// x += sum_i y[i] V_i  (y on device, complex)
void vec_combine(int64_t N, int nv, const double *V, int64_t ldv, const double *y, double *x,
                 hipStream_t st);
// h[n][t] = sum_i B[n][i] Km[i][t] with B[n][i] = Re X[i][n] (i < J), Im X[i-J][n];
// X [J][N] complex, Km [Kpad][Nt] (Kpad = 2J rounded up to 4, zero rows), h [N][Nt]
constexpr int kFsmMaxLog2 = 12;
void launch_fsm(int log2_ns, int64_t n_sig, int window, const double *H, const double *W, const double *E, double *h,
                hipStream_t st);
void launch_synthesis(int64_t N, int J, int Kpad, int Nt, const double *X, const double *Km, double *h,
                      hipStream_t st);
// scatter solution a into u, t by element kind
void vec_split_ut(int64_t n_tri, const int8_t *kind, const double *a, const double *bc, double *u,
                  double *t, hipStream_t st);
int mdot_blocks(int64_t N);

// cluster block-Jacobi preconditioner: inverses [n_clusters][kClusterDim^2]
// complex<float>; z = M^-1 v
// format kFmtBlocks: A holds the blocks gathered by cluster_gather_mf
void cluster_inverse(const DevicePlan &d, int format, const void *A, const void *A_lo, float *inv, hipStream_t st);
// the cluster blocks of the matrix-free operator (self, far rule + near corrections)
void cluster_gather_mf(const Problem &p, const KernelParams &kp, const double *nearblk, const double *selfblk,
                       float *out, hipStream_t st);
void cluster_apply(const DevicePlan &d, const float *inv, const double *v, double *z, hipStream_t st);

}  // namespace afsbem
