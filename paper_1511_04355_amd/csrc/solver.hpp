// Solver internals: device workspace, operator, GMRES.
#pragma once
#include <complex>
#include <functional>
#include <vector>

#include "internal.hpp"
#include "hmat.hpp"

namespace afsbem {

struct Workspace {
    int64_t N = 0;
    int format = -1;
    int m = 0;
    void *A = nullptr, *A_lo = nullptr;
    double *nearblk = nullptr, *selfblk = nullptr;  // matrix-free format: per-frequency blocks
    double *b = nullptr, *precond = nullptr;
    void *asm_scratch = nullptr;
    double *gemv_partial = nullptr;
    double *V = nullptr, *w = nullptr, *z = nullptr, *x = nullptr, *r = nullptr, *tmp = nullptr;
    double *rin = nullptr, *xo = nullptr;  // mixed: outer residual and outer iterate
    double *xstart = nullptr;              // extrapolated starting guess
    double *aug = nullptr;                 // augmentation vector of the first GMRES cycle (learned)
    // Krylov subspace kept from the last cycle of a mixed solve's first inner
    // GMRES, for the corrections of its later refinement steps (same FP32
    // operator): Krylov vectors 0..rc_k of V, the cycle's triangular factor
    // (columns packed as the Hessenberg) and its Givens rotations
    bool rc_valid = false;
    int rc_k = 0;
    std::vector<std::complex<double>> rc_R, rc_cs, rc_sn;
    double *dots_partial = nullptr, *small = nullptr;
    double *one = nullptr;                 // device complex 1 + 0i
    // preconditioner: 0 = 3x3 blocks (precond), 1 = element clusters (clinv)
    int prec_kind = 0;
    float *clinv = nullptr;
    float *clgath = nullptr;  // matrix-free: the gathered cluster blocks before inversion
    const DevicePlan *plan = nullptr;
    void apply_precond(const double *v, double *z, hipStream_t st) const;
    double *host_small = nullptr;          // pinned
    // GEMV timing (opts.profile): event pairs recorded around each product
    std::vector<hipEvent_t> ev;            // 2 per slot
    std::vector<int> ev_prec;              // precision of the product in each used slot
    int ev_used = 0;
    hipEvent_t ev_far[2] = {nullptr, nullptr};  // around the far-field kernel (opts.profile)
    bool far_timed = false;
    // hierarchical far field of the matrix-free operator (solve option matrix_free = 2):
    // settings, then the frequency's dense blocks, factors, ranks and product scratch
    int hm_enabled = 0;
    double hm_eps = 1e-5, hm_eta = 1.0;
    bool hm_ok = false;
    int hm_max_rank = 0;
    double hm_bytes = 0.0;                 // matrix bytes one hierarchical product streams
    float2 *hm_dense = nullptr;
    float2 *hm_pool = nullptr;             // factor terms in slots of kHmatGroup (layout in hmat.hpp)
    size_t hm_pool_cap = 0;                // complex entries
    unsigned long long *hm_ctr = nullptr;  // pool entries taken
    int64_t *hm_offs = nullptr;            // [nl][hm_slots(kmax)] pool offset of each slot of terms
    double2 *hm_t = nullptr;
    double2 *hm_xp = nullptr;              // x in tree order (product scratch)
    double2 *hm_yp = nullptr;              // partial sums of the product, [parts][3 n] in tree order
    int *hm_rank = nullptr, *hm_status = nullptr;
    int *hm_host = nullptr;                // pinned: ranks, then status flags
    int32_t *hm_items = nullptr;           // V^T x work items: block << 6 | first slot << 2 | (slots - 1)
    int32_t *hm_items_host = nullptr;      // pinned staging of hm_items
    int64_t hm_n_items = 0;
    unsigned long long *hm_used_host = nullptr;  // pinned: pool entries the build asked for
    bool hm_exhausted = false;             // the last build ran out of pool
    size_t hm_want = 0;                    // pool entries the next allocation asks for at least
    size_t hm_cap[3] = {0, 0, 0};
    void hm_alloc(const Problem &p, const HmatPlan &H);
    void hm_release();
    void reset_timing() { ev_used = 0; ev_prec.clear(); }
    ~Workspace();
    void release();
    void ensure(const Problem &p, int format, int restart_m, int prec_kind = 0);
};

// y = A x with a stored matrix: precision 0 = FP64 (C128, or hi+lo of SPLIT),
// 1 = FP32 on the hi plane; format kFmtBlocks: matrix-free (far field
// evaluated on the fly in FP64 or FP32, near/self blocks of the workspace).
// Counts applications and streamed matrix bytes.
struct Operator {
    int64_t N;
    int format, precision;
    const void *A, *A_lo;
    double *partial;
    int *counter;
    double *bytes;
    Workspace *prof = nullptr;             // non-null: record GEMV events
    const Problem *prob = nullptr;         // matrix-free: plan, frequency, blocks
    KernelParams kp{};
    const double *nearblk = nullptr, *selfblk = nullptr;
    const Workspace *hm = nullptr;         // FP32 products through the hierarchical form when built
    void apply(const double *x, double *y, hipStream_t st) const;
};

struct GmresResult {
    int iters = 0, cycles = 0;
    double est = 0.0;  // last residual norm (true residual of the operator after a restart)
    double aug_gain = 0.0;  // augmented first cycle: residual reduction by the augmentation direction alone
    bool converged = false, nan = false;
};

// Right-preconditioned GMRES(m) on op with the block-Jacobi inverses in
// ws.precond.  x (device) is the initial guess unless x_is_zero; on return it
// holds the iterate.  Stops when the residual norm is <= tol_abs.  With
// verify = false a cycle whose Arnoldi estimate meets the tolerance returns
// without forming the true residual of op (an outer loop judges it).  r0
// (nullable, with x not zero): the residual of x, already formed.  aug
// (nullable): a vector that joins the search space of the first cycle
// (flexible GMRES with aug as direction 0 and the preconditioned basis
// vectors after it), its coefficient found by the same least-squares problem.
//
// progress (nullable): called with the residual estimate after every Arnoldi
// step of the ordinary cycles.
// recycle: 0 = none; 1 = keep the last cycle's subspace in ws (rc_*); 2 = the
// first cycle (x zero, no aug) starts from the kept subspace of the same
// operator: the solution is sought in M^-1 span(kept V_K) plus the Krylov
// space of the residual's part outside span(V_{K+1}).
GmresResult gmres(const Operator &op, Workspace &ws, int64_t n_tri, const double *rhs, double rhs_norm, double *x,
                  bool x_is_zero, double tol_abs, int restart, int max_iter, hipStream_t st, bool verify,
                  const double *r0 = nullptr, double r0_norm = 0.0, const double *aug = nullptr, int recycle = 0,
                  const std::function<void(double)> &progress = {});

int solve_pipelined(Problem &p, const afsbem_solve_opts &o, int32_t n_s, const double *s, const double *bc,
                    const double *x0_user, double *a_out, double *u_out, double *t_out,
                    afsbem_solve_stats *stats, hipStream_t caller);

int solve_one(Problem &p, const afsbem_solve_opts &o, double s_re, double s_im, const double *d_bc,
              const double *d_x0, double *d_a, double *d_u, double *d_t, afsbem_solve_stats *stats,
              hipStream_t st);

}  // namespace afsbem
