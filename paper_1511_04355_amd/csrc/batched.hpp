// Batched (lockstep) solve of many systems: layout and kernel launchers.
#pragma once
#include <map>
#include <vector>

#include "internal.hpp"

namespace afsbem {

struct BSys {
    int64_t N, off, lda, chunk, part_off;
    int S, pad;
    const void *A, *A_lo;
};

struct BatchDev {
    int B = 0;
    int64_t Ntot = 0;
    int nvmax = 0;
    BSys *sys = nullptr;
    int32_t *sys_of_row = nullptr;
    int4 *items128 = nullptr, *items64 = nullptr;
    int64_t n_items128 = 0, n_items64 = 0;
    int4 *chunks = nullptr;
    int64_t n_chunks = 0;
    int32_t *chunk_ptr = nullptr;
    double *partial = nullptr, *dot_partial = nullptr;
    double *precond = nullptr;
    double *H = nullptr, *g = nullptr, *cs = nullptr, *sn = nullptr, *est = nullptr;
    int *kdone = nullptr;
};

// Device memory and streams of the batched solve, kept between calls (owned
// by the first problem of a call, released with it).
struct BatchArena {
    void *base = nullptr;
    size_t cap = 0;
    hipStream_t st_asm[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t st_sol = nullptr;
    // Instantiated graphs of Arnoldi-step blocks, kept while the arena is not
    // reallocated: a later wave with the same layout in the same slot has
    // identical kernel arguments and replays them.
    std::map<std::vector<int64_t>, std::vector<hipGraphExec_t>> graphs;
    ~BatchArena();
    void reserve(size_t bytes);
    void drop_graphs();
};

// kind 0: C128 FP64; 1: split hi plane FP32; 2: split hi+lo FP64
void bgemv(const BatchDev &b, int kind, const int *active, const double *x, double *y, hipStream_t st);
void bmdot(const BatchDev &b, const int *active, int nv, const double *V, const double *w, double *out, int ldo,
           hipStream_t st);
void bcombine(const BatchDev &b, const int *active, int nv, const int *nv_sys, const double *V, const double *h,
              int ldh, double sign, double *w, hipStream_t st);
void bnormalize(const BatchDev &b, const int *active, const double *nrm2, int ld, const double *x, double *out,
                hipStream_t st);
void bsub(const BatchDev &b, const int *active, const double *a, const double *c, double *out, hipStream_t st);
void bprecond(const BatchDev &b, const int *active, const double *v, double *z, hipStream_t st);
void bgivens(const BatchDev &b, int m, int k, int *cyc, const double *h1, const double *h2, int ldh,
             const double *nrm2, const double *tol, hipStream_t st);
void bbacksolve(const BatchDev &b, int m, const int *run, double *y, int ldy, hipStream_t st);
void bcycle_init(const BatchDev &b, int m, const int *run, const double *nrm2, const double *tol, int *cyc,
                 hipStream_t st);
void bcount(const BatchDev &b, const int *flag, int *out, hipStream_t st);

// Solves every (problem, frequency) pair; see afsbem_solve_batched_device.
int solve_batched(int n_prob, Problem *const *probs, const int32_t *n_s, const double *s,
                  const double *const *bc, double *const *a_out, double *const *u_out, double *const *t_out,
                  const afsbem_solve_opts &o, afsbem_solve_stats *stats, hipStream_t caller);

}  // namespace afsbem
