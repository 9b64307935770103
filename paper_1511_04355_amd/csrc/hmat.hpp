// Hierarchical (H-matrix) form of the matrix-free collocation operator: the
// inner (FP32-precision) operator of the mixed matrix-free solve.
//
// A binary cluster tree over the elements (recursive coordinate bisection of
// the collocation points, leaves of at most kLeafElems elements) and a
// block partition of (tree, tree): a pair of clusters whose bounding spheres
// are separated by at least eta times the larger radius, and between which
// there is no near pair, is admissible and stored as low-rank factors
// U V^T found by adaptive cross approximation with partial pivoting on the
// far rule's entries; every other leaf pair is a dense block of the operator
// (self block, far rule, near-pair correction: the sum the matrix-free
// product forms).  Indices of blocks are positions in tree order.  Factors
// are stored in FP32 (the operator serves FP32 products) in a pool carved as
// terms are found, kHmatGroup terms per slot, so memory follows the ranks
// reached.  A slot holds, for each leaf of the block's row cluster in tree
// order, the group's rows of that leaf term after term (the leaf's padded row
// count each), then the group's V terms (padded column count each): the
// product reads a leaf's rows of a whole group as one contiguous range.
#pragma once
#include "internal.hpp"

namespace afsbem {

struct Workspace;

constexpr int kHmatKmax = 128;  // terms per low-rank block at most
constexpr int kHmatGroup = 8;   // terms per pool slot
static_assert(kHmatKmax / kHmatGroup <= 16, "a V^T x item packs its first slot in four bits");
// dense blocks are column-major with an even row count (the product reads two
// rows per 16-byte load); the padding row is zero
constexpr int kHmatApplyParts = 32;  // partial sums per row of the product (parts of each leaf's block list)
__host__ __device__ inline int64_t dense_rows_padded(int64_t n_elems) { return 3 * n_elems + ((3 * n_elems) & 1); }
// entries of one pool slot of a low-rank block with RL padded rows (summed
// over its leaves) and Cp padded columns, rounded to 128 bytes
__host__ __device__ inline int64_t hm_slot_entries(int64_t RL, int64_t Cp) {
    return (kHmatGroup * (RL + Cp) + 15) & ~(int64_t)15;
}
__host__ __device__ inline int hm_slots(int kmax) { return (kmax + kHmatGroup - 1) / kHmatGroup; }

struct HmatPlan {
    double eta = 1.0;
    int64_t n = 0;
    std::vector<int32_t> perm;      // tree position -> element
    std::vector<int64_t> dense;     // [nd][4] a0, a1, b0, b1 (tree positions of elements)
    std::vector<int64_t> lowrank;   // [nl][4]
    std::vector<int64_t> dense_off; // [nd+1] offsets (complex entries) of the dense blocks (padded rows)
    int64_t lr_rows = 0;            // sum over low-rank blocks of RL + Cp (one term's padded entries)
    std::vector<int32_t> lr_order;  // low-rank blocks by size: at most 64 elements a side, at most 128, larger
    std::vector<int32_t> vt_order;  // low-rank blocks in the order of the V^T x work (width classes, then columns)
    int64_t n_small = 0, n_mid = 0;
    std::vector<int64_t> leaves;    // [nleaf][2] row ranges of the leaves
    std::vector<int64_t> leaf_ptr;  // [nleaf+1]
    std::vector<int32_t> leaf_item; // dense block d as d, low-rank block l as -(l + 1)
    std::vector<int32_t> leaf_of;   // [n] leaf of each tree position
    std::vector<int64_t> leaf_prow; // [nleaf+1] prefix sums of the leaves' padded row counts
    std::vector<int64_t> lr_rp;     // [nl][2] leaf_prow at the row cluster's first leaf, padded rows RL
    int kmax = 0;
    // device copies
    int32_t *d_perm = nullptr;
    int64_t *d_dense = nullptr, *d_lowrank = nullptr, *d_dense_off = nullptr;
    int64_t *d_leaves = nullptr, *d_leaf_ptr = nullptr;
    int32_t *d_leaf_item = nullptr;
    int32_t *d_lr_order = nullptr;
    int32_t *d_leaf_of = nullptr;
    int64_t *d_leaf_prow = nullptr, *d_lr_rp = nullptr;
    std::vector<void *> allocs;
    ~HmatPlan();
};

// cluster tree and block partition of the problem's elements (host), uploaded
// unless upload = false (host-side inspection)
void hmat_build(const Problem &p, double eta, int kmax, HmatPlan &out, bool upload = true);
// p.hmat built for this eta (rebuilt when eta changed; no work in flight may use the old one)
void hmat_ensure(Problem &p, double eta);

// per-frequency blocks: dense blocks and ACA factors into the workspace
// (after the matrix-free block setup: nearblk, selfblk), ranks and status
// copied to pinned host memory on st.  hmat_finish, once st's work has
// completed, reads them: false when an admissible block did not reach eps
// within kmax or found the pool spent (ws.hm_exhausted; the operator then
// stays the on-the-fly one unless the build is repeated).  It also lists the
// work items of the product's V^T x pass (runs of a block's slots) for the
// ranks reached, widest blocks first, and copies them to the device on st (from pinned
// memory that the next call overwrites: st must have finished the copy by then).
void hmat_setup(const Problem &p, Workspace &ws, const KernelParams &kp, double eps, hipStream_t st);
bool hmat_finish(Problem &p, Workspace &ws, hipStream_t st);
// y = A_H x
void hmat_apply(const Problem &p, const Workspace &ws, const double *x, double *y, hipStream_t st);

}  // namespace afsbem
