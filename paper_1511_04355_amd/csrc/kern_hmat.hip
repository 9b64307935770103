// Hierarchical far field of the matrix-free operator on gfx950: dense blocks
// and low-rank factors per frequency, and the product y = A_H x.
//
// Low-rank blocks: adaptive cross approximation with partial pivoting on the
// far rule's entries (evaluated in FP32, residual arithmetic in FP64, terms
// stored in FP32 in a pool whose slots of kHmatGroup terms a work-group takes
// with one atomic add per slot): at step k the residual row i_k (the block's row
// minus sum_l U_l[i_k] V_l) is evaluated, its largest entry j_k becomes the
// pivot, V_k = row / row[j_k], U_k = the residual column j_k, and the next row
// is the largest entry of U_k outside the rows already used; the block stops
// when |U_k| |V_k| <= eps |S_k|_F (|S_k|_F^2 accumulated as sum |U_l|^2 |V_l|^2,
// cross terms neglected) and eight probe rows, one in each eighth of the
// block's rows in tree order (spatially coherent sub-ranges), have residuals
// below eps times the mean row norm of S_k; a probe row that fails becomes the
// next pivot (partial pivoting alone can leave a patch of a block's rows
// unsampled, e.g. where a cluster spans separate surfaces).  One work-group per block; a row
// or column costs one element-pair block per source or target element.
//
// Product: x gathered into tree order, t_l = V_l^T x per low-rank block
// (persistent single waves over runs of a block's slots, a lane per column
// pair of the slot's eight terms), then kHmatApplyParts single-wave work-groups per
// leaf row range each sum every kHmatApplyParts-th entry of the leaf's list of
// dense blocks (column-major FP32, read coalesced) and covering low-rank blocks
// (the leaf's rows of a slot's terms, contiguous), and the partial sums are
// added in a fixed order (no atomics).
#include "hmat.hpp"
#include "kern_eval.hpp"
#include "kern_mfeval.hpp"
#include "solver.hpp"

namespace afsbem {

namespace {

constexpr int kHmKmax = kHmatKmax;

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// 3x3 block (m, n) of the matrix-free operator for m != n (far rule; with
// near = true also the pair's near correction)
__device__ void hm_pair_block(const KernelParams &kp, const double *__restrict__ colx,
                              const double *__restrict__ coly, const double *__restrict__ colz,
                              const double *__restrict__ src, const double *__restrict__ coef, int64_t m, int64_t n,
                              cd blk[9]) {
    const double *rec = src + kSrcStride * n;
    const double nx = rec[28], ny = rec[29], nz = rec[30];
    const int kind = (int)rec[31];
    const cd v0[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
    cd bdummy[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
    BlockAcc acc;
    acc.zero();
    const double xx = colx[m], xy = coly[m], xz = colz[m];
#pragma unroll 1
    for (int q = 0; q < kFarNodes; ++q) {
        PairEval E;
        eval_pair(kp, coef, xx, xy, xz, rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], nx, ny, nz, E);
        const double w = rec[4 * q + 3];
        if (kind == 0)
            acc_node<0>(E, kp, nx, ny, nz, w, 0.0, v0, acc, bdummy);
        else
            acc_node<1>(E, kp, nx, ny, nz, w, 0.0, v0, acc, bdummy);
    }
    expand_block(kind, acc, nx, ny, nz, blk);
}

// FP32 evaluation of the cross approximation's entries (the operator it
// approximates serves FP32 products): s / c_s, beta, lambda/mu, 1/(4 pi mu),
// 1/|s/c_s|^2
struct Hm32 {
    float sr, si, beta, lam, cu, iks2;
};

// three entries of the far-rule block (m, n): row a (row = true) or column a;
// T for a kind-0 source, -U for kind 1
__device__ void hm_entries32(const Hm32 &h, const float *__restrict__ col32, const float *__restrict__ src32,
                             const float *__restrict__ coef32, int64_t m, int64_t n, bool row, int a, cd out[3]) {
    const float *rec = src32 + kSrcStride * n;
    const float nx = rec[28], ny = rec[29], nz = rec[30];
    const int kind = (int)rec[31];
    const float px = col32[4 * m], py = col32[4 * m + 1], pz = col32[4 * m + 2];
    const float nn[3] = {nx, ny, nz};
    cx<float> acc[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
#pragma unroll 1
    for (int q = 0; q < kFarNodes; ++q) {
        const float dx = rec[4 * q] - px, dy = rec[4 * q + 1] - py, dz = rec[4 * q + 2] - pz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ir = inv_sqrt(r2);
        const float r = r2 * ir;
        const float rh[3] = {dx * ir, dy * ir, dz * ir};
        const MfRad<float> Rd = mf_radial<float>(cx<float>{h.sr * r, h.si * r}, h.beta, coef32, ir * ir * h.iks2);
        if (kind == 0) {
            const float f = rec[4 * q + 3] * 0.079577471545947667884f * ir * ir;
            const float rn = rh[0] * nx + rh[1] * ny + rh[2] * nz;
            const cx<float> t1 = cxsub(Rd.Psd, Rd.X);
            const cx<float> t0 = cxs(t1, rn);
            const cx<float> t2 = cxadd(cxs(Rd.X, -2.f), cxs(cxsub(cxsub(Rd.Psd, Rd.Xd), cxs(Rd.X, 2.f)), h.lam));
            const cx<float> t3 = cxs(cxsub(cxs(Rd.X, 4.f), cxs(Rd.Xd, 2.f)), rn);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int i = row ? a : b, j = row ? b : a;
                cx<float> v = cxadd(cxadd(cxs(t1, nn[i] * rh[j]), cxs(t2, rh[i] * nn[j])), cxs(t3, rh[i] * rh[j]));
                if (i == j)
                    v = cxadd(v, t0);
                acc[b] = cxadd(acc[b], cxs(v, f));
            }
        } else {
            const float g = -rec[4 * q + 3] * h.cu * ir;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int i = row ? a : b, j = row ? b : a;
                cx<float> v = cxs(Rd.X, -rh[i] * rh[j]);
                if (i == j)
                    v = cxadd(v, Rd.Psi);
                acc[b] = cxadd(acc[b], cxs(v, g));
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
        out[b] = cd{(double)acc[b].r, (double)acc[b].i};
}

// dense block d: (3 na) x (3 nb), column-major, FP32 complex
__global__ __launch_bounds__(256) void hm_dense_kernel(
    KernelParams kp, const double *__restrict__ colx, const double *__restrict__ coly, const double *__restrict__ colz,
    const double *__restrict__ src, const double *__restrict__ coef, const int64_t *__restrict__ near_ptr,
    const int32_t *__restrict__ near_col, const double *__restrict__ nearblk, const double *__restrict__ selfblk,
    const int32_t *__restrict__ perm, const int64_t *__restrict__ dense, const int64_t *__restrict__ dense_off,
    float2 *__restrict__ out) {
    const int64_t d = blockIdx.x;
    const int64_t a0 = dense[4 * d], b0 = dense[4 * d + 2];
    const int na = (int)(dense[4 * d + 1] - a0), nb = (int)(dense[4 * d + 3] - b0);
    const int64_t R = dense_rows_padded(na);
    float2 *blk_out = out + dense_off[d];
    if (R != 3 * (int64_t)na)
        for (int k = threadIdx.x; k < 3 * nb; k += 256)
            blk_out[(int64_t)k * R + R - 1] = make_float2(0.f, 0.f);
    for (int q = threadIdx.x; q < na * nb; q += 256) {
        const int r = q % na, k = q / na;
        const int64_t m = perm[a0 + r], n = perm[b0 + k];
        cd blk[9];
        if (m == n) {
            const double *sb = selfblk + 18 * m;
#pragma unroll
            for (int e = 0; e < 9; ++e)
                blk[e] = cd{sb[2 * e], sb[2 * e + 1]};
        } else {
            hm_pair_block(kp, colx, coly, colz, src, coef, m, n, blk);
            for (int64_t pp = near_ptr[m]; pp < near_ptr[m + 1]; ++pp)
                if (near_col[pp] == n) {
                    const double *nb9 = nearblk + 18 * pp;
#pragma unroll
                    for (int e = 0; e < 9; ++e)
                        blk[e] = cadd(blk[e], cd{nb9[2 * e], nb9[2 * e + 1]});
                    break;
                }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                blk_out[(3 * k + b) * R + 3 * r + a] = make_float2((float)blk[3 * a + b].r, (float)blk[3 * a + b].i);
    }
}

// work-group (NT threads) reductions through LDS
// one pass: argmax of v (index i, smallest index on ties) and the sums of a and b
struct RedMaxSum {
    double v;
    int64_t i;
    double a, b;
};
template <int NT>
__device__ __forceinline__ RedMaxSum group_argmax_sums(double v, int64_t i, double a, double b, double *sv,
                                                       int64_t *si, double *sa, double *sb) {
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = i;
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (t < h) {
            const double o = sv[t + h];
            const int64_t oi = si[t + h];
            if (o > sv[t] || (o == sv[t] && oi < si[t])) {
                sv[t] = o;
                si[t] = oi;
            }
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    RedMaxSum r{sv[0], si[0], sa[0], sb[0]};
    __syncthreads();
    return r;
}

// status: 0 converged, 1 out of terms, 2 pool exhausted.  NT threads per
// block: 64 for blocks of at most 64 elements a side (most are leaf pairs of
// 32), 128 up to 128, 256 for the larger ones; ids lists the blocks of this launch.
// Place of row r of a low-rank block in its pool slots (layout in hmat.hpp):
// the row's leaf's offset within a slot, the leaf's padded row count, and the
// row's index within the leaf.
struct HmRowPos {
    int64_t lo, rp, rl;
};
__device__ __forceinline__ HmRowPos hm_row_pos(int64_t a0, int64_t rowbase, int64_t r,
                                               const int32_t *__restrict__ leaf_of,
                                               const int64_t *__restrict__ leaves,
                                               const int64_t *__restrict__ leaf_prow) {
    const int64_t el = a0 + r / 3;
    const int32_t L = leaf_of[el];
    const int64_t L0 = leaves[2 * L];
    HmRowPos o;
    o.rp = dense_rows_padded(leaves[2 * L + 1] - L0);
    o.lo = (leaf_prow[L] - rowbase) * kHmatGroup;
    o.rl = 3 * (el - L0) + r % 3;
    return o;
}

template <int NT>
__global__ __launch_bounds__(NT) void hm_aca_kernel(
    const int32_t *__restrict__ perm,
    const int64_t *__restrict__ lowrank, const int32_t *__restrict__ ids, int kmax, double eps,
    float2 *__restrict__ pool, unsigned long long pool_cap, unsigned long long *__restrict__ ctr,
    int64_t *__restrict__ offs, int *__restrict__ rank_out, int *__restrict__ status_out, Hm32 h32,
    const float *__restrict__ col32, const float *__restrict__ src32, const float *__restrict__ coef32_g,
    const int32_t *__restrict__ leaf_of, const int64_t *__restrict__ leaves, const int64_t *__restrict__ leaf_prow,
    const int64_t *__restrict__ lr_rp) {
    __shared__ float coef32[64];
    if (threadIdx.x < 64)
        coef32[threadIdx.x] = coef32_g[threadIdx.x];
    __shared__ double sv[NT], sa[NT], sb[NT];
    __shared__ int64_t si[NT];
    __shared__ double2 cf[kHmKmax];
    __shared__ int64_t used[kHmKmax + 1];
    __shared__ int64_t sgoff[kHmKmax / kHmatGroup];  // pool offsets of the slots taken so far
    __shared__ double2 sent[3 * NT];   // one chunk of NT element pairs' entries (3 per pair)
    const int t = threadIdx.x;
    const int64_t l = ids[blockIdx.x];
    const int64_t a0 = lowrank[4 * l], b0 = lowrank[4 * l + 2];
    const int64_t na = lowrank[4 * l + 1] - a0, nb = lowrank[4 * l + 3] - b0;
    const int64_t R = 3 * na, C = 3 * nb;
    // rows padded per leaf and columns padded to even counts, so that the
    // products read two entries per 16-byte load
    const int64_t rowbase = lr_rp[2 * l], RL = lr_rp[2 * l + 1], Cp = C + (C & 1);
    const int64_t slot = hm_slot_entries(RL, Cp);
    int64_t *myoffs = offs + l * hm_slots(kmax);
    // pool index of row (at p) of U_q, and of column c of V_q
    auto upos = [&](int q, const HmRowPos &p) {
        return sgoff[q / kHmatGroup] + p.lo + (int64_t)(q % kHmatGroup) * p.rp + p.rl;
    };
    auto vpos = [&](int q, int64_t c) {
        return sgoff[q / kHmatGroup] + kHmatGroup * RL + (int64_t)(q % kHmatGroup) * Cp + c;
    };
    auto rowpos = [&](int64_t r) { return hm_row_pos(a0, rowbase, r, leaf_of, leaves, leaf_prow); };
    int64_t istar = 0;
    double S2 = 0.0;
    int k = 0, status = 1, probes_ok = 0, n_probe = 0;
    bool probing = false;
    // probe rows spread over the block's row range in tree order (spatially
    // coherent sub-ranges): the middle of the j-th eighth, component j % 3,
    // skipping rows already used (same on every thread)
    constexpr int kProbes = 8;
    auto probe_row = [&]() {
        const int j = (n_probe++) % kProbes;
        int64_t r = 3 * (((2 * (int64_t)j + 1) * na) / (2 * kProbes)) + j % 3;
        for (int tries = 0; tries <= k; ++tries) {
            bool was = false;
            for (int q = 0; q < k; ++q)
                was = was || (used[q] == r);
            if (!was)
                break;
            r = (r + 1) % R;
        }
        return r;
    };
    while (k < kmax) {
        // ---- a new slot for every kHmatGroup terms (a probe row is evaluated, not stored)
        const bool new_slot = !probing && (k % kHmatGroup) == 0;
        if (t == 0 && new_slot) {
            const unsigned long long o = atomicAdd(ctr, (unsigned long long)slot);
            const bool fits = o + (unsigned long long)slot <= pool_cap;
            sgoff[k / kHmatGroup] = fits ? (int64_t)o : -1;
            if (fits)
                myoffs[k / kHmatGroup] = (int64_t)o;
        }
        {
            const HmRowPos pi = rowpos(istar);
            for (int q = t; q < k; q += NT) {
                const float2 u = pool[upos(q, pi)];
                cf[q] = make_double2(u.x, u.y);
            }
        }
        __syncthreads();
        if (new_slot && sgoff[k / kHmatGroup] < 0) {
            status = 2;
            break;
        }
        // ---- residual row istar -> V_k (unnormalised)
        const int64_t m = perm[a0 + istar / 3];
        const int al = (int)(istar % 3);
        double best = -1.0, rn = 0.0;
        int64_t bi = 0;
        // chunks of NT element pairs: each thread evaluates one pair's three
        // entries into LDS, then the chunk's entries are taken in order by
        // consecutive threads, so that the earlier terms are read coalesced
        for (int64_t base = 0; base < nb; base += NT) {
            if (base + t < nb) {
                cd ent[3];
                hm_entries32(h32, col32, src32, coef32, m, perm[b0 + base + t], true, al, ent);
#pragma unroll
                for (int be = 0; be < 3; ++be)
                    sent[3 * t + be] = make_double2(ent[be].r, ent[be].i);
            }
            __syncthreads();
            const int64_t ce = (3 * (nb - base) < 3 * NT) ? 3 * (nb - base) : 3 * NT;
            for (int64_t e = t; e < ce; e += NT) {
                const int64_t c = 3 * base + e;
                double vr = sent[e].x, vi = sent[e].y;
#pragma unroll 4
                for (int q = 0; q < k; ++q) {
                    const double2 u = cf[q];
                    const float2 v = pool[vpos(q, c)];
                    vr -= u.x * v.x - u.y * v.y;
                    vi -= u.x * v.y + u.y * v.x;
                }
                if (!probing)
                    pool[vpos(k, c)] = make_float2((float)vr, (float)vi);
                const double a2 = vr * vr + vi * vi;
                rn += a2;
                if (a2 > best) {
                    best = a2;
                    bi = c;
                }
            }
            __syncthreads();
        }
        const RedMaxSum pv = group_argmax_sums<NT>(best, bi, rn, 0.0, sv, si, sa, sb);
        const double rn2 = pv.a;
        if (probing) {
            // after the stopping test: probe rows whose residuals are small
            // against the mean row norm of S confirm it (all kProbes in a row);
            // otherwise the probe row becomes the next pivot row
            if (rn2 <= eps * eps * S2 / (double)R) {
                if (++probes_ok >= kProbes) {
                    status = 0;
                    break;
                }
                istar = probe_row();
                continue;
            }
            probing = false;  // the probe row becomes the next pivot row: evaluate and store it
            probes_ok = 0;
            continue;
        }
        if (!(pv.v > 0.0)) {  // the residual row vanishes: nothing left to approximate
            status = 0;
            break;
        }
        const int64_t jstar = pv.i;
        float2 *Vk = pool + vpos(k, 0);
        const float2 pf = Vk[jstar];
        __syncthreads();
        const double pd = (double)pf.x * pf.x + (double)pf.y * pf.y;
        const double ir = pf.x / pd, ii = -pf.y / pd;  // 1 / pivot
        double nv = 0.0;
        for (int64_t c = t; c < C; c += NT) {
            const float2 v = Vk[c];
            const double wr = v.x * ir - v.y * ii, wi = v.x * ii + v.y * ir;
            Vk[c] = make_float2((float)wr, (float)wi);
            nv += wr * wr + wi * wi;
        }
        // ---- residual column jstar -> U_k
        for (int q = t; q < k; q += NT) {
            const float2 v = pool[vpos(q, jstar)];
            cf[q] = make_double2(v.x, v.y);
        }
        if (t == 0)
            used[k] = istar;
        __syncthreads();
        const int64_t n = perm[b0 + jstar / 3];
        const int be = (int)(jstar % 3);
        double nu = 0.0;
        best = -1.0;
        bi = 0;
        for (int64_t base = 0; base < na; base += NT) {
            if (base + t < na) {
                cd ent[3];
                hm_entries32(h32, col32, src32, coef32, perm[a0 + base + t], n, false, be, ent);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    sent[3 * t + a] = make_double2(ent[a].r, ent[a].i);
            }
            __syncthreads();
            const int64_t ce = (3 * (na - base) < 3 * NT) ? 3 * (na - base) : 3 * NT;
            for (int64_t e = t; e < ce; e += NT) {
                const int64_t r = 3 * base + e;
                const HmRowPos pr = rowpos(r);
                double ur = sent[e].x, ui = sent[e].y;
#pragma unroll 4
                for (int q = 0; q < k; ++q) {
                    const double2 v = cf[q];
                    const float2 u = pool[upos(q, pr)];
                    ur -= u.x * v.x - u.y * v.y;
                    ui -= u.x * v.y + u.y * v.x;
                }
                pool[upos(k, pr)] = make_float2((float)ur, (float)ui);
                const double a2 = ur * ur + ui * ui;
                nu += a2;
                bool was = false;
                for (int q = 0; q <= k; ++q)
                    was = was || (used[q] == r);
                if (!was && a2 > best) {
                    best = a2;
                    bi = r;
                }
            }
            __syncthreads();
        }
        const RedMaxSum nx = group_argmax_sums<NT>(best, bi, nu, nv, sv, si, sa, sb);
        const double nu2 = nx.a, nv2 = nx.b;
        ++k;
        S2 += nu2 * nv2;
        // the terms span the block (k = min(R, C): U V^T is then the block itself)
        if (k >= (R < C ? R : C) || !(nx.v >= 0.0)) {
            status = 0;
            break;
        }
        if (nu2 * nv2 <= eps * eps * S2) {  // stopping test met: confirm on probe rows
            probing = true;
            probes_ok = 0;
            istar = probe_row();
            continue;
        }
        istar = nx.i;
    }
    if (t == 0) {
        rank_out[l] = k;
        status_out[l] = status;
    }
}

// x in tree order: xp[3 q + c] = x[3 perm[q] + c]
__global__ __launch_bounds__(256) void hm_gather_kernel(int64_t n, const int32_t *__restrict__ perm,
                                                        const double2 *__restrict__ x, double2 *__restrict__ xp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < 3 * n)
        xp[i] = x[3 * (int64_t)perm[i / 3] + i % 3];
}

// t_q = V_q^T x for every term of every low-rank block, as a list of items
// of up to four slots of one block (widest blocks first, then by column
// range: the items in flight share their x), taken by a grid of single-wave
// work-groups in turn (item i by wave i mod the grid).  Lane j takes the
// column pairs j, j + 64, ... of all kHmatGroup terms of the slot: x is read
// once per pair for the eight terms and eight 16-byte loads of V are in
// flight per lane, issued unconditionally from clamped indices (the terms
// past the rank read the last term again and are not written).  The next
// item's description is loaded while the first loads of the current one are
// in flight.  The 16 sums (term, real / imaginary) are reduced over the wave
// by a butterfly that halves the set each lane keeps at every step: 17
// exchanges, after which lanes 4k .. 4k + 3 hold sum k.
constexpr int kVtWaves = 256 * 20;  // waves of the V^T x pass (20 per compute unit: the occupancy its registers allow)

struct VtItem {
    const float4 *V;    // the current slot's first term (V part), 16-byte units
    const float2 *P;    // the block's V parts: pool + kHmatGroup * (padded rows of the block)
    const int64_t *so;  // the block's slot offsets
    const double2 *x;   // the block's column range of x (tree order)
    int64_t C, st4;     // columns; float4 per term
    int64_t t0;         // index of the current slot's first t_q
    int s, send, rk;    // current slot, end of the item's slots, rank
    int last;           // terms in the current slot less one
};

// item code: block << 6 | first slot << 2 | (slots - 1)
__device__ __forceinline__ VtItem vt_item(int32_t code, const int64_t *__restrict__ lowrank, int kmax,
                                          const int *__restrict__ rank, const int64_t *__restrict__ offs,
                                          const int64_t *__restrict__ lr_rp, const float2 *__restrict__ pool,
                                          const double2 *__restrict__ xp) {
    const int64_t l = code >> 6;
    VtItem m;
    m.s = (code >> 2) & 15;
    m.send = m.s + (code & 3) + 1;
    const int64_t b0 = lowrank[4 * l + 2];
    m.C = 3 * (lowrank[4 * l + 3] - b0);
    m.st4 = (m.C + (m.C & 1)) >> 1;
    m.rk = rank[l];
    const int nq = m.rk - m.s * kHmatGroup;  // >= 1: items hold live slots only
    m.last = (nq < kHmatGroup ? nq : kHmatGroup) - 1;
    m.P = pool + kHmatGroup * lr_rp[2 * l + 1];
    m.so = offs + l * hm_slots(kmax);
    m.V = reinterpret_cast<const float4 *>(m.P + m.so[m.s]);
    m.x = xp + 3 * b0;
    m.t0 = l * kmax + m.s * kHmatGroup;
    return m;
}

// the item's next slot
__device__ __forceinline__ VtItem vt_next_slot(VtItem m) {
    m.s += 1;
    const int nq = m.rk - m.s * kHmatGroup;
    m.last = (nq < kHmatGroup ? nq : kHmatGroup) - 1;
    m.V = reinterpret_cast<const float4 *>(m.P + m.so[m.s]);
    m.t0 += kHmatGroup;
    return m;
}

// one butterfly step: lanes whose bit log2(4 H) is clear keep sums 0 .. H-1
// of their set, the others sums H .. 2H-1, each added to its partner's copy
template <int H>
__device__ __forceinline__ void vt_halve(double (&s)[16], int lane) {
    const bool hi = (lane & (4 * H)) != 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double send = hi ? s[k] : s[k + H];
        const double keep = hi ? s[k + H] : s[k];
        s[k] = keep + __shfl_xor(send, 4 * H, 64);
    }
}

__global__ __launch_bounds__(64) void hm_vt_kernel(const int32_t *__restrict__ items, int64_t n_items,
                                                   const int64_t *__restrict__ lowrank, int kmax,
                                                   const int *__restrict__ rank, const int64_t *__restrict__ offs,
                                                   const int64_t *__restrict__ lr_rp, const float2 *__restrict__ pool,
                                                   const double2 *__restrict__ xp, double2 *__restrict__ tv) {
    static_assert(kHmatGroup == 8, "eight terms per item");
    int64_t it = blockIdx.x;
    if (it >= n_items)
        return;
    const int lane = threadIdx.x;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    VtItem m = vt_item(items[it], lowrank, kmax, rank, offs, lr_rp, pool, xp);
    for (;;) {
        const int64_t nx = it + gridDim.x;
        const int64_t C2 = m.C >> 1;  // >= 1
        double sr[8], si[8];
        {
            const int64_t pc = lane < C2 ? lane : C2 - 1;
            float4 va[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                va[e] = m.V[(int64_t)(e < m.last ? e : m.last) * m.st4 + pc];
            const double2 x0 = m.x[2 * pc], x1 = m.x[2 * pc + 1];
            const bool same = m.s + 1 < m.send;
            VtItem mn = m;
            if (same)
                mn = vt_next_slot(m);
            else if (nx < n_items)
                mn = vt_item(items[nx], lowrank, kmax, rank, offs, lr_rp, pool, xp);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float4 v = lane < C2 ? va[e] : z4;
                sr[e] = (double)v.x * x0.x - (double)v.y * x0.y + (double)v.z * x1.x - (double)v.w * x1.y;
                si[e] = (double)v.x * x0.y + (double)v.y * x0.x + (double)v.z * x1.y + (double)v.w * x1.x;
            }
            for (int64_t p0 = 64; p0 < C2; p0 += 64) {
                const int64_t pa = p0 + lane;
                const int64_t pq = pa < C2 ? pa : C2 - 1;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    va[e] = m.V[(int64_t)(e < m.last ? e : m.last) * m.st4 + pq];
                const double2 y0 = m.x[2 * pq], y1 = m.x[2 * pq + 1];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float4 v = pa < C2 ? va[e] : z4;
                    sr[e] += (double)v.x * y0.x - (double)v.y * y0.y + (double)v.z * y1.x - (double)v.w * y1.y;
                    si[e] += (double)v.x * y0.y + (double)v.y * y0.x + (double)v.z * y1.y + (double)v.w * y1.x;
                }
            }
            if ((m.C & 1) && lane == 0) {  // the odd last column
                const double2 xv = m.x[m.C - 1];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float2 v =
                        reinterpret_cast<const float2 *>(m.V + (int64_t)(e < m.last ? e : m.last) * m.st4)[m.C - 1];
                    sr[e] += (double)v.x * xv.x - (double)v.y * xv.y;
                    si[e] += (double)v.x * xv.y + (double)v.y * xv.x;
                }
            }
            // sums k = 2 e + {0: real, 1: imaginary}
            double s[16];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s[2 * e] = sr[e];
                s[2 * e + 1] = si[e];
            }
            vt_halve<8>(s, lane);
            vt_halve<4>(s, lane);
            vt_halve<2>(s, lane);
            vt_halve<1>(s, lane);
            s[0] += __shfl_xor(s[0], 2, 64);
            s[0] += __shfl_xor(s[0], 1, 64);
            const int k = lane >> 2, e = k >> 1;
            if ((lane & 3) == 0 && e <= m.last)
                reinterpret_cast<double *>(tv)[2 * (m.t0 + e) + (k & 1)] = s[0];
            if (!same) {
                if (nx >= n_items)
                    break;
                it = nx;
            }
            m = mn;
        }
    }
}

// a 16-byte load marked non-temporal: the product's matrix entries are read
// once per product, and keeping them out of the way of x and t in the caches
// measured faster for the dense blocks and U (6.46 -> 5.84 ms per product
// pass at 300,516 unknowns), slower for V in the V^T x pass (4.04 -> 5.01 ms)
typedef float hm_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const hm_v4f v = __builtin_nontemporal_load(reinterpret_cast<const hm_v4f *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

constexpr int kHmSplit = kHmatApplyParts;  // single-wave work-groups per leaf: each takes every kHmSplit-th block of its list

__device__ __forceinline__ void cmac2(double &r0, double &i0, double &r1, double &i1, const float4 v,
                                      const double2 c) {
    r0 += (double)v.x * c.x - (double)v.y * c.y;
    i0 += (double)v.x * c.y + (double)v.y * c.x;
    r1 += (double)v.z * c.x - (double)v.w * c.y;
    i1 += (double)v.z * c.y + (double)v.w * c.x;
}

// one wavefront per (leaf L, part blockIdx.y): lane l owns rows 2l, 2l + 1 of
// the leaf (at most 96 rows, 48 lanes) and sums the blocks it - leaf_ptr[L] =
// blockIdx.y (mod kHmSplit) of the leaf's list: dense blocks column by column
// (16-byte loads of two rows, eight columns in flight), low-rank blocks a slot
// of kHmatGroup terms at a time (the leaf's rows of those terms are one
// contiguous range of the slot, eight terms in flight; slot offsets and t_q
// are wave-uniform scalar loads).  Partial sums in tree order, yp[part][3 n].
__global__ __launch_bounds__(64) void hm_apply_kernel(
    const int64_t *__restrict__ leaves, const int64_t *__restrict__ leaf_ptr, const int32_t *__restrict__ leaf_item,
    const int64_t *__restrict__ dense, const int64_t *__restrict__ dense_off, const int64_t *__restrict__ leaf_prow,
    const int64_t *__restrict__ lr_rp, int kmax, const int *__restrict__ rank, const int64_t *__restrict__ offs,
    const float2 *__restrict__ dblk, const float2 *__restrict__ pool, const double2 *__restrict__ tv,
    const double2 *__restrict__ xp, int64_t n_el, double2 *__restrict__ yp) {
    static_assert(kHmatGroup == 8, "the low-rank loop keeps one slot's eight terms in flight");
    const int64_t L = blockIdx.x;
    const int64_t L0 = leaves[2 * L], rows = 3 * (leaves[2 * L + 1] - L0);
    const int64_t Rp = rows + (rows & 1);
    const int64_t prow = leaf_prow[L];
    const int lane = threadIdx.x;
    const int64_t r = 2 * (int64_t)lane;
    const bool live = r < rows;
    // lanes past the leaf's rows load a live lane's entries (in bounds) and
    // drop them, so that every load of a batch is issued without a branch and
    // the batch is in flight together
    const int64_t lc = live ? lane : (Rp >> 1) - 1;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
    for (int64_t it = leaf_ptr[L] + blockIdx.y; it < leaf_ptr[L + 1]; it += kHmSplit) {
        const int32_t item = leaf_item[it];
        if (item >= 0) {
            const int64_t b0 = dense[4 * item + 2];
            const int64_t C = 3 * (dense[4 * item + 3] - b0);
            const float4 *D = reinterpret_cast<const float4 *>(dblk + dense_off[item]) + lc;
            const int64_t ld = Rp >> 1;  // float4 per column
            const double2 *xb = xp + 3 * b0;
            int64_t c = 0;
            for (; c + 8 <= C; c += 8) {
                float4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = ld_nt(&D[(c + u) * ld]);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    cmac2(a0r, a0i, a1r, a1i, live ? v[u] : z4, xb[c + u]);
            }
            for (; c < C; ++c) {
                const float4 v = ld_nt(&D[c * ld]);
                cmac2(a0r, a0i, a1r, a1i, live ? v : z4, xb[c]);
            }
        } else {
            const int64_t lb = -(int64_t)item - 1;
            const int rk = rank[lb];
            // this leaf's rows in every slot of the block: kHmatGroup terms of Rp
            // entries each (every offset even: 16-byte loads)
            const int64_t lo = (prow - lr_rp[2 * lb]) * kHmatGroup + 2 * lc;
            const int64_t *ob = offs + lb * hm_slots(kmax);
            const double2 *tb = tv + lb * kmax;
            const int64_t st4 = Rp >> 1;  // float4 per term of the leaf
            // a slot at a time; in the last one the terms past the rank load
            // the last term's rows again (in bounds) and take a zero coefficient
            for (int q = 0; q < rk; q += 8) {
                const float4 *U = reinterpret_cast<const float4 *>(pool + ob[q / 8] + lo);
                const int last = rk - q - 1;
                float4 u[8];
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    u[e] = ld_nt(&U[(e < last ? e : last) * st4]);
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    cmac2(a0r, a0i, a1r, a1i, live ? u[e] : z4, e <= last ? tb[q + e] : make_double2(0.0, 0.0));
            }
        }
    }
    if (live) {
        double2 *out = yp + (int64_t)blockIdx.y * 3 * n_el + 3 * L0 + r;
        out[0] = make_double2(a0r, a0i);
        if (r + 1 < rows)
            out[1] = make_double2(a1r, a1i);
    }
}

// y = sum of the kHmSplit partial sums (fixed order), back to element order
__global__ __launch_bounds__(256) void hm_sum_kernel(int64_t n, const int32_t *__restrict__ perm,
                                                     const double2 *__restrict__ yp, double2 *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * n)
        return;
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int p = 0; p < kHmSplit; ++p) {
        const double2 v = yp[(int64_t)p * 3 * n + i];
        ar += v.x;
        ai += v.y;
    }
    y[3 * (int64_t)perm[i / 3] + i % 3] = make_double2(ar, ai);
}

}  // namespace

void hmat_setup(const Problem &p, Workspace &ws, const KernelParams &kp, double eps, hipStream_t st) {
    const HmatPlan &H = *p.hmat;
    const DevicePlan &d = p.dev;
    const int64_t nd = (int64_t)H.dense.size() / 4, nl = (int64_t)H.lowrank.size() / 4;
    ws.hm_alloc(p, H);
    if (nd)
        hm_dense_kernel<<<(unsigned)nd, 256, 0, st>>>(kp, d.colx, d.coly, d.colz, d.src, d.coef, d.near_ptr,
                                                       d.near_col, ws.nearblk, ws.selfblk, H.d_perm, H.d_dense,
                                                       H.d_dense_off, ws.hm_dense);
    AFS_HIP(hipMemsetAsync(ws.hm_ctr, 0, sizeof(unsigned long long), st));
    const int64_t n_small = H.n_small, n_mid = H.n_mid, n_large = nl - H.n_small - H.n_mid;
    Hm32 h32;
    {
        const double sr = kp.s_re * kp.inv_cs, si = kp.s_im * kp.inv_cs, ks2 = sr * sr + si * si;
        h32 = Hm32{(float)sr, (float)si, (float)kp.beta, (float)kp.lam_over_mu, (float)kp.c_u,
                   (float)(ks2 > 0.0 ? 1.0 / ks2 : 0.0)};
    }
    if (n_small)
        hm_aca_kernel<64><<<(unsigned)n_small, 64, 0, st>>>(H.d_perm,
                                                             H.d_lowrank, H.d_lr_order, H.kmax, eps, ws.hm_pool,
                                                             (unsigned long long)ws.hm_pool_cap, ws.hm_ctr, ws.hm_offs,
                                                             ws.hm_rank, ws.hm_status, h32, d.col32, d.src32, d.coef32, H.d_leaf_of, H.d_leaves,
                                                             H.d_leaf_prow, H.d_lr_rp);
    if (n_mid)
        hm_aca_kernel<128><<<(unsigned)n_mid, 128, 0, st>>>(H.d_perm, H.d_lowrank, H.d_lr_order + n_small, H.kmax, eps,
                                                             ws.hm_pool, (unsigned long long)ws.hm_pool_cap, ws.hm_ctr,
                                                             ws.hm_offs, ws.hm_rank, ws.hm_status, h32, d.col32,
                                                             d.src32, d.coef32, H.d_leaf_of, H.d_leaves, H.d_leaf_prow,
                                                             H.d_lr_rp);
    if (n_large)
        hm_aca_kernel<256><<<(unsigned)n_large, 256, 0, st>>>(H.d_perm, H.d_lowrank, H.d_lr_order + n_small + n_mid,
                                                               H.kmax, eps, ws.hm_pool, (unsigned long long)ws.hm_pool_cap,
                                                               ws.hm_ctr, ws.hm_offs, ws.hm_rank, ws.hm_status, h32,
                                                               d.col32, d.src32, d.coef32, H.d_leaf_of, H.d_leaves,
                                                               H.d_leaf_prow, H.d_lr_rp);
    AFS_HIP(hipGetLastError());
    if (nl) {
        AFS_HIP(hipMemcpyAsync(ws.hm_host, ws.hm_rank, nl * sizeof(int), hipMemcpyDeviceToHost, st));
        AFS_HIP(hipMemcpyAsync(ws.hm_host + nl, ws.hm_status, nl * sizeof(int), hipMemcpyDeviceToHost, st));
    }
    AFS_HIP(hipMemcpyAsync(ws.hm_used_host, ws.hm_ctr, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    ws.hm_ok = false;  // until hmat_finish has read the ranks
}

bool hmat_finish(Problem &p, Workspace &ws, hipStream_t st) {
    const int64_t nl = (int64_t)p.hmat->lowrank.size() / 4;
    const std::vector<int64_t> &lr = p.hmat->lowrank;
    ws.hm_max_rank = 0;
    bool ok = true;
    // bytes one product streams: the dense blocks and every term's U and V (FP32 complex)
    double entries = 0.0;
    const std::vector<int64_t> &dn = p.hmat->dense;
    for (size_t d = 0; d < dn.size() / 4; ++d)
        entries += 9.0 * (double)(dn[4 * d + 1] - dn[4 * d]) * (double)(dn[4 * d + 3] - dn[4 * d + 2]);
    for (int64_t l = 0; l < nl; ++l) {
        ws.hm_max_rank = std::max(ws.hm_max_rank, ws.hm_host[l]);
        ok = ok && ws.hm_host[nl + l] == 0;
        entries += (double)ws.hm_host[l] * 3.0 * (double)((lr[4 * l + 1] - lr[4 * l]) + (lr[4 * l + 3] - lr[4 * l + 2]));
    }
    ws.hm_bytes = entries * 8.0;
    ws.hm_ok = ok;
    // the V^T x items of this build's ranks
    // up to four slots of a block per item (two for blocks wider than 1,536
    // columns): the slots of an item share one read of the block's x
    int64_t k = 0;
    for (const int32_t l : p.hmat->vt_order) {
        const int ns = hm_slots(std::min(ws.hm_host[l], p.hmat->kmax));
        const int per = 3 * (lr[4 * (int64_t)l + 3] - lr[4 * (int64_t)l + 2]) <= 1536 ? 4 : 2;
        for (int j = 0; j < ns; j += per)
            ws.hm_items_host[k++] = (l << 6) | (j << 2) | (std::min(per, ns - j) - 1);
    }
    ws.hm_n_items = k;
    if (k)
        AFS_HIP(hipMemcpyAsync(ws.hm_items, ws.hm_items_host, (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // a block that found the pool spent (status 2): the next build asks for
    // twice the pool or 1.5 x what this one requested, whichever is larger
    ws.hm_exhausted = false;
    for (int64_t l = 0; l < nl && !ok; ++l)
        ws.hm_exhausted = ws.hm_exhausted || ws.hm_host[nl + l] == 2;
    const double used = (double)*ws.hm_used_host;
    if (ws.hm_exhausted)
        ws.hm_want = std::max((size_t)(2 * ws.hm_pool_cap), (size_t)(1.5 * used));
    else
        p.hm_need = std::max(p.hm_need, used);
    return ok;
}

void hmat_apply(const Problem &p, const Workspace &ws, const double *x, double *y, hipStream_t st) {
    const HmatPlan &H = *p.hmat;
    const int64_t nl = (int64_t)H.lowrank.size() / 4, nleaf = (int64_t)H.leaves.size() / 2;
    const double2 *xv = reinterpret_cast<const double2 *>(x);
    hm_gather_kernel<<<(unsigned)((3 * H.n + 255) / 256), 256, 0, st>>>(H.n, H.d_perm, xv, ws.hm_xp);
    if (ws.hm_n_items)
        hm_vt_kernel<<<(unsigned)std::min<int64_t>(ws.hm_n_items, kVtWaves), 64, 0, st>>>(
            ws.hm_items, ws.hm_n_items, H.d_lowrank, H.kmax, ws.hm_rank, ws.hm_offs, H.d_lr_rp, ws.hm_pool, ws.hm_xp,
            ws.hm_t);
    hm_apply_kernel<<<dim3((unsigned)nleaf, kHmSplit), 64, 0, st>>>(
        H.d_leaves, H.d_leaf_ptr, H.d_leaf_item, H.d_dense, H.d_dense_off, H.d_leaf_prow, H.d_lr_rp, H.kmax, ws.hm_rank,
        ws.hm_offs, ws.hm_dense, ws.hm_pool, ws.hm_t, ws.hm_xp, H.n, ws.hm_yp);
    hm_sum_kernel<<<(unsigned)((3 * H.n + 255) / 256), 256, 0, st>>>(H.n, H.d_perm, ws.hm_yp,
                                                                      reinterpret_cast<double2 *>(y));
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
