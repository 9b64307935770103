// Cluster tree and block partition of the hierarchical far field (host).
#include <algorithm>
#include <cmath>
#include <functional>

#include "hmat.hpp"

namespace afsbem {

HmatPlan::~HmatPlan() {
    for (void *p : allocs)
        (void)hipFree(p);
}

namespace {

struct TNode {
    int64_t b, e;
    double c[3], r;
    int ch0 = -1, ch1 = -1;
};

template <class T>
T *up(HmatPlan &H, const std::vector<T> &v) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    hipError_t err = hipMalloc(&p, bytes);
    if (err != hipSuccess)
        throw Error{AFSBEM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(err)};
    H.allocs.push_back(p);
    if (!v.empty())
        AFS_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<T *>(p);
}

}  // namespace

void hmat_ensure(Problem &p, double eta) {
    if (p.hmat && p.hmat->eta == eta)
        return;
    delete p.hmat;
    p.hmat = nullptr;
    auto *H = new HmatPlan();
    try {
        hmat_build(p, eta, kHmatKmax, *H);
    } catch (...) {
        delete H;
        throw;
    }
    p.hmat = H;
}

void hmat_build(const Problem &p, double eta, int kmax, HmatPlan &H, bool upload) {
    const HostPlan &P = p.host;
    AFS_REQUIRE(P.disc == 0, AFSBEM_EINVAL, "the hierarchical far field is built for flat-element problems");
    const int64_t n = P.n_tri;
    H.eta = eta;
    H.kmax = kmax;
    H.n = n;
    H.perm.resize(n);
    for (int64_t e = 0; e < n; ++e)
        H.perm[e] = (int32_t)e;
    double hmax_all = 0.0;
    for (int64_t e = 0; e < n; ++e)
        hmax_all = std::max(hmax_all, P.hmax[e]);

    // ---- tree: recursive coordinate bisection, bounding spheres that hold
    // every element (centroid distance + longest edge)
    std::vector<TNode> nodes;
    std::function<int(int64_t, int64_t)> split = [&](int64_t b, int64_t e) -> int {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t q = b; q < e; ++q) {
            const double *c = &P.cen[3 * (size_t)H.perm[q]];
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], c[d]);
                hi[d] = std::max(hi[d], c[d]);
            }
        }
        TNode t;
        t.b = b;
        t.e = e;
        for (int d = 0; d < 3; ++d)
            t.c[d] = 0.5 * (lo[d] + hi[d]);
        t.r = 0.0;
        for (int64_t q = b; q < e; ++q) {
            const int32_t id = H.perm[q];
            const double *c = &P.cen[3 * (size_t)id];
            const double dx = c[0] - t.c[0], dy = c[1] - t.c[1], dz = c[2] - t.c[2];
            t.r = std::max(t.r, std::sqrt(dx * dx + dy * dy + dz * dz) + P.hmax[id]);
        }
        const int me = (int)nodes.size();
        nodes.push_back(t);
        if (e - b <= kLeafElems)
            return me;
        int ax = 0;
        for (int d = 1; d < 3; ++d)
            if (hi[d] - lo[d] > hi[ax] - lo[ax])
                ax = d;
        const int64_t mid = b + (e - b) / 2;
        auto key = [&](int32_t id) { return P.cen[3 * (size_t)id + ax]; };
        std::nth_element(H.perm.begin() + b, H.perm.begin() + mid, H.perm.begin() + e,
                         [&](int32_t u, int32_t w) { return key(u) < key(w) || (key(u) == key(w) && u < w); });
        const int c0 = split(b, mid);
        const int c1 = split(mid, e);
        nodes[me].ch0 = c0;
        nodes[me].ch1 = c1;
        return me;
    };
    split(0, n);
    std::vector<int64_t> pos(n);
    for (int64_t q = 0; q < n; ++q)
        pos[H.perm[q]] = q;

    // ---- block partition
    auto has_near = [&](const TNode &A, const TNode &B) {
        for (int64_t q = A.b; q < A.e; ++q) {
            const int32_t m = H.perm[q];
            for (int64_t pp = P.near_ptr[m]; pp < P.near_ptr[m + 1]; ++pp) {
                const int64_t pn = pos[P.near_col[pp]];
                if (pn >= B.b && pn < B.e)
                    return true;
            }
        }
        return false;
    };
    H.dense.clear();
    H.lowrank.clear();
    const double near_reach = p.pol.far_ratio * hmax_all;
    std::function<void(int, int)> part = [&](int a, int b) {
        const TNode &A = nodes[a], &B = nodes[b];
        const double dx = A.c[0] - B.c[0], dy = A.c[1] - B.c[1], dz = A.c[2] - B.c[2];
        const double gap = std::sqrt(dx * dx + dy * dy + dz * dz) - A.r - B.r;
        if (gap > 0.0 && std::max(A.r, B.r) <= eta * gap && (gap >= near_reach || !has_near(A, B))) {
            H.lowrank.insert(H.lowrank.end(), {A.b, A.e, B.b, B.e});
            return;
        }
        const bool la = A.ch0 < 0, lb = B.ch0 < 0;
        if (la && lb) {
            H.dense.insert(H.dense.end(), {A.b, A.e, B.b, B.e});
        } else if (la) {
            part(a, B.ch0);
            part(a, B.ch1);
        } else if (lb) {
            part(A.ch0, b);
            part(A.ch1, b);
        } else {
            part(A.ch0, B.ch0);
            part(A.ch0, B.ch1);
            part(A.ch1, B.ch0);
            part(A.ch1, B.ch1);
        }
    };
    part(0, 0);
    const int64_t nd = (int64_t)H.dense.size() / 4, nl = (int64_t)H.lowrank.size() / 4;
    H.dense_off.assign(nd + 1, 0);
    for (int64_t d = 0; d < nd; ++d)
        H.dense_off[d + 1] = H.dense_off[d] + dense_rows_padded(H.dense[4 * d + 1] - H.dense[4 * d]) * 3 *
                                                   (H.dense[4 * d + 3] - H.dense[4 * d + 2]);
    H.lr_order.clear();
    auto tier = [&](int64_t l) {
        const int64_t na = H.lowrank[4 * l + 1] - H.lowrank[4 * l], nb = H.lowrank[4 * l + 3] - H.lowrank[4 * l + 2];
        const int64_t big = na > nb ? na : nb;
        return big <= 64 ? 0 : (big <= 128 ? 1 : 2);
    };
    for (int tr = 0; tr < 3; ++tr) {
        for (int64_t l = 0; l < nl; ++l)
            if (tier(l) == tr)
                H.lr_order.push_back((int32_t)l);
        if (tr == 0)
            H.n_small = (int64_t)H.lr_order.size();
        if (tr == 1)
            H.n_mid = (int64_t)H.lr_order.size() - H.n_small;
    }

    H.vt_order.resize(nl);
    for (int64_t l = 0; l < nl; ++l)
        H.vt_order[l] = (int32_t)l;
    // width classes widest first (their long streams start early), within a
    // class by column range, so that the items in flight at a time read
    // neighbouring parts of x (from L2 rather than memory)
    auto wclass = [&](int32_t u) {
        const int64_t nb = H.lowrank[4 * (int64_t)u + 3] - H.lowrank[4 * (int64_t)u + 2];
        return nb > 256 ? 3 : (nb > 64 ? 2 : (nb > kLeafElems ? 1 : 0));
    };
    std::stable_sort(H.vt_order.begin(), H.vt_order.end(), [&](int32_t u, int32_t w) {
        const int cu = wclass(u), cw = wclass(w);
        if (cu != cw)
            return cu > cw;
        return H.lowrank[4 * (int64_t)u + 2] < H.lowrank[4 * (int64_t)w + 2];
    });

    // ---- per leaf row range: the dense blocks of its block row and every
    // low-rank block whose row range holds it (fixed order: dense, then low-rank)
    H.leaves.clear();
    std::vector<int64_t> leaf_of_start(n + 1, -1);
    for (const TNode &t : nodes)
        if (t.ch0 < 0) {
            leaf_of_start[t.b] = (int64_t)H.leaves.size() / 2;
            H.leaves.insert(H.leaves.end(), {t.b, t.e});
        }
    // leaves were pushed in tree (DFS) order, i.e. by increasing start
    const int64_t nleaf = (int64_t)H.leaves.size() / 2;
    // pool slot geometry: each leaf's padded rows, and per low-rank block
    // the place of its row cluster's first leaf and its padded row count
    H.leaf_of.assign(n, -1);
    H.leaf_prow.assign(nleaf + 1, 0);
    for (int64_t L = 0; L < nleaf; ++L) {
        for (int64_t q = H.leaves[2 * L]; q < H.leaves[2 * L + 1]; ++q)
            H.leaf_of[q] = (int32_t)L;
        H.leaf_prow[L + 1] = H.leaf_prow[L] + dense_rows_padded(H.leaves[2 * L + 1] - H.leaves[2 * L]);
    }
    H.lr_rp.assign(2 * nl, 0);
    H.lr_rows = 0;
    for (int64_t l = 0; l < nl; ++l) {
        const int32_t La = H.leaf_of[H.lowrank[4 * l]], Lb = H.leaf_of[H.lowrank[4 * l + 1] - 1];
        AFS_REQUIRE(La >= 0 && Lb >= La && H.leaves[2 * La] == H.lowrank[4 * l] &&
                        H.leaves[2 * Lb + 1] == H.lowrank[4 * l + 1],
                    AFSBEM_EINVAL, "internal: low-rank row cluster not a union of leaves");
        H.lr_rp[2 * l] = H.leaf_prow[La];
        H.lr_rp[2 * l + 1] = H.leaf_prow[Lb + 1] - H.leaf_prow[La];
        const int64_t C = 3 * (H.lowrank[4 * l + 3] - H.lowrank[4 * l + 2]);
        H.lr_rows += H.lr_rp[2 * l + 1] + C + (C & 1);
    }
    std::vector<std::vector<int32_t>> items(nleaf);
    for (int64_t d = 0; d < nd; ++d) {
        const int64_t L = leaf_of_start[H.dense[4 * d]];
        AFS_REQUIRE(L >= 0, AFSBEM_EINVAL, "internal: dense block not on a leaf");
        items[L].push_back((int32_t)d);
    }
    for (int64_t l = 0; l < nl; ++l) {
        int64_t L = leaf_of_start[H.lowrank[4 * l]];
        AFS_REQUIRE(L >= 0, AFSBEM_EINVAL, "internal: low-rank block not on a leaf boundary");
        for (; L < nleaf && H.leaves[2 * L] < H.lowrank[4 * l + 1]; ++L)
            items[L].push_back((int32_t)(-(l + 1)));
    }
    H.leaf_ptr.assign(nleaf + 1, 0);
    H.leaf_item.clear();
    for (int64_t L = 0; L < nleaf; ++L) {
        H.leaf_item.insert(H.leaf_item.end(), items[L].begin(), items[L].end());
        H.leaf_ptr[L + 1] = (int64_t)H.leaf_item.size();
    }
    AFS_REQUIRE(nd < ((int64_t)1 << 31) && nl < ((int64_t)1 << 25) && nleaf < ((int64_t)1 << 31), AFSBEM_EINVAL,
                "hierarchical partition too large");

    if (!upload)
        return;
    H.d_perm = up(H, H.perm);
    H.d_dense = up(H, H.dense);
    H.d_lowrank = up(H, H.lowrank);
    H.d_dense_off = up(H, H.dense_off);
    H.d_leaves = up(H, H.leaves);
    H.d_leaf_ptr = up(H, H.leaf_ptr);
    H.d_leaf_item = up(H, H.leaf_item);
    H.d_lr_order = up(H, H.lr_order);
    H.d_leaf_of = up(H, H.leaf_of);
    H.d_leaf_prow = up(H, H.leaf_prow);
    H.d_lr_rp = up(H, H.lr_rp);
}

}  // namespace afsbem
