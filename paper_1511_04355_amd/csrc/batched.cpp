// Batched solve: all (problem, frequency) systems of a call are packed into
// waves; a wave is assembled on four library streams (systems round-robin)
// and then solved in lockstep on a fifth.  Two wave slots alternate, so the
// assembly of wave w+1 (ALU-bound) runs while wave w is solved (HBM-bound).
//
// Lockstep solve, for every system of the wave: r = b - A x with the FP64
// operator; stop when ||r|| <= tol ||b||; otherwise one right-preconditioned
// GMRES cycle (up to m steps, classical Gram-Schmidt twice) on r with the
// inner operator (FP64, or the FP32 hi plane in the mixed path) gives the
// correction added to x.  One launch per step serves every system; finished
// systems are masked out; the host polls the number of systems still in the
// cycle every four steps.  Each block of four steps is captured once per wave
// as a HIP graph and replayed (the launches of a block are ~50 small kernels
// when the systems are small).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batched.hpp"

namespace afsbem {

void BatchArena::drop_graphs() {
    for (auto &kv : graphs)
        for (auto e : kv.second)
            if (e)
                (void)hipGraphExecDestroy(e);
    graphs.clear();
}

BatchArena::~BatchArena() {
    drop_graphs();
    if (base)
        (void)hipFree(base);
    for (auto &q : st_asm)
        if (q)
            (void)hipStreamDestroy(q);
    if (st_sol)
        (void)hipStreamDestroy(st_sol);
}

void BatchArena::reserve(size_t bytes) {
    if (!st_sol) {
        for (auto &q : st_asm)
            AFS_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        AFS_HIP(hipStreamCreateWithFlags(&st_sol, hipStreamNonBlocking));
    }
    if (bytes <= cap)
        return;
    if (base) {
        AFS_HIP(hipDeviceSynchronize());
        drop_graphs();
        (void)hipFree(base);
        base = nullptr;
        cap = 0;
    }
    hipError_t e = hipMalloc(&base, bytes);
    if (e != hipSuccess) {
        base = nullptr;
        throw Error{AFSBEM_ENOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e)};
    }
    cap = bytes;
}

namespace {

constexpr int kStepsPerCheck = 4;  // Arnoldi steps between host checks (one graph)

struct SysRef {
    int prob, k;
    int64_t nt, N, lda;
};

// Sub-allocation of one slot: regions aligned to 256 bytes.
struct Carve {
    char *base;
    size_t off = 0;
    template <class T>
    T *get(size_t count) {
        off = (off + 255) / 256 * 256;
        T *p = reinterpret_cast<T *>(base + off);
        off += std::max<size_t>(count * sizeof(T), 16);
        return p;
    }
};

// Everything one wave needs on the device, carved from a slot.
struct Wave {
    int first = 0, B = 0;
    BatchDev bd;
    std::vector<void *> A, Alo;
    std::vector<float *> clinv;  // cluster preconditioner inverses per system (precond 1)
    std::vector<int64_t> elem_off;
    double *b = nullptr, *x = nullptr, *r = nullptr, *w = nullptr, *z = nullptr, *tmp = nullptr, *V = nullptr;
    double *h1 = nullptr, *h2 = nullptr, *nrm = nullptr, *yv = nullptr, *ones = nullptr, *tolv = nullptr;
    int *active = nullptr, *cyc = nullptr, *cnt = nullptr;
    void *scr[4] = {nullptr, nullptr, nullptr, nullptr};
    // host copies of the metadata (kept until the wave is done)
    std::vector<BSys> hs;
    std::vector<int32_t> sor, chunk_ptr;
    std::vector<int4> it128, it64, chunks;
    std::vector<double> onesh;
    hipEvent_t asm_begin = nullptr, asm_end = nullptr;
    float t_asm = 0.f;
};

// Lays out a wave of systems all[first, first + B) in a slot starting at
// base (nullptr: only measure); returns the bytes used.
size_t layout(Wave &W, const std::vector<SysRef> &all, Problem *const *probs, int first, int B, int m, bool mixed,
              int prec, char *base) {
    W.first = first;
    W.B = B;
    BatchDev &bd = W.bd;
    bd = BatchDev();
    bd.B = B;
    bd.nvmax = m + 2;
    W.hs.assign(B, BSys{});
    W.elem_off.assign(B + 1, 0);
    W.it128.clear();
    W.it64.clear();
    W.chunks.clear();
    W.chunk_ptr.assign(B + 1, 0);
    int64_t Ntot = 0, part = 0;
    size_t scratch_max = 0;
    for (int j = 0; j < B; ++j) {
        const SysRef &r = all[first + j];
        BSys &q = W.hs[j];
        q.N = r.N;
        q.off = Ntot;
        q.lda = r.lda;
        const int64_t rb128 = (r.N + 255) / 256, rb64 = ((r.N + 1) / 2 + 255) / 256;
        // split the columns so that the wave offers about 4096 work-groups
        int64_t S = (4096 + (int64_t)B * rb128 - 1) / ((int64_t)B * rb128);
        S = std::max<int64_t>(1, std::min<int64_t>(S, std::max<int64_t>(1, r.N / 64)));
        q.chunk = (r.N + S - 1) / S;
        q.S = (int)((r.N + q.chunk - 1) / q.chunk);
        q.part_off = part;
        part += (int64_t)q.S * r.N;
        for (int64_t rb = 0; rb < rb128; ++rb)
            for (int c = 0; c < q.S; ++c)
                W.it128.push_back(make_int4(j, (int)rb, c, 0));
        for (int64_t rb = 0; rb < rb64; ++rb)
            for (int c = 0; c < q.S; ++c)
                W.it64.push_back(make_int4(j, (int)rb, c, 0));
        W.chunk_ptr[j] = (int32_t)W.chunks.size();
        for (int64_t r0 = 0; r0 < r.N; r0 += 2048)
            W.chunks.push_back(
                make_int4(j, (int)(Ntot + r0), (int)(Ntot + std::min<int64_t>(r0 + 2048, r.N)), 0));
        Ntot += r.N;
        W.elem_off[j + 1] = W.elem_off[j] + r.nt;
        scratch_max = std::max(scratch_max, assembly_scratch_bytes(*probs[r.prob]));
    }
    W.chunk_ptr[B] = (int32_t)W.chunks.size();
    AFS_REQUIRE(Ntot < ((int64_t)1 << 31), AFSBEM_EINVAL, "batched wave too large");
    bd.Ntot = Ntot;
    Carve c{base};
    W.A.assign(B, nullptr);
    W.Alo.assign(B, nullptr);
    for (int j = 0; j < B; ++j) {
        const size_t plane = (size_t)W.hs[j].N * W.hs[j].lda * (mixed ? 8 : 16);
        W.A[j] = c.get<char>(plane);
        if (mixed)
            W.Alo[j] = c.get<char>(plane);
        W.hs[j].A = W.A[j];
        W.hs[j].A_lo = W.Alo[j];
    }
    const int ldh = bd.nvmax;
    W.b = c.get<double>(2 * Ntot);
    W.x = c.get<double>(2 * Ntot);
    W.r = c.get<double>(2 * Ntot);
    W.w = c.get<double>(2 * Ntot);
    W.z = c.get<double>(2 * Ntot);
    W.tmp = c.get<double>(2 * Ntot);
    W.V = c.get<double>((size_t)2 * Ntot * (m + 1));
    bd.precond = c.get<double>((size_t)18 * W.elem_off[B]);
    bd.partial = c.get<double>((size_t)2 * part);
    bd.dot_partial = c.get<double>((size_t)2 * W.chunks.size() * bd.nvmax);
    bd.sys = c.get<BSys>(B);
    bd.sys_of_row = c.get<int32_t>(Ntot);
    bd.items128 = c.get<int4>(W.it128.size());
    bd.items64 = c.get<int4>(W.it64.size());
    bd.n_items128 = (int64_t)W.it128.size();
    bd.n_items64 = (int64_t)W.it64.size();
    bd.chunks = c.get<int4>(W.chunks.size());
    bd.n_chunks = (int64_t)W.chunks.size();
    bd.chunk_ptr = c.get<int32_t>(B + 1);
    bd.H = c.get<double>((size_t)2 * B * (m + 1) * m);
    bd.g = c.get<double>((size_t)2 * B * (m + 1));
    bd.cs = c.get<double>((size_t)B * m);
    bd.sn = c.get<double>((size_t)2 * B * m);
    bd.est = c.get<double>(B);
    bd.kdone = c.get<int>(B);
    W.h1 = c.get<double>((size_t)2 * B * ldh);
    W.h2 = c.get<double>((size_t)2 * B * ldh);
    W.nrm = c.get<double>((size_t)2 * B);
    W.yv = c.get<double>((size_t)2 * B * ldh);
    W.ones = c.get<double>((size_t)2 * B);
    W.tolv = c.get<double>(B);
    W.active = c.get<int>(B);
    W.cyc = c.get<int>(B);
    W.cnt = c.get<int>(1);
    W.clinv.assign(B, nullptr);
    if (prec == 1)
        for (int j = 0; j < B; ++j)
            W.clinv[j] = c.get<float>((size_t)std::max<int64_t>(probs[all[first + j].prob]->dev.n_clusters, 1) *
                                      kClusterDim * kClusterDim * 2);
    for (auto &s : W.scr)
        s = c.get<char>(scratch_max);
    return c.off + 256;
}

size_t system_bytes(const SysRef &r, int m, int prec) {
    // matrix (16 B per entry in both formats), vectors and basis, blocks, and
    // the cluster inverses (kClusterDim^2 complex64 per cluster; a split cell
    // leaves clusters of more than kClusterElems / 2 >= 24 elements, so
    // nt/24 + 2 bounds their count)
    return (size_t)r.N * r.lda * 16 + (size_t)r.N * (m + 8) * 16 + (size_t)r.nt * 144 +
           (prec == 1 ? (size_t)(r.nt / 24 + 2) * kClusterDim * kClusterDim * 8 : 0);
}

template <class T>
void up(T *d, const std::vector<T> &h, hipStream_t st) {
    if (!h.empty())
        AFS_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

}  // namespace

int solve_batched(int n_prob, Problem *const *probs, const int32_t *n_s, const double *s, const double *const *bc,
                  double *const *a_out, double *const *u_out, double *const *t_out, const afsbem_solve_opts &o,
                  afsbem_solve_stats *stats, hipStream_t caller) {
    const bool mixed = o.precision == AFSBEM_PREC_MIXED;
    const int fmt = mixed ? AFSBEM_FMT_SPLIT : AFSBEM_FMT_C128;
    const int m = o.restart;
    std::vector<SysRef> all;
    std::vector<int64_t> s_off(n_prob + 1, 0);
    for (int p = 0; p < n_prob; ++p) {
        s_off[p + 1] = s_off[p] + n_s[p];
        for (int k = 0; k < n_s[p]; ++k) {
            const int64_t nt = probs[p]->dev.n_tri, N = 3 * nt;
            all.push_back({p, k, nt, N, (N + 63) / 64 * 64});
        }
    }
    if (all.empty())
        return AFSBEM_OK;
    Problem &owner = *probs[0];
    if (!owner.barena)
        owner.barena = new BatchArena();
    BatchArena &ar = *owner.barena;
    // slot budget: a few GiB keep the HBM busy; never more than a share of
    // the free memory; at least the largest single system
    size_t free_b = 0, total_b = 0;
    AFS_HIP(hipMemGetInfo(&free_b, &total_b));
    const double avail = (double)free_b + (double)ar.cap;
    double slot_budget = std::min(0.3 * avail, 16.0 * (1 << 30));
    const int max_b = o.batch >= 1 ? o.batch : 64;
    // ---- pack the waves
    std::vector<std::pair<int, int>> waves;
    for (size_t f = 0; f < all.size();) {
        size_t l = f;
        double bytes = 0.0;
        while (l < all.size() && (int)(l - f) < max_b) {
            const double need = (double)system_bytes(all[l], m, o.precond);
            if (l > f && bytes + need > slot_budget)
                break;
            bytes += need;
            ++l;
        }
        waves.push_back({(int)f, (int)(l - f)});
        f = l;
    }
    const int n_waves = (int)waves.size();
    Wave slots[2];
    size_t slot_bytes = 0;
    for (auto &wv : waves)
        slot_bytes =
            std::max(slot_bytes, layout(slots[0], all, probs, wv.first, wv.second, m, mixed, o.precond, nullptr));
    slot_bytes = (slot_bytes + 4095) / 4096 * 4096;
    ar.reserve(slot_bytes * (n_waves > 1 ? 2 : 1));
    char *slot_base[2] = {static_cast<char *>(ar.base), static_cast<char *>(ar.base) + (n_waves > 1 ? slot_bytes : 0)};
    hipStream_t st = ar.st_sol;
    hipEvent_t entry, fin;
    AFS_HIP(hipEventCreate(&entry));
    AFS_HIP(hipEventCreateWithFlags(&fin, hipEventDisableTiming));
    for (auto &W : slots) {
        AFS_HIP(hipEventCreate(&W.asm_begin));
        AFS_HIP(hipEventCreate(&W.asm_end));
    }
    struct EvGuard {
        hipEvent_t *e0, *e1;
        Wave *w;
        ~EvGuard() {
            (void)hipEventDestroy(*e0);
            (void)hipEventDestroy(*e1);
            for (int i = 0; i < 2; ++i) {
                (void)hipEventDestroy(w[i].asm_begin);
                (void)hipEventDestroy(w[i].asm_end);
            }
        }
    } eg{&entry, &fin, slots};
    AFS_HIP(hipEventRecord(entry, caller));
    for (auto q : ar.st_asm)
        AFS_HIP(hipStreamWaitEvent(q, entry, 0));
    AFS_HIP(hipStreamWaitEvent(st, entry, 0));

    // launches the assembly of wave wi into its slot
    auto assemble = [&](int wi) {
        Wave &W = slots[wi & 1];
        layout(W, all, probs, waves[wi].first, waves[wi].second, m, mixed, o.precond, slot_base[wi & 1]);
        // every assembly stream must be past the previous use of this slot:
        // the host only gets here after that wave's solve has completed
        AFS_HIP(hipEventRecord(W.asm_begin, ar.st_asm[0]));
        for (int q = 1; q < 4; ++q)
            AFS_HIP(hipStreamWaitEvent(ar.st_asm[q], W.asm_begin, 0));
        for (int j = 0; j < W.B; ++j) {
            const SysRef &rf = all[W.first + j];
            const Problem &P = *probs[rf.prob];
            const size_t sidx = (size_t)(s_off[rf.prob] + rf.k);
            const KernelParams kp = kernel_params(P.mat, s[2 * sidx], s[2 * sidx + 1]);
            launch_assembly(P, kp, bc[rf.prob] + 2 * (size_t)rf.k * rf.N, fmt, W.A[j], W.Alo[j],
                            W.b + 2 * W.hs[j].off, W.bd.precond + 18 * W.elem_off[j], W.scr[j % 4],
                            ar.st_asm[j % 4]);
            if (o.precond == 1)
                cluster_inverse(P.dev, fmt, W.A[j], W.Alo[j], W.clinv[j], ar.st_asm[j % 4]);
        }
        for (int q = 1; q < 4; ++q) {
            hipEvent_t e;
            AFS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            AFS_HIP(hipEventRecord(e, ar.st_asm[q]));
            AFS_HIP(hipStreamWaitEvent(ar.st_asm[0], e, 0));
            (void)hipEventDestroy(e);
        }
        AFS_HIP(hipEventRecord(W.asm_end, ar.st_asm[0]));
    };

    int rc_all = AFSBEM_OK;
    const int kin = mixed ? 1 : 0, kout = mixed ? 2 : 0;
    const bool use_graphs = o.no_graph == 0;
    assemble(0);
    for (int wi = 0; wi < n_waves; ++wi) {
        Wave &W = slots[wi & 1];
        if (wi + 1 < n_waves)
            assemble(wi + 1);  // overlaps the solve below
        const int B = W.B;
        BatchDev &bd = W.bd;
        const int ldh = bd.nvmax;
        hipEvent_t s0, s1;
        AFS_HIP(hipEventCreate(&s0));
        AFS_HIP(hipEventCreate(&s1));
        // metadata, then wait for the wave's assembly
        W.sor.resize(bd.Ntot);
        for (int j = 0; j < B; ++j)
            std::fill(W.sor.begin() + W.hs[j].off, W.sor.begin() + W.hs[j].off + W.hs[j].N, j);
        W.onesh.assign(2 * B, 0.0);
        for (int j = 0; j < B; ++j)
            W.onesh[2 * j] = 1.0;
        up(bd.sys, W.hs, st);
        up(bd.sys_of_row, W.sor, st);
        up(bd.items128, W.it128, st);
        up(bd.items64, W.it64, st);
        up(bd.chunks, W.chunks, st);
        up(bd.chunk_ptr, W.chunk_ptr, st);
        up(W.ones, W.onesh, st);
        AFS_HIP(hipStreamWaitEvent(st, W.asm_end, 0));
        AFS_HIP(hipEventRecord(s0, st));
        // z = M^-1 v for the systems flagged in mask (point blocks), or for all
        // systems (clusters: one launch per system; unflagged rows are unused)
        auto apply_prec = [&](const int *mask, const double *v, double *z) {
            if (o.precond == 1) {
                for (int j = 0; j < B; ++j)
                    cluster_apply(probs[all[W.first + j].prob]->dev, W.clinv[j], v + 2 * W.hs[j].off,
                                  z + 2 * W.hs[j].off, st);
            } else {
                bprecond(bd, mask, v, z, st);
            }
        };
        // Arnoldi steps k0 .. k0+3 of the current cycle for every system still
        // in it, then the count of those systems (W.cnt).  With graphs on, each
        // such block is captured once per wave and replayed: its kernel
        // arguments depend only on the wave's buffers and k.
        auto arnoldi_steps = [&](int k0) {
            const int k1 = std::min(m, k0 + kStepsPerCheck);
            for (int k = k0; k < k1; ++k) {
                double *vk = W.V + 2 * (size_t)k * bd.Ntot;
                apply_prec(W.cyc, vk, W.z);
                bgemv(bd, kin, W.cyc, W.z, W.w, st);
                bmdot(bd, W.cyc, k + 1, W.V, W.w, W.h1, ldh, st);
                bcombine(bd, W.cyc, k + 1, nullptr, W.V, W.h1, ldh, -1.0, W.w, st);
                bmdot(bd, W.cyc, k + 1, W.V, W.w, W.h2, ldh, st);
                bcombine(bd, W.cyc, k + 1, nullptr, W.V, W.h2, ldh, -1.0, W.w, st);
                bmdot(bd, W.cyc, 1, W.w, W.w, W.nrm, 1, st);
                bgivens(bd, m, k, W.cyc, W.h1, W.h2, ldh, W.nrm, W.tolv, st);
                if (k + 1 < m)
                    bnormalize(bd, W.cyc, W.nrm, 1, W.w, W.V + 2 * (size_t)(k + 1) * bd.Ntot, st);
            }
            bcount(bd, W.cyc, W.cnt, st);
        };
        // graph cache key: everything the captured kernel arguments depend on
        std::vector<int64_t> gkey = {(int64_t)(wi & 1), (int64_t)(intptr_t)slot_base[wi & 1], B, bd.Ntot, m, kin,
                                     bd.n_items128, bd.n_items64, bd.n_chunks, o.precond};
        for (int j = 0; o.precond == 1 && j < B; ++j)  // the cluster launches read each problem's plan
            gkey.push_back((int64_t)(intptr_t)&probs[all[W.first + j].prob]->dev);
        for (int j = 0; j < B; ++j) {
            gkey.push_back(W.hs[j].N);
            gkey.push_back(W.hs[j].S);
        }
        if (ar.graphs.size() >= 64 && !ar.graphs.count(gkey))
            ar.drop_graphs();  // bound the cache; layouts rarely repeat beyond a few
        std::vector<hipGraphExec_t> &graphs = ar.graphs[gkey];
        if (graphs.empty())
            graphs.assign((m + kStepsPerCheck - 1) / kStepsPerCheck, nullptr);
        std::vector<int> act(B, 1), iters(B, 0), outer(B, 0), kd(B);
        up(W.active, act, st);
        bmdot(bd, W.active, 1, W.b, W.b, W.nrm, 1, st);
        std::vector<double> hn(2 * B);
        AFS_HIP(hipMemcpyAsync(hn.data(), W.nrm, 16 * B, hipMemcpyDeviceToHost, st));
        AFS_HIP(hipStreamSynchronize(st));
        std::vector<double> bnorm(B), rnorm(B), tolh(B);
        for (int j = 0; j < B; ++j) {
            bnorm[j] = std::sqrt(std::max(hn[2 * j], 0.0));
            rnorm[j] = bnorm[j];
            tolh[j] = o.tol * bnorm[j];
        }
        up(W.tolv, tolh, st);
        AFS_HIP(hipMemsetAsync(W.x, 0, (size_t)16 * bd.Ntot, st));
        AFS_HIP(hipMemcpyAsync(W.r, W.b, (size_t)16 * bd.Ntot, hipMemcpyDeviceToDevice, st));
        for (int step = 0;; ++step) {
            int n_act = 0;
            for (int j = 0; j < B; ++j) {
                act[j] = (bnorm[j] > 0.0 && rnorm[j] > tolh[j] && std::isfinite(rnorm[j]) && iters[j] < o.max_iter)
                             ? 1
                             : 0;
                n_act += act[j];
            }
            if (n_act == 0 || step > o.max_iter)
                break;
            up(W.active, act, st);
            bcycle_init(bd, m, W.active, W.nrm, W.tolv, W.cyc, st);
            bnormalize(bd, W.active, W.nrm, 1, W.r, W.V, st);
            for (int k0 = 0; k0 < m; k0 += kStepsPerCheck) {
                const int blk = k0 / kStepsPerCheck;
                if (use_graphs) {
                    if (!graphs[blk]) {
                        hipGraph_t g = nullptr;
                        AFS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                        try {
                            arnoldi_steps(k0);
                        } catch (...) {
                            (void)hipStreamEndCapture(st, &g);
                            if (g)
                                (void)hipGraphDestroy(g);
                            throw;
                        }
                        AFS_HIP(hipStreamEndCapture(st, &g));
                        hipGraphExec_t ex = nullptr;
                        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                        (void)hipGraphDestroy(g);
                        AFS_HIP(e);
                        graphs[blk] = ex;
                    }
                    AFS_HIP(hipGraphLaunch(graphs[blk], st));
                } else {
                    arnoldi_steps(k0);
                }
                int cnum = 0;
                AFS_HIP(hipMemcpyAsync(&cnum, W.cnt, 4, hipMemcpyDeviceToHost, st));
                AFS_HIP(hipStreamSynchronize(st));
                if (cnum == 0)
                    break;
            }
            // x += M^-1 V y
            bbacksolve(bd, m, W.active, W.yv, ldh, st);
            AFS_HIP(hipMemcpyAsync(kd.data(), bd.kdone, 4 * B, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipMemsetAsync(W.tmp, 0, (size_t)16 * bd.Ntot, st));
            bcombine(bd, W.active, m, bd.kdone, W.V, W.yv, ldh, 1.0, W.tmp, st);
            apply_prec(W.active, W.tmp, W.z);
            bcombine(bd, W.active, 1, nullptr, W.z, W.ones, 1, 1.0, W.x, st);
            // the true residual with the FP64 operator
            bgemv(bd, kout, W.active, W.x, W.tmp, st);
            bsub(bd, W.active, W.b, W.tmp, W.r, st);
            bmdot(bd, W.active, 1, W.r, W.r, W.nrm, 1, st);
            AFS_HIP(hipMemcpyAsync(hn.data(), W.nrm, 16 * B, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipStreamSynchronize(st));
            for (int j = 0; j < B; ++j)
                if (act[j]) {
                    rnorm[j] = std::sqrt(std::max(hn[2 * j], 0.0));
                    iters[j] += kd[j];
                    ++outer[j];
                }
        }
        // ---- outputs
        for (int j = 0; j < B; ++j) {
            const SysRef &rf = all[W.first + j];
            const size_t o2 = 2 * (size_t)rf.k * rf.N;
            const double *xj = W.x + 2 * W.hs[j].off;
            if (a_out && a_out[rf.prob])
                AFS_HIP(hipMemcpyAsync(a_out[rf.prob] + o2, xj, (size_t)16 * rf.N, hipMemcpyDeviceToDevice, st));
            double *u = u_out && u_out[rf.prob] ? u_out[rf.prob] + o2 : nullptr;
            double *tt = t_out && t_out[rf.prob] ? t_out[rf.prob] + o2 : nullptr;
            if (u || tt)
                vec_split_ut(rf.nt, probs[rf.prob]->dev.kind, xj, bc[rf.prob] + o2, u, tt, st);
        }
        AFS_HIP(hipEventRecord(s1, st));
        AFS_HIP(hipStreamSynchronize(st));
        float ta = 0.f, ts = 0.f;
        (void)hipEventElapsedTime(&ta, W.asm_begin, W.asm_end);
        (void)hipEventElapsedTime(&ts, s0, s1);
        (void)hipEventDestroy(s0);
        (void)hipEventDestroy(s1);
        for (int j = 0; j < B; ++j) {
            const SysRef &rf = all[W.first + j];
            const double rel = bnorm[j] > 0 ? rnorm[j] / bnorm[j] : 0.0;
            const int status = std::isfinite(rel) ? (rel <= o.tol ? AFSBEM_OK : AFSBEM_ENOCONV) : AFSBEM_ENAN;
            if (status != AFSBEM_OK && rc_all == AFSBEM_OK)
                rc_all = status;
            if (stats) {
                afsbem_solve_stats &S = stats[s_off[rf.prob] + rf.k];
                std::memset(&S, 0, sizeof S);
                S.iters = iters[j];
                S.refine_steps = outer[j];
                S.status = status;
                S.rel_res_fp64 = rel;
                S.t_assemble_ms = ta / B;
                S.t_solve_ms = ts / B;
                S.rel_res_start = 1.0;
            }
        }
    }
    AFS_HIP(hipEventRecord(fin, st));
    AFS_HIP(hipStreamWaitEvent(caller, fin, 0));
    return rc_all;
}

}  // namespace afsbem
