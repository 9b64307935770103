// Batched solve: all (problem, frequency) systems of a call are packed into
// waves that fit in device memory; each wave is assembled (four library
// streams, systems round-robin) and then solved in lockstep.  Outer step for
// every system: r = b - A x with the FP64 operator, stop when ||r|| <= tol ||b||;
// otherwise one right-preconditioned GMRES cycle (up to m steps, classical
// Gram-Schmidt twice) on r with the inner operator (FP64, or the FP32 hi plane
// in the mixed path) gives the correction added to x.  One launch per step
// serves every system; converged systems are masked out; the host checks the
// number of systems still iterating every four steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batched.hpp"

namespace afsbem {

namespace {

struct Pool {
    std::vector<void *> ptrs;
    ~Pool() {
        for (void *p : ptrs)
            (void)hipFree(p);
    }
    template <class T>
    T *get(size_t count) {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            throw Error{AFSBEM_ENOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e)};
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
};

template <class T>
void up(T *d, const std::vector<T> &h, hipStream_t st) {
    if (!h.empty())
        AFS_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

struct SysRef {
    int prob, k;
    int64_t nt, N, lda;
};

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
    size_t free_b = 0, total_b = 0;
    AFS_HIP(hipMemGetInfo(&free_b, &total_b));
    const double budget = 0.6 * (double)free_b;
    const int max_b = o.batch > 1 ? o.batch : 64;
    hipStream_t as[4];
    for (auto &q : as)
        AFS_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t *q;
        ~StreamGuard() {
            for (int i = 0; i < 4; ++i)
                (void)hipStreamDestroy(q[i]);
        }
    } sg{as};
    hipEvent_t entry;
    AFS_HIP(hipEventCreate(&entry));
    AFS_HIP(hipEventRecord(entry, caller));
    int rc_all = AFSBEM_OK;
    size_t first = 0;
    while (first < all.size()) {
        // ---- pack a wave
        size_t last = first;
        double bytes = 0.0;
        while (last < all.size() && (int)(last - first) < max_b) {
            const SysRef &r = all[last];
            const double need = (double)r.N * r.lda * 16.0 + (double)r.N * (m + 12) * 16.0 +
                                (double)assembly_scratch_bytes(*probs[r.prob]) / 4.0;
            if (last > first && bytes + need > budget)
                break;
            bytes += need;
            ++last;
        }
        const int B = (int)(last - first);
        Pool pool;
        BatchDev bd;
        bd.B = B;
        bd.nvmax = m + 2;
        std::vector<BSys> hs(B);
        std::vector<int64_t> elem_off(B + 1, 0);
        int64_t Ntot = 0, part = 0;
        std::vector<int4> it128, it64, chunks;
        std::vector<int32_t> chunk_ptr(B + 1, 0);
        for (int j = 0; j < B; ++j) {
            const SysRef &r = all[first + j];
            BSys &q = hs[j];
            q.N = r.N;
            q.off = Ntot;
            q.lda = r.lda;
            const int64_t rb128 = (r.N + 255) / 256, rb64 = ((r.N + 1) / 2 + 255) / 256;
            int64_t S = (4096 + (int64_t)B * rb128 - 1) / ((int64_t)B * rb128);
            S = std::max<int64_t>(1, std::min<int64_t>(S, std::max<int64_t>(1, r.N / 32)));
            q.chunk = (r.N + S - 1) / S;
            q.S = (int)((r.N + q.chunk - 1) / q.chunk);
            q.part_off = part;
            part += (int64_t)q.S * r.N;
            for (int64_t rb = 0; rb < rb128; ++rb)
                for (int c = 0; c < q.S; ++c)
                    it128.push_back(make_int4(j, (int)rb, c, 0));
            for (int64_t rb = 0; rb < rb64; ++rb)
                for (int c = 0; c < q.S; ++c)
                    it64.push_back(make_int4(j, (int)rb, c, 0));
            chunk_ptr[j] = (int32_t)chunks.size();
            for (int64_t r0 = 0; r0 < r.N; r0 += 2048)
                chunks.push_back(make_int4(j, (int)(Ntot + r0), (int)(Ntot + std::min<int64_t>(r0 + 2048, r.N)), 0));
            Ntot += r.N;
            elem_off[j + 1] = elem_off[j] + r.nt;
        }
        chunk_ptr[B] = (int32_t)chunks.size();
        AFS_REQUIRE(Ntot < (int64_t)1 << 31, AFSBEM_EINVAL, "batched wave too large");
        bd.Ntot = Ntot;
        // ---- device memory of the wave
        std::vector<void *> Ap(B), Alo(B, nullptr);
        for (int j = 0; j < B; ++j) {
            const size_t plane = (size_t)hs[j].N * hs[j].lda * (mixed ? 8 : 16);
            Ap[j] = pool.get<char>(plane);
            if (mixed)
                Alo[j] = pool.get<char>(plane);
            hs[j].A = Ap[j];
            hs[j].A_lo = Alo[j];
        }
        double *b = pool.get<double>(2 * Ntot), *x = pool.get<double>(2 * Ntot), *r = pool.get<double>(2 * Ntot);
        double *w = pool.get<double>(2 * Ntot), *z = pool.get<double>(2 * Ntot), *tmp = pool.get<double>(2 * Ntot);
        double *V = pool.get<double>((size_t)2 * Ntot * (m + 1));
        bd.precond = pool.get<double>((size_t)18 * elem_off[B]);
        bd.partial = pool.get<double>((size_t)2 * part);
        bd.dot_partial = pool.get<double>((size_t)2 * chunks.size() * bd.nvmax);
        bd.sys = pool.get<BSys>(B);
        bd.sys_of_row = pool.get<int32_t>(Ntot);
        bd.items128 = pool.get<int4>(it128.size());
        bd.items64 = pool.get<int4>(it64.size());
        bd.n_items128 = (int64_t)it128.size();
        bd.n_items64 = (int64_t)it64.size();
        bd.chunks = pool.get<int4>(chunks.size());
        bd.n_chunks = (int64_t)chunks.size();
        bd.chunk_ptr = pool.get<int32_t>(B + 1);
        bd.H = pool.get<double>((size_t)2 * B * (m + 1) * m);
        bd.g = pool.get<double>((size_t)2 * B * (m + 1));
        bd.cs = pool.get<double>((size_t)B * m);
        bd.sn = pool.get<double>((size_t)2 * B * m);
        bd.est = pool.get<double>(B);
        bd.kdone = pool.get<int>(B);
        const int ldh = bd.nvmax;
        double *h1 = pool.get<double>((size_t)2 * B * ldh), *h2 = pool.get<double>((size_t)2 * B * ldh);
        double *nrm = pool.get<double>((size_t)2 * B), *yv = pool.get<double>((size_t)2 * B * ldh);
        double *ones = pool.get<double>((size_t)2 * B), *tolv = pool.get<double>(B);
        int *active = pool.get<int>(B), *cyc = pool.get<int>(B), *cnt = pool.get<int>(1);
        std::vector<int32_t> sor(Ntot);
        for (int j = 0; j < B; ++j)
            std::fill(sor.begin() + hs[j].off, sor.begin() + hs[j].off + hs[j].N, j);
        up(bd.sys, hs, caller);
        up(bd.sys_of_row, sor, caller);
        up(bd.items128, it128, caller);
        up(bd.items64, it64, caller);
        up(bd.chunks, chunks, caller);
        up(bd.chunk_ptr, chunk_ptr, caller);
        std::vector<double> onesh(2 * B, 0.0);
        for (int j = 0; j < B; ++j)
            onesh[2 * j] = 1.0;
        up(ones, onesh, caller);
        // ---- assembly, round-robin on four streams
        hipEvent_t ea0, ea1, es1;
        AFS_HIP(hipEventCreate(&ea0));
        AFS_HIP(hipEventCreate(&ea1));
        AFS_HIP(hipEventCreate(&es1));
        AFS_HIP(hipEventRecord(ea0, caller));
        size_t scratch_max = 0;
        for (int j = 0; j < B; ++j)
            scratch_max = std::max(scratch_max, assembly_scratch_bytes(*probs[all[first + j].prob]));
        void *scr[4];
        for (int q = 0; q < 4; ++q)
            scr[q] = pool.get<char>(scratch_max);
        std::vector<hipEvent_t> done(4);
        for (int q = 0; q < 4; ++q) {
            AFS_HIP(hipEventCreate(&done[q]));
            AFS_HIP(hipStreamWaitEvent(as[q], ea0, 0));
        }
        for (int j = 0; j < B; ++j) {
            const SysRef &rf = all[first + j];
            const Problem &P = *probs[rf.prob];
            const size_t sidx = (size_t)(s_off[rf.prob] + rf.k);
            const KernelParams kp = kernel_params(P.mat, s[2 * sidx], s[2 * sidx + 1]);
            launch_assembly(P, kp, bc[rf.prob] + 2 * (size_t)rf.k * rf.N, fmt, Ap[j], Alo[j], b + 2 * hs[j].off,
                            bd.precond + 18 * elem_off[j], scr[j % 4], as[j % 4]);
        }
        for (int q = 0; q < 4; ++q) {
            AFS_HIP(hipEventRecord(done[q], as[q]));
            AFS_HIP(hipStreamWaitEvent(caller, done[q], 0));
        }
        AFS_HIP(hipEventRecord(ea1, caller));
        hipStream_t st = caller;
        // ---- lockstep solve
        const int kin = mixed ? 1 : 0, kout = mixed ? 2 : 0;
        std::vector<int> act(B, 1), iters(B, 0), outer(B, 0);
        up(active, act, st);
        bmdot(bd, active, 1, b, b, nrm, 1, st);
        std::vector<double> hn(2 * B);
        AFS_HIP(hipMemcpyAsync(hn.data(), nrm, 16 * B, hipMemcpyDeviceToHost, st));
        AFS_HIP(hipStreamSynchronize(st));
        std::vector<double> bnorm(B), rnorm(B), tolh(B);
        for (int j = 0; j < B; ++j) {
            bnorm[j] = std::sqrt(std::max(hn[2 * j], 0.0));
            rnorm[j] = bnorm[j];
            tolh[j] = o.tol * bnorm[j];
        }
        up(tolv, tolh, st);
        AFS_HIP(hipMemsetAsync(x, 0, (size_t)16 * Ntot, st));
        AFS_HIP(hipMemcpyAsync(r, b, (size_t)16 * Ntot, hipMemcpyDeviceToDevice, st));
        std::vector<int> kd(B);
        for (int step = 0;; ++step) {
            int n_act = 0;
            for (int j = 0; j < B; ++j) {
                act[j] = (bnorm[j] > 0.0 && rnorm[j] > tolh[j] && std::isfinite(rnorm[j]) && iters[j] < o.max_iter) ? 1 : 0;
                n_act += act[j];
            }
            if (n_act == 0 || step > o.max_iter)
                break;
            up(active, act, st);
            // the cycle: V0 = r / ||r||
            bcycle_init(bd, m, active, nrm, tolv, cyc, st);
            bnormalize(bd, active, nrm, 1, r, V, st);
            for (int k = 0; k < m; ++k) {
                double *vk = V + 2 * (size_t)k * Ntot;
                bprecond(bd, cyc, vk, z, st);
                bgemv(bd, kin, cyc, z, w, st);
                bmdot(bd, cyc, k + 1, V, w, h1, ldh, st);
                bcombine(bd, cyc, k + 1, nullptr, V, h1, ldh, -1.0, w, st);
                bmdot(bd, cyc, k + 1, V, w, h2, ldh, st);
                bcombine(bd, cyc, k + 1, nullptr, V, h2, ldh, -1.0, w, st);
                bmdot(bd, cyc, 1, w, w, nrm, 1, st);
                bgivens(bd, m, k, cyc, h1, h2, ldh, nrm, tolv, st);
                if (k + 1 < m)
                    bnormalize(bd, cyc, nrm, 1, w, V + 2 * (size_t)(k + 1) * Ntot, st);
                if ((k % 4) == 3) {
                    int c = 0;
                    bcount(bd, cyc, cnt, st);
                    AFS_HIP(hipMemcpyAsync(&c, cnt, 4, hipMemcpyDeviceToHost, st));
                    AFS_HIP(hipStreamSynchronize(st));
                    if (c == 0)
                        break;
                }
            }
            // x += M^-1 V y
            bbacksolve(bd, m, active, yv, ldh, st);
            AFS_HIP(hipMemcpyAsync(kd.data(), bd.kdone, 4 * B, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipMemsetAsync(tmp, 0, (size_t)16 * Ntot, st));
            bcombine(bd, active, m, bd.kdone, V, yv, ldh, 1.0, tmp, st);
            bprecond(bd, active, tmp, z, st);
            bcombine(bd, active, 1, nullptr, z, ones, 1, 1.0, x, st);
            // outer residual with the FP64 operator
            bgemv(bd, kout, active, x, tmp, st);
            bsub(bd, active, b, tmp, r, st);
            bmdot(bd, active, 1, r, r, nrm, 1, st);
            AFS_HIP(hipMemcpyAsync(hn.data(), nrm, 16 * B, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipStreamSynchronize(st));
            for (int j = 0; j < B; ++j)
                if (act[j]) {
                    rnorm[j] = std::sqrt(std::max(hn[2 * j], 0.0));
                    iters[j] += kd[j];
                    ++outer[j];
                }
        }
        AFS_HIP(hipEventRecord(es1, st));
        // ---- outputs
        for (int j = 0; j < B; ++j) {
            const SysRef &rf = all[first + j];
            const size_t o2 = 2 * (size_t)rf.k * rf.N;
            if (a_out && a_out[rf.prob])
                AFS_HIP(hipMemcpyAsync(a_out[rf.prob] + o2, x + 2 * hs[j].off, (size_t)16 * rf.N,
                                       hipMemcpyDeviceToDevice, st));
            double *u = u_out && u_out[rf.prob] ? u_out[rf.prob] + o2 : nullptr;
            double *tt = t_out && t_out[rf.prob] ? t_out[rf.prob] + o2 : nullptr;
            if (u || tt)
                vec_split_ut(rf.nt, probs[rf.prob]->dev.kind, x + 2 * hs[j].off, bc[rf.prob] + o2, u, tt, st);
        }
        AFS_HIP(hipStreamSynchronize(st));
        float ta = 0.f, ts = 0.f;
        (void)hipEventElapsedTime(&ta, ea0, ea1);
        (void)hipEventElapsedTime(&ts, ea1, es1);
        for (int j = 0; j < B; ++j) {
            const SysRef &rf = all[first + j];
            const double rel = bnorm[j] > 0 ? rnorm[j] / bnorm[j] : 0.0;
            int status = std::isfinite(rel) ? (rel <= o.tol ? AFSBEM_OK : AFSBEM_ENOCONV) : AFSBEM_ENAN;
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
        (void)hipEventDestroy(ea0);
        (void)hipEventDestroy(ea1);
        (void)hipEventDestroy(es1);
        for (auto e : done)
            (void)hipEventDestroy(e);
        first = last;
    }
    (void)hipEventDestroy(entry);
    return rc_all;
}

}  // namespace afsbem
