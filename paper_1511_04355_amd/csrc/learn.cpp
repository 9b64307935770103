// Learned warm start: a multilayer perceptron trained on the solutions of the
// frequencies solved so far predicts the solution at the next one (up to a
// complex factor, which the residual-minimising start absorbs).
//
// Training rows: one per element and solved frequency; features from
// learn_features(), targets the element's three solution components divided by
// c = (||a|| / sqrt(n_tri)) e^{i arg <a, a_ref>}, a_ref the first solution, so
// that every frequency contributes targets of unit scale and consistent phase.
// After each solve: steps_per_sample Adam steps (lr 1e-3, 0.9, 0.999, 1e-8) on
// random minibatches of all rows so far (bfloat16 matrix-core products, FP32
// master weights).
#include <cmath>
#include <complex>
#include <cstring>

#include "internal.hpp"
#include "mlp.hpp"

namespace afsbem {

static void *learn_alloc(size_t bytes) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e != hipSuccess)
        throw Error{AFSBEM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    return p;
}

static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

LearnState::~LearnState() {
    for (void *q : {(void *)P, (void *)m, (void *)v, (void *)G, (void *)work, (void *)Xtr, (void *)Ttr, (void *)Xb,
                    (void *)Tb, (void *)Y, (void *)loss, (void *)idx, (void *)ref_dev, (void *)dots, (void *)dot_out})
        if (q)
            (void)hipFree(q);
    if (idx_host)
        (void)hipHostFree(idx_host);
}

void LearnState::init(const Problem &p) {
    nt = p.dev.n_tri;
    const int64_t np = shape.n_params;
    P = (float *)learn_alloc(np * 4);
    m = (float *)learn_alloc(np * 4);
    v = (float *)learn_alloc(np * 4);
    G = (float *)learn_alloc(np * 4);
    const int64_t rows_max = std::max<int64_t>(batch, nt);
    work = (float *)learn_alloc(mlp_work_floats(shape, (int)rows_max) * 4);
    Xb = (float *)learn_alloc((size_t)rows_max * kLearnFeatures * 4);
    Tb = (float *)learn_alloc((size_t)batch * kLearnOut * 4);
    Y = (float *)learn_alloc((size_t)nt * kLearnOut * 4);
    loss = (float *)learn_alloc(16);
    idx = (int32_t *)learn_alloc((size_t)steps_per_sample * batch * 4);
    ref_dev = (double *)learn_alloc((size_t)nt * 3 * 16);
    dots = (double *)learn_alloc(mdot_scratch_bytes(3 * nt, 1));
    AFS_HIP(hipMemset(dots, 0, kMdotCounterBytes));  // multi-dot arrival counters
    dot_out = (double *)learn_alloc(64);
    AFS_HIP(hipHostMalloc((void **)&idx_host, (size_t)steps_per_sample * batch * 4, hipHostMallocDefault));
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases
    std::vector<float> hp(np);
    const int64_t off[7] = {shape.oW1, shape.ob1, shape.oW2, shape.ob2, shape.oW3, shape.ob3, np};
    const int fan[6] = {shape.d_in, shape.d_in, shape.hidden, shape.hidden, shape.hidden, shape.hidden};
    uint64_t s = 12345;
    for (int q = 0; q < 6; ++q) {
        const double bnd = 1.0 / std::sqrt((double)fan[q]);
        for (int64_t k = off[q]; k < off[q + 1]; ++k)
            hp[k] = (float)((2.0 * ((splitmix(s) >> 11) * (1.0 / 9007199254740992.0)) - 1.0) * bnd);
    }
    AFS_HIP(hipMemcpy(P, hp.data(), np * 4, hipMemcpyHostToDevice));
    AFS_HIP(hipMemset(m, 0, np * 4));
    AFS_HIP(hipMemset(v, 0, np * 4));
    // box of the collocation points
    const auto &c = p.host.cen;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t e = 0; e < nt; ++e)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], c[3 * e + d]);
            hi[d] = std::max(hi[d], c[3 * e + d]);
        }
    double half = 0.0;
    for (int d = 0; d < 3; ++d) {
        box[d] = 0.5 * (lo[d] + hi[d]);
        half = std::max(half, 0.5 * (hi[d] - lo[d]));
    }
    box[3] = half > 0 ? half : 1.0;
}

void LearnState::features(const Problem &p, double sr, double si, float *X, hipStream_t st) {
    learn_features(nt, p.dev, box, (float)(sr / s_scale), (float)(si / s_scale), X, st);
}

void LearnState::add_solution(const Problem &p, double sr, double si, const double *a, hipStream_t st) {
    const int64_t N = 3 * nt;
    // ||a||^2 and <a, a_ref> on the device; only the two numbers come back
    const bool first = ref_norm == 0.0;
    if (first)
        AFS_HIP(hipMemcpyAsync(ref_dev, a, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
    vec_mdot(N, 1, a, N, a, dots, dot_out, st);
    vec_mdot(N, 1, ref_dev, N, a, dots, dot_out + 2, st);
    double hd[4];
    AFS_HIP(hipMemcpyAsync(hd, dot_out, 32, hipMemcpyDeviceToHost, st));
    AFS_HIP(hipStreamSynchronize(st));
    const double nrm2 = hd[0];
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
        return;  // nothing to learn from (a first reference is taken again next time)
    if (first)
        ref_norm = std::sqrt(nrm2);
    const std::complex<double> dot(hd[2], hd[3]);  // sum a conj(a_ref)
    const std::complex<double> ph = std::abs(dot) > 0 ? dot / std::abs(dot) : std::complex<double>(1.0, 0.0);
    const std::complex<double> c = ph * std::sqrt(nrm2 / (double)nt);
    if (rows + nt > cap) {
        const int64_t ncap = std::max<int64_t>(2 * cap, rows + 16 * nt);
        float *nx = (float *)learn_alloc((size_t)ncap * kLearnFeatures * 4);
        float *ny = (float *)learn_alloc((size_t)ncap * kLearnOut * 4);
        if (rows) {
            AFS_HIP(hipMemcpyAsync(nx, Xtr, (size_t)rows * kLearnFeatures * 4, hipMemcpyDeviceToDevice, st));
            AFS_HIP(hipMemcpyAsync(ny, Ttr, (size_t)rows * kLearnOut * 4, hipMemcpyDeviceToDevice, st));
            AFS_HIP(hipStreamSynchronize(st));
        }
        if (Xtr)
            (void)hipFree(Xtr);
        if (Ttr)
            (void)hipFree(Ttr);
        Xtr = nx;
        Ttr = ny;
        cap = ncap;
    }
    features(p, sr, si, Xtr + (size_t)rows * kLearnFeatures, st);
    learn_targets(nt, a, c.real(), c.imag(), Ttr + (size_t)rows * kLearnOut, st);
    rows += nt;
}

void LearnState::train(int steps, hipStream_t st) {
    if (rows == 0 || steps <= 0)
        return;
    steps = std::min(steps, steps_per_sample);
    const bool full = rows <= batch;
    const int B = full ? (int)rows : batch;
    if (!full) {
        // the previous copy out of the pinned index buffer must have completed
        AFS_HIP(hipStreamSynchronize(st));
        for (int64_t k = 0; k < (int64_t)steps * B; ++k)
            idx_host[k] = (int32_t)(splitmix(rng) % (uint64_t)rows);
        AFS_HIP(hipMemcpyAsync(idx, idx_host, (size_t)steps * B * 4, hipMemcpyHostToDevice, st));
    }
    for (int q = 0; q < steps; ++q) {
        const float *X = Xtr, *T = Ttr;
        if (!full) {
            gather_rows(B, kLearnFeatures, idx + (size_t)q * B, Xtr, Xb, st);
            gather_rows(B, kLearnOut, idx + (size_t)q * B, Ttr, Tb, st);
            X = Xb;
            T = Tb;
        }
        ++t;
        mlp_train_step(shape, B, P, X, T, m, v, t, 1e-3f, 0.9f, 0.999f, 1e-8f, loss, work, st);
    }
}

void LearnState::predict(const Problem &p, double sr, double si, double *x0, hipStream_t st) {
    features(p, sr, si, Xb, st);
    mlp_forward(shape, 1, (int)nt, P, Xb, Y, work, st);
    learn_unpack(nt, Y, x0, st);
}

}  // namespace afsbem
