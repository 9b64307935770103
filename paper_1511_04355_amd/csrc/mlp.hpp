// Multilayer perceptron for the learned warm start (see kern_mlp.hip).
#pragma once
#include "internal.hpp"

namespace afsbem {

struct MlpShape {
    int d_in, hidden, d_out;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, n_params;
    MlpShape(int d_in, int hidden, int d_out);
};

// FP32 scratch (floats) for n samples
size_t mlp_work_floats(const MlpShape &s, int n);
// mode 0: FP32 FMA; 1: bfloat16 MFMA with FP32 accumulation
void mlp_forward(const MlpShape &s, int mode, int n, const float *P, const float *X, float *Y, float *work,
                 hipStream_t st);
// gradient of mean (Y - T)^2 w.r.t. the flat parameters; loss (nullable device scalar)
void mlp_loss_grad(const MlpShape &s, int mode, int n, const float *P, const float *X, const float *T, float *G,
                   float *loss, float *work, hipStream_t st);
void mlp_adam(int64_t n, float *P, const float *G, float *m, float *v, int t, float lr, float b1, float b2, float eps,
              hipStream_t st);
// one training step in mode 1: loss gradient and the Adam update of P (m, v
// its moments, t the step count from 1); the full gradient is never stored
void mlp_train_step(const MlpShape &s, int n, float *P, const float *X, const float *T, float *m, float *v, int t,
                    float lr, float b1, float b2, float eps, float *loss, float *work, hipStream_t st);

// ----------------------------------------------------- learned warm start --
constexpr int kLearnFeatures = 32;
constexpr int kLearnHidden = 256;
constexpr int kLearnOut = 6;

void learn_features(int64_t nt, const DevicePlan &d, const double box[4], float sr, float si, float *X,
                    hipStream_t st);
void learn_targets(int64_t nt, const double *a, double cr, double ci, float *T, hipStream_t st);
void learn_unpack(int64_t nt, const float *Y, double *x0, hipStream_t st);
void gather_rows(int B, int d, const int32_t *idx, const float *src, float *dst, hipStream_t st);

// Training state of the warm-start network of one problem.
struct LearnState {
    MlpShape shape{kLearnFeatures, kLearnHidden, kLearnOut};
    float *P = nullptr, *m = nullptr, *v = nullptr, *G = nullptr, *work = nullptr;
    float *Xtr = nullptr, *Ttr = nullptr;  // training rows
    float *Xb = nullptr, *Tb = nullptr, *Y = nullptr, *loss = nullptr;
    int32_t *idx = nullptr, *idx_host = nullptr;  // minibatch rows (pinned host staging)
    int64_t rows = 0, cap = 0;
    int64_t nt = 0;
    int t = 0, batch = 8192;
    int steps_per_sample = 24;
    double box[4] = {0, 0, 0, 1};
    double s_scale = 1.0;
    double ref_norm = 0.0;    // norm of the reference solution (ref_dev) fixing the phase of the targets
    uint64_t rng = 0x9e3779b97f4a7c15ull;
    // Gate on the network query: the gain of the prediction is the factor by
    // which it lowers the starting residual of the previous solution alone;
    // after three consecutive gains below 1.3 the network is not queried for
    // the next 8 frequencies (training continues), then probed again.  After
    // kRetireAfter such closures with no gain >= 1.3 in between, the network
    // is retired for this problem: no more queries, samples or training (its
    // cost would exceed its gain on the problem's frequencies).
    static constexpr int kRetireAfter = 3;
    int low_gains = 0, skip = 0, closures = 0;
    bool retired = false;
    bool query_now() {
        if (retired)
            return false;
        if (skip > 0) {
            --skip;
            return false;
        }
        return true;
    }
    void record_gain(double g) {
        if (g >= 1.3) {
            low_gains = 0;
            closures = 0;
            return;
        }
        if (++low_gains >= 3) {
            skip = 8;
            low_gains = 0;
            if (++closures >= kRetireAfter)
                retired = true;
        }
    }
    // device scratch for the target scale (two dots of N complex entries)
    double *ref_dev = nullptr, *dots = nullptr, *dot_out = nullptr;
    ~LearnState();
    void init(const Problem &p);
    void features(const Problem &p, double sr, double si, float *X, hipStream_t st);
    void add_solution(const Problem &p, double sr, double si, const double *a, hipStream_t st);
    void train(int steps, hipStream_t st);
    void predict(const Problem &p, double sr, double si, double *x0, hipStream_t st);
};

}  // namespace afsbem
