// model.h -- the join cost model object behind the fsm_model handle.
#pragma once
#include <stdint.h>

#include "internal.h"

namespace fsm {

constexpr int MODEL_HIDDEN = 64;
constexpr int MODEL_OUT = 2;
constexpr int MODEL_MAX_IN = 160;   // W1 (bf16) and its gradient fit 64 KB of LDS

int64_t model_param_count(int D);

struct Model {
    int D = 0;
    int64_t n = 0;                 // parameters
    int step = 0;                  // Adam steps taken
    DBuf<float> p, m, v, g;        // float32 master copy, moments, gradient
    DBuf<uint16_t> w;              // bfloat16 working copy
    DBuf<float> scal;              // loss accumulator
    DBuf<float> bc;                // bias corrections of the current Adam step
    DBuf<int> dstep;               // Adam steps taken (device copy)
    static constexpr int GRAPH_STEPS = 8;   // train() replays a captured step from here on
    // per join size: actual / predicted quick patterns of the last level
    // sized with the current parameters (a summed expm1 of log-space
    // predictions is biased); 0 = none yet, reset by training
    mutable double calib[8] = {};

    Model(int in_dim, const float* init, uint64_t seed);
    void reset_optimizer();
    // device row-major inputs (rows x D) -> device outputs (rows x 2)
    void predict(const float* dx, int64_t rows, float* dy) const;
    // gradient of the loss into g (device); returns the loss
    float gradient(const float* dx, const float* dt, int64_t rows);
    float train(const float* dx, const float* dt, int64_t rows, int steps, float lr);
    void params(float* host) const;
};

}  // namespace fsm

struct fsm_model {
    fsm::Model m;
    int device = 0;
    fsm_model(int D, const float* init, uint64_t seed) : m(D, init, seed) {}
};
