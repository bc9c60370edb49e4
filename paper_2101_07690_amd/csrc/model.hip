// model.hip -- the join cost model: a two-layer perceptron (D inputs, 64
// ReLU hidden units, 2 outputs) with bfloat16 weights and float32
// accumulation, trained on the device by full-batch Adam (Kingma and Ba,
// 2015, Algorithm 1) on float32 master weights.
//
// Parameter layout (float32 master copy and bfloat16 working copy): W1 (D x
// 64, row-major), b1 (64), W2 (64 x 2, row-major), b2 (2).  Loss over B rows:
// sum((y - t)^2) / (2 B).  The forward/backward kernel runs one wavefront per
// row, lane j = hidden unit j; W1 is staged in LDS as bfloat16 and dW1 is
// accumulated per block in LDS, then added to the global gradient.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "model.h"

namespace fsm {
namespace {

constexpr int TPB_M = 256;

__device__ __forceinline__ float bf_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f_to_bf(float f) {
    const __hip_bfloat16 b = __float2bfloat16(f);   // round to nearest even
    uint16_t r;
    memcpy(&r, &b, sizeof(r));
    return r;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

struct FwdArgs {
    const uint16_t* w;   // bfloat16 parameters
    int D;
    const float* x;      // rows x D
    const float* t;      // rows x 2 (training) or null
    int64_t rows;
    float inv_b;         // 1 / B
    float* y;            // rows x 2 predictions, or null
    float* grad;         // nparams, accumulated (training), or null
    float* loss;         // sum of squared errors (training), or null
};

// Forward (and, with a.grad, backward) over all rows.
__global__ __launch_bounds__(TPB_M) void k_mlp(FwdArgs a) {
    extern __shared__ unsigned char smem[];
    const int D = a.D;
    uint16_t* sw1 = reinterpret_cast<uint16_t*>(smem);                     // D*64 bf16
    float* sg1 = reinterpret_cast<float*>(smem + ((size_t)D * MODEL_HIDDEN * 2 + 15) / 16 * 16);
    const int j = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < D * MODEL_HIDDEN; i += TPB_M) {
        sw1[i] = a.w[i];
        if (a.grad) sg1[i] = 0.0f;
    }
    __syncthreads();
    const uint16_t* w = a.w;
    const float b1 = bf_to_f(w[D * MODEL_HIDDEN + j]);
    const float w20 = bf_to_f(w[D * MODEL_HIDDEN + MODEL_HIDDEN + 2 * j]);
    const float w21 = bf_to_f(w[D * MODEL_HIDDEN + MODEL_HIDDEN + 2 * j + 1]);
    const float b20 = bf_to_f(w[D * MODEL_HIDDEN + 3 * MODEL_HIDDEN]);
    const float b21 = bf_to_f(w[D * MODEL_HIDDEN + 3 * MODEL_HIDDEN + 1]);
    float gb1 = 0.f, gw20 = 0.f, gw21 = 0.f, gb20 = 0.f, gb21 = 0.f, sse = 0.f;
    const int64_t stride = (int64_t)gridDim.x * (TPB_M / 64);
    for (int64_t r = (int64_t)blockIdx.x * (TPB_M / 64) + wave; r < a.rows; r += stride) {
        const float* xr = a.x + r * D;
        float z = b1;
        for (int d = 0; d < D; ++d) z += xr[d] * bf_to_f(sw1[d * MODEL_HIDDEN + j]);
        const float h = z > 0.f ? z : 0.f;
        const float y0 = wave_sum_f(h * w20) + b20;
        const float y1 = wave_sum_f(h * w21) + b21;
        if (a.y && j == 0) {
            a.y[2 * r] = y0;
            a.y[2 * r + 1] = y1;
        }
        if (!a.grad) continue;
        const float e0 = y0 - a.t[2 * r], e1 = y1 - a.t[2 * r + 1];
        sse += e0 * e0 + e1 * e1;
        const float d0 = e0 * a.inv_b, d1 = e1 * a.inv_b;
        gw20 += h * d0;
        gw21 += h * d1;
        gb20 += d0;
        gb21 += d1;
        const float dz = z > 0.f ? d0 * w20 + d1 * w21 : 0.f;
        gb1 += dz;
        if (dz != 0.f)
            for (int d = 0; d < D; ++d) atomicAdd(&sg1[d * MODEL_HIDDEN + j], xr[d] * dz);
    }
    if (!a.grad) return;
    __syncthreads();
    for (int i = threadIdx.x; i < D * MODEL_HIDDEN; i += TPB_M)
        if (sg1[i] != 0.f) atomicAdd(&a.grad[i], sg1[i]);
    float* g = a.grad + D * MODEL_HIDDEN;
    atomicAdd(&g[j], gb1);
    atomicAdd(&g[MODEL_HIDDEN + 2 * j], gw20);
    atomicAdd(&g[MODEL_HIDDEN + 2 * j + 1], gw21);
    if (j == 0) {
        atomicAdd(&g[3 * MODEL_HIDDEN], gb20);
        atomicAdd(&g[3 * MODEL_HIDDEN + 1], gb21);
        if (a.loss) atomicAdd(a.loss, sse);
    }
}

struct AdamArgs {
    float* p;
    float* m;
    float* v;
    const float* g;
    uint16_t* w;
    int64_t n;
    float lr, beta1, beta2, eps;
    const float* bc;   // device: 1 - beta1^step, 1 - beta2^step
};

// Advance the device step counter and its bias corrections (one thread),
// so that a captured Adam step replays with identical arguments.
__global__ void k_adam_step(int* step, float beta1, float beta2, float* bc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int s = *step + 1;
        *step = s;
        bc[0] = (float)(1.0 - pow((double)beta1, (double)s));
        bc[1] = (float)(1.0 - pow((double)beta2, (double)s));
    }
}

__global__ void k_adam(AdamArgs a) {
    const float bc1 = a.bc[0], bc2 = a.bc[1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float g = a.g[i];
        const float m = a.beta1 * a.m[i] + (1.f - a.beta1) * g;
        const float v = a.beta2 * a.v[i] + (1.f - a.beta2) * g * g;
        a.m[i] = m;
        a.v[i] = v;
        const float p = a.p[i] - a.lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
        a.p[i] = p;
        a.w[i] = f_to_bf(p);
    }
}

__global__ void k_to_bf16(const float* p, uint16_t* w, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = f_to_bf(p[i]);
}

__global__ void k_zero_f32(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

size_t lds_bytes(int D, bool grad) {
    const size_t w = ((size_t)D * MODEL_HIDDEN * 2 + 15) / 16 * 16;
    return w + (grad ? (size_t)D * MODEL_HIDDEN * 4 : 0);
}

unsigned model_grid(int64_t rows) {
    int64_t g = (rows + TPB_M / 64 - 1) / (TPB_M / 64);
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// splitmix64 (Steele, Lea and Flood, 2014): the library's own initial weights
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

int64_t model_param_count(int D) {
    return (int64_t)D * MODEL_HIDDEN + MODEL_HIDDEN + MODEL_HIDDEN * MODEL_OUT + MODEL_OUT;
}

Model::Model(int in_dim, const float* init, uint64_t seed) : D(in_dim) {
    n = model_param_count(D);
    std::vector<float> h((size_t)n);
    if (init) {
        memcpy(h.data(), init, sizeof(float) * (size_t)n);
    } else {
        // uniform in +-1/sqrt(fan_in) per layer, zero biases
        uint64_t s = seed;
        auto uni = [&](float bound) {
            const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
            return (float)((2.0 * u - 1.0) * bound);
        };
        size_t o = 0;
        for (int i = 0; i < D * MODEL_HIDDEN; ++i) h[o++] = uni(1.0f / std::sqrt((float)D));
        for (int i = 0; i < MODEL_HIDDEN; ++i) h[o++] = 0.f;
        for (int i = 0; i < MODEL_HIDDEN * MODEL_OUT; ++i)
            h[o++] = uni(1.0f / std::sqrt((float)MODEL_HIDDEN));
        for (int i = 0; i < MODEL_OUT; ++i) h[o++] = 0.f;
    }
    p.alloc((size_t)n);
    m.alloc((size_t)n);
    v.alloc((size_t)n);
    g.alloc((size_t)n);
    w.alloc((size_t)n);
    scal.alloc(1);
    bc.alloc(2);
    dstep.alloc(1);
    to_device(p.p, h.data(), (size_t)n);
    reset_optimizer();
    hipStream_t st = stream();
    k_to_bf16<<<grid_for(n, 256), 256, 0, st>>>(p.p, w.p, n);
    FSM_LAUNCH_CHECK();
    FSM_HIP(hipStreamSynchronize(st));
}

void Model::reset_optimizer() {
    hipStream_t st = stream();
    k_zero_f32<<<grid_for(n, 256), 256, 0, st>>>(m.p, n);
    k_zero_f32<<<grid_for(n, 256), 256, 0, st>>>(v.p, n);
    k_zero_f32<<<1, 64, 0, st>>>(reinterpret_cast<float*>(dstep.p), 1);   // int 0
    FSM_LAUNCH_CHECK();
    step = 0;
}

void Model::predict(const float* dx, int64_t rows, float* dy) const {
    if (rows <= 0) return;
    FwdArgs a{w.p, D, dx, nullptr, rows, 0.f, dy, nullptr, nullptr};
    k_mlp<<<model_grid(rows), TPB_M, lds_bytes(D, false), stream()>>>(a);
    FSM_LAUNCH_CHECK();
}

float Model::gradient(const float* dx, const float* dt, int64_t rows) {
    hipStream_t st = stream();
    k_zero_f32<<<grid_for(n, 256), 256, 0, st>>>(g.p, n);
    k_zero_f32<<<1, 64, 0, st>>>(scal.p, 1);
    FSM_LAUNCH_CHECK();
    if (rows > 0) {
        FwdArgs a{w.p, D, dx, dt, rows, 1.0f / (float)rows, nullptr, g.p, scal.p};
        k_mlp<<<model_grid(rows), TPB_M, lds_bytes(D, true), st>>>(a);
        FSM_LAUNCH_CHECK();
    }
    return scalar_to_host(scal.p) / (2.0f * (float)(rows > 0 ? rows : 1));
}

namespace {
// Resources of one captured training loop, released on every exit path.
struct Capture {
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Capture() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev) (void)hipEventDestroy(ev);
        if (cs) (void)hipStreamDestroy(cs);
    }
};
}  // namespace

// Full-batch Adam steps; returns the loss measured in the last step's
// forward pass (before its update).  A run of GRAPH_STEPS or more steps is
// launch-bound (five small launches per step): one step is captured into a
// HIP graph on a stream of its own, ordered after the library stream, and
// replayed; shorter runs launch the same sequence directly.
float Model::train(const float* dx, const float* dt, int64_t rows, int steps, float lr) {
    for (double& c : calib) c = 0.0;   // calibration belongs to the old parameters
    hipStream_t st = stream();
    if (steps <= 0) {
        FSM_HIP(hipStreamSynchronize(st));
        return 0.f;
    }
    const float beta1 = 0.9f, beta2 = 0.999f;
    auto enqueue = [&](hipStream_t s) {
        k_zero_f32<<<grid_for(n, 256), 256, 0, s>>>(g.p, n);
        k_zero_f32<<<1, 64, 0, s>>>(scal.p, 1);
        if (rows > 0) {
            FwdArgs a{w.p, D, dx, dt, rows, 1.0f / (float)rows, nullptr, g.p, scal.p};
            k_mlp<<<model_grid(rows), TPB_M, lds_bytes(D, true), s>>>(a);
        }
        k_adam_step<<<1, 64, 0, s>>>(dstep.p, beta1, beta2, bc.p);
        AdamArgs ad{p.p, m.p, v.p, g.p, w.p, n, lr, beta1, beta2, 1e-8f, bc.p};
        k_adam<<<grid_for(n, 256), 256, 0, s>>>(ad);
        FSM_LAUNCH_CHECK();
    };
    if (steps < GRAPH_STEPS) {
        for (int k = 0; k < steps; ++k) enqueue(st);
    } else {
        Capture c;
        FSM_HIP(hipStreamCreateWithFlags(&c.cs, hipStreamNonBlocking));
        FSM_HIP(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
        FSM_HIP(hipEventRecord(c.ev, st));
        FSM_HIP(hipStreamWaitEvent(c.cs, c.ev, 0));
        FSM_HIP(hipStreamBeginCapture(c.cs, hipStreamCaptureModeThreadLocal));
        enqueue(c.cs);
        FSM_HIP(hipStreamEndCapture(c.cs, &c.graph));
        FSM_HIP(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
        for (int k = 0; k < steps; ++k) FSM_HIP(hipGraphLaunch(c.exec, c.cs));
        FSM_HIP(hipStreamSynchronize(c.cs));
    }
    step += steps;
    if (rows > 0) return scalar_to_host(scal.p) / (2.0f * (float)rows);
    FSM_HIP(hipStreamSynchronize(st));
    return 0.f;
}

void Model::params(float* host) const {
    FSM_HIP(hipMemcpyAsync(host, p.p, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, stream()));
    FSM_HIP(hipStreamSynchronize(stream()));
}

}  // namespace fsm
