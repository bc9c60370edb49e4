// abi.cpp -- the extern "C" boundary: argument validation, error codes and
// messages, allocation / stream hooks, handle lifetime.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "internal.h"
#include "model.h"

namespace fsm {
namespace {

thread_local char g_err[512] = "";

struct Hooks {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* ctx = nullptr;
    hipStream_t stream = nullptr;
};
Hooks g_hooks;

void hip_release(void* p, void*) { (void)hipFree(p); }

template <class F>
int guarded(F&& f) {
    g_err[0] = '\0';
    try {
        f();
        return FSM_OK;
    } catch (const Failure& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return FSM_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return FSM_EDEVICE;
    }
}

}  // namespace

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    throw Failure{code};
}

hipStream_t stream() { return g_hooks.stream; }

int64_t& host_syncs() {
    static thread_local int64_t n = 0;
    return n;
}

void arena_release(void* p, void* ctx) { static_cast<Arena*>(ctx)->release(p); }

void* raw_alloc(size_t bytes, void** ctx, void (**release)(void*, void*)) {
    void* p = nullptr;
    if (Arena* a = active_arena()) {
        p = a->alloc(bytes);
        if (!p)
            fail(FSM_ENOMEM, "the call needs more device memory than the %d MiB scratch of "
                 "fsm_mine_noalloc (a buffer of %zu bytes; %zu in use, largest free range %zu)",
                 FSM_NOALLOC_SCRATCH_MIB, bytes, a->in_use, a->largest_free());
        *ctx = a;
        *release = arena_release;
        return p;
    }
    if (g_hooks.alloc) {
        p = g_hooks.alloc(bytes, g_hooks.ctx);
        if (!p) fail(FSM_ENOMEM, "device allocation of %zu bytes failed", bytes);
        *ctx = g_hooks.ctx;
        *release = g_hooks.release;
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FSM_ENOMEM : FSM_EDEVICE,
             "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    *ctx = nullptr;
    *release = hip_release;
    return p;
}

}  // namespace fsm

using namespace fsm;

extern "C" {

int fsm_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    g_err[0] = '\0';
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("fsm_set_allocator: give both hooks or neither");
        return FSM_EINVAL;
    }
    g_hooks.alloc = alloc;
    g_hooks.release = release;
    g_hooks.ctx = alloc ? ctx : nullptr;
    return FSM_OK;
}

int fsm_set_stream(void* hip_stream) {
    g_err[0] = '\0';
    g_hooks.stream = static_cast<hipStream_t>(hip_stream);
    return FSM_OK;
}

int fsm_build_graph(int64_t n_vertices, int64_t n_edges, const int32_t* src, const int32_t* dst,
                    const int32_t* vertex_labels, fsm_graph** out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) fail(FSM_EINVAL, "fsm_build_graph: out is NULL");
        if (n_vertices < 1 || n_vertices > INT32_MAX)
            fail(FSM_EINVAL, "fsm_build_graph: n_vertices must be in [1, 2^31-1]");
        if (n_edges < 0) fail(FSM_EINVAL, "fsm_build_graph: n_edges < 0");
        if (!vertex_labels) fail(FSM_EINVAL, "fsm_build_graph: vertex_labels is NULL");
        if (n_edges > 0 && (!src || !dst)) fail(FSM_EINVAL, "fsm_build_graph: src/dst is NULL");
        for (int64_t e = 0; e < n_edges; ++e)
            if (src[e] < 0 || src[e] >= n_vertices || dst[e] < 0 || dst[e] >= n_vertices)
                fail(FSM_EINVAL, "fsm_build_graph: edge %lld has an endpoint out of range",
                     (long long)e);
        for (int64_t v = 0; v < n_vertices; ++v)
            if (vertex_labels[v] < 0 || vertex_labels[v] >= (1 << 24))
                fail(FSM_EINVAL, "fsm_build_graph: label of vertex %lld outside [0, 2^24)",
                     (long long)v);
        if (n_edges > (int64_t)INT32_MAX)
            fail(FSM_EUNSUPPORTED, "fsm_build_graph: more than 2^31-1 edges");
        fsm_graph* g = new fsm_graph();
        try {
            FSM_HIP(hipGetDevice(&g->device));
            build_graph(g, n_vertices, n_edges, src, dst, vertex_labels);
        } catch (...) {
            delete g;
            throw;
        }
        *out = g;
    });
}

int64_t fsm_graph_vertices(const fsm_graph* g) { return g ? g->n : -1; }
int64_t fsm_graph_edges(const fsm_graph* g) { return g ? g->nnz / 2 : -1; }

namespace {
// Argument checks shared by fsm_mine_ex and fsm_mine_noalloc.
void check_options(const fsm_graph* g, const fsm_options* opt) {
    if (opt->support < 1) fail(FSM_EINVAL, "fsm_mine: support must be >= 1");
    if (opt->max_size < 2 || opt->max_size > FSM_MAX_SIZE)
        fail(FSM_EINVAL, "fsm_mine: max_size must be in [2, %d]", FSM_MAX_SIZE);
    if (opt->mode & ~(uint32_t)(FSM_SAMPLED | FSM_LEARNED | FSM_INDUCED | FSM_SINGLE))
        fail(FSM_EINVAL, "fsm_mine: unsupported mode bits 0x%x", opt->mode);
    if ((opt->mode & FSM_SINGLE) &&
        ((opt->mode & (FSM_SAMPLED | FSM_LEARNED)) || opt->match_threshold > 0))
        fail(FSM_EINVAL, "fsm_mine: FSM_SINGLE excludes FSM_SAMPLED, FSM_LEARNED and "
                         "match_threshold");
    if ((opt->mode & FSM_LEARNED) && !opt->model)
        fail(FSM_EINVAL, "fsm_mine: FSM_LEARNED needs options.model");
    if (opt->schedule != FSM_SCHEDULE_QUEUE && opt->schedule != FSM_SCHEDULE_STATIC)
        fail(FSM_EINVAL, "fsm_mine: unknown schedule %d", opt->schedule);
    if (opt->tiles_per_wave < 0 || opt->tiles_per_wave > 4096)
        fail(FSM_EINVAL, "fsm_mine: tiles_per_wave must be in [0, 4096]");
    if (opt->pool_budget_mib < 0) fail(FSM_EINVAL, "fsm_mine: pool_budget_mib < 0");
    if (opt->model && opt->model->m.D != FSM_FEATURES)
        fail(FSM_EINVAL, "fsm_mine: the model must have FSM_FEATURES (%d) inputs", FSM_FEATURES);
    if (opt->model && opt->model->device != g->device)
        fail(FSM_EINVAL, "fsm_mine: model and graph live on different devices");
    if ((opt->mode & FSM_SAMPLED) &&
        !(opt->sampling_rate > 0.0 && opt->sampling_rate <= 1.0))
        fail(FSM_EINVAL, "fsm_mine: sampling_rate must be in (0, 1]");
    if (opt->join_threshold < 0 || opt->join_threshold > (int64_t)1 << 20)
        fail(FSM_EINVAL, "fsm_mine: join_threshold must be in [0, 2^20]");
    if (opt->match_threshold < 0) fail(FSM_EINVAL, "fsm_mine: match_threshold < 0");
    if (opt->join_threshold > 0 && (opt->mode & FSM_SAMPLED))
        fail(FSM_EINVAL, "fsm_mine: join_threshold and FSM_SAMPLED are exclusive");
}
}  // namespace

int fsm_mine_ex(const fsm_graph* g, const fsm_options* opt, fsm_result** out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!g || !opt || !out) fail(FSM_EINVAL, "fsm_mine: NULL argument");
        check_options(g, opt);
        fsm_result* r = new fsm_result();
        try {
            mine(g, *opt, r);
        } catch (...) {
            delete r;
            throw;
        }
        *out = r;
    });
}

int fsm_mine_noalloc(const fsm_graph* g, const fsm_options* opt, int64_t capacity,
                     int32_t* sizes, fsm_code* codes, int64_t* supports, int64_t* count,
                     fsm_stats* stats) {
    if (count) *count = 0;
    return guarded([&] {
        if (!g || !opt || !count) fail(FSM_EINVAL, "fsm_mine_noalloc: NULL argument");
        if (capacity < 0 || (capacity > 0 && (!sizes || !codes || !supports)))
            fail(FSM_EINVAL, "fsm_mine_noalloc: capacity < 0 or NULL output arrays");
        if (opt->record) fail(FSM_EINVAL, "fsm_mine_noalloc: record is not supported");
        check_options(g, opt);
        // the graph's own per-vertex and per-entry state of a call
        const int64_t floor_bytes = 64 * g->n + 16 * g->nnz;
        if (floor_bytes > (int64_t)scratch_bytes())
            fail(FSM_EOVERFLOW, "fsm_mine_noalloc: a graph of %lld vertices and %lld CSR "
                 "entries needs more than the %d MiB scratch", (long long)g->n,
                 (long long)g->nnz, FSM_NOALLOC_SCRATCH_MIB);
        int dev = 0;
        FSM_HIP(hipGetDevice(&dev));
        if (dev != g->device)
            fail(FSM_EINVAL, "fsm_mine_noalloc: the graph lives on device %d, device %d is "
                 "current", g->device, dev);
        std::lock_guard<std::mutex> lk(scratch_lock(dev));
        uint8_t* base = scratch_base(dev);
        fsm_result r;
        {
            Arena arena(base, scratch_bytes());
            ArenaScope scope(&arena);
            mine_in_arena(g, *opt, &r);
        }
        const int64_t n = (int64_t)r.size.size();
        *count = n;
        if (stats) *stats = r.stats;
        if (n > capacity)
            fail(FSM_EOVERFLOW, "fsm_mine_noalloc: %lld patterns, output capacity %lld",
                 (long long)n, (long long)capacity);
        for (int64_t i = 0; i < n; ++i) {
            sizes[i] = r.size[(size_t)i];
            codes[i] = r.code[(size_t)i];
            supports[i] = r.support[(size_t)i];
        }
    });
}

int fsm_mine(const fsm_graph* g, int64_t support, int32_t max_size, uint32_t mode,
             fsm_result** out) {
    if (mode & FSM_SAMPLED) {
        if (out) *out = nullptr;
        set_error("fsm_mine: FSM_SAMPLED needs fsm_mine_ex (rate and seed)");
        return FSM_EINVAL;
    }
    fsm_options o;
    memset(&o, 0, sizeof(o));
    o.support = support;
    o.max_size = max_size;
    o.mode = mode;
    o.sampling_rate = 1.0;
    return fsm_mine_ex(g, &o, out);
}

int fsm_mine_batch_ex(const fsm_graph* const* graphs, int32_t count, const int64_t* supports,
                      const fsm_batch_options* opt, fsm_result** outs) {
    if (outs && count > 0)
        for (int32_t i = 0; i < count; ++i) outs[i] = nullptr;
    std::vector<fsm_result*> rs;
    int rc = guarded([&] {
        if (!graphs || !supports || !outs || !opt)
            fail(FSM_EINVAL, "fsm_mine_batch: NULL argument");
        if (count < 1) fail(FSM_EINVAL, "fsm_mine_batch: count must be >= 1");
        if (count > 2048) fail(FSM_EUNSUPPORTED, "fsm_mine_batch: at most 2048 graphs");
        if (opt->max_size < 2 || opt->max_size > FSM_MAX_SIZE)
            fail(FSM_EINVAL, "fsm_mine_batch: max_size must be in [2, %d]", FSM_MAX_SIZE);
        if (opt->mode & ~(uint32_t)(FSM_BATCHED | FSM_LEARNED | FSM_INDUCED))
            fail(FSM_EINVAL, "fsm_mine_batch: unsupported mode bits 0x%x", opt->mode);
        if (opt->chunk_vertices < 0) fail(FSM_EINVAL, "fsm_mine_batch: chunk_vertices < 0");
        if (opt->tiles_per_wave < 0 || opt->tiles_per_wave > 4096)
            fail(FSM_EINVAL, "fsm_mine_batch: tiles_per_wave must be in [0, 4096]");
        if (opt->pool_budget_mib < 0) fail(FSM_EINVAL, "fsm_mine_batch: pool_budget_mib < 0");
        if (((opt->mode & FSM_LEARNED) || opt->learn) && !opt->model)
            fail(FSM_EINVAL, "fsm_mine_batch: FSM_LEARNED and learn need a model");
        if (opt->model && opt->model->m.D != FSM_FEATURES)
            fail(FSM_EINVAL, "fsm_mine_batch: the model must have FSM_FEATURES (%d) inputs",
                 FSM_FEATURES);
        if (opt->train_steps < 0 || opt->lr < 0.f)
            fail(FSM_EINVAL, "fsm_mine_batch: train_steps and lr must be >= 0");
        for (int32_t i = 0; i < count; ++i) {
            if (!graphs[i]) fail(FSM_EINVAL, "fsm_mine_batch: graph %d is NULL", i);
            if (supports[i] < 1) fail(FSM_EINVAL, "fsm_mine_batch: support %d must be >= 1", i);
        }
        if (count > 1 && opt->max_size > 6)
            fail(FSM_EUNSUPPORTED, "fsm_mine_batch: batches of several graphs support sizes up to 6");
        for (int32_t i = 0; i < count; ++i) rs.push_back(new fsm_result());
        mine_batch(graphs, count, supports, *opt, rs.data());
    });
    if (rc != FSM_OK) {
        for (fsm_result* r : rs) delete r;
        return rc;
    }
    for (int32_t i = 0; i < count; ++i) outs[i] = rs[(size_t)i];
    return FSM_OK;
}

int fsm_tune_batch(const fsm_graph* const* graphs, int32_t count, const int64_t* supports,
                   int32_t max_size, fsm_tuning* out) {
    return guarded([&] {
        if (!graphs || !supports || !out) fail(FSM_EINVAL, "fsm_tune_batch: NULL argument");
        if (count < 1 || count > 2048) fail(FSM_EINVAL, "fsm_tune_batch: count must be in [1, 2048]");
        if (max_size < 2 || max_size > 6)
            fail(FSM_EINVAL, "fsm_tune_batch: max_size must be in [2, 6]");
        for (int32_t i = 0; i < count; ++i) {
            if (!graphs[i]) fail(FSM_EINVAL, "fsm_tune_batch: graph %d is NULL", i);
            if (supports[i] < 1) fail(FSM_EINVAL, "fsm_tune_batch: support %d must be >= 1", i);
        }
        tune_batch(graphs, count, supports, max_size, out);
    });
}

int fsm_reset_tuning(void) {
    g_err[0] = '\0';
    set_tuning(0, 0);
    return FSM_OK;
}

int fsm_mine_batch(const fsm_graph* const* graphs, int32_t count, const int64_t* supports,
                   int32_t max_size, uint32_t mode, fsm_result** outs) {
    fsm_batch_options o;
    memset(&o, 0, sizeof(o));
    o.max_size = max_size;
    o.mode = mode;
    return fsm_mine_batch_ex(graphs, count, supports, &o, outs);
}

int64_t fsm_result_count(const fsm_result* r) { return r ? (int64_t)r->size.size() : -1; }

int64_t fsm_result_training_count(const fsm_result* r) { return r ? (int64_t)r->tl.size() : -1; }

int fsm_result_training_rows(const fsm_result* r, float* x, float* t, int32_t* level) {
    return guarded([&] {
        if (!r) fail(FSM_EINVAL, "fsm_result_training_rows: NULL result");
        if (x && !r->tx.empty()) memcpy(x, r->tx.data(), sizeof(float) * r->tx.size());
        if (t && !r->tt.empty()) memcpy(t, r->tt.data(), sizeof(float) * r->tt.size());
        if (level && !r->tl.empty()) memcpy(level, r->tl.data(), sizeof(int32_t) * r->tl.size());
    });
}

int fsm_result_patterns(const fsm_result* r, int32_t* ids, int32_t* sizes, fsm_code* codes,
                        int64_t* supports) {
    return guarded([&] {
        if (!r) fail(FSM_EINVAL, "fsm_result_patterns: NULL result");
        for (size_t i = 0; i < r->size.size(); ++i) {
            if (ids) ids[i] = (int32_t)i;
            if (sizes) sizes[i] = r->size[i];
            if (codes) codes[i] = r->code[i];
            if (supports) supports[i] = r->support[i];
        }
    });
}

int fsm_result_stats(const fsm_result* r, fsm_stats* s) {
    return guarded([&] {
        if (!r || !s) fail(FSM_EINVAL, "fsm_result_stats: NULL argument");
        *s = r->stats;
    });
}

void fsm_graph_free(fsm_graph* g) { delete g; }
void fsm_result_free(fsm_result* r) { delete r; }

int64_t fsm_model_param_count(int32_t in_dim) {
    if (in_dim < 1 || in_dim > MODEL_MAX_IN) return -1;
    return model_param_count(in_dim);
}

int fsm_model_create(int32_t in_dim, const float* params, uint64_t seed, fsm_model** out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) fail(FSM_EINVAL, "fsm_model_create: out is NULL");
        if (in_dim < 1 || in_dim > MODEL_MAX_IN)
            fail(FSM_EINVAL, "fsm_model_create: in_dim must be in [1, %d]", MODEL_MAX_IN);
        int dev = 0;
        FSM_HIP(hipGetDevice(&dev));
        fsm_model* m = new fsm_model(in_dim, params, seed);
        m->device = dev;
        *out = m;
    });
}

int32_t fsm_model_in_dim(const fsm_model* m) { return m ? m->m.D : -1; }

int fsm_model_params(const fsm_model* m, float* params) {
    return guarded([&] {
        if (!m || !params) fail(FSM_EINVAL, "fsm_model_params: NULL argument");
        m->m.params(params);
    });
}

namespace {
// host rows -> device copies for one model call
struct Rows {
    DBuf<float> x, t;
    Rows(const fsm_model* m, const float* hx, const float* ht, int64_t rows, const char* who) {
        if (!m || !hx || rows < 0) fail(FSM_EINVAL, "%s: NULL model/x or rows < 0", who);
        if (rows > ((int64_t)1 << 31) / m->m.D) fail(FSM_EUNSUPPORTED, "%s: too many rows", who);
        x.alloc((size_t)(rows * m->m.D));
        to_device(x.p, hx, (size_t)(rows * m->m.D));
        if (ht) {
            t.alloc((size_t)(rows * MODEL_OUT));
            to_device(t.p, ht, (size_t)(rows * MODEL_OUT));
        }
    }
};
}  // namespace

int fsm_model_gradient(fsm_model* m, const float* x, const float* t, int64_t rows, float* grad,
                       double* loss) {
    return guarded([&] {
        if (!t || !grad) fail(FSM_EINVAL, "fsm_model_gradient: NULL t/grad");
        Rows r(m, x, t, rows, "fsm_model_gradient");
        const float l = m->m.gradient(r.x.p, r.t.p, rows);
        FSM_HIP(hipMemcpyAsync(grad, m->m.g.p, sizeof(float) * (size_t)m->m.n,
                               hipMemcpyDeviceToHost, stream()));
        FSM_HIP(hipStreamSynchronize(stream()));
        if (loss) *loss = l;
    });
}

int fsm_model_train(fsm_model* m, const float* x, const float* t, int64_t rows, int32_t steps,
                    float lr, double* loss) {
    return guarded([&] {
        if (!t) fail(FSM_EINVAL, "fsm_model_train: NULL t");
        if (steps < 0 || !(lr > 0.f)) fail(FSM_EINVAL, "fsm_model_train: steps < 0 or lr <= 0");
        Rows r(m, x, t, rows, "fsm_model_train");
        const float l = m->m.train(r.x.p, r.t.p, rows, steps, lr);
        if (loss) *loss = l;
    });
}

int fsm_model_predict(const fsm_model* m, const float* x, int64_t rows, float* y) {
    return guarded([&] {
        if (!y) fail(FSM_EINVAL, "fsm_model_predict: NULL y");
        Rows r(m, x, nullptr, rows, "fsm_model_predict");
        DBuf<float> dy((size_t)(rows * MODEL_OUT));
        m->m.predict(r.x.p, rows, dy.p);
        to_host_into(y, dy.p, (size_t)(rows * MODEL_OUT));
    });
}

void fsm_model_free(fsm_model* m) { delete m; }

const char* fsm_last_error(void) { return g_err; }

int fsm_dissect(int32_t n, const int32_t* ids, uint32_t adj, uint32_t* l_mask, int32_t* shared) {
    return guarded([&] {
        if (n < 4 || n > FSM_MAX_SIZE || !ids || !l_mask || !shared)
            fail(FSM_EINVAL, "fsm_dissect: bad arguments");
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (ids[i] == ids[j]) fail(FSM_EINVAL, "fsm_dissect: ids must be distinct");
        uint64_t A = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if ((adj >> pair_pos(i, j, n)) & 1u) A = add_edge(A, i, j);
        if (!connected((1u << n) - 1u, A, n)) fail(FSM_EINVAL, "fsm_dissect: graph not connected");
        uint64_t ob = 0;
        for (int p = 0; p < n; ++p) {
            int r = 0;
            for (int q = 0; q < n; ++q) r += ids[q] < ids[p] ? 1 : 0;
            ob |= (uint64_t)(1u << p) << (8 * r);
        }
        uint32_t vb = 0;
        uint32_t l = dissect(n, ob, A, &vb);
        if (!l) fail(FSM_EINVAL, "fsm_dissect: no dissection");
        *l_mask = l;
        int sh = 0;
        while (!((vb >> sh) & 1u)) ++sh;
        *shared = sh;
    });
}

int fsm_proposal_thresholds(const float* pred, int64_t rows, double rate, uint64_t* thresholds) {
    return guarded([&] {
        if (rows < 0 || (rows > 0 && (!pred || !thresholds)))
            fail(FSM_EINVAL, "fsm_proposal_thresholds: NULL array or rows < 0");
        if (!(rate > 0.0 && rate <= 1.0))
            fail(FSM_EINVAL, "fsm_proposal_thresholds: rate must be in (0, 1]");
        proposal_keep_thresholds(pred, rows, rate, thresholds);
    });
}

int fsm_key_graph(uint64_t key, int32_t size, int32_t graphs, int32_t* graph) {
    return guarded([&] {
        if (!graph || size < 2 || size > FSM_MAX_SIZE || graphs < 1)
            fail(FSM_EINVAL, "fsm_key_graph: bad arguments");
        const int gi = checked_code_graph(key, size, graphs);
        if (gi < 0)
            fail(FSM_EDEVICE, "fsm_key_graph: key 0x%llx of size %d names no graph of %d",
                 (unsigned long long)key, size, graphs);
        *graph = gi;
    });
}

}  // extern "C"
