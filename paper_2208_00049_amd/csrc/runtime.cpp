// Runtime around the plans: batches of independent transforms replayed as one
// HIP graph, and a tile autotuner.
//
// Batch: the transforms of a batch have no data dependence on each other, so
// their kernel chains are captured on several streams (forked from and joined
// back into one origin stream) and instantiated as one graph.  A replay is a
// single launch on the caller's stream; the graph runs the chains
// concurrently, which fills the GPU with the small, latency-bound kernels of
// many small transforms.  The executable graph is kept per direction and
// rebuilt only when the caller's pointers change.
//
// Autotuner: the tile edge sets the work-item size of the resampling kernels,
// their LDS footprint and halo overhead, and the occupancy; the best choice
// depends on D, m, the type and the node density.  The tuner builds plans for a
// short list of candidate tiles (and work-item caps), times forward + adjoint
// on the device, and keeps the fastest plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "nfft.h"
#include "nfft_internal.hpp"

struct nfft_batch_s {
    std::vector<nfft_plan_t> plans;
    std::vector<hipStream_t> streams;  // streams[0] is the capture origin
    std::vector<hipEvent_t> done;      // one per stream (join)
    hipEvent_t start = nullptr;        // fork
    struct Graph {
        std::vector<const void *> in;
        std::vector<void *> out;
        hipGraphExec_t exec = nullptr;
    } graph[2];                        // 0 forward, 1 adjoint
};

namespace {

constexpr int kMaxBatchStreams = 16;

int hip_status(hipError_t e) {
    if (e == hipSuccess) return NFFT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return NFFT_ERR_NOMEM;
    return NFFT_ERR_HIP;
}

void drop_graph(nfft_batch_s::Graph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.in.clear();
    g.out.clear();
}

// Capture every transform of the batch (direction dir) into one executable graph.
int capture(nfft_batch_s &b, int dir, const void *const *in, void *const *out) {
    nfft_batch_s::Graph &g = b.graph[dir];
    drop_graph(g);
    const int n = (int)b.plans.size(), S = (int)b.streams.size();
    // stage timing records events; it is not part of a captured batch
    std::vector<bool> timing(n);
    for (int i = 0; i < n; ++i) {
        timing[i] = b.plans[i]->timing;
        b.plans[i]->timing = false;
    }
    int rc = NFFT_OK;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b.streams[0], hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t ec = hipEventRecord(b.start, b.streams[0]);
        for (int j = 1; j < S && ec == hipSuccess; ++j) ec = hipStreamWaitEvent(b.streams[j], b.start, 0);
        for (int i = 0; i < n && ec == hipSuccess && rc == NFFT_OK; ++i) {
            hipStream_t s = b.streams[i % S];
            rc = dir == 0 ? nfft_forward(b.plans[i], in[i], out[i], s)
                          : nfft_adjoint(b.plans[i], in[i], out[i], s);
        }
        for (int j = 1; j < S && ec == hipSuccess; ++j) {
            ec = hipEventRecord(b.done[j], b.streams[j]);
            if (ec == hipSuccess) ec = hipStreamWaitEvent(b.streams[0], b.done[j], 0);
        }
        e = hipStreamEndCapture(b.streams[0], &graph);  // always end the capture
        if (e == hipSuccess) e = ec;
    }
    for (int i = 0; i < n; ++i) b.plans[i]->timing = timing[i];
    if (rc == NFFT_OK && e == hipSuccess)
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc == NFFT_OK) rc = hip_status(e);
    if (rc != NFFT_OK) {
        drop_graph(g);
        return rc;
    }
    g.in.assign(in, in + n);
    g.out.assign(out, out + n);
    return NFFT_OK;
}

int batch_run(nfft_batch_t b, int dir, const void *const *in, void *const *out, void *stream) {
    if (!b || !in || !out) return NFFT_ERR_ARG;
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
        if (!out[i] || (dir == 0 && !in[i]) || (dir == 1 && b->plans[i]->M > 0 && !in[i]))
            return NFFT_ERR_ARG;
    nfft_batch_s::Graph &g = b->graph[dir];
    const bool same = g.exec && std::equal(g.in.begin(), g.in.end(), in) &&
                      std::equal(g.out.begin(), g.out.end(), out);
    if (!same) {
        const int rc = capture(*b, dir, in, out);
        if (rc != NFFT_OK) return rc;
    }
    return hip_status(hipGraphLaunch(g.exec, (hipStream_t)stream));
}

}  // namespace

extern "C" {

int nfft_batch_create(nfft_batch_t *out, int n, const nfft_plan_t *plans, int nstreams) {
    if (!out || n < 1 || !plans || nstreams < 1 || nstreams > kMaxBatchStreams) return NFFT_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return NFFT_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return NFFT_ERR_ARG;  // a plan's grid serves one transform at a time
    }
    nfft_batch_s *b = new nfft_batch_s();
    b->plans.assign(plans, plans + n);
    const int S = std::min(nstreams, n);
    hipError_t e = hipEventCreateWithFlags(&b->start, hipEventDisableTiming);
    for (int j = 0; j < S && e == hipSuccess; ++j) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) b->streams.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->done.push_back(ev);
    }
    if (e != hipSuccess) {
        (void)nfft_batch_destroy(b);
        return hip_status(e);
    }
    *out = b;
    return NFFT_OK;
}

int nfft_batch_forward(nfft_batch_t b, const void *const *f, void *const *fhat, void *stream) {
    return batch_run(b, 0, f, fhat, stream);
}

int nfft_batch_adjoint(nfft_batch_t b, const void *const *fhat, void *const *y, void *stream) {
    return batch_run(b, 1, fhat, y, stream);
}

int nfft_batch_destroy(nfft_batch_t b) {
    if (!b) return NFFT_OK;
    hipError_t e = hipDeviceSynchronize();
    drop_graph(b->graph[0]);
    drop_graph(b->graph[1]);
    for (hipEvent_t ev : b->done) (void)hipEventDestroy(ev);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
    return hip_status(e);
}

int nfft_plan_create_tuned(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x,
                           int m, double sigma, nfft_dtype dtype, const nfft_options *opts,
                           int reps, void *stream, double *best_ms) {
    if (!out || reps < 1) return NFFT_ERR_ARG;
    const int vrc = nfft::validate_plan_args(D, N, M, x, m, sigma, (int)dtype, opts);
    if (vrc != NFFT_OK) return vrc;
    nfft_options base{};
    if (opts) base = *opts;
    if (base.tile[0] || base.tile[1] || base.tile[2] || base.tile[3])  // tiles fixed by the caller
        return nfft_plan_create_ex(out, D, N, M, x, m, sigma, dtype, opts, stream);
    std::vector<std::vector<int>> tiles;
    if (D == 1) tiles = {{128}, {256}, {512}, {1024}};
    else if (D == 2) tiles = {{16, 16}, {16, 32}, {32, 32}, {32, 64}, {64, 64}};
    else if (D == 3) tiles = {{8, 8, 8}, {8, 8, 16}, {8, 16, 16}, {16, 16, 16}};
    else tiles = {{4, 4, 4, 4}, {4, 4, 4, 8}, {4, 4, 8, 8}, {8, 8, 8, 8}};

    hipStream_t s = (hipStream_t)stream;
    // scratch input/output for the timing runs (values do not change the work)
    int64_t nn = 1;
    for (int d = 0; d < D && N; ++d) nn *= N[d];
    const size_t cs = dtype == NFFT_C64 ? 8 : 16;
    void *f = nullptr, *fh = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nfft_plan_t best = nullptr;
    double best_t = 0.0;
    int rc = NFFT_OK, last_rc = NFFT_ERR_UNSUPPORTED;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess && nn > 0) e = hipMalloc(&f, (size_t)nn * cs);
    if (e == hipSuccess && M > 0) e = hipMalloc(&fh, (size_t)M * cs);
    if (e == hipSuccess && f) e = nfft::launch_fill_zero_complex(f, nn, dtype == NFFT_C128, s);
    if (e == hipSuccess && fh) e = nfft::launch_fill_zero_complex(fh, M, dtype == NFFT_C128, s);
    if (e != hipSuccess) rc = hip_status(e);

    auto try_one = [&](const nfft_options &o) {
        nfft_plan_t p = nullptr;
        const int prc = nfft_plan_create_ex(&p, D, N, M, x, m, sigma, dtype, &o, stream);
        if (prc != NFFT_OK) {
            if (prc != NFFT_ERR_ARG && prc != NFFT_ERR_UNSUPPORTED) last_rc = rc = prc;
            return;
        }
        last_rc = NFFT_OK;
        int xrc = nfft_forward(p, f, fh, stream);  // warm-up
        if (xrc == NFFT_OK) xrc = nfft_adjoint(p, fh, f, stream);
        hipError_t he = hipEventRecord(e0, s);
        for (int r = 0; r < reps && xrc == NFFT_OK && he == hipSuccess; ++r) {
            xrc = nfft_forward(p, f, fh, stream);
            if (xrc == NFFT_OK) xrc = nfft_adjoint(p, fh, f, stream);
        }
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (xrc == NFFT_OK && he != hipSuccess) xrc = hip_status(he);
        if (xrc != NFFT_OK) {
            rc = xrc;
            (void)nfft_plan_destroy(p);
            return;
        }
        const double t = (double)ms / reps;
        if (!best || t < best_t) {
            if (best) (void)nfft_plan_destroy(best);
            best = p;
            best_t = t;
        } else {
            (void)nfft_plan_destroy(p);
        }
    };

    // stage 1: tiles at the default work-item cap; stage 2: caps for the best tile
    for (size_t i = 0; i < tiles.size() && rc == NFFT_OK; ++i) {
        nfft_options o = base;
        for (int d = 0; d < D; ++d) o.tile[d] = tiles[i][d];
        try_one(o);
    }
    if (best && rc == NFFT_OK && base.max_block_nodes == 0) {
        int bt[4] = {0, 0, 0, 0};
        (void)nfft_plan_info(best, nullptr, nullptr, bt);
        for (int cap : {256, 512, 1024, 2048}) {
            if (rc != NFFT_OK) break;
            nfft_options o = base;
            for (int d = 0; d < D; ++d) o.tile[d] = bt[d];
            o.max_block_nodes = cap;
            try_one(o);
        }
    }
    if (rc == NFFT_OK && !best) rc = last_rc == NFFT_OK ? NFFT_ERR_UNSUPPORTED : last_rc;
    (void)hipFree(f);
    (void)hipFree(fh);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != NFFT_OK) {
        if (best) (void)nfft_plan_destroy(best);
        return rc;
    }
    if (best_ms) *best_ms = best_t;
    *out = best;
    return NFFT_OK;
}

}  // extern "C"
