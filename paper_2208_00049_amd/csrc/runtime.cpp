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
#include "common.hpp"
#include "nfft_internal.hpp"

// Fused batch: the stage launches of one direction.  A stage is one kernel launch
// over the blocks of every transform's pass (see BxFft / BxResample).
struct FusedStage {
    bool fft;        // an FFT pass (else a resampling stage)
    int kind;        // BatchFftKind / BatchResampleKind
    int dir;         // FFT direction
    bool pow2;       // every line length of the pass is a power of two
    int nblocks;
    int nthreads;    // FFT passes (the resampling kernels have a fixed workgroup size)
    size_t shm;      // dynamic LDS: the largest entry's
    size_t tab_off;  // byte offsets of the entry table and the block table in dev
    size_t b2e_off;
};

struct nfft_batch_s {
    std::vector<nfft_plan_t> plans;
    // fused mode: one launch per stage for all transforms
    bool fused = false;
    int dtype = 0, D = 0, taps = 0;
    std::vector<FusedStage> stages[2];  // 0 forward, 1 adjoint
    void *dev = nullptr;                // entry and block tables of every stage
    void **io[2] = {nullptr, nullptr};  // device, per direction: n input then n output pointers
    std::vector<const void *> io_in[2];  // of the direction's last call (empty: none yet)
    std::vector<void *> io_out[2];
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
constexpr size_t kFusedLds = 65536;  // LDS an FFT entry may grow its lines into

int hip_status(hipError_t e);

// ---- fused batches -------------------------------------------------------------
//
// The transforms of a batch have the same chain of stages when they share the
// complex type, D <= 3, the stencil width, the polynomial window and the padded-tile
// spreading (3-D column sweeps excluded).  Each stage then becomes one launch: the
// blocks of every transform's pass, transforms with the larger grids first, each
// transform's range starting at a multiple of the XCD count.  Every block runs the
// code of the single transform's kernel with that transform's parameters, so the
// results are those of the transforms' own calls, bit for bit.

bool fusable(const std::vector<nfft_plan_t> &ps) {
    const nfft_plan_s &a = *ps[0];
    for (const nfft_plan_t p : ps) {
        if (p->dtype != a.dtype || p->D != a.D || p->geom.taps != a.geom.taps) return false;
        if (p->D > 3 || p->sweep.on || p->window != NFFT_WINDOW_POLY) return false;
    }
    return true;
}

struct StageBuild {
    FusedStage st{};
    std::vector<nfft::BxFft> fft;
    std::vector<nfft::BxResample> res;
    std::vector<int> b2e;
};

// Append the entry's block range (aligned to the XCD count) to the block table.
void place(std::vector<int> &b2e, int e, int &start, int nblk) {
    while (b2e.size() % nfft::kNumXcd) b2e.push_back(-1);
    start = (int)b2e.size();
    for (int i = 0; i < nblk; ++i) b2e.push_back(e);
}

size_t csize_of(const nfft_plan_s &p) { return p.dtype == NFFT_C64 ? 8 : 16; }

// One FFT pass of plan p (transform t) as a table entry: kind, and for the strided
// kinds the axis.  B (lines or columns per block) and the LDS are set by finish_fft.
nfft::BxFft fft_entry(const nfft_plan_s &p, int t, int kind, int dir, int axis) {
    nfft::BxFft x{};
    x.t = t;
    x.grid = p.grid;
    for (int d = 0; d < nfft::kMaxD; ++d) x.dec[d] = p.deconv[d];
    if (kind == nfft::kBxContig) {
        x.c = nfft::contig_pass(p, dir < 0 ? 1 : 2, dir, 1);
        x.src_user = dir < 0;
        x.dst_user = dir > 0;
        x.src = p.grid;
        x.fl = p.line[p.D - 1];
    } else {
        x.a = nfft::axis_pass(p, axis, dir, 1, true);
        x.fl = p.line[axis];
        if (kind == nfft::kBxFromPad) {
            while (p.geom.Q[p.D - 1] % x.a.lines_per_block) x.a.lines_per_block /= 2;
            x.ps = nfft::PadSource{p.pad, p.tile_sub, p.geom, p.geom.taps, 0};
        }
    }
    return x;
}

int fft_lines(const nfft::BxFft &x, int kind) {
    return kind == nfft::kBxContig ? x.c.lines_per_block : x.a.lines_per_block;
}

size_t fft_entry_lds(const nfft_plan_s &p, nfft::BxFft &x, int kind, int B) {
    size_t shm = 0;
    x.fl = nfft::with_lds_table(p, x.fl, B, csize_of(p), shm);
    if (kind == nfft::kBxFromPad) shm += (size_t)p.geom.T[0] * (1 << (p.D - 1)) * 2 * sizeof(int);
    return shm;
}

int fft_blocks(const nfft::BxFft &x, int kind) {
    if (kind == nfft::kBxContig) return (x.c.nlines + x.c.lines_per_block - 1) / x.c.lines_per_block;
    const int B = x.a.lines_per_block;
    if (kind == nfft::kBxFromPad) return x.a.inner / B;
    return (int)((x.a.inner + B - 1) / B) * x.a.outer_len;
}

// Common workgroup size of an FFT stage: the largest B * tpl of its entries (a
// multiple of 64); entries below it take more lines per block while they fit.
void finish_fft(StageBuild &sb, const std::vector<const nfft_plan_s *> &pl) {
    const int kind = sb.st.kind;
    int nthr = 64;
    size_t shm_max = 0;
    for (size_t i = 0; i < sb.fft.size(); ++i) {
        nthr = std::max(nthr, fft_lines(sb.fft[i], kind) * sb.fft[i].fl.tpl);
        shm_max = std::max(shm_max, fft_entry_lds(*pl[i], sb.fft[i], kind, fft_lines(sb.fft[i], kind)));
    }
    nthr = (nthr + 63) / 64 * 64;
    const size_t cap = std::max(shm_max, kFusedLds);
    bool pow2 = true;
    sb.b2e.clear();
    sb.st.shm = 0;
    for (size_t i = 0; i < sb.fft.size(); ++i) {
        nfft::BxFft &x = sb.fft[i];
        const nfft_plan_s &p = *pl[i];
        int &B = kind == nfft::kBxContig ? x.c.lines_per_block : x.a.lines_per_block;
        for (;;) {
            const int B2 = 2 * B;
            if (B2 * x.fl.tpl > nthr || B2 > 64) break;
            if (kind != nfft::kBxContig && B2 > x.a.inner) break;
            if (kind == nfft::kBxFromPad && (p.geom.Q[p.D - 1] % B2 || nthr % B2)) break;
            nfft::BxFft y = x;
            if (fft_entry_lds(p, y, kind, B2) > cap) break;
            B = B2;
        }
        sb.st.shm = std::max(sb.st.shm, fft_entry_lds(p, x, kind, B));
        pow2 = pow2 && (x.fl.L & (x.fl.L - 1)) == 0;
        x.nblk = fft_blocks(x, kind);
        place(sb.b2e, (int)i, x.start, x.nblk);
    }
    sb.st.nthreads = nthr;
    sb.st.pow2 = pow2;
    sb.st.nblocks = (int)sb.b2e.size();
}

nfft::BxResample res_entry(const nfft_plan_s &p, int t, int kind) {
    nfft::BxResample x{};
    x.t = t;
    x.buf = kind == nfft::kBxInterp ? p.grid : p.pad;
    x.grid = p.grid;
    x.g = p.geom;
    x.nodes = p.nodes;
    x.perm = p.perm;
    x.subs = p.subs;
    x.tile_sub = p.tile_sub;
    x.coef = p.coef;
    x.window = p.window;
    x.m = p.m;
    for (int d = 0; d < nfft::kMaxD; ++d) {
        x.beta[d] = d < p.D ? nfft::kb_beta(p, d) : 0.0;
        x.inv_peak[d] = d < p.D ? 1.0 / nfft::window_peak(p, d) : 0.0;
    }
    x.tab = p.wtab;
    x.S = p.lin_S;
    x.wmax_prod = nfft::window_bound(p.D);
    x.nblk = kind == nfft::kBxMerge ? p.geom.ntiles : p.nsub;
    return x;
}

void finish_res(StageBuild &sb, const std::vector<const nfft_plan_s *> &pl) {
    sb.b2e.clear();
    sb.st.shm = 0;
    for (size_t i = 0; i < sb.res.size(); ++i) {
        const nfft_plan_s &p = *pl[i];
        const size_t cells = nfft::padded_cells(p.geom, p.D);
        const size_t cs = csize_of(p);
        if (sb.st.kind == nfft::kBxInterp) sb.st.shm = std::max(sb.st.shm, cells * cs);
        if (sb.st.kind == nfft::kBxSpread)  // fixed-point accumulators: 2 (c64) or 4 int64 per point
            sb.st.shm = std::max(sb.st.shm, cells * (cs == 8 ? 16 : 32));
        place(sb.b2e, (int)i, sb.res[i].start, sb.res[i].nblk);
    }
    sb.st.nthreads = nfft::resample_block_threads(pl.empty() ? 1 : pl[0]->D);
    sb.st.nblocks = (int)sb.b2e.size();
}

// Build the stages of both directions and upload their tables.
int fused_build(nfft_batch_s &b) {
    const int n = (int)b.plans.size();
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
        return b.plans[i]->G != b.plans[j]->G ? b.plans[i]->G > b.plans[j]->G
                                              : b.plans[i]->M > b.plans[j]->M;
    });
    const int D = b.plans[0]->D;
    b.dtype = b.plans[0]->dtype;
    b.D = D;
    b.taps = b.plans[0]->geom.taps;
    std::vector<StageBuild> built[2];
    // forward (plans without nodes have nothing to compute), then adjoint
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<int> ids;
        for (int i : order)
            if (dir == 1 || b.plans[i]->M > 0) ids.push_back(i);
        std::vector<const nfft_plan_s *> pl;
        for (int i : ids) pl.push_back(b.plans[i]);
        auto fft_stage = [&](int kind, int fdir, int axis) {
            StageBuild sb;
            sb.st.fft = true;
            sb.st.kind = kind;
            sb.st.dir = fdir;
            for (int i : ids) sb.fft.push_back(fft_entry(*b.plans[i], i, kind, fdir, axis));
            finish_fft(sb, pl);
            built[dir].push_back(std::move(sb));
        };
        // resampling stages: the transforms with the most nodes per work item first, so
        // that the longest workgroups do not form the launch's tail
        auto res_stage = [&](int kind) {
            StageBuild sb;
            sb.st.fft = false;
            sb.st.kind = kind;
            std::vector<int> rid = ids;
            if (kind != nfft::kBxMerge)
                std::stable_sort(rid.begin(), rid.end(), [&](int i, int j) {
                    const nfft_plan_s &a = *b.plans[i], &c = *b.plans[j];
                    return a.M * std::max(c.nsub, 1) > c.M * std::max(a.nsub, 1);
                });
            std::vector<const nfft_plan_s *> rpl;
            for (int i : rid) {
                sb.res.push_back(res_entry(*b.plans[i], i, kind));
                rpl.push_back(b.plans[i]);
            }
            finish_res(sb, rpl);
            built[dir].push_back(std::move(sb));
        };
        if (dir == 0) {
            fft_stage(nfft::kBxContig, -1, D - 1);
            for (int a = D - 2; a >= 0; --a) fft_stage(nfft::kBxStrided, -1, a);
            res_stage(nfft::kBxInterp);
        } else {
            res_stage(nfft::kBxSpread);
            if (D != 2) res_stage(nfft::kBxMerge);
            for (int a = 0; a <= D - 2; ++a)
                fft_stage(D == 2 && a == 0 ? nfft::kBxFromPad : nfft::kBxStrided, +1, a);
            fft_stage(nfft::kBxContig, +1, D - 1);
        }
    }
    // one device buffer: per stage its entry table, then its block table
    size_t bytes = 0;
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    for (int dir = 0; dir < 2; ++dir)
        for (StageBuild &sb : built[dir]) {
            sb.st.tab_off = bytes = align(bytes);
            bytes += sb.st.fft ? sb.fft.size() * sizeof(nfft::BxFft)
                               : sb.res.size() * sizeof(nfft::BxResample);
            sb.st.b2e_off = bytes = align(bytes);
            bytes += sb.b2e.size() * sizeof(int);
        }
    std::vector<unsigned char> host(std::max<size_t>(bytes, 1), 0);
    for (int dir = 0; dir < 2; ++dir)
        for (StageBuild &sb : built[dir]) {
            if (sb.st.fft)
                std::copy((const unsigned char *)sb.fft.data(),
                          (const unsigned char *)(sb.fft.data() + sb.fft.size()), host.begin() + sb.st.tab_off);
            else
                std::copy((const unsigned char *)sb.res.data(),
                          (const unsigned char *)(sb.res.data() + sb.res.size()), host.begin() + sb.st.tab_off);
            std::copy((const unsigned char *)sb.b2e.data(),
                      (const unsigned char *)(sb.b2e.data() + sb.b2e.size()), host.begin() + sb.st.b2e_off);
            b.stages[dir].push_back(sb.st);
        }
    hipError_t e = hipMalloc(&b.dev, host.size());
    if (e == hipSuccess) e = hipMemcpy(b.dev, host.data(), host.size(), hipMemcpyHostToDevice);
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir)
        e = hipMalloc((void **)&b.io[dir], 2 * (size_t)n * sizeof(void *));
    return hip_status(e);
}

int fused_launch(nfft_batch_s &b, int dir, hipStream_t s);

int fused_run(nfft_batch_s &b, int dir, const void *const *in, void *const *out, hipStream_t s) {
    const int n = (int)b.plans.size();
    const bool same = !b.io_in[dir].empty() &&
                      std::equal(b.io_in[dir].begin(), b.io_in[dir].end(), in) &&
                      std::equal(b.io_out[dir].begin(), b.io_out[dir].end(), out);
    if (!same) {
        // new pointers: the kernels of earlier calls may still read the table, so the
        // stream is drained before it is rewritten
        std::vector<const void *> host(2 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            host[i] = in[i];
            host[n + i] = out[i];
        }
        b.io_in[dir].clear();
        b.io_out[dir].clear();
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpy(b.io[dir], host.data(), host.size() * sizeof(void *), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_status(e);
        b.io_in[dir].assign(in, in + n);
        b.io_out[dir].assign(out, out + n);
    }
    if (!b.graph[dir].exec) {
        // the direction's stage launches, captured once into a graph on the batch's own
        // stream (their arguments -- the tables -- never change; the pointer table is
        // rewritten in place)
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(b.streams[0], hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_status(e);
        const int rc = fused_launch(b, dir, b.streams[0]);
        e = hipStreamEndCapture(b.streams[0], &graph);  // always end the capture
        if (rc == NFFT_OK && e == hipSuccess)
            e = hipGraphInstantiate(&b.graph[dir].exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != NFFT_OK) return rc;
        if (e != hipSuccess) {
            b.graph[dir].exec = nullptr;
            return hip_status(e);
        }
    }
    return hip_status(hipGraphLaunch(b.graph[dir].exec, s));
}

// The stage launches of one direction on stream s.
int fused_launch(nfft_batch_s &b, int dir, hipStream_t s) {
    const int n = (int)b.plans.size();
    const void *const *din = (const void *const *)b.io[dir];
    void *const *dout = (void *const *)(b.io[dir] + n);
    for (const FusedStage &st : b.stages[dir]) {
        const unsigned char *base = (const unsigned char *)b.dev;
        const int *b2e = (const int *)(base + st.b2e_off);
        hipError_t e;
        if (st.fft)
            e = nfft::launch_fft_batch(st.kind, b.dtype, b.D, st.dir, st.pow2,
                                       (const nfft::BxFft *)(base + st.tab_off), b2e, din, dout,
                                       st.nblocks, st.nthreads, st.shm, s);
        else
            e = nfft::launch_resample_batch(st.kind, b.dtype, b.D, b.taps, false,
                                            (const nfft::BxResample *)(base + st.tab_off), b2e, din,
                                            dout, st.nblocks, st.shm, s);
        if (e != hipSuccess) return hip_status(e);
    }
    return NFFT_OK;
}

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
    for (int i = 0; i < n; ++i) {  // as nfft_forward / nfft_adjoint: no fhat without nodes
        const bool has_fhat = b->plans[i]->M > 0;
        if (dir == 0 && (!in[i] || (has_fhat && !out[i]))) return NFFT_ERR_ARG;
        if (dir == 1 && (!out[i] || (has_fhat && !in[i]))) return NFFT_ERR_ARG;
    }
    if (b->fused) return fused_run(*b, dir, in, out, (hipStream_t)stream);
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
    if (fusable(b->plans)) {
        b->fused = true;
        hipStream_t cs = nullptr;  // capture stream (default priority)
        int rc = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        if (rc == NFFT_OK) b->streams.push_back(cs);
        if (rc == NFFT_OK) rc = fused_build(*b);
        if (rc != NFFT_OK) {
            (void)nfft_batch_destroy(b);
            return rc;
        }
        *out = b;
        return NFFT_OK;
    }
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
    (void)hipFree(b->dev);
    (void)hipFree(b->io[0]);
    (void)hipFree(b->io[1]);
    for (hipEvent_t ev : b->done) (void)hipEventDestroy(ev);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
    return hip_status(e);
}

int nfft_batch_info(nfft_batch_t b, int *fused, int *launches_forward, int *launches_adjoint) {
    if (!b) return NFFT_ERR_ARG;
    if (fused) *fused = b->fused ? 1 : 0;
    if (launches_forward) *launches_forward = b->fused ? (int)b->stages[0].size() : 0;
    if (launches_adjoint) *launches_adjoint = b->fused ? (int)b->stages[1].size() : 0;
    return NFFT_OK;
}

int nfft_plan_create_tuned(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x,
                           int m, double sigma, nfft_dtype dtype, const nfft_options *opts,
                           int reps, void *stream, double *best_ms) {
    if (!out || reps < 1) return NFFT_ERR_ARG;
    const int vrc = nfft::validate_plan_args(D, N, M, x, m, sigma, (int)dtype, opts);
    if (vrc != NFFT_OK) return vrc;
    nfft_options base{};
    if (opts) base = *opts;
    // tiles fixed by the caller, or D >= 5 (whose tiles are always automatic)
    if (base.tile[0] || base.tile[1] || base.tile[2] || base.tile[3] || D > 4)
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
        int bt[nfft::kMaxD] = {};
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
