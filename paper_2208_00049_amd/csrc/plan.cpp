// libnfft host side: argument validation, plan construction and the C ABI.
//
// Forward transform (paper, Algorithm 1): resampling correction + zero padding
// (fused into the last-axis FFT pass), D-variate FFT, interpolation.
// Adjoint (Algorithm 2): spreading, D-variate adjoint FFT, crop + resampling
// correction (fused into the last-axis FFT pass).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "nfft_internal.hpp"

using namespace nfft;

namespace {

constexpr int kMaxM = 10;
constexpr size_t kLdsBudget = 65536;
constexpr int kOptionTiles = 4;  // tile edges nfft_options holds
// Default cap on a work item's nodes, per D.  1-D/2-D: 1024, or 512 when the
// tiles hold at most 512 nodes on average -- then only locally dense tiles (a
// radial trajectory's centre) are split, and smaller pieces balance them better,
// while uniformly dense node sets keep fewer items per tile (each extra item adds
// a padded tile to every halo merge).  3-D tiles hold ~512 nodes on average at
// sigma = 2 and keep 1024.  D = 4 interpolates one node per wavefront, so small
// items spread a tile's nodes over many workgroups.
constexpr int kDefaultBlockNodes[kMaxD + 1] = {0, 1024, 1024, 1024, 16, 16, 16};
constexpr int kSparseBlockNodes = 512;
constexpr int kMaxChannels = 65535;  // channels of one multi-channel call (grid y dimension)

bool is_235_smooth(int64_t v) {
    for (int p : {2, 3, 5})
        while (v % p == 0) v /= p;
    return v == 1;
}

// Smallest even integer >= sigma*N whose prime factors are 2, 3 and 5 (the paper
// writes Ntilde = sigma N without saying how a non-integer product is rounded).
int64_t oversampled(int64_t N, double sigma) {
    const double target = sigma * (double)N;
    int64_t c = (int64_t)ceil(target - 1e-9 * target);
    if (c % 2) ++c;
    while (!is_235_smooth(c)) c += 2;
    return c;
}

size_t csize(nfft_dtype t) { return t == NFFT_C64 ? 8 : 16; }

// Complex values of spreading scratch per channel: the work items' padded tiles
// (D <= 3; D = 4 spreads straight into the grid).
size_t scratch_cells(const nfft_plan_s &p) {
    if (p.sweep.on) return p.M > 0 ? sweep_scratch_cells(p) : 0;
    if (p.nsub == 0 || p.D > 3) return 0;
    return (size_t)p.nsub * padded_cells(p.geom, p.D);
}

size_t rsize(nfft_dtype t) { return t == NFFT_C64 ? 4 : 8; }

size_t node_rec_size(nfft_dtype t, int D) {
    if (t == NFFT_C64) {
        switch (D) {
            case 1: return sizeof(NodeRec<float, 1>);
            case 2: return sizeof(NodeRec<float, 2>);
            case 3: return sizeof(NodeRec<float, 3>);
            case 4: return sizeof(NodeRec<float, 4>);
            case 5: return sizeof(NodeRec<float, 5>);
            default: return sizeof(NodeRec<float, 6>);
        }
    }
    switch (D) {
        case 1: return sizeof(NodeRec<double, 1>);
        case 2: return sizeof(NodeRec<double, 2>);
        case 3: return sizeof(NodeRec<double, 3>);
        case 4: return sizeof(NodeRec<double, 4>);
        case 5: return sizeof(NodeRec<double, 5>);
        default: return sizeof(NodeRec<double, 6>);
    }
}

// Factor the line length into Stockham passes (radix 8 first, then 4 or 2, 5, 3).
bool factor_line(int L, FftLine &fl) {
    int v = L, np = 0, e2 = 0;
    while (v % 2 == 0) {
        v /= 2;
        ++e2;
    }
    while (e2 >= 3) {
        fl.rad[np++] = 8;
        e2 -= 3;
    }
    if (e2 == 2) fl.rad[np++] = 4;
    if (e2 == 1) fl.rad[np++] = 2;
    while (v % 5 == 0) {
        fl.rad[np++] = 5;
        v /= 5;
    }
    while (v % 3 == 0) {
        fl.rad[np++] = 3;
        v /= 3;
    }
    if (v != 1 || np > kMaxRadixPasses || np == 0) return false;
    int rmax = 0;
    for (int i = 0; i < np; ++i) rmax = std::max(rmax, fl.rad[i]);
    fl.L = L;
    fl.npass = np;
    fl.tpl = L / rmax;
    return fl.tpl <= 1024;
}

// LDS of the interpolation kernel: tile + halo plus the staged node chunk.
size_t interp_lds(const int *Q, int D, int taps, size_t cs) {
    size_t t = cs;
    for (int d = 0; d < D; ++d) t *= (size_t)(Q[d] + taps - 1);
    return t + nfft::interp_static_lds(D, (int)cs / 2);
}

// LDS of the spreading kernel: fixed-point accumulators of the padded tile (one
// int64 per component) plus the staged node chunk.
size_t spread_lds(const int *Q, int D, int taps, size_t cs) {
    size_t t = 16;
    for (int d = 0; d < D; ++d) t *= (size_t)(Q[d] + taps - 1);
    return t + nfft::resample_static_lds(D, (int)cs / 2);
}

bool valid_tile(int64_t Nt, int Q, int taps) {
    return Q >= taps && Q > 0 && Nt % Q == 0 && Nt / Q >= 2;
}

// Largest valid tile edge <= want (a divisor of Nt, >= taps, >= 2 tiles).
int pick_edge_down(int64_t Nt, int want, int taps) {
    for (int q = std::min<int64_t>(want, Nt / 2); q >= taps; --q)
        if (valid_tile(Nt, q, taps)) return q;
    return 0;
}

// Valid tile edge closest to want: the largest one <= want, else the smallest one above.
int pick_edge(int64_t Nt, int want, int taps) {
    const int q = pick_edge_down(Nt, want, taps);
    if (q) return q;
    for (int v = std::max(want, taps); v <= Nt / 2; ++v)
        if (valid_tile(Nt, v, taps)) return v;
    return 0;
}

// D >= 4: a spreading workgroup owns one tile (its fixed-point accumulators in
// LDS) and reads the nodes of at most owner_max_tiles(D) = 3^D tiles, which tile
// edges >= taps/2 guarantee.  A tile edge is any divisor of Nt_d.  Default: per axis
// the smallest divisor >= max(8, taps/2), then the largest edge shrinks (to a
// smaller divisor >= taps/2) until the tile fits the workgroup LDS `budget`.
// req: requested edges (D = 4 only; NULL or all zero: automatic).
int choose_tiles_4d(int D, const int64_t *Nt, int taps, nfft_dtype dt, const int *req,
                    size_t budget, int *Q) {
    const size_t cs = csize(dt);
    const size_t stat = owner_static_lds(D, taps, (int)rsize(dt));
    auto fits = [&](const int *q) {
        size_t cells = 1;
        for (int d = 0; d < D; ++d) cells *= (size_t)q[d];
        return cells * owner_cell_bytes((int)cs) + stat <= budget;
    };
    auto reach_ok = [&](const int *q) {
        Geom g{};
        g.taps = taps;
        int nb = 1;
        for (int d = 0; d < D; ++d) {
            g.Q[d] = q[d];
            g.T[d] = (int)(Nt[d] / q[d]);
            nb *= owner_reach(g, d);
        }
        return nb <= owner_max_tiles(D);
    };
    if (D == 4 && req && (req[0] || req[1] || req[2] || req[3])) {
        for (int d = 0; d < 4; ++d) {
            if (req[d] < 1 || Nt[d] % req[d]) return NFFT_ERR_ARG;
            Q[d] = req[d];
        }
        return reach_ok(Q) && fits(Q) ? NFFT_OK : NFFT_ERR_UNSUPPORTED;
    }
    const int lo = std::max(1, taps / 2);
    for (int d = 0; d < D; ++d) {
        Q[d] = (int)Nt[d];
        for (int q = std::max(8, lo); q < Nt[d]; ++q)
            if (Nt[d] % q == 0) {
                Q[d] = q;
                break;
            }
    }
    while (!fits(Q)) {
        int best = -1, bq = 0;
        for (int d = 0; d < D; ++d) {
            int q = Q[d] - 1;
            while (q >= lo && Nt[d] % q) --q;
            if (q >= lo && (best < 0 || Q[d] > Q[best])) {
                best = d;
                bq = q;
            }
        }
        if (best < 0) return NFFT_ERR_UNSUPPORTED;
        Q[best] = bq;
    }
    return reach_ok(Q) ? NFFT_OK : NFFT_ERR_UNSUPPORTED;
}

int choose_tiles(int D, const int64_t *Nt, int taps, nfft_dtype dt, const int *req, size_t budget,
                 int *Q) {
    const size_t cs = csize(dt);
    if (req && (req[0] || req[1] || req[2])) {
        for (int d = 0; d < D; ++d) {
            if (!valid_tile(Nt[d], req[d], taps)) return NFFT_ERR_ARG;
            Q[d] = req[d];
        }
        return interp_lds(Q, D, taps, cs) <= budget && spread_lds(Q, D, taps, cs) <= budget
                   ? NFFT_OK : NFFT_ERR_UNSUPPORTED;
    }
    int want[3];
    if (D == 1) want[0] = 256;
    else if (D == 2) want[0] = want[1] = 32;
    else {
        want[0] = 8;
        want[1] = want[2] = 16;
    }
    for (int d = 0; d < D; ++d) {
        Q[d] = pick_edge(Nt[d], std::max(want[d], taps), taps);
        if (!Q[d]) return NFFT_ERR_UNSUPPORTED;
    }
    // shrink the largest edge until both resampling kernels fit in LDS
    while (interp_lds(Q, D, taps, cs) > budget || spread_lds(Q, D, taps, cs) > budget) {
        int best = -1;
        for (int d = 0; d < D; ++d) {
            const int q = pick_edge_down(Nt[d], Q[d] - 1, taps);
            if (q && (best < 0 || Q[d] > Q[best])) best = d;
        }
        if (best < 0) return NFFT_ERR_UNSUPPORTED;
        Q[best] = pick_edge_down(Nt[best], Q[best] - 1, taps);
    }
    return NFFT_OK;
}

// Householder QR of the Theta x Z Vandermonde matrix in s in [-1, 1]; returns
// Q^T (Z x Theta) and R (Z x Z, upper triangular), row-major.
void vandermonde_qr(int Z, int Theta, std::vector<double> &qt, std::vector<double> &r) {
    std::vector<double> A((size_t)Theta * Z), V((size_t)Theta * Z, 0.0);
    for (int v = 0; v < Theta; ++v) {
        const double s = -1.0 + 2.0 * v / (double)(Theta - 1);
        double pw = 1.0;
        for (int z = 0; z < Z; ++z) {
            A[(size_t)v * Z + z] = pw;
            pw *= s;
        }
    }
    for (int k = 0; k < Z; ++k) {
        double nrm = 0.0;
        for (int i = k; i < Theta; ++i) nrm += A[(size_t)i * Z + k] * A[(size_t)i * Z + k];
        nrm = sqrt(nrm);
        const double x0 = A[(size_t)k * Z + k];
        const double alpha = x0 >= 0 ? -nrm : nrm;
        double vn = 0.0;
        for (int i = k; i < Theta; ++i) {
            const double vi = A[(size_t)i * Z + k] - (i == k ? alpha : 0.0);
            V[(size_t)i * Z + k] = vi;
            vn += vi * vi;
        }
        vn = sqrt(vn);
        if (vn > 0)
            for (int i = k; i < Theta; ++i) V[(size_t)i * Z + k] /= vn;
        for (int j = k; j < Z; ++j) {
            double dot = 0.0;
            for (int i = k; i < Theta; ++i) dot += V[(size_t)i * Z + k] * A[(size_t)i * Z + j];
            for (int i = k; i < Theta; ++i) A[(size_t)i * Z + j] -= 2.0 * V[(size_t)i * Z + k] * dot;
        }
    }
    r.assign((size_t)Z * Z, 0.0);
    for (int i = 0; i < Z; ++i)
        for (int j = i; j < Z; ++j) r[(size_t)i * Z + j] = A[(size_t)i * Z + j];
    // thin Q = H_0 ... H_{Z-1} applied to the first Z unit vectors
    std::vector<double> E((size_t)Theta * Z, 0.0);
    for (int i = 0; i < Z; ++i) E[(size_t)i * Z + i] = 1.0;
    for (int k = Z - 1; k >= 0; --k) {
        for (int j = 0; j < Z; ++j) {
            double dot = 0.0;
            for (int i = k; i < Theta; ++i) dot += V[(size_t)i * Z + k] * E[(size_t)i * Z + j];
            for (int i = k; i < Theta; ++i) E[(size_t)i * Z + j] -= 2.0 * V[(size_t)i * Z + k] * dot;
        }
    }
    qt.assign((size_t)Z * Theta, 0.0);
    for (int i = 0; i < Theta; ++i)
        for (int j = 0; j < Z; ++j) qt[(size_t)j * Theta + i] = E[(size_t)i * Z + j];
}

// Compute units of a device (segments of the column sweep are sized to fill them).
int cus_of(int dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

// Column-sweep spreading for a 3-D plan (see spread_sweep.hip): tiles (Q_0, 16, 16)
// with the largest Q_0 in {8, 4, 2, 1} (or the requested one) whose ring of
// Q_0 + taps - 1 planes fits the LDS beside the staged nodes, and whose
// interpolation tile fits too; segments of L tiles along axis 0 (L chosen below).
// Fills p.sweep and Q; false if the plan cannot sweep.
bool plan_sweep(nfft_plan_s &p, const int *req, size_t dev_lds, int cus, int *Q) {
    const int taps = 2 * p.m + (p.wide ? 2 : 0);
    if (p.D != 3 || p.wide || taps > 10) return false;
    for (int d = 1; d < 3; ++d)
        if (p.Nt[d] % kSweepQ || p.Nt[d] < 2 * kSweepQ) return false;
    const size_t cs = csize(p.dtype);
    const size_t budget = dev_lds - 1024;
    auto fits = [&](int q0) {
        if (q0 < 1 || p.Nt[0] % q0 || p.Nt[0] / q0 < 2) return false;
        const int q[3] = {q0, kSweepQ, kSweepQ};
        const bool wn = sweep_wave_node(taps, p.window == NFFT_WINDOW_POLY);
        return sweep_ring_bytes(q0 + taps - 1, taps, wn) + sweep_static_lds(p.dtype) <= budget &&
               interp_sweep_lds(p.dtype, q0 + taps - 1, taps) <= budget &&
               interp_lds(q, 3, taps, cs) <= budget;
    };
    int q0 = 0;
    if (req && (req[0] || req[1] || req[2])) {
        if (req[1] != kSweepQ || req[2] != kSweepQ || !fits(req[0])) return false;
        q0 = req[0];
    } else {
        for (int c : {8, 4, 2, 1})
            if (fits(c)) {
                q0 = c;
                break;
            }
        if (!q0) return false;
    }
    const int T0 = (int)(p.Nt[0] / q0);
    const int ncols = (int)(p.Nt[1] / kSweepQ) * (int)(p.Nt[2] / kSweepQ);
    // Segments of L tiles (L divides T_0 and spans at least the 2m - 1 halo planes).  The
    // workgroups (one per segment, one per compute unit: the ring takes most of the LDS) run
    // in rounds of `cus`; a segment costs its L Q_0 planes of nodes plus its 2m - 1 halo
    // planes, which are only loaded and written, at about a third of a plane each (a sweep
    // of 1 .. 8 segments per column on the 3-D workloads): L minimises rounds x (3 L Q_0 +
    // 2m - 1), so a column is cut only as far as the compute units need.
    const int lmin = std::max(1, (taps - 1 + q0 - 1) / q0);
    int L = 0;
    long long best = 0;
    for (int l = lmin; l <= std::min(T0, kSweepMaxSegTiles); ++l) {
        if (T0 % l) continue;
        const long long wgs = (long long)ncols * (T0 / l);
        const long long rounds = (wgs + cus - 1) / cus;
        const long long cost = rounds * (3LL * l * q0 + taps - 1);
        if (!L || cost < best) {
            L = l;
            best = cost;
        }
    }
    if (!L) return false;
    p.sweep.on = 1;
    p.sweep.ncols = ncols;
    p.sweep.L = L;
    p.sweep.nsc = T0 / L;
    p.sweep.R = q0 + taps - 1;
    p.sweep.main_cells = (long long)p.Nt[0] * ncols * sweep_plane_cells(taps);
    p.sweep.part_off = p.sweep.main_cells +
                       (long long)ncols * p.sweep.nsc * (taps - 1) * sweep_plane_cells(taps);
    Q[0] = q0;
    Q[1] = Q[2] = kSweepQ;
    return true;
}

int validate(int D, const int64_t *N, int64_t M, const void *x, int m, double sigma, int dtype,
             const nfft_options *opts) {
    if (D < 1) return NFFT_ERR_ARG;
    if (D > kMaxD) return NFFT_ERR_UNSUPPORTED;
    if (!N) return NFFT_ERR_ARG;
    if (M < 0 || (M > 0 && !x)) return NFFT_ERR_ARG;
    if (M >= (int64_t)1 << 31) return NFFT_ERR_UNSUPPORTED;
    if (m < 1) return NFFT_ERR_ARG;
    if (m > kMaxM) return NFFT_ERR_UNSUPPORTED;
    if (!(sigma > 1.0) || !isfinite(sigma) || sigma > 16.0) return NFFT_ERR_ARG;
    if (dtype != NFFT_C64 && dtype != NFFT_C128) return NFFT_ERR_ARG;
    // D >= 4: a wavefront holds a node's D x taps weight table, at most two entries a lane
    if (D >= 4 && D * (2 * m + (opts && opts->wide ? 2 : 0)) > 128) return NFFT_ERR_UNSUPPORTED;
    int64_t G = 1;
    for (int d = 0; d < D; ++d) {
        if (N[d] < 2) return NFFT_ERR_ARG;
        const int64_t Nt = oversampled(N[d], sigma);
        if (Nt < 2 * (2 * m + (opts && opts->wide ? 2 : 0))) return NFFT_ERR_ARG;
        if (Nt > (dtype == NFFT_C64 ? 4096 : 2048)) return NFFT_ERR_UNSUPPORTED;
        G *= Nt;
        if (G >= ((int64_t)1 << 31)) return NFFT_ERR_UNSUPPORTED;
    }
    if (opts) {
        if (opts->window < NFFT_WINDOW_POLY || opts->window > NFFT_WINDOW_FULL) return NFFT_ERR_ARG;
        if (opts->window == NFFT_WINDOW_FULL && D >= 3) return NFFT_ERR_UNSUPPORTED;
        if (opts->wide != 0 && opts->wide != 1) return NFFT_ERR_ARG;
        if (opts->wide && opts->window == NFFT_WINDOW_LINEAR) return NFFT_ERR_UNSUPPORTED;
        if (opts->max_block_nodes < 0) return NFFT_ERR_ARG;
        if (opts->spread < NFFT_SPREAD_AUTO || opts->spread > NFFT_SPREAD_SWEEP) return NFFT_ERR_ARG;
        for (int i = 0; i < 2; ++i)
            if (opts->reserved[i]) return NFFT_ERR_ARG;
        for (int d = 0; d < kOptionTiles; ++d)
            if (opts->tile[d] < 0 || (d >= D && opts->tile[d] != 0)) return NFFT_ERR_ARG;
        // the options hold four tile edges: D >= 5 plans take their tiles automatically
        if (D > kOptionTiles)
            for (int d = 0; d < kOptionTiles; ++d)
                if (opts->tile[d]) return NFFT_ERR_UNSUPPORTED;
    }
    return NFFT_OK;
}

void release(nfft_plan_s *p) {
    if (!p) return;
    for (int i = 0; i < 2 * NFFT_NUM_STAGES; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    (void)hipFree(p->grid);
    for (int d = 0; d < kMaxD; ++d) {
        (void)hipFree(p->deconv[d]);
        (void)hipFree(p->twiddle[d]);
    }
    (void)hipFree(p->coef);
    (void)hipFree(p->nodes);
    (void)hipFree(p->perm);
    (void)hipFree(p->key_start);
    (void)hipFree(p->subs);
    (void)hipFree(p->tile_sub);
    (void)hipFree(p->pad);
    (void)hipFree(p->grid_many);
    (void)hipFree(p->pad_many);
    (void)hipFree(p->wtab);
    delete p;
}

int hip_rc(hipError_t e) {
    if (e == hipSuccess) return NFFT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return NFFT_ERR_NOMEM;
    return NFFT_ERR_HIP;
}

#define TRY(expr)                         \
    do {                                  \
        hipError_t e_ = (expr);           \
        if (e_ != hipSuccess) {           \
            rc = hip_rc(e_);              \
            goto fail;                    \
        }                                 \
    } while (0)

// LDS of an FFT pass: B padded lines plus the twiddle table.
size_t fft_lds(const FftLine &fl, size_t cs, int B) { return ((size_t)B * (fl.L + 1) + fl.L) * cs; }

int lines_per_block_contig(const FftLine &fl, size_t cs) {
    int B = std::max(1, 256 / fl.tpl);
    while (B > 1 && fft_lds(fl, cs, B) > kLdsBudget) --B;
    return B;
}

int lines_per_block_strided(const FftLine &fl, size_t cs, int64_t inner) {
    int B = 16;
    while (B > 1 && (fft_lds(fl, cs, B) > kLdsBudget || B * fl.tpl > 1024 || B > inner)) B /= 2;
    return B;
}

}  // namespace

namespace nfft {

ContigPass contig_pass(const nfft_plan_s &p, int mode, int dir, int K) {
    const int D = p.D;
    ContigPass c{};
    c.K = K;
    c.mode = mode;
    c.D = D;
    c.dir = dir;
    c.src_cstride = mode == 1 ? p.NN : p.G;
    c.dst_cstride = mode == 2 ? p.NN : p.G;
    c.nlines = 1;
    for (int d = 0; d < kMaxD; ++d) {
        c.N[d] = (int)p.N[d];
        c.Nt[d] = (int)p.Nt[d];
    }
    for (int d = 0; d < D - 1; ++d) {
        c.outer_len[d] = mode == 0 ? (int)p.Nt[d] : (int)p.N[d];
        c.outer_band[d] = mode == 0 ? 0 : 1;
        c.nlines *= c.outer_len[d];
    }
    c.lines_per_block = lines_per_block_contig(p.line[D - 1], csize(p.dtype));
    return c;
}

AxisPass axis_pass(const nfft_plan_s &p, int a, int dir, int K, bool pruned) {
    AxisPass ap{};
    ap.axis = a;
    ap.inner = 1;
    for (int d = a + 1; d < p.D; ++d) ap.inner *= (int)p.Nt[d];
    ap.outer_len = 1;
    for (int d = 0; d < a; ++d) {
        ap.outer_n[d] = pruned ? (int)p.N[d] : (int)p.Nt[d];
        ap.outer_band[d] = pruned ? 1 : 0;
        ap.outer_Nt[d] = (int)p.Nt[d];
        long long st = 1;
        for (int e = d + 1; e < p.D; ++e) st *= p.Nt[e];
        ap.outer_stride[d] = st;
        ap.outer_len *= ap.outer_n[d];
    }
    ap.in_band_N = pruned && dir < 0 ? (int)p.N[a] : 0;
    ap.out_band_N = pruned && dir > 0 ? (int)p.N[a] : 0;
    ap.dir = dir;
    ap.K = K;
    ap.cstride = p.G;
    ap.lines_per_block = lines_per_block_strided(p.line[a], csize(p.dtype), ap.inner);
    return ap;
}

int validate_plan_args(int D, const int64_t *N, int64_t M, const void *x, int m, double sigma,
                       int dtype, const nfft_options *opts) {
    return validate(D, N, M, x, m, sigma, dtype, opts);
}
}  // namespace nfft

extern "C" {

const char *nfft_strerror(int code) {
    switch (code) {
        case NFFT_OK: return "success";
        case NFFT_ERR_ARG: return "invalid argument";
        case NFFT_ERR_UNSUPPORTED: return "unsupported configuration";
        case NFFT_ERR_NOMEM: return "device memory allocation failed";
        case NFFT_ERR_HIP: return "HIP runtime error";
        case NFFT_ERR_NODES: return "node coordinate is NaN or infinite";
        case NFFT_ERR_SCRATCH: return "request exceeds the library's static device scratch";
        default: return "unknown error";
    }
}

int nfft_plan_create_ex(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x, int m,
                        double sigma, nfft_dtype dtype, const nfft_options *opts, void *stream) {
    if (!out) return NFFT_ERR_ARG;
    int rc = validate(D, N, M, x, m, sigma, (int)dtype, opts);
    if (rc != NFFT_OK) return rc;

    nfft_plan_s *p = new nfft_plan_s();
    p->D = D;
    p->M = M;
    p->m = m;
    p->sigma = sigma;
    p->dtype = dtype;
    p->window = opts ? opts->window : NFFT_WINDOW_POLY;
    p->wide = opts ? opts->wide : 0;
    const int taps = 2 * m + (p->wide ? 2 : 0);
    p->max_block_nodes =
        (opts && opts->max_block_nodes) ? opts->max_block_nodes : kDefaultBlockNodes[D];
    p->G = 1;
    p->NN = 1;
    for (int d = 0; d < kMaxD; ++d) {
        p->N[d] = d < D ? N[d] : 1;
        p->Nt[d] = d < D ? oversampled(N[d], sigma) : 1;
        if (d < D) p->G *= p->Nt[d];
        if (d < D) p->NN *= p->N[d];
    }
    for (int d = 0; d < D; ++d) {
        if (!factor_line((int)p->Nt[d], p->line[d])) {
            delete p;
            return NFFT_ERR_UNSUPPORTED;
        }
    }

    // ---- device work (everything above touched no HIP API) ----
    hipStream_t s = (hipStream_t)stream;
    const size_t cs = csize(dtype), rs = rsize(dtype);
    const int Z = 2 * m + 1, Theta = 2 * Z;
    int *keys = nullptr, *counts = nullptr, *keys_sorted = nullptr, *idx = nullptr, *bad = nullptr,
        *subcnt = nullptr, *substart = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_bytes = 0;
    double *polyscratch = nullptr;
    int host_bad = 0, host_nsub = 0;
    std::vector<double> qt, rr;
    int64_t subs_cap = 0;

    TRY(hipGetDevice(&p->device));
    {
        // tiles: prefer a 64 KiB LDS footprint, go up to the device limit if needed
        int dev_lds = 0;
        TRY(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
        p->lds_limit = dev_lds;
        int Q[kMaxD];
        for (int d = 0; d < kMaxD; ++d) Q[d] = 1;
        const int *req = opts && D <= kOptionTiles ? opts->tile : nullptr;
        int trc;
        const int smode = opts ? opts->spread : NFFT_SPREAD_AUTO;
        if (D == 3 && smode != NFFT_SPREAD_TILED &&
            plan_sweep(*p, req, (size_t)dev_lds, cus_of(p->device), Q)) {
            trc = NFFT_OK;
        } else if (D == 3 && smode == NFFT_SPREAD_SWEEP) {
            trc = NFFT_ERR_UNSUPPORTED;
        } else if (D >= 4) {
            trc = choose_tiles_4d(D, p->Nt, taps, dtype, req, (size_t)dev_lds, Q);
        } else {
            // sparse 3-D node sets (under 1/4 node per grid point, e.g. sigma = 2 with
            // M = |I_N|) take the larger 8 x 16 x 16 tiles that need the device's whole
            // LDS: the padded-tile scratch per node is what dominates there
            const bool sparse3d = D == 3 && 4 * M < p->G;
            const size_t first = sparse3d && (size_t)dev_lds > kLdsBudget ? (size_t)dev_lds - 1024
                                                                           : kLdsBudget;
            trc = choose_tiles(D, p->Nt, taps, dtype, req, first, Q);
            if (trc == NFFT_ERR_UNSUPPORTED && (size_t)dev_lds - 1024 > first)
                trc = choose_tiles(D, p->Nt, taps, dtype, req, (size_t)dev_lds - 1024, Q);
        }
        if (trc != NFFT_OK) {
            rc = trc;
            goto fail;
        }
        p->geom.D = D;
        p->geom.m = m;
        p->geom.taps = taps;
        p->geom.lo = taps / 2 - 1;
        p->geom.ntiles = 1;
        for (int d = 0; d < kMaxD; ++d) {
            p->geom.Nt[d] = (int)p->Nt[d];
            p->geom.Q[d] = d < D ? Q[d] : 1;
            p->geom.T[d] = d < D ? (int)(p->Nt[d] / Q[d]) : 1;
            p->geom.ntiles *= p->geom.T[d];
        }
        // D <= 3: a tile's nodes keyed by the LDS bank slot of their first value in the
        // interpolation (the complex128 column sweeps' ring, else the tile) and ordered in
        // groups of slots 8 apart (see launch_node_sort)
        p->geom.ring_R = p->sweep.on && dtype == NFFT_C128 ? p->sweep.R : 0;
        p->geom.slot_mod = D <= 3 ? (dtype == NFFT_C128 ? 32 : 64) : 0;
        if (p->geom.slot_mod && ((long long)p->geom.ntiles << 6) >= (1LL << 30)) p->geom.slot_mod = 0;
        if (!p->geom.slot_mod) p->geom.ring_R = 0;  // (the sweep then reads the class order)
        p->geom.kbits = p->geom.slot_mod == 32 ? 5 : p->geom.slot_mod == 64 ? 6 : D;
        p->nkeys = p->geom.ntiles << p->geom.kbits;
        if (!(opts && opts->max_block_nodes) && D <= 2 && M <= (int64_t)kSparseBlockNodes * p->geom.ntiles)
            p->max_block_nodes = kSparseBlockNodes;
        subs_cap = p->geom.ntiles + M / p->max_block_nodes + 1;
    }
    TRY(hipMalloc(&p->grid, (size_t)p->G * cs));
    for (int d = 0; d < D; ++d) {
        TRY(hipMalloc(&p->deconv[d], (size_t)p->N[d] * rs));
        TRY(hipMalloc(&p->twiddle[d], (size_t)p->Nt[d] * cs));
        p->line[d].tw = p->twiddle[d];
    }
    TRY(hipMalloc(&p->coef, (size_t)D * taps * Z * rs));
    TRY(hipMalloc(&p->key_start, (size_t)(p->nkeys + 1) * sizeof(int)));
    TRY(hipMalloc(&p->subs, (size_t)subs_cap * sizeof(int4)));
    TRY(hipMalloc(&counts, (size_t)(p->nkeys + 1) * sizeof(int)));
    TRY(hipMalloc(&bad, sizeof(int)));
    TRY(hipMalloc(&subcnt, (size_t)(p->geom.ntiles + 1) * sizeof(int)));
    TRY(hipMalloc(&p->tile_sub, (size_t)(p->geom.ntiles + 1) * sizeof(int)));
    substart = p->tile_sub;
    if (M > 0) {
        TRY(hipMalloc(&p->nodes, (size_t)M * node_rec_size(dtype, D)));
        TRY(hipMalloc(&p->perm, (size_t)M * sizeof(int)));
        TRY(hipMalloc(&keys, (size_t)M * sizeof(int)));
        TRY(hipMalloc(&keys_sorted, (size_t)M * sizeof(int)));
        TRY(hipMalloc(&idx, (size_t)M * sizeof(int)));
        TRY(node_sort_bytes(*p, &sort_bytes));
        TRY(hipMalloc(&sort_tmp, std::max<size_t>(sort_bytes, 1)));
    }

    // FP64 precomputation: deconvolution factors, window polynomial, twiddles
    TRY(launch_deconv_factors(*p, s));
    vandermonde_qr(Z, Theta, qt, rr);
    {
        // Q^T, R, the shape parameters and the reciprocal window peaks per axis
        std::vector<double> host((size_t)Z * Theta + (size_t)Z * Z + 2 * kMaxD);
        std::copy(qt.begin(), qt.end(), host.begin());
        std::copy(rr.begin(), rr.end(), host.begin() + (size_t)Z * Theta);
        for (int d = 0; d < kMaxD; ++d) {
            host[(size_t)Z * Theta + (size_t)Z * Z + d] = d < D ? kb_beta(*p, d) : 0.0;
            host[(size_t)Z * Theta + (size_t)Z * Z + kMaxD + d] =
                d < D ? 1.0 / window_peak(*p, d) : 0.0;
        }
        TRY(hipMalloc(&polyscratch, host.size() * sizeof(double)));
        TRY(hipMemcpyAsync(polyscratch, host.data(), host.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
        TRY(launch_window_poly(*p, polyscratch, polyscratch + (size_t)Z * Theta, Z, Theta, s));
        // the host vector must outlive the asynchronous copy
        TRY(hipStreamSynchronize(s));
    }
    for (int d = 0; d < D; ++d) TRY(launch_twiddles(*p, d, s));

    // GPU bin sort of the nodes into tiles
    TRY(launch_fill_int(counts, p->nkeys + 1, 0, s));
    TRY(launch_fill_int(bad, 1, 0, s));
    TRY(launch_node_keys(*p, x, keys, counts, bad, s));
    TRY(launch_exclusive_scan(counts, p->key_start, p->nkeys, s));
    if (M > 0) TRY(launch_node_sort(*p, x, keys, keys_sorted, idx, sort_tmp, sort_bytes, s));
    TRY(launch_subprob_count(*p, subcnt, s));
    TRY(launch_exclusive_scan(subcnt, substart, p->geom.ntiles, s));
    TRY(launch_subprob_fill(*p, substart, s));
    TRY(hipMemcpyAsync(&host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    TRY(hipMemcpyAsync(&host_nsub, substart + p->geom.ntiles, sizeof(int), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    p->nsub = host_nsub;
    if (host_bad) rc = NFFT_ERR_NODES;
    if (rc == NFFT_OK && scratch_cells(*p) > 0) TRY(hipMalloc(&p->pad, scratch_cells(*p) * cs));
    if (rc == NFFT_OK && p->window != NFFT_WINDOW_POLY && p->window != NFFT_WINDOW_DIRECT) {
        // window tables of the precomputation modes (FP64 evaluation, plan type storage)
        size_t n = 0;
        if (p->window == NFFT_WINDOW_LINEAR) {
            static const int kLinearC[8] = {3, 7, 9, 14, 17, 20, 23, 24};
            p->lin_S = (long long)m * (1LL << kLinearC[std::min(m, 8) - 1]) + 2;
            n = (size_t)D * p->lin_S;
        } else if (p->window == NFFT_WINDOW_TENSOR) {
            n = (size_t)M * D * taps;
        } else {
            n = (size_t)M * (D == 1 ? taps : taps * taps);
        }
        if (n > 0) {
            TRY(hipMalloc(&p->wtab, n * rs));
            TRY(launch_window_tables(*p, s));
            TRY(hipStreamSynchronize(s));
        }
    }

fail:
    (void)hipFree(keys);
    (void)hipFree(counts);
    (void)hipFree(keys_sorted);
    (void)hipFree(idx);
    (void)hipFree(sort_tmp);
    (void)hipFree(bad);
    (void)hipFree(subcnt);
    (void)hipFree(polyscratch);
    if (rc != NFFT_OK) {
        release(p);
        return rc;
    }
    *out = p;
    return NFFT_OK;
}

int nfft_plan_create(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x, int m,
                     double sigma, nfft_dtype dtype, void *stream) {
    return nfft_plan_create_ex(out, D, N, M, x, m, sigma, dtype, nullptr, stream);
}

int nfft_plan_destroy(nfft_plan_t p) {
    if (!p) return NFFT_OK;
    hipError_t e = hipDeviceSynchronize();
    release(p);
    return hip_rc(e);
}

int nfft_plan_info(nfft_plan_t p, int64_t *Ntilde, double *sigma_eff, int *tile) {
    if (!p) return NFFT_ERR_ARG;
    for (int d = 0; d < p->D; ++d) {
        if (Ntilde) Ntilde[d] = p->Nt[d];
        if (tile) tile[d] = p->geom.Q[d];
    }
    if (sigma_eff) *sigma_eff = (double)p->Nt[0] / (double)p->N[0];
    return NFFT_OK;
}

int nfft_plan_grid(nfft_plan_t p, void **grid) {
    if (!p || !grid) return NFFT_ERR_ARG;
    *grid = p->grid;
    return NFFT_OK;
}

int nfft_plan_spread(nfft_plan_t p, int *scheme) {
    if (!p || !scheme) return NFFT_ERR_ARG;
    *scheme = p->sweep.on ? NFFT_SPREAD_SWEEP : NFFT_SPREAD_TILED;
    return NFFT_OK;
}

int nfft_plan_window_peak(nfft_plan_t p, double *peak) {
    if (!p || !peak) return NFFT_ERR_ARG;
    for (int d = 0; d < p->D; ++d) peak[d] = window_peak(*p, d);
    return NFFT_OK;
}

}  // extern "C"

namespace {

// Record the start / stop event of a stage when timing is on.
struct StageTimer {
    const nfft_plan_s &p;
    int stage;
    hipStream_t s;
    StageTimer(const nfft_plan_s &pl, int st, hipStream_t str) : p(pl), stage(st), s(str) {
        if (p.timing) (void)hipEventRecord(p.ev[2 * stage], s);
    }
    ~StageTimer() {
        if (p.timing) {
            (void)hipEventRecord(p.ev[2 * stage + 1], s);
            const_cast<nfft_plan_s &>(p).ev_used[stage] = true;
        }
    }
};

// Forward FFT with the resampling correction fused into the first (last-axis)
// pass; K channels: f at stride prod(N), grids at stride G.
// deriv: K = D channels from one f, channel d with coefficients -2 pi i n_d f_n
hipError_t forward_fft(const nfft_plan_s &p, const void *f, void *grid, int K, hipStream_t s,
                       bool deriv = false) {
    const int D = p.D;
    ContigPass c = contig_pass(p, 1, -1, K);
    c.deriv = deriv ? 1 : 0;
    if (deriv) c.src_cstride = 0;
    hipError_t e;
    {
        StageTimer t(p, 0, s);
        e = launch_fft_contig(p, f, grid, c, s);
    }
    if (e != hipSuccess) return e;
    for (int a = D - 2; a >= 0; --a) {
        const AxisPass ap = axis_pass(p, a, -1, K, true);
        {
            StageTimer t(p, a == 0 ? 2 : 1, s);
            e = launch_fft_axis(p, grid, ap, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// adjoint FFT with crop + resampling correction fused into the last pass;
// from_pad: the first (axis-0) pass reads and merges the padded tiles of
// spreading instead of the grid (D >= 2)
hipError_t adjoint_fft(const nfft_plan_s &p, void *y, void *grid, const void *pad, int K,
                       hipStream_t s, bool from_pad) {
    const int D = p.D;
    for (int a = 0; a <= D - 2; ++a) {
        AxisPass ap = axis_pass(p, a, +1, K, true);
        const bool merge_here = from_pad && a == 0;
        if (merge_here)  // the workgroup's columns must lie in one tile column
            while (p.geom.Q[D - 1] % ap.lines_per_block) ap.lines_per_block /= 2;
        hipError_t e;
        {
            StageTimer t(p, a == 0 ? 5 : 6, s);
            e = !merge_here  ? launch_fft_axis(p, grid, ap, s)
                : p.sweep.on ? launch_fft_axis0_from_sweep(p, grid, ap, pad, s)
                             : launch_fft_axis0_from_pad(p, grid, ap, pad, s);
        }
        if (e != hipSuccess) return e;
    }
    const ContigPass c = contig_pass(p, 2, +1, K);
    StageTimer t(p, 7, s);
    return launch_fft_contig(p, grid, y, c, s);
}

// plain unpruned FFT of a whole grid, all axes
hipError_t plain_fft(const nfft_plan_s &p, void *grid, int dir, hipStream_t s) {
    const int D = p.D;
    const ContigPass c = contig_pass(p, 0, dir, 1);
    hipError_t e = launch_fft_contig(p, grid, grid, c, s);
    if (e != hipSuccess) return e;
    for (int a = D - 2; a >= 0; --a) {
        e = launch_fft_axis(p, grid, axis_pass(p, a, dir, 1, false), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Make room for K channels' grids and padded tiles (multi-channel calls).
hipError_t ensure_channels(nfft_plan_s &p, int K) {
    if (K <= p.many_cap) return hipSuccess;
    (void)hipFree(p.grid_many);
    (void)hipFree(p.pad_many);
    p.grid_many = p.pad_many = nullptr;
    p.many_cap = 0;
    const size_t cs = csize(p.dtype);
    hipError_t e = hipMalloc(&p.grid_many, (size_t)K * p.G * cs);
    if (e == hipSuccess && scratch_cells(p) > 0)
        e = hipMalloc(&p.pad_many, (size_t)K * scratch_cells(p) * cs);
    if (e == hipSuccess) p.many_cap = K;
    return e;
}

hipError_t run_forward(const nfft_plan_s &p, const void *f, void *fhat, int K, void *grid,
                       hipStream_t s) {
    hipError_t e = forward_fft(p, f, grid, K, s);
    if (e == hipSuccess) {
        StageTimer t(p, 3, s);
        e = launch_interp(p, grid, fhat, s, K);
    }
    return e;
}

hipError_t run_adjoint(const nfft_plan_s &p, const void *fhat, void *y, int K, void *grid,
                       void *pad, hipStream_t s) {
    // 2-D and 3-D column sweeps: the merge of spreading is done by the first adjoint
    // FFT pass (for 3-D padded tiles the separate merge kernel is faster: a pass's
    // columns would span one short tile edge, and each grid value gathers from up
    // to eight tiles)
    const bool fuse = p.D == 2 || p.sweep.on;
    hipError_t e;
    {
        StageTimer t(p, 4, s);
        e = launch_spread(p, fhat, grid, s, !fuse, K, pad);
    }
    if (e == hipSuccess) e = adjoint_fft(p, y, grid, pad, K, s, fuse);
    return e;
}

}  // namespace

extern "C" {

int nfft_forward(nfft_plan_t p, const void *f, void *fhat, void *stream) {
    if (!p || !f || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    if (p->M == 0) return NFFT_OK;
    return hip_rc(run_forward(*p, f, fhat, 1, p->grid, (hipStream_t)stream));
}

int nfft_adjoint(nfft_plan_t p, const void *fhat, void *y, void *stream) {
    if (!p || !y || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (p->M == 0) return hip_rc(launch_fill_zero_complex(y, p->NN, p->dtype == NFFT_C128, s));
    return hip_rc(run_adjoint(*p, fhat, y, 1, p->grid, p->pad, s));
}

int nfft_forward_many(nfft_plan_t p, int K, const void *f, void *fhat, void *stream) {
    if (!p || K < 1 || K > kMaxChannels || !f || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    if (p->M == 0) return NFFT_OK;
    hipError_t e = ensure_channels(*p, K);
    if (e == hipSuccess) e = run_forward(*p, f, fhat, K, p->grid_many, (hipStream_t)stream);
    return hip_rc(e);
}

int nfft_forward_deriv(nfft_plan_t p, const void *f, void *dfhat, void *stream) {
    if (!p || !f || (p->M > 0 && !dfhat)) return NFFT_ERR_ARG;
    if (p->M == 0) return NFFT_OK;
    hipStream_t s = (hipStream_t)stream;
    if (p->window == NFFT_WINDOW_POLY && p->D <= 3) {
        // derivative-of-window interpolation of the one oversampled spectrum
        hipError_t e = forward_fft(*p, f, p->grid, 1, s);
        if (e == hipSuccess) e = launch_interp_deriv(*p, p->grid, dfhat, s);
        return hip_rc(e);
    }
    hipError_t e = ensure_channels(*p, p->D);
    if (e == hipSuccess) e = forward_fft(*p, f, p->grid_many, p->D, s, true);
    if (e == hipSuccess) e = launch_interp(*p, p->grid_many, dfhat, s, p->D);
    return hip_rc(e);
}

int nfft_node_grad(nfft_plan_t p, const void *a, const void *dfhat, void *grad_x, void *stream) {
    if (!p || (p->M > 0 && (!a || !dfhat || !grad_x))) return NFFT_ERR_ARG;
    return hip_rc(launch_node_grad(*p, a, dfhat, grad_x, (hipStream_t)stream));
}

int nfft_adjoint_many(nfft_plan_t p, int K, const void *fhat, void *y, void *stream) {
    if (!p || K < 1 || K > kMaxChannels || !y || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (p->M == 0)
        return hip_rc(launch_fill_zero_complex(y, (int64_t)K * p->NN, p->dtype == NFFT_C128, s));
    hipError_t e = ensure_channels(*p, K);
    if (e == hipSuccess) e = run_adjoint(*p, fhat, y, K, p->grid_many, p->pad_many, s);
    return hip_rc(e);
}

int nfft_resample_forward(nfft_plan_t p, const void *grid, void *fhat, void *stream) {
    if (!p || !grid || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    return hip_rc(launch_interp(*p, grid, fhat, (hipStream_t)stream));
}

int nfft_resample_adjoint(nfft_plan_t p, const void *fhat, void *grid, void *stream) {
    if (!p || !grid || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (p->M == 0) return hip_rc(launch_fill_zero_complex(grid, p->G, p->dtype == NFFT_C128, s));
    return hip_rc(launch_spread(*p, fhat, grid, s));
}

int nfft_plan_bench_stage(nfft_plan_t p, int stage, int reps, const void *in, void *out,
                          void *stream, double *ms) {
    if (!p || !ms || reps < 1 || (stage != 3 && stage != 4)) return NFFT_ERR_ARG;
    if (p->M > 0 && ((stage == 3 && !out) || (stage == 4 && !in))) return NFFT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = NFFT_OK;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int i = 0; i < reps && e == hipSuccess && p->M > 0; ++i)
        e = stage == 3 ? launch_interp(*p, p->grid, out, s)
                       : launch_spread(*p, in, p->grid, s, p->D != 2 && !p->sweep.on);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) *ms = (double)t / reps;
    else rc = hip_rc(e);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return rc;
}

int nfft_plan_set_timing(nfft_plan_t p, int enable) {
    if (!p) return NFFT_ERR_ARG;
    if (enable && !p->ev[0]) {
        for (int i = 0; i < 2 * NFFT_NUM_STAGES; ++i) {
            hipError_t e = hipEventCreate(&p->ev[i]);
            if (e != hipSuccess) return hip_rc(e);
        }
    }
    p->timing = enable != 0;
    for (int i = 0; i < NFFT_NUM_STAGES; ++i) p->ev_used[i] = false;
    return NFFT_OK;
}

int nfft_plan_timing(nfft_plan_t p, double *ms) {
    if (!p || !ms) return NFFT_ERR_ARG;
    for (int i = 0; i < NFFT_NUM_STAGES; ++i) {
        ms[i] = 0.0;
        if (!p->ev_used[i]) continue;
        hipError_t e = hipEventSynchronize(p->ev[2 * i + 1]);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, p->ev[2 * i], p->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_rc(e);
        ms[i] = t;
    }
    return NFFT_OK;
}

int nfft_fft_grid(nfft_plan_t p, void *grid, int direction, void *stream) {
    if (!p || !grid || (direction != -1 && direction != 1)) return NFFT_ERR_ARG;
    return hip_rc(plain_fft(*p, grid, direction, (hipStream_t)stream));
}

}  // extern "C"

// ---- multi-channel forward without allocation -----------------------------

namespace {

// Device scratch of nfft_forward_many_noalloc: the K oversampled grids of a
// call, in a file-scope device array so that the call allocates nothing.  Each
// GPU the library runs on holds its own copy of it until the process ends.
static __device__ __align__(256) unsigned char scratch[NFFT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

// Device address of device dev's copy of `scratch`, resolved once per device with
// that device current (in host code the array's name is a stand-in, not a device
// address: only the resolved pointer may be passed to kernels).
hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int nfft_forward_many_noalloc(nfft_plan_t p, int K, const void *f, void *fhat,
                                         void *stream) {
    if (!p || K < 1 || K > kMaxChannels || !f || (p->M > 0 && !fhat)) return NFFT_ERR_ARG;
    if ((uint64_t)K * (uint64_t)p->G * csize(p->dtype) > (uint64_t)NFFT_NOALLOC_SCRATCH_BYTES)
        return NFFT_ERR_SCRATCH;
    if (p->M == 0) return NFFT_OK;
    // every grid value the forward passes read is written first in the same call (the
    // first pass writes whole lines of the band rows, later passes read only those),
    // so the scratch needs no clearing between calls
    void *grids = nullptr;
    hipError_t e = scratch_address(p->device, &grids);
    if (e == hipSuccess) e = run_forward(*p, f, fhat, K, grids, (hipStream_t)stream);
    return hip_rc(e);
}
