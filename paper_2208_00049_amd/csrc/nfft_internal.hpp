// Internal interfaces of libnfft: the plan object and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "nfft.h"

namespace nfft {

constexpr int kMaxD = 6;
constexpr int kMaxRadixPasses = 16;
constexpr int kResampleThreads = 256;  // workgroup size of the resampling kernels

// Nodes per staged chunk of the resampling kernels: two per thread in 1-D and
// 2-D (a typical work item then needs one chunk), fewer in 3-D, where the
// padded tile takes most of the LDS.
constexpr int stage_chunk(int D, int rs) {
    return D < 3 ? 2 * kResampleThreads : rs == 4 ? 128 : 64;
}
// Bytes of the staged chunk: D origins, D fractions, a complex value, an index.
constexpr size_t stage_bytes(int D, int rs) {
    return (size_t)stage_chunk(D, rs) * (4 * D + rs * (D + 2) + 4);
}
// LDS of the resampling kernels besides the tile: staged chunk and the scale.
constexpr size_t resample_static_lds(int D, int rs) { return stage_bytes(D, rs) + 16; }
// Interpolation stages more nodes per chunk in 3-D complex128, whose (8, 16, 16)
// tile leaves room for one node per thread: a tile's nodes (about 256 at sigma = 2)
// then come in one chunk, instead of four chunks each behind a barrier and the
// dependent loads of its node records.
constexpr int interp_chunk(int D, int rs) { return D == 3 && rs == 8 ? 512 : stage_chunk(D, rs); }
constexpr size_t interp_static_lds(int D, int rs) {
    return (size_t)interp_chunk(D, rs) * (4 * D + rs * (D + 2) + 4) + 16;
}

struct Geom {
    int D;
    int m;
    int Nt[kMaxD];   // oversampled size per axis
    int Q[kMaxD];    // tile edge per axis (divides Nt)
    int T[kMaxD];    // tiles per axis = Nt / Q
    int ntiles;      // prod T
    int taps;        // stencil points per axis: 2m, or 2m + 2 with the wide stencil
    int lo;          // stencil points before the node's cell: taps/2 - 1
    // Sort key of a node: tile << kbits | sub-key.  The sub-key is the class (a bit
    // per axis, kbits = D; D >= 4), or the LDS bank slot of the node's first value in
    // the interpolation's LDS (slot_mod > 0: its offset in values modulo slot_mod = 32
    // for complex128, 64 for complex64, a 512-byte row of the banks; kbits = 5 or 6):
    // in the ring of the complex128 column sweeps (ring_R > 0: ring_R planes of P^2
    // values, P = kSweepQ + taps - 1), else in the work item's tile with its trailing
    // halo (Q_d + taps - 1 values per axis).  Those plans sort a second time inside
    // each tile: see launch_node_sort.
    int kbits;
    int slot_mod;
    int ring_R;
};

// Tile-owner spreading (D >= 4): a workgroup owns one tile and visits the nodes
// whose stencil reaches into it.  A node binned in tile p - b along axis d can
// reach tile p only for b <= 1 + (taps - 2) / Q_d: the candidate tiles per axis
// are r_d = min(T_d, 2 + (taps - 2) / Q_d), their product at most
// owner_max_tiles(D) = 3^D (tile edges >= taps / 2 keep r_d <= 3).
__host__ __device__ inline int owner_reach(const Geom &g, int d) {
    const int r = 2 + (g.taps - 2) / g.Q[d];
    return r < g.T[d] ? r : g.T[d];
}
constexpr int owner_max_tiles(int D) { return D <= 0 ? 1 : 3 * owner_max_tiles(D - 1); }
// Candidate nodes staged per round by the tile-owner kernels (their box weights
// take at most about 32 KiB in c64, 16 KiB in c128, whose accumulator tile is
// twice as large), and the kernels' static LDS: staged candidates (sorted
// position and 3 ints per axis; D fractions, a value, the box weights), the
// candidate-tile ranges and the scale word.  Every round ends in a barrier
// behind the dependent loads node record -> perm -> fhat, so larger rounds
// expose that latency less often (4-D c64, m = 4: 128 -> 256 candidates,
// spreading 548 -> 520 us).
constexpr int owner_chunk_n(int D, int taps, int rs) {
    const int w = (rs == 4 ? 32768 : 16384) / (D * taps * rs);
    return w >= 256 ? 256 : w >= 128 ? 128 : w >= 64 ? 64 : 32;
}
constexpr size_t owner_static_lds(int D, int taps, int rs) {
    return (size_t)owner_chunk_n(D, taps, rs) * (4 * (1 + 3 * D) + (size_t)rs * (D + 2 + D * taps)) +
           4 * (2 * owner_max_tiles(D) + 3) + 256;
}
// Workgroup of the tile-owner spreading kernel: 1024 threads, 16 wavefronts per
// CU (the tile's accumulators take most of the LDS, one workgroup fits per CU),
// which hide the staging and box-walk latencies: 4-D 16^4 c64 spreading 770 -> 548
// us, c128 1105 -> 872 us against 512 threads.
constexpr int kOwnerThreads = 1024;
// Bytes per grid point of its LDS tile: 64-bit fixed-point slots, 2 (c64) or 4 (c128).
inline size_t owner_cell_bytes(int cs) { return cs == 8 ? 16 : 32; }

// LDS layout of the tile-owner accumulators: strides per axis and the cells of
// one accumulator plane.  A wavefront adds to a box spanning several rows (axis
// D-2) and planes (axis D-3) of the tile at once; with a row-major 8^4 tile the
// planes lie 64 cells apart, on the same LDS banks, and the 64-bit atomics of
// one instruction collide 3.8-fold on average (a count over all node offsets).
// Padding the rows by one cell and the planes by four brings that to 2.4, at
// 19 % more LDS; the padded layout is used where it fits.
struct OwnerLayout {
    int S[kMaxD];
    int cells;
};
inline OwnerLayout owner_layout(const Geom &g, int D, bool pad) {
    OwnerLayout l{};
    l.S[D - 1] = 1;
    for (int d = D - 2; d >= 0; --d) {
        l.S[d] = g.Q[d + 1] * l.S[d + 1];
        if (pad && d == D - 2) l.S[d] += 1;
        if (pad && d == D - 3) l.S[d] += 4;
    }
    l.cells = g.Q[0] * l.S[0];
    return l;
}

// Cells of a tile extended by the (2m-1)-wide trailing halo of every axis.
inline size_t padded_cells(const Geom &g, int D) {
    size_t c = 1;
    for (int d = 0; d < D; ++d) c *= (size_t)(g.Q[d] + g.taps - 1);
    return c;
}

// Sorted node record: stencil origin (c - m + 1) mod Nt per axis and the
// fractional cell offset frac = Nt*x - floor(Nt*x) in [0, 1).
template <typename T, int D> struct NodeRec {
    int o[D];
    T fr[D];
};

// Three-dimensional column-sweep spreading (spread_sweep.hip): columns of
// kSweepQ x kSweepQ grid points along axes 1 and 2, each cut into nsc segments
// of L tiles along axis 0; a segment's workgroup keeps a ring of R = Q_0 + taps - 1
// padded planes in LDS.  Scratch per channel: main_cells values (every grid plane
// of every column, padded to (kSweepQ + taps - 1)^2 points), then per segment its
// taps - 1 trailing halo planes, then the kSweepParts block maxima of |Re|, |Im| of
// fhat (doubles, one per complex slot).
constexpr int kSweepQ = 16;
constexpr int kSweepMaxSegTiles = 64;
constexpr int kSweepParts = 256;  // blocks of the fhat maximum
struct SweepGeom {
    int on;              // 1: the plan spreads by column sweeps
    int ncols;           // columns (T_1 T_2)
    int nsc;             // segments per column
    int L;               // tiles per segment (divides T_0)
    int R;               // ring planes
    long long main_cells;
    long long part_off;    // offset of the block maxima (main + halo values)
};

// Factorisation of one FFT line length and its twiddle table exp(-2 pi i t / L).
struct FftLine {
    int L;
    int npass;
    int rad[kMaxRadixPasses];
    int tpl;              // threads per line = L / largest radix
    const void *tw;       // device, L complex values of the plan's type
    int tw_lds;           // 1: a pass copies the table into LDS (it fits beside its lines)
};

// One axis pass of the oversampled FFT over a grid viewed as [outer][L][inner].
struct AxisPass {
    int axis;
    int inner;            // prod of Nt over the axes after `axis` (> 1: strided pass)
    int outer_len;        // number of outer (prefix) positions processed = prod outer_n
    // the outer positions enumerate the axes 0..axis-1 (the last fastest): per axis
    // outer_n[d] positions, either the band of I_N (outer_band[d], n_d -> n_d mod Nt)
    // or 0..outer_n[d]-1; outer_stride[d] = elements between consecutive grid rows of d
    int outer_n[kMaxD];
    int outer_band[kMaxD];
    int outer_Nt[kMaxD];
    long long outer_stride[kMaxD];
    int in_band_N;        // 0: load the whole line; else only the band rows (others are zero)
    int out_band_N;       // 0: store the whole line; else only the band rows
    int lines_per_block;  // B, a power of two
    int dir;              // -1 forward, +1 adjoint
    int K;                // channels (grid blockIdx.y), each a whole grid
    long long cstride;    // elements between the channels' grids
};

// Last-axis pass with the resampling correction fused in.
// Source of the first adjoint axis pass when it also performs the halo merge
// of spreading: the padded tiles of the work items (see the merge kernel).
struct PadSource {
    const void *pad;      // nsub padded tiles, complex
    const int *tile_sub;  // ntiles + 1: first work item of each tile
    Geom g;
    int M2;               // 2m
    long long cstride;    // elements between the channels' sets of padded tiles
};

// Source of the first adjoint axis pass when it also merges the column sweeps
// of 3-D spreading (see the sweep's merge kernel).
struct SweepSource {
    const void *scr;      // channel 0's sweep scratch, complex
    SweepGeom sg;
    Geom g;
    long long cstride;    // values between the channels' scratch
};

struct ContigPass {
    int mode;             // 0 plain grid->grid, 1 f -> grid (deconv + pad), 2 grid -> y (crop + deconv)
    int D;
    int nlines;           // number of lines processed
    int outer_len[kMaxD - 1];   // lengths of the outer axes 0..D-2 as enumerated
    int outer_band[kMaxD - 1];  // per outer axis: 1 = band of I_N, 0 = full
    int N[kMaxD];
    int Nt[kMaxD];
    int lines_per_block;
    int dir;
    int K;                  // channels (grid blockIdx.y)
    long long src_cstride;  // elements between channels of src
    long long dst_cstride;  // elements between channels of dst
    int deriv;              // mode 1, K = D: channel d takes -2 pi i n_d f (one shared f)
};

}  // namespace nfft

struct nfft_plan_s {
    int D;
    int64_t N[nfft::kMaxD];
    int64_t Nt[nfft::kMaxD];
    int64_t M;
    int m;
    double sigma;
    nfft_dtype dtype;
    int window;
    int wide;             // (2m+2)-point stencil
    int max_block_nodes;
    nfft::Geom geom;
    int64_t G;            // prod Nt
    int64_t NN;           // prod N
    int nkeys;            // ntiles << geom.kbits
    int nsub;             // resampling work items
    int device;
    int lds_limit;        // LDS per workgroup of the device, bytes

    // device buffers
    void *grid = nullptr;          // G complex
    void *deconv[nfft::kMaxD] = {};  // N_d reals (plan type)
    void *coef = nullptr;          // 2m x (2m+1) reals (plan type), window polynomial
    void *nodes = nullptr;         // M sorted NodeRec
    int *perm = nullptr;           // M: sorted position -> caller's node index
    int *key_start = nullptr;      // nkeys + 1
    int4 *subs = nullptr;          // nsub work items {tile, begin, end, 0}, grouped by tile
    int *tile_sub = nullptr;       // ntiles + 1: first work item of each tile
    void *pad = nullptr;           // nsub padded tiles (spreading scratch, D <= 3), complex
    void *wtab = nullptr;          // window tables: TENSOR / FULL per sorted node, LINEAR per axis
    long long lin_S = 0;           // LINEAR: entries per axis
    // multi-channel calls: K grids and K sets of padded tiles, grown on demand
    void *grid_many = nullptr;
    void *pad_many = nullptr;
    int many_cap = 0;              // channels the two buffers hold
    void *twiddle[nfft::kMaxD] = {};
    nfft::FftLine line[nfft::kMaxD];
    nfft::SweepGeom sweep{};       // 3-D column-sweep spreading (sweep.on)

    // optional per-stage timing (events recorded around each kernel launch)
    bool timing = false;
    hipEvent_t ev[2 * NFFT_NUM_STAGES] = {};
    bool ev_used[NFFT_NUM_STAGES] = {};
};

namespace nfft {

// Kaiser-Bessel shape parameter of axis d: beta = pi m (2 - 1/sigma_d), sigma_d = Nt_d / N_d.
inline double kb_beta(const nfft_plan_s &p, int d) {
    return M_PI * p.m * (2.0 - (double)p.N[d] / (double)p.Nt[d]);
}

// Peak of the convolution-side window of axis d, psi_hat_Base(0) = sinh(beta) / pi.
// The library keeps the window divided by this constant (its maximum is then 1 on
// every axis) and the resampling-correction factors multiplied by it.  The product
// of the two factors -- all the transform depends on -- is unchanged, and neither
// factor leaves the float range: the raw peaks multiply to sinh(beta)^D / pi^D, which
// overflows float for m D >= 24 or so, and the raw correction factors to its
// reciprocal, which underflows.
inline double window_peak(const nfft_plan_s &p, int d) { return sinh(kb_beta(p, d)) / M_PI; }

// Product over the axes of the normalised window's maximum (1), with a margin for
// the polynomial fit's overshoot (largest at m = 1: 4.6 % above the peak for sigma up
// to 16, under 1e-6 from m = 3): the bound of |weight product| the fixed-point
// spreading scales by.
inline double window_bound(int D) {
    double w = 1.0;
    for (int d = 0; d < D; ++d) w *= 1.0625;
    return w;
}

// plan.cpp: the argument checks of plan creation (no HIP call)
int validate_plan_args(int D, const int64_t *N, int64_t M, const void *x, int m, double sigma,
                       int dtype, const nfft_options *opts);

// precompute.hip
hipError_t launch_deconv_factors(const nfft_plan_s &p, hipStream_t s);
hipError_t launch_window_poly(const nfft_plan_s &p, const double *qt, const double *r, int Z,
                              int Theta, hipStream_t s);
hipError_t launch_twiddles(const nfft_plan_s &p, int axis, hipStream_t s);
// TENSOR / FULL weights of the sorted nodes, or the LINEAR tables (plan's window mode)
hipError_t launch_window_tables(const nfft_plan_s &p, hipStream_t s);

// binsort.hip
hipError_t launch_fill_int(int *a, int64_t n, int v, hipStream_t s);
hipError_t launch_fill_zero_complex(void *a, int64_t n, bool dbl, hipStream_t s);
hipError_t launch_node_keys(const nfft_plan_s &p, const void *x, int *keys, int *counts, int *bad,
                            hipStream_t s);
hipError_t launch_exclusive_scan(const int *in, int *out, int n, hipStream_t s);
// Stable bin sort: keys_sorted and idx hold M ints; tmp is node_sort_bytes() bytes.
hipError_t node_sort_bytes(const nfft_plan_s &p, size_t *bytes);
hipError_t launch_node_sort(nfft_plan_s &p, const void *x, int *keys, int *keys_sorted,
                            int *idx, void *tmp, size_t tmp_bytes, hipStream_t s);
hipError_t launch_subprob_count(const nfft_plan_s &p, int *counts, hipStream_t s);
hipError_t launch_subprob_fill(nfft_plan_s &p, const int *sub_start, hipStream_t s);

// fft.hip
hipError_t launch_fft_axis(const nfft_plan_s &p, void *grid, const AxisPass &a, hipStream_t s);
// axis-0 adjoint pass reading the merged padded tiles instead of the grid (D >= 2)
hipError_t launch_fft_axis0_from_pad(const nfft_plan_s &p, void *grid, const AxisPass &a,
                                     const void *pad, hipStream_t s);
// axis-0 adjoint pass reading and merging the column sweeps' scratch (3-D sweep plans)
hipError_t launch_fft_axis0_from_sweep(const nfft_plan_s &p, void *grid, const AxisPass &a,
                                       const void *scr, hipStream_t s);
hipError_t launch_fft_contig(const nfft_plan_s &p, const void *src, void *dst, const ContigPass &c,
                             hipStream_t s);

// ---- fused batches (runtime.cpp): one launch per stage for all transforms ----
//
// Block b of a stage launch serves entry b2e[b] of the stage's table (-1: an idle
// block; every entry's range starts at a multiple of the XCD count, so that the
// kernels' XCD-aware renumbering of their blocks holds inside the range) as block
// b - start of that entry's own pass.  `t` indexes the caller's pointer arrays.
struct BxFft {
    int t;
    int start, nblk;
    int src_user, dst_user;  // last-axis pass: read the caller's input / write its output
    const void *src;         // last-axis pass: the source when it is not the caller's
    void *grid;              // the plan's grid (a strided pass's data, a last-axis destination)
    FftLine fl;
    ContigPass c;
    AxisPass a;
    PadSource ps;            // first adjoint pass with the halo merge (2-D)
    const void *dec[kMaxD];  // resampling-correction factors
};
struct BxResample {
    int t;
    int start, nblk;
    void *buf;               // interpolation: the plan's grid; spreading, merge: its padded tiles
    void *grid;              // merge: the plan's grid
    Geom g;
    const void *nodes;
    const int *perm;
    const int4 *subs;
    const int *tile_sub;
    const void *coef;
    int window;
    int m;
    double beta[kMaxD];
    double inv_peak[kMaxD];
    const void *tab;
    long long S;
    double wmax_prod;
};
enum BatchFftKind { kBxContig = 0, kBxStrided = 1, kBxFromPad = 2 };
enum BatchResampleKind { kBxInterp = 0, kBxSpread = 1, kBxMerge = 2 };
// fft.hip / resample.hip: one stage launch over nblocks blocks of nthreads threads
hipError_t launch_fft_batch(int kind, int dtype, int D, int dir, bool pow2, const BxFft *tab,
                            const int *b2e, const void *const *in, void *const *out, int nblocks,
                            int nthreads, size_t shm, hipStream_t s);
hipError_t launch_resample_batch(int kind, int dtype, int D, int taps, bool gw, const BxResample *tab,
                                 const int *b2e, const void *const *in, void *const *out,
                                 int nblocks, size_t shm, hipStream_t s);
// threads of the resampling kernels' workgroups (256, 512 in 3-D)
int resample_block_threads(int D);

constexpr int kLinePad = 1;  // complex values of padding after each LDS line of an FFT pass
// The twiddle table goes to LDS when the pass's B lines leave room for it; shm: the
// pass's dynamic LDS (lines and table).
inline FftLine with_lds_table(const nfft_plan_s &p, const FftLine &fl, int B, size_t cs, size_t &shm) {
    FftLine out = fl;
    const size_t lines = (size_t)B * (fl.L + kLinePad) * cs;
    out.tw_lds = lines + (size_t)fl.L * cs <= (size_t)p.lds_limit;
    shm = lines + (out.tw_lds ? (size_t)fl.L * cs : 0);
    return out;
}

// plan.cpp: the FFT passes of a plan.  contig_pass: the last-axis pass (mode 1: f ->
// grid with the resampling correction and zero padding; mode 2: grid -> y with crop
// and correction; mode 0: plain grid -> grid).  axis_pass: the strided pass along
// axis a < D - 1, direction dir; pruned: the forward loads, the adjoint stores,
// only the band rows of I_N, and the axes before a hold only their band.
ContigPass contig_pass(const nfft_plan_s &p, int mode, int dir, int K);
AxisPass axis_pass(const nfft_plan_s &p, int a, int dir, int K, bool pruned);

// resample.hip
// out[j*D + d] = Re(conj(a_j) v[d*M + j]) for the plan's M nodes
hipError_t launch_node_grad(const nfft_plan_s &p, const void *a, const void *v, void *out,
                            hipStream_t s);

// K channels: grids at stride G, fhat at stride M, padded tiles at stride pad_elems()
hipError_t launch_interp(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                         int K = 1);
// resample_nd.hip: the resampling kernels of D = 4, 5, 6 (K channels)
hipError_t launch_interp_nd(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                            int K);
hipError_t launch_spread_nd(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                            int K);
// derivative-of-window interpolation, D <= 3 with the polynomial window: dfhat D x M
hipError_t launch_interp_deriv(const nfft_plan_s &p, const void *grid, void *dfhat, hipStream_t s);
// merge = false: only the padded tiles are produced (the next pass merges them)
hipError_t launch_spread(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                         bool merge = true, int K = 1, void *pad = nullptr);

// spread_sweep.hip: column-sweep spreading (the fhat gather and the sweep) and, with
// merge, the merge into grid (K channels); without, the first adjoint FFT pass merges
hipError_t launch_spread_sweep(const nfft_plan_s &p, const void *fhat, void *grid, hipStream_t s,
                               int K, void *pad, bool merge);
// static LDS of the sweep kernel (staged chunk, segment tables)
size_t sweep_static_lds(int dtype);
// interpolation by column sweeps (the same segments; complex128 plans): K channels
hipError_t launch_interp_sweep(const nfft_plan_s &p, const void *grid, void *fhat, hipStream_t s,
                               int K);
// LDS of the interpolation sweep: a ring of R planes of values and the staged chunk
size_t interp_sweep_lds(int dtype, int R, int taps);
// points of one padded column plane
inline int sweep_plane_cells(int taps) { return (kSweepQ + taps - 1) * (kSweepQ + taps - 1); }
// The sweep with 2m = 8 and the polynomial window maps one node to a wavefront,
// lanes over (axis-0 tap, axis-2 tap): an atomic instruction then adds to eight
// runs of eight consecutive words, one per ring plane, and a plane stride of 8
// words modulo 32 puts every four runs on disjoint LDS banks (3-D 128^3 spreading:
// complex128 1.07 -> 0.75 ms with the FP64 atomics it used then, complex64 0.63 ->
// 0.59 ms with 64-bit integer ones, whose rate depends less on the access pattern).
__host__ __device__ constexpr bool sweep_wave_node(int taps, bool poly) { return taps == 8 && poly; }
// 8-byte words per ring plane: Re and Im of every point, padded as above
__host__ __device__ constexpr int sweep_plane_stride(int taps, bool wave_node) {
    return 2 * (kSweepQ + taps - 1) * (kSweepQ + taps - 1) +
           (wave_node ? (8 - (2 * (kSweepQ + taps - 1) * (kSweepQ + taps - 1)) % 32 + 32) % 32 : 0);
}
// dynamic LDS of the sweep kernel: R planes of 8-byte words
inline size_t sweep_ring_bytes(int R, int taps, bool wave_node) {
    return (size_t)R * sweep_plane_stride(taps, wave_node) * 8;
}
inline size_t sweep_ring_bytes(const nfft_plan_s &p) {
    return sweep_ring_bytes(p.sweep.R, p.geom.taps,
                            sweep_wave_node(p.geom.taps, p.window == NFFT_WINDOW_POLY));
}
// scratch values per channel: the column planes and the segments' halo planes
inline size_t sweep_scratch_cells(const nfft_plan_s &p) {
    return (size_t)p.sweep.part_off + kSweepParts;
}

}  // namespace nfft
