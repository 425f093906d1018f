/*
 * libnfft -- nonequispaced fast Fourier transform (NFFT) on one AMD Instinct
 * MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The transform (Knopp, Boberg, Grosser, "NFFT.jl: Generic and Fast Julia
 * Implementation of the Nonequidistant Fast Fourier Transform", section
 * "Mathematical Description"):
 *
 *   forward (type 2, Algorithm 1 "Direct NFFT") approximates the NDFT
 *       fhat_j = sum_{n in I_N} f_n exp(-2 pi i n . x_j),   j = 0..M-1
 *   adjoint (type 1, Algorithm 2 "Adjoint NFFT") approximates
 *       y_n    = sum_j fhat_j exp(+2 pi i n . x_j),         n in I_N
 *
 * with I_N the centred index set (n_d = -floor(N_d/2) .. N_d - 1 - floor(N_d/2): for even
 * N_d -N_d/2 .. N_d/2-1, for odd N_d -(N_d-1)/2 .. (N_d-1)/2), an
 * oversampled grid Ntilde_d ~= sigma N_d, and a Kaiser-Bessel window truncated to
 * 2m grid points per axis.  Both are computed as resampling correction
 * (deconvolution), unnormalised oversampled FFT and window resampling
 * (interpolation for the forward transform, spreading for the adjoint), in the
 * matrix form A ~= B F D and A^H ~= D^T F^H B^T of subsection
 * "Matrix-Vector Notation".  The adjoint is not an inverse.
 *
 * Layouts (all device memory, C row-major, last axis fastest):
 *   x      M*D reals, node-major: x[j*D + d].  float for NFFT_C64, double for
 *          NFFT_C128.  Any real value is accepted; nodes are taken modulo 1
 *          (the transform is 1-periodic in x).
 *   f, y   prod(N) complex values (interleaved re, im), storage index
 *          i_d = n_d + floor(N_d/2) (centred).
 *   fhat   M complex values in the caller's node order.
 *
 * Ownership: the caller owns x, f, fhat and y.  A plan copies what it needs
 * from x while it is created and keeps no pointer to it.  The plan owns its
 * oversampled grid, sorted nodes and precomputed factors.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Transforms
 * are enqueued asynchronously on it.  Calls on one plan must be ordered (one
 * stream, or synchronised) because they share the plan's grid; a plan is not
 * re-entrant.  Plan creation synchronises `stream` before returning.
 *
 * Errors: every call returns an int status (NFFT_OK or a negative code) and
 * never throws.  Arguments are validated before any HIP call, so argument
 * errors are reported without touching the GPU.
 */
#ifndef NFFT_MI355X_H
#define NFFT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfft_plan_s *nfft_plan_t;

typedef enum {
    NFFT_C64 = 0,  /* complex float data, float nodes, FP32 accumulation */
    NFFT_C128 = 1  /* complex double data, double nodes, FP64 throughout */
} nfft_dtype;

enum {
    NFFT_OK = 0,
    NFFT_ERR_ARG = -1,         /* invalid argument (null pointer, bad size, sigma <= 1, ...) */
    NFFT_ERR_UNSUPPORTED = -2, /* valid per the paper but outside this library (D > 6, ...) */
    NFFT_ERR_NOMEM = -3,       /* device allocation failed */
    NFFT_ERR_HIP = -4,         /* a HIP runtime call failed (no device, launch failure, ...) */
    NFFT_ERR_NODES = -5,       /* a node coordinate is NaN or infinite */
    NFFT_ERR_SCRATCH = -6      /* request larger than the static scratch (no-allocation call) */
};

/* Window evaluation inside the resampling kernels. */
enum {
    NFFT_WINDOW_POLY = 0,   /* piecewise polynomial of degree 2m per tap, least-squares fit
                               to the Kaiser-Bessel window in FP64 (the paper's POLYNOMIAL
                               precomputation, subsection "Window precomputation") */
    NFFT_WINDOW_DIRECT = 1, /* evaluate sinh(beta sqrt(1-u^2)) / (pi sqrt(1-u^2)) per tap
                               (the paper's "no precomputation" option) */
    NFFT_WINDOW_TENSOR = 2, /* the paper's TENSOR precomputation: the plan stores, per node
                               and axis, the 2m polynomial-window weights (2m D M values) */
    NFFT_WINDOW_LINEAR = 3, /* the paper's LINEAR precomputation: a table of
                               S = m 2^c + 2 window samples per axis (c = 3, 7, 9, 14, 17,
                               20, 23, 24 for m = 1..8, 24 above), linear interpolation */
    NFFT_WINDOW_FULL = 4    /* the paper's FULL precomputation: per node all (2m)^D weight
                               products (the nonzeros of the sparse matrix B); D <= 2,
                               D >= 3 returns NFFT_ERR_UNSUPPORTED */
};

typedef struct {
    int tile[4];          /* tile edge per axis in grid points, all 0 = automatic.  D <= 3:
                             must divide Ntilde_d, be >= the stencil width and leave >= 2
                             tiles per axis.  D = 4: must divide Ntilde_d; the spreading
                             workgroup of a tile reads at most 81 tiles' nodes, the product
                             over the axes of min(Ntilde_d/Q_d, 2 + (taps-2)/Q_d), else
                             NFFT_ERR_UNSUPPORTED.  D >= 5: must be all 0 (automatic
                             tiles), else NFFT_ERR_UNSUPPORTED. */
    int window;           /* NFFT_WINDOW_POLY (default), _DIRECT, _TENSOR, _LINEAR or _FULL */
    int max_block_nodes;  /* cap on nodes per resampling work item (a tile's nodes are cut
                             into items of at most this many), 0 = automatic (D <= 3: 1024,
                             512 in 1-D/2-D when the tiles hold <= 512 nodes on average;
                             16 for D >= 4, whose interpolation takes one wavefront per
                             node) */
    int wide;             /* 1: (2m+2)^D-point stencil with the untruncated window, sampled
                             beyond its truncation interval (the alternative of subsection
                             "Window Size Considerations"); 0 (default): 2m points.  Not
                             available with NFFT_WINDOW_LINEAR. */
    int spread;           /* 3-D spreading scheme: NFFT_SPREAD_AUTO (0, default): column
                             sweeps where available, else padded tiles; NFFT_SPREAD_TILED:
                             padded tiles merged afterwards, exact fixed-point sums in both
                             types (bitwise reproducible); NFFT_SPREAD_SWEEP: column sweeps,
                             NFFT_ERR_UNSUPPORTED where not available.  Column sweeps need
                             D = 3, Ntilde_1 and Ntilde_2 multiples of 16 (>= 32), 2m <= 10,
                             the 2m-point stencil and tiles of 16 along axes 1 and 2;
                             complex64 sums stay exact, complex128 sums use FP64 LDS
                             atomics (correct to rounding; the last bits can differ between
                             calls).  Ignored for D != 3. */
    int reserved[2];      /* must be zero */
} nfft_options;

enum { NFFT_SPREAD_AUTO = 0, NFFT_SPREAD_TILED = 1, NFFT_SPREAD_SWEEP = 2 };

/*
 * Create a plan (Algorithm 1/2 inputs D, m, N, Ntilde and the nodes).
 *   out    receives the plan handle (unchanged on error)
 *   D      1 .. 6.  D <= 3 resamples through LDS tiles of the grid; D >= 4
 *          (whose tile plus stencil halo does not fit in LDS) interpolates from
 *          the grid in device memory, one wavefront per node, and spreads
 *          tile by tile: a workgroup owns one tile and adds every node whose
 *          stencil reaches it in exact fixed point (no global atomics, no
 *          scratch, bitwise reproducible).  D >= 4 needs D * taps <= 128
 *          (taps = 2m, or 2m + 2 with the wide stencil), else
 *          NFFT_ERR_UNSUPPORTED; D >= 5 takes its tiles automatically.
 *   N      host array of D sizes >= 2 (even or odd)
 *   M      number of nodes, >= 0 (M = 0 is allowed)
 *   x      device pointer to the nodes (may be NULL when M == 0)
 *   m      window half-width, 1..10 (the range the paper studies is 3..10)
 *   sigma  oversampling factor > 1; Ntilde_d is the smallest even integer >=
 *          sigma N_d whose prime factors are 2, 3 and 5 (see nfft_plan_info)
 *   dtype  NFFT_C64 or NFFT_C128
 *   opts   NULL for defaults (nfft_plan_create_ex only)
 * Work done on `stream`: FP64 Kaiser-Bessel deconvolution factors and window
 * polynomial, node wrap / cell / fraction in FP64, GPU bin sort of the nodes
 * into grid tiles.  Returns NFFT_ERR_NODES if a node is NaN or infinite.
 */
int nfft_plan_create(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x,
                     int m, double sigma, nfft_dtype dtype, void *stream);
int nfft_plan_create_ex(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x,
                        int m, double sigma, nfft_dtype dtype, const nfft_options *opts,
                        void *stream);

/* Release a plan and its device memory (waits for work queued on the plan's grid
 * by synchronising the device).  NULL is accepted. */
int nfft_plan_destroy(nfft_plan_t p);

/*
 * Forward NFFT (Algorithm 1): fhat = B F D f.  f: prod(N) complex (device),
 * fhat: M complex (device), overwritten (mul! semantics).  With M == 0 nothing
 * is computed.
 */
int nfft_forward(nfft_plan_t p, const void *f, void *fhat, void *stream);

/*
 * Adjoint NFFT (Algorithm 2): y = D^T F^H B^T fhat.  fhat: M complex (device),
 * y: prod(N) complex (device), overwritten.  With M == 0, y is set to zero.
 * Non-finite input: if any fhat value has a NaN or infinite part, every value of
 * y is NaN (spreading accumulates in fixed point, where such a value would be
 * lost; the work items holding one write NaN instead, and the FFT spreads it).
 * The forward transform propagates a non-finite f value by IEEE arithmetic
 * through its FFT (every fhat value non-finite).
 */
int nfft_adjoint(nfft_plan_t p, const void *fhat, void *y, void *stream);

/*
 * Multi-channel transforms: K vectors through the same node set (the
 * paper's transforms applied column by column to a K-column input).
 * Forward: f holds K arrays of prod(N) complex values one after the other
 * (channel-major), fhat K arrays of M.  Adjoint: fhat K x M in, y K x prod(N)
 * out.  Every channel gives exactly what nfft_forward / nfft_adjoint give for
 * it; the K channels share each kernel launch (second grid dimension).
 * 1 <= K <= 65535.  The plan keeps K grids and K sets of spreading scratch:
 * the first call with a K larger than any before allocates them (hipMalloc),
 * later calls with K up to that allocate nothing.
 */
int nfft_forward_many(nfft_plan_t p, int K, const void *f, void *fhat, void *stream);
int nfft_adjoint_many(nfft_plan_t p, int K, const void *fhat, void *y, void *stream);

/*
 * Multi-channel forward transform that allocates nothing, for callers that
 * cannot call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Arguments, layouts and results are those
 * of nfft_forward_many (bit for bit: the same kernels), but the K oversampled
 * grids live in a static device array of NFFT_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on every GPU it runs on until the process ends, instead of
 * the plan's multi-channel buffers.  Requires K * prod(Ntilde) * (8 for
 * NFFT_C64, 16 for NFFT_C128) <= NFFT_NOALLOC_SCRATCH_BYTES, else returns
 * NFFT_ERR_SCRATCH without touching the GPU.  The array is shared by every
 * plan on a GPU: calls on one GPU whose executions overlap (other streams,
 * other threads) race on it and must be ordered by the caller.  Its contents
 * after a call are those of that call's grids; nothing needs to be cleared.
 */
#define NFFT_NOALLOC_SCRATCH_BYTES (64u << 20)
int nfft_forward_many_noalloc(nfft_plan_t p, int K, const void *f, void *fhat, void *stream);

/*
 * Derivatives with respect to the nodes (for differentiable use).
 *   nfft_forward_deriv: dfhat[d][j] ~= sum_{n in I_N} (-2 pi i n_d) f_n exp(-2 pi i n.x_j),
 *     the partial derivative of the forward transform's output j along axis d.
 *     With the polynomial window and D <= 3 it is the derivative of the NFFT
 *     itself: one resampling correction + FFT of f, then interpolation with the
 *     derivative of the window along axis d (Nt_d P'_t(frac - 1/2)) -- the exact
 *     gradient of what nfft_forward computes.  Otherwise it is D forward NFFTs of
 *     the coefficients -2 pi i n_d f_n (one multi-channel call that reads f once;
 *     the factor is applied in the resampling-correction pass; uses the plan's
 *     multi-channel buffers, K = D).  f: prod(N) complex; dfhat: D x M complex
 *     (axis-major), device.
 *   nfft_node_grad: grad_x[j*D + d] = Re(conj(a_j) dfhat[d][j]) for j < M, d < D
 *     (a: M complex; grad_x: M x D reals of the plan's real type, node-major like
 *     the nodes).  With a = the gradient of a real loss with respect to the
 *     forward output (the conjugate-Wirtinger convention: 2 dL/d conj(fhat)),
 *     grad_x is dL/dx for the forward transform.  For the adjoint transform
 *     y = A^H fhat, dL/dx[j, d] = Re(conj(fhat_j) w[d][j]) with w =
 *     nfft_forward_deriv of the gradient with respect to y.
 */
int nfft_forward_deriv(nfft_plan_t p, const void *f, void *dfhat, void *stream);
int nfft_node_grad(nfft_plan_t p, const void *a, const void *dfhat, void *grad_x, void *stream);

/*
 * Batches of independent transforms (different plans, sizes and node sets:
 * the paper's plan/apply interface, section "Implementation", applied to many
 * plans at once; each transform is Algorithm 1 / Algorithm 2 of its plan).
 * nfft_batch_create takes n distinct plans (a plan may appear once: its grid
 * serves one transform at a time) and a stream count (1..16).
 *
 * Fused mode: when the plans share the complex type, D <= 3, the stencil
 * width, the polynomial window and the padded-tile spreading (not the 3-D
 * column sweeps), every stage of the transform chain -- each FFT pass, the
 * interpolation, the spreading and its halo merge -- is ONE kernel launch over
 * the work of all n transforms (2-D: three launches per direction; 1-D: two /
 * three; 3-D: four / five).  The launches of a direction are captured into a
 * HIP graph on the first call of that direction and replayed; results equal
 * those of the plans' own nfft_forward / nfft_adjoint calls bit for bit.
 * Otherwise each transform's kernel chain is captured into one graph over up
 * to `nstreams` streams (recaptured whenever a pointer differs from the
 * previous call's).
 *
 * nfft_batch_forward / nfft_batch_adjoint take host arrays of n device
 * pointers (in[i], out[i] as for nfft_forward / nfft_adjoint of plan i) and
 * launch on `stream`.  When a pointer differs from the direction's previous
 * call the fused mode drains `stream` and rewrites its device pointer table
 * (a synchronous copy); with unchanged pointers a call only launches.  Calls of
 * one batch must not overlap (the plans' grids are shared).  The plans must
 * outlive the batch; their per-stage timing is not recorded in batch calls.
 * nfft_batch_info reports the mode (fused: 1) and, in fused mode, the kernel
 * launches per forward and per adjoint call (NULL outputs are skipped).
 * nfft_batch_destroy synchronises the device.  Errors: NFFT_ERR_ARG (NULL or
 * repeated plans, NULL pointers where the plan needs data), NFFT_ERR_NOMEM,
 * NFFT_ERR_HIP.
 */
typedef struct nfft_batch_s *nfft_batch_t;
int nfft_batch_create(nfft_batch_t *out, int n, const nfft_plan_t *plans, int nstreams);
int nfft_batch_forward(nfft_batch_t b, const void *const *f, void *const *fhat, void *stream);
int nfft_batch_adjoint(nfft_batch_t b, const void *const *fhat, void *const *y, void *stream);
int nfft_batch_info(nfft_batch_t b, int *fused, int *launches_forward, int *launches_adjoint);
int nfft_batch_destroy(nfft_batch_t b);

/*
 * Plan creation with tile autotuning: arguments as nfft_plan_create_ex.
 * Unless opts fixes the tiles, plans are built for a short list of candidate
 * tiles (then work-item caps for the best tile), forward + adjoint is timed
 * `reps` times on `stream` for each, and the fastest plan is returned (its
 * tiles: nfft_plan_info; its mean forward + adjoint milliseconds: *best_ms,
 * which may be NULL).  Costs one plan creation and reps + 1 transform pairs per
 * candidate.
 */
int nfft_plan_create_tuned(nfft_plan_t *out, int D, const int64_t *N, int64_t M, const void *x,
                           int m, double sigma, nfft_dtype dtype, const nfft_options *opts,
                           int reps, void *stream, double *best_ms);

/*
 * The single steps, for step-wise checking and timing.  `grid` is a device
 * array of prod(Ntilde) complex values, row-major, storage index l mod Ntilde
 * (DC first).  The plan stores the window divided by its peak per axis,
 * C = prod_d psi_hat_Base(0) = prod_d sinh(beta_d)/pi (nfft_plan_window_peak), and
 * the resampling-correction factors multiplied by it, so that neither leaves the
 * float range (the transforms themselves are unchanged by this).  The steps use
 * the stored window:
 *   nfft_resample_forward : fhat_j = (1/C) sum_l ghat_l psi_tilde(x_j - l/Ntilde)
 *                           (Algorithm 1, resampling step; reads grid)
 *   nfft_resample_adjoint : ghat_l = (1/C) sum_j fhat_j psi_tilde(x_j - l/Ntilde)
 *                           (Algorithm 2, adjoint resampling; overwrites grid)
 *   nfft_fft_grid         : unnormalised D-variate FFT of grid in place;
 *                           direction -1 = forward (exp(-2 pi i n.l/Ntilde)),
 *                           +1 = adjoint (exp(+2 pi i ...)).
 * After nfft_forward the plan's grid (nfft_plan_grid) holds C F D f.
 */
int nfft_resample_forward(nfft_plan_t p, const void *grid, void *fhat, void *stream);
int nfft_resample_adjoint(nfft_plan_t p, const void *fhat, void *grid, void *stream);
int nfft_fft_grid(nfft_plan_t p, void *grid, int direction, void *stream);

/*
 * Introspection.  Ntilde receives D sizes, sigma_eff = Ntilde_0 / N_0, tile receives
 * D tile edges (any output pointer may be NULL).
 */
int nfft_plan_info(nfft_plan_t p, int64_t *Ntilde, double *sigma_eff, int *tile);

/* Device pointer to the plan's oversampled grid (prod(Ntilde) complex): after
 * nfft_forward it holds C ghat = C F D f (C: nfft_plan_window_peak), after
 * nfft_adjoint it is scratch. */
int nfft_plan_grid(nfft_plan_t p, void **grid);

/* The window peak per axis, peak[d] = psi_hat_Base(0) = sinh(beta_d)/pi with
 * beta_d = pi m (2 - 1/sigma_d) (Kaiser-Bessel window; paper, "Materials and
 * Methods"), in FP64: the constant the stored window is divided by (see the
 * single steps above).  peak: host array of D doubles.  An extension of the
 * introspection calls; NFFT_ERR_ARG for a NULL argument. */
int nfft_plan_window_peak(nfft_plan_t p, double *peak);

/* The spreading scheme the plan uses (an extension of the introspection calls):
 * *scheme = NFFT_SPREAD_SWEEP for 3-D plans that spread by column sweeps,
 * NFFT_SPREAD_TILED otherwise (padded tiles, or for D = 4 tile owners).
 * NFFT_ERR_ARG for a NULL argument. */
int nfft_plan_spread(nfft_plan_t p, int *scheme);

/*
 * Per-kernel timing.  With timing enabled, nfft_forward and nfft_adjoint
 * record a pair of HIP events on `stream` around each kernel they launch.
 * nfft_plan_timing waits for the last recorded event and returns, for the most
 * recent forward and adjoint call, the elapsed milliseconds of each stage:
 *   0 forward: resampling correction + zero pad + FFT along the last axis
 *   1 forward: FFT along axis 1 (3-D; 4-D: axes 2 and 1, the last one
 *              recorded is kept)            2 forward: FFT along axis 0
 *   3 forward: interpolation
 *   4 adjoint: spreading into the work items' padded tiles (1-D, 3-D padded
 *              tiles: and the halo merge into the grid; 3-D column sweeps: the
 *              fhat gather and the sweeps into their scratch; 4-D: straight into
 *              the grid)
 *   5 adjoint: FFT along axis 0 (2-D and 3-D column sweeps: reads the spreading
 *              scratch and performs the merge on the way)
 *   6 adjoint: FFT along axis 1 (3-D; 4-D: axes 1 and 2, the last kept)
 *   7 adjoint: FFT along the last axis + crop + resampling correction
 * Stages a plan does not run report 0.  ms must hold NFFT_NUM_STAGES values.
 * Timing adds an event record per kernel; leave it off when timing whole calls.
 */
#define NFFT_NUM_STAGES 8
int nfft_plan_set_timing(nfft_plan_t p, int enable);
int nfft_plan_timing(nfft_plan_t p, double *ms);

/*
 * Back-to-back timing of one resampling stage (a measurement aid, e.g. for
 * choosing tiles): launches the stage `reps` times on `stream` between two HIP
 * events, synchronises the stream and stores the mean milliseconds per launch
 * in *ms.
 *   stage 3 (interpolation): reads the plan's grid, writes fhat (`out`, M
 *            complex values, device).
 *   stage 4 (spreading): reads fhat (`in`, M complex values, device) and
 *            writes the plan's spreading scratch; in 1-D and with 3-D padded
 *            tiles also the halo merge into the plan's grid, as in nfft_adjoint
 *            (4-D: writes the plan's grid; 2-D and 3-D column sweeps leave the
 *            merge to the first adjoint FFT pass, as nfft_adjoint does).
 * Errors: NFFT_ERR_ARG for another stage, reps < 1 or a missing pointer
 * (when M > 0); NFFT_ERR_HIP for a failed launch or event.
 */
int nfft_plan_bench_stage(nfft_plan_t p, int stage, int reps, const void *in, void *out,
                          void *stream, double *ms);

/*
 * LDS operation rate of the current device (a measurement aid: the roof the
 * spreading kernels' LDS atomics and the interpolation's LDS reads are reported
 * against; the paper's resampling, subsections "Block-Partitioned Resampling"
 * and "Block-Partitioned Adjoint Resampling", works on a block-local copy of the
 * grid, which here lives in LDS).  Launches 8 workgroups
 * of 256 threads per compute unit, each thread performing 2048 operations of
 * kind `op` on a 16 KiB LDS buffer, `reps` times between two HIP events on
 * `stream` (after one untimed launch), and stores the lane operations per
 * second in *lane_ops_per_s.
 *   op:      NFFT_LDS_ADD_U32 / _ADD_U64 / _ADD_F32 / _ADD_F64 (atomic add,
 *            no return), NFFT_LDS_WRITE_B64 (plain 8-byte store),
 *            NFFT_LDS_RMW_B64 (8-byte load, add, store; not atomic),
 *            NFFT_LDS_READ_B64 / _READ_B128 (8- and 16-byte loads, summed:
 *            a complex64 / complex128 grid value).
 *   pattern: 0 consecutive words across the lanes, 1 a random word per lane,
 *            2 groups of 8 lanes on 8 consecutive words from a random start
 *            (the shape of one spreading instruction, and of one interpolation
 *            load: eight lanes read a node's row of 2m = 8 grid values).  A
 *            word is the operation's width.
 * Allocates and frees a small device buffer (one word per thread).
 * Errors: NFFT_ERR_ARG for an unknown op or pattern, reps < 1 or a NULL
 * output; NFFT_ERR_HIP / NFFT_ERR_NOMEM for a failed HIP call.
 */
enum {
    NFFT_LDS_ADD_U32 = 0,
    NFFT_LDS_ADD_U64 = 1,
    NFFT_LDS_ADD_F32 = 2,
    NFFT_LDS_ADD_F64 = 3,
    NFFT_LDS_WRITE_B64 = 4,
    NFFT_LDS_RMW_B64 = 5,
    NFFT_LDS_READ_B64 = 6,
    NFFT_LDS_READ_B128 = 7,
    NFFT_LDS_OPS = 8
};
int nfft_calibrate_lds(int op, int pattern, int reps, void *stream, double *lane_ops_per_s);

/* Static description of an error code (never NULL). */
const char *nfft_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* NFFT_MI355X_H */
