/*
 * slrcount: #DNN-Verification counting with Symbolic Linear Relaxation on MI355X (gfx950).
 *
 * The engine answers the counting version of DNN verification (paper §2.3): for a ReLU
 * network N, an input box P (the precondition, §2.1) and an unsafe output set given as linear
 * rows (the negated postcondition, §3), it returns a sound bracket on the fraction of P whose
 * outputs are unsafe (the violation rate, §2.3).  It follows Alg. 1 (§3): every box of one
 * branch-and-bound level is bounded at once (§3), with a lower and an upper linear equation
 * per neuron relaxed at crossing ReLUs by Eq. 1 (§2.2); boxes whose reachable set lies inside
 * the unsafe set add their volume, boxes that cannot reach it are dropped, the rest are
 * bisected (iterative refinement, §2.2).
 *
 * Conventions for every entry point:
 *   - return value: SLR_OK (0) or SLR_BUDGET (1) on success, a negative SLR_E* code on error;
 *     last_error() then holds a message (thread-local, owned by the library, valid until the
 *     next call on the same thread);
 *   - "host" pointers are read synchronously during the call and may be freed afterwards;
 *     "device" pointers are HIP device memory owned by the caller;
 *   - arrays are dense and row-major; all inputs are validated before any GPU work starts;
 *   - a stream argument is a hipStream_t (NULL = the default stream).
 */
#ifndef SLRCOUNT_H
#define SLRCOUNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SLR_OK = 0,           /* finished; for counts: nothing left undecided                    */
    SLR_BUDGET = 1,       /* depth or leaf budget reached: the result is a valid bracket     */
    SLR_EINVAL = -1,      /* bad argument: shape, NaN/Inf, lo > hi, non-float32 corner, ...   */
    SLR_ENOMEM = -2,      /* workspace too small or device allocation failed                 */
    SLR_EHIP = -3,        /* HIP runtime error                                                */
    SLR_EINTERNAL = -4,   /* an internal consistency check failed                            */
    SLR_EUNSUPPORTED = -5 /* valid input outside the sizes this build supports               */
};

/* Hidden activations of load_net_act (load_net: ReLU). */
enum { SLR_ACT_RELU = 0, SLR_ACT_TANH = 1, SLR_ACT_SIGMOID = 2 };

/* Box classes written by bound_boxes and recorded in traces. */
enum { SLR_UNDECIDED = 0, SLR_UNSAFE = 1, SLR_SAFE = 2 };

typedef struct slr_net slr_net;            /* opaque; immutable after load_net            */
typedef struct slr_property slr_property;  /* opaque; immutable after load_property       */

/*
 * load_net: copy a ReLU multilayer perceptron to the device.
 *   n_affine  number of affine layers (>= 2: at least one hidden ReLU layer, at most 8);
 *   sizes     host [n_affine + 1]: input dimension d (1..32), hidden widths (1..256), n_out
 *             (1..64);
 *   W         host [n_affine] pointers; W[l] is row-major [sizes[l+1], sizes[l]] float32;
 *   b         host [n_affine] pointers; b[l] is [sizes[l+1]] float32.
 * ReLU follows every affine layer but the last.  The float32 values are the network.
 * *out receives a handle owned by the caller (release with free_net).  NaN/Inf weights give
 * SLR_EINVAL.  The handle may be used concurrently from several threads and streams.
 */
int load_net(int32_t n_affine, const int32_t* sizes, const float* const* W,
             const float* const* b, slr_net** out);

/*
 * load_net_act: load_net with another hidden activation, SLR_ACT_TANH or SLR_ACT_SIGMOID
 * (SLR_ACT_RELU is load_net).  The paper treats ReLU networks and names other activations as
 * future work (§3); here a tanh or sigmoid neuron with pre-activation bounds [l, u] is enclosed
 * by two parallel lines lam z + b_lo <= s(z) <= lam z + b_hi: lam is the chord slope over [l, u]
 * and b_lo, b_hi bound s(z) - lam z over [l, u] (its extrema lie at l, u or where s'(z) = lam),
 * moved outward by a rounding margin.  bound_boxes, count_exact, count_exact_stack,
 * count_exact_noalloc, count_approx and plain batches accept such networks; the alpha calls,
 * alpha options and the tape-state kernel (shapes beyond the LDS bound kernel) return
 * SLR_EUNSUPPORTED.  Other act values: SLR_EINVAL.
 */
int load_net_act(int32_t n_affine, const int32_t* sizes, const float* const* W,
                 const float* const* b, int32_t act, slr_net** out);
void free_net(slr_net* net);

/*
 * load_property: the unsafe output set (the negated postcondition Q of §2.1 and §3).
 * An output y is unsafe iff every row r of C y + d is strictly positive.  A single output box
 * Y_l <= y <= Y_u is the special case with rows +e_i, -e_i (§3).
 *   rows   1..16;  C host [rows, n_out] float32;  d host [rows] float32.
 * The rows are folded into the last affine layer in FP64 (C W_L, C b_L + d) and kept on the
 * device; the handle is immutable and must be released with free_property before its net.
 */
int load_property(const slr_net* net, int32_t rows, const float* C, const float* d,
                  slr_property** out);
void free_property(slr_property* prop);

/*
 * bound_boxes: one launch of the bound kernel over n boxes (the per-level step of Alg. 1).
 *   lo, hi  device [n, d] float32 box corners (lo <= hi);
 *   g_lo, g_hi  device [n, rows] float32: lower/upper bound of each property row over the box;
 *   cls     device [n] int8 or NULL: SLR_UNSAFE if every row's lower bound is > 0, SLR_SAFE
 *           if some row's upper bound is <= 0, SLR_UNDECIDED otherwise;
 *   raw     0: bounds widened outward by the float32 rounding-error margin (sound), and boxes
 *           whose class could change within that margin re-decided in FP64;
 *           1: unwidened float32 bounds (for comparison with an FP64 reference), cls from them.
 * Asynchronous on `stream`; no allocation; n = 0 is a no-op.  The caller keeps the buffers
 * alive until the stream has passed the call.
 */
int bound_boxes(const slr_net* net, const slr_property* prop, int64_t n, const float* lo,
                const float* hi, float* g_lo, float* g_hi, int8_t* cls, int32_t raw,
                void* stream);

/*
 * bound_kernel_variant: process-wide choice of the bound kernel.
 *   0  automatic (default): the LDS-staged kernel where the shape fits its 160 KiB tiles, else
 *      (count_exact / count_approx only) the tape-state kernel of the alpha mode with the plain
 *      slopes, whose near-threshold boxes are re-decided in FP64 like the others';
 *   1  always the LDS-staged kernel;
 *   2  the register-resident kernel (shapes it cannot take then fail with SLR_EUNSUPPORTED);
 *   3  the tape-state kernel for every shape (count_exact / count_approx; bound_boxes then
 *      fails with SLR_EUNSUPPORTED).
 * All compute the same bounds up to float32 rounding.  Not synchronized with calls in flight
 * on other threads.
 */
int bound_kernel_variant(int32_t variant);

/*
 * bound_tile_shape: process-wide tile shape of the LDS-staged bound kernel for networks with
 * input dimension class of d and mt_max = ceil(max hidden width / 16): nt 16-box N tiles per
 * workgroup, uw output tiles per wavefront per layer, nw wavefronts per workgroup.  Instantiated
 * shapes: (4,1,4) (2,1,4) (1,1,4) (1,2,4), (1,1,8) for d <= 23, (1,4,4) for d <= 15, (1,2,8) for
 * d <= 11; the shape must cover the hidden tiles (mt_max * nt <= uw * nw).  nt = 0 restores the
 * default.  Results do not depend on the shape.  Used by the autotuner (a JSON cache of the
 * measured best shape per class); batches use the shape when their kernels have it.
 */
int bound_tile_shape(int32_t d, int32_t mt_max, int32_t nt, int32_t uw, int32_t nw);

/* Options of the exact count (Alg. 1). */
typedef struct {
    int32_t max_depth;      /* boxes still undecided at this depth are not split (0..62)   */
    int64_t max_leaves;     /* leaf budget, applied at level boundaries (>= 1)              */
    int32_t chunk;          /* boxes per bound launch (0 = 65536)                            */
    void* workspace;        /* device memory of at least workspace_size() bytes             */
    size_t workspace_bytes;
    void* stream;           /* hipStream_t used for all work of the call                     */
    /* optional per-box trace (host arrays, NULL to disable): for every bounded box, in level
       order, its depth, path id (root 1, children 2p and 2p+1) and final class */
    int64_t trace_capacity;
    int32_t* trace_depth;
    uint64_t* trace_path;
    int8_t* trace_cls;
    int32_t timing;         /* bit 0: time the bound-kernel launches with HIP events on
                               `stream`; bit 1: time the split launches (each timed launch is
                               bracketed by two events, which cost a few microseconds each);
                               bit 2: run every depth with the level-by-level driver (no
                               one-pass top of the tree; results are the same either way) */
    /* alpha mode: boxes that the plain bounds leave undecided at depth >= alpha_min_depth get
       alpha_steps projected-Adam steps of optimized lower slopes (0 = plain only), in batches
       of alpha_chunk boxes (the workspace must be sized for it) */
    int32_t alpha_steps;
    float alpha_lr;         /* Adam step size (0 = 0.1) */
    int32_t alpha_min_depth;
    int32_t alpha_chunk;
    /* 0: the alpha pass takes every box the plain bounds leave undecided; > 0: only those
       whose plain bounds are near a decision: for each property row the distance of the
       deciding bound from zero relative to the row's bound width, (-g_lo) / (g_hi - g_lo) for
       proving unsafe (the largest over the rows with g_lo <= 0) and g_hi / (g_hi - g_lo) for
       proving safe (the smallest over the rows); a box is taken when the smaller of the two
       is at most alpha_select.  Must be finite and >= 0. */
    float alpha_select;
    /* which side of an undecided box to bisect (the paper's iterative refinement, §2.2,
       leaves it open): 0 the widest (lowest index on ties); k in 1..8 the side, among those at
       least 2^-6 of the widest, that contributes most to the intervals of the crossing neurons
       of the first k hidden layers, sum over them of |coefficient of the side| x its width
       (the widest when none crosses).  k > 0 needs a ReLU network on the LDS bound kernel with
       at most 11 inputs (SLR_EUNSUPPORTED otherwise). */
    int32_t split_layers;
    /* optional trace of the side bisected per bounded box (host, trace_capacity entries, NULL
       to disable): the side for undecided boxes (-2 when the widest side was taken by
       split_layers = 0), -1 for decided ones */
    int8_t* trace_dim;
    /* ReLU relaxation: SLR_RELAX_ONE (Eq. 1: the upper chord's ratio u / (u - l) scales both
       equations) or SLR_RELAX_TWO (one ratio per equation, from that equation's own range:
       the upper one becomes the chord of ReLU over [min U, u], or stays U when min U >= 0; the
       lower one gets slope max L / (max L - l), or 0 when max L <= 0).  SLR_RELAX_TWO bounds
       every level with the tape-state kernel and keeps its widened float32 classes: boxes
       within the float32 rounding margin of a decision are not re-decided in FP64 and stay
       undecided (the bracket stays sound and can be slightly wider than an FP64 evaluation's).
       It needs a ReLU network with d <= 32 and no alpha or split_layers (SLR_EUNSUPPORTED
       otherwise); the workspace grows by the tape of 4096 boxes (workspace_size_exact). */
    int32_t relax;
} slr_exact_opts;

/* Values of slr_exact_opts.relax and bound_boxes_relax's relax. */
enum { SLR_RELAX_ONE = 0, SLR_RELAX_TWO = 1 };

typedef struct {
    double unsafe, safe, undecided;   /* volume fractions of the input box; they sum to 1   */
    int64_t n_unsafe, n_safe, n_undecided;   /* leaf boxes per class                        */
    int64_t n_boxes_bounded;          /* boxes evaluated by the bound kernel                 */
    int64_t n_recheck64;              /* boxes re-decided in FP64                            */
    int32_t depth_reached;            /* deepest level bounded                               */
    int32_t status;                   /* SLR_OK or SLR_BUDGET                                */
    double seconds;                   /* wall time of the call                               */
    int64_t trace_count;              /* boxes written to the trace (<= trace_capacity)      */
    double bound_ms;                  /* with timing bit 0: summed bound-kernel time (ms)    */
    int64_t bound_launches;           /* bound-kernel launches made by the call              */
    int64_t n_alpha_boxes;            /* boxes given the alpha optimization                  */
    int64_t n_alpha_decided;          /* of those, boxes the optimized bounds decided        */
    double alpha_ms;                  /* with timing: time of the alpha passes (ms)          */
    double split_ms;                  /* with timing bit 1: time of the split launches of the
                                         levels the search continued from (ms)               */
    int64_t split_bytes;              /* algorithmic HBM bytes of those split launches: every
                                         class byte, undecided parents' corners and paths,
                                         two children each, per-tile counts                  */
} slr_count_result;

/*
 * workspace_size: bytes of device workspace needed by count_exact / count_approx for a leaf
 * budget `max_leaves`, up to `samples` sample points per split (0 for count_exact only) and
 * alpha batches of `alpha_chunk` boxes (0 without alpha mode).
 */
int workspace_size(const slr_net* net, const slr_property* prop, int64_t max_leaves,
                   int32_t samples, int32_t alpha_chunk, size_t* bytes);

/*
 * workspace_size_exact: bytes of device workspace count_exact needs for `opts` (its
 * max_leaves, alpha_chunk when alpha_steps > 0, and relax; the workspace fields are ignored).
 * workspace_size gives the same figure for SLR_RELAX_ONE.
 */
int workspace_size_exact(const slr_net* net, const slr_property* prop, const slr_exact_opts* opts,
                         size_t* bytes);

/*
 * count_exact: Alg. 1 level by level on the device.
 *   lo, hi  host [d] float64 corners of the input box; each must be exactly representable
 *           in float32 (SLR_EINVAL otherwise).
 * Returns SLR_OK when nothing is left undecided, SLR_BUDGET when the depth or leaf budget
 * stopped the search (out holds the sound bracket [unsafe, unsafe + undecided]).  Volumes are
 * exact: every leaf of depth t holds 2^-t of the box.  Synchronizes `stream` before returning.
 */
int count_exact(const slr_net* net, const slr_property* prop, const double* lo, const double* hi,
                const slr_exact_opts* opts, slr_count_result* out);

/*
 * count_exact_noalloc: count_exact for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  It makes no device or host
 * allocation, creates no event and uses no pinned staging: its workspace is a static device
 * array of count_exact_noalloc_max_bytes() bytes (64 MiB) inside the library, one copy per GPU,
 * held from the library's first use on that GPU until the process ends, whose device address is
 * looked up once per GPU on the first call there.  Arguments and results are those of
 * count_exact, except:
 *   opts->workspace must be NULL and opts->workspace_bytes 0;
 *   opts->trace_capacity and opts->timing must be 0 (SLR_EINVAL otherwise);
 *   a count whose workspace_size() (with samples = 0) exceeds the static array fails with
 *   SLR_ENOMEM before any GPU work (e.g. the 5-input 6x50 network fits up to 2^19 leaves);
 *   the level counts are read back into stack memory, so each split waits for that read-back.
 * Every call on one GPU shares that GPU's array (the call re-initializes what it reads), so calls
 * that overlap on one GPU, from several threads or streams, race and must not be made.
 */
int count_exact_noalloc(const slr_net* net, const slr_property* prop, const double* lo,
                        const double* hi, const slr_exact_opts* opts, slr_count_result* out);

/* count_exact_noalloc_max_bytes: size of count_exact_noalloc's static workspace in bytes. */
size_t count_exact_noalloc_max_bytes(void);

/* ------------------------------------------------------------------------------------------
 * Depth-first stack count: Alg. 1 without a leaf budget, in bounded memory.
 *
 * The paper's exact counter keeps whole branch-and-bound levels and spills partial results to
 * disk once they outgrow memory (§4).  count_exact_stack keeps the undecided boxes on a stack
 * ordered by depth (shallowest at the bottom) and repeatedly bounds the top `chunk` boxes
 * (§3's independent per-box bounding, one launch), counts their classes per depth and pushes
 * the children of the undecided ones; so the deepest work is done first and the stack holds
 * about (max_depth + 2) * 2 * chunk boxes at most, whatever the number of leaves.  When the
 * device part of the stack would exceed `device_boxes`, its bottom half moves to the caller's
 * host buffer (out of core) and comes back once the device part has drained.  The boxes bounded
 * are exactly those of count_exact with the same max_depth and an unlimited leaf budget, so the
 * counts and exact volumes are identical; only the order differs.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
    int32_t max_depth;       /* undecided boxes at this depth are not split (0..62)           */
    int32_t chunk;           /* boxes per bound launch (1..65536; 0 = 65536)                  */
    int64_t max_boxes;       /* 0: no cap; else the count stops (SLR_BUDGET) before a chunk
                                would take the boxes bounded beyond it, and every box left on
                                the stack counts as undecided at its depth                  */
    int64_t device_boxes;    /* device stack capacity in boxes (>= 4 * chunk; 0 = the bound
                                2 * (max_depth + 2) * chunk, which never spills)             */
    void* host_spill;        /* host memory for the stack's bottom (pinned for speed), or NULL */
    size_t host_spill_bytes; /* holds host_spill_bytes / (8 d + 8) boxes                      */
    void* workspace;         /* device memory of at least stack_workspace_size() bytes        */
    size_t workspace_bytes;
    void* stream;            /* hipStream_t used for all work of the call                     */
    /* optional per-box trace (host arrays, NULL to disable): depth, path id and final class of
       every bounded box, in the order bounded (not level order) */
    int64_t trace_capacity;
    int32_t* trace_depth;
    uint64_t* trace_path;
    int8_t* trace_cls;
} slr_stack_opts;

/* stack_workspace_size: device workspace of count_exact_stack for these options (max_depth,
   chunk and device_boxes are read). */
int stack_workspace_size(const slr_net* net, const slr_property* prop, const slr_stack_opts* opts,
                         size_t* bytes);

/*
 * count_exact_stack: see above.  lo, hi as for count_exact.  out as for count_exact
 * (trace_count, n_boxes_bounded, n_recheck64, depth_reached, status; the timing and alpha
 * fields are 0).  Returns SLR_OK when nothing is left undecided, SLR_BUDGET otherwise, and
 * SLR_ENOMEM when the stack outgrows device_boxes plus the host buffer.  Synchronizes `stream`
 * before returning.
 */
int count_exact_stack(const slr_net* net, const slr_property* prop, const double* lo,
                      const double* hi, const slr_stack_opts* opts, slr_count_result* out);

/* Options of the approximate count (CountingProVe with count_exact as leaf backend, §2.3). */
typedef struct {
    int32_t trials;          /* independent trials T (1..64)                                */
    int32_t samples;         /* uniform samples per split (1..65536)                        */
    double confidence;       /* e.g. 0.99: bound <= violation rate with this probability    */
    uint64_t seed;           /* Philox4x32-10 key                                          */
    int32_t max_splits;      /* cap on splits per trial                                    */
    int32_t grid_bits;       /* split points lie on the grid lo + k (hi - lo) 2^-grid_bits  */
    double resolve_tol;      /* a subdomain is resolved when <= this fraction is undecided  */
    /* trials run at once: 0 or 1 (one after another on leaf.stream).  Larger values are
       reserved and rejected with SLR_EUNSUPPORTED: a threaded form (one stream and workspace
       slice per slot) gave identical results but crashed once inside hipEventRecord under a
       kernel-trace profiler, with no cause found in this library.  Other values: SLR_EINVAL. */
    int32_t concurrency;
    slr_exact_opts leaf;     /* options (and workspace) of each leaf count                  */
} slr_approx_opts;

typedef struct {
    double lower_bound;      /* 2^-beta min_i estimate[i], beta = log2(1/(1-confidence))/T  */
    double estimate[64];     /* per-trial estimate 2^s v f                                  */
    int32_t splits[64];      /* per-trial number of splits s                                */
    int32_t trials;
    double seconds;
} slr_approx_result;

/*
 * count_approx: probabilistic lower bound on the violation rate.  Each trial halves the
 * domain (at the lower median of the violating samples along a random dimension, keeping a
 * random side) until count_exact resolves the subdomain; see the implementation file for the
 * exact draw layout.  Synchronizes opts->leaf.stream.
 */
int count_approx(const slr_net* net, const slr_property* prop, const double* lo,
                 const double* hi, const slr_approx_opts* opts, slr_approx_result* out);

/*
 * sample_violations: concrete float32 forward pass of n points (device [n, d]) writing
 * viol[i] = 1 if every property row is > 0 at point i, else 0 (device int8 [n]).
 * Asynchronous on `stream`.
 */
int sample_violations(const slr_net* net, const slr_property* prop, int64_t n, const float* x,
                      int8_t* viol, void* stream);

/* ------------------------------------------------------------------------------------------
 * Alpha mode: optimized lower slopes.
 *
 * Eq. 1 replaces a crossing neuron (l < 0 < u) by the lines lam z (lower) and lam (z - l)
 * (upper), lam = u / (u - l).  Any slope alpha in [0, 1] also gives a valid lower line alpha z,
 * so each box may carry its own slope per hidden neuron, tuned by gradient to tighten the bound
 * that decides the box; the upper line stays the chord of Eq. 1.  Slopes are device float32
 * arrays [n][nh], nh = the sum of the hidden widths, neurons in their original order, the first
 * hidden layer first.  Only the slopes of crossing neurons are used; values are clamped to [0, 1].
 * ------------------------------------------------------------------------------------------ */

/* alpha_state_variant: process-wide placement of the alpha kernels' tile state: 0 automatic
   (LDS where it fits), 1 the same, 2 always global memory (the tape's extra slots; frees LDS for
   more resident workgroups).  Tape sizes depend on it: query alpha_tape_size after setting it. */
int alpha_state_variant(int32_t variant);

/* alpha_kernel_variant: process-wide launch structure of alpha_optimize and of the alpha pass of
   the exact count: 0 (default) one launch per forward and per adjoint pass; 1 one fused launch
   per optimization, every 16-box tile running its initial forward pass and all steps (adjoint
   with the Adam step, forward) in one workgroup (the batched alpha pass always uses this form).
   Both compute the same values. */
int alpha_kernel_variant(int32_t variant);

/* alpha_size: nh, the slopes per box. */
int alpha_size(const slr_net* net, int64_t* nh);

/* alpha_tape_size: bytes of the tape bound_boxes_alpha writes for n boxes (per 16-box tile:
   every layer's pre-activation equations and concrete bounds). */
int alpha_tape_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes);

/*
 * bound_boxes_alpha: bounds of n boxes with per-box slopes, on `stream`, asynchronous.
 *   lo, hi       device float32 [n, d]
 *   alpha        device [n, nh]: the slopes (init = 0), or written with the plain ratios lam of
 *                every crossing neuron and 1 elsewhere (init = 1); NULL = the plain relaxation
 *   g_lo, g_hi   device float32 [n, rows] output bounds of the property rows
 *   cls          device int8 [n] (optional): 1 unsafe, 2 safe, 0 undecided (no FP64 recheck)
 *   raw          1 = no rounding margins (for gradient and parity tests), 0 = sound bounds
 *   tape         device memory of at least alpha_tape_size(n) bytes, read by the adjoint
 */
int bound_boxes_alpha(const slr_net* net, const slr_property* prop, int64_t n, const float* lo,
                      const float* hi, float* alpha, int32_t init, float* g_lo, float* g_hi,
                      int8_t* cls, int32_t raw, void* tape, size_t tape_bytes, void* stream);

/*
 * bound_boxes_relax: bounds of n boxes with the plain slopes of a ReLU relaxation, from the
 * tape-state kernel (full lower and upper equations per neuron), on `stream`, asynchronous.
 *   relax        SLR_RELAX_ONE (Eq. 1, the same bounds as bound_boxes up to float32 rounding)
 *                or SLR_RELAX_TWO (one ratio per equation, slr_exact_opts.relax)
 *   lo, hi       device float32 [n, d];  g_lo, g_hi  device float32 [n, rows]
 *   cls          device int8 [n] (optional): 1 unsafe, 2 safe, 0 undecided, from g_lo / g_hi
 *                (no FP64 re-decision: count_exact with relax does that)
 *   raw          1 = no rounding margins (for comparison with an FP64 reference), 0 = sound
 *   tape         device scratch of at least bound_tape_size(n) bytes
 * ReLU networks with d <= 32 (SLR_EUNSUPPORTED otherwise).
 */
int bound_boxes_relax(const slr_net* net, const slr_property* prop, int64_t n, const float* lo,
                      const float* hi, int32_t relax, float* g_lo, float* g_hi, int8_t* cls,
                      int32_t raw, void* tape, size_t tape_bytes, void* stream);

/* bound_tape_size: bytes of the scratch tape bound_boxes_relax needs for n boxes. */
int bound_tape_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes);

/*
 * bound_boxes_backward: the hand-written adjoint of bound_boxes_alpha.  Given seeds
 * dg_lo = dJ/dg_lo and dg_hi = dJ/dg_hi (device [n, rows]; NULL = zero), writes
 * dalpha = dJ/dalpha (device [n, nh]; 0 for neurons that are not crossing).  `tape` must hold
 * what bound_boxes_alpha wrote for the same boxes, slopes and `raw`; the rounding margins are
 * treated as constants.  Asynchronous on `stream`.
 */
int bound_boxes_backward(const slr_net* net, const slr_property* prop, int64_t n,
                         const float* alpha, const void* tape, size_t tape_bytes,
                         const float* dg_lo, const float* dg_hi, float* dalpha, int32_t raw,
                         void* stream);

typedef struct {
    int32_t steps;           /* projected Adam steps (e.g. 20)                               */
    float lr, beta1, beta2, eps;   /* Adam (e.g. 0.1, 0.9, 0.999, 1e-8)                      */
    int32_t raw;             /* 1 = bounds without rounding margins                          */
} slr_alpha_opts;

/* alpha_workspace_size: device workspace of alpha_optimize for n boxes. */
int alpha_workspace_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes);

/*
 * alpha_optimize: per box, starts from the plain ratios and takes `steps` projected Adam steps
 * on the objective: if every property row is > 0 at the box center (float32 forward pass),
 * maximize min_r g_lo[r]; otherwise minimize g_hi[r*], r* = the row with the smallest value at
 * the center.  Every step's bounds are valid, so best_lo / best_hi (device [n, rows]) receive
 * their running intersection (max of the lower, min of the upper bounds) and cls (device int8
 * [n], optional) the class they decide.  alpha (device [n, nh], optional) receives the last
 * slopes.  Synchronous only through `stream` (asynchronous to the host).
 */
int alpha_optimize(const slr_net* net, const slr_property* prop, int64_t n, const float* lo,
                   const float* hi, const slr_alpha_opts* opts, float* alpha, float* best_lo,
                   float* best_hi, int8_t* cls, void* workspace, size_t workspace_bytes,
                   void* stream);

/* ------------------------------------------------------------------------------------------
 * Batches: many independent exact counts advanced level by level together (§3's
 * level-parallel bounding applied across instances).  Each instance has its own network,
 * property, box, depth and leaf budget; results equal those of count_exact on each instance
 * alone.  Levels run as a fixed launch sequence whose kernels read their work sizes on the
 * device (persistent bound kernels per kernel class pop tiles from a device work queue), so the
 * whole count can be captured once in a HIP graph and replayed with one launch and one
 * read-back.  Shapes: d <= 11, hidden widths <= 128, rows <= 16, max_leaves <= 2^22,
 * n_inst <= 1024.
 * ------------------------------------------------------------------------------------------ */
typedef struct slr_batch slr_batch;   /* opaque; owns its device memory */

/*
 * batch_create: validates every instance, allocates the batch's device memory (frontiers,
 * counters, work queues: the only allocation; batch_run allocates nothing) and, with
 * use_graph = 1, captures the launch sequence of a whole count into a graph.
 *   nets, props   [n_inst] handles (instances may share them)
 *   lo, hi        [n_inst] host float64 [d] boxes, exactly representable in float32
 *   max_depth     [n_inst], max_leaves [n_inst]: as in slr_exact_opts
 */
int batch_create(int32_t n_inst, const slr_net* const* nets, const slr_property* const* props,
                 const double* const* lo, const double* const* hi, const int32_t* max_depth,
                 const int64_t* max_leaves, int32_t use_graph, slr_batch** out);

/* Options of batch_create_opts.  With alpha_steps > 0 every level of every instance from depth
   alpha_min_depth on gets the alpha pass of slr_exact_opts inside the batch's launch sequence:
   the boxes its plain bounds leave undecided (all of them, or with alpha_select > 0 only those
   near a decision, as in slr_exact_opts) are optimized for alpha_steps projected-Adam steps and
   the boxes the optimized bounds decide take that class.  Instances share the alpha kernels of
   their template class; each class optimizes at most alpha_chunk boxes per level (0 = 8192),
   taken instance by instance in batch order and box by box in level order (the rest keep their
   plain class).  While no class runs out of room, every instance's result equals count_exact
   with the same alpha options. */
typedef struct {
    int32_t use_graph;       /* 1 = capture the launch sequence in a graph (as batch_create)   */
    int32_t alpha_steps;     /* 0 = plain counts                                              */
    float alpha_lr;          /* Adam step size (0 = 0.1)                                      */
    int32_t alpha_min_depth;
    float alpha_select;      /* finite, >= 0                                                  */
    int32_t alpha_chunk;     /* boxes per alpha class and level (0 = 8192)                    */
} slr_batch_opts;

/* batch_create_opts: batch_create with options (NULL opts: SLR_EINVAL). */
int batch_create_opts(int32_t n_inst, const slr_net* const* nets, const slr_property* const* props,
                      const double* const* lo, const double* const* hi, const int32_t* max_depth,
                      const int64_t* max_leaves, const slr_batch_opts* opts, slr_batch** out);

/*
 * batch_run: one complete count of every instance on `stream` (graph replay or the same
 * launches issued directly), then one read-back; results[i] (host, [n_inst]) as from
 * count_exact (bound_ms, trace and timing fields are 0; n_alpha_boxes and n_alpha_decided as in count_exact;
 * seconds is the batch's wall time).
 * Returns SLR_BUDGET if any instance stopped on its depth or leaf budget.  Calls on one batch
 * must not overlap.
 */
int batch_run(slr_batch* batch, void* stream, slr_count_result* results);
void batch_free(slr_batch* batch);

/* count_exact_batch: batch_create (without graph) + batch_run + batch_free. */
int count_exact_batch(int32_t n_inst, const slr_net* const* nets, const slr_property* const* props,
                      const double* const* lo, const double* const* hi, const int32_t* max_depth,
                      const int64_t* max_leaves, void* stream, slr_count_result* results);

/* Message of the last failed call on this thread ("" if none). */
const char* last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLRCOUNT_H */
