// Internal descriptors shared by the host engine and the gfx950 kernels.
//
// Device representation of one box's symbolic state (the center/radius form of the lower and
// upper equations of §3): in box-local coordinates t in [-1, 1]^d (x = mid + rad * t) every
// neuron keeps a center equation c(t) = c_0 + sum_i c_i t_i and a radius r >= 0 with
// L = c - r and U = c + r.  Eq. 1 scales both equations by the same ratio, so L and U keep
// equal slopes and the radius stays a constant; the W+/W- rule of symbolic propagation then
// becomes C' = W C + b and r' = |W| r.  A third quantity q <= r tracks how much of r is
// rounding margin (propagated like r), which tells boxes whose class could differ in exact
// arithmetic from the rest.
//
// Hidden neurons are relabeled on the device (a permutation, which leaves the network's function
// and its bounds unchanged): a layer of n neurons occupies 16-row tiles; the last tile holds
// r = n - 16 (tiles - 1) neurons, placed at rows 4 g + v in the order v-major (all g for v = 0
// first).  Row 16 mt + 4 g + v is then valid iff mt < tiles - 1 or 4 v + g < r, and the next
// layer needs only 4 (tiles - 1) + ceil(r / 4) MFMA K-steps.
#pragma once

#include <hip/hip_runtime.h>
#include "../../include/slrcount.h"
#include <stdint.h>

#define SLR_MAX_AFFINE 8
#define SLR_MAX_D 32
#define SLR_MAX_WIDTH 256
#define SLR_MAX_ROWS 16
#define SLR_MAX_OUT 64
#define SLR_MAX_LEVELS 63
#define SLR_MAX_BATCH 1024
#define SLR_MAX_CLASSES 64

// One hidden-to-hidden affine layer (its input is a hidden ReLU layer).
struct MidLayer {
    const float* wfrag;   // [mt_out][ks_alloc][64] MFMA A-operand fragments (see pack_fragments)
    const uint64_t* qfrag;  // [mt_out][ks_alloc / 4][64]: |W| of four K-steps as bf16 rounded up
                            // (A operand of the bf16 16x16x16 MFMA of the margin column)
    const float* w;       // row-major [n_out][n_in] float32 (sample forward pass)
    const float* wt;      // transposed [n_in][n_out] (FP64 recheck: coalesced across neurons)
    const float* bias;    // [16 * mt_out] by relabeled row, zero padded
    const float* b;       // [n_out] in the original neuron order (FP64 recheck, forward pass)
    const float* absrow;  // [16 * mt_out]: sum_k |W_jk|, rounded up to float32
    int n_in, n_out, mt_out, ks, ks_alloc;
    int r_out;            // neurons in the last 16-row output tile
    int frag_off;         // offset (floats) of this layer's fragments in the staged copy
    const float* wtfrag;  // [mt_in][kst_alloc][64] fragments of W^T (alpha adjoint): rows are the
                          // layer's input neurons, K runs over its output neurons
    int mt_in, kst, kst_alloc;
    float kgam;           // kappa * gamma_{n_in + 2} for float32, rounded up
    double kgam64;        // the same for float64
};

struct NetDev {
    int d;                // input dimension
    int n_affine;         // affine layers (>= 2)
    int n1, mt1;          // first hidden width and its 16-row tiles
    int mt_max;           // max 16-row tiles over hidden layers
    int n_last, mt_last;  // width (and tiles) of the last hidden layer
    int n_max;            // max hidden width
    int frag_total;       // floats of all hidden-to-hidden fragments (staged into LDS)
    const float* w1;      // [n1][d] row-major, original neuron order
    const float* b1;      // [n1]
    const float* w1p;     // [16 mt1][d], relabeled rows (zero padding)
    const float* b1p;     // [16 mt1]
    int r1;               // neurons in the last 16-row tile of the first hidden layer
    MidLayer mid[SLR_MAX_AFFINE];   // affine layers 1 .. n_affine-2
    // alpha mode: per hidden layer h, relabeled row -> neuron (-1 = padding) and the offset of
    // the layer's slopes in a box's alpha vector (original neuron order, layer after layer)
    const int* rowmap[SLR_MAX_AFFINE];
    int hoff[SLR_MAX_AFFINE];
    int nh;               // hidden neurons in total = alpha floats per box
    int act;              // hidden activation: SLR_ACT_RELU, SLR_ACT_TANH or SLR_ACT_SIGMOID
    float kfirst, kconc, krelu;     // kappa*gamma_{d+2}, kappa*gamma_{d+3}, kappa*gamma_4
    double kfirst64, kconc64, krelu64;
};

struct PropDev {
    int rows, n_last;
    const float* wg;      // [rows][n_last] folded last layer C W_L, float32
    const float* wgfrag;  // [ks_out_alloc][64] MFMA A fragments of wg (rows padded to 16)
    const uint64_t* wgqfrag;  // [ks_out_alloc / 4][64] |wg| as bf16 rounded up, four K-steps
    int ks_out, ks_out_alloc;
    const float* wgp;     // [rows][kpad] wg with relabeled, zero-padded columns
    int kpad;             // 16 * tiles of the last hidden layer
    const float* bg;      // [rows] C b_L + d
    const float* ag;      // [rows] row sums of |C| |W_L| (bounds sum_k |wg_rk|), rounded up
    const double* wg64;   // the folded layer in float64
    const double* bg64;
    const double* ag64;
    // alpha mode: the property rows are relabeled like the last tile of a hidden layer (tile row
    // 4 g + v holds property row 4 v + g), so that the adjoint needs only ceil(rows / 4) K-steps
    const float* wgfrag_a;   // [ks_out_alloc][64] A fragments of wg with relabeled rows
    const float* wgtfrag;    // [mt_last][ks_rows_alloc][64] fragments of wg^T
    int ks_rows, ks_rows_alloc;
    const float* bga;        // [16] bg by relabeled row (zero padded)
    const float* aga;        // [16] ag by relabeled row
    float kout;           // kappa * gamma_{n_last + 3}, float32
    double kout64;        // kappa * gamma_{n_last + n_out + 3}, float64
};

// Per-level counters of the exact count (device, 64-bit).
struct LevelStats {
    unsigned long long unsafe_cnt;
    unsigned long long safe_cnt;
    unsigned long long undecided_cnt;
    unsigned long long pad;
};

// Kernel launchers (slr_kernels.hip).  All are asynchronous on `stream`.
// The bound kernel writes class 3 for boxes whose class could differ in exact arithmetic and,
// if amb_list is given, appends list_base + (box index) to amb_list[atomicAdd(amb_count)].
// dimsel (with split_layers > 0): the crossing-score split rule writes each box's side to
// bisect (ReLU networks, input classes up to NCOL 14; otherwise *unsupported).
hipError_t launch_bound_f32(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                            const float* hi, float* g_lo, float* g_hi, int8_t* cls, int raw,
                            hipStream_t stream, int* unsupported, unsigned* amb_list,
                            unsigned* amb_count, unsigned list_base, int8_t* dimsel = nullptr,
                            int split_layers = 0);
// FP64 re-decision of the boxes list[0 .. *list_count), or of every class-3 box if list is NULL.
int state_stride(int mt_max);   // floats per lane row of the bound kernel's LDS state
hipError_t launch_recheck64(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                            const float* hi, float* g_lo, float* g_hi, int8_t* cls,
                            unsigned long long* counter, const unsigned* list,
                            const unsigned* list_count, hipStream_t stream);
hipError_t launch_level_count(int64_t n, const int8_t* cls, unsigned int* tile_und,
                              LevelStats* stats, hipStream_t stream);
// Top of the search tree in one pass (depths 0 .. K, K <= 15): the 2^(K+1) - 1 boxes of the complete
// subtree in heap order (path id = index + 1) built by the widest-side split rule, and after
// they are bounded, the replay that marks the boxes the level-by-level search would not visit
// (class 4) and counts the visited ones of depths 0 .. K - 1 into stats.
struct RootBox {
    float lo[SLR_MAX_D], hi[SLR_MAX_D];
};
hipError_t launch_prefix_boxes(int64_t N, int d, const RootBox& rb, float* lo, float* hi,
                               unsigned long long* path, unsigned* err, hipStream_t stream);
hipError_t launch_prefix_replay(int64_t N, int K, int8_t* cls, LevelStats* stats, hipStream_t stream);
// After the replay: one off `counter` per listed box (list[0 .. *count)) of the N top boxes that
// the level loop does not visit.
hipError_t launch_prefix_recheck_uncount(int64_t N, const unsigned* list, const unsigned* count,
                                         const int8_t* cls, unsigned long long* counter,
                                         hipStream_t stream);
// dimsel: the side of each parent chosen by the bound kernel (NULL: the widest side).
hipError_t launch_split(int64_t n, int d, const int8_t* cls, const unsigned int* tile_und,
                        const float* lo, const float* hi, const unsigned long long* path,
                        float* lo2, float* hi2, unsigned long long* path2, unsigned int* err,
                        int64_t cap, hipStream_t stream, const int8_t* dimsel = nullptr);
// Depth-first stack count (count_exact_stack): per-depth class counts of a chunk of mixed-depth
// boxes (depth from the path id), class 4 for undecided boxes at max_depth, per-tile and total
// counts of the boxes to split; all_undecided counts every box as undecided at its depth.
constexpr int kMaxDepthLevels = 63;
hipError_t launch_stack_count(int64_t n, int8_t* cls, const unsigned long long* path, int max_depth,
                              int all_undecided, unsigned* tile_und, LevelStats* stats,
                              unsigned* split_total, hipStream_t stream);
// Exact volumes summed over every level and class (undecided leaves at any depth).
hipError_t launch_stack_volume(const LevelStats* stats, int levels, double* out3,
                               unsigned long long* out_counts, unsigned* err, hipStream_t stream);
hipError_t launch_volume(const LevelStats* stats, int levels, int stop_level, int stopped,
                         double* out3, unsigned long long* out_counts, unsigned int* err,
                         hipStream_t stream);
hipError_t launch_sample_forward(const NetDev& net, const PropDev& prop, int64_t n,
                                 const float* x, int8_t* viol, hipStream_t stream);
int bound_f32_supported(const NetDev& net, const PropDev& prop);
// Tile shape of the LDS-staged bound kernel: NT 16-box N tiles per workgroup, UW units per wave,
// NW wavefronts per workgroup.  The default depends on the hidden tiles (mt_max); a per-class
// override (input-dimension class x mt_max) can replace it, e.g. from the autotuner.
struct TileShape {
    int nt, uw, nw;
};
int ncol_class_of(int d);
TileShape tile_shape_for(int d, int mt_max);
bool tile_shape_valid(int ncol, int mt_max, TileShape t);
int set_tile_shape(int d, int mt_max, TileShape t);   // nt = 0 restores the default; -1 = invalid
size_t bound_lds_bytes(int ncol, TileShape t, int mt_max, int rows);
// Bound-kernel variant: 0 automatic, 1 LDS-staged, 2 register-resident only, 3 none (the exact
// count then bounds with the tape-state kernel, as for shapes the LDS kernel cannot hold).
// Returns -1 for an unknown value.
int set_bound_variant(int v);
int bound_variant_for(const NetDev& net, const PropDev& prop);
size_t level_tiles(int64_t n);

// ---------------------------------------------------------------------------------------------
// Alpha mode (slr_alpha.hip): every box has its own lower slope per crossing hidden neuron.
// ---------------------------------------------------------------------------------------------
struct AlphaArgs {
    int64_t n;
    const float* lo;
    const float* hi;
    float* alpha;          // [n][nh]: read, or written with the plain ratios when init
    float* g_lo;           // [n][rows] bounds of this pass (forward) / used for seeds (backward)
    float* g_hi;
    float* best_lo;        // optional running intersection of all passes' bounds
    float* best_hi;
    int8_t* cls;           // optional class from the (best) bounds
    float* tape;           // per 16-box tile: pre-activation slots (+ 2 state slots if global)
    int raw, init;
    int fwd_only;          // forward pass only: one shared pre-activation slot per tile
    const float* dg_lo;    // backward seeds [n][rows], or NULL with obj
    const float* dg_hi;
    const int8_t* obj;     // [n][2] objective (mode, row) for seeds computed on the device
    float* dalpha;         // optional [n][nh]
    float* adam_m;         // optional fused projected Adam state [n][nh]
    float* adam_v;
    float lr, beta1, beta2, eps, c1, c2;
    int two_ratio;         // forward passes: one ratio per equation (plain slopes, no alpha)
};

struct AlphaShape {
    int nc;                // center columns per neuron (class >= d + 1)
    int global_state;      // 1: the tile state lives in the tape's extra slots, not in LDS
    int reg_path;          // 1: contraction results stay in registers (narrow states)
    int reg_path_bwd;      // the same for the adjoint
    int slots;             // tape slots per tile
    int slots_fwd;         // tape slots per tile of a forward-only pass
    size_t slot_floats;    // floats per slot
    size_t lds_fwd, lds_bwd;
};
AlphaShape alpha_shape(const NetDev& net, const PropDev& prop);
// Where the alpha kernels keep the tile state: 0 automatic (LDS where it fits), 1 the same,
// 2 always in the tape's global slots.  Returns -1 for an unknown value.
int set_alpha_state_variant(int v);
size_t alpha_tape_bytes(const NetDev& net, const PropDev& prop, int64_t n, int fwd_only);
hipError_t launch_alpha_forward(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                hipStream_t stream);
hipError_t launch_alpha_backward(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                 hipStream_t stream);
// 0 (default): single-instance alpha optimizations run one launch per forward/adjoint pass;
// 1: one fused launch.  Both compute the same values.  Returns -1 for an unknown value.
int set_alpha_fused(int v);
int alpha_fused();
// A whole optimization per tile in one launch: forward with init, then `steps` (adjoint with the
// projected Adam step, forward); a.obj, a.adam_m and a.adam_v must be set (the moments are
// cleared by the kernel), a.init and a.c1/a.c2 are ignored.
hipError_t launch_alpha_optimize(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                 int steps, hipStream_t stream);
// obj[b][0] = 1 if every property row is > 0 at the box center, obj[b][1] = argmin row there
// Level helpers of the alpha pass inside the exact count.
// Undecided boxes (cls 0) into list; with g_lo/g_hi ([n][rows]) only those whose decision
// distance (see slr_exact_opts.alpha_select) is at most select; total (if given) counts every
// undecided box.
hipError_t launch_collect_undecided(int64_t n, const int8_t* cls, unsigned* list, unsigned* count,
                                    hipStream_t stream, const float* g_lo = nullptr,
                                    const float* g_hi = nullptr, int rows = 0, float select = 0.f,
                                    unsigned* total = nullptr);
hipError_t launch_gather_boxes(int64_t m, int d, const unsigned* list, const float* lo,
                               const float* hi, float* lo2, float* hi2, hipStream_t stream);
hipError_t launch_scatter_classes(int64_t m, const unsigned* list, const int8_t* cls2, int8_t* cls,
                                  hipStream_t stream);
// Class 3 (and the FP64 list) for undecided boxes near a decision, from widened and raw bounds.
hipError_t launch_ambiguity(int64_t n, int rows, const float* wlo, const float* whi,
                            const float* rlo, const float* rhi, int8_t* cls, unsigned* amb_list,
                            unsigned* amb_count, unsigned base, hipStream_t stream);
hipError_t launch_center_objective(const NetDev& net, const PropDev& prop, int64_t n,
                                   const float* lo, const float* hi, int8_t* obj,
                                   hipStream_t stream);

// ---------------------------------------------------------------------------------------------
// Batches of independent instances (slr_batch.hip): every instance keeps its own frontier and
// counters in device memory; one level of all instances is a fixed sequence of launches that
// read their work sizes on the device, so the whole count can be captured in one graph.
// ---------------------------------------------------------------------------------------------
struct BatchInst {
    NetDev net;
    PropDev prop;
    float* lo[2];
    float* hi[2];
    unsigned long long* path[2];
    int8_t* cls;
    unsigned* tile_und;
    LevelStats* stats;           // [SLR_MAX_LEVELS]
    const float* root;           // [2 d]: lower corner, then upper corner
    int d, max_depth, cls_id, sp;
    long long max_leaves;
    int pk;                      // depth of the one-pass top of the tree (0: none)
    int prefix_pending;          // the top's level has not been replayed yet
    // dynamic state, reset by the init kernel
    long long n, n_next, resolved, bounded;
    long long coff, cn;          // boxes [coff, coff + cn) of the level are counted and split
    unsigned perr[16];           // inexact midpoints in the top's splits, by parent depth
    int cur, level, active, split_pending;
    int status, stop_level, stopped, levels;
    unsigned long long rechecks;
    unsigned err;
    unsigned pad;
    double vol[3];
    unsigned long long counts[3];
    // alpha pass of batches with alpha options (acls_id < 0: none for this instance)
    float* glo;                  // [max_leaves][rows] widened plain bounds of the level
    float* ghi;
    int acls_id, alpha_min_depth;
    int aslots;                  // tape slots per 16-box tile
    unsigned acand;              // candidates at this level (summed by the candidate kernel)
    unsigned aseg, alen;         // segment of the alpha class's buffers: first box (16-aligned), boxes
    unsigned long long atile_floats;   // tape floats per tile
    unsigned long long atape;    // first tape float of the segment
    long long n_alpha_boxes, n_alpha_decided;
};

// Buffers of one alpha class of a batch (instances whose alpha kernels share a template): every
// instance optimized at a level owns a segment of cap boxes; per-box rows use the class's largest
// stride (d, nh, rows) as the segment base and the instance's own stride inside it.
struct BatchAlphaBuf {
    float *lo, *hi;              // [cap][dmax]
    float *alpha, *m, *v;        // [cap][nhmax]
    float *glo, *ghi, *blo, *bhi;   // [cap][rowsmax]
    int8_t* cls;                 // [cap]
    int8_t* obj;                 // [cap][2]
    unsigned* list;              // [cap] instance-local box index
    unsigned* seg;               // [ninst] segment start of each instance of the class (plan)
    float* tape;
    int dmax, nhmax, rowsmax;
    unsigned cap;
    const int* inst;             // [ninst] instance positions
    int ninst;
};

// Device-side decision distance of a box (see slr_exact_opts.alpha_select): the smaller of the
// unsafe distance (largest (-g_lo)/(g_hi - g_lo) over rows with g_lo <= 0) and the safe distance
// (smallest g_hi/(g_hi - g_lo) over the rows).
__device__ __forceinline__ float slr_decision_distance(const float* glo, const float* ghi, int rows) {
    float du = 0.f, ds = INFINITY;
    for (int r = 0; r < rows; ++r) {
        const float w = ghi[r] - glo[r];
        if (!(w > 0.f)) continue;
        if (glo[r] <= 0.f) du = fmaxf(du, -glo[r] / w);
        ds = fminf(ds, ghi[r] / w);
    }
    return fminf(du, ds);
}

struct BatchCtl {
    unsigned head[SLR_MAX_CLASSES];     // bound work-queue heads (one queue per kernel class)
    unsigned ntiles[SLR_MAX_CLASSES];   // bound tiles per class at the current level
    int tbox[SLR_MAX_CLASSES];          // boxes per bound tile of each class
    unsigned amb_count;                 // boxes listed for the FP64 re-decision
    unsigned ctiles;                    // 1024-box bookkeeping tiles at the current level
    unsigned antiles[SLR_MAX_CLASSES];  // alpha tiles per alpha class at the current level
};

// Kernel class of the batch bound kernel: NCOL and the tile shape of the LDS-staged tile.
bool batch_class_supported(int ncol, TileShape t);
int batch_class_of(const NetDev& net, const PropDev& prop, int* ncol, TileShape* t);
size_t batch_bound_lds(int ncol, TileShape t, int mt_max, int rows);
hipError_t batch_prepare_class(int ncol, TileShape t, size_t lds, int* blocks);
hipError_t launch_batch_init(BatchInst* insts, int n_inst, hipStream_t stream);
// The one-pass top of the tree of the instances with pk > 0 (pk_max: the largest pk, d_max: the
// largest input dimension): its boxes, and the replay of its level after the re-decision.
hipError_t launch_batch_prefix(BatchInst* insts, int n_inst, int pk_max, int d_max, hipStream_t stream);
hipError_t launch_batch_prefix_replay(BatchInst* insts, int n_inst, int pk_max, BatchCtl* ctl,
                                      const unsigned* amb_list, hipStream_t stream);
hipError_t launch_batch_plan(BatchInst* insts, int n_inst, BatchCtl* ctl, unsigned* bpre,
                             unsigned* cpre, int n_classes, hipStream_t stream);
hipError_t launch_batch_bound(int ncol, TileShape t, int blocks, size_t lds, BatchInst* insts,
                              BatchCtl* ctl, const unsigned* bpre, int cbeg, int cend, int c,
                              unsigned* amb_list, hipStream_t stream);
hipError_t batch_prepare_recheck(int nrow, int ncol_max);
hipError_t launch_batch_recheck(BatchInst* insts, BatchCtl* ctl, const unsigned* amb_list,
                                int nrow, int ncol_max, hipStream_t stream);
hipError_t launch_batch_count(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                              hipStream_t stream);
hipError_t launch_batch_advance(BatchInst* insts, int n_inst, hipStream_t stream);
hipError_t launch_batch_split(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                              hipStream_t stream);
hipError_t launch_batch_volume(BatchInst* insts, int n_inst, hipStream_t stream);
// Alpha pass of a batch level (after the FP64 re-decision, before the count): candidates per
// bookkeeping tile and instance, segments per alpha class, gathered boxes; then per alpha class
// the centre objective, the fused optimizer and the scatter of decided classes.
hipError_t launch_batch_alpha_cand(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                                   unsigned* tile_cand, float select, hipStream_t stream);
hipError_t launch_batch_alpha_plan(BatchInst* insts, BatchCtl* ctl, const BatchAlphaBuf* bufs,
                                   int n_acls, hipStream_t stream);
hipError_t launch_batch_alpha_gather(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                                     const unsigned* tile_cand, const BatchAlphaBuf* bufs, float select,
                                     hipStream_t stream);
// Kernel template of an instance's alpha pass (nc class, global state, register paths) and the
// LDS of its fused optimizer; key packs the template.
int batch_alpha_key(const NetDev& net, const PropDev& prop, size_t* lds);
hipError_t batch_alpha_prepare(int key, size_t lds);
hipError_t launch_batch_alpha_class(int key, size_t lds, BatchInst* insts, BatchCtl* ctl, int c,
                                    const BatchAlphaBuf& buf, const AlphaArgs& base, int steps,
                                    hipStream_t stream);
int batch_num_cu();
