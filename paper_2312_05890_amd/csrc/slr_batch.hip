// gfx950 kernels of batched exact counts: many independent instances (each with its own network,
// property, box, depth and leaf budget) advance level by level together.
//
// Per level the launch sequence is fixed and every kernel reads its work size on the device:
//   plan     (one workgroup) applies the previous level's split, then lays out this level's
//            work: per kernel class, the bound tiles of its instances (prefix offsets), and the
//            1024-box bookkeeping tiles of all instances;
//   bound    one persistent kernel per class: workgroups pop tiles from the class's work queue
//            (an atomic head), find the tile's instance by binary search over the offsets and run
//            the LDS-staged bound tile on that instance's network (its descriptor is read from
//            device memory); ambiguous boxes are listed as (instance << 22 | box);
//   recheck  FP64 re-decision of the listed boxes, one per wavefront;
//   count    class histograms per instance and level (64-bit atomics: exact and order-free);
//   advance  the budget rule of each instance (stop at its depth, or when its leaves would
//            exceed its budget), one thread per instance;
//   split    bisection of the undecided boxes of the instances that go on.
// Instances that have stopped get no tiles; levels past every instance's depth are empty.
// The host can therefore capture all levels once and replay them as one graph.
#include "slr_device.h"

namespace {

// Largest i in [lo, hi) with pre[i] <= t (pre non-decreasing, pre[lo] = 0 <= t).
__device__ __forceinline__ int find_owner(const unsigned* __restrict__ pre, int lo, int hi,
                                          unsigned t) {
    int a = lo, b = hi - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (pre[m] <= t) a = m;
        else b = m - 1;
    }
    return a;
}

__global__ __launch_bounds__(256) void batch_init_kernel(BatchInst* insts, int n_inst) {
    const int i = blockIdx.x;
    if (i >= n_inst) return;
    BatchInst& I = insts[i];
    for (int t = threadIdx.x; t < SLR_MAX_LEVELS; t += blockDim.x) {
        I.stats[t].unsafe_cnt = 0;
        I.stats[t].safe_cnt = 0;
        I.stats[t].undecided_cnt = 0;
        I.stats[t].pad = 0;
    }
    for (int k = threadIdx.x; k < I.d; k += blockDim.x) {
        I.lo[0][k] = I.root[k];
        I.hi[0][k] = I.root[I.d + k];
    }
    if (threadIdx.x < 16) I.perr[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        I.path[0][0] = 1ull;
        I.n = 1;
        I.coff = 0;
        I.cn = 1;
        I.prefix_pending = 0;
        if (I.pk > 0) {   // first level: the top of the tree (boxes from batch_prefix_kernel)
            I.n = ((long long)2 << I.pk) - 1;
            I.coff = ((long long)1 << I.pk) - 1;
            I.cn = (long long)1 << I.pk;
            I.prefix_pending = 1;
        }
        I.n_next = 0;
        I.resolved = 0;
        I.bounded = 0;
        I.cur = 0;
        I.level = I.pk;
        I.active = 1;
        I.split_pending = 0;
        I.status = 0;
        I.stop_level = 0;
        I.stopped = 0;
        I.levels = 0;
        I.rechecks = 0;
        I.err = 0;
        I.acand = 0;
        I.aseg = 0;
        I.alen = 0;
        I.atape = 0;
        I.n_alpha_boxes = 0;
        I.n_alpha_decided = 0;
    }
}

// The complete subtree of depth pk (heap order, split rule of the level loop) of every instance
// that has one; grid: boxes x instances.
__global__ __launch_bounds__(256) void batch_prefix_kernel(BatchInst* insts, int n_inst) {
    extern __shared__ float prefix_stage[];   // 2 * 256 * (largest d) floats
    const int i = blockIdx.y;
    if (i >= n_inst) return;
    BatchInst& I = insts[i];
    if (I.pk <= 0) return;
    const int64_t N = ((int64_t)2 << I.pk) - 1;
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    if (i0 >= N) return;   // uniform over the workgroup
    const int d = I.d;
    prefix_block(N, i0, d, I.root, I.root + d, I.lo[0], I.hi[0], I.path[0], I.perr, 1, prefix_stage);
}

// Replay of the top's level once its classes are final: boxes the level loop would not visit get
// class 4, the visited ones of depths 0 .. pk - 1 are counted; grid: boxes x instances.
__global__ __launch_bounds__(256) void batch_prefix_replay_kernel(BatchInst* insts, int n_inst) {
    const int i = blockIdx.y;
    if (i >= n_inst) return;
    BatchInst& I = insts[i];
    if (!I.prefix_pending) return;
    const int64_t N = ((int64_t)2 << I.pk) - 1;
    if ((int64_t)blockIdx.x * 256 >= N) return;
    prefix_replay_block(N, I.pk, I.cls, I.stats, (int64_t)blockIdx.x * 256);
}

// The FP64 re-decisions of top boxes that the level loop does not visit (class 4 after the
// replay) are not the loop's: each such listed box takes one off its instance's counter.
__global__ __launch_bounds__(256) void batch_prefix_recheck_uncount_kernel(BatchInst* insts, const BatchCtl* ctl,
                                                                           const unsigned* __restrict__ amb_list) {
    const unsigned n = ctl->amb_count;
    for (unsigned k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const unsigned e = amb_list[k];
        BatchInst& I = insts[e >> 22];
        if (I.cls[e & 0x3FFFFFu] == 4) atomicAdd(&I.rechecks, ~0ull);   // minus one
    }
}

// One workgroup of 1024 threads, thread i = instance i (instances are sorted by kernel class,
// so each class is a contiguous run): applies the pending split, then two exclusive scans over
// the instances, of their bound tiles (bpre: offset inside the instance's class) and of their
// 1024-box bookkeeping tiles (cpre).
__device__ __forceinline__ unsigned block_exclusive_scan1024(unsigned v, unsigned* wtot, unsigned* total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned x = __shfl_up(incl, o);
        if (lane >= o) incl += x;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    unsigned pre = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) pre += wtot[w];
        all += wtot[w];
    }
    *total = all;
    __syncthreads();
    return pre + incl - v;
}

__global__ __launch_bounds__(1024) void batch_plan_kernel(BatchInst* insts, int n_inst, BatchCtl* ctl,
                                                          unsigned* __restrict__ bpre,
                                                          unsigned* __restrict__ cpre,
                                                          int n_classes) {
    __shared__ unsigned wtot[16];
    __shared__ unsigned pstart[SLR_MAX_CLASSES];
    const int i = threadIdx.x;
    if (i < n_classes) ctl->head[i] = 0;
    if (i == 0) ctl->amb_count = 0;
    unsigned tb = 0, tc = 0;
    int cid = -1;
    if (i < n_inst) {
        BatchInst& I = insts[i];
        if (I.split_pending) {
            I.n = I.n_next;
            I.coff = 0;
            I.cn = I.n;
            I.cur ^= 1;
            I.level += 1;
            I.split_pending = 0;
        }
        const long long n = I.active ? I.n : 0;
        const long long cn = I.active ? I.cn : 0;
        cid = I.cls_id;
        const int T = ctl->tbox[cid];
        tb = (unsigned)((n + T - 1) / T);
        tc = (unsigned)((cn + kTile - 1) / kTile);
    }
    unsigned tot_b, tot_c;
    const unsigned pb = block_exclusive_scan1024(tb, wtot, &tot_b);
    const unsigned pc = block_exclusive_scan1024(tc, wtot, &tot_c);
    // the first instance of each class publishes its scan value
    const bool first = i < n_inst && (i == 0 || insts[i - 1].cls_id != cid);
    if (first) pstart[cid] = pb;
    __syncthreads();
    if (i < n_inst) {
        bpre[i] = pb - pstart[cid];
        cpre[i] = pc;
        const bool last = i == n_inst - 1 || insts[i + 1].cls_id != cid;
        if (last) ctl->ntiles[cid] = pb + tb - pstart[cid];
    }
    if (i == 0) {
        cpre[n_inst] = tot_c;
        ctl->ctiles = tot_c;
    }
}

// insts is read-only here and aliases nothing the kernel writes, so descriptor loads need not be
// repeated after the tile's stores.
template <int NCOL, int NT, int UW, int NW, bool SMOOTH = false>
__global__ __launch_bounds__(NW * 64) void batch_bound_kernel(const BatchInst* __restrict__ insts,
                                                              BatchCtl* ctl,
                                                              const unsigned* __restrict__ bpre,
                                                              int cbeg, int cend, int c,
                                                              unsigned* __restrict__ amb_list) {
    __shared__ unsigned s_t;
    const unsigned total = ctl->ntiles[c];
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(&ctl->head[c], 1u);
        __syncthreads();
        // uniform across the workgroup: keeps the instance index and every descriptor field
        // in scalar registers (scalar loads) instead of per-lane copies
        const unsigned t = __builtin_amdgcn_readfirstlane(s_t);
        __syncthreads();
        if (t >= total) break;
        const int i = find_owner(bpre, cbeg, cend, t);
        const BatchInst& I = insts[i];
        const int64_t box0 = (int64_t)(t - bpre[i]) * (NT * 16);
        bound_tile<NCOL, NT, UW, NW, SMOOTH>(I.net, I.prop, I.n, box0, I.lo[I.cur], I.hi[I.cur], I.glo,
                                     I.ghi, I.cls, 0, I.sp, amb_list, &ctl->amb_count,
                                     (unsigned)i << 22);
        __syncthreads();   // the tile's LDS is reused by the next tile
    }
}

__global__ __launch_bounds__(256) void batch_recheck_kernel(BatchInst* insts, BatchCtl* ctl,
                                                            const unsigned* __restrict__ amb_list,
                                                            int nrow, int ncol_max) {
    extern __shared__ double sm[];
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    double* ws = sm + (size_t)wave * (2 * nrow * ncol_max + 2 * SLR_MAX_D);
    const unsigned total = ctl->amb_count;
    for (unsigned k = blockIdx.x * waves + wave; k < total; k += gridDim.x * waves) {
        const unsigned e = __builtin_amdgcn_readfirstlane(amb_list[k]);   // one box per wave
        BatchInst& I = insts[e >> 22];
        recheck_box(I.net, I.prop, (int64_t)(e & 0x3FFFFFu), I.lo[I.cur], I.hi[I.cur], nullptr,
                    nullptr, I.cls, &I.rechecks, ws, nrow);
    }
}

__global__ __launch_bounds__(256) void batch_count_kernel(BatchInst* insts, int n_inst,
                                                          BatchCtl* ctl,
                                                          const unsigned* __restrict__ cpre) {
    const unsigned total = ctl->ctiles;
    for (unsigned t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = find_owner(cpre, 0, n_inst, t);
        BatchInst& I = insts[i];
        count_tile(I.cn, I.cls + I.coff, I.tile_und, I.stats + I.level, (int64_t)(t - cpre[i]));
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void batch_advance_kernel(BatchInst* insts, int n_inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    BatchInst& I = insts[i];
    if (!I.active) return;
    if (I.prefix_pending) {   // the level loop's decisions at depths 0 .. pk, depth by depth
        I.prefix_pending = 0;
        for (int t = 0; t <= I.pk; ++t) {
            const LevelStats h = I.stats[t];
            const long long und = (long long)h.undecided_cnt;
            I.bounded += (long long)(h.unsafe_cnt + h.safe_cnt) + und;
            I.levels = t + 1;
            I.resolved += (long long)(h.unsafe_cnt + h.safe_cnt);
            if (und == 0) {
                I.active = 0;
                I.status = 0;
                return;
            }
            if (t == I.max_depth || I.resolved + 2 * und > I.max_leaves) {
                I.active = 0;
                I.stopped = 1;
                I.stop_level = t;
                I.status = 1;
                return;
            }
            if (t < I.pk) {
                if (I.perr[t]) I.err |= 1u;   // a split the level loop makes
            } else {
                I.split_pending = 1;
                I.n_next = 2 * und;
            }
        }
        return;
    }
    const LevelStats h = I.stats[I.level];
    I.bounded += I.n;
    I.levels = I.level + 1;
    I.resolved += (long long)(h.unsafe_cnt + h.safe_cnt);
    const long long und = (long long)h.undecided_cnt;
    if ((long long)(h.unsafe_cnt + h.safe_cnt) + und != I.n) I.err |= 4u;
    if (und == 0) {
        I.active = 0;
        I.status = 0;
    } else if (I.level == I.max_depth || I.resolved + 2 * und > I.max_leaves) {
        I.active = 0;
        I.stopped = 1;
        I.stop_level = I.level;
        I.status = 1;
    } else {
        I.split_pending = 1;
        I.n_next = 2 * und;
    }
}

__global__ __launch_bounds__(256) void batch_split_kernel(BatchInst* insts, int n_inst,
                                                          BatchCtl* ctl,
                                                          const unsigned* __restrict__ cpre) {
    extern __shared__ float split_stage[];   // 2 * kTile * kSplitStageD floats
    const unsigned total = ctl->ctiles;
    for (unsigned t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = find_owner(cpre, 0, n_inst, t);
        BatchInst& I = insts[i];
        if (!I.split_pending) continue;
        const int c = I.cur;
        const long long o = I.coff;   // the depth-pk slice of the top's level, else 0
        split_tile(I.cn, I.d, I.cls + o, I.tile_und, I.lo[c] + o * I.d, I.hi[c] + o * I.d,
                   I.path[c] + o, I.lo[c ^ 1], I.hi[c ^ 1], I.path[c ^ 1], &I.err, I.max_leaves,
                   (int64_t)(t - cpre[i]), split_stage);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Alpha pass of a level (batches with alpha options)
// ---------------------------------------------------------------------------------------------
// An instance takes part at this level when it has an alpha class, is active and has reached its
// first alpha depth; a box is a candidate when it is undecided and (select > 0) its plain bounds
// lie within select of a decision.
__device__ __forceinline__ bool alpha_level(const BatchInst& I) {
    return I.acls_id >= 0 && I.active && I.level >= I.alpha_min_depth;
}

__device__ __forceinline__ bool alpha_candidate(const BatchInst& I, int64_t b, float select) {
    if (b >= I.n || I.cls[b] != 0) return false;
    if (select <= 0.f) return true;
    const int rows = I.prop.rows;
    return slr_decision_distance(I.glo + b * rows, I.ghi + b * rows, rows) <= select;
}

// Candidates per 1024-box bookkeeping tile, and per instance.
__global__ __launch_bounds__(256) void batch_alpha_cand_kernel(BatchInst* insts, int n_inst,
                                                               BatchCtl* ctl,
                                                               const unsigned* __restrict__ cpre,
                                                               unsigned* __restrict__ tile_cand,
                                                               float select) {
    __shared__ unsigned red[4];
    const unsigned total = ctl->ctiles;
    for (unsigned t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = find_owner(cpre, 0, n_inst, t);
        BatchInst& I = insts[i];
        unsigned cnt = 0;
        if (alpha_level(I)) {
            const int64_t b0 = (int64_t)(t - cpre[i]) * kTile + threadIdx.x * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) cnt += alpha_candidate(I, b0 + q, select) ? 1u : 0u;
        }
        cnt = block_sum256(cnt, red);
        if (threadIdx.x == 0) {
            tile_cand[t] = cnt;
            if (cnt) atomicAdd(&I.acand, cnt);
        }
        __syncthreads();
    }
}

// Segments: per alpha class (one thread each), its instances in order take min(candidates,
// room) boxes at 16-aligned offsets of the class buffers, and tape room for their tiles.
__global__ void batch_alpha_plan_kernel(BatchInst* insts, BatchCtl* ctl, const BatchAlphaBuf* bufs,
                                        int n_acls) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_acls) return;
    const BatchAlphaBuf& B = bufs[c];
    unsigned used = 0;
    unsigned long long tape = 0;
    for (int k = 0; k < B.ninst; ++k) {
        BatchInst& I = insts[B.inst[k]];
        const unsigned room = B.cap - used;
        const unsigned len = min(I.acand, room);
        I.aseg = used;
        I.alen = len;
        I.atape = tape;
        I.n_alpha_boxes += len;
        I.acand = 0;
        B.seg[k] = used;
        const unsigned tiles = (len + 15) / 16;
        used += 16 * tiles;
        tape += (unsigned long long)tiles * I.atile_floats;
    }
    ctl->antiles[c] = used / 16;
}

// The candidates of one bookkeeping tile go, in box order, to their instance's segment (those
// beyond its length stay undecided with their plain bounds).
__global__ __launch_bounds__(256) void batch_alpha_gather_kernel(BatchInst* insts, int n_inst,
                                                                 BatchCtl* ctl,
                                                                 const unsigned* __restrict__ cpre,
                                                                 const unsigned* __restrict__ tile_cand,
                                                                 const BatchAlphaBuf* bufs,
                                                                 float select) {
    __shared__ unsigned red[4];
    __shared__ unsigned wpre[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned total = ctl->ctiles;
    for (unsigned t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = find_owner(cpre, 0, n_inst, t);
        const BatchInst& I = insts[i];
        if (!alpha_level(I) || I.alen == 0 || tile_cand[t] == 0) continue;   // uniform
        // candidates of the instance's earlier tiles
        unsigned pre = 0;
        for (unsigned k = cpre[i] + tid; k < t; k += 256) pre += tile_cand[k];
        const unsigned base = block_sum256(pre, red);
        const int64_t b0 = (int64_t)(t - cpre[i]) * kTile + tid * 4;
        unsigned flags = 0, cnt = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (alpha_candidate(I, b0 + q, select)) {
                flags |= 1u << q;
                ++cnt;
            }
        unsigned incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned x = __shfl_up(incl, o);
            if (lane >= o) incl += x;
        }
        if (lane == 63) wpre[wave] = incl;
        __syncthreads();
        unsigned rank = base + incl - cnt;
        for (int w = 0; w < wave; ++w) rank += wpre[w];
        const BatchAlphaBuf& B = bufs[I.acls_id];
        const int d = I.d;
        const float* lo = I.lo[I.cur];
        const float* hi = I.hi[I.cur];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!(flags & (1u << q))) continue;
            if (rank < I.alen) {
                const int64_t b = b0 + q;
                const size_t o = (size_t)I.aseg * B.dmax + (size_t)rank * d;
                for (int k = 0; k < d; ++k) {
                    B.lo[o + k] = lo[b * d + k];
                    B.hi[o + k] = hi[b * d + k];
                }
                B.list[I.aseg + rank] = (unsigned)b;
            }
            ++rank;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void batch_volume_kernel(BatchInst* insts, int n_inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    BatchInst& I = insts[i];
    volume_body(I.stats, I.levels, I.stop_level, I.stopped, I.vol, I.counts, &I.err);
}

// ---------------------------------------------------------------------------------------------
// Host side: kernel classes and launches
// ---------------------------------------------------------------------------------------------
int ncol_class_b(int d) {
    const int c = d + 3;
    if (c <= 12) return c;
    if (c <= 14) return 14;
    return -1;
}

template <int NCOL, int NT, int UW, int NW, bool SMOOTH = false>
const void* kern_ptr() {
    return (const void*)batch_bound_kernel<NCOL, NT, UW, NW, SMOOTH>;
}

// nt < 0 selects the tanh / sigmoid kernels (default shapes only) of the shape (-nt, uw, nw).
const void* class_kernel(int ncol, TileShape t) {
    if (t.nt < 0) {
#define SLR_S(C)                                                                           \
        if (ncol == C) {                                                                   \
            if (t.nt == -4 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 4, 1, 4, true>(); \
            if (t.nt == -2 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 2, 1, 4, true>(); \
            if (t.nt == -1 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 1, 1, 4, true>(); \
            if (t.nt == -1 && t.uw == 2 && t.nw == 4) return kern_ptr<C, 1, 2, 4, true>(); \
            return nullptr;                                                                \
        }
        SLR_S(4) SLR_S(5) SLR_S(6) SLR_S(7) SLR_S(8) SLR_S(9) SLR_S(10) SLR_S(11) SLR_S(12) SLR_S(14)
#undef SLR_S
        return nullptr;
    }
#define SLR_T(C)                                                                    \
    if (ncol == C) {                                                                \
        if (t.nt == 4 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 4, 1, 4>();     \
        if (t.nt == 2 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 2, 1, 4>();     \
        if (t.nt == 1 && t.uw == 1 && t.nw == 4) return kern_ptr<C, 1, 1, 4>();     \
        if (t.nt == 1 && t.uw == 2 && t.nw == 4) return kern_ptr<C, 1, 2, 4>();     \
        if (t.nt == 1 && t.uw == 1 && t.nw == 8) return kern_ptr<C, 1, 1, 8>();     \
        if (t.nt == 1 && t.uw == 2 && t.nw == 8) return kern_ptr<C, 1, 2, 8>();     \
        return nullptr;                                                             \
    }
    SLR_T(4) SLR_T(5) SLR_T(6) SLR_T(7) SLR_T(8) SLR_T(9) SLR_T(10) SLR_T(11) SLR_T(12) SLR_T(14)
#undef SLR_T
    return nullptr;
}

int g_cu = 0;

}  // namespace

int batch_num_cu() {
    if (g_cu == 0) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            g_cu = cu;
        else
            g_cu = 256;
        (void)hipGetLastError();
    }
    return g_cu;
}

bool batch_class_supported(int ncol, TileShape t) { return class_kernel(ncol, t) != nullptr; }

int batch_class_of(const NetDev& net, const PropDev& prop, int* ncol, TileShape* t) {
    (void)prop;
    *ncol = ncol_class_b(net.d);
    if (*ncol < 0 || net.mt_max > 8) return -1;
    if (net.act != SLR_ACT_RELU) {   // the smooth kernels: default shapes, marked by nt < 0
        if (net.mt_max <= 1) *t = {-4, 1, 4};
        else if (net.mt_max == 2) *t = {-2, 1, 4};
        else if (net.mt_max <= 4) *t = {-1, 1, 4};
        else *t = {-1, 2, 4};
        return batch_class_supported(*ncol, *t) ? 0 : -1;
    }
    // the tuned shape of this class when the batch kernels have it, else the default
    *t = tile_shape_for(net.d, net.mt_max);
    if (!batch_class_supported(*ncol, *t)) {
        if (net.mt_max <= 1) *t = {4, 1, 4};
        else if (net.mt_max == 2) *t = {2, 1, 4};
        else if (net.mt_max <= 4) *t = {1, 1, 4};
        else *t = {1, 2, 4};
    }
    return batch_class_supported(*ncol, *t) ? 0 : -1;
}

size_t batch_bound_lds(int ncol, TileShape t, int mt_max, int rows) {
    t.nt = t.nt < 0 ? -t.nt : t.nt;   // the smooth kernels' marker
    return bound_lds_bytes(ncol, t, mt_max, rows);
}

hipError_t batch_prepare_class(int ncol, TileShape t, size_t lds, int* blocks) {
    const void* k = class_kernel(ncol, t);
    if (!k) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, t.nw * 64, lds) != hipSuccess || nb < 1) nb = 1;
    (void)hipGetLastError();
    *blocks = nb * batch_num_cu();
    return hipSuccess;
}

hipError_t launch_batch_init(BatchInst* insts, int n_inst, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_init_kernel, dim3(n_inst), dim3(64), 0, stream, insts, n_inst);
    return hipGetLastError();
}

hipError_t launch_batch_prefix(BatchInst* insts, int n_inst, int pk_max, int d_max, hipStream_t stream) {
    if (pk_max <= 0) return hipSuccess;
    if (pk_max > 15 || d_max < 1 || d_max > SLR_MAX_D) return hipErrorInvalidValue;
    const unsigned bx = (unsigned)((((int64_t)2 << pk_max) - 1 + 255) / 256);
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_prefix_kernel, dim3(bx, n_inst), dim3(256), sizeof(float) * 2 * 256 * d_max,
                       stream, insts, n_inst);
    return hipGetLastError();
}

hipError_t launch_batch_prefix_replay(BatchInst* insts, int n_inst, int pk_max, BatchCtl* ctl,
                                      const unsigned* amb_list, hipStream_t stream) {
    if (pk_max <= 0) return hipSuccess;
    if (pk_max > 15) return hipErrorInvalidValue;
    const unsigned bx = (unsigned)((((int64_t)2 << pk_max) - 1 + 255) / 256);
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_prefix_replay_kernel, dim3(bx, n_inst), dim3(256), 0, stream, insts, n_inst);
    hipLaunchKernelGGL(batch_prefix_recheck_uncount_kernel, dim3(64), dim3(256), 0, stream, insts,
                       (const BatchCtl*)ctl, amb_list);
    return hipGetLastError();
}

hipError_t launch_batch_plan(BatchInst* insts, int n_inst, BatchCtl* ctl, unsigned* bpre,
                             unsigned* cpre, int n_classes, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(1024), 0, stream, insts, n_inst, ctl, bpre,
                       cpre, n_classes);
    return hipGetLastError();
}

hipError_t launch_batch_bound(int ncol, TileShape t, int blocks, size_t lds, BatchInst* insts,
                              BatchCtl* ctl, const unsigned* bpre, int cbeg, int cend, int c,
                              unsigned* amb_list, hipStream_t stream) {
    const void* k = class_kernel(ncol, t);
    if (!k) return hipErrorInvalidValue;
    void* args[] = {&insts, &ctl, (void*)&bpre, &cbeg, &cend, &c, &amb_list};
    (void)hipGetLastError();
    return hipLaunchKernel(k, dim3(blocks), dim3(t.nw * 64), args, lds, stream);
}

namespace {
void recheck_shape(int nrow, int ncol_max, int* waves, size_t* lds) {
    const size_t per_wave = sizeof(double) * (2 * (size_t)nrow * ncol_max + 2 * SLR_MAX_D);
    int w = 4;
    while (w > 1 && per_wave * w > 150 * 1024) --w;
    *waves = w;
    *lds = per_wave * w;
}
}  // namespace

hipError_t batch_prepare_recheck(int nrow, int ncol_max) {
    int waves;
    size_t lds;
    recheck_shape(nrow, ncol_max, &waves, &lds);
    if (lds <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)batch_recheck_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

hipError_t launch_batch_recheck(BatchInst* insts, BatchCtl* ctl, const unsigned* amb_list,
                                int nrow, int ncol_max, hipStream_t stream) {
    int waves;
    size_t lds;
    recheck_shape(nrow, ncol_max, &waves, &lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_recheck_kernel, dim3(1024), dim3(64 * waves), lds, stream, insts, ctl,
                       amb_list, nrow, ncol_max);
    return hipGetLastError();
}

hipError_t launch_batch_count(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                              hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_count_kernel, dim3(2048), dim3(256), 0, stream, insts, n_inst, ctl, cpre);
    return hipGetLastError();
}

hipError_t launch_batch_advance(BatchInst* insts, int n_inst, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_advance_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, stream,
                       insts, n_inst);
    return hipGetLastError();
}

hipError_t launch_batch_split(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                              hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_split_kernel, dim3(2048), dim3(256),
                       2 * sizeof(float) * kTile * kSplitStageD, stream, insts, n_inst, ctl, cpre);
    return hipGetLastError();
}

hipError_t launch_batch_alpha_cand(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                                   unsigned* tile_cand, float select, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_alpha_cand_kernel, dim3(2048), dim3(256), 0, stream, insts, n_inst, ctl,
                       cpre, tile_cand, select);
    return hipGetLastError();
}

hipError_t launch_batch_alpha_plan(BatchInst* insts, BatchCtl* ctl, const BatchAlphaBuf* bufs,
                                   int n_acls, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_alpha_plan_kernel, dim3(1), dim3(64), 0, stream, insts, ctl, bufs, n_acls);
    return hipGetLastError();
}

hipError_t launch_batch_alpha_gather(BatchInst* insts, int n_inst, BatchCtl* ctl, const unsigned* cpre,
                                     const unsigned* tile_cand, const BatchAlphaBuf* bufs, float select,
                                     hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_alpha_gather_kernel, dim3(2048), dim3(256), 0, stream, insts, n_inst,
                       ctl, cpre, tile_cand, bufs, select);
    return hipGetLastError();
}

hipError_t launch_batch_volume(BatchInst* insts, int n_inst, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_volume_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, stream,
                       insts, n_inst);
    return hipGetLastError();
}
