// gfx950 kernels of the SLR counter (single instance): the LDS-staged bound kernel (its tile code
// is in slr_device.h), the FP64 re-decision, level bookkeeping, the register-resident bound
// kernel and the sample forward pass; launch and shape-class selection.
#include "slr_device.h"

#include <atomic>

namespace {

// SMOOTH: tanh / sigmoid networks (parallel-line relaxation); a separate instantiation keeps the
// ReLU kernels' registers and occupancy unchanged.
// SCORE: the crossing-score split rule (the side to bisect per box into dimsel).
template <int NCOL, int NT, int UW, int NW, bool SMOOTH = false, bool SCORE = false>
__global__ __launch_bounds__(NW * 64) void bound_f32_kernel(
    NetDev net, PropDev prop, int64_t n, const float* __restrict__ blo,
    const float* __restrict__ bhi, float* __restrict__ g_lo, float* __restrict__ g_hi,
    int8_t* __restrict__ cls, int raw, int SP, unsigned* __restrict__ amb_list,
    unsigned* __restrict__ amb_count, unsigned list_base, int8_t* __restrict__ dimsel,
    int split_layers) {
    bound_tile<NCOL, NT, UW, NW, SMOOTH, SCORE>(net, prop, n, (int64_t)blockIdx.x * (NT * 16), blo,
                                                bhi, g_lo, g_hi, cls, raw, SP, amb_list, amb_count,
                                                list_base, dimsel, split_layers);
}

__global__ __launch_bounds__(256) void recheck64_kernel(NetDev net, PropDev prop, int64_t n,
                                                        const float* __restrict__ blo,
                                                        const float* __restrict__ bhi,
                                                        float* __restrict__ g_lo,
                                                        float* __restrict__ g_hi,
                                                        int8_t* __restrict__ cls,
                                                        unsigned long long* counter,
                                                        const unsigned* __restrict__ list,
                                                        const unsigned* __restrict__ list_count,
                                                        int nrow) {
    extern __shared__ double sm[];
    __shared__ int llist[256];
    __shared__ int cnt;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int waves = blockDim.x >> 6;
    const int ncol = net.d + 2;
    double* ws = sm + (size_t)wave * (2 * nrow * ncol + 2 * SLR_MAX_D);
    if (list) {
        const int64_t total = min((int64_t)*list_count, n);
        for (int64_t i = (int64_t)blockIdx.x * waves + wave; i < total; i += (int64_t)gridDim.x * waves)
            recheck_box(net, prop, list[i], blo, bhi, g_lo, g_hi, cls, counter, ws, nrow);
        return;
    }
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        if (tid == 0) cnt = 0;
        __syncthreads();
        const int64_t i = base + tid;
        if (i < n && cls[i] == 3) llist[atomicAdd(&cnt, 1)] = tid;
        __syncthreads();
        const int m = cnt;
        for (int q = wave; q < m; q += waves)
            recheck_box(net, prop, base + llist[q], blo, bhi, g_lo, g_hi, cls, counter, ws, nrow);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void level_count_kernel(int64_t n, const int8_t* __restrict__ cls,
                                                          unsigned* __restrict__ tile_und,
                                                          LevelStats* stats) {
    count_tile(n, cls, tile_und, stats, blockIdx.x);
}

__global__ __launch_bounds__(256) void split_kernel(int64_t n, int d, const int8_t* __restrict__ cls,
                                                    const unsigned* __restrict__ tile_und,
                                                    const float* __restrict__ lo,
                                                    const float* __restrict__ hi,
                                                    const unsigned long long* __restrict__ path,
                                                    float* __restrict__ lo2, float* __restrict__ hi2,
                                                    unsigned long long* __restrict__ path2,
                                                    unsigned* err, int64_t cap,
                                                    const int8_t* __restrict__ dimsel) {
    extern __shared__ float split_stage[];
    split_tile(n, d, cls, tile_und, lo, hi, path, lo2, hi2, path2, err, cap, blockIdx.x,
               d <= kSplitStageD ? split_stage : nullptr, dimsel);
}

// Depth-first stack count, one chunk of boxes of mixed depths (the depth of a box is the position
// of its path id's leading 1 bit: root 1, children 2p and 2p + 1).  Unsafe and safe boxes add to
// their depth's counters; an undecided box at max_depth (or every box, with all_undecided) adds
// to the undecided counter of its depth and, unless all_undecided, gets class 4 so the split
// leaves it; the remaining undecided boxes are counted per 1024-box tile (for the split's
// offsets) and in *split_total.  Per-depth counts go through an LDS histogram, then one 64-bit
// atomic per non-zero entry.
__global__ __launch_bounds__(256) void stack_count_kernel(int64_t n, int8_t* __restrict__ cls,
                                                          const unsigned long long* __restrict__ path,
                                                          int max_depth, int all_undecided,
                                                          unsigned* __restrict__ tile_und,
                                                          LevelStats* stats, unsigned* split_total) {
    __shared__ unsigned hist[kMaxDepthLevels * 3];
    __shared__ unsigned red[4];
    const int tid = threadIdx.x;
    for (int e = tid; e < kMaxDepthLevels * 3; e += 256) hist[e] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile + tid * 4;
    unsigned nsplit = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t i = base + q;
        if (i < n) {
            const int depth = 63 - __clzll(path[i]);
            const int8_t c = all_undecided ? 0 : cls[i];
            if (c == 1) {
                atomicAdd(&hist[depth * 3 + 0], 1u);
            } else if (c == 2) {
                atomicAdd(&hist[depth * 3 + 1], 1u);
            } else if (c == 0) {
                if (all_undecided || depth >= max_depth) {
                    atomicAdd(&hist[depth * 3 + 2], 1u);
                    if (!all_undecided) cls[i] = 4;
                } else {
                    ++nsplit;
                }
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < kMaxDepthLevels * 3; e += 256) {
        const unsigned h = hist[e];
        if (h) {
            unsigned long long* f = reinterpret_cast<unsigned long long*>(stats + e / 3) + (e % 3);
            atomicAdd(f, (unsigned long long)h);
        }
    }
    nsplit = block_sum256(nsplit, red);
    if (tid == 0) {
        if (tile_und) tile_und[blockIdx.x] = nsplit;
        if (nsplit) atomicAdd(split_total, nsplit);
    }
}

// Exact volumes of a count whose undecided leaves may lie at any depth: sum_t n_t 2^(Dm - t)
// over every level for each class in 64-bit integers (they must partition 2^Dm exactly), then
// one conversion to float64 each.
__global__ void stack_volume_kernel(const LevelStats* stats, int levels, double* out3,
                                    unsigned long long* out_counts, unsigned* err) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int Dm = levels - 1;
    unsigned long long s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int t = 0; t < levels; ++t) {
        const unsigned long long v[3] = {stats[t].unsafe_cnt, stats[t].safe_cnt, stats[t].undecided_cnt};
        for (int k = 0; k < 3; ++k) {
            s[k] += v[k] << (Dm - t);
            c[k] += v[k];
        }
    }
    if (s[0] + s[1] + s[2] != (1ull << Dm)) atomicOr(err, 2u);
    for (int k = 0; k < 3; ++k) {
        out3[k] = ldexp((double)s[k], -Dm);
        out_counts[k] = c[k];
    }
}

__global__ void volume_kernel(const LevelStats* stats, int levels, int stop_level, int stopped,
                              double* out3, unsigned long long* out_counts, unsigned* err) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    volume_body(stats, levels, stop_level, stopped, out3, out_counts, err);
}

// ------------------------------------------------------------------------------------------
// Register-resident bound kernel for narrow networks (every hidden width <= 16 MT, d + 3 <=
// NCOL).  One wavefront owns 16 boxes through the whole network: because the accumulator
// layout of the 16x16x4 MFMA equals its B-operand layout (lane 16 g + j holds neurons
// 16 mt + 4 g + v of box j), the post-activation state of M tile mt is directly the B operand
// of K-steps 4 mt .. 4 mt + 3 of the next layer.  No LDS round trips and no workgroup barriers;
// the per-box bound on |value| is a lane-local max plus two cross-lane shuffles.
// ------------------------------------------------------------------------------------------
// Accumulate K-steps s0 .. s0+nst-1 of one 16-row tile group: Z[mo] += A(mo, s) X[s % 4].
template <int NCOL, int MO>
__device__ __forceinline__ void mfma_steps(f32x4 (&Z)[MO][NCOL], const f32x4 (&X)[NCOL],
                                           const float* __restrict__ wf, int ksa, int s0, int nst) {
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) {
        if (ss < nst) {
#pragma unroll
            for (int mo = 0; mo < MO; ++mo) {
                const float aw = wf[(mo * ksa + s0 + ss) * 64];
                const float aa = fabsf(aw);
#pragma unroll
                for (int c = 0; c < NCOL - 2; ++c) Z[mo][c] = mfma16(aw, X[c][ss], Z[mo][c]);
                Z[mo][NCOL - 2] = mfma16(aa, X[NCOL - 2][ss], Z[mo][NCOL - 2]);
                Z[mo][NCOL - 1] = mfma16(aa, X[NCOL - 1][ss], Z[mo][NCOL - 1]);
            }
        }
    }
}

// Epilogue of tile mt of a hidden layer held in Y (pre-activations, bias included).
template <int NCOL, int MT>
__device__ __forceinline__ float tile_epilogue(const f32x4 (&Y)[MT][NCOL], const float (&epsv)[MT][4],
                                               int mt, int tiles, int r_last, int g,
                                               const EpiConst& ek, f32x4 (&X)[NCOL]) {
    float a[NCOL][4], eps[4];
    bool valid[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        valid[v] = mt < tiles && row_valid(mt, g, v, tiles, r_last);
        eps[v] = epsv[mt][v];
#pragma unroll
        for (int c = 0; c < NCOL; ++c) a[c][v] = Y[mt][c][v];
    }
    const float e = relu_epilogue<NCOL>(a, eps, valid, ek);
#pragma unroll
    for (int c = 0; c < NCOL; ++c) X[c] = f32x4{a[c][0], a[c][1], a[c][2], a[c][3]};
    return e;
}

// One stage: the epilogue of hidden layer Y, tile by tile, interleaved with the next affine
// layer's MFMAs (MO output tiles, fragments wf [MO][ksa][64], ksn K-steps) into Z: the VALU work
// of tile mt + 1 sits in the same basic block as the MFMAs of tile mt.
template <int NCOL, int MT, int MO>
__device__ __forceinline__ float stage(const f32x4 (&Y)[MT][NCOL], const float (&epsv)[MT][4],
                                       int tiles, int r_last, int g, const EpiConst& ek,
                                       const float* __restrict__ wf, int ksa, int ksn,
                                       f32x4 (&Z)[MO][NCOL]) {
#pragma unroll
    for (int mo = 0; mo < MO; ++mo)
#pragma unroll
        for (int c = 0; c < NCOL; ++c) Z[mo][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 Xc[NCOL];
    float en = tile_epilogue<NCOL, MT>(Y, epsv, 0, tiles, r_last, g, ek, Xc);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        f32x4 Xn[NCOL];
        const int nst = ksn - 4 * mt;
        if (nst >= 4) {
            mfma_steps<NCOL, MO>(Z, Xc, wf, ksa, 4 * mt, 4);
            if (mt + 1 < MT) en = fmaxf(en, tile_epilogue<NCOL, MT>(Y, epsv, mt + 1, tiles, r_last, g, ek, Xn));
        } else {
            mfma_steps<NCOL, MO>(Z, Xc, wf, ksa, 4 * mt, nst);
            if (mt + 1 < MT) en = fmaxf(en, tile_epilogue<NCOL, MT>(Y, epsv, mt + 1, tiles, r_last, g, ek, Xn));
        }
        if (mt + 1 < MT) {
#pragma unroll
            for (int c = 0; c < NCOL; ++c) Xc[c] = Xn[c];
        }
    }
    en = fmaxf(en, __shfl_xor(en, 16));
    return fmaxf(en, __shfl_xor(en, 32));
}

template <int NCOL, int MT>
__global__ __launch_bounds__(256) void bound_reg_kernel(
    NetDev net, PropDev prop, int64_t n, const float* __restrict__ blo,
    const float* __restrict__ bhi, float* __restrict__ g_lo, float* __restrict__ g_hi,
    int8_t* __restrict__ cls, int raw, unsigned* __restrict__ amb_list,
    unsigned* __restrict__ amb_count, unsigned list_base) {
    constexpr int D = NCOL - 3;
    constexpr int KS = 4 * MT;
    extern __shared__ __attribute__((aligned(16))) float lds[];   // 16-byte aligned after any static LDS
    const int nmid = net.n_affine - 2;
    const int d = net.d;
    // [mid fragments nmid][MT][KS][64] | output fragments [KS][64] | bias, |W| row sums
    // [nmid][2][16 MT] | first layer [16 MT][d] + [16 MT] | per-wave output tile
    float* frag = lds;
    float* ofr = frag + nmid * MT * KS * 64;
    float* aux = ofr + KS * 64;
    float* w1s = aux + nmid * 32 * MT;
    float* b1s = w1s + 16 * MT * d;
    float* obuf_all = b1s + 16 * MT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;

    for (int l = 0; l < nmid; ++l) {
        const MidLayer* L = &net.mid[l];
        for (int i = tid; i < MT * KS * 64; i += 256) {
            const int mo = i / (KS * 64), st = (i / 64) % KS, ln = i % 64;
            frag[l * MT * KS * 64 + i] = (mo < L->mt_out && st < L->ks_alloc)
                                             ? L->wfrag[(mo * L->ks_alloc + st) * 64 + ln] : 0.f;
        }
        for (int i = tid; i < 16 * MT; i += 256) {
            const bool in = i < 16 * L->mt_out;
            aux[(l * 2 + 0) * 16 * MT + i] = in ? L->bias[i] : 0.f;
            aux[(l * 2 + 1) * 16 * MT + i] = in ? L->absrow[i] : 0.f;
        }
    }
    for (int i = tid; i < KS * 64; i += 256)
        ofr[i] = (i / 64) < prop.ks_out_alloc ? prop.wgfrag[i] : 0.f;
    for (int i = tid; i < 16 * MT * d; i += 256) w1s[i] = i < 16 * net.mt1 * d ? net.w1p[i] : 0.f;
    for (int i = tid; i < 16 * MT; i += 256) b1s[i] = i < 16 * net.mt1 ? net.b1p[i] : 0.f;
    __syncthreads();
    float* obuf = obuf_all + wave * (NCOL * 256);   // [column][row 16][box 16]
    const EpiConst ek = epi_const(net, raw);
    const float eta = raw ? 0.f : kEta;

    const int64_t tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t b = tile * 16 + j;
        const bool bval = b < n;
        f32x4 Y[MT][NCOL];
        float epsv[MT][4];
        // ---- first affine layer (exact, VALU): pre-activations of hidden layer 0
        {
            float mid[D], rad[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                float l = 0.f, h = 0.f;
                if (bval && k < d) {
                    l = blo[b * d + k];
                    h = bhi[b * d + k];
                }
                const float m = 0.5f * (l + h);
                mid[k] = m;
                rad[k] = raw ? 0.5f * (h - l) : fmaxf(h - m, m - l) * (1.f + 0x1p-22f);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 16 * mt + 4 * g + v;
                    const float bb = b1s[m];
                    float c0 = bb, sm = fabsf(bb);
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const float w = k < d ? w1s[m * d + k] : 0.f;
                        c0 = fmaf(w, mid[k], c0);
                        Y[mt][k + 1][v] = w * rad[k];
                        sm += fabsf(w) * (fabsf(mid[k]) + rad[k]);
                    }
                    Y[mt][0][v] = c0;
                    Y[mt][NCOL - 2][v] = 0.f;
                    Y[mt][NCOL - 1][v] = 0.f;
                    epsv[mt][v] = raw ? 0.f : net.kfirst * sm + eta;
                }
            }
        }
        int tiles_l = net.mt1, r_l = net.r1;
        float emax = 0.f;
        // ---- hidden-to-hidden layers
        for (int l = 0; l < nmid; ++l) {
            const MidLayer* L = &net.mid[l];
            f32x4 Z[MT][NCOL];
            emax = stage<NCOL, MT, MT>(Y, epsv, tiles_l, r_l, g, ek, frag + l * MT * KS * 64 + lane,
                                       KS, L->ks, Z);
            const float* bias = aux + (l * 2 + 0) * 16 * MT;
            const float* absr = aux + (l * 2 + 1) * 16 * MT;
#pragma unroll
            for (int mo = 0; mo < MT; ++mo)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 16 * mo + 4 * g + v;
                    const float bb = bias[m];
#pragma unroll
                    for (int c = 0; c < NCOL; ++c) Y[mo][c][v] = Z[mo][c][v];
                    Y[mo][0][v] += bb;
                    epsv[mo][v] = raw ? 0.f : L->kgam * (absr[m] * emax + fabsf(bb)) + eta;
                }
            tiles_l = L->mt_out;
            r_l = L->r_out;
        }
        // ---- last hidden layer's epilogue interleaved with the output-row MFMAs
        f32x4 G[1][NCOL];
        emax = stage<NCOL, MT, 1>(Y, epsv, tiles_l, r_l, g, ek, ofr + lane, KS, prop.ks_out, G);
        wave_sync();   // the previous tile's reads of obuf are done
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) obuf[(c * 16 + 4 * g + v) * 16 + j] = G[0][c][v];
        wave_sync();
        if (g == 0 && bval) {
            const int rows = prop.rows;
            bool unsafe = true, safe = false, amb_unsafe = true, amb_safe = false;
            for (int r = 0; r < rows; ++r) {
                const float bg = prop.bg[r];
                const float G0 = obuf[(0 * 16 + r) * 16 + j] + bg;
                float Sg = 0.f;
#pragma unroll
                for (int c = 1; c <= D; ++c) Sg += fabsf(obuf[(c * 16 + r) * 16 + j]);
                const float eps = raw ? 0.f : prop.kout * (prop.ag[r] * emax + fabsf(bg)) + kEta;
                const float Rg = obuf[((NCOL - 2) * 16 + r) * 16 + j] + eps;
                const float delta = raw ? 0.f : net.kconc * (fabsf(G0) + Rg + Sg);
                const float glo = (G0 - (Rg + Sg)) - delta;
                const float ghi = (G0 + (Rg + Sg)) + delta;
                const float tau = 2.f * (obuf[((NCOL - 1) * 16 + r) * 16 + j] + eps + delta) +
                                  0x1p-14f * fmaxf(fabsf(glo), fabsf(ghi));
                if (g_lo) g_lo[b * rows + r] = glo;
                if (g_hi) g_hi[b * rows + r] = ghi;
                unsafe = unsafe && (glo > 0.f);
                safe = safe || (ghi <= 0.f);
                amb_unsafe = amb_unsafe && (glo + tau > 0.f);
                amb_safe = amb_safe || (ghi - tau <= 0.f);
            }
            int8_t kc = unsafe ? 1 : (safe ? 2 : 0);
            if (kc == 0 && !raw && (amb_unsafe || amb_safe)) {
                kc = 3;
                if (amb_list) amb_list[atomicAdd(amb_count, 1u)] = list_base + (unsigned)b;
            }
            if (cls) cls[b] = kc;
        }
    }
}

// Concrete float32 forward pass of sample points (used to place the approximate count's splits).
__global__ __launch_bounds__(256) void sample_forward_kernel(NetDev net, PropDev prop, int64_t n,
                                                             const float* __restrict__ x,
                                                             int8_t* __restrict__ viol) {
    __shared__ float h0[SLR_MAX_WIDTH], h1[SLR_MAX_WIDTH];
    __shared__ int ok;
    const int tid = threadIdx.x;
    const int d = net.d;
    for (int64_t p = blockIdx.x; p < n; p += gridDim.x) {
        if (tid < d) h1[tid] = x[p * d + tid];
        if (tid == 0) ok = 1;
        __syncthreads();
        if (tid < net.n1) {
            float s = net.b1[tid];
            for (int k = 0; k < d; ++k) s = fmaf(net.w1[tid * d + k], h1[k], s);
            h0[tid] = net.act == SLR_ACT_RELU ? fmaxf(s, 0.f) : act_eval(net.act, s);
        }
        __syncthreads();
        float* in = h0;
        float* out = h1;
        for (int l = 0; l < net.n_affine - 2; ++l) {
            const MidLayer* L = &net.mid[l];
            if (tid < L->n_out) {
                float s = L->b[tid];
                const float* wr = L->w + (size_t)tid * L->n_in;
                for (int k = 0; k < L->n_in; ++k) s = fmaf(wr[k], in[k], s);
                out[tid] = net.act == SLR_ACT_RELU ? fmaxf(s, 0.f) : act_eval(net.act, s);
            }
            __syncthreads();
            float* t = in;
            in = out;
            out = t;
        }
        if (tid < prop.rows) {
            float s = prop.bg[tid];
            for (int k = 0; k < prop.n_last; ++k) s = fmaf(prop.wg[tid * prop.n_last + k], in[k], s);
            if (!(s > 0.f)) atomicAnd(&ok, 0);
        }
        __syncthreads();
        if (tid == 0) viol[p] = (int8_t)ok;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Bound-kernel shape classes: NCOL (state columns) and (NT boxes/16, UW units per wave).
// ---------------------------------------------------------------------------------------------
// Dynamic LDS above the default 64 KiB must be allowed per kernel (gfx950 has 160 KiB per
// workgroup, static LDS included).  A failed request is cleared so it cannot leak into later
// error checks.
hipError_t allow_lds(const void* kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

int ncol_class(int d) {
    const int c = d + 3;
    if (c <= 12) return c;
    if (c <= 14) return 14;
    if (c <= 18) return 18;
    if (c <= 26) return 26;
    return 35;
}


template <int NCOL, int NT, int UW, int NW, bool SMOOTH = false, bool SCORE = false>
hipError_t launch_inst(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                       const float* hi, float* g_lo, float* g_hi, int8_t* cls, int raw,
                       hipStream_t stream, unsigned* amb_list, unsigned* amb_count,
                       unsigned list_base, int8_t* dimsel = nullptr, int split_layers = 0) {
    const size_t lds = bound_lds_bytes(NCOL, TileShape{NT, UW, NW}, net.mt_max, prop.rows);
    auto kern = bound_f32_kernel<NCOL, NT, UW, NW, SMOOTH, SCORE>;
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = (n + NT * 16 - 1) / (NT * 16);
    (void)hipGetLastError();
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), lds, stream, net, prop, n,
                       lo, hi, g_lo, g_hi, cls, raw, state_stride(net.mt_max), amb_list,
                       amb_count, list_base, dimsel, split_layers);
    return hipGetLastError();
}

// Tile shapes instantiated for the LDS-staged kernel: (NT, UW, NW).
template <int NCOL>
hipError_t launch_ncol(TileShape t, const NetDev& net, const PropDev& prop, int64_t n,
                       const float* lo, const float* hi, float* g_lo, float* g_hi, int8_t* cls,
                       int raw, hipStream_t stream, unsigned* al, unsigned* ac, unsigned lb,
                       int8_t* dimsel, int split_layers) {
    if (dimsel && split_layers > 0) {   // crossing-score split: ReLU, the default shapes only
        if constexpr (NCOL <= 14) {
#define SLR_SCORE(A, B, C)                                                                       \
            if (t.nt == A && t.uw == B && t.nw == C)                                              \
                return launch_inst<NCOL, A, B, C, false, true>(net, prop, n, lo, hi, g_lo, g_hi, \
                                                               cls, raw, stream, al, ac, lb,     \
                                                               dimsel, split_layers);
            SLR_SCORE(4, 1, 4) SLR_SCORE(2, 1, 4) SLR_SCORE(1, 1, 4) SLR_SCORE(1, 2, 4)
#undef SLR_SCORE
        }
        return hipErrorInvalidValue;
    }
    if (net.act != SLR_ACT_RELU) {   // smooth networks: the default shapes only
#define SLR_SMOOTH(A, B, C)                                                                      \
        if (t.nt == A && t.uw == B && t.nw == C)                                                  \
            return launch_inst<NCOL, A, B, C, true>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw,   \
                                                    stream, al, ac, lb);
        SLR_SMOOTH(4, 1, 4) SLR_SMOOTH(2, 1, 4) SLR_SMOOTH(1, 1, 4) SLR_SMOOTH(1, 2, 4)
        if constexpr (NCOL <= 18) {
            SLR_SMOOTH(1, 4, 4)
        }
#undef SLR_SMOOTH
        return hipErrorInvalidValue;
    }
#define SLR_SHAPE(A, B, C)                                                                       \
    if (t.nt == A && t.uw == B && t.nw == C)                                                      \
        return launch_inst<NCOL, A, B, C>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, al, \
                                          ac, lb);
    SLR_SHAPE(4, 1, 4) SLR_SHAPE(2, 1, 4) SLR_SHAPE(1, 1, 4) SLR_SHAPE(1, 2, 4)
    // eight wavefronts leave 256 registers per lane: only the shapes that do not spill
    if constexpr (NCOL <= 26) {
        SLR_SHAPE(1, 1, 8)
    }
    if constexpr (NCOL <= 18) {
        SLR_SHAPE(1, 4, 4)
    }
    if constexpr (NCOL <= 14) {
        SLR_SHAPE(1, 2, 8)
    }
#undef SLR_SHAPE
    return hipErrorInvalidValue;
}

// Compute units of the device current at the first call (a function-local static: its
// initialization is thread-safe, so concurrent callers see one value).
int num_cu() {
    static const int cu_count = [] {
        int dev = 0, cu = 0;
        const bool ok = hipGetDevice(&dev) == hipSuccess &&
                        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                        cu > 0;
        (void)hipGetLastError();
        return ok ? cu : 256;
    }();
    return cu_count;
}

size_t reg_lds_bytes(const NetDev& net, const PropDev& prop, int ncol) {
    (void)prop;
    const size_t mt = net.mt_max, ks = 4 * mt, nmid = net.n_affine - 2;
    return sizeof(float) * (nmid * mt * ks * 64 + ks * 64 + nmid * 32 * mt + 16 * mt * net.d +
                            16 * mt + 4 * (size_t)ncol * 256);
}

template <int NCOL, int MT>
hipError_t launch_reg(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                      const float* hi, float* g_lo, float* g_hi, int8_t* cls, int raw,
                      hipStream_t stream, unsigned* al, unsigned* ac, unsigned lb) {
    const int64_t waves_needed = (n + 15) / 16;
    int64_t blocks = (waves_needed + 3) / 4;
    const size_t lds = reg_lds_bytes(net, prop, NCOL);
    auto kern = bound_reg_kernel<NCOL, MT>;
    hipError_t e = allow_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as can be resident at once
    static std::atomic<int> per_cu{0};
    int pc = per_cu.load(std::memory_order_relaxed);
    if (pc == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)kern, 256, lds) != hipSuccess || nb < 1)
            nb = 1;
        (void)hipGetLastError();
        pc = nb;
        per_cu.store(pc, std::memory_order_relaxed);
    }
    const int64_t cap = (int64_t)num_cu() * pc;
    if (blocks > cap) blocks = cap;
    (void)hipGetLastError();
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, stream, net, prop, n, lo, hi,
                       g_lo, g_hi, cls, raw, al, ac, lb);
    return hipGetLastError();
}

template <int NCOL>
hipError_t launch_reg_mt(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                         const float* hi, float* g_lo, float* g_hi, int8_t* cls, int raw,
                         hipStream_t stream, unsigned* al, unsigned* ac, unsigned lb) {
    switch (net.mt_max) {
        case 1: return launch_reg<NCOL, 1>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, al, ac, lb);
        case 2: return launch_reg<NCOL, 2>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, al, ac, lb);
        case 3: return launch_reg<NCOL, 3>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, al, ac, lb);
        case 4: return launch_reg<NCOL, 4>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, al, ac, lb);
        default: return hipErrorInvalidValue;
    }
}

int g_variant = 0;   // 0 auto, 1 LDS-staged, 2 register-resident, 3 tape-state only

bool reg_fits(const NetDev& net, const PropDev& prop) {
    return net.mt_max <= 4 && net.d + 3 <= 10 && prop.rows <= 16 &&
           reg_lds_bytes(net, prop, net.d + 3) <= 160 * 1024;
}

// Top of the search tree in one pass: every box of the complete subtree of depth K
// (`prefix_box`), and after bounding, the replay to the boxes the level loop visits
// (`prefix_replay_block`).
__global__ __launch_bounds__(256) void prefix_boxes_kernel(int64_t N, int d, RootBox rb,
                                                           float* __restrict__ lo,
                                                           float* __restrict__ hi,
                                                           unsigned long long* __restrict__ path,
                                                           unsigned* err) {
    extern __shared__ float prefix_stage[];   // 2 * 256 * d floats
    prefix_block(N, (int64_t)blockIdx.x * 256, d, rb.lo, rb.hi, lo, hi, path, err, 1, prefix_stage);
}

__global__ __launch_bounds__(256) void prefix_replay_kernel(int64_t N, int K, int8_t* cls,
                                                            LevelStats* stats) {
    prefix_replay_block(N, K, cls, stats, (int64_t)blockIdx.x * 256);
}

// The FP64 re-decisions of the top's boxes that the level loop does not visit (class 4 after
// the replay) are not the loop's: each such listed box takes one off the re-decision counter.
__global__ __launch_bounds__(256) void prefix_recheck_uncount_kernel(const unsigned* __restrict__ list,
                                                                     const unsigned* __restrict__ count,
                                                                     const int8_t* __restrict__ cls,
                                                                     unsigned long long* counter) {
    const unsigned n = *count;
    for (unsigned k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256)
        if (cls[list[k]] == 4) atomicAdd(counter, ~0ull);   // minus one
}

}  // namespace

int set_bound_variant(int v) {
    if (v < 0 || v > 3) return -1;
    g_variant = v;
    return 0;
}

int bound_variant_for(const NetDev& net, const PropDev& prop) {
    if (g_variant == 2) return reg_fits(net, prop) && net.act == SLR_ACT_RELU ? 2 : -1;
    if (g_variant == 3) return -1;   // the level driver then bounds with the tape-state kernel
    return 1;
}


namespace {

TileShape g_shape_override[64][17];   // [ncol class][mt_max]: nt = 0 -> default

TileShape default_shape(int mt_max) {
    if (mt_max <= 1) return {4, 1, 4};
    if (mt_max == 2) return {2, 1, 4};
    if (mt_max <= 4) return {1, 1, 4};
    if (mt_max <= 8) return {1, 2, 4};
    return {1, 4, 4};
}

}  // namespace

int ncol_class_of(int d) { return ncol_class(d); }

// Floats per lane row of the LDS state: one 16-byte slot per input tile (quad of K-steps); the
// slots are XOR-swizzled per lane (quad_swizzle) instead of padded against bank conflicts.
int state_stride(int mt_max) { return 4 * mt_max; }

size_t bound_lds_bytes(int NCOL, TileShape t, int mt_max, int rows) {
    const int T = t.nt * 16;
    const int SP = state_stride(mt_max);
    return sizeof(float) * ((size_t)t.nt * NCOL * 64 * SP + 2 * (size_t)mt_max * T +
                            (size_t)t.nw * rows * T * NCOL);
}

bool tile_shape_valid(int ncol, int mt_max, TileShape t) {
    const bool inst = (t.nt == 4 && t.uw == 1 && t.nw == 4) || (t.nt == 2 && t.uw == 1 && t.nw == 4) ||
                      (t.nt == 1 && t.uw == 1 && t.nw == 4) || (t.nt == 1 && t.uw == 2 && t.nw == 4) ||
                      (ncol <= 26 && t.nt == 1 && t.uw == 1 && t.nw == 8) ||
                      (ncol <= 18 && t.nt == 1 && t.uw == 4 && t.nw == 4) ||
                      (ncol <= 14 && t.nt == 1 && t.uw == 2 && t.nw == 8);
    return inst && mt_max >= 1 && mt_max * t.nt <= t.uw * t.nw;
}

TileShape tile_shape_for(int d, int mt_max) {
    const int c = ncol_class(d);
    if (c < 64 && mt_max <= 16 && g_shape_override[c][mt_max].nt > 0) return g_shape_override[c][mt_max];
    return default_shape(mt_max);
}

int set_tile_shape(int d, int mt_max, TileShape t) {
    const int c = ncol_class(d);
    if (d < 1 || d > SLR_MAX_D || mt_max < 1 || mt_max > 16) return -1;
    if (t.nt == 0) {
        g_shape_override[c][mt_max] = TileShape{0, 0, 0};
        return 0;
    }
    if (!tile_shape_valid(c, mt_max, t)) return -1;
    g_shape_override[c][mt_max] = t;
    return 0;
}

int bound_f32_supported(const NetDev& net, const PropDev& prop) {
    const int v = bound_variant_for(net, prop);
    if (v == 2) return 1;
    if (v < 0) return 0;
    const int NCOL = ncol_class(net.d);
    const TileShape t = tile_shape_for(net.d, net.mt_max);
    if (!tile_shape_valid(NCOL, net.mt_max, t)) return 0;
    if (bound_lds_bytes(NCOL, t, net.mt_max, prop.rows) > 160 * 1024) return 0;
    return 1;
}

hipError_t launch_bound_f32(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                            const float* hi, float* g_lo, float* g_hi, int8_t* cls, int raw,
                            hipStream_t stream, int* unsupported, unsigned* amb_list,
                            unsigned* amb_count, unsigned list_base, int8_t* dimsel,
                            int split_layers) {
    *unsupported = 0;
    if (n <= 0) return hipSuccess;
    if (!bound_f32_supported(net, prop)) {
        *unsupported = 1;
        return hipSuccess;
    }
    if (bound_variant_for(net, prop) == 2 && !(dimsel && split_layers > 0)) {
        switch (net.d + 3) {
#define SLR_RCASE(C) \
    case C: return launch_reg_mt<C>(net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, amb_list, \
                                    amb_count, list_base);
            SLR_RCASE(4) SLR_RCASE(5) SLR_RCASE(6) SLR_RCASE(7) SLR_RCASE(8) SLR_RCASE(9) SLR_RCASE(10)
#undef SLR_RCASE
            default: break;
        }
    }
    const bool scored = dimsel && split_layers > 0;
    if (scored && (net.act != SLR_ACT_RELU || ncol_class(net.d) > 14)) {
        *unsupported = 1;
        return hipSuccess;
    }
    const TileShape t = net.act == SLR_ACT_RELU && !scored ? tile_shape_for(net.d, net.mt_max)
                                                           : default_shape(net.mt_max);
    switch (ncol_class(net.d)) {
#define SLR_CASE(C) \
    case C: return launch_ncol<C>(t, net, prop, n, lo, hi, g_lo, g_hi, cls, raw, stream, \
                                  amb_list, amb_count, list_base, dimsel, split_layers);
        SLR_CASE(4) SLR_CASE(5) SLR_CASE(6) SLR_CASE(7) SLR_CASE(8) SLR_CASE(9)
        SLR_CASE(10) SLR_CASE(11) SLR_CASE(12) SLR_CASE(14) SLR_CASE(18) SLR_CASE(26) SLR_CASE(35)
#undef SLR_CASE
        default: *unsupported = 1; return hipSuccess;
    }
}

hipError_t launch_recheck64(const NetDev& net, const PropDev& prop, int64_t n, const float* lo,
                            const float* hi, float* g_lo, float* g_hi, int8_t* cls,
                            unsigned long long* counter, const unsigned* list,
                            const unsigned* list_count, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int ncol = net.d + 2;
    const int nrow = net.n_max > prop.rows * ncol ? net.n_max : prop.rows * ncol;
    const size_t per_wave = sizeof(double) * (2 * (size_t)nrow * ncol + 2 * SLR_MAX_D);
    int waves = 4;
    while (waves > 1 && per_wave * waves > 150 * 1024) --waves;
    const size_t lds = per_wave * waves;
    hipError_t e = allow_lds((const void*)recheck64_kernel, lds);
    if (e != hipSuccess) return e;
    int64_t blocks = list ? 2048 : (n + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    (void)hipGetLastError();
    hipLaunchKernelGGL(recheck64_kernel, dim3((unsigned)blocks), dim3(64 * waves), lds, stream, net,
                       prop, n, lo, hi, g_lo, g_hi, cls, counter, list, list_count, nrow);
    return hipGetLastError();
}

size_t level_tiles(int64_t n) { return (size_t)((n + kTile - 1) / kTile); }

hipError_t launch_level_count(int64_t n, const int8_t* cls, unsigned* tile_und, LevelStats* stats,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(level_count_kernel, dim3((unsigned)level_tiles(n)), dim3(256), 0, stream, n,
                       cls, tile_und, stats);
    return hipGetLastError();
}

hipError_t launch_prefix_boxes(int64_t N, int d, const RootBox& rb, float* lo, float* hi,
                               unsigned long long* path, unsigned* err, hipStream_t stream) {
    if (N <= 0) return hipSuccess;
    (void)hipGetLastError();
    if (d < 1 || d > SLR_MAX_D) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prefix_boxes_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256),
                       sizeof(float) * 2 * 256 * d, stream, N, d, rb, lo, hi, path, err);
    return hipGetLastError();
}

hipError_t launch_prefix_replay(int64_t N, int K, int8_t* cls, LevelStats* stats, hipStream_t stream) {
    if (N <= 0 || K < 0 || K > 15) return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL(prefix_replay_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream,
                       N, K, cls, stats);
    return hipGetLastError();
}

hipError_t launch_prefix_recheck_uncount(int64_t N, const unsigned* list, const unsigned* count,
                                         const int8_t* cls, unsigned long long* counter,
                                         hipStream_t stream) {
    if (N <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(prefix_recheck_uncount_kernel, dim3((unsigned)((N + 255) / 256 < 64 ? (N + 255) / 256 : 64)),
                       dim3(256), 0, stream, list, count, cls, counter);
    return hipGetLastError();
}

hipError_t launch_split(int64_t n, int d, const int8_t* cls, const unsigned* tile_und,
                        const float* lo, const float* hi, const unsigned long long* path,
                        float* lo2, float* hi2, unsigned long long* path2, unsigned* err,
                        int64_t cap, hipStream_t stream, const int8_t* dimsel) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    const size_t lds = d <= kSplitStageD ? 2 * sizeof(float) * kTile * d : 0;
    hipLaunchKernelGGL(split_kernel, dim3((unsigned)level_tiles(n)), dim3(256), lds, stream, n, d,
                       cls, tile_und, lo, hi, path, lo2, hi2, path2, err, cap, dimsel);
    return hipGetLastError();
}

hipError_t launch_stack_count(int64_t n, int8_t* cls, const unsigned long long* path, int max_depth,
                              int all_undecided, unsigned* tile_und, LevelStats* stats,
                              unsigned* split_total, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(stack_count_kernel, dim3((unsigned)level_tiles(n)), dim3(256), 0, stream, n,
                       cls, path, max_depth, all_undecided, tile_und, stats, split_total);
    return hipGetLastError();
}

hipError_t launch_stack_volume(const LevelStats* stats, int levels, double* out3,
                               unsigned long long* out_counts, unsigned* err, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(stack_volume_kernel, dim3(1), dim3(64), 0, stream, stats, levels, out3,
                       out_counts, err);
    return hipGetLastError();
}

hipError_t launch_volume(const LevelStats* stats, int levels, int stop_level, int stopped,
                         double* out3, unsigned long long* out_counts, unsigned* err,
                         hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(volume_kernel, dim3(1), dim3(64), 0, stream, stats, levels, stop_level,
                       stopped, out3, out_counts, err);
    return hipGetLastError();
}

hipError_t launch_sample_forward(const NetDev& net, const PropDev& prop, int64_t n, const float* x,
                                 int8_t* viol, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = n < 4096 ? n : 4096;
    (void)hipGetLastError();
    hipLaunchKernelGGL(sample_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, net,
                       prop, n, x, viol);
    return hipGetLastError();
}
