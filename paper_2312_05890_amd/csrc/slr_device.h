// Device code shared by the single-instance kernels (slr_kernels.hip) and the batch kernels
// (slr_batch.hip): the LDS-staged bound tile, the FP64 re-decision of one box and the level
// bookkeeping of one 1024-box tile.  Header-only; every translation unit gets its own copy.
//
// Bound tile (one branch-and-bound level at a time, §3): a workgroup of four wavefronts takes
// 16*NT boxes.  For box b and neuron m the state is the center equation c_0..c_d, the radius r
// (see slr_internal.h) and q, the part of r that comes from rounding margins (it decides which
// boxes need the FP64 re-decision), NCOL = d + 3 floats, kept in LDS in the layout
//     S[nt][c][g][j][s]     (j = box within the 16-box N tile, (g, s) = neuron)
// where neuron k of the layer input sits at g = (k % 16) / 4, s = 4 (k / 16) + k % 4.  That is
// exactly the B-operand layout of v_mfma_f32_16x16x4f32 (lane 16 g + j supplies B[g][j] of
// K-step s) and also exactly where the same lane finds output rows 16 mt + 4 g + v of the
// accumulator D[4 g + v][j] of M tile mt.  So every hidden layer is
//     MFMA:      acc[c] += W_frag(mt, s) * S[c][s]        (c <= d, A = W)
//                acc[c] += |W_frag(mt, s)| * S[c][s]       (r column, A = |W|)
//                acc[q] += bf16(|W|) * bf16(S[q])          (q column: one bf16 16x16x16 MFMA
//                                                           per four K-steps, both operands
//                                                           rounded up, so q stays an upper bound)
//     epilogue:  lane-local on its 4 neurons x NCOL columns: bias, rounding margin,
//                concretization, Eq. 1, then one 16-byte LDS store per column.
// The first affine layer (box -> hidden) is exact and done on the VALU; the output layer with
// the folded property rows runs as split-K MFMA over the four wavefronts when it fits one tile,
// else as a VALU contraction over the LDS state.

#pragma once

#include "slr_internal.h"

#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kU32 = 0x1p-24f;     // unit roundoff of float32
constexpr float kEta = 0x1p-96f;     // absolute floor: covers flushed subnormal products
constexpr double kEta64 = 0x1p-960;
constexpr double kU64 = 0x1p-53;
constexpr int kNW = 4;               // wavefronts per workgroup of the default bound tile

// Row 16 mt + 4 g + v of a layer with `tiles` 16-row tiles whose last tile holds r neurons.
__device__ __forceinline__ bool row_valid(int mt, int g, int v, int tiles, int r) {
    return mt < tiles - 1 || 4 * v + g < r;
}

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// Four non-negative floats as bf16 rounded up (never below the input).
__device__ __forceinline__ bf16x4 bf16_up4(f32x4 x) {
    bf16x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = (short)((__float_as_uint(x[i]) + 0xFFFFu) >> 16);
    return r;
}

// One 16x16x16 bf16 MFMA: the four K-steps of a quad at once.  Lane 16 g + j supplies A[j][4 g + i]
// and B[4 g + i][j] (i = 0..3), which are exactly the K-steps 4 q + i of the float32 layout, and
// accumulates into the same D layout.
__device__ __forceinline__ f32x4 mfma_bf16_quad(uint64_t a, f32x4 b, f32x4 c) {
    bf16x4 av;
    __builtin_memcpy(&av, &a, 8);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bf16_up4(b), c, 0, 0, 0);
}

// Raw buffer loads (bounds-checked against the byte count; loads past it read 0).  Unlike plain
// loads they are not merged across a loop's back edge, so a load issued one iteration ahead
// stays ahead.
typedef __amdgpu_buffer_rsrc_t BufRsrc;

__device__ __forceinline__ BufRsrc buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ float buf_f32(BufRsrc r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Smooth activations (tanh, sigmoid) by two parallel lines: slope lam = the chord's over [l, u]
// (the derivative at l for a point), offsets bl <= min h and bh >= max h of h(z) = s(z) - lam z
// over [l, u].  Both functions are concave for z >= 0 and convex for z <= 0, so the tangent of h
// at any point a of [max(l, 0), u] bounds h from above there and the tangent at any point b of
// [l, min(u, 0)] from below; a and b are the points where s' = lam (clamped into their pieces),
// which makes the tangents flat and the bounds tight, but any a, b keep them valid.  The ends
// l, u complete the candidates.  widen: offsets moved outward by a rounding margin of the few
// float32 evaluations (library tanhf/expf/logf/atanhf within a few ulp).
__device__ __forceinline__ float act_eval(int act, float z) {
    return act == SLR_ACT_TANH ? tanhf(z) : 1.f / (1.f + expf(-z));
}

__device__ __forceinline__ float act_slope(int act, float fz) {
    return act == SLR_ACT_TANH ? 1.f - fz * fz : fz * (1.f - fz);
}

__device__ __forceinline__ void smooth_lines(int act, float l, float u, bool widen, float& lam,
                                             float& bl, float& bh) {
    const float fl = act_eval(act, l), fu = act_eval(act, u);
    const float w = u - l;
    lam = fmaxf(0.f, w > 0.f ? (fu - fl) / w : act_slope(act, fl));
    float zc;
    if (act == SLR_ACT_TANH) {
        const float t = sqrtf(fmaxf(0.f, 1.f - lam));
        zc = atanhf(fminf(t, 1.f - 0x1p-24f));
    } else {
        const float sq = sqrtf(fmaxf(0.f, 1.f - 4.f * lam));
        const float pp = fminf(0.5f * (1.f + sq), 1.f - 0x1p-24f);
        zc = logf(pp / (1.f - pp));
    }
    const float hl = fl - lam * l, hu = fu - lam * u;
    bl = fminf(hl, hu);
    bh = fmaxf(hl, hu);
    if (u > 0.f) {   // concave piece
        const float a0 = fmaxf(l, 0.f);
        const float a = fminf(fmaxf(zc, a0), u);
        const float fa = act_eval(act, a);
        const float ha = fa - lam * a, da = act_slope(act, fa) - lam;
        bh = fmaxf(bh, ha + fmaxf(da * (u - a), da * (a0 - a)));
    }
    if (l < 0.f) {   // convex piece
        const float b0 = fminf(u, 0.f);
        const float b = fmaxf(fminf(-zc, b0), l);
        const float fb = act_eval(act, b);
        const float hb = fb - lam * b, db = act_slope(act, fb) - lam;
        bl = fminf(bl, hb + fminf(db * (l - b), db * (b0 - b)));
    }
    if (widen) {
        const float m = 32.f * kU32 * (1.f + lam * (fabsf(l) + fabsf(u)));
        bl -= m;
        bh += m;
    }
}

// Scalars of the epilogue: zero margins and no rounding-up in the unwidened mode.
struct EpiConst {
    float kconc, krelu, lamfac;
    int act;
};

__device__ __forceinline__ EpiConst epi_const(const NetDev& net, int raw) {
    EpiConst k;
    k.act = net.act;
    k.kconc = raw ? 0.f : net.kconc;
    k.krelu = raw ? 0.f : net.krelu;
    // lam = hi * rcp(hi - lo): v_rcp_f32 is within 1 ulp, the product within 1/2 ulp, so a
    // factor 1 + 2^-20 keeps the computed ratio >= the chord slope (any slope in [chord, 1] is a
    // valid upper line and a valid lower slope)
    k.lamfac = raw ? 1.f : 1.f + 0x1p-20f;
    return k;
}

// Concretization, rounding margin and ReLU relaxation (Eq. 1) of four neurons of one box,
// without branches.  In: a[c][v] = pre-activation center coefficients (c = 0..d, bias included),
// the unwidened radius a[d+1][v] and margin part a[d+2][v]; eps[v] = rounding margin of the
// affine step.  Out: post-activation state in place; returns max_v bound on |value| over the box.
// SCORE (crossing-score split rule): when `score` is set, the local coefficients |c_1..c_D| of
// every crossing neuron are added to sc (per-lane sums for the side to bisect).
template <int NCOL, bool SMOOTH = false, bool SCORE = false>
__device__ __forceinline__ float relu_epilogue(float (&a)[NCOL][4], const float (&eps)[4],
                                               const bool (&valid)[4], const EpiConst& k,
                                               float* sc = nullptr, bool score = false) {
    constexpr int D = NCOL - 3;
    constexpr int R = NCOL - 2, Q = NCOL - 1;
    float emax = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float c0 = a[0][v];
        float S = 0.f;
#pragma unroll
        for (int c = 1; c <= D; ++c) S += fabsf(a[c][v]);
        const float r = a[R][v] + eps[v];
        const float q = a[Q][v] + eps[v];
        const float delta = k.kconc * (fabsf(c0) + r + S);
        const float lo = (c0 - (r + S)) - delta;
        const float hi = (c0 + (r + S)) + delta;
        if constexpr (SMOOTH) {   // tanh or sigmoid network (k.act)
            float lam = 0.f, bl = 0.f, bh = 0.f;
            if (valid[v]) smooth_lines(k.act, lo, hi, k.krelu != 0.f, lam, bl, bh);
            const float er = k.krelu * lam * (fabsf(c0) + S + r);
#pragma unroll
            for (int c = 1; c <= D; ++c) a[c][v] *= lam;
            const float c0n = fmaf(lam, c0, 0.5f * (bl + bh));
            const float rn = fmaf(lam, r, 0.5f * (bh - bl)) + er;
            a[0][v] = c0n;
            a[R][v] = rn;
            a[Q][v] = valid[v] ? fmaf(1.f + lam, q, delta + er) : 0.f;
            emax = fmaxf(emax, fabsf(c0n) + lam * S + rn);
            continue;
        }
        const bool dead = !valid[v] || !(hi > 0.f);
        const bool act = !dead && lo >= 0.f;
        const bool cross = !dead && !act;
        if constexpr (SCORE) {
            if (score && cross) {
#pragma unroll
                for (int c = 1; c <= D; ++c) sc[c - 1] += fabsf(a[c][v]);
            }
        }
        const float den = cross ? hi - lo : 1.f;
        const float lamc = fminf(1.f, hi * __builtin_amdgcn_rcpf(den) * k.lamfac);
        const float lam = dead ? 0.f : (act ? 1.f : lamc);
        const float sh = cross ? -0.5f * lamc * lo : 0.f;
        const float er = cross ? k.krelu * lamc * ((fabsf(c0) + S + r) - lo) : 0.f;
        // dead: lam = sh = er = 0 zeroes every (finite) entry; active: lam = 1, sh = er = 0
#pragma unroll
        for (int c = 1; c <= D; ++c) a[c][v] *= lam;
        const float c0n = fmaf(lam, c0, sh);
        const float rn = fmaf(lam, r, sh) + er;
        const float qf = cross ? 1.f + lamc : lam;
        const float qa = cross ? delta + er : 0.f;
        a[0][v] = c0n;
        a[R][v] = rn;
        a[Q][v] = fmaf(qf, q, qa);
        emax = fmaxf(emax, fabsf(c0n) + lam * S + rn);
    }
    // rounding is monotone, so scaling the maximum equals the maximum of the scaled values
    return emax * (1.f + 4.f * kU32);
}

// XOR swizzle of a lane's 16-byte state slots (quads of K-steps) in the LDS state buffer.  A
// lane's slots are a row of SP = 4 mq floats, so lanes j of one group sharing j mod (16 / m),
// m = gcd(mq, 16), would put the same slot on the same bank group.  XOR-ing the slot index with
// a lane pattern below m (m divides mq, so the index stays below mq) makes the 16-byte slots of
// every 8 consecutive lanes fall on 8 distinct groups of a 32-bank file and those of all 16 lanes
// on 16 distinct groups of a 64-bank one.
__device__ __forceinline__ int quad_swizzle(int mq, int j) {
    const int low = mq & -mq;
    if (low == 1) return 0;
    if (low == 2) return ((j >> 2) ^ (j >> 3)) & 1;
    if (low == 4) return ((j >> 1) ^ (j >> 3)) & 3;
    if (low == 8) return (j ^ (j >> 3)) & 7;
    return j & 15;
}

// The full K-quads of one unit (weights fragments wf/qf from global memory, the layer input's
// state sb from LDS, slot swizzle xs), software-pipelined one quad ahead.  NQ > 0: exactly NQ quads as
// straight-line code (a loop carries the accumulators and the prefetched operands across its back
// edge, where the compiler shuffles accumulator registers and folds the prefetch back into the
// iteration); NQ == 0: a loop over nq quads.
template <int NCOL, int NQ>
__device__ __forceinline__ void k_quads(f32x4 (&acc)[NCOL], const float* __restrict__ wf,
                                        const uint64_t* __restrict__ qf, const float* sb,
                                        int colstride, int nq, int nqa, int xs) {
    float af[4];
    uint64_t aq = qf[0];
    f32x4 bq[NCOL];
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) af[ss] = wf[ss * 64];
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
        bq[c] = *reinterpret_cast<const f32x4*>(sb + c * colstride + 4 * xs);
    auto quad = [&](int qi) {
        const int qn = min(qi + 1, nqa - 1);
        const int nx = qn * 4;
        const float* sn = sb + 4 * (qn ^ xs);
        float an[4];
        const uint64_t aqn = qf[nx * 16];
        f32x4 bn[NCOL];
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) an[ss] = wf[(nx + ss) * 64];
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
            bn[c] = *reinterpret_cast<const f32x4*>(sn + c * colstride);
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            const float aw = af[ss];
            const float aa = fabsf(aw);
#pragma unroll
            for (int c = 0; c < NCOL - 2; ++c) acc[c] = mfma16(aw, bq[c][ss], acc[c]);
            acc[NCOL - 2] = mfma16(aa, bq[NCOL - 2][ss], acc[NCOL - 2]);
        }
        acc[NCOL - 1] = mfma_bf16_quad(aq, bq[NCOL - 1], acc[NCOL - 1]);
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) af[ss] = an[ss];
        aq = aqn;
#pragma unroll
        for (int c = 0; c < NCOL; ++c) bq[c] = bn[c];
    };
    if constexpr (NQ > 0) {
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) quad(qi);
    } else {
        for (int qi = 0; qi < nq; ++qi) quad(qi);
    }
}

// Straight-line quads for nq <= MAXQ (the largest K-quad count a tile shape can meet: its units
// per workgroup bound the layers' tiles), a loop otherwise.
template <int NCOL, int MAXQ>
__device__ __forceinline__ void k_quads_any(f32x4 (&acc)[NCOL], const float* __restrict__ wf,
                                            const uint64_t* __restrict__ qf, const float* sb,
                                            int colstride, int nq, int nqa, int xs) {
    switch (nq) {
        case 1: k_quads<NCOL, 1>(acc, wf, qf, sb, colstride, nq, nqa, xs); return;
        case 2: k_quads<NCOL, 2>(acc, wf, qf, sb, colstride, nq, nqa, xs); return;
        case 3: k_quads<NCOL, 3>(acc, wf, qf, sb, colstride, nq, nqa, xs); return;
        case 4: k_quads<NCOL, 4>(acc, wf, qf, sb, colstride, nq, nqa, xs); return;
        case 5:
            if constexpr (MAXQ >= 5) {
                k_quads<NCOL, 5>(acc, wf, qf, sb, colstride, nq, nqa, xs);
                return;
            }
            break;
        case 6:
            if constexpr (MAXQ >= 6) {
                k_quads<NCOL, 6>(acc, wf, qf, sb, colstride, nq, nqa, xs);
                return;
            }
            break;
        case 7:
            if constexpr (MAXQ >= 7) {
                k_quads<NCOL, 7>(acc, wf, qf, sb, colstride, nq, nqa, xs);
                return;
            }
            break;
        case 8:
            if constexpr (MAXQ >= 8) {
                k_quads<NCOL, 8>(acc, wf, qf, sb, colstride, nq, nqa, xs);
                return;
            }
            break;
        default: break;
    }
    k_quads<NCOL, 0>(acc, wf, qf, sb, colstride, nq, nqa, xs);
}

template <int NCOL, int NT, int UW, int NW, bool SMOOTH = false, bool SCORE = false>
__device__ __forceinline__ void bound_tile(
    const NetDev& net, const PropDev& prop, int64_t n, int64_t box0,
    const float* __restrict__ blo, const float* __restrict__ bhi, float* __restrict__ g_lo,
    float* __restrict__ g_hi, int8_t* __restrict__ cls, int raw, int SP,
    unsigned* __restrict__ amb_list, unsigned* __restrict__ amb_count, unsigned list_base,
    int8_t* __restrict__ dimsel = nullptr, int split_layers = 0) {
    extern __shared__ __attribute__((aligned(16))) float lds[];   // 16-byte aligned after any static LDS
    constexpr int T = NT * 16;
    constexpr int D = NCOL - 3;
    // SCORE: per-lane crossing scores of each unit's box (a unit keeps its 16-box column)
    float scv[UW][D];
    if constexpr (SCORE) {
#pragma unroll
        for (int i = 0; i < UW; ++i)
#pragma unroll
            for (int c = 0; c < D; ++c) scv[i][c] = 0.f;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
    const int d = net.d;
    const int xs = quad_swizzle(SP >> 2, j);          // this lane's slot swizzle

    const EpiConst ek = epi_const(net, raw);
    float* S = lds;                                   // [NT][NCOL][4][16][SP], slots swizzled
    float* part = S + NT * NCOL * 64 * SP;            // [2 parity][mt_max][T] bound on |value|
    float* OUT = part + 2 * net.mt_max * T;           // [rows][T][NCOL]
    const int colstride = 64 * SP;
    auto part_at = [&](int par, int mt, int bj) -> float& {
        return part[(par * net.mt_max + mt) * T + bj];
    };

    // ---------------- first affine layer: exact on the VALU, then the ReLU epilogue
    {
        const int units = net.mt1 * NT;
#pragma unroll
        for (int i = 0; i < UW; ++i) {
            const int u = wave + NW * i;
            if (u < units) {
                const int mt = u / NT, nt = u - (u / NT) * NT;
                const int64_t b = box0 + nt * 16 + j;
                const bool bval = b < n;
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
                float a[NCOL][4], eps[4];
                bool valid[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 16 * mt + 4 * g + v;
                    valid[v] = row_valid(mt, g, v, net.mt1, net.r1);
                    float c0 = 0.f, s = 0.f;
                    if (valid[v]) {
                        const float bb = net.b1p[m];
                        c0 = bb;
                        s = fabsf(bb);
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const float w = k < d ? net.w1p[m * d + k] : 0.f;
                            c0 = fmaf(w, mid[k], c0);
                            a[k + 1][v] = w * rad[k];
                            s += fabsf(w) * (fabsf(mid[k]) + rad[k]);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < D; ++k) a[k + 1][v] = 0.f;
                    }
                    a[0][v] = c0;
                    a[NCOL - 2][v] = 0.f;
                    a[NCOL - 1][v] = 0.f;
                    eps[v] = raw ? 0.f : net.kfirst * s + kEta;
                }
                float emax = relu_epilogue<NCOL, SMOOTH, SCORE>(a, eps, valid, ek, scv[i],
                                                                split_layers >= 1);
                float* sb = S + ((nt * NCOL * 4 + g) * 16 + j) * SP + 4 * (mt ^ xs);
#pragma unroll
                for (int c = 0; c < NCOL; ++c) {
                    f32x4 o = {a[c][0], a[c][1], a[c][2], a[c][3]};
                    *reinterpret_cast<f32x4*>(sb + c * colstride) = o;
                }
                emax = fmaxf(emax, __shfl_xor(emax, 16));
                emax = fmaxf(emax, __shfl_xor(emax, 32));
                if (g == 0) part_at(0, mt, nt * 16 + j) = emax;
            }
        }
    }
    __syncthreads();

    // ---------------- hidden-to-hidden layers on MFMA with fused epilogues
    int rp = 0;
    int mt_prev = net.mt1;
    for (int l = 0; l < net.n_affine - 2; ++l) {
        const MidLayer* L = &net.mid[l];
        const int units = L->mt_out * NT;
        const int ks = L->ks;
        f32x4 res[UW][NCOL];
#pragma unroll
        for (int i = 0; i < UW; ++i) {
            const int u = wave + NW * i;
            if (u < units) {
                const int mt = u / NT, nt = u - (u / NT) * NT;
                f32x4 acc[NCOL];
#pragma unroll
                for (int c = 0; c < NCOL; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                const float* wf = L->wfrag + (size_t)mt * L->ks_alloc * 64 + lane;
                const float* sb = S + ((nt * NCOL * 4 + g) * 16 + j) * SP;
                // full quads of K-steps, software-pipelined one quad ahead (A from global/L2,
                // B from LDS), then the tail quad with per-step guards
                const int nq = ks >> 2;
                const int nqa = L->ks_alloc >> 2;
                const uint64_t* qf = L->qfrag + (size_t)mt * nqa * 64 + lane;
                constexpr int kMaxQ = (UW * NW) / NT >= 8 ? 8 : 4;
                k_quads_any<NCOL, kMaxQ>(acc, wf, qf, sb, colstride, nq, nqa, xs);
                // the last K-steps (ks % 4 of them) one at a time, B read as scalars: a plain
                // loop keeps the accumulators in place (no per-step selects of the whole set);
                // the margin column takes the whole partial quad in one bf16 MFMA (its A is
                // zero beyond ks)
                if (4 * nq < ks)
                    acc[NCOL - 1] = mfma_bf16_quad(
                        qf[nq * 64], *reinterpret_cast<const f32x4*>(sb + (NCOL - 1) * colstride + 4 * (nq ^ xs)),
                        acc[NCOL - 1]);
                for (int st = 4 * nq; st < ks; ++st) {
                    const float aw = wf[st * 64];
                    const float aa = fabsf(aw);
                    float bs[NCOL - 1];
#pragma unroll
                    for (int c = 0; c < NCOL - 1; ++c)
                        bs[c] = sb[c * colstride + 4 * ((st >> 2) ^ xs) + (st & 3)];
#pragma unroll
                    for (int c = 0; c < NCOL - 2; ++c) acc[c] = mfma16(aw, bs[c], acc[c]);
                    acc[NCOL - 2] = mfma16(aa, bs[NCOL - 2], acc[NCOL - 2]);
                }
#pragma unroll
                for (int c = 0; c < NCOL; ++c) res[i][c] = acc[c];
            }
        }
        __syncthreads();   // every wave has read the layer input
#pragma unroll
        for (int i = 0; i < UW; ++i) {
            const int u = wave + NW * i;
            if (u < units) {
                const int mt = u / NT, nt = u - (u / NT) * NT;
                const int bj = nt * 16 + j;
                float emax_in = 0.f;
                for (int q = 0; q < mt_prev; ++q) emax_in = fmaxf(emax_in, part_at(rp, q, bj));
                float a[NCOL][4], eps[4];
                bool valid[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 16 * mt + 4 * g + v;
                    valid[v] = row_valid(mt, g, v, L->mt_out, L->r_out);
                    const float bb = L->bias[m];
                    const float A = L->absrow[m];
#pragma unroll
                    for (int c = 0; c < NCOL; ++c) a[c][v] = res[i][c][v];
                    a[0][v] += bb;
                    eps[v] = raw ? 0.f : L->kgam * (A * emax_in + fabsf(bb)) + kEta;
                }
                float emax = relu_epilogue<NCOL, SMOOTH, SCORE>(a, eps, valid, ek, scv[i],
                                                                l + 2 <= split_layers);
                float* sb = S + ((nt * NCOL * 4 + g) * 16 + j) * SP + 4 * (mt ^ xs);
#pragma unroll
                for (int c = 0; c < NCOL; ++c) {
                    f32x4 o = {a[c][0], a[c][1], a[c][2], a[c][3]};
                    *reinterpret_cast<f32x4*>(sb + c * colstride) = o;
                }
                emax = fmaxf(emax, __shfl_xor(emax, 16));
                emax = fmaxf(emax, __shfl_xor(emax, 32));
                if (g == 0) part_at(rp ^ 1, mt, bj) = emax;
            }
        }
        rp ^= 1;
        mt_prev = L->mt_out;
        __syncthreads();   // the layer output is complete
    }

    // ---------------- output layer: folded property rows
    const int rows = prop.rows;
    const bool mfma_out = rows * NT * NCOL <= 64;
    if (mfma_out) {
        // split-K on MFMA: wave w takes K-quads w, w + 4, ...; partial sums of the valid rows go
        // to OUT as [wave][nt][c][row][box] and are added in the final loop
        const int ksq = (prop.ks_out + 3) >> 2;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            f32x4 G[NCOL];
#pragma unroll
            for (int c = 0; c < NCOL; ++c) G[c] = f32x4{0.f, 0.f, 0.f, 0.f};
            const float* sb = S + ((nt * NCOL * 4 + g) * 16 + j) * SP;
            for (int q = wave; q < ksq; q += NW) {
                f32x4 bq[NCOL];
#pragma unroll
                for (int c = 0; c < NCOL; ++c)
                    bq[c] = *reinterpret_cast<const f32x4*>(sb + c * colstride + 4 * (q ^ xs));
#pragma unroll
                for (int ss = 0; ss < 4; ++ss) {
                    if (4 * q + ss < prop.ks_out) {
                        const float aw = prop.wgfrag[(4 * q + ss) * 64 + lane];
                        const float aa = fabsf(aw);
#pragma unroll
                        for (int c = 0; c < NCOL - 2; ++c) G[c] = mfma16(aw, bq[c][ss], G[c]);
                        G[NCOL - 2] = mfma16(aa, bq[NCOL - 2][ss], G[NCOL - 2]);
                    }
                }
                G[NCOL - 1] = mfma_bf16_quad(prop.wgqfrag[q * 64 + lane], bq[NCOL - 1], G[NCOL - 1]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 4 * g + v;
                if (row < rows) {
#pragma unroll
                    for (int c = 0; c < NCOL; ++c)
                        OUT[(((wave * NT + nt) * NCOL + c) * rows + row) * 16 + j] = G[c][v];
                }
            }
        }
    } else {
        // VALU contraction over the state
        const int K = prop.kpad;
        const int items = rows * T * NCOL;
        for (int it = tid; it < items; it += NW * 64) {
            const int c = it % NCOL;
            const int bj = (it / NCOL) % T;
            const int r = it / (NCOL * T);
            const int nt = bj >> 4, jj = bj & 15;
            const float* wr = prop.wgp + r * K;
            const float* col = S + (nt * NCOL + c) * colstride + jj * SP;
            const int xj = quad_swizzle(SP >> 2, jj);
            float sacc = 0.f;
            for (int k = 0; k < K; ++k) {
                const int gg = (k >> 2) & 3;
                const int sidx = 4 * ((k >> 4) ^ xj) + (k & 3);
                float w = wr[k];
                if (c >= NCOL - 2) w = fabsf(w);
                sacc = fmaf(w, col[gg * 16 * SP + sidx], sacc);
            }
            OUT[(r * T + bj) * NCOL + c] = sacc;
        }
    }
    __syncthreads();
    auto outv = [&](int r, int bj, int c) -> float {
        if (!mfma_out) return OUT[(r * T + bj) * NCOL + c];
        const int nt = bj >> 4, jj = bj & 15;
        float acc = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) acc += OUT[(((w * NT + nt) * NCOL + c) * rows + r) * 16 + jj];
        return acc;
    };
    for (int bj = tid; bj < T; bj += NW * 64) {
        const int64_t b = box0 + bj;
        if (b >= n) continue;
        float emax = 0.f;
        for (int q = 0; q < net.mt_last; ++q) emax = fmaxf(emax, part_at(rp, q, bj));
        bool unsafe = true, safe = false, amb_unsafe = true, amb_safe = false;
        for (int r = 0; r < rows; ++r) {
            const float bg = prop.bg[r];
            const float G0 = outv(r, bj, 0) + bg;
            float Sg = 0.f;
            for (int c = 1; c <= D; ++c) Sg += fabsf(outv(r, bj, c));
            const float eps = raw ? 0.f : prop.kout * (prop.ag[r] * emax + fabsf(bg)) + kEta;
            const float R = outv(r, bj, NCOL - 2) + eps;
            const float delta = raw ? 0.f : net.kconc * (fabsf(G0) + R + Sg);
            const float glo = (G0 - (R + Sg)) - delta;
            const float ghi = (G0 + (R + Sg)) + delta;
            // distance within which the exact-arithmetic decision may differ from this one:
            // twice the propagated margins plus 2^-14 of the row's magnitude
            const float tau = 2.f * (outv(r, bj, NCOL - 1) + eps + delta) +
                              0x1p-14f * fmaxf(fabsf(glo), fabsf(ghi));
            if (g_lo) g_lo[b * rows + r] = glo;
            if (g_hi) g_hi[b * rows + r] = ghi;
            unsafe = unsafe && (glo > 0.f);
            safe = safe || (ghi <= 0.f);
            amb_unsafe = amb_unsafe && (glo + tau > 0.f);
            amb_safe = amb_safe || (ghi - tau <= 0.f);
        }
        int8_t k = unsafe ? 1 : (safe ? 2 : 0);
        if (k == 0 && !raw && (amb_unsafe || amb_safe)) {
            k = 3;
            if (amb_list) amb_list[atomicAdd(amb_count, 1u)] = list_base + (unsigned)b;
        }
        if (cls) cls[b] = k;
    }
    if constexpr (SCORE) {
        // side to bisect: per box, the scores summed in a fixed order (lanes g by xor 16, 32;
        // units in ascending order), then the largest among the sides at least 2^-6 of the
        // widest (lowest index on ties); the widest side when no neuron crossed
        if (dimsel) {
            float* scp = S;   // [NW * UW][16][D]; S is not read after the output contraction
#pragma unroll
            for (int i = 0; i < UW; ++i) {
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    float v = scv[i][c];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    if (g == 0) scp[((wave * UW + i) * 16 + j) * D + c] = v;
                }
            }
            __syncthreads();
            for (int bj = tid; bj < T; bj += NW * 64) {
                const int64_t b = box0 + bj;
                if (b >= n) continue;
                const int nt = bj >> 4, jj = bj & 15;
                float sc[D];
#pragma unroll
                for (int c = 0; c < D; ++c) sc[c] = 0.f;
                for (int u = 0; u < NW * UW; ++u) {
                    if (u % NT != nt) continue;
                    const float* p = scp + (((u % NW) * UW + u / NW) * 16 + jj) * D;
#pragma unroll
                    for (int c = 0; c < D; ++c) sc[c] += p[c];
                }
                int widest = 0, best = -1;
                float wmax = -1.f, sbest = 0.f;
                for (int kk = 0; kk < d; ++kk) {
                    const float w = bhi[b * d + kk] - blo[b * d + kk];
                    if (w > wmax) {
                        wmax = w;
                        widest = kk;
                    }
                }
#pragma unroll
                for (int kk = 0; kk < D; ++kk) {
                    if (kk >= d) break;
                    const float w = bhi[b * d + kk] - blo[b * d + kk];
                    if (w >= wmax * 0x1p-6f && sc[kk] > sbest) {
                        sbest = sc[kk];
                        best = kk;
                    }
                }
                dimsel[b] = (int8_t)(best >= 0 ? best : widest);
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// FP64 re-decision of boxes the float32 pass marked ambiguous (class 3): the same center/radius
// propagation on the VALU in double precision, one box per wavefront, neurons across lanes.
// ------------------------------------------------------------------------------------------

// LDS ordering between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Float64 twin of smooth_lines (always widened, margin 32 u64 per unit of magnitude).
__device__ __forceinline__ double act_eval64(int act, double z) {
    return act == SLR_ACT_TANH ? tanh(z) : 1.0 / (1.0 + exp(-z));
}

__device__ __forceinline__ double act_slope64(int act, double fz) {
    return act == SLR_ACT_TANH ? 1.0 - fz * fz : fz * (1.0 - fz);
}

__device__ __forceinline__ void smooth_lines64(int act, double l, double u, double& lam, double& bl,
                                               double& bh) {
    const double fl = act_eval64(act, l), fu = act_eval64(act, u);
    const double w = u - l;
    lam = fmax(0.0, w > 0.0 ? (fu - fl) / w : act_slope64(act, fl));
    double zc;
    if (act == SLR_ACT_TANH) {
        zc = atanh(fmin(sqrt(fmax(0.0, 1.0 - lam)), 1.0 - 0x1p-53));
    } else {
        const double pp = fmin(0.5 * (1.0 + sqrt(fmax(0.0, 1.0 - 4.0 * lam))), 1.0 - 0x1p-53);
        zc = log(pp / (1.0 - pp));
    }
    const double hl = fl - lam * l, hu = fu - lam * u;
    bl = fmin(hl, hu);
    bh = fmax(hl, hu);
    if (u > 0.0) {
        const double a0 = fmax(l, 0.0);
        const double a = fmin(fmax(zc, a0), u);
        const double fa = act_eval64(act, a);
        const double ha = fa - lam * a, da = act_slope64(act, fa) - lam;
        bh = fmax(bh, ha + fmax(da * (u - a), da * (a0 - a)));
    }
    if (l < 0.0) {
        const double b0 = fmin(u, 0.0);
        const double b = fmax(fmin(-zc, b0), l);
        const double fb = act_eval64(act, b);
        const double hb = fb - lam * b, db = act_slope64(act, fb) - lam;
        bl = fmin(bl, hb + fmin(db * (l - b), db * (b0 - b)));
    }
    const double m = 32.0 * kU64 * (1.0 + lam * (fabs(l) + fabs(u)));
    bl -= m;
    bh += m;
}

__device__ __forceinline__ double relu64(double* st, int ncol, double eps, double kconc,
                                         double krelu, int act = SLR_ACT_RELU) {
    // st: one neuron's row (center c_0..c_d, then the unwidened radius); returns |value| bound
    const int D = ncol - 2;
    double c0 = st[0];
    double S = 0.0;
    for (int c = 1; c <= D; ++c) S += fabs(st[c]);
    double r = st[ncol - 1] + eps;
    const double delta = kconc * (fabs(c0) + r + S);
    const double lo = (c0 - (r + S)) - delta;
    const double hi = (c0 + (r + S)) + delta;
    if (act != SLR_ACT_RELU) {
        double lam, bl, bh;
        smooth_lines64(act, lo, hi, lam, bl, bh);
        const double er = krelu * lam * (fabs(c0) + S + r);
        for (int c = 1; c <= D; ++c) st[c] *= lam;
        c0 = fma(lam, c0, 0.5 * (bl + bh));
        r = fma(lam, r, 0.5 * (bh - bl)) + er;
        st[0] = c0;
        st[ncol - 1] = r;
        return (fabs(c0) + lam * S + r) * (1.0 + 4.0 * kU64);
    }
    if (hi <= 0.0) {
        for (int c = 0; c < ncol; ++c) st[c] = 0.0;
        return 0.0;
    }
    if (lo >= 0.0) {
        st[ncol - 1] = r;
        return fabs(c0) + S + r;
    }
    const double lam = fmin(1.0, (hi / (hi - lo)) * (1.0 + 4.0 * kU64));
    const double sh = -0.5 * lam * lo;
    const double er = krelu * lam * ((fabs(c0) + S + r) - lo);
    for (int c = 1; c <= D; ++c) st[c] *= lam;
    c0 = fma(lam, c0, sh);
    r = fma(lam, r, sh) + er;
    st[0] = c0;
    st[ncol - 1] = r;
    return (fabs(c0) + lam * S + r) * (1.0 + 4.0 * kU64);
}

// NCC consecutive columns of one neuron's pre-activation state (x = the layer input's state
// from the first of those columns, row stride ncol): dot products over the n_in inputs in k
// order.  The weights are column j of the transposed [n_in][n_out] array wt, read 16 K-steps at a
// time through raw buffer loads (reads past the array return 0) into two alternating register
// sets, so the next 16 weights are in flight while these 16 are used.  RAD: the last column is the
// radius, multiplied by |w|; ROW: A_row also sums |w| (in the same k order).
template <int NCC, bool RAD, bool ROW>
__device__ __forceinline__ void recheck_chunk(const float* wt, int j, int n_out, int n_in,
                                              const double* x, int ncol, double* st,
                                              double& A_row) {
    const BufRsrc wr = buf_rsrc(wt, (uint32_t)n_in * (uint32_t)n_out * 4u);
    double acc[NCC];
#pragma unroll
    for (int v = 0; v < NCC; ++v) acc[v] = 0.0;
    auto load = [&](float (&w)[16], int k0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) w[u] = buf_f32(wr, ((uint32_t)(k0 + u) * n_out + j) * 4u);
    };
    auto step = [&](float wf, const double* xr) {
        const double w = wf;
#pragma unroll
        for (int v = 0; v < NCC; ++v) acc[v] = fma(RAD && v == NCC - 1 ? fabs(w) : w, xr[v], acc[v]);
        if (ROW) A_row += fabs(w);
    };
    auto use = [&](const float (&w)[16], int k0) {
        const int kn = n_in - k0;
        if (kn >= 16) {
#pragma unroll
            for (int u = 0; u < 16; ++u) step(w[u], x + (k0 + u) * ncol);
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (u < kn) step(w[u], x + (k0 + u) * ncol);
        }
    };
    float wa[16], wb[16];
    load(wa, 0);
    for (int k0 = 0;;) {
        load(wb, k0 + 16);
        use(wa, k0);
        k0 += 16;
        if (k0 >= n_in) break;
        load(wa, k0 + 16);
        use(wb, k0);
        k0 += 16;
        if (k0 >= n_in) break;
    }
#pragma unroll
    for (int v = 0; v < NCC; ++v) st[v] = acc[v];
}

// One box on one wavefront.  ws: this wave's LDS (2 * nrow * ncol + 2 * 32 doubles).
__device__ __forceinline__ void recheck_box(const NetDev& net, const PropDev& prop, int64_t b,
                                            const float* __restrict__ blo,
                                            const float* __restrict__ bhi,
                                            float* __restrict__ g_lo, float* __restrict__ g_hi,
                                            int8_t* __restrict__ cls, unsigned long long* counter,
                                            double* ws, int nrow) {
    const int lane = threadIdx.x & 63;
    const int d = net.d, ncol = d + 2;
    double* A = ws;
    double* B = A + nrow * ncol;
    double* mid = B + nrow * ncol;
    double* rad = mid + SLR_MAX_D;
    if (lane < d) {
        const double l = blo[b * d + lane], h = bhi[b * d + lane];
        const double m = 0.5 * (l + h);
        mid[lane] = m;
        rad[lane] = fmax(h - m, m - l) * (1.0 + 0x1p-50);
    }
    wave_sync();
    double e = 0.0;
    for (int j = lane; j < net.n1; j += 64) {
        double* st = A + j * ncol;
        const double bb = net.b1[j];
        double c0 = bb, s = fabs(bb);
        for (int k = 0; k < d; ++k) {
            const double w = net.w1[j * d + k];
            c0 = fma(w, mid[k], c0);
            st[k + 1] = w * rad[k];
            s += fabs(w) * (fabs(mid[k]) + rad[k]);
        }
        st[0] = c0;
        st[ncol - 1] = 0.0;
        e = fmax(e, relu64(st, ncol, net.kfirst64 * s + kEta64, net.kconc64, net.krelu64, net.act));
    }
    double emax = wave_max(e);
    wave_sync();
    double* in = A;
    double* out = B;
    for (int l = 0; l < net.n_affine - 2; ++l) {
        const MidLayer* L = &net.mid[l];
        e = 0.0;
        for (int j = lane; j < L->n_out; j += 64) {
            double* st = out + j * ncol;
            double A_row = 0.0;
            // columns in chunks of at most 8 register accumulators; the chunk holding column
            // ncol-1 (the radius) multiplies it by |w|, the first one also sums |w|
            for (int c0 = 0; c0 < ncol; c0 += 8) {
                const double* x = in + c0;
                if (c0 + 8 < ncol) {
                    if (c0 == 0)
                        recheck_chunk<8, false, true>(L->wt, j, L->n_out, L->n_in, x, ncol, st,
                                                      A_row);
                    else
                        recheck_chunk<8, false, false>(L->wt, j, L->n_out, L->n_in, x, ncol,
                                                       st + c0, A_row);
                    continue;
                }
                switch ((ncol - c0) + (c0 == 0 ? 8 : 0)) {
#define SLR_RC(NC, ROW, K) \
    case K:                                                                                     \
        recheck_chunk<NC, true, ROW>(L->wt, j, L->n_out, L->n_in, x, ncol, st + c0, A_row);     \
        break;
                    SLR_RC(1, false, 1) SLR_RC(2, false, 2) SLR_RC(3, false, 3)
                    SLR_RC(4, false, 4) SLR_RC(5, false, 5) SLR_RC(6, false, 6)
                    SLR_RC(7, false, 7) SLR_RC(8, false, 8) SLR_RC(1, true, 9)
                    SLR_RC(2, true, 10) SLR_RC(3, true, 11) SLR_RC(4, true, 12)
                    SLR_RC(5, true, 13) SLR_RC(6, true, 14) SLR_RC(7, true, 15)
                    SLR_RC(8, true, 16)
#undef SLR_RC
                    default: break;
                }
            }
            const double bb = L->b[j];
            st[0] += bb;
            const double eps = L->kgam64 * (A_row * (1.0 + 0x1p-40) * emax + fabs(bb)) + kEta64;
            e = fmax(e, relu64(st, ncol, eps, net.kconc64, net.krelu64, net.act));
        }
        emax = wave_max(e);
        wave_sync();
        double* t = in;
        in = out;
        out = t;
    }
    // output rows: one (row, column) item per lane
    const int rows = prop.rows;
    const int K = prop.n_last;
    for (int it = lane; it < rows * ncol; it += 64) {
        const int r = it / ncol, c = it % ncol;
        double s = 0.0;
        for (int k0 = 0; k0 < K; k0 += 8) {
            double wk[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) wk[u] = prop.wg64[r * K + min(k0 + u, K - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (k0 + u < K) {
                    const double w = c == ncol - 1 ? fabs(wk[u]) : wk[u];
                    s = fma(w, in[(k0 + u) * ncol + c], s);
                }
            }
        }
        out[it] = s;
    }
    wave_sync();
    if (lane == 0) {
        bool unsafe = true, safe = false;
        for (int r = 0; r < rows; ++r) {
            const double* o = out + r * ncol;
            const double bg = prop.bg64[r];
            const double G0 = o[0] + bg;
            double Sg = 0.0;
            for (int c = 1; c <= d; ++c) Sg += fabs(o[c]);
            const double eps = prop.kout64 * (prop.ag64[r] * emax + fabs(bg)) + kEta64;
            const double R = o[ncol - 1] + eps;
            const double delta = net.kconc64 * (fabs(G0) + R + Sg);
            const double glo = (G0 - (R + Sg)) - delta;
            const double ghi = (G0 + (R + Sg)) + delta;
            // float32 copies rounded outward
            float flo = (float)glo;
            if ((double)flo > glo) flo = nextafterf(flo, -INFINITY);
            float fhi = (float)ghi;
            if ((double)fhi < ghi) fhi = nextafterf(fhi, INFINITY);
            if (g_lo) g_lo[b * rows + r] = flo;
            if (g_hi) g_hi[b * rows + r] = fhi;
            unsafe = unsafe && (glo > 0.0);
            safe = safe || (ghi <= 0.0);
        }
        cls[b] = unsafe ? 1 : (safe ? 2 : 0);
        if (counter) atomicAdd(counter, 1ull);
    }
    wave_sync();
}

// List mode (list != NULL): boxes list[0 .. *list_count) (indices into lo/hi/cls), one per wave.
// Scan mode: every box with cls == 3 among the n boxes.
// ------------------------------------------------------------------------------------------
// Level bookkeeping: per-tile undecided counts, class histograms, compaction + bisection.
// ------------------------------------------------------------------------------------------
constexpr int kTile = 1024;   // boxes per bookkeeping workgroup (256 threads x 4)

__device__ __forceinline__ unsigned block_sum256(unsigned v, unsigned* red) {
    // returns the total; red holds 4 wave partials
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    const unsigned t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

// Class histogram of one 1024-box tile and its undecided count.
// Top of the search tree in one pass.  Box i of the complete subtree of depth K (heap order,
// path id i + 1, depth = position of the id's leading bit), built from the root corners rlo, rhi
// by the split rule of `split_tile` (widest side, lowest index on ties, float32 midpoint): the
// same operations on the same values, so its corners are those the level-by-level search makes.
// A midpoint that is not exact sets bit 0 of err[parent depth] (err_stride 1) or of *err
// (err_stride 0).
__device__ __forceinline__ void prefix_box(int64_t i, int d, const float* rlo, const float* rhi,
                                           float* __restrict__ L, float* __restrict__ H,
                                           unsigned long long* __restrict__ path, unsigned* err,
                                           int err_stride) {
    const unsigned long long P = (unsigned long long)i + 1ull;
    const int t = 63 - __clzll((long long)P);
    for (int k = 0; k < d; ++k) {
        L[k] = rlo[k];
        H[k] = rhi[k];
    }
    for (int s = t - 1; s >= 0; --s) {
        int js = 0;
        float wbest = H[0] - L[0];
        for (int k = 1; k < d; ++k) {
            const float w = H[k] - L[k];
            if (w > wbest) {
                wbest = w;
                js = k;
            }
        }
        const float m = 0.5f * (L[js] + H[js]);
        if (!(m - L[js] == H[js] - m && L[js] < m && m < H[js])) atomicOr(err + err_stride * (t - 1 - s), 1u);
        if ((P >> s) & 1ull)
            L[js] = m;
        else
            H[js] = m;
    }
    *path = P;
}

// Boxes [i0, i0 + 256) of the complete subtree (heap order), one per thread: made in the LDS
// stage (2 x 256 x d floats, each box's corners a contiguous row), then written out by the
// workgroup with consecutive threads on consecutive floats (coalesced; a box per thread would
// store with a stride of d floats).
__device__ __forceinline__ void prefix_block(int64_t N, int64_t i0, int d, const float* rlo,
                                             const float* rhi, float* __restrict__ lo,
                                             float* __restrict__ hi,
                                             unsigned long long* __restrict__ path, unsigned* err,
                                             int err_stride, float* stage) {
    const int64_t i = i0 + threadIdx.x;
    float* L = stage + threadIdx.x * d;
    float* H = stage + (256 + threadIdx.x) * d;
    if (i < N) prefix_box(i, d, rlo, rhi, L, H, path + i, err, err_stride);
    __syncthreads();
    const int nf = (int)min((int64_t)256, N - i0) * d;
    for (int e = threadIdx.x; e < nf; e += blockDim.x) {
        lo[i0 * d + e] = stage[e];
        hi[i0 * d + e] = stage[256 * d + e];
    }
}

// Which subtree boxes the level-by-level search visits: box i is bounded there iff none of its
// ancestors was decided (class 1 or 2).  Unvisited boxes get class 4 (no count, no split); the
// visited ones of depths 0 .. K - 1 are counted into stats[depth] (one block of 256 boxes, LDS
// histogram, then 64-bit atomics).  (A box's own class is final here; overwriting an unvisited
// ancestor's 0 with 4 while a descendant reads it cannot change the descendant's verdict: that
// ancestor has a decided ancestor of its own, which the descendant reads as well.)
__device__ __forceinline__ void prefix_replay_block(int64_t N, int K, int8_t* cls, LevelStats* stats,
                                                    int64_t i0) {
    __shared__ unsigned hist[16 * 3];
    for (int e = threadIdx.x; e < 16 * 3; e += blockDim.x) hist[e] = 0;
    __syncthreads();
    const int64_t i = i0 + threadIdx.x;
    if (i < N) {
        const unsigned long long P = (unsigned long long)i + 1ull;
        const int t = 63 - __clzll((long long)P);
        bool visited = true;
        for (unsigned long long a = P >> 1; a >= 1ull; a >>= 1) {
            const int8_t c = cls[a - 1];
            if (c == 1 || c == 2) {
                visited = false;
                break;
            }
        }
        const int8_t c = cls[i];
        if (!visited)
            cls[i] = 4;
        else if (t < K)
            atomicAdd(&hist[t * 3 + (c == 1 ? 0 : (c == 2 ? 1 : 2))], 1u);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * 3; e += blockDim.x) {
        const unsigned v = hist[e];
        if (!v) continue;
        LevelStats* st = stats + e / 3;
        unsigned long long* dst = e % 3 == 0 ? &st->unsafe_cnt : (e % 3 == 1 ? &st->safe_cnt : &st->undecided_cnt);
        atomicAdd(dst, (unsigned long long)v);
    }
}

__device__ __forceinline__ void count_tile(int64_t n, const int8_t* __restrict__ cls,
                                           unsigned* __restrict__ tile_und, LevelStats* stats,
                                           int64_t tile) {
    __shared__ unsigned red[4];
    const int64_t base = (int64_t)tile * kTile + threadIdx.x * 4;
    unsigned nu = 0, ns = 0, nd = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = base + q;
        if (i < n) {
            const int8_t c = cls[i];
            nu += c == 1;
            ns += c == 2;
            nd += c == 0;
        }
    }
    nu = block_sum256(nu, red);
    ns = block_sum256(ns, red);
    nd = block_sum256(nd, red);
    if (threadIdx.x == 0) {
        tile_und[tile] = nd;
        if (nu) atomicAdd(&stats->unsafe_cnt, (unsigned long long)nu);
        if (ns) atomicAdd(&stats->safe_cnt, (unsigned long long)ns);
        if (nd) atomicAdd(&stats->undecided_cnt, (unsigned long long)nd);
    }
}

// Children of the undecided boxes of one 1024-box tile, written in parent order after those of
// all earlier tiles; child pairs at index >= cap (the frontier capacity) are not written.
// Each parent is bisected at the midpoint of its widest coordinate (first one on ties).
// Phases: (1) local ranks of the undecided boxes by a workgroup scan; (2) with STAGED, a coalesced
// copy of the tile's corner rows into LDS (kSplitStageD coordinates at most); (3) one thread per
// parent picks the coordinate and midpoint and writes the child paths; (4) the children's corner
// rows, one contiguous run per tile, are written element by element (coalesced stores).
constexpr int kSplitStageD = 8;   // largest d whose 1024 x 2 x d corner floats are staged in LDS

template <bool STAGED>
__device__ __forceinline__ void split_tile_impl(int64_t n, int d, const int8_t* __restrict__ cls,
                                                const unsigned* __restrict__ tile_und,
                                                const float* __restrict__ lo,
                                                const float* __restrict__ hi,
                                                const unsigned long long* __restrict__ path,
                                                float* __restrict__ lo2, float* __restrict__ hi2,
                                                unsigned long long* __restrict__ path2,
                                                unsigned* err, int64_t cap, int64_t tile,
                                                float* stage, const int8_t* __restrict__ dimsel) {
    __shared__ unsigned red[4];
    __shared__ unsigned wpre[4];
    __shared__ unsigned short pidx[kTile];   // tile-local box index of the parent of local rank
    __shared__ unsigned char jsel[kTile];    // its bisected coordinate
    __shared__ float mval[kTile];            // and the midpoint
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // offset of this tile: undecided boxes of all earlier tiles
    unsigned pre = 0;
    for (unsigned k = tid; k < tile; k += 256) pre += tile_und[k];
    const int64_t base_out = block_sum256(pre, red);
    if (tile_und[tile] == 0) return;
    const int64_t t0 = tile * kTile;
    const int nb = (int)min((int64_t)kTile, n - t0);
    unsigned flags = 0, cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = tid * 4 + q;
        if (i < nb && cls[t0 + i] == 0) {
            flags |= 1u << q;
            ++cnt;
        }
    }
    // exclusive scan of cnt over the workgroup (thread order = box order)
    unsigned incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wpre[wave] = incl;
    __syncthreads();
    unsigned rank = incl - cnt;
    for (int w = 0; w < wave; ++w) rank += wpre[w];
    const int total = (int)(wpre[0] + wpre[1] + wpre[2] + wpre[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (flags & (1u << q)) pidx[rank++] = (unsigned short)(tid * 4 + q);
    const float* rlo = lo + t0 * d;
    const float* rhi = hi + t0 * d;
    if (STAGED) {
        const int m = nb * d;
        for (int e0 = tid; e0 < m; e0 += 256 * 4) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + 256 * u;
                a[u] = e < m ? rlo[e] : 0.f;
                b[u] = e < m ? rhi[e] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + 256 * u;
                if (e < m) {
                    stage[e] = a[u];
                    stage[kTile * d + e] = b[u];
                }
            }
        }
        rlo = stage;
        rhi = stage + kTile * d;
    }
    __syncthreads();
    // pairs whose second child still fits the frontier: global rank < floor(cap / 2)
    const int64_t fit = cap / 2 - base_out;
    const int npairs = (int)max((int64_t)0, min((int64_t)total, fit));
    for (int r = tid; r < total; r += 256) {
        const int p = pidx[r];
        const float* l = rlo + p * d;
        const float* h = rhi + p * d;
        // widest side, lowest index on ties; widths are loaded eight at a time (indices clamped
        // into the row, so every load is in bounds and none waits on the comparison before it)
        int js = 0;
        float wbest = h[0] - l[0];
        if (dimsel) js = min(max((int)dimsel[t0 + p], 0), d - 1);   // chosen by the bound kernel
        for (int k0 = 1; k0 < d && !dimsel; k0 += 8) {
            float wv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = min(k0 + u, d - 1);
                wv[u] = h[kk] - l[kk];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < d && wv[u] > wbest) {
                    wbest = wv[u];
                    js = k0 + u;
                }
        }
        const float m = 0.5f * (l[js] + h[js]);
        if (!(m - l[js] == h[js] - m && l[js] < m && m < h[js])) atomicOr(err, 1u);
        jsel[r] = (unsigned char)js;
        mval[r] = m;
        if (r < npairs) {
            const unsigned long long pp = path[t0 + p];
            path2[2 * (base_out + r)] = 2ull * pp;
            path2[2 * (base_out + r) + 1] = 2ull * pp + 1ull;
        }
    }
    __syncthreads();
    // children rows: element e of the run is coordinate k of child c = 2 r + side
    float* olo = lo2 + 2 * base_out * d;
    float* ohi = hi2 + 2 * base_out * d;
    const int m = 2 * npairs * d;
    // four elements per thread and pass, all loads before the stores (indices clamped into the
    // run, so every load is in bounds); without staging the parents' corners come from global
    // memory and a load-store chain per element would wait out one memory latency each
    for (int e0 = tid; e0 < m; e0 += 256 * 4) {
        float lv[4], hv[4], mv[4];
        bool cl[4], ch[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = min(e0 + 256 * u, m - 1);
            const int c = e / d, k = e - c * d;
            const int r = c >> 1, side = c & 1;
            const int p = pidx[r];
            const bool cut = k == jsel[r];
            mv[u] = mval[r];
            cl[u] = cut && side;
            ch[u] = cut && !side;
            lv[u] = rlo[p * d + k];
            hv[u] = rhi[p * d + k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + 256 * u;
            if (e < m) {
                olo[e] = cl[u] ? mv[u] : lv[u];
                ohi[e] = ch[u] ? mv[u] : hv[u];
            }
        }
    }
}

// stage: LDS of 2 * kTile * d floats (used when d <= kSplitStageD), or nullptr.
__device__ __forceinline__ void split_tile(int64_t n, int d, const int8_t* __restrict__ cls,
                                           const unsigned* __restrict__ tile_und,
                                           const float* __restrict__ lo,
                                           const float* __restrict__ hi,
                                           const unsigned long long* __restrict__ path,
                                           float* __restrict__ lo2, float* __restrict__ hi2,
                                           unsigned long long* __restrict__ path2,
                                           unsigned* err, int64_t cap, int64_t tile,
                                           float* stage, const int8_t* dimsel = nullptr) {
    if (stage && d <= kSplitStageD)
        split_tile_impl<true>(n, d, cls, tile_und, lo, hi, path, lo2, hi2, path2, err, cap, tile,
                              stage, dimsel);
    else
        split_tile_impl<false>(n, d, cls, tile_und, lo, hi, path, lo2, hi2, path2, err, cap, tile,
                               nullptr, dimsel);
}

// Exact leaf-volume sums: sum_t count_t 2^(Dm - t) in 64-bit integers (the totals partition
// 2^Dm exactly), converted to float64 fractions with a single rounding.
__device__ __forceinline__ void volume_body(const LevelStats* stats, int levels, int stop_level,
                                            int stopped, double* out3,
                                            unsigned long long* out_counts, unsigned* err) {
    const int Dm = levels - 1;
    unsigned long long su = 0, ss = 0, sd = 0, nu = 0, ns = 0, nd = 0;
    for (int t = 0; t < levels; ++t) {
        su += stats[t].unsafe_cnt << (Dm - t);
        ss += stats[t].safe_cnt << (Dm - t);
        nu += stats[t].unsafe_cnt;
        ns += stats[t].safe_cnt;
    }
    if (stopped) {
        sd = stats[stop_level].undecided_cnt << (Dm - stop_level);
        nd = stats[stop_level].undecided_cnt;
    }
    if (su + ss + sd != (1ull << Dm)) atomicOr(err, 2u);
    out3[0] = ldexp((double)su, -Dm);
    out3[1] = ldexp((double)ss, -Dm);
    out3[2] = ldexp((double)sd, -Dm);
    out_counts[0] = nu;
    out_counts[1] = ns;
    out_counts[2] = nd;
}

}  // namespace
