// gfx950 kernels of the alpha mode: the relaxation of Eq. 1 with a per-box, per-neuron lower
// slope alpha in [0, 1] (any such slope gives a valid lower line alpha z <= ReLU(z)), its
// hand-written adjoint, projected Adam fused into the adjoint, and the objective's center pass.
//
// State.  With its own lower slope a neuron's lower and upper equations no longer share their
// slopes, so a box keeps, per neuron, two full equations over box-local coordinates
// t in [-1, 1]^d (x = mid + rad * t): the center C = (L + U) / 2 and the radius R = (U - L) / 2,
// NC = d + 1 (or more, zero padded) coefficients each.  The W+/W- rule of symbolic propagation
// becomes two dense contractions, C' = W C + b and R' = |W| R, which run on MFMA.  Concretization
// over the box: l = (C0 - R0) - sum_i |C_i - R_i|, u = (C0 + R0) + sum_i |C_i + R_i|.
//
// Tile buffers.  A workgroup of four wavefronts takes 16 boxes.  A buffer holds, per column c and
// 16-neuron tile q, one float4 per lane:  buf[c][q][lane] = rows 16 q + 4 g + (0..3) of box j
// (lane = 16 g + j).  That is the B-operand layout of v_mfma_f32_16x16x4f32 for the 4 K-steps of
// quad q and also the accumulator layout of output tile q, so contractions read and write whole
// 1 KiB rows and every epilogue is lane-local.
//
// Tape.  The forward pass stores each layer's pre-activation C, R (with the widened radius
// constant) and the concrete bounds l, u per neuron; the adjoint reads them back.  Per tile the
// tape holds one slot per hidden layer, one for the property rows and, where the state does not
// fit in LDS, two more slots that replace the LDS state buffers.
#include "slr_internal.h"

#include <hip/hip_runtime.h>

#include <math.h>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kU32 = 0x1p-24f;
constexpr float kEta = 0x1p-96f;
constexpr int kNW = 4;

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bool row_valid(int mt, int g, int v, int tiles, int r) {
    return mt < tiles - 1 || 4 * v + g < r;
}

__device__ __forceinline__ float sgn(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// Projected Adam step constants: step size, moment decays, eps, bias corrections 1/(1 - beta^t).
struct AdamK {
    float lr, beta1, beta2, eps, c1, c2;
};

// Column groups of one contraction unit: for 2 NC <= 16 one unit takes every column (center
// columns with W, radius columns with |W|); otherwise units take CG columns of one half.
template <int NC> struct Groups;
template <> struct Groups<3>  { static constexpr int CG = 6,  NG = 1; static constexpr bool SPLIT = false; };
template <> struct Groups<4>  { static constexpr int CG = 8,  NG = 1; static constexpr bool SPLIT = false; };
template <> struct Groups<6>  { static constexpr int CG = 12, NG = 1; static constexpr bool SPLIT = false; };
template <> struct Groups<8>  { static constexpr int CG = 16, NG = 1; static constexpr bool SPLIT = false; };
template <> struct Groups<11> { static constexpr int CG = 11, NG = 2; static constexpr bool SPLIT = true; };
template <> struct Groups<14> { static constexpr int CG = 14, NG = 2; static constexpr bool SPLIT = true; };
template <> struct Groups<17> { static constexpr int CG = 9,  NG = 4; static constexpr bool SPLIT = true; };
template <> struct Groups<21> { static constexpr int CG = 11, NG = 4; static constexpr bool SPLIT = true; };
template <> struct Groups<25> { static constexpr int CG = 13, NG = 4; static constexpr bool SPLIT = true; };
template <> struct Groups<33> { static constexpr int CG = 11, NG = 6; static constexpr bool SPLIT = true; };

// Unroll factor of the epilogues' column sweeps: full for narrow states; wide states are swept
// in pairs so that the second sweep reloads (from L1/LDS) instead of keeping every column live.
template <int NC> constexpr int sweep_unroll() { return NC <= 8 ? NC : 2; }
// The adjoint's sweeps keep four column sets live (pre-activation C, R and its adjoint): sweep in
// pairs from NC = 6 on, which keeps it within 256 registers per lane (two wavefronts per SIMD).
template <int NC> constexpr int bwd_unroll() { return NC <= 4 ? NC : 2; }

// One contraction unit: output tile mt, column group grp, accumulated in registers:
//   acc[cc] = A(mt) * in[cb + cc]  (A = frag for center columns, |frag| for radius columns),
// summed over ks K-steps (frag is zero beyond them up to ks_alloc, a multiple of 4).  A comes
// from global memory (L2-resident), B from the tile buffer; the loop is software-pipelined one
// K-quad ahead.  Returns the first column cb and the number of real columns of the group.
template <int NC, typename PIn>
__device__ __forceinline__ void contract_acc(const float* __restrict__ frag, int ks, int ks_alloc,
                                             int mt, int grp, PIn in, int mtS, int lane,
                                             f32x4 (&acc)[Groups<NC>::CG], int& cb_out,
                                             int& ncols_out) {
    using G = Groups<NC>;
    constexpr int CG = G::CG;
    const int ngh = G::NG > 1 ? G::NG / 2 : 1;
    const int half = G::SPLIT ? grp / ngh : 0;
    const int first = G::SPLIT ? (grp - half * ngh) * CG : 0;
    const int cb = G::SPLIT ? half * NC + first : 0;
    const int ncols = G::SPLIT ? min(CG, NC - first) : CG;
    cb_out = cb;
    ncols_out = ncols;
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) acc[cc] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float* wf = frag + (size_t)mt * ks_alloc * 64 + lane;
    const int nq = (ks + 3) >> 2;
    auto col = [&](int cc) { return cb + (G::SPLIT ? min(cc, ncols - 1) : cc); };
    float af[4];
    f32x4 bq[CG];
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) af[ss] = wf[ss * 64];
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) bq[cc] = in[(size_t)(col(cc) * mtS) * 64 + lane];
    for (int q = 0; q < nq; ++q) {
        const int nx = min(q + 1, nq - 1);
        float an[4];
        f32x4 bn[CG];
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) an[ss] = wf[(4 * nx + ss) * 64];
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) bn[cc] = in[(size_t)(col(cc) * mtS + nx) * 64 + lane];
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            const float aw = af[ss];
            const float aa = fabsf(aw);
            const float ah = (G::SPLIT && half) ? aa : aw;
#pragma unroll
            for (int cc = 0; cc < CG; ++cc) {
                const float a = G::SPLIT ? ah : (cc >= NC ? aa : aw);
                acc[cc] = mfma16(a, bq[cc][ss], acc[cc]);
            }
        }
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) af[ss] = an[ss];
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) bq[cc] = bn[cc];
    }
}

template <int NC, typename PIn, typename POut>
__device__ __forceinline__ void contract_unit(const float* __restrict__ frag, int ks, int ks_alloc,
                                              int mt, int grp, PIn in, POut out, int mtS,
                                              const float* __restrict__ bias, int lane);

// Two output tiles (mt0, mt0 + 1) of one column group sharing every B-operand load: wide states
// keep their tile state in global memory, where B reads are the contraction's main traffic.
// The second tile is skipped when it does not exist (mt_out odd).
template <int NC, typename PIn, typename POut>
__device__ __forceinline__ void contract_unit2(const float* __restrict__ frag, int ks, int ks_alloc,
                                               int mt0, int mt_out, int grp, PIn in, POut out,
                                               int mtS, const float* __restrict__ bias, int lane) {
    using G = Groups<NC>;
    constexpr int CG = G::CG;
    const int ngh = G::NG > 1 ? G::NG / 2 : 1;
    const int half = G::SPLIT ? grp / ngh : 0;
    const int first = G::SPLIT ? (grp - half * ngh) * CG : 0;
    const int cb = G::SPLIT ? half * NC + first : 0;
    const int ncols = G::SPLIT ? min(CG, NC - first) : CG;
    const bool two = mt0 + 1 < mt_out;
    f32x4 acc[2][CG];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) acc[m][cc] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float* wf0 = frag + (size_t)mt0 * ks_alloc * 64 + lane;
    const float* wf1 = frag + (size_t)(two ? mt0 + 1 : mt0) * ks_alloc * 64 + lane;
    const int nq = (ks + 3) >> 2;
    auto col = [&](int cc) { return cb + (G::SPLIT ? min(cc, ncols - 1) : cc); };
    float af[2][4];
    f32x4 bq[CG];
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) {
        af[0][ss] = wf0[ss * 64];
        af[1][ss] = wf1[ss * 64];
    }
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) bq[cc] = in[(size_t)(col(cc) * mtS) * 64 + lane];
    for (int q = 0; q < nq; ++q) {
        const int nx = min(q + 1, nq - 1);
        float an[2][4];
        f32x4 bn[CG];
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            an[0][ss] = wf0[(4 * nx + ss) * 64];
            an[1][ss] = wf1[(4 * nx + ss) * 64];
        }
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) bn[cc] = in[(size_t)(col(cc) * mtS + nx) * 64 + lane];
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const float aw = af[m][ss];
                const float aa = fabsf(aw);
                const float ah = (G::SPLIT && half) ? aa : aw;
#pragma unroll
                for (int cc = 0; cc < CG; ++cc) {
                    const float a = G::SPLIT ? ah : (cc >= NC ? aa : aw);
                    acc[m][cc] = mfma16(a, bq[cc][ss], acc[m][cc]);
                }
            }
        }
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
            af[0][ss] = an[0][ss];
            af[1][ss] = an[1][ss];
        }
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) bq[cc] = bn[cc];
    }
    const int g = lane >> 4;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        if (m == 1 && !two) break;
        const int mt = mt0 + m;
#pragma unroll
        for (int cc = 0; cc < CG; ++cc) {
            if (G::SPLIT && cc >= ncols) continue;
            f32x4 o = acc[m][cc];
            if (bias && cb + cc == 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] += bias[16 * mt + 4 * g + v];
            }
            out[(size_t)((cb + cc) * mtS + mt) * 64 + lane] = o;
        }
    }
}

// Every unit of one contraction layer (mt_out output tiles x NG column groups) over the
// workgroup's wavefronts: pairs of output tiles for split (wide) states, single tiles otherwise.
template <int NC, typename PIn, typename POut>
__device__ __forceinline__ void contract_layer(const float* __restrict__ frag, int ks, int ks_alloc,
                                               int mt_out, PIn in, POut out, int mtS,
                                               const float* __restrict__ bias, int wave, int lane) {
    using G = Groups<NC>;
    if constexpr (G::SPLIT && NC <= 25) {   // (the widest class would spill with two tiles)
        const int pairs = (mt_out + 1) >> 1;
        for (int u = wave; u < pairs * G::NG; u += kNW)
            contract_unit2<NC>(frag, ks, ks_alloc, 2 * (u / G::NG), mt_out, u % G::NG, in, out, mtS,
                               bias, lane);
    } else {
        for (int u = wave; u < mt_out * G::NG; u += kNW)
            contract_unit<NC>(frag, ks, ks_alloc, u / G::NG, u % G::NG, in, out, mtS, bias, lane);
    }
}

// contract_acc, then out[c][mt] = acc (+ bias by relabeled row on column 0).
template <int NC, typename PIn, typename POut>
__device__ __forceinline__ void contract_unit(const float* __restrict__ frag, int ks, int ks_alloc,
                                              int mt, int grp, PIn in, POut out, int mtS,
                                              const float* __restrict__ bias, int lane) {
    using G = Groups<NC>;
    constexpr int CG = G::CG;
    f32x4 acc[CG];
    int cb, ncols;
    contract_acc<NC>(frag, ks, ks_alloc, mt, grp, in, mtS, lane, acc, cb, ncols);
    const int g = lane >> 4;
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) {
        if (G::SPLIT && cc >= ncols) continue;
        f32x4 o = acc[cc];
        if (bias && cb + cc == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] += bias[16 * mt + 4 * g + v];
        }
        out[(size_t)((cb + cc) * mtS + mt) * 64 + lane] = o;
    }
}

struct EpiK {
    float kconc, krelu, lamfac;
    int two;   // forward passes: one ratio per equation instead of Eq. 1's shared one
};

__device__ __forceinline__ EpiK epi_k(const NetDev& net, int raw, int two = 0) {
    EpiK k;
    k.kconc = raw ? 0.f : net.kconc;
    k.krelu = raw ? 0.f : net.krelu;
    k.lamfac = raw ? 1.f : 1.f + 0x1p-20f;   // keeps hi * rcp(hi - lo) >= the chord slope
    k.two = two;
    return k;
}

// Phase of one neuron from its concrete bounds, and the upper ratio (Eq. 1).
struct Phase {
    bool act, cross;
    float lam;   // upper multiplier: 0 dead, 1 active, the chord ratio when crossing
};

__device__ __forceinline__ Phase phase_of(float lo, float hi, bool valid, float lamfac) {
    Phase p;
    const bool dead = !valid || !(hi > 0.f);
    p.act = !dead && lo >= 0.f;
    p.cross = !dead && !p.act;
    const float lamc = fminf(1.f, hi * __builtin_amdgcn_rcpf(p.cross ? hi - lo : 1.f) * lamfac);
    p.lam = dead ? 0.f : (p.act ? 1.f : lamc);
    return p;
}

// Forward epilogue of one hidden tile (4 neurons per lane): widen the radius constant by the
// affine rounding margin eps, concretize, apply the alpha relaxation (or, with k.two, the
// relaxation with one ratio per equation) and write the post-activation state.  get(c) yields pre-activation column c (from the tape slot, or from the
// contraction's registers); the tape receives the widened radius constant and l, u (and, with
// cols, every pre-activation column).  Returns a bound on sum_c |C_c| + |R_c| over the lane's
// neurons (for the next layer's rounding margin).
template <int NC, int UNR, typename Get, typename PT, typename PS>
__device__ __forceinline__ float fwd_relu_core(Get get, PT tape, bool cols, PS post, int mtS,
                                               int mt, int lane, const float (&eps)[4],
                                               const bool (&valid)[4], float* __restrict__ arow,
                                               const int* __restrict__ rowmap, int init,
                                               const EpiK& k) {
    auto at = [&](int c) { return (size_t)(c * mtS + mt) * 64 + lane; };
    const int g = lane >> 4;
    f32x4 C0 = get(0);
    f32x4 R0 = get(NC);
#pragma unroll
    for (int v = 0; v < 4; ++v) R0[v] += eps[v];
    if (tape) {
        tape[at(NC)] = R0;
        if (cols) {
            tape[at(0)] = C0;
#pragma unroll
            for (int c = 1; c < NC; ++c) {
                tape[at(c)] = get(c);
                tape[at(NC + c)] = get(NC + c);
            }
        }
    }
    f32x4 SL = {0.f, 0.f, 0.f, 0.f}, SU = SL, M = SL;
#pragma unroll UNR
    for (int c = 1; c < NC; ++c) {
        const f32x4 Cc = get(c), Rc = get(NC + c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            SL[v] += fabsf(Cc[v] - Rc[v]);
            SU[v] += fabsf(Cc[v] + Rc[v]);
            M[v] += fabsf(Cc[v]) + fabsf(Rc[v]);
        }
    }
    f32x4 LO, HI;
    float al[4], au[4], sh[4];
    bool act[4], cross[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float delta = k.kconc * (fabsf(C0[v]) + fabsf(R0[v]) + M[v]);
        LO[v] = ((C0[v] - R0[v]) - SL[v]) - delta;
        HI[v] = ((C0[v] + R0[v]) + SU[v]) + delta;
        const Phase p = phase_of(LO[v], HI[v], valid[v], k.lamfac);
        act[v] = p.act;
        cross[v] = p.cross;
        au[v] = p.lam;
        sh[v] = p.cross ? LO[v] : 0.f;
        const int nrn = rowmap[16 * mt + 4 * g + v];
        float a = p.lam;
        if (arow && nrn >= 0) {
            if (init)
                arow[nrn] = p.cross ? p.lam : 1.f;
            else
                a = fminf(fmaxf(arow[nrn], 0.f), 1.f);
        }
        al[v] = p.cross ? a : p.lam;
        if (k.two && p.cross) {
            // upper: chord of ReLU over U's own range [lu, u] (U itself once lu >= 0); lower:
            // slope uL / (uL - l) from L's range [l, uL] (0 once uL <= 0); any lower slope in
            // [0, 1] is sound, the upper one is rounded up
            const float lu = ((C0[v] + R0[v]) - SU[v]) - delta;
            const float ul = ((C0[v] - R0[v]) + SL[v]) + delta;
            const bool chord = lu < 0.f;
            au[v] = chord ? fminf(1.f, HI[v] * __builtin_amdgcn_rcpf(HI[v] - lu) * k.lamfac) : 1.f;
            sh[v] = chord ? lu : 0.f;
            al[v] = ul > 0.f ? fminf(1.f, fmaxf(0.f, ul * __builtin_amdgcn_rcpf(ul - LO[v]))) : 0.f;
        }
    }
    if (tape) {
        tape[at(2 * NC)] = LO;
        tape[at(2 * NC + 1)] = HI;
    }
    f32x4 E = {0.f, 0.f, 0.f, 0.f}, mag = E;
#pragma unroll UNR
    for (int c = 1; c < NC; ++c) {
        const f32x4 Cc = get(c), Rc = get(NC + c);
        f32x4 Cn, Rn;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float Lp = al[v] * (Cc[v] - Rc[v]);
            const float Up = au[v] * (Cc[v] + Rc[v]);
            Cn[v] = act[v] ? Cc[v] : 0.5f * (Lp + Up);
            Rn[v] = act[v] ? Rc[v] : 0.5f * (Up - Lp);
            E[v] += fabsf(Lp) + fabsf(Up);
            mag[v] += fabsf(Cn[v]) + fabsf(Rn[v]);
        }
        post[at(c)] = Cn;
        post[at(NC + c)] = Rn;
    }
    f32x4 Cn, Rn;
    float emax = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float Lp = al[v] * (C0[v] - R0[v]);
        const float Up = au[v] * ((C0[v] + R0[v]) - sh[v]);
        const float er = cross[v] ? k.krelu * (E[v] + fabsf(Lp) + fabsf(Up)) : 0.f;
        Cn[v] = act[v] ? C0[v] : 0.5f * (Lp + Up);
        Rn[v] = act[v] ? R0[v] : 0.5f * (Up - Lp) + er;
        emax = fmaxf(emax, (mag[v] + fabsf(Cn[v]) + fabsf(Rn[v])) * (1.f + 4.f * kU32));
    }
    post[at(0)] = Cn;
    post[at(NC)] = Rn;
    return emax;
}

// The epilogue on a tape slot that already holds the pre-activation columns.
template <int NC, typename PT, typename PS>
__device__ __forceinline__ float fwd_relu(PT pre, PS post, int mtS, int mt, int lane,
                                          const float (&eps)[4], const bool (&valid)[4],
                                          float* __restrict__ arow, const int* __restrict__ rowmap,
                                          int init, const EpiK& k) {
    auto get = [&](int c) { return pre[(size_t)(c * mtS + mt) * 64 + lane]; };
    return fwd_relu_core<NC, sweep_unroll<NC>()>(get, pre, false, post, mtS, mt, lane, eps, valid,
                                                 arow, rowmap, init, k);
}

// The epilogue on pre-activation columns held in registers (narrow states); the tape (NULL in a
// forward-only pass) receives every column.
template <int NC, typename PT, typename PS>
__device__ __forceinline__ float fwd_relu_reg(const f32x4 (&a)[2 * NC], PT tape, PS post, int mtS,
                                              int mt, int lane, const float (&eps)[4],
                                              const bool (&valid)[4], float* __restrict__ arow,
                                              const int* __restrict__ rowmap, int init,
                                              const EpiK& k) {
    auto get = [&](int c) { return a[c]; };
    return fwd_relu_core<NC, NC>(get, tape, true, post, mtS, mt, lane, eps, valid, arow, rowmap,
                                 init, k);
}

// Adjoint of fwd_relu for one hidden tile.  In: dpost = d J / d(post-activation C, R); the tape
// slot (pre-activation, widened radius constant, l, u).  Out: dpre = d J / d(pre-activation C, R),
// d J / d alpha of the crossing neurons (written to drow and/or applied by projected Adam).
// The rounding margins are treated as constants.
template <int NC, int UNR, typename GetD, typename PT, typename PS>
__device__ __forceinline__ void bwd_relu_core(PT pre, GetD getd, PS dpre, int mtS, int mt, int lane,
                                              const bool (&valid)[4], float* __restrict__ arow,
                                              float* __restrict__ drow, float* __restrict__ mrow,
                                              float* __restrict__ vrow,
                                              const int* __restrict__ rowmap, const AdamK& A,
                                              const EpiK& k) {
    auto at = [&](int c) { return (size_t)(c * mtS + mt) * 64 + lane; };
    const int g = lane >> 4;
    const f32x4 LO = pre[at(2 * NC)], HI = pre[at(2 * NC + 1)];
    bool act[4], cross[4];
    float lam[4], al[4];
    int nrn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const Phase p = phase_of(LO[v], HI[v], valid[v], k.lamfac);
        act[v] = p.act;
        cross[v] = p.cross;
        lam[v] = p.lam;
        nrn[v] = rowmap[16 * mt + 4 * g + v];
        float a = p.lam;
        if (arow && nrn[v] >= 0) a = fminf(fmaxf(arow[nrn[v]], 0.f), 1.f);
        al[v] = p.cross ? a : p.lam;
    }
    // sweep 1: d alpha = dL'.L, d lam = dU'.(U - l e0)
    float dal[4] = {0.f, 0.f, 0.f, 0.f}, dlam[4] = {0.f, 0.f, 0.f, 0.f}, dU0[4];
#pragma unroll UNR
    for (int c = 0; c < NC; ++c) {
        const f32x4 Cc = pre[at(c)], Rc = pre[at(NC + c)];
        const f32x4 dC = getd(c), dR = getd(NC + c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float dLp = 0.5f * (dC[v] - dR[v]);
            const float dUp = 0.5f * (dC[v] + dR[v]);
            dal[v] += dLp * (Cc[v] - Rc[v]);
            dlam[v] += dUp * ((Cc[v] + Rc[v]) - (c == 0 ? LO[v] : 0.f));
            if (c == 0) dU0[v] = dUp;
        }
    }
    float dl[4], du[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        // lam = hi / (hi - lo): d lam / d lo = hi / den^2, d lam / d hi = -lo / den^2
        const float den = HI[v] - LO[v];
        const float inv2 = cross[v] ? 1.f / (den * den) : 0.f;
        dl[v] = cross[v] ? -lam[v] * dU0[v] + dlam[v] * HI[v] * inv2 : 0.f;
        du[v] = cross[v] ? -dlam[v] * LO[v] * inv2 : 0.f;
    }
    // sweep 2: adjoint of the pre-activation
#pragma unroll UNR
    for (int c = 0; c < NC; ++c) {
        const f32x4 Cc = pre[at(c)], Rc = pre[at(NC + c)];
        const f32x4 dC = getd(c), dR = getd(NC + c);
        f32x4 oC, oR;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float dLp = 0.5f * (dC[v] - dR[v]);
            const float dUp = 0.5f * (dC[v] + dR[v]);
            const float sl = c == 0 ? 1.f : -sgn(Cc[v] - Rc[v]);
            const float su = c == 0 ? 1.f : sgn(Cc[v] + Rc[v]);
            const float dL = al[v] * dLp + sl * dl[v];
            const float dU = lam[v] * dUp + su * du[v];
            oC[v] = act[v] ? dC[v] : (cross[v] ? dL + dU : 0.f);
            oR[v] = act[v] ? dR[v] : (cross[v] ? dU - dL : 0.f);
        }
        dpre[at(c)] = oC;
        dpre[at(NC + c)] = oR;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (nrn[v] < 0) continue;
        const float gr = cross[v] ? dal[v] : 0.f;
        if (drow) drow[nrn[v]] = gr;
        if (mrow) {
            const float m = A.beta1 * mrow[nrn[v]] + (1.f - A.beta1) * gr;
            const float s = A.beta2 * vrow[nrn[v]] + (1.f - A.beta2) * gr * gr;
            mrow[nrn[v]] = m;
            vrow[nrn[v]] = s;
            const float a = arow[nrn[v]] - A.lr * (m * A.c1) / (sqrtf(s * A.c2) + A.eps);
            arow[nrn[v]] = fminf(fmaxf(a, 0.f), 1.f);
        }
    }
}

template <int NC, typename PT, typename PS>
__device__ __forceinline__ void bwd_relu(PT pre, PS dpost, PS dpre, int mtS, int mt, int lane,
                                         const bool (&valid)[4], float* __restrict__ arow,
                                         float* __restrict__ drow, float* __restrict__ mrow,
                                         float* __restrict__ vrow, const int* __restrict__ rowmap,
                                         const AdamK& A, const EpiK& k) {
    auto getd = [&](int c) { return dpost[(size_t)(c * mtS + mt) * 64 + lane]; };
    bwd_relu_core<NC, bwd_unroll<NC>()>(pre, getd, dpre, mtS, mt, lane, valid, arow, drow, mrow,
                                        vrow, rowmap, A, k);
}

// The adjoint with d J / d(post-activation) held in registers (narrow states).
template <int NC, typename PT, typename PS>
__device__ __forceinline__ void bwd_relu_reg(const f32x4 (&dp)[2 * NC], PT pre, PS dpre, int mtS,
                                             int mt, int lane, const bool (&valid)[4],
                                             float* __restrict__ arow, float* __restrict__ drow,
                                             float* __restrict__ mrow, float* __restrict__ vrow,
                                             const int* __restrict__ rowmap, const AdamK& A,
                                             const EpiK& k) {
    auto getd = [&](int c) { return dp[c]; };
    bwd_relu_core<NC, NC>(pre, getd, dpre, mtS, mt, lane, valid, arow, drow, mrow, vrow, rowmap,
                          A, k);
}

__device__ __forceinline__ int hidden_tiles(const NetDev& net, int h) {
    return h == 0 ? net.mt1 : net.mid[h - 1].mt_out;
}
__device__ __forceinline__ int hidden_rem(const NetDev& net, int h) {
    return h == 0 ? net.r1 : net.mid[h - 1].r_out;
}

// ---------------------------------------------------------------------------------------------
// Forward pass: bounds of 16 boxes per workgroup with per-box slopes, tape for the adjoint.
// ---------------------------------------------------------------------------------------------
// RP: every layer's columns fit one contraction unit and its tiles one unit per wavefront, so
// contraction results stay in registers across the barrier and the epilogue reads no tape.
// The forward pass of 16-box tile `tile` (one workgroup of kNW wavefronts).
// TWO: honour A.two_ratio (the standalone forward kernel; the fused optimizer's forward passes
// always take alpha slopes)
template <int NC, bool GS, bool RP, bool TWO = false>
__device__ __forceinline__ void alpha_fwd_tile(const NetDev& net, const PropDev& prop,
                                               const AlphaArgs& A, int slots, int64_t tile,
                                               int init) {
    extern __shared__ __attribute__((aligned(16))) float lds[];   // 16-byte aligned after any static LDS
    using G = Groups<NC>;
    constexpr int NC2 = 2 * NC;
    constexpr int NCT = 2 * NC + 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, j = lane & 15;
    const int64_t b = tile * 16 + j;
    const bool bval = b < A.n;
    const int mtS = net.mt_max;
    const size_t slot = (size_t)NCT * mtS * 64;   // float4 per slot
    const int H = net.n_affine - 1;
    const int d = net.d;
    f32x4* tape = reinterpret_cast<f32x4*>(A.tape) + (size_t)tile * slots * slot;
    const EpiK k = epi_k(net, A.raw, TWO ? A.two_ratio : 0);
    float* part;
    f32x4* S;
    if constexpr (GS) {
        S = tape + (size_t)(A.fwd_only ? 1 : H + 1) * slot;
        part = lds;
    } else {
        S = reinterpret_cast<f32x4*>(lds);
        part = lds + (size_t)NC2 * mtS * 256;
    }
    auto part_at = [&](int par, int q) -> float& { return part[(par * mtS + q) * 16 + j]; };
    float* arow = (A.alpha && bval) ? A.alpha + (size_t)b * net.nh : nullptr;

    // ---- first affine layer (exact on the VALU), then the alpha epilogue
    {
        float mid[NC - 1], rad[NC - 1];
#pragma unroll
        for (int kk = 0; kk < NC - 1; ++kk) {
            float l = 0.f, h = 0.f;
            if (bval && kk < d) {
                l = A.lo[b * d + kk];
                h = A.hi[b * d + kk];
            }
            const float m = 0.5f * (l + h);
            mid[kk] = m;
            rad[kk] = A.raw ? 0.5f * (h - l) : fmaxf(h - m, m - l) * (1.f + 0x1p-22f);
        }
        f32x4* pre = tape;
        for (int mt = wave; mt < net.mt1; mt += kNW) {
            auto at = [&](int c) { return (size_t)(c * mtS + mt) * 64 + lane; };
            bool valid[4];
            float c0[4], s[4], eps[4];
            int m[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                m[v] = 16 * mt + 4 * g + v;
                valid[v] = row_valid(mt, g, v, net.mt1, net.r1);
                c0[v] = valid[v] ? net.b1p[m[v]] : 0.f;
                s[v] = fabsf(c0[v]);
            }
            f32x4 cols[NC2];
#pragma unroll
            for (int kk = 0; kk < NC - 1; ++kk) {
                f32x4 colv;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float w = (valid[v] && kk < d) ? net.w1p[m[v] * d + kk] : 0.f;
                    c0[v] = fmaf(w, mid[kk], c0[v]);
                    colv[v] = w * rad[kk];
                    s[v] += fabsf(w) * (fabsf(mid[kk]) + rad[kk]);
                }
                if constexpr (RP) cols[1 + kk] = colv;
                else pre[at(1 + kk)] = colv;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) eps[v] = A.raw ? 0.f : net.kfirst * s[v] + kEta;
            float emax;
            if constexpr (RP) {
                cols[0] = f32x4{c0[0], c0[1], c0[2], c0[3]};
#pragma unroll
                for (int c = NC; c < NC2; ++c) cols[c] = f32x4{0.f, 0.f, 0.f, 0.f};
                emax = fwd_relu_reg<NC>(cols, A.fwd_only ? nullptr : pre, S, mtS, mt, lane, eps,
                                        valid, arow ? arow + net.hoff[0] : nullptr, net.rowmap[0],
                                        init, k);
            } else {
                pre[at(0)] = f32x4{c0[0], c0[1], c0[2], c0[3]};
#pragma unroll
                for (int c = NC; c < NC2; ++c) pre[at(c)] = f32x4{0.f, 0.f, 0.f, 0.f};
                emax = fwd_relu<NC>(pre, S, mtS, mt, lane, eps, valid,
                                    arow ? arow + net.hoff[0] : nullptr, net.rowmap[0], init, k);
            }
            emax = fmaxf(emax, __shfl_xor(emax, 16));
            emax = fmaxf(emax, __shfl_xor(emax, 32));
            if (g == 0) part_at(0, mt) = emax;
        }
    }
    __syncthreads();

    // ---- hidden-to-hidden layers: MFMA contraction into the tape, then the epilogue
    int rp = 0, mt_prev = net.mt1;
    for (int l = 0; l < H - 1; ++l) {
        const MidLayer& L = net.mid[l];
        f32x4* pre = tape + (size_t)(A.fwd_only ? 0 : l + 1) * slot;
        const int units = L.mt_out * G::NG;
        f32x4 acc[G::CG];
        if constexpr (RP) {
            int cb, ncols;
            if (wave < L.mt_out)
                contract_acc<NC>(L.wfrag, L.ks, L.ks_alloc, wave, 0, S, mtS, lane, acc, cb, ncols);
        } else {
            contract_layer<NC>(L.wfrag, L.ks, L.ks_alloc, L.mt_out, S, pre, mtS, L.bias, wave, lane);
        }
        __syncthreads();
        for (int mt = wave; mt < L.mt_out; mt += kNW) {
            float emax_in = 0.f;
            for (int q = 0; q < mt_prev; ++q) emax_in = fmaxf(emax_in, part_at(rp, q));
            bool valid[4];
            float eps[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 16 * mt + 4 * g + v;
                valid[v] = row_valid(mt, g, v, L.mt_out, L.r_out);
                eps[v] = A.raw ? 0.f : L.kgam * (L.absrow[m] * emax_in + fabsf(L.bias[m])) + kEta;
            }
            float emax;
            if constexpr (RP) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[0][v] += L.bias[16 * mt + 4 * g + v];
                emax = fwd_relu_reg<NC>(acc, A.fwd_only ? nullptr : pre, S, mtS, mt, lane, eps,
                                        valid, arow ? arow + net.hoff[l + 1] : nullptr,
                                        net.rowmap[l + 1], init, k);
            } else {
                emax = fwd_relu<NC>(pre, S, mtS, mt, lane, eps, valid,
                                    arow ? arow + net.hoff[l + 1] : nullptr, net.rowmap[l + 1],
                                    init, k);
            }
            emax = fmaxf(emax, __shfl_xor(emax, 16));
            emax = fmaxf(emax, __shfl_xor(emax, 32));
            if (g == 0) part_at(rp ^ 1, mt) = emax;
        }
        rp ^= 1;
        mt_prev = L.mt_out;
        __syncthreads();
    }

    // ---- property rows (folded last layer), concretized; tile row 4 g + v is row 4 v + g
    f32x4* pre = tape + (size_t)(A.fwd_only ? 0 : H) * slot;
    for (int u = wave; u < G::NG; u += kNW)
        contract_unit<NC>(prop.wgfrag_a, prop.ks_out, prop.ks_out_alloc, 0, u, S, pre, mtS, prop.bga, lane);
    __syncthreads();
    if (wave == 0) {
        auto at = [&](int c) { return (size_t)(c * mtS) * 64 + lane; };
        const int rows = prop.rows;
        float emax = 0.f;
        for (int q = 0; q < mt_prev; ++q) emax = fmaxf(emax, part_at(rp, q));
        f32x4 C0 = pre[at(0)], R0 = pre[at(NC)];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = 4 * g + v;
            R0[v] += A.raw ? 0.f : prop.kout * (prop.aga[t] * emax + fabsf(prop.bga[t])) + kEta;
        }
        pre[at(NC)] = R0;
        f32x4 SL = {0.f, 0.f, 0.f, 0.f}, SU = SL, M = SL;
#pragma unroll sweep_unroll<NC>()
        for (int c = 1; c < NC; ++c) {
            const f32x4 Cc = pre[at(c)], Rc = pre[at(NC + c)];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                SL[v] += fabsf(Cc[v] - Rc[v]);
                SU[v] += fabsf(Cc[v] + Rc[v]);
                M[v] += fabsf(Cc[v]) + fabsf(Rc[v]);
            }
        }
        f32x4 LO, HI;
        bool unsafe = true, safe = false;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float delta = k.kconc * (fabsf(C0[v]) + fabsf(R0[v]) + M[v]);
            LO[v] = ((C0[v] - R0[v]) - SL[v]) - delta;
            HI[v] = ((C0[v] + R0[v]) + SU[v]) + delta;
            const int row = 4 * v + g;
            if (row < rows && bval) {
                const size_t o = (size_t)b * rows + row;
                if (A.g_lo) A.g_lo[o] = LO[v];
                if (A.g_hi) A.g_hi[o] = HI[v];
                float blo = LO[v], bhi = HI[v];
                if (A.best_lo) {
                    if (!init) {
                        blo = fmaxf(blo, A.best_lo[o]);
                        bhi = fminf(bhi, A.best_hi[o]);
                    }
                    A.best_lo[o] = blo;
                    A.best_hi[o] = bhi;
                }
                unsafe = unsafe && blo > 0.f;
                safe = safe || bhi <= 0.f;
            }
        }
        pre[at(NC2)] = LO;
        pre[at(NC2 + 1)] = HI;
        // every row of the box: AND / OR over the four lanes g of box j
        int us = unsafe ? 1 : 0, sf = safe ? 1 : 0;
        us &= __shfl_xor(us, 16);
        us &= __shfl_xor(us, 32);
        sf |= __shfl_xor(sf, 16);
        sf |= __shfl_xor(sf, 32);
        if (g == 0 && bval && A.cls) A.cls[b] = us ? 1 : (sf ? 2 : 0);
    }
}

// ---------------------------------------------------------------------------------------------
// Adjoint pass: d J / d alpha through the property rows, the transposed contractions W^T, |W|^T
// on MFMA and every alpha epilogue, from the tape of the forward pass with the same slopes.
// ---------------------------------------------------------------------------------------------
// The adjoint pass (with the fused projected Adam step when A.adam_m is set) of tile `tile`.
template <int NC, bool GS, bool RP>
__device__ __forceinline__ void alpha_bwd_tile(const NetDev& net, const PropDev& prop,
                                               const AlphaArgs& A, int slots, int64_t tile,
                                               const AdamK& ak) {
    extern __shared__ __attribute__((aligned(16))) float lds[];   // 16-byte aligned after any static LDS
    using G = Groups<NC>;
    constexpr int NC2 = 2 * NC;
    constexpr int NCT = 2 * NC + 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, j = lane & 15;
    const int64_t b = tile * 16 + j;
    const bool bval = b < A.n;
    const int mtS = net.mt_max;
    const size_t slot = (size_t)NCT * mtS * 64;
    const int H = net.n_affine - 1;
    f32x4* tape = reinterpret_cast<f32x4*>(A.tape) + (size_t)tile * slots * slot;
    const EpiK k = epi_k(net, A.raw);
    f32x4 *dA, *dB;   // dA: adjoint of a pre-activation, dB: of a post-activation
    if constexpr (GS) {
        dA = tape + (size_t)(H + 1) * slot;
        dB = tape + (size_t)(H + 2) * slot;
    } else {
        dA = reinterpret_cast<f32x4*>(lds);
        dB = dA + (size_t)NC2 * mtS * 64;
    }

    // ---- seeds and the adjoint of the concretized property rows
    if (wave == 0) {
        auto at = [&](int c) { return (size_t)(c * mtS) * 64 + lane; };
        const int rows = prop.rows;
        const f32x4* pre = tape + (size_t)H * slot;
        float dlo[4], dhi[4];
        int rstar = -1, mode = 0, rsel = -1;
        if (A.obj && bval) {
            mode = A.obj[2 * b];
            rsel = A.obj[2 * b + 1];
            if (mode == 1) {
                float mn = INFINITY;
                for (int r = 0; r < rows; ++r) {
                    const float x = A.g_lo[(size_t)b * rows + r];
                    if (x < mn) {
                        mn = x;
                        rstar = r;
                    }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 4 * v + g;
            dlo[v] = dhi[v] = 0.f;
            if (row < rows && bval) {
                if (A.obj) {
                    dlo[v] = (mode == 1 && row == rstar) ? -1.f : 0.f;
                    dhi[v] = (mode != 1 && row == rsel) ? 1.f : 0.f;
                } else {
                    dlo[v] = A.dg_lo ? A.dg_lo[(size_t)b * rows + row] : 0.f;
                    dhi[v] = A.dg_hi ? A.dg_hi[(size_t)b * rows + row] : 0.f;
                }
            }
        }
#pragma unroll sweep_unroll<NC>()
        for (int c = 0; c < NC; ++c) {
            const f32x4 Cc = pre[at(c)], Rc = pre[at(NC + c)];
            f32x4 oC, oR;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float dL = (c == 0 ? 1.f : -sgn(Cc[v] - Rc[v])) * dlo[v];
                const float dU = (c == 0 ? 1.f : sgn(Cc[v] + Rc[v])) * dhi[v];
                oC[v] = dL + dU;
                oR[v] = dU - dL;
            }
            dA[at(c)] = oC;
            dA[at(NC + c)] = oR;
        }
    }
    __syncthreads();
    float* arow = (A.alpha && bval) ? A.alpha + (size_t)b * net.nh : nullptr;
    float* drow = (A.dalpha && bval) ? A.dalpha + (size_t)b * net.nh : nullptr;
    float* mrow = (A.adam_m && bval) ? A.adam_m + (size_t)b * net.nh : nullptr;
    float* vrow = (A.adam_v && bval) ? A.adam_v + (size_t)b * net.nh : nullptr;
    if constexpr (RP) {
        // one LDS buffer: each wave holds the post-activation adjoint of its tile in registers
        f32x4 acc[G::CG];
        int cb, ncols;
        if (wave < net.mt_last)
            contract_acc<NC>(prop.wgtfrag, prop.ks_rows, prop.ks_rows_alloc, wave, 0, dA, mtS, lane,
                             acc, cb, ncols);
        __syncthreads();
        for (int h = H - 1; h >= 0; --h) {
            const int tiles = hidden_tiles(net, h), rem = hidden_rem(net, h);
            const int off = net.hoff[h];
            if (wave < tiles) {
                bool valid[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) valid[v] = row_valid(wave, g, v, tiles, rem);
                bwd_relu_reg<NC>(acc, tape + (size_t)h * slot, dA, mtS, wave, lane, valid,
                                 arow ? arow + off : nullptr, drow ? drow + off : nullptr,
                                 mrow ? mrow + off : nullptr, vrow ? vrow + off : nullptr,
                                 net.rowmap[h], ak, k);
            }
            if (h == 0) break;
            __syncthreads();
            const MidLayer& L = net.mid[h - 1];
            if (wave < L.mt_in)
                contract_acc<NC>(L.wtfrag, L.kst, L.kst_alloc, wave, 0, dA, mtS, lane, acc, cb, ncols);
            __syncthreads();
        }
        return;
    }
    {
        contract_layer<NC>(prop.wgtfrag, prop.ks_rows, prop.ks_rows_alloc, net.mt_last, dA, dB, mtS,
                           nullptr, wave, lane);
    }
    __syncthreads();

    for (int h = H - 1; h >= 0; --h) {
        const int tiles = hidden_tiles(net, h), rem = hidden_rem(net, h);
        const f32x4* pre = tape + (size_t)h * slot;
        const int off = net.hoff[h];
        for (int mt = wave; mt < tiles; mt += kNW) {
            bool valid[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) valid[v] = row_valid(mt, g, v, tiles, rem);
            bwd_relu<NC>(pre, dB, dA, mtS, mt, lane, valid, arow ? arow + off : nullptr,
                         drow ? drow + off : nullptr, mrow ? mrow + off : nullptr,
                         vrow ? vrow + off : nullptr, net.rowmap[h], ak, k);
        }
        if (h == 0) break;
        __syncthreads();
        const MidLayer& L = net.mid[h - 1];
        contract_layer<NC>(L.wtfrag, L.kst, L.kst_alloc, L.mt_in, dA, dB, mtS, nullptr, wave, lane);
        __syncthreads();
    }
}

template <int NC, bool GS, bool RP>
__global__ __launch_bounds__(kNW * 64, 2) void alpha_fwd_kernel(NetDev net, PropDev prop,
                                                             AlphaArgs A, int slots) {
    alpha_fwd_tile<NC, GS, RP, true>(net, prop, A, slots, blockIdx.x, A.init);
}

template <int NC, bool GS, bool RP>
__global__ __launch_bounds__(kNW * 64, 2) void alpha_bwd_kernel(NetDev net, PropDev prop,
                                                             AlphaArgs A, int slots) {
    const AdamK ak{A.lr, A.beta1, A.beta2, A.eps, A.c1, A.c2};
    alpha_bwd_tile<NC, GS, RP>(net, prop, A, slots, blockIdx.x, ak);
}

// A whole optimization of one tile: the forward pass that writes the plain ratios (init), then
// `steps` pairs (adjoint with the projected Adam step, forward).  Adam's bias corrections
// 1 / (1 - beta^t) are formed in float64 and rounded once, as a host loop would.  The tile's
// moments are cleared first.  Between passes the workgroup barrier orders the tape, LDS and
// per-box buffers, which only this workgroup touches.
template <int NC, bool GS, bool RPF, bool RPB>
__device__ __forceinline__ void alpha_opt_tile(const NetDev& net, const PropDev& prop,
                                               const AlphaArgs& A, int slots, int steps,
                                               int64_t tile) {
    {
        const int64_t b0 = tile * 16;
        const int64_t nb = min((int64_t)16, A.n - b0);
        const int64_t cnt = nb > 0 ? nb * net.nh : 0;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            A.adam_m[b0 * net.nh + e] = 0.f;
            A.adam_v[b0 * net.nh + e] = 0.f;
        }
    }
    alpha_fwd_tile<NC, GS, RPF>(net, prop, A, slots, tile, 1);
    double p1 = 1.0, p2 = 1.0;
    for (int t = 1; t <= steps; ++t) {
        p1 *= (double)A.beta1;
        p2 *= (double)A.beta2;
        const AdamK ak{A.lr, A.beta1, A.beta2, A.eps, (float)(1.0 / (1.0 - p1)), (float)(1.0 / (1.0 - p2))};
        __syncthreads();
        alpha_bwd_tile<NC, GS, RPB>(net, prop, A, slots, tile, ak);
        __syncthreads();
        alpha_fwd_tile<NC, GS, RPF>(net, prop, A, slots, tile, 0);
    }
}

template <int NC, bool GS, bool RPF, bool RPB>
__global__ __launch_bounds__(kNW * 64, 2) void alpha_opt_kernel(NetDev net, PropDev prop,
                                                             AlphaArgs A, int slots, int steps) {
    alpha_opt_tile<NC, GS, RPF, RPB>(net, prop, A, slots, steps, blockIdx.x);
}

// ---------------------------------------------------------------------------------------------
// Objective of each box from a float32 forward pass at its center: obj = (all rows > 0, argmin).
// ---------------------------------------------------------------------------------------------
// The objective of one box (the whole workgroup): a float32 forward pass at the box center;
// obj[0] = 1 if every property row is > 0 there, obj[1] = the row with the smallest value.
__device__ __forceinline__ void center_obj_box(const NetDev& net, const PropDev& prop,
                                               const float* __restrict__ lo,
                                               const float* __restrict__ hi,
                                               int8_t* __restrict__ obj, float* h0, float* h1,
                                               float* gv) {
    const int tid = threadIdx.x;
    const int d = net.d;
    if (tid < d) h1[tid] = 0.5f * (lo[tid] + hi[tid]);
    __syncthreads();
    if (tid < net.n1) {
        float s = net.b1[tid];
        for (int kk = 0; kk < d; ++kk) s = fmaf(net.w1[tid * d + kk], h1[kk], s);
        h0[tid] = fmaxf(s, 0.f);
    }
    __syncthreads();
    float* in = h0;
    float* out = h1;
    for (int l = 0; l < net.n_affine - 2; ++l) {
        const MidLayer& L = net.mid[l];
        if (tid < L.n_out) {
            float s = L.b[tid];
            const float* wr = L.w + (size_t)tid * L.n_in;
            for (int kk = 0; kk < L.n_in; ++kk) s = fmaf(wr[kk], in[kk], s);
            out[tid] = fmaxf(s, 0.f);
        }
        __syncthreads();
        float* t = in;
        in = out;
        out = t;
    }
    if (tid < prop.rows) {
        float s = prop.bg[tid];
        for (int kk = 0; kk < prop.n_last; ++kk) s = fmaf(prop.wg[tid * prop.n_last + kk], in[kk], s);
        gv[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        int all = 1, arg = 0;
        for (int r = 0; r < prop.rows; ++r) {
            all &= gv[r] > 0.f;
            if (gv[r] < gv[arg]) arg = r;
        }
        obj[0] = (int8_t)all;
        obj[1] = (int8_t)arg;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void center_obj_kernel(NetDev net, PropDev prop, int64_t n,
                                                         const float* __restrict__ lo,
                                                         const float* __restrict__ hi,
                                                         int8_t* __restrict__ obj) {
    __shared__ float h0[SLR_MAX_WIDTH], h1[SLR_MAX_WIDTH], gv[SLR_MAX_ROWS];
    const int d = net.d;
    for (int64_t p = blockIdx.x; p < n; p += gridDim.x)
        center_obj_box(net, prop, lo + p * d, hi + p * d, obj + 2 * p, h0, h1, gv);
}

// ---------------------------------------------------------------------------------------------
// Batched alpha pass: per alpha class, each instance's candidates occupy a 16-aligned segment
// of the class buffers (laid out by the plan kernel); a box or tile finds its instance by the
// segment starts.
// ---------------------------------------------------------------------------------------------
// Largest k with seg[k] <= q (seg non-decreasing, seg[0] = 0).
__device__ __forceinline__ int seg_owner(const unsigned* __restrict__ seg, int n, unsigned q) {
    int a = 0, b = n - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (seg[m] <= q) a = m;
        else b = m - 1;
    }
    return a;
}

__global__ __launch_bounds__(256) void batch_center_kernel(const BatchInst* insts, const BatchCtl* ctl,
                                                           int c, BatchAlphaBuf B) {
    __shared__ float h0[SLR_MAX_WIDTH], h1[SLR_MAX_WIDTH], gv[SLR_MAX_ROWS];
    const unsigned nb = ctl->antiles[c] * 16;
    for (unsigned q = blockIdx.x; q < nb; q += gridDim.x) {
        const int k = seg_owner(B.seg, B.ninst, q);
        const BatchInst& I = insts[B.inst[k]];
        const unsigned pos = q - I.aseg;
        if (pos >= I.alen) continue;   // padding of a segment (uniform)
        const size_t o = (size_t)I.aseg * B.dmax + (size_t)pos * I.d;
        center_obj_box(I.net, I.prop, B.lo + o, B.hi + o, B.obj + 2 * (size_t)q, h0, h1, gv);
    }
}

template <int NC, bool GS, bool RPF, bool RPB>
__global__ __launch_bounds__(kNW * 64, 2) void batch_alpha_opt_kernel(const BatchInst* insts,
                                                                   const BatchCtl* ctl, int c,
                                                                   BatchAlphaBuf B, AlphaArgs base,
                                                                   int steps) {
    const unsigned t = blockIdx.x;
    if (t >= ctl->antiles[c]) return;
    const int k = seg_owner(B.seg, B.ninst, 16 * t);
    const BatchInst& I = insts[B.inst[k]];
    const unsigned s0 = I.aseg;
    AlphaArgs A = base;
    A.n = I.alen;
    A.lo = B.lo + (size_t)s0 * B.dmax;
    A.hi = B.hi + (size_t)s0 * B.dmax;
    A.alpha = B.alpha + (size_t)s0 * B.nhmax;
    A.adam_m = B.m + (size_t)s0 * B.nhmax;
    A.adam_v = B.v + (size_t)s0 * B.nhmax;
    A.g_lo = B.glo + (size_t)s0 * B.rowsmax;
    A.g_hi = B.ghi + (size_t)s0 * B.rowsmax;
    A.best_lo = B.blo + (size_t)s0 * B.rowsmax;
    A.best_hi = B.bhi + (size_t)s0 * B.rowsmax;
    A.cls = B.cls + s0;
    A.obj = B.obj + 2 * (size_t)s0;
    A.tape = B.tape + I.atape;
    alpha_opt_tile<NC, GS, RPF, RPB>(I.net, I.prop, A, I.aslots, steps, (int64_t)(t - s0 / 16));
}

// Boxes the optimized bounds decided take their class back into the instance's level.
__global__ __launch_bounds__(256) void batch_scatter_kernel(BatchInst* insts, const BatchCtl* ctl,
                                                            int c, BatchAlphaBuf B) {
    const unsigned nb = ctl->antiles[c] * 16;
    for (unsigned q = blockIdx.x * 256 + threadIdx.x; q < nb; q += gridDim.x * 256) {
        const int k = seg_owner(B.seg, B.ninst, q);
        BatchInst& I = insts[B.inst[k]];
        if (q - I.aseg >= I.alen) continue;
        const int8_t v = B.cls[q];
        if (v != 0) {
            I.cls[B.list[q]] = v;
            atomicAdd((unsigned long long*)&I.n_alpha_decided, 1ull);
        }
    }
}

// Indices of the undecided boxes (class 0) of a level, appended with one atomic per wavefront.
// Distance of an undecided box from a decision, relative to its bound widths: the smaller of
// the unsafe distance (the largest (-g_lo)/(g_hi - g_lo) over rows with g_lo <= 0) and the safe
// distance (the smallest g_hi/(g_hi - g_lo) over the rows).
__device__ __forceinline__ float decision_distance(const float* glo, const float* ghi, int rows) {
    float du = 0.f, ds = INFINITY;
    for (int r = 0; r < rows; ++r) {
        const float w = ghi[r] - glo[r];
        if (!(w > 0.f)) continue;
        if (glo[r] <= 0.f) du = fmaxf(du, -glo[r] / w);
        ds = fminf(ds, ghi[r] / w);
    }
    return fminf(du, ds);
}

__global__ __launch_bounds__(256) void collect_kernel(int64_t n, const int8_t* __restrict__ cls,
                                                     unsigned* __restrict__ list,
                                                     unsigned* __restrict__ count,
                                                     const float* __restrict__ g_lo,
                                                     const float* __restrict__ g_hi, int rows,
                                                     float select, unsigned* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool und = i < n && cls[i] == 0;
    if (total) {   // every undecided box, selected or not
        const unsigned long long all = __ballot(und);
        if ((threadIdx.x & 63) == 0 && all) atomicAdd(total, (unsigned)__popcll(all));
    }
    if (und && g_lo) und = decision_distance(g_lo + i * rows, g_hi + i * rows, rows) <= select;
    const unsigned long long mask = __ballot(und);
    const int lane = threadIdx.x & 63;
    unsigned base = 0;
    const int leader = mask ? __ffsll((long long)mask) - 1 : 0;
    if (mask && lane == leader) base = atomicAdd(count, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    if (und) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (unsigned)i;
}

__global__ __launch_bounds__(256) void gather_kernel(int64_t m, int d, const unsigned* __restrict__ list,
                                                     const float* __restrict__ lo,
                                                     const float* __restrict__ hi,
                                                     float* __restrict__ lo2, float* __restrict__ hi2) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= m * d) return;
    const int64_t i = t / d, k = t - i * d;
    const int64_t src = (int64_t)list[i] * d + k;
    lo2[t] = lo[src];
    hi2[t] = hi[src];
}

__global__ __launch_bounds__(256) void scatter_kernel(int64_t m, const unsigned* __restrict__ list,
                                                      const int8_t* __restrict__ cls2,
                                                      int8_t* __restrict__ cls) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m && cls2[i] != 0) cls[list[i]] = cls2[i];
}

// Plain bounds from the tape-state kernel (shapes the LDS bound kernel cannot hold): boxes whose
// widened bounds leave them undecided but within twice the widening (plus 2^-14 of the row's
// magnitude) of a decision are marked 3 and listed for the FP64 re-decision, as the LDS kernel
// does from its rounding-margin column.
__global__ __launch_bounds__(256) void ambiguity_kernel(int64_t n, int rows,
                                                       const float* __restrict__ wlo,
                                                       const float* __restrict__ whi,
                                                       const float* __restrict__ rlo,
                                                       const float* __restrict__ rhi,
                                                       int8_t* __restrict__ cls,
                                                       unsigned* __restrict__ amb_list,
                                                       unsigned* __restrict__ amb_count,
                                                       unsigned base) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || cls[i] != 0) return;
    bool au = true, as = false;
    for (int r = 0; r < rows; ++r) {
        const size_t o = (size_t)i * rows + r;
        const float lo = wlo[o], hi = whi[o];
        const float t = 2.f * fmaxf(rlo[o] - lo, hi - rhi[o]) + 0x1p-14f * fmaxf(fabsf(lo), fabsf(hi));
        au = au && lo + t > 0.f;
        as = as || hi - t <= 0.f;
    }
    if (au || as) {
        cls[i] = 3;
        if (amb_list) amb_list[atomicAdd(amb_count, 1u)] = base + (unsigned)i;
    }
}

int nc_class(int d) {
    const int need = d + 1;
    const int cls[] = {3, 4, 6, 8, 11, 14, 17, 21, 25, 33};
    for (int c : cls)
        if (c >= need) return c;
    return -1;
}

size_t state_bytes(int nc, int mt_max) { return (size_t)2 * nc * mt_max * 1024; }

hipError_t allow_lds_a(const void* kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

template <int NC>
hipError_t launch_fwd_nc(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                         const AlphaShape& sh, hipStream_t stream) {
    const int64_t blocks = (a.n + 15) / 16;
    const int slots = a.fwd_only ? sh.slots_fwd : sh.slots;
    (void)hipGetLastError();
    if (sh.global_state) {
        auto kern = alpha_fwd_kernel<NC, true, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), sh.lds_fwd, stream, net, prop, a, slots);
    } else {
        if constexpr (NC <= 11) {
            auto kern = alpha_fwd_kernel<NC, false, false>;
            if constexpr (Groups<NC>::NG == 1) {
                if (sh.reg_path) kern = alpha_fwd_kernel<NC, false, true>;
            }
            hipError_t e = allow_lds_a((const void*)kern, sh.lds_fwd);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), sh.lds_fwd, stream, net, prop, a, slots);
        } else {
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int NC>
hipError_t launch_bwd_nc(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                         const AlphaShape& sh, hipStream_t stream) {
    const int64_t blocks = (a.n + 15) / 16;
    (void)hipGetLastError();
    if (sh.global_state) {
        auto kern = alpha_bwd_kernel<NC, true, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), 0, stream, net, prop, a, sh.slots);
    } else {
        if constexpr (NC <= 11) {
            auto kern = alpha_bwd_kernel<NC, false, false>;
            if constexpr (NC <= 6) {
                if (sh.reg_path_bwd) kern = alpha_bwd_kernel<NC, false, true>;
            }
            hipError_t e = allow_lds_a((const void*)kern, sh.lds_bwd);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), sh.lds_bwd, stream, net, prop, a, sh.slots);
        } else {
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int NC>
hipError_t launch_opt_nc(const NetDev& net, const PropDev& prop, const AlphaArgs& a, int steps,
                         const AlphaShape& sh, hipStream_t stream) {
    const int64_t blocks = (a.n + 15) / 16;
    (void)hipGetLastError();
    if (sh.global_state) {
        auto kern = alpha_opt_kernel<NC, true, false, false>;
        const size_t lds = sh.lds_fwd > sh.lds_bwd ? sh.lds_fwd : sh.lds_bwd;
        hipError_t e = allow_lds_a((const void*)kern, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), lds, stream, net, prop, a,
                           sh.slots, steps);
    } else {
        if constexpr (NC <= 11) {
            auto kern = alpha_opt_kernel<NC, false, false, false>;
            if constexpr (Groups<NC>::NG == 1) {
                if (sh.reg_path) kern = alpha_opt_kernel<NC, false, true, false>;
                if constexpr (NC <= 6) {
                    if (sh.reg_path_bwd) kern = alpha_opt_kernel<NC, false, true, true>;
                }
            }
            const size_t lds = sh.lds_fwd > sh.lds_bwd ? sh.lds_fwd : sh.lds_bwd;
            hipError_t e = allow_lds_a((const void*)kern, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNW * 64), lds, stream, net, prop,
                               a, sh.slots, steps);
        } else {
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace

namespace {
int g_alpha_state = 0;   // 0 automatic, 1 LDS where it fits, 2 always the tape's global slots
// 0 (default): one launch per pass; 1: one launch per optimization (alpha_opt_kernel).  With
// 65536 acas boxes the per-pass launches took 30.7 ms and the fused one 34.6 ms (the fused
// kernel spills: its step loop holds both passes' live values); the fused form pays where the
// passes are small, in the batched alpha pass.
int g_alpha_fused = 0;
}  // namespace

int set_alpha_fused(int v) {
    if (v != 0 && v != 1) return -1;
    g_alpha_fused = v;
    return 0;
}

int alpha_fused() { return g_alpha_fused; }

int set_alpha_state_variant(int v) {
    if (v < 0 || v > 2) return -1;
    g_alpha_state = v;
    return 0;
}

AlphaShape alpha_shape(const NetDev& net, const PropDev& prop) {
    (void)prop;
    AlphaShape s{};
    s.nc = nc_class(net.d);
    const size_t part = sizeof(float) * 2 * net.mt_max * 16;
    const size_t st = state_bytes(s.nc, net.mt_max);
    s.global_state = (s.nc > 11 || 2 * st + part > 150 * 1024 || g_alpha_state == 2) ? 1 : 0;
    // register path: one contraction unit per layer tile and at most one tile per wavefront
    s.reg_path = (!s.global_state && s.nc <= 8 && net.mt_max <= 4) ? 1 : 0;
    // the adjoint's register path spills beyond NC = 6 at two wavefronts per SIMD
    s.reg_path_bwd = (s.reg_path && s.nc <= 6) ? 1 : 0;
    s.lds_fwd = s.global_state ? part : st + part;
    s.lds_bwd = s.global_state ? 0 : (s.reg_path_bwd ? st : 2 * st);
    s.slots = (net.n_affine - 1) + 1 + (s.global_state ? 2 : 0);
    s.slots_fwd = 1 + (s.global_state ? 1 : 0);
    s.slot_floats = (size_t)(2 * s.nc + 2) * net.mt_max * 256;
    return s;
}

size_t alpha_tape_bytes(const NetDev& net, const PropDev& prop, int64_t n, int fwd_only) {
    const AlphaShape s = alpha_shape(net, prop);
    return sizeof(float) * (size_t)((n + 15) / 16) * (fwd_only ? s.slots_fwd : s.slots) * s.slot_floats;
}

#define SLR_ALPHA_NC(X) X(3) X(4) X(6) X(8) X(11) X(14) X(17) X(21) X(25) X(33)

hipError_t launch_alpha_forward(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    const AlphaShape sh = alpha_shape(net, prop);
    switch (sh.nc) {
#define SLR_F(C) case C: return launch_fwd_nc<C>(net, prop, a, sh, stream);
        SLR_ALPHA_NC(SLR_F)
#undef SLR_F
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_alpha_backward(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                 hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    const AlphaShape sh = alpha_shape(net, prop);
    switch (sh.nc) {
#define SLR_B(C) case C: return launch_bwd_nc<C>(net, prop, a, sh, stream);
        SLR_ALPHA_NC(SLR_B)
#undef SLR_B
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_alpha_optimize(const NetDev& net, const PropDev& prop, const AlphaArgs& a,
                                 int steps, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    const AlphaShape sh = alpha_shape(net, prop);
    switch (sh.nc) {
#define SLR_O(C) case C: return launch_opt_nc<C>(net, prop, a, steps, sh, stream);
        SLR_ALPHA_NC(SLR_O)
#undef SLR_O
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_center_objective(const NetDev& net, const PropDev& prop, int64_t n,
                                   const float* lo, const float* hi, int8_t* obj,
                                   hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = n < 8192 ? n : 8192;
    (void)hipGetLastError();
    hipLaunchKernelGGL(center_obj_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, net, prop, n,
                       lo, hi, obj);
    return hipGetLastError();
}

hipError_t launch_collect_undecided(int64_t n, const int8_t* cls, unsigned* list, unsigned* count,
                                    hipStream_t stream, const float* g_lo, const float* g_hi,
                                    int rows, float select, unsigned* total) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(collect_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n,
                       cls, list, count, g_lo, g_hi, rows, select, total);
    return hipGetLastError();
}

hipError_t launch_gather_boxes(int64_t m, int d, const unsigned* list, const float* lo,
                               const float* hi, float* lo2, float* hi2, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, stream,
                       m, d, list, lo, hi, lo2, hi2);
    return hipGetLastError();
}

hipError_t launch_scatter_classes(int64_t m, const unsigned* list, const int8_t* cls2, int8_t* cls,
                                  hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, m,
                       list, cls2, cls);
    return hipGetLastError();
}

hipError_t launch_ambiguity(int64_t n, int rows, const float* wlo, const float* whi,
                            const float* rlo, const float* rhi, int8_t* cls, unsigned* amb_list,
                            unsigned* amb_count, unsigned base, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(ambiguity_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n,
                       rows, wlo, whi, rlo, rhi, cls, amb_list, amb_count, base);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Batched alpha pass: kernel templates per alpha class
// ---------------------------------------------------------------------------------------------
int batch_alpha_key(const NetDev& net, const PropDev& prop, size_t* lds) {
    const AlphaShape sh = alpha_shape(net, prop);
    if (sh.nc < 0 || sh.nc > 14) return -1;
    const int gs = sh.global_state;
    const int rpf = (!gs && sh.nc <= 8 && sh.reg_path) ? 1 : 0;
    const int rpb = (rpf && sh.nc <= 6 && sh.reg_path_bwd) ? 1 : 0;
    if (!gs && sh.nc > 11) return -1;
    *lds = sh.lds_fwd > sh.lds_bwd ? sh.lds_fwd : sh.lds_bwd;
    return ((sh.nc * 2 + gs) * 2 + rpf) * 2 + rpb;
}

namespace {
const void* batch_opt_ptr(int key) {
#define SLR_K(NC, GS, RPF, RPB)                                                          \
    if (key == (((NC) * 2 + (GS)) * 2 + (RPF)) * 2 + (RPB))                              \
        return (const void*)batch_alpha_opt_kernel<NC, (GS) != 0, (RPF) != 0, (RPB) != 0>;
    SLR_K(3, 1, 0, 0) SLR_K(3, 0, 0, 0) SLR_K(3, 0, 1, 0) SLR_K(3, 0, 1, 1)
    SLR_K(4, 1, 0, 0) SLR_K(4, 0, 0, 0) SLR_K(4, 0, 1, 0) SLR_K(4, 0, 1, 1)
    SLR_K(6, 1, 0, 0) SLR_K(6, 0, 0, 0) SLR_K(6, 0, 1, 0) SLR_K(6, 0, 1, 1)
    SLR_K(8, 1, 0, 0) SLR_K(8, 0, 0, 0) SLR_K(8, 0, 1, 0)
    SLR_K(11, 1, 0, 0) SLR_K(11, 0, 0, 0)
    SLR_K(14, 1, 0, 0)
#undef SLR_K
    return nullptr;
}
}  // namespace

hipError_t batch_alpha_prepare(int key, size_t lds) {
    const void* k = batch_opt_ptr(key);
    if (!k) return hipErrorInvalidValue;
    return allow_lds_a(k, lds);
}

hipError_t launch_batch_alpha_class(int key, size_t lds, BatchInst* insts, BatchCtl* ctl, int c,
                                    const BatchAlphaBuf& buf, const AlphaArgs& base, int steps,
                                    hipStream_t stream) {
    const void* k = batch_opt_ptr(key);
    if (!k) return hipErrorInvalidValue;
    const unsigned tiles = buf.cap / 16;
    (void)hipGetLastError();
    hipLaunchKernelGGL(batch_center_kernel, dim3(tiles * 16 < 4096 ? tiles * 16 : 4096), dim3(256), 0,
                       stream, (const BatchInst*)insts, (const BatchCtl*)ctl, c, buf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const BatchInst* ci = insts;
    const BatchCtl* cc = ctl;
    BatchAlphaBuf b = buf;
    AlphaArgs a = base;
    int st = steps;
    void* args[] = {(void*)&ci, (void*)&cc, &c, &b, &a, &st};
    e = hipLaunchKernel(k, dim3(tiles), dim3(kNW * 64), args, lds, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_scatter_kernel, dim3(tiles * 16 / 256 + 1), dim3(256), 0, stream, insts,
                       (const BatchCtl*)ctl, c, buf);
    return hipGetLastError();
}
