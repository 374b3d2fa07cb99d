// Host engine of the SLR counter: validation, device-resident networks and properties, the
// level driver of the exact count (Alg. 1) and the approximate count built on it.
#include "../../include/slrcount.h"
#include "slr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SLR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

constexpr double kKappa = 2.0;   // safety factor on the rounding-error bounds

double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

// float32 value >= x
float round_up_f32(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Relabeling of one hidden layer of n neurons: row (padded index 16 mt + 4 g + v) of neuron i.
// Full tiles keep the order; the last tile (r neurons) fills rows v-major: t = 4 v + g.
std::vector<int> rows_to_neurons(int n) {
    const int mt = ceil_div(n, 16);
    const int r = n - 16 * (mt - 1);
    std::vector<int> at(16 * mt, -1);
    for (int i = 0; i < n; ++i) {
        if (i < 16 * (mt - 1)) {
            at[i] = i;
        } else {
            const int t = i - 16 * (mt - 1);
            const int v = t / 4, g = t % 4;
            at[16 * (mt - 1) + 4 * g + v] = i;
        }
    }
    (void)r;
    return at;
}

// K-steps that carry at least one real input neuron: 4 (tiles - 1) + ceil(r / 4).
int k_steps(int n_in) {
    const int mt = ceil_div(n_in, 16);
    const int r = n_in - 16 * (mt - 1);
    return 4 * (mt - 1) + (r + 3) / 4;
}

// MFMA A-operand fragments: frag[mt][s][lane] = W[out_at[16 mt + lane % 16]][in_at[k]] with
// k = 16 (s / 4) + 4 (lane / 16) + s % 4 the padded input row (zero where either is padding).
// out_at / in_at map padded rows to neurons (-1 = padding); W is row-major [n_out][n_in].
std::vector<float> pack_fragments(const float* W, int n_in, const std::vector<int>& out_at,
                                  const std::vector<int>& in_at, int ks, int ks_alloc) {
    const int mt_out = (int)out_at.size() / 16;
    std::vector<float> f((size_t)mt_out * ks_alloc * 64, 0.f);
    for (int mt = 0; mt < mt_out; ++mt)
        for (int s = 0; s < ks; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = out_at[16 * mt + lane % 16];
                const int kk = 16 * (s / 4) + 4 * (lane / 16) + s % 4;
                const int k = kk < (int)in_at.size() ? in_at[kk] : -1;
                if (row >= 0 && k >= 0)
                    f[((size_t)mt * ks_alloc + s) * 64 + lane] = W[(size_t)row * n_in + k];
            }
    return f;
}

// bf16 value >= |x| (x finite): the upper half of the float32 bits, rounded up.
uint16_t bf16_abs_up(float x) {
    uint32_t u;
    const float a = std::fabs(x);
    memcpy(&u, &a, 4);
    return (uint16_t)((u + 0xFFFFu) >> 16);
}

// The margin column's A operand: for each (tile, K-quad, lane) the four |W| values of K-steps
// 4 qb .. 4 qb + 3 of the float32 fragments, as bf16 rounded up, packed low to high.
std::vector<uint64_t> pack_quads_bf16(const std::vector<float>& frag, int tiles, int ks_alloc) {
    const int nq = ks_alloc / 4;
    std::vector<uint64_t> q((size_t)tiles * nq * 64, 0);
    for (int mt = 0; mt < tiles; ++mt)
        for (int qb = 0; qb < nq; ++qb)
            for (int lane = 0; lane < 64; ++lane) {
                uint64_t v = 0;
                for (int i = 0; i < 4; ++i)
                    v |= (uint64_t)bf16_abs_up(frag[((size_t)mt * ks_alloc + 4 * qb + i) * 64 + lane]) << (16 * i);
                q[((size_t)mt * nq + qb) * 64 + lane] = v;
            }
    return q;
}

bool all_finite(const float* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
           a.type == hipMemoryTypeUnified;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of multiply-xor on a
// 128-bit counter under a 64-bit key bumped by the Weyl constants between rounds.
struct Philox {
    static void block(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
        uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
        uint32_t k0 = key_in[0], k1 = key_in[1];
        for (int r = 0; r < 10; ++r) {
            if (r > 0) {
                k0 += 0x9E3779B9u;
                k1 += 0xBB67AE85u;
            }
            const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
            const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
            const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
            const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
            const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
            c0 = n0;
            c1 = lo1;
            c2 = n2;
            c3 = lo0;
        }
        out[0] = c0;
        out[1] = c1;
        out[2] = c2;
        out[3] = c3;
    }
    static double u53(uint32_t a, uint32_t b) {
        return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) / 9007199254740992.0;
    }
};

constexpr uint32_t kTagSample = 1, kTagSplit = 2;

}  // namespace

// ------------------------------------------------------------------------------------------
// Network and property handles
// ------------------------------------------------------------------------------------------
struct slr_net {
    NetDev dev{};
    void* mem = nullptr;
    int n_affine = 0;
    std::vector<int> sizes;
    std::vector<double> WL, bL;   // last affine layer in float64 (for property folding)
    std::vector<int> last_at;     // relabeling of the last hidden layer (padded row -> neuron)
};

struct slr_property {
    PropDev dev{};
    void* mem = nullptr;
    const slr_net* net = nullptr;
    int rows = 0;
};

extern "C" const char* last_error(void) { return g_err.c_str(); }

extern "C" int load_net(int32_t n_affine, const int32_t* sizes, const float* const* W,
                        const float* const* b, slr_net** out) {
    return load_net_act(n_affine, sizes, W, b, SLR_ACT_RELU, out);
}

extern "C" int load_net_act(int32_t n_affine, const int32_t* sizes, const float* const* W,
                            const float* const* b, int32_t act, slr_net** out) {
    g_err.clear();
    if (!out) return fail(SLR_EINVAL, "load_net: out is NULL");
    *out = nullptr;
    if (act != SLR_ACT_RELU && act != SLR_ACT_TANH && act != SLR_ACT_SIGMOID)
        return fail(SLR_EINVAL, "load_net: unknown activation %d", act);
    if (n_affine < 2 || n_affine > SLR_MAX_AFFINE)
        return fail(SLR_EINVAL, "load_net: n_affine must be in [2, %d], got %d", SLR_MAX_AFFINE, n_affine);
    if (!sizes || !W || !b) return fail(SLR_EINVAL, "load_net: NULL array");
    const int d = sizes[0];
    if (d < 1 || d > SLR_MAX_D) return fail(SLR_EINVAL, "load_net: input dimension %d not in [1, %d]", d, SLR_MAX_D);
    for (int l = 1; l < n_affine; ++l)
        if (sizes[l] < 1 || sizes[l] > SLR_MAX_WIDTH)
            return fail(SLR_EINVAL, "load_net: hidden width %d not in [1, %d]", sizes[l], SLR_MAX_WIDTH);
    if (sizes[n_affine] < 1 || sizes[n_affine] > SLR_MAX_OUT)
        return fail(SLR_EINVAL, "load_net: output width %d not in [1, %d]", sizes[n_affine], SLR_MAX_OUT);
    for (int l = 0; l < n_affine; ++l) {
        if (!W[l] || !b[l]) return fail(SLR_EINVAL, "load_net: layer %d has a NULL array", l);
        if (!all_finite(W[l], (size_t)sizes[l + 1] * sizes[l]) || !all_finite(b[l], sizes[l + 1]))
            return fail(SLR_EINVAL, "load_net: layer %d has a NaN or Inf", l);
    }

    // host images of every device array, then one allocation
    std::vector<std::vector<char>> blobs;
    auto add = [&](const void* p, size_t bytes) {
        blobs.emplace_back((const char*)p, (const char*)p + bytes);
        return blobs.size() - 1;
    };
    NetDev nd{};
    nd.act = act;
    nd.d = d;
    nd.n_affine = n_affine;
    nd.n1 = sizes[1];
    nd.mt1 = ceil_div(sizes[1], 16);
    nd.n_last = sizes[n_affine - 1];
    nd.mt_last = ceil_div(nd.n_last, 16);
    nd.mt_max = 0;
    nd.n_max = 0;
    nd.frag_total = 0;
    for (int l = 1; l < n_affine; ++l) {
        nd.mt_max = std::max(nd.mt_max, ceil_div(sizes[l], 16));
        nd.n_max = std::max(nd.n_max, sizes[l]);
    }
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    nd.kfirst = round_up_f32(kKappa * gamma_n(d + 2, u32));
    nd.kconc = round_up_f32(kKappa * gamma_n(d + 3, u32));
    nd.krelu = round_up_f32(kKappa * gamma_n(4, u32));
    nd.kfirst64 = kKappa * gamma_n(d + 2, u64) * (1 + 1e-12);
    nd.kconc64 = kKappa * gamma_n(d + 3, u64) * (1 + 1e-12);
    nd.krelu64 = kKappa * gamma_n(4, u64) * (1 + 1e-12);

    const size_t i_w1 = add(W[0], sizeof(float) * sizes[1] * d);
    const size_t i_b1 = add(b[0], sizeof(float) * sizes[1]);
    std::vector<std::vector<int>> at(n_affine - 1);
    for (int h = 0; h < n_affine - 1; ++h) at[h] = rows_to_neurons(sizes[h + 1]);
    nd.r1 = sizes[1] - 16 * (nd.mt1 - 1);
    std::vector<float> w1p((size_t)16 * nd.mt1 * d, 0.f), b1p(16 * nd.mt1, 0.f);
    for (int row = 0; row < 16 * nd.mt1; ++row) {
        const int i = at[0][row];
        if (i < 0) continue;
        b1p[row] = b[0][i];
        for (int k = 0; k < d; ++k) w1p[(size_t)row * d + k] = W[0][(size_t)i * d + k];
    }
    const size_t i_w1p = add(w1p.data(), w1p.size() * sizeof(float));
    const size_t i_b1p = add(b1p.data(), b1p.size() * sizeof(float));
    // alpha mode: row -> neuron maps and slope offsets of the hidden layers
    std::vector<size_t> i_rowmap(n_affine - 1);
    nd.nh = 0;
    for (int h = 0; h < n_affine - 1; ++h) {
        i_rowmap[h] = add(at[h].data(), at[h].size() * sizeof(int));
        nd.hoff[h] = nd.nh;
        nd.nh += sizes[h + 1];
    }
    struct MidIdx { size_t frag, w, wt, bias, absrow, b, wtfrag, qfrag; };
    std::vector<MidIdx> mids;
    for (int l = 1; l <= n_affine - 2; ++l) {
        const int n_in = sizes[l], n_out = sizes[l + 1];
        MidLayer& L = nd.mid[l - 1];
        L.n_in = n_in;
        L.n_out = n_out;
        L.mt_out = ceil_div(n_out, 16);
        L.ks = k_steps(n_in);
        L.r_out = n_out - 16 * (L.mt_out - 1);
        L.ks_alloc = (L.ks + 3) / 4 * 4;
        L.frag_off = nd.frag_total;
        nd.frag_total += L.mt_out * L.ks_alloc * 64;
        L.kgam = round_up_f32(kKappa * gamma_n(n_in + 2, u32));
        L.kgam64 = kKappa * gamma_n(n_in + 2, u64) * (1 + 1e-12);
        std::vector<float> frag = pack_fragments(W[l], n_in, at[l], at[l - 1], L.ks, L.ks_alloc);
        std::vector<float> bias(16 * L.mt_out, 0.f), absrow(16 * L.mt_out, 0.f);
        for (int row = 0; row < 16 * L.mt_out; ++row) {
            const int jrow = at[l][row];
            if (jrow < 0) continue;
            bias[row] = b[l][jrow];
            double s = 0;
            for (int k = 0; k < n_in; ++k) s += std::fabs((double)W[l][(size_t)jrow * n_in + k]);
            absrow[row] = round_up_f32(s * (1 + 1e-12));
        }
        MidIdx mi;
        mi.frag = add(frag.data(), frag.size() * sizeof(float));
        std::vector<uint64_t> qfrag = pack_quads_bf16(frag, L.mt_out, L.ks_alloc);
        mi.qfrag = add(qfrag.data(), qfrag.size() * sizeof(uint64_t));
        mi.w = add(W[l], sizeof(float) * n_out * n_in);
        std::vector<float> wt((size_t)n_in * n_out);
        for (int jrow = 0; jrow < n_out; ++jrow)
            for (int k = 0; k < n_in; ++k) wt[(size_t)k * n_out + jrow] = W[l][(size_t)jrow * n_in + k];
        mi.wt = add(wt.data(), wt.size() * sizeof(float));
        mi.bias = add(bias.data(), bias.size() * sizeof(float));
        mi.absrow = add(absrow.data(), absrow.size() * sizeof(float));
        mi.b = add(b[l], sizeof(float) * n_out);
        // W^T fragments for the alpha adjoint: output rows = this layer's inputs
        L.mt_in = ceil_div(n_in, 16);
        L.kst = k_steps(n_out);
        L.kst_alloc = (L.kst + 3) / 4 * 4;
        std::vector<float> tfrag = pack_fragments(wt.data(), n_out, at[l - 1], at[l], L.kst, L.kst_alloc);
        mi.wtfrag = add(tfrag.data(), tfrag.size() * sizeof(float));
        mids.push_back(mi);
    }
    std::vector<size_t> offs(blobs.size());
    size_t total = 0;
    for (size_t i = 0; i < blobs.size(); ++i) {
        offs[i] = total;
        total += (blobs[i].size() + 255) / 256 * 256;
    }
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) return fail(SLR_ENOMEM, "load_net: hipMalloc(%zu): %s", total, hipGetErrorString(e));
    std::vector<char> host(total, 0);
    for (size_t i = 0; i < blobs.size(); ++i) memcpy(host.data() + offs[i], blobs[i].data(), blobs[i].size());
    e = hipMemcpy(mem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "load_net: upload");
    }
    char* base = (char*)mem;
    nd.w1 = (const float*)(base + offs[i_w1]);
    nd.b1 = (const float*)(base + offs[i_b1]);
    nd.w1p = (const float*)(base + offs[i_w1p]);
    nd.b1p = (const float*)(base + offs[i_b1p]);
    for (int l = 0; l < n_affine - 2; ++l) {
        nd.mid[l].wfrag = (const float*)(base + offs[mids[l].frag]);
        nd.mid[l].w = (const float*)(base + offs[mids[l].w]);
        nd.mid[l].wt = (const float*)(base + offs[mids[l].wt]);
        nd.mid[l].bias = (const float*)(base + offs[mids[l].bias]);
        nd.mid[l].absrow = (const float*)(base + offs[mids[l].absrow]);
        nd.mid[l].b = (const float*)(base + offs[mids[l].b]);
        nd.mid[l].wtfrag = (const float*)(base + offs[mids[l].wtfrag]);
        nd.mid[l].qfrag = (const uint64_t*)(base + offs[mids[l].qfrag]);
    }
    for (int h = 0; h < n_affine - 1; ++h) nd.rowmap[h] = (const int*)(base + offs[i_rowmap[h]]);
    slr_net* net = new slr_net;
    net->dev = nd;
    net->mem = mem;
    net->n_affine = n_affine;
    net->sizes.assign(sizes, sizes + n_affine + 1);
    const int nL = sizes[n_affine], kL = sizes[n_affine - 1];
    net->WL.resize((size_t)nL * kL);
    net->bL.resize(nL);
    for (size_t i = 0; i < net->WL.size(); ++i) net->WL[i] = W[n_affine - 1][i];
    for (int i = 0; i < nL; ++i) net->bL[i] = b[n_affine - 1][i];
    net->last_at = at[n_affine - 2];
    *out = net;
    return SLR_OK;
}

extern "C" void free_net(slr_net* net) {
    if (!net) return;
    (void)hipFree(net->mem);
    delete net;
}

extern "C" int load_property(const slr_net* net, int32_t rows, const float* C, const float* dv,
                             slr_property** out) {
    g_err.clear();
    if (!out) return fail(SLR_EINVAL, "load_property: out is NULL");
    *out = nullptr;
    if (!net) return fail(SLR_EINVAL, "load_property: net is NULL");
    if (rows < 1 || rows > SLR_MAX_ROWS) return fail(SLR_EINVAL, "load_property: rows %d not in [1, %d]", rows, SLR_MAX_ROWS);
    if (!C || !dv) return fail(SLR_EINVAL, "load_property: NULL array");
    const int n_out = net->sizes[net->n_affine];
    const int K = net->sizes[net->n_affine - 1];
    if (!all_finite(C, (size_t)rows * n_out) || !all_finite(dv, rows))
        return fail(SLR_EINVAL, "load_property: NaN or Inf in C or d");
    std::vector<double> wg64((size_t)rows * K), bg64(rows), ag64(rows);
    std::vector<float> wg((size_t)rows * K), bg(rows), ag(rows);
    for (int r = 0; r < rows; ++r) {
        double bsum = dv[r];
        double asum = 0;
        for (int o = 0; o < n_out; ++o) bsum += (double)C[r * n_out + o] * net->bL[o];
        for (int k = 0; k < K; ++k) {
            double s = 0, sa = 0;
            for (int o = 0; o < n_out; ++o) {
                s += (double)C[r * n_out + o] * net->WL[(size_t)o * K + k];
                sa += std::fabs((double)C[r * n_out + o]) * std::fabs(net->WL[(size_t)o * K + k]);
            }
            wg64[(size_t)r * K + k] = s;
            wg[(size_t)r * K + k] = (float)s;
            asum += sa;
        }
        bg64[r] = bsum;
        bg[r] = (float)bsum;
        ag64[r] = asum * (1 + 1e-12);
        ag[r] = round_up_f32(asum * (1 + 1e-12));
    }
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    PropDev pd{};
    pd.rows = rows;
    pd.n_last = K;
    pd.kout = round_up_f32(kKappa * gamma_n(K + 3, u32));
    pd.kout64 = kKappa * gamma_n(K + n_out + 3, u64) * (1 + 1e-12);
    pd.ks_out = k_steps(K);
    pd.ks_out_alloc = (pd.ks_out + 3) / 4 * 4;
    std::vector<int> row_at(16, -1);
    for (int r = 0; r < rows; ++r) row_at[r] = r;
    std::vector<float> wgfrag = pack_fragments(wg.data(), K, row_at, net->last_at, pd.ks_out, pd.ks_out_alloc);
    std::vector<uint64_t> wgq = pack_quads_bf16(wgfrag, 1, pd.ks_out_alloc);
    pd.kpad = (int)net->last_at.size();
    std::vector<float> wgp((size_t)rows * pd.kpad, 0.f);
    for (int r = 0; r < rows; ++r)
        for (int kk = 0; kk < pd.kpad; ++kk)
            if (net->last_at[kk] >= 0) wgp[(size_t)r * pd.kpad + kk] = wg[(size_t)r * K + net->last_at[kk]];
    // alpha mode: relabeled property rows (tile row 4 g + v = property row 4 v + g) and W_g^T
    const std::vector<int> rat = rows_to_neurons(rows);
    std::vector<int> rat16(16, -1);
    for (size_t i = 0; i < rat.size() && i < 16; ++i) rat16[i] = rat[i];
    std::vector<float> wgfrag_a = pack_fragments(wg.data(), K, rat16, net->last_at, pd.ks_out, pd.ks_out_alloc);
    std::vector<float> wgT((size_t)K * rows);
    for (int r = 0; r < rows; ++r)
        for (int k = 0; k < K; ++k) wgT[(size_t)k * rows + r] = wg[(size_t)r * K + k];
    pd.ks_rows = k_steps(rows);
    pd.ks_rows_alloc = (pd.ks_rows + 3) / 4 * 4;
    std::vector<float> wgtfrag = pack_fragments(wgT.data(), rows, net->last_at, rat16, pd.ks_rows, pd.ks_rows_alloc);
    std::vector<float> bga(16, 0.f), aga(16, 0.f);
    for (int i = 0; i < 16; ++i)
        if (rat16[i] >= 0) {
            bga[i] = bg[rat16[i]];
            aga[i] = ag[rat16[i]];
        }
    const size_t s_fa = (wgfrag_a.size() * 4 + 255) / 256 * 256;
    const size_t s_ft = (wgtfrag.size() * 4 + 255) / 256 * 256;
    const size_t s_16 = 256;
    const size_t s_q = (wgq.size() * 8 + 255) / 256 * 256;
    const size_t s_wgp = (wgp.size() * 4 + 255) / 256 * 256;
    const size_t s_wg = (wg.size() * 4 + 255) / 256 * 256, s_r = (rows * 4 + 255) / 256 * 256;
    const size_t s_frag = (wgfrag.size() * 4 + 255) / 256 * 256;
    const size_t s_wg64 = (wg64.size() * 8 + 255) / 256 * 256, s_r64 = (rows * 8 + 255) / 256 * 256;
    const size_t total = s_wg + 2 * s_r + s_wg64 + 2 * s_r64 + s_frag + s_wgp + s_fa + s_ft + 2 * s_16 + s_q;
    std::vector<char> host(total, 0);
    size_t o = 0;
    memcpy(host.data() + o, wg.data(), wg.size() * 4);
    const size_t o_wg = o; o += s_wg;
    memcpy(host.data() + o, bg.data(), rows * 4);
    const size_t o_bg = o; o += s_r;
    memcpy(host.data() + o, ag.data(), rows * 4);
    const size_t o_ag = o; o += s_r;
    memcpy(host.data() + o, wg64.data(), wg64.size() * 8);
    const size_t o_wg64 = o; o += s_wg64;
    memcpy(host.data() + o, bg64.data(), rows * 8);
    const size_t o_bg64 = o; o += s_r64;
    memcpy(host.data() + o, ag64.data(), rows * 8);
    const size_t o_ag64 = o; o += s_r64;
    memcpy(host.data() + o, wgfrag.data(), wgfrag.size() * 4);
    const size_t o_frag = o; o += s_frag;
    memcpy(host.data() + o, wgp.data(), wgp.size() * 4);
    const size_t o_wgp = o; o += s_wgp;
    memcpy(host.data() + o, wgfrag_a.data(), wgfrag_a.size() * 4);
    const size_t o_fa = o; o += s_fa;
    memcpy(host.data() + o, wgtfrag.data(), wgtfrag.size() * 4);
    const size_t o_ft = o; o += s_ft;
    memcpy(host.data() + o, bga.data(), 64);
    const size_t o_bga = o; o += s_16;
    memcpy(host.data() + o, aga.data(), 64);
    const size_t o_aga = o; o += s_16;
    memcpy(host.data() + o, wgq.data(), wgq.size() * 8);
    const size_t o_q = o;
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) return fail(SLR_ENOMEM, "load_property: hipMalloc: %s", hipGetErrorString(e));
    e = hipMemcpy(mem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "load_property: upload");
    }
    char* base = (char*)mem;
    pd.wg = (const float*)(base + o_wg);
    pd.bg = (const float*)(base + o_bg);
    pd.ag = (const float*)(base + o_ag);
    pd.wg64 = (const double*)(base + o_wg64);
    pd.bg64 = (const double*)(base + o_bg64);
    pd.ag64 = (const double*)(base + o_ag64);
    pd.wgfrag = (const float*)(base + o_frag);
    pd.wgp = (const float*)(base + o_wgp);
    pd.wgfrag_a = (const float*)(base + o_fa);
    pd.wgtfrag = (const float*)(base + o_ft);
    pd.bga = (const float*)(base + o_bga);
    pd.aga = (const float*)(base + o_aga);
    pd.wgqfrag = (const uint64_t*)(base + o_q);
    slr_property* p = new slr_property;
    p->dev = pd;
    p->mem = mem;
    p->net = net;
    p->rows = rows;
    *out = p;
    return SLR_OK;
}

extern "C" void free_property(slr_property* prop) {
    if (!prop) return;
    (void)hipFree(prop->mem);
    delete prop;
}

// ------------------------------------------------------------------------------------------
// Workspace layout of the exact count (all regions 256-byte aligned)
// ------------------------------------------------------------------------------------------
namespace {

constexpr int kMaxLevels = 63;

struct Workspace {
    float *lo[2], *hi[2];
    unsigned long long* path[2];
    int8_t* cls;
    int8_t* dimsel;              // [cap] side to bisect (crossing-score split rule)
    unsigned* amb_list;          // [cap] boxes of the level that need the FP64 re-decision
    unsigned* amb_count;
    unsigned* tile_und;
    LevelStats* stats;           // [kMaxLevels]
    double* vol;                 // [3]
    unsigned long long* counts;  // [3]
    unsigned long long* rechecks;
    unsigned* err;               // [kMaxLevels + 1]: per-level split errors, then the volume check
    float* samples;              // [samples][d]
    int8_t* viol;                // [samples]
    // alpha batches of up to achunk boxes
    int64_t achunk;
    float *alo, *ahi;            // [achunk][d] gathered undecided boxes
    float *best_lo, *best_hi;    // [achunk][rows]
    float *glo, *ghi;            // [cap][rows] plain bounds of a level (alpha candidate selection)
    int8_t* acls;                // [achunk]
    char* aws;                   // alpha_optimize workspace for achunk boxes
    size_t aws_bytes;
    // shapes the LDS bound kernel cannot hold: plain bounds from the tape-state kernel in
    // batches of wchunk boxes (forward-only tape, widened and raw bounds)
    int64_t wchunk;
    float* wtape;
    float *wlo, *whi, *rlo, *rhi;   // [wchunk][rows]
    size_t bytes;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of alpha_optimize for n boxes.
struct AlphaWs {
    float* tape;
    float *m, *v, *alpha;        // [n][nh]
    float *g_lo, *g_hi;          // [n][rows]
    int8_t* obj;                 // [n][2]
    size_t tape_bytes, bytes;
};

AlphaWs layout_alpha(char* base, const NetDev& nd, const PropDev& pd, int64_t n) {
    AlphaWs w{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    w.tape_bytes = alpha_tape_bytes(nd, pd, n, 0);
    w.tape = (float*)take(w.tape_bytes);
    w.m = (float*)take(sizeof(float) * (size_t)n * nd.nh);
    w.v = (float*)take(sizeof(float) * (size_t)n * nd.nh);
    w.alpha = (float*)take(sizeof(float) * (size_t)n * nd.nh);
    w.g_lo = (float*)take(sizeof(float) * (size_t)n * pd.rows);
    w.g_hi = (float*)take(sizeof(float) * (size_t)n * pd.rows);
    w.obj = (int8_t*)take((size_t)2 * n);
    w.bytes = o;
    return w;
}

// tape_state: plain bounds from the tape-state kernel whatever the shape (the relaxation with one
// ratio per equation needs its full per-neuron equations)
// Boxes per launch of the tape-state kernel: as many as keep its tape within 128 MiB (at least
// 4096, at most 65536, a multiple of 4096; small_tape: 4096, for the static scratch of the
// allocation-free count).  Larger launches fill the GPU where one 4096-box launch is a single
// wave of tiles.
int64_t tape_chunk(const NetDev& nd, const PropDev& pd, bool small_tape) {
    if (small_tape) return 4096;
    const size_t per_tile = alpha_tape_bytes(nd, pd, 16, 1);
    const int64_t fit = per_tile > 0 ? (int64_t)((size_t)(128 << 20) / per_tile) * 16 : 65536;
    return std::max<int64_t>(4096, std::min<int64_t>(65536, fit / 4096 * 4096));
}

Workspace layout_ws(char* base, const NetDev& nd, const PropDev& pd, int64_t cap, int samples,
                    int64_t achunk, bool tape_state = false, bool small_tape = false) {
    const int d = nd.d;
    Workspace w{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    for (int s = 0; s < 2; ++s) {
        w.lo[s] = (float*)take(sizeof(float) * d * cap);
        w.hi[s] = (float*)take(sizeof(float) * d * cap);
        w.path[s] = (unsigned long long*)take(sizeof(unsigned long long) * cap);
    }
    w.cls = (int8_t*)take(cap);
    w.dimsel = (int8_t*)take(cap);
    w.amb_list = (unsigned*)take(sizeof(unsigned) * cap);
    w.amb_count = (unsigned*)take(2 * sizeof(unsigned));   // [1]: all undecided (alpha pass)
    w.tile_und = (unsigned*)take(sizeof(unsigned) * level_tiles(cap));
    w.stats = (LevelStats*)take(sizeof(LevelStats) * kMaxLevels);
    w.vol = (double*)take(sizeof(double) * 3);
    w.counts = (unsigned long long*)take(sizeof(unsigned long long) * 3);
    w.rechecks = (unsigned long long*)take(sizeof(unsigned long long));
    w.err = (unsigned*)take(sizeof(unsigned) * (kMaxLevels + 1));
    w.samples = (float*)take(sizeof(float) * (size_t)d * std::max(samples, 0));
    w.viol = (int8_t*)take(std::max(samples, 0));
    w.wchunk = 0;
    if ((tape_state || !bound_f32_supported(nd, pd)) && pd.rows > 0) {
        w.wchunk = std::min<int64_t>(cap, tape_chunk(nd, pd, small_tape));
        w.wtape = (float*)take(alpha_tape_bytes(nd, pd, w.wchunk, 1));
        w.wlo = (float*)take(sizeof(float) * pd.rows * w.wchunk);
        w.whi = (float*)take(sizeof(float) * pd.rows * w.wchunk);
        w.rlo = (float*)take(sizeof(float) * pd.rows * w.wchunk);
        w.rhi = (float*)take(sizeof(float) * pd.rows * w.wchunk);
    }
    w.achunk = achunk;
    if (achunk > 0) {
        w.alo = (float*)take(sizeof(float) * d * achunk);
        w.ahi = (float*)take(sizeof(float) * d * achunk);
        w.best_lo = (float*)take(sizeof(float) * pd.rows * achunk);
        w.best_hi = (float*)take(sizeof(float) * pd.rows * achunk);
        w.glo = (float*)take(sizeof(float) * pd.rows * cap);
        w.ghi = (float*)take(sizeof(float) * pd.rows * cap);
        w.acls = (int8_t*)take(achunk);
        w.aws_bytes = layout_alpha(nullptr, nd, pd, achunk).bytes;
        w.aws = take(w.aws_bytes);
    }
    w.bytes = o;
    return w;
}

// need_lds: the call runs the LDS bound kernel itself (otherwise wide shapes take the
// tape-state kernel)
int check_pair(const slr_net* net, const slr_property* prop, const char* who, bool need_lds = false) {
    if (!net) return fail(SLR_EINVAL, "%s: net is NULL", who);
    if (!prop) return fail(SLR_EINVAL, "%s: property is NULL", who);
    if (prop->net != net) return fail(SLR_EINVAL, "%s: property was loaded for another net", who);
    if (need_lds && !bound_f32_supported(net->dev, prop->dev))
        return fail(SLR_EUNSUPPORTED, "%s: network shape (d=%d, widths up to %d) exceeds the LDS bound kernel; "
                    "use bound_boxes_alpha (alpha = NULL) or count_exact", who, net->dev.d, net->dev.n_max);
    return SLR_OK;
}

int check_box(const slr_net* net, const double* lo, const double* hi, const char* who) {
    if (!lo || !hi) return fail(SLR_EINVAL, "%s: NULL box", who);
    for (int k = 0; k < net->dev.d; ++k) {
        if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]))
            return fail(SLR_EINVAL, "%s: non-finite box corner", who);
        if ((double)(float)lo[k] != lo[k] || (double)(float)hi[k] != hi[k])
            return fail(SLR_EINVAL, "%s: box corner %d is not exactly representable in float32", who, k);
        if (lo[k] > hi[k]) return fail(SLR_EINVAL, "%s: lo > hi in dimension %d", who, k);
    }
    return SLR_OK;
}

}  // namespace

extern "C" int workspace_size(const slr_net* net, const slr_property* prop, int64_t max_leaves,
                              int32_t samples, int32_t alpha_chunk, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(SLR_EINVAL, "workspace_size: bytes is NULL");
    if (!net) return fail(SLR_EINVAL, "workspace_size: net is NULL");
    if (max_leaves < 1) return fail(SLR_EINVAL, "workspace_size: max_leaves must be >= 1");
    if (samples < 0) return fail(SLR_EINVAL, "workspace_size: samples must be >= 0");
    if (alpha_chunk < 0) return fail(SLR_EINVAL, "workspace_size: alpha_chunk must be >= 0");
    if (alpha_chunk > 0 && !prop) return fail(SLR_EINVAL, "workspace_size: alpha mode needs the property");
    PropDev pd{};
    if (prop) pd = prop->dev;
    *bytes = layout_ws(nullptr, net->dev, pd, max_leaves, samples, alpha_chunk).bytes;
    return SLR_OK;
}

extern "C" int workspace_size_exact(const slr_net* net, const slr_property* prop,
                                    const slr_exact_opts* opts, size_t* bytes) {
    g_err.clear();
    if (!bytes || !opts) return fail(SLR_EINVAL, "workspace_size_exact: NULL argument");
    int rc = check_pair(net, prop, "workspace_size_exact");
    if (rc) return rc;
    if (opts->max_leaves < 1) return fail(SLR_EINVAL, "workspace_size_exact: max_leaves must be >= 1");
    if (opts->alpha_steps > 0 && opts->alpha_chunk < 1)
        return fail(SLR_EINVAL, "workspace_size_exact: alpha mode needs alpha_chunk >= 1");
    const int64_t achunk = opts->alpha_steps > 0 ? opts->alpha_chunk : 0;
    *bytes = layout_ws(nullptr, net->dev, prop->dev, opts->max_leaves, 0, achunk,
                       opts->relax == SLR_RELAX_TWO).bytes;
    return SLR_OK;
}

extern "C" int bound_tile_shape(int32_t d, int32_t mt_max, int32_t nt, int32_t uw, int32_t nw) {
    g_err.clear();
    if (set_tile_shape(d, mt_max, TileShape{nt, uw, nw}) != 0)
        return fail(SLR_EINVAL, "bound_tile_shape: (%d, %d, %d) is not an instantiated tile shape covering "
                    "%d hidden tiles for d = %d", nt, uw, nw, mt_max, d);
    return SLR_OK;
}

extern "C" int alpha_state_variant(int32_t variant) {
    g_err.clear();
    if (set_alpha_state_variant(variant) != 0)
        return fail(SLR_EINVAL, "alpha_state_variant: %d is not 0, 1 or 2", variant);
    return SLR_OK;
}

extern "C" int bound_kernel_variant(int32_t variant) {
    g_err.clear();
    if (set_bound_variant(variant) != 0)
        return fail(SLR_EINVAL, "bound_kernel_variant: %d is not 0, 1 or 2", variant);
    return SLR_OK;
}

extern "C" int bound_boxes(const slr_net* net, const slr_property* prop, int64_t n,
                           const float* lo, const float* hi, float* g_lo, float* g_hi,
                           int8_t* cls, int32_t raw, void* stream) {
    g_err.clear();
    int rc = check_pair(net, prop, "bound_boxes", true);
    if (rc) return rc;
    if (n < 0) return fail(SLR_EINVAL, "bound_boxes: n < 0");
    if (raw != 0 && raw != 1) return fail(SLR_EINVAL, "bound_boxes: raw must be 0 or 1");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(lo) || !is_device_ptr(hi) || !is_device_ptr(g_lo) || !is_device_ptr(g_hi))
        return fail(SLR_EINVAL, "bound_boxes: lo, hi, g_lo and g_hi must be device memory");
    if (cls && !is_device_ptr(cls)) return fail(SLR_EINVAL, "bound_boxes: cls must be device memory");
    hipStream_t s = (hipStream_t)stream;
    int unsup = 0;
    HIP_TRY(launch_bound_f32(net->dev, prop->dev, n, lo, hi, g_lo, g_hi, cls, raw, s, &unsup,
                             nullptr, nullptr, 0),
            "bound_boxes: bound kernel");
    if (unsup) return fail(SLR_EUNSUPPORTED, "bound_boxes: shape not supported");
    if (!raw && cls)
        HIP_TRY(launch_recheck64(net->dev, prop->dev, n, lo, hi, g_lo, g_hi, cls, nullptr, nullptr,
                                 nullptr, s),
                "bound_boxes: recheck kernel");
    return SLR_OK;
}

extern "C" int sample_violations(const slr_net* net, const slr_property* prop, int64_t n,
                                 const float* x, int8_t* viol, void* stream) {
    g_err.clear();
    int rc = check_pair(net, prop, "sample_violations");
    if (rc) return rc;
    if (n < 0) return fail(SLR_EINVAL, "sample_violations: n < 0");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(x) || !is_device_ptr(viol))
        return fail(SLR_EINVAL, "sample_violations: x and viol must be device memory");
    HIP_TRY(launch_sample_forward(net->dev, prop->dev, n, x, viol, (hipStream_t)stream),
            "sample_violations: kernel");
    return SLR_OK;
}

// ------------------------------------------------------------------------------------------
// Alpha mode
// ------------------------------------------------------------------------------------------
namespace {

int check_alpha_pair(const slr_net* net, const slr_property* prop, const char* who) {
    if (!net) return fail(SLR_EINVAL, "%s: net is NULL", who);
    if (!prop) return fail(SLR_EINVAL, "%s: property is NULL", who);
    if (prop->net != net) return fail(SLR_EINVAL, "%s: property was loaded for another net", who);
    if (alpha_shape(net->dev, prop->dev).nc < 0) return fail(SLR_EUNSUPPORTED, "%s: input dimension too large", who);
    if (net->dev.act != SLR_ACT_RELU)
        return fail(SLR_EUNSUPPORTED, "%s: alpha slopes are defined for ReLU networks only", who);
    return SLR_OK;
}

// Projected Adam on the slopes of n boxes (init pass + steps x (adjoint with fused update,
// forward)); every forward pass folds its bounds into best_lo / best_hi and classifies.
int alpha_run(const slr_net* net, const slr_property* prop, int64_t n, const float* lo,
              const float* hi, const slr_alpha_opts& o, float* alpha, float* best_lo,
              float* best_hi, int8_t* cls, const AlphaWs& w, hipStream_t s) {
    if (n <= 0) return SLR_OK;
    const NetDev& nd = net->dev;
    const PropDev& pd = prop->dev;
    HIP_TRY(launch_center_objective(nd, pd, n, lo, hi, w.obj, s), "alpha: center kernel");
    AlphaArgs a{};
    a.n = n;
    a.lo = lo;
    a.hi = hi;
    a.alpha = alpha ? alpha : w.alpha;
    a.g_lo = w.g_lo;
    a.g_hi = w.g_hi;
    a.best_lo = best_lo;
    a.best_hi = best_hi;
    a.cls = cls;
    a.tape = w.tape;
    a.raw = o.raw;
    a.obj = w.obj;
    a.adam_m = w.m;
    a.adam_v = w.v;
    a.lr = o.lr;
    a.beta1 = o.beta1;
    a.beta2 = o.beta2;
    a.eps = o.eps;
    if (alpha_fused()) {
        // every tile runs its whole optimization in one launch (init forward, then the steps)
        HIP_TRY(launch_alpha_optimize(nd, pd, a, o.steps, s), "alpha: optimizer kernel");
        return SLR_OK;
    }
    HIP_TRY(hipMemsetAsync(w.m, 0, sizeof(float) * (size_t)n * nd.nh, s), "alpha: clear");
    HIP_TRY(hipMemsetAsync(w.v, 0, sizeof(float) * (size_t)n * nd.nh, s), "alpha: clear");
    a.init = 1;
    AlphaArgs a0 = a;
    a0.obj = nullptr;
    a0.adam_m = a0.adam_v = nullptr;
    HIP_TRY(launch_alpha_forward(nd, pd, a0, s), "alpha: forward kernel");
    a.init = 0;
    double p1 = 1.0, p2 = 1.0;
    for (int t = 1; t <= o.steps; ++t) {
        p1 *= o.beta1;
        p2 *= o.beta2;
        a.c1 = (float)(1.0 / (1.0 - p1));
        a.c2 = (float)(1.0 / (1.0 - p2));
        HIP_TRY(launch_alpha_backward(nd, pd, a, s), "alpha: adjoint kernel");
        HIP_TRY(launch_alpha_forward(nd, pd, a, s), "alpha: forward kernel");
    }
    return SLR_OK;
}

}  // namespace

extern "C" int alpha_kernel_variant(int32_t variant) {
    g_err.clear();
    if (variant != 0 && variant != 1) return fail(SLR_EINVAL, "alpha_kernel_variant: must be 0 or 1");
    set_alpha_fused(variant);
    return SLR_OK;
}

extern "C" int alpha_size(const slr_net* net, int64_t* nh) {
    g_err.clear();
    if (!net || !nh) return fail(SLR_EINVAL, "alpha_size: NULL argument");
    *nh = net->dev.nh;
    return SLR_OK;
}

extern "C" int alpha_tape_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "alpha_tape_size");
    if (rc) return rc;
    if (!bytes || n < 0) return fail(SLR_EINVAL, "alpha_tape_size: bad argument");
    *bytes = alpha_tape_bytes(net->dev, prop->dev, n, 0);
    return SLR_OK;
}

extern "C" int alpha_workspace_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "alpha_workspace_size");
    if (rc) return rc;
    if (!bytes || n < 0) return fail(SLR_EINVAL, "alpha_workspace_size: bad argument");
    *bytes = layout_alpha(nullptr, net->dev, prop->dev, n).bytes;
    return SLR_OK;
}

extern "C" int bound_boxes_alpha(const slr_net* net, const slr_property* prop, int64_t n,
                                 const float* lo, const float* hi, float* alpha, int32_t init,
                                 float* g_lo, float* g_hi, int8_t* cls, int32_t raw, void* tape,
                                 size_t tape_bytes, void* stream) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "bound_boxes_alpha");
    if (rc) return rc;
    if (n < 0) return fail(SLR_EINVAL, "bound_boxes_alpha: n < 0");
    if ((raw != 0 && raw != 1) || (init != 0 && init != 1))
        return fail(SLR_EINVAL, "bound_boxes_alpha: raw and init must be 0 or 1");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(lo) || !is_device_ptr(hi) || !is_device_ptr(g_lo) || !is_device_ptr(g_hi))
        return fail(SLR_EINVAL, "bound_boxes_alpha: lo, hi, g_lo and g_hi must be device memory");
    if ((alpha && !is_device_ptr(alpha)) || (cls && !is_device_ptr(cls)))
        return fail(SLR_EINVAL, "bound_boxes_alpha: alpha and cls must be device memory");
    const size_t need = alpha_tape_bytes(net->dev, prop->dev, n, 0);
    if (!tape || tape_bytes < need)
        return fail(SLR_ENOMEM, "bound_boxes_alpha: tape of %zu bytes is smaller than the %zu required", tape_bytes, need);
    if (!is_device_ptr(tape)) return fail(SLR_EINVAL, "bound_boxes_alpha: tape must be device memory");
    AlphaArgs a{};
    a.n = n;
    a.lo = lo;
    a.hi = hi;
    a.alpha = alpha;
    a.init = init;
    a.g_lo = g_lo;
    a.g_hi = g_hi;
    a.cls = cls;
    a.raw = raw;
    a.tape = (float*)tape;
    HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, (hipStream_t)stream), "bound_boxes_alpha: kernel");
    return SLR_OK;
}

extern "C" int bound_boxes_relax(const slr_net* net, const slr_property* prop, int64_t n,
                                 const float* lo, const float* hi, int32_t relax, float* g_lo,
                                 float* g_hi, int8_t* cls, int32_t raw, void* tape,
                                 size_t tape_bytes, void* stream) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "bound_boxes_relax");
    if (rc) return rc;
    if (n < 0) return fail(SLR_EINVAL, "bound_boxes_relax: n < 0");
    if (raw != 0 && raw != 1) return fail(SLR_EINVAL, "bound_boxes_relax: raw must be 0 or 1");
    if (relax != SLR_RELAX_ONE && relax != SLR_RELAX_TWO)
        return fail(SLR_EINVAL, "bound_boxes_relax: relax must be SLR_RELAX_ONE or SLR_RELAX_TWO");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(lo) || !is_device_ptr(hi) || !is_device_ptr(g_lo) || !is_device_ptr(g_hi))
        return fail(SLR_EINVAL, "bound_boxes_relax: lo, hi, g_lo and g_hi must be device memory");
    if (cls && !is_device_ptr(cls)) return fail(SLR_EINVAL, "bound_boxes_relax: cls must be device memory");
    const size_t need = alpha_tape_bytes(net->dev, prop->dev, n, 1);
    if (!tape || tape_bytes < need)
        return fail(SLR_ENOMEM, "bound_boxes_relax: tape of %zu bytes is smaller than the %zu required", tape_bytes, need);
    if (!is_device_ptr(tape)) return fail(SLR_EINVAL, "bound_boxes_relax: tape must be device memory");
    AlphaArgs a{};
    a.n = n;
    a.lo = lo;
    a.hi = hi;
    a.g_lo = g_lo;
    a.g_hi = g_hi;
    a.cls = cls;
    a.raw = raw;
    a.tape = (float*)tape;
    a.fwd_only = 1;
    a.two_ratio = relax == SLR_RELAX_TWO;
    HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, (hipStream_t)stream), "bound_boxes_relax: kernel");
    return SLR_OK;
}

extern "C" int bound_tape_size(const slr_net* net, const slr_property* prop, int64_t n, size_t* bytes) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "bound_tape_size");
    if (rc) return rc;
    if (!bytes || n < 0) return fail(SLR_EINVAL, "bound_tape_size: bytes is NULL or n < 0");
    *bytes = alpha_tape_bytes(net->dev, prop->dev, n, 1);
    return SLR_OK;
}

extern "C" int bound_boxes_backward(const slr_net* net, const slr_property* prop, int64_t n,
                                    const float* alpha, const void* tape, size_t tape_bytes,
                                    const float* dg_lo, const float* dg_hi, float* dalpha,
                                    int32_t raw, void* stream) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "bound_boxes_backward");
    if (rc) return rc;
    if (n < 0) return fail(SLR_EINVAL, "bound_boxes_backward: n < 0");
    if (raw != 0 && raw != 1) return fail(SLR_EINVAL, "bound_boxes_backward: raw must be 0 or 1");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(dalpha)) return fail(SLR_EINVAL, "bound_boxes_backward: dalpha must be device memory");
    if ((alpha && !is_device_ptr(alpha)) || (dg_lo && !is_device_ptr(dg_lo)) || (dg_hi && !is_device_ptr(dg_hi)))
        return fail(SLR_EINVAL, "bound_boxes_backward: alpha, dg_lo and dg_hi must be device memory");
    const size_t need = alpha_tape_bytes(net->dev, prop->dev, n, 0);
    if (!tape || tape_bytes < need)
        return fail(SLR_ENOMEM, "bound_boxes_backward: tape of %zu bytes is smaller than the %zu required", tape_bytes, need);
    if (!is_device_ptr(tape)) return fail(SLR_EINVAL, "bound_boxes_backward: tape must be device memory");
    AlphaArgs a{};
    a.n = n;
    a.alpha = const_cast<float*>(alpha);   // read only: no Adam state is given
    a.tape = (float*)tape;
    a.raw = raw;
    a.dg_lo = dg_lo;
    a.dg_hi = dg_hi;
    a.dalpha = dalpha;
    HIP_TRY(launch_alpha_backward(net->dev, prop->dev, a, (hipStream_t)stream), "bound_boxes_backward: kernel");
    return SLR_OK;
}

extern "C" int alpha_optimize(const slr_net* net, const slr_property* prop, int64_t n,
                              const float* lo, const float* hi, const slr_alpha_opts* opts,
                              float* alpha, float* best_lo, float* best_hi, int8_t* cls,
                              void* workspace, size_t workspace_bytes, void* stream) {
    g_err.clear();
    int rc = check_alpha_pair(net, prop, "alpha_optimize");
    if (rc) return rc;
    if (!opts) return fail(SLR_EINVAL, "alpha_optimize: opts is NULL");
    if (n < 0) return fail(SLR_EINVAL, "alpha_optimize: n < 0");
    if (opts->steps < 0 || opts->steps > 1000 || !(opts->lr >= 0.f) || !(opts->beta1 >= 0.f && opts->beta1 < 1.f) ||
        !(opts->beta2 >= 0.f && opts->beta2 < 1.f) || !(opts->eps > 0.f) || (opts->raw != 0 && opts->raw != 1))
        return fail(SLR_EINVAL, "alpha_optimize: bad options");
    if (n == 0) return SLR_OK;
    if (!is_device_ptr(lo) || !is_device_ptr(hi) || !is_device_ptr(best_lo) || !is_device_ptr(best_hi))
        return fail(SLR_EINVAL, "alpha_optimize: lo, hi, best_lo and best_hi must be device memory");
    if ((alpha && !is_device_ptr(alpha)) || (cls && !is_device_ptr(cls)))
        return fail(SLR_EINVAL, "alpha_optimize: alpha and cls must be device memory");
    const AlphaWs probe = layout_alpha(nullptr, net->dev, prop->dev, n);
    if (!workspace || workspace_bytes < probe.bytes)
        return fail(SLR_ENOMEM, "alpha_optimize: workspace of %zu bytes is smaller than the %zu required", workspace_bytes, probe.bytes);
    if (!is_device_ptr(workspace)) return fail(SLR_EINVAL, "alpha_optimize: workspace must be device memory");
    const AlphaWs w = layout_alpha((char*)workspace, net->dev, prop->dev, n);
    return alpha_run(net, prop, n, lo, hi, *opts, alpha, best_lo, best_hi, cls, w, (hipStream_t)stream);
}

namespace {

// Pinned host staging for the per-level read-back (a pageable destination costs an extra staged
// copy on every level).  Allocated once per process on first use and kept; a thread-local slot
// keeps concurrent calls on different threads apart.
struct PinnedStats {
    LevelStats* p = nullptr;
    ~PinnedStats() {
        if (p) (void)hipHostFree(p);
    }
};

LevelStats* pinned_stats() {
    thread_local PinnedStats ps;
    if (!ps.p) {
        void* q = nullptr;
        if (hipHostMalloc(&q, sizeof(LevelStats) * 2, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ps.p = (LevelStats*)q;
    }
    return ps.p;
}

// Timing events of count_exact, created once per thread and device and reused (creating them on
// every call would add their cost to every timed step).  An event belongs to the device that was
// current when it was created, so the set is rebuilt when the thread's current device changes.
struct TimingEvents {
    hipEvent_t ev[6] = {};
    int device = -1;
    void release() {
        for (hipEvent_t& e : ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        device = -1;
    }
    ~TimingEvents() { release(); }
};

hipEvent_t* timing_events() {
    thread_local TimingEvents te;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (te.device != dev) {
        te.release();
        for (hipEvent_t& e : te.ev) {
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                te.release();
                return nullptr;
            }
        }
        te.device = dev;
    }
    return te.ev;
}

// Depth of the one-pass top of the tree (0: none).  Taken where the level loop bisects the widest
// side (with the LDS or the tape-state kernel, either relaxation), above the first alpha depth
// (levels with an alpha pass run level by level), for K >= 4 levels whose complete subtree
// (2^(K+1) - 1 boxes, at most 65535) fits the frontier.
int prefix_depth(const slr_net* net, const slr_exact_opts* o, const Workspace& w) {
    (void)w;
    if (o->split_layers > 0 || (o->timing & 4) || net->dev.d > SLR_MAX_D) return 0;
    int K = std::min(15, o->max_depth);
    if (o->alpha_steps > 0) K = std::min(K, o->alpha_min_depth - 1);
    while (K > 0 && ((int64_t)2 << K) - 1 > o->max_leaves) --K;
    return K >= 4 ? K : 0;
}

// no_alloc: the call makes no allocation of any kind (no pinned staging buffer, no event, no
// host heap): level counts are read back into stack memory and the split waits for them.
int count_exact_impl(const slr_net* net, const slr_property* prop, const double* lo,
                     const double* hi, const slr_exact_opts* o, const Workspace& w,
                     slr_count_result* out, bool no_alloc = false) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    const int d = net->dev.d;
    const int D = o->max_depth;
    const int64_t M = o->max_leaves;
    const int64_t chunk = o->chunk > 0 ? o->chunk : 65536;

    HIP_TRY(hipMemsetAsync(w.stats, 0, sizeof(LevelStats) * kMaxLevels, s), "count_exact: clear");
    HIP_TRY(hipMemsetAsync(w.rechecks, 0, sizeof(unsigned long long), s), "count_exact: clear");
    HIP_TRY(hipMemsetAsync(w.err, 0, sizeof(unsigned) * (kMaxLevels + 1), s), "count_exact: clear");
    float root[2 * SLR_MAX_D];   // d <= SLR_MAX_D (load_net)
    for (int k = 0; k < d; ++k) {
        root[k] = (float)lo[k];
        root[d + k] = (float)hi[k];
    }
    const unsigned long long one = 1;
    HIP_TRY(hipMemcpyAsync(w.lo[0], root, sizeof(float) * d, hipMemcpyHostToDevice, s), "count_exact: root");
    HIP_TRY(hipMemcpyAsync(w.hi[0], root + d, sizeof(float) * d, hipMemcpyHostToDevice, s), "count_exact: root");
    HIP_TRY(hipMemcpyAsync(w.path[0], &one, sizeof one, hipMemcpyHostToDevice, s), "count_exact: root");

    // timing events (thread-local, created once): the bound launches of a level, and two
    // alternating pairs around split launches (a split is counted once its level continues)
    hipEvent_t* tev = o->timing ? timing_events() : nullptr;
    if (o->timing && !tev) return fail(SLR_EHIP, "count_exact: cannot create timing events");
    hipEvent_t ev0 = tev && (o->timing & 1) ? tev[0] : nullptr;
    hipEvent_t ev1 = tev && (o->timing & 1) ? tev[1] : nullptr;
    const bool time_split = tev && (o->timing & 2);
    auto sev = [&](int t, int k) { return tev[2 + 2 * (t & 1) + k]; };
    int split_pending = -1;    // level whose timed split has not been read yet
    double split_ms = 0.0;
    int64_t split_bytes = 0;
    hipEvent_t evr = nullptr;   // marks the end of a level's read-back
    if (!no_alloc && hipEventCreateWithFlags(&evr, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        evr = nullptr;
    }
    struct EventGuard {
        hipEvent_t e;
        ~EventGuard() {
            if (e) (void)hipEventDestroy(e);
        }
    } guard{evr};
    double bound_ms = 0.0, alpha_ms = 0.0;
    int64_t launches = 0, alpha_boxes = 0, alpha_decided = 0, alpha_und_before = 0;
    int64_t n = 1, resolved = 0, bounded = 0, tcount = 0;
    int cur = 0, levels = 0, stop_level = 0, stopped = 0, status = SLR_OK;
    std::vector<unsigned long long> hpath;
    std::vector<int8_t> hcls, hdim;
    int t_begin = 0;
    bool finished = false;
    const int K = prefix_depth(net, o, w);
    if (K > 0) {
        // Depths 0 .. K in one pass: the complete subtree is built, bounded and re-decided in
        // large launches instead of K + 1 latency-bound levels; the replay keeps exactly the
        // boxes the level loop would bound (results, counts and traces are identical).
        const int64_t N = ((int64_t)2 << K) - 1;
        const int64_t sl = ((int64_t)1 << K) - 1;   // first box of depth K
        const int64_t nK = (int64_t)1 << K;
        RootBox rb{};
        for (int k = 0; k < d; ++k) {
            rb.lo[k] = root[k];
            rb.hi[k] = root[d + k];
        }
        HIP_TRY(launch_prefix_boxes(N, d, rb, w.lo[0], w.hi[0], w.path[0], w.err, s), "count_exact: prefix kernel");
        HIP_TRY(hipMemsetAsync(w.amb_count, 0, sizeof(unsigned), s), "count_exact: clear");
        if (ev0) HIP_TRY(hipEventRecord(ev0, s), "count_exact: event");
        if (w.wchunk > 0) {
            // tape-state kernel, as in the level loop below: widened classes, then (one ratio)
            // raw bounds that list the boxes near a decision for the FP64 re-decision
            for (int64_t off = 0; off < N; off += w.wchunk) {
                const int64_t m = std::min(w.wchunk, N - off);
                AlphaArgs a{};
                a.n = m;
                a.lo = w.lo[0] + off * d;
                a.hi = w.hi[0] + off * d;
                a.tape = w.wtape;
                a.fwd_only = 1;
                a.two_ratio = o->relax == SLR_RELAX_TWO;
                a.g_lo = w.wlo;
                a.g_hi = w.whi;
                a.cls = w.cls + off;
                HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, s), "count_exact: bound kernel");
                ++launches;
                if (a.two_ratio) continue;
                a.raw = 1;
                a.g_lo = w.rlo;
                a.g_hi = w.rhi;
                a.cls = nullptr;
                HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, s), "count_exact: bound kernel");
                HIP_TRY(launch_ambiguity(m, prop->dev.rows, w.wlo, w.whi, w.rlo, w.rhi, w.cls + off,
                                         w.amb_list, w.amb_count, (unsigned)off, s),
                        "count_exact: ambiguity kernel");
                ++launches;
            }
        } else {
            for (int64_t off = 0; off < N; off += chunk) {
                const int64_t m = std::min(chunk, N - off);
                int unsup = 0;
                HIP_TRY(launch_bound_f32(net->dev, prop->dev, m, w.lo[0] + off * d, w.hi[0] + off * d,
                                         nullptr, nullptr, w.cls + off, 0, s, &unsup, w.amb_list,
                                         w.amb_count, (unsigned)off),
                        "count_exact: bound kernel");
                if (unsup) return fail(SLR_EUNSUPPORTED, "count_exact: shape not supported");
                ++launches;
            }
        }
        if (ev1) HIP_TRY(hipEventRecord(ev1, s), "count_exact: event");
        if (o->relax != SLR_RELAX_TWO)
            HIP_TRY(launch_recheck64(net->dev, prop->dev, N, w.lo[0], w.hi[0], nullptr, nullptr, w.cls,
                                     w.rechecks, w.amb_list, w.amb_count, s),
                    "count_exact: recheck kernel");
        HIP_TRY(launch_prefix_replay(N, K, w.cls, w.stats, s), "count_exact: prefix replay kernel");
        HIP_TRY(launch_prefix_recheck_uncount(N, w.amb_list, w.amb_count, w.cls, w.rechecks, s),
                "count_exact: prefix replay kernel");
        HIP_TRY(launch_level_count(nK, w.cls + sl, w.tile_und, w.stats + K, s), "count_exact: count kernel");
        LevelStats hst[16];
        HIP_TRY(hipMemcpyAsync(hst, w.stats, sizeof(LevelStats) * (K + 1), hipMemcpyDeviceToHost, s),
                "count_exact: readback");
        const bool tr = o->trace_capacity > 0 && o->trace_path && o->trace_cls && o->trace_depth;
        if (tr) {
            hpath.resize(N);
            hcls.resize(N);
            HIP_TRY(hipMemcpyAsync(hpath.data(), w.path[0], N * sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "count_exact: trace");
            HIP_TRY(hipMemcpyAsync(hcls.data(), w.cls, N, hipMemcpyDeviceToHost, s), "count_exact: trace");
        }
        HIP_TRY(hipStreamSynchronize(s), "count_exact: sync");
        if (ev0) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1), "count_exact: event");
            bound_ms += ms;
        }
        // the level loop's decisions, level by level
        for (int t = 0; t <= K; ++t) {
            const LevelStats& h = hst[t];
            const int64_t und = (int64_t)h.undecided_cnt;
            const int64_t nt = (int64_t)(h.unsafe_cnt + h.safe_cnt) + und;
            if (tr) {
                const int64_t b0 = ((int64_t)1 << t) - 1, b1 = ((int64_t)2 << t) - 1;
                int64_t seen = 0;
                for (int64_t i = b0; i < b1; ++i) {
                    if (hcls[i] == 4) continue;
                    ++seen;
                    if (tcount < o->trace_capacity) {
                        o->trace_depth[tcount] = t;
                        o->trace_path[tcount] = hpath[i];
                        o->trace_cls[tcount] = hcls[i];
                        if (o->trace_dim) o->trace_dim[tcount] = hcls[i] == 0 ? (int8_t)-2 : (int8_t)-1;
                        ++tcount;
                    }
                }
                if (seen != nt)
                    return fail(SLR_EINTERNAL, "count_exact: prefix level %d lists %lld boxes, counts %lld", t,
                                (long long)seen, (long long)nt);
            }
            bounded += nt;
            levels = t + 1;
            resolved += (int64_t)(h.unsafe_cnt + h.safe_cnt);
            if (und == 0) {
                finished = true;
                break;
            }
            if (t == D || resolved + 2 * und > M) {
                stopped = 1;
                stop_level = t;
                status = SLR_BUDGET;
                finished = true;
                break;
            }
            if (t == K) {
                if (time_split) HIP_TRY(hipEventRecord(sev(K, 0), s), "count_exact: event");
                HIP_TRY(launch_split(nK, d, w.cls + sl, w.tile_und, w.lo[0] + sl * d, w.hi[0] + sl * d,
                                     w.path[0] + sl, w.lo[1], w.hi[1], w.path[1], w.err + K, M, s),
                        "count_exact: split kernel");
                if (time_split) {
                    HIP_TRY(hipEventRecord(sev(K, 1), s), "count_exact: event");
                    split_pending = K;   // read after the next level's sync
                }
                split_bytes += nK + und * (int64_t)(2 * d * sizeof(float) + 8) * 3 +
                               (int64_t)level_tiles(nK) * 4;
                n = 2 * und;
                cur = 1;
                t_begin = K + 1;
            }
        }
    }
    for (int t = t_begin; !finished && t <= D; ++t) {
        int unsup = 0;
        HIP_TRY(hipMemsetAsync(w.amb_count, 0, sizeof(unsigned), s), "count_exact: clear");
        if (ev0) HIP_TRY(hipEventRecord(ev0, s), "count_exact: event");
        if (w.wchunk > 0) {
            // tape-state kernel with the plain slopes: widened bounds classify, raw bounds
            // locate the boxes near a decision for the FP64 re-decision
            for (int64_t off = 0; off < n; off += w.wchunk) {
                const int64_t m = std::min(w.wchunk, n - off);
                AlphaArgs a{};
                a.n = m;
                a.lo = w.lo[cur] + off * d;
                a.hi = w.hi[cur] + off * d;
                a.tape = w.wtape;
                a.fwd_only = 1;
                a.two_ratio = o->relax == SLR_RELAX_TWO;
                a.g_lo = w.wlo;
                a.g_hi = w.whi;
                a.cls = w.cls + off;
                HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, s), "count_exact: bound kernel");
                ++launches;
                // two ratios: the widened float32 classes stand (no FP64 re-decision)
                if (a.two_ratio) continue;
                if (o->alpha_steps > 0 && t >= o->alpha_min_depth && o->alpha_select > 0.f) {
                    // an alpha level that selects its candidates keeps the plain bounds
                    const size_t gb = sizeof(float) * prop->dev.rows * m;
                    HIP_TRY(hipMemcpyAsync(w.glo + off * prop->dev.rows, w.wlo, gb,
                                           hipMemcpyDeviceToDevice, s), "count_exact: bounds");
                    HIP_TRY(hipMemcpyAsync(w.ghi + off * prop->dev.rows, w.whi, gb,
                                           hipMemcpyDeviceToDevice, s), "count_exact: bounds");
                }
                a.raw = 1;
                a.g_lo = w.rlo;
                a.g_hi = w.rhi;
                a.cls = nullptr;
                HIP_TRY(launch_alpha_forward(net->dev, prop->dev, a, s), "count_exact: bound kernel");
                HIP_TRY(launch_ambiguity(m, prop->dev.rows, w.wlo, w.whi, w.rlo, w.rhi, w.cls + off,
                                         w.amb_list, w.amb_count, (unsigned)off, s),
                        "count_exact: ambiguity kernel");
                ++launches;
            }
        } else {
            // an alpha level that selects its candidates keeps the plain bounds
            const bool keep_g = o->alpha_steps > 0 && t >= o->alpha_min_depth && o->alpha_select > 0.f;
            const int rows = prop->dev.rows;
            for (int64_t off = 0; off < n; off += chunk) {
                const int64_t m = std::min(chunk, n - off);
                HIP_TRY(launch_bound_f32(net->dev, prop->dev, m, w.lo[cur] + off * d, w.hi[cur] + off * d,
                                         keep_g ? w.glo + off * rows : nullptr,
                                         keep_g ? w.ghi + off * rows : nullptr, w.cls + off, 0, s,
                                         &unsup, w.amb_list, w.amb_count, (unsigned)off,
                                         o->split_layers > 0 ? w.dimsel + off : nullptr, o->split_layers),
                        "count_exact: bound kernel");
                if (unsup) return fail(SLR_EUNSUPPORTED, "count_exact: shape not supported");
                ++launches;
            }
        }
        if (ev1) {
            HIP_TRY(hipEventRecord(ev1, s), "count_exact: event");
            if (o->alpha_steps > 0) {
                HIP_TRY(hipEventSynchronize(ev1), "count_exact: event");
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1), "count_exact: event");
                bound_ms += ms;
            }
        }
        if (o->relax != SLR_RELAX_TWO)
            HIP_TRY(launch_recheck64(net->dev, prop->dev, n, w.lo[cur], w.hi[cur], nullptr, nullptr,
                                     w.cls, w.rechecks, w.amb_list, w.amb_count, s),
                    "count_exact: recheck kernel");
        if (o->alpha_steps > 0 && t >= o->alpha_min_depth) {
            if (ev0) HIP_TRY(hipEventRecord(ev0, s), "count_exact: event");
            HIP_TRY(hipMemsetAsync(w.amb_count, 0, 2 * sizeof(unsigned), s), "count_exact: clear");
            const bool sel = o->alpha_select > 0.f;
            HIP_TRY(launch_collect_undecided(n, w.cls, w.amb_list, w.amb_count, s,
                                             sel ? w.glo : nullptr, sel ? w.ghi : nullptr,
                                             prop->dev.rows, o->alpha_select, w.amb_count + 1),
                    "count_exact: collect kernel");
            unsigned cnt2[2] = {0, 0};   // boxes given the alpha pass, all undecided boxes
            HIP_TRY(hipMemcpyAsync(cnt2, w.amb_count, sizeof cnt2, hipMemcpyDeviceToHost, s), "count_exact: readback");
            HIP_TRY(hipStreamSynchronize(s), "count_exact: sync");
            const unsigned und_cnt = cnt2[0];
            slr_alpha_opts ao{};
            ao.steps = o->alpha_steps;
            ao.lr = o->alpha_lr > 0.f ? o->alpha_lr : 0.1f;
            ao.beta1 = 0.9f;
            ao.beta2 = 0.999f;
            ao.eps = 1e-8f;
            ao.raw = 0;
            const AlphaWs aw = layout_alpha(w.aws, net->dev, prop->dev, w.achunk);
            for (int64_t off = 0; off < (int64_t)und_cnt; off += w.achunk) {
                const int64_t m = std::min<int64_t>(w.achunk, (int64_t)und_cnt - off);
                HIP_TRY(launch_gather_boxes(m, d, w.amb_list + off, w.lo[cur], w.hi[cur], w.alo, w.ahi, s), "count_exact: gather kernel");
                int arc = alpha_run(net, prop, m, w.alo, w.ahi, ao, nullptr, w.best_lo, w.best_hi, w.acls, aw, s);
                if (arc) return arc;
                HIP_TRY(launch_scatter_classes(m, w.amb_list + off, w.acls, w.cls, s), "count_exact: scatter kernel");
            }
            alpha_boxes += und_cnt;
            alpha_und_before += cnt2[1];   // decided by alpha = undecided before - after
            if (ev1) {
                HIP_TRY(hipEventRecord(ev1, s), "count_exact: event");
                HIP_TRY(hipEventSynchronize(ev1), "count_exact: event");
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1), "count_exact: event");
                alpha_ms += ms;
            }
        }
        HIP_TRY(launch_level_count(n, w.cls, w.tile_und, w.stats + t, s), "count_exact: count kernel");
        // the split is enqueued before the host reads this level's counts (it runs while the
        // read-back travels); if the level turns out to be the last one its output is unused,
        // children beyond the buffers are not written and its error slot is ignored
        LevelStats hs;
        LevelStats* pin = no_alloc ? nullptr : pinned_stats();
        HIP_TRY(hipMemcpyAsync(pin ? pin : &hs, w.stats + t, sizeof hs, hipMemcpyDeviceToHost, s),
                "count_exact: readback");
        if (o->trace_capacity > 0 && o->trace_path && o->trace_cls && o->trace_depth && tcount < o->trace_capacity) {
            const int64_t m = std::min<int64_t>(n, o->trace_capacity - tcount);
            hpath.resize(m);
            hcls.resize(m);
            HIP_TRY(hipMemcpyAsync(hpath.data(), w.path[cur], m * sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "count_exact: trace");
            HIP_TRY(hipMemcpyAsync(hcls.data(), w.cls, m, hipMemcpyDeviceToHost, s), "count_exact: trace");
            if (o->trace_dim) {
                hdim.resize(m);
                if (o->split_layers > 0)
                    HIP_TRY(hipMemcpyAsync(hdim.data(), w.dimsel, m, hipMemcpyDeviceToHost, s), "count_exact: trace");
            }
            HIP_TRY(hipStreamSynchronize(s), "count_exact: sync");
            for (int64_t i = 0; i < m; ++i) {
                o->trace_depth[tcount + i] = t;
                o->trace_path[tcount + i] = hpath[i];
                o->trace_cls[tcount + i] = hcls[i];
                if (o->trace_dim) {
                    // the side bisected: chosen by the bound kernel, or the widest one
                    int8_t side = -1;
                    if (hcls[i] == 0) side = o->split_layers > 0 ? hdim[i] : (int8_t)-2;
                    o->trace_dim[tcount + i] = side;
                }
            }
            tcount += m;
        }
        // When the leaf budget cannot stop the search at this level, the split is enqueued
        // before the host reads the counts back and runs while the read-back travels (its output
        // is unused if nothing is left undecided; its error slot is checked only for levels the
        // search continues from).  Otherwise the host decides first.
        const bool spec = t < D && pin && evr && resolved + 2 * n <= M;
        if (spec) {
            HIP_TRY(hipEventRecord(evr, s), "count_exact: event");
            if (time_split) HIP_TRY(hipEventRecord(sev(t, 0), s), "count_exact: event");
            HIP_TRY(launch_split(n, d, w.cls, w.tile_und, w.lo[cur], w.hi[cur], w.path[cur],
                                 w.lo[cur ^ 1], w.hi[cur ^ 1], w.path[cur ^ 1], w.err + t, M, s,
                                 o->split_layers > 0 ? w.dimsel : nullptr),
                    "count_exact: split kernel");
            if (time_split) HIP_TRY(hipEventRecord(sev(t, 1), s), "count_exact: event");
            HIP_TRY(hipEventSynchronize(evr), "count_exact: sync");
        } else {
            HIP_TRY(hipStreamSynchronize(s), "count_exact: sync");
        }
        if (split_pending >= 0) {   // the previous level's split has completed (stream order)
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, sev(split_pending, 0), sev(split_pending, 1)),
                    "count_exact: event");
            split_ms += ms;
            split_pending = -1;
        }
        if (pin) hs = *pin;
        if (ev0 && o->alpha_steps <= 0) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1), "count_exact: event");
            bound_ms += ms;
        }
        bounded += n;
        levels = t + 1;
        resolved += (int64_t)(hs.unsafe_cnt + hs.safe_cnt);
        const int64_t und = (int64_t)hs.undecided_cnt;
        if (alpha_und_before > 0) {
            alpha_decided += alpha_und_before - und;
            alpha_und_before = 0;
        }
        if ((int64_t)(hs.unsafe_cnt + hs.safe_cnt) + und != n)
            return fail(SLR_EINTERNAL, "count_exact: level %d counts %lld boxes of %lld", t,
                        (long long)(hs.unsafe_cnt + hs.safe_cnt + und), (long long)n);
        if (und == 0) break;
        if (t == D || resolved + 2 * und > M) {
            stopped = 1;
            stop_level = t;
            status = SLR_BUDGET;
            break;
        }
        if (!spec) {
            if (time_split) HIP_TRY(hipEventRecord(sev(t, 0), s), "count_exact: event");
            HIP_TRY(launch_split(n, d, w.cls, w.tile_und, w.lo[cur], w.hi[cur], w.path[cur],
                                 w.lo[cur ^ 1], w.hi[cur ^ 1], w.path[cur ^ 1], w.err + t, M, s,
                                 o->split_layers > 0 ? w.dimsel : nullptr),
                    "count_exact: split kernel");
            if (time_split) HIP_TRY(hipEventRecord(sev(t, 1), s), "count_exact: event");
        }
        if (time_split) split_pending = t;
        // algorithmic bytes of the split: every class, the undecided parents' corners and paths,
        // two children each, and the per-tile counts
        split_bytes += n + und * (int64_t)(2 * d * sizeof(float) + 8) * 3 +
                       (int64_t)level_tiles(n) * 4;
        n = 2 * und;
        cur ^= 1;
    }
    HIP_TRY(launch_volume(w.stats, levels, stop_level, stopped, w.vol, w.counts, w.err + kMaxLevels, s),
            "count_exact: volume kernel");
    double vol[3];
    unsigned long long counts[3], rechecks = 0;
    unsigned errs[kMaxLevels + 1];
    HIP_TRY(hipMemcpyAsync(vol, w.vol, sizeof vol, hipMemcpyDeviceToHost, s), "count_exact: readback");
    HIP_TRY(hipMemcpyAsync(counts, w.counts, sizeof counts, hipMemcpyDeviceToHost, s), "count_exact: readback");
    HIP_TRY(hipMemcpyAsync(&rechecks, w.rechecks, sizeof rechecks, hipMemcpyDeviceToHost, s), "count_exact: readback");
    HIP_TRY(hipMemcpyAsync(errs, w.err, sizeof errs, hipMemcpyDeviceToHost, s), "count_exact: readback");
    HIP_TRY(hipStreamSynchronize(s), "count_exact: sync");
    unsigned err = errs[kMaxLevels];
    for (int t = 0; t + 1 < levels; ++t) err |= errs[t];   // the levels that were continued
    if (err & 1u) return fail(SLR_EINTERNAL, "count_exact: a bisection midpoint is not exact in float32 (box too deep for its coordinates)");
    if (err & 2u) return fail(SLR_EINTERNAL, "count_exact: leaf volumes do not sum to the box volume");
    out->unsafe = vol[0];
    out->safe = vol[1];
    out->undecided = vol[2];
    out->n_unsafe = (int64_t)counts[0];
    out->n_safe = (int64_t)counts[1];
    out->n_undecided = (int64_t)counts[2];
    out->n_boxes_bounded = bounded;
    out->n_recheck64 = (int64_t)rechecks;
    out->depth_reached = levels - 1;
    out->status = status;
    out->trace_count = tcount;
    out->bound_ms = bound_ms;
    out->bound_launches = launches;
    out->n_alpha_boxes = alpha_boxes;
    out->n_alpha_decided = alpha_decided;
    out->alpha_ms = alpha_ms;
    out->split_ms = split_ms;
    out->split_bytes = split_bytes;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

int check_exact_opts(const slr_net* net, const slr_property* prop, const slr_exact_opts* o,
                     int samples, Workspace* w, const char* who, bool check_device = true,
                     bool small_tape = false) {
    if (!o) return fail(SLR_EINVAL, "%s: opts is NULL", who);
    if (o->max_depth < 0 || o->max_depth > kMaxLevels - 1)
        return fail(SLR_EINVAL, "%s: max_depth must be in [0, %d]", who, kMaxLevels - 1);
    if (o->max_leaves < 1) return fail(SLR_EINVAL, "%s: max_leaves must be >= 1", who);
    if (o->chunk < 0) return fail(SLR_EINVAL, "%s: chunk must be >= 0", who);
    if (o->trace_capacity < 0) return fail(SLR_EINVAL, "%s: trace_capacity must be >= 0", who);
    if (o->alpha_steps < 0 || o->alpha_steps > 1000) return fail(SLR_EINVAL, "%s: alpha_steps must be in [0, 1000]", who);
    if (o->alpha_chunk < 0) return fail(SLR_EINVAL, "%s: alpha_chunk must be >= 0", who);
    if (o->alpha_steps > 0 && o->alpha_chunk < 1)
        return fail(SLR_EINVAL, "%s: alpha mode needs alpha_chunk >= 1 (and a workspace sized for it)", who);
    if (!(o->alpha_lr >= 0.f) || o->alpha_min_depth < 0)
        return fail(SLR_EINVAL, "%s: alpha_lr and alpha_min_depth must be >= 0", who);
    if (!(o->alpha_select >= 0.f) || !std::isfinite(o->alpha_select))
        return fail(SLR_EINVAL, "%s: alpha_select must be finite and >= 0", who);
    if (o->split_layers < 0 || o->split_layers > SLR_MAX_AFFINE)
        return fail(SLR_EINVAL, "%s: split_layers must be in [0, %d]", who, SLR_MAX_AFFINE);
    if (o->split_layers > 0 && (net->dev.act != SLR_ACT_RELU || !bound_f32_supported(net->dev, prop->dev) ||
                                bound_variant_for(net->dev, prop->dev) < 0 || net->dev.d + 3 > 14))
        return fail(SLR_EUNSUPPORTED, "%s: the crossing-score split needs a ReLU network on the LDS bound "
                    "kernel with at most 11 inputs", who);
    if (o->relax != SLR_RELAX_ONE && o->relax != SLR_RELAX_TWO)
        return fail(SLR_EINVAL, "%s: relax must be SLR_RELAX_ONE or SLR_RELAX_TWO", who);
    if (o->relax == SLR_RELAX_TWO) {
        if (net->dev.act != SLR_ACT_RELU)
            return fail(SLR_EUNSUPPORTED, "%s: the two-ratio relaxation is defined for ReLU networks only", who);
        if (o->alpha_steps > 0 || o->split_layers > 0)
            return fail(SLR_EUNSUPPORTED, "%s: the two-ratio relaxation takes neither alpha slopes nor the "
                        "crossing-score split", who);
        if (alpha_shape(net->dev, prop->dev).nc < 0)
            return fail(SLR_EUNSUPPORTED, "%s: input dimension too large for the tape-state kernel", who);
    }
    if (net->dev.act != SLR_ACT_RELU) {
        if (o->alpha_steps > 0)
            return fail(SLR_EUNSUPPORTED, "%s: alpha slopes are defined for ReLU networks only", who);
        if (!bound_f32_supported(net->dev, prop->dev) || bound_variant_for(net->dev, prop->dev) < 0)
            return fail(SLR_EUNSUPPORTED, "%s: tanh and sigmoid networks need the LDS or register bound kernel", who);
    }
    const int64_t achunk = o->alpha_steps > 0 ? o->alpha_chunk : 0;
    const bool two = o->relax == SLR_RELAX_TWO;
    const size_t need = layout_ws(nullptr, net->dev, prop->dev, o->max_leaves, samples, achunk, two,
                                  small_tape).bytes;
    if (!o->workspace || o->workspace_bytes < need)
        return fail(SLR_ENOMEM, "%s: workspace of %zu bytes is smaller than the %zu required", who,
                    o->workspace_bytes, need);
    if (check_device && !is_device_ptr(o->workspace)) return fail(SLR_EINVAL, "%s: workspace must be device memory", who);
    *w = layout_ws((char*)o->workspace, net->dev, prop->dev, o->max_leaves, samples, achunk, two,
                   small_tape);
    return SLR_OK;
}

}  // namespace

extern "C" int count_exact(const slr_net* net, const slr_property* prop, const double* lo,
                           const double* hi, const slr_exact_opts* opts, slr_count_result* out) {
    g_err.clear();
    int rc = check_pair(net, prop, "count_exact");
    if (rc) return rc;
    if (!out) return fail(SLR_EINVAL, "count_exact: out is NULL");
    if ((rc = check_box(net, lo, hi, "count_exact"))) return rc;
    Workspace w;
    if ((rc = check_exact_opts(net, prop, opts, 0, &w, "count_exact"))) return rc;
    memset(out, 0, sizeof *out);
    return count_exact_impl(net, prop, lo, hi, opts, w, out);
}

// ------------------------------------------------------------------------------------------
// Allocation-free exact count: the workspace is a file-scope device array
// ------------------------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held from the library's first use on that GPU until the process ends.
// Host code never passes this name to a kernel: it is a host-side stand-in, and the device
// address of each GPU's copy comes from hipGetSymbolAddress (scratch_address).
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch copy, looked up once per device.
int scratch_address(void** out, const char* who) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "scratch: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SLR_EUNSUPPORTED, "%s: device %d beyond %d", who, dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SLR_EHIP, "%s: hipGetSymbolAddress(scratch) failed on device %d: %s", who, dev,
                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SLR_OK;
}

}  // namespace

extern "C" size_t count_exact_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int count_exact_noalloc(const slr_net* net, const slr_property* prop, const double* lo,
                                   const double* hi, const slr_exact_opts* opts, slr_count_result* out) {
    g_err.clear();
    int rc = check_pair(net, prop, "count_exact_noalloc");
    if (rc) return rc;
    if (!out || !opts) return fail(SLR_EINVAL, "count_exact_noalloc: NULL argument");
    if ((rc = check_box(net, lo, hi, "count_exact_noalloc"))) return rc;
    if (opts->workspace || opts->workspace_bytes)
        return fail(SLR_EINVAL, "count_exact_noalloc: the workspace is the library's own; pass workspace = NULL, 0 bytes");
    if (opts->trace_capacity || opts->timing)
        return fail(SLR_EINVAL, "count_exact_noalloc: traces and timing are not available (they need host buffers and events)");
    const int64_t achunk = opts->alpha_steps > 0 ? opts->alpha_chunk : 0;
    if (opts->max_leaves >= 1 && achunk >= 0) {
        const size_t need = layout_ws(nullptr, net->dev, prop->dev, opts->max_leaves, 0, achunk,
                                      opts->relax == SLR_RELAX_TWO, /*small_tape=*/true).bytes;
        if (need > kScratchBytes)
            return fail(SLR_ENOMEM, "count_exact_noalloc: this count needs %zu bytes of workspace, more than the "
                        "%zu-byte static scratch (lower max_leaves or alpha_chunk, or use count_exact)", need, kScratchBytes);
    }
    void* base = nullptr;
    if ((rc = scratch_address(&base, "count_exact_noalloc"))) return rc;
    slr_exact_opts o = *opts;
    o.workspace = base;
    o.workspace_bytes = kScratchBytes;
    Workspace w;
    if ((rc = check_exact_opts(net, prop, &o, 0, &w, "count_exact_noalloc", /*check_device=*/false,
                               /*small_tape=*/true)))
        return rc;
    memset(out, 0, sizeof *out);
    return count_exact_impl(net, prop, lo, hi, &o, w, out, /*no_alloc=*/true);
}

// ------------------------------------------------------------------------------------------
// Depth-first stack count (bounded memory, optional host spill)
// ------------------------------------------------------------------------------------------
namespace {

struct StackWs {
    float *lo, *hi;                  // [cap][d] the stack, shallowest boxes at the bottom
    unsigned long long* path;        // [cap]
    float *clo, *chi;                // [2 chunk][d] children of the chunk just bounded
    unsigned long long* cpath;       // [2 chunk]
    int8_t* cls;                     // [chunk]
    unsigned* amb_list;              // [chunk]
    unsigned* amb_count;
    unsigned* tile_und;
    unsigned* split_total;
    LevelStats* stats;               // [kMaxLevels]
    double* vol;
    unsigned long long *counts, *rechecks;
    unsigned* err;
    int64_t cap, chunk;
    size_t bytes;
};

int64_t stack_chunk(const slr_stack_opts& o) { return o.chunk > 0 ? o.chunk : 65536; }

int64_t stack_device_boxes(const slr_stack_opts& o) {
    return o.device_boxes > 0 ? o.device_boxes : 2 * (int64_t)(o.max_depth + 2) * stack_chunk(o);
}

StackWs layout_stack(char* base, const NetDev& nd, int64_t cap, int64_t chunk) {
    const int d = nd.d;
    StackWs w{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    w.cap = cap;
    w.chunk = chunk;
    w.lo = (float*)take(sizeof(float) * d * cap);
    w.hi = (float*)take(sizeof(float) * d * cap);
    w.path = (unsigned long long*)take(sizeof(unsigned long long) * cap);
    w.clo = (float*)take(sizeof(float) * d * 2 * chunk);
    w.chi = (float*)take(sizeof(float) * d * 2 * chunk);
    w.cpath = (unsigned long long*)take(sizeof(unsigned long long) * 2 * chunk);
    w.cls = (int8_t*)take(chunk);
    w.amb_list = (unsigned*)take(sizeof(unsigned) * chunk);
    w.amb_count = (unsigned*)take(2 * sizeof(unsigned));
    w.tile_und = (unsigned*)take(sizeof(unsigned) * level_tiles(chunk));
    w.split_total = (unsigned*)take(sizeof(unsigned));
    w.stats = (LevelStats*)take(sizeof(LevelStats) * kMaxLevels);
    w.vol = (double*)take(sizeof(double) * 3);
    w.counts = (unsigned long long*)take(sizeof(unsigned long long) * 3);
    w.rechecks = (unsigned long long*)take(sizeof(unsigned long long));
    w.err = (unsigned*)take(sizeof(unsigned));
    w.bytes = o;
    return w;
}

int check_stack_opts(const slr_net* net, const slr_stack_opts* o, const char* who) {
    if (!o) return fail(SLR_EINVAL, "%s: opts is NULL", who);
    if (o->max_depth < 0 || o->max_depth > kMaxLevels - 1)
        return fail(SLR_EINVAL, "%s: max_depth must be in [0, %d]", who, kMaxLevels - 1);
    if (o->chunk < 0 || o->chunk > 65536) return fail(SLR_EINVAL, "%s: chunk must be in [0, 65536]", who);
    if (o->max_boxes < 0) return fail(SLR_EINVAL, "%s: max_boxes must be >= 0", who);
    if (o->device_boxes < 0 || (o->device_boxes > 0 && o->device_boxes < 4 * stack_chunk(*o)))
        return fail(SLR_EINVAL, "%s: device_boxes must be 0 or >= 4 * chunk", who);
    if (o->trace_capacity < 0) return fail(SLR_EINVAL, "%s: trace_capacity must be >= 0", who);
    if (o->host_spill_bytes > 0 && !o->host_spill) return fail(SLR_EINVAL, "%s: host_spill is NULL", who);
    (void)net;
    return SLR_OK;
}

// The whole count; see the header.  Invariant: stack depths are non-decreasing from the bottom
// to the top (children, in parent order, are deeper than every box left below them), so the
// top chunk holds the deepest boxes and the host part the shallowest.
int count_stack_impl(const slr_net* net, const slr_property* prop, const double* lo,
                     const double* hi, const slr_stack_opts& o, const StackWs& w,
                     slr_count_result* out) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o.stream;
    const int d = net->dev.d;
    const int D = o.max_depth;
    const int64_t chunk = w.chunk, cap = w.cap;
    const size_t rec_host = sizeof(float) * 2 * d + sizeof(unsigned long long);
    const int64_t hcap = o.host_spill ? (int64_t)(o.host_spill_bytes / rec_host) : 0;
    float* h_lo = (float*)o.host_spill;
    float* h_hi = h_lo ? h_lo + (size_t)d * hcap : nullptr;
    unsigned long long* h_path = h_lo ? (unsigned long long*)(h_hi + (size_t)d * hcap) : nullptr;

    HIP_TRY(hipMemsetAsync(w.stats, 0, sizeof(LevelStats) * kMaxLevels, s), "count_exact_stack: clear");
    HIP_TRY(hipMemsetAsync(w.rechecks, 0, sizeof(unsigned long long), s), "count_exact_stack: clear");
    HIP_TRY(hipMemsetAsync(w.err, 0, sizeof(unsigned), s), "count_exact_stack: clear");
    float root[2 * SLR_MAX_D];
    for (int k = 0; k < d; ++k) {
        root[k] = (float)lo[k];
        root[d + k] = (float)hi[k];
    }
    const unsigned long long one = 1;
    HIP_TRY(hipMemcpyAsync(w.lo, root, sizeof(float) * d, hipMemcpyHostToDevice, s), "count_exact_stack: root");
    HIP_TRY(hipMemcpyAsync(w.hi, root + d, sizeof(float) * d, hipMemcpyHostToDevice, s), "count_exact_stack: root");
    HIP_TRY(hipMemcpyAsync(w.path, &one, sizeof one, hipMemcpyHostToDevice, s), "count_exact_stack: root");

    LevelStats* pin = pinned_stats();      // pinned read-back slot (the split total goes here)
    unsigned nsplit_host = 0;
    int64_t top = 1, host_cnt = 0, bounded = 0, tcount = 0;
    int status = SLR_OK;
    std::vector<unsigned long long> hpath;
    std::vector<int8_t> hcls;
    auto copy3 = [&](float* dlo, float* dhi, unsigned long long* dpath, const float* slo,
                     const float* shi, const unsigned long long* spath, int64_t m, hipMemcpyKind k) {
        hipError_t e = hipMemcpyAsync(dlo, slo, sizeof(float) * d * m, k, s);
        if (e == hipSuccess) e = hipMemcpyAsync(dhi, shi, sizeof(float) * d * m, k, s);
        if (e == hipSuccess) e = hipMemcpyAsync(dpath, spath, sizeof(unsigned long long) * m, k, s);
        return e;
    };
    while (top > 0 || host_cnt > 0) {
        if (top == 0) {   // the device part has drained: bring back the deepest host boxes
            const int64_t k = std::min(host_cnt, cap / 2);
            const int64_t from = host_cnt - k;
            HIP_TRY(copy3(w.lo, w.hi, w.path, h_lo + from * d, h_hi + from * d, h_path + from, k,
                          hipMemcpyHostToDevice), "count_exact_stack: refill");
            host_cnt = from;
            top = k;
        }
        const int64_t m = std::min(chunk, top);
        if (o.max_boxes > 0 && bounded + m > o.max_boxes) {
            status = SLR_BUDGET;
            break;
        }
        const int64_t base = top - m;
        float* blo = w.lo + base * d;
        float* bhi = w.hi + base * d;
        unsigned long long* bpath = w.path + base;
        int unsup = 0;
        HIP_TRY(hipMemsetAsync(w.amb_count, 0, sizeof(unsigned), s), "count_exact_stack: clear");
        HIP_TRY(hipMemsetAsync(w.split_total, 0, sizeof(unsigned), s), "count_exact_stack: clear");
        HIP_TRY(launch_bound_f32(net->dev, prop->dev, m, blo, bhi, nullptr, nullptr, w.cls, 0, s, &unsup,
                                 w.amb_list, w.amb_count, 0u),
                "count_exact_stack: bound kernel");
        if (unsup) return fail(SLR_EUNSUPPORTED, "count_exact_stack: network shape exceeds the LDS bound kernel");
        HIP_TRY(launch_recheck64(net->dev, prop->dev, m, blo, bhi, nullptr, nullptr, w.cls, w.rechecks,
                                 w.amb_list, w.amb_count, s),
                "count_exact_stack: recheck kernel");
        HIP_TRY(launch_stack_count(m, w.cls, bpath, D, 0, w.tile_und, w.stats, w.split_total, s),
                "count_exact_stack: count kernel");
        HIP_TRY(launch_split(m, d, w.cls, w.tile_und, blo, bhi, bpath, w.clo, w.chi, w.cpath, w.err,
                             2 * chunk, s),
                "count_exact_stack: split kernel");
        unsigned* dst = pin ? (unsigned*)pin : &nsplit_host;
        HIP_TRY(hipMemcpyAsync(dst, w.split_total, sizeof(unsigned), hipMemcpyDeviceToHost, s),
                "count_exact_stack: readback");
        if (o.trace_capacity > 0 && o.trace_path && o.trace_cls && o.trace_depth && tcount < o.trace_capacity) {
            const int64_t k = std::min<int64_t>(m, o.trace_capacity - tcount);
            hpath.resize(k);
            hcls.resize(k);
            HIP_TRY(hipMemcpyAsync(hpath.data(), bpath, k * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                    "count_exact_stack: trace");
            HIP_TRY(hipMemcpyAsync(hcls.data(), w.cls, k, hipMemcpyDeviceToHost, s), "count_exact_stack: trace");
            HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
            for (int64_t i = 0; i < k; ++i) {
                int dep = 0;
                for (unsigned long long p = hpath[i]; p > 1; p >>= 1) ++dep;
                o.trace_depth[tcount + i] = dep;
                o.trace_path[tcount + i] = hpath[i];
                o.trace_cls[tcount + i] = hcls[i] == 4 ? 0 : hcls[i];
            }
            tcount += k;
        }
        HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
        const int64_t nsplit = pin ? (int64_t)*(unsigned*)pin : (int64_t)nsplit_host;
        bounded += m;
        int64_t b = base;
        const int64_t need = b + 2 * nsplit - cap;
        if (need > 0) {   // spill the stack's bottom (its shallowest boxes) to the host
            const int64_t h = std::max(need, (b + 1) / 2);
            if (host_cnt + h > hcap)
                return fail(SLR_ENOMEM, "count_exact_stack: the stack needs more than %lld device and %lld host boxes",
                            (long long)cap, (long long)hcap);
            HIP_TRY(copy3(h_lo + host_cnt * d, h_hi + host_cnt * d, h_path + host_cnt, w.lo, w.hi, w.path, h,
                          hipMemcpyDeviceToHost), "count_exact_stack: spill");
            // [h, b) moves down to [0, b - h); b - h <= h, so source and destination do not overlap
            HIP_TRY(copy3(w.lo, w.hi, w.path, w.lo + h * d, w.hi + h * d, w.path + h, b - h,
                          hipMemcpyDeviceToDevice), "count_exact_stack: spill");
            HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
            host_cnt += h;
            b -= h;
        }
        if (nsplit > 0)
            HIP_TRY(copy3(w.lo + b * d, w.hi + b * d, w.path + b, w.clo, w.chi, w.cpath, 2 * nsplit,
                          hipMemcpyDeviceToDevice), "count_exact_stack: push");
        top = b + 2 * nsplit;
    }
    if (status == SLR_BUDGET) {
        // every box still on the stack is undecided at its depth
        HIP_TRY(launch_stack_count(top, nullptr, w.path, D, 1, nullptr, w.stats, w.split_total, s),
                "count_exact_stack: count kernel");
        for (int64_t done = 0; done < host_cnt;) {
            const int64_t k = std::min<int64_t>(host_cnt - done, 2 * chunk);
            HIP_TRY(hipMemcpyAsync(w.cpath, h_path + done, sizeof(unsigned long long) * k, hipMemcpyHostToDevice, s),
                    "count_exact_stack: refill");
            HIP_TRY(launch_stack_count(k, nullptr, w.cpath, D, 1, nullptr, w.stats, w.split_total, s),
                    "count_exact_stack: count kernel");
            HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
            done += k;
        }
    }
    LevelStats st[kMaxLevels];
    HIP_TRY(hipMemcpyAsync(st, w.stats, sizeof st, hipMemcpyDeviceToHost, s), "count_exact_stack: readback");
    HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
    int levels = 1;
    for (int t = 0; t < kMaxLevels; ++t)
        if (st[t].unsafe_cnt + st[t].safe_cnt + st[t].undecided_cnt > 0) levels = t + 1;
    HIP_TRY(launch_stack_volume(w.stats, levels, w.vol, w.counts, w.err, s), "count_exact_stack: volume kernel");
    double vol[3];
    unsigned long long counts[3], rechecks = 0;
    unsigned err = 0;
    HIP_TRY(hipMemcpyAsync(vol, w.vol, sizeof vol, hipMemcpyDeviceToHost, s), "count_exact_stack: readback");
    HIP_TRY(hipMemcpyAsync(counts, w.counts, sizeof counts, hipMemcpyDeviceToHost, s), "count_exact_stack: readback");
    HIP_TRY(hipMemcpyAsync(&rechecks, w.rechecks, sizeof rechecks, hipMemcpyDeviceToHost, s), "count_exact_stack: readback");
    HIP_TRY(hipMemcpyAsync(&err, w.err, sizeof err, hipMemcpyDeviceToHost, s), "count_exact_stack: readback");
    HIP_TRY(hipStreamSynchronize(s), "count_exact_stack: sync");
    if (err & 1u) return fail(SLR_EINTERNAL, "count_exact_stack: a bisection midpoint is not exact in float32 (box too deep for its coordinates)");
    if (err & 2u) return fail(SLR_EINTERNAL, "count_exact_stack: leaf volumes do not sum to the box volume");
    memset(out, 0, sizeof *out);
    out->unsafe = vol[0];
    out->safe = vol[1];
    out->undecided = vol[2];
    out->n_unsafe = (int64_t)counts[0];
    out->n_safe = (int64_t)counts[1];
    out->n_undecided = (int64_t)counts[2];
    out->n_boxes_bounded = bounded;
    out->n_recheck64 = (int64_t)rechecks;
    out->depth_reached = levels - 1;
    out->trace_count = tcount;
    if (counts[2] > 0 && status == SLR_OK) status = SLR_BUDGET;
    out->status = status;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

}  // namespace

extern "C" int stack_workspace_size(const slr_net* net, const slr_property* prop, const slr_stack_opts* opts,
                                    size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(SLR_EINVAL, "stack_workspace_size: bytes is NULL");
    int rc = check_pair(net, prop, "stack_workspace_size");
    if (rc) return rc;
    if ((rc = check_stack_opts(net, opts, "stack_workspace_size"))) return rc;
    *bytes = layout_stack(nullptr, net->dev, stack_device_boxes(*opts), stack_chunk(*opts)).bytes;
    return SLR_OK;
}

extern "C" int count_exact_stack(const slr_net* net, const slr_property* prop, const double* lo,
                                 const double* hi, const slr_stack_opts* opts, slr_count_result* out) {
    g_err.clear();
    int rc = check_pair(net, prop, "count_exact_stack", /*need_lds=*/true);
    if (rc) return rc;
    if (!out) return fail(SLR_EINVAL, "count_exact_stack: out is NULL");
    if ((rc = check_box(net, lo, hi, "count_exact_stack"))) return rc;
    if ((rc = check_stack_opts(net, opts, "count_exact_stack"))) return rc;
    const int64_t cap = stack_device_boxes(*opts), chunk = stack_chunk(*opts);
    const size_t need = layout_stack(nullptr, net->dev, cap, chunk).bytes;
    if (!opts->workspace || opts->workspace_bytes < need)
        return fail(SLR_ENOMEM, "count_exact_stack: workspace of %zu bytes is smaller than the %zu required",
                    opts->workspace_bytes, need);
    if (!is_device_ptr(opts->workspace)) return fail(SLR_EINVAL, "count_exact_stack: workspace must be device memory");
    const StackWs w = layout_stack((char*)opts->workspace, net->dev, cap, chunk);
    return count_stack_impl(net, prop, lo, hi, *opts, w, out);
}

// Split point for [a, b] near med on the grid A + k (B - A) 2^-bits, kept one step inside (a, b);
// intervals narrower than two steps are bisected at the midpoint.
static double snap_split(double med, double a, double b, double A, double B, int bits) {
    const double h = (B - A) * std::ldexp(1.0, -bits);
    if (b - a < 2.0 * h || h <= 0.0) return 0.5 * (a + b);
    double k = std::floor((med - A) / h + 0.5);
    const double k_lo = std::floor((a - A) / h + 0.5) + 1;
    const double k_hi = std::floor((b - A) / h + 0.5) - 1;
    k = std::min(std::max(k, k_lo), k_hi);
    return A + k * h;
}

namespace {

// One trial of the approximate count: halve the subdomain until count_exact resolves it (or the
// split cap or the grid stops it); returns the trial's estimate 2^s v f in *E.  Every draw is a
// Philox4x32-10 block keyed by the seed with counters (point/dimension, split, trial, tag), so a
// trial's result does not depend on which thread or stream runs it.
int approx_trial(const slr_net* net, const slr_property* prop, const double* lo, const double* hi,
                 const slr_approx_opts& o, const slr_exact_opts& leaf, const Workspace& w, int t,
                 double* E, int32_t* n_splits) {
    const int d = net->dev.d;
    const uint32_t key[2] = {(uint32_t)(o.seed & 0xFFFFFFFFu), (uint32_t)(o.seed >> 32)};
    hipStream_t s = (hipStream_t)leaf.stream;
    std::vector<double> slo(lo, lo + d), shi(hi, hi + d), coords;
    std::vector<float> pts((size_t)o.samples * d);
    std::vector<int8_t> viol(o.samples);
    int splits = 0;
    slr_count_result r;
    while (true) {
        memset(&r, 0, sizeof r);
        const int rc = count_exact_impl(net, prop, slo.data(), shi.data(), &leaf, w, &r);
        if (rc < 0) return rc;
        if (r.undecided <= o.resolve_tol || splits >= o.max_splits) break;
        // uniform samples of the subdomain (float64 arithmetic, rounded to float32)
        for (int p = 0; p < o.samples; ++p)
            for (int k = 0; k < d; ++k) {
                const uint64_t q = (uint64_t)p * d + k;
                const uint32_t ctr[4] = {(uint32_t)(q >> 1), (uint32_t)splits, (uint32_t)t, kTagSample};
                uint32_t wv[4];
                Philox::block(ctr, key, wv);
                const double u = (q & 1) ? Philox::u53(wv[2], wv[3]) : Philox::u53(wv[0], wv[1]);
                pts[(size_t)p * d + k] = (float)(slo[k] + u * (shi[k] - slo[k]));
            }
        HIP_TRY(hipMemcpyAsync(w.samples, pts.data(), pts.size() * sizeof(float), hipMemcpyHostToDevice, s), "count_approx: samples");
        HIP_TRY(launch_sample_forward(net->dev, prop->dev, o.samples, w.samples, w.viol, s), "count_approx: sample kernel");
        HIP_TRY(hipMemcpyAsync(viol.data(), w.viol, o.samples, hipMemcpyDeviceToHost, s), "count_approx: readback");
        HIP_TRY(hipStreamSynchronize(s), "count_approx: sync");
        const uint32_t sctr[4] = {0u, (uint32_t)splits, (uint32_t)t, kTagSplit};
        uint32_t sw[4];
        Philox::block(sctr, key, sw);
        const int dim = (int)(((uint64_t)sw[0] * (uint64_t)d) >> 32);
        const int side = (int)(sw[1] & 1u);
        // a side as narrow as two grid steps is not split further: the trial stops here (the
        // bound holds for any stopping rule; this keeps every leaf bisection exact in float32)
        // (a side of zero width, a degenerate side of the domain, stops it too)
        const double side_w = shi[dim] - slo[dim];
        if (side_w < 2.0 * (hi[dim] - lo[dim]) * std::ldexp(1.0, -o.grid_bits) || side_w <= 0.0) break;
        coords.clear();
        for (int p = 0; p < o.samples; ++p)
            if (viol[p]) coords.push_back(pts[(size_t)p * d + dim]);
        if (coords.empty())
            for (int p = 0; p < o.samples; ++p) coords.push_back(pts[(size_t)p * d + dim]);
        std::sort(coords.begin(), coords.end());
        const double med = coords[(coords.size() - 1) / 2];
        const double m = snap_split(med, slo[dim], shi[dim], lo[dim], hi[dim], o.grid_bits);
        if ((double)(float)m != m) return fail(SLR_EINTERNAL, "count_approx: split point not exact in float32");
        if (side == 0) shi[dim] = m; else slo[dim] = m;
        ++splits;
    }
    double v = 1.0;
    for (int k = 0; k < d; ++k)
        if (hi[k] > lo[k]) v *= (shi[k] - slo[k]) / (hi[k] - lo[k]);
    *E = std::ldexp(v * r.unsafe, splits);
    *n_splits = splits;
    return SLR_OK;
}

}  // namespace

extern "C" int count_approx(const slr_net* net, const slr_property* prop, const double* lo,
                            const double* hi, const slr_approx_opts* opts, slr_approx_result* out) {
    g_err.clear();
    int rc = check_pair(net, prop, "count_approx");
    if (rc) return rc;
    if (!out || !opts) return fail(SLR_EINVAL, "count_approx: NULL argument");
    if ((rc = check_box(net, lo, hi, "count_approx"))) return rc;
    const slr_approx_opts o = *opts;
    if (o.trials < 1 || o.trials > 64) return fail(SLR_EINVAL, "count_approx: trials must be in [1, 64]");
    if (o.samples < 1 || o.samples > 65536) return fail(SLR_EINVAL, "count_approx: samples must be in [1, 65536]");
    if (!(o.confidence > 0.0 && o.confidence < 1.0)) return fail(SLR_EINVAL, "count_approx: confidence must be in (0, 1)");
    if (o.max_splits < 0 || o.max_splits > 1000) return fail(SLR_EINVAL, "count_approx: max_splits must be in [0, 1000]");
    if (o.grid_bits < 1 || o.grid_bits > 20) return fail(SLR_EINVAL, "count_approx: grid_bits must be in [1, 20]");
    if (!(o.resolve_tol >= 0.0)) return fail(SLR_EINVAL, "count_approx: resolve_tol must be >= 0");
    if (o.concurrency < 0 || o.concurrency > 64) return fail(SLR_EINVAL, "count_approx: concurrency must be in [0, 64]");
    if (o.concurrency > 1)
        return fail(SLR_EUNSUPPORTED, "count_approx: concurrent trials are disabled (a profiled run of "
                    "the threaded form crashed inside hipEventRecord; cause not found); use 0 or 1");
    Workspace w;
    if ((rc = check_exact_opts(net, prop, &o.leaf, o.samples, &w, "count_approx"))) return rc;
    memset(out, 0, sizeof *out);
    const auto t0 = std::chrono::steady_clock::now();
    for (int t = 0; t < o.trials; ++t)
        if ((rc = approx_trial(net, prop, lo, hi, o, o.leaf, w, t, &out->estimate[t], &out->splits[t])) < 0)
            return rc;
    double best = INFINITY;
    for (int t = 0; t < o.trials; ++t) best = std::min(best, out->estimate[t]);
    const double beta = std::log2(1.0 / (1.0 - o.confidence)) / o.trials;
    out->trials = o.trials;
    out->lower_bound = std::exp2(-beta) * best;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SLR_OK;
}

// ------------------------------------------------------------------------------------------
// Batches of independent exact counts
// ------------------------------------------------------------------------------------------
struct slr_batch {
    int n_inst = 0, levels = 0;
    int pk_max = 0;                   // deepest one-pass top of the tree among the instances
    int d_max = 0;                    // largest input dimension among the instances
    std::vector<int> order;           // device position -> caller index
    void* mem = nullptr;
    BatchInst* insts = nullptr;
    BatchCtl* ctl = nullptr;
    unsigned *bpre = nullptr, *cpre = nullptr, *amb = nullptr;
    struct Cls {
        int ncol;
        TileShape t;
        int cbeg, cend, blocks;
        size_t lds;
    };
    std::vector<Cls> cls;
    // alpha pass (batch_create_opts with alpha_steps > 0)
    struct ACls {
        int key;
        size_t lds;
        BatchAlphaBuf buf;
    };
    std::vector<ACls> acls;
    BatchAlphaBuf* abufs = nullptr;   // device copy of the classes' buffers
    unsigned* tile_cand = nullptr;
    int alpha_steps = 0;
    float alpha_lr = 0.1f, alpha_select = 0.f;
    int nrow = 0, ncol_max = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BatchInst> host;
};

namespace {

// The whole batch count: init, then every level's fixed launch sequence, then the volumes.
int batch_enqueue(const slr_batch* b, hipStream_t s) {
    HIP_TRY(launch_batch_init(b->insts, b->n_inst, s), "batch: init kernel");
    HIP_TRY(launch_batch_prefix(b->insts, b->n_inst, b->pk_max, b->d_max, s), "batch: prefix kernel");
    for (int t = 0; t < b->levels; ++t) {
        HIP_TRY(launch_batch_plan(b->insts, b->n_inst, b->ctl, b->bpre, b->cpre, (int)b->cls.size(), s),
                "batch: plan kernel");
        for (size_t c = 0; c < b->cls.size(); ++c) {
            const auto& k = b->cls[c];
            HIP_TRY(launch_batch_bound(k.ncol, k.t, k.blocks, k.lds, b->insts, b->ctl, b->bpre,
                                       k.cbeg, k.cend, (int)c, b->amb, s),
                    "batch: bound kernel");
        }
        HIP_TRY(launch_batch_recheck(b->insts, b->ctl, b->amb, b->nrow, b->ncol_max, s), "batch: recheck kernel");
        if (t == 0)
            HIP_TRY(launch_batch_prefix_replay(b->insts, b->n_inst, b->pk_max, b->ctl, b->amb, s),
                    "batch: prefix replay kernel");
        if (!b->acls.empty()) {
            HIP_TRY(launch_batch_alpha_cand(b->insts, b->n_inst, b->ctl, b->cpre, b->tile_cand,
                                            b->alpha_select, s), "batch: alpha candidate kernel");
            HIP_TRY(launch_batch_alpha_plan(b->insts, b->ctl, b->abufs, (int)b->acls.size(), s),
                    "batch: alpha plan kernel");
            HIP_TRY(launch_batch_alpha_gather(b->insts, b->n_inst, b->ctl, b->cpre, b->tile_cand,
                                              b->abufs, b->alpha_select, s), "batch: alpha gather kernel");
            AlphaArgs base{};
            base.lr = b->alpha_lr;
            base.beta1 = 0.9f;
            base.beta2 = 0.999f;
            base.eps = 1e-8f;
            for (size_t c = 0; c < b->acls.size(); ++c)
                HIP_TRY(launch_batch_alpha_class(b->acls[c].key, b->acls[c].lds, b->insts, b->ctl, (int)c,
                                                 b->acls[c].buf, base, b->alpha_steps, s),
                        "batch: alpha kernels");
        }
        HIP_TRY(launch_batch_count(b->insts, b->n_inst, b->ctl, b->cpre, s), "batch: count kernel");
        HIP_TRY(launch_batch_advance(b->insts, b->n_inst, s), "batch: advance kernel");
        HIP_TRY(launch_batch_split(b->insts, b->n_inst, b->ctl, b->cpre, s), "batch: split kernel");
    }
    HIP_TRY(launch_batch_volume(b->insts, b->n_inst, s), "batch: volume kernel");
    return SLR_OK;
}

}  // namespace

extern "C" void batch_free(slr_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

extern "C" int batch_create(int32_t n_inst, const slr_net* const* nets,
                            const slr_property* const* props, const double* const* lo,
                            const double* const* hi, const int32_t* max_depth,
                            const int64_t* max_leaves, int32_t use_graph, slr_batch** out) {
    slr_batch_opts o{};
    o.use_graph = use_graph;
    return batch_create_opts(n_inst, nets, props, lo, hi, max_depth, max_leaves, &o, out);
}

extern "C" int batch_create_opts(int32_t n_inst, const slr_net* const* nets,
                                 const slr_property* const* props, const double* const* lo,
                                 const double* const* hi, const int32_t* max_depth,
                                 const int64_t* max_leaves, const slr_batch_opts* opts,
                                 slr_batch** out) {
    g_err.clear();
    if (!out) return fail(SLR_EINVAL, "batch_create: out is NULL");
    *out = nullptr;
    if (!opts) return fail(SLR_EINVAL, "batch_create: opts is NULL");
    const int32_t use_graph = opts->use_graph;
    if (opts->alpha_steps < 0 || opts->alpha_steps > 1000)
        return fail(SLR_EINVAL, "batch_create: alpha_steps must be in [0, 1000]");
    if (!(opts->alpha_lr >= 0.f) || opts->alpha_min_depth < 0 || opts->alpha_chunk < 0)
        return fail(SLR_EINVAL, "batch_create: alpha_lr, alpha_min_depth and alpha_chunk must be >= 0");
    if (!(opts->alpha_select >= 0.f) || !std::isfinite(opts->alpha_select))
        return fail(SLR_EINVAL, "batch_create: alpha_select must be finite and >= 0");
    if (n_inst < 1 || n_inst > SLR_MAX_BATCH)
        return fail(SLR_EINVAL, "batch_create: n_inst must be in [1, %d]", SLR_MAX_BATCH);
    if (!nets || !props || !lo || !hi || !max_depth || !max_leaves)
        return fail(SLR_EINVAL, "batch_create: NULL array");
    if (use_graph != 0 && use_graph != 1) return fail(SLR_EINVAL, "batch_create: use_graph must be 0 or 1");
    struct Info {
        int ncol;
        TileShape t;
        int key;
    };
    std::vector<Info> info(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        char who[64];
        snprintf(who, sizeof who, "batch_create: instance %d", i);
        int rc = check_pair(nets[i], props[i], who);
        if (rc) return rc;
        if ((rc = check_box(nets[i], lo[i], hi[i], who))) return rc;
        if (max_depth[i] < 0 || max_depth[i] > kMaxLevels - 1)
            return fail(SLR_EINVAL, "%s: max_depth must be in [0, %d]", who, kMaxLevels - 1);
        if (max_leaves[i] < 1 || max_leaves[i] > (1 << 22))
            return fail(SLR_EINVAL, "%s: max_leaves must be in [1, 2^22]", who);
        Info& f = info[i];
        if (batch_class_of(nets[i]->dev, props[i]->dev, &f.ncol, &f.t) != 0)
            return fail(SLR_EUNSUPPORTED, "%s: shape (d=%d, widths up to %d) outside the batch kernels "
                        "(d <= 11, widths <= 128)", who, nets[i]->dev.d, nets[i]->dev.n_max);
        f.key = ((f.ncol * 16 + (f.t.nt + 8)) * 8 + f.t.uw) * 16 + f.t.nw;   // nt < 0: smooth kernels
    }
    slr_batch* b = new slr_batch;
    b->n_inst = n_inst;
    b->order.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return info[x].key < info[y].key; });
    // classes, in device order
    std::vector<int> cls_of(n_inst);
    for (int p = 0; p < n_inst; ++p) {
        const Info& f = info[b->order[p]];
        if (b->cls.empty() || b->cls.back().ncol != f.ncol || b->cls.back().t.nt != f.t.nt ||
            b->cls.back().t.uw != f.t.uw || b->cls.back().t.nw != f.t.nw) {
            if ((int)b->cls.size() == SLR_MAX_CLASSES) {
                batch_free(b);
                return fail(SLR_EINTERNAL, "batch_create: too many kernel classes");
            }
            b->cls.push_back({f.ncol, f.t, p, p, 0, 0});
        }
        b->cls.back().cend = p + 1;
        cls_of[p] = (int)b->cls.size() - 1;
    }
    // device memory: control block, offsets, FP64 list, then per-instance regions
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    const size_t o_insts = take(sizeof(BatchInst) * n_inst);
    const size_t o_ctl = take(sizeof(BatchCtl));
    const size_t o_bpre = take(sizeof(unsigned) * (n_inst + 1));
    const size_t o_cpre = take(sizeof(unsigned) * (n_inst + 1));
    size_t amb_cap = 0;
    for (int i = 0; i < n_inst; ++i) amb_cap += (size_t)max_leaves[i];
    const size_t o_amb = take(sizeof(unsigned) * amb_cap);
    struct Reg {
        size_t lo[2], hi[2], path[2], cls, tile_und, stats, root;
    };
    std::vector<Reg> reg(n_inst);
    for (int p = 0; p < n_inst; ++p) {
        const int i = b->order[p];
        const int d = nets[i]->dev.d;
        const int64_t cap = max_leaves[i];
        Reg& r = reg[p];
        for (int k = 0; k < 2; ++k) {
            r.lo[k] = take(sizeof(float) * d * cap);
            r.hi[k] = take(sizeof(float) * d * cap);
            r.path[k] = take(sizeof(unsigned long long) * cap);
        }
        r.cls = take(cap);
        r.tile_und = take(sizeof(unsigned) * level_tiles(cap));
        r.stats = take(sizeof(LevelStats) * SLR_MAX_LEVELS);
        r.root = take(sizeof(float) * 2 * d);
    }
    // alpha pass: classes by kernel template, plain bounds per instance, class buffers
    const bool use_alpha = opts->alpha_steps > 0;
    std::vector<int> akey(n_inst, -1), acls_of(n_inst, -1);
    std::vector<size_t> aglo(n_inst, 0), aghi(n_inst, 0);
    std::vector<std::vector<int>> ainst;
    struct ARegs {
        size_t lo, hi, alpha, m, v, glo, ghi, blo, bhi, cls, obj, list, seg, inst, tape;
    };
    std::vector<ARegs> areg;
    size_t o_abufs = 0, o_tcand = 0;
    if (use_alpha) {
        b->alpha_steps = opts->alpha_steps;
        b->alpha_lr = opts->alpha_lr > 0.f ? opts->alpha_lr : 0.1f;
        b->alpha_select = opts->alpha_select;
        const unsigned cap = (unsigned)(((opts->alpha_chunk > 0 ? opts->alpha_chunk : 8192) + 15) / 16 * 16);
        size_t ctiles = 0;
        for (int p = 0; p < n_inst; ++p) {
            const int i = b->order[p];
            size_t lds = 0;
            akey[p] = batch_alpha_key(nets[i]->dev, props[i]->dev, &lds);
            if (nets[i]->dev.act != SLR_ACT_RELU) {
                batch_free(b);
                return fail(SLR_EUNSUPPORTED, "batch_create: instance %d: alpha slopes are defined for ReLU networks only", i);
            }
            if (akey[p] < 0) {
                batch_free(b);
                return fail(SLR_EUNSUPPORTED, "batch_create: instance %d has no alpha kernel", i);
            }
            int c = -1;
            for (size_t k = 0; k < b->acls.size(); ++k)
                if (b->acls[k].key == akey[p]) c = (int)k;
            if (c < 0) {
                if ((int)b->acls.size() == SLR_MAX_CLASSES) {
                    batch_free(b);
                    return fail(SLR_EINTERNAL, "batch_create: too many alpha classes");
                }
                b->acls.push_back({akey[p], 0, BatchAlphaBuf{}});
                ainst.emplace_back();
                c = (int)b->acls.size() - 1;
                b->acls[c].buf.cap = cap;
            }
            acls_of[p] = c;
            ainst[c].push_back(p);
            auto& A = b->acls[c];
            A.lds = std::max(A.lds, lds);
            A.buf.dmax = std::max(A.buf.dmax, nets[i]->dev.d);
            A.buf.nhmax = std::max(A.buf.nhmax, nets[i]->dev.nh);
            A.buf.rowsmax = std::max(A.buf.rowsmax, props[i]->dev.rows);
            aglo[p] = take(sizeof(float) * props[i]->dev.rows * (size_t)max_leaves[i]);
            aghi[p] = take(sizeof(float) * props[i]->dev.rows * (size_t)max_leaves[i]);
            ctiles += level_tiles(max_leaves[i]);
        }
        o_tcand = take(sizeof(unsigned) * ctiles);
        o_abufs = take(sizeof(BatchAlphaBuf) * b->acls.size());
        areg.resize(b->acls.size());
        for (size_t c = 0; c < b->acls.size(); ++c) {
            const BatchAlphaBuf& B = b->acls[c].buf;
            size_t tile_floats = 0;
            for (int p : ainst[c]) {
                const int i = b->order[p];
                const AlphaShape sh = alpha_shape(nets[i]->dev, props[i]->dev);
                tile_floats = std::max(tile_floats, (size_t)sh.slots * sh.slot_floats);
            }
            ARegs& r = areg[c];
            r.lo = take(sizeof(float) * B.cap * B.dmax);
            r.hi = take(sizeof(float) * B.cap * B.dmax);
            r.alpha = take(sizeof(float) * B.cap * B.nhmax);
            r.m = take(sizeof(float) * B.cap * B.nhmax);
            r.v = take(sizeof(float) * B.cap * B.nhmax);
            r.glo = take(sizeof(float) * B.cap * B.rowsmax);
            r.ghi = take(sizeof(float) * B.cap * B.rowsmax);
            r.blo = take(sizeof(float) * B.cap * B.rowsmax);
            r.bhi = take(sizeof(float) * B.cap * B.rowsmax);
            r.cls = take(B.cap);
            r.obj = take(2 * (size_t)B.cap);
            r.list = take(sizeof(unsigned) * B.cap);
            r.seg = take(sizeof(unsigned) * ainst[c].size());
            r.inst = take(sizeof(int) * ainst[c].size());
            r.tape = take(sizeof(float) * (B.cap / 16) * tile_floats);
        }
    }
    hipError_t e = hipMalloc(&b->mem, o);
    if (e != hipSuccess) {
        delete b;
        return fail(SLR_ENOMEM, "batch_create: hipMalloc(%zu): %s", o, hipGetErrorString(e));
    }
    char* base = (char*)b->mem;
    b->insts = (BatchInst*)(base + o_insts);
    b->ctl = (BatchCtl*)(base + o_ctl);
    b->bpre = (unsigned*)(base + o_bpre);
    b->cpre = (unsigned*)(base + o_cpre);
    b->amb = (unsigned*)(base + o_amb);
    if (use_alpha) {
        b->tile_cand = (unsigned*)(base + o_tcand);
        b->abufs = (BatchAlphaBuf*)(base + o_abufs);
        for (size_t c = 0; c < b->acls.size(); ++c) {
            BatchAlphaBuf& B = b->acls[c].buf;
            const ARegs& r = areg[c];
            B.lo = (float*)(base + r.lo);
            B.hi = (float*)(base + r.hi);
            B.alpha = (float*)(base + r.alpha);
            B.m = (float*)(base + r.m);
            B.v = (float*)(base + r.v);
            B.glo = (float*)(base + r.glo);
            B.ghi = (float*)(base + r.ghi);
            B.blo = (float*)(base + r.blo);
            B.bhi = (float*)(base + r.bhi);
            B.cls = (int8_t*)(base + r.cls);
            B.obj = (int8_t*)(base + r.obj);
            B.list = (unsigned*)(base + r.list);
            B.seg = (unsigned*)(base + r.seg);
            B.tape = (float*)(base + r.tape);
            B.inst = (const int*)(base + r.inst);
            B.ninst = (int)ainst[c].size();
            e = hipMemcpy(base + r.inst, ainst[c].data(), sizeof(int) * ainst[c].size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                batch_free(b);
                return hip_fail(e, "batch_create: upload");
            }
            e = batch_alpha_prepare(b->acls[c].key, b->acls[c].lds);
            if (e != hipSuccess) {
                batch_free(b);
                return hip_fail(e, "batch_create: alpha kernel");
            }
        }
        std::vector<BatchAlphaBuf> hb;
        for (auto& a : b->acls) hb.push_back(a.buf);
        e = hipMemcpy(b->abufs, hb.data(), sizeof(BatchAlphaBuf) * hb.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            batch_free(b);
            return hip_fail(e, "batch_create: upload");
        }
    }
    b->host.assign(n_inst, BatchInst{});
    int levels = 0;
    for (int p = 0; p < n_inst; ++p) {
        const int i = b->order[p];
        BatchInst& I = b->host[p];
        const Reg& r = reg[p];
        I.net = nets[i]->dev;
        I.prop = props[i]->dev;
        for (int k = 0; k < 2; ++k) {
            I.lo[k] = (float*)(base + r.lo[k]);
            I.hi[k] = (float*)(base + r.hi[k]);
            I.path[k] = (unsigned long long*)(base + r.path[k]);
        }
        I.cls = (int8_t*)(base + r.cls);
        I.tile_und = (unsigned*)(base + r.tile_und);
        I.stats = (LevelStats*)(base + r.stats);
        I.root = (const float*)(base + r.root);
        I.d = I.net.d;
        I.max_depth = max_depth[i];
        I.max_leaves = max_leaves[i];
        I.cls_id = cls_of[p];
        I.sp = state_stride(I.net.mt_max);
        I.acls_id = -1;
        if (use_alpha) {
            const AlphaShape sh = alpha_shape(I.net, I.prop);
            I.glo = (float*)(base + aglo[p]);
            I.ghi = (float*)(base + aghi[p]);
            I.acls_id = acls_of[p];
            I.alpha_min_depth = opts->alpha_min_depth;
            I.aslots = sh.slots;
            I.atile_floats = (unsigned long long)sh.slots * sh.slot_floats;
        }
        // depths 0 .. pk in the first level (complete subtree within the leaf budget, below the
        // first alpha depth)
        int pk = std::min(15, max_depth[i]);
        while (pk > 0 && ((int64_t)2 << pk) - 1 > max_leaves[i]) --pk;
        if (use_alpha) pk = std::min(pk, opts->alpha_min_depth - 1);
        I.pk = pk >= 4 ? pk : 0;
        b->pk_max = std::max(b->pk_max, I.pk);
        b->d_max = std::max(b->d_max, I.d);
        levels = std::max(levels, max_depth[i] - I.pk + 1);
        std::vector<float> root(2 * I.d);
        for (int k = 0; k < I.d; ++k) {
            root[k] = (float)lo[i][k];
            root[I.d + k] = (float)hi[i][k];
        }
        e = hipMemcpy(base + r.root, root.data(), root.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            batch_free(b);
            return hip_fail(e, "batch_create: upload");
        }
        b->cls[cls_of[p]].lds = std::max(b->cls[cls_of[p]].lds,
                                         batch_bound_lds(b->cls[cls_of[p]].ncol, b->cls[cls_of[p]].t,
                                                         I.net.mt_max, I.prop.rows));
        const int ncol = I.d + 2;
        b->ncol_max = std::max(b->ncol_max, ncol);
        b->nrow = std::max(b->nrow, std::max(I.net.n_max, I.prop.rows * ncol));
    }
    b->levels = levels;
    BatchCtl hc{};
    for (size_t c = 0; c < b->cls.size(); ++c) hc.tbox[c] = 16 * std::abs(b->cls[c].t.nt);
    e = hipMemcpy(b->ctl, &hc, sizeof hc, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->insts, b->host.data(), sizeof(BatchInst) * n_inst, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch_create: upload");
    }
    for (auto& k : b->cls) {
        if (k.lds > 160 * 1024) {
            batch_free(b);
            return fail(SLR_EUNSUPPORTED, "batch_create: a kernel class needs %zu bytes of LDS", k.lds);
        }
        e = batch_prepare_class(k.ncol, k.t, k.lds, &k.blocks);
        if (e != hipSuccess) {
            batch_free(b);
            return hip_fail(e, "batch_create: kernel class");
        }
    }
    e = batch_prepare_recheck(b->nrow, b->ncol_max);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch_create: recheck kernel");
    }
    if (use_graph) {
        // capture the launch sequence once on a private stream (default priority)
        e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            batch_free(b);
            return hip_fail(e, "batch_create: capture");
        }
        int rc = batch_enqueue(b, b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        b->graph = g;
        if (rc) {
            const std::string msg = g_err;
            batch_free(b);
            return fail(rc, "%s", msg.c_str());
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            batch_free(b);
            return hip_fail(e, "batch_create: graph");
        }
    }
    *out = b;
    return SLR_OK;
}

extern "C" int batch_run(slr_batch* b, void* stream, slr_count_result* results) {
    g_err.clear();
    if (!b || !results) return fail(SLR_EINVAL, "batch_run: NULL argument");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        HIP_TRY(hipGraphLaunch(b->exec, s), "batch_run: graph launch");
    } else {
        int rc = batch_enqueue(b, s);
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(b->host.data(), b->insts, sizeof(BatchInst) * b->n_inst, hipMemcpyDeviceToHost, s),
            "batch_run: readback");
    HIP_TRY(hipStreamSynchronize(s), "batch_run: sync");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = SLR_OK;
    for (int p = 0; p < b->n_inst; ++p) {
        const BatchInst& I = b->host[p];
        if (I.err & 1u) return fail(SLR_EINTERNAL, "batch_run: instance %d: a bisection midpoint is not exact in float32", b->order[p]);
        if (I.err & 2u) return fail(SLR_EINTERNAL, "batch_run: instance %d: leaf volumes do not sum to the box volume", b->order[p]);
        if (I.err & 4u) return fail(SLR_EINTERNAL, "batch_run: instance %d: level counts do not add up", b->order[p]);
        if (I.active) return fail(SLR_EINTERNAL, "batch_run: instance %d did not finish", b->order[p]);
        slr_count_result& r = results[b->order[p]];
        memset(&r, 0, sizeof r);
        r.unsafe = I.vol[0];
        r.safe = I.vol[1];
        r.undecided = I.vol[2];
        r.n_unsafe = (int64_t)I.counts[0];
        r.n_safe = (int64_t)I.counts[1];
        r.n_undecided = (int64_t)I.counts[2];
        r.n_boxes_bounded = I.bounded;
        r.n_recheck64 = (int64_t)I.rechecks;
        r.depth_reached = I.levels - 1;
        r.status = I.status;
        r.seconds = secs;
        r.n_alpha_boxes = I.n_alpha_boxes;
        r.n_alpha_decided = I.n_alpha_decided;
        if (I.status == SLR_BUDGET) worst = SLR_BUDGET;
    }
    return worst;
}

extern "C" int count_exact_batch(int32_t n_inst, const slr_net* const* nets,
                                 const slr_property* const* props, const double* const* lo,
                                 const double* const* hi, const int32_t* max_depth,
                                 const int64_t* max_leaves, void* stream, slr_count_result* results) {
    slr_batch* b = nullptr;
    int rc = batch_create(n_inst, nets, props, lo, hi, max_depth, max_leaves, 0, &b);
    if (rc) return rc;
    rc = batch_run(b, stream, results);
    batch_free(b);
    return rc;
}
