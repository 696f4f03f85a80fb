// Learned densifier (Sec. III-A) host side: parameter registry, forward and backward
// sequencing over the NN kernels, AdamW, checkpoints, training-pair generation and the
// densified single-bounce solve (Sec. III-A output feeding Eq. (14)).
//
// Network (one shared encoder, three decoder heads; channels C = base x (1, 2, 4, 8)):
//   stem 3x3 conv (1 -> C0) + GELU; level 0 ConvNeXt block; for l = 1..3: 2x2 max-pool,
//   1x1 conv C[l-1] -> C[l], ConvNeXt block (depthwise 7x7, LayerNorm, 1x1 x4 + GELU, 1x1,
//   residual).  Each head (depth 1, normal 3, hit logit 1): for l = 3, 2, 1: 3x3 conv
//   C[l] -> 4 C[l-1] + pixel shuffle, concatenation with the level l-1 skip, 3x3 conv
//   2 C[l-1] -> C[l-1] + GELU; then 3x3 conv C0 -> 4 co + pixel shuffle: outputs at twice
//   the input resolution.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pe_gfb.h"
#include "pe_nn.h"
#include "pe_runtime.h"

namespace pe {

enum : int { B_GFB_COARSE = 34, B_GFB_DEPTH, B_GFB_NRM, B_GFB_PROB, B_GFB_CNT, B_GFB_USE };

constexpr int kHeads = 3;
constexpr int kHeadCo[kHeads] = {1, 3, 1};
constexpr int kPadCo = 32;       // padded channel count of the head-output gradients
constexpr int kNetBatch = 8;     // incidences per network batch in a densified solve
constexpr float kLnEps = 1e-6f;
constexpr int kRowChunk = 64;    // rows per partial of the column-sum style gradient reductions

struct Tensor {
    std::string name;
    uint64_t off = 0, n = 0;
    int shape[4] = {0, 0, 0, 0};  // unused trailing dims 0
};

struct ConvL {
    int w = -1, b = -1;
    int co = 0, k = 0, ci = 0;
    int co_pad = 0;
    uint64_t wt_off = 0;
};

struct BlockL {
    int dww = -1, dwb = -1, lng = -1, lnb = -1;
    ConvL pw1, pw2;
};

// Activation and gradient buffers of one (N, H, W) shape, carved from one arena.
struct Acts {
    uint16_t* stem_z = nullptr;
    uint16_t *bx[4] = {}, *dwo[4] = {}, *lno[4] = {}, *z1[4] = {}, *a1[4] = {}, *sk[4] = {};
    float* lst[4] = {};
    uint16_t* pooled[4] = {};
    uint8_t* arg[4] = {};
    uint16_t *cat[kHeads][4] = {}, *zf[kHeads][4] = {}, *u[kHeads][4] = {};
    float* out32[kHeads] = {};
    // backward
    uint16_t* dsk[4] = {};
    uint16_t *dzo = nullptr, *du = nullptr, *dzf = nullptr, *dcat = nullptr, *dzu = nullptr;
    uint16_t *t4 = nullptr, *dln = nullptr, *ddw = nullptr, *dxdw = nullptr, *dp = nullptr;
    float *gd = nullptr, *gn = nullptr, *gl = nullptr, *w4 = nullptr, *lpart = nullptr;
    float *ogd = nullptr, *ogn = nullptr, *ogl = nullptr;
    double* sums = nullptr;
    float* part = nullptr;
};

static uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// splitmix64 (Steele, Lea and Flood) + Box-Muller normals for the initial weights.
struct InitRng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uni() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double a = uni(), b = uni();
        return std::sqrt(-2.0 * std::log(a)) * std::cos(6.283185307179586 * b);
    }
};

}  // namespace pe

using namespace pe;

struct pe_densifier_s {
    pe_ctx ctx = nullptr;
    int base = 0;
    int C[4] = {0, 0, 0, 0};
    std::vector<Tensor> T;
    uint64_t n_params = 0;
    ConvL stem;
    BlockL enc[4];
    ConvL down[4];
    ConvL up[kHeads][4], fuse[kHeads][4], out[kHeads];
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    uint16_t* pb = nullptr;
    uint16_t* wt = nullptr;
    uint64_t wt_n = 0;
    float* dwt[4] = {nullptr, nullptr, nullptr, nullptr};  // tap-major depthwise weights
    int step = 0;
    std::mutex mu;
    std::vector<std::pair<void*, size_t>> allocs;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    int aN = -1, aH = -1, aW = -1;
    Acts A;

    void* alloc(size_t b) {
        void* q = ctx_alloc(ctx, b);
        allocs.push_back({q, b});
        return q;
    }
    ~pe_densifier_s() {
        if (arena) ctx_free(ctx, arena, arena_bytes);
        for (auto& a : allocs) ctx_free(ctx, a.first, a.second);
    }

    int add(const std::string& name, std::initializer_list<int> shape) {
        Tensor t;
        t.name = name;
        t.n = 1;
        int i = 0;
        for (int s : shape) {
            t.shape[i++] = s;
            t.n *= (uint64_t)s;
        }
        t.off = n_params;
        n_params = round_up(n_params + t.n, 64);
        T.push_back(t);
        return (int)T.size() - 1;
    }
    ConvL conv(const std::string& name, int co, int k, int ci) {
        ConvL c;
        c.w = add(name + ".w", {co, k, k, ci});
        c.b = add(name + ".b", {co});
        c.co = co;
        c.k = k;
        c.ci = ci;
        c.co_pad = (int)round_up((uint64_t)co, kPadCo);
        c.wt_off = wt_n;
        wt_n = round_up(wt_n + (uint64_t)ci * k * k * c.co_pad, 64);
        return c;
    }
    BlockL block(const std::string& name, int c) {
        BlockL b;
        b.dww = add(name + ".dw.w", {c, 7, 7});
        b.dwb = add(name + ".dw.b", {c});
        b.lng = add(name + ".ln.g", {c});
        b.lnb = add(name + ".ln.b", {c});
        b.pw1 = conv(name + ".pw1", 4 * c, 1, c);
        b.pw2 = conv(name + ".pw2", c, 1, 4 * c);
        return b;
    }
    void build_registry() {
        for (int l = 0; l < 4; l++) C[l] = base << l;
        stem.w = add("stem.w", {C[0], 3, 3, 1});
        stem.b = add("stem.b", {C[0]});
        stem.co = C[0];
        stem.k = 3;
        stem.ci = 1;
        enc[0] = block("enc0", C[0]);
        for (int l = 1; l < 4; l++) {
            down[l] = conv("down" + std::to_string(l), C[l], 1, C[l - 1]);
            enc[l] = block("enc" + std::to_string(l), C[l]);
        }
        static const char* hn[kHeads] = {"depth", "nrm", "mask"};
        for (int h = 0; h < kHeads; h++) {
            for (int l = 3; l >= 1; l--) {
                up[h][l] = conv(std::string(hn[h]) + ".up" + std::to_string(l), 4 * C[l - 1], 3, C[l]);
                fuse[h][l] = conv(std::string(hn[h]) + ".fuse" + std::to_string(l), C[l - 1], 3,
                                  2 * C[l - 1]);
            }
            out[h] = conv(std::string(hn[h]) + ".out", 4 * kHeadCo[h], 3, C[0]);
        }
    }
    std::vector<float> init_values(uint64_t seed) const {
        std::vector<float> h(n_params, 0.f);
        InitRng r{seed * 0x2545F4914F6CDD1Dull + 1};
        for (const Tensor& t : T) {
            const std::string& nm = t.name;
            double mean = 0, sd = 0;
            auto ends = [&](const char* s) {
                const size_t l = std::strlen(s);
                return nm.size() >= l && nm.compare(nm.size() - l, l, s) == 0;
            };
            if (ends(".dw.w")) sd = std::sqrt(2.0 / 49.0);
            else if (ends(".ln.g")) { mean = 1.0; sd = 0.05; }
            else if (ends(".ln.b")) sd = 0.05;
            else if (ends(".b")) sd = 0.01;
            else sd = std::sqrt(2.0 / ((double)t.shape[1] * t.shape[2] * t.shape[3]));
            for (uint64_t i = 0; i < t.n; i++) h[t.off + i] = (float)(mean + sd * r.normal());
        }
        return h;
    }

    float* P(int t) const { return p + T[t].off; }
    float* G(int t) const { return g + T[t].off; }
    uint16_t* PB(int t) const { return pb + T[t].off; }

    // ---------------------------------------------------------------- arena planning --
    size_t part_floats(int N, int H, int W) const;
    void plan(int N, int H, int W);

    // ------------------------------------------------------------------- primitives --
    void conv_fwd(const ConvL& c, const uint16_t* x, int ldx, int xoff, int N, int H, int W,
                  uint16_t* y, float* y32, int ldy, int yoff, int act, int shuffle, uint16_t* z,
                  const uint16_t* res, hipStream_t st) const {
        ConvArgs a{};
        a.x = x;
        a.ldx = ldx;
        a.xoff = xoff;
        a.N = N;
        a.H = H;
        a.W = W;
        a.Cin = c.ci;
        a.K = c.k;
        a.w = PB(c.w);
        a.Cout = c.co;
        a.Cout_store = c.co;
        a.bias = P(c.b);
        a.res = res;
        a.ldres = c.co;
        a.act = act;
        a.shuffle = shuffle;
        a.y = y;
        a.y32 = y32;
        a.ldy = ldy;
        a.yoff = yoff;
        a.z = z;
        launch_conv_fwd(a, st);
    }
    // dx = data gradient of conv c given dy (ld lddy >= co_pad, channels co..co_pad zero).
    void conv_dgrad(const ConvL& c, const uint16_t* dy, int lddy, int N, int H, int W,
                    uint16_t* dx, int lddx, int dxoff, hipStream_t st) const {
        ConvArgs a{};
        a.x = dy;
        a.ldx = lddy;
        a.N = N;
        a.H = H;
        a.W = W;
        a.Cin = c.co_pad;
        a.K = c.k;
        a.w = wt + c.wt_off;
        a.Cout = c.ci;
        a.Cout_store = c.ci;
        a.y = dx;
        a.ldy = lddx;
        a.yoff = dxoff;
        launch_conv_fwd(a, st);
    }
    static int wgrad_chunks(const ConvL& c, int M, int* chunk) {
        const int tiles = ((c.co + 63) / 64) * ((c.ci + 63) / 64) * c.k * c.k;
        int nch = std::max(1, std::min((1024 + tiles - 1) / tiles, (M + 255) / 256));
        const int ch = (int)round_up((uint64_t)((M + nch - 1) / nch), 32);
        *chunk = ch;
        return (M + ch - 1) / ch;
    }
    void conv_wgrad(const ConvL& c, const uint16_t* x, int ldx, int xoff, const uint16_t* dy,
                    int lddy, int N, int H, int W, hipStream_t st) const {
        const int M = N * H * W;
        int chunk = 0;
        const int nch = wgrad_chunks(c, M, &chunk);
        WgradArgs a{};
        a.x = x;
        a.ldx = ldx;
        a.xoff = xoff;
        a.dy = dy;
        a.lddy = lddy;
        a.N = N;
        a.H = H;
        a.W = W;
        a.Cin = c.ci;
        a.Cout = c.co;
        a.K = c.k;
        a.chunk = chunk;
        a.partial = A.part;
        launch_conv_wgrad(a, nch, st);
        const size_t n = (size_t)c.co * c.k * c.k * c.ci;
        launch_reduce_chunks(A.part, nch, n, n, (int)n, (int)n, 0, G(c.w), st);
        bias_grad(c.b, dy, lddy, M, c.co, st);
    }
    void bias_grad(int t, const uint16_t* dy, int lddy, int M, int C, hipStream_t st) const {
        const int nch = (M + kRowChunk - 1) / kRowChunk;
        launch_colsum(dy, M, lddy, 0, C, kRowChunk, A.part, st);
        launch_reduce_chunks(A.part, nch, C, C, C, C, 0, G(t), st);
    }

    void block_fwd(int l, int N, int H, int W, bool train, hipStream_t st) {
        const BlockL& b = enc[l];
        const int c = C[l], M = N * H * W;
        launch_dw_fwd(A.bx[l], N, H, W, c, dwt[l], P(b.dwb), A.dwo[l], st);
        launch_ln_fwd(A.dwo[l], M, c, P(b.lng), P(b.lnb), kLnEps, A.lno[l], A.lst[l], st);
        static const bool unfused = std::getenv("PE_NN_UNFUSED") != nullptr;
        if (!train && !unfused) {
            // inference keeps the hidden activation on chip (the same arithmetic; PE_NN_UNFUSED
            // selects the two separate convolutions)
            ConvArgs a{};
            a.x = A.lno[l];
            a.ldx = c;
            a.N = N;
            a.H = H;
            a.W = W;
            a.Cin = 4 * c;
            a.K = 1;
            a.w = PB(b.pw2.w);
            a.Cout = c;
            a.Cout_store = c;
            a.bias = P(b.pw2.b);
            a.res = A.bx[l];
            a.ldres = c;
            a.y = A.sk[l];
            a.ldy = c;
            if (launch_mlp_fwd(a, PB(b.pw1.w), P(b.pw1.b), st)) return;
        }
        conv_fwd(b.pw1, A.lno[l], c, 0, N, H, W, A.a1[l], nullptr, 4 * c, 0, 1, 0,
                 train ? A.z1[l] : nullptr, nullptr, st);
        conv_fwd(b.pw2, A.a1[l], 4 * c, 0, N, H, W, A.sk[l], nullptr, c, 0, 0, 0, nullptr, A.bx[l],
                 st);
    }

    void forward(int N, int H, int W, const float* x, bool train, hipStream_t st) {
        for (int l = 0; l < 4; l++) launch_dw_wt(P(enc[l].dww), C[l], dwt[l], st);
        launch_stem_fwd(x, N, H, W, C[0], P(stem.w), P(stem.b), A.stem_z, A.bx[0], st);
        for (int l = 0; l < 4; l++) {
            const int Hl = H >> l, Wl = W >> l;
            if (l > 0) {
                launch_pool_fwd(A.sk[l - 1], N, H >> (l - 1), W >> (l - 1), C[l - 1], A.pooled[l],
                                A.arg[l], st);
                conv_fwd(down[l], A.pooled[l], C[l - 1], 0, N, Hl, Wl, A.bx[l], nullptr, C[l], 0, 0,
                         0, nullptr, nullptr, st);
            }
            block_fwd(l, N, Hl, Wl, train, st);
        }
        for (int h = 0; h < kHeads; h++) {
            const uint16_t* u = A.sk[3];
            // a training step keeps each head's concat buffer for its weight gradient; inference
            // runs the heads one after another through head 0's buffers, whose skip half then
            // needs copying once
            const int hc = train ? h : 0;
            for (int l = 3; l >= 1; l--) {
                const int c = C[l - 1], Hl = H >> l, Wl = W >> l;
                conv_fwd(up[h][l], u, C[l], 0, N, Hl, Wl, A.cat[hc][l - 1], nullptr, 2 * c, 0, 0, 1,
                         nullptr, nullptr, st);
                if (train || h == 0)
                    launch_copy_slice(A.sk[l - 1], c, 0, N * (Hl * 2) * (Wl * 2), c,
                                      A.cat[hc][l - 1], 2 * c, c, st);
                conv_fwd(fuse[h][l], A.cat[hc][l - 1], 2 * c, 0, N, 2 * Hl, 2 * Wl, A.u[h][l - 1],
                         nullptr, c, 0, 1, 0, train ? A.zf[h][l - 1] : nullptr, nullptr, st);
                u = A.u[h][l - 1];
            }
            conv_fwd(out[h], u, C[0], 0, N, H, W, nullptr, A.out32[h], kHeadCo[h], 0, 0, 1, nullptr,
                     nullptr, st);
            if (h == 0) launch_depth_base(A.out32[0], x, N, H, W, st);
        }
    }

    // Gradient of block l: dh = gradient w.r.t. the block output; returns the gradient w.r.t.
    // the block input in A.dxdw.
    void block_bwd(int l, const uint16_t* dh, int N, int H, int W, hipStream_t st) {
        const BlockL& b = enc[l];
        const int c = C[l], M = N * H * W;
        // pw2: y = x + pw2(a1)
        conv_wgrad(b.pw2, A.a1[l], 4 * c, 0, dh, c, N, H, W, st);
        conv_dgrad(b.pw2, dh, c, N, H, W, A.t4, 4 * c, 0, st);
        launch_gelu_bwd(A.z1[l], A.t4, (size_t)M * 4 * c, A.t4, st);
        conv_wgrad(b.pw1, A.lno[l], c, 0, A.t4, 4 * c, N, H, W, st);
        conv_dgrad(b.pw1, A.t4, 4 * c, N, H, W, A.dln, c, 0, st);
        // LayerNorm
        launch_ln_bwd(A.dwo[l], A.dln, M, c, P(b.lng), A.lst[l], A.ddw, st);
        {
            const int nch = (M + kRowChunk - 1) / kRowChunk;
            launch_ln_pgrad(A.dwo[l], A.dln, M, c, A.lst[l], kRowChunk, A.part, st);
            launch_reduce_chunks(A.part, nch, (size_t)2 * c, c, 1, 2, 0, G(b.lng), st);
            launch_reduce_chunks(A.part, nch, (size_t)2 * c, c, 1, 2, 1, G(b.lnb), st);
        }
        // depthwise 7x7
        launch_dw_dgrad(A.ddw, N, H, W, c, dwt[l], A.dxdw, st);
        {
            const int nch = dw_wgrad_chunks(N, H, W, c);  // image row (segments) per partial
            launch_dw_wgrad_auto(A.bx[l], A.ddw, N, H, W, c, A.part, st);
            launch_reduce_chunks(A.part, nch, (size_t)50 * c, (size_t)49 * c, 49, 50, 0, G(b.dww), st);
            launch_reduce_chunks(A.part, nch, (size_t)50 * c, c, 1, 50, 49, G(b.dwb), st);
        }
        // residual
        launch_add(A.dxdw, c, 0, dh, c, 0, M, c, A.dxdw, c, 0, st);
    }

    void backward(int N, int H, int W, const float* x, hipStream_t st) {
        // flipped weights for the data gradients
        auto flip = [&](const ConvL& c) {
            launch_weight_flip(PB(c.w), c.co, c.k * c.k, c.ci, c.co_pad, wt + c.wt_off, st);
        };
        for (int l = 0; l < 4; l++) {
            flip(enc[l].pw1);
            flip(enc[l].pw2);
            if (l > 0) flip(down[l]);
        }
        for (int h = 0; h < kHeads; h++) {
            for (int l = 1; l < 4; l++) {
                flip(up[h][l]);
                flip(fuse[h][l]);
            }
            flip(out[h]);
        }
        for (int l = 0; l < 4; l++)
            launch_fill_u32((uint32_t*)A.dsk[l], 0u, (uint64_t)N * (H >> l) * (W >> l) * C[l] / 2, st);
        const float* og[kHeads] = {A.ogd, A.ogn, A.ogl};
        for (int h = 0; h < kHeads; h++) {
            launch_fill_u32((uint32_t*)A.dzo, 0u, (uint64_t)N * H * W * kPadCo / 2, st);
            // the depth output is head / max(H, W) + coarse depth
            const float gs = h == 0 ? 1.f / (float)std::max(H, W) : 1.f;
            launch_head_grad(og[h], N, H, W, kHeadCo[h], gs, A.dzo, kPadCo, st);
            conv_wgrad(out[h], A.u[h][0], C[0], 0, A.dzo, kPadCo, N, H, W, st);
            conv_dgrad(out[h], A.dzo, kPadCo, N, H, W, A.du, C[0], 0, st);
            for (int l = 1; l <= 3; l++) {
                const int c = C[l - 1], Hc = H >> (l - 1), Wc = W >> (l - 1), Mc = N * Hc * Wc;
                launch_gelu_bwd(A.zf[h][l - 1], A.du, (size_t)Mc * c, A.dzf, st);
                conv_wgrad(fuse[h][l], A.cat[h][l - 1], 2 * c, 0, A.dzf, c, N, Hc, Wc, st);
                conv_dgrad(fuse[h][l], A.dzf, c, N, Hc, Wc, A.dcat, 2 * c, 0, st);
                launch_add(A.dsk[l - 1], c, 0, A.dcat, 2 * c, c, Mc, c, A.dsk[l - 1], c, 0, st);
                launch_unshuffle(A.dcat, N, Hc / 2, Wc / 2, c, 2 * c, 0, A.dzu, 4 * c, st);
                const uint16_t* uin = l == 3 ? A.sk[3] : A.u[h][l];
                conv_wgrad(up[h][l], uin, C[l], 0, A.dzu, 4 * c, N, Hc / 2, Wc / 2, st);
                conv_dgrad(up[h][l], A.dzu, 4 * c, N, Hc / 2, Wc / 2, A.du, C[l], 0, st);
            }
            const int M3 = N * (H >> 3) * (W >> 3);
            launch_add(A.dsk[3], C[3], 0, A.du, C[3], 0, M3, C[3], A.dsk[3], C[3], 0, st);
        }
        for (int l = 3; l >= 1; l--) {
            const int Hl = H >> l, Wl = W >> l;
            block_bwd(l, A.dsk[l], N, Hl, Wl, st);
            conv_wgrad(down[l], A.pooled[l], C[l - 1], 0, A.dxdw, C[l], N, Hl, Wl, st);
            conv_dgrad(down[l], A.dxdw, C[l], N, Hl, Wl, A.dp, C[l - 1], 0, st);
            launch_pool_bwd(A.dp, A.arg[l], N, 2 * Hl, 2 * Wl, C[l - 1], A.dsk[l - 1], st);
        }
        block_bwd(0, A.dsk[0], N, H, W, st);
        const int M0 = N * H * W;
        launch_gelu_bwd(A.stem_z, A.dxdw, (size_t)M0 * C[0], A.dxdw, st);
        {
            const int nch = (M0 + kRowChunk - 1) / kRowChunk;
            launch_stem_wgrad(x, N, H, W, C[0], A.dxdw, kRowChunk, A.part, st);
            launch_reduce_chunks(A.part, nch, (size_t)10 * C[0], (size_t)9 * C[0], 9, 10, 0,
                                 G(stem.w), st);
            launch_reduce_chunks(A.part, nch, (size_t)10 * C[0], C[0], 1, 10, 9, G(stem.b), st);
        }
    }

    void loss(int N, int H, int W, const float* dgt, const float* ngt, const float* mgt,
              double* host6, hipStream_t st) {
        LossArgs la{};
        la.N = N;
        la.H = 2 * H;
        la.W = 2 * W;
        la.depth = A.out32[0];
        la.nrm = A.out32[1];
        la.logit = A.out32[2];
        la.depth_gt = dgt;
        la.nrm_gt = ngt;
        la.mask_gt = mgt;
        la.gd = A.gd;
        la.gn = A.gn;
        la.gl = A.gl;
        la.w4 = A.w4;
        la.partial = A.lpart;
        la.out_gd = A.ogd;
        la.out_gn = A.ogn;
        la.out_gl = A.ogl;
        const int nb = (int)(((uint64_t)N * 4 * H * W + 255) / 256);
        launch_loss(la, st);
        launch_loss_sum(A.lpart, nb, A.sums, st);
        launch_loss_scale(la, A.sums, st);
        HIPCHK(hipMemcpyAsync(host6, A.sums, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    }

    void infer(int N, int H, int W, const float* coarse, float* depth, float* nrm, float* prob,
               hipStream_t st) {
        plan(N, H, W);
        forward(N, H, W, coarse, false, st);
        const size_t n = (size_t)N * 4 * H * W;
        if (depth) HIPCHK(hipMemcpyAsync(depth, A.out32[0], n * sizeof(float), hipMemcpyDeviceToDevice, st));
        launch_head_post(A.out32[2], A.out32[1], n, prob, nrm, st);
        HIPCHK(hipGetLastError());
    }
};

size_t pe_densifier_s::part_floats(int N, int H, int W) const {
    size_t best = 0;
    auto convp = [&](const ConvL& c, int M) {
        int chunk = 0;
        const int nch = wgrad_chunks(c, M, &chunk);
        best = std::max(best, (size_t)nch * c.co * c.k * c.k * c.ci);
        best = std::max(best, (size_t)((M + kRowChunk - 1) / kRowChunk) * c.co);
    };
    for (int l = 0; l < 4; l++) {
        const int Hl = H >> l, Wl = W >> l, M = N * Hl * Wl, c = C[l];
        convp(enc[l].pw1, M);
        convp(enc[l].pw2, M);
        if (l > 0) convp(down[l], M);
        best = std::max(best, (size_t)((M + kRowChunk - 1) / kRowChunk) * 2 * c);
        best = std::max(best, (size_t)dw_wgrad_chunks(N, Hl, Wl, c) * 50 * c);
    }
    for (int h = 0; h < kHeads; h++) {
        for (int l = 1; l < 4; l++) {
            convp(fuse[h][l], N * (H >> (l - 1)) * (W >> (l - 1)));
            convp(up[h][l], N * (H >> l) * (W >> l));
        }
        convp(out[h], N * H * W);
    }
    best = std::max(best, (size_t)((N * H * W + kRowChunk - 1) / kRowChunk) * 10 * C[0]);
    return best;
}

void pe_densifier_s::plan(int N, int H, int W) {
    if (N == aN && H == aH && W == aW) return;
    // offsets first (null base), then allocate and rebase
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> list;
    auto take = [&](void** ptr, size_t bytes) {
        list.push_back({ptr, off});
        off = round_up(off + bytes, 256);
    };
    Acts a;
    const size_t M0 = (size_t)N * H * W;
    auto M = [&](int l) { return (size_t)N * (H >> l) * (W >> l); };
    take((void**)&a.stem_z, M0 * C[0] * 2);
    for (int l = 0; l < 4; l++) {
        const size_t m = M(l), c = C[l];
        take((void**)&a.bx[l], m * c * 2);
        take((void**)&a.dwo[l], m * c * 2);
        take((void**)&a.lno[l], m * c * 2);
        take((void**)&a.z1[l], m * 4 * c * 2);
        take((void**)&a.a1[l], m * 4 * c * 2);
        take((void**)&a.sk[l], m * c * 2);
        take((void**)&a.lst[l], m * 2 * 4);
        take((void**)&a.dsk[l], m * c * 2);
        if (l > 0) {
            take((void**)&a.pooled[l], m * C[l - 1] * 2);
            take((void**)&a.arg[l], m * C[l - 1]);
        }
    }
    for (int h = 0; h < kHeads; h++) {
        for (int l = 0; l < 3; l++) {
            const size_t m = M(l), c = C[l];
            take((void**)&a.cat[h][l], m * 2 * c * 2);
            take((void**)&a.zf[h][l], m * c * 2);
            take((void**)&a.u[h][l], m * c * 2);
        }
        take((void**)&a.out32[h], 4 * M0 * kHeadCo[h] * 4);
    }
    const size_t big = M0 * C[0];
    take((void**)&a.dzo, M0 * kPadCo * 2);
    take((void**)&a.du, big * 2);
    take((void**)&a.dzf, big * 2);
    take((void**)&a.dcat, 2 * big * 2);
    take((void**)&a.dzu, big * 2);
    take((void**)&a.t4, 4 * big * 2);
    take((void**)&a.dln, big * 2);
    take((void**)&a.ddw, big * 2);
    take((void**)&a.dxdw, big * 2);
    take((void**)&a.dp, big * 2);
    const size_t Mo = 4 * M0;
    take((void**)&a.gd, Mo * 4);
    take((void**)&a.gn, 3 * Mo * 4);
    take((void**)&a.gl, Mo * 4);
    take((void**)&a.w4, 2 * Mo * 4);
    take((void**)&a.lpart, ((Mo + 255) / 256) * 6 * 4);
    take((void**)&a.ogd, Mo * 4);
    take((void**)&a.ogn, 3 * Mo * 4);
    take((void**)&a.ogl, Mo * 4);
    take((void**)&a.sums, 8 * 8);
    take((void**)&a.part, part_floats(N, H, W) * 4);
    if (off > arena_bytes) {
        if (arena) {
            HIPCHK(hipDeviceSynchronize());
            ctx_free(ctx, arena, arena_bytes);
            arena = nullptr;
            arena_bytes = 0;
        }
        arena = ctx_alloc(ctx, off);
        arena_bytes = off;
    }
    for (auto& e : list) *e.first = (char*)arena + e.second;
    A = a;
    aN = N;
    aH = H;
    aW = W;
}

namespace pe {

static pe_densifier_s* as_net(pe_densifier n) { return (pe_densifier_s*)n; }

static void check_shape(int32_t b, int32_t h, int32_t w) {
    if (b < 1 || h < 8 || w < 8 || h % 8 || w % 8) throw Error{PE_EINVAL, "batch >= 1 and coarse h, w >= 8, multiples of 8"};
    if ((uint64_t)b * 4 * h * w > (1ull << 28)) throw Error{PE_EINVAL, "batch too large"};
}

// Splat with the tile-list retry; returns after the keys are final.
static void splat_checked(Batch& b, const std::vector<SlotSpec>& slots, int contrib, int prec) {
    uint32_t c[kNumCounters];
    for (int attempt = 0;; attempt++) {
        b.splat();
        b.read_counters(c);
        if (!b.overflowed(c)) return;
        if (attempt > 3) throw Error{PE_EDEVICE, "tile list overflow persists"};
        b.setup(slots, contrib, prec);
    }
}

// PO of Eq. (14) at the first bounce, with the primary rays taken from a GFB (depth t/D,
// view-frame normals, hit probability >= 0.5) on each slot's screen.
static void gfb_field(Workspace& ws, hipStream_t st, const std::vector<SlotSpec>& slots,
                      int precision, const float* depth, const float* nrm, const float* prob,
                      const uint8_t* use, double* E, double* rcs, pe_stats* acc) {
    Batch b(ws, st);
    b.setup(slots, PE_CONTRIB_LAST, precision);
    b.raygen_gfb(depth, nrm, prob, use, 0.5f);
    b.trace(true);
    b.field(E, rcs);
    uint32_t c[kNumCounters];
    b.read_counters(c);
    if (acc) {
        acc->ray_queries += b.queries(c);
        const double recs = b.records_made(c) * b.max_obs;
        acc->exit_records += recs;
        acc->po_terms += recs * b.max_freq;
    }
}

static void densified_solve(Workspace& ws, hipStream_t st, pe_scene sc, const pe_solve_desc* d,
                            double* E, double* rcs, pe_stats* acc) {
    pe_densifier_s* net = d->geometry == PE_GEOM_DENSIFIED ? as_net(d->densifier) : nullptr;
    const int W = d->screen_w, h = W / 2;
    const double tube_px = d->tube_px > 0 ? d->tube_px : 2.0;
    const int tube_k = d->tube_k;
    const double max_unc = d->max_uncertain > 0 ? d->max_uncertain : 0.25;
    const double coarse_pitch = 2.0 * sc->R / h;
    const int n_obs = d->obs_dir ? d->n_obs : 1;
    const uint64_t per_inc = (uint64_t)n_obs * d->n_freq * 4;
    for (int i0 = 0; i0 < d->n_inc; i0 += kNetBatch) {
        const int cnt = std::min(kNetBatch, d->n_inc - i0);
        std::vector<SlotSpec> cs = make_slots(sc, d, i0, cnt);
        for (auto& s : cs) {
            s.W = s.H = h;
            s.mode = PE_SPLAT_TUBE;
            s.tube_r = tube_px * coarse_pitch;
            s.max_b = 1;
        }
        Batch cb(ws, st);
        cb.topk = tube_k;
        cb.setup(cs, PE_CONTRIB_LAST, d->precision);
        splat_checked(cb, cs, PE_CONTRIB_LAST, d->precision);
        double* Ei = E + (uint64_t)i0 * per_inc * 2;
        double* Ri = rcs ? rcs + (uint64_t)i0 * per_inc : nullptr;
        uint8_t* use = ws.get<uint8_t>(B_GFB_USE, round_up((uint64_t)cnt, 4));
        if (!net) {
            // no network: PO straight from the coarse buffer, normals from its depth gradients
            float* dep = ws.get<float>(B_GFB_DEPTH, (uint64_t)cnt * h * h);
            float* nr = ws.get<float>(B_GFB_NRM, (uint64_t)cnt * h * h * 3);
            float* mk = ws.get<float>(B_GFB_PROB, (uint64_t)cnt * h * h);
            launch_target_encode(cb.dd, cnt, h * h, cb.keys, dep, nr, mk, st);
            launch_depth_normals(dep, mk, h, h, cnt, (float)h, nr, st);
            launch_fill_u32((uint32_t*)use, 0x01010101u, (cnt + 3) / 4, st);
            std::vector<SlotSpec> fs = make_slots(sc, d, i0, cnt);
            for (auto& s : fs) s.W = s.H = h;
            gfb_field(ws, st, fs, d->precision, dep, nr, mk, use, Ei, Ri, acc);
            continue;
        }
        float* coarse = ws.get<float>(B_GFB_COARSE, (uint64_t)cnt * h * h);
        launch_coarse_encode(cb.dd, cnt, h * h, cb.keys, coarse, st);
        float* dep = ws.get<float>(B_GFB_DEPTH, (uint64_t)cnt * W * W);
        float* nr = ws.get<float>(B_GFB_NRM, (uint64_t)cnt * W * W * 3);
        float* pr = ws.get<float>(B_GFB_PROB, (uint64_t)cnt * W * W);
        {
            std::lock_guard<std::mutex> lk(net->mu);
            net->infer(cnt, h, h, coarse, dep, nr, pr, st);
            // the fine batch below reuses the workspace: finish the network first
            HIPCHK(hipStreamSynchronize(st));
        }
        std::vector<SlotSpec> fs = make_slots(sc, d, i0, cnt);
        Batch fb(ws, st);
        fb.setup(fs, PE_CONTRIB_LAST, d->precision);
        uint32_t* counts = ws.get<uint32_t>(B_GFB_CNT, 2 * cnt);
        launch_fill_u32(counts, 0u, 2 * cnt, st);
        launch_gfb_uncertain(fb.dd, cnt, W * W, pr, 0.1f, 0.9f, counts, st);
        std::vector<uint32_t> hc(2 * cnt);
        HIPCHK(hipMemcpyAsync(hc.data(), counts, sizeof(uint32_t) * 2 * cnt, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<uint8_t> hu(cnt);
        std::vector<int> fallback;
        for (int s = 0; s < cnt; s++) {
            const double frac = hc[2 * s] ? (double)hc[2 * s + 1] / hc[2 * s] : 1.0;
            hu[s] = frac <= max_unc ? 1 : 0;
            if (!hu[s]) fallback.push_back(s);
        }
        HIPCHK(hipMemcpyAsync(use, hu.data(), cnt, hipMemcpyHostToDevice, st));
        gfb_field(ws, st, fs, d->precision, dep, nr, pr, use, Ei, Ri, acc);
        HIPCHK(hipStreamSynchronize(st));
        if (!fallback.empty()) {
            // uncertain network output: plain first-hit buffer for those incidences
            std::vector<SlotSpec> ps;
            for (int s : fallback) ps.push_back(fs[s]);
            std::vector<double> Et(per_inc * 2 * ps.size()), Rt(per_inc * ps.size());
            run_field_batch(ws, st, ps, PE_CONTRIB_LAST, d->precision, Et.data(), Rt.data(), acc);
            HIPCHK(hipStreamSynchronize(st));
            for (size_t j = 0; j < fallback.size(); j++) {
                std::memcpy(Ei + fallback[j] * per_inc * 2, Et.data() + j * per_inc * 2,
                            sizeof(double) * per_inc * 2);
                if (Ri) std::memcpy(Ri + fallback[j] * per_inc, Rt.data() + j * per_inc,
                                    sizeof(double) * per_inc);
            }
            if (acc) acc->densifier_fallbacks += (double)fallback.size();
        }
    }
}

static struct DensifierRegistrar {
    DensifierRegistrar() { g_densified_solve = densified_solve; }
} g_registrar;

static uint64_t fnv1a(const void* data, size_t n, uint64_t h) {
    const uint8_t* p = (const uint8_t*)data;
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

struct CkptHeader {
    char magic[8];
    int32_t version, base, step, pad;
    uint64_t n_params, checksum;
};

}  // namespace pe

extern "C" {

pe_status pe_densifier_create(pe_ctx ctx, int32_t base_ch, uint64_t seed, pe_densifier* out) {
    API_BEGIN
    if (!ctx || !out) return set_error(PE_EINVAL, "null argument");
    if (base_ch < 32 || base_ch > 128 || base_ch % 32) return set_error(PE_EINVAL, "base_ch must be 32, 64, 96 or 128");
    HIPCHK(hipSetDevice(ctx->device));
    auto net = std::make_unique<pe_densifier_s>();
    net->ctx = ctx;
    net->base = base_ch;
    net->build_registry();
    const uint64_t n = net->n_params;
    net->p = (float*)net->alloc(n * 4);
    net->g = (float*)net->alloc(n * 4);
    net->m = (float*)net->alloc(n * 4);
    net->v = (float*)net->alloc(n * 4);
    net->pb = (uint16_t*)net->alloc(n * 2);
    net->wt = (uint16_t*)net->alloc(net->wt_n * 2);
    for (int l = 0; l < 4; l++) net->dwt[l] = (float*)net->alloc((size_t)49 * net->C[l] * 4);
    std::vector<float> h = net->init_values(seed);
    HIPCHK(hipMemcpy(net->p, h.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(net->g, 0, n * 4));
    HIPCHK(hipMemset(net->m, 0, n * 4));
    HIPCHK(hipMemset(net->v, 0, n * 4));
    launch_f32_to_bf16(net->p, n, net->pb, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    *out = net.release();
    return PE_OK;
    API_END
}

pe_status pe_densifier_destroy(pe_densifier net) {
    API_BEGIN
    if (!net) return PE_OK;
    (void)hipSetDevice(net->ctx->device);
    (void)hipDeviceSynchronize();
    delete as_net(net);
    return PE_OK;
    API_END
}

pe_status pe_densifier_num_params(pe_densifier net, uint64_t* n) {
    if (!net || !n) return set_error(PE_EINVAL, "null argument");
    *n = net->n_params;
    return PE_OK;
}

pe_status pe_densifier_tensors(pe_densifier net, int32_t cap, const char** names,
                               uint64_t* offsets, int32_t* shapes, int32_t* n) {
    if (!net || !n) return set_error(PE_EINVAL, "null argument");
    *n = (int32_t)net->T.size();
    for (int32_t i = 0; i < cap && i < *n; i++) {
        const Tensor& t = net->T[i];
        if (names) names[i] = t.name.c_str();
        if (offsets) offsets[i] = t.off;
        if (shapes)
            for (int a = 0; a < 4; a++) shapes[4 * i + a] = t.shape[a];
    }
    return PE_OK;
}

pe_status pe_densifier_get(pe_densifier net, int32_t which, float* host, uint64_t n) {
    API_BEGIN
    if (!net || !host) return set_error(PE_EINVAL, "null argument");
    if (n != net->n_params) return set_error(PE_EINVAL, "n must equal the parameter count");
    const float* src = which == 0 ? net->p : which == 1 ? net->g : which == 2 ? net->m : which == 3 ? net->v : nullptr;
    if (!src) return set_error(PE_EINVAL, "which must be 0 (params), 1 (grads), 2 (m) or 3 (v)");
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host, src, n * 4, hipMemcpyDeviceToHost));
    return PE_OK;
    API_END
}

pe_status pe_densifier_set(pe_densifier net, const float* host, uint64_t n) {
    API_BEGIN
    if (!net || !host) return set_error(PE_EINVAL, "null argument");
    if (n != net->n_params) return set_error(PE_EINVAL, "n must equal the parameter count");
    for (uint64_t i = 0; i < n; i++)
        if (!std::isfinite(host[i])) return set_error(PE_EINVAL, "non-finite parameter");
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(net->p, host, n * 4, hipMemcpyHostToDevice));
    launch_f32_to_bf16(net->p, n, net->pb, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    return PE_OK;
    API_END
}

pe_status pe_densifier_save(pe_densifier net, const char* path) {
    API_BEGIN
    if (!net || !path) return set_error(PE_EINVAL, "null argument");
    const uint64_t n = net->n_params;
    std::vector<float> buf(3 * n);
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(buf.data(), net->p, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(buf.data() + n, net->m, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(buf.data() + 2 * n, net->v, n * 4, hipMemcpyDeviceToHost));
    CkptHeader hd{};
    std::memcpy(hd.magic, "PEDNSF01", 8);
    hd.version = 1;
    hd.base = net->base;
    hd.step = net->step;
    hd.n_params = n;
    hd.checksum = fnv1a(buf.data(), buf.size() * 4, 0xCBF29CE484222325ull);
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(PE_EINVAL, std::string("cannot open ") + path);
    const bool ok = std::fwrite(&hd, sizeof hd, 1, f) == 1 &&
                    std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    if (std::fclose(f) != 0 || !ok) return set_error(PE_EINVAL, std::string("write failed: ") + path);
    return PE_OK;
    API_END
}

pe_status pe_densifier_load(pe_densifier net, const char* path) {
    API_BEGIN
    if (!net || !path) return set_error(PE_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(PE_EINVAL, std::string("cannot open ") + path);
    CkptHeader hd{};
    const uint64_t n = net->n_params;
    std::vector<float> buf(3 * n);
    bool ok = std::fread(&hd, sizeof hd, 1, f) == 1;
    ok = ok && std::memcmp(hd.magic, "PEDNSF01", 8) == 0 && hd.version == 1 &&
         hd.base == net->base && hd.n_params == n;
    ok = ok && std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return set_error(PE_EINVAL, "checkpoint does not match this network");
    if (fnv1a(buf.data(), buf.size() * 4, 0xCBF29CE484222325ull) != hd.checksum)
        return set_error(PE_EINVAL, "checkpoint checksum mismatch");
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(net->p, buf.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(net->m, buf.data() + n, n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(net->v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
    launch_f32_to_bf16(net->p, n, net->pb, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    net->step = hd.step;
    return PE_OK;
    API_END
}

pe_status pe_densifier_train_step(pe_densifier net, int32_t b, int32_t h, int32_t w,
                                  const float* coarse, const float* depth_gt, const float* nrm_gt,
                                  const float* mask_gt, float lr, float weight_decay,
                                  double* loss_out, void* hip_stream) {
    API_BEGIN
    if (!net || !coarse || !depth_gt || !nrm_gt || !mask_gt) return set_error(PE_EINVAL, "null argument");
    check_shape(b, h, w);
    if (!(lr >= 0) || !std::isfinite(lr) || !(weight_decay >= 0) || !std::isfinite(weight_decay))
        return set_error(PE_EINVAL, "lr and weight_decay must be finite and >= 0");
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    net->plan(b, h, w);
    net->forward(b, h, w, coarse, true, st);
    double s[6];
    net->loss(b, h, w, depth_gt, nrm_gt, mask_gt, s, st);
    net->backward(b, h, w, coarse, st);
    launch_adamw(net->p, net->g, net->m, net->v, net->pb, net->n_params, lr, weight_decay,
                 net->step + 1, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    net->step++;
    if (loss_out) {
        const double nv = std::max(s[4], 1.0), nv4 = std::max(s[5], 1.0);
        const double total = (double)b * 4 * h * w;
        const double L1 = s[0] / nv, L2 = s[1] / nv, L3 = s[2] / total, L4 = s[3] / nv4;
        loss_out[0] = L1 + 0.5 * L2 + L3 + 0.5 * L4;
        loss_out[1] = L1;
        loss_out[2] = L2;
        loss_out[3] = L3;
        loss_out[4] = L4;
    }
    return PE_OK;
    API_END
}

pe_status pe_densifier_infer(pe_densifier net, int32_t b, int32_t h, int32_t w,
                             const float* coarse, float* depth, float* nrm, float* prob,
                             void* hip_stream) {
    API_BEGIN
    if (!net || !coarse) return set_error(PE_EINVAL, "null argument");
    check_shape(b, h, w);
    HIPCHK(hipSetDevice(net->ctx->device));
    std::lock_guard<std::mutex> lk(net->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    net->infer(b, h, w, coarse, depth, nrm, prob, st);
    HIPCHK(hipStreamSynchronize(st));
    return PE_OK;
    API_END
}

pe_status pe_densifier_make_pair(pe_ctx ctx, pe_scene scene, int32_t n_dir, const double* dirs,
                                 int32_t h, int32_t w, double tube_px, int32_t tube_k,
                                 float* coarse, float* depth_gt, float* nrm_gt, float* mask_gt,
                                 void* hip_stream) {
    API_BEGIN
    if (!ctx || !scene || !dirs) return set_error(PE_EINVAL, "null argument");
    if (scene->ctx != ctx) return set_error(PE_EINVAL, "scene belongs to another context");
    if (n_dir < 1 || n_dir > 1024) return set_error(PE_EINVAL, "n_dir must be 1..1024");
    if (h < 1 || w < 1 || (uint64_t)4 * h * w > (1u << kPixBits)) return set_error(PE_EINVAL, "bad size");
    if ((uint64_t)4 * h * w * n_dir >= 0xFFFFFFF0ull) return set_error(PE_EINVAL, "batch too large");
    if (!(tube_px > 0) || !std::isfinite(tube_px)) return set_error(PE_EINVAL, "tube_px must be > 0");
    if (tube_k < 0 || tube_k > 1024) return set_error(PE_EINVAL, "tube_k must be 0..1024");
    for (int i = 0; i < n_dir; i++) {
        const double* k = dirs + 3 * i;
        const double l = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        if (!std::isfinite(l) || !(l > 0)) return set_error(PE_EINVAL, "non-finite or zero direction");
    }
    HIPCHK(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<SlotSpec> s(n_dir);
    for (int i = 0; i < n_dir; i++) {
        s[i].sc = scene;
        for (int a = 0; a < 3; a++) s[i].k[a] = dirs[3 * i + a];
    }
    if (coarse) {
        for (auto& x : s) {
            x.W = w;
            x.H = h;
            x.mode = PE_SPLAT_TUBE;
            x.tube_r = tube_px * 2.0 * scene->R / std::max(w, h);
        }
        Batch b(*ctx->ws, st);
        b.topk = tube_k;
        b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
        splat_checked(b, s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
        launch_coarse_encode(b.dd, n_dir, h * w, b.keys, coarse, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    }
    if (depth_gt || nrm_gt || mask_gt) {
        if (!depth_gt || !nrm_gt || !mask_gt) return set_error(PE_EINVAL, "give all three targets");
        for (auto& x : s) {
            x.W = 2 * w;
            x.H = 2 * h;
            x.mode = PE_SPLAT_DISK;
        }
        Batch b(*ctx->ws, st);
        b.setup(s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
        splat_checked(b, s, PE_CONTRIB_LAST, PE_PREC_FP64PHASE);
        launch_target_encode(b.dd, n_dir, 4 * h * w, b.keys, depth_gt, nrm_gt, mask_gt, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    }
    return PE_OK;
    API_END
}

}  // extern "C"
