// Kernels of the learned densifier (Sec. III-A): a U-Net with ConvNeXt encoder blocks,
// max-pool down, sub-pixel convolution up, three decoder heads, trained with Eq. (17)-(21).
//
// Layout: activations NHWC in bf16 (uint16 storage), convolution weights OHWI in bf16 with
// fp32 master copies; every GEMM-shaped convolution runs on MFMA (v_mfma_f32_16x16x32_bf16,
// fp32 accumulation): forward and data-gradient as implicit GEMM over (pixels x Cout x taps*Cin)
// with the tiles copied from NHWC/OHWI straight into LDS (3 x 3 layers over two-dimensional
// pixel tiles whose input halo serves all nine taps), weight-gradient as GEMM over
// (Cout x Cin x pixels) with tiles transposed through LDS.  Everything that reduces
// over pixels writes per-chunk partials summed in a fixed order, so a training step is
// bit-reproducible.  Depthwise 7x7, LayerNorm, GELU, pooling, losses and AdamW are VALU kernels.
#include <float.h>

#include <algorithm>

#include "pe_device.h"
#include "pe_nn.h"

namespace pe {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline uint16_t f2bf(float f) {  // round to nearest even
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

union Frag {
    uint4 u;
    v8bf v;
};

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, formula 7.1.26: for x >= 0,
// erf x = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), t = 1 / (1 + p x), with
// absolute error at most 1.5e-7 (three orders below a bf16 step); odd in x.  Branch-free, unlike
// the library erff, whose two argument ranges diverge within a wavefront.
__device__ inline float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.f));
    const float poly =
        t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f +
                                                                          t * 1.061405429f))));
    return copysignf(1.f - poly * __expf(-ax * ax), x);
}

// GELU with the exact (erf) Gaussian CDF: 0.5 v (1 + erf(v / sqrt 2)).
__device__ inline float gelu_f(float v) { return 0.5f * v * (1.f + erf_as(v * 0.70710678118654752f)); }

// Epilogue of the convolution kernels: bias, residual, GELU, optional pre-activation copy and
// pixel shuffle, from the accumulator fragments of a BM x BN tile.  For bf16 outputs the fp32
// tile plus bias is staged in LDS (smem, at least BM x (BN + 4) floats, free when this is
// called) and each thread then takes rows of 8 channels: residual (one 16-byte load), the
// pre-activation copy, GELU and the output as 16-byte stores.  The arithmetic is per element:
// acc + bias, + residual, then GELU.
// rowm maps a tile row to its output pixel index m (m >= M: past the end, not stored).
template <int BN, int BM, int WGM, class RowM>
__device__ inline void conv_epilogue(const ConvArgs& a,
                                     const v4f (&acc)[BM / WGM / 16][BN / (4 / WGM) / 16],
                                     void* smem, RowM rowm, int n0) {
    constexpr int WGN = 4 / WGM;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int TLD = BN + 4;  // floats per staged row (rows 16-byte aligned)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int HW = a.H * a.W, M = a.N * HW;
    const int r = lane & 15;
    float bj[TN];  // bias of this lane's column in each MFMA tile column
#pragma unroll
    for (int j = 0; j < TN; j++) {
        const int co = n0 + wn * WTN + j * 16 + r;
        bj[j] = (co < a.Cout_store && a.bias) ? a.bias[co] : 0.f;
    }
    // D fragment: lane holds column (channel) r of rows (pixels) 4 * (lane / 16) + q
    if (a.y32) {
        // fp32 outputs (the heads' last layers, few channels): straight from the fragments
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++) {
                const int co = n0 + wn * WTN + j * 16 + r;
                const bool cok = co < a.Cout_store;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int m = rowm(wm * WTM + i * 16 + (lane >> 4) * 4 + q);
                    if (cok && m < M) {
                        float v = acc[i][j][q] + bj[j];
                        if (a.res) v += bf2f(a.res[(size_t)m * a.ldres + co]);
                        if (a.act == 1) v = gelu_f(v);
                        const int n = m / HW, yy = (m % HW) / a.W, xx = m % a.W;
                        size_t o;
                        if (a.shuffle) {
                            const int oc = co >> 2, sy = (co >> 1) & 1, sx = co & 1;
                            o = ((size_t)(n * 2 * a.H + 2 * yy + sy) * (2 * a.W) + 2 * xx + sx) *
                                    a.ldy + a.yoff + oc;
                        } else {
                            o = ((size_t)(n * a.H + yy) * a.W + xx) * a.ldy + a.yoff + co;
                        }
                        a.y32[o] = v;
                    }
                }
            }
        return;
    }
    float* T = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) {
            const int col = wn * WTN + j * 16 + r;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = wm * WTM + i * 16 + (lane >> 4) * 4 + q;
                T[row * TLD + col] = acc[i][j][q] + bj[j];
            }
        }
    __syncthreads();
    if (!a.shuffle) {
        constexpr int C8 = BN / 8;
        for (int c = tid; c < BM * C8; c += 256) {
            const int row = c / C8, c8 = c - row * C8, m = rowm(row), co = n0 + c8 * 8;
            if (m >= M || co >= a.Cout_store) continue;
            const int ne = min(8, a.Cout_store - co);
            float v[8];
            const float4 v0 = *reinterpret_cast<const float4*>(&T[row * TLD + c8 * 8]);
            const float4 v1 = *reinterpret_cast<const float4*>(&T[row * TLD + c8 * 8 + 4]);
            v[0] = v0.x, v[1] = v0.y, v[2] = v0.z, v[3] = v0.w;
            v[4] = v1.x, v[5] = v1.y, v[6] = v1.z, v[7] = v1.w;
            if (a.res) {
                const uint16_t* rp = a.res + (size_t)m * a.ldres + co;
                if (ne == 8 && ((uintptr_t)rp & 15) == 0) {
                    const uint4 u = *reinterpret_cast<const uint4*>(rp);
                    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int e = 0; e < 8; e++) v[e] += bf2f((uint16_t)(w[e >> 1] >> (16 * (e & 1))));
                } else {
#pragma unroll
                    for (int e = 0; e < 8; e++)
                        if (e < ne) v[e] += bf2f(rp[e]);
                }
            }
            const size_t o = (size_t)m * a.ldy + a.yoff + co;
            uint16_t h[8];
            if (a.z) {
#pragma unroll
                for (int e = 0; e < 8; e++) h[e] = f2bf(v[e]);
                uint16_t* zp = a.z + o;
                if (ne == 8 && ((uintptr_t)zp & 15) == 0) {
                    *reinterpret_cast<uint4*>(zp) =
                        make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                                   h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
                } else {
#pragma unroll
                    for (int e = 0; e < 8; e++)
                        if (e < ne) zp[e] = h[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; e++) h[e] = f2bf(a.act == 1 ? gelu_f(v[e]) : v[e]);
            uint16_t* yp = a.y + o;
            if (ne == 8 && ((uintptr_t)yp & 15) == 0) {
                *reinterpret_cast<uint4*>(yp) =
                    make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                               h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++)
                    if (e < ne) yp[e] = h[e];
            }
        }
    } else {
        // column co = 4 oc + 2 sy + sx goes to pixel (2y + sy, 2x + sx), channel oc
        constexpr int O8 = BN / 32;  // groups of 8 output channels per sub-pixel
        const int oc_end = a.Cout_store >> 2;
        for (int c = tid; c < BM * 4 * O8; c += 256) {
            const int row = c / (4 * O8), rem = c - row * (4 * O8), sub = rem / O8,
                      c8 = rem - sub * O8, m = rowm(row), oc0 = (n0 >> 2) + c8 * 8;
            if (m >= M || oc0 >= oc_end) continue;
            const int ne = min(8, oc_end - oc0);
            const int n = m / HW, yy = (m % HW) / a.W, xx = m % a.W;
            const int sy = sub >> 1, sx = sub & 1;
            const size_t o = ((size_t)(n * 2 * a.H + 2 * yy + sy) * (2 * a.W) + 2 * xx + sx) *
                                 a.ldy + a.yoff + oc0;
            uint16_t h[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int col = 4 * (c8 * 8 + e) + sub;
                float v = T[row * TLD + col];
                if (a.res && e < ne) v += bf2f(a.res[(size_t)m * a.ldres + n0 + col]);
                if (a.z && e < ne) a.z[o + e] = f2bf(v);
                h[e] = f2bf(a.act == 1 ? gelu_f(v) : v);
            }
            uint16_t* yp = a.y + o;
            if (ne == 8 && ((uintptr_t)yp & 15) == 0) {
                *reinterpret_cast<uint4*>(yp) =
                    make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                               h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++)
                    if (e < ne) yp[e] = h[e];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Convolution (stride 1, zero padding (K-1)/2) as implicit GEMM on MFMA
// ------------------------------------------------------------------------------------------
// Block: 256 threads = WGM x (4 / WGM) wavefronts over a tile of BM pixels x BN output
// channels.  Each K step covers 32 input channels of one tap: the A tile (BM pixels x 32
// channels of the shifted input) and the B tile (BN channels x 32) are copied from global memory
// straight into LDS (global_load_lds_dwordx4: each lane's 16 bytes land at the instruction's LDS
// base + 16 x lane) through NS stages, so that the copies of a K step are issued NS - 1 steps
// before its MFMAs and cost no registers.  A wavefront computes BM/WGM x BN/(4/WGM) outputs as
// tiles of v_mfma_f32_16x16x32_bf16.  A stage holds BM + BN rows of 32 bf16 (64 bytes, no
// padding); a row's four 16-byte chunks are stored at position chunk ^ ((row / 2) % 4), which
// puts the 8 rows of each phase of a fragment read on distinct banks.  Halo pixels, pixels past
// the end and weights past Cout are copied from a zero line.  Every wavefront issues the same
// number of copies per stage (padded with copies of the zero line into a spare slot) so that one
// vmcnt bound finds a stage complete in each of them.  Small layers take a smaller BM so that
// the launch still has several workgroups per CU; narrow layers stack the wavefronts along the
// pixels (WGM = 4) so that each still holds several MFMA tiles per K step.  Requirements
// (checked by the host): Cin % 32 == 0.
__device__ __attribute__((aligned(16))) uint4 g_conv_zero[4];

// One 16-byte-per-lane copy from global memory into LDS at byte address lds (wave-uniform).
// Written as inline assembly so that the compiler's own wait insertion, which treats such a
// copy as a pending write to every LDS address and would wait for all copies in flight before
// each LDS read, leaves the stage pipeline alone; the stages are waited for explicitly.  The
// copy has no register results.
__device__ inline void copy_to_lds16(const void* src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src),
                 "s"(lds)
                 : "memory", "m0");
}

template <int N>
__device__ inline void wait_stage_then_barrier() {
    // vmcnt(N) and lgkmcnt(0) (this wavefront's LDS accesses done), then the workgroup barrier;
    // the memory clobber keeps the compiler from moving memory accesses across it
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

template <int BN, int BM, int WGM, int NS>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a) {
    constexpr int WGN = 4 / WGM;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    static_assert(TM >= 1 && TN >= 1, "wavefront tile of at least one MFMA tile");
    constexpr int AI = BM / 16, BI = BN / 16;   // 1 KB copies per stage (16 rows each)
    constexpr int NI = (AI + BI + 3) / 4;       // copies per wavefront per stage
    constexpr int SU = (BM + BN) * 4;           // stage size in 16-byte units
    static_assert(BM * (BN + 4) * 4 <= NS * SU * 16, "fp32 output tile fits the stage LDS");
    __shared__ __attribute__((aligned(16))) uint4 lds[NS * SU + 64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WGM, wn = wave / WGM;
    const int HW = a.H * a.W, M = a.N * HW;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int pad = (a.K - 1) / 2, taps = a.K * a.K, kpt = a.Cin / 32, steps = taps * kpt;
    // this lane's slot in every copy: row q * 16 + lane / 4, position lane % 4, which holds
    // chunk (lane % 4) ^ ((row / 2) % 4)
    const int chunk = (lane & 3) ^ ((lane >> 3) & 3);
    const uint16_t* zero = reinterpret_cast<const uint16_t*>(g_conv_zero);
    // per copy i of this wavefront: kind (0 A, 1 B, 2 spare), LDS unit offset in a stage, and
    // the lane's source: pixel (n, y, x) or output channel
    int kind[NI], uoff[NI], py[NI], px[NI];
    bool val[NI];
    size_t base[NI];
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int q = wave + 4 * i;
        py[i] = px[i] = 0;
        base[i] = 0;
        val[i] = false;
        if (q < AI) {
            kind[i] = 0;
            uoff[i] = q * 64;
            const int m = m0 + q * 16 + (lane >> 2);
            if (m < M) {
                const int n = m / HW, y = (m % HW) / a.W, x = m % a.W;
                val[i] = true;
                py[i] = y;
                px[i] = x;
                base[i] = ((size_t)(n * a.H + y) * a.W + x) * a.ldx + a.xoff + chunk * 8;
            }
        } else if (q < AI + BI) {
            kind[i] = 1;
            uoff[i] = (q - AI) * 64 + BM * 4;
            const int co = n0 + (q - AI) * 16 + (lane >> 2);
            val[i] = co < a.Cout;
            if (val[i]) base[i] = (size_t)co * taps * a.Cin + chunk * 8;
        } else {
            kind[i] = 2;  // the spare slot after the stages
            uoff[i] = NS * SU;
        }
    }
    // next stage to copy: tap lt (offset ldy, ldx from the centre), channel lc
    int lt = 0, lc = 0, ldy = -pad, ldx = -pad;
    auto issue = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NI; i++) {
            const uint16_t* src = zero;
            if (kind[i] == 0) {
                const int y = py[i] + ldy, x = px[i] + ldx;
                if (val[i] && y >= 0 && y < a.H && x >= 0 && x < a.W)
                    src = a.x + base[i] + (ptrdiff_t)(ldy * a.W + ldx) * a.ldx + lc;
            } else if (kind[i] == 1) {
                if (val[i]) src = a.w + base[i] + (size_t)lt * a.Cin + lc;
            }
            const uint4* dst = kind[i] == 2 ? lds + NS * SU : lds + buf * SU + uoff[i];
            copy_to_lds16(src, __builtin_amdgcn_readfirstlane(
                                   (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint4*)dst));
        }
        lc += 32;
        if (lc == a.Cin) {
            lc = 0;
            lt++;
            if (++ldx > pad) {
                ldx = -pad;
                ldy++;
            }
        }
    };
    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NS - 1; s++)
        if (s < steps) issue(s);
    // fragment reads: row (local) R = tile base + lane % 16 holds chunk c at c ^ ((R / 2) % 4)
    const int r = lane & 15, pos = (lane >> 4) ^ ((r >> 1) & 3);
    for (int step = 0; step < steps; step++) {
        const int buf = step % NS;
        if (steps - 1 - step >= NS - 2) wait_stage_then_barrier<NI * (NS - 2)>();
        else wait_stage_then_barrier<0>();
        if (step + NS - 1 < steps) issue((step + NS - 1) % NS);
        const uint4* S = lds + buf * SU;
        Frag fa[TM], fb[TN];
#pragma unroll
        for (int i = 0; i < TM; i++) fa[i].u = S[(wm * WTM + i * 16 + r) * 4 + pos];
#pragma unroll
        for (int j = 0; j < TN; j++) fb[j].u = S[BM * 4 + (wn * WTN + j * 16 + r) * 4 + pos];
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v, acc[i][j], 0,
                                                                   0, 0);
    }
    // every copy has landed (the last step waited for all); all fragment reads are done
    // before the epilogue reuses the stages
    wait_stage_then_barrier<0>();
    conv_epilogue<BN, BM, WGM>(a, acc, lds, [m0](int row) { return m0 + row; }, n0);
}

template <int BN, int BM, int WGM, int NS>
static bool launch_conv_fwd_t(const ConvArgs& a, int M, unsigned gy, bool force,
                                  hipStream_t st) {
    const unsigned gx = (unsigned)((M + BM - 1) / BM);
    if (!force && (uint64_t)gx * gy < 1024) return false;
    hipLaunchKernelGGL((k_conv_fwd<BN, BM, WGM, NS>), dim3(gx, gy), dim3(256), 0, st, a);
    return true;
}

// 3 x 3 convolutions over two-dimensional pixel tiles (TH rows x 16 columns of one image): the
// K loop runs over 32-channel slices of the input and, within a slice, over the nine taps, TPS
// of them per step.  The slice's input halo ((TH + 2) x 18 pixels x 32 channels) is copied into
// LDS once and serves all nine taps, so the input is read about (TH + 2) x 18 / (16 TH) times
// instead of nine times; the weights of one step (TPS taps x BN channels x 32) go through NS
// copy stages as in k_conv_fwd.  Halo buffers are double-buffered over slices: the next slice's
// halo is copied at the first step of the current one (after that step's weights, so a step's
// wait covers it when it was issued within the last NS - 1 steps; NS - 1 < steps per slice).
// Requirements (checked by the host): K = 3, W % 16 == 0, H % TH == 0, Cin % 32 == 0.
template <int BN, int TH, int WGM, int NS, int TPS>
__global__ __launch_bounds__(256) void k_conv3_halo(ConvArgs a) {
    constexpr int TW = 16, BM = TH * TW;
    constexpr int WGN = 4 / WGM;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    static_assert(TM >= 1 && TN >= 1 && WTM % 16 == 0, "wavefront tile of whole MFMA tiles");
    constexpr int HWD = TW + 2, HT = (TH + 2) * HWD;  // halo pixels
    constexpr int HJ = (HT + 15) / 16;                 // halo copies (16 pixels each)
    constexpr int HU = HJ * 64;                        // halo buffer, 16-byte units
    constexpr int SPS = 9 / TPS;                       // steps per slice
    static_assert(SPS * TPS == 9 && NS >= 2 && NS - 1 < SPS, "taps per step divide the nine");
    constexpr int RB = BN / 16;                        // 16-row blocks of one tap's weights
    constexpr int BI = RB * TPS;                       // weight copies per step
    constexpr int NH = (HJ + 3) / 4, NB = (BI + 3) / 4;  // per wavefront
    constexpr int SU = BN * 4 * TPS;
    constexpr int UNITS = 2 * HU + NS * SU + 64;
    static_assert(BM * (BN + 4) * 4 <= UNITS * 16, "fp32 output tile fits the LDS");
    __shared__ __attribute__((aligned(16))) uint4 lds[UNITS];
    uint4* const hbuf = lds;
    uint4* const bst = lds + 2 * HU;
    uint4* const spare = bst + NS * SU;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WGM, wn = wave / WGM;
    const int tiles_x = a.W / TW, tiles_xy = tiles_x * (a.H / TH);
    const int n = blockIdx.x / tiles_xy, rem = blockIdx.x - n * tiles_xy;
    const int y0 = (rem / tiles_x) * TH, x0 = (rem % tiles_x) * TW;
    const int n0 = blockIdx.y * BN;
    const int nsl = a.Cin / 32, steps = SPS * nsl;
    const int chunk = (lane & 3) ^ ((lane >> 3) & 3);
    const uint16_t* zero = reinterpret_cast<const uint16_t*>(g_conv_zero);
    // this lane's source in each copy of this wavefront: element offset of its 8 channels at
    // slice 0 (tap 0 for the weights), or the zero line; halo copies of index >= HJ and weight
    // copies of index >= BI go to the spare slot
    size_t hsrc[NH], bsrc[NB];
    bool hval[NH], bval[NB];
#pragma unroll
    for (int i = 0; i < NH; i++) {
        const int hp = (wave + 4 * i) * 16 + (lane >> 2);
        const int y = y0 - 1 + hp / HWD, x = x0 - 1 + hp % HWD;
        hval[i] = hp < HT && y >= 0 && y < a.H && x >= 0 && x < a.W;
        hsrc[i] = hval[i] ? ((size_t)(n * a.H + y) * a.W + x) * a.ldx + a.xoff + chunk * 8 : 0;
    }
#pragma unroll
    for (int i = 0; i < NB; i++) {
        // copy q: rows (q % RB) * 16 .. + 15 of tap q / RB of the step
        const int q = wave + 4 * i, co = n0 + (q % RB) * 16 + (lane >> 2);
        bval[i] = q < BI && co < a.Cout;
        bsrc[i] = bval[i] ? ((size_t)co * 9 + q / RB) * a.Cin + chunk * 8 : 0;
    }
    auto lds_addr = [](const uint4* p) {
        return __builtin_amdgcn_readfirstlane(
            (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint4*)p);
    };
    auto copy_halo = [&](int sl) {
        uint4* const hb = hbuf + (sl & 1) * HU;
#pragma unroll
        for (int i = 0; i < NH; i++) {
            const int j = wave + 4 * i;
            copy_to_lds16(hval[i] ? a.x + hsrc[i] + sl * 32 : zero,
                          lds_addr(j < HJ ? hb + j * 64 : spare));
        }
    };
    int lt = 0, lsl = 0;  // the next weight step to copy: taps lt .. lt + TPS - 1 of slice lsl
    auto copy_weights = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const int q = wave + 4 * i;
            copy_to_lds16(bval[i] ? a.w + bsrc[i] + (size_t)lt * a.Cin + lsl * 32 : zero,
                          lds_addr(q < BI ? bst + buf * SU + q * 64 : spare));
        }
        lt += TPS;
        if (lt == 9) {
            lt = 0;
            lsl++;
        }
    };
    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    copy_halo(0);
#pragma unroll
    for (int s = 0; s < NS - 1; s++)
        if (s < steps) copy_weights(s);
    const int r = lane & 15, kc = lane >> 4;
    const int bpos = kc ^ ((r >> 1) & 3);
    int hp0[TM];  // halo pixel of this lane's row in MFMA tile i, tap (0, 0)
#pragma unroll
    for (int i = 0; i < TM; i++) {
        const int p = wm * WTM + i * 16 + r;
        hp0[i] = (p / TW) * HWD + p % TW;
    }
    for (int s = 0; s < steps; s++) {
        const int sl = s / SPS, t = s - SPS * sl;
        // copies issued after this step's weights: the next NS - 2 weight steps, plus the next
        // slice's halo when it was issued within the last NS - 1 steps
        if (steps - 1 - s < NS - 2) wait_stage_then_barrier<0>();
        else if (t >= 1 && t <= NS - 1 && sl + 1 < nsl) wait_stage_then_barrier<NB * (NS - 2) + NH>();
        else wait_stage_then_barrier<NB * (NS - 2)>();
        if (s + NS - 1 < steps) copy_weights((s + NS - 1) % NS);
        if (t == 0 && sl + 1 < nsl) copy_halo(sl + 1);
        const uint4* Hb = hbuf + (sl & 1) * HU;
#pragma unroll
        for (int tt = 0; tt < TPS; tt++) {
            const int tap = t * TPS + tt, ky = tap / 3, kx = tap - 3 * ky;
            const uint4* Bb = bst + (s % NS) * SU + tt * BN * 4;
            Frag fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; i++) {
                const int hp = hp0[i] + ky * HWD + kx;
                fa[i].u = Hb[hp * 4 + (kc ^ ((hp >> 1) & 3))];
            }
#pragma unroll
            for (int j = 0; j < TN; j++) fb[j].u = Bb[(wn * WTN + j * 16 + r) * 4 + bpos];
#pragma unroll
            for (int i = 0; i < TM; i++)
#pragma unroll
                for (int j = 0; j < TN; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v,
                                                                       acc[i][j], 0, 0, 0);
        }
    }
    wait_stage_then_barrier<0>();
    const int HWi = a.H * a.W;
    conv_epilogue<BN, BM, WGM>(
        a, acc, lds,
        [=](int row) { return n * HWi + (y0 + row / TW) * a.W + x0 + row % TW; }, n0);
}

template <int BN, int TH, int WGM, int NS, int TPS = 1>
static void launch_conv3_halo_t(const ConvArgs& a, hipStream_t st) {
    const unsigned gx = (unsigned)(a.N * (a.H / TH) * (a.W / 16));
    const unsigned gy = (unsigned)((a.Cout + BN - 1) / BN);
    hipLaunchKernelGGL((k_conv3_halo<BN, TH, WGM, NS, TPS>), dim3(gx, gy), dim3(256), 0, st, a);
}

// ConvNeXt block MLP for inference, fused: y = x2 + W2 GELU(W1 x + b1) + b2 with the 4C-wide
// hidden activation kept in LDS (the two 1 x 1 convolutions of the block write and read it
// through HBM otherwise).  A block takes 64 pixels: the x tile (64 x C) is staged once; the
// hidden channels go in chunks of 64: W1's chunk (64 x C) and W2's (C x 64) staged, GEMM 1
// into 2 x 2 wavefront tiles, bias + GELU + bf16 into the hidden tile, GEMM 2 accumulating the
// 64 x C output across chunks (wavefronts 2 x 2 over rows x channels).  The arithmetic is that
// of the two convolutions: fp32 accumulation in the same K order, the hidden value rounded to
// bf16, then acc + b2 + residual.  A: the pw2 arguments (output, bias, residual); w1, b1: pw1's.
template <int C>
__global__ __launch_bounds__(256) void k_mlp_fwd(ConvArgs a, const uint16_t* __restrict__ w1,
                                                 const float* __restrict__ b1) {
    constexpr int BM = 64, HC = 64, H4 = 4 * C;
    constexpr int XL = C + 8, HL = HC + 8;                   // padded bf16 rows
    constexpr int TN2 = C / 32;                              // GEMM 2 MFMA tiles per wavefront
    constexpr int XS = BM * XL, W1S = HC * XL, HS = BM * HL, W2S = C * HL;
    constexpr int TOT = XS + W1S + HS + W2S;                 // bf16 elements
    static_assert(BM * (C + 4) * 4 <= TOT * 2, "fp32 output tile fits the LDS");
    __shared__ __attribute__((aligned(16))) uint16_t lds[TOT];
    uint16_t* const xs = lds;
    uint16_t* const ws1 = xs + XS;
    uint16_t* const hs = ws1 + W1S;
    uint16_t* const ws2 = hs + HS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int M = a.N * a.H * a.W, m0 = blockIdx.x * BM;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    // x tile: 64 rows x C channels, 16-byte chunks (pixels past the end read as zero)
    for (int c = tid; c < BM * C / 8; c += 256) {
        const int row = c / (C / 8), k8 = c - row * (C / 8), m = m0 + row;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (m < M) v = *(const uint4*)(a.x + (size_t)m * a.ldx + a.xoff + k8 * 8);
        *(uint4*)&xs[row * XL + k8 * 8] = v;
    }
    v4f acc2[2][TN2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < TN2; j++) acc2[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int h0 = 0; h0 < H4; h0 += HC) {
        // the chunk's weights: W1 rows h0 .. h0 + 63 (C each), W2 columns h0 .. h0 + 63
        for (int c = tid; c < HC * C / 8; c += 256) {
            const int row = c / (C / 8), k8 = c - row * (C / 8);
            *(uint4*)&ws1[row * XL + k8 * 8] = *(const uint4*)(w1 + (size_t)(h0 + row) * C + k8 * 8);
        }
        for (int c = tid; c < C * HC / 8; c += 256) {
            const int row = c / (HC / 8), k8 = c - row * (HC / 8);
            *(uint4*)&ws2[row * HL + k8 * 8] = *(const uint4*)(a.w + (size_t)row * H4 + h0 + k8 * 8);
        }
        __syncthreads();
        // GEMM 1: hidden[64 x 64] = x . W1 chunk^T, wavefront tile 32 x 32
        v4f acc1[2][2];
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) acc1[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < C; k0 += 32) {
            Frag fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; i++) fa[i].u = *(const uint4*)&xs[(wm * 32 + i * 16 + r) * XL + k0 + kq];
#pragma unroll
            for (int j = 0; j < 2; j++) fb[j].u = *(const uint4*)&ws1[(wn * 32 + j * 16 + r) * XL + k0 + kq];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v,
                                                                        acc1[i][j], 0, 0, 0);
        }
        // bias + GELU, rounded to bf16 as the separate convolution stores it
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int col = wn * 32 + j * 16 + r;
            const float bias = b1 ? b1[h0 + col] : 0.f;
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int row = wm * 32 + i * 16 + (lane >> 4) * 4 + q;
                    hs[row * HL + col] = f2bf(gelu_f(acc1[i][j][q] + bias));
                }
        }
        __syncthreads();
        // GEMM 2: out[64 x C] += hidden . W2 chunk^T, wavefront tile 32 x C/2
#pragma unroll
        for (int k0 = 0; k0 < HC; k0 += 32) {
            Frag fa[2], fb[TN2];
#pragma unroll
            for (int i = 0; i < 2; i++) fa[i].u = *(const uint4*)&hs[(wm * 32 + i * 16 + r) * HL + k0 + kq];
#pragma unroll
            for (int j = 0; j < TN2; j++)
                fb[j].u = *(const uint4*)&ws2[(wn * (C / 2) + j * 16 + r) * HL + k0 + kq];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < TN2; j++)
                    acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v,
                                                                        acc2[i][j], 0, 0, 0);
        }
        __syncthreads();  // the chunk's tiles are free for the next chunk (and the epilogue)
    }
    conv_epilogue<C, BM, 2>(a, acc2, lds, [m0](int row) { return m0 + row; }, 0);
}

template <int C>
static void launch_mlp_t(const ConvArgs& a, const uint16_t* w1, const float* b1, hipStream_t st) {
    const int M = a.N * a.H * a.W;
    hipLaunchKernelGGL(k_mlp_fwd<C>, dim3((M + 63) / 64), dim3(256), 0, st, a, w1, b1);
}

bool launch_mlp_fwd(const ConvArgs& a, const uint16_t* w1, const float* b1, hipStream_t st) {
    if (a.K != 1 || a.Cout != a.Cin / 4 || a.Cout_store != a.Cout || a.shuffle || a.y32 || a.z ||
        a.act || a.xoff % 8 || a.ldx % 8)
        return false;
    // Measured (batch 8 at 256^2, us per layer, fused against the two convolutions): C = 32
    // 55.5 / 91.1, 64 41.7 / 54.5, 128 52.9 / 45.5, 256 108.8 / 40.0 (the deep layers have few
    // pixels, and the fused tile's registers and LDS leave one or two wavefronts per SIMD), so
    // only the two wide-image levels take it.
    switch (a.Cout) {
        case 32: launch_mlp_t<32>(a, w1, b1, st); return true;
        case 64: launch_mlp_t<64>(a, w1, b1, st); return true;
        default: return false;
    }
}

// Tile choice (measured, batch of 8 at 256^2 -> 512^2, inference per batch): 3 x 3 layers whose
// images split into 16-column tiles go to k_conv3_halo with 8-row tiles of 64 (or, for narrow
// outputs, 32) channels, three taps per K step and two copy stages (1.51 ms; one tap per step
// with three stages and 4-row 128-channel tiles for wide outputs 1.72 ms, three taps with those
// tiles 1.59 ms, three taps with three stages 1.83 ms); the other layers to k_conv_fwd with
// three stages and the largest tile that still gives the launch 1024 workgroups.
template <int NS>
static void launch_conv_fwd_ns(const ConvArgs& a, hipStream_t st) {
    const int M = a.N * a.H * a.W;
    if (a.Cout > 64) {
        const unsigned gy = (unsigned)((a.Cout + 127) / 128);
        if (!launch_conv_fwd_t<128, 64, 2, NS>(a, M, gy, false, st))
            launch_conv_fwd_t<128, 32, 2, NS>(a, M, gy, true, st);
    } else if (a.Cout > 32) {
        if (!launch_conv_fwd_t<64, 128, 4, NS>(a, M, 1u, false, st) &&
            !launch_conv_fwd_t<64, 64, 2, NS>(a, M, 1u, false, st))
            launch_conv_fwd_t<64, 32, 2, NS>(a, M, 1u, true, st);
    } else {
        if (!launch_conv_fwd_t<32, 128, 4, NS>(a, M, 1u, false, st))
            launch_conv_fwd_t<32, 64, 4, NS>(a, M, 1u, true, st);
    }
}

void launch_conv_fwd(const ConvArgs& a, hipStream_t st) {
    constexpr int NS = 3;
    if (a.K == 3 && a.W % 16 == 0 && a.H % 8 == 0) {
        if (a.Cout > 32) launch_conv3_halo_t<64, 8, 2, 2, 3>(a, st);
        else launch_conv3_halo_t<32, 8, 4, 2, 3>(a, st);
        return;
    }
    launch_conv_fwd_ns<NS>(a, st);
}

// Weight gradient: dW[co][t][ci] = sum_p dY[p][co] X[p + shift(t)][ci] over one chunk of
// 256 pixels per block (partials[chunk][co][t][ci], fp32), tiles 64 co x 64 ci, K = 32 pixels
// per step staged through LDS transposed so each fragment is 8 contiguous bf16.
__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs a) {
    // [channel][pixel] staging rows (32 pixels + 8 pad = 20 dwords), filled with packed pixel
    // pairs.  The x rows start 16 dwords past a multiple of 64 so that one store instruction's
    // lanes (16 pixel pairs x 2 channel groups x 2 arrays) hit 64 different banks.
    __shared__ __attribute__((aligned(16))) uint32_t stage[2 * 64 * 20 + 16];
    uint32_t* const sdy = stage;
    uint32_t* const sx = stage + 64 * 20 + 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int taps = a.K * a.K;
    const int t = blockIdx.z % taps, chunk = blockIdx.z / taps;
    const int co0 = blockIdx.x * 64, ci0 = blockIdx.y * 64;
    const int pad = (a.K - 1) / 2, dy = t / a.K - pad, dx = t % a.K - pad;
    const int HW = a.H * a.W, M = a.N * HW;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int wco = (wave & 1) * 32, wci = (wave >> 1) * 32;
    v4f acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    const int p_beg = chunk * a.chunk, p_end = min(M, p_beg + a.chunk);
    // loader: thread -> pixel pair pp, array arr (0: output gradient, 1: shifted input),
    // 8 channels from cg; each thread stores 8 packed (pixel 2pp, 2pp + 1) dwords
    const int pp = threadIdx.x & 15, arr = (threadIdx.x >> 4) & 1, cg = (threadIdx.x >> 5) * 8;
    uint32_t* const dst = arr ? sx : sdy;
    for (int p0 = p_beg; p0 < p_end; p0 += 32) {
        uint4 v[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int m = p0 + 2 * pp + h;
            v[h] = make_uint4(0, 0, 0, 0);
            if (m < p_end) {
                const int n = m / HW, y = (m % HW) / a.W, x = m % a.W;
                if (arr == 0) {
                    if (co0 + cg < a.Cout)
                        v[h] = *(const uint4*)(a.dy + ((size_t)(n * a.H + y) * a.W + x) * a.lddy +
                                               a.dyoff + co0 + cg);
                } else {
                    const int ys = y + dy, xs = x + dx;
                    if (ys >= 0 && ys < a.H && xs >= 0 && xs < a.W && ci0 + cg < a.Cin)
                        v[h] = *(const uint4*)(a.x + ((size_t)(n * a.H + ys) * a.W + xs) * a.ldx +
                                               a.xoff + ci0 + cg);
                }
            }
        }
        const uint32_t w0[4] = {v[0].x, v[0].y, v[0].z, v[0].w};
        const uint32_t w1[4] = {v[1].x, v[1].y, v[1].z, v[1].w};
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; e++) {
            // channels cg + 2e (low halves) and cg + 2e + 1 (high halves)
            dst[(cg + 2 * e) * 20 + pp] = (w0[e] & 0xFFFFu) | (w1[e] << 16);
            dst[(cg + 2 * e + 1) * 20 + pp] = (w0[e] >> 16) | (w1[e] & 0xFFFF0000u);
        }
        __syncthreads();
        Frag fa[2], fb[2];
        for (int i = 0; i < 2; i++) fa[i].u = *(const uint4*)&sdy[(wco + i * 16 + r) * 20 + kq / 2];
        for (int j = 0; j < 2; j++) fb[j].u = *(const uint4*)&sx[(wci + j * 16 + r) * 20 + kq / 2];
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i].v, fb[j].v, acc[i][j], 0,
                                                                   0, 0);
    }
    float* out = a.partial + (size_t)chunk * a.Cout * taps * a.Cin;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            const int ci = ci0 + wci + j * 16 + r;
            for (int q = 0; q < 4; q++) {
                const int co = co0 + wco + i * 16 + (lane >> 4) * 4 + q;
                if (co < a.Cout && ci < a.Cin) out[((size_t)co * taps + t) * a.Cin + ci] = acc[i][j][q];
            }
        }
}

void launch_conv_wgrad(const WgradArgs& a, int n_chunks, hipStream_t st) {
    hipLaunchKernelGGL(k_conv_wgrad, dim3((a.Cout + 63) / 64, (a.Cin + 63) / 64,
                                          n_chunks * a.K * a.K),
                       dim3(256), 0, st, a);
}

// out[i] = sum over chunks c of part[c * stride + (i / inner) * outer + i % inner + off]:
// gathers one parameter tensor out of interleaved per-chunk partials.  Few chunks: one thread
// per output sums them in chunk order.  Many chunks: one block per output, thread t sums
// chunks t, t + 256, ... in order and a fixed tree combines the threads.  Either way the
// result depends only on the shapes, never on timing.
__global__ void k_reduce_chunks(const float* __restrict__ part, int n_chunks, size_t stride,
                                size_t n, int inner, int outer, int off, float* __restrict__ out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t src = (i / inner) * outer + i % inner + off;
        float s = 0.f;
        for (int c = 0; c < n_chunks; c++) s += part[(size_t)c * stride + src];
        out[i] = s;
    }
}

__global__ __launch_bounds__(256) void k_reduce_chunks_tree(const float* __restrict__ part,
                                                            int n_chunks, size_t stride, size_t n,
                                                            int inner, int outer, int off,
                                                            float* __restrict__ out) {
    __shared__ float red[256];
    const int tid = threadIdx.x;
    for (size_t i = blockIdx.x; i < n; i += gridDim.x) {
        const size_t src = (i / inner) * outer + i % inner + off;
        float s = 0.f;
        for (int c = tid; c < n_chunks; c += 256) s += part[(size_t)c * stride + src];
        red[tid] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) out[i] = red[0];
        __syncthreads();
    }
}

void launch_reduce_chunks(const float* part, int n_chunks, size_t stride, size_t n, int inner,
                          int outer, int off, float* out, hipStream_t st) {
    if (n_chunks > 32) {
        const unsigned b = (unsigned)std::min<size_t>(n, 65536);
        hipLaunchKernelGGL(k_reduce_chunks_tree, dim3(b > 0 ? b : 1), dim3(256), 0, st, part,
                           n_chunks, stride, n, inner, outer, off, out);
        return;
    }
    int b = (int)((n + 255) / 256);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(b > 0 ? b : 1), dim3(256), 0, st, part, n_chunks,
                       stride, n, inner, outer, off, out);
}

// Column sums of a bf16 [M][ld] tensor (channels off..off+C) per chunk of rows: bias grads.
__global__ void k_colsum(const uint16_t* __restrict__ y, int M, int ld, int off, int C,
                         int chunk, float* __restrict__ part) {
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int m0 = blockIdx.x * chunk, m1 = min(M, m0 + chunk);
    float s = 0.f;
    for (int m = m0; m < m1; m++) s += bf2f(y[(size_t)m * ld + off + c]);
    part[(size_t)blockIdx.x * C + c] = s;
}

void launch_colsum(const uint16_t* y, int M, int ld, int off, int C, int chunk, float* part,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_colsum, dim3((M + chunk - 1) / chunk, (C + 63) / 64), dim3(64), 0, st, y,
                       M, ld, off, C, chunk, part);
}

// Flips a weight tensor for the data gradient: wt[ci][t'][co] = w[co][taps-1-t'][ci]
// (Cin_t = Cout padded to cpad; extra output channels zero).
__global__ void k_weight_flip(const uint16_t* __restrict__ w, int Cout, int taps, int Cin,
                              int co_pad, uint16_t* __restrict__ wt) {
    const size_t n = (size_t)Cin * taps * co_pad;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int co = (int)(i % co_pad);
        const int t = (int)((i / co_pad) % taps);
        const int ci = (int)(i / ((size_t)co_pad * taps));
        wt[i] = co < Cout ? w[((size_t)co * taps + (taps - 1 - t)) * Cin + ci] : (uint16_t)0;
    }
}

void launch_weight_flip(const uint16_t* w, int Cout, int taps, int Cin, int co_pad, uint16_t* wt,
                        hipStream_t st) {
    const size_t n = (size_t)Cin * taps * co_pad;
    int b = (int)((n + 255) / 256);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_weight_flip, dim3(b), dim3(256), 0, st, w, Cout, taps, Cin, co_pad, wt);
}

// ------------------------------------------------------------------------------------------
// Elementwise / small kernels
// ------------------------------------------------------------------------------------------

// Pixel unshuffle of a gradient: d[n][y][x][c*4 + 2 sy + sx] = g[n][2y+sy][2x+sx][goff + c].
__global__ void k_unshuffle(const uint16_t* __restrict__ g, int N, int H, int W, int C, int ldg,
                           int goff, uint16_t* __restrict__ d, int ldd) {
    const size_t n = (size_t)N * H * W * 4 * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % (4 * C));
        const size_t pix = i / (4 * C);
        const int x = (int)(pix % W), y = (int)((pix / W) % H), b = (int)(pix / ((size_t)W * H));
        const int c = k >> 2, sy = (k >> 1) & 1, sx = k & 1;
        d[pix * ldd + k] = g[((size_t)(b * 2 * H + 2 * y + sy) * (2 * W) + 2 * x + sx) * ldg + goff + c];
    }
}

void launch_unshuffle(const uint16_t* g, int N, int H, int W, int C, int ldg, int goff,
                      uint16_t* d, int ldd, hipStream_t st) {
    const size_t n = (size_t)N * H * W * 4 * C;
    int b = (int)((n + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_unshuffle, dim3(b), dim3(256), 0, st, g, N, H, W, C, ldg, goff, d, ldd);
}

// GELU backward: dz = dy * (Phi(z) + z phi(z)) (erf form, erf_as).
__global__ void k_gelu_bwd(const uint16_t* __restrict__ z, const uint16_t* __restrict__ dy,
                           size_t n, uint16_t* __restrict__ dz) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float v = bf2f(z[i]);
        const float cdf = 0.5f * (1.f + erf_as(v * 0.70710678118654752f));
        const float pdf = 0.3989422804014327f * __expf(-0.5f * v * v);
        dz[i] = f2bf(bf2f(dy[i]) * (cdf + v * pdf));
    }
}

void launch_gelu_bwd(const uint16_t* z, const uint16_t* dy, size_t n, uint16_t* dz,
                     hipStream_t st) {
    int b = (int)((n + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_gelu_bwd, dim3(b), dim3(256), 0, st, z, dy, n, dz);
}

// y[i] = a[i] + b[i] over strided channel slices: rows M, C channels.
__global__ void k_add(const uint16_t* __restrict__ a, int lda, int aoff,
                      const uint16_t* __restrict__ b, int ldb, int boff, int M, int C,
                      uint16_t* __restrict__ y, int ldy, int yoff) {
    const size_t n = (size_t)M * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t m = i / C;
        const int c = (int)(i % C);
        y[m * ldy + yoff + c] = f2bf(bf2f(a[m * lda + aoff + c]) + bf2f(b[m * ldb + boff + c]));
    }
}

void launch_add(const uint16_t* a, int lda, int aoff, const uint16_t* b, int ldb, int boff, int M,
                int C, uint16_t* y, int ldy, int yoff, hipStream_t st) {
    const size_t n = (size_t)M * C;
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_add, dim3(bl), dim3(256), 0, st, a, lda, aoff, b, ldb, boff, M, C, y, ldy,
                       yoff);
}

// Copy of a channel slice (concat of skips into a decoder buffer).
__global__ void k_copy_slice(const uint16_t* __restrict__ a, int lda, int aoff, int M, int C,
                             uint16_t* __restrict__ y, int ldy, int yoff) {
    const size_t n = (size_t)M * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t m = i / C;
        const int c = (int)(i % C);
        y[m * ldy + yoff + c] = a[m * lda + aoff + c];
    }
}

void launch_copy_slice(const uint16_t* a, int lda, int aoff, int M, int C, uint16_t* y, int ldy,
                       int yoff, hipStream_t st) {
    const size_t n = (size_t)M * C;
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_copy_slice, dim3(bl), dim3(256), 0, st, a, lda, aoff, M, C, y, ldy, yoff);
}

// Stem: 3x3 convolution of the one-channel input (fp32) into C channels, + bias, pre-activation
// z and GELU a (bf16).
__global__ void k_stem_fwd(const float* __restrict__ x, int N, int H, int W, int C,
                           const float* __restrict__ w, const float* __restrict__ b,
                           uint16_t* __restrict__ z, uint16_t* __restrict__ a) {
    // 32-bit indices: N H W C < 2^31 (the training/inference batches are far smaller)
    const uint32_t n = (uint32_t)N * H * W * C;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int c = (int)(i % (uint32_t)C);
        const uint32_t pix = i / (uint32_t)C;
        const int xx = (int)(pix % (uint32_t)W), yy = (int)((pix / (uint32_t)W) % (uint32_t)H),
                  bn = (int)(pix / ((uint32_t)W * H));
        float s = b[c];
        for (int t = 0; t < 9; t++) {
            const int y = yy + t / 3 - 1, x2 = xx + t % 3 - 1;
            if (y >= 0 && y < H && x2 >= 0 && x2 < W) s += x[(size_t)(bn * H + y) * W + x2] * w[c * 9 + t];
        }
        z[i] = f2bf(s);
        a[i] = f2bf(gelu_f(s));
    }
}

// The stem with 8 channels per thread: the 9 input taps are loaded once for 8 outputs, which
// leave as 16-byte stores (C % 8 == 0, N H W C < 2^32).
__global__ void k_stem_fwd8(const float* __restrict__ x, int N, int H, int W, int C,
                            const float* __restrict__ w, const float* __restrict__ b,
                            uint16_t* __restrict__ z, uint16_t* __restrict__ a) {
    const uint32_t G = (uint32_t)C / 8;
    const uint32_t n = (uint32_t)N * H * W * G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = i % G, pix = i / G;
        const int xx = (int)(pix % (uint32_t)W), yy = (int)((pix / (uint32_t)W) % (uint32_t)H),
                  bn = (int)(pix / ((uint32_t)W * H));
        float in[9];
#pragma unroll
        for (int t = 0; t < 9; t++) {
            const int y = yy + t / 3 - 1, x2 = xx + t % 3 - 1;
            in[t] = (y >= 0 && y < H && x2 >= 0 && x2 < W) ? x[(size_t)(bn * H + y) * W + x2] : 0.f;
        }
        uint32_t zo[4], ao[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            float v[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int c = (int)g * 8 + e + h;
                float s = b[c];
#pragma unroll
                for (int t = 0; t < 9; t++) s += in[t] * w[c * 9 + t];
                v[h] = s;
            }
            zo[e / 2] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
            ao[e / 2] = (uint32_t)f2bf(gelu_f(v[0])) | ((uint32_t)f2bf(gelu_f(v[1])) << 16);
        }
        *(uint4*)(z + (size_t)pix * C + g * 8) = make_uint4(zo[0], zo[1], zo[2], zo[3]);
        *(uint4*)(a + (size_t)pix * C + g * 8) = make_uint4(ao[0], ao[1], ao[2], ao[3]);
    }
}

void launch_stem_fwd(const float* x, int N, int H, int W, int C, const float* w, const float* b,
                     uint16_t* z, uint16_t* a, hipStream_t st) {
    if (C % 8 == 0 && (uint64_t)N * H * W * (C / 8) < (1ull << 32)) {
        const size_t n = (size_t)N * H * W * (C / 8);
        const int bl = (int)std::min<size_t>(16384, (n + 255) / 256);
        hipLaunchKernelGGL(k_stem_fwd8, dim3(bl), dim3(256), 0, st, x, N, H, W, C, w, b, z, a);
        return;
    }
    // the kernel indexes in 32 bits: split the batch so that each launch stays below 2^32
    const size_t per_img = (size_t)H * W * C;
    const int chunk = (int)std::max<size_t>(1, ((1ull << 32) - 1) / per_img);
    for (int n0 = 0; n0 < N; n0 += chunk) {
        const int nb = std::min(chunk, N - n0);
        const size_t n = (size_t)nb * per_img;
        int bl = (int)((n + 255) / 256);
        if (bl > 8192) bl = 8192;
        hipLaunchKernelGGL(k_stem_fwd, dim3(bl), dim3(256), 0, st, x + (size_t)n0 * H * W, nb, H, W,
                           C, w, b, z + (size_t)n0 * per_img, a + (size_t)n0 * per_img);
    }
}

// Stem weight/bias gradient partials: block = chunk of pixels; part[chunk][c*10 + t] (t = 9: bias).
__global__ void k_stem_wgrad(const float* __restrict__ x, int N, int H, int W, int C,
                             const uint16_t* __restrict__ dz, int chunk, float* __restrict__ part) {
    const int c = threadIdx.x;
    if (c >= C) return;
    const int M = N * H * W;
    const int m0 = blockIdx.x * chunk, m1 = min(M, m0 + chunk);
    float s[10];
    for (int t = 0; t < 10; t++) s[t] = 0.f;
    for (int m = m0; m < m1; m++) {
        const int xx = m % W, yy = (m / W) % H, bn = m / (W * H);
        const float g = bf2f(dz[(size_t)m * C + c]);
        for (int t = 0; t < 9; t++) {
            const int y = yy + t / 3 - 1, x2 = xx + t % 3 - 1;
            if (y >= 0 && y < H && x2 >= 0 && x2 < W) s[t] += g * x[(size_t)(bn * H + y) * W + x2];
        }
        s[9] += g;
    }
    for (int t = 0; t < 10; t++) part[((size_t)blockIdx.x * C + c) * 10 + t] = s[t];
}

void launch_stem_wgrad(const float* x, int N, int H, int W, int C, const uint16_t* dz, int chunk,
                       float* part, hipStream_t st) {
    const int M = N * H * W;
    hipLaunchKernelGGL(k_stem_wgrad, dim3((M + chunk - 1) / chunk), dim3(C <= 64 ? 64 : 256), 0, st,
                       x, N, H, W, C, dz, chunk, part);
}

// Tap-major copy of depthwise weights: wt[tap][c] = w[c][tap].
__global__ void k_dw_wt(const float* __restrict__ w, int C, float* __restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 49 * C) wt[i] = w[(i % C) * 49 + i / C];
}

void launch_dw_wt(const float* w, int C, float* wt, hipStream_t st) {
    hipLaunchKernelGGL(k_dw_wt, dim3((49 * C + 255) / 256), dim3(256), 0, st, w, C, wt);
}

// Depthwise 7x7 (C % 8 == 0): one thread per (pixel, 8 channels), 16-byte activation loads and
// 32-byte weight loads per tap.  FLIP = 0: y = dw(x) + b.  FLIP = 1: data gradient,
// dx[p] = sum over taps of dy[p - shift] w[tap] (no bias).
template <int FLIP>
__global__ void k_dw8(const uint16_t* __restrict__ x, int N, int H, int W, int C,
                      const float* __restrict__ wt, const float* __restrict__ b,
                      uint16_t* __restrict__ y) {
    const int G = C / 8;
    const size_t n = (size_t)N * H * W * G;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c0 = (int)(i % G) * 8;
        const size_t pix = i / G;
        const int xx = (int)(pix % W), yy = (int)((pix / W) % H), bn = (int)(pix / ((size_t)W * H));
        float acc[8];
#pragma unroll
        for (int k = 0; k < 8; k++) acc[k] = (!FLIP && b) ? b[c0 + k] : 0.f;
        for (int a = 0; a < 7; a++) {
            const int yi = FLIP ? yy - a + 3 : yy + a - 3;
            if (yi < 0 || yi >= H) continue;
            for (int q = 0; q < 7; q++) {
                const int xi = FLIP ? xx - q + 3 : xx + q - 3;
                if (xi < 0 || xi >= W) continue;
                const uint4 v = *(const uint4*)(x + ((size_t)(bn * H + yi) * W + xi) * C + c0);
                const float4 w0 = *(const float4*)(wt + (a * 7 + q) * C + c0);
                const float4 w1 = *(const float4*)(wt + (a * 7 + q) * C + c0 + 4);
                const uint16_t* h = (const uint16_t*)&v;
                acc[0] += bf2f(h[0]) * w0.x;
                acc[1] += bf2f(h[1]) * w0.y;
                acc[2] += bf2f(h[2]) * w0.z;
                acc[3] += bf2f(h[3]) * w0.w;
                acc[4] += bf2f(h[4]) * w1.x;
                acc[5] += bf2f(h[5]) * w1.y;
                acc[6] += bf2f(h[6]) * w1.z;
                acc[7] += bf2f(h[7]) * w1.w;
            }
        }
        uint4 o;
        uint16_t* oh = (uint16_t*)&o;
#pragma unroll
        for (int k = 0; k < 8; k++) oh[k] = f2bf(acc[k]);
        *(uint4*)(y + pix * C + c0) = o;
    }
}

// The same 7x7 depthwise convolution with each thread computing 4 consecutive pixels of a row
// for 8 channels: per tap row it loads the 10-pixel input window once and each tap's weights
// once for the 4 pixels (3.5x fewer loads than one pixel per thread).  32-bit indices
// (N H W C < 2^31, checked by the launcher); W % 4 == 0.
template <int FLIP>
__global__ __launch_bounds__(256, 2) void k_dw8x4(const uint16_t* __restrict__ x, int N, int H,
                                                  int W, int C,
                        const float* __restrict__ wt, const float* __restrict__ b,
                        uint16_t* __restrict__ y) {
    const uint32_t G = (uint32_t)C / 8, XB = (uint32_t)W / 4;
    const uint32_t n = (uint32_t)N * H * XB * G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = i % G, r = i / G;
        const int xb = (int)(r % XB), yy = (int)((r / XB) % H), bn = (int)(r / (XB * H));
        const int c0 = (int)g * 8, x0 = xb * 4;
        float acc[4][8];
#pragma unroll
        for (int p = 0; p < 4; p++)
#pragma unroll
            for (int k = 0; k < 8; k++) acc[p][k] = (!FLIP && b) ? b[c0 + k] : 0.f;
        for (int a = 0; a < 7; a++) {
            const int yi = FLIP ? yy - a + 3 : yy + a - 3;
            if (yi < 0 || yi >= H) continue;
            const uint16_t* row = x + ((size_t)(bn * H + yi) * W) * C + c0;
            float in[10][8];
#pragma unroll
            for (int j = 0; j < 10; j++) {
                const int xi = x0 - 3 + j;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (xi >= 0 && xi < W) v = *(const uint4*)(row + (size_t)xi * C);
                const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    in[j][2 * e] = bf2f((uint16_t)(w4[e] & 0xFFFFu));
                    in[j][2 * e + 1] = bf2f((uint16_t)(w4[e] >> 16));
                }
            }
#pragma unroll
            for (int q = 0; q < 7; q++) {
                const float4 w0 = *(const float4*)(wt + (a * 7 + q) * C + c0);
                const float4 w1 = *(const float4*)(wt + (a * 7 + q) * C + c0 + 4);
                const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
                for (int p = 0; p < 4; p++) {
                    const int j = FLIP ? p - q + 6 : p + q;  // input x = x0 - 3 + j
#pragma unroll
                    for (int k = 0; k < 8; k++) acc[p][k] += in[j][k] * wv[k];
                }
            }
        }
#pragma unroll
        for (int p = 0; p < 4; p++) {
            uint32_t o[4];
#pragma unroll
            for (int e = 0; e < 4; e++)
                o[e] = (uint32_t)f2bf(acc[p][2 * e]) | ((uint32_t)f2bf(acc[p][2 * e + 1]) << 16);
            *(uint4*)(y + ((size_t)(bn * H + yy) * W + x0 + p) * C + c0) =
                make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
}

static bool dw_fast(int N, int H, int W, int C) {
    return W % 4 == 0 && (uint64_t)N * H * W * C < (1ull << 31);
}

void launch_dw_fwd(const uint16_t* x, int N, int H, int W, int C, const float* wt, const float* b,
                   uint16_t* y, hipStream_t st) {
    if (dw_fast(N, H, W, C)) {
        const size_t n = (size_t)N * H * (W / 4) * (C / 8);
        const int bl = (int)std::min<size_t>(16384, (n + 255) / 256);
        hipLaunchKernelGGL(k_dw8x4<0>, dim3(bl), dim3(256), 0, st, x, N, H, W, C, wt, b, y);
        return;
    }
    const size_t n = (size_t)N * H * W * (C / 8);
    int bl = (int)((n + 255) / 256);
    if (bl > 16384) bl = 16384;
    hipLaunchKernelGGL(k_dw8<0>, dim3(bl), dim3(256), 0, st, x, N, H, W, C, wt, b, y);
}

void launch_dw_dgrad(const uint16_t* dy, int N, int H, int W, int C, const float* wt, uint16_t* dx,
                     hipStream_t st) {
    if (dw_fast(N, H, W, C)) {
        const size_t n = (size_t)N * H * (W / 4) * (C / 8);
        const int bl = (int)std::min<size_t>(16384, (n + 255) / 256);
        hipLaunchKernelGGL(k_dw8x4<1>, dim3(bl), dim3(256), 0, st, dy, N, H, W, C, wt, nullptr, dx);
        return;
    }
    const size_t n = (size_t)N * H * W * (C / 8);
    int bl = (int)((n + 255) / 256);
    if (bl > 16384) bl = 16384;
    hipLaunchKernelGGL(k_dw8<1>, dim3(bl), dim3(256), 0, st, dy, N, H, W, C, wt, nullptr, dx);
}

// Depthwise weight/bias gradient partials: block (row chunk, channel group of 64); each thread
// owns one channel and accumulates its 49 taps + bias over the block's rows.
__global__ void k_dw_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
                           int N, int H, int W, int C, int rows, float* __restrict__ part) {
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= C) return;
    const int NH = N * H;
    const int r0 = blockIdx.x * rows, r1 = min(NH, r0 + rows);
    float s[50];
    for (int t = 0; t < 50; t++) s[t] = 0.f;
    for (int r = r0; r < r1; r++) {
        const int bn = r / H, yy = r % H;
        for (int xx = 0; xx < W; xx++) {
            const float g = bf2f(dy[((size_t)r * W + xx) * C + c]);
            s[49] += g;
            for (int a = 0; a < 7; a++) {
                const int yi = yy + a - 3;
                if (yi < 0 || yi >= H) continue;
                for (int q = 0; q < 7; q++) {
                    const int xi = xx + q - 3;
                    if (xi < 0 || xi >= W) continue;
                    s[a * 7 + q] += g * bf2f(x[((size_t)(bn * H + yi) * W + xi) * C + c]);
                }
            }
        }
    }
    for (int t = 0; t < 50; t++) part[((size_t)blockIdx.x * C + c) * 50 + t] = s[t];
}

void launch_dw_wgrad(const uint16_t* x, const uint16_t* dy, int N, int H, int W, int C, int rows,
                     float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_dw_wgrad, dim3((N * H + rows - 1) / rows, (C + 63) / 64), dim3(64), 0, st,
                       x, dy, N, H, W, C, rows, part);
}

// The same partials per (image row, segment of kDwSeg pixels): one thread per (chunk, tap row
// a, 8 channels) slides a 7-pixel window of the input row yy + a - 3 along its segment, so each
// input and output-gradient value is loaded once per thread (16-byte loads) and used for 7 taps
// x 8 channels; the a = 0 thread also sums the bias gradient.  C % 8 == 0.
__global__ __launch_bounds__(256, 2) void k_dw_wgrad8(const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ dy, int N,
                                                      int H, int W, int C,
                                                      float* __restrict__ part) {
    const uint32_t G = (uint32_t)C / 8, nseg = (uint32_t)(W + kDwSeg - 1) / kDwSeg;
    const uint32_t n = (uint32_t)N * H * nseg * 7 * G;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = i % G;
        uint32_t t = i / G;
        const int a = (int)(t % 7);
        t /= 7;
        const uint32_t sg = t % nseg, r = t / nseg, chunk = t;
        const int bn = (int)(r / (uint32_t)H), yy = (int)(r % (uint32_t)H), yi = yy + a - 3;
        const int c0 = (int)g * 8, xs = (int)sg * kDwSeg, xe = min(W, xs + kDwSeg);
        const bool rowok = yi >= 0 && yi < H;
        float acc[7][8], bsum[8];
#pragma unroll
        for (int q = 0; q < 7; q++)
#pragma unroll
            for (int k = 0; k < 8; k++) acc[q][k] = 0.f;
#pragma unroll
        for (int k = 0; k < 8; k++) bsum[k] = 0.f;
        if (rowok || a == 0) {
            const uint16_t* xrow = x + ((size_t)(bn * H + (rowok ? yi : 0)) * W) * C + c0;
            auto ldx = [&](int xi, float* o) {
                uint4 v = make_uint4(0, 0, 0, 0);
                if (rowok && xi >= 0 && xi < W) v = *(const uint4*)(xrow + (size_t)xi * C);
                const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    o[2 * e] = bf2f((uint16_t)(w4[e] & 0xFFFFu));
                    o[2 * e + 1] = bf2f((uint16_t)(w4[e] >> 16));
                }
            };
            float win[7][8];
#pragma unroll
            for (int q = 0; q < 7; q++) ldx(xs + q - 3, win[q]);
            const uint16_t* drow = dy + ((size_t)r * W) * C + c0;
            for (int xx = xs; xx < xe; xx++) {
                const uint4 dv = *(const uint4*)(drow + (size_t)xx * C);
                const uint32_t d4[4] = {dv.x, dv.y, dv.z, dv.w};
                float d[8];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    d[2 * e] = bf2f((uint16_t)(d4[e] & 0xFFFFu));
                    d[2 * e + 1] = bf2f((uint16_t)(d4[e] >> 16));
                }
#pragma unroll
                for (int k = 0; k < 8; k++) bsum[k] += d[k];
#pragma unroll
                for (int q = 0; q < 7; q++)
#pragma unroll
                    for (int k = 0; k < 8; k++) acc[q][k] += d[k] * win[q][k];
#pragma unroll
                for (int q = 0; q < 6; q++)
#pragma unroll
                    for (int k = 0; k < 8; k++) win[q][k] = win[q + 1][k];
                ldx(xx + 4, win[6]);
            }
        }
        float* out = part + ((size_t)chunk * C + c0) * 50;
#pragma unroll
        for (int k = 0; k < 8; k++) {
#pragma unroll
            for (int q = 0; q < 7; q++) out[(size_t)k * 50 + a * 7 + q] = acc[q][k];
            if (a == 0) out[(size_t)k * 50 + 49] = bsum[k];
        }
    }
}

static bool dw_wgrad8_ok(int N, int H, int W, int C) {
    return C % 8 == 0 && (uint64_t)N * H * W * C < (1ull << 31);
}

int dw_wgrad_chunks(int N, int H, int W, int C) {
    return dw_wgrad8_ok(N, H, W, C) ? N * H * ((W + kDwSeg - 1) / kDwSeg) : N * H;
}

void launch_dw_wgrad_auto(const uint16_t* x, const uint16_t* dy, int N, int H, int W, int C,
                          float* part, hipStream_t st) {
    if (dw_wgrad8_ok(N, H, W, C)) {
        const size_t n = (size_t)dw_wgrad_chunks(N, H, W, C) * 7 * (C / 8);
        const int bl = (int)std::min<size_t>(16384, (n + 255) / 256);
        hipLaunchKernelGGL(k_dw_wgrad8, dim3(bl), dim3(256), 0, st, x, dy, N, H, W, C, part);
        return;
    }
    launch_dw_wgrad(x, dy, N, H, W, C, 1, part, st);
}

// LayerNorm over C per pixel (one wavefront per pixel): y = (x - mu) rstd * g + b; saves
// mu and rstd.
__global__ void k_ln_fwd(const uint16_t* __restrict__ x, int M, int C, const float* __restrict__ g,
                         const float* __restrict__ b, float eps, uint16_t* __restrict__ y,
                         float* __restrict__ stats) {
    const int lane = threadIdx.x & 63;
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= M) return;
    const uint16_t* xr = x + (size_t)m * C;
    float s = 0.f, s2 = 0.f;
    for (int c = lane; c < C; c += 64) {
        const float v = bf2f(xr[c]);
        s += v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float mu = s / C;
    for (int c = lane; c < C; c += 64) {
        const float v = bf2f(xr[c]) - mu;
        s2 += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    const float rstd = rsqrtf(s2 / C + eps);
    for (int c = lane; c < C; c += 64) y[(size_t)m * C + c] = f2bf((bf2f(xr[c]) - mu) * rstd * g[c] + b[c]);
    if (lane == 0) {
        stats[2 * m] = mu;
        stats[2 * m + 1] = rstd;
    }
}

// LayerNorm over channels with C / 8 lanes per pixel (8 channels = one 16-byte load each) and
// 64 / (C / 8) pixels per wavefront; C / 8 a power of two <= 64.
__global__ void k_ln_fwd8(const uint16_t* __restrict__ x, int M, int C, const float* __restrict__ g,
                          const float* __restrict__ b, float eps, uint16_t* __restrict__ y,
                          float* __restrict__ stats) {
    const int lp = C >> 3;  // lanes per pixel
    const int lane = threadIdx.x & 63, sub = lane & (lp - 1);
    const int m = (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / lp) + lane / lp;
    const bool ok = m < M;
    float v[8];
    if (ok) {
        const uint4 u = *(const uint4*)(x + (size_t)m * C + sub * 8);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v[2 * e] = bf2f((uint16_t)(w[e] & 0xFFFFu));
            v[2 * e + 1] = bf2f((uint16_t)(w[e] >> 16));
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; e++) v[e] = 0.f;
    }
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < 8; e++) s += v[e];
    for (int o = 1; o < lp; o <<= 1) s += __shfl_xor(s, o);
    const float mu = s / C;
    float s2 = 0.f;
#pragma unroll
    for (int e = 0; e < 8; e++) s2 += (v[e] - mu) * (v[e] - mu);
    for (int o = 1; o < lp; o <<= 1) s2 += __shfl_xor(s2, o);
    const float rstd = rsqrtf(s2 / C + eps);
    if (!ok) return;
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int c = sub * 8 + 2 * e;
        const uint16_t lo = f2bf((v[2 * e] - mu) * rstd * g[c] + b[c]);
        const uint16_t hi = f2bf((v[2 * e + 1] - mu) * rstd * g[c + 1] + b[c + 1]);
        w[e] = (uint32_t)lo | ((uint32_t)hi << 16);
    }
    *(uint4*)(y + (size_t)m * C + sub * 8) = make_uint4(w[0], w[1], w[2], w[3]);
    if (sub == 0) {
        stats[2 * m] = mu;
        stats[2 * m + 1] = rstd;
    }
}

void launch_ln_fwd(const uint16_t* x, int M, int C, const float* g, const float* b, float eps,
                   uint16_t* y, float* stats, hipStream_t st) {
    const int lp = C / 8;
    if (C % 8 == 0 && lp <= 64 && (lp & (lp - 1)) == 0) {
        const int per_block = 4 * (64 / lp);
        hipLaunchKernelGGL(k_ln_fwd8, dim3((M + per_block - 1) / per_block), dim3(256), 0, st, x, M,
                           C, g, b, eps, y, stats);
        return;
    }
    hipLaunchKernelGGL(k_ln_fwd, dim3((M + 3) / 4), dim3(256), 0, st, x, M, C, g, b, eps, y, stats);
}

// LayerNorm backward: dx = rstd (dxh - mean(dxh) - xh mean(dxh xh)), dxh = dy g.
__global__ void k_ln_bwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy, int M,
                         int C, const float* __restrict__ g, const float* __restrict__ stats,
                         uint16_t* __restrict__ dx) {
    const int lane = threadIdx.x & 63;
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= M) return;
    const float mu = stats[2 * m], rstd = stats[2 * m + 1];
    const uint16_t* xr = x + (size_t)m * C;
    const uint16_t* dr = dy + (size_t)m * C;
    float a = 0.f, b2 = 0.f;
    for (int c = lane; c < C; c += 64) {
        const float xh = (bf2f(xr[c]) - mu) * rstd, d = bf2f(dr[c]) * g[c];
        a += d;
        b2 += d * xh;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b2 += __shfl_xor(b2, o);
    }
    a /= C;
    b2 /= C;
    for (int c = lane; c < C; c += 64) {
        const float xh = (bf2f(xr[c]) - mu) * rstd, d = bf2f(dr[c]) * g[c];
        dx[(size_t)m * C + c] = f2bf(rstd * (d - a - xh * b2));
    }
}

void launch_ln_bwd(const uint16_t* x, const uint16_t* dy, int M, int C, const float* g,
                   const float* stats, uint16_t* dx, hipStream_t st) {
    hipLaunchKernelGGL(k_ln_bwd, dim3((M + 3) / 4), dim3(256), 0, st, x, dy, M, C, g, stats, dx);
}

// LayerNorm gamma/beta gradient partials per chunk of rows: part[chunk][c][2] = (dy*xh, dy).
__global__ void k_ln_pgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy, int M,
                           int C, const float* __restrict__ stats, int chunk,
                           float* __restrict__ part) {
    const int c = blockIdx.y * 64 + threadIdx.x;
    if (c >= C) return;
    const int m0 = blockIdx.x * chunk, m1 = min(M, m0 + chunk);
    float sg = 0.f, sb = 0.f;
    for (int m = m0; m < m1; m++) {
        const float xh = (bf2f(x[(size_t)m * C + c]) - stats[2 * m]) * stats[2 * m + 1];
        const float d = bf2f(dy[(size_t)m * C + c]);
        sg += d * xh;
        sb += d;
    }
    part[((size_t)blockIdx.x * C + c) * 2] = sg;
    part[((size_t)blockIdx.x * C + c) * 2 + 1] = sb;
}

void launch_ln_pgrad(const uint16_t* x, const uint16_t* dy, int M, int C, const float* stats,
                     int chunk, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_ln_pgrad, dim3((M + chunk - 1) / chunk, (C + 63) / 64), dim3(64), 0, st,
                       x, dy, M, C, stats, chunk, part);
}

// 2x2 max pooling (first maximum in (0,0),(0,1),(1,0),(1,1) order wins); arg in 0..3.
__global__ void k_pool_fwd(const uint16_t* __restrict__ x, int N, int H, int W, int C,
                           uint16_t* __restrict__ y, uint8_t* __restrict__ arg) {
    const int Ho = H / 2, Wo = W / 2;
    const size_t n = (size_t)N * Ho * Wo * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t pix = i / C;
        const int xo = (int)(pix % Wo), yo = (int)((pix / Wo) % Ho), bn = (int)(pix / ((size_t)Wo * Ho));
        float best = -FLT_MAX;
        int ba = 0;
        for (int k = 0; k < 4; k++) {
            const float v = bf2f(x[((size_t)(bn * H + 2 * yo + (k >> 1)) * W + 2 * xo + (k & 1)) * C + c]);
            if (v > best) {
                best = v;
                ba = k;
            }
        }
        y[i] = f2bf(best);
        arg[i] = (uint8_t)ba;
    }
}

void launch_pool_fwd(const uint16_t* x, int N, int H, int W, int C, uint16_t* y, uint8_t* arg,
                     hipStream_t st) {
    const size_t n = (size_t)N * (H / 2) * (W / 2) * C;
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_pool_fwd, dim3(bl), dim3(256), 0, st, x, N, H, W, C, y, arg);
}

// Pool backward, added into dx (which already holds the skip-path gradient): each input element
// receives the pooled gradient if it was its block's maximum.
__global__ void k_pool_bwd(const uint16_t* __restrict__ dy, const uint8_t* __restrict__ arg,
                           int N, int H, int W, int C, uint16_t* __restrict__ dx) {
    const size_t n = (size_t)N * H * W * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t pix = i / C;
        const int xx = (int)(pix % W), yy = (int)((pix / W) % H), bn = (int)(pix / ((size_t)W * H));
        const size_t o = ((size_t)(bn * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + c;
        const int k = (yy & 1) * 2 + (xx & 1);
        if (arg[o] == k) dx[i] = f2bf(bf2f(dx[i]) + bf2f(dy[o]));
    }
}

void launch_pool_bwd(const uint16_t* dy, const uint8_t* arg, int N, int H, int W, int C,
                     uint16_t* dx, hipStream_t st) {
    const size_t n = (size_t)N * H * W * C;
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_pool_bwd, dim3(bl), dim3(256), 0, st, dy, arg, N, H, W, C, dx);
}

// ------------------------------------------------------------------------------------------
// Losses (Eq. (17)-(21)) and their gradients
// ------------------------------------------------------------------------------------------
// Inputs fp32 maps [N][H][W] (depth, logit), [N][H][W][3] (normal) with targets.  One pass
// writes per-pixel gradient numerators and per-block partial sums of the four loss numerators
// and the two valid counts; the normalisations (counts) are applied by k_loss_scale.
__global__ __launch_bounds__(256) void k_loss(LossArgs a) {
    __shared__ float red[6][256];
    const int tid = threadIdx.x;
    const size_t total = (size_t)a.N * a.H * a.W;
    float acc[6] = {0, 0, 0, 0, 0, 0};  // L1num, L2num, L3num, L4num, n_valid, n_valid4
    const size_t i = (size_t)blockIdx.x * 256 + tid;
    if (i < total) {
        const int x = (int)(i % a.W), y = (int)((i / a.W) % a.H);
        const float m = a.mask_gt[i];
        const float d = a.depth[i], dg = a.depth_gt[i];
        // L1
        acc[0] = m * (d - dg) * (d - dg);
        a.gd[i] = m * 2.f * (d - dg);
        acc[4] = m;
        // L2
        const float px = a.nrm[3 * i], py = a.nrm[3 * i + 1], pz = a.nrm[3 * i + 2];
        const float gx = a.nrm_gt[3 * i], gy = a.nrm_gt[3 * i + 1], gz = a.nrm_gt[3 * i + 2];
        const float cx = py * gz - pz * gy, cy = pz * gx - px * gz, cz = px * gy - py * gx;
        const float cn = sqrtf(cx * cx + cy * cy + cz * cz);
        const float pn = sqrtf(px * px + py * py + pz * pz), gn = sqrtf(gx * gx + gy * gy + gz * gz);
        const float den = fmaxf(pn * gn, 1e-12f);
        const float s = cn / den;
        acc[1] = m * s;
        float ux = 0.f, uy = 0.f, uz = 0.f;
        if (cn > 0.f) {
            ux = cx / cn;
            uy = cy / cn;
            uz = cz / cn;
        }
        const float ip2 = pn > 0.f ? 1.f / (pn * pn) : 0.f;
        a.gn[3 * i] = m * ((gy * uz - gz * uy) / den - s * ip2 * px);
        a.gn[3 * i + 1] = m * ((gz * ux - gx * uz) / den - s * ip2 * py);
        a.gn[3 * i + 2] = m * ((gx * uy - gy * ux) / den - s * ip2 * pz);
        // L3 focal (Eq. (19), gamma = 2): h, 1 - h and their logs from the logit itself
        // (log h = -softplus(-l), log(1 - h) = -softplus(l)), exact for saturated logits where
        // 1 - h computed as a difference would round to 0
        const float lg = a.logit[i];
        const float e = expf(-fabsf(lg));                  // in (0, 1]
        const float sp = log1pf(e);                         // softplus(-|l|)
        const float h = lg >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
        const float hb = lg >= 0.f ? e / (1.f + e) : 1.f / (1.f + e);
        const float lh = -(fmaxf(-lg, 0.f) + sp), l1h = -(fmaxf(lg, 0.f) + sp);
        const float al = 0.5f;
        float l3, gl;
        if (m > 0.f) {
            l3 = -al * hb * hb * lh;
            gl = al * hb * hb * (2.f * h * lh - hb);
        } else {
            l3 = -(1.f - al) * h * h * l1h;
            gl = (1.f - al) * h * h * (h - 2.f * hb * l1h);
        }
        acc[2] = l3;
        a.gl[i] = gl;
        // L4 contribution of the quad at (y, x): needs (y, x+1), (y+1, x) hits
        if (x + 1 < a.W && y + 1 < a.H) {
            const float mr = a.mask_gt[i + 1], md = a.mask_gt[i + a.W];
            const float v = m * mr * md;
            acc[5] = v;
            if (v > 0.f) {
                const float du = a.depth[i + 1] - d, dv = a.depth[i + a.W] - d;
                const float du2 = a.depth_gt[i + 1] - dg, dv2 = a.depth_gt[i + a.W] - dg;
                const float P0 = -du, P1 = -dv, P2 = 1.f, G0 = -du2, G1 = -dv2, G2 = 1.f;
                const float c0 = P1 * G2 - P2 * G1, c1 = P2 * G0 - P0 * G2, c2 = P0 * G1 - P1 * G0;
                const float c4 = sqrtf(c0 * c0 + c1 * c1 + c2 * c2);
                const float pp = sqrtf(P0 * P0 + P1 * P1 + P2 * P2), pg = sqrtf(G0 * G0 + G1 * G1 + G2 * G2);
                const float s4 = c4 / (pp * pg);
                acc[3] = s4;
                float u0 = 0.f, u1 = 0.f, u2 = 0.f;
                if (c4 > 0.f) {
                    u0 = c0 / c4;
                    u1 = c1 / c4;
                    u2 = c2 / c4;
                }
                // d s4 / d P (components 0, 1 only; P2 is constant)
                const float w0 = (G1 * u2 - G2 * u1) / (pp * pg) - s4 / (pp * pp) * P0;
                const float w1 = (G2 * u0 - G0 * u2) / (pp * pg) - s4 / (pp * pp) * P1;
                a.w4[2 * i] = w0;
                a.w4[2 * i + 1] = w1;
            } else {
                a.w4[2 * i] = 0.f;
                a.w4[2 * i + 1] = 0.f;
            }
        } else {
            a.w4[2 * i] = 0.f;
            a.w4[2 * i + 1] = 0.f;
        }
    }
    for (int k = 0; k < 6; k++) red[k][tid] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < 6; k++) red[k][tid] += red[k][tid + s];
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < 6; k++) a.partial[blockIdx.x * 6 + k] = red[k][0];
}

void launch_loss(const LossArgs& a, hipStream_t st) {
    const size_t total = (size_t)a.N * a.H * a.W;
    hipLaunchKernelGGL(k_loss, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a);
}

// Sums the loss partials: block k sums component k, thread t over partials t, t + 256, ...,
// then a fixed tree (deterministic).
__global__ __launch_bounds__(256) void k_loss_sum(const float* __restrict__ partial, int nb,
                                                  double* __restrict__ sums) {
    __shared__ double red[256];
    const int k = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int b = tid; b < nb; b += 256) s += partial[b * 6 + k];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) sums[k] = red[0];
}

void launch_loss_sum(const float* partial, int nb, double* sums, hipStream_t st) {
    hipLaunchKernelGGL(k_loss_sum, dim3(6), dim3(256), 0, st, partial, nb, sums);
}

// Final per-pixel gradients with the normalisations and lambdas of Eq. (21); converts the
// L4 quad weights into depth gradients (each quad touches (y,x), (y,x+1), (y+1,x)).
__global__ void k_loss_scale(LossArgs a, const double* __restrict__ sums) {
    const size_t total = (size_t)a.N * a.H * a.W;
    const float nv = (float)fmax(sums[4], 1.0), nv4 = (float)fmax(sums[5], 1.0);
    const float inv_all = 1.f / (float)total;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.W), y = (int)((i / a.W) % a.H);
        float g4 = 0.f;
        // own quad: d P0/d d(y,x) = +1, d P1/d d(y,x) = +1
        g4 += a.w4[2 * i] + a.w4[2 * i + 1];
        if (x > 0) g4 -= a.w4[2 * (i - 1)];            // quad (y, x-1): P0 depends on d(y,x) with -1
        if (y > 0) g4 -= a.w4[2 * (i - a.W) + 1];       // quad (y-1, x): P1 depends on d(y,x) with -1
        a.out_gd[i] = 1.0f * a.gd[i] / nv + 0.5f * g4 / nv4;
        for (int c = 0; c < 3; c++) a.out_gn[3 * i + c] = 0.5f * a.gn[3 * i + c] / nv;
        a.out_gl[i] = 1.0f * a.gl[i] * inv_all;
    }
}

void launch_loss_scale(const LossArgs& a, const double* sums, hipStream_t st) {
    const size_t total = (size_t)a.N * a.H * a.W;
    int bl = (int)((total + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_loss_scale, dim3(bl), dim3(256), 0, st, a, sums);
}

// Gathers an fp32 head gradient map into the bf16 gradient of the head's last convolution
// output before the pixel shuffle (un-shuffle + cast): d[n][y][x][c*4+2sy+sx].
__global__ void k_head_grad(const float* __restrict__ g, int N, int H, int W, int C,
                            float scale, uint16_t* __restrict__ d, int ldd) {
    const size_t n = (size_t)N * H * W * 4 * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % (4 * C));
        const size_t pix = i / (4 * C);
        const int x = (int)(pix % W), y = (int)((pix / W) % H), b = (int)(pix / ((size_t)W * H));
        const int c = k >> 2, sy = (k >> 1) & 1, sx = k & 1;
        d[pix * ldd + k] =
            f2bf(scale * g[((size_t)(b * 2 * H + 2 * y + sy) * (2 * W) + 2 * x + sx) * C + c]);
    }
}

void launch_head_grad(const float* g, int N, int H, int W, int C, float scale, uint16_t* d,
                      int ldd, hipStream_t st) {
    const size_t n = (size_t)N * H * W * 4 * C;
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_head_grad, dim3(bl), dim3(256), 0, st, g, N, H, W, C, scale, d, ldd);
}

// AdamW on fp32 masters; refreshes the bf16 copy (the conv weights) where bf != null.
__global__ void k_adamw(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, uint16_t* __restrict__ bf, size_t n, float lr,
                        float wd, float b1, float b2, float c1, float c2, float eps) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
        p[i] = pi;
        if (bf) bf[i] = f2bf(pi);
    }
}

void launch_adamw(float* p, const float* g, float* m, float* v, uint16_t* bf, size_t n, float lr,
                  float wd, int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_adamw, dim3(bl > 0 ? bl : 1), dim3(256), 0, st, p, g, m, v, bf, n, lr, wd,
                       b1, b2, c1, c2, 1e-8f);
}

// Depth output = head value + coarse depth 1 - x of the input pixel containing the output
// pixel (0 where the input is empty).
__global__ void k_depth_base(float* __restrict__ out, const float* __restrict__ x, int N, int H,
                             int W, float scale) {
    const size_t n = (size_t)N * 4 * H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int X = (int)(i % (2 * W)), Y = (int)((i / (2 * W)) % (2 * H));
        const int b = (int)(i / ((size_t)4 * H * W));
        const float v = x[((size_t)b * H + Y / 2) * W + X / 2];
        out[i] = out[i] * scale + (v > 0.f ? 1.f - v : 0.f);
    }
}

void launch_depth_base(float* out, const float* x, int N, int H, int W, hipStream_t st) {
    const size_t n = (size_t)N * 4 * H * W;
    int b = (int)((n + 255) / 256);
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_depth_base, dim3(b), dim3(256), 0, st, out, x, N, H, W,
                       1.f / (float)(H > W ? H : W));
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, size_t n, uint16_t* __restrict__ b) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

void launch_f32_to_bf16(const float* a, size_t n, uint16_t* b, hipStream_t st) {
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(bl > 0 ? bl : 1), dim3(256), 0, st, a, n, b);
}

__global__ void k_bf16_to_f32(const uint16_t* __restrict__ a, size_t n, float* __restrict__ b) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = bf2f(a[i]);
}

void launch_bf16_to_f32(const uint16_t* a, size_t n, float* b, hipStream_t st) {
    int bl = (int)((n + 255) / 256);
    if (bl > 8192) bl = 8192;
    hipLaunchKernelGGL(k_bf16_to_f32, dim3(bl > 0 ? bl : 1), dim3(256), 0, st, a, n, b);
}

}  // namespace pe
