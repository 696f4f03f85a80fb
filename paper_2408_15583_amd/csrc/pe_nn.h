// Kernel arguments and launchers of the learned densifier (Sec. III-A).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

// Convolution, stride 1, zero padding (K-1)/2, NHWC bf16 activations, OHWI bf16 weights.
struct ConvArgs {
    const uint16_t* x;  // input [N][H][W][ldx], channels xoff .. xoff+Cin
    int ldx, xoff;
    int N, H, W, Cin, K;
    const uint16_t* w;  // [Cout][K][K][Cin]
    int Cout;           // GEMM columns (weights beyond Cout read as zero)
    int Cout_store;     // output channels written (<= Cout)
    const float* bias;  // Cout or null
    const uint16_t* res;  // residual added before the activation ([M][ldres]) or null
    int ldres;
    int act;            // 0 = none, 1 = GELU
    int shuffle;        // 1 = pixel shuffle (output at 2H x 2W with Cout/4 channels)
    uint16_t* y;        // bf16 output, or null when y32 is set
    float* y32;         // fp32 output
    int ldy, yoff;
    uint16_t* z;        // pre-activation copy (bf16) or null
};

struct WgradArgs {
    const uint16_t* x;   // forward input [N][H][W][ldx] (+xoff)
    int ldx, xoff;
    const uint16_t* dy;  // output gradient [N][H][W][lddy] (+dyoff); channels Cout..ceil8 zero
    int lddy, dyoff;
    int N, H, W, Cin, Cout, K;
    int chunk;           // pixels per partial
    float* partial;      // [n_chunks][Cout][K*K][Cin]
};

struct LossArgs {
    int N, H, W;
    const float *depth, *nrm, *logit;            // predictions [N][H][W](x3)
    const float *depth_gt, *nrm_gt, *mask_gt;    // targets
    float *gd, *gn, *gl, *w4;                    // per-pixel gradient numerators (scratch)
    float* partial;                              // [blocks][6]
    float *out_gd, *out_gn, *out_gl;             // final gradients
};

void launch_conv_fwd(const ConvArgs& a, hipStream_t st);
// Inference form of a ConvNeXt block's two 1 x 1 convolutions fused (expand x4 with GELU, then
// project with the residual): a holds the projecting convolution with a.x the block's
// normalised input and a.Cin the hidden width (4 x a.Cout); w1, b1 the expanding one.  Returns
// false (nothing launched) for shapes it does not take.
bool launch_mlp_fwd(const ConvArgs& a, const uint16_t* w1, const float* b1, hipStream_t st);
void launch_conv_wgrad(const WgradArgs& a, int n_chunks, hipStream_t st);
void launch_reduce_chunks(const float* part, int n_chunks, size_t stride, size_t n, int inner,
                          int outer, int off, float* out, hipStream_t st);
void launch_colsum(const uint16_t* y, int M, int ld, int off, int C, int chunk, float* part,
                   hipStream_t st);
void launch_weight_flip(const uint16_t* w, int Cout, int taps, int Cin, int co_pad, uint16_t* wt,
                        hipStream_t st);
void launch_unshuffle(const uint16_t* g, int N, int H, int W, int C, int ldg, int goff,
                      uint16_t* d, int ldd, hipStream_t st);
void launch_gelu_bwd(const uint16_t* z, const uint16_t* dy, size_t n, uint16_t* dz,
                     hipStream_t st);
void launch_add(const uint16_t* a, int lda, int aoff, const uint16_t* b, int ldb, int boff, int M,
                int C, uint16_t* y, int ldy, int yoff, hipStream_t st);
void launch_copy_slice(const uint16_t* a, int lda, int aoff, int M, int C, uint16_t* y, int ldy,
                       int yoff, hipStream_t st);
void launch_stem_fwd(const float* x, int N, int H, int W, int C, const float* w, const float* b,
                     uint16_t* z, uint16_t* a, hipStream_t st);
void launch_stem_wgrad(const float* x, int N, int H, int W, int C, const uint16_t* dz, int chunk,
                       float* part, hipStream_t st);
// Depthwise 7x7 over 8-channel groups (C % 8 == 0) with tap-major weights wt[49][C].
void launch_dw_wt(const float* w, int C, float* wt, hipStream_t st);
void launch_dw_fwd(const uint16_t* x, int N, int H, int W, int C, const float* wt, const float* b,
                   uint16_t* y, hipStream_t st);
void launch_dw_dgrad(const uint16_t* dy, int N, int H, int W, int C, const float* wt, uint16_t* dx,
                     hipStream_t st);
void launch_dw_wgrad(const uint16_t* x, const uint16_t* dy, int N, int H, int W, int C, int rows,
                     float* part, hipStream_t st);
// Depthwise weight/bias gradient partials [chunks][C][49 taps + bias] with the fastest kernel
// for the shape; dw_wgrad_chunks gives the number of chunks it writes.
constexpr int kDwSeg = 64;  // pixels of a row per partial in the sliding-window kernel
int dw_wgrad_chunks(int N, int H, int W, int C);
void launch_dw_wgrad_auto(const uint16_t* x, const uint16_t* dy, int N, int H, int W, int C,
                          float* part, hipStream_t st);
void launch_ln_fwd(const uint16_t* x, int M, int C, const float* g, const float* b, float eps,
                   uint16_t* y, float* stats, hipStream_t st);
void launch_ln_bwd(const uint16_t* x, const uint16_t* dy, int M, int C, const float* g,
                   const float* stats, uint16_t* dx, hipStream_t st);
void launch_ln_pgrad(const uint16_t* x, const uint16_t* dy, int M, int C, const float* stats,
                     int chunk, float* part, hipStream_t st);
void launch_pool_fwd(const uint16_t* x, int N, int H, int W, int C, uint16_t* y, uint8_t* arg,
                     hipStream_t st);
void launch_pool_bwd(const uint16_t* dy, const uint8_t* arg, int N, int H, int W, int C,
                     uint16_t* dx, hipStream_t st);
void launch_loss(const LossArgs& a, hipStream_t st);
void launch_loss_sum(const float* partial, int nb, double* sums, hipStream_t st);
void launch_loss_scale(const LossArgs& a, const double* sums, hipStream_t st);
// Output-map gradient of one head into its last convolution's (unshuffled) layout, times scale.
void launch_head_grad(const float* g, int N, int H, int W, int C, float scale, uint16_t* d,
                      int ldd, hipStream_t st);
void launch_adamw(float* p, const float* g, float* m, float* v, uint16_t* bf, size_t n, float lr,
                  float wd, int step, hipStream_t st);
// Depth output = head / max(H, W) + coarse depth (1 - x where x > 0, else 0), in place: one
// unit of the head is one coarse pixel pitch of depth (t/D).
void launch_depth_base(float* out, const float* x, int N, int H, int W, hipStream_t st);
void launch_f32_to_bf16(const float* a, size_t n, uint16_t* b, hipStream_t st);
void launch_bf16_to_f32(const uint16_t* a, size_t n, float* b, hipStream_t st);

}  // namespace pe
