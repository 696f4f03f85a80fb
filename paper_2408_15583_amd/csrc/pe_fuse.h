// GFB edge filtering and grid fusion into splats (Sec. III-B, Algorithm 3, Eq. (22)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

constexpr int kFuseMaxViews = 64;  // contributing views are kept as a 64-bit mask per cell
constexpr int kFuseWords = 8;      // per cell: 3 position sums, 3 normal sums, count, view mask

struct FuseArgs {
    int n_views, w, h;        // square buffers (w == h), pitch 2R / w
    const float* depth;       // n x h x w, t / D (D = 2R)
    const float* nrm;         // n x h x w x 3, view frame (u, v, -k)
    const float* hit;         // n x h x w, hit where >= 0.5
    const float* basis;       // n x 9: u, v, k of each view (device)
    float R;                  // screens of side 2R about the frame centre
    float g[3];               // 5-tap Gaussian (centre, +-1, +-2), normalised
    float thr2_lo, thr2_hi;   // squared thresholds on the Sobel sums (m^2)
    float tan22;              // tan(22.5 deg), sector boundary of the gradient direction
    int dilate;               // pixels within this Chebyshev distance of an edge are dropped
    float half;               // grid: cube of side 2 half about the centre
    float L;                  // grid cell edge = 2 half / G
    int G;                    // grid cells per axis
    double qpos;              // fixed-point quantum of fused positions (m)
    double c[3];              // frame centre (world, m)
};

void launch_fuse_blur(const FuseArgs& a, float* blur, hipStream_t st);
void launch_fuse_classify(const FuseArgs& a, const float* blur, uint8_t* cls, hipStream_t st);
void launch_fuse_hysteresis(const FuseArgs& a, uint8_t* cls, uint32_t* changed, hipStream_t st);
void launch_fuse_drop(const FuseArgs& a, const uint8_t* cls, uint8_t* drop, uint8_t* edge,
                      hipStream_t st);
void launch_fuse_accum(const FuseArgs& a, const uint8_t* drop, unsigned long long* acc,
                       hipStream_t st);
void launch_fuse_flag(const unsigned long long* acc, size_t n_cells, uint32_t* flag,
                      hipStream_t st);
void launch_fuse_emit(const FuseArgs& a, const unsigned long long* acc,
                      const uint32_t* flag, const uint32_t* off, size_t n_cells, double* xyz,
                      float* nrm, float* radius, uint32_t* count, uint64_t cap, hipStream_t st);

}  // namespace pe
