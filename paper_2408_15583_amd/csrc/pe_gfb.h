// Launchers of the GFB kernels (network data encoding and GFB-sourced primary rays).
#pragma once

#include "pe_device.h"

namespace pe {

void launch_coarse_encode(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                          float* out, hipStream_t st);
void launch_target_encode(const SlotDesc* d, int n_slots, int max_pix, const uint64_t* keys,
                          float* depth, float* nrm, float* mask, hipStream_t st);
void launch_depth_normals(const float* depth, const float* hit, int W, int H, int n_img,
                          float scale, float* nrm, hipStream_t st);
void launch_gfb_uncertain(const SlotDesc* d, int n_slots, int max_pix, const float* prob, float lo,
                          float hi, uint32_t* counts, hipStream_t st);
void launch_gfb_raygen(const SlotDesc* d, int n_slots, int max_pix, const float* depth,
                       const float* nrm, const float* prob, const uint8_t* use, float thresh,
                       uint32_t* wg_count, uint32_t* wg_off, uint32_t* list, RayState rs,
                       uint64_t* hitkey, uint32_t* n_out, uint32_t* scan_ws, hipStream_t st);
// Algorithm 1 with a K-point heap over TUBE slots (binned like the TUBE raster); keys hold the
// Euclidean depth |p - o| of the chosen point.
void launch_raster_topk(const SlotDesc* d, int n_slots, int max_tiles, const uint32_t* tile_off,
                        const uint32_t* tile_count, const uint32_t* list, uint32_t capacity, int K,
                        uint64_t* keys, hipStream_t st);
void launch_head_post(const float* logit, const float* nrm_raw, size_t n, float* prob, float* nrm,
                      hipStream_t st);

}  // namespace pe
