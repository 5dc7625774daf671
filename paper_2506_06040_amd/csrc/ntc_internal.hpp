// Internal interfaces between the C-ABI layer (ntc_api.hip) and the kernel
// translation units. Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ntc_device.hpp"

// FP16 / BF16 images carry the first layer's bias in the weights (two K-slots
// fed with the constant 1, holding the bias split into a high and a low part)
// and the decode adds the output layer's bias inside the sigmoid; 0 keeps
// both biases as accumulator initial values read from LDS.
#ifndef NTC_FOLD_BIAS
#define NTC_FOLD_BIAS 1
#endif

namespace ntc {

// Shape summary of an MLP accepted by the library.
struct MlpShape {
  int32_t n_layers;  // linear layers, 2..kMaxLayers
  int32_t in_dim;    // 3 * n_levels + 2
  int32_t hid;       // common hidden width: 16, 32 or 64
  int32_t n_out;     // 1..16
};

// ---------------------------------------------------------------------------
// Packed weight images (written by the pack kernels, read by the decoders).
//
// FP32 (plain decode): per layer, W padded to [rows_pad][cols_pad] followed
// by b[rows_pad]; layer 0 has cols_pad = 16, the last layer rows_pad = 16.
//
// Matrix-core images (FP16 / FP8): for every layer a run of A-operand
// fragments [m][c][lane][e] (M-tile m of 32 output rows, K-step c of 16
// inputs (FP16, 8 halves per lane) or 64 inputs (E4M3, 32 bytes per lane)),
// then bias fragments [m][lane half][16] floats laid out like the 32x32
// accumulator, then (FP8) three floats per layer: the input scale s_a, the
// epilogue scale and the weight scale s_w. With NTC_FOLD_BIAS, the first
// layer's FP16 / BF16 fragments hold its bias in K-slots 3 and 7 of lane
// half 1 (high part, then the remainder), which the decode feeds with 1.
// ---------------------------------------------------------------------------
struct PackLayout {
  size_t total;
  uint32_t w_off[kMaxLayers];     // bytes
  uint32_t b_off[kMaxLayers];     // bytes
  uint32_t scale_off;             // bytes (FP8 scales; FP16 ReLU-by-clamp flag)
  uint32_t exp_off;               // bytes (FP16: per-neuron scale exponents)
  int32_t mt[kMaxLayers];         // M-tiles (32 rows) per layer
  int32_t kc[kMaxLayers];         // K-steps per layer
  int32_t frag_elems;             // operand elements per lane (8 FP16, 32 E4M3)
  int32_t rows_pad[kMaxLayers];   // FP32 image
  int32_t cols_pad[kMaxLayers];   // FP32 image
  int32_t elem_bytes;             // 4 (FP32), 2 (FP16), 1 (FP8)
};

PackLayout pack_layout(const MlpShape &s, int compute);

struct MlpPtrs {
  const float *W[kMaxLayers];
  const float *b[kMaxLayers];
  int32_t dims[kMaxLayers + 1];
};

hipError_t launch_pack(const MlpShape &s, const MlpPtrs &p, int compute, const float *act_amax,
                       uint8_t *packed, const PackLayout &lay, hipStream_t st);

// Arguments of the decode kernels.
struct DecodeArgs {
  LatArgs lat;
  const uint8_t *packed;
  const float2 *uv;
  void *out;
  int64_t n;
  int64_t n_tiles;      // ceil(n / 64)
  int32_t n_out;
  int32_t out_f16;
  int32_t stage_cap;    // texels per wave in LDS
  int32_t n_layers;
  PackLayout lay;
  const int32_t *pix;   // optional: sample s is pixel pix[s] of the uv / out images
  int64_t img_px;       // pixels of those images
};

hipError_t launch_decode_plain(const DecodeArgs &a, const MlpShape &s, float *calib_amax, int n_cus,
                               hipStream_t st);
hipError_t launch_decode_mfma(const DecodeArgs &a, const MlpShape &s, int compute, int grid_waves, hipStream_t st);
// FP32 decode of float latents on the matrix cores (up to 4 layers).
hipError_t launch_forward_f32(const DecodeArgs &a, const MlpShape &s, hipStream_t st);
int decode_span_tiles(int hid, int n_layers, int compute);  // 64-pixel tiles per span of the matrix-core decode
hipError_t launch_bc1_texels(const LevelArgs &L, float *out, uint16_t *numer, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);

// Backward. Workspace (256-byte aligned sections): per-block FP32 partial
// sums of the weight gradients, the feature gradient dL/dx of every sample,
// and for clamp addressing the spatial bins of the latent-gradient scatter
// (per-bin counts, then start offsets; running cursors; sample indices
// grouped by bin).
struct BwdLayout {
  int32_t n_blocks, n_params, n_feat;
  int32_t bin_tex, bins_x, bins_y, n_bins;  // n_bins = 0: no binning (wrap addressing)
  int32_t bin_lds;                          // LDS floats of one bin's texel windows
  size_t wpart_off, dx_off, count_off, cursor_off, perm_off, total;
};
BwdLayout backward_layout(const MlpShape &s, const LatArgs &lat, int64_t n);

struct BackwardArgs {
  LatArgs lat;
  const float *W[kMaxLayers];
  const float *b[kMaxLayers];
  const float2 *uv;
  const float *grad_out;
  float *grad_lat[kMaxLevels];
  float *wpart;          // [n_blocks][n_params] FP32 per-block partial sums
  float *dx;             // [n][n_feat] dL/d(feature) of every sample
  int32_t *bin_count;    // [n_bins]
  int32_t *bin_cursor;   // [n_bins]
  int32_t *perm;         // [n]
  int64_t n;
  int32_t n_params;
  int32_t n_blocks;
  int32_t n_feat;
  int32_t bin_tex, bins_x, bins_y, n_bins, bin_lds;
  int32_t dims[kMaxLayers + 1];
  int32_t n_layers;
};
hipError_t launch_backward(const BackwardArgs &a, const MlpShape &s, float *const *grad_W,
                           float *const *grad_b, hipStream_t st);

// Many materials in one launch.
struct BatchMaterial {
  DecodeArgs a;       // decode arguments of the material (FP16 image)
  int32_t shape_id;   // 3 * log2(hid / 16) + (n_layers - 2)
  int32_t hid;
  int32_t n_layers;
  int32_t pad_;
};

struct BatchItem {
  int32_t mat;
  int32_t shape_id;
  int64_t first_tile;
  int64_t n_tiles;
};

struct BatchPlanHeader {
  uint32_t magic;
  uint32_t version;
  int32_t n_mats;
  int32_t n_items;
  int32_t n_waves;
  int32_t stage_cap;
  uint64_t mats_off;        // bytes from plan start
  uint64_t items_off;
  uint64_t wave_start_off;  // int32 [n_waves + 1]: items of wave w are [start[w], start[w+1])
  uint64_t total_bytes;
};

constexpr uint32_t kPlanMagic = 0x4E544350u;  // "NTCP"
constexpr uint32_t kPlanVersion = 1;

hipError_t launch_decode_batched(const uint8_t *plan_dev, const BatchPlanHeader &h, hipStream_t st);
int shape_id_of(int hid, int n_layers);
size_t plan_bytes(int n_mats, int64_t n_items, int n_waves);
int64_t count_items(const int64_t *n_px, int n_mats, int item_tiles);
int plan_waves(int64_t n_items, int n_cus, int waves_per_cu);
void build_plan(const BatchMaterial *mats, int n_mats, int item_tiles, int n_waves, int stage_cap, uint8_t *out,
                size_t bytes);

// Trainable BC1 levels (ntc_qat.hip): FP32 logits of the rounding
// midpoints (k + 1/2) / M of the 5-, 6- and 2-bit fields.
struct QatTables {
  float mid5[31];
  float mid6[63];
  float mid2[3];
};
QatTables qat_tables();
hipError_t launch_qat_texels(const float *params, int w, int h, float *texels, hipStream_t st);
hipError_t launch_qat_backward(const float *params, int w, int h, const float *grad_texels, float *grad_params,
                               hipStream_t st);
hipError_t launch_qat_export(const float *params, int w, int h, uint64_t *blocks, hipStream_t st);

// Frame classification (ntc_classify.hip).
int classify_chunks(int w, int h);
size_t classify_workspace_bytes(int w, int h, int n_mats);
hipError_t launch_classify(const uint16_t *mat, int w, int h, int n_mats, int32_t *list, int32_t *mat_offsets,
                           int32_t *mat_simple, uint8_t *tile_class, void *workspace, hipStream_t st);
size_t classify_scratch_bytes();       // capacity of the allocation-free variant's scratch
hipError_t classify_scratch(void **ptr);  // this device's scratch address
hipError_t launch_gather_uv(const float *uv_image, const int32_t *list, int64_t n, float *uv, hipStream_t st);
hipError_t launch_scatter_rows(const void *rows, const int32_t *list, int64_t n, int c, int elem_bytes, void *image,
                               hipStream_t st);

// Filtered decode over mip chains (ntc_filtered.hip).
constexpr int kMaxMips = 12;
constexpr int kMaxAniso = 16;
struct MipArgs {
  const uint2 *bc1;
  int32_t w, h, bw;
  float fw, fh;  // w and h as floats
  int32_t pad_;
};
struct FilterArgs {
  DecodeArgs d;            // packed image, uv, out, n, shapes (d.lat is unused)
  const float4 *duv;       // [n]: du/dx, dv/dx, du/dy, dv/dy
  MipArgs mip[kMaxLevels][kMaxMips];
  int32_t n_mips[kMaxLevels];
  float w0[kMaxLevels], h0[kMaxLevels];  // mip 0 sizes
  float sx[kMaxLevels], sy[kMaxLevels];  // shifts in texels of each mip
  // shared_lod: every level's mip 0 is level 0's mip 0 scaled by 2^-e_k on
  // both axes (lod_shift[k] = e_k), so its squared footprint axes are level
  // 0's times 4^-e_k exactly and its level of detail is level 0's minus e_k
  float lod_shift[kMaxLevels];
  int32_t shift_i[kMaxLevels];  // lod_shift as integers
  int32_t shared_lod;
  int32_t n_levels, filter, max_aniso;
};
hipError_t launch_decode_filtered(const FilterArgs &f, const MlpShape &s, int grid_waves, hipStream_t st);

}  // namespace ntc
