// Fused BC1 + MLP decode on the CDNA4 matrix cores (FP16 or E4M3 operands,
// FP32 accumulation).
//
// The paper evaluates the MLP per 8x4 pixel tile on the matrix engines of its
// GPUs through cooperative vectors, with all threads of a workgroup sharing
// one weight matrix (Sec. 4). Here one wavefront owns a 64-pixel tile and
// every layer is a [out x in] x [in x 64 px] product of 16x16x32 MFMA tiles:
//
//   * Weights are the A operand (16 output rows per M-tile, 32 inputs per
//     K-chunk) and stay in VGPRs for the whole persistent wave.
//   * Pixels are the B operand, 16 per N-tile (4 N-tiles per tile). Lane
//     l = 16 g + n holds 8 K-elements of pixel n; for the first layer lane
//     group g samples latent level g, so the four BC1 levels are decoded in
//     parallel by the four lane groups.
//   * The accumulator of a 16x16 tile leaves lane 16 g + n with rows
//     4g .. 4g+3 of pixel n. Two consecutive M-tiles therefore give exactly
//     the 8 K-elements that lane needs as B operand of the next layer, once
//     the next layer's weight columns are permuted accordingly at pack
//     time. Layers chain in registers; only ReLU and the conversion run in
//     between. Biases enter as the accumulator's initial value.
//   * Before the MLP, the wave computes the texel bounding box of its tile on
//     every level, decodes each texel of the boxes once (integer BC1
//     decode) into its own LDS region, and the bilinear taps then read the
//     packed texel words from LDS. A tile whose boxes do not fit falls back
//     to fetching its blocks directly.
#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"
#include "ntc_mfma_tile.hpp"

namespace ntc {

template <class P, int HID, int NL, int TP>
__global__ __launch_bounds__(64) void decode_mfma_kernel(DecodeArgs a) {
  extern __shared__ f32x4 stage[];
  const int lane = threadIdx.x;
  const int g = lane >> 4;

  MfmaWeights<P, HID, NL> W;
  W.load(a.packed, a.lay, lane);
  const __amdgpu_buffer_rsrc_t wrs = make_rsrc(a.packed, (uint32_t)a.lay.total);
  const bool has_level = g < a.lat.n_levels;
  const LaneLevel L = lane_level(a.lat, g);

  // XCD-aware numbering: consecutive workgroups land on different XCDs;
  // renumber so that each XCD walks a contiguous range of tiles at a time.
  const int nb = gridDim.x;
  int vb = blockIdx.x;
  if ((nb & 7) == 0) vb = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int64_t n_iter = (a.n_tiles + TP - 1) / TP;
  for (int64_t it = vb; it < n_iter; it += nb)
    decode_tiles<P, HID, NL, TP>(a, L, has_level, it * TP, a.n, stage, W, wrs);
}

template <class P, int HID, int TP>
static hipError_t launch_mfma_tp(const DecodeArgs &a, int n_layers, int grid, hipStream_t st) {
  const size_t lds = (size_t)a.stage_cap * sizeof(f32x4);
  switch (n_layers) {
    case 2: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 2, TP>), dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 3, TP>), dim3(grid), dim3(64), lds, st, a); break;
    case 4: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 4, TP>), dim3(grid), dim3(64), lds, st, a); break;
    case 5: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 5, TP>), dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class P, int HID>
static hipError_t launch_mfma_hid(const DecodeArgs &a, int n_layers, int tp, int grid, hipStream_t st) {
  return tp == 2 ? launch_mfma_tp<P, HID, 2>(a, n_layers, grid, st) : launch_mfma_tp<P, HID, 1>(a, n_layers, grid, st);
}

template <class P>
static hipError_t launch_mfma_prec(const DecodeArgs &a, const MlpShape &s, int tp, int grid, hipStream_t st) {
  switch (s.hid) {
    case 16: return launch_mfma_hid<P, 16>(a, s.n_layers, tp, grid, st);
    case 32: return launch_mfma_hid<P, 32>(a, s.n_layers, tp, grid, st);
    case 64: return launch_mfma_hid<P, 64>(a, s.n_layers, tp, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decode_mfma(const DecodeArgs &a, const MlpShape &s, int compute, int tiles_per_iter,
                              int grid_waves, hipStream_t st) {
  const int tp = tiles_per_iter == 2 ? 2 : 1;
  int64_t grid = grid_waves;
  const int64_t n_iter = (a.n_tiles + tp - 1) / tp;
  if (grid > n_iter) grid = n_iter;
  if (grid >= 8) grid &= ~(int64_t)7;
  if (grid < 1) grid = 1;
  if (compute == 1) return launch_mfma_prec<PrecF16>(a, s, tp, (int)grid, st);
  if (compute == 3) return launch_mfma_prec<PrecF8>(a, s, tp, (int)grid, st);
  return hipErrorInvalidValue;
}

}  // namespace ntc
