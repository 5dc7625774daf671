// Fused BC1 + MLP decode on the CDNA4 matrix cores (FP16 or E4M3 operands,
// FP32 accumulation), one persistent wavefront per workgroup.
//
// The paper evaluates the MLP per 8x4 pixel tile on the matrix engines of its
// GPUs through cooperative vectors, with all threads of a workgroup sharing
// one weight matrix (Sec. 4). Here a wavefront keeps the whole MLP in
// registers and walks spans of 256 or 512 pixels; every layer is a product of
// 32x32 tiles (v_mfma_f32_32x32x16_f16, or the 32x32x64 E4M3 form), the
// full-rate matrix instructions of gfx950. The tile-level data flow is
// described in ntc_mfma_tile.hpp.
#include <hip/hip_runtime.h>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"
#include "ntc_mfma_tile.hpp"

namespace ntc {

template <class P, int HID, int NL, int VEC4>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NTC_WAVES_PER_SIMD, NTC_WAVES_PER_SIMD))) void decode_mfma_kernel(DecodeArgs a) {
  constexpr int ST = span_tiles_for(HID, NL, P::kF16Tex);
  constexpr int SPX = 64 * ST;
  extern __shared__ f32x4 smem[];
  f32x4 *stage = smem;
  f32x4 *bias = smem + a.stage_cap;
  f32x4 *ltab = bias + BiasLds<HID, NL>::kCount;
  // output staging for widths that are not a multiple of 4 (32 x 16 floats)
  float *obuf = VEC4 ? nullptr : reinterpret_cast<float *>(ltab + LevelTab::kCount);
  const int lane = threadIdx.x;

  MfmaWeights<P, HID, NL> W;
  W.load(a.packed, a.lay, lane);
  BiasLds<HID, NL>::fill(bias, a.packed, a.lay, lane);
  LevelTab::fill(ltab, a.lat, lane);
  W.ready();
  __syncthreads();

  // XCD-aware numbering: consecutive workgroups land on different XCDs;
  // renumber so that each XCD walks a contiguous range of spans at a time.
  const int nb = gridDim.x;
  int vb = blockIdx.x;
  if ((nb & 7) == 0) vb = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int64_t n_spans = (a.n + SPX - 1) / SPX;
  SpanUv<ST> uvs;
  if (vb < n_spans) {
    uvs.load(a.uv, (int64_t)vb * SPX, a.n);
    // completed before the loop, so that the loop is entered with the same
    // pending loads as its back edge has
    uvs.ready();
  }
  for (int64_t it = vb; it < n_spans; it += nb) {
    const int64_t nx = it + nb;
    decode_span<P, HID, NL, ST, VEC4>(a, it * SPX, a.n, stage, bias, ltab, W, uvs, nx < n_spans ? nx * SPX : -1,
                                      a.n, obuf);
  }
}

template <class P, int HID, int VEC4>
static hipError_t launch_mfma_v(const DecodeArgs &a, int n_layers, int grid, hipStream_t st) {
  const size_t lds =
      (size_t)(a.stage_cap + BiasLds<HID, 5>::kCount + LevelTab::kCount + (VEC4 ? 0 : 32 * 16 / 4)) * sizeof(f32x4);
  switch (n_layers) {
    case 2: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 2, VEC4>), dim3(grid), dim3(64), lds, st, a); break;
    case 3: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 3, VEC4>), dim3(grid), dim3(64), lds, st, a); break;
    case 4: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 4, VEC4>), dim3(grid), dim3(64), lds, st, a); break;
    case 5: hipLaunchKernelGGL((decode_mfma_kernel<P, HID, 5, VEC4>), dim3(grid), dim3(64), lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class P, int HID>
static hipError_t launch_mfma_hid(const DecodeArgs &a, int n_layers, int grid, hipStream_t st) {
  switch (out_class(a.n_out)) {
    case kOut4: return launch_mfma_v<P, HID, kOut4>(a, n_layers, grid, st);
    case kOut4x2: return launch_mfma_v<P, HID, kOut4x2>(a, n_layers, grid, st);
    default: return launch_mfma_v<P, HID, kOutAny>(a, n_layers, grid, st);
  }
}

template <class P>
static hipError_t launch_mfma_prec(const DecodeArgs &a, const MlpShape &s, int grid, hipStream_t st) {
  switch (s.hid) {
    case 16: return launch_mfma_hid<P, 16>(a, s.n_layers, grid, st);
    case 32: return launch_mfma_hid<P, 32>(a, s.n_layers, grid, st);
    case 64: return launch_mfma_hid<P, 64>(a, s.n_layers, grid, st);
    default: return hipErrorInvalidValue;
  }
}

int decode_span_tiles(int hid, int n_layers, int compute) {
  return span_tiles_for(hid, n_layers, compute == 1 ? PrecF16::kF16Tex : (compute == 2 ? PrecBF16::kF16Tex : PrecF8::kF16Tex));
}

hipError_t launch_decode_mfma(const DecodeArgs &a, const MlpShape &s, int compute, int grid_waves, hipStream_t st) {
  int64_t grid = grid_waves;
  const int span = decode_span_tiles(s.hid, s.n_layers, compute);
  const int64_t n_iter = (a.n_tiles + span - 1) / span;
  if (grid > n_iter) grid = n_iter;
  if (grid >= 8) grid &= ~(int64_t)7;
  if (grid < 1) grid = 1;
  if (compute == 1) return launch_mfma_prec<PrecF16>(a, s, (int)grid, st);
  if (compute == 2) return launch_mfma_prec<PrecBF16>(a, s, (int)grid, st);
  if (compute == 3) return launch_mfma_prec<PrecF8>(a, s, (int)grid, st);
  return hipErrorInvalidValue;
}

}  // namespace ntc
