// Filtered decode over mip chains (Sec. 3.2: the mips of a latent texture are
// separate BC1 textures; Sec. 3.3: the latents are fetched with trilinear or
// anisotropic filtering, which the network tolerates without retraining).
//
// One lane per pixel, as in the direct path of the matrix-core decode: each
// lane computes the filtered features of its pixel (level of detail from the
// screen derivatives, bilinear samples of the chosen mips with direct block
// fetches, blended), then a wavefront runs the FP16 MLP of its 64 pixels on
// the matrix cores and stores. The span staging of the unfiltered decode
// does not apply: the footprint now depends on the derivatives.
#include <hip/hip_runtime.h>

#include "ntc_internal.hpp"
#include "ntc_mfma_tile.hpp"

namespace ntc {

namespace {

// Bilinear sample of mip m of level k (clamp to edge), coordinates sanitised
// as in the unfiltered decode.
__device__ __forceinline__ float3 mip_sample(const FilterArgs &f, int k, int m, float u, float v) {
  const MipArgs &M = f.mip[k][m];
  TabLevel L;
  L.fw = (float)M.w;
  L.fh = (float)M.h;
  L.cx = f.sx[k] - 0.5f;
  L.cy = f.sy[k] - 0.5f;
  L.wm2 = (float)(M.w - 2);
  L.hm2 = (float)(M.h - 2);
  L.w = M.w;
  L.h = M.h;
  L.bw = M.bw;
  L.bc1 = M.bc1;
  // FP16 texels and blend, as the unfiltered FP16 decode samples a level (a
  // footprint of one texel gives its result bit for bit)
  const Tex16 c = sample_direct16(L, tap_coord(u), tap_coord(v), 0);
  return make_float3((float)c.rg[0], (float)c.rg[1], (float)c.b1[0]);
}

// Trilinear sample at level of detail lod (already clamped to [0, n_mips - 1]).
__device__ __forceinline__ float3 trilinear(const FilterArgs &f, int k, float lod, float u, float v) {
  const int nm = f.n_mips[k];
  int m0 = (int)floorf(lod);
  m0 = m0 < 0 ? 0 : (m0 > nm - 1 ? nm - 1 : m0);
  const float t = lod - (float)m0;
  float3 c = mip_sample(f, k, m0, u, v);
  if (t > 0.0f && m0 + 1 < nm) {
    const float3 c1 = mip_sample(f, k, m0 + 1, u, v);
    c.x = fmaf(t, c1.x - c.x, c.x);
    c.y = fmaf(t, c1.y - c.y, c.y);
    c.z = fmaf(t, c1.z - c.z, c.z);
  }
  return c;
}

template <int FILTER>
__device__ __forceinline__ float3 filtered_level(const FilterArgs &f, int k, float u, float v, float4 d) {
  const float w0 = f.w0[k], h0 = f.h0[k];
  // squared footprint axes in mip-0 texels, each operation rounded once
  const float ax = __fmul_rn(d.x, w0), bx = __fmul_rn(d.y, h0);
  const float ay = __fmul_rn(d.z, w0), by = __fmul_rn(d.w, h0);
  const float px2 = __fadd_rn(__fmul_rn(ax, ax), __fmul_rn(bx, bx));
  const float py2 = __fadd_rn(__fmul_rn(ay, ay), __fmul_rn(by, by));
  const float top = (float)(f.n_mips[k] - 1);
  if (FILTER == 1) {
    const float lod = fminf(fmaxf(0.5f * __log2f(fmaxf(px2, py2)), 0.0f), top);  // NaN and -inf give 0
    return trilinear(f, k, lod, u, v);
  }
  const float pmax2 = fmaxf(px2, py2), pmin2 = fminf(px2, py2);
  int n = f.max_aniso;
  for (int i = 1; i < f.max_aniso; ++i)
    if (__fmul_rn((float)(i * i), pmin2) >= pmax2) {
      n = i;
      break;
    }
  const float lod = fminf(fmaxf(0.5f * __log2f(pmax2) - __log2f((float)n), 0.0f), top);
  const bool major_x = px2 >= py2;
  const float du = major_x ? d.x : d.z, dv = major_x ? d.y : d.w;
  float3 acc = make_float3(0.f, 0.f, 0.f);
  for (int i = 1; i <= n; ++i) {
    const float t = (float)i / (float)(n + 1) - 0.5f;
    const float3 c = trilinear(f, k, lod, fmaf(t, du, u), fmaf(t, dv, v));
    acc.x += c.x;
    acc.y += c.y;
    acc.z += c.z;
  }
  const float inv = 1.0f / (float)n;
  return make_float3(acc.x * inv, acc.y * inv, acc.z * inv);
}

template <class P, int HID, int NL, int VEC4, int FILTER>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NTC_WAVES_PER_SIMD, NTC_WAVES_PER_SIMD))) void decode_filtered_kernel(FilterArgs f) {
  extern __shared__ f32x4 smem[];
  const DecodeArgs &a = f.d;
  const int lane = threadIdx.x & 63;
  f32x4 *bias = smem;
  MfmaWeights<P, HID, NL> W;
  W.load(a.packed, a.lay, lane);
  BiasLds<HID, NL>::fill(bias, a.packed, a.lay, lane);
  W.ready();
  __syncthreads();
  const int64_t n_sub = (a.n + 63) / 64;
  for (int64_t s = blockIdx.x; s < n_sub; s += gridDim.x) {
    const int64_t first = s * 64;
    const int64_t left = a.n - first;
    const int64_t pix = first + (lane < left ? lane : left - 1);
    const float2 uv = a.uv[pix];
    const float4 d = f.duv[pix];
    float xl[8], xh[8];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      float3 c = make_float3(0.f, 0.f, 0.f);
      if (k < f.n_levels) c = filtered_level<FILTER>(f, k, uv.x, uv.y, d);
      put_level(xl, xh, k, c);
    }
    typename P::Frag bx[2];
    pixel_operands<P>(xl, xh, uv.x, uv.y, W.in_scale, bx);
    const int span = left < 64 ? (int)left : 64;
    subspan_mlp<P, HID, NL, VEC4, false>(a, W, bias, span_out(a, first, span), bx, 0, (int)first);
  }
}

template <int HID, int VEC4, int FILTER>
hipError_t launch_nl(const FilterArgs &f, int n_layers, int grid, hipStream_t st) {
  const size_t lds = (size_t)BiasLds<HID, 5>::kCount * sizeof(f32x4);
  switch (n_layers) {
    case 2: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 2, VEC4, FILTER>), dim3(grid), dim3(64), lds, st, f); break;
    case 3: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 3, VEC4, FILTER>), dim3(grid), dim3(64), lds, st, f); break;
    case 4: hipLaunchKernelGGL((decode_filtered_kernel<PrecF16, HID, 4, VEC4, FILTER>), dim3(grid), dim3(64), lds, st, f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int HID, int VEC4>
hipError_t launch_filter(const FilterArgs &f, int n_layers, int grid, hipStream_t st) {
  return f.filter == 1 ? launch_nl<HID, VEC4, 1>(f, n_layers, grid, st) : launch_nl<HID, VEC4, 2>(f, n_layers, grid, st);
}

template <int HID>
hipError_t launch_vec(const FilterArgs &f, int n_layers, int grid, hipStream_t st) {
  switch (out_class(f.d.n_out)) {
    case kOut4: return launch_filter<HID, kOut4>(f, n_layers, grid, st);
    case kOut4x2: return launch_filter<HID, kOut4x2>(f, n_layers, grid, st);
    default: return launch_filter<HID, kOutAny>(f, n_layers, grid, st);
  }
}

}  // namespace

hipError_t launch_decode_filtered(const FilterArgs &f, const MlpShape &s, int grid_waves, hipStream_t st) {
  int64_t grid = grid_waves;
  const int64_t n_sub = (f.d.n + 63) / 64;
  if (grid > n_sub) grid = n_sub;
  if (grid < 1) grid = 1;
  switch (s.hid) {
    case 16: return launch_vec<16>(f, s.n_layers, (int)grid, st);
    case 32: return launch_vec<32>(f, s.n_layers, (int)grid, st);
    case 64: return launch_vec<64>(f, s.n_layers, (int)grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ntc
