// Filtered decode over mip chains (Sec. 3.2: the mips of a latent texture are
// separate BC1 textures; Sec. 3.3: the latents are fetched with trilinear or
// anisotropic filtering, which the network tolerates without retraining).
//
// One lane per pixel: on every latent level a lane selects its mips and taps
// (level of detail from the screen derivatives; one position for trilinear,
// n positions along the footprint's major axis for anisotropic) and blends
// bilinear samples of those mips; a wavefront then runs the FP16 MLP of its
// 64 pixels on the matrix cores and stores.
//
// Footprint staging. The positions of a span (64 consecutive pixels) on a
// level mostly fall on two consecutive mips, m_lo and m_lo + 1, m_lo the
// span's lowest first mip. For each level and each of those two mips (a
// region), the texels under all the span's positions (a box spanned by the
// extreme coordinates: the tap is monotonic in the coordinate) are decoded
// once into LDS as FP16 texels when they fit; a sample from a staged region
// reads its four texels there instead of fetching and decoding four BC1
// texels. Samples of other mips or of regions that did not fit fetch
// directly. Both ways take the same FP16 texels and the same blend, so a
// result does not depend on the way its samples went.
#include <hip/hip_runtime.h>

#include "ntc_internal.hpp"
#include "ntc_mfma_tile.hpp"

namespace ntc {

namespace {

constexpr int kFiltStageTexels = 2048;  // LDS texels (8 bytes each) per wavefront
constexpr int kRegions = 2 * kMaxLevels;

// Mip m of level k as a sampling table entry (clamp to edge).
__device__ __forceinline__ TabLevel mip_level(const FilterArgs &f, int k, int m) {
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
  return L;
}

__device__ __forceinline__ float3 tex_f3(Tex16 c) {
  return make_float3((float)c.rg[0], (float)c.rg[1], (float)c.b1[0]);
}

// Level-of-detail selection of one pixel on level k: first mip m0, blend
// weight t towards m0 + 1 (0: m0 alone), and for anisotropic filtering the
// tap count n and the major axis (du, dv).
struct LodSel {
  int m0, n;
  float t, du, dv;
};

template <int FILTER>
__device__ __forceinline__ LodSel lod_select(const FilterArgs &f, int k, float4 d) {
  LodSel s;
  const float w0 = f.w0[k], h0 = f.h0[k];
  // squared footprint axes in mip-0 texels, each operation rounded once
  const float ax = __fmul_rn(d.x, w0), bx = __fmul_rn(d.y, h0);
  const float ay = __fmul_rn(d.z, w0), by = __fmul_rn(d.w, h0);
  const float px2 = __fadd_rn(__fmul_rn(ax, ax), __fmul_rn(bx, bx));
  const float py2 = __fadd_rn(__fmul_rn(ay, ay), __fmul_rn(by, by));
  const int nm = f.n_mips[k];
  const float top = (float)(nm - 1);
  float lod;
  if (FILTER == 1) {
    lod = fminf(fmaxf(0.5f * __log2f(fmaxf(px2, py2)), 0.0f), top);  // NaN and -inf give 0
    s.n = 1;
    s.du = 0.0f;
    s.dv = 0.0f;
  } else {
    const float pmax2 = fmaxf(px2, py2), pmin2 = fminf(px2, py2);
    int n = f.max_aniso;
    for (int i = 1; i < f.max_aniso; ++i)
      if (__fmul_rn((float)(i * i), pmin2) >= pmax2) {
        n = i;
        break;
      }
    lod = fminf(fmaxf(0.5f * __log2f(pmax2) - __log2f((float)n), 0.0f), top);
    const bool major_x = px2 >= py2;
    s.n = n;
    s.du = major_x ? d.x : d.z;
    s.dv = major_x ? d.y : d.w;
  }
  int m0 = (int)floorf(lod);
  m0 = m0 < 0 ? 0 : (m0 > nm - 1 ? nm - 1 : m0);
  const float t = lod - (float)m0;
  s.m0 = m0;
  s.t = (t > 0.0f && m0 + 1 < nm) ? t : 0.0f;
  return s;
}

// Offset of anisotropic tap i (1..n) along the major axis, in units of it.
__device__ __forceinline__ float aniso_offset(int i, int n) { return (float)i / (float)(n + 1) - 0.5f; }

// Filtered features of one level; smp(m, x, y) is the bilinear sample of mip
// m at (x, y) as float3.
template <int FILTER, class SMP>
__device__ __forceinline__ float3 filter_level(const LodSel &s, float u, float v, SMP &&smp) {
  auto tri = [&](float x, float y) {
    float3 c = smp(s.m0, x, y);
    if (s.t > 0.0f) {
      const float3 c1 = smp(s.m0 + 1, x, y);
      c.x = fmaf(s.t, c1.x - c.x, c.x);
      c.y = fmaf(s.t, c1.y - c.y, c.y);
      c.z = fmaf(s.t, c1.z - c.z, c.z);
    }
    return c;
  };
  if (FILTER == 1) return tri(u, v);
  float3 acc = make_float3(0.f, 0.f, 0.f);
  for (int i = 1; i <= s.n; ++i) {
    const float t = aniso_offset(i, s.n);
    const float3 c = tri(fmaf(t, s.du, u), fmaf(t, s.dv, v));
    acc.x += c.x;
    acc.y += c.y;
    acc.z += c.z;
  }
  const float inv = 1.0f / (float)s.n;
  return make_float3(acc.x * inv, acc.y * inv, acc.z * inv);
}

// Staged regions of one span: region r = 2 k + j is mip m_lo[k] + j of level
// k; bit r of `staged` is set when its texels are in LDS, texel (i, j) at
// kbase[r] + j kbw[r] + i.
struct FiltStage {
  int m_lo[kMaxLevels];
  unsigned staged;
  int kbw[kRegions], kbase[kRegions];
};

__device__ __forceinline__ int wave_min_i(int v) {
  const int r = row_min_i(v);
  const int a = __builtin_amdgcn_readlane(r, 0), b = __builtin_amdgcn_readlane(r, 16);
  const int c = __builtin_amdgcn_readlane(r, 32), d = __builtin_amdgcn_readlane(r, 48);
  return min(min(a, b), min(c, d));
}

// Footprints of the span and their staging. sel: this lane's selections,
// (u, v) its pixel; stage: kFiltStageTexels texels; srec: 2 kRegions
// records. Regions are taken in order while they fit.
template <int FILTER>
__device__ __forceinline__ FiltStage stage_footprints(const FilterArgs &f, const LodSel (&sel)[kMaxLevels], float u,
                                                      float v, uint2 *stage, f32x4 *srec, int salt) {
  const int lane = threadIdx.x & 63;
  FiltStage st;
  // extreme coordinates of every position of every used level of this pixel
  float umin = tap_coord(u), umax = umin, vmin = tap_coord(v), vmax = vmin;
  if (FILTER != 1) {
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      if (k >= f.n_levels) break;
      const LodSel &s = sel[k];
      const float ta = aniso_offset(1, s.n), tb = aniso_offset(s.n, s.n);
      const float xa = tap_coord(fmaf(ta, s.du, u)), xb = tap_coord(fmaf(tb, s.du, u));
      const float ya = tap_coord(fmaf(ta, s.dv, v)), yb = tap_coord(fmaf(tb, s.dv, v));
      umin = fminf(umin, fminf(xa, xb));
      umax = fmaxf(umax, fmaxf(xa, xb));
      vmin = fminf(vmin, fminf(ya, yb));
      vmax = fmaxf(vmax, fmaxf(ya, yb));
    }
  }
  umin = wave_min_key(umin);
  umax = wave_max_key(umax);
  vmin = wave_min_key(vmin);
  vmax = wave_max_key(vmax);
#pragma unroll
  for (int k = 0; k < kMaxLevels; ++k) st.m_lo[k] = k < f.n_levels ? wave_min_i(sel[k].m0) : 0;
  // lane 4 r + q (r < kRegions): tap index of an extreme coordinate on
  // region r; q = 0: left tap of umin, 1: left tap of umax, 2: top tap of
  // vmin, 3: top tap of vmax
  const int r = (lane >> 2) & (kRegions - 1), q = lane & 3, k = r >> 1;
  const int mlo = k == 0 ? st.m_lo[0] : (k == 1 ? st.m_lo[1] : (k == 2 ? st.m_lo[2] : st.m_lo[3]));
  const int m = mlo + (r & 1);
  const bool valid = lane < 4 * kRegions && k < f.n_levels && m < f.n_mips[k];
  const MipArgs &M = f.mip[k][valid ? m : 0];
  const bool ay = q >= 2;
  const float dim = ay ? (float)M.h : (float)M.w;
  const float ext = q == 0 ? umin : (q == 1 ? umax : (q == 2 ? vmin : vmax));
  const int ti = (int)tap_floor(ext, dim, (ay ? f.sy[k] : f.sx[k]) - 0.5f, dim - 2.0f);
  // every lane of quad r receives the four values of region r
  const int qbx = __builtin_amdgcn_mov_dpp(ti, 0x00, 0xF, 0xF, false);
  const int qex = __builtin_amdgcn_mov_dpp(ti, 0x55, 0xF, 0xF, false);
  const int qby = __builtin_amdgcn_mov_dpp(ti, 0xAA, 0xF, 0xF, false);
  const int qey = __builtin_amdgcn_mov_dpp(ti, 0xFF, 0xF, 0xF, false);
  // the whole blocks spanning texel columns [bx, ex + 1] on texel rows
  // [by, ey + 1]; a staging item is one texel row of one block (4 texels)
  const int qcol0 = qbx >> 2;
  const int qncol = ((qex + 1) >> 2) - qcol0 + 1;
  const int qitems = valid ? __mul24(qncol, qey - qby + 2) : 0;
  int kib[kRegions], total = 0;
  st.staged = 0u;
#pragma unroll
  for (int rr = 0; rr < kRegions; ++rr) {
    const int items = __builtin_amdgcn_readlane(qitems, 4 * rr);
    kib[rr] = total;
    st.kbw[rr] = 4 * __builtin_amdgcn_readlane(qncol, 4 * rr);
    st.kbase[rr] = 4 * total - __builtin_amdgcn_readlane(qby, 4 * rr) * st.kbw[rr] -
                   4 * __builtin_amdgcn_readlane(qcol0, 4 * rr);
    if (items > 0 && 4 * (total + items) <= kFiltStageTexels) {
      st.staged |= 1u << rr;
      total += items;
    }
  }
  // records of the staged regions, by the lead lane of each quad: {first
  // item, blocks per staged row, 1 / that, first block column} and {first
  // texel row, blocks per mip row, block pointer}
  srec += opaque_zero(salt);
  if (q == 0 && lane < 4 * kRegions && ((st.staged >> r) & 1u)) {
    int ib = kib[0];
#pragma unroll
    for (int rr = 1; rr < kRegions; ++rr) ib = r == rr ? kib[rr] : ib;
    const unsigned long long bp = (unsigned long long)M.bc1;
    srec[2 * r] = (f32x4){__int_as_float(ib), __int_as_float(qncol), __builtin_amdgcn_rcpf((float)qncol),
                          __int_as_float(qcol0)};
    srec[2 * r + 1] = (f32x4){__int_as_float(qby), __int_as_float(M.bw), __uint_as_float((unsigned)bp),
                              __uint_as_float((unsigned)(bp >> 32))};
  }
  // item t of the staged regions: region = the last staged region whose
  // first item is at most t (regions left out hold no items); its row inside
  // the region is (t - first + 1/2) / ncol rounded down, exact as in the
  // unfiltered staging (t < 2^10)
  for (int t = lane; t < total; t += 64) {
    int rg = -1;
#pragma unroll
    for (int rr = 0; rr < kRegions; ++rr)
      if (((st.staged >> rr) & 1u) && t >= kib[rr]) rg = rr;
    const f32x4 r0 = srec[2 * rg], r1 = srec[2 * rg + 1];
    const int tl = t - __float_as_int(r0[0]);
    const int ncol = __float_as_int(r0[1]);
    const int row = (int)(((float)tl + 0.5f) * r0[2]);
    const int col = tl - __mul24(row, ncol);
    const int Y = __float_as_int(r1[0]) + row;
    const uint2 *blk = (const uint2 *)(((unsigned long long)__float_as_uint(r1[3]) << 32) | __float_as_uint(r1[2]));
    // rows and blocks of the region lie inside the mip
    const uint2 b = gload2u(blk + (__mul24(Y >> 2, __float_as_int(r1[1])) + __float_as_int(r0[3]) + col));
    const uint32_t pos = (uint32_t)(Y & 3) << 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) stage[4 * t + i] = tex16_bits(tex16_of(texel_f32(bc1_numer(b.x, b.y, pos + i))));
  }
  return st;
}

// Bilinear sample of a staged region: the taps of clamp_tap, four texels
// from LDS, the FP16 blend (the same values sample_direct16 computes).
__device__ __forceinline__ Tex16 staged_sample(const uint2 *stage, float fw, float fh, float cx, float cy,
                                               int kbw, int kbase, float x, float y) {
  int i0, j0;
  float fx, fy;
  clamp_tap(tap_coord(x), fw, cx, fw - 2.0f, i0, fx);
  clamp_tap(tap_coord(y), fh, cy, fh - 2.0f, j0, fy);
  const uint2 *t = stage + kbase + __mul24(j0, kbw) + i0;
  return lerp_tex16(tex16_from(t[0]), tex16_from(t[1]), tex16_from(t[kbw]), tex16_from(t[kbw + 1]), fx, fy);
}

template <class P, int HID, int NL, int VEC4, int FILTER>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NTC_WAVES_PER_SIMD, NTC_WAVES_PER_SIMD))) void decode_filtered_kernel(FilterArgs f) {
  extern __shared__ f32x4 smem[];
  const DecodeArgs &a = f.d;
  const int lane = threadIdx.x & 63;
  f32x4 *bias = smem;
  f32x4 *srec = bias + BiasLds<HID, NL>::kCount;
  uint2 *stage = reinterpret_cast<uint2 *>(srec + 2 * kRegions);
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
    LodSel sel[kMaxLevels];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) sel[k] = lod_select<FILTER>(f, k < f.n_levels ? k : 0, d);
    const FiltStage st = stage_footprints<FILTER>(f, sel, uv.x, uv.y, stage, srec, (int)s);
    float xl[8], xh[8];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
      float3 c = make_float3(0.f, 0.f, 0.f);
      if (k < f.n_levels) {
        // this level's two staged regions, as uniform values
        const bool s0 = (st.staged >> (2 * k)) & 1u, s1 = (st.staged >> (2 * k + 1)) & 1u;
        const int mlo = st.m_lo[k];
        const float cx = f.sx[k] - 0.5f, cy = f.sy[k] - 0.5f;
        const MipArgs &M0 = f.mip[k][mlo];
        const MipArgs &M1 = f.mip[k][mlo + 1 < kMaxMips ? mlo + 1 : mlo];
        const float w0 = (float)M0.w, h0 = (float)M0.h, w1 = (float)M1.w, h1 = (float)M1.h;
        auto smp = [&](int m, float x, float y) -> float3 {
          const int j = m - mlo;
          if ((j == 0 && s0) || (j == 1 && s1)) {
            const bool one = j == 1;
            return tex_f3(staged_sample(stage, one ? w1 : w0, one ? h1 : h0, cx, cy, one ? st.kbw[2 * k + 1] : st.kbw[2 * k],
                                        one ? st.kbase[2 * k + 1] : st.kbase[2 * k], x, y));
          }
          return tex_f3(sample_direct16(mip_level(f, k, m), tap_coord(x), tap_coord(y), 0));
        };
        c = filter_level<FILTER>(sel[k], uv.x, uv.y, smp);
      }
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
  const size_t lds = (size_t)(BiasLds<HID, 5>::kCount + 2 * kRegions) * sizeof(f32x4) + kFiltStageTexels * sizeof(uint2);
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
